"""Shared helpers of the GPU tests: run the HIP library and the FP64 oracle on the same inputs."""
import numpy as np

import oracle
from synth import make_inputs, make_workload

try:
    from threadpoolctl import threadpool_limits
except ImportError:  # pragma: no cover
    threadpool_limits = None


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def gpu_run(d, r, iters, *, mu=1e-2, rho1=1e-2, rho2=1e-2, eta=1.0, precision="fp32", pinv_mode=0,
            history=False, want=("W", "Z"), x0=True, y0=True, seed=0, track=False, rank_tol=0.0, rank_every=0,
            xsolve=0):
    """Run the HIP path; returns dict with requested results and the f0 history."""
    from paper_2005_09838_amd import Completion
    c = Completion(to_dev(d["G"]), to_dev(d["omega"]), r, mu=mu, rho1=rho1, rho2=rho2, eta=eta,
                   precision=precision, pinv_mode=pinv_mode, X0=to_dev(d["X0"]) if x0 else None,
                   Y0=to_dev(d["Y0"]) if y0 else None, seed=seed, rank_tol=rank_tol, rank_every=rank_every,
                   xsolve=xsolve)
    if track:
        c.track_termination(True)
    f = [c.objective()] if history else []
    if history:
        for _ in range(iters):
            c.step(1)
            f.append(c.objective())
    else:
        c.step(iters)
    res = c.result(**{k: True for k in want})
    out = {k: v.cpu().numpy().astype(np.float64) for k, v in res.items()}
    out["f0"] = f if history else [c.objective()]
    out["ctx"] = c
    return out


def oracle_run(d, r, iters, *, mu=1e-2, rho1=1e-2, rho2=1e-2, eta=1.0, history=False):
    def go():
        return oracle.complete(d["G"], d["omega"], r, d["X0"], d["Y0"], iters, mu, rho1, rho2, eta,
                               record_objective=history)
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            st, info = go()
    else:
        st, info = go()
    return st, info


__all__ = ["rel", "to_dev", "gpu_run", "oracle_run", "make_inputs", "make_workload", "oracle"]
