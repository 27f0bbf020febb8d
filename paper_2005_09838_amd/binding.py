"""ctypes binding of the C ABI declared in include/tctf2r.h (argument marshalling only).

Every function of the header is exposed under the same name and takes the same arguments
(device pointers as Python ints or torch tensors).  ``Completion`` and ``complete`` wrap
them for torch users: torch provides the device memory (the workspace and the result
tensors are torch tensors) and the stream; all computation happens in the HIP library.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtctf2r.so")

TCTF_OK, TCTF_E_ARG, TCTF_E_SHAPE, TCTF_E_NONFINITE, TCTF_E_HIP, TCTF_E_WORKSPACE, TCTF_E_STATE = 0, -1, -2, -3, -4, -5, -6
TCTF_FP32, TCTF_MIXED_BF16 = 0, 1
TCTF_NOALLOC_SCRATCH_BYTES = 32 << 20   # static scratch of tctf_complete_noalloc (the header's constant)
STAGES = {"slice": 0, "zgemm": 1, "agemm": 2, "hsolve": 3, "bgemm": 4, "ystep": 5, "pinvy": 6, "iteration": 7}


class tctf_params(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("n3", ctypes.c_int32), ("r", ctypes.c_int32),
                ("mu", ctypes.c_double), ("rho1", ctypes.c_double), ("rho2", ctypes.c_double),
                ("eta", ctypes.c_double), ("precision", ctypes.c_int32), ("pinv_mode", ctypes.c_int32),
                ("eps", ctypes.c_double), ("rank_tol", ctypes.c_double), ("rank_every", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("xsolve", ctypes.c_int32)]


class TctfError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {status_string(status)} ({status}): {detail}")
        self.status = status


_lib = None


def library() -> ctypes.CDLL:
    """Load libtctf2r.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    P, S, I32, I64, U64, D = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    PP = ctypes.POINTER(tctf_params)
    sig = {
        "tctf_default_params": (None, [PP]),
        "tctf_workspace_bytes": (I32, [PP, ctypes.POINTER(S)]),
        "tctf_create": (I32, [PP, P, P, P, P, U64, P, S, P, ctypes.POINTER(P)]),
        "tctf_step": (I32, [P, I32]),
        "tctf_objective": (I32, [P, ctypes.POINTER(D)]),
        "tctf_termination": (I32, [P, ctypes.POINTER(D)]),
        "tctf_stationarity": (I32, [P, ctypes.POINTER(D)]),
        "tctf_get_result": (I32, [P, P, P, P, P]),
        "tctf_state_bytes": (I32, [P, ctypes.POINTER(S)]),
        "tctf_get_state": (I32, [P, P, S]),
        "tctf_set_state": (I32, [P, P, S]),
        "tctf_iterations": (I32, [P, ctypes.POINTER(I64)]),
        "tctf_rank_vector": (I32, [P, ctypes.POINTER(I32)]),
        "tctf_tuning": (I32, [P, ctypes.POINTER(I32)]),
        "tctf_destroy": (None, [P]),
        "tctf_complete": (I32, [PP, P, P, P, P, U64, I32, P, S, P, P, ctypes.POINTER(D)]),
        "tctf_time_stage": (I32, [P, I32, I32, ctypes.POINTER(D)]),
        "tctf_profile": (I32, [P, ctypes.c_uint32]),
        "tctf_run": (I32, [P, I32, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "tctf_track_termination": (I32, [P, I32]),
        "tctf_complete_noalloc": (I32, [PP, P, P, P, P, U64, I32, P, P, ctypes.POINTER(D)]),
        "tctf_adjoint_workspace_bytes": (I32, [PP, ctypes.POINTER(S)]),
        "tctf_adjoint_step": (I32, [P, P, P, P, P, P, P, P, S]),
        "tctf_adjoint_initial": (I32, [P, P, P, P, P]),
        "tctf_objective_gradient": (I32, [P, P, P, P, S]),
        "tctf_batch_workspace_bytes": (I32, [I32, PP, ctypes.POINTER(S)]),
        "tctf_batch_create": (I32, [I32, PP, P, P, P, P, P, P, S, P, ctypes.POINTER(P)]),
        "tctf_batch_step": (I32, [P, I32]),
        "tctf_batch_size": (I32, [P, ctypes.POINTER(I32)]),
        "tctf_batch_member": (I32, [P, I32, ctypes.POINTER(P)]),
        "tctf_batch_destroy": (None, [P]),
        "tctf_profile_read": (I32, [P, ctypes.POINTER(D), ctypes.POINTER(I64)]),
        "tctf_status_string": (ctypes.c_char_p, [I32]),
        "tctf_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(x):
    """Device pointer of a torch tensor, an int, or None (NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _check(status: int, where: str):
    if status != TCTF_OK:
        raise TctfError(status, where, tctf_last_error())


# ---------------------------------------------------------------- the C functions, same names

def tctf_default_params(p: tctf_params | None = None) -> tctf_params:
    p = p or tctf_params()
    library().tctf_default_params(ctypes.byref(p))
    return p


def tctf_workspace_bytes(p: tctf_params) -> int:
    n = ctypes.c_size_t(0)
    _check(library().tctf_workspace_bytes(ctypes.byref(p), ctypes.byref(n)), "tctf_workspace_bytes")
    return n.value


def tctf_create(p: tctf_params, G, omega, X0, Y0, seed: int, workspace, ws_bytes: int, stream: int | None):
    ctx = ctypes.c_void_p()
    _check(library().tctf_create(ctypes.byref(p), _ptr(G), _ptr(omega), _ptr(X0), _ptr(Y0), seed,
                                 _ptr(workspace), ws_bytes, stream, ctypes.byref(ctx)), "tctf_create")
    return ctx


def tctf_step(ctx, iters: int):
    _check(library().tctf_step(ctx, iters), "tctf_step")


def tctf_track_termination(ctx, on: bool):
    _check(library().tctf_track_termination(ctx, 1 if on else 0), "tctf_track_termination")


def tctf_objective(ctx) -> float:
    v = ctypes.c_double()
    _check(library().tctf_objective(ctx, ctypes.byref(v)), "tctf_objective")
    return v.value


def tctf_termination(ctx) -> tuple:
    v = (ctypes.c_double * 4)()
    _check(library().tctf_termination(ctx, v), "tctf_termination")
    return tuple(v)


def tctf_stationarity(ctx) -> tuple:
    v = (ctypes.c_double * 3)()
    _check(library().tctf_stationarity(ctx, v), "tctf_stationarity")
    return tuple(v)


def tctf_get_result(ctx, W=None, Z=None, X=None, Y=None):
    _check(library().tctf_get_result(ctx, _ptr(W), _ptr(Z), _ptr(X), _ptr(Y)), "tctf_get_result")


def tctf_state_bytes(ctx) -> int:
    n = ctypes.c_size_t(0)
    _check(library().tctf_state_bytes(ctx, ctypes.byref(n)), "tctf_state_bytes")
    return n.value


def tctf_get_state(ctx, dst, nbytes: int):
    _check(library().tctf_get_state(ctx, _ptr(dst), nbytes), "tctf_get_state")


def tctf_set_state(ctx, src, nbytes: int):
    _check(library().tctf_set_state(ctx, _ptr(src), nbytes), "tctf_set_state")


def tctf_rank_vector(ctx, nb: int) -> list:
    v = (ctypes.c_int32 * nb)()
    _check(library().tctf_rank_vector(ctx, v), "tctf_rank_vector")
    return list(v)


def tctf_tuning(ctx) -> tuple:
    v = (ctypes.c_int32 * 5)()
    _check(library().tctf_tuning(ctx, v), "tctf_tuning")
    return tuple(v)


def tctf_iterations(ctx) -> int:
    v = ctypes.c_int64()
    _check(library().tctf_iterations(ctx, ctypes.byref(v)), "tctf_iterations")
    return v.value


def tctf_destroy(ctx):
    library().tctf_destroy(ctx)


def tctf_complete(p: tctf_params, G, omega, X0, Y0, seed: int, iters: int, workspace, ws_bytes: int,
                  stream: int | None, W_out) -> float:
    f0 = ctypes.c_double()
    _check(library().tctf_complete(ctypes.byref(p), _ptr(G), _ptr(omega), _ptr(X0), _ptr(Y0), seed, iters,
                                   _ptr(workspace), ws_bytes, stream, _ptr(W_out), ctypes.byref(f0)),
           "tctf_complete")
    return f0.value


def tctf_complete_noalloc(p: tctf_params, G, omega, X0, Y0, seed: int, iters: int, stream: int | None,
                          W_out) -> float:
    f0 = ctypes.c_double()
    _check(library().tctf_complete_noalloc(ctypes.byref(p), _ptr(G), _ptr(omega), _ptr(X0), _ptr(Y0), seed, iters,
                                           stream, _ptr(W_out), ctypes.byref(f0)), "tctf_complete_noalloc")
    return f0.value


def tctf_adjoint_workspace_bytes(p: tctf_params) -> int:
    n = ctypes.c_size_t(0)
    _check(library().tctf_adjoint_workspace_bytes(ctypes.byref(p), ctypes.byref(n)), "tctf_adjoint_workspace_bytes")
    return n.value


def tctf_adjoint_step(ctx, state_in, state_out, xt_bar, yt_bar, w_bar, theta_bar, workspace, ws_bytes: int):
    _check(library().tctf_adjoint_step(ctx, _ptr(state_in), _ptr(state_out), _ptr(xt_bar), _ptr(yt_bar), _ptr(w_bar),
                                       _ptr(theta_bar), _ptr(workspace), ws_bytes), "tctf_adjoint_step")


def tctf_adjoint_initial(ctx, xt_bar, yt_bar, x0_bar, y0_bar):
    _check(library().tctf_adjoint_initial(ctx, _ptr(xt_bar), _ptr(yt_bar), _ptr(x0_bar), _ptr(y0_bar)),
           "tctf_adjoint_initial")


def tctf_objective_gradient(ctx, x_grad, y_grad, workspace, ws_bytes: int):
    _check(library().tctf_objective_gradient(ctx, _ptr(x_grad), _ptr(y_grad), _ptr(workspace), ws_bytes),
           "tctf_objective_gradient")


def tctf_time_stage(ctx, stage: int, reps: int) -> float:
    v = ctypes.c_double()
    _check(library().tctf_time_stage(ctx, stage, reps, ctypes.byref(v)), "tctf_time_stage")
    return v.value


def tctf_profile(ctx, mask: int) -> None:
    _check(library().tctf_profile(ctx, mask), "tctf_profile")


def tctf_profile_read(ctx):
    """Per stage 0..6: (summed microseconds, launches) recorded since tctf_profile(ctx, mask)."""
    tot = (ctypes.c_double * 7)()
    cnt = (ctypes.c_int64 * 7)()
    _check(library().tctf_profile_read(ctx, tot, cnt), "tctf_profile_read")
    return [(tot[k], cnt[k]) for k in range(7)]


def tctf_status_string(status: int) -> str:
    return library().tctf_status_string(status).decode()


def status_string(status: int) -> str:
    try:
        return tctf_status_string(status)
    except ImportError:
        return "status"


def tctf_last_error() -> str:
    s = library().tctf_last_error()
    return s.decode() if s else ""


# ---------------------------------------------------------------- torch convenience layer

def make_params(n1, n2, n3, r, mu=1e-2, rho1=1e-2, rho2=1e-2, eta=1.0, precision="fp32", pinv_mode=0,
                eps=1e-6, rank_tol=0.0, rank_every=0, autotune=False, xsolve=0) -> tctf_params:
    p = tctf_default_params()
    p.n1, p.n2, p.n3, p.r = int(n1), int(n2), int(n3), int(r)
    p.mu, p.rho1, p.rho2, p.eta = float(mu), float(rho1), float(rho2), float(eta)
    p.precision = {"fp32": TCTF_FP32, "mixed": TCTF_MIXED_BF16, "bf16": TCTF_MIXED_BF16}[precision] \
        if isinstance(precision, str) else int(precision)
    p.pinv_mode = int(pinv_mode)
    p.eps = float(eps)
    p.rank_tol = float(rank_tol)
    p.rank_every = int(rank_every)
    p.autotune = 1 if autotune else 0
    p.xsolve = int(xsolve)
    return p


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Completion:
    """One completion on the current GPU: owns the workspace tensor and the C context."""

    @classmethod
    def _member(cls, ctx, G, r, params):
        """A view of a batch member's context (owned by the batch, not closed here)."""
        import torch
        self = cls.__new__(cls)
        self.torch = torch
        self.G = G
        self.shape = tuple(G.shape)
        self.r = r
        self.params = params
        self.ctx = ctx
        self._owned = False
        return self

    def __init__(self, G, omega, r, *, mu=1e-2, rho1=1e-2, rho2=1e-2, eta=1.0, precision="fp32",
                 pinv_mode=0, eps=1e-6, X0=None, Y0=None, seed=0, stream=None, rank_tol=0.0, rank_every=0,
                 autotune=False, xsolve=0):
        import torch
        self._owned = True
        if not (G.is_cuda and omega.is_cuda):
            raise ValueError("G and omega must be device tensors")
        n1, n2, n3 = G.shape
        self.torch = torch
        self.G = G.contiguous().to(torch.float32)
        self.omega = omega.contiguous().to(torch.uint8)
        self.X0 = None if X0 is None else X0.contiguous().to(torch.float32)
        self.Y0 = None if Y0 is None else Y0.contiguous().to(torch.float32)
        self.params = make_params(n1, n2, n3, r, mu, rho1, rho2, eta, precision, pinv_mode, eps, rank_tol,
                                  rank_every, autotune, xsolve)
        self.shape = (n1, n2, n3)
        self.r = r
        self.stream = stream
        nbytes = tctf_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=G.device)
        base = self.workspace.data_ptr()
        self.ws_ptr = (base + 255) & ~255
        self.ws_bytes = nbytes
        self.ctx = tctf_create(self.params, self.G, self.omega, self.X0, self.Y0, seed, self.ws_ptr, nbytes,
                               _stream_handle(stream))

    def close(self):
        if getattr(self, "ctx", None) and getattr(self, "_owned", True):
            tctf_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, iters=1):
        tctf_step(self.ctx, iters)
        return self

    def run(self, max_iters, check_every=10):
        """Iterate until the step-6 termination test holds; returns (iterations run, converged)."""
        n, conv = ctypes.c_int32(), ctypes.c_int32()
        _check(library().tctf_run(self.ctx, max_iters, check_every, ctypes.byref(n), ctypes.byref(conv)),
               "tctf_run")
        return n.value, bool(conv.value)

    def track_termination(self, on=True):
        """Evaluate step 6 after every later step() call (needed by termination())."""
        tctf_track_termination(self.ctx, on)
        return self

    def objective(self):
        return tctf_objective(self.ctx)

    def termination(self):
        return tctf_termination(self.ctx)

    def stationarity(self):
        return tctf_stationarity(self.ctx)

    def tuning(self):
        """(slice path, columns per X~^* W~ block, columns per Y-step block, from the cache,
        half-width of the H_rho1^{-1} stencil in the X-update or -1 for the separate solve)."""
        return tctf_tuning(self.ctx)

    def rank_vector(self):
        """Step 5's rank vector r_b of the stored frequencies b = 0 .. n3 / 2."""
        return tctf_rank_vector(self.ctx, self.shape[2] // 2 + 1)

    @property
    def iterations(self):
        return tctf_iterations(self.ctx)

    def result(self, W=True, Z=False, X=False, Y=False):
        torch = self.torch
        n1, n2, n3 = self.shape
        dev = self.G.device
        out = {}
        if W:
            out["W"] = torch.empty((n1, n2, n3), dtype=torch.float32, device=dev)
        if Z:
            out["Z"] = torch.empty((n1, n2, n3), dtype=torch.float32, device=dev)
        if X:
            out["X"] = torch.empty((n1, self.r, n3), dtype=torch.float32, device=dev)
        if Y:
            out["Y"] = torch.empty((self.r, n2, n3), dtype=torch.float32, device=dev)
        tctf_get_result(self.ctx, out.get("W"), out.get("Z"), out.get("X"), out.get("Y"))
        return out

    def adjoint_workspace(self):
        """(pointer, bytes) of this completion's adjoint workspace (a torch tensor, made once)."""
        if getattr(self, "_adj_ws", None) is None:
            n = tctf_adjoint_workspace_bytes(self.params)
            buf = self.torch.empty(n + 256, dtype=self.torch.uint8, device=self.G.device)
            self._adj_ws = (buf, (buf.data_ptr() + 255) & ~255, n)
        return self._adj_ws[1], self._adj_ws[2]

    def objective_gradient(self):
        """(d f0 / d X, d f0 / d Y) at the current iterate: float64 tensors [n1][r][n3], [r][n2][n3]."""
        torch = self.torch
        n1, n2, n3 = self.shape
        gx = torch.empty((n1, self.r, n3), dtype=torch.float64, device=self.G.device)
        gy = torch.empty((self.r, n2, n3), dtype=torch.float64, device=self.G.device)
        ws, nbytes = self.adjoint_workspace()
        tctf_objective_gradient(self.ctx, gx, gy, ws, nbytes)
        return gx, gy

    def get_state(self):
        n = tctf_state_bytes(self.ctx)
        buf = self.torch.empty(n, dtype=self.torch.uint8, device=self.G.device)
        tctf_get_state(self.ctx, buf, n)
        return buf

    def set_state(self, buf):
        tctf_set_state(self.ctx, buf, buf.numel())

    def time_stage(self, stage, reps=20):
        return tctf_time_stage(self.ctx, STAGES[stage] if isinstance(stage, str) else int(stage), reps)

    def profile(self, stages):
        """Bracket every launch of the named stages in later steps with HIP events (empty: stop)."""
        mask = 0
        for st in stages:
            mask |= 1 << (STAGES[st] if isinstance(st, str) else int(st))
        tctf_profile(self.ctx, mask)

    def profile_read(self):
        """{stage name: (mean microseconds per launch, launches)} of the recorded launches."""
        names = {v: k for k, v in STAGES.items()}
        return {names[k]: (tot / cnt if cnt else None, cnt)
                for k, (tot, cnt) in enumerate(tctf_profile_read(self.ctx))}


class Batch:
    """Independent completions of possibly different sizes run together (tctf_batch_*).

    problems: list of dicts with keys G, omega (device tensors), r and optionally mu, rho1,
    rho2, eta, precision, X0, Y0, seed."""

    def __init__(self, problems, stream=None):
        import torch
        n = len(problems)
        self.torch = torch
        self.params = (tctf_params * n)()
        keep = []
        ptrs = {k: (ctypes.c_void_p * n)() for k in ("G", "omega", "X0", "Y0")}
        seeds = (ctypes.c_uint64 * n)()
        self.shapes = []
        for k, pr in enumerate(problems):
            G = pr["G"].contiguous().to(torch.float32)
            om = pr["omega"].contiguous().to(torch.uint8)
            n1, n2, n3 = G.shape
            self.params[k] = make_params(n1, n2, n3, pr["r"], pr.get("mu", 1e-2), pr.get("rho1", 1e-2),
                                         pr.get("rho2", 1e-2), pr.get("eta", 1.0), pr.get("precision", "fp32"),
                                         autotune=pr.get("autotune", False))
            ptrs["G"][k], ptrs["omega"][k] = G.data_ptr(), om.data_ptr()
            keep += [G, om]
            for key in ("X0", "Y0"):
                if pr.get(key) is not None:
                    t = pr[key].contiguous().to(torch.float32)
                    keep.append(t)
                    ptrs[key][k] = t.data_ptr()
            seeds[k] = pr.get("seed", 0)
            self.shapes.append((G, pr["r"]))
        nbytes = ctypes.c_size_t()
        _check(library().tctf_batch_workspace_bytes(n, self.params, ctypes.byref(nbytes)),
               "tctf_batch_workspace_bytes")
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=problems[0]["G"].device)
        ws = (self.workspace.data_ptr() + 255) & ~255
        out = ctypes.c_void_p()
        _check(library().tctf_batch_create(n, self.params, ptrs["G"], ptrs["omega"], ptrs["X0"], ptrs["Y0"], seeds,
                                           ws, nbytes.value, _stream_handle(stream), ctypes.byref(out)),
               "tctf_batch_create")
        self.batch = out.value
        self.members = []
        for k in range(n):
            m = ctypes.c_void_p()
            _check(library().tctf_batch_member(self.batch, k, ctypes.byref(m)), "tctf_batch_member")
            G, r = self.shapes[k]
            self.members.append(Completion._member(m.value, G, r, self.params[k]))

    def step(self, iters=1):
        _check(library().tctf_batch_step(self.batch, iters), "tctf_batch_step")
        return self

    def __len__(self):
        return len(self.members)

    def __getitem__(self, k):
        return self.members[k]

    def close(self):
        if getattr(self, "batch", None):
            for m in self.members:
                m.ctx = None
            library().tctf_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def complete(M, omega, r, lam=1e-2, rho1=1e-2, rho2=1e-2, iters=50, precision="fp32", X0=None, Y0=None,
             seed=0, eta=1.0):
    """Complete M observed on omega (device tensors); returns (W, info) with info['f0']."""
    c = Completion(M, omega, r, mu=lam, rho1=rho1, rho2=rho2, eta=eta, precision=precision, X0=X0, Y0=Y0,
                   seed=seed)
    try:
        c.step(iters)
        W = c.result()["W"]
        return W, {"f0": c.objective(), "iterations": c.iterations}
    finally:
        c.close()
