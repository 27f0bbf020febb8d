"""The allocation-free entry point (static per-device scratch) against tctf_complete.

Two calls in a row through the C ABI, the second on a smaller problem: each must give, bit
for bit, what tctf_complete gives with a caller-allocated workspace (the kernels are the
same; only the workspace's address differs).  Also: a problem larger than the scratch is
rejected before any device work."""
import numpy as np
import pytest

from tests.gpu_helpers import make_inputs, to_dev

pytestmark = pytest.mark.gpu


def _with_workspace(B, p, d, iters):
    import torch
    n = B.tctf_workspace_bytes(p)
    ws = torch.empty(n + 256, dtype=torch.uint8, device="cuda:0")
    ptr = (ws.data_ptr() + 255) & ~255
    W = torch.empty(d["G"].shape, dtype=torch.float32, device="cuda:0")
    f0 = B.tctf_complete(p, to_dev(d["G"]), to_dev(d["omega"]), to_dev(d["X0"]), to_dev(d["Y0"]), 0, iters, ptr,
                         n, None, W)
    return W.cpu().numpy(), f0


def test_noalloc_matches_complete_on_two_calls_in_a_row():
    import torch
    from paper_2005_09838_amd import binding as B
    cases = [(144, 288, 28, 8, 0.4, 12), (36, 48, 7, 3, 0.3, 9)]   # the second call is smaller
    for n1, n2, n3, r, p, iters in cases:
        print(f"no-alloc case {n1}x{n2}x{n3} r{r} {iters} iterations", flush=True)
        d = make_inputs(n1, n2, n3, r, p=p, seed=n1 + n3, weekly=True, noise=0.02)
        prm = B.make_params(n1, n2, n3, r)
        ref_w, ref_f0 = _with_workspace(B, prm, d, iters)
        W = torch.empty((n1, n2, n3), dtype=torch.float32, device="cuda:0")
        f0 = B.tctf_complete_noalloc(prm, to_dev(d["G"]), to_dev(d["omega"]), to_dev(d["X0"]), to_dev(d["Y0"]), 0,
                                     iters, None, W)
        w = W.cpu().numpy()
        assert np.array_equal(w, ref_w), float(np.abs(w - ref_w).max())
        assert f0 == ref_f0, (f0, ref_f0)


def test_noalloc_rejects_a_problem_larger_than_the_scratch():
    from paper_2005_09838_amd import binding as B
    prm = B.make_params(529, 96, 112, 16)
    assert B.tctf_workspace_bytes(prm) > B.TCTF_NOALLOC_SCRATCH_BYTES
    with pytest.raises(B.TctfError) as e:
        B.tctf_complete_noalloc(prm, 4096, 4096, None, None, 0, 1, None, 4096)
    assert e.value.status == B.TCTF_E_WORKSPACE
