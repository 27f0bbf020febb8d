"""Host-side checks of the C ABI that need no GPU: the library loads, exports every symbol
the header declares, and rejects bad parameters before any device work."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tctf2r.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(tctf_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for n in ("tctf_create", "tctf_step", "tctf_objective", "tctf_get_result", "tctf_complete",
              "tctf_workspace_bytes", "tctf_destroy", "tctf_stationarity", "tctf_get_state", "tctf_set_state"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2005_09838_amd import binding
    lib = binding.library()
    for n in _declared_functions():
        assert hasattr(lib, n), n


def test_default_params_and_status_strings():
    from paper_2005_09838_amd import binding as B
    p = B.tctf_default_params()
    assert (p.mu, p.rho1, p.rho2, p.eta, p.precision, p.pinv_mode, p.eps) == (1e-2, 1e-2, 1e-2, 1.0, 0, 0, 1e-6)
    assert B.tctf_status_string(0) == "ok"
    assert B.tctf_status_string(-3) == "non-finite value"


@pytest.mark.parametrize("kw,status", [
    (dict(n1=0, n2=4, n3=4, r=1), -2),
    (dict(n1=8, n2=4, n3=4, r=5), -2),          # r > min(n1, n2)
    (dict(n1=8, n2=40, n3=40, r=33), -2),       # r > 32
    (dict(n1=8, n2=4, n3=9000, r=2), -2),       # tube length above the limit
    (dict(n1=9000, n2=4, n3=4, r=2), -2),       # n1 above the limit
    (dict(n1=8, n2=1100, n3=16, r=2), -2),      # n2 above the limit
    (dict(n1=8, n2=4, n3=4, r=2, mu=-1.0), -1),
    (dict(n1=8, n2=4, n3=4, r=2, rho2=float("nan")), -1),
    (dict(n1=8, n2=4, n3=4, r=2, eta=2.0), -1),
    (dict(n1=8, n2=4, n3=4, r=2, eta=0.0), -1),
    (dict(n1=8, n2=4, n3=4, r=2, precision=7), -1),
    (dict(n1=8, n2=4, n3=4, r=2, pinv_mode=3), -1),
])
def test_parameter_validation(kw, status):
    from paper_2005_09838_amd import binding as B
    p = B.make_params(**kw)
    with pytest.raises(B.TctfError) as e:
        B.tctf_workspace_bytes(p)
    assert e.value.status == status
    assert B.tctf_last_error()


def test_workspace_size_grows_with_the_problem():
    from paper_2005_09838_amd import binding as B
    a = B.tctf_workspace_bytes(B.make_params(36, 48, 7, 3))
    b = B.tctf_workspace_bytes(B.make_params(529, 96, 112, 16))
    c = B.tctf_workspace_bytes(B.make_params(529, 96, 112, 16, precision="mixed"))
    assert 0 < a < c < b
    assert b % 256 == 0


def test_create_rejects_null_arguments_before_device_work():
    from paper_2005_09838_amd import binding as B
    p = B.make_params(8, 6, 4, 2)
    n = B.tctf_workspace_bytes(p)
    with pytest.raises(B.TctfError) as e:
        B.tctf_create(p, None, None, None, None, 0, None, n, None)
    assert e.value.status == B.TCTF_E_ARG
    with pytest.raises(B.TctfError) as e:
        B.tctf_create(p, 4096, 4096, None, None, 0, None, n, None)
    assert e.value.status == B.TCTF_E_WORKSPACE
    with pytest.raises(B.TctfError) as e:
        B.tctf_create(p, 4096, 4096, None, None, 0, 4096 + 8, n, None)
    assert e.value.status == B.TCTF_E_WORKSPACE
    with pytest.raises(B.TctfError) as e:
        B.tctf_create(p, 4096, 4096, None, None, 0, 4096, n - 1, None)
    assert e.value.status == B.TCTF_E_WORKSPACE


def test_adjoint_workspace_and_precision_checks():
    from paper_2005_09838_amd import binding as B
    n = B.tctf_adjoint_workspace_bytes(B.make_params(144, 288, 28, 8))
    assert n > 0 and n % 256 == 0
    with pytest.raises(B.TctfError) as e:
        B.tctf_adjoint_workspace_bytes(B.make_params(144, 288, 28, 8, precision="mixed"))
    assert e.value.status == B.TCTF_E_ARG


def test_noalloc_scratch_constant_matches_the_header():
    from paper_2005_09838_amd import binding as B
    text = open(HEADER).read()
    m = re.search(r"#define TCTF_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == B.TCTF_NOALLOC_SCRATCH_BYTES
