"""The generated straight-line tube transforms of the slice kernel, compiled for the host
with g++ and compared with the oracle's transform pair (CPU only)."""
import ctypes
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GEN = os.path.join(ROOT, "paper_2005_09838_amd", "csrc", "gen_tube_dft.py")


@pytest.fixture(scope="module")
def host_lib(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("tubedft")
    hdr = d / "tube_dft_gen.h"
    subprocess.run([sys.executable, GEN, str(hdr)], check=True)
    sys.path.insert(0, os.path.dirname(GEN))
    import gen_tube_dft
    sizes = gen_tube_dft.SIZES
    src = ["#include <cmath>", "#define TUBE_DFT_QUAL inline", f'#include "{hdr}"']
    for n in sizes:
        nb = n // 2 + 1
        src.append(f'extern "C" void fwd_{n}(const float* x, float* re, float* im) {{ float a[{n}], r[{nb}], i[{nb}]; '
                   f'for (int k = 0; k < {n}; k++) a[k] = x[k]; tube_fwd<{n}>(a, r, i); '
                   f'for (int b = 0; b < {nb}; b++) {{ re[b] = r[b]; im[b] = i[b]; }} }}')
        src.append(f'extern "C" void inv_{n}(const float* re, const float* im, float* x) {{ float a[{n}], r[{nb}], i[{nb}]; '
                   f'for (int b = 0; b < {nb}; b++) {{ r[b] = re[b]; i[b] = im[b]; }} tube_inv<{n}>(r, i, a); '
                   f'for (int k = 0; k < {n}; k++) x[k] = a[k]; }}')
    (d / "t.cpp").write_text("\n".join(src))
    so = d / "libt.so"
    subprocess.run(["g++", "-O1", "-shared", "-fPIC", "-o", str(so), str(d / "t.cpp")], check=True)
    return ctypes.CDLL(str(so)), sizes


def test_forward_and_inverse_match_the_paper_transform(host_lib):
    lib, sizes = host_lib
    rng = np.random.default_rng(0)
    P = ctypes.POINTER(ctypes.c_float)
    for n in sizes:
        nb = n // 2 + 1
        for _ in range(3):
            x = rng.normal(size=n).astype(np.float32)
            re = np.zeros(nb, np.float32)
            im = np.zeros(nb, np.float32)
            getattr(lib, f"fwd_{n}")(x.ctypes.data_as(P), re.ctypes.data_as(P), im.ctypes.data_as(P))
            ref = oracle.dft3(x.astype(np.float64).reshape(1, 1, n))[0, 0, :nb]
            assert np.abs(re + 1j * im - ref).max() <= 4e-7 * np.abs(ref).max(), n
            xr = rng.normal(size=nb).astype(np.float32)
            xi = rng.normal(size=nb).astype(np.float32)
            out = np.zeros(n, np.float32)
            getattr(lib, f"inv_{n}")(xr.ctypes.data_as(P), xi.ctypes.data_as(P), out.ctypes.data_as(P))
            spec = xr.astype(float) + 1j * xi.astype(float)
            spec[0] = spec[0].real
            if n % 2 == 0:
                spec[n // 2] = spec[n // 2].real
            full = np.concatenate([spec, np.conj(spec[1:n - nb + 1][::-1])])
            ref2 = oracle.idft3(full.reshape(1, 1, n))[0, 0]
            assert np.abs(ref2.imag).max() < 1e-12
            assert np.abs(out - ref2.real).max() <= 4e-7 * np.abs(ref2).max(), n
