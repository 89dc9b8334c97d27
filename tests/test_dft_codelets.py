"""The generated DFT codelets, compiled for the host with g++, against numpy.fft.

The codelet header is device code; the test strips its HIP include and
supplies host stand-ins for float2/make_float2 and the __device__ qualifiers,
so the exact same arithmetic runs on the CPU.
"""
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2010_00520_amd", "csrc")

SHIM = r"""
#include <cmath>
#include <cstdio>
#include <cstdlib>
#define __device__
#define __forceinline__ inline
#define __restrict__
struct float2 { float x, y; };
static inline float2 make_float2(float a, float b) { float2 r; r.x = a; r.y = b; return r; }
"""

MAIN = r"""
int main() {
  // reads: kind n then n_in complex values; prints outputs
  char kind[16]; int n;
  while (scanf("%15s %d", kind, &n) == 2) {
    float2 x[64], y[64];
    bool full = kind[1] == 'F' || kind[1] == 'I';
    int nin = (kind[0] == 'f' && !full) ? n / 2 : n;
    for (int i = 0; i < nin; ++i) scanf("%f %f", &x[i].x, &x[i].y);
    int nout = (kind[0] == 'i') ? n / 2 : n;
    bool ok = !full;
    if (ok) switch (n) {
#define CASE(N) case N: if (kind[0]=='f') dft_fwd_##N(x, y); else dft_inv_##N(x, y); break;
      CASE(2) CASE(4) CASE(6) CASE(8) CASE(12) CASE(16) CASE(24) CASE(32) CASE(48) CASE(64)
      default: ok = false;
    }
    if (!ok) {
      switch (n) {
#define SCASE(N) case N: if (kind[1]=='F') dft_full_fwd_##N(x, y); else dft_full_inv_##N(x, y); break;
        SCASE(1) SCASE(2) SCASE(3) SCASE(4) SCASE(5) SCASE(6) SCASE(7) SCASE(8) SCASE(12) SCASE(16) SCASE(24)
        SCASE(32)
      }
      nout = n;
    }
    for (int i = 0; i < nout; ++i) printf("%.9e %.9e\n", y[i].x, y[i].y);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def codelet_exe(tmp_path_factory):
    d = tmp_path_factory.mktemp("dft")
    hdr = os.path.join(d, "dft_codelets.h")
    subprocess.check_call(["python3", os.path.join(CSRC, "gen_dft.py"), hdr])
    text = open(hdr).read().replace("#include <hip/hip_runtime.h>", "")
    src = os.path.join(d, "t.cpp")
    with open(src, "w") as f:
        f.write(SHIM + text + MAIN)
    exe = os.path.join(d, "t")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-o", exe, src])
    return exe


def _run(exe, kind, n, x):
    inp = f"{kind} {n}\n" + "\n".join(f"{v.real:.9e} {v.imag:.9e}" for v in x) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split()
    v = np.array(out, dtype=np.float64).reshape(-1, 2)
    return v[:, 0] + 1j * v[:, 1]


@pytest.mark.parametrize("n", [2, 4, 6, 8, 12, 16, 24, 32, 48, 64])
def test_pruned_codelets_match_numpy(codelet_exe, n):
    rng = np.random.default_rng(n)
    x = (rng.standard_normal(n // 2) + 1j * rng.standard_normal(n // 2)).astype(np.complex64)
    y = _run(codelet_exe, "f", n, x)
    ref = np.fft.fft(np.concatenate([x.astype(np.complex128), np.zeros(n - n // 2)]))
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 2e-7
    z = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    yi = _run(codelet_exe, "i", n, z)
    refi = np.fft.ifft(z.astype(np.complex128))[: n // 2] * n
    assert np.linalg.norm(yi - refi) / np.linalg.norm(refi) < 2e-7


@pytest.mark.parametrize("t", [1, 2, 3, 4, 5, 6, 7, 8, 12, 16, 24, 32])
def test_full_codelets_match_numpy(codelet_exe, t):
    rng = np.random.default_rng(100 + t)
    x = (rng.standard_normal(t) + 1j * rng.standard_normal(t)).astype(np.complex64)
    ref = np.fft.fft(x.astype(np.complex128))
    assert np.linalg.norm(_run(codelet_exe, "fF", t, x) - ref) / np.linalg.norm(ref) < 2e-7
    refi = np.fft.ifft(x.astype(np.complex128)) * t
    assert np.linalg.norm(_run(codelet_exe, "iI", t, x) - refi) / np.linalg.norm(refi) < 2e-7


@pytest.mark.parametrize("n3", [8, 16, 24, 32, 48, 64])
def test_even_odd_split_of_the_pruned_z_transform(codelet_exe, n3):
    """The three-pass z-stage's pencil transform, in the codelets' own arithmetic:
    X[2m] = DFT_K(x)[m], X[2m+1] = DFT_K(x w^z)[m] (K = n3/2 nonzero inputs), then
    y[z] = IDFT_K(P_even)[z] + w^-z IDFT_K(P_odd)[z] for z < K, against the pruned
    transform pair written out with numpy."""
    K = n3 // 2
    rng = np.random.default_rng(300 + n3)
    x = (rng.standard_normal(K) + 1j * rng.standard_normal(K)).astype(np.complex64)
    t = (rng.standard_normal(n3) + 1j * rng.standard_normal(n3)).astype(np.complex64)
    w = np.exp(-2j * np.pi * np.arange(K) / n3)
    E = _run(codelet_exe, "fF", K, x)
    O = _run(codelet_exe, "fF", K, (x * w).astype(np.complex64))
    ye = _run(codelet_exe, "iI", K, (E * t[0::2]).astype(np.complex64))
    yo = _run(codelet_exe, "iI", K, (O * t[1::2]).astype(np.complex64))
    y = ye + np.conj(w) * yo
    X = np.fft.fft(np.concatenate([x.astype(np.complex128), np.zeros(K)]))
    ref = (np.fft.ifft(X * t.astype(np.complex128)) * n3)[:K]
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-6
