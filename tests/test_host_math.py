"""Host logic of the library (setup mathematics in host_math.cpp), on the CPU.

The library's compressor, eigensolver, FFT and quadrature nodes are compiled
with g++ into a small driver and checked against definitions and library
routines: reconstructions from the emitted factors (Eqs. (8), (9), (11), (13),
(14) written out with einsum) must be within the tolerance of the input tensor,
planted low-rank structure must be recovered exactly, and ranks must agree with
the oracle's within one (singular-value ties near the cut may differ).
"""
import os
import struct
import subprocess

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2010_00520_amd", "csrc")
FMT = {"full": 0, "tucker3d": 1, "tt3d": 2, "tucker4d": 3, "tt4d": 4, "htucker4d": 5}


@pytest.fixture(scope="module")
def drv(tmp_path_factory):
    d = tmp_path_factory.mktemp("host")
    exe = os.path.join(d, "host_driver")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-pthread", "-I" + CSRC,
                           os.path.join(ROOT, "tests", "host_driver.cpp"), os.path.join(CSRC, "host_math.cpp"),
                           "-o", exe])
    return exe, d


def compress(drv, That, fmt, gamma):
    exe, d = drv
    ndir, n1, n2, n3 = That.shape
    fin, fout = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
    with open(fin, "wb") as f:
        f.write(struct.pack("<5i", FMT[fmt], ndir, n1, n2, n3))
        f.write(struct.pack("<d", gamma))
        f.write(np.ascontiguousarray(That, dtype=np.complex128).tobytes())
    subprocess.check_call([exe, "compress", fin, fout])
    b = open(fout, "rb").read()
    (nr,) = struct.unpack_from("<i", b, 0)
    ranks = list(struct.unpack_from(f"<{nr}i", b, 4))
    off = 4 + 4 * nr
    rel, mx, sec = struct.unpack_from("<3d", b, off)
    off += 24
    (nd,) = struct.unpack_from("<q", b, off)
    data = np.frombuffer(b, dtype=np.complex128, count=nd, offset=off + 8)
    return ranks, rel, mx, sec, data


def reconstruct(fmt, ranks, data, n, ndir):
    """Restore T~[p][x][y][z] from the import layout by the defining equations."""
    n1, n2, n3 = n
    pos = [0]

    def take(shape):
        cnt = int(np.prod(shape))
        v = data[pos[0]:pos[0] + cnt].reshape(shape)
        pos[0] += cnt
        return v

    if fmt == "tucker3d":
        out = []
        for p in range(ndir):
            r1, r2, r3 = ranks[3 * p:3 * p + 3]
            C, U1, U2, U3 = take((r1, r2, r3)), take((n1, r1)), take((n2, r2)), take((n3, r3))
            out.append(np.einsum("abc,xa,yb,zc->xyz", C, U1, U2, U3))
        return np.stack(out)
    if fmt == "tt3d":
        out = []
        for p in range(ndir):
            r1, r2 = ranks[2 * p:2 * p + 2]
            U1, C, U3 = take((n1, r1)), take((r1, n2, r2)), take((n3, r2))
            out.append(np.einsum("xa,ayb,zb->xyz", U1, C, U3))
        return np.stack(out)
    if fmt == "tucker4d":
        r1, r2, r3, r4 = ranks
        C, U1, U2, U3, U4 = take((r1, r2, r3, r4)), take((n1, r1)), take((n2, r2)), take((n3, r3)), take((ndir, r4))
        return np.einsum("abcd,xa,yb,zc,pd->pxyz", C, U1, U2, U3, U4)
    if fmt == "tt4d":
        r1, r2, r3 = ranks
        U1, C1, C2, U3 = take((n1, r1)), take((r1, n2, r2)), take((r2, n3, r3)), take((ndir, r3))
        return np.einsum("xa,ayb,bzc,pc->pxyz", U1, C1, C2, U3)
    if fmt == "htucker4d":
        r1, r2, r3, r4, r12, r34 = ranks
        U1, U2, U3, U4 = take((n1, r1)), take((n2, r2)), take((n3, r3)), take((ndir, r4))
        C12, C34, B = take((r1, r2, r12)), take((r3, r4, r34)), take((r12, r34))
        G = np.einsum("abi,ij,cdj->abcd", C12, B, C34)
        return np.einsum("abcd,xa,yb,zc,pd->pxyz", G, U1, U2, U3, U4)
    raise ValueError(fmt)


def test_gauss_legendre(drv):
    exe, d = drv
    for n in (1, 2, 3, 15, 30):
        f = os.path.join(d, "gl.bin")
        subprocess.check_call([exe, "gl", str(n), f])
        v = np.fromfile(f, dtype=np.float64)
        x, w = np.polynomial.legendre.leggauss(n)
        np.testing.assert_allclose(v[:n], x, atol=1e-14)
        np.testing.assert_allclose(v[n:], w, atol=1e-14)


def test_hermitian_eigensolver(drv):
    exe, d = drv
    rng = np.random.default_rng(1)
    n = 40
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = X @ X.conj().T
    A[:5] *= 1e-9  # widely spread spectrum, like a Gram matrix
    A[:, :5] *= 1e-9
    fin, fout = os.path.join(d, "e.bin"), os.path.join(d, "eo.bin")
    with open(fin, "wb") as f:
        f.write(struct.pack("<i", n))
        f.write(A.astype(np.complex128).tobytes())
    subprocess.check_call([exe, "eig", fin, fout])
    b = open(fout, "rb").read()
    vals = np.frombuffer(b, dtype=np.float64, count=n)
    vecs = np.frombuffer(b, dtype=np.complex128, offset=8 * n).reshape(n, n)
    ref = np.sort(np.linalg.eigvalsh(A))[::-1]
    np.testing.assert_allclose(vals, ref, rtol=1e-10, atol=1e-12 * ref[0])
    np.testing.assert_allclose(vecs.conj().T @ vecs, np.eye(n), atol=1e-12)
    np.testing.assert_allclose(A @ vecs, vecs * vals, atol=1e-10 * ref[0])


def test_fft3d(drv):
    exe, d = drv
    rng = np.random.default_rng(2)
    for shape in [(2, 8, 12, 6), (1, 16, 16, 16), (3, 24, 8, 48)]:
        x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        fin, fout = os.path.join(d, "f.bin"), os.path.join(d, "fo.bin")
        with open(fin, "wb") as f:
            f.write(struct.pack("<4i", *shape))
            f.write(x.tobytes())
        subprocess.check_call([exe, "fft", fin, fout])
        X = np.fromfile(fout, dtype=np.complex128).reshape(shape)
        np.testing.assert_allclose(X, np.fft.fftn(x, axes=(1, 2, 3)), atol=1e-10 * np.abs(x).sum() / x.size * 100)


@pytest.fixture(scope="module")
def tiny_op():
    return O.build_operator((4, 4, 4), 0.5, 2 * np.pi, 5)[3]


@pytest.mark.parametrize("gamma", [1e-3, 1e-5])
@pytest.mark.parametrize("fmt", ["tucker3d", "tt3d", "tucker4d", "tt4d", "htucker4d"])
def test_compressor_error_bound_and_ranks(drv, tiny_op, fmt, gamma):
    Th = tiny_op
    ranks, rel, mx, sec, data = compress(drv, Th, fmt, gamma)
    R = reconstruct(fmt, ranks, data, Th.shape[1:], Th.shape[0])
    if fmt.endswith("3d"):
        errs = [np.linalg.norm(R[p] - Th[p]) / np.linalg.norm(Th[p]) for p in range(Th.shape[0])]
        assert max(errs) <= gamma * (1 + 1e-6)
        assert abs(mx - max(errs)) <= 1e-3 * max(errs) + 1e-7  # norm identity: ~sqrt(eps) absolute
        true = np.linalg.norm(R - Th) / np.linalg.norm(Th)
    else:
        true = np.linalg.norm(R - Th) / np.linalg.norm(Th)
        assert true <= gamma * (1 + 1e-6)
    assert abs(rel - true) <= 1e-3 * true + 1e-7
    ref = O.ranks(O.compress(Th, fmt, gamma))
    if fmt.endswith("3d"):
        mine = np.array(ranks).reshape(len(ref), -1)
        assert np.all(np.abs(mine - np.array(ref)) <= 1)
    else:
        assert np.all(np.abs(np.array(ranks) - np.array(ref)) <= 1)


def test_compressor_recovers_planted_structure(drv):
    """Exact low-rank inputs: the truncation must stop at the planted ranks.  The library
    finds singular values through FP64 Gram matrices, whose eigenvalue noise is about
    eps * lambda_max, so ranks are resolvable for gamma down to about 1e-7; use 1e-6."""
    rng = np.random.default_rng(3)
    R = lambda s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    n = (6, 8, 10)
    # per-direction Tucker with ranks (2,3,4)
    T = np.stack([np.einsum("abc,xa,yb,zc->xyz", R((2, 3, 4)), R((6, 2)), R((8, 3)), R((10, 4))) for _ in range(3)])
    ranks, *_ = compress(drv, T, "tucker3d", 1e-6)
    assert ranks == [2, 3, 4] * 3
    # 4-D Tucker with ranks (2,3,2,3)
    T4 = np.einsum("abcd,xa,yb,zc,pd->pxyz", R((2, 3, 2, 3)), R((6, 2)), R((8, 3)), R((10, 2)), R((7, 3)))
    ranks, *_ = compress(drv, T4, "tucker4d", 1e-6)
    assert ranks == [2, 3, 2, 3]
    # TT with ranks (2, 3, 2)
    Tt = np.einsum("xa,ayb,bzc,pc->pxyz", R((6, 2)), R((2, 8, 3)), R((3, 10, 2)), R((7, 2)))
    ranks, *_ = compress(drv, Tt, "tt4d", 1e-6)
    assert ranks == [2, 3, 2]
    # H-Tucker with leaves (2,3,2,3) and r12 = r34 = 4
    G = np.einsum("abi,ij,cdj->abcd", R((2, 3, 4)), R((4, 4)), R((2, 3, 4)))
    Th = np.einsum("abcd,xa,yb,zc,pd->pxyz", G, R((6, 2)), R((8, 3)), R((10, 2)), R((7, 3)))
    ranks, *_ = compress(drv, Th, "htucker4d", 1e-6)
    assert ranks == [2, 3, 2, 3, 4, 4]
