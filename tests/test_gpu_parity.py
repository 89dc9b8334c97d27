"""GPU parity: libtfmm's HIP translation against the FP64 oracle, through the C ABI.

Two kinds of checks:
* arithmetic parity -- the same synthetic factors go to the oracle's restoration
  (Figs. 3-4) + Eq. (5) and to the library via tfmm_op_import; the FP32 GPU
  result must match to 2e-5 relative L2 (FP32 FFTs of length <= 64 and
  FP32 contractions of length <= 64 stay near 1e-6);
* end-to-end parity -- the library samples, FFTs and compresses the operator
  itself (tfmm_setup_compressed); its result must match the exact FP64
  translation (the plain pairwise sum, or the FFT form with the exact
  operator) within 10*gamma + 1e-6.
"""
import math
import zlib

import numpy as np
import pytest

import oracle as O
import synth
from factor_layout import random_factors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ARITH_TOL = 2e-5


def seed_of(*parts):
    """Deterministic seed (str hashes are salted per process)."""
    return zlib.crc32(repr(parts).encode())


@pytest.fixture(scope="module")
def ctx():
    import paper_2010_00520_amd as P

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = P.Context(0)
    yield c
    c.close()


def gpu_translate(ctx, op, A):
    Ad = torch.from_numpy(np.ascontiguousarray(A.astype(np.complex64))).to("cuda")
    Bd = torch.zeros_like(Ad)
    ctx.translate(op, Ad, Bd)
    torch.cuda.synchronize()
    return Bd.cpu().numpy().astype(np.complex128)


def test_full_tiny_matches_direct_sum(ctx):
    w = synth.TINY
    op = ctx.setup(K=w.K, box=w.box, k=w.k, L=w.L, fmt="full")
    info = op.info()
    assert info["n_dir"] == 72 and info["L"] == 5
    A = synth.patterns_for(w, nrhs=2)
    khat, _ = O.directions(w.L)
    T = O.sample_operator(w.K, w.box, w.k, w.L, khat)
    ref = O.translate_direct(A, T)
    got = gpu_translate(ctx, op, A)
    assert O.rel_l2(got, ref) < ARITH_TOL
    op.release()


@pytest.mark.parametrize("K", [(8, 8, 8), (8, 12, 4), (4, 16, 8)])
@pytest.mark.parametrize("fmt", ["full", "tucker3d", "tt3d", "tucker4d", "tt4d", "htucker4d"])
def test_import_arithmetic_parity(ctx, fmt, K):
    n = tuple(2 * k for k in K)
    L = 3
    ndir = (L + 1) * 2 * (L + 1)
    rng = np.random.default_rng(seed_of(fmt, K))
    ranks = {"tucker4d": (5, 6, 3, 7), "tt4d": (5, 9, 7), "htucker4d": (4, 5, 3, 6, 9, 8)}.get(fmt)
    rk, data, comp = random_factors(fmt, n, ndir, rng, ranks)
    op = ctx.import_factors(K, L, fmt, rk, data)
    A = synth.gaussian_patterns((2, ndir) + tuple(K), 7)
    ref = O.translate_compressed(A, comp)
    got = gpu_translate(ctx, op, A)
    assert O.rel_l2(got, ref) < ARITH_TOL, (fmt, K)
    # per-RHS and per-direction check too (a wrong direction index would hide in the global norm)
    for s in range(2):
        for p in (0, ndir // 2, ndir - 1):
            assert O.rel_l2(got[s, p], ref[s, p]) < 5 * ARITH_TOL
    op.release()


@pytest.mark.parametrize("fmt", ["tucker3d", "tt3d", "tucker4d", "tt4d", "htucker4d"])
def test_setup_end_to_end_tiny(ctx, fmt):
    w = synth.TINY
    gamma = 1e-4
    op = ctx.setup(K=w.K, box=w.box, k=w.k, L=w.L, fmt=fmt, tol=gamma)
    info = op.info()
    assert info["rel_err_fro"] <= gamma * 1.05
    A = synth.patterns_for(w, nrhs=1)
    khat, _ = O.directions(w.L)
    T = O.sample_operator(w.K, w.box, w.k, w.L, khat)
    ref = O.translate_direct(A, T)
    got = gpu_translate(ctx, op, A)
    assert O.rel_l2(got, ref) <= 10 * gamma + 1e-6
    op.release()


def test_plain_16cubed_tucker3d_end_to_end(ctx):
    w = synth.PLAIN
    op = ctx.setup(K=w.K, box=w.box, k=w.k, L=w.L, fmt="tucker3d", tol=w.tol)
    info = op.info()
    assert info["n_dir"] == 242
    assert info["rel_err_fro"] <= w.tol * 1.05
    A = synth.patterns_for(w)
    _, _, _, Th = O.build_operator(w.K, w.box, w.k, w.L)
    ref = O.translate_fft(A, Th)
    got = gpu_translate(ctx, op, A)
    err = O.rel_l2(got, ref)
    assert err <= 10 * w.tol + 1e-6
    # every direction individually within the bound as well
    per = [O.rel_l2(got[0, p], ref[0, p]) for p in range(0, 242, 11)]
    assert max(per) <= 10 * w.tol + 1e-6
    op.release()


def test_plain_16cubed_full_matches_exact(ctx):
    w = synth.PLAIN
    op = ctx.setup(K=w.K, box=w.box, k=w.k, L=w.L, fmt="full")
    A = synth.patterns_for(w)
    _, _, _, Th = O.build_operator(w.K, w.box, w.k, w.L)
    got = gpu_translate(ctx, op, A)
    assert O.rel_l2(got, O.translate_fft(A, Th)) < ARITH_TOL
    op.release()


def test_invalid_arguments(ctx):
    import paper_2010_00520_amd as P

    op = ctx.setup(K=(4, 4, 4), box=0.5, L=3, fmt="full")
    A = torch.zeros((1, 32, 4, 4, 4), dtype=torch.complex64, device="cuda")
    with pytest.raises(P.TfmmError) as e:
        ctx.translate(op, A, A)  # aliasing
    assert e.value.status == 1
    with pytest.raises(P.TfmmError) as e:
        ctx.setup(K=(5, 4, 4), box=0.5, L=3, fmt="full")
    assert e.value.status == 2
    with pytest.raises(P.TfmmError) as e:
        ctx.import_factors((4, 4, 4), 3, "tucker4d", [2, 2, 2], np.zeros(10))
    assert e.value.status == 1
    op.release()


@pytest.mark.parametrize("fmt", ["full", "tucker3d", "tt3d", "tt4d", "htucker4d"])
def test_three_pass_and_fused_agree(fmt):
    """The fused kernel (cubic grids <= 32^3) and the three-pass pipeline compute the same
    translation; both are checked against the oracle on the same imported factors."""
    import os

    import paper_2010_00520_amd as P

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    K, L = (16, 16, 16), 4
    n = (32, 32, 32)
    ndir = (L + 1) * 2 * (L + 1)
    rng = np.random.default_rng(99)
    ranks = {"tt4d": (9, 21, 11), "htucker4d": (7, 8, 6, 9, 15, 13)}.get(fmt)
    rk, data, comp = random_factors(fmt, n, ndir, rng, ranks)
    A = synth.gaussian_patterns((3, ndir) + K, 5)
    ref = O.translate_compressed(A, comp)
    outs = []
    for no_fused in ("0", "1"):
        os.environ["TFMM_NO_FUSED"] = no_fused
        try:
            c = P.Context(0)
        finally:
            os.environ.pop("TFMM_NO_FUSED", None)
        op = c.import_factors(K, L, fmt, rk, data)
        outs.append(gpu_translate(c, op, A))
        op.release()
        c.close()
    for got in outs:
        assert O.rel_l2(got, ref) < ARITH_TOL
    assert O.rel_l2(outs[0], outs[1]) < ARITH_TOL


# Split-BF16 restoration: each FP32 operand x = hi + lo + r with hi = bf16(x),
# lo = bf16(x - hi) (both round to nearest), so |r| <= 2^-18 |x|; the dropped
# lo*lo term is <= 2^-18 |x y| as well, so a product carries <= ~3 * 2^-18 =
# 1.1e-5 relative error.  Three chained contractions (Fig. 3a / Fig. 4) then
# stay below ~3.5e-5 of the restored operator, to which the FP32 FFTs add
# ~1e-6; 1e-4 leaves a margin for the norm of sums of random terms.
BF_TOL = 1e-4


@pytest.mark.parametrize("K", [(8, 8, 8), (8, 12, 4)])
@pytest.mark.parametrize("fmt", ["tucker3d", "tt3d", "tucker4d", "tt4d", "htucker4d"])
def test_import_bf16x3_parity(ctx, fmt, K):
    n = tuple(2 * k for k in K)
    L = 3
    ndir = (L + 1) * 2 * (L + 1)
    rng = np.random.default_rng(seed_of("bf", fmt, K))
    ranks = {"tucker4d": (5, 6, 3, 7), "tt4d": (5, 9, 7), "htucker4d": (4, 5, 3, 6, 9, 8)}.get(fmt)
    rk, data, comp = random_factors(fmt, n, ndir, rng, ranks)
    op = ctx.import_factors(K, L, fmt, rk, data, prec="bf16x3")
    assert op.info()["prec"] == 1
    A = synth.gaussian_patterns((2, ndir) + tuple(K), 8)
    ref = O.translate_compressed(A, comp)
    got = gpu_translate(ctx, op, A)
    err = O.rel_l2(got, ref)
    assert err < BF_TOL, (fmt, K, err)
    # the split arithmetic must actually be more accurate than plain bf16 (~4e-3)
    for s in range(2):
        for p in (0, ndir - 1):
            assert O.rel_l2(got[s, p], ref[s, p]) < 5 * BF_TOL
    op.release()


def test_plain_16cubed_tucker3d_bf16x3_end_to_end(ctx):
    w = synth.PLAIN
    op = ctx.setup(K=w.K, box=w.box, k=w.k, L=w.L, fmt="tucker3d", tol=w.tol, prec="bf16x3")
    A = synth.patterns_for(w)
    _, _, _, Th = O.build_operator(w.K, w.box, w.k, w.L)
    got = gpu_translate(ctx, op, A)
    assert O.rel_l2(got, O.translate_fft(A, Th)) <= 10 * w.tol + 1e-6
    op.release()


# x axes of 64 and 128 boxes (FFT lengths 128 and 256, split 16 x NB in LDS)
@pytest.mark.parametrize("K", [(64, 4, 8), (128, 8, 8), (64, 32, 4)])
@pytest.mark.parametrize("fmt", ["full", "tucker3d", "tt3d", "tt4d", "htucker4d"])
def test_long_x_import_parity(ctx, fmt, K):
    n = tuple(2 * k for k in K)
    L = 3
    ndir = (L + 1) * 2 * (L + 1)
    rng = np.random.default_rng(seed_of("lx", fmt, K))
    ranks = {"tt4d": (6, 10, 7), "htucker4d": (6, 5, 4, 7, 12, 9)}.get(fmt)
    rk, data, comp = random_factors(fmt, n, ndir, rng, ranks)
    op = ctx.import_factors(K, L, fmt, rk, data)
    A = synth.gaussian_patterns((2, ndir) + tuple(K), 9)
    ref = O.translate_compressed(A, comp)
    got = gpu_translate(ctx, op, A)
    assert O.rel_l2(got, ref) < ARITH_TOL, (fmt, K)
    for s in range(2):
        for p in (0, ndir // 3, ndir - 1):
            assert O.rel_l2(got[s, p], ref[s, p]) < 5 * ARITH_TOL
    op.release()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_long_x_setup_end_to_end(ctx, prec):
    """An elongated 64 x 4 x 4 box grid, sampled and compressed by the library,
    against the exact FP64 FFT-form translation."""
    K, box, L, gamma = (64, 4, 4), 0.5, 5, 1e-4
    op = ctx.setup(K=K, box=box, k=2 * math.pi, L=L, fmt="tt3d", tol=gamma, prec=prec)
    _, _, _, Th = O.build_operator(K, box, 2 * math.pi, L)
    A = synth.gaussian_patterns((1, Th.shape[0]) + K, 10)
    got = gpu_translate(ctx, op, A)
    assert O.rel_l2(got, O.translate_fft(A, Th)) <= 10 * gamma + 1e-6
    op.release()


def test_unsupported_grids_rejected(ctx):
    import paper_2010_00520_amd as P

    for K in [(64, 64, 4), (256, 4, 4), (4, 64, 4), (6, 4, 4)]:
        with pytest.raises(P.TfmmError) as e:
            ctx.setup(K=K, box=0.5, L=3, fmt="full")
        assert e.value.status == 2, K


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("no_fused", ["0", "1"])
@pytest.mark.parametrize("fmt", ["tucker3d", "tucker4d", "htucker4d", "tt3d", "tt4d"])
def test_lds_staged_tucker_restoration(fmt, no_fused, prec):
    """The LDS-staged restoration (block GEMMs through LDS, used when the
    register-chained one does not fit; TFMM_NO_TK2=1 forces it) against the
    oracle, on the fused and the three-pass paths, for the Tucker family and
    the TT formats."""
    import os

    import paper_2010_00520_amd as P

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    K, L = (16, 16, 16), 3
    n = tuple(2 * k for k in K)
    ndir = (L + 1) * 2 * (L + 1)
    rng = np.random.default_rng(seed_of("staged", fmt))
    ranks = {"tucker4d": (9, 11, 7, 13), "htucker4d": (8, 9, 7, 10, 12, 11), "tt4d": (7, 13, 9)}.get(fmt)
    rk, data, comp = random_factors(fmt, n, ndir, rng, ranks)
    old = {k: os.environ.get(k) for k in ("TFMM_NO_TK2", "TFMM_NO_FUSED")}
    os.environ["TFMM_NO_TK2"] = "1"
    os.environ["TFMM_NO_FUSED"] = no_fused
    try:
        c = P.Context(0)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    op = c.import_factors(K, L, fmt, rk, data, prec=prec)
    plan = op.plan()
    assert not plan["register_chained"] and plan["fused"] == (no_fused == "0")
    A = synth.gaussian_patterns((2, ndir) + K, 38)
    ref = O.translate_compressed(A, comp)
    got = gpu_translate(c, op, A)
    tol = 1e-4 if prec == "bf16x3" else ARITH_TOL
    assert O.rel_l2(got, ref) < tol
    for p in (0, ndir // 2, ndir - 1):
        assert O.rel_l2(got[:, p], ref[:, p]) < 5 * tol
    op.release()
    c.close()


@pytest.mark.parametrize("eps", [1.0, 2 - 1j, 2 - 8j])
@pytest.mark.parametrize("K,L", [((4, 4, 4), 5), ((64, 4, 4), 14)])
def test_fp64_sampler_matches_oracle(ctx, K, L, eps):
    """FP64 operator sampling on the device (Eq. (7), readings R1-R3), then the host
    FP64 FFT: the uncompressed operator read back with tfmm_op_export must match the
    oracle's sampled and FFT'ed operator to 1e-12 relative (the FP64 rounding level of
    the spherical-Hankel and Legendre recurrences), and its inverse FFT the spatial
    samples, both per direction.  64 x 4 x 4 boxes at L = 14 reach l > kR for every
    offset, where an unstable recurrence for h_l would show.  Lossy media (Section
    III-A-5, Table IV permittivities) give a complex wavenumber k = k0 sqrt(eps_r):
    at eps_r = 2 - 8j the far samples decay by up to e^-355."""
    w = synth.TINY.with_(K=K, L=L)
    k = w.k * np.sqrt(complex(eps)) if eps != 1.0 else w.k
    op = ctx.setup(K=K, box=w.box, k=k, L=L, fmt="full")
    n = tuple(2 * k for k in K)
    got = op.export().reshape((w.n_dir,) + n)
    op.release()
    khat, _ = O.directions(L)
    T = O.sample_operator(K, w.box, k, L, khat)
    That = O.fft_operator(T)
    assert O.rel_l2(got, That) <= 1e-12
    spatial = np.fft.ifftn(got, axes=(-3, -2, -1))
    for p in range(w.n_dir):
        assert O.rel_l2(got[p], That[p]) <= 1e-12, p
        assert O.rel_l2(spatial[p], T[p]) <= 1e-12, p


@pytest.mark.parametrize("fmt", ["tucker3d", "htucker4d", "tt4d"])
def test_lossy_medium_translation(ctx, fmt):
    """Section III-A-5: translation in a lossy medium (eps_r = 2 - 2j, complex
    wavenumber) through the compressed operator matches the exact FP64 translation
    within 10 gamma + 1e-6, and the loss lowers the stored memory against the same
    grid in the lossless medium eps_r = 2 (Table IV trend)."""
    K, L, tol = (8, 8, 8), 10, 1e-4
    w = synth.TINY.with_(K=K, L=L)
    k_loss = w.k * np.sqrt(2 - 2j)
    op = ctx.setup(K=K, box=0.5, k=k_loss, L=L, fmt=fmt, tol=tol)
    lossless = ctx.setup(K=K, box=0.5, k=w.k * np.sqrt(2.0), L=L, fmt=fmt, tol=tol)
    assert op.info()["bytes_stored"] < lossless.info()["bytes_stored"]
    lossless.release()
    A = synth.patterns_for(w, nrhs=2)
    got = gpu_translate(ctx, op, A)
    op.release()
    khat, _ = O.directions(L)
    for p in (0, 17, 101, w.n_dir - 1):
        Th = O.fft_operator(O.sample_operator(K, 0.5, k_loss, L, khat[p:p + 1]))
        ref = O.translate_fft(A[:, p:p + 1].astype(np.complex128), Th)
        assert O.rel_l2(got[:, p:p + 1], ref) <= 10 * tol + 1e-6, p


def _ctx_with_env(env):
    import os

    import paper_2010_00520_amd as P

    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return P.Context(0)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("K", [(16, 16, 16), (12, 12, 12)])
@pytest.mark.parametrize("fmt", ["tucker4d", "htucker4d"])
def test_formed_x_mode_product_restoration(fmt, K, prec):
    """4-D formats on the three-pass path restore from the x-mode product
    W1 = U1 x_1 C_p formed by a batched GEMM per direction chunk (Fig. 3(a) step
    1 moved ahead of the z-stage); TFMM_NO_W1=1 keeps the product inside the
    z-stage.  Both against the oracle, with an odd r2 and an r3 that leaves a
    partial chunk of 8 core columns."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L = 3
    n = tuple(2 * k for k in K)
    ndir = (L + 1) * 2 * (L + 1)
    rng = np.random.default_rng(seed_of("w1", fmt, K))
    ranks = {"tucker4d": (9, 11, 13, 7), "htucker4d": (10, 9, 13, 8, 12, 11)}[fmt]
    rk, data, comp = random_factors(fmt, n, ndir, rng, ranks)
    A = synth.gaussian_patterns((3, ndir) + K, seed_of("w1A", K))
    ref = O.translate_compressed(A, comp)
    tol = 1e-4 if prec == "bf16x3" else ARITH_TOL
    for env, formed in (({"TFMM_NO_FUSED": "1"}, True), ({"TFMM_NO_FUSED": "1", "TFMM_NO_W1": "1"}, False)):
        c = _ctx_with_env(env)
        op = c.import_factors(K, L, fmt, rk, data, prec=prec)
        plan = op.plan()
        assert not plan["fused"] and plan["register_chained"] and plan["w1_formed"] == formed
        got = gpu_translate(c, op, A)
        assert O.rel_l2(got, ref) < tol, (formed, O.rel_l2(got, ref))
        for s in range(A.shape[0]):
            for p in (0, ndir // 2, ndir - 1):
                assert O.rel_l2(got[s, p], ref[s, p]) < 5 * tol
        op.release()
        c.close()


@pytest.mark.parametrize("fmt", ["tucker4d", "htucker4d", "tt4d", "tt3d"])
def test_bf16x3_per_call_gemms(ctx, fmt):
    """An operator restored in bf16x3 whose factors were compressed at tol >=
    1e-5 forms its per-call GEMMs (4-D cores, formed products) in bf16x3 too;
    imported without a tolerance it keeps them in FP32.  Both within the bf16x3
    arithmetic tolerance of the oracle, and not the same bits (a non-cubic
    grid: the three-pass path, where TT-3D forms its x-y products)."""
    K, L = (24, 12, 12), 3
    n = tuple(2 * k for k in K)
    ndir = (L + 1) * 2 * (L + 1)
    rng = np.random.default_rng(seed_of("bfgemm", fmt))
    ranks = {"tucker4d": (9, 11, 13, 17), "htucker4d": (10, 9, 13, 15, 12, 11), "tt4d": (9, 15, 13)}.get(fmt)
    rk, data, comp = random_factors(fmt, n, ndir, rng, ranks)
    A = synth.gaussian_patterns((2, ndir) + K, seed_of("bfgemmA", fmt))
    ref = O.translate_compressed(A, comp)
    got = {}
    for tol in (0.0, 1e-4):
        op = ctx.import_factors(K, L, fmt, rk, data, prec="bf16x3", tol=tol)
        got[tol] = gpu_translate(ctx, op, A)
        assert O.rel_l2(got[tol], ref) < 1e-4, (tol, O.rel_l2(got[tol], ref))
        op.release()
    assert not np.array_equal(got[0.0], got[1e-4])
