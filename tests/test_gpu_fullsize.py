"""GPU parity at the full sizes of the batching and precision workloads, in the
launch configuration the bench times (tile plan from tfmm_autotune, all RHS in
one translation), on sampled directions the FP64 oracle computes one by one:
the exact operator of each sampled direction is sampled (Eq. (7)), FFT'ed and
applied to every RHS (Eq. (5)); the GPU result of each RHS must be within
10 gamma + 1e-6 of it (relative L2 per direction and RHS).
"""
import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    import paper_2010_00520_amd as P

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = P.Context(0)
    yield c
    c.close()


def _check_sampled(ctx, w, fmt, prec, n_sample, seed):
    A_np = synth.patterns_for(w)
    A = torch.from_numpy(A_np).cuda()
    B = torch.zeros_like(A)
    op = ctx.setup(K=w.K, box=w.box, k=w.k, L=w.L, fmt=fmt, tol=w.tol, prec=prec)
    assert op.info()["n_dir"] == w.n_dir
    ctx.autotune(op, nrhs=w.nrhs, reps=3)
    ctx.translate(op, A, B)
    torch.cuda.synchronize()
    got = B.cpu().numpy().astype(np.complex128)
    op.release()
    khat, _ = O.directions(w.L, w.grid)
    rng = np.random.default_rng(seed)
    # first and last directions plus a seeded sample in between
    sample = sorted({0, w.n_dir - 1} | {int(p) for p in rng.choice(w.n_dir, size=n_sample, replace=False)})
    worst = 0.0
    for p in sample:
        Th = O.fft_operator(O.sample_operator(w.K, w.box, w.k, w.L, khat[p:p + 1]))
        ref = O.translate_fft(A_np[:, p:p + 1].astype(np.complex128), Th)
        for s in range(w.nrhs):
            e = O.rel_l2(got[s, p], ref[s, 0])
            worst = max(worst, e)
            assert e <= 10 * w.tol + 1e-6, (fmt, prec, p, s, e)
    return worst


@pytest.mark.parametrize("fmt", ["tt3d", "tucker4d"])
def test_batching_workload_full_size(ctx, fmt):
    """24^3 boxes (48^3 FFT grid), 162 directions, 8 RHS, gamma = 1e-4, bf16x3."""
    w = synth.BATCHING
    assert (w.K, w.n_dir, w.nrhs) == ((24, 24, 24), 162, 8)
    _check_sampled(ctx, w, fmt, "bf16x3", 4, 11)


@pytest.mark.parametrize("fmt,prec", [("htucker4d", "fp32"), ("tt4d", "bf16x3")])
def test_precision_workload_full_size(ctx, fmt, prec):
    """128x8x8 boxes (256x16x16 FFT grid, 256-point x lines), 338 directions, 4 RHS,
    gamma = 1e-4."""
    w = synth.PRECISION
    assert (w.K, w.n_dir, w.nrhs) == ((128, 8, 8), 338, 4)
    _check_sampled(ctx, w, fmt, prec, 4, 12)
