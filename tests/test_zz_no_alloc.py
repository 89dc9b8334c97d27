"""tfmm_translate_noalloc, the allocation-free entry point: the same translation
as tfmm_translate with every byte of scratch in the library's fixed device array.

Its results must equal tfmm_translate's bit for bit (the same kernels; the
direction chunk may differ, and each direction's arithmetic does not depend on
the chunk), on two calls in a row, the second with a smaller input, for the
fused path, the three-pass path with per-call core contractions, and a
translation whose scratch exceeds the fixed array (so the chunk shrinks).
A translation that cannot fit even one direction is refused before any work.
"""
import numpy as np
import pytest

import synth
from factor_layout import random_factors

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


CASES = [
    # fmt, K, L, ranks, (nrhs first call, nrhs second call)
    ("tucker3d", (16, 16, 16), 4, None, (3, 1)),          # fused path
    ("tucker4d", (16, 8, 8), 3, (6, 5, 4, 9), (4, 2)),    # three-pass + core contraction, z-major copies
    ("tt4d", (24, 24, 24), 8, (9, 40, 30), (8, 3)),       # 162 directions x 8 RHS: 573 MB of half spectrum
]


@pytest.mark.parametrize("fmt,K,L,ranks,nr", CASES, ids=[c[0] + "-" + "x".join(map(str, c[1])) for c in CASES])
def test_noalloc_matches_translate(ctx, fmt, K, L, ranks, nr):
    print(f"\n[noalloc] {fmt} K={K} L={L} nrhs={nr}", flush=True)
    n = tuple(2 * k for k in K)
    ndir = (L + 1) * 2 * (L + 1)
    rk, data, _ = random_factors(fmt, n, ndir, np.random.default_rng(31), ranks)
    op = ctx.import_factors(K, L, fmt, rk, data)
    for call, nrhs in enumerate(nr):
        A = torch.from_numpy(synth.gaussian_patterns((nrhs, ndir) + K, 40 + call)).cuda()
        B_ref = torch.zeros_like(A)
        B_na = torch.full_like(A, float("nan"))
        ctx.translate(op, A, B_ref)
        ctx.translate_noalloc(op, A, B_na)
        torch.cuda.synchronize()
        assert torch.equal(B_na, B_ref), f"call {call}: allocation-free result differs"
    op.release()


def test_noalloc_refuses_what_cannot_fit(ctx):
    """TT-4D on 32^3 boxes with 1058 directions and r2 = 256: the per-direction
    slices alone (1058 x 64 x 256 complex64 = 139 MB) exceed the fixed scratch."""
    import paper_2010_00520_amd as P

    K, L, ranks = (32, 32, 32), 22, (8, 256, 16)
    n = tuple(2 * k for k in K)
    ndir = (L + 1) * 2 * (L + 1)
    rk, data, _ = random_factors("tt4d", n, ndir, np.random.default_rng(2), ranks)
    op = ctx.import_factors(K, L, "tt4d", rk, data)
    A = torch.zeros((1, ndir) + K, dtype=torch.complex64, device="cuda")
    B = torch.full_like(A, 7.0)
    with pytest.raises(P.TfmmError) as e:
        ctx.translate_noalloc(op, A, B)
    assert e.value.status == 2 and "fixed scratch" in e.value.detail
    torch.cuda.synchronize()
    assert bool((B == 7.0).all())  # nothing was enqueued
    op.release()
