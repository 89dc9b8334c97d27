"""GPU parity of the far-field matvec around the translation: point-dipole
patterns (Eq. (3), FP64 setup, stored complex64), aggregation into box
radiation patterns (Eq. (4)), projection onto the basis with the direction
quadrature (Eq. (6)), and the whole far-field product
(aggregate -> translate -> project), all through the C ABI, against the FP64
oracle; and, with the exact operator, against the plain pairwise sum of the
dyadic Green's function the expansion approximates.
"""
import numpy as np
import pytest

import oracle as O
from oracle import farfield_oracle as F
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


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.complex64))).cuda()


@pytest.mark.parametrize("K,n", [((8, 8, 8), 700), ((16, 8, 8), 1500)])
def test_aggregate_and_project_match_oracle(ctx, K, n):
    box, k, L = 0.5, synth.K0, 5
    pos, u = synth.sphere_dipoles(K, box, n, 11)
    op = ctx.setup(K=K, box=box, k=k, L=L, fmt="full")
    b = ctx.basis(op, pos, u)
    ndir = op.info()["n_dir"]
    khat, w = O.directions(L)
    Pp = F.dipole_patterns(khat, k, pos, u, box, K, +1)
    Pm = F.dipole_patterns(khat, k, pos, u, box, K, -1)
    I = synth.current_vector(n, 3, 12)
    A = torch.zeros((6, ndir) + K, dtype=torch.complex64, device="cuda")
    ctx.aggregate(b, _dev(I), A)
    Bn = synth.gaussian_patterns((6, ndir) + K, 13)
    y = torch.zeros((3, n), dtype=torch.complex64, device="cuda")
    ctx.disaggregate(b, _dev(Bn), y)
    torch.cuda.synchronize()
    refA = F.aggregate(Pp, I, pos, box, K)
    refy = F.disaggregate(Pm, Bn.astype(np.complex128), w, pos, box, K)
    assert O.rel_l2(A.cpu().numpy().astype(np.complex128), refA) < 2e-6
    assert O.rel_l2(y.cpu().numpy().astype(np.complex128), refy) < 2e-6
    b.release()
    op.release()


@pytest.mark.parametrize("fmt,tol", [("full", 0.0), ("tucker3d", 1e-4), ("htucker4d", 1e-4)])
def test_farfield_matvec(ctx, fmt, tol):
    """aggregate -> translate -> project on the GPU against the oracle's far-field
    product with the exact operator: FP32 arithmetic for the uncompressed
    operator, 10 gamma + 1e-6 for the compressed ones."""
    K, box, k, L, n = (8, 8, 8), 0.5, synth.K0, 8, 900
    pos, u = synth.sphere_dipoles(K, box, n, 21)
    op = ctx.setup(K=K, box=box, k=k, L=L, fmt=fmt, tol=tol if tol else 1e-4)
    b = ctx.basis(op, pos, u)
    I = synth.current_vector(n, 2, 22)
    y = torch.zeros((2, n), dtype=torch.complex64, device="cuda")
    ctx.farfield_matvec(op, b, _dev(I), y)
    torch.cuda.synchronize()
    khat, _ = O.directions(L)
    That = O.fft_operator(O.sample_operator(K, box, k, L, khat))
    ref = F.farfield_matvec(I.astype(np.complex128), pos, u, K, box, k, L, That)
    err = O.rel_l2(y.cpu().numpy().astype(np.complex128), ref)
    assert err < (2e-5 if fmt == "full" else 10 * tol + 1e-6), err
    b.release()
    op.release()


def test_farfield_matvec_matches_dyadic_pair_sum(ctx):
    """With dipoles near their box centres the plane-wave expansion at L = 12
    reproduces the far-pair sum of the dyadic Green's function to ~1e-7 in FP64;
    the GPU product (FP32) must be within 2e-5 of it."""
    K, box, k, L, n = (8, 8, 8), 0.5, synth.K0, 12, 300
    pos, u = synth.dipoles_near_centres(K, box, n, 31)
    op = ctx.setup(K=K, box=box, k=k, L=L, fmt="full")
    b = ctx.basis(op, pos, u)
    I = synth.current_vector(n, 1, 32)
    y = torch.zeros((1, n), dtype=torch.complex64, device="cuda")
    ctx.farfield_matvec(op, b, _dev(I), y)
    torch.cuda.synchronize()
    ref = F.farfield_direct(I.astype(np.complex128), pos, u, K, box, k)
    assert O.rel_l2(y.cpu().numpy().astype(np.complex128), ref) < 2e-5
    b.release()
    op.release()
