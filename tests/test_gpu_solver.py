"""GPU parity of the iterative solution of Eq. (2): (Zn + Zfar) I = V by TFQMR
on the device (FP64 Krylov vectors, complex64 operator products), with Zfar the
library's far-field product and Zn a synthetic near-field matrix (CSR), against
the oracle's TFQMR on the dense FP64 matrix of the same system.
"""
import numpy as np
import pytest

import oracle as O
from oracle import farfield_oracle as F
from oracle import tfqmr_oracle as Q
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


def _dense(rp, ci, val, n):
    Z = np.zeros((n, n), complex)
    for m in range(n):
        Z[m, ci[rp[m]:rp[m + 1]]] = val[rp[m]:rp[m + 1]]
    return Z


def test_near_matvec_matches_csr(ctx):
    K, box, n = (8, 8, 8), 0.5, 400
    pos, u = synth.dipoles_near_centres(K, box, n, 41)
    rp, ci, val = synth.near_field_csr(F.box_index(pos, box, K), K, 42, 3 + 1j, 0.3)
    nf = ctx.near(n, rp, ci, val)
    x = synth.current_vector(n, 2, 43)
    y = torch.zeros((2, n), dtype=torch.complex64, device="cuda")
    ctx.near_matvec(nf, torch.from_numpy(x).cuda(), y)
    torch.cuda.synchronize()
    ref = x.astype(np.complex128) @ _dense(rp, ci, val, n).T
    assert O.rel_l2(y.cpu().numpy().astype(np.complex128), ref) < 1e-6
    nf.release()


@pytest.mark.parametrize("fmt", ["full", "htucker4d"])
def test_tfqmr_solve_matches_oracle(ctx, fmt):
    K, box, k, L, n = (8, 8, 8), 0.5, synth.K0, 8, 300
    pos, u = synth.dipoles_near_centres(K, box, n, 51)
    khat, _ = O.directions(L)
    That = O.fft_operator(O.sample_operator(K, box, k, L, khat))
    Zfar = F.farfield_matvec(np.eye(n), pos, u, K, box, k, L, That).T   # column j = Zfar e_j
    s = np.abs(Zfar).sum(axis=1).max()
    rp, ci, val = synth.near_field_csr(F.box_index(pos, box, K), K, 52, 2.0 * s * (1 + 0.5j), 0.05 * s)
    Z = _dense(rp, ci, val, n) + Zfar
    V = synth.current_vector(n, 1, 53)[0]
    x_or, it_or, _, _ = Q.tfqmr(lambda v: Z @ v, V.astype(np.complex128), tol=1e-6, maxit=200)
    op = ctx.setup(K=K, box=box, k=k, L=L, fmt=fmt, tol=1e-4)
    b = ctx.basis(op, pos, u)
    nf = ctx.near(n, rp, ci, val)
    Vd = torch.from_numpy(V).cuda()
    Id = torch.zeros_like(Vd)
    it, rr = ctx.solve_tfqmr(op, b, nf, Vd, Id, tol=1e-6, maxit=200)
    x = Id.cpu().numpy().astype(np.complex128)
    print(f"\n[tfqmr] {fmt}: GPU {it} iterations, rel res {rr:.2e}; oracle {it_or} iterations", flush=True)
    assert rr <= 1e-6
    # the GPU operator differs from the exact one by FP32 rounding (full) or the
    # compression (gamma = 1e-4), so the solutions agree to that level
    tol = 1e-5 if fmt == "full" else 1e-3
    assert O.rel_l2(x, x_or) < tol
    assert np.linalg.norm(V - Z @ x) / np.linalg.norm(V) < tol
    nf.release()
    b.release()
    op.release()
