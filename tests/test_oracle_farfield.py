"""Pins of the far-field matvec oracle (aggregation Eq. (4), projection Eq. (6),
point-dipole patterns Eq. (3)) against what the mathematics fixes:

* with the exact operator, aggregation + translation + projection reproduces the
  plain pairwise sum of the dyadic Green's function over far box pairs
  (Gegenbauer addition theorem with the transverse projection), with an error
  that falls as L grows; a wrong phase sign, a dropped conjugate, a missing
  weight or a swapped component gives an O(1) error;
* the dyadic Green's function against finite differences of exp(-jkR)/R;
* reciprocity: the far-field matrix is symmetric (u_m.G.u_n = u_n.G.u_m).
"""
import math

import numpy as np

import oracle as O
from oracle import farfield_oracle as F
import synth


def test_dyadic_green_finite_differences():
    k = 2 * math.pi
    R0 = np.array([0.9, -0.4, 0.7])
    h = 1e-4
    g = lambda R: np.exp(-1j * k * np.linalg.norm(R)) / np.linalg.norm(R)
    H = np.zeros((3, 3), complex)
    for i in range(3):
        for j in range(3):
            ei, ej = np.eye(3)[i] * h, np.eye(3)[j] * h
            H[i, j] = (g(R0 + ei + ej) - g(R0 + ei - ej) - g(R0 - ei + ej) + g(R0 - ei - ej)) / (4 * h * h)
    ref = g(R0) * np.eye(3) + H / k ** 2
    np.testing.assert_allclose(F.dyadic_green(R0, k), ref, rtol=1e-6, atol=1e-8)


def _fmm_vs_direct(L, K=(4, 4, 4), n=40, seed=3):
    box, k = 0.5, synth.K0
    pos, u = synth.dipoles_near_centres(K, box, n, seed)
    I = synth.current_vector(n, 2, seed + 1).astype(np.complex128)
    khat, _ = O.directions(L)
    That = O.fft_operator(O.sample_operator(K, box, k, L, khat))
    y = F.farfield_matvec(I, pos, u, K, box, k, L, That)
    ref = F.farfield_direct(I, pos, u, K, box, k)
    return O.rel_l2(y, ref)


def test_farfield_matvec_matches_dyadic_pair_sum():
    # measured: L = 6, 8, 10, 14 -> 5.5e-4, 1.7e-5, 7.7e-7, 2.8e-9
    e8, e14 = _fmm_vs_direct(8), _fmm_vs_direct(14)
    assert e8 < 1e-4, e8
    assert e14 < 1e-7, e14


def test_farfield_matrix_is_symmetric():
    K, box, k, L, n = (4, 4, 4), 0.5, synth.K0, 8, 12
    pos, u = synth.dipoles_near_centres(K, box, n, 9)
    khat, _ = O.directions(L)
    That = O.fft_operator(O.sample_operator(K, box, k, L, khat))
    Z = F.farfield_matvec(np.eye(n), pos, u, K, box, k, L, That)   # column n = response to I = e_n
    np.testing.assert_allclose(Z, Z.T, rtol=1e-10, atol=1e-12 * np.abs(Z).max())


def test_aggregation_sums_box_members():
    """Eq. (4): each box holds the sum over its members; empty boxes hold zero."""
    K, box, k, L = (4, 4, 4), 0.5, synth.K0, 3
    pos, u = synth.dipoles_near_centres(K, box, 30, 5)
    khat, _ = O.directions(L)
    P = F.dipole_patterns(khat, k, pos, u, box, K)
    I = synth.current_vector(30, 1, 6).astype(np.complex128)
    A = F.aggregate(P, I, pos, box, K)
    v = F.box_index(pos, box, K)
    total = np.einsum("pnc,n->cp", P, I[0])
    np.testing.assert_allclose(A.sum(axis=(2, 3, 4)), total, rtol=1e-12)
    occupied = np.zeros(K, bool)
    occupied[tuple(v.T)] = True
    assert np.all(A[:, :, ~occupied] == 0)
