"""Pins for the oracle's directions, multipole rule and translation operator.

Each test checks the oracle against something other than itself: closed
forms, the paper's printed direction counts, the Gegenbauer addition theorem,
or a symmetry that any correct evaluation of Eq. (7) must have.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_gauss_legendre_closed_forms():
    x, w = O.gauss_legendre(2)
    np.testing.assert_allclose(x, [-1 / math.sqrt(3), 1 / math.sqrt(3)], rtol=1e-15)
    np.testing.assert_allclose(w, [1, 1], rtol=1e-15)
    x, w = O.gauss_legendre(3)
    np.testing.assert_allclose(x, [-math.sqrt(0.6), 0, math.sqrt(0.6)], atol=1e-15)
    np.testing.assert_allclose(w, [5 / 9, 8 / 9, 5 / 9], rtol=1e-14)


@pytest.mark.parametrize("L", [5, 10])
def test_direction_grid_quadrature(L):
    khat, w = O.directions(L)
    assert khat.shape == ((L + 1) * 2 * (L + 1), 3)
    np.testing.assert_allclose(np.linalg.norm(khat, axis=1), 1.0, rtol=1e-14)
    np.testing.assert_allclose(w.sum(), 4 * math.pi, rtol=1e-14)
    x, y, z = khat.T
    # exact sphere integrals of low-degree monomials (degree <= 2L+1 is integrated exactly)
    np.testing.assert_allclose(np.sum(w * x * x), 4 * math.pi / 3, rtol=1e-13)
    np.testing.assert_allclose(np.sum(w * x * x * y * y * z * z), 4 * math.pi / 105, rtol=1e-12)
    np.testing.assert_allclose(np.sum(w * z), 0.0, atol=1e-13)
    # ordering: p = i_theta * n_phi + j_phi, theta nodes ascending in cos(theta)
    nphi = 2 * (L + 1)
    cz = khat[::nphi, 2]
    assert np.all(np.diff(cz) > 0)
    np.testing.assert_allclose(khat[1, :2] / np.linalg.norm(khat[1, :2]),
                               [math.cos(2 * math.pi / nphi), math.sin(2 * math.pi / nphi)], rtol=1e-13)


def test_paper_direction_grid_count():
    khat, w = O.directions(14, grid="paper")
    assert khat.shape[0] == 435
    np.testing.assert_allclose(w.sum(), 4 * math.pi, rtol=1e-14)


def test_multipole_rule_matches_printed_direction_counts():
    gold = json.load(open(os.path.join(GOLD, "direction_counts.json")))
    for case in gold["cases"]:
        eps = complex(*case["eps_r"])
        k_abs = 2 * math.pi * abs(np.sqrt(eps))
        L = O.multipole_order(k_abs, case["box"], case["digits"], rounding="floor")
        assert (L + 1) * (2 * L + 1) == case["n_dir"], case


def test_multipole_rule_serving_ceil():
    # 0.5 lambda boxes, 4 digits, rounding up: L = 14 (450 directions on the (L+1) x 2(L+1) grid)
    assert O.multipole_order(2 * math.pi, 0.5, 4, rounding="ceil") == 14


def test_hankel_closed_forms_and_wronskian():
    x = np.array([0.7, 1.0, 3.3, 6.28, 12.0, 40.0])
    np.testing.assert_allclose(O.hankel2(0, x), 1j * np.exp(-1j * x) / x, rtol=1e-14)
    np.testing.assert_allclose(O.hankel2(1, x), np.exp(-1j * x) * (1j / x ** 2 - 1 / x), rtol=1e-13)
    for l in range(1, 15):
        h = O.hankel2(l, x)
        j, y = h.real, -h.imag
        hm = O.hankel2(l - 1, x)
        jm, ym = hm.real, -hm.imag
        # DLMF 10.50.3: j_l y_{l-1} - j_{l-1} y_l = 1/x^2
        np.testing.assert_allclose(j * ym - jm * y, 1 / x ** 2, rtol=1e-9)


def test_legendre_values():
    t = np.linspace(-1, 1, 11)
    np.testing.assert_allclose(O.legendre(2, t), (3 * t * t - 1) / 2, atol=1e-15)
    np.testing.assert_allclose(O.legendre(3, t), (5 * t ** 3 - 3 * t) / 2, atol=1e-15)
    for l in range(20):
        assert abs(O.legendre(l, 1.0) - 1) < 1e-14
        assert abs(O.legendre(l, -1.0) - (-1) ** l) < 1e-14


def _addition_error(L, X, d, k=2 * math.pi):
    khat, w = O.directions(L)
    exact = np.exp(-1j * k * np.linalg.norm(X + d)) / np.linalg.norm(X + d)
    TL = O.operator_value(khat, X[None, :], k, L)
    approx = -(1j * k / (4 * math.pi)) * np.sum(w * np.exp(-1j * k * khat @ d) * TL)
    return abs(approx - exact) / abs(exact)


def test_addition_theorem_pins_equation7():
    """Gegenbauer + plane-wave expansion: the plane-wave translation of Eq. (7) reproduces
    exp(-jk|X+d|)/|X+d| for |d| < |X|, with an error that falls as L grows.  A wrong sign of
    (-j)^l, a missing l = 0 term, the wrong Hankel kind or a missing (2l+1) all give O(1) errors."""
    a = 0.5
    rng = np.random.default_rng(7)
    Xs = [np.array([2, 2, 0.0]) * a, np.array([3, -2, 2.0]) * a, np.array([2, 0, 0.0]) * a]
    ds = [rng.uniform(-a / 2, a / 2, 3) - rng.uniform(-a / 2, a / 2, 3) for _ in range(4)]
    e8 = max(_addition_error(8, X, d) for X in Xs for d in ds)
    e14 = max(_addition_error(14, X, d) for X in Xs for d in ds)
    assert e8 < 2e-2
    assert e14 < 1e-4
    assert e14 < e8 / 100


def test_operator_antipodal_symmetry():
    rng = np.random.default_rng(3)
    khat = rng.standard_normal((20, 3))
    khat /= np.linalg.norm(khat, axis=1, keepdims=True)
    R = rng.uniform(-3, 3, (20, 3))
    t1 = O.operator_value(-khat, R, 2 * math.pi, 9)
    t2 = O.operator_value(khat, -R, 2 * math.pi, 9)
    np.testing.assert_allclose(t1, t2, rtol=1e-13)


def test_near_rules():
    D, V = O.offset_grid((4, 4, 4))
    near = O.near_mask(D, "cheb", 1)
    assert int(np.sum(near & V)) == 27
    # kappa = 4: 4|d|^2 < 48  <=>  |d|^2 < 12 -> integer offsets with |d|^2 <= 11
    nk = O.near_mask(D, "kappa", 4.0)
    count = sum(1 for x in range(-3, 4) for y in range(-3, 4) for z in range(-3, 4) if x * x + y * y + z * z <= 11)
    assert int(np.sum(nk & V)) == count


def test_sampled_operator_structure():
    K = (3, 4, 5)
    khat, _ = O.directions(3)
    T = O.sample_operator(K, 0.5, 2 * math.pi, 3, khat)
    assert T.shape == (khat.shape[0], 6, 8, 10)
    # unused slot m_i = K_i and the near boxes are zero
    assert np.all(T[:, 3, :, :] == 0) and np.all(T[:, :, 4, :] == 0) and np.all(T[:, :, :, 5] == 0)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                assert np.all(T[:, dx % 6, dy % 8, dz % 10] == 0)
    # a far sample equals Eq. (7) at R = a d for d = v' - v
    p, d = 5, np.array([2, -3, 1])
    val = O.operator_value(khat[p], 0.5 * d.astype(float), 2 * math.pi, 3)
    np.testing.assert_allclose(T[p, 2, -3 % 8, 1], val, rtol=1e-14)


def test_direction_mode_rank_is_spherical_degree():
    """T_L(k, R) is a polynomial of degree <= L on the sphere, so the direction mode has
    rank (L+1)^2 (Table II lists r4 = r3 = 225 for L = 14).  Dropping l = 0 would give (L+1)^2 - 1."""
    L = 5
    khat, _, T, Th = O.build_operator((4, 4, 4), 0.5, 2 * math.pi, L)
    s = np.linalg.svd(Th.reshape(Th.shape[0], -1), compute_uv=False)
    r = int(np.sum(s > 1e-11 * s[0]))
    assert r == (L + 1) ** 2


# Relative permittivities of the lossy-medium test (Table IV); k = k0 sqrt(eps_r),
# Im k < 0 under the e^{jwt} convention of Section II-A.
LOSSY_EPS = (2 - 1j, 2 - 2j, 2 - 8j)


def test_hankel_complex_argument():
    """h_l^(2) at complex arguments (Section III-A-5).  Where the loss is mild the
    oracle's finite sum agrees with the library's j_l - i y_l (an independent
    route); where it is strong (|Im x| up to 90, j_l and y_l ~ e^{90}) it still
    satisfies the closed forms of h_0, h_1 and the three-term recurrence
    h_{l-1} + h_{l+1} = (2l+1)/x h_l (DLMF 10.51.1) to rounding."""
    from scipy import special

    z = np.array([1.0, 3.3, 6.28, 12.0]) * np.sqrt(2 - 1j)
    for l in range(15):
        ref = special.spherical_jn(l, z) - 1j * special.spherical_yn(l, z)
        np.testing.assert_allclose(O.hankel2(l, z), ref, rtol=1e-11)
    z = np.array([1.0, 3.3, 6.28, 12.0, 40.0]) * np.sqrt(2 - 8j)
    np.testing.assert_allclose(O.hankel2(0, z), 1j * np.exp(-1j * z) / z, rtol=1e-14)
    np.testing.assert_allclose(O.hankel2(1, z), np.exp(-1j * z) * (1j / z ** 2 - 1 / z), rtol=1e-13)
    for l in range(1, 15):
        lhs = O.hankel2(l - 1, z) + O.hankel2(l + 1, z)
        np.testing.assert_allclose(lhs, (2 * l + 1) / z * O.hankel2(l, z), rtol=1e-13)
    # the real-axis limit of the complex route is the real route
    x = np.array([0.7, 3.3, 12.0])
    for l in (0, 5, 14):
        np.testing.assert_allclose(O.hankel2(l, x + 0j), O.hankel2(l, x), rtol=1e-12)


@pytest.mark.parametrize("eps", LOSSY_EPS)
def test_addition_theorem_lossy_medium(eps):
    """Eq. (7) with a complex wavenumber still reproduces the decaying Green's function
    exp(-jk|X+d|)/|X+d| through the plane-wave expansion, with an error that falls as L
    grows (L = 10 -> 18: 2.7e-4 -> 3.5e-7, 1.8e-3 -> 1.7e-6, 1.7 -> 9.5e-4 for the three
    permittivities)."""
    k = 2 * math.pi * np.sqrt(complex(eps))
    a = 0.5
    rng = np.random.default_rng(7)
    Xs = [np.array([2, 2, 0.0]) * a, np.array([3, -2, 2.0]) * a, np.array([2, 0, 0.0]) * a]
    ds = [rng.uniform(-a / 2, a / 2, 3) - rng.uniform(-a / 2, a / 2, 3) for _ in range(4)]
    e10 = max(_addition_error(10, X, d, k) for X in Xs for d in ds)
    e18 = max(_addition_error(18, X, d, k) for X in Xs for d in ds)
    assert e18 < 2e-3
    assert e18 < e10 / 100


def test_loss_lowers_ranks_and_memory():
    """Table IV and Section III-A-5: the loss of the medium lowers the ranks, so the
    memory of the compressed operator falls as the permittivity's imaginary part grows
    (6^3 boxes, 0.5 wavelength, L = 8, gamma = 1e-4)."""
    khat, _ = O.directions(8)
    stored = {}
    for eps in (2,) + LOSSY_EPS:
        k = 2 * math.pi * np.sqrt(complex(eps))
        Th = O.fft_operator(O.sample_operator((6, 6, 6), 0.5, k, 8, khat))
        stored[eps] = {f: O.stored_elements(O.compress(Th, f, 1e-4)) for f in ("htucker4d", "tt4d")}
    for f in ("htucker4d", "tt4d"):
        seq = [stored[e][f] for e in (2,) + LOSSY_EPS]
        assert all(b < a for a, b in zip(seq, seq[1:])), (f, seq)
