"""Plain FP64 CPU oracle of the steps around the translation: aggregation of
far-field patterns into box radiation patterns (Eq. (4)) and their projection
back onto the basis functions with the direction quadrature (Eq. (6)), for
point-dipole basis functions (Eq. (3) with a delta-function basis).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The GPU library never
calls it and shares no code with it.

Conventions (readings, listed in the design notes):
F1  A basis function is a point dipole b_n(r) = u_n delta(r - r_n) (unit vector
    u_n); its far-field pattern along k_p (Eq. (3), sign +) is
    P+(k_p, b_n) = (I - k_p k_p) u_n exp(+jk k_p . (r_n - r_v)),
    kept as its theta and phi components (theta_p . u_n, phi_p . u_n) times the
    phase, theta_p = (cos th cos ph, cos th sin ph, -sin th), phi_p = (-sin ph, cos ph, 0).
F2  Component c (theta, phi) of right-hand side r is RHS 2 r + c of the
    translation (each component is one scalar field, reading R17).
F3  The receive pattern of Eq. (6) is P-(k_p, b_m) = (I - k_p k_p) u_m
    exp(-jk k_p . (r_m - r_v')): the conjugate of P+ for a real k, as the paper
    states; the same expression stays correct for a complex k (lossy medium).
F4  Box v of a point r is floor(r / a) per axis (grid corner at the origin),
    its centre r_v = (v + 1/2) a.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

from . import tfmm_oracle as T


def box_index(pos: np.ndarray, box: float, K) -> np.ndarray:
    """Integer box coordinates (N, 3) of points pos (N, 3) (reading F4)."""
    v = np.floor(np.asarray(pos, dtype=np.float64) / box).astype(np.int64)
    if (v < 0).any() or (v >= np.asarray(K)).any():
        raise ValueError("point outside the box grid")
    return v


def box_centres(v: np.ndarray, box: float) -> np.ndarray:
    return (v.astype(np.float64) + 0.5) * box


def polar_unit_vectors(khat: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """theta_p and phi_p unit vectors of each direction k_p (n_dir, 3)."""
    th = np.arccos(np.clip(khat[:, 2], -1.0, 1.0))
    ph = np.arctan2(khat[:, 1], khat[:, 0])
    et = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], axis=1)
    ep = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], axis=1)
    return et, ep


def dipole_patterns(khat: np.ndarray, k, pos: np.ndarray, orient: np.ndarray, box: float, K, sign: int = +1):
    """Eq. (3) for point dipoles: pattern (n_dir, N, 2) of theta/phi components,
    exp(sign jk k_p . (r_n - r_v)) (F1, F3)."""
    v = box_index(pos, box, K)
    d = np.asarray(pos, dtype=np.float64) - box_centres(v, box)          # r_n - r_v
    et, ep = polar_unit_vectors(khat)
    gt = et @ orient.T                                                    # (n_dir, N)
    gp = ep @ orient.T
    phase = np.exp(sign * 1j * k * (khat @ d.T))                          # (n_dir, N)
    return np.stack([gt * phase, gp * phase], axis=-1)


def aggregate(Pplus: np.ndarray, I: np.ndarray, pos: np.ndarray, box: float, K) -> np.ndarray:
    """Eq. (4): A_v(k_p) = sum_{n in B_v} P+(k_p, b_n) I_n for every box and
    direction; I (nrhs, N) -> A (2 nrhs, n_dir, Kx, Ky, Kz) (F2), zero for
    empty boxes."""
    I = np.atleast_2d(np.asarray(I, dtype=np.complex128))
    v = box_index(pos, box, K)
    ndir, N, _ = Pplus.shape
    A = np.zeros((2 * I.shape[0], ndir) + tuple(K), dtype=np.complex128)
    for n in range(N):
        x, y, z = v[n]
        for r in range(I.shape[0]):
            for c in range(2):
                A[2 * r + c, :, x, y, z] += Pplus[:, n, c] * I[r, n]
    return A


def disaggregate(Pminus: np.ndarray, B: np.ndarray, w: np.ndarray, pos: np.ndarray, box: float, K) -> np.ndarray:
    """Eq. (6): y_m = sum_p w_p P-(k_p, b_m) . B_{v'(m)}(k_p), summed over the theta
    and phi components; B (2 nrhs, n_dir, Kx, Ky, Kz) -> y (nrhs, N)."""
    v = box_index(pos, box, K)
    nrhs = B.shape[0] // 2
    ndir, N, _ = Pminus.shape
    y = np.zeros((nrhs, N), dtype=np.complex128)
    for m in range(N):
        x, yy, z = v[m]
        for r in range(nrhs):
            for c in range(2):
                y[r, m] += np.sum(w * Pminus[:, m, c] * B[2 * r + c, :, x, yy, z])
    return y


def farfield_matvec(I, pos, orient, K, box, k, L, That, grid="bj"):
    """Far-field part of the matrix-vector product: Eq. (4), the translation of
    Eq. (5) with the FFT'ed operator That (n_dir, n1, n2, n3), then Eq. (6)."""
    khat, w = T.directions(L, grid)
    Pp = dipole_patterns(khat, k, pos, orient, box, K, +1)
    Pm = dipole_patterns(khat, k, pos, orient, box, K, -1)
    A = aggregate(Pp, I, pos, box, K)
    B = T.translate_fft(A, That)
    return disaggregate(Pm, B, w, pos, box, K)


def dyadic_green(R: np.ndarray, k) -> np.ndarray:
    """(I + grad grad / k^2) exp(-jkR)/R for separations R (..., 3): (..., 3, 3)."""
    R = np.asarray(R, dtype=np.float64)
    r = np.asarray(np.linalg.norm(R, axis=-1))
    rh = R / r[..., None]
    kr = np.asarray(k * r)
    g = np.asarray(np.exp(-1j * kr) / r)
    a = np.asarray(1 - 1j / kr - 1 / kr ** 2)
    b = np.asarray(-1 + 3j / kr + 3 / kr ** 2)
    eye = np.eye(3)
    return g[..., None, None] * (a[..., None, None] * eye + b[..., None, None] * rh[..., :, None] * rh[..., None, :])


def farfield_direct(I, pos, orient, K, box, k, near_rule="cheb", near_param=1.0) -> np.ndarray:
    """The plain definition the far-field matvec approximates: for every pair of
    dipoles in far box pairs (the near rule of the translation operator), the
    plane-wave expansion of Eqs. (3)-(7) sums to
    (4 pi / (-jk)) u_m . (I + grad grad / k^2) exp(-jk|r_m - r_n|)/|r_m - r_n| . u_n I_n
    (Gegenbauer addition theorem with the transverse projection of Eq. (3))."""
    I = np.atleast_2d(np.asarray(I, dtype=np.complex128))
    v = box_index(pos, box, K)
    D = v[:, None, :] - v[None, :, :]                                   # v' - v for (m, n)
    near = T.near_mask(D, near_rule, near_param)
    R = pos[:, None, :] - pos[None, :, :]
    np.fill_diagonal(near, True)
    R[near] = 1.0                                                        # placeholder, masked below
    G = dyadic_green(R, k)
    Z = np.einsum("mi,mnij,nj->mn", orient, G, orient) * (4 * np.pi / (-1j * k))
    Z[near] = 0.0
    return I @ Z.T
