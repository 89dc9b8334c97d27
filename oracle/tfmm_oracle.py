"""Plain FP64 CPU oracle for FFT-based translation with compressed operators.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The GPU library never
calls it and shares no code with it.

It computes, in complex128 with numpy/scipy, what the iterative-solution-stage
translation of an FMM-FFT surface-integral-equation solver computes when the
FFT'ed translation operators are held in compressed form (Qian & Yucel,
"On the Compression of Translation Operator Tensors in FMM-FFT-Accelerated SIE
Simulators via Tensor Decompositions"):

* plane-wave directions and the multipole order (Section II-A, text after
  Eq. (4));
* the translation operator sampled on the box-offset grid (Eq. (7)) and its
  3-D FFT (Section II-B, first paragraph);
* Tucker (Eqs. (8)-(10), Algorithm 1), H-Tucker (Eqs. (11)-(12),
  Algorithm 2) and tensor-train (Eqs. (13)-(14), Algorithm 3) compression;
* per-direction restoration (Section II-C, Figs. 3 and 4);
* the FFT convolution of Eq. (5), and the plain pairwise sum it equals.

Readings taken where the paper is silent, garbled or inconsistent (each is
listed with its evidence in the design notes):

R1  Eq. (7) sums l = 0..L (the printed lower limit 1 breaks the addition
    theorem and the (L+1)^2 direction rank of Table II).
R2  The physical prefactor of Eq. (7) is an optional global scale (default 1);
    it changes neither ranks nor relative errors.
R3  h_l^(2) = j_l - i y_l and (-j)^l with j = sqrt(-1).
R4  Direction grid: (L+1) Gauss-Legendre nodes in cos(theta), ascending,
    times n_phi uniform phi_j = 2 pi j / n_phi; direction p = i_theta*n_phi + j.
R5  L = round(x + 1.8 d^(2/3) x^(1/3)), x = 2 k R^s = |k| a sqrt(3), d = digits;
    the paper's printed direction counts follow floor, the serving workload
    uses ceil.
R6  Near-field offsets are zeroed in the operator: by default the 27 nearest
    boxes (max_i |d_i| <= 1); the kappa rule of Section II-A (R < kappa R^s,
    kappa = 4) is available.
R7  Offset index m in [0, 2K): d = m for m < K, d = m - 2K for m > K, the slot
    m = K is unused and holds zero; R = a d with d = v' - v.
R8  Forward FFT unnormalised (exp(-2 pi i m k / n)), inverse scaled by 1/N.
R9  Truncation keeps the smallest r >= 1 whose discarded singular values have
    root-sum-square <= (gamma / sqrt(m)) ||X||_F, with m = d for Tucker,
    d - 1 for TT and 6 for H-Tucker.
R10 Classical T-HOSVD: every mode unfolds the original tensor.
R11 Projections use conjugate transposes throughout.
R12 H-Tucker uses the balanced tree {1,2}{3,4}; leaves are truncated with
    gamma/sqrt(6) like the interior nodes; r34 is taken from the transpose of
    the same matricisation (so r34 = r12).
R13 TT naming: U1 = first core (n1 x r1), last factor = last core transposed
    (n_d x r_{d-1}); interior cores r_{i} x n_{i+1} x r_{i+1}.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np
from scipy import special

# ---------------------------------------------------------------------------
# Directions and multipole order (Section II-A, text after Eq. (4))
# ---------------------------------------------------------------------------


def gauss_legendre(n: int) -> Tuple[np.ndarray, np.ndarray]:
    """Gauss-Legendre nodes (ascending) and weights on [-1, 1] (library routine)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def directions(L: int, grid: str = "bj", n_theta: int = 0, n_phi: int = 0):
    """Plane-wave directions k_p and quadrature weights w_p on the unit sphere.

    The sphere is sampled by the Cartesian product of Gauss-Legendre nodes in
    cos(theta) and uniform nodes in phi (reading R4).  Returns (khat, w) with
    khat of shape (n_dir, 3) and sum(w) = 4 pi.
    """
    nt = n_theta or (L + 1)
    if n_phi:
        nph = n_phi
    elif grid == "bj":
        nph = 2 * (L + 1)
    elif grid == "paper":
        nph = 2 * L + 1
    else:
        raise ValueError(grid)
    x, wt = gauss_legendre(nt)
    theta = np.arccos(x)
    phi = 2.0 * np.pi * np.arange(nph) / nph
    th = np.repeat(theta, nph)
    ph = np.tile(phi, nt)
    khat = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    w = np.repeat(wt, nph) * (2.0 * np.pi / nph)
    return khat, w


def multipole_order(k_abs: float, box: float, digits: float, rounding: str = "floor") -> int:
    """Number of multipoles L from the box size and the desired digits (reading R5)."""
    x = k_abs * box * math.sqrt(3.0)  # 2 k R^s, R^s = a sqrt(3) / 2
    val = x + 1.8 * digits ** (2.0 / 3.0) * x ** (1.0 / 3.0)
    return int(math.floor(val)) if rounding == "floor" else int(math.ceil(val))


# ---------------------------------------------------------------------------
# Box-offset grid and near field (Section II-A; Eq. (5) circular placement)
# ---------------------------------------------------------------------------


def axis_offsets(Ki: int) -> Tuple[np.ndarray, np.ndarray]:
    """Signed box offset d for each FFT index m in [0, 2Ki) and a validity mask (R7)."""
    m = np.arange(2 * Ki)
    d = np.where(m < Ki, m, m - 2 * Ki)
    valid = m != Ki
    return d, valid


def offset_grid(K: Sequence[int]):
    """Integer offsets d (n1, n2, n3, 3) and the mask of usable slots."""
    dx, vx = axis_offsets(K[0])
    dy, vy = axis_offsets(K[1])
    dz, vz = axis_offsets(K[2])
    D = np.stack(np.meshgrid(dx, dy, dz, indexing="ij"), axis=-1)
    V = vx[:, None, None] & vy[None, :, None] & vz[None, None, :]
    return D, V


def near_mask(D: np.ndarray, rule: str = "cheb", param: float = 1.0) -> np.ndarray:
    """True where the box pair at integer offset D is near (handled classically, R6).

    "cheb": max_i |d_i| <= param.  "kappa": R < kappa R^s, i.e. 4|d|^2 < 3 kappa^2.
    Offset zero is always near.
    """
    if rule == "cheb":
        near = np.max(np.abs(D), axis=-1) <= param
    elif rule == "kappa":
        near = 4 * np.sum(D.astype(np.int64) ** 2, axis=-1) < 3 * param * param
    else:
        raise ValueError(rule)
    return near | np.all(D == 0, axis=-1)


# ---------------------------------------------------------------------------
# Translation operator, Eq. (7)
# ---------------------------------------------------------------------------


def hankel2(l, x):
    """Spherical Hankel function of the second kind, h_l^(2) = j_l - i y_l (R3).

    Real x: the library's j_l and y_l.  Complex x (a lossy medium, Section
    III-A-5, has a complex wavenumber): j_l and y_l both grow like e^{|Im x|}
    while h_l^(2) decays like e^{-|Im x|} for Im x < 0, so their difference
    cancels; the finite closed form of h_l^(2) (DLMF section 10.49(i)) is summed
    instead: h_l^(2)(x) = e^{-ix} sum_{k=0}^{l} (-i)^{k-l-1} a_k / x^{k+1},
    a_k = (l+k)! / (2^k k! (l-k)!).
    """
    if not np.iscomplexobj(x):
        return special.spherical_jn(l, x) - 1j * special.spherical_yn(l, x)
    x = np.asarray(x, dtype=np.complex128)
    total = np.zeros_like(x)
    for k in range(l + 1):
        a_k = math.factorial(l + k) / (2.0 ** k * math.factorial(k) * math.factorial(l - k))
        total = total + ((-1j) ** (k - l - 1)) * a_k / x ** (k + 1)
    return np.exp(-1j * x) * total


def legendre(l, t):
    """Legendre polynomial P_l(t) (library routine)."""
    return special.eval_legendre(l, t)


def operator_value(khat: np.ndarray, R: np.ndarray, k, L: int, scale: complex = 1.0):
    """T_L(khat, R) = scale * sum_{l=0}^{L} (-i)^l (2l+1) h_l^(2)(k|R|) P_l(khat . Rhat).

    khat: (..., 3) unit vectors, R: (..., 3) nonzero separations; broadcast together.
    k: real, or complex with Im k < 0 in a lossy medium (Section III-A-5).
    """
    khat = np.asarray(khat, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    r = np.linalg.norm(R, axis=-1)
    cos = np.sum(khat * R, axis=-1) / r
    cos = np.clip(cos, -1.0, 1.0)
    x = k * r
    total = np.zeros(np.broadcast(cos, x).shape, dtype=np.complex128)
    for l in range(L + 1):
        total = total + ((-1j) ** l) * (2 * l + 1) * hankel2(l, x) * legendre(l, cos)
    return scale * total


def sample_operator(K: Sequence[int], box: float, k: float, L: int, khat: np.ndarray,
                    near_rule: str = "cheb", near_param: float = 1.0, scale: complex = 1.0):
    """Spatial translation-operator samples T_p(m) on the 2K grid, shape (n_dir, n1, n2, n3).

    Far offsets get Eq. (7); near offsets and the unused slot m_i = K_i are 0.
    """
    D, V = offset_grid(K)
    far = V & ~near_mask(D, near_rule, near_param)
    R = box * D[far].astype(np.float64)                     # (n_far, 3)
    n = tuple(2 * x for x in K)
    out = np.zeros((khat.shape[0],) + n, dtype=np.complex128)
    vals = operator_value(khat[:, None, :], R[None, :, :], k, L, scale)  # (n_dir, n_far)
    out[:, far] = vals
    return out


def fft_operator(T: np.ndarray) -> np.ndarray:
    """FFT'ed operator T~_p = FFT3(T_p) over the last three axes (R8)."""
    return np.fft.fftn(T, axes=(-3, -2, -1))


# ---------------------------------------------------------------------------
# Truncation rule (Algorithms 1-3, reading R9)
# ---------------------------------------------------------------------------


def truncation_rank(s: np.ndarray, budget: float) -> int:
    """Smallest r >= 1 such that sqrt(sum_{j >= r} s_j^2) <= budget (s descending)."""
    s = np.asarray(s, dtype=np.float64)
    tail = np.sqrt(np.concatenate([np.cumsum((s ** 2)[::-1])[::-1], [0.0]]))  # tail[r] = rss(s[r:])
    for r in range(1, len(s) + 1):
        if tail[r] <= budget:
            return r
    return len(s)


def leading_left_singular(M: np.ndarray, budget: float):
    """Left singular vectors of M truncated by the tail budget; also returns all singular values."""
    U, s, _ = np.linalg.svd(M, full_matrices=False)
    r = truncation_rank(s, budget)
    return U[:, :r], s


# ---------------------------------------------------------------------------
# Tucker: Eqs. (8)-(10), Algorithm 1
# ---------------------------------------------------------------------------


def unfold(X: np.ndarray, mode: int) -> np.ndarray:
    """Mode-`mode` unfolding: rows index that mode, columns the others (C order)."""
    return np.moveaxis(X, mode, 0).reshape(X.shape[mode], -1)


def mode_product(X: np.ndarray, U: np.ndarray, mode: int) -> np.ndarray:
    """Eq. (10): Y = X x_mode U, i.e. Y[.., v, ..] = sum_i X[.., i, ..] U[v, i]."""
    Y = np.tensordot(U, X, axes=([1], [mode]))  # new axis first
    return np.moveaxis(Y, 0, mode)


def tucker_svd(X: np.ndarray, gamma: float):
    """Algorithm 1 (truncated HOSVD): returns (core, [U_1..U_d])."""
    d = X.ndim
    budget = gamma / math.sqrt(d) * np.linalg.norm(X)
    Us = []
    for i in range(d):
        U, _ = leading_left_singular(unfold(X, i), budget)
        Us.append(U)
    C = X
    for i in range(d):
        C = mode_product(C, Us[i].conj().T, i)
    return C, Us


def tucker_restore(C: np.ndarray, Us: Sequence[np.ndarray]) -> np.ndarray:
    """Eq. (8)/(9): C x_1 U1 x_2 U2 ... (Fig. 3(a) for the 3-D case)."""
    X = C
    for i, U in enumerate(Us):
        X = mode_product(X, U, i)
    return X


def tucker3d_restore_figure3a(C: np.ndarray, U1, U2, U3) -> np.ndarray:
    """Fig. 3(a): core as matrix times U1, reshape, times U2, reshape, times U3."""
    r1, r2, r3 = C.shape
    n1, n2, n3 = U1.shape[0], U2.shape[0], U3.shape[0]
    T = U1 @ C.reshape(r1, r2 * r3)                                  # step 1: n1 x (r2 r3)
    T = T.reshape(n1, r2, r3).transpose(1, 0, 2).reshape(r2, n1 * r3)
    T = U2 @ T                                                         # step 2: n2 x (n1 r3)
    T = T.reshape(n2, n1, r3).transpose(2, 1, 0).reshape(r3, n1 * n2)
    T = U3 @ T                                                         # step 3: n3 x (n1 n2)
    return T.reshape(n3, n1, n2).transpose(1, 2, 0)                    # step 4: n1 x n2 x n3


# ---------------------------------------------------------------------------
# H-Tucker: Eqs. (11)-(12), Algorithm 2
# ---------------------------------------------------------------------------


def htucker_svd(X: np.ndarray, gamma: float) -> Dict[str, object]:
    """Algorithm 2 on a 4-D tensor with the balanced tree {1,2}{3,4} (reading R12)."""
    assert X.ndim == 4
    budget = gamma / math.sqrt(6.0) * np.linalg.norm(X)
    Us = [leading_left_singular(unfold(X, i), budget)[0] for i in range(4)]   # step 3
    W = X
    for i in range(4):                                                         # step 4
        W = mode_product(W, Us[i].conj().T, i)
    r1, r2, r3, r4 = W.shape
    W12 = W.reshape(r1 * r2, r3 * r4)                                          # step 5
    C12, s12 = leading_left_singular(W12, budget)                              # steps 6-7
    C34, s34 = leading_left_singular(W12.T, budget)                            # step 8
    B = C12.conj().T @ W12 @ C34.conj()                                        # steps 9-10
    return {"U": Us, "C12": C12.reshape(r1, r2, -1), "C34": C34.reshape(r3, r4, -1), "B": B,
            "s12": s12, "s34": s34}


def htucker_contract_core(ht) -> np.ndarray:
    """Eq. (11) core: G = (C34 x_3 C1234) x_3^3 C12, as an r1 x r2 x r3 x r4 array."""
    Y = mode_product(ht["C34"], ht["B"], 2)                   # r3 x r4 x r12
    # Eq. (12): Z[a1,a2,a3,a4] = sum_b C12[a1,a2,b] Y[a3,a4,b]
    return np.tensordot(ht["C12"], Y, axes=([2], [2]))


def htucker_restore(ht) -> np.ndarray:
    return tucker_restore(htucker_contract_core(ht), ht["U"])


def htucker_direction_core(ht, p: int) -> np.ndarray:
    """Fig. 3(c): the r1 x r2 x r3 core of direction p."""
    C34 = ht["C34"]
    r3, r4, r34 = C34.shape
    C12 = ht["C12"]
    r1, r2, r12 = C12.shape
    u4 = ht["U"][3][p, :]                                                  # p-th row of U4
    X1 = np.einsum("abc,b->ac", C34, u4)                                   # r3 x r34
    X2 = X1 @ ht["B"].T                                                    # r3 x r12
    Cp = C12.reshape(r1 * r2, r12) @ X2.T                                  # (r1 r2) x r3
    return Cp.reshape(r1, r2, r3)


# ---------------------------------------------------------------------------
# Tensor train: Eqs. (13)-(14), Algorithm 3
# ---------------------------------------------------------------------------


def tt_svd(X: np.ndarray, gamma: float):
    """Algorithm 3: returns (U1, [interior cores], U_last) (reading R13)."""
    d = X.ndim
    budget = gamma / math.sqrt(d - 1) * np.linalg.norm(X)
    n = X.shape
    C = X.reshape(n[0], -1)
    r_prev = 1
    cores = []
    for i in range(d - 1):
        if i > 0:
            C = C.reshape(r_prev * n[i], -1)
        U, s, Vh = np.linalg.svd(C, full_matrices=False)
        r = truncation_rank(s, budget)
        cores.append(U[:, :r].reshape(r_prev, n[i], r))
        C = s[:r, None] * Vh[:r, :]
        r_prev = r
    U1 = cores[0].reshape(n[0], -1)
    Ulast = C.T                                                   # n_d x r_{d-1}
    return U1, cores[1:], Ulast


def tt3d_restore(U1, C, U3) -> np.ndarray:
    """Fig. 4(a): T1 = U1 * C (n1 n2 x r2), then T1 * U3^T, reshaped to n1 x n2 x n3."""
    r1, n2, r2 = C.shape
    n1, n3 = U1.shape[0], U3.shape[0]
    T1 = (U1 @ C.reshape(r1, n2 * r2)).reshape(n1 * n2, r2)
    return (T1 @ U3.T).reshape(n1, n2, n3)


def tt4d_restore_direction(U1, C1, C2, U3, p: int) -> np.ndarray:
    """Fig. 4(b): column p of C2 * U3^T reshaped r2 x n3, multiplied by T1 = U1 * C1."""
    r1, n2, r2 = C1.shape
    _, n3, r3 = C2.shape
    n1 = U1.shape[0]
    T1 = (U1 @ C1.reshape(r1, n2 * r2)).reshape(n1 * n2, r2)
    col = C2.reshape(r2 * n3, r3) @ U3[p, :]                      # p-th column of T2
    return (T1 @ col.reshape(r2, n3)).reshape(n1, n2, n3)


def tt_restore(U1, cores, Ulast) -> np.ndarray:
    """Full reconstruction of a TT tensor (any d)."""
    X = U1
    for G in cores:
        X = np.tensordot(X, G, axes=([-1], [0]))
    return np.tensordot(X, Ulast, axes=([-1], [1]))


# ---------------------------------------------------------------------------
# The five methodologies applied to the FFT'ed operator (Section II-B)
# ---------------------------------------------------------------------------


def compress(That: np.ndarray, fmt: str, gamma: float) -> Dict[str, object]:
    """Compress the FFT'ed operators (n_dir, n1, n2, n3) in the named format."""
    ndir = That.shape[0]
    if fmt == "full":
        return {"fmt": fmt, "T": That}
    if fmt == "tucker3d":
        per = [tucker_svd(That[p], gamma) for p in range(ndir)]
        return {"fmt": fmt, "per": per}
    if fmt == "tt3d":
        per = []
        for p in range(ndir):
            U1, cores, U3 = tt_svd(That[p], gamma)
            per.append((U1, cores[0], U3))
        return {"fmt": fmt, "per": per}
    X4 = np.moveaxis(That, 0, -1)                              # n1 x n2 x n3 x n_dir (R14)
    if fmt == "tucker4d":
        C, Us = tucker_svd(X4, gamma)
        return {"fmt": fmt, "C": C, "U": Us}
    if fmt == "tt4d":
        U1, cores, U3 = tt_svd(X4, gamma)
        return {"fmt": fmt, "U1": U1, "C1": cores[0], "C2": cores[1], "U3": U3}
    if fmt == "htucker4d":
        ht = htucker_svd(X4, gamma)
        ht["fmt"] = fmt
        return ht
    raise ValueError(fmt)


def restore_direction(comp: Dict[str, object], p: int) -> np.ndarray:
    """T~_p restored from the compressed form, following Figs. 3 and 4."""
    fmt = comp["fmt"]
    if fmt == "full":
        return comp["T"][p]
    if fmt == "tucker3d":
        C, Us = comp["per"][p]
        return tucker3d_restore_figure3a(C, *Us)
    if fmt == "tt3d":
        return tt3d_restore(*comp["per"][p])
    if fmt == "tucker4d":
        C, Us = comp["C"], comp["U"]
        r1, r2, r3, r4 = C.shape
        Cp = (C.reshape(r1 * r2 * r3, r4) @ Us[3][p, :]).reshape(r1, r2, r3)   # Fig. 3(b)
        return tucker3d_restore_figure3a(Cp, Us[0], Us[1], Us[2])
    if fmt == "tt4d":
        return tt4d_restore_direction(comp["U1"], comp["C1"], comp["C2"], comp["U3"], p)
    if fmt == "htucker4d":
        Cp = htucker_direction_core(comp, p)
        return tucker3d_restore_figure3a(Cp, comp["U"][0], comp["U"][1], comp["U"][2])
    raise ValueError(fmt)


def restore_all(comp: Dict[str, object], ndir: int) -> np.ndarray:
    return np.stack([restore_direction(comp, p) for p in range(ndir)])


def ranks(comp: Dict[str, object]):
    """Ranks of a compressed operator: per-direction list for 3-D formats, a tuple for 4-D."""
    fmt = comp["fmt"]
    if fmt == "tucker3d":
        return [C.shape for C, _ in comp["per"]]
    if fmt == "tt3d":
        return [(C.shape[0], C.shape[2]) for _, C, _ in comp["per"]]
    if fmt == "tucker4d":
        return comp["C"].shape
    if fmt == "tt4d":
        return (comp["C1"].shape[0], comp["C1"].shape[2], comp["C2"].shape[2])
    if fmt == "htucker4d":
        r1, r2, r12 = comp["C12"].shape
        r3, r4, r34 = comp["C34"].shape
        return (r1, r2, r3, r4, r12, r34)
    return ()


def stored_elements(comp: Dict[str, object]) -> int:
    """Complex entries held by the compressed representation (cores and factors)."""
    fmt = comp["fmt"]
    if fmt == "full":
        return int(comp["T"].size)
    if fmt == "tucker3d":
        return int(sum(C.size + sum(U.size for U in Us) for C, Us in comp["per"]))
    if fmt == "tt3d":
        return int(sum(a.size + b.size + c.size for a, b, c in comp["per"]))
    if fmt == "tucker4d":
        return int(comp["C"].size + sum(U.size for U in comp["U"]))
    if fmt == "tt4d":
        return int(sum(comp[k].size for k in ("U1", "C1", "C2", "U3")))
    if fmt == "htucker4d":
        return int(sum(U.size for U in comp["U"]) + comp["C12"].size + comp["C34"].size + comp["B"].size)
    raise ValueError(fmt)


# ---------------------------------------------------------------------------
# Translation, Eq. (5), and the pairwise sum it equals
# ---------------------------------------------------------------------------


def translate_fft(A: np.ndarray, That: np.ndarray) -> np.ndarray:
    """B_{s,p} = IFFT3(T~_p * FFT3(zero-padded A_{s,p})) cropped to the box grid.

    A: (nrhs, n_dir, Kx, Ky, Kz); That: (n_dir, n1, n2, n3).
    """
    A = np.asarray(A, dtype=np.complex128)
    K = A.shape[-3:]
    n = That.shape[-3:]
    Ah = np.fft.fftn(A, s=n, axes=(-3, -2, -1))               # zero-pads at the high end
    Bfull = np.fft.ifftn(Ah * That[None], axes=(-3, -2, -1))
    return Bfull[..., :K[0], :K[1], :K[2]]


def translate_compressed(A: np.ndarray, comp: Dict[str, object]) -> np.ndarray:
    """Eq. (5) with each T~_p restored one by one from its compressed form."""
    A = np.asarray(A, dtype=np.complex128)
    ndir = A.shape[1]
    out = np.empty_like(A)
    for p in range(ndir):
        Tp = restore_direction(comp, p)
        out[:, p] = translate_fft(A[:, p:p + 1], Tp[None])[:, 0]
    return out


def translate_direct(A: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Plain pairwise sum B_{s,p}[v'] = sum_v T_p(v' - v) A_{s,p}[v] with spatial samples T.

    T: (n_dir, n1, n2, n3) indexed by offset slot (R7).  O(K^2) per direction.
    """
    A = np.asarray(A, dtype=np.complex128)
    Kx, Ky, Kz = A.shape[-3:]
    n1, n2, n3 = T.shape[-3:]
    vx, vy, vz = np.meshgrid(np.arange(Kx), np.arange(Ky), np.arange(Kz), indexing="ij")
    out = np.zeros_like(A)
    for x in range(Kx):
        for y in range(Ky):
            for z in range(Kz):
                mx = (vx - x) % n1
                my = (vy - y) % n2
                mz = (vz - z) % n3
                out += T[None, :, mx, my, mz] * A[:, :, x:x + 1, y:y + 1, z:z + 1]
    return out


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b||_2 / ||b||_2."""
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


# ---------------------------------------------------------------------------
# Convenience: the whole operator for a workload
# ---------------------------------------------------------------------------


def build_operator(K, box, k, L, grid="bj", near_rule="cheb", near_param=1.0, scale=1.0):
    """Returns (khat, w, T spatial, T~ FFT'ed) for a box grid."""
    khat, w = directions(L, grid)
    T = sample_operator(K, box, k, L, khat, near_rule, near_param, scale)
    return khat, w, T, fft_operator(T)
