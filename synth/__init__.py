"""Seeded synthetic workloads shared by the oracle-side tests and the GPU path.

This module holds workload *definitions* (box grids, box size, wavenumber,
multipole order, format, tolerance, number of right-hand sides) and seeded
random-number generators.  It contains none of the method's arithmetic: no
operator sampling, no FFT, no decomposition, no translation.

The paper's real inputs are aggregated radiation patterns of RWG-discretised
scatterers (Section III-B/C).  Those meshes are not available, so every input
here is an i.i.d. complex Gaussian stand-in of the same shape
(nrhs, n_dir, Kx, Ky, Kz): real and imaginary parts N(0, 1), drawn in float64
from numpy's PCG64 and rounded once to complex64.  Both sides consume the
rounded values (the oracle upcasts them to complex128), so input rounding is
never counted as error.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

# Seed base shared by every workload; workload i uses SEED_BASE + i.
SEED_BASE = 20100520

WAVELENGTH = 1.0
K0 = 2.0 * math.pi / WAVELENGTH  # free-space wavenumber with lambda = 1

FORMATS = ("full", "tucker3d", "tt3d", "tucker4d", "tt4d", "htucker4d")


@dataclass(frozen=True)
class Workload:
    """One translation workload, in the paper's problem-statement terms."""

    name: str
    K: Tuple[int, int, int]          # box grid Kx, Ky, Kz
    box: float                       # box edge a (wavelengths)
    L: int                           # multipole order
    fmt: str = "tucker3d"            # compression format
    tol: float = 1e-4                # decomposition tolerance gamma
    nrhs: int = 1                    # right-hand sides (each theta/phi component is one)
    k: float = K0                    # wavenumber
    grid: str = "bj"                 # direction grid: "bj" = (L+1) x 2(L+1), "paper" = (L+1) x (2L+1)
    near: str = "cheb"               # near-field rule: "cheb" (max|d_i| <= near_param) or "kappa"
    near_param: float = 1.0
    seed: int = SEED_BASE
    precision: str = "fp32"          # arithmetic of the GPU reconstruction

    @property
    def n(self) -> Tuple[int, int, int]:
        return tuple(2 * k for k in self.K)

    @property
    def n_theta(self) -> int:
        return self.L + 1

    @property
    def n_phi(self) -> int:
        return 2 * (self.L + 1) if self.grid == "bj" else 2 * self.L + 1

    @property
    def n_dir(self) -> int:
        return self.n_theta * self.n_phi

    @property
    def boxes(self) -> int:
        return self.K[0] * self.K[1] * self.K[2]

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# The five workloads the measurements are quoted on (index 0..4).
TINY = Workload("tiny-4^3", (4, 4, 4), 0.5, 5, fmt="tucker3d", tol=1e-6, nrhs=1, seed=SEED_BASE + 0)
PLAIN = Workload("plain-16^3", (16, 16, 16), 0.5, 10, fmt="tucker3d", tol=1e-4, nrhs=1, seed=SEED_BASE + 1)
BATCHING = Workload("batching-24^3", (24, 24, 24), 0.25, 8, fmt="tucker4d", tol=1e-4, nrhs=8, seed=SEED_BASE + 2)
PRECISION = Workload("precision-128x8x8", (128, 8, 8), 0.5, 12, fmt="htucker4d", tol=1e-4, nrhs=4,
                     seed=SEED_BASE + 3)
SERVING_GRIDS = ((8, 8, 8), (12, 12, 12), (16, 16, 16), (24, 24, 24), (32, 32, 32), (64, 16, 16))
SERVING_FORMATS = ("tucker3d", "tt4d")
SERVING_RATE_HZ = 200.0
SERVING_SEED = SEED_BASE + 5

WORKLOADS = (TINY, PLAIN, BATCHING, PRECISION)


def gaussian_patterns(shape, seed: int) -> np.ndarray:
    """Complex64 array of i.i.d. N(0,1)+iN(0,1) values, drawn in float64 then rounded."""
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im).astype(np.complex64)


def patterns_for(w: Workload, nrhs: Optional[int] = None, seed: Optional[int] = None) -> np.ndarray:
    """Aggregated-pattern stand-in A of shape (nrhs, n_dir, Kx, Ky, Kz), complex64."""
    s = w.nrhs if nrhs is None else nrhs
    return gaussian_patterns((s, w.n_dir) + tuple(w.K), w.seed if seed is None else seed)


def random_complex(shape, rng: np.random.Generator, scale: float = 1.0) -> np.ndarray:
    """Complex128 Gaussian array (used for synthetic compressed factors)."""
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def serving_requests(count: int, seed: int = SERVING_SEED, rate_hz: float = SERVING_RATE_HZ):
    """Seeded Poisson request stream: list of dicts (arrival_s, grid, fmt, nrhs, seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate_hz)
        grid = SERVING_GRIDS[int(rng.integers(len(SERVING_GRIDS)))]
        fmt = SERVING_FORMATS[int(rng.integers(len(SERVING_FORMATS)))]
        nrhs = int(rng.integers(1, 17))
        out.append({"id": i, "arrival_s": t, "grid": grid, "fmt": fmt, "nrhs": nrhs,
                    "seed": seed * 1000 + i})
    return out


# ---------------------------------------------------------------------------
# Basis functions of the far-field matvec (aggregation, Eq. (4); projection,
# Eq. (6)): point dipoles with seeded positions and unit orientations.
# ---------------------------------------------------------------------------

def dipoles_near_centres(K, box: float, n: int, seed: int, spread: float = 0.25):
    """n dipoles in random boxes of the grid, each within +-spread*box of its box
    centre per axis; returns (pos (n, 3), orient (n, 3) unit vectors)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = np.stack([rng.integers(0, k, n) for k in K], axis=1)
    pos = (v + 0.5) * box + rng.uniform(-spread, spread, (n, 3)) * box
    u = rng.standard_normal((n, 3))
    return pos, u / np.linalg.norm(u, axis=1, keepdims=True)


def sphere_dipoles(K, box: float, n: int, seed: int, radius_frac: float = 0.45):
    """n dipoles on a sphere centred in the box grid (radius radius_frac times the
    smallest grid extent), oriented tangentially at random: a stand-in for the
    RWG basis of a scattering surface (only boxes the surface crosses are
    non-empty).  Returns (pos (n, 3), orient (n, 3))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ext = np.asarray(K, dtype=np.float64) * box
    c = ext / 2
    R = radius_frac * ext.min()
    x = rng.standard_normal((n, 3))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    t = rng.standard_normal((n, 3))
    t -= np.sum(t * x, axis=1, keepdims=True) * x
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    return c + R * x, t


def current_vector(n: int, nrhs: int, seed: int) -> np.ndarray:
    """Basis-function coefficients I (nrhs, n), complex64 Gaussian."""
    return gaussian_patterns((nrhs, n), seed)


def near_field_csr(box_of: np.ndarray, K, seed: int, diag: complex, offdiag: float):
    """A synthetic near-field matrix in CSR form for basis functions with box
    coordinates box_of (n, 3): for every pair (m, n) whose boxes are within one
    box of each other (max |v_m - v_n| <= 1), a seeded complex Gaussian entry of
    scale `offdiag`; `diag` on the diagonal.  Returns (row_ptr, cols, vals)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = np.asarray(box_of)
    n = v.shape[0]
    rows, cols, vals = [0], [], []
    for m in range(n):
        near = np.nonzero(np.max(np.abs(v - v[m]), axis=1) <= 1)[0]
        for j in near:
            cols.append(int(j))
            if j == m:
                vals.append(complex(diag))
            else:
                vals.append(offdiag * complex(rng.standard_normal(), rng.standard_normal()))
        rows.append(len(cols))
    return np.array(rows, np.int32), np.array(cols, np.int32), np.array(vals, np.complex128)
