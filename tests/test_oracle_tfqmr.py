"""Pins of the TFQMR oracle (the iterative solver of Eq. (2)) against exact
linear algebra: the solution of a seeded, well-conditioned complex system
equals the direct solve within the tolerance times the condition number; the
true residual at the stop is within the tolerance and below Freund's bound
tau sqrt(m+1); the residual bound decreases overall; a system of dimension n
is solved to rounding within about n iterations (the Krylov space is exhausted).
"""
import numpy as np

from oracle import tfqmr_oracle as Q


def _system(n, seed, shift=3.0):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    A += shift * np.eye(n) * (1 + 0.5j)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, b


def test_tfqmr_matches_direct_solve():
    A, b = _system(80, 1)
    x, it, bounds, checks = Q.tfqmr(lambda v: A @ v, b, tol=1e-8, maxit=200)
    ref = np.linalg.solve(A, b)
    assert checks[-1] <= 1e-8
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= np.linalg.cond(A) * 1e-8
    assert it < 80


def test_tfqmr_true_residual_below_bound():
    A, b = _system(50, 2, shift=1.5)
    x, it, bounds, checks = Q.tfqmr(lambda v: A @ v, b, tol=1e-6, maxit=200)
    res = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert res <= 1e-6 and res <= bounds[-1] * (1 + 1e-9)
    assert bounds[-1] < bounds[0] * 1e-4


def test_tfqmr_exhausts_krylov_space():
    A, b = _system(12, 3, shift=3.0)
    x, it, bounds, checks = Q.tfqmr(lambda v: A @ v, b, tol=1e-12, maxit=100)
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-11
    assert it <= 12 + 2
