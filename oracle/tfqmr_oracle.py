"""Plain FP64 CPU oracle of the iterative solution of the method-of-moments
system Z I = V (Eq. (2)) with the transpose-free quasi-minimal residual method
(TFQMR) the paper uses (Section II-A, tolerance 1e-6), in the steps and
notation of Freund's algorithm: two half steps per iteration sharing one
Lanczos-type coefficient alpha, a quasi-minimisation of the residual norm bound
tau, and the iterate updated along the smoothed direction d.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The GPU library never
calls it and shares no code with it.

Readings (listed in the design notes):
Q1  Inner product (x, y) = y^H x; shadow residual r0* = r0; initial guess 0.
Q2  Stopping: when the bound tau sqrt(m + 1) on the residual norm of half step
    m falls below tol ||V||, the true residual ||V - Z I|| / ||V|| is computed and
    the iteration stops if it is <= tol; otherwise it continues.
"""
from __future__ import annotations

import math
from typing import Callable, List, Tuple

import numpy as np


def tfqmr(matvec: Callable[[np.ndarray], np.ndarray], b: np.ndarray, tol: float = 1e-6, maxit: int = 500
          ) -> Tuple[np.ndarray, int, List[float], List[float]]:
    """Solve A x = b.  Returns (x, iterations, bounds, true_residuals): the residual
    bound tau sqrt(m+1) of every half step and the true relative residual at each
    convergence check."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b)
    r0 = b - matvec(x)
    nb = np.linalg.norm(b)
    w = r0.copy()
    u = r0.copy()                      # u_m (y in Freund's notation)
    v = matvec(u)                      # v_m = A u_m
    Au = v.copy()                      # A u_m
    d = np.zeros_like(b)
    tau = np.linalg.norm(r0)
    theta = 0.0
    eta = 0.0
    rstar = r0.copy()
    rho = np.vdot(rstar, r0)
    bounds, checks = [], []
    alpha = 0.0
    it = 0
    if tau <= tol * nb:
        return x, 0, bounds, [tau / nb]
    for it in range(1, maxit + 1):
        sigma = np.vdot(rstar, v)
        alpha = rho / sigma
        u_next = u - alpha * v         # second Lanczos vector of this iteration
        for half in range(2):
            m = 2 * (it - 1) + half
            um = u if half == 0 else u_next
            Aum = Au if half == 0 else matvec(u_next)
            if half == 1:
                Au_next = Aum
            w = w - alpha * Aum
            d = um + (theta * theta * eta / alpha) * d
            theta = np.linalg.norm(w) / tau
            c = 1.0 / math.sqrt(1.0 + theta * theta)
            tau = tau * theta * c
            eta = c * c * alpha
            x = x + eta * d
            bound = tau * math.sqrt(m + 2)
            bounds.append(bound / nb)
            if bound <= tol * nb:
                res = np.linalg.norm(b - matvec(x)) / nb
                checks.append(res)
                if res <= tol:
                    return x, it, bounds, checks
        rho_new = np.vdot(rstar, w)
        beta = rho_new / rho
        rho = rho_new
        u = w + beta * u_next
        Au = matvec(u)
        v = Au + beta * (Au_next + beta * v)
    return x, it, bounds, checks
