"""Damped Newton iteration for convex energies (oracle side).

Every nonlinear problem in the method is the Euler-Lagrange equation of a
strictly convex energy (monotone f, coercive a; Section 2, Assumption A):
    E(y) = 1/2 y^T K y + sum_j m_j F(z_j(y)) - sum_j m_j g_j z_j(y),
with z(y) = B y linear.  The paper leaves the nonlinear solver open (a
fixed-point or a Newton-type iteration, Section 3).  The reading used here: Newton steps
d = -J^{-1} R with backtracking (halving) until the Armijo decrease
E(y + t d) <= E(y) + 1e-4 t R.d holds; the test allows for rounding in E by
adding 1e-12 times the sum of the magnitudes of E's three terms.  The
iteration stops as soon as a computed Newton direction is small (a rule
supplied by the caller; the direction is then applied in full, without
evaluating the energy there, since such a step changes E only at rounding
level), when an accepted damped update is small, or when the update stops
decreasing (stagnation at rounding level).
"""
from __future__ import annotations

import numpy as np

ARMIJO_C = 1e-4
ENERGY_ROUNDING = 1e-12
MAX_HALVINGS = 40


def newton_minimize(y0, grad_hess, energy, solve, converged, max_iter=50,
                    stagnation=True):
    """Minimise a strictly convex energy by damped Newton.

    grad_hess(y) -> (R, J); energy(y) -> (E, scale); solve(J, R) -> J^{-1} R;
    converged(step, y) -> bool.  Returns (y, iterations, converged_flag).
    """
    y = np.array(y0, dtype=np.float64, copy=True)
    E, scale = energy(y)
    prev_norm = np.inf
    rises = 0
    for it in range(1, max_iter + 1):
        R, J = grad_hess(y)
        d = -solve(J, R)
        if np.all(np.isfinite(d)) and converged(d, y):
            return y + d, it, True
        slope = float(R @ d)
        t = 1.0
        for _ in range(MAX_HALVINGS):
            y_try = y + t * d
            E_try, scale_try = energy(y_try)
            if E_try <= E + ARMIJO_C * t * slope + ENERGY_ROUNDING * max(scale, scale_try):
                break
            t *= 0.5
        step = t * d
        y, E, scale = y_try, E_try, scale_try
        if converged(step, y):
            return y, it, True
        nrm = float(np.linalg.norm(step))
        if stagnation:
            rises = rises + 1 if nrm >= prev_norm else 0
            if rises >= 2:
                return y, it, True
        prev_norm = nrm
    return y, max_iter, False
