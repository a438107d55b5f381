"""Rate-and-state friction and the equilibrium solve (oracle).

* strength tau = sigma_n [f_* + a ln(V/V_*) + b ln(V_* theta / D_c)]
  (Section 2.2, eq. "R&S_friction"; the printed form has b ln(V theta / D_c),
  read as b ln(V_* theta / D_c), the form whose steady state is theta = D_c / V_*
  as the paper states next to it);
* intermediate state law dtheta/dt = (1/eps)[(V theta/D_c)^(-eps) - 1] V theta / D_c,
  eps = 1 giving the aging law dtheta/dt = 1 - V theta / D_c (eq. "state_evolution_law");
* the state after a step at constant slip rate in closed form (the reading
  taken when the explicit state update would leave theta <= 0, see seas.py);
* equilibrium on every element (eq. "force_balance" with the traction split of
  eq. "superimposition2"):  tau0 + f - mu/(2 cs) V = strength(V, theta),
  solved for V by Newton-Raphson (Section 2.4, step 2).

The unknown is x = ln V.  g(x) = A - eta e^x - sigma_n [f_* + a (x - ln V_*) +
b ln(V_* theta/D_c)] is strictly decreasing and concave, so the root is unique.
From the right of the root (g < 0) every Newton step is downward and stays
right of it (the tangent of a concave function lies above it), so downward
steps are taken whole. From the left (g > 0) the tangent can overshoot far to
the right; there A - c - sigma_n a x > eta e^x > 0, and at the root
eta e^x* = A - c - sigma_n a x* < A - c - sigma_n a x, so the root lies below
ln((A - c - sigma_n a x)/eta): upward steps longer than 1 stop there (but move
at least 1; near the root that bound is lost to cancellation and the steps are
short anyway). x is kept >= X_MIN =
-690 (V >= ~1e-300: a rate that is zero for every purpose), where a root below
it leaves the iterate. Stop when |dx| <= tol max(1, |x|).
"""
from __future__ import annotations

import numpy as np


def strength(V, theta, a, b, Dc, sigma_n, V0, f0):
    return sigma_n * (f0 + a * np.log(V / V0) + b * np.log(V0 * theta / Dc))


def state_rate(V, theta, Dc, eps=1.0):
    r = V * theta / Dc
    if np.all(np.asarray(eps) == 1.0):
        return 1.0 - r
    return (1.0 / eps) * (r ** (-eps) - 1.0) * r


def state_at_constant_rate(theta0, V, Dc, dt, eps=1.0):
    """State after dt at a constant slip rate V, from the state law integrated in
    closed form: with u = (V theta / Dc)^eps the law reads du/dt = (V/Dc)(1 - u),
    so u(dt) = 1 + (u(0) - 1) exp(-V dt / Dc) and theta = (Dc/V) u^(1/eps)
    (eps = 1: theta = Dc/V + (theta0 - Dc/V) exp(-V dt/Dc), the aging law).
    Positive for every dt, unlike the explicit update. Written as
    theta0 e^-x + (Dc/V)(1 - e^-x), x = V dt/Dc, with 1 - e^-x = -expm1(-x), so
    that a locked element (x ~ 1e-25) keeps its state instead of losing it to
    cancellation."""
    x = V * dt / Dc
    e = np.exp(-x)
    one_m = -np.expm1(-x)
    eps = np.asarray(eps, float)
    if np.all(eps == 1.0):
        return theta0 * e + Dc / V * one_m
    u0 = (V * theta0 / Dc) ** eps
    return Dc / V * (u0 * e + one_m) ** (1.0 / eps)


class NotConverged(RuntimeError):
    pass


X_MIN = -690.0


def solve_velocity(A, theta, eta, a, b, Dc, sigma_n, V0, f0, x0, tol=1e-14, max_iter=50):
    """Vectorised Newton on x = ln V for  A - eta V = strength(V, theta).

    Every element iterates independently (a converged element is frozen), so the
    result equals a scalar Newton run element by element."""
    A = np.asarray(A, float)
    x = np.maximum(np.array(x0, dtype=float, copy=True), X_MIN) * np.ones_like(A)
    c = sigma_n * (f0 - a * np.log(V0) + b * np.log(V0 * theta / Dc))
    active = np.ones(A.shape, bool)
    for _ in range(max_iter):
        if not active.any():
            break
        ex = np.exp(x)
        g = A - eta * ex - c - sigma_n * a * x
        dg = -eta * ex - sigma_n * a
        step = -g / dg
        with np.errstate(invalid="ignore", divide="ignore"):
            cap = np.log(np.maximum(A - c - sigma_n * a * x, 1e-300) / eta)
        up = np.where(step > 1.0, np.minimum(step, np.maximum(cap - x, 1.0)), step)
        xn = np.where(step > 0, x + up, np.maximum(x + step, X_MIN))
        dx = np.where(active, xn - x, 0.0)
        x = x + dx
        active = active & (np.abs(dx) > tol * np.maximum(1.0, np.abs(x)))
    if active.any():
        raise NotConverged(f"{int(active.sum())} elements did not converge")
    if not np.all(np.isfinite(x)):
        raise NotConverged(f"{int(np.sum(~np.isfinite(x)))} elements met a non-finite force balance")
    return np.exp(x)
