"""Fault discretisation (oracle).

Each fault is a straight segment split into ``n_elem`` equal piecewise-constant
elements collocated at their midpoints (Section 2.3.1, "Discretization &
truncation"; Section 3.1 for the local frame e1' = e3 x e2', e2' = n).
The time step is a fixed fraction beta of the shortest element crossing time
(Section 2.3.1; Section 3.1 gives beta = 1/2 and the worked value of dt_min).
"""
from __future__ import annotations

import numpy as np


class Fault:
    def __init__(self, d):
        self.c = np.array([d["cx"], d["cy"]], dtype=np.float64)
        n = np.array([d["nx"], d["ny"]], dtype=np.float64)
        self.n = n / np.hypot(n[0], n[1])
        # e1' = e3 x e2' with e2' = n (right-handed local basis)
        self.t = np.array([-self.n[1], self.n[0]])
        self.L = float(d["length"])
        self.Np = int(d["n_elem"])
        self.dx = self.L / self.Np
        # xi_j measured from the fault centre: -L/2 + (j + 1/2) dx
        self.xi = -0.5 * self.L + (np.arange(self.Np) + 0.5) * self.dx
        self.mid = self.c[None, :] + self.xi[:, None] * self.t[None, :]
        self.ends = np.stack([self.c - 0.5 * self.L * self.t, self.c + 0.5 * self.L * self.t])


def discretize(faults):
    return [Fault(d) for d in faults]


def mirror_images(faults, y0):
    """Method of images for a traction-free line y = y0 (anti-plane): each fault's
    reflection. Reflection maps the normal (nx, ny) to (nx, -ny) and reverses the
    order of the elements along the tangent; the image is given the opposite
    normal (-nx, ny), which restores the order (element j of the image is the
    reflection of element j), so that the even continuation of the displacement,
    whose jump across the reflected normal equals the original slip, is a slip of
    minus the original's across this normal."""
    return [dict(f, cx=float(f["cx"]), cy=2.0 * y0 - float(f["cy"]), nx=-float(f["nx"]), ny=float(f["ny"]))
            for f in faults]


def offsets(geo):
    """Global index of each fault's first element."""
    off = [0]
    for f in geo:
        off.append(off[-1] + f.Np)
    return off


def time_step(geo, cs, beta=0.5):
    """dt_min = beta * min_i(dx_i) / cs."""
    return beta * min(f.dx for f in geo) / cs
