"""Selective H-matrix block partition (oracle).

Section 2.3.2 of the paper ("Fault-wise hierarchical decomposition,
admissibility, and block extraction"):

* one binary cluster tree per fault, built by recursive subdivision until a
  cluster holds no more than eta_leaf elements;
* each cluster is enclosed in a bounding circle: centre c = mean of the element
  centroids, radius r = max_i(|x_i - c| + ds/2);
* two clusters are admissible (well separated) when |c_obs - c_src| >
  eta_H (r_obs + r_src) (eq. "admissibility_condition");
* a dual-tree traversal from the two roots of every ordered pair (receiver a,
  source b), a != b, records admissible blocks, labels failing leaf-leaf pairs
  near-field, and otherwise splits the cluster with the larger radius unless it
  is a leaf (then the other); on equal radii the receiver cluster is split.

Subdivision halves a cluster's element range (the first child takes the lower
half, floor(n/2) elements).  For a straight, uniformly meshed fault the circle's
centre is the midpoint of the cluster and its radius is n ds / 2; both the
literal max-formula and this closed form are provided, and the traversal uses
the closed form so that ties between equal clusters are decided exactly.
"""
from __future__ import annotations

import numpy as np


class Cluster:
    __slots__ = ("lo", "hi", "c", "r", "kids")

    def __init__(self, lo, hi, c, r):
        self.lo, self.hi, self.c, self.r, self.kids = lo, hi, c, r, None

    @property
    def n(self):
        return self.hi - self.lo

    def is_leaf(self):
        return self.kids is None


def circle_literal(f, lo, hi):
    """Centre = mean of centroids; radius = max |x_i - c| + ds/2 (as printed)."""
    pts = f.mid[lo:hi]
    c = pts.mean(axis=0)
    r = float(np.max(np.hypot(pts[:, 0] - c[0], pts[:, 1] - c[1]) + 0.5 * f.dx))
    return c, r


def circle_closed(f, lo, hi):
    """Same circle for a straight uniform mesh: centre at the cluster midpoint,
    radius (hi - lo) ds / 2."""
    s = -0.5 * f.L + 0.5 * (lo + hi) * f.dx
    return f.c + s * f.t, 0.5 * (hi - lo) * f.dx


def build_tree(f, leaf):
    def rec(lo, hi):
        c, r = circle_closed(f, lo, hi)
        node = Cluster(lo, hi, c, r)
        if hi - lo > leaf:
            mid = lo + (hi - lo) // 2
            node.kids = (rec(lo, mid), rec(mid, hi))
        return node
    return rec(0, f.Np)


def admissible(co, cs_, eta_H):
    d = float(np.hypot(co.c[0] - cs_.c[0], co.c[1] - cs_.c[1]))
    return d > eta_H * (co.r + cs_.r)


def dual_traversal(tr, ts, eta_H):
    """Blocks of one ordered pair as (r_lo, r_hi, s_lo, s_hi, is_admissible),
    in depth-first order (first child before second)."""
    out = []

    def rec(o, s):
        if admissible(o, s, eta_H):
            out.append((o.lo, o.hi, s.lo, s.hi, True))
            return
        if o.is_leaf() and s.is_leaf():
            out.append((o.lo, o.hi, s.lo, s.hi, False))
            return
        if o.r > s.r:
            split_obs = not o.is_leaf()
        elif s.r > o.r:
            split_obs = s.is_leaf()
        else:
            split_obs = not o.is_leaf()
        if split_obs:
            for k in o.kids:
                rec(k, s)
        else:
            for k in s.kids:
                rec(o, k)

    rec(tr, ts)
    return out


def partition(geo, eta_H, leaf):
    """Block lists of every ordered pair (a, b), a != b (self blocks excluded)."""
    trees = [build_tree(f, leaf) for f in geo]
    blocks = {}
    for a in range(len(geo)):
        for b in range(len(geo)):
            if a != b:
                blocks[(a, b)] = dual_traversal(trees[a], trees[b], eta_H)
    return blocks
