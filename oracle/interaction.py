"""Fault-to-fault space-time interaction (oracle).

Follows Section 2.3.2 of the paper:

* the antiplane primitives I_31, I_32 (eq. "primitives"), with H(0) = 0 and
  sgn(0) = 0, so that every primitive vanishes at t = 0;
* the discrete kernel as a space-time finite difference of the primitives over
  the source element (eq. "kernel_interactions");
* the stress at a receiver as -mu/(2 cs) times the receiver normal (expressed in
  the source element's frame) contracted with the kernel, summed over source
  elements and lags (eq. "fault-to-fault_interactions_discretized");
* the causality window [T_init, T_end] of each fault pair ("Truncation of
  elastodynamic time-window" paragraph, eq. "early_time");
* the static dipole stress used for slip that has left a pair's window (the
  late-time limit of the same kernel: the 2-D kernel does not decay to zero, so
  the slip that leaves a window keeps its static stress).

Everything is dense and uncompressed, FP64.
"""
from __future__ import annotations

import math

import numpy as np


def _heaviside(x):
    """H(x) = 1 for x > 0, else 0 (so H(0) = 0)."""
    return (x > 0).astype(np.float64)


def primitive_I31(r1, r2, t, cs):
    """I_31 = -(r2/(pi r)) H(t - r/cs) sqrt((cs t / r)^2 - 1).

    (cs t/r)^2 - 1 is evaluated as (cs t - r)(cs t + r)/r^2 (same value, no
    cancellation near the front)."""
    r1, r2 = np.broadcast_arrays(np.asarray(r1, float), np.asarray(r2, float))
    r = np.hypot(r1, r2)
    ct = cs * np.asarray(t, float)
    on = ct > r
    Q = np.sqrt(np.where(on, (ct - r) * (ct + r), 0.0))   # = r sqrt((ct/r)^2 - 1)
    rr = np.where(r > 0, r * r, 1.0)
    return np.where(on, -r2 * Q / (math.pi * rr), 0.0)


def primitive_I32(r1, r2, t, cs):
    """I_32 = H(r1) H(t - |r2|/cs)
              + (1/pi) sgn(r1) H(t - r/cs) [ |r1|/r sqrt((cs t/r)^2 - 1)
                                             - arccos(|r1| / sqrt((cs t)^2 - r2^2)) ].

    Inside the active region cs t > r, arccos(|r1|/S) with S^2 = (cs t)^2 - r2^2
    equals atan2(sqrt(S^2 - r1^2), |r1|) = atan2(Q, |r1|), Q^2 = (cs t)^2 - r^2,
    which is the same angle without arccos's loss of accuracy near 1."""
    r1, r2 = np.broadcast_arrays(np.asarray(r1, float), np.asarray(r2, float))
    r = np.hypot(r1, r2)
    ct = cs * np.asarray(t, float)
    plane = _heaviside(r1) * _heaviside(ct - np.abs(r2))
    on = ct > r
    Q = np.sqrt(np.where(on, (ct - r) * (ct + r), 0.0))
    ar1 = np.abs(r1)
    rr = np.where(r > 0, r * r, 1.0)
    cyl = np.where(on, ar1 * Q / rr - np.arctan2(Q, ar1), 0.0)
    return plane + np.sign(r1) * cyl / math.pi


def local_offsets(geo, a, b):
    """Receiver (fault a) midpoints in the frame of each source element of fault b.

    Returns r1' (p x q), r2' (p x q) and the receiver normal in the source frame
    n1' = n_a . e1'_b, n2' = n_a . e2'_b."""
    A, B = geo[a], geo[b]
    d = A.mid[:, None, :] - B.mid[None, :, :]
    r1p = d[..., 0] * B.t[0] + d[..., 1] * B.t[1]
    r2p = d[..., 0] * B.n[0] + d[..., 1] * B.n[1]
    n1p = float(A.n @ B.t)
    n2p = float(A.n @ B.n)
    return r1p, r2p, n1p, n2p


def kernel_from_offsets(r1p, r2p, n1p, n2p, ds, T, dt, cs):
    """K^T = n1' K_31^T + n2' K_32^T with

    K_3l^T = I_3l(r1'+ds/2, r2', (T+1)dt) - I_3l(r1'-ds/2, r2', (T+1)dt)
           - I_3l(r1'+ds/2, r2', T dt)     + I_3l(r1'-ds/2, r2', T dt)."""
    t1 = (T + 1) * dt
    t0 = T * dt
    out = 0.0
    for w, prim in ((n1p, primitive_I31), (n2p, primitive_I32)):
        if w == 0.0:
            continue
        k = (prim(r1p + 0.5 * ds, r2p, t1, cs) - prim(r1p - 0.5 * ds, r2p, t1, cs)
             - prim(r1p + 0.5 * ds, r2p, t0, cs) + prim(r1p - 0.5 * ds, r2p, t0, cs))
        out = out + w * k
    return out


def pair_kernel(geo, a, b, T, dt, cs):
    """Dense kernel matrix of the (receiver a, source b) pair at lag T, p x q."""
    r1p, r2p, n1p, n2p = local_offsets(geo, a, b)
    return kernel_from_offsets(r1p, r2p, n1p, n2p, geo[b].dx, T, dt, cs)


def pair_kernel_row(geo, a, i, b, T, dt, cs):
    """Row i of the pair kernel at lag T (receiver i of fault a, all sources of b)."""
    A, B = geo[a], geo[b]
    d = A.mid[i][None, :] - B.mid
    r1p = d[:, 0] * B.t[0] + d[:, 1] * B.t[1]
    r2p = d[:, 0] * B.n[0] + d[:, 1] * B.n[1]
    return kernel_from_offsets(r1p, r2p, float(A.n @ B.t), float(A.n @ B.n), B.dx, T, dt, cs)


def pair_kernel_stack(geo, a, b, lags, dt, cs):
    r1p, r2p, n1p, n2p = local_offsets(geo, a, b)
    out = np.empty((len(lags),) + r1p.shape)
    for k, T in enumerate(lags):
        out[k] = kernel_from_offsets(r1p, r2p, n1p, n2p, geo[b].dx, T, dt, cs)
    return out


# ----------------------------------------------------------------------------
# Causality window of a fault pair
# ----------------------------------------------------------------------------
def arrival_times(geo, a, b, cs):
    """T_arr(i, j) = min(r, |r2'|)/cs if r1' > 0, else r/cs (element centres)."""
    r1p, r2p, _, _ = local_offsets(geo, a, b)
    r = np.hypot(r1p, r2p)
    return np.where(r1p > 0, np.minimum(r, np.abs(r2p)), r) / cs


def pair_window_times(geo, a, b, cs, eta_tmin, eta_tmax):
    """(T_init, T_end) in seconds: T_init = (1 - eta_Tmin) min T_arr; T_max is the
    largest distance from a source midpoint to an end point of the receiver
    fault, over cs; T_end = (1 + eta_Tmax) T_max."""
    T_earl = float(arrival_times(geo, a, b, cs).min())
    ends = geo[a].ends
    src = geo[b].mid
    dmax = float(np.sqrt(((src[:, None, :] - ends[None, :, :]) ** 2).sum(-1)).max())
    return (1.0 - eta_tmin) * T_earl, (1.0 + eta_tmax) * dmax / cs


def pair_window_lags(geo, a, b, cs, dt, eta_tmin, eta_tmax):
    """Lag window: T_init rounded down and T_end rounded up to whole steps."""
    t0, t1 = pair_window_times(geo, a, b, cs, eta_tmin, eta_tmax)
    return int(math.floor(t0 / dt)), int(math.ceil(t1 / dt))


def block_window_end(geo, a, b, blk, cs, dt, eta_tmax):
    """Upper lag of one H-matrix block under cluster-level truncation (Section 4.3
    proposes truncating at the level of the cluster pairs of the hierarchical
    partition instead of whole fault pairs): the pair rule applied to the block,
    T_max = the largest distance from a source midpoint of the source cluster to an
    end point of the receiver cluster (its outer element edges), over cs;
    T_end = ceil((1 + eta_Tmax) T_max / dt)."""
    r0, r1, s0, s1 = blk[:4]
    A, B = geo[a], geo[b]
    ends = np.array([A.c + (-0.5 * A.L + r0 * A.dx) * A.t, A.c + (-0.5 * A.L + r1 * A.dx) * A.t])
    src = B.mid[s0:s1]
    dmax = float(np.sqrt(((src[:, None, :] - ends[None, :, :]) ** 2).sum(-1)).max())
    return int(math.ceil((1.0 + eta_tmax) * dmax / cs / dt))


# ----------------------------------------------------------------------------
# Static dipole stress (late-time limit of -mu/(2cs) K^T / dt)
# ----------------------------------------------------------------------------
def static_from_offsets(r1p, r2p, n1p, n2p, ds, mu):
    """Static stress per unit slip of a source element seen at offsets (r1', r2')
    in its frame, receiver normal (n1', n2') in the same frame:

    sigma_31 = (mu/2pi) r2' (1/r_+^2 - 1/r_-^2)
    sigma_32 = -(mu/2pi) (r1_+/r_+^2 - r1_-/r_-^2),    r1_+- = r1' +- ds/2,
    G = n1' sigma_31 + n2' sigma_32."""
    rp1, rm1 = r1p + 0.5 * ds, r1p - 0.5 * ds
    rp2 = rp1 * rp1 + r2p * r2p
    rm2 = rm1 * rm1 + r2p * r2p
    s31 = mu / (2 * math.pi) * r2p * (1.0 / rp2 - 1.0 / rm2)
    s32 = -mu / (2 * math.pi) * (rp1 / rp2 - rm1 / rm2)
    return n1p * s31 + n2p * s32


def static_dipole(geo, a, b, mu):
    """Stress at receivers of fault a per unit slip on each element of fault b
    (two screw dislocations at the element's ends), p x q."""
    r1p, r2p, n1p, n2p = local_offsets(geo, a, b)
    return static_from_offsets(r1p, r2p, n1p, n2p, geo[b].dx, mu)


# ----------------------------------------------------------------------------
# Dense operator and its application
# ----------------------------------------------------------------------------
class DenseInteraction:
    """All ordered pairs (a != b): lag windows, dense kernel stacks over the
    window, and the static tail matrices."""

    def __init__(self, geo, mu, cs, dt, eta_tmin=0.01, eta_tmax=0.01, windowed=True,
                 max_lag=None, with_tail=True, blocks=None, images=None):
        """``blocks`` (the partition of every pair, from hpartition.partition):
        cluster-level windows, every entry (i, j) truncated at the upper lag of the
        block that holds it (``block_window_end``, at most the pair's T_end); its
        older slip then contributes the static stress per block.

        ``images``: the discretised mirror images of the faults (free surface,
        geometry.mirror_images): every receiver fault a also takes the pair (a,
        image of b) for every b, a included, whose kernel and static matrix enter with
        sign -1 (the image carries minus the slip of b across its own normal) and act
        on the slip rates of fault b. Those pairs are keyed (a, n_faults + b); with
        ``blocks`` the partition must cover them under the same keys."""
        nf = len(geo)
        self.nf = nf
        self.geo_all = list(geo) + (list(images) if images is not None else [])
        geo = self.geo_all
        self.geo, self.mu, self.cs, self.dt = geo, mu, cs, dt
        self.off = [0]
        for f in geo[:nf]:
            self.off.append(self.off[-1] + f.Np)
        self.pairs = {}
        for a in range(nf):
            for b in range(len(geo)):
                if a == b:
                    continue
                if windowed:
                    T0, T1 = pair_window_lags(geo, a, b, cs, dt, eta_tmin, eta_tmax)
                else:
                    T0, T1 = 0, int(max_lag)
                # lags beyond max_lag are not stored; callers guarantee they only
                # meet zero history there (checked in stress()).
                T1s = T1 if max_lag is None else min(T1, int(max_lag))
                lags = np.arange(T0, T1s + 1)
                sgn = -1.0 if b >= nf else 1.0
                K = sgn * pair_kernel_stack(geo, a, b, lags, dt, cs)
                G = sgn * static_dipole(geo, a, b, mu) if with_tail else None
                P = dict(T0=T0, T1=T1, T1s=T1s, K=K, G=G, src=b % nf)
                if blocks is not None:
                    bl = [(r0, r1, s0, s1, min(T1, block_window_end(geo, a, b, (r0, r1, s0, s1), cs, dt, eta_tmax)))
                          for r0, r1, s0, s1, _ in blocks[(a, b)]]
                    Tend = np.full(K.shape[1:], -1, dtype=np.int64)
                    for r0, r1, s0, s1, te in bl:
                        Tend[r0:r1, s0:s1] = te
                    assert np.all(Tend >= 0), "the partition must cover the pair"
                    P["blocks"] = bl
                    P["Tend"] = Tend
                    # entries past their block's window are dropped from the stack
                    P["K"] = np.where(lags[:, None, None] <= Tend[None], K, 0.0)
                self.pairs[(a, b)] = P

    def stress(self, Vh, head, first, min_lag=0, expired=None):
        """f_i = -mu/(2cs) sum_{b != a} sum_{T=max(T_init,min_lag)}^{T_end} sum_j K^T_ij V_j^{head-T}
        (+ sum_j G_ij E^{ab}_j, the static stress of slip that left the window,
        when ``expired`` maps (a, b) to E^{ab}).

        ``Vh[m - first]`` is the global slip-rate vector of step m; rates before
        ``first`` are zero (no history)."""
        eta = self.mu / (2 * self.cs)
        f = np.zeros(self.off[-1])
        for (a, b), P in self.pairs.items():
            rb = slice(self.off[P["src"]], self.off[P["src"] + 1])
            if P["T1s"] < P["T1"] and head - (P["T1s"] + 1) >= first:
                raise ValueError("history reaches lags that were not stored")
            lags = np.arange(P["T0"], P["T1s"] + 1)
            ms = head - lags
            ok = (ms >= first) & (lags >= min_lag)
            acc = np.zeros(self.geo[a].Np)
            if ok.any():
                hv = Vh[ms[ok] - first][:, rb]                  # (n_lags, q)
                acc = -eta * np.einsum("tpq,tq->p", P["K"][ok], hv, optimize=False)
            if expired is not None and P["G"] is not None:
                if "blocks" in P:
                    # per block: slip older than the block's window, static stress
                    for r0, r1, s0, s1, te in P["blocks"]:
                        last = head - te - 1
                        if last >= first:
                            c0 = self.off[P["src"]]
                            E = self.dt * np.sum(Vh[: last - first + 1, c0 + s0:c0 + s1], axis=0)
                            acc[r0:r1] += P["G"][r0:r1, s0:s1] @ E
                else:
                    acc = acc + P["G"] @ expired[(a, b)]
            f[self.off[a]:self.off[a + 1]] += acc
        return f

    def lag0_apply(self, v):
        """-mu/(2cs) K^0 v over the pairs whose window starts at lag 0."""
        eta = self.mu / (2 * self.cs)
        f = np.zeros(self.off[-1])
        for (a, b), P in self.pairs.items():
            if P["T0"] == 0:
                sb = P["src"]
                f[self.off[a]:self.off[a + 1]] += -eta * (P["K"][0] @ v[self.off[sb]:self.off[sb + 1]])
        return f

    def expired_slip(self, Vh, head, first, dt):
        """E^{ab}_j = dt sum_{first <= m <= head - T_end - 1} V_j^m for every pair."""
        out = {}
        for (a, b), P in self.pairs.items():
            last = head - P["T1"] - 1
            rb = slice(self.off[P["src"]], self.off[P["src"] + 1])
            if last >= first:
                out[(a, b)] = dt * np.sum(Vh[: last - first + 1, rb], axis=0)
            else:
                out[(a, b)] = np.zeros(self.geo[b].Np)
        return out


# ----------------------------------------------------------------------------
# Row-sampled evaluation (large networks: kernel rows evaluated on the fly)
# ----------------------------------------------------------------------------
def stress_rows(geo, rows, Vh, head, first, mu, cs, dt, eta_tmin=0.01, eta_tmax=0.01,
                min_lag=0, with_tail=True):
    """The same sum as ``DenseInteraction.stress`` for the global receiver indices
    ``rows`` only, with each receiver's kernel row computed lag by lag."""
    off = [0]
    for f in geo:
        off.append(off[-1] + f.Np)
    eta = mu / (2 * cs)
    win = {}
    out = np.zeros(len(rows))
    for k, r in enumerate(rows):
        a = int(np.searchsorted(off, r, side="right") - 1)
        i = r - off[a]
        acc = 0.0
        for b in range(len(geo)):
            if b == a:
                continue
            if (a, b) not in win:
                win[(a, b)] = pair_window_lags(geo, a, b, cs, dt, eta_tmin, eta_tmax)
            T0, T1 = win[(a, b)]
            A, B = geo[a], geo[b]
            d = A.mid[i][None, :] - B.mid
            r1p = d[:, 0] * B.t[0] + d[:, 1] * B.t[1]
            r2p = d[:, 0] * B.n[0] + d[:, 1] * B.n[1]
            n1p, n2p = float(A.n @ B.t), float(A.n @ B.n)
            lags = np.arange(max(T0, min_lag), T1 + 1)
            ms = head - lags
            ok = ms >= first
            if ok.any():
                Kr = kernel_from_offsets(r1p[None, :], r2p[None, :], n1p, n2p, B.dx,
                                         lags[ok][:, None], dt, cs)
                hv = Vh[ms[ok] - first][:, off[b]:off[b + 1]]
                acc += -eta * float(np.sum(Kr * hv))
            if with_tail:
                last = head - T1 - 1
                if last >= first:
                    E = dt * np.sum(Vh[: last - first + 1, off[b]:off[b + 1]], axis=0)
                    G = static_from_offsets(r1p, r2p, n1p, n2p, B.dx, mu)
                    acc += float(G @ E)
        out[k] = acc
    return out
