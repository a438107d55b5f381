"""Prescribed-history stress evaluation and the SEAS predictor-corrector (oracle).

The stress transfer is the history functional f of eq. "superimposition2"
(radiation damping excluded), split as in eq. "traction_decomposition" into the
spectral self term of each fault and the fault-to-fault space-time term.

Time indexing (Section 2.3.2 and Section 2.4, as read here):
V^m is the slip rate held over [t_m, t_{m+1}]; the interaction stress at t_{h+1}
is sum_T K^T V^{h-T}; the self term at t_s uses D^{s-T}, T = 0..W_n, where D^s is
the transform of the slip at t_s.

* prescribed mode (stress evaluation of a given rate history): for n = 1..n_steps,
  delta^n = delta^{n-1} + dt V^{n-1}, f^n = f_self(D^n, D^{n-1}, ...) +
  f_int(V^{n-1}, V^{n-2}, ...);
* SEAS mode, one step t_n -> t_{n+1} (Section 2.4 steps 2 and 3): predictor with
  delta* = delta^n + dt V^n, theta* = theta^n + dt thetadot^n, D* = DFT(delta*),
  Newton for V*; corrector with the averages of V and thetadot, in which only the
  lag-0 terms change; V** and D** are appended to the histories;
* adaptive steps (Section 2.4.1, step 1): a step of g = ceil(min_i xi Dc_i/V_i /
  dt) grid steps (at least 1) with the histories kept on the dt grid; the interior
  grid rows of a step are filled as SeasState.step states.
"""
from __future__ import annotations

import math

import numpy as np

from . import friction, geometry, hpartition, interaction, selfterm


class Problem:
    def __init__(self, faults, params, n_hist_max=None, use_c=True, dense=True):
        p = dict(params)
        self.p = p
        self.geo = geometry.discretize(faults)
        self.off = geometry.offsets(self.geo)
        self.N = self.off[-1]
        self.mu, self.cs = float(p["mu"]), float(p["cs"])
        self.eta = self.mu / (2 * self.cs)
        self.dt = geometry.time_step(self.geo, self.cs, float(p.get("beta", 0.5)))
        self.with_tail = bool(p.get("int_tail", 1))
        self.inter = None
        # free surface (method of images): the mirror images act as extra sources
        self.images = None
        if int(p.get("free_surface", 0)):
            self.images = geometry.discretize(geometry.mirror_images(faults, float(p.get("surface_y", 0.0))))
        if dense:
            blocks = None
            if int(p.get("cluster_windows", 0)):
                blocks = hpartition.partition(self.geo + (self.images or []), float(p.get("eta_H", 2.0)),
                                              int(p.get("leaf", 50)))
            self.inter = interaction.DenseInteraction(
                self.geo, self.mu, self.cs, self.dt, float(p.get("eta_tmin", 0.01)),
                float(p.get("eta_tmax", 0.01)), windowed=True, max_lag=n_hist_max,
                with_tail=self.with_tail, blocks=blocks, images=self.images)
        self.selfs = []
        cache = {}
        for f in self.geo:
            key = (f.Np, f.L)
            if key not in cache:
                cache[key] = selfterm.SelfTerm(f.Np, f.L, self.mu, self.cs, self.dt,
                                               float(p.get("eta_w", 1.5)), int(p.get("q_w", 0)),
                                               int(p.get("mode_cap", 0)), use_c=use_c,
                                               tail=bool(int(p.get("self_tail", 0))))
            self.selfs.append(cache[key])

    # ------------------------------------------------------------------ helpers
    def dfts(self, delta):
        return [self.selfs[k].dft(delta[self.off[k]:self.off[k + 1]]) for k in range(len(self.geo))]

    def self_stress(self, Dh, t, first, D_now=None):
        f = np.zeros(self.N)
        for k in range(len(self.geo)):
            now = None if D_now is None else D_now[k]
            f[self.off[k]:self.off[k + 1]] = self.selfs[k].stress(Dh[k], t, first, now)
        return f

    def expired(self, Vh, head, first):
        return self.inter.expired_slip(Vh, head, first, self.dt) if self.with_tail else None


def prescribed(prob, V, prior_V=None, delta0=None):
    """Stress history f^n, n = 1..n_steps, for the slip rates V[m], m = 0..n_steps-1.

    ``prior_V`` (H x N, oldest first) are the rates of steps -H..-1; slip before
    t = 0 follows from delta^{m+1} = delta^m + dt V^m with delta^0 = ``delta0``."""
    V = np.asarray(V, float)
    n_steps, N = V.shape
    H = 0 if prior_V is None else len(prior_V)
    Vall = V if H == 0 else np.concatenate([prior_V, V])
    first = -H
    d0 = np.zeros(N) if delta0 is None else np.asarray(delta0, float)
    # slip at t_m for m = -H..n_steps
    delta = np.empty((H + n_steps + 1, N))
    delta[H] = d0
    for m in range(-1, -H - 1, -1):
        delta[m + H] = delta[m + 1 + H] - prob.dt * Vall[m + H]
    for m in range(0, n_steps):
        delta[m + 1 + H] = delta[m + H] + prob.dt * Vall[m + H]
    nf = len(prob.geo)
    Dh = [np.array([prob.selfs[k].dft(delta[i, prob.off[k]:prob.off[k + 1]])
                    for i in range(len(delta))]) for k in range(nf)]
    out = np.zeros((n_steps, N))
    for n in range(1, n_steps + 1):
        head = n - 1
        f_int = prob.inter.stress(Vall, head, first, expired=prob.expired(Vall, head, first))
        f_self = prob.self_stress(Dh, n, first)
        out[n - 1] = f_self + f_int
    return out


class SeasState:
    """SEAS state and the predictor-corrector step of Section 2.4.

    ``state_update``: "explicit" is the update as printed (theta* = theta +
    dt thetadot, the corrector with the average of the two state rates);
    "exact" integrates the state law in closed form over the step at constant
    slip rate (V^n in the predictor, the averaged rate in the corrector), the
    update of the scheme the paper follows for its step, which keeps theta > 0
    where the explicit form cannot (a rate that jumps by many decades in one
    step, as at the nucleation of the paper's two-fault benchmark)."""

    def __init__(self, prob, fric, V0, theta0, tau0, tau0_rate=None, delta0=None,
                 prior_V=None, eps=1.0, state_update="explicit", adaptive=False, xi=0.5, gamma_max=1 << 20):
        self.prob = prob
        self.adaptive = bool(adaptive)
        self.xi = xi
        self.gamma_max = int(gamma_max)
        self.fric = {k: np.asarray(v, float) for k, v in fric.items()}
        self.eps = eps
        assert state_update in ("explicit", "exact")
        self.exact = state_update == "exact"
        N = prob.N
        H = 0 if prior_V is None else len(prior_V)
        self.first = -H
        self.n = 0
        self.V = np.asarray(V0, float).copy()
        self.theta = np.asarray(theta0, float).copy()
        self.tau0 = np.asarray(tau0, float).copy()
        self.tau0_rate = np.zeros(N) if tau0_rate is None else np.asarray(tau0_rate, float)
        self.delta = np.zeros(N) if delta0 is None else np.asarray(delta0, float).copy()
        self.thetadot = friction.state_rate(self.V, self.theta, self.fric["Dc"], eps)
        Vh = [] if prior_V is None else list(np.asarray(prior_V, float))
        Vh.append(self.V.copy())
        self.Vh = Vh                               # rows m = first..n
        dl = [self.delta.copy()]
        for m in range(-1, -H - 1, -1):
            dl.insert(0, dl[0] - prob.dt * Vh[m + H])
        self.Dh = [[prob.selfs[k].dft(d[prob.off[k]:prob.off[k + 1]]) for d in dl]
                   for k in range(len(prob.geo))]
        self.last = {}

    def _solve(self, A, theta, x0):
        F = self.fric
        return friction.solve_velocity(A, theta, self.prob.eta, F["a"], F["b"], F["Dc"],
                                       F["sigma_n"], F["V0"], F["f0"], x0)

    def gamma(self):
        """Length of the next step in units of Delta t_min (Section 2.4.1, step 1):
        gamma = ceil(Delta t_ev / Delta t_min), Delta t_ev = min_i xi Dc_i / V_i, at
        least 1 and at most gamma_max; 1 for the fixed step."""
        if not self.adaptive:
            return 1
        dt_ev = float(np.min(self.xi * self.fric["Dc"] / self.V))
        return max(1, min(int(math.ceil(dt_ev / self.prob.dt)), self.gamma_max))

    def step(self):
        """Advance one predictor-corrector step t_n -> t_{n+g}, g = gamma().

        The rate and slip histories stay on the Delta t_min grid of the kernels.
        Row m of the rate history stands for the interval [t_m, t_m+1); the step's
        intervals are n .. n+g-1, whose last one is the lag-0 interval of the new
        time (its rate: V^n in the predictor, the averaged rate in the corrector).
        Its interior intervals n+1 .. n+g-2 enter the history sums at the step's
        starting rate V^n (one history evaluation per step), and the slip
        coefficients of the interior grid times at the straight line from D^n to the
        predicted D*. Committed: the interior rows n+1 .. n+g-1 take the averaged
        rate (the rate of the slip increment), row n+g the corrected rate, the
        interior slip coefficients the line from D^n to D**. With g = 1 this is the
        fixed step."""
        P = self.prob
        n = self.n
        g = self.gamma()
        dt = g * P.dt
        for _ in range(1, g):                       # interior rows at the starting rate
            self.Vh.append(self.V.copy())
        head = n + g - 1
        Vh = np.array(self.Vh)
        # interaction history part (lags >= 1) and the static tail
        f_hist = P.inter.stress(Vh, head, self.first, min_lag=1, expired=P.expired(Vh, head, self.first))
        # ---- predictor
        d_star = self.delta + dt * self.V
        if self.exact:
            th_star = friction.state_at_constant_rate(self.theta, self.V, self.fric["Dc"], dt, self.eps)
        else:
            th_star = self.theta + dt * self.thetadot
        D_star = P.dfts(d_star)
        D_n = [self.Dh[k][-1] for k in range(len(P.geo))]
        for k in range(len(P.geo)):                 # interior slip coefficients, predicted
            for m in range(1, g):
                self.Dh[k].append(D_n[k] + (m / g) * (D_star[k] - D_n[k]))
        Dh = [np.array(d) for d in self.Dh]
        fs_star = P.self_stress(Dh, n + g, self.first, D_now=D_star)
        fi_star = f_hist + P.inter.lag0_apply(self.V)
        tau0 = self.tau0 + self.tau0_rate * (n + g) * P.dt
        V_star = self._solve(tau0 + fs_star + fi_star, th_star, np.log(self.V))
        thd_star = friction.state_rate(V_star, th_star, self.fric["Dc"], self.eps)
        # ---- corrector
        Vbar = 0.5 * (self.V + V_star)
        thd_bar = 0.5 * (self.thetadot + thd_star)
        d_2 = self.delta + dt * Vbar
        if self.exact:
            th_2 = friction.state_at_constant_rate(self.theta, Vbar, self.fric["Dc"], dt, self.eps)
        else:
            th_2 = self.theta + dt * thd_bar
        D_2 = P.dfts(d_2)
        fs_2 = P.self_stress(Dh, n + g, self.first, D_now=D_2)
        fi_2 = f_hist + P.inter.lag0_apply(Vbar)
        V_2 = self._solve(tau0 + fs_2 + fi_2, th_2, np.log(V_star))
        thd_2 = friction.state_rate(V_2, th_2, self.fric["Dc"], self.eps)
        self.last = dict(f_hist=f_hist, f_self=fs_2, f_int=fi_2, V_star=V_star, gamma=g)
        # ---- commit and append
        self.delta, self.theta, self.V, self.thetadot = d_2, th_2, V_2, thd_2
        for m in range(1, g):
            self.Vh[n + m - self.first] = Vbar.copy()
            for k in range(len(P.geo)):
                self.Dh[k][n + m - self.first] = D_n[k] + (m / g) * (D_2[k] - D_n[k])
        self.Vh.append(V_2.copy())
        for k in range(len(P.geo)):
            self.Dh[k].append(D_2[k])
        self.n = n + g


def prescribed_rows(prob, V_all, first, n, rows, delta0=None):
    """f^n at the global receivers ``rows`` for the rate history V_all[m - first]
    (m = first .. n-1), without building dense operators: interaction rows on the
    fly, the self term of each fault that holds a sampled receiver in full."""
    V_all = np.asarray(V_all, float)
    head = n - 1
    p = prob.p
    f_int = interaction.stress_rows(prob.geo, rows, V_all, head, first, prob.mu, prob.cs, prob.dt,
                                    float(p.get("eta_tmin", 0.01)), float(p.get("eta_tmax", 0.01)),
                                    with_tail=prob.with_tail)
    # slip at t_m for m = first .. n, delta^{first} from delta^0 going backwards
    N = prob.N
    d0 = np.zeros(N) if delta0 is None else np.asarray(delta0, float)
    cum = np.cumsum(V_all[: n - first], axis=0) * prob.dt           # sum_{k < m} V^k, m = first+1..n
    before = np.sum(V_all[: -first], axis=0) * prob.dt if first < 0 else np.zeros(N)
    delta = np.vstack([np.zeros((1, N)), cum]) + (d0 - before)[None, :]   # rows m = first..n
    out = np.zeros(len(rows))
    faults_needed = sorted({int(np.searchsorted(prob.off, r, side="right") - 1) for r in rows})
    for k in faults_needed:
        st = prob.selfs[k]
        lo = max(first, n - st.reach)
        Dh = st.dft(delta[lo - first:n - first + 1, prob.off[k]:prob.off[k + 1]])
        fs = st.stress(Dh, n, lo)
        for idx, r in enumerate(rows):
            if prob.off[k] <= r < prob.off[k + 1]:
                out[idx] = fs[r - prob.off[k]]
    return out + f_int


def lag0_partners(prob, fault):
    """Global indices of the source elements of other faults that act on some
    receiver of ``fault`` through the lag-0 kernel (pairs whose window starts at
    lag 0)."""
    P = prob
    out = set()
    for b in range(len(P.geo)):
        if b == fault:
            continue
        T0, _ = interaction.pair_window_lags(P.geo, fault, b, P.cs, P.dt, float(P.p.get("eta_tmin", 0.01)),
                                             float(P.p.get("eta_tmax", 0.01)))
        if T0 == 0:
            K = interaction.pair_kernel(P.geo, fault, b, 0, P.dt, P.cs)
            out |= {int(P.off[b] + j) for j in np.nonzero(np.any(K != 0.0, axis=0))[0]}
    return sorted(out)


def step_fault(prob, fric, st, fault, f_hist, eps=1.0):
    """One predictor-corrector step (Section 2.4, steps 2 and 3) for the elements
    of one fault of a network too large for dense operators.

    ``st`` holds the state at step n: full-network arrays V, theta, thetadot,
    delta, tau0, tau0_rate, the step index n, and ``Dh``: for every fault g a
    list (first_g, rows) of slip coefficients D^m, m = first_g..n (earlier ones
    zero). ``f_hist`` maps a global receiver index to its interaction history
    part at this step (lags >= 1 and the static tail, e.g. from
    ``interaction.stress_rows``); it must cover the fault's elements and the
    elements of other faults that reach them through the lag-0 kernel.

    The step is SeasState.step restricted to those elements: the corrector's
    self term needs the averaged rate over the whole fault, and its lag-0 term
    the averaged rates of the coupled elements, so the predictor is solved on
    both. Returns V, theta, delta at n + 1 on the fault's elements."""
    P = prob
    dt, n = P.dt, st["n"]
    off = P.off
    eta = P.eta
    rk = np.arange(off[fault], off[fault + 1])
    # lag-0 coupling of the fault's receivers (pairs whose window starts at lag 0)
    partners = lag0_partners(P, fault)
    # the partners' own lag-0 terms at the predictor
    def lag0_at(rows, v):
        out = np.zeros(len(rows))
        for idx, r in enumerate(rows):
            a = int(np.searchsorted(off, r, side="right") - 1)
            for b in range(len(P.geo)):
                if b == a:
                    continue
                T0, _ = interaction.pair_window_lags(P.geo, a, b, P.cs, dt, float(P.p.get("eta_tmin", 0.01)),
                                                     float(P.p.get("eta_tmax", 0.01)))
                if T0 != 0:
                    continue
                Krow = interaction.pair_kernel_row(P.geo, a, r - off[a], b, 0, dt, P.cs)
                out[idx] += -eta * float(Krow @ v[off[b]:off[b + 1]])
        return out
    rows = list(rk) + [r for r in partners if not (off[fault] <= r < off[fault + 1])]
    rows = np.array(rows, dtype=int)
    F = {k: np.asarray(v, float) for k, v in fric.items()}
    fh = np.array([f_hist[int(r)] for r in rows])
    tau0 = st["tau0"][rows] + st["tau0_rate"][rows] * (n + 1) * dt
    faults_of = [int(np.searchsorted(off, r, side="right") - 1) for r in rows]

    def self_at(delta_new):
        out = np.zeros(len(rows))
        for g in sorted(set(faults_of)):
            first_g, Dg = st["Dh"][g]
            Dn = P.selfs[g].dft(delta_new[off[g]:off[g + 1]])
            fs = P.selfs[g].stress(np.asarray(Dg), n + 1, first_g, D_now=Dn)
            for idx, r in enumerate(rows):
                if faults_of[idx] == g:
                    out[idx] = fs[r - off[g]]
        return out
    V, th, thd, de = st["V"], st["theta"], st["thetadot"], st["delta"]
    sub = lambda x: np.asarray(x)[rows]
    # ---- predictor (every involved element)
    d_star = de + dt * V
    th_star = sub(th) + dt * sub(thd)
    fs_star = self_at(d_star)
    fi_star = fh + lag0_at(rows, V)
    solve = lambda A, theta, x0: friction.solve_velocity(A, theta, eta, sub(F["a"]), sub(F["b"]), sub(F["Dc"]),
                                                         sub(F["sigma_n"]), sub(F["V0"]), sub(F["f0"]), x0)
    V_star = solve(tau0 + fs_star + fi_star, th_star, np.log(sub(V)))
    e_ = eps if np.isscalar(eps) else sub(eps)
    thd_star = friction.state_rate(V_star, th_star, sub(F["Dc"]), e_)
    # ---- corrector (the fault's elements; its self term needs the whole fault)
    Vbar_full = V.copy()
    Vbar_full[rows] = 0.5 * (sub(V) + V_star)
    nk = len(rk)
    thd_bar = 0.5 * (sub(thd)[:nk] + thd_star[:nk])
    d2_full = de.copy()
    d2_full[rk] = de[rk] + dt * Vbar_full[rk]
    th2 = sub(th)[:nk] + dt * thd_bar
    first_k, Dk = st["Dh"][fault]
    D2 = P.selfs[fault].dft(d2_full[rk])
    fs2 = P.selfs[fault].stress(np.asarray(Dk), n + 1, first_k, D_now=D2)
    fi2 = fh[:nk] + lag0_at(list(rk), Vbar_full)
    Fk = {k: v[rk] for k, v in F.items()}
    V2 = friction.solve_velocity(tau0[:nk] + fs2 + fi2, th2, eta, Fk["a"], Fk["b"], Fk["Dc"], Fk["sigma_n"],
                                 Fk["V0"], Fk["f0"], np.log(V_star[:nk]))
    return dict(V=V2, theta=th2, delta=d2_full[rk], rows=rk, f_self=fs2, f_int=fi2, partners=partners)
