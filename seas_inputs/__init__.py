"""Seeded synthetic inputs for the 2-D antiplane SEAS stress-transfer path.

This module only draws random numbers and lays out geometry, parameters and
initial fields. It holds none of the method's arithmetic (no kernels, no
convolutions, no friction solves), so that the oracle under ``oracle/`` and the
HIP library under ``paper_2603_00383_amd/`` can both consume the same inputs
without sharing any computational code.

Faults are dictionaries ``{cx, cy, nx, ny, length, n_elem}``: centroid, unit
normal (the along-fault tangent is e3 x n = (-ny, nx), see the paper's
two-fault set-up, Section 3.1) and element count.  All values are SI units.
"""
from __future__ import annotations

import math

import numpy as np

# Material of every workload (antiplane, Section 2; mu and cs of the
# stress-evaluation workloads).
MU = 32.0e9
CS = 3464.0


def fault(cx, cy, strike_deg, length, n_elem):
    """A straight fault whose tangent makes ``strike_deg`` (counter-clockwise
    from +x) and whose normal is chosen so that e3 x n equals that tangent."""
    phi = math.radians(strike_deg)
    return dict(cx=float(cx), cy=float(cy), nx=math.sin(phi), ny=-math.cos(phi),
                length=float(length), n_elem=int(n_elem))


def free_surface_network(n_elem=32, dx=50.0, y0=0.0):
    """Two faults below a traction-free line y = y0: a vertical one whose upper end
    touches the line (the BP1-FD geometry of the paper's appendix, shortened) and a
    buried one dipping 30 degrees whose upper end sits 200 m below the line."""
    L = n_elem * dx
    f1 = fault(0.0, y0 - 0.5 * L, 90.0, L, n_elem)
    phi = math.radians(30.0)
    top = (700.0, y0 - 200.0)
    f2 = fault(top[0] + 0.5 * L * math.cos(phi), top[1] - 0.5 * L * math.sin(phi), -30.0, L, n_elem)
    return [f1, f2]


def fault_nodes(f):
    """Element end points of a fault, shape (n_elem+1, 2) (input validation only)."""
    tx, ty = -f["ny"], f["nx"]
    s = np.linspace(-0.5 * f["length"], 0.5 * f["length"], f["n_elem"] + 1)
    return np.stack([f["cx"] + s * tx, f["cy"] + s * ty], axis=1)


def fault_midpoints(f):
    tx, ty = -f["ny"], f["nx"]
    dx = f["length"] / f["n_elem"]
    s = -0.5 * f["length"] + (np.arange(f["n_elem"]) + 0.5) * dx
    return np.stack([f["cx"] + s * tx, f["cy"] + s * ty], axis=1)


def _min_midpoint_node_distance(faults):
    best = np.inf
    for a, fa in enumerate(faults):
        mid = fault_midpoints(fa)
        for b, fb in enumerate(faults):
            if a == b:
                continue
            nod = fault_nodes(fb)
            d = np.sqrt(((mid[:, None, :] - nod[None, :, :]) ** 2).sum(-1))
            best = min(best, float(d.min()))
    return best


def closest_to_other_faults(faults, k=8):
    """Global indices of the k collocation points nearest another fault's segment
    (point-to-segment distance over the input geometry; near a fault crossing the
    stress sums of a receiver cancel most), and the smallest such distance."""
    mids = [fault_midpoints(f) for f in faults]
    ends = [fault_nodes(f)[[0, -1]] for f in faults]
    dist = []
    for a, m in enumerate(mids):
        d = np.full(len(m), np.inf)
        for b, e in enumerate(ends):
            if a == b:
                continue
            u = e[1] - e[0]
            t = np.clip(((m - e[0]) @ u) / (u @ u), 0.0, 1.0)
            d = np.minimum(d, np.linalg.norm(m - (e[0] + t[:, None] * u[None, :]), axis=1))
        dist.append(d)
    d = np.concatenate(dist)
    return [int(i) for i in np.argsort(d, kind="stable")[:k]], float(d.min())


def default_params(**over):
    """Parameter set; the values the paper leaves open (leaf size, window safety
    factors, self-window factor and modulation) are fixed here."""
    p = dict(mu=MU, cs=CS, beta=0.5,
             eta_H=2.0, aca_tol=1e-6, leaf=50, compress=1,
             eta_tmin=0.01, eta_tmax=0.01, int_tail=1,
             eta_w=1.5, q_w=0, mode_cap=0,
             factor_dtype="f64")
    p.update(over)
    return p


# ----------------------------------------------------------------------------
# Workload 1: two 12.8 km faults, 128 elements each, prescribed slip rate.
# ----------------------------------------------------------------------------
def two_fault_prescribed_faults(n_elem=128, dx=100.0, offset=1000.0, angle_deg=20.0):
    """Fault 1 on the x axis centred at the origin; fault 2 centred at
    (0, offset) and rotated by ``angle_deg`` about its centre."""
    L = n_elem * dx
    return [fault(0.0, 0.0, 0.0, L, n_elem),
            fault(0.0, offset, angle_deg, L, n_elem)]


def smoothed_loguniform_field(rng, n_steps, n_elem, sig_t=8.0, sig_x=4.0,
                              lo_exp=-9.0, hi_exp=0.0):
    """Gaussian-filtered white noise over (step, element), normalised to unit
    variance and mapped through the normal CDF so that the marginal of log10 V
    is uniform on [lo_exp, hi_exp]."""
    from scipy.ndimage import gaussian_filter
    from scipy.special import ndtr
    z = rng.standard_normal((n_steps, n_elem))
    z = gaussian_filter(z, sigma=(sig_t, sig_x), mode="reflect")
    z = (z - z.mean()) / z.std()
    return 10.0 ** (lo_exp + (hi_exp - lo_exp) * ndtr(z))


def prescribed_slip_rate(faults, n_steps, seed, lo_exp=-9.0, hi_exp=0.0):
    """Slip-rate history V[m, j] (m = 0..n_steps-1, j over all elements in fault
    order), each fault drawn independently from one seeded PCG64 stream."""
    rng = np.random.default_rng(seed)
    cols = [smoothed_loguniform_field(rng, n_steps, f["n_elem"], lo_exp=lo_exp,
                                      hi_exp=hi_exp) for f in faults]
    return np.ascontiguousarray(np.concatenate(cols, axis=1))


# ----------------------------------------------------------------------------
# The paper's two-fault benchmark (Section 3.1, Table 1): geometry, material,
# friction and initial conditions as printed (tests/golden/two_fault_benchmark.json).
# ----------------------------------------------------------------------------
def two_fault_benchmark(gold, n_elem=1000):
    """Faults, material and friction of the benchmark, each fault cut into
    ``n_elem`` elements (the paper uses 1000)."""
    faults = [dict(f, n_elem=int(n_elem)) for f in gold["faults"]]
    fr = gold["friction"]
    N = 2 * int(n_elem)
    fric = dict(a=np.full(N, fr["a"]), b=np.full(N, fr["a"] * fr["b_over_a"]), Dc=np.full(N, fr["Dc"]),
                sigma_n=np.full(N, fr["sigma_n"]), V0=np.full(N, fr["V_star"]), f0=np.full(N, fr["f_star"]))
    return faults, fric


def two_fault_benchmark_state(gold, faults, fric):
    """Steady sliding at V_* everywhere, tau0 = f_* sigma_n + mu V_* / (2 cs) (the
    printed 30 MPa), and on the first fault the overstress 2 tau_eq B(x') with
    w = 500 m, kappa = 2.5 about its centre."""
    fr = gold["friction"]
    N = len(fric["a"])
    V = np.full(N, fr["V_star"])
    theta = fric["Dc"] / V
    tau_eq = fr["f_star"] * fr["sigma_n"] + gold["mu"] / (2 * gold["cs"]) * fr["V_star"]
    tau0 = np.full(N, tau_eq)
    n = faults[0]["n_elem"]
    xi = (-0.5 + (np.arange(n) + 0.5) / n) * faults[0]["length"]
    w, kappa = 500.0, 2.5
    B = np.where(xi <= 0, 0.5 * (np.tanh(kappa * (xi / w + 1.0)) + 1.0),
                 0.5 * (1.0 - np.tanh(kappa * (xi / w - 1.0))))
    tau0[:n] += 2.0 * tau_eq * B
    return dict(V=V, theta=theta, tau0=tau0, tau0_rate=np.zeros(N))


def two_fault_benchmark_params(gold, n_elem=1000, **over):
    """Table 1's H-matrix and truncation parameters (eps_SVD -> ACA tolerance,
    q_w = 200 for 1000 elements, i.e. N_p / 5)."""
    p = default_params(mu=gold["mu"], cs=gold["cs"], beta=gold["beta"], eta_H=1.5, aca_tol=1e-6, leaf=50,
                       eta_tmin=gold["eta_tmin"], eta_tmax=gold["eta_tmax"], eta_w=1.5,
                       q_w=int(round(n_elem / 5)), state_update="exact")
    p.update(over)
    return p


# ----------------------------------------------------------------------------
# Workload 2/3: five 30 km faults, 600 elements each, full SEAS loop.
# ----------------------------------------------------------------------------
def random_network(seed, n_faults, n_elem, dx, box, strike_range, min_clear_frac=0.1,
                   max_tries=1000):
    """Seeded random straight faults: centres uniform in ``box`` = (W, H) metres,
    strikes uniform in ``strike_range`` degrees.  A draw is rejected (and the
    next one from the same stream taken) when a collocation point lies within
    ``min_clear_frac*dx`` of an element end point of another fault, where the
    kernels are unbounded."""
    rng = np.random.default_rng(seed)
    L = n_elem * dx
    for _ in range(max_tries):
        cx = rng.uniform(0.0, box[0], n_faults)
        cy = rng.uniform(0.0, box[1], n_faults)
        st = rng.uniform(strike_range[0], strike_range[1], n_faults)
        fl = [fault(cx[i], cy[i], st[i], L, n_elem) for i in range(n_faults)]
        if n_faults < 2 or _min_midpoint_node_distance(fl) > min_clear_frac * dx:
            return fl
    raise RuntimeError("no admissible fault layout found")


def five_fault_network(seed=0, n_elem=600, dx=50.0):
    """Five faults (600 x 50 m) in a 40 x 20 km box, strikes U(0, 40) degrees.
    Reduced meshes keep the same fault lengths and layout (dx scaled up)."""
    L = 600 * 50.0
    return random_network(seed, 5, n_elem, L / n_elem, (40e3, 20e3), (0.0, 40.0))


def rate_state_fields(faults, a=0.010, b_vw=0.015, b_vs=0.005, vw_frac=0.6,
                      Dc=5e-3, sigma_n=50e6, V0=1e-6, f0=0.6):
    """Aging-law parameters per element: b = b_vw on the central ``vw_frac`` of
    every fault, b_vs elsewhere."""
    out = {k: [] for k in ("a", "b", "Dc", "sigma_n", "V0", "f0")}
    for f in faults:
        n = f["n_elem"]
        s = (np.arange(n) + 0.5) / n - 0.5
        bb = np.where(np.abs(s) <= 0.5 * vw_frac, b_vw, b_vs)
        out["a"].append(np.full(n, a))
        out["b"].append(bb)
        out["Dc"].append(np.full(n, Dc))
        out["sigma_n"].append(np.full(n, sigma_n))
        out["V0"].append(np.full(n, V0))
        out["f0"].append(np.full(n, f0))
    return {k: np.concatenate(v) for k, v in out.items()}


def near_nucleation_state(faults, fric, seed=0, V_init=1e-9, mu=MU, cs=CS,
                          bump_width=500.0, kappa=2.5, bump_amp=2.0):
    """Initial slip rate, state and background stress.

    Steady state at ``V_init`` with theta = Dc/V_init and tau0 equal to the
    frictional strength plus the radiation term at that rate (the paper's
    initial-condition recipe, Section 3.1), plus a smooth tanh overstress of
    ``bump_amp`` times the equilibrium stress on one seeded fault, centred at a
    seeded point of its velocity-weakening patch."""
    rng = np.random.default_rng(10_000 + seed)
    N = sum(f["n_elem"] for f in faults)
    V = np.full(N, V_init)
    theta = fric["Dc"] / V_init
    tau_eq = fric["sigma_n"] * (fric["f0"] + (fric["a"] - fric["b"]) *
                                np.log(V_init / fric["V0"])) + mu / (2 * cs) * V_init
    tau0 = tau_eq.copy()
    which = int(rng.integers(len(faults)))
    off = 0
    for i, f in enumerate(faults):
        n = f["n_elem"]
        if i == which:
            xi = (-0.5 + (np.arange(n) + 0.5) / n) * f["length"]
            c = rng.uniform(-0.2, 0.2) * f["length"]
            x = xi - c
            B = np.where(x <= 0,
                         0.5 * (np.tanh(kappa * (x / bump_width + 1.0)) + 1.0),
                         0.5 * (1.0 - np.tanh(kappa * (x / bump_width - 1.0))))
            tau0[off:off + n] += bump_amp * tau_eq[off:off + n] * B
        off += n
    return dict(V=V, theta=theta, tau0=tau0, tau0_rate=np.zeros(N), delta=np.zeros(N))


def saturated_history(faults, n_hist, seed, lo_exp=-10.0, hi_exp=-6.0):
    """A seeded slip-rate history V[m, j] for the ``n_hist`` steps before t = 0
    (oldest first), used to start a run with full history windows."""
    return prescribed_slip_rate(faults, n_hist, 20_000 + seed, lo_exp, hi_exp)


# ----------------------------------------------------------------------------
# Workload 4: ensemble of friction variants on one geometry.
# ----------------------------------------------------------------------------
def ensemble_network(seed=0, n_elem=750, dx=50.0):
    L = 750 * 50.0
    scale = math.sqrt(6000 / 3000)
    return random_network(seed, 8, n_elem, L / n_elem, (40e3 * scale, 20e3 * scale), (0.0, 60.0))


def ensemble_variants(n_variants=64, seed=0, a=0.010):
    rng = np.random.default_rng(30_000 + seed)
    amb = rng.uniform(-0.006, -0.002, n_variants)
    Dc = 10.0 ** rng.uniform(math.log10(2e-3), math.log10(20e-3), n_variants)
    return dict(a=np.full(n_variants, a), b=a - amb, Dc=Dc)


# ----------------------------------------------------------------------------
# Workload 5: request stream for the serving loop.
# ----------------------------------------------------------------------------
def serving_templates(seed=0, n_templates=8, dx=50.0, sizes=(500, 1000, 2000, 4000, 8000)):
    rng = np.random.default_rng(40_000 + seed)
    out = []
    for t in range(n_templates):
        N = int(rng.choice(sizes))
        nf = int(rng.integers(2, 11))
        per = max(N // nf, 8)
        box = 40e3 * math.sqrt(N / 3000.0), 20e3 * math.sqrt(N / 3000.0)
        out.append(random_network(int(rng.integers(1 << 30)), nf, per, dx, box, (0.0, 180.0)))
    return out


def poisson_requests(n_requests=256, rate=4.0, seed=0, n_templates=8,
                     min_steps=2000, max_steps=20000):
    rng = np.random.default_rng(50_000 + seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    tpl = rng.integers(0, n_templates, n_requests)
    steps = rng.integers(min_steps, max_steps + 1, n_requests)
    seeds = rng.integers(0, 1 << 30, n_requests)
    return [dict(arrival=float(t[i]), template=int(tpl[i]), n_steps=int(steps[i]),
                 seed=int(seeds[i])) for i in range(n_requests)]


def flat(faults):
    """Faults as a (n_faults, 6) float array: cx, cy, nx, ny, length, n_elem."""
    return np.array([[f["cx"], f["cy"], f["nx"], f["ny"], f["length"], f["n_elem"]]
                     for f in faults], dtype=np.float64)
