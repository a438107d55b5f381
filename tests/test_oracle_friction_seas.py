"""Pins of the oracle's friction solve, block partition and step composition (CPU).

* the two-fault benchmark's printed equilibrium stress tau_eq = 30 MPa and
  L_b = 450 m (Section 3.1) from the Table 1 values;
* steady state and the unique Newton root against bisection;
* the aging law integrated by the predictor-corrector against its closed form;
* the block partition covers every receiver-source pair once, admissible blocks
  pass the admissibility test, eta_H = 20 gives an all-near-field partition
  (the paper's uncompressed reference, Appendix C), the closed-form bounding
  circle equals the printed definition;
* prescribed-mode stress is causal and equals the kernel for a rate impulse;
* with the elastic coupling switched off (mu -> 0) the SEAS step reduces to
  Heun's method for the state ODE, second order in dt.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import friction as FR, geometry, hpartition as HP, interaction as I, seas
import seas_inputs as SI

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_printed_equilibrium_stress_and_Lb():
    gd = json.load(open(os.path.join(GOLD, "two_fault_benchmark.json")))
    fr = gd["friction"]
    b = fr["a"] * fr["b_over_a"]
    V = fr["V_star"]
    theta = fr["Dc"] / V
    tau = FR.strength(V, theta, fr["a"], b, fr["Dc"], fr["sigma_n"], fr["V_star"], fr["f_star"])
    tau_eq = tau + gd["mu"] / (2 * gd["cs"]) * V
    assert abs(tau_eq - gd["printed_tau_eq"]) / gd["printed_tau_eq"] < 1e-6
    Lb = gd["mu"] * fr["Dc"] / (b * fr["sigma_n"])
    assert Lb == pytest.approx(gd["printed_Lb"], rel=1e-12)


def test_steady_state_friction():
    V = np.array([1e-12, 1e-9, 1e-3, 2.0])
    a, b, Dc, sn, V0, f0 = 0.01, 0.015, 5e-3, 50e6, 1e-6, 0.6
    tau = FR.strength(V, Dc / V, a, b, Dc, sn, V0, f0)
    assert np.allclose(tau, sn * (f0 + (a - b) * np.log(V / V0)), rtol=1e-14)
    assert np.allclose(FR.state_rate(V, Dc / V, Dc), 0.0, atol=1e-15)


def test_newton_root_matches_bisection():
    rng = np.random.default_rng(0)
    n = 64
    a = rng.uniform(0.005, 0.02, n)
    b = rng.uniform(0.003, 0.02, n)
    Dc, sn, V0, f0 = 5e-3, 50e6, 1e-6, 0.6
    eta = SI.MU / (2 * SI.CS)
    theta = 10 ** rng.uniform(-3, 8, n)
    A = sn * 0.6 + rng.uniform(-5e6, 5e6, n)
    V = FR.solve_velocity(A, theta, eta, a, b, Dc, sn, V0, f0, np.log(1e-9))

    def g(v):
        return A - eta * v - FR.strength(v, theta, a, b, Dc, sn, V0, f0)
    lo, hi = np.full(n, -80.0), np.full(n, 10.0)          # ln V bracket
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        pos = g(np.exp(mid)) > 0
        lo, hi = np.where(pos, mid, lo), np.where(pos, hi, mid)
    assert np.allclose(np.log(V), 0.5 * (lo + hi), rtol=0, atol=1e-12)


def test_newton_far_roots_and_the_rate_floor():
    # Roots far below the start (a stress deficit of hundreds of MPa, as at an
    # element next to a fault crossing after a rupture) are reached within the
    # iteration limit from either side; a root below ln V = -690 leaves V at the
    # floor exp(-690) (zero for every purpose) instead of underflowing to 0.
    eta = SI.MU / (2 * SI.CS)
    a, b, Dc, sn, V0, f0 = 0.01, 0.015, 5e-3, 50e6, 1e-6, 0.6
    theta = np.full(4, 1e3)
    c = sn * (f0 - a * np.log(V0) + b * np.log(V0 * theta / Dc))
    x_root = np.array([-600.0, -300.0, -120.0, 5.0])
    A = c + sn * a * x_root + eta * np.exp(x_root)       # the force balance holds at x_root
    for x0 in (np.log(1e-9), 2.0, -650.0):
        V = FR.solve_velocity(A, theta, eta, a, b, Dc, sn, V0, f0, np.full(4, x0))
        assert np.allclose(np.log(V), x_root, rtol=0, atol=1e-9), x0
    A_deep = c[:1] + sn * a * (-3400.0)
    V = FR.solve_velocity(A_deep, theta[:1], eta, a, b, Dc, sn, V0, f0, np.log(1e-9))
    assert V[0] == np.exp(FR.X_MIN) and V[0] > 0


def test_intermediate_law_limits():
    V, th, Dc = 1e-3, 3.0, 5e-3
    assert FR.state_rate(V, th, Dc, 1.0) == pytest.approx(1 - V * th / Dc)
    r = V * th / Dc
    assert FR.state_rate(V, th, Dc, 1e-7) == pytest.approx(-r * math.log(r), rel=1e-5)


# ------------------------------------------------------------------ partition
def _net(eta_H=2.0, leaf=16):
    faults = [SI.fault(0, 0, 10.0, 6400.0, 64), SI.fault(2000.0, 5000.0, 35.0, 4000.0, 40),
              SI.fault(-3000.0, 2000.0, 80.0, 3000.0, 30)]
    return geometry.discretize(faults), HP.partition(geometry.discretize(faults), eta_H, leaf)


def test_partition_covers_each_pair_once():
    geo, blocks = _net()
    for (a, b), bl in blocks.items():
        cover = np.zeros((geo[a].Np, geo[b].Np), int)
        for r0, r1, s0, s1, adm in bl:
            cover[r0:r1, s0:s1] += 1
        assert np.all(cover == 1)
    assert (0, 0) not in blocks


def test_partition_admissibility_and_leaves():
    geo, blocks = _net()
    trees = [HP.build_tree(f, 16) for f in geo]
    for (a, b), bl in blocks.items():
        for r0, r1, s0, s1, adm in bl:
            co, _ = HP.circle_literal(geo[a], r0, r1)[0], None
            c_o, r_o = HP.circle_literal(geo[a], r0, r1)
            c_s, r_s = HP.circle_literal(geo[b], s0, s1)
            d = math.hypot(*(c_o - c_s))
            if adm:
                assert d > 2.0 * (r_o + r_s) * (1 - 1e-12)
            else:
                assert r1 - r0 <= 16 and s1 - s0 <= 16


def test_circle_closed_form_equals_definition():
    geo, _ = _net()
    for f in geo:
        for lo, hi in ((0, f.Np), (3, 17), (f.Np // 2, f.Np)):
            c1, r1 = HP.circle_literal(f, lo, hi)
            c2, r2 = HP.circle_closed(f, lo, hi)
            assert np.allclose(c1, c2, rtol=0, atol=1e-9)
            assert r1 == pytest.approx(r2, rel=1e-12)


def test_large_eta_is_all_near_field():
    faults = SI.two_fault_prescribed_faults()
    geo = geometry.discretize(faults)
    blocks = HP.partition(geo, 20.0, 50)
    assert all(not adm for bl in blocks.values() for *_, adm in bl)


# ------------------------------------------------------------------ composition
def test_prescribed_impulse_response_is_the_kernel():
    faults = [SI.fault(0, 0, 0, 1200.0, 12), SI.fault(200.0, 700.0, 30.0, 1000.0, 10)]
    params = SI.default_params(int_tail=0)
    prob = seas.Problem(faults, params)
    n_steps = 40
    V = np.zeros((n_steps, prob.N))
    m0, j = 5, prob.off[1] + 3                     # impulse on fault 1, element 3
    V[m0, j] = 1.0
    f = seas.prescribed(prob, V)
    # f^n (row n-1) sees rates up to V^{n-1}: rows before the impulse are silent
    assert np.abs(f[:m0]).max() == 0.0
    T0, T1 = prob.inter.pairs[(0, 1)]["T0"], prob.inter.pairs[(0, 1)]["T1"]
    for n in range(m0 + 1, n_steps + 1):
        T = n - 1 - m0
        ref = -prob.eta * I.pair_kernel(prob.geo, 0, 1, T, prob.dt, prob.cs)[:, 3] if T0 <= T <= T1 else 0.0
        assert np.allclose(f[n - 1, :prob.off[1]], ref, rtol=1e-12, atol=1e-6)


def test_seas_step_reduces_to_heun_without_coupling():
    # mu -> 0 removes f and the radiation term: V follows from tau0 = strength(V, theta)
    # and theta obeys the aging law; the predictor-corrector is Heun's method.
    faults = [SI.fault(0, 0, 0, 400.0, 4)]
    # velocity strengthening (a > b): a smooth, stable state evolution
    fr = dict(a=np.full(4, 0.015), b=np.full(4, 0.011), Dc=np.full(4, 5e-3),
              sigma_n=np.full(4, 50e6), V0=np.full(4, 1e-6), f0=np.full(4, 0.6))
    tau0 = 50e6 * (0.6 + np.array([0.002, 0.004, 0.006, 0.008]))
    theta0 = np.array([1.0, 5.0, 20.0, 100.0])         # V ~ 3e-5 .. 6e-4 m/s
    T_end = 20.0

    def exact():
        def rhs(t, th):
            x = (tau0 / 50e6 - 0.6 - 0.011 * np.log(1e-6 * th / 5e-3)) / 0.015
            V = 1e-6 * np.exp(x)
            return 1 - V * th / 5e-3
        return solve_ivp(rhs, (0, T_end), theta0, rtol=1e-12, atol=1e-12, method="DOP853").y[:, -1]

    ref = exact()
    errs = []
    for mu_scale, nsteps in ((1e-12, 1000), (1e-12, 2000)):
        p = SI.default_params(mu=SI.MU * mu_scale, int_tail=0)
        prob = seas.Problem(faults, p)
        prob.dt = T_end / nsteps
        st = seas.SeasState(prob, fr, V0=np.full(4, 1e-9), theta0=theta0, tau0=tau0)
        # first V must satisfy the equilibrium: take it from the first solve
        st.V = FR.solve_velocity(tau0, theta0, prob.eta, fr["a"], fr["b"], fr["Dc"],
                                 fr["sigma_n"], fr["V0"], fr["f0"], np.log(1e-9))
        st.thetadot = FR.state_rate(st.V, st.theta, fr["Dc"])
        st.Vh[-1] = st.V.copy()
        for _ in range(nsteps):
            st.step()
        errs.append(np.abs(st.theta - ref).max() / np.abs(ref).max())
    assert errs[0] < 1e-4
    assert 3.0 < errs[0] / errs[1] < 5.0                # second order in dt


@pytest.mark.parametrize("eps", [1.0, 0.5, 0.2])
def test_state_at_constant_rate_solves_the_state_law(eps):
    # The closed form against the state law of eq. "state_evolution_law"
    # integrated numerically at constant slip rate (RK4, 20000 substeps), from
    # x = V dt / Dc = 1e-25 (a locked element) to 40 (seismic slip over a step),
    # and from states below and above steady state.
    Dc = 1e-2
    rate = lambda th, V: FR.state_rate(V, th, Dc, eps)
    for V, th0, dt in ((1e-25, 1e7, 1.4e-3), (1e-9, 1e7, 1.4e-3), (1e-3, 3.0, 1.4e-3), (14.0, 1e7, 1.4e-3),
                       (14.0, 1e-4, 0.03), (0.5, 2e-2, 0.8)):
        h = dt / 20000
        th = th0
        for _ in range(20000):
            k1 = rate(th, V)
            k2 = rate(th + 0.5 * h * k1, V)
            k3 = rate(th + 0.5 * h * k2, V)
            k4 = rate(th + h * k3, V)
            th = th + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        got = FR.state_at_constant_rate(th0, V, Dc, dt, eps)
        assert got > 0
        assert abs(got - th) <= 1e-9 * abs(th) + 1e-300, (V, th0, dt, got, th)


def test_state_at_constant_rate_is_second_order_close_to_explicit():
    # For small x the closed form and the explicit update theta + dt thetadot
    # differ by O(x^2) of the state.
    Dc, V, th0 = 1e-2, 1e-3, 7.0
    d = []
    for dt in (1e-2, 5e-3):
        exact = FR.state_at_constant_rate(th0, V, Dc, dt)
        expl = th0 + dt * FR.state_rate(V, th0, Dc)
        d.append(abs(exact - expl))
    assert 3.5 < d[0] / d[1] < 4.5


def _two_fault_gold():
    return json.load(open(os.path.join(os.path.dirname(__file__), "golden", "two_fault_benchmark.json")))


def test_two_fault_benchmark_inputs():
    # Section 3.1 / Table 1: L_b = mu Dc / (b sigma_n) = 450 m, tau_eq = 30 MPa,
    # the overstress peaks near 3 tau_eq at the centre of the first fault
    gd = _two_fault_gold()
    faults, fric = SI.two_fault_benchmark(gd, 1000)
    ini = SI.two_fault_benchmark_state(gd, faults, fric)
    Lb = gd["mu"] * fric["Dc"][0] / (fric["b"][0] * fric["sigma_n"][0])
    assert abs(Lb - gd["printed_Lb"]) < 1e-6 * gd["printed_Lb"]
    assert abs(ini["tau0"][1500] - gd["printed_tau_eq"]) / gd["printed_tau_eq"] < 1e-6
    # "approximately 3 tau_eq": 1 + 2 B(0) = 1 + tanh(2.5) + 1 = 2.987
    assert abs(ini["tau0"][:1000].max() / ini["tau0"][1500] - 3.0) < 0.02
    p = SI.two_fault_benchmark_params(gd, 1000)
    assert p["q_w"] == 200 and p["eta_H"] == 1.5 and p["aca_tol"] == 1e-6


def test_explicit_state_update_cannot_start_the_benchmark():
    # The explicit update as printed leaves theta <= 0 in the first step of the
    # two-fault benchmark (the rate jumps by ten decades); the closed-form update
    # at constant rate runs it (reading R19).
    gd = _two_fault_gold()
    n = 50
    faults, fric = SI.two_fault_benchmark(gd, n)
    ini = SI.two_fault_benchmark_state(gd, faults, fric)
    prob = seas.Problem(faults, SI.two_fault_benchmark_params(gd, n))
    o = seas.SeasState(prob, fric, ini["V"], ini["theta"], ini["tau0"], ini["tau0_rate"])
    with np.errstate(invalid="ignore", divide="ignore"):
        try:
            o.step()
            bad = not np.all(o.theta > 0)
        except FR.NotConverged:
            bad = True
    assert bad
    o = seas.SeasState(prob, fric, ini["V"], ini["theta"], ini["tau0"], ini["tau0_rate"], state_update="exact")
    for _ in range(10):
        o.step()
    assert np.all(o.theta > 0) and o.V.max() > 1.0


def test_two_fault_benchmark_partition():
    # Table 1's eta_H = 1.5 makes every block of both pairs admissible (one low-rank
    # block per leaf-level pairing, 26 in all). Appendix C calls eta_H = 20 the
    # uncompressed reference; with leaves of at most eta_leaf = 50 elements (the
    # text's rule) this geometry still has admissible blocks at eta_H = 20, so
    # the sweep's reference is the operator stored without compression (reading R20).
    gd = _two_fault_gold()
    faults, _ = SI.two_fault_benchmark(gd, 1000)
    geo = geometry.discretize(faults)
    b15 = [adm for bl in HP.partition(geo, 1.5, 50).values() for *_, adm in bl]
    assert len(b15) == 26 and all(b15)
    b20 = [adm for bl in HP.partition(geo, 20.0, 50).values() for *_, adm in bl]
    assert 0 < sum(b20) < len(b20)
