"""Pins of the oracle's adaptive time step (Section 2.4.1, step 1) (CPU).

* gamma = ceil(Delta t_ev / Delta t_min), Delta t_ev = min_i xi Dc_i / V_i, checked
  in exact rational arithmetic on the floating-point inputs, with its floor 1
  and cap gamma_max;
* a step of gamma = 1 is the fixed step, bit for bit, with coupling, loading and
  both state updates;
* with the elastic coupling switched off the adaptive step is Heun's method for
  the state ODE with the steps the rule chooses: it matches an accurate ODE
  solution, second order in the step length (xi halved: error / 4);
* a step of gamma grid steps advances time by gamma Delta t_min and slip by
  gamma Delta t_min times the averaged rate, and commits its interior grid rows as
  stated (the averaged rate; slip coefficients on the line to D**).

What the interior grid rows hold while a step evaluates its history sums is a
reading (the paper gives the grid, not the rows); its GPU form is compared with
this oracle, and its effect is first order in the step length.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import seas_inputs as SI
from oracle import friction as FR, seas


def _two_fault(n_elem=24):
    faults = SI.two_fault_prescribed_faults(n_elem=n_elem, dx=50.0)
    return faults, seas.Problem(faults, SI.default_params(compress=0))


def test_gamma_rule_exact():
    faults, prob = _two_fault(8)
    fric = SI.rate_state_fields(faults)
    N = prob.N
    rng = np.random.default_rng(3)
    for xi, gmax in ((0.5, 1 << 20), (0.1, 1 << 20), (0.5, 7), (1e-9, 100)):
        st = seas.SeasState(prob, fric, np.full(N, 1e-6), np.full(N, 1.0), np.zeros(N), adaptive=True, xi=xi,
                            gamma_max=gmax)
        for _ in range(20):
            st.V = 10 ** rng.uniform(-9, 0, N)
            # exact: ceil(min_i xi Dc_i / V_i / dt) of the floating-point values, then the clamps
            q = min(Fraction(xi) * Fraction(float(d)) / Fraction(float(v)) for d, v in zip(st.fric["Dc"], st.V))
            exact = math.ceil(q / Fraction(prob.dt))
            want = max(1, min(exact, gmax))
            got = st.gamma()
            # the rule evaluates in floating point: the exact ratio may sit on the other side
            # of an integer only when it is within rounding of it
            if got != want:
                assert abs(float(q / Fraction(prob.dt)) - round(float(q / Fraction(prob.dt)))) < 1e-9
            assert 1 <= got <= gmax
    fixed = seas.SeasState(prob, fric, np.full(N, 1e-12), np.full(N, 1.0), np.zeros(N))
    assert fixed.gamma() == 1


@pytest.mark.parametrize("update", ["explicit", "exact"])
def test_gamma_one_is_the_fixed_step(update):
    faults, prob = _two_fault()
    fric = SI.rate_state_fields(faults)
    ini = SI.near_nucleation_state(faults, fric, seed=2, V_init=1e-6, bump_amp=0.1)
    rate = 1e3 * np.linspace(0.5, 2.0, prob.N)
    a = seas.SeasState(prob, fric, ini["V"], ini["theta"], ini["tau0"], rate, state_update=update)
    b = seas.SeasState(prob, fric, ini["V"], ini["theta"], ini["tau0"], rate, state_update=update,
                       adaptive=True, xi=1e-12)
    for _ in range(40):
        a.step()
        b.step()
        assert b.last["gamma"] == 1
    for k in ("V", "theta", "delta", "thetadot"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    assert a.n == b.n == 40


def test_uncoupled_adaptive_is_variable_step_heun():
    # mu -> 0 removes the history functional and the radiation term; V follows from
    # tau0 = strength(V, theta) and theta obeys the aging law (velocity strengthening)
    faults = [SI.fault(0, 0, 0, 400.0, 4)]
    fr = dict(a=np.full(4, 0.015), b=np.full(4, 0.011), Dc=np.full(4, 5e-3),
              sigma_n=np.full(4, 50e6), V0=np.full(4, 1e-6), f0=np.full(4, 0.6))
    tau0 = 50e6 * (0.6 + np.array([0.002, 0.004, 0.006, 0.008]))
    theta0 = np.array([1.0, 5.0, 20.0, 100.0])

    def rhs(t, th):
        x = (tau0 / 50e6 - 0.6 - 0.011 * np.log(1e-6 * th / 5e-3)) / 0.015
        return 1 - 1e-6 * np.exp(x) * th / 5e-3

    sol = solve_ivp(rhs, (0, 30.0), theta0, rtol=1e-12, atol=1e-12, method="DOP853", dense_output=True)
    errs, steps = [], []
    for xi in (0.02, 0.01):
        p = SI.default_params(mu=SI.MU * 1e-12, int_tail=0)
        prob = seas.Problem(faults, p)
        prob.dt = 1e-3
        st = seas.SeasState(prob, fr, V0=np.full(4, 1e-9), theta0=theta0, tau0=tau0, adaptive=True, xi=xi)
        st.V = FR.solve_velocity(tau0, theta0, prob.eta, fr["a"], fr["b"], fr["Dc"], fr["sigma_n"], fr["V0"],
                                 fr["f0"], np.log(1e-9))
        st.thetadot = FR.state_rate(st.V, st.theta, fr["Dc"])
        st.Vh[-1] = st.V.copy()
        k = 0
        gammas = []
        while st.n * prob.dt < 20.0:
            g_rule = math.ceil(float(np.min(xi * fr["Dc"] / st.V)) / prob.dt)
            st.step()
            gammas.append(st.last["gamma"])
            assert st.last["gamma"] == max(1, g_rule)
            k += 1
        t = st.n * prob.dt                         # time is the sum of the steps' grid lengths
        assert st.n == sum(gammas)
        errs.append(np.abs(st.theta - sol.sol(t)).max() / np.abs(sol.sol(t)).max())
        steps.append(k)
        assert max(gammas) > 10                    # the steps grow as the slip rate falls
    assert errs[0] < 1e-4
    assert 3.0 < errs[0] / errs[1] < 5.5           # second order in the step length


def test_interior_rows_and_slip_of_a_long_step():
    faults, prob = _two_fault()
    fric = SI.rate_state_fields(faults)
    ini = SI.near_nucleation_state(faults, fric, seed=1, V_init=1e-6, bump_amp=0.05)
    st = seas.SeasState(prob, fric, ini["V"], ini["theta"], ini["tau0"], adaptive=True, gamma_max=5)
    st.step()                                      # a first step (gamma 5)
    n0, V0, d0 = st.n, st.V.copy(), st.delta.copy()
    D0 = [st.Dh[k][-1].copy() for k in range(2)]
    st.step()
    g = st.last["gamma"]
    assert g == 5 and st.n == n0 + 5
    Vbar = 0.5 * (V0 + st.last["V_star"])
    assert np.allclose(st.delta - d0, 5 * prob.dt * Vbar, rtol=1e-12, atol=0)
    for m in range(1, 5):
        assert np.array_equal(st.Vh[n0 + m - st.first], Vbar)
        for k in range(2):
            line = D0[k] + (m / 5) * (st.Dh[k][-1] - D0[k])
            assert np.allclose(st.Dh[k][n0 + m - st.first], line, rtol=1e-13, atol=1e-30)
    assert np.array_equal(st.Vh[n0 + 5 - st.first], st.V)
    assert np.array_equal(st.Vh[n0 - st.first], V0)   # the step's first row keeps its starting rate
