"""GPU parity of adaptive time steps (Section 2.4.1, step 1) through the C ABI.

Each step is gamma Delta t_min with gamma = ceil(min_i xi Dc_i / V_i / Delta t_min)
(at least 1, at most gamma_max) and the histories stay on the Delta t_min grid
(interior grid rows as the oracle's SeasState.step states). Compared with the
FP64 oracle on a two-fault network through a nucleation, where gamma falls from
tens to 1: the gamma of every step, and slip, rate and state at the end (FP64
factors at 1e-9; FP32 factors at 1e-5; cluster-level windows at 1e-9). gamma_max
above the largest window (every lag of a step's history sum inside the step)
and below it; a rule that always gives gamma = 1 reproduces fixed steps bit for
bit.
"""
import numpy as np
import pytest

import seas_inputs as SI
from oracle import seas as OS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2603_00383_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.init()
    yield


def _stream():
    return torch.cuda.current_stream().cuda_stream


def rel_err(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


FAULTS = SI.two_fault_prescribed_faults(n_elem=24, dx=50.0)


def _setup(V_init=5e-5, bump=0.005, load=1e6):
    # seeded near-nucleation state: with xi = 0.01 the first step is longer than the
    # largest window, the next ones shorten as the rate grows, then gamma = 1
    fric = SI.rate_state_fields(FAULTS)
    ini = SI.near_nucleation_state(FAULTS, fric, seed=6, V_init=V_init, bump_amp=bump)
    N = len(ini["V"])
    rate = load * np.where(np.arange(N) < N // 2, 1.0, 1.5)
    return fric, ini, rate


SLOW = dict(V_init=3e-5, bump=0.01, load=1e5)     # gamma from ~230 down to ~4 over 70 steps
CASES = [
    ("f64", 0, 300, 1e-9, {}, dict(factor_dtype="f64", compress=0)),
    ("f64_gmax12", 0, 12, 1e-9, {}, dict(factor_dtype="f64", compress=1, aca_tol=1e-12)),
    ("f32_slow", 0, 300, 1e-5, SLOW, dict(factor_dtype="f32", compress=0)),
    ("f64_cluster", 1, 300, 1e-9, {}, dict(factor_dtype="f64", compress=1, aca_tol=1e-12, leaf=8)),
]


@pytest.mark.parametrize("name,cluster,gmax,tol,init,kw", CASES, ids=[c[0] for c in CASES])
def test_adaptive_steps_match_the_oracle(name, cluster, gmax, tol, init, kw):
    xi = 0.01
    p = SI.default_params(time_block=1, state_update="exact", adaptive_dt=1, adapt_xi=xi, gamma_max=gmax,
                          cluster_windows=cluster, **kw)
    op = P.Operator(FAULTS, p)
    assert op.info["max_lag"] < 300
    fric, ini, rate = _setup(**init)
    s = _stream()
    st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], rate, stream=s)
    prob = OS.Problem(FAULTS, p)
    o = OS.SeasState(prob, fric, ini["V"], ini["theta"], ini["tau0"], rate, state_update="exact",
                     adaptive=True, xi=xi, gamma_max=gmax)
    gammas = []
    for k in range(70):
        st.step(1, stream=s)
        o.step()
        g = st.progress()["last_gamma"]
        gammas.append(o.last["gamma"])
        assert g == o.last["gamma"], (k, g, o.last["gamma"])
    st.check(stream=s)
    assert st.step_index == o.n
    pr = st.progress()
    assert pr["steps_taken"] == 70 and pr["time_s"] == pytest.approx(o.n * prob.dt, rel=1e-15)
    print(f"[gpu] adaptive {name}: gammas {gammas[:6]} .. {gammas[-6:]}, grid index {o.n}", flush=True)
    assert max(gammas) > 1 and min(gammas) >= 1 and len(set(gammas)) > 3
    if gmax > op.info["max_lag"]:
        assert max(gammas) > op.info["max_lag"] + 2      # whole windows inside one step
    else:
        assert gmax in gammas and min(gammas) < gmax
    for k, ref in (("V", o.V), ("theta", o.theta), ("delta", o.delta)):
        e = rel_err(st.read(k, stream=s), ref)
        print(f"[gpu] adaptive {name} {k}: {e:.2e}", flush=True)
        assert e < tol, k


def test_adaptive_with_unit_gamma_is_the_fixed_step():
    fric, ini, rate = _setup()
    s = _stream()
    out = []
    for adaptive in (0, 1):
        p = SI.default_params(time_block=1, factor_dtype="f64", compress=0, state_update="exact",
                              adaptive_dt=adaptive, adapt_xi=1e-12)
        op = P.Operator(FAULTS, p)
        st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], rate, stream=s)
        st.step(50, stream=s)
        st.check(stream=s)
        out.append({k: st.read(k, stream=s) for k in ("V", "theta", "delta", "f_int")})
        assert st.step_index == 50
        if adaptive:
            assert st.progress()["last_gamma"] == 1
    for k in out[0]:
        assert np.array_equal(out[0][k], out[1][k]), k


def test_adaptive_needs_unblocked_steps():
    with pytest.raises(P.SeasError):
        P.Operator(FAULTS, SI.default_params(time_block=8, adaptive_dt=1))


def test_state_gamma_cap():
    # a per-state cap below the operator's: the steps of an oracle whose cap is the same
    fric, ini, rate = _setup()
    s = _stream()
    p = SI.default_params(time_block=1, factor_dtype="f64", compress=0, state_update="exact", adaptive_dt=1,
                          adapt_xi=0.01, gamma_max=300)
    op = P.Operator(FAULTS, p)
    st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], rate, stream=s)
    o = OS.SeasState(OS.Problem(FAULTS, p), fric, ini["V"], ini["theta"], ini["tau0"], rate, state_update="exact",
                     adaptive=True, xi=0.01, gamma_max=1)
    st.set_gamma_cap(1)
    st.step(3, stream=s)
    for _ in range(3):
        o.step()
    assert st.step_index == o.n == 3
    st.set_gamma_cap(20)
    o.gamma_max = 20
    for _ in range(10):
        st.step(1, stream=s)
        o.step()
        assert st.progress()["last_gamma"] == o.last["gamma"] <= 20
    st.check(stream=s)
    assert rel_err(st.read("V", stream=s), o.V) < 1e-9
