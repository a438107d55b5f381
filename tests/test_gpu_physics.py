"""GPU parity of the physics variants of the step (through the C ABI, against the FP64 oracle).

* The intermediate state law of Section 2.2 (eq. "state_evolution_law") with an
  exponent eps < 1, varying per element (eps = 1 is the aging law), with the
  explicit state update and with the closed-form update at constant rate.
* Tectonic loading: a background stress that grows at a constant rate per
  element (Section 3.2 loads the faults this way).

Both run the full predictor-corrector of Section 2.4 over 120 steps of a
two-fault network and compare slip, rate, state and the stress parts with the
oracle at the FP64 tolerance.
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


def _run(p, fric, ini, eps, n_steps, state_update="explicit"):
    op = P.Operator(FAULTS, p)
    s = _stream()
    fr = dict(fric)
    fr["eps"] = eps
    st = P.State(op, fr, ini["V"], ini["theta"], ini["tau0"], ini["tau0_rate"], stream=s)
    st.step(n_steps, stream=s)
    st.check(stream=s)
    g = {k: st.read(k, stream=s) for k in ("V", "theta", "delta", "thetadot", "f_self", "f_int")}
    prob = OS.Problem(FAULTS, p)
    o = OS.SeasState(prob, fric, ini["V"], ini["theta"], ini["tau0"], ini["tau0_rate"], eps=eps,
                     state_update=state_update)
    for _ in range(n_steps):
        o.step()
    return g, o


@pytest.mark.parametrize("S,update", [(1, "explicit"), (8, "explicit"), (8, "exact")])
def test_intermediate_state_law(S, update):
    p = SI.default_params(compress=0, time_block=S, state_update=update)
    fric = SI.rate_state_fields(FAULTS)
    ini = SI.near_nucleation_state(FAULTS, fric, seed=2, V_init=1e-6, bump_amp=0.1)
    N = len(ini["V"])
    eps = np.where(np.arange(N) % 3 == 0, 1.0, np.where(np.arange(N) % 3 == 1, 0.5, 0.2))
    # off steady state, so that the state law's exponent matters
    ini = dict(ini)
    ini["theta"] = ini["theta"] * np.linspace(0.5, 2.0, N)
    g, o = _run(p, fric, ini, eps, 120, update)
    errs = {k: rel_err(g[k], ref) for k, ref in (("V", o.V), ("theta", o.theta), ("delta", o.delta),
                                               ("thetadot", o.thetadot), ("f_self", o.last["f_self"]),
                                               ("f_int", o.last["f_int"]))}
    print(f"[gpu] intermediate law S={S} {update}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()),
          flush=True)
    for k, e in errs.items():
        assert e < 1e-9, k
    # the exponent changed the trajectory (not an aging-law run in disguise)
    ga, _ = _run(p, fric, ini, np.ones(N), 120, update)
    assert rel_err(ga["theta"], g["theta"]) > 1e-4


@pytest.mark.parametrize("S", [1, 8])
def test_tectonic_loading_rate(S):
    p = SI.default_params(compress=1, aca_tol=1e-12, time_block=S)
    fric = SI.rate_state_fields(FAULTS)
    ini = SI.near_nucleation_state(FAULTS, fric, seed=3, V_init=1e-6, bump_amp=0.05)
    N = len(ini["V"])
    dt = P.Operator(FAULTS, p).info["dt"]
    ini = dict(ini)
    # half a percent of the background stress per 120 steps, more on the second fault
    ini["tau0_rate"] = 0.005 * ini["tau0"] / (120 * dt) * np.where(np.arange(N) < N // 2, 1.0, 2.0)
    g, o = _run(p, fric, ini, np.ones(N), 120)
    errs = {k: rel_err(g[k], ref) for k, ref in (("V", o.V), ("theta", o.theta), ("delta", o.delta),
                                               ("f_int", o.last["f_int"]))}
    print(f"[gpu] loading rate S={S}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    for k, e in errs.items():
        assert e < 1e-9, k
    g0, _ = _run(p, fric, dict(ini, tau0_rate=np.zeros(N)), np.ones(N), 120)
    assert rel_err(g0["V"], g["V"]) > 1e-3      # the loading is visible in the slip rate
