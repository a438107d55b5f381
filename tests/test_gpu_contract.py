"""GPU tests of the boundary's state contract (Section 2.4 unknowns), through the C ABI.

* A Newton failure leaves the failing variant at its last good step: its slip,
  rate and state read back unchanged, and its histories (rate ring, slip
  coefficients, expired-slip accumulators, the far part of the current time
  block) are intact, so restoring the one value that made it fail and stepping
  on reproduces a run that never failed.
* In an ensemble, a failed variant is held while the others step on exactly as
  they would without it.
* seas_write_state overwrites V, theta and delta at the current step with the
  same meaning as the oracle's state (V also the newest rate row, delta also the
  newest slip-coefficient row, the state rate recomputed).

The failure is forced from the host by a background stress that is not finite:
the solve meets a non-finite force balance, which fails it (every kernel still
runs to completion).
"""
import numpy as np
import pytest

import seas_inputs as SI
from oracle import friction as OF, seas as OS

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


def _setup(seed=0):
    fric = SI.rate_state_fields(FAULTS)
    ini = SI.near_nucleation_state(FAULTS, fric, seed=seed, V_init=1e-6, bump_amp=0.1)
    return fric, ini


@pytest.mark.parametrize("S", [1, 8])
def test_newton_failure_holds_last_good_step(S):
    p = SI.default_params(compress=1, aca_tol=1e-10, time_block=S)
    fric, ini = _setup()
    op = P.Operator(FAULTS, p)
    s = _stream()
    ref = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], stream=s)
    ref.step(53, stream=s)
    ref.check(stream=s)
    want = {k: ref.read(k, stream=s) for k in ("V", "theta", "delta")}

    st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], stream=s)
    st.step(33, stream=s)
    st.check(stream=s)
    good = {k: st.read(k, stream=s) for k in ("V", "theta", "delta", "thetadot", "tau0")}
    bad = good["tau0"].copy()
    bad[5] = np.nan
    st.write("tau0", bad, stream=s)
    print(f"[gpu] forced Newton failure S={S}", flush=True)
    st.step(7, stream=s)                       # fails at step 34; 35..40 leave it alone
    with pytest.raises(P.SeasError) as e:
        st.check(stream=s)
    assert e.value.code == -4
    assert st.step_index == 33
    failed, at = st.variant_status(stream=s)
    assert not failed[0] and at[0] == 33       # flag cleared by the check, held at 33
    for k in ("V", "theta", "delta", "thetadot"):
        assert np.array_equal(st.read(k, stream=s), good[k]), k
    # put back the stress that made it fail: the run continues as if nothing happened
    st.write("tau0", good["tau0"], stream=s)
    st.step(20, stream=s)
    st.check(stream=s)
    assert st.step_index == 53
    for k in ("V", "theta", "delta"):
        e = rel_err(st.read(k, stream=s), want[k])
        print(f"[gpu] resumed after failure S={S} {k}: {e:.2e}", flush=True)
        assert e < 1e-13


def test_failed_variant_is_held_and_the_others_step_on():
    nv = 16
    # leaf 8: admissible blocks, so the 16-bit segment kernel runs beside the FP32 list
    p = SI.default_params(factor_dtype="bf16", aca_tol=1e-6, time_block=1, n_variants=nv, leaf=8)
    op = P.Operator(FAULTS, p)
    assert op.info["far_entries"] > op.info["far_entries_f32"]
    N = op.N
    s = _stream()
    fric, ini = _setup()
    tile = lambda x: np.tile(x, nv)
    fr = {k: tile(v) for k, v in fric.items()}
    V = tile(ini["V"])
    t0 = tile(ini["tau0"])
    t0_bad = t0.copy()
    t0_bad[3 * N + 7] = np.nan
    runs = []
    for tau0 in (t0, t0_bad):
        st = P.State(op, fr, V, tile(ini["theta"]), tau0, stream=s)
        st.step(40, stream=s)
        runs.append(st)
    runs[0].check(stream=s)
    with pytest.raises(P.SeasError):
        runs[1].check(stream=s)
    failed, at = runs[1].variant_status(stream=s)
    assert failed.tolist() == [v == 3 for v in range(nv)]
    assert at[3] == 0 and all(at[v] == 40 for v in range(nv) if v != 3)
    assert np.array_equal(runs[1].read("V", stream=s, variant=3), V[3 * N:4 * N])
    assert np.array_equal(runs[1].read("delta", stream=s, variant=3), np.zeros(N))
    for v in (0, 2, 4, 15):
        for k in ("V", "theta", "delta"):
            assert np.array_equal(runs[1].read(k, stream=s, variant=v), runs[0].read(k, stream=s, variant=v))
    # a new window in the failed slot clears it
    runs[1].reset_variant(3, fric, ini["V"], ini["theta"], ini["tau0"], stream=s)
    runs[1].step(5, stream=s)
    runs[1].check(stream=s)
    failed, at = runs[1].variant_status(stream=s)
    assert not failed.any() and at[3] == 45


@pytest.mark.parametrize("S", [1, 8])
def test_write_state_matches_the_oracle(S):
    p = SI.default_params(compress=0, time_block=S)
    fric, ini = _setup(1)
    op = P.Operator(FAULTS, p)
    s = _stream()
    st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], stream=s)
    prob = OS.Problem(FAULTS, p)
    o = OS.SeasState(prob, fric, ini["V"], ini["theta"], ini["tau0"])
    n0, n1 = 25, 15
    st.step(n0, stream=s)
    st.check(stream=s)
    for _ in range(n0):
        o.step()
    # new values, written on both sides from each side's own state
    g = {k: st.read(k, stream=s) for k in ("V", "theta", "delta")}
    st.write("V", 1.5 * g["V"], stream=s)
    st.write("theta", 0.8 * g["theta"], stream=s)
    st.write("delta", g["delta"] + 1e-4, stream=s)
    o.V, o.theta, o.delta = 1.5 * o.V, 0.8 * o.theta, o.delta + 1e-4
    o.thetadot = OF.state_rate(o.V, o.theta, o.fric["Dc"])
    o.Vh[-1] = o.V.copy()
    D = prob.dfts(o.delta)
    for k in range(len(prob.geo)):
        o.Dh[k][-1] = D[k]
    st.step(n1, stream=s)
    st.check(stream=s)
    for _ in range(n1):
        o.step()
    for k, ref in (("V", o.V), ("theta", o.theta), ("delta", o.delta)):
        e = rel_err(st.read(k, stream=s), ref)
        print(f"[gpu] write_state S={S} {k}: {e:.2e}", flush=True)
        assert e < 1e-9


def test_write_state_rejects_bad_input():
    op = P.Operator(FAULTS, SI.default_params())
    fric, ini = _setup()
    s = _stream()
    st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], stream=s)
    with pytest.raises(P.SeasError):
        st.write("V", -ini["V"], stream=s)
    with pytest.raises(P.SeasError):
        st.write("f_hist", ini["V"], stream=s)
    with pytest.raises(P.SeasError):
        st.write("theta", ini["theta"][:-1], stream=s)
