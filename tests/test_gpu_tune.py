"""Tile tuning of the FP32 far pass (seas_operator_tune / seas_operator_set_tune).

The three compiled variants of the FP32 one-variant segment kernel differ only in
prefetch depth and register budget, so stepping with each must give the same
fields bit for bit; the tuner times every variant on the state's history, keeps
the fastest, and leaves the state's fields as they were. Operators without
variants report none.
"""
import numpy as np
import pytest

import seas_inputs as SI

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


FIVE = SI.five_fault_network(seed=0, n_elem=48)
FIELDS = ("V", "theta", "delta", "f_hist", "f_int", "f_self")


def _state(op):
    fric = SI.rate_state_fields(FIVE)
    ini = SI.near_nucleation_state(FIVE, fric, seed=5, V_init=1e-6, bump_amp=0.1)
    return P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], stream=_stream())


@pytest.mark.parametrize("S", [16, 32])
def test_variants_step_identically_and_tuning_keeps_the_state(S):
    op = P.Operator(FIVE, SI.default_params(factor_dtype="f32", aca_tol=1e-8, leaf=8, time_block=S,
                                            state_update="exact"))
    assert op.info["n_segments"] > 0
    s = _stream()
    st = _state(op)
    st.step(S + 3, stream=s)
    snap = st.save(stream=s)
    before = {k: st.read(k, stream=s) for k in FIELDS}
    r = op.tune(st, stream=s, reps=2)
    print(f"[gpu] tune S={S}: {r}", flush=True)
    assert r["choice"] in (0, 1, 2) and all(m > 0 for m in r["ms"])
    assert r["ms"][r["choice"]] == min(r["ms"])
    for k in FIELDS:
        assert np.array_equal(before[k], st.read(k, stream=s)), k
    out = []
    for v in (0, 1, 2):
        op.set_tune(v)
        st.restore(snap, stream=s)
        st.step(3 * S + 5, stream=s)
        st.check(stream=s)
        out.append({k: st.read(k, stream=s) for k in FIELDS})
    for v in (1, 2):
        for k in FIELDS:
            assert np.array_equal(out[0][k], out[v][k]), (v, k)


def test_operators_without_variants():
    op = P.Operator(FIVE, SI.default_params(factor_dtype="f64", aca_tol=1e-8, leaf=8, time_block=8))
    st = _state(op)
    r = op.tune(st, stream=_stream())
    assert r == {"ms": [-1.0, -1.0, -1.0], "choice": 0}
    with pytest.raises(P.SeasError):
        op.set_tune(3)
