"""Tile tuning of the far pass (seas_operator_tune / seas_operator_set_tune).

The three compiled variants of the segment kernel (FP32 one variant; BF16 / FP16
one variant and ensembles) differ only in prefetch depth and register budget, so
stepping with each must give the same fields bit for bit; the tuner times every
variant on the state's history, keeps the fastest, and leaves the state's fields
as they were. Operators without variants report none.
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


TWO = SI.two_fault_prescribed_faults(n_elem=24, dx=50.0)


def _state(op, faults=FIVE, nv=1):
    fric = SI.rate_state_fields(faults)
    ini = SI.near_nucleation_state(faults, fric, seed=5, V_init=1e-6, bump_amp=0.1)
    if nv > 1:
        rng = np.random.default_rng(2)
        t = lambda x: np.tile(x, nv)
        fr = {k: t(v) for k, v in fric.items()}
        fr["Dc"] = fr["Dc"] * np.repeat(10 ** rng.uniform(-0.2, 0.2, nv), len(ini["V"]))
        return P.State(op, fr, t(ini["V"]), t(ini["theta"]), t(ini["tau0"]), stream=_stream())
    return P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], stream=_stream())


CASES = [
    ("f32_S16", FIVE, 1, dict(factor_dtype="f32", time_block=16)),
    ("f32_S32", FIVE, 1, dict(factor_dtype="f32", time_block=32)),
    ("f16_S16", FIVE, 1, dict(factor_dtype="f16", time_block=16)),
    ("bf16_ens16", TWO, 16, dict(factor_dtype="bf16", time_block=1, n_variants=16)),
]


@pytest.mark.parametrize("name,faults,nv,kw", CASES, ids=[c[0] for c in CASES])
def test_variants_step_identically_and_tuning_keeps_the_state(name, faults, nv, kw):
    op = P.Operator(faults, SI.default_params(aca_tol=1e-8, leaf=8, state_update="exact", **kw))
    assert op.info["n_segments"] > 0
    S = op.info["time_block"]
    s = _stream()
    st = _state(op, faults, nv)
    st.step(S + 3, stream=s)
    snap = st.save(stream=s)
    before = {k: st.read(k, stream=s) for k in FIELDS}
    r = op.tune(st, stream=s, reps=2)
    print(f"[gpu] tune {name}: {r}", flush=True)
    assert r["choice"] in (0, 1, 2) and all(m > 0 for m in r["ms"])
    assert r["ms"][r["choice"]] == min(r["ms"])
    for k in FIELDS:
        assert np.array_equal(before[k], st.read(k, stream=s)), k
    out = []
    for v in (0, 1, 2):
        op.set_tune(v)
        st.restore(snap, stream=s)
        st.step(3 * max(S, 16) + 5, stream=s)
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
