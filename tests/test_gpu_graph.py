"""Captured steps (seas_state_set_graph) against plain launches, bit for bit.

Two states of one operator start from the same state; one steps with plain
launches, the other with graph replays of whole time blocks. Both advance in
uneven chunks (eager steps up to a block start, several replays, a remainder),
with reads and synchronisations between the chunks, and every field must be
equal after every chunk: each replay is checked against the plain result. The
configurations cover the kernels a step records: the vector-ALU item kernels
(FP64, S = 1 and 8), the FP32 segment and near-field matrix-core kernels
(S = 16), the 16-bit segment kernel, an ensemble of BF16 variants with its FP32
list, the static tails of the pairs and of the self term, and a loading rate
(the stage reads the step's time). Switching the evaluation order recaptures.
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


TWO = SI.two_fault_prescribed_faults(n_elem=24, dx=50.0)
FIVE = SI.five_fault_network(seed=0, n_elem=48)
FIELDS = ("V", "theta", "delta", "f_self", "f_int", "f_hist")


def _init(faults, nv=1):
    fric = SI.rate_state_fields(faults)
    ini = SI.near_nucleation_state(faults, fric, seed=3, V_init=1e-6, bump_amp=0.1)
    N = len(ini["V"])
    rate = 2e3 * np.linspace(0.5, 1.5, N)
    if nv == 1:
        return fric, ini["V"], ini["theta"], ini["tau0"], rate
    rng = np.random.default_rng(9)
    t = lambda x: np.tile(x, nv)
    fr = {k: t(v) for k, v in fric.items()}
    fr["Dc"] = fr["Dc"] * np.repeat(10 ** rng.uniform(-0.2, 0.2, nv), N)
    return fr, t(ini["V"]), t(ini["theta"]), t(ini["tau0"]), t(rate)


CASES = [
    ("f64_S1", TWO, 1, dict(factor_dtype="f64", compress=0, time_block=1, self_tail=1)),
    ("f64_S8", TWO, 1, dict(factor_dtype="f64", compress=1, aca_tol=1e-12, time_block=8)),
    ("f32_S16_seg", FIVE, 1, dict(factor_dtype="f32", aca_tol=1e-8, leaf=8, time_block=16)),
    ("f16_S16", FIVE, 1, dict(factor_dtype="f16", aca_tol=1e-8, leaf=8, time_block=16)),
    ("f32_S32_seg", FIVE, 1, dict(factor_dtype="f32", aca_tol=1e-8, leaf=8, time_block=32)),
    ("bf16_ens16", TWO, 16, dict(factor_dtype="bf16", aca_tol=1e-8, leaf=8, time_block=1, n_variants=16)),
]
CHUNKS = [5, 37, 3, 50, 40, 1, 70]


@pytest.mark.parametrize("name,faults,nv,kw", CASES, ids=[c[0] for c in CASES])
def test_graph_replays_equal_plain_steps(name, faults, nv, kw):
    p = SI.default_params(state_update="exact", **kw)
    op = P.Operator(faults, p)
    if "seg" in name or name.startswith("f16"):
        assert op.info["n_segments"] > 0
    s = _stream()
    fr, V, th, tau0, rate = _init(faults, nv)
    plain = P.State(op, fr, V, th, tau0, rate, stream=s)
    graph = P.State(op, fr, V, th, tau0, rate, stream=s)
    graph.set_graph(True)
    print(f"[gpu] graph {name}: N={op.N} nv={nv} S={op.info['time_block']}", flush=True)
    for c in CHUNKS:
        plain.step(c, stream=s)
        graph.step(c, stream=s)
        assert graph.step_index == plain.step_index
        for k in FIELDS:
            a, b = plain.read(k, stream=s), graph.read(k, stream=s)
            assert np.array_equal(a, b), (name, c, k, float(np.abs(a - b).max()))
    plain.check(stream=s)
    graph.check(stream=s)
    info = graph.graph_info()
    unit = 16 if op.info["time_block"] == 1 else op.info["time_block"]
    assert info["steps_per_replay"] == unit and info["replays"] >= (4 if unit <= 16 else 2)
    print(f"[gpu] graph {name}: {info['replays']} replays of {unit} steps, all fields equal", flush=True)


def test_graph_recaptures_when_the_order_changes():
    p = SI.default_params(factor_dtype="f64", compress=1, aca_tol=1e-12, time_block=8, state_update="exact")
    op = P.Operator(TWO, p)
    s = _stream()
    fr, V, th, tau0, rate = _init(TWO)
    plain = P.State(op, fr, V, th, tau0, rate, stream=s)
    graph = P.State(op, fr, V, th, tau0, rate, stream=s)
    graph.set_graph(True)
    for S, n in ((1, 40), (8, 27), (1, 33)):
        for st in (plain, graph):
            st.set_time_block(S)
            st.step(n, stream=s)
        assert graph.graph_info()["steps_per_replay"] == (16 if S == 1 else 8)
        for k in FIELDS:
            assert np.array_equal(plain.read(k, stream=s), graph.read(k, stream=s)), (S, k)
    graph.set_graph(False)
    for st in (plain, graph):
        st.step(20, stream=s)
    for k in FIELDS:
        assert np.array_equal(plain.read(k, stream=s), graph.read(k, stream=s)), k


def test_graph_is_refused_for_adaptive_steps():
    op = P.Operator(TWO, SI.default_params(time_block=1, adaptive_dt=1))
    fr, V, th, tau0, rate = _init(TWO)
    st = P.State(op, fr, V, th, tau0, rate, stream=_stream())
    with pytest.raises(P.SeasError):
        st.set_graph(True)
