"""GPU tests of the block lookahead of seas_step (time-blocked builds), through the C ABI.

The stress at the S steps of a time block from lags >= 2S needs rates up to the
step before the previous block only (the history sum of Section 2.4, eq.
"fault-to-fault_interactions_discretized"), so that part of the far list runs for
the next block on a second stream while the current block steps. The same
kernels write the same partial sums either way, so a trajectory with the
lookahead must equal the one without it bit for bit, however the steps are split
over calls; and both must match the FP64 oracle.

Covered: the FP32 segment kernel (S = 16), a 16-bit build whose near-field far
lags run on the FP32 item kernel (list 2, S = 16), and the FP64 item kernel
(S = 16).
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


def _faults():
    # two 2 km faults: windows from lag 0 to beyond 2S, so both far parts are populated
    return SI.two_fault_prescribed_faults(n_elem=40, dx=50.0)


CASES = [
    ("f32", 16, dict(factor_dtype="f32", aca_tol=1e-8, time_block=16)),
    ("f32_S32", 32, dict(factor_dtype="f32", aca_tol=1e-8, time_block=32)),
    ("f16", 16, dict(factor_dtype="f16", aca_tol=1e-8, time_block=16, leaf=10)),  # both 16-bit and FP32 far lists
    ("f64", 16, dict(factor_dtype="f64", aca_tol=1e-12, time_block=16)),
]


@pytest.mark.parametrize("name,S,kw", CASES, ids=[c[0] for c in CASES])
def test_lookahead_is_bitwise_neutral(name, S, kw):
    faults = _faults()
    p = SI.default_params(**kw)
    op = P.Operator(faults, p)
    inf = op.info
    assert inf["far_entries_first"] > 0
    assert inf["far_entries"] - inf["far_entries_first"] > 0
    if name == "f16":
        assert inf["far_entries_f32"] > 0 and inf["far_entries_first_f32"] > 0
        assert inf["far_entries"] > inf["far_entries_f32"]
    fric = SI.rate_state_fields(faults)
    ini = SI.near_nucleation_state(faults, fric, seed=4, V_init=1e-6, bump_amp=0.1)
    s = _stream()
    n_steps = 7 * S + 5
    runs = {}
    for mode, chunks in (("off", [n_steps]), ("on", [n_steps]), ("on_split", [3, 2 * S + 1, S, n_steps - 3 * S - 4])):
        st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], stream=s)
        st.set_overlap(mode != "off")
        st.set_timing(True)
        st.read_timing(stream=s)
        launches = 0
        for c in chunks:
            st.step(c, stream=s)
            launches += st.read_timing(stream=s)[1]
        st.check(stream=s)
        runs[mode] = {k: st.read(k, stream=s) for k in ("V", "theta", "delta", "f_int", "f_hist")}
        # one timed far launch (the lags >= 2S) per block start, whichever stream ran it
        print(f"[gpu] lookahead {name} {mode}: {launches} timed far launches over {n_steps} steps", flush=True)
        assert launches == -(-n_steps // S)
        st.close()
    for mode in ("on", "on_split"):
        for k in runs["off"]:
            assert np.array_equal(runs[mode][k], runs["off"][k]), (mode, k)
    # and the trajectory is the method's (FP64 oracle, same windows and tail)
    if name == "f64":
        prob = OS.Problem(faults, p)
        o = OS.SeasState(prob, fric, ini["V"], ini["theta"], ini["tau0"])
        for _ in range(n_steps):
            o.step()
        for k, ref in (("V", o.V), ("theta", o.theta), ("delta", o.delta)):
            e = rel_err(runs["on"][k], ref)
            print(f"[gpu] lookahead f64 vs oracle {k}: {e:.2e}", flush=True)
            assert e < 1e-9, k
