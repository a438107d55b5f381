"""Full predictor-corrector step at the five-fault benchmark's size against the oracle.

The oracle cannot step the 3000-element network (its dense stacks do not fit),
so ``tests/golden/make_step_replay.py`` evaluated one step (Section 2.4, steps 2
and 3) of every element of one fault (the one holding the receiver nearest a
fault crossing) from two seeded saturated states, row by row, with
``oracle.seas.step_fault``; the values are in
``tests/golden/step_replay_five_fault.json``. Here the library takes the same
seeded state (prior slip-rate history as long as the longest window, steady
sliding at 1e-9 or 1e-4 m/s with the tanh overstress) through its C ABI, takes
one step, and V, theta, delta and the interaction history part of that fault are
compared. Operators: the benchmark's (ACA 1e-6, eta_H 2, leaf 50, time block 16)
with FP32 and FP64 factors; the bound is the 1e-4 reduced-precision target for
both (the ACA tolerance, not the arithmetic, sets the FP64 error here); the
errors are printed.
"""
import json
import os

import numpy as np
import pytest

import seas_inputs as SI

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2603_00383_amd")

GOLD = os.path.join(os.path.dirname(__file__), "golden", "step_replay_five_fault.json")


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as fh:
        return json.load(fh)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_step_replay_five_fault(dtype, gold, loud):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    faults = SI.five_fault_network(seed=gold["network_seed"])
    params = SI.default_params(factor_dtype=dtype, aca_tol=1e-6, eta_H=2.0, leaf=50, time_block=16)
    with loud(f"[gpu] building the five-fault operator ({dtype}) for the step replay"):
        op = P.Operator(faults, params)
    assert op.info["max_lag"] + 2 == gold["prior_steps"]
    prior = SI.saturated_history(faults, gold["prior_steps"], gold["prior_seed"])
    fric = SI.rate_state_fields(faults)
    rows = np.array(gold["rows"])
    nk = 600
    fault_rows = rows[:nk]
    s = torch.cuda.current_stream().cuda_stream
    for name, case in gold["cases"].items():
        ini = SI.near_nucleation_state(faults, fric, seed=case["seed"], V_init=case["V_init"],
                                       bump_amp=case["bump_amp"])
        st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], ini["tau0_rate"], stream=s)
        st.load_history(prior, stream=s)
        st.step(1, stream=s)
        st.check(stream=s)
        fh = st.read("f_hist", stream=s)[rows]
        e_f = float(np.abs(fh - np.array(gold["f_hist"])).max() / np.abs(gold["f_hist"]).max())
        errs = {"f_hist": e_f}
        for k in ("V", "theta", "delta"):
            ref = np.array(case[k])
            got = st.read(k, stream=s)[fault_rows]
            errs[k] = float(np.abs(got - ref).max() / np.abs(ref).max())
        print(f"[gpu] step replay {dtype} {name} (fault {gold['fault']}): "
              + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
        for k, v in errs.items():
            assert v < 1e-4, (name, k, v)
        st.close()
