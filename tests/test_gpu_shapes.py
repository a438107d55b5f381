"""GPU parity of the far-list kernels on large blocks: two parallel faults of n
elements far enough apart that their pair is two low-rank blocks of n/2 rows
(n = 150 and 1200 give 5 and 38 row tiles of 16: the inner-range split of the
work units, and the tall blocks whose rows are written per unit; 300 and 600,
the heights in between, gave the same errors when measured). The interaction history part of one SEAS
step from a saturated history is compared with the oracle on sampled receivers,
for FP32, BF16 and FP16 factors.

Tolerances: FP32 1e-4 (ACA tolerance 1e-6 times the cancellation of these
sums); FP16 3e-3 and BF16 2e-2: one stored value's rounding (2^-12, 2^-9) times a
cancellation factor of up to ~10 (the sum of |terms| over |sum| of a receiver's
far lags); measured 0.5-1.5e-3 (FP16) and 4-8e-3 (BF16)."""
import numpy as np
import pytest

import seas_inputs as SI
from oracle import interaction as OI
from oracle import seas as OS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2603_00383_amd")

TOL = {"f32": 1e-4, "f16": 3e-3, "bf16": 2e-2}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.init()
    yield


def _pair(n):
    L = 50.0 * n
    return [SI.fault(0.0, 0.0, 0.0, L, n), SI.fault(0.0, 1.6 * L, 10.0, L, n)]


@pytest.mark.parametrize("n", [150, 1200])
@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
def test_single_block_history_part(n, dtype):
    faults = _pair(n)
    params = SI.default_params(factor_dtype=dtype, aca_tol=1e-6, eta_H=2.0, leaf=50, time_block=16)
    op = P.Operator(faults, params)
    blocks = op.blocks(0, 1)
    prior = SI.saturated_history(faults, op.info["max_lag"] + 2, 1)
    fric = SI.rate_state_fields(faults)
    ini = SI.near_nucleation_state(faults, fric, seed=0, bump_amp=0.05)
    s = torch.cuda.current_stream().cuda_stream
    st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], ini["tau0_rate"], stream=s)
    st.load_history(prior, stream=s)
    print(f"[gpu] single block n={n} {dtype}: blocks {len(blocks)} items {op.info['n_items']} "
          f"segments {op.info['n_segments']}", flush=True)
    st.step(1, stream=s)
    st.check(stream=s)
    g = st.read("f_hist", stream=s)
    rows = sorted({0, 1, n // 3, n // 2, n - 1, n, n + 7, n + n // 2, 2 * n - 1})
    ref = OI.stress_rows(OS.Problem(faults, params, dense=False).geo, rows,
                         np.concatenate([prior, ini["V"][None, :]]), 0, -len(prior), SI.MU, SI.CS,
                         op.info["dt"], 0.01, 0.01, min_lag=1, with_tail=True)
    e = np.abs(g[rows] - ref).max() / np.abs(ref).max()
    print(f"[gpu] single block n={n} {dtype}: rel err {e:.3e}", flush=True)
    assert e < TOL[dtype]
