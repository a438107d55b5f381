"""Full-size parity of the ensemble path (eight 750-element faults, 64 variants,
BF16 and FP16 factors): every variant gets the same seeded slip-rate history
and near-nucleation state, so each variant's interaction history part must be
the oracle's; sampled receivers (with the ones nearest a fault crossing) are
compared, and all 64 variants must agree with each other bit for bit (product
columns are formed on their own, FP16 panels with a scale per variant).

The prior history covers 1200 steps (the longest windows are ~3500 lags: the
older lags multiply zero history, the static tail and lags up to 1200 are
exercised). Both formats keep near-field blocks, lags below 16 and the static
tail in FP32 (BF16 ensembles stage those from the FP64 history). Tolerances:
those of the small ensemble tests, 8e-3 (BF16, outside the 1e-4 band) and 1e-4
(FP16); the errors are printed."""
import numpy as np
import pytest

import seas_inputs as SI
from oracle import interaction as OI
from oracle import seas as OS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2603_00383_amd")

TOL = {"bf16": 8e-3, "f16": 1e-4}


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_ensemble_fullsize_history_part(dtype, loud):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    nv, H = 64, 1200
    faults = SI.ensemble_network(seed=0)
    params = SI.default_params(factor_dtype=dtype, aca_tol=1e-6, eta_H=2.0, leaf=50, time_block=1, n_variants=nv)
    with loud(f"[gpu] building the ensemble operator ({dtype})"):
        op = P.Operator(faults, params)
    N = op.N
    fric = SI.rate_state_fields(faults)
    ini = SI.near_nucleation_state(faults, fric, seed=0, bump_amp=0.05)
    prior = SI.saturated_history(faults, H, 0)
    s = torch.cuda.current_stream().cuda_stream
    tile = lambda a: np.tile(a, nv)
    st = P.State(op, {k: tile(v) for k, v in fric.items()}, tile(ini["V"]), tile(ini["theta"]), tile(ini["tau0"]),
                 tile(ini["tau0_rate"]), stream=s)
    print(f"[gpu] loading {H} prior steps for {nv} variants", flush=True)
    st.load_history(np.repeat(prior[:, None, :], nv, axis=1), stream=s)
    st.step(1, stream=s)
    st.check(stream=s)
    g0 = st.read("f_hist", stream=s, variant=0)
    for v in (1, 17, 63):
        assert np.array_equal(st.read("f_hist", stream=s, variant=v), g0)
    rng = np.random.default_rng(3)
    rows = sorted(set(rng.integers(0, N, 24).tolist()) | set(SI.closest_to_other_faults(faults, 6)[0]))
    prob = OS.Problem(faults, params, dense=False)
    Vh = np.concatenate([prior, ini["V"][None, :]])
    ref = OI.stress_rows(prob.geo, rows, Vh, 0, -len(prior), prob.mu, prob.cs, prob.dt, 0.01, 0.01,
                         min_lag=1, with_tail=True)
    err = np.abs(g0[rows] - ref) / np.abs(ref).max()
    print(f"[gpu] ensemble full size {dtype}: max sampled rel err {err.max():.3e} at row {rows[int(err.argmax())]}; "
          f"median {np.median(err):.2e}", flush=True)
    assert err.max() < TOL[dtype]
