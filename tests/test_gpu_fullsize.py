"""Full-size parity at the benchmark's configuration (five 600-element faults,
ACA 1e-6, eta_H 2, leaf 50, saturated history windows), FP32 factors and the
16-bit forms.

The oracle cannot evaluate all 3000 receivers at every lag in seconds, so it is
compared on sampled receivers (kernel rows evaluated on the fly) at the same
steps, including the receivers nearest a fault crossing.  Tolerances: 1e-4
relative for FP32 (FP32 accumulation per work item;
ACA 1e-6) and FP16 (11-bit factors and history with per-item scales), 2e-3 for
BF16 (one BF16 rounding, 2^-9; BF16 does not reach 1e-4)."""
import numpy as np
import pytest

import seas_inputs as SI
from oracle import interaction as OI
from oracle import seas as OS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2603_00383_amd")

# fault ends and interiors of every fault, and the eight receivers nearest a
# fault crossing (the worst-conditioned sums; the closest lies 2.9 m from one)
ROWS = sorted(set([0, 37, 301, 599, 600, 899, 1200, 1511, 1799, 1800, 2222, 2400, 2650, 2999]
                  + SI.closest_to_other_faults(SI.five_fault_network(seed=0))[0]))


TOL = {"f32": 1e-4, "f16": 1e-4, "bf16": 2e-3}
# (factor dtype, time block): FP32 with 16 and 32 windows per far launch
FORMS = {"f32": ("f32", 16), "f32_S32": ("f32", 32), "f16": ("f16", 16), "bf16": ("bf16", 16)}


@pytest.fixture(scope="module", params=list(FORMS))
def fullsize(request, loud):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    faults = SI.five_fault_network(seed=0)
    dtype, S = FORMS[request.param]
    params = SI.default_params(factor_dtype=dtype, aca_tol=1e-6, eta_H=2.0, leaf=50, time_block=S)
    with loud(f"[gpu] building the five-fault operator ({request.param})"):
        op = P.Operator(faults, params)
    prior = SI.saturated_history(faults, op.info["max_lag"] + 2, 0)
    print(f"[gpu] built {request.param}: items={op.info['n_items']} max_lag={op.info['max_lag']}", flush=True)
    oracle = OS.Problem(faults, params, dense=False)
    return faults, params, op, prior, oracle


def test_fullsize_prescribed_sampled(fullsize):
    faults, params, op, prior, oracle = fullsize
    N = op.N
    s = torch.cuda.current_stream().cuda_stream
    fr = SI.rate_state_fields(faults)
    st = P.State(op, fr, np.full(N, 1e-9), np.full(N, 5e6), np.zeros(N), stream=s)
    st.load_history(prior, stream=s)
    V = SI.saturated_history(faults, 3, 1)
    Vd = torch.from_numpy(V).cuda()
    fd = torch.empty_like(Vd)
    st.eval_prescribed(Vd, 3, fd, stream=s)
    torch.cuda.synchronize()
    f = fd.cpu().numpy()
    Vall = np.concatenate([prior, V])
    first = -len(prior)
    for n in (1, 3):
        ref = OS.prescribed_rows(oracle, Vall, first, n, ROWS)
        e = np.abs(f[n - 1, ROWS] - ref).max() / np.abs(ref).max()
        print(f"[gpu] full-size {params['factor_dtype']} prescribed step {n}: sampled rel err {e:.3e}", flush=True)
        assert e < TOL[params["factor_dtype"]]


def test_fullsize_seas_step_history_part(fullsize):
    faults, params, op, prior, oracle = fullsize
    s = torch.cuda.current_stream().cuda_stream
    fric = SI.rate_state_fields(faults)
    ini = SI.near_nucleation_state(faults, fric, seed=0, bump_amp=0.05)
    st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], ini["tau0_rate"], stream=s)
    st.load_history(prior, stream=s)
    st.step(1, stream=s)
    st.check(stream=s)
    g = st.read("f_hist", stream=s)      # first step of a time block: far and near parts
    Vh = np.concatenate([prior, ini["V"][None, :]])
    ref = OI.stress_rows(oracle.geo, ROWS, Vh, 0, -len(prior), oracle.mu, oracle.cs, oracle.dt,
                         params["eta_tmin"], params["eta_tmax"], min_lag=1, with_tail=True)
    e = np.abs(g[ROWS] - ref).max() / np.abs(ref).max()
    print(f"[gpu] full-size {params['factor_dtype']} SEAS history part: sampled rel err {e:.3e}", flush=True)
    assert e < TOL[params["factor_dtype"]]
