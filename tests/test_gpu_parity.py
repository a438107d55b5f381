"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Error measure: e = max_n |f_gpu^n - f_ref^n|_inf / max_n |f_ref^n|_inf (global over
steps), and the same for state fields.  Tolerances: 1e-10 for the FP64 path with
the operator uncompressed or compressed far below that level, the ACA tolerance
(times a small factor) for compressed operators, 1e-4 for FP32 factors.
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


def _dummy_friction(N):
    return dict(a=np.full(N, 0.01), b=np.full(N, 0.015), Dc=np.full(N, 5e-3), sigma_n=np.full(N, 50e6),
                V0=np.full(N, 1e-6), f0=np.full(N, 0.6))


def gpu_prescribed(faults, params, V, prior=None):
    op = P.Operator(faults, params)
    N = op.N
    s = _stream()
    st = P.State(op, _dummy_friction(N), np.full(N, 1e-9), np.full(N, 5e6), np.zeros(N), stream=s)
    if prior is not None:
        st.load_history(prior, stream=s)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    fd = torch.empty_like(Vd)
    print(f"[gpu] prescribed N={N} steps={V.shape[0]} items={op.info['n_items']}", flush=True)
    st.eval_prescribed(Vd, V.shape[0], fd, stream=s)
    torch.cuda.synchronize()
    return fd.cpu().numpy(), op


def rel_err(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


_REF = {}


def oracle_prescribed(key, faults, params, V, prior=None):
    if key not in _REF:
        prob = OS.Problem(faults, params)
        _REF[key] = OS.prescribed(prob, V, prior_V=prior)
    return _REF[key]


# ----------------------------------------------------------------- workload 1
C1 = SI.two_fault_prescribed_faults()


@pytest.mark.parametrize("seed,S", [(0, 1), (1, 1), (0, 8)])
def test_two_fault_prescribed_fp64_uncompressed(seed, S):
    V = SI.prescribed_slip_rate(C1, 256, seed)
    p = SI.default_params(compress=0, time_block=S)
    f, op = gpu_prescribed(C1, p, V)
    ref = oracle_prescribed(("c1", seed), C1, p, V)
    assert op.info["lag0_nnz"] > 0          # the faults intersect: lag-0 coupling exercised
    e = rel_err(f, ref)
    print(f"[gpu] two-fault fp64 dense seed {seed}: err {e:.3e}")
    assert e < 1e-10


def test_two_fault_prescribed_fp64_compressed_tight():
    V = SI.prescribed_slip_rate(C1, 256, 0)
    p = SI.default_params(compress=1, aca_tol=1e-13, eta_H=2.0, leaf=50)
    f, op = gpu_prescribed(C1, p, V)
    ref = oracle_prescribed(("c1", 0), C1, SI.default_params(compress=0), V)
    e = rel_err(f, ref)
    print(f"[gpu] two-fault fp64 aca 1e-13: err {e:.3e}")
    assert e < 1e-10


def test_two_fault_prescribed_aca_1e6_fp64_and_fp32():
    V = SI.prescribed_slip_rate(C1, 256, 0)
    ref = oracle_prescribed(("c1", 0), C1, SI.default_params(compress=0), V)
    f64, op = gpu_prescribed(C1, SI.default_params(aca_tol=1e-6), V)
    e64 = rel_err(f64, ref)
    f32, _ = gpu_prescribed(C1, SI.default_params(aca_tol=1e-6, factor_dtype="f32"), V)
    e32 = rel_err(f32, ref)
    f16b, _ = gpu_prescribed(C1, SI.default_params(aca_tol=1e-6, factor_dtype="f32", time_block=16), V)
    e16b = rel_err(f16b, ref)
    f32b, op32 = gpu_prescribed(C1, SI.default_params(aca_tol=1e-6, factor_dtype="f32", time_block=32), V)
    e32b = rel_err(f32b, ref)
    print(f"[gpu] aca 1e-6: fp64 err {e64:.3e}, fp32 err {e32:.3e}, fp32 S=16 (MFMA) err {e16b:.3e}, "
          f"fp32 S=32 err {e32b:.3e}, stored/dense {op.info['stored_entries'] / op.info['dense_entries']:.3f}")
    assert op32.info["n_segments"] > 0
    assert e64 < 1e-5
    assert e32 < 1e-4
    assert e16b < 1e-4
    assert e32b < 1e-4


FIVE60 = SI.five_fault_network(seed=3, n_elem=60)


@pytest.mark.parametrize("dtype,S,tol", [("f64", 1, 1e-5), ("f32", 32, 1e-4)])
def test_partial_aca_prescribed_against_oracle(dtype, S, tol):
    # aca_partial = 1: admissible blocks at lags behind both wave fronts are built
    # from rows and columns of the block (partial pivoting, truncated SVD); a prior
    # history longer than every window makes the evaluation read all of those lags
    kw = dict(aca_tol=1e-6, leaf=10, eta_H=2.0, factor_dtype=dtype, time_block=S)
    V = SI.prescribed_slip_rate(FIVE60, 40, 7, lo_exp=-6, hi_exp=0)
    full = P.Operator(FIVE60, SI.default_params(host_only=1, **kw))
    prior = SI.prescribed_slip_rate(FIVE60, full.info["max_lag"] + 10, 8, lo_exp=-6, hi_exp=0)
    ref = oracle_prescribed(("five60", 0), FIVE60, SI.default_params(compress=0, leaf=10, eta_H=2.0), V, prior)
    f, op = gpu_prescribed(FIVE60, SI.default_params(aca_partial=1, **kw), V, prior=prior)
    f0, _ = gpu_prescribed(FIVE60, SI.default_params(**kw), V, prior=prior)
    e, e0 = rel_err(f, ref), rel_err(f0, ref)
    print(f"[gpu] partial aca {dtype} S={S}: err {e:.3e} (full pivoting {e0:.3e}), stored "
          f"{op.info['stored_entries']} vs {full.info['stored_entries']}")
    assert op.info["stored_entries"] != full.info["stored_entries"]
    assert not np.array_equal(f, f0)
    assert e < tol


# ----------------------------------------------------------------- ragged, saturated windows
RAG = [SI.fault(0, 0, 5.0, 1300.0, 13), SI.fault(300.0, 900.0, 70.0, 2900.0, 29),
       SI.fault(-1500.0, 2200.0, 140.0, 2000.0, 40)]


@pytest.mark.parametrize("tail,S", [(1, 1), (0, 1), (1, 4), (1, 16)])
def test_ragged_network_with_prior_history(tail, S):
    # odd sizes, leaf 5 (many tiny blocks), history longer than every window so that
    # slip expires into the static tail; a prior history before t = 0
    p = SI.default_params(compress=1, aca_tol=1e-13, eta_H=1.5, leaf=5, int_tail=tail, time_block=S)
    n_steps = 140
    V = SI.prescribed_slip_rate(RAG, n_steps, 7, lo_exp=-6, hi_exp=0)
    prior = SI.prescribed_slip_rate(RAG, 90, 8, lo_exp=-6, hi_exp=0)
    f, op = gpu_prescribed(RAG, p, V, prior=prior)
    assert op.info["max_lag"] < n_steps + len(prior) - 20     # slip expires into the tail
    ref = oracle_prescribed(("rag", tail), RAG, p, V, prior)
    e = rel_err(f, ref)
    print(f"[gpu] ragged tail={tail} S={S}: err {e:.3e}")
    assert e < 1e-10


def test_empty_prescribed_call_is_a_no_op():
    op = P.Operator(C1[:1] + [SI.fault(0, 3000.0, 10.0, 1000.0, 10)], SI.default_params())
    N = op.N
    st = P.State(op, _dummy_friction(N), np.full(N, 1e-9), np.full(N, 5e6), np.zeros(N), stream=_stream())
    st.eval_prescribed(0, 0, 0, stream=_stream())
    torch.cuda.synchronize()
    assert st.step_index == 0


# ----------------------------------------------------------------- SEAS steps
def _seas_setup(faults, seed, prior_len=0, V_init=1e-9, bump=0.05):
    # explicit state updates need dt small against Dc/V (the predictor of the aging
    # law goes negative otherwise): mild perturbations on well-resolved meshes
    fric = SI.rate_state_fields(faults)
    ini = SI.near_nucleation_state(faults, fric, seed=seed, V_init=V_init, bump_amp=bump)
    prior = SI.saturated_history(faults, prior_len, seed) if prior_len else None
    return fric, ini, prior


def _gpu_seas(faults, params, fric, ini, prior, n_steps, fields=("V", "theta", "delta")):
    op = P.Operator(faults, params)
    s = _stream()
    st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], ini["tau0_rate"], stream=s)
    if prior is not None:
        st.load_history(prior, stream=s)
    print(f"[gpu] seas N={op.N} steps={n_steps}", flush=True)
    st.step(n_steps, stream=s)
    st.check(stream=s)
    return {k: st.read(k, stream=s) for k in fields}, st, op


def _oracle_seas(faults, params, fric, ini, prior, n_steps):
    prob = OS.Problem(faults, params)
    st = OS.SeasState(prob, fric, ini["V"], ini["theta"], ini["tau0"], ini["tau0_rate"], prior_V=prior)
    for _ in range(n_steps):
        st.step()
    return st


@pytest.mark.parametrize("S", [1, 8])
def test_seas_trajectory_two_faults(S):
    faults = SI.two_fault_prescribed_faults(n_elem=24, dx=50.0)
    p = SI.default_params(compress=0, time_block=S)
    fric, ini, _ = _seas_setup(faults, 0, V_init=1e-6, bump=0.1)
    g, _, _ = _gpu_seas(faults, p, fric, ini, None, 120, ("V", "theta", "delta", "f_self", "f_int"))
    o = _oracle_seas(faults, p, fric, ini, None, 120)
    print(f"[gpu] seas two-fault 120 steps S={S}: " + ", ".join(
        f"{k} {rel_err(g[k], v):.2e}" for k, v in (("V", o.V), ("theta", o.theta), ("delta", o.delta))))
    assert rel_err(g["V"], o.V) < 1e-9
    assert rel_err(g["theta"], o.theta) < 1e-9
    assert rel_err(g["delta"], o.delta) < 1e-9
    assert rel_err(g["f_self"], o.last["f_self"]) < 1e-9
    assert rel_err(g["f_int"], o.last["f_int"]) < 1e-9


@pytest.mark.parametrize("S", [1, 4])
def test_seas_step_from_saturated_history_five_faults(S):
    faults = SI.five_fault_network(seed=0, n_elem=24)
    p = SI.default_params(compress=1, aca_tol=1e-13, eta_H=2.0, leaf=6, time_block=S)
    fric, ini, prior = _seas_setup(faults, 0, prior_len=160)
    g, _, op = _gpu_seas(faults, p, fric, ini, prior, 6, ("V", "theta", "delta", "f_hist"))
    assert op.info["max_lag"] < 160
    o = _oracle_seas(faults, p, fric, ini, prior, 6)
    print(f"[gpu] seas five-fault saturated: f_hist {rel_err(g['f_hist'], o.last['f_hist']):.2e} "
          f"V {rel_err(g['V'], o.V):.2e}")
    assert rel_err(g["f_hist"], o.last["f_hist"]) < 1e-10
    assert rel_err(g["V"], o.V) < 1e-9
    assert rel_err(g["theta"], o.theta) < 1e-10
    assert rel_err(g["delta"], o.delta) < 1e-10


@pytest.mark.parametrize("S", [1, 8])
def test_checkpoint_resume_is_bitwise(S):
    # with S = 8 the checkpoint is taken in the middle of a time block
    faults = SI.two_fault_prescribed_faults(n_elem=16, dx=50.0)
    p = SI.default_params(time_block=S)
    fric, ini, _ = _seas_setup(faults, 1, V_init=1e-6, bump=0.1)
    op = P.Operator(faults, p)
    s = _stream()
    st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], stream=s)
    st.step(20, stream=s)
    ck = st.save(stream=s)
    st.step(15, stream=s)
    a = st.read("V", stream=s)
    st.restore(ck, stream=s)
    assert st.step_index == 20
    st.step(15, stream=s)
    b = st.read("V", stream=s)
    assert np.array_equal(a, b)


def test_newton_failure_is_reported():
    # a background stress that is not finite fails the solve
    faults = SI.two_fault_prescribed_faults(n_elem=8, dx=1600.0)
    op = P.Operator(faults, SI.default_params())
    N = op.N
    fr = _dummy_friction(N)
    s = _stream()
    tau0 = np.full(N, 0.6 * 50e6)
    tau0[3] = np.nan
    st = P.State(op, fr, np.full(N, 1e-9), np.full(N, 5e-3 / 1e-6), tau0, stream=s)
    st.step(1, stream=s)
    with pytest.raises(P.SeasError) as e:
        st.check(stream=s)
    assert e.value.code == -4
    st.check(stream=s)   # flag cleared


def test_kernel_timing_counts_launches():
    faults = SI.two_fault_prescribed_faults(n_elem=32, dx=50.0)
    op = P.Operator(faults, SI.default_params())
    fric, ini, _ = _seas_setup(faults, 2)
    s = _stream()
    st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], stream=s)
    st.set_timing(True)
    st.step(7, stream=s)
    ms, n = st.read_timing(stream=s)
    assert n == 7 and ms > 0


@pytest.mark.parametrize("SB", [8, 16, 32])
def test_plain_and_blocked_orders_agree(SB):
    # one operator built with S = SB, evaluated once per step (S = 1) and per block
    # (S = 16 in FP32 runs on the matrix cores)
    faults = SI.five_fault_network(seed=2, n_elem=32)
    p = SI.default_params(aca_tol=1e-8, factor_dtype="f32", time_block=SB)
    V = SI.prescribed_slip_rate(faults, 40, 3, lo_exp=-6, hi_exp=0)
    out = []
    for S in (1, SB):
        op = P.Operator(faults, p)
        N = op.N
        st = P.State(op, _dummy_friction(N), np.full(N, 1e-9), np.full(N, 5e6), np.zeros(N), stream=_stream())
        st.set_time_block(S)
        Vd = torch.from_numpy(V).cuda()
        fd = torch.empty_like(Vd)
        st.eval_prescribed(Vd, 40, fd, stream=_stream())
        torch.cuda.synchronize()
        out.append(fd.cpu().numpy())
    e = rel_err(out[1], out[0])
    print(f"[gpu] plain vs blocked S={SB} (FP32): {e:.2e}")
    assert e < 2e-5


def test_fp32_segment_kernel_matches_item_kernel(monkeypatch):
    # FP32 with S = 16 runs the far list in the segment layout (rows grouped per
    # workgroup, inner index fastest); SEAS_NO_SEG builds the same operator for the
    # one-item-per-workgroup kernel. Same factors, FP32 sums in another order.
    faults = SI.five_fault_network(seed=3, n_elem=48)
    p = SI.default_params(aca_tol=1e-6, factor_dtype="f32", time_block=16, leaf=12)
    V = SI.prescribed_slip_rate(faults, 48, 5, lo_exp=-6, hi_exp=0)
    prior = SI.prescribed_slip_rate(faults, 400, 6, lo_exp=-6, hi_exp=0)
    fs, op_s = gpu_prescribed(faults, p, V, prior)
    monkeypatch.setenv("SEAS_NO_SEG", "1")
    fi, op_i = gpu_prescribed(faults, p, V, prior)
    assert op_s.info["n_segments"] > 0 and op_i.info["n_segments"] == 0
    assert op_s.info["stored_entries"] == op_i.info["stored_entries"]
    e = rel_err(fs, fi)
    print(f"[gpu] FP32 segment vs item kernel: {e:.2e} ({op_s.info['n_segments']} segments, "
          f"{op_i.info['n_items']} items)", flush=True)
    assert e < 1e-5


# ----------------------------------------------------------------- cluster-level windows
@pytest.mark.parametrize("S", [1, 16])
def test_cluster_windows_prescribed_against_oracle(S):
    # per-block upper lags (Section 4.3's cluster-level truncation) with the static
    # tail per block: the ragged network with a prior history long enough for slip
    # to leave every block window
    p = SI.default_params(compress=1, aca_tol=1e-13, eta_H=1.5, leaf=5, int_tail=1, time_block=S,
                          cluster_windows=1)
    n_steps = 140
    V = SI.prescribed_slip_rate(RAG, n_steps, 7, lo_exp=-6, hi_exp=0)
    prior = SI.prescribed_slip_rate(RAG, 90, 8, lo_exp=-6, hi_exp=0)
    f, op = gpu_prescribed(RAG, p, V, prior=prior)
    assert any(te < op.windows()[(0, 1)][1] for te in op.block_windows(0, 1))
    ref = oracle_prescribed(("rag-cluster",), RAG, p, V, prior)
    e = rel_err(f, ref)
    print(f"[gpu] ragged cluster windows S={S}: err {e:.3e}")
    assert e < 1e-10
    # and the windows changed the result (the pair-window sum differs)
    ref_pair = oracle_prescribed(("rag", 1), RAG, dict(p, cluster_windows=0), V, prior)
    assert rel_err(ref, ref_pair) > 1e-6


def test_cluster_windows_seas_trajectory():
    faults = [SI.fault(0.0, 0.0, 0.0, 1200.0, 24), SI.fault(110.0, 35.0, 63.0, 1000.0, 20),
              SI.fault(-300.0, 900.0, 150.0, 800.0, 16)]
    p = SI.default_params(compress=1, aca_tol=1e-13, eta_H=1.5, leaf=4, time_block=8, cluster_windows=1)
    fric, ini, prior = _seas_setup(faults, 5, prior_len=120, V_init=1e-6, bump=0.1)
    g, _, op = _gpu_seas(faults, p, fric, ini, prior, 60, ("V", "theta", "delta", "f_hist"))
    o = _oracle_seas(faults, p, fric, ini, prior, 60)
    errs = {k: rel_err(g[k], ref) for k, ref in (("V", o.V), ("theta", o.theta), ("delta", o.delta),
                                               ("f_hist", o.last["f_hist"]))}
    print("[gpu] cluster windows SEAS: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    for k, v in errs.items():
        assert v < 1e-9, k
