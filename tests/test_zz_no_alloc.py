"""GPU test of seas_eval_prescribed_noalloc, the entry point for callers that
cannot allocate: through the C ABI it must give exactly what
seas_eval_prescribed gives on a twin state, on two calls in a row whose second
input is smaller (a smaller operator, and a shorter continuation), and it must
refuse an operator whose partial sums exceed its fixed scratch array."""
import numpy as np
import pytest

import seas_inputs as SI

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2603_00383_amd")

SCRATCH = 32 << 20


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.init()
    yield


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _states(op, prior=None):
    N = op.N
    fr = dict(a=np.full(N, 0.01), b=np.full(N, 0.015), Dc=np.full(N, 5e-3), sigma_n=np.full(N, 50e6),
              V0=np.full(N, 1e-6), f0=np.full(N, 0.6))
    out = []
    for _ in range(2):
        st = P.State(op, fr, np.full(N, 1e-9), np.full(N, 5e6), np.zeros(N), stream=_stream())
        if prior is not None:
            st.load_history(prior, stream=_stream())
        out.append(st)
    return out


def _both(a, b, V):
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    fa, fb = torch.empty_like(Vd), torch.empty_like(Vd)
    a.eval_prescribed(Vd, V.shape[0], fa, stream=_stream())
    b.eval_prescribed_noalloc(Vd, V.shape[0], fb, stream=_stream())
    torch.cuda.synchronize()
    return fa.cpu().numpy(), fb.cpu().numpy()


def test_noalloc_matches_eval_prescribed():
    # first call: five faults x 48 elements, FP32 factors, time block 16 (segment kernel)
    f1 = SI.five_fault_network(seed=0, n_elem=48)
    op1 = P.Operator(f1, SI.default_params(factor_dtype="f32", time_block=16, leaf=12))
    assert 0 < op1.info["partial_bytes"] <= SCRATCH and op1.info["n_segments"] > 0
    prior = SI.prescribed_slip_rate(f1, 300, 6, lo_exp=-6, hi_exp=0)
    V1 = SI.prescribed_slip_rate(f1, 40, 3, lo_exp=-6, hi_exp=0)
    a1, b1 = _states(op1, prior)
    print(f"[gpu] noalloc call 1: N={op1.N} partial bytes {op1.info['partial_bytes']}", flush=True)
    fa, fb = _both(a1, b1, V1)
    assert np.array_equal(fa, fb) and np.abs(fa).max() > 0
    # second call: a smaller input, two faults x 16 elements, FP64, time block 1
    f2 = SI.two_fault_prescribed_faults(n_elem=16, dx=200.0)
    op2 = P.Operator(f2, SI.default_params())
    assert op2.info["partial_bytes"] < op1.info["partial_bytes"]
    V2 = SI.prescribed_slip_rate(f2, 12, 4)
    a2, b2 = _states(op2)
    print(f"[gpu] noalloc call 2: N={op2.N} partial bytes {op2.info['partial_bytes']}", flush=True)
    fa, fb = _both(a2, b2, V2)
    assert np.array_equal(fa, fb) and np.abs(fa).max() > 0
    # and the first states continue with a shorter call
    fa, fb = _both(a1, b1, SI.prescribed_slip_rate(f1, 9, 5, lo_exp=-6, hi_exp=0))
    assert np.array_equal(fa, fb)


def test_noalloc_refuses_what_it_cannot_hold():
    f = SI.five_fault_network(seed=0, n_elem=200)
    op = P.Operator(f, SI.default_params(factor_dtype="f64", time_block=16))
    assert op.info["partial_bytes"] > SCRATCH
    a, _ = _states(op)
    V = torch.zeros((2, op.N), dtype=torch.float64, device="cuda")
    out = torch.empty_like(V)
    with pytest.raises(P.SeasError) as e:
        a.eval_prescribed_noalloc(V, 2, out, stream=_stream())
    assert e.value.code == -1 and "scratch" in str(e.value)
    # kernel timing creates events: refused on this path
    f2 = SI.two_fault_prescribed_faults(n_elem=16, dx=200.0)
    op2 = P.Operator(f2, SI.default_params())
    b, _ = _states(op2)
    b.set_timing(True)
    V2 = torch.zeros((2, op2.N), dtype=torch.float64, device="cuda")
    with pytest.raises(P.SeasError) as e:
        b.eval_prescribed_noalloc(V2, 2, torch.empty_like(V2), stream=_stream())
    assert e.value.code == -5
