"""GPU parity of the self term's optional static tail (self_tail = 1) through the C ABI.

With the tail each mode's history sum has one more lag, W_n + 1, whose
coefficient is R_n (the integral of the kernel past the window); the library
keeps it as the last entry of the mode's table and one more slot of its
coefficient ring. Compared with the FP64 oracle built with the same option:

* prescribed histories on a ragged three-fault network with a prior history
  longer than the self windows (so the tail reads coefficients of the prior
  history, rebuilt by load_history), FP64 plain and time-blocked, FP32 factors
  on the segment kernel;
* SEAS trajectories past the longest window, fixed steps (time blocks 1 and 8)
  and adaptive steps (the interior coefficient rows of long steps reach the tail).

Each case also checks that the tail changes the result by far more than the
tolerance.
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


RAG = [SI.fault(0, 0, 5.0, 1300.0, 13), SI.fault(300.0, 900.0, 70.0, 2900.0, 29),
       SI.fault(-1500.0, 2200.0, 140.0, 2000.0, 40)]
_REF = {}


def _oracle_prescribed(tail, p, V, prior):
    if tail not in _REF:
        q = dict(p, self_tail=tail, factor_dtype="f64", time_block=1)
        _REF[tail] = OS.prescribed(OS.Problem(RAG, q), V, prior_V=prior)
    return _REF[tail]


CASES = [
    ("f64_S1", 1e-10, dict(compress=1, aca_tol=1e-13, time_block=1)),
    ("f64_S16", 1e-10, dict(compress=1, aca_tol=1e-13, time_block=16)),
    ("f32_seg_S16", 1e-5, dict(factor_dtype="f32", compress=1, aca_tol=1e-10, time_block=16)),
    ("f32_seg_S32", 1e-5, dict(factor_dtype="f32", compress=1, aca_tol=1e-10, time_block=32)),
]


@pytest.mark.parametrize("name,tol,kw", CASES, ids=[c[0] for c in CASES])
def test_prescribed_with_self_tail(name, tol, kw):
    p = SI.default_params(eta_H=1.5, leaf=5, self_tail=1, **kw)
    V = SI.prescribed_slip_rate(RAG, 140, 7, lo_exp=-6, hi_exp=0)
    prior = SI.prescribed_slip_rate(RAG, 90, 8, lo_exp=-6, hi_exp=0)
    op = P.Operator(RAG, p)
    assert op.info["max_self_window"] + 1 < 140 + 90          # the tail reaches the prior history
    N = op.N
    s = _stream()
    fr = dict(a=np.full(N, 0.01), b=np.full(N, 0.015), Dc=np.full(N, 5e-3), sigma_n=np.full(N, 5e7),
              V0=np.full(N, 1e-6), f0=np.full(N, 0.6))
    st = P.State(op, fr, np.full(N, 1e-9), np.full(N, 5e6), np.zeros(N), stream=s)
    st.load_history(prior, stream=s)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    fd = torch.empty_like(Vd)
    print(f"[gpu] self tail prescribed {name} N={N}", flush=True)
    st.eval_prescribed(Vd, V.shape[0], fd, stream=s)
    torch.cuda.synchronize()
    f = fd.cpu().numpy()
    ref = _oracle_prescribed(1, p, V, prior)
    e = rel_err(f, ref)
    print(f"[gpu] self tail prescribed {name}: {e:.2e}", flush=True)
    assert e < tol
    assert rel_err(_oracle_prescribed(0, p, V, prior), ref) > 100 * tol


def _two_fault_setup():
    faults = SI.two_fault_prescribed_faults(n_elem=24, dx=50.0)
    fric = SI.rate_state_fields(faults)
    ini = SI.near_nucleation_state(faults, fric, seed=0, V_init=1e-6, bump_amp=0.1)
    return faults, fric, ini


@pytest.mark.parametrize("S", [1, 8])
def test_seas_with_self_tail(S):
    faults, fric, ini = _two_fault_setup()
    p = SI.default_params(compress=0, time_block=S, self_tail=1, state_update="exact")
    op = P.Operator(faults, p)
    n = 150
    assert op.info["max_self_window"] < n - 20
    s = _stream()
    st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], stream=s)
    print(f"[gpu] self tail seas S={S}", flush=True)
    st.step(n, stream=s)
    st.check(stream=s)
    outs = {}
    for tail in (1, 0):
        o = OS.SeasState(OS.Problem(faults, dict(p, self_tail=tail)), fric, ini["V"], ini["theta"], ini["tau0"],
                         state_update="exact")
        for _ in range(n):
            o.step()
        outs[tail] = o
    o = outs[1]
    for k, ref in (("V", o.V), ("theta", o.theta), ("delta", o.delta), ("f_self", o.last["f_self"])):
        e = rel_err(st.read(k, stream=s), ref)
        print(f"[gpu] self tail seas S={S} {k}: {e:.2e}", flush=True)
        assert e < 1e-9, k
    assert rel_err(outs[0].last["f_self"], o.last["f_self"]) > 1e-6


def test_adaptive_steps_with_self_tail():
    faults = SI.two_fault_prescribed_faults(n_elem=24, dx=50.0)
    fric = SI.rate_state_fields(faults)
    ini = SI.near_nucleation_state(faults, fric, seed=6, V_init=5e-5, bump_amp=0.005)
    N = len(ini["V"])
    rate = 1e6 * np.where(np.arange(N) < N // 2, 1.0, 1.5)
    p = SI.default_params(time_block=1, factor_dtype="f64", compress=0, state_update="exact", adaptive_dt=1,
                          adapt_xi=0.01, gamma_max=300, self_tail=1)
    op = P.Operator(faults, p)
    s = _stream()
    st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], rate, stream=s)
    o = OS.SeasState(OS.Problem(faults, p), fric, ini["V"], ini["theta"], ini["tau0"], rate, state_update="exact",
                     adaptive=True, xi=0.01, gamma_max=300)
    gammas = []
    for k in range(60):
        st.step(1, stream=s)
        o.step()
        gammas.append(o.last["gamma"])
        assert st.progress()["last_gamma"] == o.last["gamma"], k
    st.check(stream=s)
    assert max(gammas) > op.info["max_self_window"]         # whole windows and the tail inside one step
    for k, ref in (("V", o.V), ("theta", o.theta), ("delta", o.delta)):
        e = rel_err(st.read(k, stream=s), ref)
        print(f"[gpu] self tail adaptive {k}: {e:.2e}", flush=True)
        assert e < 1e-9, k
