"""GPU parity of the traction-free surface (method of images) through the C ABI.

Two faults below the line y = 0: a vertical one reaching it (its own image acts
on it from lag 0, through the lag-0 coupling) and a buried dipping one. Against
the FP64 oracle with the same images: the prescribed-history stress (FP64, the
uncompressed and the ACA operator, time blocks 1 and 8; FP32 factors on the
time-blocked segment kernel, also with partial ACA; BF16 / FP16 factors on the
16-bit segment kernel; cluster-level windows) and a SEAS trajectory. The
surface also changes the answer (the images are not negligible).

beta = 0.45: with beta = 1/2 the receiver next to the surface sits exactly
cs dt from the first edge of its own image, so the lag-0 kernel there is taken
on the wave front, where the square root in the primitive magnifies rounding
(the library and the oracle then differ by ~1e-9, both correct to rounding).
FP64 tolerance 3e-10: the kernel entries agree to 1e-12 per lag matrix
(test_lib_host), but the images put sources within one element of the
receivers next to the surface, and those near-field terms cancel in the sums
(the FP64 two-fault test of the unbounded medium measures up to 4e-11 for the
same reason).
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


FAULTS = SI.free_surface_network(n_elem=32, dx=50.0)


def _prescribed(p, V):
    op = P.Operator(FAULTS, p)
    N = op.N
    s = _stream()
    fr = dict(a=np.full(N, 0.01), b=np.full(N, 0.015), Dc=np.full(N, 5e-3), sigma_n=np.full(N, 5e7),
              V0=np.full(N, 1e-6), f0=np.full(N, 0.6))
    st = P.State(op, fr, np.full(N, 1e-9), np.full(N, 5e6), np.zeros(N), stream=s)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    fd = torch.empty_like(Vd)
    st.eval_prescribed(Vd, V.shape[0], fd, stream=s)
    torch.cuda.synchronize()
    return fd.cpu().numpy(), op


CASES = [
    ("f64_dense_S1", 3e-10, dict(factor_dtype="f64", compress=0, time_block=1)),
    ("f64_aca_S8", 3e-10, dict(factor_dtype="f64", aca_tol=1e-13, time_block=8, leaf=8)),  # blocks compressed
    ("f32_seg_S16", 1e-5, dict(factor_dtype="f32", aca_tol=1e-10, time_block=16)),
    ("f32_seg_S32", 1e-5, dict(factor_dtype="f32", aca_tol=1e-10, time_block=32)),
    ("f64_cluster", 3e-10, dict(factor_dtype="f64", aca_tol=1e-13, time_block=8, cluster_windows=1, leaf=8)),
    # 16-bit factors: three roundings of 2^-9 (BF16) or 2^-12 (FP16) per lag matrix,
    # with room for the cancellation of the sums
    # (leaf 8: admissible blocks, whose far lags the 16-bit segment kernel applies;
    # with one leaf per fault every block is near-field and stays in FP32)
    ("bf16_seg_S16", 1e-2, dict(factor_dtype="bf16", aca_tol=1e-10, time_block=16, leaf=8)),
    ("f16_seg_S16", 1.5e-3, dict(factor_dtype="f16", aca_tol=1e-10, time_block=16, leaf=8)),
    ("f32_seg_S32_partial_aca", 1e-5, dict(factor_dtype="f32", aca_tol=1e-10, time_block=32, leaf=8, aca_partial=1)),
]


@pytest.mark.parametrize("name,tol,kw", CASES, ids=[c[0] for c in CASES])
def test_prescribed_with_free_surface(name, tol, kw):
    p = SI.default_params(free_surface=1, surface_y=0.0, beta=0.45, **kw)
    V = SI.prescribed_slip_rate(FAULTS, 120, 4)
    f, op = _prescribed(p, V)
    if "_seg_" in name:
        assert op.info["n_segments"] > 0 and op.info["time_block"] == kw["time_block"]
    if name == "f64_aca_S8":
        dense = P.Operator(FAULTS, dict(p, compress=0, host_only=1))
        assert op.info["stored_entries"] < dense.info["stored_entries"]
    if kw.get("aca_partial"):
        full = P.Operator(FAULTS, dict(p, aca_partial=0, host_only=1))
        assert op.info["stored_entries"] != full.info["stored_entries"]
    ref = OS.prescribed(OS.Problem(FAULTS, p), V)
    e = rel_err(f, ref)
    print(f"[gpu] free surface {name}: {e:.2e}", flush=True)
    assert e < tol
    if name == "f64_dense_S1":
        # without the surface the stress differs by far more than the tolerance
        ref0 = OS.prescribed(OS.Problem(FAULTS, SI.default_params(beta=0.45, **kw)), V)
        assert rel_err(ref0, ref) > 1e-2


def test_seas_trajectory_with_free_surface():
    p = SI.default_params(free_surface=1, surface_y=0.0, beta=0.45, factor_dtype="f64", compress=1,
                          aca_tol=1e-12, time_block=8, state_update="exact")
    op = P.Operator(FAULTS, p)
    fric = SI.rate_state_fields(FAULTS)
    ini = SI.near_nucleation_state(FAULTS, fric, seed=7, V_init=1e-6, bump_amp=0.1)
    s = _stream()
    st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], stream=s)
    st.step(100, stream=s)
    st.check(stream=s)
    o = OS.SeasState(OS.Problem(FAULTS, p), fric, ini["V"], ini["theta"], ini["tau0"], state_update="exact")
    for _ in range(100):
        o.step()
    for k, ref in (("V", o.V), ("theta", o.theta), ("delta", o.delta)):
        e = rel_err(st.read(k, stream=s), ref)
        print(f"[gpu] free surface SEAS {k}: {e:.2e}", flush=True)
        assert e < 1e-9, k
