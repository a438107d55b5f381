"""GPU tests of continuous batching: a window started in a variant slot of a
running ensemble state evolves as a fresh state would (bit for bit: every
product column is formed on its own, with its own history scale), and the request loop
(seas_server_run), with requests joining and leaving running batches on two
geometries, returns for every request the result it gets alone."""
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


def _window(faults, seed, bump=0.1, quiet=False):
    """One request's friction and initial values (arrays of N)."""
    fric = SI.rate_state_fields(faults)
    N = len(fric["a"])
    if quiet:  # velocity strengthening everywhere, at steady state
        fric["b"] = np.full(N, 0.005)
        ini = SI.near_nucleation_state(faults, fric, seed=seed, V_init=1e-9, bump_amp=0.0)
    else:
        var = SI.ensemble_variants(1, seed=seed)
        fric["b"] = np.where(fric["b"] > 0.01, var["b"][0], fric["b"])
        fric["Dc"] = np.full(N, var["Dc"][0])
        ini = SI.near_nucleation_state(faults, fric, seed=seed, V_init=1e-6, bump_amp=bump)
    return dict(fric=fric, V=ini["V"], theta=ini["theta"], tau0=ini["tau0"], tau0_rate=ini["tau0_rate"])


def _state(op, windows):
    nv = op.info["n_variants"]
    cat = lambda k: np.concatenate([w[k] for w in windows])
    fric = {k: np.concatenate([w["fric"][k] for w in windows]) for k in ("a", "b", "Dc", "sigma_n", "V0", "f0")}
    assert len(windows) == nv
    return P.State(op, fric, cat("V"), cat("theta"), cat("tau0"), cat("tau0_rate"), stream=_stream())


FAULTS = SI.two_fault_prescribed_faults(n_elem=24, dx=50.0)


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_reset_slot_evolves_like_a_fresh_state(dtype):
    # leaf 8: admissible blocks, so the 16-bit segment kernel (per-variant history
    # scales) runs beside the FP32 list
    op = P.Operator(FAULTS, SI.default_params(factor_dtype=dtype, aca_tol=1e-6, time_block=1, n_variants=16, leaf=8))
    assert op.info["far_entries"] > op.info["far_entries_f32"]
    s = _stream()
    req = _window(FAULTS, 7)
    quiet = _window(FAULTS, 0, quiet=True)
    # alone: the request in slot 0 of a fresh state, quiet windows elsewhere
    a = _state(op, [req] + [quiet] * 15)
    a.step(60, stream=s)
    a.check(stream=s)
    ref = {k: a.read(k, stream=s, variant=0) for k in ("V", "theta", "delta")}
    # in the mix: other windows running for 23 steps, then the request joins slot 9
    others = [_window(FAULTS, 100 + v) for v in range(16)]
    b = _state(op, others)
    b.step(23, stream=s)
    b.reset_variant(9, req["fric"], req["V"], req["theta"], req["tau0"], req["tau0_rate"], stream=s)
    b.step(60, stream=s)
    b.check(stream=s)
    for k in ("V", "theta", "delta"):
        got = b.read(k, stream=s, variant=9)
        e = float(np.abs(got - ref[k]).max() / np.abs(ref[k]).max())
        print(f"[gpu] reset slot {dtype} {k}: rel diff {e:.2e}", flush=True)
        assert np.array_equal(got, ref[k])


def test_server_results_alone_and_in_the_mix():
    geo = [FAULTS, SI.two_fault_prescribed_faults(n_elem=32, dx=50.0)]
    ops = [P.Operator(g, SI.default_params(factor_dtype="bf16", aca_tol=1e-6, time_block=1, n_variants=16, leaf=8))
           for g in geo]
    assert all(o.info["far_entries"] > o.info["far_entries_f32"] for o in ops)
    idle = [_window(g, 0, quiet=True) for g in geo]
    rng = np.random.default_rng(11)
    reqs = []
    t = 0.0
    for i in range(24):
        t += rng.exponential(0.02)
        pool = int(rng.integers(0, 2))
        reqs.append(dict(pool=pool, n_steps=int(rng.integers(20, 90)), arrival_s=t,
                         window=_window(geo[pool], 200 + i)))
    budget = sum(o.state_bytes(16) for o in ops)  # both pools fit
    sv = P.Server(ops, idle, budget, chunk_steps=8)
    print(f"[gpu] server: {len(reqs)} requests on 2 pools", flush=True)
    res = sv.run(reqs)
    lat = np.array([r["finish_s"] - q["arrival_s"] for r, q in zip(res, reqs)])
    print(f"[gpu] server latency p50 {np.percentile(lat, 50) * 1e3:.1f} ms p99 {np.percentile(lat, 99) * 1e3:.1f} ms",
          flush=True)
    assert all(r["status"] == 0 for r in res)
    assert all(r["finish_s"] >= q["arrival_s"] and r["admit_s"] >= q["arrival_s"] for r, q in zip(res, reqs))
    # each request alone, through the same loop on an otherwise empty trace
    for i in (0, 5, 11, 23):
        q = dict(reqs[i])
        q["arrival_s"] = 0.0
        alone = sv.run([q])[0]
        for k in ("V", "theta", "delta"):
            assert np.array_equal(alone[k], res[i][k]), (i, k)
    # a request that cannot converge ends alone, with its last good step; the
    # others keep the results they get alone
    bad = dict(reqs[3])
    bw = dict(bad["window"])
    bw["tau0"] = bw["tau0"].copy()
    bw["tau0"][4] = np.nan
    bad["window"] = bw
    mixed = list(reqs[:8])
    mixed[3] = bad
    resb = sv.run(mixed)
    assert resb[3]["status"] == -4
    assert np.array_equal(resb[3]["V"], bw["V"]) and np.array_equal(resb[3]["theta"], bw["theta"])
    assert np.array_equal(resb[3]["delta"], np.zeros(len(bw["V"])))
    for i in range(8):
        if i != 3:
            assert resb[i]["status"] == 0
            for k in ("V", "theta", "delta"):
                assert np.array_equal(resb[i][k], res[i][k]), (i, k)
    # memory-bound admission: a budget of one pool's state serialises the pools
    sv1 = P.Server(ops, idle, max(o.state_bytes(16) for o in ops), chunk_steps=8)
    res1 = sv1.run(reqs[:8])
    for i in range(8):
        for k in ("V", "theta", "delta"):
            assert np.array_equal(res1[i][k], res[i][k]), (i, k)
