#!/usr/bin/env python3
"""Throughput of the SEAS step loop on one MI355X.

Workload (default): five seeded 30 km faults of 600 elements (N = 3000, dx = 50 m)
in a 40 x 20 km box, strikes U(0, 40) degrees; H-matrix with eta_H = 2, leaf 50,
ACA tolerance 1e-6; FP32 factors, FP64 state and friction; aging law with the
velocity-weakening central patch; a seeded slip-rate history as long as the
longest causality window is loaded first, so every timed step evaluates full
windows.  A step is one predictor-corrector step: history push, interaction
convolution over the H-stack with its static tail and lag-0 terms, spectral self
term, two Newton solves and the state update.

Prints one JSON line: element-steps/s (N x steps / wall time), the roofline of
the dominant kernel (the H-matrix apply, timed with HIP events on its launch
stream) and the oracle's CPU rate on a bounded sample of receivers.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0   # dense matrix-core peak
METRIC = "element-steps/s (stress eval) vs plain at rel err≤1e-4; p50/p99 window latency"

def measured_traffic(kname, args=None, variant=0):
    """HBM bytes per far pass from the table below (for the tuned variant of the
    segment kernel in use), or None when a source file it depends on changed since
    the counters were taken or the inputs are not the default ones (seed 0, ACA 1e-6)
    the counters were taken on."""
    import hashlib
    entry = MEASURED_TRAFFIC.get((kname, variant))
    if args is not None and (args.seed != 0 or args.aca != 1e-6):
        return None
    if entry is None:
        return None
    value, files = entry
    for src, sha in files.items():
        with open(os.path.join(ROOT, "paper_2603_00383_amd", "csrc", src), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != sha:
                return None
    return value


KIB = 1024
# HBM bytes of the timed far launch (five-fault workload, the part with lags >= 2S at the
# form's time block: 32 for the FP32 headline, 16 for the other forms), from rocprofv3
# --pmc FETCH_SIZE and WRITE_SIZE runs of this script (KiB per dispatch), scaled by what the same counters read for a plain 2 GiB copy (2.0 for
# FETCH_SIZE, 1.0 for WRITE_SIZE); each entry names the SHA-256 of the sources it was
# measured on. The 16-bit forms' timed launch is the 16-bit kernel plus the FP32 pass
# over the near-field blocks (k_hmat_mfma16).
_K = "b356a4168284d5794ec84ff58826d368597de9aab75841010a57eca0cdfdbd6e"    # kernels.hip
_X = "acde92eb022c298f9c457827ac8ce58d10afdfe13f6a663bd201dd9fcbc2ebaa"    # kernels_x16.hip
_B = "cddf8d433d1bec38691053ddc4ec3a3d96373d0561bbdbc4743646ed0153b68b"    # build.cpp (item layout)
_SRC = {"kernels.hip": _K, "kernels_x16.hip": _X, "build.cpp": _B}
# (kernel, tuned variant of the segment kernel) -> bytes per timed launch
MEASURED_TRAFFIC = {
    ("k_hmat_x16<f32,32 columns>", 0): (2.0 * 10_265_900 * KIB + 885_138 * KIB, _SRC),
    ("k_hmat_x16<f32,32 columns>", 1): (2.0 * 9_526_570 * KIB + 594_729 * KIB, _SRC),
    ("k_hmat_x16<f32,32 columns>", 2): (2.0 * 9_529_830 * KIB + 601_923 * KIB, _SRC),
    ("k_hmat_x16<f32,16 columns>", 0): (2.0 * 10_049_300 * KIB + 239_933 * KIB, _SRC),
    ("k_hmat_x16<f16,16 columns>", 0): (2.0 * 4_516_800 * KIB + 102_364 * KIB + 2.0 * 1_252_080 * KIB + 22_340 * KIB,
                                        _SRC),
    ("k_hmat_x16<bf16,16 columns>", 0): (2.0 * 4_412_090 * KIB + 102_407 * KIB + 2.0 * 1_252_080 * KIB + 22_340 * KIB,
                                         _SRC),
    # the 64-variant BF16 ensemble's far pass (workload 4): the 16-bit kernel and the FP32 list
    ("k_hmat_x16<bf16,64 columns>", 0): (2.0 * 32_277_300 * KIB + 1_215_790 * KIB + 2.0 * 6_920_150 * KIB
                                         + 39_376 * KIB, _SRC),
}


def graph_leg(n_steps=640):
    """SEAS steps of a small network (two 12.8 km faults x 128 elements, FP64, ACA
    1e-12, time block 16), plain launches against graph replays of whole blocks
    (seas_state_set_graph), from the same state; the results are identical."""
    import numpy as np
    import torch
    import paper_2603_00383_amd as P
    import seas_inputs as SI
    s = torch.cuda.current_stream().cuda_stream
    faults = SI.two_fault_prescribed_faults()
    op = P.Operator(faults, SI.default_params(factor_dtype="f64", aca_tol=1e-12, time_block=16,
                                              state_update="exact"))
    fric = SI.rate_state_fields(faults)
    ini = SI.near_nucleation_state(faults, fric, seed=0, V_init=1e-9, bump_amp=0.05)
    res = {}
    fields = {}
    for mode in ("plain", "graph"):
        st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], stream=s)
        st.set_graph(mode == "graph")
        st.step(32, stream=s)                       # warm-up (captures the graph)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        st.step(n_steps, stream=s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        st.check(stream=s)
        fields[mode] = st.read("V", stream=s)
        res[mode] = {"ms_per_step": wall / n_steps * 1e3, "value": op.N * n_steps / wall}
        if mode == "graph":
            res[mode].update(st.graph_info())
        st.close()
    op.close()
    return {"workload": "SEAS steps, two faults x 128 elements (N=256), FP64, ACA 1e-12, time block 16, "
                        f"{n_steps} steps after 32", "unit": "element-steps/s", **res,
            "speedup": res["plain"]["ms_per_step"] / res["graph"]["ms_per_step"],
            "identical": bool(np.array_equal(fields["plain"], fields["graph"]))}


def cpu_cores():
    """Host cores the CPU legs use: the process's CPU affinity (what nproc reports),
    at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


_W = {}


def _rows_init(seed, n_prior):
    """Worker set-up: the seeded workload and its prior history, generated in the
    worker (no large arrays cross process boundaries)."""
    from threadpoolctl import threadpool_limits
    import seas_inputs as SI
    from oracle import geometry
    _W["limit"] = threadpool_limits(limits=1)
    faults = SI.five_fault_network(seed=seed)
    _W["geo"] = geometry.discretize(faults)
    _W["prior"] = SI.saturated_history(faults, n_prior, seed)
    _W["dt"] = geometry.time_step(_W["geo"], SI.CS)


def _rows_work(job):
    """Oracle interaction history part (lags >= 1 and the static tail) of some
    receivers at one head, and its wall time."""
    import seas_inputs as SI
    from oracle import interaction as OI
    rows, head = job
    t0 = time.perf_counter()
    v = OI.stress_rows(_W["geo"], rows, _W["prior"], head, -len(_W["prior"]), SI.MU, SI.CS, _W["dt"],
                       0.01, 0.01, min_lag=1, with_tail=True)
    return rows, head, v, time.perf_counter() - t0


def cpu_leg(seed):
    """The oracle on the host, before the GPU is touched: (a) the five-fault
    workload's interaction history part on a bounded sample of receivers at five
    saturated heads (the sampled values also give each GPU form's error), plus
    the full self term of every fault, as element-steps/s of one step; (b) the
    two-fault FP64 workload's 256 prescribed steps in full."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    import seas_inputs as SI
    from oracle import interaction as OI
    from oracle import seas as OS
    cores = cpu_cores()
    faults = SI.five_fault_network(seed=seed)
    params = SI.default_params(factor_dtype="f64")
    prob = OS.Problem(faults, params, dense=False)
    N = prob.N
    max_lag = max(OI.pair_window_lags(prob.geo, a, b, prob.cs, prob.dt, 0.01, 0.01)[1]
                  for a in range(len(faults)) for b in range(len(faults)) if a != b)
    n_prior = max_lag + 8
    worst, dmin = SI.closest_to_other_faults(faults)
    rows = sorted(set(worst) | set(int(r) for r in np.linspace(0, N - 1, 96).astype(int)))
    heads = [0, -1, -2, -3, -4]
    chunks = [rows[i::cores] for i in range(cores)]
    jobs = [(c, h) for h in heads for c in chunks if c]
    t_head = {h: 0.0 for h in heads}
    ref0 = {}
    ctx = mp.get_context("spawn")
    w0 = time.perf_counter()
    with ctx.Pool(cores, initializer=_rows_init, initargs=(seed, n_prior)) as pool:
        for rr, h, v, dt_ in pool.imap_unordered(_rows_work, jobs):
            t_head[h] += dt_
            if h == 0:
                ref0.update(zip(rr, v))
    wall_rows = time.perf_counter() - w0
    # self term of every fault at a saturated step (faults of one size share tables)
    prior = SI.saturated_history(faults, n_prior, seed)
    with threadpool_limits(limits=1):
        delta = np.vstack([np.zeros((1, N)), np.cumsum(prior, axis=0) * prob.dt])
        delta = delta - delta[-1][None, :]
        t0 = time.perf_counter()
        for k in range(len(faults)):
            st = prob.selfs[k]
            W = int(st.W.max())
            Dh = st.dft(delta[-W - 1:, prob.off[k]:prob.off[k + 1]])
            st.stress(Dh, 0, -W)
        t_self = time.perf_counter() - t0
    # rows run `cores` at a time: one step's interaction rows take their summed
    # time / cores of wall time; the self term ran on one core
    per_step = [t_head[h] / len(rows) * N / cores + t_self for h in heads]
    med = float(np.median(per_step))
    # (b) two-fault workload: the dense oracle over all 256 steps
    f1 = SI.two_fault_prescribed_faults()
    p1 = SI.default_params(factor_dtype="f64", compress=0)
    V1 = SI.prescribed_slip_rate(f1, 256, seed)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        prob1 = OS.Problem(f1, p1)
        t1 = time.perf_counter()
        ref1 = OS.prescribed(prob1, V1)
        t2 = time.perf_counter()
    out = {"value": N / med, "unit": "element-steps/s", "cores": cores, "kind": "oracle",
           "sample": (f"five-fault workload (N={N}): the oracle's interaction history part (all lags >= 1 "
                      f"of every pair window, kernel evaluated on the fly, static tail) of {len(rows)} "
                      f"receivers (96 evenly spaced, {len(worst)} nearest a fault crossing, the closest "
                      f"{dmin:.1f} m) at 5 saturated steps on {cores} worker processes, plus the full self "
                      f"term of all {len(faults)} faults on one core; per-step time = summed row time x "
                      f"N / {len(rows)} / {cores} + self term, median of the 5 steps; "
                      f"{wall_rows:.1f} s wall for the rows"),
           "per_step_s": per_step,
           "two_fault_fp64": {"value": 256 * 256 / (t2 - t1), "unit": "element-steps/s", "cores": 1,
                              "eval_s": t2 - t1, "setup_s": t1 - t0,
                              "sample": "all 256 steps of the two-fault prescribed-history workload "
                                        "(2 x 128 elements), dense FP64 stacks, direct self term"}}
    return out, dict(rows=rows, worst=worst, ref0=np.array([ref0[r] for r in rows]), n_prior=n_prior,
                     max_lag=max_lag, ref1=ref1, V1=V1)


def run_precision(args):
    """Trajectory error of the reduced-precision forms: the five-fault SEAS step loop
    (5 x 600 elements, time block 16, and 32 for the FP32 headline form) from one
    near-nucleation state with no prior slip, stepped 20,000 steps with FP64, FP32,
    FP16 and BF16 factors; slip, slip rate and stress (f_self + f_int) compared with
    the FP64 run at 1k, 5k and 20k steps. The FP64 path is the one the parity tests
    hold to the oracle at 1e-10."""
    import numpy as np
    import torch

    import paper_2603_00383_amd as P
    import seas_inputs as SI

    marks = (1000, 5000, 20000)
    faults = SI.five_fault_network(seed=args.seed)
    fric = SI.rate_state_fields(faults)
    ini = SI.near_nucleation_state(faults, fric, seed=args.seed, bump_amp=args.bump)
    os.environ.setdefault("SEAS_VERBOSE", "1")
    s = torch.cuda.current_stream().cuda_stream
    snaps, timing, failed, peak = {}, {}, {}, {}
    forms = {"f64": ("f64", 16), "f32": ("f32", 16), "f32_S32": ("f32", 32), "f16": ("f16", 16),
             "bf16": ("bf16", 16)}
    for d, (dtype, S) in forms.items():
        params = SI.default_params(factor_dtype=dtype, aca_tol=args.aca, eta_H=2.0, leaf=50, time_block=S,
                                   state_update=args.state_update)
        print(f"[bench] building the {d} operator", file=sys.stderr, flush=True)
        op = P.Operator(faults, params)
        st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], ini["tau0_rate"], stream=s)
        snaps[d] = {}
        vmax = 0.0
        done, t_run = 0, 0.0
        try:
            for m in marks:
                while done < m:
                    k = min(1000, m - done)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    st.step(k, stream=s)
                    st.check(stream=s)
                    t_run += time.perf_counter() - t0
                    done += k
                    vmax = max(vmax, float(st.read("V", stream=s).max()))
                    print(f"[bench] {d}: {done} steps", file=sys.stderr, flush=True)
                snaps[d][m] = {"delta": st.read("delta", stream=s), "V": st.read("V", stream=s),
                               "stress": st.read("f_self", stream=s) + st.read("f_int", stream=s)}
        except RuntimeError as e:
            failed[d] = f"step {done}: {e}"
            print(f"[bench] {d} stopped: {failed[d]}", file=sys.stderr, flush=True)
        timing[d] = t_run / max(done, 1) * 1e3
        peak[d] = vmax
        st.close()
        op.close()
    ref = snaps["f64"]
    errors = {}
    for d in [f for f in forms if f != "f64"]:
        errors[d] = {}
        for m in marks:
            if m not in snaps[d] or m not in ref:
                continue
            e = {}
            for k in ("delta", "V", "stress"):
                e[k] = float(np.abs(snaps[d][m][k] - ref[m][k]).max() / np.abs(ref[m][k]).max())
            errors[d][str(m)] = e
    out = {"metric": "slip, slip-rate and stress error of the reduced-precision forms vs the FP64 path",
           "data": "synthetic",
           "config": {"workload": "five-fault SEAS step loop, 5 x 600 elements (N=3000, dx=50 m), time block "
                                  f"16 (f32_S32: 32), ACA 1e-6, eta_H 2, leaf 50, near-nucleation state (tanh overstress "
                                  f"{args.bump:g} tau_eq), no prior slip, {args.state_update} state update",
                      "seed": args.seed, "steps": list(marks)},
           "errors": errors, "ms_per_step": timing, "failed": failed,
           "peak_slip_rate_sampled": peak,
           "note": "max |x - x_f64| / max |x_f64| over all elements at each mark; stress = f_self + f_int; "
                   "peak slip rate over the 1000-step marks"}
    print(json.dumps(out), flush=True)


def run_two_fault(args):
    """The paper's two-fault benchmark (Section 3.1, Table 1) at its resolution (2 x 1000
    elements) from the printed initial state to T_end = 2 s, and the admissibility
    sweep of Appendix C: for each eta_H the operator is built with ACA 1e-6 (the
    paper's SVD tolerance) in FP64, and the slip rate at the two fault midpoints at
    T_end is compared with the run of the operator stored without compression."""
    import numpy as np
    import torch

    import paper_2603_00383_amd as P
    import seas_inputs as SI

    with open(os.path.join(ROOT, "tests", "golden", "two_fault_benchmark.json")) as fh:
        gold = json.load(fh)
    n = args.elements
    faults, fric = SI.two_fault_benchmark(gold, n)
    ini = SI.two_fault_benchmark_state(gold, faults, fric)
    os.environ.setdefault("SEAS_VERBOSE", "1")
    s = torch.cuda.current_stream().cuda_stream
    mids = [n // 2, n + n // 2]
    runs = {}
    etas = [float(x) for x in args.etas.split(",")]
    for key in ["dense"] + etas:
        over = dict(compress=0) if key == "dense" else dict(eta_H=key)
        p = SI.two_fault_benchmark_params(gold, n, time_block=16, factor_dtype="f64", **over)
        print(f"[bench] two-fault benchmark: building ({key})", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        op = P.Operator(faults, p)
        bs = time.perf_counter() - t0
        info = op.info
        steps = int(np.ceil(2.0 / info["dt"] - 1e-9))
        st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], ini["tau0_rate"], stream=s)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        st.step(steps, stream=s)
        st.check(stream=s)
        wall = time.perf_counter() - w0
        V = st.read("V", stream=s)
        runs[key] = {"V": V, "delta": st.read("delta", stream=s), "build_s": bs, "ms_per_step": wall / steps * 1e3,
                     "steps": steps, "stored_over_dense": info["stored_entries"] / info["dense_entries"],
                     "far_GB": info["far_bytes"] / 1e9, "n_blocks": info["n_blocks"]}
        print(f"[bench]   {steps} steps in {wall:.2f} s, stored/dense {runs[key]['stored_over_dense']:.3f}, "
              f"V at midpoints {V[mids[0]]:.4e} {V[mids[1]]:.4e}", file=sys.stderr, flush=True)
        st.close()
        op.close()
    ref = runs["dense"]
    rows = {}
    for key, r in runs.items():
        rows[str(key)] = {
            "ms_per_step": r["ms_per_step"], "build_s": r["build_s"], "stored_over_dense": r["stored_over_dense"],
            "far_GB": r["far_GB"], "n_blocks": r["n_blocks"],
            "V_mid": [float(r["V"][m]) for m in mids],
            "rel_err_V_mid": [float(abs(r["V"][m] - ref["V"][m]) / abs(ref["V"][m])) for m in mids],
            "rel_err_V": float(np.abs(r["V"] - ref["V"]).max() / np.abs(ref["V"]).max()),
            "rel_err_slip": float(np.abs(r["delta"] - ref["delta"]).max() / np.abs(ref["delta"]).max())}
    out = {"metric": "two-fault benchmark: slip-rate error at the fault midpoints at T_end vs the uncompressed "
                     "operator, time per step, compression, per eta_H",
           "data": "synthetic (the paper's printed benchmark inputs)",
           "config": {"workload": f"two-fault benchmark of Section 3.1 / Table 1, 2 x {n} elements, FP64, ACA 1e-6, "
                                  "leaf 50, time block 16, closed-form state update, T_end = 2 s",
                      "steps": runs["dense"]["steps"], "dt": float(2.0 / runs["dense"]["steps"])},
           "paper": {"compression_eta_1.5": 0.247,
                     "note": "Section 3.1 prints a total compression of about 24.7% at eta_H = 1.5"},
           "runs": rows}
    print(json.dumps(out), flush=True)


def adaptive_leg(n=1000, max_steps=3000, t_target=60.0):
    """Adaptive steps (Section 2.4.1, step 1) on the paper's two-fault benchmark (Section
    3.1, Table 1) at 2 x n elements, FP64 factors: two steps of gamma = 1 settle the
    printed initial state (a rate held under the overstress), then gamma follows the
    rule (xi = 0.5) through the rupture and after it, until t_target seconds or
    max_steps steps. Reports the steps, the Delta t_min grid steps they cover and the
    element-steps per second of both."""
    import numpy as np
    import torch

    import paper_2603_00383_amd as P
    import seas_inputs as SI

    with open(os.path.join(ROOT, "tests", "golden", "two_fault_benchmark.json")) as fh:
        gold = json.load(fh)
    faults, fric = SI.two_fault_benchmark(gold, n)
    ini = SI.two_fault_benchmark_state(gold, faults, fric)
    p = SI.two_fault_benchmark_params(gold, n, time_block=1, factor_dtype="f64", adaptive_dt=1, adapt_xi=0.5)
    s = torch.cuda.current_stream().cuda_stream
    t0 = time.perf_counter()
    op = P.Operator(faults, p)
    bs = time.perf_counter() - t0
    N, dt = op.N, op.info["dt"]
    st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], ini["tau0_rate"], stream=s)
    st.set_gamma_cap(1)
    st.step(2, stream=s)
    st.check(stream=s)
    st.set_gamma_cap(0)
    g0 = st.step_index
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    gammas = []
    while len(gammas) < max_steps and st.step_index * dt < t_target:
        st.step(1, stream=s)
        gammas.append(st.progress()["last_gamma"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    st.check(stream=s)
    V = st.read("V", stream=s)
    grid = st.step_index - g0
    k1 = next((i for i, g in enumerate(gammas) if g > 1 and i > 10), None)
    out = {"workload": f"two-fault benchmark of Section 3.1 / Table 1, 2 x {n} elements, FP64, eta_H 1.5, ACA 1e-6, "
                       "per-step evaluation (time block 1), adaptive steps xi = 0.5 after two steps of gamma = 1",
           "steps": len(gammas), "grid_steps": int(grid), "time_reached_s": float(st.step_index * dt),
           "wall_s": wall, "ms_per_step": wall / max(len(gammas), 1) * 1e3,
           "element_steps_per_s": N * len(gammas) / wall,
           "grid_element_steps_per_s": N * grid / wall,
           "fixed_steps_for_same_time": int(grid), "step_reduction": grid / max(len(gammas), 1),
           "gamma_first_above_1_at_step": k1, "gamma_max": int(max(gammas)),
           "gamma_median": float(np.median(gammas)), "V_max_end": [float(V[:n].max()), float(V[n:].max())],
           "build_s": bs}
    st.close()
    op.close()
    return out


def run_adaptive(args):
    print(json.dumps({"adaptive": adaptive_leg(args.elements, args.adaptive_steps, args.adaptive_time)}), flush=True)


def run_ensemble(args):
    """Ensemble throughput: one geometry, many friction variants stepped together;
    the interaction sums of all variants are one 16-bit product per work item."""
    import numpy as np
    import torch

    import paper_2603_00383_amd as P
    import seas_inputs as SI

    dtype = args.dtype or "bf16"
    nv = args.variants
    faults = SI.ensemble_network(seed=args.seed)
    params = SI.default_params(factor_dtype=dtype, aca_tol=args.aca, eta_H=2.0, leaf=50, time_block=1,
                               n_variants=nv)
    os.environ.setdefault("SEAS_VERBOSE", "1")
    print("[bench] building the ensemble operator", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    op = P.Operator(faults, params)
    build_s = time.perf_counter() - t0
    info = op.info
    N = op.N
    print(f"[bench] operator built in {build_s:.1f} s: N={N} items={info['n_items']} segments="
          f"{info['n_segments']} far bytes={info['far_bytes'] / 1e9:.2f} GB max_lag={info['max_lag']}",
          file=sys.stderr, flush=True)
    base = SI.rate_state_fields(faults)
    var = SI.ensemble_variants(nv, seed=args.seed)
    fric = {k: np.tile(base[k], nv) for k in ("sigma_n", "V0", "f0")}
    fric["a"] = np.repeat(var["a"], N)
    fric["b"] = np.repeat(var["b"], N)
    fric["Dc"] = np.repeat(var["Dc"], N)
    V, th, t0_, t0r = [], [], [], []
    for v in range(nv):
        fv = {k: fric[k][v * N:(v + 1) * N] for k in ("a", "b", "Dc", "sigma_n", "V0", "f0")}
        ini = SI.near_nucleation_state(faults, fv, seed=args.seed, bump_amp=0.05)
        V.append(ini["V"]); th.append(ini["theta"]); t0_.append(ini["tau0"]); t0r.append(ini["tau0_rate"])
    stream = torch.cuda.current_stream()
    s = stream.cuda_stream
    st = P.State(op, fric, np.concatenate(V), np.concatenate(th), np.concatenate(t0_), np.concatenate(t0r),
                 stream=s)
    print(f"[bench] state of {nv} variants created, warmup {args.warmup}", file=sys.stderr, flush=True)
    st.step(args.warmup, stream=s)
    st.check(stream=s)
    tune = op.tune(st, stream=s, reps=2)
    print(f"[bench] tuned far-pass variant {tune['choice']}: {tune['ms']} ms per launch", file=sys.stderr,
          flush=True)
    st.set_timing(True)
    st.read_timing(stream=s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record(stream)
    st.step(args.steps, stream=s)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms, n = st.read_timing(stream=s)
    st.check(stream=s)
    avg = ms / max(n, 1)
    # the 16-bit entries at 2 B, the FP32 list (near-field blocks, early lags, tail) at 4 B
    alg_bytes = (info["far_entries"] - info["far_entries_f32"]) * 2 + info["far_entries_f32"] * 4
    flops = 2.0 * info["far_entries"] * info["ncols"]
    achieved = alg_bytes / (avg * 1e-3) / 1e9
    kname = f"k_hmat_x16<{dtype},{info['ncols']} columns>"
    tflops = flops / (avg * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": N * nv * args.steps / wall,
        "unit": "element-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": f"ensemble: 8 faults x 750 elements (N=6000, dx=50 m), {nv} friction variants "
                               f"(a-b, Dc per variant), {dtype.upper()} factors and history operand, FP32 "
                               "accumulation, FP64 state, ACA 1e-6, eta_H 2, leaf 50",
                   "seed": args.seed, "N": N, "variants": nv, "max_lag": info["max_lag"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kname, args, tune["choice"]),
                     "kernel": kname, "kernel_avg_ms": avg,
                     "algorithmic_bytes": alg_bytes, "launches_per_step": n / args.steps,
                     "mfma": {"achieved": tflops, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                              "frac": tflops / BF16_PEAK_TFLOPS, "flops_per_launch": flops}},
        "gpu_event_ms_per_step": e0.elapsed_time(e1) / args.steps,
        "build_s": build_s,
        "stored_over_dense": info["stored_entries"] / info["dense_entries"],
        "autotune": {"choice": tune["choice"], "ms_per_launch": tune["ms"],
                     "variants": ["prefetch 8", "prefetch 4", "prefetch 12"],
                     "note": "far launch per variant of the 16-bit segment kernel on this operator and state "
                             "(seas_operator_tune); the fastest is used for the timed steps"},
    }
    print(f"[bench] timed {args.steps} steps: {wall:.3f} s", file=sys.stderr, flush=True)
    # the same steps as replays of one captured graph of 16 steps (no kernel timing inside)
    st.set_timing(False)
    st.set_graph(True)
    st.step(16, stream=s)
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    st.step(args.steps, stream=s)
    torch.cuda.synchronize()
    wall_g = time.perf_counter() - w1
    st.check(stream=s)
    gi = st.graph_info()
    out["captured"] = {"value": N * nv * args.steps / wall_g, "ms_per_step": wall_g / args.steps * 1e3,
                       "replays": gi["replays"], "steps_per_replay": gi["steps_per_replay"],
                       "note": "the timed steps again, whole 16-step blocks replayed from one HIP graph "
                               "(seas_state_set_graph)"}
    print(f"[bench] captured: {wall_g / args.steps * 1e3:.3f} ms per step ({gi['replays']} replays)",
          file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def _window(SI, np, faults, seed, quiet=False):
    """One request's seeded friction (a - b and Dc drawn per request on the
    velocity-weakening patches) and its near-nucleation initial state."""
    fric = SI.rate_state_fields(faults)
    N = len(fric["a"])
    if quiet:  # velocity strengthening at steady state: an idle slot
        fric["b"] = np.full(N, 0.005)
        ini = SI.near_nucleation_state(faults, fric, seed=seed, bump_amp=0.0)
    else:
        var = SI.ensemble_variants(1, seed=seed)
        fric["b"] = np.where(fric["b"] > 0.01, var["b"][0], fric["b"])
        fric["Dc"] = np.full(N, var["Dc"][0])
        ini = SI.near_nucleation_state(faults, fric, seed=seed, bump_amp=0.05)
    return dict(fric=fric, V=ini["V"], theta=ini["theta"], tau0=ini["tau0"], tau0_rate=ini["tau0_rate"])


def serving_leg(seed, dtype, templates, sizes, n_requests, rate, min_steps, max_steps, chunk, budget_gb,
                slots=16):
    """Serving: a Poisson stream of simulation-window requests on seeded geometry
    templates, admitted into variant slots of one ensemble state per template
    (continuous batching); p50/p99 completion latency and throughput."""
    import numpy as np

    import paper_2603_00383_amd as P
    import seas_inputs as SI

    tpls = SI.serving_templates(seed=seed, n_templates=templates, sizes=sizes)
    reqs = SI.poisson_requests(n_requests=n_requests, rate=rate, seed=seed, n_templates=templates,
                               min_steps=min_steps, max_steps=max_steps)
    ops, build_s = [], 0.0
    for k, f in enumerate(tpls):
        t0 = time.perf_counter()
        ops.append(P.Operator(f, SI.default_params(factor_dtype=dtype, aca_tol=1e-6, eta_H=2.0, leaf=50,
                                                   time_block=1, n_variants=slots)))
        build_s += time.perf_counter() - t0
        print(f"[bench] template {k}: N={ops[-1].N} faults={len(f)} built", file=sys.stderr, flush=True)
    idle = [_window(SI, np, f, 0, quiet=True) for f in tpls]
    budget = int(budget_gb * 2 ** 30)
    sv = P.Server(ops, idle, budget, chunk_steps=chunk)
    trace = [dict(pool=q["template"], n_steps=q["n_steps"], arrival_s=q["arrival"],
                  window=_window(SI, np, tpls[q["template"]], q["seed"])) for q in reqs]
    print(f"[bench] serving {len(trace)} requests over {reqs[-1]['arrival']:.1f} s", file=sys.stderr, flush=True)
    w0 = time.perf_counter()
    res = sv.run(trace)
    wall = time.perf_counter() - w0
    lat = np.array([r["finish_s"] - q["arrival_s"] for r, q in zip(res, trace)])
    work = float(sum(ops[q["pool"]].N * q["n_steps"] for q in trace))
    bad = sum(1 for r in res if r["status"] != 0)
    sv.close()
    for o in ops:
        o.close()
    return {
        "value": work / wall, "unit": "element-steps/s",
        "workload": f"serving: {len(trace)} Poisson requests (rate {rate}/s), {templates} seeded templates "
                    f"with N in {list(sizes)} and 2-10 faults, windows {min_steps}-{max_steps} steps, "
                    f"{slots} slots per template, {dtype.upper()} factors, chunks of {chunk} steps",
        "templates": [o.N for o in ops], "requests": len(trace),
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "max": float(lat.max())},
        "makespan_s": wall, "trace_span_s": float(reqs[-1]["arrival"]), "failed_requests": bad,
        "build_s": build_s, "budget_GiB": budget_gb,
    }


def run_serving(args):
    dtype = args.dtype or "f16"
    os.environ.setdefault("SEAS_VERBOSE", "1")    # build and request-loop progress on stderr
    sizes = tuple(int(x) for x in args.sizes.split(","))
    r = serving_leg(args.seed, dtype, args.templates, sizes, args.requests, args.rate,
                    args.min_steps, args.max_steps, args.chunk, args.budget_gb)
    out = {"metric": METRIC, "value": r["value"], "unit": r["unit"], "n_gpus": 1,
           "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": {"workload": r["workload"], "seed": args.seed, "templates": r["templates"],
                      "budget_GiB": args.budget_gb},
           "latency_s": r["latency_s"], "makespan_s": r["makespan_s"], "trace_span_s": r["trace_span_s"],
           "failed_requests": r["failed_requests"], "build_s": r["build_s"]}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=160)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="seas",
                    choices=["seas", "ensemble", "serving", "precision", "two-fault", "adaptive"],
                    help="seas: five-fault step loop (one variant); ensemble: eight faults x 750 elements, "
                         "64 friction variants in one launch (BF16); precision: 20,000-step trajectories of "
                         "the reduced-precision forms against FP64")
    ap.add_argument("--dtype", default=None, choices=["f32", "f64", "bf16", "f16"],
                    help="factor dtype (default f32; bf16 for the ensemble)")
    ap.add_argument("--variants", type=int, default=64, help="ensemble: friction variants (16, 32 or 64)")
    ap.add_argument("--elements", type=int, default=1000, help="two-fault: elements per fault")
    ap.add_argument("--bump", type=float, default=2.0,
                    help="precision: overstress of the initial state in units of tau_eq (2: the paper's)")
    ap.add_argument("--state-update", default="exact", choices=["explicit", "exact"],
                    help="precision: state update (exact: closed form at constant rate)")
    ap.add_argument("--etas", default="1.0,1.5,2.0,3.0,5.0,20.0", help="two-fault: eta_H values of the sweep")
    ap.add_argument("--templates", type=int, default=4, help="serving: geometry templates")
    ap.add_argument("--requests", type=int, default=32, help="serving: requests in the trace")
    ap.add_argument("--rate", type=float, default=4.0, help="serving: arrivals per second")
    ap.add_argument("--min-steps", type=int, default=200, help="serving: shortest window")
    ap.add_argument("--max-steps", type=int, default=2000, help="serving: longest window")
    ap.add_argument("--chunk", type=int, default=16, help="serving: steps per launch chunk")
    ap.add_argument("--sizes", default="500,1000,2000", help="serving: template sizes N to draw from")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serving: device memory for states")
    ap.add_argument("--aca", type=float, default=1e-6)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--time-block", type=int, default=None,
                    help="S: lags >= S applied once per S steps (1 = plain per-step form); default 32 for "
                         "FP32 factors, 16 for the 16-bit and FP64 ones")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-form measurement")
    ap.add_argument("--no-forms", action="store_true", help="skip the 16-bit forms (FP32 runs only)")
    ap.add_argument("--forms", default="f16,bf16,f64,cluster",
                    help="forms measured beside the FP32 headline (comma list of f16, bf16, f64, cluster)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle CPU leg (the forms' errors are then not measured)")
    ap.add_argument("--no-serving", action="store_true", help="skip the bounded serving leg")
    ap.add_argument("--no-two-fault", action="store_true", help="skip the two-fault FP64 workload")
    ap.add_argument("--no-graph", action="store_true", help="skip the captured-steps leg")
    ap.add_argument("--adaptive", action="store_true",
                    help="add the adaptive-step leg (two-fault benchmark, ~90 s with its operator build)")
    ap.add_argument("--adaptive-steps", type=int, default=3000, help="adaptive: steps at most")
    ap.add_argument("--adaptive-time", type=float, default=60.0, help="adaptive: simulated seconds to reach")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy a 2 GiB buffer three times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = 1 << 29
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "launches": 3}))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: runs on one GPU; --gpus N > 1 is not supported "
              "(the path is not sharded over GPUs)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2603_00383_amd as P
    import seas_inputs as SI

    cpu, ref = None, None
    if args.workload == "seas" and not args.no_cpu_baseline:
        # the oracle runs first, in worker processes, before anything uses the GPU
        print(f"[bench] oracle CPU leg on {cpu_cores()} cores", file=sys.stderr, flush=True)
        cpu, ref = cpu_leg(args.seed)
        print(f"[bench] oracle: {cpu['value']:.3g} element-steps/s", file=sys.stderr, flush=True)
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    if args.workload == "ensemble":
        return run_ensemble(args)
    if args.workload == "serving":
        return run_serving(args)
    if args.workload == "precision":
        return run_precision(args)
    if args.workload == "two-fault":
        return run_two_fault(args)
    if args.workload == "adaptive":
        return run_adaptive(args)
    if args.dtype is None:
        args.dtype = "f32"
    if args.time_block is None:
        args.time_block = 32 if args.dtype == "f32" else 16
    faults = SI.five_fault_network(seed=args.seed)
    os.environ.setdefault("SEAS_VERBOSE", "1")
    fric = SI.rate_state_fields(faults)
    # a mild overstress keeps the explicit aging-law update away from its stiff limit
    ini = SI.near_nucleation_state(faults, fric, seed=args.seed, bump_amp=0.05)
    stream = torch.cuda.current_stream()
    s = stream.cuda_stream
    prior_cache = {}
    K, W = args.steps, max(args.warmup, 1)

    def rel_sample(st):
        """Error of the interaction history part after the first step (head 0) on the
        oracle's sampled receivers (max abs difference / max abs reference)."""
        if ref is None:
            return None
        f = st.read("f_hist", stream=s)[ref["rows"]]
        return float(np.abs(f - ref["ref0"]).max() / np.abs(ref["ref0"]).max())

    def prepare(dtype, cluster=0, S=None):
        """Operator of one factor dtype and a state with full history windows: the
        first step is compared with the oracle, then the rest of the warmup."""
        params = SI.default_params(factor_dtype=dtype, aca_tol=args.aca, eta_H=2.0, leaf=50,
                                   time_block=S or args.time_block, cluster_windows=cluster)
        print(f"[bench] building the {dtype} operator", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        op = P.Operator(faults, params)
        bs = time.perf_counter() - t0
        inf = op.info
        print(f"[bench] operator built in {bs:.1f} s: N={op.N} items={inf['n_items']} "
              f"stored/dense={inf['stored_entries'] / inf['dense_entries']:.3f} max_lag={inf['max_lag']}",
              file=sys.stderr, flush=True)
        n_prior = ref["n_prior"] if ref is not None else inf["max_lag"] + 8
        assert n_prior >= inf["max_lag"] + 8
        if n_prior not in prior_cache:
            prior_cache[n_prior] = SI.saturated_history(faults, n_prior, args.seed)
        st = P.State(op, fric, ini["V"], ini["theta"], ini["tau0"], ini["tau0_rate"], stream=s)
        st.load_history(prior_cache[n_prior], stream=s)
        st.step(1, stream=s)
        st.check(stream=s)
        err = rel_sample(st)
        print(f"[bench] history loaded ({n_prior} steps); sampled error vs oracle {err}, warmup {W}",
              file=sys.stderr, flush=True)
        st.step(W - 1, stream=s)
        st.check(stream=s)
        return op, inf, st, bs, err

    def alg_bytes(inf, eb, S=16):
        """Stored far-factor bytes the timed far launch reads: with time blocks (S > 1)
        the part with lags >= 2S (the block-start items, lags S..2S-1, run in a launch
        of their own), in the plain form (S = 1) all of them. 16-bit forms keep the
        near-field blocks in FP32 (far_entries_f32)."""
        far, f32 = inf["far_entries"], inf["far_entries_f32"]
        if S > 1:
            far, f32 = far - inf["far_entries_first"], f32 - inf["far_entries_first_f32"]
        if eb == 2:
            return (far - f32) * 2 + f32 * 4
        return far * eb

    def timed_on(st, inf, eb, S, n, overlap=True):
        """n steps timed from the start of a time block: the region holds every far
        launch its steps need (ceil(n / S)), none run before the timer starts (the
        block lookahead only runs ahead inside one step call)."""
        st.set_time_block(S)          # the next step starts a new block
        st.set_overlap(overlap)
        st.set_timing(True)
        st.read_timing(stream=s)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record(stream)
        st.step(n, stream=s)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ms, launches = st.read_timing(stream=s)
        st.check(stream=s)
        want = -(-n // S)
        assert launches == want, f"{launches} far launches for {n} steps at S = {S} (expected {want})"
        avg = ms / max(launches, 1)
        gbs = alg_bytes(inf, eb, S) / (avg * 1e-3) / 1e9
        st.set_overlap(True)
        return dict(wall=wall, ev_ms=e0.elapsed_time(e1), avg_ms=avg, launches=launches, gbs=gbs,
                    value=inf_N(inf) * n / wall, ms_per_step=wall / n * 1e3)

    def inf_N(inf):
        return inf["n_elem"]

    op, info, st, build_s, err32 = prepare(args.dtype)
    N = op.N
    # tile tuning of the far pass on this operator and state (FP32 segment builds)
    tune = op.tune(st, stream=s, reps=3)
    print(f"[bench] tuned far-pass variant {tune['choice']}: {tune['ms']} ms per launch", file=sys.stderr,
          flush=True)
    elem_bytes = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}[args.dtype]
    S = info["time_block"]
    main_run = timed_on(st, info, elem_bytes, S, K)
    steady = timed_on(st, info, elem_bytes, S, 10 * S)
    serial = timed_on(st, info, elem_bytes, S, 10 * S, overlap=False) if S > 1 else None
    # the plain per-step form (S = 1) on the operator built for 16 windows, as the segment
    # kernel forms all its windows in every launch
    plain = None if (args.no_plain or S not in (2, 4, 8, 16)) else timed_on(st, info, elem_bytes, 1, K)
    wall, avg_ms, achieved = main_run["wall"], main_run["avg_ms"], main_run["gbs"]
    hmat_bytes = alg_bytes(info, elem_bytes, S)
    if args.dtype in ("bf16", "f16"):
        kname = f"k_hmat_x16<{'bf16' if args.dtype == 'bf16' else 'f16'},16 columns>"
    elif args.dtype == "f32" and S in (16, 32) and info["n_segments"] > 0:
        kname = f"k_hmat_x16<f32,{S} columns>"  # the segment kernel, FP32 instance
    elif args.dtype == "f32" and S == 16 and not os.environ.get("SEAS_NO_MFMA"):
        kname = "k_hmat_mfma16"
    else:
        t = 'float' if args.dtype == 'f32' else 'double'
        kname = f"k_hmat<{t},{t},{S}>"
    traffic = measured_traffic(kname, args, tune["choice"])
    out = {
        "metric": METRIC,
        "value": N * K / wall,
        "unit": "element-steps/s",
        "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": "five-fault SEAS step loop, 5 x 600 elements (N=3000, dx=50 m), "
                               f"{args.dtype.upper()} factors" + (" (near-field blocks and lags < 16 in FP32)" if elem_bytes == 2 else "")
                               + f", FP64 state, ACA {args.aca:g}, eta_H 2, leaf 50, saturated history windows, "
                               f"time block {S}, timed from a block start",
                   "seed": args.seed, "N": N, "max_lag": info["max_lag"], "time_block": S},
        "rel_err": err32,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kname,
                     "kernel_avg_ms": avg_ms, "algorithmic_bytes": hmat_bytes,
                     "launches": main_run["launches"],
                     "launches_per_step": main_run["launches"] / K},
        "gpu_event_ms_per_step": main_run["ev_ms"] / K,
        "steady_state": {"value": steady["value"], "ms_per_step": steady["ms_per_step"], "steps": 10 * S,
                         "launches": steady["launches"], "kernel_avg_ms": steady["avg_ms"],
                         "frac": steady["gbs"] / HBM_PEAK_GBS,
                         "note": f"{10 * S} steps from a block start (whole time blocks)"},
        "block_lookahead": None if serial is None else {
            "note": "far lags >= 2S of the next time block run on a second stream beside the current "
                    "block's steps (seas_state_set_overlap); the block-start lags S..2S-1 at the block start",
            "block_start_share_of_far_entries": info["far_entries_first"] / info["far_entries"],
            "steady_state_serial_value": serial["value"], "steady_state_serial_ms_per_step": serial["ms_per_step"],
            "steady_state_serial_kernel_avg_ms": serial["avg_ms"]},
        "build_s": build_s,
        "stored_over_dense": info["stored_entries"] / info["dense_entries"],
        "autotune": {"choice": tune["choice"], "ms_per_launch": tune["ms"],
                     "variants": (["prefetch 2, 4 waves/SIMD", "prefetch 2, 3 waves/SIMD", "prefetch 3, 3 waves/SIMD"]
                                  if args.dtype == "f32" else ["prefetch 8", "prefetch 4", "prefetch 12"]),
                     "note": "far launch of one time block per variant of the FP32 segment kernel on this "
                             "operator and state (seas_operator_tune); the fastest is used for the timed steps; "
                             "-1 where the operator has one form"},
    }
    if plain is not None:
        out["plain"] = {"value": plain["value"], "ms_per_step": plain["ms_per_step"],
                        "kernel_avg_ms": plain["avg_ms"], "achieved_GBs": plain["gbs"],
                        "frac": plain["gbs"] / HBM_PEAK_GBS, "rel_err": err32,
                        "speedup_of_value": (N * K / wall) / plain["value"],
                        "note": "same operator and state, every lag applied every step (S = 1)"}
    print(f"[bench] timed {K} steps: {wall:.3f} s", file=sys.stderr, flush=True)
    st.close()
    op.close()
    if args.dtype == "f32" and S == 32 and not args.no_plain:
        # 16 windows per far launch (the FP32 form with half the columns per factor byte),
        # and the plain per-step form on that operator
        op_d, inf_d, st_d, bs_d, err_d = prepare("f32", S=16)
        r = timed_on(st_d, inf_d, 4, 16, K)
        r_ss = timed_on(st_d, inf_d, 4, 16, 160)
        pl = timed_on(st_d, inf_d, 4, 1, K)
        kn = "k_hmat_x16<f32,16 columns>"
        out.setdefault("forms", {})["f32_S16"] = {
            "value": r["value"], "ms_per_step": r["ms_per_step"], "steady_state_value": r_ss["value"],
            "kernel": kn, "kernel_avg_ms": r["avg_ms"], "achieved_GBs": r["gbs"], "frac": r["gbs"] / HBM_PEAK_GBS,
            "algorithmic_bytes": alg_bytes(inf_d, 4, 16), "rel_err": err_d,
            "within_1e-4": None if err_d is None else bool(err_d <= 1e-4),
            "traffic": measured_traffic(kn, args), "build_s": bs_d,
            "note": "FP32 factors, time block 16 (16 windows per far launch)"}
        out["plain"] = {"value": pl["value"], "ms_per_step": pl["ms_per_step"], "kernel_avg_ms": pl["avg_ms"],
                        "achieved_GBs": pl["gbs"], "frac": pl["gbs"] / HBM_PEAK_GBS, "rel_err": err_d,
                        "speedup_of_value": (N * K / wall) / pl["value"],
                        "note": "FP32 operator with time block 16, every lag applied every step (S = 1)"}
        print(f"[bench] form f32 S=16: {r['value']:.3e} element-steps/s; plain {pl['value']:.3e}",
              file=sys.stderr, flush=True)
        st_d.close()
        op_d.close()
    if args.dtype == "f32" and not args.no_forms and S in (16, 32):
        # the other forms of the same workload (same geometry, state and history)
        out.setdefault("forms", {})
        wanted = set(args.forms.split(","))
        for d in [d for d in ("f16", "bf16", "f64") if d in wanted]:
            op_d, inf_d, st_d, bs_d, err_d = prepare(d, S=16)
            eb = {"f16": 2, "bf16": 2, "f64": 8}[d]
            r = timed_on(st_d, inf_d, eb, 16, K)
            r_ss = timed_on(st_d, inf_d, eb, 16, 160)
            kn = f"k_hmat_x16<{d},16 columns>" if eb == 2 else "k_hmat<double,double,16>"
            out["forms"][d] = {"value": r["value"], "ms_per_step": r["ms_per_step"],
                               "steady_state_value": r_ss["value"], "kernel": kn, "kernel_avg_ms": r["avg_ms"],
                               "achieved_GBs": r["gbs"], "frac": r["gbs"] / HBM_PEAK_GBS,
                               "algorithmic_bytes": alg_bytes(inf_d, eb, 16), "rel_err": err_d,
                               "within_1e-4": None if err_d is None else bool(err_d <= 1e-4),
                               "traffic": measured_traffic(kn, args), "build_s": bs_d,
                               "note": ("admissible blocks' lags >= 16 in 16 bits; near-field blocks, lags "
                                        "1..15 and the static tail in FP32" if eb == 2 else
                                        "FP64 factors, history and accumulation (vector ALUs)")}
            print(f"[bench] form {d}: {r['value']:.3e} element-steps/s, error {err_d}", file=sys.stderr,
                  flush=True)
            st_d.close()
            op_d.close()
    if args.dtype == "f32" and not args.no_forms and S in (16, 32) and "cluster" in args.forms.split(","):
        # cluster-level windows (Section 4.3): FP32, each block truncated at its own upper lag
        op_c, inf_c, st_c, bs_c, err_c = prepare("f32", cluster=1)
        r = timed_on(st_c, inf_c, 4, S, K)
        r_ss = timed_on(st_c, inf_c, 4, S, 10 * S)
        out["forms"]["f32_cluster_windows"] = {
            "value": r["value"], "ms_per_step": r["ms_per_step"], "steady_state_value": r_ss["value"],
            "kernel": f"k_hmat_x16<f32,{S} columns>", "kernel_avg_ms": r["avg_ms"], "achieved_GBs": r["gbs"],
            "frac": r["gbs"] / HBM_PEAK_GBS, "algorithmic_bytes": alg_bytes(inf_c, 4, S),
            "stored_entries": inf_c["stored_entries"], "stored_entries_pair_windows": info["stored_entries"],
            "rel_err": err_c, "within_1e-4": None if err_c is None else bool(err_c <= 1e-4), "build_s": bs_c,
            "note": "FP32 factors, every block truncated at the pair rule applied to its clusters, static "
                    "stress of older slip per block; the error is against the oracle with pair windows "
                    "(the truncation's own error)"}
        print(f"[bench] form f32 cluster windows: {r['value']:.3e} element-steps/s, stored "
              f"{inf_c['stored_entries'] / info['stored_entries']:.3f} of the pair-window operator, "
              f"error {err_c}", file=sys.stderr, flush=True)
        st_c.close()
        op_c.close()
    if not args.no_two_fault:
        # two-fault prescribed-history workload: FP64, H-matrix (ACA 1e-12), 256 steps
        f1 = SI.two_fault_prescribed_faults()
        p1 = SI.default_params(factor_dtype="f64", aca_tol=1e-12, time_block=16)
        op1 = P.Operator(f1, p1)
        V1 = ref["V1"] if ref is not None else SI.prescribed_slip_rate(f1, 256, args.seed)
        Vd = torch.from_numpy(np.ascontiguousarray(V1)).cuda()
        fd = torch.empty_like(Vd)
        N1 = op1.N
        fr1 = {k: np.full(N1, v) for k, v in (("a", 0.01), ("b", 0.015), ("Dc", 5e-3), ("sigma_n", 50e6),
                                               ("V0", 1e-6), ("f0", 0.6))}
        times = []
        for rep in range(3):
            st1 = P.State(op1, fr1, np.full(N1, 1e-9), np.full(N1, 5e6), np.zeros(N1), stream=s)
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            st1.eval_prescribed(Vd, 256, fd, stream=s)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - w0)
            st1.close()
        e1 = None
        if ref is not None:
            f = fd.cpu().numpy()
            e1 = float(np.abs(f - ref["ref1"]).max() / np.abs(ref["ref1"]).max())
        out["two_fault_fp64"] = {"value": N1 * 256 / min(times[1:]), "unit": "element-steps/s",
                                 "ms_per_step": min(times[1:]) / 256 * 1e3, "rel_err": e1,
                                 "workload": "two 12.8 km faults x 128 elements (N=256), prescribed slip-rate "
                                             "history, 256 steps, FP64 H-matrix (ACA 1e-12), time block 16; "
                                             "best of two timed repetitions after one warm one",
                                 "cpu_oracle": cpu["two_fault_fp64"] if cpu else None}
        op1.close()
        print(f"[bench] two-fault FP64: {out['two_fault_fp64']['value']:.3e} element-steps/s, error {e1}",
              file=sys.stderr, flush=True)
    if not args.no_graph:
        out["captured_steps"] = graph_leg()
        g = out["captured_steps"]
        print(f"[bench] captured steps: {g['graph']['ms_per_step']:.4f} ms/step vs {g['plain']['ms_per_step']:.4f} "
              f"plain ({g['speedup']:.2f}x)", file=sys.stderr, flush=True)
    if args.adaptive:
        out["adaptive"] = adaptive_leg(1000, args.adaptive_steps, args.adaptive_time)
        a = out["adaptive"]
        print(f"[bench] adaptive: {a['steps']} steps to t = {a['time_reached_s']:.3g} s ({a['grid_steps']} grid steps, "
              f"{a['wall_s']:.1f} s wall, gamma up to {a['gamma_max']})", file=sys.stderr, flush=True)
    if not args.no_serving:
        out["serving"] = serving_leg(args.seed, "f16", 3, (500, 1000, 2000), 24, 4.0, 200, 1000, 16, 64.0)
        print(f"[bench] serving p50 {out['serving']['latency_s']['p50']:.2f} s p99 "
              f"{out['serving']['latency_s']['p99']:.2f} s", file=sys.stderr, flush=True)
    if cpu is not None:
        out["cpu_baseline"] = {k: v for k, v in cpu.items() if k != "two_fault_fp64"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
