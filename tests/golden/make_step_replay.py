"""Writes step_replay_five_fault.json: the oracle's one predictor-corrector step
(Section 2.4) on every element of one fault of the five-fault benchmark network
(5 x 600 elements), from seeded saturated states, for the GPU replay test.

Inputs are the seeded generators of ``seas_inputs`` only: the network (seed 0),
its rate-and-state fields, a prior slip-rate history as long as the longest pair
window plus two steps, and two initial states (steady sliding at 1e-9 m/s, and at
1e-4 m/s, each with the tanh overstress). The expected values come from
``oracle`` only: the interaction history part of the fault's receivers (and of
the receivers coupled to them at lag 0) row by row, then ``seas.step_fault``.

    python tests/golden/make_step_replay.py [workers]
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "step_replay_five_fault.json")
CASES = {"slow": dict(seed=0, V_init=1e-9), "fast": dict(seed=1, V_init=1e-4)}
_W = {}


def _init(n_prior):
    import seas_inputs as SI
    from oracle import geometry
    from threadpoolctl import threadpool_limits
    _W["lim"] = threadpool_limits(limits=1)
    faults = SI.five_fault_network(seed=0)
    _W["geo"] = geometry.discretize(faults)
    _W["dt"] = geometry.time_step(_W["geo"], SI.CS)
    _W["prior"] = SI.saturated_history(faults, n_prior, 0)


def _rows(rows):
    import seas_inputs as SI
    from oracle import interaction as OI
    v = OI.stress_rows(_W["geo"], rows, _W["prior"], 0, -len(_W["prior"]), SI.MU, SI.CS, _W["dt"],
                       0.01, 0.01, min_lag=1, with_tail=True)
    return rows, v


def main(workers):
    import numpy as np
    import seas_inputs as SI
    from oracle import interaction as OI, seas as OS
    faults = SI.five_fault_network(seed=0)
    params = SI.default_params(factor_dtype="f64")
    prob = OS.Problem(faults, params, dense=False)
    nf = len(faults)
    max_lag = max(OI.pair_window_lags(prob.geo, a, b, prob.cs, prob.dt, 0.01, 0.01)[1]
                  for a in range(nf) for b in range(nf) if a != b)
    n_prior = max_lag + 2
    worst, _ = SI.closest_to_other_faults(faults, 1)
    fault = int(np.searchsorted(prob.off, worst[0], side="right") - 1)
    rows = list(range(prob.off[fault], prob.off[fault + 1])) + OS.lag0_partners(prob, fault)
    t0 = time.time()
    f_hist = {}
    chunks = [rows[i::workers] for i in range(workers)]
    with mp.get_context("spawn").Pool(workers, initializer=_init, initargs=(n_prior,)) as pool:
        for rr, v in pool.imap_unordered(_rows, [c for c in chunks if c]):
            f_hist.update(zip(rr, v))
    print(f"interaction rows: {len(rows)} in {time.time() - t0:.0f} s", flush=True)
    prior = SI.saturated_history(faults, n_prior, 0)
    fric = SI.rate_state_fields(faults)
    out = {"description": "oracle: one predictor-corrector step of every element of one fault of the five-fault "
                          "network from seeded saturated states (tests/golden/make_step_replay.py)",
           "network_seed": 0, "prior_steps": n_prior, "prior_seed": 0, "fault": fault,
           "rows": [int(r) for r in rows], "f_hist": [float(f_hist[r]) for r in rows], "cases": {}}
    W = max(int(s.W.max()) for s in prob.selfs)
    for name, c in CASES.items():
        ini = SI.near_nucleation_state(faults, fric, seed=c["seed"], V_init=c["V_init"], bump_amp=0.05)
        N = prob.N
        # slip before t = 0 from the prior rates, D rows for the last W + 1 steps
        delta = np.zeros((W + 1, N))
        for m in range(W - 1, -1, -1):                      # rows m' = m - W (times -W..0)
            delta[m] = delta[m + 1] - prob.dt * prior[len(prior) - (W - m)]
        Dh = [(-W, prob.selfs[g].dft(delta[:, prob.off[g]:prob.off[g + 1]])) for g in range(nf)]
        from oracle import friction as OF
        st = dict(V=ini["V"], theta=ini["theta"], thetadot=OF.state_rate(ini["V"], ini["theta"], fric["Dc"]),
                  delta=np.zeros(N), tau0=ini["tau0"], tau0_rate=ini["tau0_rate"], n=0, Dh=Dh)
        r = OS.step_fault(prob, fric, st, fault, f_hist)
        out["cases"][name] = {"seed": c["seed"], "V_init": c["V_init"], "bump_amp": 0.05,
                              "V": [float(x) for x in r["V"]], "theta": [float(x) for x in r["theta"]],
                              "delta": [float(x) for x in r["delta"]]}
        print(f"case {name}: V in [{r['V'].min():.3e}, {r['V'].max():.3e}]", flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh)
    print("wrote", OUT)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1))
