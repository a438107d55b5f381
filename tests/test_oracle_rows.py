"""Pins of the oracle's row-sampled sums and of the static tail's window edge (CPU only).

``interaction.stress_rows`` and ``seas.prescribed_rows`` are the references of
every full-size GPU test (the dense stacks do not fit there); here they are held
to the dense evaluation (``DenseInteraction.stress`` / ``seas.prescribed``) on a
ragged three-fault network with a prior history long enough for slip to leave
every pair window, with and without the static tail.

The impulse test pins the window edge of the static tail (Section 2.3.2,
truncation of the elastodynamic time window; the tail itself is the reading
that slip older than a pair's window keeps its static stress): a unit slip-rate
impulse of one step on one source element must be seen through the dynamic
kernel for lags T_init..T_end, and from lag T_end + 1 on as exactly dt times the
static dislocation stress, with no lag counted twice or dropped.
"""
import numpy as np
import pytest

import seas_inputs as SI
from oracle import geometry, interaction as I, seas as OS

RAG = [SI.fault(0, 0, 5.0, 1300.0, 13), SI.fault(300.0, 900.0, 70.0, 2900.0, 29),
       SI.fault(-1500.0, 2200.0, 140.0, 2000.0, 40)]


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def rag():
    p = SI.default_params(eta_H=1.5, leaf=5)
    prob = OS.Problem(RAG, p)
    prior = SI.prescribed_slip_rate(RAG, 90, 8, lo_exp=-6, hi_exp=0)
    V = SI.prescribed_slip_rate(RAG, 140, 7, lo_exp=-6, hi_exp=0)
    return prob, prior, V


@pytest.mark.parametrize("tail", [1, 0])
@pytest.mark.parametrize("min_lag", [0, 1])
def test_stress_rows_equals_dense_sum(rag, tail, min_lag):
    prob, prior, V = rag
    Vall = np.concatenate([prior, V])
    first = -len(prior)
    rows = list(range(prob.N))
    # slip has left some pair windows at the later heads (and not at the first)
    assert min(P["T1"] for P in prob.inter.pairs.values()) < 139 + len(prior) - 1
    for head in (-40, 5, 77, 139):
        exp = prob.inter.expired_slip(Vall, head, first, prob.dt) if tail else None
        ref = prob.inter.stress(Vall, head, first, min_lag=min_lag, expired=exp)
        got = I.stress_rows(prob.geo, rows, Vall, head, first, prob.mu, prob.cs, prob.dt,
                            min_lag=min_lag, with_tail=bool(tail))
        assert _rel(got, ref) < 1e-13, (head, _rel(got, ref))
        if tail and head == 139:
            # the static tail is a visible part of the sum at these heads
            plain = prob.inter.stress(Vall, head, first, min_lag=min_lag)
            assert _rel(plain, ref) > 1e-3


def test_prescribed_rows_equals_prescribed(rag):
    prob, prior, V = rag
    n_steps = 60
    ref = OS.prescribed(prob, V[:n_steps], prior_V=prior)
    Vall = np.concatenate([prior, V[:n_steps]])
    rows = [0, 6, 12, 13, 27, 41, 42, 60, 81]
    for n in (1, 2, 17, 60):
        got = OS.prescribed_rows(prob, Vall, -len(prior), n, rows)
        assert _rel(got, ref[n - 1][rows]) < 1e-12, n


@pytest.mark.parametrize("m0,first", [(0, 0), (-5, -12)])
def test_tail_impulse_hands_over_at_window_edge(m0, first):
    # two faults of the prescribed-history geometry (coarse mesh), every pair
    geo_f = SI.two_fault_prescribed_faults(n_elem=12, dx=400.0)
    p = SI.default_params()
    prob = OS.Problem(geo_f, p)
    eta = prob.mu / (2 * prob.cs)
    off = prob.off
    for (a, b), P in prob.inter.pairs.items():
        T0, T1 = P["T0"], P["T1"]
        G = I.static_dipole(prob.geo, a, b, prob.mu)
        for jj in (0, 7):
            j = off[b] + jj
            last_head = m0 + T1 + 6
            Vh = np.zeros((last_head - first + 1, prob.N))
            Vh[m0 - first, j] = 1.0
            ra = slice(off[a], off[a + 1])
            for head in range(m0, last_head + 1):
                T = head - m0
                exp = prob.inter.expired_slip(Vh, head, first, prob.dt)
                f = prob.inter.stress(Vh, head, first, expired=exp)[ra]
                if T < T0:
                    assert np.all(f == 0.0), (a, b, T)
                elif T <= T1:
                    K = I.pair_kernel(prob.geo, a, b, T, prob.dt, prob.cs)[:, jj]
                    assert np.allclose(f, -eta * K, rtol=1e-14, atol=0.0), (a, b, T)
                    assert np.all(exp[(a, b)] == 0.0)
                else:
                    # exactly dt of slip has expired, once: the static stress of a
                    # dislocation of that size
                    assert exp[(a, b)][jj] == prob.dt and np.count_nonzero(exp[(a, b)]) == 1
                    assert np.allclose(f, G[:, jj] * prob.dt, rtol=1e-14, atol=0.0), (a, b, T)
            # the row-sampled sum agrees at the two heads around the edge
            for head in (m0 + T1, m0 + T1 + 1):
                exp = prob.inter.expired_slip(Vh, head, first, prob.dt)
                ref = prob.inter.stress(Vh, head, first, expired=exp)[ra]
                got = I.stress_rows(prob.geo, list(range(off[a], off[a + 1])), Vh, head, first,
                                    prob.mu, prob.cs, prob.dt)
                assert np.allclose(got, ref, rtol=1e-13, atol=1e-30 + 1e-13 * np.abs(ref).max())


def test_static_tail_is_the_late_kernel_limit_at_every_receiver():
    # The tail's stress per unit expired slip is the limit of the dynamic kernel
    # per unit time: -mu/(2cs) K^T / dt -> G, the O(T^-2) approach of the 2-D kernel.
    g = geometry.discretize(RAG)
    dt = geometry.time_step(g, SI.CS)
    for a, b in ((0, 1), (2, 0), (1, 2)):
        G = I.static_dipole(g, a, b, SI.MU)
        K = I.pair_kernel(g, a, b, 20000, dt, SI.CS)
        assert _rel(-SI.MU / (2 * SI.CS) * K / dt, G) < 1e-3


def test_step_fault_equals_dense_step():
    # Section 2.4 step restricted to one fault (the large-network form): the same
    # V, theta, delta as the dense SeasState step on every fault of a crossing
    # network with lag-0 coupling, a prior history and the static tail.
    faults = [SI.fault(0.0, 0.0, 0.0, 1200.0, 24), SI.fault(110.0, 35.0, 63.0, 1000.0, 20),
              SI.fault(-300.0, 900.0, 150.0, 800.0, 16)]
    p = SI.default_params()
    prob = OS.Problem(faults, p)
    assert any(P["T0"] == 0 for P in prob.inter.pairs.values())        # faults cross
    fric = SI.rate_state_fields(faults)
    ini = SI.near_nucleation_state(faults, fric, seed=4, V_init=1e-5, bump_amp=0.2)
    prior = SI.prescribed_slip_rate(faults, 70, 9, lo_exp=-7, hi_exp=-3)
    eps = np.where(np.arange(prob.N) % 2 == 0, 1.0, 0.6)
    tau0_rate = np.full(prob.N, 1e3)
    dense = OS.SeasState(prob, fric, ini["V"], ini["theta"], ini["tau0"], tau0_rate, prior_V=prior, eps=eps)
    for _ in range(3):
        dense.step()
    # state at n = 3 for the row form
    st = dict(V=dense.V.copy(), theta=dense.theta.copy(), thetadot=dense.thetadot.copy(),
              delta=dense.delta.copy(), tau0=dense.tau0, tau0_rate=dense.tau0_rate, n=dense.n,
              Dh=[(dense.first, np.array(dense.Dh[k])) for k in range(len(faults))])
    Vh = np.array(dense.Vh)
    rows = list(range(prob.N))
    fh = I.stress_rows(prob.geo, rows, Vh, dense.n, dense.first, prob.mu, prob.cs, prob.dt, min_lag=1)
    f_hist = dict(zip(rows, fh))
    dense.step()
    for k in range(len(faults)):
        got = OS.step_fault(prob, fric, st, k, f_hist, eps=eps)
        r = got["rows"]
        for key, ref in (("V", dense.V), ("theta", dense.theta), ("delta", dense.delta)):
            assert _rel(got[key], ref[r]) < 1e-12, (k, key, _rel(got[key], ref[r]))
        assert _rel(got["f_int"], dense.last["f_int"][r]) < 1e-12
        if k == 0:
            assert len(got["partners"]) > 0


# ----------------------------------------------------------------- cluster-level windows
def test_cluster_windows_with_one_block_per_pair_are_the_pair_windows(rag):
    # Section 4.3's cluster-level truncation reduces to the pair rule when a pair
    # is one block (leaves as large as the faults)
    prob, prior, V = rag
    p1 = SI.default_params(eta_H=1.5, leaf=10_000, cluster_windows=1)
    pc = OS.Problem(RAG, p1)
    Vall = np.concatenate([prior, V])
    first = -len(prior)
    for (a, b), P in pc.inter.pairs.items():
        assert len(P["blocks"]) == 1 and P["blocks"][0][4] == P["T1"]
    for head in (5, 139):
        ref = prob.inter.stress(Vall, head, first, expired=prob.inter.expired_slip(Vall, head, first, prob.dt))
        got = pc.inter.stress(Vall, head, first, expired={})
        assert _rel(got, ref) < 1e-14


def test_cluster_windows_shorten_blocks_and_hand_over_per_block():
    # every entry is seen through the dynamic kernel up to its block's upper lag and
    # from the next lag on as exactly dt times the static stress of the dislocation
    faults = [SI.fault(0.0, 0.0, 0.0, 2000.0, 20), SI.fault(200.0, 1800.0, 30.0, 1600.0, 16)]
    p = SI.default_params(eta_H=1.5, leaf=4, cluster_windows=1)
    prob = OS.Problem(faults, p)
    eta = prob.mu / (2 * prob.cs)
    off = prob.off
    shortened = 0
    for (a, b), P in prob.inter.pairs.items():
        G = I.static_dipole(prob.geo, a, b, prob.mu)
        shortened += sum(te < P["T1"] for *_, te in P["blocks"])
        for r0, r1, s0, s1, te in P["blocks"][:: max(1, len(P["blocks"]) // 5)]:
            assert P["T0"] <= te <= P["T1"]
            jj = s0
            i = r0
            Vh = np.zeros((te + 4, prob.N))
            Vh[0, off[b] + jj] = 1.0
            for head in (te - 1, te, te + 1, te + 3):
                f = prob.inter.stress(Vh, head, 0, expired={})[off[a] + i]
                if head <= te:
                    K = I.pair_kernel(prob.geo, a, b, head, prob.dt, prob.cs)[i, jj]
                    assert np.isclose(f, -eta * K, rtol=1e-14, atol=0.0)
                else:
                    assert np.isclose(f, G[i, jj] * prob.dt, rtol=1e-14, atol=0.0)
    assert shortened > 0
