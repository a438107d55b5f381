"""Pins of the oracle's interaction kernel, windows and static tail (CPU only).

Each test checks the oracle against something other than its own formulas:
printed numbers of the paper's two-fault benchmark, textbook closed forms
(static screw-dislocation stresses), invariants (causality, the radiation-damping
value of the lag-0 self entry, coplanar symmetry, reciprocity) and limits.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import geometry, interaction as I
import seas_inputs as SI

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _single(n=12, L=1200.0):
    return geometry.discretize([SI.fault(0.0, 0.0, 0.0, L, n)])


def test_lag0_self_entry_is_radiation_damping():
    # Classical self-block at lag 0: K^0_ii = 1, i.e. -mu/(2cs) V (Section 2.3,
    # radiation damping); the wave has not reached any neighbour yet.
    g = _single()
    cs = SI.CS
    dt = geometry.time_step(g, cs)
    r1, r2, n1, n2 = I.local_offsets(g, 0, 0)
    K0 = I.kernel_from_offsets(r1, r2, n1, n2, g[0].dx, 0, dt, cs)
    assert np.allclose(np.diag(K0), 1.0, atol=0, rtol=0)
    assert np.abs(K0 - np.diag(np.diag(K0))).max() == 0.0


def test_static_self_stiffness_closed_form():
    # Uniform slip on one element: stress at its own centre is -2 mu / (pi ds)
    # (two screw dislocations at distance ds/2).
    g = _single()
    G = I.static_dipole(g, 0, 0, SI.MU)
    assert np.allclose(np.diag(G), -2 * SI.MU / (math.pi * g[0].dx), rtol=1e-14)


def test_loading_ahead_of_slipping_element():
    g = _single(n=20)
    G = I.static_dipole(g, 0, 0, SI.MU)
    i = 10
    off = np.arange(20) != i
    assert np.all(G[off, i] > 0)          # every other element on the line is loaded
    # textbook magnitude on the line: (mu/2pi) ds / (x^2 - ds^2/4)
    x = (np.arange(20) - i) * g[0].dx
    ds = g[0].dx
    ref = SI.MU / (2 * math.pi) * ds / (x[off] ** 2 - ds * ds / 4)
    assert np.allclose(G[off, i], ref, rtol=1e-12)


@pytest.mark.parametrize("geom", ["twofault", "offplane"])
def test_dynamic_kernel_tends_to_static_dipole(geom):
    # -mu/(2cs) K^T / dt -> G (static) with an O(T^-2) remainder.
    if geom == "twofault":
        faults = SI.two_fault_prescribed_faults(n_elem=16, dx=100.0)
    else:
        faults = [SI.fault(0, 0, 0, 1600.0, 16), SI.fault(300.0, 2500.0, 55.0, 1200.0, 12)]
    g = geometry.discretize(faults)
    cs, mu = SI.CS, SI.MU
    dt = geometry.time_step(g, cs)
    G = I.static_dipole(g, 0, 1, mu)
    errs = []
    for T in (400, 4000):
        K = I.pair_kernel(g, 0, 1, T, dt, cs)
        errs.append(np.abs(-mu / (2 * cs) * K / dt - G).max() / np.abs(G).max())
    assert errs[1] < 2e-4                 # ~ (r / cs t)^2 at T = 4000
    assert errs[0] / errs[1] > 50          # ~100x for a 10x larger lag


def test_causality_zero_before_first_arrival():
    # No entry may be nonzero before a wave from the nearest point of the source
    # element can arrive: K^T_ij = 0 whenever (T+1) dt cs <= dist(x_i, segment j).
    faults = [SI.fault(0, 0, 0, 1600.0, 16), SI.fault(300.0, 900.0, 35.0, 1200.0, 12)]
    g = geometry.discretize(faults)
    cs = SI.CS
    dt = geometry.time_step(g, cs)
    A, B = g[0], g[1]
    # distance from receiver midpoints to source segments (brute force sampling)
    s = np.linspace(-0.5, 0.5, 2001) * B.dx
    pts = B.mid[:, None, :] + s[None, :, None] * B.t[None, None, :]
    d = np.sqrt(((A.mid[:, None, None, :] - pts[None]) ** 2).sum(-1)).min(-1)
    for T in range(0, 30):
        K = I.pair_kernel(g, 0, 1, T, dt, cs)
        silent = (T + 1) * dt * cs <= d - 1e-6 * B.dx
        assert np.all(K[silent] == 0.0)
        late = T * dt * cs > d + B.dx
        if late.any():
            assert np.any(K[late] != 0.0)


def test_coplanar_kernel_is_symmetric_toeplitz():
    # Two collinear faults with the same normal: K^T depends only on the
    # receiver-source offset and is even in it.
    faults = [SI.fault(0, 0, 0, 800.0, 8), SI.fault(1600.0, 0, 0, 800.0, 8)]
    g = geometry.discretize(faults)
    cs = SI.CS
    dt = geometry.time_step(g, cs)
    for T in (5, 17, 40):
        K01 = I.pair_kernel(g, 0, 1, T, dt, cs)
        K10 = I.pair_kernel(g, 1, 0, T, dt, cs)
        # K10[j, i] sees the mirrored offset y_j - x_i of K01[i, j]
        assert np.allclose(K01, K10.T, rtol=1e-12, atol=1e-15)
        # Toeplitz: constant along diagonals
        for k in range(-7, 8):
            dg = np.diagonal(K01, k)
            assert np.allclose(dg, dg[0], rtol=1e-11, atol=1e-14)


def test_static_reciprocity():
    # Betti: G_ij(a<-b) ds_a ~= G_ji(b<-a) ds_b up to O((ds/r)^2) for collocation.
    faults = [SI.fault(0, 0, 10.0, 2000.0, 10), SI.fault(500.0, 9000.0, 70.0, 3000.0, 12)]
    g = geometry.discretize(faults)
    Gab = I.static_dipole(g, 0, 1, SI.MU)
    Gba = I.static_dipole(g, 1, 0, SI.MU)
    lhs, rhs = Gab * g[0].dx, Gba.T * g[1].dx
    rel = np.abs(lhs - rhs).max() / np.abs(lhs).max()
    assert rel < 0.02


def test_two_fault_benchmark_dt_and_window():
    # Section 3.1: dt_min ~ 1.38e-3 s, maximum truncation time T_end ~ 3.76 s.
    gd = json.load(open(os.path.join(GOLD, "two_fault_benchmark.json")))
    g = geometry.discretize(gd["faults"])
    dt = geometry.time_step(g, gd["cs"], gd["beta"])
    assert round(dt, 5) == gd["printed_dt_min"]
    tmax = max(I.pair_window_times(g, a, b, gd["cs"], gd["eta_tmin"], gd["eta_tmax"])[1]
               for a, b in ((0, 1), (1, 0)))
    # "~3.76 s": within 0.3% (dropping the (1 + eta_Tmax) factor would be 1% off)
    assert abs(tmax - gd["printed_T_end"]) / gd["printed_T_end"] < 3e-3


def test_windows_bracket_nonzero_lags_two_fault_prescribed():
    # Lags before T_init carry no signal for the prescribed-history workload
    # geometry, and T_end is past the last lag that workload reaches.
    faults = SI.two_fault_prescribed_faults()
    g = geometry.discretize(faults)
    cs = SI.CS
    dt = geometry.time_step(g, cs)
    for a, b in ((0, 1), (1, 0)):
        T0, T1 = I.pair_window_lags(g, a, b, cs, dt, 0.01, 0.01)
        assert T1 >= 256
        for T in range(0, T0):
            assert np.all(I.pair_kernel(g, a, b, T, dt, cs) == 0.0)
