"""Pins of the self term's optional static tail, a correction not in the paper (CPU).

The window of eq. "funcational_discretized_form" drops the part of K(n, .) beyond
the cell of lag W_n. With the tail, slip older than the window responds with the
rest of the kernel: F_n gains R_n D_n^{t-W_n-1}, R_n = |k_n| times the integral of
K(n, .) over t >= (W_n + 1/2) dt.

* static limit: slip held for longer than every window gives, with the tail, the
  static stress of the fault computed element by element from the closed-form
  dislocation stress (interaction.static_dipole of the fault with itself),
  converging at second order in the element size for a smooth slip; without the
  tail the windowed self term misses it by ~0.6% at every resolution;
* R_n is the continuation of the cell integrals: R_n(W) - R_n(W') equals the sum
  of the cells W+1..W' (the C helper's quadrature, a different rule);
* the tail term reads the first lag outside the window (t - W_n - 1): a slip
  history constant before the window edge and random inside it gives the
  untruncated sum (cells over a longer window, plus that window's tail);
* far from the window, R_n matches the kernel's large-time expansion
  K(n, t) = (2/pi) sum_m c_m J_m (a t)^-(2m+1), a = n pi cs / L,
  c_m the coefficients of sqrt(1 - y), J_m = int_0^{n pi} u^{2m} cos u du.
"""
import math

import numpy as np
import pytest

import seas_inputs as SI
from oracle import geometry, interaction, selfterm as ST

MU, CS, DX = 3.2e10, 3464.0, 50.0


def _self(Np, tail, eta_w=1.5):
    L = Np * DX
    dt = 0.5 * DX / CS
    return ST.SelfTerm(Np, L, MU, CS, dt, eta_w=eta_w, tail=tail), L, dt


def _static_error(Np, tail):
    st, L, dt = _self(Np, tail)
    x = (np.arange(Np) + 0.5) / Np
    slip = np.sin(np.pi * x) ** 4
    D = st.dft(slip)
    Dh = np.tile(D, (st.reach + 2, 1))            # the same slip for longer than every window
    t = st.reach + 1
    f = st.stress(Dh, t, 0)
    geo = geometry.discretize([SI.fault(0.0, 0.0, 0.0, L, Np)])
    ref = interaction.static_dipole(geo, 0, 0, MU) @ slip
    return float(np.abs(f - ref).max() / np.abs(ref).max())


def test_static_limit_is_the_static_stress():
    e32, e64 = _static_error(32, True), _static_error(64, True)
    assert e64 < 1e-3
    assert 3.0 < e32 / e64 < 5.5                      # second order in the element size
    # the literal window misses the static level by a resolution-independent amount
    n32, n64 = _static_error(32, False), _static_error(64, False)
    assert n32 > 4e-3 and n64 > 4e-3 and n64 > 0.8 * n32


@pytest.mark.parametrize("n", [1, 2, 7, 32])
def test_tail_continues_the_cells(n):
    Np = 32
    st, L, dt = _self(Np, True)
    W = int(st.W[n - 1])
    W2 = W + 300                                      # past t = L/cs for every mode here
    cells = n * math.pi / L * ST.K_cells(n, W2, dt, L, CS)
    R1 = st.R[n - 1]
    R2 = n * math.pi / L * ST.K_tail_integral(n, (W2 + 0.5) * dt, L, CS)
    assert R1 == pytest.approx(R2 + cells[W + 1:].sum(), rel=1e-11, abs=1e-15 * abs(cells).max())


def test_tail_reads_the_first_lag_outside_the_window():
    Np = 16
    st, L, dt = _self(Np, True)
    big, _, _ = _self(Np, True, eta_w=4.0)          # same cells, longer windows
    assert np.all(big.W > st.W + 2)
    rng = np.random.default_rng(5)
    t = int(big.W.max()) + 5
    Dc = st.dft(rng.standard_normal(Np))
    Dh = np.tile(Dc, (t + 1, 1)).astype(complex)
    F = st.modal_stress(Dh, t, 0)                    # placeholder to size the output
    for i, n in enumerate(st.modes):
        W = int(st.W[i])
        hist = np.tile(Dc, (t + 1, 1)).astype(complex)
        for m in range(t - W, t + 1):                 # random inside the window only
            hist[m] = st.dft(rng.standard_normal(Np))
        got = st.modal_stress(hist, t, 0)[n]
        Kb = big.table(i)
        Wb = int(big.W[i])
        brute = sum(Kb[T] * hist[t - T, n] for T in range(Wb + 1)) + big.R[i] * hist[t - Wb - 1, n]
        ref = -(MU * CS * st.k[i] / 2.0) * brute
        assert abs(got - ref) <= 1e-11 * abs(ref), (n, got, ref)
    assert F.shape == (Np + 1,)


def _series_tail(n, t0, L):
    # (2/pi) sum_{m>=1} c_m J_m / (2m a^{2m+1} t0^{2m}), the large-time expansion integrated
    a = n * math.pi * CS / L
    X = n * math.pi
    cosX = -1.0 if n % 2 else 1.0
    C, S = [0.0], [1.0 - cosX]                        # int_0^X u^k cos u, sin u du, k = 0
    for k in range(1, 9):
        C.append(-k * S[k - 1])                       # sin X = 0
        S.append(-X ** k * cosX + k * C[k - 1])
    c = [1.0, -0.5, -0.125, -0.0625, -5.0 / 128.0]
    return 2.0 / math.pi * sum(c[m] * C[2 * m] / (2 * m * a ** (2 * m + 1) * t0 ** (2 * m)) for m in range(1, 5))


@pytest.mark.parametrize("n", [1, 3, 8])
def test_tail_far_from_the_window_is_the_large_time_expansion(n):
    L = 32 * DX
    t0 = 20.0 * L / CS
    got = ST.K_tail_integral(n, t0, L, CS)
    ref = _series_tail(n, t0, L)
    assert got == pytest.approx(ref, rel=1e-8)
    assert got != 0.0
