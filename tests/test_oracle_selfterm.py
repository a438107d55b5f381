"""Pins of the oracle's spectral self term (CPU only).

Closed forms: K(n, t) = J1(x)/x before the wave reaches the fault end (the
psi-average of cos^2 psi cos(x sin psi)), K(n, 0) = 1/2, the late-time asymptote
-2 n (-1)^n / x^3, the time integral int_0^inf K dt = 2 L Si(n pi) / (pi^2 n cs).
Library special cases: the explicit DFT equals numpy's rfft of the padded slip.
Physics: the spectral self term agrees at the percent level with the classical
space-time self block built from the interaction primitives.
"""
import math

import numpy as np
import pytest
from scipy.special import j1, sici

from oracle import geometry, interaction as I, selfterm as S
import seas_inputs as SI

L, CS = 12800.0, SI.CS


@pytest.mark.parametrize("n", [1, 2, 7, 40, 128])
def test_early_kernel_is_bessel(n):
    lib = S._lib()
    for frac in (0.0001, 0.03, 0.3, 0.77, 0.999):
        t = frac * L / CS
        x = n * math.pi * CS * t / L
        assert abs(lib.oracle_K_mode(n, t, L, CS) - j1(x) / x) < 5e-14


def test_kernel_at_zero_and_continuity():
    lib = S._lib()
    for n in (1, 3, 10):
        assert lib.oracle_K_mode(n, 0.0, L, CS) == pytest.approx(0.5, abs=1e-15)
        tl = L / CS
        a = lib.oracle_K_mode(n, tl * (1 - 1e-14), L, CS)
        b = lib.oracle_K_mode(n, tl * (1 + 1e-14), L, CS)
        assert abs(a - b) < 1e-13


@pytest.mark.parametrize("n", [1, 2, 5, 11])
def test_late_kernel_asymptote(n):
    lib = S._lib()
    for m in (20.0, 60.0):
        t = m * L / CS
        x = n * math.pi * CS * t / L
        ref = -2.0 * n * (-1) ** n / x ** 3
        assert lib.oracle_K_mode(n, t, L, CS) / ref == pytest.approx(1.0, abs=4.0 / m ** 2)


@pytest.mark.parametrize("n", [1, 2, 3, 8])
def test_time_integral_closed_form(n):
    # sum over centred cells covering [0, T_big dt] -> 2 L Si(n pi) / (pi^2 n cs)
    dt = 0.5 * 100.0 / CS
    W = 40000
    cells = S.K_cells(n, W, dt, L, CS)
    ref = 2 * L * sici(n * math.pi)[0] / (math.pi ** 2 * n * CS)
    # remaining tail beyond (W+1/2) dt is O(1/x^2): bound it by the asymptote
    xb = n * math.pi * CS * (W + 0.5) * dt / L
    tail = n * L / (n * math.pi * CS) / xb ** 2
    assert abs(cells.sum() - ref) < 2 * tail + 1e-12


def test_c_helper_matches_numpy_rule():
    dt = 0.5 * 100.0 / CS
    for n in (1, 4, 9):
        W = S.mode_window(n, 128, L, CS, dt, 1.5, 26)
        c = S.K_cells(n, W, dt, L, CS)
        p = S.K_cells_numpy(n, W, dt, L, CS)
        assert np.abs(c - p).max() < 1e-15


def test_windows():
    dt = 0.5 * 100.0 / CS
    # W_1 = eta_w L / (cs dt) = 1.5 * 256 = 384 for 128 x 100 m
    assert S.mode_window(1, 128, L, CS, dt, 1.5, 26) == 384
    # q_w = N_p/2 gives L(n) = 1: every mode keeps the lowest mode's window
    assert all(S.mode_window(n, 128, L, CS, dt, 1.5, 64) == 384 for n in range(1, 129))
    # q_w = 1 gives T_end(n) = T_end(1)/n
    assert S.mode_window(4, 128, L, CS, dt, 1.5, 1) == 96
    w = [S.mode_window(n, 128, L, CS, dt, 1.5, 26) for n in range(1, 129)]
    assert all(a >= b for a, b in zip(w, w[1:]))


def test_dft_is_padded_rfft():
    rng = np.random.default_rng(3)
    st = S.SelfTerm(24, 2400.0, SI.MU, CS, 0.5 * 100 / CS, use_c=True)
    d = rng.standard_normal(24)
    D = st.dft(d)
    ref = np.fft.rfft(np.concatenate([d, np.zeros(24)]))
    assert np.abs(D - ref).max() < 1e-13
    # inverse of a Hermitian spectrum: irfft of the full 2N_p spectrum, first N_p samples
    F = rng.standard_normal(25) + 1j * rng.standard_normal(25)
    F[0] = F[0].real
    F[24] = F[24].real
    f = st.idft(F)
    assert np.abs(f - np.fft.irfft(F, 48)[:24]).max() < 1e-13


@pytest.mark.slow
def test_spectral_vs_classical_self_block():
    # A smooth slip-rate history on one fault: the spectral self term (displacement
    # form, centred cells, long windows) matches the classical space-time self block
    # minus its lag-0 radiation-damping diagonal at the percent level.
    Np, dx = 64, 100.0
    f = SI.fault(0, 0, 0, Np * dx, Np)
    g = geometry.discretize([f])
    dt = geometry.time_step(g, CS)
    st = S.SelfTerm(Np, Np * dx, SI.MU, CS, dt, eta_w=4.0, q_w=Np // 2)
    n_steps = 200
    xi = g[0].xi / (Np * dx)
    tt = np.arange(n_steps)[:, None] / n_steps
    V = np.exp(-((xi[None, :] - 0.1 * np.sin(3 * tt)) / 0.18) ** 2) * (0.2 + tt)
    delta = np.vstack([np.zeros(Np), np.cumsum(V, axis=0) * dt])
    Dh = np.array([st.dft(d) for d in delta])
    r1, r2, n1, n2 = I.local_offsets(g, 0, 0)
    Kst = np.array([I.kernel_from_offsets(r1, r2, n1, n2, g[0].dx, T, dt, CS) for T in range(n_steps)])
    eta = SI.MU / (2 * CS)
    errs = []
    for n in range(60, n_steps, 20):
        fs = st.stress(Dh, n, 0)
        fc = -eta * np.einsum("tij,tj->i", Kst[:n], V[n - 1::-1][:n]) + eta * V[n - 1]
        errs.append(np.abs(fs - fc).max() / np.abs(fc).max())
    assert max(errs) < 1e-2
