"""Non-replicating spectral self term (oracle).

Section 2.3.1 of the paper, followed step by step:

* slip sampled at the N_p element midpoints, zero-padded to the period 2L
  (M = 2 N_p samples), expanded in Fourier modes k_n = pi n / L;
* each mode is convolved in time with K(n, t) (eq. "non_replicant_kernel"),
  F_n = -(mu cs k_n^2 / 2) (K(n, .) * D_n), discretised with the fixed step dt as
  F_n^t = -(pi mu cs n / (2L)) sum_{T=0}^{W_n} K_n^T D_n^{t-T}
  (eq. "funcational_discretized_form"), where K_n^T = |k_n| times the integral of
  K(n, .) over the centred time cell of lag T (the paper calls the kernel
  "pre-integrated" without giving the rule; the centred cell is the reading
  taken here);
* mode-dependent windows T_end(n) = T_end(1) L(n), T_end(1) = eta_w L / cs
  (eq. "mode_dependent_truncation");
* the transforms are explicit sums (no FFT): D_n = sum_j delta_j e^{-2 pi i n j / M},
  n = 0..N_p, and the inverse keeps the real part of the Hermitian sum;
* optional static tail of the truncated kernel (a correction, not in the paper):
  the window drops the part of K(n, .) beyond the cell of lag W_n,
  which carries static response; with ``tail=True`` each mode adds
  R_n D_n^{t-W_n-1}, R_n = |k_n| times the integral of K(n, .) over
  t >= (W_n + 1/2) dt, i.e. slip older than the window responds with the rest
  of the kernel. The full integral is finite (K decays as t^-3 for integer n),
  and with it a slip held long enough gives the static stress of the fault.
  Pins: that static limit against the element-wise static stress (second order
  in the element size), R_n against the cell integrals it continues and against
  the kernel's large-time expansion (tests/test_oracle_selftail.py).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _gl(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def K_mode(n, t, L, cs):
    """K(n, t) by quadrature of its psi-integral (numpy, vectorised over t)."""
    t = np.atleast_1d(np.asarray(t, float))
    out = np.empty_like(t)
    gx, gw = _gl(20)
    for k, tk in enumerate(t):
        x = n * math.pi * cs * tk / L
        if cs * tk < L:
            m = 4 * int(math.ceil((abs(x) + 20.0 * abs(x) ** (1.0 / 3.0) + 48.0) / 4.0))
            psi = 2 * math.pi * np.arange(m) / m
            out[k] = np.mean(np.cos(psi) ** 2 * np.cos(x * np.sin(psi)))
        else:
            psim = math.asin(L / (cs * tk))
            panels = n // 2 + 4
            h = psim / panels
            mids = (np.arange(panels) + 0.5) * h
            psi = (mids[:, None] + 0.5 * h * gx[None, :]).ravel()
            w = np.tile(0.5 * h * gw, panels)
            out[k] = 2.0 / math.pi * np.sum(w * np.cos(psi) ** 2 * np.cos(x * np.sin(psi)))
    return out


def K_cells_numpy(n, W, dt, L, cs):
    """Integral of K(n, .) over the centred cells [max(0,(T-1/2)dt), (T+1/2)dt],
    T = 0..W (Gauss-Legendre in t, split at t = L/cs, with t = L/cs + D s^2 on
    the late side)."""
    gx, gw = _gl(20)
    tl = L / cs
    out = np.zeros(W + 1)
    for T in range(W + 1):
        t0, t1 = max(0.0, (T - 0.5) * dt), (T + 0.5) * dt
        s = 0.0
        if t0 < tl:
            b = min(t1, tl)
            h = b - t0
            s += np.sum(0.5 * h * gw * K_mode(n, 0.5 * (t0 + b) + 0.5 * h * gx, L, cs))
        if t1 > tl:
            a = max(t0, tl)
            if a > tl:
                h = t1 - a
                s += np.sum(0.5 * h * gw * K_mode(n, 0.5 * (a + t1) + 0.5 * h * gx, L, cs))
            else:
                D = t1 - tl
                sn = 0.5 * (1 + gx)
                s += np.sum(0.5 * gw * 2 * D * sn * K_mode(n, tl + D * sn * sn, L, cs))
        out[T] = s
    return out


def _K_early_integral(n, t0, t1, L, cs):
    """Integral of K(n, t) over [t0, t1] inside t <= L/cs (Gauss-Legendre panels,
    about two per oscillation of K)."""
    if t1 <= t0:
        return 0.0
    gx, gw = _gl(20)
    edges = np.linspace(t0, t1, n + 5)
    s = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        h = b - a
        s += np.sum(0.5 * h * gw * K_mode(n, 0.5 * (a + b) + 0.5 * h * gx, L, cs))
    return s


def _K_late_integral(n, t1, L, cs):
    """Integral of K(n, t) over t >= t1 >= L/cs. With t = L / (cs sin phi), the
    late branch of the definition reads K = (2/pi) int_0^phi cos^2 psi
    cos((n pi / sin phi) sin psi) dpsi and dt = (L/cs) cos phi / sin^2 phi dphi;
    K ~ t^-3 makes the integrand vanish like sin phi at phi = 0, so the infinite
    range becomes the finite, smooth phi in (0, asin(L / (cs t1))]."""
    gx, gw = _gl(20)
    phi1 = math.asin(min(1.0, L / (cs * t1)))
    edges = np.linspace(0.0, phi1, n + 9)
    h = edges[1] - edges[0]
    phi = ((0.5 * (edges[:-1] + edges[1:]))[:, None] + 0.5 * h * gx[None, :]).ravel()
    wphi = np.tile(0.5 * h * gw, len(edges) - 1)
    # inner psi-integral for every phi at once: psi = phi * u, u in [0, 1]
    ip = n // 2 + 4
    ue = np.linspace(0.0, 1.0, ip + 1)
    uh = ue[1] - ue[0]
    u = ((0.5 * (ue[:-1] + ue[1:]))[:, None] + 0.5 * uh * gx[None, :]).ravel()
    wu = np.tile(0.5 * uh * gw, ip)
    psi = phi[:, None] * u[None, :]
    x = n * math.pi / np.sin(phi)
    K = 2.0 / math.pi * phi * ((np.cos(psi) ** 2 * np.cos(x[:, None] * np.sin(psi))) @ wu)
    return (L / cs) * float(np.sum(wphi * K * np.cos(phi) / np.sin(phi) ** 2))


def K_tail_integral(n, t0, L, cs):
    """Integral of K(n, t) over t >= t0 (the part a window ending at t0 drops)."""
    tl = L / cs
    return _K_early_integral(n, t0, tl, L, cs) + _K_late_integral(n, max(t0, tl), L, cs)


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "_selfkernel.so")
        if not os.path.exists(path):
            build_helper()
        lib = ctypes.CDLL(path)
        lib.oracle_K_table.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_void_p]
        lib.oracle_K_mode.restype = ctypes.c_double
        lib.oracle_K_mode.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        _LIB = lib
    return _LIB


def K_cells(n, W, dt, L, cs):
    """Cell integrals of K(n, .) for T = 0..W through the C helper (same rule as
    ``K_cells_numpy``)."""
    modes = np.array([n], dtype=np.int32)
    Ws = np.array([W], dtype=np.int32)
    offs = np.array([0], dtype=np.int64)
    out = np.zeros(W + 1)
    _lib().oracle_K_table(1, modes.ctypes.data, Ws.ctypes.data, offs.ctypes.data,
                          float(dt), float(L), float(cs), out.ctypes.data)
    return out


def build_helper():
    """Compile the plain-C quadrature helper with gcc (no GPU code involved)."""
    import subprocess
    src = os.path.join(_HERE, "csrc", "selfkernel.c")
    out = os.path.join(_HERE, "_selfkernel.so")
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, out)


def mode_window(n, Np, L, cs, dt, eta_w, q_w):
    """W_n = floor(T_end(n) / dt), T_end(n) = eta_w (L/cs) L(n),
    L(n) = 1/|n| + (q_w - 1)/(N_p/2 - 1) (1 - 1/|n|).  A relative 1e-12 guard keeps
    values that are integers in exact arithmetic from rounding down."""
    if Np / 2.0 - 1.0 <= 0.0:      # N_p <= 2: the only admissible q_w is N_p/2, L(n) = 1
        Ln = 1.0
    else:
        Ln = 1.0 / n + (q_w - 1.0) / (Np / 2.0 - 1.0) * (1.0 - 1.0 / n)
    return int(math.floor(eta_w * (L / cs) * Ln / dt * (1.0 + 1e-12)))


def default_qw(Np):
    return int(round(Np / 5.0))


class SelfTerm:
    """Self-term tables of one fault: windows W_n and K_n^T for n = 1..N_p."""

    def __init__(self, Np, L, mu, cs, dt, eta_w=1.5, q_w=0, mode_cap=0, use_c=True, tail=False):
        self.Np, self.L, self.mu, self.cs, self.dt = Np, L, mu, cs, dt
        self.M = 2 * Np
        q = q_w if q_w > 0 else default_qw(Np)
        self.q_w = q
        nmax = Np if mode_cap <= 0 else min(mode_cap, Np)
        self.modes = np.arange(1, nmax + 1)
        self.W = np.array([mode_window(n, Np, L, cs, dt, eta_w, q) for n in self.modes], dtype=np.int32)
        self.k = math.pi * self.modes / L
        offs = np.concatenate([[0], np.cumsum(self.W + 1)]).astype(np.int64)
        self.offs = offs
        flat = np.zeros(int(offs[-1]))
        if use_c:
            lib = _lib()
            m32 = self.modes.astype(np.int32)
            lib.oracle_K_table(len(m32), m32.ctypes.data, self.W.ctypes.data, offs.ctypes.data,
                               dt, L, cs, flat.ctypes.data)
        else:
            for i, n in enumerate(self.modes):
                flat[offs[i]:offs[i + 1]] = K_cells_numpy(int(n), int(self.W[i]), dt, L, cs)
        # K_n^T = |k_n| * cell integral
        for i in range(len(self.modes)):
            flat[offs[i]:offs[i + 1]] *= self.k[i]
        self.flat = flat
        # static tail of each mode: R_n = |k_n| int_{(W_n + 1/2) dt}^inf K(n, t) dt
        self.tail = bool(tail)
        self.R = np.zeros(len(self.modes))
        if self.tail:
            for i, n in enumerate(self.modes):
                self.R[i] = self.k[i] * K_tail_integral(int(n), (self.W[i] + 0.5) * dt, L, cs)
        # oldest lag whose coefficients the stress reads
        self.reach = int(self.W.max()) + (1 if self.tail else 0) if len(self.W) else 0

    def table(self, i):
        return self.flat[self.offs[i]:self.offs[i + 1]]

    # ---------------------------------------------------------------- transforms
    def dft(self, delta):
        """D_n = sum_{j<N_p} delta_j exp(-2 pi i n j / M), n = 0..N_p (explicit sum);
        ``delta`` may hold several slip vectors as rows."""
        if getattr(self, "_E", None) is None:
            n = np.arange(self.Np + 1)[:, None]
            j = np.arange(self.Np)[None, :]
            self._E = np.exp(-2j * math.pi * ((n * j) % self.M) / self.M)
        d = np.asarray(delta, float)
        return (self._E @ d.T).T if d.ndim == 2 else self._E @ d

    def idft(self, F):
        """f_j = (1/M) [F_0 + 2 Re sum_{n=1}^{N_p-1} F_n e^{2 pi i n j/M} + Re F_{N_p} (-1)^j]."""
        Np, M = self.Np, self.M
        j = np.arange(Np)[:, None]
        n = np.arange(1, Np)[None, :]
        E = np.exp(2j * math.pi * ((n * j) % M) / M)
        f = F[0].real + 2.0 * (E @ F[1:Np]).real + F[Np].real * np.where(np.arange(Np) % 2 == 0, 1.0, -1.0)
        return f / M

    # ---------------------------------------------------------------- stress
    def modal_stress(self, Dh, t, first, D_now=None):
        """F_n = -(mu cs |k_n| / 2) (sum_{T=0}^{W_n} K_n^T D_n^{t-T} [+ R_n D_n^{t-W_n-1}]).

        ``Dh[m - first]`` holds D^m (length N_p+1) for m >= first; earlier
        coefficients are zero (no slip history).  When ``D_now`` is given it is
        used as D^t (the T = 0 term) instead of the stored row. The bracketed
        static tail is added when the table was built with ``tail=True``."""
        F = np.zeros(self.Np + 1, dtype=complex)
        for i, n in enumerate(self.modes):
            Kt = self.table(i)
            W = int(self.W[i])
            ms = t - np.arange(W + 1)
            ok = ms >= first
            if D_now is not None:
                ok[0] = False
            vals = Dh[ms[ok] - first, n] if ok.any() else np.zeros(0, complex)
            s = np.dot(Kt[ok], vals)
            if D_now is not None:
                s = s + Kt[0] * D_now[n]
            if self.tail and t - W - 1 >= first:
                s = s + self.R[i] * Dh[t - W - 1 - first, n]
            F[n] = -(self.mu * self.cs * self.k[i] / 2.0) * s
        return F

    def stress(self, Dh, t, first, D_now=None):
        return self.idft(self.modal_stress(Dh, t, first, D_now))
