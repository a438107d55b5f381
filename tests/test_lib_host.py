"""CPU checks of the C-ABI library (no GPU): it loads, exports every function
include/seas.h declares, and its host-side build (windows, H-matrix partition,
self-kernel tables, per-lag factors) agrees with the oracle.  Operators here are
built with host_only = 1, which keeps everything on the host."""
import math
import os
import re

import numpy as np
import pytest

import seas_inputs as SI
from oracle import geometry, hpartition as HP, interaction as I, selfterm as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

P = pytest.importorskip("paper_2603_00383_amd")


def _lib_or_skip():
    try:
        return P.lib()
    except (RuntimeError, OSError) as e:
        pytest.skip(f"library not built: {e}")


def test_exports_every_declared_symbol():
    L = _lib_or_skip()
    hdr = open(os.path.join(ROOT, "include", "seas.h")).read()
    names = set(re.findall(r"\b(seas_[a-z_0-9]+)\s*\(", hdr))
    assert len(names) >= 20
    for n in sorted(names):
        assert hasattr(L, n), n


def _op(faults, **kw):
    _lib_or_skip()
    p = SI.default_params(host_only=1, **kw)
    return P.Operator(faults, p)


def test_windows_and_partition_match_oracle():
    faults = SI.two_fault_prescribed_faults()
    for seed_faults in (faults, SI.five_fault_network(seed=1, n_elem=64)):
        op = _op(seed_faults, eta_H=2.0, leaf=16)
        geo = geometry.discretize(seed_faults)
        dt = geometry.time_step(geo, SI.CS)
        assert op.info["dt"] == dt
        win = op.windows()
        blocks = HP.partition(geo, 2.0, 16)
        for (a, b), (t0, t1) in win.items():
            assert (t0, t1) == I.pair_window_lags(geo, a, b, SI.CS, dt, 0.01, 0.01)
            assert op.blocks(a, b) == blocks[(a, b)]


def test_self_tables_match_oracle():
    faults = SI.two_fault_prescribed_faults()
    op = _op(faults)
    geo = geometry.discretize(faults)
    dt = geometry.time_step(geo, SI.CS)
    st = S.SelfTerm(128, 12800.0, SI.MU, SI.CS, dt)
    worst = 0.0
    for n in (1, 2, 3, 17, 64, 127, 128):
        lt = op.self_table(0, n)
        ot = st.table(n - 1)
        assert len(lt) == len(ot)
        worst = max(worst, np.abs(lt - ot).max() / np.abs(ot).max())
    assert worst < 1e-12


def test_self_tail_matches_oracle():
    # the library's tail (exchanged order to 64 max(t0, L/cs), closed-form terms past
    # it) against the oracle's (substitution t = L/(cs sin phi)); the cells unchanged
    faults = SI.two_fault_prescribed_faults(n_elem=48, dx=100.0)
    op = _op(faults, self_tail=1)
    op0 = _op(faults)
    geo = geometry.discretize(faults)
    dt = geometry.time_step(geo, SI.CS)
    st = S.SelfTerm(48, 4800.0, SI.MU, SI.CS, dt, tail=True)
    assert op.info["max_self_window"] == op0.info["max_self_window"] + 1
    for n in (1, 2, 3, 10, 24, 47, 48):
        lt, l0 = op.self_table(0, n), op0.self_table(0, n)
        W = int(st.W[n - 1])
        assert len(lt) == W + 2 and len(l0) == W + 1
        assert np.array_equal(lt[:W + 1], l0)
        # both quadratures reach ~1e-15 absolute (the late-time integrand cancels); that
        # is ~1e-10 of the smallest R_n and ~1e-13 of the mode's whole kernel
        assert abs(lt[W + 1] - st.R[n - 1]) <= 1e-11 * np.abs(l0).sum()
        assert abs(lt[W + 1]) > 1e-3 * np.abs(l0).sum()


@pytest.mark.parametrize("compress,S,dtype", [(0, 1, "f64"), (1, 1, "f64"), (1, 4, "f64"), (0, 16, "f64"),
                                              (0, 16, "f32"), (1, 16, "f32"), (1, 32, "f32")])
def test_lag_matrices_match_dense_kernel(compress, S, dtype):
    # FP32 with S = 16 packs its far list in the segment layout of the matrix-core
    # kernel (inner index fastest, rows padded to 8 values, items grouped by rows)
    faults = SI.two_fault_prescribed_faults(n_elem=64, dx=200.0)
    tol = 1e-6
    op = _op(faults, compress=compress, aca_tol=tol, eta_H=1.0, leaf=16, time_block=S, factor_dtype=dtype)
    assert op.info["time_block"] == S
    if S > 1:
        assert op.info["n_items_near"] > 0
    if dtype == "f32" and S == 16:
        assert op.info["n_segments"] > 0
    exact = 1e-12 if dtype == "f64" else 1e-6  # storage rounding
    geo = geometry.discretize(faults)
    dt = geometry.time_step(geo, SI.CS)
    for (a, b), (t0, t1) in op.windows().items():
        for T in sorted({0, 1, max(t0, 1), t0 + 3, (t0 + t1) // 2, t1}):
            if T < t0 or T > t1:
                continue
            K = I.pair_kernel(geo, a, b, T, dt, SI.CS)
            R = op.lag_matrix(a, b, T, 64, 64)
            nrm = np.linalg.norm(K)
            if nrm == 0:
                assert np.all(R == 0)
                continue
            err = np.linalg.norm(R - K) / nrm
            if T == 0:
                assert err < 1e-12, (a, b, T, err)
            elif compress == 0:
                assert err < exact, (a, b, T, err)
            else:
                assert err < 2 * tol + exact, (a, b, T, err)
        # static tail stored as -G/eta
        G = I.static_dipole(geo, a, b, SI.MU)
        R = op.lag_matrix(a, b, -1, 64, 64)
        eta = SI.MU / (2 * SI.CS)
        assert np.linalg.norm(R + G / eta) / np.linalg.norm(G / eta) < (exact if compress == 0 else 2 * tol + exact)


@pytest.mark.parametrize("dtype,nv,S", [("bf16", 1, 16), ("f16", 1, 16), ("bf16", 16, 1), ("bf16", 64, 1),
                                        ("f16", 16, 1), ("f16", 64, 1)])
def test_16bit_lag_matrices_match_dense_kernel(dtype, nv, S):
    """16-bit factors with per-item power-of-two scales: the reconstructed lag
    matrices are the FP64 kernel to the format's rounding (BF16 keeps 8
    significant bits, FP16 11), plus the ACA tolerance for low-rank blocks. Lags
    below S stay in FP32 (near list); ensembles keep lags below 16, near-field
    blocks and the static tail in FP32 (the one-variant rule)."""
    faults = SI.two_fault_prescribed_faults(n_elem=64, dx=200.0)
    op = _op(faults, compress=1, aca_tol=1e-6, eta_H=1.0, leaf=16, time_block=S, factor_dtype=dtype,
             n_variants=nv)
    info = op.info
    assert info["n_variants"] == nv and info["ncols"] == S * nv and info["n_segments"] > 0
    fp32_early = nv > 1
    if fp32_early:
        assert info["far_entries_f32"] > 0
    # BF16 keeps 8 significant bits (half-ulp 2^-9), FP16 11 (2^-12); low-rank
    # lags round both factors
    rel = {"bf16": 2.0 ** -9, "f16": 2.0 ** -12}[dtype] * 3
    geo = geometry.discretize(faults)
    dt = geometry.time_step(geo, SI.CS)
    seen16 = 0
    for (a, b), (t0, t1) in op.windows().items():
        for T in sorted({max(t0, 1), t0 + 3, S, S + 1, (t0 + t1) // 2, t1}):
            if T < max(t0, 1) or T > t1:
                continue
            K = I.pair_kernel(geo, a, b, T, dt, SI.CS)
            R = op.lag_matrix(a, b, T, 64, 64)
            nrm = np.linalg.norm(K)
            if nrm == 0:
                assert np.all(R == 0)
                continue
            err = np.linalg.norm(R - K) / nrm
            if T < S or (fp32_early and T < 16):
                assert err < 2e-6, (a, b, T, err)  # FP32 near list (ensembles: list 3)
            else:
                seen16 += 1
                assert err < rel + 2e-6, (a, b, T, err)
                assert err > 1e-9, "16-bit storage expected"
        G = I.static_dipole(geo, a, b, SI.MU)
        R = op.lag_matrix(a, b, -1, 64, 64)
        eta = SI.MU / (2 * SI.CS)
        e = np.linalg.norm(R + G / eta) / np.linalg.norm(G / eta)
        assert e < (rel + 2e-6 if (nv > 1 and not fp32_early) else 2e-6), e
    assert seen16 > 0


def test_ensemble_row_slices_reconstruct_the_kernel():
    """Ensemble builds slice receiver clusters taller than a segment's rows (256
    for 64 variants) into row slices; the lag matrices they rebuild are still the
    kernel to BF16 rounding."""
    faults = SI.two_fault_prescribed_faults(n_elem=320, dx=40.0)
    op = _op(faults, compress=1, aca_tol=1e-6, eta_H=2.0, leaf=400, time_block=1, factor_dtype="bf16",
             n_variants=64)
    blocks = op.blocks(0, 1)
    assert any(r1 - r0 > 256 for r0, r1, _, _, _ in blocks)  # a tall block exists
    geo = geometry.discretize(faults)
    dt = geometry.time_step(geo, SI.CS)
    (t0, t1) = op.windows()[(0, 1)]
    for T in (max(t0, 1), (t0 + t1) // 2, t1):
        K = I.pair_kernel(geo, 0, 1, T, dt, SI.CS)
        R = op.lag_matrix(0, 1, T, 320, 320)
        assert np.linalg.norm(R - K) / np.linalg.norm(K) < 3 * 2.0 ** -9, T


def _first_lag_behind_fronts(geo, a, b, r0, r1, s0, s1, dt):
    """Smallest T with cs T dt beyond every distance from a receiver midpoint of the
    block to an edge of its source elements (both fronts of the primitive passed)."""
    B = geo[b]
    edges = B.c[None, :] + (-0.5 * B.L + np.arange(s0, s1 + 1) * B.dx)[:, None] * B.t[None, :]
    d = np.linalg.norm(geo[a].mid[r0:r1, None, :] - edges[None, :, :], axis=2).max()
    return int(np.floor(d / (SI.CS * dt))) + 1


@pytest.mark.parametrize("dtype,S,nv", [("f64", 1, 1), ("f32", 32, 1), ("bf16", 16, 1), ("f16", 1, 16)])
def test_partial_aca_behind_the_fronts(dtype, S, nv):
    """aca_partial = 1: admissible blocks at lags behind both wave fronts are built
    from rows and columns (partial pivoting, then truncated SVD), and reproduce the
    dense kernel block by block within the tolerance (plus the storage rounding).
    With FP64 / FP32 storage every other block-lag and the static tails are the
    same bits as with full pivoting; 16-bit items share one power-of-two scale over
    their lags, so there the other block-lags are held to the rounding bound."""
    faults = SI.five_fault_network(seed=3, n_elem=100)
    tol = 1e-6
    kw = dict(compress=1, aca_tol=tol, eta_H=2.0, leaf=20, time_block=S, factor_dtype=dtype, n_variants=nv)
    op0, op1 = _op(faults, **kw), _op(faults, aca_partial=1, **kw)
    geo = geometry.discretize(faults)
    dt = geometry.time_step(geo, SI.CS)
    wide = dtype in ("f64", "f32")
    exact = 1e-12 if dtype == "f64" else 1e-6
    # 16-bit lags (three roundings of 2^-9 / 2^-12); lags below S, and for ensembles
    # below 16, stay in FP32
    rel16 = {"bf16": 2.0 ** -9, "f16": 2.0 ** -12}.get(dtype, 0.0) * 3
    fp32_below = 16 if nv > 1 else S
    behind = changed = same = 0
    for (a, b), (t0, t1) in op1.windows().items():
        blks = op1.blocks(a, b)
        first = [_first_lag_behind_fronts(geo, a, b, r0, r1, s0, s1, dt) for (r0, r1, s0, s1, _) in blks]
        for T in sorted({int(x) for x in np.linspace(max(t0, 1), t1, 8)}):
            K = I.pair_kernel(geo, a, b, T, dt, SI.CS)
            R0 = op0.lag_matrix(a, b, T, 100, 100)
            R1 = op1.lag_matrix(a, b, T, 100, 100)
            rnd = exact if (wide or T < fp32_below) else rel16 + 2e-6
            for (r0, r1, s0, s1, adm), f in zip(blks, first):
                sl = np.s_[r0:r1, s0:s1]
                nrm = np.linalg.norm(K[sl])
                if not adm or T <= f - 2:
                    if wide:
                        assert np.array_equal(R1[sl], R0[sl]), (a, b, T, r0, s0)
                    else:
                        assert np.linalg.norm(R1[sl] - K[sl]) <= (2 * tol + rnd) * nrm, (a, b, T, r0, s0)
                    same += 1
                elif T >= f + 1:
                    assert np.linalg.norm(R1[sl] - K[sl]) <= (2 * tol + rnd) * nrm, (a, b, T, r0, s0)
                    behind += 1
                    changed += not np.array_equal(R1[sl], R0[sl])
        if wide:
            assert np.array_equal(op1.lag_matrix(a, b, -1, 100, 100), op0.lag_matrix(a, b, -1, 100, 100))
    assert behind > 200 and same > 200
    assert changed > behind // 2
    assert op1.info["stored_entries"] < 1.01 * op0.info["stored_entries"]


def test_16bit_rounding_matches_numpy():
    """The host conversions round to nearest even: FP16 against numpy's float16,
    BF16 against the top 16 bits of the FP32 pattern rounded to nearest even."""
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-1, 1, 4000), rng.uniform(-1e-4, 1e-4, 1000),
                        [0.0, -0.0, 1.0, -1.0, 2.0 ** -24, 2.0 ** -14, 0.999999]]).astype(np.float32)
    L = _lib_or_skip()
    got16 = np.array([L.seas_round_factor(float(v), 3) for v in x], dtype=np.float64)
    assert np.array_equal(got16, x.astype(np.float16).astype(np.float64))
    u = x.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint32) << 16
    assert np.array_equal(np.array([L.seas_round_factor(float(v), 2) for v in x]), r.view(np.float32).astype(np.float64))


def test_compression_reduces_storage():
    faults = SI.five_fault_network(seed=0, n_elem=100)
    dense = _op(faults, compress=0, eta_H=2.0, leaf=25).info
    comp = _op(faults, compress=1, eta_H=2.0, leaf=25, aca_tol=1e-6).info
    assert comp["stored_entries"] < 0.8 * dense["stored_entries"]
    assert dense["n_blocks"] == comp["n_blocks"]


def test_rejects_degenerate_input():
    _lib_or_skip()
    bad = [SI.fault(0, 0, 0, 1000.0, 10), dict(cx=0.0, cy=500.0, nx=0.0, ny=0.0, length=1000.0, n_elem=10)]
    with pytest.raises(P.SeasError) as e:
        P.Operator(bad, SI.default_params(host_only=1))
    assert e.value.code == -1
    with pytest.raises(P.SeasError):
        P.Operator([SI.fault(0, 0, 0, 1000.0, 1)], SI.default_params(host_only=1))
    with pytest.raises(P.SeasError):
        P.Operator([SI.fault(0, 0, 0, 1000.0, 10)], SI.default_params(host_only=1, beta=0.7))
    # fault 2's element end point at (-450, 0) sits on fault 1's first midpoint
    f1 = SI.fault(0, 0, 0, 1000.0, 10)
    f2 = SI.fault(-450.0, 0.0, 90.0, 1000.0, 10)
    with pytest.raises(P.SeasError) as e:
        P.Operator([f1, f2], SI.default_params(host_only=1))
    assert e.value.code == -1


@pytest.mark.parametrize("kw", [
    dict(time_block=32, factor_dtype="f64"),          # 32 windows need FP32 on the segment kernel
    dict(time_block=32, factor_dtype="f16"),          # one-variant 16-bit forms need 16
    dict(time_block=64, factor_dtype="f32"),
    dict(time_block=12, factor_dtype="f32"),
    dict(self_tail=2),
    dict(aca_partial=2),
    dict(free_surface=2),
    dict(adaptive_dt=1, time_block=16),              # adaptive steps need unblocked evaluation
    dict(adaptive_dt=2),
    dict(gamma_max=-1, adaptive_dt=1),
    dict(n_variants=8, factor_dtype="bf16", time_block=1),
    dict(n_variants=16, factor_dtype="f32", time_block=1),
    dict(n_variants=16, factor_dtype="bf16", time_block=16),
])
def test_rejects_invalid_options(kw):
    _lib_or_skip()
    with pytest.raises(P.SeasError) as e:
        P.Operator(SI.two_fault_prescribed_faults(n_elem=16, dx=100.0), SI.default_params(host_only=1, **kw))
    assert e.value.code == -1


def test_accepts_the_valid_time_blocks():
    faults = SI.two_fault_prescribed_faults(n_elem=16, dx=100.0)
    for S, d in ((0, "f64"), (1, "f32"), (2, "f64"), (4, "f32"), (8, "f64"), (16, "f32"), (32, "f32"), (16, "f16")):
        op = _op(faults, time_block=S, factor_dtype=d)
        assert op.info["time_block"] == max(S, 1)


def test_host_only_operator_refuses_evaluation():
    op = _op(SI.two_fault_prescribed_faults(n_elem=16, dx=800.0))
    n = op.N
    fr = dict(a=np.full(n, 0.01), b=np.full(n, 0.015), Dc=np.full(n, 5e-3), sigma_n=np.full(n, 5e7),
              V0=np.full(n, 1e-6), f0=np.full(n, 0.6))
    with pytest.raises(P.SeasError) as e:
        P.State(op, fr, np.full(n, 1e-9), np.full(n, 5e6), np.full(n, 3e7))
    assert e.value.code == -5


@pytest.mark.slow
@pytest.mark.parametrize("dtype,S,partial", [("f64", 16, 0), ("f32", 32, 0), ("f32", 32, 1)])
def test_wide_cluster_is_split_into_column_slices(dtype, S, partial):
    # two parallel 400-element faults whose root clusters are admissible: with
    # S = 16 the 400-wide source cluster exceeds the kernel's history buffer and is
    # packed as column slices, each compressed on its own (with aca_partial, each
    # slice from the first lag behind both fronts of its own columns)
    faults = [SI.fault(0, 0, 0, 400.0, 400), SI.fault(0, 100.0, 0, 400.0, 400)]
    kw = dict(compress=1, aca_tol=1e-6, eta_H=0.2, leaf=50, time_block=S, factor_dtype=dtype)
    op = _op(faults, aca_partial=partial, **kw)
    assert op.blocks(0, 1) == [(0, 400, 0, 400, True)]
    if partial:
        assert op.info["stored_entries"] != _op(faults, **kw).info["stored_entries"]
    geo = geometry.discretize(faults)
    dt = geometry.time_step(geo, SI.CS)
    t0, t1 = op.windows()[(0, 1)]
    for T in (t0 + 5, t0 + 40, (t0 + t1) // 2, t1 - 30, t1 - 8, t1):
        K = I.pair_kernel(geo, 0, 1, T, dt, SI.CS)
        R = op.lag_matrix(0, 1, T, 400, 400)
        assert np.linalg.norm(K) > 0
        assert np.linalg.norm(R - K) / np.linalg.norm(K) < 3e-6


@pytest.mark.parametrize("dtype,S", [("f64", 1), ("f32", 16)])
def test_cluster_windows_match_oracle(dtype, S):
    """Cluster-level windows (cluster_windows = 1): every block's upper lag is the
    oracle's block_window_end (at most the pair's T_end, some shorter), and the
    reconstructed lag matrices are the dense kernel with each entry cut at its
    block's upper lag; the static-tail matrix is unchanged."""
    faults = SI.five_fault_network(seed=1, n_elem=40)
    op = _op(faults, compress=0, eta_H=1.5, leaf=6, time_block=S, factor_dtype=dtype, cluster_windows=1)
    geo = geometry.discretize(faults)
    dt = geometry.time_step(geo, SI.CS)
    blocks = HP.partition(geo, 1.5, 6)
    shortened = 0
    for (a, b), (t0, t1) in op.windows().items():
        tw = op.block_windows(a, b)
        for blk, te in zip(blocks[(a, b)], tw):
            assert te == min(t1, I.block_window_end(geo, a, b, blk, SI.CS, dt, 0.01))
            shortened += te < t1
        Tend = np.zeros((40, 40), dtype=int)
        for (r0, r1, s0, s1, _), te in zip(blocks[(a, b)], tw):
            Tend[r0:r1, s0:s1] = te
        for T in sorted({max(t0, 1), int(np.median(tw)), min(tw), max(tw), t1}):
            if T < max(t0, 1):
                continue
            K = np.where(T <= Tend, I.pair_kernel(geo, a, b, T, dt, SI.CS), 0.0)
            R = op.lag_matrix(a, b, T, 40, 40)
            nrm = max(np.linalg.norm(K), 1e-300)
            # (FP64: rounding of late-lag entries, differences of two time levels)
            assert np.linalg.norm(R - K) / nrm < (1e-11 if dtype == "f64" else 1e-6), (a, b, T)
    assert shortened > 0


def test_free_surface_image_pairs_match_oracle():
    # method of images: the library's pairs (a, image of b) take the oracle's windows
    # and partition of the receiver fault against the mirrored source fault
    y0 = 0.0
    faults = SI.free_surface_network(n_elem=32, y0=y0)
    op = _op(faults, free_surface=1, surface_y=y0, eta_H=2.0, leaf=8)
    geo = geometry.discretize(faults + geometry.mirror_images(faults, y0))
    dt = op.info["dt"]
    blocks = HP.partition(geo, 2.0, 8)
    nf = len(faults)
    for a in range(nf):
        for b in range(nf):
            t = op.pair_window(a, nf + b)
            assert t == I.pair_window_lags(geo, a, nf + b, SI.CS, dt, 0.01, 0.01), (a, b)
            assert op.blocks(a, nf + b) == blocks[(a, nf + b)]
    assert op.pair_window(0, nf + 0)[0] == 0            # the surface fault touches its image
    with pytest.raises(P.SeasError):
        _op(faults, free_surface=1, surface_y=-200.0)  # a fault reaching above the surface


@pytest.mark.parametrize("compress", [0, 1])
def test_free_surface_cross_pairs_sum_direct_and_image(compress):
    # the pair (a, b) of a free-surface operator holds the blocks against fault b and
    # against its image on the same source columns; the reconstruction sums both
    # (dense items included), each inside its own window, tails too
    y0 = 0.0
    faults = SI.free_surface_network(n_elem=64, y0=y0)
    nf = len(faults)
    op = _op(faults, free_surface=1, surface_y=y0, compress=compress, aca_tol=1e-10, eta_H=2.0, leaf=8)
    dt = op.info["dt"]
    geo = geometry.discretize(faults + geometry.mirror_images(faults, y0))
    eta = SI.MU / (2 * SI.CS)
    tol = 1e-11 if compress == 0 else 1e-9
    for a in range(nf):
        for b in range(nf):
            if a == b:
                continue
            d0, d1 = I.pair_window_lags(geo, a, b, SI.CS, dt, 0.01, 0.01)
            m0, m1 = I.pair_window_lags(geo, a, nf + b, SI.CS, dt, 0.01, 0.01)
            assert d1 != m1   # the two windows differ: some lags hold one of the two kernels only
            for T in sorted({1, d0, m0, (d0 + d1) // 2, d1, d1 + 1, m1}):
                ref = np.zeros((64, 64))
                if d0 <= T <= d1:
                    ref += I.pair_kernel(geo, a, b, T, dt, SI.CS)
                if m0 <= T <= m1:
                    ref -= I.pair_kernel(geo, a, nf + b, T, dt, SI.CS)
                got = op.lag_matrix(a, b, T, 64, 64)
                assert np.abs(got - ref).max() <= tol * max(np.abs(ref).max(), 1e-300), (a, b, T)
            G = I.static_dipole(geo, a, b, SI.MU) - I.static_dipole(geo, a, nf + b, SI.MU)
            got = op.lag_matrix(a, b, -1, 64, 64)
            assert np.abs(got + G / eta).max() <= tol * np.abs(G / eta).max()


@pytest.mark.parametrize("cluster_windows", [0, 1])
def test_partial_aca_with_images_and_cluster_windows(cluster_windows):
    # aca_partial on image pairs (sign -1) and on per-block windows: every lag matrix
    # within the tolerance of the full-pivoting build, the static tails the same bits
    y0 = 0.0
    faults = SI.free_surface_network(n_elem=64, y0=y0)
    nf = len(faults)
    tol = 1e-6
    kw = dict(free_surface=1, surface_y=y0, compress=1, aca_tol=tol, eta_H=2.0, leaf=8,
              cluster_windows=cluster_windows)
    op0, op1 = _op(faults, **kw), _op(faults, aca_partial=1, **kw)
    changed = 0
    for a in range(nf):
        for b in list(range(nf)) + [nf + a]:
            if a == b:
                continue
            t0, t1 = op1.pair_window(a, b)
            for T in range(max(t0, 1), t1 + 1, 3):
                R0, R1 = op0.lag_matrix(a, b, T, 64, 64), op1.lag_matrix(a, b, T, 64, 64)
                assert np.linalg.norm(R1 - R0) <= 2 * tol * np.linalg.norm(R0), (a, b, T)
                changed += not np.array_equal(R0, R1)
            assert np.array_equal(op1.lag_matrix(a, b, -1, 64, 64), op0.lag_matrix(a, b, -1, 64, 64))
    assert changed > 5


def test_free_surface_own_image_matrices_match_oracle():
    # the stored kernel of a surface-reaching fault with its own image, lag by lag and
    # its static tail, against the oracle's mirrored pair (sign -1 included)
    y0 = 0.0
    f1 = SI.free_surface_network(n_elem=24, y0=y0)[0]
    op = _op([f1], free_surface=1, surface_y=y0, compress=0, factor_dtype="f64")
    dt = op.info["dt"]
    geo = geometry.discretize([f1] + geometry.mirror_images([f1], y0))
    T0, T1 = op.pair_window(0, 1)
    assert T0 == 0
    for T in sorted({0, 1, 2, 7, T1 // 2, T1}):
        got = op.lag_matrix(0, 1, T, 24, 24)
        ref = -I.pair_kernel(geo, 0, 1, T, dt, SI.CS)
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max(), T
    tail = op.lag_matrix(0, 1, -1, 24, 24)
    G = -I.static_dipole(geo, 0, 1, SI.MU)
    assert np.allclose(tail, -G / (SI.MU / (2 * SI.CS)), rtol=1e-12, atol=0)


@pytest.mark.parametrize("dtype,S,nv,compress,partial", [
    ("f64", 1, 1, 0, 0), ("f64", 8, 1, 1, 1), ("f32", 32, 1, 0, 0), ("f32", 32, 1, 1, 1), ("f32", 16, 1, 1, 0),
    ("bf16", 16, 1, 1, 1), ("f16", 16, 1, 0, 0), ("bf16", 1, 16, 1, 0), ("f16", 1, 32, 1, 1)])
def test_option_matrix_against_oracle_with_images(dtype, S, nv, compress, partial):
    # storage types, time blocks, ensembles and both ACA forms on a free-surface
    # network: every pair's lag matrices (direct kernel plus the image's, each inside
    # its window) against the oracle, to the tolerance plus the storage rounding
    y0 = 0.0
    faults = SI.free_surface_network(n_elem=48, y0=y0)
    nf = len(faults)
    tol = 1e-7
    op = _op(faults, factor_dtype=dtype, time_block=S, n_variants=nv, compress=compress, aca_partial=partial,
             aca_tol=tol, eta_H=2.0, leaf=8, free_surface=1, surface_y=y0)
    dt = op.info["dt"]
    geo = geometry.discretize(faults + geometry.mirror_images(faults, y0))
    rounding = {"f64": 1e-11, "f32": 1e-6}.get(dtype, 1e-6 + 3 * {"bf16": 2.0 ** -9, "f16": 2.0 ** -12}.get(dtype, 0))
    bound = 2 * tol * compress + rounding
    checked = 0
    for a in range(nf):
        for b in range(nf):
            if a == b:
                continue
            wins = [(b, 1.0) + I.pair_window_lags(geo, a, b, SI.CS, dt, 0.01, 0.01),
                    (nf + b, -1.0) + I.pair_window_lags(geo, a, nf + b, SI.CS, dt, 0.01, 0.01)]
            hi = max(w[3] for w in wins)
            for T in sorted({S - 1, S, S + 1, 2 * S, hi - 1, hi} | set(range(1, hi + 1, max(1, hi // 12)))):
                if T < 1 or T > hi:
                    continue
                ref = np.zeros((48, 48))
                for (bb, sg, t0, t1) in wins:
                    if t0 <= T <= t1:
                        ref += sg * I.pair_kernel(geo, a, bb, T, dt, SI.CS)
                got = op.lag_matrix(a, b, T, 48, 48)
                assert np.linalg.norm(got - ref) <= bound * np.linalg.norm(ref), (a, b, T)
                checked += 1
    assert checked >= 30


@pytest.mark.parametrize("S,dtype,nv", [(1, "f64", 1), (8, "f64", 1), (32, "f32", 1), (16, "bf16", 1), (1, "f16", 16)])
def test_entry_counts_of_an_uncompressed_operator(S, dtype, nv):
    # the counts behind the bench's algorithmic bytes, tallied from the oracle: with
    # compress = 0 every block-lag holding a nonzero kernel entry stores p q values,
    # every block one static tail of p q; far entries are the lags >= S (at S = 1
    # every stored entry, tails included), block-start entries the lags S..2S-1.
    # FP32 part of 16-bit builds: one variant, the far lags of near-field blocks;
    # ensembles, near-field blocks, lags below 16 and the tails
    faults = SI.five_fault_network(seed=2, n_elem=40)
    geo = geometry.discretize(faults)
    op = _op(faults, compress=0, eta_H=2.0, leaf=10, time_block=S, factor_dtype=dtype, n_variants=nv)
    info = op.info
    dt = info["dt"]
    parts = HP.partition(geo, 2.0, 10)
    stored = far = first = dense = f32 = 0
    x16 = dtype in ("bf16", "f16")
    nf = len(faults)
    for a in range(nf):
        for b in range(nf):
            if a == b:
                continue
            t0, t1 = I.pair_window_lags(geo, a, b, SI.CS, dt, 0.01, 0.01)
            dense += (t1 - t0 + 1) * 40 * 40
            for T in range(max(t0, 1), t1 + 1):
                K = I.pair_kernel(geo, a, b, T, dt, SI.CS)
                for (r0, r1, s0, s1, adm) in parts[(a, b)]:
                    if np.any(K[r0:r1, s0:s1] != 0):
                        n = (r1 - r0) * (s1 - s0)
                        stored += n
                        far += n if (S == 1 or T >= S) else 0
                        first += n if (S > 1 and S <= T < 2 * S) else 0
                        if x16 and nv == 1 and T >= S and not adm:
                            f32 += n
                        if x16 and nv > 1 and (not adm or T < 16):
                            f32 += n
            tails = sum((r1 - r0) * (s1 - s0) for (r0, r1, s0, s1, _) in parts[(a, b)])
            stored += tails
            far += tails if S == 1 else 0
            f32 += tails if (x16 and nv > 1) else 0
    assert (info["stored_entries"], info["far_entries"], info["far_entries_first"], info["dense_entries"]) == \
        (stored, far, first, dense)
    if x16:
        assert 0 < info["far_entries_f32"] < info["far_entries"]
        assert info["far_entries_f32"] == f32


@pytest.mark.parametrize("eta_w,q_w,mode_cap", [(2.5, 5, 0), (1.0, 0, 20), (1.5, 40, 64)])
def test_self_window_options_match_oracle(eta_w, q_w, mode_cap):
    # the self windows W_n under other window factors, modulation integers and mode
    # caps: the library's tables against the oracle's, and the entry count they add up to
    faults = SI.two_fault_prescribed_faults(n_elem=96, dx=100.0)
    op = _op(faults, eta_w=eta_w, q_w=q_w, mode_cap=mode_cap)
    dt = op.info["dt"]
    total = 0
    for k, f in enumerate(faults):
        st = S.SelfTerm(f["n_elem"], f["length"], SI.MU, SI.CS, dt, eta_w=eta_w, q_w=q_w, mode_cap=mode_cap)
        nm = len(st.W)
        assert nm == (f["n_elem"] if mode_cap == 0 else min(mode_cap, f["n_elem"]))
        total += int(np.sum(st.W + 1))
        for n in sorted({1, 2, nm // 2, nm}):
            lt, ot = op.self_table(k, n), st.table(n - 1)
            assert len(lt) == len(ot) == st.W[n - 1] + 1
            assert np.abs(lt - ot).max() <= 1e-12 * np.abs(ot).max()
        if nm < f["n_elem"]:
            with pytest.raises(P.SeasError):
                op.self_table(k, nm + 1)
    assert op.info["self_entries"] == total


def test_build_is_independent_of_the_thread_count():
    # blocks are built in parallel and merged in a fixed order: one thread and eight
    # give the same operator bit for bit
    faults = SI.five_fault_network(seed=5, n_elem=60)
    kw = dict(compress=1, aca_tol=1e-6, eta_H=2.0, leaf=10, time_block=32, factor_dtype="f32")
    ops = [_op(faults, n_threads=t, **kw) for t in (1, 8)]
    i0, i1 = ({k: v for k, v in o.info.items() if k != "build_seconds"} for o in ops)
    assert i0 == i1
    for (a, b), (t0, t1) in ops[0].windows().items():
        for T in sorted({max(t0, 1), 31, 32, 64, (t0 + t1) // 2, t1, -1}):
            if T != -1 and not (max(t0, 1) <= T <= t1):
                continue
            assert np.array_equal(ops[0].lag_matrix(a, b, T, 60, 60), ops[1].lag_matrix(a, b, T, 60, 60)), (a, b, T)


def test_cluster_windows_on_image_pairs_match_oracle():
    # per-block upper lags of the pairs with mirror images (free surface), and the pair
    # (a, b) as the evaluation applies it: the direct and the image kernel, each entry
    # cut at its own block's upper lag. Receivers of a surface-reaching fault sit at
    # (m + 1/2) dx from the element edges of its own image, the fronts at beta T dx:
    # beta = 0.4373 keeps every lag off them (beta = 1/2 or 0.45 = 9/20 puts whole
    # lags on a front, where the square root of the primitive magnifies rounding and
    # library and oracle differ by ~1e-8)
    y0 = 0.0
    faults = SI.free_surface_network(n_elem=40, y0=y0)
    nf = len(faults)
    op = _op(faults, compress=0, eta_H=1.5, leaf=6, free_surface=1, surface_y=y0, cluster_windows=1, beta=0.4373)
    geo = geometry.discretize(faults + geometry.mirror_images(faults, y0))
    dt = op.info["dt"]
    blocks = HP.partition(geo, 1.5, 6)
    shortened = checked = 0
    for a in range(nf):
        cut = {}
        for bb in [c for c in range(nf) if c != a] + [nf + c for c in range(nf)]:
            t0, t1 = op.pair_window(a, bb)
            te_all = op.block_windows(a, bb)
            Te = np.full((40, 40), -1)
            for blk, te in zip(blocks[(a, bb)], te_all):
                assert te == min(t1, I.block_window_end(geo, a, bb, blk, SI.CS, dt, 0.01)), (a, bb, blk)
                shortened += te < t1
                Te[blk[0]:blk[1], blk[2]:blk[3]] = te
            cut[bb] = (t0, Te)

        def kernel(bb, T, sg):
            t0, Te = cut[bb]
            return sg * np.where(T <= Te, I.pair_kernel(geo, a, bb, T, dt, SI.CS), 0.0) if T >= t0 else 0.0

        for b in list(range(nf)) + [nf + a]:
            if b == a:
                continue
            terms = [(nf + a, -1.0)] if b == nf + a else [(b, 1.0), (nf + b, -1.0)]
            hi = max(cut[bb][1].max() for bb, _ in terms)
            for T in range(1, hi + 1, 3):
                K = sum(kernel(bb, T, sg) for bb, sg in terms) + np.zeros((40, 40))
                R = op.lag_matrix(a, b, T, 40, 40)
                assert np.linalg.norm(R - K) <= 1e-11 * max(np.linalg.norm(K), 1e-300), (a, b, T)
                checked += 1
    assert shortened > 0 and checked > 50


@pytest.mark.parametrize("kw", [dict(factor_dtype="f64"), dict(factor_dtype="f32", time_block=32, aca_partial=1),
                                dict(factor_dtype="bf16", time_block=16, leaf=8),
                                dict(factor_dtype="f16", n_variants=16, leaf=8),
                                dict(factor_dtype="f64", cluster_windows=1, leaf=8)])
def test_dropping_the_static_tail_changes_nothing_else(kw):
    # int_tail = 0 removes the static-tail matrices and nothing else: every lag matrix
    # (direct and image pairs) is the same bits as with the tail, the tails are zero
    y0 = 0.0
    faults = SI.free_surface_network(n_elem=40, y0=y0)
    base = dict(free_surface=1, surface_y=y0, beta=0.4373, aca_tol=1e-8, **kw)
    with_tail, without = _op(faults, int_tail=1, **base), _op(faults, int_tail=0, **base)
    for a in range(2):
        for b in (1 - a, 2 + a):
            t0, t1 = with_tail.pair_window(a, b)
            for T in range(max(t0, 1), t1 + 1, 7):
                assert np.array_equal(with_tail.lag_matrix(a, b, T, 40, 40), without.lag_matrix(a, b, T, 40, 40))
            assert not without.lag_matrix(a, b, -1, 40, 40).any()
            assert with_tail.lag_matrix(a, b, -1, 40, 40).any()
    assert without.info["stored_entries"] < with_tail.info["stored_entries"]
