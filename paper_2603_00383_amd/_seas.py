"""ctypes binding of libseas.so (argument marshalling only).

Every computation of the stress-transfer path runs in the HIP library; this
module converts Python values to the C structs of include/seas.h, passes device
pointers (integers, e.g. ``tensor.data_ptr()``) and stream handles (``int``,
e.g. ``torch.cuda.current_stream().cuda_stream``) through, and raises on any
non-zero status.  It fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libseas.so")

SEAS_F64, SEAS_F32, SEAS_BF16, SEAS_F16 = 0, 1, 2, 3
FIELDS = dict(V=0, theta=1, delta=2, thetadot=3, f_hist=4, f_self=5, f_int=6, tau0=7)
STATUS = {0: "OK", -1: "INVALID_ARG", -2: "OOM", -3: "HIP", -4: "NOT_CONVERGED", -5: "MISMATCH",
          -6: "INTERNAL"}


class SeasError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Fault(C.Structure):
    _fields_ = [("cx", C.c_double), ("cy", C.c_double), ("nx", C.c_double), ("ny", C.c_double),
                ("length", C.c_double), ("n_elem", C.c_int32), ("reserved", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("mu", C.c_double), ("cs", C.c_double), ("beta", C.c_double), ("eta_H", C.c_double),
                ("aca_tol", C.c_double), ("eta_tmin", C.c_double), ("eta_tmax", C.c_double),
                ("eta_w", C.c_double), ("leaf", C.c_int32), ("compress", C.c_int32),
                ("int_tail", C.c_int32), ("q_w", C.c_int32), ("mode_cap", C.c_int32),
                ("factor_dtype", C.c_int32), ("n_threads", C.c_int32), ("host_only", C.c_int32),
                ("time_block", C.c_int32), ("n_variants", C.c_int32), ("state_update", C.c_int32),
                ("cluster_windows", C.c_int32), ("adaptive_dt", C.c_int32), ("gamma_max", C.c_int32),
                ("adapt_xi", C.c_double), ("free_surface", C.c_int32), ("reserved_fs", C.c_int32),
                ("surface_y", C.c_double), ("self_tail", C.c_int32), ("aca_partial", C.c_int32)]


class OpInfo(C.Structure):
    _fields_ = [("n_faults", C.c_int32), ("n_elem", C.c_int32), ("dt", C.c_double),
                ("max_lag", C.c_int32), ("max_self_window", C.c_int32), ("n_blocks", C.c_int64),
                ("n_items", C.c_int64), ("dense_entries", C.c_int64), ("stored_entries", C.c_int64),
                ("lag0_nnz", C.c_int64), ("self_entries", C.c_int64), ("bytes_per_step", C.c_double),
                ("flops_per_step", C.c_double), ("build_seconds", C.c_double),
                ("factor_dtype", C.c_int32), ("time_block", C.c_int32), ("far_entries", C.c_int64),
                ("n_items_near", C.c_int64), ("n_variants", C.c_int32), ("ncols", C.c_int32),
                ("n_segments", C.c_int64), ("far_bytes", C.c_int64), ("far_entries_f32", C.c_int64),
                ("partial_bytes", C.c_int64), ("far_entries_first", C.c_int64),
                ("far_entries_first_f32", C.c_int64)]


class Friction(C.Structure):
    _fields_ = [(k, C.POINTER(C.c_double)) for k in ("a", "b", "Dc", "sigma_n", "V0", "f0", "eps")]


class Request(C.Structure):
    _fields_ = [("pool", C.c_int32), ("n_steps", C.c_int32), ("arrival_s", C.c_double), ("fric", Friction),
                ("V_init", C.POINTER(C.c_double)), ("theta_init", C.POINTER(C.c_double)),
                ("tau0", C.POINTER(C.c_double)), ("tau0_rate", C.POINTER(C.c_double)),
                ("delta_init", C.POINTER(C.c_double)), ("V_out", C.POINTER(C.c_double)),
                ("theta_out", C.POINTER(C.c_double)), ("delta_out", C.POINTER(C.c_double)),
                ("admit_s", C.c_double), ("finish_s", C.c_double), ("status", C.c_int32),
                ("reserved", C.c_int32)]


_lib = None


def lib():
    """The loaded library; raises if libseas.so is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2603_00383_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
        sig = {
            "seas_last_error": (C.c_char_p, []),
            "seas_version": (C.c_char_p, []),
            "seas_round_factor": (C.c_double, [C.c_double, i32]),
            "seas_build_operator": (i32, [C.POINTER(Fault), i32, C.POINTER(Params), C.POINTER(vp)]),
            "seas_operator_destroy": (None, [vp]),
            "seas_operator_info": (i32, [vp, C.POINTER(OpInfo)]),
            "seas_operator_windows": (i32, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
            "seas_operator_blocks": (i32, [vp, i32, i32, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
            "seas_operator_pair_window": (i32, [vp, i32, i32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
            "seas_operator_self_table": (i32, [vp, i32, i32, dp, i32, C.POINTER(C.c_int32)]),
            "seas_operator_lag_matrix": (i32, [vp, i32, i32, i32, dp]),
            "seas_state_bytes": (C.c_size_t, [vp, i32]),
            "seas_state_create": (i32, [vp, i32, C.POINTER(Friction), dp, dp, dp, dp, dp, vp, C.POINTER(vp)]),
            "seas_state_destroy": (None, [vp]),
            "seas_state_load_history": (i32, [vp, dp, i32, vp]),
            "seas_state_reset_variant": (i32, [vp, i32, C.POINTER(Friction), dp, dp, dp, dp, dp, vp]),
            "seas_eval_prescribed": (i32, [vp, vp, vp, i32, vp, vp]),
            "seas_eval_prescribed_noalloc": (i32, [vp, vp, vp, i32, vp, vp]),
            "seas_step": (i32, [vp, vp, i32, vp]),
            "seas_state_check": (i32, [vp, vp]),
            "seas_state_variant_status": (i32, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64), vp]),
            "seas_write_state": (i32, [vp, i32, i32, vp, C.c_size_t, i32, vp]),
            "seas_read_state": (i32, [vp, i32, i32, vp, C.c_size_t, i32, vp]),
            "seas_state_step_index": (i64, [vp]),
            "seas_state_set_timing": (i32, [vp, i32]),
            "seas_state_set_overlap": (i32, [vp, i32]),
            "seas_state_set_graph": (i32, [vp, i32]),
            "seas_operator_tune": (i32, [vp, vp, vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
            "seas_operator_set_tune": (i32, [vp, i32]),
            "seas_state_graph_info": (i32, [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
            "seas_state_progress": (i32, [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
            "seas_state_set_gamma_cap": (i32, [vp, C.c_int64]),
            "seas_state_set_time_block": (i32, [vp, i32]),
            "seas_state_read_timing": (i32, [vp, vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
            "seas_state_checkpoint_bytes": (C.c_size_t, [vp]),
            "seas_state_save": (i32, [vp, vp, C.c_size_t, vp]),
            "seas_state_restore": (i32, [vp, vp, C.c_size_t, vp]),
            "seas_server_create": (i32, [C.POINTER(vp), i32, C.POINTER(Request), C.c_size_t, i32,
                                         C.POINTER(vp)]),
            "seas_server_run": (i32, [vp, C.POINTER(Request), i32]),
            "seas_server_destroy": (None, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise SeasError(rc, lib().seas_last_error().decode())


def _dptr(a):
    """Host float64 array -> (keepalive, POINTER(c_double))."""
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=np.float64)
    return arr, arr.ctypes.data_as(C.POINTER(C.c_double))


def _ptr(x):
    """Device pointer / stream from an int or an object with data_ptr()."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return C.c_void_p(x.data_ptr())
    return C.c_void_p(int(x))


_DTYPE = {"f64": SEAS_F64, "f32": SEAS_F32, "bf16": SEAS_BF16, "f16": SEAS_F16,
          SEAS_F64: SEAS_F64, SEAS_F32: SEAS_F32, SEAS_BF16: SEAS_BF16, SEAS_F16: SEAS_F16}


def make_params(p):
    q = Params()
    q.mu, q.cs, q.beta = p["mu"], p["cs"], p.get("beta", 0.5)
    q.eta_H, q.aca_tol = p.get("eta_H", 2.0), p.get("aca_tol", 1e-6)
    q.eta_tmin, q.eta_tmax = p.get("eta_tmin", 0.01), p.get("eta_tmax", 0.01)
    q.eta_w = p.get("eta_w", 1.5)
    q.leaf, q.compress = int(p.get("leaf", 50)), int(p.get("compress", 1))
    q.int_tail, q.q_w, q.mode_cap = int(p.get("int_tail", 1)), int(p.get("q_w", 0)), int(p.get("mode_cap", 0))
    q.factor_dtype = _DTYPE[p.get("factor_dtype", "f64")]
    q.n_threads = int(p.get("n_threads", 0))
    q.host_only = int(p.get("host_only", 0))
    q.time_block = int(p.get("time_block", 1))
    q.n_variants = int(p.get("n_variants", 1))
    q.state_update = {"explicit": 0, "exact": 1, 0: 0, 1: 1}[p.get("state_update", "explicit")]
    q.cluster_windows = int(p.get("cluster_windows", 0))
    q.adaptive_dt = int(p.get("adaptive_dt", 0))
    q.gamma_max = int(p.get("gamma_max", 0))
    q.adapt_xi = float(p.get("adapt_xi", 0.0))
    q.free_surface = int(p.get("free_surface", 0))
    q.surface_y = float(p.get("surface_y", 0.0))
    q.self_tail = int(p.get("self_tail", 0))
    q.aca_partial = int(p.get("aca_partial", 0))
    return q


class Operator:
    def __init__(self, faults, params):
        arr = (Fault * len(faults))()
        for i, f in enumerate(faults):
            arr[i] = Fault(f["cx"], f["cy"], f["nx"], f["ny"], f["length"], int(f["n_elem"]), 0)
        self._prm = make_params(params)
        h = C.c_void_p()
        _check(lib().seas_build_operator(arr, len(faults), C.byref(self._prm), C.byref(h)))
        self.h = h
        self.n_faults = len(faults)
        self.info = self._info()
        self.N = self.info["n_elem"]

    def _info(self):
        i = OpInfo()
        _check(lib().seas_operator_info(self.h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in OpInfo._fields_ if k != "reserved"}

    def windows(self):
        n = self.n_faults * (self.n_faults - 1)
        a, b = (C.c_int32 * n)(), (C.c_int32 * n)()
        _check(lib().seas_operator_windows(self.h, a, b))
        out, k = {}, 0
        for i in range(self.n_faults):
            for j in range(self.n_faults):
                if i != j:
                    out[(i, j)] = (a[k], b[k])
                    k += 1
        return out

    def pair_window(self, a, b):
        """(T_init, T_end) of pair (a, b); b >= n_faults selects the image of fault b - n_faults."""
        t0, t1 = C.c_int32(0), C.c_int32(0)
        _check(lib().seas_operator_pair_window(self.h, a, b, C.byref(t0), C.byref(t1)))
        return t0.value, t1.value

    def blocks(self, a, b):
        cnt = C.c_int64(0)
        _check(lib().seas_operator_blocks(self.h, a, b, None, C.byref(cnt)))
        buf = (C.c_int32 * (6 * cnt.value))()
        _check(lib().seas_operator_blocks(self.h, a, b, buf, C.byref(cnt)))
        v = np.frombuffer(buf, dtype=np.int32).reshape(-1, 6)
        return [(int(r[0]), int(r[1]), int(r[2]), int(r[3]), bool(r[4])) for r in v]

    def block_windows(self, a, b):
        """Upper lag of every block of the pair (a, b), in the order of ``blocks``."""
        cnt = C.c_int64(0)
        _check(lib().seas_operator_blocks(self.h, a, b, None, C.byref(cnt)))
        buf = (C.c_int32 * (6 * cnt.value))()
        _check(lib().seas_operator_blocks(self.h, a, b, buf, C.byref(cnt)))
        return [int(x) for x in np.frombuffer(buf, dtype=np.int32).reshape(-1, 6)[:, 5]]

    def self_table(self, k, n):
        """K_n^T, T = 0..W_n, and with self_tail the tail coefficient R_n last."""
        W = C.c_int32(0)
        _check(lib().seas_operator_self_table(self.h, k, n, None, 0, C.byref(W)))
        m = W.value + 1 + int(self._prm.self_tail)
        out = np.zeros(m)
        _check(lib().seas_operator_self_table(self.h, k, n, out.ctypes.data_as(C.POINTER(C.c_double)),
                                              m, C.byref(W)))
        return out

    def tune(self, state, stream=0, reps=3):
        """Time the far launch of each compiled variant on the state's history and keep
        the fastest: {"ms": [per variant, -1 where not applicable], "choice": variant}."""
        ms = (C.c_double * 3)()
        ch = C.c_int32(0)
        _check(lib().seas_operator_tune(self.h, state.h, _ptr(stream), int(reps), ms, C.byref(ch)))
        return {"ms": [float(x) for x in ms], "choice": ch.value}

    def set_tune(self, variant):
        _check(lib().seas_operator_set_tune(self.h, int(variant)))

    def lag_matrix(self, a, b, T, p, q):
        out = np.zeros((p, q))
        _check(lib().seas_operator_lag_matrix(self.h, a, b, T, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def state_bytes(self, n_variants=1):
        return int(lib().seas_state_bytes(self.h, n_variants))

    def close(self):
        if getattr(self, "h", None):
            lib().seas_operator_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class State:
    """Per-element arrays are (n_variants x N), variant-major (plain N for one variant)."""

    def __init__(self, op, fric, V, theta, tau0, tau0_rate=None, delta=None, stream=0):
        self.op = op
        self.nv = int(op.info["n_variants"])
        keep = []
        fr = Friction()
        for k in ("a", "b", "Dc", "sigma_n", "V0", "f0", "eps"):
            arr, p = _dptr(fric.get(k))
            keep.append(arr)
            setattr(fr, k, p)
        args = [_dptr(x) for x in (V, theta, tau0, tau0_rate, delta)]
        h = C.c_void_p()
        _check(lib().seas_state_create(op.h, self.nv, C.byref(fr), *[p for _, p in args], _ptr(stream),
                                       C.byref(h)))
        self.h = h

    def reset_variant(self, variant, fric, V, theta, tau0, tau0_rate=None, delta=None, stream=0):
        """Start a new window in one variant slot (arrays of N) at the current step."""
        keep = []
        fr = Friction()
        for k in ("a", "b", "Dc", "sigma_n", "V0", "f0", "eps"):
            arr, p = _dptr(fric.get(k))
            keep.append(arr)
            setattr(fr, k, p)
        args = [_dptr(x) for x in (V, theta, tau0, tau0_rate, delta)]
        _check(lib().seas_state_reset_variant(self.h, int(variant), C.byref(fr), *[p for _, p in args],
                                              _ptr(stream)))

    def load_history(self, V_hist, stream=0):
        arr = np.ascontiguousarray(V_hist, dtype=np.float64)
        _check(lib().seas_state_load_history(self.h, arr.ctypes.data_as(C.POINTER(C.c_double)), arr.shape[0],
                                             _ptr(stream)))  # (n_hist, N) or (n_hist, n_variants, N)

    def eval_prescribed(self, V_dev, n_steps, f_dev, stream=0):
        _check(lib().seas_eval_prescribed(self.op.h, self.h, _ptr(V_dev), n_steps, _ptr(f_dev), _ptr(stream)))

    def eval_prescribed_noalloc(self, V_dev, n_steps, f_dev, stream=0):
        _check(lib().seas_eval_prescribed_noalloc(self.op.h, self.h, _ptr(V_dev), n_steps, _ptr(f_dev),
                                                  _ptr(stream)))

    def step(self, n_steps=1, stream=0):
        _check(lib().seas_step(self.op.h, self.h, n_steps, _ptr(stream)))

    def check(self, stream=0):
        _check(lib().seas_state_check(self.h, _ptr(stream)))

    def variant_status(self, stream=0):
        """(failed[nv] bool array, last good step[nv] int array)."""
        f = np.zeros(self.nv, dtype=np.int32)
        g = np.zeros(self.nv, dtype=np.int64)
        _check(lib().seas_state_variant_status(self.h, f.ctypes.data_as(C.POINTER(C.c_int32)),
                                               g.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(stream)))
        return f.astype(bool), g

    def write(self, field, values, stream=0, variant=0):
        arr = np.ascontiguousarray(values, dtype=np.float64)
        _check(lib().seas_write_state(self.h, FIELDS[field], int(variant), C.c_void_p(arr.ctypes.data),
                                      arr.size, 0, _ptr(stream)))

    def read(self, field, stream=0, variant=0):
        out = np.zeros(self.op.N)
        _check(lib().seas_read_state(self.h, FIELDS[field], int(variant), C.c_void_p(out.ctypes.data), self.op.N,
                                     0, _ptr(stream)))
        return out

    def set_time_block(self, S):
        _check(lib().seas_state_set_time_block(self.h, int(S)))

    def set_timing(self, enable=True):
        _check(lib().seas_state_set_timing(self.h, 1 if enable else 0))

    def set_gamma_cap(self, cap):
        _check(lib().seas_state_set_gamma_cap(self.h, int(cap)))

    def progress(self):
        """Steps taken, gamma of the last step and the time reached (seconds)."""
        n, g, t = C.c_int64(0), C.c_int64(0), C.c_double(0.0)
        _check(lib().seas_state_progress(self.h, C.byref(n), C.byref(g), C.byref(t)))
        return {"steps_taken": n.value, "last_gamma": g.value, "time_s": t.value}

    def set_overlap(self, enable=True):
        _check(lib().seas_state_set_overlap(self.h, 1 if enable else 0))

    def set_graph(self, enable=True):
        """Fixed steps of whole time blocks as replays of one captured HIP graph."""
        _check(lib().seas_state_set_graph(self.h, 1 if enable else 0))

    def graph_info(self):
        r, u = C.c_int64(0), C.c_int32(0)
        _check(lib().seas_state_graph_info(self.h, C.byref(r), C.byref(u)))
        return {"replays": r.value, "steps_per_replay": u.value}

    def read_timing(self, stream=0):
        ms, n = C.c_double(0), C.c_int64(0)
        _check(lib().seas_state_read_timing(self.h, _ptr(stream), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    @property
    def step_index(self):
        return int(lib().seas_state_step_index(self.h))

    def save(self, stream=0):
        n = int(lib().seas_state_checkpoint_bytes(self.h))
        buf = np.zeros(n, dtype=np.uint8)
        _check(lib().seas_state_save(self.h, C.c_void_p(buf.ctypes.data), n, _ptr(stream)))
        return buf

    def restore(self, buf, stream=0):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib().seas_state_restore(self.h, C.c_void_p(buf.ctypes.data), buf.nbytes, _ptr(stream)))

    def close(self):
        if getattr(self, "h", None):
            lib().seas_state_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _request(pool, n_steps, arrival_s, window, keep, outputs=True, N=None):
    """Fill a Request from a dict window with keys fric (dict of N arrays), V, theta,
    tau0 (and optional tau0_rate, delta)."""
    r = Request()
    r.pool, r.n_steps, r.arrival_s = int(pool), int(n_steps), float(arrival_s)
    fr = Friction()
    for k in ("a", "b", "Dc", "sigma_n", "V0", "f0", "eps"):
        arr, p = _dptr(window["fric"].get(k))
        keep.append(arr)
        setattr(fr, k, p)
    r.fric = fr
    for name, key in (("V_init", "V"), ("theta_init", "theta"), ("tau0", "tau0"), ("tau0_rate", "tau0_rate"),
                      ("delta_init", "delta")):
        arr, p = _dptr(window.get(key))
        keep.append(arr)
        setattr(r, name, p)
    out = {}
    if outputs:
        for name, key in (("V_out", "V"), ("theta_out", "theta"), ("delta_out", "delta")):
            a = np.zeros(N)
            keep.append(a)
            out[key] = a
            setattr(r, name, a.ctypes.data_as(C.POINTER(C.c_double)))
    return r, out


class Server:
    """Request loop with continuous batching (seas_server_*): one pool per operator."""

    def __init__(self, ops, idle_windows, device_budget, chunk_steps=16):
        self.ops = list(ops)
        self._keep = []
        idle = (Request * len(self.ops))()
        for k, w in enumerate(idle_windows):
            idle[k], _ = _request(k, 1, 0.0, w, self._keep, outputs=False)
        self._idle = idle
        arr = (C.c_void_p * len(self.ops))(*[o.h.value for o in self.ops])
        h = C.c_void_p()
        _check(lib().seas_server_create(arr, len(self.ops), idle, int(device_budget), int(chunk_steps),
                                        C.byref(h)))
        self.h = h

    def run(self, requests):
        """requests: list of dict(pool, n_steps, arrival_s, window). Returns a list of
        dict(admit_s, finish_s, status, V, theta, delta)."""
        keep, outs = [], []
        arr = (Request * len(requests))()
        for i, q in enumerate(requests):
            arr[i], o = _request(q["pool"], q["n_steps"], q["arrival_s"], q["window"], keep,
                                 N=self.ops[q["pool"]].N)
            outs.append(o)
        _check(lib().seas_server_run(self.h, arr, len(requests)))
        res = []
        for i, o in enumerate(outs):
            d = dict(o)
            d.update(admit_s=arr[i].admit_s, finish_s=arr[i].finish_s, status=arr[i].status)
            res.append(d)
        return res

    def close(self):
        if getattr(self, "h", None):
            lib().seas_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
