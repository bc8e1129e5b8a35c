"""ctypes binding of libzpl (include/zpl.h): argument marshalling only.

Every step of the computation runs in the library's HIP kernels.  PyTorch is
used only to hold device memory (tensor.data_ptr()) and to name HIP streams
(torch.cuda.Stream.cuda_stream).  If the library is not built this module
raises on use: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from pathlib import Path
from typing import Iterable, Optional, Sequence

import numpy as np

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "libzpl.so"

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, EBUSY, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
FLAG_ALL_ONES, FLAG_TAIL_CAPPED, FLAG_BISECT, FLAG_NOCONV = 1, 2, 4, 8
LAUNCH_BATCHED, LAUNCH_PLAIN = 0, 1
FORM_AUTO, FORM_LANE, FORM_WAVE, FORM_HEAVY = 0, 1, 2, 3
_FORMS = {"auto": FORM_AUTO, "lane": FORM_LANE, "wave": FORM_WAVE, "heavy": FORM_HEAVY}
_LAUNCH = {"batched": LAUNCH_BATCHED, "plain": LAUNCH_PLAIN}
TABLE_H = 4096


class ZplError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("zpl error %d: %s" % (status, msg))
        self.status = status


class Cell(C.Structure):
    _fields_ = [("alpha", C.c_double), ("n", C.c_int64), ("replicates", C.c_int64),
                ("seed", C.c_uint64), ("stream", C.c_uint32), ("kmax", C.c_uint32),
                ("xmin", C.c_int64)]


class ServeOpts(C.Structure):
    _fields_ = [("mem_budget_bytes", C.c_uint64), ("max_batch", C.c_int32),
                ("max_queue", C.c_int32), ("slice_us", C.c_int32), ("reserved2", C.c_int32)]


class ServeResult(C.Structure):
    _fields_ = [("done", C.c_int32), ("status", C.c_int32), ("alpha_hat", C.c_double),
                ("D", C.c_double), ("p_value", C.c_double), ("flags", C.c_uint32),
                ("batch_size", C.c_int32), ("queue_ms", C.c_double), ("latency_ms", C.c_double),
                ("launches", C.c_int32), ("reserved", C.c_int32)]


class TuneEntry(C.Structure):
    _fields_ = [("alpha", C.c_double), ("n", C.c_int64), ("ns_per_replicate", C.c_double * 3)]


class SimOpts(C.Structure):
    _fields_ = [("launch", C.c_int32), ("form", C.c_int32), ("use_graph", C.c_int32),
                ("reserved", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(
                "libzpl.so is not built (run python -m paper_1305_6738_amd._build); "
                "there is no CPU fallback")
        L = C.CDLL(str(LIB_PATH))
        vp, i32, i64, u32, u64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
        P = C.POINTER
        L.zpl_create.argtypes = [P(vp), i32, u64]
        L.zpl_create.restype = i32
        L.zpl_destroy.argtypes = [vp]
        L.zpl_destroy.restype = None
        L.zpl_last_error.argtypes = []
        L.zpl_last_error.restype = C.c_char_p
        L.zpl_simulate_cells.argtypes = [vp, P(Cell), i32, P(u32), P(u32), i32, P(d), vp, vp,
                                         vp, vp, P(SimOpts), vp]
        L.zpl_simulate_cells.restype = i32
        L.zpl_set_timing.argtypes = [vp, i32]
        L.zpl_set_timing.restype = i32
        L.zpl_get_timing.argtypes = [vp, P(d)]
        L.zpl_get_timing.restype = i32
        L.zpl_fit.argtypes = [vp, vp, i64, i32, P(d), P(d), P(u32), vp]
        L.zpl_fit.restype = i32
        L.zpl_fit_truncated.argtypes = [vp, vp, i64, i32, u32, P(d), P(d), P(u32), vp]
        L.zpl_fit_truncated.restype = i32
        L.zpl_bootstrap_pvalue.argtypes = [vp, vp, i64, i32, i64, u64, u32, P(d), P(d), P(d),
                                           P(u32), vp]
        L.zpl_bootstrap_pvalue.restype = i32
        L.zpl_serve_start.argtypes = [vp, P(ServeOpts)]
        L.zpl_serve_start.restype = i32
        L.zpl_serve_submit.argtypes = [vp, vp, i64, i32, i64, u64, u32, P(u64)]
        L.zpl_serve_submit.restype = i32
        L.zpl_serve_poll.argtypes = [vp, u64, i32, P(ServeResult)]
        L.zpl_serve_poll.restype = i32
        L.zpl_serve_stop.argtypes = [vp]
        L.zpl_serve_stop.restype = i32
        L.zpl_sample_draws.argtypes = [vp, d, u32, i64, i64, u64, u32, i64, i64, vp, vp, vp]
        L.zpl_sample_draws.restype = i32
        L.zpl_cdf_table.argtypes = [vp, d, u32, i64, vp, vp]
        L.zpl_cdf_table.restype = i32
        L.zpl_autotune.argtypes = [vp, P(d), i32, P(i64), i32, P(TuneEntry), vp]
        L.zpl_autotune.restype = i32
        L.zpl_set_tuning.argtypes = [vp, P(TuneEntry), i32]
        L.zpl_set_tuning.restype = i32
        L.zpl_plan_forms.argtypes = [P(TuneEntry), i32, P(Cell), i32, P(i32)]
        L.zpl_plan_forms.restype = i32
        L.zpl_critical_table.argtypes = [vp, P(d), i32, P(i64), i32, u32, i32, u64, i64, P(u32),
                                         P(u32), i32, P(d), P(d), vp]
        L.zpl_critical_table.restype = i32
        L.zpl_fit_scan.argtypes = [vp, vp, i64, i32, P(i64), i32, P(d), P(d), P(i64), P(u32),
                                   P(i32), vp]
        L.zpl_fit_scan.restype = i32
        L.zpl_fit_xmin.argtypes = [vp, vp, i64, i32, i64, P(d), P(d), P(i64), P(u32), vp]
        L.zpl_fit_xmin.restype = i32
        L.zpl_fit_noalloc.argtypes = [vp, vp, i64, u32, vp, vp, vp, vp, vp]
        L.zpl_fit_noalloc.restype = i32
        _lib = L
    return _lib


def exported_symbols() -> list:
    return ["zpl_create", "zpl_destroy", "zpl_last_error", "zpl_simulate_cells",
            "zpl_set_timing", "zpl_get_timing", "zpl_fit", "zpl_bootstrap_pvalue",
            "zpl_serve_start", "zpl_serve_submit", "zpl_serve_poll", "zpl_serve_stop",
            "zpl_sample_draws", "zpl_cdf_table", "zpl_autotune", "zpl_set_tuning",
            "zpl_plan_forms", "zpl_fit_truncated", "zpl_critical_table", "zpl_fit_scan",
            "zpl_fit_xmin", "zpl_fit_noalloc"]


FORM_NAMES = {FORM_LANE: "lane", FORM_WAVE: "wave", FORM_HEAVY: "heavy"}


def _tune_array(table) -> tuple:
    """A tuning table (list of dicts alpha, n, ns_per_replicate[3]) as a ctypes array."""
    if not table:
        return None, 0
    arr = (TuneEntry * len(table))()
    for k, e in enumerate(table):
        arr[k].alpha = float(e["alpha"])
        arr[k].n = int(e["n"])
        for f in range(3):
            arr[k].ns_per_replicate[f] = float(e["ns_per_replicate"][f])
    return arr, len(table)


def _tune_list(arr) -> list:
    return [{"alpha": e.alpha, "n": e.n, "ns_per_replicate": [e.ns_per_replicate[f] for f in range(3)]}
            for e in arr]


def plan_forms(cells: Sequence, table=None) -> list:
    """The planner's form ("lane" / "wave" / "heavy") for each cell under a
    tuning table (None: the built-in rule).  Host-only."""
    arr, cnt = _tune_array(table)
    cs = _cells(cells)
    out = (C.c_int32 * len(cs))()
    _check(lib().zpl_plan_forms(arr, cnt, cs, len(cs), out))
    return [FORM_NAMES[int(v)] for v in out]


def save_tuning(path, table):
    import json
    Path(path).write_text(json.dumps({"zpl_tuning": 1, "entries": table}, indent=1))


def load_tuning(path) -> list:
    import json
    doc = json.loads(Path(path).read_text())
    if doc.get("zpl_tuning") != 1:
        raise ValueError("%s is not a zpl tuning table" % path)
    return doc["entries"]


def _check(st: int):
    if st != OK:
        raise ZplError(st, lib().zpl_last_error().decode())


def _dptr(t) -> Optional[int]:
    if t is None:
        return None
    if not getattr(t, "is_cuda", False):
        raise ValueError("device buffers must be CUDA (HIP) tensors")
    if not t.is_contiguous():
        raise ValueError("device buffers must be contiguous")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


@dataclass
class CellSpec:
    alpha: float
    n: int
    replicates: int
    seed: int = 0
    stream: int = 0
    kmax: int = 0  # 0: pure law; K in 2..4096: truncated law on 1..K
    xmin: int = 0  # 0 or 1: none; else the pure law on k >= xmin


def cell_array(cells: Sequence) -> C.Array:
    """The cells (CellSpec, dict or tuple each) as a zpl_cell array.  Every
    call that takes cells also takes such an array as it is, so a caller that
    repeats a call converts its cells once."""
    if isinstance(cells, C.Array) and cells._type_ is Cell:
        return cells
    arr = (Cell * len(cells))()
    for i, c in enumerate(cells):
        if isinstance(c, dict):
            c = CellSpec(**c)
        elif not isinstance(c, CellSpec):
            c = CellSpec(*c)
        arr[i] = Cell(float(c.alpha), int(c.n), int(c.replicates), int(c.seed), int(c.stream),
                      int(c.kmax), int(c.xmin))
    return arr


_cells = cell_array


class Context:
    """One libzpl context on one HIP device."""

    def __init__(self, device: int = 0, mem_budget_bytes: int = 0):
        h = C.c_void_p()
        _check(lib().zpl_create(C.byref(h), int(device), int(mem_budget_bytes)))
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            lib().zpl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- zpl_simulate_cells -------------------------------------------------
    def simulate_cells(self, cells: Sequence, quantiles: Iterable = ((9, 10), (95, 100), (99, 100)),
                       d_out=None, alpha_hat_out=None, flags_out=None, fingerprint_out=None,
                       launch: str = "batched", form: str = "auto", use_graph: bool = False,
                       stream=None) -> Optional[np.ndarray]:
        cs = _cells(cells)
        q = list(quantiles) if quantiles is not None else []
        nq = len(q)
        qn = (C.c_uint32 * max(nq, 1))(*[a for a, _ in q])
        qd = (C.c_uint32 * max(nq, 1))(*[b for _, b in q])
        out = np.zeros((len(cs), max(nq, 1)))
        opts = SimOpts(_LAUNCH[launch], _FORMS[form], 1 if use_graph else 0, 0)
        _check(lib().zpl_simulate_cells(
            self._h, cs, len(cs), qn, qd, nq,
            out.ctypes.data_as(C.POINTER(C.c_double)) if nq else None,
            _dptr(d_out), _dptr(alpha_hat_out), _dptr(flags_out), _dptr(fingerprint_out),
            C.byref(opts), _stream(stream)))
        return out[:, :nq] if nq else None

    # -- zpl_critical_table -------------------------------------------------
    def critical_table(self, gammas: Sequence[float], ns: Sequence[int], kmax: int = 0,
                       seeds: int = 10, seed0: int = 1, replicates: int = 50000,
                       quantiles: Iterable = ((9, 10), (95, 100), (99, 100), (999, 1000)),
                       per_run: bool = False, stream=None):
        """A critical-value table as the paper's Tables 1-6 (zpl_critical_table):
        array [len(ns), len(gammas), n_q] of quantiles averaged over `seeds`
        runs; with per_run also the runs' own quantiles [.., .., seeds, n_q]."""
        g = (C.c_double * len(gammas))(*[float(v) for v in gammas])
        n = (C.c_int64 * len(ns))(*[int(v) for v in ns])
        q = list(quantiles)
        qn = (C.c_uint32 * len(q))(*[a for a, _ in q])
        qd = (C.c_uint32 * len(q))(*[b for _, b in q])
        tab = np.zeros((len(ns), len(gammas), len(q)))
        runs = np.zeros((len(ns), len(gammas), int(seeds), len(q))) if per_run else None
        dp = C.POINTER(C.c_double)
        _check(lib().zpl_critical_table(
            self._h, g, len(gammas), n, len(ns), int(kmax), int(seeds), int(seed0),
            int(replicates), qn, qd, len(q), tab.ctypes.data_as(dp),
            runs.ctypes.data_as(dp) if per_run else None, _stream(stream)))
        return (tab, runs) if per_run else tab

    # -- timing ---------------------------------------------------------------
    def autotune(self, alphas: Sequence[float], ns: Sequence[int], stream=None) -> list:
        """Measure every eligible form on the grid alphas x ns and install the
        table (zpl_autotune).  Returns it as a list of dicts, alpha-major."""
        a = (C.c_double * len(alphas))(*[float(v) for v in alphas])
        n = (C.c_int64 * len(ns))(*[int(v) for v in ns])
        out = (TuneEntry * (len(alphas) * len(ns)))()
        _check(lib().zpl_autotune(self._h, a, len(alphas), n, len(ns), out, _stream(stream)))
        return _tune_list(out)

    def set_tuning(self, table):
        """Install a saved table (None or [] removes it)."""
        arr, cnt = _tune_array(table)
        _check(lib().zpl_set_tuning(self._h, arr, cnt))

    def set_timing(self, enable: bool = True):
        _check(lib().zpl_set_timing(self._h, 1 if enable else 0))

    def timing(self) -> dict:
        """Milliseconds per kernel group of the last timed simulation."""
        ms = (C.c_double * 4)()
        _check(lib().zpl_get_timing(self._h, ms))
        return {"tables": ms[0], "simulate": ms[1], "heavy": ms[2], "select": ms[3]}

    # -- zpl_fit ------------------------------------------------------------
    def fit(self, x, kmax: int = 0, xmin: int = 1, stream=None) -> dict:
        """zpl_fit (kmax = 0), zpl_fit_truncated (kmax = K) or zpl_fit_xmin
        (xmin > 1: the values >= xmin under the law with that cutoff)."""
        ptr, n, on_dev, keep = _xarg(x)
        a, D, f = C.c_double(), C.c_double(), C.c_uint32()
        if xmin > 1:
            if kmax:
                raise ValueError("xmin > 1 needs the pure law (kmax = 0)")
            m = C.c_int64()
            st = lib().zpl_fit_xmin(self._h, ptr, n, on_dev, int(xmin), C.byref(a), C.byref(D),
                                    C.byref(m), C.byref(f), _stream(stream))
            del keep
            if st not in (OK, ENOCONV):
                _check(st)
            return {"alpha_hat": a.value, "D": D.value, "flags": f.value, "status": st,
                    "n_tail": m.value}
        if kmax:
            st = lib().zpl_fit_truncated(self._h, ptr, n, on_dev, int(kmax), C.byref(a),
                                         C.byref(D), C.byref(f), _stream(stream))
        else:
            st = lib().zpl_fit(self._h, ptr, n, on_dev, C.byref(a), C.byref(D), C.byref(f),
                               _stream(stream))
        del keep
        if st not in (OK, ENOCONV):
            _check(st)
        return {"alpha_hat": a.value, "D": D.value, "flags": f.value, "status": st}

    # -- zpl_fit_noalloc ----------------------------------------------------
    def fit_noalloc(self, x, alpha_hat_out, D_out, flags_out, status_out, kmax: int = 0,
                    stream=None):
        """zpl_fit_noalloc: enqueue the fit of the device dataset x (int64
        tensor) into the one-element device tensors alpha_hat_out, D_out
        (float64), flags_out and status_out (int32/uint32); no allocation, no
        synchronisation."""
        import torch
        if not getattr(x, "is_cuda", False) or x.dtype != torch.int64 or not x.is_contiguous():
            raise ValueError("x must be a contiguous int64 device tensor")
        for t, dt in ((alpha_hat_out, torch.float64), (D_out, torch.float64),
                      (flags_out, torch.int32), (status_out, torch.int32)):
            if t.dtype not in (dt, torch.uint32) or t.numel() < 1:
                raise ValueError("outputs: one-element float64 / int32 device tensors")
        _check(lib().zpl_fit_noalloc(self._h, C.c_void_p(x.data_ptr()), int(x.numel()),
                                     int(kmax), C.c_void_p(_dptr(alpha_hat_out)),
                                     C.c_void_p(_dptr(D_out)), C.c_void_p(_dptr(flags_out)),
                                     C.c_void_p(_dptr(status_out)), _stream(stream)))

    # -- zpl_bootstrap_pvalue -----------------------------------------------
    def bootstrap_pvalue(self, x, B: int, seed: int, stream_id: int = 0, stream=None) -> dict:
        ptr, n, on_dev, keep = _xarg(x)
        a, D, p, f = C.c_double(), C.c_double(), C.c_double(), C.c_uint32()
        st = lib().zpl_bootstrap_pvalue(self._h, ptr, n, on_dev, int(B), int(seed),
                                        int(stream_id), C.byref(a), C.byref(D), C.byref(p),
                                        C.byref(f), _stream(stream))
        del keep
        _check(st)
        return {"alpha_hat": a.value, "D": D.value, "p_value": p.value, "flags": f.value}

    # -- serving (continuous batching) ---------------------------------------
    def serve_start(self, mem_budget_bytes: int = 0, max_batch: int = 0, max_queue: int = 0,
                    slice_us: int = 0):
        o = ServeOpts(int(mem_budget_bytes), int(max_batch), int(max_queue), int(slice_us), 0)
        _check(lib().zpl_serve_start(self._h, C.byref(o)))

    def serve_submit(self, x, B: int, seed: int, stream_id: int = 0) -> int:
        """Queue a request; x is a host array or an int64 device tensor."""
        ptr, n, on_dev, keep = _xarg(x)
        t = C.c_uint64()
        st = lib().zpl_serve_submit(self._h, ptr, n, on_dev, int(B), int(seed), int(stream_id),
                                    C.byref(t))
        del keep
        _check(st)
        return t.value

    def serve_poll(self, ticket: int, wait_ms: int = 0) -> Optional[dict]:
        r = ServeResult()
        _check(lib().zpl_serve_poll(self._h, int(ticket), int(wait_ms), C.byref(r)))
        if not r.done:
            return None
        return {"status": r.status, "alpha_hat": r.alpha_hat, "D": r.D, "p_value": r.p_value,
                "flags": r.flags, "batch_size": r.batch_size, "queue_ms": r.queue_ms,
                "latency_ms": r.latency_ms, "launches": r.launches}

    def serve_stop(self):
        _check(lib().zpl_serve_stop(self._h))

    # -- zpl_sample_draws / zpl_cdf_table -----------------------------------
    def sample_draws(self, alpha: float, n: int, seed: int, stream_id: int, rep_lo: int,
                     count: int, x_out, flags_out, kmax: int = 0, xmin: int = 1, stream=None):
        _check(lib().zpl_sample_draws(self._h, float(alpha), int(kmax), int(xmin), int(n),
                                      int(seed), int(stream_id), int(rep_lo), int(count),
                                      _dptr(x_out), _dptr(flags_out), _stream(stream)))

    def cdf_table(self, alpha: float, T_out, kmax: int = 0, xmin: int = 1, stream=None):
        _check(lib().zpl_cdf_table(self._h, float(alpha), int(kmax), int(xmin), _dptr(T_out),
                                   _stream(stream)))

    # -- zpl_fit_scan ---------------------------------------------------------
    def fit_scan(self, x, xmins: Sequence[int], stream=None) -> dict:
        """The KS-minimising lower cutoff among the candidates (zpl_fit_scan):
        per-candidate alpha_hat, D, n_tail, flags and the index `best`."""
        ptr, n, on_dev, keep = _xarg(x)
        c = np.ascontiguousarray(np.asarray(xmins), dtype=np.int64)
        k = int(c.size)
        A, D = np.zeros(k), np.zeros(k)
        M = np.zeros(k, dtype=np.int64)
        F = np.zeros(k, dtype=np.uint32)
        best = C.c_int32()
        P = C.POINTER
        _check(lib().zpl_fit_scan(
            self._h, ptr, n, on_dev, c.ctypes.data_as(P(C.c_int64)), k,
            A.ctypes.data_as(P(C.c_double)), D.ctypes.data_as(P(C.c_double)),
            M.ctypes.data_as(P(C.c_int64)), F.ctypes.data_as(P(C.c_uint32)), C.byref(best),
            _stream(stream)))
        del keep
        return {"best": best.value, "alpha_hat": A, "D": D, "n_tail": M, "flags": F}


def _xarg(x):
    """(pointer, n, on_device, keepalive) for an int64 dataset."""
    if getattr(x, "is_cuda", False):
        import torch
        if x.dtype != torch.int64:
            raise ValueError("x must be int64")
        x = x.contiguous()
        return C.c_void_p(x.data_ptr()), int(x.numel()), 1, x
    a = np.ascontiguousarray(np.asarray(x), dtype=np.int64)
    return C.c_void_p(a.ctypes.data), int(a.size), 0, a
