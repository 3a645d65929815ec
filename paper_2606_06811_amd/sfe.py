"""Python binding of libsfe.so (include/sfe.h): argument marshalling only.

Every step of the computation runs in the HIP library; this module converts
numpy arrays / torch tensors to the C structs and pointers and back.  If the
library is not built the import of the product path fails loudly: there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfe.so")
_lib = None

SFE_OK, SFE_EINVAL, SFE_ENOMEM, SFE_ECAPACITY, SFE_ERANGE, SFE_EDEVICE, SFE_EINTERNAL, SFE_EIO = \
    0, -1, -2, -3, -4, -5, -6, -7
SFE_XDROP_RAW = 1
SFE_ALN_PASSED = 1
SFE_SCHED_PLAIN, SFE_SCHED_PERSISTENT, SFE_SCHED_ADAPTIVE, SFE_SCHED_BINNED = 0, 1, 2, 3
SFE_POLICY_DEFER, SFE_POLICY_PREFIX = 0, 1
SFE_FILTER_XDROP, SFE_FILTER_YDROP = 0, 1

HIT_DTYPE = np.dtype([("t", "<u4"), ("q", "<u4"), ("query_id", "<u4"), ("strand", "u1"), ("pad", "u1", (3,))])
HSP_DTYPE = np.dtype([("t0", "<u4"), ("q0", "<u4"), ("len", "<u4"), ("score", "<i4"), ("query_id", "<u4"),
                      ("strand", "u1"), ("pad", "u1", (3,))])
ALN_DTYPE = np.dtype([("t_start", "<u4"), ("t_end", "<u4"), ("q_start", "<u4"), ("q_end", "<u4"),
                      ("score", "<i4"), ("query_id", "<u4"), ("anchor_t", "<u4"), ("anchor_q", "<u4"),
                      ("ops_offset", "<u8"), ("cells", "<u8"), ("ops_len", "<u4"), ("strand", "u1"),
                      ("flags", "u1"), ("pad", "u1", (2,))])
assert HIT_DTYPE.itemsize == 16 and HSP_DTYPE.itemsize == 24 and ALN_DTYPE.itemsize == 56


class SfeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"sfe status {status}: {msg}")
        self.status = status


class _Seq(ctypes.Structure):
    _fields_ = [("residues", ctypes.c_void_p), ("length", ctypes.c_int64)]


class _SeedSpec(ctypes.Structure):
    _fields_ = [("pattern", ctypes.c_char_p), ("transitions", ctypes.c_int32), ("step", ctypes.c_int32)]


class _Scoring(ctypes.Structure):
    _fields_ = [("sub", ctypes.c_int32 * 25), ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32),
                ("xdrop", ctypes.c_int32), ("hsp_thresh", ctypes.c_int32), ("ydrop", ctypes.c_int32),
                ("gapped_thresh", ctypes.c_int32)]


class _AlignOpts(ctypes.Structure):
    _fields_ = [("round_k", ctypes.c_int32), ("schedule", ctypes.c_int32), ("strands", ctypes.c_int32),
                ("max_cells_per_lane", ctypes.c_int32), ("policy", ctypes.c_int32), ("near_band", ctypes.c_int32),
                ("arena_bytes", ctypes.c_int64), ("model", ctypes.c_void_p), ("filter", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class _Tuning(ctypes.Structure):
    _fields_ = [("wave_group_cap", ctypes.c_int32), ("use_graphs", ctypes.c_int32), ("wide_scores", ctypes.c_int32),
                ("persist_waves_per_cu", ctypes.c_int32), ("adaptive_halves", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


class _TuneEntry(ctypes.Structure):
    _fields_ = [("cells_per_lane", ctypes.c_int32), ("schedule", ctypes.c_int32), ("wave_group_cap", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("ms_extend", ctypes.c_double)]


class _TuneReport(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("best", ctypes.c_int32), ("entries", _TuneEntry * 32)]


class _Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("seed_hits", "hsps_raw", "hsps", "rounds", "extensions", "committed",
                                               "shadow", "cells", "overflow_reruns", "xdrop_columns",
                                               "ydrop_launches", "ydrop_kernel_cells", "seed_xdrop_launches")] + \
               [(n, ctypes.c_double) for n in ("ms_seed_xdrop", "ms_hsp_set", "ms_extend", "ms_total",
                                               "ms_ydrop_kernel", "ms_seed_xdrop_kernel")] + \
               [("predicted_halves", ctypes.c_int64), ("mispredicted_halves", ctypes.c_int64),
                ("ms_predict", ctypes.c_double), ("narrow_launches", ctypes.c_int64),
                ("graph_launches", ctypes.c_int64), ("graph_records", ctypes.c_int64)]

MLP_NFEAT, MLP_NOUT, MLP_NPARAMS = 16, 4, 9668
NOALLOC_MAX_SAMPLES = 16384


def lib():
    """The loaded libsfe.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.sfe_ctx_create.argtypes = [ctypes.c_int, P, ctypes.POINTER(P)]
        L.sfe_ctx_destroy.argtypes = [P]
        L.sfe_build_index.argtypes = [P, ctypes.POINTER(_Seq), ctypes.POINTER(_SeedSpec), ctypes.POINTER(P)]
        L.sfe_index_destroy.argtypes = [P]
        L.sfe_seed_hits.argtypes = [P, P, ctypes.POINTER(_Seq), I32, I32, P, I64, ctypes.POINTER(I64)]
        L.sfe_ungapped_xdrop.argtypes = [P, P, ctypes.POINTER(_Seq), I32, P, I64, ctypes.POINTER(_Scoring), I32, P,
                                         I64, ctypes.POINTER(I64)]
        L.sfe_gapped_ydrop.argtypes = [P, P, ctypes.POINTER(_Seq), I32, P, I64, ctypes.POINTER(_Scoring), P, P, I64,
                                       ctypes.POINTER(I64)]
        L.sfe_align.argtypes = [P, P, ctypes.POINTER(_Seq), I32, ctypes.POINTER(_Scoring), ctypes.POINTER(_AlignOpts),
                                P, I64, ctypes.POINTER(I64), P, I64, ctypes.POINTER(I64), ctypes.POINTER(_Stats)]
        L.sfe_ctx_set_tuning.argtypes = [P, ctypes.POINTER(_Tuning)]
        L.sfe_ctx_get_tuning.argtypes = [P, ctypes.POINTER(_Tuning)]
        L.sfe_autotune.argtypes = [P, P, ctypes.POINTER(_Seq), I32, ctypes.POINTER(_Scoring), I64,
                                   ctypes.POINTER(_AlignOpts), ctypes.POINTER(_TuneReport)]
        L.sfe_hsp_features.argtypes = [P, P, ctypes.POINTER(_Seq), I32, P, I64, P]
        L.sfe_extension_log.argtypes = [P, P, ctypes.POINTER(_Seq), I32, P, I64, ctypes.POINTER(_Scoring), P, P]
        L.sfe_model_create.argtypes = [P, P, ctypes.POINTER(P)]
        L.sfe_model_destroy.argtypes = [P]
        L.sfe_model_params.argtypes = [P, P]
        L.sfe_model_predict.argtypes = [P, P, I64, P]
        L.sfe_model_grad.argtypes = [P, P, P, I64, P, P]
        L.sfe_model_train.argtypes = [P, P, P, I64, P, I64, I32, ctypes.c_float, P]
        L.sfe_model_grad_noalloc.argtypes = [P, P, P, I64, P, P]
        L.sfe_model_save.argtypes = [P, ctypes.c_char_p]
        L.sfe_model_load.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(P)]
        L.sfe_align_opts_resolve.argtypes = [ctypes.POINTER(_AlignOpts), ctypes.POINTER(_AlignOpts)]
        L.sfe_status_str.argtypes = [I32]
        L.sfe_status_str.restype = ctypes.c_char_p
        L.sfe_last_error.argtypes = [P]
        L.sfe_last_error.restype = ctypes.c_char_p
        for f in ("sfe_ctx_create", "sfe_build_index", "sfe_seed_hits", "sfe_ungapped_xdrop", "sfe_gapped_ydrop",
                  "sfe_align", "sfe_ctx_set_tuning", "sfe_ctx_get_tuning", "sfe_autotune", "sfe_hsp_features", "sfe_extension_log", "sfe_model_create", "sfe_model_params",
                  "sfe_model_predict", "sfe_model_grad", "sfe_model_train", "sfe_model_save", "sfe_model_load",
                  "sfe_align_opts_resolve", "sfe_model_grad_noalloc"):
            getattr(L, f).restype = I32
        _lib = L
    return _lib


def _check(st, ctx=None):
    if st != SFE_OK:
        msg = lib().sfe_last_error(ctx.ptr if ctx is not None else None)
        raise SfeError(st, msg.decode() if msg else "")


def _ptr(a):
    """Raw address of a numpy array or a torch tensor (host or device)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _seq_arrays(seqs):
    """Keeps the residue buffers alive and builds the sfe_seq array."""
    keep = []
    arr = (_Seq * max(1, len(seqs)))()
    for i, s in enumerate(seqs):
        if isinstance(s, (bytes, bytearray)):
            s = np.frombuffer(bytes(s), dtype=np.uint8)
        if hasattr(s, "data_ptr"):
            n = s.numel()
        else:
            s = np.ascontiguousarray(s, dtype=np.uint8)
            n = s.shape[0]
        keep.append(s)
        arr[i].residues = _ptr(s) if n else None
        arr[i].length = n
    return arr, keep


def scoring_struct(d: dict) -> _Scoring:
    s = _Scoring()
    flat = [int(v) for row in d["sub"] for v in row]
    for i, v in enumerate(flat):
        s.sub[i] = v
    for f in ("gap_open", "gap_extend", "xdrop", "hsp_thresh", "ydrop", "gapped_thresh"):
        setattr(s, f, int(d[f]))
    return s


class Context:
    def __init__(self, device: int = 0, stream=None):
        import weakref
        p = ctypes.c_void_p()
        _check(lib().sfe_ctx_create(int(device), stream, ctypes.byref(p)))
        self.ptr = p
        self._children = weakref.WeakSet()      # models and indexes: closed before the context

    def close(self):
        if self.ptr:
            for ch in list(self._children):
                ch.close()
            lib().sfe_ctx_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Index:
    def __init__(self, ctx: Context, ptr, nt: int):
        self.ctx, self.ptr, self.nt = ctx, ptr, nt
        ctx._children.add(self)

    def close(self):
        if self.ptr:
            lib().sfe_index_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sfe_ctx_create(device: int = 0, stream=None) -> Context:
    return Context(device, stream)


def sfe_ctx_set_tuning(ctx: Context, wave_group_cap: int = 0, use_graphs: int = 0, wide_scores: int = 0,
                       persist_waves_per_cu: int = 0, adaptive_halves: int = 0):
    t = _Tuning()
    t.wave_group_cap = int(wave_group_cap)
    t.use_graphs = int(use_graphs)
    t.wide_scores = int(wide_scores)
    t.persist_waves_per_cu = int(persist_waves_per_cu)
    t.adaptive_halves = int(adaptive_halves)
    _check(lib().sfe_ctx_set_tuning(ctx.ptr, ctypes.byref(t)), ctx)


def sfe_ctx_get_tuning(ctx: Context) -> dict:
    t = _Tuning()
    _check(lib().sfe_ctx_get_tuning(ctx.ptr, ctypes.byref(t)), ctx)
    return {"wave_group_cap": t.wave_group_cap, "use_graphs": t.use_graphs, "wide_scores": t.wide_scores,
            "persist_waves_per_cu": t.persist_waves_per_cu, "adaptive_halves": t.adaptive_halves}


def sfe_autotune(ctx: Context, idx: Index, queries, scoring: dict, sample_bases: int, model=None,
                 round_k: int = 0, policy: int = SFE_POLICY_DEFER):
    """Returns (chosen {max_cells_per_lane, schedule, wave_group_cap}, list of candidate timings)."""
    seqs, keep = _seq_arrays(queries)
    sc = scoring_struct(scoring)
    opts = _AlignOpts(int(round_k), SFE_SCHED_PLAIN, 3, 0, int(policy), 0, 0,
                      model.ptr if model is not None else None, SFE_FILTER_XDROP, 0)
    rep = _TuneReport()
    _check(lib().sfe_autotune(ctx.ptr, idx.ptr, seqs, len(queries), ctypes.byref(sc), int(sample_bases),
                              ctypes.byref(opts), ctypes.byref(rep)), ctx)
    entries = [dict(cells_per_lane=e.cells_per_lane, schedule=e.schedule, wave_group_cap=e.wave_group_cap,
                    waves_per_cu=e.waves_per_cu, ms_extend=e.ms_extend) for e in rep.entries[:rep.n]]
    tun = sfe_ctx_get_tuning(ctx)
    chosen = dict(max_cells_per_lane=opts.max_cells_per_lane, schedule=opts.schedule,
                  wave_group_cap=tun["wave_group_cap"], persist_waves_per_cu=tun["persist_waves_per_cu"])
    return chosen, entries


def sfe_build_index(ctx: Context, target, pattern: str = "1110100110010101111", transitions: int = 1,
                    step: int = 1) -> Index:
    seqs, keep = _seq_arrays([target])
    spec = _SeedSpec(pattern.encode(), int(transitions), int(step))
    p = ctypes.c_void_p()
    _check(lib().sfe_build_index(ctx.ptr, seqs, ctypes.byref(spec), ctypes.byref(p)), ctx)
    return Index(ctx, p, seqs[0].length)


def _two_call(fn, dtype, guess):
    """Runs fn(buffer, cap) -> (status, needed) with the capacity protocol."""
    cap = max(int(guess), 1)
    while True:
        buf = np.zeros(cap, dtype)
        st, need = fn(buf, cap)
        if st == SFE_ECAPACITY and need > cap:
            cap = need
            continue
        return st, buf[:need] if st == SFE_OK else buf[:0], need


def sfe_seed_hits(ctx: Context, idx: Index, queries, strands: int = 3) -> np.ndarray:
    seqs, keep = _seq_arrays(queries)
    n = ctypes.c_int64()

    def fn(buf, cap):
        st = lib().sfe_seed_hits(ctx.ptr, idx.ptr, seqs, len(queries), int(strands), _ptr(buf), cap, ctypes.byref(n))
        return st, n.value

    st, out, _ = _two_call(fn, HIT_DTYPE, 1 << 16)
    _check(st, ctx)
    return out


def sfe_ungapped_xdrop(ctx: Context, idx: Index, queries, hits: np.ndarray, scoring: dict, raw: bool = False):
    seqs, keep = _seq_arrays(queries)
    hits = np.ascontiguousarray(hits, HIT_DTYPE)
    sc = scoring_struct(scoring)
    n = ctypes.c_int64()

    def fn(buf, cap):
        st = lib().sfe_ungapped_xdrop(ctx.ptr, idx.ptr, seqs, len(queries), _ptr(hits), hits.shape[0],
                                      ctypes.byref(sc), SFE_XDROP_RAW if raw else 0, _ptr(buf), cap, ctypes.byref(n))
        return st, n.value

    st, out, _ = _two_call(fn, HSP_DTYPE, max(hits.shape[0], 1) if raw else 1 << 14)
    _check(st, ctx)
    return out


def sfe_gapped_ydrop(ctx: Context, idx: Index, queries, hsps: np.ndarray, scoring: dict):
    seqs, keep = _seq_arrays(queries)
    hsps = np.ascontiguousarray(hsps, HSP_DTYPE)
    sc = scoring_struct(scoring)
    out = np.zeros(hsps.shape[0], ALN_DTYPE)
    n = ctypes.c_int64()
    cap = 1 << 16
    while True:
        ops = np.zeros(cap, np.uint32)
        st = lib().sfe_gapped_ydrop(ctx.ptr, idx.ptr, seqs, len(queries), _ptr(hsps), hsps.shape[0],
                                    ctypes.byref(sc), _ptr(out), _ptr(ops), cap, ctypes.byref(n))
        if st == SFE_ECAPACITY and n.value > cap:
            cap = n.value
            continue
        _check(st, ctx)
        return out, ops[:n.value]


def sfe_align(ctx: Context, idx: Index, queries, scoring: dict, round_k: int = 0, schedule: int = SFE_SCHED_PLAIN,
              strands: int = 3, max_cells_per_lane: int = 0, arena_bytes: int = 0, policy: int = SFE_POLICY_DEFER,
              cap: int = 1 << 12, ops_cap: int = 1 << 18, model=None, near_band: int = 0,
              filter: int = SFE_FILTER_XDROP):
    """Whole pipeline; returns (alignments, ops, stats dict).  When the results
    do not fit cap / ops_cap the call is made again with the sizes the library
    reported (the whole pipeline runs twice), so size them generously."""
    seqs, keep = _seq_arrays(queries)
    sc = scoring_struct(scoring)
    opts = _AlignOpts(int(round_k), int(schedule), int(strands), int(max_cells_per_lane), int(policy),
                      int(near_band), int(arena_bytes), model.ptr if model is not None else None, int(filter), 0)
    na, no = ctypes.c_int64(), ctypes.c_int64()
    stats = _Stats()
    while True:
        out = np.zeros(cap, ALN_DTYPE)
        ops = np.zeros(ops_cap, np.uint32)
        st = lib().sfe_align(ctx.ptr, idx.ptr, seqs, len(queries), ctypes.byref(sc), ctypes.byref(opts),
                             _ptr(out), cap, ctypes.byref(na), _ptr(ops), ops_cap, ctypes.byref(no),
                             ctypes.byref(stats))
        if st == SFE_ECAPACITY and (na.value > cap or no.value > ops_cap):
            cap, ops_cap = max(cap, na.value), max(ops_cap, no.value)
            continue
        _check(st, ctx)
        s = {f: getattr(stats, f) for f, _ in _Stats._fields_}
        return out[:na.value], ops[:no.value], s


def sfe_align_opts_resolve(round_k: int = 0, schedule: int = SFE_SCHED_PLAIN, strands: int = 0,
                           max_cells_per_lane: int = 0, policy: int = SFE_POLICY_DEFER, near_band: int = 0,
                           arena_bytes: int = 0, filter: int = SFE_FILTER_XDROP) -> dict:
    """The options sfe_align would run with (host only; raises SfeError on invalid ones)."""
    o = _AlignOpts(int(round_k), int(schedule), int(strands), int(max_cells_per_lane), int(policy),
                   int(near_band), int(arena_bytes), None, int(filter), 0)
    r = _AlignOpts()
    st = lib().sfe_align_opts_resolve(ctypes.byref(o), ctypes.byref(r))
    if st != SFE_OK:
        raise SfeError(st, "invalid sfe_align options")
    return {f: getattr(r, f) for f, _ in _AlignOpts._fields_ if f not in ("model", "pad")}


def sfe_model_check_file(path: str) -> int:
    """Status of sfe_model_load's file check alone (no device): SFE_OK, SFE_EINVAL or SFE_EIO."""
    return int(lib().sfe_model_load(None, os.fsencode(path), None))


def _f32(a, shape=None):
    if hasattr(a, "data_ptr"):
        return a
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None:
        a = a.reshape(shape)
    return a


def sfe_hsp_features(ctx: Context, idx: Index, queries, hsps: np.ndarray) -> np.ndarray:
    seqs, keep = _seq_arrays(queries)
    hsps = np.ascontiguousarray(hsps, HSP_DTYPE)
    out = np.zeros((hsps.shape[0], MLP_NFEAT), np.float32)
    _check(lib().sfe_hsp_features(ctx.ptr, idx.ptr, seqs, len(queries), _ptr(hsps), hsps.shape[0], _ptr(out)), ctx)
    return out


def sfe_extension_log(ctx: Context, idx: Index, queries, hsps: np.ndarray, scoring: dict):
    """(features n x 16, targets n x 4) of the plain pipeline's extensions of `hsps`."""
    seqs, keep = _seq_arrays(queries)
    hsps = np.ascontiguousarray(hsps, HSP_DTYPE)
    sc = scoring_struct(scoring)
    f = np.zeros((hsps.shape[0], MLP_NFEAT), np.float32)
    t = np.zeros((hsps.shape[0], MLP_NOUT), np.float32)
    _check(lib().sfe_extension_log(ctx.ptr, idx.ptr, seqs, len(queries), _ptr(hsps), hsps.shape[0],
                                   ctypes.byref(sc), _ptr(f), _ptr(t)), ctx)
    return f, t


class Model:
    """The cost model's parameters on the device of `ctx`."""

    def __init__(self, ctx: Context, params):
        self.ctx = ctx
        params = _f32(params)
        if not hasattr(params, "data_ptr") and params.shape != (MLP_NPARAMS,):
            raise ValueError(f"need {MLP_NPARAMS} parameters")
        p = ctypes.c_void_p()
        _check(lib().sfe_model_create(ctx.ptr, _ptr(params), ctypes.byref(p)), ctx)
        self.ptr = p
        ctx._children.add(self)

    def params(self) -> np.ndarray:
        out = np.zeros(MLP_NPARAMS, np.float32)
        _check(lib().sfe_model_params(self.ptr, _ptr(out)), self.ctx)
        return out

    def predict(self, x) -> np.ndarray:
        x = _f32(x, (-1, MLP_NFEAT))
        out = np.zeros((x.shape[0], MLP_NOUT), np.float32)
        _check(lib().sfe_model_predict(self.ptr, _ptr(x), x.shape[0], _ptr(out)), self.ctx)
        return out

    def grad(self, x, t):
        x = _f32(x, (-1, MLP_NFEAT))
        t = _f32(t, (-1, MLP_NOUT))
        g = np.zeros(MLP_NPARAMS, np.float32)
        loss = np.zeros(1, np.float32)
        _check(lib().sfe_model_grad(self.ptr, _ptr(x), _ptr(t), x.shape[0], _ptr(g), _ptr(loss)), self.ctx)
        return float(loss[0]), g

    def grad_noalloc(self, x, t, grad, loss):
        """sfe_model_grad_noalloc on device tensors (x n x 16, t n x 4, grad 9668, loss 1, float32);
        ordered on the context's stream, returns without waiting."""
        _check(lib().sfe_model_grad_noalloc(self.ptr, _ptr(x), _ptr(t), int(x.shape[0]), _ptr(grad), _ptr(loss)),
               self.ctx)

    def train(self, x, t, order, batch: int, lr: float) -> np.ndarray:
        x = _f32(x, (-1, MLP_NFEAT))
        t = _f32(t, (-1, MLP_NOUT))
        order = np.ascontiguousarray(order, np.int32)
        steps = (order.shape[0] + batch - 1) // batch
        losses = np.zeros(max(steps, 1), np.float32)
        _check(lib().sfe_model_train(self.ptr, _ptr(x), _ptr(t), x.shape[0], _ptr(order), order.shape[0],
                                     int(batch), float(lr), _ptr(losses)), self.ctx)
        return losses[:steps]

    def save(self, path: str):
        _check(lib().sfe_model_save(self.ptr, os.fsencode(path)), self.ctx)

    @classmethod
    def load(cls, ctx: Context, path: str) -> "Model":
        p = ctypes.c_void_p()
        _check(lib().sfe_model_load(ctx.ptr, os.fsencode(path), ctypes.byref(p)), ctx)
        m = cls.__new__(cls)
        m.ctx, m.ptr = ctx, p
        ctx._children.add(m)
        return m

    def close(self):
        if self.ptr:
            lib().sfe_model_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
