"""CPU oracle of the seed -> X-drop -> Y-drop pipeline.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product library never does, and
this package imports nothing from the product.  The arithmetic lives in the
plain C file ``oracle.c`` (single-threaded, one obviously-correct loop per
definition); this module marshals numpy arrays and performs the two library
steps the method leaves to a sort: collapsing duplicate HSPs and putting them
in the order the serial algorithm walks them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

NEG = -(1 << 30)


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (the checker, not the product)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


class Scoring(ctypes.Structure):
    _fields_ = [("sub", ctypes.c_int32 * 25), ("gap_open", ctypes.c_int32),
                ("gap_extend", ctypes.c_int32), ("xdrop", ctypes.c_int32),
                ("hsp_thresh", ctypes.c_int32), ("ydrop", ctypes.c_int32),
                ("gapped_thresh", ctypes.c_int32)]


class Half(ctypes.Structure):
    _fields_ = [("best", ctypes.c_int32), ("pad", ctypes.c_int32), ("i_end", ctypes.c_int64),
                ("j_end", ctypes.c_int64), ("cells", ctypes.c_int64), ("n_ops", ctypes.c_int64)]


HSP_DTYPE = np.dtype([("t0", "<i8"), ("q0", "<i8"), ("len", "<i8"), ("score", "<i8"), ("work", "<i8")])
ALN_DTYPE = np.dtype([("t_start", "<i8"), ("t_end", "<i8"), ("q_start", "<i8"), ("q_end", "<i8"),
                      ("score", "<i8"), ("anchor_t", "<i8"), ("anchor_q", "<i8"), ("cells", "<i8"),
                      ("ops_off", "<i8"), ("ops_len", "<i8"), ("query_id", "<i4"), ("strand", "<i4")])


class Result(ctypes.Structure):
    _fields_ = [("alns", ctypes.c_void_p), ("n_alns", ctypes.c_int64), ("cap_alns", ctypes.c_int64),
                ("ops", ctypes.c_void_p), ("n_ops", ctypes.c_int64), ("cap_ops", ctypes.c_int64),
                ("n_extensions", ctypes.c_int64), ("ext_cells", ctypes.c_int64)]


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        I64, I32 = ctypes.c_int64, ctypes.c_int32
        _lib.orc_encode.argtypes = [P, I64, P, P]
        _lib.orc_encode.restype = ctypes.c_int
        _lib.orc_revcomp.argtypes = [P, P, I64, P, P]
        _lib.orc_seed_hits.argtypes = [P, P, I64, P, P, I64, ctypes.c_char_p, I32, I32, P, P, I64]
        _lib.orc_seed_hits.restype = I64
        _lib.orc_xdrop_batch.argtypes = [P, I64, P, I64, P, P, I64, I32, P, P]
        _lib.orc_ydrop_half.argtypes = [P, I64, P, I64, P, P, P, I64]
        _lib.orc_ydrop_half.restype = I64
        _lib.orc_extend.argtypes = [P, I64, P, I64, I64, I64, P, P, P, I64]
        _lib.orc_extend.restype = I64
        _lib.orc_commit_unit.argtypes = [P, I64, P, I64, P, I64, P, I64, I32, I32, P]
        _lib.orc_result_new.restype = ctypes.POINTER(Result)
        _lib.orc_result_free.argtypes = [ctypes.POINTER(Result)]
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def scoring(d: dict) -> Scoring:
    s = Scoring()
    flat = [int(v) for row in d["sub"] for v in row]
    assert len(flat) == 25
    for i, v in enumerate(flat):
        s.sub[i] = v
    for f in ("gap_open", "gap_extend", "xdrop", "hsp_thresh", "ydrop", "gapped_thresh"):
        setattr(s, f, int(d[f]))
    return s


def encode(txt) -> tuple[np.ndarray, np.ndarray]:
    """ASCII letters -> (codes 0..4, soft-mask flags)."""
    a = np.ascontiguousarray(np.frombuffer(bytes(txt), dtype=np.uint8) if not isinstance(txt, np.ndarray) else txt,
                             dtype=np.uint8)
    code = np.empty(a.shape[0], np.uint8)
    soft = np.empty(a.shape[0], np.uint8)
    if lib().orc_encode(_p(a), a.shape[0], _p(code), _p(soft)) != 0:
        raise ValueError("sequence holds a letter outside ACGTN / IUPAC")
    return code, soft


def revcomp(code: np.ndarray, soft: np.ndarray):
    rc = np.empty_like(code)
    rs = np.empty_like(soft)
    lib().orc_revcomp(_p(code), _p(soft), code.shape[0], _p(rc), _p(rs))
    return rc, rs


def pattern_span(pattern: str) -> int:
    return len(pattern)


def seed_hits(tc, ts, qc, qs, pattern, transitions=1, step=1):
    """All (t, q) hits of one query strand, ordered by (q, t)."""
    n = lib().orc_seed_hits(_p(tc), _p(ts), tc.shape[0], _p(qc), _p(qs), qc.shape[0],
                            pattern.encode(), transitions, step, None, None, 0)
    if n < 0:
        raise ValueError("bad seed pattern")
    t = np.empty(n, np.uint32)
    q = np.empty(n, np.uint32)
    lib().orc_seed_hits(_p(tc), _p(ts), tc.shape[0], _p(qc), _p(qs), qc.shape[0],
                        pattern.encode(), transitions, step, _p(t), _p(q), n)
    return t, q


def xdrop(tc, qc, t, q, span, sc: dict) -> np.ndarray:
    """X-drop HSP of every hit (t[x], q[x]) on one strand."""
    t = np.ascontiguousarray(t, np.uint32)
    q = np.ascontiguousarray(q, np.uint32)
    out = np.empty(t.shape[0], HSP_DTYPE)
    s = scoring(sc)
    lib().orc_xdrop_batch(_p(tc), tc.shape[0], _p(qc), qc.shape[0], _p(t), _p(q), t.shape[0], span,
                          ctypes.byref(s), _p(out))
    return out


def ydrop_filter(tc, qc, t, q, span, sc: dict) -> np.ndarray:
    """The two-dimensional filter proposed in place of X-drop (Sec. 8, Sec. 9):
    both gapped halves around the middle column of each hit's seed window,
    pruned with Y := the X-drop value; the hit's window becomes an HSP carrying
    that total (kept when it reaches the HSP threshold, as X-drop HSPs are)."""
    fsc = dict(sc)
    fsc["ydrop"] = sc["xdrop"]
    off = (span - 1) // 2
    out = np.zeros(np.asarray(t).shape[0], HSP_DTYPE)
    for x in range(out.shape[0]):
        a, _ = extend(tc, qc, int(t[x]) + off, int(q[x]) + off, fsc)
        out[x] = (int(t[x]), int(q[x]), span, int(a["score"]), int(a["cells"]))
    return out


def hsp_set(hsps: np.ndarray, hsp_thresh: int) -> np.ndarray:
    """Passing HSPs of one (query, strand) unit, exact duplicates collapsed,
    in the order the serial algorithm walks them: score descending, then
    t0, q0, len ascending."""
    h = hsps[hsps["score"] >= hsp_thresh]
    if h.shape[0] == 0:
        return h.copy()
    key = np.stack([h["t0"], h["q0"], h["len"]], axis=1)
    _, first = np.unique(key, axis=0, return_index=True)
    h = h[np.sort(first)]
    order = np.lexsort((h["len"], h["q0"], h["t0"], -h["score"]))
    return h[order].copy()


def ydrop_half(A, B, sc: dict):
    """One half on already-oriented code arrays; returns (best, i_end, j_end,
    cells, ops) with ops in emission order (end cell back to the anchor), one
    code per step: 0 M, 1 I, 2 D."""
    A = np.ascontiguousarray(A, np.uint8)
    B = np.ascontiguousarray(B, np.uint8)
    res = Half()
    s = scoring(sc)
    cap = A.shape[0] + B.shape[0] + 1
    ops = np.empty(cap, np.uint8)
    n = lib().orc_ydrop_half(_p(A), A.shape[0], _p(B), B.shape[0], ctypes.byref(s), ctypes.byref(res), _p(ops), cap)
    return res.best, res.i_end, res.j_end, res.cells, ops[:n].copy()


def extend(tc, qc, ta, qa, sc: dict):
    """Both halves around anchor column (ta, qa): (alignment record, run-length ops)."""
    out = np.zeros(1, ALN_DTYPE)
    s = scoring(sc)
    cap = tc.shape[0] + qc.shape[0] + 2
    ops = np.empty(cap, np.uint32)
    n = lib().orc_extend(_p(tc), tc.shape[0], _p(qc), qc.shape[0], int(ta), int(qa), ctypes.byref(s),
                         _p(out), _p(ops), cap)
    return out[0], ops[:n].copy()


def commit_unit(tc, qc, hsps: np.ndarray, sc: dict, K: int = 0, query_id: int = 0, strand: int = 0):
    """Alg. 1 (K <= 0) or Alg. 3 with batch size K over one unit's ordered HSPs.
    Returns (alignments, ops, n_extensions, extension_cells)."""
    hsps = np.ascontiguousarray(hsps, HSP_DTYPE)
    s = scoring(sc)
    r = lib().orc_result_new()
    try:
        lib().orc_commit_unit(_p(tc), tc.shape[0], _p(qc), qc.shape[0], _p(hsps), hsps.shape[0],
                              ctypes.byref(s), int(K), int(query_id), int(strand), r)
        res = r.contents
        alns = np.zeros(res.n_alns, ALN_DTYPE)
        ops = np.zeros(res.n_ops, np.uint32)
        if res.n_alns:
            ctypes.memmove(_p(alns), res.alns, res.n_alns * ALN_DTYPE.itemsize)
        if res.n_ops:
            ctypes.memmove(_p(ops), res.ops, res.n_ops * 4)
        return alns, ops, res.n_extensions, res.ext_cells
    finally:
        lib().orc_result_free(r)


def pipeline(target, queries, sc: dict, pattern="1110100110010101111", transitions=1, step=1,
             strands=3, K=0, filter="xdrop"):
    """The whole path for ASCII target/queries: seeds -> X-drop (or the 2-D
    Y-drop filter, filter="ydrop") -> HSP set -> Alg. 1 (or Alg. 3 with batch
    size K) per (query, strand).  Returns a dict
    with per-unit hits and HSPs, and the committed alignments (ordered by
    query, strand, t_start, q_start, t_end, q_end, anchor_t, anchor_q) with
    their run-length ops."""
    span = len(pattern)
    tc, ts = encode(target)
    units = []
    all_alns, all_ops = [], []
    nops = 0
    n_ext = cells = 0
    for qid, qtxt in enumerate(queries):
        qc0, qs0 = encode(qtxt)
        for strand in (0, 1):
            if not (strands >> strand) & 1:
                continue
            qc, qs = (qc0, qs0) if strand == 0 else revcomp(qc0, qs0)
            t, q = seed_hits(tc, ts, qc, qs, pattern, transitions, step)
            raw = xdrop(tc, qc, t, q, span, sc) if filter == "xdrop" else ydrop_filter(tc, qc, t, q, span, sc)
            hs = hsp_set(raw, sc["hsp_thresh"])
            alns, ops, ne, nc = commit_unit(tc, qc, hs, sc, K, qid, strand)
            n_ext += ne
            cells += nc
            alns = alns.copy()
            alns["ops_off"] += nops
            nops += ops.shape[0]
            all_alns.append(alns)
            all_ops.append(ops)
            units.append(dict(query_id=qid, strand=strand, hits_t=t, hits_q=q, raw=raw, hsps=hs,
                              n_alns=alns.shape[0]))
    alns = np.concatenate(all_alns) if all_alns else np.zeros(0, ALN_DTYPE)
    ops = np.concatenate(all_ops) if all_ops else np.zeros(0, np.uint32)
    order = np.lexsort((alns["anchor_q"], alns["anchor_t"], alns["q_end"], alns["t_end"], alns["q_start"],
                        alns["t_start"], alns["strand"], alns["query_id"]))
    return dict(units=units, alns=alns[order], ops=ops, n_extensions=n_ext, ext_cells=cells)


def aln_ops(res: dict, x: int) -> np.ndarray:
    a = res["alns"][x]
    return res["ops"][a["ops_off"]:a["ops_off"] + a["ops_len"]]
