"""Thin ctypes binding of ``libplast_hip.so`` (C ABI in ``include/plast.h``).

Argument marshalling only: device memory comes from torch tensors, the stream is
torch's current stream, and every step of the search runs in the HIP library.
Importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libplast_hip.so")

NKEYS = 8800
PAD_CODE = 20
PAD_LEN = 20
NBR = 20
PLAIN, BATCHED = 0, 1
MODES = {"plain": PLAIN, "batched": BATCHED}

OK, E_ARG, E_ALPHABET, E_CAPACITY, E_WORKSPACE, E_HIP, E_LAYOUT = 0, -1, -2, -3, -4, -5, -6

EXPORTS = ("plast_index_bytes", "plast_build_index", "plast_ungapped_workspace_bytes", "plast_ungapped_extend",
           "plast_gapped_filter", "plast_timing_enable", "plast_timing_read", "plast_tuning_default",
           "plast_autotune", "plast_pipeline_workspace_bytes", "plast_pipeline_create", "plast_pipeline_launch",
           "plast_pipeline_result", "plast_pipeline_index", "plast_pipeline_destroy",
           "plast_search_workspace_bytes", "plast_search_enqueue", "plast_search_result",
           "plast_translate_ws_bytes", "plast_translate_count", "plast_translate_write",
           "plast_align_workspace_bytes", "plast_align", "plast_probe_peak", "plast_ungapped_extend_noalloc",
           "plast_strerror", "plast_last_error")

# plast_probe_peak kinds and the unit of each rate
PROBES = {"valu_i32": (0, "op/s"), "valu_pk_i16": (1, "op/s"), "valu_pk_f16": (2, "op/s"),
          "lds_lookup": (3, "lookup/s"), "hbm_copy": (4, "B/s"), "lds_b64": (5, "B/s"), "sclk": (6, "Hz")}

TUNE_CLASSES = 4
TUNE_WIDTHS = (1024, 2048, 4096, 8192, 16384)
GAPPED_THREADS = (128, 256, 512)


class PlastError(RuntimeError):
    def __init__(self, code, where, detail):
        super().__init__("%s failed: %s (%d)%s" % (where, _strerror(code), code, (": " + detail) if detail else ""))
        self.code = code


class IndexView(ctypes.Structure):
    _fields_ = [("codes", ctypes.c_void_p), ("seq_start", ctypes.c_void_p), ("n_seqs", ctypes.c_int32),
                ("n_padded", ctypes.c_int64), ("key_off", ctypes.c_void_p), ("occ", ctypes.c_void_p),
                ("occ_seq", ctypes.c_void_p), ("scan_codes", ctypes.c_void_p), ("n_words", ctypes.c_int64)]


class Timing(ctypes.Structure):
    _fields_ = [("index_ms", ctypes.c_float), ("plan_ms", ctypes.c_float), ("ungapped_ms", ctypes.c_float),
                ("gapped_ms", ctypes.c_float), ("ungapped_launches", ctypes.c_int64), ("align_ms", ctypes.c_float)]


class Tuning(ctypes.Structure):
    """Launch shapes (``plast_tuning_t``): size classes by n2, item width per
    class, work queues (1 or 8), gapped workgroup size."""
    _fields_ = [("class_min_n2", ctypes.c_int32 * TUNE_CLASSES), ("item_cols", ctypes.c_int32 * TUNE_CLASSES),
                ("xcd_queues", ctypes.c_int32), ("gapped_threads", ctypes.c_int32)]

    def as_dict(self):
        return {"class_min_n2": list(self.class_min_n2), "item_cols": list(self.item_cols),
                "xcd_queues": int(self.xcd_queues), "gapped_threads": int(self.gapped_threads)}

    @classmethod
    def from_dict(cls, d):
        t = tuning_default()
        for k in ("class_min_n2", "item_cols"):
            if k in d:
                getattr(t, k)[:] = [int(v) for v in d[k]]
        for k in ("xcd_queues", "gapped_threads"):
            if k in d:
                setattr(t, k, int(d[k]))
        return t


class TuneReport(ctypes.Structure):
    _fields_ = [("class_ext", ctypes.c_int64 * TUNE_CLASSES),
                ("class_ms", (ctypes.c_float * len(TUNE_WIDTHS)) * TUNE_CLASSES),
                ("queue_ms", ctypes.c_float * 2), ("gapped_ms", ctypes.c_float * 3)]

    def as_dict(self):
        return {"class_ext": list(self.class_ext), "class_ms": [list(r) for r in self.class_ms],
                "queue_ms": list(self.queue_ms), "gapped_ms": list(self.gapped_ms)}


class UngappedParams(ctypes.Structure):
    _fields_ = [("nbr", ctypes.c_int32), ("s1", ctypes.c_int32), ("matrix", ctypes.c_void_p),
                ("tuning", ctypes.c_void_p)]


class GappedParams(ctypes.Structure):
    _fields_ = [("window", ctypes.c_int32), ("band", ctypes.c_int32), ("gap_open", ctypes.c_int32),
                ("gap_extend", ctypes.c_int32), ("s2", ctypes.c_int32), ("matrix", ctypes.c_void_p),
                ("tuning", ctypes.c_void_p)]


class BankDesc(ctypes.Structure):
    _fields_ = [("codes", ctypes.c_void_p), ("seq_start", ctypes.c_void_p), ("n_seqs", ctypes.c_int32),
                ("n_padded", ctypes.c_int64)]


class MatchRec(ctypes.Structure):
    _fields_ = [("seq1", ctypes.c_int32), ("pos1", ctypes.c_int32), ("seq2", ctypes.c_int32),
                ("pos2", ctypes.c_int32), ("score", ctypes.c_int32), ("gscore", ctypes.c_int32)]


class AlignParams(ctypes.Structure):
    _fields_ = [("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32), ("max_len1", ctypes.c_int32),
                ("max_len2", ctypes.c_int32), ("n_waves", ctypes.c_int32), ("max_pieces", ctypes.c_int32),
                ("matrix", ctypes.c_void_p)]


# columns of a plast_alignment_t record
ALIGN_FIELDS = ("seq1", "seq2", "seed1", "seed2", "start1", "end1", "start2", "end2", "score", "length",
                "identities", "mismatches", "gap_opens", "hit")


class PipelineResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_items", ctypes.c_int32), ("n_hits", ctypes.c_int64),
                ("n_ext", ctypes.c_int64), ("n_words_a", ctypes.c_int64), ("n_words_b", ctypes.c_int64)]


_lib = None


def load():
    """Load the in-tree library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libplast_hip.so is not built (run __graft_entry__.build() or "
                              "python paper_0804_3643_amd/build.py); there is no CPU fallback")
        lib = ctypes.CDLL(LIB_PATH)
        P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        lib.plast_index_bytes.argtypes = [i64, i32, ctypes.POINTER(sz), ctypes.POINTER(sz)]
        lib.plast_build_index.argtypes = [P, P, i32, i64, P, sz, P, sz, ctypes.POINTER(IndexView), P]
        IV = ctypes.POINTER(IndexView)
        lib.plast_ungapped_workspace_bytes.argtypes = [IV, IV, i32, ctypes.POINTER(Tuning), ctypes.POINTER(sz),
                                                       ctypes.POINTER(i64), ctypes.POINTER(i64), P]
        lib.plast_ungapped_extend.argtypes = [ctypes.POINTER(IndexView), ctypes.POINTER(IndexView),
                                              ctypes.POINTER(UngappedParams), i32, P, sz, P, i64,
                                              ctypes.POINTER(i64), ctypes.POINTER(i64), P]
        lib.plast_gapped_filter.argtypes = [ctypes.POINTER(IndexView), ctypes.POINTER(IndexView), P, i64,
                                            ctypes.POINTER(GappedParams), P, P, P]
        lib.plast_timing_enable.argtypes = [ctypes.c_int]
        lib.plast_timing_read.argtypes = [ctypes.POINTER(Timing)]
        lib.plast_tuning_default.argtypes = [ctypes.POINTER(Tuning)]
        lib.plast_autotune.argtypes = [IV, IV, ctypes.POINTER(UngappedParams), ctypes.POINTER(GappedParams), i32, P,
                                       sz, P, i64, P, P, ctypes.POINTER(Tuning), ctypes.POINTER(TuneReport), P]
        BD = ctypes.POINTER(BankDesc)
        lib.plast_pipeline_workspace_bytes.argtypes = [BD, BD, i64, ctypes.POINTER(sz)]
        lib.plast_pipeline_create.argtypes = [BD, BD, ctypes.POINTER(UngappedParams), ctypes.POINTER(GappedParams),
                                              i64, P, sz, P, i64, P, P, ctypes.POINTER(P)]
        lib.plast_pipeline_launch.argtypes = [P, P]
        lib.plast_pipeline_result.argtypes = [P, ctypes.POINTER(PipelineResult), P]
        lib.plast_pipeline_index.argtypes = [P, i32, IV]
        lib.plast_pipeline_destroy.argtypes = [P]
        lib.plast_search_workspace_bytes.argtypes = [BD, i64, ctypes.POINTER(sz)]
        lib.plast_search_enqueue.argtypes = [BD, IV, ctypes.POINTER(UngappedParams), ctypes.POINTER(GappedParams),
                                             i64, P, sz, P, i64, P, P, P, P, i32, P, P]
        lib.plast_search_result.argtypes = [P, ctypes.POINTER(PipelineResult), ctypes.POINTER(i64), P]
        lib.plast_translate_ws_bytes.argtypes = [i32, ctypes.POINTER(sz)]
        lib.plast_translate_count.argtypes = [P, P, i32, i64, P, sz, ctypes.POINTER(i64), ctypes.POINTER(i64), P]
        lib.plast_translate_write.argtypes = [P, P, i32, i64, P, sz, P, i64, P, P, i64, P]
        AP = ctypes.POINTER(AlignParams)
        lib.plast_align_workspace_bytes.argtypes = [i64, AP, ctypes.POINTER(sz)]
        lib.plast_align.argtypes = [IV, IV, P, P, P, i64, AP, P, sz, P, P, ctypes.POINTER(i64), P]
        lib.plast_probe_peak.argtypes = [i32, P, sz, i32, ctypes.POINTER(ctypes.c_double), P]
        lib.plast_ungapped_extend_noalloc.argtypes = [IV, IV, ctypes.POINTER(UngappedParams), P, i64,
                                                      ctypes.POINTER(i64), ctypes.POINTER(i64), P]
        for f in EXPORTS[:-2]:
            getattr(lib, f).restype = ctypes.c_int
        lib.plast_strerror.argtypes = [ctypes.c_int]
        lib.plast_strerror.restype = ctypes.c_char_p
        lib.plast_last_error.argtypes = []
        lib.plast_last_error.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def _strerror(code):
    return load().plast_strerror(code).decode()


def _check(rc, where):
    if rc != OK:
        raise PlastError(rc, where, load().plast_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _alloc(nbytes, device):
    # 256-byte alignment is required by the library; torch's caching allocator
    # returns blocks aligned to at least 512 bytes.
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


class BankIndex:
    """A bank resident on the device plus its built index (owns the tensors)."""

    def __init__(self, codes, seq_start, index_buf, view):
        self.codes = codes
        self.seq_start = seq_start
        self.index_buf = index_buf
        self.view = view

    @property
    def n_words(self):
        return int(self.view.n_words)

    @property
    def n_seqs(self):
        return int(self.view.n_seqs)

    def key_off(self):
        return _view_tensor(self.index_buf, self.view.key_off, NKEYS + 1, torch.int64)

    def occ(self):
        return _view_tensor(self.index_buf, self.view.occ, self.n_words, torch.int32)

    def occ_seq(self):
        return _view_tensor(self.index_buf, self.view.occ_seq, self.n_words, torch.int32)


def _view_tensor(buf, ptr, n, dtype):
    off = int(ptr) - buf.data_ptr()
    esz = torch.empty(0, dtype=dtype).element_size()
    return buf[off:off + n * esz].view(dtype)


def bank_to_device(bank, device="cuda"):
    """Copy a bank in the padded layout (numpy ``codes``/``seq_start``) to the device."""
    codes = torch.from_numpy(np.ascontiguousarray(bank.codes, dtype=np.uint8)).to(device)
    seq_start = torch.from_numpy(np.ascontiguousarray(bank.seq_start, dtype=np.int64)).to(device)
    return codes, seq_start


def index_bytes(n_padded, n_seqs):
    ib, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    _check(load().plast_index_bytes(int(n_padded), int(n_seqs), ctypes.byref(ib), ctypes.byref(wb)),
           "plast_index_bytes")
    return ib.value, wb.value


def build_index(codes, seq_start, stream=None, workspace=None, out_buf=None):
    """Stage 0 on the device: ``codes`` uint8 and ``seq_start`` int64 CUDA tensors.
    ``workspace`` / ``out_buf`` (uint8 device tensors of at least
    :func:`index_bytes` sizes) are used instead of allocating when given."""
    assert codes.is_cuda and codes.dtype == torch.uint8 and seq_start.dtype == torch.int64
    n_seqs = seq_start.numel() - 1
    n_padded = codes.numel()
    ib, wb = index_bytes(n_padded, n_seqs)
    buf = out_buf if out_buf is not None and out_buf.numel() >= ib else _alloc(ib, codes.device)
    ws = workspace if workspace is not None and workspace.numel() >= wb else _alloc(wb, codes.device)
    view = IndexView()
    _check(load().plast_build_index(_ptr(codes), _ptr(seq_start), n_seqs, n_padded, _ptr(buf), buf.numel(),
                                    _ptr(ws), ws.numel(), ctypes.byref(view), _stream(stream)),
           "plast_build_index")
    return BankIndex(codes, seq_start, buf, view)


def _matrix_ptr(matrix):
    if matrix is None:
        return None, ctypes.c_void_p(0)
    m = np.ascontiguousarray(np.asarray(matrix, dtype=np.int8).reshape(20, 20))
    return m, ctypes.c_void_p(m.ctypes.data)


def tuning_default():
    t = Tuning()
    _check(load().plast_tuning_default(ctypes.byref(t)), "plast_tuning_default")
    return t


def _tuning(t):
    """Accepts None, a Tuning or a dict; returns (object kept alive, pointer)."""
    if t is None:
        return None, ctypes.c_void_p(0)
    if isinstance(t, dict):
        t = Tuning.from_dict(t)
    return t, ctypes.c_void_p(ctypes.addressof(t))


def ungapped_workspace_bytes(ia, ib, mode="batched", stream=None, tuning=None):
    """Returns (workspace bytes, pairs to score, BATCHED work-list length)."""
    sz, n_ext, n_items = ctypes.c_size_t(0), ctypes.c_int64(0), ctypes.c_int64(0)
    t, _ = _tuning(tuning)
    _check(load().plast_ungapped_workspace_bytes(ctypes.byref(ia.view), ctypes.byref(ib.view), MODES[mode],
                                                 ctypes.byref(t) if t is not None else None, ctypes.byref(sz),
                                                 ctypes.byref(n_ext), ctypes.byref(n_items), _stream(stream)),
           "plast_ungapped_workspace_bytes")
    return sz.value, n_ext.value, n_items.value


def default_capacity(n_ext):
    return int(n_ext * 0.004) + 4096


class Extender:
    """Reusable ungapped-extension call: holds the workspace and the hit buffer
    so that repeated calls (benchmark steps) allocate nothing."""

    def __init__(self, ia, ib, s1, mode="batched", capacity=None, matrix=None, stream=None, tuning=None):
        self.ia, self.ib, self.mode = ia, ib, MODES[mode]
        self._tun, tp = _tuning(tuning)
        wsb, self.n_ext_expected, self.n_items = ungapped_workspace_bytes(ia, ib, mode, stream, self._tun)
        self.ws = _alloc(wsb, ia.codes.device)
        if capacity is None:
            capacity = default_capacity(self.n_ext_expected)
        self.hits = torch.empty((int(capacity), 5), dtype=torch.int32, device=ia.codes.device)
        self._mat, mp = _matrix_ptr(matrix)
        self.params = UngappedParams(NBR, int(s1), mp, tp)
        self.stream = stream

    def run(self, ia=None, ib=None):
        """One extension call; ``ia``/``ib`` replace the index views (same sizes)."""
        if ia is not None:
            self.ia = ia
        if ib is not None:
            self.ib = ib
        n_hits, n_ext = ctypes.c_int64(0), ctypes.c_int64(0)
        while True:
            rc = load().plast_ungapped_extend(ctypes.byref(self.ia.view), ctypes.byref(self.ib.view),
                                              ctypes.byref(self.params), self.mode, _ptr(self.ws), self.ws.numel(),
                                              _ptr(self.hits), self.hits.shape[0], ctypes.byref(n_hits),
                                              ctypes.byref(n_ext), _stream(self.stream))
            if rc == E_CAPACITY:
                self.hits = torch.empty((int(n_hits.value * 1.1) + 1024, 5), dtype=torch.int32,
                                        device=self.ia.codes.device)
                continue
            _check(rc, "plast_ungapped_extend")
            return self.hits[:n_hits.value], n_ext.value


def ungapped_extend(ia, ib, s1, mode="batched", capacity=None, matrix=None, stream=None, tuning=None):
    """Stage 2: returns (hits int32[n, 5] device tensor in unspecified order, n_ext)."""
    return Extender(ia, ib, s1, mode, capacity, matrix, stream, tuning).run()


NOALLOC_SCRATCH_BYTES = 8 << 20


def ungapped_extend_noalloc(ia, ib, s1, hits, matrix=None, stream=None, tuning=None):
    """Stage 2, BATCHED, through ``plast_ungapped_extend_noalloc`` (the library's
    static scratch instead of a workspace): ``hits`` is the caller's int32[cap, 5]
    device tensor; returns (hits[:n], n_ext).  Raises PlastError (E_CAPACITY
    with the required count in the message, E_WORKSPACE when the work list does
    not fit the static scratch)."""
    t, tp = _tuning(tuning)
    m, mp = _matrix_ptr(matrix)
    params = UngappedParams(NBR, int(s1), mp, tp)
    n_hits, n_ext = ctypes.c_int64(0), ctypes.c_int64(0)
    rc = load().plast_ungapped_extend_noalloc(ctypes.byref(ia.view), ctypes.byref(ib.view), ctypes.byref(params),
                                              _ptr(hits), hits.shape[0], ctypes.byref(n_hits), ctypes.byref(n_ext),
                                              _stream(stream))
    _check(rc, "plast_ungapped_extend_noalloc")
    return hits[:n_hits.value], n_ext.value


def gapped_filter(ia, ib, hits, s2, window=64, band=16, gap_open=11, gap_extend=1, matrix=None, stream=None,
                  out=None, tuning=None):
    """Stage 3.1: returns (gscore int32[n], pass uint8[n]) device tensors."""
    n = hits.shape[0]
    dev = ia.codes.device
    if out is None:
        gs = torch.empty(n, dtype=torch.int32, device=dev)
        ps = torch.empty(n, dtype=torch.uint8, device=dev)
    else:
        gs, ps = out[0][:n], out[1][:n]
    m, mp = _matrix_ptr(matrix)
    t, tp = _tuning(tuning)
    g = GappedParams(int(window), int(band), int(gap_open), int(gap_extend), int(s2), mp, tp)
    hp = hits if hits.is_contiguous() else hits.contiguous()
    _check(load().plast_gapped_filter(ctypes.byref(ia.view), ctypes.byref(ib.view), _ptr(hp), n, ctypes.byref(g),
                                      _ptr(gs), _ptr(ps), _stream(stream)), "plast_gapped_filter")
    del m, t
    return gs, ps


def autotune(ia, ib, s1, s2, reps=3, capacity=None, matrix=None, window=64, band=16, gap_open=11, gap_extend=1,
             start=None, stream=None):
    """Measures the launch shapes for these banks (``plast_autotune``).
    Returns (Tuning, report dict)."""
    dev = ia.codes.device
    smallest = tuning_default()
    smallest.item_cols[:] = [TUNE_WIDTHS[0]] * TUNE_CLASSES
    wsb, n_ext, _ = ungapped_workspace_bytes(ia, ib, "batched", stream, smallest)
    if capacity is None:  # one extension call to learn the hit count
        h, _ = Extender(ia, ib, s1, "batched", None, matrix, stream, start).run()
        capacity = h.shape[0] + 1024
        del h
    ws = _alloc(wsb, dev)
    cap = int(capacity)
    hits = torch.empty((cap, 5), dtype=torch.int32, device=dev)
    gs = torch.empty(cap, dtype=torch.int32, device=dev)
    ps = torch.empty(cap, dtype=torch.uint8, device=dev)
    m, mp = _matrix_ptr(matrix)
    st, sp = _tuning(start)
    u = UngappedParams(NBR, int(s1), mp, sp)
    g = GappedParams(int(window), int(band), int(gap_open), int(gap_extend), int(s2), mp, sp)
    out, rep = Tuning(), TuneReport()
    _check(load().plast_autotune(ctypes.byref(ia.view), ctypes.byref(ib.view), ctypes.byref(u), ctypes.byref(g),
                                 int(reps), _ptr(ws), ws.numel(), _ptr(hits), cap, _ptr(gs), _ptr(ps),
                                 ctypes.byref(out), ctypes.byref(rep), _stream(stream)), "plast_autotune")
    del m, st
    return out, rep.as_dict()


class Pipeline:
    """Graph-replayed whole search over two device banks (``plast_pipeline_*``).
    Owns its workspace and output tensors; ``launch()`` enqueues one replay,
    ``result()`` waits and returns the counts and status."""

    def __init__(self, codes_a, starts_a, codes_b, starts_b, s1, s2, max_items, capacity, matrix=None,
                 tuning=None, window=64, band=16, gap_open=11, gap_extend=1):
        dev = codes_a.device
        self._keep = (codes_a, starts_a, codes_b, starts_b)
        self.a = BankDesc(codes_a.data_ptr(), starts_a.data_ptr(), starts_a.numel() - 1, codes_a.numel())
        self.b = BankDesc(codes_b.data_ptr(), starts_b.data_ptr(), starts_b.numel() - 1, codes_b.numel())
        sz = ctypes.c_size_t(0)
        _check(load().plast_pipeline_workspace_bytes(ctypes.byref(self.a), ctypes.byref(self.b), int(max_items),
                                                     ctypes.byref(sz)), "plast_pipeline_workspace_bytes")
        self.ws = _alloc(sz.value, dev)
        self.capacity = int(capacity)
        self.hits = torch.empty((max(self.capacity, 1), 5), dtype=torch.int32, device=dev)
        self.gscore = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=dev)
        self.passed = torch.empty(max(self.capacity, 1), dtype=torch.uint8, device=dev)
        m, mp = _matrix_ptr(matrix)
        t, tp = _tuning(tuning)
        u = UngappedParams(NBR, int(s1), mp, tp)
        g = GappedParams(int(window), int(band), int(gap_open), int(gap_extend), int(s2), mp, tp)
        h = ctypes.c_void_p(0)
        torch.cuda.synchronize(dev)  # inputs written by torch are complete before the capture
        _check(load().plast_pipeline_create(ctypes.byref(self.a), ctypes.byref(self.b), ctypes.byref(u),
                                            ctypes.byref(g), int(max_items), _ptr(self.ws), self.ws.numel(),
                                            _ptr(self.hits), self.capacity, _ptr(self.gscore), _ptr(self.passed),
                                            ctypes.byref(h)), "plast_pipeline_create")
        del m, t
        self.handle = h

    def launch(self, stream=None):
        _check(load().plast_pipeline_launch(self.handle, _stream(stream)), "plast_pipeline_launch")

    def result(self, stream=None):
        r = PipelineResult()
        _check(load().plast_pipeline_result(self.handle, ctypes.byref(r), _stream(stream)), "plast_pipeline_result")
        return {"status": int(r.status), "n_items": int(r.n_items), "n_hits": int(r.n_hits), "n_ext": int(r.n_ext),
                "n_words_a": int(r.n_words_a), "n_words_b": int(r.n_words_b)}

    def outputs(self, n_hits):
        n = min(int(n_hits), self.capacity)
        return self.hits[:n], self.gscore[:n], self.passed[:n]

    def index_view(self, which):
        v = IndexView()
        _check(load().plast_pipeline_index(self.handle, int(which), ctypes.byref(v)), "plast_pipeline_index")
        return v

    def close(self):
        if getattr(self, "handle", None):
            h, self.handle = self.handle, None
            _check(load().plast_pipeline_destroy(h), "plast_pipeline_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def canonical_hits(hits):
    """Host copy of a hit tensor sorted lexicographically (seq1, pos1, seq2, pos2, score)."""
    h = hits.detach().to("cpu").numpy().astype(np.int64).reshape(-1, 5)
    if len(h) == 0:
        return h
    return h[np.lexsort(h.T[::-1])]


_timing = False


def timing_on():
    """Whether timing_enable(True) is in force (as last set through this module)."""
    return _timing


def timing_enable(on=True):
    global _timing
    _check(load().plast_timing_enable(1 if on else 0), "plast_timing_enable")
    _timing = bool(on)


def probe_peak(kind, buf, reps=3, stream=None):
    """Measured peak rate of one kind of work (a key of ``PROBES``) with the
    caller's device buffer ``buf`` (a uint8 tensor, 256-byte aligned): the
    best of ``reps`` HIP-event timed launches after one warm-up."""
    code, _unit = PROBES[kind]
    rate = ctypes.c_double(0.0)
    _check(load().plast_probe_peak(code, _ptr(buf), buf.numel() * buf.element_size(), reps, ctypes.byref(rate),
                                   _stream(stream)), "plast_probe_peak")
    return rate.value


def timing_read():
    t = Timing()
    _check(load().plast_timing_read(ctypes.byref(t)), "plast_timing_read")
    return {"index_ms": t.index_ms, "plan_ms": t.plan_ms, "ungapped_ms": t.ungapped_ms, "gapped_ms": t.gapped_ms,
            "ungapped_launches": int(t.ungapped_launches), "align_ms": t.align_ms}


class Searcher:
    """One query-versus-resident search slot (``plast_search_*``): device
    buffers for a query bank of up to ``max_padded`` codes / ``max_seqs``
    sequences, a work list of ``max_items`` items and ``capacity`` hits, all
    allocated once.  ``enqueue`` only enqueues on ``stream``; ``result`` waits
    for it.  Matches (hits passing the gapped filter, with both scores) are
    written to ``self.matches`` as int32[n, 6]."""

    def __init__(self, resident, max_padded, max_seqs, max_items, capacity, s1, s2, matrix=None, tuning=None,
                 window=64, band=16, gap_open=11, gap_extend=1):
        dev = resident.codes.device
        self.resident = resident
        self.max_padded, self.max_seqs = int(max_padded), int(max_seqs)
        self.max_items, self.capacity = int(max_items), int(capacity)
        self.codes = torch.empty(self.max_padded, dtype=torch.uint8, device=dev)
        self.starts = torch.empty(self.max_seqs + 1, dtype=torch.int64, device=dev)
        big = BankDesc(0, 0, self.max_seqs, self.max_padded)
        sz = ctypes.c_size_t(0)
        _check(load().plast_search_workspace_bytes(ctypes.byref(big), self.max_items, ctypes.byref(sz)),
               "plast_search_workspace_bytes")
        self.ws = _alloc(sz.value, dev)
        self.hits = torch.empty((max(self.capacity, 1), 5), dtype=torch.int32, device=dev)
        self.gscore = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=dev)
        self.passed = torch.empty(max(self.capacity, 1), dtype=torch.uint8, device=dev)
        self.matches = torch.empty((max(self.capacity, 1), 6), dtype=torch.int32, device=dev)
        self.seg_first = torch.empty(self.max_seqs + 2, dtype=torch.int32, device=dev)
        self.seg_off = torch.empty(2 * (self.max_seqs + 2), dtype=torch.int64, device=dev)
        self._mat, mp = _matrix_ptr(matrix)
        self._tun, tp = _tuning(tuning)
        self.u = UngappedParams(NBR, int(s1), mp, tp)
        self.g = GappedParams(int(window), int(band), int(gap_open), int(gap_extend), int(s2), mp, tp)

    def enqueue(self, n_padded, n_seqs, n_seg=0, stream=None):
        """Search the query bank already in ``self.codes[:n_padded]`` /
        ``self.starts[:n_seqs + 1]`` (padded layout) against the resident index.
        With ``n_seg`` > 0, ``self.seg_first[:n_seg + 1]`` cuts the bank into
        segments and the matches come out grouped by segment (offsets in
        ``self.seg_off[:n_seg + 1]``)."""
        assert 0 < n_padded <= self.max_padded and 0 <= n_seqs <= self.max_seqs and 0 <= n_seg <= n_seqs + 1
        a = BankDesc(self.codes.data_ptr(), self.starts.data_ptr(), int(n_seqs), int(n_padded))
        seg = _ptr(self.seg_first) if n_seg > 0 else ctypes.c_void_p(0)
        _check(load().plast_search_enqueue(ctypes.byref(a), ctypes.byref(self.resident.view), ctypes.byref(self.u),
                                           ctypes.byref(self.g), self.max_items, _ptr(self.ws), self.ws.numel(),
                                           _ptr(self.hits), self.capacity, _ptr(self.gscore), _ptr(self.passed),
                                           _ptr(self.matches), seg, int(n_seg), _ptr(self.seg_off),
                                           _stream(stream)), "plast_search_enqueue")

    def result(self, stream=None):
        r, nm = PipelineResult(), ctypes.c_int64(0)
        _check(load().plast_search_result(_ptr(self.ws), ctypes.byref(r), ctypes.byref(nm), _stream(stream)),
               "plast_search_result")
        return {"status": int(r.status), "n_items": int(r.n_items), "n_hits": int(r.n_hits), "n_ext": int(r.n_ext),
                "n_words_a": int(r.n_words_a), "n_matches": int(nm.value)}


def dna_to_device(dna, device="cuda"):
    """Copy a nucleotide bank (numpy ``codes`` in 0..3, ``start``) to the device."""
    codes = torch.from_numpy(np.ascontiguousarray(dna.codes, dtype=np.uint8)).to(device)
    start = torch.from_numpy(np.ascontiguousarray(dna.start, dtype=np.int64)).to(device)
    return codes, start


class Translator:
    """Six-frame translation of a device nucleotide bank (``plast_translate_*``):
    ``run`` returns (codes uint8, seq_start int64, frag int32[n, 3]) device
    tensors of the fragment bank; the workspace is kept for repeated calls."""

    def __init__(self, dna_codes, dna_start):
        self.dna, self.start = dna_codes, dna_start
        self.n_dna = dna_start.numel() - 1
        sz = ctypes.c_size_t(0)
        _check(load().plast_translate_ws_bytes(self.n_dna, ctypes.byref(sz)), "plast_translate_ws_bytes")
        self.ws = _alloc(sz.value, dna_codes.device)
        self.out = None

    def count(self, stream=None):
        nf, npad = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(load().plast_translate_count(_ptr(self.dna), _ptr(self.start), self.n_dna, self.dna.numel(),
                                            _ptr(self.ws), self.ws.numel(), ctypes.byref(nf), ctypes.byref(npad),
                                            _stream(stream)), "plast_translate_count")
        return nf.value, npad.value

    def run(self, stream=None):
        n_frags, n_padded = self.count(stream)
        dev = self.dna.device
        if self.out is None or self.out[0].numel() != n_padded or self.out[1].numel() != n_frags + 1:
            self.out = (torch.empty(n_padded, dtype=torch.uint8, device=dev),
                        torch.empty(n_frags + 1, dtype=torch.int64, device=dev),
                        torch.empty((max(n_frags, 1), 3), dtype=torch.int32, device=dev))
        codes, starts, frag = self.out
        _check(load().plast_translate_write(_ptr(self.dna), _ptr(self.start), self.n_dna, self.dna.numel(),
                                            _ptr(self.ws), self.ws.numel(), _ptr(codes), n_padded, _ptr(starts),
                                            _ptr(frag), n_frags, _stream(stream)), "plast_translate_write")
        return codes, starts, frag[:n_frags]


def translate(dna_codes, dna_start, stream=None):
    return Translator(dna_codes, dna_start).run(stream)


def max_seq_len(ix):
    """Longest sequence of an indexed bank (host read of its sequence offsets)."""
    st = ix.seq_start.cpu().numpy()
    return int((np.diff(st) - PAD_LEN).max(initial=1))


def align_workspace_bytes(n_hits, params):
    sz = ctypes.c_size_t(0)
    _check(load().plast_align_workspace_bytes(int(n_hits), ctypes.byref(params), ctypes.byref(sz)),
           "plast_align_workspace_bytes")
    return int(sz.value)


def align_params(ia, ib, gap_open=11, gap_extend=1, max_len1=None, max_len2=None, n_waves=0, max_pieces=4096,
                 matrix=None):
    """plast_align_params_t (and the matrix buffer it points to, to keep alive)."""
    m, mp = _matrix_ptr(matrix)
    p = AlignParams(int(gap_open), int(gap_extend), int(max_len1 if max_len1 else max_seq_len(ia)),
                    int(max_len2 if max_len2 else max_seq_len(ib)), int(n_waves), int(max_pieces), mp)
    return p, m


class Aligner:
    """Stage 3.2 with buffers allocated once for up to ``capacity`` input hits
    (records, cover array, workspace)."""

    def __init__(self, ia, ib, capacity, gap_open=11, gap_extend=1, max_len1=None, max_len2=None, n_waves=0,
                 max_pieces=4096, matrix=None):
        self.ia, self.ib = ia, ib
        self.capacity = int(capacity)
        dev = ia.codes.device
        self.params, self._m = align_params(ia, ib, gap_open, gap_extend, max_len1, max_len2, n_waves, max_pieces,
                                            matrix)
        self.out = torch.empty((max(self.capacity, 1), len(ALIGN_FIELDS)), dtype=torch.int32, device=dev)
        self.cover = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=dev)
        self.ws = _alloc(align_workspace_bytes(self.capacity, self.params), dev)

    def run(self, hits, gscore, passed, stream=None):
        n = hits.shape[0]
        if n > self.capacity:
            raise ValueError("%d hits exceed the aligner capacity %d" % (n, self.capacity))
        n_out = ctypes.c_int64(0)
        hp = hits if hits.is_contiguous() else hits.contiguous()
        _check(load().plast_align(ctypes.byref(self.ia.view), ctypes.byref(self.ib.view), _ptr(hp), _ptr(gscore),
                                  _ptr(passed), n, ctypes.byref(self.params), _ptr(self.ws), self.ws.numel(),
                                  _ptr(self.out), _ptr(self.cover), ctypes.byref(n_out), _stream(stream)),
               "plast_align")
        return self.out[:n_out.value], self.cover[:n]


def align(ia, ib, hits, gscore, passed, gap_open=11, gap_extend=1, max_len1=None, max_len2=None, n_waves=0,
          max_pieces=4096, matrix=None, stream=None):
    """Stage 3.2 (``plast_align``): full gapped alignments of the hits that
    passed the gapped filter.  Returns (records int32[n_out, 14] with columns
    ALIGN_FIELDS, in no particular order; cover int32[n_hits]) device tensors."""
    a = Aligner(ia, ib, hits.shape[0], gap_open, gap_extend, max_len1, max_len2, n_waves, max_pieces, matrix)
    return a.run(hits, gscore, passed, stream)


def canonical_alignments(rec):
    """Alignment records sorted lexicographically by their columns (int64 numpy)."""
    r = rec.cpu().numpy().astype(np.int64) if isinstance(rec, torch.Tensor) else np.asarray(rec, np.int64)
    r = r.reshape(-1, len(ALIGN_FIELDS))
    return r[np.lexsort(r.T[::-1])] if len(r) else r
