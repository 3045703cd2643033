"""ctypes front end of the plain C oracle (plast_oracle.c) — TEST INFRASTRUCTURE.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this.  ``build()`` compiles the C file with gcc; ``load()`` compiles it when the
shared object is missing or older than its source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import plast_oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "plast_oracle.c")
LIB = os.path.join(HERE, "liborc.so")
PAD = 20  # pad-run length of the bank storage format

_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-pthread", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


def declare(lib):
    """Set the argument and result types of the library's entry points on a
    ctypes handle (of liborc.so, or of another build of the same source)."""
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.orc_build_index.restype = i64
    lib.orc_build_index.argtypes = [P, P, i32, i32, P, P, P]
    lib.orc_ungapped.restype = i64
    lib.orc_ungapped.argtypes = [P, P, i32, P, P, P, P, P, i32, P, P, P, i32, P, i32, i32, i32, P, i32,
                                 i32, P, i64, P]
    lib.orc_gapped.restype = None
    lib.orc_gapped.argtypes = [P, P, P, P, i32, P, i64, P, i32, i32, i32, i32, i32, P]
    lib.orc_full_align.restype = i64
    lib.orc_full_align.argtypes = [P, P, P, P, i32, P, P, P, i64, P, i32, i32, i32, P, P]
    return lib


def load():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = declare(ctypes.CDLL(LIB))
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _bank_arrays(bank):
    return (np.ascontiguousarray(bank.codes, dtype=np.uint8),
            np.ascontiguousarray(bank.seq_start, dtype=np.int64))


def build_index(bank):
    lib = load()
    codes, start = _bank_arrays(bank)
    n = len(start) - 1
    cap = max(1, int(len(codes)))
    key_off = np.zeros(O.NKEYS + 1, dtype=np.int64)
    occ_seq = np.zeros(cap, dtype=np.int32)
    occ_pos = np.zeros(cap, dtype=np.int32)
    nw = lib.orc_build_index(_ptr(codes), _ptr(start), n, PAD, _ptr(key_off), _ptr(occ_seq), _ptr(occ_pos))
    return key_off, occ_seq[:nw].copy(), occ_pos[:nw].copy()


def _matrix(matrix):
    m = np.ascontiguousarray(np.asarray(matrix, dtype=np.int8).reshape(20, 20))
    return m


def ungapped_hits(bank1, bank2, s1, keys=None, idx1=None, idx2=None, nthreads=None,
                  matrix=O.BLOSUM62, nbr=O.NBR, right=O.RIGHT, canonicalize=True, capacity=None):
    """Hit rows int64[n, 5] (canonical order unless ``canonicalize=False``) and
    the number of pairs scored.  ``capacity`` is the first guess of the hit
    count (the call runs again with the exact count when the guess is short)."""
    lib = load()
    c1, st1 = _bank_arrays(bank1)
    c2, st2 = _bank_arrays(bank2)
    idx1 = idx1 if idx1 is not None else build_index(bank1)
    idx2 = idx2 if idx2 is not None else build_index(bank2)
    mat = _matrix(matrix)
    nthreads = nthreads or os.cpu_count() or 1
    karr = None if keys is None else np.ascontiguousarray(np.asarray(keys, dtype=np.int32))
    kp = None if karr is None else _ptr(karr)
    nk = 0 if karr is None else len(karr)
    cap = max(1, int(capacity)) if capacity else 1 << 16
    while True:
        out = np.zeros((cap, 5), dtype=np.int32)
        n_ext = ctypes.c_int64(0)
        n = lib.orc_ungapped(_ptr(c1), _ptr(st1), len(st1) - 1, _ptr(idx1[0]), _ptr(idx1[1]), _ptr(idx1[2]),
                             _ptr(c2), _ptr(st2), len(st2) - 1, _ptr(idx2[0]), _ptr(idx2[1]), _ptr(idx2[2]),
                             PAD, _ptr(mat), int(s1), int(nbr), int(right), kp, nk, int(nthreads), _ptr(out),
                             cap, ctypes.byref(n_ext))
        if n <= cap:
            hits = out[:n].astype(np.int64)
            return (O.canonical(hits) if canonicalize else hits), int(n_ext.value)
        cap = int(n)


def gapped_scores(bank1, bank2, hits, window=O.GAP_WINDOW, band=O.GAP_BAND, gap_open=O.GAP_OPEN,
                  gap_extend=O.GAP_EXTEND, matrix=O.BLOSUM62, nthreads=None):
    lib = load()
    c1, st1 = _bank_arrays(bank1)
    c2, st2 = _bank_arrays(bank2)
    h = np.ascontiguousarray(np.asarray(hits, dtype=np.int32).reshape(-1, 5))
    g = np.zeros(len(h), dtype=np.int32)
    mat = _matrix(matrix)
    lib.orc_gapped(_ptr(c1), _ptr(st1), _ptr(c2), _ptr(st2), PAD, _ptr(h), len(h), _ptr(mat), int(window),
                   int(band), int(gap_open), int(gap_extend), int(nthreads or os.cpu_count() or 1), _ptr(g))
    return g.astype(np.int64)


def full_alignments(bank1, bank2, hits, gscore, passed, gap_open=O.GAP_OPEN, gap_extend=O.GAP_EXTEND,
                    matrix=O.BLOSUM62, nthreads=None):
    """Stage 3.2, same contract as ``plast_oracle.full_alignments``: records
    (int64, columns ALIGN_FIELDS, canonical order) and cover (int64[n])."""
    lib = load()
    c1, st1 = _bank_arrays(bank1)
    c2, st2 = _bank_arrays(bank2)
    h = np.ascontiguousarray(np.asarray(hits, dtype=np.int32).reshape(-1, 5))
    g = np.ascontiguousarray(np.asarray(gscore, dtype=np.int32).reshape(-1))
    ps = np.ascontiguousarray(np.asarray(passed).reshape(-1).astype(np.uint8))
    n = len(h)
    out = np.zeros((max(1, n), len(O.ALIGN_FIELDS)), dtype=np.int32)
    cover = np.zeros(max(1, n), dtype=np.int32)
    mat = _matrix(matrix)
    m = lib.orc_full_align(_ptr(c1), _ptr(st1), _ptr(c2), _ptr(st2), PAD, _ptr(h), _ptr(g), _ptr(ps), n,
                           _ptr(mat), int(gap_open), int(gap_extend), int(nthreads or os.cpu_count() or 1),
                           _ptr(out), _ptr(cover))
    rec = out[:m].astype(np.int64)
    if m:
        rec = rec[np.lexsort(rec.T[::-1])]
    return rec, cover[:n].astype(np.int64)
