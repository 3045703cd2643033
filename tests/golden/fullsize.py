"""Full-size parity goldens: order-free digests of the oracle's output on the
large seeded workloads -- TEST INFRASTRUCTURE.

The hit lists of the full-size workloads (up to 1.6e8 records) are too large to
store, and too slow to recompute with the CPU oracle inside a GPU test.  This
module stores, per workload, what the oracle computes there, in a form that an
unordered GPU hit list can be compared with exactly:

* the number of candidate pairs (ungapped extensions), hits, and hits whose
  gapped score passes S2;
* a 64-bit multiset digest of the hit records (seq1, pos1, seq2, pos2, score),
  of the records with their gapped score appended, and of the passing records:
  the count, the sum modulo 2^64 and the exclusive-or of a 64-bit mix of every
  record.  Both reductions are independent of the order of the records, and a
  record reported twice changes the count and cancels itself out of the xor;
* the same three numbers for the records with gapped scores per block of 80
  consecutive seed keys, which names the keys of a mismatch;
* SHA-256 of the generated banks (a changed generator would make every digest
  meaningless) and, for the translated workloads, of the oracle's fragment
  bank and fragment table, which the device translation must equal byte for
  byte.

Writing the goldens calls only ``oracle/`` (and the seeded input generators):

    python tests/golden/fullsize.py 1 2 3 x [--threads N]

writes ``fullsize_cfg<c>.json`` next to this file (``x`` is the PLAST-X
workload).  The digest functions below are shared by the GPU tests and the
benchmark, which apply them to the device's output.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))

KEYS_PER_BLOCK = 80
N_BLOCKS = 110            # 8800 seed keys / 80

_C1 = np.uint64(0xFF51AFD7ED558CCD)
_C2 = np.uint64(0xC4CEB9FE1A85EC53)
_S33 = np.uint64(33)
_S32 = np.uint64(32)
_LO32 = np.uint64(0xFFFFFFFF)


def _fmix(x):
    """64-bit finaliser of MurmurHash3 (a bijection on uint64)."""
    x = x ^ (x >> _S33)
    x = x * _C1
    x = x ^ (x >> _S33)
    x = x * _C2
    return x ^ (x >> _S33)


def _u64(a):
    return np.asarray(a).astype(np.int64).astype(np.uint64) & _LO32


def record_mix(hits, gscore=None):
    """uint64 mix of every record: hits int[n, 5] (seq1, pos1, seq2, pos2,
    score), gscore int[n] or None."""
    h = np.asarray(hits).reshape(-1, 5)
    with np.errstate(over="ignore"):
        z = _fmix((_u64(h[:, 0]) << _S32) | _u64(h[:, 1]))
        z = _fmix(z ^ ((_u64(h[:, 2]) << _S32) | _u64(h[:, 3])))
        tail = _u64(h[:, 4]) << _S32
        if gscore is not None:
            tail = tail | _u64(gscore) | np.uint64(1 << 63)
        return _fmix(z ^ tail)


def digest(hits, gscore=None):
    """{"count", "sum", "xor"} of ``record_mix`` (sum modulo 2^64; hex strings)."""
    m = record_mix(hits, gscore)
    s = int(np.sum(m, dtype=np.uint64)) if m.size else 0
    x = int(np.bitwise_xor.reduce(m)) if m.size else 0
    return {"count": int(m.size), "sum": "%016x" % s, "xor": "%016x" % x}


def _merge(d, m):
    """Adds the mixes m to an accumulating (count, sum, xor) triple."""
    c, s, x = d
    if m.size:
        s = (s + int(np.sum(m, dtype=np.uint64))) & 0xFFFFFFFFFFFFFFFF
        x ^= int(np.bitwise_xor.reduce(m))
    return (c + int(m.size), s, x)


def _as_dict(t):
    return {"count": t[0], "sum": "%016x" % t[1], "xor": "%016x" % t[2]}


def block_digests(hits, gscore, key):
    """Per block of KEYS_PER_BLOCK seed keys: [count, sum, xor] of the records
    with gapped scores; key = seed key of every record."""
    m = record_mix(hits, gscore)
    blk = (np.asarray(key, dtype=np.int64) // KEYS_PER_BLOCK).astype(np.uint8)
    order = np.argsort(blk, kind="stable")          # radix sort on 8-bit keys
    m = m[order]
    bounds = np.searchsorted(blk[order], np.arange(N_BLOCKS + 1))
    out = []
    for b in range(N_BLOCKS):
        t = _merge((0, 0, 0), m[bounds[b]:bounds[b + 1]])
        out.append([t[0], "%016x" % t[1], "%016x" % t[2]])
    return out


def seed_keys(bank1, hits):
    """Seed key of every hit record, from the bank-1 word at (seq1, pos1)."""
    from oracle import plast_oracle as O
    h = np.asarray(hits).reshape(-1, 5)
    c = bank1.codes
    q = bank1.seq_start[h[:, 0].astype(np.int64)] + h[:, 1].astype(np.int64)
    return O.seed_key(*(c[q + i].astype(np.int64) for i in range(4)))


def device_summary(hits, gscore, s2, bank1, n_ext):
    """``summary`` (with block digests) of a device result: hits int32[n, 5]
    and gscore int32[n] torch tensors (or numpy arrays), bank1 the host bank
    whose words give the seed keys."""
    h = hits.cpu().numpy() if hasattr(hits, "cpu") else np.asarray(hits)
    g = gscore.cpu().numpy() if hasattr(gscore, "cpu") else np.asarray(gscore)
    out = summary(h, g, s2, seed_keys(bank1, h))
    out["n_ext"] = int(n_ext)
    return out


def summary(hits, gscore, s2, key=None):
    """The comparable part of a golden, computed from one full hit list."""
    g = np.asarray(gscore).reshape(-1)
    ok = g >= s2
    h = np.asarray(hits).reshape(-1, 5)
    out = {"n_hits": int(h.shape[0]), "n_pass": int(ok.sum()),
           "hits": digest(h), "hits_gscore": digest(h, g), "passing": digest(h[ok], g[ok])}
    if key is not None:
        out["blocks"] = block_digests(h, g, key)
    return out


def golden_path(cfg):
    return os.path.join(HERE, "fullsize_cfg%s.json" % cfg)


def load(cfg):
    """The stored golden of workload ``cfg`` (1, 2, 3 or "x"), or None."""
    p = golden_path(cfg)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        return json.load(f)


def compare(golden, got):
    """List of the fields where ``got`` (a ``summary`` plus "n_ext") differs
    from ``golden``; empty when equal.  Block digests are compared only when
    both sides have them."""
    bad = []
    for k in ("n_ext", "n_hits", "n_pass", "hits", "hits_gscore", "passing"):
        if k in got and got[k] != golden[k]:
            bad.append(k)
    if "blocks" in got and "blocks" in golden:
        for b, (x, y) in enumerate(zip(golden["blocks"], got["blocks"])):
            if list(x) != list(y):
                bad.append("block %d (keys %d..%d)" % (b, b * KEYS_PER_BLOCK, (b + 1) * KEYS_PER_BLOCK - 1))
    return bad


def sha256_arrays(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


# --------------------------------------------------------------------- writer

def _oracle_run(bank1, bank2, s1, s2, threads, with_blocks, log):
    """Oracle over all keys, one block of keys at a time: counts, digests and
    per-block digests of (hits, gapped scores)."""
    from oracle import coracle as C
    from oracle import plast_oracle as O

    t0 = time.perf_counter()
    idx1, idx2 = C.build_index(bank1), C.build_index(bank2)
    work = np.diff(idx1[0]) * np.diff(idx2[0])
    n_ext = 0
    acc = {"hits": (0, 0, 0), "hits_gscore": (0, 0, 0), "passing": (0, 0, 0)}
    blocks = []
    n_pass = 0
    for b in range(N_BLOCKS):
        keys = np.arange(b * KEYS_PER_BLOCK, (b + 1) * KEYS_PER_BLOCK, dtype=np.int32)
        keys = keys[work[keys] > 0]
        blk = (0, 0, 0)
        if len(keys):
            guess = int(work[keys].sum() * 0.004) + 4096
            h, ne = C.ungapped_hits(bank1, bank2, s1, keys=keys, idx1=idx1, idx2=idx2, nthreads=threads,
                                    canonicalize=False, capacity=guess)
            n_ext += ne
            g = C.gapped_scores(bank1, bank2, h, nthreads=threads) if len(h) else np.zeros(0, np.int64)
            ok = g >= s2
            n_pass += int(ok.sum())
            acc["hits"] = _merge(acc["hits"], record_mix(h))
            mg = record_mix(h, g)
            acc["hits_gscore"] = _merge(acc["hits_gscore"], mg)
            acc["passing"] = _merge(acc["passing"], mg[ok])
            blk = _merge(blk, mg)
        blocks.append([blk[0], "%016x" % blk[1], "%016x" % blk[2]])
        if b % 10 == 9:
            log("  block %d/%d: %d hits so far, %.0f s" % (b + 1, N_BLOCKS, acc["hits"][0],
                                                          time.perf_counter() - t0))
    assert n_ext == O.n_extensions(idx1, idx2)
    out = {"n_ext": int(n_ext), "n_hits": acc["hits"][0], "n_pass": n_pass}
    out.update({k: _as_dict(v) for k, v in acc.items()})
    if with_blocks:
        out["blocks"] = blocks
    out["oracle_seconds"] = round(time.perf_counter() - t0, 1)
    return out


def _fragment_bank(dna):
    """The oracle's six-frame translation of a nucleotide bank, as a padded
    protein bank plus the int32 (dna, frame, offset) table."""
    from oracle import plast_oracle as O
    from paper_0804_3643_amd import synth
    frags, table = O.translate6(dna.codes, dna.start)
    return synth.Bank.from_seqs(frags), table.astype(np.int32)


def write(cfg, threads, log=print):
    from paper_0804_3643_amd import synth
    from oracle import plast_oracle as O

    with open(os.path.join(HERE, "thresholds.json")) as f:
        th = json.load(f)
    s1, s2 = int(th["s1"]), int(th["s2"])
    g = {"workload": None, "writer": "tests/golden/fullsize.py (CPU oracle only)",
         "params": {"S1": s1, "S2": s2, "nbr": O.NBR, "gap_window": O.GAP_WINDOW, "gap_band": O.GAP_BAND,
                    "gap_open": O.GAP_OPEN, "gap_extend": O.GAP_EXTEND, "matrix": "BLOSUM62"},
         "digest": "record mix = fmix64(fmix64(fmix64(seq1<<32|pos1) ^ (seq2<<32|pos2)) ^ (score<<32 [| gscore "
                   "| 1<<63])); sum mod 2^64 and xor over the records; blocks of %d seed keys" % KEYS_PER_BLOCK}
    if cfg in ("1", "2", "0"):
        w = synth.make_workload(int(cfg))
        g["workload"] = "PLAST-P configuration %s: %s" % (cfg, w.description)
        g["bank_sha256"] = [w.bank1.sha256(), w.bank2.sha256()]
        bank1, bank2 = w.bank1, w.bank2
    elif cfg == "3":
        w = synth.make_tplastn()
        g["workload"] = w.description
        log("translating %d DNA sequences (oracle)" % w.dna.n_seqs)
        bank2, table = _fragment_bank(w.dna)
        g["bank_sha256"] = [w.bank1.sha256(), sha256_arrays(w.dna.codes, w.dna.start)]
        g["fragments"] = [{"n": int(table.shape[0]), "codes_sha256": sha256_arrays(bank2.codes),
                           "seq_start_sha256": sha256_arrays(bank2.seq_start.astype(np.int64)),
                           "table_sha256": sha256_arrays(table)}]
        bank1 = w.bank1
    elif cfg == "x":
        w = synth.make_plastx()
        g["workload"] = w.description
        g["bank_sha256"] = [sha256_arrays(w.dna1.codes, w.dna1.start), sha256_arrays(w.dna2.codes, w.dna2.start)]
        g["fragments"] = []
        banks = []
        for d in (w.dna1, w.dna2):
            log("translating %d DNA sequences (oracle)" % d.n_seqs)
            fb, table = _fragment_bank(d)
            banks.append(fb)
            g["fragments"].append({"n": int(table.shape[0]), "codes_sha256": sha256_arrays(fb.codes),
                                   "seq_start_sha256": sha256_arrays(fb.seq_start.astype(np.int64)),
                                   "table_sha256": sha256_arrays(table)})
        bank1, bank2 = banks
    else:
        raise SystemExit("unknown workload %r" % cfg)
    log("oracle over all keys of %s" % g["workload"])
    g.update(_oracle_run(bank1, bank2, s1, s2, threads, True, log))
    with open(golden_path(cfg), "w") as f:
        json.dump(g, f, indent=1)
        f.write("\n")
    log("wrote %s: %d extensions, %d hits, %d pass (%.0f s)" % (golden_path(cfg), g["n_ext"], g["n_hits"],
                                                                 g["n_pass"], g["oracle_seconds"]))
    return g


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("configs", nargs="+", help="workloads: 0, 1, 2, 3 (TPLAST-N) or x (PLAST-X)")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    sys.path.insert(0, ROOT)
    for c in args.configs:
        write(c, args.threads, log=lambda m: print(m, flush=True))


if __name__ == "__main__":
    main()
