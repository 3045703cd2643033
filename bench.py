#!/usr/bin/env python3
"""Benchmark of the PLAST-P bank-versus-bank hot path on one MI355X.

One step = the whole hot path over one pair of banks already resident in HBM:
index bank 1 and bank 2 (stage 0), batched ungapped extension of every
candidate pair with hit compaction (stage 2), small gapped filter on the hits
(stage 3.1).  The step is replayed from one HIP graph (``plast_pipeline_*``),
with launch shapes measured by the library's autotuner first.  ``value`` =
candidate pairs (ungapped extensions) per second of step wall time.  Also
reported:
  * the same step made of the separate eager calls (with their host
    synchronisations) and its per-stage device times, and a check that graph
    and eager calls give the same hits;
  * the ungapped stage alone, PLAIN (one grid per key) vs BATCHED (persistent
    work queue), device time from HIP events, after checking that both give the
    same hit multiset;
  * bank-vs-bank wall time from host-resident encoded banks to the host hit
    list (host-to-device copy, both indexes, ungapped, gapped, device-to-host),
    for both schedules;
  * ``roofline`` for the dominant kernel (the persistent ungapped kernel):
    algorithmic int16 ALU operations (44 additions and 44 maxima per
    extension) per second against the packed-int16 VALU peak;
  * ``stage32``: stage 3.2 (full gapped alignment, with the list of pieces of
    computed alignments) over the hits that pass the filter, outside the step:
    wall time of the call, DP cells per second, and the C oracle on a seeded
    sample of sequence pairs checked against the GPU records;
  * ``cpu_baseline``: the CPU oracle (plain C, all allotted host threads) on a
    seeded sample of keys of the same workload, scaled to the whole job, and
    its hits compared with the GPU's for those keys.

Usage: python bench.py [--steps K] [--warmup W] [--config 1|2|3] [--serving] [--plastx]
"""
import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ungapped extensions/sec and bank-vs-bank wall time (plain vs batched, bit-exact)"
# Ungapped extension, per candidate pair: 44 scan steps, each one substitution
# lookup, one addition and one maximum.  The kernel serves the lookups from an
# LDS profile (2 bytes per step), so its VALU work is the 88 additions and
# maxima and its LDS work is 88 bytes; counting the lookups as ALU operations
# too gives 132 operations per pair.
OPS_PER_EXT = 88
OPS_PER_EXT_WITH_LOOKUPS = 132
LDS_BYTES_PER_EXT = 88
# MI355X: 256 CUs x 64 VALU lanes x 2 int16 ops per packed instruction x 2.4 GHz
PEAK_INT16_TOPS = 256 * 64 * 2 * 2.4e9 / 1e12
# LDS, 8-byte reads: 256 bytes per CU per clock (one 64-lane ds_read_b64 every
# two clocks); the 64-bit LDS probe sustains 226 bytes per CU per clock
# (rocprofv3 counters), above the 128 of earlier CDNA parts
PEAK_LDS_TBS = 256 * 256 * 2.4e9 / 1e12
# Gapped filter: about 8 operations per DP cell (E: 2, F: 2, H: lookup, add and
# two maxima, best: 1), packed 16-bit
GAPPED_OPS_PER_CELL = 8
# Stage 3.2: 7 int32 operations per DP cell (E: subtract, max; F: subtract, max;
# diagonal add; two maxima for H) against 256 CUs x 64 VALU lanes x 2.4 GHz
ALIGN_OPS_PER_CELL = 7
PEAK_INT32_TOPS = 256 * 64 * 2.4e9 / 1e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ungapped_persistent_cfg1_traffic.md")
KERNEL_SRC = os.path.join(ROOT, "paper_0804_3643_amd", "csrc", "ungapped.hip")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash(src=KERNEL_SRC):
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def recorded_traffic(path, src=KERNEL_SRC, key="traffic_bytes_per_launch"):
    """HBM bytes per launch of a kernel from a committed rocprofv3 counter
    summary, if it was taken on the current kernel source (``key`` names the
    figure, e.g. the one for a given workgroup size)."""
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    b = re.search(r"^%s:\s*([0-9.eE+]+)" % re.escape(key), txt, re.M)
    if not m or not b or m.group(1) != kernel_source_hash(src):
        return None
    return float(b.group(1))


def traffic_file(kernel, cfg):
    return os.path.join(ROOT, "profiles", "%s_cfg%s_traffic.md" % (kernel, cfg))


def golden_check(cfg, hits, gscore, s2, n_ext, bank1, banks_sha):
    """The whole run against the oracle's full-size golden of workload ``cfg``
    (tests/golden/fullsize.py): counts and 64-bit multiset digests of the hit
    records and their gapped scores, whole run and per block of 80 keys."""
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import fullsize
    golden = fullsize.load(cfg)
    if golden is None:
        return {"golden": None, "equal": False, "mismatch": ["no stored golden for workload %s" % cfg]}
    if golden["bank_sha256"] != banks_sha:
        return {"golden": os.path.basename(fullsize.golden_path(cfg)), "equal": False,
                "mismatch": ["generated banks differ from the golden's"]}
    got = fullsize.device_summary(hits, gscore, s2, bank1, n_ext)
    bad = fullsize.compare(golden, got)
    return {"golden": os.path.basename(fullsize.golden_path(cfg)), "equal": not bad, "mismatch": bad,
            "n_hits": got["n_hits"], "n_pass": got["n_pass"], "digest": got["hits_gscore"]}


def gapped_cells(np, bank1, bank2, hits, window=64, band=16):
    """DP cells of the gapped filter over a hit list (host int arrays): both
    sides of every hit, each the cells (i, j) != (0, 0), 0 <= i <= lx,
    0 <= j <= ly, |i - j| <= band of its clipped windows (at most 1872 per
    side)."""
    lx = np.arange(window + 1)[:, None]
    ly = np.arange(window + 1)[None, :]
    table = np.zeros((window + 1, window + 1), dtype=np.int64)
    for i in range(window + 1):
        lo, hi = max(0, i - band), i + band
        row = np.clip(np.minimum(ly, hi) - lo + 1, 0, None)           # cells of row i when ly is given
        table += np.where(lx >= i, row, 0)
    h = np.asarray(hits, dtype=np.int64)
    la = np.diff(bank1.seq_start) - 20
    lb = np.diff(bank2.seq_start) - 20
    s1, p1, s2, p2 = h[:, 0], h[:, 1], h[:, 2], h[:, 3]
    right = table[np.minimum(window, la[s1] - p1), np.minimum(window, lb[s2] - p2)]
    left = table[np.minimum(window, p1), np.minimum(window, p2)]
    return int(right.sum() + left.sum()) - 2 * len(h)   # the anchor cell (0, 0) of each side is given


def copy_calibration(torch, dev):
    """Elementwise kernel of known traffic for scaling rocprofv3 FETCH_SIZE /
    WRITE_SIZE: reads 256 MiB and writes 256 MiB per launch (int32 negation)."""
    src = torch.ones(64 << 20, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()


def pair_keys_device(torch, hits):
    """Sorted 64-bit pair keys and their scores (positions < 2^11, bank-2
    sequence ids < 2^19, bank-1 ids < 2^22)."""
    h = hits.to(torch.int64)
    k = (((h[:, 0] << 11) | h[:, 1]) << 30) | (h[:, 2] << 11) | h[:, 3]
    k, o = torch.sort(k)
    return k, h[o, 4]


def cpu_baseline(w, gpu_hits_host, gpu_gscore_host, n_ext_total, sample_ext, s1, s2):
    """Oracle (plain C) on a seeded key sample; returns the JSON object.  The
    GPU's hits and gapped scores of the sampled keys are compared with the
    oracle's (``oracle_hits_equal_gpu_on_sample``,
    ``oracle_gapped_equal_gpu_on_sample``)."""
    import numpy as np

    from oracle import coracle as C
    from oracle import plast_oracle as O

    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    t0 = time.perf_counter()
    i1, i2 = C.build_index(w.bank1), C.build_index(w.bank2)
    t_index = time.perf_counter() - t0
    work = np.diff(i1[0]) * np.diff(i2[0])
    rng = np.random.default_rng(6513)
    keys = []
    acc = 0
    for k in rng.permutation(np.nonzero(work)[0]):
        keys.append(int(k))
        acc += int(work[k])
        if acc >= sample_ext:
            break
    keys_1t = np.array(sorted(keys[: max(1, len(keys) // 16)]), dtype=np.int32)  # same random order
    keys = np.array(sorted(keys), dtype=np.int32)
    t0 = time.perf_counter()
    ref, n_ext_s = C.ungapped_hits(w.bank1, w.bank2, s1, keys=keys, idx1=i1, idx2=i2, nthreads=cores)
    t_ung = time.perf_counter() - t0
    t0 = time.perf_counter()
    g = C.gapped_scores(w.bank1, w.bank2, ref, nthreads=cores)
    t_gap = time.perf_counter() - t0
    # bit-exact check of the GPU hits on the sampled keys
    c = w.bank1.codes
    q = w.bank1.seq_start[gpu_hits_host[:, 0]] + gpu_hits_host[:, 1]
    hk = O.seed_key(c[q].astype(np.int64), c[q + 1].astype(np.int64), c[q + 2].astype(np.int64),
                    c[q + 3].astype(np.int64))
    sel = np.isin(hk, keys)
    mine_h, mine_g = gpu_hits_host[sel], gpu_gscore_host[sel]
    order = np.lexsort(mine_h.T[::-1])
    mine_h, mine_g = mine_h[order], mine_g[order]
    equal = bool(np.array_equal(mine_h, ref))
    g_equal = bool(equal and np.array_equal(mine_g, g))
    t_job = t_index + (t_ung + t_gap) * (n_ext_total / max(1, n_ext_s))
    # one thread, ungapped loop only, on a sixteenth of the sampled keys
    t0 = time.perf_counter()
    _, n_ext_1 = C.ungapped_hits(w.bank1, w.bank2, s1, keys=keys_1t, idx1=i1, idx2=i2, nthreads=1,
                                 canonicalize=False)
    t_1 = time.perf_counter() - t0
    # configuration 0 end to end: both indexes, every key, the gapped filter and the sorted list
    from paper_0804_3643_amd import synth
    w0 = synth.make_workload(0)
    e2e = {}
    for nt in (cores, 1):
        t0 = time.perf_counter()
        j1, j2 = C.build_index(w0.bank1), C.build_index(w0.bank2)
        r0, n0 = C.ungapped_hits(w0.bank1, w0.bank2, s1, idx1=j1, idx2=j2, nthreads=nt)
        C.gapped_scores(w0.bank1, w0.bank2, r0, nthreads=nt)
        e2e["%d_threads_s" % nt] = time.perf_counter() - t0
    e2e["extensions"] = int(n0)
    return {
        "value": n_ext_total / t_job, "unit": "ext/s", "cores": cores, "kind": "oracle",
        "sample": ("plain C oracle, %d threads: index of both full banks (%.2f s) + %d seeded random keys "
                   "(%d extensions, %.1f%% of the job; ungapped %.2f s, gapped on its %d hits %.2f s), "
                   "scaled to all %d extensions" % (cores, t_index, len(keys), n_ext_s, 100.0 * n_ext_s /
                                                    n_ext_total, t_ung, len(ref), t_gap, n_ext_total)),
        "oracle_hits_equal_gpu_on_sample": equal, "oracle_gapped_equal_gpu_on_sample": g_equal,
        "n_gapped_pass_sample": int((g >= s2).sum()),
        "single_thread": {"ext_per_s": n_ext_1 / t_1,
                          "sample": "ungapped loop, 1 thread, %d of the sampled keys (%d extensions) in %.2f s"
                                    % (len(keys_1t), n_ext_1, t_1)},
        "config0_end_to_end": e2e,
    }


# Published MI355X figures the measured peaks stand for: 256 CUs at up to
# 2.4 GHz, 64 int32 / 128 packed 16-bit lane operations per clock per CU, LDS
# 32 lookups of 4 bytes and 256 bytes of 8-byte reads per clock per CU, HBM3E
# 8 TB/s.
PUBLISHED_PEAKS = {"valu_i32": 256 * 64 * 2.4e9, "valu_pk_i16": 256 * 128 * 2.4e9, "valu_pk_f16": 256 * 128 * 2.4e9,
                   "lds_lookup": 256 * 32 * 2.4e9, "hbm_copy": 8e12, "lds_b64": 256 * 256 * 2.4e9,
                   "sclk": 2.4e9}


def machine_info():
    """Host CPU (model, sockets, threads) and the GPU's engine clock levels
    as sysfs lists them (the current level is starred), when readable."""
    info = {"host_logical_cpus": os.cpu_count()}
    try:
        info["host_cpus_allowed"] = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    try:
        txt = open("/proc/cpuinfo").read()
        models = re.findall(r"^model name\s*:\s*(.+)$", txt, re.M)
        info["host_cpu_model"] = models[0].strip() if models else None
        info["host_sockets"] = len(set(re.findall(r"^physical id\s*:\s*(\d+)$", txt, re.M))) or None
    except OSError:
        pass
    clocks = []
    for path in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk"))[:8]:
        try:
            clocks.append(" ".join(open(path).read().split()))
        except OSError:
            pass
    info["gpu_sclk_levels"] = clocks or None
    return info


def measured_peaks(B, torch, dev):
    """plast_probe_peak rates (best of 3) beside the published figures."""
    buf = B._alloc(4 << 30, dev)  # the copy moves 2 GiB each way
    out = {}
    for kind, (_code, unit) in B.PROBES.items():
        r = B.probe_peak(kind, buf, reps=3)
        out[kind] = {"rate": r, "unit": unit, "published": PUBLISHED_PEAKS[kind],
                     "frac_of_published": r / PUBLISHED_PEAKS[kind]}
    del buf
    # lane operations per CU per clock at the published 2.4 GHz and at the engine clock the clock probe
    # measured inside its kernel (64 int32 and 128 packed 16-bit by the published figures)
    out["valu_i32_lane_ops_per_cu_clock_at_2_4_ghz"] = out["valu_i32"]["rate"] / (256 * 2.4e9)
    sclk = out["sclk"]["rate"]
    out["per_cu_clock_at_measured_sclk"] = {
        k: out[k]["rate"] / (256 * sclk) for k in ("valu_i32", "valu_pk_i16", "valu_pk_f16", "lds_lookup", "lds_b64")}
    return out


def plant_recall(torch, np, w, hits, passed):
    """Planted homologous pairs with at least one ungapped hit and with at
    least one hit passing the gapped filter, by bins of realised identity."""
    if not w.plants:
        return None
    n2 = w.bank2.n_seqs
    h = hits.to(torch.int64)
    key = h[:, 0] * n2 + h[:, 2]
    pk = torch.tensor([p.src * n2 + p.dst for p in w.plants], dtype=torch.int64, device=hits.device)
    found = torch.isin(pk, key).cpu().numpy()
    found_g = torch.isin(pk, key[passed.to(torch.bool)]).cpu().numpy()
    ident = np.array([p.identity for p in w.plants])
    bins = []
    for lo in np.arange(0.20, 0.70, 0.05):
        m = (ident >= lo - 1e-9) & (ident < lo + 0.05 - 1e-9)
        if m.any():
            bins.append({"identity": [round(float(lo), 2), round(float(lo + 0.05), 2)], "pairs": int(m.sum()),
                         "with_hit": int(found[m].sum()), "passing_gapped": int(found_g[m].sum())})
    return {"pairs": len(w.plants), "with_hit": int(found.sum()), "passing_gapped": int(found_g.sum()),
            "by_realised_identity": bins}


def key_stats(torch, np, ia, ib):
    """Bucket sizes per seed key (bank 2) and the share of the work in the 16
    heaviest keys (n1 x n2)."""
    n1 = torch.diff(ia.key_off()).to(torch.float64)
    n2 = torch.diff(ib.key_off()).to(torch.float64)
    work = n1 * n2
    c2 = n2.cpu().numpy()
    nz = c2[c2 > 0]
    hist = np.bincount(np.floor(np.log2(nz)).astype(np.int64)) if nz.size else np.zeros(0, np.int64)
    return {
        "bank2_nonempty_keys": int(nz.size),
        "bank2_max": int(nz.max()) if nz.size else 0,
        "bank2_min_nonempty": int(nz.min()) if nz.size else 0,
        "bank2_quantiles_50_90_99": [float(np.quantile(nz, q)) for q in (0.5, 0.9, 0.99)] if nz.size else None,
        "bank2_log2_histogram": {"%d-%d" % (1 << k, (2 << k) - 1): int(c) for k, c in enumerate(hist) if c},
        "top16_work_share": float(torch.topk(work, 16).values.sum().item() / max(1.0, work.sum().item())),
    }


def run_stage32(B, torch, np, w, ia, ib, hits, gs, ps, reps, cpu):
    """Stage 3.2 over the hits that passed the gapped filter: wall time of the
    synchronous call (grouping sort, alignment kernel), alignments, covered
    hits, DP cells (both sides of every computed alignment), and optionally the
    C oracle on a seeded sample of sequence pairs, checked against the GPU."""
    from oracle import coracle as C
    from oracle import plast_oracle as O
    n = hits.shape[0]
    al = B.Aligner(ia, ib, n)
    al.run(hits, gs, ps)
    torch.cuda.synchronize()
    walls, kernel_ms = [], []
    B.timing_enable(True)
    for _ in range(reps):
        t1 = time.perf_counter()
        rec, cov = al.run(hits, gs, ps)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t1)
        kernel_ms.append(B.timing_read()["align_ms"])
    B.timing_enable(False)
    F = {k: i for i, k in enumerate(B.ALIGN_FIELDS)}
    r = rec.cpu().numpy().astype(np.int64)
    la = np.diff(w.bank1.seq_start) - B.PAD_LEN
    lb = np.diff(w.bank2.seq_start) - B.PAD_LEN
    s1, s2, p1, p2 = r[:, F["seq1"]], r[:, F["seq2"]], r[:, F["seed1"]], r[:, F["seed2"]]
    cells = int(((la[s1] - p1) * (lb[s2] - p2) + p1 * p2).sum())
    n_pass = int(ps.sum().item())
    ms = 1e3 * float(np.min(walls))
    kms = float(np.mean(kernel_ms))
    achieved = cells * ALIGN_OPS_PER_CELL / (kms * 1e-3) / 1e12
    out = {"passing_hits": n_pass, "alignments": len(r), "covered_hits": n_pass - len(r), "call_ms": ms,
           "kernel_ms": kms, "dp_cells": cells, "dp_cells_per_s": cells / (ms * 1e-3),
           "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_INT32_TOPS, "unit": "TOP/s",
                        "frac": achieved / PEAK_INT32_TOPS, "traffic": None, "kernel": "k_align",
                        "ops_per_cell": ALIGN_OPS_PER_CELL},
           "mean_score": float(r[:, F["score"]].mean()) if len(r) else 0.0,
           "call": "plast_align: key pass, radix sort by (seq1, seq2, -gscore, pos1, pos2), alignment kernel; "
                   "wall time of the synchronous call, best of %d" % reps}
    if cpu:
        hh = hits.cpu().numpy().astype(np.int64)
        gg = gs.cpu().numpy().astype(np.int64)
        pp = ps.cpu().numpy().astype(bool)
        idx = np.nonzero(pp)[0]
        key = hh[idx, 0] * (1 << 20) + hh[idx, 2]
        ukeys = np.unique(key)
        pick = np.random.default_rng(7).choice(ukeys, size=min(len(ukeys), max(1, len(ukeys) // 50)), replace=False)
        sel = idx[np.isin(key, pick)]
        threads = min(16, os.cpu_count() or 1)
        t1 = time.perf_counter()
        ref, rcov = C.full_alignments(w.bank1, w.bank2, hh[sel], gg[sel], np.ones(len(sel), bool), nthreads=threads)
        cpu_s = time.perf_counter() - t1
        ref[:, F["hit"]] = sel[ref[:, F["hit"]]]
        ref = ref[np.lexsort(ref.T[::-1])]
        rk = r[:, F["seq1"]] * (1 << 20) + r[:, F["seq2"]]
        got = r[np.isin(rk, pick)]
        got = got[np.lexsort(got.T[::-1])]
        cov_h = cov.cpu().numpy().astype(np.int64)
        same = bool(np.array_equal(got, ref) and np.array_equal(cov_h[sel], sel[rcov]))
        rs1, rs2, rp1, rp2 = ref[:, F["seq1"]], ref[:, F["seq2"]], ref[:, F["seed1"]], ref[:, F["seed2"]]
        rcells = int(((la[rs1] - rp1) * (lb[rs2] - rp2) + rp1 * rp2).sum())
        out["oracle_equals_gpu_on_sample_pairs"] = same
        out["cpu_oracle"] = {"dp_cells_per_s": rcells / max(cpu_s, 1e-9), "cores": threads, "kind": "oracle",
                             "sample": "plain C oracle, %d threads, on %d seeded random sequence pairs (%d passing "
                                       "hits, %d alignments, %d DP cells) in %.2f s" % (
                                           threads, len(pick), len(sel), len(ref), rcells, cpu_s)}
    return out


def serving_leg(args, n_requests=None, oracle_checks=True):
    """Serving workload (config 4): a resident bank of 1M proteins indexed once
    in HBM, query banks of 1-500 proteins with Poisson arrivals at 0.7 x the
    saturation throughput measured first, continuous batching over several
    slots.  Checks, asserted by the caller: sampled requests give the same
    matches alone as in the mix, and the smallest requests' matches equal the
    oracle's (ungapped hits that pass the gapped filter, with both scores)."""
    import numpy as np
    import torch

    from paper_0804_3643_amd import binding as B
    from paper_0804_3643_amd import params
    from paper_0804_3643_amd import serving as S
    from paper_0804_3643_amd import synth

    B.load()
    n_requests = n_requests or args.serving_requests
    log("generating the serving workload (scale %.3g, %d requests)" % (args.serving_scale, n_requests))
    w = synth.make_serving(n_requests=n_requests, scale=args.serving_scale)
    log("indexing the resident bank (%d proteins, %d residues)" % (w.resident.n_seqs, w.resident.n_residues))
    t1 = time.perf_counter()
    res = S.Resident(w.resident.codes, w.resident.seq_start)
    torch.cuda.synchronize()
    index_s = time.perf_counter() - t1
    srv = S.Server(res, slots=args.serving_slots)

    def reqs(arrivals):
        return [S.Request(i, b.codes, b.seq_start, arrival=float(t)) for i, (b, t) in enumerate(zip(w.requests, arrivals))]

    n_sat = min(len(w.requests), max(1, len(w.requests) // 2))
    log("saturation run (%d requests at t=0)" % n_sat)
    srv.run(reqs([0.0] * len(w.requests))[:n_sat])  # warm-up
    sat = reqs([0.0] * len(w.requests))[:n_sat]
    e0, l0 = srv.total_ext, len(srv.batch_log)
    span = srv.run(sat)
    slog = np.array(srv.batch_log[l0:], dtype=np.float64).reshape(-1, 6)
    cap_rps = n_sat / span
    sat_ext = (srv.total_ext - e0) / span
    rate = 0.7 * cap_rps
    rng = np.random.default_rng(6513)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(w.requests)))
    log("Poisson run: %d requests at %.1f req/s (0.7 x %.1f)" % (len(w.requests), rate, cap_rps))
    mix = reqs(arrivals)
    e0, b0, s0, l0 = srv.total_ext, srv.batches, srv.splits, len(srv.batch_log)
    span = srv.run(mix, progress=lambda d, n: log("served %d/%d" % (d, n)))
    ext = srv.total_ext - e0
    stats = S.latency_stats(mix)
    blog = np.array(srv.batch_log[l0:], dtype=np.float64).reshape(-1, 6)
    busy = span - float(arrivals[0])
    log("identity check: sampled requests alone")
    pick = np.random.default_rng(7).choice(len(w.requests), size=min(16, len(w.requests)), replace=False)
    same = True
    for i in pick:
        alone = reqs([0.0] * len(w.requests))[int(i)]
        srv.run([alone])
        same &= bool(np.array_equal(S.canonical(alone.matches), S.canonical(mix[int(i)].matches)))
    # planted homolog pairs (query sequence, resident sequence) among the matches, on the sampled requests
    found = planted = 0
    for i in pick:
        h = np.asarray(w.homologs[int(i)], dtype=np.int64).reshape(-1, 2)
        mk = mix[int(i)].matches[:, 0].astype(np.int64) * (1 << 21) + mix[int(i)].matches[:, 2]
        found += int(np.isin(h[:, 0] * (1 << 21) + h[:, 1], mk).sum())
        planted += len(h)
    bit_exact = {"alone_equals_mix_on_%d_sampled_requests" % len(pick): same}
    if oracle_checks:
        from oracle import coracle as C
        small = np.argsort([b.n_seqs for b in w.requests], kind="stable")[:3]
        log("oracle on the %d smallest requests" % len(small))
        idx_res = C.build_index(w.resident)
        eq = True
        for i in small:
            q = w.requests[int(i)]
            hq, _ = C.ungapped_hits(q, w.resident, params.S1, idx2=idx_res,
                                    nthreads=min(16, os.cpu_count() or 1))
            gq = C.gapped_scores(q, w.resident, hq, nthreads=min(16, os.cpu_count() or 1))
            ok = gq >= params.S2
            ref = S.canonical(np.column_stack([hq[ok], gq[ok]]))
            eq &= bool(np.array_equal(ref, S.canonical(mix[int(i)].matches)))
        bit_exact["oracle_equals_gpu_on_%d_smallest_requests" % len(small)] = eq
    bit_exact["all"] = all(bit_exact.values())
    return {
        "value": ext / busy, "unit": "ext/s",
        "p50_ms": stats["p50_ms"], "p99_ms": stats["p99_ms"], "mean_ms": stats["mean_ms"], "max_ms": stats["max_ms"],
        "requests": len(mix), "arrival_rate_rps": rate, "saturation_rps": cap_rps, "saturation_ext_per_s": sat_ext,
        "batches": srv.batches - b0, "splits": srv.splits - s0,
        "mean_batch_requests": float(np.mean([r.batch_size for r in mix])),
        "saturation_batch_means": {"requests": float(slog[:, 0].mean()), "ext": float(slog[:, 1].mean()),
                                   "hits": float(slog[:, 2].mean()), "device_ms": float(slog[:, 4].mean()),
                                   "host_split_ms": float(slog[:, 5].mean()), "batches": int(len(slog))},
        "batch_means": {"requests": float(blog[:, 0].mean()), "ext": float(blog[:, 1].mean()),
                        "hits": float(blog[:, 2].mean()), "matches": float(blog[:, 3].mean()),
                        "device_ms": float(blog[:, 4].mean()), "host_split_ms": float(blog[:, 5].mean()),
                        "device_ext_per_s": float(blog[:, 1].sum() / (blog[:, 4].sum() * 1e-3))},
        "slots": args.serving_slots, "resident_index_s": index_s,
        "bit_exact": bit_exact,
        "planted_homologs_found_on_sampled_requests": "%d/%d" % (found, planted),
        "matches_per_request_mean": float(np.mean([len(r.matches) for r in mix])),
        "workload": w.description, "resident_residues": w.resident.n_residues,
        "query_proteins": int(sum(b.n_seqs for b in w.requests)),
    }


def run_serving(args):
    """``--serving``: the serving workload alone, as its own JSON line."""
    leg = serving_leg(args, oracle_checks=not args.no_cpu_baseline)
    if not leg["bit_exact"]["all"]:
        log("MISMATCH in the serving run: %s" % leg["bit_exact"])
        sys.exit(1)
    out = {"metric": "serving: p50/p99 request latency and extensions/s under Poisson arrivals",
           "n_gpus": 1, "higher_is_better": True, "dtype": "int16 (exact, carried in binary16)",
           "data": "synthetic", "config": {"workload": leg.pop("workload"),
                                           "resident_residues": leg.pop("resident_residues"),
                                           "query_proteins": leg.pop("query_proteins")}}
    out.update(leg)
    print(json.dumps(out), flush=True)


def translated_oracle_checks(B, np, synth, params, w, dnas, res, h, plastx):
    """CPU-baseline leg of the translated runs (after the timed region): the
    oracle's six-frame translation of 4 sampled DNA sequences per bank and its
    hits on 24 sampled keys, against the GPU's."""
    from oracle import coracle as C
    from oracle import plast_oracle as O

    rng = np.random.default_rng(3)
    tr_equal = True
    frag_banks = []
    for d_bank, (c_t, s_t, f_t) in zip(dnas, res):
        fr = f_t.cpu().numpy()
        st_h = s_t.cpu().numpy()
        codes_h = c_t.cpu().numpy()
        for d in rng.choice(d_bank.n_seqs, size=min(4, d_bank.n_seqs), replace=False):
            frags, table = O.translate6(d_bank.seq(int(d)), np.array([0, int(d_bank.start[d + 1] - d_bank.start[d])]))
            sel = np.nonzero(fr[:, 0] == d)[0]
            got = [codes_h[st_h[j]:st_h[j + 1] - B.PAD_LEN] for j in sel]
            tr_equal &= len(got) == len(frags) and all(np.array_equal(a, b) for a, b in zip(got, frags))
            tr_equal &= bool(np.array_equal(fr[sel, 1:], table[:, 1:]))
        frag_banks.append(synth.Bank(codes_h, st_h))
    bank_a = frag_banks[0] if plastx else w.bank1
    bank_b = frag_banks[-1]
    i1, i2 = C.build_index(bank_a), C.build_index(bank_b)
    work = np.diff(i1[0]) * np.diff(i2[0])
    keys = np.sort(rng.choice(np.nonzero(work)[0], size=24, replace=False)).astype(np.int32)
    ref, _ = C.ungapped_hits(bank_a, bank_b, params.S1, keys=keys, idx1=i1, idx2=i2)
    hh = h.cpu().numpy().astype(np.int64)
    c1 = bank_a.codes
    q = bank_a.seq_start[hh[:, 0]] + hh[:, 1]
    hk = O.seed_key(c1[q].astype(np.int64), c1[q + 1].astype(np.int64), c1[q + 2].astype(np.int64),
                    c1[q + 3].astype(np.int64))
    hits_equal = bool(np.array_equal(O.canonical(hh[np.isin(hk, keys)]), ref))
    return {"translation_equals_oracle_on_sampled_dna": bool(tr_equal),
            "hits_equal_oracle_on_24_sampled_keys": hits_equal}


def run_translated(args, plastx=False):
    """TPLAST-N (configuration 3: 5000 proteins against 2000 DNA sequences of
    50-200 kb) or PLAST-X (200 against 1000 DNA sequences of 20-50 kb, both
    translated): the DNA banks are translated on the device in six frames every
    step; one step = translation + index of both banks + batched extension +
    gapped filter."""
    import numpy as np
    import torch

    from paper_0804_3643_amd import binding as B
    from paper_0804_3643_amd import params, synth

    B.load()
    dev = torch.device("cuda:0")
    if plastx:
        log("generating the PLAST-X workload")
        w = synth.make_plastx()
        dnas = [w.dna1, w.dna2]
    else:
        log("generating configuration 3")
        w = synth.make_tplastn()
        dnas = [w.dna]
    trs = [B.Translator(*B.dna_to_device(d, dev)) for d in dnas]
    outs = [t.run() for t in trs]
    if plastx:
        (ca, sa, fa), (cb, sb, fb) = outs
    else:
        ca, sa = B.bank_to_device(w.bank1, dev)
        cb, sb, fb = outs[0]
    ia = B.build_index(ca, sa)
    ib = B.build_index(cb, sb)
    tuning = None
    if not args.no_autotune:
        log("autotuning launch shapes")
        tuning, _ = B.autotune(ia, ib, params.S1, params.S2, reps=args.tune_reps)
    ext = B.Extender(ia, ib, params.S1, mode="batched", tuning=tuning)
    hits, n_ext = ext.run()
    cap = ext.hits.shape[0]
    gbuf = torch.empty(cap, dtype=torch.int32, device=dev)
    pbuf = torch.empty(cap, dtype=torch.uint8, device=dev)
    iba, wba = B.index_bytes(ca.numel(), sa.numel() - 1)
    ibb, wbb = B.index_bytes(cb.numel(), sb.numel() - 1)
    buf_a, buf_b, ws_idx = B._alloc(iba, dev), B._alloc(ibb, dev), B._alloc(max(wba, wbb), dev)

    def step():
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record()
        res = [t.run() for t in trs]
        if plastx:
            (xca, xsa, _), (xcb, xsb, _) = res
        else:
            xca, xsa = ca, sa
            xcb, xsb, _ = res[0]
        ev[1].record()
        xa = B.build_index(xca, xsa, workspace=ws_idx, out_buf=buf_a)
        xb = B.build_index(xcb, xsb, workspace=ws_idx, out_buf=buf_b)
        ev[2].record()
        h, ne = ext.run(xa, xb)
        ev[3].record()
        B.gapped_filter(xa, xb, h, params.S2, out=(gbuf, pbuf), tuning=tuning)
        ev[4].record()
        return h, ne, ev, res

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    t0 = time.perf_counter()
    stage = []
    for _ in range(args.steps):
        h, ne, ev, res = step()
        torch.cuda.synchronize()
        stage.append([ev[k].elapsed_time(ev[k + 1]) for k in range(4)])
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    stage = np.mean(np.array(stage), axis=0)
    n_hits = int(h.shape[0])
    n_pass = int(pbuf[:n_hits].sum().item())
    frag_tables = [f_t.cpu().numpy() for (_c, _s, f_t) in res]
    # the whole run against the oracle's full-size golden: the fragment banks
    # byte for byte, then every hit and gapped score
    log("whole run against the oracle's golden")
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import fullsize
    gkey = "x" if plastx else "3"
    golden = fullsize.load(gkey)
    frag_banks = [synth.Bank(c_t.cpu().numpy(), s_t.cpu().numpy()) for (c_t, s_t, _f) in res]
    if plastx:
        banks_sha = [fullsize.sha256_arrays(w.dna1.codes, w.dna1.start), fullsize.sha256_arrays(w.dna2.codes, w.dna2.start)]
    else:
        banks_sha = [w.bank1.sha256(), fullsize.sha256_arrays(w.dna.codes, w.dna.start)]
    if golden is None:
        gcheck = {"golden": None, "equal": False, "mismatch": ["no stored golden"]}
    elif golden["bank_sha256"] != banks_sha:
        gcheck = {"golden": os.path.basename(fullsize.golden_path(gkey)), "equal": False,
                  "mismatch": ["generated banks differ from the golden's"]}
    else:
        bad = []
        for fb, ft, ref in zip(frag_banks, frag_tables, golden["fragments"]):
            if (ft.shape[0] != ref["n"] or fullsize.sha256_arrays(fb.codes) != ref["codes_sha256"] or
                    fullsize.sha256_arrays(fb.seq_start.astype(np.int64)) != ref["seq_start_sha256"] or
                    fullsize.sha256_arrays(np.ascontiguousarray(ft, dtype=np.int32)) != ref["table_sha256"]):
                bad.append("fragment bank")
        got = fullsize.device_summary(h, gbuf[:n_hits], params.S2, frag_banks[0] if plastx else w.bank1, n_ext)
        bad += fullsize.compare(golden, got)
        gcheck = {"golden": os.path.basename(fullsize.golden_path(gkey)), "equal": not bad, "mismatch": bad,
                  "n_hits": got["n_hits"], "n_pass": got["n_pass"], "digest": got["hits_gscore"]}
    if not gcheck["equal"]:
        log("MISMATCH against the oracle's golden: %s" % gcheck["mismatch"])
        sys.exit(1)
    checks = None
    if not args.no_cpu_baseline:
        log("checks against the oracle")
        checks = translated_oracle_checks(B, np, synth, params, w, dnas, res, h, plastx)
        if not (checks["translation_equals_oracle_on_sampled_dna"] and checks["hits_equal_oracle_on_24_sampled_keys"]):
            log("MISMATCH against the oracle on the sampled DNA sequences or keys: %s" % checks)
            sys.exit(1)
    name = "PLAST-X" if plastx else "TPLAST-N"
    out = {
        "metric": "%s: ungapped extensions/s, whole step including the six-frame translation%s"
                  % (name, " of both banks" if plastx else ""),
        "value": n_ext / (ms * 1e-3), "unit": "ext/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "dtype": "int16 (exact, carried in binary16)",
        "data": "synthetic",
        "stages_device_ms": {"translate": stage[0], "index": stage[1], "ungapped": stage[2], "gapped": stage[3]},
        "bit_exact": {"oracle_golden_whole_run": gcheck},
        "n_ext": n_ext, "n_hits": n_hits, "n_gapped_pass": n_pass,
        "n_fragments": [int(f.shape[0]) for f in frag_tables],
        "tuning": tuning.as_dict() if tuning is not None else None,
        "cpu_baseline": {"kind": "oracle", "checks": checks} if checks is not None else None,
        "config": {"workload": w.description, "dna_nt": [int(d.codes.shape[0]) for d in dnas]},
    }
    print(json.dumps(out, default=float), flush=True)


def run_index_only(args):
    """``--index-only``: stage 0 alone on the banks of configuration 1, 2 or 3
    (for 3, the protein bank and the device translation of the DNA bank): each
    index built once to set up and ``--steps`` times timed with the library's
    HIP events, the CSR of the protein banks checked against the oracle's.
    One JSON line; a profiling aid, not a headline."""
    import numpy as np
    import torch

    from oracle import coracle as C
    from paper_0804_3643_amd import binding as B
    from paper_0804_3643_amd import synth

    B.load()
    dev = torch.device("cuda:0")
    banks = []
    if args.config == 3:
        w = synth.make_tplastn()
        codes, starts, _ = B.translate(*B.dna_to_device(w.dna, dev))
        banks = [("proteins", w.bank1, B.bank_to_device(w.bank1, dev)), ("fragments", None, (codes, starts))]
    else:
        w = synth.make_workload(args.config)
        banks = [("bank1", w.bank1, B.bank_to_device(w.bank1, dev)), ("bank2", w.bank2, B.bank_to_device(w.bank2, dev))]
    out = {"metric": "index build (stage 0) device time per bank", "unit": "ms", "config": args.config, "banks": {}}
    for name, host, (c, st) in banks:
        ib, wb = B.index_bytes(c.numel(), st.numel() - 1)
        buf, ws = B._alloc(ib, dev), B._alloc(wb, dev)
        ix = B.build_index(c, st, workspace=ws, out_buf=buf)
        B.timing_enable(True)
        ms = []
        for _ in range(args.steps):
            ix = B.build_index(c, st, workspace=ws, out_buf=buf)
            ms.append(B.timing_read()["index_ms"])
        B.timing_enable(False)
        rec = {"positions": int(c.numel()), "sequences": int(st.numel() - 1), "words": ix.n_words,
               "ms_min": float(np.min(ms)), "ms_median": float(np.median(ms))}
        if host is not None and not args.no_cpu_baseline:
            k, o, q = C.build_index(host)
            rec["csr_equals_oracle"] = bool(np.array_equal(ix.key_off().cpu().numpy(), k) and
                                            np.array_equal(ix.occ_seq().cpu().numpy().astype(np.int64), o))
            if not rec["csr_equals_oracle"]:
                log("MISMATCH: index of %s differs from the oracle's" % name)
                sys.exit(1)
        out["banks"][name] = rec
        log("%s: %d positions, %d words, %.3f ms" % (name, rec["positions"], rec["words"], rec["ms_min"]))
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2,
                    help="synthetic workload (2 = skewed 20,000 x 300,000 proteins, the default; 1 = 10,000 x "
                         "100,000; 3 = TPLAST-N, 5,000 proteins x 2,000 DNA sequences)")
    ap.add_argument("--plain-reps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-ext", type=float, default=1.5e9)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB device copy (counter scaling for rocprofv3 --pmc runs)")
    ap.add_argument("--no-autotune", action="store_true", help="use the built-in launch shapes")
    ap.add_argument("--tuning", default=None,
                    help="launch shapes as JSON (plast_tuning_t fields); skips the autotuner")
    ap.add_argument("--tune-reps", type=int, default=2)
    ap.add_argument("--serving", action="store_true",
                    help="serving workload instead: resident bank, Poisson query stream, p50/p99 latency")
    ap.add_argument("--serving-requests", type=int, default=1000)
    ap.add_argument("--serving-scale", type=float, default=1.0, help="resident bank size factor (1 = 1M proteins)")
    ap.add_argument("--serving-slots", type=int, default=3)
    ap.add_argument("--serving-leg-requests", type=int, default=200,
                    help="requests of the serving leg of the default run (1M resident proteins)")
    ap.add_argument("--no-serving-leg", dest="serving_leg", action="store_false",
                    help="skip the serving leg of the default run")
    ap.add_argument("--plastx", action="store_true",
                    help="PLAST-X: both banks nucleotide, translated on the device in six frames")
    ap.add_argument("--index-only", action="store_true",
                    help="only stage 0: time the index builds of the configuration's banks")
    ap.add_argument("--probes-only", action="store_true",
                    help="only the measured peaks (plast_probe_peak), e.g. under rocprofv3 counters")
    ap.add_argument("--no-stage32", dest="stage32", action="store_false",
                    help="skip stage 3.2 (full gapped alignment of the passing hits, reported apart from the step)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only (the hot path is single-GPU); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0804_3643_amd import binding as B
    from paper_0804_3643_amd import params, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.index_only:
        run_index_only(args)
        return
    if args.probes_only:
        B.load()
        print(json.dumps({"measured_peaks": measured_peaks(B, torch, dev), "machine": machine_info()}), flush=True)
        return
    if args.serving:
        run_serving(args)
        return
    if args.config == 3 or args.plastx:
        run_translated(args, plastx=args.plastx)
        return
    B.load()
    log("generating configuration %d" % args.config)
    w = synth.make_workload(args.config)
    spec = synth.CONFIGS[args.config]

    # ---- resident inputs and preallocated buffers
    ca, sa = B.bank_to_device(w.bank1, dev)
    cb, sb = B.bank_to_device(w.bank2, dev)
    iba, wba = B.index_bytes(ca.numel(), sa.numel() - 1)
    ibb, wbb = B.index_bytes(cb.numel(), sb.numel() - 1)
    buf_a = B._alloc(iba, dev)
    buf_b = B._alloc(ibb, dev)
    ws_idx = B._alloc(max(wba, wbb), dev)
    ia = B.build_index(ca, sa, workspace=ws_idx, out_buf=buf_a)
    ib = B.build_index(cb, sb, workspace=ws_idx, out_buf=buf_b)
    tuning, tune_report, tune_s = None, None, 0.0
    if args.tuning:
        tuning = B.Tuning.from_dict(json.loads(args.tuning))
    elif not args.no_autotune:
        log("autotuning launch shapes")
        t1 = time.perf_counter()
        tuning, tune_report = B.autotune(ia, ib, params.S1, params.S2, reps=args.tune_reps)
        tune_s = time.perf_counter() - t1
        log("tuned: %s (%.1f s)" % (tuning.as_dict(), tune_s))
    ext = B.Extender(ia, ib, params.S1, mode="batched", tuning=tuning)
    hits, n_ext = ext.run()
    cap = ext.hits.shape[0]
    gbuf = torch.empty(cap, dtype=torch.int32, device=dev)
    pbuf = torch.empty(cap, dtype=torch.uint8, device=dev)

    index_a_ms = []

    def step():
        xa = B.build_index(ca, sa, workspace=ws_idx, out_buf=buf_a)
        if B.timing_on():  # the build synchronised its stream: bank a's index time is final
            index_a_ms.append(B.timing_read()["index_ms"])
        xb = B.build_index(cb, sb, workspace=ws_idx, out_buf=buf_b)
        h, ne = ext.run(xa, xb)
        B.gapped_filter(xa, xb, h, params.S2, out=(gbuf, pbuf), tuning=tuning)
        return h, ne

    # ---- the step as one graph replay
    log("capturing the pipeline graph")
    pipe = B.Pipeline(ca, sa, cb, sb, params.S1, params.S2, ext.n_items, cap, tuning=tuning)
    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        pipe.launch()
    torch.cuda.synchronize()
    log("timing %d graph steps" % args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pipe.launch()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    res = pipe.result()
    assert res["status"] == B.OK, res

    # ---- the same step from the eager calls, with per-stage device times
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    B.timing_enable(True)
    stage_ms = {"index_ms": [], "plan_ms": [], "ungapped_ms": [], "gapped_ms": []}
    log("timing %d eager steps" % args.steps)
    t0 = time.perf_counter()
    index_a_ms.clear()
    for _ in range(args.steps):
        hits, n_ext = step()
        t = B.timing_read()  # waits for this step's last kernel
        t["index_ms"] += index_a_ms[-1]  # both banks' builds
        for k in stage_ms:
            stage_ms[k].append(t[k])
    torch.cuda.synchronize()
    eager_ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    n_hits = int(hits.shape[0])
    n_pass = int(pbuf[:n_hits].sum().item())
    batched_kernel_ms = float(np.mean(stage_ms["ungapped_ms"]))
    step_dev = np.sum([stage_ms[k] for k in ("index_ms", "plan_ms", "ungapped_ms", "gapped_ms")], axis=0)
    # graph replay == eager calls: same counts, same hit multiset, same gapped pass count
    gh, gg, gp = pipe.outputs(res["n_hits"])
    kg, sg = pair_keys_device(torch, gh)
    ke, se = pair_keys_device(torch, hits)
    graph_eq = bool(res["n_ext"] == n_ext and res["n_hits"] == n_hits and torch.equal(kg, ke) and
                    torch.equal(sg, se) and int(gp.sum().item()) == n_pass)
    assert graph_eq, "graph replay and eager calls differ"
    del kg, sg, ke, se
    # the whole run against the oracle's full-size golden, before any time is reported
    log("whole run against the oracle's golden")
    golden = golden_check(str(args.config), gh, gg, params.S2, res["n_ext"], w.bank1,
                          [w.bank1.sha256(), w.bank2.sha256()])
    if not golden["equal"]:
        log("MISMATCH against the oracle's golden: %s" % golden["mismatch"])
        sys.exit(1)
    del gh, gg, gp

    # ---- PLAIN vs BATCHED (ungapped stage only), same output required
    log("plain vs batched")
    if args.plain_reps < 1:
        B.timing_enable(False)
        out = {"metric": METRIC, "value": n_ext / (ms_per_step * 1e-3), "unit": "ext/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
               "eager_ms_per_step": eager_ms_per_step,
               "tuning": tuning.as_dict() if tuning is not None else None,
               "note": "profiling run (--plain-reps 0): plain schedule, wall times and baselines skipped",
               "stages_device_ms": {k: float(np.mean(v)) for k, v in stage_ms.items()}}
        if args.stage32:
            log("stage 3.2")
            out["stage32"] = run_stage32(B, torch, np, w, ia, ib, hits, gbuf[:n_hits], pbuf[:n_hits], 1, False)
        if args.copy_calibration:
            copy_calibration(torch, dev)
        print(json.dumps(out), flush=True)
        return
    ext_p = B.Extender(ia, ib, params.S1, mode="plain", capacity=cap)
    plain_ms, plain_wall = [], []
    for _ in range(args.plain_reps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        hp, ne_p = ext_p.run()
        plain_wall.append(time.perf_counter() - t1)
        tp = B.timing_read()
        plain_ms.append(tp["ungapped_ms"])
        plain_launches = tp["ungapped_launches"]
    batched_wall = []
    for _ in range(args.plain_reps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        hb, ne_b = ext.run()
        batched_wall.append(time.perf_counter() - t1)
    kp, sp = pair_keys_device(torch, hp)
    kb, sbat = pair_keys_device(torch, hb)
    plain_eq = bool(ne_p == ne_b == n_ext and torch.equal(kp, kb) and torch.equal(sp, sbat))
    assert plain_eq, "PLAIN and BATCHED hit lists differ"
    no_dups = bool((kb[1:] != kb[:-1]).all().item()) if kb.numel() > 1 else True
    assert no_dups, "a candidate pair is reported twice"
    del kp, sp, kb, sbat, hp
    B.timing_enable(False)

    # ---- bank-vs-bank wall time from host-resident banks to the host hit list
    def bank_vs_bank(mode):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        xa_c, xa_s = B.bank_to_device(w.bank1, dev)
        xb_c, xb_s = B.bank_to_device(w.bank2, dev)
        xa = B.build_index(xa_c, xa_s, workspace=ws_idx, out_buf=buf_a)
        xb = B.build_index(xb_c, xb_s, workspace=ws_idx, out_buf=buf_b)
        e = ext if mode == "batched" else ext_p
        h, _ = e.run(xa, xb)
        g, p = B.gapped_filter(xa, xb, h, params.S2, out=(gbuf, pbuf), tuning=tuning)
        host = (h.cpu(), g.cpu(), p.cpu())
        torch.cuda.synchronize()
        return time.perf_counter() - t1, host
    log("bank-vs-bank wall")
    wall_b, host_b = bank_vs_bank("batched")
    wall_p, _ = bank_vs_bank("plain")
    ext.run(ia, ib)  # restore views on the resident banks

    if args.copy_calibration:
        copy_calibration(torch, dev)

    # the wall-time runs above reused the hit and filter buffers: recompute both on the resident banks
    h_fin, _ = ext.run(ia, ib)
    g_fin, p_fin = B.gapped_filter(ia, ib, h_fin, params.S2, out=(gbuf, pbuf), tuning=tuning)
    recall = plant_recall(torch, np, w, h_fin, p_fin)
    keys_report = key_stats(torch, np, ia, ib)
    stage32 = None
    if args.stage32:
        log("stage 3.2 (full gapped alignment of the passing hits)")
        stage32 = run_stage32(B, torch, np, w, ia, ib, h_fin, g_fin, p_fin, 3, not args.no_cpu_baseline)
        log("stage 3.2: %d alignments in %.1f ms" % (stage32["alignments"], stage32["call_ms"]))
    log("measured peaks")
    peaks = measured_peaks(B, torch, dev)

    achieved = n_ext * OPS_PER_EXT / (batched_kernel_ms * 1e-3) / 1e12
    lds_achieved = n_ext * LDS_BYTES_PER_EXT / (batched_kernel_ms * 1e-3) / 1e12
    gapped_threads = (tuning if tuning is not None else B.tuning_default()).as_dict()["gapped_threads"]
    gapped_kernel_ms = float(np.mean(stage_ms["gapped_ms"]))
    h_host = host_b[0].numpy()
    cells = gapped_cells(np, w.bank1, w.bank2, h_host)
    gapped_achieved = cells * GAPPED_OPS_PER_CELL / (gapped_kernel_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": n_ext / (ms_per_step * 1e-3),
        "unit": "ext/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int16 (exact, carried in binary16)",
        "dtype_note": ("exact integer arithmetic: every score and partial sum is an integer of magnitude < 2048, "
                       "carried in packed binary16 registers where that is exact (BLOSUM62); an int16 ungapped path "
                       "and an int32 gapped path serve matrices outside that range"),
        "data": "synthetic",
        "config": {
            "workload": "PLAST-P configuration %d: %s; seeded lognormal lengths (mean 300, clamped 50-1000), "
                        "BLOSUM62 background residues; N=20, S1=%d, gapped window 64 band 16 open 11 extend 1 "
                        "S2=%d" % (args.config, spec.description, params.S1, params.S2),
            "bank1_proteins": w.bank1.n_seqs, "bank2_proteins": w.bank2.n_seqs,
            "bank1_residues": w.bank1.n_residues, "bank2_residues": w.bank2.n_residues,
            "step": "index both banks + batched ungapped extension + gapped filter, replayed as one HIP graph",
        },
        "eager_ms_per_step": eager_ms_per_step,
        "tuning": tuning.as_dict() if tuning is not None else None,
        "autotune": dict(tune_report, wall_s=tune_s) if tune_report is not None else None,
        "n_ext": n_ext, "n_hits": n_hits, "n_gapped_pass": n_pass,
        "stages_device_ms": {k: float(np.mean(v)) for k, v in stage_ms.items()},
        # per eager step: the sum of the four stages' device times (HIP events in the library)
        "step_device_ms": {"median": float(np.median(step_dev)), "min": float(np.min(step_dev)),
                           "max": float(np.max(step_dev)), "steps": len(step_dev)},
        "ungapped": {
            "batched_kernel_ms": batched_kernel_ms,
            "batched_ext_per_s": n_ext / (batched_kernel_ms * 1e-3),
            "plain_kernels_ms": float(np.mean(plain_ms)),
            "plain_ext_per_s": n_ext / (float(np.mean(plain_ms)) * 1e-3),
            "plain_launches": int(plain_launches),
            "batched_call_wall_ms": 1e3 * float(np.min(batched_wall)),
            "plain_call_wall_ms": 1e3 * float(np.min(plain_wall)),
            "batched_over_plain_speedup": float(np.mean(plain_ms)) / batched_kernel_ms,
        },
        "bank_vs_bank_wall_s": {"batched": wall_b, "plain": wall_p},
        "bit_exact": {"plain_equals_batched": plain_eq, "no_duplicate_pairs": no_dups,
                      "graph_equals_eager": graph_eq},
        "roofline": {
            "bound": "alu", "achieved": achieved, "peak": PEAK_INT16_TOPS, "unit": "TOP/s",
            "frac": achieved / PEAK_INT16_TOPS,
            "traffic": recorded_traffic(traffic_file("ungapped_persistent", args.config)),
            "kernel": "k_ungapped_persistent", "ops_per_ext": OPS_PER_EXT,
            "kernel_ms": batched_kernel_ms, "extensions_per_launch": n_ext,
            "measured_peak": peaks["valu_pk_f16"]["rate"] / 1e12,
            "frac_of_measured_peak": achieved / (peaks["valu_pk_f16"]["rate"] / 1e12),
            "note": "88 algorithmic operations per extension (44 additions, 44 maxima) against 2 packed "
                    "16-bit operations per lane per clock; the kernel's three-way maximum does two maxima "
                    "per half in one instruction, so this fraction can pass 1 by a little: the instruction "
                    "stream (about 41 lane instructions per extension, profiles/sq_counters_cfg1.md) uses "
                    "about 0.9 of the VALU issue slots",
            "with_lookups_as_alu_ops": {
                "ops_per_ext": OPS_PER_EXT_WITH_LOOKUPS,
                "achieved": achieved * OPS_PER_EXT_WITH_LOOKUPS / OPS_PER_EXT,
                "frac": achieved * OPS_PER_EXT_WITH_LOOKUPS / OPS_PER_EXT / PEAK_INT16_TOPS,
                "note": "counts the 44 substitution lookups per pair as ALU operations; the kernel serves them "
                        "from LDS (one ds_read_b64 gives 4 rows), so this fraction can exceed 1 and the VALU "
                        "(88 ops) and LDS (88 bytes) fractions are the binding ones"},
            "lds": {"bound": "lds", "achieved": lds_achieved, "peak": PEAK_LDS_TBS, "unit": "TB/s",
                    "frac": lds_achieved / PEAK_LDS_TBS, "bytes_per_ext": LDS_BYTES_PER_EXT,
                    "measured_peak": peaks["lds_b64"]["rate"] / 1e12,
                    "frac_of_measured_peak": lds_achieved / (peaks["lds_b64"]["rate"] / 1e12),
                    "note": "profile lookups: 44 scores of 2 bytes per pair, read 4 rows at a time with "
                            "ds_read_b64, against 256 B per CU per clock"},
            "gapped": {"bound": "alu", "kernel": "k_gapped_f16", "achieved": gapped_achieved,
                       "peak": PEAK_INT16_TOPS, "unit": "TOP/s", "frac": gapped_achieved / PEAK_INT16_TOPS,
                       "kernel_ms": gapped_kernel_ms, "dp_cells": cells, "ops_per_cell": GAPPED_OPS_PER_CELL,
                       "traffic": recorded_traffic(traffic_file("gapped", args.config),
                                                   os.path.join(ROOT, "paper_0804_3643_amd", "csrc", "gapped.hip"),
                                                   "traffic_bytes_per_launch_threads_%d" % gapped_threads)},
        },
        "cpu_baseline": None,
        "stage32": stage32,
        "plant_recall": recall,
        "key_stats": keys_report,
        "measured_peaks": peaks,
        "machine": machine_info(),
    }
    if stage32 is not None:
        r = stage32["roofline"]
        r["measured_peak"] = peaks["valu_i32"]["rate"] / 1e12
        r["frac_of_measured_peak"] = r["achieved"] / r["measured_peak"]
    out["bit_exact"]["oracle_golden_whole_run"] = golden
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a key sample)")
        hh = host_b[0].numpy().astype(np.int64)
        cb_ = cpu_baseline(w, hh, host_b[1].numpy().astype(np.int64), n_ext, args.cpu_sample_ext, params.S1,
                           params.S2)
        out["bit_exact"]["oracle_equals_gpu_on_sample_keys"] = cb_.pop("oracle_hits_equal_gpu_on_sample")
        out["bit_exact"]["oracle_gapped_equals_gpu_on_sample_keys"] = cb_.pop("oracle_gapped_equal_gpu_on_sample")
        out["cpu_baseline"] = cb_
        if not (out["bit_exact"]["oracle_equals_gpu_on_sample_keys"] and
                out["bit_exact"]["oracle_gapped_equals_gpu_on_sample_keys"]):
            log("MISMATCH against the oracle on the sampled keys")
            sys.exit(1)
    if stage32 is not None and "oracle_equals_gpu_on_sample_pairs" in stage32 and \
            not stage32["oracle_equals_gpu_on_sample_pairs"]:
        log("MISMATCH of stage 3.2 against the oracle on the sampled sequence pairs")
        sys.exit(1)
    if args.serving_leg:
        del host_b, h_fin, g_fin, p_fin, ext, ext_p, pipe
        torch.cuda.empty_cache()
        log("serving leg")
        out["serving"] = serving_leg(args, n_requests=args.serving_leg_requests,
                                     oracle_checks=not args.no_cpu_baseline)
        if not out["serving"]["bit_exact"]["all"]:
            log("MISMATCH in the serving leg: %s" % out["serving"]["bit_exact"])
            sys.exit(1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
