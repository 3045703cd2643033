"""CPU checks of the benchmark's report helpers on configuration 0, fed with the
oracle's hits (the helpers take tensors on any device): recall of the planted
homologs by identity bin, the key-bucket statistics, and the machine record."""
import os
import sys

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from oracle import coracle as C  # noqa: E402
from paper_0804_3643_amd import params  # noqa: E402


class _Index:
    """Stands in for a device index: only key_off is read."""

    def __init__(self, key_off):
        self._k = torch.from_numpy(np.asarray(key_off, dtype=np.int64))

    def key_off(self):
        return self._k


@pytest.fixture(scope="module")
def cfg0_hits(cfg0):
    hits, _ = C.ungapped_hits(cfg0.bank1, cfg0.bank2, params.S1)
    g = C.gapped_scores(cfg0.bank1, cfg0.bank2, hits)
    return torch.from_numpy(hits.astype(np.int32)), torch.from_numpy((g >= params.S2).astype(np.uint8))


def test_plant_recall_counts_and_bins(cfg0, cfg0_hits):
    h, p = cfg0_hits
    r = bench.plant_recall(torch, np, cfg0, h, p)
    assert r["pairs"] == len(cfg0.plants) == 20
    assert sum(b["pairs"] for b in r["by_realised_identity"]) == r["pairs"]
    assert sum(b["with_hit"] for b in r["by_realised_identity"]) == r["with_hit"]
    assert r["passing_gapped"] <= r["with_hit"] <= r["pairs"]
    assert r["with_hit"] >= 19  # planted pairs at 40% identity share seeds
    # with no hit at all nothing is found
    none = bench.plant_recall(torch, np, cfg0, h[:0], p[:0])
    assert none["with_hit"] == 0 and none["passing_gapped"] == 0


def test_key_stats_match_the_index(cfg0):
    k1, k2 = C.build_index(cfg0.bank1)[0], C.build_index(cfg0.bank2)[0]
    ks = bench.key_stats(torch, np, _Index(k1), _Index(k2))
    n2 = np.diff(k2)
    assert ks["bank2_nonempty_keys"] == int((n2 > 0).sum())
    assert ks["bank2_max"] == int(n2.max()) and ks["bank2_min_nonempty"] == int(n2[n2 > 0].min())
    assert sum(ks["bank2_log2_histogram"].values()) == ks["bank2_nonempty_keys"]
    work = np.diff(k1).astype(np.float64) * n2
    assert abs(ks["top16_work_share"] - np.sort(work)[-16:].sum() / work.sum()) < 1e-12


def test_machine_info_runs_anywhere():
    m = bench.machine_info()
    assert m["host_logical_cpus"] >= 1
    assert "gpu_sclk_levels" in m


def test_published_peaks_cover_every_probe():
    from paper_0804_3643_amd import binding
    assert set(bench.PUBLISHED_PEAKS) == set(binding.PROBES)


def test_gapped_cells_equals_a_cell_by_cell_count(cfg0, cfg0_hits):
    """DP cells of the gapped filter (the roofline's work count) against a plain
    count of the in-band cells of both clipped windows of every hit."""
    h = cfg0_hits[0].numpy().astype(np.int64)[:300]
    la = np.diff(cfg0.bank1.seq_start) - 20
    lb = np.diff(cfg0.bank2.seq_start) - 20
    want = 0
    for s1, p1, s2, p2, _ in h:
        for lx, ly in ((min(64, la[s1] - p1), min(64, lb[s2] - p2)), (min(64, p1), min(64, p2))):
            want += sum(1 for i in range(lx + 1) for j in range(ly + 1) if abs(i - j) <= 16) - 1
    assert bench.gapped_cells(np, cfg0.bank1, cfg0.bank2, h) == want


def test_golden_check_accepts_the_oracle_and_rejects_a_slip(cfg0, cfg0_hits):
    h, _ = cfg0_hits
    g = torch.from_numpy(C.gapped_scores(cfg0.bank1, cfg0.bank2, h.numpy()).astype(np.int32))
    n_ext = int(sum(np.diff(C.build_index(cfg0.bank1)[0]) * np.diff(C.build_index(cfg0.bank2)[0])))
    sha = [cfg0.bank1.sha256(), cfg0.bank2.sha256()]
    p = torch.randperm(h.shape[0])
    ok = bench.golden_check("0", h[p], g[p], params.S2, n_ext, cfg0.bank1, sha)
    assert ok["equal"] and ok["mismatch"] == []
    g2 = g.clone()
    g2[5] += 1
    bad = bench.golden_check("0", h, g2, params.S2, n_ext, cfg0.bank1, sha)
    assert not bad["equal"] and "hits_gscore" in bad["mismatch"]
    assert not bench.golden_check("0", h, g, params.S2, n_ext + 1, cfg0.bank1, sha)["equal"]
    assert not bench.golden_check("0", h, g, params.S2, n_ext, cfg0.bank1, sha[::-1])["equal"]


def test_recorded_traffic_reads_the_figure_of_the_current_source(tmp_path):
    """A counter summary gives its figure only for the kernel source it was taken
    on, and the gapped filter's only for the workgroup size asked for."""
    src = tmp_path / "k.hip"
    src.write_text("kernel text\n")
    h = bench.kernel_source_hash(str(src))
    f = tmp_path / "t.md"
    f.write_text("# summary\n\nkernel_source_sha256_16: %s\ntraffic_bytes_per_launch: 1.5e+10\n"
                 "traffic_bytes_per_launch_threads_256: 2.5e+10\n" % h)
    assert bench.recorded_traffic(str(f), str(src)) == 1.5e10
    assert bench.recorded_traffic(str(f), str(src), "traffic_bytes_per_launch_threads_256") == 2.5e10
    assert bench.recorded_traffic(str(f), str(src), "traffic_bytes_per_launch_threads_512") is None
    src.write_text("kernel text, changed\n")
    assert bench.recorded_traffic(str(f), str(src)) is None
    # the committed summaries carry one figure per gapped workgroup size
    txt = open(bench.traffic_file("gapped", 2)).read()
    for nt in (128, 256, 512):
        assert "traffic_bytes_per_launch_threads_%d:" % nt in txt
