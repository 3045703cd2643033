"""GPU tests of the BATCHED schedule's launch shapes, the autotuner and the
graph-replayed pipeline: every shape, the tuned one and every graph replay give
exactly the oracle's hits and gapped scores."""
import sys

import numpy as np
import pytest
import torch

from oracle import coracle as C
from paper_0804_3643_amd import params, synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _say(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_0804_3643_amd import binding
    binding.load()
    return binding


def _index(B, bank):
    return B.build_index(*B.bank_to_device(bank, "cuda"))


def _skewed(seed=5, n1=60, n2=2500):
    rng = np.random.default_rng(seed)
    return synth.random_bank(rng, n1, 20, 120, 3), synth.random_bank(rng, n2, 20, 120, 3)


SHAPES = [
    {"item_cols": [1024, 1024, 1024, 1024]},
    {"item_cols": [16384, 16384, 16384, 16384], "xcd_queues": 8},
    {"class_min_n2": [1, 100, 1000, 5000], "item_cols": [512, 2048, 8192, 1536], "xcd_queues": 8},
    {"class_min_n2": [1, 2, 3, 4], "item_cols": [4096, 512, 16384, 3072], "xcd_queues": 1},
]


@pytest.mark.parametrize("shape", range(len(SHAPES)))
def test_batched_shapes_give_identical_hits(B, shape):
    """Item widths per size class and the queue count change the work list, not
    the hits: every shape returns the oracle's hit list."""
    t = SHAPES[shape]
    _say("batched shape %s" % t)
    b1, b2 = _skewed()
    ia, ib = _index(B, b1), _index(B, b2)
    ref, ref_ext = C.ungapped_hits(b1, b2, 30)
    hits, n_ext = B.ungapped_extend(ia, ib, 30, mode="batched", tuning=t)
    assert n_ext == ref_ext
    assert np.array_equal(B.canonical_hits(hits), ref)


def test_work_list_length_follows_the_shape(B):
    b1, b2 = _skewed()
    ia, ib = _index(B, b1), _index(B, b2)
    n1 = np.diff(ia.key_off().cpu().numpy())
    n2 = np.diff(ib.key_off().cpu().numpy())
    for t in SHAPES:
        tun = B.Tuning.from_dict(t)
        lo, cols = list(tun.class_min_n2), list(tun.item_cols)
        cls = np.searchsorted(np.asarray(lo), n2, side="right") - 1
        w = np.asarray(cols)[np.clip(cls, 0, 3)]
        live = (n1 > 0) & (n2 > 0)
        expect = int((((n1 + 31) // 32) * ((n2 + w - 1) // w))[live].sum())
        _, _, items = B.ungapped_workspace_bytes(ia, ib, "batched", tuning=tun)
        assert items == expect, t


@pytest.mark.parametrize("threads", [128, 256, 512])
def test_gapped_workgroup_sizes(B, cfg0, threads):
    _say("gapped threads %d" % threads)
    ia, ib = _index(B, cfg0.bank1), _index(B, cfg0.bank2)
    hits, _ = B.ungapped_extend(ia, ib, params.S1, mode="batched")
    gs, ps = B.gapped_filter(ia, ib, hits, params.S2, tuning={"gapped_threads": threads})
    ref = C.gapped_scores(cfg0.bank1, cfg0.bank2, hits.cpu().numpy().astype(np.int64))
    assert np.array_equal(gs.cpu().numpy().astype(np.int64), ref)
    assert np.array_equal(ps.cpu().numpy().astype(bool), ref >= params.S2)


def test_autotune_returns_a_valid_measured_tuning(B):
    _say("autotune skewed banks")
    b1, b2 = _skewed(7, 80, 3000)
    ia, ib = _index(B, b1), _index(B, b2)
    tun, rep = B.autotune(ia, ib, 30, params.S2, reps=2)
    d = tun.as_dict()
    assert d["class_min_n2"] == [1, 2048, 8192, 32768]
    assert all(c in B.TUNE_WIDTHS for c in d["item_cols"])
    assert d["xcd_queues"] in (1, 8) and d["gapped_threads"] in B.GAPPED_THREADS
    n2 = np.diff(ib.key_off().cpu().numpy())
    n1 = np.diff(ia.key_off().cpu().numpy())
    live = (n1 > 0) & (n2 > 0)
    for c in range(4):
        hi = d["class_min_n2"][c + 1] if c < 3 else 1 << 40
        sel = live & (n2 >= d["class_min_n2"][c]) & (n2 < hi)
        assert rep["class_ext"][c] == int((n1[sel] * n2[sel]).sum())
        if rep["class_ext"][c]:
            assert rep["class_ms"][c][0] > 0          # the smallest width always runs
            ran = [i for i, ms in enumerate(rep["class_ms"][c]) if ms > 0]
            best = min(ran, key=lambda i: rep["class_ms"][c][i])
            assert d["item_cols"][c] == B.TUNE_WIDTHS[best]
        else:
            assert d["item_cols"][c] == 4096
    assert min(rep["queue_ms"]) > 0 and min(rep["gapped_ms"]) > 0
    ref, _ = C.ungapped_hits(b1, b2, 30)
    hits, _ = B.ungapped_extend(ia, ib, 30, mode="batched", tuning=tun)
    assert np.array_equal(B.canonical_hits(hits), ref)


# --------------------------------------------------------------------------- graph pipeline

def _shuffle_residues(bank, seed):
    """Same layout (sequence lengths, separators), other residues."""
    rng = np.random.default_rng(seed)
    codes = bank.codes.copy()
    st = bank.seq_start
    for i in range(len(st) - 1):
        a, b = int(st[i]), int(st[i + 1]) - synth.PAD_LEN
        codes[a:b] = rng.permutation(codes[a:b])
    return synth.Bank(codes=codes, seq_start=st.copy())


def _pipeline(B, w, capacity=None, max_items=None, tuning=None):
    ca, sa = B.bank_to_device(w.bank1, "cuda")
    cb, sb = B.bank_to_device(w.bank2, "cuda")
    ia, ib = B.build_index(ca, sa), B.build_index(cb, sb)
    _, n_ext, n_items = B.ungapped_workspace_bytes(ia, ib, "batched", tuning=tuning)
    cap = capacity if capacity is not None else B.default_capacity(n_ext)
    mi = max_items if max_items is not None else 2 * n_items  # headroom for replays on other contents
    return B.Pipeline(ca, sa, cb, sb, params.S1, params.S2, mi, cap, tuning=tuning), (ca, sa, cb, sb)


def _check_replay(B, pl, bank1, bank2):
    r = pl.result()
    assert r["status"] == B.OK, r
    hits, gs, ps = pl.outputs(r["n_hits"])
    ref, ref_ext = C.ungapped_hits(bank1, bank2, params.S1)
    assert r["n_ext"] == ref_ext and r["n_hits"] == len(ref)
    assert np.array_equal(B.canonical_hits(hits), ref)
    h = hits.cpu().numpy().astype(np.int64)
    gref = C.gapped_scores(bank1, bank2, h)
    assert np.array_equal(gs.cpu().numpy().astype(np.int64), gref)
    assert np.array_equal(ps.cpu().numpy().astype(bool), gref >= params.S2)
    return r


def test_pipeline_replays_match_oracle_with_eager_work_between(B, cfg0):
    """The captured graph replayed several times, with the library's eager calls
    and torch work between replays, and with bank contents changed in place:
    every replay equals the oracle."""
    _say("pipeline replays cfg0")
    pl, (ca, sa, cb, sb) = _pipeline(B, cfg0, tuning={"xcd_queues": 8})
    for rep in range(3):
        pl.launch()
        r = _check_replay(B, pl, cfg0.bank1, cfg0.bank2)
        assert r["n_words_a"] == C.build_index(cfg0.bank1)[0][-1]
        # eager work between replays, on the same stream and buffers of its own
        ia, ib = B.build_index(ca, sa), B.build_index(cb, sb)
        eh, _ = B.ungapped_extend(ia, ib, params.S1, mode="batched")
        x = torch.arange(1 << 20, device="cuda", dtype=torch.float32).sum()
        assert eh.shape[0] == r["n_hits"] and float(x) > 0
    # new residues, same layout: the next replay reads the new contents
    other = _shuffle_residues(cfg0.bank1, 3)
    ca.copy_(torch.from_numpy(other.codes).to("cuda"))
    pl.launch()
    _check_replay(B, pl, other, cfg0.bank2)
    pl.close()


def test_pipeline_status_codes(B):
    _say("pipeline status codes")
    w = synth.make_workload(0, scale=0.3)
    # hit buffer too small: status CAPACITY, the first `capacity` hits scored
    pl, _ = _pipeline(B, w, capacity=5)
    pl.launch()
    r = pl.result()
    assert r["status"] == B.E_CAPACITY and r["n_hits"] > 5
    hits, gs, _ = pl.outputs(r["n_hits"])
    assert hits.shape[0] == 5
    assert np.array_equal(gs.cpu().numpy().astype(np.int64),
                          C.gapped_scores(w.bank1, w.bank2, hits.cpu().numpy().astype(np.int64)))
    pl.close()
    # work list longer than max_items: status WORKSPACE, no hits
    pl, _ = _pipeline(B, w, max_items=3)
    pl.launch()
    r = pl.result()
    assert r["status"] == B.E_WORKSPACE and r["n_hits"] == 0 and r["n_items"] > 3
    pl.close()
    # alphabet and layout errors in a bank: status set, no hits, later replays recover
    pl, (ca, sa, cb, sb) = _pipeline(B, w)
    good_codes, good_starts = ca.clone(), sa.clone()
    ca[int(w.bank1.seq_start[1]) + 3] = 25
    pl.launch()
    r = pl.result()
    assert r["status"] == B.E_ALPHABET and r["n_hits"] == 0
    ca.copy_(good_codes)
    sa[0] += 1                      # the first sequence must start after one separator run
    pl.launch()
    r = pl.result()
    assert r["status"] == B.E_LAYOUT and r["n_hits"] == 0
    sa.copy_(good_starts)
    pl.launch()
    _check_replay(B, pl, w.bank1, w.bank2)
    pl.close()
