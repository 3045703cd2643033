"""Full-size skewed configuration 2 (20,000 x 300,000 proteins, 5% carrying
low-complexity repeats) on the GPU: index parity, the number of extensions,
the whole hit list and every gapped score of the graph replay against the
oracle's full-size golden (count and 64-bit multiset digests, whole run and per
block of 80 keys), PLAIN == BATCHED == other launch shapes == graph replay, and
the hits and gapped scores of sampled keys (the 32 heaviest, the 4 lightest,
256 random) against the oracle computed key by key."""
import os
import sys

import numpy as np
import pytest
import torch

from oracle import coracle as C
from oracle import plast_oracle as O
from paper_0804_3643_amd import params, synth

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import fullsize  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _say(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


def _pair_sorted(h):
    """Device-sorted 64-bit pair keys and scores: 11-bit positions, bank-2 ids < 2^19."""
    h = h.to(torch.int64)
    k = (((h[:, 0] << 11) | h[:, 1]) << 30) | (h[:, 2] << 11) | h[:, 3]
    k, o = torch.sort(k)
    return k, h[o, 4]


@pytest.mark.timeout(900)
def test_config2_full_size():
    from paper_0804_3643_amd import binding as B
    B.load()
    _say("cfg2 generate")
    w = synth.make_workload(2)
    assert w.bank1.lengths.max() < 2048 and w.bank2.lengths.max() < 2048 and w.bank2.n_seqs < (1 << 19)
    idx1, idx2 = C.build_index(w.bank1), C.build_index(w.bank2)
    n2 = np.diff(idx2[0])
    assert n2.max() > 1000 * n2[n2 > 0].min()           # buckets skewed over 3 orders of magnitude
    _say("cfg2 index")
    ca, sa = B.bank_to_device(w.bank1, "cuda")
    cb, sb = B.bank_to_device(w.bank2, "cuda")
    ia, ib = B.build_index(ca, sa), B.build_index(cb, sb)
    for ix, ref in ((ia, idx1), (ib, idx2)):
        assert np.array_equal(ix.key_off().cpu().numpy(), ref[0])
        st = ix.seq_start.cpu().numpy()
        occ_seq = ix.occ_seq().cpu().numpy().astype(np.int64)
        assert np.array_equal(occ_seq, ref[1])
        assert np.array_equal(ix.occ().cpu().numpy() - st[occ_seq], ref[2])
    _say("cfg2 batched")
    hb, n_ext = B.ungapped_extend(ia, ib, params.S1, mode="batched")
    assert n_ext == O.n_extensions(idx1, idx2)
    kb, sb_ = _pair_sorted(hb)
    assert bool((kb[1:] != kb[:-1]).all())               # no pair twice
    for t in ({"item_cols": [1024, 4096, 16384, 16384], "xcd_queues": 8}, None):
        mode = "plain" if t is None else "batched"
        _say("cfg2 %s %s" % (mode, t))
        h, ne = B.ungapped_extend(ia, ib, params.S1, mode=mode, tuning=t)
        k, s = _pair_sorted(h)
        assert ne == n_ext and torch.equal(k, kb) and torch.equal(s, sb_), (mode, t)
        del h, k, s
    _say("cfg2 graph replay")
    _, _, n_items = B.ungapped_workspace_bytes(ia, ib, "batched")
    pl = B.Pipeline(ca, sa, cb, sb, params.S1, params.S2, n_items, hb.shape[0] + 1024)
    pl.launch()
    r = pl.result()
    assert r["status"] == B.OK and r["n_ext"] == n_ext and r["n_hits"] == hb.shape[0], r
    gh, gg, gp = pl.outputs(r["n_hits"])
    k, s = _pair_sorted(gh)
    assert torch.equal(k, kb) and torch.equal(s, sb_)
    del k, s
    _say("cfg2 whole run against the oracle's full-size golden")
    golden = fullsize.load(2)
    assert golden is not None and golden["bank_sha256"] == [w.bank1.sha256(), w.bank2.sha256()]
    got = fullsize.device_summary(gh, gg, params.S2, w.bank1, r["n_ext"])
    assert fullsize.compare(golden, got) == [], fullsize.compare(golden, got)
    assert int(gp.sum().item()) == golden["n_pass"]
    # sampled keys against the oracle: 32 heaviest (6.5e9 extensions), 4 lightest, 256 random
    work = np.diff(idx1[0]) * n2
    nz = np.nonzero(work)[0]
    order = nz[np.argsort(work[nz])]
    rng = np.random.default_rng(2)
    keys = np.unique(np.concatenate([order[-32:], order[:4], rng.choice(nz, 256, replace=False)])).astype(np.int32)
    _say("cfg2 oracle on %d sampled keys (%.3g extensions)" % (len(keys), work[keys].sum()))
    ref, _ = C.ungapped_hits(w.bank1, w.bank2, params.S1, keys=keys, idx1=idx1, idx2=idx2)
    hh = gh.cpu().numpy().astype(np.int64)
    c = w.bank1.codes
    q = w.bank1.seq_start[hh[:, 0]] + hh[:, 1]
    hk = O.seed_key(c[q].astype(np.int64), c[q + 1].astype(np.int64), c[q + 2].astype(np.int64),
                    c[q + 3].astype(np.int64))
    sel = np.isin(hk, keys)
    assert np.array_equal(O.canonical(hh[sel]), ref)
    _say("cfg2 gapped scores of the sampled hits (%d)" % int(sel.sum()))
    g_ref = C.gapped_scores(w.bank1, w.bank2, hh[sel])
    assert np.array_equal(gg.cpu().numpy()[sel].astype(np.int64), g_ref)
    assert np.array_equal(gp.cpu().numpy()[sel].astype(bool), g_ref >= params.S2)
    pl.close()


@pytest.mark.timeout(900)
def test_config2_keys_heavy_in_both_banks():
    """Configuration 2 with 1% of each bank's sequences carrying a run over the
    same two letters (A, L), so that 16 seed keys hold 4,000-6,600 bank-1 and
    60,000-177,000 bank-2 occurrences at once: the load balance of the
    persistent schedule on keys heavy on both sides.  S1 is raised to 120 for
    this test only, so that the repeat-against-repeat pairs (nearly all above
    38) give about 3M hits.  PLAIN == BATCHED == other launch shapes exactly, the
    number of extensions equals the oracle's, and the hits of the 4 heaviest
    keys (2.3e9 extensions) and of 32 random keys equal the oracle's."""
    from paper_0804_3643_amd import binding as B
    B.load()
    s1 = 120
    _say("cfg2 shared-repeat variant generate")
    w = synth.shared_repeat_variant(synth.make_workload(2))
    idx1, idx2 = C.build_index(w.bank1), C.build_index(w.bank2)
    work = np.diff(idx1[0]) * np.diff(idx2[0])
    ia = B.build_index(*B.bank_to_device(w.bank1, "cuda"))
    ib = B.build_index(*B.bank_to_device(w.bank2, "cuda"))
    _say("cfg2 variant batched (tuned-like shape)")
    hb, n_ext = B.ungapped_extend(ia, ib, s1, mode="batched",
                                  tuning={"item_cols": [2048, 8192, 16384, 16384], "xcd_queues": 8})
    assert n_ext == int(work.sum())
    kb, sb_ = _pair_sorted(hb)
    assert bool((kb[1:] != kb[:-1]).all())
    for t in ({"item_cols": [1024, 4096, 4096, 4096], "xcd_queues": 1}, None):
        mode = "plain" if t is None else "batched"
        _say("cfg2 variant %s %s" % (mode, t))
        h, ne = B.ungapped_extend(ia, ib, s1, mode=mode, tuning=t)
        k, s = _pair_sorted(h)
        assert ne == n_ext and torch.equal(k, kb) and torch.equal(s, sb_), (mode, t)
        del h, k, s
    order = np.argsort(work)[::-1]
    heavy = order[:4]
    assert (np.diff(idx1[0])[heavy] > 4000).all() and (np.diff(idx2[0])[heavy] > 80000).all()
    rng = np.random.default_rng(5)
    keys = np.unique(np.concatenate([heavy, rng.choice(np.nonzero(work)[0], 32, replace=False)])).astype(np.int32)
    _say("cfg2 variant oracle on %d keys (%.3g extensions)" % (len(keys), work[keys].sum()))
    ref, _ = C.ungapped_hits(w.bank1, w.bank2, s1, keys=keys, idx1=idx1, idx2=idx2)
    hh = hb.cpu().numpy().astype(np.int64)
    c = w.bank1.codes
    q = w.bank1.seq_start[hh[:, 0]] + hh[:, 1]
    hk = O.seed_key(c[q].astype(np.int64), c[q + 1].astype(np.int64), c[q + 2].astype(np.int64),
                    c[q + 3].astype(np.int64))
    assert np.array_equal(O.canonical(hh[np.isin(hk, keys)]), ref)
