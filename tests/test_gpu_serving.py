"""GPU tests of the serving path: query banks searched against a resident
index with continuous batching.  Each request's matches (hits passing the
gapped filter, with both scores) equal the oracle's, and are identical alone
and in the mix, also when batches overflow and are split."""
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
def setup():
    from paper_0804_3643_amd import binding as B
    from paper_0804_3643_amd import serving as S
    B.load()
    # 10% of the serving resident bank: 100,000 proteins (about 30M residues)
    w = synth.make_serving(n_resident=1_000_000, n_requests=24, max_query=60, scale=0.1)
    res = S.Resident(w.resident.codes, w.resident.seq_start)
    return B, S, w, res


def _requests(S, w, arrivals):
    return [S.Request(i, b.codes, b.seq_start, arrival=float(t)) for i, (b, t) in enumerate(zip(w.requests, arrivals))]


def _oracle_matches(query, resident):
    hits, _ = C.ungapped_hits(query, resident, params.S1)
    g = C.gapped_scores(query, resident, hits)
    keep = g >= params.S2
    m = np.concatenate([hits[keep], g[keep, None]], axis=1)
    return m[np.lexsort(m.T[::-1])] if len(m) else m.reshape(0, 6)


def test_serving_matches_oracle_and_alone_equals_mix(setup):
    B, S, w, res = setup
    _say("serving mix of %d requests" % len(w.requests))
    rng = np.random.default_rng(3)
    # groups of four simultaneous arrivals, so that some batches hold several requests
    arrivals = np.repeat(np.sort(rng.uniform(0, 0.05, len(w.requests) // 4)), 4)
    reqs = _requests(S, w, arrivals)
    srv = S.Server(res, slots=2, max_seqs=150, max_padded=60_000, capacity=4_000_000)
    srv.run(reqs)
    assert all(r.done >= r.arrival for r in reqs) and srv.batches >= 1
    assert any(r.batch_size > 1 for r in reqs)          # requests were batched together
    st = S.latency_stats(reqs)
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    for i in (0, 5, 11):
        _say("oracle for request %d (%d proteins)" % (i, w.requests[i].n_seqs))
        assert np.array_equal(S.canonical(reqs[i].matches), _oracle_matches(w.requests[i], w.resident))
    planted = sum(len(h) for h in w.homologs)
    found = sum(len({(q, s) for q, s in h} & {(int(a), int(b)) for a, b in reqs[i].matches[:, [0, 2]]})
                for i, h in enumerate(w.homologs))
    assert planted > 0 and found >= 0.8 * planted       # planted homologs come back as matches
    _say("each request alone")
    for i in range(len(w.requests)):
        alone = _requests(S, w, [0.0] * len(w.requests))[i]
        srv.run([alone])
        assert alone.batch_size == 1
        assert np.array_equal(S.canonical(alone.matches), S.canonical(reqs[i].matches)), i


def test_serving_overflow_splits_batches(setup):
    B, S, w, res = setup
    _say("serving with a hit capacity that forces splits")
    reqs = _requests(S, w, [0.0] * len(w.requests))
    ref = _requests(S, w, [0.0] * len(w.requests))
    big = S.Server(res, slots=1, max_seqs=2000, max_padded=700_000, capacity=8_000_000)
    big.run(ref)
    assert big.batches == 1 and big.splits == 0          # all requests in one batch
    total = big.batch_hits[0]
    # capacity for half the batch's hits; admission that expects almost no hits
    small = S.Server(res, slots=2, max_seqs=2000, max_padded=700_000, capacity=total // 2 + 1, hit_rate=1e-9)
    small.run(reqs)
    assert small.splits > 0 and max(small.batch_hits) <= total // 2 + 1
    for a, b in zip(reqs, ref):
        assert np.array_equal(S.canonical(a.matches), S.canonical(b.matches))


def test_search_grouped_and_ungrouped_matches(setup):
    """plast_search_enqueue with and without segments: the same matches, and
    with segments each segment's matches lie in its own slice."""
    B, S, w, res = setup
    reqs = [S.Request(i, b.codes, b.seq_start) for i, b in enumerate(w.requests[:5])]
    codes, starts, first = S.merge(reqs)
    sr = B.Searcher(res.index, codes.shape[0], starts.shape[0] - 1, res.items_bound(codes.shape[0], None),
                    4_000_000, params.S1, params.S2)
    sr.codes[:codes.shape[0]].copy_(torch.from_numpy(codes))
    sr.starts[:starts.shape[0]].copy_(torch.from_numpy(starts))
    sr.enqueue(codes.shape[0], starts.shape[0] - 1)
    r0 = sr.result()
    flat = sr.matches[:r0["n_matches"]].cpu().numpy()
    seg = np.array(first + [starts.shape[0] - 1], dtype=np.int32)
    sr.seg_first[:seg.shape[0]].copy_(torch.from_numpy(seg))
    sr.enqueue(codes.shape[0], starts.shape[0] - 1, n_seg=len(first))
    r1 = sr.result()
    grouped = sr.matches[:r1["n_matches"]].cpu().numpy()
    off = sr.seg_off[:len(first) + 1].cpu().numpy()
    assert r0["status"] == r1["status"] == B.OK and r0["n_matches"] == r1["n_matches"] > 0
    assert off[0] == 0 and off[-1] == r1["n_matches"] and (np.diff(off) >= 0).all()
    assert np.array_equal(S.canonical(flat), S.canonical(grouped))
    for j in range(len(first)):
        part = grouped[off[j]:off[j + 1]]
        assert ((part[:, 0] >= seg[j]) & (part[:, 0] < seg[j + 1])).all()
