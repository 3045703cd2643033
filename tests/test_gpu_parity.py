"""GPU parity: the HIP library, called through its C ABI, against the CPU oracle
on the same seeded inputs.  Integer work, so every comparison is exact."""
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


@pytest.fixture(scope="module")
def B():
    from paper_0804_3643_amd import binding
    binding.load()
    return binding


def _index(B, bank):
    return B.build_index(*B.bank_to_device(bank, "cuda"))


def _gpu_csr(ix):
    key_off = ix.key_off().cpu().numpy()
    occ = ix.occ().cpu().numpy().astype(np.int64)
    occ_seq = ix.occ_seq().cpu().numpy().astype(np.int64)
    st = ix.seq_start.cpu().numpy()
    return key_off, occ_seq, occ - st[occ_seq]


def _assert_index_equal(B, bank):
    ix = _index(B, bank)
    k, s, p = _gpu_csr(ix)
    rk, rs, rp = C.build_index(bank)
    assert ix.n_words == rk[-1]
    assert np.array_equal(k, rk)
    assert np.array_equal(s, rs)
    assert np.array_equal(p, rp)
    return ix


# --------------------------------------------------------------------------- index

def test_index_config0_matches_oracle(B, cfg0):
    _say("index cfg0 bank1/bank2")
    _assert_index_equal(B, cfg0.bank1)
    _assert_index_equal(B, cfg0.bank2)


def test_index_edge_cases(B):
    _say("index edge cases")
    rng = np.random.default_rng(21)
    cases = [
        synth.Bank.from_seqs([]),                                           # empty bank
        synth.Bank.from_seqs([np.zeros(0, np.uint8)] * 5),                  # only empty sequences
        synth.Bank.from_strings(["ACD", "", "W", "ACDE", "MKV"]),           # shorter than a seed
        synth.Bank.from_strings(["A" * 5000]),                              # one huge key
        synth.random_bank(rng, 300, 0, 90, 3),                              # skewed, ragged
        synth.random_bank(rng, 4000, 0, 12, 20),                            # many short sequences
        _boundary_bank(rng),                                                # starts on tile boundaries
    ]
    for bank in cases:
        _assert_index_equal(B, bank)


def _boundary_bank(rng):
    """Sequence starts exactly on, one before and one after the 2048-position
    tiles and 4096-position check chunks of the index build, a run of empty
    sequences across a tile boundary, and n_padded a multiple of 4096."""
    starts = [20, 2048, 4095, 6145, 8192] + [8192 + 20 * k for k in range(1, 12)] + [10239, 12289]
    end = 16384
    lens = [b - a - 20 for a, b in zip(starts, starts[1:] + [end])]
    assert min(lens) >= 0
    bank = synth.Bank.from_seqs([rng.integers(0, 20, n).astype(np.uint8) for n in lens])
    assert list(bank.seq_start[:-1]) == starts and int(bank.seq_start[-1]) == end
    return bank


def test_index_rejects_bad_input(B):
    _say("index error paths")
    bank = synth.Bank.from_strings(["ACDEFGHIK", "LMNPQ"])
    codes, st = B.bank_to_device(bank, "cuda")
    bad = codes.clone()
    bad[int(bank.seq_start[1]) + 2] = 25                    # residue code out of range
    with pytest.raises(B.PlastError) as e:
        B.build_index(bad, st)
    assert e.value.code == B.E_ALPHABET
    bad = codes.clone()
    bad[int(bank.seq_start[1]) - 3] = 4                     # separator overwritten
    with pytest.raises(B.PlastError) as e:
        B.build_index(bad, st)
    assert e.value.code == B.E_ALPHABET
    st_bad = st.clone()
    st_bad[1] = st_bad[0] + 3                               # runs overlap
    with pytest.raises(B.PlastError) as e:
        B.build_index(codes, st_bad)
    assert e.value.code == B.E_LAYOUT
    # the library still works after rejecting input
    _assert_index_equal(B, bank)


# --------------------------------------------------------------------------- ungapped

@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_ungapped_config0_matches_oracle(B, cfg0, mode):
    _say("ungapped cfg0 " + mode)
    ia, ib = _index(B, cfg0.bank1), _index(B, cfg0.bank2)
    hits, n_ext = B.ungapped_extend(ia, ib, params.S1, mode=mode)
    ref, ref_ext = C.ungapped_hits(cfg0.bank1, cfg0.bank2, params.S1)
    assert n_ext == ref_ext
    assert np.array_equal(B.canonical_hits(hits), ref)


def _skewed_banks(seed, n1=60, n2=2500, lo=20, hi=120, alpha=3):
    rng = np.random.default_rng(seed)
    return synth.random_bank(rng, n1, lo, hi, alpha), synth.random_bank(rng, n2, lo, hi, alpha)


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_ungapped_multi_tile_ragged(B, mode):
    """Keys with several 32-row tiles and several 2048-column chunks, ragged at
    both ends."""
    _say("ungapped skewed multi-tile " + mode)
    b1, b2 = _skewed_banks(5)
    ia, ib = _index(B, b1), _index(B, b2)
    n1 = np.diff(ia.key_off().cpu().numpy())
    n2 = np.diff(ib.key_off().cpu().numpy())
    assert n1.max() > 64 and n2.max() > 4096 and (n1 % 32 != 0).any()
    hits, n_ext = B.ungapped_extend(ia, ib, 30, mode=mode)
    ref, ref_ext = C.ungapped_hits(b1, b2, 30)
    assert n_ext == ref_ext
    assert np.array_equal(B.canonical_hits(hits), ref)


def test_ungapped_row_tile_sizes(B):
    """Keys with exactly 1, 4, 5, 8, 9, 12, 13, 16, 17, 31, 32, 33 and 64 bank-1
    occurrences (each bank-1 sequence is one 4-letter word), so that every
    size of row tile the kernel has (4, 8, 12, 16 and 32 rows) meets its full
    and its one-past-full row count; with s1 = 4 every candidate pair is a hit,
    so every row of every tile reports."""
    _say("ungapped row-tile sizes")
    rng = np.random.default_rng(17)
    counts = [1, 4, 5, 8, 9, 12, 13, 16, 17, 31, 32, 33, 64]
    words = []
    while len(words) < len(counts):  # words of pairwise different keys
        w = rng.integers(0, 20, 4)
        if all(O.seed_key(*w) != O.seed_key(*v) for v in words):
            words.append(w)
    seqs1 = [w for w, n in zip(words, counts) for _ in range(n)]
    seqs2 = [np.concatenate([rng.integers(0, 20, int(rng.integers(0, 30))), w, rng.integers(0, 20, int(rng.integers(0, 30)))])
             for w in words for _ in range(7)]
    b1 = synth.Bank.from_flat(np.concatenate(seqs1), [4] * len(seqs1))
    b2 = synth.Bank.from_flat(np.concatenate(seqs2), [len(x) for x in seqs2])
    ia, ib = _index(B, b1), _index(B, b2)
    n1 = np.diff(ia.key_off().cpu().numpy())
    assert sorted(n1[n1 > 0].tolist()) == counts
    ref, ref_ext = C.ungapped_hits(b1, b2, 4)
    assert len(ref) == ref_ext
    for mode in ("plain", "batched"):
        hits, n_ext = B.ungapped_extend(ia, ib, 4, mode=mode)
        assert n_ext == ref_ext
        assert np.array_equal(B.canonical_hits(hits), ref)


def test_ungapped_threshold_4_is_every_candidate_pair(B):
    """Score >= 4 always, so s1 = 4 must return every candidate pair exactly once:
    the work decomposition covers each (key, i, j) once."""
    _say("ungapped all pairs")
    w = synth.make_workload(0, plants=False, scale=0.5)
    ia, ib = _index(B, w.bank1), _index(B, w.bank2)
    for mode in ("plain", "batched"):
        hits, n_ext = B.ungapped_extend(ia, ib, 4, mode=mode)
        assert hits.shape[0] == n_ext
        ref, ref_ext = C.ungapped_hits(w.bank1, w.bank2, 4)
        assert n_ext == ref_ext == len(ref)
        assert np.array_equal(B.canonical_hits(hits), ref)


def test_ungapped_capacity_contract(B, cfg0):
    _say("ungapped capacity")
    ia, ib = _index(B, cfg0.bank1), _index(B, cfg0.bank2)
    ref, _ = C.ungapped_hits(cfg0.bank1, cfg0.bank2, params.S1)
    ext = B.Extender(ia, ib, params.S1, mode="batched", capacity=7)
    assert ext.hits.shape[0] == 7
    hits, _ = ext.run()          # retries after PLAST_E_CAPACITY
    assert hits.shape[0] == len(ref)
    assert np.array_equal(B.canonical_hits(hits), ref)
    hits0, _ = B.Extender(ia, ib, params.S1, mode="plain", capacity=0).run()
    assert np.array_equal(B.canonical_hits(hits0), ref)


@pytest.mark.parametrize("symmetric", [True, False])
def test_ungapped_custom_matrix(B, symmetric):
    """A caller-supplied matrix, also a non-symmetric one, so a transposed
    operand (bank-a letter vs bank-b letter) shows."""
    _say("ungapped custom matrix symmetric=%s" % symmetric)
    rng = np.random.default_rng(8)
    M = rng.integers(-6, 9, size=(20, 20))
    if symmetric:
        M = np.triu(M) + np.triu(M, 1).T
    np.fill_diagonal(M, rng.integers(-2, 12, 20))  # includes non-positive diagonal entries
    w = synth.make_workload(0, scale=0.3)
    ia, ib = _index(B, w.bank1), _index(B, w.bank2)
    for mode in ("plain", "batched"):
        hits, _ = B.ungapped_extend(ia, ib, 25, mode=mode, matrix=M)
        ref, _ = C.ungapped_hits(w.bank1, w.bank2, 25, matrix=M)
        assert np.array_equal(B.canonical_hits(hits), ref)


def test_ungapped_wide_matrix_uses_int16_path(B):
    """Entries beyond +-23 take the int16 scan (the f16 scan is exact only for
    small entries); scores reach the thousands."""
    _say("ungapped wide-range matrix")
    rng = np.random.default_rng(12)
    M = rng.integers(-120, 128, size=(20, 20))
    np.fill_diagonal(M, 127)
    w = synth.make_workload(0, scale=0.2)
    ia, ib = _index(B, w.bank1), _index(B, w.bank2)
    for mode in ("plain", "batched"):
        hits, _ = B.ungapped_extend(ia, ib, 600, mode=mode, matrix=M)
        ref, _ = C.ungapped_hits(w.bank1, w.bank2, 600, matrix=M)
        assert len(ref) > 100 and ref[:, 4].max() > 1024
        assert np.array_equal(B.canonical_hits(hits), ref)


def test_ungapped_f16_boundary_matrix(B):
    """Largest entries the f16 scan accepts (|M| = 23), thresholds at and beyond
    the score range."""
    _say("ungapped f16 boundary")
    rng = np.random.default_rng(13)
    M = rng.integers(-23, 24, size=(20, 20))
    np.fill_diagonal(M, 23)
    w = synth.make_workload(0, scale=0.2)
    ia, ib = _index(B, w.bank1), _index(B, w.bank2)
    for s1 in (150, 0, -5, 2000):
        hits, n_ext = B.ungapped_extend(ia, ib, s1, mode="batched", matrix=M)
        ref, _ = C.ungapped_hits(w.bank1, w.bank2, s1, matrix=M)
        assert np.array_equal(B.canonical_hits(hits), ref)
        if s1 <= 0:
            assert len(ref) == n_ext


def test_ungapped_empty_and_disjoint_banks(B):
    _say("ungapped empty banks")
    e = synth.Bank.from_seqs([])
    a = synth.Bank.from_strings(["ACDEFGHIKLMN"])
    b = synth.Bank.from_strings(["WWWWWWWW"])
    for x, y in ((e, a), (a, e), (a, b)):
        ix, iy = _index(B, x), _index(B, y)
        for mode in ("plain", "batched"):
            hits, n_ext = B.ungapped_extend(ix, iy, params.S1, mode=mode)
            assert hits.shape[0] == 0 and n_ext == 0


# --------------------------------------------------------------------------- gapped

# band 16 with moderate costs takes the packed-f16 kernel, the others the
# generic int32 kernel
@pytest.mark.parametrize("window,band,go,ge", [(64, 16, 11, 1), (32, 8, 5, 2), (17, 0, 11, 1), (64, 16, 0, 0),
                                               (40, 16, 5, 2), (7, 16, 11, 1), (64, 16, 900, 50), (1, 16, 3, 1)])
def test_gapped_matches_oracle(B, cfg0, window, band, go, ge):
    _say("gapped cfg0 w=%d band=%d open=%d ext=%d" % (window, band, go, ge))
    ia, ib = _index(B, cfg0.bank1), _index(B, cfg0.bank2)
    hits, _ = B.ungapped_extend(ia, ib, params.S1, mode="batched")
    gs, ps = B.gapped_filter(ia, ib, hits, params.S2, window=window, band=band, gap_open=go, gap_extend=ge)
    h = hits.cpu().numpy().astype(np.int64)
    ref = C.gapped_scores(cfg0.bank1, cfg0.bank2, h, window=window, band=band, gap_open=go, gap_extend=ge)
    assert np.array_equal(gs.cpu().numpy().astype(np.int64), ref)
    assert np.array_equal(ps.cpu().numpy().astype(bool), ref >= params.S2)


@pytest.mark.parametrize("wide", [False, True])
def test_gapped_custom_matrix(B, wide):
    _say("gapped custom matrix wide=%s" % wide)
    rng = np.random.default_rng(31)
    M = rng.integers(-60, 61, size=(20, 20)) if wide else rng.integers(-5, 9, size=(20, 20))
    w = synth.make_workload(0, scale=0.3)
    ia, ib = _index(B, w.bank1), _index(B, w.bank2)
    hits, _ = B.ungapped_extend(ia, ib, 30, mode="batched", matrix=M)
    assert hits.shape[0] > 100
    gs, ps = B.gapped_filter(ia, ib, hits, 40, matrix=M)
    ref = C.gapped_scores(w.bank1, w.bank2, hits.cpu().numpy(), matrix=M)
    assert np.array_equal(gs.cpu().numpy().astype(np.int64), ref)
    assert np.array_equal(ps.cpu().numpy().astype(bool), ref >= 40)


def _edge_matrix(rng, m):
    """Mismatch-heavy integer matrix: +m on the diagonal, off it mostly in
    [-m, -1] (10% in [1, m/2]) with -m present, so that |M| = m exactly and the
    DP cells of unrelated windows run deep into negative values."""
    M = rng.integers(-m, 0, size=(20, 20))
    pos = rng.random((20, 20)) < 0.1
    M[pos] = rng.integers(1, m // 2 + 1, size=int(pos.sum()))
    np.fill_diagonal(M, m)
    M[3, 7] = -m
    return M


# The packed-binary16 kernel is taken iff band == 16, window <= 64 and
# 64 |M| + 3 (open + extend) + 280 extend <= 2000: each pair below sits on the
# last admitted value (1998, 1999) and the first rejected one (2001, 2002).
@pytest.mark.parametrize("m,go,ge,bound", [(26, 17, 1, 1998), (26, 18, 1, 2001), (20, 51, 2, 1999),
                                           (20, 52, 2, 2002)])
def test_gapped_at_the_binary16_bound(B, m, go, ge, bound):
    assert 64 * m + 3 * (go + ge) + 280 * ge == bound
    _say("gapped at the f16 bound |M|=%d open=%d ext=%d (%d)" % (m, go, ge, bound))
    rng = np.random.default_rng(bound)
    M = _edge_matrix(rng, m)
    # gap-heavy pairs: bank 2 holds copies of bank-1 sequences with a letter
    # deleted every 5 (or inserted every 7) letters, and random sequences
    b1 = synth.random_bank(rng, 60, 150, 400)
    seqs2 = []
    for i in range(b1.n_seqs):
        s = b1.seq(i).copy()
        if i % 2:
            seqs2.append(np.delete(s, np.arange(4, len(s), 5)))
        else:
            seqs2.append(np.insert(s, np.arange(6, len(s), 7), rng.integers(0, 20, size=len(range(6, len(s), 7)))))
    seqs2 += [rng.integers(0, 20, size=int(n)).astype(np.uint8) for n in rng.integers(100, 400, size=60)]
    b2 = synth.Bank.from_seqs(seqs2)
    ia, ib = _index(B, b1), _index(B, b2)
    hits, _ = B.ungapped_extend(ia, ib, 3 * m, mode="batched", matrix=M)
    assert hits.shape[0] > 10000
    gs, ps = B.gapped_filter(ia, ib, hits, 200, gap_open=go, gap_extend=ge, matrix=M)
    h = hits.cpu().numpy().astype(np.int64)
    ref = C.gapped_scores(b1, b2, h, gap_open=go, gap_extend=ge, matrix=M)
    assert np.array_equal(gs.cpu().numpy().astype(np.int64), ref)
    assert np.array_equal(ps.cpu().numpy().astype(bool), ref >= 200)
    # alignments through the gaps of the edited copies score far above the seed
    assert (ref >= 200).sum() > 1000


def test_gapped_sequence_ends_and_bad_records(B):
    _say("gapped edges")
    rng = np.random.default_rng(4)
    b1 = synth.random_bank(rng, 30, 4, 80, 4)
    b2 = synth.random_bank(rng, 40, 4, 80, 4)
    ia, ib = _index(B, b1), _index(B, b2)
    hits, _ = B.ungapped_extend(ia, ib, 4, mode="batched")
    assert hits.shape[0] > 1000
    gs, _ = B.gapped_filter(ia, ib, hits, 0)
    ref = C.gapped_scores(b1, b2, hits.cpu().numpy())
    assert np.array_equal(gs.cpu().numpy().astype(np.int64), ref)
    bad = torch.tensor([[999, 0, 0, 0, 0], [0, -1, 0, 0, 0], [0, 0, 0, 10**6, 0], [-3, 0, 0, 0, 0]],
                       dtype=torch.int32, device="cuda")
    gs, ps = B.gapped_filter(ia, ib, bad, 0)
    assert (gs.cpu().numpy() == -1).all() and (ps.cpu().numpy() == 0).all()


# --------------------------------------------------------------------------- full size

def _pair_keys(h):
    h = np.asarray(h, dtype=np.int64)
    # 11-bit positions, bank-2 sequence ids below 2^19: 56 bits in all
    return (((h[:, 0] << 11) | h[:, 1]) << 30) | (h[:, 2] << 11) | h[:, 3]


def _sorted_by_pair(h):
    k = _pair_keys(h)
    o = np.argsort(k, kind="stable")
    return k[o], np.asarray(h[:, 4], dtype=np.int64)[o]


@pytest.mark.timeout(600)
def test_config1_full_size_plain_batched_and_sampled_keys(B):
    """Full-size configuration 1 (10,000 x 100,000 proteins), in the launch
    configuration the benchmark times: the whole hit list and every gapped
    score equal the oracle's full-size golden (count and 64-bit multiset
    digests, whole run and per block of 80 keys), PLAIN == BATCHED exactly, the
    number of extensions equals the oracle's, and the hits of sampled keys
    (heavy, light and random) equal the oracle's computed key by key."""
    _say("cfg1 generate")
    w = synth.make_workload(1)
    assert w.bank1.lengths.max() < 2048 and w.bank2.lengths.max() < 2048  # 11-bit positions in _pair_keys
    _say("cfg1 index")
    ia, ib = _index(B, w.bank1), _index(B, w.bank2)
    _say("cfg1 batched")
    hb, n_ext = B.ungapped_extend(ia, ib, params.S1, mode="batched")
    _say("cfg1 gapped filter, whole run against the oracle's full-size golden")
    gs, _ = B.gapped_filter(ia, ib, hb, params.S2)
    got = fullsize.device_summary(hb, gs, params.S2, w.bank1, n_ext)
    golden = fullsize.load(1)
    assert golden is not None and golden["bank_sha256"] == [w.bank1.sha256(), w.bank2.sha256()]
    assert fullsize.compare(golden, got) == [], fullsize.compare(golden, got)
    del gs
    hb = hb.cpu().numpy()
    _say("cfg1 plain")
    hp, n_ext_p = B.ungapped_extend(ia, ib, params.S1, mode="plain")
    hp = hp.cpu().numpy()
    _say("cfg1 compare")
    assert n_ext == n_ext_p
    kb, sb = _sorted_by_pair(hb)
    kp, sp = _sorted_by_pair(hp)
    assert np.array_equal(kb, kp) and np.array_equal(sb, sp)
    assert len(np.unique(kb)) == len(kb)          # no pair reported twice
    _say("cfg1 batched, other launch shapes")
    for t in ({"item_cols": [1024, 2048, 8192, 16384], "xcd_queues": 8}, {"item_cols": [16384] * 4}):
        ht, n_ext_t = B.ungapped_extend(ia, ib, params.S1, mode="batched", tuning=t)
        kt, st_ = _sorted_by_pair(ht.cpu().numpy())
        assert n_ext_t == n_ext and np.array_equal(kt, kb) and np.array_equal(st_, sb), t
        del ht
    idx1, idx2 = C.build_index(w.bank1), C.build_index(w.bank2)
    assert n_ext == O.n_extensions(idx1, idx2)
    # index parity at full size
    k1, s1_, p1_ = _gpu_csr(ia)
    assert np.array_equal(k1, idx1[0]) and np.array_equal(s1_, idx1[1]) and np.array_equal(p1_, idx1[2])
    # sampled keys: 8 heaviest by work, 8 lightest non-empty, 32 random
    work = np.diff(idx1[0]) * np.diff(idx2[0])
    nz = np.nonzero(work)[0]
    order = nz[np.argsort(work[nz])]
    rng = np.random.default_rng(1)
    keys = np.unique(np.concatenate([order[-8:], order[:8], rng.choice(nz, 32, replace=False)])).astype(np.int32)
    _say("cfg1 oracle on %d sampled keys" % len(keys))
    ref, _ = C.ungapped_hits(w.bank1, w.bank2, params.S1, keys=keys, idx1=idx1, idx2=idx2)
    starts = w.bank1.seq_start
    # key of each GPU hit from its bank-1 seed word
    c = w.bank1.codes
    q = starts[hb[:, 0]] + hb[:, 1]
    hk = O.seed_key(c[q].astype(np.int64), c[q + 1].astype(np.int64), c[q + 2].astype(np.int64),
                    c[q + 3].astype(np.int64))
    mine = hb[np.isin(hk, keys)]
    assert np.array_equal(O.canonical(mine), ref)
