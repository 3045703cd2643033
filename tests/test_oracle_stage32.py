"""Pins of the stage 3.2 oracle (full gapped alignment and the list of pieces
of computed alignments, Sec. 3.3.4) against facts that do not come from it:
exhaustive path enumeration on tiny inputs, closed forms, a hand example, the
stage 3.1 oracle as a restriction, and identities of the output record."""
import numpy as np
import pytest

from oracle import coracle as C
from oracle import plast_oracle as O
from paper_0804_3643_amd import params, synth

M = O.BLOSUM62
AL = O.ALPHABET


def _enc(s):
    return np.array([AL.index(c) for c in s], dtype=np.int64)


def _all_paths(x, y, go, ge):
    """Every monotone path from (0, 0) (all prefixes included) with its score:
    substitutions minus (go + k*ge) per maximal run of k same-kind gap moves."""
    out = []
    stack = [(0, 0, 0, None, "")]
    while stack:
        i, j, s, last, path = stack.pop()
        out.append((i, j, s, path))
        for mv, di, dj in (("D", 1, 1), ("F", 1, 0), ("E", 0, 1)):
            ni, nj = i + di, j + dj
            if ni > len(x) or nj > len(y):
                continue
            ns = s + int(M[x[i], y[j]]) if mv == "D" else s - ge - (0 if last == mv else go)
            stack.append((ni, nj, ns, mv, path + mv))
    return out


def _rule_path(paths, end, top, go):
    """The trace-back rule applied to the enumerated paths.  Reading backward from
    the end cell among the optimal paths into it, each step takes the first move
    kind (in the order below) that one of them continues with: after a pair (or
    at the end cell) a pair, then y against a gap (E), then x against a gap (F);
    inside an E run, ending the run (a pair, then F) before extending it; inside
    an F run, a pair, then E, then extending.  With no opening cost every run may
    end at every cell, so inside a run the order after a pair applies."""
    cands = [p for i, j, s, p in paths if (i, j) == end and s == top]
    suffix = ""
    while suffix not in cands:
        live = [p for p in cands if p.endswith(suffix)]
        nxt = {p[-len(suffix) - 1] for p in live if len(p) > len(suffix)}
        order = "DFE" if suffix[:1] == "E" and go > 0 else "DEF"
        suffix = next(c for c in order if c in nxt) + suffix
    return suffix


def _path_record(x, y, path):
    """(end1, end2, length, identities, mismatches, gap openings) of a path read
    from the anchor at the starts of x and y."""
    i = j = ident = mism = opens = 0
    prev = None
    for m in path:
        if m == "D":
            ident += int(x[i] == y[j])
            mism += int(x[i] != y[j])
            i, j = i + 1, j + 1
        else:
            opens += int(m != prev)
            i, j = i + (m == "F"), j + (m == "E")
        prev = m
    return i, j, len(path), ident, mism, opens


def test_full_side_equals_exhaustive_enumeration():
    """The Python full side, and the C one through a one-hit alignment anchored at
    the starts of both sequences, against every path enumerated."""
    rng = np.random.default_rng(11)
    by_cost = {}
    # pairs where two optimal paths into the end cell differ in length and gap
    # openings, so that the rule's choice shows in the record (gaps 3 + 2 k)
    fixed = [("CAG", "WACG"), ("GGWC", "WGC"), ("AGCWG", "WCG")]
    for case in range(300 + len(fixed)):
        lx, ly = int(rng.integers(0, 6)), int(rng.integers(0, 6))
        x = rng.integers(0, 20 if case % 3 else 3, lx)
        y = rng.integers(0, 20 if case % 3 else 3, ly)
        if case % 5 == 4:  # W and P only: W/W 11, P/P 7, W/P -4, frequent ties between paths
            x, y = 18 * (x % 2) + 12 * (1 - x % 2), 18 * (y % 2) + 12 * (1 - y % 2)
        go, ge = [(11, 1), (1, 1), (0, 2), (3, 0)][case % 4]
        if case >= 300:
            x, y = _enc(fixed[case - 300][0]), _enc(fixed[case - 300][1])
            lx, ly, go, ge = len(x), len(y), 3, 2
        best, end, moves = O.full_side(x, y, go, ge)
        paths = _all_paths(x, y, go, ge)
        top = max(p[2] for p in paths)
        assert best == top, (x, y, go, ge)
        # end cell: first cell in row-major order reached by an optimal path
        first = min((i, j) for i, j, s, _ in paths if s == top)
        assert end == first
        # the traced path is the optimal path into the end cell that the rule picks
        rule = _rule_path(paths, end, top, go)
        assert "".join(moves) == rule, (x, y, go, ge)
        assert O.path_score(x, y, moves, go, ge) == best
        if lx and ly:
            by_cost.setdefault((go, ge), []).append((x, y, top, rule))
    F = {k: i for i, k in enumerate(O.ALIGN_FIELDS)}
    cols = [F[k] for k in ("end1", "end2", "length", "identities", "mismatches", "gap_opens")]
    for (go, ge), cases in by_cost.items():
        b1 = synth.Bank.from_flat(np.concatenate([c[0] for c in cases]), [len(c[0]) for c in cases])
        b2 = synth.Bank.from_flat(np.concatenate([c[1] for c in cases]), [len(c[1]) for c in cases])
        hits = np.array([(k, 0, k, 0, 0) for k in range(len(cases))], dtype=np.int64)
        rec, cover = C.full_alignments(b1, b2, hits, np.zeros(len(cases)), np.ones(len(cases), bool), go, ge)
        assert cover.tolist() == list(range(len(cases)))
        rec = rec[np.argsort(rec[:, F["hit"]])]
        for r, (x, y, top, rule) in zip(rec, cases):
            assert r[F["score"]] == top and tuple(r[cols]) == _path_record(x, y, rule), (x, y, go, ge)


def test_full_side_hand_example_one_gap():
    """Ten W against five W, G, five W: one gap of length 1 (cost 12) beats the
    W/G mismatch (-2) only because it keeps all ten W/W pairs (11 each)."""
    x = _enc("W" * 10)
    y = _enc("W" * 5 + "G" + "W" * 5)
    best, end, moves = O.full_side(x, y)
    assert best == 10 * 11 - 12 == 98
    assert end == (10, 11)
    assert "".join(moves) == "DDDDDEDDDDD"


def test_full_side_hand_example_gap_tie():
    """x = PPW, y = WPW with gaps of 1 per letter and no opening cost.  The first
    pair P/W scores -4, a gap on either side -1, so cell (1, 1) holds -2 both from
    the left (E: y's W against a gap, after x's P against one) and from above
    (F).  Then P/P (7) and W/W (11): best 16 at (3, 3), against 14 for the plain
    diagonal.  Tracing back, cell (1, 1) is in state H, not on the diagonal, and
    the rule takes E before F; read from the anchor the path is x's P against a
    gap, y's W against a gap, then the two pairs."""
    best, end, moves = O.full_side(_enc("PPW"), _enc("WPW"), 0, 1)
    assert best == -1 - 1 + 7 + 11 == 16 and end == (3, 3)
    assert "".join(moves) == "FEDD"


def test_full_side_closed_forms():
    for lx in range(0, 15):
        for ly in range(0, 15):
            best, end, moves = O.full_side(np.zeros(lx, np.int64), np.zeros(ly, np.int64))
            assert best == 4 * min(lx, ly)
            assert end == (min(lx, ly), min(lx, ly)) and set(moves) <= {"D"}
    rng = np.random.default_rng(3)
    for _ in range(20):
        a = rng.integers(0, 20, int(rng.integers(1, 60)))
        best, end, moves = O.full_side(a, a)
        assert best == int(M[a, a].sum()) and end == (len(a), len(a))


def test_full_side_is_the_unbanded_unwindowed_stage31_side():
    rng = np.random.default_rng(4)
    for _ in range(60):
        x = rng.integers(0, 20, int(rng.integers(0, 45)))
        y = rng.integers(0, 20, int(rng.integers(0, 45)))
        best, _, moves = O.full_side(x, y)
        assert best == O.gapped_side(x, y, band=len(x) + len(y) + 1)
        assert O.path_score(x, y, moves) == best
        assert best >= O.gapped_side(x, y, band=3)


@pytest.fixture(scope="module")
def cfg0_stage32():
    w = synth.make_workload(0)
    h, _ = C.ungapped_hits(w.bank1, w.bank2, params.S1)
    g = C.gapped_scores(w.bank1, w.bank2, h)
    return w, h, g, g >= params.S2


def _alignment_moves(a, p1, b, p2):
    _, _, mR = O.full_side(a[p1:], b[p2:])
    _, _, mL = O.full_side(a[:p1][::-1], b[:p2][::-1])
    return mR, mL


def test_stage32_records_are_consistent(cfg0_stage32):
    w, h, g, ps = cfg0_stage32
    rec, cover = C.full_alignments(w.bank1, w.bank2, h, g, ps)
    A, B = O.sequences(w.bank1), O.sequences(w.bank2)
    F = {k: i for i, k in enumerate(O.ALIGN_FIELDS)}
    assert (cover[~ps] == -1).all() and (cover[ps] >= 0).all()
    assert len(rec) == int((cover == np.arange(len(h))).sum())
    # every computed alignment scores at least the banded, windowed filter score
    assert (rec[:, F["score"]] >= g[rec[:, F["hit"]]]).all()
    pairs = rec[:, F["identities"]] + rec[:, F["mismatches"]]
    assert (rec[:, F["length"]] == (rec[:, F["end1"]] - rec[:, F["start1"]])
            + (rec[:, F["end2"]] - rec[:, F["start2"]]) - pairs).all()
    rng = np.random.default_rng(0)
    for r in rec[rng.choice(len(rec), size=min(40, len(rec)), replace=False)]:
        a, b = A[r[F["seq1"]]], B[r[F["seq2"]]]
        p1, p2 = int(r[F["seed1"]]), int(r[F["seed2"]])
        mR, mL = _alignment_moves(a, p1, b, p2)
        # rescore the alignment as printed: pairs, gap runs on each side
        sub = 0
        i, j = p1, p2
        for m in mR:
            if m == "D":
                sub += int(M[a[i], b[j]])
            i += m in "DF"
            j += m in "DE"
        i, j = p1 - 1, p2 - 1
        for m in mL:
            if m == "D":
                sub += int(M[a[i], b[j]])
            i -= m in "DF"
            j -= m in "DE"
        gaps = r[F["length"]] - (r[F["identities"]] + r[F["mismatches"]])
        assert sub - 11 * r[F["gap_opens"]] - 1 * gaps == r[F["score"]]


def test_stage32_cover_relation(cfg0_stage32):
    """A covered hit lies on a diagonal run of the alignment of its cover, which
    precedes it in the group order; a computed hit lies on no run of any
    alignment before it."""
    w, h, g, ps = cfg0_stage32
    rec, cover = C.full_alignments(w.bank1, w.bank2, h, g, ps)
    A, B = O.sequences(w.bank1), O.sequences(w.bank2)
    runs = {}

    def diag_runs(o):
        if o not in runs:
            s1, p1, s2, p2 = (int(v) for v in h[o, :4])
            a, b = A[s1], B[s2]
            mR, mL = _alignment_moves(a, p1, b, p2)
            cells = set()
            i, j = p1, p2
            for m in mR:
                if m == "D":
                    cells.add((i, j))
                i += m in "DF"
                j += m in "DE"
            i, j = p1 - 1, p2 - 1
            for m in mL:
                if m == "D":
                    cells.add((i, j))
                i -= m in "DF"
                j -= m in "DE"
            runs[o] = cells
        return runs[o]

    def order_key(k):
        return (-int(g[k]), int(h[k, 1]), int(h[k, 3]))

    idx = np.nonzero(ps)[0]
    rng = np.random.default_rng(1)
    for k in rng.choice(idx, size=min(150, len(idx)), replace=False):
        o = int(cover[k])
        assert h[o, 0] == h[k, 0] and h[o, 2] == h[k, 2]
        same = [m for m in idx if h[m, 0] == h[k, 0] and h[m, 2] == h[k, 2]]
        earlier = [m for m in same if order_key(m) < order_key(k) and cover[m] == m]
        on = [m for m in earlier if (int(h[k, 1]), int(h[k, 3])) in diag_runs(m)]
        if o == k:
            assert not on
        else:
            assert on and o == min(on, key=order_key)


def test_stage32_identical_pair_closed_form():
    """Two identical sequences: the best seed's alignment is the whole sequence
    with no gap (score = sum of the diagonal of BLOSUM62), and every same-
    diagonal hit is covered by it."""
    rng = np.random.default_rng(8)
    s = rng.integers(0, 20, 120)
    bank1 = synth.Bank.from_flat(s, [len(s)])
    bank2 = synth.Bank.from_flat(s, [len(s)])
    h, _ = C.ungapped_hits(bank1, bank2, params.S1)
    g = C.gapped_scores(bank1, bank2, h)
    ps = g >= params.S2
    rec, cover = O.full_alignments(bank1, bank2, h, g, ps)
    F = {k: i for i, k in enumerate(O.ALIGN_FIELDS)}
    main = ps & (h[:, 1] == h[:, 3])
    assert main.any()
    first = int(np.nonzero(main)[0][0])
    owner = cover[first]
    r = rec[rec[:, F["hit"]] == owner][0]
    assert r[F["score"]] == int(M[s, s].sum())
    assert (r[F["start1"]], r[F["end1"]], r[F["start2"]], r[F["end2"]]) == (0, 120, 0, 120)
    assert r[F["identities"]] == 120 and r[F["gap_opens"]] == 0
    assert (cover[main] == owner).all()
    rc, cc = C.full_alignments(bank1, bank2, h, g, ps)
    assert np.array_equal(rc, rec) and np.array_equal(cc, cover)


def test_stage32_numpy_and_c_oracles_agree(cfg0_stage32):
    w, h, g, ps = cfg0_stage32
    A, B = O.sequences(w.bank1), O.sequences(w.bank2)
    la = np.array([len(a) for a in A])
    lb = np.array([len(b) for b in B])
    keys = h[:, 0] * 10 ** 6 + h[:, 2]
    small = ps & (la[h[:, 0]] < 300) & (lb[h[:, 2]] < 300)
    mask = ps & np.isin(keys, np.unique(keys[small])[:30])
    rp, cp = O.full_alignments(w.bank1, w.bank2, h, g, mask)
    rc, cc = C.full_alignments(w.bank1, w.bank2, h, g, mask)
    assert len(rp) > 10
    assert np.array_equal(rp, rc) and np.array_equal(cp, cc)


def test_stage32_c_matches_python_on_tiny_random_pairs():
    """The C oracle against the pinned Python one on small random sequence pairs
    over four letters (W, A, G, C: many equal-score paths, so the trace-back
    rule decides the records), several hits per pair, all passing."""
    rng = np.random.default_rng(21)
    letters = [AL.index(c) for c in "WAGC"]
    n = 400
    seqs1 = [rng.choice(letters, int(rng.integers(1, 10))) for _ in range(n)]
    seqs2 = [rng.choice(letters, int(rng.integers(1, 10))) for _ in range(n)]
    bank1 = synth.Bank.from_flat(np.concatenate(seqs1), [len(s) for s in seqs1])
    bank2 = synth.Bank.from_flat(np.concatenate(seqs2), [len(s) for s in seqs2])
    hits = []
    for s in range(n):
        for _ in range(int(rng.integers(1, 4))):
            hits.append((s, int(rng.integers(0, len(seqs1[s]))), s, int(rng.integers(0, len(seqs2[s]))), 0))
    hits = np.array(hits, dtype=np.int64)
    g = rng.integers(0, 50, len(hits))
    ps = np.ones(len(hits), dtype=bool)
    for go, ge in ((11, 1), (3, 2), (1, 1)):
        rp, cp = O.full_alignments(bank1, bank2, hits, g, ps, go, ge)
        rc, cc = C.full_alignments(bank1, bank2, hits, g, ps, go, ge, nthreads=2)
        assert np.array_equal(rp, rc) and np.array_equal(cp, cc), (go, ge)
