"""CPU oracle for the PLAST-P bank-versus-bank hot path — TEST INFRASTRUCTURE.

This module is the plain, slow, obviously correct statement of what the GPU
library computes.  Only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import it; the product path never does, and it shares no code,
table or constant with the GPU library (it has its own BLOSUM62 transcription
and its own seed-class table).

Paper: Nguyen & Lavenier, "Fine-grained parallelization of similarity search
between protein sequences", INRIA RR-6513 (2008).

What is computed (paper section in brackets)
--------------------------------------------
* seed key (Sec. 3.3.1, subset-seed table and the AQAA/APAA/ASAA example):
  a 4-letter word maps to a class tuple with 20 x 2 x 11 x 20 = 8800 values;
* index (Sec. 3.3.1, look-up table plus occurrence lists): every position of
  every sequence that starts a full 4-letter word, grouped by key, in ascending
  (sequence, position) order inside a key;
* candidate pairs (Sec. 3.2 generic algorithm, Sec. 3.3.3): every pair of an
  occurrence in bank1 and an occurrence in bank2 with the same key, one-hit;
* ungapped score (Sec. 3.3.3 and the GPU kernel of Annex 4): a rightward scan
  from the first seed letter over at most W + N = 24 letters, then a leftward
  scan over at most N = 20 letters; each side keeps the best prefix sum (the
  empty prefix, 0, included) and the pair scores the sum of both bests.
  Scans stop at sequence ends.  Kept iff score >= S1;
* small gapped filter (Sec. 3.3.4 stage 3.1; Sec. 5.2.2 one-sided extensions on
  either side of the seed): an anchored, banded affine-gap alignment rightward
  from the seed start and another leftward from the letters just before it,
  each over at most G letters per sequence, cells restricted to |i - j| <= band;
  gapped score = best right + best left, pass iff >= S2;
* full gapped alignment (Sec. 3.3.4 stage 3.2 and its list of the ungapped
  pieces of computed alignments): for the hits that pass S2, the same anchored
  affine-gap recurrences with no band and no window, traced back; a hit lying
  on a piece of an alignment already computed for its sequence pair is
  covered and computes nothing.

Readings taken where the paper is silent or garbled: the seed table's rows 1
and 4 list every letter (I is missing in the text), row 3's class f is
{F,Y,W}, N = 20, hits are score >= S1, no X-drop, gapped window G = 64, band
16, a gap of length k costs 11 + k.  Stage 3.2 (the paper asks only for a
standard dynamic-programming alignment): no X-drop, the survivors of one sequence pair
in order of decreasing gapped score then seed position, end cell and path
chosen by the fixed preferences given in :func:`full_side`.
* six-frame translation (Sec. 6, TPLAST-N; the paper gives no details): the
  standard genetic code; frames 0..2 start at nucleotides 0..2 of the forward
  strand, frames 3..5 at nucleotides 0..2 of the reverse complement; a
  trailing partial codon is dropped; stop codons split a frame into fragments,
  each fragment (non-empty) a protein sequence of its own.
"""
from __future__ import annotations

import numpy as np

ALPHABET = "ACDEFGHIKLMNPQRSTVWY"
NKEYS = 20 * 2 * 11 * 20
W = 4           # seed length
NBR = 20        # neighbourhood letters beyond each end of the seed
RIGHT = W + NBR  # letters scanned rightward, seed included

# BLOSUM62, lower triangle in ALPHABET order (A C D E F G H I K L M N P Q R S T V W Y).
_B62_LOWER = """
A  4
C  0  9
D -2 -3  6
E -1 -4  2  5
F -2 -2 -3 -3  6
G  0 -3 -1 -2 -3  6
H -2 -3 -1  0 -1 -2  8
I -1 -1 -3 -3  0 -4 -3  4
K -1 -3 -1  1 -3 -2 -1 -3  5
L -1 -1 -4 -3  0 -4 -3  2 -2  4
M -1 -1 -3 -2  0 -3 -2  1 -1  2  5
N -2 -3  1  0 -3  0  1 -3  0 -3 -2  6
P -1 -3 -1 -1 -4 -2 -2 -3 -1 -3 -2 -2  7
Q -1 -3  0  2 -3 -2  0 -3  1 -2  0  0 -1  5
R -1 -3 -2  0 -3 -2  0 -3  2 -2 -1  0 -2  1  5
S  1 -1  0  0 -2  0 -1 -2  0 -2 -1  1 -1  0 -1  4
T  0 -1 -1 -1 -2 -2 -2 -1 -1 -1 -1  0 -1 -1 -1  1  5
V  0 -1 -3 -2 -1 -3 -3  3 -2  1  1 -3 -2 -2 -3 -2  0  4
W -3 -2 -4 -3  1 -2 -2 -3 -3 -2 -1 -4 -4 -2 -3 -3 -2 -3 11
Y -2 -2 -3 -2  3 -3  2 -1 -2 -1 -1 -2 -3 -1 -2 -2 -2 -1  2  7
"""


def _blosum62() -> np.ndarray:
    m = np.zeros((20, 20), dtype=np.int64)
    for i, line in enumerate(_B62_LOWER.strip().splitlines()):
        parts = line.split()
        assert parts[0] == ALPHABET[i]
        for j, v in enumerate(parts[1:]):
            m[i, j] = m[j, i] = int(v)
    return m


BLOSUM62 = _blosum62()

# Subset seed (Sec. 3.3.1).  Positions 1 and 4: every amino acid is its own
# class.  Position 2: two classes.  Position 3: eleven classes, in the order the
# paper lists them.
SEED_POS2 = ["CFYWMLIV", "GPATSNHQEDRK"]
SEED_POS3 = ["A", "C", "FYW", "G", "IV", "ML", "NH", "P", "QED", "RK", "TS"]


def _class_of(classes):
    out = np.full(20, -1, dtype=np.int64)
    for k, letters in enumerate(classes):
        for c in letters:
            out[ALPHABET.index(c)] = k
    assert (out >= 0).all()
    return out


CLASS2 = _class_of(SEED_POS2)
CLASS3 = _class_of(SEED_POS3)


def seed_key(w0, w1, w2, w3):
    """kappa(w) = ((id(w0)*2 + c2(w1))*11 + c3(w2))*20 + id(w3)  (Sec. 3.3.1)."""
    return ((np.asarray(w0, np.int64) * 2 + CLASS2[w1]) * 11 + CLASS3[w2]) * 20 + np.asarray(w3, np.int64)


def sequences(bank):
    """Residue arrays of a bank: either an object with ``codes``/``seq_start`` in
    the padded storage layout (a pad run of 20 codes after every sequence; pads
    are never read here) or a list of code arrays."""
    if hasattr(bank, "codes"):
        codes, seq_start = bank.codes, bank.seq_start
        return [np.asarray(codes[seq_start[i]:seq_start[i + 1] - 20], dtype=np.int64)
                for i in range(len(seq_start) - 1)]
    return [np.asarray(s, dtype=np.int64) for s in bank]


# --------------------------------------------------------------------------- index

def build_index(bank):
    """Stage 0 (Sec. 3.3.1): key -> occurrences, as CSR.

    Returns ``key_off`` int64[8801], ``occ_seq`` int32[n], ``occ_pos`` int32[n];
    the occurrences of key k are entries ``key_off[k]:key_off[k+1]``, ascending
    by (sequence, position).
    """
    seqs = sequences(bank)
    keys, sid, pos = [], [], []
    for s, a in enumerate(seqs):
        n = len(a) - W + 1
        if n <= 0:
            continue
        keys.append(seed_key(a[0:n], a[1:n + 1], a[2:n + 2], a[3:n + 3]))
        sid.append(np.full(n, s, dtype=np.int64))
        pos.append(np.arange(n, dtype=np.int64))
    if keys:
        keys, sid, pos = np.concatenate(keys), np.concatenate(sid), np.concatenate(pos)
    else:
        keys = sid = pos = np.zeros(0, dtype=np.int64)
    order = np.argsort(keys, kind="stable")   # input is already (seq, pos) ascending
    counts = np.bincount(keys, minlength=NKEYS)
    key_off = np.zeros(NKEYS + 1, dtype=np.int64)
    key_off[1:] = np.cumsum(counts)
    return key_off, sid[order].astype(np.int32), pos[order].astype(np.int32)


def n_extensions(idx1, idx2) -> int:
    """Number of candidate pairs, sum over keys of n1(k) * n2(k)."""
    return int((np.diff(idx1[0]) * np.diff(idx2[0])).sum())


# --------------------------------------------------------------- ungapped score

def ungapped_score(a, p1, b, p2, matrix=BLOSUM62, nbr=NBR, right=RIGHT) -> int:
    """Score of one candidate pair, written as the definition (scalar loops).

    Rmax = max over 0 <= r <= rmax of sum_{t<r} M[a[p1+t], b[p2+t]],
           rmax = min(right, |a| - p1, |b| - p2);
    Lmax = max over 0 <= l <= lmax of sum_{t=1..l} M[a[p1-t], b[p2-t]],
           lmax = min(nbr, p1, p2);
    score = Rmax + Lmax.
    """
    rmax = min(right, len(a) - p1, len(b) - p2)
    s = best_r = 0
    for t in range(rmax):
        s += int(matrix[a[p1 + t], b[p2 + t]])
        best_r = max(best_r, s)
    lmax = min(nbr, p1, p2)
    s = best_l = 0
    for t in range(1, lmax + 1):
        s += int(matrix[a[p1 - t], b[p2 - t]])
        best_l = max(best_l, s)
    return best_r + best_l


def ungapped_hits(bank1, bank2, s1, matrix=BLOSUM62, keys=None, idx1=None, idx2=None,
                  nbr=NBR, right=RIGHT, return_all=False):
    """Stage 2 over whole banks (Sec. 3.2, generic algorithm: all pairs of the
    two neighbourhood blocks of a key): every candidate pair of every key (or of
    the listed ``keys``) is scored with the definition of
    :func:`ungapped_score`, vectorised over the pairs of one key.

    Returns int64[n, 5] rows (seq1, pos1, seq2, pos2, score) with score >= s1,
    sorted lexicographically.  ``return_all`` keeps every candidate pair.
    """
    A, B = sequences(bank1), sequences(bank2)
    idx1 = idx1 if idx1 is not None else build_index(A)
    idx2 = idx2 if idx2 is not None else build_index(B)
    lenA = np.array([len(a) for a in A], dtype=np.int64)
    lenB = np.array([len(b) for b in B], dtype=np.int64)
    catA = _concat(A)
    catB = _concat(B)
    startA = np.concatenate([[0], np.cumsum(lenA)])[:-1] if len(A) else np.zeros(0, np.int64)
    startB = np.concatenate([[0], np.cumsum(lenB)])[:-1] if len(B) else np.zeros(0, np.int64)
    mat = np.asarray(matrix, dtype=np.int64)
    out = []
    key_list = range(NKEYS) if keys is None else keys
    for k in key_list:
        o1 = slice(idx1[0][k], idx1[0][k + 1])
        o2 = slice(idx2[0][k], idx2[0][k + 1])
        s_1, p_1 = idx1[1][o1].astype(np.int64), idx1[2][o1].astype(np.int64)
        s_2, p_2 = idx2[1][o2].astype(np.int64), idx2[2][o2].astype(np.int64)
        if len(s_1) == 0 or len(s_2) == 0:
            continue
        step = max(1, 4_000_000 // (len(s_2) * right))
        for c0 in range(0, len(s_1), step):
            c = slice(c0, c0 + step)
            sc = _key_scores(catA, startA[s_1[c]], lenA[s_1[c]], p_1[c],
                             catB, startB[s_2], lenB[s_2], p_2, mat, nbr, right)
            keep = np.ones_like(sc, dtype=bool) if return_all else sc >= s1
            ii, jj = np.nonzero(keep)
            if len(ii):
                out.append(np.stack([s_1[c][ii], p_1[c][ii], s_2[jj], p_2[jj], sc[ii, jj]], axis=1))
    res = np.concatenate(out) if out else np.zeros((0, 5), dtype=np.int64)
    return canonical(res)


def _concat(seqs):
    return np.concatenate(seqs).astype(np.int64) if seqs else np.zeros(0, np.int64)


def _key_scores(catA, stA, lnA, pA, catB, stB, lnB, pB, mat, nbr, right):
    """Score matrix [n1, n2] for one key (definition vectorised over pairs)."""
    NEG = np.int64(-(1 << 40))
    # right side: t = 0 .. right-1, letter index p + t; allowed while t < rmax
    t = np.arange(right)
    remA = lnA - pA                      # letters available from the anchor on
    remB = lnB - pB
    ia = np.minimum(pA[:, None] + t, np.maximum(lnA[:, None] - 1, 0))
    ib = np.minimum(pB[:, None] + t, np.maximum(lnB[:, None] - 1, 0))
    la = catA[stA[:, None] + ia]
    lb = catB[stB[:, None] + ib]
    sc = mat[la[:, None, :], lb[None, :, :]]            # [n1, n2, right]
    cs = np.cumsum(sc, axis=2)
    rmax = np.minimum(np.minimum(remA[:, None], remB[None, :]), right)
    cs = np.where(t[None, None, :] < rmax[:, :, None], cs, NEG)
    best_r = np.maximum(cs.max(axis=2), 0)
    # left side: t = 1 .. nbr, letter index p - t; allowed while t <= lmax
    t = np.arange(1, nbr + 1)
    ia = np.maximum(pA[:, None] - t, 0)
    ib = np.maximum(pB[:, None] - t, 0)
    la = catA[stA[:, None] + ia] if len(catA) else np.zeros((len(pA), nbr), np.int64)
    lb = catB[stB[:, None] + ib]
    sc = mat[la[:, None, :], lb[None, :, :]]
    cs = np.cumsum(sc, axis=2)
    lmax = np.minimum(np.minimum(pA[:, None], pB[None, :]), nbr)
    cs = np.where(t[None, None, :] <= lmax[:, :, None], cs, NEG)
    best_l = np.maximum(cs.max(axis=2), 0)
    return best_r + best_l


def canonical(hits):
    """Sort hit rows lexicographically by (seq1, pos1, seq2, pos2, score)."""
    hits = np.asarray(hits, dtype=np.int64).reshape(-1, 5)
    if len(hits) == 0:
        return hits
    order = np.lexsort(hits.T[::-1])
    return hits[order]


# ------------------------------------------------------------ small gapped filter

GAP_WINDOW = 64
GAP_BAND = 16
GAP_OPEN = 11
GAP_EXTEND = 1


def gapped_side(x, y, band=GAP_BAND, gap_open=GAP_OPEN, gap_extend=GAP_EXTEND, matrix=BLOSUM62):
    """Best anchored banded affine-gap alignment score of prefixes of x and y.

    Scalar Gotoh recurrences written out; cell (i, j) (i letters of x, j of y)
    exists iff |i - j| <= band.  A gap of length k costs gap_open + k*gap_extend.
    best = max(0, max over existing cells of H(i, j)).  ``gap_open=None`` means
    gaps are forbidden.
    """
    lx, ly = len(x), len(y)
    NEG = -(1 << 40)
    oe = None if gap_open is None else gap_open + gap_extend
    H = [[NEG] * (ly + 1) for _ in range(lx + 1)]
    E = [[NEG] * (ly + 1) for _ in range(lx + 1)]
    F = [[NEG] * (ly + 1) for _ in range(lx + 1)]
    H[0][0] = 0
    best = 0
    for i in range(lx + 1):
        for j in range(ly + 1):
            if abs(i - j) > band or (i == 0 and j == 0):
                continue
            if oe is not None:
                if j >= 1 and abs(i - (j - 1)) <= band:
                    E[i][j] = max(E[i][j - 1] - gap_extend, H[i][j - 1] - oe)
                if i >= 1 and abs((i - 1) - j) <= band:
                    F[i][j] = max(F[i - 1][j] - gap_extend, H[i - 1][j] - oe)
            d = H[i - 1][j - 1] + int(matrix[x[i - 1], y[j - 1]]) if i >= 1 and j >= 1 else NEG
            H[i][j] = max(d, E[i][j], F[i][j])
            best = max(best, H[i][j])
    return best


def gapped_windows(a, p1, b, p2, window=GAP_WINDOW):
    """The two one-sided subsequence pairs of a hit (Sec. 5.2.2): right from the
    seed start, left (reversed) from the letter before it, clipped to the
    sequences and to ``window`` letters."""
    xr = a[p1:p1 + window]
    yr = b[p2:p2 + window]
    xl = a[max(0, p1 - window):p1][::-1]
    yl = b[max(0, p2 - window):p2][::-1]
    return (xr, yr), (xl, yl)


def gapped_score(a, p1, b, p2, window=GAP_WINDOW, band=GAP_BAND, gap_open=GAP_OPEN,
                 gap_extend=GAP_EXTEND, matrix=BLOSUM62) -> int:
    (xr, yr), (xl, yl) = gapped_windows(a, p1, b, p2, window)
    return (gapped_side(xr, yr, band, gap_open, gap_extend, matrix)
            + gapped_side(xl, yl, band, gap_open, gap_extend, matrix))


def gapped_scores(bank1, bank2, hits, window=GAP_WINDOW, band=GAP_BAND, gap_open=GAP_OPEN,
                  gap_extend=GAP_EXTEND, matrix=BLOSUM62):
    """Gapped scores for many hits: the recurrences of :func:`gapped_side`,
    vectorised over hits (one numpy lane per hit), cell loops explicit."""
    A, B = sequences(bank1), sequences(bank2)
    hits = np.asarray(hits, dtype=np.int64).reshape(-1, 5)
    n = len(hits)
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    mat = np.asarray(matrix, dtype=np.int64)
    total = np.zeros(n, dtype=np.int64)
    for side in (+1, -1):
        X = np.full((n, window), 0, dtype=np.int64)
        Y = np.full((n, window), 0, dtype=np.int64)
        lx = np.zeros(n, dtype=np.int64)
        ly = np.zeros(n, dtype=np.int64)
        for h in range(n):
            s1_, p1_, s2_, p2_ = (int(v) for v in hits[h, :4])
            (xr, yr), (xl, yl) = gapped_windows(A[s1_], p1_, B[s2_], p2_, window)
            x, y = (xr, yr) if side > 0 else (xl, yl)
            X[h, :len(x)] = x
            Y[h, :len(y)] = y
            lx[h], ly[h] = len(x), len(y)
        total += _gapped_vec(X, Y, lx, ly, window, band, gap_open, gap_extend, mat)
    return total


def _gapped_vec(X, Y, lx, ly, window, band, gap_open, gap_extend, mat):
    NEG = np.int64(-(1 << 40))
    n = X.shape[0]
    oe = gap_open + gap_extend
    Hprev = np.full((window + 1, n), NEG, dtype=np.int64)
    Fprev = np.full((window + 1, n), NEG, dtype=np.int64)
    best = np.zeros(n, dtype=np.int64)
    for i in range(window + 1):
        Hcur = np.full((window + 1, n), NEG, dtype=np.int64)
        Fcur = np.full((window + 1, n), NEG, dtype=np.int64)
        Ecur = np.full((window + 1, n), NEG, dtype=np.int64)
        for j in range(max(0, i - band), min(window, i + band) + 1):
            exists = (i <= lx) & (j <= ly)
            if i == 0 and j == 0:
                h = np.where(exists, 0, NEG)
            else:
                e = f = d = np.full(n, NEG, dtype=np.int64)
                if j >= 1 and abs(i - (j - 1)) <= band:
                    e = np.maximum(Ecur[j - 1] - gap_extend, Hcur[j - 1] - oe)
                if i >= 1 and abs((i - 1) - j) <= band:
                    f = np.maximum(Fprev[j] - gap_extend, Hprev[j] - oe)
                if i >= 1 and j >= 1:
                    d = Hprev[j - 1] + mat[X[:, i - 1], Y[:, j - 1]]
                h = np.maximum(np.maximum(d, e), f)
                h = np.where(exists, h, NEG)
                Ecur[j] = np.where(exists, e, NEG)
                Fcur[j] = np.where(exists, f, NEG)
            # keep sentinels from drifting upward through repeated additions
            Hcur[j] = np.maximum(h, NEG)
            best = np.where(exists, np.maximum(best, h), best)
        Hprev, Fprev = Hcur, Fcur
    return best


# --------------------------------------------------------------------------- full gapped alignment (stage 3.2)

def full_side(x, y, gap_open=GAP_OPEN, gap_extend=GAP_EXTEND, matrix=BLOSUM62):
    """One-sided full gapped extension (Sec. 3.3.4, stage 3-2): the anchored
    affine-gap recurrences of :func:`gapped_side` over the whole of x and y, with
    no band and no window, plus the end cell and the path that reaches it.

    Cell (i, j) covers the first i letters of x and the first j of y; H(0, 0) = 0.
    best = max over all cells of H (so >= 0); the end cell is the first cell in
    row-major order (smallest i, then smallest j) whose H equals best.
    The path is traced back from the end cell with fixed preferences: a cell in
    state H came from the diagonal if that gives H, else from E, else from F; a
    cell in state E (or F) came from a gap opening (H of the left / upper cell
    minus open + extend) if that gives its value, else from an extension.
    Row 0 is one gap in x (state E) and column 0 one gap in y (state F).

    Returns (best, (i_end, j_end), moves) with moves read from the anchor outward:
    'D' pairs x[i] with y[j], 'E' puts y[j] against a gap, 'F' puts x[i] against a gap.
    """
    lx, ly = len(x), len(y)
    NEG = -(1 << 40)
    oe = gap_open + gap_extend
    H = [[NEG] * (ly + 1) for _ in range(lx + 1)]
    E = [[NEG] * (ly + 1) for _ in range(lx + 1)]
    F = [[NEG] * (ly + 1) for _ in range(lx + 1)]
    H[0][0] = 0
    best, end = 0, (0, 0)
    for i in range(lx + 1):
        for j in range(ly + 1):
            if i == 0 and j == 0:
                continue
            if j >= 1:
                E[i][j] = max(E[i][j - 1] - gap_extend, H[i][j - 1] - oe)
            if i >= 1:
                F[i][j] = max(F[i - 1][j] - gap_extend, H[i - 1][j] - oe)
            d = H[i - 1][j - 1] + int(matrix[x[i - 1], y[j - 1]]) if i >= 1 and j >= 1 else NEG
            H[i][j] = max(d, E[i][j], F[i][j])
            if H[i][j] > best:
                best, end = H[i][j], (i, j)
    moves = []
    i, j = end
    state = "H"
    while i > 0 or j > 0:
        if state == "H":
            if i >= 1 and j >= 1 and H[i][j] == H[i - 1][j - 1] + int(matrix[x[i - 1], y[j - 1]]):
                moves.append("D")
                i, j = i - 1, j - 1
                continue
            state = "E" if H[i][j] == E[i][j] else "F"
        elif state == "E":
            moves.append("E")
            state = "H" if E[i][j] == H[i][j - 1] - oe else "E"
            j -= 1
        else:
            moves.append("F")
            state = "H" if F[i][j] == H[i - 1][j] - oe else "F"
            i -= 1
    return best, end, moves[::-1]


def path_score(x, y, moves, gap_open=GAP_OPEN, gap_extend=GAP_EXTEND, matrix=BLOSUM62):
    """Score of an anchored path: substitution scores of its pairs minus, for each
    run of k consecutive moves of one gap kind, gap_open + k * gap_extend."""
    i = j = 0
    s = 0
    prev = None
    for m in moves:
        if m == "D":
            s += int(matrix[x[i], y[j]])
            i, j = i + 1, j + 1
        else:
            s -= gap_extend + (gap_open if m != prev else 0)
            if m == "E":
                j += 1
            else:
                i += 1
        prev = m
    return s


ALIGN_FIELDS = ("seq1", "seq2", "seed1", "seed2", "start1", "end1", "start2", "end2", "score",
                "length", "identities", "mismatches", "gap_opens", "hit")


def _side_walk(a, p1, b, p2, moves, step):
    """Pairs, segments and counts of one side's path in sequence coordinates.
    step = +1: the right side (pairs a[p1 + i], b[p2 + j]); -1: the left side
    (pairs a[p1 - 1 - i], b[p2 - 1 - j]).  Segments are maximal runs of pairs,
    as (diagonal p - q, first position in a, one past the last)."""
    i = j = 0
    segs, ident, mism, opens = [], 0, 0, 0
    run = None
    prev = None
    for m in moves:
        if m == "D":
            pa = p1 + i if step > 0 else p1 - 1 - i
            pb = p2 + j if step > 0 else p2 - 1 - j
            if a[pa] == b[pb]:
                ident += 1
            else:
                mism += 1
            if run is None:
                run = [pa - pb, pa, pa + 1]
            if step > 0:
                run[2] = pa + 1
            else:
                run[1] = pa
            i, j = i + 1, j + 1
        else:
            if run is not None:
                segs.append(tuple(run))
                run = None
            if m != prev:
                opens += 1
            if m == "E":
                j += 1
            else:
                i += 1
        prev = m
    if run is not None:
        segs.append(tuple(run))
    return segs, ident, mism, opens, i, j


def full_alignments(bank1, bank2, hits, gscore, passed, gap_open=GAP_OPEN, gap_extend=GAP_EXTEND,
                    matrix=BLOSUM62):
    """Stage 3.2 over the hits that passed the small gapped filter (Sec. 3.3.4:
    full dynamic programming for the survivors of stage 3.1, and the list of the
    ungapped pieces of the alignments already computed, kept per diagonal, that
    lets a hit lying on one of them skip its own computation).

    Reading: the surviving hits of one sequence pair are taken in order of
    decreasing gapped score, then increasing seed position in bank1, then in
    bank2.  A hit (p1, p2) is covered if an earlier alignment of the same pair
    has a piece on diagonal p1 - p2 whose positions in bank1 include p1; a
    covered hit computes nothing.  Otherwise its alignment is the left side
    (letters before the seed, read backwards) joined to the right side (from the
    seed start onwards), each from :func:`full_side` over the whole rest of the
    two sequences.

    Returns (records, cover): records is an int64 array with the columns of
    ALIGN_FIELDS, one row per computed alignment, in canonical order (sorted by
    its columns); cover[h] is the index of the hit whose alignment covers hit h
    (h itself if it computed one), -1 for hits that did not pass.
    """
    A, B = sequences(bank1), sequences(bank2)
    hits = np.asarray(hits, dtype=np.int64).reshape(-1, 5)
    gscore = np.asarray(gscore, dtype=np.int64).reshape(-1)
    passed = np.asarray(passed).reshape(-1).astype(bool)
    n = len(hits)
    cover = np.full(n, -1, dtype=np.int64)
    groups = {}
    for h in np.nonzero(passed)[0]:
        groups.setdefault((int(hits[h, 0]), int(hits[h, 2])), []).append(int(h))
    records = []
    for (s1, s2), members in groups.items():
        members.sort(key=lambda h: (-int(gscore[h]), int(hits[h, 1]), int(hits[h, 3])))
        a, b = A[s1], B[s2]
        pieces = []   # (diagonal, first, one past last, owning hit)
        for h in members:
            p1, p2 = int(hits[h, 1]), int(hits[h, 3])
            owner = next((o for d, f, t, o in pieces if d == p1 - p2 and f <= p1 < t), None)
            if owner is not None:
                cover[h] = owner
                continue
            cover[h] = h
            bR, _, mR = full_side(a[p1:], b[p2:], gap_open, gap_extend, matrix)
            bL, _, mL = full_side(a[:p1][::-1], b[:p2][::-1], gap_open, gap_extend, matrix)
            sR, iR, xR, oR, i_r, j_r = _side_walk(a, p1, b, p2, mR, +1)
            sL, iL, xL, oL, i_l, j_l = _side_walk(a, p1, b, p2, mL, -1)
            pieces.extend((d, f, t, h) for d, f, t in sR + sL)
            records.append((s1, s2, p1, p2, p1 - i_l, p1 + i_r, p2 - j_l, p2 + j_r, bR + bL,
                            len(mR) + len(mL), iR + iL, xR + xL, oR + oL, h))
    rec = np.asarray(records, dtype=np.int64).reshape(-1, len(ALIGN_FIELDS))
    if len(rec):
        rec = rec[np.lexsort(rec.T[::-1])]
    return rec, cover


# --------------------------------------------------------------------------- six-frame translation

# Standard genetic code (NCBI translation table 1): amino acid of codon
# b1 b2 b3 with bases in the order T C A G, first base slowest; '*' = stop.
_CODE_TCAG = "FFLLSSSSYY**CC*WLLLLPPPPHHQQRRRRIIIMTTTTNNKKSSRRVVVVAAAADDEEGGGG"
DNA = "ACGT"     # nucleotide codes 0..3
STOP = -1


def codon_table() -> np.ndarray:
    """int[64], indexed by 16 b1 + 4 b2 + b3 with nucleotide codes (A0 C1 G2 T3):
    the amino acid code in ALPHABET order, or STOP."""
    tcag = "TCAG"
    t = np.empty(64, dtype=np.int64)
    for i1, b1 in enumerate(tcag):
        for i2, b2 in enumerate(tcag):
            for i3, b3 in enumerate(tcag):
                aa = _CODE_TCAG[16 * i1 + 4 * i2 + i3]
                t[16 * DNA.index(b1) + 4 * DNA.index(b2) + DNA.index(b3)] = STOP if aa == "*" else ALPHABET.index(aa)
    return t


CODONS = codon_table()


def frame_codons(dna: np.ndarray, frame: int) -> np.ndarray:
    """Amino acid codes (or STOP) of one reading frame of one sequence."""
    s = np.asarray(dna, dtype=np.int64)
    if frame >= 3:
        s = (3 - s)[::-1]               # reverse complement
    s = s[frame % 3:]
    n = len(s) // 3                     # a trailing partial codon is dropped
    c = s[:3 * n].reshape(n, 3)
    return CODONS[16 * c[:, 0] + 4 * c[:, 1] + c[:, 2]]


def translate6(dna_codes, dna_start):
    """Fragments of all six frames of every sequence, in the order (sequence,
    frame, position): (list of uint8 arrays, int64[n, 3] table of
    (sequence, frame, offset of the fragment's first amino acid in its frame))."""
    frags, table = [], []
    for d in range(len(dna_start) - 1):
        seq = dna_codes[int(dna_start[d]):int(dna_start[d + 1])]
        for f in range(6):
            aa = frame_codons(seq, f)
            i, n = 0, len(aa)
            while i < n:
                if aa[i] == STOP:
                    i += 1
                    continue
                j = i
                while j < n and aa[j] != STOP:
                    j += 1
                frags.append(aa[i:j].astype(np.uint8))
                table.append((d, f, i))
                i = j
    return frags, np.array(table, dtype=np.int64).reshape(-1, 3)


def frame_position(dna_len: int, frame: int, aa_offset: int) -> int:
    """Forward-strand coordinate of the first nucleotide of codon aa_offset of
    a frame (for frames 3..5 the codon reads leftward from this nucleotide)."""
    p = frame % 3 + 3 * aa_offset
    return p if frame < 3 else dna_len - 1 - p
