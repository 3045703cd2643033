"""Seeded synthetic protein banks standing in for the paper's PIR / SWISS-PROT banks.

This module only generates inputs. It holds none of the search method's
arithmetic (no seed keys, no scoring, no extension); both the CPU oracle and the
GPU path consume what it produces.

Storage format of a bank (the "padded layout")
---------------------------------------------
``codes`` is one ``uint8`` array: a run of ``PAD_LEN`` pad codes (value
``PAD_CODE`` = 20), sequence 0, another pad run, sequence 1, ..., the last
sequence and a final pad run.  Residues are coded 0..19 in the order
``ALPHABET``.  ``seq_start`` is ``int64[n+1]``: ``seq_start[i]`` is the offset of
the first residue of sequence ``i`` and ``seq_start[n] == len(codes)``, so the
length of sequence ``i`` is ``seq_start[i+1] - seq_start[i] - PAD_LEN``.

Workload recipe (the paper's banks, Annex 1, are not available)
---------------------------------------------------------------
* lengths: ``clamp(round(exp(mu + sigma*Z)), 50, 1000)`` with ``sigma = 0.6`` and
  ``mu = ln 300 - sigma^2/2`` (unclamped mean 300);
* residues: i.i.d. from the BLOSUM62 background composition;
* planted homologs: a bank1 sequence is mutated (per position with probability
  ``1 - identity``, the new residue ``b != a`` drawn with probability
  proportional to ``f_b exp(lambda s_ab)``, the BLOSUM62 target frequencies),
  with indels at rate 0.02 per position (half insertions of background
  residues, half deletions, length ``min(Geom(1/2), 5)``), and the result
  replaces a bank2 sequence;
* low-complexity repeats (skewed configuration): 5% of the sequences of each
  bank receive one run of length U[100, 400] (clamped to the sequence) drawn
  uniformly from one of three small alphabets of 2, 3 and 4 letters.  Each
  bank has its own pool of three alphabets, and the two pools share no letter
  (18 distinct letters, drawn once per seed): the words of a bank-1 run and of
  a bank-2 run then differ in their first letter, so they never share a seed
  key.  With one shared pool every pair of same-alphabet runs sharing a key
  scores above S1 (about 1.5e10 hits, 300 GB of hit records), which no single
  device holds; with disjoint pools the buckets stay just as skewed (each
  run's words pile into a few keys of its own bank) and a repeat window is only
  paired with ordinary windows of the other bank.

Random streams: ``numpy.random.SeedSequence(651300 + cfg).spawn(6)`` gives the
independent streams (lengths, residues, plant choice, mutation, indels,
repeats).
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np

ALPHABET = "ACDEFGHIKLMNPQRSTVWY"
PAD_CODE = 20
PAD_LEN = 20

# BLOSUM62 background amino-acid frequencies (Henikoff & Henikoff 1992), in
# ALPHABET order.  Used here only to draw residues and homolog substitutions.
_BG = {
    "A": .074, "R": .052, "N": .045, "D": .054, "C": .025, "Q": .034, "E": .054,
    "G": .074, "H": .026, "I": .068, "L": .099, "K": .058, "M": .025, "F": .047,
    "P": .039, "S": .057, "T": .051, "W": .013, "Y": .032, "V": .073,
}
BACKGROUND = np.array([_BG[c] for c in ALPHABET], dtype=np.float64)

# BLOSUM62 in the NCBI row order ARNDCQEGHILKMFPSTWYV; this generator's own copy,
# used only to draw realistic substitutions in planted homologs.
_B62_ORDER = "ARNDCQEGHILKMFPSTWYV"
_B62_ROWS = """
 4 -1 -2 -2  0 -1 -1  0 -2 -1 -1 -1 -1 -2 -1  1  0 -3 -2  0
-1  5  0 -2 -3  1  0 -2  0 -3 -2  2 -1 -3 -2 -1 -1 -3 -2 -3
-2  0  6  1 -3  0  0  0  1 -3 -3  0 -2 -3 -2  1  0 -4 -2 -3
-2 -2  1  6 -3  0  2 -1 -1 -3 -4 -1 -3 -3 -1  0 -1 -4 -3 -3
 0 -3 -3 -3  9 -3 -4 -3 -3 -1 -1 -3 -1 -2 -3 -1 -1 -2 -2 -1
-1  1  0  0 -3  5  2 -2  0 -3 -2  1  0 -3 -1  0 -1 -2 -1 -2
-1  0  0  2 -4  2  5 -2  0 -3 -3  1 -2 -3 -1  0 -1 -3 -2 -2
 0 -2  0 -1 -3 -2 -2  6 -2 -4 -4 -2 -3 -3 -2  0 -2 -2 -3 -3
-2  0  1 -1 -3  0  0 -2  8 -3 -3 -1 -2 -1 -2 -1 -2 -2  2 -3
-1 -3 -3 -3 -1 -3 -3 -4 -3  4  2 -3  1  0 -3 -2 -1 -3 -1  3
-1 -2 -3 -4 -1 -2 -3 -4 -3  2  4 -2  2  0 -3 -2 -1 -2 -1  1
-1  2  0 -1 -3  1  1 -2 -1 -3 -2  5 -1 -3 -1  0 -1 -3 -2 -2
-1 -1 -2 -3 -1  0 -2 -3 -2  1  2 -1  5  0 -2 -1 -1 -1 -1  1
-2 -3 -3 -3 -2 -3 -3 -3 -1  0  0 -3  0  6 -4 -2 -2  1  3 -1
-1 -2 -2 -1 -3 -1 -1 -2 -2 -3 -3 -1 -2 -4  7 -1 -1 -4 -3 -2
 1 -1  1  0 -1  0  0  0 -1 -2 -2  0 -1 -2 -1  4  1 -3 -2 -2
 0 -1  0 -1 -1 -1 -1 -2 -2 -1 -1 -1 -1 -2 -1  1  5 -2 -2  0
-3 -3 -4 -4 -2 -2 -3 -2 -2 -3 -2 -3 -1  1 -4 -3 -2 11  2 -3
-2 -2 -2 -3 -2 -1 -2 -3  2 -1 -1 -2 -1  3 -3 -2 -2  2  7 -1
 0 -3 -3 -3 -1 -2 -2 -3 -3  3  1 -2  1 -1 -2 -2  0 -3 -1  4
"""


def _b62_in_alphabet_order() -> np.ndarray:
    raw = np.array([[int(x) for x in r.split()] for r in _B62_ROWS.strip().splitlines()])
    perm = [_B62_ORDER.index(c) for c in ALPHABET]
    return raw[np.ix_(perm, perm)]


def _substitution_probs() -> np.ndarray:
    """Row-stochastic matrix P[a, b] (b != a) proportional to f_b exp(lam s_ab)."""
    s = _b62_in_alphabet_order().astype(np.float64)
    ff = np.outer(BACKGROUND, BACKGROUND)
    lo, hi = 0.05, 2.0  # bisection on sum f_a f_b exp(lam s_ab) = 1
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if (ff * np.exp(mid * s)).sum() > 1.0:
            hi = mid
        else:
            lo = mid
    q = ff * np.exp(lo * s)
    np.fill_diagonal(q, 0.0)
    return q / q.sum(axis=1, keepdims=True)


@dataclasses.dataclass
class Bank:
    codes: np.ndarray      # uint8, padded layout
    seq_start: np.ndarray  # int64[n+1]

    @property
    def n_seqs(self) -> int:
        return int(self.seq_start.shape[0] - 1)

    @property
    def lengths(self) -> np.ndarray:
        return (np.diff(self.seq_start) - PAD_LEN).astype(np.int64)

    @property
    def n_residues(self) -> int:
        return int(self.lengths.sum())

    def seq(self, i: int) -> np.ndarray:
        s = int(self.seq_start[i])
        return self.codes[s:s + int(self.lengths[i])]

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(self.codes.tobytes())
        h.update(self.seq_start.tobytes())
        return h.hexdigest()

    @staticmethod
    def from_seqs(seqs) -> "Bank":
        lens = np.array([len(s) for s in seqs], dtype=np.int64)
        n = len(seqs)
        seq_start = np.empty(n + 1, dtype=np.int64)
        seq_start[0] = PAD_LEN
        if n:
            seq_start[1:] = PAD_LEN + np.cumsum(lens + PAD_LEN)
        codes = np.full(int(seq_start[-1]), PAD_CODE, dtype=np.uint8)
        for i, s in enumerate(seqs):
            codes[seq_start[i]:seq_start[i] + lens[i]] = np.asarray(s, dtype=np.uint8)
        return Bank(codes, seq_start)

    @staticmethod
    def from_flat(flat, lens) -> "Bank":
        """Bank from concatenated residues ``flat`` and sequence lengths ``lens``."""
        lens = np.asarray(lens, dtype=np.int64)
        n = len(lens)
        seq_start = np.empty(n + 1, dtype=np.int64)
        seq_start[0] = PAD_LEN
        seq_start[1:] = PAD_LEN + np.cumsum(lens + PAD_LEN)
        codes = np.full(int(seq_start[-1]), PAD_CODE, dtype=np.uint8)
        # residue r of sequence i goes to seq_start[i] + r: shift each residue by PAD_LEN * (i + 1)
        seq_of = np.repeat(np.arange(n, dtype=np.int64), lens)
        codes[np.arange(int(lens.sum()), dtype=np.int64) + PAD_LEN * (seq_of + 1)] = flat
        return Bank(codes, seq_start)

    @staticmethod
    def from_strings(strs) -> "Bank":
        return Bank.from_seqs([encode(s) for s in strs])


def encode(s: str) -> np.ndarray:
    lut = {c: i for i, c in enumerate(ALPHABET)}
    return np.array([lut[c] for c in s.upper()], dtype=np.uint8)


def decode(codes) -> str:
    return "".join(ALPHABET[int(c)] for c in codes)


@dataclasses.dataclass
class Plant:
    src: int            # bank1 sequence index
    dst: int            # bank2 sequence index it replaced
    target_identity: float
    identity: float     # realised identity over aligned (non-indel) columns
    colmap: np.ndarray  # int32, per homolog position: source position or -1 (insertion)


@dataclasses.dataclass
class Workload:
    cfg: int
    bank1: Bank
    bank2: Bank
    plants: list
    description: str
    repeat_pools: tuple = ()  # per bank, the alphabets its repeat runs are drawn from


@dataclasses.dataclass(frozen=True)
class ConfigSpec:
    n1: int
    n2: int
    n_plants: int
    identity: tuple          # (lo, hi); lo == hi means fixed
    repeats: bool
    description: str


CONFIGS = {
    0: ConfigSpec(200, 2_000, 20, (0.40, 0.40), False,
                  "PLAST-P tiny: 200 x 2,000 proteins, 20 planted homologs at 40% identity"),
    1: ConfigSpec(10_000, 100_000, 500, (0.30, 0.60), False,
                  "PLAST-P: 10,000 x 100,000 proteins, 500 planted homologs at 30-60% identity"),
    2: ConfigSpec(20_000, 300_000, 0, (0.40, 0.40), True,
                  "PLAST-P skewed: 20,000 x 300,000 proteins, 5% carry 2-4-letter repeats"),
}

_SIGMA = 0.6
_MU = math.log(300.0) - _SIGMA ** 2 / 2
INDEL_RATE = 0.02


def _lengths(rng, n):
    z = rng.standard_normal(n)
    return np.clip(np.rint(np.exp(_MU + _SIGMA * z)), 50, 1000).astype(np.int64)


def _mutate(src: np.ndarray, identity: float, rng_mut, rng_indel, subst):
    out, colmap = [], []
    n = len(src)
    mutate = rng_mut.random(n) >= identity
    u = rng_mut.random(n)
    cum = np.cumsum(subst, axis=1)
    indel_at = rng_indel.random(n) < INDEL_RATE
    p = 0
    while p < n:
        if indel_at[p]:
            length = min(int(rng_indel.geometric(0.5)), 5)
            if rng_indel.random() < 0.5:  # insertion before position p
                ins = rng_indel.choice(20, size=length, p=BACKGROUND)
                out.extend(int(x) for x in ins)
                colmap.extend([-1] * length)
                indel_at[p] = False        # then emit position p normally
                continue
            p += length                    # deletion of `length` source positions
            continue
        a = int(src[p])
        if mutate[p]:
            b = int(min(np.searchsorted(cum[a], u[p] * cum[a, -1], side="right"), 19))
            if b == a:  # guard against rounding at the cumulative edge
                b = (a + 1) % 20
            out.append(b)
        else:
            out.append(a)
        colmap.append(p)
        p += 1
    out = np.array(out, dtype=np.uint8)
    colmap = np.array(colmap, dtype=np.int32)
    aligned = colmap >= 0
    ident = float(np.mean(out[aligned] == src[colmap[aligned]])) if aligned.any() else 0.0
    return out, colmap, ident


def _mutate_vec(src: np.ndarray, identity: float, rng, cum):
    """The mutation model of ``_mutate`` (BLOSUM62-conditional substitutions at
    rate 1 - identity, indels at INDEL_RATE of length min(Geom(1/2), 5), half
    insertions of background residues) drawn with vectorised numpy; used for
    the many homologs of the serving workload."""
    n = len(src)
    out = src.copy()
    mut = np.nonzero(rng.random(n) >= identity)[0]
    if len(mut):
        a = out[mut].astype(np.int64)
        u = rng.random(len(mut)) * cum[a, -1]
        b = np.minimum((cum[a] <= u[:, None]).sum(axis=1), 19)
        b = np.where(b == a, (a + 1) % 20, b)
        out[mut] = b.astype(np.uint8)
    ev = np.nonzero(rng.random(n) < INDEL_RATE)[0]
    if not len(ev):
        return out
    pieces, p = [], 0
    for e in ev:
        if e < p:
            continue
        length = min(int(rng.geometric(0.5)), 5)
        pieces.append(out[p:e])
        if rng.random() < 0.5:
            pieces.append(rng.choice(20, size=length, p=BACKGROUND).astype(np.uint8))
            p = e
        else:
            p = e + length
    pieces.append(out[p:])
    return np.concatenate(pieces)


def _add_repeats(seqs, rng, pool):
    n = len(seqs)
    chosen = rng.choice(n, size=max(1, int(round(0.05 * n))), replace=False)
    for i in np.sort(chosen):
        s = seqs[i]
        L = min(int(rng.integers(100, 401)), len(s))
        off = int(rng.integers(0, len(s) - L + 1))
        alpha = pool[int(rng.integers(0, len(pool)))]
        s[off:off + L] = rng.choice(alpha, size=L)
    return chosen


def _split(flat, lens):
    offs = np.concatenate([[0], np.cumsum(lens)])
    return [flat[offs[i]:offs[i + 1]].copy() for i in range(len(lens))]


def make_workload(cfg: int, plants: bool = True, scale: float = 1.0) -> Workload:
    """Build configuration ``cfg`` deterministically.

    ``plants=False`` skips homolog planting (used to calibrate thresholds on
    purely random banks).  ``scale`` shrinks both banks proportionally (for
    quick tests); the random streams are the same.
    """
    spec = CONFIGS[cfg]
    n1 = max(1, int(round(spec.n1 * scale)))
    n2 = max(1, int(round(spec.n2 * scale)))
    ss = np.random.SeedSequence(651300 + cfg).spawn(6)
    r_len, r_res, r_plant, r_mut, r_indel, r_rep = [np.random.Generator(np.random.PCG64(s)) for s in ss]
    lens = _lengths(r_len, n1 + n2)
    flat = r_res.choice(20, size=int(lens.sum()), p=BACKGROUND).astype(np.uint8)
    seqs = _split(flat, lens)
    s1, s2 = seqs[:n1], seqs[n1:]
    if spec.repeats:
        letters = r_rep.permutation(20)
        pool1 = [letters[0:2], letters[2:5], letters[5:9]]
        pool2 = [letters[9:11], letters[11:14], letters[14:18]]
        _add_repeats(s1, r_rep, pool1)
        _add_repeats(s2, r_rep, pool2)
        pools = (pool1, pool2)
    else:
        pools = ()
    planted = []
    n_pl = min(spec.n_plants, n1, n2) if plants else 0
    if n_pl:
        subst = _substitution_probs()
        src = r_plant.choice(n1, size=n_pl, replace=False)
        dst = r_plant.choice(n2, size=n_pl, replace=False)
        lo, hi = spec.identity
        ids = np.full(n_pl, lo) if lo == hi else r_plant.uniform(lo, hi, size=n_pl)
        for k in range(n_pl):
            hom, colmap, ident = _mutate(s1[src[k]], float(ids[k]), r_mut, r_indel, subst)
            s2[dst[k]] = hom
            planted.append(Plant(int(src[k]), int(dst[k]), float(ids[k]), ident, colmap))
    return Workload(cfg, Bank.from_seqs(s1), Bank.from_seqs(s2), planted, spec.description, pools)


def shared_repeat_variant(w: Workload, frac: float = 0.01, letters=(0, 9), run=(100, 400),
                          seed: int = 6513) -> Workload:
    """A variant of a workload in which ``frac`` of the sequences of each bank
    carry one run (length U[run], clamped to the sequence) drawn from the same
    small alphabet ``letters`` (default A and L) in both banks, so that the few
    seed keys of that alphabet are heavy in both banks at once.  The banks are
    copied; the workload's own streams are not touched (the runs come from
    SeedSequence(seed))."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    alpha = np.asarray(letters, dtype=np.uint8)
    banks = []
    for bank in (w.bank1, w.bank2):
        codes = bank.codes.copy()
        lens = bank.lengths
        chosen = rng.choice(bank.n_seqs, size=max(1, int(round(frac * bank.n_seqs))), replace=False)
        for i in np.sort(chosen):
            L = min(int(rng.integers(run[0], run[1] + 1)), int(lens[i]))
            off = int(rng.integers(0, int(lens[i]) - L + 1))
            a = int(bank.seq_start[i]) + off
            codes[a:a + L] = rng.choice(alpha, size=L)
        banks.append(Bank(codes, bank.seq_start.copy()))
    return Workload(w.cfg, banks[0], banks[1], w.plants, w.description + "; %.0f%% of each bank's sequences carry a "
                    "run over the same %d letters" % (100 * frac, len(alpha)), w.repeat_pools)


def random_bank(rng, n, lo=1, hi=60, alphabet_size=20) -> Bank:
    """Small random bank for tests: ``n`` sequences of length U[lo, hi]."""
    lens = rng.integers(lo, hi + 1, size=n)
    return Bank.from_seqs([rng.integers(0, alphabet_size, size=int(L)).astype(np.uint8) for L in lens])


# --------------------------------------------------------------------------- serving workload

@dataclasses.dataclass
class ServingWorkload:
    resident: Bank
    requests: list      # query banks
    homologs: list      # per request: (query sequence, resident sequence) of each planted homolog
    description: str


def make_serving(n_resident: int = 1_000_000, n_requests: int = 1000, max_query: int = 500,
                 homolog_frac: float = 0.10, identity=(0.30, 0.60), scale: float = 1.0) -> ServingWorkload:
    """Serving configuration: a resident bank of ``n_resident`` proteins with the
    distributions of configuration 0, and ``n_requests`` query banks of
    U{1..max_query} proteins each, ``homolog_frac`` of them (rounded) planted
    homologs of random resident proteins (mutated as in ``make_workload``).
    ``scale`` shrinks the resident bank.  Streams: SeedSequence(651304).spawn(6)."""
    ss = np.random.SeedSequence(651300 + 4).spawn(6)
    r_len, r_res, r_req, r_plant, r_mut, r_indel = [np.random.Generator(np.random.PCG64(s)) for s in ss]
    n_res = max(1, int(round(n_resident * scale)))
    lens = _lengths(r_len, n_res)
    flat = r_res.choice(20, size=int(lens.sum()), p=BACKGROUND).astype(np.uint8)
    resident = Bank.from_flat(flat, lens)
    cum = np.cumsum(_substitution_probs(), axis=1)
    requests, homologs = [], []
    for _ in range(n_requests):
        m = int(r_req.integers(1, max_query + 1))
        ql = _lengths(r_req, m)
        seqs = _split(r_req.choice(20, size=int(ql.sum()), p=BACKGROUND).astype(np.uint8), ql)
        k = int(round(homolog_frac * m))
        pl = []
        if k:
            slots = r_plant.choice(m, size=k, replace=False)
            srcs = r_plant.choice(n_res, size=k, replace=False)
            ids = r_plant.uniform(identity[0], identity[1], size=k)
            for q, rs, idt in zip(slots, srcs, ids):
                a, b = int(resident.seq_start[rs]), int(resident.seq_start[rs + 1]) - PAD_LEN
                src = resident.codes[a:b]
                hom = _mutate_vec(src, float(idt), r_mut, cum)
                seqs[int(q)] = hom if len(hom) else src.copy()
                pl.append((int(q), int(rs)))
        requests.append(Bank.from_seqs(seqs))
        homologs.append(pl)
    return ServingWorkload(resident, requests, homologs,
                           "serving: %d resident proteins, %d requests of 1-%d query proteins, %d%% planted homologs"
                           % (n_res, n_requests, max_query, round(100 * homolog_frac)))


# --------------------------------------------------------------------------- nucleotide banks (TPLAST-N)

DNA_ALPHABET = "ACGT"  # codes 0..3; the complement of code c is 3 - c

# Standard genetic code, written as the codons of each amino acid (for reverse
# translation of planted homologs).
_SYNONYMS = {
    "A": "GCT GCC GCA GCG", "C": "TGT TGC", "D": "GAT GAC", "E": "GAA GAG", "F": "TTT TTC",
    "G": "GGT GGC GGA GGG", "H": "CAT CAC", "I": "ATT ATC ATA", "K": "AAA AAG",
    "L": "TTA TTG CTT CTC CTA CTG", "M": "ATG", "N": "AAT AAC", "P": "CCT CCC CCA CCG", "Q": "CAA CAG",
    "R": "CGT CGC CGA CGG AGA AGG", "S": "TCT TCC TCA TCG AGT AGC", "T": "ACT ACC ACA ACG",
    "V": "GTT GTC GTA GTG", "W": "TGG", "Y": "TAT TAC",
}


def synonym_codons():
    """code (0..19) -> list of codons as int8[3] arrays of nucleotide codes."""
    lut = {c: i for i, c in enumerate(DNA_ALPHABET)}
    return [[np.array([lut[b] for b in cod], dtype=np.uint8) for cod in _SYNONYMS[a].split()] for a in ALPHABET]


@dataclasses.dataclass
class DnaBank:
    codes: np.ndarray   # uint8 in 0..3, sequences concatenated
    start: np.ndarray   # int64[n + 1]

    @property
    def n_seqs(self) -> int:
        return int(self.start.shape[0] - 1)

    def seq(self, i: int) -> np.ndarray:
        return self.codes[int(self.start[i]):int(self.start[i + 1])]

    @staticmethod
    def from_seqs(seqs) -> "DnaBank":
        lens = np.array([len(s) for s in seqs], dtype=np.int64)
        start = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        codes = np.concatenate([np.asarray(s, dtype=np.uint8) for s in seqs]) if len(seqs) else np.zeros(0, np.uint8)
        return DnaBank(codes, start)


@dataclasses.dataclass
class DnaPlant:
    protein: int   # bank-1 sequence
    dna: int       # DNA sequence carrying the homolog
    strand: int    # +1 or -1
    offset: int    # first nucleotide of the coding region on the forward strand
    n_codons: int


@dataclasses.dataclass
class TplastnWorkload:
    bank1: Bank
    dna: DnaBank
    plants: list
    description: str


def make_tplastn(n_proteins: int = 5000, n_dna: int = 2000, dna_len=(50_000, 200_000), n_plants: int = 100,
                 identity: float = 0.40, gc: float = 0.40, scale: float = 1.0) -> TplastnWorkload:
    """Configuration 3: ``n_proteins`` proteins with configuration 0's
    distributions against ``n_dna`` random DNA sequences of U[dna_len]
    nucleotides (GC content ``gc``), carrying ``n_plants`` homologs of bank-1
    proteins (mutated at ``identity`` as in ``make_workload``) reverse-translated
    with uniformly chosen synonymous codons, each written over a random
    position on a random strand.  ``scale`` shrinks the sequence counts.
    Streams: SeedSequence(651303).spawn(6)."""
    ss = np.random.SeedSequence(651300 + 3).spawn(6)
    r_len, r_res, r_dna, r_plant, r_mut, r_indel = [np.random.Generator(np.random.PCG64(s)) for s in ss]
    n1 = max(1, int(round(n_proteins * scale)))
    nd = max(1, int(round(n_dna * scale)))
    lens = _lengths(r_len, n1)
    s1 = _split(r_res.choice(20, size=int(lens.sum()), p=BACKGROUND).astype(np.uint8), lens)
    p_nt = np.array([(1 - gc) / 2, gc / 2, gc / 2, (1 - gc) / 2])  # A C G T
    dl = r_dna.integers(dna_len[0], dna_len[1] + 1, size=nd)
    dna = _split(r_dna.choice(4, size=int(dl.sum()), p=p_nt).astype(np.uint8), dl)
    syn = synonym_codons()
    subst = _substitution_probs()
    plants = []
    for k, src in enumerate(r_plant.choice(n1, size=min(n_plants, n1), replace=False)):
        hom, _, _ = _mutate(s1[int(src)], identity, r_mut, r_indel, subst)
        coding = np.concatenate([syn[a][int(r_plant.integers(len(syn[a])))] for a in hom]) if len(hom) else \
            np.zeros(0, np.uint8)
        d = int(r_plant.integers(nd))
        if len(coding) == 0 or len(coding) > len(dna[d]):
            continue
        off = int(r_plant.integers(0, len(dna[d]) - len(coding) + 1))
        strand = 1 if r_plant.random() < 0.5 else -1
        dna[d][off:off + len(coding)] = coding if strand > 0 else (3 - coding)[::-1]
        plants.append(DnaPlant(int(src), d, strand, off, len(hom)))
    return TplastnWorkload(Bank.from_seqs(s1), DnaBank.from_seqs(dna), plants,
                           "TPLAST-N: %d proteins vs %d DNA sequences of %d-%d nt (GC %.0f%%), %d planted homologs "
                           "at %.0f%% identity" % (n1, nd, dna_len[0], dna_len[1], 100 * gc, len(plants),
                                                   100 * identity))


@dataclasses.dataclass
class PlastxWorkload:
    dna1: DnaBank
    dna2: DnaBank
    plants: list        # (DnaPlant in dna1, DnaPlant in dna2) of each homolog pair
    description: str


def _plant_coding(seqs, prot, rng, syn, d):
    coding = np.concatenate([syn[a][int(rng.integers(len(syn[a])))] for a in prot])
    if len(coding) == 0 or len(coding) > len(seqs[d]):
        return None
    off = int(rng.integers(0, len(seqs[d]) - len(coding) + 1))
    strand = 1 if rng.random() < 0.5 else -1
    seqs[d][off:off + len(coding)] = coding if strand > 0 else (3 - coding)[::-1]
    return DnaPlant(-1, d, strand, off, len(prot))


def make_plastx(n_dna1: int = 200, n_dna2: int = 1000, dna_len=(20_000, 50_000), n_plants: int = 50,
                identity: float = 0.40, gc: float = 0.40, scale: float = 1.0) -> PlastxWorkload:
    """PLAST-X (both banks nucleotide): two random DNA banks (GC content
    ``gc``) sharing ``n_plants`` homologous coding regions: a random protein
    with configuration 0's length distribution, reverse-translated with random
    synonymous codons into bank 1, and a copy mutated at ``identity``
    reverse-translated into bank 2, each at a random offset on a random strand.
    Streams: SeedSequence(651305).spawn(6)."""
    ss = np.random.SeedSequence(651300 + 5).spawn(6)
    r_len, r_res, r_dna, r_plant, r_mut, r_indel = [np.random.Generator(np.random.PCG64(s)) for s in ss]
    n1, n2 = max(1, int(round(n_dna1 * scale))), max(1, int(round(n_dna2 * scale)))
    p_nt = np.array([(1 - gc) / 2, gc / 2, gc / 2, (1 - gc) / 2])

    def bank(n):
        dl = r_dna.integers(dna_len[0], dna_len[1] + 1, size=n)
        return _split(r_dna.choice(4, size=int(dl.sum()), p=p_nt).astype(np.uint8), dl)

    d1, d2 = bank(n1), bank(n2)
    syn = synonym_codons()
    subst = _substitution_probs()
    plants = []
    for L in _lengths(r_len, n_plants):
        prot = r_res.choice(20, size=int(L), p=BACKGROUND).astype(np.uint8)
        hom, _, _ = _mutate(prot, identity, r_mut, r_indel, subst)
        a = _plant_coding(d1, prot, r_plant, syn, int(r_plant.integers(n1)))
        b = _plant_coding(d2, hom, r_plant, syn, int(r_plant.integers(n2)))
        if a is not None and b is not None:
            plants.append((a, b))
    return PlastxWorkload(DnaBank.from_seqs(d1), DnaBank.from_seqs(d2), plants,
                          "PLAST-X: %d x %d DNA sequences of %d-%d nt (GC %.0f%%), %d planted homologous coding "
                          "regions at %.0f%% identity" % (n1, n2, dna_len[0], dna_len[1], 100 * gc, len(plants),
                                                          100 * identity))
