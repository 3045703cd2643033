"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake (a mistyped table entry, an off-by-one
limit, a dropped term, a wrong sign, a transposed operand, a wrong tie-break)
in a copy of the oracle's source, puts the copy in the oracle's place for the
pin tests (test_oracle_pins.py, test_oracle_stage32.py) and runs them: at least
one pin must fail.  The oracle's files are never modified; C mutants are built
into pytest's temporary directory.  The pins closest to the mutated function run
first and the run stops at the first failure, so a case takes a few seconds.
"""
import ctypes
import functools
import os
import subprocess
import types

import numpy as np
import pytest

import test_oracle_pins as P
import test_oracle_stage32 as S
from oracle import coracle as C
from oracle import plast_oracle as O
from paper_0804_3643_amd import params

ORACLE_DIR = os.path.dirname(os.path.abspath(O.__file__))
PY_SRC = os.path.join(ORACLE_DIR, "plast_oracle.py")
C_SRC = os.path.join(ORACLE_DIR, "plast_oracle.c")

# (case, stage, text in the oracle, replacement); every text occurs exactly once.
PY_MUTANTS = [
    ("blosum62 cell mistyped", "matrix", "H -2 -3 -1  0 -1 -2  8", "H -2 -3 -1  0 -1 -2  7"),
    ("blosum62 sign dropped", "matrix", "W -3 -2 -4 -3  1", "W -3 -2 -4 -3 -1"),
    ("seed class split wrongly", "seed", '"G", "IV", "ML",', '"G", "I", "VML",'),
    ("seed position-2 class", "seed", '["CFYWMLIV", "GPATSNHQEDRK"]', '["CFYWMLIVG", "PATSNHQEDRK"]'),
    ("seed radix", "seed", "* 2 + CLASS2[w1]) * 11", "* 2 + CLASS2[w1]) * 12"),
    ("index drops the last word", "index", "n = len(a) - W + 1", "n = len(a) - W"),
    ("index positions off by one", "index", "pos.append(np.arange(n, dtype=np.int64))",
     "pos.append(np.arange(1, n + 1, dtype=np.int64))"),
    ("ungapped right window short", "ungapped", "rmax = min(right, len(a) - p1, len(b) - p2)",
     "rmax = min(right - 1, len(a) - p1, len(b) - p2)"),
    ("ungapped left window short", "ungapped", "for t in range(1, lmax + 1):", "for t in range(1, lmax):"),
    ("ungapped matrix transposed", "ungapped", "s += int(matrix[a[p1 + t], b[p2 + t]])",
     "s += int(matrix[b[p2 + t], a[p1 + t]])"),
    ("ungapped last prefix instead of best", "ungapped", "best_r = max(best_r, s)", "best_r = s"),
    ("ungapped (vectorised) right limit", "ungapped", "cs = np.where(t[None, None, :] < rmax[:, :, None], cs, NEG)",
     "cs = np.where(t[None, None, :] <= rmax[:, :, None], cs, NEG)"),
    ("ungapped (vectorised) empty left side dropped", "ungapped", "best_l = np.maximum(cs.max(axis=2), 0)",
     "best_l = cs.max(axis=2)"),
    ("ungapped (vectorised) left letters shifted", "ungapped", "ia = np.maximum(pA[:, None] - t, 0)",
     "ia = np.maximum(pA[:, None] - t + 1, 0)"),
    ("gapped open without extend", "gapped", "oe = None if gap_open is None else gap_open + gap_extend",
     "oe = None if gap_open is None else gap_open"),
    ("gapped band one too wide", "gapped", "if abs(i - j) > band or (i == 0 and j == 0):",
     "if abs(i - j) > band + 1 or (i == 0 and j == 0):"),
    ("gapped extension charged as an opening", "gapped",
     "                    E[i][j] = max(E[i][j - 1] - gap_extend, H[i][j - 1] - oe)",
     "                    E[i][j] = max(E[i][j - 1] - oe, H[i][j - 1] - oe)"),
    ("gapped matrix transposed", "gapped",
     "                    F[i][j] = max(F[i - 1][j] - gap_extend, H[i - 1][j] - oe)\n"
     "            d = H[i - 1][j - 1] + int(matrix[x[i - 1], y[j - 1]])",
     "                    F[i][j] = max(F[i - 1][j] - gap_extend, H[i - 1][j] - oe)\n"
     "            d = H[i - 1][j - 1] + int(matrix[y[j - 1], x[i - 1]])"),
    ("gapped left window not reversed", "gapped", "xl = a[max(0, p1 - window):p1][::-1]",
     "xl = a[max(0, p1 - window):p1]"),
    ("gapped right window starts after the seed", "gapped", "yr = b[p2:p2 + window]", "yr = b[p2 + 1:p2 + window]"),
    ("gapped (vectorised) row limit", "gapped", "exists = (i <= lx) & (j <= ly)", "exists = (i < lx) & (j <= ly)"),
    ("gapped (vectorised) vertical opening", "gapped", "f = np.maximum(Fprev[j] - gap_extend, Hprev[j] - oe)",
     "f = np.maximum(Fprev[j] - gap_extend, Hprev[j] - gap_extend)"),
    ("full side last best cell", "full", "if H[i][j] > best:", "if H[i][j] >= best:"),
    ("full side prefers F over E", "full", 'state = "E" if H[i][j] == E[i][j] else "F"',
     'state = "F" if H[i][j] == F[i][j] else "E"'),
    ("full side matrix transposed", "full",
     "            if i >= 1:\n"
     "                F[i][j] = max(F[i - 1][j] - gap_extend, H[i - 1][j] - oe)\n"
     "            d = H[i - 1][j - 1] + int(matrix[x[i - 1], y[j - 1]])",
     "            if i >= 1:\n"
     "                F[i][j] = max(F[i - 1][j] - gap_extend, H[i - 1][j] - oe)\n"
     "            d = H[i - 1][j - 1] + int(matrix[y[j - 1], x[i - 1]])"),
    ("path score opens every gap move", "full", "s -= gap_extend + (gap_open if m != prev else 0)",
     "s -= gap_extend + (gap_open if m == prev else 0)"),
    ("identities and mismatches swapped", "full", "if a[pa] == b[pb]:", "if a[pa] != b[pb]:"),
    ("gap openings counted per move", "full", "            if m != prev:\n                opens += 1",
     "            if True:\n                opens += 1"),
    ("cover misses a piece's first position", "full", "d == p1 - p2 and f <= p1 < t", "d == p1 - p2 and f < p1 < t"),
    ("hits of a pair by increasing score", "full", "members.sort(key=lambda h: (-int(gscore[h]),",
     "members.sort(key=lambda h: (int(gscore[h]),"),
    ("codon TGA read as W", "translate", '_CODE_TCAG = "FFLLSSSSYY**CC*W', '_CODE_TCAG = "FFLLSSSSYY**CCWW'),
    ("reverse strand not reversed", "translate", "s = (3 - s)[::-1]", "s = (3 - s)"),
    ("frame offset", "translate", "s = s[frame % 3:]", "s = s[(frame + 1) % 3:]"),
    ("reverse frame coordinate", "translate", "return p if frame < 3 else dna_len - 1 - p",
     "return p if frame < 3 else dna_len - p"),
]

C_MUTANTS = [
    ("C ungapped right window short", "ungapped", "int64_t rmax = right;", "int64_t rmax = right - 1;"),
    ("C ungapped left window short", "ungapped", "for (int64_t t = 1; t <= lmax; ++t) {",
     "for (int64_t t = 1; t < lmax; ++t) {"),
    ("C ungapped matrix transposed", "ungapped", "s += mat[a[p1 + t] * 20 + b[p2 + t]];",
     "s += mat[b[p2 + t] * 20 + a[p1 + t]];"),
    ("C seed class split wrongly", "index", '"G", "IV", "ML",', '"G", "I", "VML",'),
    ("C index positions off by one", "index", "occ_pos[slot] = (int32_t)p;", "occ_pos[slot] = (int32_t)p + 1;"),
    ("C gapped band one too wide", "gapped", "if ((i > j ? i - j : j - i) > band) continue;",
     "if ((i > j ? i - j : j - i) > band + 1) continue;"),
    ("C gapped open without extend", "gapped",
     "<= band) {\n        int e1 = E[c - 1] - ext, e2 = H[c - 1] - open - ext;",
     "<= band) {\n        int e1 = E[c - 1] - ext, e2 = H[c - 1] - open;"),
    ("C full side prefers F over E", "full", "state = H[c] == E[c] ? 'E' : 'F';",
     "state = H[c] == F[c] ? 'F' : 'E';"),
    ("C full side last best cell", "full", "      if (h > best) {\n        best = h;",
     "      if (h >= best) {\n        best = h;"),
    ("C identities and mismatches swapped", "full", "if (a[pa] == b[pb]) st[0]++;", "if (a[pa] != b[pb]) st[0]++;"),
    ("C cover misses a piece's first position", "full", "pieces[q].first <= p1 && p1 < pieces[q].last",
     "pieces[q].first < p1 && p1 < pieces[q].last"),
    ("C hits of a pair by increasing score", "full",
     "return orc_sort_gscore[a] > orc_sort_gscore[b] ? -1 : 1;",
     "return orc_sort_gscore[a] < orc_sort_gscore[b] ? -1 : 1;"),
]


@pytest.fixture(scope="module")
def stage32_case(cfg0):
    h, _ = C.ungapped_hits(cfg0.bank1, cfg0.bank2, params.S1)
    g = C.gapped_scores(cfg0.bank1, cfg0.bank2, h)
    return cfg0, h, g, g >= params.S2


def _battery(cfg0, cfg0_random, stage32):
    """(stage, name, call) for every pin the mutants are run against."""
    part = functools.partial
    pins = [
        ("matrix", "blosum62 published facts", P.test_blosum62_shape_and_published_facts),
        ("matrix", "blosum62 lambda and entropy", P.test_blosum62_karlin_altschul_lambda_and_entropy),
        ("matrix", "blosum62 second transcription", P.test_blosum62_matches_generator_transcription),
        ("seed", "seed examples of the paper", P.test_seed_key_paper_examples),
        ("seed", "seed key image", P.test_seed_key_image_is_8800_and_partitions),
        ("ungapped", "matrix orientation", P.test_matrix_orientation_closed_forms),
        ("ungapped", "segment enumeration", P.test_score_equals_segment_enumeration),
        ("ungapped", "self hit", P.test_score_self_hit_closed_form),
        ("ungapped", "poly-A", P.test_poly_a_closed_form),
        ("gapped", "gapped path enumeration", P.test_gapped_side_equals_path_enumeration),
        ("gapped", "gapped without gaps", P.test_gapped_no_gaps_reduces_to_ungapped_prefix),
        ("gapped", "gapped poly-A and symmetry", P.test_gapped_poly_a_and_swap_symmetry),
        ("gapped", "matrix orientation", P.test_matrix_orientation_closed_forms),
        ("gapped", "gapped band edge", P.test_gapped_band_edge_closed_form),
        ("gapped", "gapped vectorised, C and scalar", part(P.test_gapped_vectorised_and_c_match_scalar, cfg0)),
        ("full", "full side enumeration", S.test_full_side_equals_exhaustive_enumeration),
        ("full", "full side hand example", S.test_full_side_hand_example_one_gap),
        ("full", "full side gap tie", S.test_full_side_hand_example_gap_tie),
        ("full", "full side closed forms", S.test_full_side_closed_forms),
        ("full", "full side is the unbanded stage 3.1 side", S.test_full_side_is_the_unbanded_unwindowed_stage31_side),
        ("full", "matrix orientation", P.test_matrix_orientation_closed_forms),
        ("full", "identical pair", S.test_stage32_identical_pair_closed_form),
        ("full", "records", part(S.test_stage32_records_are_consistent, stage32)),
        ("full", "cover relation", part(S.test_stage32_cover_relation, stage32)),
        ("full", "numpy and C stage 3.2", part(S.test_stage32_numpy_and_c_oracles_agree, stage32)),
        ("full", "numpy and C stage 3.2, tiny pairs", S.test_stage32_c_matches_python_on_tiny_random_pairs),
        ("translate", "codon table facts", P.test_codon_table_textbook_facts),
        ("translate", "codon table second transcription", P.test_codon_table_agrees_with_generator_transcription),
        ("translate", "six-frame hand example", P.test_translate6_hand_example),
        ("translate", "reverse translation round trip",
         part(P.test_reverse_translation_round_trip_and_frame_coordinates, 1)),
    ]
    pins += [("index", "index brute force %d" % s, part(P.test_index_csr_invariants_and_brute_force, s))
             for s in range(6)]
    pins += [("index", "extension count", P.test_n_extensions_equals_pair_count)]
    pins += [("ungapped", "hit list brute force %d" % s, part(P.test_hit_list_equals_all_diagonal_brute_force, s, t))
             for s, t in [(0, 15), (1, 25), (2, 4), (3, 38)]]
    pins += [("ungapped", "threshold 4 keeps every pair", part(P.test_threshold_at_most_4_keeps_every_candidate,
                                                               cfg0_random)),
             ("ungapped", "numpy and C on config 0", part(P.test_numpy_and_c_oracles_agree_on_config0, cfg0))]
    return pins


def _first_failure(stage, pins):
    for st, name, call in sorted(pins, key=lambda p: p[0] != stage):
        try:
            call()
        except Exception as e:  # a failing pin is what the case expects
            return "%s (%s)" % (name, type(e).__name__)
    return None


def _mutate(src, old, new):
    assert src.count(old) == 1, "mutation site must occur exactly once: %r" % old
    return src.replace(old, new)


@pytest.mark.parametrize("case,stage,old,new", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_python_oracle_mutant_is_caught(case, stage, old, new, monkeypatch, cfg0, cfg0_random, stage32_case):
    with open(PY_SRC) as f:
        src = _mutate(f.read(), old, new)
    mod = types.ModuleType("plast_oracle_mutant")
    mod.__file__ = PY_SRC
    exec(compile(src, PY_SRC, "exec"), mod.__dict__)
    monkeypatch.setattr(P, "O", mod)
    monkeypatch.setattr(S, "O", mod)
    caught = _first_failure(stage, _battery(cfg0, cfg0_random, stage32_case))
    assert caught is not None, "no pin catches: " + case


@pytest.mark.parametrize("case,stage,old,new", C_MUTANTS, ids=[m[0] for m in C_MUTANTS])
def test_c_oracle_mutant_is_caught(case, stage, old, new, monkeypatch, tmp_path, cfg0, cfg0_random, stage32_case):
    with open(C_SRC) as f:
        src = _mutate(f.read(), old, new)
    c_file = tmp_path / "mutant.c"
    c_file.write_text(src)
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-pthread", str(c_file), "-o", str(so)])
    monkeypatch.setattr(C, "_lib", C.declare(ctypes.CDLL(str(so))))
    caught = _first_failure(stage, _battery(cfg0, cfg0_random, stage32_case))
    assert caught is not None, "no pin catches: " + case


def test_unmutated_oracle_passes_the_battery(cfg0, cfg0_random, stage32_case):
    """The battery itself passes on the real oracle, so a failure above is the
    mutant's doing."""
    assert _first_failure("none", _battery(cfg0, cfg0_random, stage32_case)) is None
