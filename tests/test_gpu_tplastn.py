"""TPLAST-N on the GPU: six-frame translation against the oracle's (fragments,
layout and fragment table byte for byte, edge cases and errors), and the
search of a protein bank against the translated fragments through the same
index / extension / gapped path, against the oracle; planted homologs come
back in their DNA sequence, frame and codon."""
import sys

import numpy as np
import pytest
import torch

from oracle import coracle as C
from oracle import plast_oracle as O
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


def _gpu_translate(B, dna):
    codes, starts, frag = B.translate(*B.dna_to_device(dna, "cuda"))
    return codes.cpu().numpy(), starts.cpu().numpy(), frag.cpu().numpy().astype(np.int64)


def _check_translation(B, dna):
    codes, starts, frag = _gpu_translate(B, dna)
    frags, table = O.translate6(dna.codes, dna.start)
    ref = synth.Bank.from_seqs(frags)
    assert np.array_equal(codes, ref.codes)
    assert np.array_equal(starts, ref.seq_start)
    assert np.array_equal(frag, table)
    return ref, table


def test_translation_edge_cases(B):
    _say("translation edge cases")
    seqs = ["", "A", "AC", "ATG", "ATGA", "TAATAGTGA", "TTTTT", "ATGGCCTAAGGG", "CATTAGCTA" * 7]
    lut = {c: i for i, c in enumerate("ACGT")}
    dna = synth.DnaBank.from_seqs([np.array([lut[c] for c in s], dtype=np.uint8) for s in seqs])
    _check_translation(B, dna)
    rng = np.random.default_rng(5)
    dna = synth.DnaBank.from_seqs([rng.integers(0, 4, size=int(n)).astype(np.uint8)
                                   for n in rng.integers(0, 3000, size=60)])
    _check_translation(B, dna)


def test_translation_rejects_bad_input(B):
    dna = synth.DnaBank.from_seqs([np.array([0, 1, 2, 3, 0, 1], dtype=np.uint8)] * 3)
    codes, start = B.dna_to_device(dna, "cuda")
    bad = codes.clone()
    bad[4] = 7
    with pytest.raises(B.PlastError) as e:
        B.translate(bad, start)
    assert e.value.code == B.E_ALPHABET
    bad_start = start.clone()
    bad_start[1] = 100
    with pytest.raises(B.PlastError) as e:
        B.translate(codes, bad_start)
    assert e.value.code == B.E_LAYOUT


def test_tplastn_search_matches_oracle_and_finds_plants(B):
    _say("tplastn small workload")
    w = synth.make_tplastn(scale=0.02, dna_len=(3000, 30000), n_plants=30)
    ref_bank, table = _check_translation(B, w.dna)
    codes, starts, frag = B.translate(*B.dna_to_device(w.dna, "cuda"))
    ia = B.build_index(*B.bank_to_device(w.bank1, "cuda"))
    ib = B.build_index(codes, starts)
    hits, n_ext = B.ungapped_extend(ia, ib, params.S1, mode="batched")
    ref, ref_ext = C.ungapped_hits(w.bank1, ref_bank, params.S1)
    assert n_ext == ref_ext and np.array_equal(B.canonical_hits(hits), ref)
    gs, ps = B.gapped_filter(ia, ib, hits, params.S2)
    h = hits.cpu().numpy().astype(np.int64)
    g_ref = C.gapped_scores(w.bank1, ref_bank, h)
    assert np.array_equal(gs.cpu().numpy().astype(np.int64), g_ref)
    # every planted homolog: a passing hit in its DNA sequence, on its strand, inside its coding region
    passing = h[ps.cpu().numpy().astype(bool)]
    found = 0
    for pl in w.plants:
        sel = passing[passing[:, 0] == pl.protein]
        for s1, p1, s2, p2, _ in sel:
            d, f, a0 = table[s2]
            if d != pl.dna or (f < 3) != (pl.strand > 0):
                continue
            L = int(w.dna.start[d + 1] - w.dna.start[d])
            nt = O.frame_position(L, int(f), int(a0 + p2))
            if pl.offset <= nt < pl.offset + 3 * pl.n_codons:
                found += 1
                break
    assert found >= 0.9 * len(w.plants), (found, len(w.plants))


def test_plastx_search_matches_oracle_and_finds_plants(B):
    """PLAST-X: both banks translated on the device (6 x 6 frame pairs through
    one search); hits and gapped scores equal the oracle's on the oracle's
    translations, and planted homologous coding regions are found."""
    _say("plastx small workload")
    w = synth.make_plastx(scale=0.05, dna_len=(3000, 20000), n_plants=20)
    ref1, t1 = _check_translation(B, w.dna1)
    ref2, t2 = _check_translation(B, w.dna2)
    c1, s1, _ = B.translate(*B.dna_to_device(w.dna1, "cuda"))
    c2, s2, _ = B.translate(*B.dna_to_device(w.dna2, "cuda"))
    ia, ib = B.build_index(c1, s1), B.build_index(c2, s2)
    hits, n_ext = B.ungapped_extend(ia, ib, params.S1, mode="batched")
    ref, ref_ext = C.ungapped_hits(ref1, ref2, params.S1)
    assert n_ext == ref_ext and np.array_equal(B.canonical_hits(hits), ref)
    gs, ps = B.gapped_filter(ia, ib, hits, params.S2)
    h = hits.cpu().numpy().astype(np.int64)
    assert np.array_equal(gs.cpu().numpy().astype(np.int64), C.gapped_scores(ref1, ref2, h))
    passing = h[ps.cpu().numpy().astype(bool)]
    L1 = np.diff(w.dna1.start)
    L2 = np.diff(w.dna2.start)
    found = 0
    for a, b in w.plants:
        for s1_, p1, s2_, p2, _ in passing:
            d1, f1, o1 = t1[s1_]
            d2, f2, o2 = t2[s2_]
            if d1 != a.dna or d2 != b.dna or (f1 < 3) != (a.strand > 0) or (f2 < 3) != (b.strand > 0):
                continue
            n1 = O.frame_position(int(L1[d1]), int(f1), int(o1 + p1))
            n2 = O.frame_position(int(L2[d2]), int(f2), int(o2 + p2))
            if a.offset <= n1 < a.offset + 3 * a.n_codons and b.offset <= n2 < b.offset + 3 * b.n_codons:
                found += 1
                break
    assert found >= 0.85 * len(w.plants), (found, len(w.plants))
