"""Full-size TPLAST-N (5,000 proteins against 2,000 DNA sequences of 50-200 kb)
and PLAST-X (200 against 1,000 DNA sequences of 20-50 kb, both translated) on
the GPU, against the oracle's full-size goldens: the device six-frame
translation equals the oracle's fragment bank and fragment table byte for byte
(SHA-256), and the whole hit list with every gapped score equals the oracle's
(count and 64-bit multiset digests, whole run and per block of 80 keys)."""
import os
import sys

import numpy as np
import pytest
import torch

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


def _translate_checked(B, dna, ref):
    """Device translation of a DNA bank, checked against the golden's SHA-256 of
    the oracle's fragment bank; returns the device tensors and the host bank."""
    codes, starts, frag = B.translate(*B.dna_to_device(dna, "cuda"))
    torch.cuda.synchronize()
    c, st, fr = codes.cpu().numpy(), starts.cpu().numpy(), frag.cpu().numpy()
    assert fr.shape == (ref["n"], 3)
    assert fullsize.sha256_arrays(c) == ref["codes_sha256"]
    assert fullsize.sha256_arrays(st.astype(np.int64)) == ref["seq_start_sha256"]
    assert fullsize.sha256_arrays(np.ascontiguousarray(fr, dtype=np.int32)) == ref["table_sha256"]
    return codes, starts, synth.Bank(c, st)


def _search_checked(B, golden, ca, sa, cb, sb, bank1):
    ia, ib = B.build_index(ca, sa), B.build_index(cb, sb)
    tuning = {"item_cols": [2048, 8192, 16384, 16384], "xcd_queues": 8, "gapped_threads": 512}
    hits, n_ext = B.ungapped_extend(ia, ib, params.S1, mode="batched", tuning=tuning)
    gs, _ = B.gapped_filter(ia, ib, hits, params.S2, tuning=tuning)
    _say("digest of %d hits" % hits.shape[0])
    got = fullsize.device_summary(hits, gs, params.S2, bank1, n_ext)
    assert fullsize.compare(golden, got) == [], fullsize.compare(golden, got)


@pytest.mark.timeout(600)
def test_tplastn_full_size_against_golden(B):
    golden = fullsize.load(3)
    assert golden is not None
    _say("tplastn generate")
    w = synth.make_tplastn()
    assert golden["bank_sha256"] == [w.bank1.sha256(), fullsize.sha256_arrays(w.dna.codes, w.dna.start)]
    _say("tplastn translate %d DNA sequences" % w.dna.n_seqs)
    cb, sb, _ = _translate_checked(B, w.dna, golden["fragments"][0])
    ca, sa = B.bank_to_device(w.bank1, "cuda")
    _say("tplastn search")
    _search_checked(B, golden, ca, sa, cb, sb, w.bank1)


@pytest.mark.timeout(600)
def test_plastx_full_size_against_golden(B):
    golden = fullsize.load("x")
    assert golden is not None
    _say("plastx generate")
    w = synth.make_plastx()
    assert golden["bank_sha256"] == [fullsize.sha256_arrays(w.dna1.codes, w.dna1.start),
                                     fullsize.sha256_arrays(w.dna2.codes, w.dna2.start)]
    _say("plastx translate both banks")
    ca, sa, bank1 = _translate_checked(B, w.dna1, golden["fragments"][0])
    cb, sb, _ = _translate_checked(B, w.dna2, golden["fragments"][1])
    _say("plastx search")
    _search_checked(B, golden, ca, sa, cb, sb, bank1)
