"""CPU checks of the full-size goldens (tests/golden/fullsize.py): the multiset
digest sees every kind of slip a hit list can carry, the block-wise writer
equals the plain numpy oracle over a whole workload, and every stored golden
still describes the banks the seeded generator makes and the frozen
parameters."""
import json
import os
import sys

import numpy as np
import pytest

from oracle import plast_oracle as O
from paper_0804_3643_amd import params, synth

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import fullsize  # noqa: E402


@pytest.fixture(scope="module")
def cfg0_full():
    w = synth.make_workload(0)
    hits = O.ungapped_hits(w.bank1, w.bank2, params.S1)
    hits = hits[0] if isinstance(hits, tuple) else hits
    g = O.gapped_scores(w.bank1, w.bank2, hits)
    return w, np.asarray(hits, dtype=np.int64), np.asarray(g, dtype=np.int64)


def test_digest_is_order_free_and_sees_every_slip(cfg0_full):
    _, h, g = cfg0_full
    ref = fullsize.summary(h, g, params.S2)
    p = np.random.default_rng(3).permutation(len(h))
    assert fullsize.summary(h[p], g[p], params.S2) == ref
    # a changed field in any column of one record
    for col in range(5):
        h2 = h.copy()
        h2[17, col] += 1
        s = fullsize.summary(h2, g, params.S2)
        assert s["hits"] != ref["hits"] and s["hits_gscore"] != ref["hits_gscore"]
        assert s["hits"]["count"] == ref["hits"]["count"]
    g2 = g.copy()
    g2[17] -= 1
    s = fullsize.summary(h, g2, params.S2)
    assert s["hits"] == ref["hits"] and s["hits_gscore"] != ref["hits_gscore"]
    # a dropped record, a record reported twice, two records swapping scores
    assert fullsize.summary(h[1:], g[1:], params.S2)["hits"] != ref["hits"]
    twice = fullsize.summary(np.vstack([h, h[:1]]), np.concatenate([g, g[:1]]), params.S2)
    assert twice["hits"]["count"] == ref["hits"]["count"] + 1 and twice["hits"]["sum"] != ref["hits"]["sum"]
    h3 = h.copy()
    h3[[3, 4], 4] = h3[[4, 3], 4]
    if h3[3, 4] != h[3, 4]:
        assert fullsize.summary(h3, g, params.S2)["hits"] != ref["hits"]


def test_stored_cfg0_golden_equals_the_numpy_oracle(cfg0_full):
    """The writer (C oracle, one block of keys at a time) against the numpy
    oracle's whole canonical list: counts, digests and every block digest."""
    w, h, g = cfg0_full
    gold = fullsize.load(0)
    assert gold is not None and gold["bank_sha256"] == [w.bank1.sha256(), w.bank2.sha256()]
    got = fullsize.summary(h, g, params.S2, fullsize.seed_keys(w.bank1, h))
    got["n_ext"] = O.n_extensions(O.build_index(w.bank1), O.build_index(w.bank2))
    assert fullsize.compare(gold, got) == []
    assert sum(b[0] for b in gold["blocks"]) == gold["n_hits"] == len(h)


@pytest.mark.parametrize("cfg", ["1", "2", "3", "x"])
def test_stored_goldens_match_generator_and_parameters(cfg):
    gold = fullsize.load(cfg)
    assert gold is not None, "missing golden: python tests/golden/fullsize.py %s" % cfg
    th = json.load(open(os.path.join(HERE, "golden", "thresholds.json")))
    assert gold["params"] == {"S1": th["s1"], "S2": th["s2"], "nbr": params.NBR, "gap_window": params.GAP_WINDOW,
                              "gap_band": params.GAP_BAND, "gap_open": params.GAP_OPEN,
                              "gap_extend": params.GAP_EXTEND, "matrix": "BLOSUM62"}
    if cfg in ("1", "2"):
        w = synth.make_workload(int(cfg))
        assert gold["bank_sha256"] == [w.bank1.sha256(), w.bank2.sha256()]
    elif cfg == "3":
        w = synth.make_tplastn()
        assert gold["bank_sha256"] == [w.bank1.sha256(), fullsize.sha256_arrays(w.dna.codes, w.dna.start)]
    else:
        w = synth.make_plastx()
        assert gold["bank_sha256"] == [fullsize.sha256_arrays(w.dna1.codes, w.dna1.start),
                                       fullsize.sha256_arrays(w.dna2.codes, w.dna2.start)]
    assert len(gold["blocks"]) == fullsize.N_BLOCKS
    assert sum(b[0] for b in gold["blocks"]) == gold["n_hits"] == gold["hits"]["count"]
    assert gold["passing"]["count"] == gold["n_pass"] <= gold["n_hits"] <= gold["n_ext"]
