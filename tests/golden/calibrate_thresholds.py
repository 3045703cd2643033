"""Freeze the thresholds S1 and S2 (the paper gives no values) — calls only the oracle.

S1: the smallest integer whose pass rate over all candidate pairs of the
    configuration-0 banks without planted homologs is <= 0.186%, the stage-2
    selectivity the paper reports for its unoptimised and SIMD versions
    (Sec. 4.4.3 selectivity table).
S2: the smallest integer such that at most 10% of those S1 survivors pass the
    small gapped filter, following the paper's remark that about 90% of small
    gapped alignments do not go on to the full gapped stage (Sec. 3.3.4).

Writes thresholds.json next to this file.  Run: python tests/golden/calibrate_thresholds.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import coracle  # noqa: E402
from paper_0804_3643_amd import synth  # noqa: E402

SELECTIVITY = 0.00186
GAPPED_PASS = 0.10


def calibrate():
    w = synth.make_workload(0, plants=False)
    allpairs, n_ext = coracle.ungapped_hits(w.bank1, w.bank2, -10**6)
    sc = allpairs[:, 4]
    s1 = next(s for s in range(int(sc.min()), int(sc.max()) + 2) if (sc >= s).mean() <= SELECTIVITY)
    surv = allpairs[sc >= s1]
    g = coracle.gapped_scores(w.bank1, w.bank2, surv)
    s2 = next(s for s in range(int(g.min()), int(g.max()) + 2) if (g >= s).mean() <= GAPPED_PASS)
    return {"s1": int(s1), "s2": int(s2), "n_ext": int(n_ext), "s1_pass_rate": float((sc >= s1).mean()),
            "s2_pass_rate": float((g >= s2).mean()), "n_survivors": int(len(surv))}


if __name__ == "__main__":
    res = calibrate()
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "thresholds.json"), "w") as f:
        json.dump(res, f, indent=1)
    print(res)
