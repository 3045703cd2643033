"""The allocation-free ungapped entry point (plast_ungapped_extend_noalloc,
static device scratch) against plast_ungapped_extend (BATCHED, caller
workspace) and the oracle, through the C ABI: two calls in a row, the second on
a smaller input, then a work list too long for the scratch (rejected with
PLAST_E_WORKSPACE) followed by a call that works again."""
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


def _sorted(h):
    """Rows sorted lexicographically (seq1, pos1, seq2, pos2, score), int64."""
    h = h.cpu().numpy().astype(np.int64)
    return h[np.lexsort(h.T[::-1])] if len(h) else h


def _indexes(B, w):
    ia = B.build_index(*B.bank_to_device(w.bank1, "cuda"))
    ib = B.build_index(*B.bank_to_device(w.bank2, "cuda"))
    return ia, ib


@pytest.mark.timeout(300)
def test_noalloc_equals_workspace_entry_point_twice_then_smaller():
    from paper_0804_3643_amd import binding as B
    B.load()
    tuning = {"item_cols": [1024, 2048, 4096, 8192], "xcd_queues": 8}
    for name, w in (("cfg1 x0.1", synth.make_workload(1, scale=0.1)), ("cfg0", synth.make_workload(0))):
        _say("noalloc %s" % name)
        ia, ib = _indexes(B, w)
        _, n_ext_ws, n_items = B.ungapped_workspace_bytes(ia, ib, "batched", tuning=tuning)
        assert 0 < n_items * 16 < B.NOALLOC_SCRATCH_BYTES
        ref, n_ext_ref = B.ungapped_extend(ia, ib, params.S1, mode="batched", tuning=tuning)
        cap = ref.shape[0] + 4096
        out = torch.full((cap, 5), -7, dtype=torch.int32, device="cuda")
        got, n_ext = B.ungapped_extend_noalloc(ia, ib, params.S1, out, tuning=tuning)
        torch.cuda.synchronize()
        assert n_ext == n_ext_ref == n_ext_ws
        g, r = _sorted(got), _sorted(ref)
        assert np.array_equal(g, r), name
        assert (out[got.shape[0]:] == -7).all()                  # nothing written past the hits
        if name == "cfg0":                                        # and the oracle's canonical list
            o, n_o = C.ungapped_hits(w.bank1, w.bank2, params.S1)
            assert n_o == n_ext and np.array_equal(g, o)
        del ia, ib, ref, got, out


@pytest.mark.timeout(300)
def test_noalloc_rejects_a_work_list_beyond_the_scratch_then_recovers():
    from paper_0804_3643_amd import binding as B
    B.load()
    _say("noalloc rejection: cfg1 with 512-column items")
    w = synth.make_workload(1)
    ia, ib = _indexes(B, w)
    narrow = {"item_cols": [512, 512, 512, 512]}
    _, _, n_items = B.ungapped_workspace_bytes(ia, ib, "batched", tuning=narrow)
    assert n_items * 16 > B.NOALLOC_SCRATCH_BYTES
    out = torch.empty((1 << 20, 5), dtype=torch.int32, device="cuda")
    with pytest.raises(B.PlastError) as e:
        B.ungapped_extend_noalloc(ia, ib, params.S1, out, tuning=narrow)
    assert e.value.code == B.E_WORKSPACE and str(n_items) in str(e.value)
    _say("noalloc after the rejection: capacity retry contract, then the full list")
    wide = {"item_cols": [2048, 8192, 16384, 16384], "xcd_queues": 8}
    with pytest.raises(B.PlastError) as e:
        B.ungapped_extend_noalloc(ia, ib, params.S1, out[:1000], tuning=wide)
    assert e.value.code == B.E_CAPACITY
    ref, n_ext_ref = B.ungapped_extend(ia, ib, params.S1, mode="batched", tuning=wide)
    big = torch.empty((ref.shape[0] + 1024, 5), dtype=torch.int32, device="cuda")
    got, n_ext = B.ungapped_extend_noalloc(ia, ib, params.S1, big, tuning=wide)
    assert n_ext == n_ext_ref and got.shape[0] == ref.shape[0]
    assert np.array_equal(_sorted(got), _sorted(ref))
