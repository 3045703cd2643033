"""The measured denominators (plast_probe_peak) on the GPU: every probe runs
and reports a rate of the right order of magnitude against MI355X's published figures
(256 CUs at up to 2.4 GHz; 64 int32 or 128 packed 16-bit lane operations per
clock per CU; LDS: 32 lookups of 4 bytes, or 256 bytes of 8-byte reads (the
ungapped kernel's profile access), per clock per CU; 8 TB/s of HBM)."""
import sys

import pytest
import torch

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

PUBLISHED = {"valu_i32": 256 * 64 * 2.4e9, "valu_pk_i16": 256 * 128 * 2.4e9, "valu_pk_f16": 256 * 128 * 2.4e9,
             "lds_lookup": 256 * 32 * 2.4e9, "hbm_copy": 8e12, "lds_b64": 256 * 256 * 2.4e9, "sclk": 2.4e9}


def test_probes_report_plausible_peaks():
    from paper_0804_3643_amd import binding as B
    B.load()
    buf = B._alloc(1 << 30, torch.device("cuda:0"))
    for kind in B.PROBES:
        print("[gpu-test] probe %s" % kind, flush=True)
        sys.stdout.flush()
        rate = B.probe_peak(kind, buf, reps=2)
        frac = rate / PUBLISHED[kind]
        print("[gpu-test] probe %s: %.3g %s (%.2f of the published figure)" % (kind, rate, B.PROBES[kind][1], frac),
              flush=True)
        # right order of magnitude (the box may run above the published clock or issue faster)
        assert 0.2 < frac < 2.5, (kind, rate)
    with pytest.raises(B.PlastError) as e:
        B.probe_peak("hbm_copy", buf[: 1 << 19])
    assert e.value.code == B.E_WORKSPACE
