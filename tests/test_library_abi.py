"""CPU-side checks of the C ABI: the built library loads, exports every entry
point declared in include/plast.h, struct layouts agree with the binding, and
argument validation rejects bad calls before touching a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "plast.h")

binding = pytest.importorskip("paper_0804_3643_amd.binding")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(plast_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = _declared()
    assert set(names) == set(binding.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (plast_\w+)", out))
    assert set(names) <= exported


def test_struct_layouts_match_binding(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "plast.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\\n", sizeof(plast_index_t), offsetof(plast_index_t, n_words),
         offsetof(plast_index_t, scan_codes), sizeof(plast_ungapped_params_t), sizeof(plast_gapped_params_t));
  printf("%zu %d %d %d %d\\n", sizeof(plast_hit_t), PLAST_NKEYS, PLAST_PAD_CODE, PLAST_PAD_LEN, PLAST_NBR);
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(plast_tuning_t), offsetof(plast_tuning_t, xcd_queues),
         sizeof(plast_tune_report_t), offsetof(plast_tune_report_t, class_ms),
         offsetof(plast_tune_report_t, queue_ms), offsetof(plast_tune_report_t, gapped_ms), sizeof(plast_bank_t),
         offsetof(plast_bank_t, n_padded), sizeof(plast_pipeline_result_t),
         offsetof(plast_pipeline_result_t, n_words_b));
  printf("%zu %zu %d %d %zu\\n", offsetof(plast_ungapped_params_t, tuning), offsetof(plast_gapped_params_t, tuning),
         PLAST_TUNE_CLASSES, PLAST_TUNE_WIDTHS, sizeof(plast_match_t));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I" + os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    a, b, c, d = subprocess.check_output([str(exe)], text=True).strip().splitlines()
    a, b, c, d = ([int(x) for x in line.split()] for line in (a, b, c, d))
    T, R, BD, PR = binding.Tuning, binding.TuneReport, binding.BankDesc, binding.PipelineResult
    assert c == [ctypes.sizeof(T), T.xcd_queues.offset, ctypes.sizeof(R), R.class_ms.offset, R.queue_ms.offset,
                 R.gapped_ms.offset, ctypes.sizeof(BD), BD.n_padded.offset, ctypes.sizeof(PR), PR.n_words_b.offset]
    assert d == [binding.UngappedParams.tuning.offset, binding.GappedParams.tuning.offset, binding.TUNE_CLASSES,
                 len(binding.TUNE_WIDTHS), ctypes.sizeof(binding.MatchRec)]
    assert a == [ctypes.sizeof(binding.IndexView), binding.IndexView.n_words.offset,
                 binding.IndexView.scan_codes.offset, ctypes.sizeof(binding.UngappedParams),
                 ctypes.sizeof(binding.GappedParams)]
    assert b == [20, binding.NKEYS, binding.PAD_CODE, binding.PAD_LEN, binding.NBR]


def test_strerror_and_argument_validation_without_gpu():
    lib = binding.load()
    assert lib.plast_strerror(0) == b"ok"
    assert lib.plast_strerror(binding.E_CAPACITY) == b"hit buffer too small"
    ib, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.plast_index_bytes(10, 1, ctypes.byref(ib), ctypes.byref(wb)) == binding.E_ARG
    assert lib.plast_index_bytes(100, -1, ctypes.byref(ib), ctypes.byref(wb)) == binding.E_ARG
    assert lib.plast_index_bytes(1 << 31, 5, ctypes.byref(ib), ctypes.byref(wb)) == binding.E_ARG
    assert lib.plast_index_bytes(1000, 5, ctypes.byref(ib), ctypes.byref(wb)) == binding.OK
    # the sort keeps a 64-bit entry for each of up to n_padded - 20 words
    assert ib.value > 8 * 1000 and wb.value >= 8 * (1000 - 20)
    view = binding.IndexView()
    assert lib.plast_build_index(None, None, 0, 20, None, 0, None, 0, ctypes.byref(view), None) == binding.E_ARG
    assert b"null" in lib.plast_last_error()
    # fake device pointers are never dereferenced: validation fails first
    fake = ctypes.c_void_p(0x1000)
    assert lib.plast_build_index(fake, fake, 1, 1000, fake, 1, fake, 1, ctypes.byref(view), None) == \
        binding.E_WORKSPACE
    p = binding.UngappedParams(binding.NBR, 38, None, None)
    n = ctypes.c_int64(0)
    assert lib.plast_ungapped_extend(None, None, ctypes.byref(p), 1, fake, 256, fake, 10, ctypes.byref(n), None,
                                     None) == binding.E_ARG
    v = binding.IndexView(fake.value, fake.value, 1, 1000, fake.value, fake.value, fake.value, fake.value, 10)
    p_bad = binding.UngappedParams(7, 38, None, None)
    assert lib.plast_ungapped_extend(ctypes.byref(v), ctypes.byref(v), ctypes.byref(p_bad), 1, fake, 256, fake, 10,
                                     ctypes.byref(n), None, None) == binding.E_ARG
    assert lib.plast_ungapped_extend(ctypes.byref(v), ctypes.byref(v), ctypes.byref(p), 7, fake, 256, fake, 10,
                                     ctypes.byref(n), None, None) == binding.E_ARG
    g = binding.GappedParams(0, 16, 11, 1, 48, None, None)
    assert lib.plast_gapped_filter(ctypes.byref(v), ctypes.byref(v), fake, 5, ctypes.byref(g), fake, fake,
                                   None) == binding.E_ARG
    g = binding.GappedParams(64, 17, 11, 1, 48, None, None)
    assert lib.plast_gapped_filter(ctypes.byref(v), ctypes.byref(v), fake, 5, ctypes.byref(g), fake, fake,
                                   None) == binding.E_ARG
    g = binding.GappedParams(64, 16, 11, 1, 48, None, None)
    assert lib.plast_gapped_filter(ctypes.byref(v), ctypes.byref(v), fake, 0, ctypes.byref(g), fake, fake,
                                   None) == binding.OK


def test_tuning_validation_without_gpu():
    lib = binding.load()
    t = binding.tuning_default()
    assert list(t.class_min_n2) == [1, 2048, 8192, 32768] and list(t.item_cols) == [4096] * 4
    assert (t.xcd_queues, t.gapped_threads) == (1, 256)
    fake = ctypes.c_void_p(0x1000)
    v = binding.IndexView(fake.value, fake.value, 1, 1000, fake.value, fake.value, fake.value, fake.value, 10)
    n = ctypes.c_int64(0)

    def extend_rc(tun):
        p = binding.UngappedParams(binding.NBR, 38, None, ctypes.addressof(tun))
        return lib.plast_ungapped_extend(ctypes.byref(v), ctypes.byref(v), ctypes.byref(p), 1, fake, 256, fake, 10,
                                         ctypes.byref(n), None, None)

    for field, value in (("item_cols", [4096, 1000, 4096, 4096]), ("item_cols", [4096, 4096, 4096, 32768]),
                         ("class_min_n2", [0, 2048, 8192, 32768]), ("class_min_n2", [1, 2048, 2048, 32768]),
                         ("xcd_queues", 4), ("gapped_threads", 64)):
        bad = binding.Tuning.from_dict(t.as_dict())
        if isinstance(value, list):
            getattr(bad, field)[:] = value
        else:
            setattr(bad, field, value)
        assert extend_rc(bad) == binding.E_ARG, (field, value)
        assert b"tuning" in lib.plast_last_error()
    g = binding.GappedParams(64, 16, 11, 1, 48, None, None)
    bad = binding.Tuning.from_dict({"gapped_threads": 100})
    g.tuning = ctypes.addressof(bad)
    assert lib.plast_gapped_filter(ctypes.byref(v), ctypes.byref(v), fake, 5, ctypes.byref(g), fake, fake,
                                   None) == binding.E_ARG


def test_autotune_and_pipeline_validation_without_gpu():
    lib = binding.load()
    fake = ctypes.c_void_p(0x1000)
    v = binding.IndexView(fake.value, fake.value, 1, 1000, fake.value, fake.value, fake.value, fake.value, 10)
    u = binding.UngappedParams(binding.NBR, 38, None, None)
    g = binding.GappedParams(64, 16, 11, 1, 48, None, None)
    out, rep = binding.Tuning(), binding.TuneReport()
    for reps in (0, 21):
        assert lib.plast_autotune(ctypes.byref(v), ctypes.byref(v), ctypes.byref(u), ctypes.byref(g), reps, fake,
                                  1 << 20, fake, 10, fake, fake, ctypes.byref(out), ctypes.byref(rep),
                                  None) == binding.E_ARG
    a = binding.BankDesc(fake.value, fake.value, 3, 1000)
    b = binding.BankDesc(fake.value, fake.value, 30, 100000)
    sz0, sz1 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.plast_pipeline_workspace_bytes(ctypes.byref(a), ctypes.byref(b), 0, ctypes.byref(sz0)) == binding.OK
    assert lib.plast_pipeline_workspace_bytes(ctypes.byref(a), ctypes.byref(b), 1000, ctypes.byref(sz1)) == \
        binding.OK
    ia, wa = binding.index_bytes(1000, 3)
    ib, wb = binding.index_bytes(100000, 30)
    assert sz0.value >= ia + ib + max(wa, wb) and sz1.value - sz0.value >= 16 * 1000
    assert lib.plast_pipeline_workspace_bytes(ctypes.byref(a), ctypes.byref(b), -1, ctypes.byref(sz0)) == \
        binding.E_ARG
    bad = binding.BankDesc(fake.value, fake.value, 3, 10)  # shorter than one separator run
    assert lib.plast_pipeline_workspace_bytes(ctypes.byref(bad), ctypes.byref(b), 0, ctypes.byref(sz0)) == \
        binding.E_ARG
    h = ctypes.c_void_p(0)
    odd = ctypes.c_void_p(0x1010)
    assert lib.plast_pipeline_create(ctypes.byref(a), ctypes.byref(b), ctypes.byref(u), ctypes.byref(g), 10, odd,
                                     1 << 30, fake, 10, fake, fake, ctypes.byref(h)) == binding.E_ARG  # misaligned
    ws = ctypes.c_void_p(0x10000)
    assert lib.plast_pipeline_create(ctypes.byref(a), ctypes.byref(b), ctypes.byref(u), ctypes.byref(g), 10, ws,
                                     256, fake, 10, fake, fake, ctypes.byref(h)) == binding.E_WORKSPACE
    assert lib.plast_pipeline_launch(None, None) == binding.E_ARG
    assert lib.plast_pipeline_destroy(None) == binding.OK
    # query search against a resident index; the size query needs no pointers
    sizes_only = binding.BankDesc(0, 0, 3, 1000)
    assert lib.plast_search_workspace_bytes(ctypes.byref(sizes_only), 0, ctypes.byref(sz0)) == binding.OK
    assert lib.plast_pipeline_workspace_bytes(ctypes.byref(sizes_only), ctypes.byref(sizes_only), 0,
                                              ctypes.byref(sz1)) == binding.OK
    assert lib.plast_search_workspace_bytes(ctypes.byref(a), 0, ctypes.byref(sz0)) == binding.OK
    assert lib.plast_search_workspace_bytes(ctypes.byref(a), 1000, ctypes.byref(sz1)) == binding.OK
    assert sz0.value >= ia + wa and sz1.value - sz0.value >= 16 * 1000
    assert lib.plast_search_enqueue(ctypes.byref(a), ctypes.byref(v), ctypes.byref(u), ctypes.byref(g), 10, odd,
                                    1 << 30, fake, 10, fake, fake, None, None, 0, None, None) == binding.E_ARG  # misaligned
    assert lib.plast_search_enqueue(ctypes.byref(a), ctypes.byref(v), ctypes.byref(u), ctypes.byref(g), 10, ws,
                                    256, fake, 10, fake, fake, None, None, 0, None, None) == binding.E_WORKSPACE
    assert lib.plast_search_enqueue(ctypes.byref(a), None, ctypes.byref(u), ctypes.byref(g), 10, ws,
                                    1 << 30, fake, 10, fake, fake, None, None, 0, None, None) == binding.E_ARG
    # segments need the match buffer, the offsets and a sane count
    assert lib.plast_search_enqueue(ctypes.byref(a), ctypes.byref(v), ctypes.byref(u), ctypes.byref(g), 10, ws,
                                    1 << 30, fake, 10, fake, fake, None, fake, 2, fake, None) == binding.E_ARG
    assert lib.plast_search_enqueue(ctypes.byref(a), ctypes.byref(v), ctypes.byref(u), ctypes.byref(g), 10, ws,
                                    1 << 30, fake, 10, fake, fake, fake, fake, 5, fake, None) == binding.E_ARG
    assert lib.plast_search_result(None, ctypes.byref(binding.PipelineResult()), None, None) == binding.E_ARG


def test_product_code_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_0804_3643_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", src, re.M), f
                assert "plast_oracle" not in src and "coracle" not in src, f


def test_translate_validation_without_gpu():
    lib = binding.load()
    sz = ctypes.c_size_t(0)
    assert lib.plast_translate_ws_bytes(10, ctypes.byref(sz)) == binding.OK and sz.value >= 256 + 2 * 8 * 61
    assert lib.plast_translate_ws_bytes(-1, ctypes.byref(sz)) == binding.E_ARG
    fake, odd = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1010)
    nf, npad = ctypes.c_int64(0), ctypes.c_int64(0)
    assert lib.plast_translate_count(fake, None, 10, 100, fake, 1 << 20, ctypes.byref(nf), ctypes.byref(npad),
                                     None) == binding.E_ARG
    assert lib.plast_translate_count(fake, fake, 10, 100, odd, 1 << 20, ctypes.byref(nf), ctypes.byref(npad),
                                     None) == binding.E_ARG
    assert lib.plast_translate_count(fake, fake, 10, 100, fake, 16, ctypes.byref(nf), ctypes.byref(npad),
                                     None) == binding.E_WORKSPACE
    assert lib.plast_translate_write(fake, fake, 10, 100, fake, 1 << 20, fake, 10, fake, fake, 5,
                                     None) == binding.E_ARG   # n_padded too small for 5 fragments


def test_align_layout_and_validation_without_gpu(tmp_path):
    prog = tmp_path / "alayout.c"
    prog.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "plast.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(plast_alignment_t), offsetof(plast_alignment_t, score),
         offsetof(plast_alignment_t, hit), sizeof(plast_align_params_t), offsetof(plast_align_params_t, matrix),
         sizeof(plast_timing_t), offsetof(plast_timing_t, align_ms));
  return 0;
}
""")
    exe = tmp_path / "alayout"
    subprocess.check_call(["gcc", "-std=c99", "-I" + os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)], text=True).split()]
    AP = binding.AlignParams
    nf = len(binding.ALIGN_FIELDS)
    assert got == [4 * nf, 4 * binding.ALIGN_FIELDS.index("score"), 4 * binding.ALIGN_FIELDS.index("hit"),
                   ctypes.sizeof(AP), AP.matrix.offset, ctypes.sizeof(binding.Timing), binding.Timing.align_ms.offset]

    lib = binding.load()
    sz = ctypes.c_size_t(0)
    ok = binding.AlignParams(11, 1, 1000, 1000, 64, 4096, None)
    assert lib.plast_align_workspace_bytes(1000, ctypes.byref(ok), ctypes.byref(sz)) == binding.OK
    # per wavefront: 16 strips x 133 dwords of 8 steps x 64 lanes of trace, 4096 pieces of 16 bytes
    assert sz.value >= 64 * (16 * 133 * 64 * 4 + 4096 * 16)
    # the longest sequences allowed still fit the LDS of one workgroup
    big = binding.AlignParams(11, 1, 16384, 16384, 64, 4096, None)
    assert lib.plast_align_workspace_bytes(10, ctypes.byref(big), ctypes.byref(sz)) == binding.OK
    for bad in (binding.AlignParams(11, 0, 1000, 1000, 64, 4096, None),        # extend < 1
                binding.AlignParams(11, 1, 0, 1000, 64, 4096, None),           # max_len1 < 1
                binding.AlignParams(11, 1, 1000, 20000, 64, 4096, None),       # max_len2 > 16384
                binding.AlignParams(11, 1, 1000, 1000, 64, 8, None)):          # max_pieces < 16
        assert lib.plast_align_workspace_bytes(1000, ctypes.byref(bad), ctypes.byref(sz)) == binding.E_ARG
    assert lib.plast_align_workspace_bytes(-1, ctypes.byref(ok), ctypes.byref(sz)) == binding.E_ARG
    n_out = ctypes.c_int64(5)
    iv = binding.IndexView()
    assert lib.plast_align(ctypes.byref(iv), ctypes.byref(iv), None, None, None, 10, ctypes.byref(ok), None, 0,
                           None, None, ctypes.byref(n_out), None) == binding.E_ARG


def test_probe_validation_without_gpu():
    """plast_probe_peak rejects bad arguments before any HIP call."""
    lib = binding.load()
    rate = ctypes.c_double(0.0)
    fake = ctypes.c_void_p(0x1000)
    assert lib.plast_probe_peak(0, None, 1 << 30, 3, ctypes.byref(rate), None) == binding.E_ARG
    assert lib.plast_probe_peak(0, fake, 1 << 30, 3, None, None) == binding.E_ARG
    assert lib.plast_probe_peak(7, fake, 1 << 30, 3, ctypes.byref(rate), None) == binding.E_ARG
    assert lib.plast_probe_peak(-1, fake, 1 << 30, 3, ctypes.byref(rate), None) == binding.E_ARG
    assert lib.plast_probe_peak(0, fake, 1 << 30, 0, ctypes.byref(rate), None) == binding.E_ARG
    assert lib.plast_probe_peak(0, ctypes.c_void_p(0x1001), 1 << 30, 3, ctypes.byref(rate), None) == binding.E_ARG
    assert lib.plast_probe_peak(0, fake, 1 << 20, 3, ctypes.byref(rate), None) == binding.E_WORKSPACE
    assert lib.plast_probe_peak(4, fake, 1 << 19, 3, ctypes.byref(rate), None) == binding.E_WORKSPACE
    assert b"probe" in lib.plast_last_error()
    assert set(binding.PROBES) == {"valu_i32", "valu_pk_i16", "valu_pk_f16", "lds_lookup", "hbm_copy", "lds_b64",
                                   "sclk"}
    # the clock probe needs 32 KiB for its counters beyond the 2 MiB of the compute probes
    assert lib.plast_probe_peak(6, fake, 2 << 20, 3, ctypes.byref(rate), None) == binding.E_WORKSPACE
