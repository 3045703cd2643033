// C ABI entry points, argument validation, error reporting and the library's
// tables (BLOSUM62 and the subset-seed classes).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "plast_internal.h"

namespace plast {

const char kNcbiOrder[21] = "ARNDCQEGHILKMFPSTWYV";

// BLOSUM62, Henikoff & Henikoff (1992), NCBI row/column order.
const int8_t kBlosum62Ncbi[20][20] = {
    /* A */ {4, -1, -2, -2, 0, -1, -1, 0, -2, -1, -1, -1, -1, -2, -1, 1, 0, -3, -2, 0},
    /* R */ {-1, 5, 0, -2, -3, 1, 0, -2, 0, -3, -2, 2, -1, -3, -2, -1, -1, -3, -2, -3},
    /* N */ {-2, 0, 6, 1, -3, 0, 0, 0, 1, -3, -3, 0, -2, -3, -2, 1, 0, -4, -2, -3},
    /* D */ {-2, -2, 1, 6, -3, 0, 2, -1, -1, -3, -4, -1, -3, -3, -1, 0, -1, -4, -3, -3},
    /* C */ {0, -3, -3, -3, 9, -3, -4, -3, -3, -1, -1, -3, -1, -2, -3, -1, -1, -2, -2, -1},
    /* Q */ {-1, 1, 0, 0, -3, 5, 2, -2, 0, -3, -2, 1, 0, -3, -1, 0, -1, -2, -1, -2},
    /* E */ {-1, 0, 0, 2, -4, 2, 5, -2, 0, -3, -3, 1, -2, -3, -1, 0, -1, -3, -2, -2},
    /* G */ {0, -2, 0, -1, -3, -2, -2, 6, -2, -4, -4, -2, -3, -3, -2, 0, -2, -2, -3, -3},
    /* H */ {-2, 0, 1, -1, -3, 0, 0, -2, 8, -3, -3, -1, -2, -1, -2, -1, -2, -2, 2, -3},
    /* I */ {-1, -3, -3, -3, -1, -3, -3, -4, -3, 4, 2, -3, 1, 0, -3, -2, -1, -3, -1, 3},
    /* L */ {-1, -2, -3, -4, -1, -2, -3, -4, -3, 2, 4, -2, 2, 0, -3, -2, -1, -2, -1, 1},
    /* K */ {-1, 2, 0, -1, -3, 1, 1, -2, -1, -3, -2, 5, -1, -3, -1, 0, -1, -3, -2, -2},
    /* M */ {-1, -1, -2, -3, -1, 0, -2, -3, -2, 1, 2, -1, 5, 0, -2, -1, -1, -1, -1, 1},
    /* F */ {-2, -3, -3, -3, -2, -3, -3, -3, -1, 0, 0, -3, 0, 6, -4, -2, -2, 1, 3, -1},
    /* P */ {-1, -2, -2, -1, -3, -1, -1, -2, -2, -3, -3, -1, -2, -4, 7, -1, -1, -4, -3, -2},
    /* S */ {1, -1, 1, 0, -1, 0, 0, 0, -1, -2, -2, 0, -1, -2, -1, 4, 1, -3, -2, -2},
    /* T */ {0, -1, 0, -1, -1, -1, -1, -2, -2, -1, -1, -1, -1, -2, -1, 1, 5, -2, -2, 0},
    /* W */ {-3, -3, -4, -4, -2, -2, -3, -2, -2, -3, -2, -3, -1, 1, -4, -3, -2, 11, 2, -3},
    /* Y */ {-2, -2, -2, -3, -2, -1, -2, -3, 2, -1, -1, -2, -1, 3, -3, -2, -2, 2, 7, -1},
    /* V */ {0, -3, -3, -3, -1, -2, -2, -3, -3, 3, 1, -2, 1, -1, -2, -2, 0, -3, -1, 4},
};

static const char kCodeOrder[] = "ACDEFGHIKLMNPQRSTVWY";

static int code_of(char c) {
  for (int i = 0; i < 20; ++i)
    if (kCodeOrder[i] == c) return i;
  return -1;
}

void blosum62_code_order(int8_t* m) {
  for (int r = 0; r < 20; ++r)
    for (int c = 0; c < 20; ++c) m[code_of(kNcbiOrder[r]) * 20 + code_of(kNcbiOrder[c])] = kBlosum62Ncbi[r][c];
}

SeedClasses seed_classes() {
  // Sec. 3.3.1 subset seed: position 2 classes c and g, position 3 classes
  // A, C, f, G, i, m, n, P, q, r, t (ids in that order).
  static const char* pos2_g = "GPATSNHQEDRK";
  static const char* pos3[11] = {"A", "C", "FYW", "G", "IV", "ML", "NH", "P", "QED", "RK", "TS"};
  SeedClasses sc{0u, 0ull, 0ull};
  for (const char* p = pos2_g; *p; ++p) sc.pos2_g_mask |= 1u << code_of(*p);
  for (int k = 0; k < 11; ++k)
    for (const char* p = pos3[k]; *p; ++p) {
      int c = code_of(*p);
      if (c < 16)
        sc.pos3_lo |= (uint64_t)k << (4 * c);
      else
        sc.pos3_hi |= (uint64_t)k << (4 * (c - 16));
    }
  return sc;
}

static thread_local char g_last_error[512] = "";

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return code;
}

int hip_check(hipError_t e, const char* what) {
  return set_error(PLAST_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------- timing
static bool g_timing = false;
static hipEvent_t g_ev[kNumStages][2];
static bool g_ev_made = false;
static bool g_ev_used[kNumStages];
static int64_t g_launches = 0;

bool timing_on() { return g_timing; }

void timing_mark(TimedStage st, bool stop, hipStream_t s) {
  if (!g_timing) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;  // not inside a graph
  if (hipEventRecord(g_ev[st][stop ? 1 : 0], s) == hipSuccess && stop) g_ev_used[st] = true;
}

void timing_launches(int64_t n) { g_launches = n; }

}  // namespace plast

using namespace plast;

extern "C" {

const char* plast_strerror(int code) {
  switch (code) {
    case PLAST_OK: return "ok";
    case PLAST_E_ARG: return "invalid argument";
    case PLAST_E_ALPHABET: return "residue code outside 0..19 or separator code not 20";
    case PLAST_E_CAPACITY: return "hit buffer too small";
    case PLAST_E_WORKSPACE: return "workspace or index buffer too small";
    case PLAST_E_HIP: return "HIP runtime error";
    case PLAST_E_LAYOUT: return "sequence offsets do not describe a padded bank";
    default: return "unknown error";
  }
}

const char* plast_last_error(void) { return g_last_error; }

int plast_timing_enable(int on) {
  g_last_error[0] = 0;
  if (on && !g_ev_made) {
    for (int i = 0; i < kNumStages; ++i)
      for (int j = 0; j < 2; ++j) PLAST_HIP(hipEventCreate(&g_ev[i][j]));
    g_ev_made = true;
  }
  g_timing = on != 0;
  for (int i = 0; i < kNumStages; ++i) g_ev_used[i] = false;
  return PLAST_OK;
}

int plast_timing_read(plast_timing_t* out) {
  g_last_error[0] = 0;
  if (!out) return set_error(PLAST_E_ARG, "null output pointer");
  float ms[kNumStages] = {};
  for (int i = 0; i < kNumStages; ++i) {
    if (!g_ev_made || !g_ev_used[i]) continue;
    PLAST_HIP(hipEventSynchronize(g_ev[i][1]));
    PLAST_HIP(hipEventElapsedTime(&ms[i], g_ev[i][0], g_ev[i][1]));
  }
  out->index_ms = ms[kStageIndex];
  out->plan_ms = ms[kStagePlan];
  out->ungapped_ms = ms[kStageUngapped];
  out->gapped_ms = ms[kStageGapped];
  out->ungapped_launches = g_launches;
  out->align_ms = ms[kStageAlign];
  return PLAST_OK;
}

int plast_index_bytes(int64_t n_padded, int32_t n_seqs, size_t* index_bytes, size_t* ws_bytes) {
  if (!index_bytes || !ws_bytes) return set_error(PLAST_E_ARG, "null output pointer");
  if (n_seqs < 0 || n_padded < kPadLen || n_padded > (int64_t)INT32_MAX - 2 * kScanSlack)
    return set_error(PLAST_E_ARG, "bad sizes n_padded=%lld n_seqs=%d", (long long)n_padded, n_seqs);
  *index_bytes = index_layout(n_padded).total;
  *ws_bytes = index_ws_bytes(n_padded);
  return PLAST_OK;
}

int plast_build_index(const uint8_t* d_codes, const int64_t* d_seq_start, int32_t n_seqs, int64_t n_padded,
                      void* d_index, size_t index_bytes, void* d_ws, size_t ws_bytes, plast_index_t* out,
                      void* stream) {
  g_last_error[0] = 0;
  if (!d_codes || !d_seq_start || !d_index || !d_ws || !out) return set_error(PLAST_E_ARG, "null pointer");
  size_t need_idx = 0, need_ws = 0;
  int rc = plast_index_bytes(n_padded, n_seqs, &need_idx, &need_ws);
  if (rc != PLAST_OK) return rc;
  if (index_bytes < need_idx || ws_bytes < need_ws)
    return set_error(PLAST_E_WORKSPACE, "index buffer %zu < %zu or workspace %zu < %zu", index_bytes, need_idx,
                     ws_bytes, need_ws);
  if (((uintptr_t)d_index & 255) || ((uintptr_t)d_ws & 255))
    return set_error(PLAST_E_ARG, "index and workspace buffers must be 256-byte aligned");
  return build_index_impl(d_codes, d_seq_start, n_seqs, n_padded, d_index, d_ws, out, (hipStream_t)stream);
}

static int check_index(const plast_index_t* x, const char* name) {
  if (!x) return set_error(PLAST_E_ARG, "%s: null index", name);
  if (!x->codes || !x->seq_start || !x->key_off || !x->occ || !x->occ_seq || !x->scan_codes || x->n_seqs < 0 ||
      x->n_words < 0 || x->n_padded < kPadLen)
    return set_error(PLAST_E_ARG, "%s: index view is incomplete (not from plast_build_index?)", name);
  return PLAST_OK;
}

static int tuning_or_default(const plast_tuning_t* t, plast_tuning_t* out) {
  if (!t) {
    tuning_default(out);
    return PLAST_OK;
  }
  *out = *t;
  return check_tuning(out);
}

int plast_tuning_default(plast_tuning_t* out) {
  g_last_error[0] = 0;
  if (!out) return set_error(PLAST_E_ARG, "null output pointer");
  tuning_default(out);
  return PLAST_OK;
}

int plast_ungapped_workspace_bytes(const plast_index_t* a, const plast_index_t* b, int32_t mode,
                                   const plast_tuning_t* tuning, size_t* bytes, int64_t* n_ext, int64_t* n_items,
                                   void* stream) {
  g_last_error[0] = 0;
  int rc;
  if ((rc = check_index(a, "a")) || (rc = check_index(b, "b"))) return rc;
  if (!bytes) return set_error(PLAST_E_ARG, "null output pointer");
  if (mode != PLAST_PLAIN && mode != PLAST_BATCHED) return set_error(PLAST_E_ARG, "unknown mode %d", mode);
  plast_tuning_t t;
  if ((rc = tuning_or_default(tuning, &t))) return rc;
  return ungapped_ws_bytes_impl(a, b, mode, t, bytes, n_ext, n_items, (hipStream_t)stream);
}

static int check_uparams(const plast_ungapped_params_t* p) {
  if (!p) return set_error(PLAST_E_ARG, "null ungapped parameters");
  if (p->nbr != kNbr) return set_error(PLAST_E_ARG, "nbr=%d unsupported (only %d)", p->nbr, kNbr);
  plast_tuning_t t;
  return tuning_or_default(p->tuning, &t);
}

static int check_gparams(const plast_gapped_params_t* g) {
  if (!g) return set_error(PLAST_E_ARG, "null gapped parameters");
  if (g->window < 1 || g->window > 64 || g->band < 0 || g->band > 16 || g->gap_open < 0 || g->gap_extend < 0 ||
      g->gap_open + g->gap_extend > 1000)
    return set_error(PLAST_E_ARG, "gapped parameters out of range (window 1..64, band 0..16, costs >= 0)");
  plast_tuning_t t;
  return tuning_or_default(g->tuning, &t);
}

// Sizes only (workspace queries); check_bank also wants the device pointers.
static int check_bank_sizes(const plast_bank_t* x, const char* name) {
  if (!x) return set_error(PLAST_E_ARG, "%s: null bank", name);
  size_t ib = 0, wb = 0;
  return plast_index_bytes(x->n_padded, x->n_seqs, &ib, &wb);
}

static int check_bank(const plast_bank_t* x, const char* name) {
  if (!x || !x->codes || !x->seq_start) return set_error(PLAST_E_ARG, "%s: null bank pointer", name);
  return check_bank_sizes(x, name);
}

int plast_ungapped_extend(const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                          int32_t mode, void* d_ws, size_t ws_bytes, plast_hit_t* d_hits, int64_t capacity,
                          int64_t* h_n_hits, int64_t* h_n_ext, void* stream) {
  g_last_error[0] = 0;
  int rc;
  if ((rc = check_index(a, "a")) || (rc = check_index(b, "b"))) return rc;
  if (!p || !h_n_hits || !d_ws || capacity < 0 || (capacity > 0 && !d_hits))
    return set_error(PLAST_E_ARG, "null pointer or negative capacity");
  if ((rc = check_uparams(p))) return rc;
  if (mode != PLAST_PLAIN && mode != PLAST_BATCHED) return set_error(PLAST_E_ARG, "unknown mode %d", mode);
  if ((uintptr_t)d_ws & 255) return set_error(PLAST_E_ARG, "workspace must be 256-byte aligned");
  return ungapped_extend_impl(a, b, p, mode, d_ws, ws_bytes, d_hits, capacity, h_n_hits, h_n_ext,
                              (hipStream_t)stream);
}

int plast_ungapped_extend_noalloc(const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                                  plast_hit_t* d_hits, int64_t capacity, int64_t* h_n_hits, int64_t* h_n_ext,
                                  void* stream) {
  g_last_error[0] = 0;
  int rc;
  if ((rc = check_index(a, "a")) || (rc = check_index(b, "b"))) return rc;
  if (!p || !h_n_hits || capacity < 0 || (capacity > 0 && !d_hits))
    return set_error(PLAST_E_ARG, "null pointer or negative capacity");
  if ((rc = check_uparams(p))) return rc;
  return ungapped_extend_noalloc_impl(a, b, p, d_hits, capacity, h_n_hits, h_n_ext, (hipStream_t)stream);
}

int plast_gapped_filter(const plast_index_t* a, const plast_index_t* b, const plast_hit_t* d_hits, int64_t n_hits,
                        const plast_gapped_params_t* g, int32_t* d_gscore, uint8_t* d_pass, void* stream) {
  g_last_error[0] = 0;
  int rc;
  if ((rc = check_index(a, "a")) || (rc = check_index(b, "b"))) return rc;
  if (!g || n_hits < 0 || (n_hits > 0 && (!d_hits || !d_gscore || !d_pass)))
    return set_error(PLAST_E_ARG, "null pointer or negative hit count");
  if ((rc = check_gparams(g))) return rc;
  if (n_hits == 0) return PLAST_OK;
  return gapped_filter_impl(a, b, d_hits, n_hits, nullptr, g, d_gscore, d_pass, (hipStream_t)stream);
}

int plast_autotune(const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                   const plast_gapped_params_t* g, int32_t reps, void* d_ws, size_t ws_bytes,
                   plast_hit_t* d_hits, int64_t capacity, int32_t* d_gscore, uint8_t* d_pass,
                   plast_tuning_t* out, plast_tune_report_t* report, void* stream) {
  g_last_error[0] = 0;
  int rc;
  if ((rc = check_index(a, "a")) || (rc = check_index(b, "b")) || (rc = check_uparams(p)) || (rc = check_gparams(g)))
    return rc;
  if (!out || !d_ws || capacity < 0 || (capacity > 0 && (!d_hits || !d_gscore || !d_pass)))
    return set_error(PLAST_E_ARG, "null pointer or negative capacity");
  if (reps < 1 || reps > 20) return set_error(PLAST_E_ARG, "reps=%d outside 1..20", reps);
  if ((uintptr_t)d_ws & 255) return set_error(PLAST_E_ARG, "workspace must be 256-byte aligned");
  return autotune_impl(a, b, p, g, reps, d_ws, ws_bytes, d_hits, capacity, d_gscore, d_pass, out, report,
                       (hipStream_t)stream);
}

int plast_pipeline_workspace_bytes(const plast_bank_t* a, const plast_bank_t* b, int64_t max_items, size_t* bytes) {
  g_last_error[0] = 0;
  int rc;
  if ((rc = check_bank_sizes(a, "a")) || (rc = check_bank_sizes(b, "b"))) return rc;
  if (!bytes || max_items < 0 || max_items > INT32_MAX)
    return set_error(PLAST_E_ARG, "null output pointer or max_items outside [0, 2^31)");
  *bytes = pipeline_ws_bytes(a, b, max_items);
  return PLAST_OK;
}

int plast_pipeline_create(const plast_bank_t* a, const plast_bank_t* b, const plast_ungapped_params_t* p,
                          const plast_gapped_params_t* g, int64_t max_items, void* d_ws, size_t ws_bytes,
                          plast_hit_t* d_hits, int64_t capacity, int32_t* d_gscore, uint8_t* d_pass,
                          plast_pipeline_t** out) {
  g_last_error[0] = 0;
  int rc;
  if ((rc = check_bank(a, "a")) || (rc = check_bank(b, "b")) || (rc = check_uparams(p)) || (rc = check_gparams(g)))
    return rc;
  if (!out || !d_ws || capacity < 0 || (capacity > 0 && (!d_hits || !d_gscore || !d_pass)) || max_items < 0 ||
      max_items > INT32_MAX)
    return set_error(PLAST_E_ARG, "null pointer, negative capacity or max_items outside [0, 2^31)");
  if ((uintptr_t)d_ws & 255) return set_error(PLAST_E_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < pipeline_ws_bytes(a, b, max_items))
    return set_error(PLAST_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, pipeline_ws_bytes(a, b, max_items));
  return pipeline_create_impl(a, b, p, g, max_items, d_ws, d_hits, capacity, d_gscore, d_pass, out);
}

int plast_pipeline_launch(plast_pipeline_t* pl, void* stream) {
  g_last_error[0] = 0;
  if (!pl) return set_error(PLAST_E_ARG, "null pipeline");
  return pipeline_launch_impl(pl, (hipStream_t)stream);
}

int plast_pipeline_result(plast_pipeline_t* pl, plast_pipeline_result_t* out, void* stream) {
  g_last_error[0] = 0;
  if (!pl || !out) return set_error(PLAST_E_ARG, "null pointer");
  return pipeline_result_impl(pl, out, (hipStream_t)stream);
}

int plast_pipeline_index(const plast_pipeline_t* pl, int32_t which, plast_index_t* out) {
  g_last_error[0] = 0;
  if (!pl || !out || (which != 0 && which != 1)) return set_error(PLAST_E_ARG, "null pointer or which not 0/1");
  return pipeline_index_impl(pl, which, out);
}

int plast_pipeline_destroy(plast_pipeline_t* pl) {
  g_last_error[0] = 0;
  if (!pl) return PLAST_OK;
  return pipeline_destroy_impl(pl);
}

int plast_search_workspace_bytes(const plast_bank_t* a, int64_t max_items, size_t* bytes) {
  g_last_error[0] = 0;
  int rc;
  if ((rc = check_bank_sizes(a, "a"))) return rc;
  if (!bytes || max_items < 0 || max_items > INT32_MAX)
    return set_error(PLAST_E_ARG, "null output pointer or max_items outside [0, 2^31)");
  *bytes = search_ws_bytes(a, max_items);
  return PLAST_OK;
}

int plast_search_enqueue(const plast_bank_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                         const plast_gapped_params_t* g, int64_t max_items, void* d_ws, size_t ws_bytes,
                         plast_hit_t* d_hits, int64_t capacity, int32_t* d_gscore, uint8_t* d_pass,
                         plast_match_t* d_matches, const int32_t* d_seg_first, int32_t n_seg, int64_t* d_seg_off,
                         void* stream) {
  g_last_error[0] = 0;
  int rc;
  if ((rc = check_bank(a, "a")) || (rc = check_index(b, "b")) || (rc = check_uparams(p)) || (rc = check_gparams(g)))
    return rc;
  if (!d_ws || capacity < 0 || (capacity > 0 && (!d_hits || !d_gscore || !d_pass)) || max_items < 0 ||
      max_items > INT32_MAX)
    return set_error(PLAST_E_ARG, "null pointer, negative capacity or max_items outside [0, 2^31)");
  if ((uintptr_t)d_ws & 255) return set_error(PLAST_E_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < search_ws_bytes(a, max_items))
    return set_error(PLAST_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, search_ws_bytes(a, max_items));
  if (d_seg_first && (!d_matches || !d_seg_off || n_seg < 1 || n_seg > a->n_seqs + 1 || n_seg > 65536))
    return set_error(PLAST_E_ARG, "segments need matches, offsets and 1 <= n_seg <= min(n_seqs + 1, 65536)");
  return search_enqueue_impl(a, b, p, g, max_items, d_ws, d_hits, capacity, d_gscore, d_pass, d_matches,
                             d_seg_first, d_seg_first ? n_seg : 0, d_seg_off, (hipStream_t)stream);
}

int plast_search_result(const void* d_ws, plast_pipeline_result_t* out, int64_t* n_matches, void* stream) {
  g_last_error[0] = 0;
  if (!d_ws || !out) return set_error(PLAST_E_ARG, "null pointer");
  return search_result_impl(d_ws, out, n_matches, (hipStream_t)stream);
}

int plast_translate_ws_bytes(int32_t n_dna, size_t* bytes) {
  g_last_error[0] = 0;
  if (!bytes || n_dna < 0 || n_dna > (1 << 28)) return set_error(PLAST_E_ARG, "null output or n_dna out of range");
  *bytes = translate_ws_bytes(n_dna);
  return PLAST_OK;
}

static int check_translate(const uint8_t* d_dna, const int64_t* d_dna_start, int32_t n_dna, int64_t n_nt, void* d_ws,
                           size_t ws_bytes) {
  if (!d_dna_start || !d_ws || (n_nt > 0 && !d_dna)) return set_error(PLAST_E_ARG, "null pointer");
  if (n_dna < 0 || n_dna > (1 << 28) || n_nt < 0) return set_error(PLAST_E_ARG, "bad sizes");
  if ((uintptr_t)d_ws & 255) return set_error(PLAST_E_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < translate_ws_bytes(n_dna))
    return set_error(PLAST_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, translate_ws_bytes(n_dna));
  return PLAST_OK;
}

int plast_translate_count(const uint8_t* d_dna, const int64_t* d_dna_start, int32_t n_dna, int64_t n_nt, void* d_ws,
                          size_t ws_bytes, int64_t* h_n_frags, int64_t* h_n_padded, void* stream) {
  g_last_error[0] = 0;
  int rc;
  if ((rc = check_translate(d_dna, d_dna_start, n_dna, n_nt, d_ws, ws_bytes))) return rc;
  if (!h_n_frags || !h_n_padded) return set_error(PLAST_E_ARG, "null output pointer");
  return translate_count_impl(d_dna, d_dna_start, n_dna, n_nt, d_ws, h_n_frags, h_n_padded, (hipStream_t)stream);
}

int plast_translate_write(const uint8_t* d_dna, const int64_t* d_dna_start, int32_t n_dna, int64_t n_nt, void* d_ws,
                          size_t ws_bytes, uint8_t* d_codes, int64_t n_padded, int64_t* d_seq_start, int32_t* d_frag,
                          int64_t n_frags, void* stream) {
  g_last_error[0] = 0;
  int rc;
  if ((rc = check_translate(d_dna, d_dna_start, n_dna, n_nt, d_ws, ws_bytes))) return rc;
  if (!d_codes || !d_seq_start || (n_frags > 0 && !d_frag) || n_frags < 0 || n_padded < kPadLen * (n_frags + 1))
    return set_error(PLAST_E_ARG, "null output or sizes not from plast_translate_count");
  return translate_write_impl(d_dna, d_dna_start, n_dna, n_nt, d_ws, d_codes, n_padded, d_seq_start, d_frag, n_frags,
                              (hipStream_t)stream);
}

static int check_aparams(const plast_align_params_t* p) {
  if (!p) return set_error(PLAST_E_ARG, "null alignment parameters");
  if (p->gap_open < 0 || p->gap_extend < 1 || p->gap_open > 1000 || p->gap_extend > 1000)
    return set_error(PLAST_E_ARG, "gap_open=%d, gap_extend=%d (need 0..1000 and 1..1000)", p->gap_open,
                     p->gap_extend);
  if (p->max_len1 < 1 || p->max_len1 > 16384 || p->max_len2 < 1 || p->max_len2 > 16384)
    return set_error(PLAST_E_ARG, "max_len1=%d, max_len2=%d outside 1..16384", p->max_len1, p->max_len2);
  if (p->n_waves < 0 || p->n_waves > (1 << 20)) return set_error(PLAST_E_ARG, "n_waves=%d", p->n_waves);
  if (p->max_pieces < 16 || p->max_pieces > (1 << 24)) return set_error(PLAST_E_ARG, "max_pieces=%d", p->max_pieces);
  if (p->matrix) {
    for (int k = 0; k < 400; ++k)
      if (p->matrix[k] < -100 || p->matrix[k] > 100) return set_error(PLAST_E_ARG, "matrix entry outside -100..100");
  }
  return PLAST_OK;
}

int plast_align_workspace_bytes(int64_t n_hits, const plast_align_params_t* p, size_t* bytes) {
  g_last_error[0] = 0;
  int rc;
  if ((rc = check_aparams(p))) return rc;
  if (!bytes || n_hits < 0 || n_hits > INT32_MAX) return set_error(PLAST_E_ARG, "null output or n_hits outside [0, 2^31)");
  int64_t waves = 0;
  if ((rc = align_default_waves(*p, &waves))) return rc;
  *bytes = align_ws_bytes(n_hits, *p, waves);
  return PLAST_OK;
}

int plast_align(const plast_index_t* a, const plast_index_t* b, const plast_hit_t* d_hits, const int32_t* d_gscore,
                const uint8_t* d_pass, int64_t n_hits, const plast_align_params_t* p, void* d_ws, size_t ws_bytes,
                plast_alignment_t* d_out, int32_t* d_cover, int64_t* h_n_out, void* stream) {
  g_last_error[0] = 0;
  int rc;
  if ((rc = check_index(a, "a")) || (rc = check_index(b, "b")) || (rc = check_aparams(p))) return rc;
  if (!h_n_out || n_hits < 0 || n_hits > INT32_MAX) return set_error(PLAST_E_ARG, "null count or n_hits outside [0, 2^31)");
  *h_n_out = 0;
  if (n_hits == 0) return PLAST_OK;
  if (!d_hits || !d_gscore || !d_pass || !d_out || !d_cover || !d_ws)
    return set_error(PLAST_E_ARG, "null device pointer");
  if ((uintptr_t)d_ws & 255) return set_error(PLAST_E_ARG, "workspace must be 256-byte aligned");
  return align_impl(a, b, d_hits, d_gscore, d_pass, n_hits, p, d_ws, ws_bytes, d_out, d_cover, h_n_out,
                    (hipStream_t)stream);
}

}  // extern "C"
