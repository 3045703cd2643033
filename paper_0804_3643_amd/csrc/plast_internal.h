// Internal declarations of the gfx950 PLAST-P library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plast.h"

namespace plast {

constexpr int kNKeys = PLAST_NKEYS;
constexpr int kSeed = PLAST_SEED_LEN;
constexpr int kNbr = PLAST_NBR;
constexpr int kRight = kSeed + kNbr;     // letters scanned rightward, seed included
constexpr int kSpan = kRight + kNbr;     // 44 scan steps per pair
constexpr int kPadCode = PLAST_PAD_CODE;
constexpr int kPadLen = PLAST_PAD_LEN;
constexpr int kNLet = 21;                // 20 residues + separator
constexpr int kScale = 8;                // scan_codes[p] = codes[p] * kScale
constexpr int kScanSlack = 128;          // separator bytes appended to scan_codes

// ---------------------------------------------------------------- tables
// BLOSUM62 (Henikoff & Henikoff 1992); this library's transcription, rows and
// columns in the NCBI order ARNDCQEGHILKMFPSTWYV, permuted to code order when
// kernels stage it.
extern const char kNcbiOrder[21];
extern const int8_t kBlosum62Ncbi[20][20];
// Fill m[20*20] (code order ACDEFGHIKLMNPQRSTVWY) with BLOSUM62.
void blosum62_code_order(int8_t* m);

// Subset seed of Sec. 3.3.1: position 2 has two classes, position 3 eleven.
// Class ids are packed 4 bits per residue code (code c at bits 4c of a
// 128-bit value split in two words) so kernels evaluate them in registers.
struct SeedClasses {
  uint32_t pos2_g_mask;   // bit c set iff residue c is in class g (id 1), else class c (id 0)
  uint64_t pos3_lo;       // codes 0..15
  uint64_t pos3_hi;       // codes 16..19
};
SeedClasses seed_classes();

__device__ __forceinline__ int seed_key_dev(const SeedClasses& sc, int w0, int w1, int w2, int w3) {
  int c2 = (sc.pos2_g_mask >> w1) & 1;
  int c3 = (int)((w2 < 16 ? (sc.pos3_lo >> (4 * w2)) : (sc.pos3_hi >> (4 * (w2 - 16)))) & 15u);
  return ((w0 * 2 + c2) * 11 + c3) * 20 + w3;
}

// ---------------------------------------------------------------- errors
int set_error(int code, const char* fmt, ...);
int hip_check(hipError_t e, const char* what);
#define PLAST_HIP(call)                                   \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return ::plast::hip_check(e_, #call); \
  } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------- timing
enum TimedStage {
  kStageIndex = 0,
  kStagePlan = 1,
  kStageUngapped = 2,
  kStageGapped = 3,
  kStageAlign = 4,
  kNumStages = 5
};
bool timing_on();
// Record the start / stop event of a stage on `s` (no-ops while timing is off).
void timing_mark(TimedStage st, bool stop, hipStream_t s);
void timing_launches(int64_t n);

// ---------------------------------------------------------------- index build
struct IndexLayout {
  size_t key_off, occ, occ_seq, scan, total;
};
IndexLayout index_layout(int64_t n_padded);
// Workspace of one index build; it grows with n_padded only.
size_t index_ws_bytes(int64_t n_padded);

// Enqueues the whole build (no host synchronisation).  d_err[0] receives error
// bits (1: layout, 2: alphabet), d_err[1] the number of words.  After a layout
// error the kernels that would follow seq_start do nothing.  *out is filled
// except n_words (-1).
int index_enqueue(const uint8_t* d_codes, const int64_t* d_seq_start, int32_t n_seqs, int64_t n_padded,
                  void* d_index, void* d_ws, int32_t* d_err, plast_index_t* out, hipStream_t stream);
int build_index_impl(const uint8_t* d_codes, const int64_t* d_seq_start, int32_t n_seqs, int64_t n_padded,
                     void* d_index, void* d_ws, plast_index_t* out, hipStream_t stream);

// ---------------------------------------------------------------- scans
// Exclusive int32 scan of n elements in place; d_tmp needs scan_tmp_bytes(n).
size_t scan_tmp_bytes(int64_t n);
void exclusive_scan_i32(int32_t* d_data, int64_t n, int32_t* d_total, void* d_tmp, hipStream_t s);

// ---------------------------------------------------------------- ungapped
constexpr int kTileRows = 32;           // bank-a occurrences per work item (profile rows)
constexpr int kRowGroups = kTileRows / 4;
constexpr int kThreads = 512;           // threads per workgroup (8 wavefronts share one profile)
constexpr int kMaxColsPerLane = 32;     // bank-b occurrences per lane per item, at most
constexpr int kMaxItemCols = kThreads * kMaxColsPerLane;  // 16384
constexpr int kClasses = PLAST_TUNE_CLASSES;
constexpr int kMaxQueues = 8;           // one per XCD

void tuning_default(plast_tuning_t* t);
int check_tuning(const plast_tuning_t* t);  // PLAST_OK or PLAST_E_ARG (with detail)

struct WorkItem {
  int32_t key, row0, col0, ncols;
};

int ungapped_extend_impl(const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                         int32_t mode, void* d_ws, size_t ws_bytes, plast_hit_t* d_hits, int64_t capacity,
                         int64_t* h_n_hits, int64_t* h_n_ext, hipStream_t stream);
// plast_ungapped_extend_noalloc: the BATCHED schedule with its workspace in a
// static device array (PLAST_NOALLOC_SCRATCH_BYTES per device).
int ungapped_extend_noalloc_impl(const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                                 plast_hit_t* d_hits, int64_t capacity, int64_t* h_n_hits, int64_t* h_n_ext,
                                 hipStream_t stream);
int ungapped_ws_bytes_impl(const plast_index_t* a, const plast_index_t* b, int32_t mode, const plast_tuning_t& t,
                           size_t* bytes, int64_t* n_ext, int64_t* n_items, hipStream_t stream);

// Bytes of the BATCHED workspace before the work list, and the list length
// that a workspace of ws_bytes holds.
size_t ungapped_ws_fixed_bytes();
int64_t ungapped_ws_max_items(size_t ws_bytes);
// Work-list length for these key tables (host copies, kNKeys + 1 each) under
// tuning t, restricted to the classes in class_mask; *n_ext likewise.
int64_t plan_items_host(const int64_t* ha, const int64_t* hb, const plast_tuning_t& t, uint32_t class_mask,
                        int64_t* n_ext);
int read_key_offsets(const plast_index_t* x, int64_t* h, hipStream_t s);  // h: kNKeys + 1

// Enqueues the BATCHED schedule (counter reset, work list, persistent kernel)
// with no host synchronisation.  Only keys of the classes in class_mask get
// items.  err_a / err_b (may be null) are index error words: if either is
// non-zero on the device the list is left empty.  ev0 / ev1 (may be null) are
// recorded around the persistent kernel.
int ungapped_enqueue_batched(const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                             const plast_tuning_t& t, uint32_t class_mask, void* d_ws, size_t ws_bytes,
                             plast_hit_t* d_hits, int64_t capacity, const int32_t* err_a, const int32_t* err_b,
                             hipEvent_t ev0, hipEvent_t ev1, hipStream_t stream);
// Device counters of the last BATCHED run at the start of d_ws: hits, pairs,
// work-list length (the int32 scan total, and the same count summed in 64 bits
// to catch a list too long for int32), overflow flag (1: list longer than the
// workspace holds, 2: an index error).
struct UngappedCounters {
  unsigned long long n_hits, n_ext;
  int32_t n_items, overflow;
  unsigned long long n_items64;
};
const void* ungapped_counters_dev(const void* d_ws);
unsigned long long* ungapped_n_hits_dev(void* d_ws);

// ---------------------------------------------------------------- gapped
// d_n (may be null): device hit count; when given, min(*d_n, n_hits) records
// are scored and n_hits is only the bound the grid is sized for.
int gapped_filter_impl(const plast_index_t* a, const plast_index_t* b, const plast_hit_t* d_hits, int64_t n_hits,
                       const unsigned long long* d_n, const plast_gapped_params_t* g, int32_t* d_gscore,
                       uint8_t* d_pass, hipStream_t stream);

// ---------------------------------------------------------------- autotuner, graph pipeline
int autotune_impl(const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                  const plast_gapped_params_t* g, int32_t reps, void* d_ws, size_t ws_bytes, plast_hit_t* d_hits,
                  int64_t capacity, int32_t* d_gscore, uint8_t* d_pass, plast_tuning_t* out,
                  plast_tune_report_t* report, hipStream_t stream);
// Occupancy queries of the persistent kernels, made once before any graph capture.
int ungapped_prepare();
int gapped_prepare();

size_t pipeline_ws_bytes(const plast_bank_t* a, const plast_bank_t* b, int64_t max_items);
int pipeline_create_impl(const plast_bank_t* a, const plast_bank_t* b, const plast_ungapped_params_t* p,
                         const plast_gapped_params_t* g, int64_t max_items, void* d_ws, plast_hit_t* d_hits,
                         int64_t capacity, int32_t* d_gscore, uint8_t* d_pass, plast_pipeline_t** out);
int pipeline_launch_impl(plast_pipeline_t* pl, hipStream_t s);
int pipeline_result_impl(plast_pipeline_t* pl, plast_pipeline_result_t* out, hipStream_t s);
int pipeline_index_impl(const plast_pipeline_t* pl, int32_t which, plast_index_t* out);
int pipeline_destroy_impl(plast_pipeline_t* pl);

size_t search_ws_bytes(const plast_bank_t* a, int64_t max_items);
int search_enqueue_impl(const plast_bank_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                        const plast_gapped_params_t* g, int64_t max_items, void* d_ws, plast_hit_t* d_hits,
                        int64_t capacity, int32_t* d_gscore, uint8_t* d_pass, plast_match_t* d_matches,
                        const int32_t* d_seg_first, int32_t n_seg, int64_t* d_seg_off, hipStream_t s);
int search_result_impl(const void* d_ws, plast_pipeline_result_t* out, int64_t* n_matches, hipStream_t s);

// ---------------------------------------------------------------- six-frame translation
size_t translate_ws_bytes(int32_t n_dna);
int translate_count_impl(const uint8_t* d_dna, const int64_t* d_dna_start, int32_t n_dna, int64_t n_nt, void* d_ws,
                         int64_t* h_n_frags, int64_t* h_n_padded, hipStream_t s);
int translate_write_impl(const uint8_t* d_dna, const int64_t* d_dna_start, int32_t n_dna, int64_t n_nt, void* d_ws,
                         uint8_t* d_codes, int64_t n_padded, int64_t* d_seq_start, int32_t* d_frag, int64_t n_frags,
                         hipStream_t s);

// ---------------------------------------------------------------- stage 3.2
// Wavefronts of the alignment kernel (p.n_waves, or as many as stay resident).
int align_default_waves(const plast_align_params_t& p, int64_t* waves);
size_t align_ws_bytes(int64_t n_hits, const plast_align_params_t& p, int64_t waves);
int align_impl(const plast_index_t* a, const plast_index_t* b, const plast_hit_t* d_hits, const int32_t* d_gscore,
               const uint8_t* d_pass, int64_t n_hits, const plast_align_params_t* p, void* d_ws, size_t ws_bytes,
               plast_alignment_t* d_out, int32_t* d_cover, int64_t* h_n_out, hipStream_t s);

}  // namespace plast
