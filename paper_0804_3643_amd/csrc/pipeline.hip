// Launch-shape autotuner and the graph-replayed whole-search pipeline.
//
// Autotuner.  The BATCHED schedule has three shape parameters that change
// speed but not results: the item width of each size class of keys (bank-b
// occurrences per work item), the number of work queues (one, or one per XCD),
// and the gapped filter's workgroup size.  They are measured on the device for
// the banks at hand: each class alone at every candidate width, then the whole
// list with each queue count, then the gapped filter at each workgroup size;
// every figure is the best of `reps` runs between two HIP events.
//
// Pipeline.  Stage 0 for both banks, the work list, the persistent extension
// kernel and the gapped filter are captured once from a stream the pipeline
// owns and replayed as one HIP graph.  The captured kernels are the ones the
// separate calls launch; the host-side checks those calls make between stages
// are replaced by device-side flags (a bank with an error gets an empty work
// list, the gapped filter reads the hit count from device memory), so a replay
// needs no host round trip.  Counters are cleared by kernels, not memset nodes.
#include <string.h>

#include <new>
#include <vector>

#include "plast_internal.h"

struct plast_pipeline {
  hipStream_t cap = nullptr;  // capture stream (default priority)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int32_t* err_a = nullptr;   // device: [flags, n_words] per bank
  int32_t* err_b = nullptr;
  void* uws = nullptr;        // ungapped workspace inside the caller's buffer
  int64_t capacity = 0;
  plast_index_t va{}, vb{};
};

namespace plast {

namespace {

struct PipelineLayout {
  size_t idx_a, idx_b, build, uws, total;
};

PipelineLayout pipeline_layout(const plast_bank_t* a, const plast_bank_t* b, int64_t max_items) {
  PipelineLayout L;
  size_t off = 256;  // error words of both banks
  L.idx_a = off;
  off = align_up(off + index_layout(a->n_padded).total, 256);
  L.idx_b = off;
  off = align_up(off + index_layout(b->n_padded).total, 256);
  L.build = off;
  const size_t wa = index_ws_bytes(a->n_padded), wb = index_ws_bytes(b->n_padded);
  off = align_up(off + (wa > wb ? wa : wb), 256);
  L.uws = off;
  off = align_up(off + ungapped_ws_fixed_bytes() + sizeof(WorkItem) * (size_t)max_items, 256);
  L.total = off;
  return L;
}

struct EventPair {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~EventPair() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

}  // namespace

size_t pipeline_ws_bytes(const plast_bank_t* a, const plast_bank_t* b, int64_t max_items) {
  return pipeline_layout(a, b, max_items).total;
}

int pipeline_create_impl(const plast_bank_t* a, const plast_bank_t* b, const plast_ungapped_params_t* p,
                         const plast_gapped_params_t* g, int64_t max_items, void* d_ws, plast_hit_t* d_hits,
                         int64_t capacity, int32_t* d_gscore, uint8_t* d_pass, plast_pipeline_t** out) {
  const PipelineLayout L = pipeline_layout(a, b, max_items);
  plast_tuning_t T;
  if (p->tuning)
    T = *p->tuning;
  else
    tuning_default(&T);
  int rc = ungapped_prepare();
  if (rc == PLAST_OK) rc = gapped_prepare();
  if (rc != PLAST_OK) return rc;
  plast_pipeline* P = new (std::nothrow) plast_pipeline;
  if (!P) return set_error(PLAST_E_ARG, "out of host memory");
  uint8_t* base = (uint8_t*)d_ws;
  P->err_a = (int32_t*)base;
  P->err_b = (int32_t*)(base + 8);
  P->uws = base + L.uws;
  P->capacity = capacity;
  hipError_t e = hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete P;
    return hip_check(e, "hipStreamCreateWithFlags");
  }
  e = hipStreamBeginCapture(P->cap, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    pipeline_destroy_impl(P);
    return hip_check(e, "hipStreamBeginCapture");
  }
  rc = index_enqueue(a->codes, a->seq_start, a->n_seqs, a->n_padded, base + L.idx_a, base + L.build, P->err_a,
                     &P->va, P->cap);
  if (rc == PLAST_OK)
    rc = index_enqueue(b->codes, b->seq_start, b->n_seqs, b->n_padded, base + L.idx_b, base + L.build, P->err_b,
                       &P->vb, P->cap);
  if (rc == PLAST_OK)
    rc = ungapped_enqueue_batched(&P->va, &P->vb, p, T, ~0u, P->uws, L.total - L.uws, d_hits, capacity, P->err_a,
                                  P->err_b, nullptr, nullptr, P->cap);
  if (rc == PLAST_OK && capacity > 0)
    rc = gapped_filter_impl(&P->va, &P->vb, d_hits, capacity, ungapped_n_hits_dev(P->uws), g, d_gscore, d_pass,
                            P->cap);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(P->cap, &graph);
  P->graph = graph;
  if (rc != PLAST_OK) {
    pipeline_destroy_impl(P);
    return rc;
  }
  if (e != hipSuccess) {
    pipeline_destroy_impl(P);
    return hip_check(e, "hipStreamEndCapture");
  }
  e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    pipeline_destroy_impl(P);
    return hip_check(e, "hipGraphInstantiate");
  }
  *out = P;
  return PLAST_OK;
}

int pipeline_launch_impl(plast_pipeline_t* pl, hipStream_t s) {
  PLAST_HIP(hipGraphLaunch(pl->exec, s));
  return PLAST_OK;
}

int pipeline_result_impl(plast_pipeline_t* pl, plast_pipeline_result_t* out, hipStream_t s) {
  int32_t err[4] = {0, 0, 0, 0};
  UngappedCounters c{0, 0, 0, 0, 0};
  PLAST_HIP(hipMemcpyAsync(err, pl->err_a, sizeof(err), hipMemcpyDeviceToHost, s));
  PLAST_HIP(hipMemcpyAsync(&c, ungapped_counters_dev(pl->uws), sizeof(c), hipMemcpyDeviceToHost, s));
  PLAST_HIP(hipStreamSynchronize(s));
  out->n_items = c.n_items;
  out->n_hits = (int64_t)c.n_hits;
  out->n_ext = (int64_t)c.n_ext;
  out->n_words_a = err[1];
  out->n_words_b = err[3];
  pl->va.n_words = err[1];
  pl->vb.n_words = err[3];
  const int32_t flags = err[0] | err[2];
  if (flags & 1)
    out->status = PLAST_E_LAYOUT;
  else if (flags & 2)
    out->status = PLAST_E_ALPHABET;
  else if (c.overflow)
    out->status = PLAST_E_WORKSPACE;
  else if ((int64_t)c.n_hits > pl->capacity)
    out->status = PLAST_E_CAPACITY;
  else
    out->status = PLAST_OK;
  return PLAST_OK;
}

int pipeline_index_impl(const plast_pipeline_t* pl, int32_t which, plast_index_t* out) {
  *out = which == 0 ? pl->va : pl->vb;
  return PLAST_OK;
}

int pipeline_destroy_impl(plast_pipeline_t* pl) {
  hipError_t e = hipSuccess, x;
  if (pl->exec && (x = hipGraphExecDestroy(pl->exec)) != hipSuccess) e = x;
  if (pl->graph && (x = hipGraphDestroy(pl->graph)) != hipSuccess) e = x;
  if (pl->cap && (x = hipStreamDestroy(pl->cap)) != hipSuccess) e = x;
  delete pl;
  if (e != hipSuccess) return hip_check(e, "pipeline destroy");
  return PLAST_OK;
}

// ---------------------------------------------------------------- query search (serving)
namespace {

// [0, 256): SearchHeader; then the ungapped workspace (its counters at a fixed
// offset, so plast_search_result needs no sizes), bank a's index, build scratch.
struct SearchHeader {
  int32_t err[2];             // bank a: error bits, words
  unsigned long long n_match;
  int64_t capacity;           // hit capacity of the search, for the status
  int64_t n_words_b;
};
static_assert(sizeof(SearchHeader) <= 256, "search header");
constexpr size_t kSearchUws = 256;

struct SearchLayout {
  size_t uws, idx_a, build, total;
};

SearchLayout search_layout(const plast_bank_t* a, int64_t max_items) {
  SearchLayout L;
  size_t off = kSearchUws;
  L.uws = off;
  off = align_up(off + ungapped_ws_fixed_bytes() + sizeof(WorkItem) * (size_t)max_items, 256);
  L.idx_a = off;
  off = align_up(off + index_layout(a->n_padded).total, 256);
  L.build = off;
  off = align_up(off + index_ws_bytes(a->n_padded), 256);
  L.total = off;
  return L;
}

__global__ void k_search_header(SearchHeader* h, int64_t capacity, int64_t n_words_b) {
  if (threadIdx.x == 0) {
    h->n_match = 0ull;
    h->capacity = capacity;
    h->n_words_b = n_words_b;
  }
}

constexpr int kCompactThreads = 256;
constexpr int kCompactBlocks = 1024;

// Hits with pass[i] set, among the first min(*n_dev, cap), appended to out in
// wavefront-sized groups (one atomic per wavefront).
__global__ __launch_bounds__(kCompactThreads) void k_compact_matches(
    const plast_hit_t* __restrict__ hits, const int32_t* __restrict__ gscore, const uint8_t* __restrict__ pass,
    const unsigned long long* __restrict__ n_dev, int64_t cap, plast_match_t* __restrict__ out,
    unsigned long long* __restrict__ n_out) {
  const int64_t n = min((int64_t)*n_dev, cap);
  const int lane = __lane_id();
  for (int64_t base = (int64_t)blockIdx.x * kCompactThreads; base < n; base += (int64_t)gridDim.x * kCompactThreads) {
    const int64_t i = base + threadIdx.x;
    const bool take = i < n && pass[i];
    const unsigned long long m = __ballot(take);
    if (!m) continue;
    const int leader = __ffsll((long long)m) - 1;
    unsigned long long b = 0;
    if (lane == leader) b = atomicAdd(n_out, (unsigned long long)__popcll(m));
    b = __shfl(b, leader);
    if (take) {
      const plast_hit_t h = hits[i];
      plast_match_t o;
      o.seq1 = h.seq1;
      o.pos1 = h.pos1;
      o.seq2 = h.seq2;
      o.pos2 = h.pos2;
      o.score = h.score;
      o.gscore = gscore[i];
      out[b + __popcll(m & ((1ull << lane) - 1ull))] = o;
    }
  }
}

// Segment of query sequence q: the s with seg_first[s] <= q < seg_first[s + 1].
__device__ __forceinline__ int segment_of(const int32_t* __restrict__ seg_first, int n_seg, int q) {
  int lo = 0, hi = n_seg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seg_first[mid] <= q) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Lanes of the wavefront with the same segment id (valid lanes only), from one
// ballot per id bit.
__device__ __forceinline__ unsigned long long segment_peers(int seg, bool valid) {
  unsigned long long peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    const int bit = (seg >> b) & 1;
    const unsigned long long m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// Pass 1: matches per segment (off[0 .. n_seg) must be zero); one atomic per
// (wavefront, segment).
__global__ __launch_bounds__(kCompactThreads) void k_segment_count(
    const plast_hit_t* __restrict__ hits, const uint8_t* __restrict__ pass, const unsigned long long* __restrict__ n_dev,
    int64_t cap, const int32_t* __restrict__ seg_first, int n_seg, unsigned long long* __restrict__ cnt) {
  const int64_t n = min((int64_t)*n_dev, cap);
  const int lane = __lane_id();
  for (int64_t base = (int64_t)blockIdx.x * kCompactThreads; base < n; base += (int64_t)gridDim.x * kCompactThreads) {
    const int64_t i = base + threadIdx.x;
    const bool take = i < n && pass[i];
    if (!__ballot(take)) continue;
    const int seg = take ? segment_of(seg_first, n_seg, hits[i].seq1) : 0;
    const unsigned long long peers = segment_peers(seg, take);
    if (take && lane == __ffsll((long long)peers) - 1) atomicAdd(&cnt[seg], (unsigned long long)__popcll(peers));
  }
}

// Exclusive scan of the n_seg counts (one workgroup): off[0..n_seg], the write
// cursors cur[s] = off[s], and the total in *n_out.
__global__ __launch_bounds__(256) void k_segment_scan(unsigned long long* __restrict__ off, int n_seg,
                                                      unsigned long long* __restrict__ cur,
                                                      unsigned long long* __restrict__ n_out) {
  __shared__ unsigned long long carry;
  __shared__ unsigned long long part[256];
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n_seg; base += 256) {
    const int s = base + threadIdx.x;
    const unsigned long long v = s < n_seg ? off[s] : 0ull;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {  // inclusive Hillis-Steele scan
      const unsigned long long t = threadIdx.x >= d ? part[threadIdx.x - d] : 0ull;
      __syncthreads();
      part[threadIdx.x] += t;
      __syncthreads();
    }
    const unsigned long long excl = carry + part[threadIdx.x] - v;
    if (s < n_seg) {
      off[s] = excl;
      cur[s] = excl;
    }
    __syncthreads();
    if (threadIdx.x == 255) carry += part[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    off[n_seg] = carry;
    *n_out = carry;
  }
}

// Pass 2: each passing hit to its segment's next slot; one atomic per
// (wavefront, segment), lanes ranked inside their group.
__global__ __launch_bounds__(kCompactThreads) void k_segment_scatter(
    const plast_hit_t* __restrict__ hits, const int32_t* __restrict__ gscore, const uint8_t* __restrict__ pass,
    const unsigned long long* __restrict__ n_dev, int64_t cap, const int32_t* __restrict__ seg_first, int n_seg,
    unsigned long long* __restrict__ cur, plast_match_t* __restrict__ out) {
  const int64_t n = min((int64_t)*n_dev, cap);
  const int lane = __lane_id();
  for (int64_t base = (int64_t)blockIdx.x * kCompactThreads; base < n; base += (int64_t)gridDim.x * kCompactThreads) {
    const int64_t i = base + threadIdx.x;
    const bool take = i < n && pass[i];
    if (!__ballot(take)) continue;
    plast_hit_t h = {0, 0, 0, 0, 0};
    if (take) h = hits[i];
    const int seg = take ? segment_of(seg_first, n_seg, h.seq1) : 0;
    const unsigned long long peers = segment_peers(seg, take);
    const int leader = take ? __ffsll((long long)peers) - 1 : 0;
    unsigned long long at = 0;
    if (take && lane == leader) at = atomicAdd(&cur[seg], (unsigned long long)__popcll(peers));
    at = __shfl(at, leader);
    if (take) {
      plast_match_t o;
      o.seq1 = h.seq1;
      o.pos1 = h.pos1;
      o.seq2 = h.seq2;
      o.pos2 = h.pos2;
      o.score = h.score;
      o.gscore = gscore[i];
      out[at + __popcll(peers & ((1ull << lane) - 1ull))] = o;
    }
  }
}

__global__ void k_zero_u64(unsigned long long* __restrict__ p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

}  // namespace

size_t search_ws_bytes(const plast_bank_t* a, int64_t max_items) { return search_layout(a, max_items).total; }

int search_enqueue_impl(const plast_bank_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                        const plast_gapped_params_t* g, int64_t max_items, void* d_ws, plast_hit_t* d_hits,
                        int64_t capacity, int32_t* d_gscore, uint8_t* d_pass, plast_match_t* d_matches,
                        const int32_t* d_seg_first, int32_t n_seg, int64_t* d_seg_off, hipStream_t s) {
  const SearchLayout L = search_layout(a, max_items);
  plast_tuning_t T;
  if (p->tuning)
    T = *p->tuning;
  else
    tuning_default(&T);
  uint8_t* base = (uint8_t*)d_ws;
  SearchHeader* hdr = (SearchHeader*)base;
  plast_index_t va;
  hipLaunchKernelGGL(k_search_header, dim3(1), dim3(64), 0, s, hdr, capacity, b->n_words);
  int rc = index_enqueue(a->codes, a->seq_start, a->n_seqs, a->n_padded, base + L.idx_a, base + L.build, hdr->err,
                         &va, s);
  if (rc != PLAST_OK) return rc;
  void* uws = base + L.uws;
  rc = ungapped_enqueue_batched(&va, b, p, T, ~0u, uws, L.idx_a - L.uws, d_hits, capacity, hdr->err, nullptr, nullptr,
                                nullptr, s);
  if (rc != PLAST_OK) return rc;
  if (capacity > 0) {
    rc = gapped_filter_impl(&va, b, d_hits, capacity, ungapped_n_hits_dev(uws), g, d_gscore, d_pass, s);
    if (rc != PLAST_OK) return rc;
    const int64_t blocks = min((int64_t)kCompactBlocks, (capacity + kCompactThreads - 1) / kCompactThreads);
    const unsigned long long* nh = ungapped_n_hits_dev(uws);
    if (d_matches && d_seg_first) {
      unsigned long long* off = (unsigned long long*)d_seg_off;
      unsigned long long* cur = off + (n_seg + 1);
      hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, off, n_seg + 1);
      hipLaunchKernelGGL(k_segment_count, dim3((unsigned)blocks), dim3(kCompactThreads), 0, s,
                         (const plast_hit_t*)d_hits, (const uint8_t*)d_pass, nh, capacity, d_seg_first, (int)n_seg,
                         off);
      hipLaunchKernelGGL(k_segment_scan, dim3(1), dim3(256), 0, s, off, (int)n_seg, cur, &hdr->n_match);
      hipLaunchKernelGGL(k_segment_scatter, dim3((unsigned)blocks), dim3(kCompactThreads), 0, s,
                         (const plast_hit_t*)d_hits, (const int32_t*)d_gscore, (const uint8_t*)d_pass, nh, capacity,
                         d_seg_first, (int)n_seg, cur, d_matches);
    } else if (d_matches) {
      hipLaunchKernelGGL(k_compact_matches, dim3((unsigned)blocks), dim3(kCompactThreads), 0, s,
                         (const plast_hit_t*)d_hits, (const int32_t*)d_gscore, (const uint8_t*)d_pass, nh, capacity,
                         d_matches, &hdr->n_match);
    }
  }
  PLAST_HIP(hipGetLastError());
  return PLAST_OK;
}

int search_result_impl(const void* d_ws, plast_pipeline_result_t* out, int64_t* n_matches, hipStream_t s) {
  SearchHeader h;
  UngappedCounters c{0, 0, 0, 0, 0};
  PLAST_HIP(hipMemcpyAsync(&h, d_ws, sizeof(h), hipMemcpyDeviceToHost, s));
  PLAST_HIP(hipMemcpyAsync(&c, ungapped_counters_dev((const uint8_t*)d_ws + kSearchUws), sizeof(c),
                           hipMemcpyDeviceToHost, s));
  PLAST_HIP(hipStreamSynchronize(s));
  const int64_t capacity = h.capacity;
  out->n_items = c.n_items;
  out->n_hits = (int64_t)c.n_hits;
  out->n_ext = (int64_t)c.n_ext;
  out->n_words_a = h.err[1];
  out->n_words_b = h.n_words_b;
  if (h.err[0] & 1)
    out->status = PLAST_E_LAYOUT;
  else if (h.err[0] & 2)
    out->status = PLAST_E_ALPHABET;
  else if (c.overflow)
    out->status = PLAST_E_WORKSPACE;
  else if ((int64_t)c.n_hits > capacity)
    out->status = PLAST_E_CAPACITY;
  else
    out->status = PLAST_OK;
  if (n_matches) *n_matches = (int64_t)h.n_match;
  return PLAST_OK;
}

// ---------------------------------------------------------------- autotuner
namespace {

constexpr int kWidths[PLAST_TUNE_WIDTHS] = {1024, 2048, 4096, 8192, 16384};
constexpr int kGapThreads[3] = {128, 256, 512};

// One timed BATCHED run; *ms = persistent-kernel time.
int timed_ungapped(const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                   const plast_tuning_t& t, uint32_t mask, void* d_ws, size_t ws_bytes, plast_hit_t* d_hits,
                   int64_t capacity, const EventPair& ev, hipStream_t s, float* ms, UngappedCounters* c) {
  int rc = ungapped_enqueue_batched(a, b, p, t, mask, d_ws, ws_bytes, d_hits, capacity, nullptr, nullptr, ev.e0,
                                    ev.e1, s);
  if (rc != PLAST_OK) return rc;
  PLAST_HIP(hipMemcpyAsync(c, ungapped_counters_dev(d_ws), sizeof(*c), hipMemcpyDeviceToHost, s));
  PLAST_HIP(hipStreamSynchronize(s));
  PLAST_HIP(hipEventElapsedTime(ms, ev.e0, ev.e1));
  if (c->overflow) return set_error(PLAST_E_WORKSPACE, "workspace too small for the work list");
  return PLAST_OK;
}

int best_ungapped(const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                  const plast_tuning_t& t, uint32_t mask, int reps, void* d_ws, size_t ws_bytes,
                  plast_hit_t* d_hits, int64_t capacity, const EventPair& ev, hipStream_t s, float* best,
                  UngappedCounters* c) {
  *best = 0.f;
  for (int r = 0; r < reps; ++r) {
    float ms = 0.f;
    int rc = timed_ungapped(a, b, p, t, mask, d_ws, ws_bytes, d_hits, capacity, ev, s, &ms, c);
    if (rc != PLAST_OK) return rc;
    if (r == 0 || ms < *best) *best = ms;
  }
  return PLAST_OK;
}

}  // namespace

int autotune_impl(const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                  const plast_gapped_params_t* g, int32_t reps, void* d_ws, size_t ws_bytes, plast_hit_t* d_hits,
                  int64_t capacity, int32_t* d_gscore, uint8_t* d_pass, plast_tuning_t* out,
                  plast_tune_report_t* report, hipStream_t s) {
  plast_tuning_t T;
  if (p->tuning)
    T = *p->tuning;
  else
    tuning_default(&T);
  plast_tune_report_t R;
  memset(&R, 0, sizeof(R));
  std::vector<int64_t> ha(kNKeys + 1), hb(kNKeys + 1);
  int rc;
  if ((rc = read_key_offsets(a, ha.data(), s)) || (rc = read_key_offsets(b, hb.data(), s))) return rc;
  EventPair ev;
  PLAST_HIP(hipEventCreate(&ev.e0));
  PLAST_HIP(hipEventCreate(&ev.e1));
  const int64_t max_items = ungapped_ws_max_items(ws_bytes);
  UngappedCounters c{0, 0, 0, 0, 0};

  // 1. item width per size class, each class alone
  for (int cl = 0; cl < kClasses; ++cl) {
    const uint32_t mask = 1u << cl;
    plan_items_host(ha.data(), hb.data(), T, mask, &R.class_ext[cl]);
    if (R.class_ext[cl] == 0) continue;
    int64_t max_n2 = 0;
    for (int k = 0; k < kNKeys; ++k) {
      const int64_t n1 = ha[k + 1] - ha[k], n2 = hb[k + 1] - hb[k];
      const bool in = n1 > 0 && n2 >= T.class_min_n2[cl] && (cl + 1 == kClasses || n2 < T.class_min_n2[cl + 1]);
      if (in && n2 > max_n2) max_n2 = n2;
    }
    float best = 0.f;
    int best_w = -1;
    for (int wi = 0; wi < PLAST_TUNE_WIDTHS; ++wi) {
      if (wi > 0 && kWidths[wi - 1] >= max_n2) break;  // same items as the previous width
      plast_tuning_t t = T;
      t.item_cols[cl] = kWidths[wi];
      if (plan_items_host(ha.data(), hb.data(), t, mask, nullptr) > max_items) continue;
      float ms = 0.f;
      if ((rc = best_ungapped(a, b, p, t, mask, reps, d_ws, ws_bytes, d_hits, capacity, ev, s, &ms, &c))) return rc;
      R.class_ms[cl][wi] = ms;
      if (best_w < 0 || ms < best) {
        best = ms;
        best_w = kWidths[wi];
      }
    }
    if (best_w > 0) T.item_cols[cl] = best_w;
  }

  // 2. queue count over the whole list
  if (plan_items_host(ha.data(), hb.data(), T, ~0u, nullptr) > max_items)
    return set_error(PLAST_E_WORKSPACE, "workspace too small for the work list");
  const int queues[2] = {1, kMaxQueues};
  for (int qi = 0; qi < 2; ++qi) {
    plast_tuning_t t = T;
    t.xcd_queues = queues[qi];
    if ((rc = best_ungapped(a, b, p, t, ~0u, reps, d_ws, ws_bytes, d_hits, capacity, ev, s, &R.queue_ms[qi], &c)))
      return rc;
  }
  T.xcd_queues = R.queue_ms[1] < R.queue_ms[0] ? kMaxQueues : 1;

  // 3. gapped workgroup size over the hits of a final extension run
  float ms = 0.f;
  if ((rc = timed_ungapped(a, b, p, T, ~0u, d_ws, ws_bytes, d_hits, capacity, ev, s, &ms, &c))) return rc;
  if ((int64_t)c.n_hits > capacity)
    return set_error(PLAST_E_CAPACITY, "%lld hits > capacity %lld", (long long)c.n_hits, (long long)capacity);
  const int64_t n = (int64_t)c.n_hits;
  if (n > 0) {
    int best_t = -1;
    for (int ti = 0; ti < 3; ++ti) {
      plast_tuning_t t = T;
      t.gapped_threads = kGapThreads[ti];
      plast_gapped_params_t gg = *g;
      gg.tuning = &t;
      float bt = 0.f;
      for (int r = 0; r < reps; ++r) {
        PLAST_HIP(hipEventRecord(ev.e0, s));
        if ((rc = gapped_filter_impl(a, b, d_hits, n, nullptr, &gg, d_gscore, d_pass, s))) return rc;
        PLAST_HIP(hipEventRecord(ev.e1, s));
        PLAST_HIP(hipEventSynchronize(ev.e1));
        float x = 0.f;
        PLAST_HIP(hipEventElapsedTime(&x, ev.e0, ev.e1));
        if (r == 0 || x < bt) bt = x;
      }
      R.gapped_ms[ti] = bt;
      if (best_t < 0 || bt < R.gapped_ms[best_t]) best_t = ti;
    }
    T.gapped_threads = kGapThreads[best_t];
  }
  *out = T;
  if (report) *report = R;
  return PLAST_OK;
}

}  // namespace plast
