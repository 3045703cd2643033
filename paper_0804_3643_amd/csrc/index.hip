// Stage 0, bank indexing (Sec. 3.3.1): subset-seed key of every word, then a
// stable counting sort by key into CSR form (key_off, occ, occ_seq).
//
// Layout: the bank is cut into contiguous position chunks (about 16K
// positions, at most 16384 chunks), one wavefront each.
// Pass 1 counts keys per chunk in LDS (8800 counters) and writes them key-major,
// an exclusive scan over (key, chunk) gives every chunk its first slot in each
// key's run, and pass 2 re-reads the chunk and scatters positions in order.
// Inside a wavefront, equal keys are ranked with 14 ballots (one per key bit),
// so the order inside a key is the position order: ascending (sequence,
// position), independent of scheduling.  HBM traffic is ~2 reads of the codes
// plus 8 bytes written per word.
#include "plast_internal.h"

namespace plast {

namespace {

constexpr int kChunkWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t peers_of(int key, bool valid) {
  // Lanes of the wavefront holding a valid word with the same key.
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 14; ++b) {
    int bit = (key >> b) & 1;
    uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

__device__ __forceinline__ int word_key(const uint8_t* __restrict__ codes, int64_t q, int64_t end,
                                        const SeedClasses& sc) {
  if (q >= end) return -1;
  int w0 = codes[q], w1 = codes[q + 1], w2 = codes[q + 2], w3 = codes[q + 3];
  if ((w0 | w1 | w2 | w3) >= 32 || w0 >= 20 || w1 >= 20 || w2 >= 20 || w3 >= 20) return -1;
  return seed_key_dev(sc, w0, w1, w2, w3);
}

__global__ void k_layout_check(const int64_t* __restrict__ seq_start, int32_t n_seqs, int64_t n_padded,
                               int32_t* __restrict__ err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n_seqs) return;
  int64_t s = seq_start[i];
  bool bad = s < kPadLen || s > n_padded;
  if (i == 0 && s != kPadLen) bad = true;
  if (i == n_seqs && s != n_padded) bad = true;
  if (i < n_seqs && seq_start[i + 1] - s < kPadLen) bad = true;
  if (bad) atomicOr(err, 1);
}

// Validation and scan codes, position-parallel (so that banks of many short
// sequences, such as translated fragments, keep every lane busy).  Each
// wavefront takes kCheckChunk consecutive positions of [0, scan_len): it finds
// the sequence holding its first position by binary search, then walks its
// positions in order.  Position p is a residue iff some sequence s has
// seq_start[s] <= p < seq_start[s + 1] - kPadLen; every other position below
// n_padded must hold the separator code, and the tail slack is set to it.
constexpr int64_t kCheckChunk = 4096;

__global__ __launch_bounds__(kChunkWave) void k_codes_check(const uint8_t* __restrict__ codes,
                                                            const int64_t* __restrict__ seq_start, int32_t n_seqs,
                                                            int64_t n_padded, uint8_t* __restrict__ scan,
                                                            int64_t scan_len, int32_t* __restrict__ err) {
  if (*err & 1) return;  // no walk over a bad layout
  const int lane = lane_id();
  const int64_t beg = (int64_t)blockIdx.x * kCheckChunk;
  const int64_t end = min(beg + kCheckChunk, scan_len);
  // s_cur: the last sequence with seq_start <= beg (-1 before the first one)
  int lo = -1, hi = n_seqs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seq_start[mid] <= beg) lo = mid; else hi = mid - 1;
  }
  int s_cur = lo;
  bool bad = false;
  for (int64_t base = beg; base < end; base += 64) {
    const int64_t p = base + lane;
    // at most 4 sequence starts in a window (each sequence takes >= kPadLen
    // positions): lanes 0..7 load the next 8 and every lane counts its own
    const int64_t nxt = (lane < 8 && s_cur + 1 + lane < n_seqs) ? seq_start[s_cur + 1 + lane] : INT64_MAX;
    int s = s_cur;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += p >= __shfl(nxt, j) ? 1 : 0;
    if (p < end) {
      if (p < n_padded) {
        const bool residue = s >= 0 && p < seq_start[s + 1] - kPadLen;
        const uint8_t c = codes[p];
        bad |= residue ? (c >= 20) : (c != kPadCode);
        scan[p] = (uint8_t)((residue && c < 20 ? c : kPadCode) * kScale);
      } else {
        scan[p] = (uint8_t)(kPadCode * kScale);
      }
    }
    s_cur = __shfl(s, 63);
  }
  if (bad) atomicOr(err, 2);
}

__global__ __launch_bounds__(kChunkWave) void k_index_count(const uint8_t* __restrict__ codes, int64_t n_padded,
                                                            int64_t chunk, int32_t nchunks, SeedClasses sc,
                                                            int32_t* __restrict__ counts) {
  __shared__ int32_t cnt[kNKeys];
  const int lane = lane_id();
  for (int k = lane; k < kNKeys; k += 64) cnt[k] = 0;
  __syncthreads();
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = min(beg + chunk, n_padded - (kSeed - 1));
  // the next window's letters are loaded one window ahead
  int key_next = beg < end ? word_key(codes, beg + lane, end, sc) : -1;
  for (int64_t base = beg; base < end; base += 64) {
    const int key = key_next;
    key_next = word_key(codes, base + 64 + lane, end, sc);
    uint64_t peers = peers_of(key, key >= 0);
    if (key >= 0 && lane == 63 - __clzll(peers)) cnt[key] += __popcll(peers);
  }
  __syncthreads();
  for (int k = lane; k < kNKeys; k += 64) counts[(int64_t)k * nchunks + blockIdx.x] = cnt[k];
}

__global__ __launch_bounds__(kChunkWave) void k_index_scatter(const uint8_t* __restrict__ codes,
                                                              const int64_t* __restrict__ seq_start,
                                                              int32_t n_seqs, int64_t n_padded, int64_t chunk,
                                                              int32_t nchunks, SeedClasses sc,
                                                              const int32_t* __restrict__ offs,
                                                              int32_t* __restrict__ occ,
                                                              int32_t* __restrict__ occ_seq) {
  __shared__ int32_t cur[kNKeys];
  const int lane = lane_id();
  for (int k = lane; k < kNKeys; k += 64) cur[k] = offs[(int64_t)k * nchunks + blockIdx.x];
  __syncthreads();
  if (n_seqs == 0) return;
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = min(beg + chunk, n_padded - (kSeed - 1));
  // sequence holding position beg: largest s with seq_start[s] <= beg (0 if none)
  int lo = 0, hi = n_seqs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (seq_start[mid] <= beg) lo = mid; else hi = mid - 1;
  }
  int s_cur = lo;
  int key_next = beg < end ? word_key(codes, beg + lane, end, sc) : -1;  // one window ahead
  for (int64_t base = beg; base < end; base += 64) {
    int64_t q = base + lane;
    const int key = key_next;
    key_next = word_key(codes, q + 64, end, sc);
    // Every sequence takes at least kPadLen positions (its separator run), so
    // a 64-position window meets at most 5 sequence starts: lanes 0..7 load the
    // next 8 starts at once and every lane counts those at or before q.
    const int64_t nxt = (lane < 8 && s_cur + 1 + lane < n_seqs) ? seq_start[s_cur + 1 + lane] : INT64_MAX;
    int s = s_cur;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += q >= __shfl(nxt, j) ? 1 : 0;
    uint64_t peers = peers_of(key, key >= 0);
    if (key >= 0) {
      int rank = __popcll(peers & ((1ull << lane) - 1ull));
      int slot = cur[key] + rank;
      occ[slot] = (int32_t)q;
      occ_seq[slot] = s;
    }
    if (key >= 0 && lane == 63 - __clzll(peers)) cur[key] += __popcll(peers);
    s_cur = __shfl(s, 63);
  }
}

__global__ void k_clear2(int32_t* __restrict__ p) {
  if (threadIdx.x < 2) p[threadIdx.x] = 0;
}

__global__ void k_key_off(const int32_t* __restrict__ offs, int32_t nchunks, const int32_t* __restrict__ total,
                          int64_t* __restrict__ key_off) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < kNKeys) key_off[k] = offs[(int64_t)k * nchunks];
  else if (k == kNKeys) key_off[k] = *total;
}

// ---------------------------------------------------------------- scan
constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanBlock = kScanThreads * kScanPer;

__device__ __forceinline__ int block_excl_scan(int v, int* total) {
  __shared__ int wsum[kScanThreads / 64];
  int lane = lane_id(), wid = threadIdx.x / 64;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) {
    before += (w < wid) ? wsum[w] : 0;
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_local(int32_t* __restrict__ data, int64_t n,
                                                             int32_t* __restrict__ tops) {
  int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  int v[kScanPer];
  int sum = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    v[i] = (base + i < n) ? data[base + i] : 0;
    sum += v[i];
  }
  int total;
  int run = block_excl_scan(sum, &total);
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    if (base + i < n) data[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == 0) tops[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tops(int32_t* __restrict__ tops, int64_t nb,
                                                            int32_t* __restrict__ grand) {
  int carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kScanBlock) {
    int64_t base = b0 + (int64_t)threadIdx.x * kScanPer;
    int v[kScanPer];
    int sum = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
      v[i] = (base + i < nb) ? tops[base + i] : 0;
      sum += v[i];
    }
    int total;
    int run = carry + block_excl_scan(sum, &total);
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
      if (base + i < nb) tops[base + i] = run;
      run += v[i];
    }
    carry += total;
  }
  if (threadIdx.x == 0 && grand) *grand = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int32_t* __restrict__ data, int64_t n,
                                                           const int32_t* __restrict__ tops) {
  int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  int add = tops[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanPer; ++i)
    if (base + i < n) data[base + i] += add;
}

}  // namespace

size_t scan_tmp_bytes(int64_t n) { return align_up(sizeof(int32_t) * (size_t)((n + kScanBlock - 1) / kScanBlock + 1), 256); }

void exclusive_scan_i32(int32_t* d_data, int64_t n, int32_t* d_total, void* d_tmp, hipStream_t s) {
  int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb == 0) nb = 1;
  int32_t* tops = (int32_t*)d_tmp;
  hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kScanThreads), 0, s, d_data, n, tops);
  hipLaunchKernelGGL(k_scan_tops, dim3(1), dim3(kScanThreads), 0, s, tops, nb, d_total);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, d_data, n, (const int32_t*)tops);
}

IndexLayout index_layout(int64_t n_padded) {
  IndexLayout L;
  size_t off = 0;
  L.key_off = off;
  off = align_up(off + sizeof(int64_t) * (kNKeys + 1), 256);
  L.occ = off;
  off = align_up(off + sizeof(int32_t) * (size_t)n_padded, 256);
  L.occ_seq = off;
  off = align_up(off + sizeof(int32_t) * (size_t)n_padded, 256);
  L.scan = off;
  off = align_up(off + (size_t)n_padded + kScanSlack, 256);
  L.total = off;
  return L;
}

// About 16K positions per wavefront, up to 16384 wavefronts (the per-chunk key
// counts then take 8800 x 16384 x 4 bytes of scratch at most).
constexpr int64_t kMaxChunks = 16384;

IndexChunks index_chunks(int64_t n_padded) {
  int64_t nch = (n_padded + 16383) / 16384;
  nch = nch < 1 ? 1 : (nch > kMaxChunks ? kMaxChunks : nch);
  int64_t chunk = (n_padded + nch - 1) / nch;
  chunk = (chunk + 63) / 64 * 64;
  if (chunk < 64) chunk = 64;
  IndexChunks c;
  c.chunk = chunk;
  c.nchunks = (int32_t)((n_padded + chunk - 1) / chunk);
  if (c.nchunks < 1) c.nchunks = 1;
  return c;
}

// workspace: [counters (256 B)] [counts: kNKeys * nchunks int32] [scan tops]
size_t index_ws_bytes(int64_t n_padded) {
  IndexChunks c = index_chunks(n_padded);
  int64_t n = (int64_t)kNKeys * c.nchunks;
  return 256 + align_up(sizeof(int32_t) * (size_t)n, 256) + scan_tmp_bytes(n);
}

int index_enqueue(const uint8_t* d_codes, const int64_t* d_seq_start, int32_t n_seqs, int64_t n_padded,
                  void* d_index, void* d_ws, int32_t* d_err, plast_index_t* out, hipStream_t stream) {
  IndexLayout L = index_layout(n_padded);
  IndexChunks C = index_chunks(n_padded);
  uint8_t* base = (uint8_t*)d_index;
  int64_t* key_off = (int64_t*)(base + L.key_off);
  int32_t* occ = (int32_t*)(base + L.occ);
  int32_t* occ_seq = (int32_t*)(base + L.occ_seq);
  uint8_t* scan = base + L.scan;
  int64_t scan_len = (int64_t)(L.total - L.scan);

  uint8_t* ws = (uint8_t*)d_ws;
  int32_t* total = d_err + 1;
  int64_t ncount = (int64_t)kNKeys * C.nchunks;
  int32_t* counts = (int32_t*)(ws + 256);
  void* tmp = ws + 256 + align_up(sizeof(int32_t) * (size_t)ncount, 256);

  SeedClasses sc = seed_classes();
  timing_mark(kStageIndex, false, stream);
  // a fill kernel rather than a memset node, so that the sequence can be captured in a graph
  hipLaunchKernelGGL(k_clear2, dim3(1), dim3(64), 0, stream, d_err);
  hipLaunchKernelGGL(k_layout_check, dim3((unsigned)((n_seqs + 1 + 255) / 256)), dim3(256), 0, stream, d_seq_start,
                     n_seqs, n_padded, d_err);
  hipLaunchKernelGGL(k_codes_check, dim3((unsigned)((scan_len + kCheckChunk - 1) / kCheckChunk)), dim3(kChunkWave), 0,
                     stream, d_codes, d_seq_start, n_seqs, n_padded, scan, scan_len, d_err);
  // Counting and scattering read seq_start only as bounds of a search over
  // [0, n_seqs), so they stay in bounds after a layout error.
  hipLaunchKernelGGL(k_index_count, dim3((unsigned)C.nchunks), dim3(kChunkWave), 0, stream, d_codes, n_padded,
                     C.chunk, C.nchunks, sc, counts);
  exclusive_scan_i32(counts, ncount, total, tmp, stream);
  hipLaunchKernelGGL(k_index_scatter, dim3((unsigned)C.nchunks), dim3(kChunkWave), 0, stream, d_codes,
                     d_seq_start, n_seqs, n_padded, C.chunk, C.nchunks, sc, (const int32_t*)counts, occ, occ_seq);
  hipLaunchKernelGGL(k_key_off, dim3((kNKeys + 1 + 255) / 256), dim3(256), 0, stream, (const int32_t*)counts,
                     C.nchunks, (const int32_t*)total, key_off);
  timing_mark(kStageIndex, true, stream);
  PLAST_HIP(hipGetLastError());

  out->codes = d_codes;
  out->seq_start = d_seq_start;
  out->n_seqs = n_seqs;
  out->n_padded = n_padded;
  out->key_off = key_off;
  out->occ = occ;
  out->occ_seq = occ_seq;
  out->scan_codes = scan;
  out->n_words = -1;
  return PLAST_OK;
}

int build_index_impl(const uint8_t* d_codes, const int64_t* d_seq_start, int32_t n_seqs, int64_t n_padded,
                     void* d_index, void* d_ws, plast_index_t* out, hipStream_t stream) {
  int32_t* err = (int32_t*)d_ws;  // [0] error bits, [1] word total
  plast_index_t view;
  int rc = index_enqueue(d_codes, d_seq_start, n_seqs, n_padded, d_index, d_ws, err, &view, stream);
  if (rc != PLAST_OK) return rc;
  int32_t h_err[2] = {0, 0};
  PLAST_HIP(hipMemcpyAsync(h_err, err, sizeof(h_err), hipMemcpyDeviceToHost, stream));
  PLAST_HIP(hipStreamSynchronize(stream));
  if (h_err[0] & 1) return set_error(PLAST_E_LAYOUT, "seq_start does not describe the padded layout");
  if (h_err[0] & 2) return set_error(PLAST_E_ALPHABET, "a residue code is > 19 or a separator code is not 20");
  view.n_words = h_err[1];
  *out = view;
  return PLAST_OK;
}

}  // namespace plast
