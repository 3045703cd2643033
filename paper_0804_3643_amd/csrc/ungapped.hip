// Stage 2, ungapped extension (Sec. 3.2 generic algorithm, Sec. 3.3.3), with
// hit compaction and two schedules over the same tile routine.
//
// Tile routine.  A work item is (key, 32 bank-a occurrences, up to 16384 bank-b
// occurrences; the width is set per size class of the key).  The 32 rows become a profile in LDS: for scan step t (t < 24:
// letter p+t; t >= 24: letter p-(t-23)) and bank-b letter c, an 8-byte entry
// holds the substitution scores of four rows (59 KB for 32 rows x 44 steps x 21
// letters).  Each lane owns one bank-b occurrence at a time: its 44-letter
// window sits in 11 registers as (letter * 8) bytes, so one bit-field extract
// gives the LDS address of the entry and eight 8-byte LDS reads give the scores
// of all 32 rows (an item with at most 4, 8, 12 or 16 rows, such as the last
// row tile of a key, builds and scans only that many rows, in 4-row groups).
// Running sums and running bests are packed pairs, two rows per register.  At step 24 the running sum is reset to the running best, so the
// best leftward prefix is added to the best rightward prefix (the composition of
// the GPU kernel of Annex 4).  Letters outside a sequence are separators scoring
// kSepScore <= 0 against everything; the separator run after a sequence is at
// least as long as the scan, so a scan that leaves its sequence only meets
// separators and its best prefix is the clipped one.
//
// Two arithmetic variants give identical integers:
//   * f16 (used when |M| <= 23, which covers BLOSUM62): every partial sum is an
//     integer of magnitude <= 44 * 23 < 1024, exactly representable in binary16,
//     so packed f16 adds are exact; two steps cost two v_pk_add_f16 and one
//     v_pk_maximum3_f16 per register;
//   * int16 (any int8 matrix): v_pk_add_u16 / v_pk_max_i16, one add and one max
//     per step and register.
//
// Hits: a 32-bit row mask per lane comes from the sign bits of (threshold -
// best), rotated into place; hits are staged in LDS and written out once per
// item with one global atomic (a wavefront whose reservation does not fit the
// staging area writes directly).  Order of hits is unspecified.
//
// Schedules.  PLAIN: one grid per key with candidate pairs, in key order, one
// item of 4096 columns per workgroup (the paper's one-launch-per-seed GPU
// offload, Sec. 5.2.1, without its per-seed copies).  BATCHED: a device work
// list over all keys, item widths chosen per size class of n2, and one
// persistent kernel whose workgroups pop items from atomic counters (the
// dynamic seed distribution of the multicore version, Sec. 5.1).  The list is
// in key order with the row tiles of one column range next to each other, so
// consecutive items read the same bank-b windows; with one queue per XCD each
// XCD works through its own contiguous part of the list under its own L2, and
// a workgroup whose queue is empty takes items from the others.
#include <stddef.h>
#include <string.h>

#include <mutex>
#include <type_traits>
#include <vector>

#include "plast_internal.h"

namespace plast {

namespace {

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));

constexpr int kSepScore = -4;
constexpr int kF16MaxEntry = 23;                  // 44 * 23 = 1012 < 1024
constexpr int kProfT = kNLet * 8;                 // bytes per scan step
constexpr int kProfRG = kSpan * kProfT;           // bytes per 4-row group
constexpr int kProfBytes = kRowGroups * kProfRG;  // 59136
constexpr int kPairs = 2 * kRowGroups;            // packed registers per lane (16)
static_assert(kProfBytes + 4096 < 65536, "profile offsets must fit the LDS instruction offset field");
static_assert(kPadCode * kScale < 256, "scaled codes must fit a byte");
static_assert(kTileRows == 32 && kPairs == 16, "row mask layout assumes at most 32 rows");
static_assert(kSpan * kF16MaxEntry < 1024, "f16 partial sums must stay exact");

struct BankView {
  const int64_t* key_off;
  const int32_t* occ;
  const int32_t* occ_seq;
  const uint8_t* scan;
  const int64_t* seq_start;
};

struct UngappedArgs {
  BankView a, b;
  uint32_t thr;                // packed pair: threshold - 1 (int16) or threshold - 0.5 (f16)
  int32_t s1;
  plast_hit_t* hits;
  int64_t capacity;
  unsigned long long* n_hits;
  int16_t mat[kNLet * kNLet];  // [a letter][b letter], separator row/column = kSepScore
};

// Hits found in an item are staged in LDS as (row | score << 5, seq2, pos2).
constexpr int kHitSlots = 1024;

struct __align__(16) Smem {
  uint8_t prof[kProfBytes];            // 8-byte entries (offset 0)
  uint8_t rowlet[kSpan * kTileRows];   // read as 4-byte groups
  int32_t rowq[kTileRows];
  int32_t rowseq[kTileRows];
  int32_t rowpos[kTileRows];
  uint32_t hit_rs[kHitSlots];          // row | score << 5
  int32_t hit_seq[kHitSlots];
  int32_t hit_pos[kHitSlots];
  int32_t n_hit;                       // slots reserved so far in this item
  int32_t n_fit;                       // start of the reservation that straddles the end of the staging
                                       // area (kHitSlots if none)
  int32_t n_flush;                     // staged hits of the item being flushed
  int32_t item;
  unsigned long long hit_base;
  uint16_t mat[kNLet * kNLet];         // profile values (int16 or binary16 bits)
};
static_assert(offsetof(Smem, rowlet) % 16 == 0 && offsetof(Smem, rowq) % 4 == 0, "LDS alignment");

template <bool F16>
using vec2 = typename std::conditional<F16, h16x2, s16x2>::type;

template <bool F16>
__device__ __forceinline__ vec2<F16> as_vec(uint32_t v) {
  return __builtin_bit_cast(vec2<F16>, v);
}

template <bool F16>
__device__ __forceinline__ vec2<F16> vmax(vec2<F16> a, vec2<F16> b) {
  if constexpr (F16)
    return __builtin_elementwise_maximum(a, b);
  else
    return __builtin_elementwise_max(a, b);
}

template <bool F16>
__device__ __forceinline__ vec2<F16> vmax3(vec2<F16> a, vec2<F16> b, vec2<F16> c) {
  if constexpr (F16) {
    // the compiler fuses the nested maxima into one v_pk_maximum3_f16
    return __builtin_elementwise_maximum(__builtin_elementwise_maximum(a, b), c);
  } else {
    return __builtin_elementwise_max(a, __builtin_elementwise_max(b, c));
  }
}

template <bool F16>
__device__ __forceinline__ int to_int(vec2<F16> v, int half) {
  return half ? (int)v.y : (int)v.x;
}

template <bool F16>
__device__ __forceinline__ void smem_init(const UngappedArgs& A, Smem& S) {
  for (int i = threadIdx.x; i < kNLet * kNLet; i += kThreads) {
    if constexpr (F16)
      S.mat[i] = __builtin_bit_cast(uint16_t, (_Float16)A.mat[i]);
    else
      S.mat[i] = (uint16_t)A.mat[i];
  }
  if (threadIdx.x == 0) {
    S.n_hit = 0;
    S.n_fit = kHitSlots;
  }
}

// Rows of the tile (bank-a occurrences row0 .. row0+rows-1 of the key) and
// the 44-step profile of its first `groups` 4-row groups (rows past `rows`
// hold separators).  Called by all threads (contains barriers).
__device__ __forceinline__ void build_profile(const UngappedArgs& A, const WorkItem& it, int64_t a0, int rows,
                                              int groups, Smem& S) {
  const int tid = threadIdx.x;
  if (tid < kTileRows) {
    int q = -1, sq = 0, ps = 0;
    if (tid < rows) {
      int64_t o = a0 + it.row0 + tid;
      q = A.a.occ[o];
      sq = A.a.occ_seq[o];
      ps = q - (int)A.a.seq_start[sq];
    }
    S.rowq[tid] = q;
    S.rowseq[tid] = sq;
    S.rowpos[tid] = ps;
  }
  __syncthreads();
  const int nr = 4 * groups;
  for (int idx = tid; idx < kSpan * nr; idx += kThreads) {
    int t = idx / nr, r = idx - t * nr;
    int q = S.rowq[r];
    int letter = kPadCode;
    if (q >= 0) {
      int off = t < kRight ? q + t : q - (t - kRight + 1);
      letter = A.a.scan[off] / kScale;
    }
    S.rowlet[t * kTileRows + r] = (uint8_t)letter;
  }
  __syncthreads();
  // prof[rg][t][c] = scores of rows 4rg..4rg+3 at step t against bank-b letter c
  for (int e = tid; e < groups * kSpan * kNLet; e += kThreads) {
    int rg = e / (kSpan * kNLet);
    int rem = e - rg * (kSpan * kNLet);
    int t = rem / kNLet;
    int c = rem - t * kNLet;
    uint32_t l4 = *(const uint32_t*)&S.rowlet[t * kTileRows + 4 * rg];
    uint32_t v0 = S.mat[(l4 & 0xff) * kNLet + c];
    uint32_t v1 = S.mat[((l4 >> 8) & 0xff) * kNLet + c];
    uint32_t v2 = S.mat[((l4 >> 16) & 0xff) * kNLet + c];
    uint32_t v3 = S.mat[(l4 >> 24) * kNLet + c];
    uint2 w;
    w.x = v0 | (v1 << 16);
    w.y = v2 | (v3 << 16);
    *(uint2*)&S.prof[rg * kProfRG + t * kProfT + c * 8] = w;
  }
  __syncthreads();
}

// The 44-step scan of one bank-b window against the first 4 RG profile rows.
// win: the window as (letter * 8) bytes, byte b = position q - 20 + b.
// m receives best-right + best-left of every row (register i: rows 2i, 2i+1).
template <bool F16, int RG>
__device__ __forceinline__ void scan_window(const Smem& S, const uint32_t (&win)[11], vec2<F16> (&m)[2 * RG]) {
  typedef vec2<F16> V;
  constexpr int NP = 2 * RG;
  V s[NP];
  uint2 cur[RG], nxt[RG];
  auto load = [&](int t, uint2(&dst)[RG]) {
    const int bidx = t < kRight ? kNbr + t : (kSpan - 1) - t;
    const uint32_t c8 = (win[bidx >> 2] >> (8 * (bidx & 3))) & 0xffu;
    const uint8_t* p = S.prof + c8 + t * kProfT;
#pragma unroll
    for (int rg = 0; rg < RG; ++rg) dst[rg] = *(const uint2*)(p + rg * kProfRG);
  };
  auto val = [&](const uint2(&src)[RG], int i) {
    return as_vec<F16>((i & 1) ? src[i >> 1].y : src[i >> 1].x);
  };
  const V zero = {0, 0};
  load(0, cur);
  load(1, nxt);
#pragma unroll
  for (int i = 0; i < NP; ++i) s[i] = val(cur, i);
#pragma unroll
  for (int rg = 0; rg < RG; ++rg) cur[rg] = nxt[rg];
  // Steps 1 .. 43; the scores of step t are in cur when step t is applied.
#pragma unroll
  for (int t = 1; t < kSpan; ++t) {
    if (t + 1 < kSpan) load(t + 1, nxt);
    if (t == kRight) {
#pragma unroll
      for (int i = 0; i < NP; ++i) s[i] = m[i];  // best right prefix, then left
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const V prev = s[i];
      s[i] = prev + val(cur, i);
      if constexpr (F16) {
        // Running best after every odd step: right prefixes (0,1) with the
        // empty prefix, (2,3), ..., (22,23); after the reset the left prefixes
        // (24,25), ..., (42,43).  Every prefix sum enters one 3-way maximum.
        if (t == 1)
          m[i] = vmax3<F16>(zero, prev, s[i]);
        else if (t & 1)
          m[i] = vmax3<F16>(m[i], prev, s[i]);
      } else {
        if (t == 1) m[i] = vmax<F16>(prev, zero);
        m[i] = vmax<F16>(m[i], s[i]);
      }
    }
    if (t + 1 < kSpan) {
#pragma unroll
      for (int rg = 0; rg < RG; ++rg) cur[rg] = nxt[rg];
    }
  }
}

// Bit layout of the row mask: row r is bit 8 (r & 3) + (r >> 2), so that the
// sign bits of four rows (two registers) land in one byte-permuted dword at
// bits 7, 15, 23, 31 and one shift and one and-or place them (hit_mask).
__host__ __device__ constexpr uint32_t row_bit(int r) { return 1u << (8 * (r & 3) + (r >> 2)); }

__device__ __forceinline__ uint32_t valid_rows_mask(int rows) {
  uint32_t m = 0;
#pragma unroll
  for (int r = 0; r < kTileRows; ++r)
    if (r < rows) m |= row_bit(r);
  return m;
}

template <bool F16, int RG>
__device__ __forceinline__ uint32_t hit_mask(uint32_t thr, const vec2<F16> (&m)[2 * RG]) {
  typedef vec2<F16> V;
  const V th = as_vec<F16>(thr);
  uint32_t d[2 * RG];
#pragma unroll
  for (int i = 0; i < 2 * RG; ++i) d[i] = __builtin_bit_cast(uint32_t, th - m[i]);  // negative where best >= s1
  uint32_t mask = 0;
#pragma unroll
  for (int k = 0; k < RG; ++k) {
    // the high bytes of both halves of registers 2k and 2k + 1: the sign bits
    // of rows 4k .. 4k + 3 at bits 7, 15, 23, 31
    const uint32_t w = __builtin_amdgcn_perm(d[2 * k + 1], d[2 * k], 0x07050301u);
    mask |= (w >> (7 - k)) & (0x01010101u << k);
  }
  return mask;
}

// Hit rows of this lane in register order (rows 2i and 2i+1 from register i);
// every register index is a compile-time constant, and a block whose bits are
// clear in every lane of the wavefront is skipped as a whole.
// `any` is the OR of every lane's mask, so the test of a register is a
// scalar branch and only the registers that hold a hit in some lane cost
// vector instructions.
template <bool F16, int RG, typename Put>
__device__ __forceinline__ void for_each_hit(const vec2<F16> (&m)[2 * RG], uint32_t mask, uint32_t any, Put put) {
#pragma unroll
  for (int i = 0; i < 2 * RG; ++i) {
    const uint32_t lo = row_bit(2 * i), hi = row_bit(2 * i + 1);
    if (any & (lo | hi)) {
      if (mask & lo) put(2 * i, to_int<F16>(m[i], 0));
      if (mask & hi) put(2 * i + 1, to_int<F16>(m[i], 1));
    }
  }
}

// OR of v over the wavefront: an inclusive OR-scan of each row of 16 lanes
// (wavefront DPP row shifts), then the row totals broadcast down (row_bcast
// 15 and 31); lane 63 holds the result.
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
  int x = (int)v;
  x |= __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x |= __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x |= __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x |= __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x |= __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x |= __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane(x, 63);
}

// Each lane with hits reserves its slots with one LDS atomic (hits are rare:
// a few lanes of a wavefront per column).  Reservations grow monotonically,
// so the ones that fit form a prefix of the staging area; the one that
// straddles its end (at most one) records where the prefix stops, and it and
// every later one write their hits directly.
template <bool F16, int RG>
__device__ __forceinline__ void emit_hits(const UngappedArgs& A, Smem& S, const vec2<F16> (&m)[2 * RG],
                                          uint32_t mask, int s2, int p2) {
  const uint32_t any = wave_or(mask);  // every lane of the wavefront takes part
  if (!any || !mask) return;
  const int cnt = __popc(mask);
  int at = atomicAdd(&S.n_hit, cnt);
  if (at + cnt <= kHitSlots) {  // staged in LDS
    for_each_hit<F16, RG>(m, mask, any, [&](int r, int score) {
      S.hit_rs[at] = (uint32_t)r | ((uint32_t)score << 5);
      S.hit_seq[at] = s2;
      S.hit_pos[at] = p2;
      ++at;
    });
  } else {  // staging area full: write directly
    if (at < kHitSlots) S.n_fit = at;
    unsigned long long g = atomicAdd(A.n_hits, (unsigned long long)cnt);
    for_each_hit<F16, RG>(m, mask, any, [&](int r, int score) {
      if (g < (unsigned long long)A.capacity) {
        plast_hit_t h;
        h.seq1 = S.rowseq[r];
        h.pos1 = S.rowpos[r];
        h.seq2 = s2;
        h.pos2 = p2;
        h.score = score;
        A.hits[g] = h;
      }
      ++g;
    });
  }
}

// Called by all threads (contains barriers); ends with a barrier so the next
// item may overwrite the staging area and the row data.
__device__ __forceinline__ void flush_hits(const UngappedArgs& A, Smem& S) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const int n = min(S.n_hit, S.n_fit);
    S.n_flush = n;
    S.hit_base = n ? atomicAdd(A.n_hits, (unsigned long long)n) : 0ull;
    S.n_hit = 0;
    S.n_fit = kHitSlots;
  }
  __syncthreads();
  const int n = __builtin_amdgcn_readfirstlane(S.n_flush);
  const unsigned long long base = S.hit_base;
  for (int e = threadIdx.x; e < n; e += kThreads) {
    if (base + e < (unsigned long long)A.capacity) {
      const uint32_t rs = S.hit_rs[e];
      plast_hit_t h;
      h.seq1 = S.rowseq[rs & 31u];
      h.pos1 = S.rowpos[rs & 31u];
      h.seq2 = S.hit_seq[e];
      h.pos2 = S.hit_pos[e];
      h.score = (int)(rs >> 5);
      A.hits[base + e] = h;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void load_window_raw(const UngappedArgs& A, int q2, uint32_t (&raw)[12]) {
  const uint32_t* src = (const uint32_t*)A.b.scan + ((q2 - kNbr) >> 2);
#pragma unroll
  for (int i = 0; i < 12; ++i) raw[i] = src[i];
}

// The item's columns against its first 4 RG rows (rows <= 4 RG), then the
// flush of its hits.  Called by all threads (contains barriers).
template <bool F16, int RG>
__device__ void run_tile(const UngappedArgs& A, const WorkItem& it, int64_t a0, int64_t b0, int rows, Smem& S) {
  const int tid = threadIdx.x;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t valid = valid_rows_mask(rows);
  build_profile(A, it, a0, rows, RG, S);

  // Lane columns: col0 + tid + kThreads * k.  Column data is software-pipelined:
  // the occurrence two columns ahead and the window one column ahead are in
  // flight while the current column is scanned.
  const int col_end = it.col0 + it.ncols;
  int nk = 0;  // column steps of this wavefront
  while (nk < kMaxColsPerLane && it.col0 + wid * 64 + kThreads * nk < col_end) ++nk;
  nk = __builtin_amdgcn_readfirstlane(nk);
  auto occ_index = [&](int k) {
    const int j = it.col0 + tid + kThreads * k;
    return b0 + (j < col_end ? j : it.col0);
  };
  int q_cur = 0, s_cur = 0, q_nxt = 0, s_nxt = 0;
  uint32_t raw[12];
  if (nk > 0) {
    const int64_t o = occ_index(0);
    q_cur = A.b.occ[o];
    s_cur = A.b.occ_seq[o];
    load_window_raw(A, q_cur, raw);
  }
  if (nk > 1) {
    const int64_t o = occ_index(1);
    q_nxt = A.b.occ[o];
    s_nxt = A.b.occ_seq[o];
  }
  for (int k = 0; k < nk; ++k) {
    const bool active = it.col0 + tid + kThreads * k < col_end;
    const int q2 = q_cur, s2 = s_cur;
    uint32_t win[11];
    const int sh = (q2 - kNbr) & 3;
#pragma unroll
    for (int i = 0; i < 11; ++i) win[i] = __builtin_amdgcn_alignbyte(raw[i + 1], raw[i], sh);
    if (k + 1 < nk) {
      load_window_raw(A, q_nxt, raw);
      q_cur = q_nxt;
      s_cur = s_nxt;
    }
    if (k + 2 < nk) {
      const int64_t o = occ_index(k + 2);
      q_nxt = A.b.occ[o];
      s_nxt = A.b.occ_seq[o];
    }
    const int st2 = (int)A.b.seq_start[s2];
    vec2<F16> m[2 * RG];
    scan_window<F16, RG>(S, win, m);
    const uint32_t mask = active ? (hit_mask<F16, RG>(A.thr, m) & valid) : 0u;
    emit_hits<F16, RG>(A, S, m, mask, s2, q2 - st2);
  }
  flush_hits(A, S);
}

// All threads of the workgroup call run_item with the same item (it contains
// barriers); every branch around a barrier depends only on wave-uniform values.
// A tile with at most 4, 8, 12 or 16 rows (the last row tile of a key, and
// most tiles of a small query bank) scans only 1, 2, 3 or 4 row groups.
template <bool F16>
__device__ void run_item(const UngappedArgs& A, const WorkItem it, Smem& S) {
  const int64_t a0 = A.a.key_off[it.key];
  const int n1 = (int)(A.a.key_off[it.key + 1] - a0);
  const int rows = __builtin_amdgcn_readfirstlane(min(kTileRows, n1 - it.row0));
  const int64_t b0 = A.b.key_off[it.key];
  if (rows <= 4)
    run_tile<F16, 1>(A, it, a0, b0, rows, S);
  else if (rows <= 8)
    run_tile<F16, 2>(A, it, a0, b0, rows, S);
  else if (rows <= 12)
    run_tile<F16, 3>(A, it, a0, b0, rows, S);
  else if (rows <= 16)
    run_tile<F16, 4>(A, it, a0, b0, rows, S);
  else
    run_tile<F16, kRowGroups>(A, it, a0, b0, rows, S);
}

constexpr int kPlainCols = 4096;  // item width of the PLAIN schedule

template <bool F16>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_ungapped_plain(UngappedArgs A, int32_t key, int32_t n_row_tiles, int32_t n2) {
  __shared__ Smem S;
  smem_init<F16>(A, S);
  __syncthreads();
  WorkItem it;
  it.key = key;
  it.row0 = (int32_t)(blockIdx.x % n_row_tiles) * kTileRows;
  it.col0 = (int32_t)(blockIdx.x / n_row_tiles) * kPlainCols;
  it.ncols = min(kPlainCols, n2 - it.col0);
  run_item<F16>(A, it, S);
}

// Workspace header of the BATCHED schedule: UngappedCounters at 0, queue
// counters at 32 (kMaxQueues int32), both cleared by the first kernel.
constexpr int kCtrOffset = 32;
constexpr int kHeaderDwords = 16;
static_assert(sizeof(UngappedCounters) <= kCtrOffset, "counter header");
static_assert(kCtrOffset + 4 * kMaxQueues <= 4 * kHeaderDwords, "queue counters");

template <bool F16>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_ungapped_persistent(UngappedArgs A, const WorkItem* __restrict__ items,
                           const UngappedCounters* __restrict__ cnt, int32_t* __restrict__ ctr, int32_t n_queues) {
  __shared__ Smem S;
  smem_init<F16>(A, S);
  const int n_items = __builtin_amdgcn_readfirstlane(cnt->overflow ? 0 : cnt->n_items);
  const int q0 = (int)(blockIdx.x % (unsigned)n_queues);  // workgroups are dealt to XCDs round robin
  for (int j = 0; j < n_queues; ++j) {
    const int q = (q0 + j) % n_queues;
    const int beg = (int)((int64_t)n_items * q / n_queues), end = (int)((int64_t)n_items * (q + 1) / n_queues);
    // The item index is read back as a scalar so that the loop exit is
    // uniform: with a per-lane exit the compiler may let lanes other than
    // thread 0 reach a barrier before thread 0 has fetched the next item.  The
    // second barrier keeps thread 0 from overwriting S.item (next item or next
    // queue) before every wavefront has read it.
    for (;;) {
      if (threadIdx.x == 0) S.item = atomicAdd(&ctr[q], 1);
      __syncthreads();
      const int i = __builtin_amdgcn_readfirstlane(S.item) + beg;
      __syncthreads();
      if (i >= end) break;
      run_item<F16>(A, items[i], S);
    }
  }
}

// ---------------------------------------------------------------- planning
// Size classes by n2 and the item width of each, for the planning kernels.
struct PlanShape {
  int32_t min_n2[kClasses];
  int32_t cols[kClasses];
  uint32_t mask;  // classes that get items
};

__host__ __device__ __forceinline__ int64_t items_of(const PlanShape& P, int64_t n1, int64_t n2, int32_t* width) {
  if (n1 <= 0 || n2 <= 0) return 0;
  int c = 0;
#pragma unroll
  for (int i = 1; i < kClasses; ++i)
    if (n2 >= P.min_n2[i]) c = i;
  if (!((P.mask >> c) & 1u)) return 0;
  *width = P.cols[c];
  return ((n1 + kTileRows - 1) / kTileRows) * ((n2 + P.cols[c] - 1) / P.cols[c]);
}

__global__ void k_plan_count(const int64_t* __restrict__ a_off, const int64_t* __restrict__ b_off, PlanShape P,
                             int32_t* __restrict__ keycnt, UngappedCounters* __restrict__ cnt) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kNKeys) return;
  int64_t n1 = a_off[k + 1] - a_off[k], n2 = b_off[k + 1] - b_off[k];
  int32_t w = 0;
  const int64_t c = items_of(P, n1, n2, &w);
  keycnt[k] = (int32_t)min(c, (int64_t)INT32_MAX);
  if (c > 0) {
    atomicAdd(&cnt->n_ext, (unsigned long long)(n1 * n2));
    atomicAdd(&cnt->n_items64, (unsigned long long)c);
  }
}

__global__ void k_plan_emit(const int64_t* __restrict__ a_off, const int64_t* __restrict__ b_off, PlanShape P,
                            const int32_t* __restrict__ item_off, UngappedCounters* __restrict__ cnt,
                            int64_t max_items, const int32_t* __restrict__ err_a, const int32_t* __restrict__ err_b,
                            WorkItem* __restrict__ items) {
  const int k = blockIdx.x;
  const unsigned long long n = cnt->n_items64;
  const int flag = (n > (unsigned long long)max_items || n > (unsigned long long)INT32_MAX)
                       ? 1
                       : (((err_a && *err_a) || (err_b && *err_b)) ? 2 : 0);
  if (flag) {
    if (k == 0 && threadIdx.x == 0) cnt->overflow = flag;
    return;
  }
  int64_t n1 = a_off[k + 1] - a_off[k], n2 = b_off[k + 1] - b_off[k];
  int32_t width = 0;
  const int ni = (int)items_of(P, n1, n2, &width);
  if (ni == 0) return;
  const int nrt = (int)((n1 + kTileRows - 1) / kTileRows);
  for (int idx = threadIdx.x; idx < ni; idx += blockDim.x) {
    const int rt = idx % nrt, ct = idx / nrt;  // row tiles of one column range are adjacent
    WorkItem w;
    w.key = k;
    w.row0 = rt * kTileRows;
    w.col0 = ct * width;
    w.ncols = (int)min((int64_t)width, n2 - (int64_t)w.col0);
    items[item_off[k] + idx] = w;
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- workspace
// [0, 256): UngappedCounters, queue counters
// [256, ...): per-key item counts/offsets (int32[kNKeys]), scan scratch, items
struct UngappedWs {
  UngappedCounters* cnt;
  int32_t* ctr;
  int32_t* keycnt;
  void* scan_tmp;
  WorkItem* items;
  int64_t max_items;
};

UngappedWs carve(void* d_ws, size_t ws_bytes) {
  UngappedWs W;
  uint8_t* p = (uint8_t*)d_ws;
  W.cnt = (UngappedCounters*)p;
  W.ctr = (int32_t*)(p + kCtrOffset);
  W.keycnt = (int32_t*)(p + 256);
  W.scan_tmp = p + 256 + align_up(sizeof(int32_t) * kNKeys, 256);
  W.items = (WorkItem*)(p + ungapped_ws_fixed_bytes());
  W.max_items = ungapped_ws_max_items(ws_bytes);
  return W;
}

PlanShape shape_of(const plast_tuning_t& t, uint32_t mask) {
  PlanShape P;
  for (int c = 0; c < kClasses; ++c) {
    P.min_n2[c] = t.class_min_n2[c];
    P.cols[c] = t.item_cols[c];
  }
  P.mask = mask;
  return P;
}

// Returns true when the f16 variant is exact for this matrix.
bool fill_args(UngappedArgs& A, const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
               plast_hit_t* d_hits, int64_t capacity, unsigned long long* n_hits) {
  A.a = BankView{a->key_off, a->occ, a->occ_seq, a->scan_codes, a->seq_start};
  A.b = BankView{b->key_off, b->occ, b->occ_seq, b->scan_codes, b->seq_start};
  A.s1 = p->s1;
  A.hits = d_hits;
  A.capacity = capacity;
  A.n_hits = n_hits;
  int8_t m[400];
  if (p->matrix)
    memcpy(m, p->matrix, sizeof(m));
  else
    blosum62_code_order(m);
  int maxabs = -kSepScore;
  for (int x = 0; x < kNLet; ++x)
    for (int y = 0; y < kNLet; ++y) {
      A.mat[x * kNLet + y] = (x < 20 && y < 20) ? m[x * 20 + y] : kSepScore;
      maxabs = max(maxabs, abs((int)A.mat[x * kNLet + y]));
    }
  const bool f16 = maxabs <= kF16MaxEntry;
  // Threshold register: hit iff thr - best < 0.  Scores lie in [0, 44 * maxabs].
  if (f16) {
    // best is an integer in [0, 1012]: thr = s1 - 1/2 clamped to [-1/2, 1012.5], exact in binary16
    const float t = (float)min(max(p->s1, 0), kSpan * kF16MaxEntry + 1) - 0.5f;
    const uint16_t h = __builtin_bit_cast(uint16_t, (_Float16)t);
    A.thr = (uint32_t)h | ((uint32_t)h << 16);
  } else {
    const int t = min(max(p->s1, -20000), 20000) - 1;
    const uint16_t h = (uint16_t)(int16_t)t;
    A.thr = (uint32_t)h | ((uint32_t)h << 16);
  }
  return f16;
}

template <bool F16>
int persistent_grid() {
  static int cached = 0;
  if (!cached) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_ungapped_persistent<F16>, kThreads, 0) != hipSuccess)
      return 0;
    cached = cus * (per > 0 ? per : 1);
  }
  return cached;
}

}  // namespace

void tuning_default(plast_tuning_t* t) {
  const int32_t lo[kClasses] = {1, 2048, 8192, 32768};
  for (int c = 0; c < kClasses; ++c) {
    t->class_min_n2[c] = lo[c];
    t->item_cols[c] = 4096;
  }
  t->xcd_queues = 1;
  t->gapped_threads = 256;
}

int check_tuning(const plast_tuning_t* t) {
  if (t->class_min_n2[0] != 1) return set_error(PLAST_E_ARG, "tuning: class_min_n2[0] must be 1");
  for (int c = 0; c < kClasses; ++c) {
    if (c > 0 && t->class_min_n2[c] <= t->class_min_n2[c - 1])
      return set_error(PLAST_E_ARG, "tuning: class_min_n2 must be strictly ascending");
    const int w = t->item_cols[c];
    if (w < kThreads || w > kMaxItemCols || w % kThreads)
      return set_error(PLAST_E_ARG, "tuning: item_cols[%d]=%d not a multiple of %d in [%d, %d]", c, w, kThreads,
                       kThreads, kMaxItemCols);
  }
  if (t->xcd_queues != 1 && t->xcd_queues != kMaxQueues)
    return set_error(PLAST_E_ARG, "tuning: xcd_queues must be 1 or %d", kMaxQueues);
  if (t->gapped_threads != 128 && t->gapped_threads != 256 && t->gapped_threads != 512)
    return set_error(PLAST_E_ARG, "tuning: gapped_threads must be 128, 256 or 512");
  return PLAST_OK;
}

int ungapped_prepare() {
  return (persistent_grid<true>() > 0 && persistent_grid<false>() > 0)
             ? PLAST_OK
             : set_error(PLAST_E_HIP, "cannot query device occupancy");
}

size_t ungapped_ws_fixed_bytes() { return 256 + align_up(sizeof(int32_t) * kNKeys, 256) + scan_tmp_bytes(kNKeys); }

int64_t ungapped_ws_max_items(size_t ws_bytes) {
  const size_t f = ungapped_ws_fixed_bytes();
  return ws_bytes > f ? (int64_t)((ws_bytes - f) / sizeof(WorkItem)) : 0;
}

const void* ungapped_counters_dev(const void* d_ws) { return d_ws; }
unsigned long long* ungapped_n_hits_dev(void* d_ws) { return &((UngappedCounters*)d_ws)->n_hits; }

int read_key_offsets(const plast_index_t* x, int64_t* h, hipStream_t s) {
  PLAST_HIP(hipMemcpyAsync(h, x->key_off, sizeof(int64_t) * (kNKeys + 1), hipMemcpyDeviceToHost, s));
  PLAST_HIP(hipStreamSynchronize(s));
  return PLAST_OK;
}

int64_t plan_items_host(const int64_t* ha, const int64_t* hb, const plast_tuning_t& t, uint32_t class_mask,
                        int64_t* n_ext) {
  const PlanShape P = shape_of(t, class_mask);
  int64_t items = 0, ext = 0;
  for (int k = 0; k < kNKeys; ++k) {
    const int64_t n1 = ha[k + 1] - ha[k], n2 = hb[k + 1] - hb[k];
    int32_t w = 0;
    const int64_t c = items_of(P, n1, n2, &w);
    if (c > 0) ext += n1 * n2;
    items += c;
  }
  if (n_ext) *n_ext = ext;
  return items;
}

int ungapped_ws_bytes_impl(const plast_index_t* a, const plast_index_t* b, int32_t mode, const plast_tuning_t& t,
                           size_t* bytes, int64_t* n_ext, int64_t* n_items, hipStream_t stream) {
  std::vector<int64_t> ha(kNKeys + 1), hb(kNKeys + 1);
  int rc;
  if ((rc = read_key_offsets(a, ha.data(), stream)) || (rc = read_key_offsets(b, hb.data(), stream))) return rc;
  const int64_t items = plan_items_host(ha.data(), hb.data(), t, ~0u, n_ext);
  if (n_items) *n_items = items;
  *bytes = mode == PLAST_BATCHED ? ungapped_ws_fixed_bytes() + sizeof(WorkItem) * (size_t)items : 256;
  if (items > INT32_MAX) return set_error(PLAST_E_ARG, "too many work items");
  return PLAST_OK;
}

int ungapped_enqueue_batched(const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                             const plast_tuning_t& t, uint32_t class_mask, void* d_ws, size_t ws_bytes,
                             plast_hit_t* d_hits, int64_t capacity, const int32_t* err_a, const int32_t* err_b,
                             hipEvent_t ev0, hipEvent_t ev1, hipStream_t stream) {
  if (ws_bytes < ungapped_ws_fixed_bytes())
    return set_error(PLAST_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, ungapped_ws_fixed_bytes());
  UngappedWs W = carve(d_ws, ws_bytes);
  UngappedArgs A;
  const bool f16 = fill_args(A, a, b, p, d_hits, capacity, &W.cnt->n_hits);
  const int grid = f16 ? persistent_grid<true>() : persistent_grid<false>();
  if (grid <= 0) return set_error(PLAST_E_HIP, "cannot query device occupancy");
  const PlanShape P = shape_of(t, class_mask);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, (uint32_t*)d_ws, (int64_t)kHeaderDwords, 0u);
  timing_mark(kStagePlan, false, stream);
  hipLaunchKernelGGL(k_plan_count, dim3((kNKeys + 255) / 256), dim3(256), 0, stream, a->key_off, b->key_off, P,
                     W.keycnt, W.cnt);
  exclusive_scan_i32(W.keycnt, kNKeys, &W.cnt->n_items, W.scan_tmp, stream);
  hipLaunchKernelGGL(k_plan_emit, dim3(kNKeys), dim3(256), 0, stream, a->key_off, b->key_off, P,
                     (const int32_t*)W.keycnt, W.cnt, W.max_items, err_a, err_b, W.items);
  timing_mark(kStagePlan, true, stream);
  timing_mark(kStageUngapped, false, stream);
  if (ev0) PLAST_HIP(hipEventRecord(ev0, stream));
  if (f16)
    hipLaunchKernelGGL(k_ungapped_persistent<true>, dim3(grid), dim3(kThreads), 0, stream, A,
                       (const WorkItem*)W.items, (const UngappedCounters*)W.cnt, W.ctr, (int32_t)t.xcd_queues);
  else
    hipLaunchKernelGGL(k_ungapped_persistent<false>, dim3(grid), dim3(kThreads), 0, stream, A,
                       (const WorkItem*)W.items, (const UngappedCounters*)W.cnt, W.ctr, (int32_t)t.xcd_queues);
  if (ev1) PLAST_HIP(hipEventRecord(ev1, stream));
  timing_mark(kStageUngapped, true, stream);
  timing_launches(1);
  PLAST_HIP(hipGetLastError());
  return PLAST_OK;
}

int ungapped_extend_impl(const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                         int32_t mode, void* d_ws, size_t ws_bytes, plast_hit_t* d_hits, int64_t capacity,
                         int64_t* h_n_hits, int64_t* h_n_ext, hipStream_t stream) {
  if (ws_bytes < 256) return set_error(PLAST_E_WORKSPACE, "workspace smaller than 256 bytes");
  plast_tuning_t T;
  if (p->tuning)
    T = *p->tuning;
  else
    tuning_default(&T);
  UngappedCounters c{0, 0, 0, 0, 0};

  if (mode == PLAST_PLAIN) {
    UngappedArgs A;
    const bool f16 = fill_args(A, a, b, p, d_hits, capacity, &((UngappedCounters*)d_ws)->n_hits);
    std::vector<int64_t> ha(kNKeys + 1), hb(kNKeys + 1);
    int rc;
    if ((rc = read_key_offsets(a, ha.data(), stream)) || (rc = read_key_offsets(b, hb.data(), stream))) return rc;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, (uint32_t*)d_ws, (int64_t)8, 0u);
    int64_t n_ext = 0, launches = 0;
    timing_mark(kStageUngapped, false, stream);
    for (int k = 0; k < kNKeys; ++k) {
      int64_t n1 = ha[k + 1] - ha[k], n2 = hb[k + 1] - hb[k];
      if (n1 <= 0 || n2 <= 0) continue;
      n_ext += n1 * n2;
      int64_t nrt = (n1 + kTileRows - 1) / kTileRows, nct = (n2 + kPlainCols - 1) / kPlainCols;
      if (f16)
        hipLaunchKernelGGL(k_ungapped_plain<true>, dim3((unsigned)(nrt * nct)), dim3(kThreads), 0, stream, A, k,
                           (int32_t)nrt, (int32_t)n2);
      else
        hipLaunchKernelGGL(k_ungapped_plain<false>, dim3((unsigned)(nrt * nct)), dim3(kThreads), 0, stream, A, k,
                           (int32_t)nrt, (int32_t)n2);
      ++launches;
    }
    timing_mark(kStageUngapped, true, stream);
    timing_launches(launches);
    PLAST_HIP(hipGetLastError());
    PLAST_HIP(hipMemcpyAsync(&c.n_hits, d_ws, sizeof(unsigned long long), hipMemcpyDeviceToHost, stream));
    PLAST_HIP(hipStreamSynchronize(stream));
    c.n_ext = (unsigned long long)n_ext;
  } else {
    int rc = ungapped_enqueue_batched(a, b, p, T, ~0u, d_ws, ws_bytes, d_hits, capacity, nullptr, nullptr, nullptr,
                                      nullptr, stream);
    if (rc != PLAST_OK) return rc;
    PLAST_HIP(hipMemcpyAsync(&c, d_ws, sizeof(c), hipMemcpyDeviceToHost, stream));
    PLAST_HIP(hipStreamSynchronize(stream));
    if (c.overflow == 1)
      return set_error(PLAST_E_WORKSPACE, "work list of %llu items exceeds the %lld that %zu workspace bytes hold",
                       c.n_items64, (long long)ungapped_ws_max_items(ws_bytes), ws_bytes);
    if (c.overflow) return set_error(PLAST_E_WORKSPACE, "work list not built (index error flag)");
  }
  *h_n_hits = (int64_t)c.n_hits;
  if (h_n_ext) *h_n_ext = (int64_t)c.n_ext;
  if ((int64_t)c.n_hits > capacity)
    return set_error(PLAST_E_CAPACITY, "%lld hits > capacity %lld", (long long)c.n_hits, (long long)capacity);
  return PLAST_OK;
}

// ---------------------------------------------------------------- allocation-free variant
// The BATCHED workspace (counters, per-key item counts, scan scratch, work
// list) of plast_ungapped_extend_noalloc lives in this fixed device array
// instead of caller memory.  Every GPU the library runs on holds its own copy
// until the process ends.  In host code the name `scratch` is only a host-side
// stand-in: the address kernels need comes from hipGetSymbolAddress, taken once
// per device with that device current and kept in g_scratch_dev.
namespace {
constexpr size_t kStaticScratchBytes = PLAST_NOALLOC_SCRATCH_BYTES;
static_assert(kStaticScratchBytes % 256 == 0, "scratch size");
__device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device.
int static_scratch(void** out) {
  int dev = -1;
  PLAST_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_error(PLAST_E_ARG, "device %d outside 0..%d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    PLAST_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || ((uintptr_t)p & 255)) return set_error(PLAST_E_HIP, "static scratch address %p unusable", p);
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return PLAST_OK;
}
}  // namespace

int ungapped_extend_noalloc_impl(const plast_index_t* a, const plast_index_t* b, const plast_ungapped_params_t* p,
                                 plast_hit_t* d_hits, int64_t capacity, int64_t* h_n_hits, int64_t* h_n_ext,
                                 hipStream_t stream) {
  void* ws = nullptr;
  const int rc = static_scratch(&ws);
  if (rc != PLAST_OK) return rc;
  // The schedule's first kernel clears the counter header; the per-key counts,
  // the scan scratch and the work list are written in full before being read,
  // so what an earlier call left in the array does not matter.
  return ungapped_extend_impl(a, b, p, PLAST_BATCHED, ws, kStaticScratchBytes, d_hits, capacity, h_n_hits, h_n_ext,
                              stream);
}

}  // namespace plast
