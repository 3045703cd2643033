// Stage 3.2 of Sec. 3.3.4: full gapped alignment of the hits that passed the
// small gapped filter, with the per-pair list of ungapped pieces (diagonal,
// first and one-past-last position in bank a) of the alignments already
// computed, which lets a hit lying on one of them skip its own computation.
//
// Order of work.  The surviving hits of one sequence pair form a group, taken
// in order of decreasing gapped score, then seed position in bank a, then in
// bank b; a hit is covered when an earlier alignment of its group has a piece
// on diagonal p1 - p2 holding p1.  Groups are independent, so one wavefront
// takes a whole group at a time from a global counter and walks it in order.
//
// One side (rightward from the seed start, or leftward from the letters before
// it) is the anchored affine-gap recurrence of stage 3.1 with no band and no
// window: H(0,0) = 0, E from the left, F from above, H = max(diagonal, E, F),
// a gap of k letters costing open + k * extend, best = max over cells of H, the
// end cell the first in row-major order holding best.  A wavefront sweeps
// strips of 64 rows (one row per lane) across the columns as a skewed front:
// at step t lane r holds column t - r; H (less the gap-opening cost) and F move
// one lane down per step through a wavefront DPP shift, and the strip's last
// row waits in a per-wavefront global buffer for the next strip.  A score pass over the whole matrix
// finds the best and its end cell; a trace pass over the rectangle up to the
// end cell stores a 4-bit trace per cell (source of H; whether E and F opened)
// in a per-wavefront buffer; the trace-back reads it through an LDS window of
// 64 rows x 64 steps.
//
// Layout of the trace: strip s, lane r and step u = j + r hold the nibble
// (u & 7) of dword ((s * nu8 + (u >> 3)) * 64 + r), nu8 = (ly + 71) / 8 for the
// trace pass's ly, so every eighth step the wavefront stores one coalesced
// 256-byte row.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "plast_internal.h"

namespace plast {
namespace {

constexpr int kANeg = -(1 << 28);
constexpr int kSortTile = 4096;     // radix-sort elements per tile (one wavefront, 64 per lane)
constexpr int kTStride = 32;        // entries per row of the LDS score table
constexpr int kWall = -16256;       // table entry of any pair with the sentinel letter (low byte 0x80: -128 as 8 bits)
constexpr int kYScale = 64 * 2;     // bytes per letter row of the per-lane profile (64 int16)
constexpr int kWalkDwords = 512;    // trace-back window: 8 dwords (64 steps) x 64 rows
constexpr size_t kMaxLds = 160 * 1024;
constexpr int kRowsMax = 4;         // most rows per lane in the multi-row score pass (one profile dword)
constexpr int kProfLaneBytes = 4;   // profile bytes per lane and letter: the larger of 2 (trace pass) and 4
static_assert(kRowsMax <= 4, "the score pass's switch and the profile size cover up to 4 rows per lane");

struct AlignHeader {
  int32_t status;                 // bit 1: sequence longer than its max_len; 2: piece list full; 4: bad hit;
                                  // 8: internal (end cell not found)
  int32_t sort_total;
  int32_t pass_total;             // passing hits (scan total of the per-wavefront counts)
  int32_t group_total;            // sequence pairs (likewise)
  unsigned long long n_pass;
  unsigned long long n_groups;
  unsigned long long next_group;
  unsigned long long n_out;
};

struct Piece {
  int32_t diag, first, last, owner;
};

struct AlignArgs {
  const uint8_t* a_codes;
  const int64_t* a_start;
  const uint8_t* b_codes;
  const int64_t* b_start;
  int32_t a_nseq, b_nseq;
  int32_t max_len1, max_len2;
  int32_t gap_open, gap_extend;
  int32_t max_pieces;
  int32_t rows8;  // 1: every score-table entry of two letters fits 8 bits (the multi-row score pass)
  int8_t mat[20 * 20];
};

struct AlignLayout {
  size_t hdr, tbl, hidx, klo, khi, perm0, perm1, counts, pcount, scan_tmp, heads, tb, pieces, strip, total;
  int64_t tiles;
  size_t tb_words_per_wave;
};

// Columns of a wavefront's strip buffer (the row above the current strip, as
// (H' - open, F') per column, with the columns the front's last steps read),
// a multiple of 8 so that every wavefront's buffer starts on 64 bytes.
__host__ __device__ int64_t strip_cols(int max_len2) { return ((int64_t)max_len2 + 72 + 7) & ~(int64_t)7; }

int bits_for(int64_t v) {  // bits needed for values 0..v
  int b = 0;
  while (b < 63 && (v >> b) > 0) ++b;
  return b;
}

int64_t tb_words(int max_len1, int max_len2) {
  const int64_t strips = (max_len1 + 63) / 64;
  const int64_t nu8 = (max_len2 + 71) / 8;  // steps of a strip, rounded up to 8, over 8
  return strips * nu8 * 64;
}

AlignLayout align_layout(int64_t n, const plast_align_params_t& p, int64_t waves) {
  AlignLayout L;
  L.tiles = (n + kSortTile - 1) / kSortTile;
  if (L.tiles == 0) L.tiles = 1;
  size_t off = 0;
  L.hdr = off;
  off = align_up(off + sizeof(AlignHeader), 256);
  L.tbl = off;
  off = align_up(off + sizeof(int16_t) * 21 * kTStride, 256);
  L.hidx = off;
  off = align_up(off + sizeof(int32_t) * (size_t)n, 256);
  L.klo = off;
  off = align_up(off + sizeof(uint64_t) * (size_t)n, 256);
  L.khi = off;
  off = align_up(off + sizeof(uint64_t) * (size_t)n, 256);
  L.perm0 = off;
  off = align_up(off + sizeof(int32_t) * (size_t)n, 256);
  L.perm1 = off;
  off = align_up(off + sizeof(int32_t) * (size_t)n, 256);
  L.counts = off;
  off = align_up(off + sizeof(int32_t) * 256 * (size_t)L.tiles, 256);
  const int64_t wave_slots = (n + 63) / 64 + 1;
  L.pcount = off;
  off = align_up(off + sizeof(int32_t) * (size_t)wave_slots, 256);
  L.scan_tmp = off;
  const int64_t scan_n = 256 * L.tiles > wave_slots ? 256 * L.tiles : wave_slots;
  off = align_up(off + scan_tmp_bytes(scan_n), 256);
  L.heads = off;
  off = align_up(off + sizeof(int32_t) * (size_t)n, 256);
  L.tb_words_per_wave = (size_t)tb_words(p.max_len1, p.max_len2);
  L.tb = off;
  off = align_up(off + sizeof(uint32_t) * L.tb_words_per_wave * (size_t)waves, 256);
  L.pieces = off;
  off = align_up(off + sizeof(Piece) * (size_t)p.max_pieces * (size_t)waves, 256);
  L.strip = off;
  off = align_up(off + sizeof(int2) * (size_t)strip_cols(p.max_len2) * (size_t)waves, 256);
  L.total = off;
  return L;
}

// LDS of one alignment workgroup: the strip's per-lane profile, y letters by
// column and the trace-back window.  The score table the profiles are built
// from, the x letters and the row above the current strip stay in global
// memory (the row above is read one block of 8 columns ahead): the kernel
// needs as many resident wavefronts as the registers allow (12 per CU), and
// with the row above in LDS it had 10.
size_t align_lds_bytes(int max_len2) {
  size_t b = 21 * 64 * kProfLaneBytes;
  b += align_up((size_t)max_len2 + 136, 16);   // y letters, 64 sentinels before column 0
  b += sizeof(uint32_t) * kWalkDwords;         // trace-back window
  return b;
}

// The row above a strip for the 8 columns of block t8 (all lanes load it; only
// lane 0 uses it).
__device__ __forceinline__ void feed_load(const int2* strip, int t8, int4& a, int4& b, int4& c, int4& d) {
  const int4* sf = (const int4*)(strip + t8);
  a = sf[0];
  b = sf[1];
  c = sf[2];
  d = sf[3];
}

__device__ __forceinline__ int seq_len(const int64_t* start, int s) {
  return (int)(start[s + 1] - start[s] - kPadLen);
}

// ------------------------------------------------------------------ keys and sort

// A passing hit with ids and positions inside its banks (and sequences within
// max_len): it gets a compact index.  Error bits otherwise (count pass only).
__device__ __forceinline__ bool align_hit_ok(const AlignArgs& A, const plast_hit_t* hits, const uint8_t* pass,
                                             int64_t h, int64_t n, AlignHeader* hdr, bool report) {
  if (h >= n || !pass[h]) return false;
  const plast_hit_t r = hits[h];
  if (r.seq1 < 0 || r.seq1 >= A.a_nseq || r.seq2 < 0 || r.seq2 >= A.b_nseq) {
    if (report) atomicOr(&hdr->status, 4);
    return false;
  }
  const int la = seq_len(A.a_start, r.seq1), lb = seq_len(A.b_start, r.seq2);
  if (la > A.max_len1 || lb > A.max_len2) {
    if (report) atomicOr(&hdr->status, 1);
    return false;
  }
  if (r.pos1 < 0 || r.pos1 >= la || r.pos2 < 0 || r.pos2 >= lb) {
    if (report) atomicOr(&hdr->status, 4);
    return false;
  }
  return true;
}

// Compaction of the passing hits in two passes (no shared counter: one
// atomic per wavefront on a single address serialises in L2): per-wavefront
// counts, an exclusive scan, then each wavefront writes at its offset.
__global__ __launch_bounds__(256) void k_align_count(AlignArgs A, const plast_hit_t* hits, const uint8_t* pass,
                                                     int64_t n, AlignHeader* hdr, int32_t* pcount, int32_t* cover) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h < n) cover[h] = -1;
  const uint64_t mask = __ballot(align_hit_ok(A, hits, pass, h, n, hdr, true));
  if ((threadIdx.x & 63) == 0 && (h >> 6) < (n + 63) / 64) pcount[h >> 6] = (int32_t)__popcll(mask);
}

// Sort keys of the compacted hits: (seq1, seq2) in khi, (16383 - gscore, pos1,
// pos2) in klo, so ascending order is the group order.
__global__ __launch_bounds__(256) void k_align_keys(AlignArgs A, const plast_hit_t* hits, const int32_t* gscore,
                                                    const uint8_t* pass, int64_t n, int bp1, int bp2, int b2,
                                                    AlignHeader* hdr, const int32_t* poffset, int32_t* hidx,
                                                    uint64_t* klo, uint64_t* khi) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = align_hit_ok(A, hits, pass, h, n, hdr, false);
  const uint64_t mask = __ballot(ok);
  if (!ok) return;
  const int lane = threadIdx.x & 63;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int64_t c = (int64_t)poffset[h >> 6] + __popcll(mask & below);
  const plast_hit_t r = hits[h];
  int g = gscore[h];
  g = g < 0 ? 0 : (g > 16383 ? 16383 : g);
  hidx[c] = (int32_t)h;
  klo[c] = ((uint64_t)(16383 - g) << (bp1 + bp2)) | ((uint64_t)r.pos1 << bp2) | (uint64_t)r.pos2;
  khi[c] = ((uint64_t)r.seq1 << b2) | (uint64_t)r.seq2;
}

__global__ __launch_bounds__(64) void k_align_clear(AlignHeader* hdr) {
  if (threadIdx.x == 0) *hdr = AlignHeader{0, 0, 0, 0, 0, 0, 0, 0};
}

__global__ __launch_bounds__(64) void k_align_npass(AlignHeader* hdr) {
  if (threadIdx.x == 0) hdr->n_pass = (unsigned long long)hdr->pass_total;
}

__global__ __launch_bounds__(256) void k_iota(int32_t* perm, const AlignHeader* hdr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)hdr->n_pass) perm[i] = (int32_t)i;
}

// Digit histogram of one tile (one wavefront, kSortTile elements in order).
__global__ __launch_bounds__(64) void k_rs_count(const int32_t* perm, const uint64_t* key, int shift,
                                                 const AlignHeader* hdr, int32_t* counts, int64_t tiles) {
  __shared__ int32_t hist[256];
  const int lane = threadIdx.x;
  for (int d = lane; d < 256; d += 64) hist[d] = 0;
  __syncthreads();
  const int64_t m = (int64_t)hdr->n_pass;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int k = 0; k < kSortTile / 64; ++k) {
    const int64_t i = base + k * 64 + lane;
    if (i < m) atomicAdd(&hist[(int)((key[perm[i]] >> shift) & 255)], 1);
  }
  __syncthreads();
  for (int d = lane; d < 256; d += 64) counts[(int64_t)d * tiles + blockIdx.x] = hist[d];
}

// Stable scatter: the tile's elements in order, ranked among equal digits of
// the same 64-element round with ballots, after the earlier rounds' counts.
__global__ __launch_bounds__(64) void k_rs_scatter(const int32_t* perm_in, const uint64_t* key, int shift,
                                                   const AlignHeader* hdr, const int32_t* offsets, int64_t tiles,
                                                   int32_t* perm_out) {
  __shared__ int32_t run[256];
  const int lane = threadIdx.x;
  for (int d = lane; d < 256; d += 64) run[d] = offsets[(int64_t)d * tiles + blockIdx.x];
  __syncthreads();
  const int64_t m = (int64_t)hdr->n_pass;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int k = 0; k < kSortTile / 64; ++k) {
    const int64_t i = base + k * 64 + lane;
    const bool valid = i < m;
    const int32_t c = valid ? perm_in[i] : 0;
    const int d = valid ? (int)((key[c] >> shift) & 255) : 0;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t ones = __ballot(valid && ((d >> b) & 1));
      peers &= ((d >> b) & 1) ? ones : ~ones;
    }
    const int rank = __popcll(peers & below);
    const int start = run[d];
    __syncthreads();
    if (valid) {
      perm_out[start + rank] = c;
      if (rank == 0) run[d] = start + __popcll(peers);
    }
    __syncthreads();
  }
}

// First element of each sequence pair in sorted order, compacted in two passes
// like the passing hits.
__device__ __forceinline__ bool is_head(const int32_t* perm, const uint64_t* khi, const AlignHeader* hdr, int64_t i) {
  return i < (int64_t)hdr->n_pass && (i == 0 || khi[perm[i]] != khi[perm[i - 1]]);
}

__global__ __launch_bounds__(256) void k_align_head_count(const int32_t* perm, const uint64_t* khi,
                                                          const AlignHeader* hdr, int32_t* hcount) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t mask = __ballot(is_head(perm, khi, hdr, i));
  if ((threadIdx.x & 63) == 0 && i < (int64_t)hdr->n_pass) hcount[i >> 6] = (int32_t)__popcll(mask);
}

__global__ __launch_bounds__(256) void k_align_heads(const int32_t* perm, const uint64_t* khi, AlignHeader* hdr,
                                                     const int32_t* hoffset, int32_t* heads) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool head = is_head(perm, khi, hdr, i);
  const uint64_t mask = __ballot(head);
  if (!head) return;
  const int lane = threadIdx.x & 63;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  heads[hoffset[i >> 6] + __popcll(mask & below)] = (int32_t)i;
}

__global__ __launch_bounds__(64) void k_align_ngroups(AlignHeader* hdr) {
  if (threadIdx.x == 0) hdr->n_groups = (unsigned long long)hdr->group_total;
}

// ------------------------------------------------------------------ alignment

struct SideStats {
  int best;
  int i_end, j_end;     // letters of x and y the side consumes
  int length, ident, mism, opens;
};

__device__ __forceinline__ int shr1(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xf, 0xf, false);  // wave_shr:1, lane 0 keeps old
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// The strips of one DP over lx rows and the columns 0 .. steps - 64 (x letters
// x[r * dx] in global memory, read once per strip for the profile; y letters by
// column in yo, sentinels past both ends; the row above strip 0 in strip[]).
//
// Values are carried shifted by (i + j) * extend (H' = H + (i + j) ext, and
// likewise E', F'), which removes the extension term from both gap recurrences:
// E'(i, j) = max(E'(i, j-1), H'(i, j-1) - open), F' likewise from above, and
// the diagonal is H'(i-1, j-1) + score + 2 ext.  Each lane carries hm = H' -
// open and F' one lane down per step, so the diagonal is hm(i-1, j-1) + T[x][y]
// with T = score + open + 2 extend.  On the skewed front every lane of a step
// lies on the same anti-diagonal i + j = 64 s + 1 + t, so unshifting for the
// best is one subtraction of a uniform value.  Every register starts a strip at
// NEG and column 0 of row 0 feeds lane 0, so column 0 comes out of the same
// recurrence; letters past either end are the sentinel, whose negative T entry
// makes every cell beyond the matrix strictly smaller (unshifted) than some
// cell inside it, so the best needs no range test.
// TRACE = false: scores only; the lane's best (unshifted) value and the first
// block of 8 steps where it reached it, as (strip << 16) | (block start + 1).
// TRACE = true: the 4-bit trace of every cell into tb, and in jf the first
// column of row `row` (per lane: -1 elsewhere) whose H equals `target`.
template <bool TRACE>
__device__ __forceinline__ void side_dp(int lx, int ly, int steps, int ge, int go, const int16_t* T, int16_t* prof,
                                        const uint8_t* x, int dx, const uint8_t* yo, int2* strip, uint32_t* tb,
                                        int& best,
                                        int& bpos, int row = 0, int target = 0, int* jf = nullptr) {
  const int lane = threadIdx.x;
  const int nu8 = steps >> 3;
  const int strips = (lx + 63) >> 6;
  for (int s = 0; s < strips; ++s) {
    // this strip's profile: prof[y * 64 + lane] = T[x of the lane's row][y], so
    // that every lane's lookup falls in its own LDS bank
    {
      const int r = s * 64 + lane;
      const int16_t* trow = T + (r < lx ? (int)x[(int64_t)r * dx] : kPadCode) * kTStride;
      int16_t v[21];
#pragma unroll
      for (int yc = 0; yc < 21; ++yc) v[yc] = trow[yc];
#pragma unroll
      for (int yc = 0; yc < 21; ++yc) prof[yc * 64 + lane] = v[yc];
    }
    const uint8_t* pcol = (const uint8_t*)(prof + lane);
    const uint8_t* ycol = yo + 64 - lane;  // the letter of this lane's column t - lane at step t
    int hm = kANeg, f = kANeg, hup = kANeg, eleft = kANeg, hmleft = kANeg;
    uint32_t* tbs = tb + (size_t)s * nu8 * 64 + lane;
    const int sbase = s << 16;
    const bool my_row = TRACE && s * 64 + lane + 1 == row;
    // Only lane 0 uses the block's inputs (the others take theirs from the
    // lane above), but every lane loads them: the registers are then fresh
    // each block and the DPP shifts, whose lane 0 keeps the old value, write
    // into them without a copy.  They are loaded one block ahead.
    // The last strip's rows sit in its first `lanes` lanes and no strip reads
    // its last row, so it ends once lane lanes - 1 has passed column ly.
    const bool last = s + 1 == strips;
    const int lanes = last ? lx - s * 64 : 64;
    const int steps_s = last ? min(steps, (ly + lanes + 7) & ~7) : steps;
    int4 n0, n1, n2, n3;
    feed_load(strip, 0, n0, n1, n2, n3);
    for (int t8 = 0; t8 < steps_s; t8 += 8) {
      const int4 s0 = n0, s1 = n1, s2 = n2, s3 = n3;
      if (t8 + 8 < steps_s) feed_load(strip, t8 + 8, n0, n1, n2, n3);
      const int fh[8] = {s0.x, s0.z, s1.x, s1.z, s2.x, s2.z, s3.x, s3.z};
      const int ff[8] = {s0.y, s0.w, s1.y, s1.w, s2.y, s2.w, s3.y, s3.w};
      int sc[8];
      uint32_t yw[2];
      __builtin_memcpy(yw, ycol + t8, 8);
#pragma unroll
      for (int k = 0; k < 8; ++k)
        sc[k] = *(const int16_t*)(pcol + __builtin_amdgcn_ubfe(yw[k >> 2], 8 * (k & 3), 8) * kYScale);
      int oh[8], of[8];
      uint32_t acc = 0;
      int bmax = kANeg;
      const int diag0 = (s * 64 + 1 + t8) * ge;  // (i + j) * extend of the block's first step
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int hdiag = hup;
        hup = shr1(fh[k], hm);
        const int fup = shr1(ff[k], f);
        const int e = max(eleft, hmleft);
        f = max(fup, hup);
        const int d = hdiag + sc[k];
        const int h = max(max(d, e), f);
        if (TRACE) {
          const uint32_t nib =
              (h == d ? 0u : (h == e ? 1u : 2u)) | (hmleft >= eleft ? 4u : 0u) | (hup >= fup ? 8u : 0u);
          acc |= nib << (4 * k);
          if (my_row && h - (diag0 + k * ge) == target && *jf < 0) *jf = t8 + k - lane;
        } else {
          bmax = max(bmax, h - k * ge);
        }
        hm = h - go;
        hmleft = hm;
        eleft = e;
        oh[k] = hm;
        of[k] = f;
      }
      if (!TRACE) bmax -= diag0;
      if (TRACE) {
        tbs[(t8 >> 3) * 64] = acc;
      } else if (bmax > best) {
        best = bmax;
        bpos = sbase + t8 + 1;
      }
      if (!last && lane == 63) {  // lane 63 finished columns t8 - 63 .. t8 - 56 of the strip's last row
        if (t8 >= 63 && t8 - 56 <= ly) {
#pragma unroll
          for (int k = 0; k < 8; ++k) strip[t8 + k - 63] = make_int2(oh[k], of[k]);
        } else {
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int j = t8 + k - 63;
            if (j >= 0 && j <= ly) strip[j] = make_int2(oh[k], of[k]);
          }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
  }
}

// The score pass with R rows per lane, for score tables that fit 8 bits: the
// same recurrence and values as side_dp over one strip of rows s0 + 1 .. s0 +
// 64 R.  Lane r holds rows s0 + r R + 1 .. s0 + r R + R, all in the column t
// - r at step t, so one pair of wavefront shifts per step serves R cells: a
// row's diagonal and vertical inputs come from the lane's row above (its
// values of the previous step and of this one), those of the lane's first
// row from the last row of the lane above, as in side_dp.  The profile holds
// per y letter and lane the R scores of the lane's rows as bytes of one
// dword, so each step reads them with one LDS access.  The sentinel's entry
// is -128 (the low byte of kWall): it only has to make every cell past the
// matrix lower than some cell inside it, which any negative unshifted score
// does (see side_dp).  Cell (i, j) of row q at step t8 + k carries the
// shift (i + j) ext = off0 + (q + k) ext, so the block maximum of H' - k ext,
// less off0 + q ext, is the row's best over the block.  Each row keeps its
// best value and the first block that reached it; the lane then keeps, over
// its rows in order and over the strips, the first row holding its largest
// value (rows past lx lie below a cell of an earlier row, see side_dp), with
// the last column of that row's block (bjhi) as the bound for the trace pass.
template <int R>
__device__ __forceinline__ void side_score8(int s0, int lx, int ly, int steps, int ge, int go, const int16_t* T,
                                            uint32_t* prof, const uint8_t* x, int dx, const uint8_t* yo, int2* strip,
                                            int& best, int& brow, int& bjhi) {
  const int lane = threadIdx.x;
  {
    // each row's line of the score table (entries 0..23, 16-byte aligned);
    // the low byte of an entry is its 8-bit value, the wall's included
    uint4 tr[R][3];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i0 = s0 + lane * R + q;
      const uint4* line = (const uint4*)(T + (i0 < lx ? (int)x[(int64_t)i0 * dx] : kPadCode) * kTStride);
#pragma unroll
      for (int c = 0; c < 3; ++c) tr[q][c] = line[c];
    }
#pragma unroll
    for (int yc = 0; yc < 21; ++yc) {
      uint32_t w = 0u;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const uint4 v = tr[q][yc >> 3];
        const uint32_t d = (yc & 6) == 0 ? v.x : ((yc & 6) == 2 ? v.y : ((yc & 6) == 4 ? v.z : v.w));
        w |= ((d >> (16 * (yc & 1))) & 255u) << (8 * q);
      }
      prof[yc * 64 + lane] = w;
    }
  }
  __syncthreads();
  int hml[R], el[R], rbest[R], rpos[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    hml[q] = kANeg;
    el[q] = kANeg;
    rbest[q] = 0;
    rpos[q] = -1;
  }
  int hup = kANeg, flast = kANeg;
  const uint8_t* ycol = yo + 64 - lane;
  const uint32_t* pl = prof + lane;
  // the last strip ends once its last lane with rows has passed column ly
  // (see side_dp)
  const bool last = s0 + 64 * R >= lx;
  const int lanes = last ? (lx - s0 + R - 1) / R : 64;
  const int steps_s = last ? min(steps, (ly + lanes + 7) & ~7) : steps;
  int4 n0, n1, n2, n3;  // the row above, one block ahead (see side_dp)
  feed_load(strip, 0, n0, n1, n2, n3);
  for (int t8 = 0; t8 < steps_s; t8 += 8) {
    const int4 s0v = n0, s1v = n1, s2v = n2, s3v = n3;
    if (t8 + 8 < steps_s) feed_load(strip, t8 + 8, n0, n1, n2, n3);
    const int fh[8] = {s0v.x, s0v.z, s1v.x, s1v.z, s2v.x, s2v.z, s3v.x, s3v.z};
    const int ff[8] = {s0v.y, s0v.w, s1v.y, s1v.w, s2v.y, s2v.w, s3v.y, s3v.w};
    uint32_t yw[2];
    __builtin_memcpy(yw, ycol + t8, 8);
    int bm[R];
#pragma unroll
    for (int q = 0; q < R; ++q) bm[q] = kANeg;
    int oh[8], of[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t w = pl[__builtin_amdgcn_ubfe(yw[k >> 2], 8 * (k & 3), 8) * 64];
      const int hdiag = hup;
      hup = shr1(fh[k], hml[R - 1]);
      const int fup = shr1(ff[k], flast);
      int dsrc = hdiag, fa = fup, ha = hup;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int sc = (int)(int8_t)(w >> (8 * q));
        const int e = max(el[q], hml[q]);
        const int f = max(fa, ha);
        const int h = max(max(dsrc + sc, e), f);
        bm[q] = max(bm[q], h - k * ge);
        dsrc = hml[q];
        hml[q] = h - go;
        el[q] = e;
        fa = f;
        ha = hml[q];
      }
      flast = fa;
      oh[k] = ha;
      of[k] = fa;
    }
    const int off0 = (s0 + lane * (R - 1) + 1 + t8) * ge;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int u = bm[q] - off0 - q * ge;
      if (u > rbest[q]) {
        rbest[q] = u;
        rpos[q] = t8;
      }
    }
    if (!last && lane == 63) {  // the strip's last row, columns t8 - 63 .. t8 - 56
      if (t8 >= 63 && t8 - 56 <= ly) {
#pragma unroll
        for (int k = 0; k < 8; ++k) strip[t8 + k - 63] = make_int2(oh[k], of[k]);
      } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int j = t8 + k - 63;
          if (j >= 0 && j <= ly) strip[j] = make_int2(oh[k], of[k]);
        }
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __syncthreads();
#pragma unroll
  for (int q = 0; q < R; ++q) {
    if (rpos[q] >= 0 && rbest[q] > best) {
      best = rbest[q];
      brow = s0 + lane * R + q + 1;
      bjhi = rpos[q] + 7 - lane;
    }
  }
}

// Letters of a DP over lx x ly: x past lx and y past ly (and column 0) are the
// sentinel; the row above strip 0 is row 0, shifted: H'(0, 0) = 0 and H'(0, k)
// = -(open + k ext) + k ext = -open, so hm(0, 0) = -open, hm(0, k) = -2 open,
// F' = NEG, and NEG past ly.
__device__ __forceinline__ void side_pad(int ly, int steps, int go, uint8_t* yo, int2* strip) {
  const int lane = threadIdx.x;
  for (int k = ly + 1 + lane; k < steps; k += 64) yo[64 + k] = (uint8_t)kPadCode;
  yo[lane] = (uint8_t)kPadCode;  // columns -64 .. -1
  if (lane == 0) yo[64] = (uint8_t)kPadCode;
  for (int k = lane; k < steps; k += 64)
    strip[k] = make_int2(k == 0 ? -go : (k <= ly ? -2 * go : kANeg), kANeg);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __syncthreads();
}

// One side.  x (lx letters, step dx) runs down the rows, y (ly letters) across
// the columns; dir = +1 (pairs a[p1 + i - 1], b[p2 + j - 1]) or -1 (pairs
// a[p1 - i], b[p2 - j]).  A score pass over the whole matrix finds the best and
// its end cell; a trace pass over rows 1..i_end and columns 1..j_end (which
// depend on no other cell) recomputes the same values with their traces, and
// the trace-back reads those.  Appends the side's pieces to P (count np).
__device__ __forceinline__ SideStats align_side(const AlignArgs& A, const uint8_t* x, int lx, int dx,
                                                const uint8_t* y, int ly, int dy, int dir, int p1, int p2, int owner,
                                                const int16_t* T, int16_t* prof, uint8_t* yo, int2* strip,
                                                uint32_t* walk, uint32_t* tb, Piece* P, int& np, int32_t* status) {
  const int lane = threadIdx.x;
  const int ge = A.gap_extend, go = A.gap_open;
  SideStats st = {0, 0, 0, 0, 0, 0, 0};
  if (lx == 0 || ly == 0) return st;
  const int steps = (ly + 64 + 7) & ~7;
  for (int k = lane; k < ly; k += 64) yo[65 + k] = y[(int64_t)k * dy];
  side_pad(ly, steps, go, yo, strip);
  // the lane's best value, its first row and the last column of the block of
  // 8 steps where that row first reached it (brow 0: cell (0, 0))
  int best = 0, brow = 0, bjhi = 0;
  if (A.rows8) {
    for (int s0 = 0; s0 < lx;) {  // strips of up to 64 kRowsMax rows, each as narrow as its rows allow
      const int rows = min(kRowsMax, (lx - s0 + 63) >> 6);
      switch (rows) {
#define PLAST_SCORE_CASE(n) \
  case n:                   \
    side_score8<n>(s0, lx, ly, steps, ge, go, T, (uint32_t*)prof, x, dx, yo, strip, best, brow, bjhi); \
    break;
        PLAST_SCORE_CASE(1)
        PLAST_SCORE_CASE(2)
        PLAST_SCORE_CASE(3)
        PLAST_SCORE_CASE(4)
#undef PLAST_SCORE_CASE
        default:
          break;
      }
      s0 += 64 * rows;
    }
  } else {
    int bpos = 0;  // (strip << 16) | (block start + 1)
    side_dp<false>(lx, ly, steps, ge, go, T, prof, x, dx, yo, strip, tb, best, bpos);
    if (bpos != 0) {
      const int s = bpos >> 16, t8 = (bpos & 0xffff) - 1;
      brow = s * 64 + lane + 1;
      bjhi = t8 + 7 - lane;
    }
  }

  // best over the wavefront: largest value, then first row (bjhi goes with
  // the row)
  for (int o = 32; o >= 1; o >>= 1) {
    const int ob = __shfl_xor(best, o), orow = __shfl_xor(brow, o), oj = __shfl_xor(bjhi, o);
    if (ob > best || (ob == best && orow < brow)) {
      best = ob;
      brow = orow;
      bjhi = oj;
    }
  }
  best = uni(best);
  brow = uni(brow);
  bjhi = uni(bjhi);
  st.best = best;
  st.i_end = brow;
  st.j_end = 0;

  // The trace of rows 1..i_end up to the end of the best's block (those cells
  // depend on no other); the end cell is the first cell of row i_end there
  // whose H is the best.
  int nu8 = 0;
  if (st.i_end > 0) {
    const int r_end = (st.i_end - 1) & 63;
    const int j_hi = min(ly, bjhi);
    const int steps2 = (j_hi + 64 + 7) & ~7;
    side_pad(j_hi, steps2, go, yo, strip);
    int unused0 = 0, unused1 = 0, jf = -1;
    side_dp<true>(st.i_end, j_hi, steps2, ge, go, T, prof, x, dx, yo, strip, tb, unused0, unused1, st.i_end, best,
                  &jf);
    nu8 = steps2 >> 3;
    st.j_end = __shfl(jf, r_end);
    st.j_end = uni(st.j_end);
    if (st.j_end < 1) {  // cannot happen: the block holds a cell with the best value
      if (lane == 0) atomicOr(status, 8);
      st.j_end = j_hi;
    }
  }

  // trace-back, uniform across the wavefront.  The trace and the pieces are
  // private to this wavefront and re-read by it on the same compute unit, so
  // ordering at workgroup scope suffices (an agent-scope fence would write back
  // the whole L2 of the XCD).
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  int i = st.i_end, j = st.j_end;
  int state = 0;           // 0: H, 1: E, 2: F
  int prev = 0;            // last move: 0 none, 1 D, 2 E, 3 F
  int run_a = -1, run_b = -1, run_diag = 0;  // current piece: positions in a (inclusive)
  int blk_s = -1, blk_g0 = 0;
  // the two sequences from their first letter (x and y start at the seed, or
  // at the letters before it)
  const uint8_t* aseq = x - (dir > 0 ? p1 : p1 - 1);
  const uint8_t* bseq = y - (dir > 0 ? p2 : p2 - 1);
  // a piece ends: its identities are counted by the whole wavefront, 64
  // letter pairs at a time
  auto close_run = [&]() {
    if (run_a >= 0) {
      const int lo = min(run_a, run_b), len = max(run_a, run_b) + 1 - lo;
      int same = 0;
      for (int k0 = 0; k0 < len; k0 += 64) {
        const int k = k0 + lane;
        const bool eq = k < len && aseq[lo + k] == bseq[lo + k - run_diag];
        same += __popcll(__ballot(eq));
      }
      st.ident += same;
      st.mism += len - same;
      st.length += len;
      const int q = np;
      if (q < A.max_pieces) {
        if (lane == 0) P[q] = Piece{run_diag, lo, lo + len, owner};
        np = q + 1;
      } else if (lane == 0) {
        atomicOr(status, 2);
      }
      run_a = -1;
    }
  };
  while (i > 0 || j > 0) {
    // the walk's state is the same in every lane: keep it scalar
    i = uni(i);
    j = uni(j);
    state = uni(state);
    prev = uni(prev);
    run_a = uni(run_a);
    run_b = uni(run_b);
    run_diag = uni(run_diag);
    blk_s = uni(blk_s);
    blk_g0 = uni(blk_g0);
    if (i == 0 || j == 0) {  // the rest is one gap along row 0 or column 0
      const int mv = i == 0 ? 2 : 3;
      close_run();
      if (prev != mv) st.opens++;
      st.length += i + j;
      prev = mv;
      break;
    }
    const int s = (i - 1) >> 6, r = (i - 1) & 63, u = j + r, g = u >> 3;
    if (s != blk_s || g < blk_g0 || g >= blk_g0 + 8) {
      blk_s = s;
      blk_g0 = g - 7 > 0 ? g - 7 : 0;
      const uint32_t* src = tb + ((size_t)s * nu8 + blk_g0) * 64;
      for (int c = 0; c < 8; ++c)
        if (blk_g0 + c < nu8) walk[c * 64 + lane] = src[c * 64 + lane];
      __syncthreads();
    }
    const uint32_t nib = (uint32_t)uni((int)((walk[(g - blk_g0) * 64 + r] >> ((u & 7) * 4)) & 15u));
    if (state == 0) {
      const uint32_t src = nib & 3u;
      if (src == 0) {
        const int pa = dir > 0 ? p1 + i - 1 : p1 - i;
        const int pb = dir > 0 ? p2 + j - 1 : p2 - j;
        if (run_a < 0) {
          run_a = pa;
          run_diag = pa - pb;
        }
        run_b = pa;
        prev = 1;
        --i;
        --j;
      } else {
        state = (int)src;
      }
    } else if (state == 1) {
      close_run();
      if (prev != 2) st.opens++;
      st.length++;
      prev = 2;
      state = (nib & 4u) ? 0 : 1;
      --j;
    } else {
      close_run();
      if (prev != 3) st.opens++;
      st.length++;
      prev = 3;
      state = (nib & 8u) ? 0 : 2;
      --i;
    }
  }
  close_run();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  return st;
}

// The score table of the shifted recurrence: T[x][y] = score + open + 2 extend
// for letters, kWall where either is the sentinel (row and column 20).
__global__ __launch_bounds__(64) void k_align_table(AlignArgs A, int16_t* __restrict__ T) {
  const int t_add = A.gap_open + 2 * A.gap_extend;  // the diagonal term in shifted values
  for (int k = threadIdx.x; k < 21 * kTStride; k += 64) {
    const int xa = k / kTStride, yc = k % kTStride;
    T[k] = (int16_t)((xa < 20 && yc < 20) ? (int)A.mat[xa * 20 + yc] + t_add : kWall);
  }
}

// At most 168 VGPRs (3 wavefronts per SIMD, 12 per CU): the LDS of a
// workgroup (15.1 KB for sequences of up to 1000 letters) holds the number of
// resident workgroups to 10 per CU, so the registers cost no occupancy, and
// with fewer the kernel spills.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_align(
    AlignArgs A, const int16_t* __restrict__ T, const plast_hit_t* hits, const int32_t* hidx, const int32_t* perm,
    const uint64_t* khi, const int32_t* heads, AlignHeader* hdr, uint32_t* tb_all, size_t tb_words, Piece* pieces_all,
    int2* strip_all, plast_alignment_t* out, int32_t* cover) {
  extern __shared__ __align__(16) uint8_t lds[];
  int16_t* prof = (int16_t*)lds;
  uint8_t* yo = (uint8_t*)lds + 21 * 64 * kProfLaneBytes;
  uint32_t* walk = (uint32_t*)(yo + ((A.max_len2 + 136 + 15) & ~15));
  const int lane = threadIdx.x;
  __syncthreads();

  uint32_t* tb = tb_all + (size_t)blockIdx.x * tb_words;
  Piece* P = pieces_all + (size_t)blockIdx.x * A.max_pieces;
  int2* strip = strip_all + (size_t)blockIdx.x * (size_t)strip_cols(A.max_len2);
  const int64_t m = (int64_t)hdr->n_pass;
  const int64_t n_groups = (int64_t)hdr->n_groups;
  for (;;) {
    // fewer than 2^31 groups, and each wavefront overshoots the count once
    unsigned long long gq = 0;
    if (lane == 0) gq = atomicAdd(&hdr->next_group, 1ull);
    const int g = uni((int)gq);
    if (g >= n_groups) break;
    const int64_t k0 = heads[g];
    const uint64_t gkey = khi[perm[k0]];
    int np = 0;
    for (int64_t k = k0; k < m; ++k) {
      const int32_t c = uni(perm[k]);
      if (k > k0 && khi[c] != gkey) break;
      const int32_t h = uni(hidx[c]);
      const plast_hit_t r = hits[h];
      const int s1 = uni(r.seq1), p1 = uni(r.pos1), s2 = uni(r.seq2), p2 = uni(r.pos2);
      // covered by a piece of an earlier alignment of the group?
      int owner = -1;
      for (int q0 = 0; q0 < np; q0 += 64) {
        const int q = q0 + lane;
        bool on = false;
        int own = 0;
        if (q < np) {
          const Piece pc = P[q];
          on = pc.diag == p1 - p2 && pc.first <= p1 && p1 < pc.last;
          own = pc.owner;
        }
        const uint64_t b = __ballot(on);
        if (b) {
          owner = __shfl(own, __ffsll((long long)b) - 1);
          break;
        }
      }
      owner = uni(owner);
      if (owner >= 0) {
        if (lane == 0) cover[h] = owner;
        continue;
      }
      if (lane == 0) cover[h] = h;
      const uint8_t* a = A.a_codes + A.a_start[s1];
      const uint8_t* b = A.b_codes + A.b_start[s2];
      const int la = seq_len(A.a_start, s1), lb = seq_len(A.b_start, s2);
      const SideStats R = align_side(A, a + p1, la - p1, 1, b + p2, lb - p2, 1, +1, p1, p2, h, T, prof, yo, strip,
                                     walk, tb, P, np, &hdr->status);
      const SideStats L = align_side(A, a + p1 - 1, p1, -1, b + p2 - 1, p2, -1, -1, p1, p2, h, T, prof, yo, strip,
                                     walk, tb, P, np, &hdr->status);
      if (lane == 0) {
        const unsigned long long o = atomicAdd(&hdr->n_out, 1ull);
        plast_alignment_t rec;
        rec.seq1 = s1;
        rec.seq2 = s2;
        rec.seed1 = p1;
        rec.seed2 = p2;
        rec.start1 = p1 - L.i_end;
        rec.end1 = p1 + R.i_end;
        rec.start2 = p2 - L.j_end;
        rec.end2 = p2 + R.j_end;
        rec.score = R.best + L.best;
        rec.length = R.length + L.length;
        rec.identities = R.ident + L.ident;
        rec.mismatches = R.mism + L.mism;
        rec.gap_opens = R.opens + L.opens;
        rec.hit = h;
        out[o] = rec;
      }
    }
  }
}

}  // namespace

int align_default_waves(const plast_align_params_t& p, int64_t* waves) {
  const size_t lds = align_lds_bytes(p.max_len2);
  if (lds > kMaxLds)  // not reached for max_len2 <= 16384; kept against a change of the layout
    return set_error(PLAST_E_ARG, "max_len2=%d needs %zu bytes of LDS (limit %zu)", p.max_len2, lds, kMaxLds);
  if (p.n_waves > 0) {
    *waves = p.n_waves;
    return PLAST_OK;
  }
  int dev = 0, cus = 0, per_cu = 0;
  PLAST_HIP(hipGetDevice(&dev));
  PLAST_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  PLAST_HIP(hipFuncSetAttribute((const void*)k_align, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  PLAST_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_align, 64, lds));
  if (per_cu < 1) return set_error(PLAST_E_ARG, "alignment kernel does not fit a compute unit with %zu bytes of LDS", lds);
  *waves = (int64_t)per_cu * cus;
  return PLAST_OK;
}

size_t align_ws_bytes(int64_t n_hits, const plast_align_params_t& p, int64_t waves) {
  return align_layout(n_hits, p, waves).total;
}

int align_impl(const plast_index_t* a, const plast_index_t* b, const plast_hit_t* d_hits, const int32_t* d_gscore,
               const uint8_t* d_pass, int64_t n_hits, const plast_align_params_t* p, void* d_ws, size_t ws_bytes,
               plast_alignment_t* d_out, int32_t* d_cover, int64_t* h_n_out, hipStream_t s) {
  int64_t waves = 0;
  int rc = align_default_waves(*p, &waves);
  if (rc) return rc;
  const AlignLayout L = align_layout(n_hits, *p, waves);
  if (ws_bytes < L.total) return set_error(PLAST_E_WORKSPACE, "alignment workspace %zu < %zu bytes", ws_bytes, L.total);
  uint8_t* ws = (uint8_t*)d_ws;
  AlignHeader* hdr = (AlignHeader*)(ws + L.hdr);
  int32_t* hidx = (int32_t*)(ws + L.hidx);
  uint64_t* klo = (uint64_t*)(ws + L.klo);
  uint64_t* khi = (uint64_t*)(ws + L.khi);
  int32_t* perm[2] = {(int32_t*)(ws + L.perm0), (int32_t*)(ws + L.perm1)};
  int32_t* counts = (int32_t*)(ws + L.counts);
  int32_t* heads = (int32_t*)(ws + L.heads);
  uint32_t* tb = (uint32_t*)(ws + L.tb);
  Piece* pieces = (Piece*)(ws + L.pieces);

  AlignArgs A;
  A.a_codes = a->codes;
  A.a_start = a->seq_start;
  A.b_codes = b->codes;
  A.b_start = b->seq_start;
  A.a_nseq = a->n_seqs;
  A.b_nseq = b->n_seqs;
  A.max_len1 = p->max_len1;
  A.max_len2 = p->max_len2;
  A.gap_open = p->gap_open;
  A.gap_extend = p->gap_extend;
  A.max_pieces = p->max_pieces;
  if (p->matrix) {
    for (int k = 0; k < 400; ++k) A.mat[k] = p->matrix[k];
  } else {
    blosum62_code_order(A.mat);
  }
  A.rows8 = 1;
  for (int k = 0; k < 400; ++k) {
    const int t = (int)A.mat[k] + p->gap_open + 2 * p->gap_extend;
    if (t < -127 || t > 127) A.rows8 = 0;
  }

  const int bp1 = bits_for(p->max_len1), bp2 = bits_for(p->max_len2);
  const int b1 = bits_for(a->n_seqs), b2 = bits_for(b->n_seqs);
  hipLaunchKernelGGL(k_align_clear, dim3(1), dim3(64), 0, s, hdr);
  const unsigned nb = (unsigned)((n_hits + 255) / 256);
  int32_t* pcount = (int32_t*)(ws + L.pcount);
  const int64_t wave_slots = (n_hits + 63) / 64;
  hipLaunchKernelGGL(k_align_count, dim3(nb ? nb : 1), dim3(256), 0, s, A, d_hits, d_pass, n_hits, hdr, pcount,
                     d_cover);
  exclusive_scan_i32(pcount, wave_slots, &hdr->pass_total, ws + L.scan_tmp, s);
  hipLaunchKernelGGL(k_align_npass, dim3(1), dim3(64), 0, s, hdr);
  hipLaunchKernelGGL(k_align_keys, dim3(nb ? nb : 1), dim3(256), 0, s, A, d_hits, d_gscore, d_pass, n_hits, bp1, bp2,
                     b2, hdr, (const int32_t*)pcount, hidx, klo, khi);
  AlignHeader h0;
  PLAST_HIP(hipMemcpyAsync(&h0, hdr, sizeof(h0), hipMemcpyDeviceToHost, s));
  PLAST_HIP(hipStreamSynchronize(s));
  const int64_t m = (int64_t)h0.n_pass;
  if (m > 0) {
    const int64_t tiles = (m + kSortTile - 1) / kSortTile;
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, perm[0], hdr);
    int cur = 0;
    const int lo_bits = 14 + bp1 + bp2, hi_bits = b1 + b2;
    for (int pass_key = 0; pass_key < 2; ++pass_key) {
      const uint64_t* key = pass_key == 0 ? klo : khi;
      const int nbits = pass_key == 0 ? lo_bits : hi_bits;
      for (int shift = 0; shift < nbits; shift += 8) {
        hipLaunchKernelGGL(k_rs_count, dim3((unsigned)tiles), dim3(64), 0, s, perm[cur], key, shift, hdr, counts,
                           tiles);
        exclusive_scan_i32(counts, 256 * tiles, &hdr->sort_total, ws + L.scan_tmp, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)tiles), dim3(64), 0, s, perm[cur], key, shift, hdr, counts,
                           tiles, perm[cur ^ 1]);
        cur ^= 1;
      }
    }
    const unsigned mb = (unsigned)((m + 255) / 256);
    hipLaunchKernelGGL(k_align_head_count, dim3(mb), dim3(256), 0, s, perm[cur], khi, hdr, pcount);
    exclusive_scan_i32(pcount, (m + 63) / 64, &hdr->group_total, ws + L.scan_tmp, s);
    hipLaunchKernelGGL(k_align_ngroups, dim3(1), dim3(64), 0, s, hdr);
    hipLaunchKernelGGL(k_align_heads, dim3(mb), dim3(256), 0, s, perm[cur], khi, hdr, (const int32_t*)pcount, heads);
    const size_t lds = align_lds_bytes(p->max_len2);
    PLAST_HIP(hipFuncSetAttribute((const void*)k_align, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int16_t* tbl = (int16_t*)(ws + L.tbl);
    hipLaunchKernelGGL(k_align_table, dim3(1), dim3(64), 0, s, A, tbl);
    timing_mark(kStageAlign, false, s);
    hipLaunchKernelGGL(k_align, dim3((unsigned)waves), dim3(64), lds, s, A, (const int16_t*)tbl, d_hits, hidx,
                       perm[cur], khi, heads, hdr, tb, L.tb_words_per_wave, pieces, (int2*)(ws + L.strip), d_out,
                       d_cover);
    timing_mark(kStageAlign, true, s);
    PLAST_HIP(hipGetLastError());
    PLAST_HIP(hipMemcpyAsync(&h0, hdr, sizeof(h0), hipMemcpyDeviceToHost, s));
    PLAST_HIP(hipStreamSynchronize(s));
  }
  *h_n_out = (int64_t)h0.n_out;
  if (h0.status & 1) return set_error(PLAST_E_ARG, "a hit's sequence is longer than max_len1 / max_len2");
  if (h0.status & 4) return set_error(PLAST_E_ARG, "a passing hit lies outside its banks");
  if (h0.status & 2) return set_error(PLAST_E_WORKSPACE, "a sequence pair needs more than max_pieces=%d pieces",
                                      p->max_pieces);
  if (h0.status & 8) return set_error(PLAST_E_HIP, "internal: an alignment's end cell was not found");
  return PLAST_OK;
}

}  // namespace plast
