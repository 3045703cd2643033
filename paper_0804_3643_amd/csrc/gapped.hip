// Stage 3.1, small gapped filter (Sec. 3.3.4; Sec. 5.2.2: for each hit, one
// extension to the right of the seed start and one to the left of it).
//
// Each side is an anchored banded affine-gap DP (Gotoh): cell (i, j) aligns the
// first i letters of x with the first j letters of y and exists iff
// |i - j| <= band; a gap of length k costs gap_open + k * gap_extend.  The side
// scores max(0, best existing cell) and the hit scores right + left.
//
// One thread per hit.  The band of row i is held in registers, indexed by
// d = j - i + 16 (33 cells), so H and F of the previous row are read at d
// (diagonal) and d + 1 (vertical) and overwritten in place; E runs left to
// right inside the row.  The letters of y under the band slide by one register
// per row.  The thread's windows are staged in LDS; y positions past the clipped
// length hold a wall letter with a non-positive substitution score.  A cell past
// the end of y never feeds a cell inside it, and is reached only from cells
// inside through wall letters or gaps, which cannot raise the score; so it never
// exceeds the best existing cell and no per-cell length test is needed.
//
// Fast path (band 16, window <= 64, and every finite DP value an integer of
// magnitude < 2048, which holds for BLOSUM62 with open 11 / extend 1): one lane
// per hit computes both extensions at once, the right one in the low and the
// left one in the high half of packed binary16 registers.  Sums of such
// integers are exact in binary16, -inf marks cells outside the band or before
// the anchor, and v_pk_maximum3_f16 takes H = max(diagonal, E, F) in one
// instruction.  Letters are fetched from global memory one block of rows
// ahead as aligned dwords (four letters per load).
//
// Fast-path arithmetic: every value of cell (i, j) is carried shifted by
// (i + j) * extend.  The shift turns the Gotoh recurrences into
//   H' = max(H'(i-1, j-1) + s + 2 extend, E', F'),
//   E'(i, j+1) = max(E'(i, j), H'(i, j) - open),  F'(i+1, j) = max(F'(i, j), H'(i, j) - open),
// one addition and two maxima fewer per cell; the 2 extend is folded into the
// substitution table.  The best cell is recovered per anti-diagonal (all cells
// of one anti-diagonal share the shift): an odd row folds each new cell together
// with the cell two slots to its right in the row above (still in its register)
// into that anti-diagonal's running maximum, and an anti-diagonal is unshifted
// once no later row reaches it.
// Scores come from a pair table in LDS: one 4-byte entry holds the scores of
// an x letter against two consecutive y letters, i.e. of two neighbouring cells
// of a row, so one lookup per side serves two cells.  The workgroup size is a
// launch-shape parameter (128, 256 or 512 threads); each resident workgroup
// builds the 37 KB table once and strides over the hits.  The last four blocks
// of rows are peeled at compile time and skip their cells right of column 64,
// which no window reaches (about 5% of the band).
#include <type_traits>

#include "plast_internal.h"

namespace plast {

namespace {

constexpr int kGThreads = 128;
constexpr int kGMaxWin = 64;
constexpr int kGMaxBand = 16;
constexpr int kGCells = 2 * kGMaxBand + 1;  // 33
constexpr int kGYLen = kGMaxWin + kGMaxBand + 16;  // 96 y letters staged per side
constexpr int kWall = 21;                   // letter code of the wall
constexpr int kWallScore = -1000;          // any value <= 0 works: a cell past y only loses score
constexpr int kNeg = -(1 << 28);

struct GappedArgs {
  const uint8_t* a_scan;
  const int64_t* a_seq_start;
  const uint8_t* b_scan;
  const int64_t* b_seq_start;
  int32_t a_nseq, b_nseq;
  int32_t window, band, gap_open, gap_extend, s2, pad_;
  int16_t mat[kNLet * 22];     // [x letter][y letter or wall]
  uint16_t tbl16[kNLet * kNLet];  // binary16 [x letter][y letter], -inf where either is the separator (20)
};

struct GSmem {
  int32_t mat[kNLet * 22];
  uint8_t x[kGThreads][kGMaxWin];
  uint8_t y[kGThreads][kGYLen];
};

template <int BAND>
__device__ int gapped_side(const GappedArgs& G, GSmem& S, int t, int lx, int ly, int band) {
  const int oe = G.gap_open + G.gap_extend;
  const int ext = G.gap_extend;
  const uint8_t* xs = S.x[t];
  const uint8_t* ys = S.y[t];
  int H[kGCells], F[kGCells], Y[kGCells];
  // row 0: H(0, j) = -(open + j*ext) for 0 < j <= band, H(0,0) = 0
#pragma unroll
  for (int d = 0; d < kGCells; ++d) {
    const int j = d - kGMaxBand;
    const bool inband = BAND == kGMaxBand ? true : (j >= -band && j <= band);
    H[d] = (j < 0 || !inband) ? kNeg : (j == 0 ? 0 : -(G.gap_open + j * ext));
    F[d] = kNeg;
    // letter of y[j' - 1] for row 1, j' = 1 + d - 16 -> index d - 16
    Y[d] = (d - kGMaxBand >= 0) ? ys[d - kGMaxBand] : kWall;
  }
  int best = 0;
  for (int i = 1; i <= lx; ++i) {
    const int* mrow = &S.mat[xs[i - 1] * 22];
    int e = kNeg, hleft = kNeg;
    const int ynext = ys[i + kGMaxBand];  // y index (i+1) + 32 - 17 for the next row
#pragma unroll
    for (int d = 0; d < kGCells; ++d) {
      const int diag = H[d] + mrow[Y[d]];
      const int f = d + 1 < kGCells ? max(F[d + 1] - ext, H[d + 1] - oe) : kNeg;
      e = max(e - ext, hleft - oe);
      int h = max(max(diag, e), f);
      int fv = f;
      if (BAND != kGMaxBand) {
        const int j = i + d - kGMaxBand;
        if (j - i < -band || j - i > band) {
          h = kNeg;
          fv = kNeg;
          e = kNeg;
        }
      }
      h = max(h, kNeg);
      best = max(best, h);
      H[d] = h;
      F[d] = max(fv, kNeg);
      hleft = h;
    }
#pragma unroll
    for (int d = 0; d + 1 < kGCells; ++d) Y[d] = Y[d + 1];
    Y[kGCells - 1] = ynext;
  }
  (void)ly;
  return best;
}

template <int BAND>
__global__ __launch_bounds__(kGThreads) void k_gapped(GappedArgs G, const plast_hit_t* __restrict__ hits,
                                                      int64_t n_hits, const unsigned long long* __restrict__ n_dev,
                                                      int32_t* __restrict__ gscore, uint8_t* __restrict__ pass) {
  __shared__ GSmem S;
  for (int i = threadIdx.x; i < kNLet * 22; i += kGThreads) S.mat[i] = G.mat[i];
  if (n_dev) n_hits = min(n_hits, (int64_t)*n_dev);
  __syncthreads();
  const int t = threadIdx.x;
  const int64_t h = (int64_t)blockIdx.x * kGThreads + t;
  const bool live = h < n_hits;
  plast_hit_t hit = live ? hits[h] : plast_hit_t{0, 0, 0, 0, 0};
  int total = 0;
  bool sane = live && hit.seq1 >= 0 && hit.seq1 < G.a_nseq && hit.seq2 >= 0 && hit.seq2 < G.b_nseq;
  int64_t sa = 0, sb = 0;
  int la = 0, lb = 0;
  if (sane) {
    sa = G.a_seq_start[hit.seq1];
    sb = G.b_seq_start[hit.seq2];
    la = (int)(G.a_seq_start[hit.seq1 + 1] - sa - kPadLen);
    lb = (int)(G.b_seq_start[hit.seq2 + 1] - sb - kPadLen);
    sane = hit.pos1 >= 0 && hit.pos1 < la && hit.pos2 >= 0 && hit.pos2 < lb;
  }
  if (live && !sane) {  // not a hit of these banks: flagged, nothing read
    gscore[h] = -1;
    pass[h] = 0;
  }
  if (sane) {
    const int64_t qa = sa + hit.pos1, qb = sb + hit.pos2;
    for (int side = 0; side < 2; ++side) {
      int lx, ly;
      if (side == 0) {
        lx = min(G.window, la - hit.pos1);
        ly = min(G.window, lb - hit.pos2);
        for (int k = 0; k < lx; ++k) S.x[t][k] = G.a_scan[qa + k] / kScale;
        for (int k = 0; k < kGYLen; ++k) S.y[t][k] = k < ly ? G.b_scan[qb + k] / kScale : kWall;
      } else {
        lx = min(G.window, hit.pos1);
        ly = min(G.window, hit.pos2);
        for (int k = 0; k < lx; ++k) S.x[t][k] = G.a_scan[qa - 1 - k] / kScale;
        for (int k = 0; k < kGYLen; ++k) S.y[t][k] = k < ly ? G.b_scan[qb - 1 - k] / kScale : kWall;
      }
      total += gapped_side<BAND>(G, S, t, lx, ly, G.band);
    }
    gscore[h] = total;
    pass[h] = total >= G.s2 ? 1 : 0;
  }
}


// ---------------------------------------------------------------- packed f16 path
typedef _Float16 gh2 __attribute__((ext_vector_type(2)));
// Rows per unrolled block and register budget of the fast path: the fastest
// of a sweep on MI355X (4 rows per block, up to 256 VGPRs, i.e. 2 wavefronts
// per SIMD; 3 wavefronts per SIMD and 2-row blocks were not faster).
constexpr int kFBlock = 4;                      // rows per unrolled block (1..4)
static_assert(kFBlock >= 1 && kFBlock <= 4, "rows per block");
constexpr int kFY = kGCells + kFBlock;          // y letters held for a block (37)
constexpr uint32_t kWall8 = kPadCode * kScale;  // the separator letter serves as wall: it scores -inf
// Pair table: dword (x * 21 + y1) * 21 + y2 holds the binary16 scores of x
// against y1 (low half) and against y2 (high half), so one 4-byte lookup
// serves two neighbouring cells of a row (y1 and y2 are consecutive y letters).
constexpr int kPairRow = kNLet * kNLet;         // dwords per x letter (441)
constexpr int kPairDwords = kNLet * kPairRow;   // 9261 (37 KB of LDS)
constexpr uint32_t kXRowBytes = 4 * kPairRow;
static_assert(kPairDwords * 4 < 65536, "table offsets must fit 16 bits");

// The last kTailBlocks blocks of the fast path (up to row 64) are peeled at
// compile time, so that their cells right of column 64 are not computed.
constexpr int kTailBlocks = 4;

// Cell d (band index, column j = i + d - 16) of row r of block blk (rows
// 4 blk + 1 ..): true when it lies left of column 0 or right of column 64.
// Such a cell is outside every window (windows hold at most 64 letters): a cell
// left of column 0 is -inf and feeds only cells left of column 0, and a cell
// right of column 64 feeds only cells right of column 64, so neither changes a
// cell inside.  blk < 0 (the generic body) skips nothing.
__host__ __device__ constexpr bool gapped_skip_cell(int blk, int r, int d) {
  return blk >= 0 && ((4 * blk + r + 1) + d - kGMaxBand < 0 || (4 * blk + r + 1) + d - kGMaxBand > kGMaxWin);
}

__device__ __forceinline__ gh2 gmax3(gh2 a, gh2 b, gh2 c) {
  return __builtin_elementwise_maximum(__builtin_elementwise_maximum(a, b), c);
}
__device__ __forceinline__ gh2 gmax(gh2 a, gh2 b) { return __builtin_elementwise_maximum(a, b); }

// Four consecutive scan-code bytes of `buf` from byte offset `off` (which may be
// unaligned or negative): one aligned dword pair and a funnel shift.  The pair is
// clamped at the start of the buffer and the buffer carries kScanSlack bytes of
// tail slack, so no read leaves it; bytes outside the sequence are masked by
// the caller.
__device__ __forceinline__ uint32_t load4(const uint8_t* __restrict__ buf, int64_t off) {
  const uint32_t* p = (const uint32_t*)buf + (off >= 0 ? (off >> 2) : 0);
  return __builtin_amdgcn_alignbyte(p[1], p[0], (uint32_t)(off & 3));
}

__device__ __forceinline__ uint32_t byte_of(uint32_t v, int k) { return (v >> (8 * k)) & 0xffu; }

// Letters of one hit: x rows i = 1.. and y indices k = 0.. for the rightward
// (R) and leftward (L) extension, in scan-code units; walls outside.
struct GLetters {
  const uint8_t* A;  // bank a scan codes
  const uint8_t* B;  // bank b scan codes
  int64_t qa, qb;    // anchor offsets
  int lxR, lxL, lyR, lyL;
  // rows i0 .. i0+n-1 (n <= 4) of both extensions: table row offsets of this lane's copy
  template <int n>
  __device__ __forceinline__ void xrows(int i0, uint32_t (&xbR)[n], uint32_t (&xbL)[n]) const {
    const uint32_t r4 = load4(A, qa + i0 - 1);      // byte r: x_R row i0 + r
    const uint32_t l4 = load4(A, qa - i0 - 3);      // byte 3 - r: x_L row i0 + r
#pragma unroll
    for (int r = 0; r < n; ++r) {
      const uint32_t sr = i0 + r <= lxR ? byte_of(r4, r) : kWall8;
      const uint32_t sl = i0 + r <= lxL ? byte_of(l4, 3 - r) : kWall8;
      xbR[r] = (sr / kScale) * kXRowBytes;
      xbL[r] = (sl / kScale) * kXRowBytes;
    }
  }
  // y indices k0 .. k0+3 of both extensions: packed letters (R low, L high)
  __device__ __forceinline__ void ycols(int k0, uint32_t (&y)[4]) const {
    const uint32_t r4 = load4(B, qb + k0);          // byte t: y_R index k0 + t
    const uint32_t l4 = load4(B, qb - 4 - k0);      // byte 3 - t: y_L index k0 + t
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = k0 + t;
      const uint32_t sr = (k >= 0 && k < lyR) ? byte_of(r4, t) : kWall8;
      const uint32_t sl = (k >= 0 && k < lyL) ? byte_of(l4, 3 - t) : kWall8;
      y[t] = (sr / kScale) | ((sl / kScale) << 16);
    }
  }
};

// Packed pair-table offsets of the letter pairs (a, b), R and L halves.
__device__ __forceinline__ uint32_t pair_off(uint32_t a, uint32_t b) {
  return (a * (uint32_t)(kNLet * 4) + b * 4u) & 0xffffu | ((((a >> 16) * (uint32_t)(kNLet * 4) + (b >> 16) * 4u)) << 16);
}

__device__ __forceinline__ void gapped_hit_f16(const GappedArgs& G, const uint32_t* tbl,
                                               const plast_hit_t* __restrict__ hits, int64_t h, int64_t n_hits,
                                               int32_t* __restrict__ gscore, uint8_t* __restrict__ pass) {
  const bool live = h < n_hits;
  plast_hit_t hit = live ? hits[h] : plast_hit_t{0, 0, 0, 0, 0};
  bool sane = live && hit.seq1 >= 0 && hit.seq1 < G.a_nseq && hit.seq2 >= 0 && hit.seq2 < G.b_nseq;
  int64_t sa = 0, sb = 0;
  int la = 0, lb = 0;
  if (sane) {
    sa = G.a_seq_start[hit.seq1];
    sb = G.b_seq_start[hit.seq2];
    la = (int)(G.a_seq_start[hit.seq1 + 1] - sa - kPadLen);
    lb = (int)(G.b_seq_start[hit.seq2 + 1] - sb - kPadLen);
    sane = hit.pos1 >= 0 && hit.pos1 < la && hit.pos2 >= 0 && hit.pos2 < lb;
  }
  GLetters L;
  L.A = G.a_scan;
  L.B = G.b_scan;
  L.qa = sane ? sa + hit.pos1 : kPadLen;  // a lane without a valid record reads separators
  L.qb = sane ? sb + hit.pos2 : kPadLen;
  L.lxR = sane ? min(G.window, la - hit.pos1) : 0;
  L.lyR = sane ? min(G.window, lb - hit.pos2) : 0;
  L.lxL = sane ? min(G.window, hit.pos1) : 0;
  L.lyL = sane ? min(G.window, hit.pos2) : 0;
  const int rows = max(L.lxR, L.lxL);

  const _Float16 ninf = -__builtin_inff16();
  const gh2 NEG = {ninf, ninf};
  // Values are carried shifted by (i + j) * extend (see the kernel comment):
  // the table holds s + 2 * extend, and both gap recurrences lose their
  // per-cell extension term.
  const _Float16 op = (_Float16)G.gap_open, ex = (_Float16)G.gap_extend;
  const gh2 OP = {op, op};
  gh2 H[kGCells], F[kGCells];
  // YY[k]: packed pair-table offsets of the letters at y indices i0 + k - 17 and
  // i0 + k - 16 for the block at row i0; ylast: packed letters at y index i0 + 19
  uint32_t YY[kFY - 1];
  uint32_t ylast;
  // row 0 (shifted): H(0, 0) = 0, H(0, j) + j * extend = -open for 0 < j <= 16; F holds F(1, j)
#pragma unroll
  for (int d = 0; d < kGCells; ++d) {
    const int j = d - kGMaxBand;
    const _Float16 v = j < 0 ? ninf : (j == 0 ? (_Float16)0 : -op);
    H[d] = gh2{v, v};
    F[d] = H[d] - OP;
  }
  // letters under the band of the first block (rows 1..4): y indices -16 .. 20
  {
    uint32_t prev = 0;
#pragma unroll
    for (int g = 0; g < (kFY + 3) / 4; ++g) {
      uint32_t y4[4];
      L.ycols(4 * g - kGMaxBand, y4);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = 4 * g + t;
        if (k > 0 && k < kFY) YY[k - 1] = pair_off(prev, y4[t]);
        prev = y4[t];
      }
    }
    ylast = 0;
#pragma unroll
    for (int g = 0; g < (kFY + 3) / 4; ++g) {
      // the letter at position kFY - 1 of the first block (y index 20)
      if (4 * g <= kFY - 1 && kFY - 1 < 4 * g + 4) {
        uint32_t y4[4];
        L.ycols(4 * g - kGMaxBand, y4);
        ylast = y4[(kFY - 1) - 4 * g];
      }
    }
  }
  uint32_t xbR[kFBlock], xbL[kFBlock];
  L.xrows<kFBlock>(1, xbR, xbL);
  gh2 best = {(_Float16)0, (_Float16)0};  // H(0, 0) = 0: the empty alignment
  // best shifted value per anti-diagonal i + j = 2 i0 - 16 + t of the current block
  constexpr int kAcc = 2 * (kFBlock - 1) + kGCells;  // 39
  constexpr int kAccShift = 2 * kFBlock;             // anti-diagonals completed per block
  gh2 acc[kAcc];
#pragma unroll
  for (int t = 0; t < kAcc; ++t) acc[t] = NEG;
  int i0 = 1;
  // shift of anti-diagonal 2 i0 - 16 of the current block, (2 i0 - 16) * extend,
  // stepped by extend per anti-diagonal (integers below 2048: exact in binary16)
  const gh2 EX = {ex, ex};
  gh2 sh = gh2{(_Float16)(2 - kGMaxBand), (_Float16)(2 - kGMaxBand)} * EX;
  const char* tb = (const char*)tbl;
  // One block of kFBlock rows starting at row i0.  BLK >= 0 names the block
  // (rows 4 BLK + 1 ..) at compile time: its cells outside every window are
  // skipped (gapped_skip_cell); BLK < 0 is the generic body that computes every
  // cell.
  auto block = [&](auto blk_c) {
    constexpr int BLK = decltype(blk_c)::value;
    // raw letters of the next block (x rows, and the y indices entering the band),
    // decoded after this block's rows
    const uint32_t nx4R = load4(L.A, L.qa + i0 + kFBlock - 1), nx4L = load4(L.A, L.qa - i0 - kFBlock - 3);
    const int k0 = i0 + kFY - kGMaxBand - 1;
    const uint32_t ny4R = load4(L.B, L.qb + k0), ny4L = load4(L.B, L.qb - 4 - k0);
    // The block's cells in row-major order of cell pairs (2p, 2p + 1); the two
    // table lookups of a pair (right side in A, left side in B) are issued
    // kAhead pairs before the pair is computed (they depend on letters only).
    constexpr int kPairs = (kGCells + 1) / 2;
    constexpr int kSeq = kFBlock * kPairs;
    constexpr int kAhead = 5;
    uint32_t A[kSeq], B[kSeq];
    auto issue = [&](int q) {
      const int r = q / kPairs, p = q % kPairs;
      if (gapped_skip_cell(BLK, r, 2 * p) && gapped_skip_cell(BLK, r, 2 * p + 1)) return;
      const uint32_t yy = YY[2 * p + r];
      A[q] = *(const uint32_t*)(tb + xbR[r] + (yy & 0xffffu));
      B[q] = *(const uint32_t*)(tb + xbL[r] + (yy >> 16));
    };
#pragma unroll
    for (int q = 0; q < kAhead; ++q) issue(q);
    gh2 e = NEG;
#pragma unroll
    for (int q = 0; q < kSeq; ++q) {
      if (q + kAhead < kSeq) issue(q + kAhead);
      const int r = q / kPairs, p = q % kPairs;
      if (p == 0) e = NEG;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int d = 2 * p + c;
        if (d < kGCells) {
          // cell (i0 + r, d) lies on anti-diagonal 2 i0 - 16 + (2 r + d); in an odd
          // row it shares it with cell d + 2 of the row above, still in H[d + 2]
          const int t = 2 * r + d;
          const bool own = !gapped_skip_cell(BLK, r, d);
          const bool above = (r & 1) && d + 2 < kGCells && !gapped_skip_cell(BLK, r - 1, d + 2);
          if (own) {
            const gh2 sc = __builtin_bit_cast(gh2, __builtin_amdgcn_perm(B[q], A[q], c ? 0x07060302u : 0x05040100u));
            const gh2 diag = H[d] + sc;
            const gh2 f = d + 1 < kGCells ? F[d + 1] : NEG;
            const gh2 hh = gmax3(diag, e, f);
            if (r & 1)
              acc[t] = above ? gmax3(acc[t], hh, H[d + 2]) : gmax(acc[t], hh);
            else if (d < 2)
              acc[t] = gmax(acc[t], hh);
            const gh2 ho = hh - OP;
            e = gmax(e, ho);
            F[d] = gmax(f, ho);
            H[d] = hh;
          } else if (above) {
            acc[t] = gmax(acc[t], H[d + 2]);
          }
        }
      }
    }
    // anti-diagonals below 2 (i0 + 4) - 16 are complete: unshift and fold into best
    {
#pragma unroll
      for (int t = 0; t < kAccShift; ++t) {
        best = gmax(best, acc[t] - sh);
        sh = sh + EX;  // after the block: the shift of the next block's first anti-diagonal
      }
#pragma unroll
      for (int t = 0; t < kAcc; ++t) acc[t] = t + kAccShift < kAcc ? acc[t + kAccShift] : NEG;
    }
#pragma unroll
    for (int k = 0; k + kFBlock < kFY - 1; ++k) YY[k] = YY[k + kFBlock];
    const int i1 = i0 + kFBlock;
#pragma unroll
    for (int t = 0; t < kFBlock; ++t) {
      const int k = k0 + t;
      const uint32_t sr = (k >= 0 && k < L.lyR) ? byte_of(ny4R, t) : kWall8;
      const uint32_t sl = (k >= 0 && k < L.lyL) ? byte_of(ny4L, 3 - t) : kWall8;
      const uint32_t y = (sr / kScale) | ((sl / kScale) << 16);
      YY[kFY - 1 - kFBlock + t] = pair_off(ylast, y);
      ylast = y;
      const uint32_t xr = i1 + t <= L.lxR ? byte_of(nx4R, t) : kWall8;
      const uint32_t xl = i1 + t <= L.lxL ? byte_of(nx4L, 3 - t) : kWall8;
      xbR[t] = (xr / kScale) * kXRowBytes;
      xbL[t] = (xl / kScale) * kXRowBytes;
    }
    i0 = i1;
  };
  // The generic body runs the blocks up to row 4 (kNBlocks - kTailBlocks), the
  // peeled bodies the tail blocks; every block runs only while a lane of the
  // wavefront still has rows.  Scheduling barriers keep each peeled block's
  // instructions inside it.  (Peeling the head blocks too, whose cells left of
  // column 0 are wasted, made the register allocation spill.)
  static_assert(kFBlock == 4 && kGMaxWin == 64 && kTailBlocks <= 4, "peeled blocks assume 4-row blocks over 64 rows");
  constexpr int kNBlocks = kGMaxWin / kFBlock;
  auto more = [&]() { return __builtin_amdgcn_readfirstlane(__ballot(i0 <= rows) != 0) != 0; };
  auto peeled = [&](auto blk_c) {
    if (more()) {
      __builtin_amdgcn_sched_barrier(0);
      block(blk_c);
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  while (i0 <= kFBlock * (kNBlocks - kTailBlocks) && more()) block(std::integral_constant<int, -1>{});
  if constexpr (kTailBlocks >= 4) peeled(std::integral_constant<int, kNBlocks - 4>{});
  if constexpr (kTailBlocks >= 3) peeled(std::integral_constant<int, kNBlocks - 3>{});
  if constexpr (kTailBlocks >= 2) peeled(std::integral_constant<int, kNBlocks - 2>{});
  if constexpr (kTailBlocks >= 1) peeled(std::integral_constant<int, kNBlocks - 1>{});
#pragma unroll
  for (int t = 0; t < kAcc; ++t) {
    best = gmax(best, acc[t] - sh);
    sh = sh + EX;
  }
  if (live) {
    const int total = sane ? (int)best.x + (int)best.y : -1;
    gscore[h] = total;
    pass[h] = (sane && total >= G.s2) ? 1 : 0;
  }
}

template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2)))
void k_gapped_f16(GappedArgs G, const plast_hit_t* __restrict__ hits, int64_t n_hits,
                  const unsigned long long* __restrict__ n_dev, int32_t* __restrict__ gscore,
                  uint8_t* __restrict__ pass) {
  __shared__ uint32_t tbl[kPairDwords];  // filled once per workgroup
  for (int i = threadIdx.x; i < kPairDwords; i += NT) {
    const int x = i / kPairRow, y1 = (i / kNLet) % kNLet, y2 = i % kNLet;
    tbl[i] = (uint32_t)G.tbl16[x * kNLet + y1] | ((uint32_t)G.tbl16[x * kNLet + y2] << 16);
  }
  if (n_dev) n_hits = min(n_hits, (int64_t)*n_dev);
  __syncthreads();
  // grid-stride over blocks of NT hits; no barrier inside the loop
  for (int64_t h = (int64_t)blockIdx.x * NT + threadIdx.x; h - threadIdx.x < n_hits; h += (int64_t)gridDim.x * NT)
    gapped_hit_f16(G, tbl, hits, h, n_hits, gscore, pass);
}

// Workgroups of k_gapped_f16<NT> resident on the device at once (0 on error).
template <int NT>
int64_t fast_resident() {
  static int64_t cached = 0;
  if (!cached) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_gapped_f16<NT>, NT, 0) != hipSuccess)
      return 0;
    cached = (int64_t)cus * (per > 0 ? per : 1);
  }
  return cached;
}

// The grid is at most one resident wave of workgroups: each workgroup builds
// the 37 KB pair table once and then strides over the hits.
template <int NT>
int launch_fast(const GappedArgs& G, const plast_hit_t* d_hits, int64_t n_hits, const unsigned long long* d_n,
                int32_t* d_gscore, uint8_t* d_pass, hipStream_t stream) {
  const int64_t resident = fast_resident<NT>();
  if (resident <= 0) return set_error(PLAST_E_HIP, "cannot query device occupancy");
  const int64_t need = (n_hits + NT - 1) / NT;
  const int64_t grid = need < resident ? need : resident;
  hipLaunchKernelGGL(k_gapped_f16<NT>, dim3((unsigned)grid), dim3(NT), 0, stream, G, d_hits, n_hits, d_n, d_gscore,
                     d_pass);
  return PLAST_OK;
}

}  // namespace

int gapped_prepare() {
  return (fast_resident<128>() > 0 && fast_resident<256>() > 0 && fast_resident<512>() > 0)
             ? PLAST_OK
             : set_error(PLAST_E_HIP, "cannot query device occupancy");
}

int gapped_filter_impl(const plast_index_t* a, const plast_index_t* b, const plast_hit_t* d_hits, int64_t n_hits,
                       const unsigned long long* d_n, const plast_gapped_params_t* g, int32_t* d_gscore,
                       uint8_t* d_pass, hipStream_t stream) {
  GappedArgs G;
  G.a_scan = a->scan_codes;
  G.a_seq_start = a->seq_start;
  G.b_scan = b->scan_codes;
  G.b_seq_start = b->seq_start;
  G.a_nseq = a->n_seqs;
  G.b_nseq = b->n_seqs;
  G.window = g->window;
  G.band = g->band;
  G.gap_open = g->gap_open;
  G.gap_extend = g->gap_extend;
  G.s2 = g->s2;
  G.pad_ = 0;
  int8_t m[400];
  if (g->matrix) {
    for (int i = 0; i < 400; ++i) m[i] = g->matrix[i];
  } else {
    blosum62_code_order(m);
  }
  int maxabs = 0;
  for (int x = 0; x < kNLet; ++x)
    for (int y = 0; y < 22; ++y) {
      G.mat[x * 22 + y] = (x < 20 && y < 20) ? m[x * 20 + y] : kWallScore;
      if (x < 20 && y < 20) maxabs = max(maxabs, abs((int)m[x * 20 + y]));
    }
  const uint16_t ninf16 = 0xFC00;  // binary16 -inf
  for (int x = 0; x < kNLet; ++x)
    for (int y = 0; y < kNLet; ++y)
      G.tbl16[x * kNLet + y] =
          (x < 20 && y < 20) ? __builtin_bit_cast(uint16_t, (_Float16)(m[x * 20 + y] + 2 * g->gap_extend)) : ninf16;
  // Every finite DP value lies within [-(64 |M| + 3 (open + extend) + 130 extend), 64 |M|],
  // and the fast path adds (i + j) * extend <= 150 extend to it: integers of that
  // range are exact in binary16 when the bound stays below 2048.
  const bool fast = g->band == kGMaxBand && g->window <= kGMaxWin &&
                    64 * maxabs + 3 * (g->gap_open + g->gap_extend) + 280 * g->gap_extend <= 2000;
  const int threads = g->tuning ? g->tuning->gapped_threads : 256;
  if (n_hits <= 0) return PLAST_OK;
  timing_mark(kStageGapped, false, stream);
  if (fast) {
    const int rc = threads == 128   ? launch_fast<128>(G, d_hits, n_hits, d_n, d_gscore, d_pass, stream)
                   : threads == 512 ? launch_fast<512>(G, d_hits, n_hits, d_n, d_gscore, d_pass, stream)
                                    : launch_fast<256>(G, d_hits, n_hits, d_n, d_gscore, d_pass, stream);
    if (rc != PLAST_OK) return rc;
  } else {
    unsigned blocks = (unsigned)((n_hits + kGThreads - 1) / kGThreads);
    if (g->band == kGMaxBand)
      hipLaunchKernelGGL(k_gapped<kGMaxBand>, dim3(blocks), dim3(kGThreads), 0, stream, G, d_hits, n_hits, d_n,
                         d_gscore, d_pass);
    else
      hipLaunchKernelGGL(k_gapped<-1>, dim3(blocks), dim3(kGThreads), 0, stream, G, d_hits, n_hits, d_n, d_gscore,
                         d_pass);
  }
  timing_mark(kStageGapped, true, stream);
  PLAST_HIP(hipGetLastError());
  return PLAST_OK;
}

}  // namespace plast
