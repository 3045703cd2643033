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
  int16_t mat[kNLet * 22];  // [x letter][y letter or wall]
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
                                                      int64_t n_hits, int32_t* __restrict__ gscore,
                                                      uint8_t* __restrict__ pass) {
  __shared__ GSmem S;
  for (int i = threadIdx.x; i < kNLet * 22; i += kGThreads) S.mat[i] = G.mat[i];
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

}  // namespace

int gapped_filter_impl(const plast_index_t* a, const plast_index_t* b, const plast_hit_t* d_hits, int64_t n_hits,
                       const plast_gapped_params_t* g, int32_t* d_gscore, uint8_t* d_pass, hipStream_t stream) {
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
  for (int x = 0; x < kNLet; ++x)
    for (int y = 0; y < 22; ++y)
      G.mat[x * 22 + y] = (x < 20 && y < 20) ? m[x * 20 + y] : kWallScore;
  unsigned blocks = (unsigned)((n_hits + kGThreads - 1) / kGThreads);
  timing_mark(kStageGapped, false, stream);
  if (g->band == kGMaxBand)
    hipLaunchKernelGGL(k_gapped<kGMaxBand>, dim3(blocks), dim3(kGThreads), 0, stream, G, d_hits, n_hits, d_gscore,
                       d_pass);
  else
    hipLaunchKernelGGL(k_gapped<-1>, dim3(blocks), dim3(kGThreads), 0, stream, G, d_hits, n_hits, d_gscore, d_pass);
  timing_mark(kStageGapped, true, stream);
  PLAST_HIP(hipGetLastError());
  return PLAST_OK;
}

}  // namespace plast
