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
// ahead as aligned dwords (four letters per load).  Substitution scores come
// from a dense binary16 table in LDS.  The workgroup size is a launch-shape
// parameter (128, 256 or 512 threads).
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
// per SIMD; replicated tables and 3 wavefronts per SIMD were not faster).
constexpr int kFBlock = 4;                      // rows per unrolled block (1..4)
static_assert(kFBlock >= 1 && kFBlock <= 4, "rows per block");
constexpr int kFY = kGCells + kFBlock - 1;      // y letters held for a block (36)
constexpr int kTblDwords = (kNLet * kNLet + 1) / 2;
constexpr uint32_t kWall8 = kPadCode * kScale;  // the separator letter serves as wall: it scores -inf
// Table entry (x, y) is the binary16 at byte offset x * kRowBytes + y * kEntry.
constexpr uint32_t kEntry = 2;
constexpr uint32_t kRowBytes = kNLet * kEntry;
static_assert(kNLet * kRowBytes < 65536, "table offsets must fit 16 bits");

__device__ __forceinline__ gh2 gmax3(gh2 a, gh2 b, gh2 c) {
  uint32_t r;
  asm("v_pk_maximum3_f16 %0, %1, %2, %3"
      : "=v"(r)
      : "v"(__builtin_bit_cast(uint32_t, a)), "v"(__builtin_bit_cast(uint32_t, b)),
        "v"(__builtin_bit_cast(uint32_t, c)));
  return __builtin_bit_cast(gh2, r);
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
      xbR[r] = (sr / kScale) * kRowBytes;
      xbL[r] = (sl / kScale) * kRowBytes;
    }
  }
  // y indices k0 .. k0+3 of both extensions: packed table column offsets
  __device__ __forceinline__ void ycols(int k0, uint32_t (&y)[4]) const {
    const uint32_t r4 = load4(B, qb + k0);          // byte t: y_R index k0 + t
    const uint32_t l4 = load4(B, qb - 4 - k0);      // byte 3 - t: y_L index k0 + t
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = k0 + t;
      const uint32_t sr = (k >= 0 && k < lyR) ? byte_of(r4, t) : kWall8;
      const uint32_t sl = (k >= 0 && k < lyL) ? byte_of(l4, 3 - t) : kWall8;
      y[t] = (sr / kScale) * kEntry | (((sl / kScale) * kEntry) << 16);
    }
  }
};

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
  const _Float16 oe = (_Float16)(G.gap_open + G.gap_extend), ex = (_Float16)G.gap_extend;
  const gh2 OE = {oe, oe}, EX = {ex, ex};
  gh2 H[kGCells], F[kGCells];
  uint32_t Y[kFY];
  // row 0: H(0, j) = 0 at j = 0, -(open + j * extend) for 0 < j <= 16; F holds F(1, j)
#pragma unroll
  for (int d = 0; d < kGCells; ++d) {
    const int j = d - kGMaxBand;
    const _Float16 v = j < 0 ? ninf : (j == 0 ? (_Float16)0 : (_Float16)(-(G.gap_open + j * G.gap_extend)));
    H[d] = gh2{v, v};
    F[d] = H[d] - OE;
  }
  // letters under the band of the first block (rows 1..4): Y[k] = y index k - 16
#pragma unroll
  for (int g = 0; g < (kFY + 3) / 4; ++g) {
    uint32_t y4[4];
    L.ycols(4 * g - kGMaxBand, y4);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (4 * g + t < kFY) Y[4 * g + t] = y4[t];
  }
  uint32_t xbR[kFBlock], xbL[kFBlock];
  L.xrows<kFBlock>(1, xbR, xbL);
  gh2 best = {(_Float16)0, (_Float16)0};
  const char* tb = (const char*)tbl;
  for (int i0 = 1; __builtin_amdgcn_readfirstlane(__ballot(i0 <= rows) != 0); i0 += kFBlock) {
    // raw letters of the next block (x rows, and the y indices entering the band),
    // decoded after this block's rows
    const uint32_t nx4R = load4(L.A, L.qa + i0 + kFBlock - 1), nx4L = load4(L.A, L.qa - i0 - kFBlock - 3);
    const int k0 = i0 + kFY - kGMaxBand - 1;
    const uint32_t ny4R = load4(L.B, L.qb + k0), ny4L = load4(L.B, L.qb - 4 - k0);
#pragma unroll
    for (int r = 0; r < kFBlock; ++r) {
      gh2 e = NEG, hprev = NEG;
#pragma unroll
      for (int d = 0; d < kGCells; ++d) {
        const uint32_t y = Y[d + r];
        const _Float16 scR = *(const _Float16*)(tb + xbR[r] + (y & 0xffffu));
        const _Float16 scL = *(const _Float16*)(tb + xbL[r] + (y >> 16));
        const gh2 diag = H[d] + gh2{scR, scL};
        const gh2 f = d + 1 < kGCells ? F[d + 1] : NEG;
        const gh2 hh = gmax3(diag, e, f);
        if (d & 1) best = gmax3(best, hprev, hh);
        else if (d == kGCells - 1) best = gmax(best, hh);
        hprev = hh;
        const gh2 ho = hh - OE;
        e = gmax(e - EX, ho);
        F[d] = gmax(f - EX, ho);
        H[d] = hh;
      }
    }
#pragma unroll
    for (int k = 0; k + kFBlock < kFY; ++k) Y[k] = Y[k + kFBlock];
    const int i1 = i0 + kFBlock;
#pragma unroll
    for (int t = 0; t < kFBlock; ++t) {
      const int k = k0 + t;
      const uint32_t sr = (k >= 0 && k < L.lyR) ? byte_of(ny4R, t) : kWall8;
      const uint32_t sl = (k >= 0 && k < L.lyL) ? byte_of(ny4L, 3 - t) : kWall8;
      Y[kFY - kFBlock + t] = (sr / kScale) * kEntry | (((sl / kScale) * kEntry) << 16);
      const uint32_t xr = i1 + t <= L.lxR ? byte_of(nx4R, t) : kWall8;
      const uint32_t xl = i1 + t <= L.lxL ? byte_of(nx4L, 3 - t) : kWall8;
      xbR[t] = (xr / kScale) * kRowBytes;
      xbL[t] = (xl / kScale) * kRowBytes;
    }
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
  __shared__ uint32_t tbl[kTblDwords];  // filled once per workgroup
  for (int i = threadIdx.x; i < kTblDwords; i += NT) {
    const uint32_t lo = G.tbl16[2 * i], hi = 2 * i + 1 < kNLet * kNLet ? G.tbl16[2 * i + 1] : 0;
    tbl[i] = lo | (hi << 16);
  }
  if (n_dev) n_hits = min(n_hits, (int64_t)*n_dev);
  __syncthreads();
  // grid-stride over blocks of NT hits; no barrier inside the loop
  for (int64_t h = (int64_t)blockIdx.x * NT + threadIdx.x; h - threadIdx.x < n_hits; h += (int64_t)gridDim.x * NT)
    gapped_hit_f16(G, tbl, hits, h, n_hits, gscore, pass);
}

template <int NT>
int launch_fast(const GappedArgs& G, const plast_hit_t* d_hits, int64_t n_hits, const unsigned long long* d_n,
                int32_t* d_gscore, uint8_t* d_pass, hipStream_t stream) {
  const int64_t grid = (n_hits + NT - 1) / NT;
  hipLaunchKernelGGL(k_gapped_f16<NT>, dim3((unsigned)grid), dim3(NT), 0, stream, G, d_hits, n_hits, d_n, d_gscore,
                     d_pass);
  return PLAST_OK;
}

}  // namespace

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
      G.tbl16[x * kNLet + y] = (x < 20 && y < 20) ? __builtin_bit_cast(uint16_t, (_Float16)m[x * 20 + y]) : ninf16;
  // Every finite DP value lies within [-(64 |M| + 3 (open + extend) + 130 extend), 64 |M|]:
  // integers of that range are exact in binary16 when the bound stays below 2048.
  const bool fast = g->band == kGMaxBand && g->window <= kGMaxWin &&
                    64 * maxabs + 3 * (g->gap_open + g->gap_extend) + 130 * g->gap_extend <= 2000;
  const int threads = g->tuning ? g->tuning->gapped_threads : 256;
  if (n_hits <= 0) return PLAST_OK;
  timing_mark(kStageGapped, false, stream);
  if (fast) {
    if (threads == 128)
      launch_fast<128>(G, d_hits, n_hits, d_n, d_gscore, d_pass, stream);
    else if (threads == 512)
      launch_fast<512>(G, d_hits, n_hits, d_n, d_gscore, d_pass, stream);
    else
      launch_fast<256>(G, d_hits, n_hits, d_n, d_gscore, d_pass, stream);
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
