// TPLAST-N (Sec. 6): six-frame translation of a nucleotide bank on the device.
//
// Frames 0..2 read the forward strand from nucleotide 0, 1 or 2; frames 3..5
// read the reverse complement the same way; a trailing partial codon is
// dropped.  The standard genetic code maps each codon to an amino acid or a
// stop, and stops cut every frame into fragments; each non-empty fragment
// becomes one protein sequence of the output bank (padded layout), so that seed
// windows never cross a stop.  Fragment j is described by (DNA sequence, frame,
// offset of its first amino acid in the frame).
//
// One workgroup per (sequence, frame) stream.  Pass 1 counts the stream's
// fragments and amino acids; an exclusive scan over the streams gives each
// stream its first fragment and first residue; pass 2 writes every amino acid
// to 20 (fragment + 1) + (residues before it), since the layout is a separator
// run, fragment 0, a run, fragment 1, ... .  Pass 1 only sums each thread's
// counts; inside a stream, pass 2 ranks fragment starts and amino acids with a
// workgroup scan per 1024-codon chunk (four consecutive codons per thread).
#include "plast_internal.h"

namespace plast {

namespace {

// Standard genetic code (NCBI table 1): the amino acid of codon b1 b2 b3, bases
// in the order A C G T, first base slowest; '*' = stop.  This library's
// transcription.
constexpr char kCodeACGT[65] = "KNKNTTTTRSRSIIMIQHQHPPPPRRRRLLLLEDEDAAAAGGGGVVVV*Y*YSSSS*CWCLFLF";
constexpr uint8_t kStop = 0xff;
constexpr int kTrThreads = 256;

struct CodonTable {
  uint8_t aa[64];  // residue code (ACDEFGHIKLMNPQRSTVWY order) or kStop
};

CodonTable codon_table() {
  static const char* kOrder = "ACDEFGHIKLMNPQRSTVWY";
  CodonTable t;
  for (int i = 0; i < 64; ++i) {
    const char c = kCodeACGT[i];
    t.aa[i] = kStop;
    for (int k = 0; k < 20; ++k)
      if (kOrder[k] == c) t.aa[i] = (uint8_t)k;
  }
  return t;
}

struct Stream {
  int64_t start, len;  // the DNA sequence
  int frame;
  int64_t n_codons;
};

__device__ __forceinline__ Stream stream_of(const int64_t* __restrict__ dna_start, int32_t n_dna, int64_t n_nt,
                                            int s, int32_t* __restrict__ err) {
  Stream S;
  const int d = s / 6;
  S.frame = s % 6;
  S.start = dna_start[d];
  const int64_t end = dna_start[d + 1];
  S.len = end - S.start;
  if (S.start < 0 || end > n_nt || S.len < 0) {  // inconsistent offsets: an empty stream
    if (threadIdx.x == 0 && S.frame == 0) atomicOr(err, 1);
    S.start = 0;
    S.len = 0;
  }
  const int off = S.frame % 3;
  S.n_codons = S.len > off ? (S.len - off) / 3 : 0;
  return S;
}

// Residue code of codon i of a stream, or kStop.
__device__ __forceinline__ uint8_t codon_aa(const uint8_t* __restrict__ dna, const Stream& S, int64_t i,
                                            const CodonTable& T) {
  const int64_t q = S.frame % 3 + 3 * i;  // first nucleotide in the frame's strand
  uint32_t b1, b2, b3;
  if (S.frame < 3) {
    const uint8_t* p = dna + S.start + q;
    b1 = p[0];
    b2 = p[1];
    b3 = p[2];
  } else {  // reverse complement: strand position q is forward position len - 1 - q
    const uint8_t* p = dna + S.start + S.len - 1 - q;
    b1 = 3u - p[0];
    b2 = 3u - p[-1];
    b3 = 3u - p[-2];
  }
  return T.aa[((b1 & 3u) << 4) | ((b2 & 3u) << 2) | (b3 & 3u)];
}

__device__ __forceinline__ int wave_incl_sum(int v) {
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

// Workgroup-wide inclusive scan of v (all threads call it; contains barriers).
__device__ __forceinline__ int block_incl_sum(int v, int* wtot, int* total) {
  const int w = threadIdx.x >> 6, lane = __lane_id();
  const int incl = wave_incl_sum(v);
  if (lane == 63) wtot[w] = incl;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < kTrThreads / 64; ++k) {
    before += k < w ? wtot[k] : 0;
    all += wtot[k];
  }
  __syncthreads();
  *total = all;
  return before + incl;
}

// Workgroup-wide sum (all threads call it; contains barriers).
__device__ __forceinline__ long long block_sum64(long long v, long long* wsum) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  __syncthreads();  // wsum may still be read by a previous call
  if (__lane_id() == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  long long t = 0;
#pragma unroll
  for (int k = 0; k < kTrThreads / 64; ++k) t += wsum[k];
  return t;
}

// Pass 1: per stream, fragments and amino acids; frame-0 workgroups also check
// that every nucleotide code is 0..3.
__global__ __launch_bounds__(kTrThreads) void k_tr_count(const uint8_t* __restrict__ dna,
                                                         const int64_t* __restrict__ dna_start, int32_t n_dna,
                                                         int64_t n_nt, CodonTable T, int64_t* __restrict__ nfrag,
                                                         int64_t* __restrict__ nres, int32_t* __restrict__ err) {
  __shared__ long long wsum[kTrThreads / 64];
  const int s = blockIdx.x;
  const Stream S = stream_of(dna_start, n_dna, n_nt, s, err);
  if (S.frame == 0) {
    bool bad = false;
    for (int64_t p = threadIdx.x; p < S.len; p += kTrThreads) bad |= dna[S.start + p] > 3;
    if (bad) atomicOr(err, 2);
  }
  // each thread counts its own codons; one sum over the workgroup at the end
  long long frags = 0, res = 0;
  for (int64_t i = threadIdx.x; i < S.n_codons; i += kTrThreads) {
    const bool aa_ok = codon_aa(dna, S, i, T) != kStop;
    frags += (aa_ok && (i == 0 || codon_aa(dna, S, i - 1, T) == kStop)) ? 1 : 0;
    res += aa_ok ? 1 : 0;
  }
  frags = block_sum64(frags, wsum);
  res = block_sum64(res, wsum);
  if (threadIdx.x == 0) {
    nfrag[s] = frags;
    nres[s] = res;
  }
}

// Exclusive scans of both counts over the streams (one workgroup), totals at [n].
__global__ __launch_bounds__(kTrThreads) void k_tr_scan(int64_t* __restrict__ nfrag, int64_t* __restrict__ nres,
                                                        int n) {
  __shared__ long long part[2][kTrThreads];
  __shared__ long long carry[2];
  if (threadIdx.x == 0) carry[0] = carry[1] = 0;
  __syncthreads();
  for (int base = 0; base < n; base += kTrThreads) {
    const int s = base + threadIdx.x;
    const long long f = s < n ? nfrag[s] : 0, r = s < n ? nres[s] : 0;
    part[0][threadIdx.x] = f;
    part[1][threadIdx.x] = r;
    __syncthreads();
    for (int d = 1; d < kTrThreads; d <<= 1) {
      const long long tf = threadIdx.x >= d ? part[0][threadIdx.x - d] : 0;
      const long long tr = threadIdx.x >= d ? part[1][threadIdx.x - d] : 0;
      __syncthreads();
      part[0][threadIdx.x] += tf;
      part[1][threadIdx.x] += tr;
      __syncthreads();
    }
    if (s < n) {
      nfrag[s] = carry[0] + part[0][threadIdx.x] - f;
      nres[s] = carry[1] + part[1][threadIdx.x] - r;
    }
    __syncthreads();
    if (threadIdx.x == kTrThreads - 1) {
      carry[0] += part[0][kTrThreads - 1];
      carry[1] += part[1][kTrThreads - 1];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    nfrag[n] = carry[0];
    nres[n] = carry[1];
  }
}

__global__ void k_tr_clear(int32_t* __restrict__ err) {
  if (threadIdx.x == 0) *err = 0;
}

__global__ void k_tr_fill(uint8_t* __restrict__ codes, int64_t n, int64_t* __restrict__ seq_start, int64_t n_frags) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) codes[i] = kPadCode;
  if (blockIdx.x == 0 && threadIdx.x == 0) seq_start[n_frags] = n;
}

// Pass 2: amino acids, fragment starts and the fragment table.
__global__ __launch_bounds__(kTrThreads) void k_tr_write(const uint8_t* __restrict__ dna,
                                                         const int64_t* __restrict__ dna_start, int32_t n_dna,
                                                         int64_t n_nt, CodonTable T,
                                                         const int64_t* __restrict__ frag0,
                                                         const int64_t* __restrict__ res0, uint8_t* __restrict__ codes,
                                                         int64_t n_padded, int64_t* __restrict__ seq_start,
                                                         int32_t* __restrict__ frag, int64_t n_frags,
                                                         int32_t* __restrict__ err) {
  __shared__ int wtot[kTrThreads / 64];
  const int s = blockIdx.x;
  const Stream S = stream_of(dna_start, n_dna, n_nt, s, err);
  int64_t cf = frag0[s], cr = res0[s];  // fragments and residues before this chunk
  // Chunks of 4 * kTrThreads codons, four consecutive codons per thread: the
  // workgroup ranks thread totals (each at most 4, so a chunk's totals fit the
  // 16-bit halves of the scan), then every thread walks its own codons.
  constexpr int kPer = 4;
  for (int64_t base = 0; base < S.n_codons; base += kPer * kTrThreads) {
    const int64_t i0 = base + kPer * threadIdx.x;
    uint8_t aa[kPer];
    bool first[kPer];
    uint8_t prev = (i0 == 0 || i0 > S.n_codons) ? kStop : codon_aa(dna, S, i0 - 1, T);
    int nf = 0, nr = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int64_t i = i0 + k;
      aa[k] = i < S.n_codons ? codon_aa(dna, S, i, T) : kStop;
      first[k] = aa[k] != kStop && prev == kStop;
      prev = aa[k];
      nf += first[k] ? 1 : 0;
      nr += aa[k] != kStop ? 1 : 0;
    }
    const int mine = (nf << 16) | nr;
    int tot = 0;
    const int excl = block_incl_sum(mine, wtot, &tot) - mine;
    int64_t j = cf + (excl >> 16) - 1;  // fragment of the last start before this thread's codons
    int64_t r = cr + (excl & 0xffff);   // residues before them
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (aa[k] == kStop) continue;
      if (first[k]) ++j;
      const int64_t pos = (int64_t)kPadLen * (j + 1) + r;
      if (j >= 0 && j < n_frags && pos < n_padded) {
        codes[pos] = aa[k];
        if (first[k]) {
          seq_start[j] = pos;
          frag[3 * j] = s / 6;
          frag[3 * j + 1] = S.frame;
          frag[3 * j + 2] = (int32_t)(i0 + k);
        }
      }
      ++r;
    }
    cf += tot >> 16;
    cr += tot & 0xffff;
  }
}

struct TrWs {
  int32_t* err;
  int64_t* nfrag;
  int64_t* nres;
};

TrWs tr_carve(void* d_ws, int32_t n_dna) {
  uint8_t* p = (uint8_t*)d_ws;
  TrWs W;
  W.err = (int32_t*)p;
  W.nfrag = (int64_t*)(p + 256);
  W.nres = (int64_t*)(p + 256 + align_up(sizeof(int64_t) * (6 * (size_t)n_dna + 1), 256));
  return W;
}

}  // namespace

size_t translate_ws_bytes(int32_t n_dna) {
  return 256 + 2 * align_up(sizeof(int64_t) * (6 * (size_t)n_dna + 1), 256);
}

int translate_count_impl(const uint8_t* d_dna, const int64_t* d_dna_start, int32_t n_dna, int64_t n_nt, void* d_ws,
                         int64_t* h_n_frags, int64_t* h_n_padded, hipStream_t s) {
  TrWs W = tr_carve(d_ws, n_dna);
  const CodonTable T = codon_table();
  const int streams = 6 * n_dna;
  hipLaunchKernelGGL(k_tr_clear, dim3(1), dim3(64), 0, s, W.err);
  hipLaunchKernelGGL(k_tr_count, dim3((unsigned)(streams > 0 ? streams : 1)), dim3(kTrThreads), 0, s, d_dna,
                     d_dna_start, n_dna, n_nt, T, W.nfrag, W.nres, W.err);
  hipLaunchKernelGGL(k_tr_scan, dim3(1), dim3(kTrThreads), 0, s, W.nfrag, W.nres, streams);
  PLAST_HIP(hipGetLastError());
  int32_t err = 0;
  int64_t tf = 0, tr = 0;
  PLAST_HIP(hipMemcpyAsync(&err, W.err, sizeof(err), hipMemcpyDeviceToHost, s));
  PLAST_HIP(hipMemcpyAsync(&tf, W.nfrag + streams, sizeof(tf), hipMemcpyDeviceToHost, s));
  PLAST_HIP(hipMemcpyAsync(&tr, W.nres + streams, sizeof(tr), hipMemcpyDeviceToHost, s));
  PLAST_HIP(hipStreamSynchronize(s));
  if (err & 1) return set_error(PLAST_E_LAYOUT, "dna_start is not ascending within [0, n_nt]");
  if (err & 2) return set_error(PLAST_E_ALPHABET, "a nucleotide code is > 3");
  *h_n_frags = tf;
  *h_n_padded = (int64_t)kPadLen * (tf + 1) + tr;
  return PLAST_OK;
}

int translate_write_impl(const uint8_t* d_dna, const int64_t* d_dna_start, int32_t n_dna, int64_t n_nt, void* d_ws,
                         uint8_t* d_codes, int64_t n_padded, int64_t* d_seq_start, int32_t* d_frag, int64_t n_frags,
                         hipStream_t s) {
  TrWs W = tr_carve(d_ws, n_dna);
  const CodonTable T = codon_table();
  const int streams = 6 * n_dna;
  const int64_t fill_blocks = (n_padded + 255) / 256 < 4096 ? (n_padded + 255) / 256 : 4096;
  hipLaunchKernelGGL(k_tr_fill, dim3((unsigned)(fill_blocks > 0 ? fill_blocks : 1)), dim3(256), 0, s, d_codes,
                     n_padded, d_seq_start, n_frags);
  if (streams > 0)
    hipLaunchKernelGGL(k_tr_write, dim3((unsigned)streams), dim3(kTrThreads), 0, s, d_dna, d_dna_start, n_dna, n_nt,
                       T, (const int64_t*)W.nfrag, (const int64_t*)W.nres, d_codes, n_padded, d_seq_start, d_frag,
                       n_frags, W.err);
  PLAST_HIP(hipGetLastError());
  return PLAST_OK;
}

}  // namespace plast
