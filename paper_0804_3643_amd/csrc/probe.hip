// Measured denominators for the rooflines: short kernels that run one kind of
// work at the highest rate the chip sustains, timed with HIP events.
//
// * VALU, int32: independent add-then-max chains (two VALU operations per
//   update), the operation mix of the DP recurrences.
// * VALU, packed 16-bit integer and packed binary16: the same chains on
//   two-element vectors, two operations per lane per instruction.
// * LDS: 32-bit table lookups, each 64-lane read on 64 consecutive words (no
//   bank conflict), the access pattern of the per-lane score profiles of the
//   alignment kernel.
// * LDS, 64-bit: the access of the ungapped kernel's profile: per step, one
//   bit-field extract of the lane's letter and eight 8-byte reads, each
//   64-lane read spread over the 21 letter entries of one step (8 bytes
//   apart), so lanes with equal letters share an address.
// * HBM: a copy between the two halves of a buffer, four 16-byte loads in
//   flight per lane.
// * Engine clock: the int32 chains, timed inside the kernel by the
//   engine-clock and constant-rate counters, so that a rate can be put per
//   clock of the clock the chip actually ran at.
//
// Every compute probe writes one value per thread, so no chain is dead code.
#include <algorithm>
#include <vector>

#include "plast_internal.h"

namespace plast {

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeBlocks = 2048;  // 8 waves per SIMD on 256 CUs
constexpr int kChains = 8;

typedef short short2v __attribute__((ext_vector_type(2)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(kProbeThreads) void k_probe_i32(int32_t* __restrict__ out, int iters, int seed) {
  int a[kChains];
  const int x = (seed ^ (int)threadIdx.x) & 7, y = -seed;
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = (int)threadIdx.x + k * seed;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = max((int)((unsigned)a[k] + (unsigned)x), y + k);
  }
  int s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s ^= a[k];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// The same chains, with the first wavefront of each workgroup reading the
// engine-clock counter (s_memtime) and the constant-rate counter
// (s_memrealtime) on both sides of its loop: over the loop, the ratio of the
// two deltas times the constant rate is the engine clock the chains ran at.
__global__ __launch_bounds__(kProbeThreads) void k_probe_i32_clock(int32_t* __restrict__ out,
                                                                   uint64_t* __restrict__ clk, int iters, int seed) {
  const bool first = threadIdx.x < 64;
  uint64_t c0 = 0, w0 = 0;
  if (first) {
    c0 = __builtin_amdgcn_s_memtime();
    w0 = __builtin_amdgcn_s_memrealtime();
  }
  int a[kChains];
  const int x = (seed ^ (int)threadIdx.x) & 7, y = -seed;
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = (int)threadIdx.x + k * seed;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = max((int)((unsigned)a[k] + (unsigned)x), y + k);
  }
  int s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s ^= a[k];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
  if (first) {
    const uint64_t c1 = __builtin_amdgcn_s_memtime(), w1 = __builtin_amdgcn_s_memrealtime();
    if (threadIdx.x == 0) {
      clk[2 * blockIdx.x] = c1 - c0;
      clk[2 * blockIdx.x + 1] = w1 - w0;
    }
  }
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_pk_i16(int32_t* __restrict__ out, int iters, int seed) {
  short2v a[kChains];
  const short2v x = {(short)((seed ^ threadIdx.x) & 7), (short)(seed & 3)};
  const short2v y = {(short)-seed, (short)(1 - seed)};
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = short2v{(short)(threadIdx.x + k), (short)(k * seed)};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = __builtin_elementwise_max(a[k] + x, y);
  }
  int s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s ^= (int)a[k].x ^ ((int)a[k].y << 16);
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_pk_f16(int32_t* __restrict__ out, int iters, int seed) {
  half2v a[kChains];
  const half2v x = {(_Float16)(-(int)((seed ^ threadIdx.x) & 3)), (_Float16)(-1)};
  const half2v y = {(_Float16)(-seed), (_Float16)(-2 * seed)};
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = half2v{(_Float16)(int)(threadIdx.x & 63), (_Float16)k};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = __builtin_elementwise_max(a[k] + x, y);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += (float)a[k].x + (float)a[k].y;
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = (int32_t)s;
}

constexpr int kLdsWords = 64 * 64;  // 16 KB table

__global__ __launch_bounds__(kProbeThreads) void k_probe_lds(int32_t* __restrict__ out, int iters, int seed) {
  __shared__ int32_t tbl[kLdsWords];
  for (int i = threadIdx.x; i < kLdsWords; i += blockDim.x) tbl[i] = i * 3 + seed;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  int acc[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) acc[k] = 0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) acc[k] += tbl[lane + 64 * ((it + 8 * k) & 63)];
  }
  int s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s ^= acc[k];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

constexpr int kL64Steps = 16;
constexpr int kL64Letters = 21;

// Per iteration 16 steps x 8 reads of 8 bytes; the letters rotate every
// iteration so that no read can be hoisted out of the loop.
__global__ __launch_bounds__(kProbeThreads) void k_probe_lds_b64(int32_t* __restrict__ out, int iters, int seed) {
  __shared__ uint2 tbl[kChains][kL64Steps][kL64Letters];
  uint2* flat = &tbl[0][0][0];
  for (int i = threadIdx.x; i < kChains * kL64Steps * kL64Letters; i += blockDim.x)
    flat[i] = make_uint2((uint32_t)(i * 3 + seed), (uint32_t)(i ^ seed));
  __syncthreads();
  const int lane = threadIdx.x & 63;
  uint32_t let[4];  // 16 letters as (letter * 8) bytes
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t w = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) w |= (uint32_t)(((lane * 5 + (4 * j + b) * 7 + seed) % kL64Letters) * 8) << (8 * b);
    let[j] = w;
  }
  uint2 acc[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) acc[k] = make_uint2(0u, 0u);
  const uint8_t* base = (const uint8_t*)flat;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int t = 0; t < kL64Steps; ++t) {
      const uint32_t c8 = __builtin_amdgcn_ubfe(let[t >> 2], 8 * (t & 3), 8);
      const uint8_t* p = base + c8 + t * (kL64Letters * 8);
#pragma unroll
      for (int k = 0; k < kChains; ++k) {
        const uint2 v = *(const uint2*)(p + k * (kL64Steps * kL64Letters * 8));
        acc[k].x ^= v.x;
        acc[k].y += v.y;
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) let[j] = __builtin_amdgcn_alignbit(let[j], let[j], 8);
  }
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s ^= acc[k].x + acc[k].y;
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = (int32_t)s;
}

// Four independent 16-byte loads in flight per lane before their stores.
__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const int4* __restrict__ src, int4* __restrict__ dst,
                                                              int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const int4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

}  // namespace plast

extern "C" int plast_probe_peak(int32_t kind, void* d_buf, size_t buf_bytes, int32_t reps, double* rate,
                                void* stream_) {
  using namespace plast;
  hipStream_t stream = (hipStream_t)stream_;
  if (!d_buf || !rate) return set_error(PLAST_E_ARG, "plast_probe_peak: null pointer");
  if (kind < PLAST_PROBE_VALU_I32 || kind > PLAST_PROBE_SCLK)
    return set_error(PLAST_E_ARG, "plast_probe_peak: unknown kind %d", (int)kind);
  if (reps < 1 || reps > 100) return set_error(PLAST_E_ARG, "plast_probe_peak: reps must be in 1..100");
  if ((uintptr_t)d_buf & 255) return set_error(PLAST_E_ARG, "plast_probe_peak: buffer must be 256-byte aligned");
  const size_t out_bytes = sizeof(int32_t) * (size_t)kProbeBlocks * kProbeThreads;
  const size_t clk_bytes = sizeof(uint64_t) * 2 * (size_t)kProbeBlocks;  // the clock probe's counter deltas
  const size_t need =
      kind == PLAST_PROBE_HBM_COPY ? ((size_t)1 << 20) : out_bytes + (kind == PLAST_PROBE_SCLK ? clk_bytes : 0);
  if (buf_bytes < need)
    return set_error(PLAST_E_WORKSPACE, "plast_probe_peak: buffer of %zu bytes, needs at least %zu", buf_bytes, need);
  // about 3.5 ms per launch at the published peaks (1.7 ms for the LDS probe)
  const int iters = kind == PLAST_PROBE_LDS ? 8192 : kind == PLAST_PROBE_LDS_B64 ? 512 : 16384;
  const double threads = (double)kProbeBlocks * kProbeThreads;
  double work = 0.0;  // operations, lookups or bytes per launch
  int64_t n16 = 0;
  switch (kind) {
    case PLAST_PROBE_VALU_I32:
    case PLAST_PROBE_SCLK: work = threads * iters * kChains * 2.0; break;
    case PLAST_PROBE_VALU_PK_I16:
    case PLAST_PROBE_VALU_PK_F16: work = threads * iters * kChains * 4.0; break;
    case PLAST_PROBE_LDS: work = threads * iters * kChains; break;
    case PLAST_PROBE_LDS_B64: work = threads * iters * kL64Steps * kChains * 8.0; break;
    default:
      n16 = (int64_t)(buf_bytes / 2 / 16);
      work = 2.0 * 16.0 * (double)n16;
      break;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = PLAST_OK;
  double best = 0.0;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = set_error(PLAST_E_HIP, "plast_probe_peak: hipEventCreate failed");
  }
  for (int r = 0; rc == PLAST_OK && r <= reps; ++r) {  // launch 0 warms up
    (void)hipEventRecord(e0, stream);
    int32_t* out = (int32_t*)d_buf;
    switch (kind) {
      case PLAST_PROBE_VALU_I32:
        hipLaunchKernelGGL(k_probe_i32, dim3(kProbeBlocks), dim3(kProbeThreads), 0, stream, out, iters, r + 1);
        break;
      case PLAST_PROBE_VALU_PK_I16:
        hipLaunchKernelGGL(k_probe_pk_i16, dim3(kProbeBlocks), dim3(kProbeThreads), 0, stream, out, iters, r + 1);
        break;
      case PLAST_PROBE_VALU_PK_F16:
        hipLaunchKernelGGL(k_probe_pk_f16, dim3(kProbeBlocks), dim3(kProbeThreads), 0, stream, out, iters, r + 1);
        break;
      case PLAST_PROBE_LDS:
        hipLaunchKernelGGL(k_probe_lds, dim3(kProbeBlocks), dim3(kProbeThreads), 0, stream, out, iters, r + 1);
        break;
      case PLAST_PROBE_LDS_B64:
        hipLaunchKernelGGL(k_probe_lds_b64, dim3(kProbeBlocks), dim3(kProbeThreads), 0, stream, out, iters, r + 1);
        break;
      case PLAST_PROBE_SCLK:
        hipLaunchKernelGGL(k_probe_i32_clock, dim3(kProbeBlocks), dim3(kProbeThreads), 0, stream, out,
                           (uint64_t*)((uint8_t*)d_buf + out_bytes), iters, r + 1);
        break;
      default: {
        const int4* src = (const int4*)d_buf;
        int4* dst = (int4*)((uint8_t*)d_buf + (size_t)n16 * 16);
        hipLaunchKernelGGL(k_probe_copy, dim3(kProbeBlocks), dim3(kProbeThreads), 0, stream, src, dst, n16);
      }
    }
    if (hipGetLastError() != hipSuccess || hipEventRecord(e1, stream) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess) {
      rc = set_error(PLAST_E_HIP, "plast_probe_peak: launch or event failed");
      break;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.f) {
      rc = set_error(PLAST_E_HIP, "plast_probe_peak: hipEventElapsedTime failed");
      break;
    }
    if (r > 0 && work / (ms * 1e-3) > best) best = work / (ms * 1e-3);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc == PLAST_OK && kind == PLAST_PROBE_SCLK) {
    // median over the workgroups of the last launch of (engine cycles /
    // constant-rate ticks) times the constant rate
    std::vector<uint64_t> d(2 * (size_t)kProbeBlocks);
    int dev = 0, khz = 0;
    if (hipMemcpyAsync(d.data(), (uint8_t*)d_buf + out_bytes, clk_bytes, hipMemcpyDeviceToHost, stream) !=
            hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
      return set_error(PLAST_E_HIP, "plast_probe_peak: reading the clock counters failed");
    std::vector<double> ratio;
    for (int b = 0; b < kProbeBlocks; ++b)
      if (d[2 * b + 1] > 0) ratio.push_back((double)d[2 * b] / (double)d[2 * b + 1]);
    if (ratio.empty()) return set_error(PLAST_E_HIP, "plast_probe_peak: the constant-rate counter did not advance");
    std::nth_element(ratio.begin(), ratio.begin() + ratio.size() / 2, ratio.end());
    best = ratio[ratio.size() / 2] * (double)khz * 1e3;
  }
  if (rc == PLAST_OK) *rate = best;
  return rc;
}
