// Per-slice reductions for convergence and parity checks over the tiled
// state layout (padding lanes skipped): ||A-B||^2,
// ||B||^2, max |A-B| and a non-finite flag, with wavefront shuffles inside a
// workgroup and a fixed-order second pass, so results are bitwise
// reproducible for a given launch shape.

#include <hip/hip_runtime.h>

#include "wadg_internal.h"

namespace wadg {

constexpr int kNormThreads = 256;

__device__ inline void wave_reduce(double& sdd, double& sbb, double& mx, double& bad) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    sdd += __shfl_xor(sdd, off, 64);
    sbb += __shfl_xor(sbb, off, 64);
    mx = fmax(mx, __shfl_xor(mx, off, 64));
    bad = fmax(bad, __shfl_xor(bad, off, 64));
  }
}

__global__ __launch_bounds__(kNormThreads) void norms_partial_kernel(
    const double* __restrict__ A, const double* __restrict__ B, int64_t n, int tile, int K,
    int nblk, double* __restrict__ partials) {
  // one block per (slice, partial): slice-major, so the grid's one
  // dimension holds any slice count up to 2^31 / nblk
  const int s = blockIdx.x / nblk, blk = blockIdx.x - s * nblk, tid = threadIdx.x;
  const double* a = A + (size_t)s * n;
  const double* b = B ? B + (size_t)s * n : nullptr;
  double sdd = 0.0, sbb = 0.0, mx = 0.0, bad = 0.0;
  for (int64_t i = (int64_t)blk * kNormThreads + tid; i < n; i += (int64_t)nblk * kNormThreads) {
    // tiled layout: element = 64 * (i / tile) + (i % 64); skip padding lanes
    if ((i / tile) * kWave + (i & (kWave - 1)) >= K) continue;
    const double av = a[i];
    const double bv = b ? b[i] : 0.0;
    const double d = av - bv;
    sdd += d * d;
    sbb += bv * bv;
    mx = fmax(mx, fabs(d));
    if (!isfinite(av)) bad = 1.0;
  }
  wave_reduce(sdd, sbb, mx, bad);
  __shared__ double part[kNormThreads / 64][4];
  const int wv = tid >> 6, lane = tid & 63;
  if (lane == 0) {
    part[wv][0] = sdd; part[wv][1] = sbb; part[wv][2] = mx; part[wv][3] = bad;
  }
  __syncthreads();
  if (tid == 0) {
    double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
    for (int w = 0; w < kNormThreads / 64; ++w) {
      r0 += part[w][0]; r1 += part[w][1];
      r2 = fmax(r2, part[w][2]); r3 = fmax(r3, part[w][3]);
    }
    double* o = partials + ((size_t)s * nblk + blk) * 4;
    o[0] = r0; o[1] = r1; o[2] = r2; o[3] = r3;
  }
}

__global__ void norms_final_kernel(const double* __restrict__ partials, int nblk, int S,
                                   double* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
  for (int b = 0; b < nblk; ++b) {
    const double* o = partials + ((size_t)s * nblk + b) * 4;
    r0 += o[0]; r1 += o[1]; r2 = fmax(r2, o[2]); r3 = fmax(r3, o[3]);
  }
  out[4 * s + 0] = r0; out[4 * s + 1] = r1; out[4 * s + 2] = r2; out[4 * s + 3] = r3;
}

int launch_norms_final(const double* partials, int nblk, int32_t S, double* out, void* stream) {
  hipLaunchKernelGGL(norms_final_kernel, dim3((S + 63) / 64), dim3(64), 0,
                     static_cast<hipStream_t>(stream), partials, nblk, S, out);
  return (int)hipGetLastError();
}

int launch_norms(const double* A, const double* B, int32_t S, int64_t n_per_slice, int32_t tile,
                 int32_t K, double* partials, int nblk, double* out, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (nblk < 1 || S < 1 || (int64_t)nblk * S > INT32_MAX) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(norms_partial_kernel, dim3(nblk * S), dim3(kNormThreads), 0, st, A, B,
                     n_per_slice, tile, K, nblk, partials);
  int e = (int)hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(norms_final_kernel, dim3((S + 63) / 64), dim3(64), 0, st, partials, nblk, S,
                     out);
  return (int)hipGetLastError();
}

}  // namespace wadg
