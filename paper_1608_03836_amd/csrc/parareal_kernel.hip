// Parareal correction update for one slice, in FP64 on the GPU:
//
//   U_{s+1}^{k+1} = G(U_s^{k+1}) + F(U_s^k) - G(U_s^k)
//
// fused with the bookkeeping of the iteration: the new coarse value replaces
// the stored one, and the per-slice reductions of the change
// ||U_{s+1}^{k+1} - U_{s+1}^k||^2, ||U_{s+1}^{k+1}||^2, max |change| and a
// non-finite flag are written as block partials (fixed-order reduction, as
// for the norms).  Padding lanes of the tiled layout are skipped.

#include <hip/hip_runtime.h>

#include "wadg_internal.h"

namespace wadg {

constexpr int kCorrThreads = 256;

__global__ __launch_bounds__(kCorrThreads) void parareal_correct_kernel(
    const double* __restrict__ g, const double* __restrict__ f, double* __restrict__ gold,
    double* __restrict__ u, int64_t n, int tile, int K, int nblk, double* __restrict__ partials) {
  const int blk = blockIdx.x, tid = threadIdx.x;
  double sdd = 0.0, snn = 0.0, mx = 0.0, bad = 0.0;
  for (int64_t i = (int64_t)blk * kCorrThreads + tid; i < n; i += (int64_t)nblk * kCorrThreads) {
    if ((i / tile) * kWave + (i & (kWave - 1)) >= K) continue;
    const double gv = g[i];
    const double nv = gv + f[i] - gold[i];
    const double d = nv - u[i];
    u[i] = nv;
    gold[i] = gv;
    sdd += d * d;
    snn += nv * nv;
    mx = fmax(mx, fabs(d));
    if (!isfinite(nv)) bad = 1.0;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    sdd += __shfl_xor(sdd, off, 64);
    snn += __shfl_xor(snn, off, 64);
    mx = fmax(mx, __shfl_xor(mx, off, 64));
    bad = fmax(bad, __shfl_xor(bad, off, 64));
  }
  __shared__ double part[kCorrThreads / 64][4];
  const int wv = tid >> 6, lane = tid & 63;
  if (lane == 0) {
    part[wv][0] = sdd; part[wv][1] = snn; part[wv][2] = mx; part[wv][3] = bad;
  }
  __syncthreads();
  if (tid == 0) {
    double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
    for (int w = 0; w < kCorrThreads / 64; ++w) {
      r0 += part[w][0]; r1 += part[w][1];
      r2 = fmax(r2, part[w][2]); r3 = fmax(r3, part[w][3]);
    }
    double* o = partials + (size_t)blk * 4;
    o[0] = r0; o[1] = r1; o[2] = r2; o[3] = r3;
  }
}

int launch_parareal_correct(const double* g, const double* f, double* gold, double* u,
                            int64_t n, int32_t tile, int32_t K, double* partials, int nblk,
                            void* stream) {
  hipLaunchKernelGGL(parareal_correct_kernel, dim3(nblk), dim3(kCorrThreads), 0,
                     static_cast<hipStream_t>(stream), g, f, gold, u, n, tile, K, nblk, partials);
  return (int)hipGetLastError();
}

}  // namespace wadg
