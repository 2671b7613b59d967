// Per-slice L2 norms with the element maps' Jacobians (the norm of the L2
// errors of Section 5.2), on the tiled state layout:
//
//   ||A_s - B_s||^2 = sum_k sum_q w_q J_kq sum_f ((V_q (A_s - B_s)_f)_kq)^2
//
// over the context's volume rule (q = i + nq j, w_q = w_i w_j), and ||B_s||^2
// likewise.  One wave per (slice, 64-element group) item, one element per
// lane: the field values are interpolated to the quadrature points by the
// tensor-product operator V (rows in r, then in s), squared and weighted by
// w_q J_q = w_q / (1/J)_q from the geometry.  Padding lanes contribute
// nothing.  Each item's two sums go to `partials` [S * nEG][2]; a second
// kernel adds a slice's partials in a fixed order (no atomics), so the
// result is bitwise reproducible.

#include <hip/hip_runtime.h>

#include "reference_tables.h"
#include "stage_common.h"
#include "wadg_internal.h"

namespace wadg {
namespace {

using namespace dev;

constexpr int kL2FinalThreads = 256;

// sum_q wj_q ((V (x) V) x)_q^2 for one field's nodal values x of this lane.
template <int N, int NQ>
__device__ __forceinline__ double quad_square(const double (&x)[(N + 1) * (N + 1)],
                                              const double (&wj)[NQ * NQ]) {
  constexpr ct::Ops<double, N, NQ> T = ct::make_ops<double, N, NQ>();
  constexpr int NP1 = N + 1;
  double t[NP1][NQ];
#pragma unroll
  for (int b = 0; b < NP1; ++b)
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < NP1; ++a) s = mad(T.V[i][a], x[a + NP1 * b], s);
      t[b][i] = s;
    }
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < NQ; ++j)
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      double v = 0.0;
#pragma unroll
      for (int b = 0; b < NP1; ++b) v = mad(T.V[j][b], t[b][i], v);
      acc = mad(wj[i + NQ * j], v * v, acc);
    }
  return acc;
}

template <int N, int NQ>
__global__ __launch_bounds__(kWave) void l2_partial_kernel(const double* __restrict__ A,
                                                           const double* __restrict__ B,
                                                           const double* __restrict__ vol,
                                                           int nEG, int K,
                                                           double* __restrict__ partials) {
  constexpr ct::Tables<N, NQ> tb = ct::make_tables<N, NQ>();
  constexpr int NP = (N + 1) * (N + 1), NQ2 = NQ * NQ;
  constexpr size_t tile = (size_t)3 * NP * kWave;
  const int item = blockIdx.x;
  const int s = item / nEG, g = item - s * nEG;
  const int lane = threadIdx.x;
  const bool active = g * kWave + lane < K;
  const size_t off = ((size_t)s * nEG + g) * tile + lane;
  const double* a = A + off;
  const double* b = B ? B + off : nullptr;
  const double* inv_j = vol + ((size_t)g * 6 * NQ2 + 5 * NQ2) * kWave + lane;
  double wj[NQ2];
#pragma unroll
  for (int q = 0; q < NQ2; ++q)
    wj[q] = active ? (tb.wq[q % NQ] * tb.wq[q / NQ]) / inv_j[q * kWave] : 0.0;
  double sd = 0.0, sb = 0.0;
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    double d[NP], e[NP];
#pragma unroll
    for (int n = 0; n < NP; ++n) {
      const double av = a[(f * NP + n) * kWave];
      const double bv = b ? b[(f * NP + n) * kWave] : 0.0;
      d[n] = av - bv;
      e[n] = bv;
    }
    sd += quad_square<N, NQ>(d, wj);
    if (b) sb += quad_square<N, NQ>(e, wj);
  }
  // padding lanes may hold anything (their weights are zero, but 0 * inf
  // is not): they are dropped here
  if (!active) sd = sb = 0.0;
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) {
    sd += __shfl_xor(sd, o, kWave);
    sb += __shfl_xor(sb, o, kWave);
  }
  if (lane == 0) {
    partials[2 * (size_t)item] = sd;
    partials[2 * (size_t)item + 1] = sb;
  }
}

// One block per slice: each thread adds a strided run of the slice's item
// partials in order, then a fixed tree over the block.
__global__ __launch_bounds__(kL2FinalThreads) void l2_final_kernel(
    const double* __restrict__ partials, int nEG, double* __restrict__ out) {
  __shared__ double acc[2][kL2FinalThreads];
  const int s = blockIdx.x, t = threadIdx.x;
  const double* p = partials + 2 * (size_t)s * nEG;
  double sd = 0.0, sb = 0.0;
  for (int g = t; g < nEG; g += kL2FinalThreads) {
    sd += p[2 * (size_t)g];
    sb += p[2 * (size_t)g + 1];
  }
  acc[0][t] = sd;
  acc[1][t] = sb;
  __syncthreads();
  for (int w = kL2FinalThreads / 2; w >= 1; w >>= 1) {
    if (t < w) {
      acc[0][t] += acc[0][t + w];
      acc[1][t] += acc[1][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[2 * s] = acc[0][0];
    out[2 * s + 1] = acc[1][0];
  }
}

template <int N, int NQ>
int launch_nq(const double* A, const double* B, const double* vol, int32_t S, int32_t nEG,
              int32_t K, double* partials, double* out, hipStream_t st) {
  hipLaunchKernelGGL((l2_partial_kernel<N, NQ>), dim3(S * nEG), dim3(kWave), 0, st, A, B, vol,
                     nEG, K, partials);
  int e = (int)hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(l2_final_kernel, dim3(S), dim3(kL2FinalThreads), 0, st, partials, nEG, out);
  return (int)hipGetLastError();
}

template <int N>
int launch_n(int nq, const double* A, const double* B, const double* vol, int32_t S,
             int32_t nEG, int32_t K, double* partials, double* out, hipStream_t st) {
  switch (nq - N) {
    case 1: return launch_nq<N, N + 1>(A, B, vol, S, nEG, K, partials, out, st);
    case 2: return launch_nq<N, N + 2>(A, B, vol, S, nEG, K, partials, out, st);
    case 3: return launch_nq<N, N + 3>(A, B, vol, S, nEG, K, partials, out, st);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace

int launch_l2_norms(int N, int nq, const double* A, const double* B, const double* vol,
                    int32_t S, int32_t nEG, int32_t K, double* partials, double* out,
                    void* stream) {
  if (S < 1 || nEG < 1 || (int64_t)S * nEG > INT32_MAX) return (int)hipErrorInvalidValue;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (N) {
    case 1: return launch_n<1>(nq, A, B, vol, S, nEG, K, partials, out, st);
    case 2: return launch_n<2>(nq, A, B, vol, S, nEG, K, partials, out, st);
    case 3: return launch_n<3>(nq, A, B, vol, S, nEG, K, partials, out, st);
    case 4: return launch_n<4>(nq, A, B, vol, S, nEG, K, partials, out, st);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace wadg
