// Adjoint mass step of the discrete adjoint sweep (FP64, gfx950).
//
// The semi-discrete operator is L = Mtilde^{-1} A, with Mtilde^{-1} the
// block-diagonal weight-adjusted inverse (Section 4; Section 7 for c^2) and
// A the strong-weak DG operator (Section 4.1).  In the strong-weak form the
// volume and central-flux couplings of p with (u, v) are exact negative
// transposes of each other and the penalty blocks are symmetric, so
// A^T = D A D with D = diag(1, -1, -1), and since Mtilde^{-1} is symmetric,
//
//     L^T rbar = D A (D Mtilde^{-1} rbar).
//
// The reverse sweep of one 2N-storage stage i (rbar += B_i ybar;
// ybar += dt L^T rbar; rbar *= A_i) is therefore two launches: this kernel,
//
//     rbar <- a rbar + B_i ybar     (a = A_{i+1}, folded in from stage i+1)
//     z    <- D Mtilde^{-1} rbar
//     part <- part + sum_p rbar_p (r_i - A_i r_{i-1})_p,
//
// whose last line accumulates the sensitivity to a scale gamma of c^2
// (c^2 enters L only through the pressure rows, linearly, and
// dt L q_{i-1} = r_i - A_i r_{i-1} from the forward residuals), then the
// stage kernel in apply-A mode: ybar <- ybar + dt D A z.
//
// One workgroup per (slice, 64-element group), two waves: wave 0 the
// pressure field (weights c2_scale c^2/J) and the sensitivity term, wave 1
// the two velocity fields (weights 1/J).  One partial-sum slot per
// workgroup, updated by that workgroup only: deterministic, no atomics.

#include <hip/hip_runtime.h>

#include "stage_common.h"

namespace wadg {
namespace {

using namespace dev;

struct AdjMass {
  double* rbar;
  const double* ybar;
  double* z;
  const double* r_i;
  const double* r_prev;
  const double* vol;
  double* part;
  int32_t K, S, nEG;
  double a_next, b_i, a_i, c2s;
};

template <int N, int NQ>
__global__ __launch_bounds__(2 * kWave) void adjoint_mass_kernel(const AdjMass a) {
  constexpr int NP = (N + 1) * (N + 1), NQ2 = NQ * NQ;
  constexpr unsigned tile = 3u * NP * kWave;
  constexpr unsigned tb = tile * sizeof(double);
  constexpr unsigned KP = kWave * sizeof(double);
  const int w = blockIdx.x;   // slice * nEG + group
  const int eg = w % a.nEG;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & (kWave - 1);
  const unsigned kb = (unsigned)lane * sizeof(double);
  const size_t t0 = (size_t)w * tile;
  const rsrc_t rb_r = make_rsrc(a.rbar + t0, a.a_next != 0.0 ? tb : 0u);
  const rsrc_t rb_w = make_rsrc(a.rbar + t0, tb);
  const rsrc_t yb = make_rsrc(a.ybar + t0, tb);
  const rsrc_t zw = make_rsrc(a.z + t0, tb);
  const rsrc_t ri = make_rsrc(a.r_i + t0, tb);
  const rsrc_t rp = make_rsrc(a.r_prev ? a.r_prev + t0 : a.r_i + t0,
                              (a.a_i != 0.0 && a.r_prev) ? tb : 0u);
  const rsrc_t vol = make_rsrc(a.vol + (size_t)eg * 6 * NQ2 * kWave, 6u * NQ2 * KP);
  const bool active = eg * kWave + lane < a.K;

  const int c0 = wave == 0 ? 0 : 1, c1 = wave == 0 ? 1 : 3;
  double wq[NQ2];
#pragma unroll
  for (int q = 0; q < NQ2; ++q)
    wq[q] = wave == 0 ? a.c2s * ldr<double>(vol, kb, (4 * NQ2 + q) * KP)
                      : ldr<double>(vol, kb, (5 * NQ2 + q) * KP);
  double dot = 0.0;
  for (int c = c0; c < c1; ++c) {
    double r[NP];
#pragma unroll
    for (int n = 0; n < NP; ++n) {
      const unsigned so = (c * NP + n) * KP;
      r[n] = mad(a.a_next, ldr<double>(rb_r, kb, so), a.b_i * ldr<double>(yb, kb, so));
    }
    if (c == 0) {
#pragma unroll
      for (int n = 0; n < NP; ++n) {
        const unsigned so = n * KP;
        dot = mad(r[n], mad(-a.a_i, ldr<double>(rp, kb, so), ldr<double>(ri, kb, so)), dot);
      }
    }
    double dq[NP];
    wadg_inverse<double, N, NQ>(r, wq, dq);
    if (active) {
      const double sg = c == 0 ? 1.0 : -1.0;
#pragma unroll
      for (int n = 0; n < NP; ++n) {
        const unsigned so = (c * NP + n) * KP;
        st(rb_w, kb, so, r[n]);
        st(zw, kb, so, sg * dq[n]);
      }
    }
  }
  if (wave == 0) {
    if (!active) dot = 0.0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) dot += __shfl_xor(dot, off, 64);
    if (lane == 0) a.part[w] += dot;
  }
}

template <int N, int NQ>
int launch_nq(const AdjMass& a, void* stream) {
  hipLaunchKernelGGL((adjoint_mass_kernel<N, NQ>), dim3(a.nEG * a.S), dim3(2 * kWave), 0,
                     static_cast<hipStream_t>(stream), a);
  return (int)hipGetLastError();
}

template <int N>
int launch_n(int nq, const AdjMass& a, void* stream) {
  switch (nq - N) {
    case 1: return launch_nq<N, N + 1>(a, stream);
    case 2: return launch_nq<N, N + 2>(a, stream);
    case 3: return launch_nq<N, N + 3>(a, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace

int launch_adjoint_mass(int N, int nq, const StageParams& p, double* rbar, const double* ybar,
                        double* z, const double* r_i, const double* r_prev, double a_next,
                        double b_i, double a_i, double* part, void* stream) {
  AdjMass a{rbar, ybar, z, r_i, r_prev, static_cast<const double*>(p.vol), part,
            p.K, p.S, p.nEG, a_next, b_i, a_i, p.c2_scale};
  switch (N) {
    case 1: return launch_n<1>(nq, a, stream);
    case 2: return launch_n<2>(nq, a, stream);
    case 3: return launch_n<3>(nq, a, stream);
    case 4: return launch_n<4>(nq, a, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace wadg
