// Fused WADG stage kernel for gfx950, split-work variant.
//
// The same stage (or right-hand side, or the adjoint's apply-A product) and
// the same arithmetic as the other stage kernels (stage_common.h), with one
// 64-element group of one slice spread over four waves instead of two, so
// that each wave carries about a quarter of the item and two workgroups
// share a CU (two waves per SIMD):
//
//   wave 0  pressure volume term (Section 4.1), then the pressure mass
//           inverse and update;
//   wave 1  velocity volume term, then the u mass inverse and update;
//   wave 2  traces, fluxes and lifts of faces 0 and 2 for all three fields
//           (Section 6.4: each face's traces interpolated once), then the
//           v mass inverse and update;
//   wave 3  the same for faces 1 and 3.
//
// The face waves leave each face's terms in LDS; the volume waves add them
// in face order 0..3 (as every stage kernel does) and wave 1 hands b_v to
// wave 2 through LDS.  Three workgroup barriers per item: the input tile,
// the face terms, b_v.
//
// Metric terms.  Both volume waves walk the NQ quadrature columns and need
// each column's four metric planes; a column of compute is shorter than a
// global load under full HBM load, so no register prefetch distance that
// fits hides them.  Instead everything the volume phase reads is requested
// with the tile: the first and last columns by each volume wave into its
// own registers, the NQ-2 middle columns by the face waves (which have
// registers to spare) into LDS, shared by both volume waves.  The staged
// columns are dead once the face-terms barrier has passed, and b_v reuses
// their space.
//
// Workgroup -> (slice, element group): the streamed kernel's XCD-aware tile
// order (wadg_set_schedule).

#include <hip/hip_runtime.h>

#include "stage_common.h"

namespace wadg {
namespace {

using namespace dev;

template <typename R, int N, int NQ>
struct Split {
  static constexpr int NP1 = N + 1, NP = NP1 * NP1, NQ2 = NQ * NQ;
  static constexpr unsigned tile = 3u * NP * kWave;        // input tile [3][NP][64]
  static constexpr unsigned xf = 4u * 3 * NP1 * kWave;     // face terms [4][3][NP1][64]
  static constexpr int NM = NQ - 2;                        // metric columns staged in LDS
  // staged metric columns [NM][4][NQ][64]; after the face-terms barrier
  // b_v and the residuals of fields 0 and 1, [3][NP][64]
  static constexpr unsigned xm =
      (unsigned)(NM * 4 * NQ > 3 * NP ? NM * 4 * NQ : 3 * NP) * kWave;
};

// Global geometry and state resources of one work item; the last five
// only in the fused apply-A + mass mode (rbar read and written, z, r_i,
// r_{i-1}).
struct SplitBufs {
  rsrc_t qin, qout, res, resw, qslice, vol, face, nbr;
  rsrc_t rbr, rbw, zo, ri, rp;
};

template <typename R, int NQ>
__device__ __forceinline__ void split_metric_column(const SplitBufs& B, int i, unsigned kb,
                                                    R (&g)[4][NQ]) {
  constexpr unsigned KP = kWave * sizeof(R);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int j = 0; j < NQ; ++j) g[p][j] = ldr<R>(B.vol, kb, (p * NQ * NQ + i + NQ * j) * KP);
}

template <typename R, int NQ>
__device__ __forceinline__ void split_weights(const SplitBufs& B, unsigned wplane, unsigned kb,
                                              R (&w)[NQ * NQ]) {
  constexpr unsigned KP = kWave * sizeof(R);
#pragma unroll
  for (int q = 0; q < NQ * NQ; ++q) w[q] = ldr<R>(B.vol, kb, (wplane + q) * KP);
}

// Volume waves: the volume term of field group PRESSURE (b0 = b_p) or the
// velocity (b0 = b_u, b1 = b_v).  Metric column 0 arrives in ga, column
// NQ-1 in gb (both requested with the tile), the middle columns from the
// LDS stage xm; ga is reused for them once column 0 is done.  The mass
// weights of the wave's field (plane wplane) are requested before the last
// column, when ga is free again.
template <typename R, int N, int NQ, bool PRESSURE, bool WEIGHTS, typename FP, typename FU,
          typename FV>
__device__ __forceinline__ void split_volume(const SplitBufs& B, unsigned kb, unsigned wplane,
                                             const R* xm, int lane, const FP& P, const FU& U,
                                             const FV& V, R (&ga)[4][NQ], const R (&gb)[4][NQ],
                                             R (&b0)[(N + 1) * (N + 1)],
                                             R (&b1)[(N + 1) * (N + 1)], R (&w)[NQ * NQ]) {
  constexpr int NP = (N + 1) * (N + 1);
#pragma unroll
  for (int n = 0; n < NP; ++n) b0[n] = b1[n] = R(0);
  auto column = [&](int i, const R(&g)[4][NQ]) {
    if constexpr (PRESSURE) {
      pressure_volume_column<R, N, NQ>(i, U, V, g, b0);
      pin(b0);
    } else {
      velocity_volume_column<R, N, NQ>(i, P, g, b0, b1);
      pin(b0);
      pin(b1);
    }
  };
  column(0, ga);
#pragma unroll
  for (int i = 1; i + 1 < NQ; ++i) {
    order();
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int j = 0; j < NQ; ++j) ga[q][j] = xm[(((i - 1) * 4 + q) * NQ + j) * kWave + lane];
    column(i, ga);
  }
  order();
  if constexpr (WEIGHTS) split_weights<R, NQ>(B, wplane, kb, w);
  order();
  column(NQ - 1, gb);
}

// Face waves: request metric planes Q0 and Q0+1 of the middle columns
// (with the tile), and store them into the LDS stage once they arrive.
template <typename R, int NQ, int Q0>
struct MetricStage {
  static constexpr int NM = NQ - 2 > 0 ? NQ - 2 : 1;
  R v[NM][2][NQ];

  __device__ __forceinline__ void load(const SplitBufs& B, unsigned kb) {
    constexpr unsigned KP = kWave * sizeof(R);
#pragma unroll
    for (int c = 0; c + 2 < NQ; ++c)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int j = 0; j < NQ; ++j)
          v[c][q][j] = ldr<R>(B.vol, kb, ((Q0 + q) * NQ * NQ + c + 1 + NQ * j) * KP);
  }
  __device__ __forceinline__ void store(R* xm, int lane) const {
#pragma unroll
    for (int c = 0; c + 2 < NQ; ++c)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int j = 0; j < NQ; ++j) xm[((c * 4 + Q0 + q) * NQ + j) * kWave + lane] = v[c][q][j];
  }
};

// Face waves: the terms of faces FA and FB for all three fields, into LDS.
template <typename R, int N, int NQ, int FA, int FB, typename FP, typename FU, typename FV>
__device__ __forceinline__ void split_faces(const StageScalars<R>& k, const SplitBufs& B,
                                            unsigned kb, int lane, const FP& P, const FU& U,
                                            const FV& V, R* xf) {
  constexpr int NP1 = N + 1;
  constexpr unsigned KP = kWave * sizeof(R);
  NbrOffsets nbo;
  load_nbr(B.nbr, lane, nbo);
  Trace<R, N> tr[2];
  R g[2][3][NQ];
  gather_trace<R, N>(B.qslice, nbo, FA, tr[0]);
  gather_trace<R, N>(B.qslice, nbo, FB, tr[1]);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      g[0][c][j] = ldr<R>(B.face, kb, (c * 4 * NQ + FA * NQ + j) * KP);
      g[1][c][j] = ldr<R>(B.face, kb, (c * 4 * NQ + FB * NQ + j) * KP);
    }
  order();
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int f = q == 0 ? FA : FB;
    R sp[NP1], su[NP1], sv[NP1];
    face_terms<R, N, NQ, true, true>(f, P, U, V, tr[q], g[q], k.tau_p, k.tau_u, sp, su, sv);
#pragma unroll
    for (int m = 0; m < NP1; ++m) {
      xf[((f * 3 + 0) * NP1 + m) * kWave + lane] = sp[m];
      xf[((f * 3 + 1) * NP1 + m) * kWave + lane] = su[m];
      xf[((f * 3 + 2) * NP1 + m) * kWave + lane] = sv[m];
    }
  }
}

// Add the four faces' terms of field c to b, in face order.
template <typename R, int N>
__device__ __forceinline__ void add_face_terms(const R* xf, int c, int lane,
                                               R (&b)[(N + 1) * (N + 1)]) {
  constexpr int NP1 = N + 1;
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int m = 0; m < NP1; ++m) b[fnode<N>(f, m)] += xf[((f * 3 + c) * NP1 + m) * kWave + lane];
}

// Fused apply-A + mass mode, field c: the apply-A update of ybar (as
// finish_field), then the next reverse stage's mass step on the new ybar,
// in the adjoint mass kernel's order of operations.  w: the field's mass
// weights (c2_scale c^2/J for p, 1/J for u, v).  Returns the pressure
// sensitivity partial of this lane (0 for u, v).
template <int N, int NQ>
__device__ __forceinline__ double apply_a_mass_field(const StageScalars<double>& k,
                                                     const SplitBufs& B, const AdjMassParams& am,
                                                     int c, unsigned kb, bool active,
                                                     const double (&resv)[(N + 1) * (N + 1)],
                                                     const double (&b)[(N + 1) * (N + 1)],
                                                     const double (&w)[NQ * NQ]) {
  constexpr int NP = (N + 1) * (N + 1);
  constexpr unsigned KP = kWave * sizeof(double);
  const double sdt = c == 0 ? k.dt : -k.dt;
  double y[NP], r[NP], dq[NP];
#pragma unroll
  for (int n = 0; n < NP; ++n) y[n] = mad(sdt, b[n], resv[n]);
  if (active) {
#pragma unroll
    for (int n = 0; n < NP; ++n) st(B.qout, kb, (c * NP + n) * KP, y[n]);
  }
#pragma unroll
  for (int n = 0; n < NP; ++n)
    r[n] = mad(am.a_next, ldr<double>(B.rbr, kb, (c * NP + n) * KP), am.b * y[n]);
  double dot = 0.0;
  if (c == 0) {
#pragma unroll
    for (int n = 0; n < NP; ++n)
      dot = mad(r[n], mad(-am.a, ldr<double>(B.rp, kb, n * KP), ldr<double>(B.ri, kb, n * KP)),
                dot);
  }
  wadg_inverse<double, N, NQ>(r, w, dq);
  if (active) {
    const double sg = c == 0 ? 1.0 : -1.0;
#pragma unroll
    for (int n = 0; n < NP; ++n) {
      const unsigned so = (c * NP + n) * KP;
      st(B.rbw, kb, so, r[n]);
      st(B.zo, kb, so, sg * dq[n]);
    }
  }
  return dot;
}

}  // namespace

// One work item -- a 64-element group of one slice -- over the four waves of
// the workgroup.  B: the item's resources; k: the stage's scalars; active:
// this lane holds an element; tq, xf, xm: the workgroup's LDS (Split<>);
// am, part: the fused apply-A + mass mode's scalars and this item's slot in
// am.part.
template <typename R, int N, int NQ, int MODE>
__device__ __forceinline__ void split_item(const SplitBufs& B, const StageScalars<R>& k,
                                           bool active, R* tq, R* xf, R* xm,
                                           const AdjMassParams& am = AdjMassParams{},
                                           int part = 0) {
  using L = Split<R, N, NQ>;
  constexpr int NP = L::NP, NQ2 = L::NQ2;
  constexpr unsigned tile = L::tile;
  R* const xv = xm;                         // b_v, once the staged metric
  R* const xr = xm + (size_t)L::NP * kWave;  // columns are dead; residuals 0, 1
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & (kWave - 1);
  const unsigned kb = (unsigned)lane * sizeof(R);
  // Apply-A modes (the adjoint's outer factor) take the load vector itself:
  // no mass inverse; the fused apply-A + mass mode still needs the weights.
  constexpr bool kInv = MODE != kApplyA && MODE != kApplyAMass;
  constexpr bool kW = MODE != kApplyA;
  auto inverse = [](const R(&b)[NP], const R(&w)[NQ2], R(&dq)[NP]) {
    if constexpr (kInv) {
      wadg_inverse<R, N, NQ>(b, w, dq);
    } else {
#pragma unroll
      for (int n = 0; n < NP; ++n) dq[n] = b[n];
    }
  };

  // The input tile into LDS, 16-byte chunks over all four waves, and with
  // it the volume phase's metric terms: columns 0 and NQ-1 into the volume
  // waves' registers, the middle columns into LDS through the face waves.
  // Each role runs its own copy of this prologue (the branch is
  // wave-uniform), so that the registers of one role's loads are not held
  // live across the other's.
  constexpr unsigned chunks = tile * sizeof(R) / 16;
  constexpr unsigned per_thread = (chunks + 4 * kWave - 1) / (4 * kWave);
  auto tile_copy = [&](auto&& more_loads, auto&& more_stores) {
    u32x4 v[per_thread];
#pragma unroll
    for (unsigned i = 0; i < per_thread; ++i) {
      const unsigned c = tid + i * 4 * kWave;
      if (c < chunks) v[i] = ld128(B.qin, c * 16u);
    }
    more_loads();
#pragma unroll
    for (unsigned i = 0; i < per_thread; ++i) {
      const unsigned c = tid + i * 4 * kWave;
      if (c < chunks) *reinterpret_cast<u32x4*>(reinterpret_cast<char*>(tq) + c * 16u) = v[i];
    }
    more_stores();
    __syncthreads();                                   // tile in LDS
  };

  auto P = [&](int n) { return tq[n * kWave + lane]; };
  auto U = [&](int n) { return tq[(NP + n) * kWave + lane]; };
  auto V = [&](int n) { return tq[(2 * NP + n) * kWave + lane]; };

  if (wave <= 1) {
    R ga[4][NQ], gb[4][NQ];
    tile_copy(
        [&] {
          split_metric_column<R, NQ>(B, 0, kb, ga);
          split_metric_column<R, NQ>(B, NQ - 1, kb, gb);
        },
        [] {});
    R b0[NP], b1[NP], w[NQ2];
    if (wave == 0)
      split_volume<R, N, NQ, true, kW>(B, kb, 4 * NQ2, xm, lane, P, U, V, ga, gb, b0, b1, w);
    else
      split_volume<R, N, NQ, false, kW>(B, kb, 5 * NQ2, xm, lane, P, U, V, ga, gb, b0, b1, w);
    __syncthreads();                                   // face terms ready
    R resv[NP], dq[NP];
    if (wave == 0) {
      add_face_terms<R, N>(xf, 0, lane, b0);
      __syncthreads();                                 // b_v, residuals handed over
#pragma unroll
      for (int n = 0; n < NP; ++n) resv[n] = xr[n * kWave + lane];
      if constexpr (kW) {
#pragma unroll
        for (int q = 0; q < NQ2; ++q) w[q] *= k.c2s;
      }
      inverse(b0, w, dq);
      if constexpr (MODE == kApplyAMass) {
        double dot = apply_a_mass_field<N, NQ>(k, B, am, 0, kb, active, resv, dq, w);
        if (!active) dot = 0.0;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) dot += __shfl_xor(dot, off, 64);
        if (lane == 0) am.part[part] += dot;
      } else {
        finish_field<R, NP, MODE>(k, B.qout, B.resw, P, 0, kb, active, resv, dq);
      }
    } else {
      add_face_terms<R, N>(xf, 1, lane, b0);
      add_face_terms<R, N>(xf, 2, lane, b1);
#pragma unroll
      for (int n = 0; n < NP; ++n) xv[n * kWave + lane] = b1[n];
      __syncthreads();                                 // b_v, residuals handed over
#pragma unroll
      for (int n = 0; n < NP; ++n) resv[n] = xr[(NP + n) * kWave + lane];
      inverse(b0, w, dq);
      if constexpr (MODE == kApplyAMass)
        (void)apply_a_mass_field<N, NQ>(k, B, am, 1, kb, active, resv, dq, w);
      else
        finish_field<R, NP, MODE>(k, B.qout, B.resw, P, 1, kb, active, resv, dq);
    }
  } else {
    if (wave == 2) {
      MetricStage<R, NQ, 0> m;
      tile_copy([&] { m.load(B, kb); }, [&] { m.store(xm, lane); });
    } else {
      MetricStage<R, NQ, 2> m;
      tile_copy([&] { m.load(B, kb); }, [&] { m.store(xm, lane); });
    }
    if (wave == 2)
      split_faces<R, N, NQ, 0, 2>(k, B, kb, lane, P, U, V, xf);
    else
      split_faces<R, N, NQ, 1, 3>(k, B, kb, lane, P, U, V, xf);
    if (wave == 2) {
      R w[NQ2], resv[NP];
      if constexpr (kW) split_weights<R, NQ>(B, 5 * NQ2, kb, w);
      load_res<R, NP, MODE>(k, B.res, 2, kb, resv);
      __syncthreads();                                 // face terms ready
      __syncthreads();                                 // b_v handed over
      R bv[NP], dq[NP];
#pragma unroll
      for (int n = 0; n < NP; ++n) bv[n] = xv[n * kWave + lane];
      inverse(bv, w, dq);
      if constexpr (MODE == kApplyAMass)
        (void)apply_a_mass_field<N, NQ>(k, B, am, 2, kb, active, resv, dq, w);
      else
        finish_field<R, NP, MODE>(k, B.qout, B.resw, P, 2, kb, active, resv, dq);
    } else {
      // the residuals of fields 0 and 1, requested for the volume waves
      // while they finish their volume terms
      R r0[NP], r1[NP];
      load_res<R, NP, MODE>(k, B.res, 0, kb, r0);
      load_res<R, NP, MODE>(k, B.res, 1, kb, r1);
      __syncthreads();                                 // face terms ready
#pragma unroll
      for (int n = 0; n < NP; ++n) {
        xr[n * kWave + lane] = r0[n];
        xr[(NP + n) * kWave + lane] = r1[n];
      }
      __syncthreads();                                 // residuals handed over
    }
  }
}

// Workgroup bid of a launch of nb workgroups: its work item of launch p
// (slice, element group) in the launch's order, run over the workgroup's
// LDS arrays (Split<>).
template <typename R, int N, int NQ, int MODE>
__device__ __forceinline__ void split_run(const StageParams& p, int bid, int nb, R* tq, R* xf,
                                          R* xm) {
  static_assert((MODE != kApplyA && MODE != kApplyAMass) || sizeof(R) == sizeof(double),
                "apply-A modes are FP64 only");
  using L = Split<R, N, NQ>;
  constexpr int NQ2 = L::NQ2;
  constexpr unsigned tile = L::tile;
  constexpr unsigned KP = kWave * sizeof(R);

  const int w = item_of(bid, nb, p.reverse);
  const int Be = p.tile_groups, Bs = p.tile_slices, nEG = p.nEG;
  const int sb = w / (Bs * nEG);
  const int r = w - sb * Bs * nEG;
  const int bs = min(Bs, p.S - sb * Bs);
  const int eb = r / (Be * bs);
  const int r2 = r - eb * Be * bs;
  const int be = min(Be, nEG - eb * Be);
  const int s = sb * Bs + r2 / be;
  const int eg = eb * Be + r2 % be;
  const int lane = threadIdx.x & (kWave - 1);

  const R* Qin = static_cast<const R*>(p.Qin);
  const size_t slice = (size_t)s * p.nEG * tile;
  const size_t grp = slice + (size_t)eg * tile;
  SplitBufs B;
  B.qin = make_rsrc(Qin + grp, tile * sizeof(R));
  B.qout = make_rsrc(static_cast<R*>(p.Qout) + grp, tile * sizeof(R));
  B.res = make_rsrc(static_cast<R*>(MODE == kRhs ? p.Qout : p.res) + grp, tile * sizeof(R));
  B.resw = make_rsrc(static_cast<R*>(p.res_out ? p.res_out : p.res) + grp,
                     MODE == kStage && !p.res_dead ? tile * sizeof(R) : 0u);
  B.qslice = make_rsrc(Qin + slice, (unsigned)p.nEG * tile * sizeof(R));
  B.vol = make_rsrc(static_cast<const R*>(p.vol) + (size_t)eg * 6 * NQ2 * kWave, 6u * NQ2 * KP);
  B.face = make_rsrc(static_cast<const R*>(p.face) + (size_t)eg * 12 * NQ * kWave,
                     12u * NQ * KP);
  B.nbr = make_rsrc(p.nbr + (size_t)eg * 8 * kWave, 8u * kWave * 4u);
  if constexpr (MODE == kApplyAMass) {
    const AdjMassParams& am = p.adj;
    const unsigned tb = tile * sizeof(R);
    B.rbr = make_rsrc(am.rbar + grp, am.a_next != 0.0 ? tb : 0u);
    B.rbw = make_rsrc(am.rbar + grp, tb);
    B.zo = make_rsrc(am.z + grp, tb);
    B.ri = make_rsrc(am.r + grp, tb);
    B.rp = make_rsrc(am.r_prev ? am.r_prev + grp : am.r + grp,
                     (am.a != 0.0 && am.r_prev) ? tb : 0u);
  }
  split_item<R, N, NQ, MODE>(B, stage_scalars<R>(p), eg * kWave + lane < p.K, tq, xf, xm, p.adj,
                             s * nEG + eg);
}

template <typename R, int N, int NQ, int MODE>
__global__ __launch_bounds__(4 * kWave) void split_kernel(const StageParams p) {
  using L = Split<R, N, NQ>;
  __shared__ __attribute__((aligned(16))) R tq[L::tile];
  __shared__ __attribute__((aligned(16))) R xf[L::xf];
  __shared__ __attribute__((aligned(16))) R xm[L::xm];
  split_run<R, N, NQ, MODE>(p, blockIdx.x, gridDim.x, tq, xf, xm);
}

// Two independent launches in one grid (FP64): the first na workgroups run
// the items of launch a in mode MA (an apply-A mode), the others the LSRK
// stage items of launch b.  The adjoint's reverse sweep pairs each
// transposed stage of one slice with a recompute stage of the slice before
// it, so that the two one-slice launches share the CUs (two workgroups per
// CU) instead of following each other.  Each item computes exactly what it
// computes in its own launch.
template <int N, int NQ, int MA>
__global__ __launch_bounds__(4 * kWave) void split_pair_kernel(const StageParams a,
                                                               const StageParams b, int na) {
  using L = Split<double, N, NQ>;
  __shared__ __attribute__((aligned(16))) double tq[L::tile];
  __shared__ __attribute__((aligned(16))) double xf[L::xf];
  __shared__ __attribute__((aligned(16))) double xm[L::xm];
  if ((int)blockIdx.x < na)
    split_run<double, N, NQ, MA>(a, blockIdx.x, na, tq, xf, xm);
  else
    split_run<double, N, NQ, kStage>(b, blockIdx.x - na, gridDim.x - na, tq, xf, xm);
}

// Batched LSRK stage (FP64) over a work list of (problem, slice, element
// group) items of many independent problems: the split-work item above, the
// problem's state offset, geometry groups and dt taken from its descriptor.
// One workgroup per item (grid = nitems), XCD-remapped.  Not persistent: a
// loop over items keeps the kernel's operator constants live across
// iterations and spills scalar registers; the persistent batch kernel is the
// streamed one (stage_kernel.hip).
template <int N, int NQ>
__global__ __launch_bounds__(4 * kWave) void batch_split_kernel(const BatchParams bp) {
  using R = double;
  using L = Split<R, N, NQ>;
  constexpr int NQ2 = L::NQ2;
  constexpr unsigned tile = L::tile;
  constexpr unsigned KP = kWave * sizeof(R);
  __shared__ __attribute__((aligned(16))) R tq[tile];
  __shared__ __attribute__((aligned(16))) R xf[L::xf];
  __shared__ __attribute__((aligned(16))) R xm[L::xm];
  const int lane = threadIdx.x & (kWave - 1);

  {
    const int it = xcd_remap(blockIdx.x, gridDim.x);
    if (it >= bp.nitems) return;
    const int pi = bp.items[2 * it], local = bp.items[2 * it + 1];
    const BatchProb pr = bp.prob[pi];
    const int s = local / pr.nEG, eg = local - s * pr.nEG;
    const size_t slice = (size_t)pr.qoff + (size_t)s * pr.nEG * tile;
    const size_t grp = slice + (size_t)eg * tile;
    const size_t gg = (size_t)pr.g0 + eg;
    SplitBufs B;
    B.qin = make_rsrc(bp.Qin + grp, tile * sizeof(R));
    B.qout = make_rsrc(bp.Qout + grp, tile * sizeof(R));
    B.res = make_rsrc(bp.res + grp, tile * sizeof(R));
    B.resw = make_rsrc(bp.res + grp, bp.res_dead ? 0u : tile * sizeof(R));
    B.qslice = make_rsrc(bp.Qin + slice, (unsigned)pr.nEG * tile * sizeof(R));
    B.vol = make_rsrc(bp.vol + gg * 6 * NQ2 * kWave, 6u * NQ2 * KP);
    B.face = make_rsrc(bp.face + gg * 12 * NQ * kWave, 12u * NQ * KP);
    B.nbr = make_rsrc(bp.nbr + gg * 8 * kWave, 8u * kWave * 4u);
    StageScalars<R> k;
    k.tau_p = bp.tau_p;
    k.tau_u = bp.tau_u;
    k.A = bp.rkA;
    k.B = bp.rkB;
    k.dt = pr.dt;
    k.c2s = 1.0;
    split_item<R, N, NQ, kStage>(B, k, eg * kWave + lane < pr.K, tq, xf, xm);
  }
}

namespace {

template <typename R, int N, int NQ>
int launch_nq(int mode, const StageParams& p, void* stream) {
  const dim3 grid(p.nEG * p.S), block(4 * kWave);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (mode == kStage) {
    hipLaunchKernelGGL((split_kernel<R, N, NQ, kStage>), grid, block, 0, st, p);
  } else if constexpr (sizeof(R) == sizeof(double)) {
    if (mode == kRhs)
      hipLaunchKernelGGL((split_kernel<R, N, NQ, kRhs>), grid, block, 0, st, p);
    else if (mode == kApplyA)
      hipLaunchKernelGGL((split_kernel<R, N, NQ, kApplyA>), grid, block, 0, st, p);
    else if (mode == kApplyAMass)
      hipLaunchKernelGGL((split_kernel<R, N, NQ, kApplyAMass>), grid, block, 0, st, p);
    else
      return (int)hipErrorInvalidValue;
  } else {
    return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

template <typename R, int N>
int launch_n(int nq, int mode, const StageParams& p, void* stream) {
  switch (nq - N) {
    case 1: return launch_nq<R, N, N + 1>(mode, p, stream);
    case 2: return launch_nq<R, N, N + 2>(mode, p, stream);
    case 3: return launch_nq<R, N, N + 3>(mode, p, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

template <typename R>
int launch_r(int N, int nq, int mode, const StageParams& p, void* stream) {
  switch (N) {
    case 1: return launch_n<R, 1>(nq, mode, p, stream);
    case 2: return launch_n<R, 2>(nq, mode, p, stream);
    case 3: return launch_n<R, 3>(nq, mode, p, stream);
    case 4: return launch_n<R, 4>(nq, mode, p, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

template <int N, int NQ>
int launch_pair_nq(int mode_a, const StageParams& a, const StageParams& b, void* stream) {
  const int na = a.nEG * a.S, nb = b.nEG * b.S;
  const dim3 grid(na + nb), block(4 * kWave);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (mode_a == kApplyAMass)
    hipLaunchKernelGGL((split_pair_kernel<N, NQ, kApplyAMass>), grid, block, 0, st, a, b, na);
  else if (mode_a == kApplyA)
    hipLaunchKernelGGL((split_pair_kernel<N, NQ, kApplyA>), grid, block, 0, st, a, b, na);
  else
    return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

template <int N>
int launch_pair_n(int nq, int mode_a, const StageParams& a, const StageParams& b,
                  void* stream) {
  switch (nq - N) {
    case 1: return launch_pair_nq<N, N + 1>(mode_a, a, b, stream);
    case 2: return launch_pair_nq<N, N + 2>(mode_a, a, b, stream);
    case 3: return launch_pair_nq<N, N + 3>(mode_a, a, b, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

template <int N, int NQ>
int launch_batch_nq(const BatchParams& p, void* stream) {
  hipLaunchKernelGGL((batch_split_kernel<N, NQ>), dim3(p.nitems), dim3(4 * kWave), 0,
                     static_cast<hipStream_t>(stream), p);
  return (int)hipGetLastError();
}

template <int N>
int launch_batch_n(int nq, const BatchParams& p, void* stream) {
  switch (nq - N) {
    case 1: return launch_batch_nq<N, N + 1>(p, stream);
    case 2: return launch_batch_nq<N, N + 2>(p, stream);
    case 3: return launch_batch_nq<N, N + 3>(p, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace

int launch_batch_split(int N, int nq, const BatchParams& p, void* stream) {
  if (p.nitems <= 0) return 0;
  switch (N) {
    case 1: return launch_batch_n<1>(nq, p, stream);
    case 2: return launch_batch_n<2>(nq, p, stream);
    case 3: return launch_batch_n<3>(nq, p, stream);
    case 4: return launch_batch_n<4>(nq, p, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_stage_pair(int N, int nq, int mode_a, const StageParams& a, const StageParams& b,
                      void* stream) {
  if ((int64_t)a.nEG * a.S + (int64_t)b.nEG * b.S >= (1LL << 31)) return (int)hipErrorInvalidValue;
  switch (N) {
    case 1: return launch_pair_n<1>(nq, mode_a, a, b, stream);
    case 2: return launch_pair_n<2>(nq, mode_a, a, b, stream);
    case 3: return launch_pair_n<3>(nq, mode_a, a, b, stream);
    case 4: return launch_pair_n<4>(nq, mode_a, a, b, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_stage_split(int N, int nq, int mode, const StageParams& p, void* stream) {
  return launch_r<double>(N, nq, mode, p, stream);
}

int launch_stage_split_fp32(int N, int nq, const StageParams& p, void* stream) {
  return launch_r<float>(N, nq, kStage, p, stream);
}

}  // namespace wadg
