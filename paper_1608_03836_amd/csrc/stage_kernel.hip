// Fused WADG stage kernel for gfx950, streamed-geometry variant.
//
// One LSRK stage of the WADG acoustic sweep for S slices at once, or one
// right-hand-side evaluation, in arithmetic type R (double; float for the
// FP32-bulk propagator).  A workgroup owns one 64-element group of one
// slice and has two waves: lane l of wave 0 computes the pressure equation
// of element l, lane l of wave 1 the two velocity equations of the same
// element.  State and geometry are tiled by element group with the lane
// index fastest, so every per-node access of a wave is one contiguous
// 64-lane access at a compile-time offset inside the group's tile, and
// every reference-operator entry is wave-uniform: the 1D tables are
// compile-time constants folded into the instruction stream.
//
// This variant reads the geometry of its element group from global memory
// (L2-resident, shared by all slices) for every work item.  It serves every
// (N, nq) the library supports.  The split-work kernel (split_kernel.hip),
// which computes the same item over four waves, is the default; this one
// remains selectable, and the persistent batch kernel below uses its
// per-wave code.
//
// The group's input tile (3 (N+1)^2 x 64 values) is first copied into LDS
// with 16-byte coalesced loads; the waves then re-read their own nodal
// values from LDS (lane-contiguous, conflict-free).  Every global operand
// is requested one phase ahead of its use: the metric terms of volume
// column i+1 during column i, the first face's operands during the last
// volume column, face f+1's during face f, and the mass-inverse weights
// and the first residual during the last face; the neighbour offsets and
// volume column 0 are requested with the tile.  Per lane:
//
//   a1  own face nodes (LDS) and the neighbours' face nodes (gathered from
//       the input slice through precomputed offsets, flip-aware),
//       interpolated to the face Gauss points;
//   a2  volume term of the strong-weak form;
//   a3  penalised numerical flux and its lift;
//   a4  weight-adjusted mass inverse;
//   a5  the 2N-storage stage update res <- A res + dt dQ, Q <- Q + B res,
//       reading Q from one buffer and writing the other, so that neighbour
//       gathers never see a partly updated state.
//
// Workgroup -> (slice, element group): workgroups are dealt to the 8 XCDs
// round-robin; each XCD receives a contiguous range of a logical order made
// of tiles of Be element groups x Bs slices, slice-major inside a tile.  With
// all slices in one tile, an XCD keeps its element groups' geometry in its
// L2 for every slice, and the neighbouring groups of one slice (whose face
// values it gathers) are processed back to back.

#include <hip/hip_runtime.h>

#include "stage_common.h"

namespace wadg {
namespace {

using namespace dev;

// Buffer resources of one workgroup: the group's tiles of the state arrays
// and of the geometry, and the whole input slice for neighbour gathers.
struct Bufs {
  rsrc_t qin, qout, res, resw, qslice, vol, face, nbr;
};

// The NQ^2 weights of the weight-adjusted inverse (geometry plane `wplane`).
template <typename R, int NQ>
__device__ __forceinline__ void load_weights(const Bufs& B, unsigned wplane, unsigned kb,
                                             R (&w)[NQ * NQ]) {
  constexpr unsigned KP = kWave * sizeof(R);
#pragma unroll
  for (int q = 0; q < NQ * NQ; ++q) w[q] = ldr<R>(B.vol, kb, (wplane + q) * KP);
}

// Operands of one face: the neighbour's trace and the face geometry at the
// face Gauss points.
template <typename R, int N, int NQ>
struct FaceData {
  Trace<R, N> t;
  R g[3][NQ];   // nx, ny, w sJ
};

template <typename R, int N, int NQ>
__device__ __forceinline__ void load_face(const Bufs& B, const NbrOffsets& o, int f,
                                          unsigned kb, FaceData<R, N, NQ>& d) {
  constexpr unsigned KP = kWave * sizeof(R);
  gather_trace<R, N>(B.qslice, o, f, d.t);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < NQ; ++j) d.g[c][j] = ldr<R>(B.face, kb, (c * 4 * NQ + f * NQ + j) * KP);
}

// Metric planes 0..3 (W ys, -W xs, -W yr, W xr) of volume column i.
template <typename R, int NQ>
__device__ __forceinline__ void load_metric_column(const Bufs& B, int i, unsigned kb,
                                                   R (&g)[4][NQ]) {
  constexpr unsigned KP = kWave * sizeof(R);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int j = 0; j < NQ; ++j) g[p][j] = ldr<R>(B.vol, kb, (p * NQ * NQ + i + NQ * j) * KP);
}

// One wave's share of a work item: the pressure equation (wave 0) or the two
// velocity equations (wave 1).
template <typename R, int N, int NQ, int MODE, bool PRESSURE>
__device__ __forceinline__ void stage_wave(const StageScalars<R>& k, const Bufs& B, const R* tq,
                                           unsigned kb, int lane, bool active,
                                           const NbrOffsets& nbo, const R (&g0)[4][NQ]) {
  constexpr int NP1 = N + 1, NP = NP1 * NP1, NQ2 = NQ * NQ;
  auto P = [&](int n) { return tq[n * kWave + lane]; };
  auto U = [&](int n) { return tq[(NP + n) * kWave + lane]; };
  auto V = [&](int n) { return tq[(2 * NP + n) * kWave + lane]; };

  R b0[NP], b1[NP];   // pressure: b0; velocity: b0 = b_u, b1 = b_v
#pragma unroll
  for (int n = 0; n < NP; ++n) b0[n] = b1[n] = R(0);
  FaceData<R, N, NQ> fd[2];

  // a2, metric terms one column ahead
  R gc[4][NQ], gn[4][NQ];
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int j = 0; j < NQ; ++j) gc[g][j] = g0[g][j];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    if (i + 1 < NQ)
      load_metric_column<R, NQ>(B, i + 1, kb, gn);
    else
      load_face<R, N, NQ>(B, nbo, 0, kb, fd[0]);
    order();
    if constexpr (PRESSURE) {
      pressure_volume_column<R, N, NQ>(i, U, V, gc, b0);
      pin(b0);
    } else {
      velocity_volume_column<R, N, NQ>(i, P, gc, b0, b1);
      pin(b0);
      pin(b1);
    }
    if (i + 1 < NQ) {
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int j = 0; j < NQ; ++j) gc[g][j] = gn[g][j];
    }
  }

  // a1 + a3, face operands one face ahead
  R w[NQ2], resv[NP];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    if (f + 1 < 4) {
      load_face<R, N, NQ>(B, nbo, f + 1, kb, fd[(f + 1) & 1]);
    } else {
      if constexpr (MODE != kApplyA) load_weights<R, NQ>(B, (PRESSURE ? 4 : 5) * NQ2, kb, w);
      load_res<R, NP, MODE>(k, B.res, PRESSURE ? 0 : 1, kb, resv);
    }
    order();
    const FaceData<R, N, NQ>& d = fd[f & 1];
    if constexpr (PRESSURE) {
      pressure_face<R, N, NQ>(f, P, U, V, d.t, d.g, k.tau_p, b0);
      pin(b0);
    } else {
      velocity_face<R, N, NQ>(f, P, U, V, d.t, d.g, k.tau_u, b0, b1);
      pin(b0);
      pin(b1);
    }
  }

  // a4 + a5; the velocity wave reuses the weights (1/J) for both fields and
  // requests the second residual before the first field's stores.  The
  // pressure weights c^2/J carry the wave-speed scale.  Apply-A mode (the
  // transposed operator's outer factor) takes the load vector itself.
  order();
  if constexpr (PRESSURE && MODE != kApplyA) {
#pragma unroll
    for (int q = 0; q < NQ2; ++q) w[q] *= k.c2s;
  }
  R dq[NP];
  if constexpr (MODE == kApplyA) {
#pragma unroll
    for (int n = 0; n < NP; ++n) dq[n] = b0[n];
  } else {
    wadg_inverse<R, N, NQ>(b0, w, dq);
  }
  if constexpr (PRESSURE) {
    finish_field<R, NP, MODE>(k, B.qout, B.resw, P, 0, kb, active, resv, dq);
  } else {
    R resv2[NP];
    load_res<R, NP, MODE>(k, B.res, 2, kb, resv2);
    order();
    finish_field<R, NP, MODE>(k, B.qout, B.resw, P, 1, kb, active, resv, dq);
    order();
    if constexpr (MODE == kApplyA) {
#pragma unroll
      for (int n = 0; n < NP; ++n) dq[n] = b1[n];
    } else {
      wadg_inverse<R, N, NQ>(b1, w, dq);
    }
    finish_field<R, NP, MODE>(k, B.qout, B.resw, P, 2, kb, active, resv2, dq);
  }
}

}  // namespace

template <typename R, int N, int NQ, int MODE>
__global__ __launch_bounds__(2 * kWave) void stage_kernel(const StageParams p) {
  constexpr int NP = (N + 1) * (N + 1);
  constexpr int NQ2 = NQ * NQ;
  constexpr unsigned tile = 3u * NP * kWave;   // values per group tile
  constexpr unsigned KP = kWave * sizeof(R);
  __shared__ __attribute__((aligned(16))) R tq[tile];

  const int w = item_of(blockIdx.x, gridDim.x, p.reverse);
  // work item -> (slice, element group): tiles of Be element groups x Bs
  // slices, ordered (slice block, element block), slice-major inside a tile
  const int Be = p.tile_groups, Bs = p.tile_slices, nEG = p.nEG;
  const int sb = w / (Bs * nEG);
  const int r = w - sb * Bs * nEG;
  const int bs = min(Bs, p.S - sb * Bs);
  const int eb = r / (Be * bs);
  const int r2 = r - eb * Be * bs;
  const int be = min(Be, nEG - eb * Be);
  const int s = sb * Bs + r2 / be;
  const int eg = eb * Be + r2 % be;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & (kWave - 1);

  const R* Qin = static_cast<const R*>(p.Qin);
  const size_t slice = (size_t)s * p.nEG * tile;
  const size_t grp = slice + (size_t)eg * tile;
  Bufs B;
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

  // stage the input tile in LDS (16-byte chunks, consecutive threads on
  // consecutive chunks); the neighbour offsets and the metric terms of
  // volume column 0 are requested while the tile is in flight
  constexpr unsigned chunks = tile * sizeof(R) / 16;
  constexpr unsigned per_thread = (chunks + 2 * kWave - 1) / (2 * kWave);
  u32x4 v[per_thread];
#pragma unroll
  for (unsigned i = 0; i < per_thread; ++i) {
    const unsigned c = tid + i * 2 * kWave;
    if (c < chunks) v[i] = ld128(B.qin, c * 16u);
  }
  const unsigned kb = (unsigned)lane * sizeof(R);
  NbrOffsets nbo;
  load_nbr(B.nbr, lane, nbo);
  R g0[4][NQ];
  load_metric_column<R, NQ>(B, 0, kb, g0);
  order();
#pragma unroll
  for (unsigned i = 0; i < per_thread; ++i) {
    const unsigned c = tid + i * 2 * kWave;
    if (c < chunks) *reinterpret_cast<u32x4*>(reinterpret_cast<char*>(tq) + c * 16u) = v[i];
  }
  __syncthreads();

  const StageScalars<R> k = stage_scalars<R>(p);
  const bool active = eg * kWave + lane < p.K;
  if (wave == 0)
    stage_wave<R, N, NQ, MODE, true>(k, B, tq, kb, lane, active, nbo, g0);
  else
    stage_wave<R, N, NQ, MODE, false>(k, B, tq, kb, lane, active, nbo, g0);
}

// Batched LSRK stage over a work list of (problem, slice, element group)
// items of many independent problems: the same per-item work as
// stage_kernel, the problem's state offset, geometry groups and dt taken
// from its descriptor.  Persistent: workgroup w takes items w, w + grid, ...
// (w XCD-remapped, so each XCD sweeps a contiguous range of the list at
// every round); with grid = nitems it is one item per workgroup.
template <int N, int NQ>
__global__ __launch_bounds__(2 * kWave) void batch_stage_kernel(const BatchParams bp) {
  using R = double;
  constexpr int NP = (N + 1) * (N + 1);
  constexpr int NQ2 = NQ * NQ;
  constexpr unsigned tile = 3u * NP * kWave;
  constexpr unsigned KP = kWave * sizeof(R);
  constexpr unsigned chunks = tile * sizeof(R) / 16;
  constexpr unsigned per_thread = (chunks + 2 * kWave - 1) / (2 * kWave);
  __shared__ __attribute__((aligned(16))) R tq[tile];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & (kWave - 1);
  const unsigned kb = (unsigned)lane * sizeof(R);

  for (int it = xcd_remap(blockIdx.x, gridDim.x); it < bp.nitems; it += gridDim.x) {
    const int pi = bp.items[2 * it], local = bp.items[2 * it + 1];
    const BatchProb pr = bp.prob[pi];
    const int s = local / pr.nEG, eg = local - s * pr.nEG;
    const size_t slice = (size_t)pr.qoff + (size_t)s * pr.nEG * tile;
    const size_t grp = slice + (size_t)eg * tile;
    const size_t gg = (size_t)pr.g0 + eg;
    Bufs B;
    B.qin = make_rsrc(bp.Qin + grp, tile * sizeof(R));
    B.qout = make_rsrc(bp.Qout + grp, tile * sizeof(R));
    B.res = make_rsrc(bp.res + grp, tile * sizeof(R));
    B.resw = make_rsrc(bp.res + grp, bp.res_dead ? 0u : tile * sizeof(R));
    B.qslice = make_rsrc(bp.Qin + slice, (unsigned)pr.nEG * tile * sizeof(R));
    B.vol = make_rsrc(bp.vol + gg * 6 * NQ2 * kWave, 6u * NQ2 * KP);
    B.face = make_rsrc(bp.face + gg * 12 * NQ * kWave, 12u * NQ * KP);
    B.nbr = make_rsrc(bp.nbr + gg * 8 * kWave, 8u * kWave * 4u);

    u32x4 v[per_thread];
#pragma unroll
    for (unsigned i = 0; i < per_thread; ++i) {
      const unsigned c = tid + i * 2 * kWave;
      if (c < chunks) v[i] = ld128(B.qin, c * 16u);
    }
    NbrOffsets nbo;
    load_nbr(B.nbr, lane, nbo);
    R g0[4][NQ];
    load_metric_column<R, NQ>(B, 0, kb, g0);
    order();
#pragma unroll
    for (unsigned i = 0; i < per_thread; ++i) {
      const unsigned c = tid + i * 2 * kWave;
      if (c < chunks) *reinterpret_cast<u32x4*>(reinterpret_cast<char*>(tq) + c * 16u) = v[i];
    }
    __syncthreads();

    StageScalars<R> k;
    k.tau_p = bp.tau_p;
    k.tau_u = bp.tau_u;
    k.A = bp.rkA;
    k.B = bp.rkB;
    k.dt = pr.dt;
    k.c2s = 1.0;
    const bool active = eg * kWave + lane < pr.K;
    if (wave == 0)
      stage_wave<R, N, NQ, kStage, true>(k, B, tq, kb, lane, active, nbo, g0);
    else
      stage_wave<R, N, NQ, kStage, false>(k, B, tq, kb, lane, active, nbo, g0);
    __syncthreads();   // the tile is rewritten by the next item
  }
}

namespace {

template <int N, int NQ>
int launch_batch_nq(const BatchParams& p, int grid, void* stream) {
  hipLaunchKernelGGL((batch_stage_kernel<N, NQ>), dim3(grid), dim3(2 * kWave), 0,
                     static_cast<hipStream_t>(stream), p);
  return (int)hipGetLastError();
}

template <int N>
int launch_batch_n(int nq, const BatchParams& p, int grid, void* stream) {
  switch (nq - N) {
    case 1: return launch_batch_nq<N, N + 1>(p, grid, stream);
    case 2: return launch_batch_nq<N, N + 2>(p, grid, stream);
    case 3: return launch_batch_nq<N, N + 3>(p, grid, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

template <typename R, int N, int NQ>
int launch_nq(int mode, const StageParams& p, void* stream) {
  const dim3 grid(p.nEG * p.S), block(2 * kWave);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (mode == kStage) {
    hipLaunchKernelGGL((stage_kernel<R, N, NQ, kStage>), grid, block, 0, st, p);
  } else if constexpr (sizeof(R) == sizeof(double)) {
    if (mode == kRhs)
      hipLaunchKernelGGL((stage_kernel<R, N, NQ, kRhs>), grid, block, 0, st, p);
    else if (mode == kApplyA)
      hipLaunchKernelGGL((stage_kernel<R, N, NQ, kApplyA>), grid, block, 0, st, p);
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

}  // namespace

bool stage_supported(int N, int nq) { return N >= 1 && N <= 4 && nq >= N + 1 && nq <= N + 3; }

int launch_stage_streamed(int N, int nq, int mode, const StageParams& p, void* stream) {
  return launch_r<double>(N, nq, mode, p, stream);
}

int launch_stage_streamed_fp32(int N, int nq, const StageParams& p, void* stream) {
  return launch_r<float>(N, nq, kStage, p, stream);
}

int launch_batch_stage(int N, int nq, const BatchParams& p, int grid, void* stream) {
  if (p.nitems <= 0) return 0;
  switch (N) {
    case 1: return launch_batch_n<1>(nq, p, grid, stream);
    case 2: return launch_batch_n<2>(nq, p, grid, stream);
    case 3: return launch_batch_n<3>(nq, p, grid, stream);
    case 4: return launch_batch_n<4>(nq, p, grid, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace wadg
