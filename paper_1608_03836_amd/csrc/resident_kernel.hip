// Fused WADG stage kernel for gfx950, LDS-resident-geometry variant.
//
// Same stage (or right-hand side) and the same arithmetic as the streamed
// kernel (stage_common.h), organised for CDNA4's 160 KiB of LDS per CU:
//
// * A workgroup of four waves owns one 64-element group and a contiguous
//   range of slices.  It copies the group's geometry -- metric terms, mass
//   weights and face factors, the bulk of the per-element data -- into LDS
//   once, and keeps it there for every slice of its range, instead of
//   re-reading it from L2 for each (slice, group) work item.
// * The four waves form two pairs (pressure wave, velocity wave); pair q
//   takes slices s0 + q, s0 + 2 + q, ...  Each pair has its own state tile
//   in LDS.  Lane l of a pressure wave computes the pressure equation of
//   element l, lane l of a velocity wave the two velocity equations.
// * Per work item each wave issues all of its global reads up front (the
//   neighbours' traces of the four faces and the residual), then computes
//   from LDS and registers.  The pressure wave also fetches the next
//   slice's tile of its pair into registers, after this item's other reads
//   so that their waits leave it in flight; after the whole workgroup is
//   done with the current tiles it writes it into LDS.
// * The LDS allocation admits one workgroup per CU, i.e. one wave per SIMD
//   with the whole register file (up to 512 registers per lane) for
//   operands in flight.
//
// Workgroup -> (element group, slice range): XCD-aware (contiguous logical
// ranges per XCD), element group major, so an XCD's workgroups process
// neighbouring element groups of the same slices at the same time and the
// neighbour gathers hit in its L2.

#include <hip/hip_runtime.h>

#include "stage_common.h"

namespace wadg {
namespace {

using namespace dev;

constexpr unsigned kLdsBytes = 160u * 1024u;
constexpr int kResidentWaves = 4;

template <typename R, int N, int NQ>
struct Resident {
  static constexpr int NP = (N + 1) * (N + 1), NQ2 = NQ * NQ;
  static constexpr unsigned vol = 6u * NQ2 * kWave;    // values: [6][NQ2][64]
  static constexpr unsigned face = 12u * NQ * kWave;   // [3][4][NQ][64]
  static constexpr unsigned tile = 3u * NP * kWave;    // [3][NP][64]
  static constexpr unsigned values = vol + face + 2u * tile;
  static constexpr bool fits = values * sizeof(R) <= kLdsBytes;
  static constexpr unsigned tile_chunks = tile * sizeof(R) / 16;     // 16-byte chunks
  static constexpr unsigned pre = (tile_chunks + kWave - 1) / kWave;  // per lane of one wave
};

// Field c of a tile (NP values), read without a branch: the residual
// resource is empty (reads return zero) in the first LSRK stage, whose
// residual buffer may hold anything.  Zeros in right-hand-side mode.
template <typename R, int NP, int MODE>
__device__ __forceinline__ void load_field(rsrc_t r, int c, unsigned kb, R (&v)[NP]) {
  constexpr unsigned KP = kWave * sizeof(R);
#pragma unroll
  for (int n = 0; n < NP; ++n) v[n] = MODE == kRhs ? R(0) : ldr<R>(r, kb, (c * NP + n) * KP);
}

// One work item of a pressure (PRESSURE) or velocity wave.  `tq` is the
// pair's tile, `gv`/`gf` the resident geometry, `qs` the input slice, `qo`
// this group's output tile, `rr`/`rw` its residual tile for reading (empty
// in the first LSRK stage) and for writing; `qn` the next tile of the pair
// (empty resource when there is none), fetched into `pre` by the pressure
// wave.
template <typename R, int N, int NQ, int MODE, bool PRESSURE>
__device__ __forceinline__ void resident_item(const StageScalars<R>& k, rsrc_t qs, rsrc_t qo,
                                              rsrc_t rr, rsrc_t rw, rsrc_t qn, const R* tq,
                                              const R* gv,
                                              const R* gf, const NbrOffsets& nbo, int lane,
                                              bool active,
                                              u32x4 (&pre)[Resident<R, N, NQ>::pre]) {
  using L = Resident<R, N, NQ>;
  constexpr int NP = L::NP, NQ2 = L::NQ2;
  const unsigned kb = (unsigned)lane * sizeof(R);
  auto P = [&](int n) { return tq[n * kWave + lane]; };
  auto U = [&](int n) { return tq[(NP + n) * kWave + lane]; };
  auto V = [&](int n) { return tq[(2 * NP + n) * kWave + lane]; };
  auto G = [&](int plane) { return gv[plane * kWave + lane]; };

  // global operands of this item
  Trace<R, N> tr[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) gather_trace<R, N>(qs, nbo, f, tr[f]);
  R res0[NP];
  load_field<R, NP, MODE>(rr, PRESSURE ? 0 : 1, kb, res0);
  order();

  // a2
  R b0[NP], b1[NP];   // pressure: b0; velocity: b0 = b_u, b1 = b_v
#pragma unroll
  for (int n = 0; n < NP; ++n) b0[n] = b1[n] = R(0);
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    R g[4][NQ];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < NQ; ++j) g[c][j] = G(c * NQ2 + i + NQ * j);
    if constexpr (PRESSURE) {
      pressure_volume_column<R, N, NQ>(i, U, V, g, b0);
      pin(b0);
    } else {
      velocity_volume_column<R, N, NQ>(i, P, g, b0, b1);
      pin(b0);
      pin(b1);
    }
  }
  order();

  // next tile of the pair (pressure wave) / second residual (velocity wave)
  R res1[NP];
  if constexpr (PRESSURE) {
#pragma unroll
    for (unsigned c = 0; c < L::pre; ++c) pre[c] = ld128(qn, (c * kWave + lane) * 16u);
  } else {
    load_field<R, NP, MODE>(rr, 2, kb, res1);
  }
  order();

  // a1 + a3
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    R g[3][NQ];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int j = 0; j < NQ; ++j) g[c][j] = gf[(c * 4 * NQ + f * NQ + j) * kWave + lane];
    if constexpr (PRESSURE) {
      pressure_face<R, N, NQ>(f, P, U, V, tr[f], g, k.tau_p, b0);
      pin(b0);
    } else {
      velocity_face<R, N, NQ>(f, P, U, V, tr[f], g, k.tau_u, b0, b1);
      pin(b0);
      pin(b1);
    }
  }

  // a4 + a5
  R w[NQ2];
#pragma unroll
  for (int q = 0; q < NQ2; ++q)
    w[q] = PRESSURE ? k.c2s * G(4 * NQ2 + q) : G(5 * NQ2 + q);
  R dq[NP];
  wadg_inverse<R, N, NQ>(b0, w, dq);
  if constexpr (PRESSURE) {
    finish_field<R, NP, MODE>(k, qo, rw, P, 0, kb, active, res0, dq);
  } else {
    finish_field<R, NP, MODE>(k, qo, rw, P, 1, kb, active, res0, dq);
    order();
    wadg_inverse<R, N, NQ>(b1, w, dq);
    finish_field<R, NP, MODE>(k, qo, rw, P, 2, kb, active, res1, dq);
  }
}

// Copy `chunks` 16-byte chunks from a buffer resource into LDS with
// `threads` threads (thread t takes chunks t, t + threads, ...).
template <unsigned chunks, unsigned threads>
__device__ __forceinline__ void copy_to_lds(rsrc_t src, void* dst, int tid) {
  constexpr unsigned per = (chunks + threads - 1) / threads;
  u32x4 v[per];
#pragma unroll
  for (unsigned i = 0; i < per; ++i) {
    const unsigned c = tid + i * threads;
    if (c < chunks) v[i] = ld128(src, c * 16u);
  }
#pragma unroll
  for (unsigned i = 0; i < per; ++i) {
    const unsigned c = tid + i * threads;
    if (c < chunks) *reinterpret_cast<u32x4*>(static_cast<char*>(dst) + c * 16u) = v[i];
  }
}

}  // namespace

template <typename R, int N, int NQ, int MODE>
__global__ __launch_bounds__(kResidentWaves * kWave) void resident_kernel(const StageParams p) {
  static_assert(MODE == kStage || MODE == kRhs, "stage and right-hand-side modes only");
  constexpr bool RHS = MODE == kRhs;
  using L = Resident<R, N, NQ>;
  constexpr unsigned tile = L::tile;
  constexpr unsigned tile_bytes = tile * sizeof(R);
  __shared__ __attribute__((aligned(16))) R lds[L::values];
  R* const gv = lds;                   // [6][NQ2][64]
  R* const gf = lds + L::vol;          // [3][4][NQ][64]
  R* const tiles = gf + L::face;       // [2][tile]

  // workgroup -> (element group, slice range)
  const int w = item_of(blockIdx.x, gridDim.x, p.reverse);
  const int ranges = gridDim.x / p.nEG;
  const int eg = w / ranges, rg = w - eg * ranges;
  const int spr = (p.S + ranges - 1) / ranges;
  const int s0 = rg * spr, s1 = min(p.S, s0 + spr);
  const int items = (spr + 1) / 2;   // per pair; the same in every workgroup

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & (kWave - 1);
  const int pair = wave >> 1;
  const bool pressure = (wave & 1) == 0;
  R* const tq = tiles + pair * tile;

  const R* Qin = static_cast<const R*>(p.Qin);
  const size_t slice_vals = (size_t)p.nEG * tile;
  const size_t goff = (size_t)eg * tile;
  auto tile_rsrc = [&](const R* base, int s) {
    return make_rsrc(base + (size_t)s * slice_vals + goff, s < s1 ? tile_bytes : 0u);
  };

  // prologue: resident geometry and the first tile of each pair
  copy_to_lds<L::vol * sizeof(R) / 16, kResidentWaves * kWave>(
      make_rsrc(static_cast<const R*>(p.vol) + (size_t)eg * L::vol, L::vol * sizeof(R)), gv, tid);
  copy_to_lds<L::face * sizeof(R) / 16, kResidentWaves * kWave>(
      make_rsrc(static_cast<const R*>(p.face) + (size_t)eg * L::face, L::face * sizeof(R)), gf,
      tid);
  copy_to_lds<L::tile_chunks, kResidentWaves * kWave>(tile_rsrc(Qin, s0), tiles, tid);
  copy_to_lds<L::tile_chunks, kResidentWaves * kWave>(tile_rsrc(Qin, s0 + 1), tiles + tile, tid);
  NbrOffsets nbo;
  load_nbr(make_rsrc(p.nbr + (size_t)eg * 8 * kWave, 8u * kWave * 4u), lane, nbo);
  __syncthreads();

  const StageScalars<R> k = stage_scalars<R>(p);
  const bool active = eg * kWave + lane < p.K;
  R* const Qout = static_cast<R*>(p.Qout);
  R* const Res = static_cast<R*>(RHS ? p.Qout : p.res);
  R* const ResW = static_cast<R*>(RHS ? p.Qout : (p.res_out ? p.res_out : p.res));
  u32x4 pre[L::pre];

  for (int it = 0; it < items; ++it) {
    const int s = s0 + 2 * it + pair;
    if (s < s1) {
      const rsrc_t qs = make_rsrc(Qin + (size_t)s * slice_vals, (unsigned)(slice_vals * sizeof(R)));
      const rsrc_t qo = tile_rsrc(Qout, s);
      const size_t toff = (size_t)s * slice_vals + goff;
      const rsrc_t rr = make_rsrc(Res + toff, (RHS || k.A == R(0)) ? 0u : tile_bytes);
      const rsrc_t rw = make_rsrc(ResW + toff, RHS || p.res_dead ? 0u : tile_bytes);
      const rsrc_t qn = tile_rsrc(Qin, s + 2);
      if (pressure)
        resident_item<R, N, NQ, MODE, true>(k, qs, qo, rr, rw, qn, tq, gv, gf, nbo, lane,
                                            active, pre);
      else
        resident_item<R, N, NQ, MODE, false>(k, qs, qo, rr, rw, qn, tq, gv, gf, nbo, lane,
                                             active, pre);
    }
    __syncthreads();
    if (pressure && s + 2 < s1) {
#pragma unroll
      for (unsigned c = 0; c < L::pre; ++c) {
        const unsigned chunk = c * kWave + lane;
        if (chunk < L::tile_chunks)
          *reinterpret_cast<u32x4*>(reinterpret_cast<char*>(tq) + chunk * 16u) = pre[c];
      }
    }
    __syncthreads();
  }
}

namespace {

template <typename R, int N, int NQ>
int launch_nq(int mode, const StageParams& p, int ranges, void* stream) {
  if constexpr (!Resident<R, N, NQ>::fits) {
    return (int)hipErrorInvalidValue;
  } else {
    const dim3 grid(p.nEG * ranges), block(kResidentWaves * kWave);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (mode == kStage)
      hipLaunchKernelGGL((resident_kernel<R, N, NQ, kStage>), grid, block, 0, st, p);
    else if (mode == kRhs && sizeof(R) == sizeof(double))
      hipLaunchKernelGGL((resident_kernel<R, N, NQ, kRhs>), grid, block, 0, st, p);
    else
      return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
  }
}

template <typename R, int N>
int launch_n(int nq, int mode, const StageParams& p, int ranges, void* stream) {
  switch (nq - N) {
    case 1: return launch_nq<R, N, N + 1>(mode, p, ranges, stream);
    case 2: return launch_nq<R, N, N + 2>(mode, p, ranges, stream);
    case 3: return launch_nq<R, N, N + 3>(mode, p, ranges, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

template <typename R>
int launch_r(int N, int nq, int mode, const StageParams& p, int ranges, void* stream) {
  switch (N) {
    case 1: return launch_n<R, 1>(nq, mode, p, ranges, stream);
    case 2: return launch_n<R, 2>(nq, mode, p, ranges, stream);
    case 3: return launch_n<R, 3>(nq, mode, p, ranges, stream);
    case 4: return launch_n<R, 4>(nq, mode, p, ranges, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

template <typename R>
bool fits_r(int N, int nq) {
  const int NP = (N + 1) * (N + 1);
  const size_t values = (6u * nq * nq + 12u * nq + 6u * NP) * (size_t)kWave;
  return values * sizeof(R) <= kLdsBytes;
}

}  // namespace

bool resident_supported(int N, int nq, bool fp32) {
  if (!stage_supported(N, nq)) return false;
  return fp32 ? fits_r<float>(N, nq) : fits_r<double>(N, nq);
}

// Slice ranges per element group: enough workgroups to give every CU one
// (the LDS allocation admits one per CU), each pair at least one slice.
int resident_ranges(int nEG, int S, int cus) {
  int r = cus / (nEG > 0 ? nEG : 1);
  const int max_r = (S + 1) / 2;
  if (r > max_r) r = max_r;
  return r < 1 ? 1 : r;
}

int launch_stage_resident(int N, int nq, int mode, const StageParams& p, int ranges,
                          void* stream) {
  return launch_r<double>(N, nq, mode, p, ranges, stream);
}

int launch_stage_resident_fp32(int N, int nq, const StageParams& p, int ranges, void* stream) {
  return launch_r<float>(N, nq, kStage, p, ranges, stream);
}

}  // namespace wadg
