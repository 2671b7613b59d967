// Fused WADG stage kernel for gfx950, persistent pipelined variant.
//
// The same LSRK stage and the same arithmetic as the other stage kernels
// (stage_common.h: the strong-weak volume and surface terms of Section 6.4,
// the weight-adjusted mass inverse of Section 6.2, the 2N-storage update of
// Section 5.2), in the same order of operations, so its results are bitwise
// those of the split kernel.  What differs is how the work reaches the CU:
//
//   * One workgroup of eight waves per CU owns one 64-element group and a
//     run of consecutive slices of it, and walks them one after another.
//     The group's geometry is read once per workgroup, not once per item:
//     the four metric planes stay in LDS, the mass weights, face factors
//     and neighbour offsets stay in the registers of the waves that use
//     them.
//   * Wave 7 is a loader: while an item is computed it streams the next
//     slice's input tile into the other half of an LDS double buffer with
//     gfx950's direct-to-LDS buffer loads (no registers involved), so the
//     HBM latency of the tile is off the item's critical path.
//   * The face waves gather the next slice's neighbour traces into
//     registers as soon as their face terms are written, and the update
//     waves request the next slice's residual as soon as they have stored
//     this one's, each a full item ahead of its use.
//
// Roles per item (two barriers):
//   phase F  wave 0  pressure volume term        (Section 4.1, weak form)
//            wave 1  velocity volume terms, b_v handed to wave 6 in LDS
//            waves 2..5  traces, flux and lift of face 0..3 (all fields)
//            wave 7  tile of the next slice -> LDS
//   -- barrier: face terms and b_v in LDS
//   phase B  waves 0, 1, 6  face terms added in face order 0..3, mass
//            inverse and stage update of p, u, v
//            wave 7  waits for its tile
//   -- barrier: the current tile, face terms and b_v are free again
//
// LDS at N = 3, FP64: two input tiles (48 KB), the metric planes (50 KB),
// face terms (24 KB) and b_v (8 KB): 130 KB, one workgroup per CU with two
// waves per SIMD.  Instantiated where this fits in the CU's 160 KB.

#include <hip/hip_runtime.h>

#include "stage_common.h"

namespace wadg {
namespace {

using namespace dev;

template <typename R, int N, int NQ>
struct Pipe {
  static constexpr int NP1 = N + 1, NP = NP1 * NP1, NQ2 = NQ * NQ;
  static constexpr unsigned tile = 3u * NP * kWave;            // values of one input tile
  static constexpr unsigned tile_bytes = tile * sizeof(R);
  // the loader moves whole 1 KB rows (64 lanes x 16 B); the buffers are
  // padded to whole rows so that the last row's lanes stay inside them
  static constexpr unsigned rows = (tile_bytes + 1023u) / 1024u;
  static constexpr unsigned tile_alloc = rows * 1024u / sizeof(R);
  static constexpr unsigned metric = 4u * NQ2 * kWave;         // planes 0..3 of the geometry
  static constexpr unsigned xf = 4u * 3 * NP1 * kWave;         // face terms [4][3][NP1][64]
  static constexpr unsigned bv = (unsigned)NP * kWave;         // b_v [NP][64]
  static constexpr size_t lds_bytes = (2 * tile_alloc + metric + xf + bv) * sizeof(R);
  static constexpr bool fits = lds_bytes <= 160u * 1024u;
};

// Lane-parallel copy of `n16` 16-byte chunks from global memory into LDS by
// the waves [w0, w0 + nw) of the workgroup (prologue only).
__device__ __forceinline__ void copy_to_lds(rsrc_t src, void* dst, unsigned n16, int tid0,
                                            int nthreads) {
  for (unsigned c = (unsigned)tid0; c < n16; c += (unsigned)nthreads)
    *reinterpret_cast<u32x4*>(static_cast<char*>(dst) + c * 16u) = ld128(src, c * 16u);
}

// The loader wave's request of one input tile: `rows` direct-to-LDS loads of
// 64 lanes x 16 B, row r landing at dst + 1 KB r.
template <unsigned ROWS>
__device__ __forceinline__ void tile_to_lds(rsrc_t src, void* dst, int lane) {
#pragma unroll
  for (unsigned r = 0; r < ROWS; ++r)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(
        src, (__attribute__((address_space(3))) void*)(static_cast<char*>(dst) + r * 1024u), 16,
        (r * 64u + (unsigned)lane) * 16u, 0, 0, 0);
}

// Wait until every vector memory operation of this wave has completed
// (vmcnt = 0; the other counters left at their maxima).
__device__ __forceinline__ void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Face wave of face F: its factors and neighbour offsets held for the
// whole run, its traces gathered one slice ahead.  Barriers as the other
// roles: one after the prologue, two per item.
template <typename R, int N, int NQ, int F>
__device__ __forceinline__ void pipe_face_role(const StageParams& p, const StageScalars<R>& k,
                                               int g, int s0, int nit, int lane, unsigned kb,
                                               rsrc_t face, R (*tq)[Pipe<R, N, NQ>::tile_alloc],
                                               R* xf) {
  using L = Pipe<R, N, NQ>;
  constexpr int NP1 = L::NP1, NP = L::NP;
  constexpr unsigned KP = kWave * sizeof(R);
  const R* Qin = static_cast<const R*>(p.Qin);
  const size_t slice_vals = (size_t)p.nEG * L::tile;
  R gf[3][NQ];
#pragma unroll
  for (int cc = 0; cc < 3; ++cc)
#pragma unroll
    for (int jj = 0; jj < NQ; ++jj) gf[cc][jj] = ldr<R>(face, kb, (cc * 4 * NQ + F * NQ + jj) * KP);
  NbrOffsets nbo;
  load_nbr(make_rsrc(p.nbr + (size_t)g * 8 * kWave, 8u * kWave * 4u), lane, nbo);
  Trace<R, N> tr;
  gather_trace<R, N>(make_rsrc(Qin + (size_t)s0 * slice_vals, (unsigned)(slice_vals * sizeof(R))),
                     nbo, F, tr);
  __syncthreads();                                           // prologue done
  for (int it = 0; it < nit; ++it) {
    const R* t = tq[it & 1];
    auto Pt = [&](int n) { return t[n * kWave + lane]; };
    auto Ut = [&](int n) { return t[(NP + n) * kWave + lane]; };
    auto Vt = [&](int n) { return t[(2 * NP + n) * kWave + lane]; };
    R sp[NP1], su[NP1], sv[NP1];
    face_terms<R, N, NQ, true, true>(F, Pt, Ut, Vt, tr, gf, k.tau_p, k.tau_u, sp, su, sv);
#pragma unroll
    for (int m = 0; m < NP1; ++m) {
      xf[((F * 3 + 0) * NP1 + m) * kWave + lane] = sp[m];
      xf[((F * 3 + 1) * NP1 + m) * kWave + lane] = su[m];
      xf[((F * 3 + 2) * NP1 + m) * kWave + lane] = sv[m];
    }
    if (it + 1 < nit)
      gather_trace<R, N>(
          make_rsrc(Qin + (size_t)(s0 + it + 1) * slice_vals, (unsigned)(slice_vals * sizeof(R))),
          nbo, F, tr);
    __syncthreads();                                         // face terms, b_v ready
    __syncthreads();                                         // item done
  }
}

}  // namespace

// Workgroup b: element group g and slices [s0, s1) (see launch below);
// grid = nEG * chunks, chunk j of group g holds slices
// [j S / chunks, (j + 1) S / chunks).  LSRK stage mode only.
template <typename R, int N, int NQ>
__global__ __launch_bounds__(8 * kWave) void pipe_kernel(const StageParams p, int chunks) {
  using L = Pipe<R, N, NQ>;
  constexpr int NP1 = L::NP1, NP = L::NP, NQ2 = L::NQ2;
  constexpr unsigned tile = L::tile;
  constexpr unsigned KP = kWave * sizeof(R);
  __shared__ __attribute__((aligned(1024))) R tq[2][L::tile_alloc];
  __shared__ __attribute__((aligned(16))) R xm[L::metric];
  __shared__ __attribute__((aligned(16))) R xf[L::xf];
  __shared__ __attribute__((aligned(16))) R xv[L::bv];

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & (kWave - 1);
  const unsigned kb = (unsigned)lane * sizeof(R);

  // workgroup -> (group, slice run), XCD-aware: each XCD takes a
  // contiguous range of groups, so most neighbour traces are read by
  // workgroups of the same XCD
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  const int g = w / chunks, j = w - g * chunks;
  if (g >= p.nEG) return;                 // whole workgroup: no barrier reached
  const int s0 = (int)((int64_t)j * p.S / chunks);
  const int s1 = (int)((int64_t)(j + 1) * p.S / chunks);
  const int nit = s1 - s0;
  if (nit <= 0) return;
  const bool active = g * kWave + lane < p.K;
  const StageScalars<R> k = stage_scalars<R>(p);

  const R* Qin = static_cast<const R*>(p.Qin);
  R* Qout = static_cast<R*>(p.Qout);
  R* res = static_cast<R*>(p.res);
  R* resw = static_cast<R*>(p.res_out ? p.res_out : p.res);
  const size_t slice_vals = (size_t)p.nEG * tile;
  auto grp = [&](int s) { return (size_t)s * slice_vals + (size_t)g * tile; };
  const rsrc_t vol = make_rsrc(static_cast<const R*>(p.vol) + (size_t)g * 6 * NQ2 * kWave,
                               6u * NQ2 * KP);
  const rsrc_t face = make_rsrc(static_cast<const R*>(p.face) + (size_t)g * 12 * NQ * kWave,
                                12u * NQ * KP);

  auto P = [&](const R* t, int n) { return t[n * kWave + lane]; };

  // ---------------------------------------------------------------- prologue
  // metric planes 0..3 of the group into LDS (all waves but the loader)
  if (wave < 7) copy_to_lds(vol, xm, L::metric * sizeof(R) / 16u, tid, 7 * kWave);
  if (wave == 7)
    tile_to_lds<L::rows>(make_rsrc(Qin + grp(s0), L::tile_bytes), tq[0], lane);

  // ------------------------------------------------------------------ roles
  if (wave == 0 || wave == 1 || wave == 6) {
    // update waves: field c = 0 (p), 1 (u), 2 (v).  Mass weights c^2/J
    // (times the c^2 scale) or 1/J, held for the whole run.
    const int c = wave == 6 ? 2 : wave;
    R wq[NQ2];
#pragma unroll
    for (int q = 0; q < NQ2; ++q) wq[q] = ldr<R>(vol, kb, ((c == 0 ? 4 : 5) * NQ2 + q) * KP);
    if (c == 0) {
#pragma unroll
      for (int q = 0; q < NQ2; ++q) wq[q] *= k.c2s;
    }
    R resv[NP];
    load_res<R, NP, kStage>(k, make_rsrc(res + grp(s0), tile * sizeof(R)), c, kb, resv);
    __syncthreads();                                         // prologue done
    for (int it = 0; it < nit; ++it) {
      const int s = s0 + it;
      const R* t = tq[it & 1];
      auto Pt = [&](int n) { return P(t, n); };
      auto Ut = [&](int n) { return P(t, NP + n); };
      auto Vt = [&](int n) { return P(t, 2 * NP + n); };
      R b0[NP], b1[NP];
      if (c == 0) {
#pragma unroll
        for (int n = 0; n < NP; ++n) b0[n] = R(0);
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
          R gc[4][NQ];
          order();
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int jj = 0; jj < NQ; ++jj) gc[q][jj] = xm[(q * NQ2 + i + NQ * jj) * kWave + lane];
          pressure_volume_column<R, N, NQ>(i, Ut, Vt, gc, b0);
          pin(b0);
        }
      } else if (c == 1) {
#pragma unroll
        for (int n = 0; n < NP; ++n) b0[n] = b1[n] = R(0);
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
          R gc[4][NQ];
          order();
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int jj = 0; jj < NQ; ++jj) gc[q][jj] = xm[(q * NQ2 + i + NQ * jj) * kWave + lane];
          velocity_volume_column<R, N, NQ>(i, Pt, gc, b0, b1);
          pin(b0);
          pin(b1);
        }
#pragma unroll
        for (int n = 0; n < NP; ++n) xv[n * kWave + lane] = b1[n];
      }
      __syncthreads();                                       // face terms, b_v ready
      if (c == 2) {
#pragma unroll
        for (int n = 0; n < NP; ++n) b0[n] = xv[n * kWave + lane];
      }
#pragma unroll
      for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int m = 0; m < NP1; ++m)
          b0[fnode<N>(f, m)] += xf[((f * 3 + c) * NP1 + m) * kWave + lane];
      R dq[NP];
      wadg_inverse<R, N, NQ>(b0, wq, dq);
      const rsrc_t qo = make_rsrc(Qout + grp(s), tile * sizeof(R));
      const rsrc_t rw = make_rsrc(resw + grp(s), tile * sizeof(R));
      finish_field<R, NP, kStage>(k, qo, rw, Pt, c, kb, active, resv, dq);
      if (it + 1 < nit)
        load_res<R, NP, kStage>(k, make_rsrc(res + grp(s + 1), tile * sizeof(R)), c, kb, resv);
      __syncthreads();                                       // item done
    }
  } else if (wave == 7) {
    // loader: the next slice's tile while this one is computed
    wait_vm_all();
    __syncthreads();                                         // prologue done
    for (int it = 0; it < nit; ++it) {
      if (it + 1 < nit)
        tile_to_lds<L::rows>(make_rsrc(Qin + grp(s0 + it + 1), L::tile_bytes), tq[(it + 1) & 1],
                             lane);
      __syncthreads();                                       // face terms, b_v ready
      wait_vm_all();                                         // next tile in LDS
      __syncthreads();                                       // item done
    }
  } else if (wave == 2) {
    pipe_face_role<R, N, NQ, 0>(p, k, g, s0, nit, lane, kb, face, tq, xf);
  } else if (wave == 3) {
    pipe_face_role<R, N, NQ, 1>(p, k, g, s0, nit, lane, kb, face, tq, xf);
  } else if (wave == 4) {
    pipe_face_role<R, N, NQ, 2>(p, k, g, s0, nit, lane, kb, face, tq, xf);
  } else {
    pipe_face_role<R, N, NQ, 3>(p, k, g, s0, nit, lane, kb, face, tq, xf);
  }
}

namespace {

// Slice runs per element group: enough workgroups to give every CU one
// (grid = nEG * chunks), at most one per slice.
int pipe_chunks(int nEG, int S, int cus) {
  int c = cus / (nEG > 0 ? nEG : 1);
  if (c < 1) c = 1;
  if (c > S) c = S;
  return c;
}

template <typename R, int N, int NQ>
int launch_nq(const StageParams& p, int cus, void* stream) {
  if constexpr (!Pipe<R, N, NQ>::fits) {
    return (int)hipErrorInvalidValue;
  } else {
    const int chunks = pipe_chunks(p.nEG, p.S, cus);
    if ((int64_t)p.nEG * chunks >= (1LL << 31)) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL((pipe_kernel<R, N, NQ>), dim3(p.nEG * chunks), dim3(8 * kWave), 0,
                       static_cast<hipStream_t>(stream), p, chunks);
    return (int)hipGetLastError();
  }
}

template <typename R, int N>
int launch_n(int nq, const StageParams& p, int cus, void* stream) {
  switch (nq - N) {
    case 1: return launch_nq<R, N, N + 1>(p, cus, stream);
    case 2: return launch_nq<R, N, N + 2>(p, cus, stream);
    case 3: return launch_nq<R, N, N + 3>(p, cus, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

template <typename R>
int launch_r(int N, int nq, const StageParams& p, int cus, void* stream) {
  switch (N) {
    case 1: return launch_n<R, 1>(nq, p, cus, stream);
    case 2: return launch_n<R, 2>(nq, p, cus, stream);
    case 3: return launch_n<R, 3>(nq, p, cus, stream);
    case 4: return launch_n<R, 4>(nq, p, cus, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

template <typename R, int N>
bool fits_n(int nq) {
  switch (nq - N) {
    case 1: return Pipe<R, N, N + 1>::fits;
    case 2: return Pipe<R, N, N + 2>::fits;
    case 3: return Pipe<R, N, N + 3>::fits;
    default: return false;
  }
}

}  // namespace

bool pipe_supported(int N, int nq, bool fp32) {
  switch (N) {
    case 1: return fp32 ? fits_n<float, 1>(nq) : fits_n<double, 1>(nq);
    case 2: return fp32 ? fits_n<float, 2>(nq) : fits_n<double, 2>(nq);
    case 3: return fp32 ? fits_n<float, 3>(nq) : fits_n<double, 3>(nq);
    case 4: return fp32 ? fits_n<float, 4>(nq) : fits_n<double, 4>(nq);
    default: return false;
  }
}

int launch_stage_pipe(int N, int nq, const StageParams& p, int cus, void* stream) {
  return launch_r<double>(N, nq, p, cus, stream);
}

int launch_stage_pipe_fp32(int N, int nq, const StageParams& p, int cus, void* stream) {
  return launch_r<float>(N, nq, p, cus, stream);
}

}  // namespace wadg
