// Fused WADG stage kernel for gfx950.
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
// The group's input tile (3 (N+1)^2 x 64 values) is first copied into LDS
// by both waves with 16-byte coalesced loads, so every first-touch HBM read
// of the stage is in flight at once; the waves then re-read their own nodal
// values from LDS (lane-contiguous, conflict-free) instead of keeping them
// in registers.  Per lane:
//
//   a1  own face nodes (LDS) and the neighbours' face nodes (gathered from
//       the input slice through precomputed offsets, flip-aware),
//       interpolated to the face Gauss points;
//   a2  volume term of the strong-weak form (Section 4.1; Section 5.4,
//       volume kernel): u, v (pressure wave) or grad p (velocity wave) at the
//       volume Gauss points through the tensor factors of V_q, V_q^r, V_q^s,
//       times the weighted metric terms, and back to the nodes through the
//       transposed factors -- one quadrature column at a time, with the next
//       column's metric terms loaded while the current one is computed;
//   a3  penalised numerical flux and its lift (Section 5.4, surface kernel;
//       with GLL nodes the lift of face f touches only that face's nodes);
//   a4  weight-adjusted mass inverse P_q diag(w_q) V_q (Section 5.2, the
//       matrix-free product; w = c2/J for p and 1/J for u, v, Section 6),
//       with Mhat^{-1} folded into the first factor (V_q Mhat^{-1});
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

#include "reference_tables.h"
#include "wadg_internal.h"

namespace wadg {
namespace {

// Memory access through buffer resources: the base address and size of an
// array live in four scalar registers, the per-plane offset (node, field,
// quadrature point -- wave-uniform) in the instruction's offset fields, and
// the per-lane offset in one vector register shared by every access to the
// same tile.  Accesses outside the resource return zero instead of faulting.
using rsrc_t = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2 __attribute__((vector_size(8)));
typedef unsigned int u32x4 __attribute__((vector_size(16)));
constexpr int kRsrcWord3 = 0x00020000;   // raw dword buffer, gfx9 family

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           kRsrcWord3);
}
__device__ __forceinline__ void ld(rsrc_t r, unsigned voff, unsigned soff, double& v) {
  v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void ld(rsrc_t r, unsigned voff, unsigned soff, float& v) {
  v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <typename R>
__device__ __forceinline__ R ldr(rsrc_t r, unsigned voff, unsigned soff) {
  R v;
  ld(r, voff, soff, v);
  return v;
}
__device__ __forceinline__ void st(rsrc_t r, unsigned voff, unsigned soff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}
__device__ __forceinline__ void st(rsrc_t r, unsigned voff, unsigned soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
__device__ __forceinline__ int ldi(rsrc_t r, unsigned voff, unsigned soff) {
  return (int)__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
}

// Compiler-only barriers (no instructions are emitted).  order() keeps memory
// operations on their side of it, so a column's prefetches are issued before
// the previous column's arithmetic and LDS re-reads are not hoisted;
// pin(a) forces the values of `a` to be computed at that point, so the
// arithmetic of a quadrature column or face is not sunk towards the final
// stores (which would keep every loaded operand live to the end).
__device__ __forceinline__ void order() { asm volatile("" ::: "memory"); }
template <typename R, int M>
__device__ __forceinline__ void pin(R (&a)[M]) {
#pragma unroll
  for (int i = 0; i < M; ++i) asm volatile("" : "+v"(a[i]));
}

// local node index of face node m (face parameter order) on face f
template <int N>
__device__ constexpr int fnode(int f, int m) {
  return f == 0 ? m : f == 1 ? (N + (N + 1) * m) : f == 2 ? (m + (N + 1) * N) : ((N + 1) * m);
}

// Buffer resources of one workgroup: the group's tiles of the state arrays
// and of the geometry, and the whole input slice for neighbour gathers.
struct Bufs {
  rsrc_t qin, qout, res, qslice, vol, face, nbr;
};

// Stage-wide constants of one launch.
template <typename R>
struct StageScalars {
  R tau_p, tau_u, A, B, dt;
};

// dq = P_q diag(w) (V_q Mhat^{-1}) b in tensor form; w at the volume points
// (planes wplane .. wplane + NQ^2 of the geometry tile).
template <typename R, int N, int NQ>
__device__ __forceinline__ void wadg_inverse(const R (&b)[(N + 1) * (N + 1)], const Bufs& B,
                                             unsigned wplane, unsigned kb,
                                             R (&dq)[(N + 1) * (N + 1)]) {
  constexpr ct::Ops<R, N, NQ> T = ct::make_ops<R, N, NQ>();
  constexpr int NP1 = N + 1;
  constexpr unsigned KP = kWave * sizeof(R);
#pragma unroll
  for (int n = 0; n < NP1 * NP1; ++n) dq[n] = R(0);
  R wc[NQ], wn[NQ];
#pragma unroll
  for (int j = 0; j < NQ; ++j) wc[j] = ldr<R>(B.vol, kb, (wplane + NQ * j) * KP);
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    if (i + 1 < NQ) {
#pragma unroll
      for (int j = 0; j < NQ; ++j) wn[j] = ldr<R>(B.vol, kb, (wplane + i + 1 + NQ * j) * KP);
    }
    order();
    R t[NP1];
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb) {
      R acc = R(0);
#pragma unroll
      for (int a = 0; a < NP1; ++a) acc += T.Vt[i][a] * b[a + NP1 * bb];
      t[bb] = acc;
    }
    R c[NP1];
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb) c[bb] = R(0);
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      R rq = R(0);
#pragma unroll
      for (int bb = 0; bb < NP1; ++bb) rq += T.Vt[j][bb] * t[bb];
      rq *= wc[j];
#pragma unroll
      for (int bb = 0; bb < NP1; ++bb) c[bb] += T.P[bb][j] * rq;
    }
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb)
#pragma unroll
      for (int a = 0; a < NP1; ++a) dq[a + NP1 * bb] += T.P[a][i] * c[bb];
    pin(dq);
#pragma unroll
    for (int j = 0; j < NQ; ++j) wc[j] = wn[j];
  }
}

// a5 for field c: res <- A res + dt dq; Qout <- Qin + B res  (or dQ/dt).
// `resv` holds the residual prefetched before the WADG product.
template <typename R, int NP, bool RHS>
__device__ __forceinline__ void finish_field(const StageScalars<R>& k, const Bufs& B,
                                             const R* tq, int c, unsigned kb, int lane,
                                             bool active, const R (&resv)[NP],
                                             const R (&dq)[NP]) {
  constexpr unsigned KP = kWave * sizeof(R);
  if (!active) return;
  if constexpr (RHS) {
#pragma unroll
    for (int n = 0; n < NP; ++n) st(B.qout, kb, (c * NP + n) * KP, dq[n]);
  } else {
#pragma unroll
    for (int n = 0; n < NP; ++n) {
      const unsigned so = (c * NP + n) * KP;
      const R r = k.A * resv[n] + k.dt * dq[n];
      st(B.res, kb, so, r);
      st(B.qout, kb, so, tq[(c * NP + n) * kWave + lane] + k.B * r);
    }
  }
}

// Residual of field c, read before the WADG product so that its latency
// overlaps the arithmetic; not read at all when A = 0 (first stage).
template <typename R, int NP, bool RHS>
__device__ __forceinline__ void load_res(const StageScalars<R>& k, const Bufs& B, int c,
                                         unsigned kb, R (&resv)[NP]) {
  constexpr unsigned KP = kWave * sizeof(R);
  if constexpr (!RHS) {
    if (k.A != R(0)) {
#pragma unroll
      for (int n = 0; n < NP; ++n) resv[n] = ldr<R>(B.res, kb, (c * NP + n) * KP);
      return;
    }
  }
#pragma unroll
  for (int n = 0; n < NP; ++n) resv[n] = R(0);
}

// Neighbour face nodes of face f (in my face's parameter order) and the
// face geometry at the face's Gauss points.
template <typename R, int N, int NQ>
__device__ __forceinline__ void face_data(const Bufs& B, int f, unsigned kb, R (&pn)[N + 1],
                                          R (&un)[N + 1], R (&vn)[N + 1], R (&fg)[3][NQ]) {
  constexpr int NP = (N + 1) * (N + 1);
  constexpr unsigned KP = kWave * sizeof(R);
  // offset (in values, within the slice) of the neighbour's value at my
  // face node 0, and the step along my face parameter
  const unsigned nb0 = (unsigned)ldi(B.nbr, kb / sizeof(R) * 4, (0 * 4 + f) * kWave * 4);
  const int nstep = ldi(B.nbr, kb / sizeof(R) * 4, (1 * 4 + f) * kWave * 4);
#pragma unroll
  for (int m = 0; m <= N; ++m) {
    const unsigned off = (nb0 + (unsigned)(nstep * m)) * sizeof(R);
    pn[m] = ldr<R>(B.qslice, off, 0);
    un[m] = ldr<R>(B.qslice, off, NP * KP);
    vn[m] = ldr<R>(B.qslice, off, 2 * NP * KP);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < NQ; ++j) fg[c][j] = ldr<R>(B.face, kb, (c * 4 * NQ + f * NQ + j) * KP);
}

// Pressure equation: b_p = int u.grad(v) J - int 1/2(2{u}.n - tau_p [p]) v sJ.
template <typename R, int N, int NQ, bool RHS>
__device__ __forceinline__ void pressure_wave(const StageScalars<R>& k, const Bufs& B,
                                              const R* tq, unsigned kb, int lane, bool active) {
  constexpr ct::Ops<R, N, NQ> T = ct::make_ops<R, N, NQ>();
  constexpr int NP1 = N + 1, NP = NP1 * NP1, NQ2 = NQ * NQ;
  constexpr unsigned KP = kWave * sizeof(R);
  auto U = [&](int n) { return tq[(NP + n) * kWave + lane]; };
  auto V = [&](int n) { return tq[(2 * NP + n) * kWave + lane]; };
  auto P = [&](int n) { return tq[n * kWave + lane]; };

  R bp[NP];
#pragma unroll
  for (int n = 0; n < NP; ++n) bp[n] = R(0);

  // a2: sum_q w_q J (l_r (Jr_x u + Jr_y v) + l_s (Js_x u + Js_y v))
  R gc[4][NQ], gn[4][NQ];
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int j = 0; j < NQ; ++j) gc[g][j] = ldr<R>(B.vol, kb, (g * NQ2 + NQ * j) * KP);
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    if (i + 1 < NQ) {
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int j = 0; j < NQ; ++j) gn[g][j] = ldr<R>(B.vol, kb, (g * NQ2 + i + 1 + NQ * j) * KP);
    }
    order();
    R tu[NP1], tv[NP1];
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb) {
      R su = R(0), sv = R(0);
#pragma unroll
      for (int a = 0; a < NP1; ++a) {
        su += T.V[i][a] * U(a + NP1 * bb);
        sv += T.V[i][a] * V(a + NP1 * bb);
      }
      tu[bb] = su;
      tv[bb] = sv;
    }
    R cr[NP1], cs[NP1];
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb) cr[bb] = cs[bb] = R(0);
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      R uq = R(0), vq = R(0);
#pragma unroll
      for (int bb = 0; bb < NP1; ++bb) {
        uq += T.V[j][bb] * tu[bb];
        vq += T.V[j][bb] * tv[bb];
      }
      const R Ur = gc[0][j] * uq + gc[1][j] * vq;
      const R Us = gc[2][j] * uq + gc[3][j] * vq;
#pragma unroll
      for (int bb = 0; bb < NP1; ++bb) {
        cr[bb] += T.V[j][bb] * Ur;
        cs[bb] += T.D[j][bb] * Us;
      }
    }
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb)
#pragma unroll
      for (int a = 0; a < NP1; ++a) bp[a + NP1 * bb] += T.D[i][a] * cr[bb] + T.V[i][a] * cs[bb];
    pin(bp);
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int j = 0; j < NQ; ++j) gc[g][j] = gn[g][j];
  }

  // a1 + a3
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    order();
    R pn[NP1], un[NP1], vn[NP1], fg[3][NQ];
    face_data<R, N, NQ>(B, f, kb, pn, un, vn, fg);
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      R pm = R(0), um = R(0), vm = R(0), pp = R(0), up = R(0), vp = R(0);
#pragma unroll
      for (int m = 0; m < NP1; ++m) {
        pm += T.V[j][m] * P(fnode<N>(f, m));
        um += T.V[j][m] * U(fnode<N>(f, m));
        vm += T.V[j][m] * V(fnode<N>(f, m));
        pp += T.V[j][m] * pn[m];
        up += T.V[j][m] * un[m];
        vp += T.V[j][m] * vn[m];
      }
      const R nx = fg[0][j], ny = fg[1][j], wsJ = fg[2][j];
      const R fp = R(0.5) * wsJ * ((up + um) * nx + (vp + vm) * ny - k.tau_p * (pp - pm));
#pragma unroll
      for (int m = 0; m < NP1; ++m) bp[fnode<N>(f, m)] -= T.V[j][m] * fp;
    }
    pin(bp);
  }

  // a4 + a5
  order();
  R resv[NP], dq[NP];
  load_res<R, NP, RHS>(k, B, 0, kb, resv);
  wadg_inverse<R, N, NQ>(bp, B, 4 * NQ2, kb, dq);
  finish_field<R, NP, RHS>(k, B, tq, 0, kb, lane, active, resv, dq);
}

// Velocity equations: b_u = -int grad(p) . tau J - int 1/2([p] - tau_u [u].n) tau.n sJ.
template <typename R, int N, int NQ, bool RHS>
__device__ __forceinline__ void velocity_wave(const StageScalars<R>& k, const Bufs& B,
                                              const R* tq, unsigned kb, int lane, bool active) {
  constexpr ct::Ops<R, N, NQ> T = ct::make_ops<R, N, NQ>();
  constexpr int NP1 = N + 1, NP = NP1 * NP1, NQ2 = NQ * NQ;
  constexpr unsigned KP = kWave * sizeof(R);
  auto U = [&](int n) { return tq[(NP + n) * kWave + lane]; };
  auto V = [&](int n) { return tq[(2 * NP + n) * kWave + lane]; };
  auto P = [&](int n) { return tq[n * kWave + lane]; };

  R bu[NP], bv[NP];
#pragma unroll
  for (int n = 0; n < NP; ++n) bu[n] = bv[n] = R(0);

  // a2: -sum_q w_q J l (p_x, p_y)
  R gc[4][NQ], gn[4][NQ];
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int j = 0; j < NQ; ++j) gc[g][j] = ldr<R>(B.vol, kb, (g * NQ2 + NQ * j) * KP);
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    if (i + 1 < NQ) {
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int j = 0; j < NQ; ++j) gn[g][j] = ldr<R>(B.vol, kb, (g * NQ2 + i + 1 + NQ * j) * KP);
    }
    order();
    R td[NP1], tp[NP1];
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb) {
      R sd = R(0), sp = R(0);
#pragma unroll
      for (int a = 0; a < NP1; ++a) {
        const R pa = P(a + NP1 * bb);
        sd += T.D[i][a] * pa;
        sp += T.V[i][a] * pa;
      }
      td[bb] = sd;
      tp[bb] = sp;
    }
    R cx[NP1], cy[NP1];
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb) cx[bb] = cy[bb] = R(0);
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      R pr = R(0), ps = R(0);
#pragma unroll
      for (int bb = 0; bb < NP1; ++bb) {
        pr += T.V[j][bb] * td[bb];
        ps += T.D[j][bb] * tp[bb];
      }
      const R Gx = gc[0][j] * pr + gc[2][j] * ps;
      const R Gy = gc[1][j] * pr + gc[3][j] * ps;
#pragma unroll
      for (int bb = 0; bb < NP1; ++bb) {
        cx[bb] += T.V[j][bb] * Gx;
        cy[bb] += T.V[j][bb] * Gy;
      }
    }
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb)
#pragma unroll
      for (int a = 0; a < NP1; ++a) {
        bu[a + NP1 * bb] -= T.V[i][a] * cx[bb];
        bv[a + NP1 * bb] -= T.V[i][a] * cy[bb];
      }
    pin(bu);
    pin(bv);
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int j = 0; j < NQ; ++j) gc[g][j] = gn[g][j];
  }

  // a1 + a3
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    order();
    R pn[NP1], un[NP1], vn[NP1], fg[3][NQ];
    face_data<R, N, NQ>(B, f, kb, pn, un, vn, fg);
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      R pm = R(0), um = R(0), vm = R(0), pp = R(0), up = R(0), vp = R(0);
#pragma unroll
      for (int m = 0; m < NP1; ++m) {
        pm += T.V[j][m] * P(fnode<N>(f, m));
        um += T.V[j][m] * U(fnode<N>(f, m));
        vm += T.V[j][m] * V(fnode<N>(f, m));
        pp += T.V[j][m] * pn[m];
        up += T.V[j][m] * un[m];
        vp += T.V[j][m] * vn[m];
      }
      const R nx = fg[0][j], ny = fg[1][j], wsJ = fg[2][j];
      const R fu = R(0.5) * wsJ * ((pp - pm) - k.tau_u * ((up - um) * nx + (vp - vm) * ny));
      const R fx = fu * nx, fy = fu * ny;
#pragma unroll
      for (int m = 0; m < NP1; ++m) {
        bu[fnode<N>(f, m)] -= T.V[j][m] * fx;
        bv[fnode<N>(f, m)] -= T.V[j][m] * fy;
      }
    }
    pin(bu);
    pin(bv);
  }

  // a4 + a5, one field at a time
  order();
  R resv[NP], dq[NP];
  load_res<R, NP, RHS>(k, B, 1, kb, resv);
  wadg_inverse<R, N, NQ>(bu, B, 5 * NQ2, kb, dq);
  finish_field<R, NP, RHS>(k, B, tq, 1, kb, lane, active, resv, dq);
  order();
  load_res<R, NP, RHS>(k, B, 2, kb, resv);
  wadg_inverse<R, N, NQ>(bv, B, 5 * NQ2, kb, dq);
  finish_field<R, NP, RHS>(k, B, tq, 2, kb, lane, active, resv, dq);
}

}  // namespace

template <typename R, int N, int NQ, bool RHS>
__global__ __launch_bounds__(2 * kWave) void stage_kernel(const StageParams p) {
  constexpr int NP = (N + 1) * (N + 1);
  constexpr int NQ2 = NQ * NQ;
  constexpr unsigned tile = 3u * NP * kWave;   // values per group tile
  constexpr unsigned KP = kWave * sizeof(R);
  __shared__ __attribute__((aligned(16))) R tq[tile];

  // workgroup -> work item (XCD-aware): XCD x = bid % 8 receives the
  // contiguous logical range [x q8 + min(x, r8), ...) in launch order
  const int nb = gridDim.x, bid = blockIdx.x;
  const int q8 = nb >> 3, r8 = nb & 7;
  const int xcd = bid & 7, jx = bid >> 3;
  const int w = xcd * q8 + (xcd < r8 ? xcd : r8) + jx;
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
  B.res = make_rsrc(static_cast<R*>(RHS ? p.Qout : p.res) + grp, tile * sizeof(R));
  B.qslice = make_rsrc(Qin + slice, (unsigned)p.nEG * tile * sizeof(R));
  B.vol = make_rsrc(static_cast<const R*>(p.vol) + (size_t)eg * 6 * NQ2 * kWave, 6u * NQ2 * KP);
  B.face = make_rsrc(static_cast<const R*>(p.face) + (size_t)eg * 12 * NQ * kWave,
                     12u * NQ * KP);
  B.nbr = make_rsrc(p.nbr + (size_t)eg * 8 * kWave, 8u * kWave * 4u);

  // stage the input tile in LDS: 16-byte chunks, consecutive threads on
  // consecutive chunks
  constexpr unsigned chunks = tile * sizeof(R) / 16;
  for (unsigned c = tid; c < chunks; c += 2 * kWave) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(B.qin, c * 16u, 0, 0);
    *reinterpret_cast<u32x4*>(reinterpret_cast<char*>(tq) + c * 16u) = v;
  }
  __syncthreads();

  StageScalars<R> k;
  k.tau_p = (R)p.tau_p;
  k.tau_u = (R)p.tau_u;
  k.A = (R)p.rkA;
  k.B = (R)p.rkB;
  k.dt = (R)p.dt;
  const bool active = eg * kWave + lane < p.K;
  const unsigned kb = (unsigned)lane * sizeof(R);
  if (wave == 0)
    pressure_wave<R, N, NQ, RHS>(k, B, tq, kb, lane, active);
  else
    velocity_wave<R, N, NQ, RHS>(k, B, tq, kb, lane, active);
}

namespace {

template <typename R, int N, int NQ>
int launch_nq(bool rhs, const StageParams& p, void* stream) {
  const int nwg = p.nEG * p.S;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (rhs)
    hipLaunchKernelGGL((stage_kernel<R, N, NQ, true>), dim3(nwg), dim3(2 * kWave), 0, st, p);
  else
    hipLaunchKernelGGL((stage_kernel<R, N, NQ, false>), dim3(nwg), dim3(2 * kWave), 0, st, p);
  return (int)hipGetLastError();
}

template <typename R, int N>
int launch_n(int nq, bool rhs, const StageParams& p, void* stream) {
  switch (nq - N) {
    case 1: return launch_nq<R, N, N + 1>(rhs, p, stream);
    case 2: return launch_nq<R, N, N + 2>(rhs, p, stream);
    case 3: return launch_nq<R, N, N + 3>(rhs, p, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

template <typename R>
int launch_r(int N, int nq, bool rhs, const StageParams& p, void* stream) {
  switch (N) {
    case 1: return launch_n<R, 1>(nq, rhs, p, stream);
    case 2: return launch_n<R, 2>(nq, rhs, p, stream);
    case 3: return launch_n<R, 3>(nq, rhs, p, stream);
    case 4: return launch_n<R, 4>(nq, rhs, p, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace

bool stage_supported(int N, int nq) { return N >= 1 && N <= 4 && nq >= N + 1 && nq <= N + 3; }

int launch_stage(int N, int nq, bool rhs, const StageParams& p, void* stream) {
  return launch_r<double>(N, nq, rhs, p, stream);
}

int launch_stage_fp32(int N, int nq, const StageParams& p, void* stream) {
  return launch_r<float>(N, nq, false, p, stream);
}

}  // namespace wadg
