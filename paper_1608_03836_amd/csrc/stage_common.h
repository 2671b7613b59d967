// Device building blocks shared by the WADG stage kernels (streamed
// geometry, LDS-resident geometry, split work, batched problems).
//
// Every kernel maps one element to one lane and uses the same arithmetic,
// written once here, so they produce bit-identical results:
//
//   * pressure / velocity volume term of one quadrature column (Section 4.1,
//     strong-weak form; Section 6.4, volume kernel), through the tensor
//     factors of V_q and its derivatives and the weighted metric terms;
//   * penalised numerical flux on one face and its lift (Section 6.4,
//     surface kernel; with GLL nodes the lift of a face touches only that
//     face's nodes);
//   * the weight-adjusted mass inverse P_q diag(w) (V_q Mhat^{-1})
//     (Section 6.2, matrix-free product; w = c2/J for p, 1/J for u and v,
//     Section 7);
//   * the 2N-storage LSRK update (Section 5.2).
//
// Operands are nodal values of one element (lane) read through accessors,
// so the caller decides where they live (LDS tile, registers).
#pragma once

#include <hip/hip_runtime.h>

#include "reference_tables.h"
#include "wadg_internal.h"

// Every multiply-add below is an explicit fused multiply-add in a fixed
// order, and the compiler forms no others: the stage kernels, which inline
// these helpers into different contexts, then round identically.
#pragma clang fp contract(off)

namespace wadg {
namespace dev {

__device__ __forceinline__ double mad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float mad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

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
__device__ __forceinline__ u32x4 ld128(rsrc_t r, unsigned voff) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0);
}

// Compiler-only barriers (no instructions are emitted).  order() keeps memory
// operations on their side of it, so prefetches are issued before the
// arithmetic they overlap and LDS re-reads are not hoisted; pin(a) forces
// the values of `a` to be computed at that point, so the arithmetic of a
// quadrature column or face is not sunk towards the final stores (which
// would keep every loaded operand live to the end).
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

// Stage-wide constants of one launch.
template <typename R>
struct StageScalars {
  R tau_p, tau_u, A, B, dt, c2s;
};

template <typename R>
__device__ __forceinline__ StageScalars<R> stage_scalars(const StageParams& p) {
  StageScalars<R> k;
  k.tau_p = (R)p.tau_p;
  k.tau_u = (R)p.tau_u;
  k.A = (R)p.rkA;
  k.B = (R)p.rkB;
  k.dt = (R)p.dt;
  k.c2s = (R)p.c2_scale;
  return k;
}

// Per-lane neighbour addressing of the four faces: offset (in values, within
// the slice) of the neighbour's value at my face node 0, and the step along
// my face parameter.  The same for every slice.
struct NbrOffsets {
  unsigned base[4];
  int step[4];
};

__device__ __forceinline__ void load_nbr(rsrc_t nbr, int lane, NbrOffsets& o) {
  const unsigned kb4 = (unsigned)lane * 4u;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    o.base[f] = (unsigned)ldi(nbr, kb4, (0 * 4 + f) * kWave * 4);
    o.step[f] = ldi(nbr, kb4, (1 * 4 + f) * kWave * 4);
  }
}

// The neighbour's p, u, v at my face nodes of face f (my face's parameter
// order), gathered from the input slice.
template <typename R, int N>
struct Trace {
  R p[N + 1], u[N + 1], v[N + 1];
};

template <typename R, int N>
__device__ __forceinline__ void gather_trace(rsrc_t qslice, const NbrOffsets& o, int f,
                                             Trace<R, N>& t) {
  constexpr int NP = (N + 1) * (N + 1);
  constexpr unsigned KP = kWave * sizeof(R);
#pragma unroll
  for (int m = 0; m <= N; ++m) {
    const unsigned off = (o.base[f] + (unsigned)(o.step[f] * m)) * sizeof(R);
    t.p[m] = ldr<R>(qslice, off, 0);
    t.u[m] = ldr<R>(qslice, off, NP * KP);
    t.v[m] = ldr<R>(qslice, off, 2 * NP * KP);
  }
}

// ---------------------------------------------------------------------------
// Arithmetic.  `P`, `U`, `V` are accessors n -> nodal value of this lane's
// element; `g` holds geometry values of this lane.

// Pressure volume term, quadrature column i:
//   bp += sum_j w J (l_r (Jr_x u + Jr_y v) + l_s (Js_x u + Js_y v))
// with g[0..3][j] = W ys, -W xs, -W yr, W xr at point (i, j).
template <typename R, int N, int NQ, typename FU, typename FV>
__device__ __forceinline__ void pressure_volume_column(int i, const FU& U, const FV& V,
                                                       const R (&g)[4][NQ],
                                                       R (&bp)[(N + 1) * (N + 1)]) {
  constexpr ct::Ops<R, N, NQ> T = ct::make_ops<R, N, NQ>();
  constexpr int NP1 = N + 1;
  R tu[NP1], tv[NP1];
#pragma unroll
  for (int bb = 0; bb < NP1; ++bb) {
    R su = R(0), sv = R(0);
#pragma unroll
    for (int a = 0; a < NP1; ++a) {
      su = mad(T.V[i][a], U(a + NP1 * bb), su);
      sv = mad(T.V[i][a], V(a + NP1 * bb), sv);
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
      uq = mad(T.V[j][bb], tu[bb], uq);
      vq = mad(T.V[j][bb], tv[bb], vq);
    }
    const R Ur = mad(g[0][j], uq, g[1][j] * vq);
    const R Us = mad(g[2][j], uq, g[3][j] * vq);
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb) {
      cr[bb] = mad(T.V[j][bb], Ur, cr[bb]);
      cs[bb] = mad(T.D[j][bb], Us, cs[bb]);
    }
  }
#pragma unroll
  for (int bb = 0; bb < NP1; ++bb)
#pragma unroll
    for (int a = 0; a < NP1; ++a)
      bp[a + NP1 * bb] = mad(T.D[i][a], cr[bb], mad(T.V[i][a], cs[bb], bp[a + NP1 * bb]));
}

// Velocity volume term, quadrature column i:  (bu, bv) -= sum_j w J l grad p.
template <typename R, int N, int NQ, typename FP>
__device__ __forceinline__ void velocity_volume_column(int i, const FP& P, const R (&g)[4][NQ],
                                                       R (&bu)[(N + 1) * (N + 1)],
                                                       R (&bv)[(N + 1) * (N + 1)]) {
  constexpr ct::Ops<R, N, NQ> T = ct::make_ops<R, N, NQ>();
  constexpr int NP1 = N + 1;
  R td[NP1], tp[NP1];
#pragma unroll
  for (int bb = 0; bb < NP1; ++bb) {
    R sd = R(0), sp = R(0);
#pragma unroll
    for (int a = 0; a < NP1; ++a) {
      const R pa = P(a + NP1 * bb);
      sd = mad(T.D[i][a], pa, sd);
      sp = mad(T.V[i][a], pa, sp);
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
      pr = mad(T.V[j][bb], td[bb], pr);
      ps = mad(T.D[j][bb], tp[bb], ps);
    }
    const R Gx = mad(g[0][j], pr, g[2][j] * ps);
    const R Gy = mad(g[1][j], pr, g[3][j] * ps);
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb) {
      cx[bb] = mad(T.V[j][bb], Gx, cx[bb]);
      cy[bb] = mad(T.V[j][bb], Gy, cy[bb]);
    }
  }
#pragma unroll
  for (int bb = 0; bb < NP1; ++bb)
#pragma unroll
    for (int a = 0; a < NP1; ++a) {
      bu[a + NP1 * bb] = mad(-T.V[i][a], cx[bb], bu[a + NP1 * bb]);
      bv[a + NP1 * bb] = mad(-T.V[i][a], cy[bb], bv[a + NP1 * bb]);
    }
}

// Own and neighbour traces of p, u, v at face Gauss point j of face f.
template <typename R, int N, int NQ, typename FP, typename FU, typename FV>
__device__ __forceinline__ void face_point(int f, int j, const FP& P, const FU& U, const FV& V,
                                           const Trace<R, N>& t, R& pm, R& um, R& vm, R& pp,
                                           R& up, R& vp) {
  constexpr ct::Ops<R, N, NQ> T = ct::make_ops<R, N, NQ>();
  pm = um = vm = pp = up = vp = R(0);
#pragma unroll
  for (int m = 0; m <= N; ++m) {
    pm = mad(T.V[j][m], P(fnode<N>(f, m)), pm);
    um = mad(T.V[j][m], U(fnode<N>(f, m)), um);
    vm = mad(T.V[j][m], V(fnode<N>(f, m)), vm);
    pp = mad(T.V[j][m], t.p[m], pp);
    up = mad(T.V[j][m], t.u[m], up);
    vp = mad(T.V[j][m], t.v[m], vp);
  }
}

// Flux at face Gauss point j and its lifting weight: the pressure flux
//   fp = 1/2 w sJ (2{u}.n - tau_p [p])
// and the velocity flux vector (fx, fy) = 1/2 w sJ ([p] - tau_u [u].n) n,
// g[c][j] = nx, ny, w sJ.
template <typename R, int NQ>
__device__ __forceinline__ R pressure_flux(int j, R pm, R um, R vm, R pp, R up, R vp,
                                           const R (&g)[3][NQ], R tau_p) {
  const R nx = g[0][j], ny = g[1][j], wsJ = g[2][j];
  const R un = mad(up + um, nx, (vp + vm) * ny);          // 2 {u}.n
  return (R(0.5) * wsJ) * mad(-tau_p, pp - pm, un);
}
template <typename R, int NQ>
__device__ __forceinline__ void velocity_flux(int j, R pm, R um, R vm, R pp, R up, R vp,
                                              const R (&g)[3][NQ], R tau_u, R& fx, R& fy) {
  const R nx = g[0][j], ny = g[1][j], wsJ = g[2][j];
  const R jn = mad(up - um, nx, (vp - vm) * ny);          // [u].n
  const R fu = (R(0.5) * wsJ) * mad(-tau_u, jn, pp - pm);
  fx = fu * nx;
  fy = fu * ny;
}

// Surface terms of face f at the face's nodes m = 0..N (node fnode(f, m)):
//   sp[m] = -sum_j V[j][m] fp_j,  (su, sv)[m] = -sum_j V[j][m] (fx, fy)_j,
// each summed over the face's Gauss points on its own; the caller adds the
// faces' terms to the load vector in face order 0..3.
template <typename R, int N, int NQ, bool PRESS, bool VEL, typename FP, typename FU, typename FV>
__device__ __forceinline__ void face_terms(int f, const FP& P, const FU& U, const FV& V,
                                           const Trace<R, N>& t, const R (&g)[3][NQ], R tau_p,
                                           R tau_u, R (&sp)[N + 1], R (&su)[N + 1],
                                           R (&sv)[N + 1]) {
  constexpr ct::Ops<R, N, NQ> T = ct::make_ops<R, N, NQ>();
#pragma unroll
  for (int m = 0; m <= N; ++m) sp[m] = su[m] = sv[m] = R(0);
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    R pm, um, vm, pp, up, vp;
    face_point<R, N, NQ>(f, j, P, U, V, t, pm, um, vm, pp, up, vp);
    if constexpr (PRESS) {
      const R fp = pressure_flux<R, NQ>(j, pm, um, vm, pp, up, vp, g, tau_p);
#pragma unroll
      for (int m = 0; m <= N; ++m) sp[m] = mad(-T.V[j][m], fp, sp[m]);
    }
    if constexpr (VEL) {
      R fx, fy;
      velocity_flux<R, NQ>(j, pm, um, vm, pp, up, vp, g, tau_u, fx, fy);
#pragma unroll
      for (int m = 0; m <= N; ++m) {
        su[m] = mad(-T.V[j][m], fx, su[m]);
        sv[m] = mad(-T.V[j][m], fy, sv[m]);
      }
    }
  }
}

// Pressure surface term of face f added to bp.
template <typename R, int N, int NQ, typename FP, typename FU, typename FV>
__device__ __forceinline__ void pressure_face(int f, const FP& P, const FU& U, const FV& V,
                                              const Trace<R, N>& t, const R (&g)[3][NQ], R tau_p,
                                              R (&bp)[(N + 1) * (N + 1)]) {
  R sp[N + 1], su[N + 1], sv[N + 1];
  face_terms<R, N, NQ, true, false>(f, P, U, V, t, g, tau_p, R(0), sp, su, sv);
#pragma unroll
  for (int m = 0; m <= N; ++m) bp[fnode<N>(f, m)] += sp[m];
}

// Velocity surface terms of face f added to (bu, bv).
template <typename R, int N, int NQ, typename FP, typename FU, typename FV>
__device__ __forceinline__ void velocity_face(int f, const FP& P, const FU& U, const FV& V,
                                              const Trace<R, N>& t, const R (&g)[3][NQ], R tau_u,
                                              R (&bu)[(N + 1) * (N + 1)],
                                              R (&bv)[(N + 1) * (N + 1)]) {
  R sp[N + 1], su[N + 1], sv[N + 1];
  face_terms<R, N, NQ, false, true>(f, P, U, V, t, g, R(0), tau_u, sp, su, sv);
#pragma unroll
  for (int m = 0; m <= N; ++m) {
    bu[fnode<N>(f, m)] += su[m];
    bv[fnode<N>(f, m)] += sv[m];
  }
}

// dq = P_q diag(w) (V_q Mhat^{-1}) b in tensor form; w holds the NQ^2
// weights at the volume points (point i + NQ j).
template <typename R, int N, int NQ>
__device__ __forceinline__ void wadg_inverse(const R (&b)[(N + 1) * (N + 1)],
                                             const R (&w)[NQ * NQ],
                                             R (&dq)[(N + 1) * (N + 1)]) {
  constexpr ct::Ops<R, N, NQ> T = ct::make_ops<R, N, NQ>();
  constexpr int NP1 = N + 1;
#pragma unroll
  for (int n = 0; n < NP1 * NP1; ++n) dq[n] = R(0);
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    R t[NP1];
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb) {
      R acc = R(0);
#pragma unroll
      for (int a = 0; a < NP1; ++a) acc = mad(T.Vt[i][a], b[a + NP1 * bb], acc);
      t[bb] = acc;
    }
    R c[NP1];
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb) c[bb] = R(0);
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      R rq = R(0);
#pragma unroll
      for (int bb = 0; bb < NP1; ++bb) rq = mad(T.Vt[j][bb], t[bb], rq);
      rq *= w[i + NQ * j];
#pragma unroll
      for (int bb = 0; bb < NP1; ++bb) c[bb] = mad(T.P[bb][j], rq, c[bb]);
    }
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb)
#pragma unroll
      for (int a = 0; a < NP1; ++a) dq[a + NP1 * bb] = mad(T.P[a][i], c[bb], dq[a + NP1 * bb]);
    pin(dq);
  }
}

// The per-field operand of the final update: the residual in stage mode
// (zeros, not read, when A = 0 -- the first stage), the adjoint state ybar
// in apply-A mode, nothing in right-hand-side mode.
template <typename R, int NP, int MODE>
__device__ __forceinline__ void load_res(const StageScalars<R>& k, rsrc_t res, int c,
                                         unsigned kb, R (&resv)[NP]) {
  constexpr unsigned KP = kWave * sizeof(R);
  if constexpr (MODE != kRhs) {
    if (MODE == kApplyA || MODE == kApplyAMass || k.A != R(0)) {
#pragma unroll
      for (int n = 0; n < NP; ++n) resv[n] = ldr<R>(res, kb, (c * NP + n) * KP);
      return;
    }
  }
#pragma unroll
  for (int n = 0; n < NP; ++n) resv[n] = R(0);
}

// a5 for field c.  Stage mode: res <- A res + dt dq (written through
// `resw`), Qout <- Qin + B res.  Right-hand-side mode: Qout <- dq.  Apply-A
// mode: Qout <- ybar + dt D dq with dq the load vector and D = diag(1,-1,-1).
// `qin(n)` is the input value of node n.
template <typename R, int NP, int MODE, typename FQ>
__device__ __forceinline__ void finish_field(const StageScalars<R>& k, rsrc_t qout, rsrc_t resw,
                                             const FQ& qin, int c, unsigned kb, bool active,
                                             const R (&resv)[NP], const R (&dq)[NP]) {
  constexpr unsigned KP = kWave * sizeof(R);
  if (!active) return;
  if constexpr (MODE == kRhs) {
#pragma unroll
    for (int n = 0; n < NP; ++n) st(qout, kb, (c * NP + n) * KP, dq[n]);
  } else if constexpr (MODE == kApplyA) {
    const R sdt = c == 0 ? k.dt : -k.dt;
#pragma unroll
    for (int n = 0; n < NP; ++n) st(qout, kb, (c * NP + n) * KP, mad(sdt, dq[n], resv[n]));
  } else {
#pragma unroll
    for (int n = 0; n < NP; ++n) {
      const unsigned so = (c * NP + n) * KP;
      const R r = mad(k.A, resv[n], k.dt * dq[n]);
      st(resw, kb, so, r);
      st(qout, kb, so, mad(k.B, r, qin(c * NP + n)));
    }
  }
}

// Workgroup -> logical work index, XCD-aware: workgroups are dealt to the 8
// XCDs round-robin, so XCD x = bid % 8 receives the contiguous logical range
// [x q8 + min(x, r8), ...) in launch order.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int q8 = nb >> 3, r8 = nb & 7;
  const int xcd = bid & 7, jx = bid >> 3;
  return xcd * q8 + (xcd < r8 ? xcd : r8) + jx;
}

// Work item of workgroup bid: the XCD-aware order above, or the same order
// run backwards (each XCD still takes one contiguous run of items).
// Successive dependent launches alternate the direction, so that a launch
// starts on the items whose inputs the previous launch wrote last -- the
// ones most likely still held in the memory-side cache.
__device__ __forceinline__ int item_of(int bid, int nb, int reverse) {
  const int w = xcd_remap(bid, nb);
  return reverse ? nb - 1 - w : w;
}

}  // namespace dev
}  // namespace wadg
