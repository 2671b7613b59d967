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
//     the four metric planes and the pressure mass weights stay in LDS, the
//     velocity mass weights in the registers of their waves, the face
//     factors and neighbour offsets in the registers of the face waves.
//   * The items go through a two-stage pipeline: in step j the volume and
//     face waves build item j's load vector (volume term, then the face
//     terms in face order 0..3) and hand it over through LDS, while the
//     inverse waves apply the mass inverse and the stage update to item
//     j - 1.  The two halves of an item's work run on different waves, so
//     all four SIMDs compute in every phase.
//   * The v volume wave also loads the tiles: while an item is computed it
//     streams the next slice's input tile into the other half of an LDS
//     double buffer with gfx950's direct-to-LDS buffer loads (no registers
//     involved).  The face waves gather the next slice's neighbour traces
//     into registers as soon as their face terms are written, and the
//     inverse waves request the next residual as soon as they have used
//     this one, each a full item ahead of its use.
//
// Waves (wave w runs on SIMD w mod 4), two barriers per step:
//   wave 0  pressure volume term (Section 4.1, weak form)
//   waves 1, 2  the u and v components of the velocity volume term
//   wave 3  pressure mass inverse and update      wave 4  faces 0, 1
//   waves 5, 6  u, v mass inverses and updates    wave 7  faces 2, 3
//   -- barrier: face terms of item j in LDS
//   waves 0..2 add them in face order and hand the load vectors over
//   -- barrier: load vectors handed over, the next tile in LDS
// Between the two waves of a SIMD the inverse waves have issue priority,
// then the pressure volume wave, then the velocity volume waves.
//
// A first stage (A = 0) requests no residual; the last stage of a step,
// whose residual is never read again, is a kernel instance of its own that
// stores none.  The batched kernel runs the same roles over a list of runs
// of many problems, and lets the copies of a packed mesh share one copy's
// geometry.
//
// LDS at N = 3, FP64: two input tiles (48 KB), the metric planes (50 KB),
// face terms (24 KB), the handed-over load vectors (24 KB) and the pressure
// mass weights (12.5 KB): 158.5 KB, one workgroup per CU with two waves per
// SIMD.  Instantiated where this fits in the CU's 160 KB.

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
  static constexpr unsigned metric_rows = metric * sizeof(R) / 1024u;   // whole 1 KB rows
  static_assert(metric * sizeof(R) % 1024u == 0, "the metric planes are whole 1 KB rows");
  static constexpr unsigned xf = 4u * 3 * NP1 * kWave;         // face terms [4][3][NP1][64]
  static constexpr unsigned xb = 3u * NP * kWave;              // load vectors handed over [3][NP][64]
  static constexpr unsigned wp = NQ2 * kWave;                  // pressure mass weights [NQ2][64]
  static constexpr size_t lds_bytes = (2 * tile_alloc + metric + xf + xb + wp) * sizeof(R);
  static constexpr bool fits = lds_bytes <= 160u * 1024u;
};

// Rows r = w, w + nw, ... < ROWS of 1 KB (64 lanes x 16 B) from global
// memory into LDS (row r at dst + 1 KB r) with direct-to-LDS loads, by wave
// w of nw sharing the copy: the loads are issued back to back and land
// without registers; the caller waits (vmcnt) before the barrier that
// publishes them.
template <unsigned ROWS>
__device__ __forceinline__ void rows_to_lds(rsrc_t src, void* dst, int w, int nw, int lane) {
  for (unsigned r = (unsigned)w; r < ROWS; r += (unsigned)nw)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(
        src, (__attribute__((address_space(3))) void*)(static_cast<char*>(dst) + r * 1024u), 16,
        (r * 64u + (unsigned)lane) * 16u, 0, 0, 0);
}

// Lane L of a direct-to-LDS row load moves values 2 (L mod 32) and the next
// of a 64-value (512 B) plane row: whether they include one of the first
// `elems` lanes' values.  Batches skip the rest (padding, or values that
// every group reads from its problem's first group).
__device__ __forceinline__ bool row_lane_needed(int lane, int elems) {
  return 2 * (lane & 31) < elems;
}

// The tile loader's request of one input tile: `rows` direct-to-LDS loads of
// 64 lanes x 16 B, row r landing at dst + 1 KB r.
template <unsigned ROWS>
__device__ __forceinline__ void tile_to_lds(rsrc_t src, void* dst, int lane) {
#pragma unroll
  for (unsigned r = 0; r < ROWS; ++r)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(
        src, (__attribute__((address_space(3))) void*)(static_cast<char*>(dst) + r * 1024u), 16,
        (r * 64u + (unsigned)lane) * 16u, 0, 0, 0);
}

// Buffer stores with the non-temporal hint, for launches whose state is far
// larger than the caches: nothing they write is read again before the
// whole launch has streamed through.  The residual is loaded with it too
// (only its own item reads it); the input tile is not (its lines are also
// the neighbours' traces).
__device__ __forceinline__ void st_nt(rsrc_t r, unsigned voff, unsigned soff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 2);
}
__device__ __forceinline__ void st_nt(rsrc_t r, unsigned voff, unsigned soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 2);
}

// a5 of the LSRK stage for field c (finish_field's stage mode, the same
// operations in the same order) with non-temporal stores.
template <typename R>
__device__ __forceinline__ R ldr_nt(rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(R) == 8)
    return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 2));
  else
    return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 2));
}

template <typename R, int NP, typename FQ>
__device__ __forceinline__ void finish_field_nt(const StageScalars<R>& k, rsrc_t qout,
                                                rsrc_t resw, const FQ& qin, int c, unsigned kb,
                                                bool active, const R (&resv)[NP],
                                                const R (&dq)[NP]) {
  constexpr unsigned KP = kWave * sizeof(R);
  if (!active) return;
#pragma unroll
  for (int n = 0; n < NP; ++n) {
    const unsigned so = (c * NP + n) * KP;
    const R r = mad(k.A, resv[n], k.dt * dq[n]);
    st_nt(resw, kb, so, r);
    st_nt(qout, kb, so, mad(k.B, r, qin(c * NP + n)));
  }
}

// Wait until every vector memory operation of this wave has completed
// (vmcnt = 0; the other counters left at their maxima).
__device__ __forceinline__ void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Component C (1: u, 2: v) of the velocity volume term of quadrature
// column i: the operations velocity_volume_column performs for that
// component, in the same order, without the other component's.
template <typename R, int N, int NQ, int C, typename FP>
__device__ __forceinline__ void velocity_component_column(int i, const FP& P,
                                                          const R (&g)[4][NQ],
                                                          R (&b)[(N + 1) * (N + 1)]) {
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
  R cc[NP1];
#pragma unroll
  for (int bb = 0; bb < NP1; ++bb) cc[bb] = R(0);
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    R pr = R(0), ps = R(0);
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb) {
      pr = mad(T.V[j][bb], td[bb], pr);
      ps = mad(T.D[j][bb], tp[bb], ps);
    }
    const R G = C == 1 ? mad(g[0][j], pr, g[2][j] * ps) : mad(g[1][j], pr, g[3][j] * ps);
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb) cc[bb] = mad(T.V[j][bb], G, cc[bb]);
  }
#pragma unroll
  for (int bb = 0; bb < NP1; ++bb)
#pragma unroll
    for (int a = 0; a < NP1; ++a) b[a + NP1 * bb] = mad(-T.V[i][a], cc[bb], b[a + NP1 * bb]);
}

// The mass inverse of wadg_inverse with every accumulator formed by the
// same operations in the same order, but all quadrature columns' partial
// results computed before any is projected back: the columns' independent
// chains interleave instead of following one another, which hides the
// latency of each dependent FMA.
template <typename R, int N, int NQ>
__device__ __forceinline__ void wadg_inverse_wide(const R (&b)[(N + 1) * (N + 1)],
                                                  const R (&w)[NQ * NQ],
                                                  R (&dq)[(N + 1) * (N + 1)]) {
  constexpr ct::Ops<R, N, NQ> T = ct::make_ops<R, N, NQ>();
  constexpr int NP1 = N + 1;
  R t[NQ][NP1];
#pragma unroll
  for (int i = 0; i < NQ; ++i)
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb) {
      R acc = R(0);
#pragma unroll
      for (int a = 0; a < NP1; ++a) acc = mad(T.Vt[i][a], b[a + NP1 * bb], acc);
      t[i][bb] = acc;
    }
  R c[NQ][NP1];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb) c[i][bb] = R(0);
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      R rq = R(0);
#pragma unroll
      for (int bb = 0; bb < NP1; ++bb) rq = mad(T.Vt[j][bb], t[i][bb], rq);
      rq *= w[i + NQ * j];
#pragma unroll
      for (int bb = 0; bb < NP1; ++bb) c[i][bb] = mad(T.P[bb][j], rq, c[i][bb]);
    }
  }
#pragma unroll
  for (int n = 0; n < NP1 * NP1; ++n) dq[n] = R(0);
#pragma unroll
  for (int i = 0; i < NQ; ++i)
#pragma unroll
    for (int bb = 0; bb < NP1; ++bb)
#pragma unroll
      for (int a = 0; a < NP1; ++a) dq[a + NP1 * bb] = mad(T.P[a][i], c[i][bb], dq[a + NP1 * bb]);
}

// One workgroup's work: element group g of a state whose slice s starts at
// qin + s slice_vals (likewise qout, res, resw), slices [s0, s0 + nit); the
// group's geometry resources; the elements of the group's lanes that are
// real: e = 64 g + lane is updated iff e < kfull, or e < klast in slice
// slast (the last virtual slice of a packed batch problem, whose unused
// copies are skipped; slast = -1 otherwise).
template <typename R>
struct PipeRun {
  const R* qin;
  R* qout;
  const R* res;
  R* resw;
  size_t slice_vals;
  int g, s0, nit;
  rsrc_t vol, face, nbr;
  int kfull, slast, klast;
  // Batches: where this lane's geometry is.  A problem packed as copies of
  // a K-element mesh has the same geometry in every copy, so element
  // 64 g + lane reads that of copy 0's element e = (64 g + lane) mod K:
  //   K < 64:  in the first group at lane e; the metric rows of that group
  //            are copied whole for lanes < gelems = K, and the volume
  //            terms read them at glane = e;
  //   K >= 64: in group e / 64 at lane e % 64 (gelems = 0): this lane's
  //            values are loaded one by one into its own LDS lane
  //            (glane = lane);
  // otherwise its own group and lane (glane = lane, gelems = 64).
  // gvoff, gfoff: byte offsets of this lane's values in `vol` and `face`.
  int glane, gelems;
  unsigned gvoff, gfoff;
  unsigned res_bytes;   // bytes of a residual tile written: 0 drops the stores
  size_t goff;   // g times the values of one tile
  // offset (in values) of the group's tile in slice s
  __device__ __forceinline__ size_t grp(int s) const { return (size_t)s * slice_vals + goff; }
  // real elements of the group in slice s
  __device__ __forceinline__ int kact(int s) const {
    const int k = (s == slast ? klast : kfull) - g * kWave;
    return k < 0 ? 0 : k > kWave ? kWave : k;
  }
};

// The run is a two-stage pipeline over its items: in step j the volume and
// face waves compute item j's load vector (volume term plus the face terms
// in face order 0..3, Section 6.4) and hand it over through LDS, while the
// inverse waves apply the mass inverse and the stage update to item j - 1.
// Steps j = 0..nit, two barriers each (face terms ready; load vectors
// handed over), one barrier after the prologue.

// Face wave of faces F0 and F1: their factors and neighbour offsets held
// for the whole run, their traces gathered one item ahead.
template <typename R, int N, int NQ, int F0, int F1, bool BATCH>
__device__ __forceinline__ void pipe_face_role(const PipeRun<R>& run, const StageScalars<R>& k,
                                               int lane, unsigned kb,
                                               R (*tq)[Pipe<R, N, NQ>::tile_alloc], R* xf) {
  using L = Pipe<R, N, NQ>;
  constexpr int NP1 = L::NP1, NP = L::NP;
  constexpr unsigned KP = kWave * sizeof(R);
  const int nit = run.nit;
  auto slice = [&](int s) {
    return make_rsrc(run.qin + (size_t)s * run.slice_vals,
                     (unsigned)(run.slice_vals * sizeof(R)));
  };
  R gf0[3][NQ], gf1[3][NQ];
#pragma unroll
  for (int cc = 0; cc < 3; ++cc)
#pragma unroll
    for (int jj = 0; jj < NQ; ++jj) {
      gf0[cc][jj] = ldr<R>(run.face, BATCH ? run.gfoff : kb, (cc * 4 * NQ + F0 * NQ + jj) * KP);
      gf1[cc][jj] = ldr<R>(run.face, BATCH ? run.gfoff : kb, (cc * 4 * NQ + F1 * NQ + jj) * KP);
    }
  NbrOffsets nbo;
  load_nbr(run.nbr, lane, nbo);
  Trace<R, N> tr0, tr1;
  gather_trace<R, N>(slice(run.s0), nbo, F0, tr0);
  gather_trace<R, N>(slice(run.s0), nbo, F1, tr1);
  __syncthreads();                                           // prologue done
  for (int it = 0; it <= nit; ++it) {
    if (it < nit) {
      const R* t = tq[it & 1];
      auto Pt = [&](int n) { return t[n * kWave + lane]; };
      auto Ut = [&](int n) { return t[(NP + n) * kWave + lane]; };
      auto Vt = [&](int n) { return t[(2 * NP + n) * kWave + lane]; };
      auto face = [&](int F, const Trace<R, N>& tr, const R (&gf)[3][NQ]) {
        R sp[NP1], su[NP1], sv[NP1];
        face_terms<R, N, NQ, true, true>(F, Pt, Ut, Vt, tr, gf, k.tau_p, k.tau_u, sp, su, sv);
#pragma unroll
        for (int m = 0; m < NP1; ++m) {
          xf[((F * 3 + 0) * NP1 + m) * kWave + lane] = sp[m];
          xf[((F * 3 + 1) * NP1 + m) * kWave + lane] = su[m];
          xf[((F * 3 + 2) * NP1 + m) * kWave + lane] = sv[m];
        }
      };
      face(F0, tr0, gf0);
      face(F1, tr1, gf1);
      if (it + 1 < nit) {
        gather_trace<R, N>(slice(run.s0 + it + 1), nbo, F0, tr0);
        gather_trace<R, N>(slice(run.s0 + it + 1), nbo, F1, tr1);
      }
    }
    __syncthreads();                                         // face terms ready
    __syncthreads();                                         // load vectors handed over
  }
}

// Volume wave of field C (0: p, 1: u, 2: v): the pressure term, or one
// component of the velocity term, of item j; once the face terms are in
// LDS it adds them in face order 0..3 and hands the load vector over (xb).
// The v wave also loads the next item's tile (LOADER).
template <typename R, int N, int NQ, int C, bool LOADER, bool BATCH>
__device__ __forceinline__ void pipe_volume_role(const PipeRun<R>& run, int lane,
                                                 R (*tq)[Pipe<R, N, NQ>::tile_alloc],
                                                 const R* xm, const R* xf, R* xb) {
  using L = Pipe<R, N, NQ>;
  constexpr int NP1 = L::NP1, NP = L::NP, NQ2 = L::NQ2;
  const int nit = run.nit;
  auto tile_src = [&](int s) { return make_rsrc(run.qin + run.grp(s), L::tile_bytes); };
  // (batches: only the rows' values of the slice's real elements)
  auto tile_in = [&](int s, R* dst) {
    if (!BATCH || row_lane_needed(lane, run.kact(s))) tile_to_lds<L::rows>(tile_src(s), dst, lane);
  };
  if constexpr (LOADER) tile_in(run.s0, tq[0]);
  wait_vm_all();                                             // metric rows (and tile) in LDS
  __syncthreads();                                           // prologue done
  for (int it = 0; it <= nit; ++it) {
    R b[NP];
    if (it < nit) {
      if constexpr (LOADER) {
        if (it + 1 < nit) tile_in(run.s0 + it + 1, tq[(it + 1) & 1]);
      }
      const R* t = tq[it & 1];
      // the nodal values the volume term reads, in registers for all of its
      // columns: u and v (pressure), p (velocity)
      R x0[NP], x1[C == 0 ? NP : 1];
#pragma unroll
      for (int n = 0; n < NP; ++n) {
        x0[n] = t[((C == 0 ? NP : 0) + n) * kWave + lane];
        if constexpr (C == 0) x1[n] = t[(2 * NP + n) * kWave + lane];
      }
      auto X0 = [&](int n) { return x0[n]; };
      auto X1 = [&](int n) { return x1[n]; };
#pragma unroll
      for (int n = 0; n < NP; ++n) b[n] = R(0);
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        // this column's metric terms, requested before its first products
        // (which need only the nodal values) so that they arrive meanwhile
        R gc[4][NQ];
        order();
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int jj = 0; jj < NQ; ++jj)
            if (C == 0 || q == C - 1 || q == C + 1)
              gc[q][jj] = xm[(q * NQ2 + i + NQ * jj) * kWave + (BATCH ? run.glane : lane)];
            else
              gc[q][jj] = R(0);
        if constexpr (C == 0)
          pressure_volume_column<R, N, NQ>(i, X0, X1, gc, b);
        else
          velocity_component_column<R, N, NQ, C>(i, X0, gc, b);
        pin(b);
      }
    }
    __syncthreads();                                         // face terms ready
    if (it < nit) {
#pragma unroll
      for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int m = 0; m < NP1; ++m)
          b[fnode<N>(f, m)] += xf[((f * 3 + C) * NP1 + m) * kWave + lane];
#pragma unroll
      for (int n = 0; n < NP; ++n) xb[(C * NP + n) * kWave + lane] = b[n];
    }
    if constexpr (LOADER) wait_vm_all();                     // next tile in LDS
    __syncthreads();                                         // load vectors handed over
  }
}

// Inverse wave of field C: in step j the mass inverse and the stage update
// of item j - 1 from the handed-over load vector, with mass weights c^2/J
// (times the c^2 scale; LDS) or 1/J (registers), the residual requested one
// item ahead, and the item's input values of the field kept in registers
// from the step before (the tile buffer is refilled meanwhile).  RD: the
// residual is not stored (the last stage of a step); NT: the outputs are
// stored with the non-temporal hint.
template <typename R, int N, int NQ, int C, bool RD, bool NT, bool BATCH>
__device__ __forceinline__ void pipe_inverse_role(const PipeRun<R>& run, const StageScalars<R>& k,
                                                  int lane, unsigned kb,
                                                  R (*tq)[Pipe<R, N, NQ>::tile_alloc],
                                                  const R* xb, R* xw) {
  using L = Pipe<R, N, NQ>;
  constexpr int NP = L::NP, NQ2 = L::NQ2;
  constexpr unsigned tile = L::tile;
  constexpr unsigned KP = kWave * sizeof(R);
  const int s0 = run.s0, nit = run.nit;
  const rsrc_t vol = run.vol;
  const int e = run.g * kWave + lane;
  auto grp = [&](int s) { return run.grp(s); };
  R wq[C == 0 ? 1 : NQ2];
  if constexpr (C == 0) {
#pragma unroll
    for (int q = 0; q < NQ2; ++q)
      xw[q * kWave + lane] = ldr<R>(vol, BATCH ? run.gvoff : kb, (4 * NQ2 + q) * KP) * k.c2s;
  } else {
#pragma unroll
    for (int q = 0; q < NQ2; ++q) wq[q] = ldr<R>(vol, BATCH ? run.gvoff : kb, (5 * NQ2 + q) * KP);
  }
  R resv[NP], qv[NP];
  load_res<R, NP, kStage>(k, make_rsrc(run.res + grp(s0), tile * sizeof(R)), C, kb, resv);
  if constexpr (C == 0) wait_vm_all();                       // metric rows in LDS
  __syncthreads();                                           // prologue done
  for (int it = 0; it <= nit; ++it) {
    if (it > 0) {
      const int s = s0 + it - 1;
      R b[NP];
#pragma unroll
      for (int n = 0; n < NP; ++n) b[n] = xb[(C * NP + n) * kWave + lane];
      R dq[NP];
      if constexpr (C == 0) {
        R wl[NQ2];
#pragma unroll
        for (int q = 0; q < NQ2; ++q) wl[q] = xw[q * kWave + lane];
        wadg_inverse_wide<R, N, NQ>(b, wl, dq);
      } else {
        wadg_inverse_wide<R, N, NQ>(b, wq, dq);
      }
      const rsrc_t qo = make_rsrc(run.qout + grp(s), tile * sizeof(R));
      const rsrc_t rw = make_rsrc(run.resw + grp(s), run.res_bytes);
      const bool active = e < (s == run.slast ? run.klast : run.kfull);
      auto Qv = [&](int n) { return qv[n - C * NP]; };
      if constexpr (!RD) {
        if constexpr (NT)
          finish_field_nt<R, NP>(k, qo, rw, Qv, C, kb, active, resv, dq);
        else
          finish_field<R, NP, kStage>(k, qo, rw, Qv, C, kb, active, resv, dq);
      } else if (active) {
        // finish_field's arithmetic without the residual's stores
#pragma unroll
        for (int n = 0; n < NP; ++n) {
          const R r = mad(k.A, resv[n], k.dt * dq[n]);
          const R q = mad(k.B, r, qv[n]);
          if constexpr (NT)
            st_nt(qo, kb, (C * NP + n) * KP, q);
          else
            st(qo, kb, (C * NP + n) * KP, q);
        }
      }
      // the next item's residual; in a first stage (A = 0) resv keeps the
      // zeros the prologue gave it (batches: only for real elements)
      if (it < nit && k.A != R(0) && (!BATCH || lane < run.kact(s + 1))) {
        const rsrc_t rn = make_rsrc(run.res + grp(s + 1), tile * sizeof(R));
#pragma unroll
        for (int n = 0; n < NP; ++n)
          resv[n] = NT ? ldr_nt<R>(rn, kb, (C * NP + n) * KP) : ldr<R>(rn, kb, (C * NP + n) * KP);
      }
    }
    if (it < nit) {
      // item it's input values of this field, before its buffer is refilled
      const R* t = tq[it & 1];
#pragma unroll
      for (int n = 0; n < NP; ++n) qv[n] = t[(C * NP + n) * kWave + lane];
    }
    __syncthreads();                                         // face terms ready
    __syncthreads();                                         // load vectors handed over
  }
}

// One run over the eight waves of the workgroup, on the workgroup's LDS
// arrays (Pipe<>).  Wave w runs on SIMD w mod 4: waves 0..2 the volume
// terms of p, u, v (wave 2 also loads the tiles), waves 3, 5, 6 the mass
// inverses and updates of p, u, v, waves 4 and 7 the faces 0, 1 and 2, 3.
template <typename R, int N, int NQ, bool RD, bool NT, bool BATCH>
__device__ __forceinline__ void pipe_run(const PipeRun<R>& run, const StageScalars<R>& k,
                                         R (*tq)[Pipe<R, N, NQ>::tile_alloc], R* xm, R* xf,
                                         R* xb, R* xw) {
  using L = Pipe<R, N, NQ>;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & (kWave - 1);
  const unsigned kb = (unsigned)lane * sizeof(R);

  // prologue: metric planes 0..3 of the group into LDS by waves 0..3 (the
  // face waves gather their first traces meanwhile)
  if (wave <= 3) {
    const int w = wave;
    if (!BATCH || run.gelems > 0) {
      if (!BATCH || row_lane_needed(lane, run.gelems))
        rows_to_lds<L::metric_rows>(run.vol, xm, w, 4, lane);
    } else {
      constexpr unsigned KP = kWave * sizeof(R);
      for (int pp = w; pp < 4 * L::NQ2; pp += 4)
        xm[pp * kWave + lane] = ldr<R>(run.vol, run.gvoff, (unsigned)pp * KP);
    }
  }
  // Issue priority between the waves of a SIMD (s_setprio): the inverse
  // waves, which issue each item's stores and residual loads, first; then
  // the pressure volume wave, the longest role; then the velocity volume
  // waves; the face waves keep the default.
  if (wave == 0) __builtin_amdgcn_s_setprio(2);
  if (wave == 1) __builtin_amdgcn_s_setprio(1);
  if (wave == 2) __builtin_amdgcn_s_setprio(1);
  if (wave == 3) __builtin_amdgcn_s_setprio(3);
  if (wave == 5) __builtin_amdgcn_s_setprio(3);
  if (wave == 6) __builtin_amdgcn_s_setprio(3);
  if (wave == 0) {
    pipe_volume_role<R, N, NQ, 0, false, BATCH>(run, lane, tq, xm, xf, xb);
  } else if (wave == 1) {
    pipe_volume_role<R, N, NQ, 1, false, BATCH>(run, lane, tq, xm, xf, xb);
  } else if (wave == 2) {
    pipe_volume_role<R, N, NQ, 2, true, BATCH>(run, lane, tq, xm, xf, xb);
  } else if (wave == 3) {
    pipe_inverse_role<R, N, NQ, 0, RD, NT, BATCH>(run, k, lane, kb, tq, xb, xw);
  } else if (wave == 5) {
    pipe_inverse_role<R, N, NQ, 1, RD, NT, BATCH>(run, k, lane, kb, tq, xb, xw);
  } else if (wave == 6) {
    pipe_inverse_role<R, N, NQ, 2, RD, NT, BATCH>(run, k, lane, kb, tq, xb, xw);
  } else if (wave == 4) {
    pipe_face_role<R, N, NQ, 0, 1, BATCH>(run, k, lane, kb, tq, xf);
  } else {
    pipe_face_role<R, N, NQ, 2, 3, BATCH>(run, k, lane, kb, tq, xf);
  }
}

}  // namespace

// Workgroup b: element group g and slices [s0, s1) of one problem;
// grid = nEG * chunks, chunk j of group g holds slices
// [j S / chunks, (j + 1) S / chunks).  LSRK stage mode only; RD = p.res_dead
// (the last stage of a step, a kernel of its own so that the other stages'
// code is not shaped by the branch); NT: non-temporal stores (launches
// whose state is far larger than the caches).
template <typename R, int N, int NQ, bool RD, bool NT>
__global__ __launch_bounds__(8 * kWave) void pipe_kernel(const StageParams p, int chunks) {
  using L = Pipe<R, N, NQ>;
  constexpr int NQ2 = L::NQ2;
  constexpr unsigned KP = kWave * sizeof(R);
  __shared__ __attribute__((aligned(1024))) R tq[2][L::tile_alloc];
  __shared__ __attribute__((aligned(16))) R xm[L::metric];
  __shared__ __attribute__((aligned(16))) R xf[L::xf];
  __shared__ __attribute__((aligned(16))) R xb[L::xb];
  __shared__ __attribute__((aligned(16))) R xw[L::wp];

  // workgroup -> (group, slice run), XCD-aware: each XCD takes a
  // contiguous range of groups, so most neighbour traces are read by
  // workgroups of the same XCD
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  const int g = w / chunks, j = w - g * chunks;
  if (g >= p.nEG) return;                 // whole workgroup: no barrier reached
  const int s0 = (int)((int64_t)j * p.S / chunks);
  const int s1 = (int)((int64_t)(j + 1) * p.S / chunks);
  if (s1 <= s0) return;
  PipeRun<R> run;
  run.qin = static_cast<const R*>(p.Qin);
  run.qout = static_cast<R*>(p.Qout);
  run.res = static_cast<const R*>(p.res);
  run.resw = static_cast<R*>(p.res_out ? p.res_out : p.res);
  run.slice_vals = (size_t)p.nEG * L::tile;
  run.g = g;
  run.goff = (size_t)g * L::tile;
  run.s0 = s0;
  run.nit = s1 - s0;
  run.vol = make_rsrc(static_cast<const R*>(p.vol) + (size_t)g * 6 * NQ2 * kWave, 6u * NQ2 * KP);
  run.face = make_rsrc(static_cast<const R*>(p.face) + (size_t)g * 12 * NQ * kWave, 12u * NQ * KP);
  run.nbr = make_rsrc(p.nbr + (size_t)g * 8 * kWave, 8u * kWave * 4u);
  run.kfull = p.K;
  run.slast = -1;
  run.klast = p.K;
  run.glane = 0;                          // (batches only)
  run.gelems = kWave;
  run.gvoff = run.gfoff = 0;
  run.res_bytes = RD ? 0u : L::tile * sizeof(R);
  pipe_run<R, N, NQ, RD, NT, false>(run, stage_scalars<R>(p), tq, xm, xf, xb, xw);
}

// Batched LSRK stage (FP64) over a list of runs of many independent
// problems: run r = (problem, element group of its virtual mesh, first
// virtual slice, slice count) for workgroup r (problem -1: nothing to do;
// the list is laid out for the XCD each workgroup lands on).  The problem's
// descriptor supplies the state offset, geometry groups and dt, and the
// real element count of every virtual slice (unused copies of a packed
// last slice are not written).  RD, NT as for pipe_kernel.
template <int N, int NQ, bool RD, bool NT>
__global__ __launch_bounds__(8 * kWave) void batch_pipe_kernel(const BatchParams bp,
                                                               const int32_t* runs, int nruns) {
  using R = double;
  using L = Pipe<R, N, NQ>;
  constexpr int NQ2 = L::NQ2;
  constexpr unsigned KP = kWave * sizeof(R);
  __shared__ __attribute__((aligned(1024))) R tq[2][L::tile_alloc];
  __shared__ __attribute__((aligned(16))) R xm[L::metric];
  __shared__ __attribute__((aligned(16))) R xf[L::xf];
  __shared__ __attribute__((aligned(16))) R xb[L::xb];
  __shared__ __attribute__((aligned(16))) R xw[L::wp];
  const int r = blockIdx.x;
  if (r >= nruns || runs[4 * r] < 0) return;   // whole workgroup: no barrier reached
  const int pi = runs[4 * r], g = runs[4 * r + 1];
  const BatchProb pr = bp.prob[pi];
  PipeRun<R> run;
  run.qin = bp.Qin + pr.qoff;
  run.qout = bp.Qout + pr.qoff;
  run.res = bp.res + pr.qoff;
  run.resw = bp.res + pr.qoff;
  run.slice_vals = (size_t)pr.nEG * L::tile;
  run.g = g;
  run.goff = (size_t)g * L::tile;
  run.s0 = runs[4 * r + 2];
  run.nit = runs[4 * r + 3];
  const size_t gg = (size_t)pr.g0 + g;
  // a problem of fewer than 64 elements has the same geometry in every
  // copy: every group reads its first group's (which holds copy 0 in lanes
  // 0..K-1) at lane (64 g + lane) mod K, shared through the cache
  const int lane = threadIdx.x & (kWave - 1);
  const int ec = pr.kc ? (g * kWave + lane) % pr.kc : lane;   // copy 0's element
  const unsigned gvs = 6u * NQ2 * KP, gfs = 12u * NQ * KP;     // bytes per group
  const size_t gv = pr.kc ? (size_t)pr.g0 : gg;
  const unsigned ngv = pr.kc ? (unsigned)(pr.kc + kWave - 1) / kWave : 1u;
  if (pr.kc == 0 || pr.kc >= kWave) {
    run.glane = lane;
    run.gelems = pr.kc ? 0 : kWave;
    run.gvoff = (unsigned)(ec / kWave) * gvs + (unsigned)(ec % kWave) * sizeof(R);
    run.gfoff = (unsigned)(ec / kWave) * gfs + (unsigned)(ec % kWave) * sizeof(R);
  } else {
    run.glane = ec;
    run.gelems = pr.kc;
    run.gvoff = run.gfoff = (unsigned)ec * sizeof(R);
  }
  run.vol = make_rsrc(bp.vol + gv * 6 * NQ2 * kWave, ngv * gvs);
  run.face = make_rsrc(bp.face + gv * 12 * NQ * kWave, ngv * gfs);
  run.nbr = make_rsrc(bp.nbr + gg * 8 * kWave, 8u * kWave * 4u);
  run.kfull = pr.K;
  run.slast = pr.S - 1;
  run.klast = pr.klast;
  run.res_bytes = RD ? 0u : L::tile * sizeof(R);
  StageScalars<R> k;
  k.tau_p = bp.tau_p;
  k.tau_u = bp.tau_u;
  k.A = bp.rkA;
  k.B = bp.rkB;
  k.dt = pr.dt;
  k.c2s = 1.0;
  pipe_run<R, N, NQ, RD, NT, true>(run, k, tq, xm, xf, xb, xw);
}

namespace {

// Non-temporal stores where a launch's state (Q_in, Q_out and the residual:
// three times `bytes`, one array) is well beyond the 256 MB memory-side
// cache; below that the next launch may still find what this one wrote.
// Measured on MI355X, 128x128 elements x 256 slices (4.8 GB): about 1 %
// faster per launch in FP64 and FP32, results unchanged.
bool nt_stores(int64_t bytes) { return 3 * bytes > (int64_t)512 << 20; }

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
    // two workgroups per CU where two fit in LDS (16 waves of at most 128
    // registers: FP32), else one
    const int per_cu = Pipe<R, N, NQ>::lds_bytes <= 80u * 1024u ? 2 : 1;
    const int chunks = pipe_chunks(p.nEG, p.S, cus * per_cu);
    if ((int64_t)p.nEG * chunks >= (1LL << 31)) return (int)hipErrorInvalidValue;
    const dim3 grid(p.nEG * chunks), block(8 * kWave);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (nt_stores((int64_t)p.S * p.nEG * Pipe<R, N, NQ>::tile_bytes)) {
      if (p.res_dead)
        hipLaunchKernelGGL((pipe_kernel<R, N, NQ, true, true>), grid, block, 0, st, p, chunks);
      else
        hipLaunchKernelGGL((pipe_kernel<R, N, NQ, false, true>), grid, block, 0, st, p, chunks);
    } else {
      if (p.res_dead)
        hipLaunchKernelGGL((pipe_kernel<R, N, NQ, true, false>), grid, block, 0, st, p, chunks);
      else
        hipLaunchKernelGGL((pipe_kernel<R, N, NQ, false, false>), grid, block, 0, st, p, chunks);
    }
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

namespace {

template <int N, int NQ>
int launch_batch_nq(const BatchParams& p, const int32_t* runs, int32_t nruns, void* stream) {
  if constexpr (!Pipe<double, N, NQ>::fits) {
    return (int)hipErrorInvalidValue;
  } else {
    const dim3 grid(nruns), block(8 * kWave);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (nt_stores((int64_t)p.nitems * Pipe<double, N, NQ>::tile_bytes)) {
      if (p.res_dead)
        hipLaunchKernelGGL((batch_pipe_kernel<N, NQ, true, true>), grid, block, 0, st, p, runs, nruns);
      else
        hipLaunchKernelGGL((batch_pipe_kernel<N, NQ, false, true>), grid, block, 0, st, p, runs,
                           nruns);
    } else {
      if (p.res_dead)
        hipLaunchKernelGGL((batch_pipe_kernel<N, NQ, true, false>), grid, block, 0, st, p, runs,
                           nruns);
      else
        hipLaunchKernelGGL((batch_pipe_kernel<N, NQ, false, false>), grid, block, 0, st, p, runs,
                           nruns);
    }
    return (int)hipGetLastError();
  }
}

template <int N>
int launch_batch_n(int nq, const BatchParams& p, const int32_t* runs, int32_t nruns,
                   void* stream) {
  switch (nq - N) {
    case 1: return launch_batch_nq<N, N + 1>(p, runs, nruns, stream);
    case 2: return launch_batch_nq<N, N + 2>(p, runs, nruns, stream);
    case 3: return launch_batch_nq<N, N + 3>(p, runs, nruns, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace

bool batch_pipe_supported(int N, int nq) { return pipe_supported(N, nq, false); }

int launch_batch_pipe(int N, int nq, const BatchParams& p, const int32_t* runs, int32_t nruns,
                      void* stream) {
  if (nruns <= 0) return 0;
  switch (N) {
    case 1: return launch_batch_n<1>(nq, p, runs, nruns, stream);
    case 2: return launch_batch_n<2>(nq, p, runs, nruns, stream);
    case 3: return launch_batch_n<3>(nq, p, runs, nruns, stream);
    case 4: return launch_batch_n<4>(nq, p, runs, nruns, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_stage_pipe(int N, int nq, const StageParams& p, int cus, void* stream) {
  return launch_r<double>(N, nq, p, cus, stream);
}

int launch_stage_pipe_fp32(int N, int nq, const StageParams& p, int cus, void* stream) {
  return launch_r<float>(N, nq, p, cus, stream);
}

}  // namespace wadg
