// Internal declarations shared by the host setup, the kernels and the C ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace wadg {

constexpr int kMaxNp1 = 5;   // N <= 4
constexpr int kMaxNq = 7;    // nq1 <= N + 3
constexpr int kWave = 64;    // elements per workgroup: one element per lane

// 1D reference operators of the tensor-product nodal basis.  All 2D
// operators are tensor products of these (the reference square is a tensor
// product and the GLL nodal basis is l_a(r) l_b(s)).
//   V[i][a]  = l_a(x_i)                 Lagrange basis at Gauss points
//   D[i][a]  = l_a'(x_i)
//   Vt[i][a] = (V M1^{-1})[i][a]        interpolation of Mhat^{-1} b
//   P[a][i]  = (M1^{-1} V^T W)[a][i]    quadrature-based L2 projection
// with M1 the 1D nodal mass matrix.  Section 6.2 defines V_q and
// P_q = Mhat^{-1} V_q^T diag(w_q); Mhat = M1 (x) M1 and V_q = V (x) V.
struct RefOps {
  int N = 0, nq = 0;
  double xg[kMaxNp1] = {};
  double xq[kMaxNq] = {}, wq[kMaxNq] = {};
  double V[kMaxNq][kMaxNp1] = {};
  double D[kMaxNq][kMaxNp1] = {};
  double Vt[kMaxNq][kMaxNp1] = {};
  double P[kMaxNp1][kMaxNq] = {};
};

// Build the 1D operators for degree N and an nq-point Gauss rule.
bool build_ref_ops(int N, int nq, RefOps* ops, std::string* err);

struct MeshIn {
  int N, nq1, K;
  const double *x, *y;
  const int32_t *etoe, *etof;
  const double* c2q;
};

// Host geometry arrays, P planes of K values each:
//   vol  P = 6 nq^2   W ys, -W xs, -W yr, W xr, c2/J, 1/J at each point
//   face P = 12 nq    nx, ny, w sJ for each face and point
//   nbr  P = 8        offset (in values), within one slice of the tiled
//                     state layout, of the neighbour's value at my face
//                     node 0 (field 0), and the step along my face parameter
// written into caller-owned arrays (any may be NULL) either untiled,
// [P][K] (element index fastest), or tiled, [G][P][64] with G = ceil(K/64)
// and the padding lanes of the last group zero (the device layout).  On
// failure the contents are unspecified.  Runs on the host's threads.
int build_geometry(const MeshIn& m, const RefOps& ops, double* vol, double* face,
                   int32_t* nbr, bool tiled, std::string* err);

// Physical coordinates of the volume quadrature points, [K][nq*nq].
void quadrature_points(const MeshIn& m, const RefOps& ops, double* xq, double* yq);

// The adjoint mass step of the next reverse stage, fused into an apply-A
// launch (mode kApplyAMass; split kernel, FP64).  With y the new ybar:
//   rbar <- a_next rbar + b y;   z <- D Mtilde^{-1} rbar;
//   part[group] += sum over pressure values of rbar (r - a r_prev).
struct AdjMassParams {
  double* rbar;           // one slice, read (unless a_next = 0) and written
  double* z;              // one slice, written; not the launch's Qin
  const double* r;        // stage residual r_i of the mass stage
  const double* r_prev;   // r_{i-1}; NULL when a = 0
  double* part;           // [groups] sensitivity partials
  double a_next, b, a;
};

// Arrays are of the kernel's arithmetic type (double, or float for the
// FP32-bulk propagator) except the int32 neighbour offsets.
struct StageParams {
  const void* Qin;       // [S][G][3][Np][64]
  void* Qout;            // [S][G][3][Np][64]  (rhs mode: dQ/dt; adjoint mode: ybar out)
  void* res;             // [S][G][3][Np][64]  LSRK residual read (stage mode; adjoint
                         //                    mode: ybar in)
  void* res_out;         // residual written (stage mode); NULL: same as res
  const void* vol;       // [G][6][Nq][64]
  const void* face;      // [G][3][4][nq][64]
  const int32_t* nbr;    // [G][2][4][64]
  int32_t K, S, nEG;
  int32_t tile_groups, tile_slices;   // schedule tile (clamped to nEG, S)
  double tau_p, tau_u;
  double rkA, rkB, dt;
  double c2_scale;       // c^2 multiplier (pressure mass weights)
  int32_t reverse;       // nonzero: the work items in reverse order
  int32_t res_dead;      // nonzero (stage mode): the residual this stage writes is never
                         // read -- the last stage of a step, the next step starting with
                         // A = 0 -- so the kernel may drop its store
  AdjMassParams adj;     // kApplyAMass only
};

// What a stage-kernel launch computes from the load vector b = A Qin:
//   kStage   LSRK stage: res_out <- A res + dt M^-1 b; Qout <- Qin + B res_out
//   kRhs     Qout <- M^-1 b
//   kApplyA  adjoint stage part: Qout <- res + dt D b, D = diag(1, -1, -1)
//            (no mass inverse; streamed and split kernels)
//   kApplyAMass  kApplyA, then the next reverse stage's mass step on the
//            new Qout (AdjMassParams; split kernel, FP64)
enum StageMode { kStage = 0, kRhs = 1, kApplyA = 2, kApplyAMass = 3 };

// Launch one stage (rhs == false: LSRK stage update; rhs == true: write
// dQ/dt to Qout).  Returns a hipError_t as int.
//
// Streamed-geometry kernel: one workgroup per (slice, element group), the
// group's geometry read from global memory; every supported (N, nq).
int launch_stage_streamed(int N, int nq, int mode, const StageParams& p, void* stream);
// The same LSRK stage in FP32 (arrays of float).
int launch_stage_streamed_fp32(int N, int nq, const StageParams& p, void* stream);
// Split-work kernel: the streamed kernel's work item spread over four
// waves (volume p, volume u/v, faces 0+2, faces 1+3); stage and rhs modes.
int launch_stage_split(int N, int nq, int mode, const StageParams& p, void* stream);
int launch_stage_split_fp32(int N, int nq, const StageParams& p, void* stream);
// Split-work kernel over two independent launches in one grid (FP64): the
// items of launch a in mode_a (kApplyA or kApplyAMass), then the LSRK stage
// items of launch b; each item as in its own launch.
int launch_stage_pair(int N, int nq, int mode_a, const StageParams& a, const StageParams& b,
                      void* stream);
// Resident-geometry kernel: one workgroup per (element group, slice range)
// with the group's geometry held in LDS; grid = nEG * ranges.  Only where
// resident_supported(N, nq, fp32).
bool resident_supported(int N, int nq, bool fp32);
int resident_ranges(int nEG, int S, int cus);
int launch_stage_resident(int N, int nq, int mode, const StageParams& p, int ranges,
                          void* stream);
// Adjoint mass step, elementwise (one workgroup per (slice, element group)):
//   rbar <- a rbar + b ybar   (rbar not read when a == 0)
//   z    <- D Mtilde^-1 rbar  (WADG inverse per field, c2_scale on p)
//   part[w] += sum over p entries of rbar * (r_i - a_i r_prev)   (r_prev not
//            read when a_i == 0), w = slice * nEG + group, one slot per workgroup
int launch_adjoint_mass(int N, int nq, const StageParams& p, double* rbar, const double* ybar,
                        double* z, const double* r_i, const double* r_prev, double a_next,
                        double b_i, double a_i, double* part, void* stream);
int launch_stage_resident_fp32(int N, int nq, const StageParams& p, int ranges, void* stream);
// Elementwise precision conversion of n values (FP64 <-> FP32).
int launch_to_fp32(const double* in, float* out, size_t n, void* stream);
int launch_to_fp64(const float* in, double* out, size_t n, void* stream);
// Device copy of n doubles as a kernel (capture-safe; no runtime copy node).
int launch_copy(const double* in, double* out, size_t n, void* stream);
bool stage_supported(int N, int nq);
// Persistent pipelined kernel (pipe_kernel.hip): one eight-wave workgroup
// per (element group, slice run), grid = nEG * chunks with chunks chosen
// from the CU count; LSRK stage mode only, where its LDS fits.
bool pipe_supported(int N, int nq, bool fp32);
int launch_stage_pipe(int N, int nq, const StageParams& p, int cus, void* stream);
int launch_stage_pipe_fp32(int N, int nq, const StageParams& p, int cus, void* stream);

// Batched stage over many independent problems (same N, nq, penalties):
// one work item = one 64-element group of one slice of one problem.
struct BatchProb {
  int64_t qoff;          // first value of the problem in the batch state arrays
  int32_t nEG, S, K;     // element groups per slice, slices, elements (lanes in use)
  int32_t g0;            // first element group of the problem in the geometry arrays
  int32_t klast;         // elements holding real slices in the last (virtual) slice
  int32_t kc;            // copies of a K-element mesh (or K < 64): K, and every group
                         // reads copy 0's geometry (the first groups); else 0
  double dt;
};
struct BatchParams {
  const BatchProb* prob;
  const int32_t* items;  // [nitems][2]: problem, slice * nEG + group
  int32_t nitems;
  const double* Qin;
  double* Qout;
  double* res;
  const double* vol;     // [all groups][6][Nq][64]
  const double* face;    // [all groups][3][4][nq][64]
  const int32_t* nbr;    // [all groups][2][4][64]
  double tau_p, tau_u, rkA, rkB;
  int32_t res_dead;      // as StageParams::res_dead
};
// Streamed kernel, persistent two-wave workgroups: grid = number of
// workgroups (each loops over items with stride grid), or nitems for one
// workgroup per item.
int launch_batch_stage(int N, int nq, const BatchParams& p, int grid, void* stream);
// Split-work kernel, one four-wave workgroup per item.
int launch_batch_split(int N, int nq, const BatchParams& p, void* stream);
// Pipelined kernel (FP64), one eight-wave workgroup per run: runs[4 r ..] =
// (problem, element group, first virtual slice, slice count); items are not
// read from p.items.  Only where batch_pipe_supported(N, nq).
bool batch_pipe_supported(int N, int nq);
int launch_batch_pipe(int N, int nq, const BatchParams& p, const int32_t* runs, int32_t nruns,
                      void* stream);

// Per-slice norms over the tiled layout (padding skipped): partial sums into
// `partials` [S][nblk][4] then a fixed-order reduction into `out` [S][4].
int launch_norms(const double* A, const double* B, int32_t S, int64_t n_per_slice, int32_t tile,
                 int32_t K, double* partials, int nblk, double* out, void* stream);

// Per-slice L2 norms with the Jacobian (l2_kernel.hip): item partials into
// `partials` [S * nEG][2], then per slice out[s] = (||A_s - B_s||^2,
// ||B_s||^2) [S][2] (squares); B may be NULL.
int launch_l2_norms(int N, int nq, const double* A, const double* B, const double* vol,
                    int32_t S, int32_t nEG, int32_t K, double* partials, double* out,
                    void* stream);

// Second pass of a per-slice reduction: partials [S][nblk][4] -> out [S][4].
int launch_norms_final(const double* partials, int nblk, int32_t S, double* out, void* stream);

// Parareal correction of one slice (see parareal_kernel.hip); writes block
// partials [nblk][4] of ||change||^2, ||new||^2, max |change|, non-finite.
int launch_parareal_correct(const double* g, const double* f, double* gold, double* u,
                            int64_t n, int32_t tile, int32_t K, double* partials, int nblk,
                            void* stream);

}  // namespace wadg
