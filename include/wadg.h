/*
 * wadg.h -- C ABI of the MI355X (gfx950) weight-adjusted discontinuous
 * Galerkin (WADG) sweep for the acoustic wave equation on curvilinear
 * quadrilateral meshes.
 *
 * Method (Chan, Hewett, Warburton, "Weight-adjusted discontinuous Galerkin
 * methods: curvilinear meshes"):
 *   - semi-discrete system  M dQ/dt = A_h Q  with M block diagonal,
 *     blocks M_{J^k}  (Section 4, opening);
 *   - A_h Q is the strong-weak DG form of the first-order acoustic system,
 *     rho = 1, penalties tau_p, tau_u (Section 4.1, equations of the
 *     strong-weak formulation; Section 6.4 for its volume/surface terms);
 *   - the mass inverse is replaced by the weight-adjusted approximation
 *       M_{J}^{-1}     ~ Mhat^{-1} M_{1/J}   Mhat^{-1}   (velocity),
 *       M_{J/c2}^{-1}  ~ Mhat^{-1} M_{c2/J}  Mhat^{-1}   (pressure),
 *     applied matrix-free as P_q diag(w_q) V_q  (Section 4; Section 6.2,
 *     equation of the matrix-free product; Section 7 for heterogeneous c2);
 *   - time stepping by the low-storage five-stage fourth-order Runge-Kutta
 *     scheme (Section 5.2).
 * The system is autonomous, so no start time is needed: a slice is advanced
 * by nsteps steps of size dt from the state it holds.
 *
 * Discretisation on the boundary:
 *   reference square [-1,1]^2, tensor space Q^N; nodal basis at the
 *   (N+1)^2 Gauss-Lobatto-Legendre (GLL) points, local node
 *   n = a + (N+1) b (a along r, b along s); nq1-point Gauss-Legendre rule
 *   per direction for volume integrals and per face for surface integrals.
 *   Faces: 0: s=-1 (parameter r), 1: r=+1 (s), 2: s=+1 (r), 3: r=-1 (s).
 *
 * State layout (device, caller-owned, float64, C-contiguous), tiled by
 * groups of 64 elements:
 *   Q[s][g][f][n][l]   slice s in [0,S), element group g in [0,G) with
 *                      G = ceil(K/64), field f in {p, u, v}, node n in
 *                      [0,(N+1)^2), lane l in [0,64); element k = 64 g + l.
 * One slice holds G*3*(N+1)^2*64 doubles; entries with 64 g + l >= K are
 * padding: never read as state, ignored by the reductions, unspecified on
 * output.
 * wadg_state_doubles() gives the per-slice count.
 *
 * Errors: every int-returning call returns WADG_OK (0) or a negative code.
 * Arguments are validated before any HIP call.  wadg_last_error() gives a
 * thread-local message for the last failure.  Nothing throws across the ABI.
 *
 * Threading: a context may be used from one host thread at a time.  Calls
 * on one context that run on different streams must not overlap in time.
 */
#ifndef WADG_H
#define WADG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WADG_OK 0
#define WADG_E_INVALID (-1)     /* null pointer, bad size or range          */
#define WADG_E_GEOMETRY (-2)    /* J <= 0, non-finite or non-conforming mesh */
#define WADG_E_UNSUPPORTED (-3) /* degree / quadrature not compiled in      */
#define WADG_E_DEVICE (-4)      /* HIP runtime error (see wadg_last_error)  */
#define WADG_E_NONFINITE (-5)   /* a result contains Inf or NaN             */

#define WADG_MAX_N 4            /* degrees 1..4 are compiled in            */

/* Stage-kernel variants (wadg_set_kernel). */
#define WADG_KERNEL_AUTO 0      /* the fastest measured per launch kind     */
#define WADG_KERNEL_STREAMED 1  /* geometry read from global memory per item */
#define WADG_KERNEL_RESIDENT 2  /* geometry held in LDS per element group    */
#define WADG_KERNEL_SPLIT 3     /* one work item over four waves            */
#define WADG_KERNEL_PIPE 4      /* persistent, pipelined over slice runs    */

typedef struct wadg_ctx_s* wadg_ctx;
typedef struct wadg_batch_s* wadg_batch;

/* Mesh and problem description.  All pointers are host memory, read during
 * the call only (the library copies what it needs).
 *   N        polynomial degree, 1 <= N <= WADG_MAX_N.
 *   nq1      Gauss points per direction and per face, N+1 <= nq1 <= N+3.
 *            (N+1 points are exact to degree 2N+1 in each variable, the
 *            degree prescribed in Section 4; the workloads use N+2, so that
 *            the rule has more points than the basis has nodes, as the
 *            simplex rules of the paper do.)
 *   K        number of elements, K >= 1.
 *   x, y     [K][(N+1)^2] physical coordinates of each element's GLL nodes;
 *            the element map is their degree-N interpolant (isoparametric).
 *   etoe     [K][4] neighbour element across each local face.
 *   etof     [K][4] neighbour's local face | (flip << 2); flip = 1 when the
 *            neighbour parametrises the shared face in the opposite
 *            direction.  Periodic meshes are allowed: matched face points
 *            must coincide up to an integer translation.
 *   c2q      [K][nq1*nq1] c^2 at the volume quadrature points q = i + nq1 j
 *            (obtain their coordinates with wadg_quadrature_points), or NULL
 *            for c^2 = 1.  Must be finite and > 0.
 *   tau_p, tau_u  flux penalties >= 0 (1: upwind, 0: central; Section 4.1).
 */
typedef struct {
  int32_t N;
  int32_t nq1;
  int32_t K;
  const double* x;
  const double* y;
  const int32_t* etoe;
  const int32_t* etof;
  const double* c2q;
  double tau_p;
  double tau_u;
} wadg_mesh;

/* Host-only: physical coordinates of the volume quadrature points,
 * xq, yq: caller-owned host arrays [K][nq1*nq1].  No GPU needed.
 * Ignores mesh->c2q.  Returns WADG_E_INVALID / WADG_E_UNSUPPORTED on bad
 * input. */
int wadg_quadrature_points(const wadg_mesh* mesh, double* xq, double* yq);

/* Host-only: the per-element geometric data the device kernels stream
 * (Section 6.4: geometric factors at quadrature points; Section 6.2: 1/J at
 * quadrature points; Section 7: c2/J), returned untiled.  Caller-owned host
 * arrays:
 *   vol  [6][nq1*nq1][K]: W ys, -W xs, -W yr, W xr (quadrature weight W
 *        times J times r_x, r_y, s_x, s_y), c2/J, 1/J;
 *   face [3][4][nq1][K]: outward unit normal n_x, n_y and w sJ (face
 *        quadrature weight times surface Jacobian).
 * Either pointer may be NULL.  Returns WADG_E_GEOMETRY if J <= 0 anywhere,
 * a value is non-finite or the faces do not conform (the arrays' contents
 * are then unspecified).  No GPU needed; runs on the host's threads. */
int wadg_geometry(const wadg_mesh* mesh, double* vol, double* face);

/* Host-only: the CFL number of a step of size dt on the mesh with c^2 =
 * c2_scale * c2q,
 *   nu = dt c_max (N+1)^2 / h,
 * c_max^2 the largest c^2 at a volume quadrature point and h the smallest
 * element size 4 |D_k| / |dD_k| (area over perimeter, both by the context's
 * quadrature rules: the side length of a square element).  The paper fixes
 * no step size; WADG_CFL_MAX is the largest nu that the parareal coarse
 * step may take: the spectra of the assembled operator on curved periodic
 * meshes (N = 1..4, tau = 0 and 1) keep every eigenvalue inside the
 * stability region of the Runge-Kutta scheme of Section 5.2 up to nu = 1.38
 * or more.  nu: host out.  Returns WADG_E_INVALID / WADG_E_GEOMETRY /
 * WADG_E_UNSUPPORTED as wadg_geometry does.  No GPU needed. */
#define WADG_CFL_MAX 1.25
int wadg_cfl_number(const wadg_mesh* mesh, double dt, double c2_scale, double* nu);

/* Build a context on HIP device `device` (-1: the current device): validates
 * the mesh, builds reference operators and geometry on the host (on up to
 * 16 threads, directly in the tiled device layout) and copies them to
 * library-owned device memory, where an FP32 copy of the geometry is rounded
 * for the FP32-bulk path (on the null stream, awaited before returning).
 * On success *out holds the context; on failure *out is NULL. */
int wadg_create(const wadg_mesh* mesh, int32_t device, wadg_ctx* out);

/* Release the context and its device memory.  NULL is accepted. */
void wadg_destroy(wadg_ctx ctx);

/* Doubles in one slice of the tiled state layout: ceil(K/64)*3*(N+1)^2*64. */
int wadg_state_doubles(wadg_ctx ctx, size_t* count);

/* Bytes of caller-owned device workspace wadg_integrate needs for S slices
 * (one residual array and one second state buffer: 2 * S * 8 *
 * wadg_state_doubles). */
int wadg_workspace_bytes(wadg_ctx ctx, int32_t S, size_t* bytes);

/* One evaluation of the right-hand side dQ/dt = Mtilde^{-1} A_h Q for S
 * slices (Section 4, opening; the WADG inverse of Section 6.2).
 *   Q     device, S slices in the tiled state layout; input, not modified.
 *   dQdt  device, same layout; output; must not alias Q.
 *   stream  hipStream_t or NULL (the null stream).  Asynchronous. */
int wadg_rhs(wadg_ctx ctx, const double* Q, double* dQdt, int32_t S, void* stream);

/* Advance each of S independent slice states by nsteps LSRK(5,4) steps of
 * size dt (Section 5.2), all slices concurrently.
 *   Q     device, S slices in the tiled state layout; in: start states,
 *         out: end states.
 *   work  device workspace of wadg_workspace_bytes(S) bytes, 256-B aligned,
 *         not aliasing Q; its contents on entry are ignored and on return
 *         unspecified (the residual of each step's last stage, which the
 *         2N-storage scheme never reads, is not stored).
 *   dt > 0 and finite, nsteps >= 0.  Asynchronous on `stream`. */
int wadg_integrate(wadg_ctx ctx, double* Q, double* work, int32_t S, double dt,
                   int32_t nsteps, void* stream);

/* FP32-bulk propagation: the same sweep as wadg_integrate with the slice
 * interior in single precision.  Q (FP64, tiled layout) is rounded to an
 * FP32 copy, advanced by nsteps LSRK(5,4) steps with FP32 state, residual,
 * geometry and operators, and widened back into Q; start and end states and
 * everything done on them (norms, corrections) stay FP64.  Its error against
 * the FP64 sweep is that of FP32 rounding in the interior (about 1e-7
 * relative per step, measured by the tests).
 *   work  device workspace of wadg_workspace_bytes_fp32(S) bytes
 *         (3 * S * wadg_state_doubles * 4), not aliasing Q. */
int wadg_workspace_bytes_fp32(wadg_ctx ctx, int32_t S, size_t* bytes);
int wadg_integrate_fp32(wadg_ctx ctx, double* Q, void* work, int32_t S, double dt,
                        int32_t nsteps, void* stream);

/* Parareal iteration over S time slices of length dT = dt * nsteps_fine
 * (concurrent propagation and correction of the slices; the paper defines
 * only the propagators, the iteration is the standard parareal one):
 *   U_0 = y0,  U_{s+1}^0 = G(U_s^0),
 *   U_{s+1}^{k+1} = G(U_s^{k+1}) + F(U_s^k) - G(U_s^k),
 * F = nsteps_fine LSRK steps of dt (all S slices in one wadg_integrate, or
 * wadg_integrate_fp32 when fine_fp32 != 0), G = nsteps_coarse steps of
 * dT / nsteps_coarse, always FP64, one slice after another; the correction
 * update and the convergence norm run in FP64 on the GPU.  Stops when
 * max_s ||U_s^{k+1} - U_s^k||_2 / ||U_s^{k+1}||_2 <= tol or after max_iter
 * iterations; after k iterations U_0..U_k equal the serial fine sweep (to
 * rounding), after S iterations all of them do.
 *   y0  device, one slice (tiled layout); may be U itself.
 *   U   device, S+1 slices: out, U_s ~ y(t0 + s dT).
 *   work  device workspace of wadg_parareal_workspace_bytes bytes.
 *   iterations, last_change: host out.  Synchronises `stream` once per
 *   iteration.  Returns WADG_E_INVALID, before any work, when the coarse
 *   step dt * nsteps_fine / nsteps_coarse has a CFL number (wadg_cfl_number
 *   at the context's c^2 scale) above WADG_CFL_MAX, and WADG_E_NONFINITE if
 *   an iterate is not finite. */
int wadg_parareal_workspace_bytes(wadg_ctx ctx, int32_t S, int32_t fine_fp32, size_t* bytes);
int wadg_parareal(wadg_ctx ctx, const double* y0, double* U, void* work, int32_t S, double dt,
                  int32_t nsteps_fine, int32_t nsteps_coarse, int32_t max_iter, double tol,
                  int32_t fine_fp32, int32_t* iterations, double* last_change, void* stream);

/* Wave-speed scale: every later launch of `ctx` uses c^2 = scale * c2q (the
 * c2q given to wadg_create).  c^2 enters the scheme only through the
 * pressure mass weights c^2/J (Section 7), which are multiplied by `scale`.
 * Default 1 (bitwise the unscaled scheme).  Returns WADG_E_INVALID unless
 * scale is finite and > 0. */
int wadg_set_c2_scale(wadg_ctx ctx, double scale);

/* Discrete adjoint of the sweep of ONE trajectory (one slice of the state
 * layout) over S consecutive time slices of nsteps LSRK steps each (the
 * sensitivity problem: gradient of an objective of the final state).
 *
 * wadg_forward_checkpoints: chk (device, S+1 slices of the state layout):
 *   chk[0] is the start state (in); chk[s+1] = chk[s] advanced by nsteps
 *   steps of dt (out).  work: device, wadg_adjoint_workspace_bytes bytes.
 *   Asynchronous on `stream`.
 *
 * wadg_adjoint: given chk from wadg_forward_checkpoints (same ctx, dt,
 *   nsteps, c^2 scale) and seed = dJ/dq(T) (device, one slice), writes
 *   grad = dJ/dq(0) (device, one slice; may alias seed) and the host scalar
 *   dJ_dscale = gamma dJ/dgamma for c^2 = gamma c2q at the current scale
 *   gamma.  It runs the reverse sweep of the 2N-storage LSRK recursion
 *   (Section 5.2) with the transposed operator L^T = D A D Mtilde^{-1},
 *   D = diag(1,-1,-1) (the strong-weak DG operator A of Section 4.1 has
 *   skew p-u coupling and symmetric penalty blocks; Mtilde^{-1} is the
 *   symmetric WADG inverse of Section 4), recomputing each slice's forward
 *   stage residuals from its checkpoint (held for one slice at a time,
 *   double-buffered: the workspace is about 10 nsteps + 6 slices).  With
 *   the split kernel (WADG_KERNEL_AUTO or _SPLIT) the recompute of the next
 *   slice shares each reverse-stage launch on `stream`; with the streamed
 *   kernel it runs on a second stream owned by the context, ordered against
 *   `stream` with events.  The context must not be used from two threads at
 *   once.  Padding entries of seed must be zero; grad padding is
 *   unspecified.  Synchronises `stream` once at the end.  Returns
 *   WADG_E_NONFINITE if dJ_dscale is not finite.  work must not overlap
 *   chk, seed or grad. */
int wadg_adjoint_workspace_bytes(wadg_ctx ctx, int32_t nsteps, size_t* bytes);
int wadg_forward_checkpoints(wadg_ctx ctx, double* chk, void* work, int32_t S, double dt,
                             int32_t nsteps, void* stream);
int wadg_adjoint(wadg_ctx ctx, const double* chk, const double* seed, double* grad, void* work,
                 int32_t S, double dt, int32_t nsteps, double* dJ_dscale, void* stream);

/* Batches of independent problems (many meshes of one degree, each with
 * its own slices and dt), advanced together: one launch per LSRK stage
 * covers every (problem, slice, 64-element group) work item -- Section 6.1's
 * batching of elements per workgroup, taken across problems.
 *
 * wadg_batch_create: meshes[nprob] (host; all with the same N, nq1, tau_p,
 *   tau_u; validated like wadg_create), S[nprob] slices per problem.  A
 *   problem's slices are stored P at a time side by side, as P disjoint
 *   copies of its mesh (a virtual mesh of P K elements), so that small or
 *   ragged meshes fill the 64 lanes of their element groups.  P in
 *   [1, min(S, 64)] is chosen per problem to move the fewest bytes per stage
 *   (state tiles per work item plus geometry per virtual element group;
 *   ties: the smaller P), with a virtual slice under 2 GiB.  Returns
 *   WADG_E_GEOMETRY / WADG_E_INVALID naming the offending problem.
 * wadg_batch_layout: offset[nprob + 1] (host out, int64) -- problem i
 *   occupies doubles [offset[i], offset[i+1]) of the batch state;
 *   pack[nprob] (host out) -- P_i.  Problem i is stored as ceil(S_i / P_i)
 *   virtual slices in the tiled state layout of a virtual mesh of P_i K_i
 *   elements: slice s is copy s % P_i of virtual slice s / P_i, and its
 *   element k is virtual element (s % P_i) K_i + k.  Either pointer may be
 *   NULL.
 * wadg_batch_workspace_bytes: device workspace for integrate (2 states).
 * wadg_batch_integrate: every problem advanced by nsteps LSRK steps of its
 *   own dt[i] (host array, finite > 0), all slices at once.  Q (device):
 *   the batch state, in/out; work: device workspace.  Asynchronous.
 * wadg_batch_set_runs: run_slices >= 1 selects the pipelined kernel (as
 *   WADG_KERNEL_PIPE): for every problem and element group of its virtual
 *   mesh, the virtual slices in which the group holds a real slice are cut
 *   into runs of at most run_slices (nearly equal lengths), one 512-thread
 *   workgroup per run with the group's geometry on chip; elements of unused
 *   copies in a last virtual slice are neither computed into the state nor
 *   written (their values in Q are unspecified).  0 returns to the item
 *   schedule of wadg_batch_set_schedule.  Default 16 where the kernel's LDS
 *   plan fits (N <= 3 with nq1 <= N + 2), else 0.  Returns
 *   WADG_E_UNSUPPORTED for run_slices > 0 where it does not fit.
 * wadg_batch_set_schedule: item schedule (and run_slices = 0).  wg_per_cu
 *   0: one four-wave workgroup per work item (the split-work kernel, as
 *   WADG_KERNEL_SPLIT); 1..64: that many persistent two-wave workgroups per
 *   CU looping over the list (the streamed kernel).  order: 0 problem-major,
 *   1 round-robin over problems.
 * Results are bitwise independent of the schedule and of the runs.
 * wadg_batch_tune: the autotuner -- times one stage of every candidate
 *   (runs of 4, 8, 16, 32, 128 slices where the pipelined kernel fits; 1, 2,
 *   4, 8 persistent workgroups per CU or one per item, both orders) reps
 *   times on the device, keeps the fastest and returns it (host out:
 *   wg_per_cu, order, run_slices -- 0 unless the pipelined kernel won --
 *   and best_us per stage).  Q is read only; work is scratch.  Synchronises
 *   `stream`.
 * wadg_batch_capture: records the whole nsteps sweep of wadg_batch_integrate
 *   for these Q, work and dt into a HIP graph (on a stream of its own); the
 *   graph reads its own copy of the per-problem dt, so later integrate calls
 *   with other dt do not change what it computes.  wadg_batch_replay
 *   launches it on `stream` (each replay advances Q by nsteps steps again).
 *   wadg_batch_release_graph frees it (after the device has drained, so
 *   replays still queued finish first; so does a new capture, which replaces
 *   the graph); set_schedule, set_runs and tune refuse while a graph is
 *   held.
 * A call that changes the device-side work list (set_schedule, set_runs,
 * tune) or
 * the per-problem dt (integrate, tune, capture with dt other than the last)
 * first waits for the device to drain, so that no queued launch of the
 * batch reads a table while it is rewritten. */
int wadg_batch_create(const wadg_mesh* meshes, int32_t nprob, const int32_t* S, int32_t device,
                      wadg_batch* out);
void wadg_batch_destroy(wadg_batch b);
int wadg_batch_layout(wadg_batch b, int64_t* offset, int32_t* pack);
int wadg_batch_workspace_bytes(wadg_batch b, size_t* bytes);
int wadg_batch_integrate(wadg_batch b, double* Q, double* work, const double* dt, int32_t nsteps,
                         void* stream);
int wadg_batch_set_schedule(wadg_batch b, int32_t wg_per_cu, int32_t order);
int wadg_batch_set_runs(wadg_batch b, int32_t run_slices);
int wadg_batch_tune(wadg_batch b, const double* Q, double* work, const double* dt, int32_t reps,
                    int32_t* wg_per_cu, int32_t* order, int32_t* run_slices, double* best_us,
                    void* stream);
int wadg_batch_capture(wadg_batch b, double* Q, double* work, const double* dt, int32_t nsteps);
int wadg_batch_replay(wadg_batch b, void* stream);
int wadg_batch_release_graph(wadg_batch b);

/* Per-slice reductions (the norms the convergence checks use):
 *   out[s][0] = ||A_s - B_s||_2,  out[s][1] = ||B_s||_2,
 *   out[s][2] = max |A_s - B_s|,  out[s][3] = 1 if every A_s entry is finite
 *   else 0, over the 3*(N+1)^2*K state entries of slice s (padding is
 *   skipped).  B may be NULL (treated as zero: out[s][0] = ||A_s||,
 *   out[s][1] = 0).
 *   A, B     device, S slices in the tiled state layout;  out: host [S][4].
 *   scratch  caller-owned device memory of scratch_bytes bytes, at least
 *            wadg_norms_workspace_bytes(S) (= 8 * 260 * S: 64 partial sums
 *            of 4 values per slice, then the S x 4 sums), 8-byte aligned,
 *            not overlapping A or B; its contents on entry are ignored.
 * The library allocates nothing.  Synchronises `stream`.  Deterministic:
 * fixed reduction order.  Returns WADG_E_NONFINITE (after filling out) if
 * some A entry is not finite, WADG_E_INVALID for a missing or short scratch
 * and for S >= 2^25 (64 partial sums per slice in one launch). */
int wadg_norms_workspace_bytes(wadg_ctx ctx, int32_t S, size_t* bytes);
int wadg_norms(wadg_ctx ctx, const double* A, const double* B, int32_t S, void* scratch,
               size_t scratch_bytes, double* out, void* stream);

/* wadg_norms for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc)
 * and hold no scratch buffer of their own: the same reduction, the same
 * kernels and launch shape (so bitwise the same out as wadg_norms), run in
 * a fixed 2,129,920-byte scratch array that the library keeps on every GPU
 * it runs on until the process ends.  Its device address is taken once
 * per device when the first context on that device is created.
 *   A, B, S, out, stream: as for wadg_norms; S <= WADG_NORMS_NOALLOC_MAX_S.
 * Allocates nothing.  Every call on one GPU shares that GPU's array, so
 * calls that overlap on one GPU (other streams, other threads) race; calls
 * on one stream do not.  The kernels overwrite every scratch value they
 * read, so nothing is cleared between calls.  Synchronises `stream`.
 * Returns WADG_E_INVALID, before any HIP call, for S above the maximum,
 * and as wadg_norms otherwise. */
#define WADG_NORMS_NOALLOC_MAX_S 1024
int wadg_norms_noalloc(wadg_ctx ctx, const double* A, const double* B, int32_t S, double* out,
                       void* stream);

/* L2 norms with the element maps' Jacobians (the norm of Section 5.2's L2
 * errors), per slice:
 *   out[s][0] = ||A_s - B_s||_{L2},  out[s][1] = ||B_s||_{L2},
 * the square root of the integral over the mesh of p^2 + u^2 + v^2 of the
 * difference (of B), by the context's volume rule (nq1 x nq1 Gauss points
 * per element, each field interpolated there from its nodes, weighted by
 * w_q J_q).  B may be NULL (treated as zero: out[s][1] = 0).
 *   A, B     device, S slices in the tiled state layout;  out: host [S][2].
 *   scratch  caller-owned device memory of at least
 *            wadg_l2_norms_workspace_bytes(S) (= 16 S (ceil(K/64) + 1))
 *            bytes, 8-byte aligned, not overlapping A or B.
 * The library allocates nothing.  Synchronises `stream`.  Deterministic:
 * fixed reduction order.  Returns WADG_E_NONFINITE (after filling out) if a
 * norm is not finite, WADG_E_INVALID for a missing or short scratch. */
int wadg_l2_norms_workspace_bytes(wadg_ctx ctx, int32_t S, size_t* bytes);
int wadg_l2_norms(wadg_ctx ctx, const double* A, const double* B, int32_t S, void* scratch,
                  size_t scratch_bytes, double* out, void* stream);

/* Tuning: the order in which (slice, 64-element group) work items are
 * launched.  Items are grouped in tiles of groups_per_tile element groups x
 * slices_per_tile slices (0: all slices), slice-major inside a tile; each
 * XCD takes a contiguous range of tiles.  Successive stage launches of a
 * context walk this order in alternating directions, so that a launch
 * starts on the items the previous one wrote last (memory-side cache
 * reuse).  Results do not depend on the order (bitwise).  Defaults: 8, 0.
 * Not thread-safe per context.  Returns WADG_E_INVALID for
 * groups_per_tile < 1 or slices_per_tile < 0. */
int wadg_set_schedule(wadg_ctx ctx, int32_t groups_per_tile, int32_t slices_per_tile);

/* Tuning: which stage kernel runs (Section 6.4's volume, surface and update
 * kernels, fused).
 *   WADG_KERNEL_STREAMED: one 128-thread workgroup (two waves) per (slice,
 *     64-element group), the group's geometry read from global memory for
 *     each; follows wadg_set_schedule.
 *   WADG_KERNEL_SPLIT: the same work item over a 256-thread workgroup of
 *     four waves (pressure volume, velocity volume, two face waves), two
 *     workgroups per CU; follows wadg_set_schedule.
 *   WADG_KERNEL_RESIDENT: 256-thread workgroups that each hold one element
 *     group's geometry in LDS (up to 160 KiB) and sweep a range of its
 *     slices; ignores wadg_set_schedule.  Its FP64 geometry fits for N <= 2,
 *     or N = 3 with nq1 <= 5; elsewhere a RESIDENT request falls back to
 *     the streamed kernel for that precision.
 *   WADG_KERNEL_PIPE: LSRK stages only (FP64 and FP32-bulk): one
 *     512-thread workgroup per CU (two in FP32 where both fit in LDS) that
 *     owns one element group and a run of its slices, keeps the group's
 *     geometry on chip for the whole run, streams the next slice's input tile into LDS while
 *     computing the current one, and applies one slice's mass inverse and
 *     update while the next slice's volume and face terms are formed (a
 *     two-stage pipeline over the slices); ignores wadg_set_schedule.
 *     Needs two input tiles, the metric planes, the face terms, the
 *     handed-over load vectors and the pressure mass weights in LDS (FP64:
 *     N <= 3 with nq1 <= N + 2; FP32: every N, nq1); launches of fewer than
 *     two slices, right-hand sides and the adjoint's launches take the
 *     split kernel.  Launches whose state (Q in, Q out and the residual)
 *     exceeds 512 MB store their outputs and load the residual with the
 *     non-temporal cache hint.
 *   WADG_KERNEL_AUTO (default): LSRK stages (FP64 and FP32) of two or more
 *     slices take the pipelined kernel where it fits, else the split
 *     kernel; right-hand-side launches the resident kernel where it fits,
 *     else the split kernel -- the fastest measured on MI355X.
 * All variants give bitwise-identical results.  The adjoint's operator
 * launches (apply-A) take the split kernel under AUTO and SPLIT, else the
 * streamed kernel (the resident kernel has no apply-A mode).  Returns
 * WADG_E_INVALID for an
 * unknown value and WADG_E_UNSUPPORTED when the resident or pipelined
 * kernel is requested for an (N, nq1) whose FP64 data do not fit. */
int wadg_set_kernel(wadg_ctx ctx, int32_t kernel);

/* The kernel variant that `ctx` launches for LSRK stages (rhs == 0; FP64
 * for fp32 == 0, FP32-bulk for fp32 != 0) or for wadg_rhs (rhs != 0,
 * fp32 == 0).  kernel: host out. */
int wadg_kernel_in_use(wadg_ctx ctx, int32_t rhs, int32_t fp32, int32_t* kernel);

/* Static description of a status code; never NULL. */
const char* wadg_status_string(int status);

/* Thread-local detail of the last failure on this thread ("" if none). */
const char* wadg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WADG_H */
