// C ABI of the WADG sweep (declared in include/wadg.h): validation, host
// setup, device memory of the context, and the stage loop.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "wadg.h"
#include "wadg_internal.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// LSRK(5,4) 2N-storage coefficients (Carpenter & Kennedy 1994), the
// integrator of the paper's experiments (Section 4.2.1).
const double kRkA[5] = {0.0,
                        -567301805773.0 / 1357537059087.0,
                        -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0,
                        -1275806237668.0 / 842570457699.0};
const double kRkB[5] = {1432997174477.0 / 9575080441755.0,
                        5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0,
                        3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};

constexpr int kNormBlocks = 64;

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) return;
    ok = (dev == prev) || hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int check_mesh(const wadg_mesh* m) {
  if (!m) return fail(WADG_E_INVALID, "mesh is NULL");
  if (m->N < 1 || m->N > WADG_MAX_N)
    return fail(WADG_E_UNSUPPORTED, "degree N must be in [1, " + std::to_string(WADG_MAX_N) + "]");
  if (m->nq1 < m->N + 1 || m->nq1 > m->N + 3)
    return fail(WADG_E_UNSUPPORTED, "nq1 must be in [N+1, N+3]");
  if (m->K < 1) return fail(WADG_E_INVALID, "K must be >= 1");
  if (!m->x || !m->y || !m->etoe || !m->etof)
    return fail(WADG_E_INVALID, "mesh arrays must not be NULL");
  if (!(m->tau_p >= 0.0) || !(m->tau_u >= 0.0) || !std::isfinite(m->tau_p) ||
      !std::isfinite(m->tau_u))
    return fail(WADG_E_INVALID, "tau_p and tau_u must be finite and >= 0");
  // one slice of the tiled state must be addressable with 31-bit byte offsets
  const long long groups = ((long long)m->K + wadg::kWave - 1) / wadg::kWave;
  if (groups * 3 * (m->N + 1) * (m->N + 1) * wadg::kWave * 8 >= (1LL << 31))
    return fail(WADG_E_INVALID, "K too large: one slice must stay below 2 GiB");
  return WADG_OK;
}

wadg::MeshIn mesh_in(const wadg_mesh* m) {
  return wadg::MeshIn{m->N, m->nq1, m->K, m->x, m->y, m->etoe, m->etof, m->c2q};
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

}  // namespace

struct wadg_ctx_s {
  int device = 0;
  int N = 0, nq1 = 0, K = 0;
  double tau_p = 1.0, tau_u = 1.0;
  int tile_groups = 8;   // schedule: element groups per tile
  int tile_slices = 0;   // slices per tile (0: all)
  int kernel = WADG_KERNEL_AUTO;
  int cus = 256;         // compute units of the device
  double c2_scale = 1.0; // multiplies c^2 (wadg_set_c2_scale)
  unsigned order_flip = 0;  // item order of the next stage launch (launch_stage)
  double* d_vol = nullptr;
  double* d_face = nullptr;
  float* d_vol32 = nullptr;      // geometry rounded to FP32 (FP32-bulk path)
  float* d_face32 = nullptr;
  int32_t* d_nbr = nullptr;
  double* d_partials = nullptr;  // norms scratch, grown on demand
  double* d_out = nullptr;
  int32_t norms_cap = 0;
  // adjoint: a second stream (default priority) for the forward recompute
  // that overlaps the reverse sweep, and the events that order the two
  hipStream_t aux = nullptr;
  hipEvent_t ev_in = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};
  int groups() const { return (K + wadg::kWave - 1) / wadg::kWave; }
  size_t tile() const { return (size_t)3 * (N + 1) * (N + 1) * wadg::kWave; }
  size_t slice_doubles() const { return (size_t)groups() * tile(); }
  size_t state_doubles(int32_t S) const { return (size_t)S * slice_doubles(); }
};

namespace {

void free_ctx(wadg_ctx c) {
  if (!c) return;
  if (c->d_vol) (void)hipFree(c->d_vol);
  if (c->d_face) (void)hipFree(c->d_face);
  if (c->d_vol32) (void)hipFree(c->d_vol32);
  if (c->d_face32) (void)hipFree(c->d_face32);
  if (c->d_nbr) (void)hipFree(c->d_nbr);
  if (c->d_partials) (void)hipFree(c->d_partials);
  if (c->d_out) (void)hipFree(c->d_out);
  for (hipEvent_t e : {c->ev_in, c->ev_rec[0], c->ev_rec[1], c->ev_rev[0], c->ev_rev[1]})
    if (e) (void)hipEventDestroy(e);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  delete c;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(WADG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define WADG_HIP(call)                                  \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #call);   \
  } while (0)

int check_slices(wadg_ctx c, int32_t S) {
  if (!c) return fail(WADG_E_INVALID, "context is NULL");
  if (S < 1) return fail(WADG_E_INVALID, "S must be >= 1");
  const long long nEG = (c->K + wadg::kWave - 1) / wadg::kWave;
  if (nEG * (long long)S >= (1LL << 31)) return fail(WADG_E_INVALID, "too many slices");
  return WADG_OK;
}

// Kernel variant that runs for this context, precision and launch mode.
// Automatic choice, from measurement on MI355X (64x64 and 128x128
// elements, N = 3, FP64 and FP32): LSRK stages take the split-work kernel;
// right-hand-side launches take the resident-geometry kernel where the
// geometry fits in LDS, else the split-work kernel; the adjoint's apply-A
// launches take the split-work kernel (the resident kernel has no apply-A
// mode, so an explicit RESIDENT or STREAMED choice runs them streamed).
int kernel_path(wadg_ctx c, bool fp32, int mode) {
  const bool fits = wadg::resident_supported(c->N, c->nq1, fp32);
  if (mode == wadg::kApplyAMass) return WADG_KERNEL_SPLIT;   // split kernel only
  if (mode == wadg::kApplyA)   // no resident apply-A mode
    return c->kernel == WADG_KERNEL_AUTO || c->kernel == WADG_KERNEL_SPLIT ? WADG_KERNEL_SPLIT
                                                                           : WADG_KERNEL_STREAMED;
  if (c->kernel == WADG_KERNEL_RESIDENT && fits) return WADG_KERNEL_RESIDENT;
  if (c->kernel != WADG_KERNEL_AUTO) return c->kernel == WADG_KERNEL_RESIDENT
                                                ? WADG_KERNEL_STREAMED : c->kernel;
  if (mode == wadg::kRhs && fits) return WADG_KERNEL_RESIDENT;
  return WADG_KERNEL_SPLIT;
}

int launch_stage(wadg_ctx c, int mode, bool fp32, const wadg::StageParams& p0, void* stream) {
  const int path = kernel_path(c, fp32, mode);
  // alternate the item order from one launch to the next (item_of)
  wadg::StageParams p = p0;
  c->order_flip ^= 1;
  p.reverse = (int32_t)c->order_flip;
  if (path == WADG_KERNEL_SPLIT)
    return fp32 ? wadg::launch_stage_split_fp32(c->N, c->nq1, p, stream)
                : wadg::launch_stage_split(c->N, c->nq1, mode, p, stream);
  if (path == WADG_KERNEL_RESIDENT) {
    const int ranges = wadg::resident_ranges(p.nEG, p.S, c->cus);
    return fp32 ? wadg::launch_stage_resident_fp32(c->N, c->nq1, p, ranges, stream)
                : wadg::launch_stage_resident(c->N, c->nq1, mode, p, ranges, stream);
  }
  return fp32 ? wadg::launch_stage_streamed_fp32(c->N, c->nq1, p, stream)
              : wadg::launch_stage_streamed(c->N, c->nq1, mode, p, stream);
}

wadg::StageParams base_params(wadg_ctx c, int32_t S) {
  wadg::StageParams p{};
  p.vol = c->d_vol;
  p.face = c->d_face;
  p.nbr = c->d_nbr;
  p.K = c->K;
  p.S = S;
  p.nEG = (c->K + wadg::kWave - 1) / wadg::kWave;
  p.tile_groups = c->tile_groups < p.nEG ? c->tile_groups : p.nEG;
  p.tile_slices = (c->tile_slices == 0 || c->tile_slices > S) ? S : c->tile_slices;
  p.tau_p = c->tau_p;
  p.tau_u = c->tau_u;
  p.c2_scale = c->c2_scale;
  p.res_out = nullptr;
  return p;
}

}  // namespace

extern "C" {

int wadg_quadrature_points(const wadg_mesh* mesh, double* xq, double* yq) {
  int st = check_mesh(mesh);
  if (st) return st;
  if (!xq || !yq) return fail(WADG_E_INVALID, "output arrays must not be NULL");
  wadg::RefOps ops;
  std::string err;
  if (!wadg::build_ref_ops(mesh->N, mesh->nq1, &ops, &err)) return fail(WADG_E_UNSUPPORTED, err);
  wadg::quadrature_points(mesh_in(mesh), ops, xq, yq);
  return WADG_OK;
}

int wadg_geometry(const wadg_mesh* mesh, double* vol, double* face) {
  int st = check_mesh(mesh);
  if (st) return st;
  wadg::RefOps ops;
  std::string err;
  if (!wadg::build_ref_ops(mesh->N, mesh->nq1, &ops, &err)) return fail(WADG_E_UNSUPPORTED, err);
  std::vector<double> v, f;
  int g = wadg::build_geometry(mesh_in(mesh), ops, &v, &f, nullptr, &err);
  if (g) return fail(g == -1 ? WADG_E_INVALID : WADG_E_GEOMETRY, err);
  if (vol) std::memcpy(vol, v.data(), v.size() * sizeof(double));
  if (face) std::memcpy(face, f.data(), f.size() * sizeof(double));
  return WADG_OK;
}

int wadg_create(const wadg_mesh* mesh, int32_t device, wadg_ctx* out) {
  if (!out) return fail(WADG_E_INVALID, "out is NULL");
  *out = nullptr;
  int st = check_mesh(mesh);
  if (st) return st;
  if (!wadg::stage_supported(mesh->N, mesh->nq1))
    return fail(WADG_E_UNSUPPORTED, "degree / quadrature not compiled in");
  wadg::RefOps ops;
  std::string err;
  if (!wadg::build_ref_ops(mesh->N, mesh->nq1, &ops, &err)) return fail(WADG_E_UNSUPPORTED, err);
  std::vector<double> vol0, face0;
  std::vector<int32_t> nbr0;
  int g = wadg::build_geometry(mesh_in(mesh), ops, &vol0, &face0, &nbr0, &err);
  if (g) return fail(g == -1 ? WADG_E_INVALID : WADG_E_GEOMETRY, err);
  const int nq = mesh->nq1;
  std::vector<double> vol = wadg::tile_planes(vol0, 6 * nq * nq, mesh->K);
  std::vector<double> face = wadg::tile_planes(face0, 12 * nq, mesh->K);
  std::vector<int32_t> nbr = wadg::tile_planes(nbr0, 8, mesh->K);
  std::vector<float> vol32(vol.begin(), vol.end()), face32(face.begin(), face.end());

  int dev = device;
  if (dev < 0) WADG_HIP(hipGetDevice(&dev));
  DeviceGuard guard(dev);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select HIP device " + std::to_string(dev));

  wadg_ctx c = new wadg_ctx_s();
  c->device = dev;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      cus > 0)
    c->cus = cus;
  c->N = mesh->N;
  c->nq1 = mesh->nq1;
  c->K = mesh->K;
  c->tau_p = mesh->tau_p;
  c->tau_u = mesh->tau_u;
  hipError_t e;
  if ((e = hipMalloc(&c->d_vol, vol.size() * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&c->d_face, face.size() * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&c->d_nbr, nbr.size() * sizeof(int32_t))) != hipSuccess ||
      (e = hipMemcpy(c->d_vol, vol.data(), vol.size() * sizeof(double),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->d_face, face.data(), face.size() * sizeof(double),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->d_nbr, nbr.data(), nbr.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMalloc(&c->d_vol32, vol32.size() * sizeof(float))) != hipSuccess ||
      (e = hipMalloc(&c->d_face32, face32.size() * sizeof(float))) != hipSuccess ||
      (e = hipMemcpy(c->d_vol32, vol32.data(), vol32.size() * sizeof(float),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->d_face32, face32.data(), face32.size() * sizeof(float),
                     hipMemcpyHostToDevice)) != hipSuccess) {
    free_ctx(c);
    return hip_fail(e, "wadg_create device setup");
  }
  *out = c;
  return WADG_OK;
}

void wadg_destroy(wadg_ctx ctx) {
  if (!ctx) return;
  DeviceGuard guard(ctx->device);
  free_ctx(ctx);
}

int wadg_state_doubles(wadg_ctx ctx, size_t* count) {
  if (!ctx) return fail(WADG_E_INVALID, "context is NULL");
  if (!count) return fail(WADG_E_INVALID, "count is NULL");
  *count = ctx->slice_doubles();
  return WADG_OK;
}

int wadg_workspace_bytes(wadg_ctx ctx, int32_t S, size_t* bytes) {
  int st = check_slices(ctx, S);
  if (st) return st;
  if (!bytes) return fail(WADG_E_INVALID, "bytes is NULL");
  *bytes = 2 * ctx->state_doubles(S) * sizeof(double);
  return WADG_OK;
}

int wadg_set_schedule(wadg_ctx ctx, int32_t groups_per_tile, int32_t slices_per_tile) {
  if (!ctx) return fail(WADG_E_INVALID, "context is NULL");
  if (groups_per_tile < 1 || slices_per_tile < 0)
    return fail(WADG_E_INVALID, "groups_per_tile must be >= 1 and slices_per_tile >= 0");
  ctx->tile_groups = groups_per_tile;
  ctx->tile_slices = slices_per_tile;
  return WADG_OK;
}

int wadg_set_kernel(wadg_ctx ctx, int32_t kernel) {
  if (!ctx) return fail(WADG_E_INVALID, "context is NULL");
  if (kernel != WADG_KERNEL_AUTO && kernel != WADG_KERNEL_STREAMED &&
      kernel != WADG_KERNEL_RESIDENT && kernel != WADG_KERNEL_SPLIT)
    return fail(WADG_E_INVALID, "unknown kernel variant");
  if (kernel == WADG_KERNEL_RESIDENT && !wadg::resident_supported(ctx->N, ctx->nq1, false))
    return fail(WADG_E_UNSUPPORTED, "the element group's geometry does not fit in LDS");
  ctx->kernel = kernel;
  return WADG_OK;
}

int wadg_set_c2_scale(wadg_ctx ctx, double scale) {
  if (!ctx) return fail(WADG_E_INVALID, "context is NULL");
  if (!(scale > 0.0) || !std::isfinite(scale))
    return fail(WADG_E_INVALID, "the c^2 scale must be finite and > 0");
  ctx->c2_scale = scale;
  return WADG_OK;
}

int wadg_kernel_in_use(wadg_ctx ctx, int32_t rhs, int32_t fp32, int32_t* kernel) {
  if (!ctx) return fail(WADG_E_INVALID, "context is NULL");
  if (!kernel) return fail(WADG_E_INVALID, "kernel is NULL");
  if (rhs && fp32) return fail(WADG_E_INVALID, "there is no FP32 right-hand-side launch");
  *kernel = kernel_path(ctx, fp32 != 0, rhs ? wadg::kRhs : wadg::kStage);
  return WADG_OK;
}

int wadg_rhs(wadg_ctx ctx, const double* Q, double* dQdt, int32_t S, void* stream) {
  int st = check_slices(ctx, S);
  if (st) return st;
  if (!Q || !dQdt) return fail(WADG_E_INVALID, "Q and dQdt must not be NULL");
  const size_t nbytes = ctx->state_doubles(S) * sizeof(double);
  if (overlaps(Q, nbytes, dQdt, nbytes)) return fail(WADG_E_INVALID, "dQdt must not alias Q");
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the context's device");
  wadg::StageParams p = base_params(ctx, S);
  p.Qin = Q;
  p.Qout = dQdt;
  p.res = nullptr;
  int e = launch_stage(ctx, wadg::kRhs, false, p, stream);
  if (e) return hip_fail((hipError_t)e, "stage kernel launch");
  return WADG_OK;
}

int wadg_integrate(wadg_ctx ctx, double* Q, double* work, int32_t S, double dt, int32_t nsteps,
                   void* stream) {
  int st = check_slices(ctx, S);
  if (st) return st;
  if (!Q || !work) return fail(WADG_E_INVALID, "Q and work must not be NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(WADG_E_INVALID, "dt must be finite and > 0");
  if (nsteps < 0) return fail(WADG_E_INVALID, "nsteps must be >= 0");
  const size_t n = ctx->state_doubles(S);
  if (overlaps(Q, n * sizeof(double), work, 2 * n * sizeof(double)))
    return fail(WADG_E_INVALID, "work must not alias Q");
  if (nsteps == 0) return WADG_OK;
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the context's device");
  double* res = work;
  double* other = work + n;
  double* cur = Q;
  wadg::StageParams p = base_params(ctx, S);
  p.res = res;
  p.dt = dt;
  for (int stp = 0; stp < nsteps; ++stp)
    for (int i = 0; i < 5; ++i) {
      p.Qin = cur;
      p.Qout = (cur == Q) ? other : Q;
      p.rkA = kRkA[i];
      p.rkB = kRkB[i];
      int e = launch_stage(ctx, wadg::kStage, false, p, stream);
      if (e) return hip_fail((hipError_t)e, "stage kernel launch");
      cur = static_cast<double*>(p.Qout);
    }
  if (cur != Q) {
    int e = wadg::launch_copy(cur, Q, n, stream);
    if (e) return hip_fail((hipError_t)e, "copy kernel launch");
  }
  return WADG_OK;
}

int wadg_workspace_bytes_fp32(wadg_ctx ctx, int32_t S, size_t* bytes) {
  int st = check_slices(ctx, S);
  if (st) return st;
  if (!bytes) return fail(WADG_E_INVALID, "bytes is NULL");
  *bytes = 3 * ctx->state_doubles(S) * sizeof(float);
  return WADG_OK;
}

int wadg_integrate_fp32(wadg_ctx ctx, double* Q, void* work, int32_t S, double dt,
                        int32_t nsteps, void* stream) {
  int st = check_slices(ctx, S);
  if (st) return st;
  if (!Q || !work) return fail(WADG_E_INVALID, "Q and work must not be NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(WADG_E_INVALID, "dt must be finite and > 0");
  if (nsteps < 0) return fail(WADG_E_INVALID, "nsteps must be >= 0");
  const size_t n = ctx->state_doubles(S);
  if (overlaps(Q, n * sizeof(double), work, 3 * n * sizeof(float)))
    return fail(WADG_E_INVALID, "work must not alias Q");
  if (nsteps == 0) return WADG_OK;
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the context's device");
  float* q0 = static_cast<float*>(work);
  float* q1 = q0 + n;
  float* res = q1 + n;
  int e = wadg::launch_to_fp32(Q, q0, n, stream);
  if (e) return hip_fail((hipError_t)e, "conversion kernel launch");
  wadg::StageParams p = base_params(ctx, S);
  p.vol = ctx->d_vol32;
  p.face = ctx->d_face32;
  p.res = res;
  p.dt = dt;
  float* cur = q0;
  for (int stp = 0; stp < nsteps; ++stp)
    for (int i = 0; i < 5; ++i) {
      p.Qin = cur;
      p.Qout = (cur == q0) ? q1 : q0;
      p.rkA = kRkA[i];
      p.rkB = kRkB[i];
      e = launch_stage(ctx, wadg::kStage, true, p, stream);
      if (e) return hip_fail((hipError_t)e, "stage kernel launch");
      cur = static_cast<float*>(p.Qout);
    }
  e = wadg::launch_to_fp64(cur, Q, n, stream);
  if (e) return hip_fail((hipError_t)e, "conversion kernel launch");
  return WADG_OK;
}

namespace {
size_t fine_work_bytes(wadg_ctx ctx, int32_t S, int32_t fine_fp32) {
  const size_t n = ctx->state_doubles(S);
  return fine_fp32 ? 3 * n * sizeof(float) : 2 * n * sizeof(double);
}
size_t parareal_bytes(wadg_ctx ctx, int32_t S, int32_t fine_fp32) {
  const size_t n1 = ctx->slice_doubles();
  return (2 * (size_t)S + 3) * n1 * sizeof(double) + fine_work_bytes(ctx, S, fine_fp32) +
         ((size_t)S * kNormBlocks * 4 + (size_t)S * 4) * sizeof(double);
}
}  // namespace

int wadg_parareal_workspace_bytes(wadg_ctx ctx, int32_t S, int32_t fine_fp32, size_t* bytes) {
  int st = check_slices(ctx, S);
  if (st) return st;
  if (!bytes) return fail(WADG_E_INVALID, "bytes is NULL");
  *bytes = parareal_bytes(ctx, S, fine_fp32);
  return WADG_OK;
}

int wadg_parareal(wadg_ctx ctx, const double* y0, double* U, void* work, int32_t S, double dt,
                  int32_t nsteps_fine, int32_t nsteps_coarse, int32_t max_iter, double tol,
                  int32_t fine_fp32, int32_t* iterations, double* last_change, void* stream) {
  int st = check_slices(ctx, S);
  if (st) return st;
  if (!y0 || !U || !work || !iterations || !last_change)
    return fail(WADG_E_INVALID, "y0, U, work, iterations and last_change must not be NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(WADG_E_INVALID, "dt must be finite and > 0");
  if (nsteps_fine < 1 || nsteps_coarse < 1 || max_iter < 0)
    return fail(WADG_E_INVALID, "nsteps_fine, nsteps_coarse >= 1 and max_iter >= 0 required");
  if (!(tol >= 0.0)) return fail(WADG_E_INVALID, "tol must be >= 0");
  const size_t n1 = ctx->slice_doubles();
  const size_t ubytes = (S + 1) * n1 * sizeof(double);
  const size_t wbytes = parareal_bytes(ctx, S, fine_fp32);
  if (overlaps(U, ubytes, work, wbytes)) return fail(WADG_E_INVALID, "work must not alias U");
  if (y0 != U && overlaps(y0, n1 * sizeof(double), U, ubytes))
    return fail(WADG_E_INVALID, "y0 must be U itself or not overlap U");
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the context's device");
  hipStream_t hs = static_cast<hipStream_t>(stream);

  double* F = static_cast<double*>(work);
  double* Gold = F + (size_t)S * n1;
  double* tmp = Gold + (size_t)S * n1;
  double* cwork = tmp + n1;
  char* fwork = reinterpret_cast<char*>(cwork + 2 * n1);
  double* partials = reinterpret_cast<double*>(fwork + fine_work_bytes(ctx, S, fine_fp32));
  double* dout = partials + (size_t)S * kNormBlocks * 4;
  const double dtc = dt * nsteps_fine / nsteps_coarse;
  const int32_t tile = (int32_t)ctx->tile();
  const size_t sb = n1 * sizeof(double);

  auto coarse = [&](double* q) { return wadg_integrate(ctx, q, cwork, 1, dtc, nsteps_coarse, stream); };
  if (y0 != U) WADG_HIP(hipMemcpyAsync(U, y0, sb, hipMemcpyDeviceToDevice, hs));
  // coarse prediction U_{s+1}^0 = G(U_s^0), remembered as G(U_s^0)
  for (int s = 0; s < S; ++s) {
    WADG_HIP(hipMemcpyAsync(Gold + s * n1, U + s * n1, sb, hipMemcpyDeviceToDevice, hs));
    if ((st = coarse(Gold + s * n1))) return st;
    WADG_HIP(hipMemcpyAsync(U + (s + 1) * n1, Gold + s * n1, sb, hipMemcpyDeviceToDevice, hs));
  }
  std::vector<double> out((size_t)S * 4);
  double change = INFINITY;
  int32_t it = 0;
  for (int k = 0; k < max_iter; ++k) {
    // fine propagation of all slices at once: F_s = F(U_s^k)
    WADG_HIP(hipMemcpyAsync(F, U, (size_t)S * sb, hipMemcpyDeviceToDevice, hs));
    st = fine_fp32 ? wadg_integrate_fp32(ctx, F, fwork, S, dt, nsteps_fine, stream)
                   : wadg_integrate(ctx, F, reinterpret_cast<double*>(fwork), S, dt, nsteps_fine,
                                    stream);
    if (st) return st;
    // serial coarse sweep with the correction update
    for (int s = 0; s < S; ++s) {
      WADG_HIP(hipMemcpyAsync(tmp, U + s * n1, sb, hipMemcpyDeviceToDevice, hs));
      if ((st = coarse(tmp))) return st;
      int e = wadg::launch_parareal_correct(tmp, F + s * n1, Gold + s * n1, U + (s + 1) * n1,
                                            (int64_t)n1, tile, ctx->K,
                                            partials + (size_t)s * kNormBlocks * 4, kNormBlocks,
                                            stream);
      if (e) return hip_fail((hipError_t)e, "parareal correction launch");
    }
    int e = wadg::launch_norms_final(partials, kNormBlocks, S, dout, stream);
    if (e) return hip_fail((hipError_t)e, "reduction launch");
    WADG_HIP(hipMemcpyAsync(out.data(), dout, out.size() * sizeof(double), hipMemcpyDeviceToHost,
                            hs));
    WADG_HIP(hipStreamSynchronize(hs));
    it = k + 1;
    change = 0.0;
    for (int s = 0; s < S; ++s) {
      if (out[4 * s + 3] != 0.0) {
        *iterations = it;
        *last_change = NAN;
        return fail(WADG_E_NONFINITE, "non-finite parareal iterate");
      }
      const double c = out[4 * s + 1] > 0.0 ? std::sqrt(out[4 * s] / out[4 * s + 1])
                                             : std::sqrt(out[4 * s]);
      change = c > change ? c : change;
    }
    if (change <= tol) break;
  }
  *iterations = it;
  *last_change = change;
  return WADG_OK;
}

namespace {
// Adjoint workspace: two sets of the 5 stage residuals of every step of one
// slice (one being recomputed while the other is read), two alternating
// stage states, ybar, rbar, two alternating z (one slice each), then the
// per-workgroup sensitivity partials.  (wadg_forward_checkpoints uses the
// first five slices of it.)
size_t adjoint_bytes(wadg_ctx ctx, int32_t nsteps) {
  const size_t n1 = ctx->slice_doubles();
  return (10 * (size_t)nsteps + 6) * n1 * sizeof(double) + (size_t)ctx->groups() * sizeof(double);
}

// One slice recomputed from its start state chk_s, keeping every stage
// residual r_{m,i} at R + (5 m + i) n1; stage j = 5 m + i writes T[j % 2]
// and reads what stage j - 1 wrote (chk_s for j = 0), never its own output.
int adjoint_recompute(wadg_ctx ctx, const double* chk_s, double* R, double* const (&T)[2],
                      double dt, int32_t nsteps, void* stream) {
  const size_t n1 = ctx->slice_doubles();
  wadg::StageParams p = base_params(ctx, 1);
  p.dt = dt;
  const double* cur = chk_s;
  for (int m = 0; m < nsteps; ++m) {
    for (int i = 0; i < 5; ++i) {
      double* out = T[(5 * m + i) % 2];
      p.Qin = cur;
      p.Qout = out;
      p.res = R + (5 * (size_t)m + (i == 0 ? 0 : i - 1)) * n1;
      p.res_out = R + (5 * (size_t)m + i) * n1;
      p.rkA = kRkA[i];
      p.rkB = kRkB[i];
      int e = launch_stage(ctx, wadg::kStage, false, p, stream);
      if (e) return hip_fail((hipError_t)e, "stage kernel launch");
      cur = out;
    }
  }
  return WADG_OK;
}

// One LSRK step of one slice from `in` to `out` (distinct), through t0, t1.
int one_step(wadg_ctx ctx, const double* in, double* out, double* t0, double* t1, double* res,
             double dt, void* stream) {
  wadg::StageParams p = base_params(ctx, 1);
  p.res = res;
  p.dt = dt;
  const double* cur = in;
  for (int i = 0; i < 5; ++i) {
    p.Qin = cur;
    p.Qout = i == 4 ? out : (i % 2 == 0 ? t0 : t1);
    p.rkA = kRkA[i];
    p.rkB = kRkB[i];
    int e = launch_stage(ctx, wadg::kStage, false, p, stream);
    if (e) return hip_fail((hipError_t)e, "stage kernel launch");
    cur = static_cast<const double*>(p.Qout);
  }
  return WADG_OK;
}
}  // namespace

int wadg_adjoint_workspace_bytes(wadg_ctx ctx, int32_t nsteps, size_t* bytes) {
  if (!ctx) return fail(WADG_E_INVALID, "context is NULL");
  if (!bytes) return fail(WADG_E_INVALID, "bytes is NULL");
  if (nsteps < 1) return fail(WADG_E_INVALID, "nsteps must be >= 1");
  *bytes = adjoint_bytes(ctx, nsteps);
  return WADG_OK;
}

int wadg_forward_checkpoints(wadg_ctx ctx, double* chk, void* work, int32_t S, double dt,
                             int32_t nsteps, void* stream) {
  if (!ctx) return fail(WADG_E_INVALID, "context is NULL");
  if (!chk || !work) return fail(WADG_E_INVALID, "chk and work must not be NULL");
  if (S < 1 || nsteps < 1) return fail(WADG_E_INVALID, "S >= 1 and nsteps >= 1 required");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(WADG_E_INVALID, "dt must be finite and > 0");
  const size_t n1 = ctx->slice_doubles();
  if (overlaps(chk, (S + 1) * n1 * sizeof(double), work, adjoint_bytes(ctx, nsteps)))
    return fail(WADG_E_INVALID, "work must not alias chk");
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the context's device");
  double* w = static_cast<double*>(work);
  double *t0 = w, *t1 = w + n1, *res = w + 2 * n1, *t2 = w + 3 * n1;
  for (int s = 0; s < S; ++s) {
    const double* cur = chk + s * n1;
    for (int m = 0; m < nsteps; ++m) {
      double* out = m == nsteps - 1 ? chk + (s + 1) * n1 : (m % 2 == 0 ? t2 : t0 + 4 * n1);
      int st = one_step(ctx, cur, out, t0, t1, res, dt, stream);
      if (st) return st;
      cur = out;
    }
  }
  return WADG_OK;
}

int wadg_adjoint(wadg_ctx ctx, const double* chk, const double* seed, double* grad, void* work,
                 int32_t S, double dt, int32_t nsteps, double* dJ_dscale, void* stream) {
  if (!ctx) return fail(WADG_E_INVALID, "context is NULL");
  if (!chk || !seed || !grad || !work || !dJ_dscale)
    return fail(WADG_E_INVALID, "chk, seed, grad, work and dJ_dscale must not be NULL");
  if (S < 1 || nsteps < 1) return fail(WADG_E_INVALID, "S >= 1 and nsteps >= 1 required");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(WADG_E_INVALID, "dt must be finite and > 0");
  const size_t n1 = ctx->slice_doubles();
  const size_t sb = n1 * sizeof(double);
  const size_t wb = adjoint_bytes(ctx, nsteps);
  if (overlaps(chk, (S + 1) * sb, work, wb) || overlaps(seed, sb, work, wb) ||
      overlaps(grad, sb, work, wb))
    return fail(WADG_E_INVALID, "work must not alias chk, seed or grad");
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the context's device");
  hipStream_t hs = static_cast<hipStream_t>(stream);

  double* R = static_cast<double*>(work);       // two residual sets of 5 nsteps slices
  double* const T[2] = {R + 10 * (size_t)nsteps * n1, R + (10 * (size_t)nsteps + 1) * n1};
  double* yb = T[1] + n1;
  double* rb = yb + n1;
  double* zc = rb + n1;    // z read by the next apply-A launch
  double* zn = zc + n1;    // z written by a fused apply-A + mass launch
  double* part = zn + n1;
  // With the split kernel, the mass step of reverse stage j-1 runs at the
  // end of the apply-A launch of stage j (it needs only the item's own new
  // ybar and rbar): one launch per stage instead of two, except at the
  // first stage of each slice (its residuals are recomputed just before)
  // and the last (no next stage in the slice).
  const bool fused = kernel_path(ctx, false, wadg::kApplyA) == WADG_KERNEL_SPLIT;
  const int G = ctx->groups();
  WADG_HIP(hipMemsetAsync(part, 0, (size_t)G * sizeof(double), hs));
  WADG_HIP(hipMemcpyAsync(yb, seed, sb, hipMemcpyDeviceToDevice, hs));

  wadg::StageParams p = base_params(ctx, 1);
  p.dt = dt;
  // The forward recompute of slice s-1 (on the context's second stream)
  // runs while the reverse sweep of slice s (on `stream`) reads the other
  // residual set: ev_rec[b] = residual set b is ready, ev_rev[b] = the
  // reverse sweep that read set b is done.
  if (!ctx->aux) {
    WADG_HIP(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
    for (hipEvent_t* e : {&ctx->ev_in, &ctx->ev_rec[0], &ctx->ev_rec[1], &ctx->ev_rev[0],
                          &ctx->ev_rev[1]})
      WADG_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
  }
  hipStream_t aux = ctx->aux;
  WADG_HIP(hipEventRecord(ctx->ev_in, hs));          // chk and seed are written
  WADG_HIP(hipStreamWaitEvent(aux, ctx->ev_in, 0));
  double* const Rs[2] = {R, R + 5 * (size_t)nsteps * n1};
  auto recompute = [&](int s) -> int {
    const int b = s % 2;
    if (s + 2 <= S - 1) WADG_HIP(hipStreamWaitEvent(aux, ctx->ev_rev[b], 0));
    int st = adjoint_recompute(ctx, chk + s * n1, Rs[b], T, dt, nsteps, aux);
    if (st) return st;
    WADG_HIP(hipEventRecord(ctx->ev_rec[b], aux));
    return WADG_OK;
  };
  int st = recompute(S - 1);
  if (st) return st;
  for (int s = S - 1; s >= 0; --s) {
    if (s >= 1 && (st = recompute(s - 1))) return st;
    const double* Rs_ = Rs[s % 2];
    WADG_HIP(hipStreamWaitEvent(hs, ctx->ev_rec[s % 2], 0));
    for (int m = nsteps - 1; m >= 0; --m) {
      const double* Rm = Rs_ + 5 * (size_t)m * n1;
      // reverse stages: rbar += B_i ybar; ybar += dt L^T rbar; rbar *= A_i
      for (int i = 4; i >= 0; --i) {
        int e = 0;
        if (!fused || (m == nsteps - 1 && i == 4)) {
          e = wadg::launch_adjoint_mass(ctx->N, ctx->nq1, p, rb, yb, zc, Rm + i * n1,
                                        i > 0 ? Rm + (i - 1) * n1 : nullptr,
                                        i == 4 ? 0.0 : kRkA[i + 1], kRkB[i], kRkA[i], part,
                                        stream);
          if (e) return hip_fail((hipError_t)e, "adjoint mass kernel launch");
        }
        wadg::StageParams q = p;
        q.Qin = zc;
        q.res = yb;
        q.Qout = yb;
        if (fused && (m > 0 || i > 0)) {
          // the mass step of the next reverse stage (m2, i2) of this slice
          const int m2 = i > 0 ? m : m - 1, i2 = i > 0 ? i - 1 : 4;
          const double* R2 = Rs_ + 5 * (size_t)m2 * n1;
          q.adj.rbar = rb;
          q.adj.z = zn;
          q.adj.r = R2 + i2 * n1;
          q.adj.r_prev = i2 > 0 ? R2 + (i2 - 1) * n1 : nullptr;
          q.adj.part = part;
          q.adj.a_next = i2 == 4 ? 0.0 : kRkA[i2 + 1];
          q.adj.b = kRkB[i2];
          q.adj.a = kRkA[i2];
          e = launch_stage(ctx, wadg::kApplyAMass, false, q, stream);
          std::swap(zc, zn);
        } else {
          e = launch_stage(ctx, wadg::kApplyA, false, q, stream);
        }
        if (e) return hip_fail((hipError_t)e, "stage kernel launch (apply A)");
      }
    }
    WADG_HIP(hipEventRecord(ctx->ev_rev[s % 2], hs));
  }
  if (grad != yb) WADG_HIP(hipMemcpyAsync(grad, yb, sb, hipMemcpyDeviceToDevice, hs));
  std::vector<double> h(G);
  WADG_HIP(hipMemcpyAsync(h.data(), part, (size_t)G * sizeof(double), hipMemcpyDeviceToHost, hs));
  WADG_HIP(hipStreamSynchronize(hs));
  double acc = 0.0;
  for (int g = 0; g < G; ++g) acc += h[g];
  *dJ_dscale = acc;
  if (!std::isfinite(acc)) return fail(WADG_E_NONFINITE, "non-finite sensitivity");
  return WADG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of independent problems.

struct wadg_batch_s {
  int device = 0, N = 0, nq1 = 0, cus = 256, nprob = 0;
  double tau_p = 1.0, tau_u = 1.0;
  std::vector<int32_t> pack, K, S;            // per problem: copies per lane group, elements, slices
  std::vector<int32_t> Kv, Sv, nEG, g0;       // packed (virtual) mesh and its slices
  std::vector<int64_t> offset;                 // [nprob + 1] state offsets in doubles
  std::vector<double> dt;                      // per problem (last uploaded)
  int64_t groups = 0, items = 0;
  double* d_vol = nullptr;
  double* d_face = nullptr;
  int32_t* d_nbr = nullptr;
  wadg::BatchProb* d_prob = nullptr;
  int32_t* d_items = nullptr;
  int grid_mult = 0;                           // persistent workgroups per CU (0: one per item)
  int order = 0;                               // 0 problem-major, 1 interleaved
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void free_batch(wadg_batch b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  for (void* ptr : {(void*)b->d_vol, (void*)b->d_face, (void*)b->d_nbr, (void*)b->d_prob,
                    (void*)b->d_items})
    if (ptr) (void)hipFree(ptr);
  delete b;
}

// Work list in the current order: problem-major (all items of problem 0,
// then problem 1, ...) or interleaved (round-robin over problems, one slice
// of each at a time).
std::vector<int32_t> batch_items(const wadg_batch b) {
  std::vector<int32_t> it;
  it.reserve(2 * b->items);
  if (b->order == 0) {
    for (int i = 0; i < b->nprob; ++i)
      for (int l = 0; l < b->Sv[i] * b->nEG[i]; ++l) {
        it.push_back(i);
        it.push_back(l);
      }
  } else {
    int smax = 0;
    for (int i = 0; i < b->nprob; ++i) smax = std::max(smax, b->Sv[i]);
    for (int s = 0; s < smax; ++s)
      for (int i = 0; i < b->nprob; ++i)
        if (s < b->Sv[i])
          for (int g = 0; g < b->nEG[i]; ++g) {
            it.push_back(i);
            it.push_back(s * b->nEG[i] + g);
          }
  }
  return it;
}

int batch_upload_items(wadg_batch b) {
  std::vector<int32_t> it = batch_items(b);
  WADG_HIP(hipMemcpy(b->d_items, it.data(), it.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  return WADG_OK;
}

int batch_upload_dt(wadg_batch b, const double* dt) {
  bool same = !b->dt.empty();
  for (int i = 0; same && i < b->nprob; ++i) same = b->dt[i] == dt[i];
  if (same) return WADG_OK;
  std::vector<wadg::BatchProb> pr(b->nprob);
  for (int i = 0; i < b->nprob; ++i) {
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i]))
      return fail(WADG_E_INVALID, "dt[" + std::to_string(i) + "] must be finite and > 0");
    pr[i] = wadg::BatchProb{b->offset[i], b->nEG[i], b->Sv[i], b->Kv[i], b->g0[i], dt[i]};
  }
  WADG_HIP(hipMemcpy(b->d_prob, pr.data(), pr.size() * sizeof(wadg::BatchProb),
                     hipMemcpyHostToDevice));
  b->dt.assign(dt, dt + b->nprob);
  return WADG_OK;
}

int batch_grid(const wadg_batch b) {
  if (b->grid_mult == 0 || (int64_t)b->grid_mult * b->cus >= b->items) return (int)b->items;
  return b->grid_mult * b->cus;
}

int batch_stage(wadg_batch b, const double* qin, double* qout, double* res, int i, void* stream) {
  wadg::BatchParams p{};
  p.prob = b->d_prob;
  p.items = b->d_items;
  p.nitems = (int32_t)b->items;
  p.Qin = qin;
  p.Qout = qout;
  p.res = res;
  p.vol = b->d_vol;
  p.face = b->d_face;
  p.nbr = b->d_nbr;
  p.tau_p = b->tau_p;
  p.tau_u = b->tau_u;
  p.rkA = kRkA[i];
  p.rkB = kRkB[i];
  // one workgroup per item: the split-work kernel; persistent workgroups:
  // the streamed kernel (wadg_batch_set_schedule)
  int e = b->grid_mult == 0 ? wadg::launch_batch_split(b->N, b->nq1, p, stream)
                            : wadg::launch_batch_stage(b->N, b->nq1, p, batch_grid(b), stream);
  if (e) return hip_fail((hipError_t)e, "batch stage kernel launch");
  return WADG_OK;
}

int batch_sweep(wadg_batch b, double* Q, double* work, int32_t nsteps, void* stream) {
  const size_t n = (size_t)b->offset[b->nprob];
  double* res = work;
  double* other = work + n;
  double* cur = Q;
  for (int stp = 0; stp < nsteps; ++stp)
    for (int i = 0; i < 5; ++i) {
      double* out = cur == Q ? other : Q;
      int st = batch_stage(b, cur, out, res, i, stream);
      if (st) return st;
      cur = out;
    }
  if (cur != Q) {   // a kernel, not a runtime copy: the sweep is captured into graphs
    int e = wadg::launch_copy(cur, Q, n, stream);
    if (e) return hip_fail((hipError_t)e, "copy kernel launch");
  }
  return WADG_OK;
}

}  // namespace

extern "C" {

int wadg_batch_create(const wadg_mesh* meshes, int32_t nprob, const int32_t* S, int32_t device,
                      wadg_batch* out) {
  if (!out) return fail(WADG_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!meshes || !S || nprob < 1) return fail(WADG_E_INVALID, "meshes, S and nprob >= 1 required");
  const int N = meshes[0].N, nq = meshes[0].nq1;
  if (!wadg::stage_supported(N, nq))
    return fail(WADG_E_UNSUPPORTED, "degree / quadrature not compiled in");
  wadg::RefOps ops;
  std::string err;
  if (!wadg::build_ref_ops(N, nq, &ops, &err)) return fail(WADG_E_UNSUPPORTED, err);
  wadg_batch b = new wadg_batch_s();
  b->N = N;
  b->nq1 = nq;
  b->nprob = nprob;
  b->tau_p = meshes[0].tau_p;
  b->tau_u = meshes[0].tau_u;
  const int Np = (N + 1) * (N + 1);
  const size_t tile = (size_t)3 * Np * wadg::kWave;
  std::vector<double> vol, face;
  std::vector<int32_t> nbr;
  b->offset.push_back(0);
  for (int i = 0; i < nprob; ++i) {
    const wadg_mesh& m = meshes[i];
    int st = check_mesh(&m);
    if (st) {
      free_batch(b);
      return fail(st, "problem " + std::to_string(i) + ": " + g_last_error);
    }
    if (m.N != N || m.nq1 != nq || m.tau_p != b->tau_p || m.tau_u != b->tau_u) {
      free_batch(b);
      return fail(WADG_E_INVALID, "all problems of a batch share N, nq1, tau_p and tau_u");
    }
    if (S[i] < 1) {
      free_batch(b);
      return fail(WADG_E_INVALID, "S[" + std::to_string(i) + "] must be >= 1");
    }
    // meshes of at most half a lane group carry several slices side by side
    const int P = m.K <= wadg::kWave / 2 ? wadg::kWave / m.K : 1;
    const int Kv = P * m.K;
    std::vector<double> x((size_t)Kv * Np), y((size_t)Kv * Np), c2;
    std::vector<int32_t> etoe((size_t)Kv * 4), etof((size_t)Kv * 4);
    const int nqq = nq * nq;
    if (m.c2q) c2.resize((size_t)Kv * nqq);
    for (int j = 0; j < P; ++j) {
      std::memcpy(&x[(size_t)j * m.K * Np], m.x, sizeof(double) * m.K * Np);
      std::memcpy(&y[(size_t)j * m.K * Np], m.y, sizeof(double) * m.K * Np);
      for (int k = 0; k < m.K * 4; ++k) {
        etoe[(size_t)j * m.K * 4 + k] = m.etoe[k] + j * m.K;
        etof[(size_t)j * m.K * 4 + k] = m.etof[k];
      }
      if (m.c2q) std::memcpy(&c2[(size_t)j * m.K * nqq], m.c2q, sizeof(double) * m.K * nqq);
    }
    wadg::MeshIn mi{N, nq, Kv, x.data(), y.data(), etoe.data(), etof.data(),
                    m.c2q ? c2.data() : nullptr};
    std::vector<double> v0, f0;
    std::vector<int32_t> n0;
    int g = wadg::build_geometry(mi, ops, &v0, &f0, &n0, &err);
    if (g) {
      free_batch(b);
      return fail(g == -1 ? WADG_E_INVALID : WADG_E_GEOMETRY,
                  "problem " + std::to_string(i) + ": " + err);
    }
    std::vector<double> vt = wadg::tile_planes(v0, 6 * nqq, Kv);
    std::vector<double> ft = wadg::tile_planes(f0, 12 * nq, Kv);
    std::vector<int32_t> nt = wadg::tile_planes(n0, 8, Kv);
    vol.insert(vol.end(), vt.begin(), vt.end());
    face.insert(face.end(), ft.begin(), ft.end());
    nbr.insert(nbr.end(), nt.begin(), nt.end());
    const int nEG = (Kv + wadg::kWave - 1) / wadg::kWave;
    const int Sv = (S[i] + P - 1) / P;
    b->pack.push_back(P);
    b->K.push_back(m.K);
    b->S.push_back(S[i]);
    b->Kv.push_back(Kv);
    b->Sv.push_back(Sv);
    b->nEG.push_back(nEG);
    b->g0.push_back((int32_t)b->groups);
    b->groups += nEG;
    b->items += (int64_t)Sv * nEG;
    b->offset.push_back(b->offset.back() + (int64_t)Sv * nEG * (int64_t)tile);
  }
  if (b->items >= (1LL << 31) || b->groups >= (1LL << 31)) {
    free_batch(b);
    return fail(WADG_E_INVALID, "batch too large");
  }
  int dev = device;
  if (dev < 0 && hipGetDevice(&dev) != hipSuccess) {
    free_batch(b);
    return fail(WADG_E_DEVICE, "no current HIP device");
  }
  DeviceGuard guard(dev);
  if (!guard.ok) {
    free_batch(b);
    return fail(WADG_E_DEVICE, "cannot select HIP device " + std::to_string(dev));
  }
  b->device = dev;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      cus > 0)
    b->cus = cus;
  hipError_t e;
  if ((e = hipMalloc(&b->d_vol, vol.size() * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&b->d_face, face.size() * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&b->d_nbr, nbr.size() * sizeof(int32_t))) != hipSuccess ||
      (e = hipMalloc(&b->d_prob, (size_t)nprob * sizeof(wadg::BatchProb))) != hipSuccess ||
      (e = hipMalloc(&b->d_items, (size_t)b->items * 2 * sizeof(int32_t))) != hipSuccess ||
      (e = hipMemcpy(b->d_vol, vol.data(), vol.size() * sizeof(double),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b->d_face, face.data(), face.size() * sizeof(double),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b->d_nbr, nbr.data(), nbr.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice)) != hipSuccess) {
    free_batch(b);
    return hip_fail(e, "wadg_batch_create device setup");
  }
  int st = batch_upload_items(b);
  if (st) {
    free_batch(b);
    return st;
  }
  *out = b;
  return WADG_OK;
}

void wadg_batch_destroy(wadg_batch b) {
  if (!b) return;
  DeviceGuard guard(b->device);
  free_batch(b);
}

int wadg_batch_layout(wadg_batch b, int64_t* offset, int32_t* pack) {
  if (!b) return fail(WADG_E_INVALID, "batch is NULL");
  if (offset) std::memcpy(offset, b->offset.data(), (b->nprob + 1) * sizeof(int64_t));
  if (pack) std::memcpy(pack, b->pack.data(), b->nprob * sizeof(int32_t));
  return WADG_OK;
}

int wadg_batch_workspace_bytes(wadg_batch b, size_t* bytes) {
  if (!b) return fail(WADG_E_INVALID, "batch is NULL");
  if (!bytes) return fail(WADG_E_INVALID, "bytes is NULL");
  *bytes = 2 * (size_t)b->offset[b->nprob] * sizeof(double);
  return WADG_OK;
}

int wadg_batch_integrate(wadg_batch b, double* Q, double* work, const double* dt, int32_t nsteps,
                         void* stream) {
  if (!b) return fail(WADG_E_INVALID, "batch is NULL");
  if (!Q || !work || !dt) return fail(WADG_E_INVALID, "Q, work and dt must not be NULL");
  if (nsteps < 0) return fail(WADG_E_INVALID, "nsteps must be >= 0");
  const size_t n = (size_t)b->offset[b->nprob];
  if (overlaps(Q, n * sizeof(double), work, 2 * n * sizeof(double)))
    return fail(WADG_E_INVALID, "work must not alias Q");
  if (nsteps == 0) return WADG_OK;
  DeviceGuard guard(b->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the batch's device");
  int st = batch_upload_dt(b, dt);
  if (st) return st;
  return batch_sweep(b, Q, work, nsteps, stream);
}

int wadg_batch_set_schedule(wadg_batch b, int32_t wg_per_cu, int32_t order) {
  if (!b) return fail(WADG_E_INVALID, "batch is NULL");
  if (wg_per_cu < 0 || wg_per_cu > 64 || (order != 0 && order != 1))
    return fail(WADG_E_INVALID, "wg_per_cu in [0, 64] and order in {0, 1} required");
  if (b->exec) return fail(WADG_E_INVALID, "release the captured graph first");
  DeviceGuard guard(b->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the batch's device");
  b->grid_mult = wg_per_cu;
  if (order != b->order) {
    b->order = order;
    int st = batch_upload_items(b);
    if (st) return st;
  }
  return WADG_OK;
}

int wadg_batch_tune(wadg_batch b, const double* Q, double* work, const double* dt, int32_t reps,
                    int32_t* wg_per_cu, int32_t* order, double* best_us, void* stream) {
  if (!b) return fail(WADG_E_INVALID, "batch is NULL");
  if (!Q || !work || !dt || !wg_per_cu || !order || !best_us)
    return fail(WADG_E_INVALID, "Q, work, dt and the outputs must not be NULL");
  if (reps < 1) return fail(WADG_E_INVALID, "reps must be >= 1");
  if (b->exec) return fail(WADG_E_INVALID, "release the captured graph first");
  const size_t n = (size_t)b->offset[b->nprob];
  if (overlaps(Q, n * sizeof(double), work, 2 * n * sizeof(double)))
    return fail(WADG_E_INVALID, "work must not alias Q");
  DeviceGuard guard(b->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the batch's device");
  int st = batch_upload_dt(b, dt);
  if (st) return st;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(hipErrorUnknown, "hipEventCreate");
  }
  // candidates: persistent grids of 1, 2, 4, 8 two-wave workgroups per CU
  // (streamed kernel) or one four-wave workgroup per item (split kernel), in
  // both item orders; each timed on a stage with a residual read (Q is only
  // read, the workspace is scratch)
  const int mults[] = {1, 2, 4, 8, 0};
  double best = 1e300;
  const int m0 = b->grid_mult, o0 = b->order;
  int bm = m0, bo = o0;
  for (int o = 0; o < 2 && !st; ++o) {
    for (int m : mults) {
      if ((st = wadg_batch_set_schedule(b, m, o))) break;
      if ((st = batch_stage(b, Q, work, work + n, 1, stream))) break;
      if (hipEventRecord(e0, hs) != hipSuccess) { st = hip_fail(hipErrorUnknown, "event"); break; }
      for (int r = 0; r < reps && !st; ++r) st = batch_stage(b, Q, work, work + n, 1, stream);
      if (st) break;
      float ms = 0.f;
      if (hipEventRecord(e1, hs) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = hip_fail(hipErrorUnknown, "event timing");
        break;
      }
      const double us = 1e3 * ms / reps;
      if (us < best) {
        best = us;
        bm = m;
        bo = o;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) {
    (void)wadg_batch_set_schedule(b, m0, o0);   // leave the schedule as it was
    return st;
  }
  if ((st = wadg_batch_set_schedule(b, bm, bo))) return st;
  *wg_per_cu = bm;
  *order = bo;
  *best_us = best;
  return WADG_OK;
}

int wadg_batch_capture(wadg_batch b, double* Q, double* work, const double* dt, int32_t nsteps) {
  if (!b) return fail(WADG_E_INVALID, "batch is NULL");
  if (!Q || !work || !dt || nsteps < 1)
    return fail(WADG_E_INVALID, "Q, work, dt and nsteps >= 1 required");
  const size_t n = (size_t)b->offset[b->nprob];
  if (overlaps(Q, n * sizeof(double), work, 2 * n * sizeof(double)))
    return fail(WADG_E_INVALID, "work must not alias Q");
  DeviceGuard guard(b->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the batch's device");
  int st = batch_upload_dt(b, dt);
  if (st) return st;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  if (!b->capture_stream)
    WADG_HIP(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
  WADG_HIP(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
  st = batch_sweep(b, Q, work, nsteps, b->capture_stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->capture_stream, &g);
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  b->graph = g;
  WADG_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return WADG_OK;
}

int wadg_batch_replay(wadg_batch b, void* stream) {
  if (!b) return fail(WADG_E_INVALID, "batch is NULL");
  if (!b->exec) return fail(WADG_E_INVALID, "no captured sweep (wadg_batch_capture)");
  DeviceGuard guard(b->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the batch's device");
  WADG_HIP(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
  return WADG_OK;
}

int wadg_batch_release_graph(wadg_batch b) {
  if (!b) return fail(WADG_E_INVALID, "batch is NULL");
  DeviceGuard guard(b->device);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  return WADG_OK;
}

int wadg_norms(wadg_ctx ctx, const double* A, const double* B, int32_t S, double* out,
               void* stream) {
  int st = check_slices(ctx, S);
  if (st) return st;
  if (!A || !out) return fail(WADG_E_INVALID, "A and out must not be NULL");
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the context's device");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  if (S > ctx->norms_cap) {
    // scratch grows with the largest S seen; the stream is drained first so
    // that no queued reduction still reads the old buffers
    WADG_HIP(hipStreamSynchronize(hs));
    if (ctx->d_partials) (void)hipFree(ctx->d_partials);
    if (ctx->d_out) (void)hipFree(ctx->d_out);
    ctx->d_partials = nullptr;
    ctx->d_out = nullptr;
    ctx->norms_cap = 0;
    WADG_HIP(hipMalloc(&ctx->d_partials, (size_t)S * kNormBlocks * 4 * sizeof(double)));
    WADG_HIP(hipMalloc(&ctx->d_out, (size_t)S * 4 * sizeof(double)));
    ctx->norms_cap = S;
  }
  const int64_t per = (int64_t)ctx->slice_doubles();
  int e = wadg::launch_norms(A, B, S, per, (int32_t)ctx->tile(), ctx->K, ctx->d_partials,
                             kNormBlocks, ctx->d_out, stream);
  if (e) return hip_fail((hipError_t)e, "norms kernel launch");
  WADG_HIP(hipMemcpyAsync(out, ctx->d_out, (size_t)S * 4 * sizeof(double),
                          hipMemcpyDeviceToHost, hs));
  WADG_HIP(hipStreamSynchronize(hs));
  bool all_finite = true;
  for (int s = 0; s < S; ++s) {
    out[4 * s + 0] = std::sqrt(out[4 * s + 0]);
    out[4 * s + 1] = std::sqrt(out[4 * s + 1]);
    if (out[4 * s + 3] != 0.0) all_finite = false;
    out[4 * s + 3] = out[4 * s + 3] != 0.0 ? 0.0 : 1.0;
  }
  if (!all_finite) return fail(WADG_E_NONFINITE, "non-finite entries in A");
  return WADG_OK;
}

const char* wadg_status_string(int status) {
  switch (status) {
    case WADG_OK: return "ok";
    case WADG_E_INVALID: return "invalid argument";
    case WADG_E_GEOMETRY: return "invalid geometry";
    case WADG_E_UNSUPPORTED: return "unsupported degree or quadrature";
    case WADG_E_DEVICE: return "HIP device error";
    case WADG_E_NONFINITE: return "non-finite values";
    default: return "unknown status";
  }
}

const char* wadg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
