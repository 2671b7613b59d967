// C ABI of the WADG sweep (declared in include/wadg.h): validation, host
// setup, device memory of the context, the sweep (right-hand side, LSRK
// stages, FP32-bulk, parareal) and the norms.  The adjoint and the batches
// are in api_adjoint.hip and api_batch.hip, the stage-launch policy in
// launch.hip.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "api_internal.h"

namespace wadg {
namespace host {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(WADG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

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

void mesh_scales(const double* vol, const double* face, int K, int nq, const double* wq,
                 bool tiled, double* h_min, double* c2_max) {
  const int nqq = nq * nq;
  const int KB = wadg::kWave;
  // value of plane p (of P planes) of element k
  auto at = [&](const double* a, int P, int p, int k) {
    return tiled ? a[((size_t)(k / KB) * P + p) * KB + k % KB] : a[(size_t)p * K + k];
  };
  double h = INFINITY, c2 = 0.0;
  for (int k = 0; k < K; ++k) {
    double area = 0.0, perim = 0.0;
    for (int q = 0; q < nqq; ++q) {
      const double rJ = at(vol, 6 * nqq, 5 * nqq + q, k);      // 1/J
      area += wq[q % nq] * wq[q / nq] / rJ;
      c2 = std::max(c2, at(vol, 6 * nqq, 4 * nqq + q, k) / rJ);
    }
    for (int f = 0; f < 4; ++f)
      for (int j = 0; j < nq; ++j) perim += at(face, 12 * nq, 2 * 4 * nq + f * nq + j, k);
    h = std::min(h, 4.0 * area / perim);
  }
  *h_min = h;
  *c2_max = c2;
}

int check_slices(wadg_ctx c, int32_t S) {
  if (!c) return fail(WADG_E_INVALID, "context is NULL");
  if (S < 1) return fail(WADG_E_INVALID, "S must be >= 1");
  const long long nEG = (c->K + wadg::kWave - 1) / wadg::kWave;
  if (nEG * (long long)S >= (1LL << 31)) return fail(WADG_E_INVALID, "too many slices");
  return WADG_OK;
}

}  // namespace host
}  // namespace wadg

using namespace wadg::host;

namespace {

constexpr int kNormBlocks = 64;

// Scratch of wadg_norms_noalloc: the 64 x 4 partial sums and the 4 sums of
// up to WADG_NORMS_NOALLOC_MAX_S slices.  Host code never uses this name as
// an address: each device's copy is reached through the address that
// hipGetSymbolAddress returns with that device current (noalloc_scratch).
constexpr size_t kNoallocDoubles = (size_t)WADG_NORMS_NOALLOC_MAX_S * (kNormBlocks * 4 + 4);
static __device__ __align__(256) double scratch[kNoallocDoubles];

// The device address of `scratch` on device `dev`, which must be current;
// looked up once per device and kept until the process ends.
int noalloc_scratch(int dev, double** out) {
  static std::mutex mu;
  static std::map<int, double*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                               "hipGetSymbolAddress(norms scratch)");
    it = addr.emplace(dev, static_cast<double*>(p)).first;
  }
  *out = it->second;
  return WADG_OK;
}

void free_ctx(wadg_ctx c) {
  if (!c) return;
  if (c->d_vol) (void)hipFree(c->d_vol);
  if (c->d_face) (void)hipFree(c->d_face);
  if (c->d_vol32) (void)hipFree(c->d_vol32);
  if (c->d_face32) (void)hipFree(c->d_face32);
  if (c->d_nbr) (void)hipFree(c->d_nbr);
  for (hipEvent_t e : {c->ev_in, c->ev_rec[0], c->ev_rec[1], c->ev_rev[0], c->ev_rev[1]})
    if (e) (void)hipEventDestroy(e);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  delete c;
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
  int g = wadg::build_geometry(mesh_in(mesh), ops, vol, face, nullptr, false, &err);
  if (g) return fail(g == -1 ? WADG_E_INVALID : WADG_E_GEOMETRY, err);
  return WADG_OK;
}

int wadg_cfl_number(const wadg_mesh* mesh, double dt, double c2_scale, double* nu) {
  int st = check_mesh(mesh);
  if (st) return st;
  if (!nu) return fail(WADG_E_INVALID, "nu is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt) || !(c2_scale > 0.0) || !std::isfinite(c2_scale))
    return fail(WADG_E_INVALID, "dt and c2_scale must be finite and > 0");
  wadg::RefOps ops;
  std::string err;
  if (!wadg::build_ref_ops(mesh->N, mesh->nq1, &ops, &err)) return fail(WADG_E_UNSUPPORTED, err);
  const size_t nq = mesh->nq1, K = mesh->K;
  std::vector<double> vol(6 * nq * nq * K), face(12 * nq * K);
  int g = wadg::build_geometry(mesh_in(mesh), ops, vol.data(), face.data(), nullptr, false, &err);
  if (g) return fail(g == -1 ? WADG_E_INVALID : WADG_E_GEOMETRY, err);
  double h = 0.0, c2 = 0.0;
  mesh_scales(vol.data(), face.data(), mesh->K, mesh->nq1, ops.wq, false, &h, &c2);
  *nu = cfl_number(dt, mesh->N, h, c2 * c2_scale);
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
  // geometry straight into the tiled device layout (no untiled copy); its
  // FP32 copy for the FP32-bulk path is rounded on the device
  const int nq = mesh->nq1;
  const size_t G = ((size_t)mesh->K + wadg::kWave - 1) / wadg::kWave;
  const size_t nv = G * 6 * nq * nq * wadg::kWave, nf = G * 12 * nq * wadg::kWave,
               nn = G * 8 * wadg::kWave;
  std::unique_ptr<double[]> vol(new double[nv]), face(new double[nf]);
  std::unique_ptr<int32_t[]> nbr(new int32_t[nn]);
  int g = wadg::build_geometry(mesh_in(mesh), ops, vol.get(), face.get(), nbr.get(), true, &err);
  if (g) return fail(g == -1 ? WADG_E_INVALID : WADG_E_GEOMETRY, err);

  double h_min = 0.0, c2_max = 0.0;
  mesh_scales(vol.get(), face.get(), mesh->K, nq, ops.wq, true, &h_min, &c2_max);

  int dev = device;
  if (dev < 0) WADG_HIP(hipGetDevice(&dev));
  DeviceGuard guard(dev);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select HIP device " + std::to_string(dev));

  wadg_ctx c = new wadg_ctx_s();
  c->h_min = h_min;
  c->c2_max = c2_max;
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
  if ((e = hipMalloc(&c->d_vol, nv * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&c->d_face, nf * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&c->d_nbr, nn * sizeof(int32_t))) != hipSuccess ||
      (e = hipMemcpy(c->d_vol, vol.get(), nv * sizeof(double), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(c->d_face, face.get(), nf * sizeof(double), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(c->d_nbr, nbr.get(), nn * sizeof(int32_t), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMalloc(&c->d_vol32, nv * sizeof(float))) != hipSuccess ||
      (e = hipMalloc(&c->d_face32, nf * sizeof(float))) != hipSuccess ||
      (e = (hipError_t)wadg::launch_to_fp32(c->d_vol, c->d_vol32, nv, nullptr)) != hipSuccess ||
      (e = (hipError_t)wadg::launch_to_fp32(c->d_face, c->d_face32, nf, nullptr)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(nullptr)) != hipSuccess) {
    free_ctx(c);
    return hip_fail(e, "wadg_create device setup");
  }
  if ((st = noalloc_scratch(dev, &c->d_noalloc)) != WADG_OK) {
    free_ctx(c);
    return st;
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
      kernel != WADG_KERNEL_RESIDENT && kernel != WADG_KERNEL_SPLIT &&
      kernel != WADG_KERNEL_PIPE)
    return fail(WADG_E_INVALID, "unknown kernel variant");
  if (kernel == WADG_KERNEL_RESIDENT && !wadg::resident_supported(ctx->N, ctx->nq1, false))
    return fail(WADG_E_UNSUPPORTED, "the element group's geometry does not fit in LDS");
  if (kernel == WADG_KERNEL_PIPE && !wadg::pipe_supported(ctx->N, ctx->nq1, false))
    return fail(WADG_E_UNSUPPORTED, "the pipelined kernel's tiles do not fit in LDS");
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
  *kernel = kernel_path(ctx, fp32 != 0, rhs ? wadg::kRhs : wadg::kStage, INT32_MAX);
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
      p.res_dead = i == 4;
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
      p.res_dead = i == 4;
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
  const double dtc = dt * nsteps_fine / nsteps_coarse;
  const double nu_c = cfl_number(dtc, ctx->N, ctx->h_min, ctx->c2_max * ctx->c2_scale);
  if (!(nu_c <= WADG_CFL_MAX))
    return fail(WADG_E_INVALID, "coarse step dt * nsteps_fine / nsteps_coarse has CFL number " +
                                    std::to_string(nu_c) + " > " + std::to_string(WADG_CFL_MAX) +
                                    ": raise nsteps_coarse");
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

size_t norms_scratch_doubles(int32_t S) { return (size_t)S * (kNormBlocks * 4 + 4); }
size_t l2_scratch_doubles(wadg_ctx ctx, int32_t S) {
  return ((size_t)S * ctx->groups() + S) * 2;
}

// Caller-owned device scratch of a reduction: present, 8-byte aligned, at
// least `need` doubles and not overlapping the operands.
int check_scratch(const void* scratch, size_t bytes, size_t need, const double* A,
                  const double* B, size_t nA) {
  if (!scratch) return fail(WADG_E_INVALID, "scratch must not be NULL");
  if (reinterpret_cast<uintptr_t>(scratch) % alignof(double))
    return fail(WADG_E_INVALID, "scratch must be 8-byte aligned");
  if (bytes < need * sizeof(double))
    return fail(WADG_E_INVALID, "scratch holds " + std::to_string(bytes) + " bytes; " +
                                    std::to_string(need * sizeof(double)) + " needed");
  const size_t sb = need * sizeof(double);
  if (overlaps(scratch, sb, A, nA) || (B && overlaps(scratch, sb, B, nA)))
    return fail(WADG_E_INVALID, "scratch must not overlap A or B");
  return WADG_OK;
}

// Square roots and the finite flag of the S x 4 sums of a norms launch.
int finish_norms(int32_t S, double* out) {
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

// The reduction of wadg_norms into device scratch `partials` (S x 64 x 4)
// and `dout` (S x 4), then the sums copied to `out` (synchronises).
int run_norms(wadg_ctx ctx, const double* A, const double* B, int32_t S, double* partials,
              double* dout, double* out, void* stream) {
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const int64_t per = (int64_t)ctx->slice_doubles();
  int e = wadg::launch_norms(A, B, S, per, (int32_t)ctx->tile(), ctx->K, partials, kNormBlocks,
                             dout, stream);
  if (e) return hip_fail((hipError_t)e, "norms kernel launch");
  WADG_HIP(hipMemcpyAsync(out, dout, (size_t)S * 4 * sizeof(double), hipMemcpyDeviceToHost, hs));
  WADG_HIP(hipStreamSynchronize(hs));
  return finish_norms(S, out);
}

int check_norms_args(wadg_ctx ctx, const double* A, int32_t S, const double* out) {
  int st = check_slices(ctx, S);
  if (st) return st;
  if (!A || !out) return fail(WADG_E_INVALID, "A and out must not be NULL");
  if ((int64_t)S * kNormBlocks > INT32_MAX)
    return fail(WADG_E_INVALID, "too many slices for one reduction (S * 64 must stay below 2^31)");
  return WADG_OK;
}

}  // namespace

int wadg_norms_workspace_bytes(wadg_ctx ctx, int32_t S, size_t* bytes) {
  int st = check_slices(ctx, S);
  if (st) return st;
  if (!bytes) return fail(WADG_E_INVALID, "bytes is NULL");
  if ((int64_t)S * kNormBlocks > INT32_MAX)
    return fail(WADG_E_INVALID, "too many slices for one reduction (S * 64 must stay below 2^31)");
  *bytes = norms_scratch_doubles(S) * sizeof(double);
  return WADG_OK;
}

int wadg_norms(wadg_ctx ctx, const double* A, const double* B, int32_t S, void* scratch,
               size_t scratch_bytes, double* out, void* stream) {
  int st = check_norms_args(ctx, A, S, out);
  if (st) return st;
  if ((st = check_scratch(scratch, scratch_bytes, norms_scratch_doubles(S), A, B,
                          ctx->state_doubles(S) * sizeof(double))))
    return st;
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the context's device");
  double* partials = static_cast<double*>(scratch);
  return run_norms(ctx, A, B, S, partials, partials + (size_t)S * kNormBlocks * 4, out, stream);
}

int wadg_norms_noalloc(wadg_ctx ctx, const double* A, const double* B, int32_t S, double* out,
                       void* stream) {
  int st = check_norms_args(ctx, A, S, out);
  if (st) return st;
  if (S > WADG_NORMS_NOALLOC_MAX_S)
    return fail(WADG_E_INVALID, "S = " + std::to_string(S) + " exceeds the static scratch (" +
                                    std::to_string(WADG_NORMS_NOALLOC_MAX_S) +
                                    " slices); use wadg_norms with caller scratch");
  if (!ctx->d_noalloc) return fail(WADG_E_DEVICE, "the context has no static norms scratch");
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the context's device");
  double* partials = ctx->d_noalloc;
  return run_norms(ctx, A, B, S, partials, partials + (size_t)S * kNormBlocks * 4, out, stream);
}

int wadg_l2_norms_workspace_bytes(wadg_ctx ctx, int32_t S, size_t* bytes) {
  int st = check_slices(ctx, S);
  if (st) return st;
  if (!bytes) return fail(WADG_E_INVALID, "bytes is NULL");
  *bytes = l2_scratch_doubles(ctx, S) * sizeof(double);
  return WADG_OK;
}

int wadg_l2_norms(wadg_ctx ctx, const double* A, const double* B, int32_t S, void* scratch,
                  size_t scratch_bytes, double* out, void* stream) {
  int st = check_slices(ctx, S);
  if (st) return st;
  if (!A || !out) return fail(WADG_E_INVALID, "A and out must not be NULL");
  if ((st = check_scratch(scratch, scratch_bytes, l2_scratch_doubles(ctx, S), A, B,
                          ctx->state_doubles(S) * sizeof(double))))
    return st;
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the context's device");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const int32_t nEG = ctx->groups();
  double* partials = static_cast<double*>(scratch);
  double* dout = partials + (size_t)S * nEG * 2;
  int e = wadg::launch_l2_norms(ctx->N, ctx->nq1, A, B, ctx->d_vol, S, nEG, ctx->K, partials,
                                dout, stream);
  if (e) return hip_fail((hipError_t)e, "L2 norms kernel launch");
  WADG_HIP(hipMemcpyAsync(out, dout, (size_t)S * 2 * sizeof(double), hipMemcpyDeviceToHost, hs));
  WADG_HIP(hipStreamSynchronize(hs));
  bool finite = true;
  for (int s = 0; s < 2 * S; ++s) {
    out[s] = std::sqrt(out[s]);
    if (!std::isfinite(out[s])) finite = false;
  }
  if (!finite) return fail(WADG_E_NONFINITE, "an L2 norm is not finite");
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
