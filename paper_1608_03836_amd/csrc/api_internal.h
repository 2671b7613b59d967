// Host-side internals shared by the sources of the C ABI: the context,
// error reporting, device selection, argument checks and the stage-launch
// policy (launch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "wadg.h"
#include "wadg_internal.h"

struct wadg_ctx_s {
  int device = 0;
  int N = 0, nq1 = 0, K = 0;
  double tau_p = 1.0, tau_u = 1.0;
  int tile_groups = 8;   // schedule: element groups per tile
  int tile_slices = 0;   // slices per tile (0: all)
  int kernel = WADG_KERNEL_AUTO;
  int cus = 256;         // compute units of the device
  double c2_scale = 1.0; // multiplies c^2 (wadg_set_c2_scale)
  double h_min = 0.0;    // min over elements of 4 area / perimeter (mesh_scales)
  double c2_max = 0.0;   // max of c^2 over the volume points (unscaled)
  unsigned order_flip = 0;  // item order of the next stage launch (launch_stage)
  double* d_vol = nullptr;
  double* d_face = nullptr;
  float* d_vol32 = nullptr;      // geometry rounded to FP32 (FP32-bulk path)
  float* d_face32 = nullptr;
  int32_t* d_nbr = nullptr;
  double* d_noalloc = nullptr;    // this device's static norms scratch (not owned)
  // adjoint: a second stream (default priority) for the forward recompute
  // that overlaps the reverse sweep, and the events that order the two
  hipStream_t aux = nullptr;
  hipEvent_t ev_in = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};
  int groups() const { return (K + wadg::kWave - 1) / wadg::kWave; }
  size_t tile() const { return (size_t)3 * (N + 1) * (N + 1) * wadg::kWave; }
  size_t slice_doubles() const { return (size_t)groups() * tile(); }
  size_t state_doubles(int32_t S) const { return (size_t)S * slice_doubles(); }
};

namespace wadg {
namespace host {

// The last failure's detail, per thread (wadg_last_error).
extern thread_local std::string g_last_error;

// Records msg as the thread's last error and returns code.
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define WADG_HIP(call)                                  \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #call);   \
  } while (0)

// LSRK(5,4) 2N-storage coefficients (launch.hip).
extern const double kRkA[5];
extern const double kRkB[5];

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

int check_mesh(const wadg_mesh* m);

// Length and speed scales of a mesh from its geometry arrays (untiled,
// tiled = false: vol [6][nq^2][K], face [3][4][nq][K]; or tiled in groups
// of 64 lanes): h = min over elements of 4 |D_k| / |dD_k| (the side of a
// square element: area = sum_q w_q J_q, perimeter = sum over faces and
// points of w sJ) and the largest c^2 = (c2/J) / (1/J) at a volume point.
void mesh_scales(const double* vol, const double* face, int K, int nq, const double* wq,
                 bool tiled, double* h_min, double* c2_max);

// CFL number of a step dt: dt c_max (N+1)^2 / h.
inline double cfl_number(double dt, int N, double h_min, double c2_max) {
  return dt * std::sqrt(c2_max) * (N + 1) * (N + 1) / h_min;
}
int check_slices(wadg_ctx c, int32_t S);

inline wadg::MeshIn mesh_in(const wadg_mesh* m) {
  return wadg::MeshIn{m->N, m->nq1, m->K, m->x, m->y, m->etoe, m->etof, m->c2q};
}

inline bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

// The stage kernel that runs for this context, precision and launch mode.
// The kernel variant for a launch of S slices (WADG_KERNEL_PIPE needs at
// least kPipeMinSlices of them; S = 0 asks for a large launch).
constexpr int32_t kPipeMinSlices = 2;
int kernel_path(wadg_ctx c, bool fp32, int mode, int32_t S);
// Launch one stage of `mode` with the context's kernel choice and the
// alternating work-item order.
int launch_stage(wadg_ctx c, int mode, bool fp32, const wadg::StageParams& p0, void* stream);
// Launch an apply-A stage (mode_a) and an independent LSRK stage in one grid
// of the split kernel (launch_stage_pair), with the alternating item order.
int launch_stage_pair(wadg_ctx c, int mode_a, const wadg::StageParams& a0,
                      const wadg::StageParams& b0, void* stream);
// Stage parameters of the context for S slices (geometry, schedule, penalties).
wadg::StageParams base_params(wadg_ctx c, int32_t S);

}  // namespace host
}  // namespace wadg
