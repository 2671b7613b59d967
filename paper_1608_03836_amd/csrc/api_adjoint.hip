// C ABI, adjoint of the sweep (declared in include/wadg.h): forward sweep
// with checkpoints and the reverse (adjoint) sweep.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "api_internal.h"

using namespace wadg::host;

extern "C" {

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
    p.res_dead = i == 4;
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
  const bool fused = kernel_path(ctx, false, wadg::kApplyA, 1) == WADG_KERNEL_SPLIT;
  const int G = ctx->groups();
  WADG_HIP(hipMemsetAsync(part, 0, (size_t)G * sizeof(double), hs));
  WADG_HIP(hipMemcpyAsync(yb, seed, sb, hipMemcpyDeviceToDevice, hs));

  wadg::StageParams p = base_params(ctx, 1);
  p.dt = dt;
  double* const Rs[2] = {R, R + 5 * (size_t)nsteps * n1};
  // Each slice's residuals are recomputed from its checkpoint (into the
  // residual set of its parity) before its reverse stages read them.  With
  // the split kernel for both, the recompute of slice s-1 rides along in the
  // launches of slice s's reverse stages, one stage each (launch_stage_pair:
  // the two one-slice launches share the CUs), on `stream` alone.  Otherwise
  // it runs on the context's second stream while the reverse sweep of slice
  // s runs on `stream`: ev_rec[b] = residual set b is ready, ev_rev[b] = the
  // reverse sweep that read set b is done.
  const bool paired = fused && kernel_path(ctx, false, wadg::kStage, 1) == WADG_KERNEL_SPLIT;
  hipStream_t aux = nullptr;
  if (!paired) {
    if (!ctx->aux) {
      WADG_HIP(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
      for (hipEvent_t* e : {&ctx->ev_in, &ctx->ev_rec[0], &ctx->ev_rec[1], &ctx->ev_rev[0],
                            &ctx->ev_rev[1]})
        WADG_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
    }
    aux = ctx->aux;
    WADG_HIP(hipEventRecord(ctx->ev_in, hs));          // chk and seed are written
    WADG_HIP(hipStreamWaitEvent(aux, ctx->ev_in, 0));
  }
  auto recompute = [&](int s) -> int {
    const int b = s % 2;
    if (s + 2 <= S - 1) WADG_HIP(hipStreamWaitEvent(aux, ctx->ev_rev[b], 0));
    int st = adjoint_recompute(ctx, chk + s * n1, Rs[b], T, dt, nsteps, aux);
    if (st) return st;
    WADG_HIP(hipEventRecord(ctx->ev_rec[b], aux));
    return WADG_OK;
  };
  int st = paired ? adjoint_recompute(ctx, chk + (S - 1) * n1, Rs[(S - 1) % 2], T, dt, nsteps, hs)
                  : recompute(S - 1);
  if (st) return st;
  for (int s = S - 1; s >= 0; --s) {
    if (!paired && s >= 1 && (st = recompute(s - 1))) return st;
    const double* Rs_ = Rs[s % 2];
    if (!paired) WADG_HIP(hipStreamWaitEvent(hs, ctx->ev_rec[s % 2], 0));
    // paired: the recompute of slice s-1 (stage t of it with reverse stage t
    // of slice s), as adjoint_recompute does it
    double* const Rn = Rs[(s + 1) % 2];
    const double* cur = s >= 1 ? chk + (s - 1) * n1 : nullptr;
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
        int mode = wadg::kApplyA;
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
          mode = wadg::kApplyAMass;
        }
        if (paired && s >= 1) {
          const int t = 5 * (nsteps - 1 - m) + (4 - i), m1 = t / 5, i1 = t % 5;
          wadg::StageParams r = p;
          r.Qin = cur;
          r.Qout = T[t % 2];
          r.res = Rn + (5 * (size_t)m1 + (i1 == 0 ? 0 : i1 - 1)) * n1;
          r.res_out = Rn + (5 * (size_t)m1 + i1) * n1;
          r.rkA = kRkA[i1];
          r.rkB = kRkB[i1];
          e = launch_stage_pair(ctx, mode, q, r, stream);
          cur = T[t % 2];
        } else {
          e = launch_stage(ctx, mode, false, q, stream);
        }
        if (mode == wadg::kApplyAMass) std::swap(zc, zn);
        if (e) return hip_fail((hipError_t)e, "stage kernel launch (apply A)");
      }
    }
    if (!paired) WADG_HIP(hipEventRecord(ctx->ev_rev[s % 2], hs));
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
