// The stage-launch policy of the C ABI: which stage kernel runs (the
// automatic choice), the alternating work-item order, and the stage
// parameters of a context.

#include "api_internal.h"

namespace wadg {
namespace host {

// LSRK(5,4) 2N-storage coefficients (Carpenter & Kennedy 1994), the
// integrator of the paper's experiments (Section 5.2).
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

// Kernel variant that runs for this context, precision and launch mode.
// Automatic choice, from measurement on MI355X (64x64 and 128x128
// elements, N = 3, FP64 and FP32): LSRK stages of two or more slices take
// the pipelined kernel where its LDS plan fits, else the split-work
// kernel; right-hand-side launches take the resident-geometry kernel where
// the geometry fits in LDS, else the split-work kernel; the adjoint's
// apply-A launches take the split-work kernel (the resident kernel has no
// apply-A mode, so an explicit RESIDENT or STREAMED choice runs them
// streamed).
int kernel_path(wadg_ctx c, bool fp32, int mode, int32_t S) {
  if (mode == wadg::kStage && (c->kernel == WADG_KERNEL_PIPE || c->kernel == WADG_KERNEL_AUTO) &&
      S >= kPipeMinSlices && wadg::pipe_supported(c->N, c->nq1, fp32))
    return WADG_KERNEL_PIPE;
  if (c->kernel == WADG_KERNEL_PIPE) return WADG_KERNEL_SPLIT;  // its other launches
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
  const int path = kernel_path(c, fp32, mode, p0.S);
  if (path == WADG_KERNEL_PIPE)
    return fp32 ? wadg::launch_stage_pipe_fp32(c->N, c->nq1, p0, c->cus, stream)
                : wadg::launch_stage_pipe(c->N, c->nq1, p0, c->cus, stream);
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

int launch_stage_pair(wadg_ctx c, int mode_a, const wadg::StageParams& a0,
                      const wadg::StageParams& b0, void* stream) {
  wadg::StageParams a = a0, b = b0;
  c->order_flip ^= 1;
  a.reverse = b.reverse = (int32_t)c->order_flip;
  return wadg::launch_stage_pair(c->N, c->nq1, mode_a, a, b, stream);
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
  p.res_dead = 0;
  return p;
}

}  // namespace host
}  // namespace wadg
