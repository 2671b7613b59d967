// C ABI, batches of independent problems (declared in include/wadg.h).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "api_internal.h"

using namespace wadg::host;

// ---------------------------------------------------------------------------
// Batches of independent problems.

struct wadg_batch_s {
  int device = 0, N = 0, nq1 = 0, cus = 256, nprob = 0;
  double tau_p = 1.0, tau_u = 1.0;
  std::vector<int32_t> pack, K, S;            // per problem: copies per lane group, elements, slices
  std::vector<int32_t> Kv, Sv, nEG, g0;       // packed (virtual) mesh and its slices
  std::vector<int64_t> offset;                 // [nprob + 1] state offsets in doubles
  std::vector<double> dt;                      // per problem (last uploaded to d_prob)
  int64_t groups = 0, items = 0;
  double* d_vol = nullptr;
  double* d_face = nullptr;
  int32_t* d_nbr = nullptr;
  wadg::BatchProb* d_prob = nullptr;           // descriptors of eager sweeps
  wadg::BatchProb* d_prob_graph = nullptr;     // descriptors the captured graph reads
  int32_t* d_items = nullptr;
  int32_t* d_runs = nullptr;                   // pipelined kernel's runs [nruns][4]
  int64_t nruns = 0;
  int grid_mult = 0;                           // persistent workgroups per CU (0: one per item)
  int order = 0;                               // 0 problem-major, 1 interleaved
  int run_slices = 0;                          // > 0: pipelined kernel, runs of this many slices
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

// Default slices per run of the pipelined batch kernel.
constexpr int kBatchRunSlices = 16;

void free_batch(wadg_batch b) {
  if (!b) return;
  if (b->exec || b->graph) (void)hipDeviceSynchronize();   // replays still queued
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  for (void* ptr : {(void*)b->d_vol, (void*)b->d_face, (void*)b->d_nbr, (void*)b->d_prob,
                    (void*)b->d_prob_graph, (void*)b->d_items, (void*)b->d_runs})
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

// Device tables that launches already queued may still read (the work
// list, the descriptors) are rewritten only after the device has drained:
// a rewrite is then ordered after every earlier launch of the batch, on
// whatever stream it ran, and (the copy being synchronous) before every
// later one.  Rewrites happen only when the schedule or a dt changes.
int batch_upload_items(wadg_batch b) {
  std::vector<int32_t> it = batch_items(b);
  WADG_HIP(hipDeviceSynchronize());
  WADG_HIP(hipMemcpy(b->d_items, it.data(), it.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  return WADG_OK;
}

// Elements of problem i's virtual mesh that hold real slices in its last
// virtual slice (the first copies; a packed last slice may have unused ones).
int32_t last_slice_elements(const wadg_batch b, int i) {
  return (b->S[i] - (b->Sv[i] - 1) * b->pack[i]) * b->K[i];
}

// Runs of the pipelined kernel: for every problem and element group of its
// virtual mesh, the virtual slices in which the group holds a real element
// (all but, possibly, the last), cut into ceil(n / run_slices) runs of
// nearly equal length.  Placement: workgroups are dealt to the eight XCDs
// round-robin (block b on XCD b % 8), so the list is laid out per block.
// Whole problems go to one XCD each (largest first, to the XCD with the
// least work so far), so that the neighbour traces a group reads come from
// tiles its own XCD has just loaded; each XCD then takes its runs longest
// first (runs of equal length problem-major).  Blocks past the end of
// their XCD's list get an empty run (problem -1).  Uploaded like the work
// list.
int batch_upload_runs(wadg_batch b) {
  using Run = std::array<int32_t, 4>;
  std::vector<std::vector<Run>> per(b->nprob);
  std::vector<int64_t> work(b->nprob, 0);
  for (int i = 0; i < b->nprob; ++i)
    for (int g = 0; g < b->nEG[i]; ++g) {
      const int n = b->Sv[i] - (g * wadg::kWave >= last_slice_elements(b, i) ? 1 : 0);
      const int c = (n + b->run_slices - 1) / b->run_slices;
      for (int j = 0; j < c; ++j) {
        const int s0 = (int)((int64_t)j * n / c), s1 = (int)((int64_t)(j + 1) * n / c);
        per[i].push_back({i, g, s0, s1 - s0});
      }
      work[i] += n;
    }
  std::vector<int> order(b->nprob);
  for (int i = 0; i < b->nprob; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
  constexpr int kXcds = 8;
  std::vector<std::vector<Run>> xcd(kXcds);
  int64_t load[kXcds] = {};
  for (int i : order) {
    int x = 0;
    for (int y = 1; y < kXcds; ++y)
      if (load[y] < load[x]) x = y;
    load[x] += work[i];
    xcd[x].insert(xcd[x].end(), per[i].begin(), per[i].end());
  }
  size_t longest = 0;
  for (auto& l : xcd) {
    std::stable_sort(l.begin(), l.end(), [](const Run& u, const Run& v) { return u[3] > v[3]; });
    longest = std::max(longest, l.size());
  }
  std::vector<int32_t> r;
  r.reserve(longest * kXcds * 4);
  for (size_t j = 0; j < longest; ++j)
    for (int x = 0; x < kXcds; ++x) {
      const Run e = j < xcd[x].size() ? xcd[x][j] : Run{-1, 0, 0, 0};
      r.insert(r.end(), e.begin(), e.end());
    }
  if (r.size() / 4 >= (size_t)1 << 31) return fail(WADG_E_INVALID, "too many runs");
  WADG_HIP(hipDeviceSynchronize());
  if (b->d_runs) WADG_HIP(hipFree(b->d_runs));
  b->d_runs = nullptr;
  b->nruns = (int64_t)(r.size() / 4);
  if (b->nruns == 0) return WADG_OK;
  WADG_HIP(hipMalloc(&b->d_runs, r.size() * sizeof(int32_t)));
  WADG_HIP(hipMemcpy(b->d_runs, r.data(), r.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  return WADG_OK;
}

int check_dt(const wadg_batch b, const double* dt) {
  for (int i = 0; i < b->nprob; ++i)
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i]))
      return fail(WADG_E_INVALID, "dt[" + std::to_string(i) + "] must be finite and > 0");
  return WADG_OK;
}

// Elements of one copy whose geometry every group of problem i reads
// (wadg::BatchProb::kc), or 0: a packed mesh, or one of fewer than 64
// elements, whose first groups' geometry a 32-bit buffer range can hold.
int32_t copy_elements(const wadg_batch b, int i) {
  if (b->pack[i] == 1 && b->K[i] >= wadg::kWave) return 0;
  const int64_t groups = (b->K[i] + wadg::kWave - 1) / wadg::kWave;
  const int64_t vol = 6LL * b->nq1 * b->nq1 * wadg::kWave * (int64_t)sizeof(double);
  const int64_t face = 12LL * b->nq1 * wadg::kWave * (int64_t)sizeof(double);
  return groups * (vol > face ? vol : face) < (1LL << 31) ? b->K[i] : 0;
}

int write_descriptors(const wadg_batch b, const double* dt, wadg::BatchProb* dst) {
  std::vector<wadg::BatchProb> pr(b->nprob);
  for (int i = 0; i < b->nprob; ++i)
    pr[i] = wadg::BatchProb{b->offset[i], b->nEG[i], b->Sv[i], b->Kv[i], b->g0[i],
                            last_slice_elements(b, i), copy_elements(b, i), dt[i]};
  WADG_HIP(hipDeviceSynchronize());
  WADG_HIP(hipMemcpy(dst, pr.data(), pr.size() * sizeof(wadg::BatchProb),
                     hipMemcpyHostToDevice));
  return WADG_OK;
}

// The descriptors of eager sweeps, rewritten when a dt differs from the
// last upload.  The captured graph keeps its own (d_prob_graph).
int batch_upload_dt(wadg_batch b, const double* dt) {
  int st = check_dt(b, dt);
  if (st) return st;
  bool same = !b->dt.empty();
  for (int i = 0; same && i < b->nprob; ++i) same = b->dt[i] == dt[i];
  if (same) return WADG_OK;
  if ((st = write_descriptors(b, dt, b->d_prob))) return st;
  b->dt.assign(dt, dt + b->nprob);
  return WADG_OK;
}

// Frees the captured graph, if any, once the device has drained, so that
// no replay still queued on any stream runs from a destroyed graph.
int drop_graph(wadg_batch b) {
  if (!b->exec && !b->graph) return WADG_OK;
  WADG_HIP(hipDeviceSynchronize());
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  return WADG_OK;
}

int batch_grid(const wadg_batch b) {
  if (b->grid_mult == 0 || (int64_t)b->grid_mult * b->cus >= b->items) return (int)b->items;
  return b->grid_mult * b->cus;
}

int batch_stage(wadg_batch b, const wadg::BatchProb* prob, const double* qin, double* qout,
                double* res, int i, void* stream) {
  wadg::BatchParams p{};
  p.prob = prob;
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
  p.res_dead = i == 4;
  // runs of slices: the pipelined kernel (wadg_batch_set_runs); one
  // workgroup per item: the split-work kernel; persistent workgroups: the
  // streamed kernel (wadg_batch_set_schedule)
  int e = b->run_slices > 0
              ? wadg::launch_batch_pipe(b->N, b->nq1, p, b->d_runs, (int32_t)b->nruns, stream)
          : b->grid_mult == 0
              ? wadg::launch_batch_split(b->N, b->nq1, p, stream)
              : wadg::launch_batch_stage(b->N, b->nq1, p, batch_grid(b), stream);
  if (e) return hip_fail((hipError_t)e, "batch stage kernel launch");
  return WADG_OK;
}

int batch_sweep(wadg_batch b, const wadg::BatchProb* prob, double* Q, double* work,
                int32_t nsteps, void* stream) {
  const size_t n = (size_t)b->offset[b->nprob];
  double* res = work;
  double* other = work + n;
  double* cur = Q;
  for (int stp = 0; stp < nsteps; ++stp)
    for (int i = 0; i < 5; ++i) {
      double* out = cur == Q ? other : Q;
      int st = batch_stage(b, prob, cur, out, res, i, stream);
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

namespace {

// Copies of a K-element mesh per virtual slice (its S slices side by side in
// a virtual mesh of P K elements, ceil(S / P) virtual slices): the P in
// [1, min(S, 64)] that moves the fewest bytes per stage, counting each work
// item's state tiles (Q and the residual, read and written) and each
// virtual element group's geometry once (a problem's items share it through
// the cache); the smallest such P.  At P = 64 the copies fill whole groups,
// so a larger P gains nothing; nor may a virtual slice outgrow the 2 GiB a
// slice may take.
int pack_copies(int K, int S, int Np, int nq) {
  const double state_item = 4.0 * 3 * Np * wadg::kWave * sizeof(double);
  const double geo_group = ((6.0 * nq * nq + 12.0 * nq) * sizeof(double) + 8 * sizeof(int32_t)) *
                           wadg::kWave;
  int best = 1;
  double best_bytes = -1.0;
  for (int P = 1; P <= std::min(S, wadg::kWave); ++P) {
    const int64_t g = ((int64_t)P * K + wadg::kWave - 1) / wadg::kWave;
    if (P > 1 && g * 3 * Np * wadg::kWave * (int64_t)sizeof(double) >= (1LL << 31)) break;
    const double groups = (double)g;
    const double items = (double)((S + P - 1) / P) * groups;
    const double bytes = items * state_item + groups * geo_group;
    if (best_bytes < 0.0 || bytes < best_bytes) {
      best_bytes = bytes;
      best = P;
    }
  }
  return best;
}

}  // namespace

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
    const int P = pack_copies(m.K, S[i], Np, nq);
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
    const size_t Gv = ((size_t)Kv + wadg::kWave - 1) / wadg::kWave;
    std::vector<double> vt(Gv * 6 * nqq * wadg::kWave), ft(Gv * 12 * nq * wadg::kWave);
    std::vector<int32_t> nt(Gv * 8 * wadg::kWave);
    int g = wadg::build_geometry(mi, ops, vt.data(), ft.data(), nt.data(), true, &err);
    if (g) {
      free_batch(b);
      return fail(g == -1 ? WADG_E_INVALID : WADG_E_GEOMETRY,
                  "problem " + std::to_string(i) + ": " + err);
    }
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
      (e = hipMalloc(&b->d_prob_graph, (size_t)nprob * sizeof(wadg::BatchProb))) != hipSuccess ||
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
  if (!st && wadg::batch_pipe_supported(N, nq)) {   // the default schedule
    b->run_slices = kBatchRunSlices;
    st = batch_upload_runs(b);
  }
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
  return batch_sweep(b, b->d_prob, Q, work, nsteps, stream);
}

int wadg_batch_set_schedule(wadg_batch b, int32_t wg_per_cu, int32_t order) {
  if (!b) return fail(WADG_E_INVALID, "batch is NULL");
  if (wg_per_cu < 0 || wg_per_cu > 64 || (order != 0 && order != 1))
    return fail(WADG_E_INVALID, "wg_per_cu in [0, 64] and order in {0, 1} required");
  if (b->exec) return fail(WADG_E_INVALID, "release the captured graph first");
  DeviceGuard guard(b->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the batch's device");
  b->grid_mult = wg_per_cu;
  b->run_slices = 0;
  if (order != b->order) {
    b->order = order;
    int st = batch_upload_items(b);
    if (st) return st;
  }
  return WADG_OK;
}

int wadg_batch_set_runs(wadg_batch b, int32_t run_slices) {
  if (!b) return fail(WADG_E_INVALID, "batch is NULL");
  if (run_slices < 0) return fail(WADG_E_INVALID, "run_slices must be >= 0");
  if (b->exec) return fail(WADG_E_INVALID, "release the captured graph first");
  if (run_slices > 0 && !wadg::batch_pipe_supported(b->N, b->nq1))
    return fail(WADG_E_UNSUPPORTED, "the pipelined kernel's tiles do not fit in LDS");
  DeviceGuard guard(b->device);
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the batch's device");
  if (run_slices == b->run_slices) return WADG_OK;
  b->run_slices = run_slices;
  return run_slices > 0 ? batch_upload_runs(b) : WADG_OK;
}

int wadg_batch_tune(wadg_batch b, const double* Q, double* work, const double* dt, int32_t reps,
                    int32_t* wg_per_cu, int32_t* order, int32_t* run_slices, double* best_us,
                    void* stream) {
  if (!b) return fail(WADG_E_INVALID, "batch is NULL");
  if (!Q || !work || !dt || !wg_per_cu || !order || !run_slices || !best_us)
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
  // candidates: the pipelined kernel with runs of 4..128 slices per
  // workgroup (tile = one element group x a run of slices); persistent grids
  // of 1, 2, 4, 8 two-wave workgroups per CU (streamed kernel) or one
  // four-wave workgroup per item (split kernel), in both item orders; each
  // timed on a stage with a residual read (Q is only read, the workspace is
  // scratch)
  struct Cand { int m, o, r; };
  std::vector<Cand> cands;
  if (wadg::batch_pipe_supported(b->N, b->nq1))
    for (int r : {4, 8, 16, 32, 128}) cands.push_back({0, 0, r});
  for (int o = 0; o < 2; ++o)
    for (int m : {1, 2, 4, 8, 0}) cands.push_back({m, o, 0});
  double best = 1e300;
  const Cand c0{b->grid_mult, b->order, b->run_slices};
  Cand bc = c0;
  auto apply = [&](const Cand& c) {
    int s = wadg_batch_set_schedule(b, c.m, c.o);
    return s ? s : wadg_batch_set_runs(b, c.r);
  };
  for (const Cand& c : cands) {
    if ((st = apply(c))) break;
    if ((st = batch_stage(b, b->d_prob, Q, work, work + n, 1, stream))) break;
    if (hipEventRecord(e0, hs) != hipSuccess) { st = hip_fail(hipErrorUnknown, "event"); break; }
    for (int r = 0; r < reps && !st; ++r)
      st = batch_stage(b, b->d_prob, Q, work, work + n, 1, stream);
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
      bc = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) {
    (void)apply(c0);   // leave the schedule as it was
    return st;
  }
  if ((st = apply(bc))) return st;
  *wg_per_cu = bc.m;
  *order = bc.o;
  *run_slices = bc.r;
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
  int st = check_dt(b, dt);
  if (st) return st;
  if ((st = drop_graph(b))) return st;
  // the graph's own descriptors, written once here (after any replay of an
  // earlier graph has drained); eager sweeps never touch them
  if ((st = write_descriptors(b, dt, b->d_prob_graph))) return st;
  if (!b->capture_stream)
    WADG_HIP(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
  WADG_HIP(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
  st = batch_sweep(b, b->d_prob_graph, Q, work, nsteps, b->capture_stream);
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
  if (!guard.ok) return fail(WADG_E_DEVICE, "cannot select the batch's device");
  return drop_graph(b);
}

}  // extern "C"
