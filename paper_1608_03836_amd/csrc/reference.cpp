// Host setup: 1D reference operators of the nodal tensor basis and the
// per-element geometric data streamed by the stage kernel.
//
// The 1D operators are the compile-time tables of reference_tables.h.
// Geometry: isoparametric map (degree-N interpolant of the GLL node
// coordinates); metric terms of Section 6.4 at volume quadrature points,
// outward normals and surface Jacobians at face quadrature points.

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <memory>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "reference_tables.h"
#include "wadg_internal.h"

namespace wadg {

namespace {

template <int N, int NQ>
void copy_tables(RefOps* o) {
  constexpr const ct::Tables<N, NQ>& t = ct::Ref<N, NQ>::t;
  *o = RefOps();
  o->N = N;
  o->nq = NQ;
  for (int a = 0; a <= N; ++a) o->xg[a] = t.xg[a];
  for (int i = 0; i < NQ; ++i) {
    o->xq[i] = t.xq[i];
    o->wq[i] = t.wq[i];
    for (int a = 0; a <= N; ++a) {
      o->V[i][a] = t.V[i][a];
      o->D[i][a] = t.D[i][a];
      o->Vt[i][a] = t.Vt[i][a];
      o->P[a][i] = t.P[a][i];
    }
  }
}

template <int N>
bool copy_n(int nq, RefOps* o) {
  switch (nq - N) {
    case 1: copy_tables<N, N + 1>(o); return true;
    case 2: copy_tables<N, N + 2>(o); return true;
    case 3: copy_tables<N, N + 3>(o); return true;
    default: return false;
  }
}

}  // namespace

bool build_ref_ops(int N, int nq, RefOps* ops, std::string* err) {
  bool ok = false;
  switch (N) {
    case 1: ok = copy_n<1>(nq, ops); break;
    case 2: ok = copy_n<2>(nq, ops); break;
    case 3: ok = copy_n<3>(nq, ops); break;
    case 4: ok = copy_n<4>(nq, ops); break;
    default: ok = false;
  }
  if (!ok && err) *err = "unsupported degree or quadrature size";
  return ok;
}

void quadrature_points(const MeshIn& m, const RefOps& o, double* xq, double* yq) {
  const int Np1 = m.N + 1, nq = m.nq1, Nq = nq * nq;
  for (int k = 0; k < m.K; ++k) {
    const double* X = m.x + (size_t)k * Np1 * Np1;
    const double* Y = m.y + (size_t)k * Np1 * Np1;
    for (int j = 0; j < nq; ++j)
      for (int i = 0; i < nq; ++i) {
        double sx = 0.0, sy = 0.0;
        for (int b = 0; b < Np1; ++b)
          for (int a = 0; a < Np1; ++a) {
            double w = o.V[i][a] * o.V[j][b];
            sx += w * X[a + Np1 * b];
            sy += w * Y[a + Np1 * b];
          }
        xq[(size_t)k * Nq + i + nq * j] = sx;
        yq[(size_t)k * Nq + i + nq * j] = sy;
      }
  }
}

namespace {
// local node index of face node m (parameter order) on face f
inline int face_node(int f, int m, int N) {
  const int Np1 = N + 1;
  switch (f) {
    case 0: return m;                   // s = -1, b = 0
    case 1: return N + Np1 * m;         // r = +1, a = N
    case 2: return m + Np1 * N;         // s = +1, b = N
    default: return Np1 * m;            // r = -1, a = 0
  }
}
inline bool near_integer_shift(double d, double tol) {
  return std::fabs(d - std::nearbyint(d)) <= tol;
}
}  // namespace

namespace {

// Work of one element of build_geometry's first pass: metric terms and
// weights at the volume quadrature points into lv[6][Nq][KB] at lane l,
// normals and w sJ at the face points into lf[3][4][nq][KB], and the
// physical face points into fx, fy [4][nq] of the element.  Returns 0, or
// the error code with its message in err.
int element_geometry(const MeshIn& m, const RefOps& o, int k, int l, int KB, double* lv,
                     double* lf, double* fx, double* fy, std::string* err) {
  const int N = m.N, Np1 = N + 1, nq = m.nq1, Nq = nq * nq;
  char buf[256];
  const double* X = m.x + (size_t)k * Np1 * Np1;
  const double* Y = m.y + (size_t)k * Np1 * Np1;
  for (int n = 0; n < Np1 * Np1; ++n)
    if (!std::isfinite(X[n]) || !std::isfinite(Y[n])) {
      std::snprintf(buf, sizeof buf, "non-finite node coordinate (element %d)", k);
      *err = buf;
      return -2;
    }
  for (int j = 0; j < nq; ++j)
    for (int i = 0; i < nq; ++i) {
      double xr = 0, xs = 0, yr = 0, ys = 0;
      for (int b = 0; b < Np1; ++b)
        for (int a = 0; a < Np1; ++a) {
          double wr = o.D[i][a] * o.V[j][b], ws = o.V[i][a] * o.D[j][b];
          xr += wr * X[a + Np1 * b]; xs += ws * X[a + Np1 * b];
          yr += wr * Y[a + Np1 * b]; ys += ws * Y[a + Np1 * b];
        }
      double J = xr * ys - xs * yr;
      int q = i + nq * j;
      double c2 = m.c2q ? m.c2q[(size_t)k * Nq + q] : 1.0;
      if (!(J > 0.0) || !std::isfinite(J)) {
        std::snprintf(buf, sizeof buf, "non-positive Jacobian %.3e (element %d, point %d)", J, k,
                      q);
        *err = buf;
        return -2;
      }
      if (!(c2 > 0.0) || !std::isfinite(c2)) {
        std::snprintf(buf, sizeof buf, "c^2 must be finite and > 0 (element %d, point %d)", k, q);
        *err = buf;
        return -1;
      }
      double W = o.wq[i] * o.wq[j];
      lv[(0 * Nq + q) * KB + l] = W * ys;
      lv[(1 * Nq + q) * KB + l] = -W * xs;
      lv[(2 * Nq + q) * KB + l] = -W * yr;
      lv[(3 * Nq + q) * KB + l] = W * xr;
      lv[(4 * Nq + q) * KB + l] = c2 / J;
      lv[(5 * Nq + q) * KB + l] = 1.0 / J;
    }
  // faces: tangent along the face parameter from the face nodes only
  for (int f = 0; f < 4; ++f)
    for (int j = 0; j < nq; ++j) {
      double xt = 0, yt = 0, xp = 0, yp = 0;
      for (int mm = 0; mm < Np1; ++mm) {
        int n = face_node(f, mm, N);
        xt += o.D[j][mm] * X[n]; yt += o.D[j][mm] * Y[n];
        xp += o.V[j][mm] * X[n]; yp += o.V[j][mm] * Y[n];
      }
      // outward normal times sJ: faces 0,1 -> (yt, -xt); faces 2,3 -> (-yt, xt)
      double ax = (f < 2) ? yt : -yt, ay = (f < 2) ? -xt : xt;
      double sJ = std::hypot(ax, ay);
      if (!(sJ > 0.0) || !std::isfinite(sJ)) {
        std::snprintf(buf, sizeof buf, "degenerate face (element %d, face %d)", k, f);
        *err = buf;
        return -2;
      }
      lf[((0 * 4 + f) * nq + j) * KB + l] = ax / sJ;
      lf[((1 * 4 + f) * nq + j) * KB + l] = ay / sJ;
      lf[((2 * 4 + f) * nq + j) * KB + l] = o.wq[j] * sJ;
      fx[f * nq + j] = xp;
      fy[f * nq + j] = yp;
    }
  return 0;
}

// Runs body(first, last) over [0, n) split into contiguous ranges on the
// host's threads (at most 16), and returns the error of the lowest index
// that failed: body returns (index, code) of its first failure, or
// (last, 0).  The result and the reported error do not depend on the split.
template <typename F>
int parallel_ranges(int n, int grain, std::string* err, F body) {
  unsigned hw = std::thread::hardware_concurrency();
  int T = (int)std::max(1u, std::min(hw ? hw : 1u, 16u));
  T = std::max(1, std::min(T, (n + grain - 1) / grain));
  std::vector<int> at(T, n), code(T, 0);
  std::vector<std::string> msg(T);
  auto run = [&](int t) {
    const int a = (int)((long long)n * t / T), b = (int)((long long)n * (t + 1) / T);
    auto r = body(a, b, &msg[t]);
    at[t] = r.first;
    code[t] = r.second;
  };
  std::vector<std::thread> th;
  for (int t = 1; t < T; ++t) th.emplace_back(run, t);
  run(0);
  for (auto& x : th) x.join();
  for (int t = 0; t < T; ++t)   // ranges are ordered: the first failing range wins
    if (code[t]) {
      *err = msg[t];
      return code[t];
    }
  return 0;
}

}  // namespace

int build_geometry(const MeshIn& m, const RefOps& o, double* vol, double* face, int32_t* nbr,
                   bool tiled, std::string* err) {
  const int N = m.N, Np1 = N + 1, nq = m.nq1, Nq = nq * nq, K = m.K;
  const size_t KK = (size_t)K;
  // face point coordinates for the conformity check [K][4][nq]
  std::unique_ptr<double[]> fx(new double[KK * 4 * nq]), fy(new double[KK * 4 * nq]);

  // first pass, in blocks of KB = 64 elements (one element group): each
  // block computed into local [plane][point][64] buffers -- the group's
  // tile -- then written to the output, tiled as one contiguous copy or
  // untiled one contiguous row at a time
  constexpr int KB = kWave;
  const int nblocks = (K + KB - 1) / KB;
  const size_t PV = 6 * (size_t)Nq, PF = 3 * 4 * (size_t)nq;
  int st = parallel_ranges(nblocks, 16, err, [&](int b0, int b1, std::string* e) {
    std::vector<double> lv(PV * KB, 0.0), lf(PF * KB, 0.0);
    for (int bk = b0; bk < b1; ++bk) {
      const int k0 = bk * KB, nk = std::min(KB, K - k0);
      for (int l = 0; l < nk; ++l) {
        const int k = k0 + l;
        int c = element_geometry(m, o, k, l, KB, lv.data(), lf.data(),
                                 fx.get() + (size_t)k * 4 * nq, fy.get() + (size_t)k * 4 * nq, e);
        if (c) return std::make_pair(bk, c);
      }
      if (tiled) {
        if (nk < KB) {   // the padding lanes of a partial (last) group are zero
          for (size_t r = 0; r < PV; ++r)
            std::fill(lv.begin() + r * KB + nk, lv.begin() + (r + 1) * KB, 0.0);
          for (size_t r = 0; r < PF; ++r)
            std::fill(lf.begin() + r * KB + nk, lf.begin() + (r + 1) * KB, 0.0);
        }
        if (vol) std::copy(lv.begin(), lv.end(), vol + (size_t)bk * PV * KB);
        if (face) std::copy(lf.begin(), lf.end(), face + (size_t)bk * PF * KB);
      } else {
        if (vol)
          for (size_t r = 0; r < PV; ++r)
            std::copy(lv.begin() + r * KB, lv.begin() + r * KB + nk, vol + r * KK + k0);
        if (face)
          for (size_t r = 0; r < PF; ++r)
            std::copy(lf.begin() + r * KB, lf.begin() + r * KB + nk, face + r * KK + k0);
      }
    }
    return std::make_pair(b1, 0);
  });
  if (st) return st;

  // second pass: connectivity symmetric, and matched face points coincide
  // (mod 1); the neighbour offsets of the tiled state
  const int base[4] = {0, N, Np1 * N, 0};
  const int stride[4] = {1, Np1, 1, Np1};
  if (nbr && tiled)   // padding lanes of the last group
    for (int k = K; k < nblocks * KB; ++k)
      for (int p = 0; p < 8; ++p) nbr[((size_t)(k / KB) * 8 + p) * KB + k % KB] = 0;
  auto nbr_at = [&](int p, int k) -> int32_t& {
    return tiled ? nbr[((size_t)(k / KB) * 8 + p) * KB + k % KB] : nbr[(size_t)p * KK + k];
  };
  return parallel_ranges(K, 4096, err, [&](int ka, int kb, std::string* e) {
    char buf[256];
    for (int k = ka; k < kb; ++k)
      for (int f = 0; f < 4; ++f) {
        int kn = m.etoe[4 * k + f], info = m.etof[4 * k + f];
        int fn = info & 3, flip = (info >> 2) & 1;
        if (kn < 0 || kn >= K || (info & ~7) != 0) {
          std::snprintf(buf, sizeof buf, "bad connectivity (element %d, face %d)", k, f);
          *e = buf;
          return std::make_pair(k, -1);
        }
        int back = m.etoe[4 * kn + fn], binfo = m.etof[4 * kn + fn];
        if (back != k || (binfo & 3) != f || ((binfo >> 2) & 1) != flip) {
          std::snprintf(buf, sizeof buf, "asymmetric connectivity (element %d, face %d)", k, f);
          *e = buf;
          return std::make_pair(k, -2);
        }
        for (int j = 0; j < nq; ++j) {
          int jn = flip ? nq - 1 - j : j;
          double dx = fx[((size_t)kn * 4 + fn) * nq + jn] - fx[((size_t)k * 4 + f) * nq + j];
          double dy = fy[((size_t)kn * 4 + fn) * nq + jn] - fy[((size_t)k * 4 + f) * nq + j];
          if (!near_integer_shift(dx, 1e-9) || !near_integer_shift(dy, 1e-9)) {
            std::snprintf(buf, sizeof buf, "faces do not conform (element %d, face %d)", k, f);
            *e = buf;
            return std::make_pair(k, -2);
          }
        }
        if (nbr) {
          // tiled state: element kn is lane kn % 64 of group kn / 64; a group
          // holds 3 * Np node planes of 64 values
          const long long Np = (long long)Np1 * Np1;
          const int n0 = base[fn] + (flip ? stride[fn] * N : 0);
          const int dn = flip ? -stride[fn] : stride[fn];
          const long long off =
              (long long)(kn / kWave) * 3 * Np * kWave + (long long)n0 * kWave + kn % kWave;
          nbr_at(0 * 4 + f, k) = (int32_t)off;
          nbr_at(1 * 4 + f, k) = dn * kWave;
        }
      }
    return std::make_pair(kb, 0);
  });
}

}  // namespace wadg
