// Host setup: 1D reference operators of the nodal tensor basis and the
// per-element geometric data streamed by the stage kernel.
//
// The 1D operators are the compile-time tables of reference_tables.h.
// Geometry: isoparametric map (degree-N interpolant of the GLL node
// coordinates); metric terms of Section 5.4 at volume quadrature points,
// outward normals and surface Jacobians at face quadrature points.

#include <cmath>
#include <cstdio>

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

int build_geometry(const MeshIn& m, const RefOps& o, std::vector<double>* vol,
                   std::vector<double>* face, std::vector<int32_t>* nbr, std::string* err) {
  const int N = m.N, Np1 = N + 1, nq = m.nq1, Nq = nq * nq, K = m.K;
  const size_t KK = (size_t)K;
  if (vol) vol->assign(6 * (size_t)Nq * KK, 0.0);
  if (face) face->assign(3 * 4 * (size_t)nq * KK, 0.0);
  if (nbr) nbr->assign(2 * 4 * KK, 0);
  char buf[256];
  // face point coordinates for the conformity check [K][4][nq]
  std::vector<double> fx(KK * 4 * nq), fy(KK * 4 * nq);

  for (int k = 0; k < K; ++k) {
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
          std::snprintf(buf, sizeof buf, "non-positive Jacobian %.3e (element %d, point %d)", J,
                        k, q);
          *err = buf;
          return -2;
        }
        if (!(c2 > 0.0) || !std::isfinite(c2)) {
          std::snprintf(buf, sizeof buf, "c^2 must be finite and > 0 (element %d, point %d)", k,
                        q);
          *err = buf;
          return -1;
        }
        double W = o.wq[i] * o.wq[j];
        if (vol) {
          double* V = vol->data();
          V[(0 * (size_t)Nq + q) * KK + k] = W * ys;
          V[(1 * (size_t)Nq + q) * KK + k] = -W * xs;
          V[(2 * (size_t)Nq + q) * KK + k] = -W * yr;
          V[(3 * (size_t)Nq + q) * KK + k] = W * xr;
          V[(4 * (size_t)Nq + q) * KK + k] = c2 / J;
          V[(5 * (size_t)Nq + q) * KK + k] = 1.0 / J;
        }
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
        if (face) {
          double* F = face->data();
          F[((0 * 4 + f) * (size_t)nq + j) * KK + k] = ax / sJ;
          F[((1 * 4 + f) * (size_t)nq + j) * KK + k] = ay / sJ;
          F[((2 * 4 + f) * (size_t)nq + j) * KK + k] = o.wq[j] * sJ;
        }
        fx[((size_t)k * 4 + f) * nq + j] = xp;
        fy[((size_t)k * 4 + f) * nq + j] = yp;
      }
  }

  // connectivity: symmetric, and matched face points coincide (mod 1)
  const int base[4] = {0, N, Np1 * N, 0};
  const int stride[4] = {1, Np1, 1, Np1};
  for (int k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) {
      int kn = m.etoe[4 * k + f], info = m.etof[4 * k + f];
      int fn = info & 3, flip = (info >> 2) & 1;
      if (kn < 0 || kn >= K || (info & ~7) != 0) {
        std::snprintf(buf, sizeof buf, "bad connectivity (element %d, face %d)", k, f);
        *err = buf;
        return -1;
      }
      int back = m.etoe[4 * kn + fn], binfo = m.etof[4 * kn + fn];
      if (back != k || (binfo & 3) != f || ((binfo >> 2) & 1) != flip) {
        std::snprintf(buf, sizeof buf, "asymmetric connectivity (element %d, face %d)", k, f);
        *err = buf;
        return -2;
      }
      for (int j = 0; j < nq; ++j) {
        int jn = flip ? nq - 1 - j : j;
        double dx = fx[((size_t)kn * 4 + fn) * nq + jn] - fx[((size_t)k * 4 + f) * nq + j];
        double dy = fy[((size_t)kn * 4 + fn) * nq + jn] - fy[((size_t)k * 4 + f) * nq + j];
        if (!near_integer_shift(dx, 1e-9) || !near_integer_shift(dy, 1e-9)) {
          std::snprintf(buf, sizeof buf, "faces do not conform (element %d, face %d)", k, f);
          *err = buf;
          return -2;
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
        int32_t* B = nbr->data();
        B[(0 * 4 + f) * KK + k] = (int32_t)off;
        B[(1 * 4 + f) * KK + k] = dn * kWave;
      }
    }
  return 0;
}

}  // namespace wadg
