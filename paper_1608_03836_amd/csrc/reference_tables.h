// Compile-time 1D reference operators of the tensor-product nodal basis.
//
// Everything here depends only on (N, nq): Gauss-Legendre points and
// weights (Newton on P_n), Gauss-Lobatto-Legendre points (Newton on the
// Jacobi polynomial P^{(1,1)}_{N-1}, proportional to P_N'), the GLL Lagrange
// basis and its derivative at the Gauss points, the 1D nodal mass matrix and
// the two products the WADG inverse needs.  Being constexpr, the tables are
// folded into the kernels as immediate constants, and the host geometry
// uses exactly the same values.
#pragma once

namespace wadg {
namespace ct {

constexpr double kPi = 3.14159265358979323846;

constexpr double cabs(double x) { return x < 0 ? -x : x; }

// cos on [0, pi] by its Taylor series after reflection to [0, pi/2]; used
// only for Newton starting guesses.
constexpr double ccos(double x) {
  bool neg = false;
  if (x > kPi / 2) {
    x = kPi - x;
    neg = true;
  }
  double term = 1.0, sum = 1.0;
  const double x2 = x * x;
  for (int k = 1; k < 30; ++k) {
    term *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return neg ? -sum : sum;
}

struct PD {
  double p, dp;
};

// Legendre P_n and P_n' by the three-term recurrence.
constexpr PD legendre(int n, double x) {
  if (n == 0) return {1.0, 0.0};
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    const double d2 = d0 + (2 * k + 1) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  return {p1, d1};
}

// Jacobi P^{(1,1)}_n and derivative:
//   n (n+2) P_n = (2n+1)(n+1) x P_{n-1} - n (n+1) P_{n-2},  P_0 = 1, P_1 = 2x.
constexpr PD jacobi11(int n, double x) {
  if (n == 0) return {1.0, 0.0};
  double p0 = 1.0, d0 = 0.0, p1 = 2.0 * x, d1 = 2.0;
  for (int k = 2; k <= n; ++k) {
    const double a = (2.0 * k + 1.0) * (k + 1.0), b = k * (k + 1.0), c = k * (k + 2.0);
    const double p2 = (a * x * p1 - b * p0) / c;
    const double d2 = (a * (p1 + x * d1) - b * d0) / c;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  return {p1, d1};
}

template <int N, int NQ>
struct Tables {
  double xg[N + 1];            // GLL nodes
  double xq[NQ], wq[NQ];       // Gauss points and weights
  double V[NQ][N + 1];         // l_a(x_i)
  double D[NQ][N + 1];         // l_a'(x_i)
  double Vt[NQ][N + 1];        // (V M1^{-1})[i][a]
  double P[N + 1][NQ];         // (M1^{-1} V^T W)[a][i]
};

template <int N, int NQ>
constexpr Tables<N, NQ> make_tables() {
  Tables<N, NQ> t{};
  // Gauss-Legendre
  for (int i = 0; i < NQ; ++i) {
    double z = -ccos(kPi * (i + 0.75) / (NQ + 0.5));
    for (int it = 0; it < 100; ++it) {
      const PD v = legendre(NQ, z);
      const double dz = v.p / v.dp;
      z -= dz;
      if (cabs(dz) < 1e-16) break;
    }
    const PD v = legendre(NQ, z);
    t.xq[i] = z;
    t.wq[i] = 2.0 / ((1.0 - z * z) * v.dp * v.dp);
  }
  for (int i = 0; i < NQ / 2; ++i) {
    const double a = 0.5 * (t.xq[NQ - 1 - i] - t.xq[i]);
    const double b = 0.5 * (t.wq[i] + t.wq[NQ - 1 - i]);
    t.xq[i] = -a; t.xq[NQ - 1 - i] = a;
    t.wq[i] = b; t.wq[NQ - 1 - i] = b;
  }
  if (NQ % 2) t.xq[NQ / 2] = 0.0;
  // Gauss-Lobatto-Legendre
  t.xg[0] = -1.0;
  t.xg[N] = 1.0;
  for (int i = 1; i < N; ++i) {
    double z = -ccos(kPi * i / N);
    for (int it = 0; it < 100; ++it) {
      const PD v = jacobi11(N - 1, z);
      const double dz = v.p / v.dp;
      z -= dz;
      if (cabs(dz) < 1e-16) break;
    }
    t.xg[i] = z;
  }
  for (int i = 0; i <= N / 2; ++i) {
    const double a = 0.5 * (t.xg[N - i] - t.xg[i]);
    t.xg[i] = -a; t.xg[N - i] = a;
  }
  if (N % 2 == 0) t.xg[N / 2] = 0.0;
  // Lagrange basis of the GLL nodes and its derivative at the Gauss points
  for (int i = 0; i < NQ; ++i)
    for (int a = 0; a <= N; ++a) {
      double val = 1.0, der = 0.0;
      for (int m = 0; m <= N; ++m) {
        if (m == a) continue;
        const double f = (t.xq[i] - t.xg[m]) / (t.xg[a] - t.xg[m]);
        der = der * f + val / (t.xg[a] - t.xg[m]);
        val *= f;
      }
      t.V[i][a] = val;
      t.D[i][a] = der;
    }
  // 1D nodal mass matrix and its inverse (Gauss-Jordan, partial pivoting)
  double M[N + 1][2 * (N + 1)] = {};
  for (int a = 0; a <= N; ++a)
    for (int c = 0; c <= N; ++c) {
      double s = 0.0;
      for (int i = 0; i < NQ; ++i) s += t.wq[i] * t.V[i][a] * t.V[i][c];
      M[a][c] = s;
      M[a][N + 1 + c] = (a == c) ? 1.0 : 0.0;
    }
  for (int c = 0; c <= N; ++c) {
    int piv = c;
    for (int r = c + 1; r <= N; ++r)
      if (cabs(M[r][c]) > cabs(M[piv][c])) piv = r;
    for (int j = 0; j < 2 * (N + 1); ++j) {
      const double tmp = M[c][j];
      M[c][j] = M[piv][j];
      M[piv][j] = tmp;
    }
    const double d = M[c][c];
    for (int j = 0; j < 2 * (N + 1); ++j) M[c][j] /= d;
    for (int r = 0; r <= N; ++r) {
      if (r == c) continue;
      const double f = M[r][c];
      for (int j = 0; j < 2 * (N + 1); ++j) M[r][j] -= f * M[c][j];
    }
  }
  for (int i = 0; i < NQ; ++i)
    for (int a = 0; a <= N; ++a) {
      double s = 0.0;
      for (int c = 0; c <= N; ++c) s += t.V[i][c] * M[c][N + 1 + a];
      t.Vt[i][a] = s;
    }
  for (int a = 0; a <= N; ++a)
    for (int i = 0; i < NQ; ++i) {
      double s = 0.0;
      for (int c = 0; c <= N; ++c) s += M[a][N + 1 + c] * t.V[i][c];
      t.P[a][i] = s * t.wq[i];
    }
  return t;
}

template <int N, int NQ>
struct Ref {
  static constexpr Tables<N, NQ> t = make_tables<N, NQ>();
};

// The operators the kernels use, rounded once to the arithmetic type R.
template <typename R, int N, int NQ>
struct Ops {
  R V[NQ][N + 1], D[NQ][N + 1], Vt[NQ][N + 1], P[N + 1][NQ];
};

template <typename R, int N, int NQ>
constexpr Ops<R, N, NQ> make_ops() {
  const Tables<N, NQ> t = make_tables<N, NQ>();
  Ops<R, N, NQ> o{};
  for (int i = 0; i < NQ; ++i)
    for (int a = 0; a <= N; ++a) {
      o.V[i][a] = static_cast<R>(t.V[i][a]);
      o.D[i][a] = static_cast<R>(t.D[i][a]);
      o.Vt[i][a] = static_cast<R>(t.Vt[i][a]);
      o.P[a][i] = static_cast<R>(t.P[a][i]);
    }
  return o;
}

}  // namespace ct
}  // namespace wadg
