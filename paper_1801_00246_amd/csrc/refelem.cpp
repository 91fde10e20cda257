// Reference-triangle construction (host, FP64).  See refelem.hpp.
#include "refelem.hpp"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <stdexcept>
#include <string>

namespace ipdg {
namespace {

using Mat = std::vector<double>;  // row-major square or rectangular

// Orthonormal Jacobi polynomial P_n^{(a,b)} (weight (1-x)^a (1+x)^b) by the
// three-term recurrence of the orthonormal family.
double jacobi(double x, double a, double b, int n) {
  double p0 = std::sqrt(std::pow(2.0, -a - b - 1.0) * std::tgamma(a + b + 2.0) /
                        (std::tgamma(a + 1.0) * std::tgamma(b + 1.0)));
  if (n == 0) return p0;
  double p1 = p0 * ((a + b + 2.0) * x / 2.0 + (a - b) / 2.0) *
              std::sqrt((a + b + 3.0) / ((a + 1.0) * (b + 1.0)));
  if (n == 1) return p1;
  double aold = 2.0 / (2.0 + a + b) * std::sqrt((a + 1.0) * (b + 1.0) / (a + b + 3.0));
  for (int i = 1; i < n; ++i) {
    double h1 = 2.0 * i + a + b;
    double anew = 2.0 / (h1 + 2.0) *
                  std::sqrt((i + 1.0) * (i + 1.0 + a + b) * (i + 1.0 + a) * (i + 1.0 + b) /
                            ((h1 + 1.0) * (h1 + 3.0)));
    double bnew = -(a * a - b * b) / (h1 * (h1 + 2.0));
    double p2 = (-aold * p0 + (x - bnew) * p1) / anew;
    aold = anew;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

double djacobi(double x, double a, double b, int n) {
  if (n == 0) return 0.0;
  return std::sqrt(n * (n + a + b + 1.0)) * jacobi(x, a + 1.0, b + 1.0, n - 1);
}

// Legendre P_n and P_n' (classical normalisation) by recurrence.
void legendre(int n, double x, double& p, double& dp) {
  double pm = 1.0, pc = x;
  if (n == 0) { p = 1.0; dp = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double pn = ((2.0 * k - 1.0) * x * pc - (k - 1.0) * pm) / k;
    pm = pc;
    pc = pn;
  }
  p = pc;
  dp = n * (x * pc - pm) / (x * x - 1.0);
}

// Gauss-Lobatto-Legendre points: +-1 and the zeros of P_N', by Newton from the
// Chebyshev-Lobatto points.
std::vector<double> gll(int N) {
  std::vector<double> x(N + 1);
  x[0] = -1.0;
  x[N] = 1.0;
  for (int k = 1; k < N; ++k) {
    double t = -std::cos(M_PI * k / N);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(N, t, p, dp);
      // P_N'' from the Legendre equation (1-x^2) P'' = 2x P' - N(N+1) P
      double d2p = (2.0 * t * dp - N * (N + 1.0) * p) / (1.0 - t * t);
      double step = dp / d2p;
      t -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    x[k] = t;
  }
  std::sort(x.begin(), x.end());
  for (int k = 1; k <= N; ++k)
    if (!(x[k] > x[k - 1] + 1e-8)) throw std::runtime_error("GLL Newton did not separate roots");
  return x;
}

Mat inverse(const Mat& A, int n) {
  Mat a(A), inv(n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[r * n + c]) > std::fabs(a[piv * n + c])) piv = r;
    if (a[piv * n + c] == 0.0) throw std::runtime_error("singular matrix in reference setup");
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(a[c * n + k], a[piv * n + k]);
        std::swap(inv[c * n + k], inv[piv * n + k]);
      }
    double d = 1.0 / a[c * n + c];
    for (int k = 0; k < n; ++k) { a[c * n + k] *= d; inv[c * n + k] *= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = a[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        a[r * n + k] -= f * a[c * n + k];
        inv[r * n + k] -= f * inv[c * n + k];
      }
    }
  }
  return inv;
}

Mat matmul(const Mat& A, const Mat& B, int m, int k, int n) {
  Mat C(m * n, 0.0);
  for (int i = 0; i < m; ++i)
    for (int p = 0; p < k; ++p) {
      double a = A[i * k + p];
      for (int j = 0; j < n; ++j) C[i * n + j] += a * B[p * n + j];
    }
  return C;
}

Mat transpose(const Mat& A, int m, int n) {
  Mat T(n * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) T[j * m + i] = A[i * n + j];
  return T;
}

// Blend parameters alpha (N = 1..15) of the optimised Warp & Blend family.
const double kAlpha[15] = {0.0000, 0.0000, 1.4152, 0.1001, 0.2751, 0.9800, 1.0999, 1.2832,
                           1.3648, 1.4773, 1.4959, 1.5743, 1.5770, 1.6223, 1.6258};

// Edge warp: equispaced -> GLL displacement interpolated at t, over 1 - t^2.
double warp(int N, double t) {
  std::vector<double> xg = gll(N);
  double w = 0.0;
  for (int i = 0; i <= N; ++i) {
    double xi = -1.0 + 2.0 * i / N;
    double li = 1.0;
    for (int j = 0; j <= N; ++j)
      if (j != i) li *= (t - (-1.0 + 2.0 * j / N)) / (xi - (-1.0 + 2.0 * j / N));
    w += (xg[i] - xi) * li;
  }
  if (std::fabs(t) < 1.0 - 1e-10) return w / (1.0 - t * t);
  return 0.0;
}

void wb_nodes(int N, std::vector<double>& r, std::vector<double>& s) {
  const double a = kAlpha[N - 1];
  const double sq3 = std::sqrt(3.0);
  r.clear();
  s.clear();
  for (int j = 0; j <= N; ++j)
    for (int i = 0; i <= N - j; ++i) {
      double L1 = double(j) / N, L3 = double(i) / N, L2 = 1.0 - L1 - L3;
      double x = -L2 + L3, y = (-L2 - L3 + 2.0 * L1) / sq3;
      double w1 = 4.0 * L2 * L3 * warp(N, L3 - L2) * (1.0 + (a * L1) * (a * L1));
      double w2 = 4.0 * L1 * L3 * warp(N, L1 - L3) * (1.0 + (a * L2) * (a * L2));
      double w3 = 4.0 * L1 * L2 * warp(N, L2 - L1) * (1.0 + (a * L3) * (a * L3));
      x += w1 + std::cos(2.0 * M_PI / 3.0) * w2 + std::cos(4.0 * M_PI / 3.0) * w3;
      y += std::sin(2.0 * M_PI / 3.0) * w2 + std::sin(4.0 * M_PI / 3.0) * w3;
      double l1 = (sq3 * y + 1.0) / 3.0;
      double l2 = (-3.0 * x - sq3 * y + 2.0) / 6.0;
      double l3 = (3.0 * x - sq3 * y + 2.0) / 6.0;
      r.push_back(-l2 + l3 - l1);
      s.push_back(-l2 - l3 + l1);
    }
}

// Dubiner basis values and gradients at (r, s); columns ordered (i, j), i+j<=N.
void dubiner(int N, double r, double s, double* v, double* vr, double* vs) {
  double a = (std::fabs(1.0 - s) > 1e-14) ? 2.0 * (1.0 + r) / (1.0 - s) - 1.0 : -1.0;
  double b = s;
  int m = 0;
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N - i; ++j, ++m) {
      double fa = jacobi(a, 0, 0, i), dfa = djacobi(a, 0, 0, i);
      double gb = jacobi(b, 2 * i + 1, 0, j), dgb = djacobi(b, 2 * i + 1, 0, j);
      double omb = 1.0 - b;
      v[m] = M_SQRT2 * fa * gb * std::pow(omb, i);
      if (vr) {
        if (i == 0) {
          vr[m] = 0.0;
          vs[m] = M_SQRT2 * fa * dgb;
        } else {
          double pim1 = std::pow(omb, i - 1);
          vr[m] = M_SQRT2 * dfa * gb * 2.0 * pim1;
          vs[m] = M_SQRT2 * (dfa * gb * pim1 * (1.0 + a) + fa * (dgb * pim1 * omb - i * gb * pim1));
        }
      }
    }
}

int node_id(int N, int i, int j) { return j * (N + 1) - j * (j - 1) / 2 + i; }

RefOps build(int N) {
  RefOps R;
  R.N = N;
  R.Np = np_of(N);
  R.Nfp = N + 1;
  const int Np = R.Np, Nfp = R.Nfp;
  wb_nodes(N, R.r, R.s);
  R.fmask.resize(3 * Nfp);
  for (int k = 0; k < Nfp; ++k) {
    R.fmask[0 * Nfp + k] = node_id(N, k, 0);
    R.fmask[1 * Nfp + k] = node_id(N, N - k, k);
    R.fmask[2 * Nfp + k] = node_id(N, 0, N - k);
  }
  Mat V(Np * Np), Vr(Np * Np), Vs(Np * Np);
  for (int n = 0; n < Np; ++n) dubiner(N, R.r[n], R.s[n], &V[n * Np], &Vr[n * Np], &Vs[n * Np]);
  Mat Vi = inverse(V, Np);
  R.Dr = matmul(Vr, Vi, Np, Np, Np);
  R.Ds = matmul(Vs, Vi, Np, Np, Np);
  Mat VVt = matmul(V, transpose(V, Np, Np), Np, Np, Np);
  R.Minv = VVt;
  R.M = inverse(VVt, Np);
  R.Sr = matmul(R.M, R.Dr, Np, Np, Np);
  R.Ss = matmul(R.M, R.Ds, Np, Np, Np);
  // 1-D face mass from the orthonormal Legendre Vandermonde at GLL points
  std::vector<double> xg = gll(N);
  Mat V1(Nfp * Nfp);
  for (int i = 0; i < Nfp; ++i)
    for (int m = 0; m < Nfp; ++m) V1[i * Nfp + m] = jacobi(xg[i], 0, 0, m);
  R.M1D = inverse(matmul(V1, transpose(V1, Nfp, Nfp), Nfp, Nfp, Nfp), Nfp);
  Mat E(Np * 3 * Nfp, 0.0);
  for (int f = 0; f < 3; ++f)
    for (int m = 0; m < Nfp; ++m)
      for (int k = 0; k < Nfp; ++k)
        E[R.fmask[f * Nfp + m] * 3 * Nfp + f * Nfp + k] = R.M1D[m * Nfp + k];
  R.LIFT = matmul(VVt, E, Np, Np, 3 * Nfp);
  // rotations of the vertex labels: lattice (i', j') of the rotated frame
  // sits at barycentric lattice a'_m = a_{(m+k)%3} of the original one.
  for (int k = 0; k < 3; ++k) {
    R.rot[k].resize(Np);
    for (int jp = 0; jp <= N; ++jp)
      for (int ip = 0; ip <= N - jp; ++ip) {
        int a0 = N - ip - jp;
        int i, j;
        if (k == 0) { i = ip; j = jp; }
        else if (k == 1) { i = a0; j = ip; }
        else { i = jp; j = a0; }
        R.rot[k][node_id(N, ip, jp)] = node_id(N, i, j);
      }
    // the node set must be invariant: check coordinates
    for (int n = 0; n < Np; ++n) {
      double lp[3] = {-(R.r[n] + R.s[n]) / 2, (1 + R.r[n]) / 2, (1 + R.s[n]) / 2};
      int o = R.rot[k][n];
      double lo[3] = {-(R.r[o] + R.s[o]) / 2, (1 + R.r[o]) / 2, (1 + R.s[o]) / 2};
      for (int m = 0; m < 3; ++m)
        if (std::fabs(lo[(m + k) % 3] - lp[m]) > 1e-12)
          throw std::runtime_error("node set not rotation invariant at N=" + std::to_string(N));
    }
  }
  return R;
}

}  // namespace

const RefOps& ref_ops(int N) {
  static std::mutex mu;
  static RefOps cache[kMaxN + 1];
  if (N < 1 || N > kMaxN) throw std::runtime_error("degree out of range");
  std::lock_guard<std::mutex> lk(mu);
  if (cache[N].N == 0) cache[N] = build(N);
  return cache[N];
}

namespace {

// q-point Gauss-Legendre rule: zeros of P_q by Newton from the Chebyshev
// guesses, weights 2 / ((1 - x^2) P_q'(x)^2).
void gauss(int q, std::vector<double>& x, std::vector<double>& w) {
  x.resize(q);
  w.resize(q);
  for (int k = 0; k < q; ++k) {
    double t = -std::cos(M_PI * (k + 0.75) / (q + 0.5));
    double p = 0.0, dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      legendre(q, t, p, dp);
      const double step = p / dp;
      t -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    legendre(q, t, p, dp);
    x[k] = t;
    w[k] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

CubOps build_cub(int N) {
  const RefOps& R = ref_ops(N);
  CubOps C;
  C.N = N;
  C.Np = R.Np;
  C.Nfp = R.Nfp;
  C.q = cub_points(N);
  C.Nc = C.q * C.q;
  C.Nfc = C.q;
  const int Np = C.Np, Nfp = C.Nfp, Nc = C.Nc, Nfc = C.Nfc;
  std::vector<double> g, gw;
  gauss(C.q, g, gw);
  // inverse Vandermonde at the nodes: the Lagrange basis at a point is
  // psi(point)^T V^{-1}
  Mat V(Np * Np);
  for (int n = 0; n < Np; ++n) dubiner(N, R.r[n], R.s[n], &V[n * Np], nullptr, nullptr);
  Mat Vi = inverse(V, Np);
  Mat Q(Nc * Np), Qr(Nc * Np), Qs(Nc * Np);
  std::vector<double> wc(Nc);
  for (int a = 0; a < C.q; ++a)
    for (int b = 0; b < C.q; ++b) {
      const int i = a * C.q + b;
      const double r = (1.0 + g[a]) * (1.0 - g[b]) / 2.0 - 1.0, s = g[b];
      wc[i] = gw[a] * gw[b] * (1.0 - g[b]) / 2.0;
      dubiner(N, r, s, &Q[i * Np], &Qr[i * Np], &Qs[i * Np]);
    }
  C.I = matmul(Q, Vi, Nc, Np, Np);
  Mat Ir = matmul(Qr, Vi, Nc, Np, Np), Is = matmul(Qs, Vi, Nc, Np, Np);
  Mat WIr(Np * Nc), WIs(Np * Nc);
  for (int i = 0; i < Nc; ++i)
    for (int m = 0; m < Np; ++m) {
      WIr[m * Nc + i] = wc[i] * Ir[i * Np + m];
      WIs[m * Nc + i] = wc[i] * Is[i * Np + m];
    }
  C.Pr = matmul(R.Minv, WIr, Np, Np, Nc);
  C.Ps = matmul(R.Minv, WIs, Np, Np, Nc);
  for (int f = 0; f < 3; ++f) {
    Mat F(Nfc * Np);
    for (int j = 0; j < Nfc; ++j) {
      const double t = g[j];
      const double r = f == 0 ? t : (f == 1 ? -t : -1.0);
      const double s = f == 0 ? -1.0 : (f == 1 ? t : -t);
      dubiner(N, r, s, &F[j * Np], nullptr, nullptr);
    }
    Mat L = matmul(F, Vi, Nfc, Np, Np);
    C.If[f].assign(Nfc * Nfp, 0.0);
    for (int j = 0; j < Nfc; ++j)
      for (int k = 0; k < Nfp; ++k) C.If[f][j * Nfp + k] = L[j * Np + R.fmask[f * Nfp + k]];
    // the restriction of P_N to a face is fixed by the face nodes: the other
    // basis functions vanish there
    for (int j = 0; j < Nfc; ++j)
      for (int m = 0; m < Np; ++m) {
        bool face_node = false;
        for (int k = 0; k < Nfp; ++k) face_node = face_node || R.fmask[f * Nfp + k] == m;
        if (!face_node && std::fabs(L[j * Np + m]) > 1e-10)
          throw std::runtime_error("interior basis function not zero on a face at N=" + std::to_string(N));
      }
    Mat WL(Np * Nfc);
    for (int j = 0; j < Nfc; ++j)
      for (int m = 0; m < Np; ++m) WL[m * Nfc + j] = gw[j] * L[j * Np + m];
    C.Lc[f] = matmul(R.Minv, WL, Np, Np, Nfc);
  }
  return C;
}

}  // namespace

const CubOps& cub_ops(int N) {
  static std::mutex mu;
  static CubOps cache[kMaxN + 1];
  if (N < 1 || N > kMaxN) throw std::runtime_error("degree out of range");
  std::lock_guard<std::mutex> lk(mu);
  if (cache[N].N == 0) cache[N] = build_cub(N);
  return cache[N];
}

std::vector<double> interp_matrix(int Nc, int Nf) {
  const RefOps& C = ref_ops(Nc);
  const RefOps& F = ref_ops(Nf);
  int npc = C.Np, npf = F.Np;
  Mat Vc(npc * npc);
  for (int n = 0; n < npc; ++n) dubiner(Nc, C.r[n], C.s[n], &Vc[n * npc], nullptr, nullptr);
  Mat Vci = inverse(Vc, npc);
  Mat P(npf * npc);
  for (int n = 0; n < npf; ++n) dubiner(Nc, F.r[n], F.s[n], &P[n * npc], nullptr, nullptr);
  return matmul(P, Vci, npf, npc, npc);
}

}  // namespace ipdg
