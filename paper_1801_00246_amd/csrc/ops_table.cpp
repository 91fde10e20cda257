#include "ops_table.hpp"

#include <stdexcept>

#include "refelem.hpp"
#include "tri.hpp"

namespace ipdg {
namespace {
std::vector<double> mul(const std::vector<double>& A, const std::vector<double>& B, int m, int k, int n) {
  std::vector<double> C((size_t)m * n, 0.0);
  for (int i = 0; i < m; ++i)
    for (int p = 0; p < k; ++p)
      for (int j = 0; j < n; ++j) C[i * n + j] += A[i * k + p] * B[p * n + j];
  return C;
}
}  // namespace

std::vector<double> build_ops_table(int N) {
  const RefOps& R = ref_ops(N);
  const int Np = R.Np, Nfp = R.Nfp;
  std::vector<double> Krr = mul(R.Sr, R.Dr, Np, Np, Np);
  std::vector<double> Kss = mul(R.Ss, R.Ds, Np, Np, Np);
  std::vector<double> Krs = mul(R.Sr, R.Ds, Np, Np, Np);
  std::vector<double> Ksr = mul(R.Ss, R.Dr, Np, Np, Np);
  for (size_t i = 0; i < Krs.size(); ++i) Krs[i] += Ksr[i];
  std::vector<double> QR = mul(R.Sr, R.LIFT, Np, Np, 3 * Nfp);
  std::vector<double> QS = mul(R.Ss, R.LIFT, Np, Np, 3 * Nfp);
  std::vector<double> t;
  t.reserve(ops_table_len(N));
  auto put = [&](const std::vector<double>& v) { t.insert(t.end(), v.begin(), v.end()); };
  put(R.Dr);
  put(R.Ds);
  put(Krr);
  put(Krs);
  put(Kss);
  put(R.M);
  put(R.Minv);
  put(QR);
  put(QS);
  put(R.LIFT);
  put(R.M1D);
  for (int j = 0; j < Np; ++j) {
    for (int m = 0; m < Nfp; ++m) t.push_back(R.Dr[m * Np + j]);
    for (int m = 0; m < Nfp; ++m) t.push_back(R.Ds[m * Np + j]);
  }
  std::vector<double> E = mul(R.M, R.LIFT, Np, Np, 3 * Nfp);
  for (int i = 0; i < Np; ++i) {
    auto row = [&](const std::vector<double>& A, int n) {
      t.insert(t.end(), A.begin() + (size_t)i * n, A.begin() + (size_t)(i + 1) * n);
    };
    row(Krr, Np);
    row(Krs, Np);
    row(Kss, Np);
    row(QR, 3 * Nfp);
    row(QS, 3 * Nfp);
    row(E, 3 * Nfp);
    row(R.M, Np);
  }
  // cooperative-kernel streams (layout CoopLayout<N> in tri.hpp)
  auto fm = [&](int f, int k) {
    auto id = [&](int i, int j) { return j * (N + 1) - (j * (j - 1)) / 2 + i; };
    return f == 0 ? id(k, 0) : (f == 1 ? id(N - k, k) : id(0, N - k));
  };
  for (int f = 0; f < 3; ++f)
    for (int j = 0; j < Np; ++j)
      for (int k = 0; k < Nfp; ++k) {
        t.push_back(R.Dr[fm(f, k) * Np + j]);
        t.push_back(R.Ds[fm(f, k) * Np + j]);
      }
  for (int f2 = 0; f2 < 3; ++f2)
    for (int p = 0; p < Nfp; ++p)
      for (int q = 0; q < 3 * Nfp; ++q) t.push_back(R.LIFT[fm(f2, p) * 3 * Nfp + q]);
  const int W = 3;
  for (int w = 0; w < W; ++w) {
    const int b = (w * Np + W - 1) / W, e = ((w + 1) * Np + W - 1) / W;
    for (int j = 0; j < Np; ++j)
      for (int i = b; i < e; ++i) {
        t.push_back(Krr[i * Np + j]);
        t.push_back(Krs[i * Np + j]);
        t.push_back(Kss[i * Np + j]);
      }
    for (int j = 0; j < Np; ++j)
      for (int i = b; i < e; ++i) t.push_back(R.M[i * Np + j]);
    for (int q = 0; q < 3 * Nfp; ++q)
      for (int i = b; i < e; ++i) {
        t.push_back(QR[i * 3 * Nfp + q]);
        t.push_back(QS[i * 3 * Nfp + q]);
      }
  }
  // matrix-core operand blocks (layout MfmaLayout<N> in tri.hpp)
  {
    const int RB = (Np + 15) / 16, KBV = (Np + 3) / 4, KBF = (3 * Nfp + 3) / 4;
    auto blocks = [&](const std::vector<double>& A, int ncol, int kbn, double sign) {
      for (int rb = 0; rb < RB; ++rb)
        for (int kb = 0; kb < kbn; ++kb)
          for (int l = 0; l < 64; ++l) {
            const int i = 16 * rb + l % 16, k = 4 * kb + l / 16;
            t.push_back(i < Np && k < ncol ? sign * A[(size_t)i * ncol + k] : 0.0);
          }
    };
    blocks(Krr, Np, KBV, 1.0);
    blocks(Krs, Np, KBV, 1.0);
    blocks(Kss, Np, KBV, 1.0);
    blocks(R.M, Np, KBV, 1.0);
    blocks(QR, 3 * Nfp, KBF, 1.0);
    blocks(QS, 3 * Nfp, KBF, 1.0);
    blocks(E, 3 * Nfp, KBF, -1.0);
  }
  if ((int)t.size() != ops_table_len(N)) throw std::logic_error("operator table length mismatch");
  return t;
}

}  // namespace ipdg
