#include "ops_table.hpp"

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
  t.reserve(ops_total(N));
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
  return t;
}

}  // namespace ipdg
