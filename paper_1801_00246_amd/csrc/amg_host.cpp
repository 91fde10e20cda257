// Host construction of the aggregation AMG hierarchy (Sec. 3, pMG-AMG):
// aggregation, aggregate graphs, Galerkin products, Gershgorin bounds and the
// inverse of the coarsest matrix.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <tuple>

#include "amg.hpp"

namespace ipdg {

int amg_aggregate(const std::vector<int>& ptr, const std::vector<int>& adj, std::vector<int>& agg) {
  const int n = int(ptr.size()) - 1;
  agg.assign(n, -1);
  int na = 0;
  for (int i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    bool free_nbhd = true;
    for (int k = ptr[i]; k < ptr[i + 1] && free_nbhd; ++k) free_nbhd = agg[adj[k]] < 0;
    if (!free_nbhd) continue;
    agg[i] = na;
    for (int k = ptr[i]; k < ptr[i + 1]; ++k) agg[adj[k]] = na;
    ++na;
  }
  const std::vector<int> first = agg;
  for (int i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    // neighbours are ascending: the first one with an aggregate is the lowest
    for (int k = ptr[i]; k < ptr[i + 1]; ++k)
      if (first[adj[k]] >= 0) {
        agg[i] = first[adj[k]];
        break;
      }
  }
  return na;
}

void amg_coarse_graph(const std::vector<int>& ptr, const std::vector<int>& adj, const std::vector<int>& agg,
                      int na, std::vector<int>& cptr, std::vector<int>& cadj) {
  const int n = int(ptr.size()) - 1;
  std::vector<std::pair<int, int>> e;
  for (int i = 0; i < n; ++i)
    for (int k = ptr[i]; k < ptr[i + 1]; ++k)
      if (agg[adj[k]] != agg[i]) e.emplace_back(agg[i], agg[adj[k]]);
  std::sort(e.begin(), e.end());
  e.erase(std::unique(e.begin(), e.end()), e.end());
  cptr.assign(na + 1, 0);
  cadj.resize(e.size());
  for (size_t k = 0; k < e.size(); ++k) {
    ++cptr[e[k].first + 1];
    cadj[k] = e[k].second;
  }
  for (int a = 0; a < na; ++a) cptr[a + 1] += cptr[a];
}

Csr amg_galerkin(const Csr& A, const std::vector<int>& agg, int na) {
  std::vector<std::tuple<int, int, double>> t;
  t.reserve(A.val.size());
  for (int i = 0; i < A.n; ++i)
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) t.emplace_back(agg[i], agg[A.col[k]], A.val[k]);
  // stable: equal (row, column) pairs are summed in the fine matrix's order
  std::stable_sort(t.begin(), t.end(), [](const auto& a, const auto& b) {
    return std::get<0>(a) != std::get<0>(b) ? std::get<0>(a) < std::get<0>(b) : std::get<1>(a) < std::get<1>(b);
  });
  Csr C;
  C.n = na;
  C.ptr.assign(na + 1, 0);
  for (size_t k = 0; k < t.size();) {
    const int r = std::get<0>(t[k]), c = std::get<1>(t[k]);
    double v = 0.0;
    for (; k < t.size() && std::get<0>(t[k]) == r && std::get<1>(t[k]) == c; ++k) v += std::get<2>(t[k]);
    C.col.push_back(c);
    C.val.push_back(v);
    ++C.ptr[r + 1];
  }
  for (int a = 0; a < na; ++a) C.ptr[a + 1] += C.ptr[a];
  return C;
}

double amg_gershgorin(const Csr& A) {
  double mx = 0.0;
  for (int i = 0; i < A.n; ++i) {
    double s = 0.0, d = 0.0;
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      s += std::fabs(A.val[k]);
      if (A.col[k] == i) d = A.val[k];
    }
    mx = std::max(mx, s / d);
  }
  return mx;
}

bool amg_spd_inverse(const Csr& A, std::vector<double>& inv) {
  const int n = A.n;
  std::vector<double> L((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) L[(size_t)i * n + A.col[k]] = A.val[k];
  // A = L L^T (lower triangle, in place, by rows)
  for (int i = 0; i < n; ++i) {
    double* Li = &L[(size_t)i * n];
    for (int j = 0; j <= i; ++j) {
      const double* Lj = &L[(size_t)j * n];
      double s = Li[j];
      for (int k = 0; k < j; ++k) s -= Li[k] * Lj[k];
      if (j < i) {
        Li[j] = s / Lj[j];
      } else {
        if (!(s > 0.0)) return false;
        Li[i] = std::sqrt(s);
      }
    }
    for (int j = i + 1; j < n; ++j) Li[j] = 0.0;
  }
  // W = L^-1 (lower triangular), by forward substitution per column
  std::vector<double> W((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    W[(size_t)c * n + c] = 1.0 / L[(size_t)c * n + c];
    for (int i = c + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = c; k < i; ++k) s += L[(size_t)i * n + k] * W[(size_t)k * n + c];
      W[(size_t)i * n + c] = -s / L[(size_t)i * n + i];
    }
  }
  // A^-1 = W^T W
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = 0.0;
      for (int k = i; k < n; ++k) s += W[(size_t)k * n + i] * W[(size_t)k * n + j];
      inv[(size_t)i * n + j] = s;
      inv[(size_t)j * n + i] = s;
    }
  return true;
}

}  // namespace ipdg
