// Aggregation algebraic multigrid below the degree-1 p-multigrid level
// (Sec. 3, the pMG-AMG hybrid): host construction of the hierarchy
// (amg_host.cpp) and the device kernels of its cycle (amg.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

namespace ipdg {

// Sparse matrix in compressed rows, columns ascending within a row.
struct Csr {
  int n = 0;
  std::vector<int> ptr, col;
  std::vector<double> val;
};

// Greedy aggregation of a graph (adjacency lists in compressed form,
// neighbours ascending, no self loops).  First pass: nodes in index order; a
// node that is still free and whose neighbours are all free starts an
// aggregate holding it and its neighbours.  Second pass: a node left free
// joins the first-pass aggregate of its lowest-index neighbour that has one.
// Aggregates are numbered in order of creation; the choices depend on the
// graph alone.  Returns the number of aggregates; agg[i] is node i's.
int amg_aggregate(const std::vector<int>& ptr, const std::vector<int>& adj, std::vector<int>& agg);

// Graph of the aggregates: a and b adjacent when some member of a is
// adjacent to some member of b (a != b); lists ascending.
void amg_coarse_graph(const std::vector<int>& ptr, const std::vector<int>& adj, const std::vector<int>& agg,
                      int na, std::vector<int>& cptr, std::vector<int>& cadj);

// Galerkin product P^T A P for the 0/1 aggregate map P (entries of A summed
// into their aggregates' rows and columns).
Csr amg_galerkin(const Csr& A, const std::vector<int>& agg, int na);

// Gershgorin bound of the spectral radius of D^-1 A: max_i sum_j |A_ij| / A_ii.
double amg_gershgorin(const Csr& A);

// Inverse of a symmetric positive definite matrix (dense, row-major, n x n)
// by Cholesky factorisation; false when a pivot is not positive.
bool amg_spd_inverse(const Csr& A, std::vector<double>& inv);

// ---- device kernels (T = float when fp32, else double); every launch is a
// no-op while *skip is set (skip may be null) ----
// y = A x (compressed rows)
hipError_t amg_spmv(bool fp32, const int* ptr, const int* col, const void* val, const void* x, void* y, int n,
                    const int* skip, hipStream_t s);
// rc[i] = sum over the members j of aggregate i of (f[j] - t[j]) (t may be
// null: f alone); members listed by mptr/mem (ascending)
hipError_t amg_restrict(bool fp32, const int* mptr, const int* mem, const void* f, const void* t, void* rc, int nc,
                        const int* skip, hipStream_t s);
// z[j] += zc[agg[j]]
hipError_t amg_prolong(bool fp32, const int* agg, const void* zc, void* z, int n, const int* skip, hipStream_t s);
// z = inv f (dense n x n, row-major)
hipError_t amg_dense(bool fp32, const void* inv, const void* f, void* z, int n, const int* skip, hipStream_t s);
// r = f - t
hipError_t amg_sub(bool fp32, const void* f, const void* t, void* r, size_t n, const int* skip, hipStream_t s);
// x += y
hipError_t amg_add(bool fp32, void* x, const void* y, size_t n, const int* skip, hipStream_t s);

}  // namespace ipdg
