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

// Scalars of one K-cycle coarse correction (two flexible-CG steps on the next
// level): (v1, rc), (v1, w1), (rc, rc), (v2, w1), (v2, w2), (v2, r2), and the
// flag that skips the second step (set when the first reduced |rc| to
// kcycle_t of its start or less, or when the correction itself is skipped).
struct KScal {
  double rho1 = 0, a1 = 0, rr = 0, g = 0, b = 0, rho2 = 0;
  int flag = 0, pad = 0;
};

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

// K-cycle steps (dots summed in FP64 by one block, in a fixed order):
//   kdot1: S.rho1 = (v1, rc), S.a1 = (v1, w1), S.rr = (rc, rc)
//   kres:  r2 = rc - (rho1 / a1) w1; S.flag = (r2, r2) <= t2 S.rr (1 also when
//          *skip is set, so that the second step is skipped with it)
//   kdot2: S.g = (v2, w1), S.b = (v2, w2), S.rho2 = (v2, r2) (no-op on S.flag)
//   kcomb: ec = (rho1 / a1) v1 when S.flag, else the two-step combination
//          (rho1 / a1 - g rho2 / (a1 a2)) v1 + (rho2 / a2) v2, a2 = b - g^2 / a1
hipError_t amg_kdot1(bool fp32, const void* v1, const void* rc, const void* w1, int n, KScal* S, const int* skip,
                     hipStream_t s);
hipError_t amg_kres(bool fp32, const void* rc, const void* w1, void* r2, int n, KScal* S, double t2, const int* skip,
                    hipStream_t s);
hipError_t amg_kdot2(bool fp32, const void* v2, const void* w1, const void* w2, const void* r2, int n, KScal* S,
                     hipStream_t s);
hipError_t amg_kcomb(bool fp32, const void* v1, const void* v2, void* ec, int n, const KScal* S, const int* skip,
                     hipStream_t s);

}  // namespace ipdg
