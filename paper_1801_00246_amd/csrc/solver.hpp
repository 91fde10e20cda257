// PCG solvers on the device (Sec. 3): Jacobi, block inverse-mass and
// p-multigrid preconditioning, FP64 or mixed precision.
#pragma once
#include "handle.hpp"

namespace ipdg {

struct SolverWork {
  virtual ~SolverWork() = default;
};

ipdg_status pcg_solve(ipdg_mesh_s* m, double lambda, double tau, const double* b, double* x,
                      double tol, const ipdg_solve_opts& o, ipdg_solve_info* info, hipStream_t s);
ipdg_status precond_apply(ipdg_mesh_s* m, double lambda, double tau, const ipdg_solve_opts& o,
                          const double* r, double* z, ipdg_solve_info* info, hipStream_t s);
ipdg_status solve_batch(int nb, ipdg_mesh_s* const* meshes, const double* lambdas, double tau,
                        const double* const* b, double* const* x, double tol,
                        const ipdg_solve_opts& o, int* iters, double* relres, hipStream_t s);

}  // namespace ipdg
