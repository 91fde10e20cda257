// PCG without device allocation: its work memory is a fixed file-scope
// device array (noalloc.hip).
#pragma once
#include <cstddef>

#include "handle.hpp"

namespace ipdg {

// Largest K * Np the allocation-free solve accepts.
constexpr size_t kNoAllocMaxDofs = size_t(1) << 20;

// Looks up this device's scratch address (loading the array's code object);
// called at mesh creation so that the solve itself finds it ready.
void noalloc_prepare();

ipdg_status pcg_solve_noalloc(ipdg_mesh_s* m, double lambda, double tau, const double* b, double* x,
                              double tol, const ipdg_solve_opts& o, ipdg_solve_info* info,
                              hipStream_t s);

}  // namespace ipdg
