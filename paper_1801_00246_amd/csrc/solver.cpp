#include "solver.hpp"

namespace ipdg {

ipdg_status pcg_solve(ipdg_mesh_s*, double, double, const double*, double*, double,
                      const ipdg_solve_opts&, ipdg_solve_info*, hipStream_t) {
  throw Error(IPDG_EUNSUPPORTED, "pcg_solve not built yet");
}
ipdg_status precond_apply(ipdg_mesh_s*, double, double, const ipdg_solve_opts&, const double*,
                          double*, ipdg_solve_info*, hipStream_t) {
  throw Error(IPDG_EUNSUPPORTED, "precond_apply not built yet");
}
ipdg_status solve_batch(int, ipdg_mesh_s* const*, const double*, double, const double* const*,
                        double* const*, double, const ipdg_solve_opts&, int*, double*, hipStream_t) {
  throw Error(IPDG_EUNSUPPORTED, "solve_batch not built yet");
}

}  // namespace ipdg
