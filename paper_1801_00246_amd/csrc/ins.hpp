// One step of the algebraic splitting scheme (Sec. 2.2, Eq. INS_TD_3); ins.cpp.
#pragma once
#include "handle.hpp"

namespace ipdg {

// Velocity, pressure and Dirichlet velocity data at one time level (device
// FP64 vectors of K Np values; gu, gv may be null for zero data).
struct InsState {
  const double* u = nullptr;
  const double* v = nullptr;
  const double* p = nullptr;
  const double* p_prev = nullptr;   // input only: P^{n-1}
  const double* gu = nullptr;
  const double* gv = nullptr;
  // > 0: the advection stage is the semi-Lagrangian subcycle (Sec. 2.3) of
  // this many Runge-Kutta substeps instead of one explicit step
  int subcycles = 0;
};
struct InsOut {
  double* u = nullptr;
  double* v = nullptr;
  double* p = nullptr;
  const double* gu = nullptr;       // data at t^{n+1}
  const double* gv = nullptr;
};

// Returns the first non-OK status of the three solves (iters: their
// iteration counts, velocity u, v and pressure; may be null).
ipdg_status ins_step(ipdg_mesh_s* m, ipdg_mesh_s* pm, double nu, double dt, double tau, const InsState& in,
                     const InsOut& out, double tol, const ipdg_solve_opts& vo, const ipdg_solve_opts& po, int* iters,
                     hipStream_t s);

}  // namespace ipdg
