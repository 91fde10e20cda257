// One step of the algebraic splitting scheme of Sec. 2.2 (Eq. INS_TD_3),
// first order in time (gamma = beta_0 = alpha_0 = 1) with the pressure
// increment over the second-order extrapolation sigma P = 2 P^n - P^{n-1}:
//
//   U^   = U^n - dt N(U^n)                                   (Eq. INS_TD_3_1)
//   (gamma / (nu dt) M - Lap) U^^ = M (U^ / (nu dt) - G sigma P / nu) + b_g  (INS_TD_3_2)
//   -Lap dP = -(gamma / dt) D U^^                            (Eq. INS_TD_3_3)
//   U^{n+1} = U^^ - (dt / gamma) G dP,  P^{n+1} = dP + sigma P   (Eq. INS_TD_3_4)
//
// With subcycles > 0 the first line is the Lagrangian form of Sec. 2.3 at
// first order (S = 0): U^ = U~(t^{n+1}), where dU~/dt = -N~(U^n, U~) is
// advanced from U~(t^n) = U^n by that many low-storage Runge-Kutta substeps,
// the Dirichlet data of U~ interpolated linearly between t^n and t^{n+1}.
//
// Every step runs in the library's kernels (advection, gradient,
// divergence, Dirichlet data, vector updates) and its PCG; the velocity mesh
// carries the velocity boundary flags, the pressure mesh the same triangles
// with the flags swapped.  A pressure mesh without Dirichlet faces has the
// constants as null space: the right-hand side's component along them is
// removed first (it is only the boundary flux of the interpolated data).
#include <cstring>
#include <string>

#include "gradiv.hpp"
#include "ins.hpp"
#include "solver.hpp"
#include "subcycle.hpp"

namespace ipdg {

ipdg_status ins_step(ipdg_mesh_s* m, ipdg_mesh_s* pm, double nu, double dt, double tau, const InsState& in,
                     const InsOut& out, double tol, const ipdg_solve_opts& vo, const ipdg_solve_opts& po, int* iters,
                     hipStream_t s) {
  const HostMesh& h = m->host;
  if (pm->host.N != h.N || pm->host.K != h.K || pm->host.EToV != h.EToV)
    throw Error(IPDG_EINVAL, "the pressure mesh must hold the velocity mesh's triangles at its degree");
  if (!(nu > 0.0) || !(dt > 0.0)) throw Error(IPDG_EINVAL, "nu and dt must be positive");
  const int N = h.N, K = h.K;
  const size_t n = (size_t)K * m->Np;
  const double gamma = 1.0;
  const double* geo = m->geo64.as<double>();
  const Conn* conn = m->conn.as<Conn>();
  const double* ops = static_cast<const double*>(device_ops(N, Kind::F64));
  const bool sub = in.subcycles > 0;
  const bool data = in.gu || in.gv || out.gu || out.gv;
  DevBuf work(((sub && data) ? 13 : 9) * n * sizeof(double) + 64);
  double* w = work.as<double>();
  double *uh = w, *vh = w + n, *bu = w + 2 * n, *bv = w + 3 * n, *uhh = w + 4 * n, *vhh = w + 5 * n;
  double *bp = w + 6 * n, *dp = w + 7 * n, *sp = w + 8 * n;
  double* scal = w + 9 * n;

  if (sub) {
    // Sec. 2.3: U^ = U~(t^{n+1}) with Ubar = U^n; data g(tau) = g^n + tau (g^{n+1} - g^n) / dt
    SubArgs sa;
    sa.ub0 = in.u;
    sa.vb0 = in.v;
    if (data) {
      double *g0u = w + 9 * n + 8, *g0v = g0u + n, *g1u = g0v + n, *g1v = g1u + n;
      IPDG_HIP(hipMemsetAsync(g0u, 0, 4 * n * sizeof(double), s));
      if (in.gu) IPDG_HIP(hipMemcpyAsync(g0u, in.gu, n * sizeof(double), hipMemcpyDeviceToDevice, s));
      if (in.gv) IPDG_HIP(hipMemcpyAsync(g0v, in.gv, n * sizeof(double), hipMemcpyDeviceToDevice, s));
      // g1 = (g^{n+1} - g^n) / dt (absent data are zero)
      IPDG_HIP(axpby(1.0 / dt, out.gu ? out.gu : g1u, -1.0 / dt, g0u, g1u, n, s));
      IPDG_HIP(axpby(1.0 / dt, out.gv ? out.gv : g1v, -1.0 / dt, g0v, g1v, n, s));
      sa.gu0 = g0u;
      sa.gv0 = g0v;
      sa.gu1 = g1u;
      sa.gv1 = g1v;
    }
    IPDG_HIP(hipMemcpyAsync(uh, in.u, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    IPDG_HIP(hipMemcpyAsync(vh, in.v, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    subcycle_advect(m, sa, dt, in.subcycles, uh, vh, s);
  }

  // Eq. INS_TD_3_1 (data at t^n)
  AdvectArgs aa;
  aa.u = in.u;
  aa.v = in.v;
  aa.gu = in.gu;
  aa.gv = in.gv;
  aa.base_u = in.u;
  aa.base_v = in.v;
  aa.a_base = 1.0;
  aa.a_adv = -dt;
  aa.out_u = uh;
  aa.out_v = vh;
  aa.geo = geo;
  aa.conn = conn;
  aa.ops = ops;
  aa.K = K;
  if (!sub) IPDG_HIP(advect_apply(N, aa, s));
  IPDG_HIP(axpby(2.0, in.p, -1.0, in.p_prev, sp, n, s));

  // Eq. INS_TD_3_2 (data at t^{n+1})
  GradArgs ga;
  ga.p = sp;
  ga.base_x = uh;
  ga.base_y = vh;
  ga.a_base = 1.0 / (nu * dt);
  ga.a_grad = -1.0 / nu;
  ga.mass = true;
  ga.out_x = bu;
  ga.out_y = bv;
  ga.geo = geo;
  ga.conn = conn;
  ga.ops = ops;
  ga.K = K;
  IPDG_HIP(grad_apply(N, ga, s));
  DirichletArgs da;
  da.kap = m->has_kappa ? m->kap64.as<double>() : nullptr;
  da.ctau = ctau_of(N, tau);
  da.geo = geo;
  da.conn = conn;
  da.ops = ops;
  da.K = K;
  if (out.gu) {
    da.g = out.gu;
    da.b = bu;
    IPDG_HIP(dirichlet_rhs(N, da, s));
  }
  if (out.gv) {
    da.g = out.gv;
    da.b = bv;
    IPDG_HIP(dirichlet_rhs(N, da, s));
  }
  IPDG_HIP(hipMemcpyAsync(uhh, in.u, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  IPDG_HIP(hipMemcpyAsync(vhh, in.v, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  ipdg_solve_info info{};
  const double lam = gamma / (nu * dt);
  ipdg_status st = pcg_solve(m, lam, tau, bu, uhh, tol, vo, &info, s);
  if (iters) iters[0] = info.iters;
  if (st != IPDG_OK) return st;
  st = pcg_solve(m, lam, tau, bv, vhh, tol, vo, &info, s);
  if (iters) iters[1] = info.iters;
  if (st != IPDG_OK) return st;

  // Eq. INS_TD_3_3 (data at t^{n+1})
  DivArgs dv;
  dv.u = uhh;
  dv.v = vhh;
  dv.gu = out.gu;
  dv.gv = out.gv;
  dv.out = bp;
  dv.scale = -gamma / dt;
  dv.mass = true;
  dv.geo = geo;
  dv.conn = conn;
  dv.ops = ops;
  dv.K = K;
  IPDG_HIP(div_apply(N, dv, s));
  bool pure_neumann = true;
  for (int8_t b : pm->host.EToB) pure_neumann = pure_neumann && b != IPDG_BC_DIRICHLET;
  if (pure_neumann) {
    double area = 0.0;
    for (double J : h.J) area += 2.0 * J;
    IPDG_HIP(remove_mean(N, bp, area, geo, ops, K, scal, s));
  }
  IPDG_HIP(hipMemsetAsync(dp, 0, n * sizeof(double), s));
  st = pcg_solve(pm, 0.0, tau, bp, dp, tol, po, &info, s);
  if (iters) iters[2] = info.iters;
  if (st != IPDG_OK) return st;

  // Eq. INS_TD_3_4
  GradArgs gc;
  gc.p = dp;
  gc.base_x = uhh;
  gc.base_y = vhh;
  gc.a_base = 1.0;
  gc.a_grad = -dt / gamma;
  gc.out_x = out.u;
  gc.out_y = out.v;
  gc.add_p = sp;
  gc.p_out = out.p;
  gc.geo = geo;
  gc.conn = conn;
  gc.ops = ops;
  gc.K = K;
  IPDG_HIP(grad_apply(N, gc, s));
  IPDG_HIP(hipStreamSynchronize(s));
  return IPDG_OK;
}

}  // namespace ipdg
