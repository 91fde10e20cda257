// DG gradient and divergence with central fluxes (Sec. 2.1, Eq. INS_SD_4_1
// and INS_SD_4_2) and the element-local steps of the algebraic splitting
// scheme around its two elliptic solves (Sec. 2.2, Eq. INS_TD_3_2 to
// INS_TD_3_4); kernels in gradiv.hip, FP64.
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace ipdg {

struct GradArgs {
  const double* p = nullptr;       // pressure-like field
  const double* base_x = nullptr;  // optional: added fields (a_base times)
  const double* base_y = nullptr;
  double* out_x = nullptr;
  double* out_y = nullptr;
  double a_base = 0.0, a_grad = 1.0;
  bool mass = false;               // out = J M (a_base base + a_grad G p) when set
  const double* add_p = nullptr;   // optional: p_out = p + add_p
  double* p_out = nullptr;
  const double* geo = nullptr;     // r_x, s_x, r_y, s_y per element
  const Conn* conn = nullptr;
  const double* ops = nullptr;     // FP64 reference operators of the degree
  int K = 0;
};

struct DivArgs {
  const double* u = nullptr;
  const double* v = nullptr;
  const double* gu = nullptr;      // Dirichlet data (nodal fields, face nodes used); null = 0
  const double* gv = nullptr;
  double* out = nullptr;
  double scale = 1.0;
  bool mass = false;               // out = scale J M D (u, v) when set, else scale D (u, v)
  const double* geo = nullptr;
  const Conn* conn = nullptr;
  const double* ops = nullptr;
  int K = 0;
};

// b += the right-hand-side terms of inhomogeneous Dirichlet data g (a nodal
// field; its face-node values on the Dirichlet faces) for the SIPDG operator:
// -kappa (g, d_n l_i)_F + 2 tau_F (g, l_i)_F, tau_F = c_tau kappa |F| / |E|
struct DirichletArgs {
  const double* g = nullptr;
  double* b = nullptr;
  const double* kap = nullptr;     // per-element coefficient, null = 1
  double ctau = 0.0;
  const double* geo = nullptr;
  const Conn* conn = nullptr;
  const double* ops = nullptr;
  int K = 0;
};
hipError_t dirichlet_rhs(int N, const DirichletArgs& a, hipStream_t s);

// out = a_base base + a_adv N(u, v): the nodal Lax-Friedrichs advection term
// of Eq. INS_SD_2 / INS_SD_3 per velocity component (Dirichlet faces take
// u+ = g, Neumann faces u+ = u-)
struct AdvectArgs {
  const double* u = nullptr;
  const double* v = nullptr;
  const double* gu = nullptr;      // Dirichlet data (nodal fields), null = 0
  const double* gv = nullptr;
  const double* base_u = nullptr;  // optional
  const double* base_v = nullptr;
  double a_base = 0.0, a_adv = 1.0;
  double* out_u = nullptr;
  double* out_v = nullptr;
  const double* geo = nullptr;
  const Conn* conn = nullptr;
  const double* ops = nullptr;
  int K = 0;
};
hipError_t advect_apply(int N, const AdvectArgs& a, hipStream_t s);

// z = a x + b y (n values)
hipError_t axpby(double a, const double* x, double b, const double* y, double* z, size_t n, hipStream_t s);
// b -= (sum b / area) J M 1: removes the component of b that a pure-Neumann
// Laplacian cannot reach (its null space is the constants); work: 1 double
hipError_t remove_mean(int N, double* b, double area, const double* geo, const double* ops, int K, double* work,
                       hipStream_t s);

// Matrix-core form of the gradient and the advection term (degrees 2-8) and
// the divergence: 16 elements
// per wave as the columns of v_mfma_f64_16x16x4f64 blocks, the operators as A
// operands in lane order (64 values per block; entries outside the operators
// zero):
//   Dr, Ds [RB][KB]      lane l: D[16 R + l%16][4 kb + l/16]          (Np x Np)
//   L      [3][RB][KF]   lane l: LIFT[16 R + l%16][f Nfp + 4 kb + l/16] (face f's columns)
//   M      [RB][RB][4]   lane l: M[16 R + l%16][16 R2 + 4 t + l/16]
struct GdDims {
  int Np, Nfp, RB, KB, KF;
  int oDr, oDs, oL, oM, total;
};
__host__ __device__ constexpr GdDims gd_dims(int N) {
  GdDims d{};
  d.Np = (N + 1) * (N + 2) / 2;
  d.Nfp = N + 1;
  d.RB = (d.Np + 15) / 16;
  d.KB = (d.Np + 3) / 4;
  d.KF = (d.Nfp + 3) / 4;
  d.oDr = 0;
  d.oDs = d.oDr + 64 * d.RB * d.KB;
  d.oL = d.oDs + 64 * d.RB * d.KB;
  d.oM = d.oL + 64 * 3 * d.RB * d.KF;
  d.total = d.oM + 64 * d.RB * d.RB * 4;
  return d;
}
// Device copy of that table for degree N (cached per device; gradiv_host.cpp).
const double* device_gd_tab(int N);

// out = a_base base + a_grad G p (or J M of it), p_out = p + add_p
hipError_t grad_apply(int N, const GradArgs& a, hipStream_t s);
// out = scale D (u, v) (or scale J M D (u, v))
hipError_t div_apply(int N, const DivArgs& a, hipStream_t s);

}  // namespace ipdg
