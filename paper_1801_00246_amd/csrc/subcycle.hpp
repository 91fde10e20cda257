// Subcycling advection (Sec. 2.3, Eq. SS_3 and INS_CUB_N; Sec. 5.3, Eq.
// KSS_3, Alg. SSV and SSS): the operator N~(Ubar, U~) with cubature, and the
// five-stage low-storage Runge-Kutta subcycle; kernels in subcycle.hip, host
// side in subcycle.cpp.  FP64.
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "handle.hpp"

namespace ipdg {

// Sizes of the matrix-core form of the operator at degree N.  A wave handles
// 16 elements (the columns of 16 x 16 blocks); operators are A operands of
// v_mfma_f64_16x16x4f64 stored in lane order, 64 values per block:
//   I   [TC][KB]      lane l: I[16 T + l%16][4 kb + l/16]          (Nc x Np)
//   Pr  [RB][TC][4]   lane l: Pr[16 R + l%16][16 T + 4 t + l/16]   (Np x Nc)
//   Ps  like Pr
//   If  [3][KF]       lane l: I^f[l%16][4 kb + l/16]               (Nfc x Nfp)
//   Lc  [3][RB][KT]   lane l: Lc^f[16 R + l%16][4 t + l/16]        (Np x Nfc)
// entries outside the operators are zero.
struct SubDims {
  int Np, Nfp, q, Nc, Nfc, TC, KB, RB, KF, KT;
  int oI, oPr, oPs, oIf, oLc, total;  // offsets and size in doubles
};
__host__ __device__ constexpr SubDims sub_dims(int N) {
  SubDims d{};
  d.Np = (N + 1) * (N + 2) / 2;
  d.Nfp = N + 1;
  d.q = 3 * N / 2 + 1;
  d.Nc = d.q * d.q;
  d.Nfc = d.q;
  d.TC = (d.Nc + 15) / 16;
  d.KB = (d.Np + 3) / 4;
  d.RB = (d.Np + 15) / 16;
  d.KF = (d.Nfp + 3) / 4;
  d.KT = (d.Nfc + 3) / 4;
  d.oI = 0;
  d.oPr = d.oI + 64 * d.TC * d.KB;
  d.oPs = d.oPr + 64 * d.RB * d.TC * 4;
  d.oIf = d.oPs + 64 * d.RB * d.TC * 4;
  d.oLc = d.oIf + 64 * 3 * d.KF;
  d.total = d.oLc + 64 * 3 * d.RB * d.KT;
  return d;
}

// Fields are device FP64 vectors of K Np values.  The advecting field is
// Ubar(tau) = ub0 + tau ub1, the Dirichlet data of U~ g(tau) = g0 + tau g1
// (the *1 fields may be null: zero rate; g0 null: zero data).
struct SubArgs {
  const double* ub0 = nullptr;
  const double* vb0 = nullptr;
  const double* ub1 = nullptr;
  const double* vb1 = nullptr;
  const double* u = nullptr;
  const double* v = nullptr;
  const double* gu0 = nullptr;
  const double* gv0 = nullptr;
  const double* gu1 = nullptr;
  const double* gv1 = nullptr;
  double tau = 0.0;
  // plain output: N~ (the selected parts)
  double* out_u = nullptr;
  double* out_v = nullptr;
  // Runge-Kutta stage: res = a res - dt N~;  new = U~ + b res
  double* res_u = nullptr;
  double* res_v = nullptr;
  double* new_u = nullptr;
  double* new_v = nullptr;
  double rk_a = 0.0, rk_b = 0.0, dt = 0.0;
  const double* geo = nullptr;   // r_x, s_x, r_y, s_y per element
  const Conn* conn = nullptr;
  const double* tab = nullptr;   // operators in the SubDims layout
  int K = 0;
};

// parts: 1 volume (Alg. SSV), 2 surface (Alg. SSS), 3 both; stage: false
// writes N~ to out, true performs the Runge-Kutta stage.
hipError_t subcycle_launch(int N, int parts, bool stage, const SubArgs& a, hipStream_t s);

// Device copy of the operators of degree N (cached per device).
const double* device_sub_ops(int N);

// N~(Ubar, U~) of the selected parts.
void subcycle_rhs(ipdg_mesh_s* m, const SubArgs& in, int parts, double* nu, double* nv, hipStream_t s);

// Ns steps over [0, T] of dU~/dtau = -N~(Ubar(tau), U~) (u, v in place).
void subcycle_advect(ipdg_mesh_s* m, const SubArgs& in, double T, int Ns, double* u, double* v, hipStream_t s);

}  // namespace ipdg
