// Subcycling advection operator with cubature (Sec. 5.3, Eq. KSS_3; the
// volume term of Alg. SSV and the surface term of Alg. SSS) on the matrix
// cores, FP64:
//
//   N~ = -[P_r (r_x F_x + r_y F_y) + P_s (s_x F_x + s_y F_y)]
//        + sum_f (|F| / |E|) L_c^f n . F~*,
//
// F~ = Ubar (x) U~ at the volume cubature nodes; n . F~* the local
// Lax-Friedrichs flux at the face Gauss points with Lambda = max(|n . Ubar-|,
// |n . Ubar+|).  The geometric factors are folded into the fluxes before the
// projection (contravariant fluxes), so the projection is two products with
// P_r, P_s per velocity component instead of the four per component of
// Alg. SSV.
//
// A wave computes 16 elements as the columns of 16 x 16 blocks of
// v_mfma_f64_16x16x4f64: interpolation I (Nc x Np) times the 16 elements'
// nodal values (B operands held in registers), the fluxes formed lane by lane
// on the accumulators, and the accumulators fed straight back as B operands
// of the projection: accumulator entry r of lane l is row l/16 + 4 r of its
// block, exactly the B operand of k-step r for cubature rows 4 r .. 4 r + 3.
// The face part does the same with the face interpolation I^f and the lift
// L_c^f.  Results leave through LDS as one contiguous block per wave.
#include <hip/hip_runtime.h>

#include <cmath>

#include "subcycle.hpp"
#include "tri.hpp"

namespace ipdg {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kSubWaves = 2;   // waves per block, 16 elements each (two blocks of 2 waves beat one of 4)

// x0[i] + tau x1[i] (x1 may be null)
__device__ __forceinline__ double lin(const double* __restrict__ x0, const double* __restrict__ x1, double tau,
                                      size_t i) {
  double x = x0[i];
  if (x1) x += tau * x1[i];
  return x;
}

// Waves per SIMD the kernels are compiled for (measured per degree on
// 524,288 triangles).  Left alone, the compiler gives the volume and fused
// kernels one or two waves from degree 7, with the wave's latency exposed;
// two are 1.2-1.7x faster there.  Three are 10-16 % faster for the fused
// kernel at degrees 3 and 4 and a few per cent for the volume kernel at 3-6;
// the fused kernel at 5 and 6 and the surface kernel keep the compiler's
// choice.
template <int N, int PARTS>
constexpr int sub_waves_per_eu() {
  if (PARTS == 2) return 1;
  if (N >= 7) return 2;
  if (PARTS == 3) return N == 3 || N == 4 ? 3 : 1;
  return N >= 3 ? 3 : 1;
}

template <int N, int PARTS, bool STAGE>
__global__ __launch_bounds__(64 * kSubWaves) __attribute__((amdgpu_waves_per_eu(sub_waves_per_eu<N, PARTS>())))
void k_subcycle(SubArgs a) {
  using Tr = Tri<N>;
  constexpr SubDims D = sub_dims(N);
  constexpr int Np = D.Np, Nfp = D.Nfp;
  static_assert(D.Nfc <= 16, "face points must fit one block row");
  __shared__ double stage[kSubWaves][2][16 * Np];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nn = lane & 15, kk = lane >> 4;
  const int e0 = (blockIdx.x * kSubWaves + w) * 16;
  const int e = e0 + nn;
  const int ec = e < a.K ? e : a.K - 1;      // lanes past the end read a valid element
  const double* __restrict__ tab = a.tab;
  const double* __restrict__ u = a.u;
  const double* __restrict__ v = a.v;
  const double rx = a.geo[4 * (size_t)ec], sx = a.geo[4 * (size_t)ec + 1];
  const double ry = a.geo[4 * (size_t)ec + 2], sy = a.geo[4 * (size_t)ec + 3];
  v4d au[D.RB], av[D.RB];
#pragma unroll
  for (int R = 0; R < D.RB; ++R) {
    au[R] = v4d{0.0, 0.0, 0.0, 0.0};
    av[R] = v4d{0.0, 0.0, 0.0, 0.0};
  }

  if constexpr ((PARTS & 1) != 0) {
    // B operands: node 4 kb + l/16 of element l%16 (rows past Np meet zero
    // columns of I)
    double bub[D.KB], bvb[D.KB], bu[D.KB], bv[D.KB];
#pragma unroll
    for (int kb = 0; kb < D.KB; ++kb) {
      const int j = 4 * kb + kk < Np ? 4 * kb + kk : Np - 1;
      const size_t i = (size_t)ec * Np + j;
      bub[kb] = lin(a.ub0, a.ub1, a.tau, i);
      bvb[kb] = lin(a.vb0, a.vb1, a.tau, i);
      bu[kb] = u[i];
      bv[kb] = v[i];
    }
#pragma unroll 1
    for (int tc = 0; tc < D.TC; ++tc) {
      v4d d0 = {0.0, 0.0, 0.0, 0.0}, d1 = d0, d2 = d0, d3 = d0;
#pragma unroll
      for (int kb = 0; kb < D.KB; ++kb) {
        const double A = tab[D.oI + (tc * D.KB + kb) * 64 + lane];
        d0 = mma(A, bub[kb], d0);
        d1 = mma(A, bvb[kb], d1);
        d2 = mma(A, bu[kb], d2);
        d3 = mma(A, bv[kb], d3);
      }
      // contravariant fluxes at cubature rows 16 tc + l/16 + 4 r, with the
      // sign of the volume term
      double gru[4], gsu[4], grv[4], gsv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double ar = rx * d0[r] + ry * d1[r];
        const double as = sx * d0[r] + sy * d1[r];
        gru[r] = -ar * d2[r];
        gsu[r] = -as * d2[r];
        grv[r] = -ar * d3[r];
        gsv[r] = -as * d3[r];
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int R = 0; R < D.RB; ++R) {
          const int o = ((R * D.TC + tc) * 4 + t) * 64 + lane;
          const double pr = tab[D.oPr + o], ps = tab[D.oPs + o];
          au[R] = mma(pr, gru[t], au[R]);
          au[R] = mma(ps, gsu[t], au[R]);
          av[R] = mma(pr, grv[t], av[R]);
          av[R] = mma(ps, gsv[t], av[R]);
        }
    }
  }

  if constexpr ((PARTS & 2) != 0) {
    const Conn c = a.conn[ec];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const int bc = conn_bc(c.info, f), fp = conn_fp(c.info, f), nb = c.nb[f];
      // traces at face node 4 kb + l/16 (in this element's orientation):
      // interior (m) and exterior (p) values of Ubar and U~
      double m0[D.KF], m1[D.KF], m2[D.KF], m3[D.KF], p0[D.KF], p1[D.KF], p2[D.KF], p3[D.KF];
#pragma unroll
      for (int kb = 0; kb < D.KF; ++kb) {
        const int k = 4 * kb + kk < Nfp ? 4 * kb + kk : Nfp - 1;
        const size_t im = (size_t)ec * Np + Tr::fm(f, k);
        m0[kb] = lin(a.ub0, a.ub1, a.tau, im);
        m1[kb] = lin(a.vb0, a.vb1, a.tau, im);
        m2[kb] = u[im];
        m3[kb] = v[im];
        if (bc == 0) {
          const size_t ip = (size_t)nb * Np + Tr::fm(fp, N - k);
          p0[kb] = lin(a.ub0, a.ub1, a.tau, ip);
          p1[kb] = lin(a.vb0, a.vb1, a.tau, ip);
          p2[kb] = u[ip];
          p3[kb] = v[ip];
        } else {
          // boundary: Ubar+ = Ubar-; U~+ = g on Dirichlet faces, U~- on
          // Neumann faces
          p0[kb] = m0[kb];
          p1[kb] = m1[kb];
          if (bc == 1) {
            p2[kb] = a.gu0 ? lin(a.gu0, a.gu1, a.tau, im) : 0.0;
            p3[kb] = a.gv0 ? lin(a.gv0, a.gv1, a.tau, im) : 0.0;
          } else {
            p2[kb] = m2[kb];
            p3[kb] = m3[kb];
          }
        }
      }
      v4d dm0 = {0.0, 0.0, 0.0, 0.0}, dm1 = dm0, dm2 = dm0, dm3 = dm0, dp0 = dm0, dp1 = dm0, dp2 = dm0, dp3 = dm0;
#pragma unroll
      for (int kb = 0; kb < D.KF; ++kb) {
        const double A = tab[D.oIf + (f * D.KF + kb) * 64 + lane];
        dm0 = mma(A, m0[kb], dm0);
        dm1 = mma(A, m1[kb], dm1);
        dm2 = mma(A, m2[kb], dm2);
        dm3 = mma(A, m3[kb], dm3);
        dp0 = mma(A, p0[kb], dp0);
        dp1 = mma(A, p1[kb], dp1);
        dp2 = mma(A, p2[kb], dp2);
        dp3 = mma(A, p3[kb], dp3);
      }
      // scaled normal (|F| / |E|) n: the flux below carries the face scale
      double fx, fy;
      face_vec(f, rx, sx, ry, sy, fx, fy);
      double fu[4], fv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double anm = fx * dm0[r] + fy * dm1[r];
        const double anp = fx * dp0[r] + fy * dp1[r];
        const double lam = fmax(fabs(anm), fabs(anp));
        fu[r] = 0.5 * (anm * dm2[r] + anp * dp2[r] + lam * (dm2[r] - dp2[r]));
        fv[r] = 0.5 * (anm * dm3[r] + anp * dp3[r] + lam * (dm3[r] - dp3[r]));
      }
#pragma unroll
      for (int t = 0; t < D.KT; ++t)
#pragma unroll
        for (int R = 0; R < D.RB; ++R) {
          const double A = tab[D.oLc + ((f * D.RB + R) * D.KT + t) * 64 + lane];
          au[R] = mma(A, fu[t], au[R]);
          av[R] = mma(A, fv[t], av[R]);
        }
    }
  }

  const int ne = a.K - e0 < 16 ? a.K - e0 : 16;
  const size_t g0 = (size_t)e0 * Np;
  // Runge-Kutta stage at degrees whose wave covers at most 7 values per lane
  // and register (N <= 6): the registers' old values are loaded before the
  // staging barrier, so that their latency overlaps it (beyond that the extra
  // live values cost more than they hide)
  constexpr int kIt = (16 * Np + 63) / 64;
  constexpr bool kPre = STAGE && kIt <= 7;
  double oru[kPre ? kIt : 1], orv[kPre ? kIt : 1], ou[kPre ? kIt : 1], ov[kPre ? kIt : 1];
  if constexpr (kPre) {
#pragma unroll
    for (int j = 0; j < kIt; ++j) {
      const int idx = lane + 64 * j;
      const size_t gi = idx < ne * Np ? g0 + idx : 0;   // index 0 is valid (K >= 1)
      oru[j] = a.rk_a != 0.0 ? a.res_u[gi] : 0.0;
      orv[j] = a.rk_a != 0.0 ? a.res_v[gi] : 0.0;
      ou[j] = u[gi];
      ov[j] = v[gi];
    }
  }
  // accumulator entry r of lane l: node 16 R + l/16 + 4 r of element l%16
  double* su = stage[w][0];
  double* sv = stage[w][1];
#pragma unroll
  for (int R = 0; R < D.RB; ++R)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = 16 * R + kk + 4 * r;
      if (n < Np) {
        su[nn * Np + n] = au[R][r];
        sv[nn * Np + n] = av[R][r];
      }
    }
  __syncthreads();
  if constexpr (kPre) {
#pragma unroll
    for (int j = 0; j < kIt; ++j) {
      const int idx = lane + 64 * j;
      if (idx < ne * Np) {
        const size_t gi = g0 + idx;
        const double ru = a.rk_a * oru[j] - a.dt * su[idx];
        const double rv = a.rk_a * orv[j] - a.dt * sv[idx];
        a.res_u[gi] = ru;
        a.res_v[gi] = rv;
        a.new_u[gi] = ou[j] + a.rk_b * ru;
        a.new_v[gi] = ov[j] + a.rk_b * rv;
      }
    }
  } else {
    for (int idx = lane; idx < ne * Np; idx += 64) {
      const size_t gi = g0 + idx;
      if constexpr (!STAGE) {
        a.out_u[gi] = su[idx];
        a.out_v[gi] = sv[idx];
      } else {
        const double ru = (a.rk_a != 0.0 ? a.rk_a * a.res_u[gi] : 0.0) - a.dt * su[idx];
        const double rv = (a.rk_a != 0.0 ? a.rk_a * a.res_v[gi] : 0.0) - a.dt * sv[idx];
        a.res_u[gi] = ru;
        a.res_v[gi] = rv;
        a.new_u[gi] = u[gi] + a.rk_b * ru;
        a.new_v[gi] = v[gi] + a.rk_b * rv;
      }
    }
  }
}

template <int N>
hipError_t launch_n(int parts, bool stage, const SubArgs& a, hipStream_t s) {
  const dim3 grid((a.K + 16 * kSubWaves - 1) / (16 * kSubWaves)), block(64 * kSubWaves);
  if (stage) {
    if (parts != 3) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_subcycle<N, 3, true>), grid, block, 0, s, a);
  } else if (parts == 1) {
    hipLaunchKernelGGL((k_subcycle<N, 1, false>), grid, block, 0, s, a);
  } else if (parts == 2) {
    hipLaunchKernelGGL((k_subcycle<N, 2, false>), grid, block, 0, s, a);
  } else if (parts == 3) {
    hipLaunchKernelGGL((k_subcycle<N, 3, false>), grid, block, 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t subcycle_launch(int N, int parts, bool stage, const SubArgs& a, hipStream_t s) {
  if (a.K == 0) return hipSuccess;
  switch (N) {
    case 1: return launch_n<1>(parts, stage, a, s);
    case 2: return launch_n<2>(parts, stage, a, s);
    case 3: return launch_n<3>(parts, stage, a, s);
    case 4: return launch_n<4>(parts, stage, a, s);
    case 5: return launch_n<5>(parts, stage, a, s);
    case 6: return launch_n<6>(parts, stage, a, s);
    case 7: return launch_n<7>(parts, stage, a, s);
    case 8: return launch_n<8>(parts, stage, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ipdg
