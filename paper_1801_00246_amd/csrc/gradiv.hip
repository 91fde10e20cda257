// DG gradient G and divergence D with central fluxes (Sec. 2.1, Eq.
// INS_SD_4_1 and INS_SD_4_2), in strong nodal form per element:
//   G p = grad p + LIFT (|F|/|E|) n (p* - p-),
//   D u = div u  + LIFT (|F|/|E|) n . (u* - u-),
// p* = {p}, u* = {u} on interior faces; on Dirichlet (velocity) faces
// u* = g_D and p* = p-, on Neumann faces u* = u- and p* = 0.  One element per
// lane; the reference operators D_r, D_s, LIFT and M come from the degree's
// FP64 table through wave-uniform loads, the normals and face scales
// |F|/|E| from the element's metric terms (face 0: -grad s, face 1:
// grad r + grad s, face 2: -grad r; each vector's length is |F|/|E|).
#include <hip/hip_runtime.h>

#include <cmath>

#include "gradiv.hpp"
#include "tri.hpp"

namespace ipdg {
namespace {

// Elements per block: a block stages its elements' contiguous fields through
// one LDS buffer of kElems x pitch values, so that global loads and stores
// are coalesced while each lane works on one element from registers.
template <int N>
constexpr int kElems() {
  return Tri<N>::Np <= 15 ? 256 : 128;
}
// LDS row pitch in doubles: odd, so that the lanes' rows start in different
// banks
template <int N>
constexpr int kPitchGD() {
  constexpr int Np = Tri<N>::Np;
  return (Np % 2) ? Np : Np + 1;
}

// the block's n elements' values of src, row by row, into the lanes'
// registers r[] through the LDS buffer (coalesced global reads)
template <int N>
__device__ __forceinline__ void load_rows(const double* __restrict__ src, double* lds, int e0, int n,
                                          double (&r)[Tri<N>::Np]) {
  constexpr int Np = Tri<N>::Np, P = kPitchGD<N>(), B = kElems<N>();
  const int total = n * Np;
  for (int i = threadIdx.x; i < total; i += B) lds[(i / Np) * P + i % Np] = src[(size_t)e0 * Np + i];
  __syncthreads();
  if ((int)threadIdx.x < n)
#pragma unroll
    for (int j = 0; j < Np; ++j) r[j] = lds[threadIdx.x * P + j];
  __syncthreads();
}
// the rows the lanes wrote into the LDS buffer, out to dst (coalesced)
template <int N>
__device__ __forceinline__ void store_rows(const double* lds, double* __restrict__ dst, int e0, int n) {
  constexpr int Np = Tri<N>::Np, P = kPitchGD<N>(), B = kElems<N>();
  __syncthreads();
  const int total = n * Np;
  for (int i = threadIdx.x; i < total; i += B) dst[(size_t)e0 * Np + i] = lds[(i / Np) * P + i % Np];
  __syncthreads();
}

// J M x for one element's values (registers)
template <int N>
__device__ __forceinline__ void mass_rows(const double* __restrict__ ops, double J, double (&x)[Tri<N>::Np]) {
  using L = OpsLayout<N>;
  constexpr int Np = Tri<N>::Np;
  double y[Np];
  for (int i = 0; i < Np; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < Np; ++j) s += ops[L::M + i * Np + j] * x[j];
    y[i] = J * s;
  }
#pragma unroll
  for (int i = 0; i < Np; ++i) x[i] = y[i];
}

template <int N, bool MASS>
__global__ __launch_bounds__(kElems<N>()) void k_grad(GradArgs a) {
  using T = Tri<N>;
  using L = OpsLayout<N>;
  constexpr int Np = T::Np, Nfp = T::Nfp, B = kElems<N>(), P = kPitchGD<N>();
  __shared__ double buf[B * P];
  const int e0 = blockIdx.x * B;
  const int n = min(B, a.K - e0);
  const double* __restrict__ ops = a.ops;
  const double* __restrict__ p = a.p;
  double pe[Np];
  load_rows<N>(p, buf, e0, n, pe);
  const int t = threadIdx.x, e = e0 + t;
  double gx[Np], gy[Np];
  if (t < n) {
    const double rx = a.geo[4 * (size_t)e], sx = a.geo[4 * (size_t)e + 1];
    const double ry = a.geo[4 * (size_t)e + 2], sy = a.geo[4 * (size_t)e + 3];
    // face terms (p* - p-) per face node
    double fl[3][Nfp];
    double fax[3], fay[3];
    const Conn c = a.conn[e];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const int bc = conn_bc(c.info, f);
      const int fp = conn_fp(c.info, f), nb = c.nb[f];
      face_vec(f, rx, sx, ry, sy, fax[f], fay[f]);
#pragma unroll
      for (int k = 0; k < Nfp; ++k) {
        const double pm = pe[T::fm(f, k)];
        // Dirichlet: p* = p-; Neumann: p* = 0; interior: p* = {p}
        fl[f][k] = bc == 1 ? 0.0 : (bc == 0 ? 0.5 * (p[(size_t)nb * Np + T::fm(fp, N - k)] - pm) : -pm);
      }
    }
    for (int i = 0; i < Np; ++i) {
      double dr = 0.0, ds = 0.0;
#pragma unroll
      for (int j = 0; j < Np; ++j) {
        dr += ops[L::Dr + i * Np + j] * pe[j];
        ds += ops[L::Ds + i * Np + j] * pe[j];
      }
      double vx = rx * dr + sx * ds, vy = ry * dr + sy * ds;
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < Nfp; ++k) s += ops[L::LIFT + i * 3 * Nfp + f * Nfp + k] * fl[f][k];
        vx += fax[f] * s;
        vy += fay[f] * s;
      }
      gx[i] = a.a_grad * vx;
      gy[i] = a.a_grad * vy;
    }
    if (a.base_x) {
#pragma unroll
      for (int i = 0; i < Np; ++i) {
        gx[i] += a.a_base * a.base_x[(size_t)e * Np + i];
        gy[i] += a.a_base * a.base_y[(size_t)e * Np + i];
      }
    }
    if constexpr (MASS) {
      const double J = 1.0 / (rx * sy - ry * sx);
      mass_rows<N>(ops, J, gx);
      mass_rows<N>(ops, J, gy);
    }
#pragma unroll
    for (int i = 0; i < Np; ++i) buf[t * P + i] = gx[i];
  }
  store_rows<N>(buf, a.out_x, e0, n);
  if (t < n)
#pragma unroll
    for (int i = 0; i < Np; ++i) buf[t * P + i] = gy[i];
  store_rows<N>(buf, a.out_y, e0, n);
  if (a.p_out) {
    if (t < n)
#pragma unroll
      for (int i = 0; i < Np; ++i) buf[t * P + i] = pe[i];
    __syncthreads();
    const int total = n * Np;
    for (int i = threadIdx.x; i < total; i += B)
      a.p_out[(size_t)e0 * Np + i] = buf[(i / Np) * P + i % Np] + a.add_p[(size_t)e0 * Np + i];
  }
}

template <int N, bool MASS>
__global__ __launch_bounds__(kElems<N>()) void k_div(DivArgs a) {
  using T = Tri<N>;
  using L = OpsLayout<N>;
  constexpr int Np = T::Np, Nfp = T::Nfp, B = kElems<N>(), P = kPitchGD<N>();
  __shared__ double buf[B * P];
  const int e0 = blockIdx.x * B;
  const int n = min(B, a.K - e0);
  const double* __restrict__ ops = a.ops;
  const double* __restrict__ u = a.u;
  const double* __restrict__ v = a.v;
  double ue[Np], ve[Np];
  load_rows<N>(u, buf, e0, n, ue);
  load_rows<N>(v, buf, e0, n, ve);
  const int t = threadIdx.x, e = e0 + t;
  if (t < n) {
    const double rx = a.geo[4 * (size_t)e], sx = a.geo[4 * (size_t)e + 1];
    const double ry = a.geo[4 * (size_t)e + 2], sy = a.geo[4 * (size_t)e + 3];
    // face terms n . (u* - u-) per face node
    double fl[3][Nfp];
    const Conn c = a.conn[e];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const int bc = conn_bc(c.info, f);
      const int fp = conn_fp(c.info, f), nb = c.nb[f];
      double ax, ay;
      face_vec(f, rx, sx, ry, sy, ax, ay);
#pragma unroll
      for (int k = 0; k < Nfp; ++k) {
        const int m = T::fm(f, k);
        const double um = ue[m], vm = ve[m];
        double ju = 0.0, jv = 0.0;   // Neumann: u* = u-
        if (bc == 0) {
          const size_t ip = (size_t)nb * Np + T::fm(fp, N - k);
          ju = 0.5 * (u[ip] - um);
          jv = 0.5 * (v[ip] - vm);
        } else if (bc == 1) {
          const size_t im = (size_t)e * Np + m;
          ju = (a.gu ? a.gu[im] : 0.0) - um;
          jv = (a.gv ? a.gv[im] : 0.0) - vm;
        }
        fl[f][k] = ax * ju + ay * jv;
      }
    }
    double d[Np];
    for (int i = 0; i < Np; ++i) {
      double ur = 0.0, us = 0.0, vr = 0.0, vs = 0.0;
#pragma unroll
      for (int j = 0; j < Np; ++j) {
        const double dr = ops[L::Dr + i * Np + j], ds = ops[L::Ds + i * Np + j];
        ur += dr * ue[j];
        us += ds * ue[j];
        vr += dr * ve[j];
        vs += ds * ve[j];
      }
      double di = (rx * ur + sx * us) + (ry * vr + sy * vs);
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < Nfp; ++k) s += ops[L::LIFT + i * 3 * Nfp + f * Nfp + k] * fl[f][k];
        di += s;
      }
      d[i] = di;
    }
    if constexpr (MASS) mass_rows<N>(ops, 1.0 / (rx * sy - ry * sx), d);
#pragma unroll
    for (int i = 0; i < Np; ++i) buf[t * P + i] = a.scale * d[i];
  }
  store_rows<N>(buf, a.out, e0, n);
}

// One element per lane; only elements with Dirichlet faces add anything.
// Face integrals from the face-node values: with h = (|F| / 2) M1D g (the
// face mass on [-1, 1] times the half face length), (g, l_i)_F = h at the
// face nodes, and (g, d_n l_i)_F = sum_k h_k (d_n l_i)(x_k), d_n l_i at a
// face node read off the derivative matrices (exact: both traces are
// polynomials the face nodes represent).
template <int N>
__global__ __launch_bounds__(256) void k_dirichlet_rhs(DirichletArgs a) {
  using T = Tri<N>;
  using L = OpsLayout<N>;
  constexpr int Np = T::Np, Nfp = T::Nfp;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= a.K) return;
  const Conn c = a.conn[e];
  if (conn_bc(c.info, 0) != 1 && conn_bc(c.info, 1) != 1 && conn_bc(c.info, 2) != 1) return;
  const double* __restrict__ ops = a.ops;
  const double rx = a.geo[4 * (size_t)e], sx = a.geo[4 * (size_t)e + 1];
  const double ry = a.geo[4 * (size_t)e + 2], sy = a.geo[4 * (size_t)e + 3];
  const double J = 1.0 / (rx * sy - ry * sx);
  const double kap = a.kap ? a.kap[e] : 1.0;
  double* b = a.b + (size_t)e * Np;
  for (int f = 0; f < 3; ++f) {
    if (conn_bc(c.info, f) != 1) continue;
    double ax, ay;
    face_vec(f, rx, sx, ry, sy, ax, ay);
    const double fs = sqrt(ax * ax + ay * ay);          // |F| / |E|
    const double nx = ax / fs, ny = ay / fs;
    const double half_len = fs * J;                     // |F| / 2 (|E| = 2 J)
    const double tau = a.ctau * kap * fs;
    double gk[Nfp], h[Nfp];
#pragma unroll
    for (int k = 0; k < Nfp; ++k) gk[k] = a.g[(size_t)e * Np + T::fm(f, k)];
#pragma unroll
    for (int k = 0; k < Nfp; ++k) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < Nfp; ++m) s += ops[L::M1D + k * Nfp + m] * gk[m];
      h[k] = half_len * s;
    }
    // -kappa (g, d_n l_i)_F for every row i
    for (int i = 0; i < Np; ++i) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < Nfp; ++k) {
        const int q = T::fm(f, k);
        const double dx = rx * ops[L::Dr + q * Np + i] + sx * ops[L::Ds + q * Np + i];
        const double dy = ry * ops[L::Dr + q * Np + i] + sy * ops[L::Ds + q * Np + i];
        s += h[k] * (nx * dx + ny * dy);
      }
      b[i] -= kap * s;
    }
    // 2 tau_F (g, l_i)_F on the face nodes
#pragma unroll
    for (int k = 0; k < Nfp; ++k) b[T::fm(f, k)] += 2.0 * tau * h[k];
  }
}

template <int N>
__global__ __launch_bounds__(kElems<N>()) void k_advect(AdvectArgs a) {
  using T = Tri<N>;
  using L = OpsLayout<N>;
  constexpr int Np = T::Np, Nfp = T::Nfp, B = kElems<N>(), P = kPitchGD<N>();
  __shared__ double buf[B * P];
  const int e0 = blockIdx.x * B;
  const int n = min(B, a.K - e0);
  const double* __restrict__ ops = a.ops;
  const double* __restrict__ u = a.u;
  const double* __restrict__ v = a.v;
  double ue[Np], ve[Np];
  load_rows<N>(u, buf, e0, n, ue);
  load_rows<N>(v, buf, e0, n, ve);
  const int t = threadIdx.x, e = e0 + t;
  double nu[Np], nv[Np];
  if (t < n) {
    const double rx = a.geo[4 * (size_t)e], sx = a.geo[4 * (size_t)e + 1];
    const double ry = a.geo[4 * (size_t)e + 2], sy = a.geo[4 * (size_t)e + 3];
    // div (u_c u) from the nodal products
    for (int i = 0; i < Np; ++i) {
      double uur = 0.0, uus = 0.0, uvr = 0.0, uvs = 0.0, vvr = 0.0, vvs = 0.0;
#pragma unroll
      for (int j = 0; j < Np; ++j) {
        const double dr = ops[L::Dr + i * Np + j], ds = ops[L::Ds + i * Np + j];
        const double uu = ue[j] * ue[j], uv = ue[j] * ve[j], vv = ve[j] * ve[j];
        uur += dr * uu;
        uus += ds * uu;
        uvr += dr * uv;
        uvs += ds * uv;
        vvr += dr * vv;
        vvs += ds * vv;
      }
      nu[i] = (rx * uur + sx * uus) + (ry * uvr + sy * uvs);
      nv[i] = (rx * uvr + sx * uvs) + (ry * vvr + sy * vvs);
    }
    const Conn c = a.conn[e];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const int bc = conn_bc(c.info, f);
      const int fp = conn_fp(c.info, f), nb = c.nb[f];
      double ax, ay;
      face_vec(f, rx, sx, ry, sy, ax, ay);
      const double fs = sqrt(ax * ax + ay * ay);
      const double nx = ax / fs, ny = ay / fs;
      double fu[Nfp], fv[Nfp];
#pragma unroll
      for (int k = 0; k < Nfp; ++k) {
        const int m = T::fm(f, k);
        const double um = ue[m], vm = ve[m];
        double up = um, vp = vm;                       // Neumann: u+ = u-
        if (bc == 0) {
          const size_t ip = (size_t)nb * Np + T::fm(fp, N - k);
          up = u[ip];
          vp = v[ip];
        } else if (bc == 1) {
          const size_t im = (size_t)e * Np + m;
          up = a.gu ? a.gu[im] : 0.0;
          vp = a.gv ? a.gv[im] : 0.0;
        }
        const double unm = nx * um + ny * vm, unp = nx * up + ny * vp;
        const double lam = 2.0 * fmax(fabs(unm), fabs(unp));
        fu[k] = fs * (0.5 * (um * unm + up * unp) + 0.5 * lam * (um - up) - um * unm);
        fv[k] = fs * (0.5 * (vm * unm + vp * unp) + 0.5 * lam * (vm - vp) - vm * unm);
      }
      for (int i = 0; i < Np; ++i) {
        double su = 0.0, sv = 0.0;
#pragma unroll
        for (int k = 0; k < Nfp; ++k) {
          const double l = ops[L::LIFT + i * 3 * Nfp + f * Nfp + k];
          su += l * fu[k];
          sv += l * fv[k];
        }
        nu[i] += su;
        nv[i] += sv;
      }
    }
    for (int i = 0; i < Np; ++i) {
      nu[i] *= a.a_adv;
      nv[i] *= a.a_adv;
    }
    if (a.base_u)
      for (int i = 0; i < Np; ++i) {
        nu[i] += a.a_base * a.base_u[(size_t)e * Np + i];
        nv[i] += a.a_base * a.base_v[(size_t)e * Np + i];
      }
#pragma unroll
    for (int i = 0; i < Np; ++i) buf[t * P + i] = nu[i];
  }
  store_rows<N>(buf, a.out_u, e0, n);
  if (t < n)
#pragma unroll
    for (int i = 0; i < Np; ++i) buf[t * P + i] = nv[i];
  store_rows<N>(buf, a.out_v, e0, n);
}

__global__ __launch_bounds__(256) void k_axpby(double a, const double* __restrict__ x, double b,
                                               const double* __restrict__ y, double* __restrict__ z, size_t n) {
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) z[i] = a * x[i] + b * y[i];
}

// one block: work[0] = sum b (fixed order)
__global__ __launch_bounds__(1024) void k_sum(const double* __restrict__ b, size_t n, double* __restrict__ work) {
  __shared__ double red[16];
  double s = 0.0;
  for (size_t i = threadIdx.x; i < n; i += 1024) s += b[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w];
    work[0] = t;
  }
}

// b_i -= (work[0] / area) J_e sum_j M_ij
template <int N>
__global__ __launch_bounds__(256) void k_sub_mean(double* __restrict__ b, double area, const double* __restrict__ geo,
                                                  const double* __restrict__ ops, int K,
                                                  const double* __restrict__ work) {
  using L = OpsLayout<N>;
  constexpr int Np = Tri<N>::Np;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= K) return;
  const double c = work[0] / area;
  const double J = 1.0 / (geo[4 * (size_t)e] * geo[4 * (size_t)e + 3] - geo[4 * (size_t)e + 2] * geo[4 * (size_t)e + 1]);
  for (int i = 0; i < Np; ++i) {
    double s = 0.0;
    for (int j = 0; j < Np; ++j) s += ops[L::M + i * Np + j];
    b[(size_t)e * Np + i] -= c * J * s;
  }
}


template <int N>
int blocks(int K) { return (K + kElems<N>() - 1) / kElems<N>(); }

}  // namespace

hipError_t dirichlet_rhs(int N, const DirichletArgs& a, hipStream_t s) {
  if (a.K == 0) return hipSuccess;
  const dim3 g((a.K + 255) / 256);
  switch (N) {
#define IPDG_R(n) \
  case n: hipLaunchKernelGGL(k_dirichlet_rhs<n>, g, dim3(256), 0, s, a); break;
    IPDG_R(1) IPDG_R(2) IPDG_R(3) IPDG_R(4) IPDG_R(5) IPDG_R(6) IPDG_R(7) IPDG_R(8)
#undef IPDG_R
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t advect_apply(int N, const AdvectArgs& a, hipStream_t s) {
  if (a.K == 0) return hipSuccess;
  switch (N) {
#define IPDG_A(n) \
  case n: hipLaunchKernelGGL(k_advect<n>, dim3(blocks<n>(a.K)), dim3(kElems<n>()), 0, s, a); break;
    IPDG_A(1) IPDG_A(2) IPDG_A(3) IPDG_A(4) IPDG_A(5) IPDG_A(6) IPDG_A(7) IPDG_A(8)
#undef IPDG_A
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t axpby(double a, const double* x, double b, const double* y, double* z, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)g), dim3(256), 0, s, a, x, b, y, z, n);
  return hipGetLastError();
}

hipError_t remove_mean(int N, double* b, double area, const double* geo, const double* ops, int K, double* work,
                       hipStream_t s) {
  if (K == 0) return hipSuccess;
  const size_t n = (size_t)K * ((N + 1) * (N + 2) / 2);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, s, b, n, work);
  const dim3 g((K + 255) / 256);
  switch (N) {
#define IPDG_M(nn) \
  case nn: hipLaunchKernelGGL(k_sub_mean<nn>, g, dim3(256), 0, s, b, area, geo, ops, K, work); break;
    IPDG_M(1) IPDG_M(2) IPDG_M(3) IPDG_M(4) IPDG_M(5) IPDG_M(6) IPDG_M(7) IPDG_M(8)
#undef IPDG_M
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t grad_apply(int N, const GradArgs& a, hipStream_t s) {
  if (a.K == 0) return hipSuccess;
  switch (N) {
#define IPDG_G(n) \
  case n:                                                                                    \
    if (a.mass) hipLaunchKernelGGL((k_grad<n, true>), dim3(blocks<n>(a.K)), dim3(kElems<n>()), 0, s, a);  \
    else hipLaunchKernelGGL((k_grad<n, false>), dim3(blocks<n>(a.K)), dim3(kElems<n>()), 0, s, a);       \
    break;
    IPDG_G(1) IPDG_G(2) IPDG_G(3) IPDG_G(4) IPDG_G(5) IPDG_G(6) IPDG_G(7) IPDG_G(8)
#undef IPDG_G
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t div_apply(int N, const DivArgs& a, hipStream_t s) {
  if (a.K == 0) return hipSuccess;
  switch (N) {
#define IPDG_D(n) \
  case n:                                                                                    \
    if (a.mass) hipLaunchKernelGGL((k_div<n, true>), dim3(blocks<n>(a.K)), dim3(kElems<n>()), 0, s, a);   \
    else hipLaunchKernelGGL((k_div<n, false>), dim3(blocks<n>(a.K)), dim3(kElems<n>()), 0, s, a);        \
    break;
    IPDG_D(1) IPDG_D(2) IPDG_D(3) IPDG_D(4) IPDG_D(5) IPDG_D(6) IPDG_D(7) IPDG_D(8)
#undef IPDG_D
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ipdg
