// Host side of the subcycling advection (Sec. 2.3, Eq. SS_3; Sec. 5.3,
// Eq. KSS_3): operator tables in the matrix-core layout of SubDims, and the
// low-storage Runge-Kutta subcycle.
//
// Time stepping: the five-stage fourth-order 2N-storage scheme of Carpenter
// and Kennedy (the method the paper cites for its subcycles):
//   res = a_k res + dt R(tau + c_k dt, U~),  U~ = U~ + b_k res,  k = 0..4,
// with R = -N~(Ubar(tau), U~).  Each stage is one launch of the operator
// kernel that also performs the two register updates; the updated field goes
// to the other buffer of a pair, since the same launch still reads the old
// field's traces across faces.
#include <map>
#include <stdexcept>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "refelem.hpp"
#include "subcycle.hpp"

namespace ipdg {
namespace {

// Carpenter & Kennedy (1994), five-stage fourth-order low-storage scheme.
constexpr double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                            -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
constexpr double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                            1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                            2277821191437.0 / 14882151754819.0};
constexpr double kRkC[5] = {0.0, 1432997174477.0 / 9575080441755.0, 2526269341429.0 / 6820363962896.0,
                            2006345519317.0 / 3224310063776.0, 2802321613138.0 / 2924317926251.0};

std::vector<double> pack(int N) {
  const CubOps& C = cub_ops(N);
  const SubDims D = sub_dims(N);
  if (C.Np != D.Np || C.Nc != D.Nc || C.Nfc != D.Nfc) throw std::runtime_error("cubature sizes disagree");
  std::vector<double> t(D.total, 0.0);
  for (int tc = 0; tc < D.TC; ++tc)
    for (int kb = 0; kb < D.KB; ++kb)
      for (int l = 0; l < 64; ++l) {
        const int i = 16 * tc + l % 16, j = 4 * kb + l / 16;
        if (i < D.Nc && j < D.Np) t[D.oI + (tc * D.KB + kb) * 64 + l] = C.I[i * D.Np + j];
      }
  for (int R = 0; R < D.RB; ++R)
    for (int tc = 0; tc < D.TC; ++tc)
      for (int k = 0; k < 4; ++k)
        for (int l = 0; l < 64; ++l) {
          const int n = 16 * R + l % 16, i = 16 * tc + 4 * k + l / 16;
          if (n < D.Np && i < D.Nc) {
            const int o = ((R * D.TC + tc) * 4 + k) * 64 + l;
            t[D.oPr + o] = C.Pr[n * D.Nc + i];
            t[D.oPs + o] = C.Ps[n * D.Nc + i];
          }
        }
  for (int f = 0; f < 3; ++f) {
    for (int kb = 0; kb < D.KF; ++kb)
      for (int l = 0; l < 64; ++l) {
        const int j = l % 16, k = 4 * kb + l / 16;
        if (j < D.Nfc && k < D.Nfp) t[D.oIf + (f * D.KF + kb) * 64 + l] = C.If[f][j * D.Nfp + k];
      }
    for (int R = 0; R < D.RB; ++R)
      for (int k = 0; k < D.KT; ++k)
        for (int l = 0; l < 64; ++l) {
          const int n = 16 * R + l % 16, j = 4 * k + l / 16;
          if (n < D.Np && j < D.Nfc) t[D.oLc + ((f * D.RB + R) * D.KT + k) * 64 + l] = C.Lc[f][n * D.Nfc + j];
        }
  }
  return t;
}

std::mutex g_mu;
std::map<std::pair<int, int>, void*> g_tabs;   // (device, N) -> table, kept until exit

SubArgs with_mesh(ipdg_mesh_s* m, const SubArgs& in) {
  SubArgs a = in;
  a.geo = m->geo64.as<double>();
  a.conn = m->conn.as<Conn>();
  a.tab = device_sub_ops(m->host.N);
  a.K = m->host.K;
  return a;
}

}  // namespace

const double* device_sub_ops(int N) {
  int dev = 0;
  IPDG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, N);
  auto it = g_tabs.find(key);
  if (it != g_tabs.end()) return static_cast<const double*>(it->second);
  const std::vector<double> t = pack(N);
  void* p = nullptr;
  IPDG_HIP(hipMalloc(&p, t.size() * sizeof(double)));
  IPDG_HIP(hipMemcpy(p, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
  g_tabs[key] = p;
  return static_cast<const double*>(p);
}

void subcycle_rhs(ipdg_mesh_s* m, const SubArgs& in, int parts, double* nu, double* nv, hipStream_t s) {
  SubArgs a = with_mesh(m, in);
  a.out_u = nu;
  a.out_v = nv;
  IPDG_HIP(subcycle_launch(m->host.N, parts, false, a, s));
}

void subcycle_advect(ipdg_mesh_s* m, const SubArgs& in, double T, int Ns, double* u, double* v, hipStream_t s) {
  const size_t n = (size_t)m->host.K * m->Np;
  m->sub_work.ensure(4 * n * sizeof(double));
  double* w = m->sub_work.as<double>();
  SubArgs a = with_mesh(m, in);
  a.res_u = w;
  a.res_v = w + n;
  double* cur_u = u;
  double* cur_v = v;
  double* nxt_u = w + 2 * n;
  double* nxt_v = w + 3 * n;
  const double dt = T / Ns;
  a.dt = dt;
  for (int step = 0; step < Ns; ++step)
    for (int k = 0; k < 5; ++k) {
      a.tau = (step + kRkC[k]) * dt;
      a.rk_a = kRkA[k];
      a.rk_b = kRkB[k];
      a.u = cur_u;
      a.v = cur_v;
      a.new_u = nxt_u;
      a.new_v = nxt_v;
      IPDG_HIP(subcycle_launch(m->host.N, 3, true, a, s));
      std::swap(cur_u, nxt_u);
      std::swap(cur_v, nxt_v);
    }
  if (cur_u != u) {
    IPDG_HIP(hipMemcpyAsync(u, cur_u, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    IPDG_HIP(hipMemcpyAsync(v, cur_v, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
}

}  // namespace ipdg
