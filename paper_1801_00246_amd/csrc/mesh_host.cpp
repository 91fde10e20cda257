#include "mesh_host.hpp"

#include <cmath>
#include <unordered_map>

#include "refelem.hpp"

namespace ipdg {

std::string build_host_mesh(int N, int Nv, const double* VX, const double* VY, int K,
                            const int32_t* EToV, const int8_t* EToB, HostMesh& m) {
  if (N < 1 || N > kMaxN) return "degree outside 1..8";
  if (K < 0 || Nv < 0) return "negative size";
  if (K > 0 && (!VX || !VY || !EToV || !EToB)) return "null mesh array";
  m = HostMesh();
  m.N = N;
  m.K = K;
  m.Nv = Nv;
  m.VX.assign(VX, VX + Nv);
  m.VY.assign(VY, VY + Nv);
  m.EToV.assign(EToV, EToV + 3 * (size_t)K);
  m.EToB.assign(EToB, EToB + 3 * (size_t)K);
  m.geo.resize(4 * (size_t)K);
  m.J.resize(K);
  for (int e = 0; e < K; ++e) {
    int v[3];
    for (int i = 0; i < 3; ++i) {
      v[i] = m.EToV[3 * e + i];
      if (v[i] < 0 || v[i] >= Nv) return "vertex id out of range in element " + std::to_string(e);
    }
    // x = -(r+s)/2 x0 + (1+r)/2 x1 + (1+s)/2 x2
    const double xr = 0.5 * (VX[v[1]] - VX[v[0]]), xs = 0.5 * (VX[v[2]] - VX[v[0]]);
    const double yr = 0.5 * (VY[v[1]] - VY[v[0]]), ys = 0.5 * (VY[v[2]] - VY[v[0]]);
    const double J = xr * ys - xs * yr;
    if (!(J > 0.0)) return "non-positive Jacobian in element " + std::to_string(e);
    m.J[e] = J;
    m.geo[4 * e + 0] = ys / J;    // r_x
    m.geo[4 * e + 1] = -yr / J;   // s_x
    m.geo[4 * e + 2] = -xs / J;   // r_y
    m.geo[4 * e + 3] = xr / J;    // s_y
  }
  // face matching on the sorted vertex pair
  m.EToE.assign(3 * (size_t)K, -1);
  m.EToF.assign(3 * (size_t)K, -1);
  std::unordered_map<uint64_t, int> seen;
  seen.reserve(3 * (size_t)K);
  for (int e = 0; e < K; ++e)
    for (int f = 0; f < 3; ++f) {
      uint32_t a = m.EToV[3 * e + f], b = m.EToV[3 * e + (f + 1) % 3];
      if (a > b) std::swap(a, b);
      const uint64_t key = (uint64_t(a) << 32) | b;
      auto it = seen.find(key);
      if (it == seen.end()) {
        seen.emplace(key, 3 * e + f);
        continue;
      }
      const int g = it->second;
      if (g < 0) return "face shared by more than two elements";
      const int e2 = g / 3, f2 = g % 3;
      m.EToE[3 * e + f] = e2;
      m.EToF[3 * e + f] = int8_t(f2);
      m.EToE[3 * e2 + f2] = e;
      m.EToF[3 * e2 + f2] = int8_t(f);
      it->second = -1;
    }
  m.conn.resize(K);
  for (int e = 0; e < K; ++e) {
    Conn c{};
    int info = 0;
    for (int f = 0; f < 3; ++f) {
      const int bc = m.EToB[3 * e + f];
      const int nb = m.EToE[3 * e + f];
      if (bc < 0 || bc > 2) return "unknown boundary flag";
      if (nb >= 0 && bc != 0) return "matched face flagged as boundary";
      if (nb < 0 && bc == 0) return "unmatched face flagged interior";
      c.nb[f] = nb >= 0 ? nb : e;
      info |= (nb >= 0 ? int(m.EToF[3 * e + f]) : 0) << (2 * f);
      info |= bc << (8 + 2 * f);
    }
    c.info = info;
    m.conn[e] = c;
  }
  return "";
}

void host_node_coords(const HostMesh& m, std::vector<double>& x, std::vector<double>& y) {
  const RefOps& R = ref_ops(m.N);
  x.resize((size_t)m.K * R.Np);
  y.resize((size_t)m.K * R.Np);
  for (int e = 0; e < m.K; ++e) {
    const int* v = &m.EToV[3 * e];
    for (int n = 0; n < R.Np; ++n) {
      const double r = R.r[n], s = R.s[n];
      x[(size_t)e * R.Np + n] = 0.5 * (-(r + s) * m.VX[v[0]] + (1 + r) * m.VX[v[1]] + (1 + s) * m.VX[v[2]]);
      y[(size_t)e * R.Np + n] = 0.5 * (-(r + s) * m.VY[v[0]] + (1 + r) * m.VY[v[1]] + (1 + s) * m.VY[v[2]]);
    }
  }
}

}  // namespace ipdg
