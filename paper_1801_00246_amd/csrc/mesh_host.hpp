// Host-side mesh processing: validation, face matching and per-element
// metric terms (Sec. 2.1 partition into triangles; Sec. 5.2, Eq. operators1
// and operators2, affine map to the bi-unit triangle).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "device_common.hpp"

namespace ipdg {

struct HostMesh {
  int N = 0, K = 0, Nv = 0;
  std::vector<double> VX, VY;
  std::vector<int32_t> EToV;     // K x 3
  std::vector<int8_t> EToB;      // K x 3
  std::vector<int32_t> EToE;     // K x 3, -1 on boundary faces
  std::vector<int8_t> EToF;      // K x 3, -1 on boundary faces
  std::vector<double> geo;       // K x 4: r_x, s_x, r_y, s_y
  std::vector<double> J;         // K
  std::vector<Conn> conn;        // K
};

// Returns an empty string on success, else the reason (mesh errors).
std::string build_host_mesh(int N, int Nv, const double* VX, const double* VY, int K,
                            const int32_t* EToV, const int8_t* EToB, HostMesh& out);

// Physical node coordinates (K x Np each).
void host_node_coords(const HostMesh& m, std::vector<double>& x, std::vector<double>& y);

}  // namespace ipdg
