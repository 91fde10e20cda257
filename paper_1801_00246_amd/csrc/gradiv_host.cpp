// Operator table of the matrix-core gradient and divergence (layout GdDims in
// gradiv.hpp): D_r, D_s, the three face blocks of LIFT and M of the degree,
// in the lane order of the A operands of v_mfma_f64_16x16x4f64.
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "gradiv.hpp"
#include "handle.hpp"
#include "refelem.hpp"

namespace ipdg {
namespace {

std::vector<double> pack(int N) {
  const RefOps& R = ref_ops(N);
  const GdDims D = gd_dims(N);
  const int Np = D.Np, Nfp = D.Nfp;
  std::vector<double> t(D.total, 0.0);
  for (int rb = 0; rb < D.RB; ++rb)
    for (int kb = 0; kb < D.KB; ++kb)
      for (int l = 0; l < 64; ++l) {
        const int i = 16 * rb + l % 16, j = 4 * kb + l / 16;
        if (i < Np && j < Np) {
          t[D.oDr + (rb * D.KB + kb) * 64 + l] = R.Dr[i * Np + j];
          t[D.oDs + (rb * D.KB + kb) * 64 + l] = R.Ds[i * Np + j];
        }
      }
  for (int f = 0; f < 3; ++f)
    for (int rb = 0; rb < D.RB; ++rb)
      for (int kb = 0; kb < D.KF; ++kb)
        for (int l = 0; l < 64; ++l) {
          const int i = 16 * rb + l % 16, k = 4 * kb + l / 16;
          if (i < Np && k < Nfp) t[D.oL + ((f * D.RB + rb) * D.KF + kb) * 64 + l] = R.LIFT[i * 3 * Nfp + f * Nfp + k];
        }
  for (int rb = 0; rb < D.RB; ++rb)
    for (int r2 = 0; r2 < D.RB; ++r2)
      for (int q = 0; q < 4; ++q)
        for (int l = 0; l < 64; ++l) {
          const int i = 16 * rb + l % 16, j = 16 * r2 + 4 * q + l / 16;
          if (i < Np && j < Np) t[D.oM + ((rb * D.RB + r2) * 4 + q) * 64 + l] = R.M[i * Np + j];
        }
  return t;
}

std::mutex g_mu;
std::map<std::pair<int, int>, void*> g_tabs;   // (device, N) -> table, kept until exit

}  // namespace

const double* device_gd_tab(int N) {
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

}  // namespace ipdg
