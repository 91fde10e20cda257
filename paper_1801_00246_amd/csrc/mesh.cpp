// Mesh handle: upload of metric terms and connectivity, device operator
// tables.
#include <map>
#include <mutex>
#include <tuple>

#include "handle.hpp"
#include "ops_table.hpp"
#include "refelem.hpp"
#include "solver.hpp"

namespace ipdg {

void DevBuf::alloc(size_t bytes) {
  if (bytes == 0) return;
  hipError_t e = hipMalloc(&p_, bytes);
  if (e != hipSuccess) {
    p_ = nullptr;
    throw Error(e == hipErrorOutOfMemory ? IPDG_ENOMEM : IPDG_EHIP,
                std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  n_ = bytes;
}

void DevBuf::release() {
  if (p_) (void)hipFree(p_);
  p_ = nullptr;
  n_ = 0;
}

namespace {

std::mutex g_mu;
std::map<std::tuple<int, int, int>, void*> g_ops;      // (device, N, fp32)
std::map<std::tuple<int, int, int, int>, void*> g_interp;  // (device, Nc, Nf, fp32)

void* upload(const std::vector<double>& v, bool fp32) {
  void* p = nullptr;
  const size_t n = v.size();
  if (fp32) {
    std::vector<float> f(v.begin(), v.end());
    IPDG_HIP(hipMalloc(&p, n * sizeof(float)));
    IPDG_HIP(hipMemcpy(p, f.data(), n * sizeof(float), hipMemcpyHostToDevice));
  } else {
    IPDG_HIP(hipMalloc(&p, n * sizeof(double)));
    IPDG_HIP(hipMemcpy(p, v.data(), n * sizeof(double), hipMemcpyHostToDevice));
  }
  return p;
}

}  // namespace

const void* device_ops(int N, Kind kind) {
  int dev = 0;
  IPDG_HIP(hipGetDevice(&dev));
  const int fp32 = kind != Kind::F64;
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_tuple(dev, N, fp32);
  auto it = g_ops.find(key);
  if (it != g_ops.end()) return it->second;
  void* p = upload(build_ops_table(N), fp32);
  g_ops[key] = p;
  return p;
}

const void* device_ops_resident(int N, Kind kind) {
  int dev = 0;
  IPDG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ops.find(std::make_tuple(dev, N, int(kind != Kind::F64)));
  return it == g_ops.end() ? nullptr : it->second;
}

const void* device_interp(int Nc, int Nf, bool fp32) {
  int dev = 0;
  IPDG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_tuple(dev, Nc, Nf, int(fp32));
  auto it = g_interp.find(key);
  if (it != g_interp.end()) return it->second;
  void* p = upload(interp_matrix(Nc, Nf), fp32);
  g_interp[key] = p;
  return p;
}

ElemArgs elem_args(const ipdg_mesh_s* m, int N, Kind kind, double lambda, double ctau) {
  ElemArgs a;
  a.geo = geo_for(m, kind);
  a.conn = m->conn.as<Conn>();
  a.kap = kap_for(m, kind);
  a.ops = device_ops(N, kind);
  a.lambda = lambda;
  a.ctau = ctau;
  a.K = m->host.K;
  return a;
}

}  // namespace ipdg

ipdg_mesh_s::~ipdg_mesh_s() = default;
