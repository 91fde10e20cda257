// Preconditioned conjugate-gradient solvers (Sec. 3) on the device.
//
// Outer iteration (one fixed launch sequence, all scalars device-resident):
//   Ap = A p, (p, Ap)              element kernel with fused dot
//   alpha = (r, z) / (p, Ap)        finalize
//   x += alpha p, r -= alpha Ap     fused update (+ Jacobi z = D^-1 r, dots)
//   z = B r                         block inverse mass / V-cycle
//   beta                            finalize: textbook (r+, z+)/(r, z) or
//                                   flexible -(z+, Ap)/(p, Ap) (Notay)
//   p = z + beta p
// The host reads the scalars every check_every iterations.  A stop is
// accepted only on the true FP64 residual b - A x; otherwise the recurrence
// restarts from it (residual replacement).  In mixed precision the
// preconditioner runs in FP32 while the outer operator, x, r, p, the dots and
// the true residual stay in FP64; optionally (reliable_drop > 0) the residual
// is also replaced whenever ||r|| fell by that factor since the last
// replacement.  With the FP32 outer operator (IPDG_PREC_FP32_OPERATOR) A p is
// applied in FP32 too, and the residual is always replaced (with the
// direction restarted) after every fall by reliable_drop (default 1e-3).
//
// p-multigrid (Sec. 3, the degree-coarsening part of pMG-AMG): levels of
// degree N_0 > N_1 > ... rediscretise the operator with penalty constant
// c_tau ((N_l+1)/(N_0+1))^2; restriction P^T and prolongation P (nodal
// interpolation); Chebyshev smoothing of D^-1 A over [lo rho, hi rho] before
// and after the coarse correction; the coarsest level is solved by
// Jacobi-PCG to a relative residual or an iteration cap.
#include "solver.hpp"

#include <algorithm>
#include <atomic>
#include <mutex>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <cstdlib>
#include <random>

#include "blas.hpp"
#include "refelem.hpp"

namespace ipdg {
namespace {

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t) {
  return std::chrono::duration<double, std::milli>(clk::now() - t).count();
}

struct Level {
  int N = 0, Np = 0;
  size_t n = 0;
  double ctau = 0, rho = 0;
  bool fp32 = false;
  Kind kind = Kind::F64;
  DevBuf dinv64, dinv32;
  DevBuf f, z, r, d, t;            // V-cycle work (level precision)
  DevBuf cr, cr2, cz, cp, cp2, cs2, cAp, cw2;   // coarsest level: Jacobi-PCG work
                                               // (r, w, s double-buffered)
  const void* P = nullptr;         // interpolation from the next level
  const void* dinv() const { return fp32 ? dinv32.get() : dinv64.get(); }
};

struct Work : SolverWork {
  // configuration the setup was built for
  double lambda = NAN, ctau = NAN;
  int pc = -1, prec = -1, cheb_degree = 0, coarse_max = 0, nlev = 0, rho_steps = 0;
  double cheb_lo = 0, cheb_hi = 0, coarse_tol = 0;
  int degrees[IPDG_MAX_LEVELS] = {0};
  double rho_in[IPDG_MAX_LEVELS] = {0};
  bool has_kappa = false;
  unsigned kappa_version = 0;
  double setup_ms = 0;

  size_t n = 0;
  DevBuf r, p, Ap, z, t64, xw, partials, cpartials, scal, cscal, dinv64, dinv32;
  DevBuf p32, Ap32;                // FP32 outer operator: p and A p in FP32
  DevBuf cbar;                     // persistent coarse solve: 2 barrier counters + 3 status ints
  int coarse_grid = 0;             // resident grid of the persistent coarse solve (0: not used)
  std::vector<Level> lv;
  CGScal* host_scal = nullptr;     // pinned
  hipStream_t gs = nullptr;        // internal stream of the solver (default priority)
  hipGraphExec_t graph = nullptr;  // check_every captured outer iterations
  int graph_iters = 0;
  // one outer iteration split at its coarsest-level solve (batched coarse
  // mode), and that solve's right-hand side and solution buffers
  hipGraphExec_t graph_pre = nullptr, graph_post = nullptr;
  const void* split_f = nullptr;
  void* split_x = nullptr;
  unsigned long long setup_id = 0;   // changes with every new setup (never reused)

  void drop_main() {
    if (graph) (void)hipGraphExecDestroy(graph);
    graph = nullptr;
    graph_iters = 0;
  }
  void drop_split() {
    if (graph_pre) (void)hipGraphExecDestroy(graph_pre);
    if (graph_post) (void)hipGraphExecDestroy(graph_post);
    graph_pre = graph_post = nullptr;
    split_f = nullptr;
    split_x = nullptr;
  }
  void drop_graph() {
    drop_main();
    drop_split();
  }
  ~Work() override {
    drop_graph();
    if (gs) (void)hipStreamDestroy(gs);
    if (host_scal) (void)hipHostFree(host_scal);
  }
};

size_t off_done() { return offsetof(CGScal, done); }

unsigned long long next_setup_id() {
  static std::atomic<unsigned long long> n{0};
  return ++n;
}
const int* done_ptr(const DevBuf& sc) {
  return reinterpret_cast<const int*>(static_cast<const char*>(sc.get()) + off_done());
}

// Largest eigenvalue of a symmetric tridiagonal matrix (Jacobi rotations on
// the dense copy; k <= a few dozen).
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
  const int k = int(a.size());
  std::vector<double> A(k * k, 0.0);
  for (int i = 0; i < k; ++i) {
    A[i * k + i] = a[i];
    if (i + 1 < k) A[i * k + i + 1] = A[(i + 1) * k + i] = b[i];
  }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) off += A[p * k + q] * A[p * k + q];
    if (off < 1e-30) break;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = A[p * k + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double th = (A[q * k + q] - A[p * k + p]) / (2 * apq);
        const double t = (th >= 0 ? 1 : -1) / (std::fabs(th) + std::sqrt(th * th + 1));
        const double c = 1 / std::sqrt(t * t + 1), s = t * c;
        for (int i = 0; i < k; ++i) {
          const double aip = A[i * k + p], aiq = A[i * k + q];
          A[i * k + p] = c * aip - s * aiq;
          A[i * k + q] = s * aip + c * aiq;
        }
        for (int i = 0; i < k; ++i) {
          const double api = A[p * k + i], aqi = A[q * k + i];
          A[p * k + i] = c * api - s * aqi;
          A[q * k + i] = s * api + c * aqi;
        }
      }
  }
  double mx = -INFINITY;
  for (int i = 0; i < k; ++i) mx = std::max(mx, A[i * k + i]);
  return mx;
}

class Solver {
 public:
  // persistent: the coarsest pMG level may run as one persistent launch
  // (off when several solves share the device at once, since their grids
  // would not all be resident together)
  Solver(ipdg_mesh_s* m, double lambda, double tau, const ipdg_solve_opts& o, hipStream_t s,
         bool persistent = true)
      : m_(m), o_(o), s_(s), persistent_(persistent) {
    N_ = m->host.N;
    if (o_.pc == IPDG_PC_PMG && o_.n_levels == 0) {
      // automatic levels: halve the degree down to 1 (7 -> 3 -> 1, 8 -> 4 -> 2 -> 1)
      int L = 0;
      for (int d = N_; L < IPDG_MAX_LEVELS; d /= 2) {
        o_.degrees[L++] = d;
        if (d == 1) break;
      }
      o_.n_levels = L;
    }
    K_ = m->host.K;
    n_ = (size_t)K_ * m->Np;
    lambda_ = lambda;
    ctau_ = ctau_of(N_, tau);
    mixed_ = o.prec == IPDG_PREC_MIXED || o.prec == IPDG_PREC_FP32_OPERATOR;
    op32_ = o.prec == IPDG_PREC_FP32_OPERATOR;
    // the FP32 outer operator's recurrence drifts from the true residual:
    // reliable updates are always on (default: after every 1e3 fall)
    drop_ = o.reliable_drop > 0.0 ? o.reliable_drop : (op32_ ? 1e-3 : 0.0);
    flexible_ = o.flexible < 0 ? (o.pc == IPDG_PC_PMG || mixed_) : o.flexible != 0;
    validate();
    if (elem_grid(K_) > kMaxPartials) throw Error(IPDG_EUNSUPPORTED, "mesh too large for one launch");
    if (!m->work) m->work = std::make_unique<Work>();
    w_ = static_cast<Work*>(m->work.get());
    if (!w_->gs) IPDG_HIP(hipStreamCreateWithFlags(&w_->gs, hipStreamNonBlocking));
    user_ = s;
    // the caller's queued work (b, x producers) completes before the solve
    IPDG_HIP(hipStreamSynchronize(user_));
    s_ = w_->gs;
    use_graph_ = std::getenv("IPDG_NO_GRAPH") == nullptr;
    setup();
  }

  // z = B r for one FP64 vector (ipdg_precond_apply)
  void apply_precond(const double* r, double* z, ipdg_solve_info* info) {
    CGScal sc{};
    IPDG_HIP(set_scal(w_->scal.as<CGScal>(), sc, s_));
    IPDG_HIP(hipMemcpyAsync(w_->r.get(), r, n_ * sizeof(double), hipMemcpyDeviceToDevice, s_));
    precond();
    if (mixed_) IPDG_HIP(convert(false, z, w_->z.get(), n_, nullptr, s_));
    else IPDG_HIP(hipMemcpyAsync(z, w_->z.get(), n_ * sizeof(double), hipMemcpyDeviceToDevice, s_));
    IPDG_HIP(hipStreamSynchronize(s_));
    fill_info(info, 0, 0.0, 0, 0.0);
  }

  // ---- phases of one solve (shared by solve() and the batched solver) ----
  struct Run {
    const double* b = nullptr;
    double* x_user = nullptr;
    double tol = 0, bb = 0, rr_ref = 0, relres = 0;
    int restarts = 0;
    ipdg_status status = IPDG_OK;
    bool finished = false;
    clk::time_point t0;
  };

  // enqueue: x copy, scalars, r = b - A x; the scalars are copied to the host
  void start(Run& R, const double* b, double* x_user, double tol) {
    if (!(tol > 0.0)) throw Error(IPDG_EINVAL, "tol must be positive");
    R = Run();
    R.b = b;
    R.x_user = x_user;
    R.tol = tol;
    R.t0 = clk::now();
    double* x = w_->xw.as<double>();
    IPDG_HIP(hipMemcpyAsync(x, x_user, n_ * sizeof(double), hipMemcpyDeviceToDevice, s_));
    CGScal init{};
    init.tol = tol;
    init.max_iters = o_.max_iters;
    init.flexible = flexible_;
    IPDG_HIP(set_scal(w_->scal.as<CGScal>(), init, s_));
    true_residual(b, x);
    copy_scal();
  }

  // after the stream has reached the end of start(): z = B r, p = z
  void after_start(Run& R) {
    R.bb = w_->host_scal->bb;
    if (R.bb == 0.0) {
      IPDG_HIP(hipMemsetAsync(R.x_user, 0, n_ * sizeof(double), s_));
      mark_done();
      R.finished = true;
      return;
    }
    R.rr_ref = w_->host_scal->rr;
    R.relres = std::sqrt(R.rr_ref / R.bb);
    restart(w_->xw.as<double>());
  }

  // after `every` iterations and a copy of the scalars: decide to continue,
  // replace the residual, stop or fail.  Returns true when finished.
  bool after_step(Run& R) {
    const CGScal& h = *w_->host_scal;
    double* x = w_->xw.as<double>();
    if (h.breakdown) {
      R.status = IPDG_EBREAKDOWN;
      R.relres = NAN;
      mark_done();
      return R.finished = true;
    }
    const double drop2 = drop_ * drop_;
    const bool stopped = h.done != 0;
    const bool replace = stopped || (drop2 > 0.0 && h.rr <= drop2 * R.rr_ref);
    if (!replace) return false;
    const int iters_now = h.iters;
    true_residual(R.b, x);
    read_scal();
    const double rr_true = w_->host_scal->rr;
    R.relres = std::sqrt(rr_true / R.bb);
    if (!(rr_true == rr_true)) R.status = IPDG_EBREAKDOWN;
    else if (rr_true <= R.tol * R.tol * R.bb) R.status = IPDG_OK;
    else if (iters_now >= o_.max_iters) R.status = IPDG_NOT_CONVERGED;
    else {
      R.rr_ref = rr_true;
      ++R.restarts;
      // Residual replacement (van der Vorst and Ye): the recurrence continues
      // from the true residual with the current search direction.  Only when
      // the recurrence had already stopped (its last direction update was not
      // applied), or the outer operator is FP32 (its directions have lost
      // A-conjugacy at the FP32 level), is the direction rebuilt from z = B r.
      if (stopped || op32_) restart(x);
      return false;
    }
    mark_done();
    return R.finished = true;
  }

  void finish(Run& R, ipdg_solve_info* info) {
    if (R.bb != 0.0)
      IPDG_HIP(hipMemcpyAsync(R.x_user, w_->xw.get(), n_ * sizeof(double), hipMemcpyDeviceToDevice, s_));
    IPDG_HIP(hipStreamSynchronize(s_));
    fill_info(info, R.bb != 0.0 ? w_->host_scal->iters : 0, R.bb != 0.0 ? R.relres : 0.0, R.restarts,
              ms_since(R.t0));
    if (R.status == IPDG_EBREAKDOWN) throw Error(IPDG_EBREAKDOWN, "CG breakdown (p^T A p <= 0 or not finite)");
  }

  ipdg_status solve(const double* b, double* x_user, double tol, ipdg_solve_info* info) {
    Run R;
    start(R, b, x_user, tol);
    IPDG_HIP(hipStreamSynchronize(s_));
    after_start(R);
    const int every = std::max(1, o_.check_every);
    while (!R.finished) {
      run_iterations(w_->xw.as<double>(), every);
      read_scal();
      after_step(R);
    }
    finish(R, info);
    return R.status;
  }

  // `every` outer iterations launched on this solve's own stream (its
  // captured graph)
  void launch_iterations(int every) { run_iterations(w_->xw.as<double>(), every); }
  hipStream_t stream() const { return s_; }

  // Batched coarse mode: one outer iteration captured as two graphs, the part
  // before the coarsest-level solve and the part after it; the caller runs
  // the coarsest-level solves of all members of a batch together in between
  // (reading coarse_rhs(), writing coarse_sol()).  Only p-multigrid has one.
  void capture_split() {
    Work& w = *w_;
    if (w.graph_pre && w.graph_post) return;   // captured for this setup already
    w.drop_split();
    split_count_ = 0;
    splitting_ = true;
    hipGraph_t g = nullptr;
    IPDG_HIP(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
    try {
      iteration(w.xw.as<double>());
    } catch (...) {
      splitting_ = false;
      (void)hipStreamEndCapture(s_, &g);
      if (g) (void)hipGraphDestroy(g);
      w.drop_split();
      throw;
    }
    splitting_ = false;
    IPDG_HIP(hipStreamEndCapture(s_, &g));
    hipError_t e = hipGraphInstantiate(&w.graph_post, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    IPDG_HIP(e);
    if (split_count_ != 1 || !w.graph_pre) {
      w.drop_split();
      throw Error(IPDG_EUNSUPPORTED, "an outer iteration does not reach the coarsest level exactly once");
    }
  }
  unsigned long long setup_id() const { return w_->setup_id; }
  // Iteration cap of the coarsest-level Jacobi-PCG: the option, or when it is
  // negative max(20, ceil(0.414 sqrt(K))).  Jacobi-PCG needs iterations
  // growing like 1/h on the degree-1 level; the factor puts the cap at 150
  // for 131,072 triangles, where 150 was the measured optimum of time to
  // solution (see the design notes for the sweep), and at 75 for 32,768.
  int coarse_cap() const {
    if (o_.coarse_max_iters >= 0) return o_.coarse_max_iters;
    return std::max(20, (int)std::ceil(0.414 * std::sqrt((double)K_)));
  }
  void launch_pre() { IPDG_HIP(hipGraphLaunch(w_->graph_pre, s_)); }
  void launch_post() { IPDG_HIP(hipGraphLaunch(w_->graph_post, s_)); }
  const Level& coarsest() const { return w_->lv.back(); }
  const void* coarse_rhs() const { return w_->split_f; }
  void* coarse_sol() const { return w_->split_x; }
  ipdg_mesh_s* mesh() const { return m_; }
  double lambda() const { return lambda_; }
  const int* done_flag() const { return outer_done(); }
  void copy_scal() {
    IPDG_HIP(hipMemcpyAsync(w_->host_scal, w_->scal.get(), sizeof(CGScal), hipMemcpyDeviceToHost, s_));
  }

 private:
  void validate() {
    if (o_.pc < IPDG_PC_NONE || o_.pc > IPDG_PC_PMG) throw Error(IPDG_EINVAL, "bad preconditioner");
    if (o_.prec != IPDG_PREC_FP64 && o_.prec != IPDG_PREC_MIXED && o_.prec != IPDG_PREC_FP32_OPERATOR)
      throw Error(IPDG_EINVAL, "bad precision");
    if (o_.max_iters < 0) throw Error(IPDG_EINVAL, "max_iters < 0");
    if (o_.pc == IPDG_PC_PMG) {
      if (o_.n_levels < 1 || o_.n_levels > IPDG_MAX_LEVELS) throw Error(IPDG_EINVAL, "n_levels out of range");
      if (o_.degrees[0] != N_) throw Error(IPDG_EINVAL, "degrees[0] must equal the mesh degree");
      for (int l = 1; l < o_.n_levels; ++l)
        if (!(o_.degrees[l] < o_.degrees[l - 1]) || o_.degrees[l] < 1)
          throw Error(IPDG_EINVAL, "degrees must be strictly decreasing and >= 1");
      if (o_.cheb_degree < 1) throw Error(IPDG_EINVAL, "cheb_degree < 1");
      if (!(o_.cheb_hi > o_.cheb_lo) || !(o_.cheb_lo > 0)) throw Error(IPDG_EINVAL, "bad Chebyshev interval");
      // coarse_max_iters < 0: the automatic cap (coarse_cap())
      if (o_.coarse_persistent != 0 && o_.coarse_persistent != 1)
        throw Error(IPDG_EINVAL, "coarse_persistent must be 0 or 1");
    }
  }

  bool same_setup() const {
    const Work& w = *w_;
    if (w.n != n_ || w.lambda != lambda_ || w.ctau != ctau_ || w.pc != o_.pc || w.prec != o_.prec ||
        w.has_kappa != m_->has_kappa)
      return false;
    if (m_->has_kappa && w.kappa_version != m_->kappa_version) return false;
    if (o_.pc == IPDG_PC_PMG) {
      if (w.nlev != o_.n_levels || w.cheb_degree != o_.cheb_degree || w.cheb_lo != o_.cheb_lo ||
          w.cheb_hi != o_.cheb_hi || w.coarse_max != o_.coarse_max_iters ||
          w.coarse_tol != o_.coarse_tol || w.rho_steps != o_.rho_steps)
        return false;
      for (int l = 0; l < o_.n_levels; ++l)
        if (w.degrees[l] != o_.degrees[l] || w.rho_in[l] != o_.rho[l]) return false;
    }
    return true;
  }

  void setup() {
    Work& w = *w_;
    if (same_setup()) {
      select_coarse();
      return;
    }
    const auto t0 = clk::now();
    w.drop_graph();
    w.setup_id = next_setup_id();
    w.lv.clear();
    w.n = n_;
    w.xw.ensure(n_ * 8);
    w.r.ensure(n_ * 8);
    w.p.ensure(n_ * 8);
    w.t64.ensure(n_ * 8);
    w.Ap.ensure(n_ * 8);
    w.z.ensure(n_ * (mixed_ ? 4 : 8));
    if (op32_) {
      w.p32.ensure(n_ * 4);
      w.Ap32.ensure(n_ * 4);
    }
    w.partials.ensure(3 * kMaxPartials * sizeof(double));
    w.cpartials.ensure(6 * kMaxPartials * sizeof(double));
    w.scal.ensure(sizeof(CGScal));
    w.cscal.ensure(sizeof(CGScal));
    if (!w.host_scal) IPDG_HIP(hipHostMalloc(reinterpret_cast<void**>(&w.host_scal), sizeof(CGScal)));
    if (o_.pc == IPDG_PC_JACOBI || o_.pc == IPDG_PC_NONE) {
      w.dinv64.ensure(n_ * 8);
      w.dinv32.ensure(n_ * 4);
      if (o_.pc == IPDG_PC_JACOBI) {
        ElemArgs a = elem_args(m_, N_, Kind::F64, lambda_, ctau_);
        a.y = w.dinv64.get();
        IPDG_HIP(diag(N_, Kind::F64, a, s_));
      } else {
        std::vector<double> ones(n_, 1.0);
        IPDG_HIP(hipMemcpyAsync(w.dinv64.get(), ones.data(), n_ * 8, hipMemcpyHostToDevice, s_));
        IPDG_HIP(hipStreamSynchronize(s_));
        IPDG_HIP(recip(w.dinv64.as<double>(), nullptr, n_, s_));   // keeps 1
      }
      if (o_.pc == IPDG_PC_JACOBI) IPDG_HIP(recip(w.dinv64.as<double>(), w.dinv32.as<float>(), n_, s_));
    }
    if (o_.pc == IPDG_PC_PMG) setup_pmg();
    // every operator table a captured iteration uses exists before capture
    (void)device_ops(N_, Kind::F64);
    (void)device_ops(N_, Kind::F32);
    for (const Level& v : w.lv) {
      (void)device_ops(v.N, Kind::F64);
      (void)device_ops(v.N, Kind::F32);
    }
    IPDG_HIP(hipStreamSynchronize(s_));
    w.lambda = lambda_;
    w.ctau = ctau_;
    w.pc = o_.pc;
    w.prec = o_.prec;
    w.has_kappa = m_->has_kappa;
    w.kappa_version = m_->kappa_version;
    w.nlev = o_.n_levels;
    w.cheb_degree = o_.cheb_degree;
    w.cheb_lo = o_.cheb_lo;
    w.cheb_hi = o_.cheb_hi;
    w.coarse_max = o_.coarse_max_iters;
    w.coarse_tol = o_.coarse_tol;
    w.rho_steps = o_.rho_steps;
    for (int l = 0; l < IPDG_MAX_LEVELS; ++l) {
      w.degrees[l] = o_.degrees[l];
      w.rho_in[l] = o_.rho[l];
    }
    w.setup_ms = ms_since(t0);
  }

  void setup_pmg() {
    Work& w = *w_;
    const int L = o_.n_levels;
    w.lv.resize(L);
    for (int l = 0; l < L; ++l) {
      Level& v = w.lv[l];
      v.N = o_.degrees[l];
      v.Np = np_of(v.N);
      v.n = (size_t)K_ * v.Np;
      const double q = double(v.N + 1) / double(N_ + 1);
      v.ctau = ctau_ * q * q;
      v.fp32 = mixed_;
      v.kind = mixed_ ? Kind::F32 : Kind::F64;
      const size_t w8 = v.fp32 ? 4 : 8;
      v.dinv64.ensure(v.n * 8);
      v.dinv32.ensure(v.n * 4);
      ElemArgs a = elem_args(m_, v.N, Kind::F64, lambda_, v.ctau);
      a.y = v.dinv64.get();
      IPDG_HIP(diag(v.N, Kind::F64, a, s_));
      IPDG_HIP(recip(v.dinv64.as<double>(), v.dinv32.as<float>(), v.n, s_));
      if (l > 0) v.f.ensure(v.n * w8);
      if (l > 0 || l + 1 < L) v.z.ensure(v.n * w8);
      v.r.ensure(v.n * w8);
      v.d.ensure(v.n * w8);
      v.t.ensure(v.n * w8);
      if (l == 0 && mixed_) v.f.ensure(v.n * w8);
      if (l == L - 1) {
        v.cr.ensure(v.n * w8);
        v.cz.ensure(v.n * w8);
        v.cp.ensure(v.n * w8);
        v.cp2.ensure(v.n * w8);
        v.cAp.ensure(v.n * w8);
        v.cr2.ensure(v.n * w8);
        v.cw2.ensure(v.n * w8);
        v.cs2.ensure(v.n * w8);
        if (!v.z.get()) v.z.ensure(v.n * w8);
      }
      if (l > 0) w.lv[l - 1].P = device_interp(v.N, w.lv[l - 1].N, mixed_);
    }
    for (int l = 0; l < L; ++l) {
      Level& v = w.lv[l];
      v.rho = o_.rho[l] > 0.0 ? o_.rho[l] : lanczos_rho(v, l);
    }
    CGScal c{};
    c.tol = o_.coarse_tol;
    c.max_iters = coarse_cap();
    c.flexible = 0;
    IPDG_HIP(set_scal(w.cscal.as<CGScal>(), c, s_));
    w.cbar.ensure(8 * sizeof(int));
    IPDG_HIP(zero_ints(w.cbar.get(), 8, s_));
    w.coarse_grid = -1;
    select_coarse();
  }

  // persistent single-launch coarse solve or ordinary launches; a change
  // invalidates the captured iteration graph
  void select_coarse() {
    Work& w = *w_;
    if (o_.pc != IPDG_PC_PMG || w.lv.empty()) return;
    const Level& cl = w.lv.back();
    const int g = (persistent_ && o_.coarse_persistent == 1) ? coarse_pcg_grid(cl.N, cl.kind, K_) : 0;
    if (g != w.coarse_grid) {
      w.drop_graph();
      w.coarse_grid = g;
    }
  }

  // rho_steps Jacobi-PCG (Lanczos) steps on a level operator in FP64 from a
  // seeded N(0,1) right-hand side; largest Ritz value of D^-1 A.
  double lanczos_rho(Level& v, int l) {
    Work& w = *w_;
    const int steps = std::max(2, o_.rho_steps);
    std::mt19937_64 gen(1234 + l);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<double> bh(v.n);
    for (auto& e : bh) e = nd(gen);
    DevBuf b(v.n * 8), x(v.n * 8), r(v.n * 8), z(v.n * 8), p(v.n * 8), Ap(v.n * 8);
    IPDG_HIP(hipMemcpyAsync(b.get(), bh.data(), v.n * 8, hipMemcpyHostToDevice, s_));
    CGScal c{};
    c.tol = 0.0;
    c.max_iters = steps + 1;
    CGScal* sc = w.cscal.as<CGScal>();
    IPDG_HIP(set_scal(sc, c, s_));
    IPDG_HIP(cg_start0(false, b.get(), v.dinv64.get(), x.get(), r.get(), z.get(), p.get(), v.n,
                       w.cpartials.as<double>(), nullptr, s_));
    IPDG_HIP(cg_start_fin(w.cpartials.as<double>(), flat_grid(v.n), sc, nullptr, s_));
    std::vector<double> al, be;
    ElemArgs a = elem_args(m_, v.N, Kind::F64, lambda_, v.ctau);
    for (int k = 0; k < steps; ++k) {
      a.x = p.get();
      a.y = Ap.get();
      a.partials = w.cpartials.as<double>();
      a.skip = nullptr;
      IPDG_HIP(ax(v.N, Kind::F64, a, s_));
      IPDG_HIP(finalize(w.cpartials.as<double>(), ax_partials(v.N, false, K_), 1, sc, kFinAlpha, s_));
      IPDG_HIP(cg_update_state(false, x.get(), r.get(), p.get(), Ap.get(), v.dinv64.get(), z.get(), sc,
                               v.n, w.cpartials.as<double>(), s_));
      IPDG_HIP(finalize(w.cpartials.as<double>(), flat_grid(v.n), 3, sc, kFinBeta, s_));
      IPDG_HIP(hipMemcpyAsync(w.host_scal, sc, sizeof(CGScal), hipMemcpyDeviceToHost, s_));
      IPDG_HIP(hipStreamSynchronize(s_));
      if (w.host_scal->done && w.host_scal->iters <= k) break;
      al.push_back(w.host_scal->alpha);
      be.push_back(w.host_scal->beta);
      IPDG_HIP(cg_pupdate_state(false, p.get(), z.get(), sc, v.n, s_));
    }
    const int k = int(al.size());
    if (k == 0) return 1.0;
    std::vector<double> diag_(k), off(k > 1 ? k - 1 : 0);
    for (int i = 0; i < k; ++i) {
      diag_[i] = 1.0 / al[i] + (i > 0 ? be[i - 1] / al[i - 1] : 0.0);
      if (i + 1 < k) off[i] = std::sqrt(be[i]) / al[i];
    }
    return tridiag_max_eig(diag_, off);
  }

  void read_scal() {
    copy_scal();
    IPDG_HIP(hipStreamSynchronize(s_));
  }

  // keep a finished solve's kernels idle (its iterations may still be replayed
  // inside a batched graph)
  void mark_done() {
    CGScal d{};
    d.done = 1;
    d.iters = w_->host_scal->iters;
    IPDG_HIP(set_scal(w_->scal.as<CGScal>(), d, s_));
  }

  // r = b - A x in FP64 and (r, r), (b, b)
  void true_residual(const double* b, const double* x) {
    ElemArgs a = elem_args(m_, N_, Kind::F64, lambda_, ctau_);
    a.x = x;
    a.y = w_->t64.get();
    IPDG_HIP(ax(N_, Kind::F64, a, s_));
    IPDG_HIP(residual(b, w_->t64.as<double>(), w_->r.as<double>(), n_, w_->partials.as<double>(), s_));
    IPDG_HIP(finalize(w_->partials.as<double>(), flat_grid(n_), 2, w_->scal.as<CGScal>(), kFinResidual, s_));
  }

  // z = B r, (r, z), p = z
  void restart(double*) {
    precond();
    IPDG_HIP(dots_rz(mixed_, w_->r.as<double>(), w_->z.get(), nullptr, w_->scal.as<CGScal>(), n_,
                     w_->partials.as<double>(), s_));
    IPDG_HIP(finalize(w_->partials.as<double>(), flat_grid(n_), 3, w_->scal.as<CGScal>(), kFinInit, s_));
    if (mixed_) IPDG_HIP(convert(false, w_->p.get(), w_->z.get(), n_, nullptr, s_));
    else IPDG_HIP(hipMemcpyAsync(w_->p.get(), w_->z.get(), n_ * 8, hipMemcpyDeviceToDevice, s_));
  }

  const int* outer_done() const { return done_ptr(w_->scal); }

  // z = B r (outer precision of z)
  void precond() {
    Work& w = *w_;
    switch (o_.pc) {
      case IPDG_PC_NONE:
      case IPDG_PC_JACOBI:
        IPDG_HIP(jacobi(mixed_, w.r.as<double>(), w.dinv64.as<double>(), w.z.get(), n_, s_));
        break;
      case IPDG_PC_BLOCK_MASS: {
        const Kind k = mixed_ ? Kind::F32_IN64 : Kind::F64;
        ElemArgs a = elem_args(m_, N_, k, 0.0, 0.0);
        a.x = w.r.get();
        a.y = w.z.get();
        a.skip = outer_done();
        IPDG_HIP(minv(N_, k, a, s_));
        break;
      }
      case IPDG_PC_PMG: {
        Level& v0 = w.lv[0];
        if (mixed_) IPDG_HIP(convert(true, v0.f.get(), w.r.get(), n_, outer_done(), s_));
        vcycle(0, mixed_ ? v0.f.get() : w.r.get(), w.z.get());
        break;
      }
    }
  }

  void level_ax(const Level& v, const void* x, void* y) {
    ElemArgs a = elem_args(m_, v.N, v.kind, lambda_, v.ctau);
    a.x = x;
    a.y = y;
    a.skip = outer_done();
    IPDG_HIP(ax(v.N, v.kind, a, s_));
  }

  void smooth(const Level& v, const void* f, void* z, bool from_zero) {
    const double lo = o_.cheb_lo * v.rho, hi = o_.cheb_hi * v.rho;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    double rho = 1.0 / sigma;
    if (from_zero) {
      IPDG_HIP(cheb(v.fp32, 0, f, nullptr, v.dinv(), z, v.d.get(), v.r.get(), 1.0 / theta, 0, 0, v.n,
                    outer_done(), s_));
    } else {
      level_ax(v, z, v.t.get());
      IPDG_HIP(cheb(v.fp32, 1, f, v.t.get(), v.dinv(), z, v.d.get(), v.r.get(), 1.0 / theta, 0, 0, v.n,
                    outer_done(), s_));
    }
    for (int k = 1; k < o_.cheb_degree; ++k) {
      const double rho_new = 1.0 / (2.0 * sigma - rho);
      level_ax(v, v.d.get(), v.t.get());
      IPDG_HIP(cheb(v.fp32, 2, nullptr, v.t.get(), v.dinv(), z, v.d.get(), v.r.get(), 0,
                    rho_new * rho, 2.0 * rho_new / delta, v.n, outer_done(), s_));
      rho = rho_new;
    }
  }

  void vcycle(int l, const void* f, void* z) {
    Work& w = *w_;
    Level& v = w.lv[l];
    if (l + 1 == (int)w.lv.size()) {
      coarse_solve(v, f, z);
      return;
    }
    Level& c = w.lv[l + 1];
    smooth(v, f, z, true);
    level_ax(v, z, v.t.get());
    TransferArgs ta;
    ta.f = f;
    ta.Az = v.t.get();
    ta.coarse = c.f.get();
    ta.P = v.P;
    ta.K = K_;
    ta.skip = outer_done();
    IPDG_HIP(restrict_(v.N, c.N, v.kind, ta, s_));
    vcycle(l + 1, c.f.get(), c.z.get());
    TransferArgs tp;
    tp.coarse = c.z.get();
    tp.fine = z;
    tp.P = v.P;
    tp.K = K_;
    tp.skip = outer_done();
    IPDG_HIP(prolong(v.N, c.N, v.kind, tp, s_));
    smooth(v, f, z, false);
  }

  // Jacobi-PCG from zero on the coarsest level, coarse_max iterations at most
  void coarse_solve(Level& v, const void* f, void* x) {
    Work& w = *w_;
    if (splitting_) {
      // batched coarse mode: close the graph of the part before, open the
      // one of the part after; the batch solves this level in between
      w.split_f = f;
      w.split_x = x;
      ++split_count_;
      hipGraph_t g = nullptr;
      IPDG_HIP(hipStreamEndCapture(s_, &g));
      if (w.graph_pre) (void)hipGraphExecDestroy(w.graph_pre);
      w.graph_pre = nullptr;
      hipError_t e = hipGraphInstantiate(&w.graph_pre, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      IPDG_HIP(e);
      IPDG_HIP(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
      return;
    }
    if (w.coarse_grid > 0) {
      // one persistent launch; a kernel node resets the two barrier counters
      // (the status words keep the last executed solve's record, since the
      // launch is a no-op once the outer solve is done)
      IPDG_HIP(zero_ints(w.cbar.get(), 2, s_));
      CoarseArgs ca;
      ca.f = f;
      ca.x = x;
      ca.r = v.cr.get();
      ca.z = v.cz.get();
      ca.p = v.cp.get();
      ca.Ap = v.cAp.get();
      ca.dinv = v.dinv();
      ca.op = elem_args(m_, v.N, v.kind, lambda_, v.ctau);
      ca.tol = o_.coarse_tol;
      ca.max_iters = coarse_cap();
      ca.partials = w.cpartials.as<double>();
      ca.bar = w.cbar.as<unsigned>();
      ca.status = w.cbar.as<int>() + 2;
      ca.skip = outer_done();
      IPDG_HIP(coarse_pcg(v.N, v.kind, ca, w.coarse_grid, s_));
      return;
    }
    CGScal* sc = w.cscal.as<CGScal>();
    double* part = w.cpartials.as<double>();     // two sets of 3 partial slots
    double* set[2] = {part, part + 3 * (size_t)kMaxPartials};
    void* rb[2] = {v.cr.get(), v.cr2.get()};
    void* wb[2] = {v.cAp.get(), v.cw2.get()};
    void* sb[2] = {v.cp2.get(), v.cs2.get()};
    // x = 0, r = f, u = D^-1 f and the (r, r), (r, u) partials (set 0, slots 0, 1)
    IPDG_HIP(cg_start0(v.fp32, f, v.dinv(), x, rb[0], v.cz.get(), v.cp.get(), v.n, part, outer_done(), s_));
    // w = A u and the (u, w) partials (set 0, slot 2)
    ElemArgs a = elem_args(m_, v.N, v.kind, lambda_, v.ctau);
    a.x = v.cz.get();
    a.y = wb[0];
    a.partials = part + 2 * (size_t)kMaxPartials;
    a.skip = outer_done();
    IPDG_HIP(ax(v.N, v.kind, a, s_));
    CoarseStepArgs ca;
    ca.x = x;
    ca.p = v.cp.get();
    ca.u = v.cz.get();
    ca.dinv = v.dinv();
    ca.op = elem_args(m_, v.N, v.kind, lambda_, v.ctau);
    ca.sc = sc;
    ca.outer = outer_done();
    const int ne = elem_grid(K_);
    for (int it = 0; it < coarse_cap(); ++it) {
      const int o = it & 1, nw = 1 - o;
      ca.it = it;
      ca.r_old = rb[o];
      ca.r_new = rb[nw];
      ca.w_old = wb[o];
      ca.w_new = wb[nw];
      ca.s_old = sb[o];
      ca.s_new = sb[nw];
      ca.pin = set[o];
      ca.pout = set[nw];
      ca.n_rr = ca.n_g = it == 0 ? flat_grid(v.n) : ne;
      // the first (u, w) partials come from the operator launch above
      ca.n_d = it == 0 ? ax_partials(v.N, v.fp32, K_) : ne;
      IPDG_HIP(coarse_step(v.N, v.kind, ca, s_));
    }
  }

  // `every` outer iterations: replayed from a captured graph (all pointers
  // are internal buffers, fixed for the lifetime of the setup)
  void run_iterations(double* x, int every) {
    if (!use_graph_) {
      for (int k = 0; k < every; ++k) iteration(x);
      return;
    }
    Work& w = *w_;
    if (!w.graph || w.graph_iters != every) {
      w.drop_main();
      hipGraph_t g = nullptr;
      IPDG_HIP(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
      try {
        for (int k = 0; k < every; ++k) iteration(x);
      } catch (...) {
        (void)hipStreamEndCapture(s_, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      IPDG_HIP(hipStreamEndCapture(s_, &g));
      hipError_t e = hipGraphInstantiate(&w.graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      IPDG_HIP(e);
      w.graph_iters = every;
    }
    IPDG_HIP(hipGraphLaunch(w.graph, s_));
  }

  void iteration(double* x) {
    Work& w = *w_;
    CGScal* sc = w.scal.as<CGScal>();
    // With IPDG_PREC_MIXED the outer operator is FP64: an FP32 product A p
    // loses relative accuracy ~ u32 cond(A) on the smooth directions late CG
    // builds, which stalls the recurrence; FP32 stays inside the
    // preconditioner, where its error only perturbs a flexible
    // preconditioner.  IPDG_PREC_FP32_OPERATOR applies A p in FP32 too (p
    // rounded to FP32, the product widened back, (p, A p) summed in FP64),
    // with reliable updates of the residual.
    if (op32_) {
      IPDG_HIP(convert(true, w.p32.get(), w.p.get(), n_, outer_done(), s_));
      ElemArgs a = elem_args(m_, N_, Kind::F32, lambda_, ctau_);
      a.x = w.p32.get();
      a.y = w.Ap32.get();
      a.partials = w.partials.as<double>();
      a.skip = outer_done();
      IPDG_HIP(ax(N_, Kind::F32, a, s_));
      IPDG_HIP(finalize(w.partials.as<double>(), ax_partials(N_, true, K_), 1, sc, kFinAlpha, s_));
      IPDG_HIP(convert(false, w.Ap.get(), w.Ap32.get(), n_, outer_done(), s_));
    } else {
      ElemArgs a = elem_args(m_, N_, Kind::F64, lambda_, ctau_);
      a.x = w.p.get();
      a.y = w.Ap.get();
      a.partials = w.partials.as<double>();
      a.skip = outer_done();
      IPDG_HIP(ax(N_, Kind::F64, a, s_));
      IPDG_HIP(finalize(w.partials.as<double>(), ax_partials(N_, false, K_), 1, sc, kFinAlpha, s_));
    }
    const bool jac = o_.pc == IPDG_PC_JACOBI || o_.pc == IPDG_PC_NONE;
    IPDG_HIP(cg_update(mixed_, jac, x, w.r.as<double>(), w.p.as<double>(), w.Ap.as<double>(), w.dinv64.as<double>(),
                       w.z.get(), sc, n_, w.partials.as<double>(), s_));
    if (!jac) {
      precond();
      IPDG_HIP(dots_rz(mixed_, w.r.as<double>(), w.z.get(), w.Ap.as<double>(), sc, n_, w.partials.as<double>(), s_));
    }
    IPDG_HIP(finalize(w.partials.as<double>(), flat_grid(n_), 3, sc, kFinBeta, s_));
    IPDG_HIP(pupdate(mixed_, w.p.as<double>(), w.z.get(), sc, n_, s_));
  }

  // status of the persistent coarse solve: [0] iterations, [1] barrier
  // timeout, [2] breakdown
  int coarse_status() {
    Work& w = *w_;
    if (o_.pc != IPDG_PC_PMG || w.lv.empty()) return -1;
    if (w.coarse_grid == 0) {
      CGScal c{};
      IPDG_HIP(hipMemcpyAsync(&c, w.cscal.get(), sizeof(c), hipMemcpyDeviceToHost, s_));
      IPDG_HIP(hipStreamSynchronize(s_));
      return c.iters;
    }
    int st[3] = {0, 0, 0};
    IPDG_HIP(hipMemcpyAsync(st, w.cbar.as<int>() + 2, sizeof(st), hipMemcpyDeviceToHost, s_));
    IPDG_HIP(hipStreamSynchronize(s_));
    if (st[1]) throw Error(IPDG_EHIP, "coarse solve: grid barrier timed out");
    return st[0];
  }

  void fill_info(ipdg_solve_info* info, int iters, double relres, int restarts, double solve_ms) {
    const int citers = coarse_status();
    if (!info) return;
    std::memset(info, 0, sizeof(*info));
    info->coarse_iters = citers;
    info->iters = iters;
    info->relres = relres;
    info->restarts = restarts;
    for (size_t l = 0; l < w_->lv.size() && l < IPDG_MAX_LEVELS; ++l) info->rho_used[l] = w_->lv[l].rho;
    info->setup_ms = w_->setup_ms;
    info->solve_ms = solve_ms;
  }

  ipdg_mesh_s* m_;
  ipdg_solve_opts o_;
  hipStream_t s_;
  hipStream_t user_ = nullptr;
  bool use_graph_ = true;
  bool persistent_ = true;
  Work* w_ = nullptr;
  int N_ = 0, K_ = 0;
  size_t n_ = 0;
  double lambda_ = 0, ctau_ = 0;
  bool mixed_ = false, flexible_ = false;
  bool op32_ = false;                // FP32 outer operator (IPDG_PREC_FP32_OPERATOR)
  double drop_ = 0.0;                // reliable-update factor in use
  bool splitting_ = false;           // capturing the two halves of a split iteration
  int split_count_ = 0;
};

}  // namespace

ipdg_status pcg_solve(ipdg_mesh_s* m, double lambda, double tau, const double* b, double* x, double tol,
                      const ipdg_solve_opts& o, ipdg_solve_info* info, hipStream_t s) {
  if (m->host.K == 0) {
    if (info) std::memset(info, 0, sizeof(*info));
    return IPDG_OK;
  }
  if (!b || !x) throw Error(IPDG_EINVAL, "null vector");
  Solver sv(m, lambda, tau, o, s);
  return sv.solve(b, x, tol, info);
}

ipdg_status precond_apply(ipdg_mesh_s* m, double lambda, double tau, const ipdg_solve_opts& o,
                          const double* r, double* z, ipdg_solve_info* info, hipStream_t s) {
  if (m->host.K == 0) return IPDG_OK;
  if (!r || !z) throw Error(IPDG_EINVAL, "null vector");
  Solver sv(m, lambda, tau, o, s);
  sv.apply_precond(r, z, info);
  return IPDG_OK;
}

namespace {

// The coarsest levels of a batch's solves, concatenated (CoarseBatchArgs),
// with the captured graph of one batched coarse solve and the events that
// order it against the solves' own streams.
struct CoarseBatchSet {
  DevBuf ent, tile_solve, x, p, u, dinv, r0, r1, w0, w1, s0, s1, geo, conn, kap, partials, sc;
  CoarseBatchArgs a;
  int max_iters = 0;               // the largest member cap: coarse launches per solve
  hipStream_t stream = nullptr;
  hipGraphExec_t graph = nullptr;
  std::vector<hipEvent_t> ev;
  hipEvent_t ev_done = nullptr;
  ~CoarseBatchSet() {
    if (graph) (void)hipGraphExecDestroy(graph);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (ev_done) (void)hipEventDestroy(ev_done);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

// IPDG_BATCH_COARSE=separate keeps every solve's coarsest level on its own
// launches (the fused form is the default).
bool batch_coarse_fused() {
  const char* v = std::getenv("IPDG_BATCH_COARSE");
  return !(v && std::strcmp(v, "separate") == 0);
}

// Null when the solves' coarsest levels differ in degree or precision (the
// caller then keeps them separate).
std::unique_ptr<CoarseBatchSet> make_coarse_batch(std::vector<std::unique_ptr<Solver>>& sv,
                                                  const ipdg_solve_opts& o) {
  const int na = int(sv.size());
  const Level& c0 = sv[0]->coarsest();
  for (int k = 1; k < na; ++k) {
    const Level& c = sv[k]->coarsest();
    if (c.N != c0.N || c.kind != c0.kind) return nullptr;
  }
  const int Nc = c0.N, Np = c0.Np;
  const Kind kind = c0.kind;
  const size_t w = c0.fp32 ? 4 : 8;
  std::unique_ptr<CoarseBatchSet> cb(new CoarseBatchSet);
  IPDG_HIP(hipStreamCreateWithFlags(&cb->stream, hipStreamNonBlocking));
  std::vector<CoarseBatchEntry> ent(na);
  int off = 0;
  bool any_kappa = false;
  for (int k = 0; k < na; ++k) {
    const int K = sv[k]->mesh()->host.K;
    const int nt = (K + kBlock - 1) / kBlock;
    ent[k].off = off;
    ent[k].K = K;
    ent[k].tile0 = off / kBlock;
    ent[k].ntiles = nt;
    ent[k].lambda = sv[k]->lambda();
    ent[k].ctau = sv[k]->coarsest().ctau;
    ent[k].outer = sv[k]->done_flag();
    ent[k].f = sv[k]->coarse_rhs();
    ent[k].z = sv[k]->coarse_sol();
    off += nt * kBlock;
    any_kappa = any_kappa || sv[k]->mesh()->has_kappa;
  }
  const int Kt = off, tiles = off / kBlock;
  int per;
  const int grid = xcd_grid(tiles, per);
  if (grid > kMaxPartials) throw Error(IPDG_EUNSUPPORTED, "batch too large for one coarse launch");
  std::vector<int> ts(grid, -1);
  for (int k = 0; k < na; ++k)
    for (int t = 0; t < ent[k].ntiles; ++t) ts[ent[k].tile0 + t] = k;
  std::vector<Conn> conn((size_t)Kt, Conn{});
  for (int k = 0; k < na; ++k) {
    const auto& hc = sv[k]->mesh()->host.conn;
    for (int e = 0; e < ent[k].K; ++e) {
      Conn c = hc[e];
      for (int f = 0; f < 3; ++f) c.nb[f] += ent[k].off;
      conn[(size_t)ent[k].off + e] = c;
    }
  }
  const size_t nv = (size_t)Kt * Np * w;
  hipStream_t cs = cb->stream;
  cb->ent.alloc(na * sizeof(CoarseBatchEntry));
  cb->tile_solve.alloc(grid * sizeof(int));
  cb->conn.alloc((size_t)Kt * sizeof(Conn));
  IPDG_HIP(hipMemcpyAsync(cb->ent.get(), ent.data(), na * sizeof(CoarseBatchEntry), hipMemcpyHostToDevice, cs));
  IPDG_HIP(hipMemcpyAsync(cb->tile_solve.get(), ts.data(), grid * sizeof(int), hipMemcpyHostToDevice, cs));
  IPDG_HIP(hipMemcpyAsync(cb->conn.get(), conn.data(), (size_t)Kt * sizeof(Conn), hipMemcpyHostToDevice, cs));
  for (DevBuf* b : {&cb->x, &cb->p, &cb->u, &cb->dinv, &cb->r0, &cb->r1, &cb->w0, &cb->w1, &cb->s0, &cb->s1})
    b->alloc(nv);
  cb->geo.alloc((size_t)Kt * 4 * w);
  if (any_kappa) cb->kap.alloc((size_t)Kt * w);
  for (int k = 0; k < na; ++k) {
    ipdg_mesh_s* m = sv[k]->mesh();
    const int K = ent[k].K;
    char* g = cb->geo.as<char>() + (size_t)ent[k].off * 4 * w;
    IPDG_HIP(hipMemcpyAsync(g, geo_for(m, kind), (size_t)K * 4 * w, hipMemcpyDeviceToDevice, cs));
    char* d = cb->dinv.as<char>() + (size_t)ent[k].off * Np * w;
    IPDG_HIP(hipMemcpyAsync(d, sv[k]->coarsest().dinv(), (size_t)K * Np * w, hipMemcpyDeviceToDevice, cs));
    if (any_kappa) {
      char* q = cb->kap.as<char>() + (size_t)ent[k].off * w;
      if (m->has_kappa) {
        const void* src = c0.fp32 ? m->kap32.get() : m->kap64.get();
        IPDG_HIP(hipMemcpyAsync(q, src, (size_t)K * w, hipMemcpyDeviceToDevice, cs));
      } else {
        const std::vector<float> one32(c0.fp32 ? K : 0, 1.0f);
        const std::vector<double> one64(c0.fp32 ? 0 : K, 1.0);
        const void* src = c0.fp32 ? (const void*)one32.data() : (const void*)one64.data();
        IPDG_HIP(hipMemcpyAsync(q, src, (size_t)K * w, hipMemcpyHostToDevice, cs));
        IPDG_HIP(hipStreamSynchronize(cs));   // before the host vectors go
      }
    }
  }
  cb->partials.alloc(6 * (size_t)kMaxPartials * sizeof(double));
  std::vector<CGScal> sc(na);
  cb->max_iters = 0;
  for (int k = 0; k < na; ++k) {
    sc[k].tol = o.coarse_tol;
    sc[k].max_iters = sv[k]->coarse_cap();
    cb->max_iters = std::max(cb->max_iters, sc[k].max_iters);
  }
  cb->sc.alloc(na * sizeof(CGScal));
  IPDG_HIP(hipMemcpyAsync(cb->sc.get(), sc.data(), na * sizeof(CGScal), hipMemcpyHostToDevice, cs));
  IPDG_HIP(hipStreamSynchronize(cs));
  CoarseBatchArgs& a = cb->a;
  a.ent = cb->ent.as<CoarseBatchEntry>();
  a.tile_solve = cb->tile_solve.as<int>();
  a.grid = grid;
  a.per = per;
  a.x = cb->x.get();
  a.p = cb->p.get();
  a.u = cb->u.get();
  a.dinv = cb->dinv.get();
  a.r[0] = cb->r0.get();
  a.r[1] = cb->r1.get();
  a.w[0] = cb->w0.get();
  a.w[1] = cb->w1.get();
  a.s[0] = cb->s0.get();
  a.s[1] = cb->s1.get();
  a.geo = cb->geo.get();
  a.conn = cb->conn.as<Conn>();
  a.kap = any_kappa ? cb->kap.get() : nullptr;
  a.ops = device_ops(Nc, kind);
  a.partials = cb->partials.as<double>();
  a.sc = cb->sc.as<CGScal>();
  // one batched coarse solve: start, coarse_max iterations, copy-out
  hipGraph_t g = nullptr;
  IPDG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  try {
    IPDG_HIP(coarse_batch(Nc, kind, a, -1, cs));
    for (int it = 0; it < cb->max_iters; ++it) IPDG_HIP(coarse_batch(Nc, kind, a, it, cs));
    IPDG_HIP(coarse_batch(Nc, kind, a, -2, cs));
  } catch (...) {
    (void)hipStreamEndCapture(cs, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  IPDG_HIP(hipStreamEndCapture(cs, &g));
  hipError_t e = hipGraphInstantiate(&cb->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  IPDG_HIP(e);
  cb->ev.assign(na, nullptr);
  for (int k = 0; k < na; ++k) IPDG_HIP(hipEventCreateWithFlags(&cb->ev[k], hipEventDisableTiming));
  IPDG_HIP(hipEventCreateWithFlags(&cb->ev_done, hipEventDisableTiming));
  return cb;
}

// What a batched coarse set was built for: the solves' setups (ids are never
// reused, so a destroyed mesh never matches), their coarse buffers and
// constants, the coarse options and the device.
struct CoarseBatchKey {
  std::vector<unsigned long long> ids;
  std::vector<const void*> ptrs;
  std::vector<double> lambdas;
  double coarse_tol = 0;
  int coarse_max = 0, device = -1;
  bool operator==(const CoarseBatchKey& o) const {
    return ids == o.ids && ptrs == o.ptrs && lambdas == o.lambdas && coarse_tol == o.coarse_tol &&
           coarse_max == o.coarse_max && device == o.device;
  }
};

CoarseBatchKey coarse_batch_key(const std::vector<std::unique_ptr<Solver>>& sv, const ipdg_solve_opts& o) {
  CoarseBatchKey k;
  for (const auto& s : sv) {
    k.ids.push_back(s->setup_id());
    k.ptrs.push_back(s->coarse_rhs());
    k.ptrs.push_back(s->coarse_sol());
    k.ptrs.push_back(s->done_flag());
    k.lambdas.push_back(s->lambda());
  }
  k.coarse_tol = o.coarse_tol;
  k.coarse_max = o.coarse_max_iters;
  (void)hipGetDevice(&k.device);
  return k;
}

// The last batched coarse set, reused by the next batch of the same solves
// (a serving loop); held until it is replaced (never freed at process exit,
// when the runtime may already be gone).
std::mutex g_cb_mu;
CoarseBatchSet* g_cb = nullptr;
bool g_cb_valid = false;
CoarseBatchKey g_cb_key;

}  // namespace

ipdg_status solve_batch(int nb, ipdg_mesh_s* const* meshes, const double* lambdas, double tau,
                        const double* const* b, double* const* x, double tol, const ipdg_solve_opts& o,
                        int* iters, double* relres, hipStream_t s) {
  // Every solve keeps its own device state, stream and captured graph; the
  // host advances all of them by check_every iterations per round.
  for (int i = 0; i < nb; ++i) {
    if (!meshes[i]) throw Error(IPDG_EINVAL, "null mesh in batch");
    if (!b[i] || !x[i]) throw Error(IPDG_EINVAL, "null vector in batch");
    for (int j = 0; j < i; ++j)
      if (meshes[j] == meshes[i]) throw Error(IPDG_EINVAL, "a mesh handle appears twice in the batch");
  }
  std::vector<std::unique_ptr<Solver>> sv;
  std::vector<Solver::Run> runs(nb);
  std::vector<int> active;
  for (int i = 0; i < nb; ++i) {
    if (meshes[i]->host.K == 0) continue;
    sv.emplace_back(new Solver(meshes[i], lambdas[i], tau, o, s, /*persistent=*/false));
    active.push_back(i);
  }
  const int na = int(sv.size());
  for (int k = 0; k < na; ++k) sv[k]->start(runs[k], b[active[k]], x[active[k]], tol);
  for (int k = 0; k < na; ++k) IPDG_HIP(hipStreamSynchronize(sv[k]->stream()));
  for (int k = 0; k < na; ++k) sv[k]->after_start(runs[k]);
  const int every = std::max(1, o.check_every);
  int left = 0;
  for (int k = 0; k < na; ++k) left += !runs[k].finished;
  std::unique_ptr<CoarseBatchSet> own_cb;
  CoarseBatchSet* cb = nullptr;
  std::unique_lock<std::mutex> lk(g_cb_mu, std::defer_lock);
  if (left > 0 && o.pc == IPDG_PC_PMG && na >= 2 && batch_coarse_fused()) {
    for (int k = 0; k < na; ++k) sv[k]->capture_split();
    const CoarseBatchKey key = coarse_batch_key(sv, o);
    if (lk.try_lock()) {
      if (!g_cb_valid || !(g_cb_key == key)) {
        delete g_cb;
        g_cb = nullptr;
        g_cb_valid = false;
        g_cb = make_coarse_batch(sv, o).release();
        g_cb_key = key;
        g_cb_valid = true;
      }
      cb = g_cb;
    } else {
      own_cb = make_coarse_batch(sv, o);   // another thread holds the cached set
      cb = own_cb.get();
    }
  }
  if (cb) {
    // Fused coarse mode: every outer iteration runs each solve's part before
    // its coarsest-level solve on its own stream, then the coarsest-level
    // solves of all solves together (one launch per coarse iteration over the
    // concatenated levels), then each solve's part after it.
    int it = 0;
    while (left > 0) {
      for (int k = 0; k < na; ++k) {
        if (runs[k].finished) continue;
        sv[k]->launch_pre();
        IPDG_HIP(hipEventRecord(cb->ev[k], sv[k]->stream()));
        IPDG_HIP(hipStreamWaitEvent(cb->stream, cb->ev[k], 0));
      }
      IPDG_HIP(hipGraphLaunch(cb->graph, cb->stream));
      IPDG_HIP(hipEventRecord(cb->ev_done, cb->stream));
      for (int k = 0; k < na; ++k) {
        if (runs[k].finished) continue;
        IPDG_HIP(hipStreamWaitEvent(sv[k]->stream(), cb->ev_done, 0));
        sv[k]->launch_post();
      }
      if (++it % every != 0) continue;
      for (int k = 0; k < na; ++k)
        if (!runs[k].finished) sv[k]->copy_scal();
      for (int k = 0; k < na; ++k) IPDG_HIP(hipStreamSynchronize(sv[k]->stream()));
      IPDG_HIP(hipStreamSynchronize(cb->stream));
      left = 0;
      for (int k = 0; k < na; ++k)
        if (!runs[k].finished) left += !sv[k]->after_step(runs[k]);
    }
    IPDG_HIP(hipStreamSynchronize(cb->stream));
  }
  // Otherwise each solve replays its own captured graph of `every`
  // iterations on its own stream; the launches of all unfinished solves are
  // issued before any is waited for, so the device runs the solves' small
  // kernels concurrently (one stream per solve, spread over the hardware
  // queues).
  while (left > 0) {
    for (int k = 0; k < na; ++k)
      if (!runs[k].finished) sv[k]->launch_iterations(every);
    for (int k = 0; k < na; ++k)
      if (!runs[k].finished) sv[k]->copy_scal();
    for (int k = 0; k < na; ++k) IPDG_HIP(hipStreamSynchronize(sv[k]->stream()));
    left = 0;
    for (int k = 0; k < na; ++k)
      if (!runs[k].finished) left += !sv[k]->after_step(runs[k]);
    // residual replacements were enqueued on the solves' own streams and run
    // before their next graph launch (same stream)
  }
  ipdg_status worst = IPDG_OK;
  for (int k = 0; k < na; ++k) {
    ipdg_solve_info info{};
    sv[k]->finish(runs[k], &info);
    if (iters) iters[active[k]] = info.iters;
    if (relres) relres[active[k]] = info.relres;
    if (runs[k].status != IPDG_OK) worst = runs[k].status;
  }
  for (int i = 0; i < nb; ++i)
    if (meshes[i]->host.K == 0) {
      if (iters) iters[i] = 0;
      if (relres) relres[i] = 0.0;
    }
  return worst;
}

}  // namespace ipdg
