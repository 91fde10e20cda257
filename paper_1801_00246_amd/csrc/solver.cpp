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

#include "amg.hpp"
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

constexpr int kAmgMaxLevels = 12;     // levels of the algebraic hierarchy, the degree-1 level included
constexpr int kAmgMaxCoarse = 2048;   // largest coarsest level (inverted densely on the host)

// Algebraic levels below the degree-1 level (pMG-AMG, Sec. 3).  Level 0 is
// the degree-1 p-multigrid level itself (matrix-free); level 1 holds one
// value per element; further levels one per aggregate.
// Two flexible-CG steps on one level (the K-cycle's coarse correction): the
// two inner cycles' results, their products with A, the second residual, the
// combined correction and the scalars (KScal)
struct KBufs {
  DevBuf v1, w1, r2, v2, w2, ec, s;
};
struct AmgLevel {
  int n = 0;
  double rho = 0;                  // Gershgorin bound of D^-1 A
  DevBuf ptr, col, val, dinv;      // A in compressed rows (level precision)
  DevBuf f, z, t, r, d;            // cycle work
  KBufs k;                         // K-cycle steps on this level
};
constexpr double kKcycleT = 0.25;   // second K-cycle step only while |r2| > 0.25 |rc|
struct AmgXfer {                   // level l -> l + 1
  int n = 0, nc = 0;
  DevBuf agg, mptr, mem;           // aggregate of each node; members of each aggregate
};
struct AmgSet {
  std::vector<int> sizes;          // unknowns per level, the degree-1 level first
  std::vector<AmgLevel> lv;        // lv[0] unused (the degree-1 level is the p-level)
  std::vector<AmgXfer> xf;
  DevBuf inv;                      // inverse of the coarsest matrix (dense, level precision)
  DevBuf t0, res0, z0;             // degree-1 work of repeated cycles
  KBufs k0;                        // the flexible-CG steps on the degree-1 level (amg_top_krylov)
};

struct Work : SolverWork {
  // configuration the setup was built for
  double lambda = NAN, ctau = NAN;
  int pc = -1, prec = -1, cheb_degree = 0, coarse_max = 0, nlev = 0, rho_steps = 0;
  double cheb_lo = 0, cheb_hi = 0, coarse_tol = 0;
  int coarse_amg = 0, amg_coarse_size = 0, amg_cycles = 0, amg_kcycle = 0, amg_top = 0;
  std::unique_ptr<AmgSet> amg;
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
  // right-hand side and solution of the coarsest-level solve, as recorded
  // for a fused batch
  const void* coarse_f = nullptr;
  void* coarse_x = nullptr;
  unsigned long long setup_id = 0;   // changes with every new setup (never reused)

  void drop_main() {
    if (graph) (void)hipGraphExecDestroy(graph);
    graph = nullptr;
    graph_iters = 0;
  }
  void drop_graph() {
    drop_main();
    coarse_f = nullptr;
    coarse_x = nullptr;
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

// One launch of an outer iteration, recorded for a fused batch (several
// solves advanced by shared launches): the arguments of the solve's own
// launch, its grid and, for element kernels, that grid's die stride.
enum class OpType { kAx, kAxDirect, kMinv, kTransfer, kVec, kCoarse };
struct BatchOp {
  OpType type = OpType::kVec;
  int N = 0, Nc = 0;
  Kind kind = Kind::F64;
  bool kap = false, restrict_op = false;
  int variant = 0;                 // operator variant (kAx)
  VecOp vop = VecOp::kUpdate;
  bool fp32 = false, flag = false;
  ElemArgs ea;
  TransferArgs ta;
  VecArgs va;
  int nb = 0, per = 0;
};

// Whether two recorded launches can share one batched launch (the same
// kernel; an operator variant without a batched form never shares).
bool same_launch(const BatchOp& a, const BatchOp& b) {
  if (a.type != b.type) return false;
  switch (a.type) {
    case OpType::kAx: return a.N == b.N && a.kind == b.kind && a.kap == b.kap && a.variant == b.variant;
    case OpType::kAxDirect: return false;
    case OpType::kMinv: return a.N == b.N && a.kind == b.kind;
    case OpType::kTransfer:
      return a.N == b.N && a.Nc == b.Nc && a.kind == b.kind && a.restrict_op == b.restrict_op;
    case OpType::kVec: return a.vop == b.vop && a.fp32 == b.fp32 && a.flag == b.flag;
    case OpType::kCoarse: return a.N == b.N && a.kind == b.kind;
  }
  return false;
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

  // Fused batch: one outer iteration's launches recorded into ops instead of
  // issued (the coarsest-level solve as one kCoarse op whose right-hand side
  // and solution buffers coarse_rhs() and coarse_sol() name).
  void record_iteration(std::vector<BatchOp>& ops) {
    rec_ = &ops;
    try {
      iteration(w_->xw.as<double>());
    } catch (...) {
      rec_ = nullptr;
      throw;
    }
    rec_ = nullptr;
  }
  const CGScal* scal_dev() const { return w_->scal.as<CGScal>(); }
  void set_host_scal(const CGScal& c) { *w_->host_scal = c; }
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
  const Level& coarsest() const { return w_->lv.back(); }
  const void* coarse_rhs() const { return w_->coarse_f; }
  void* coarse_sol() const { return w_->coarse_x; }
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
      if (o_.coarse_amg != 0 && o_.coarse_amg != 1) throw Error(IPDG_EINVAL, "coarse_amg must be 0 or 1");
      if (o_.coarse_amg == 1) {
        if (o_.amg_kcycle_levels < 0) throw Error(IPDG_EINVAL, "amg_kcycle_levels < 0");
        if (o_.amg_top_krylov != 0 && o_.amg_top_krylov != 1)
          throw Error(IPDG_EINVAL, "amg_top_krylov must be 0 or 1");
        if (o_.amg_top_krylov == 1 && o_.amg_cycles != 1)
          throw Error(IPDG_EINVAL, "amg_top_krylov takes one cycle per step (amg_cycles = 1)");
        if (o_.degrees[o_.n_levels - 1] != 1)
          throw Error(IPDG_EINVAL, "the algebraic levels start below degree 1: the last p-level must be 1");
        if (o_.amg_coarse_size < 1) throw Error(IPDG_EINVAL, "amg_coarse_size < 1");
        if (o_.amg_coarse_size > kAmgMaxCoarse)
          throw Error(IPDG_EINVAL, "amg_coarse_size above " + std::to_string(kAmgMaxCoarse));
        if (o_.amg_cycles < 1) throw Error(IPDG_EINVAL, "amg_cycles < 1");
      }
    }
  }

  // Launch helpers: issue the launch on the solver's stream, or, while an
  // iteration is being recorded, append it to the recorded ops.
  void op_ax(int N, Kind k, const ElemArgs& a) {
    if (!rec_) {
      IPDG_HIP(ax(N, k, a, s_));
      return;
    }
    BatchOp o;
    o.N = N;
    o.kind = k;
    o.ea = a;
    o.kap = a.kap != nullptr;
    const int v = ax_variant(N, k == Kind::F32);
    o.variant = v;
    if (!ax_batch_variant(v)) {
      o.type = OpType::kAxDirect;   // the LDS-staged variants have no batched form
    } else {
      o.type = OpType::kAx;
      if (v == kAxCoop) o.nb = xcd_grid((a.K + kCoopTileElems - 1) / kCoopTileElems, o.per);
      else o.nb = xcd_grid(elem_tiles(a.K), o.per);
    }
    rec_->push_back(o);
  }
  void op_minv(int N, Kind k, const ElemArgs& a) {
    if (!rec_) {
      IPDG_HIP(minv(N, k, a, s_));
      return;
    }
    BatchOp o;
    o.type = OpType::kMinv;
    o.N = N;
    o.kind = k;
    o.ea = a;
    o.nb = xcd_grid(elem_tiles(a.K), o.per);
    rec_->push_back(o);
  }
  void op_transfer(bool restrict_op, int Nf, int Nc, Kind k, const TransferArgs& t) {
    if (!rec_) {
      IPDG_HIP(restrict_op ? restrict_(Nf, Nc, k, t, s_) : prolong(Nf, Nc, k, t, s_));
      return;
    }
    BatchOp o;
    o.type = OpType::kTransfer;
    o.N = Nf;
    o.Nc = Nc;
    o.kind = k;
    o.restrict_op = restrict_op;
    o.ta = t;
    o.nb = xcd_grid(elem_tiles(t.K), o.per);
    rec_->push_back(o);
  }
  void push_vec(VecOp op, bool fp32, bool flag, const VecArgs& v, int nb) {
    BatchOp o;
    o.type = OpType::kVec;
    o.vop = op;
    o.fp32 = fp32;
    o.flag = flag;
    o.va = v;
    o.nb = nb;
    rec_->push_back(o);
  }
  void op_finalize(double* partials, int nparts, int nslots, CGScal* sc, int op) {
    if (!rec_) {
      IPDG_HIP(finalize(partials, nparts, nslots, sc, op, s_));
      return;
    }
    VecArgs v;
    v.a = partials;
    v.nparts = nparts;
    v.nslots = nslots;
    v.scw = sc;
    v.op = op;
    push_vec(VecOp::kFinalize, false, false, v, 1);
  }
  void op_convert(bool to_fp32, void* dst, const void* src, size_t n, const int* skip) {
    if (!rec_) {
      IPDG_HIP(convert(to_fp32, dst, src, n, skip, s_));
      return;
    }
    VecArgs v;
    v.x = dst;
    v.a = src;
    v.n = n;
    v.skip = skip;
    push_vec(VecOp::kConvert, false, to_fp32, v, flat_grid(n));
  }
  void op_update(bool fp32z, bool jac, double* x, double* r, const double* p, const double* Ap,
                 const double* dinv, void* z, const CGScal* sc, size_t n, double* partials) {
    if (!rec_) {
      IPDG_HIP(cg_update(fp32z, jac, x, r, p, Ap, dinv, z, sc, n, partials, s_));
      return;
    }
    VecArgs v;
    v.x = x;
    v.y = r;
    v.a = p;
    v.b = Ap;
    v.c = dinv;
    v.z = z;
    v.sc = sc;
    v.n = n;
    v.partials = partials;
    push_vec(VecOp::kUpdate, fp32z, jac, v, flat_grid(n));
  }
  void op_dots_rz(bool fp32z, const double* r, const void* z, const double* Ap, const CGScal* sc, size_t n,
                  double* partials) {
    if (!rec_) {
      IPDG_HIP(dots_rz(fp32z, r, z, Ap, sc, n, partials, s_));
      return;
    }
    VecArgs v;
    v.a = r;
    v.b = z;
    v.c = Ap;
    v.sc = sc;
    v.n = n;
    v.partials = partials;
    push_vec(VecOp::kDotsRz, fp32z, false, v, flat_grid(n));
  }
  void op_pupdate(bool fp32z, double* p, const void* z, const CGScal* sc, size_t n) {
    if (!rec_) {
      IPDG_HIP(pupdate(fp32z, p, z, sc, n, s_));
      return;
    }
    VecArgs v;
    v.x = p;
    v.a = z;
    v.sc = sc;
    v.n = n;
    push_vec(VecOp::kPupdate, fp32z, false, v, flat_grid(n));
  }
  void op_jacobi(bool fp32z, const double* r, const double* dinv, void* z, size_t n) {
    if (!rec_) {
      IPDG_HIP(jacobi(fp32z, r, dinv, z, n, s_));
      return;
    }
    VecArgs v;
    v.a = r;
    v.b = dinv;
    v.z = z;
    v.n = n;
    push_vec(VecOp::kJacobi, fp32z, false, v, flat_grid(n));
  }
  void op_cheb(bool fp32, int mode, const void* f, const void* t, const void* dinv, void* z, void* d, void* r,
               double c0, double c1, double c2, size_t n, const int* skip) {
    if (!rec_) {
      IPDG_HIP(cheb(fp32, mode, f, t, dinv, z, d, r, c0, c1, c2, n, skip, s_));
      return;
    }
    VecArgs v;
    v.mode = mode;
    v.a = f;
    v.b = t;
    v.c = dinv;
    v.z = z;
    v.x = d;
    v.y = r;
    v.c0 = c0;
    v.c1 = c1;
    v.c2 = c2;
    v.n = n;
    v.skip = skip;
    push_vec(VecOp::kCheb, fp32, false, v, flat_grid(n));
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
          w.coarse_tol != o_.coarse_tol || w.rho_steps != o_.rho_steps || w.coarse_amg != o_.coarse_amg ||
          (o_.coarse_amg && (w.amg_coarse_size != o_.amg_coarse_size || w.amg_cycles != o_.amg_cycles ||
                             w.amg_kcycle != o_.amg_kcycle_levels || w.amg_top != o_.amg_top_krylov)))
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
    w.amg.reset();
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
    w.coarse_amg = o_.pc == IPDG_PC_PMG ? o_.coarse_amg : 0;
    w.amg_coarse_size = o_.amg_coarse_size;
    w.amg_cycles = o_.amg_cycles;
    w.amg_kcycle = o_.amg_kcycle_levels;
    w.amg_top = o_.amg_top_krylov;
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
    if (o_.coarse_amg == 1) setup_amg();
    select_coarse();
  }

  // The algebraic levels (see AmgSet): the element-level matrix P0^T A P0
  // read off the degree-1 operator, then aggregation, Galerkin products and
  // Gershgorin bounds until at most amg_coarse_size unknowns remain (or 12
  // levels, counting the degree-1 level, or aggregation stalls); the
  // coarsest matrix is inverted.
  void setup_amg() {
    Work& w = *w_;
    const Level& v = w.lv.back();
    const HostMesh& hm = m_->host;
    const int K = K_;
    std::unique_ptr<AmgSet> A(new AmgSet);
    // element graph through interior faces
    std::vector<int> gptr(K + 1, 0), gadj;
    for (int e = 0; e < K; ++e) {
      int nb[3], c = 0;
      for (int f = 0; f < 3; ++f) {
        const int o = hm.EToE[3 * e + f];
        if (o >= 0 && o != e) nb[c++] = o;
      }
      std::sort(nb, nb + c);
      c = int(std::unique(nb, nb + c) - nb);
      for (int k = 0; k < c; ++k) gadj.push_back(nb[k]);
      gptr[e + 1] = int(gadj.size());
    }
    const Csr AE = element_matrix(v, gptr, gadj);
    A->sizes = {int(v.n), K};
    std::vector<Csr> mats{AE};
    std::vector<std::vector<int>> aggs;
    Csr cur = AE;
    for (;;) {
      if (cur.n <= o_.amg_coarse_size || int(A->sizes.size()) >= kAmgMaxLevels) break;
      std::vector<int> agg;
      const int na = amg_aggregate(gptr, gadj, agg);
      if (na == cur.n) break;
      std::vector<int> cptr, cadj;
      amg_coarse_graph(gptr, gadj, agg, na, cptr, cadj);
      cur = amg_galerkin(cur, agg, na);
      aggs.push_back(std::move(agg));
      gptr.swap(cptr);
      gadj.swap(cadj);
      mats.push_back(cur);
      A->sizes.push_back(na);
    }
    const int L = int(A->sizes.size());
    const bool f32 = v.fp32;
    const size_t w8 = f32 ? 4 : 8;
    auto upload = [&](DevBuf& b, const void* src, size_t bytes) {
      b.ensure(std::max<size_t>(bytes, 16));
      if (bytes) IPDG_HIP(hipMemcpyAsync(b.get(), src, bytes, hipMemcpyHostToDevice, s_));
    };
    auto upload_t = [&](DevBuf& b, const std::vector<double>& src) {
      if (f32) {
        std::vector<float> t(src.begin(), src.end());
        upload(b, t.data(), t.size() * 4);
        IPDG_HIP(hipStreamSynchronize(s_));
      } else {
        upload(b, src.data(), src.size() * 8);
      }
    };
    A->lv.resize(L);
    for (int l = 1; l < L; ++l) {
      AmgLevel& a = A->lv[l];
      const Csr& M = mats[l - 1];
      a.n = M.n;
      a.f.ensure(a.n * w8);
      a.z.ensure(a.n * w8);
      if (l == L - 1) continue;   // the coarsest level is solved by its inverse
      a.rho = amg_gershgorin(M);
      std::vector<double> dinv(M.n, 0.0);
      for (int i = 0; i < M.n; ++i)
        for (int k = M.ptr[i]; k < M.ptr[i + 1]; ++k)
          if (M.col[k] == i) dinv[i] = 1.0 / M.val[k];
      upload(a.ptr, M.ptr.data(), M.ptr.size() * 4);
      upload(a.col, M.col.data(), M.col.size() * 4);
      upload_t(a.val, M.val);
      upload_t(a.dinv, dinv);
      for (DevBuf* b : {&a.t, &a.r, &a.d}) b->ensure(a.n * w8);
    }
    // K-cycle corrections: level l < amg_kcycle_levels whose next level is
    // not the coarsest corrects from level l + 1 by two flexible-CG steps
    auto kbufs = [&](KBufs& k, size_t n) {
      for (DevBuf* b : {&k.v1, &k.w1, &k.r2, &k.v2, &k.w2, &k.ec}) b->ensure(n * w8);
      k.s.ensure(sizeof(KScal));
    };
    for (int l = 0; l < o_.amg_kcycle_levels && l + 2 < L; ++l) kbufs(A->lv[l + 1].k, A->lv[l + 1].n);
    if (o_.amg_top_krylov) kbufs(A->k0, v.n);
    // transfers: degree-1 nodes -> elements (node j of element j / Np), then
    // the aggregates
    A->xf.resize(L - 1);
    for (int l = 0; l + 1 < L; ++l) {
      AmgXfer& x = A->xf[l];
      x.n = A->sizes[l];
      x.nc = A->sizes[l + 1];
      std::vector<int> agg(x.n);
      if (l == 0) {
        for (int j = 0; j < x.n; ++j) agg[j] = j / v.Np;
      } else {
        agg = aggs[l - 1];
      }
      std::vector<int> mptr(x.nc + 1, 0), mem(x.n);
      for (int j = 0; j < x.n; ++j) ++mptr[agg[j] + 1];
      for (int i = 0; i < x.nc; ++i) mptr[i + 1] += mptr[i];
      std::vector<int> fill(mptr.begin(), mptr.end() - 1);
      for (int j = 0; j < x.n; ++j) mem[fill[agg[j]]++] = j;   // members ascending
      upload(x.agg, agg.data(), agg.size() * 4);
      upload(x.mptr, mptr.data(), mptr.size() * 4);
      upload(x.mem, mem.data(), mem.size() * 4);
      IPDG_HIP(hipStreamSynchronize(s_));
    }
    std::vector<double> inv;
    if (!amg_spd_inverse(mats.back(), inv))
      throw Error(IPDG_EUNSUPPORTED, "the coarsest algebraic level is not positive definite (a pure Neumann "
                                     "problem with lambda = 0 has constants in its null space)");
    upload_t(A->inv, inv);
    if (o_.amg_cycles > 1)
      for (DevBuf* b : {&A->t0, &A->res0, &A->z0}) b->ensure(v.n * w8);
    IPDG_HIP(hipStreamSynchronize(s_));
    w.amg = std::move(A);
  }

  // P0^T A P0 of the degree-1 operator (P0: one value per element to its
  // nodes), read off operator applications: elements whose closed
  // neighbourhoods are disjoint (a distance-2 colouring) are probed together
  // with x = 1 on their nodes; A x on element e' of the neighbourhood of a
  // probed element e, summed over the nodes of e', is entry (e', e).
  Csr element_matrix(const Level& v, const std::vector<int>& gptr, const std::vector<int>& gadj) {
    const int K = K_, Np = v.Np;
    std::vector<int> color(K, -1), mark;
    int ncol = 0;
    for (int e = 0; e < K; ++e) {
      mark.clear();
      for (int k = gptr[e]; k < gptr[e + 1]; ++k) {
        const int a = gadj[k];
        if (color[a] >= 0) mark.push_back(color[a]);
        for (int q = gptr[a]; q < gptr[a + 1]; ++q)
          if (color[gadj[q]] >= 0) mark.push_back(color[gadj[q]]);
      }
      std::sort(mark.begin(), mark.end());
      int c = 0;
      for (int m : mark)
        if (m == c) ++c;
        else if (m > c) break;
      color[e] = c;
      ncol = std::max(ncol, c + 1);
    }
    const size_t n = v.n;
    DevBuf xb(n * 8), yb(n * 8);
    std::vector<double> x(n), y(n);
    std::vector<std::vector<std::pair<int, double>>> rows(K);
    ElemArgs a = elem_args(m_, 1, Kind::F64, lambda_, v.ctau);
    a.x = xb.get();
    a.y = yb.get();
    for (int c = 0; c < ncol; ++c) {
      std::fill(x.begin(), x.end(), 0.0);
      for (int e = 0; e < K; ++e)
        if (color[e] == c)
          for (int k = 0; k < Np; ++k) x[(size_t)e * Np + k] = 1.0;
      IPDG_HIP(hipMemcpyAsync(xb.get(), x.data(), n * 8, hipMemcpyHostToDevice, s_));
      IPDG_HIP(ax(1, Kind::F64, a, s_));
      IPDG_HIP(hipMemcpyAsync(y.data(), yb.get(), n * 8, hipMemcpyDeviceToHost, s_));
      IPDG_HIP(hipStreamSynchronize(s_));
      for (int e = 0; e < K; ++e) {
        if (color[e] != c) continue;
        auto put = [&](int r) {
          double sum = 0.0;
          for (int k = 0; k < Np; ++k) sum += y[(size_t)r * Np + k];
          rows[r].emplace_back(e, sum);
        };
        put(e);
        for (int k = gptr[e]; k < gptr[e + 1]; ++k) put(gadj[k]);
      }
    }
    Csr M;
    M.n = K;
    M.ptr.assign(K + 1, 0);
    for (int r = 0; r < K; ++r) {
      std::sort(rows[r].begin(), rows[r].end());
      for (const auto& cv : rows[r]) {
        M.col.push_back(cv.first);
        M.val.push_back(cv.second);
      }
      M.ptr[r + 1] = int(M.col.size());
    }
    return M;
  }

  // persistent single-launch coarse solve or ordinary launches; a change
  // invalidates the captured iteration graph
  void select_coarse() {
    Work& w = *w_;
    if (o_.pc != IPDG_PC_PMG || w.lv.empty()) return;
    const Level& cl = w.lv.back();
    const int g = (persistent_ && o_.coarse_persistent == 1 && !w.amg) ? coarse_pcg_grid(cl.N, cl.kind, K_) : 0;
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
        op_jacobi(mixed_, w.r.as<double>(), w.dinv64.as<double>(), w.z.get(), n_);
        break;
      case IPDG_PC_BLOCK_MASS: {
        const Kind k = mixed_ ? Kind::F32_IN64 : Kind::F64;
        ElemArgs a = elem_args(m_, N_, k, 0.0, 0.0);
        a.x = w.r.get();
        a.y = w.z.get();
        a.skip = outer_done();
        op_minv(N_, k, a);
        break;
      }
      case IPDG_PC_PMG: {
        Level& v0 = w.lv[0];
        if (mixed_) op_convert(true, v0.f.get(), w.r.get(), n_, outer_done());
        vcycle(0, mixed_ ? v0.f.get() : w.r.get(), w.z.get());
        break;
      }
    }
  }

  void level_ax(const Level& v, const void* x, void* y, const int* skip = nullptr) {
    ElemArgs a = elem_args(m_, v.N, v.kind, lambda_, v.ctau);
    a.x = x;
    a.y = y;
    a.skip = skip ? skip : outer_done();
    op_ax(v.N, v.kind, a);
  }

  // Chebyshev smoothing of D^-1 A over [lo rho, hi rho] (Saad Alg. 12.1),
  // from zero or from z; apply(x, y) is y = A x on the level
  template <typename Apply>
  void cheb_smooth(bool fp32, double rho_l, size_t n, const void* dinv, void* d, void* r, void* t, const void* f,
                   void* z, bool from_zero, const int* skip, Apply apply) {
    const double lo = o_.cheb_lo * rho_l, hi = o_.cheb_hi * rho_l;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    double rho = 1.0 / sigma;
    if (from_zero) {
      op_cheb(fp32, 0, f, nullptr, dinv, z, d, r, 1.0 / theta, 0, 0, n, skip);
    } else {
      apply(z, t);
      op_cheb(fp32, 1, f, t, dinv, z, d, r, 1.0 / theta, 0, 0, n, skip);
    }
    for (int k = 1; k < o_.cheb_degree; ++k) {
      const double rho_new = 1.0 / (2.0 * sigma - rho);
      apply(d, t);
      op_cheb(fp32, 2, nullptr, t, dinv, z, d, r, 0, rho_new * rho, 2.0 * rho_new / delta, n, skip);
      rho = rho_new;
    }
  }

  void smooth(const Level& v, const void* f, void* z, bool from_zero, const int* skip = nullptr) {
    if (!skip) skip = outer_done();
    cheb_smooth(v.fp32, v.rho, v.n, v.dinv(), v.d.get(), v.r.get(), v.t.get(), f, z, from_zero, skip,
                [&](const void* x, void* y) { level_ax(v, x, y, skip); });
  }

  void amg_spmv_level(const AmgLevel& a, bool fp32, const void* x, void* y, const int* skip) {
    IPDG_HIP(amg_spmv(fp32, a.ptr.as<int>(), a.col.as<int>(), a.val.get(), x, y, a.n, skip, s_));
  }

  // One cycle of the algebraic hierarchy from zero on level l (0: the
  // degree-1 level), the same smoother before and after the coarse
  // correction, the coarsest level solved by its inverse.  On the first
  // amg_kcycle_levels levels (while the next level is not the coarsest) the
  // coarse correction is the K-cycle's two flexible-CG steps on the next
  // level, each preconditioned by one cycle there (the second skipped when
  // the first already reduced the coarse residual to 0.25 of its norm);
  // below, a V-cycle.  Every launch is a no-op while *skip is set.
  void amg_cycle(int l, const void* f, void* z, const int* skip) {
    AmgSet& A = *w_->amg;
    const Level& v = w_->lv.back();
    const bool f32 = v.fp32;
    const int L = int(A.sizes.size());
    if (l == L - 1) {
      IPDG_HIP(amg_dense(f32, A.inv.get(), f, z, A.sizes[l], skip, s_));
      return;
    }
    const void* t;
    if (l == 0) {
      smooth(v, f, z, true, skip);
      level_ax(v, z, v.t.get(), skip);
      t = v.t.get();
    } else {
      AmgLevel& a = A.lv[l];
      cheb_smooth(f32, a.rho, a.n, a.dinv.get(), a.d.get(), a.r.get(), a.t.get(), f, z, true, skip,
                  [&](const void* x, void* y) { amg_spmv_level(a, f32, x, y, skip); });
      amg_spmv_level(a, f32, z, a.t.get(), skip);
      t = a.t.get();
    }
    AmgLevel& c = A.lv[l + 1];
    const AmgXfer& x = A.xf[l];
    IPDG_HIP(amg_restrict(f32, x.mptr.as<int>(), x.mem.as<int>(), f, t, c.f.get(), x.nc, skip, s_));
    const void* ec = c.z.get();
    if (l < o_.amg_kcycle_levels && l + 2 < L) {
      krylov_step(l + 1, c.f.get(), c.k.ec.get(), skip);
      ec = c.k.ec.get();
    } else {
      amg_cycle(l + 1, c.f.get(), c.z.get(), skip);
    }
    IPDG_HIP(amg_prolong(f32, x.agg.as<int>(), ec, z, x.n, skip, s_));
    if (l == 0) {
      smooth(v, f, z, false, skip);
    } else {
      AmgLevel& a = A.lv[l];
      cheb_smooth(f32, a.rho, a.n, a.dinv.get(), a.d.get(), a.r.get(), a.t.get(), f, z, false, skip,
                  [&](const void* x, void* y) { amg_spmv_level(a, f32, x, y, skip); });
    }
  }

  // Approximate solution of A_lk e = rc on level lk (0: the degree-1 level)
  // by two flexible-CG steps from zero, each preconditioned by one cycle on
  // that level; the second step is skipped (device flag) once the first
  // reduced |rc| to 0.25 of its norm or less.
  void krylov_step(int lk, const void* rc, void* e, const int* skip) {
    AmgSet& A = *w_->amg;
    const Level& v = w_->lv.back();
    const bool f32 = v.fp32;
    KBufs& B = lk == 0 ? A.k0 : A.lv[lk].k;
    const int n = A.sizes[lk];
    auto apply = [&](const void* x, void* y, const int* sk) {
      if (lk == 0) level_ax(v, x, y, sk);
      else amg_spmv_level(A.lv[lk], f32, x, y, sk);
    };
    KScal* S = B.s.as<KScal>();
    const int* second = &S->flag;
    amg_cycle(lk, rc, B.v1.get(), skip);
    apply(B.v1.get(), B.w1.get(), skip);
    IPDG_HIP(amg_kdot1(f32, B.v1.get(), rc, B.w1.get(), n, S, skip, s_));
    IPDG_HIP(amg_kres(f32, rc, B.w1.get(), B.r2.get(), n, S, kKcycleT * kKcycleT, skip, s_));
    amg_cycle(lk, B.r2.get(), B.v2.get(), second);
    apply(B.v2.get(), B.w2.get(), second);
    IPDG_HIP(amg_kdot2(f32, B.v2.get(), B.w1.get(), B.w2.get(), B.r2.get(), n, S, s_));
    IPDG_HIP(amg_kcomb(f32, B.v1.get(), B.v2.get(), e, n, S, skip, s_));
  }

  // amg_cycles cycles on the degree-1 level: the first from zero, each
  // further one on the residual of the current x (iterative refinement)
  void amg_solve(const void* f, void* x) {
    AmgSet& A = *w_->amg;
    const Level& v = w_->lv.back();
    if (o_.amg_top_krylov) {
      krylov_step(0, f, x, outer_done());
      return;
    }
    amg_cycle(0, f, x, outer_done());
    for (int c = 1; c < o_.amg_cycles; ++c) {
      level_ax(v, x, A.t0.get());
      IPDG_HIP(amg_sub(v.fp32, f, A.t0.get(), A.res0.get(), v.n, outer_done(), s_));
      amg_cycle(0, A.res0.get(), A.z0.get(), outer_done());
      IPDG_HIP(amg_add(v.fp32, x, A.z0.get(), v.n, outer_done(), s_));
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
    op_transfer(true, v.N, c.N, v.kind, ta);
    vcycle(l + 1, c.f.get(), c.z.get());
    TransferArgs tp;
    tp.coarse = c.z.get();
    tp.fine = z;
    tp.P = v.P;
    tp.K = K_;
    tp.skip = outer_done();
    op_transfer(false, v.N, c.N, v.kind, tp);
    smooth(v, f, z, false);
  }

  // Jacobi-PCG from zero on the coarsest level, coarse_max iterations at most
  void coarse_solve(Level& v, const void* f, void* x) {
    Work& w = *w_;
    if (w.amg) {
      if (rec_) throw Error(IPDG_EUNSUPPORTED, "a fused batch solves its coarsest levels by Jacobi-PCG");
      amg_solve(f, x);
      return;
    }
    if (rec_) {
      // fused batch: the batch solves this level for all its solves at once
      w.coarse_f = f;
      w.coarse_x = x;
      BatchOp o;
      o.type = OpType::kCoarse;
      o.N = v.N;
      o.kind = v.kind;
      rec_->push_back(o);
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
      op_convert(true, w.p32.get(), w.p.get(), n_, outer_done());
      ElemArgs a = elem_args(m_, N_, Kind::F32, lambda_, ctau_);
      a.x = w.p32.get();
      a.y = w.Ap32.get();
      a.partials = w.partials.as<double>();
      a.skip = outer_done();
      op_ax(N_, Kind::F32, a);
      op_finalize(w.partials.as<double>(), ax_partials(N_, true, K_), 1, sc, kFinAlpha);
      op_convert(false, w.Ap.get(), w.Ap32.get(), n_, outer_done());
    } else {
      ElemArgs a = elem_args(m_, N_, Kind::F64, lambda_, ctau_);
      a.x = w.p.get();
      a.y = w.Ap.get();
      a.partials = w.partials.as<double>();
      a.skip = outer_done();
      op_ax(N_, Kind::F64, a);
      op_finalize(w.partials.as<double>(), ax_partials(N_, false, K_), 1, sc, kFinAlpha);
    }
    const bool jac = o_.pc == IPDG_PC_JACOBI || o_.pc == IPDG_PC_NONE;
    op_update(mixed_, jac, x, w.r.as<double>(), w.p.as<double>(), w.Ap.as<double>(), w.dinv64.as<double>(),
              w.z.get(), sc, n_, w.partials.as<double>());
    if (!jac) {
      precond();
      op_dots_rz(mixed_, w.r.as<double>(), w.z.get(), w.Ap.as<double>(), sc, n_, w.partials.as<double>());
    }
    op_finalize(w.partials.as<double>(), flat_grid(n_), 3, sc, kFinBeta);
    op_pupdate(mixed_, w.p.as<double>(), w.z.get(), sc, n_);
  }

  // status of the persistent coarse solve: [0] iterations, [1] barrier
  // timeout, [2] breakdown
  int coarse_status() {
    Work& w = *w_;
    if (o_.pc != IPDG_PC_PMG || w.lv.empty()) return -1;
    if (w.amg) return 0;
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
    info->precond_bytes = (int64_t)precond_bytes();
    if (w_->amg) {
      info->amg_levels = int(w_->amg->sizes.size());
      for (int l = 0; l < info->amg_levels && l < IPDG_AMG_MAX_LEVELS; ++l) info->amg_n[l] = w_->amg->sizes[l];
    }
    info->iters = iters;
    info->relres = relres;
    info->restarts = restarts;
    for (size_t l = 0; l < w_->lv.size() && l < IPDG_MAX_LEVELS; ++l) info->rho_used[l] = w_->lv[l].rho;
    info->setup_ms = w_->setup_ms;
    info->solve_ms = solve_ms;
  }

  // device bytes of the p-multigrid levels and the algebraic hierarchy
  size_t precond_bytes() const {
    const Work& w = *w_;
    size_t b = 0;
    for (const Level& v : w.lv)
      for (const DevBuf* d : {&v.dinv64, &v.dinv32, &v.f, &v.z, &v.r, &v.d, &v.t, &v.cr, &v.cr2, &v.cz, &v.cp,
                              &v.cp2, &v.cs2, &v.cAp, &v.cw2})
        b += d->size();
    if (w.amg) {
      const AmgSet& A = *w.amg;
      for (const DevBuf* d : {&A.inv, &A.t0, &A.res0, &A.z0, &A.k0.v1, &A.k0.w1, &A.k0.r2, &A.k0.v2, &A.k0.w2,
                              &A.k0.ec, &A.k0.s})
        b += d->size();
      for (const AmgLevel& a : A.lv)
        for (const DevBuf* d : {&a.ptr, &a.col, &a.val, &a.dinv, &a.f, &a.z, &a.t, &a.r, &a.d, &a.k.v1, &a.k.w1,
                                &a.k.r2, &a.k.v2, &a.k.w2, &a.k.ec, &a.k.s})
          b += d->size();
      for (const AmgXfer& x : A.xf)
        for (const DevBuf* d : {&x.agg, &x.mptr, &x.mem}) b += d->size();
    }
    return b;
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
  std::vector<BatchOp>* rec_ = nullptr;   // recording an iteration (fused batch)
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

// The coarsest levels of a batch's solves, concatenated (CoarseBatchArgs).
struct CoarseBatchSet {
  DevBuf ent, tile_solve, x, p, u, dinv, r0, r1, w0, w1, s0, s1, geo, conn, kap, partials, sc;
  CoarseBatchArgs a;
  int N = 0;
  Kind kind = Kind::F64;
  int max_iters = 0;               // the largest member cap: coarse launches per solve
};

// IPDG_BATCH=separate advances every solve of a batch on its own stream with
// its own launches (the fused form is the default).
bool batch_fused() {
  const char* v = std::getenv("IPDG_BATCH");
  return !(v && std::strcmp(v, "separate") == 0);
}

// Null when the solves' coarsest levels differ in degree or precision.
std::unique_ptr<CoarseBatchSet> make_coarse_batch(std::vector<std::unique_ptr<Solver>>& sv,
                                                  const ipdg_solve_opts& o, hipStream_t cs) {
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
  cb->N = Nc;
  cb->kind = kind;
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
  return cb;
}

// One launch of a fused batch: the recorded launches of several solves that
// share a kernel (their argument records and block map at the given arena
// offsets), a solve's own launch (an operator variant without a batched
// form), or the coarsest-level solves of all solves.
struct FusedStep {
  BatchOp proto;
  std::vector<BatchOp> ops;        // the members' recorded launches
  size_t tab_off = 0, map_off = 0;
  int nblocks = 0;
};

// Merge the solves' recorded launch sequences into shared launches.  Each
// solve keeps its own order; a step takes the next launch of the solve with
// the most launches left before its coarsest-level solve (so that solves
// with more levels run ahead until the others can join their launches) and
// every solve whose next launch has the same kernel; the coarsest-level
// solve runs when every solve has reached it.
std::vector<FusedStep> merge_launches(const std::vector<std::vector<BatchOp>>& ops) {
  const int na = int(ops.size());
  std::vector<size_t> pos(na, 0);
  std::vector<FusedStep> steps;
  auto before_coarse = [&](int k) {
    size_t j = pos[k];
    while (j < ops[k].size() && ops[k][j].type != OpType::kCoarse) ++j;
    return j - pos[k];
  };
  for (;;) {
    int lead = -1;
    size_t most = 0;
    int left = 0, at_coarse = 0;
    for (int k = 0; k < na; ++k) {
      if (pos[k] >= ops[k].size()) continue;
      ++left;
      const size_t r = before_coarse(k);
      if (r == 0) {
        ++at_coarse;
      } else if (lead < 0 || r > most) {
        lead = k;
        most = r;
      }
    }
    if (left == 0) break;
    FusedStep st;
    if (lead < 0) {
      if (at_coarse != na) throw Error(IPDG_EUNSUPPORTED, "the batch's solves reach their coarsest levels unevenly");
      st.proto = ops[0][pos[0]];
      for (int k = 0; k < na; ++k) {
        if (!same_launch(st.proto, ops[k][pos[k]]))
          throw Error(IPDG_EUNSUPPORTED, "the batch's coarsest levels differ in degree or precision");
        st.ops.push_back(ops[k][pos[k]]);
        ++pos[k];
      }
      steps.push_back(std::move(st));
      continue;
    }
    st.proto = ops[lead][pos[lead]];
    for (int k = 0; k < na; ++k) {
      if (pos[k] >= ops[k].size()) continue;
      if (k == lead || same_launch(st.proto, ops[k][pos[k]])) {
        st.ops.push_back(ops[k][pos[k]]);
        ++pos[k];
      }
    }
    steps.push_back(std::move(st));
  }
  return steps;
}

// A fused batch: `every` outer iterations of all its solves as one launch
// sequence (captured as one graph), followed by a gather of every solve's CG
// scalars for one copy to the host.
struct FusedBatch {
  std::unique_ptr<CoarseBatchSet> cb;
  std::vector<FusedStep> steps;
  DevBuf arena, scal_src, scal_all;
  CGScal* host = nullptr;          // pinned, one record per solve
  int na = 0, every = 0;
  hipStream_t stream = nullptr;
  hipGraphExec_t graph = nullptr;
  ~FusedBatch() {
    if (graph) (void)hipGraphExecDestroy(graph);
    if (stream) (void)hipStreamDestroy(stream);
    if (host) (void)hipHostFree(host);
  }

  void issue(hipStream_t s) const {
    const char* base = arena.as<char>();
    for (int it = 0; it < every; ++it)
      for (const FusedStep& st : steps) {
        const BatchOp& p = st.proto;
        const BlockRef* map = reinterpret_cast<const BlockRef*>(base + st.map_off);
        const void* tab = base + st.tab_off;
        switch (p.type) {
          case OpType::kAx:
            IPDG_HIP(ax_batch(p.N, p.kind, p.kap, p.variant, static_cast<const ElemArgs*>(tab), map, st.nblocks, s));
            break;
          case OpType::kAxDirect:
            IPDG_HIP(ax(p.N, p.kind, p.ea, s));
            break;
          case OpType::kMinv:
            IPDG_HIP(minv_batch(p.N, p.kind, static_cast<const ElemArgs*>(tab), map, st.nblocks, s));
            break;
          case OpType::kTransfer:
            IPDG_HIP(transfer_batch(p.N, p.Nc, p.restrict_op, p.kind, static_cast<const TransferArgs*>(tab), map,
                                    st.nblocks, s));
            break;
          case OpType::kVec:
            IPDG_HIP(vec_batch(p.vop, p.fp32, p.flag, static_cast<const VecArgs*>(tab), map, st.nblocks, s));
            break;
          case OpType::kCoarse:
            // start, the iterations up to the largest member cap, copy-out
            IPDG_HIP(coarse_batch(cb->N, cb->kind, cb->a, -1, s));
            for (int c = 0; c < cb->max_iters; ++c) IPDG_HIP(coarse_batch(cb->N, cb->kind, cb->a, c, s));
            IPDG_HIP(coarse_batch(cb->N, cb->kind, cb->a, -2, s));
            break;
        }
      }
    IPDG_HIP(scal_gather(scal_src.as<const CGScal* const>(), scal_all.as<CGScal>(), na, s));
  }

  // `every` iterations of every solve, then their scalars on the host
  void run(bool use_graph) {
    if (use_graph) IPDG_HIP(hipGraphLaunch(graph, stream));
    else issue(stream);
    IPDG_HIP(hipMemcpyAsync(host, scal_all.get(), na * sizeof(CGScal), hipMemcpyDeviceToHost, stream));
    IPDG_HIP(hipStreamSynchronize(stream));
  }
};

std::unique_ptr<FusedBatch> make_fused_batch(std::vector<std::unique_ptr<Solver>>& sv, const ipdg_solve_opts& o,
                                             int every, bool use_graph) {
  const int na = int(sv.size());
  std::unique_ptr<FusedBatch> fb(new FusedBatch);
  fb->na = na;
  fb->every = every;
  IPDG_HIP(hipStreamCreateWithFlags(&fb->stream, hipStreamNonBlocking));
  std::vector<std::vector<BatchOp>> ops(na);
  bool coarse = false;
  for (int k = 0; k < na; ++k) {
    sv[k]->record_iteration(ops[k]);
    for (const BatchOp& b : ops[k]) coarse = coarse || b.type == OpType::kCoarse;
  }
  if (coarse) {
    fb->cb = make_coarse_batch(sv, o, fb->stream);
    if (!fb->cb) return nullptr;
  }
  fb->steps = merge_launches(ops);
  // argument records and block maps of every shared launch, in one arena
  std::vector<char> img;
  auto put = [&img](const void* p, size_t bytes) {
    const size_t off = (img.size() + 63) / 64 * 64;
    img.resize(off + bytes);
    std::memcpy(img.data() + off, p, bytes);
    return off;
  };
  for (FusedStep& st : fb->steps) {
    const OpType t = st.proto.type;
    if (t == OpType::kCoarse || t == OpType::kAxDirect) continue;
    std::vector<BlockRef> map;
    for (size_t i = 0; i < st.ops.size(); ++i)
      for (int b = 0; b < st.ops[i].nb; ++b) map.push_back(BlockRef{int(i), b, st.ops[i].nb, st.ops[i].per});
    if (t == OpType::kAx || t == OpType::kMinv) {
      std::vector<ElemArgs> tab;
      for (const BatchOp& b : st.ops) tab.push_back(b.ea);
      st.tab_off = put(tab.data(), tab.size() * sizeof(ElemArgs));
    } else if (t == OpType::kTransfer) {
      std::vector<TransferArgs> tab;
      for (const BatchOp& b : st.ops) tab.push_back(b.ta);
      st.tab_off = put(tab.data(), tab.size() * sizeof(TransferArgs));
    } else {
      std::vector<VecArgs> tab;
      for (const BatchOp& b : st.ops) tab.push_back(b.va);
      st.tab_off = put(tab.data(), tab.size() * sizeof(VecArgs));
    }
    st.map_off = put(map.data(), map.size() * sizeof(BlockRef));
    st.nblocks = int(map.size());
  }
  fb->arena.alloc(std::max<size_t>(img.size(), 64));
  IPDG_HIP(hipMemcpyAsync(fb->arena.get(), img.data(), img.size(), hipMemcpyHostToDevice, fb->stream));
  std::vector<const CGScal*> src(na);
  for (int k = 0; k < na; ++k) src[k] = sv[k]->scal_dev();
  fb->scal_src.alloc(na * sizeof(const CGScal*));
  fb->scal_all.alloc(na * sizeof(CGScal));
  IPDG_HIP(hipMemcpyAsync(fb->scal_src.get(), src.data(), na * sizeof(const CGScal*), hipMemcpyHostToDevice,
                          fb->stream));
  IPDG_HIP(hipHostMalloc(reinterpret_cast<void**>(&fb->host), na * sizeof(CGScal), hipHostMallocDefault));
  IPDG_HIP(hipStreamSynchronize(fb->stream));
  if (use_graph) {
    hipGraph_t g = nullptr;
    IPDG_HIP(hipStreamBeginCapture(fb->stream, hipStreamCaptureModeThreadLocal));
    try {
      fb->issue(fb->stream);
    } catch (...) {
      (void)hipStreamEndCapture(fb->stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    IPDG_HIP(hipStreamEndCapture(fb->stream, &g));
    hipError_t e = hipGraphInstantiate(&fb->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    IPDG_HIP(e);
  }
  return fb;
}

// What a fused batch was built for: the solves' setups in batch order (ids
// are never reused, so a destroyed mesh never matches; a setup fixes every
// buffer and constant its launches name), the iterations per check, the
// operator variants in force, graph use and the device.
struct FusedKey {
  std::vector<unsigned long long> ids;
  std::vector<int> variants;
  int every = 0, device = -1;
  bool graph = true;
  bool operator==(const FusedKey& o) const {
    return ids == o.ids && variants == o.variants && every == o.every && device == o.device && graph == o.graph;
  }
};

FusedKey fused_key(const std::vector<std::unique_ptr<Solver>>& sv, int every, bool graph) {
  FusedKey k;
  for (const auto& s : sv) k.ids.push_back(s->setup_id());
  for (int N = 1; N <= kMaxN; ++N) {
    k.variants.push_back(ax_variant(N, false));
    k.variants.push_back(ax_variant(N, true));
  }
  k.every = every;
  k.graph = graph;
  (void)hipGetDevice(&k.device);
  return k;
}

// The last fused batch, reused by the next batch of the same solves (a
// serving loop); held until it is replaced (never freed at process exit,
// when the runtime may already be gone).
std::mutex g_fb_mu;
FusedBatch* g_fb = nullptr;
bool g_fb_valid = false;
FusedKey g_fb_key;

}  // namespace

ipdg_status solve_batch(int nb, ipdg_mesh_s* const* meshes, const double* lambdas, double tau,
                        const double* const* b, double* const* x, double tol, const ipdg_solve_opts& o,
                        int* iters, double* relres, hipStream_t s) {
  // Every solve keeps its own device state and stream; the host advances all
  // of them by check_every iterations per round.
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
  std::unique_ptr<FusedBatch> own_fb;
  FusedBatch* fb = nullptr;
  std::unique_lock<std::mutex> lk(g_fb_mu, std::defer_lock);
  const bool use_graph = std::getenv("IPDG_NO_GRAPH") == nullptr;
  if (left > 0 && na >= 2 && batch_fused() && !(o.pc == IPDG_PC_PMG && o.coarse_amg == 1)) {
    const FusedKey key = fused_key(sv, every, use_graph);
    if (lk.try_lock()) {
      if (!g_fb_valid || !(g_fb_key == key)) {
        delete g_fb;
        g_fb = nullptr;
        g_fb_valid = false;
        g_fb = make_fused_batch(sv, o, every, use_graph).release();
        g_fb_key = key;
        g_fb_valid = g_fb != nullptr;
      }
      fb = g_fb;
    } else {
      own_fb = make_fused_batch(sv, o, every, use_graph);   // another thread holds the cached batch
      fb = own_fb.get();
    }
  }
  if (fb) {
    // Fused mode: one launch per operation and kernel for all solves (a
    // finished solve's launches are no-ops on its done flag); residual
    // replacements and stops run on the solves' own streams in between.
    while (left > 0) {
      for (int k = 0; k < na; ++k) IPDG_HIP(hipStreamSynchronize(sv[k]->stream()));
      fb->run(use_graph);
      left = 0;
      for (int k = 0; k < na; ++k) {
        if (runs[k].finished) continue;
        sv[k]->set_host_scal(fb->host[k]);
        left += !sv[k]->after_step(runs[k]);
      }
    }
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
