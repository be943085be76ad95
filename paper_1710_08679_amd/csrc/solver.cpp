// Host side of the multi-case solver: Algorithm 1 of the paper.
//
//  (a) outer loop, FP64: flexible CG whose preconditioner is a rough inner
//      solve, stopped when max_j ||r_j|| / ||f_j|| <= tol;
//  (b) inner loops: block-Jacobi CG to a squared relative residual eps or N
//      steps, on the aggregates of the corners (level 2, MG3 only), then on
//      the linear mesh made of the corners (level 1), then on the quadratic
//      mesh (level 0), in FP32 (MIXED) or FP64.
//  PCGE (Section 4) is the outer loop with z = M^-1 r instead of lines 8-17.
//
// All per-case scalars live on the device (solver_kernels.hip).  The host
// enqueues iterations and reads the loop flags after a few of them; kernels
// enqueued past convergence see the cleared flag and return at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "ebe_internal.h"
#include "solver_state.h"

using namespace ebe;

namespace {

constexpr int kMaxBlocks = 1024;

struct Bufs {
  double *r, *p, *q;  // outer, [N][3][n] FP64
  void *rb, *ub, *e0, *p0, *q0;  // level 0
  void *r1, *u1, *e1, *p1, *q1;  // level 1
  void *r2, *u2, *e2, *p2, *q2;  // level 2
};

ebe_status ensure_workspace(ebe_mesh* m, int nr) {
  Workspace& w = m->ws;
  const size_t v0 = size_t(m->n_nodes) * 3 * nr * sizeof(double);
  const size_t v1 = size_t(m->n_vertices) * 3 * nr * sizeof(double);
  ebe_status st = EBE_OK;
  DBuf* outer[] = {&w.r, &w.p, &w.q, &w.rb, &w.ub, &w.e0, &w.p0, &w.q0};
  for (DBuf* b : outer)
    if ((st = b->alloc(v0)) != EBE_OK) return st;
  DBuf* coarse[] = {&w.r1, &w.u1, &w.e1, &w.p1, &w.q1};
  for (DBuf* b : coarse)
    if ((st = b->alloc(v1)) != EBE_OK) return st;
  const size_t v2 = size_t(std::max<int64_t>(m->n_agg, 1)) * 3 * nr * sizeof(double);
  DBuf* agg[] = {&w.r2, &w.u2, &w.e2, &w.p2, &w.q2};
  for (DBuf* b : agg)
    if ((st = b->alloc(v2)) != EBE_OK) return st;
  if ((st = w.scal.alloc(sizeof(SolverScalars))) != EBE_OK) return st;
  if ((st = w.partials.alloc(size_t(kMaxBlocks) * 3 * EBE_MAX_RHS * sizeof(double))) != EBE_OK) return st;
  if ((st = w.counter.alloc(64)) != EBE_OK) return st;
  if (!w.host_flags) {
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&w.host_flags), sizeof(SolverScalars), 0);
    if (e != hipSuccess) {
      w.host_flags = nullptr;
      set_error("hipHostMalloc failed: %s", hipGetErrorString(e));
      return EBE_ERR_OOM;
    }
  }
  w.nrhs_cap = std::max(w.nrhs_cap, nr);
  return EBE_OK;
}

// Copy the scalar block to pinned host memory and wait for the stream.
ebe_status read_scalars(ebe_mesh* m, hipStream_t s, SolverScalars** out) {
  SolverScalars* h = reinterpret_cast<SolverScalars*>(m->ws.host_flags);
  EBE_TRY_HIP(hipMemcpyAsync(h, m->ws.scal.as<void>(), sizeof(SolverScalars), hipMemcpyDeviceToHost, s));
  EBE_TRY_HIP(hipStreamSynchronize(s));
  *out = h;
  return EBE_OK;
}

#define EBE_K(call)                                        \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) {                                \
      set_error("%s: %s", #call, hipGetErrorString(e_));   \
      return EBE_ERR_HIP;                                  \
    }                                                      \
  } while (0)

template <typename T>
constexpr ebe_dtype dtype_of() {
  return sizeof(T) == 8 ? EBE_F64 : EBE_F32;
}

constexpr size_t kMaxGraphs = 24;

// Enqueue a fixed run of solver steps on s: directly, or (graphs on, s not
// the legacy default stream) by replaying a graph captured from the same run
// the first time it is met.  key holds everything the run's kernels take as
// arguments, and the product forms that pick those kernels, so a replay is
// exactly the run it stands for.
template <class Steps>
ebe_status enqueue_steps(ebe_mesh* m, std::vector<uintptr_t>&& key, bool graphs, hipStream_t s, Steps&& steps) {
  if (!graphs || s == nullptr) return steps();
  auto& G = m->ws.graphs;
  for (auto& g : G)
    if (g.key == key) {
      EBE_TRY_HIP(hipGraphLaunch(g.exec, s));
      return EBE_OK;
    }
  if (G.size() >= kMaxGraphs) {
    for (auto& g : G) (void)hipGraphExecDestroy(g.exec);
    G.clear();
  }
  EBE_TRY_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  const ebe_status st = steps();
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(s, &graph);
  if (st != EBE_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    if (st != EBE_OK) return st;
    set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e));
    return EBE_ERR_HIP;
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    set_error("hipGraphInstantiate failed: %s", hipGetErrorString(e));
    return EBE_ERR_HIP;
  }
  G.push_back(Workspace::Graph{std::move(key), exec});
  ++m->ws.captures;
  EBE_TRY_HIP(hipGraphLaunch(exec, s));
  return EBE_OK;
}

uintptr_t bits_of(double v) {
  uintptr_t b = 0;
  std::memcpy(&b, &v, sizeof(v) < sizeof(b) ? sizeof(v) : sizeof(b));
  return b;
}

uintptr_t addr(const void* p) { return reinterpret_cast<uintptr_t>(p); }

// Algorithm 1(b) on one level: approximately solve A u = r starting from u.
// The level's operator: EBE products on levels 0 and 1, the assembled A2 on level 2.
// det (deterministic solves): products whose sums have a fixed order (the
// deterministic form on the quadratic level, the assembled operators on the
// coarse levels), and (x, K x) summed by a node-case pass in a fixed order
// instead of inside the product (whose cross-workgroup fold uses atomics).
template <typename T>
hipError_t level_product(const ebe_mesh* m, int level, int nr, const T* x, T* y, const int* gate, hipStream_t s,
                         double* gamma = nullptr, bool half = false, bool det = false,
                         SolverState* st = nullptr) {
  // all solver vectors are kept zero on fixed DOFs, so inputs need no masking
  double* g = det ? nullptr : gamma;
  auto then_dot = [&](hipError_t e) -> hipError_t {
    if (e != hipSuccess || !det || !gamma) return e;
    return sk_dot<T>(m, level, x, y, nr, gamma, gate, *st, s);
  };
  if constexpr (sizeof(T) == 4) {
    if (half && level >= 1) return then_dot(launch_asm_half(m, level, nr, x, y, false, true, false, gate, s, g));
  }
  if (level == 2) return then_dot(launch_level2(m, dtype_of<T>(), nr, x, y, false, true, false, gate, s, g));
  if (det)
    return then_dot(launch_ebe_form(m, level == 0 ? 2 : 1, level == 0 ? EBE_FORM_DETERMINISTIC : EBE_FORM_ASSEMBLED,
                                    dtype_of<T>(), nr, x, y, false, true, false, gate, s, nullptr));
  return then_dot(launch_ebe(m, level == 0 ? 2 : 1, dtype_of<T>(), nr, x, y, false, true, false, gate, s, g));
}

template <typename T>
ebe_status inner_solve(ebe_mesh* m, int level, T* r, T* u, T* e, T* p, T* q, int nr, double eps, int nmax,
                       bool graphs, bool half, bool det, SolverState& st, hipStream_t s) {
  InnerScalars* din = &st.sc->inner[level];
  half = half && sizeof(T) == 4 && level >= 1;
  EBE_K(level_product<T>(m, level, nr, u, q, &st.sc->outer_active, s, nullptr, half, det, &st));
  EBE_K(sk_inner_init<T>(m, level, r, q, e, nr, eps, nmax, st, s));
  int enq = 0;
  int chunk = level == 0 ? 3 : (level == 1 ? 4 : 8);
  while (enq < nmax - 1) {
    const int k = std::min(chunk, nmax - 1 - enq);
    const void* data = level == 2 ? m->a2.val[sizeof(T) == 8 ? 0 : 1].as<void>() : m->pl[level].stage.as<void>();
    const uintptr_t form = (half ? uintptr_t(64)  // the FP16 assembled operator
                                 : (level == 2 ? uintptr_t(EBE_FORM_ASSEMBLED)
                                               : (det ? uintptr_t(level == 0 ? EBE_FORM_DETERMINISTIC
                                                                             : EBE_FORM_ASSEMBLED) |
                                                            (uintptr_t(m->fvar[0][sizeof(T) == 8 ? 0 : 1][nr]) << 8)
                                                      : product_key(m, level == 0 ? 2 : 1, dtype_of<T>(), nr)))) |
                           (det ? uintptr_t(1) << 16 : 0);
    ebe_status rs = enqueue_steps(
        m,
        {1, uintptr_t(level), uintptr_t(k), uintptr_t(nr), sizeof(T), uintptr_t(form), addr(e), addr(p), addr(q),
         addr(u),
         addr(st.sc), addr(st.partials), addr(st.counter), addr(data), addr(m->gacc.as<void>()),
         addr(m->minv64[level].as<void>()), addr(m->minv32[level].as<void>()), bits_of(eps), uintptr_t(nmax)},
        graphs, s, [&]() -> ebe_status {
          for (int c = 0; c < k; ++c) {
            EBE_K(sk_inner_p<T>(m, level, e, p, q, nr, st, s));
            EBE_K(level_product<T>(m, level, nr, p, q, &din->active, s, din->gamma, half, det, &st));
            EBE_K(sk_inner_update<T>(m, level, e, u, q, p, nr, eps, nmax, st, s));
          }
          return EBE_OK;
        });
    if (rs != EBE_OK) return rs;
    enq += k;
    SolverScalars* h = nullptr;
    rs = read_scalars(m, s, &h);
    if (rs != EBE_OK) return rs;
    if (!h->inner[level].active) break;
    chunk = std::min(chunk * 2, level == 2 ? 64 : 32);
  }
  return EBE_OK;
}

// Lines 9-18 of Algorithm 1(a): z from r through the inner levels (2 when
// MG3), 1 and 0, then the new search direction p from z.
template <typename T>
ebe_status mg_precondition(ebe_mesh* m, int nr, const ebe_pcg_opts& o, const Bufs& b, SolverState& st,
                           hipStream_t s) {
  T* rb = static_cast<T*>(b.rb);
  T* ub = static_cast<T*>(b.ub);
  T* r1 = static_cast<T*>(b.r1);
  T* u1 = static_cast<T*>(b.u1);
  const ebe_dtype dt = dtype_of<T>();
  EBE_K(sk_cast_bj<T>(m, b.r, rb, ub, nr, st, s));            // r_bar <= r ; u_bar <= M0^-1 r_bar
  EBE_K(launch_restrict(m, dt, nr, rb, r1, true, s));          // r1 <= P1^T r_bar
  if (o.coarse_guess == 1) {
    EBE_K(hipMemcpyAsync(u1, ub, size_t(m->n_vertices) * 3 * nr * sizeof(T), hipMemcpyDeviceToDevice, s));
  } else {
    EBE_K(launch_restrict(m, dt, nr, ub, u1, true, s));        // u1 <= P1^T u_bar
  }
  if (o.precond == EBE_PREC_MG3) {
    T* r2 = static_cast<T*>(b.r2);
    T* u2 = static_cast<T*>(b.u2);
    EBE_K(launch_restrict_p2(m, dt, nr, r1, r2, s));           // r2 <= P2^T r1
    EBE_K(launch_restrict_p2(m, dt, nr, u1, u2, s));           // u2 <= P2^T u1
    ebe_status r2s = inner_solve<T>(m, 2, r2, u2, static_cast<T*>(b.e2), static_cast<T*>(b.p2),
                                    static_cast<T*>(b.q2), nr, o.inner_eps[2], o.inner_max[2], o.graphs != 0,
                                    o.coarse_half != 0, o.deterministic != 0, st, s);
    if (r2s != EBE_OK) return r2s;
    EBE_K(launch_prolong_p2(m, dt, nr, u2, u1, s));            // u1 <= P2 u2
  }
  ebe_status rs = inner_solve<T>(m, 1, r1, u1, static_cast<T*>(b.e1), static_cast<T*>(b.p1),
                                 static_cast<T*>(b.q1), nr, o.inner_eps[1], o.inner_max[1], o.graphs != 0,
                                 o.coarse_half != 0, o.deterministic != 0, st, s);
  if (rs != EBE_OK) return rs;
  EBE_K(launch_prolong(m, dt, nr, u1, ub, true, s));           // u_bar <= P1 u1
  rs = inner_solve<T>(m, 0, rb, ub, static_cast<T*>(b.e0), static_cast<T*>(b.p0), static_cast<T*>(b.q0), nr,
                      o.inner_eps[0], o.inner_max[0], o.graphs != 0, false, o.deterministic != 0, st, s);
  if (rs != EBE_OK) return rs;
  EBE_K(sk_outer_z_cast<T>(m, ub, b.r, b.q, nr, st, s));  // z = u_bar: (z,q), (z,r), beta
  EBE_K(sk_outer_p_cast<T>(m, ub, b.p, nr, st, s));       // p <= z + beta p
  return EBE_OK;
}

ebe_status check_opts(const ebe_pcg_opts& o) {
  if ((o.precond != EBE_PREC_PCGE && o.precond != EBE_PREC_MG2 && o.precond != EBE_PREC_MG3) ||
      (o.mode != EBE_MODE_FP64 && o.mode != EBE_MODE_MIXED) || !(o.tol > 0.0) || o.max_outer < 1 ||
      o.check_every < 1 || o.inner_max[0] < 1 || o.inner_max[1] < 1 || o.inner_max[2] < 1 ||
      !(o.inner_eps[0] >= 0.0) || !(o.inner_eps[1] >= 0.0) || !(o.inner_eps[2] >= 0.0) ||
      (o.coarse_guess != 0 && o.coarse_guess != 1) || (o.graphs != 0 && o.graphs != 1) ||
      (o.coarse_half != 0 && o.coarse_half != 1) || (o.deterministic != 0 && o.deterministic != 1)) {
    set_error("ebe_pcg_solve: invalid options");
    return EBE_ERR_ARG;
  }
  return EBE_OK;
}

}  // namespace

extern "C" {

void ebe_pcg_default_opts(ebe_pcg_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precond = EBE_PREC_MG3;
  o->mode = EBE_MODE_MIXED;
  o->tol = 1e-8;
  o->max_outer = 10000;
  o->check_every = 8;
  o->inner_eps[0] = 0.1;   // Table 2, level 0
  o->inner_eps[1] = 0.05;  // Table 2, level 1
  o->inner_eps[2] = 0.025; // Table 2, level 2
  o->inner_max[0] = 30;
  o->inner_max[1] = 300;
  o->inner_max[2] = 3000;
  o->use_x0 = 0;
  o->coarse_guess = 0;
  o->graphs = 1;
}

ebe_status ebe_pcg_solve(ebe_mesh* m, int32_t nr, const double* f, double* u, const ebe_pcg_opts* opts,
                         ebe_pcg_stats* stats, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!m || !f || !u || f == u) {
    set_error("ebe_pcg_solve: null or aliasing argument");
    return EBE_ERR_ARG;
  }
  if (!aligned16(f) || !aligned16(u)) {
    set_error("ebe_pcg_solve: device buffers must be 16-byte aligned");
    return EBE_ERR_ARG;
  }
  if (nr < 1 || nr > EBE_MAX_RHS) {
    set_error("ebe_pcg_solve: nrhs %d outside 1..%d", nr, EBE_MAX_RHS);
    return EBE_ERR_ARG;
  }
  ebe_pcg_opts o;
  if (opts) o = *opts;
  else ebe_pcg_default_opts(&o);
  ebe_status st_ = check_opts(o);
  if (st_ != EBE_OK) return st_;
  if (o.deterministic && m->curved) {
    set_error("ebe_pcg_solve: deterministic solves need straight-sided elements (the curved kernel sums with "
              "atomics)");
    return EBE_ERR_ARG;
  }
  // level 2's set-up sums a coarse row in LDS: past its limit, run MG2
  if (o.precond == EBE_PREC_MG3 && m->a2_maxlen > kA2MaxRow) o.precond = EBE_PREC_MG2;
  const int64_t captures0 = m->ws.captures;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st_ = ensure_blocks(m, s)) != EBE_OK) return st_;
  if ((st_ = ensure_stage(m, nr, sizeof(double))) != EBE_OK) return st_;
  if ((st_ = ensure_workspace(m, nr)) != EBE_OK) return st_;
  if ((st_ = ensure_geometry(m, EBE_F64, s)) != EBE_OK) return st_;
  if (o.mode == EBE_MODE_MIXED && (st_ = ensure_geometry(m, EBE_F32, s)) != EBE_OK) return st_;

  Workspace& w = m->ws;
  SolverState st;
  st.sc = w.scal.as<SolverScalars>();
  st.partials = w.partials.as<void>();
  st.counter = w.counter.as<unsigned>();
  Bufs b{w.r.as<double>(), w.p.as<double>(), w.q.as<double>(), w.rb.as<void>(),
         w.ub.as<void>(), w.e0.as<void>(), w.p0.as<void>(), w.q0.as<void>(), w.r1.as<void>(),
         w.u1.as<void>(), w.e1.as<void>(), w.p1.as<void>(), w.q1.as<void>(), w.r2.as<void>(),
         w.u2.as<void>(), w.e2.as<void>(), w.p2.as<void>(), w.q2.as<void>()};
  const size_t vbytes = size_t(m->n_nodes) * 3 * nr * sizeof(double);

  // Pick the product forms this solve uses, once per mesh and case count,
  // before anything is captured into a graph (tuning waits on the stream).
  const bool mg = o.precond == EBE_PREC_MG2 || o.precond == EBE_PREC_MG3;
  const ebe_dtype inner_dt = o.mode == EBE_MODE_MIXED ? EBE_F32 : EBE_F64;
  const size_t v1bytes = size_t(m->n_vertices) * 3 * nr * sizeof(double);
  struct Tune {
    int level;
    ebe_dtype dt;
    void *x, *y;
    size_t bytes;
  } tunes[3] = {{0, EBE_F64, b.p, b.q, vbytes}, {0, inner_dt, b.p0, b.q0, vbytes}, {1, inner_dt, b.p1, b.q1, v1bytes}};
  const bool det = o.deterministic != 0;
  for (int t = 0; t < (mg ? 3 : 1) && !det; ++t) {  // a deterministic solve uses fixed forms
    const Tune& k = tunes[t];
    if (m->form[k.level][k.dt == EBE_F64 ? 0 : 1][nr] != EBE_FORM_AUTO) continue;
    EBE_K(launch_fill_zero(k.x, k.bytes, s));
    double ms[EBE_NUM_FORMS];
    if ((st_ = tune_product(m, k.level, k.dt, nr, k.x, k.y, s, ms)) != EBE_OK) return st_;
  }
  for (int t = 0; t < (mg ? 3 : 1); ++t)
    if ((st_ = prepare_products(m, tunes[t].level, tunes[t].dt, nr, s)) != EBE_OK) return st_;
  if (det && mg && (st_ = ensure_assembled(m, inner_dt, s)) != EBE_OK) return st_;
  if (o.precond == EBE_PREC_MG3 && (st_ = ensure_level2(m, inner_dt, s)) != EBE_OK) return st_;
  if (o.coarse_half && o.mode != EBE_MODE_MIXED) o.coarse_half = 0;  // FP16 coarse operators feed FP32 loops only
  if (mg && o.coarse_half && (st_ = ensure_half(m, 1, s)) != EBE_OK) return st_;
  if (o.precond == EBE_PREC_MG3 && o.coarse_half && (st_ = ensure_half(m, 2, s)) != EBE_OK) return st_;

  EBE_K(launch_fill_zero(st.sc, sizeof(SolverScalars), s));
  EBE_K(launch_fill_zero(st.counter, 64, s));
  EBE_K(launch_fill_zero(b.p, vbytes, s));
  if (o.use_x0) EBE_K(sk_mask_u(m, u, nr, st, s));
  else EBE_K(launch_fill_zero(u, vbytes, s));
  // lines 4-5: r <= f - sum_i K_i u_i
  EBE_K(level_product<double>(m, 0, nr, u, b.q, nullptr, s, nullptr, false, det, &st));
  EBE_K(sk_outer_init(m, f, b.q, b.r, nr, o.tol, st, s));

  if (!mg) EBE_K(sk_outer_z_bj(m, b.r, b.q, nr, st, s));  // first z = M^-1 r: rho (beta = 0 at iteration 0)
  SolverScalars* h = nullptr;
  ebe_status rs = read_scalars(m, s, &h);
  if (rs != EBE_OK) return rs;
  const int per_check = mg ? 1 : o.check_every;
  int enq = 0;
  while (h->outer_active && !h->err && enq < o.max_outer) {
    const int k = std::min(per_check, o.max_outer - enq);
    // q <= K p, gamma <= (p, K p); alpha; r, u updates
    auto product_and_update = [&]() -> ebe_status {
      EBE_K(level_product<double>(m, 0, nr, b.p, b.q, &st.sc->outer_active, s, st.sc->gamma, false, det, &st));
      EBE_K(sk_outer_update(m, b.r, u, b.q, b.p, nr, o.tol, o.max_outer, st, s));
      return EBE_OK;
    };
    if (mg) {
      for (int c = 0; c < k; ++c) {
        rs = (o.mode == EBE_MODE_MIXED) ? mg_precondition<float>(m, nr, o, b, st, s)
                                        : mg_precondition<double>(m, nr, o, b, st, s);
        if (rs != EBE_OK) return rs;
        if ((rs = product_and_update()) != EBE_OK) return rs;
      }
    } else {
      rs = enqueue_steps(m,
                         {2, uintptr_t(k), uintptr_t(nr),
                          det ? (uintptr_t(EBE_FORM_DETERMINISTIC) | (uintptr_t(m->fvar[0][0][nr]) << 8) |
                                 (uintptr_t(1) << 16))
                              : product_key(m, 2, EBE_F64, nr),
                          addr(b.r),
                          addr(b.p), addr(b.q), addr(u), addr(st.sc),
                          addr(st.partials), addr(st.counter), addr(m->pl[0].stage.as<void>()),
                          addr(m->gacc.as<void>()), addr(m->minv64[0].as<void>()), bits_of(o.tol),
                          uintptr_t(o.max_outer)},
                         o.graphs != 0, s, [&]() -> ebe_status {
                           for (int c = 0; c < k; ++c) {
                             EBE_K(sk_outer_p_bj(m, b.r, b.p, nr, st, s));  // p <= z + beta p, z = M^-1 r
                             // q <= K p, gamma <= (p, K p); alpha; r, u updates; next (z,q), (z,r), beta
                             EBE_K(level_product<double>(m, 0, nr, b.p, b.q, &st.sc->outer_active, s,
                                                         st.sc->gamma, false, det, &st));
                             EBE_K(sk_outer_update_z_bj(m, b.r, u, b.q, b.p, nr, o.tol, o.max_outer, st, s));
                           }
                           return EBE_OK;
                         });
      if (rs != EBE_OK) return rs;
    }
    enq += k;
    if ((rs = read_scalars(m, s, &h)) != EBE_OK) return rs;
  }
  ebe_status result = EBE_OK;
  if (h->err) result = h->err;
  else if (!(h->max_rel <= o.tol)) result = EBE_NOT_CONVERGED;
  if (stats) {
    stats->outer_iters = h->outer_iter;
    stats->inner_iters[0] = h->inner[0].steps;
    stats->inner_iters[1] = h->inner[1].steps;
    stats->inner_iters[2] = h->inner[2].steps;
    stats->max_rel_res = h->max_rel;
    stats->status = result;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats->precond_used = o.precond;
    stats->graphs_captured = int32_t(m->ws.captures - captures0);
  }
  if (result < 0) set_error("ebe_pcg_solve: %s", ebe_status_string(result));
  return result;
}

}  // extern "C"
