// One registration problem on one GPU: buffers, RK2 sweeps, the reduced
// gradient, the Gauss-Newton Hessian matvec, PCG, the outer iteration and the
// deformation gradient.
#pragma once

#include <chrono>
#include <cstdio>
#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <cstdlib>
#include <type_traits>
#include <vector>

#include "../../include/nkreg.h"
#include "group.hpp"
#include "trace.hpp"
#include "kernels_analysis.hpp"
#include "spectral.hpp"

namespace nk {

// b_l(t) = T_{l-1}(2t - 1): shifted Chebyshev polynomials (e:expansion).
inline void cheb_basis(int nc, double t, double* out) {
  const double s = 2.0 * t - 1.0;
  double t0 = 1.0, t1 = s;
  for (int l = 0; l < nc; ++l) {
    if (l == 0) out[l] = 1.0;
    else if (l == 1) out[l] = s;
    else {
      const double t2 = 2.0 * s * t1 - t0;
      t0 = t1;
      t1 = t2;
      out[l] = t2;
    }
  }
}

template <typename R>
struct DevBuf {
  R* p = nullptr;
  size_t count = 0;
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    if (hipMalloc(&p, n * sizeof(R)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      throw HipError(-3, "hipMalloc of " + std::to_string(n * sizeof(R)) + " bytes failed");
    }
    count = n;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    count = 0;
  }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

// Host-visible FP64 reduction slots.
class Reducer {
 public:
  hipStream_t s = nullptr;
  DevBuf<double> partial;   // [4][kRedBlocks]
  DevBuf<double> result;    // slots
  double* host = nullptr;   // pinned
  static constexpr int kSlots = 16;

  void init(hipStream_t stream) {
    s = stream;
    partial.alloc(4 * kRedBlocks);
    result.alloc(kSlots);
    NK_HIP(hipHostMalloc(&host, kSlots * sizeof(double), hipHostMallocDefault));
  }
  ~Reducer() {
    if (host) (void)hipHostFree(host);
  }

  // While set, reductions are recorded for a batch group instead of issued.
  Recorder* rec = nullptr;

  template <typename R>
  void enqueue(int op, const R* x, const R* y, long long cnt, int slot) {
    const int nb = (int)std::max<long long>(1, std::min<long long>(kRedBlocks, (cnt + kRedThreads - 1) / kRedThreads));
    if (rec) {
      LaunchRec a;
      a.kind = LaunchRec::RED;
      switch (op) {
        case RED_DOT: a.kernel = (const void*)k_reduce_t<R, RED_DOT>; break;
        case RED_SUMSQ: a.kernel = (const void*)k_reduce_t<R, RED_SUMSQ>; break;
        case RED_SUM: a.kernel = (const void*)k_reduce_t<R, RED_SUM>; break;
        case RED_SUMSQDIFF: a.kernel = (const void*)k_reduce_t<R, RED_SUMSQDIFF>; break;
        default: a.kernel = (const void*)k_reduce_t<R, RED_MAXABS>; break;
      }
      a.grid = dim3(nb);
      a.block = dim3(kRedThreads);
      a.cnt = cnt;
      a.set_entry(RedPtrs<R>{x, y, partial.p});
      rec->recs.push_back(a);
      LaunchRec f;
      f.kind = LaunchRec::REDF;
      f.kernel = op == RED_MAXABS ? (const void*)k_reduce_final_t<true> : (const void*)k_reduce_final_t<false>;
      f.grid = dim3(1);
      f.block = dim3(kRedThreads);
      f.iarg = nb;
      f.set_entry(RedFinalPtrs{partial.p, result.p + slot});
      rec->recs.push_back(f);
      return;
    }
    switch (op) {
      case RED_DOT: hipLaunchKernelGGL((k_reduce<R, RED_DOT>), dim3(nb), dim3(kRedThreads), 0, s, x, y, cnt, partial.p); break;
      case RED_SUMSQ: hipLaunchKernelGGL((k_reduce<R, RED_SUMSQ>), dim3(nb), dim3(kRedThreads), 0, s, x, y, cnt, partial.p); break;
      case RED_SUM: hipLaunchKernelGGL((k_reduce<R, RED_SUM>), dim3(nb), dim3(kRedThreads), 0, s, x, y, cnt, partial.p); break;
      case RED_SUMSQDIFF: hipLaunchKernelGGL((k_reduce<R, RED_SUMSQDIFF>), dim3(nb), dim3(kRedThreads), 0, s, x, y, cnt, partial.p); break;
      default: hipLaunchKernelGGL((k_reduce<R, RED_MAXABS>), dim3(nb), dim3(kRedThreads), 0, s, x, y, cnt, partial.p); break;
    }
    NK_LAUNCHED();
    if (op == RED_MAXABS)
      hipLaunchKernelGGL((k_reduce_final<true>), dim3(1), dim3(kRedThreads), 0, s, partial.p, nb, result.p + slot);
    else
      hipLaunchKernelGGL((k_reduce_final<false>), dim3(1), dim3(kRedThreads), 0, s, partial.p, nb, result.p + slot);
    NK_LAUNCHED();
  }
  // |x|^2 into slot and <x, y> into slot + 1, each equal to its own enqueue (issued only)
  template <typename R>
  void enqueue_sumsq_dot(const R* x, const R* y, long long cnt, int slot) {
    if (rec) throw HipError(NKREG_EHIP, "paired reduction is not recorded");
    const int nb = (int)std::max<long long>(1, std::min<long long>(kRedBlocks, (cnt + kRedThreads - 1) / kRedThreads));
    hipLaunchKernelGGL((k_reduce_sumsq_dot<R>), dim3(nb), dim3(kRedThreads), 0, s, x, y, cnt, partial.p);
    NK_LAUNCHED();
    hipLaunchKernelGGL(k_reduce_final_n, dim3(2), dim3(kRedThreads), 0, s, (const double*)partial.p, nb,
                       result.p + slot);
    NK_LAUNCHED();
  }
  // copies slots [0, n) to the host and waits
  void fetch(int n) {
    NK_HIP(hipMemcpyAsync(host, result.p, n * sizeof(double), hipMemcpyDeviceToHost, s));
    NK_HIP(hipStreamSynchronize(s));
  }
  template <typename R>
  double one(int op, const R* x, const R* y, long long cnt) {
    enqueue<R>(op, x, y, cnt, 0);
    fetch(1);
    return host[0];
  }
};

inline int launch_blocks(long long cnt) {
  return (int)std::max<long long>(1, std::min<long long>((cnt + 255) / 256, 8192));
}

class ProblemBase {
 public:
  nkreg_config cfg{};
  std::string assembly_timing;  // the last grouped Hessian assembly's sweep-form timing
  virtual ~ProblemBase() = default;
  virtual void set_images(const void* mT, const void* mR) = 0;
  virtual void forward(const void* v, void* m1) = 0;
  virtual void objective(const void* v, double* J, double* Jd, double* Jr) = 0;
  virtual void objective_gradient(const void* v, double* J, double* Jd, double* Jr, void* g) = 0;
  virtual void hessian_matvec(const void* vt, void* out) = 0;
  virtual void precond(const void* r, void* z) = 0;
  virtual void project(const void* f, void* out) = 0;
  virtual int pcg(const void* rhs, void* s, double rtol, int maxit, int* iters, double* relres) = 0;
  // The same PCG in steps, so that a batch can run many at once with one batched matvec
  // per iteration: pcg_begin starts it (false: nothing to iterate); while pcg_active(),
  // the caller computes q = H p into pcg_q() from pcg_p(), pcg_step enqueues the rest of
  // the iteration and the read-back of its scalars, and once the handle's stream has
  // been synchronised pcg_finish takes the iteration's decisions. pcg_result reports.
  virtual bool pcg_begin(const void* rhs, void* s, double rtol, int maxit) = 0;
  virtual bool pcg_active() const = 0;
  virtual const void* pcg_p() const = 0;
  virtual void* pcg_q() = 0;
  virtual void pcg_step() = 0;
  // pcg_step issued on st: replays a graph of the step's launches (captured once per
  // solution vector) while graphs are in use, else launches them directly on st.
  virtual void pcg_step_on(hipStream_t st) = 0;
  virtual void pcg_finish() = 0;
  virtual int pcg_result(int* iters, double* relres) const = 0;
  // Sends the handle's launches to st (nullptr: back to the handle's own stream).
  virtual void route_launches(hipStream_t st) = 0;
  virtual void det_grad_y(const void* v, void* detF, double* stats) = 0;
  virtual int newton(void* v, const nkreg_solve_opts* o, nkreg_solve_report* rep) = 0;
  virtual int picard(void* v, const nkreg_solve_opts* o, const nkreg_picard_opts* po, nkreg_solve_report* rep) = 0;
  virtual int continuation(void* v, const double* betas, int levels, const nkreg_solve_opts* o,
                           nkreg_solve_report* reps) = 0;
  virtual int beta_search(void* v, const nkreg_beta_search_opts* o, nkreg_beta_search_report* rep) = 0;
  virtual void gradient(const void* u, void* g) = 0;
  virtual void divergence(const void* w, void* s) = 0;
  virtual void apply_reg(const void* x, void* out) = 0;
  virtual double dot(const void* a, const void* b, long long cnt) = 0;
  virtual hipStream_t stream() const = 0;
  virtual void set_beta(double beta) = 0;
  virtual void set_hessian(int mode) = 0;
  virtual void assemble_hessian(void* H) = 0;
  // The cached state a matvec is taken at: valid flag, velocity (FP64) and images
  // (transport precision), for handles that replicate it.
  virtual bool state_ready() const = 0;
  virtual const double* velocity() const = 0;
  virtual void images(const void** mT, const void** mR) const = 0;
  // The template mean subtracted from the images, and setting already centred images.
  virtual double image_shift() const = 0;
  virtual void set_centred_images(const void* mT, const void* mR, double shift) = 0;
  virtual int lanczos(int steps, double* ritz, int* count) = 0;
  virtual int hessian_mode() const = 0;
  virtual void use_graph_capture(bool on) = 0;
  virtual std::string describe() = 0;
  // Records one matvec's launches (nothing is issued); checks the cached state.
  // col_variant >= 0 records with that column pass (8 or 0 = tiled, which give
  // identical values) instead of the handle's own choice.
  virtual void record_matvec(const void* vt, void* out, Recorder& r, int col_variant = -1) = 0;
  // Records one objective and gradient evaluation at v (g may be null: the handle's own
  // buffer) the same way; gradient_done then reads J and marks the state valid once the
  // recorded launches have run. check_cfl applies the CFL bound of the configuration.
  virtual void record_gradient(const void* v, void* g, Recorder& r, int col_variant = -1) = 0;
  virtual void gradient_done(double* J, double* Jd, double* Jr) = 0;
  virtual void check_cfl(const void* v) = 0;
  virtual bool tiled_pass_applies() const = 0;
  virtual int col_variant() const = 0;
  virtual hipStream_t caller_stream() const = 0;
  // bumped whenever captured graphs become stale (beta change, graph switch, timer)
  unsigned generation = 0;
  virtual void matvec_bytes(const void* vt, void* out, double* bytes, int* launches) = 0;
  virtual void timer_arm(int id, int capacity) = 0;
  virtual void timer_read(int* launches, double* avg_ms, double* bytes) = 0;
};

// R is the transport precision (state, adjoint and incremental sweeps, their
// FFTs and the trajectory). The control space -- velocity coefficients,
// gradients, Krylov vectors and the spectral finalize (beta A, K, the
// preconditioner) -- is FP64 in both modes: the H2 symbol |k|^4 would amplify
// FP32 rounding of a velocity at the grid's corner wavenumbers far above the
// gradient itself, while control-space work is O(1) per matvec against the
// O(nt) transport work.
// Column-tile choices made by the autotuner, shared by every handle of the
// process: one entry per (grid, transport precision). The candidates round
// differently, so sharing the choice keeps all handles of one shape
// bit-identical to each other.
struct TuneTable {
  std::mutex m;
  std::map<std::array<int, 4>, int> col_e;
};
inline TuneTable& tune_table() {
  static TuneTable t;
  return t;
}

template <typename R>
class ProblemT final : public ProblemBase {
 public:
  static constexpr bool kF64 = std::is_same<R, double>::value;
  Grid g;
  // Every call runs on the caller's stream (which may be the null stream, where
  // capture is not possible); graphs are captured on a stream of the handle's own
  // and replayed on the caller's.
  hipStream_t user_s;      // the caller's stream
  hipStream_t cap_s;       // used only while capturing or autotuning
  hipStream_t s;           // where launches go: user_s, or cap_s while capturing
  Spectral<R> sp;          // transport precision
  Spectral<double> sp64;   // control space
  Reducer red;
  int nc, d, nt;
  long long n, nv;     // points per scalar field; values per velocity (nc*d*n)
  bool have_images = false;
  bool state_valid = false;

  // transport precision
  DevBuf<R> mT, mR, traj, acc, lam, m1, mt1, vR, vtR, F;
  DevBuf<cplx<R>> T, Ts, S1, S2, U, Dsp;
  // trajectory checkpointing: m at the start of every K-step segment, and the
  // scratch of the segment recomputation (disjoint from the sweeps' buffers).
  // The trajectory buffer has S slots of one segment each; segment s lives in
  // slot s % S, and held[slot] names the segment a slot currently holds.
  int K = 0, nseg = 1, seglen = 0, S = 1;
  std::vector<int> held;
  DevBuf<R> ckpt, accr, mr;
  DevBuf<cplx<R>> Tr, Tsr, S1r, S2r;
  // control space (FP64)
  DevBuf<double> v, tmpv, kx, kr, kz, kp, kq, gbuf, sbuf, vtrial, rhsbuf;
  DevBuf<cplx<double>> Xs, Ys;

  static hipStream_t make_stream() {
    hipStream_t st;
    NK_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));  // default priority
    return st;
  }

  ProblemT(const nkreg_config& c, hipStream_t stream)
      : g(make_grid(c.dim, c.n)), user_s(stream), cap_s(make_stream()), s(stream), sp(g, stream),
        sp64(g, stream) {
    const char* ng = std::getenv("NKREG_NO_GRAPHS");
    use_graphs = !(ng && ng[0] == '1');
    cfg = c;
    nc = c.nc;
    d = c.dim;
    nt = c.nt;
    n = g.npts;
    nv = (long long)nc * d * n;
    red.init(s);
    mT.alloc(n); mR.alloc(n);
    K = (c.checkpoint_every > 0 && c.checkpoint_every < nt) ? c.checkpoint_every : 0;
    nseg = K ? (nt + K - 1) / K : 1;
    seglen = K ? K : nt;
    S = K ? std::max(1, std::min(c.trajectory_slots, nseg)) : 1;
    held.assign(S, -1);
    traj.alloc((size_t)2 * S * seglen * d * n);
    if (K) {
      ckpt.alloc((size_t)nseg * n);
      accr.alloc(n); mr.alloc(n);
      Tr.alloc(g.nspec); Tsr.alloc(g.nspec); S1r.alloc(g.nspec); S2r.alloc(g.nspec);
    }
    acc.alloc(n); lam.alloc(n); m1.alloc(n); mt1.alloc(n);
    F.alloc(nv);
    if (!kF64) { vR.alloc(nv); vtR.alloc(nv); }
    T.alloc(g.nspec); Ts.alloc(g.nspec); S1.alloc(g.nspec); S2.alloc(g.nspec);
    U.alloc((size_t)3 * g.nspec); Dsp.alloc(g.nspec);
    v.alloc(nv); tmpv.alloc(nv);
    Xs.alloc((size_t)nc * d * g.nspec); Ys.alloc((size_t)nc * d * g.nspec);
    kx.alloc(nv); kr.alloc(nv); kz.alloc(nv); kp.alloc(nv); kq.alloc(nv);
    gbuf.alloc(nv); sbuf.alloc(nv); vtrial.alloc(nv); rhsbuf.alloc(nv);
    tune_columns();
  }

  hipStream_t stream() const override { return user_s; }

  // Sends every launch of this handle (both spectral engines and the reducer) to st.
  void route(hipStream_t st) {
    s = st;
    sp.s = st;
    sp64.s = st;
    red.s = st;
  }
  // Launches go to the capture stream while an object of this type lives.
  struct OnCaptureStream {
    ProblemT& p;
    explicit OnCaptureStream(ProblemT& q) : p(q) { p.route(p.cap_s); }
    ~OnCaptureStream() { p.route(p.user_s); }
  };

  // ---- Hessian: Gauss-Newton (default) or full Newton (e:second-order-opt-cond) ----
  // The full-Newton matvec reads the gradient's adjoint states (lam^{j+1}, lam*_j
  // per step, kept by the gradient's adjoint sweep) and its own incremental
  // state gradients (grad m~^j, grad m~*_j, kept by its incremental sweep).
  bool full_newton = false;
  DevBuf<R> ltraj, mtraj;
  R* ltp(int j, int k) { return ltraj.p + ((size_t)(2 * j + k)) * n; }
  R* mtp(int j, int k) { return mtraj.p + ((size_t)(2 * j + k)) * d * n; }
  void set_hessian(int mode) override {
    if (mode != 0 && mode != 1) throw HipError(NKREG_EINVAL, "Hessian mode must be 0 (GN) or 1 (full Newton)");
    NK_HIP(hipStreamSynchronize(s));
    if (mode == 1 && !ltraj.p) {
      ltraj.alloc((size_t)2 * nt * n);
      mtraj.alloc((size_t)2 * nt * d * n);
    }
    if ((mode == 1) != full_newton) state_valid = false;  // the adjoint states must be recorded
    full_newton = mode == 1;
    drop_graphs();
  }
  int hessian_mode() const override { return full_newton ? 1 : 0; }

  // ---- HIP graph of the Hessian matvec, keyed by its (input, output) pointers ----
  bool use_graphs = true;
  struct GraphEntry {
    const void* in = nullptr;
    void* out = nullptr;
    hipGraphExec_t exec = nullptr;
  } mv_graph;
  // the PCG step's launches (pcg_step_on), keyed by the solution vector it updates
  struct StepGraph {
    const double* x = nullptr;
    hipGraphExec_t exec = nullptr;
  } step_graph;
  void drop_graphs() {
    if (mv_graph.exec) (void)hipGraphExecDestroy(mv_graph.exec);
    mv_graph = GraphEntry{};
    if (step_graph.exec) (void)hipGraphExecDestroy(step_graph.exec);
    step_graph = StepGraph{};
    ++generation;
  }
  hipStream_t caller_stream() const override { return user_s; }
  ~ProblemT() override {
    (void)hipStreamSynchronize(user_s);
    (void)hipStreamSynchronize(cap_s);
    drop_graphs();
    (void)hipStreamDestroy(cap_s);
  }
  void use_graph_capture(bool on) override {
    NK_HIP(hipStreamSynchronize(s));
    drop_graphs();
    use_graphs = on;
  }
  void set_beta(double beta) override {
    cfg.beta = beta;
    drop_graphs();  // beta is a kernel argument of the captured finalize
  }

  KernelTimer timer;
  // One eager matvec that adds up the algorithmic bytes of all its launches.
  void matvec_bytes(const void* vt, void* out, double* bytes, int* launches) override {
    if (!state_valid) throw HipError(NKREG_ESTATE, "no gradient computed at the current velocity");
    ByteTally t;
    sp.tally = sp64.tally = &t;
    try {
      matvec_body(vt, out);
    } catch (...) {
      sp.tally = sp64.tally = nullptr;
      throw;
    }
    sp.tally = sp64.tally = nullptr;
    NK_HIP(hipStreamSynchronize(s));
    if (bytes) *bytes = t.bytes;
    if (launches) *launches = (int)t.launches;
  }
  void timer_arm(int id, int capacity) override {
    NK_HIP(hipStreamSynchronize(s));
    timer.arm(id, capacity);
    sp.timer = &timer;
  }
  void timer_read(int* launches, double* avg_ms, double* bytes) override {
    const double ms = timer.average_ms();
    if (launches) *launches = timer.used;
    if (avg_ms) *avg_ms = ms;
    if (bytes) *bytes = timer.used ? timer.bytes / timer.used : 0.0;
    timer.armed = -1;
    sp.timer = nullptr;
    drop_graphs();
  }

  // grad m^j (stage 0) and grad m*_j (stage 1) of the steps held in the trajectory buffer
  R* trajp(int j, int stage) {
    const size_t slot = K ? (size_t)((j / K) % S) : 0;
    const int jj = K ? j % K : j;
    return traj.p + (slot * 2 * seglen + (size_t)(2 * jj + stage)) * d * n;
  }

  void basis(double t, R* out) {
    double b[kMaxNc];
    cheb_basis(nc, t, b);
    for (int l = 0; l < kMaxNc; ++l) out[l] = l < nc ? (R)b[l] : R(0);
  }

  // Recording for batch groups: while rec is set, the matvec's launches are
  // recorded (here and in both spectral engines) instead of issued.
  Recorder* rec = nullptr;
  // Marks the start of a time-loop iteration (loop: LOOP_*) or the end of a loop in
  // the recording, so that items with different step counts can share launches.
  void mark(int loop, int step) {
    if (rec) rec->mark(loop, step);
  }
  void record_matvec(const void* vt, void* out, Recorder& r, int col_variant) override {
    if (!state_valid) throw HipError(NKREG_ESTATE, "no gradient computed at the current velocity");
    const int keep = sp.colE, keep64 = sp64.colE;
    if (col_variant >= 0) sp.colE = sp64.colE = col_variant;
    rec = sp.rec = sp64.rec = &r;
    try {
      matvec_body(vt, out);
    } catch (...) {
      rec = sp.rec = sp64.rec = nullptr;
      sp.colE = keep;
      sp64.colE = keep64;
      throw;
    }
    rec = sp.rec = sp64.rec = nullptr;
    sp.colE = keep;
    sp64.colE = keep64;
  }
  void record_gradient(const void* vin, void* gout, Recorder& r, int col_variant) override {
    need_images();
    state_valid = false;
    const int keep = sp.colE, keep64 = sp64.colE;
    if (col_variant >= 0) sp.colE = sp64.colE = col_variant;
    rec = sp.rec = sp64.rec = red.rec = &r;
    try {
      gradient_body(vin, gout);
    } catch (...) {
      rec = sp.rec = sp64.rec = red.rec = nullptr;
      sp.colE = keep;
      sp64.colE = keep64;
      held.assign(S, -1);
      throw;
    }
    rec = sp.rec = sp64.rec = red.rec = nullptr;
    sp.colE = keep;
    sp64.colE = keep64;
  }
  bool tiled_pass_applies() const override { return sp.any_tiled_pass(); }
  int col_variant() const override { return sp.colE; }

  void copy(void* dst, const void* src, size_t bytes) {
    if (rec) {
      LaunchRec r;
      r.kind = LaunchRec::COPY;
      r.dst = dst;
      r.src = src;
      r.bytes = bytes;
      rec->recs.push_back(r);
      return;
    }
    NK_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
  }
  template <typename RS, typename RD>
  void convert(long long cnt, const RS* x, RD* y) {
    if (rec) {
      LaunchRec r;
      r.kind = LaunchRec::CONV;
      r.kernel = (const void*)k_convert_t<RS, RD>;
      r.grid = dim3(launch_blocks(cnt));
      r.block = dim3(256);
      r.cnt = cnt;
      r.conv = (sizeof(RS) == 8 && sizeof(RD) == 4) ? 1 : ((sizeof(RS) == 4 && sizeof(RD) == 8) ? 2 : 0);
      r.set_entry(ConvPtrs<RS, RD>{x, y});
      rec->recs.push_back(r);
      return;
    }
    if (sp.tally) sp.tally->add((double)cnt * (sizeof(RS) + sizeof(RD)));
    hipLaunchKernelGGL((k_convert<RS, RD>), dim3(launch_blocks(cnt)), dim3(256), 0, s, cnt, x, y);
    NK_LAUNCHED();
  }
  void fill(long long cnt, R v, R* y) {
    if (rec) {
      LaunchRec r;
      r.kind = LaunchRec::FILL;
      r.kernel = (const void*)k_fill_t<R>;
      r.grid = dim3(launch_blocks(cnt));
      r.block = dim3(256);
      r.cnt = cnt;
      r.fval = (double)v;
      r.f64 = kF64;
      r.set_entry(y);
      rec->recs.push_back(r);
      return;
    }
    if (sp.tally) sp.tally->add((double)cnt * sizeof(R));
    hipLaunchKernelGGL((k_fill<R>), dim3(launch_blocks(cnt)), dim3(256), 0, s, cnt, v, y);
    NK_LAUNCHED();
  }

  // FP64 control vector -> transport precision (aliases in FP64 mode)
  const R* to_transport(const double* x, DevBuf<R>& dst) {
    if constexpr (kF64) {
      return x;
    } else {
      convert<double, R>(nv, x, dst.p);
      return dst.p;
    }
  }
  // beta A x + K[F] for the body force F in the transport precision (read as FP32 and
  // widened by the R2C when the transport runs in FP32)
  void hess_vecop(const double* x, double* out) {
    if constexpr (kF64)
      sp64.vecop(OP_HESS, x, (const double*)F.p, out, nc, cfg.reg, cfg.incompressible, cfg.beta, Xs.p, Ys.p);
    else
      sp64.vecop(OP_HESS, x, nullptr, out, nc, cfg.reg, cfg.incompressible, cfg.beta, Xs.p, Ys.p,
                 (const float*)F.p);
  }

  // The images are kept centred: the template's mean c is subtracted from both.
  // Transport carries a constant exactly and the objective, the adjoint, the
  // gradient and the Hessian see only differences and gradients of the images, so
  // nothing changes but the round-off: the transforms' rounding error scales with
  // the field's norm, mean included, and in FP32 the spectral derivative amplifies
  // it by the grid's wavenumbers. m_1 is returned with c added back.
  double shift = 0.0;
  void set_images(const void* a, const void* b) override {
    copy(mT.p, a, n * sizeof(R));
    copy(mR.p, b, n * sizeof(R));
    shift = red.one<R>(RED_SUM, mT.p, nullptr, n) / (double)n;
    if (!std::isfinite(shift)) throw HipError(NKREG_ENONFINITE, "template image is not finite");
    shift_images(-shift);
    have_images = true;
    state_valid = false;
  }
  void shift_images(double c) {
    hipLaunchKernelGGL((k_shift<R>), dim3(launch_blocks(n)), dim3(256), 0, s, n, (R)c, (const R*)mT.p, mT.p);
    hipLaunchKernelGGL((k_shift<R>), dim3(launch_blocks(n)), dim3(256), 0, s, n, (R)c, (const R*)mR.p, mR.p);
    NK_LAUNCHED();
  }
  // Images already centred by another handle (with their shift): copied as they are.
  void set_centred_images(const void* a, const void* b, double c) override {
    copy(mT.p, a, n * sizeof(R));
    copy(mR.p, b, n * sizeof(R));
    shift = c;
    have_images = true;
    state_valid = false;
  }
  double image_shift() const override { return shift; }

  // ---- state equation (Heun) ----
  struct SweepBufs {
    cplx<R>* T;
    cplx<R>* Ts;
    cplx<R>* S1;
    cplx<R>* S2;
    R* acc;
  };
  SweepBufs main_bufs() { return {T.p, Ts.p, S1.p, S2.p, acc.p}; }
  SweepBufs recompute_bufs() { return {Tr.p, Tsr.p, S1r.p, S2r.p, accr.p}; }

  // Steps j0..j1-1 from m^{j0} = m_start; m_state receives m^{j+1} after each
  // step. record: store grad m^j, grad m*_j in the trajectory buffer.
  // store_ckpt: copy m at every segment boundary into the checkpoints.
  void state_steps(const R* vl, int j0, int j1, const R* m_start, R* m_state, const SweepBufs& B, bool record,
                   bool store_ckpt) {
    const R h = R(1.0 / nt);
    sp.r2c(m_start, B.T, 1);
    for (int j = j0; j < j1; ++j) {
      mark(LOOP_STATE, j - j0);
      sp.deriv_cols(B.T, B.S1, B.S2);
      StageArgs<R> a{};
      a.spec = B.T; a.s1 = B.S1; a.s2 = B.S2; a.out0 = B.Ts;
      a.vl = vl; a.nc = nc; a.h = h; a.acc = B.acc;
      a.g0w = record ? trajp(j, 0) : nullptr;
      a.mreal = (j == j0) ? m_start : m_state;
      basis(j * (double)h, a.b0);
      sp.template row<ST_FWD1>(a, 1);
      sp.deriv_cols(B.Ts, B.S1, B.S2);
      StageArgs<R> b{};
      b.spec = B.Ts; b.s1 = B.S1; b.s2 = B.S2; b.out0 = B.T;
      b.vl = vl; b.nc = nc; b.h = h; b.acc = B.acc;
      b.g1w = record ? trajp(j, 1) : nullptr;
      basis((j + 1) * (double)h, b.b1);
      b.out_real = m_state;  // m^{j+1}
      sp.template row<ST_FWD2>(b, 1);
      if (store_ckpt && (j + 1) % K == 0 && j + 1 < nt) copy(ckpt.p + (size_t)((j + 1) / K) * n, m_state, n * sizeof(R));
    }
    mark(LOOP_NONE, 0);
  }

  // Forward solve from m_T; m1out receives m_1. With record, the trajectory is
  // kept in full or, when checkpointing, as m at the segment starts plus the
  // last S segments, which the adjoint sweep needs first. The recorded part
  // restarts from its checkpoint exactly as a recomputation does, so the
  // buffer holds the same values either way.
  void forward_sweep(const R* vl, bool record, R* m1out) {
    const Range range("state sweep");
    if (!K) {
      state_steps(vl, 0, nt, mT.p, m1out, main_bufs(), record, false);
    } else if (!record) {
      state_steps(vl, 0, nt, mT.p, m1out, main_bufs(), false, false);
    } else {
      const int s0 = nseg - S, jl = s0 * K;
      held.assign(S, -1);
      copy(ckpt.p, mT.p, n * sizeof(R));
      if (jl > 0) state_steps(vl, 0, jl, mT.p, m1out, main_bufs(), false, true);
      state_steps(vl, jl, nt, jl > 0 ? m1out : mT.p, m1out, main_bufs(), true, true);
      for (int sg = s0; sg < nseg; ++sg) held[sg % S] = sg;
    }
  }

  // Makes the trajectory of segment sgi available: recomputed from its
  // checkpoint unless its slot still holds it. After every adjoint sweep the
  // slots hold the segments 0..S-1 (the sweep ends there), and a matvec leaves
  // them so, whether it runs eagerly or as a captured graph.
  void load_segment(const R* vl, int sgi) {
    if (!K || held[sgi % S] == sgi) return;
    const int j0 = sgi * K, j1 = std::min(nt, j0 + K);
    held[sgi % S] = -1;
    state_steps(vl, j0, j1, ckpt.p + (size_t)sgi * n, mr.p, recompute_bufs(), true, false);
    held[sgi % S] = sgi;
  }

  // ---- adjoint (conservative, backward Heun) with body-force accumulation ----
  // lam(1) = ca*src_a + cb*src_b; F (nc*d fields) = time-integrated lam grad m.
  // record_lam keeps lam^{j+1} and lam*_j per step (for the full-Newton matvec).
  // NEWT: the full-Newton incremental adjoint (e:sec-order-iadj), with v~ = vtl and
  // the gradient's adjoint states and this matvec's grad m~ trajectories.
  template <bool NEWT>
  void adjoint_sweep_k(const R* vl, const R* vtl, R ca, const R* src_a, R cb, const R* src_b, R* Fout,
                       bool record_lam) {
    const Range range("adjoint sweep");
    constexpr int KI = NEWT ? ST_NADJINIT : ST_ADJINIT;
    constexpr int K1 = NEWT ? ST_NADJ1 : ST_ADJ1;
    constexpr int K2 = NEWT ? ST_NADJ2 : ST_ADJ2;
    const R h = R(1.0 / nt);
    const long long ns = g.nspec;
    cplx<R>* U0 = U.p;
    cplx<R>* U1 = U.p + ns;
    cplx<R>* U2 = U.p + 2 * ns;
    StageArgs<R> a{};
    a.vl = vl; a.nc = nc; a.h = h;
    a.src_a = src_a; a.src_b = src_b; a.ca = ca; a.cb = cb;
    a.lam = lam.p; a.out0 = U0; a.out1 = U1; a.out2 = U2;
    if (NEWT) { a.vtl = vtl; a.lt0 = ltp(nt - 1, 0); }
    basis(1.0, a.bv);
    sp.template row<KI>(a, 1);
    for (int j = nt - 1; j >= 0; --j) {
      mark(LOOP_ADJOINT, nt - 1 - j);
      if (K && (j == nt - 1 || (j + 1) % K == 0)) load_segment(vl, j / K);
      sp.div_cols(U0, U1, U2, S2.p, Dsp.p);
      StageArgs<R> b{};
      b.spec = Dsp.p; b.vl = vl; b.nc = nc; b.h = h;
      b.lam = lam.p; b.acc = acc.p; b.F = Fout;
      b.zero_state = (j == nt - 1);   // the first step overwrites the force accumulators
      b.g0 = trajp(j, 0); b.g1 = trajp(j, 1);
      if (record_lam) { b.lamw0 = ltp(j, 0); b.lamw1 = ltp(j, 1); }
      if (NEWT) { b.vtl = vtl; b.lt0 = ltp(j, 0); b.lt1 = ltp(j, 1); b.gt0 = mtp(j, 0); b.gt1 = mtp(j, 1); }
      basis(j * (double)h, b.b0);
      basis((j + 1) * (double)h, b.b1);
      basis(j * (double)h, b.bv);
      b.out0 = U0; b.out1 = U1; b.out2 = U2;
      sp.template row<K1>(b, 1);
      sp.div_cols(U0, U1, U2, S2.p, Dsp.p);
      StageArgs<R> c{};
      c.spec = Dsp.p; c.vl = vl; c.nc = nc; c.h = h;
      c.lam = lam.p; c.acc = acc.p;
      basis(j * (double)h, c.bv);
      c.skip_out = (j == 0);
      if (NEWT) { c.vtl = vtl; c.lt0 = j > 0 ? ltp(j - 1, 0) : nullptr; }   // lam^j
      c.out0 = U0; c.out1 = U1; c.out2 = U2;
      sp.template row<K2>(c, 1);
    }
    mark(LOOP_NONE, 0);
  }

  // ---- incremental state (GN), m~(0) = 0; writes m~_1 to mt1 ----
  // With checkpointing, the segments still held from the last adjoint sweep
  // (of the gradient or of the previous matvec, both at the current velocity)
  // are not recomputed; nothing else writes the trajectory buffer while the
  // gradient state is valid.
  void incremental_sweep(const R* vl, const R* vtl) {
    const Range range("incremental state sweep");
    const R h = R(1.0 / nt);
    for (int j = 0; j < nt; ++j) {
      mark(LOOP_INCREMENTAL, j);
      if (K && j % K == 0) load_segment(vl, j / K);
      if (j > 0) sp.deriv_cols(T.p, S1.p, S2.p);
      StageArgs<R> a{};
      a.spec = T.p; a.s1 = S1.p; a.s2 = S2.p; a.out0 = Ts.p;
      a.vl = vl; a.vtl = vtl; a.nc = nc; a.h = h; a.acc = acc.p;
      a.g0 = trajp(j, 0);
      if (full_newton) a.g0w = mtp(j, 0);
      a.zero_state = (j == 0);
      a.mreal = mt1.p;
      basis(j * (double)h, a.b0);
      sp.template row<ST_INC1>(a, 1);
      sp.deriv_cols(Ts.p, S1.p, S2.p);
      StageArgs<R> b{};
      b.spec = Ts.p; b.s1 = S1.p; b.s2 = S2.p; b.out0 = T.p;
      b.vl = vl; b.vtl = vtl; b.nc = nc; b.h = h; b.acc = acc.p;
      b.g1 = trajp(j, 1);
      if (full_newton) b.g1w = mtp(j, 1);
      basis((j + 1) * (double)h, b.b1);
      b.out_real = mt1.p;  // m~^{j+1}; m~_1 after the last step
      sp.template row<ST_INC2>(b, 1);
    }
    mark(LOOP_NONE, 0);
  }

  // h_t max over i of (sum_l max|v_l^i|) / h_x^i; bounds the CFL number since
  // |T_l| <= 1 on [0, 1] (equal to it for nc = 1).
  double cfl_number(const double* vl) {
    double worst = 0.0;
    for (int i = 0; i < d; ++i) {
      double bound = 0.0;
      for (int l = 0; l < nc; ++l)
        bound += red.one<double>(RED_MAXABS, vl + ((long long)l * d + i) * n, nullptr, n);
      worst = std::max(worst, bound / (2.0 * M_PI / g.n[i]));
    }
    return worst / nt;
  }

  void check_velocity_cfl(const double* vl) {
    if (cfg.cfl_max <= 0) return;
    const double cfl = cfl_number(vl);
    if (!(cfl <= cfg.cfl_max)) throw HipError(NKREG_ECFL, "CFL number " + std::to_string(cfl) + " above cfl_max");
  }

  void need_images() {
    if (!have_images) throw HipError(NKREG_ESTATE, "set_images has not been called");
  }

  void forward(const void* vin, void* m1out) override {
    need_images();
    copy(v.p, vin, nv * sizeof(double));
    const R* vl = to_transport(v.p, vR);
    forward_sweep(vl, true, m1.p);
    if (m1out) {
      hipLaunchKernelGGL((k_shift<R>), dim3(launch_blocks(n)), dim3(256), 0, s, n, (R)shift, (const R*)m1.p,
                         (R*)m1out);
      NK_LAUNCHED();
    }
    state_valid = false;  // the adjoint solve of a gradient is still needed before matvecs
  }

  // J_dist (FP64 reduction of the transport-precision mismatch) and J_reg (FP64):
  // the reductions land in slots 0 and 1; objective_read waits for them.
  void objective_enqueue(const double* vl) {
    sp64.vecop(OP_A, vl, nullptr, tmpv.p, nc, cfg.reg, 0, cfg.beta, Xs.p, Ys.p);
    red.enqueue<R>(RED_SUMSQDIFF, mR.p, m1.p, n, 0);
    red.enqueue<double>(RED_DOT, vl, tmpv.p, nv, 1);
  }
  void objective_read(double* Jd, double* Jr, bool require_finite = true) {
    red.fetch(2);
    *Jd = 0.5 * g.hd * red.host[0];
    *Jr = 0.5 * cfg.beta * g.hd * red.host[1];
    if (require_finite && (!std::isfinite(*Jd) || !std::isfinite(*Jr)))
      throw HipError(NKREG_ENONFINITE, "objective is not finite");
  }
  void objective_terms(const double* vl, double* Jd, double* Jr, bool require_finite = true) {
    objective_enqueue(vl);
    objective_read(Jd, Jr, require_finite);
  }

  // J at a line-search trial point; +inf if the trial's transport overflowed,
  // which rejects the trial (the line search then halves the step).
  double trial_objective(const double* vl) {
    forward_sweep(to_transport(vl, vtR), false, m1.p);
    state_valid = false;
    double jd, jr;
    objective_terms(vl, &jd, &jr, false);
    const double J = jd + jr;
    return std::isfinite(J) ? J : HUGE_VAL;
  }

  void objective(const void* vin, double* J, double* Jd, double* Jr) override {
    need_images();
    const double* vl = (const double*)vin;
    forward_sweep(to_transport(vl, vtR), false, m1.p);
    state_valid = false;
    double jd, jr;
    objective_terms(vl, &jd, &jr);
    if (J) *J = jd + jr;
    if (Jd) *Jd = jd;
    if (Jr) *Jr = jr;
  }

  // One objective and gradient evaluation as a sequence of launches: forward sweep
  // (keeping the trajectory), the objective's reductions, adjoint sweep with the
  // body force, and the spectral finalize g = beta A v + K[f]. Nothing waits.
  void gradient_body(const void* vin, void* gout) {
    copy(v.p, vin, nv * sizeof(double));
    const R* vl = to_transport(v.p, vR);
    forward_sweep(vl, true, m1.p);
    objective_enqueue(v.p);
    adjoint_sweep_k<false>(vl, nullptr, R(1), mR.p, R(-1), m1.p, F.p, full_newton);
    double* gdst = gout ? (double*)gout : gbuf.p;
    hess_vecop(v.p, gdst);
  }

  void objective_gradient(const void* vin, double* J, double* Jd, double* Jr, void* gout) override {
    need_images();
    check_velocity_cfl((const double*)vin);
    state_valid = false;
    gradient_body(vin, gout);
    gradient_done(J, Jd, Jr);
  }

  // After a gradient's launches: reads J (waits), checks it, marks the state valid.
  void gradient_done(double* J, double* Jd, double* Jr) override {
    double jd, jr;
    objective_read(&jd, &jr);
    state_valid = true;
    if (J) *J = jd + jr;
    if (Jd) *Jd = jd;
    if (Jr) *Jr = jr;
  }
  void check_cfl(const void* vin) override {
    need_images();
    check_velocity_cfl((const double*)vin);
  }

  void hessian_matvec(const void* vtin, void* out) override {
    if (!state_valid) throw HipError(NKREG_ESTATE, "no gradient computed at the current velocity");
    // HIP events recorded by graph nodes cannot be timed, so an armed kernel
    // timer makes the matvec launch eagerly.
    if (!use_graphs || timer.armed >= 0) {
      matvec_body(vtin, out);
      return;
    }
    if (!(mv_graph.exec && mv_graph.in == vtin && mv_graph.out == out)) {
      drop_graphs();
      mv_graph.exec = capture_matvec(vtin, out);
      mv_graph.in = vtin;
      mv_graph.out = out;
    }
    NK_HIP(hipGraphLaunch(mv_graph.exec, s));
  }

  // Captures one matvec on the capture stream; nothing runs until the graph is launched.
  // On small square grids the transport sweeps may run in the persistent kernel (from the
  // recorded launch sequence and its argument table, kept in mv_tab while the graph lives):
  // it is timed against the direct launches (once per pointer pair; the values are the
  // same), and the faster is kept.
  DevBuf<unsigned char> mv_tab;
  bool small_sweeps = false;
  std::string sweep_timing;
  // The matvec's launches captured as they are issued (kernels take their arguments
  // directly).
  hipGraphExec_t capture_direct(const void* vtin, void* out) {
    hipGraph_t graph = nullptr;
    OnCaptureStream on(*this);
    NK_HIP(hipStreamBeginCapture(cap_s, hipStreamCaptureModeThreadLocal));
    try {
      matvec_body(vtin, out);
    } catch (...) {
      (void)hipStreamEndCapture(cap_s, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    NK_HIP(hipStreamEndCapture(cap_s, &graph));
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) throw HipError(NKREG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return exec;
  }

  // The matvec graph. On small square grids the persistent form of its sweeps
  // (group.hpp, small.hpp) is timed against the direct launches and the faster kept;
  // NKREG_SMALL=1 forces the persistent form.
  hipGraphExec_t capture_matvec(const void* vtin, void* out) {
    small_sweeps = false;
    hipGraphExec_t direct = capture_direct(vtin, out);
    if (!small_config(cfg)) return direct;
    try {
      GroupPlan gp;
      gp.items = {0};
      gp.recs.resize(1);
      record_matvec(vtin, out, gp.recs[0], 8);
      gp.small_ops = small_prefix(gp.recs[0].recs);
      if (!gp.small_ops) return direct;
      NK_HIP(hipStreamSynchronize(user_s));   // the timing replays run on the capture stream
      bool persistent = small_forced();
      if (!persistent) {
        const float t_pers = time_group(gp, cap_s);
        const float t_dir = time_exec(direct, cap_s);
        sweep_timing = "persistent " + std::to_string(1e3f * t_pers) + " us, launches " +
                       std::to_string(1e3f * t_dir) + " us per matvec";
        persistent = t_pers < t_dir;
      }
      if (!persistent) return direct;
      std::vector<unsigned char> host;
      add_tables(gp, host);
      NK_HIP(hipStreamSynchronize(s));   // an earlier graph may still read the old table
      mv_tab.alloc(host.size());
      NK_HIP(hipMemcpy(mv_tab.p, host.data(), host.size(), hipMemcpyHostToDevice));
      hipGraphExec_t ex = capture_group(gp, mv_tab.p, cap_s);
      (void)hipGraphExecDestroy(direct);
      small_sweeps = true;
      return ex;
    } catch (...) {
      (void)hipStreamSynchronize(cap_s);
      (void)hipGraphExecDestroy(direct);
      throw;
    }
  }

  // Column-pass autotuner, run once per handle at creation: the candidates are
  // the one-workgroup-per-column-group pass with 8 complex elements per lane and,
  // where an axis allows it, the LDS-tiled pass. Both run the same register FFT
  // on the same values, so the choice changes the schedule and never a result.
  // For each candidate a HIP graph of kTuneReps derivative and divergence column
  // passes over zeroed spectra is captured on the capture stream and replayed
  // under HIP events; the fastest is kept and shared by every handle of the same
  // grid and precision in the process. NKREG_COL_E in the environment fixes the
  // choice (8, 4 or tiled; 4 elements per lane rounds differently), for every grid
  // or per grid (col_env_variant).
  static constexpr int kTuneReps = 16;
  static std::string col_variant_name(int ce) { return ce == 0 ? "col=tiled" : "col_E=" + std::to_string(ce); }
  std::string tuning;
  std::array<int, 4> tune_key() const { return {g.n[0], g.n[1], g.n[2], kF64 ? 64 : 32}; }
  void tune_columns() {
    if (col_env_variant(g) >= 0) {
      tuning = col_variant_name(sp.colE) + " (fixed)";
      return;
    }
    TuneTable& tt = tune_table();
    std::lock_guard<std::mutex> lk(tt.m);
    if (auto it = tt.col_e.find(tune_key()); it != tt.col_e.end()) {
      sp.colE = it->second;
      tuning = col_variant_name(sp.colE) + " (chosen earlier in this process for this grid)";
      return;
    }
    const long long ns = g.nspec;
    std::vector<int> cands = {8};
    if (sp.any_tiled_pass()) cands.push_back(0);
    if (cands.size() == 1) {
      sp.colE = 8;
      tt.col_e[tune_key()] = 8;
      tuning = "col_E=8 (no tiled pass applies to this grid)";
      return;
    }
    // timed on the capture stream, which the host waits for before returning
    OnCaptureStream on(*this);
    hipLaunchKernelGGL((k_fill<R>), dim3(launch_blocks(2 * ns)), dim3(256), 0, s, 2 * ns, R(0), (R*)T.p);
    hipLaunchKernelGGL((k_fill<R>), dim3(launch_blocks(6 * ns)), dim3(256), 0, s, 6 * ns, R(0), (R*)U.p);
    NK_LAUNCHED();
    hipEvent_t e0, e1;
    NK_HIP(hipEventCreate(&e0));
    NK_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    int bestE = sp.colE;
    for (int ce : cands) {
      sp.colE = ce;
      hipGraph_t graph = nullptr;
      NK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      for (int r = 0; r < kTuneReps; ++r) {
        sp.deriv_cols(T.p, S1.p, S2.p);
        sp.div_cols(U.p, U.p + ns, U.p + 2 * ns, S2.p, Dsp.p);
      }
      NK_HIP(hipStreamEndCapture(s, &graph));
      hipGraphExec_t ex = nullptr;
      const hipError_t ie = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) throw HipError(NKREG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
      NK_HIP(hipGraphLaunch(ex, s));  // warm-up
      NK_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 3; ++r) NK_HIP(hipGraphLaunch(ex, s));
      NK_HIP(hipEventRecord(e1, s));
      NK_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      NK_HIP(hipEventElapsedTime(&ms, e0, e1));
      (void)hipGraphExecDestroy(ex);
      const float us_per_pass = 1e3f * ms / (3.0f * kTuneReps * (g.d == 2 ? 2 : 4));
      tuning += (tuning.empty() ? "" : ", ") + col_variant_name(ce) + ": " + std::to_string(us_per_pass) + " us/pass";
      if (ms < best) { best = ms; bestE = ce; }
    }
    sp.colE = bestE;
    tt.col_e[tune_key()] = bestE;
    tuning += "; chose " + col_variant_name(bestE);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  std::string col_symbols() const {
    std::string out;
    for (int axis = g.d - 2; axis >= 0; --axis)
      out += (out.empty() ? "\"" : ", \"") + sp.col_deriv_symbol(axis) + "\"";
    return out;
  }
  std::string describe() override {
    return std::string("{\"transport_precision\": ") + (kF64 ? "64" : "32") + ", \"graphs\": " +
           (use_graphs ? "true" : "false") + ", \"persistent_sweeps\": " + (small_sweeps ? "true" : "false") + ", \"sweep_timing\": \"" + sweep_timing + "\", \"assembly_sweeps\": \"" + assembly_timing + "\"" +
           ", \"spec_fused\": " + (sp64.spec_fused() ? "true" : "false") +
           ", \"row_E\": " + std::to_string(sp.rowE) + ", \"col_E\": " +
           std::to_string(sp.colE) + ", \"col_deriv_symbols\": [" + col_symbols() + "], \"autotune\": \"" + tuning +
           "\"}";
  }

  // One Gauss-Newton matvec as a sequence of launches on the current launch stream.
  void matvec_body(const void* vtin, void* out) {
    const double* vt = (const double*)vtin;
    const R* vl = kF64 ? (const R*)v.p : vR.p;
    const R* vtl = to_transport(vt, vtR);
    try {
      incremental_sweep(vl, vtl);
      if (full_newton) adjoint_sweep_k<true>(vl, vtl, R(-1), mt1.p, R(0), nullptr, F.p, false);
      else adjoint_sweep_k<false>(vl, nullptr, R(-1), mt1.p, R(0), nullptr, F.p, false);
    } catch (...) {
      state_valid = false;  // the slots may no longer hold what the next matvec expects
      held.assign(S, -1);
      throw;
    }
    hess_vecop(vt, (double*)out);
  }

  void precond(const void* r, void* z) override {
    sp64.vecop(OP_PINV, (const double*)r, nullptr, (double*)z, nc, cfg.reg, 0, cfg.beta, Xs.p, Ys.p);
  }
  void project(const void* f, void* out) override {
    sp64.vecop(OP_K, (const double*)f, nullptr, (double*)out, nc, cfg.reg, 1, cfg.beta, Xs.p, Ys.p);
  }
  void apply_reg(const void* x, void* out) override {
    sp64.vecop(OP_A, (const double*)x, nullptr, (double*)out, nc, cfg.reg, 0, cfg.beta, Xs.p, Ys.p);
  }
  void gradient(const void* u, void* gout) override {
    sp.gradient((const R*)u, (R*)gout, 1, T.p, S1.p, S2.p);
  }
  void divergence(const void* w, void* out) override {
    sp.divergence((const R*)w, (R*)out, U.p, S2.p, Dsp.p);
  }
  double dot(const void* a, const void* b, long long cnt) override {
    return red.one<double>(RED_DOT, (const double*)a, (const double*)b, cnt);
  }

  void axpby(long long cnt, double a, const double* x, double b, double* y) {
    hipLaunchKernelGGL((k_axpby<double>), dim3(launch_blocks(cnt)), dim3(256), 0, s, cnt, a, x, b, y);
    NK_LAUNCHED();
  }
  void lincomb(long long cnt, double a, const double* x, double b, const double* y, double* z) {
    hipLaunchKernelGGL((k_lincomb<double>), dim3(launch_blocks(cnt)), dim3(256), 0, s, cnt, a, x, b, y, z);
    NK_LAUNCHED();
  }

  // ---- PCG (textbook preconditioned CG, x0 = 0) ----
  // ---- PCG (x0 = 0; stop when |r| <= rtol |rhs|; non-positive curvature ends it) ----
  // Reduction slots: 0 = |r|^2, 1 = r.z (read by the next step), 2 = p.Hp. One host read
  // per iteration: the step length is formed on the device from p.Hp and r.z, and p.Hp
  // is checked when the new residual is read.
  struct PcgRun {
    double* x = nullptr;
    double nb = 0.0, tol = 0.0, rz = 0.0, rn = 0.0;
    int it = 0, maxit = 0;
    bool ok = false, active = false;
  } pr;
  bool pcg_begin(const void* rhsin, void* sout, double rtol, int maxit) override {
    if (!state_valid) throw HipError(NKREG_ESTATE, "no gradient computed at the current velocity");
    pr = PcgRun{};
    pr.x = (double*)sout;
    pr.maxit = maxit <= 0 ? (int)std::min<long long>(nv, 1 << 30) : maxit;
    hipLaunchKernelGGL((k_fill<double>), dim3(launch_blocks(nv)), dim3(256), 0, s, nv, 0.0, pr.x);
    NK_LAUNCHED();
    copy(kr.p, rhsin, nv * sizeof(double));
    pr.nb = std::sqrt(red.one<double>(RED_SUMSQ, kr.p, nullptr, nv));
    if (!std::isfinite(pr.nb)) throw HipError(NKREG_ENONFINITE, "right-hand side is not finite");
    if (pr.nb == 0.0) {
      pr.ok = true;
      return false;
    }
    pr.tol = rtol * pr.nb;
    precond(kr.p, kz.p);
    copy(kp.p, kz.p, nv * sizeof(double));
    red.enqueue<double>(RED_DOT, kr.p, kz.p, nv, 1);
    red.fetch(2);
    pr.rz = red.host[1];
    pr.rn = pr.nb;
    pr.ok = pr.rn <= pr.tol;
    pr.active = !pr.ok && pr.it < pr.maxit;
    return pr.active;
  }
  bool pcg_active() const override { return pr.active; }
  void route_launches(hipStream_t st) override { route(st ? st : user_s); }
  const void* pcg_p() const override { return kp.p; }
  void* pcg_q() override { return kq.p; }
  void pcg_step() override {
    red.enqueue<double>(RED_DOT, kp.p, kq.p, nv, 2);
    hipLaunchKernelGGL(k_pcg_step, dim3(launch_blocks(nv)), dim3(256), 0, s, nv, (const double*)red.result.p + 1,
                       (const double*)red.result.p + 2, (const double*)kp.p, (const double*)kq.p, pr.x, kr.p);
    NK_LAUNCHED();
    precond(kr.p, kz.p);
    red.enqueue_sumsq_dot<double>(kr.p, kz.p, nv, 0);   // |r|^2 and <r, z> in one pass
    NK_HIP(hipMemcpyAsync(red.host, red.result.p, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  void pcg_step_on(hipStream_t st) override {
    if (!use_graphs) {
      const hipStream_t prev = s;
      route(st);
      pcg_step();
      route(prev);
      return;
    }
    if (!step_graph.exec || step_graph.x != pr.x) {
      if (step_graph.exec) (void)hipGraphExecDestroy(step_graph.exec);
      step_graph = StepGraph{};
      const hipStream_t prev = s;
      hipGraph_t graph = nullptr;
      {
        OnCaptureStream on(*this);
        NK_HIP(hipStreamBeginCapture(cap_s, hipStreamCaptureModeThreadLocal));
        try {
          pcg_step();
        } catch (...) {
          (void)hipStreamEndCapture(cap_s, &graph);
          if (graph) (void)hipGraphDestroy(graph);
          route(prev);
          throw;
        }
        NK_HIP(hipStreamEndCapture(cap_s, &graph));
      }
      route(prev);
      hipGraphExec_t exec = nullptr;
      const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) throw HipError(NKREG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      step_graph.exec = exec;
      step_graph.x = pr.x;
    }
    NK_HIP(hipGraphLaunch(step_graph.exec, st));
  }
  void pcg_finish() override {
    const double pq = red.host[2];
    if (!std::isfinite(pq)) throw HipError(NKREG_ENONFINITE, "p.Hp is not finite");
    if (pq <= 0.0) {  // non-positive curvature ends the iteration (x and r were left unchanged)
      if (pr.it == 0) copy(pr.x, kp.p, nv * sizeof(double));  // then x = P^-1 rhs, a descent direction
      pr.active = false;
      return;
    }
    ++pr.it;
    pr.rn = std::sqrt(red.host[0]);
    const double rz_new = red.host[1];
    if (pr.rn <= pr.tol) {
      pr.ok = true;
      pr.active = false;
      return;
    }
    lincomb(nv, 1.0, kz.p, rz_new / pr.rz, kp.p, kp.p);
    pr.rz = rz_new;
    pr.active = pr.it < pr.maxit;
  }
  int pcg_result(int* iters, double* relres) const override {
    if (iters) *iters = pr.it;
    if (relres) *relres = pr.nb == 0.0 ? 0.0 : pr.rn / pr.nb;
    return pr.ok ? NKREG_OK : NKREG_ENOCONV;
  }
  int pcg(const void* rhsin, void* sout, double rtol, int maxit, int* iters, double* relres) override {
    pcg_begin(rhsin, sout, rtol, maxit);
    while (pr.active) {
      const Range iter("pcg iteration", pr.it);
      hessian_matvec(kp.p, kq.p);
      pcg_step();
      NK_HIP(hipStreamSynchronize(s));
      pcg_finish();
    }
    return pcg_result(iters, relres);
  }
  // Armijo backtracking along sbuf from alpha = 1 (c1 = 1e-4, at most 20
  // halvings; Section "Numerical Optimization"); gbuf holds the gradient at vk.
  bool armijo(const double* vk, double J, double* alpha_out, int* n_pde) {
    const double slope = g.hd * red.one<double>(RED_DOT, gbuf.p, sbuf.p, nv);
    double alpha = 1.0;
    for (int trial = 0; trial <= 20; ++trial) {
      lincomb(nv, 1.0, vk, alpha, sbuf.p, vtrial.p);
      const double Jt = trial_objective(vtrial.p);
      *n_pde += 1;
      if (Jt <= J + 1e-4 * alpha * slope) {
        *alpha_out = alpha;
        return true;
      }
      alpha *= 0.5;
    }
    *alpha_out = 0.0;
    return false;
  }
  // Halves sbuf until vk + sbuf satisfies the CFL bound (before the line search).
  void cfl_guard(const double* vk) {
    if (cfg.cfl_max <= 0) return;
    for (int h = 0; h < 30; ++h) {
      lincomb(nv, 1.0, vk, 1.0, sbuf.p, vtrial.p);
      if (cfl_number(vtrial.p) <= cfg.cfl_max) break;
      axpby(nv, 0.0, sbuf.p, 0.5, sbuf.p);
    }
  }

  // One row of the per-iterate history (nkreg_solve_opts::h_history) and, with verbose,
  // one line on stderr: k, J, J_dist, ||g||_inf, PCG iterations, alpha, the CFL number of
  // v_k and, when asked for, det F_1's extremes at v_k (an extra FP64 solve, which uses
  // buffers of its own and leaves the cached state alone).
  void log_iterate(const nkreg_solve_opts& opt, int& rows, const char* tag, int k, const double* vk, double J,
                   double Jd, double Jr, double ginf, double rel, int its, double alpha, int n_pde) {
    if (!opt.verbose && !(opt.h_history && rows < opt.history_cap)) return;
    const double cfl = cfl_number(vk);
    double st[4] = {NAN, NAN, NAN, NAN};
    if (opt.history_detf) det_grad_y(vk, nullptr, st);
    if (opt.h_history && rows < opt.history_cap) {
      double* row = opt.h_history + (size_t)rows * NKREG_HISTORY_COLS;
      const double vals[NKREG_HISTORY_COLS] = {(double)k, J,     Jd,  Jr,    ginf, (double)its,
                                               alpha,     (double)n_pde, cfl, st[0], st[1]};
      std::copy(vals, vals + NKREG_HISTORY_COLS, row);
      ++rows;
    }
    if (opt.verbose) {
      if (opt.history_detf)
        fprintf(stderr,
                "[nkreg] %s k=%d J=%.6e Jd=%.6e Jr=%.6e |g|inf=%.3e rel=%.3e cg=%d alpha=%g n_pde=%d cfl=%.3f "
                "detF=[%.4f, %.4f]\n",
                tag, k, J, Jd, Jr, ginf, rel, its, alpha, n_pde, cfl, st[0], st[1]);
      else
        fprintf(stderr, "[nkreg] %s k=%d J=%.6e Jd=%.6e Jr=%.6e |g|inf=%.3e rel=%.3e cg=%d alpha=%g n_pde=%d cfl=%.3f\n",
                tag, k, J, Jd, Jr, ginf, rel, its, alpha, n_pde, cfl);
    }
  }

  // ---- globalised Picard iteration (preconditioned gradient descent, e:picard) ----
  // s_k = -alpha~ P^-1 g_k (the Picard iterate minus v_k), Armijo from alpha = 1;
  // alpha~ shrinks by alpha after backtracking and doubles after alpha = 1.
  int picard(void* vio, const nkreg_solve_opts* o, const nkreg_picard_opts* po, nkreg_solve_report* rep) override {
    need_images();
    auto t0 = std::chrono::steady_clock::now();
    nkreg_solve_opts opt{};
    opt.max_outer = 500; opt.gtol = 1e-3;
    if (o) opt = *o;
    if (!(opt.gtol > 0)) throw HipError(NKREG_EINVAL, "the Picard iteration stops on the relative gradient rule (gtol > 0)");
    nkreg_picard_opts pop{};
    pop.memory = 1; pop.stagnation_count = 10; pop.stagnation_tol = 1e-6;
    if (po) pop = *po;
    nkreg_solve_report r{};
    double* vk = (double*)vio;
    double J, Jd, Jr;
    objective_gradient(vk, &J, &Jd, &Jr, gbuf.p);
    r.n_pde += 2;
    r.J0 = J;
    double ginf = red.one<double>(RED_MAXABS, gbuf.p, nullptr, nv);
    r.gnorm0_inf = ginf;
    const double g0inf = opt.gref_inf > 0 ? opt.gref_inf : ginf;
    double at = 1.0;
    int flat = 0, k = 0;
    bool conv = false;
    log_iterate(opt, r.history_rows, "picard", 0, vk, J, Jd, Jr, ginf, ginf / g0inf, 0, 0.0, r.n_pde);
    while (true) {
      if (ginf <= opt.gtol * g0inf || g0inf == 0.0) { conv = true; r.stop_reason = 1; break; }
      if (pop.stagnation_count > 0 && flat >= pop.stagnation_count) { conv = true; r.stop_reason = 6; break; }
      if (k >= opt.max_outer) { r.stop_reason = 4; break; }
      const Range outer("picard iteration", k);
      precond(gbuf.p, sbuf.p);
      axpby(nv, 0.0, sbuf.p, pop.memory ? -at : -1.0, sbuf.p);
      if (cfg.incompressible) project(sbuf.p, sbuf.p);
      if (opt.cfl_guard) cfl_guard(vk);
      double alpha = 0.0;
      if (!armijo(vk, J, &alpha, &r.n_pde)) { r.line_search_failed = 1; r.stop_reason = 5; break; }
      if (pop.memory) at = alpha < 1.0 ? at * alpha : 2.0 * at;
      axpby(nv, alpha, sbuf.p, 1.0, vk);
      const double Jprev = J;
      objective_gradient(vk, &J, &Jd, &Jr, gbuf.p);
      r.n_pde += 2;
      flat = std::fabs(Jprev - J) <= pop.stagnation_tol * (1.0 + r.J0) ? flat + 1 : 0;
      ginf = red.one<double>(RED_MAXABS, gbuf.p, nullptr, nv);
      ++k;
      log_iterate(opt, r.history_rows, "picard", k, vk, J, Jd, Jr, ginf, ginf / g0inf, 0, alpha, r.n_pde);
    }
    NK_HIP(hipStreamSynchronize(s));
    r.iterations = k;
    r.converged = conv ? 1 : 0;
    r.J = J; r.J_dist = Jd; r.J_reg = Jr;
    r.gnorm_inf = ginf;
    r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = r;
    return conv && !r.line_search_failed ? NKREG_OK : NKREG_ENOCONV;
  }

  // ---- outer iteration (GN-PCG, Armijo, relative-gradient or C1-C5 rule) ----
  int newton(void* vio, const nkreg_solve_opts* o, nkreg_solve_report* rep) override {
    need_images();
    auto t0 = std::chrono::steady_clock::now();
    nkreg_solve_opts opt{};
    opt.max_outer = 50; opt.gtol = 1e-3; opt.tau_J = 1e-3; opt.pcg_maxit = 0; opt.cfl_guard = 0;
    if (o) opt = *o;
    nkreg_solve_report r{};
    double* vk = (double*)vio;
    double J, Jd, Jr;
    objective_gradient(vk, &J, &Jd, &Jr, gbuf.p);
    r.n_pde += 2;
    r.J0 = J;
    const double gstart = red.one<double>(RED_MAXABS, gbuf.p, nullptr, nv);
    const double g0inf = opt.gref_inf > 0 ? opt.gref_inf : gstart;
    const double g0two = std::sqrt(red.one<double>(RED_SUMSQ, gbuf.p, nullptr, nv));
    r.gnorm0_inf = gstart;
    double ginf = gstart, gtwo = g0two;
    double Jprev = J;
    int k = 0;
    bool conv = false;
    log_iterate(opt, r.history_rows, "newton", 0, vk, J, Jd, Jr, ginf, ginf / g0inf, 0, 0.0, r.n_pde);
    const double eps = 2.220446049250313e-16;  // FP64 machine precision in C4 for both transports
    while (true) {
      if (opt.gtol > 0) {
        // relative gradient rule, at most max_outer iterations
        if (ginf <= opt.gtol * g0inf || g0inf == 0.0) { conv = true; r.stop_reason = 1; break; }
        if (k >= opt.max_outer) { r.stop_reason = 4; break; }
      } else {
        // e:stopping-criteria combined as e:converged, n_opt = max_outer:
        // (C1 and C2 and C3) or C4 or C5; C1-C3 compare two iterates
        const bool c4 = ginf < 1e3 * eps;
        const bool c5 = k > opt.max_outer;
        bool c123 = false;
        if (k > 0) {
          const double dv = red.one<double>(RED_MAXABS, sbuf.p, nullptr, nv);  // |v_{k-1} - v_k| = alpha |s|
          const double vinf = red.one<double>(RED_MAXABS, vk, nullptr, nv);
          const bool c1 = (Jprev - J) < opt.tau_J * (1.0 + r.J0);
          const bool c2 = dv < std::sqrt(opt.tau_J) * (1.0 + vinf);
          const bool c3 = ginf < std::cbrt(opt.tau_J) * (1.0 + r.J0);
          c123 = c1 && c2 && c3;
        }
        if (c123 || c4) { conv = true; r.stop_reason = c123 ? 2 : 3; break; }
        if (c5) { r.stop_reason = 4; break; }
      }
      const Range outer("newton outer iteration", k);
      const double eta = std::min(0.5, std::sqrt(gtwo / g0two));
      lincomb(nv, -1.0, gbuf.p, 0.0, gbuf.p, rhsbuf.p);
      int its = 0;
      double rr = 0;
      (void)pcg(rhsbuf.p, sbuf.p, eta, opt.pcg_maxit, &its, &rr);
      r.cg_iterations += its;
      r.n_pde += 2 * its;
      if (cfg.incompressible) project(sbuf.p, sbuf.p);
      if (opt.cfl_guard) cfl_guard(vk);
      double alpha = 0.0;
      if (!armijo(vk, J, &alpha, &r.n_pde)) { r.line_search_failed = 1; r.stop_reason = 5; break; }
      axpby(nv, alpha, sbuf.p, 1.0, vk);
      axpby(nv, 0.0, sbuf.p, alpha, sbuf.p);  // keep alpha*s for C2
      Jprev = J;
      objective_gradient(vk, &J, &Jd, &Jr, gbuf.p);
      r.n_pde += 2;
      ginf = red.one<double>(RED_MAXABS, gbuf.p, nullptr, nv);
      gtwo = std::sqrt(red.one<double>(RED_SUMSQ, gbuf.p, nullptr, nv));
      ++k;
      log_iterate(opt, r.history_rows, "newton", k, vk, J, Jd, Jr, ginf, ginf / g0inf, its, alpha, r.n_pde);
    }
    NK_HIP(hipStreamSynchronize(s));
    r.iterations = k;
    r.converged = conv ? 1 : 0;
    r.J = J; r.J_dist = Jd; r.J_reg = Jr;
    r.gnorm_inf = ginf;
    r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = r;
    if (r.line_search_failed) return NKREG_ENOCONV;
    return conv ? NKREG_OK : NKREG_ENOCONV;
  }

  // ---- Hessian analysis (Section "Spectral Analysis", Table t:eigenvalues) ----
  // Row j of H (nv x nv doubles) = H e_j, by nv matvecs at the cached state.
  bool state_ready() const override { return state_valid; }
  const double* velocity() const override { return v.p; }
  void images(const void** a, const void** b) const override {
    *a = mT.p;
    *b = mR.p;
  }

  void assemble_hessian(void* Hout) override {
    if (!state_valid) throw HipError(NKREG_ESTATE, "no gradient computed at the current velocity");
    double* H = (double*)Hout;
    DevBuf<double> e(nv), col(nv);
    for (long long j = 0; j < nv; ++j) {
      hipLaunchKernelGGL((k_unit<double>), dim3(launch_blocks(nv)), dim3(256), 0, s, nv, j, e.p);
      NK_LAUNCHED();
      hessian_matvec(e.p, col.p);
      NK_HIP(hipMemcpyAsync(H + (size_t)j * nv, col.p, nv * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    NK_HIP(hipStreamSynchronize(s));
  }

  // Lanczos on H (Euclidean inner product; H is symmetric) with full
  // reorthogonalisation, from a fixed pseudo-random start; returns the Ritz
  // values (ascending) of the tridiagonal matrix after at most `steps` steps.
  static constexpr int kMaxLanczos = 512;
  int lanczos(int steps, double* ritz, int* count) override {
    if (!state_valid) throw HipError(NKREG_ESTATE, "no gradient computed at the current velocity");
    if (steps <= 0 || steps > kMaxLanczos) throw HipError(NKREG_EINVAL, "Lanczos steps must lie in [1, 512]");
    const int m = (int)std::min<long long>(steps, nv);
    DevBuf<double> Q((size_t)(m + 1) * nv), w(nv), qin(nv), c(m + 1), part((size_t)(m + 1) * kDotParts);
    auto q = [&](int i) { return Q.p + (size_t)i * nv; };
    hipLaunchKernelGGL(k_hash_fill, dim3(launch_blocks(nv)), dim3(256), 0, s, nv, q(0));
    NK_LAUNCHED();
    axpby(nv, 0.0, q(0), 1.0 / std::sqrt(red.one<double>(RED_SUMSQ, q(0), nullptr, nv)), q(0));
    std::vector<double> a, b;
    double anorm = 0.0;
    for (int k = 0; k < m; ++k) {
      copy(qin.p, q(k), nv * sizeof(double));
      hessian_matvec(qin.p, w.p);
      const double ak = red.one<double>(RED_DOT, q(k), w.p, nv);
      a.push_back(ak);
      // w -= a_k q_k + b_k q_{k-1}, then twice Gram-Schmidt against q_0..q_k
      lincomb(nv, 1.0, w.p, -ak, q(k), w.p);
      if (k > 0) axpby(nv, -b.back(), q(k - 1), 1.0, w.p);
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_multidot_part, dim3(k + 1, kDotParts), dim3(256), 0, s, Q.p, (long long)nv, w.p,
                           part.p);
        hipLaunchKernelGGL(k_multidot_sum, dim3((k + 1 + 63) / 64), dim3(64), 0, s, part.p, kDotParts, k + 1, c.p);
        hipLaunchKernelGGL(k_multi_axpy, dim3(launch_blocks(nv)), dim3(256), 0, s, Q.p, k + 1, (long long)nv, c.p,
                           w.p);
        NK_LAUNCHED();
      }
      const double bk = std::sqrt(red.one<double>(RED_SUMSQ, w.p, nullptr, nv));
      anorm = std::max(anorm, std::fabs(ak) + bk + (b.empty() ? 0.0 : b.back()));
      if (k + 1 == m || !(bk > 1e-13 * anorm)) break;   // done, or an invariant subspace
      b.push_back(bk);
      lincomb(nv, 1.0 / bk, w.p, 0.0, w.p, q(k + 1));
    }
    const std::vector<double> ev = tridiagonal_eigenvalues(a, b);
    for (size_t i = 0; i < ev.size(); ++i) ritz[i] = ev[i];
    if (count) *count = (int)ev.size();
    return NKREG_OK;
  }
  // Eigenvalues (ascending) of the symmetric tridiagonal matrix with diagonal a
  // and off-diagonal b, by bisection on Sturm sequence counts.
  static std::vector<double> tridiagonal_eigenvalues(const std::vector<double>& a, const std::vector<double>& b) {
    const int m = (int)a.size();
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < m; ++i) {
      const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
      lo = std::min(lo, a[i] - r);
      hi = std::max(hi, a[i] + r);
    }
    // number of eigenvalues below x: negative pivots of the LDL^T factorisation of T - x I
    auto below = [&](double x) {
      int cnt = 0;
      double dprev = 1.0;
      for (int i = 0; i < m; ++i) {
        double di = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / dprev : 0.0);
        if (di == 0.0) di = -1e-300;
        if (di < 0) ++cnt;
        dprev = di;
      }
      return cnt;
    };
    std::vector<double> ev(m);
    const double tol = 4e-16 * std::max(std::fabs(lo), std::fabs(hi));
    for (int i = 0; i < m; ++i) {
      double l = lo, h = hi;
      for (int it = 0; it < 200 && h - l > tol; ++it) {
        const double mid = 0.5 * (l + h);
        if (below(mid) > i) h = mid;
        else l = mid;
      }
      ev[i] = 0.5 * (l + h);
    }
    return ev;
  }

  // ---- deformation gradient in FP64 ----
  // ---- beta continuation (Section "Parameter Selection") ----
  int continuation(void* vio, const double* betas, int levels, const nkreg_solve_opts* o,
                   nkreg_solve_report* reps) override {
    if (levels < 0 || (levels > 0 && !betas)) throw HipError(NKREG_EINVAL, "bad beta levels");
    for (int i = 0; i < levels; ++i)
      if (!(betas[i] > 0)) throw HipError(NKREG_EINVAL, "beta must be positive");
    nkreg_solve_opts so{};
    so.max_outer = 50; so.gtol = 1e-3; so.tau_J = 1e-3;
    if (o) so = *o;
    double gref = so.gref_inf;
    int status = NKREG_OK;
    for (int i = 0; i < levels; ++i) {
      set_beta(betas[i]);
      so.gref_inf = gref;
      nkreg_solve_report r{};
      if (newton(vio, &so, &r) != NKREG_OK) status = NKREG_ENOCONV;
      if (so.h_history) {  // the next level appends its rows
        so.h_history += (size_t)r.history_rows * NKREG_HISTORY_COLS;
        so.history_cap -= r.history_rows;
      }
      if (gref <= 0) gref = r.gnorm0_inf;
      if (reps) reps[i] = r;
    }
    return status;
  }

  // Parameter continuation in beta with a lower bound on det F_1 (Table
  // t:para-cont): decade descent, then arithmetic bisection between the last
  // accepted and the breaching beta; every trial warm-starts from the last
  // accepted solution.
  int beta_search(void* vio, const nkreg_beta_search_opts* oin, nkreg_beta_search_report* out) override {
    need_images();
    if (!oin) throw HipError(NKREG_EINVAL, "beta search options are required");
    nkreg_beta_search_opts o = *oin;
    if (!(o.eps_F > 0.0 && o.eps_F < 1.0)) throw HipError(NKREG_EINVAL, "eps_F must lie in (0, 1)");
    if (o.beta_start <= 0) o.beta_start = 1.0;
    if (o.beta_min <= 0) o.beta_min = 1e-6;
    if (o.dbeta_rel <= 0) o.dbeta_rel = 0.05;
    if (o.l2_rel_min <= 0) o.l2_rel_min = 1e-2;
    if (o.max_steps <= 0 || o.max_steps > NKREG_MAX_BETA_TRIALS) o.max_steps = NKREG_MAX_BETA_TRIALS;
    const auto t0 = std::chrono::steady_clock::now();
    nkreg_beta_search_report r{};
    double* v = (double*)vio;
    DevBuf<double> vstart(nv), vok(nv);
    copy(vstart.p, v, nv * sizeof(double));
    red.enqueue<R>(RED_SUMSQDIFF, mR.p, mT.p, n, 0);
    red.fetch(1);
    const double r0 = std::sqrt(red.host[0]);
    bool have_ok = false;
    double beta_ok = 0, det_ok = 0, l2_ok = 0;
    double gref = o.solve.gref_inf;
    auto trial = [&](double beta) -> bool {
      set_beta(beta);
      copy(v, have_ok ? vok.p : vstart.p, nv * sizeof(double));
      nkreg_solve_opts so = o.solve;
      so.h_history = nullptr;  // the search reports its trials instead
      so.gref_inf = gref;
      nkreg_solve_report nr{};
      newton(v, &so, &nr);
      if (gref <= 0) gref = nr.gnorm0_inf;
      double st[4];
      det_grad_y(v, nullptr, st);
      const double l2 = r0 > 0 ? std::sqrt(2.0 * nr.J_dist / g.hd) / r0 : 0.0;
      const bool acc = st[0] >= o.eps_F;
      const int k = r.steps++;
      r.trial_beta[k] = beta;
      r.trial_min_det[k] = st[0];
      r.trial_l2_rel[k] = l2;
      r.trial_accepted[k] = acc;
      r.newton_iterations += nr.iterations;
      r.cg_iterations += nr.cg_iterations;
      if (acc) {
        copy(vok.p, v, nv * sizeof(double));
        have_ok = true;
        beta_ok = beta;
        det_ok = st[0];
        l2_ok = l2;
      }
      return acc;
    };
    double beta = o.beta_start, breach = 0.0;
    while (true) {
      const double prev_l2 = l2_ok;
      const bool had_ok = have_ok;
      if (!trial(beta)) {
        breach = beta;
        break;
      }
      if (r.steps >= o.max_steps) { r.reason = 4; break; }
      if (had_ok && std::fabs(prev_l2 - l2_ok) < o.l2_rel_min * prev_l2) { r.reason = 2; break; }
      if (beta / 10.0 < o.beta_min) { r.reason = 3; break; }
      beta /= 10.0;
    }
    int status = NKREG_OK;
    if (breach > 0.0) {
      r.breached = 1;
      if (!have_ok) {
        r.reason = 5;
        status = NKREG_ENOCONV;
      } else {
        double lo = breach, hi = beta_ok;
        r.dbeta_min = o.dbeta_rel * breach;
        r.reason = 1;
        while ((hi - lo) / 2.0 >= r.dbeta_min) {
          if (r.steps >= o.max_steps) { r.reason = 4; break; }
          const double mid = (lo + hi) / 2.0;
          if (trial(mid)) hi = mid;
          else lo = mid;
        }
      }
    }
    if (have_ok) {
      copy(v, vok.p, nv * sizeof(double));
      set_beta(beta_ok);
      r.beta_star = beta_ok;
      r.min_det_star = det_ok;
      r.l2_rel_star = l2_ok;
    } else {
      r.beta_star = r.min_det_star = r.l2_rel_star = std::nan("");
    }
    NK_HIP(hipStreamSynchronize(s));
    r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (out) *out = r;
    return status;
  }

  void det_grad_y(const void* vin, void* detF, double* stats) override {
    Spectral<double>& q = sp64;
    const long long dd = (long long)d * d;
    DevBuf<double> vel((size_t)d * n), gv((size_t)dd * n), Fm((size_t)dd * n), Fs((size_t)dd * n),
        Ac((size_t)dd * n), gF((size_t)dd * d * n), det(n);
    DevBuf<cplx<double>> Tq((size_t)dd * g.nspec), S1q((size_t)dd * g.nspec), S2q((size_t)dd * g.nspec);
    const double* vl = (const double*)vin;
    const double h = 1.0 / nt;
    auto vel_at = [&](double t) {
      Weights w{};
      cheb_basis(nc, t, w.w);
      hipLaunchKernelGGL((k_vel_at<double>), dim3(launch_blocks((long long)d * n)), dim3(256), 0, s,
                         (long long)d * n, nc, vl, w, vel.p);
      NK_LAUNCHED();
      q.gradient(vel.p, gv.p, d, Tq.p, S1q.p, S2q.p);
    };
    if (d == 2) hipLaunchKernelGGL((k_identity_tensor<2>), dim3(launch_blocks(n)), dim3(256), 0, s, n, Fm.p);
    else hipLaunchKernelGGL((k_identity_tensor<3>), dim3(launch_blocks(n)), dim3(256), 0, s, n, Fm.p);
    NK_LAUNCHED();
    vel_at(0.0);
    for (int j = 0; j < nt; ++j) {
      if (nc > 1 && j > 0) vel_at(j * h);
      q.gradient(Fm.p, gF.p, (int)dd, Tq.p, S1q.p, S2q.p);
      if (d == 2) hipLaunchKernelGGL((k_defgrad_stage<2>), dim3(launch_blocks(n)), dim3(256), 0, s, n, h, vel.p, gv.p, Fm.p, gF.p, Ac.p, Fs.p, 0);
      else hipLaunchKernelGGL((k_defgrad_stage<3>), dim3(launch_blocks(n)), dim3(256), 0, s, n, h, vel.p, gv.p, Fm.p, gF.p, Ac.p, Fs.p, 0);
      NK_LAUNCHED();
      if (nc > 1) vel_at((j + 1) * h);
      q.gradient(Fs.p, gF.p, (int)dd, Tq.p, S1q.p, S2q.p);
      if (d == 2) hipLaunchKernelGGL((k_defgrad_stage<2>), dim3(launch_blocks(n)), dim3(256), 0, s, n, h, vel.p, gv.p, Fs.p, gF.p, Ac.p, Fm.p, 1);
      else hipLaunchKernelGGL((k_defgrad_stage<3>), dim3(launch_blocks(n)), dim3(256), 0, s, n, h, vel.p, gv.p, Fs.p, gF.p, Ac.p, Fm.p, 1);
      NK_LAUNCHED();
    }
    if (d == 2) hipLaunchKernelGGL((k_det<2>), dim3(launch_blocks(n)), dim3(256), 0, s, n, Fm.p, det.p);
    else hipLaunchKernelGGL((k_det<3>), dim3(launch_blocks(n)), dim3(256), 0, s, n, Fm.p, det.p);
    NK_LAUNCHED();
    // statistics: min, max, mean, population std (two passes for the std)
    const int nb = (int)std::max<long long>(1, std::min<long long>(kRedBlocks, (n + kRedThreads - 1) / kRedThreads));
    hipLaunchKernelGGL(k_stats, dim3(nb), dim3(kRedThreads), 0, s, det.p, n, 0.0, red.partial.p);
    NK_LAUNCHED();
    std::vector<double> part(4 * nb);
    NK_HIP(hipMemcpyAsync(part.data(), red.partial.p, 4 * nb * sizeof(double), hipMemcpyDeviceToHost, s));
    NK_HIP(hipStreamSynchronize(s));
    double mn = INFINITY, mx = -INFINITY, sum = 0.0;
    for (int b = 0; b < nb; ++b) {
      mn = std::min(mn, -part[b]);
      mx = std::max(mx, part[nb + b]);
      sum += part[2 * nb + b];
    }
    const double mean = sum / (double)n;
    hipLaunchKernelGGL(k_stats, dim3(nb), dim3(kRedThreads), 0, s, det.p, n, mean, red.partial.p);
    NK_LAUNCHED();
    NK_HIP(hipMemcpyAsync(part.data(), red.partial.p, 4 * nb * sizeof(double), hipMemcpyDeviceToHost, s));
    NK_HIP(hipStreamSynchronize(s));
    double ss = 0.0;
    for (int b = 0; b < nb; ++b) ss += part[3 * nb + b];
    if (stats) {
      stats[0] = mn; stats[1] = mx; stats[2] = mean; stats[3] = std::sqrt(ss / (double)n);
    }
    if (detF) NK_HIP(hipMemcpyAsync(detF, det.p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    NK_HIP(hipStreamSynchronize(s));
  }
};

// Handle factories, one per transport precision, each defined (and its kernels
// instantiated) in a translation unit of its own so the two compile in parallel.
ProblemBase* make_problem_f32(const nkreg_config& c, hipStream_t s);
ProblemBase* make_problem_f64(const nkreg_config& c, hipStream_t s);
inline ProblemBase* make_problem(const nkreg_config& c, hipStream_t s) {
  return c.precision == 32 ? make_problem_f32(c, s) : make_problem_f64(c, s);
}

}  // namespace nk
