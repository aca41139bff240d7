// Host-side launchers of the spectral pipelines on one grid and one stream.
#pragma once

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include <hip/hip_ext.h>

#include "kernels_wave.hpp"

namespace nk {

// Sets the text nkreg_last_error returns on this thread.
void set_last_error(const std::string& msg);

struct HipError : std::runtime_error {
  int code;
  HipError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define NK_HIP(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      throw ::nk::HipError(-4, std::string(#call) + ": " + hipGetErrorString(e_));           \
  } while (0)

#define NK_LAUNCHED()                                                                         \
  do {                                                                                        \
    hipError_t e_ = hipGetLastError();                                                        \
    if (e_ != hipSuccess) throw ::nk::HipError(-4, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

struct Grid {
  int d = 2;
  int n[3] = {1, 1, 1};
  long long npts = 0;    // real values per scalar field
  long long nspec = 0;   // complex values per scalar field (npts / 2)
  int L = 0;             // last axis length
  long long rows = 0;    // rows along the last axis
  int lmax = 0;          // longest axis (twiddle table length)
  double hd = 0.0;       // cell volume prod(2 pi / N_i)
};

// The column-pass variant NKREG_COL_E fixes for a grid: "8", "4" or "tiled" for every
// grid, or comma-separated grid=variant entries ("512x512=8,256x256x256=tiled") for
// the grids they name. -1 when nothing fixes it (the autotuner chooses).
inline int col_env_variant(const Grid& g) {
  const char* ce = std::getenv("NKREG_COL_E");
  if (!ce || !*ce) return -1;
  auto parse = [](const std::string& v) { return (v == "tiled" || v == "0") ? 0 : (v == "4" ? 4 : 8); };
  const std::string s(ce);
  if (s.find('=') == std::string::npos) return parse(s);
  std::string key = std::to_string(g.n[0]) + "x" + std::to_string(g.n[1]);
  if (g.d == 3) key += "x" + std::to_string(g.n[2]);
  size_t p = 0;
  while (p < s.size()) {
    size_t q = s.find(',', p);
    if (q == std::string::npos) q = s.size();
    const std::string e = s.substr(p, q - p);
    const size_t eq = e.find('=');
    if (eq != std::string::npos && e.substr(0, eq) == key) return parse(e.substr(eq + 1));
    p = q + 1;
  }
  return -1;
}

inline Grid make_grid(int d, const int* n) {
  Grid g;
  g.d = d;
  g.npts = 1;
  g.lmax = 0;
  g.hd = 1.0;
  for (int i = 0; i < d; ++i) {
    g.n[i] = n[i];
    g.npts *= n[i];
    g.lmax = std::max(g.lmax, n[i]);
    g.hd *= 2.0 * M_PI / n[i];
  }
  g.L = n[d - 1];
  g.rows = g.npts / g.L;
  g.nspec = g.npts / 2;
  return g;
}

// Complex elements per lane of the row-stage and column transforms.
constexpr int kRowE = 4;
// Complex elements per lane of an L-point real row transform (L / 2 complex points):
// kRowE, except 2 on 128- and 256-point rows. With 2, one wavefront holds one 256-point
// row (one 128-point row per half-wavefront) instead of two, which doubles the
// wavefronts in flight where rows are few (a 256 x 256 grid has 256 rows for 256 CUs)
// and shortens each wavefront's chain of loads and butterflies; the extra radix-2
// exchange passes cost less than that. row_e4 is the layout with kRowE everywhere.
constexpr int row_e4_n(int L) { return (L / 2 >= kRowE) ? kRowE : (L / 2 >= 4 ? 4 : 2); }
constexpr int row_e_n(int L) { return (L == 128 || L == 256) ? 2 : row_e4_n(L); }
template <int L>
constexpr int row_e4() { return row_e4_n(L); }
template <int L>
constexpr int row_e() { return row_e_n(L); }

// Kernel identifiers for launch timing: row-stage kinds are 0..10 (StageKind),
// column passes are 20 + ColMode.
constexpr int kColIdBase = 20;

// Records a pair of HIP events around every launch of one armed kernel and
// accumulates that launch's algorithmic bytes (field reads + writes).
struct KernelTimer {
  int armed = -1;
  int used = 0;
  double bytes = 0.0;
  std::vector<hipEvent_t> ev;
  ~KernelTimer() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  void arm(int id, int capacity) {
    if ((int)ev.size() < 2 * capacity) {
      const size_t old = ev.size();
      ev.resize(2 * capacity);
      for (size_t i = old; i < ev.size(); ++i) NK_HIP(hipEventCreate(&ev[i]));
    }
    armed = id;
    used = 0;
    bytes = 0.0;
  }
  bool want(int id) const { return id == armed && 2 * (used + 1) <= (int)ev.size(); }
  // Events of the next timed launch. They are handed to hipExtLaunchKernelGGL,
  // which stamps them with the dispatch's own start and end, so the elapsed
  // time is the kernel's execution time without the queue's dispatch latency.
  hipEvent_t start_event() const { return ev[2 * used]; }
  hipEvent_t stop_event() const { return ev[2 * used + 1]; }
  void done(double b) {
    ++used;
    bytes += b;
  }
  // average launch duration (ms) over the recorded launches; synchronises
  double average_ms() {
    if (used == 0) return 0.0;
    NK_HIP(hipEventSynchronize(ev[2 * used - 1]));
    double tot = 0.0;
    for (int i = 0; i < used; ++i) {
      float ms = 0.f;
      NK_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
      tot += ms;
    }
    return tot / used;
  }
};

// A kernel launch recorded for a batch group instead of being issued: the
// group (table) form of the kernel, its grid, this item's table entry and the
// arguments every item of a group shares. A batch replays each position of
// equal-shaped recordings as one launch over all items of the group.
struct LaunchRec {
  enum Kind { ROW, COL, FILL, CONV, SPEC, COPY, RED, REDF, SPECCOL };
  int kind = ROW;
  const void* kernel = nullptr;      // group form of the kernel
  dim3 grid, block;
  std::vector<unsigned char> entry;  // this item's table entry
  const void* tw = nullptr;          // ROW, COL: twiddle table (equal across a group)
  int iarg = 0;                      // ROW: lmax; COL, SPECCOL: twb; SPEC: op; REDF: partials
  int nfz = 1;                       // COL: fields per item
  ColArgs ca{};
  double scale = 0.0, fval = 0.0;    // COL scale, FILL value
  bool f64 = false;                  // precision of scale and fval
  long long cnt = 0;                 // FILL, CONV, RED element counts
  void* dst = nullptr;               // COPY (issued per item)
  const void* src = nullptr;
  size_t bytes = 0;
  // What the launch computes, for running it inside a persistent kernel instead:
  // ROW: stage kind, row length, dimension, stationary velocity; COL: mode, axis
  // length, elements per lane (0 = tiled); CONV: 1 = FP64 to FP32, 2 = FP32 to FP64.
  int stage = -1, len = 0, dim = 0, elems = 0, conv = 0;
  bool nc1 = false;
  template <typename T>
  void set_entry(const T& v) {
    entry.resize(sizeof(T));
    std::memcpy(entry.data(), &v, sizeof(T));
  }
  bool same_shape(const LaunchRec& o) const {
    return kind == o.kind && kernel == o.kernel && grid.x == o.grid.x && grid.y == o.grid.y &&
           grid.z == o.grid.z && block.x == o.block.x && iarg == o.iarg && nfz == o.nfz &&
           std::memcmp(&ca, &o.ca, sizeof(ColArgs)) == 0 && scale == o.scale && fval == o.fval && f64 == o.f64 &&
           cnt == o.cnt && entry.size() == o.entry.size() && bytes == o.bytes && stage == o.stage && len == o.len &&
           dim == o.dim && elems == o.elems && conv == o.conv && nc1 == o.nc1;
  }
};
// Time loops of a recorded operation (Recorder::mark).
enum TimeLoop { LOOP_NONE = 0, LOOP_STATE = 1, LOOP_INCREMENTAL = 2, LOOP_ADJOINT = 3 };

struct Recorder {
  std::vector<LaunchRec> recs;
  // Time-loop marks: the records from position pos on belong to iteration `step` of
  // time loop `loop` (0: outside every time loop), until the next mark.
  struct Mark {
    size_t pos;
    int loop, step;
  };
  std::vector<Mark> marks;
  void mark(int loop, int step) { marks.push_back({recs.size(), loop, step}); }
};

// Algorithmic bytes (fields read plus fields written) of every launch while set.
struct ByteTally {
  double bytes = 0.0;
  long long launches = 0;
  void add(double b) {
    bytes += b;
    ++launches;
  }
};

template <typename R>
class Spectral {
 public:
  Grid g;
  hipStream_t s = nullptr;
  cplx<R>* tw = nullptr;  // exp(-2 pi i m / lmax), m < lmax
  KernelTimer* timer = nullptr;
  Recorder* rec = nullptr;  // when set, launches are recorded instead of issued
  ByteTally* tally = nullptr;  // when set, every launch adds its algorithmic bytes
  // Column-pass variant, chosen by the autotuner: 8 or 4 = one workgroup per
  // column group with that many complex elements per lane (8: one wavefront per
  // 512-point column, 4: two); 0 = tiled through LDS (k_col_t) wherever the
  // axis is long enough and the columns split into whole tiles, else 8.
  int colE = 8;

  // Launches a kernel on the handle's stream; a timed launch carries the timer's events.
  template <typename... KArgs, typename... Args>
  void launch(void (*k)(KArgs...), dim3 grid, dim3 block, bool timed, Args... args) {
    if (timed)
      hipExtLaunchKernelGGL(k, grid, block, 0, s, timer->start_event(), timer->stop_event(), 0, args...);
    else
      hipLaunchKernelGGL(k, grid, block, 0, s, args...);
    NK_LAUNCHED();
  }

  // Twiddle table exp(-2 pi i m / lmax), m < lmax, computed in FP64 on the host.
  static void twiddles(int lmax, cplx<R>* h) {
    for (int m = 0; m < lmax; ++m) {
      const double a = -2.0 * M_PI * (double)m / (double)lmax;
      h[m] = {(R)std::cos(a), (R)std::sin(a)};
    }
  }

  Spectral() = default;
  Spectral(const Grid& grid, hipStream_t stream) : g(grid), s(stream) {
    read_col_env();
    read_row_env();
    std::vector<cplx<R>> h(g.lmax);
    twiddles(g.lmax, h.data());
    NK_HIP(hipMalloc(&tw, sizeof(cplx<R>) * g.lmax));
    owns_tw = true;
    NK_HIP(hipMemcpy(tw, h.data(), sizeof(cplx<R>) * g.lmax, hipMemcpyHostToDevice));
  }
  // Launchers over a twiddle table the caller provides (and keeps filled); allocates nothing.
  Spectral(const Grid& grid, hipStream_t stream, cplx<R>* table) : g(grid), s(stream), tw(table) {
    read_col_env();
    read_row_env();
  }
  // Complex elements per lane of this grid's row transforms (row_e); NKREG_ROW_E=4 keeps
  // four on every row length (the layout before 2 became the default on 128 and 256 points).
  int rowE = 0;
  void read_row_env() {
    const char* e = std::getenv("NKREG_ROW_E");
    rowE = (e && e[0] == '4') ? row_e4_n(g.L) : row_e_n(g.L);
  }
  Spectral(const Spectral&) = delete;
  Spectral& operator=(const Spectral&) = delete;
  ~Spectral() {
    if (tw && owns_tw) (void)hipFree(tw);
  }
  void read_col_env() {
    const int v = col_env_variant(g);
    if (v >= 0) colE = v;
    const char* f = std::getenv("NKREG_FUSED_SPEC");
    fuseSpec = !(f && f[0] == '0');
  }
  // The control-space multiplier as one fused column pass (k_col_spec) on 2D grids, except
  // with the 4-per-lane column variant (which rounds differently, so its handles keep the
  // separate passes). Launched and recorded alike, so batch items round like their
  // handles. NKREG_FUSED_SPEC=0 keeps the separate passes.
  bool fuseSpec = true;
  bool spec_fused() const { return fuseSpec && g.d == 2 && colE != 4; }
  bool owns_tw = false;

  // ---- column passes ----
  // axis 0 = x1 for any d; axis 1 = x2 for d = 3.
  // Length, outer count and stride (complex elements) of the columns along an axis.
  void col_geometry(int axis, int& N, int& outer, long long& inner) const {
    const int M = g.L / 2;
    if (g.d == 2) { N = g.n[0]; outer = 1; inner = M; }
    else if (axis == 0) { N = g.n[0]; outer = 1; inner = (long long)g.n[1] * M; }
    else { N = g.n[1]; outer = g.n[0]; inner = M; }
  }
  // Columns per tile of the tiled pass: one cache line (128 bytes) of each row,
  // halved until the tile data stays within 40 KiB of LDS, at least 4.
  static constexpr int tile_ct_n(int N) {
    int ct = 128 / (int)sizeof(cplx<R>);
    while (ct > 4 && (long long)N * ct * (long long)sizeof(cplx<R>) > 40960) ct /= 2;
    return ct;
  }
  template <int N>
  static constexpr int tile_ct() { return tile_ct_n(N); }
  static bool tile_ok(int N, long long inner) { return N >= 64 && inner % tile_ct_n(N) == 0; }
  // True if the tiled variant applies to at least one column pass of this grid.
  bool any_tiled_pass() const {
    for (int axis = 0; axis < g.d - 1; ++axis) {
      int N, outer;
      long long inner;
      col_geometry(axis, N, outer, inner);
      if (tile_ok(N, inner)) return true;
    }
    return false;
  }
  // Kernel symbol of the derivative pass along an axis with the current variant.
  std::string col_deriv_symbol(int axis) const {
    int N, outer;
    long long inner;
    col_geometry(axis, N, outer, inner);
    const std::string t = sizeof(R) == 4 ? "float" : "double";
    if (colE == 0 && tile_ok(N, inner))
      return "k_col_t<" + t + ", " + std::to_string(N) + ", " + std::to_string(tile_ct_n(N)) + ", 2>";
    return "k_col_w<" + t + ", " + std::to_string(N) + ", " + std::to_string(colE == 4 ? 4 : 8) + ", 2>";
  }

  void col(int mode, int axis, const cplx<R>* in, const cplx<R>* add, cplx<R>* out, int nf, R scale) {
    int N, outer;
    long long inner;
    col_geometry(axis, N, outer, inner);
    switch (N) {
      case 8: col_n<8>(mode, in, add, out, nf, scale, outer, inner); break;
      case 16: col_n<16>(mode, in, add, out, nf, scale, outer, inner); break;
      case 32: col_n<32>(mode, in, add, out, nf, scale, outer, inner); break;
      case 64: col_n<64>(mode, in, add, out, nf, scale, outer, inner); break;
      case 128: col_n<128>(mode, in, add, out, nf, scale, outer, inner); break;
      case 256: col_n<256>(mode, in, add, out, nf, scale, outer, inner); break;
      case 512: col_n<512>(mode, in, add, out, nf, scale, outer, inner); break;
      default: throw HipError(-2, "unsupported axis length");
    }
  }

  // Forward column transforms, multiplier and inverse column transforms of the 2D
  // spectra a.X (and a.Y) into a.out, one launch.
  void col_spec(const SpecArgs<R>& a, int op, int nf) {
    switch (g.n[0]) {
      case 8: col_spec_n<8>(a, op, nf); break;
      case 16: col_spec_n<16>(a, op, nf); break;
      case 32: col_spec_n<32>(a, op, nf); break;
      case 64: col_spec_n<64>(a, op, nf); break;
      case 128: col_spec_n<128>(a, op, nf); break;
      case 256: col_spec_n<256>(a, op, nf); break;
      case 512: col_spec_n<512>(a, op, nf); break;
      default: throw HipError(-2, "unsupported axis length");
    }
  }
  template <int N>
  void col_spec_n(const SpecArgs<R>& a, int op, int nf) {
    // one component per wavefront unless the op mixes them (K, the Stokes Hessian)
    switch (op) {
      case OP_HESS:
        if (!a.Y) throw HipError(-1, "the Hessian multiplier needs the body force");
        if (a.proj) col_spec_k<N, true, 2, OP_HESS>(a, nf);
        else col_spec_k<N, true, 1, OP_HESS>(a, nf);
        break;
      case OP_PINV: col_spec_k<N, false, 1, OP_PINV>(a, nf); break;
      case OP_A: col_spec_k<N, false, 1, OP_A>(a, nf); break;
      case OP_K: col_spec_k<N, false, 2, OP_K>(a, nf); break;
      default: throw HipError(-1, "unknown spectral multiplier");
    }
  }
  template <int N, bool HAS_Y, int DW, int OP>
  void col_spec_k(const SpecArgs<R>& a, int nf) {
    constexpr int SPW = ColShape<N, 8>::SPW;
    const int inner = g.L / 2;
    const dim3 grid((unsigned)((inner + SPW - 1) / SPW), (unsigned)(a.nc * (2 / DW)));
    const int twb = g.lmax / N;
    if (rec) {
      LaunchRec r;
      r.kind = LaunchRec::SPECCOL;
      r.kernel = (const void*)k_col_spec_t<R, N, HAS_Y, DW, OP>;
      r.grid = grid;
      r.block = dim3(64);
      r.iarg = twb;
      r.ca.inner = inner;
      r.tw = tw;
      r.f64 = sizeof(R) == 8;
      r.set_entry(a);
      rec->recs.push_back(r);
      return;
    }
    if (tally) tally->add((double)nf * g.nspec * sizeof(cplx<R>) * (HAS_Y ? 3 : 2));
    hipLaunchKernelGGL((k_col_spec<R, N, HAS_Y, DW, OP>), grid, dim3(64), 0, s, a, inner, (const cplx<R>*)tw, twb);
    NK_LAUNCHED();
  }

  // ---- row stages ----
  template <int KIND>
  void row(StageArgs<R>& a, int nf) {
    a.n = g.npts;
    if (g.d == 2) row_d<KIND, 2>(a, nf);
    else row_d<KIND, 3>(a, nf);
  }

  // ---- composite pipelines ----
  // S1 (and S2 in 3D) = column derivatives of the row spectrum T.
  void deriv_cols(const cplx<R>* T, cplx<R>* S1, cplx<R>* S2, int nf = 1) {
    if (g.d == 3) col(COL_DERIV, 1, T, nullptr, S2, nf, R(1) / R(g.n[1]));
    col(COL_DERIV, 0, T, nullptr, S1, nf, R(1) / R(g.n[0]));
  }
  // D = row spectrum of div(w) from U0, U1 (2D: U1 already times ik_2) [, U2 times ik_3].
  void div_cols(const cplx<R>* U0, const cplx<R>* U1, const cplx<R>* U2, cplx<R>* tmp, cplx<R>* D) {
    if (g.d == 2) {
      col(COL_DERIV, 0, U0, U1, D, 1, R(1) / R(g.n[0]));
    } else {
      col(COL_DERIV, 1, U1, U2, tmp, 1, R(1) / R(g.n[1]));
      col(COL_DERIV, 0, U0, tmp, D, 1, R(1) / R(g.n[0]));
    }
  }

  void r2c(const R* in, cplx<R>* out, int nf) {
    StageArgs<R> a{};
    a.src_a = in;
    a.out0 = out;
    a.fstride_in = g.npts;
    a.fstride_out = g.nspec;
    row<ST_R2C>(a, nf);
  }
  // R2C of nf fields of X into Xs and nf fields of Y (or of Yf, FP32) into Ys, one launch.
  void r2c2(const R* X, cplx<R>* Xs, const R* Y, const float* Yf, cplx<R>* Ys, int nf) {
    StageArgs<R> a{};
    a.src_a = X;
    a.src_b = Yf ? nullptr : Y;
    a.src_bf = Yf;
    a.split = nf;
    a.out0 = Xs;
    a.out1 = Ys;
    a.fstride_in = g.npts;
    a.fstride_out = g.nspec;
    row<ST_R2C>(a, 2 * nf);
  }
  void c2r(const cplx<R>* in, R* out, int nf, R scale) {
    StageArgs<R> a{};
    a.spec = in;
    a.out_real = out;
    a.scale = scale;
    a.fstride_in = g.nspec;
    a.fstride_out = g.npts;
    row<ST_C2R>(a, nf);
  }

  // g (nf x d fields) = gradient of nf scalar fields u; T, S1, S2 hold nf spectra each.
  void gradient(const R* u, R* out, int nf, cplx<R>* T, cplx<R>* S1, cplx<R>* S2) {
    r2c(u, T, nf);
    deriv_cols(T, S1, S2, nf);
    StageArgs<R> a{};
    a.spec = T; a.s1 = S1; a.s2 = S2;
    a.out_real = out;
    a.scale = R(1);
    a.fstride_in = g.nspec;
    a.fstride_out = (long long)g.d * g.npts;
    row<ST_GRAD>(a, nf);
  }

  // s = div w for one vector field w (d fields); U holds d spectra, tmp/D one each.
  void divergence(const R* w, R* out, cplx<R>* U, cplx<R>* tmp, cplx<R>* D) {
    r2c(w, U, g.d);
    ik_last(U + (g.d - 1) * g.nspec);  // the last component is differentiated in the row domain
    div_cols(U, U + g.nspec, g.d == 3 ? U + 2 * g.nspec : nullptr, tmp, D);
    StageArgs<R> b{};
    b.spec = D;
    b.out_real = out;
    b.scale = R(1);
    b.fstride_in = g.nspec;
    b.fstride_out = g.npts;
    row<ST_DIV>(b, 1);
  }

  // in-place multiplication of one row spectrum by i k_last (Nyquist and k = 0 -> 0)
  void ik_last(cplx<R>* T);

  // out (nc x d fields) = op(X, Y); Xs, Ys workspace of nc*d spectra each.
  // out = the op's multiplier applied to X (and Y: OP_HESS), all [nc][d] fields; Y may
  // instead be given in FP32 (Yf), which the R2C widens as it reads.
  void vecop(int op, const R* X, const R* Y, R* out, int nc, int reg, int proj, R beta, cplx<R>* Xs,
             cplx<R>* Ys, const float* Yf = nullptr) {
    const int nf = nc * g.d;
    const bool hasY = Y || Yf;
    if (hasY) r2c2(X, Xs, Y, Yf, Ys, nf);
    else r2c(X, Xs, nf);
    SpecArgs<R> a{};
    a.X = Xs; a.Y = hasY ? Ys : nullptr; a.out = Xs;
    a.n1 = g.n[0]; a.n2 = g.n[1]; a.n3 = g.d == 3 ? g.n[2] : 1;
    a.d = g.d; a.nc = nc; a.reg = reg; a.proj = proj;
    a.beta = beta;
    double sc = 1.0;
    for (int i = 0; i < g.d - 1; ++i) sc /= g.n[i];
    a.scale = (R)sc;
    a.nspec = g.nspec;
    if (spec_fused()) {
      // 2D launches: the column transforms and the multiplier in one pass (same bits)
      col_spec(a, op, nf);
      c2r(Xs, out, nf, R(1));
      return;
    }
    if (g.d == 3) {
      col(COL_FWD, 1, Xs, nullptr, Xs, nf, R(1));
      if (hasY) col(COL_FWD, 1, Ys, nullptr, Ys, nf, R(1));
    }
    col(COL_FWD, 0, Xs, nullptr, Xs, nf, R(1));
    if (hasY) col(COL_FWD, 0, Ys, nullptr, Ys, nf, R(1));
    const long long work = (long long)nc * g.nspec;
    const int blocks = (int)std::min<long long>((work + 255) / 256, 4096);
    if (rec) {
      LaunchRec r;
      r.kind = LaunchRec::SPEC;
      r.kernel = g.d == 2 ? (const void*)k_spec_mul_t<R, 2> : (const void*)k_spec_mul_t<R, 3>;
      r.grid = dim3(blocks);
      r.block = dim3(256);
      r.iarg = op;
      r.set_entry(a);
      rec->recs.push_back(r);
    } else {
      if (tally) tally->add((double)nf * g.nspec * sizeof(cplx<R>) * (hasY ? 3 : 2));
      if (g.d == 2) hipLaunchKernelGGL((k_spec_mul<R, 2>), dim3(blocks), dim3(256), 0, s, a, op);
      else hipLaunchKernelGGL((k_spec_mul<R, 3>), dim3(blocks), dim3(256), 0, s, a, op);
      NK_LAUNCHED();
    }
    col(COL_INV, 0, Xs, nullptr, Xs, nf, R(1));
    if (g.d == 3) col(COL_INV, 1, Xs, nullptr, Xs, nf, R(1));
    c2r(Xs, out, nf, R(1));
  }

 private:
  // Column transforms: one or two wavefronts per column workgroup.
  void record_col(const void* k, dim3 grid, dim3 block, int nf, const ColArgs& a, R scale, int twb,
                  const cplx<R>* in, const cplx<R>* add, cplx<R>* out) {
    LaunchRec r;
    r.kind = LaunchRec::COL;
    r.kernel = k;
    r.grid = grid;
    r.block = block;
    r.nfz = nf;
    r.ca = a;
    r.scale = (double)scale;
    r.f64 = sizeof(R) == 8;
    r.tw = tw;
    r.iarg = twb;
    r.set_entry(ColPtrs<R>{in, add, out, 0});
    rec->recs.push_back(r);
  }
  template <int N>
  void col_n(int mode, const cplx<R>* in, const cplx<R>* add, cplx<R>* out, int nf, R scale, int outer,
             long long inner) {
    if constexpr (N >= 64) {
      if (colE == 0 && tile_ok(N, inner)) {
        col_tiled<N>(mode, in, add, out, nf, scale, outer, inner);
        return;
      }
    }
    if (colE == 4 && N >= 8) col_ne<N, 4>(mode, in, add, out, nf, scale, outer, inner);
    else col_ne<N, 8>(mode, in, add, out, nf, scale, outer, inner);
  }
  template <int N>
  void col_tiled(int mode, const cplx<R>* in, const cplx<R>* add, cplx<R>* out, int nf, R scale, int outer,
                 long long inner) {
    constexpr int CT = tile_ct<N>();
    using TS = TileShape<R, N, CT>;
    ColArgs a{};
    a.inner = (int)inner;
    a.ctile = CT;
    a.field = g.nspec;
    a.ntx = (int)(inner / CT);
    a.ntiles = a.ntx * outer;
    dim3 grid((unsigned)a.ntiles, 1u, (unsigned)nf);
    const int twb = g.lmax / N;
    if (rec) {
      const void* k = mode == COL_FWD   ? (const void*)k_col_tt<R, N, CT, COL_FWD>
                      : mode == COL_INV ? (const void*)k_col_tt<R, N, CT, COL_INV>
                                        : (const void*)k_col_tt<R, N, CT, COL_DERIV>;
      record_col(k, grid, dim3(TileShape<R, N, CT>::NT), nf, a, scale, twb, in, add, out);
      rec->recs.back().stage = mode;
      rec->recs.back().len = N;
      rec->recs.back().elems = 0;
      return;
    }
    const bool timed = timer && timer->want(kColIdBase + mode);
    if (tally) tally->add((double)nf * g.nspec * sizeof(cplx<R>) * (add ? 3 : 2));
    const cplx<R>* twc = tw;
    switch (mode) {
      case COL_FWD: launch(k_col_t<R, N, CT, COL_FWD>, grid, dim3(TileShape<R, N, CT>::NT), timed, in, add, out, a, scale, twc, twb); break;
      case COL_INV: launch(k_col_t<R, N, CT, COL_INV>, grid, dim3(TileShape<R, N, CT>::NT), timed, in, add, out, a, scale, twc, twb); break;
      default: launch(k_col_t<R, N, CT, COL_DERIV>, grid, dim3(TileShape<R, N, CT>::NT), timed, in, add, out, a, scale, twc, twb); break;
    }
    if (timed) timer->done((double)nf * g.nspec * sizeof(cplx<R>) * (add ? 3 : 2));
  }
  template <int N, int E>
  void col_ne(int mode, const cplx<R>* in, const cplx<R>* add, cplx<R>* out, int nf, R scale, int outer,
              long long inner) {
    using CS = ColShape<N, E>;
    constexpr int SPW = CS::SPW;
    ColArgs a{};
    a.inner = (int)inner;
    a.ctile = SPW;
    a.field = g.nspec;
    dim3 grid((unsigned)((inner + SPW - 1) / SPW), (unsigned)outer, (unsigned)nf);
    const int twb = g.lmax / N;
    if (rec) {
      const void* k = mode == COL_FWD   ? (const void*)k_col_wt<R, N, E, COL_FWD>
                      : mode == COL_INV ? (const void*)k_col_wt<R, N, E, COL_INV>
                                        : (const void*)k_col_wt<R, N, E, COL_DERIV>;
      record_col(k, grid, dim3(CS::NT), nf, a, scale, twb, in, add, out);
      rec->recs.back().stage = mode;
      rec->recs.back().len = N;
      rec->recs.back().elems = E;
      return;
    }
    const bool timed = timer && timer->want(kColIdBase + mode);
    if (tally) tally->add((double)nf * g.nspec * sizeof(cplx<R>) * (add ? 3 : 2));
    switch (mode) {
      case COL_FWD:
        launch(k_col_w<R, N, E, COL_FWD>, grid, dim3(CS::NT), timed, in, add, out, a, scale, (const cplx<R>*)tw, twb);
        break;
      case COL_INV:
        launch(k_col_w<R, N, E, COL_INV>, grid, dim3(CS::NT), timed, in, add, out, a, scale, (const cplx<R>*)tw, twb);
        break;
      default:
        launch(k_col_w<R, N, E, COL_DERIV>, grid, dim3(CS::NT), timed, in, add, out, a, scale, (const cplx<R>*)tw,
               twb);
        break;
    }
    if (timed) timer->done((double)nf * g.nspec * sizeof(cplx<R>) * (add ? 3 : 2));
  }

  template <int KIND, int D>
  void row_d(StageArgs<R>& a, int nf) {
    switch (g.L) {
      case 8: row_l<KIND, D, 8>(a, nf); break;
      case 16: row_l<KIND, D, 16>(a, nf); break;
      case 32: row_l<KIND, D, 32>(a, nf); break;
      case 64: row_l<KIND, D, 64>(a, nf); break;
      case 128: row_l<KIND, D, 128>(a, nf); break;
      case 256: row_l<KIND, D, 256>(a, nf); break;
      case 512: row_l<KIND, D, 512>(a, nf); break;
      default: throw HipError(-2, "unsupported row length");
    }
  }

  template <int KIND, int D, int L>
  void row_l(StageArgs<R>& a, int nf) {
    constexpr int E = row_e<L>();
    constexpr int E4 = row_e4<L>();
    if constexpr (E != E4) {
      if (rowE == E4) {
        row_le<KIND, D, L, E4>(a, nf);
        return;
      }
    }
    row_le<KIND, D, L, E>(a, nf);
  }

  template <int KIND, int D, int L, int E>
  void row_le(StageArgs<R>& a, int nf) {
    constexpr int SPW = 64 / WavePlan<L / 2, E>::LS;
    dim3 grid((unsigned)((g.rows + SPW - 1) / SPW), (unsigned)nf);
    constexpr int BK = base_kind(KIND);
    constexpr bool uses_nc = (BK == ST_FWD1 || BK == ST_FWD2 || BK == ST_INC1 || BK == ST_INC2 ||
                              BK == ST_ADJINIT || BK == ST_ADJ1 || BK == ST_ADJ2);
    if (rec) {
      LaunchRec r;
      r.kind = LaunchRec::ROW;
      if (!uses_nc || a.nc <= 1) r.kernel = (const void*)k_row_wt<R, L, E, KIND, D, true>;
      else if constexpr (uses_nc) r.kernel = (const void*)k_row_wt<R, L, E, KIND, D, false>;
      r.grid = grid;
      r.block = dim3(64);
      r.tw = tw;
      r.iarg = g.lmax;
      r.f64 = sizeof(R) == 8;
      r.stage = KIND;
      r.len = L;
      r.dim = D;
      r.nc1 = !uses_nc || a.nc <= 1;
      r.set_entry(a);
      rec->recs.push_back(r);
      return;
    }
    const bool timed = timer && timer->want(KIND);
    if (tally) {
      double b = (double)nf * stage_fields<KIND>(a, D) * g.npts * sizeof(R);
      // fields read in FP32 by a two-source R2C
      if (KIND == ST_R2C && a.src_bf) b -= (double)(nf - a.split) * g.npts * (sizeof(R) - sizeof(float));
      tally->add(b);
    }
    if (!uses_nc || a.nc <= 1)
      launch(k_row_w<R, L, E, KIND, D, true>, grid, dim3(64), timed, a, (const cplx<R>*)tw, g.lmax);
    else if constexpr (uses_nc)
      launch(k_row_w<R, L, E, KIND, D, false>, grid, dim3(64), timed, a, (const cplx<R>*)tw, g.lmax);
    if (timed) timer->done((double)nf * stage_fields<KIND>(a, D) * g.npts * sizeof(R));
  }

  // Scalar fields (real field or row spectrum, same size) one launch of a row
  // stage reads plus writes, per batch item.
  template <int KIND>
  static double stage_fields(const StageArgs<R>& a, int D) {
    const double v = (double)a.nc * D;  // velocity coefficient fields
    switch (KIND) {
      case ST_FWD1: return D + 1 + v + (a.g0w ? D : 0) + 2;
      case ST_FWD2: return D + v + 1 + (a.g1w ? D : 0) + 2;
      case ST_INC1: return (a.zero_state ? 0 : D + 1) + 2 * v + D + 2 + (a.g0w ? D : 0);
      case ST_INC2: return D + 2 * v + D + 1 + 2 + (a.g1w ? D : 0);
      case ST_ADJINIT: return (a.src_b ? 2 : 1) + v + 1 + D;
      case ST_ADJ1: return 1 + 1 + 2 * D + 2 * v + 1 + D + v + (a.lamw0 ? 2 : 0);
      case ST_ADJ2: return a.skip_out ? 3 : 2 + v + 1 + D;
      case ST_NADJINIT: return (a.src_b ? 2 : 1) + 2 * v + 2 + D;
      case ST_NADJ1: return 1 + 1 + 4 * D + 2 * v + 1 + D + 2 * v + 2;
      case ST_NADJ2: return a.skip_out ? 3 : 2 + 2 * v + 2 + D;
      case ST_R2C: case ST_C2R: case ST_DIV: return 2;
      case ST_GRAD: return D + D;
      default: return 0;
    }
  }
};

template <typename R>
__global__ void k_ik_last(cplx<R>* T, long long rows, int M) {
  const long long tot = rows * M;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (long long)gridDim.x * blockDim.x) {
    const int q = (int)(i % M);
    T[i] = q == 0 ? cplx<R>{R(0), R(0)} : cmul_i(T[i], R(q));
  }
}

template <typename R>
void Spectral<R>::ik_last(cplx<R>* T) {
  const long long tot = g.nspec;
  const int blocks = (int)std::min<long long>((tot + 255) / 256, 4096);
  if (rec) throw HipError(-1, "ik_last cannot be recorded for a batch group");
  hipLaunchKernelGGL((k_ik_last<R>), dim3(blocks), dim3(256), 0, s, T, g.rows, g.L / 2);
  NK_LAUNCHED();
}

}  // namespace nk
