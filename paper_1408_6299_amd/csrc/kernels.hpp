// Kernels of the transport sweeps and spectral operators.
//
// Spectral layout ("row spectrum"): every row along the contiguous last axis
// (length L) is stored as its packed half spectrum, L/2 complex values:
// P[0] = (X_0, X_{L/2}) and P[q] = X_q for 0 < q < L/2. A real field and its
// row spectrum have the same size. Transforms along the other axes act on the
// row spectrum in place of a full spectrum; the packed column q = 0 carries two
// real sequences as one complex sequence, which a first derivative along
// another axis (a purely imaginary, odd multiplier) keeps intact.
//
// All transforms are unnormalised; the 1/N factors are folded into the
// derivative multipliers (1/N_axis), the row C2R epilogues (1/L) or the
// spectral multiplier (1/prod N).
#pragma once

#include "common.hpp"

namespace nk {

// ---------------------------------------------------------------------------
// Column pass: FFT along a strided axis of a row spectrum (kernel k_col_w in
// kernels_wave.hpp). Field layout: element (o, x, c) at o * (N * inner) + x * inner + c.
// ---------------------------------------------------------------------------
enum ColMode { COL_FWD = 0, COL_INV = 1, COL_DERIV = 2 };

struct ColArgs {
  int inner;        // complex elements between consecutive x
  int ctile;        // columns per workgroup (per tile for the tiled pass)
  long long field;  // complex elements between fields (blockIdx.z)
  int ntx;          // tiled pass: tiles across the inner extent
  int ntiles;       // tiled pass: tiles per field (ntx * outer)
};

// ---------------------------------------------------------------------------
// Row stage: per row of the last axis, (1) C2R of KIN input row spectra,
// (2) a pointwise epilogue (Heun stage, forcing, body force, ...),
// (3) R2C of KOUT new real rows. One kernel per RK2 stage of every sweep;
// the kernel itself is k_row_w (kernels_wave.hpp).
// ---------------------------------------------------------------------------
enum StageKind {
  ST_FWD1 = 0,   // state, stage 1: store grad m^j, acc = m + h/2 r1, out m + h r1
  ST_FWD2 = 1,   // state, stage 2: store grad m*_j, m^{j+1} = acc + h/2 r2 (real and spectrum)
  ST_INC1 = 2,   // incremental state, stage 1 (forcing -v~(t_j) . grad m^j)
  ST_INC2 = 3,   // incremental state, stage 2 (forcing -v~(t_{j+1}) . grad m*_j)
  ST_ADJINIT = 4,// lam = a*src_a + b*src_b; out v(t_nt) lam
  ST_ADJ1 = 5,   // adjoint stage 1: s1 = div(v(t_{j+1}) lam); body force; out v(t_j) lam*
  ST_ADJ2 = 6,   // adjoint stage 2: lam^j = acc + h/2 s2; out v(t_j) lam^j
  ST_R2C = 7,    // plain R2C of a batch of real fields
  ST_C2R = 8,    // plain C2R of a batch of row spectra (times scale)
  ST_GRAD = 9,   // write the gradient of a batch of scalar fields
  ST_DIV = 10,   // write the divergence (already summed spectrum) as a real field
  // Full-Newton incremental adjoint (e:sec-order-iadj): the adjoint kinds with the
  // lambda terms kept. Outputs v lam~ + v~ lam (lam from the gradient's adjoint
  // solve); stage 1 adds lam* grad m~^j + lam grad m~*_j to the body force.
  ST_NADJINIT = 11,
  ST_NADJ1 = 12,
  ST_NADJ2 = 13
};

// The adjoint kind a full-Newton kind extends (identity for the others).
__host__ __device__ constexpr int base_kind(int k) {
  return k == ST_NADJINIT ? ST_ADJINIT : (k == ST_NADJ1 ? ST_ADJ1 : (k == ST_NADJ2 ? ST_ADJ2 : k));
}
__host__ __device__ constexpr bool newton_kind(int k) { return k >= ST_NADJINIT && k <= ST_NADJ2; }

template <typename R>
struct StageArgs {
  const cplx<R>* spec;       // T / T* (grad kinds) or D (adjoint kinds) or batch input
  const cplx<R>* s1;         // column derivative along x1 of spec (grad kinds)
  const cplx<R>* s2;         // column derivative along x2 (3D grad kinds)
  cplx<R>* out0;             // output row spectra (first / only)
  cplx<R>* out1;             // second output spectrum (adjoint: w_2 or w_2 times ik_3)
  cplx<R>* out2;             // third output spectrum (3D adjoint: w_3 times ik_3)
  const R* vl;               // velocity coefficients [nc][d][n]
  const R* vtl;              // incremental velocity coefficients [nc][d][n]
  const R* g0;               // grad m^j   [d][n]
  const R* g1;               // grad m*_j  [d][n]
  R* g0w;                    // where FWD1 stores grad m^j (INC1: grad m~^j)
  R* g1w;                    // where FWD2 stores grad m*_j (INC2: grad m~*_j)
  R* lamw0;                  // ADJ1, if set: stores lam^{j+1} here ...
  R* lamw1;                  // ... and lam*_j here (the full-Newton matvec reads them)
  const R* lt0;              // full-Newton kinds: lam of the gradient's solve at the output time
  const R* lt1;              //   (NADJ1: lt0 = lam^{j+1}, lt1 = lam*_j; NADJINIT, NADJ2: lt0 only)
  const R* gt0;              // NADJ1: grad m~^j  [d][n]
  const R* gt1;              // NADJ1: grad m~*_j [d][n]
  R* acc;                    // Heun accumulator [n]
  R* lam;                    // adjoint state [n]
  R* F;                      // body force accumulators [nc][d][n]
  R* out_real;               // real output (new state of stage 2, gradient, divergence, C2R result)
  const R* mreal;            // stage 1: the transported field at t_j as a real array
  const R* src_a;
  const R* src_b;
  R ca, cb;                  // lam = ca * src_a + cb * src_b (src_b may be null)
  const float* src_bf;       // ST_R2C with a second source: src_b or, in FP32 (widened), src_bf
  int split;                 // ST_R2C: fields fy >= split come from the second source at fy - split and go to out1
  R h;                       // time step
  R scale;                   // C2R output scale (ST_C2R, ST_GRAD, ST_DIV multiply by scale/L)
  int nc;
  int zero_state;            // INC1 at j = 0: the incremental state is zero; ADJ1 at j = nt - 1: F starts at zero
  int inactive;              // batch groups: this item has no work in this launch (its time loop has ended)
  int skip_out;              // ADJ2 at j = 0: no further spectra needed
  long long n;               // points per scalar field
  long long fstride_in;      // batch stride (elements) of inputs (ST_R2C: reals, else complex)
  long long fstride_out;     // batch stride of outputs
  R b0[kMaxNc];              // b_l(t_j): velocity / force weights at the earlier node
  R b1[kMaxNc];              // b_l(t_{j+1})
  R bv[kMaxNc];              // weights of the velocity used for the outputs (ADJINIT/ADJ1/ADJ2)
};

template <int KIND0, int D>
struct StageShape {
  static constexpr int KIND = base_kind(KIND0);
  // KIN: input row spectra after C2R; KOUT: real rows transformed by R2C.
  // The transport stages need only the gradient of the transported field: the
  // field itself travels as a real array (stage 2 stores it, stage 1 reads it).
  static constexpr int KIN = (KIND == ST_FWD1 || KIND == ST_FWD2 || KIND == ST_INC1 || KIND == ST_INC2 ||
                              KIND == ST_GRAD)
                                 ? D
                                 : (KIND == ST_ADJ1 || KIND == ST_ADJ2 || KIND == ST_C2R || KIND == ST_DIV) ? 1 : 0;
  static constexpr int KOUT = (KIND == ST_FWD1 || KIND == ST_FWD2 || KIND == ST_INC1 || KIND == ST_INC2 ||
                               KIND == ST_R2C)
                                  ? 1
                                  : (KIND == ST_ADJINIT || KIND == ST_ADJ1 || KIND == ST_ADJ2) ? D : 0;
  static constexpr int KMAX = KIN > KOUT ? (KIN > 0 ? KIN : 1) : (KOUT > 0 ? KOUT : 1);
};

template <typename R>
__device__ __forceinline__ R vel_comb(const R* __restrict__ v, const R* w, int nc, int comp, int d,
                                      long long n, long long p) {
  if (nc == 1) return w[0] * v[(long long)comp * n + p];
  R s = R(0);
  for (int l = 0; l < nc; ++l) s += w[l] * v[((long long)l * d + comp) * n + p];
  return s;
}

// ---------------------------------------------------------------------------
// Spectral multiplier on vector fields in full-spectrum layout (after the
// forward transforms along every axis). Per coefficient l and mode k:
//   OP_HESS: out = scale * (beta a(k) X + [K] Y)
//   OP_PINV: out = scale * X / (beta a(k))  (k = 0: X)
//   OP_A   : out = scale * a(k) X
//   OP_K   : out = scale * K X
// The packed plane q = 0 holds Z = A + iB with A the k_last = 0 plane and B the
// k_last = N_last/2 plane; they are separated with the partner mode -k'.
// ---------------------------------------------------------------------------
enum SpecOp { OP_HESS = 0, OP_PINV = 1, OP_A = 2, OP_K = 3 };

template <typename R>
struct SpecArgs {
  const cplx<R>* X;   // [nc][d][nspec]
  const cplx<R>* Y;   // [nc][d][nspec] (OP_HESS)
  cplx<R>* out;       // [nc][d][nspec]
  int n1, n2, n3;     // grid (n3 = 1 for 2D); the last axis holds M = N_last/2 packed columns
  int d, nc, reg, proj;
  R beta, scale;
  long long nspec;    // complex per scalar field
};

template <typename R, int D>
__device__ __forceinline__ void spec_apply(const SpecArgs<R>& a, int op, const R kv[3], const R kt[3],
                                           const cplx<R>* x, const cplx<R>* y, cplx<R>* o) {
  R k2 = R(0), kt2 = R(0);
#pragma unroll
  for (int i = 0; i < D; ++i) { k2 += kv[i] * kv[i]; kt2 += kt[i] * kt[i]; }
  const R sym = (a.reg == 1) ? k2 : k2 * k2;
  cplx<R> kx = {R(0), R(0)};
  if ((op == OP_K || (op == OP_HESS && a.proj)) && kt2 > R(0)) {
    const cplx<R>* src = (op == OP_K) ? x : y;
#pragma unroll
    for (int i = 0; i < D; ++i) kx = cadd(kx, cscale(src[i], kt[i]));
    kx = cscale(kx, R(1) / kt2);
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {
    cplx<R> r;
    if (op == OP_HESS) {
      cplx<R> yy = y[i];
      if (a.proj) yy = csub(yy, cscale(kx, kt[i]));
      r = cadd(cscale(x[i], a.beta * sym), yy);
    } else if (op == OP_PINV) {
      r = (sym > R(0)) ? cscale(x[i], R(1) / (a.beta * sym)) : x[i];
    } else if (op == OP_A) {
      r = cscale(x[i], sym);
    } else {
      r = csub(x[i], cscale(kx, kt[i]));
    }
    o[i] = cscale(r, a.scale);
  }
}

// The multiplier's output at one mode of the full-spectrum layout. kv/kt hold the
// wavenumbers of the axes before the last; q is the packed column.
// spec_plain, q > 0: x and y are the inputs at the mode (y read only when has_y).
template <typename R, int D>
__device__ __forceinline__ void spec_plain(const SpecArgs<R>& a, int op, R kv[3], R kt[3], int q, bool has_y,
                                           const cplx<R>* x, const cplx<R>* y, cplx<R>* out) {
  kv[D - 1] = R(q); kt[D - 1] = R(q);
  cplx<R> yy[3];
#pragma unroll
  for (int i = 0; i < D; ++i) yy[i] = has_y ? y[i] : cplx<R>{R(0), R(0)};
  spec_apply<R, D>(a, op, kv, kt, x, yy, out);
}
// spec_packed, q = 0: x and y hold Z = A + iB at the mode and xp, yp the values at the
// partner mode -k' of the same packed plane; A and B are separated, the multiplier is
// applied on both planes (k_last = 0 and the Nyquist plane, whose even symbol keeps
// N_last/2 and whose derivative wavenumber is 0), and out = oA + i oB. Every mode is
// formed from its own and its partner's inputs, so the outputs keep the planes' Hermitian
// symmetry exactly (the multipliers are even).
template <typename R, int D>
__device__ __forceinline__ void spec_packed(const SpecArgs<R>& a, int op, R kv[3], R kt[3], bool has_y,
                                            const cplx<R>* x, const cplx<R>* y, const cplx<R>* xp,
                                            const cplx<R>* yp, cplx<R>* out) {
  cplx<R> zA[3], zB[3], yA[3], yB[3];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const cplx<R> z = x[i], zp = xp[i];
    zA[i] = {R(0.5) * (z.x + zp.x), R(0.5) * (z.y - zp.y)};    // (z + conj zp)/2
    zB[i] = {R(0.5) * (z.y + zp.y), -R(0.5) * (z.x - zp.x)};   // (z - conj zp)/(2i)
    if (has_y) {
      const cplx<R> w = y[i], wp = yp[i];
      yA[i] = {R(0.5) * (w.x + wp.x), R(0.5) * (w.y - wp.y)};
      yB[i] = {R(0.5) * (w.y + wp.y), -R(0.5) * (w.x - wp.x)};
    } else {
      yA[i] = yB[i] = {R(0), R(0)};
    }
  }
  const int nl = (D == 2) ? a.n2 : a.n3;
  cplx<R> oA[3], oB[3];
  kv[D - 1] = R(0); kt[D - 1] = R(0);
  spec_apply<R, D>(a, op, kv, kt, zA, yA, oA);
  kv[D - 1] = R(-(nl / 2));
  spec_apply<R, D>(a, op, kv, kt, zB, yB, oB);
#pragma unroll
  for (int i = 0; i < D; ++i) out[i] = {oA[i].x - oB[i].y, oA[i].y + oB[i].x};   // oA + i oB
}
template <typename R, int D>
__device__ __forceinline__ void spec_mode(const SpecArgs<R>& a, int op, R kv[3], R kt[3], int q, bool has_y,
                                          const cplx<R>* x, const cplx<R>* y, const cplx<R>* xp,
                                          const cplx<R>* yp, cplx<R>* out) {
  if (q > 0) spec_plain<R, D>(a, op, kv, kt, q, has_y, x, y, out);
  else spec_packed<R, D>(a, op, kv, kt, has_y, x, y, xp, yp, out);
}

template <typename R, int D>
__device__ __forceinline__ void spec_mul_body(const SpecArgs<R>& a, int op) {
  const int nl = (D == 2) ? a.n2 : a.n3;   // last axis length
  const int M = nl / 2;
  const long long rows = (long long)a.n1 * (D == 3 ? a.n2 : 1);
  const long long tot = rows * M * a.nc;
  const bool has_y = a.Y != nullptr;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot;
       t += (long long)gridDim.x * blockDim.x) {
    const int l = (int)(t / (rows * M));
    const long long mi = t - (long long)l * rows * M;
    const long long row = mi / M;
    const int q = (int)(mi - row * M);
    int i1, i2 = 0;
    if (D == 2) { i1 = (int)row; } else { i1 = (int)(row / a.n2); i2 = (int)(row - (long long)i1 * a.n2); }
    R kv[3], kt[3];
    kv[0] = R(wavenumber(i1, a.n1)); kt[0] = R(deriv_wavenumber(i1, a.n1));
    if (D == 3) { kv[1] = R(wavenumber(i2, a.n2)); kt[1] = R(deriv_wavenumber(i2, a.n2)); }
    const long long base = (long long)l * D * a.nspec;
    cplx<R> x[3], y[3], o[3];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      x[i] = a.X[base + i * a.nspec + mi];
      if (has_y) y[i] = a.Y[base + i * a.nspec + mi];
    }
    if (q > 0) {
      spec_mode<R, D>(a, op, kv, kt, q, has_y, x, y, x, y, o);
#pragma unroll
      for (int i = 0; i < D; ++i) a.out[base + i * a.nspec + mi] = o[i];
      continue;
    }
    // packed plane: the pair (k', -k') is read and written by one thread (the smaller
    // row index), since the output may overwrite the input
    const int j1 = (a.n1 - i1) % a.n1;
    const int j2 = (D == 3) ? (a.n2 - i2) % a.n2 : 0;
    const long long prow = (D == 2) ? j1 : (long long)j1 * a.n2 + j2;
    if (prow < row) continue;
    const long long mp = prow * M;
    cplx<R> xp[3], yp[3], op_[3];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      xp[i] = a.X[base + i * a.nspec + mp];
      if (has_y) yp[i] = a.Y[base + i * a.nspec + mp];
    }
    R kvp[3], ktp[3];
    kvp[0] = R(wavenumber(j1, a.n1)); ktp[0] = R(deriv_wavenumber(j1, a.n1));
    if (D == 3) { kvp[1] = R(wavenumber(j2, a.n2)); ktp[1] = R(deriv_wavenumber(j2, a.n2)); }
    spec_mode<R, D>(a, op, kv, kt, 0, has_y, x, y, xp, yp, o);
    spec_mode<R, D>(a, op, kvp, ktp, 0, has_y, xp, yp, x, y, op_);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      a.out[base + i * a.nspec + mi] = o[i];
      if (prow != row) a.out[base + i * a.nspec + mp] = op_[i];
    }
  }
}

template <typename R, int D>
__global__ __launch_bounds__(256) void k_spec_mul(SpecArgs<R> a, int op) {
  spec_mul_body<R, D>(a, op);
}
// One launch over the items of a batch group: item blockIdx.z uses tab[blockIdx.z].
template <typename R, int D>
__global__ __launch_bounds__(256) void k_spec_mul_t(const SpecArgs<R>* __restrict__ tab, int op) {
  spec_mul_body<R, D>(tab[blockIdx.z], op);
}

// ---------------------------------------------------------------------------
// FP64 reductions (deterministic: fixed grid, fixed tree) and vector updates.
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 512;
constexpr int kRedThreads = 256;

__device__ __forceinline__ double warp_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}
__device__ __forceinline__ double warp_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  return v;
}

template <bool MAX>
__device__ __forceinline__ void block_reduce_store(double v, double* out) {
  __shared__ double part[kRedThreads / 64];
  v = MAX ? warp_max(v) : warp_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) part[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = part[0];
    for (int i = 1; i < kRedThreads / 64; ++i) s = MAX ? fmax(s, part[i]) : s + part[i];
    *out = s;
  }
}

enum RedOp { RED_DOT = 0, RED_SUMSQ = 1, RED_MAXABS = 2, RED_SUM = 3, RED_SUMSQDIFF = 4 };

// partial[blockIdx.x] = reduction over a grid-stride slice. A NaN anywhere
// propagates into the sum (and is caught on the host); RED_MAXABS also turns a
// NaN into +inf so that it is detected.
template <typename R, int OP>
__device__ __forceinline__ void reduce_body(const R* __restrict__ x, const R* __restrict__ y, long long cnt,
                                            double* partial) {
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * kRedThreads) {
    const double a = (double)x[i];
    if (OP == RED_DOT) acc += a * (double)y[i];
    else if (OP == RED_SUMSQ) acc += a * a;
    else if (OP == RED_SUM) acc += a;
    else if (OP == RED_SUMSQDIFF) { const double d = a - (double)y[i]; acc += d * d; }
    else { const double m = fabs(a); acc = (m != m) ? INFINITY : fmax(acc, m); }
  }
  block_reduce_store<OP == RED_MAXABS>(acc, partial + blockIdx.x);
}
template <typename R, int OP>
__global__ __launch_bounds__(kRedThreads) void k_reduce(const R* __restrict__ x, const R* __restrict__ y,
                                                        long long cnt, double* partial) {
  reduce_body<R, OP>(x, y, cnt, partial);
}

template <bool MAX>
__device__ __forceinline__ void reduce_final_body(const double* __restrict__ partial, int np, double* out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += kRedThreads) acc = MAX ? fmax(acc, partial[i]) : acc + partial[i];
  block_reduce_store<MAX>(acc, out);
}
template <bool MAX>
__global__ __launch_bounds__(kRedThreads) void k_reduce_final(const double* __restrict__ partial, int np,
                                                              double* out) {
  reduce_final_body<MAX>(partial, np, out);
}

// |x|^2 and <x, y> in one pass over x and y: each block's two partial sums are formed in
// the order of the single reductions (RED_SUMSQ, RED_DOT), so each result equals its own
// reduction bit for bit. partial holds [2][gridDim.x].
template <typename R>
__global__ __launch_bounds__(kRedThreads) void k_reduce_sumsq_dot(const R* __restrict__ x, const R* __restrict__ y,
                                                                  long long cnt, double* partial) {
  double s2 = 0.0, sd = 0.0;
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * kRedThreads) {
    const double a = (double)x[i];
    s2 += a * a;
    sd += a * (double)y[i];
  }
  block_reduce_store<false>(s2, partial + blockIdx.x);
  __syncthreads();
  block_reduce_store<false>(sd, partial + gridDim.x + blockIdx.x);
}
// Final stage of np partial sums per reduction for gridDim.x reductions side by side.
static __global__ __launch_bounds__(kRedThreads) void k_reduce_final_n(const double* __restrict__ partial,
                                                                       int np, double* out) {
  reduce_final_body<false>(partial + (long long)blockIdx.x * np, np, out + blockIdx.x);
}

// Batch-group forms of the two reduction stages: each item takes its pointers
// from the table (blockIdx.z); the per-item grid and summation order are those of the
// plain forms.
template <typename R>
struct RedPtrs {
  const R* x;
  const R* y;
  double* partial;
};
struct RedFinalPtrs {
  const double* partial;
  double* out;
};
template <typename R, int OP>
__global__ __launch_bounds__(kRedThreads) void k_reduce_t(long long cnt, const RedPtrs<R>* __restrict__ tab) {
  const RedPtrs<R> p = tab[blockIdx.z];
  reduce_body<R, OP>(p.x, p.y, cnt, p.partial);
}
template <bool MAX>
__global__ __launch_bounds__(kRedThreads) void k_reduce_final_t(int np, const RedFinalPtrs* __restrict__ tab) {
  const RedFinalPtrs p = tab[blockIdx.z];
  reduce_final_body<MAX>(p.partial, np, p.out);
}

// min / max / sum / sum of squares about a shift, of an FP64 field (det F statistics)
static __global__ __launch_bounds__(kRedThreads) void k_stats(const double* __restrict__ x, long long cnt, double shift,
                                                       double* partial /* [4][blocks] */) {
  double mn = INFINITY, mx = -INFINITY, s = 0.0, s2 = 0.0;
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * kRedThreads) {
    const double v = x[i];
    mn = fmin(mn, v); mx = fmax(mx, v);
    s += v;
    s2 += (v - shift) * (v - shift);
  }
  const int nb = gridDim.x;
  // min via max of negatives
  block_reduce_store<true>(-mn, partial + blockIdx.x);
  __syncthreads();
  block_reduce_store<true>(mx, partial + nb + blockIdx.x);
  __syncthreads();
  block_reduce_store<false>(s, partial + 2 * nb + blockIdx.x);
  __syncthreads();
  block_reduce_store<false>(s2, partial + 3 * nb + blockIdx.x);
}

// y = a*x + b*y   (a, b host scalars)
template <typename R>
__global__ void k_axpby(long long cnt, R a, const R* __restrict__ x, R b, R* __restrict__ y) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

// One PCG update with the step length taken on the device: alpha = rz / pq from
// the reduction slots, then x += alpha p and r -= alpha q, written as the two
// axpby launches would (a x + b y with b = 1). Curvature pq <= 0 (or NaN) leaves
// x and r unchanged; the host sees pq at its next read and stops there.
static __global__ void k_pcg_step(long long cnt, const double* __restrict__ rz, const double* __restrict__ pq,
                           const double* __restrict__ p, const double* __restrict__ q, double* __restrict__ x,
                           double* __restrict__ r) {
  const double c = *pq;
  if (!(c > 0.0)) return;
  const double a = *rz / c;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x) {
    x[i] = a * p[i] + 1.0 * x[i];
    r[i] = -a * q[i] + 1.0 * r[i];
  }
}

// z = a*x + b*y
template <typename R>
__global__ void k_lincomb(long long cnt, R a, const R* __restrict__ x, R b, const R* __restrict__ y,
                          R* __restrict__ z) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x)
    z[i] = a * x[i] + b * y[i];
}

// y = x + c (c a host scalar); x and y may alias
template <typename R>
__global__ void k_shift(long long cnt, R c, const R* x, R* y) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = x[i] + c;
}

template <typename R>
__global__ void k_fill(long long cnt, R v, R* __restrict__ y) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = v;
}

template <typename RS, typename RD>
__global__ void k_convert(long long cnt, const RS* __restrict__ x, RD* __restrict__ y) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = (RD)x[i];
}

// Batch-group forms: item blockIdx.z takes its pointers from the table.
template <typename R>
__global__ void k_fill_t(long long cnt, R v, R* const* __restrict__ tab) {
  R* __restrict__ y = tab[blockIdx.z];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = v;
}
template <typename RS, typename RD>
struct ConvPtrs {
  const RS* x;
  RD* y;
};
template <typename RS, typename RD>
__global__ void k_convert_t(long long cnt, const ConvPtrs<RS, RD>* __restrict__ tab) {
  const RS* __restrict__ x = tab[blockIdx.z].x;
  RD* __restrict__ y = tab[blockIdx.z].y;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = (RD)x[i];
}

// ---------------------------------------------------------------------------
// Deformation gradient (FP64): Heun on dt F = -(v . grad) F + (grad v) F.
// F, gradF: [d][d][n] and [d][d][d][n] (gradF[i][j][k] = D_k F_ij); gv: [d][d][n]
// (gv[i][k] = D_k v^i); v: [d][n].
// mode 0: Fs = F + h rhs(F), acc = F + h/2 rhs(F);  mode 1: F = acc + h/2 rhs(Fs)
// ---------------------------------------------------------------------------
template <int D>
__global__ void k_defgrad_stage(long long n, double h, const double* __restrict__ v,
                                const double* __restrict__ gv, const double* __restrict__ Fin,
                                const double* __restrict__ gradF, double* __restrict__ acc,
                                double* __restrict__ Fout, int mode) {
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    double vv[D], G[D][D], Fm[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      vv[i] = v[i * n + p];
#pragma unroll
      for (int k = 0; k < D; ++k) { G[i][k] = gv[(i * D + k) * n + p]; Fm[i][k] = Fin[(i * D + k) * n + p]; }
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
#pragma unroll
      for (int j = 0; j < D; ++j) {
        double r = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) r += -vv[k] * gradF[((i * D + j) * D + k) * n + p] + G[i][k] * Fm[k][j];
        const long long o = (i * D + j) * n + p;
        if (mode == 0) {
          acc[o] = Fm[i][j] + 0.5 * h * r;
          Fout[o] = Fm[i][j] + h * r;
        } else {
          Fout[o] = acc[o] + 0.5 * h * r;
        }
      }
    }
  }
}

template <int D>
__global__ void k_det(long long n, const double* __restrict__ F, double* __restrict__ out) {
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    if (D == 2) {
      out[p] = F[0 * n + p] * F[3 * n + p] - F[1 * n + p] * F[2 * n + p];
    } else {
      const double a = F[0 * n + p], b = F[1 * n + p], c = F[2 * n + p];
      const double d = F[3 * n + p], e = F[4 * n + p], f = F[5 * n + p];
      const double g = F[6 * n + p], hh = F[7 * n + p], i = F[8 * n + p];
      out[p] = a * (e * i - f * hh) - b * (d * i - f * g) + c * (d * hh - e * g);
    }
  }
}

template <int D>
__global__ void k_identity_tensor(long long n, double* __restrict__ F) {
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) F[(i * D + j) * n + p] = (i == j) ? 1.0 : 0.0;
  }
}

// v(t) = sum_l b_l v_l converted to FP64 (det F works in FP64)
struct Weights {
  double w[kMaxNc];
};

template <typename R>
__global__ void k_vel_at(long long cnt /* d*n */, int nc, const R* __restrict__ vl, Weights b,
                         double* __restrict__ out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int l = 0; l < nc; ++l) s += b.w[l] * (double)vl[(long long)l * cnt + i];
    out[i] = s;
  }
}

}  // namespace nk
