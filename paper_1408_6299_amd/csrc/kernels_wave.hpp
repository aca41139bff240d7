// Row-stage and column-pass kernels built on register-resident wave FFTs.
//
// Row stage: one wavefront per workgroup; each row of the contiguous last
// axis (length L, M = L/2 complex) is held by LS = M/E lanes. Global loads of
// every operand the pointwise epilogue needs are issued at kernel start, so
// their latency overlaps the inverse transforms. The real <-> half-complex
// packing is done in registers on (q, M - q) pairs; transforms exchange data
// only inside the wavefront.
//
// Column pass: one wavefront per workgroup handling 64 / LS columns (lanes of
// neighbouring columns are adjacent, so loads of small transforms coalesce);
// workgroups are ordered so that neighbouring columns share an XCD and its L2.
#pragma once

#include "kernels.hpp"
#include "wave_fft.hpp"

namespace nk {

// pointwise product of two real pairs stored as cplx
template <typename R>
__device__ __forceinline__ cplx<R> pmul(cplx<R> a, cplx<R> b) { return {a.x * b.x, a.y * b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> pfma(cplx<R> a, cplx<R> b, cplx<R> c) { return {a.x * b.x + c.x, a.y * b.y + c.y}; }

// C2R packing step on a pair (q, M - q): packed half spectrum -> Z of the
// half-length complex transform (scaled so the unnormalised inverse gives L x).
template <typename R>
__device__ __forceinline__ void c2r_pair(cplx<R> xq, cplx<R> xm, cplx<R> w, cplx<R>& zq, cplx<R>& zm) {
  const cplx<R> e = {xq.x + xm.x, xq.y - xm.y};
  const cplx<R> dq = {xq.x - xm.x, xq.y + xm.y};
  const cplx<R> o = cmulc(dq, w);
  zq = {e.x - o.y, e.y + o.x};
  zm = {e.x + o.y, o.x - e.y};
}

// R2C unpacking step on a pair: Z of the half-length transform -> packed half spectrum.
template <typename R>
__device__ __forceinline__ void r2c_pair(cplx<R> zq, cplx<R> zm, cplx<R> w, cplx<R>& xq, cplx<R>& xm) {
  const cplx<R> e = {R(0.5) * (zq.x + zm.x), R(0.5) * (zq.y - zm.y)};
  const cplx<R> o = {R(0.5) * (zq.y + zm.y), -R(0.5) * (zq.x - zm.x)};
  const cplx<R> wo = cmul(o, w);
  xq = cadd(e, wo);
  xm = cconj(csub(e, wo));
}

// velocity-like combination sum_l w_l f[(l*D + c) n + p] as a real pair
template <typename R, int D, bool NC1>
__device__ __forceinline__ cplx<R> comb2(const R* __restrict__ f, const R* w, int nc, int c, long long n,
                                         long long pc) {
  const cplx<R>* F = reinterpret_cast<const cplx<R>*>(f);
  const long long n2 = n / 2;
  if (NC1) return cscale(F[(long long)c * n2 + pc], w[0]);
  cplx<R> s = {R(0), R(0)};
  for (int l = 0; l < nc; ++l) s = cadd(s, cscale(F[((long long)l * D + c) * n2 + pc], w[l]));
  return s;
}

// LDS scratch of one wavefront's row stage: SPW rows of KMAX padded sequences.
template <typename R, int L, int E, int KIND0, int D>
struct RowLds {
  static constexpr int M = L / 2;
  static constexpr int SPW = 64 / WavePlan<M, E>::LS;   // rows per wavefront
  static constexpr int PADM = padded_e<E>(M);
  static constexpr int SIZE = SPW * StageShape<KIND0, D>::KMAX * PADM;   // complex elements
};

// One wavefront's share of a row stage: row group rgroup (rows rgroup * SPW ..), field
// fy of a batched launch, scratch lds (RowLds::SIZE elements), lane 0..63.
template <typename R, int L, int E, int KIND0, int D, bool NC1>
__device__ __forceinline__ void row_body_at(const StageArgs<R>& a, const cplx<R>* __restrict__ tw, int lmax,
                                            long long rgroup, int fy, cplx<R>* lds, int lane) {
  constexpr int KIND = base_kind(KIND0);    // full-Newton kinds run their adjoint kind's code ...
  constexpr bool NEWT = newton_kind(KIND0);  // ... plus the lambda terms
  constexpr int M = L / 2;
  using P = WavePlan<M, E>;
  constexpr int LS = P::LS;
  constexpr int SPW = 64 / LS;
  constexpr int PADM = padded_e<E>(M);
  constexpr int H = E / 2;
  using SH = StageShape<KIND0, D>;
  constexpr int KIN = SH::KIN, KOUT = SH::KOUT, KMAX = SH::KMAX;
  constexpr bool FWDK = (KIND == ST_FWD1 || KIND == ST_FWD2);
  constexpr bool INCK = (KIND == ST_INC1 || KIND == ST_INC2);
  constexpr bool ADJOUT = (KIND == ST_ADJINIT || KIND == ST_ADJ1 || KIND == ST_ADJ2);

  const int sr = lane / LS, j = lane - sr * LS;
  const long long rows = a.n / L;
  const long long rowr = rgroup * SPW + sr;
  const bool live = rowr < rows;
  const long long row = live ? rowr : rows - 1;
  const long long n = a.n;
  const long long c0 = row * M;  // first complex slot (point pair) of the row
  cplx<R>* S = lds + sr * KMAX * PADM;
  const int twl = lmax / L;
  const R invL = R(1) / R(L);
  const R h = a.h;
  const R hh = R(0.5) * a.h;

  WaveTwiddles<R, M, E> T;
  T.load(j, tw, lmax / M);
  cplx<R> wq[H];
  int qa[H], qb[H];
#pragma unroll
  for (int t = 0; t < H; ++t) {
    const bool sp = (j == 0 && t == 0);
    qa[t] = sp ? 0 : j + LS * t;
    qb[t] = sp ? M / 2 : M - (j + LS * t);
    wq[t] = tw[(sp ? M / 2 : qa[t]) * twl];
  }
  auto pidx = [&](int e) -> long long { return c0 + j + LS * e; };
  auto ld2 = [&](const R* f, int e) -> cplx<R> { return reinterpret_cast<const cplx<R>*>(f)[pidx(e)]; };
  auto st2 = [&](R* f, int e, cplx<R> v) {
    if (live) reinterpret_cast<cplx<R>*>(f)[pidx(e)] = v;
  };

  // ---- input row spectra (pair layout), loaded first: the C2R packing and the
  // inverse transforms can start as soon as they arrive, while the epilogue's
  // operands below are still in flight. All of them are loaded before any LDS
  // store, so no load waits behind the packing of an earlier input. ----
  constexpr int KA = KIN > 0 ? KIN : 1;
  const int zero_in = (KIND == ST_INC1) ? a.zero_state : 0;
  cplx<R> XA[KA][H], XB[KA][H];
  if constexpr (KIN > 0) {
    if (!zero_in) {
      const long long fin = (long long)fy * a.fstride_in;
#pragma unroll
      for (int k = 0; k < KIN; ++k) {
        const cplx<R>* src;
        if constexpr (KIND == ST_GRAD || FWDK || INCK) {
          // gradient components: column derivatives, then i k_last times the row spectrum
          if (k == D - 1) src = a.spec;
          else src = (k == 0) ? a.s1 : a.s2;
        } else {
          src = a.spec;
        }
        src += fin + c0;
#pragma unroll
        for (int t = 0; t < H; ++t) { XA[k][t] = src[qa[t]]; XB[k][t] = src[qb[t]]; }
      }
    }
  }

  // ---- prefetch the epilogue's operands (natural layout, point pairs) ----
  constexpr int DV = (FWDK || INCK || ADJOUT) ? D : 1;
  constexpr int DW = (INCK || NEWT) ? D : 1;
  constexpr int DG = (INCK || KIND == ST_ADJ1) ? D : 1;
  constexpr int DF = (KIND == ST_ADJ1 && NC1) ? D : 1;
  constexpr int DT = (NEWT && KIND == ST_ADJ1) ? D : 1;
  cplx<R> V[DV][E], W[DW][E], G0[DG][E], G1[DG][E], FV[DF][E], X1[E], X2[E];
  cplx<R> LT0[E], LT1[E], GT0[DT][E], GT1[DT][E];
  const R* wv = (KIND == ST_FWD1 || KIND == ST_INC1) ? a.b0 : ((KIND == ST_FWD2 || KIND == ST_INC2) ? a.b1 : a.bv);
  // ST_R2C: this field comes from the second source (and goes to out1)
  const bool r2c_second = KIND == ST_R2C && (a.src_b || a.src_bf) && fy >= a.split;
  const bool need_v = !(KIND == ST_ADJ2 && a.skip_out);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if constexpr (FWDK || INCK || ADJOUT) {
      // loaded even where the last adjoint stage skips its output (the velocity is
      // always valid), so no wait sits inside a branch
#pragma unroll
      for (int c = 0; c < D; ++c) V[c][e] = comb2<R, D, NC1>(a.vl, wv, a.nc, c, n, pidx(e));
    }
    if constexpr (INCK) {
#pragma unroll
      for (int c = 0; c < D; ++c) {
        W[c][e] = comb2<R, D, NC1>(a.vtl, wv, a.nc, c, n, pidx(e));
        G0[c][e] = ld2((KIND == ST_INC1 ? a.g0 : a.g1) + (long long)c * n, e);
      }
    }
    if constexpr (KIND == ST_ADJ1) {
#pragma unroll
      for (int c = 0; c < D; ++c) {
        G0[c][e] = ld2(a.g0 + (long long)c * n, e);
        G1[c][e] = ld2(a.g1 + (long long)c * n, e);
        if constexpr (NC1) FV[c][e] = ld2(a.F + (long long)c * n, e);
      }
      X1[e] = ld2(a.lam, e);
    }
    if constexpr (NEWT) {
      if (need_v) {
#pragma unroll
        for (int c = 0; c < D; ++c) W[c][e] = comb2<R, D, NC1>(a.vtl, wv, a.nc, c, n, pidx(e));
        LT0[e] = ld2(a.lt0, e);
      }
      if constexpr (KIND == ST_ADJ1) {
        LT1[e] = ld2(a.lt1, e);
#pragma unroll
        for (int c = 0; c < D; ++c) {
          GT0[c][e] = ld2(a.gt0 + (long long)c * n, e);
          GT1[c][e] = ld2(a.gt1 + (long long)c * n, e);
        }
      }
    }
    if constexpr (KIND == ST_FWD2 || KIND == ST_INC2 || KIND == ST_ADJ2) X1[e] = ld2(a.acc, e);
    if constexpr (KIND == ST_FWD1) X2[e] = ld2(a.mreal, e);
    if constexpr (KIND == ST_INC1) {
      // loaded on the first step too (the buffer is always valid), so no wait sits
      // inside a branch; the zero initial state discards the value
      const cplx<R> m = ld2(a.mreal, e);
      X2[e] = a.zero_state ? cplx<R>{R(0), R(0)} : m;
    }
    if constexpr (KIND == ST_ADJINIT) {
      X1[e] = ld2(a.src_a, e);
      X2[e] = a.src_b ? ld2(a.src_b, e) : cplx<R>{R(0), R(0)};
    }
    if constexpr (KIND == ST_R2C) {
      if (!r2c_second) {
        X1[e] = ld2(a.src_a + (long long)fy * a.fstride_in, e);
      } else if (a.src_bf) {
        const float2 f = reinterpret_cast<const float2*>(a.src_bf + (long long)(fy - a.split) * a.fstride_in)[pidx(e)];
        X1[e] = {R(f.x), R(f.y)};
      } else {
        X1[e] = ld2(a.src_b + (long long)(fy - a.split) * a.fstride_in, e);
      }
    }
  }

  // ---- input row spectra: C2R packing -> natural layout -> inverse FFT ----
  cplx<R> A[KA][E];
  if constexpr (KIN > 0) {
    if (!zero_in) {
#pragma unroll
      for (int k = 0; k < KIN; ++k) {
        const bool ik = (KIND == ST_GRAD || FWDK || INCK) && k == D - 1;
        cplx<R>* xa = XA[k];
        cplx<R>* xb = XB[k];
#pragma unroll
        for (int t = 0; t < H; ++t) {
          if (ik) {
            xa[t] = (qa[t] == 0) ? cplx<R>{R(0), R(0)} : cmul_i(xa[t], R(qa[t]));
            xb[t] = cmul_i(xb[t], R(qb[t]));
          }
          cplx<R> za, zb;
          if (j == 0 && t == 0) {
            za = {xa[t].x + xa[t].y, xa[t].x - xa[t].y};
            cplx<R> unused;
            c2r_pair(xb[t], xb[t], wq[t], zb, unused);
          } else {
            c2r_pair(xa[t], xb[t], wq[t], za, zb);
          }
          S[k * PADM + pad_e<E>(qa[t])] = za;
          S[k * PADM + pad_e<E>(qb[t])] = zb;
        }
      }
      wave_lds_sync();
#pragma unroll
      for (int k = 0; k < KIN; ++k)
#pragma unroll
        for (int e = 0; e < E; ++e) A[k][e] = S[k * PADM + pad_e<E>(j + LS * e)];
      wave_lds_sync();
      wave_fft_multi<R, M, E, true, KIN>(A, j, S, PADM, T);
    }
  }

  // ---- pointwise epilogue (natural layout) ----
  constexpr int KO = KOUT > 0 ? KOUT : 1;
  cplx<R> O[KO][E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if constexpr (FWDK) {
      cplx<R> r = {R(0), R(0)};
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const cplx<R> gc = cscale(A[c][e], invL);
        if (KIND == ST_FWD1) { if (a.g0w) st2(a.g0w + (long long)c * n, e, gc); }
        else { if (a.g1w) st2(a.g1w + (long long)c * n, e, gc); }
        r = csub(r, pmul(V[c][e], gc));
      }
      if (KIND == ST_FWD1) {
        const cplx<R> m = X2[e];
        st2(a.acc, e, cadd(m, cscale(r, hh)));
        O[0][e] = cadd(m, cscale(r, h));
      } else {
        const cplx<R> mn = cadd(X1[e], cscale(r, hh));
        st2(a.out_real, e, mn);
        O[0][e] = mn;
      }
    } else if constexpr (INCK) {
      cplx<R> r = {R(0), R(0)};
      R* gw = (KIND == ST_INC1) ? a.g0w : a.g1w;   // grad m~ of this stage, for the full-Newton matvec
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const cplx<R> gc = zero_in ? cplx<R>{R(0), R(0)} : cscale(A[c][e], invL);
        if (gw) st2(gw + (long long)c * n, e, gc);
        r = csub(r, pmul(V[c][e], gc));
      }
#pragma unroll
      for (int c = 0; c < D; ++c) r = csub(r, pmul(W[c][e], G0[c][e]));
      if (KIND == ST_INC1) {
        const cplx<R> m = X2[e];
        st2(a.acc, e, cadd(m, cscale(r, hh)));
        O[0][e] = cadd(m, cscale(r, h));
      } else {
        const cplx<R> mn = cadd(X1[e], cscale(r, hh));
        st2(a.out_real, e, mn);
        O[0][e] = mn;
      }
    } else if constexpr (KIND == ST_ADJINIT) {
      const cplx<R> lam = cadd(cscale(X1[e], a.ca), cscale(X2[e], a.cb));
      st2(a.lam, e, lam);
#pragma unroll
      for (int c = 0; c < D; ++c) {
        O[c][e] = pmul(V[c][e], lam);
        if constexpr (NEWT) O[c][e] = pfma(W[c][e], LT0[e], O[c][e]);
      }
    } else if constexpr (KIND == ST_ADJ1) {
      const cplx<R> s1 = cscale(A[0][e], invL);
      const cplx<R> lam = X1[e];
      const cplx<R> lams = cadd(lam, cscale(s1, h));
      st2(a.acc, e, cadd(lam, cscale(s1, hh)));
      if constexpr (!NEWT) {
        if (a.lamw0) {
          st2(a.lamw0, e, lam);
          st2(a.lamw1, e, lams);
        }
      }
#pragma unroll
      for (int c = 0; c < D; ++c) {
        cplx<R> t0 = pmul(lams, G0[c][e]);
        cplx<R> t1 = pmul(lam, G1[c][e]);
        if constexpr (NEWT) {
          t0 = pfma(LT1[e], GT0[c][e], t0);   // lam*_j grad m~^j
          t1 = pfma(LT0[e], GT1[c][e], t1);   // lam^{j+1} grad m~*_j
        }
        // the first adjoint step starts the accumulators at zero (their contents are ignored)
        if constexpr (NC1) {
          const cplx<R> f0 = a.zero_state ? cplx<R>{R(0), R(0)} : FV[c][e];
          const cplx<R> f = cadd(f0, cscale(cadd(cscale(t0, a.b0[0]), cscale(t1, a.b1[0])), hh));
          st2(a.F + (long long)c * n, e, f);
        } else {
          for (int l = 0; l < a.nc; ++l) {
            R* fp = a.F + ((long long)l * D + c) * n;
            const cplx<R> f0 = a.zero_state ? cplx<R>{R(0), R(0)} : ld2(fp, e);
            st2(fp, e, cadd(f0, cscale(cadd(cscale(t0, a.b0[l]), cscale(t1, a.b1[l])), hh)));
          }
        }
        O[c][e] = pmul(V[c][e], lams);
        if constexpr (NEWT) O[c][e] = pfma(W[c][e], LT1[e], O[c][e]);   // + v~(t_j) lam*_j
      }
    } else if constexpr (KIND == ST_ADJ2) {
      const cplx<R> s2 = cscale(A[0][e], invL);
      const cplx<R> lam = cadd(X1[e], cscale(s2, hh));
      st2(a.lam, e, lam);
      if (!a.skip_out) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
          O[c][e] = pmul(V[c][e], lam);
          if constexpr (NEWT) O[c][e] = pfma(W[c][e], LT0[e], O[c][e]);   // + v~(t_j) lam^j
        }
      }
    } else if constexpr (KIND == ST_R2C) {
      O[0][e] = X1[e];
    } else if constexpr (KIND == ST_C2R || KIND == ST_DIV) {
      st2(a.out_real + (long long)fy * a.fstride_out, e, cscale(A[0][e], invL * a.scale));
    } else if constexpr (KIND == ST_GRAD) {
#pragma unroll
      for (int c = 0; c < D; ++c)
        st2(a.out_real + (long long)fy * a.fstride_out + (long long)c * n, e,
            cscale(A[c][e], invL * a.scale));
    }
  }

  // ---- forward FFT of the new rows -> R2C unpacking -> store in pair layout ----
  if constexpr (KOUT > 0) {
    if (KIND == ST_ADJ2 && a.skip_out) return;  // uniform across the workgroup
    wave_fft_multi<R, M, E, false, KOUT>(O, j, S, PADM, T);
#pragma unroll
    for (int k = 0; k < KOUT; ++k)
#pragma unroll
      for (int e = 0; e < E; ++e) S[k * PADM + pad_e<E>(j + LS * e)] = O[k][e];
    wave_lds_sync();
    const long long fo = (long long)(r2c_second ? fy - a.split : fy) * a.fstride_out;
#pragma unroll
    for (int k = 0; k < KOUT; ++k) {
      cplx<R>* dst;
      if constexpr (ADJOUT) dst = (k == 0) ? a.out0 : (k == 1 ? a.out1 : a.out2);
      else dst = r2c_second ? a.out1 : a.out0;
      dst += fo + c0;
      const bool ik = ADJOUT && D > 1 && k == D - 1;
#pragma unroll
      for (int t = 0; t < H; ++t) {
        const cplx<R> za = S[k * PADM + pad_e<E>(qa[t])];
        const cplx<R> zb = S[k * PADM + pad_e<E>(qb[t])];
        cplx<R> xa, xb;
        if (j == 0 && t == 0) {
          xa = {za.x + za.y, za.x - za.y};
          cplx<R> unused;
          r2c_pair(zb, zb, wq[t], xb, unused);
        } else {
          r2c_pair(za, zb, wq[t], xa, xb);
        }
        if (ik) {
          xa = (qa[t] == 0) ? cplx<R>{R(0), R(0)} : cmul_i(xa, R(qa[t]));
          xb = cmul_i(xb, R(qb[t]));
        }
        if (live) {
          dst[qa[t]] = xa;
          dst[qb[t]] = xb;
        }
      }
    }
  }
}

// A row stage with one wavefront per workgroup: row group blockIdx.x, field blockIdx.y.
template <typename R, int L, int E, int KIND0, int D, bool NC1>
__device__ __forceinline__ void row_body(const StageArgs<R>& a, const cplx<R>* __restrict__ tw, int lmax) {
  __shared__ cplx<R> lds[RowLds<R, L, E, KIND0, D>::SIZE];
  row_body_at<R, L, E, KIND0, D, NC1>(a, tw, lmax, (long long)blockIdx.x, (int)blockIdx.y, lds, (int)threadIdx.x);
}

template <typename R, int L, int E, int KIND, int D, bool NC1>
__global__ __launch_bounds__(64) void k_row_w(StageArgs<R> a, const cplx<R>* __restrict__ tw, int lmax) {
  row_body<R, L, E, KIND, D, NC1>(a, tw, lmax);
}
// One launch over the items of a batch group: item blockIdx.z uses tab[blockIdx.z].
template <typename R, int L, int E, int KIND, int D, bool NC1>
__global__ __launch_bounds__(64) void k_row_wt(const StageArgs<R>* __restrict__ tab, const cplx<R>* __restrict__ tw,
                                               int lmax) {
  if (tab[blockIdx.z].inactive) return;
  row_body<R, L, E, KIND, D, NC1>(tab[blockIdx.z], tw, lmax);
}

// Pointers of one column pass (per batch item in the group forms).
template <typename R>
struct ColPtrs {
  const cplx<R>* in;
  const cplx<R>* add;
  cplx<R>* out;
  int inactive;   // batch groups: this item has no work in this launch
};

template <int N, int E>
struct ColShape {
  static constexpr int LS = WavePlan<N, E>::LS;       // lanes per column
  static constexpr int SPW = LS >= 64 ? 1 : 64 / LS;  // columns per workgroup
  static constexpr int NT = LS >= 64 ? LS : 64;       // threads per workgroup
  static constexpr bool BLOCK = LS > 64;              // a column spans several waves
};

// One workgroup's column group of a column pass: columns bx * SPW .., outer slice by,
// field fz; scratch lds (SPW padded columns), lane 0..NT-1.
template <typename R, int N, int E, int MODE>
__device__ __forceinline__ void col_w_at(const cplx<R>* in, const cplx<R>* add, cplx<R>* out, const ColArgs& a,
                                         R scale, const cplx<R>* __restrict__ tw, int twb, int fz, int bx, int by,
                                         cplx<R>* lds, int lane) {
  using CS = ColShape<N, E>;
  constexpr int LS = CS::LS;
  constexpr int SPW = CS::SPW;
  constexpr bool BLK = CS::BLOCK;
  constexpr int PADN = padded_e<E>(N);
  const int c = lane % SPW, j = lane / SPW;
  const long long colr = (long long)bx * SPW + c;
  const bool live = colr < a.inner;
  const long long col = live ? colr : a.inner - 1;
  const long long base = (long long)fz * a.field + (long long)by * N * a.inner + col;
  cplx<R> v[E], ad[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = in[base + (long long)(j + LS * e) * a.inner];
  const bool has_add = (MODE == COL_DERIV) && add != nullptr;
  if (has_add) {
#pragma unroll
    for (int e = 0; e < E; ++e) ad[e] = add[base + (long long)(j + LS * e) * a.inner];
  }
  WaveTwiddles<R, N, E> T;
  T.load(j, tw, twb);
  cplx<R>* S = lds + c * PADN;
  if (MODE == COL_INV) {
    wave_fft<R, N, E, true, BLK>(v, j, S, T);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cscale(v[e], scale);
  } else {
    wave_fft<R, N, E, false, BLK>(v, j, S, T);
  }
  if (MODE == COL_DERIV) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cmul_i(v[e], R(deriv_wavenumber(j + LS * e, N)) * scale);
    wave_fft<R, N, E, true, BLK>(v, j, S, T);
    if (has_add) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = cadd(v[e], ad[e]);
    }
  }
  if (live) {
#pragma unroll
    for (int e = 0; e < E; ++e) out[base + (long long)(j + LS * e) * a.inner] = v[e];
  }
}

// A column pass with one column group per workgroup; consecutive column groups are
// renumbered onto one XCD (the dispatcher deals workgroups to the 8 XCDs in turn).
template <typename R, int N, int E, int MODE>
__device__ __forceinline__ void col_w_body(const cplx<R>* in, const cplx<R>* add, cplx<R>* out, const ColArgs& a,
                                           R scale, const cplx<R>* __restrict__ tw, int twb, int fz) {
  using CS = ColShape<N, E>;
  __shared__ cplx<R> lds[CS::SPW * padded_e<E>(N)];
  const int nbx = gridDim.x;
  const int bx = (nbx % 8 == 0) ? (int)(blockIdx.x % 8) * (nbx / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
  col_w_at<R, N, E, MODE>(in, add, out, a, scale, tw, twb, fz, bx, (int)blockIdx.y, lds, (int)threadIdx.x);
}

template <typename R, int N, int E, int MODE>
__global__ __launch_bounds__((ColShape<N, E>::NT)) void k_col_w(const cplx<R>* in, const cplx<R>* add, cplx<R>* out,
                                                              ColArgs a, R scale, const cplx<R>* __restrict__ tw,
                                                              int twb) {
  col_w_body<R, N, E, MODE>(in, add, out, a, scale, tw, twb, (int)blockIdx.z);
}
// Batch-group form: blockIdx.z = item * nfz + field.
template <typename R, int N, int E, int MODE>
__global__ __launch_bounds__((ColShape<N, E>::NT)) void k_col_wt(const ColPtrs<R>* __restrict__ tab, ColArgs a, R scale,
                                                               const cplx<R>* __restrict__ tw, int twb, int nfz) {
  const ColPtrs<R> p = tab[blockIdx.z / nfz];
  if (p.inactive) return;
  col_w_body<R, N, E, MODE>(p.in, p.add, p.out, a, scale, tw, twb, (int)(blockIdx.z % nfz));
}

// The 2D control-space multiplier between its column transforms, in one pass: each
// column group takes column q of DW components (all D when the op mixes them: K, or the
// Hessian with the Stokes projection; else one, blockIdx.y = l * D + component) of
// coefficient l of X and, with HAS_Y, of Y; transforms them forward, applies the multiplier
// per mode (spec_plain, spec_packed) and transforms the results back into out (which may
// be X). Column 0 holds the packed planes, whose partner values (row -k_1 of the same
// column) come through LDS. The transforms run in lockstep (wave_fft_multi), so the result
// rounds like the separate forward pass, k_spec_mul and inverse pass up to the order of
// the butterflies' products. OP is a template argument so that each instance holds one
// multiplier's code.
template <typename R, int N, bool HAS_Y, int DW, int OP>
__device__ __forceinline__ void col_spec_body(const SpecArgs<R>& sa, int inner, const cplx<R>* __restrict__ tw,
                                              int twb) {
  constexpr int E = 8, D = 2;
  static_assert(DW == 1 || DW == D, "components per wavefront");
  using CS = ColShape<N, E>;
  static_assert(!CS::BLOCK && CS::NT == 64, "one wavefront per column group");
  constexpr int LS = CS::LS, SPW = CS::SPW;
  constexpr int PADN = padded_e<E>(N);
  constexpr int NF = HAS_Y ? 2 * DW : DW;
  // per column: NF sequences (FFT scratch, then the packed column's staged spectra), and
  // the packed column's DW results
  constexpr int SLOT = (NF + DW) * PADN;
  __shared__ cplx<R> lds[SPW * SLOT];
  const int lane = threadIdx.x;
  const int c = lane % SPW, j = lane / SPW;
  const int nbx = gridDim.x;
  const int bx = (nbx % 8 == 0) ? (int)(blockIdx.x % 8) * (nbx / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
  const long long colr = (long long)bx * SPW + c;
  const bool live = colr < inner;
  const int q = (int)(live ? colr : inner - 1);
  const int l = (int)blockIdx.y / (D / DW);
  const int c0 = ((int)blockIdx.y % (D / DW)) * DW;   // first component of this group
  const long long base = (long long)l * D * sa.nspec + (long long)c0 * sa.nspec + q;
  cplx<R>* S = lds + c * SLOT;
  WaveTwiddles<R, N, E> T;
  T.load(j, tw, twb);
  cplx<R> v[NF][E];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const cplx<R>* src = (f < DW ? sa.X : sa.Y) + base + (long long)(f % DW) * sa.nspec;
#pragma unroll
    for (int e = 0; e < E; ++e) v[f][e] = src[(long long)(j + LS * e) * inner];
  }
  wave_fft_multi<R, N, E, false, NF, NF>(v, j, S, PADN, T);
  // Column q > 0: each lane applies the multiplier to its E modes in registers. The packed
  // column q = 0 (in the group that holds column 0, the same for every lane of the
  // wavefront) stages its transformed sequences in LDS, where each mode finds its partner
  // at row -k_1, and runs one loop over its modes there (kept out of the unrolled code, so
  // the other columns' instruction stream stays short); its results return through LDS.
  const cplx<R> zero = {R(0), R(0)};
  // component i of the multiplier's input: sequence i; with one component per wavefront
  // the group's component sits in slot 0 and slot 1 is zero (the op does not mix them, so
  // slot 0's output is that component's, whichever it is)
  auto gather = [&](int i, const cplx<R>* seq, cplx<R>& xi, cplx<R>& yi) {
    const bool mine = DW == D || i == 0;
    xi = mine ? seq[DW == D ? i : 0] : zero;
    if (HAS_Y) yi = mine ? seq[DW + (DW == D ? i : 0)] : zero;
  };
  const bool packed = bx == 0;
  if (packed) {
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int e = 0; e < E; ++e) S[f * N + j + LS * e] = v[f][e];
    wave_lds_sync();
    if (q == 0) {
      cplx<R>* Sout = S + NF * N;   // DW result sequences
#pragma unroll 1
      for (int e = 0; e < E; ++e) {
        const int i1 = j + LS * e, ip = (N - i1) & (N - 1);
        R kv[3], kt[3];
        kv[0] = R(wavenumber(i1, N)); kt[0] = R(deriv_wavenumber(i1, N));
        cplx<R> own[NF], par[NF], x[D], y[D], xp[D], yp[D], o[D];
#pragma unroll
        for (int f = 0; f < NF; ++f) { own[f] = S[f * N + i1]; par[f] = S[f * N + ip]; }
#pragma unroll
        for (int i = 0; i < D; ++i) { gather(i, own, x[i], y[i]); gather(i, par, xp[i], yp[i]); }
        spec_packed<R, D>(sa, OP, kv, kt, HAS_Y, x, y, xp, yp, o);
#pragma unroll
        for (int i = 0; i < DW; ++i) Sout[i * N + i1] = o[i];
      }
    }
    wave_lds_sync();
    if (q == 0) {
#pragma unroll
      for (int i = 0; i < DW; ++i)
#pragma unroll
        for (int e = 0; e < E; ++e) v[i][e] = S[NF * N + i * N + j + LS * e];
    }
    wave_lds_sync();   // the result reads precede the inverse transforms' exchanges
  }
  if (q > 0) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i1 = j + LS * e;
      R kv[3], kt[3];
      kv[0] = R(wavenumber(i1, N)); kt[0] = R(deriv_wavenumber(i1, N));
      cplx<R> own[NF], x[D], y[D], o[D];
#pragma unroll
      for (int f = 0; f < NF; ++f) own[f] = v[f][e];
#pragma unroll
      for (int i = 0; i < D; ++i) gather(i, own, x[i], y[i]);
      spec_plain<R, D>(sa, OP, kv, kt, q, HAS_Y, x, y, o);
#pragma unroll
      for (int i = 0; i < DW; ++i) v[i][e] = o[i];
    }
  }
  wave_fft_multi<R, N, E, true, DW, NF>(v, j, S, PADN, T);
  if (live) {
#pragma unroll
    for (int i = 0; i < DW; ++i)
#pragma unroll
      for (int e = 0; e < E; ++e) sa.out[base + (long long)i * sa.nspec + (long long)(j + LS * e) * inner] = v[i][e];
  }
}

template <typename R, int N, bool HAS_Y, int DW, int OP>
__global__ __launch_bounds__(64) void k_col_spec(SpecArgs<R> sa, int inner, const cplx<R>* __restrict__ tw, int twb) {
  col_spec_body<R, N, HAS_Y, DW, OP>(sa, inner, tw, twb);
}
// One launch over the items of a batch group: item blockIdx.z uses tab[blockIdx.z].
template <typename R, int N, bool HAS_Y, int DW, int OP>
__global__ __launch_bounds__(64) void k_col_spec_t(const SpecArgs<R>* __restrict__ tab, int inner,
                                                  const cplx<R>* __restrict__ tw, int twb) {
  col_spec_body<R, N, HAS_Y, DW, OP>(tab[blockIdx.z], inner, tw, twb);
}

// Tiled column pass for long strided axes. A workgroup owns CT adjacent
// columns (CT * sizeof(cplx) = 64 or 128 bytes, a whole cache line per row):
// it stages the N x CT tile through LDS with row-coalesced loads, transforms
// the columns with the register wave FFT (E = 8), using each column's own tile
// slots as its exchange scratch, and writes the tile back row-coalesced.
// Column passes of the plain kernel touch one 8- or 16-byte element per row
// and rely on neighbouring workgroups to use the rest of each line; here every
// byte a row load fetches is used by the same workgroup. The tile is stored
// column by column (element r of column c at c * CPITCH + r + r / 8) with
// CPITCH = 2 mod 32, which keeps both the row-wise staging and the column
// transforms free of LDS bank conflicts. One tile per workgroup: the small
// register footprint lets four workgroups share a compute unit, which hides
// the staging latency better than prefetching the next tile would.
template <typename R, int N, int CT>
struct TileShape {
  static constexpr int E = 8;
  static constexpr int LS = WavePlan<N, E>::LS;   // lanes per column
  static_assert(LS <= 64, "a column fits one wavefront");
  static constexpr int SPW = 64 / LS;             // columns per wavefront per round
  static_assert(SPW <= CT, "a wavefront's columns fit in the tile");
  static constexpr int W = (CT / SPW) < 4 ? (CT / SPW) : 4;   // wavefronts per workgroup
  static constexpr int NT = 64 * W;
  static constexpr int PER_ROUND = W * SPW;       // divides CT: every lane owns a column
  static constexpr int ROUNDS = CT / PER_ROUND;
  static constexpr int CPITCH = ((padded_e<E>(N) + 29) / 32) * 32 + 2;   // >= padded length, = 2 mod 32
  static constexpr int ROWS_PER_STEP = NT / CT;   // tile rows per coalesced load step
  static_assert(CT % PER_ROUND == 0 && NT % CT == 0 && N % (NT / CT) == 0, "tile shape");
  static_assert(CPITCH >= padded_e<E>(N) && CPITCH % 32 == 2, "tile pitch");
};

template <typename R, int N, int CT, int MODE>
__device__ __forceinline__ void col_t_body(const cplx<R>* in, const cplx<R>* add, cplx<R>* out, const ColArgs& a,
                                           R scale, const cplx<R>* __restrict__ tw, int twb, int fz) {
  using TS = TileShape<R, N, CT>;
  constexpr int E = TS::E, LS = TS::LS, SPW = TS::SPW, CP = TS::CPITCH;
  constexpr int RPS = TS::ROWS_PER_STEP;
  constexpr int K = N / RPS;                      // tile elements each thread moves
  __shared__ cplx<R> tile[CT * CP];
  const int t = threadIdx.x;
  const int tc0 = t % CT, r0 = t / CT;
  const int w = t >> 6, lane = t & 63;
  const int cl = lane / LS, j = lane % LS;        // a half-wavefront's exchanges stay in one column
  // tile (x, y) covers columns x * CT .. x * CT + CT - 1 of outer slice y
  const int x = (int)blockIdx.x % a.ntx, y = (int)blockIdx.x / a.ntx;
  const long long base = (long long)fz * a.field + (long long)y * N * a.inner + (long long)x * CT;
  // row-coalesced load of the N x CT tile
#pragma unroll
  for (int k = 0; k < K; ++k)
    tile[tc0 * CP + pad_e<E>(r0 + k * RPS)] = in[base + (long long)(r0 + k * RPS) * a.inner + tc0];
  WaveTwiddles<R, N, E> T;
  T.load(j, tw, twb);
  __syncthreads();
#pragma unroll 1
  for (int rd = 0; rd < TS::ROUNDS; ++rd) {
    cplx<R>* col = tile + (rd * TS::PER_ROUND + w * SPW + cl) * CP;
    cplx<R> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = col[pad_e<E>(j + LS * e)];
    // the wavefront's reads of its columns complete before exchanges overwrite them
    wave_lds_sync();
    if (MODE == COL_INV) {
      wave_fft<R, N, E, true>(v, j, col, T);
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = cscale(v[e], scale);
    } else {
      wave_fft<R, N, E, false>(v, j, col, T);
    }
    if (MODE == COL_DERIV) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = cmul_i(v[e], R(deriv_wavenumber(j + LS * e, N)) * scale);
      wave_fft<R, N, E, true>(v, j, col, T);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) col[pad_e<E>(j + LS * e)] = v[e];
  }
  __syncthreads();
  const bool has_add = (MODE == COL_DERIV) && add != nullptr;
#pragma unroll 4
  for (int k = 0; k < K; ++k) {
    const int r = r0 + k * RPS;
    const long long gi = base + (long long)r * a.inner + tc0;
    cplx<R> v = tile[tc0 * CP + pad_e<E>(r)];
    if (has_add) v = cadd(v, add[gi]);
    out[gi] = v;
  }
}

template <typename R, int N, int CT, int MODE>
__global__ __launch_bounds__((TileShape<R, N, CT>::NT)) void k_col_t(const cplx<R>* in, const cplx<R>* add,
                                                                     cplx<R>* out, ColArgs a, R scale,
                                                                     const cplx<R>* __restrict__ tw, int twb) {
  col_t_body<R, N, CT, MODE>(in, add, out, a, scale, tw, twb, (int)blockIdx.z);
}
// Batch-group form: blockIdx.z = item * nfz + field.
template <typename R, int N, int CT, int MODE>
__global__ __launch_bounds__((TileShape<R, N, CT>::NT)) void k_col_tt(const ColPtrs<R>* __restrict__ tab, ColArgs a,
                                                                      R scale, const cplx<R>* __restrict__ tw, int twb,
                                                                      int nfz) {
  const ColPtrs<R> p = tab[blockIdx.z / nfz];
  if (p.inactive) return;
  col_t_body<R, N, CT, MODE>(p.in, p.add, p.out, a, scale, tw, twb, (int)(blockIdx.z % nfz));
}

}  // namespace nk
