// Batched complex FFTs staged in LDS, plus the real<->half-complex packing
// steps, for power-of-two lengths.
//
// Layout: NSEQ sequences of length M live in LDS; element e of sequence s is
// at buf[s * ss + e * es]. The transform is a Stockham autosort (natural order
// in, natural order out), radix-4 passes and one radix-2 pass when log2(M) is
// odd. Every thread of the workgroup must call these routines (they contain
// __syncthreads). Twiddles come from a table tw[m] = exp(-2 pi i m / Lmax)
// computed on the host in FP64; a length-M transform reads it with stride
// Lmax / M (passed as twb).
#pragma once

#include "common.hpp"

namespace nk {

template <typename R, bool INV>
__device__ __forceinline__ void dft4(cplx<R>& a0, cplx<R>& a1, cplx<R>& a2, cplx<R>& a3) {
  const cplx<R> s02 = cadd(a0, a2), d02 = csub(a0, a2);
  const cplx<R> s13 = cadd(a1, a3), d13 = csub(a1, a3);
  // forward: y1 = d02 - i d13, y3 = d02 + i d13; inverse swaps the signs of i
  const cplx<R> id13 = INV ? cplx<R>{-d13.y, d13.x} : cplx<R>{d13.y, -d13.x};
  a0 = cadd(s02, s13);
  a2 = csub(s02, s13);
  a1 = cadd(d02, id13);
  a3 = csub(d02, id13);
}

template <typename R, bool INV>
__device__ __forceinline__ cplx<R> twiddle(const cplx<R>* __restrict__ tw, int idx) {
  cplx<R> w = tw[idx];
  if (INV) w.y = -w.y;
  return w;
}

// In-place batched FFT of NSEQ (<= nseq_max) sequences of length M.
// SEQ_FAST selects the thread -> butterfly mapping: consecutive threads take
// consecutive sequences (for strided column tiles) or consecutive elements of
// one sequence (for contiguous rows); both keep LDS accesses conflict-light.
template <typename R, int M, int NSEQ_MAX, int NT, bool INV, bool SEQ_FAST>
__device__ __forceinline__ void fft_lds(cplx<R>* buf, int nseq, int ss, int es,
                                        const cplx<R>* __restrict__ tw, int twb) {
  static_assert((M & (M - 1)) == 0 && M >= 2, "power-of-two length");
  constexpr int LOG = ilog2(M);
  constexpr int NP4 = LOG / 2;  // radix-4 passes
  constexpr int Q = M / 4;      // radix-4 butterflies per sequence
  const int tid = threadIdx.x;
  if constexpr (NP4 > 0) {
    constexpr int BPT = (NSEQ_MAX * Q + NT - 1) / NT;
    const int tot = nseq * Q;
#pragma unroll
    for (int pass = 0; pass < NP4; ++pass) {
      const int Ns = 1 << (2 * pass);
      cplx<R> a[BPT][4];
      int dst[BPT];
#pragma unroll
      for (int i = 0; i < BPT; ++i) {
        const int b = tid + i * NT;
        dst[i] = -1;
        if (b < tot) {
          int s, j;
          if (SEQ_FAST) { s = b % nseq; j = b / nseq; }
          else { s = b / Q; j = b % Q; }
          cplx<R>* base = buf + s * ss;
#pragma unroll
          for (int r = 0; r < 4; ++r) a[i][r] = base[(j + r * Q) * es];
          const int k = j & (Ns - 1);
          if (pass > 0) {
            // exp(-2 pi i r k / (4 Ns)) = tw[r k (M / (4 Ns)) twb]
            const int step = (M / (4 * Ns)) * twb * k;
            a[i][1] = cmul(a[i][1], twiddle<R, INV>(tw, step));
            a[i][2] = cmul(a[i][2], twiddle<R, INV>(tw, 2 * step));
            a[i][3] = cmul(a[i][3], twiddle<R, INV>(tw, 3 * step));
          }
          dft4<R, INV>(a[i][0], a[i][1], a[i][2], a[i][3]);
          dst[i] = s * ss + ((j - k) * 4 + k) * es;
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < BPT; ++i) {
        if (dst[i] >= 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r) buf[dst[i] + r * Ns * es] = a[i][r];
        }
      }
      __syncthreads();
    }
  }
  if constexpr (LOG & 1) {
    // Final radix-2 pass with Ns = M/2: butterfly j reads and writes j and j + M/2.
    constexpr int H = M / 2;
    constexpr int BPT2 = (NSEQ_MAX * H + NT - 1) / NT;
    const int tot2 = nseq * H;
#pragma unroll
    for (int i = 0; i < BPT2; ++i) {
      const int b = tid + i * NT;
      if (b < tot2) {
        int s, j;
        if (SEQ_FAST) { s = b % nseq; j = b / nseq; }
        else { s = b / H; j = b % H; }
        cplx<R>* base = buf + s * ss;
        cplx<R> a0 = base[j * es];
        cplx<R> a1 = base[(j + H) * es];
        if (M > 2) a1 = cmul(a1, twiddle<R, INV>(tw, j * twb));
        base[j * es] = cadd(a0, a1);
        base[(j + H) * es] = csub(a0, a1);
      }
    }
    __syncthreads();
  }
}

// After a forward complex FFT of length M of z[n] = x[2n] + i x[2n+1] (x real,
// length L = 2M), rewrite each sequence in place as the packed half spectrum
// of x: P[0] = (X_0, X_M) (both real), P[q] = X_q for 0 < q < M.
// twl = Lmax / L.
template <typename R, int M, int NT>
__device__ __forceinline__ void r2c_post(cplx<R>* buf, int nseq, int ss,
                                         const cplx<R>* __restrict__ tw, int twl) {
  constexpr int P = M / 2 + 1;
  const int tot = nseq * P;
  for (int b = threadIdx.x; b < tot; b += NT) {
    const int s = b / P, q = b % P;
    cplx<R>* base = buf + s * ss;
    if (q == 0) {
      const cplx<R> z = base[0];
      base[0] = {z.x + z.y, z.x - z.y};
    } else {
      const cplx<R> zq = base[q];
      const cplx<R> zm = base[M - q];
      const cplx<R> e = {R(0.5) * (zq.x + zm.x), R(0.5) * (zq.y - zm.y)};
      // o = (zq - conj(zm)) / (2i)
      const cplx<R> o = {R(0.5) * (zq.y + zm.y), -R(0.5) * (zq.x - zm.x)};
      const cplx<R> wo = cmul(o, tw[q * twl]);
      base[q] = cadd(e, wo);
      if (q != M - q) base[M - q] = cconj(csub(e, wo));
    }
  }
  __syncthreads();
}

// Inverse of r2c_post up to a factor: turns a packed half spectrum of a real
// row x of length L = 2M into Z such that the unnormalised inverse complex FFT
// of length M gives z[n] = L x[2n] + i L x[2n+1].
template <typename R, int M, int NT>
__device__ __forceinline__ void c2r_pre(cplx<R>* buf, int nseq, int ss,
                                        const cplx<R>* __restrict__ tw, int twl) {
  constexpr int P = M / 2 + 1;
  const int tot = nseq * P;
  for (int b = threadIdx.x; b < tot; b += NT) {
    const int s = b / P, q = b % P;
    cplx<R>* base = buf + s * ss;
    if (q == 0) {
      const cplx<R> p0 = base[0];
      base[0] = {p0.x + p0.y, p0.x - p0.y};
    } else {
      const cplx<R> xq = base[q];
      const cplx<R> xm = base[M - q];
      const cplx<R> e = {xq.x + xm.x, xq.y - xm.y};     // xq + conj(xm)
      const cplx<R> dq = {xq.x - xm.x, xq.y + xm.y};    // xq - conj(xm)
      const cplx<R> o = cmulc(dq, tw[q * twl]);          // dq * conj(w^q)
      base[q] = {e.x - o.y, e.y + o.x};                  // e + i o
      if (q != M - q) base[M - q] = {e.x + o.y, o.x - e.y};  // conj(e) + i conj(o)
    }
  }
  __syncthreads();
}

}  // namespace nk
