// Register-resident FFTs inside one wavefront.
//
// A length-M sequence is held by LS = M / E lanes of a wavefront, E elements
// per lane, lane j holding x[j + LS * e] in a[e] ("natural layout"). The
// transform is a Stockham autosort with radix-E passes and, when log2(M) is
// not a multiple of log2(E), one final pass of smaller radix. Each pass reads
// its inputs from registers; intermediate passes exchange through a
// wave-private LDS scratch region; the last pass leaves its outputs in natural
// layout in the same registers, so a transform costs (passes - 1) exchanges.
// Twiddles come from the FP64-computed table tw[m] = exp(-2 pi i m / Lmax);
// a lane's twiddles for all passes are loaded up front into registers.
#pragma once

#include "common.hpp"

namespace nk {

// Orders this wavefront's LDS accesses across an exchange: the LDS unit runs a
// wavefront's instructions in issue order, so a read issued after the writes of
// the other lanes sees them, and a later write cannot overtake an earlier read;
// what must not happen is the compiler moving an access across this point, which
// the wavefront-scope fences forbid. No wait is issued here: the LDS writes of an
// exchange overlap the reads that follow them, and results are waited for only
// where registers use them. Other waves are not involved.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename R, bool INV>
__device__ __forceinline__ void bfly2(cplx<R>& a, cplx<R>& b) {
  const cplx<R> t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

// 4-point DFT in place: a[0..3] -> y[0..3] (forward uses exp(-2 pi i / 4))
template <typename R, bool INV>
__device__ __forceinline__ void dft4r(cplx<R>& a0, cplx<R>& a1, cplx<R>& a2, cplx<R>& a3) {
  const cplx<R> s02 = cadd(a0, a2), d02 = csub(a0, a2);
  const cplx<R> s13 = cadd(a1, a3), d13 = csub(a1, a3);
  const cplx<R> id13 = INV ? cplx<R>{-d13.y, d13.x} : cplx<R>{d13.y, -d13.x};
  a0 = cadd(s02, s13);
  a2 = csub(s02, s13);
  a1 = cadd(d02, id13);
  a3 = csub(d02, id13);
}

// 8-point DFT in place (decimation in frequency into two 4-point DFTs).
template <typename R, bool INV>
__device__ __forceinline__ void dft8r(cplx<R> (&a)[8]) {
  constexpr R h = R(0.70710678118654752440);
  cplx<R> b0 = cadd(a[0], a[4]), b4 = csub(a[0], a[4]);
  cplx<R> b1 = cadd(a[1], a[5]), b5 = csub(a[1], a[5]);
  cplx<R> b2 = cadd(a[2], a[6]), b6 = csub(a[2], a[6]);
  cplx<R> b3 = cadd(a[3], a[7]), b7 = csub(a[3], a[7]);
  // b5 *= w8, b6 *= w8^2, b7 *= w8^3 with w8 = exp(-+ i pi / 4)
  if (!INV) {
    b5 = {h * (b5.x + b5.y), h * (b5.y - b5.x)};
    b6 = {b6.y, -b6.x};
    b7 = {h * (b7.y - b7.x), -h * (b7.x + b7.y)};
  } else {
    b5 = {h * (b5.x - b5.y), h * (b5.y + b5.x)};
    b6 = {-b6.y, b6.x};
    b7 = {-h * (b7.x + b7.y), h * (b7.x - b7.y)};
  }
  dft4r<R, INV>(b0, b1, b2, b3);
  dft4r<R, INV>(b4, b5, b6, b7);
  a[0] = b0; a[2] = b1; a[4] = b2; a[6] = b3;
  a[1] = b4; a[3] = b5; a[5] = b6; a[7] = b7;
}

template <typename R, bool INV, int RR>
__device__ __forceinline__ void dft_small(cplx<R> (&v)[RR]) {
  if constexpr (RR == 2) {
    bfly2<R, INV>(v[0], v[1]);
  } else if constexpr (RR == 4) {
    dft4r<R, INV>(v[0], v[1], v[2], v[3]);
  } else {
    dft8r<R, INV>(v);
  }
}

// Compile-time plan of a length-M transform with E elements per lane.
template <int M, int E>
struct WavePlan {
  static_assert((M & (M - 1)) == 0 && (E == 2 || E == 4 || E == 8) && M >= E, "plan");
  static_assert(M / E <= 256, "a sequence spans at most four wavefronts");
  static constexpr int LOG = ilog2(M);
  static constexpr int LE = ilog2(E);
  static constexpr int NFULL = LOG / LE;           // radix-E passes
  static constexpr int REM = LOG % LE;             // last pass radix 2^REM if REM > 0
  static constexpr int NP = NFULL + (REM ? 1 : 0);
  static constexpr int LS = M / E;                 // lanes per sequence
  static constexpr int RLAST = REM ? (1 << REM) : E;
  // twiddles per lane: passes 1..NFULL-1 need E-1 each; the remainder pass (if any)
  // has E / RLAST butterflies of RLAST - 1 twiddles
  static constexpr int NTW = (NFULL - 1) * (E - 1) + (REM ? (E / RLAST) * (RLAST - 1) : 0);
  static constexpr int NTWA = NTW > 0 ? NTW : 1;
  static constexpr int ns(int p) {  // Ns before pass p
    int v = 1;
    for (int i = 0; i < p; ++i) v *= E;
    return v;
  }
};

template <typename R, int M, int E>
struct WaveTwiddles {
  using P = WavePlan<M, E>;
  cplx<R> w[P::NTWA];
  // twb = Lmax / M
  __device__ __forceinline__ void load(int j, const cplx<R>* __restrict__ tw, int twb) {
    int c = 0;
#pragma unroll
    for (int p = 1; p < P::NFULL; ++p) {
      const int Ns = P::ns(p);
      const int kk = j % Ns;                       // one butterfly per lane in radix-E passes
      const int step = (M / (E * Ns)) * twb * kk;
#pragma unroll
      for (int r = 1; r < E; ++r) w[c++] = tw[r * step];
    }
    if constexpr (P::REM > 0) {
      constexpr int RR = P::RLAST;
      constexpr int Ns = M / RR;
      constexpr int BPL = E / RR;
#pragma unroll
      for (int b = 0; b < BPL; ++b) {
        const int kk = (j + b * P::LS) % Ns;
        const int step = (M / (RR * Ns)) * twb * kk;
#pragma unroll
        for (int r = 1; r < RR; ++r) w[c++] = tw[r * step];
      }
    }
  }
};

// Scratch layout of a sequence: element i at s[i + i / E] (one pad slot per E
// elements). The first Stockham pass writes each lane's E outputs at unit
// stride, i.e. lanes E elements apart; the pad spreads those lanes over all
// LDS banks (and keeps unit-stride accesses conflict-free).
template <int E>
__device__ __forceinline__ int pad_e(int i) { return i + i / E; }
template <int E>
constexpr int padded_e(int m) { return m + m / E + 1; }

// Butterflies of Stockham pass p on one lane's E elements (a[b + r * BPL] is
// input r of butterfly b). Passes after the first take their twiddles from T in
// pass order, E - 1 (or RLAST - 1) per butterfly.
template <typename R, int M, int E, bool INV>
__device__ __forceinline__ void fft_pass(cplx<R> (&a)[E], int p, const WaveTwiddles<R, M, E>& T) {
  using P = WavePlan<M, E>;
  const bool rem = (P::REM > 0) && (p == P::NP - 1);
  const int RR = rem ? P::RLAST : E;
  const int BPL = E / RR;
  int c = p > 0 ? (p - 1) * (E - 1) : 0;
#pragma unroll
  for (int b = 0; b < BPL; ++b) {
    if (RR == E) {
      cplx<R> v[E];
#pragma unroll
      for (int r = 0; r < E; ++r) v[r] = a[b + r * BPL];
      if (p > 0) {
#pragma unroll
        for (int r = 1; r < E; ++r) {
          cplx<R> w = T.w[c++];
          if (INV) w.y = -w.y;
          v[r] = cmul(v[r], w);
        }
      }
      dft_small<R, INV, E>(v);
#pragma unroll
      for (int r = 0; r < E; ++r) a[b + r * BPL] = v[r];
    } else {
      constexpr int RL = P::RLAST;
      cplx<R> v[RL];
#pragma unroll
      for (int r = 0; r < RL; ++r) v[r] = a[b + r * BPL];
      if (p > 0) {
#pragma unroll
        for (int r = 1; r < RL; ++r) {
          cplx<R> w = T.w[c++];
          if (INV) w.y = -w.y;
          v[r] = cmul(v[r], w);
        }
      }
      dft_small<R, INV, RL>(v);
#pragma unroll
      for (int r = 0; r < RL; ++r) a[b + r * BPL] = v[r];
    }
  }
}

// Scatter of pass p's outputs into the sequence's scratch: the outputs of
// butterfly k = j + b * LS go to (k / Ns) * RR * Ns + k % Ns + r * Ns.
template <typename R, int M, int E>
__device__ __forceinline__ void fft_scatter(const cplx<R> (&a)[E], int p, int j, cplx<R>* s) {
  using P = WavePlan<M, E>;
  constexpr int LS = P::LS;
  const bool rem = (P::REM > 0) && (p == P::NP - 1);
  const int RR = rem ? P::RLAST : E;
  const int BPL = E / RR;
  const int Ns = P::ns(p);
#pragma unroll
  for (int b = 0; b < BPL; ++b) {
    const int k = j + b * LS;
    const int kk = k % Ns;
    const int base = (k - kk) * RR + kk;
#pragma unroll
    for (int r = 0; r < RR; ++r) s[pad_e<E>(base + r * Ns)] = a[b + r * BPL];
  }
}

// Lane j's elements j + LS * e of the sequence in scratch.
template <typename R, int M, int E>
__device__ __forceinline__ void fft_gather(cplx<R> (&a)[E], int j, const cplx<R>* s) {
  constexpr int LS = WavePlan<M, E>::LS;
#pragma unroll
  for (int e = 0; e < E; ++e) a[e] = s[pad_e<E>(j + LS * e)];
}

// Exchange canary: the sequence's lanes overwrite its whole scratch with NaN. Issued
// (and fenced) before a scatter, it checks that the gather after the scatter's fence
// sees the scatter (a read served before the wavefront's earlier writes would return
// NaN); issued after the gather's fence, it checks that no later write overtakes the
// gather's reads. Each poison sits where the production code has a fence, so the
// compiler cannot move it past the exchange it brackets.
template <typename R, int M, int E>
__device__ __forceinline__ void poison_scratch(int j, cplx<R>* s) {
  constexpr int LS = WavePlan<M, E>::LS;
  const R nan = __builtin_nan("");
  for (int i = j; i < padded_e<E>(M); i += LS) s[i] = cplx<R>{nan, nan};
}

// BLOCK = true when a sequence spans several wavefronts of the workgroup
// (M / E > 64 lanes): exchanges then synchronise the whole workgroup. POISON runs the
// exchange canary around every exchange (test builds only; same results when the
// exchanges are ordered).
template <typename R, int M, int E, bool INV, bool BLOCK = false, bool POISON = false>
__device__ __forceinline__ void wave_fft(cplx<R> (&a)[E], int j, cplx<R>* s, const WaveTwiddles<R, M, E>& T) {
  using P = WavePlan<M, E>;
#pragma unroll
  for (int p = 0; p < P::NP; ++p) {
    fft_pass<R, M, E, INV>(a, p, T);
    if (p != P::NP - 1) {
      if (POISON) {
        poison_scratch<R, M, E>(j, s);
        wave_lds_sync();
      }
      fft_scatter<R, M, E>(a, p, j, s);
      if (BLOCK) __syncthreads(); else wave_lds_sync();
      fft_gather<R, M, E>(a, j, s);
      if (BLOCK) __syncthreads(); else wave_lds_sync();
      if (POISON) poison_scratch<R, M, E>(j, s);
    }
  }
}

// NK independent sequences of one wavefront (a[k], scratch s + k * pitch)
// transformed in lockstep: each pass runs on every sequence before the one
// exchange wait, so the LDS round trips of the sequences overlap. Per sequence
// the arithmetic is that of wave_fft.
template <typename R, int M, int E, bool INV, int NK, int KA, bool POISON = false>
__device__ __forceinline__ void wave_fft_multi(cplx<R> (&a)[KA][E], int j, cplx<R>* s, int pitch,
                                               const WaveTwiddles<R, M, E>& T) {
  static_assert(NK >= 1 && NK <= KA, "sequence count");
  using P = WavePlan<M, E>;
  static_assert(P::LS <= 64, "a sequence fits one wavefront");
#pragma unroll
  for (int p = 0; p < P::NP; ++p) {
#pragma unroll
    for (int k = 0; k < NK; ++k) fft_pass<R, M, E, INV>(a[k], p, T);
    if (p != P::NP - 1) {
      if (POISON) {
        for (int k = 0; k < NK; ++k) poison_scratch<R, M, E>(j, s + k * pitch);
        wave_lds_sync();
      }
#pragma unroll
      for (int k = 0; k < NK; ++k) fft_scatter<R, M, E>(a[k], p, j, s + k * pitch);
      wave_lds_sync();
#pragma unroll
      for (int k = 0; k < NK; ++k) fft_gather<R, M, E>(a[k], j, s + k * pitch);
      wave_lds_sync();
      if (POISON)
        for (int k = 0; k < NK; ++k) poison_scratch<R, M, E>(j, s + k * pitch);
    }
  }
}

}  // namespace nk
