// Common device/host definitions of the gfx950 registration library.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace nk {

template <typename R>
struct alignas(2 * sizeof(R)) cplx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ cplx<R> cmulc(cplx<R> a, cplx<R> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename R>
__device__ __forceinline__ cplx<R> cconj(cplx<R> a) { return {a.x, -a.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) { return {a.x * s, a.y * s}; }
// multiply by i*s
template <typename R>
__device__ __forceinline__ cplx<R> cmul_i(cplx<R> a, R s) { return {-a.y * s, a.x * s}; }

// Signed integer wavenumber of FFT index i on an axis of length n (n even):
// 0..n/2-1 -> itself, n/2..n-1 -> i - n (so the Nyquist index maps to -n/2).
__device__ __forceinline__ int wavenumber(int i, int n) { return i < n / 2 ? i : i - n; }
// First-derivative wavenumber: as above but the Nyquist wavenumber -n/2 is 0.
__device__ __forceinline__ int deriv_wavenumber(int i, int n) {
  return i == n / 2 ? 0 : (i < n / 2 ? i : i - n);
}

constexpr int kMaxNc = 16;   // Chebyshev coefficients supported
constexpr int kMaxN = 512;   // largest axis length
constexpr int kMinN = 8;     // smallest axis length

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

}  // namespace nk
