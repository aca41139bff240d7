// Exchange canary of the register FFTs (test instrumentation): a forward and an inverse
// transform of `count` sequences, with or without NaN poisoning of the LDS scratch
// around every exchange. The transforms order each wavefront's exchanges with fences
// and no wait, relying on the LDS unit running a wavefront's instructions in order; if
// a read were served before the wavefront's earlier writes, or a later write overtook a
// read, the poison would reach the output.
#include <string>
#include <vector>

#include "../../include/nkreg.h"
#include "spectral.hpp"

namespace nk {
namespace {

template <typename R, int M, int E, int NK, bool POISON>
__global__ __launch_bounds__(64) void k_fft_canary(const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out,
                                                   int count, const cplx<R>* __restrict__ tw) {
  using P = WavePlan<M, E>;
  constexpr int LS = P::LS, SPW = 64 / LS, PADM = padded_e<E>(M);
  __shared__ cplx<R> lds[SPW * NK * PADM];
  const int lane = threadIdx.x, sr = lane / LS, j = lane % LS;
  const long long seq0 = ((long long)blockIdx.x * SPW + sr) * NK;
  cplx<R> a[NK][E];
#pragma unroll
  for (int k = 0; k < NK; ++k)
#pragma unroll
    for (int e = 0; e < E; ++e)
      a[k][e] = seq0 + k < count ? in[(seq0 + k) * M + j + LS * e] : cplx<R>{R(0), R(0)};
  WaveTwiddles<R, M, E> T;
  T.load(j, tw, 1);
  cplx<R>* S = lds + sr * NK * PADM;
  if constexpr (NK == 1) {
    wave_fft<R, M, E, false, false, POISON>(a[0], j, S, T);
    wave_fft<R, M, E, true, false, POISON>(a[0], j, S, T);
  } else {
    wave_fft_multi<R, M, E, false, NK, NK, POISON>(a, j, S, PADM, T);
    wave_fft_multi<R, M, E, true, NK, NK, POISON>(a, j, S, PADM, T);
  }
#pragma unroll
  for (int k = 0; k < NK; ++k)
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (seq0 + k < count) out[(seq0 + k) * M + j + LS * e] = a[k][e];
}

template <typename R, int M, int E, int NK>
void run(bool poison, const void* in, void* out, int count, hipStream_t st) {
  std::vector<cplx<R>> h(M);
  Spectral<R>::twiddles(M, h.data());
  cplx<R>* tw = nullptr;
  NK_HIP(hipMalloc(&tw, sizeof(cplx<R>) * M));
  NK_HIP(hipMemcpy(tw, h.data(), sizeof(cplx<R>) * M, hipMemcpyHostToDevice));
  constexpr int SPW = 64 / WavePlan<M, E>::LS;
  const dim3 grid((unsigned)((count + SPW * NK - 1) / (SPW * NK)));
  if (poison)
    hipLaunchKernelGGL((k_fft_canary<R, M, E, NK, true>), grid, dim3(64), 0, st, (const cplx<R>*)in, (cplx<R>*)out,
                       count, (const cplx<R>*)tw);
  else
    hipLaunchKernelGGL((k_fft_canary<R, M, E, NK, false>), grid, dim3(64), 0, st, (const cplx<R>*)in,
                       (cplx<R>*)out, count, (const cplx<R>*)tw);
  const hipError_t e = hipGetLastError();
  const hipError_t s = hipStreamSynchronize(st);
  (void)hipFree(tw);
  if (e != hipSuccess || s != hipSuccess) throw HipError(-4, "canary kernel failed");
}

// The (length, elements per lane, lockstep sequences) forms the library's kernels use.
template <typename R>
bool dispatch(int m, int e, int nk, bool poison, const void* in, void* out, int count, hipStream_t st) {
  if (e == 4 && nk == 1) {
    if (m == 32) { run<R, 32, 4, 1>(poison, in, out, count, st); return true; }
    if (m == 128) { run<R, 128, 4, 1>(poison, in, out, count, st); return true; }
    if (m == 256) { run<R, 256, 4, 1>(poison, in, out, count, st); return true; }
  } else if (e == 4 && nk == 2) {
    if (m == 32) { run<R, 32, 4, 2>(poison, in, out, count, st); return true; }
    if (m == 128) { run<R, 128, 4, 2>(poison, in, out, count, st); return true; }
    if (m == 256) { run<R, 256, 4, 2>(poison, in, out, count, st); return true; }
  } else if (e == 2 && nk == 1) {
    if (m == 64) { run<R, 64, 2, 1>(poison, in, out, count, st); return true; }
    if (m == 128) { run<R, 128, 2, 1>(poison, in, out, count, st); return true; }
  } else if (e == 2 && nk == 2) {
    if (m == 64) { run<R, 64, 2, 2>(poison, in, out, count, st); return true; }
    if (m == 128) { run<R, 128, 2, 2>(poison, in, out, count, st); return true; }
  } else if (e == 8 && nk == 1) {
    if (m == 64) { run<R, 64, 8, 1>(poison, in, out, count, st); return true; }
    if (m == 256) { run<R, 256, 8, 1>(poison, in, out, count, st); return true; }
    if (m == 512) { run<R, 512, 8, 1>(poison, in, out, count, st); return true; }
  }
  return false;
}

}  // namespace
}  // namespace nk

extern "C" int nkreg_exchange_canary(int precision, int m, int elems, int lockstep, int poison, const void* d_in,
                                     void* d_out, int count, void* hip_stream) {
  if (!d_in || !d_out || count < 0 || (precision != 32 && precision != 64)) {
    nk::set_last_error("bad canary arguments");
    return NKREG_EINVAL;
  }
  try {
    hipStream_t st = (hipStream_t)hip_stream;
    const bool ok = precision == 32 ? nk::dispatch<float>(m, elems, lockstep, poison != 0, d_in, d_out, count, st)
                                    : nk::dispatch<double>(m, elems, lockstep, poison != 0, d_in, d_out, count, st);
    if (!ok) {
      nk::set_last_error("no canary instance for this transform shape");
      return NKREG_ENOTIMPL;
    }
  } catch (const nk::HipError& e) {
    nk::set_last_error(e.what());
    return e.code;
  }
  return NKREG_OK;
}
