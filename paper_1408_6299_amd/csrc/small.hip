// Instances of the persistent small-grid kernel (square 2D grids of 8 to 64 points).
#include "small.hpp"

namespace nk {

namespace {

template <typename R, int N, bool NC1>
void launch_n(int items, const SmallOp* prog, int nops, const unsigned char* tab, const void* tw, int lmax,
              hipStream_t st) {
  hipLaunchKernelGGL((k_small<R, N, N, NC1>), dim3(items), dim3(SmallWaves<R>::NT), 0, st, prog, nops, tab,
                     (const cplx<R>*)tw, lmax);
}

template <typename R, bool NC1>
bool launch_r(int n, int items, const SmallOp* prog, int nops, const unsigned char* tab, const void* tw, int lmax,
              hipStream_t st) {
  switch (n) {
    case 8: launch_n<R, 8, NC1>(items, prog, nops, tab, tw, lmax, st); return true;
    case 16: launch_n<R, 16, NC1>(items, prog, nops, tab, tw, lmax, st); return true;
    case 32: launch_n<R, 32, NC1>(items, prog, nops, tab, tw, lmax, st); return true;
    case 64: launch_n<R, 64, NC1>(items, prog, nops, tab, tw, lmax, st); return true;
    default: return false;
  }
}

}  // namespace

bool launch_small(bool f64, int n1, int l, bool nc1, int items, const SmallOp* prog, int nops,
                  const unsigned char* tab, const void* tw, int lmax, hipStream_t st) {
  if (n1 != l) return false;
  bool ok;
  if (f64) ok = nc1 ? launch_r<double, true>(n1, items, prog, nops, tab, tw, lmax, st)
                    : launch_r<double, false>(n1, items, prog, nops, tab, tw, lmax, st);
  else ok = nc1 ? launch_r<float, true>(n1, items, prog, nops, tab, tw, lmax, st)
                : launch_r<float, false>(n1, items, prog, nops, tab, tw, lmax, st);
  if (ok) NK_LAUNCHED();
  return ok;
}

}  // namespace nk
