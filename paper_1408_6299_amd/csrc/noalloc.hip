// Spectral gradient that allocates nothing: the row spectra and the twiddle table
// live in one file-scope device array (`scratch`), so the call needs neither a
// handle (whose creation allocates) nor any device allocation. It runs the kernels
// of nkreg_gradient on the same values in the same order, so the results are the
// same bits.
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/nkreg.h"
#include "spectral.hpp"

namespace {

// Twiddles (at most 512 complex doubles = 8 KiB) in the first 16 KiB, then up to three
// row spectra of the field (x1 and x2 derivatives in 3D), 8 MiB together.
constexpr size_t kTwiddleBytes = 16u << 10;
constexpr size_t kSpectraBytes = 8u << 20;
constexpr size_t kScratchBytes = kTwiddleBytes + kSpectraBytes;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each GPU, looked up once per device with that device
// current (the array's name is a host-side stand-in, never a device address).
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

unsigned char* scratch_on_current_device() {
  int dev = -1;
  NK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw nk::HipError(NKREG_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      throw nk::HipError(NKREG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = ptr;
  }
  return static_cast<unsigned char*>(g_scratch[dev]);
}

template <typename R>
void gradient_in_scratch(const nk::Grid& g, const R* u, R* out, hipStream_t st, unsigned char* base) {
  // the host table is uploaded on every call (8 KiB at most): calls on one GPU share
  // the array, and a call may follow one of another grid or precision
  static thread_local nk::cplx<R> host_tw[nk::kMaxN];
  nk::Spectral<R>::twiddles(g.lmax, host_tw);
  nk::cplx<R>* tw = reinterpret_cast<nk::cplx<R>*>(base);
  NK_HIP(hipMemcpyAsync(tw, host_tw, sizeof(nk::cplx<R>) * g.lmax, hipMemcpyHostToDevice, st));
  nk::cplx<R>* T = reinterpret_cast<nk::cplx<R>*>(base + kTwiddleBytes);
  nk::cplx<R>* S1 = T + g.nspec;
  nk::cplx<R>* S2 = S1 + g.nspec;
  nk::Spectral<R> sp(g, st, tw);
  sp.gradient(u, out, 1, T, S1, S2);
}

bool pow2_in_range(int v) { return v >= nk::kMinN && v <= nk::kMaxN && (v & (v - 1)) == 0; }

int fail(int code, const std::string& msg) {
  nk::set_last_error(msg);
  return code;
}

}  // namespace

extern "C" int nkreg_gradient_noalloc(int dim, const int* n, int precision, const void* d_u, void* d_g,
                                      void* hip_stream) {
  if (!n || !d_u || !d_g) return fail(NKREG_EINVAL, "null argument");
  if (dim != 2 && dim != 3) return fail(NKREG_EINVAL, "dim must be 2 or 3");
  if (precision != 32 && precision != 64) return fail(NKREG_EINVAL, "precision must be 32 or 64");
  for (int i = 0; i < dim; ++i)
    if (!pow2_in_range(n[i])) return fail(NKREG_ESHAPE, "grid sizes must be powers of two in [8, 512]");
  const nk::Grid g = nk::make_grid(dim, n);
  const size_t rsize = precision == 32 ? sizeof(float) : sizeof(double);
  const int spectra = dim == 3 ? 3 : 2;
  if ((size_t)g.npts * rsize * spectra > kSpectraBytes)
    return fail(NKREG_ESHAPE, "grid too large for the fixed scratch: " + std::to_string(spectra) +
                                  " spectra of " + std::to_string((size_t)g.npts * rsize) + " bytes exceed " +
                                  std::to_string(kSpectraBytes) + " bytes");
  try {
    unsigned char* base = scratch_on_current_device();
    hipStream_t st = (hipStream_t)hip_stream;
    if (precision == 32) gradient_in_scratch<float>(g, (const float*)d_u, (float*)d_g, st, base);
    else gradient_in_scratch<double>(g, (const double*)d_u, (double*)d_g, st, base);
  } catch (const nk::HipError& e) {
    return fail(e.code, e.what());
  } catch (...) {
    return fail(NKREG_EHIP, "unknown error");
  }
  return NKREG_OK;
}
