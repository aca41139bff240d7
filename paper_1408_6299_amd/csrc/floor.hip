// Latency floor of chains of dependent launches (measurement instrumentation): HIP graphs of
// empty kernels and of plain row- or column-pattern copies of a complex FP32 array, each
// launch reading what the previous one wrote, timed per node. A transport matvec on a
// launch-bound grid is a chain of the same length whose nodes also do the transforms, so
// the copy chain is the time it could not go below with one launch per phase.
#include <string>

#include "../../include/nkreg.h"
#include "common.hpp"

namespace nk {
void set_last_error(const std::string& msg);
namespace {

__global__ void k_floor_empty(const float2* in, float2* out, int cols) {
  if (cols < 0 && threadIdx.x == 0) out[blockIdx.x] = in[blockIdx.x];   // never taken
}

// One wavefront per row: lane j copies elements j, j + 64, ... of row blockIdx.x.
__global__ __launch_bounds__(64) void k_floor_row(const float2* __restrict__ in, float2* __restrict__ out, int cols) {
  const long long base = (long long)blockIdx.x * cols;
  for (int c = threadIdx.x; c < cols; c += 64) out[base + c] = in[base + c];
}

// One wavefront per column: lane j copies rows j, j + 64, ... of column c; consecutive
// columns are renumbered onto one XCD as the column pass does.
__global__ __launch_bounds__(64) void k_floor_col(const float2* __restrict__ in, float2* __restrict__ out, int rows,
                                                  int cols) {
  const int nbx = gridDim.x;
  const int c = (nbx % 8 == 0) ? (int)(blockIdx.x % 8) * (nbx / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
  for (int r = threadIdx.x; r < rows; r += 64) out[(long long)r * cols + c] = in[(long long)r * cols + c];
}

}  // namespace
}  // namespace nk

extern "C" int nkreg_launch_floor(int kind, int rows, int cols, int nodes, void* hip_stream, double* h_us_per_node) {
  if (!h_us_per_node || kind < 0 || kind > 3 || rows < 64 || cols < 64 || rows > 4096 || cols > 4096 ||
      rows % 64 || cols % 64 || nodes < 2 || nodes > 4096) {
    nk::set_last_error("launch floor: bad arguments");
    return NKREG_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t n = (size_t)rows * cols;
  float2 *a = nullptr, *b = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t ex = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int status = NKREG_OK;
  auto ok = [&](hipError_t e) {
    if (e != hipSuccess && status == NKREG_OK) {
      status = e == hipErrorOutOfMemory ? NKREG_ENOMEM : NKREG_EHIP;
      nk::set_last_error(std::string("launch floor: ") + hipGetErrorString(e));
    }
    return status == NKREG_OK;
  };
  if (ok(hipMalloc(&a, n * sizeof(float2))) && ok(hipMalloc(&b, n * sizeof(float2))) &&
      ok(hipMemsetAsync(a, 0, n * sizeof(float2), st)) && ok(hipMemsetAsync(b, 0, n * sizeof(float2), st)) &&
      ok(hipStreamSynchronize(st)) && ok(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) &&
      ok(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal))) {
    for (int i = 0; i < nodes; ++i) {
      const float2* in = (i % 2) ? b : a;
      float2* out = (i % 2) ? a : b;
      const int k = kind == 3 ? 1 + (i % 2) : kind;
      if (k == 0) hipLaunchKernelGGL(nk::k_floor_empty, dim3(cols), dim3(64), 0, cap, in, out, cols);
      else if (k == 1) hipLaunchKernelGGL(nk::k_floor_row, dim3(rows), dim3(64), 0, cap, in, out, cols);
      else hipLaunchKernelGGL(nk::k_floor_col, dim3(cols), dim3(64), 0, cap, in, out, rows, cols);
    }
    hipError_t ce = hipStreamEndCapture(cap, &graph);
    if (ok(ce) && ok(hipGetLastError()) && ok(hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0)) &&
        ok(hipEventCreate(&e0)) && ok(hipEventCreate(&e1)) && ok(hipGraphLaunch(ex, st)) &&
        ok(hipEventRecord(e0, st))) {
      const int reps = 5;
      for (int r = 0; r < reps && status == NKREG_OK; ++r) ok(hipGraphLaunch(ex, st));
      float ms = 0.f;
      if (ok(hipEventRecord(e1, st)) && ok(hipEventSynchronize(e1)) && ok(hipEventElapsedTime(&ms, e0, e1)))
        *h_us_per_node = 1e3 * (double)ms / ((double)reps * nodes);
    }
  }
  (void)hipStreamSynchronize(st);
  if (ex) (void)hipGraphExecDestroy(ex);
  if (graph) (void)hipGraphDestroy(graph);
  if (cap) (void)hipStreamDestroy(cap);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  return status;
}
