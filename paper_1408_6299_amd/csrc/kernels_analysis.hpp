// Kernels of the Hessian analysis (dense assembly and Lanczos): unit vectors,
// a deterministic start vector, and the block inner products and updates of
// the full reorthogonalisation.
#pragma once

#include "common.hpp"

namespace nk {

// y = e_j (unit vector), for assembling the Hessian column by column.
template <typename R>
__global__ void k_unit(long long cnt, long long j, R* __restrict__ y) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = i == j ? R(1) : R(0);
}

// Y[i] = e_{j0 + i} for i < G (G vectors of length cnt, one after another); a
// column index at or beyond cnt gives a zero vector.
static __global__ void k_unit_block(long long cnt, int G, long long j0, double* __restrict__ Y) {
  const long long tot = cnt * G;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot;
       t += (long long)gridDim.x * blockDim.x)
    Y[t] = (t % cnt) == j0 + t / cnt ? 1.0 : 0.0;
}

// Deterministic start vector in [-1, 1] (a fixed integer hash of the index).
static __global__ void k_hash_fill(long long cnt, double* __restrict__ y) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x) {
    unsigned long long x = (unsigned long long)i * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    x ^= x >> 31;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 29;
    y[i] = (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

// Partial inner products <Q_i, w> of the k vectors Q_0..Q_{k-1} (stride nv):
// workgroup (i, p) sums the elements p * 256 + t (mod P * 256) of vector i
// into part[i * P + p], P = gridDim.y. Many workgroups per vector keep the
// whole GPU streaming where one per vector would leave it mostly idle.
constexpr int kDotParts = 64;
static __global__ __launch_bounds__(256) void k_multidot_part(const double* __restrict__ Q, long long nv,
                                                       const double* __restrict__ w, double* __restrict__ part) {
  const double* q = Q + (long long)blockIdx.x * nv;
  const long long stride = (long long)gridDim.y * blockDim.x;
  double sum = 0.0;
  for (long long t = (long long)blockIdx.y * blockDim.x + threadIdx.x; t < nv; t += stride) sum += q[t] * w[t];
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_down(sum, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) part[(long long)blockIdx.x * gridDim.y + blockIdx.y] = red[0] + red[1] + red[2] + red[3];
}
// c[i] = sum of vector i's P partials, in order.
static __global__ void k_multidot_sum(const double* __restrict__ part, int P, int k, double* __restrict__ c) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  double s = 0.0;
  for (int p = 0; p < P; ++p) s += part[(long long)i * P + p];
  c[i] = s;
}

// w -= sum_i c[i] Q_i over the k vectors.
static __global__ void k_multi_axpy(const double* __restrict__ Q, int k, long long nv, const double* __restrict__ c,
                             double* __restrict__ w) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < nv;
       t += (long long)gridDim.x * blockDim.x) {
    double acc = w[t];
    for (int i = 0; i < k; ++i) acc -= c[i] * Q[(long long)i * nv + t];
    w[t] = acc;
  }
}

}  // namespace nk
