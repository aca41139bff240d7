// Persistent form of a small problem's transport sweeps: one workgroup runs every
// launch of an item's recorded sequence (row stages, column passes, fills and
// conversions) one after another, with a workgroup barrier where the launch path
// has a kernel boundary. Its wavefronts share each launch's row or column groups
// and run the same device code on the same values as the launches, so the results
// are the same bits. The items of a batch group run as concurrent workgroups.
#pragma once

#include "spectral.hpp"

namespace nk {

enum SmallOpKind { SOP_ROW = 0, SOP_COL = 1, SOP_FILL = 2, SOP_CONV = 3 };

// One recorded launch as the persistent kernel runs it. Per-item arguments are the
// launch's table entries: item i's entry at tab + off + i * esize.
struct SmallOp {
  int kind;        // SmallOpKind
  int sub;         // ROW: stage kind; COL: column mode
  long long off;   // table offset of the first item's entry
  int esize;       // bytes per item entry
  int gx, gy, gz;  // ROW: row groups, fields; COL: column groups, outer slices, fields
  ColArgs ca;      // COL
  double scale;    // COL: multiplier scale; FILL: value
  int twb;         // COL: twiddle stride
  long long cnt;   // FILL, CONV: elements
};

// Wavefronts per workgroup: eight in FP32; four in FP64, whose row stages need more than
// the 256 registers per lane that eight wavefronts per CU leave (more would spill).
template <typename R>
struct SmallWaves {
  static constexpr int W = sizeof(R) == 8 ? 4 : 8;
  static constexpr int NT = 64 * W;
};

// Per-wavefront LDS scratch: the largest row-stage or column-pass need of the grid.
template <typename R, int N1, int L>
struct SmallShape {
  static constexpr int E = row_e<L>();
  static constexpr int ROW = RowLds<R, L, E, ST_ADJ1, 2>::SIZE > RowLds<R, L, E, ST_INC1, 2>::SIZE
                                 ? RowLds<R, L, E, ST_ADJ1, 2>::SIZE
                                 : RowLds<R, L, E, ST_INC1, 2>::SIZE;
  static constexpr int COL = ColShape<N1, 8>::SPW * padded_e<8>(N1);
  static constexpr int SLOT = ROW > COL ? ROW : COL;
};

template <typename R, int L, int KIND, bool NC1>
__device__ __forceinline__ void small_rows(const SmallOp& op, const StageArgs<R>& a, const cplx<R>* tw, int lmax,
                                           cplx<R>* lds, int wave, int lane) {
  for (int fy = 0; fy < op.gy; ++fy)
    for (int g = wave; g < op.gx; g += SmallWaves<R>::W)
      row_body_at<R, L, row_e<L>(), KIND, 2, NC1>(a, tw, lmax, g, fy, lds, lane);
}

// Bytes of one launch's staged table entry (the largest is StageArgs<double>).
constexpr int kSmallArgBytes = 1024;

template <typename R, int N1, int L, bool NC1>
__global__ __launch_bounds__(SmallWaves<R>::NT) void k_small(const SmallOp* __restrict__ prog, int nops,
                                                         const unsigned char* __restrict__ tab,
                                                         const cplx<R>* __restrict__ tw, int lmax) {
  static_assert(sizeof(StageArgs<R>) <= kSmallArgBytes, "staged entry");
  using SS = SmallShape<R, N1, L>;
  constexpr int W = SmallWaves<R>::W, NT = SmallWaves<R>::NT;
  __shared__ cplx<R> lds[W * SS::SLOT];
  // The current launch's table entry and the next one's: the first wavefront copies the
  // next entry while the current launch runs, so no launch waits for its arguments.
  __shared__ __align__(16) unsigned long long args[2][kSmallArgBytes / 8];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  cplx<R>* my = lds + wave * SS::SLOT;
  const long long item = blockIdx.x;
  auto entry_word = [&](const SmallOp& op, int w) -> unsigned long long {
    const unsigned long long* e =
        reinterpret_cast<const unsigned long long*>(tab + op.off + item * op.esize);
    return w * 8 < op.esize ? e[w] : 0ull;
  };
  if (wave == 0) {
    args[0][lane] = entry_word(prog[0], lane);
    args[0][lane + 64] = entry_word(prog[0], lane + 64);
  }
  __syncthreads();
  for (int o = 0; o < nops; ++o) {
    const SmallOp& op = prog[o];   // uniform: read in place by scalar loads
    const bool more = o + 1 < nops;
    unsigned long long w0 = 0, w1 = 0;
    if (wave == 0 && more) {
      w0 = entry_word(prog[o + 1], lane);
      w1 = entry_word(prog[o + 1], lane + 64);
    }
    const unsigned char* e = reinterpret_cast<const unsigned char*>(args[o & 1]);
    if (op.kind == SOP_ROW) {
      const StageArgs<R>& a = *reinterpret_cast<const StageArgs<R>*>(e);
      if (!a.inactive) switch (op.sub) {
        case ST_INC1: small_rows<R, L, ST_INC1, NC1>(op, a, tw, lmax, my, wave, lane); break;
        case ST_INC2: small_rows<R, L, ST_INC2, NC1>(op, a, tw, lmax, my, wave, lane); break;
        case ST_ADJINIT: small_rows<R, L, ST_ADJINIT, NC1>(op, a, tw, lmax, my, wave, lane); break;
        case ST_ADJ1: small_rows<R, L, ST_ADJ1, NC1>(op, a, tw, lmax, my, wave, lane); break;
        default: small_rows<R, L, ST_ADJ2, NC1>(op, a, tw, lmax, my, wave, lane); break;
      }
    } else if (op.kind == SOP_COL) {
      const ColPtrs<R> p = *reinterpret_cast<const ColPtrs<R>*>(e);
      if (!p.inactive)
      for (int fz = 0; fz < op.gz; ++fz)
        for (int by = 0; by < op.gy; ++by)
          for (int bx = wave; bx < op.gx; bx += W)
            col_w_at<R, N1, 8, COL_DERIV>(p.in, p.add, p.out, op.ca, (R)op.scale, tw, op.twb, fz, bx, by, my, lane);
    } else if (op.kind == SOP_FILL) {
      R* y = *reinterpret_cast<R* const*>(e);
      const R v = (R)op.scale;
      for (long long i = threadIdx.x; i < op.cnt; i += NT) y[i] = v;
    } else {
      const ConvPtrs<double, R> p = *reinterpret_cast<const ConvPtrs<double, R>*>(e);
      for (long long i = threadIdx.x; i < op.cnt; i += NT) p.y[i] = (R)p.x[i];
    }
    if (wave == 0 && more) {
      args[(o + 1) & 1][lane] = w0;
      args[(o + 1) & 1][lane + 64] = w1;
    }
    __syncthreads();
  }
}

// Square 2D grids up to this size run their sweeps in the persistent kernel.
constexpr int kSmallMaxN = 64;

// Launches k_small for `items` items over a program at prog (device) with nops
// launches; defined for N1 = L in {8, 16, 32, 64}. Returns false if no instance fits.
bool launch_small(bool f64, int n1, int l, bool nc1, int items, const SmallOp* prog, int nops,
                  const unsigned char* tab, const void* tw, int lmax, hipStream_t st);

}  // namespace nk
