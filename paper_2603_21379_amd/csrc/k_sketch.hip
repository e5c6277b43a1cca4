// Sampled range sketches of every mode (or tree node) in one launch.
//
// Fiber sampling (Section 3.1): column j of the unfolding X^(S) is the fiber
// X[a, :, b] of X viewed as (A, n_S, B) with (a, b) = divmod(j, B); it is read
// directly from the C-ordered tensor, no unfolding is formed.  Each block
// gathers a 64-row x 32-column tile of Y_S = X^(S) E_S into LDS (optionally
// writing it out for the W step) and multiplies it by the matching 32 rows
// of Omega_S in FP64.  Per-chunk partial products go to the workspace and a
// second kernel sums them in a fixed order, so Z_S = Y_S Omega_S is
// deterministic.
#include <type_traits>

#include "tk_kernels.hpp"

namespace tk {
namespace {

template <typename TX, typename TO, typename S>
__global__ __launch_bounds__(256) void sketch_gather_kernel(const S b) {
  __shared__ double sY[kSketchRows][kSketchCols + 1];
  __shared__ double sO[kSketchCols][64 + 1];
  __shared__ int64_t sFib[kSketchCols];   // offset of element 0 of each fiber, or -1
  const int64_t blk = blockIdx.x;
  // the unit's descriptor in registers: read through a reference into a device
  // table, every field would be reloaded after each store of the kernel (the
  // stores may alias the table), thousands of extra loads per block
  const SketchUnit U = wave_uniform(b.get(b.find_block(blk)));
  // fiber chunks vary fastest: blocks running together share rows, which
  // keeps the pages they touch few when fibers are strided (B > 1)
  const int64_t lb = blk - U.block_begin;
  const int64_t rb = lb / U.nchunks;
  const int64_t chunk = lb - rb * U.nchunks;
  const int64_t i0 = rb * kSketchRows, t0 = chunk * kSketchCols;
  const TX* __restrict__ X = static_cast<const TX*>(U.X);
  TX* __restrict__ Y = static_cast<TX*>(U.Y);
  const int tid = threadIdx.x;
  const bool rows_fast = (U.B == 1);  // fibers contiguous: walk along the fiber
  // the block's fibers: column j of the unfolding is X[a, :, b], (a, b) = divmod(j, B)
  if (tid < kSketchCols) {
    const int64_t gt = t0 + tid;
    int64_t off = -1;
    if (gt < U.s) {
      const int64_t j = U.idx ? U.idx[gt] : gt;
      if (j >= 0 && j < U.A * U.B) {  // a column index outside the unfolding reads nothing
        const int64_t a = j / U.B;
        off = a * U.n * U.B + (j - a * U.B);
      } else {
        off = -2;
      }
    }
    sFib[tid] = off;
  }
  __syncthreads();
  // every load of the tile first, then the stores
  constexpr int kPer = kSketchRows * kSketchCols / 256;
  TX xv[kPer];
  bool ok[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = tid + 256 * q;
    int i, t;
    if (rows_fast) { i = e % kSketchRows; t = e / kSketchRows; }
    else { t = e % kSketchCols; i = e / kSketchCols; }
    const int64_t gi = i0 + i, f = sFib[t];
    ok[q] = gi < U.n && f >= 0;
    xv[q] = ok[q] ? X[f + gi * U.B] : TX{};
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = tid + 256 * q;
    int i, t;
    if (rows_fast) { i = e % kSketchRows; t = e / kSketchRows; }
    else { t = e % kSketchCols; i = e / kSketchCols; }
    const int64_t gi = i0 + i, f = sFib[t];
    double v = 0.0;
    if (ok[q]) {
      v = to_double(xv[q]);
      if (Y) Y[gi * U.s + t0 + t] = xv[q];
    } else if (gi < U.n && f == -2) {
      v = __builtin_nan("");
    }
    sY[i][t] = v;
  }
  const TO* Om = static_cast<const TO*>(U.omega);
  const int row = tid >> 2, lane4 = tid & 3;
  const int64_t gi = i0 + row;
  // thread (row, lane4) forms columns lane4 + 4 q of the 64-column chunk; only
  // the accumulators the sketch width needs are formed (QN of 16), and rows
  // past n skip the products (a wave of such rows skips them entirely)
  auto tile = [&](int e0, auto qn) {
    constexpr int QN = decltype(qn)::value;
    double acc[QN];
#pragma unroll
    for (int q = 0; q < QN; ++q) acc[q] = 0.0;
    if (gi < U.n) {
      // (unrolled by two only: a full unroll hoists every load of the 32
      // steps and spills to scratch)
#pragma unroll 2
      for (int t = 0; t < kSketchCols; ++t) {
        const double y = sY[row][t];
#pragma unroll
        for (int q = 0; q < QN; ++q) acc[q] = fma(y, sO[t][lane4 + 4 * q], acc[q]);
      }
#pragma unroll
      for (int q = 0; q < QN; ++q) {
        const int jj = e0 + lane4 + 4 * q;
        if (jj < U.ell) U.partial[(chunk * U.n + gi) * U.ell + jj] = acc[q];
      }
    }
  };
  for (int e0 = 0; e0 < U.ell; e0 += 64) {
    __syncthreads();
    for (int e = tid; e < kSketchCols * 64; e += blockDim.x) {
      const int t = e >> 6, jj = e & 63;
      const int64_t gt = t0 + t;
      sO[t][jj] = (gt < U.s && e0 + jj < U.ell) ? to_double(Om[gt * U.ell + e0 + jj]) : 0.0;
    }
    __syncthreads();
    const int width = U.ell - e0 < 64 ? U.ell - e0 : 64;
    if (width <= 16) tile(e0, std::integral_constant<int, 4>{});
    else if (width <= 32) tile(e0, std::integral_constant<int, 8>{});
    else if (width <= 48) tile(e0, std::integral_constant<int, 12>{});
    else tile(e0, std::integral_constant<int, 16>{});
  }
}

template <typename S>
__global__ __launch_bounds__(256) void sketch_reduce_kernel(const S b) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= b.total_out) return;
  const SketchUnit U = b.get(b.find_out(g));   // by value: fields loaded once
  const int64_t e = g - U.out_begin;
  const int64_t plane = U.n * U.ell;
  double acc = 0.0;
  for (int c = 0; c < U.nchunks; ++c) acc += U.partial[c * plane + e];
  U.Z[e] = acc;
}

template <typename TX, typename TO, typename S>
hipError_t run(const S& b, hipStream_t st) {
  if (b.total_blocks > 0)
    hipLaunchKernelGGL((sketch_gather_kernel<TX, TO, S>), dim3((unsigned)b.total_blocks), dim3(256), 0,
                       st, b);
  if (b.total_out > 0)
    hipLaunchKernelGGL(sketch_reduce_kernel<S>, dim3((unsigned)ceil_div(b.total_out, 256)), dim3(256),
                       0, st, b);
  return hipGetLastError();
}

template <typename S>
hipError_t dispatch(int dtype, const S& b, hipStream_t st) {
  switch (dtype) {
    case TK_F64: return run<double, double>(b, st);
    case TK_F32: return run<float, float>(b, st);
    case TK_BF16: return run<bf16, float>(b, st);
    case TK_F16: return run<f16, float>(b, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_sketch(int dtype, const SketchBatch& b, hipStream_t st) { return dispatch(dtype, b, st); }

hipError_t launch_sketch_list(int dtype, const SketchList& b, hipStream_t st) { return dispatch(dtype, b, st); }

}  // namespace tk
