// Unfolded products for the vector-Jacobian products of the core projection
// and the reconstruction (derived from the TTM definition of Section 2.2):
//   out[i][a] (+)= sum_{p,q} A[p][i][q] B[p][a][q]
// i.e. A^(k) (B^(k))^T for two tensors that differ only in mode k (A has n_k
// there, B has c_k), both viewed as (pre, ., post).
//
// The (p, q) range is split into `splits` ranges; block (i, split, chunk)
// forms up to CMAX outputs (columns chunk*CMAX ..) of row i over its range,
// reduces them across the block in a fixed order, writes them as a partial,
// and a second kernel sums the partials in index order (deterministic, no
// atomics).
#include "tk_kernels.hpp"

namespace tk {
namespace {

template <typename TA, typename TB, int CMAX>
__global__ __launch_bounds__(256) void unfold_gemm_kernel(const UnfoldGemm g) {
  __shared__ double red[4 * CMAX];
  const int i = blockIdx.x, split = blockIdx.y, tid = threadIdx.x;
  const int a0 = blockIdx.z * CMAX, cc = min(CMAX, g.c - a0);
  const int64_t R = g.pre * g.post;
  const int64_t per = (R + g.splits - 1) / g.splits;
  const int64_t r0 = split * per, r1 = min(R, r0 + per);
  const TA* A = static_cast<const TA*>(g.A);
  const TB* B = static_cast<const TB*>(g.B);
  double acc[CMAX];
#pragma unroll
  for (int a = 0; a < CMAX; ++a) acc[a] = 0.0;
  for (int64_t r = r0 + tid; r < r1; r += 256) {
    const int64_t p = r / g.post, q = r - p * g.post;
    const double x = to_double(A[(p * g.n + i) * g.post + q]);
    const TB* b = B + (p * g.c + a0) * g.post + q;
#pragma unroll
    for (int a = 0; a < CMAX; ++a)
      if (a < cc) acc[a] = fma(x, to_double(b[(int64_t)a * g.post]), acc[a]);
  }
  // every accumulator reduced across the wave (fixed butterfly order), then
  // the four waves' sums in a fixed order; acc stays in registers (a loop
  // over a with barriers inside would index it dynamically)
#pragma unroll
  for (int a = 0; a < CMAX; ++a) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc[a] += __shfl_xor(acc[a], off);
  }
  if ((tid & 63) == 0) {
#pragma unroll
    for (int a = 0; a < CMAX; ++a) red[(tid >> 6) * CMAX + a] = acc[a];
  }
  __syncthreads();
  double* out = g.partials + ((int64_t)split * g.n + i) * g.c + a0;
  if (tid < cc) out[tid] = (red[tid] + red[CMAX + tid]) + (red[2 * CMAX + tid] + red[3 * CMAX + tid]);
}

// The same product for wide outputs (n >= 64, c >= 16), where re-reading B for
// every row i would dominate: 64 x 64 output tiles, (p, q) in chunks of 16
// staged through LDS (A as [k][i], B as [k][a]), 4 x 4 outputs per thread,
// the (p, q) range split over blocks into the same fixed-order partials.
constexpr int kTK = 16;
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void unfold_tiled_kernel(const UnfoldGemm g) {
  __shared__ double sA[kTK][64 + 1];
  __shared__ double sB[kTK][64 + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.x * 64, a0 = blockIdx.y * 64;
  const int64_t R = g.pre * g.post;
  const int64_t per = (R + g.splits - 1) / g.splits;
  const int64_t r0 = (int64_t)blockIdx.z * per, r1 = min(R, r0 + per);
  const TA* A = static_cast<const TA*>(g.A);
  const TB* B = static_cast<const TB*>(g.B);
  const bool rows = g.post == 1;   // (p, q) = (r, 0): a row of A or B is contiguous
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += kTK) {
    if (rows) {
      // consecutive threads along the row (i or a), four k per thread
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = tid + 256 * u, col = e & 63, kk = e >> 6;
        const int64_t r = rb + kk;
        const bool ok = r < r1;
        sA[kk][col] = (ok && i0 + col < g.n) ? to_double(A[r * g.n + i0 + col]) : 0.0;
        sB[kk][col] = (ok && a0 + col < g.c) ? to_double(B[r * g.c + a0 + col]) : 0.0;
      }
    } else {
      // consecutive threads along q; this thread's k is the same for all four
      const int kk = tid & 15;
      const int64_t r = rb + kk;
      const bool ok = r < r1;
      const int64_t p = ok ? r / g.post : 0, q = ok ? r - p * g.post : 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int col = (tid >> 4) + 16 * u;
        sA[kk][col] = (ok && i0 + col < g.n) ? to_double(A[(p * g.n + i0 + col) * g.post + q]) : 0.0;
        sB[kk][col] = (ok && a0 + col < g.c) ? to_double(B[(p * g.c + a0 + col) * g.post + q]) : 0.0;
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kTK; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = sA[kk][ty + 16 * u];
        bv[u] = sB[kk][tx + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
    }
    __syncthreads();
  }
  double* out = g.partials + (int64_t)blockIdx.z * g.n * g.c;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = i0 + ty + 16 * u;
    if (i >= g.n) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = a0 + tx + 16 * v;
      if (a < g.c) out[(int64_t)i * g.c + a] = acc[u][v];
    }
  }
}

bool tiled(int64_t n, int64_t c) { return n >= 64 && c >= 16; }

template <typename TO>
__global__ void unfold_sum_kernel(const UnfoldGemm g) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nc = (int64_t)g.n * g.c;
  if (e >= nc) return;
  double v = 0.0;
  for (int s = 0; s < g.splits; ++s) v += g.partials[s * nc + e];
  TO* out = static_cast<TO*>(g.out);
  if (g.accumulate) v += to_double(out[e]);
  out[e] = from_double<TO>(v);
}

template <typename TA, typename TB>
hipError_t run(const UnfoldGemm& g, int out_dt, hipStream_t st) {
  const dim3 grid((unsigned)g.n, (unsigned)g.splits);
  if (tiled(g.n, g.c))
    hipLaunchKernelGGL((unfold_tiled_kernel<TA, TB>),
                       dim3((unsigned)ceil_div(g.n, 64), (unsigned)ceil_div(g.c, 64), (unsigned)g.splits),
                       dim3(256), 0, st, g);
  else if (g.c <= 16) hipLaunchKernelGGL((unfold_gemm_kernel<TA, TB, 16>), grid, dim3(256), 0, st, g);
  else if (g.c <= 32) hipLaunchKernelGGL((unfold_gemm_kernel<TA, TB, 32>), grid, dim3(256), 0, st, g);
  else
    hipLaunchKernelGGL((unfold_gemm_kernel<TA, TB, 64>),
                       dim3((unsigned)g.n, (unsigned)g.splits, (unsigned)ceil_div(g.c, 64)), dim3(256),
                       0, st, g);
  const dim3 g2((unsigned)ceil_div((int64_t)g.n * g.c, 256));
  if (out_dt == TK_F64) hipLaunchKernelGGL((unfold_sum_kernel<double>), g2, dim3(256), 0, st, g);
  else hipLaunchKernelGGL((unfold_sum_kernel<float>), g2, dim3(256), 0, st, g);
  return hipGetLastError();
}

template <typename TA>
hipError_t by_b(const UnfoldGemm& g, int b_dt, int out_dt, hipStream_t st) {
  switch (b_dt) {
    case TK_F64: return run<TA, double>(g, out_dt, st);
    case TK_F32: return run<TA, float>(g, out_dt, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace

int32_t unfold_gemm_splits(int64_t n, int64_t c, int64_t pre_post) {
  // the tiled form: about 16K (p, q) per block, and at least about 512 blocks
  // while every split keeps 16 (p, q); non-decreasing in pre_post, so a plan
  // sized with a larger pre_post holds the partials
  if (tiled(n, c)) {
    const int64_t tiles = ceil_div(n, 64) * ceil_div(c, 64);
    int64_t sp = std::max<int64_t>(ceil_div(pre_post, 16384), ceil_div(512, tiles));
    sp = std::min<int64_t>(sp, std::max<int64_t>(1, pre_post / 16));
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(256, sp));
  }
  // enough blocks to cover the chip, each with at least 64K products
  int64_t s = ceil_div(1024, std::max<int64_t>(1, n));
  s = std::min<int64_t>(s, std::max<int64_t>(1, pre_post / 65536));
  return (int32_t)std::max<int64_t>(1, std::min<int64_t>(s, 256));
}

hipError_t launch_unfold_gemm(const UnfoldGemm& g, int a_dt, int b_dt, int out_dt, hipStream_t st) {
  if (g.n == 0 || g.c == 0) return hipSuccess;
  switch (a_dt) {
    case TK_F64: return by_b<double>(g, b_dt, out_dt, st);
    case TK_F32: return by_b<float>(g, b_dt, out_dt, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace tk
