// Generic mode products (the TTM of Section 2.2) used by the core projection,
// the reconstruction and their VJPs for any order, sizes and dtypes:
//
//   out[a][p][b] = sum_q in[a][q][b] * M[p][q]
//
// over a tensor viewed as (A, Q, B).  A contraction with F^T takes
// M[p][q] = F[q][p]; an expansion with F takes M[p][q] = F[p][q].  All
// arithmetic is FP64 (FP64 and non-packed FP32 FMA have the same rate on
// CDNA4), with the output rounded to its storage type.
//
// Two layouts: B == 1 (the contracted mode is the contiguous one) stages a
// 64-row x 64-column tile of `in` through LDS so the loads are coalesced;
// B > 1 maps consecutive threads to consecutive b so every load of a fixed q
// is coalesced.  The last expansion of a reconstruction is fused with the
// squared residual against the reference tensor (FP64 partial sums per
// block, then a fixed-order final sum).
#include <algorithm>

#include "tk_kernels.hpp"

namespace tk {
namespace {

template <typename T> __device__ __forceinline__ double ld(const void* p, int64_t i) {
  return to_double(static_cast<const T*>(p)[i]);
}

// M staged as a zero-padded FP64 table Mt[q][p] (ld = padded P): every read
// of it in the inner loops is a fixed, contiguous, wave-uniform run, which
// the compiler turns into scalar loads (no LDS traffic, no bounds checks).
__global__ void stage_factor_kernel(const void* M, int m_dt, int64_t rs, int64_t cs, int P,
                                    int64_t Q, int ld, double* Mt) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= Q * ld) return;
  const int64_t q = g / ld;
  const int p = (int)(g - q * ld);
  double v = 0.0;
  if (p < P) {
    const int64_t i = p * rs + q * cs;
    v = m_dt == TK_F64 ? static_cast<const double*>(M)[i] : (double)static_cast<const float*>(M)[i];
  }
  Mt[g] = v;
}

template <typename TIn, typename TOut, int PMAX>
__global__ __launch_bounds__(256) void mode_rows_kernel(const ModeProduct mp, int ld) {
  // B == 1: out[a][p] = sum_q in[a][q] M[p][q]; 64 rows per block, a
  // 64 x 64 tile of `in` staged through LDS (coalesced), the next tile's
  // loads in flight while this one is multiplied; 4 p-groups of PMAX / 4
  // consecutive p, one per wave, each reading its entries of the staged
  // factor table with wave-uniform (scalar) loads
  __shared__ double sX[64][65];
  const int tid = threadIdx.x;
  const int row = tid & 63;
  const int pg = __builtin_amdgcn_readfirstlane(tid >> 6);  // one p-group per wave
  constexpr int PK = PMAX / 4;
  constexpr int kXE = 64 * 64 / 256;
  const int64_t a0 = (int64_t)blockIdx.x * 64;
  const int p0 = blockIdx.y * PMAX;
  const int rows = (int)min<int64_t>(64, mp.A - a0);
  const TIn* in = static_cast<const TIn*>(mp.in);
  const double* __restrict__ Mt = mp.Mt;
  double xr[kXE];
  // the tile at q0 (rows past the matrix and q past Q read as zero; a q0
  // past Q loads nothing that is used)
  auto load = [&](int64_t q0) {
    const int64_t qn = min<int64_t>(64, mp.Q - q0);
#pragma unroll
    for (int u = 0; u < kXE; ++u) {
      const int e = tid + 256 * u, rr = e >> 6, qq = e & 63;
      xr[u] = (rr < rows && qq < qn) ? to_double(in[(a0 + rr) * mp.Q + q0 + qq]) : 0.0;
    }
  };
  double acc[PK];
#pragma unroll
  for (int k = 0; k < PK; ++k) acc[k] = 0.0;
  load(0);
  for (int64_t q0 = 0; q0 < mp.Q; q0 += 64) {
    __syncthreads();   // the previous tile's products are done
#pragma unroll
    for (int u = 0; u < kXE; ++u) {
      const int e = tid + 256 * u;
      sX[e >> 6][e & 63] = xr[u];
    }
    __syncthreads();
    load(q0 + 64);
    const int qn = (int)min<int64_t>(64, mp.Q - q0);
#pragma unroll 4
    for (int qq = 0; qq < qn; ++qq) {
      const double x = sX[row][qq];
      const double* mq = Mt + (q0 + qq) * ld + p0 + pg * PK;   // this wave's PK contiguous entries
#pragma unroll
      for (int k = 0; k < PK; ++k) acc[k] = fma(x, mq[k], acc[k]);
    }
  }
  if (row < rows) {
    TOut* out = static_cast<TOut*>(mp.out);
#pragma unroll
    for (int k = 0; k < PK; ++k) {
      const int p = p0 + pg * PK + k;
      if (p < mp.P) {
        const int64_t o = (a0 + row) * mp.P + p;
        double v = acc[k];
        if (mp.accumulate) v += to_double(out[o]);
        out[o] = from_double<TOut>(v);
      }
    }
  }
}

template <typename TIn, typename TOut, int PMAX, int NB>
__global__ __launch_bounds__(256) void mode_strided_kernel(const ModeProduct mp, int ld) {
  // out[a][p][b] = sum_q in[a][q][b] M[p][q]; NB (a, b) points per thread,
  // 256 apart, so each load instruction stays coalesced; M comes from the
  // staged table with scalar loads.  With gridDim.z > 1, block z sums the
  // z-th range of q into its own partial output.
  const int tid = threadIdx.x;
  const int64_t AB = mp.A * mp.B;
  const int p0 = blockIdx.y * PMAX;
  const TIn* __restrict__ in = static_cast<const TIn*>(mp.in);
  const double* __restrict__ Mt = mp.Mt;
  int64_t base[NB];
  bool live[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int64_t g = ((int64_t)blockIdx.x * NB + u) * 256 + tid;
    live[u] = g < AB;
    const int64_t a = live[u] ? g / mp.B : 0;
    const int64_t bb = live[u] ? g - a * mp.B : 0;
    base[u] = a * mp.Q * mp.B + bb;
  }
  double acc[NB][PMAX];
#pragma unroll
  for (int u = 0; u < NB; ++u)
#pragma unroll
    for (int k = 0; k < PMAX; ++k) acc[u][k] = 0.0;
  const int64_t qper = (mp.Q + gridDim.z - 1) / gridDim.z;
  const int64_t qb = (int64_t)blockIdx.z * qper, qe = min(mp.Q, qb + qper);
  int64_t q = qb;
  for (; q + 4 <= qe; q += 4) {
    double x[4][NB];
#pragma unroll
    for (int w = 0; w < 4; ++w)
#pragma unroll
      for (int u = 0; u < NB; ++u)
        x[w][u] = live[u] ? to_double(in[base[u] + (q + w) * mp.B]) : 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const double* mq = Mt + (q + w) * ld + p0;
#pragma unroll
      for (int k = 0; k < PMAX; ++k) {
        const double m = mq[k];
#pragma unroll
        for (int u = 0; u < NB; ++u) acc[u][k] = fma(x[w][u], m, acc[u][k]);
      }
    }
  }
  for (; q < qe; ++q) {
    double x[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) x[u] = live[u] ? to_double(in[base[u] + q * mp.B]) : 0.0;
    const double* mq = Mt + q * ld + p0;
#pragma unroll
    for (int k = 0; k < PMAX; ++k) {
      const double m = mq[k];
#pragma unroll
      for (int u = 0; u < NB; ++u) acc[u][k] = fma(x[u], m, acc[u][k]);
    }
  }
  TOut* out = static_cast<TOut*>(mp.out);
  const int pn = min(PMAX, mp.P - p0);
  const bool split = gridDim.z > 1;
  double* part = split ? mp.part + (int64_t)blockIdx.z * mp.A * mp.P * mp.B : nullptr;
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    if (!live[u]) continue;
    const int64_t g = ((int64_t)blockIdx.x * NB + u) * 256 + tid;
    const int64_t a = g / mp.B, bb = g - a * mp.B;
#pragma unroll
    for (int k = 0; k < PMAX; ++k) {
      if (k < pn) {
        const int64_t o = (a * mp.P + p0 + k) * mp.B + bb;
        if (split) {
          part[o] = acc[u][k];
        } else {
          double v = acc[u][k];
          if (mp.accumulate) v += to_double(out[o]);
          out[o] = from_double<TOut>(v);
        }
      }
    }
  }
}

// out (+)= the sum of the q-range partials, in split order
template <typename TOut>
__global__ __launch_bounds__(256) void mode_split_sum_kernel(const ModeProduct mp, int splits) {
  const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = mp.A * mp.P * mp.B;
  if (o >= n) return;
  double v = 0.0;
  for (int z = 0; z < splits; ++z) v += mp.part[(int64_t)z * n + o];
  TOut* out = static_cast<TOut*>(mp.out);
  if (mp.accumulate) v += to_double(out[o]);
  out[o] = from_double<TOut>(v);
}

int width_of(int P) { return P <= 16 ? 16 : P <= 32 ? 32 : 64; }

template <typename TIn, typename TOut>
hipError_t mode_product(const ModeProduct& mp, int m_dt, hipStream_t st) {
  if (mp.A == 0 || mp.B == 0 || mp.P < 1) return hipSuccess;
  const int width = width_of(mp.P);
  const unsigned pchunks = (unsigned)ceil_div(mp.P, width);
  const int ld = (int)pchunks * width;
  hipLaunchKernelGGL(stage_factor_kernel, dim3((unsigned)ceil_div(mp.Q * ld, 256)), dim3(256), 0,
                     st, mp.M, m_dt, (int64_t)mp.rs, (int64_t)mp.cs, mp.P, mp.Q, ld, mp.Mt);
  if (mp.B == 1) {
    // up to 192 columns in one block, so each row of `in` is read once (for
    // 64 < P <= 192 the table's ld, a multiple of 64, is exactly 128 or 192);
    // wider products keep 64-column blocks, whose reads stay inside ld
    const int wr = mp.P <= 64 ? width : mp.P <= 128 ? 128 : mp.P <= 192 ? 192 : 64;
    const dim3 grid((unsigned)ceil_div(mp.A, 64), (unsigned)ceil_div(mp.P, wr));
    if (wr == 16)
      hipLaunchKernelGGL((mode_rows_kernel<TIn, TOut, 16>), grid, dim3(256), 0, st, mp, ld);
    else if (wr == 32)
      hipLaunchKernelGGL((mode_rows_kernel<TIn, TOut, 32>), grid, dim3(256), 0, st, mp, ld);
    else if (wr == 64)
      hipLaunchKernelGGL((mode_rows_kernel<TIn, TOut, 64>), grid, dim3(256), 0, st, mp, ld);
    else if (wr == 128)
      hipLaunchKernelGGL((mode_rows_kernel<TIn, TOut, 128>), grid, dim3(256), 0, st, mp, ld);
    else
      hipLaunchKernelGGL((mode_rows_kernel<TIn, TOut, 192>), grid, dim3(256), 0, st, mp, ld);
  } else {
    // several points per thread when there are enough of them to keep every
    // CU busy (64 accumulators per thread at most)
    const bool wide = mp.A * mp.B >= (int64_t)256 * 4 * 1024;
    const int nb = !wide ? 1 : width == 16 ? 4 : width == 32 ? 2 : 1;
    // few output points and a long contraction: split q so that about 2048
    // blocks run (when the caller gave room for the partials)
    const int64_t pts_blocks = ceil_div(mp.A * mp.B, 256 * nb) * pchunks;
    int splits = 1;
    if (mp.part && mp.qsplit_max > 1 && pts_blocks < 1024)
      splits = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)mp.qsplit_max, ceil_div(2048, pts_blocks),
                                                            mp.Q / 256}));
    const dim3 grid((unsigned)ceil_div(mp.A * mp.B, 256 * nb), pchunks, (unsigned)splits);
    if (width == 16) {
      if (wide) hipLaunchKernelGGL((mode_strided_kernel<TIn, TOut, 16, 4>), grid, dim3(256), 0, st, mp, ld);
      else hipLaunchKernelGGL((mode_strided_kernel<TIn, TOut, 16, 1>), grid, dim3(256), 0, st, mp, ld);
    } else if (width == 32) {
      if (wide) hipLaunchKernelGGL((mode_strided_kernel<TIn, TOut, 32, 2>), grid, dim3(256), 0, st, mp, ld);
      else hipLaunchKernelGGL((mode_strided_kernel<TIn, TOut, 32, 1>), grid, dim3(256), 0, st, mp, ld);
    } else {
      hipLaunchKernelGGL((mode_strided_kernel<TIn, TOut, 64, 1>), grid, dim3(256), 0, st, mp, ld);
    }
    if (splits > 1)
      hipLaunchKernelGGL((mode_split_sum_kernel<TOut>), dim3((unsigned)ceil_div(mp.A * mp.P * mp.B, 256)),
                         dim3(256), 0, st, mp, splits);
  }
  return hipGetLastError();
}

template <typename TIn>
hipError_t by_out(const ModeProduct& mp, int out_dt, int m_dt, hipStream_t st) {
  return out_dt == TK_F64 ? mode_product<TIn, double>(mp, m_dt, st)
                          : mode_product<TIn, float>(mp, m_dt, st);
}

// ------------------------------------------------------------------ fused residual
constexpr int kResidBlocks = 2048;

template <typename TX, typename TF>
__global__ __launch_bounds__(256) void expand_residual_kernel(const ExpandResidual e) {
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  const int64_t total = e.A * e.n;
  const TF* F = static_cast<const TF*>(e.F);
  const TX* X = static_cast<const TX*>(e.X);
  TF* Xh = static_cast<TF*>(e.Xhat);
  TF* D = static_cast<TF*>(e.D);
  const double ds = e.smul * (e.scale ? *e.scale : 1.0);
  double r2 = 0.0, x2 = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * 256 + tid; g < total; g += (int64_t)gridDim.x * 256) {
    const int64_t a = g / e.n, i = g - a * e.n;
    const double* t = e.T + a * e.c;
    const TF* f = F + i * e.c;
    double v = 0.0;
    for (int j = 0; j < e.c; ++j) v = fma(t[j], to_double(f[j]), v);
    if (Xh) Xh[g] = from_double<TF>(e.accumulate ? v + to_double(Xh[g]) : v);
    if (X) {
      const double x = to_double(X[g]);
      const double d = x - v;
      r2 = fma(d, d, r2);
      x2 = fma(x, x, x2);
      if (D) D[g] = from_double<TF>(ds * d);
    }
  }
  if (!e.partials) return;
  red[0][tid] = r2;
  red[1][tid] = x2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      red[0][tid] += red[0][tid + s];
      red[1][tid] += red[1][tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    e.partials[2 * blockIdx.x] = red[0][0];
    e.partials[2 * blockIdx.x + 1] = red[1][0];
  }
}

// The same for a short last mode (n <= 256): thread (r, i) of a block owns
// column i of rows r, r + RP, ... (RP = 256 / n rows per step), so F[i][:]
// stays in registers, the lanes of a wave share one or two rows of T (cached
// loads) and no element index is divided.  Same partials as above.
template <typename TX, typename TF, int CB>
__global__ __launch_bounds__(256) void expand_residual_rows_kernel(const ExpandResidual e) {
  __shared__ double red[2][4];
  const int tid = threadIdx.x;
  const int n = (int)e.n, RP = 256 / n;
  const int r = tid / n, i = tid - r * n;
  const bool on = r < RP;
  const TF* F = static_cast<const TF*>(e.F);
  const TX* X = static_cast<const TX*>(e.X);
  TF* Xh = static_cast<TF*>(e.Xhat);
  TF* D = static_cast<TF*>(e.D);
  const double ds = e.smul * (e.scale ? *e.scale : 1.0);
  double f[CB];
#pragma unroll
  for (int k = 0; k < CB; ++k) f[k] = (on && k < e.c) ? to_double(F[(int64_t)i * e.c + k]) : 0.0;
  double r2 = 0.0, x2 = 0.0;
  if (on) {
    for (int64_t a = (int64_t)blockIdx.x * RP + r; a < e.A; a += (int64_t)gridDim.x * RP) {
      const double* t = e.T + a * e.c;
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < CB; ++k) v = fma(k < e.c ? t[k] : 0.0, f[k], v);
      const int64_t g = a * n + i;
      if (Xh) Xh[g] = from_double<TF>(e.accumulate ? v + to_double(Xh[g]) : v);
      if (X) {
        const double x = to_double(X[g]);
        const double d = x - v;
        r2 = fma(d, d, r2);
        x2 = fma(x, x, x2);
        if (D) D[g] = from_double<TF>(ds * d);
      }
    }
  }
  if (!e.partials) return;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    r2 += __shfl_xor(r2, off);
    x2 += __shfl_xor(x2, off);
  }
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = r2;
    red[1][tid >> 6] = x2;
  }
  __syncthreads();
  if (tid == 0) {
    e.partials[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    e.partials[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

__global__ __launch_bounds__(256) void final_sum_kernel(const double* partials, int nblocks,
                                                        double* out) {
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int i = tid; i < nblocks; i += 256) {
    a += partials[2 * i];
    b += partials[2 * i + 1];
  }
  red[0][tid] = a;
  red[1][tid] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      red[0][tid] += red[0][tid + s];
      red[1][tid] += red[1][tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = red[0][0];
    out[1] = red[1][0];
  }
}

template <typename TX, typename TF>
hipError_t expand_residual(const ExpandResidual& e, hipStream_t st) {
  const int nb = (int)expand_residual_blocks(e.A * e.n);
  if (e.n <= 256 && e.c <= 64) {
    if (e.c <= 16)
      hipLaunchKernelGGL((expand_residual_rows_kernel<TX, TF, 16>), dim3(nb), dim3(256), 0, st, e);
    else if (e.c <= 32)
      hipLaunchKernelGGL((expand_residual_rows_kernel<TX, TF, 32>), dim3(nb), dim3(256), 0, st, e);
    else
      hipLaunchKernelGGL((expand_residual_rows_kernel<TX, TF, 64>), dim3(nb), dim3(256), 0, st, e);
  } else {
    hipLaunchKernelGGL((expand_residual_kernel<TX, TF>), dim3(nb), dim3(256), 0, st, e);
  }
  if (e.partials && e.resid2)
    hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(256), 0, st, e.partials, nb, e.resid2);
  return hipGetLastError();
}

template <typename TF>
hipError_t er_by_x(const ExpandResidual& e, int x_dt, hipStream_t st) {
  switch (x_dt) {
    case TK_F64: return expand_residual<double, TF>(e, st);
    case TK_F32: return expand_residual<float, TF>(e, st);
    case TK_BF16: return expand_residual<bf16, TF>(e, st);
    case TK_F16: return expand_residual<f16, TF>(e, st);
  }
  return hipErrorInvalidValue;
}

template <typename TO>
__global__ void convert_kernel(const double* in, TO* out, int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) out[g] = from_double<TO>(in[g]);
}

template <typename TI>
__global__ void to_f64_kernel(const TI* in, double* out, int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) out[g] = to_double(in[g]);
}

}  // namespace

int64_t expand_residual_blocks(int64_t total) {
  return std::max<int64_t>(1, std::min<int64_t>(kResidBlocks, ceil_div(total, 256)));
}

int64_t mode_product_scratch(int64_t P, int64_t Q) {
  const int w = width_of((int)std::min<int64_t>(P, 1 << 20));
  return ceil_div(P, w) * w * Q;
}

hipError_t launch_mode_product(const ModeProduct& mp, int in_dt, int out_dt, int m_dt,
                               hipStream_t st) {
  if (!mp.Mt) return hipErrorInvalidValue;
  switch (in_dt) {
    case TK_F64: return by_out<double>(mp, out_dt, m_dt, st);
    case TK_F32: return by_out<float>(mp, out_dt, m_dt, st);
    case TK_BF16: return by_out<bf16>(mp, out_dt, m_dt, st);
    case TK_F16: return by_out<f16>(mp, out_dt, m_dt, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_expand_residual(const ExpandResidual& e, int x_dt, int f_dt, hipStream_t st) {
  if (e.A * e.n == 0) return hipSuccess;
  return f_dt == TK_F64 ? er_by_x<double>(e, x_dt, st) : er_by_x<float>(e, x_dt, st);
}

hipError_t launch_convert(const double* in, void* out, int out_dt, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const dim3 grid((unsigned)ceil_div(n, 256));
  if (out_dt == TK_F64)
    hipLaunchKernelGGL((convert_kernel<double>), grid, dim3(256), 0, st, in,
                       static_cast<double*>(out), n);
  else
    hipLaunchKernelGGL((convert_kernel<float>), grid, dim3(256), 0, st, in,
                       static_cast<float*>(out), n);
  return hipGetLastError();
}

hipError_t launch_to_f64(const void* in, int in_dt, double* out, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const dim3 grid((unsigned)ceil_div(n, 256));
  switch (in_dt) {
    case TK_F64: hipLaunchKernelGGL((to_f64_kernel<double>), grid, dim3(256), 0, st, static_cast<const double*>(in), out, n); break;
    case TK_F32: hipLaunchKernelGGL((to_f64_kernel<float>), grid, dim3(256), 0, st, static_cast<const float*>(in), out, n); break;
    case TK_BF16: hipLaunchKernelGGL((to_f64_kernel<bf16>), grid, dim3(256), 0, st, static_cast<const bf16*>(in), out, n); break;
    case TK_F16: hipLaunchKernelGGL((to_f64_kernel<f16>), grid, dim3(256), 0, st, static_cast<const f16*>(in), out, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tk
