// Full tensor of an H-Tucker format and its residual (Section 4: root
// relation and nestedness of the bases).
//
// The root relation gives X^(Rl) = U_Rl B_R U_Rr^T for the nested bases of the
// root's two children, so with T = U_Rl B_R (n_l x r_r, small) every entry is
//     xhat[a][b] = sum_k T[a][k] U_Rr[b][k],
// a rank-r_r expansion of the n_l x n_r matricisation.  ht_expand_kernel
// streams it once: a workgroup owns a tile of columns b and a range of rows a;
// each lane keeps U_Rr[b][:] of its columns in registers, each row's T[a][:]
// is wave-uniform (scalar loads), so an entry costs r_r FP64 FMAs (r_r padded
// to 8, 12, 16, 32 or 64) and the only HBM traffic is the reference tensor
// (and the output, if written).  The next group of rows is loaded while the
// current one is multiplied.
// The residual ||X - Xhat||^2 and ||X||^2 are accumulated in FP64 per lane,
// reduced per workgroup and summed in a fixed order.
#include <type_traits>

#include "tk_kernels.hpp"

namespace tk {
namespace {

struct None {};

template <typename T> struct IsNone { static constexpr bool value = false; };
template <> struct IsNone<None> { static constexpr bool value = true; };

// C[j][k][i] = B[i][j][k] (to_core != 0) or B[i][j][k] = C[j][k][i]
__global__ __launch_bounds__(256) void permute_transfer_kernel(const double* in, double* out, int rS,
                                                               int rl, int rr, int to_core) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)rS * rl * rr;
  if (g >= total) return;
  const int64_t jk = g % ((int64_t)rl * rr);
  const int64_t i = g / ((int64_t)rl * rr);
  const int64_t c = jk * rS + i;   // (j rr + k) rS + i
  if (to_core)
    out[c] = in[g];
  else
    out[g] = in[c];
}

// out[a][e][b] = om[(a B + b) ell + e]: the Gaussian of a dense node sketch in
// the (pre, ell, post) layout of an unfolded product
template <typename T>
__global__ __launch_bounds__(256) void omega_unfold_kernel(const T* om, T* out, int64_t A, int64_t B, int ell) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = A * B * ell;
  if (g >= total) return;
  const int64_t b = g % B, ae = g / B;
  const int64_t e = ae % ell, a = ae / ell;
  out[g] = om[(a * B + b) * ell + e];
}

// out[c][r] = in[r][c] for an rows x cols FP64 matrix
__global__ __launch_bounds__(256) void transpose_f64_kernel(const double* in, double* out, int64_t rows,
                                                            int64_t cols) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= rows * cols) return;
  const int64_t r = g / cols, c = g - r * cols;
  out[c * rows + r] = in[g];
}

// T[a][k] = sum_j UL[a][j] BR[j][k] for k < rr; 0 for rr <= k < rpad
__global__ __launch_bounds__(256) void ht_rowmat_kernel(const double* UL, const double* BR, double* T,
                                                        int64_t nL, int rl, int rr, int rpad) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= nL * rpad) return;
  const int64_t a = g / rpad;
  const int k = (int)(g - a * rpad);
  double v = 0.0;
  if (k < rr)
    for (int j = 0; j < rl; ++j) v = fma(UL[a * rl + j], BR[j * rr + k], v);
  T[g] = v;
}

template <typename TX, typename TO, int R>
__global__ __launch_bounds__(256) void ht_expand_kernel(const HTExpand p) {
  constexpr int C = 64 / R;          // columns per lane
  constexpr int kRows = 4;           // rows per group; the next group's loads are in
                                     // flight while this group is multiplied
  constexpr bool kX = !IsNone<TX>::value, kO = !IsNone<TO>::value;
  using TL = typename std::conditional<kX, TX, float>::type;
  __shared__ double red[2][4];
  const int tid = threadIdx.x;
  const int64_t tile = blockIdx.x % p.ntile, grp = blockIdx.x / p.ntile;
  const int64_t a0 = grp * p.rows_per_group;
  const int64_t a1 = min(a0 + p.rows_per_group, p.nL);
  int64_t col[C];
  bool ok[C];
  double ur[C][R];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int64_t b = tile * (256 * C) + tid + 256 * c;
    ok[c] = b < p.nR;
    col[c] = ok[c] ? b : 0;          // in-range address for the idle columns
#pragma unroll
    for (int k = 0; k < R; ++k) ur[c][k] = (ok[c] && k < p.rr) ? p.UR[col[c] * p.rr + k] : 0.0;
  }
  const TL* X = static_cast<const TL*>(p.X);
  TO* Xh = static_cast<TO*>(p.Xh);
  double r2 = 0.0, x2 = 0.0;
  // rows past a1 - 1 load row a1 - 1 again (always in range) and add nothing
  auto load = [&](int64_t a, TL (&buf)[kRows][C]) {
    if constexpr (kX) {
#pragma unroll
      for (int u = 0; u < kRows; ++u) {
        const int64_t row = min(a + u, a1 - 1);
#pragma unroll
        for (int c = 0; c < C; ++c) buf[u][c] = X[row * p.nR + col[c]];
      }
    }
  };
  auto multiply = [&](int64_t a, const TL (&buf)[kRows][C]) {
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
      const bool live = a + u < a1;
      const int64_t row = min(a + u, a1 - 1);
      const double* t = p.T + row * R;
      double tk[R];
#pragma unroll
      for (int k = 0; k < R; ++k) tk[k] = t[k];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        double xh = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) xh = fma(tk[k], ur[c][k], xh);
        if constexpr (kX) {
          const double x = (live && ok[c]) ? to_double(buf[u][c]) : 0.0;
          const double d = (live && ok[c]) ? x - xh : 0.0;
          r2 = fma(d, d, r2);
          x2 = fma(x, x, x2);
        }
        if constexpr (kO) {
          if (live && ok[c]) Xh[row * p.nR + col[c]] = from_double<TO>(xh);
        }
      }
    }
  };
  // groups in pairs (ping-pong buffers); a pair past the end multiplies rows
  // that are not live and adds nothing
  // (the scheduling fences keep each prefetch ahead of the multiply that
  // precedes its use; without them the loads sink below it and the wave waits
  // for every load in flight)
  TL bA[kRows][C], bB[kRows][C];
  load(a0, bA);
  const int pairs = (int)((a1 - a0 + 2 * kRows - 1) / (2 * kRows));
  int64_t a = a0;
  for (int it = 0; it < pairs; ++it, a += 2 * kRows) {
    load(a + kRows, bB);
    __builtin_amdgcn_sched_barrier(0);
    multiply(a, bA);
    __builtin_amdgcn_sched_barrier(0);
    load(a + 2 * kRows, bA);
    __builtin_amdgcn_sched_barrier(0);
    multiply(a + kRows, bB);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (!p.partials) return;
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
    p.partials[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    p.partials[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

// Residual-only form for FP32 X and r_r <= 16 on v_mfma_f64_16x16x4f64: the
// same workgroup partition (a column tile of 256 C columns and a group of
// rows), each wave a quarter of the columns in strips of 64, each 16 x 16
// tile of X_hat as K = rpad / 4 MFMA steps (A operand T[a][4 s + l/16], B
// operand U_Rr[b][4 s + l/16] for column b = l%16 of the tile).  Register v
// of lane l is row l/16 + 4 v, column l%16, so X comes in as four b32 loads
// per tile (rows of 16 consecutive columns), the next row tile in flight
// while this one is multiplied; the squares are FP64.  The VALU form spends
// about 22 instructions per entry at r_r = 12.
template <int KS>
__global__ __launch_bounds__(256) void ht_resid_mfma_kernel(const HTExpand p) {
  typedef double doublex4 __attribute__((ext_vector_type(4)));
  constexpr int R = 4 * KS;
  constexpr int C = 64 / R;                 // columns per lane in the VALU form's partition
  constexpr int kStrips = C;                // 64-column strips per wave (a quarter of 256 C columns)
  __shared__ double red[2][4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int64_t tile = blockIdx.x % p.ntile, grp = blockIdx.x / p.ntile;
  const int64_t a0 = grp * p.rows_per_group;
  const int64_t a1 = min(a0 + p.rows_per_group, p.nL);
  const int nrt = (int)((a1 - a0 + 15) / 16);
  const float* X = static_cast<const float*>(p.X);
  double r2 = 0.0, x2 = 0.0;
  for (int cs = 0; cs < kStrips; ++cs) {
    const int64_t cb = tile * (256 * C) + (int64_t)(wv * kStrips + cs) * 64;
    // B operands of the strip's four column tiles
    double ub[4][KS];
    uint32_t coff[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int64_t b = cb + 16 * ct + l16;
#pragma unroll
      for (int k = 0; k < KS; ++k) ub[ct][k] = (b < p.nR && 4 * k + g < p.rr) ? p.UR[b * p.rr + 4 * k + g] : 0.0;
      coff[ct] = b < p.nR ? (uint32_t)(b * 4) : 0x80000000u;
    }
    auto issue = [&](int rt, float (&xv)[4][4]) {
      const int64_t row0 = a0 + 16 * (int64_t)rt;
      const int64_t rows = rt < nrt ? min<int64_t>(16, a1 - row0) : 0;
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float*>(X) + (rows > 0 ? row0 * p.nR : 0), (short)0, (int)(rows * p.nR * 4), 0x00020000);
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          xv[ct][v] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
              rs, coff[ct] + (uint32_t)((g + 4 * v) * p.nR * 4), 0, 0));
    };
    auto tile_rt = [&](int rt, const float (&xv)[4][4]) {
      const int64_t row = a0 + 16 * (int64_t)rt + l16;
      double ta[KS];
#pragma unroll
      for (int k = 0; k < KS; ++k) ta[k] = row < a1 ? p.T[row * p.rpad + 4 * k + g] : 0.0;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        doublex4 acc = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < KS; ++k) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ta[k], ub[ct][k], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double x = (double)xv[ct][v], d = x - acc[v];
          r2 = fma(d, d, r2);
          x2 = fma(x, x, x2);
        }
      }
    };
    // the next row tile in flight while this one is multiplied (four in
    // flight was slower: 12.9 against 10.5 ms at 18^8)
    float xa[4][4], xb[4][4];
    issue(0, xa);
    int rt = 0;
    for (; rt + 2 <= nrt; rt += 2) {
      issue(rt + 1, xb);
      __builtin_amdgcn_sched_barrier(0);
      tile_rt(rt, xa);
      issue(rt + 2, xa);
      __builtin_amdgcn_sched_barrier(0);
      tile_rt(rt + 1, xb);
    }
    if (rt < nrt) tile_rt(rt, xa);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    r2 += __shfl_xor(r2, off);
    x2 += __shfl_xor(x2, off);
  }
  if (lane == 0) {
    red[0][wv] = r2;
    red[1][wv] = x2;
  }
  __syncthreads();
  if (tid == 0) {
    p.partials[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    p.partials[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

// out[0..1] = sums of the workgroup partials, in a fixed order
__global__ __launch_bounds__(256) void ht_sum_kernel(const double* partials, int64_t nblocks, double* out) {
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = tid; i < nblocks; i += 256) {
    s0 += partials[2 * i];
    s1 += partials[2 * i + 1];
  }
  red[0][tid] = s0;
  red[1][tid] = s1;
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

template <typename TX, typename TO>
hipError_t expand_by_r(const HTExpand& p, hipStream_t st) {
  const dim3 grid((unsigned)(p.ntile * p.groups));
  switch (p.rpad) {
    case 8: hipLaunchKernelGGL((ht_expand_kernel<TX, TO, 8>), grid, dim3(256), 0, st, p); break;
    case 12: hipLaunchKernelGGL((ht_expand_kernel<TX, TO, 12>), grid, dim3(256), 0, st, p); break;
    case 16: hipLaunchKernelGGL((ht_expand_kernel<TX, TO, 16>), grid, dim3(256), 0, st, p); break;
    case 32: hipLaunchKernelGGL((ht_expand_kernel<TX, TO, 32>), grid, dim3(256), 0, st, p); break;
    default: hipLaunchKernelGGL((ht_expand_kernel<TX, TO, 64>), grid, dim3(256), 0, st, p); break;
  }
  return hipGetLastError();
}

template <typename TX>
hipError_t expand_by_out(const HTExpand& p, int out_dt, hipStream_t st) {
  switch (out_dt) {
    case -1: return expand_by_r<TX, None>(p, st);
    case TK_F64: return expand_by_r<TX, double>(p, st);
    case TK_F32: return expand_by_r<TX, float>(p, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace

int ht_expand_rpad(int rr) {
  return rr <= 8 ? 8 : rr <= 12 ? 12 : rr <= 16 ? 16 : rr <= 32 ? 32 : rr <= 64 ? 64 : 0;
}

void ht_expand_grid(HTExpand& p) {
  const int C = 64 / p.rpad;
  p.ntile = ceil_div(p.nR, 256 * C);
  int64_t groups = std::max<int64_t>(1, std::min<int64_t>(p.nL, ceil_div(4096, p.ntile)));
  p.rows_per_group = ceil_div(p.nL, groups);
  p.groups = ceil_div(p.nL, p.rows_per_group);
}

hipError_t launch_ht_rowmat(const double* UL, const double* BR, double* T, int64_t nL, int rl, int rr,
                            int rpad, hipStream_t st) {
  const int64_t n = nL * rpad;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(ht_rowmat_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, UL, BR, T,
                     nL, rl, rr, rpad);
  return hipGetLastError();
}

hipError_t launch_transpose_f64(const double* in, double* out, int64_t rows, int64_t cols, hipStream_t st) {
  const int64_t n = rows * cols;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(transpose_f64_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, in, out, rows,
                     cols);
  return hipGetLastError();
}

hipError_t launch_omega_to_unfolded(const void* om, void* out, int dt, int64_t A, int64_t B, int ell,
                                    hipStream_t st) {
  const int64_t n = A * B * ell;
  if (n == 0) return hipSuccess;
  const dim3 grid((unsigned)ceil_div(n, 256));
  if (dt == TK_F64)
    hipLaunchKernelGGL(omega_unfold_kernel<double>, grid, dim3(256), 0, st, static_cast<const double*>(om),
                       static_cast<double*>(out), A, B, ell);
  else if (dt == TK_F32)
    hipLaunchKernelGGL(omega_unfold_kernel<float>, grid, dim3(256), 0, st, static_cast<const float*>(om),
                       static_cast<float*>(out), A, B, ell);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_permute_transfer(const double* in, double* out, int rS, int rl, int rr, bool to_core,
                                   hipStream_t st) {
  const int64_t n = (int64_t)rS * rl * rr;
  hipLaunchKernelGGL(permute_transfer_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, in, out,
                     rS, rl, rr, to_core ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_ht_expand(const HTExpand& p, int x_dt, int out_dt, hipStream_t st) {
  if (p.rpad != 8 && p.rpad != 12 && p.rpad != 16 && p.rpad != 32 && p.rpad != 64)
    return hipErrorInvalidValue;
  hipError_t e = hipErrorInvalidValue;
  if (x_dt == TK_F32 && out_dt == -1 && p.partials && p.rpad <= 16 && p.nR * 64 < (int64_t(1) << 31)) {
    const dim3 grid((unsigned)(p.ntile * p.groups));
    if (p.rpad == 8) hipLaunchKernelGGL(ht_resid_mfma_kernel<2>, grid, dim3(256), 0, st, p);
    else if (p.rpad == 12) hipLaunchKernelGGL(ht_resid_mfma_kernel<3>, grid, dim3(256), 0, st, p);
    else hipLaunchKernelGGL(ht_resid_mfma_kernel<4>, grid, dim3(256), 0, st, p);
    e = hipGetLastError();
  } else switch (x_dt) {
    case -1: e = out_dt == -1 ? hipErrorInvalidValue : expand_by_out<None>(p, out_dt, st); break;
    case TK_F64: e = expand_by_out<double>(p, out_dt, st); break;
    case TK_F32: e = expand_by_out<float>(p, out_dt, st); break;
    case TK_BF16: e = expand_by_out<bf16>(p, out_dt, st); break;
    case TK_F16: e = expand_by_out<f16>(p, out_dt, st); break;
  }
  if (e != hipSuccess) return e;
  if (p.partials && p.resid2) {
    hipLaunchKernelGGL(ht_sum_kernel, dim3(1), dim3(256), 0, st, p.partials, p.ntile * p.groups, p.resid2);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace tk
