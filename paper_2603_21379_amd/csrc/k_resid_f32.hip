// Streaming residual of the Tucker reconstruction for FP32 tensors on MFMA:
//   X_hat[a] = F_I T[a] F_J^T      (n_I x n_J, for the A slabs of X)
//   sum (X[a] - X_hat[a])^2,  sum X[a]^2    (FP64, per wave, then a fixed-order sum)
// where T[a] (c_I x c_J, FP32) is the core expanded over the leading modes.
// This is the last two expansions of the reconstruction (Tucker format,
// Section 3) fused with the error of the approximation, so X_hat is never
// stored unless asked for.
//
// Per slab and 128-column block b0 (one wave, persistent over slabs):
//  stage 1  P = T[a] F_J^T on v_mfma_f32_32x32x2f32: M = j (rows of T), K = j',
//           four N tiles whose column n stands for b = b0 + 4 n + c;
//  stage 2  X_hat = F_I P: for every 32-row tile of i, register v of a P
//           accumulator holds rows j = 8 (v/4) + 4 (l/32) + v%4 for column n,
//           which is the B operand of a K = 2 step over the row pair
//           {j, j + 4}, so P feeds stage 2 without moving; F_I comes from LDS.
//  The output tiles of components c = 2 q, 2 q + 1 line up with a float2 of X
//  per lane (X[a][i][b0 + 4 n + 2 q .. +1]), loaded coalesced and compared in
//  FP64.  The next (row tile, component pair) of X is loaded while the
//  current one is multiplied.
#include "tk_kernels.hpp"

namespace tk {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

constexpr int kCols = 128;
constexpr int kWaves = 4;
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(256, 1) void resid2_f32_kernel(const ResidFused2 p) {
  extern __shared__ float lds[];
  const int nIt = (p.nI + 31) / 32;             // 32-row tiles of i
  const int nH = (p.nJ + kCols - 1) / kCols;    // 128-column blocks
  float* sFI = lds;                              // [nIt * 32][32], zero padded
  float* sFJ = lds + nIt * 32 * 32;              // [nH * 128][32], zero padded
  for (int e = threadIdx.x; e < nIt * 32 * 32; e += blockDim.x) {
    const int i = e >> 5, j = e & 31;
    sFI[e] = (i < p.nI && j < p.cI) ? p.FI[i * p.cI + j] : 0.0f;
  }
  for (int e = threadIdx.x; e < nH * kCols * 32; e += blockDim.x) {
    const int b = e >> 5, j = e & 31;
    sFJ[e] = (b < p.nJ && j < p.cJ) ? p.FJ[b * p.cJ + j] : 0.0f;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, kh = lane >> 5, l32 = lane & 31;
  const int gwave = __builtin_amdgcn_readfirstlane((int)blockIdx.x * kWaves + (threadIdx.x >> 6));
  const int nwaves = p.nwaves;
  const int A32 = (int)p.A;
  const int64_t nIJ = (int64_t)p.nI * p.nJ;
  const uint32_t slab_bytes = (uint32_t)(nIJ * 4);
  double r2 = 0.0, x2 = 0.0;

  for (int slab = gwave; slab < A32; slab += nwaves) {
    const float* Ta = p.T + (int64_t)slab * p.cI * p.cJ;
    const float* base = p.X + (int64_t)slab * nIJ;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, (int)slab_bytes, kRsrcWord3);
    const bool want_xh = p.Xhat != nullptr;
    const __amdgpu_buffer_rsrc_t rxh = __builtin_amdgcn_make_buffer_rsrc(
        want_xh ? p.Xhat + (int64_t)slab * nIJ : const_cast<float*>(base), (short)0,
        want_xh ? (int)slab_bytes : 0, kRsrcWord3);

#pragma unroll 1
    for (int h = 0; h < nH; ++h) {
      const int b0 = h * kCols;
      const int b = b0 + 4 * l32;
      const bool colok = b < p.nJ;
      // one component pair q (columns b0 + 4 n + 2 q, + 1) at a time keeps two P
      // tiles live instead of four; stage 1 costs the same either way
#pragma unroll 1
      for (int q = 0; q < 2; ++q) {
        // stage 1: P_c[j][n] = sum_j' T[a][j][j'] F_J[b0 + 4 n + c][j'], c = 2 q + {0, 1}
        floatx16 P0 = floatx16{}, P1 = floatx16{};
#pragma unroll 4
        for (int k = 0; k < 16; ++k) {
          // A = T[a][j = l32][j' = 2 k + kh] (4 KB per slab, cache resident)
          const int jp = 2 * k + kh;
          const float t = (l32 < p.cI && jp < p.cJ) ? Ta[l32 * p.cJ + jp] : 0.0f;
          P0 = mfma32(t, sFJ[(b + 2 * q) * 32 + jp], P0);
          P1 = mfma32(t, sFJ[(b + 2 * q + 1) * 32 + jp], P1);
        }
        auto load_unit = [&](int it, floatx2 (&buf)[16]) {
          // lanes past the column tail point far outside the range: they read zero
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int i = it * 32 + 8 * (v >> 2) + 4 * kh + (v & 3);
            const uint32_t off =
                (colok && i < p.nI) ? (uint32_t)((i * p.nJ + b + 2 * q) * 4) : 0x80000000u;
            buf[v] = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 2);
          }
        };
        auto unit = [&](int it, const floatx2 (&xb)[16]) {
          floatx16 o0 = floatx16{}, o1 = floatx16{};
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            // K pair {j, j + 4}, j = 8 (v/4) + v%4; A = F_I[it*32 + l32][j + 4 kh]
            const int j = 8 * (v >> 2) + 4 * kh + (v & 3);
            const float f = sFI[(it * 32 + l32) * 32 + j];
            o0 = mfma32(f, P0[v], o0);
            o1 = mfma32(f, P1[v], o1);
          }
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int i = it * 32 + 8 * (v >> 2) + 4 * kh + (v & 3);
            if (colok && i < p.nI) {
              const double x0 = xb[v][0], x1 = xb[v][1];
              const double d0 = x0 - (double)o0[v], d1 = x1 - (double)o1[v];
              r2 = fma(d0, d0, fma(d1, d1, r2));
              x2 = fma(x0, x0, fma(x1, x1, x2));
              if (want_xh) {
                floatx2 w;
                w[0] = o0[v];
                w[1] = o1[v];
                __builtin_amdgcn_raw_buffer_store_b64(w, rxh, (uint32_t)((i * p.nJ + b + 2 * q) * 4), 0, 0);
              }
            }
          }
        };
        // stage 2 over row tiles with the next tile of X in flight
        floatx2 bufA[16], bufB[16];
        load_unit(0, bufA);
#pragma unroll 1
        for (int it = 0; it < nIt; it += 2) {
          if (it + 1 < nIt) load_unit(it + 1, bufB);
          __builtin_amdgcn_sched_barrier(0);
          unit(it, bufA);
          if (it + 1 >= nIt) break;
          if (it + 2 < nIt) load_unit(it + 2, bufA);
          __builtin_amdgcn_sched_barrier(0);
          unit(it + 1, bufB);
        }
      }
    }
  }
  // wave sum, then one partial pair per wave
  for (int off = 32; off > 0; off >>= 1) {
    r2 += __shfl_xor(r2, off);
    x2 += __shfl_xor(x2, off);
  }
  if (lane == 0 && gwave < nwaves) {
    p.partials[2 * gwave] = r2;
    p.partials[2 * gwave + 1] = x2;
  }
}

__global__ __launch_bounds__(256) void resid_sum_kernel(const double* partials, int n, double* out) {
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int i = tid; i < n; i += 256) {
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

}  // namespace

size_t resid2_lds_bytes(int nI, int nJ) {
  return (size_t)(((nI + 31) / 32) * 32 + ((nJ + kCols - 1) / kCols) * kCols) * 32 * sizeof(float);
}

bool resid2_supported(int dtype, int order, const int64_t* dims, const int32_t* cols) {
  if (dtype != TK_F32 || order < 3) return false;
  const int64_t nI = dims[order - 2], nJ = dims[order - 1];
  int64_t A = 1;
  for (int k = 0; k < order - 2; ++k) A *= dims[k];
  if (nI > 1024 || nJ > 1024 || A >= (int64_t(1) << 31)) return false;
  return nJ % 4 == 0 && nJ >= 64 && cols[order - 2] <= 32 && cols[order - 1] <= 32 && A >= 256 &&
         resid2_lds_bytes((int)nI, (int)nJ) <= 64 * 1024;
}

int64_t resid2_waves(int64_t A) {
  return std::max<int64_t>(1, std::min<int64_t>(ceil_div(A, kWaves), 1024)) * kWaves;
}

hipError_t launch_resid2_f32(const ResidFused2& pin, hipStream_t st) {
  ResidFused2 p = pin;
  const int64_t waves = resid2_waves(p.A);
  p.nwaves = (int32_t)waves;
  hipLaunchKernelGGL(resid2_f32_kernel, dim3((unsigned)(waves / kWaves)), dim3(256),
                     resid2_lds_bytes(p.nI, p.nJ), st, p);
  if (p.resid2)
    hipLaunchKernelGGL(resid_sum_kernel, dim3(1), dim3(256), 0, st, p.partials, (int)waves,
                       p.resid2);
  return hipGetLastError();
}

}  // namespace tk
