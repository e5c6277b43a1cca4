// Streaming residual of the Tucker reconstruction for FP32 tensors on MFMA:
//   X_hat[a] = F_I T[a] F_J^T      (n_I x n_J, for the A slabs of X)
//   sum (X[a] - X_hat[a])^2,  sum X[a]^2    (FP64 per wave, the squared
//   differences first summed in FP32 over 32 entries; a fixed-order final sum)
// where T[a] (c_I x c_J, FP32) is the core expanded over the leading modes.
// This is the last two expansions of the reconstruction (Tucker format,
// Section 3) fused with the error of the approximation, so X_hat is never
// stored unless asked for.
//
// Per slab and 128-column block b0 (one wave, persistent over slabs):
//  stage 1  P = T[a] F_J^T on v_mfma_f32_32x32x2f32: M = j (rows of T), K = j',
//           four N tiles whose column n stands for b = b0 + 4 n + c;
//  stage 2  X_hat = F_I P on v_mfma_f32_32x32x16_bf16 at FP32 accuracy: P and
//           F_I are split into three BF16 pieces (x = h + m + l exactly) and
//           the six piece products of rank sum <= 4 are accumulated in FP32
//           (the three dropped are ~2^-27 relative).  Register v of a P
//           accumulator holds row j = 8 (v/4) + 4 (l/32) + v%4 for column n;
//           K step ks takes registers 8 ks .. 8 ks + 7 as its K slots and the
//           F_I pieces in LDS follow the same j order, so P feeds stage 2
//           without moving between lanes.
//  The block is taken as two halves of 64 columns, q = 0, 1: in half q,
//  lane n owns columns b0 + 64 q + 2 n + {0, 1}, a float2 of X per lane, so
//  each load covers two 256-byte row segments and a half's cache lines are
//  used within that half.  The two output tiles of a half line up with that
//  float2 and are compared in FP64.  The next row tile of X is loaded while
//  the current one is multiplied.
//  Optionally D = s (X - X_hat) is written in place of (or beside) X_hat,
//  with s a device scalar times a constant (the adjoint of ||X - X_hat||^2).
#include "tk_kernels.hpp"

namespace tk {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));

constexpr int kCols = 128;
constexpr int kWaves = 4;
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx16 mma_bf16(bf16x8 a, bf16x8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// x (8 FP32 values) -> BF16 pieces h, m, l with x = h + m + l exactly:
// h = rne(x), m = rne(x - h), l = rne(x - h - m), each difference exact in FP32
__device__ __forceinline__ void split3(const float (&x)[8], bf16x8& h, bf16x8& m, bf16x8& l) {
  uintx4 hh, mm, ll;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const floatx2 v = {x[2 * w], x[2 * w + 1]};
    const uint32_t hb = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
    const floatx2 r1 = {v[0] - __uint_as_float(hb << 16), v[1] - __uint_as_float(hb & 0xFFFF0000u)};
    const uint32_t mb = __builtin_bit_cast(uint32_t, __builtin_convertvector(r1, bf16x2));
    const floatx2 r2 = {r1[0] - __uint_as_float(mb << 16), r1[1] - __uint_as_float(mb & 0xFFFF0000u)};
    hh[w] = hb;
    mm[w] = mb;
    ll[w] = __builtin_bit_cast(uint32_t, __builtin_convertvector(r2, bf16x2));
  }
  h = __builtin_bit_cast(bf16x8, hh);
  m = __builtin_bit_cast(bf16x8, mm);
  l = __builtin_bit_cast(bf16x8, ll);
}

__global__ __launch_bounds__(256, 1) void resid2_f32_kernel(const ResidFused2 p) {
  extern __shared__ float lds[];
  const int nIt = (p.nI + 31) / 32;             // 32-row tiles of i
  const int nH = (p.nJ + kCols - 1) / kCols;    // 128-column blocks
  // F_I as the A operand of stage 2 in BF16 pieces: sFIp[it][ks][piece][lane]
  // (BF16x8) = F_I[32 it + l%32][j] for the K slots 8 (l/32) + v of step ks,
  // j = 8 (2 ks + v/4) + 4 (l/32) + v%4 (the order the stage-1 accumulator
  // holds j in, so P needs no exchange between lanes)
  uint32_t* sFIp = reinterpret_cast<uint32_t*>(lds);
  float* sFJ = lds + nIt * 2 * 3 * 64 * 4;       // [nH * 128][32], zero padded
  for (int e = threadIdx.x; e < nIt * 2 * 64; e += blockDim.x) {
    const int it = e >> 7, ks = (e >> 6) & 1, ln = e & 63, g = ln >> 5, i = it * 32 + (ln & 31);
    float x[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int j = 8 * (2 * ks + (v >> 2)) + 4 * g + (v & 3);
      x[v] = (i < p.nI && j < p.cI) ? p.FI[i * p.cI + j] : 0.0f;
    }
    bf16x8 h, m, l;
    split3(x, h, m, l);
    const uintx4 uh = __builtin_bit_cast(uintx4, h), um = __builtin_bit_cast(uintx4, m),
                 ul = __builtin_bit_cast(uintx4, l);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      sFIp[((((it * 2 + ks) * 3) + 0) * 64 + ln) * 4 + w] = uh[w];
      sFIp[((((it * 2 + ks) * 3) + 1) * 64 + ln) * 4 + w] = um[w];
      sFIp[((((it * 2 + ks) * 3) + 2) * 64 + ln) * 4 + w] = ul[w];
    }
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
  const bool want_d = p.D != nullptr;
  const float dscale = (float)(p.smul * (p.scale ? *p.scale : 1.0));

  // the A operand of stage 1, T[a][j = l32][j' = 2 k + kh] (k = 0..15), is
  // loaded one slab ahead so the multiplies never wait on it
  auto load_t = [&](int slab, float (&t)[16]) {
    const float* Ta = p.T + (int64_t)min(slab, A32 - 1) * p.cI * p.cJ;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int jp = 2 * k + kh;
      t[k] = (slab < A32 && l32 < p.cI && jp < p.cJ) ? Ta[l32 * p.cJ + jp] : 0.0f;
    }
  };
  float tnext[16];
  load_t(gwave, tnext);
  for (int slab = gwave; slab < A32; slab += nwaves) {
    float tcur[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) tcur[k] = tnext[k];
    load_t(slab + nwaves, tnext);
    const float* base = p.X + (int64_t)slab * nIJ;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, (int)slab_bytes, kRsrcWord3);
    const bool want_xh = p.Xhat != nullptr;
    const __amdgpu_buffer_rsrc_t rxh = __builtin_amdgcn_make_buffer_rsrc(
        want_xh ? p.Xhat + (int64_t)slab * nIJ : const_cast<float*>(base), (short)0,
        want_xh ? (int)slab_bytes : 0, kRsrcWord3);
    const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(
        want_d ? p.D + (int64_t)slab * nIJ : const_cast<float*>(base), (short)0,
        want_d ? (int)slab_bytes : 0, kRsrcWord3);

#pragma unroll 1
    for (int h = 0; h < nH; ++h) {
      const int b0 = h * kCols;
      // one half q of the block (columns b0 + 64 q + 2 n, + 1 for lane n) at a
      // time keeps two P tiles live instead of four; stage 1 costs the same
#pragma unroll 1
      for (int q = 0; q < 2; ++q) {
        const int b = b0 + 64 * q + 2 * l32;
        const bool colok = b < p.nJ;
        auto load_unit = [&](int it, floatx2 (&buf)[16]) {
          // lanes past the column tail point far outside the range: they read zero
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int i = it * 32 + 8 * (v >> 2) + 4 * kh + (v & 3);
            const uint32_t off =
                (colok && i < p.nI) ? (uint32_t)((i * p.nJ + b) * 4) : 0x80000000u;
            buf[v] = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 2);
          }
        };
        // the first row tile of X is in flight during stage 1
        floatx2 bufA[16], bufB[16];
        load_unit(0, bufA);
        // stage 1: P_c[j][n] = sum_j' T[a][j][j'] F_J[b0 + 64 q + 2 n + c][j'], c = 0, 1
        floatx16 P0 = floatx16{}, P1 = floatx16{};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          // A = T[a][j = l32][j' = 2 k + kh]
          const int jp = 2 * k + kh;
          P0 = mfma32(tcur[k], sFJ[b * 32 + jp], P0);
          P1 = mfma32(tcur[k], sFJ[(b + 1) * 32 + jp], P1);
        }
        // P in BF16 pieces as the B operand of stage 2: step ks takes the
        // accumulator registers 8 ks .. 8 ks + 7 (j = 8 (v/4) + 4 kh + v%4)
        bf16x8 ph0[2][3], ph1[2][3];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          float x0[8], x1[8];
#pragma unroll
          for (int v = 0; v < 8; ++v) {
            x0[v] = P0[8 * ks + v];
            x1[v] = P1[8 * ks + v];
          }
          split3(x0, ph0[ks][0], ph0[ks][1], ph0[ks][2]);
          split3(x1, ph1[ks][0], ph1[ks][1], ph1[ks][2]);
        }
        auto unit = [&](int it, const floatx2 (&xb)[16]) {
          // stage 2: X_hat tile = F_I P from six BF16 piece products per K
          // step (hh, hm, mh, hl, mm, lh; the dropped ones are ~2^-27
          // relative), each exact in the FP32 accumulator
          floatx16 o0 = floatx16{}, o1 = floatx16{};
#pragma unroll
          for (int ks = 0; ks < 2; ++ks) {
            const uint32_t* fa = sFIp + (((it * 2 + ks) * 3) * 64 + lane) * 4;
            bf16x8 a[3];
#pragma unroll
            for (int pc = 0; pc < 3; ++pc)
              a[pc] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uintx4*>(fa + pc * 64 * 4));
            o0 = mma_bf16(a[0], ph0[ks][0], o0);
            o1 = mma_bf16(a[0], ph1[ks][0], o1);
            o0 = mma_bf16(a[0], ph0[ks][1], o0);
            o1 = mma_bf16(a[0], ph1[ks][1], o1);
            o0 = mma_bf16(a[1], ph0[ks][0], o0);
            o1 = mma_bf16(a[1], ph1[ks][0], o1);
            o0 = mma_bf16(a[0], ph0[ks][2], o0);
            o1 = mma_bf16(a[0], ph1[ks][2], o1);
            o0 = mma_bf16(a[1], ph0[ks][1], o0);
            o1 = mma_bf16(a[1], ph1[ks][1], o1);
            o0 = mma_bf16(a[2], ph0[ks][0], o0);
            o1 = mma_bf16(a[2], ph1[ks][0], o1);
          }
          // (x - x_hat)^2 in FP32 over the tile's 32 entries of this lane (x
          // and x_hat are FP32, their difference is exact or within u |d|),
          // then added to the FP64 sum; x^2 exactly in FP64.  Rows past n_I
          // and columns past n_J hold x = x_hat = 0 and add nothing.
          float r2t = 0.0f;
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const float d0 = xb[v][0] - o0[v], d1 = xb[v][1] - o1[v];
            r2t = fmaf(d0, d0, fmaf(d1, d1, r2t));
            const double x0 = xb[v][0], x1 = xb[v][1];
            x2 = fma(x0, x0, fma(x1, x1, x2));
          }
          r2 += (double)r2t;
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int i = it * 32 + 8 * (v >> 2) + 4 * kh + (v & 3);
            if ((want_xh || want_d) && colok && i < p.nI) {
              if (want_xh) {
                floatx2 w;
                w[0] = o0[v];
                w[1] = o1[v];
                __builtin_amdgcn_raw_buffer_store_b64(w, rxh, (uint32_t)((i * p.nJ + b) * 4), 0, 0);
              }
              if (want_d) {
                floatx2 w;
                w[0] = dscale * (xb[v][0] - o0[v]);
                w[1] = dscale * (xb[v][1] - o1[v]);
                __builtin_amdgcn_raw_buffer_store_b64(w, rd, (uint32_t)((i * p.nJ + b) * 4), 0, 0);
              }
            }
          }
        };
        // stage 2 over row tiles with the next tile of X in flight; every
        // step issues the next tile's loads (past n_I they read zero), so the
        // waits count loads instead of waiting for all of them
        int it = 0;
#pragma unroll 1
        for (; it + 2 <= nIt; it += 2) {
          load_unit(it + 1, bufB);
          __builtin_amdgcn_sched_barrier(0);
          unit(it, bufA);
          load_unit(it + 2, bufA);
          __builtin_amdgcn_sched_barrier(0);
          unit(it + 1, bufB);
        }
        if (it < nIt) unit(it, bufA);
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
  // F_I pieces (6 KB per 32-row tile) and F_J in FP32
  return (size_t)((nI + 31) / 32) * 2 * 3 * 64 * 16 + (size_t)((nJ + kCols - 1) / kCols) * kCols * 32 * sizeof(float);
}

bool resid2_supported(int dtype, int order, const int64_t* dims, const int32_t* cols) {
  if (dtype != TK_F32 || order < 3) return false;
  const int64_t nI = dims[order - 2], nJ = dims[order - 1];
  int64_t A = 1;
  for (int k = 0; k < order - 2; ++k) A *= dims[k];
  if (nI > 1024 || nJ > 1024 || A >= (int64_t(1) << 31)) return false;
  return nJ % 4 == 0 && nJ >= 64 && cols[order - 2] <= 32 && cols[order - 1] <= 32 && A >= 256 &&
         resid2_lds_bytes((int)nI, (int)nJ) <= 128 * 1024;
}

int64_t resid2_waves(int64_t A) {
  // one workgroup per CU on 256 CUs: every wave resident, persistent over slabs
  return std::max<int64_t>(1, std::min<int64_t>(ceil_div(A, kWaves), 256)) * kWaves;
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
