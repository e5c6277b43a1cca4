// Streaming residual of the Tucker reconstruction (Tucker format, Section 3)
// for tensors whose two trailing modes are small (n <= 64, ranks <= 16),
// BF16, FP16 or FP32 tensors, FP32 factors, on 16x16 FP32 MFMA tiles:
//   X_hat[a] = F_I T[a] F_J^T   (n_I x n_J, for the A slabs of X)
//   sum (X[a] - X_hat[a])^2, sum X[a]^2
// where T[a] (c_I x c_J, FP32) is the core expanded over the leading modes,
// so the pass reads X once and X_hat is never stored.
//
// One wave per slab at a time, persistent over slabs:
//  stage 1  P = T[a] F_J^T on v_mfma_f32_16x16x4f32 (A operand: lane l
//           gives T[a][l%16][4 ks + l/16]; B operand F_J^T from LDS), written
//           to the wave's LDS area so that it can serve as a B operand;
//  stage 2  X_hat tiles = F_I P (A operand F_I from LDS, B operand P),
//           register v of lane l holding row 16 it + 4 (l/16) + v, column
//           16 jt + l%16: the slab's values of X are loaded in that layout at
//           the start of the slab (a buffer range of one slab: rows past n_I
//           and the lanes of columns past n_J read zero) and meet X_hat in
//           registers (loading the next slab ahead instead was slower: it
//           costs a wave of occupancy per SIMD).
// The squares of a slab are summed in FP32 per lane (at most 64 terms), then
// added into FP64 per-lane sums; one pair per wave, summed in a fixed order
// by a second kernel.
#include "tk_kernels.hpp"

namespace tk {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kRsrcWord3 = 0x00020000;
constexpr int kMaxN = 64, kMaxC = 16;

__device__ __forceinline__ floatx4 mma16(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename TX> struct SlabLoad;
template <> struct SlabLoad<float> {
  static __device__ __forceinline__ float at(__amdgpu_buffer_rsrc_t r, uint32_t e) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, e * 4u, 0, 0));
  }
};
template <> struct SlabLoad<bf16> {
  static __device__ __forceinline__ float at(__amdgpu_buffer_rsrc_t r, uint32_t e) {
    const uint32_t u = __builtin_amdgcn_raw_buffer_load_b16(r, e * 2u, 0, 0);
    return __uint_as_float(u << 16);
  }
};
template <> struct SlabLoad<f16> {
  static __device__ __forceinline__ float at(__amdgpu_buffer_rsrc_t r, uint32_t e) {
    const unsigned short u = __builtin_amdgcn_raw_buffer_load_b16(r, e * 2u, 0, 0);
    return (float)__builtin_bit_cast(_Float16, u);
  }
};

template <typename TX, int NT>
__global__ __launch_bounds__(64 * kWaves) void resid_slab_kernel(const ResidSlab p) {
  __shared__ float sFI[kMaxN][kMaxC + 1];
  __shared__ float sFJ[kMaxN][kMaxC + 1];
  __shared__ float sP[kWaves][kMaxC][kMaxN + 1];
  const int nI = p.nI, nJ = p.nJ, cI = p.cI, cJ = p.cJ;
  for (int e = threadIdx.x; e < kMaxN * kMaxC; e += blockDim.x) {
    const int i = e / kMaxC, j = e - i * kMaxC;
    sFI[i][j] = (i < nI && j < cI) ? p.FI[i * cI + j] : 0.0f;
    sFJ[i][j] = (i < nJ && j < cJ) ? p.FJ[i * cJ + j] : 0.0f;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, l16 = lane & 15;
  const int gwave = __builtin_amdgcn_readfirstlane((int)blockIdx.x * kWaves + wave);
  const int kI = (cI + 3) / 4, kJ = (cJ + 3) / 4;
  const uint32_t slab = (uint32_t)(nI * nJ);
  // this lane's element offsets within a slab for tile (it, jt), register v;
  // columns past n_J point far outside the slab (read zero)
  uint32_t off[NT][NT];
#pragma unroll
  for (int it = 0; it < NT; ++it)
#pragma unroll
    for (int jt = 0; jt < NT; ++jt) {
      const int col = 16 * jt + l16;
      off[it][jt] = col < nJ ? (uint32_t)((16 * it + 4 * g) * nJ + col) : 0x20000000u;
    }
  double r2 = 0.0, x2 = 0.0;
  for (int64_t a = gwave; a < p.A; a += p.nwaves) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<TX*>(static_cast<const TX*>(p.X)) + a * slab, (short)0, (int)(slab * sizeof(TX)), kRsrcWord3);
    // the slab's X in the stage-2 output layout, loads first
    float xv[NT][NT][4];
#pragma unroll
    for (int it = 0; it < NT; ++it)
#pragma unroll
      for (int jt = 0; jt < NT; ++jt)
#pragma unroll
        for (int v = 0; v < 4; ++v) xv[it][jt][v] = SlabLoad<TX>::at(rs, off[it][jt] + (uint32_t)(v * nJ));
    const float* Ta = p.T + a * cI * cJ;
    float ta[kMaxC / 4];
#pragma unroll
    for (int ks = 0; ks < kMaxC / 4; ++ks) {
      const int k = 4 * ks + g;
      ta[ks] = (l16 < cI && k < cJ) ? Ta[l16 * cJ + k] : 0.0f;
    }
    // stage 1: P = T[a] F_J^T
#pragma unroll
    for (int jt = 0; jt < NT; ++jt) {
      floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < kMaxC / 4; ++ks)
        if (ks < kJ) acc = mma16(ta[ks], sFJ[16 * jt + l16][4 * ks + g], acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) sP[wave][4 * g + v][16 * jt + l16] = acc[v];
    }
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    // stage 2 and the squares
    float r2t = 0.0f, x2t = 0.0f;
#pragma unroll
    for (int it = 0; it < NT; ++it)
#pragma unroll
      for (int jt = 0; jt < NT; ++jt) {
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < kMaxC / 4; ++ks)
          if (ks < kI) acc = mma16(sFI[16 * it + l16][4 * ks + g], sP[wave][4 * ks + g][16 * jt + l16], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float x = xv[it][jt][v], d = x - acc[v];
          r2t = fmaf(d, d, r2t);
          x2t = fmaf(x, x, x2t);
        }
      }
    r2 += (double)r2t;
    x2 += (double)x2t;
    __builtin_amdgcn_wave_barrier();   // this slab's reads of sP precede the next slab's writes
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
  for (int o = 32; o > 0; o >>= 1) {
    r2 += __shfl_xor(r2, o);
    x2 += __shfl_xor(x2, o);
  }
  if (lane == 0) {
    p.partials[2 * gwave] = r2;
    p.partials[2 * gwave + 1] = x2;
  }
}

template <typename TX>
hipError_t launch_typed(const ResidSlab& p, int nt, hipStream_t st) {
  const dim3 grid((unsigned)(p.nwaves / kWaves));
  switch (nt) {
    case 1: hipLaunchKernelGGL((resid_slab_kernel<TX, 1>), grid, dim3(64 * kWaves), 0, st, p); break;
    case 2: hipLaunchKernelGGL((resid_slab_kernel<TX, 2>), grid, dim3(64 * kWaves), 0, st, p); break;
    case 3: hipLaunchKernelGGL((resid_slab_kernel<TX, 3>), grid, dim3(64 * kWaves), 0, st, p); break;
    default: hipLaunchKernelGGL((resid_slab_kernel<TX, 4>), grid, dim3(64 * kWaves), 0, st, p); break;
  }
  return hipGetLastError();
}

}  // namespace

bool resid_slab_supported(int x_dtype, int order, const int64_t* dims, const int32_t* cols) {
  if (x_dtype != TK_F32 && x_dtype != TK_BF16 && x_dtype != TK_F16) return false;
  if (order < 3) return false;
  const int64_t nI = dims[order - 2], nJ = dims[order - 1];
  int64_t A = 1;
  for (int k = 0; k < order - 2; ++k) A *= dims[k];
  return nI <= kMaxN && nJ <= kMaxN && cols[order - 2] <= kMaxC && cols[order - 1] <= kMaxC && A >= 1 &&
         A < (int64_t(1) << 40);
}

int64_t resid_slab_waves(int64_t A) {
  // persistent: up to eight workgroups of four waves per CU on 256 CUs
  return std::max<int64_t>(1, std::min<int64_t>(ceil_div(A, kWaves), 2048)) * kWaves;
}

hipError_t launch_resid_slab(const ResidSlab& pin, int x_dtype, hipStream_t st) {
  if (slab_resid_pipe_supported(x_dtype, pin.nI, pin.nJ))
    return launch_slab_resid_pipe(pin, x_dtype, (int)resid_slab_waves(pin.A), st);
  ResidSlab p = pin;
  p.nwaves = (int32_t)resid_slab_waves(p.A);
  const int nt = (int)ceil_div(std::max(p.nI, p.nJ), 16);
  hipError_t e;
  switch (x_dtype) {
    case TK_F32: e = launch_typed<float>(p, nt, st); break;
    case TK_BF16: e = launch_typed<bf16>(p, nt, st); break;
    default: e = launch_typed<f16>(p, nt, st); break;
  }
  if (e != hipSuccess) return e;
  if (p.resid2) return launch_pair_sum(p.partials, p.nwaves, p.resid2, st);
  return hipSuccess;
}

}  // namespace tk
