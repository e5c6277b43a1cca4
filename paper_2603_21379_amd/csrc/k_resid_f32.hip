// Streaming residual of the Tucker reconstruction for FP32 tensors on MFMA:
//   X_hat[a] = F_I T[a] F_J^T      (n_I x n_J, for the A slabs of X)
//   sum (X[a] - X_hat[a])^2,  sum X[a]^2
// where T[a] (c_I x c_J, FP32) is the core expanded over the leading modes.
// This is the last two expansions of the reconstruction (Tucker format,
// Section 3) fused with the error of the approximation, so X_hat is never
// stored unless asked for.
//
// Work unit: one 32-row tile of one 64-column half of a 128-column block of a
// slab.  Each wave walks its slabs (a, a + nwaves, ...) half-block by
// half-block and tile by tile, with the loads of the next NB - 1 units in
// flight while it computes one.  Eight waves per workgroup and one
// workgroup per CU (the -F_I pieces and F_J^T in LDS are shared by all
// eight) put two waves on each SIMD, so one wave's multiplies overlap the
// other's loads, LDS reads and sums.  Per unit (rows 32 it .., columns
// b0 + n and b0 + 32 + n for lane n):
//  stage 1  (first tile of a half-block) P = T[a] F_J^T on
//           v_mfma_f32_32x32x2f32: M = j (rows of T), K = j', one N tile per
//           32-column group;
//  stage 2  D = X - F_I P on v_mfma_f32_32x32x16_bf16 at FP32 accuracy: the
//           accumulators start from the tile of X itself (register v of lane
//           l holds row 8 (v/4) + 4 (l/32) + v%4 and column l%32, the MFMA
//           output layout, so each b32 load lands where the MFMA reads it),
//           and -F_I and P enter as three BF16 pieces each (x = h + m + l
//           exactly), of which the six products of rank sum <= 4 are
//           accumulated (the three dropped are ~2^-27 relative).  Starting
//           from X keeps the rounding error of D near u |D| (plus 2^-8 u |X|
//           from the first product) instead of u |X|.  Register v of a P
//           accumulator holds row j = 8 (v/4) + 4 (l/32) + v%4; K step ks
//           takes registers 8 ks .. 8 ks + 7 and the -F_I pieces in LDS
//           follow the same j order, so P feeds stage 2 without moving
//           between lanes;
//  sums     x^2 and d^2 over the lane's 32 entries of the tile in FP32
//           (relative error below 32 u), added into FP64 per-wave sums; one
//           pair per wave, summed in a fixed order by a second kernel.
//  Optionally X_hat and/or E = s D are written (s a device scalar times a
//  constant: the adjoint of ||X - X_hat||^2); E may alias X.  With X_hat
//  asked for, the accumulators start from zero (X_hat rounded once, as a
//  reconstruction) and D = X - X_hat follows in FP32.
#include "tk_kernels.hpp"

namespace tk {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));

constexpr int kCols = 128;
constexpr int kWaves = 8;                // two per SIMD: at most 256 VGPRs each
constexpr int kNB = 2;                   // row tiles per wave: NB - 1 in flight
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

// row stride of F_J^T in LDS: the 64 lanes of a stage-1 read hit 64 banks
__device__ __host__ __forceinline__ int fjt_stride(int nJ) {
  return ((nJ + kCols - 1) / kCols) * kCols + 32;
}

struct Cursor {
  int slab, hq, it;   // slab, half-block (block hq / 2, half hq % 2), row tile
};

// MODE bit 0: write X_hat; bit 1: write E = s (X - X_hat)
template <int NB, int MODE>
__global__ __launch_bounds__(64 * kWaves, 1) void resid2_f32_kernel(const ResidFused2 p) {
  extern __shared__ float lds[];
  const int nI = p.nI, nJ = p.nJ;
  const int nIt = (nI + 31) / 32;             // 32-row tiles of i
  const int nH = (nJ + kCols - 1) / kCols;    // 128-column blocks
  const int W = fjt_stride(nJ);
  // -F_I as the A operand of stage 2 in BF16 pieces: sFIp[it][ks][piece][lane]
  // (BF16x8) = -F_I[32 it + l%32][j] for the K slots 8 (l/32) + v of step ks,
  // j = 8 (2 ks + v/4) + 4 (l/32) + v%4 (the order the stage-1 accumulator
  // holds j in)
  uint32_t* sFIp = reinterpret_cast<uint32_t*>(lds);
  float* sFJt = lds + nIt * 2 * 3 * 64 * 4;      // F_J^T: [32][W], zero padded
  for (int e = threadIdx.x; e < nIt * 2 * 64; e += blockDim.x) {
    const int it = e >> 7, ks = (e >> 6) & 1, ln = e & 63, g = ln >> 5, i = it * 32 + (ln & 31);
    float x[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int j = 8 * (2 * ks + (v >> 2)) + 4 * g + (v & 3);
      x[v] = (i < nI && j < p.cI) ? -p.FI[i * p.cI + j] : 0.0f;
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
  for (int e = threadIdx.x; e < 32 * W; e += blockDim.x) {
    const int j = e / W, b = e - j * W;
    sFJt[e] = (b < nJ && j < p.cJ) ? p.FJ[b * p.cJ + j] : 0.0f;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, kh = lane >> 5, l32 = lane & 31;
  const int gwave = __builtin_amdgcn_readfirstlane((int)blockIdx.x * kWaves + (threadIdx.x >> 6));
  const int nwaves = p.nwaves;
  const int A32 = (int)p.A;
  const int64_t nIJ = (int64_t)nI * nJ;
  const uint32_t slab_bytes = (uint32_t)(nIJ * 4);
  const uint32_t row_bytes = (uint32_t)nJ * 4;
  const int nsl = gwave < A32 ? (A32 - 1 - gwave) / nwaves + 1 : 0;
  const int total = nsl * nH * 2 * nIt;
  double r2 = 0.0, x2 = 0.0;
  const float dscale = (MODE & 2) ? (float)(p.smul * (p.scale ? *p.scale : 1.0)) : 0.0f;

  auto advance = [&](Cursor& c) {
    if (++c.it == nIt) {
      c.it = 0;
      if (++c.hq == 2 * nH) {
        c.hq = 0;
        c.slab += nwaves;
      }
    }
  };
  // byte offset in the slab of this lane's entry of row 0 of a unit (row 4 kh
  // of the tile) in column group g; columns past n_J point far outside the
  // slab and read zero (and their stores are dropped), and so do rows past
  // n_I, the slowest index of a slab
  auto lane_off = [&](int hq, int g) -> uint32_t {
    const int b = (hq >> 1) * kCols + 64 * (hq & 1) + 32 * g + l32;
    return b < nJ ? (uint32_t)(4 * kh * nJ + b) * 4u : 0x80000000u;
  };
  auto row_off = [&](int it, int v) -> uint32_t {
    return (uint32_t)(it * 32 + 8 * (v >> 2) + (v & 3)) * row_bytes;
  };
  auto issue = [&](const Cursor& c, float (&xb)[2][16]) {
    // past the wave's last unit the range is empty: the loads return zero
    // without touching memory
    const bool live = c.slab < A32;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(p.X) + (int64_t)(live ? c.slab : 0) * nIJ, (short)0,
        live ? (int)slab_bytes : 0, kRsrcWord3);
    const uint32_t o0 = lane_off(c.hq, 0), o1 = lane_off(c.hq, 1);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const uint32_t r = row_off(c.it, v);
      xb[0][v] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, o0 + r, 0, 2));
      xb[1][v] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, o1 + r, 0, 2));
    }
  };

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
  float tcur[16], tnext[16];
  load_t(gwave, tnext);
  bf16x8 ph[2][2][3];   // P pieces: [column group][K step][piece]
#pragma unroll
  for (int g = 0; g < 2; ++g)
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int pc = 0; pc < 3; ++pc) ph[g][ks][pc] = bf16x8{};

  auto compute = [&](const Cursor& c, const float (&xb)[2][16]) {
    if (c.it == 0) {
      if (c.hq == 0) {
#pragma unroll
        for (int k = 0; k < 16; ++k) tcur[k] = tnext[k];
        load_t(c.slab + nwaves, tnext);
      }
      // stage 1: P_g[j][n] = sum_j' T[a][j][j'] F_J[b + 32 g][j'],
      // b = b0 + 64 (hq % 2) + n
      const int b = (c.hq >> 1) * kCols + 64 * (c.hq & 1) + l32;
      floatx16 P0 = floatx16{}, P1 = floatx16{};
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const float* fj = sFJt + (2 * k + kh) * W + b;
        P0 = mfma32(tcur[k], fj[0], P0);
        P1 = mfma32(tcur[k], fj[32], P1);
      }
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        float x0[8], x1[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          x0[v] = P0[8 * ks + v];
          x1[v] = P1[8 * ks + v];
        }
        split3(x0, ph[0][ks][0], ph[0][ks][1], ph[0][ks][2]);
        split3(x1, ph[1][ks][0], ph[1][ks][1], ph[1][ks][2]);
      }
    }
    // with X_hat asked for the accumulators start from zero instead, so that
    // X_hat itself is rounded once (D then follows as X + (-X_hat))
    floatx16 o0, o1;
    float x2t = 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      o0[v] = (MODE & 1) ? 0.0f : xb[0][v];
      o1[v] = (MODE & 1) ? 0.0f : xb[1][v];
      x2t = fmaf(xb[0][v], xb[0][v], fmaf(xb[1][v], xb[1][v], x2t));
    }
    // stage 2: D = X + (-F_I) P from six BF16 piece products per K step (hh,
    // hm, mh, hl, mm, lh), each exact in the FP32 accumulator
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const uint32_t* fa = sFIp + (((c.it * 2 + ks) * 3) * 64 + lane) * 4;
      bf16x8 a[3];
#pragma unroll
      for (int pc = 0; pc < 3; ++pc)
        a[pc] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uintx4*>(fa + pc * 64 * 4));
      o0 = mma_bf16(a[0], ph[0][ks][0], o0);
      o1 = mma_bf16(a[0], ph[1][ks][0], o1);
      o0 = mma_bf16(a[0], ph[0][ks][1], o0);
      o1 = mma_bf16(a[0], ph[1][ks][1], o1);
      o0 = mma_bf16(a[1], ph[0][ks][0], o0);
      o1 = mma_bf16(a[1], ph[1][ks][0], o1);
      o0 = mma_bf16(a[0], ph[0][ks][2], o0);
      o1 = mma_bf16(a[0], ph[1][ks][2], o1);
      o0 = mma_bf16(a[1], ph[0][ks][1], o0);
      o1 = mma_bf16(a[1], ph[1][ks][1], o1);
      o0 = mma_bf16(a[2], ph[0][ks][0], o0);
      o1 = mma_bf16(a[2], ph[1][ks][0], o1);
    }
    // rows past n_I and columns past n_J hold x = 0 and x_hat = 0 (zero
    // padded F_I rows and F_J^T columns): d = 0 there
    floatx16 d0 = o0, d1 = o1;
    if (MODE & 1) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        d0[v] = xb[0][v] + o0[v];
        d1[v] = xb[1][v] + o1[v];
      }
    }
    float r2t = 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v) r2t = fmaf(d0[v], d0[v], fmaf(d1[v], d1[v], r2t));
    r2 += (double)r2t;
    x2 += (double)x2t;
    if (MODE != 0) {
      const int64_t so = (int64_t)c.slab * nIJ;
      const uint32_t q0 = lane_off(c.hq, 0), q1 = lane_off(c.hq, 1);
      const __amdgpu_buffer_rsrc_t rxh = __builtin_amdgcn_make_buffer_rsrc(
          (MODE & 1) ? p.Xhat + so : const_cast<float*>(p.X), (short)0,
          (MODE & 1) ? (int)slab_bytes : 0, kRsrcWord3);
      const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(
          (MODE & 2) ? p.D + so : const_cast<float*>(p.X), (short)0,
          (MODE & 2) ? (int)slab_bytes : 0, kRsrcWord3);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const uint32_t r = row_off(c.it, v);
        if (MODE & 1) {
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(-o0[v]), rxh, q0 + r, 0, 0);
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(-o1[v]), rxh, q1 + r, 0, 0);
        }
        if (MODE & 2) {
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(dscale * d0[v]), rd, q0 + r, 0, 0);
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(dscale * d1[v]), rd, q1 + r, 0, 0);
        }
      }
    }
  };

  Cursor cl{gwave, 0, 0}, cc{gwave, 0, 0};
  float xb[NB][2][16];
#pragma unroll
  for (int k = 0; k < NB - 1; ++k) {
    issue(cl, xb[k]);
    advance(cl);
  }
#pragma unroll 1
  for (int u = 0; u < total; u += NB) {
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      issue(cl, xb[(k + NB - 1) % NB]);
      advance(cl);
      __builtin_amdgcn_sched_barrier(0);
      if (u + k < total) {
        compute(cc, xb[k]);
        advance(cc);
      }
      __builtin_amdgcn_sched_barrier(0);
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
  // -F_I pieces (6 KB per 32-row tile) and F_J^T in FP32
  return (size_t)((nI + 31) / 32) * 2 * 3 * 64 * 16 + (size_t)32 * fjt_stride(nJ) * sizeof(float);
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
  const dim3 grid((unsigned)(waves / kWaves));
  const size_t lds = resid2_lds_bytes(p.nI, p.nJ);
  const int mode = (p.Xhat ? 1 : 0) | (p.D ? 2 : 0);
  switch (mode) {
    case 0: hipLaunchKernelGGL((resid2_f32_kernel<kNB, 0>), grid, dim3(64 * kWaves), lds, st, p); break;
    case 1: hipLaunchKernelGGL((resid2_f32_kernel<kNB, 1>), grid, dim3(64 * kWaves), lds, st, p); break;
    case 2: hipLaunchKernelGGL((resid2_f32_kernel<kNB, 2>), grid, dim3(64 * kWaves), lds, st, p); break;
    default: hipLaunchKernelGGL((resid2_f32_kernel<kNB, 3>), grid, dim3(64 * kWaves), lds, st, p); break;
  }
  if (p.resid2)
    hipLaunchKernelGGL(resid_sum_kernel, dim3(1), dim3(256), 0, st, p.partials, (int)waves,
                       p.resid2);
  return hipGetLastError();
}

}  // namespace tk
