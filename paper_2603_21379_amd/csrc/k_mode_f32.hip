// Contraction of one leading or middle mode of an FP32 tensor on MFMA (the
// TTM of Section 2.2 with F^T):
//   out[a][p][b] = sum_q F[q][p] in[a][q][b]      (p < P <= 32)
// used for the modes that remain after the streaming pass of the core, where
// `in` is the partial core (much smaller than X but still hundreds of MB for
// large tensors).
//
// One wavefront owns a unit (a, 32 VEC consecutive b, VEC = 4, 2 or 1) and
// walks q two rows at a time with v_mfma_f32_32x32x2f32: the A operand is F^T
// from LDS (lane l gives F[q + l/32][p = l%32]), the B operand comes from VEC
// floats per lane, in[a][q + l/32][b0 + VEC (l%32) .. + VEC - 1], whose
// component c is the B tile of accumulator c for columns b = b0 + VEC n + c.
// The launcher takes the widest VEC that still gives about eight waves per CU
// (a contraction with few (a, column block) units gets narrower blocks).  Rows
// past Q read zero through the buffer range check; columns past B only feed
// output columns that are not stored.
#include "tk_kernels.hpp"

namespace tk {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

constexpr int kWaves = 4;
constexpr int kKB = 8;        // row pairs per load batch
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// VEC columns per lane (4, 2 or 1): a unit covers 32 VEC columns, so tensors
// with few (a, column block) units still fill the chip with narrower blocks.
template <int VEC> struct ColVec;
template <> struct ColVec<4> {
  typedef floatx4 T;
  static __device__ __forceinline__ T load(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
  }
  static __device__ __forceinline__ float at(const T& v, int c) { return v[c]; }
};
template <> struct ColVec<2> {
  typedef floatx2 T;
  static __device__ __forceinline__ T load(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
  }
  static __device__ __forceinline__ float at(const T& v, int c) { return v[c]; }
};
template <> struct ColVec<1> {
  typedef float T;
  static __device__ __forceinline__ T load(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
  }
  static __device__ __forceinline__ float at(const T& v, int) { return v; }
};

template <typename TOut, int VEC>
__global__ __launch_bounds__(256) void mode_mfma_f32_kernel(const ModeMfma m) {
  typedef typename ColVec<VEC>::T vec_t;
  constexpr int kBlk = 32 * VEC;   // columns per unit
  extern __shared__ float sF[];   // [Qp][32], zero padded
  const int Qp = (int)((m.Q + 2 * kKB - 1) / (2 * kKB)) * 2 * kKB;
  for (int e = threadIdx.x; e < Qp * 32; e += blockDim.x) {
    const int q = e >> 5, p = e & 31;
    sF[e] = (q < m.Q && p < m.P) ? m.F[(int64_t)q * m.P + p] : 0.0f;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, kh = lane >> 5, l32 = lane & 31;
  const int64_t nBb = (m.B + kBlk - 1) / kBlk;
  const int64_t unit = wave_uniform((int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6));
  if (unit >= m.A * nBb) return;  // no barrier follows
  const int64_t a = unit / nBb;
  const int64_t b0 = (unit - a * nBb) * kBlk;
  const int64_t slab = m.Q * m.B;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(m.in + a * slab), (short)0, (int)(slab * 4), kRsrcWord3);
  const int64_t b = b0 + VEC * l32;
  const bool colok = b < m.B;
  const uint32_t rowb = (uint32_t)(m.B * 4);

  auto load = [&](int q0, vec_t (&buf)[kKB]) {
#pragma unroll
    for (int u = 0; u < kKB; ++u) {
      const int q = q0 + 2 * u + kh;
      const uint32_t off = (colok && q < m.Q) ? (uint32_t)q * rowb + (uint32_t)(b * 4) : 0x80000000u;
      buf[u] = ColVec<VEC>::load(rs, off);
    }
  };
  floatx16 acc[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) acc[c] = floatx16{};
  auto compute = [&](int q0, const vec_t (&buf)[kKB]) {
    const float* f = sF + (q0 + kh) * 32 + l32;
#pragma unroll
    for (int u = 0; u < kKB; ++u) {
      const float fv = f[u * 64];
#pragma unroll
      for (int c = 0; c < VEC; ++c) acc[c] = mfma32(fv, ColVec<VEC>::at(buf[u], c), acc[c]);
    }
  };
  // batches of kKB row pairs, double buffered: every step issues the next
  // batch's loads (past Q they read zero) before multiplying the current one,
  // so the waits count loads and one batch stays in flight
  const int nb = Qp / (2 * kKB);
  vec_t bufA[kKB], bufB[kKB];
  load(0, bufA);
  int bq = 0;
  for (; bq + 2 <= nb; bq += 2) {
    load((bq + 1) * 2 * kKB, bufB);
    __builtin_amdgcn_sched_barrier(0);
    compute(bq * 2 * kKB, bufA);
    load((bq + 2) * 2 * kKB, bufA);
    __builtin_amdgcn_sched_barrier(0);
    compute((bq + 1) * 2 * kKB, bufB);
  }
  if (bq < nb) compute(bq * 2 * kKB, bufA);
  // acc[c] register v: p = 8 (v/4) + 4 kh + v%4, column b + c
  TOut* out = static_cast<TOut*>(m.out) + a * (int64_t)m.P * m.B;
  if (!colok) return;
  const int ncol = (int)min<int64_t>(VEC, m.B - b);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int p = 8 * (v >> 2) + 4 * kh + (v & 3);
    if (p >= m.P) continue;
    TOut* o = out + (int64_t)p * m.B + b;
#pragma unroll
    for (int c = 0; c < VEC; ++c)
      if (c < ncol) o[c] = (TOut)acc[c][v];
  }
}

// The last mode (B = 1) on MFMA:
//   out[a][p] = sum_q in[a][q] F[q][p]
// (a contraction by F_k with P = c_k, or with ftrans an expansion by F_k,
// F[q][p] = F_k[p][q] and P = n_k).
// A block keeps a slice of up to 96 columns of F (every q, zero padded) in
// LDS, read once, and is persistent over row tiles: each of its 8 waves forms
// a 32-row x 32-column tile per 32-column group with v_mfma_f32_32x32x2f32,
// the A operand from `in` (lane l: row a0 + l%32) and the B operand from the
// LDS slice (lane l: column p0 + l%32), so an accumulator register holds 32
// consecutive columns of one row and the stores are coalesced.  Per 32-q step
// a lane reads 16 consecutive q of its row (four 16-byte buffer loads; the
// half-waves take q0..q0+15 and q0+16..q0+31, which pairs the two k rows of
// the MFMA with the same q in both operands); the next step's loads are in
// flight while the current one is multiplied.  Rows past A read zero through
// the buffer range check; q past Q (the next row's values) is dropped.
constexpr int kLastWaves = 8;
constexpr int kLastQC = 32;     // q per step
constexpr int kLastMaxPT = 3;   // 32-column groups per block (96 columns)
constexpr int kLastLdf = 32 * kLastMaxPT + 2;  // LDS row stride: half-waves on disjoint banks

template <typename TOut>
__global__ __launch_bounds__(64 * kLastWaves) void mode_last_mfma_kernel(const ModeMfma m) {
  extern __shared__ float sL[];   // [Qp][kLastLdf]
  const int tid = threadIdx.x;
  const int p0 = blockIdx.y * 32 * kLastMaxPT;
  const int npt = min(kLastMaxPT, (int)((m.P - p0 + 31) / 32));
  const int nsteps = (int)((m.Q + kLastQC - 1) / kLastQC);
  const int Qp = nsteps * kLastQC;
  for (int e = tid; e < Qp * 32 * kLastMaxPT; e += 64 * kLastWaves) {
    const int q = e / (32 * kLastMaxPT), pp = e - q * (32 * kLastMaxPT);
    const int p = p0 + pp;
    float f = 0.0f;
    if (q < m.Q && p < m.P) f = m.ftrans ? m.F[(int64_t)p * m.Q + q] : m.F[(int64_t)q * m.P + p];
    sL[q * kLastLdf + pp] = f;
  }
  __syncthreads();
  const int lane = tid & 63, kh = lane >> 5, l32 = lane & 31;
  const int wave = tid >> 6;
  const int64_t tiles = (m.A + 31) / 32;
  // the launcher keeps A Q 4 below 2^31
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(m.in), (short)0, (int)(m.A * m.Q * 4), kRsrcWord3);
  TOut* out = static_cast<TOut*>(m.out);
  for (int64_t tile = (int64_t)blockIdx.x * kLastWaves + wave; tile < tiles;
       tile += (int64_t)gridDim.x * kLastWaves) {
    const int64_t row = tile * 32 + l32;
    const bool rok = row < m.A;
    auto load = [&](int step, floatx4 (&b)[4]) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = step * kLastQC + 16 * kh + 4 * u;
        const uint32_t off = (rok && step < nsteps) ? (uint32_t)((row * m.Q + q) * 4) : 0x80000000u;
        b[u] = __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
      }
    };
    floatx16 acc[kLastMaxPT];
#pragma unroll
    for (int t = 0; t < kLastMaxPT; ++t) acc[t] = floatx16{};
    auto compute = [&](int step, const floatx4 (&b)[4]) {
      const bool tail = (step + 1) * kLastQC > m.Q;   // wave-uniform
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int ql = step * kLastQC + 16 * kh + 4 * u + c;
          float xv = b[u][c];
          if (tail && ql >= m.Q) xv = 0.0f;
          const float* fr = sL + ql * kLastLdf + l32;
#pragma unroll
          for (int t = 0; t < kLastMaxPT; ++t)
            if (t < npt) acc[t] = mfma32(xv, fr[32 * t], acc[t]);
        }
      }
    };
    floatx4 bufA[4], bufB[4];
    load(0, bufA);
    for (int s = 0; s < nsteps; s += 2) {
      load(s + 1, bufB);
      __builtin_amdgcn_sched_barrier(0);
      compute(s, bufA);
      load(s + 2, bufA);
      __builtin_amdgcn_sched_barrier(0);
      if (s + 1 < nsteps) compute(s + 1, bufB);
    }
    // acc[t] register v: row tile*32 + 8 (v/4) + 4 kh + v%4, column p0 + 32 t + l32
#pragma unroll
    for (int t = 0; t < kLastMaxPT; ++t) {
      const int p = p0 + 32 * t + l32;
      if (t >= npt || p >= m.P) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t r = tile * 32 + 8 * (v >> 2) + 4 * kh + (v & 3);
        if (r < m.A) out[r * m.P + p] = (TOut)acc[t][v];
      }
    }
  }
}

}  // namespace

bool mode_mfma_supported(int64_t Q, int64_t B, int32_t P) {
  // F^T staged in LDS (at most 64 KB); one (Q x B) slab addressed in 31 bits
  return P >= 1 && P <= 32 && Q >= 1 && Q <= 512 && B >= 1 && Q * B * 4 < (int64_t(1) << 31);
}

template <int VEC>
hipError_t launch_mode_vec(const ModeMfma& m, int out_dt, size_t lds, hipStream_t st) {
  const int64_t units = m.A * ((m.B + 32 * VEC - 1) / (32 * VEC));
  const dim3 grid((unsigned)ceil_div(units, kWaves));
  if (out_dt == TK_F64)
    hipLaunchKernelGGL((mode_mfma_f32_kernel<double, VEC>), grid, dim3(256), lds, st, m);
  else
    hipLaunchKernelGGL((mode_mfma_f32_kernel<float, VEC>), grid, dim3(256), lds, st, m);
  return hipGetLastError();
}

hipError_t launch_mode_mfma_f32(const ModeMfma& m, int out_dt, hipStream_t st) {
  if (m.A * m.B == 0) return hipSuccess;
  const int64_t Qp = (m.Q + 2 * kKB - 1) / (2 * kKB) * 2 * kKB;
  const size_t lds = (size_t)Qp * 32 * sizeof(float);
  // the widest column block that still gives about eight waves per CU
  const int64_t want = 2048;
  const int64_t u4 = m.A * ((m.B + 127) / 128), u2 = m.A * ((m.B + 63) / 64);
  if (u4 >= want) return launch_mode_vec<4>(m, out_dt, lds, st);
  if (u2 >= want) return launch_mode_vec<2>(m, out_dt, lds, st);
  return launch_mode_vec<1>(m, out_dt, lds, st);
}

}  // namespace tk

namespace tk {

bool mode_last_mfma_supported(int64_t A, int64_t Q, int32_t P) {
  // the F slice of every q in LDS (at most 150.5 KB); one buffer range for `in`
  // (the launcher splits the rows so that each launch's input stays within 2^31 bytes)
  return P >= 1 && P <= 4096 && Q >= 1 && Q <= 384 && A >= 1;
}

namespace {
constexpr int kPairBlocks = 2048;

// sums of (X - Xh)^2 and X^2 (FP64) per block; with D, also D = s (X - Xh)
// (D may alias X or Xh: every entry is read and written by one thread)
__global__ __launch_bounds__(256) void resid_pair_kernel(const float* X, const float* Xh, float* D,
                                                         const double* scale, double smul, int64_t n,
                                                         double* __restrict__ partials) {
  __shared__ double red[2][4];
  const int tid = threadIdx.x;
  const float ds = (float)(smul * (scale ? *scale : 1.0));
  double r2 = 0.0, x2 = 0.0;
  const int64_t n4 = n / 4;
  const float4* X4 = reinterpret_cast<const float4*>(X);
  const float4* H4 = reinterpret_cast<const float4*>(Xh);
  float4* D4 = reinterpret_cast<float4*>(D);
  for (int64_t g = (int64_t)blockIdx.x * 256 + tid; g < n4; g += (int64_t)gridDim.x * 256) {
    const float4 x = X4[g], h = H4[g];
    const double d0 = (double)x.x - h.x, d1 = (double)x.y - h.y, d2 = (double)x.z - h.z,
                 d3 = (double)x.w - h.w;
    r2 = fma(d0, d0, fma(d1, d1, fma(d2, d2, fma(d3, d3, r2))));
    x2 = fma((double)x.x, x.x, fma((double)x.y, x.y, fma((double)x.z, x.z, fma((double)x.w, x.w, x2))));
    if (D) D4[g] = make_float4(ds * (float)d0, ds * (float)d1, ds * (float)d2, ds * (float)d3);
  }
  if (blockIdx.x == 0 && tid < (int)(n - 4 * n4)) {
    const double x = X[4 * n4 + tid], d = x - (double)Xh[4 * n4 + tid];
    r2 = fma(d, d, r2);
    x2 = fma(x, x, x2);
    if (D) D[4 * n4 + tid] = ds * (float)d;
  }
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
    partials[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    partials[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

__global__ __launch_bounds__(256) void pair_sum_kernel(const double* partials, int nb, double* out) {
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int i = tid; i < nb; i += 256) {
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

int64_t resid_pair_blocks(int64_t n) {
  return std::max<int64_t>(1, std::min<int64_t>(kPairBlocks, ceil_div(n / 4, 256)));
}

hipError_t launch_resid_pair_f32(const float* X, const float* Xh, int64_t n, float* D, const double* scale,
                                 double smul, double* partials, double* resid2, hipStream_t st) {
  const int nb = (int)resid_pair_blocks(n);
  hipLaunchKernelGGL(resid_pair_kernel, dim3(nb), dim3(256), 0, st, X, Xh, D, scale, smul, n, partials);
  if (resid2) hipLaunchKernelGGL(pair_sum_kernel, dim3(1), dim3(256), 0, st, partials, nb, resid2);
  return hipGetLastError();
}

hipError_t launch_pair_sum(const double* partials, int64_t npairs, double* resid2, hipStream_t st) {
  hipLaunchKernelGGL(pair_sum_kernel, dim3(1), dim3(256), 0, st, partials, (int)npairs, resid2);
  return hipGetLastError();
}

hipError_t launch_mode_last_mfma_f32(const ModeMfma& m, int out_dt, hipStream_t st) {
  if (m.A == 0) return hipSuccess;
  const int groups = (m.P + 32 * kLastMaxPT - 1) / (32 * kLastMaxPT);
  const int64_t Qp = (m.Q + kLastQC - 1) / kLastQC * kLastQC;
  const size_t lds = (size_t)Qp * kLastLdf * sizeof(float);
  // rows per launch: the input's byte offsets (buffer range) stay below 2^31
  const int64_t chunk = ((int64_t(1) << 31) - 1) / (m.Q * 4) / 32 * 32;
  for (int64_t a0 = 0; a0 < m.A; a0 += chunk) {
    ModeMfma c = m;
    c.A = std::min<int64_t>(chunk, m.A - a0);
    c.in = m.in + a0 * m.Q;
    c.out = out_dt == TK_F64 ? (void*)(static_cast<double*>(m.out) + a0 * m.P)
                             : (void*)(static_cast<float*>(m.out) + a0 * m.P);
    // one resident block per CU (the slice takes most of the LDS), persistent
    const int64_t tiles = (c.A + 31) / 32;
    const int64_t per_group =
        std::max<int64_t>(1, std::min<int64_t>(ceil_div(tiles, kLastWaves), 256 / groups));
    const dim3 grid((unsigned)per_group, (unsigned)groups);
    if (out_dt == TK_F64)
      hipLaunchKernelGGL((mode_last_mfma_kernel<double>), grid, dim3(64 * kLastWaves), lds, st, c);
    else
      hipLaunchKernelGGL((mode_last_mfma_kernel<float>), grid, dim3(64 * kLastWaves), lds, st, c);
  }
  return hipGetLastError();
}

}  // namespace tk
