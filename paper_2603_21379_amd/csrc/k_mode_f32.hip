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
