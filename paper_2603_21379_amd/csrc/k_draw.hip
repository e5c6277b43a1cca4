// Device-side seeded draw of the sampled sketches (the sampling step of
// Algorithm 1, Section 3.1: fiber indices uniform without repetition and a
// Gaussian test matrix), from one counter-based stream so the draw needs no
// host generation or upload and any process can reproduce it.
//
// Stream: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011) keyed by
// (seed, unit), unit = the sketch's position in the call.
// * indices: Floyd's algorithm.  Step i = 0..s-1 considers j_i = N - s + i,
//   draws t_i = high 64 bits of w (j_i + 1), w = word 0 of the block at
//   counter (i, 0, 0, 0), and takes t_i if it is new, else j_i.  The walk is
//   resolved in parallel: after step i-1 the chosen set is every earlier
//   draw t_k together with j_k for each earlier step k that was rejected, so
//   step i is rejected exactly when t_i repeats an earlier draw or equals j_k
//   of a rejected step k < i (k = t_i - (N - s)).  Repeats are found by
//   sorting the pairs (t_i, i); the second condition is a chain to a strictly
//   earlier step, resolved by pointer jumping in ceil(log2 s) rounds; the
//   chosen values are then sorted (bitonic sorts in LDS, 1024 threads).
// * Omega[t][e]: the block at counter (t ell + e, 1, 0, 0) gives
//   u1 = ((w0 >> 11) + 1) 2^-53, u2 = (w1 >> 11) 2^-53 and the normal
//   sqrt(-2 ln u1) cos(2 pi u2) (FP64, stored as FP32 or FP64).
#include "tk_kernels.hpp"

namespace tk {
namespace {

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
constexpr int kDrawThreads = 1024;

struct Block4 {
  uint64_t w[4];
};

__device__ __forceinline__ Block4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(kM0, c0), lo0 = kM0 * c0;
    const uint64_t hi1 = __umul64hi(kM1, c2), lo1 = kM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += kW0;
    k1 += kW1;
  }
  return Block4{{c0, c1, c2, c3}};
}

// Ascending bitonic sort of n = 2^m keys (with an optional payload that
// breaks ties), by the whole workgroup.
template <bool kPayload>
__device__ void bitonic_sort(int64_t* key, int32_t* pay, int n) {
  const int half = n >> 1;
  for (int k = 2; k <= n; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int q = threadIdx.x; q < half; q += kDrawThreads) {
        const int i = 2 * jj * (q / jj) + q % jj, l = i + jj;
        const int64_t a = key[i], c = key[l];
        bool gt = a > c;
        if (kPayload) gt = gt || (a == c && pay[i] > pay[l]);
        if (gt == ((i & k) == 0)) {
          key[i] = c;
          key[l] = a;
          if (kPayload) {
            const int32_t t = pay[i];
            pay[i] = pay[l];
            pay[l] = t;
          }
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(kDrawThreads) void draw_indices_kernel(const DrawBatch b) {
  extern __shared__ int64_t dl[];
  const DrawUnit& U = b.u[blockIdx.x];
  const int s = U.s, tid = threadIdx.x;
  if (s == 0) return;
  int P = 1;
  while (P < s) P <<= 1;
  int64_t* key = dl;                                        // [P] draws, then the chosen set
  int32_t* pos = reinterpret_cast<int32_t*>(dl + P);        // [P] step of each draw
  int32_t* link = pos + P;                                  // [P] by step: rejected << 16 | (k + 1)
  const int64_t j0 = U.ncols - s;                           // j_i = j0 + i
  const uint64_t key0 = b.seed, key1 = (uint64_t)blockIdx.x;
  for (int i = tid; i < P; i += kDrawThreads) {
    if (i < s) {
      const uint64_t w = philox4x64_10((uint64_t)i, 0, 0, 0, key0, key1).w[0];
      key[i] = (int64_t)__umul64hi(w, (uint64_t)(j0 + i) + 1);   // uniform on [0, j_i]
    } else {
      key[i] = INT64_MAX;                                        // padding sorts last
    }
    pos[i] = i;
  }
  __syncthreads();
  bitonic_sort<true>(key, pos, P);
  // a draw repeats an earlier one iff its predecessor in (t, i) order has the
  // same t; the chain link goes to the step whose j_k equals t_i, if earlier
  for (int p = tid; p < s; p += kDrawThreads) {
    const int64_t t = key[p];
    const int i = pos[p];
    const int rep = (p > 0 && key[p - 1] == t) ? 1 : 0;
    const int k = (t >= j0 && t - j0 < i) ? (int)(t - j0) : -1;
    link[i] = (rep << 16) | (k + 1);
  }
  __syncthreads();
  for (int span = 1; span < s; span <<= 1) {
    int32_t nv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = tid + r * kDrawThreads;
      if (i < s) {
        int32_t v = link[i];
        const int k = (v & 0xFFFF) - 1;
        if (k >= 0) {
          const int32_t w = link[k];
          v = ((v | w) & 0x10000) | (w & 0xFFFF);
        }
        nv[r] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = tid + r * kDrawThreads;
      if (i < s) link[i] = nv[r];
    }
    __syncthreads();
  }
  for (int p = tid; p < s; p += kDrawThreads) {
    const int i = pos[p];
    if (link[i] >> 16) key[p] = j0 + i;
  }
  __syncthreads();
  bitonic_sort<false>(key, nullptr, P);
  for (int i = tid; i < s; i += kDrawThreads) U.idx[i] = key[i];
}

template <typename TO>
__global__ __launch_bounds__(256) void draw_omega_kernel(const DrawBatch b) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= b.omega_begin[b.count]) return;
  int k = 0;
  while (k + 1 < b.count && b.omega_begin[k + 1] <= g) ++k;
  const DrawUnit& U = b.u[k];
  const int64_t e = g - b.omega_begin[k];    // t ell + e of this unit
  const Block4 w = philox4x64_10((uint64_t)e, 1, 0, 0, b.seed, (uint64_t)k);
  const double u1 = (double)((w.w[0] >> 11) + 1) * 0x1.0p-53;
  const double u2 = (double)(w.w[1] >> 11) * 0x1.0p-53;
  const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  static_cast<TO*>(U.omega)[e] = (TO)z;
}

}  // namespace

size_t draw_indices_lds_bytes(int smax) {
  int P = 1;
  while (P < smax) P <<= 1;
  return (size_t)P * (sizeof(int64_t) + 2 * sizeof(int32_t));
}

hipError_t launch_draw(const DrawBatch& b, int smax, hipStream_t st) {
  if (b.count == 0) return hipSuccess;
  hipLaunchKernelGGL(draw_indices_kernel, dim3(b.count), dim3(kDrawThreads), draw_indices_lds_bytes(smax), st, b);
  const int64_t n = b.omega_begin[b.count];
  if (n > 0) {
    const dim3 grid((unsigned)ceil_div(n, 256));
    if (b.omega_dtype == TK_F64)
      hipLaunchKernelGGL(draw_omega_kernel<double>, grid, dim3(256), 0, st, b);
    else
      hipLaunchKernelGGL(draw_omega_kernel<float>, grid, dim3(256), 0, st, b);
  }
  return hipGetLastError();
}

}  // namespace tk
