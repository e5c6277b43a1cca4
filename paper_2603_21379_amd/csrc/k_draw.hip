// Device-side seeded draw of the sampled sketches (the sampling step of
// Algorithm 1, Section 3.1: fiber indices uniform without repetition and a
// Gaussian test matrix), from one counter-based stream so the draw needs no
// host generation or upload and any process can reproduce it.
//
// Stream: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011) keyed by
// (seed, unit), unit = the sketch's position in the call.
// * indices: Floyd's algorithm.  Step i = 0..s-1 considers j = N - s + i,
//   draws t = high 64 bits of w (j + 1), w = word 0 of the block at counter
//   (i, 0, 0, 0), and takes t if it is new, else j.  The draws are made by
//   all threads at once; one thread then walks the steps against a hash set
//   in LDS, and the workgroup sorts the result (bitonic, in LDS).
// * Omega[t][e]: the block at counter (t ell + e, 1, 0, 0) gives
//   u1 = ((w0 >> 11) + 1) 2^-53, u2 = (w1 >> 11) 2^-53 and the normal
//   sqrt(-2 ln u1) cos(2 pi u2) (FP64, stored as FP32 or FP64).
#include "tk_kernels.hpp"

namespace tk {
namespace {

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
constexpr int kHashBits = 13;               // 8192-slot table for s <= 4096
constexpr int64_t kEmpty = -1;

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

__global__ __launch_bounds__(256) void draw_indices_kernel(const DrawBatch b) {
  extern __shared__ int64_t dl[];
  const DrawUnit& U = b.u[blockIdx.x];
  const int s = U.s, tid = threadIdx.x;
  if (s == 0) return;
  int P = 1;
  while (P < s) P <<= 1;
  int64_t* sel = dl;                 // [P]: draws, then the chosen set, then sorted
  int64_t* tab = dl + P;             // [1 << kHashBits]: hash set of chosen indices
  const uint64_t key0 = b.seed, key1 = (uint64_t)blockIdx.x;
  for (int i = tid; i < P; i += 256) {
    if (i < s) {
      const uint64_t w = philox4x64_10((uint64_t)i, 0, 0, 0, key0, key1).w[0];
      const uint64_t j = (uint64_t)(U.ncols - s + i);
      sel[i] = (int64_t)__umul64hi(w, j + 1);   // uniform on [0, j]
    } else {
      sel[i] = INT64_MAX;                       // padding sorts last
    }
  }
  for (int i = tid; i < (1 << kHashBits); i += 256) tab[i] = kEmpty;
  __syncthreads();
  if (tid == 0) {
    // Floyd: take t unless already chosen, then take j (never chosen before)
    for (int i = 0; i < s; ++i) {
      const int64_t t = sel[i];
      uint32_t h = (uint32_t)(((uint64_t)t * kW0) >> (64 - kHashBits));
      bool found = false;
      while (tab[h] != kEmpty) {
        if (tab[h] == t) { found = true; break; }
        h = (h + 1) & ((1u << kHashBits) - 1);
      }
      int64_t v = t;
      if (found) {
        v = U.ncols - s + i;
        h = (uint32_t)(((uint64_t)v * kW0) >> (64 - kHashBits));
        while (tab[h] != kEmpty) h = (h + 1) & ((1u << kHashBits) - 1);
      }
      tab[h] = v;
      sel[i] = v;
    }
  }
  __syncthreads();
  // bitonic sort of sel[0..P) ascending
  for (int k = 2; k <= P; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int i = tid; i < P; i += 256) {
        const int l = i ^ jj;
        if (l > i) {
          const int64_t a = sel[i], c = sel[l];
          const bool up = (i & k) == 0;
          if ((a > c) == up) {
            sel[i] = c;
            sel[l] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < s; i += 256) U.idx[i] = sel[i];
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
  return ((size_t)P + ((size_t)1 << kHashBits)) * sizeof(int64_t);
}

hipError_t launch_draw(const DrawBatch& b, int smax, hipStream_t st) {
  if (b.count == 0) return hipSuccess;
  hipLaunchKernelGGL(draw_indices_kernel, dim3(b.count), dim3(256), draw_indices_lds_bytes(smax), st, b);
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
