// Factor gradients of the two trailing modes of a Tucker contraction, one
// read of the FP32 tensor, on FP32 matrix cores.
//
// The vector-Jacobian products of the core projection and of the
// reconstruction (the TTM definition of Section 2.2 differentiated) need, for
// every mode k,
//   Fbar_k = (Y x_{j != k} F_j^T)^(k) (C^(k))^T
// with (Y, C) = (X, Gbar) for the core and (H, G) for the reconstruction.
// View Y as A slabs Y[a] of n_I x n_J (the two trailing modes) and let
// K = C x_{j < d-2} F_j (the adjoint expanded in the leading modes,
// K[a] of c_I x c_J).  Then
//   Fbar_J = sum_a Y[a]^T W[a],  W[a] = F_I K[a]     (n_I x c_J)
//   Fbar_I = sum_a Y[a] V[a],    V[a] = F_J K[a]^T   (n_J x c_I)
// so both trailing gradients come from one pass over Y.
//
// A workgroup (four waves) is persistent over slabs.  Per slab it forms W[a]
// and V[a] in LDS (small MFMA products from K[a]), then streams the slab in
// tiles of 32 rows through LDS (the next tile's global loads are in flight
// while the current one is multiplied):
//  * Fbar_J: v_mfma_f32_32x32x2f32 with the tile as the A operand (M = column
//    b, K = row i: lanes read 32 consecutive columns of one row) and W's rows
//    as the B operand;
//  * Fbar_I: the tile as the A operand with M = row i and K = column b (lanes
//    read one column of 32 rows; the LDS row stride n_J + 1 puts those rows
//    in different banks) and V's rows as the B operand.
// Every wave owns the 32-column blocks b = 32 (w + 4 s): it accumulates
// Fbar_J for them outright and Fbar_I over them (its share of the
// contraction).  At the end the four waves' Fbar_I shares are summed in a
// fixed order and each workgroup writes its partial gradients; a second
// kernel sums the partials of all workgroups in FP64, in workgroup order.
#include "tk_kernels.hpp"

namespace tk {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kMaxN = 256;               // n_I, n_J (padded to 32) per kernel
constexpr int kMaxTiles = kMaxN / 32;    // 32-row tiles of a slab, 32-column blocks
constexpr int kSlots = kMaxTiles / kWaves;  // column blocks (and W/V tiles) per wave
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// LDS layout (floats): tile [32][ldx], W [nIp][33], V [nJp][33], K [32][33]
struct Lds {
  float* x;
  float* w;
  float* v;
  float* k;
  int ldx;
};

__device__ __forceinline__ Lds carve(float* base, int nIp, int nJp) {
  Lds s;
  s.ldx = nJp + 1;
  s.x = base;
  s.w = s.x + 32 * s.ldx;
  s.v = s.w + nIp * 33;
  s.k = s.v + nJp * 33;
  return s;
}

__global__ __launch_bounds__(kThreads, 1) void vjp_trail_kernel(const VjpTrail p) {
  extern __shared__ float lds_raw[];
  const int nIp = (p.nI + 31) / 32 * 32, nJp = (p.nJ + 31) / 32 * 32;
  const int nIt = nIp / 32, nJt = nJp / 32;
  const Lds s = carve(lds_raw, nIp, nJp);
  const int tid = threadIdx.x, lane = tid & 63, l32 = lane & 31, kh = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t nIJ = (int64_t)p.nI * p.nJ;

  floatx16 accJ[kSlots], accI[kMaxTiles];
#pragma unroll
  for (int sl = 0; sl < kSlots; ++sl) accJ[sl] = floatx16{};
#pragma unroll
  for (int r = 0; r < kMaxTiles; ++r) accI[r] = floatx16{};

  // this thread's float4s of a 32-row tile: element e = 4 (tid + 256 q),
  // row e / nJp, column e % nJp (n_J % 4 == 0: a float4 never crosses a row)
  const int per = 32 * nJp / (4 * kThreads);   // 1 .. 8
  auto load_tile = [&](int64_t a, int r, floatx4 (&buf)[8]) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(p.X + a * nIJ), (short)0, (int)(nIJ * 4), kRsrcWord3);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = 4 * (tid + kThreads * q);
      const int row = e / nJp, col = e - row * nJp;
      const int gi = 32 * r + row;
      const uint32_t off = (q < per && col < p.nJ && gi < p.nI)
                               ? (uint32_t)(((int64_t)gi * p.nJ + col) * 4) : 0x80000000u;
      buf[q] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 2);
    }
  };
  auto store_tile = [&](const floatx4 (&buf)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q < per) {
        const int e = 4 * (tid + kThreads * q);
        const int row = e / nJp, col = e - row * nJp;
        float* d = s.x + row * s.ldx + col;
        d[0] = buf[q][0];
        d[1] = buf[q][1];
        d[2] = buf[q][2];
        d[3] = buf[q][3];
      }
    }
  };

  floatx4 buf[8];
  int64_t a = blockIdx.x;
  if (a < p.A) load_tile(a, 0, buf);
  for (; a < p.A; a += gridDim.x) {
    // K[a] into LDS (zero padded to 32 x 32)
    __syncthreads();   // the previous slab's last tile and W/V are consumed
    const float* Ka = p.K + a * p.cI * p.cJ;
    for (int e = tid; e < 32 * 32; e += kThreads) {
      const int al = e >> 5, be = e & 31;
      s.k[al * 33 + be] = (al < p.cI && be < p.cJ) ? Ka[al * p.cJ + be] : 0.0f;
    }
    __syncthreads();
    // W = F_I K[a] (tiles of 32 rows i) and V = F_J K[a]^T (tiles of 32 rows
    // b); the A operands are rows of F_I and F_J (lane l: row 32 tile + l%32,
    // columns 2t + l/32), read from global memory (cached: the same every slab)
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      const int ti = wave + kWaves * sl;
      const int i = 32 * ti + l32;
      if (ti < nIt) {
        floatx16 c = floatx16{};
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int al = 2 * t + kh;
          const float f = (i < p.nI && al < p.cI) ? p.FI[(int64_t)i * p.cI + al] : 0.0f;
          c = mfma32(f, s.k[al * 33 + l32], c);
        }
#pragma unroll
        for (int v = 0; v < 16; ++v)
          s.w[(32 * ti + 8 * (v >> 2) + 4 * kh + (v & 3)) * 33 + l32] = c[v];
      }
      if (ti < nJt) {
        floatx16 c = floatx16{};
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int be = 2 * t + kh;
          const float f = (i < p.nJ && be < p.cJ) ? p.FJ[(int64_t)i * p.cJ + be] : 0.0f;
          c = mfma32(f, s.k[l32 * 33 + be], c);
        }
#pragma unroll
        for (int v = 0; v < 16; ++v)
          s.v[(32 * ti + 8 * (v >> 2) + 4 * kh + (v & 3)) * 33 + l32] = c[v];
      }
    }
#pragma unroll
    for (int r = 0; r < kMaxTiles; ++r) {
      if (r < nIt) {
        __syncthreads();   // the previous tile is consumed (and W, V are written)
        store_tile(buf);
        // the next tile (or the next slab's first) in flight during the products
        if (r + 1 < nIt) load_tile(a, r + 1, buf);
        else if (a + gridDim.x < p.A) load_tile(a + gridDim.x, 0, buf);
        __syncthreads();
#pragma unroll
        for (int sl = 0; sl < kSlots; ++sl) {
          const int bt = wave + kWaves * sl;
          if (bt < nJt) {
            const float* xc = s.x + 32 * bt;
            const float* xr = s.x + l32 * s.ldx + 32 * bt;
            const float* wr = s.w + 32 * r * 33 + l32;
            const float* vr = s.v + 32 * bt * 33 + l32;
#pragma unroll 4
            for (int t = 0; t < 16; ++t) {
              const int k = 2 * t + kh;
              // Fbar_J[b][beta] += sum_i Y[i][b] W[i][beta]
              accJ[sl] = mfma32(xc[k * s.ldx + l32], wr[k * 33], accJ[sl]);
              // Fbar_I[i][alpha] += sum_b Y[i][b] V[b][alpha]
              accI[r] = mfma32(xr[k], vr[k * 33], accI[r]);
            }
          }
        }
      }
    }
  }

  // Fbar_J: every column block belongs to one wave; rows b = 32 bt + m,
  // m = 8 (v/4) + 4 kh + v%4, column beta = l%32
  float* pj = p.partJ + (int64_t)blockIdx.x * nJp * 32;
#pragma unroll
  for (int sl = 0; sl < kSlots; ++sl) {
    const int bt = wave + kWaves * sl;
    if (bt < nJt)
#pragma unroll
      for (int v = 0; v < 16; ++v)
        pj[(32 * bt + 8 * (v >> 2) + 4 * kh + (v & 3)) * 32 + l32] = accJ[sl][v];
  }
  // Fbar_I: the four waves' shares of each 32-row tile summed in wave order
  float* pi = p.partI + (int64_t)blockIdx.x * nIp * 32;
  float* red = lds_raw;   // [4][32][32]
#pragma unroll
  for (int r = 0; r < kMaxTiles; ++r) {
    if (r < nIt) {
      __syncthreads();
#pragma unroll
      for (int v = 0; v < 16; ++v)
        red[(wave * 32 + 8 * (v >> 2) + 4 * kh + (v & 3)) * 32 + l32] = accI[r][v];
      __syncthreads();
      for (int e = tid; e < 32 * 32; e += kThreads) {
        float t = red[e];
        for (int w = 1; w < kWaves; ++w) t += red[w * 1024 + e];
        pi[32 * r * 32 + e] = t;
      }
    }
  }
}

// out[i][c] (+)= sum over workgroups of part[wg][i][c], FP64, workgroup order
template <typename TO>
__global__ __launch_bounds__(256) void vjp_trail_reduce_kernel(const float* part, int nwg, int rows_p,
                                                               int rows, int cols, TO* out,
                                                               int accumulate) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int i = e / cols, c = e - i * cols;
  const int64_t stride = (int64_t)rows_p * 32;
  const float* src = part + i * 32 + c;
  double acc = 0.0;
  for (int g = 0; g < nwg; ++g) acc += (double)src[g * stride];
  if (accumulate) acc += (double)out[e];
  out[e] = (TO)acc;
}

}  // namespace

bool vjp_trail_supported(int64_t nI, int64_t nJ, int cI, int cJ, int64_t A) {
  return nI >= 1 && nJ >= 4 && nI <= kMaxN && nJ <= kMaxN && nJ % 4 == 0 && cI <= 32 && cJ <= 32 &&
         nI * nJ * 4 < (int64_t(1) << 31) && A >= 1;
}

int vjp_trail_blocks(int64_t A) { return (int)std::max<int64_t>(1, std::min<int64_t>(A, 256)); }

size_t vjp_trail_lds(int nI, int nJ) {
  const int nIp = (nI + 31) / 32 * 32, nJp = (nJ + 31) / 32 * 32;
  const size_t fl = (size_t)32 * (nJp + 1) + (size_t)nIp * 33 + (size_t)nJp * 33 + 32 * 33;
  return std::max<size_t>(fl, 4 * 32 * 32) * sizeof(float);
}

hipError_t launch_vjp_trail(const VjpTrail& p, void* FbarI, void* FbarJ, int out_dt, int accumulate,
                            hipStream_t st) {
  const int nb = p.nblocks;
  hipLaunchKernelGGL(vjp_trail_kernel, dim3(nb), dim3(kThreads), vjp_trail_lds(p.nI, p.nJ), st, p);
  const int nIp = (p.nI + 31) / 32 * 32, nJp = (p.nJ + 31) / 32 * 32;
  auto reduce = [&](const float* part, int rows_p, int rows, int cols, void* out) {
    if (!out) return;
    const unsigned g = (unsigned)ceil_div((int64_t)rows * cols, 256);
    if (out_dt == TK_F64)
      hipLaunchKernelGGL((vjp_trail_reduce_kernel<double>), dim3(g), dim3(256), 0, st, part, nb, rows_p,
                         rows, cols, static_cast<double*>(out), accumulate);
    else
      hipLaunchKernelGGL((vjp_trail_reduce_kernel<float>), dim3(g), dim3(256), 0, st, part, nb, rows_p,
                         rows, cols, static_cast<float*>(out), accumulate);
  };
  reduce(p.partI, nIp, p.nI, p.cI, FbarI);
  reduce(p.partJ, nJp, p.nJ, p.cJ, FbarJ);
  return hipGetLastError();
}

}  // namespace tk
