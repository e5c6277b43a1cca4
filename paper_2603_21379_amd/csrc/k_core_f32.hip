// Streaming pass of the core projection for FP32 tensors on MFMA: the two
// trailing modes of X are contracted in one read of the tensor.
//
// X is viewed as A slabs X[a] of n_I x n_J (n_J contiguous).  For each slab
//   T[a] = F_I^T X[a] F_J        (c_I x c_J, c_I, c_J <= 32)
// which is two TTMs of the core step of Algorithm 1 (the remaining modes are
// contracted afterwards from T, 1/(n_I n_J / c_I c_J) of the data).
//
// One wavefront owns a slab at a time (persistent over slabs).  Stage 1 uses
// v_mfma_f32_32x32x2f32 with X as the A operand: lane l loads the float4
// X[a][i0 + l/32][b0 + 4 (l%32) .. +3] (two 512-byte row segments per load,
// fully coalesced) and component c of it is the A tile whose row m stands for
// column b = b0 + 4 m + c; the B operand is F_I (rows i0, i0+1) from LDS.  The
// four accumulators hold D^T[b][j] = sum_i X[a][i][b] F_I[i][j] for 128
// columns b.  Stage 2 contracts b with F_J: register v of an accumulator holds
// rows m = 8 (v/4) + 4 (l/32) + v%4 of D^T for column j = l%32, which is
// exactly the A operand of a K = 2 MFMA over the column pair
// {b(m), b(m + 4)}, so the stage-1 result feeds stage 2 without any data
// movement; only F_J[b][j'] is read from LDS.  Loads of the next batch of 8
// row pairs are issued before the current batch is multiplied.
#include <stdio.h>
#include <stdlib.h>

#include "tk_kernels.hpp"

namespace tk {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kCols = 128;    // columns of X per lane group (32 lanes x float4)
constexpr int kWaves = 4;     // waves per workgroup

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

struct Cursor {
  int slab;       // slab index, or -1 past the end
  int h;          // column block
  int kb;         // first row pair of the batch
};

// The cursor is the same for all lanes of a wave; saying so keeps its
// arithmetic, the buffer descriptors and the branches on it scalar.
__device__ __forceinline__ Cursor uniform(Cursor c) {
  c.slab = __builtin_amdgcn_readfirstlane(c.slab);
  c.h = __builtin_amdgcn_readfirstlane(c.h);
  c.kb = __builtin_amdgcn_readfirstlane(c.kb);
  return c;
}

// Buffer descriptor word 3 for raw (untyped) buffer access on CDNA.
constexpr int kRsrcWord3 = 0x00020000;

// KB row pairs per batch, NBUF rotating batch buffers (NBUF - 1 batches in
// flight while one is multiplied), NT: non-temporal (streaming) loads, MINB:
// workgroups per CU the register budget is sized for (2: 256 registers per
// lane, 1: 512).
//
// X is read with raw buffer loads over one slab: rows past n_I, the column
// tail past n_J and slabs past the end fall outside the descriptor's range
// and read as zero in hardware, so the loop has no per-element bounds
// branches.  The LDS copies of F_I and F_J are zero padded to whole batches
// and column blocks for the same reason.
template <int KB, int NBUF, bool NT, int MINB>
__global__ __launch_bounds__(256, MINB) void fused2_f32_kernel(const CoreFused2 p) {
  extern __shared__ float lds[];
  const int nK = (p.nI + 1) / 2;                // row pairs per column block
  const int nB = (nK + KB - 1) / KB;            // batches per column block
  const int nH = (p.nJ + kCols - 1) / kCols;    // column blocks per slab
  const int rowsI = nB * KB * 2, rowsJ = nH * kCols;
  float* sFI = lds;                 // [rowsI][32], zero padded
  float* sFJ = lds + rowsI * 32;    // [rowsJ][32], zero padded
  for (int e = threadIdx.x; e < rowsI * 32; e += blockDim.x) {
    const int i = e >> 5, j = e & 31;
    sFI[e] = (i < p.nI && j < p.cI) ? p.FI[i * p.cI + j] : 0.0f;
  }
  for (int e = threadIdx.x; e < rowsJ * 32; e += blockDim.x) {
    const int b = e >> 5, j = e & 31;
    sFJ[e] = (b < p.nJ && j < p.cJ) ? p.FJ[b * p.cJ + j] : 0.0f;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, kh = lane >> 5, l32 = lane & 31;
  const int gwave = __builtin_amdgcn_readfirstlane((int)blockIdx.x * kWaves + (threadIdx.x >> 6));
  const int nwaves = p.nwaves;  // a kernel argument keeps the cursor math scalar
  const int64_t nIJ = (int64_t)p.nI * p.nJ;
  const uint32_t slab_bytes = (uint32_t)(nIJ * 4);
  const uint32_t row_pair_bytes = (uint32_t)(2 * p.nJ * 4);

  auto load_batch = [&](Cursor c, floatx4 (&buf)[KB]) {
    c = uniform(c);
    const bool live = c.slab >= 0;
    const float* base = p.X + (live ? (int64_t)c.slab * nIJ : 0);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(base), (short)0, live ? (int)slab_bytes : 0, kRsrcWord3);
    const int b = c.h * kCols + 4 * l32;
    // lanes past the column tail point far outside the range: they read zero
    const uint32_t off0 = b < p.nJ ? (uint32_t)(((2 * c.kb + kh) * p.nJ + b) * 4) : 0x80000000u;
#pragma unroll
    for (int u = 0; u < KB; ++u)
      buf[u] = __builtin_amdgcn_raw_buffer_load_b128(rs, off0 + u * row_pair_bytes, 0, NT ? 2 : 0);
  };
  const int A32 = (int)p.A;  // < 2^31, checked on the host
  auto advance = [&](Cursor c) {
    c = uniform(c);
    if (c.slab < 0) return c;
    c.kb += KB;
    if (c.kb >= nB * KB) {
      c.kb = 0;
      if (++c.h >= nH) {
        c.h = 0;
        c.slab = c.slab + nwaves < A32 ? c.slab + nwaves : -1;
      }
    }
    return uniform(c);
  };

  if (gwave >= A32) return;  // no barrier follows
  floatx16 acc[4], tacc;
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = floatx16{};
  tacc = floatx16{};

  // one batch of KB row pairs (+ stage 2 / slab output when a block or slab ends)
  auto compute = [&](Cursor c, const floatx4 (&buf)[KB]) {
    c = uniform(c);
    const float* fi = sFI + (2 * c.kb + kh) * 32 + l32;
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const float f = fi[u * 64];
      acc[0] = mfma32(buf[u][0], f, acc[0]);
      acc[1] = mfma32(buf[u][1], f, acc[1]);
      acc[2] = mfma32(buf[u][2], f, acc[2]);
      acc[3] = mfma32(buf[u][3], f, acc[3]);
    }
    if (c.kb + KB >= nB * KB) {
      // column block complete: tacc += D^T(block)^T F_J(block)
      const float* fj = sFJ + (c.h * kCols + 16 * kh) * 32 + l32;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          // column b = h*128 + 4 (8 (v/4) + 4 kh + v%4) + q
          const float g = fj[(4 * (8 * (v >> 2) + (v & 3)) + q) * 32];
          tacc = mfma32(acc[q][v], g, tacc);
        }
        acc[q] = floatx16{};
      }
      if (c.h == nH - 1) {
        // slab complete: T[a][j][j'] with j' = l32, j = 8 (v/4) + 4 kh + v%4
        const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(
            p.T + (int64_t)c.slab * p.cI * p.cJ, (short)0, p.cI * p.cJ * 4, kRsrcWord3);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int j = 8 * (v >> 2) + 4 * kh + (v & 3);
          const uint32_t off = (j < p.cI && l32 < p.cJ) ? (uint32_t)((j * p.cJ + l32) * 4) : 0x80000000u;
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(tacc[v]), ro, off, 0, kOutStorePolicy);
        }
        tacc = floatx16{};
      }
    }
  };

  // Step t multiplies buffer t % NBUF after issuing the load of step
  // t + NBUF - 1 into buffer (t - 1) % NBUF, which step t - 1 has finished.
  // The wave's batches (its slabs gwave, gwave + nwaves, ... times nH nB) run
  // in full groups of NBUF steps with no exit test inside (an exit test there
  // would leave loads of skipped steps pending at the loop head and force a
  // wait for every load in flight); the tail multiplies the batches already
  // in flight.
  const int steps = ((A32 - 1 - gwave) / nwaves + 1) * nH * nB;
  floatx4 buf[NBUF][KB];
  Cursor cc[NBUF];
  cc[0] = Cursor{gwave, 0, 0};
  load_batch(cc[0], buf[0]);
  Cursor last = cc[0];
#pragma unroll
  for (int s = 1; s < NBUF - 1; ++s) {
    last = advance(last);
    cc[s] = last;
    load_batch(cc[s], buf[s]);
  }
  int left = steps;
  for (; left >= NBUF; left -= NBUF) {
#pragma unroll
    for (int s = 0; s < NBUF; ++s) {
      const int lb = (s + NBUF - 1) % NBUF;
      last = advance(last);
      cc[lb] = last;
      load_batch(cc[lb], buf[lb]);
      // keep these loads ahead of the multiplies below: without the barrier
      // the scheduler sinks them past the MFMAs and nothing is in flight
      __builtin_amdgcn_sched_barrier(0);
      compute(cc[s], buf[s]);
    }
  }
#pragma unroll
  for (int s = 0; s < NBUF - 1; ++s)
    if (s < left) compute(cc[s], buf[s]);
}

}  // namespace

// LDS of the padded factor tables for batch size kb
size_t fused2_lds_bytes(int nI, int nJ, int kb) {
  const int nK = (nI + 1) / 2, nB = (nK + kb - 1) / kb, nH = (nJ + kCols - 1) / kCols;
  return (size_t)(nB * kb * 2 + nH * kCols) * 32 * sizeof(float);
}

bool fused2_supported(int dtype, int order, const int64_t* dims, const int32_t* cols) {
  if (dtype != TK_F32 || order < 3) return false;
  const int64_t nI = dims[order - 2], nJ = dims[order - 1];
  const int cI = cols[order - 2], cJ = cols[order - 1];
  int64_t A = 1;
  for (int k = 0; k < order - 2; ++k) A *= dims[k];
  if (nI > 1024 || nJ > 1024) return false;
  if (A >= (int64_t(1) << 31)) return false;
  return nJ % 4 == 0 && nJ >= 64 && nI >= 2 && cI <= 32 && cJ <= 32 && A >= 256 &&
         fused2_lds_bytes((int)nI, (int)nJ, 16) <= 64 * 1024;
}

int64_t fused2_grid(int64_t A) {
  return std::max<int64_t>(1, std::min<int64_t>(ceil_div(A, kWaves), 1024));
}

// Pipeline: batches of 8 row pairs, two buffers, non-temporal loads of X,
// two workgroups per CU (the fastest of the variants measured at 256^4)
hipError_t launch_fused2_f32(const CoreFused2& pin, hipStream_t st) {
  constexpr int kKB = 8;
  const size_t lds = fused2_lds_bytes(pin.nI, pin.nJ, kKB);
  const dim3 grid((unsigned)fused2_grid(pin.A));
  CoreFused2 p = pin;
  p.nwaves = (int32_t)grid.x * kWaves;
  hipLaunchKernelGGL((fused2_f32_kernel<kKB, 2, true, 2>), grid, dim3(256), lds, st, p);
  return hipGetLastError();
}

}  // namespace tk
