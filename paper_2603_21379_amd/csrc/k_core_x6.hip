// Streaming pass of the core projection (Algorithm 1, core step) for FP32
// tensors, with the stage-1 products on BF16 matrix cores at FP32 accuracy:
//   T[a] = F_I^T X[a] F_J        (X[a]: n_I x n_J, c_I, c_J <= 32)
//
// FP32 arithmetic from BF16 pieces: every FP32 operand x is split into
// x = h + m + l, h = rne(x), m = rne(x - h), l = rne(x - h - m) (each a BF16
// value, each difference exact in FP32), 24 significant bits in all.  Of the
// nine piece products the six with rank sum <= 4 are kept (hh, hm, mh, hl, mm,
// lh); the three dropped are ~2^-27 relative, below FP32 rounding.  Each BF16
// x BF16 product is exact in the FP32 accumulator, so the stage-1 sum has the
// accuracy of an FP32 MFMA sum.  Six v_mfma_f32_32x32x16_bf16 cost 2.7x less
// than the FP32 MFMA work they replace.  (Values beyond 3.3e38 in magnitude
// would round to infinity in h and are not supported.)
//
// Stage 1 contracts the rows: E^T[b][j] = sum_i X[a][i][b] F_I[i][j].  X is
// the A operand with the rows as K: lane l loads the float4
// X[a][16 ks + 8 (l/32) + r][128 h + 4 (l%32) .. +3] for r = 0..7 (each load
// covers two 512-byte row segments), and component c of the eight float4s,
// split into BF16 pieces, is the A operand (K slots 8 (l/32) + r) of the
// tile whose row m stands for column b = 128 h + 4 m + c.  The F_I pieces
// (B operand, K <-> the same rows, N <-> j) come from LDS.  After the last
// row step of a column block, register v of accumulator c holds E^T at
// m = 8 (v/4) + 4 (l/32) + v%4, j = l%32: the A operand of a K = 2 FP32 MFMA
// over the column pair {b(m), b(m + 4)} of stage 2,
//   T[j][j'] += sum_b E[j][b] F_J[b][j'],
// with F_J read from LDS in FP32.  Waves are persistent over (slab, column
// block, row step) units, NBUF units of loads in flight; rows past n_I and
// slabs past the end read zero through the buffer range check, lanes whose
// columns start past n_J point outside the range.
#include <stdlib.h>

#include "tk_kernels.hpp"

namespace tk {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kRsrcWord3 = 0x00020000;
constexpr int kCols = 128;      // columns of a block (32 lanes x float4)
constexpr int kRowStep = 16;    // rows per unit (K of one MFMA)

__device__ __forceinline__ floatx16 mma_bf16(bf16x8 a, bf16x8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx16 mma_f32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// x (8 FP32 values as two float4) -> BF16 pieces h, m, l
__device__ __forceinline__ void split3(const floatx4 x0, const floatx4 x1, bf16x8& h, bf16x8& m,
                                       bf16x8& l) {
  uintx4 hh, mm, ll;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const floatx2 v = {w < 2 ? x0[2 * w] : x1[2 * w - 4], w < 2 ? x0[2 * w + 1] : x1[2 * w - 3]};
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

struct Cur {
  int slab, h, ks;   // slab = -1 past the end
};

template <int NBUF>
__global__ __launch_bounds__(256, 2) void fused2x6_kernel(const CoreFused2 p) {
  extern __shared__ uint32_t lds[];
  const int nKS = (p.nI + kRowStep - 1) / kRowStep, nH = (p.nJ + kCols - 1) / kCols;
  const int tid = threadIdx.x, lane = tid & 63, kh = lane >> 5, l32 = lane & 31;
  // F_I pieces: sFI[ks][piece][lane] as BF16x8 (4 dwords):
  //   F_I[16 ks + 8 kh + v][l32], v = 0..7
  uint32_t* sFI = lds;
  // F_J: sFJ[b][32] in FP32, rows zero padded to whole column blocks
  float* sFJ = reinterpret_cast<float*>(lds + nKS * 3 * 64 * 4);
  for (int e = tid; e < nKS * 64; e += blockDim.x) {
    const int ks = e >> 6, ln = e & 63, g = ln >> 5, j = ln & 31;
    floatx4 x0, x1;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int i = kRowStep * ks + 8 * g + v;
      const float f = (i < p.nI && j < p.cI) ? p.FI[i * p.cI + j] : 0.0f;
      if (v < 4) x0[v] = f; else x1[v - 4] = f;
    }
    bf16x8 h, m, l;
    split3(x0, x1, h, m, l);
    const uintx4 uh = __builtin_bit_cast(uintx4, h), um = __builtin_bit_cast(uintx4, m),
                 ul = __builtin_bit_cast(uintx4, l);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      sFI[((ks * 3 + 0) * 64 + ln) * 4 + w] = uh[w];
      sFI[((ks * 3 + 1) * 64 + ln) * 4 + w] = um[w];
      sFI[((ks * 3 + 2) * 64 + ln) * 4 + w] = ul[w];
    }
  }
  for (int e = tid; e < nH * kCols * 32; e += blockDim.x) {
    const int b = e >> 5, j = e & 31;
    sFJ[e] = (b < p.nJ && j < p.cJ) ? p.FJ[b * p.cJ + j] : 0.0f;
  }
  __syncthreads();

  const int gwave = __builtin_amdgcn_readfirstlane((int)blockIdx.x * kWaves + (tid >> 6));
  const int nwaves = p.nwaves;
  const int A32 = (int)p.A;
  if (gwave >= A32) return;  // no barrier follows

  const uint32_t slab_bytes = (uint32_t)(p.nI * p.nJ * 4);

  auto uni = [](Cur c) {
    c.slab = __builtin_amdgcn_readfirstlane(c.slab);
    c.h = __builtin_amdgcn_readfirstlane(c.h);
    c.ks = __builtin_amdgcn_readfirstlane(c.ks);
    return c;
  };
  auto advance = [&](Cur c) {
    c = uni(c);
    if (c.slab < 0) return c;
    if (++c.ks >= nKS) {
      c.ks = 0;
      if (++c.h >= nH) {
        c.h = 0;
        c.slab = c.slab + nwaves < A32 ? c.slab + nwaves : -1;
      }
    }
    return uni(c);
  };
  // one unit: rows 16 ks + 8 kh + r (r = 0..7), columns 128 h + 4 l32 .. +3
  auto load_unit = [&](Cur c, floatx4 (&buf)[8]) {
    c = uni(c);
    const bool live = c.slab >= 0;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(p.X + (live ? (int64_t)c.slab * p.nI * p.nJ : 0)), (short)0,
        live ? (int)slab_bytes : 0, kRsrcWord3);
    const int col = kCols * c.h + 4 * l32;
    const int row0 = kRowStep * c.ks + 8 * kh;
    const uint32_t off0 = col < p.nJ ? (uint32_t)(row0 * p.nJ + col) * 4u : 0x80000000u;
    const uint32_t row_bytes = (uint32_t)p.nJ * 4u;
#pragma unroll
    for (int r = 0; r < 8; ++r) buf[r] = __builtin_amdgcn_raw_buffer_load_b128(rs, off0 + r * row_bytes, 0, 2);
  };

  floatx16 acc[4], tacc;
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = floatx16{};
  tacc = floatx16{};

  auto compute = [&](Cur c, floatx4 (&buf)[8]) {
    c = uni(c);
    const uint32_t* fi = sFI + ((c.ks * 3) * 64 + lane) * 4;
    bf16x8 bp[3];
#pragma unroll
    for (int pc = 0; pc < 3; ++pc)
      bp[pc] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uintx4*>(fi + pc * 64 * 4));
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      const floatx4 x0 = {buf[0][cc], buf[1][cc], buf[2][cc], buf[3][cc]};
      const floatx4 x1 = {buf[4][cc], buf[5][cc], buf[6][cc], buf[7][cc]};
      bf16x8 h, m, l;
      split3(x0, x1, h, m, l);
      acc[cc] = mma_bf16(h, bp[0], acc[cc]);
      acc[cc] = mma_bf16(h, bp[1], acc[cc]);
      acc[cc] = mma_bf16(m, bp[0], acc[cc]);
      acc[cc] = mma_bf16(h, bp[2], acc[cc]);
      acc[cc] = mma_bf16(m, bp[1], acc[cc]);
      acc[cc] = mma_bf16(l, bp[0], acc[cc]);
    }
    if (c.ks != nKS - 1) return;
    // column block complete: tacc += E(block) F_J(block)
    const float* fj = sFJ + (kCols * c.h + 16 * kh) * 32 + l32;
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        // column b = 128 h + 4 (8 (v/4) + 4 kh + v%4) + cc
        const float g = fj[(4 * (8 * (v >> 2) + (v & 3)) + cc) * 32];
        tacc = mma_f32(acc[cc][v], g, tacc);
      }
      acc[cc] = floatx16{};
    }
    if (c.h != nH - 1) return;
    // slab complete: lane holds T[8 (v/4) + 4 kh + v%4][l32]
    const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(
        p.T + (int64_t)c.slab * p.cI * p.cJ, (short)0, p.cI * p.cJ * 4, kRsrcWord3);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int j = 8 * (v >> 2) + 4 * kh + (v & 3);
      const uint32_t off = (j < p.cI && l32 < p.cJ) ? (uint32_t)((j * p.cJ + l32) * 4) : 0x80000000u;
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(tacc[v]), ro, off, 0, kOutStorePolicy);
    }
    tacc = floatx16{};
  };

  // The wave's units (its slabs gwave, gwave + nwaves, ... times nH nKS) run
  // in full groups of NBUF with no exit test inside (an exit test there would
  // leave loads of skipped units pending at the loop head and force a wait
  // for every load in flight); the tail computes the units already in flight.
  const int units = ((A32 - 1 - gwave) / nwaves + 1) * nH * nKS;
  floatx4 buf[NBUF][8];
  Cur cc[NBUF];
  cc[0] = Cur{gwave, 0, 0};
  load_unit(cc[0], buf[0]);
  Cur last = cc[0];
#pragma unroll
  for (int s = 1; s < NBUF - 1; ++s) {
    last = advance(last);
    cc[s] = last;
    load_unit(cc[s], buf[s]);
  }
  int left = units;
  for (; left >= NBUF; left -= NBUF) {
#pragma unroll
    for (int s = 0; s < NBUF; ++s) {
      const int lb = (s + NBUF - 1) % NBUF;
      last = advance(last);
      cc[lb] = last;
      load_unit(cc[lb], buf[lb]);
      __builtin_amdgcn_sched_barrier(0);
      compute(cc[s], buf[s]);
    }
  }
#pragma unroll
  for (int s = 0; s < NBUF - 1; ++s)
    if (s < left) compute(cc[s], buf[s]);
}

}  // namespace

size_t fused2x6_lds_bytes(int nI, int nJ) {
  const int nKS = (nI + kRowStep - 1) / kRowStep, nH = (nJ + kCols - 1) / kCols;
  return (size_t)nKS * 3 * 64 * 16 + (size_t)nH * kCols * 32 * 4;
}

bool fused2x6_supported(int dtype, int order, const int64_t* dims, const int32_t* cols) {
  if (dtype != TK_F32 || order < 3) return false;
  const int64_t nI = dims[order - 2], nJ = dims[order - 1];
  int64_t A = 1;
  for (int k = 0; k < order - 2; ++k) A *= dims[k];
  if (nI < 64 || nJ < 64 || nJ % 4 != 0) return false;
  if (A < 256 || A >= (int64_t(1) << 31) || (nI + kRowStep) * nJ * 4 >= (int64_t(1) << 31)) return false;
  return cols[order - 2] <= 32 && cols[order - 1] <= 32 &&
         fused2x6_lds_bytes((int)nI, (int)nJ) <= 80 * 1024;
}

template <int NBUF>
hipError_t launch_x6_depth(CoreFused2 p, hipStream_t st) {
  const size_t lds = fused2x6_lds_bytes(p.nI, p.nJ);
  auto kern = fused2x6_kernel<NBUF>;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(p.A, kWaves), (int64_t)per_cu * cus));
  p.nwaves = (int32_t)(blocks * kWaves);
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), lds, st, p);
  return hipGetLastError();
}

// two units of loads in the register pipeline (three spill)
hipError_t launch_fused2x6(const CoreFused2& p, hipStream_t st) { return launch_x6_depth<2>(p, st); }

}  // namespace tk
