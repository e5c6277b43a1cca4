// Root transfer tensor of Sub-R-RtL-HT (Algorithm 2, root step; Section 4):
//   B_R(0, j, k) = sum_{a,b} U_l[a][j] X^(l)[a][b] U_r[b][k]
// for an FP32 tensor viewed as the n_l x n_r matrix X^(l) (rows: the modes of
// the root's left child), in one read of X, on FP64 MFMA.
//
// FP64 is needed: B_R feeds the whole format, and at relative errors of the
// order of 1e-5 an FP32 sum over n_r ~ 1e5 terms would move the error of the
// approximation by far more than the FP32 tolerance.  X converts to FP64
// exactly; v_mfma_f64_16x16x4f64 accumulates in FP64.
//
// A workgroup owns 256 rows (four waves of four 16-row tiles) and walks the
// columns in chunks of 64: the chunk of U_r (64 x 16, FP64) is staged in LDS
// once for the workgroup, each lane loads float4s of X (rows 16 t + l%16,
// columns 16 s + 4 (l/16) .. +3; component c is the A operand of one K = 4
// step, K <-> column 16 s + 4 k + c), and the B operand (a row of U_r) is
// shared by the four tiles.  At the end the tile accumulators are the B
// operand of U_l^T T, so T = X U_r never leaves the registers: in the FP64
// 16x16 MFMA result, register v of lane l holds row l/16 + 4 v, column l%16,
// so step v of that product takes K <-> rows k + 4 v of the tile.  The four
// waves' 16 x 16 partials are added in a fixed order and one per workgroup is
// written; two more kernels sum them in fixed order (segments of workgroups,
// then the segments).  U_r of the next chunk is loaded into registers while
// the current chunk is multiplied and every step issues the same loads, so
// the waits count loads.  64-column chunks (16 KB of X in flight per wave,
// two waves per SIMD) against 32 (8 KB, three waves): equal at 18^8, 4 %
// faster at 15^8.
#include "tk_kernels.hpp"

namespace tk {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kRows = 256;        // rows per workgroup
constexpr int kChunk = 64;        // columns per chunk
constexpr int kS = kChunk / 16;   // float4 column groups per lane and chunk
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ doublex4 mma64(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(256) void root_pass_kernel(const RootPass p) {
  __shared__ double sU[2][kChunk][16];        // U_r chunks, double buffered
  __shared__ doublex4 sPart[4][64];           // per-wave partials of U_l^T T
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 4, l16 = lane & 15;
  // workgroup = (row block, column split); the splits of a row block cover
  // consecutive chunk ranges
  const int rb = blockIdx.x / p.qsplit, qs = blockIdx.x - rb * p.qsplit;
  const int64_t row0 = (int64_t)rb * kRows;
  const int64_t rows = min<int64_t>(kRows, p.nL - row0);
  // this workgroup's rows of X; rows past n_l fall outside and read zero
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(p.X + row0 * p.nR), (short)0, (int)(rows * p.nR * 4), kRsrcWord3);
  const int allchunks = (int)((p.nR + kChunk - 1) / kChunk);
  const int per = (allchunks + p.qsplit - 1) / p.qsplit;
  const int c0 = qs * per;
  const int nchunks = max(0, min(allchunks, c0 + per) - c0);

  // U_r rows of chunk ck (64 x 16 FP64, four per thread), loaded into
  // registers one chunk ahead and written to LDS slot ck % 2 after the
  // previous multiply; rows past n_r and chunks past the end read zero
  constexpr int kUPer = kChunk * 16 / 256;
  auto load_u = [&](int ck, double (&u)[kUPer]) {
#pragma unroll
    for (int w = 0; w < kUPer; ++w) {
      const int e = tid + 256 * w, q = e >> 4, k = e & 15;
      const int64_t b = (int64_t)(c0 + ck) * kChunk + q;
      u[w] = (ck < nchunks && b < p.nR && k < p.rR) ? p.UR[b * p.rR + k] : 0.0;
    }
  };
  auto store_u = [&](int slot, const double (&u)[kUPer]) {
#pragma unroll
    for (int w = 0; w < kUPer; ++w) {
      const int e = tid + 256 * w;
      sU[slot][e >> 4][e & 15] = u[w];
    }
  };
  // X of one chunk for this wave: 4 tiles x 4 column groups of float4; chunks
  // past the end read zero (every step issues the same loads, so the waits
  // count loads)
  auto load_x = [&](int ck, floatx4 (&buf)[4][kS]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t r = (int64_t)wv * 64 + 16 * t + l16;
#pragma unroll
      for (int s = 0; s < kS; ++s) {
        const int64_t b = (int64_t)(c0 + ck) * kChunk + 16 * s + 4 * g;
        const uint32_t off =
            (ck < nchunks && r < rows && b < p.nR) ? (uint32_t)((r * p.nR + b) * 4) : 0x80000000u;
        buf[t][s] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
      }
    }
  };
  // columns of a float4 past n_r meet zero rows of U_r; the lanes that hold
  // them read the next row's (finite) entries or zero
  doublex4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = doublex4{};
  auto compute = [&](int slot, const floatx4 (&buf)[4][kS]) {
#pragma unroll
    for (int s = 0; s < kS; ++s)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double u = sU[slot][16 * s + 4 * g + c][l16];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = mma64((double)buf[t][s][c], u, acc[t]);
      }
  };
  // step ck: issue U_r(ck + 1) and X(ck + 1), multiply chunk ck, then put
  // U_r(ck + 1) into the other LDS slot (its last readers, step ck - 1, are
  // past the barrier that ended that step)
  double u[kUPer];
  floatx4 bufA[4][kS], bufB[4][kS];
  load_u(0, u);
  load_x(0, bufA);
  store_u(0, u);
  __syncthreads();
  int ck = 0;
  for (; ck + 2 <= nchunks; ck += 2) {
    load_u(ck + 1, u);
    load_x(ck + 1, bufB);
    __builtin_amdgcn_sched_barrier(0);
    compute(0, bufA);
    store_u(1, u);
    __syncthreads();
    load_u(ck + 2, u);
    load_x(ck + 2, bufA);
    __builtin_amdgcn_sched_barrier(0);
    compute(1, bufB);
    store_u(0, u);
    __syncthreads();
  }
  if (ck < nchunks) compute(0, bufA);
  // U_l^T T over this wave's 64 rows: A = U_l[row][j] (lane: j = l%16, k = l/16)
  doublex4 part = doublex4{};
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = (int64_t)wv * 64 + 16 * t + g + 4 * v;
      const double ul = (r < rows && l16 < p.rL) ? p.UL[(row0 + r) * p.rL + l16] : 0.0;
      part = mma64(ul, acc[t][v], part);
    }
  sPart[wv][lane] = part;
  __syncthreads();
  if (wv == 0) {
    const doublex4 sum = ((sPart[0][lane] + sPart[1][lane]) + sPart[2][lane]) + sPart[3][lane];
    // lane holds B[j = g + 4 v][k = l16]
    double* out = p.partials + (int64_t)blockIdx.x * 256;
#pragma unroll
    for (int v = 0; v < 4; ++v) out[(g + 4 * v) * 16 + l16] = sum[v];
  }
}

// The workgroup partials are summed in two fixed-order levels: kSumSeg
// segments of consecutive workgroups (eight loads in flight per thread), then
// the segment sums.  A single workgroup walking every partial in turn took
// 0.77 ms at 18^8 (2048 dependent loads per thread).
constexpr int kSumSeg = 64;

__global__ __launch_bounds__(256) void root_sum_seg_kernel(const RootPass p) {
  const int e = threadIdx.x, g = blockIdx.x;
  const int per = (p.nblocks + kSumSeg - 1) / kSumSeg;
  const int b0 = g * per, b1 = min(p.nblocks, b0 + per);
  double s = 0.0;
  int b = b0;
  for (; b + 8 <= b1; b += 8) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = p.partials[(int64_t)(b + u) * 256 + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += t[u];
  }
  for (; b < b1; ++b) s += p.partials[(int64_t)b * 256 + e];
  p.partials[((int64_t)p.nblocks + g) * 256 + e] = s;
}

__global__ __launch_bounds__(256) void root_sum_kernel(const RootPass p) {
  const int e = threadIdx.x, j = e >> 4, k = e & 15;
  double t[kSumSeg];
#pragma unroll
  for (int g = 0; g < kSumSeg; ++g) t[g] = p.partials[((int64_t)p.nblocks + g) * 256 + e];
  double s = 0.0;
#pragma unroll
  for (int g = 0; g < kSumSeg; ++g) s += t[g];
  if (j < p.rL && k < p.rR) p.out[j * p.rR + k] = s;
}

}  // namespace

bool root_pass_supported(int dtype, int64_t nL, int64_t nR, int rL, int rR) {
  return dtype == TK_F32 && rL >= 1 && rL <= 16 && rR >= 1 && rR <= 16 && nL >= 1 && nR >= 1 &&
         (int64_t)kRows * nR * 4 < (int64_t(1) << 31);
}

// column splits per row block: enough workgroups to fill the chip several times
static int root_qsplit(int64_t nL, int64_t nR) {
  const int64_t rb = ceil_div(nL, kRows), chunks = ceil_div(nR, kChunk);
  return (int)std::max<int64_t>(1, std::min<int64_t>(chunks, ceil_div(2048, rb)));
}

int64_t root_pass_blocks(int64_t nL, int64_t nR) { return ceil_div(nL, kRows) * root_qsplit(nL, nR); }

// doubles of the partials buffer: the workgroup partials and the segment sums
int64_t root_pass_partials(int64_t nL, int64_t nR) { return (root_pass_blocks(nL, nR) + kSumSeg) * 256; }

hipError_t launch_root_pass(const RootPass& pin, hipStream_t st) {
  RootPass p = pin;
  p.qsplit = root_qsplit(p.nL, p.nR);
  p.nblocks = (int32_t)root_pass_blocks(p.nL, p.nR);
  hipError_t e = profile_begin(st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(root_pass_kernel, dim3((unsigned)p.nblocks), dim3(256), 0, st, p);
  if ((e = profile_end(st)) != hipSuccess) return e;
  hipLaunchKernelGGL(root_sum_seg_kernel, dim3(kSumSeg), dim3(256), 0, st, p);
  hipLaunchKernelGGL(root_sum_kernel, dim3(1), dim3(256), 0, st, p);
  return hipGetLastError();
}

}  // namespace tk
