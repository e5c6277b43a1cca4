// Two-sided product of an FP32 matrix in one read (Algorithm 2 with dense
// children of the root, Section 4.2.1's sampling rule): for X (n1 x n2,
// row-major; the tensor viewed through the root's split)
//   O1 = X P1     (n1 x k1)       P1: n2 x k1
//   O2 = P2^T X   (k2 x n2)       P2: n1 x k2
// on v_mfma_f64_16x16x4f64 with FP64 accumulation (X converts exactly).  The
// dense left child's sketch X Omega_l and the right child's Omega_r^T X are
// one call; after the QR, the two W-step products Q_l^T X and X Q_r are the
// other.  k1, k2 <= 16.
//
// A workgroup (eight waves) owns a 1024 x 1024 tile and walks it in strips of
// 16 rows.  Wave w owns the strip's columns 128 w .. 128 w + 127: it loads
// them (16-byte loads, next strip ahead), stages them in its own LDS block,
// and reads them back in the two operand layouts:
//   O1: A operand X[16 rows][K = 4 columns], B operand P1 rows (in registers
//       for the whole tile); the eight waves' 16 x k1 partials of a strip are
//       summed in wave order through LDS and written per column tile;
//   O2: A operand P2^T (the strip's 16 rows of P2), B operand X[K = 4 rows]
//       [16 columns]; the 16 x 128 accumulators stay in registers over the
//       tile's 64 strips and are written per row tile.
// Second kernels sum the per-tile partials in tile order (fixed order, so the
// result does not depend on scheduling).  In the FP64 16x16 MFMA result,
// register v of lane l is row l/16 + 4 v, column l%16.
#include "tk_kernels.hpp"

namespace tk {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 1024;               // rows and columns of a workgroup's tile
constexpr int kWaves = 8;
constexpr int kWaveCols = kTile / kWaves; // 128
constexpr int kStrip = 16;
constexpr int kSW = kWaveCols + 4;        // LDS row stride of a wave's strip block (floats)
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ doublex4 mma64(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename TP>
__device__ __forceinline__ double pval(const TP* p, int64_t i) {
  return (double)p[i];
}

template <typename TP>
__global__ __launch_bounds__(64 * kWaves, 1) void twoside_kernel(const TwoSide ts) {
  __shared__ float sX[kWaves][kStrip][kSW];
  __shared__ double sRed[2][kWaves][4][64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int rt = blockIdx.x / ts.nct, ct = blockIdx.x - rt * ts.nct;
  const int64_t r0 = (int64_t)rt * kTile, c0 = (int64_t)ct * kTile + wv * kWaveCols;
  const TP* P1 = static_cast<const TP*>(ts.P1);
  const TP* P2 = static_cast<const TP*>(ts.P2);
  // O1's B operand for the wave's 128 columns: P1[c0 + 4 s + l/16][l%16]
  double p1[kWaveCols / 4];
#pragma unroll
  for (int s = 0; s < kWaveCols / 4; ++s) {
    const int64_t j = c0 + 4 * s + g;
    p1[s] = (j < ts.n2 && l16 < ts.k1) ? pval(P1, j * ts.k1 + l16) : 0.0;
  }
  doublex4 acc2[kWaveCols / 16];
#pragma unroll
  for (int t = 0; t < kWaveCols / 16; ++t) acc2[t] = doublex4{0.0, 0.0, 0.0, 0.0};
  const int nstrips = (int)min<int64_t>(kTile / kStrip, (ts.n1 - r0 + kStrip - 1) / kStrip);
  // this lane's part of a strip: element (u * 64 + lane) * 4 of the 16 x 128
  // block is row e / 128, columns e % 128 .. + 3
  uint32_t xoff[8];
  int xvalid[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int e = (u * 64 + lane) * 4, row = e / kWaveCols, col = e % kWaveCols;
    const int64_t left = ts.n2 - (c0 + col);   // valid columns from this one on
    xvalid[u] = (int)max<int64_t>(0, min<int64_t>(4, left));
    xoff[u] = xvalid[u] > 0 ? (uint32_t)((row * ts.n2 + c0 + col) * 4) : 0x80000000u;
  }
  auto issue = [&](int s, uintx4 (&xr)[8]) {
    const int64_t row0 = r0 + (int64_t)s * kStrip;
    const int64_t rows = s < nstrips ? min<int64_t>(kStrip, ts.n1 - row0) : 0;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(ts.X) + (rows > 0 ? row0 * ts.n2 : 0), (short)0, (int)(rows * ts.n2 * 4), kRsrcWord3);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      xr[u] = __builtin_bit_cast(uintx4, __builtin_amdgcn_raw_buffer_load_b128(rs, xoff[u], 0, 0));
  };
  uintx4 xr[8];
  issue(0, xr);
  float (*mine)[kSW] = sX[wv];
  for (int s = 0; s < nstrips; ++s) {
    // this strip's values into the wave's block (columns past n2 zeroed: a
    // load that straddles the end of a row would carry the next row's values)
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = (u * 64 + lane) * 4, row = e / kWaveCols, col = e % kWaveCols;
      uintx4 v = xr[u];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c >= xvalid[u]) v[c] = 0u;
      *reinterpret_cast<floatx4*>(&mine[row][col]) = __builtin_bit_cast(floatx4, v);
    }
    issue(s + 1, xr);   // the next strip in flight while this one is multiplied
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    // O1: 16 rows x k1 over the wave's 128 columns
    doublex4 acc1 = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kWaveCols / 4; ++k) acc1 = mma64((double)mine[l16][4 * k + g], p1[k], acc1);
    // O2: k2 x 128 over the strip's 16 rows (A operand P2[row0 + 4 k + l/16][l%16])
    const int64_t row0 = r0 + (int64_t)s * kStrip;
    double p2[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t i = row0 + 4 * k + g;
      p2[k] = (i < ts.n1 && l16 < ts.k2) ? pval(P2, i * ts.k2 + l16) : 0.0;
    }
#pragma unroll
    for (int t = 0; t < kWaveCols / 16; ++t)
#pragma unroll
      for (int k = 0; k < 4; ++k) acc2[t] = mma64(p2[k], (double)mine[4 * k + g][16 * t + l16], acc2[t]);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();   // the reads of the block precede the next strip's writes
    // the eight waves' O1 partials of this strip, summed in wave order
    const int b = s & 1;
#pragma unroll
    for (int v = 0; v < 4; ++v) sRed[b][wv][v][lane] = acc1[v];
    __syncthreads();
    if (tid < 256) {
      const int v = tid >> 6, l = tid & 63;
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) sum += sRed[b][w][v][l];
      const int64_t i = row0 + (l >> 4) + 4 * v;
      const int k = l & 15;
      if (i < ts.n1 && k < ts.k1) ts.part1[((int64_t)ct * ts.n1 + i) * 16 + k] = sum;
    }
  }
  // O2 partial of this row tile: row l/16 + 4 v (k2), column 16 t + l%16
#pragma unroll
  for (int t = 0; t < kWaveCols / 16; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = g + 4 * v;
      const int64_t j = c0 + 16 * t + l16;
      if (k < ts.k2 && j < ts.n2) ts.part2[((int64_t)rt * 16 + k) * ts.n2 + j] = acc2[t][v];
    }
}

// O1[i][k] = sum over column tiles, in order
__global__ void twoside_sum1_kernel(const TwoSide ts) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ts.n1 * ts.k1) return;
  const int64_t i = e / ts.k1;
  const int k = (int)(e - i * ts.k1);
  double sum = 0.0;
  for (int c = 0; c < ts.nct; ++c) sum += ts.part1[((int64_t)c * ts.n1 + i) * 16 + k];
  ts.out1[e] = sum;
}

// O2[k][j] = sum over row tiles, in order; written k2 x n2 or, transposed, n2 x k2
__global__ void twoside_sum2_kernel(const TwoSide ts) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ts.n2 * ts.k2) return;
  const int k = (int)(e / ts.n2);
  const int64_t j = e - (int64_t)k * ts.n2;
  double sum = 0.0;
  for (int r = 0; r < ts.nrt; ++r) sum += ts.part2[((int64_t)r * 16 + k) * ts.n2 + j];
  if (ts.out2_transposed) ts.out2[j * ts.k2 + k] = sum;
  else ts.out2[e] = sum;
}

}  // namespace

bool twoside_supported(int x_dtype, int64_t n1, int64_t n2, int k1, int k2) {
  return x_dtype == TK_F32 && n1 >= 1 && n2 >= 1 && k1 >= 1 && k1 <= 16 && k2 >= 1 && k2 <= 16 &&
         (int64_t)kStrip * n2 * 4 < (int64_t(1) << 31) && n1 * n2 < (int64_t(1) << 40);
}

int64_t twoside_partials(int64_t n1, int64_t n2) {
  // part1: column tiles x n1 x 16, part2: row tiles x 16 x n2
  return ceil_div(n2, kTile) * n1 * 16 + ceil_div(n1, kTile) * 16 * n2;
}

hipError_t launch_twoside(const TwoSide& pin, int p_dtype, hipStream_t st) {
  TwoSide ts = pin;
  ts.nrt = (int32_t)ceil_div(ts.n1, kTile);
  ts.nct = (int32_t)ceil_div(ts.n2, kTile);
  ts.part2 = ts.part1 + (int64_t)ts.nct * ts.n1 * 16;
  const dim3 grid((unsigned)((int64_t)ts.nrt * ts.nct));
  if (p_dtype == TK_F64) hipLaunchKernelGGL(twoside_kernel<double>, grid, dim3(64 * kWaves), 0, st, ts);
  else hipLaunchKernelGGL(twoside_kernel<float>, grid, dim3(64 * kWaves), 0, st, ts);
  if (hipError_t e = hipGetLastError()) return e;
  hipLaunchKernelGGL(twoside_sum1_kernel, dim3((unsigned)ceil_div(ts.n1 * ts.k1, 256)), dim3(256), 0, st, ts);
  if (hipError_t e = hipGetLastError()) return e;
  hipLaunchKernelGGL(twoside_sum2_kernel, dim3((unsigned)ceil_div(ts.n2 * ts.k2, 256)), dim3(256), 0, st, ts);
  return hipGetLastError();
}

}  // namespace tk
