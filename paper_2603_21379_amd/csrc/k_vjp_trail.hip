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
// tiles of 128 rows x 64 columns through LDS (the next tile's global loads
// are in flight while the current one is multiplied), all products on
// v_mfma_f32_32x32x2f32.  In a tile, wave w
//  * adds to Fbar_J for the 32 columns 32 (w % 2) of the tile over the 64
//    rows 64 (w / 2): the tile as the A operand with M = column b and
//    K = row i (lanes read 32 consecutive columns of a row), W's rows as B;
//  * adds to Fbar_I for the 32 rows 32 w over the tile's 64 columns: the
//    tile as the A operand with M = row i and K = column b (lanes read one
//    column of 32 rows; the LDS row stride 65 puts them in distinct banks),
//    V's rows as B.
// So every wave does the same work per tile, a wave's Fbar_I rows are its
// own, and the two waves that share Fbar_J columns add their sums at the end
// in a fixed order.  Each workgroup writes its partial gradients; a second
// kernel sums the partials of all workgroups in FP64, in workgroup order.
#include "tk_kernels.hpp"

namespace tk {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kMaxN = 256;            // n_I, n_J per kernel
constexpr int kRows = 128;            // rows of a tile (a row group)
constexpr int kCols = 64;             // columns of a tile (a column chunk)
constexpr int kMaxGroups = kMaxN / kRows;
constexpr int kLdx = kCols + 1;       // LDS row stride of a tile
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// NJC column chunks of 64 (n_J <= 64 NJC); row groups of 128 at run time
template <int NJC>
__global__ __launch_bounds__(kThreads, 1) void vjp_trail_kernel(const VjpTrail p) {
  extern __shared__ float lds_raw[];
  constexpr int nJp = kCols * NJC, nJt = nJp / 32;
  const int nG = (p.nI + kRows - 1) / kRows, nIp = nG * kRows, nIt = nIp / 32;
  float* sx = lds_raw;                  // [kRows][kLdx]
  float* sw = sx + kRows * kLdx;        // W [nIp][33]
  float* sv = sw + nIp * 33;            // V [nJp][33]
  float* sk = sv + nJp * 33;            // K [32][33]
  const int tid = threadIdx.x, lane = tid & 63, l32 = lane & 31, kh = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wc = wave & 1, wh = wave >> 1;
  const int64_t nIJ = (int64_t)p.nI * p.nJ;

  // A operands of the W and V products (reloaded per slab from the cache):
  // lane l holds row 32 tile + l%32, columns 2t + l/32; zero past the ends
  const __amdgpu_buffer_rsrc_t rfi = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(p.FI), (short)0, p.nI * p.cI * 4, kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rfj = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(p.FJ), (short)0, p.nJ * p.cJ * 4, kRsrcWord3);
  auto load_f = [&](const __amdgpu_buffer_rsrc_t& rs, int n, int c, int ti, float (&f)[16]) {
    const int i = 32 * ti + l32;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int al = 2 * t + kh;
      const uint32_t off = (i < n && al < c) ? (uint32_t)((i * c + al) * 4) : 0x80000000u;
      f[t] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
    }
  };

  floatx16 accJ[NJC], accI[kMaxGroups];
#pragma unroll
  for (int c = 0; c < NJC; ++c) accJ[c] = floatx16{};
#pragma unroll
  for (int g = 0; g < kMaxGroups; ++g) accI[g] = floatx16{};

  // this thread's float4s of a tile: index e = tid + 256 q, row e / 16,
  // columns 4 (e % 16) .. + 3 (n_J % 4 == 0: a float4 never crosses a row);
  // rows past n_I and columns past n_J read zero
  auto load_tile = [&](int64_t a, int g, int cc, floatx4 (&buf)[8]) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(p.X + a * nIJ), (short)0, (int)(nIJ * 4), kRsrcWord3);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + kThreads * q;
      const int gi = kRows * g + (e >> 4), col = kCols * cc + 4 * (e & 15);
      const uint32_t off = (col < p.nJ && gi < p.nI) ? (uint32_t)((gi * p.nJ + col) * 4) : 0x80000000u;
      buf[q] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 2);
    }
  };
  auto store_tile = [&](const floatx4 (&buf)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + kThreads * q;
      float* d = sx + (e >> 4) * kLdx + 4 * (e & 15);
      d[0] = buf[q][0];
      d[1] = buf[q][1];
      d[2] = buf[q][2];
      d[3] = buf[q][3];
    }
  };

  floatx4 buf[8];
  int64_t a = blockIdx.x;
  if (a < p.A) load_tile(a, 0, 0, buf);
  for (; a < p.A; a += gridDim.x) {
    // K[a] into LDS (zero padded to 32 x 32)
    __syncthreads();   // the previous slab's last tile and W/V are consumed
    const float* Ka = p.K + a * p.cI * p.cJ;
    for (int e = tid; e < 32 * 32; e += kThreads) {
      const int al = e >> 5, be = e & 31;
      sk[al * 33 + be] = (al < p.cI && be < p.cJ) ? Ka[al * p.cJ + be] : 0.0f;
    }
    __syncthreads();
    // W = F_I K[a] (tiles of 32 rows i) and V = F_J K[a]^T (tiles of 32 rows b)
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int ti = wave + kWaves * sl;
      float fa[16], fb[16];
      load_f(rfi, p.nI, p.cI, ti, fa);
      load_f(rfj, p.nJ, p.cJ, ti, fb);
      if (ti < nIt) {
        float kb[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) kb[t] = sk[(2 * t + kh) * 33 + l32];
        floatx16 c = floatx16{};
#pragma unroll
        for (int t = 0; t < 16; ++t) c = mfma32(fa[t], kb[t], c);
#pragma unroll
        for (int v = 0; v < 16; ++v)
          sw[(32 * ti + 8 * (v >> 2) + 4 * kh + (v & 3)) * 33 + l32] = c[v];
      }
      if (ti < nJt) {
        float kb[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) kb[t] = sk[l32 * 33 + 2 * t + kh];
        floatx16 c = floatx16{};
#pragma unroll
        for (int t = 0; t < 16; ++t) c = mfma32(fb[t], kb[t], c);
#pragma unroll
        for (int v = 0; v < 16; ++v)
          sv[(32 * ti + 8 * (v >> 2) + 4 * kh + (v & 3)) * 33 + l32] = c[v];
      }
    }
#pragma unroll
    for (int g = 0; g < kMaxGroups; ++g) {
      if (g < nG) {
#pragma unroll
        for (int cc = 0; cc < NJC; ++cc) {
          __syncthreads();   // the previous tile is consumed (and W, V are written)
          store_tile(buf);
          // the next tile (or the next slab's first) in flight during the products
          if (cc + 1 < NJC) load_tile(a, g, cc + 1, buf);
          else if (g + 1 < nG) load_tile(a, g + 1, 0, buf);
          else if (a + gridDim.x < p.A) load_tile(a + gridDim.x, 0, 0, buf);
          __syncthreads();
          // Fbar_J: A = tile[64 wh + k][32 wc + l%32], B = W[128 g + 64 wh + k][l%32]
          // Fbar_I: A = tile[32 w + l%32][k],          B = V[64 cc + k][l%32]
          const float* xj = sx + 64 * wh * kLdx + 32 * wc + l32;
          const float* wj = sw + (kRows * g + 64 * wh) * 33 + l32;
          const float* xi = sx + (32 * wave + l32) * kLdx;
          const float* vi = sv + kCols * cc * 33 + l32;
          // operands of four K steps per chunk (K = 32 steps of two for both
          // products); the next chunk's LDS reads go out before this chunk's
          // products
          float op[2][4][4];
          auto fetch = [&](int c, float (&o)[4][4]) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int k = 2 * (4 * c + u) + kh;
              o[u][0] = xj[k * kLdx];
              o[u][1] = wj[k * 33];
              o[u][2] = xi[k];
              o[u][3] = vi[k * 33];
            }
          };
          fetch(0, op[0]);
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            if (c + 1 < 8) fetch(c + 1, op[(c + 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              accJ[cc] = mfma32(op[c & 1][u][0], op[c & 1][u][1], accJ[cc]);
              accI[g] = mfma32(op[c & 1][u][2], op[c & 1][u][3], accI[g]);
            }
          }
        }
      }
    }
  }

  // Fbar_J: columns 64 cc + 32 wc + m (m = 8 (v/4) + 4 kh + v%4), beta = l%32;
  // the row-half-1 waves' sums are added to the row-half-0 waves' in LDS
  __syncthreads();
  float* red = lds_raw;   // [2 column halves][NJC][32][32]
  if (wh == 1) {
#pragma unroll
    for (int cc = 0; cc < NJC; ++cc)
#pragma unroll
      for (int v = 0; v < 16; ++v)
        red[((wc * NJC + cc) * 32 + 8 * (v >> 2) + 4 * kh + (v & 3)) * 32 + l32] = accJ[cc][v];
  }
  __syncthreads();
  float* pj = p.partJ + (int64_t)blockIdx.x * nJp * 32;
  if (wh == 0) {
#pragma unroll
    for (int cc = 0; cc < NJC; ++cc)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int m = 8 * (v >> 2) + 4 * kh + (v & 3);
        pj[(kCols * cc + 32 * wc + m) * 32 + l32] =
            accJ[cc][v] + red[((wc * NJC + cc) * 32 + m) * 32 + l32];
      }
  }
  // Fbar_I: rows 128 g + 32 w + m, alpha = l%32 (this wave's own rows)
  float* pi = p.partI + (int64_t)blockIdx.x * nIp * 32;
#pragma unroll
  for (int g = 0; g < kMaxGroups; ++g)
    if (g < nG)
#pragma unroll
      for (int v = 0; v < 16; ++v)
        pi[(kRows * g + 32 * wave + 8 * (v >> 2) + 4 * kh + (v & 3)) * 32 + l32] = accI[g][v];
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

// rows of the per-workgroup partials: n_I padded to 128, n_J padded to 64
int64_t vjp_trail_rows_i(int64_t nI) { return (nI + kRows - 1) / kRows * kRows; }
int64_t vjp_trail_rows_j(int64_t nJ) { return (nJ + kCols - 1) / kCols * kCols; }

size_t vjp_trail_lds(int nI, int nJ) {
  const size_t nIp = vjp_trail_rows_i(nI), nJp = vjp_trail_rows_j(nJ);
  const size_t fl = (size_t)kRows * kLdx + nIp * 33 + nJp * 33 + 32 * 33;
  const size_t red = (size_t)2 * (nJp / kCols) * 32 * 32;
  return std::max(fl, red) * sizeof(float);
}

hipError_t launch_vjp_trail(const VjpTrail& p, void* FbarI, void* FbarJ, int out_dt, int accumulate,
                            hipStream_t st) {
  const int nb = p.nblocks;
  const size_t lds = vjp_trail_lds(p.nI, p.nJ);
  switch ((p.nJ + kCols - 1) / kCols) {
    case 1: hipLaunchKernelGGL((vjp_trail_kernel<1>), dim3(nb), dim3(kThreads), lds, st, p); break;
    case 2: hipLaunchKernelGGL((vjp_trail_kernel<2>), dim3(nb), dim3(kThreads), lds, st, p); break;
    case 3: hipLaunchKernelGGL((vjp_trail_kernel<3>), dim3(nb), dim3(kThreads), lds, st, p); break;
    case 4: hipLaunchKernelGGL((vjp_trail_kernel<4>), dim3(nb), dim3(kThreads), lds, st, p); break;
    default: return hipErrorInvalidValue;
  }
  const int64_t nIp = vjp_trail_rows_i(p.nI), nJp = vjp_trail_rows_j(p.nJ);
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
  reduce(p.partI, (int)nIp, p.nI, p.cI, FbarI);
  reduce(p.partJ, (int)nJp, p.nJ, p.cJ, FbarJ);
  return hipGetLastError();
}

}  // namespace tk
