// Batched thin QR of the sketches (CholeskyQR2 with an FP64 Gram, shifted
// first pass when the Gram is not safely positive definite) and the rank
// truncation W step of Algorithm 1: W = dominant r left singular vectors of
// M = Q^T Y, computed as the dominant eigenvectors of the FP64 Gram M M^T by
// cyclic Jacobi in one wavefront; U = Q W with a deterministic column sign.
//
// Every reduction runs in a fixed order (partials per row chunk or column
// chunk, then summed in index order), so results are bitwise repeatable.
#include "tk_kernels.hpp"

namespace tk {
namespace {

constexpr double kUnit = 1.1102230246251565e-16;  // 2^-53

// ------------------------------------------------------------------ Gram partials
// gpart[rc] = Z[rows of rc]^T Z[rows of rc]
template <typename S>
__global__ __launch_bounds__(256) void gram_partial_kernel(const S b, int pass) {
  const QRMat& M = b.get(blockIdx.y);
  const int rc = blockIdx.x;
  if (rc >= M.nrc || M.small) return;
  if (pass > 1 && M.state[0] == 0) return;
  __shared__ double sZ[64][kMaxEll + 1];
  const int ell = M.ell, tid = threadIdx.x;
  const int64_t r0 = (int64_t)rc * kQRRowChunk;
  const int64_t r1 = min<int64_t>(M.m, r0 + kQRRowChunk);
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int64_t s0 = r0; s0 < r1; s0 += 64) {
    const int rows = (int)min<int64_t>(64, r1 - s0);
    __syncthreads();
    for (int e = tid; e < 64 * ell; e += 256) {
      const int rr = e / ell, j = e - rr * ell;
      sZ[rr][j] = rr < rows ? M.Z[(s0 + rr) * ell + j] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q;
      if (e < ell * ell) {
        const int p = e / ell, c = e - p * ell;
        double a = acc[q];
        for (int rr = 0; rr < rows; ++rr) a = fma(sZ[rr][p], sZ[rr][c], a);
        acc[q] = a;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q;
    if (e < ell * ell) M.gpart[(int64_t)rc * ell * ell + e] = acc[q];
  }
}

// ------------------------------------------------------------------ Cholesky (one wave)
// Upper Cholesky factor of the summed Gram (+ shift) in LDS.  Returns true on
// success.  Called uniformly by the 64 lanes.
__device__ bool cholesky_upper(double (*G)[kMaxEll + 1], int n, int lane, double tol) {
  __shared__ int ok;
  if (lane == 0) ok = 1;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double piv = G[j][j];
    if (!(piv > tol)) {  // also catches NaN
      if (lane == 0) ok = 0;
      __syncthreads();
      return false;
    }
    const double rjj = sqrt(piv);
    __syncthreads();
    for (int i = j + 1 + lane; i < n; i += 64) G[j][i] = G[j][i] / rjj;
    __syncthreads();
    if (lane == 0) G[j][j] = rjj;
    // trailing update of the upper triangle
    const int m = n - j - 1;
    for (int e = lane; e < m * m; e += 64) {
      const int p = j + 1 + e / m, q = j + 1 + e % m;
      if (q >= p) G[p][q] -= G[j][p] * G[j][q];
    }
    __syncthreads();
  }
  return ok != 0;
}

// state[0]: CholeskyQR passes still owed (a plain pass pays one, a shifted
// pass leaves two owed); state[1]: whether this pass applies R^{-1}.
template <typename S>
__global__ __launch_bounds__(64) void chol_kernel(const S b, int pass) {
  const QRMat& M = b.get(blockIdx.x);
  if (M.small) return;
  if (pass > 1 && M.state[0] == 0) {
    if (threadIdx.x == 0) M.state[1] = 0;
    return;
  }
  __shared__ double G[kMaxEll][kMaxEll + 1];
  __shared__ double red[64];
  const int n = M.ell, lane = threadIdx.x;
  auto load = [&](double shift) {
    for (int e = lane; e < n * n; e += 64) {
      const int p = e / n, q = e - p * n;
      double v = 0.0;
      for (int c = 0; c < M.nrc; ++c) v += M.gpart[(int64_t)c * n * n + e];
      G[p][q] = v + (p == q ? shift : 0.0);
    }
    __syncthreads();
  };
  load(0.0);
  double mx = 0.0, tr = 0.0;
  for (int j = lane; j < n; j += 64) { mx = fmax(mx, G[j][j]); tr += G[j][j]; }
  red[lane] = mx;
  __syncthreads();
  if (lane == 0) {
    double a = 0.0;
    for (int i = 0; i < 64; ++i) a = fmax(a, red[i]);
    red[0] = a;
  }
  __syncthreads();
  mx = red[0];
  __syncthreads();
  red[lane] = tr;
  __syncthreads();
  if (lane == 0) {
    double a = 0.0;
    for (int i = 0; i < 64; ++i) a += red[i];
    red[1] = a;
  }
  __syncthreads();
  tr = red[1];
  // a pivot below this means cond(Z) beyond what two CholeskyQR passes repair
  const double tol = 1e-14 * mx;
  int status = 0;
  bool ok = mx > 0.0 && cholesky_upper(G, n, lane, tol);
  if (!ok) {
    // shifted CholeskyQR (Fukaya et al. 2020): s = 11 (m n + n (n+1)) u ||Z||^2,
    // with ||Z||_2^2 bounded by the trace of the Gram
    const double shift = 11.0 * ((double)M.m * n + (double)n * (n + 1)) * kUnit * fmax(tr, 1e-300);
    __syncthreads();
    load(shift);
    status = 1;
    ok = cholesky_upper(G, n, lane, 0.0);
    if (!ok) status = 2;
  }
  __syncthreads();
  for (int e = lane; e < n * n; e += 64) {
    const int p = e / n, q = e - p * n;
    double v = q >= p ? G[p][q] : 0.0;
    if (!ok && p == q && !(v > 0.0)) v = 1.0;  // keep the solve finite; flagged in info
    M.R[e] = v;
  }
  if (lane == 0) {
    const int owed = pass == 1 ? 2 : M.state[0];
    M.state[0] = status != 0 ? 2 : owed - 1;
    M.state[1] = 1;
    if (M.info) {
      // bit 0: first pass shifted; bit 1: a later pass shifted; bit 2: Cholesky
      // failed even with the shift
      int v = pass == 1 ? 0 : *M.info;
      if (status != 0) v |= pass == 1 ? 1 : 2;
      if (status == 2) v |= 4;
      *M.info = v;
    }
  }
}

// Q = Z R^{-1} row by row (forward substitution on q R = z), in place.
template <typename S>
__global__ __launch_bounds__(64) void apply_rinv_kernel(const S b, int pass) {
  const QRMat& M = b.get(blockIdx.y);
  const int rb = blockIdx.x;
  if (rb >= M.nrb || M.small) return;
  if (M.state[1] == 0) return;
  (void)pass;
  __shared__ double R[kMaxEll][kMaxEll + 1];
  __shared__ double sZ[kMaxEll][65];
  const int n = M.ell, lane = threadIdx.x;
  const int64_t r0 = (int64_t)rb * kQRRowBlock;
  const int rows = (int)min<int64_t>(kQRRowBlock, M.m - r0);
  for (int e = lane; e < n * n; e += 64) R[e / n][e % n] = M.R[e];
  for (int e = lane; e < rows * n; e += 64) {
    const int rr = e / n, j = e - rr * n;
    sZ[j][rr] = M.Z[(r0 + rr) * n + j];
  }
  __syncthreads();
  if (lane < rows) {
    for (int j = 0; j < n; ++j) {
      double v = sZ[j][lane];
      for (int k = 0; k < j; ++k) v = fma(-sZ[k][lane], R[k][j], v);
      sZ[j][lane] = v / R[j][j];
    }
  }
  __syncthreads();
  for (int e = lane; e < rows * n; e += 64) {
    const int rr = e / n, j = e - rr * n;
    M.Z[(r0 + rr) * n + j] = sZ[j][rr];
  }
}

// ------------------------------------------------------------------ small matrices
// Every CholeskyQR pass of one matrix in one 256-thread workgroup (m x ell <=
// kQRSmallElems): Gram from 32-row chunks staged in LDS, Cholesky in LDS, and
// Q = Z R^{-1} by forward substitution with each row held in registers.
// Same passes, shift rule and info bits as the multi-kernel path.
constexpr int kSmallChunk = 32;

// Within one wavefront LDS operations complete in issue order, so lanes of
// that wave only need the compiler kept from reordering across this point.
#define TK_WAVE_SYNC()                          \
  do {                                          \
    __atomic_signal_fence(__ATOMIC_SEQ_CST);    \
    __builtin_amdgcn_wave_barrier();            \
    __atomic_signal_fence(__ATOMIC_SEQ_CST);    \
  } while (0)

// Upper Cholesky factor in place, by the 64 lanes of one wave (no barriers).
__device__ bool cholesky_upper_wave(double (*G)[kMaxEll + 1], int n, int lane, double tol) {
  for (int j = 0; j < n; ++j) {
    const double piv = G[j][j];
    if (!(piv > tol)) return false;  // uniform: every lane read the same pivot
    const double rjj = sqrt(piv), inv = 1.0 / rjj;
    TK_WAVE_SYNC();
    // lane q owns column q (n <= 64): scale row j, then the trailing update
    // of its column, rows j < p <= q (row p's multiplier is a broadcast)
    const int q = lane;
    double gjq = 0.0;
    if (q > j && q < n) {
      gjq = G[j][q] * inv;
      G[j][q] = gjq;
    }
    if (lane == 0) G[j][j] = rjj;
    TK_WAVE_SYNC();
    if (q > j && q < n)
      for (int p = j + 1; p <= q; ++p) G[p][q] -= G[j][p] * gjq;
    TK_WAVE_SYNC();
  }
  return true;
}

// In-place inverse of the upper triangular R by one wave (as LAPACK's
// unblocked trti2): column j of R^{-1} is -R^{-1}_{jj} R^{-1}(0:j, 0:j) R(0:j, j).
__device__ void upper_inverse_wave(double (*R)[kMaxEll + 1], int n, int lane) {
  for (int j = 0; j < n; ++j) {
    const double rjj = 1.0 / R[j][j];
    TK_WAVE_SYNC();
    // four independent partial sums so the LDS reads pipeline
    double x0 = 0.0, x1 = 0.0, x2 = 0.0, x3 = 0.0;
    if (lane < j) {
      int k = lane;
      for (; k + 4 <= j; k += 4) {
        x0 = fma(R[lane][k], R[k][j], x0);
        x1 = fma(R[lane][k + 1], R[k + 1][j], x1);
        x2 = fma(R[lane][k + 2], R[k + 2][j], x2);
        x3 = fma(R[lane][k + 3], R[k + 3][j], x3);
      }
      for (; k < j; ++k) x0 = fma(R[lane][k], R[k][j], x0);
    }
    const double x = (x0 + x1) + (x2 + x3);
    TK_WAVE_SYNC();
    if (lane < j) R[lane][j] = -rjj * x;
    if (lane == 0) R[j][j] = rjj;
    TK_WAVE_SYNC();
  }
}

// Q = Z R^{-1} in place on the LDS copy of Z, 64 rows at a time: thread t
// forms the 4 x 4 output tile (rows 4 (t / 16), columns 4 (t % 16)) in
// registers; the chunk is overwritten once every thread has read its rows.
__device__ void apply_inverse_lds(double* sZ, int64_t m, int n, const double (*Ri)[kMaxEll + 1],
                                  int tid) {
  const int ti = tid >> 4, tj = tid & 15;
  const int jmax = min(n, 4 * tj + 4);   // R^{-1} is upper triangular: k <= j
  for (int64_t r0 = 0; r0 < m; r0 += 64) {
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[a][c] = 0.0;
    int64_t rows[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) rows[a] = min<int64_t>(r0 + 4 * ti + a, m - 1);
#pragma unroll 4
    for (int k = 0; k < jmax; ++k) {
      double z[4], w[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) z[a] = sZ[rows[a] * n + k];
#pragma unroll
      for (int c = 0; c < 4; ++c) w[c] = (4 * tj + c < n) ? Ri[k][4 * tj + c] : 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = fma(z[a], w[c], acc[a][c]);
    }
    __syncthreads();   // every read of this chunk is done
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int64_t row = r0 + 4 * ti + a;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int j = 4 * tj + c;
        if (row < m && j < n) sZ[row * n + j] = acc[a][c];
      }
    }
    __syncthreads();
  }
}

template <typename S>
__global__ __launch_bounds__(256) void cholqr_small_kernel(const S b) {
  const QRMat& M = b.get(blockIdx.x);
  if (!M.small) return;
  // Z stays in LDS for every pass (row stride ell): one coalesced read at the
  // start, one write of Q at the end, no global latency inside the passes
  extern __shared__ double sZ[];
  __shared__ double G[kMaxEll][kMaxEll + 1];
  __shared__ double red[2];
  __shared__ int ok;
  const int n = M.ell, tid = threadIdx.x;
  const int64_t mn = M.m * n;
  for (int64_t e = tid; e < mn; e += 256) sZ[e] = M.Z[e];
  __syncthreads();
  const int ti = tid >> 4, tj = tid & 15;
  int owed = 2, info = 0;
  for (int pass = 1; pass <= kQRMaxPasses && owed > 0; ++pass) {
    // Gram: thread t owns the 4 x 4 tile (4 (t / 16), 4 (t % 16)) of G, so a
    // row costs 8 LDS reads for 16 FMAs; the tile stays in registers for a
    // shifted retry
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[a][c] = 0.0;
    int ca[4], cc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      ca[a] = min(4 * ti + a, n - 1);
      cc[a] = min(4 * tj + a, n - 1);
    }
#pragma unroll 4
    for (int64_t r = 0; r < M.m; ++r) {
      const double* zr = sZ + r * n;
      double x[4], y[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) x[a] = zr[ca[a]];
#pragma unroll
      for (int c = 0; c < 4; ++c) y[c] = zr[cc[c]];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = fma(x[a], y[c], acc[a][c]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int p = 4 * ti + a, q = 4 * tj + c;
        if (p < n && q < n) G[p][q] = acc[a][c];
      }
    __syncthreads();
    if (tid == 0) {
      double mx = 0.0, tr = 0.0;
      for (int j = 0; j < n; ++j) { mx = fmax(mx, G[j][j]); tr += G[j][j]; }
      red[0] = mx;
      red[1] = tr;
    }
    __syncthreads();
    const double mx = red[0], tr = red[1];
    // Cholesky by wave 0; on failure every thread rewrites its tile of the
    // Gram with the shift and wave 0 factors again
    if (tid < 64) {
      const bool good = mx > 0.0 && cholesky_upper_wave(G, n, tid, 1e-14 * mx);
      if (tid == 0) ok = good ? 0 : 1;
    }
    __syncthreads();
    if (ok != 0) {
      const double shift = 11.0 * ((double)M.m * n + (double)n * (n + 1)) * kUnit * fmax(tr, 1e-300);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int p = 4 * ti + a, q = 4 * tj + c;
          if (p < n && q < n) G[p][q] = acc[a][c] + (p == q ? shift : 0.0);
        }
      __syncthreads();
      if (tid < 64) {
        const bool good = cholesky_upper_wave(G, n, tid, 0.0);
        if (!good) {
          TK_WAVE_SYNC();
          for (int j = tid; j < n; j += 64)
            if (!(G[j][j] > 0.0)) G[j][j] = 1.0;  // keep the solve finite; flagged
        }
        if (tid == 0) ok = good ? 1 : 2;
      }
    }
    // the triangular inverse by wave 0 (zero the strict lower triangle left
    // over from the Gram first)
    if (tid < 64) {
      TK_WAVE_SYNC();
      for (int e = tid; e < n * n; e += 64)
        if (e / n > e % n) G[e / n][e % n] = 0.0;
      TK_WAVE_SYNC();
      upper_inverse_wave(G, n, tid);
    }
    __syncthreads();
    const int status = ok;
    apply_inverse_lds(sZ, M.m, n, G, tid);
    if (status != 0) info |= pass == 1 ? 1 : 2;
    if (status == 2) info |= 4;
    owed = status != 0 ? 2 : owed - 1;
  }
  for (int64_t e = tid; e < mn; e += 256) M.Z[e] = sZ[e];
  if (tid == 0) {
    if (M.info) *M.info = info;
    M.state[0] = 0;
    M.state[1] = 0;
  }
}

// ------------------------------------------------------------------ W step
// mpart[rc][p][t] = sum_{rows in rc} Q[row][p] Y[row][t], t in column chunk cc.
// Each thread owns a 4 x 4 register tile (p = 4 pr + i, t = 4 tc + j), so an
// FMA costs half an LDS read instead of two.
// Blocks form one flat list over the matrices (qty_begin: prefix of nrc * ncc),
// so a batch of very different shapes launches no empty blocks.
template <typename TY, typename S>
__global__ __launch_bounds__(256) void qty_partial_kernel(const S b, int count) {
  const int64_t blk = blockIdx.x;
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.get(mid).qty_begin <= blk) lo = mid; else hi = mid - 1;
  }
  const QRMat& M = b.get(lo);
  const int64_t lb = blk - M.qty_begin;
  const int rc = (int)(lb / M.ncc), cc = (int)(lb - (int64_t)rc * M.ncc);
  if (rc >= M.nrc) return;
  __shared__ double sQ[64][kMaxEll + 1];
  __shared__ double sY[64][kQRColChunk + 1];
  const int ell = M.ell, tid = threadIdx.x;
  const int pr = tid >> 4, tc = tid & 15;   // 16 x 16 threads over 64 x 64 outputs
  const TY* Y = static_cast<const TY*>(M.Y);
  const int64_t t0 = (int64_t)cc * kQRColChunk;
  const int cols = (int)min<int64_t>(kQRColChunk, M.s - t0);
  const int64_t r0 = (int64_t)rc * kQRRowChunk;
  const int64_t r1 = min<int64_t>(M.m, r0 + kQRRowChunk);
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int64_t s0 = r0; s0 < r1; s0 += 64) {
    const int rows = (int)min<int64_t>(64, r1 - s0);
    __syncthreads();
    for (int e = tid; e < 64 * kMaxEll; e += 256) {
      const int rr = e / kMaxEll, j = e - rr * kMaxEll;
      sQ[rr][j] = (rr < rows && j < ell) ? M.Z[(s0 + rr) * ell + j] : 0.0;
    }
    for (int e = tid; e < 64 * kQRColChunk; e += 256) {
      const int rr = e / kQRColChunk, t = e - rr * kQRColChunk;
      sY[rr][t] = (rr < rows && t < cols) ? to_double(Y[(s0 + rr) * M.s + t0 + t]) : 0.0;
    }
    __syncthreads();
    for (int rr = 0; rr < rows; ++rr) {
      double q[4], y[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) q[i] = sQ[rr][4 * pr + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) y[j] = sY[rr][4 * tc + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(q[i], y[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int p = 4 * pr + i;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = 4 * tc + j;
      if (p < ell && t < cols) M.mpart[((int64_t)rc * ell + p) * M.s + t0 + t] = acc[i][j];
    }
  }
}

// cpart[cc] = M_cc M_cc^T with M_cc = sum_rc mpart[rc][:, cc]
template <typename S>
__global__ __launch_bounds__(256) void mgram_kernel(const S b) {
  const QRMat& M = b.get(blockIdx.y);
  const int cc = blockIdx.x;
  if (cc >= M.ncc) return;
  __shared__ double sM[kMaxEll][kQRColChunk + 1];
  const int ell = M.ell, tid = threadIdx.x;
  const int64_t t0 = (int64_t)cc * kQRColChunk;
  const int cols = (int)min<int64_t>(kQRColChunk, M.s - t0);
  for (int e = tid; e < ell * kQRColChunk; e += 256) {
    const int p = e / kQRColChunk, t = e - p * kQRColChunk;
    double v = 0.0;
    if (t < cols)
      for (int rc = 0; rc < M.nrc; ++rc) v += M.mpart[((int64_t)rc * ell + p) * M.s + t0 + t];
    sM[p][t] = v;
  }
  __syncthreads();
  for (int e = tid; e < ell * ell; e += 256) {
    const int p = e / ell, q = e - p * ell;
    double a = 0.0;
    for (int t = 0; t < cols; ++t) a = fma(sM[p][t], sM[q][t], a);
    M.cpart[(int64_t)cc * ell * ell + e] = a;
  }
}

// Cyclic Jacobi (parallel round-robin ordering) on the summed ell x ell Gram;
// W = eigenvectors of the r largest eigenvalues, in descending order.
// One 256-thread workgroup per matrix: each round computes the ell/2
// disjoint rotations, then applies them to rows (A <- J^T A) and to columns
// (A <- A J, V <- V J); every thread owns a fixed set of (pair, index) items,
// precomputed once, so a round is three barriers and a few FMAs per thread.
// A rotation is skipped once |a_pq| <= 4 u max(|a_pp|, |a_qq|): the rotation
// it would apply is then below rounding level relative to the pair's own
// scale (a signal/noise pair is decoupled to ~u), whereas the stricter test
// |a_pq| <= u sqrt(a_pp a_qq) can be unreachable in floating point for
// strongly graded pairs.
constexpr int kEigThreads = 256;

template <typename S>
__global__ __launch_bounds__(kEigThreads) void eig_kernel(const S b) {
  const QRMat& M = b.get(blockIdx.x);
  __shared__ double A[kMaxEll][kMaxEll + 1];
  __shared__ double V[kMaxEll][kMaxEll + 1];
  __shared__ double rc_[kMaxEll / 2], rs_[kMaxEll / 2];
  __shared__ int rp_[kMaxEll / 2], rq_[kMaxEll / 2];
  __shared__ int rotations;   // any rotation in this sweep (written by wave 0)
  const int n = M.ell, np = n + (n & 1), half = np / 2, tid = threadIdx.x;
  // rotations stop below rounding level of the output precision (relative to
  // the pair's own scale): FP64 bases need ~u, FP32 bases ~1e-12 suffices
  const double tol = M.udtype == TK_F64 ? 4.0 * kUnit : 1e-12;
  // summed Gram: every thread's elements over groups of four column chunks,
  // all loads of a group in flight together (each element still sums the
  // chunks in index order)
  {
    constexpr int kE = kMaxEll * kMaxEll / kEigThreads;
    double v[kE];
#pragma unroll
    for (int k = 0; k < kE; ++k) v[k] = 0.0;
    for (int c0 = 0; c0 < M.ncc; c0 += 4) {
      double t[kE][4];
#pragma unroll
      for (int k = 0; k < kE; ++k) {
        const int e = tid + kEigThreads * k, p = e / np, q = e - (e / np) * np;
        const bool live = e < np * np && p < n && q < n;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          t[k][u] = (live && c0 + u < M.ncc) ? M.cpart[(int64_t)(c0 + u) * n * n + p * n + q] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < kE; ++k)
#pragma unroll
        for (int u = 0; u < 4; ++u) v[k] += t[k][u];
    }
#pragma unroll
    for (int k = 0; k < kE; ++k) {
      const int e = tid + kEigThreads * k;
      if (e < np * np) {
        const int p = e / np, q = e - p * np;
        A[p][q] = v[k];
        V[p][q] = p == q ? 1.0 : 0.0;
      }
    }
  }
  // this thread's items, in two loops of one kind each so a wave never runs
  // both kinds: the half x half 2x2 blocks of A (pair k1 rows, pair k2
  // columns: A <- J^T A J on the block) and the np x half column pairs of V
  // (V <- V J); codes k1 * 64 + k2 and k * 64 + i, or -1 past the end
  constexpr int kItemsA = (kMaxEll / 2) * (kMaxEll / 2) / kEigThreads;
  constexpr int kItemsV = kMaxEll * (kMaxEll / 2) / kEigThreads;
  int itemA[kItemsA], itemV[kItemsV];
  const int nblk = half * half, nv = np * half;
#pragma unroll
  for (int t = 0; t < kItemsA; ++t) {
    const int e = tid + kEigThreads * t;
    itemA[t] = e < nblk ? (e / half) * 64 + (e % half) : -1;
  }
#pragma unroll
  for (int t = 0; t < kItemsV; ++t) {
    const int e = tid + kEigThreads * t;
    itemV[t] = e < nv ? (e / np) * 64 + (e % np) : -1;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) rotations = 0;
    __syncthreads();
    for (int round = 0; round < np - 1; ++round) {
      bool rot = false;
      if (tid < half) {
        int p, q;
        if (tid == 0) { p = np - 1; q = round; }
        else {
          p = round + tid; if (p >= np - 1) p -= np - 1;
          q = round - tid; if (q < 0) q += np - 1;
        }
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p][q], app = A[p][p], aqq = A[q][q];
          if (fabs(apq) > tol * fmax(fabs(app), fabs(aqq))) {
            // t = tan of the rotation angle, the root of t^2 + 2 theta t - 1
            // of smaller magnitude, theta = (a_qq - a_pp) / (2 a_pq):
            // t = 2 a_pq / (d + sign(d) sqrt(d^2 + 4 a_pq^2)), d = a_qq - a_pp
            // (one square root and one division); c = 1 / sqrt(1 + t^2)
            const double d = aqq - app;
            const double root = sqrt(fma(d, d, 4.0 * apq * apq));
            const double t = (2.0 * apq) / (d >= 0.0 ? d + root : d - root);
            c = 1.0 / sqrt(fma(t, t, 1.0));
            s = t * c;
            rot = true;
          }
        }
        rc_[tid] = c; rs_[tid] = s; rp_[tid] = p; rq_[tid] = q;
      }
      if (tid < 64) {   // half <= 32: every rotation of the round is in wave 0
        const bool any = __any(rot);
        if (tid == 0 && any) rotations = 1;
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < kItemsA; ++t) {
        const int code = itemA[t];
        if (code < 0) break;
        const int k1 = code >> 6, k2 = code & 63;
        const double s1 = rs_[k1], s2 = rs_[k2];
        if (s1 != 0.0 || s2 != 0.0) {
          const double c1 = rc_[k1], c2 = rc_[k2];
          const int p1 = rp_[k1], q1 = rq_[k1], p2 = rp_[k2], q2 = rq_[k2];
          const double a = A[p1][p2], bb = A[p1][q2], cc = A[q1][p2], dd = A[q1][q2];
          // rows (J^T from the left), then columns (J from the right)
          const double ra = c1 * a - s1 * cc, rb = c1 * bb - s1 * dd;
          const double rc = s1 * a + c1 * cc, rd = s1 * bb + c1 * dd;
          A[p1][p2] = c2 * ra - s2 * rb;
          A[p1][q2] = s2 * ra + c2 * rb;
          A[q1][p2] = c2 * rc - s2 * rd;
          A[q1][q2] = s2 * rc + c2 * rd;
        }
      }
#pragma unroll
      for (int t = 0; t < kItemsV; ++t) {
        const int code = itemV[t];
        if (code < 0) break;
        const int k = code >> 6, i = code & 63;
        const double sv = rs_[k];
        if (sv != 0.0) {
          const double cv = rc_[k];
          const int p = rp_[k], q = rq_[k];
          const double vip = V[i][p], viq = V[i][q];
          V[i][p] = cv * vip - sv * viq;
          V[i][q] = sv * vip + cv * viq;
        }
      }
      __syncthreads();
    }
    const int done = rotations == 0;
    __syncthreads();
    if (done) break;
  }
  // rank of each eigenvalue in descending order (ties: lower index first)
  __shared__ int rank_of[kMaxEll];
  for (int i = tid; i < n; i += kEigThreads) {
    const double li = A[i][i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = A[j][j];
      rank += (lj > li) || (lj == li && j < i);
    }
    rank_of[i] = rank;
    if (rank < M.r && !M.small)
      for (int k = 0; k < n; ++k) M.W[k * M.r + rank] = V[k][i];
  }
  if (!M.small) return;
  __syncthreads();
  // W into A (A[k][rank] = V[k][i]), then U = Q W with the column sign rule
  for (int e = tid; e < n * n; e += kEigThreads) {
    const int k = e / n, i = e - k * n;
    if (rank_of[i] < M.r) A[k][rank_of[i]] = V[k][i];
  }
  __syncthreads();
  const int r = M.r;
  const int tpc = kEigThreads / r;            // threads per column
  const int j = tid % r, slot = tid / r;      // column and this thread's row slot
  const bool active = slot < tpc;
  __shared__ double sQ[32][kMaxEll + 1];
  double best = -1.0, bval = 0.0;
  int64_t bidx = INT64_MAX;
  const bool f64 = M.udtype == TK_F64;
  // rows of Q in chunks of 32, the next chunk's loads in flight (registers)
  // while the current one is multiplied
  constexpr int kPre = 32 * kMaxEll / kEigThreads;
  double pre[kPre];
  auto fetch = [&](int64_t r0) {
    const int rows = (int)min<int64_t>(32, M.m - r0);
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int e = tid + kEigThreads * u;
      pre[u] = (r0 < M.m && e < rows * n) ? M.Z[r0 * n + e] : 0.0;
    }
  };
  fetch(0);
  for (int64_t r0 = 0; r0 < M.m; r0 += 32) {
    const int rows = (int)min<int64_t>(32, M.m - r0);
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int e = tid + kEigThreads * u;
      if (e < rows * n) sQ[e / n][e % n] = pre[u];
    }
    fetch(r0 + 32);
    __syncthreads();
    if (active) {
      for (int rr = slot; rr < rows; rr += tpc) {
        double v = 0.0;
        for (int k = 0; k < n; ++k) v = fma(sQ[rr][k], A[k][j], v);
        const int64_t row = r0 + rr;
        if (fabs(v) > best) { best = fabs(v); bval = v; bidx = row; }  // rows ascend
        if (f64) static_cast<double*>(M.U)[row * r + j] = v;
        else static_cast<float*>(M.U)[row * r + j] = (float)v;
      }
    }
    __syncthreads();
  }
  // per column: largest |u|, lowest row on ties
  __shared__ double cand_v[kEigThreads], cand_a[kEigThreads];
  __shared__ int64_t cand_i[kEigThreads];
  __shared__ double sgn[kMaxEll];
  cand_a[tid] = active ? best : -1.0;
  cand_v[tid] = bval;
  cand_i[tid] = bidx;
  __syncthreads();
  if (tid < r) {
    double ba = -1.0, bv = 0.0;
    int64_t bi = INT64_MAX;
    for (int s2 = 0; s2 < tpc; ++s2) {
      const int t = s2 * r + tid;
      if (cand_a[t] > ba || (cand_a[t] == ba && cand_i[t] < bi)) {
        ba = cand_a[t]; bv = cand_v[t]; bi = cand_i[t];
      }
    }
    sgn[tid] = bv < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  // flip the columns that need it (exact in either storage type); each thread
  // rewrites only entries it wrote itself
  if (active && sgn[j] < 0.0) {
    for (int64_t row = slot; row < M.m; row += tpc) {
      if (f64) { double* U = static_cast<double*>(M.U); U[row * r + j] = -U[row * r + j]; }
      else { float* U = static_cast<float*>(M.U); U[row * r + j] = -U[row * r + j]; }
    }
  }
}

// utmp = Q W for a block of 64 rows, plus per-block column argmax of |u|.
template <typename S>
__global__ __launch_bounds__(64) void urows_kernel(const S b) {
  const QRMat& M = b.get(blockIdx.y);
  const int rb = blockIdx.x;
  if (rb >= M.nrb || M.small) return;
  __shared__ double sQ[kMaxEll][65];
  __shared__ double sW[kMaxEll][kMaxEll + 1];
  const int n = M.ell, r = M.r, lane = threadIdx.x;
  const int64_t r0 = (int64_t)rb * kQRRowBlock;
  const int rows = (int)min<int64_t>(kQRRowBlock, M.m - r0);
  for (int e = lane; e < rows * n; e += 64) {
    const int rr = e / n, j = e - rr * n;
    sQ[j][rr] = M.Z[(r0 + rr) * n + j];
  }
  for (int e = lane; e < n * r; e += 64) sW[e / r][e % r] = M.W[e];
  __syncthreads();
  for (int j = 0; j < r; ++j) {
    double u = 0.0;
    if (lane < rows) {
      for (int k = 0; k < n; ++k) u = fma(sQ[k][lane], sW[k][j], u);
      M.utmp[(r0 + lane) * r + j] = u;
    }
    // argmax of |u| over the block, lowest row on ties
    double best = lane < rows ? fabs(u) : -1.0;
    double val = u;
    int64_t idx = r0 + lane;
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const double ov = __shfl_xor(val, off);
      const int64_t oi = __shfl_xor(idx, off);
      if (ob > best || (ob == best && oi < idx)) { best = ob; val = ov; idx = oi; }
    }
    if (lane == 0) {
      M.amax_v[(int64_t)rb * r + j] = val;
      M.amax_i[(int64_t)rb * r + j] = idx;
    }
  }
}

template <typename TU, typename S>
__global__ __launch_bounds__(64) void usign_kernel(const S b) {
  const QRMat& M = b.get(blockIdx.y);
  const int rb = blockIdx.x;
  if (rb >= M.nrb || M.small) return;
  __shared__ double sgn[kMaxEll];
  const int r = M.r, lane = threadIdx.x;
  for (int j = 0; j < r; ++j) {
    double best = -1.0, val = 0.0;
    int64_t idx = INT64_MAX;
    for (int q = lane; q < M.nrb; q += 64) {
      const double v = M.amax_v[(int64_t)q * r + j];
      const int64_t i = M.amax_i[(int64_t)q * r + j];
      if (fabs(v) > best || (fabs(v) == best && i < idx)) { best = fabs(v); val = v; idx = i; }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const double ov = __shfl_xor(val, off);
      const int64_t oi = __shfl_xor(idx, off);
      if (ob > best || (ob == best && oi < idx)) { best = ob; val = ov; idx = oi; }
    }
    if (lane == 0) sgn[j] = val < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  const int64_t r0 = (int64_t)rb * kQRRowBlock;
  const int rows = (int)min<int64_t>(kQRRowBlock, M.m - r0);
  TU* U = static_cast<TU*>(M.U);
  for (int e = lane; e < rows * r; e += 64) {
    const int j = e % r;
    U[r0 * r + e] = from_double<TU>(sgn[j] * M.utmp[r0 * r + e]);
  }
}

int max_field(const QRMat* m, int count, int which) {
  int v = 0;
  for (int i = 0; i < count; ++i) v = max(v, which == 0 ? m[i].nrc : which == 1 ? m[i].ncc : m[i].nrb);
  return v;
}

// `src` gives the kernels the matrix descriptors (kernel arguments or a
// device table); `host` is the same table on the host, for the grid sizes
template <typename S>
hipError_t cholqr_impl(const S& src, const QRMat* host, int count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  const int nrc = max_field(host, count, 0), nrb = max_field(host, count, 2);
  bool any_small = false, any_big = false;
  for (int i = 0; i < count; ++i) (host[i].small ? any_small : any_big) = true;
  if (any_small) {
    int64_t lds = 0;
    for (int i = 0; i < count; ++i)
      if (host[i].small) lds = std::max<int64_t>(lds, host[i].m * host[i].ell * (int64_t)sizeof(double));
    hipLaunchKernelGGL(cholqr_small_kernel<S>, dim3(count), dim3(256), (size_t)lds, st, src);
  }
  if (!any_big) return hipGetLastError();
  // CholeskyQR2 needs two passes; every shifted pass owes two more plain ones,
  // so an exactly rank-deficient sketch (shift, shift, plain, plain) needs four.
  for (int pass = 1; pass <= kQRMaxPasses; ++pass) {
    hipLaunchKernelGGL(gram_partial_kernel<S>, dim3(nrc, count), dim3(256), 0, st, src, pass);
    hipLaunchKernelGGL(chol_kernel<S>, dim3(count), dim3(64), 0, st, src, pass);
    hipLaunchKernelGGL(apply_rinv_kernel<S>, dim3(nrb, count), dim3(64), 0, st, src, pass);
  }
  return hipGetLastError();
}

template <typename S>
hipError_t wstep_impl(const S& src, const QRMat* host, int count, int ydtype, int udtype, hipStream_t st) {
  if (count == 0) return hipSuccess;
  const int ncc = max_field(host, count, 1), nrb = max_field(host, count, 2);
  int64_t qty_blocks = 0;
  for (int i = 0; i < count; ++i) qty_blocks = host[i].qty_begin + (int64_t)host[i].nrc * host[i].ncc;
  const dim3 gq((unsigned)qty_blocks);
  switch (ydtype) {
    case TK_F64: hipLaunchKernelGGL((qty_partial_kernel<double, S>), gq, dim3(256), 0, st, src, count); break;
    case TK_F32: hipLaunchKernelGGL((qty_partial_kernel<float, S>), gq, dim3(256), 0, st, src, count); break;
    case TK_BF16: hipLaunchKernelGGL((qty_partial_kernel<bf16, S>), gq, dim3(256), 0, st, src, count); break;
    case TK_F16: hipLaunchKernelGGL((qty_partial_kernel<f16, S>), gq, dim3(256), 0, st, src, count); break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(mgram_kernel<S>, dim3(ncc, count), dim3(256), 0, st, src);
  hipLaunchKernelGGL(eig_kernel<S>, dim3(count), dim3(kEigThreads), 0, st, src);
  bool any_big = false;
  for (int i = 0; i < count; ++i) any_big |= !host[i].small;
  if (!any_big) return hipGetLastError();
  hipLaunchKernelGGL(urows_kernel<S>, dim3(nrb, count), dim3(64), 0, st, src);
  if (udtype == TK_F64)
    hipLaunchKernelGGL((usign_kernel<double, S>), dim3(nrb, count), dim3(64), 0, st, src);
  else
    hipLaunchKernelGGL((usign_kernel<float, S>), dim3(nrb, count), dim3(64), 0, st, src);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_cholqr(const QRBatch& b, hipStream_t st) { return cholqr_impl(b, b.m, b.count, st); }

hipError_t launch_wstep(const QRBatch& b, int ydtype, int udtype, hipStream_t st) {
  return wstep_impl(b, b.m, b.count, ydtype, udtype, st);
}

hipError_t launch_cholqr_list(const QRList& dev, const QRMat* host, hipStream_t st) {
  return cholqr_impl(dev, host, dev.count, st);
}

hipError_t launch_wstep_list(const QRList& dev, const QRMat* host, int ydtype, int udtype, hipStream_t st) {
  return wstep_impl(dev, host, dev.count, ydtype, udtype, st);
}

}  // namespace tk
