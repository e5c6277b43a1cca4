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
// Left-looking: lane q owns column q and step j forms
//   R[j][q] = (G[j][q] - sum_{k<j} R[k][j] R[k][q]) / R[j][j]   (q >= j),
// reading only rows k < j, which are final; the dot products keep four
// partial sums so their loads pipeline, and each step stores one entry per
// lane.  The lower triangle is not touched (the Gram is reloaded from
// registers for a shifted retry).
__device__ bool cholesky_upper_wave(double (*G)[kMaxEll + 1], int n, int lane, double tol) {
  const int q = lane;
  const bool mine = q < n;
  for (int j = 0; j < n; ++j) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (mine && q >= j) {
      int k = 0;
      for (; k + 4 <= j; k += 4) {
        s0 = fma(G[k][j], G[k][q], s0);
        s1 = fma(G[k + 1][j], G[k + 1][q], s1);
        s2 = fma(G[k + 2][j], G[k + 2][q], s2);
        s3 = fma(G[k + 3][j], G[k + 3][q], s3);
      }
      for (; k < j; ++k) s0 = fma(G[k][j], G[k][q], s0);
    }
    const double val = (mine && q >= j) ? G[j][q] - ((s0 + s1) + (s2 + s3)) : 0.0;
    const double piv = __shfl(val, j);
    if (!(piv > tol)) return false;  // uniform: every lane holds lane j's pivot
    const double rjj = sqrt(piv), inv = 1.0 / rjj;
    if (mine && q > j) G[j][q] = val * inv;
    if (q == j) G[j][j] = rjj;
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
// precomputed once.  The pairs of a round follow the fixed round-robin
// schedule, so every wave computes all of the round's rotations itself (no
// wave waits for another's parameters) and every thread derives its items'
// indices arithmetically; a round is two barriers, one batch of LDS loads
// per thread and the stores of the entries a rotation changes.
// A rotation is skipped once |a_pq| <= 4 u max(|a_pp|, |a_qq|): the rotation
// it would apply is then below rounding level relative to the pair's own
// scale (a signal/noise pair is decoupled to ~u), whereas the stricter test
// |a_pq| <= u sqrt(a_pp a_qq) can be unreachable in floating point for
// strongly graded pairs.
constexpr int kEigThreads = 256;
constexpr int kEigMaxSweeps = 60;

// IA, IV: A-block and V-pair items per thread, sized by the launcher for the
// widest sketch of the batch so the per-round loads are straight-line code
template <typename S, int IA, int IV, int E>
__global__ __launch_bounds__(kEigThreads) void eig_kernel(const S b) {
  const QRMat& M = b.get(blockIdx.x);
  __shared__ double A[E][E + 1];
  __shared__ double V[E][E + 1];
  // (c, s) of the current round's rotations, one copy per wave
  __shared__ double2 rot_cs[kEigThreads / 64][E / 2];
  const int n = M.ell, np = n + (n & 1), half = np / 2, tid = threadIdx.x;
  // rotations stop below rounding level of the output precision (relative to
  // the pair's own scale): FP64 bases need ~u, FP32 bases ~1e-12 suffices
  const double tol = M.udtype == TK_F64 ? 4.0 * kUnit : 1e-12;
  // summed Gram: every thread's elements over groups of four column chunks,
  // all loads of a group in flight together (each element still sums the
  // chunks in index order)
  {
    constexpr int kE = E * E / kEigThreads;
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
  constexpr int kItemsA = IA, kItemsV = IV;
  int itemA[kItemsA], itemV[kItemsV];
  const int nblk = half * half, nv = np * half;
#pragma unroll
  for (int t = 0; t < kItemsA; ++t) {
    const int e = tid + kEigThreads * t;
    itemA[t] = e < nblk ? (e / half) * 64 + (e % half) : -1;   // -1: none (loads a dummy)
  }
#pragma unroll
  for (int t = 0; t < kItemsV; ++t) {
    const int e = tid + kEigThreads * t;
    itemV[t] = e < nv ? (e / np) * 64 + (e % np) : -1;
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  // the pair (p < q) of rotation k in a round: fixed by the round-robin
  // ordering, so every thread computes it instead of reading it
  // (selects only: a branch here would split every item's loads)
  auto pair_of = [&](int k, int round, int& p, int& q) {
    const int m = np - 1;
    int a = round + k, c = round - k;
    a = a >= m ? a - m : a;
    c = c < 0 ? c + m : c;
    a = k == 0 ? m : a;
    c = k == 0 ? round : c;
    p = min(a, c);
    q = max(a, c);
  };
  // Pairs of two indices that currently rank below the r largest diagonal
  // entries are not rotated: such a rotation only mixes directions that are
  // dropped, so it changes neither the kept eigenvectors nor their decoupling.
  // Once no other pair rotates, a Gershgorin bound checks that the unreduced
  // block of those indices lies below every kept diagonal entry (so the kept
  // ones are the r largest eigenvalues); if it does not, full sweeps resume.
  bool skip_dropped = M.r < n;
  bool converged = false;
  for (int sweep = 0; sweep < kEigMaxSweeps; ++sweep) {
    bool rotated = false;   // any rotation in this sweep (wave-uniform, equal in every wave)
    uint64_t dropped = 0;   // indices ranked r or later by diagonal (ties: lower index first)
    if (skip_dropped) {
      bool d = false;
      if (lane < n) {
        const double di = A[lane][lane];
        int rk = 0;
        for (int j = 0; j < n; ++j) {
          const double dj = A[j][j];
          rk += (dj > di) || (dj == di && j < lane);
        }
        d = rk >= M.r;
      }
      dropped = __ballot(d);
    }
    for (int round = 0; round < np - 1; ++round) {
      // every wave computes the round's ell/2 disjoint rotations (lane k:
      // rotation k), so no wave waits for another's parameters
      bool rot_now = false;
      if (lane < half) {
        int p, q;
        pair_of(lane, round, p, q);
        double c = 1.0, sn = 0.0;
        if (q < n && !(((dropped >> p) & 1) && ((dropped >> q) & 1))) {
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
            sn = t * c;
            rot_now = true;
          }
        }
        rot_cs[wave][lane] = make_double2(c, sn);
      }
      // identical in every wave, so every wave takes the same branch
      const bool round_rot = __any(rot_now);
      rotated |= round_rot;
      __syncthreads();   // every read of A for the rotations is done
      if (!round_rot) continue;
      // every load of this thread's items first (straight-line: an absent
      // item loads the entries of block (0, 0)), then the updates; an item
      // whose rotations are both the identity stores nothing
      double blk[kItemsA][4], vv[kItemsV][2];
      double2 r1[kItemsA], r2[kItemsA], rv[kItemsV];
      int ia[kItemsA][4], iv[kItemsV][3];
#pragma unroll
      for (int t = 0; t < kItemsA; ++t) {
        const int code = itemA[t] < 0 ? 0 : itemA[t];
        const int k1 = code >> 6, k2 = code & 63;
        pair_of(k1, round, ia[t][0], ia[t][1]);
        pair_of(k2, round, ia[t][2], ia[t][3]);
        r1[t] = rot_cs[wave][k1];
        r2[t] = rot_cs[wave][k2];
        blk[t][0] = A[ia[t][0]][ia[t][2]];
        blk[t][1] = A[ia[t][0]][ia[t][3]];
        blk[t][2] = A[ia[t][1]][ia[t][2]];
        blk[t][3] = A[ia[t][1]][ia[t][3]];
      }
#pragma unroll
      for (int t = 0; t < kItemsV; ++t) {
        const int code = itemV[t] < 0 ? 0 : itemV[t];
        const int k = code >> 6;
        iv[t][0] = code & 63;
        pair_of(k, round, iv[t][1], iv[t][2]);
        rv[t] = rot_cs[wave][k];
        vv[t][0] = V[iv[t][0]][iv[t][1]];
        vv[t][1] = V[iv[t][0]][iv[t][2]];
      }
#pragma unroll
      for (int t = 0; t < kItemsA; ++t) {
        if (itemA[t] >= 0 && (r1[t].y != 0.0 || r2[t].y != 0.0)) {
          const double c1 = r1[t].x, s1 = r1[t].y, c2 = r2[t].x, s2 = r2[t].y;
          const double a = blk[t][0], bb = blk[t][1], cc = blk[t][2], dd = blk[t][3];
          // rows (J^T from the left), then columns (J from the right)
          const double ra = c1 * a - s1 * cc, rb = c1 * bb - s1 * dd;
          const double rc = s1 * a + c1 * cc, rd = s1 * bb + c1 * dd;
          A[ia[t][0]][ia[t][2]] = c2 * ra - s2 * rb;
          A[ia[t][0]][ia[t][3]] = s2 * ra + c2 * rb;
          A[ia[t][1]][ia[t][2]] = c2 * rc - s2 * rd;
          A[ia[t][1]][ia[t][3]] = s2 * rc + c2 * rd;
        }
      }
#pragma unroll
      for (int t = 0; t < kItemsV; ++t) {
        if (itemV[t] >= 0 && rv[t].y != 0.0) {
          const double cv = rv[t].x, sv = rv[t].y;
          const double vip = vv[t][0], viq = vv[t][1];
          V[iv[t][0]][iv[t][1]] = cv * vip - sv * viq;
          V[iv[t][0]][iv[t][2]] = sv * vip + cv * viq;
        }
      }
      __syncthreads();
    }
    if (!rotated) {
      converged = true;
      if (dropped == 0) break;
      double top_min = INFINITY, drop_max = -INFINITY;
      if (lane < n) {
        const double di = A[lane][lane];
        if ((dropped >> lane) & 1) {
          double rad = 0.0;
          for (int j = 0; j < n; ++j)
            if (j != lane && ((dropped >> j) & 1)) rad += fabs(A[lane][j]);
          drop_max = di + rad;
        } else {
          top_min = di;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        top_min = fmin(top_min, __shfl_xor(top_min, off));
        drop_max = fmax(drop_max, __shfl_xor(drop_max, off));
      }
      if (drop_max < top_min) break;
      converged = false;
      skip_dropped = false;
    }
  }
  // sweeps exhausted with rotations still firing: W may be inaccurate
  if (!converged && tid == 0 && M.info) *M.info |= 8;
  // rank of each eigenvalue in descending order (ties: lower index first)
  __shared__ int rank_of[E];
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
  __shared__ double sQ[32][E + 1];
  double best = -1.0, bval = 0.0;
  int64_t bidx = INT64_MAX;
  const bool f64 = M.udtype == TK_F64;
  // rows of Q in chunks of 32, the next chunk's loads in flight (registers)
  // while the current one is multiplied
  constexpr int kPre = 32 * E / kEigThreads;
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
  __shared__ double sgn[E];
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
  // (eight loads in flight, then the eight stores)
  if (active && sgn[j] < 0.0) {
    constexpr int kB = 8;
    for (int64_t row0 = slot; row0 < M.m; row0 += (int64_t)kB * tpc) {
      double u[kB];
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        const int64_t row = row0 + (int64_t)q * tpc;
        if (row < M.m)
          u[q] = f64 ? static_cast<const double*>(M.U)[row * r + j]
                     : (double)static_cast<const float*>(M.U)[row * r + j];
      }
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        const int64_t row = row0 + (int64_t)q * tpc;
        if (row < M.m) {
          if (f64) static_cast<double*>(M.U)[row * r + j] = -u[q];
          else static_cast<float*>(M.U)[row * r + j] = (float)-u[q];
        }
      }
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

// gram_given: every matrix's cpart already holds the Gram of Q^T Y (ncc = 1),
// so the Q^T Y and Gram kernels are skipped
template <typename S>
hipError_t wstep_impl(const S& src, const QRMat* host, int count, int ydtype, int udtype, hipStream_t st,
                      bool gram_given = false) {
  if (count == 0) return hipSuccess;
  const int ncc = max_field(host, count, 1), nrb = max_field(host, count, 2);
  int64_t qty_blocks = 0;
  for (int i = 0; i < count; ++i) qty_blocks = host[i].qty_begin + (int64_t)host[i].nrc * host[i].ncc;
  if (!gram_given) {
    const dim3 gq((unsigned)qty_blocks);
    switch (ydtype) {
      case TK_F64: hipLaunchKernelGGL((qty_partial_kernel<double, S>), gq, dim3(256), 0, st, src, count); break;
      case TK_F32: hipLaunchKernelGGL((qty_partial_kernel<float, S>), gq, dim3(256), 0, st, src, count); break;
      case TK_BF16: hipLaunchKernelGGL((qty_partial_kernel<bf16, S>), gq, dim3(256), 0, st, src, count); break;
      case TK_F16: hipLaunchKernelGGL((qty_partial_kernel<f16, S>), gq, dim3(256), 0, st, src, count); break;
      default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(mgram_kernel<S>, dim3(ncc, count), dim3(256), 0, st, src);
  }
  // items per thread for the widest sketch: half^2 A blocks and np * half V pairs
  int ellmax = 1;
  for (int i = 0; i < count; ++i) ellmax = std::max(ellmax, host[i].ell);
  const int np = ellmax + (ellmax & 1), half = np / 2;
  const int ia = (int)ceil_div((int64_t)half * half, kEigThreads);
  const int iv = (int)ceil_div((int64_t)np * half, kEigThreads);
  // LDS sized for the widest sketch too (E = 32 or 64): narrow sketches then
  // fit several workgroups per CU, which a batch of many matrices needs
  if (np <= 32)
    hipLaunchKernelGGL((eig_kernel<S, 1, 2, 32>), dim3(count), dim3(kEigThreads), 0, st, src);
  else if (ia <= 2 && iv <= 4)
    hipLaunchKernelGGL((eig_kernel<S, 2, 4, 64>), dim3(count), dim3(kEigThreads), 0, st, src);
  else if (ia <= 3 && iv <= 6)
    hipLaunchKernelGGL((eig_kernel<S, 3, 6, 64>), dim3(count), dim3(kEigThreads), 0, st, src);
  else
    hipLaunchKernelGGL((eig_kernel<S, 4, 8, 64>), dim3(count), dim3(kEigThreads), 0, st, src);
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

hipError_t launch_wstep_gram(const QRBatch& b, int udtype, hipStream_t st) {
  return wstep_impl(b, b.m, b.count, TK_F64, udtype, st, true);
}

hipError_t launch_cholqr_list(const QRList& dev, const QRMat* host, hipStream_t st) {
  return cholqr_impl(dev, host, dev.count, st);
}

hipError_t launch_wstep_list(const QRList& dev, const QRMat* host, int ydtype, int udtype, hipStream_t st) {
  return wstep_impl(dev, host, dev.count, ydtype, udtype, st);
}

}  // namespace tk
