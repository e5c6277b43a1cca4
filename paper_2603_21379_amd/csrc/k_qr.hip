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
__global__ __launch_bounds__(256) void gram_partial_kernel(const QRBatch b, int pass) {
  const QRMat& M = b.m[blockIdx.y];
  const int rc = blockIdx.x;
  if (rc >= M.nrc) return;
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
__global__ __launch_bounds__(64) void chol_kernel(const QRBatch b, int pass) {
  const QRMat& M = b.m[blockIdx.x];
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
__global__ __launch_bounds__(64) void apply_rinv_kernel(const QRBatch b, int pass) {
  const QRMat& M = b.m[blockIdx.y];
  const int rb = blockIdx.x;
  if (rb >= M.nrb) return;
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

// ------------------------------------------------------------------ W step
// mpart[rc][p][t] = sum_{rows in rc} Q[row][p] Y[row][t], t in column chunk cc
template <typename TY>
__global__ __launch_bounds__(256) void qty_partial_kernel(const QRBatch b) {
  const QRMat& M = b.m[blockIdx.z];
  const int rc = blockIdx.x, cc = blockIdx.y;
  if (rc >= M.nrc || cc >= M.ncc) return;
  __shared__ double sQ[64][kMaxEll + 1];
  __shared__ double sY[64][kQRColChunk + 1];
  const int ell = M.ell, tid = threadIdx.x;
  const TY* Y = static_cast<const TY*>(M.Y);
  const int64_t t0 = (int64_t)cc * kQRColChunk;
  const int cols = (int)min<int64_t>(kQRColChunk, M.s - t0);
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
      sQ[rr][j] = rr < rows ? M.Z[(s0 + rr) * ell + j] : 0.0;
    }
    for (int e = tid; e < 64 * kQRColChunk; e += 256) {
      const int rr = e / kQRColChunk, t = e - rr * kQRColChunk;
      sY[rr][t] = (rr < rows && t < cols) ? to_double(Y[(s0 + rr) * M.s + t0 + t]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q;  // e = p * 64 + t
      const int p = e >> 6, t = e & 63;
      if (p < ell) {
        double a = acc[q];
        for (int rr = 0; rr < rows; ++rr) a = fma(sQ[rr][p], sY[rr][t], a);
        acc[q] = a;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q;
    const int p = e >> 6, t = e & 63;
    if (p < ell && t < cols) M.mpart[((int64_t)rc * ell + p) * M.s + t0 + t] = acc[q];
  }
}

// cpart[cc] = M_cc M_cc^T with M_cc = sum_rc mpart[rc][:, cc]
__global__ __launch_bounds__(256) void mgram_kernel(const QRBatch b) {
  const QRMat& M = b.m[blockIdx.y];
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
// Lane j owns column j of the row updates and row j of the column updates, so
// a round is three passes over the ell/2 disjoint rotations with no index
// arithmetic.  A rotation is skipped once |a_pq| <= 4 u max(|a_pp|, |a_qq|):
// the rotation it would apply is then below rounding level relative to the
// pair's own scale (so a signal/noise pair is decoupled to ~u), while the
// stricter test |a_pq| <= u sqrt(a_pp a_qq) can be unreachable in floating
// point for strongly graded pairs.
__global__ __launch_bounds__(64) void eig_kernel(const QRBatch b) {
  const QRMat& M = b.m[blockIdx.x];
  __shared__ double A[kMaxEll][kMaxEll + 1];
  __shared__ double V[kMaxEll][kMaxEll + 1];
  __shared__ double rc_[kMaxEll / 2], rs_[kMaxEll / 2];
  __shared__ int rp_[kMaxEll / 2], rq_[kMaxEll / 2];
  __shared__ int rotations;
  const int n = M.ell, np = n + (n & 1), half = np / 2, lane = threadIdx.x;
  for (int e = lane; e < np * np; e += 64) {
    const int p = e / np, q = e - p * np;
    double v = 0.0;
    if (p < n && q < n)
      for (int c = 0; c < M.ncc; ++c) v += M.cpart[(int64_t)c * n * n + p * n + q];
    A[p][q] = v;
    V[p][q] = p == q ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (lane == 0) rotations = 0;
    __syncthreads();
    for (int round = 0; round < np - 1; ++round) {
      if (lane < half) {
        int p, q;
        if (lane == 0) { p = np - 1; q = round; }
        else {
          p = round + lane; if (p >= np - 1) p -= np - 1;
          q = round - lane; if (q < 0) q += np - 1;
        }
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p][q], app = A[p][p], aqq = A[q][q];
          const double aa = fabs(apq);
          if (aa > 4.0 * kUnit * fmax(fabs(app), fabs(aqq))) {
            const double th = (aqq - app) / (2.0 * apq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            atomicAdd(&rotations, 1);
          }
        }
        rc_[lane] = c; rs_[lane] = s; rp_[lane] = p; rq_[lane] = q;
      }
      __syncthreads();
      if (lane < np) {          // rows p, q of every pair: A <- J^T A
        const int j = lane;
        for (int k = 0; k < half; ++k) {
          const double s = rs_[k];
          if (s != 0.0) {
            const double c = rc_[k];
            const int p = rp_[k], q = rq_[k];
            const double apj = A[p][j], aqj = A[q][j];
            A[p][j] = c * apj - s * aqj;
            A[q][j] = s * apj + c * aqj;
          }
        }
      }
      __syncthreads();
      if (lane < np) {          // columns p, q: A <- A J, V <- V J
        const int i = lane;
        for (int k = 0; k < half; ++k) {
          const double s = rs_[k];
          if (s != 0.0) {
            const double c = rc_[k];
            const int p = rp_[k], q = rq_[k];
            const double aip = A[i][p], aiq = A[i][q];
            A[i][p] = c * aip - s * aiq;
            A[i][q] = s * aip + c * aiq;
            const double vip = V[i][p], viq = V[i][q];
            V[i][p] = c * vip - s * viq;
            V[i][q] = s * vip + c * viq;
          }
        }
      }
      __syncthreads();
    }
    const int done = rotations == 0;
    __syncthreads();
    if (done) break;
  }
  // rank of each eigenvalue in descending order (ties: lower index first)
  for (int i = lane; i < n; i += 64) {
    const double li = A[i][i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = A[j][j];
      rank += (lj > li) || (lj == li && j < i);
    }
    if (rank < M.r)
      for (int k = 0; k < n; ++k) M.W[k * M.r + rank] = V[k][i];
  }
}

// utmp = Q W for a block of 64 rows, plus per-block column argmax of |u|.
__global__ __launch_bounds__(64) void urows_kernel(const QRBatch b) {
  const QRMat& M = b.m[blockIdx.y];
  const int rb = blockIdx.x;
  if (rb >= M.nrb) return;
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

template <typename TU>
__global__ __launch_bounds__(64) void usign_kernel(const QRBatch b) {
  const QRMat& M = b.m[blockIdx.y];
  const int rb = blockIdx.x;
  if (rb >= M.nrb) return;
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

int max_field(const QRBatch& b, int which) {
  int v = 0;
  for (int i = 0; i < b.count; ++i) {
    const QRMat& M = b.m[i];
    v = max(v, which == 0 ? M.nrc : which == 1 ? M.ncc : M.nrb);
  }
  return v;
}

}  // namespace

hipError_t launch_cholqr(const QRBatch& b, hipStream_t st) {
  if (b.count == 0) return hipSuccess;
  const int nrc = max_field(b, 0), nrb = max_field(b, 2);
  // CholeskyQR2 needs two passes; every shifted pass owes two more plain ones,
  // so an exactly rank-deficient sketch (shift, shift, plain, plain) needs four.
  for (int pass = 1; pass <= kQRMaxPasses; ++pass) {
    hipLaunchKernelGGL(gram_partial_kernel, dim3(nrc, b.count), dim3(256), 0, st, b, pass);
    hipLaunchKernelGGL(chol_kernel, dim3(b.count), dim3(64), 0, st, b, pass);
    hipLaunchKernelGGL(apply_rinv_kernel, dim3(nrb, b.count), dim3(64), 0, st, b, pass);
  }
  return hipGetLastError();
}

template <typename TY>
static void launch_qty(const QRBatch& b, int nrc, int ncc, hipStream_t st) {
  hipLaunchKernelGGL((qty_partial_kernel<TY>), dim3(nrc, ncc, b.count), dim3(256), 0, st, b);
}

hipError_t launch_wstep(const QRBatch& b, int ydtype, int udtype, hipStream_t st) {
  if (b.count == 0) return hipSuccess;
  const int nrc = max_field(b, 0), ncc = max_field(b, 1), nrb = max_field(b, 2);
  switch (ydtype) {
    case TK_F64: launch_qty<double>(b, nrc, ncc, st); break;
    case TK_F32: launch_qty<float>(b, nrc, ncc, st); break;
    case TK_BF16: launch_qty<bf16>(b, nrc, ncc, st); break;
    case TK_F16: launch_qty<f16>(b, nrc, ncc, st); break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(mgram_kernel, dim3(ncc, b.count), dim3(256), 0, st, b);
  hipLaunchKernelGGL(eig_kernel, dim3(b.count), dim3(64), 0, st, b);
  hipLaunchKernelGGL(urows_kernel, dim3(nrb, b.count), dim3(64), 0, st, b);
  if (udtype == TK_F64)
    hipLaunchKernelGGL((usign_kernel<double>), dim3(nrb, b.count), dim3(64), 0, st, b);
  else
    hipLaunchKernelGGL((usign_kernel<float>), dim3(nrb, b.count), dim3(64), 0, st, b);
  return hipGetLastError();
}

}  // namespace tk
