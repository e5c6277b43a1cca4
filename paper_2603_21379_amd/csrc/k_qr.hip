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
// kQRSmallElems), Z resident in LDS:
//  * Gram G = Z^T Z on v_mfma_f64_16x16x4f64 (wave w: tiles w, w + 4, ... of
//    the 16 x 16 tiling; lane l supplies Z[k0 + l/16][16 t + l%16] for both
//    operands, register v of the result is row 16 ti + l/16 + 4 v, column
//    16 tj + l%16);
//  * upper Cholesky factor R by one wave, right-looking, lane q holding
//    column q of G in registers; row j of R goes through LDS to every lane
//    for the rank-one update;
//  * X = R^{-1} by one wave (lane j: column j in registers), written
//    transposed over the unused lower triangle of the array that holds R;
//  * Q = Z X on MFMA, each wave overwriting its own 16-row tiles of Z.
// Same passes, shift rule and info bits as the multi-kernel path.

// Within one wavefront LDS operations complete in issue order, so lanes of
// that wave only need the compiler kept from reordering across this point.
#define TK_WAVE_SYNC()                          \
  do {                                          \
    __atomic_signal_fence(__ATOMIC_SEQ_CST);    \
    __builtin_amdgcn_wave_barrier();            \
    __atomic_signal_fence(__ATOMIC_SEQ_CST);    \
  } while (0)

typedef double doublex4 __attribute__((ext_vector_type(4)));

// 1 / x and 1 / sqrt(x) for normal positive x: the hardware estimates and
// two Newton steps (within 2 u; no division or square-root sequence with its
// range scaling on a chain of dependent steps)
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  return fma(y, fma(-x, y, 1.0), y);
}
__device__ __forceinline__ double rsq_nr(double x) {
  const double hx = 0.5 * x;
  double y = __builtin_amdgcn_rsq(x);
  y *= fma(-hx * y, y, 1.5);
  return y * fma(-hx * y, y, 1.5);
}
__device__ __forceinline__ double lane_value(double v, int i) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), i);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), i);
  return __hiloint2double(hi, lo);
}

// Upper Cholesky factor of G (n x n in LDS, zero past n in an E x E array,
// E >= n) by the 64 lanes of one wave.  Lane q keeps column q in registers;
// step j takes the pivot from lane j, forms row j of R (zero left of the
// diagonal, so that column q ends up holding exactly column q of R), passes
// it to every lane through rowbuf and applies the rank-one update to the
// trailing columns.  A pivot not above tol fails the factorization (returns
// false) unless `force`, which keeps the solve finite with r_jj = 1 instead.
// On return with success or `force`, G holds R (zero below the diagonal and
// past n) and rinv[j] = 1 / r_jj (zero past n).
template <int E>
__device__ __forceinline__ bool chol_wave(double (*G)[E + 1], int n, int lane, double tol, bool force,
                                          double* rowbuf, double* rinv) {
  const int q = lane < E ? lane : E - 1;   // lanes past E mirror column E - 1 and store nothing
  double col[E];
#pragma unroll
  for (int p = 0; p < E; ++p) col[p] = G[p][q];
  bool good = true;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    if (j < n && good) {
      const double piv = lane_value(col[j], j);
      double rj = 1.0, inv = 1.0;
      if (piv > tol && piv >= 2.2250738585072014e-308) {
        inv = rsq_nr(piv);
        rj = piv * inv;
      } else if (!force) {
        good = false;
      }
      if (good) {
        int lj = lane;
        asm volatile("" : "+v"(lj));   // the compares below stay in this step
        const double rjq = lj > j ? col[j] * inv : (lj == j ? rj : 0.0);
        col[j] = rjq;
        TK_WAVE_SYNC();   // the previous step's reads of rowbuf are done
        rowbuf[lane] = rjq;
        TK_WAVE_SYNC();
        if constexpr (E <= 48) {
          // row j of R: every load issued before the updates
          double rj_row[E];
#pragma unroll
          for (int p = j + 1; p < E; ++p) rj_row[p] = rowbuf[p];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int p = j + 1; p < E; ++p) col[p] = fma(-rj_row[p], rjq, col[p]);
          __builtin_amdgcn_sched_barrier(0);
        } else {
          // (64 columns: a second register row would not fit)
#pragma unroll
          for (int p = j + 1; p < E; ++p) col[p] = fma(-rowbuf[p], rjq, col[p]);
        }
        if (lane == 0) rinv[j] = inv;
      }
    }
  }
  if (!good) return false;
  TK_WAVE_SYNC();   // every lane has read G
  if (lane < E) {
#pragma unroll
    for (int p = 0; p < E; ++p) G[p][lane] = col[p];
    if (lane >= n) rinv[lane] = 0.0;
  }
  TK_WAVE_SYNC();
  return true;
}

template <typename S, int E>
__global__ __launch_bounds__(256) void cholqr_small_kernel(const S b) {
  const QRMat& M = b.get(blockIdx.x);
  if (!M.small) return;
  // Z stays in LDS for every pass (row stride ell, then 4 ell + E zeros so
  // that the Gram's row groups and a row's registers can run past the end
  // without a bound check): one coalesced read at the start, one write of Q
  // at the end
  extern __shared__ double sZ[];
  __shared__ double G[E][E + 1];
  __shared__ double rowbuf[64], rinv[E];
  __shared__ double red[2];
  __shared__ int ok;
  const int n = M.ell, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int l16 = lane & 15, g = lane >> 4;
  const int64_t m = M.m, mn = m * n;
  for (int64_t e = tid; e < mn; e += 256) sZ[e] = M.Z[e];
  for (int64_t e = tid; e < 4 * n + E; e += 256) sZ[mn + e] = 0.0;
  for (int e = tid; e < E * (E + 1); e += 256) (&G[0][0])[e] = 0.0;
  __syncthreads();
  int owed = 2, info = 0;
  for (int pass = 1; pass <= kQRMaxPasses && owed > 0; ++pass) {
    // Gram on MFMA: wave w takes the row groups 4 k + (0..3), k = w, w + 4,
    // ..., eight groups at a time with all their loads issued first, and
    // accumulates every tile (ti <= tj) of the upper triangle in its own
    // accumulator (independent chains); the loads need no bounds: columns
    // past n read the next row (those tiles' entries past n are not kept)
    // and rows past m read the zero padding
    {
      constexpr int kT = E / 16, kTiles = kT * (kT + 1) / 2, kB = 8;
      doublex4 acc[kTiles];
#pragma unroll
      for (int t = 0; t < kTiles; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
      for (int64_t k0 = 4 * wave; k0 < m; k0 += 16 * kB) {
        double zt[kB][kT];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          // groups past m start in the padding or beyond: read row m - 1's
          // neighbourhood instead and contribute zero
          const int64_t row = k0 + 16 * u + g;
          const bool live = k0 + 16 * u < m;
          const double* zr = sZ + (live ? row : 0) * n + l16;
#pragma unroll
          for (int t = 0; t < kT; ++t) zt[u][t] = live ? zr[16 * t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          int t = 0;
#pragma unroll
          for (int ti = 0; ti < kT; ++ti)
#pragma unroll
            for (int tj = ti; tj < kT; ++tj, ++t)
              acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(zt[u][ti], zt[u][tj], acc[t], 0, 0, 0);
        }
      }
      // the four waves' partial tiles, summed in wave order
      for (int w = 0; w < 4; ++w) {
        if (wave == w) {
          int t = 0;
#pragma unroll
          for (int ti = 0; ti < kT; ++ti)
#pragma unroll
            for (int tj = ti; tj < kT; ++tj, ++t)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int pr = 16 * ti + g + 4 * v, qc = 16 * tj + l16;
                if (pr < n && qc < n) {
                  const double x = w == 0 ? acc[t][v] : G[pr][qc] + acc[t][v];
                  G[pr][qc] = x;
                  if (w == 3 && ti != tj) G[qc][pr] = x;
                }
              }
        }
        __syncthreads();
      }
    }
    if (tid == 0) {
      double mx = 0.0, tr = 0.0;
      for (int j = 0; j < n; ++j) { mx = fmax(mx, G[j][j]); tr += G[j][j]; }
      red[0] = mx;
      red[1] = tr;
    }
    __syncthreads();
    const double mx = red[0], tr = red[1];
    // Cholesky by wave 0; on failure again with the shift of shifted
    // CholeskyQR (Fukaya et al. 2020): s = 11 (m n + n (n+1)) u ||Z||^2, with
    // ||Z||_2^2 bounded by the trace of the Gram
    if (wave == 0) {
      int status = 0;
      if (!(mx > 0.0 && chol_wave<E>(G, n, lane, 1e-14 * mx, false, rowbuf, rinv))) {
        const double shift = 11.0 * ((double)m * n + (double)n * (n + 1)) * kUnit * fmax(tr, 1e-300);
        if (lane < n) G[lane][lane] += shift;
        TK_WAVE_SYNC();
        status = chol_wave<E>(G, n, lane, 0.0, false, rowbuf, rinv) ? 1 : 2;
        if (status == 2) chol_wave<E>(G, n, lane, 0.0, true, rowbuf, rinv);   // finite; flagged
      }
      if (lane == 0) ok = status;
    }
    __syncthreads();
    // X = R^{-1} by wave 0 (lane j: column j of X in registers, rows
    // descending), written transposed below the diagonal of G (R, above it,
    // is read only; the diagonal 1 / r_jj is rinv):
    //   x_ij = (delta_ij - sum_{k>i} r_ik x_kj) / r_ii
    // (rows past j come out zero: every x_kj with k > i > j is zero)
    if (wave == 0 && lane < E) {
      double x[E];
#pragma unroll
      for (int i = E - 1; i >= 0; --i) {
        // delta_ij as a 0/1 factor from integer arithmetic (a compare here
        // would be kept as a mask for every row at once)
        const double delta = (double)(1 - min(1, abs(lane - i)));
        if constexpr (E <= 48) {
          // row i of R: every load issued before the products
          double ri[E];
#pragma unroll
          for (int k = i + 1; k < E; ++k) ri[k] = G[i][k];
          const double rii = rinv[i];
          __builtin_amdgcn_sched_barrier(0);
          double s0 = 0.0, s1 = 0.0;
#pragma unroll
          for (int k = i + 1; k < E; ++k) {
            if ((k - i) & 1) s0 = fma(ri[k], x[k], s0);
            else s1 = fma(ri[k], x[k], s1);
          }
          x[i] = (delta - (s0 + s1)) * rii;
          __builtin_amdgcn_sched_barrier(0);
        } else {
          // (64 columns: a register row of R would not fit beside x)
          double s0 = 0.0, s1 = 0.0;
#pragma unroll
          for (int k = i + 1; k < E; ++k) {
            if ((k - i) & 1) s0 = fma(G[i][k], x[k], s0);
            else s1 = fma(G[i][k], x[k], s1);
          }
          x[i] = (delta - (s0 + s1)) * rinv[i];
          if ((i & 3) == 0) __builtin_amdgcn_sched_barrier(0);
        }
      }
      TK_WAVE_SYNC();   // every read of R is done
#pragma unroll
      for (int i = 0; i < E; ++i)
        if (i < lane) G[lane][i] = x[i];
    }
    __syncthreads();
    // Q = Z X on MFMA, in place: wave w takes the 16-row tiles w, w + 4, ...
    // (each reads and writes only its own rows); lane l supplies
    // Z[r0 + l%16][k0 + l/16] and X[k0 + l/16][16 ct + l%16].  X's operands
    // are loaded once, a tile's Z operands all before its multiplies.
    {
      constexpr int kT = E / 16, kK = E / 4;
      double xb[kK][kT];
#pragma unroll
      for (int ks = 0; ks < kK; ++ks)
#pragma unroll
        for (int ct = 0; ct < kT; ++ct) {
          const int k = 4 * ks + g, j = 16 * ct + l16;
          xb[ks][ct] = k < j ? G[j][k] : (k == j ? rinv[j] : 0.0);
        }
      for (int64_t r0 = 16 * wave; r0 < m; r0 += 64) {
        const int64_t arow = r0 + l16;
        const bool rowok = arow < m;
        double a[kK];
#pragma unroll
        for (int ks = 0; ks < kK; ++ks) {
          const int k = 4 * ks + g;
          a[ks] = (rowok && k < n) ? sZ[arow * n + k] : 0.0;
        }
        doublex4 acc[kT];
#pragma unroll
        for (int ct = 0; ct < kT; ++ct) acc[ct] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < kK; ++ks)
#pragma unroll
          for (int ct = 0; ct < kT; ++ct)
            acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], xb[ks][ct], acc[ct], 0, 0, 0);
        __builtin_amdgcn_wave_barrier();   // the wave's reads of these rows precede its writes
#pragma unroll
        for (int ct = 0; ct < kT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t row = r0 + g + 4 * v;
            const int j = 16 * ct + l16;
            if (row < m && j < n) sZ[row * n + j] = acc[ct][v];
          }
      }
    }
    __syncthreads();
    const int status = ok;
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

// Small matrices (m x ell in one workgroup's reach), both products of the
// Gram of M = Q^T Y in one kernel on v_mfma_f64_16x16x4f64, one workgroup per
// 64-column chunk cc of Y:
//   M_cc = Q^T Y[:, cc]   (ell x 64, K = m; wave w: columns 16 w .., every
//                          16-row tile of ell; eight K steps of loads in
//                          flight ahead of their multiplies)
//   cpart[cc] = M_cc M_cc^T (K = 64, M_cc through LDS; wave w: tiles w,
//                          w + 4, ... of the upper triangle)
template <typename TY, typename S>
__global__ __launch_bounds__(256) void qty_gram_kernel(const S b) {
  const QRMat& M = b.get(blockIdx.y);
  const int cc = blockIdx.x;
  if (cc >= M.ncc) return;
  __shared__ double sM[kMaxEll][kQRColChunk + 1];
  const int ell = M.ell, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int l16 = lane & 15, g = lane >> 4;
  const int nt = (ell + 15) / 16;
  const TY* Y = static_cast<const TY*>(M.Y);
  const int64_t t = (int64_t)cc * kQRColChunk + 16 * wave + l16;   // this lane's column of Y
  const bool tok = t < M.s;
  constexpr int kMT = kMaxEll / 16, kB = 8;
  doublex4 acc[kMT];
#pragma unroll
  for (int pt = 0; pt < kMT; ++pt) acc[pt] = doublex4{0.0, 0.0, 0.0, 0.0};
  auto fetch = [&](int64_t k0, double (&qa)[kB][kMT], double (&yb)[kB]) {
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int64_t k = k0 + 4 * u + g;
      const bool kok = k < M.m;
      yb[u] = (kok && tok) ? to_double(Y[k * M.s + t]) : 0.0;
#pragma unroll
      for (int pt = 0; pt < kMT; ++pt) {
        const int p = 16 * pt + l16;
        qa[u][pt] = (kok && pt < nt && p < ell) ? M.Z[k * ell + p] : 0.0;
      }
    }
  };
  auto multiply = [&](const double (&qa)[kB][kMT], const double (&yb)[kB]) {
#pragma unroll
    for (int u = 0; u < kB; ++u)
#pragma unroll
      for (int pt = 0; pt < kMT; ++pt)
        if (pt < nt) acc[pt] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[u][pt], yb[u], acc[pt], 0, 0, 0);
  };
  // two batches of loads: the next one in flight while the current one is
  // multiplied (a batch past m loads zeros)
  double qa0[kB][kMT], yb0[kB], qa1[kB][kMT], yb1[kB];
  fetch(0, qa0, yb0);
  for (int64_t k0 = 0; k0 < M.m; k0 += 8 * kB) {
    fetch(k0 + 4 * kB, qa1, yb1);
    multiply(qa0, yb0);
    if (k0 + 4 * kB >= M.m) break;
    fetch(k0 + 8 * kB, qa0, yb0);
    multiply(qa1, yb1);
  }
  // register v of an accumulator: row 16 pt + l/16 + 4 v, column 16 w + l%16
#pragma unroll
  for (int pt = 0; pt < kMT; ++pt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int p = 16 * pt + g + 4 * v;
      if (pt < nt && p < ell) sM[p][16 * wave + l16] = acc[pt][v];
    }
  __syncthreads();
  double* C = M.cpart + (int64_t)cc * ell * ell;
  const int ntiles = nt * (nt + 1) / 2;
  for (int tile = wave; tile < ntiles; tile += 4) {
    int pi = 0, rem = tile;
    while (rem >= nt - pi) { rem -= nt - pi; ++pi; }
    const int pj = pi + rem;
    doublex4 c = {0.0, 0.0, 0.0, 0.0};
    const int ri = 16 * pi + l16, rj = 16 * pj + l16;
#pragma unroll
    for (int k0 = 0; k0 < kQRColChunk; k0 += 4) {
      const double a = ri < ell ? sM[ri][k0 + g] : 0.0;
      const double bb = rj < ell ? sM[rj][k0 + g] : 0.0;
      c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, c, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int p = 16 * pi + g + 4 * v, q = 16 * pj + l16;
      if (p < ell && q < ell) {
        C[p * ell + q] = c[v];
        if (pi != pj) C[q * ell + p] = c[v];
      }
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

// W step: W = eigenvectors of the r largest eigenvalues (descending) of the
// summed ell x ell Gram of M = Q^T Y, by cyclic Jacobi (parallel round-robin
// ordering), then U = Q W with the column sign rule.  One 256-thread
// workgroup per matrix.
//  * A round computes its ell/2 disjoint rotations in every wave (lane k:
//    rotation k, so no wave waits for another's parameters) and applies them
//    to 2x2 blocks of A (A <- J^T A J) and to column pairs of V (V <- V J),
//    each thread owning a fixed set of blocks and pairs.  A is double
//    buffered: a round reads one copy and writes every block of the other, so
//    one barrier per round suffices.
//  * The rotation of a pair comes from the hardware estimates of 1/sqrt and
//    1/x with two Newton steps each (within 2 u), not from the division and
//    square-root sequences, whose range scaling would sit on the chain.  A is
//    scaled by a power of two first (exact), so that its largest entry lies
//    in [1, 2).
//  * A rotation is skipped once |a_pq| <= tol max(|a_pp|, |a_qq|) (tol = 4 u
//    for FP64 bases, 1e-12 for FP32 bases): the rotation it would apply is
//    then below rounding level relative to the pair's own scale (a
//    signal/noise pair is decoupled to ~u), whereas the stricter test
//    |a_pq| <= u sqrt(a_pp a_qq) can be unreachable in floating point for
//    strongly graded pairs.
//  * Pairs of two indices that currently rank below the r largest diagonal
//    entries are not rotated: such a rotation only mixes directions that are
//    dropped.  Once no other pair rotates, a Gershgorin bound checks that the
//    unreduced block of those indices lies below every kept diagonal entry
//    (so the kept ones are the r largest eigenvalues); if it does not, full
//    sweeps resume.  Sweeps exhausted with rotations still firing set info
//    bit 3 (W may be inaccurate).
//  * U = Q W on v_mfma_f64_16x16x4f64, twice: the first pass finds each
//    column's entry of largest magnitude (lowest row on ties), the second
//    stores U with that entry made positive.
constexpr int kEigThreads = 256;
constexpr int kEigMaxSweeps = 60;

// IA, IV: A-block and V-pair items per thread, sized by the launcher for the
// widest sketch of the batch so the per-round loads are straight-line code
// The end of the W step for one matrix: the eigenvalues on the diagonal of
// A, the eigenvectors in the columns of V (both in LDS); W (an E x (E + 1)
// LDS array free for use) receives W.  Ranks the eigenvalues, then writes W
// to global memory (large matrices) or U = Q W with the sign rule (small
// ones).  Called by every thread of the 256-thread workgroup.
template <int E>
__device__ __forceinline__ void wstep_finish(const QRMat& M, double (*A)[E + 1], double (*V)[E + 1],
                                             double (*W)[E + 1], int tid) {
  const int n = M.ell, wave = tid >> 6, lane = tid & 63;
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
  const int r = M.r;
  const int kp = (n + 3) & ~3, rp = (r + 15) & ~15;   // K padded to 4, columns to 16
  for (int e = tid; e < kp * rp; e += kEigThreads) {
    const int k = e / rp, j = e - k * rp;
    W[k][j] = 0.0;
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += kEigThreads) {
    const int k = e / n, i = e - k * n;
    if (rank_of[i] < r) W[k][rank_of[i]] = V[k][i];
  }
  __syncthreads();
  // U = Q W: wave w takes row tiles w, w + 4, ...; lane l supplies
  // Q[row0 + l%16][k0 + l/16] and W[k0 + l/16][16 ct + l%16]; register v of
  // an accumulator holds row row0 + l/16 + 4 v, column 16 ct + l%16
  constexpr int kCT = E / 16;
  const int nct = rp / 16, nks = kp / 4, l16 = lane & 15, g = lane >> 4;
  const int64_t nrt = (M.m + 15) / 16;
  auto tile = [&](int64_t rt, doublex4 (&acc)[kCT]) {
#pragma unroll
    for (int ct = 0; ct < kCT; ++ct) acc[ct] = doublex4{0.0, 0.0, 0.0, 0.0};
    const int64_t row = rt * 16 + l16;
    for (int ks = 0; ks < nks; ++ks) {
      const int k = 4 * ks + g;
      const double a = (row < M.m && k < n) ? M.Z[row * n + k] : 0.0;
#pragma unroll
      for (int ct = 0; ct < kCT; ++ct)
        if (ct < nct) acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, W[k][16 * ct + l16], acc[ct], 0, 0, 0);
    }
  };
  // pass 1: per column, the entry of largest magnitude (lowest row on ties)
  double best[kCT], bval[kCT];
  int64_t bidx[kCT];
#pragma unroll
  for (int ct = 0; ct < kCT; ++ct) {
    best[ct] = -1.0;
    bval[ct] = 0.0;
    bidx[ct] = INT64_MAX;
  }
  for (int64_t rt = wave; rt < nrt; rt += kEigThreads / 64) {
    doublex4 acc[kCT];
    tile(rt, acc);
#pragma unroll
    for (int ct = 0; ct < kCT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = rt * 16 + g + 4 * v;   // ascending within a lane
        const double u = acc[ct][v];
        if (row < M.m && fabs(u) > best[ct]) {
          best[ct] = fabs(u);
          bval[ct] = u;
          bidx[ct] = row;
        }
      }
  }
  __shared__ double cand_a[kEigThreads / 16][E], cand_v[kEigThreads / 16][E];
  __shared__ int64_t cand_i[kEigThreads / 16][E];
  __shared__ double sgn[E];
#pragma unroll
  for (int ct = 0; ct < kCT; ++ct)
    if (ct < nct) {
      cand_a[tid >> 4][16 * ct + l16] = best[ct];
      cand_v[tid >> 4][16 * ct + l16] = bval[ct];
      cand_i[tid >> 4][16 * ct + l16] = bidx[ct];
    }
  __syncthreads();
  if (tid < r) {
    double ba = -1.0, bv = 0.0;
    int64_t bi = INT64_MAX;
    for (int s2 = 0; s2 < kEigThreads / 16; ++s2) {
      const double ca = cand_a[s2][tid];
      const int64_t ci = cand_i[s2][tid];
      if (ca > ba || (ca == ba && ci < bi)) {
        ba = ca;
        bv = cand_v[s2][tid];
        bi = ci;
      }
    }
    sgn[tid] = bv < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  // pass 2: U with the sign rule applied
  const bool f64 = M.udtype == TK_F64;
  for (int64_t rt = wave; rt < nrt; rt += kEigThreads / 64) {
    doublex4 acc[kCT];
    tile(rt, acc);
#pragma unroll
    for (int ct = 0; ct < kCT; ++ct) {
      const int j = 16 * ct + l16;
      if (ct < nct && j < r) {
        const double sj = sgn[j];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = rt * 16 + g + 4 * v;
          if (row < M.m) {
            if (f64) static_cast<double*>(M.U)[row * r + j] = sj * acc[ct][v];
            else static_cast<float*>(M.U)[row * r + j] = (float)(sj * acc[ct][v]);
          }
        }
      }
    }
  }
}

template <typename S, int IA, int IV, int E>
__global__ __launch_bounds__(kEigThreads) void eig_kernel(const S b) {
  const QRMat& M = b.get(blockIdx.x);
  __shared__ double Abuf[2][E][E + 1];
  __shared__ double V[E][E + 1];
  // (c, s) of the current round's rotations, one copy per wave
  __shared__ double2 rot_cs[kEigThreads / 64][E / 2];
  __shared__ double red[kEigThreads / 64];
  const int n = M.ell, np = n + (n & 1), half = np / 2, tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const double tol = M.udtype == TK_F64 ? 4.0 * kUnit : 1e-12;
  // summed Gram: every thread's elements over groups of four column chunks,
  // all loads of a group in flight together (each element still sums the
  // chunks in index order); then scaled by a power of two
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
    double amax = 0.0;
#pragma unroll
    for (int k = 0; k < kE; ++k) amax = fmax(amax, fabs(v[k]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off));
    if (lane == 0) red[wave] = amax;
    __syncthreads();
    amax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const double sc = amax > 0.0 ? ldexp(1.0, -ilogb(amax)) : 1.0;
#pragma unroll
    for (int k = 0; k < kE; ++k) {
      const int e = tid + kEigThreads * k;
      if (e < np * np) {
        const int p = e / np, q = e - p * np;
        Abuf[0][p][q] = v[k] * sc;
        V[p][q] = p == q ? 1.0 : 0.0;
      }
    }
  }
  // this thread's items, in two loops of one kind each so a wave never runs
  // both kinds: the half x half 2x2 blocks of A (pair k1 rows, pair k2
  // columns: A <- J^T A J on the block) and the np x half column pairs of V
  // (V <- V J); codes k1 * 64 + k2 and k * 64 + i, or -1 past the end
  int itemA[IA], itemV[IV];
  const int nblk = half * half, nv = np * half;
#pragma unroll
  for (int t = 0; t < IA; ++t) {
    const int e = tid + kEigThreads * t;
    itemA[t] = e < nblk ? (e / half) * 64 + (e % half) : -1;   // -1: none (loads a dummy)
  }
#pragma unroll
  for (int t = 0; t < IV; ++t) {
    const int e = tid + kEigThreads * t;
    itemV[t] = e < nv ? (e / np) * 64 + (e % np) : -1;
  }
  __syncthreads();
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
  int cur = 0;   // the copy of A that holds the current matrix
  bool skip_dropped = M.r < n;
  bool converged = false;
  for (int sweep = 0; sweep < kEigMaxSweeps; ++sweep) {
    double (*A)[E + 1] = Abuf[cur];
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
      double (*Ac)[E + 1] = Abuf[cur];
      double (*An)[E + 1] = Abuf[cur ^ 1];
      bool rot_now = false;
      if (lane < half) {
        int p, q;
        pair_of(lane, round, p, q);
        // t = tan of the rotation angle, the root of t^2 + 2 theta t - 1 of
        // smaller magnitude, theta = (a_qq - a_pp) / (2 a_pq):
        // t = 2 a_pq / (d + sign(d) sqrt(d^2 + 4 a_pq^2)), d = a_qq - a_pp;
        // c = 1 / sqrt(1 + t^2).  A pair whose d^2 + 4 a_pq^2 is below the
        // normal range (entries below 1e-154 of the largest) counts as
        // decoupled.  Computed for every pair (selects, no branch: the pad
        // index np - 1 exists in A), then kept or replaced by the identity.
        const double apq = Ac[p][q], app = Ac[p][p], aqq = Ac[q][q];
        const double d = aqq - app;
        const double x = fma(d, d, 4.0 * apq * apq);
        rot_now = q < n && !(((dropped >> p) & 1) && ((dropped >> q) & 1)) &&
                  fabs(apq) > tol * fmax(fabs(app), fabs(aqq)) && x >= 2.2250738585072014e-308;
        const double xs = rot_now ? x : 1.0;
        const double root = xs * rsq_nr(xs);
        const double t = 2.0 * apq * rcp_nr(d >= 0.0 ? d + root : d - root);
        const double c = rsq_nr(fma(t, t, 1.0));
        rot_cs[wave][lane] = rot_now ? make_double2(c, t * c) : make_double2(1.0, 0.0);
      }
      // identical in every wave, so every wave takes the same branch
      const bool round_rot = __any(rot_now);
      if (!round_rot) continue;
      rotated = true;
      __builtin_amdgcn_wave_barrier();
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      // every load of this thread's items first (straight-line: an absent
      // item loads the entries of block (0, 0)), then the updates; every
      // block of the other copy is written
      double blk[IA][4], vv[IV][2];
      double2 r1[IA], r2[IA], rv[IV];
      int ia[IA][4], iv[IV][3];
#pragma unroll
      for (int t = 0; t < IA; ++t) {
        const int code = itemA[t] < 0 ? 0 : itemA[t];
        const int k1 = code >> 6, k2 = code & 63;
        pair_of(k1, round, ia[t][0], ia[t][1]);
        pair_of(k2, round, ia[t][2], ia[t][3]);
        r1[t] = rot_cs[wave][k1];
        r2[t] = rot_cs[wave][k2];
        blk[t][0] = Ac[ia[t][0]][ia[t][2]];
        blk[t][1] = Ac[ia[t][0]][ia[t][3]];
        blk[t][2] = Ac[ia[t][1]][ia[t][2]];
        blk[t][3] = Ac[ia[t][1]][ia[t][3]];
      }
#pragma unroll
      for (int t = 0; t < IV; ++t) {
        const int code = itemV[t] < 0 ? 0 : itemV[t];
        const int k = code >> 6;
        iv[t][0] = code & 63;
        pair_of(k, round, iv[t][1], iv[t][2]);
        rv[t] = rot_cs[wave][k];
        vv[t][0] = V[iv[t][0]][iv[t][1]];
        vv[t][1] = V[iv[t][0]][iv[t][2]];
      }
#pragma unroll
      for (int t = 0; t < IA; ++t) {
        if (itemA[t] >= 0) {
          const double c1 = r1[t].x, s1 = r1[t].y, c2 = r2[t].x, s2 = r2[t].y;
          const double a = blk[t][0], bb = blk[t][1], cc = blk[t][2], dd = blk[t][3];
          // rows (J^T from the left), then columns (J from the right)
          const double ra = c1 * a - s1 * cc, rb = c1 * bb - s1 * dd;
          const double rc = s1 * a + c1 * cc, rd = s1 * bb + c1 * dd;
          An[ia[t][0]][ia[t][2]] = c2 * ra - s2 * rb;
          An[ia[t][0]][ia[t][3]] = s2 * ra + c2 * rb;
          An[ia[t][1]][ia[t][2]] = c2 * rc - s2 * rd;
          An[ia[t][1]][ia[t][3]] = s2 * rc + c2 * rd;
        }
      }
#pragma unroll
      for (int t = 0; t < IV; ++t) {
        if (itemV[t] >= 0 && rv[t].y != 0.0) {
          const double cv = rv[t].x, sv = rv[t].y;
          const double vip = vv[t][0], viq = vv[t][1];
          V[iv[t][0]][iv[t][1]] = cv * vip - sv * viq;
          V[iv[t][0]][iv[t][2]] = sv * vip + cv * viq;
        }
      }
      __syncthreads();
      cur ^= 1;
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
  double (*A)[E + 1] = Abuf[cur];
  double (*W)[E + 1] = Abuf[cur ^ 1];   // W[k][rank], zero padded
  wstep_finish<E>(M, A, V, W, tid);
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
      if (host[i].small)
        lds = std::max<int64_t>(lds, ((host[i].m + 4) * host[i].ell + 64) * (int64_t)sizeof(double));
    int ellmax = 1;
    for (int i = 0; i < count; ++i)
      if (host[i].small) ellmax = std::max(ellmax, host[i].ell);
    if (ellmax <= 32)
      hipLaunchKernelGGL((cholqr_small_kernel<S, 32>), dim3(count), dim3(256), (size_t)lds, st, src);
    else if (ellmax <= 48)
      hipLaunchKernelGGL((cholqr_small_kernel<S, 48>), dim3(count), dim3(256), (size_t)lds, st, src);
    else
      hipLaunchKernelGGL((cholqr_small_kernel<S, 64>), dim3(count), dim3(256), (size_t)lds, st, src);
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
  bool all_small = true;
  for (int i = 0; i < count; ++i) all_small &= host[i].small != 0;
  if (!gram_given && all_small) {
    const dim3 gg((unsigned)ncc, (unsigned)count);
    switch (ydtype) {
      case TK_F64: hipLaunchKernelGGL((qty_gram_kernel<double, S>), gg, dim3(256), 0, st, src); break;
      case TK_F32: hipLaunchKernelGGL((qty_gram_kernel<float, S>), gg, dim3(256), 0, st, src); break;
      case TK_BF16: hipLaunchKernelGGL((qty_gram_kernel<bf16, S>), gg, dim3(256), 0, st, src); break;
      case TK_F16: hipLaunchKernelGGL((qty_gram_kernel<f16, S>), gg, dim3(256), 0, st, src); break;
      default: return hipErrorInvalidValue;
    }
  } else if (!gram_given) {
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
  // LDS sized for the widest sketch of the batch (E = 32 or 64): narrow
  // sketches then fit several workgroups per CU, which a batch of many
  // matrices needs
  // items per thread for the widest sketch: half^2 A blocks and np * half V
  // pairs; LDS sized for the widest sketch too (E = 32 or 64): narrow
  // sketches then fit several workgroups per CU, which a batch of many
  // matrices needs
  int ellmax = 1;
  for (int i = 0; i < count; ++i) ellmax = std::max(ellmax, host[i].ell);
  const int np = ellmax + (ellmax & 1), half = np / 2;
  const int ia = (int)ceil_div((int64_t)half * half, kEigThreads);
  const int iv = (int)ceil_div((int64_t)np * half, kEigThreads);
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
