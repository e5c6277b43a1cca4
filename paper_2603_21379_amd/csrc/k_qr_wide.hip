// Thin QR and W step of Algorithm 1 for sketch widths 64 < ell <= 192, where
// the ell x ell matrices no longer fit the one-wave LDS kernels of the narrow
// path (a rank of 150 with oversampling 10 gives ell = 160).
//
// Same mathematics and the same rules as the narrow path: CholeskyQR2 with an
// FP64 Gram and a shifted pass when the Gram is not safely positive definite,
// then W = dominant r eigenvectors of the FP64 Gram of M = Q^T Y, U = Q W with
// the largest-magnitude entry of every column made positive.  The layout
// differs:
//  * products (Z^T Z, Y^T Q, M M^T) run as one tiled FP64 kernel over row
//    chunks, partials per chunk summed in chunk order by the consumer;
//  * the Cholesky factor and the Jacobi matrix live in LDS as a packed upper
//    triangle (ell (ell+1)/2 doubles, 148 KB at ell = 192), one workgroup;
//  * a Jacobi sweep records its rotations; the eigenvector matrix V is
//    rotated row by row by a separate many-workgroup kernel, so the sweep's
//    workgroup touches nothing but LDS.
// Every reduction has a fixed order, so results are bitwise repeatable.
#include "tk_kernels.hpp"

namespace tk {
namespace {

constexpr double kUnit = 1.1102230246251565e-16;  // 2^-53
constexpr int kTile = 32;

__device__ __forceinline__ int64_t pk(int p, int q, int n) {
  // packed upper triangle, row by row: (p, q) with p <= q
  return (int64_t)p * n - ((int64_t)p * (p - 1)) / 2 + (q - p);
}
__device__ __forceinline__ int64_t pks(int x, int y, int n) { return x <= y ? pk(x, y, n) : pk(y, x, n); }

// round-robin pairing of np (even) indices: round t in [0, np - 1), pair k in
// [0, np / 2); index np - 1 stays fixed, the others turn (circle method)
__device__ __forceinline__ void pair_of(int t, int k, int np, int& p, int& q) {
  const int m = np - 1;
  if (k == 0) {
    p = t;
    q = m;
  } else {
    p = (t + k) % m;
    q = (t - k + m) % m;
  }
  if (p > q) { const int x = p; p = q; q = x; }
}

// out[z][p][q] = sum over rows i of chunk z of A[i][p] * B[i][q]
template <typename TA>
__global__ __launch_bounds__(256) void tn_partial_kernel(const TA* __restrict__ A, int64_t lda,
                                                         const double* __restrict__ B, int64_t ldb,
                                                         int64_t rows, int P, int Q, int64_t chunk,
                                                         double* __restrict__ out) {
  __shared__ double sA[kTile][kTile + 1];
  __shared__ double sB[kTile][kTile + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int p0 = blockIdx.x * kTile, q0 = blockIdx.y * kTile;
  const int64_t i0 = (int64_t)blockIdx.z * chunk;
  const int64_t i1 = min(rows, i0 + chunk);
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int64_t ib = i0; ib < i1; ib += kTile) {
    for (int e = tid; e < kTile * kTile; e += 256) {
      const int ii = e / kTile, c = e - ii * kTile;
      const int64_t gi = ib + ii;
      const bool in = gi < i1;
      sA[ii][c] = (in && p0 + c < P) ? to_double(A[gi * lda + p0 + c]) : 0.0;
      sB[ii][c] = (in && q0 + c < Q) ? B[gi * ldb + q0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int ii = 0; ii < kTile; ++ii) {
      const double a0 = sA[ii][ty], a1 = sA[ii][ty + 16];
      const double b0 = sB[ii][tx], b1 = sB[ii][tx + 16];
      acc[0][0] = fma(a0, b0, acc[0][0]);
      acc[0][1] = fma(a0, b1, acc[0][1]);
      acc[1][0] = fma(a1, b0, acc[1][0]);
      acc[1][1] = fma(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
  double* o = out + (int64_t)blockIdx.z * P * Q;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int p = p0 + ty + 16 * a, q = q0 + tx + 16 * b;
      if (p < P && q < Q) o[(int64_t)p * Q + q] = acc[a][b];
    }
}

// Upper Cholesky factor of the packed matrix in LDS, in place; every thread
// of the workgroup calls it.  False when a pivot is not above tol (or NaN).
__device__ bool cholesky_packed(double* G, int n, double tol) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int j = 0; j < n; ++j) {
    __syncthreads();
    const double piv = G[pk(j, j, n)];
    if (!(piv > tol)) return false;  // uniform: every thread read the same value
    const double rjj = sqrt(piv);
    for (int i = j + 1 + tid; i < n; i += nt) G[pk(j, i, n)] /= rjj;
    __syncthreads();
    if (tid == 0) G[pk(j, j, n)] = rjj;
    // trailing update of the upper triangle, one row segment per item
    const int m = n - j - 1;
    for (int e = tid; e < m * m; e += nt) {
      const int p = j + 1 + e / m, q = j + 1 + e % m;
      if (q >= p) G[pk(p, q, n)] -= G[pk(j, p, n)] * G[pk(j, q, n)];
    }
  }
  __syncthreads();
  return true;
}

// state[0]: CholeskyQR passes still owed (a plain pass pays one, a shifted
// pass leaves two owed); state[1]: whether this pass applies R^{-1}.
__global__ __launch_bounds__(1024) void wide_chol_kernel(const WideQR w, int pass) {
  extern __shared__ double G[];
  __shared__ double stat[2];
  const int n = w.ell, tid = threadIdx.x;
  if (pass > 1 && w.state[0] == 0) {
    if (tid == 0) w.state[1] = 0;
    return;
  }
  const int64_t nn = (int64_t)n * n;
  auto load = [&](double shift) {
    __syncthreads();
    for (int64_t e = tid; e < nn; e += blockDim.x) {
      const int p = (int)(e / n), q = (int)(e - (int64_t)p * n);
      if (q < p) continue;
      double v = 0.0;
      for (int z = 0; z < w.gsplit; ++z) v += w.gpart[(int64_t)z * nn + e];
      G[pk(p, q, n)] = v + (p == q ? shift : 0.0);
    }
    __syncthreads();
  };
  load(0.0);
  if (tid == 0) {
    double mx = 0.0, tr = 0.0;
    for (int j = 0; j < n; ++j) {
      const double g = G[pk(j, j, n)];
      mx = fmax(mx, g);
      tr += g;
    }
    stat[0] = mx;
    stat[1] = tr;
  }
  __syncthreads();
  const double mx = stat[0], tr = stat[1];
  // a pivot below this means cond(Z) beyond what two CholeskyQR passes repair
  const double tol = 1e-14 * mx;
  int status = 0;
  bool ok = mx > 0.0 && cholesky_packed(G, n, tol);
  if (!ok) {
    // shifted CholeskyQR (Fukaya et al. 2020): s = 11 (m n + n (n+1)) u ||Z||^2,
    // with ||Z||_2^2 bounded by the trace of the Gram
    const double shift = 11.0 * ((double)w.m * n + (double)n * (n + 1)) * kUnit * fmax(tr, 1e-300);
    load(shift);
    status = 1;
    ok = cholesky_packed(G, n, 0.0);
    if (!ok) status = 2;
  }
  __syncthreads();
  for (int64_t e = tid; e < nn; e += blockDim.x) {
    const int p = (int)(e / n), q = (int)(e - (int64_t)p * n);
    double v = q >= p ? G[pk(p, q, n)] : 0.0;
    if (!ok && p == q && !(v > 0.0)) v = 1.0;  // keep the solve finite; flagged in info
    w.R[e] = v;
  }
  if (tid == 0) {
    const int owed = pass == 1 ? 2 : w.state[0];
    w.state[0] = status != 0 ? 2 : owed - 1;
    w.state[1] = 1;
    if (w.info) {
      // bit 0: first pass shifted; bit 1: a later pass shifted; bit 2: Cholesky
      // failed even with the shift
      int v = pass == 1 ? 0 : *w.info;
      if (status != 0) v |= pass == 1 ? 1 : 2;
      if (status == 2) v |= 4;
      *w.info = v;
    }
  }
}

// Q = Z R^{-1} for 64 rows per workgroup (one row per lane), forward
// substitution on q R = z in place; R staged in LDS sixteen columns at a time
// (transposed, so a column is contiguous and every lane reads the same word).
constexpr int kApplyCols = 16;
__global__ __launch_bounds__(64) void wide_apply_kernel(const WideQR w) {
  if (w.state[1] == 0) return;
  extern __shared__ double lds[];
  const int n = w.ell, lane = threadIdx.x;
  double* sZ = lds;                          // [n][65]
  double* Rt = lds + (int64_t)n * 65;        // [kApplyCols][n]
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int rows = (int)min<int64_t>(64, w.m - r0);
  for (int e = lane; e < rows * n; e += 64) {
    const int rr = e / n, j = e - rr * n;
    sZ[j * 65 + rr] = w.Z[(r0 + rr) * n + j];
  }
  for (int j0 = 0; j0 < n; j0 += kApplyCols) {
    const int jc = min(kApplyCols, n - j0);
    __syncthreads();
    for (int e = lane; e < jc * n; e += 64) {
      const int jj = e / n, k = e - jj * n;
      Rt[jj * n + k] = w.R[(int64_t)k * n + j0 + jj];
    }
    __syncthreads();
    if (lane < rows) {
      for (int jj = 0; jj < jc; ++jj) {
        const int j = j0 + jj;
        const double* rc = Rt + jj * n;
        // four partial sums (k mod 4), combined in a fixed order: the loads
        // of a step do not wait on the previous step's sum
        double v0 = sZ[j * 65 + lane], v1 = 0.0, v2 = 0.0, v3 = 0.0;
        int k = 0;
        for (; k + 4 <= j; k += 4) {
          v0 = fma(-sZ[k * 65 + lane], rc[k], v0);
          v1 = fma(-sZ[(k + 1) * 65 + lane], rc[k + 1], v1);
          v2 = fma(-sZ[(k + 2) * 65 + lane], rc[k + 2], v2);
          v3 = fma(-sZ[(k + 3) * 65 + lane], rc[k + 3], v3);
        }
        for (; k < j; ++k) v0 = fma(-sZ[k * 65 + lane], rc[k], v0);
        sZ[j * 65 + lane] = ((v0 + v1) + (v2 + v3)) / rc[j];
      }
    }
  }
  __syncthreads();
  for (int e = lane; e < rows * n; e += 64) {
    const int rr = e / n, j = e - rr * n;
    w.Z[(r0 + rr) * n + j] = sZ[j * 65 + rr];
  }
}

// One cyclic Jacobi sweep (np - 1 rounds of np / 2 disjoint rotations) on the
// packed matrix.  Sweep 0 forms the matrix from the Gram partials (zero row
// and column for the padding index of an odd ell).  Rotation (c, s) of pair
// (p, q), p < q, is J with J_pp = J_qq = c, J_pq = s, J_qp = -s; A <- J^T A J
// zeroes a_pq.  It is skipped once |a_pq| <= tol max(|a_pp|, |a_qq|) (the
// rotation is then below rounding level relative to the pair's own scale).
// Every thread owns a fixed set of (pair a, pair b), a <= b, items, the same
// in every round; a round's pairs and rotations sit in LDS.
// state[2]: converged; state[3 + k]: rotations of sweep k.
constexpr int kSweepThreads = 1024;
constexpr int kSweepItems = (kWideMaxEll / 2 * (kWideMaxEll / 2 + 1) / 2 + kSweepThreads - 1) / kSweepThreads;
__global__ __launch_bounds__(kSweepThreads) void wide_sweep_kernel(const WideQR w, int sweep, double tol) {
  extern __shared__ double A[];
  __shared__ double rc[kWideMaxEll / 2], rs[kWideMaxEll / 2], rt[kWideMaxEll / 2];
  __shared__ int ract[kWideMaxEll / 2], sp[kWideMaxEll / 2], sq[kWideMaxEll / 2];
  __shared__ int op[kWideMaxEll / 2], oq[kWideMaxEll / 2];   // rowoff of the pair's p and q
  __shared__ int rowoff[kWideMaxEll];   // pk(x, y) = rowoff[x] + y for x <= y
  __shared__ int count;
  const int n = w.ell, np = w.np, half = np / 2, tid = threadIdx.x;
  if (sweep > 0 && w.state[2]) return;
  for (int x = tid; x < np; x += kSweepThreads) rowoff[x] = (int)pk(x, 0, np);
  if (sweep == 0) {
    if (tid == 0) w.state[2] = 0;
    for (int k = tid; k < kWideMaxSweeps; k += kSweepThreads) w.state[3 + k] = 0;
    const int64_t nn = (int64_t)n * n;
    for (int64_t e = tid; e < (int64_t)np * np; e += kSweepThreads) {
      const int p = (int)(e / np), q = (int)(e - (int64_t)p * np);
      if (q < p) continue;
      double v = 0.0;
      if (q < n)
        for (int z = 0; z < w.csplit; ++z) v += w.cpart[(int64_t)z * nn + (int64_t)p * n + q];
      A[pk(p, q, np)] = v;
    }
  } else {
    const int64_t tot = (int64_t)np * (np + 1) / 2;
    for (int64_t e = tid; e < tot; e += kSweepThreads) A[e] = w.Ap[e];
  }
  // this thread's items: (a, b) with a <= b, triangular index tid + 1024 j
  int item[kSweepItems];
  const int T = half * (half + 1) / 2;
#pragma unroll
  for (int j = 0; j < kSweepItems; ++j) {
    int e = tid + kSweepThreads * j, a = 0;
    item[j] = -1;
    if (e < T) {
      while (e >= half - a) { e -= half - a; ++a; }
      item[j] = a | ((a + e) << 8);
    }
  }
  if (tid == 0) count = 0;
  __syncthreads();
  for (int t = 0; t < np - 1; ++t) {
    if (tid < half) {
      int p, q;
      pair_of(t, tid, np, p, q);
      const double app = A[rowoff[p] + p], aqq = A[rowoff[q] + q], apq = A[rowoff[p] + q];
      double c = 1.0, s = 0.0, tn = 0.0;
      const bool act = fabs(apq) > tol * fmax(fabs(app), fabs(aqq));
      if (act) {
        const double theta = (aqq - app) / (2.0 * apq);
        tn = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(fma(theta, theta, 1.0)));
        c = 1.0 / sqrt(fma(tn, tn, 1.0));
        s = tn * c;
        atomicAdd(&count, 1);
      }
      rc[tid] = c;
      rs[tid] = s;
      rt[tid] = tn;
      ract[tid] = act;
      sp[tid] = p;
      sq[tid] = q;
      op[tid] = rowoff[p];
      oq[tid] = rowoff[q];
      double* ro = w.rot + 2 * ((int64_t)t * half + tid);
      ro[0] = c;
      ro[1] = s;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSweepItems; ++j) {
      if (item[j] < 0) continue;
      const int a = item[j] & 255, b = item[j] >> 8;
      if (!ract[a] && !ract[b]) continue;
      // every address from the pair tables directly (no second LDS lookup)
      const int pa = sp[a], qa = sq[a], opa = op[a], oqa = oq[a];
      if (a == b) {
        const int ipq = opa + qa;
        const double apq = A[ipq];
        A[opa + pa] -= rt[a] * apq;
        A[oqa + qa] += rt[a] * apq;
        A[ipq] = 0.0;
        continue;
      }
      const int pb = sp[b], qb = sq[b], opb = op[b], oqb = oq[b];
      double& r00 = A[pa <= pb ? opa + pb : opb + pa];
      double& r01 = A[pa <= qb ? opa + qb : oqb + pa];
      double& r10 = A[qa <= pb ? oqa + pb : opb + qa];
      double& r11 = A[qa <= qb ? oqa + qb : oqb + qa];
      const double x00 = r00, x01 = r01, x10 = r10, x11 = r11;
      const double ca = rc[a], sa = rs[a], cb = rc[b], sb = rs[b];
      // right factor J_b on the columns, then J_a^T on the rows
      const double y00 = cb * x00 - sb * x01, y01 = sb * x00 + cb * x01;
      const double y10 = cb * x10 - sb * x11, y11 = sb * x10 + cb * x11;
      r00 = ca * y00 - sa * y10;
      r10 = sa * y00 + ca * y10;
      r01 = ca * y01 - sa * y11;
      r11 = sa * y01 + ca * y11;
    }
    __syncthreads();
  }
  const int64_t tot = (int64_t)np * (np + 1) / 2;
  for (int64_t e = tid; e < tot; e += kSweepThreads) w.Ap[e] = A[e];
  if (tid == 0) {
    w.state[3 + sweep] = count;
    if (count == 0) w.state[2] = 1;
  }
}

// V <- V J for every rotation of a sweep, one row of V per workgroup (the
// rotations of a round touch disjoint pairs of a row).  Sweep 0 starts from
// the identity.  The next round's (c, s) loads are issued before the current
// round's rotations.
constexpr int kVrotPairs = (kWideMaxEll / 2 + 63) / 64;
__global__ __launch_bounds__(64) void wide_vrot_kernel(const WideQR w, int sweep) {
  __shared__ double row[kWideMaxEll];
  const int np = w.np, half = np / 2, lane = threadIdx.x, i = blockIdx.x;
  const bool rotate = w.state[3 + sweep] > 0;
  if (sweep > 0 && !rotate) return;
  double* vr = w.V + (int64_t)i * np;
  for (int j = lane; j < np; j += 64) row[j] = sweep == 0 ? (j == i ? 1.0 : 0.0) : vr[j];
  if (rotate) {
    double2 cur[kVrotPairs], nxt[kVrotPairs];
    auto fetch = [&](int t, double2 (&d)[kVrotPairs]) {
#pragma unroll
      for (int u = 0; u < kVrotPairs; ++u) {
        const int k = lane + 64 * u;
        d[u] = (t < np - 1 && k < half)
                   ? *reinterpret_cast<const double2*>(w.rot + 2 * ((int64_t)t * half + k))
                   : make_double2(1.0, 0.0);
      }
    };
    fetch(0, cur);
    for (int t = 0; t < np - 1; ++t) {
      fetch(t + 1, nxt);
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kVrotPairs; ++u) {
        const int k = lane + 64 * u;
        if (k < half) {
          int p, q;
          pair_of(t, k, np, p, q);
          const double vp = row[p], vq = row[q];
          row[p] = cur[u].x * vp - cur[u].y * vq;
          row[q] = cur[u].y * vp + cur[u].x * vq;
        }
      }
#pragma unroll
      for (int u = 0; u < kVrotPairs; ++u) cur[u] = nxt[u];
    }
  }
  __syncthreads();
  for (int j = lane; j < np; j += 64) vr[j] = row[j];
}

// W = eigenvectors of the r largest eigenvalues, descending (ties: lower index first)
__global__ __launch_bounds__(256) void wide_select_kernel(const WideQR w) {
  const int n = w.ell, np = w.np;
  // no sweep ended without a rotation: W may be inaccurate (info bit 3)
  if (threadIdx.x == 0 && !w.state[2] && w.info) *w.info |= 8;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double li = w.Ap[pk(i, i, np)];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = w.Ap[pk(j, j, np)];
      rank += (lj > li) || (lj == li && j < i);
    }
    if (rank < w.r)
      for (int k = 0; k < n; ++k) w.W[(int64_t)k * w.r + rank] = w.V[(int64_t)k * np + i];
  }
}

// Column j of U = Q W per workgroup, then the sign rule: the entry of largest
// magnitude (lowest row on ties) made positive; each thread flips only the
// entries it wrote.
template <typename TU>
__global__ __launch_bounds__(256) void wide_u_kernel(const WideQR w) {
  __shared__ double sw[kWideMaxEll];
  __shared__ double cv[256], ca[256];
  __shared__ int64_t ci[256];
  const int n = w.ell, r = w.r, j = blockIdx.x, tid = threadIdx.x;
  for (int k = tid; k < n; k += 256) sw[k] = w.W[(int64_t)k * r + j];
  __syncthreads();
  TU* U = static_cast<TU*>(w.U);
  double best = -1.0, bval = 0.0;
  int64_t bidx = INT64_MAX;
  for (int64_t i = tid; i < w.m; i += 256) {
    const double* q = w.Z + i * n;
    double u = 0.0;
    for (int k = 0; k < n; ++k) u = fma(q[k], sw[k], u);
    if (fabs(u) > best) { best = fabs(u); bval = u; bidx = i; }  // rows ascend
    U[i * r + j] = from_double<TU>(u);
  }
  ca[tid] = best;
  cv[tid] = bval;
  ci[tid] = bidx;
  __syncthreads();
  if (tid == 0) {
    double ba = -1.0, bv = 0.0;
    int64_t bi = INT64_MAX;
    for (int t = 0; t < 256; ++t)
      if (ca[t] > ba || (ca[t] == ba && ci[t] < bi)) { ba = ca[t]; bv = cv[t]; bi = ci[t]; }
    cv[0] = bv < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  if (cv[0] < 0.0)
    for (int64_t i = tid; i < w.m; i += 256) U[i * r + j] = from_double<TU>(-to_double(U[i * r + j]));
}

template <typename TA>
void tn_partial(const TA* A, int64_t lda, const double* B, int64_t ldb, int64_t rows, int P, int Q,
                int64_t chunk, double* out, hipStream_t st) {
  const dim3 grid((unsigned)ceil_div(P, kTile), (unsigned)ceil_div(Q, kTile),
                  (unsigned)ceil_div(rows, chunk));
  hipLaunchKernelGGL((tn_partial_kernel<TA>), grid, dim3(256), 0, st, A, lda, B, ldb, rows, P, Q,
                     chunk, out);
}

}  // namespace

size_t wide_chol_lds(int ell) { return (size_t)ell * (ell + 1) / 2 * sizeof(double); }
size_t wide_apply_lds(int ell) { return (size_t)ell * (65 + kApplyCols) * sizeof(double); }
size_t wide_sweep_lds(int np) { return (size_t)np * (np + 1) / 2 * sizeof(double); }

hipError_t launch_qr_wide(const WideQR& w, int ydtype, bool wstep, hipStream_t st) {
  // CholeskyQR2 (up to four passes when a pass is shifted)
  for (int pass = 1; pass <= kQRMaxPasses; ++pass) {
    tn_partial<double>(w.Z, w.ell, w.Z, w.ell, w.m, w.ell, w.ell, kWideRowChunk, w.gpart, st);
    hipLaunchKernelGGL(wide_chol_kernel, dim3(1), dim3(1024), wide_chol_lds(w.ell), st, w, pass);
    hipLaunchKernelGGL(wide_apply_kernel, dim3((unsigned)ceil_div(w.m, 64)), dim3(64),
                       wide_apply_lds(w.ell), st, w);
  }
  if (!wstep) return hipGetLastError();
  // M^T = Y^T Q (s x ell, one chunk: every row of the column sum in order),
  // then the Gram M M^T = (M^T)^T M^T over chunks of s
  switch (ydtype) {
    case TK_F64: tn_partial(static_cast<const double*>(w.Y), w.s, w.Z, w.ell, w.m, (int)w.s, w.ell, w.m, w.Mt, st); break;
    case TK_F32: tn_partial(static_cast<const float*>(w.Y), w.s, w.Z, w.ell, w.m, (int)w.s, w.ell, w.m, w.Mt, st); break;
    case TK_BF16: tn_partial(static_cast<const bf16*>(w.Y), w.s, w.Z, w.ell, w.m, (int)w.s, w.ell, w.m, w.Mt, st); break;
    case TK_F16: tn_partial(static_cast<const f16*>(w.Y), w.s, w.Z, w.ell, w.m, (int)w.s, w.ell, w.m, w.Mt, st); break;
    default: return hipErrorInvalidValue;
  }
  tn_partial<double>(w.Mt, w.ell, w.Mt, w.ell, w.s, w.ell, w.ell, kWideRowChunk, w.cpart, st);
  // rotations stop below rounding level of the output precision (relative to
  // the pair's own scale): FP64 bases need ~u, FP32 bases ~1e-12 suffices
  const double tol = w.udtype == TK_F64 ? 4.0 * kUnit : 1e-12;
  for (int sweep = 0; sweep < kWideMaxSweeps; ++sweep) {
    hipLaunchKernelGGL(wide_sweep_kernel, dim3(1), dim3(kSweepThreads), wide_sweep_lds(w.np), st, w, sweep, tol);
    hipLaunchKernelGGL(wide_vrot_kernel, dim3((unsigned)w.np), dim3(64), 0, st, w, sweep);
  }
  hipLaunchKernelGGL(wide_select_kernel, dim3(1), dim3(256), 0, st, w);
  if (w.udtype == TK_F64)
    hipLaunchKernelGGL((wide_u_kernel<double>), dim3((unsigned)w.r), dim3(256), 0, st, w);
  else
    hipLaunchKernelGGL((wide_u_kernel<float>), dim3((unsigned)w.r), dim3(256), 0, st, w);
  return hipGetLastError();
}

}  // namespace tk
