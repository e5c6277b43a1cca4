// Host-side launchers of the kernels (one translation unit per kernel family).
#pragma once

#include "tk_common.hpp"

namespace tk {

// ---------------------------------------------------------------- sampled sketches
// One unit = one mode (or tree node) S of a tensor viewed as (A, n, B):
// column j of the unfolding is the fiber X[a, :, b], (a, b) = divmod(j, B).
struct SketchUnit {
  const void* X;
  int64_t A, n, B;
  int64_t s;
  const int64_t* idx;   // sorted column indices, or nullptr = every column
  const void* omega;    // [s x ell], double for F64 tensors, float otherwise
  double* partial;      // [nchunks][n][ell]
  double* Z;            // [n][ell]
  void* Y;              // [n][s] in the tensor dtype, or nullptr
  int64_t block_begin;  // first block of this unit in the gather launch
  int64_t out_begin;    // first entry of this unit in the reduce launch
  int32_t ell;
  int32_t nchunks;      // ceil(s / kSketchCols)
  int32_t rowblocks;    // ceil(n / kSketchRows)
  int32_t pad;
};
struct SketchBatch {
  int32_t count;
  int64_t total_blocks;
  int64_t total_out;    // sum over units of n * ell (reduce launch)
  SketchUnit u[kMaxUnits];
  __device__ const SketchUnit& get(int i) const { return u[i]; }
  __device__ int find_block(int64_t blk) const {
    int i = 0;
    while (i + 1 < count && u[i + 1].block_begin <= blk) ++i;
    return i;
  }
  __device__ int find_out(int64_t g) const {
    int i = 0;
    while (i + 1 < count && u[i + 1].out_begin <= g) ++i;
    return i;
  }
};
// the same units in a device table (any number), found by binary search
struct SketchList {
  const SketchUnit* u;
  const int32_t* block_unit;   // unit of every gather block
  int32_t count;
  int32_t pad;
  int64_t total_blocks;
  int64_t total_out;
  __device__ const SketchUnit& get(int i) const { return u[i]; }
  __device__ int find_block(int64_t blk) const { return block_unit[blk]; }
  __device__ int find_out(int64_t g) const {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (u[mid].out_begin <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
  }
};
constexpr int kSketchRows = 64;
constexpr int kSketchCols = 32;
hipError_t launch_sketch(int dtype, const SketchBatch& b, hipStream_t st);
hipError_t launch_sketch_list(int dtype, const SketchList& b, hipStream_t st);

// ---------------------------------------------------------------- CholeskyQR2 + W step
struct QRMat {
  double* Z;            // m x ell, becomes Q
  const void* Y;        // m x s or nullptr
  void* U;              // m x r output or nullptr
  int32_t* info;        // element or nullptr
  double* gpart;        // [nrc][ell][ell]
  double* R;            // [ell][ell]
  int32_t* state;       // [2] pass bookkeeping (passes owed, apply flag)
  double* mpart;        // [nrc][ell][s]
  double* cpart;        // [ncc][ell][ell]
  double* W;            // [ell][r]
  double* utmp;         // [m][r]
  double* amax_v;       // [nrb][r]
  int64_t* amax_i;      // [nrb][r]
  int64_t m, s;
  int32_t ell, r;
  int32_t nrc, ncc, nrb; // row chunks (Gram / Q^T Y), column chunks, row blocks (apply)
  int64_t qty_begin;     // first block of this matrix in the Q^T Y launch
  int32_t small;         // m x ell (and m x r) small enough for the one-workgroup kernels
  int32_t udtype;        // TK_F64 or TK_F32
  int32_t pad2;
};
// a matrix is handled by one workgroup when its rows times columns fit this
// (the FP64 copy of Z, 120 KB, and the Gram share the workgroup's LDS)
constexpr int kQRSmallElems = 15360;
constexpr int kQRSmallRows = 4096;
constexpr int kQRMaxBatch = 16;
constexpr int kQRMaxPasses = 4;
constexpr int kQRRowChunk = 256;
constexpr int kQRColChunk = 64;
constexpr int kQRRowBlock = 64;
struct QRBatch {
  int32_t count;
  QRMat m[kQRMaxBatch];
  __device__ const QRMat& get(int i) const { return m[i]; }
};
// the same descriptors in a device table (batches of any size)
struct QRList {
  const QRMat* m;
  int32_t count;
  int32_t pad;
  __device__ const QRMat& get(int i) const { return m[i]; }
};
// Thin QR and W step for sketch widths kMaxEll < ell <= kWideMaxEll: one
// matrix per launch sequence, its ell x ell matrices in global workspace and
// (packed) in LDS.
constexpr int kWideMaxEll = 192;     // packed FP64 triangle of 192 x 192 in LDS (148 KB)
constexpr int kWideMaxSweeps = 24;   // Jacobi sweeps launched (converged ones exit at once)
constexpr int kWideRowChunk = 1024;  // rows per partial of the Gram products
struct WideQR {
  double* Z;            // m x ell, becomes Q
  const void* Y;        // m x s or nullptr
  void* U;              // m x r output or nullptr
  int32_t* info;        // element or nullptr
  double* gpart;        // [gsplit][ell][ell] partial Grams of Z
  double* R;            // [ell][ell]
  int32_t* state;       // [3 + kWideMaxSweeps] passes owed, apply flag, converged, rotations per sweep
  double* Mt;           // [s][ell] = (Q^T Y)^T
  double* cpart;        // [csplit][ell][ell] partial Grams of M
  double* Ap;           // packed upper triangle of the np x np Jacobi matrix
  double* V;            // [np][np] eigenvectors (columns)
  double* rot;          // [np - 1][np / 2][2] (c, s) of the current sweep
  double* W;            // [ell][r]
  int64_t m, s;
  int32_t ell, r, np;   // np = ell rounded up to even
  int32_t gsplit, csplit;
  int32_t udtype;
};
hipError_t launch_qr_wide(const WideQR& w, int ydtype, bool wstep, hipStream_t st);
hipError_t launch_cholqr(const QRBatch& b, hipStream_t st);
hipError_t launch_wstep(const QRBatch& b, int ydtype, int udtype, hipStream_t st);
// the W step from a given Gram of Q^T Y (cpart, ncc = 1): eigenvectors and U only
hipError_t launch_wstep_gram(const QRBatch& b, int udtype, hipStream_t st);
// host: the table `dev.m` points to, as a host copy (grid sizes, path choice)
hipError_t launch_cholqr_list(const QRList& dev, const QRMat* host, hipStream_t st);
hipError_t launch_wstep_list(const QRList& dev, const QRMat* host, int ydtype, int udtype, hipStream_t st);

// ---------------------------------------------------------------- generic mode products
// out[a][p][b] = sum_q in[a][q][b] * M[p][q],  M[p][q] = Mp[p*rs + q*cs]
struct ModeProduct {
  const void* in;
  void* out;
  const void* M;        // factor dtype (double or float)
  double* Mt;           // scratch of mode_product_scratch(P, Q) doubles
  int64_t A, Q, B;
  int32_t P;
  int32_t rs, cs;
  int32_t accumulate;   // out += instead of out =
  // optional: when B > 1 and there are few output points, the contraction
  // range may be split over up to qsplit_max blocks whose partial sums go to
  // `part` (qsplit_max * A * P * B doubles) and are summed in split order
  int32_t qsplit_max;
  double* part;
};
// doubles of scratch a mode product needs (M as a padded FP64 [Q][P'] table)
int64_t mode_product_scratch(int64_t P, int64_t Q);
// in_dt: dtype of `in`; out_dt, m_dt: TK_F64 or TK_F32
hipError_t launch_mode_product(const ModeProduct& mp, int in_dt, int out_dt, int m_dt,
                               hipStream_t st);

// Last-mode expansion fused with the residual: xhat[a][i] = sum_j T[a][j] F[i][j]
// (T is FP64 A x c, F is n x c in f_dt); optional write of xhat (f_dt) and
// per-block partial sums of (x - xhat)^2 and x^2.
struct ExpandResidual {
  const double* T;
  const void* F;
  const void* X;        // reference or nullptr
  void* Xhat;           // output or nullptr
  void* D;              // output D = s (X - xhat) in f_dt (needs X; may alias it), or nullptr
  const double* scale;  // s = smul * (*scale or 1)
  double smul;
  double* partials;     // [nblocks][2] or nullptr
  double* resid2;       // final [2] or nullptr
  int64_t A, n;
  int32_t c;
  int32_t accumulate;   // Xhat += instead of Xhat =
};
int64_t expand_residual_blocks(int64_t total);
hipError_t launch_expand_residual(const ExpandResidual& e, int x_dt, int f_dt, hipStream_t st);

// ---------------------------------------------------------------- FP32 fused streaming core
// T[a] = F_I^T X[a] F_J for the A slabs X[a] (n_I x n_J) of an FP32 tensor.
struct CoreFused2 {
  const float* X;
  const float* FI;     // n_I x c_I
  const float* FJ;     // n_J x c_J
  float* T;            // A x c_I x c_J
  int64_t A;
  int32_t nI, nJ, cI, cJ;
  int32_t nwaves;      // set by the launcher: waves in the grid
  int32_t pad;
};
bool fused2_supported(int dtype, int order, const int64_t* dims, const int32_t* cols);
hipError_t launch_fused2_f32(const CoreFused2& p, hipStream_t st);
// the same pass with the stage-1 products on BF16 matrix cores at FP32
// accuracy (three-piece split, six products); n_I, n_J in [64, 512]
bool fused2x6_supported(int dtype, int order, const int64_t* dims, const int32_t* cols);
hipError_t launch_fused2x6(const CoreFused2& p, hipStream_t st);

// ---------------------------------------------------------------- small-mode streaming core
// T[a] = F_I^T X[a] F_J for the slabs X[a] (n_I x n_J) of an FP32, BF16 or
// FP16 tensor, or (FH != nullptr) T3[r] = sum_h F_H[h] (x) F_I^T X[r,h] F_J.
struct CoreSlab {
  const void* X;
  const float* FH;      // nH x cH, or nullptr
  const float* FI;      // nI x cI
  const float* FJ;      // nJ x cJ
  float* T;             // (items, [cH,] cI, cJ)
  int64_t items;        // slabs, or runs of nH slabs
  int32_t nH, nI, nJ;
  int32_t cH, cI, cJ;
  int32_t nwaves;       // set by the launcher
  int32_t pad;
};
bool slab_supported(int dtype, int64_t nI, int64_t nJ, int32_t cI, int32_t cJ);
hipError_t launch_core_slab(const CoreSlab& p, int xdt, hipStream_t st);

// ---------------------------------------------------------------- batching form
// Streaming pass of many FP32 tensors (two trailing modes, n <= 96, c <= 16).
struct BatchTensor {
  const float* X;
  const float* FI;      // nI x cI
  const float* FJ;      // nJ x cJ
  float* T;             // (A, cI, cJ)
  int64_t A;            // slabs
  int32_t nI, nJ, cI, cJ;
};
struct BatchChunk {
  int32_t tensor;
  int32_t pad;
  int64_t a0, a1;       // slabs [a0, a1) of the tensor
};
struct BatchSlab {
  const BatchTensor* tensors;
  const BatchChunk* chunks;
  const int32_t* order;        // chunk ids in the order the waves take them
  int32_t* queue;              // one counter, cleared by the launcher
  int32_t nwaves;              // resident waves launched
  int32_t nchunks;
};
constexpr int kBatchMaxN = 96;
constexpr int kBatchMaxC = 16;
size_t batch_slab_lds_bytes();
int batch_slab_waves(int tg, int nbuf);   // resident waves of a variant
hipError_t launch_batch_slab(const BatchSlab& bs, int tg, int nbuf, hipStream_t st);

// Residual of every tensor of a batch over its chunks (taken by the waves
// from a queue in `order`): each chunk writes (r2, x2) into partials[2 chunk],
// then resid2[2 t], resid2[2 t + 1] is the sum over tensor t's chunks
// [tensor_chunk_begin[t], [t + 1]).  T of each tensor holds its core expanded
// over the leading modes.
struct BatchResid {
  const BatchTensor* tensors;
  const BatchChunk* chunks;
  const int32_t* order;         // chunk ids, largest first
  const int32_t* tensor_chunk_begin;
  double* partials;
  double* resid2;
  int32_t* queue;               // one counter, cleared by the launcher
  int32_t nwaves;
  int32_t nchunks;
  int32_t count;
  int32_t pad;
};
int batch_resid_waves();
hipError_t launch_batch_resid(const BatchResid& br, hipStream_t st);

// One remaining mode of many tensors: out[a][p][b] = sum_q F[q][p] in[a][q][b]
// (a projection by F = U_k, Q x P), or with ftrans the expansion
// out[a][p][b] = sum_q F[p][q] in[a][q][b] by rows [p0, p0 + P) of U_k (F
// then points at row p0, row length Q; out at row p0 of the first slab).
struct BatchModeDesc {
  const float* in;
  const float* F;
  float* out;
  int64_t A, Q, B;
  int64_t out_slab;     // floats between consecutive a in out (P B, or n_k B for an expansion)
  int64_t unit_begin;   // first unit (multiple of 4) of this descriptor
  int32_t P;            // <= 32
  int32_t ftrans;
};
struct BatchMode {
  const BatchModeDesc* descs;
  int32_t count;
  int32_t pad;
};
int64_t batch_mode_units(int64_t A, int64_t B);   // padded to whole workgroups
size_t batch_mode_lds_bytes(int64_t Qmax);
hipError_t launch_batch_mode(const BatchMode& bm, int64_t total_units, int64_t Qmax, hipStream_t st);

// ---------------------------------------------------------------- FP32 MFMA mode contraction
// out[a][p][b] = sum_q F[q][p] in[a][q][b] for an FP32 (A, Q, B) tensor, P <= 32.
struct ModeMfma {
  const float* in;
  const float* F;       // Q x P row-major
  void* out;            // (A, P, B), FP32 or FP64
  int64_t A, Q, B;
  int32_t P;
  int32_t ftrans;       // last-mode kernel: F is P x Q row-major (an expansion by F_k)
};
bool mode_mfma_supported(int64_t Q, int64_t B, int32_t P);
hipError_t launch_mode_mfma_f32(const ModeMfma& m, int out_dt, hipStream_t st);
// the last mode (B = 1), up to 192 columns: out[a][p] = sum_q in[a][q] F[q][p]
bool mode_last_mfma_supported(int64_t A, int64_t Q, int32_t P);
hipError_t launch_mode_last_mfma_f32(const ModeMfma& m, int out_dt, hipStream_t st);
// sum (X - Xh)^2 and sum X^2 over n FP32 entries (FP64): per-block pairs into
// partials (2 resid_pair_blocks(n) doubles), summed into resid2[2] in a fixed
// order when resid2 != NULL; with D, also D = smul (*scale or 1) (X - Xh)
// (D may alias X or Xh)
int64_t resid_pair_blocks(int64_t n);
hipError_t launch_resid_pair_f32(const float* X, const float* Xh, int64_t n, float* D, const double* scale,
                                 double smul, double* partials, double* resid2, hipStream_t st);
// resid2 = the fixed-order sum of npairs (r, x) pairs
hipError_t launch_pair_sum(const double* partials, int64_t npairs, double* resid2, hipStream_t st);

// ---------------------------------------------------------------- FP32 fused streaming residual
// sum (X[a] - F_I T[a] F_J^T)^2 and sum X[a]^2 over the A slabs of an FP32 tensor.
struct ResidFused2 {
  const float* X;
  const float* T;      // A x c_I x c_J, the core expanded over the leading modes
  const float* FI;     // n_I x c_I
  const float* FJ;     // n_J x c_J
  float* Xhat;         // optional output, prod(dims)
  float* D;            // optional output D = s (X - X_hat), s = smul * (*scale or 1); may alias X
  const double* scale; // device scalar or nullptr
  double smul;
  double* partials;    // [resid2_waves(A)][2]
  double* resid2;      // [2] or nullptr
  int64_t A;
  int32_t nI, nJ, cI, cJ;
  int32_t nwaves;      // set by the launcher
  int32_t pad;
};
bool resid2_supported(int dtype, int order, const int64_t* dims, const int32_t* cols);
int64_t resid2_waves(int64_t A);
hipError_t launch_resid2_f32(const ResidFused2& p, hipStream_t st);

// ---------------------------------------------------------------- small-mode streaming residual
// sum (X[a] - F_I T[a] F_J^T)^2 and sum X[a]^2 over the A slabs (n_I x n_J,
// both <= 64; ranks <= 16) of a BF16, FP16 or FP32 tensor, FP32 factors and T
struct ResidSlab {
  const void* X;
  const float* T;       // A x c_I x c_J
  const float* FI;      // n_I x c_I
  const float* FJ;      // n_J x c_J
  double* partials;     // [resid_slab_waves(A)][2]
  double* resid2;       // [2] or nullptr
  int64_t A;
  int32_t nI, nJ, cI, cJ;
  int32_t nwaves;       // set by the launcher
  int32_t pad;
};
bool resid_slab_supported(int x_dtype, int order, const int64_t* dims, const int32_t* cols);
// the pipelined form (several slabs in flight per wave, 16- or 8-byte loads of
// four entries), used by launch_resid_slab where it applies
bool slab_resid_pipe_supported(int x_dtype, int64_t nI, int64_t nJ);
hipError_t launch_slab_resid_pipe(const ResidSlab& p, int x_dtype, int max_waves, hipStream_t st);
int64_t resid_slab_waves(int64_t A);
hipError_t launch_resid_slab(const ResidSlab& p, int x_dtype, hipStream_t st);

// ---------------------------------------------------------------- H-Tucker transfers
// B[i][j][k] = sum_{a,b} US[a*nr + b][i] Ul[a][j] Ur[b][k]
struct Transfer {
  const void* US; const void* Ul; const void* Ur;
  void* Bout;
  double* V;            // workspace [nl][rS][rr]
  double* Mt;           // workspace: mode_product_scratch(rr, nr) doubles
  int64_t nl, nr;
  int32_t rS, rl, rr;
  int32_t pad;
};
hipError_t launch_transfer(const Transfer& t, int f_dt, hipStream_t st);

// ---------------------------------------------------------------- two-sided product
// O1 = X P1 (n1 x k1) and O2 = P2^T X (k2 x n2) in one read of an FP32 X
// (n1 x n2 row-major), FP64 accumulation, P1 / P2 FP32 or FP64, k1, k2 <= 16.
struct TwoSide {
  const float* X;
  const void* P1;       // n2 x k1
  const void* P2;       // n1 x k2
  double* out1;         // n1 x k1
  double* out2;         // k2 x n2, or n2 x k2 with out2_transposed
  double* part1;        // twoside_partials(n1, n2) doubles (part2 follows part1)
  double* part2;        // set by the launcher
  int64_t n1, n2;
  int32_t k1, k2;
  int32_t out2_transposed;
  int32_t nrt, nct;     // set by the launcher
  int32_t pad;
};
bool twoside_supported(int x_dtype, int64_t n1, int64_t n2, int k1, int k2);
int64_t twoside_partials(int64_t n1, int64_t n2);
hipError_t launch_twoside(const TwoSide& ts, int p_dtype, hipStream_t st);

// ---------------------------------------------------------------- H-Tucker root pass
// B_R[j][k] = sum_{a,b} UL[a][j] X[a][b] UR[b][k] for an FP32 X (nL x nR), FP64 bases.
struct RootPass {
  const float* X;
  const double* UL;     // nL x rL
  const double* UR;     // nR x rR
  double* partials;     // root_pass_partials(nL, nR) doubles: workgroup partials, then segment sums
  double* out;          // rL x rR
  int64_t nL, nR;
  int32_t rL, rR;
  int32_t nblocks;      // set by the launcher
  int32_t qsplit;       // column splits per row block, set by the launcher
};
bool root_pass_supported(int dtype, int64_t nL, int64_t nR, int rL, int rR);
int64_t root_pass_blocks(int64_t nL, int64_t nR);
int64_t root_pass_partials(int64_t nL, int64_t nR);   // doubles of RootPass::partials
// brackets the streaming kernel with the profiler's events
hipError_t launch_root_pass(const RootPass& p, hipStream_t st);

// ---------------------------------------------------------------- H-Tucker full tensor
// xhat[a][b] = sum_k T[a][k] UR[b][k] over the n_l x n_r matricisation, with
// T = U_Rl B_R padded to rpad columns; optional reference X (partials of
// ||X - xhat||^2 and ||X||^2) and optional output Xh.
struct HTExpand {
  const double* T;      // nL x rpad (columns rr.. rpad-1 zero)
  const double* UR;     // nR x rr
  const void* X;        // reference (x_dt) or nullptr
  void* Xh;             // output (out_dt) or nullptr
  double* partials;     // [ntile * groups][2] or nullptr
  double* resid2;       // final [2] or nullptr
  int64_t nL, nR;
  int32_t rr, rpad;     // rpad = ht_expand_rpad(rr)
  int64_t ntile, groups, rows_per_group;   // set by ht_expand_grid
};
int ht_expand_rpad(int rr);           // 8, 12, 16, 32 or 64; 0 = rank above 64
void ht_expand_grid(HTExpand& p);     // fills ntile, groups, rows_per_group
hipError_t launch_ht_expand(const HTExpand& p, int x_dt, int out_dt, hipStream_t st);   // dt -1 = absent
hipError_t launch_ht_rowmat(const double* UL, const double* BR, double* T, int64_t nL, int rl, int rr,
                            int rpad, hipStream_t st);
// out[c][r] = in[r][c] (rows x cols, FP64)
hipError_t launch_transpose_f64(const double* in, double* out, int64_t rows, int64_t cols, hipStream_t st);
// Omega of a dense node sketch, [(a B + b)][e] -> [a][e][b] (dtype TK_F32 or TK_F64)
hipError_t launch_omega_to_unfolded(const void* om, void* out, int dt, int64_t A, int64_t B, int ell,
                                    hipStream_t st);
// C[j][k][i] = B[i][j][k] (to_core) or the inverse permutation
hipError_t launch_permute_transfer(const double* in, double* out, int rS, int rl, int rr, bool to_core,
                                   hipStream_t st);

// ---------------------------------------------------------------- unfolded products (VJPs)
// out[i][a] (+)= sum_{p,q} A[p][i][q] B[p][a][q]: A is (pre, n, post), B is
// (pre, c, post); the mode-k unfolding product A^(k) (B^(k))^T.
struct UnfoldGemm {
  const void* A;        // a_dt
  const void* B;        // b_dt
  void* out;            // n x c, out_dt
  double* partials;     // [splits][n][c]
  int64_t pre, post;
  int32_t n, c;
  int32_t splits;       // partial sums over ranges of (p, q), summed in order
  int32_t accumulate;
};
int32_t unfold_gemm_splits(int64_t n, int64_t c, int64_t pre_post);
hipError_t launch_unfold_gemm(const UnfoldGemm& g, int a_dt, int b_dt, int out_dt, hipStream_t st);

// ---------------------------------------------------------------- trailing factor gradients
// Fbar_J = sum_a Y[a]^T F_I K[a], Fbar_I = sum_a Y[a] F_J K[a]^T over the A
// slabs Y[a] (n_I x n_J) of an FP32 tensor, K[a] c_I x c_J (one pass on MFMA;
// per-workgroup partials, then an FP64 sum in workgroup order).
struct VjpTrail {
  const float* X;       // A x n_I x n_J
  const float* K;       // A x c_I x c_J
  const float* FI;      // n_I x c_I
  const float* FJ;      // n_J x c_J
  float* partI;         // [nblocks][vjp_trail_rows_i(n_I)][32]
  float* partJ;         // [nblocks][vjp_trail_rows_j(n_J)][32]
  int64_t A;
  int32_t nI, nJ, cI, cJ;
  int32_t nblocks;
  int32_t pad;
};
bool vjp_trail_supported(int64_t nI, int64_t nJ, int cI, int cJ, int64_t A);
int vjp_trail_blocks(int64_t A);
int64_t vjp_trail_rows_i(int64_t nI);
int64_t vjp_trail_rows_j(int64_t nJ);
// out_dt: dtype of Fbar (TK_F32 or TK_F64); either Fbar may be NULL
hipError_t launch_vjp_trail(const VjpTrail& p, void* FbarI, void* FbarJ, int out_dt, int accumulate,
                            hipStream_t st);

// ---------------------------------------------------------------- conversions
hipError_t launch_convert(const double* in, void* out, int out_dt, int64_t n, hipStream_t st);
hipError_t launch_to_f64(const void* in, int in_dt, double* out, int64_t n, hipStream_t st);

// ---------------------------------------------------------------- measurement
int stream_read_blocks();
hipError_t launch_stream_read(const void* x, int64_t bytes, double* partials, int32_t blocks, hipStream_t st);

// ---------------------------------------------------------------- seeded sketch draw
constexpr int kDrawMaxS = 4096;   // fibers per sketch (LDS sort of at most 4096 keys)
struct DrawUnit {
  int64_t ncols;        // columns of the unfolding
  int64_t* idx;         // [s] out: sorted distinct indices
  void* omega;          // [s][ell] out: Gaussian test matrix
  int32_t s, ell;
};
struct DrawBatch {
  DrawUnit u[kMaxUnits];
  int64_t omega_begin[kMaxUnits + 1];   // prefix of s ell
  uint64_t seed;
  int32_t count;
  int32_t omega_dtype;
};
size_t draw_indices_lds_bytes(int smax);
hipError_t launch_draw(const DrawBatch& b, int smax, hipStream_t st);

}  // namespace tk
