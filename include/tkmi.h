/*
 * tkmi -- randomized (H-)Tucker decomposition on MI355X (gfx950).
 *
 * C ABI of libtkmi.so.  The operations follow the problem statements of
 * Sub-R-HOSVD (Algorithm 1: [S, {U_k}] = Sub-R-HOSVD(X, r, p, s)) and
 * Sub-R-RtL-HT (Algorithm 2: [{U_k}, {B_S}] = Sub-R-RtL-HT(X, T, r, w, p)) of
 * "A practical mode-parallel implementation of the (H-)Tucker decomposition
 * via randomization".  The random quantities of those algorithms (the fiber
 * samples E_k and the Gaussian matrices Omega_k) are passed in: drawn by the
 * caller, or on the device by tucker_draw_sketches from a seeded stream.
 *
 * Conventions shared by every entry point
 *  - Layout: dense tensors are C-ordered (last mode fastest).  The column
 *    index of the mode-k unfolding X^(k) is the C-order linear index of the
 *    remaining modes in increasing mode order; the rows of a multi-mode
 *    unfolding X^(S) are C-ordered over the modes of S.  Matrices are
 *    row-major.  All sizes and indices are 64-bit.
 *  - Ownership: every data pointer is a device pointer owned by the caller;
 *    the library never allocates or frees caller memory.  Descriptor structs
 *    and pointer arrays are host memory, read during the call only.
 *  - Workspace: `ws` is caller-provided device memory of *ws_bytes bytes.
 *    Calling with ws == NULL is a size query: the required byte count is
 *    written to *ws_bytes, TK_OK is returned and nothing is enqueued.
 *  - Asynchrony: work is enqueued on `stream` (a hipStream_t; NULL = the
 *    default stream) and the call returns without synchronising.  Calls on
 *    one stream that share a workspace are ordered by the stream.
 *  - Errors: arguments are validated on the host before anything is
 *    enqueued, so a call that returns an error has no side effects.
 *    tk_last_error() returns the calling thread's message for the last
 *    non-OK status.  Numerical events (a Gram matrix that is not numerically
 *    positive definite) are reported through a device `info` array, as in
 *    LAPACK.
 *  - Determinism: the same inputs on the same device give bitwise-identical
 *    outputs (all reductions have a fixed order, no floating-point atomics).
 */
#ifndef TKMI_H
#define TKMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TK_MAX_ORDER 16

/* Bits of the device `info` words of tucker_qr and htucker_decompose. */
#define TK_INFO_SHIFT_FIRST 1        /* the first CholeskyQR pass was shifted */
#define TK_INFO_SHIFT_LATER 2        /* a later CholeskyQR pass was shifted */
#define TK_INFO_CHOL_FAILED 4        /* a Cholesky failed even with the shift */
#define TK_INFO_EIG_NOT_CONVERGED 8  /* the W step's eigensolver ran out of sweeps */

typedef enum { TK_F64 = 0, TK_F32 = 1, TK_BF16 = 2, TK_F16 = 3 } tk_dtype;

typedef enum {
  TK_OK = 0,
  TK_EINVAL = 1,        /* invalid argument (message in tk_last_error) */
  TK_EWORKSPACE = 2,    /* workspace smaller than the size query returned */
  TK_ENOTPD = 3,        /* reserved: numerical failure reported on the host */
  TK_EDEVICE = 4,       /* a HIP call or kernel launch failed */
  TK_EUNSUPPORTED = 5   /* valid request outside what this build implements */
} tk_status;

/* Dense order-d tensor in device memory (C-order).  Factors, cores, sketches
 * and bases that belong to a tensor use its "factor dtype": TK_F64 for an
 * F64 tensor, TK_F32 for F32, BF16 and F16 tensors. */
typedef struct {
  int32_t order;                 /* 1 .. TK_MAX_ORDER */
  int32_t dtype;                 /* tk_dtype of the stored entries */
  int64_t dims[TK_MAX_ORDER];    /* n_1 .. n_d, each >= 1 */
  const void* data;              /* device pointer to prod(dims) entries */
} tk_tensor;

/* Fiber sample and Gaussian test matrix of one mode (or one tree node):
 * the sampling matrix E_k of Section 3.1 and Omega_k of Algorithm 1. */
typedef struct {
  int64_t s;             /* number of sampled columns, ell <= s <= ncols */
  int32_t ell;           /* sketch width r + p (>= 1) */
  int32_t reserved;      /* must be 0 */
  const int64_t* idx;    /* device [s]: strictly increasing column indices of the
                            unfolding, each in [0, ncols); NULL = every column
                            (then s must equal ncols: the dense R-HOSVD sketch) */
  const void* omega;     /* device [s x ell] row-major, factor dtype */
} tk_sketch;

/* Balanced dimension tree (Section 4, dimension-tree definition), heap order,
 * node 0 = root.  Every node covers the contiguous modes
 * first_mode[t] .. first_mode[t] + num_modes[t] - 1; left/right are child
 * node indices or -1 for a leaf, and the left child covers the first modes. */
typedef struct {
  int32_t num_nodes;
  const int32_t* left;
  const int32_t* right;
  const int32_t* first_mode;
  const int32_t* num_modes;
} tk_tree;

/* Range sketches of every mode in one call (Algorithm 1, fiber sampling and
 * sketch steps; Section 3.1):  Y_k = X^(k) E_k  (n_k x s_k, the sampled mode-k
 * fibers, gathered without forming any unfolding) and Z_k = Y_k Omega_k
 * (n_k x ell_k).
 *   X      tensor (any dtype).
 *   sk     host array [order] of sketches, one per mode.
 *   Z      host array [order] of device pointers, Z[k] is n_k x ell_k FP64,
 *          row-major (accumulated in FP64 whatever the tensor dtype).
 *   Y      NULL, or host array [order] of device pointers (entries may be
 *          NULL): Y[k] receives Y_k (n_k x s_k, row-major, X's dtype), the
 *          input of the W step of tucker_qr.
 * Errors: TK_EINVAL for a bad descriptor, ell > s, s > ncols, a non-zero
 * reserved field or NULL required pointers; TK_EUNSUPPORTED for ell > 192;
 * TK_EWORKSPACE; TK_EDEVICE. */
tk_status tucker_sketch_all_modes(const tk_tensor* X, const tk_sketch* sk, double* const* Z,
                                  void* const* Y, void* ws, size_t* ws_bytes, void* stream);

/* tucker_sketch_all_modes for callers that cannot allocate device memory or
 * provide a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): same arguments, validation, kernels and
 * results, with the per-chunk partial sketches kept in a fixed 64 MiB device
 * array inside the library instead of a caller workspace.  No hipMalloc,
 * hipFree or other allocation is made.  Each GPU holds its own copy of the
 * array from the first call on it until the process ends; every call on a
 * GPU reuses it, so calls that overlap on one GPU (two streams, two host
 * threads) race and must be ordered by the caller.  The scratch a call needs
 * is sum over modes of ceil(s_k / 32) n_k ell_k doubles (256-byte aligned per
 * mode): about 27.5 MB for four modes of n = 256, s = 2560, ell = 42.
 * Errors: as tucker_sketch_all_modes, and TK_EUNSUPPORTED when the call
 * needs more than the fixed 64 MiB (the message gives the size). */
tk_status tucker_sketch_all_modes_noalloc(const tk_tensor* X, const tk_sketch* sk, double* const* Z,
                                          void* const* Y, void* stream);

/* Thin QR of a batch of sketches and the rank truncation of Algorithm 1
 * (orthonormal basis step, then W_k = dominant r_k left singular vectors of
 * Q_k^T Y_k and U_k = Q_k W_k).  The QR is CholeskyQR2 with an FP64 Gram and
 * FP64 Cholesky.  When a Cholesky pivot is not safely positive that pass is
 * shifted (shifted CholeskyQR, Fukaya et al. 2020) and two plain passes
 * follow it, so an exactly rank-deficient Z_i still yields ell_i orthonormal
 * columns (at most four passes).  info[i]: bit 0 = first pass shifted,
 * bit 1 = a later pass shifted, bit 2 = a Cholesky failed even with the
 * shift (the result is then not reliable), bit 3 = the W step's Jacobi
 * eigensolver used up its sweeps with rotations still above the stopping
 * test (W_i may then be inaccurate).  Q_i is unique up to rounding
 * when Z_i has full column rank (R_ii > 0).
 *   nmat     number of matrices.
 *   m, ell   host arrays [nmat]: rows and columns of Z_i (ell_i <= m_i).
 *   Z        host array [nmat] of device FP64 m_i x ell_i row-major, replaced
 *            by Q_i.
 *   Y        NULL (QR only) or host array [nmat] of device m_i x s_i row-major
 *            matrices of dtype ydtype.
 *   s, r     host arrays [nmat] (ignored when Y is NULL): columns of Y_i and
 *            target rank r_i (1 <= r_i <= ell_i).
 *   U        host array [nmat] of device m_i x r_i row-major outputs in
 *            udtype (TK_F64 or TK_F32); each column's largest-magnitude entry
 *            (first on ties) is made positive.  With r_i = ell_i the columns
 *            of U_i span Range(Q_i).
 *   info     device int32 [nmat] (may be NULL).
 * Widths up to 64 run as one batch (one workgroup per matrix); wider ones,
 * up to 192, one matrix at a time with the same arithmetic rules (their
 * ell x ell matrices packed in LDS and in the workspace).  When a call has
 * both, the wide ones run on a library-owned second stream of the current
 * device, forked from and joined back into `stream` within the call; calls
 * from several host threads take turns on it (serialised by a lock around
 * the enqueue), so they stay correct but their wide matrices do not overlap.
 * Errors: TK_EINVAL, TK_EUNSUPPORTED (ell_i > 192), TK_EWORKSPACE, TK_EDEVICE. */
tk_status tucker_qr(int32_t nmat, const int64_t* m, const int32_t* ell, double* const* Z,
                    const void* const* Y, int32_t ydtype, const int64_t* s, const int32_t* r,
                    void* const* U, int32_t udtype, int32_t* info, void* ws, size_t* ws_bytes,
                    void* stream);

/* Core projection (Algorithm 1, core step):  G = X x_1 F_1^T x_2 ... x_d F_d^T.
 * The one full read of X.
 *   F      host array [order] of device n_k x c_k row-major factors in the
 *          factor dtype.
 *   cols   host array [order]: c_k (1 <= c_k <= n_k, c_k <= 192).
 *   G      device output c_1 x ... x c_d (C-order), factor dtype.
 * Accumulation: FP64 for F64 tensors; FP32 MFMA with FP64 combination of
 * partial sums for F32; BF16/F16 MFMA with FP32 accumulation for BF16/F16
 * tensors (factors enter as a hi+lo pair).  Modes that no fused pass covers
 * are contracted one at a time, the largest reduction n_k / c_k first.
 * Errors: TK_EINVAL, TK_EUNSUPPORTED (c_k > 192), TK_EWORKSPACE, TK_EDEVICE. */
tk_status tucker_core(const tk_tensor* X, const void* const* F, const int32_t* cols, void* G,
                      void* ws, size_t* ws_bytes, void* stream);

/* Reconstruction X_hat = G x_1 F_1 x_2 ... x_d F_d (Tucker format, Section 3)
 * and, fused with it, the squared residual against a reference tensor.
 *   dims, order  size n_1..n_d of X_hat; G is c_1 x ... x c_d in the factor
 *                dtype `fdtype`, F as in tucker_core.
 *   Xref   NULL or the reference tensor (same dims; its dtype decides fdtype).
 *   Xhat   NULL or a device output of prod(dims) entries in fdtype.
 *   resid2 NULL or device double[2]: ||Xref - X_hat||_F^2 and ||Xref||_F^2,
 *          accumulated in FP64 (requires Xref; the FP32 matrix-core pass sums
 *          the squared differences of 32 entries in FP32 before adding them
 *          to the FP64 sum).
 * At least one of Xhat and resid2 must be non-NULL.
 * Errors: TK_EINVAL, TK_EWORKSPACE, TK_EDEVICE. */
tk_status tucker_reconstruct(int32_t order, const int64_t* dims, int32_t fdtype, const void* G,
                             const void* const* F, const int32_t* cols, const tk_tensor* Xref,
                             void* Xhat, double* resid2, void* ws, size_t* ws_bytes,
                             void* stream);

/* Sub-R-RtL-HT (Algorithm 2) on a balanced dimension tree: for every non-root
 * node S the sampled sketch Y_S = X^(S) E_S, Z_S = Y_S Omega_S, its QR and W
 * step giving the explicit basis U_S (n_S x r_S); the transfer tensor
 * B_S(i,j,k) = <U_S(:,i), U_Sl(:,j) kron U_Sr(:,k)> of every internal non-root
 * node (transfer-tensor equation of Section 4); and the root transfer
 * B_R(0,j,k) = <vec X, U_Rl(:,j) kron U_Rr(:,k)> (one full read of X).
 *   X       tensor (any dtype).
 *   tree    balanced tree over X's modes (num_nodes = 2 order - 1).
 *   rank    host int32 [num_nodes]: r_S for every node (rank[0] is ignored;
 *           the root rank is 1).
 *   sk      host array [num_nodes] of sketches (sk[0] ignored).
 *   U       host array [num_nodes] of device outputs, U[t] is n_S x r_S
 *           row-major FP64 (U[0] ignored).
 *   B       host array [num_nodes] of device outputs, B[t] is r_t x r_l x r_r
 *           (C-order) for internal nodes, 1 x r_l x r_r for the root, FP64;
 *           entries for leaves are ignored.  Bases and transfers are FP64 for
 *           every tensor dtype (they are small, and their storage precision
 *           would otherwise bound the accuracy of the format).
 *   info    device int32 [num_nodes] or NULL (as in tucker_qr, index = node).
 * Errors: TK_EINVAL (also for a tree that is not the balanced heap tree of
 * this order), TK_EWORKSPACE, TK_EDEVICE. */
tk_status htucker_decompose(const tk_tensor* X, const tk_tree* tree, const int32_t* rank,
                            const tk_sketch* sk, void* const* U, void* const* B, int32_t* info,
                            void* ws, size_t* ws_bytes, void* stream);

/* Full tensor of an H-Tucker format and its residual (Section 4: the root
 * relation X^(Rl) = U_Rl B_R U_Rr^T and the nestedness U_S = (U_Sl kron U_Sr)
 * (B_S^(1))^T of the bases of internal nodes).  The nested bases of the
 * internal non-root nodes are formed from the leaves upwards; the root
 * expansion xhat[a][b] = sum_k (U_Rl B_R)[a][k] U_Rr[b][k] over the
 * n_Rl x n_Rr matricisation is one streaming pass, fused with the residual.
 *   order, dims  n_1 .. n_d (order >= 2).
 *   tree    the balanced heap tree of this order (as for htucker_decompose).
 *   rank    host int32 [num_nodes]: r_t of every node (rank[0] ignored).
 *   U       host array [num_nodes]: U[t] for every leaf t is n_t x r_t
 *           row-major FP64 (device); other entries ignored.
 *   B       host array [num_nodes]: B[t] for every internal node is
 *           r_t x r_l x r_r (C-order) FP64 (device), the root's 1 x r_l x r_r;
 *           entries of leaves ignored.  The format is the output layout of
 *           htucker_decompose (its leaf bases and transfer tensors).
 *   Xref    NULL or a reference tensor of the same dims (any dtype).
 *   Xhat    NULL or a device output of prod(dims) entries in xhat_dtype
 *           (TK_F32 or TK_F64); computed in FP64.
 *   resid2  NULL or device double[2]: ||Xref - Xhat||_F^2 and ||Xref||_F^2
 *           (FP64 sums in a fixed order; requires Xref).
 * At least one of Xhat and resid2 must be non-NULL.  The rank of the root's
 * right child is at most 64.
 * Errors: TK_EINVAL, TK_EUNSUPPORTED (that rank above 64), TK_EWORKSPACE,
 * TK_EDEVICE. */
tk_status htucker_reconstruct(int32_t order, const int64_t* dims, const tk_tree* tree, const int32_t* rank,
                              const void* const* U, const void* const* B, const tk_tensor* Xref,
                              void* Xhat, int32_t xhat_dtype, double* resid2, void* ws, size_t* ws_bytes,
                              void* stream);

/* Vector-Jacobian product of the H-Tucker format's full tensor with respect
 * to its parameters (the differentiation form of the format; chain rule
 * through the two relations above): given H = dL/dXhat (prod(dims) entries,
 * h_dtype TK_F32 or TK_F64),
 *   root:      Bbar_R = U_Rl^T H U_Rr,  Ubar_Rl = H U_Rr B_R^T,
 *              Ubar_Rr = H^T U_Rl B_R   (H viewed as n_Rl x n_Rr);
 *   internal:  with K = U_l kron U_r,  Bbar_S^(1) = Ubar_S^T K and
 *              Ubar_l, Ubar_r the contractions of Ubar_S B_S^(1) with U_r, U_l;
 * from the root's children down to the leaves.
 *   Bbar    host array [num_nodes] of device FP64 outputs shaped like B
 *           (every internal node, root included; leaf entries ignored).
 *   Ubar    host array [num_nodes] of device FP64 outputs shaped like U
 *           (every leaf; other entries ignored).
 * Other arguments as for htucker_reconstruct.  H is read twice (one
 * one-sided contraction and one unfolded product).
 * Errors: TK_EINVAL, TK_EUNSUPPORTED, TK_EWORKSPACE, TK_EDEVICE. */
tk_status htucker_reconstruct_vjp(int32_t order, const int64_t* dims, const tk_tree* tree,
                                  const int32_t* rank, const void* const* U, const void* const* B,
                                  const void* H, int32_t h_dtype, void* const* Bbar, void* const* Ubar,
                                  void* ws, size_t* ws_bytes, void* stream);

/* Vector-Jacobian product of the core projection G = X x_k F_k^T (the
 * differentiation form of the method; follows from the TTM definition of
 * Section 2.2): given Gbar (c_1 x .. x c_d),
 *   Xbar  (+)= Gbar x_1 F_1 .. x_d F_d             (prod(dims), factor dtype)
 *   Fbar_k (+)= (X x_{j!=k} F_j^T)^(k) (Gbar^(k))^T  (n_k x c_k, factor dtype)
 * Xbar or Fbar (or individual Fbar[k]) may be NULL to skip them.  accumulate
 * != 0 adds to the outputs instead of overwriting them.  X is recontracted,
 * no unfolding is stored: for FP32 tensors whose two trailing modes take a
 * fused streaming pass (sizes up to 256, c up to 32) the factor gradients
 * read X twice (the partial core of the trailing modes, then one matrix-core
 * pass for their gradients); otherwise once per mode.
 * Errors: TK_EINVAL, TK_EWORKSPACE, TK_EDEVICE. */
tk_status tucker_core_vjp(const tk_tensor* X, const void* const* F, const int32_t* cols,
                          const void* Gbar, void* Xbar, void* const* Fbar, int32_t accumulate,
                          void* ws, size_t* ws_bytes, void* stream);

/* Vector-Jacobian product of the reconstruction X_hat = G x_k F_k: given
 * H = dL/dX_hat (prod(dims), factor dtype),
 *   Gbar   = H x_1 F_1^T .. x_d F_d^T                  (c_1 x .. x c_d)
 *   Fbar_k = H^(k) ((G x_{j!=k} F_j)^(k))^T            (n_k x c_k)
 * Gbar or Fbar may be NULL.  Errors as above. */
tk_status tucker_reconstruct_vjp(int32_t order, const int64_t* dims, int32_t fdtype,
                                 const void* G, const void* const* F, const int32_t* cols,
                                 const void* H, void* Gbar, void* const* Fbar, void* ws,
                                 size_t* ws_bytes, void* stream);

/* Backward of the projection loss L(X, F) = ||X - (X x_k F_k^T) x_k F_k||_F^2
 * (the core projection followed by the reconstruction, F_k free n_k x c_k
 * matrices; the two VJPs above chained with the loss's direct term):
 *   H     = dL/dX_hat = -2 lbar (X - X_hat)
 *   Gbar  = H x_k F_k^T
 *   Fbar_k = H^(k) ((G x_{j!=k} F_j)^(k))^T + (X x_{j!=k} F_j^T)^(k) (Gbar^(k))^T
 *   Xbar  = Gbar x_k F_k + 2 lbar (X - X_hat)
 *   X      tensor, TK_F64 or TK_F32; F, cols as in tucker_core.
 *   G      the forward's core X x_k F_k^T (c_1 x .. x c_d, X's dtype).
 *   lbar   device double: the adjoint of L (NULL = 1).
 *   Xbar   NULL or a device output shaped like X (X's dtype).  It also holds
 *          H during the call; without it the workspace holds an X-sized H.
 *   Fbar   NULL or host array of device outputs n_k x c_k (entries may be NULL).
 * X is read three times and H is written once and read three times (in Xbar
 * when given); no other X-sized buffer is used.
 * Errors: TK_EINVAL, TK_EUNSUPPORTED (other dtypes, c_k > 192), TK_EWORKSPACE,
 * TK_EDEVICE. */
tk_status tucker_projection_loss_vjp(const tk_tensor* X, const void* const* F, const int32_t* cols,
                                     const void* G, const double* lbar, void* Xbar, void* const* Fbar,
                                     void* ws, size_t* ws_bytes, void* stream);

/* Batching form of Sub-R-HOSVD (Algorithm 1 for many independent tensors at
 * once): every mode of every tensor is sketched, orthonormalised, truncated
 * and projected by one fixed sequence of persistent launches (sketch, QR,
 * W step, streaming core pass, remaining modes), whatever the orders and
 * sizes of the tensors; optionally followed by the reconstruction residual
 * of every tensor (Tucker format, Section 3: the core expanded back over the
 * leading modes, then one pass over X that never stores X_hat).  A plan holds the descriptor tables in the caller's
 * workspace; running it allocates nothing, does not synchronise and records
 * no memset, so a run can be captured in a HIP graph and replayed.
 *
 * tucker_batch_plan_create
 *   count   number of tensors (>= 1).
 *   X       host array [count] of FP32 tensors of order >= 3, the two
 *           trailing modes at most 96, at most 2^29 entries each.
 *   ranks   host int32 [sum of orders]: r_k of every mode, tensor by tensor
 *           (1 <= r_k <= ell_k; r_k <= 16 for the two trailing modes and
 *           <= 32 for the others).
 *   sk      host array [sum of orders] of sketches, as in
 *           tucker_sketch_all_modes (omega FP32).
 *   U       host array [sum of orders] of device outputs, n_k x r_k FP32
 *           row-major (U_k = Q_k W_k, sign rule as in tucker_qr).
 *   G       host array [count] of device outputs, r_1 x .. x r_d FP32.
 *   info    device int32 [sum of orders] or NULL (as in tucker_qr).
 *   resid2  NULL, or device double [2 count]: every run then also writes
 *           ||X_t - X_hat_t||_F^2 and ||X_t||_F^2 of tensor t at [2t], [2t+1]
 *           (X_hat_t = G_t x_1 U_1 .. x_d U_d from this run's outputs; FP32
 *           products, FP64 sums in an order fixed by the plan).
 *   ws      caller workspace; NULL is a size query (nothing else happens).
 *   stream  stream for the table upload (the call waits for it).
 *   plan    receives the plan (host object; valid while ws, the tensors,
 *           sketches and outputs stay allocated).
 * tucker_batch_run enqueues one run on `stream`.
 * tucker_batch_autotune runs the plan once, then times the streaming pass
 *   for each tile grouping, load-pipeline depth and chunk size and keeps
 *   the fastest; it synchronises (do not call it while capturing).  A text
 *   report is written to `report` (may be NULL).
 * Errors: TK_EINVAL, TK_EUNSUPPORTED, TK_EWORKSPACE, TK_EDEVICE. */
typedef struct tk_batch_plan tk_batch_plan;
tk_status tucker_batch_plan_create(int32_t count, const tk_tensor* X, const int32_t* ranks,
                                   const tk_sketch* sk, void* const* U, void* const* G, int32_t* info,
                                   double* resid2, void* ws, size_t* ws_bytes, void* stream,
                                   tk_batch_plan** plan);
tk_status tucker_batch_run(const tk_batch_plan* plan, void* stream);
tk_status tucker_batch_autotune(tk_batch_plan* plan, void* stream, char* report, size_t report_bytes);
void tucker_batch_plan_destroy(tk_batch_plan* plan);

/* The streaming pass's schedule of a plan (what tucker_batch_autotune
 * chooses), so that a caller can store a tuned choice and apply it to a later
 * plan of the same shapes without timing again.
 *   tiles_per_unit, buffers  the pass's form: (0, 0) whole slabs in a
 *           pipeline of several slabs per wave, or 16-row tile units with
 *           (1, 2), (2, 2) or (1, 3) (tiles per unit, buffers in flight).
 *   chunk_bytes  bytes of X per scheduled chunk, in [32 KiB, 64 MiB].
 * tucker_batch_set_schedule rebuilds and uploads the chunk schedule on
 * `stream` and waits for it (do not call it while capturing).  Results do not
 * depend on the schedule.
 * Errors: TK_EINVAL (NULL arguments, another form, chunk size out of range),
 * TK_EDEVICE. */
tk_status tucker_batch_get_schedule(const tk_batch_plan* plan, int32_t* tiles_per_unit, int32_t* buffers,
                                    int64_t* chunk_bytes);
tk_status tucker_batch_set_schedule(tk_batch_plan* plan, int32_t tiles_per_unit, int32_t buffers,
                                    int64_t chunk_bytes, void* stream);

/* Seeded device-side draw of sampled sketches (the sampling of Algorithm 1,
 * Section 3.1: column indices uniform without repetition and a Gaussian
 * test matrix), so no host generation or upload is needed.  For each unit
 * k < nunits (nunits <= 32):
 *   idx[k]   device int64[s[k]]: s[k] distinct indices of [0, ncols[k]),
 *            sorted ascending (Floyd's algorithm);
 *   omega[k] device [s[k]][ell[k]] row-major, omega_dtype TK_F32 or TK_F64:
 *            standard normals (Box-Muller, computed in FP64);
 * both from Philox4x64-10 keyed by (seed, k): index step i uses word 0 of the
 * block at counter (i, 0, 0, 0) and takes t = floor(w (j + 1) / 2^64) for
 * j = ncols - s + i (t if not yet chosen, else j); Omega[t][e] uses words 0
 * and 1 of the block at counter (t ell + e, 1, 0, 0) as
 * u1 = ((w0 >> 11) + 1) 2^-53, u2 = (w1 >> 11) 2^-53, sqrt(-2 ln u1) cos(2 pi u2).
 * Asynchronous on `stream`; the caller owns idx and omega.
 * Errors: TK_EINVAL (nunits outside [1, 32], s > ncols, s > 4096, ell < 1,
 * NULL buffers for s > 0, other omega dtypes), TK_EDEVICE. */
tk_status tucker_draw_sketches(int32_t nunits, const int64_t* ncols, const int32_t* s, const int32_t* ell,
                               uint64_t seed, int64_t* const* idx, void* const* omega, int32_t omega_dtype,
                               void* stream);

/* Profiling of the streaming pass.  While enabled, every tucker_core,
 * tucker_reconstruct and htucker_decompose call brackets the kernel that
 * streams X (the one full read of the tensor) with HIP events recorded on the
 * call's stream.  tk_profile_read waits for the recorded events, writes the
 * summed elapsed milliseconds and the number of bracketed launches, and
 * clears the record when reset != 0.  Returns TK_OK or TK_EDEVICE.
 * Not thread-safe: profile from one host thread at a time. */
void tk_profile_enable(int32_t on);
tk_status tk_profile_read(double* ms, int64_t* launches, int32_t reset);

/* Measurement helper, not a step of the method: the read-only streaming
 * reference against which the streaming passes are compared.  Reads
 * floor(bytes / 16) float4s of the device buffer x once (each 16-byte-per-lane
 * load one contiguous 1 KB piece, persistent waves, two workgroups per CU) and
 * writes one checksum per workgroup to partials (device, FP64).  npartials
 * must be at least tk_stream_read_blocks().  Asynchronous on `stream`.
 * Returns TK_EINVAL (null buffer, negative size, partials too small) or
 * TK_EDEVICE. */
int32_t tk_stream_read_blocks(void);
tk_status tk_stream_read(const void* x, int64_t bytes, double* partials, int32_t npartials, void* stream);

/* Message for the calling thread's last non-OK status ("" if none). */
const char* tk_last_error(void);

/* Library version string. */
const char* tk_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TKMI_H */
