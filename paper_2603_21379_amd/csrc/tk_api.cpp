// Host layer of libtkmi: argument validation, workspace planning and the
// orchestration of the kernels behind the C ABI declared in tkmi.h.
//
// Every entry point validates all arguments before touching the device, so
// a failing call has no side effects, and a call with ws == NULL only
// reports the workspace size.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include <stdlib.h>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "tk_kernels.hpp"

namespace tk {

static thread_local std::string g_last_error;

tk_status set_error(tk_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}
void clear_error() { g_last_error.clear(); }

// a roctx range around each C-ABI call, named after the entry point (seen
// by rocprofv3 --marker-trace; free when no tool listens)
struct ApiRange {
  explicit ApiRange(const char* name) { roctxRangePushA(name); }
  ~ApiRange() { roctxRangePop(); }
  ApiRange(const ApiRange&) = delete;
  ApiRange& operator=(const ApiRange&) = delete;
};

// ------------------------------------------------------------------ profiler
static bool g_prof_on = false;
static std::vector<hipEvent_t> g_prof_events;  // start/stop pairs, reused
static size_t g_prof_used = 0;                 // events recorded since the last reset

bool profiling() { return g_prof_on; }

static hipError_t prof_record(hipStream_t st) {
  if (g_prof_used == g_prof_events.size()) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    g_prof_events.push_back(e);
  }
  return hipEventRecord(g_prof_events[g_prof_used++], st);
}
hipError_t profile_begin(hipStream_t st) { return g_prof_on ? prof_record(st) : hipSuccess; }
hipError_t profile_end(hipStream_t st) { return g_prof_on ? prof_record(st) : hipSuccess; }

// Scratch of tucker_sketch_all_modes_noalloc (the per-chunk partial sketches
// of every mode), a fixed device array: each GPU the library runs on holds
// its own copy until the process ends.  In host code the array's name is
// not a device address; its address on the current device comes from
// hipGetSymbolAddress, taken once per device and kept.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

tk_status noalloc_scratch(char** out) {
  static std::mutex mu;
  static char* per_dev[64] = {};
  int dev = 0;
  TK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return set_error(TK_EUNSUPPORTED, "device index %d above 63", dev);
  std::lock_guard<std::mutex> lock(mu);
  if (!per_dev[dev]) {
    void* p = nullptr;
    TK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return set_error(TK_EDEVICE, "hipGetSymbolAddress returned a NULL scratch address");
    per_dev[dev] = static_cast<char*>(p);
  }
  *out = per_dev[dev];
  return TK_OK;
}

namespace {

bool valid_dtype(int dt) { return dt == TK_F64 || dt == TK_F32 || dt == TK_BF16 || dt == TK_F16; }

tk_status check_tensor(const tk_tensor* X, const char* name, int64_t* N) {
  if (!X) return set_error(TK_EINVAL, "%s: tensor descriptor is NULL", name);
  if (X->order < 1 || X->order > TK_MAX_ORDER)
    return set_error(TK_EINVAL, "%s: order %d outside [1, %d]", name, X->order, TK_MAX_ORDER);
  if (!valid_dtype(X->dtype)) return set_error(TK_EINVAL, "%s: unknown dtype %d", name, X->dtype);
  if (!X->data) return set_error(TK_EINVAL, "%s: data pointer is NULL", name);
  int64_t n = 1;
  for (int k = 0; k < X->order; ++k) {
    if (X->dims[k] < 1) return set_error(TK_EINVAL, "%s: dims[%d] = %lld < 1", name, k, (long long)X->dims[k]);
    if (n > INT64_MAX / X->dims[k]) return set_error(TK_EINVAL, "%s: element count overflows", name);
    n *= X->dims[k];
  }
  *N = n;
  return TK_OK;
}

int64_t prod(const int64_t* d, int lo, int hi) {
  int64_t p = 1;
  for (int k = lo; k < hi; ++k) p *= d[k];
  return p;
}

// maxell: kWideMaxEll for the sketches of tucker_sketch_all_modes (their QR
// has a wide path), kMaxEll elsewhere
tk_status check_sketch(const tk_sketch& s, int64_t nrows, int64_t ncols, const char* what, int k,
                       int maxell = kMaxEll) {
  if (s.reserved != 0) return set_error(TK_EINVAL, "%s %d: reserved field must be 0", what, k);
  if (s.ell < 1 || s.ell > maxell)
    return set_error(s.ell > maxell ? TK_EUNSUPPORTED : TK_EINVAL,
                     "%s %d: ell = %d outside [1, %d]", what, k, s.ell, maxell);
  if (s.ell > nrows) return set_error(TK_EINVAL, "%s %d: ell = %d exceeds the %lld rows", what, k, s.ell, (long long)nrows);
  if (s.s < s.ell || s.s > ncols)
    return set_error(TK_EINVAL, "%s %d: s = %lld outside [ell = %d, ncols = %lld]", what, k,
                     (long long)s.s, s.ell, (long long)ncols);
  if (!s.idx && s.s != ncols)
    return set_error(TK_EINVAL, "%s %d: idx is NULL (every column) but s = %lld != %lld", what, k,
                     (long long)s.s, (long long)ncols);
  if (!s.omega) return set_error(TK_EINVAL, "%s %d: omega is NULL", what, k);
  return TK_OK;
}

// Fill one sketch unit and reserve its partial buffer.
void plan_unit(Workspace& ws, SketchUnit& u, const void* X, int64_t A, int64_t n, int64_t B,
               const tk_sketch& s, double* Z, void* Y, int64_t& blocks, int64_t& outs) {
  u = SketchUnit{};
  u.X = X;
  u.A = A;
  u.n = n;
  u.B = B;
  u.s = s.s;
  u.idx = s.idx;
  u.omega = s.omega;
  u.ell = s.ell;
  u.nchunks = (int32_t)ceil_div(s.s, kSketchCols);
  u.rowblocks = (int32_t)ceil_div(n, kSketchRows);
  u.partial = ws.take<double>((size_t)u.nchunks * n * s.ell);
  u.Z = Z;
  u.Y = Y;
  u.block_begin = blocks;
  u.out_begin = outs;
  blocks += (int64_t)u.nchunks * u.rowblocks;
  outs += n * s.ell;
}

// Plan the QR (+ W step) workspace of one matrix.
void plan_qr(Workspace& ws, QRMat& q, double* Z, int64_t m, int ell, bool wstep, const void* Y,
             int64_t s, int r, void* U, int32_t* info) {
  q = QRMat{};
  q.Z = Z;
  q.Y = Y;
  q.U = U;
  q.info = info;
  q.m = m;
  q.s = wstep ? s : 0;
  q.ell = ell;
  q.r = wstep ? r : 0;
  q.nrc = (int32_t)ceil_div(m, kQRRowChunk);
  q.ncc = wstep ? (int32_t)ceil_div(s, kQRColChunk) : 0;
  q.nrb = (int32_t)ceil_div(m, kQRRowBlock);
  // the one-workgroup kernels: QR needs m ell <= kQRSmallElems; the fused U = Q W
  // gives each of 256 / r threads per column at most 64 rows
  q.small = (m <= kQRSmallRows && m * ell <= kQRSmallElems && (!wstep || m <= 64 * (256 / r)))
                ? 1 : 0;
  q.gpart = ws.take<double>((size_t)q.nrc * ell * ell);
  q.R = ws.take<double>((size_t)ell * ell);
  q.state = ws.take<int32_t>(2);
  if (wstep) {
    q.mpart = ws.take<double>((size_t)q.nrc * ell * s);
    q.cpart = ws.take<double>((size_t)q.ncc * ell * ell);
    q.W = ws.take<double>((size_t)ell * r);
    q.utmp = ws.take<double>((size_t)m * r);
    q.amax_v = ws.take<double>((size_t)q.nrb * r);
    q.amax_i = ws.take<int64_t>((size_t)q.nrb * r);
  }
}

// Plan the wide-path QR (+ W step) workspace of one matrix (ell > kMaxEll).
void plan_wide(Workspace& ws, WideQR& q, double* Z, int64_t m, int ell, bool wstep, const void* Y,
               int64_t s, int r, void* U, int32_t* info) {
  q = WideQR{};
  q.Z = Z;
  q.Y = Y;
  q.U = U;
  q.info = info;
  q.m = m;
  q.s = wstep ? s : 0;
  q.ell = ell;
  q.r = wstep ? r : 0;
  q.np = ell + (ell & 1);
  q.gsplit = (int32_t)ceil_div(m, kWideRowChunk);
  q.gpart = ws.take<double>((size_t)q.gsplit * ell * ell);
  q.R = ws.take<double>((size_t)ell * ell);
  q.state = ws.take<int32_t>(3 + kWideMaxSweeps);
  if (wstep) {
    const int64_t np = q.np;
    q.csplit = (int32_t)ceil_div(s, kWideRowChunk);
    q.Mt = ws.take<double>((size_t)s * ell);
    q.cpart = ws.take<double>((size_t)q.csplit * ell * ell);
    q.Ap = ws.take<double>((size_t)(np * (np + 1) / 2));
    q.V = ws.take<double>((size_t)(np * np));
    q.rot = ws.take<double>((size_t)((np - 1) * (np / 2) * 2));
    q.W = ws.take<double>((size_t)ell * r);
  }
}

// A second stream per device (default priority) and its fork / join events,
// created on first use and kept for the process: the wide QR path, mostly
// single-workgroup launches, overlaps the batched narrow matrices on it.
// Callers hold `mu` from the fork record through the join record, so calls
// from several host threads never interleave their uses of the two events.
struct SideStream {
  hipStream_t st = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  std::mutex mu;
};
tk_status side_stream(SideStream** out) {
  static std::mutex mu;
  static SideStream per_dev[64];
  int dev = 0;
  TK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return set_error(TK_EUNSUPPORTED, "device index %d above 63", dev);
  std::lock_guard<std::mutex> lock(mu);
  SideStream& s = per_dev[dev];
  if (!s.st) {
    TK_HIP(hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking));
    TK_HIP(hipEventCreateWithFlags(&s.fork, hipEventDisableTiming));
    TK_HIP(hipEventCreateWithFlags(&s.join, hipEventDisableTiming));
  }
  *out = &s;
  return TK_OK;
}

tk_status run_qr(std::vector<QRMat>& mats, int ydtype, int udtype, bool wstep, hipStream_t st) {
  for (size_t g = 0; g < mats.size(); g += kQRMaxBatch) {
    QRBatch b{};
    b.count = (int32_t)std::min<size_t>(kQRMaxBatch, mats.size() - g);
    int64_t qb = 0;
    for (int i = 0; i < b.count; ++i) {
      b.m[i] = mats[g + i];
      b.m[i].udtype = udtype;
      b.m[i].qty_begin = qb;
      qb += (int64_t)b.m[i].nrc * b.m[i].ncc;
    }
    TK_HIP(launch_cholqr(b, st));
    if (wstep) TK_HIP(launch_wstep(b, ydtype, udtype, st));
  }
  return TK_OK;
}

// The W step alone (CholeskyQR already done); gram: the matrices' cpart
// holds the Gram of Q^T Y (ncc = 1)
tk_status run_wstep(std::vector<QRMat>& mats, int ydtype, int udtype, bool gram, hipStream_t st) {
  for (size_t g = 0; g < mats.size(); g += kQRMaxBatch) {
    QRBatch b{};
    b.count = (int32_t)std::min<size_t>(kQRMaxBatch, mats.size() - g);
    int64_t qb = 0;
    for (int i = 0; i < b.count; ++i) {
      b.m[i] = mats[g + i];
      b.m[i].udtype = udtype;
      b.m[i].qty_begin = qb;
      qb += (int64_t)b.m[i].nrc * b.m[i].ncc;
    }
    if (gram) TK_HIP(launch_wstep_gram(b, udtype, st));
    else TK_HIP(launch_wstep(b, ydtype, udtype, st));
  }
  return TK_OK;
}

tk_status check_factors(int order, const int64_t* dims, const void* const* F, const int32_t* cols,
                        const char* who) {
  if (!F) return set_error(TK_EINVAL, "%s: factor array is NULL", who);
  if (!cols) return set_error(TK_EINVAL, "%s: cols array is NULL", who);
  for (int k = 0; k < order; ++k) {
    if (!F[k]) return set_error(TK_EINVAL, "%s: F[%d] is NULL", who, k);
    if (cols[k] < 1 || cols[k] > dims[k])
      return set_error(TK_EINVAL, "%s: cols[%d] = %d outside [1, n_k = %lld]", who, k, cols[k],
                       (long long)dims[k]);
    if (cols[k] > kMaxCols)
      return set_error(TK_EUNSUPPORTED, "%s: cols[%d] = %d exceeds %d", who, k, cols[k], kMaxCols);
  }
  return TK_OK;
}

// Chain of contractions G = X x_k F_k^T, last mode first.  The streaming
// pass contracts the two (or three) trailing modes in one read of X when a
// fused kernel covers the shape; the rest runs on the partial core.
// Intermediates are FP64, except the FP32 partial cores of the fused passes
// and their MFMA successors.
enum CoreKind { kCoreGeneric = 0, kCoreFused2 = 1, kCoreSlab2 = 2, kCoreSlab3 = 3 };
struct CorePlan {
  double* buf[2] = {nullptr, nullptr};
  float* t32 = nullptr;
  double* mt = nullptr;   // staged factor table of the mode products
  int kind = kCoreGeneric;
  int fused_modes = 0;
  // modes in contraction order (after the fused ones): the generic chain takes
  // the largest reduction n_k / c_k first (ties: the later mode first), so
  // the pass that reads X is the cheapest and every later one reads less
  int order[TK_MAX_ORDER] = {};
  int nsteps = 0;
};

void chain_order(const int64_t* dims, const int32_t* cols, int first, CorePlan& p) {
  bool used[TK_MAX_ORDER] = {};
  p.nsteps = 0;
  for (int step = 0; step <= first; ++step) {
    int best = -1;
    for (int k = first; k >= 0; --k) {
      if (used[k]) continue;
      // n_k / c_k > n_b / c_b, compared exactly in integers
      if (best < 0 || dims[k] * (int64_t)cols[best] > dims[best] * (int64_t)cols[k]) best = k;
    }
    used[best] = true;
    p.order[p.nsteps++] = best;
  }
}

// allow_h3: a third trailing mode may be folded into the pass (the
// gradient path needs the partial core of exactly two trailing modes)
int core_kind(int xdt, int order, const int64_t* dims, const int32_t* cols, bool allow_h3 = true) {
  if (fused2_supported(xdt, order, dims, cols)) return kCoreFused2;
  if (order < 3) return kCoreGeneric;
  const int64_t nI = dims[order - 2], nJ = dims[order - 1];
  if (!slab_supported(xdt, nI, nJ, cols[order - 2], cols[order - 1])) return kCoreGeneric;
  const int64_t A = prod(dims, 0, order - 2);
  if (A >= (int64_t(1) << 31)) return kCoreGeneric;
  // accumulate the third mode in registers when that still leaves work for
  // every wave of the grid (it shrinks the partial core n_H / c_H times)
  if (allow_h3 && order >= 4 && cols[order - 3] <= 16 && dims[order - 3] <= 512 &&
      A / dims[order - 3] >= 2048)
    return kCoreSlab3;
  return kCoreSlab2;
}

tk_status plan_core(Workspace& ws, int xdt, int order, const int64_t* dims, const int32_t* cols,
                    CorePlan& p, bool allow_h3 = true) {
  int64_t shape[TK_MAX_ORDER];
  for (int k = 0; k < order; ++k) shape[k] = dims[k];
  p.kind = core_kind(xdt, order, dims, cols, allow_h3);
  p.fused_modes = p.kind == kCoreGeneric ? 0 : p.kind == kCoreSlab3 ? 3 : 2;
  int64_t mx = 0;
  const int first = p.fused_modes ? order - 1 - p.fused_modes : order - 1;
  if (p.fused_modes) {
    for (int k = order - p.fused_modes; k < order; ++k) shape[k] = cols[k];
    p.t32 = ws.take<float>((size_t)prod(shape, 0, order));
  }
  if (p.kind == kCoreGeneric) {
    chain_order(dims, cols, first, p);
  } else {
    p.nsteps = 0;
    for (int k = first; k >= 0; --k) p.order[p.nsteps++] = k;
  }
  for (int i = 0; i + 1 < p.nsteps; ++i) {
    shape[p.order[i]] = cols[p.order[i]];
    mx = std::max(mx, prod(shape, 0, order));
  }
  p.buf[0] = ws.take<double>((size_t)mx);
  p.buf[1] = ws.take<double>((size_t)mx);
  int64_t smax = 0;
  for (int k = 0; k < order; ++k) smax = std::max(smax, mode_product_scratch(cols[k], dims[k]));
  p.mt = ws.take<double>((size_t)smax);
  return TK_OK;
}

// The streaming pass of the core (the trailing modes fused into one read of
// X, partial core into p.t32); nothing when the plan has no fused pass.
tk_status run_core_pass(const void* X, int xdt, int order, const int64_t* dims,
                        const void* const* F, const int32_t* cols, const CorePlan& p, hipStream_t st) {
  if (p.kind == kCoreFused2) {
    // the two trailing modes in one MFMA pass over X
    CoreFused2 f{};
    f.X = static_cast<const float*>(X);
    f.FI = static_cast<const float*>(F[order - 2]);
    f.FJ = static_cast<const float*>(F[order - 1]);
    f.T = p.t32;
    f.A = prod(dims, 0, order - 2);
    f.nI = (int32_t)dims[order - 2];
    f.nJ = (int32_t)dims[order - 1];
    f.cI = cols[order - 2];
    f.cJ = cols[order - 1];
    const bool x6 = fused2x6_supported(xdt, order, dims, cols);
    TK_HIP(profile_begin(st));
    TK_HIP(x6 ? launch_fused2x6(f, st) : launch_fused2_f32(f, st));
    TK_HIP(profile_end(st));
  } else if (p.kind == kCoreSlab2 || p.kind == kCoreSlab3) {
    // two or three trailing modes in one MFMA pass over X (16x16 tiles)
    const bool h3 = p.kind == kCoreSlab3;
    CoreSlab f{};
    f.X = X;
    f.FH = h3 ? static_cast<const float*>(F[order - 3]) : nullptr;
    f.FI = static_cast<const float*>(F[order - 2]);
    f.FJ = static_cast<const float*>(F[order - 1]);
    f.T = p.t32;
    f.items = prod(dims, 0, order - (h3 ? 3 : 2));
    f.nH = h3 ? (int32_t)dims[order - 3] : 1;
    f.nI = (int32_t)dims[order - 2];
    f.nJ = (int32_t)dims[order - 1];
    f.cH = h3 ? cols[order - 3] : 1;
    f.cI = cols[order - 2];
    f.cJ = cols[order - 1];
    TK_HIP(profile_begin(st));
    TK_HIP(launch_core_slab(f, xdt, st));
    TK_HIP(profile_end(st));
  }
  return TK_OK;
}

// The modes the streaming pass did not contract, from its partial core (or
// from X itself when there is no fused pass), into G.
tk_status run_core_rest(const void* X, int xdt, int order, const int64_t* dims,
                        const void* const* F, const int32_t* cols, void* G, int fdt, const CorePlan& p,
                        hipStream_t st) {
  int64_t shape[TK_MAX_ORDER];
  for (int k = 0; k < order; ++k) shape[k] = dims[k];
  const void* cur = X;
  int cur_dt = xdt;
  if (p.fused_modes) {
    for (int k = order - p.fused_modes; k < order; ++k) shape[k] = cols[k];
    cur = p.t32;
    cur_dt = TK_F32;
  }
  for (int i = 0; i < p.nsteps; ++i) {
    const int k = p.order[i];
    const bool last = i + 1 == p.nsteps;
    // the launch that reads X (no fused pass before it)
    const bool streaming = i == 0 && !p.fused_modes;
    if (cur_dt == TK_F32 && fdt == TK_F32 &&
        mode_mfma_supported(shape[k], prod(shape, k + 1, order), cols[k])) {
      // FP32 partial core: MFMA contraction, FP32 intermediates
      ModeMfma mm{};
      mm.in = static_cast<const float*>(cur);
      mm.F = static_cast<const float*>(F[k]);
      mm.A = prod(shape, 0, k);
      mm.Q = shape[k];
      mm.B = prod(shape, k + 1, order);
      mm.P = cols[k];
      void* out = last ? G : (void*)p.buf[i & 1];
      mm.out = out;
      if (streaming) TK_HIP(profile_begin(st));
      TK_HIP(launch_mode_mfma_f32(mm, TK_F32, st));
      if (streaming) TK_HIP(profile_end(st));
      shape[k] = cols[k];
      cur = out;
      continue;
    }
    if (cur_dt == TK_F32 && fdt == TK_F32 && prod(shape, k + 1, order) == 1 &&
        mode_last_mfma_supported(prod(shape, 0, k), shape[k], cols[k])) {
      // the last mode of an FP32 partial core (or of X): MFMA, FP32 out
      ModeMfma mm{};
      mm.in = static_cast<const float*>(cur);
      mm.F = static_cast<const float*>(F[k]);
      mm.A = prod(shape, 0, k);
      mm.Q = shape[k];
      mm.B = 1;
      mm.P = cols[k];
      void* out = last ? G : (void*)p.buf[i & 1];
      mm.out = out;
      if (streaming) TK_HIP(profile_begin(st));
      TK_HIP(launch_mode_last_mfma_f32(mm, TK_F32, st));
      if (streaming) TK_HIP(profile_end(st));
      shape[k] = cols[k];
      cur = out;
      continue;
    }
    ModeProduct mp{};
    mp.in = cur;
    mp.A = prod(shape, 0, k);
    mp.Q = shape[k];
    mp.B = prod(shape, k + 1, order);
    mp.P = cols[k];
    mp.M = F[k];
    mp.Mt = p.mt;
    mp.rs = 1;          // M[p][q] = F[q][p]
    mp.cs = cols[k];
    void* out = last ? G : (void*)p.buf[i & 1];
    mp.out = out;
    if (streaming) TK_HIP(profile_begin(st));
    TK_HIP(launch_mode_product(mp, cur_dt, last ? fdt : TK_F64, fdt, st));
    if (streaming) TK_HIP(profile_end(st));
    shape[k] = cols[k];
    cur = out;
    cur_dt = TK_F64;
  }
  return TK_OK;
}

tk_status run_core(const void* X, int xdt, int order, const int64_t* dims,
                   const void* const* F, const int32_t* cols, void* G, int fdt, const CorePlan& p,
                   hipStream_t st) {
  if (tk_status s = run_core_pass(X, xdt, order, dims, F, cols, p, st)) return s;
  return run_core_rest(X, xdt, order, dims, F, cols, G, fdt, p, st);
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------------------------ VJP chains
// Buffers shared by the chains of the VJPs: two FP64 ping-pong intermediates
// large enough for every chain, the staged factor table, the partials of
// the unfolded products and of the last expansion.
struct VjpPlan {
  double* buf[2] = {nullptr, nullptr};
  double* mt = nullptr;
  double* upart = nullptr;
  double* epart = nullptr;
};

// Order of the contractions of X in every mode but k: the largest reduction
// n_j / c_j first (ties: the later mode first), as in the core chain.
int contract_order(int d, const int64_t* dims, const int32_t* cols, int k, int* order) {
  bool used[TK_MAX_ORDER] = {};
  int n = 0;
  for (int step = 0; step < d - (k >= 0 ? 1 : 0); ++step) {
    int best = -1;
    for (int j = d - 1; j >= 0; --j) {
      if (j == k || used[j]) continue;
      if (best < 0 || dims[j] * (int64_t)cols[best] > dims[best] * (int64_t)cols[j]) best = j;
    }
    used[best] = true;
    order[n++] = best;
  }
  return n;
}

// contractions: room for the chains that contract X in every mode but k
// (the generic factor gradients); without them only the expansions
void plan_vjp(Workspace& ws, int d, const int64_t* dims, const int32_t* cols, VjpPlan& vp,
              bool contractions = true) {
  int64_t mx = 1;
  int64_t shape[TK_MAX_ORDER];
  // contractions of X in every mode but k
  for (int k = 0; k < d && contractions; ++k) {
    for (int j = 0; j < d; ++j) shape[j] = dims[j];
    int order[TK_MAX_ORDER];
    const int n = contract_order(d, dims, cols, k, order);
    for (int i = 0; i < n; ++i) {
      shape[order[i]] = cols[order[i]];
      mx = std::max(mx, prod(shape, 0, d));
    }
  }
  // expansions of a core in every mode but k, and in every mode but the last
  for (int k = -1; k < d; ++k) {
    for (int j = 0; j < d; ++j) shape[j] = cols[j];
    mx = std::max(mx, prod(shape, 0, d));
    for (int j = 0; j < d; ++j) {
      if (j == k || (k < 0 && j == d - 1)) continue;
      shape[j] = dims[j];
      mx = std::max(mx, prod(shape, 0, d));
    }
  }
  vp.buf[0] = ws.take<double>((size_t)mx);
  vp.buf[1] = ws.take<double>((size_t)mx);
  int64_t smax = 0, umax = 0;
  for (int k = 0; k < d; ++k) {
    smax = std::max(smax, mode_product_scratch(cols[k], dims[k]));
    smax = std::max(smax, mode_product_scratch(dims[k], cols[k]));
    int64_t rest = 1;
    for (int j = 0; j < d; ++j)
      if (j != k) rest *= std::max<int64_t>(dims[j], cols[j]);
    umax = std::max(umax, (int64_t)unfold_gemm_splits(dims[k], cols[k], rest) * dims[k] * cols[k]);
  }
  vp.mt = ws.take<double>((size_t)smax);
  vp.upart = ws.take<double>((size_t)umax);
  vp.epart = ws.take<double>((size_t)2 * expand_residual_blocks(prod(dims, 0, d)));
}

// X x_{j != k} F_j^T: result in FP64 (or X itself when order is 1)
tk_status contract_all_but(const void* X, int xdt, int d, const int64_t* dims, const void* const* F,
                           const int32_t* cols, int k, const VjpPlan& vp, hipStream_t st,
                           const void** out, int* out_dt) {
  int64_t shape[TK_MAX_ORDER];
  for (int j = 0; j < d; ++j) shape[j] = dims[j];
  const void* cur = X;
  int cur_dt = xdt;
  int which = 0;
  int order[TK_MAX_ORDER];
  const int nsteps = contract_order(d, dims, cols, k, order);
  for (int i = 0; i < nsteps; ++i) {
    const int j = order[i];
    ModeProduct mp{};
    mp.in = cur;
    mp.A = prod(shape, 0, j);
    mp.Q = shape[j];
    mp.B = prod(shape, j + 1, d);
    mp.P = cols[j];
    mp.M = F[j];
    mp.Mt = vp.mt;
    mp.rs = 1;
    mp.cs = cols[j];
    mp.out = vp.buf[which];
    TK_HIP(launch_mode_product(mp, cur_dt, TK_F64, factor_dtype(xdt), st));
    shape[j] = cols[j];
    cur = vp.buf[which];
    cur_dt = TK_F64;
    which ^= 1;
  }
  *out = cur;
  *out_dt = cur_dt;
  return TK_OK;
}

// G x_{j != k} F_j: result in FP64 (or G itself when order is 1)
tk_status expand_all_but(const void* G, int fdt, int d, const int64_t* dims, const void* const* F,
                         const int32_t* cols, int k, const VjpPlan& vp, hipStream_t st,
                         const void** out, int* out_dt) {
  int64_t shape[TK_MAX_ORDER];
  for (int j = 0; j < d; ++j) shape[j] = cols[j];
  const void* cur = G;
  int cur_dt = fdt;
  int which = 0;
  for (int j = 0; j < d; ++j) {
    if (j == k) continue;
    ModeProduct mp{};
    mp.in = cur;
    mp.A = prod(shape, 0, j);
    mp.Q = shape[j];
    mp.B = prod(shape, j + 1, d);
    mp.P = (int32_t)dims[j];
    mp.M = F[j];
    mp.Mt = vp.mt;
    mp.rs = cols[j];
    mp.cs = 1;
    mp.out = vp.buf[which];
    TK_HIP(launch_mode_product(mp, cur_dt, TK_F64, fdt, st));
    shape[j] = dims[j];
    cur = vp.buf[which];
    cur_dt = TK_F64;
    which ^= 1;
  }
  *out = cur;
  *out_dt = cur_dt;
  return TK_OK;
}

// out (+)= Gc x_1 F_1 .. x_d F_d (prod(dims) entries, fdt)
tk_status expand_full(const void* Gc, int fdt, int d, const int64_t* dims, const void* const* F,
                      const int32_t* cols, void* out, bool accumulate, const VjpPlan& vp,
                      hipStream_t st) {
  int64_t shape[TK_MAX_ORDER];
  for (int j = 0; j < d; ++j) shape[j] = cols[j];
  const void* cur = Gc;
  int cur_dt = fdt;
  int which = 0;
  for (int j = 0; j < d - 1; ++j) {
    ModeProduct mp{};
    mp.in = cur;
    mp.A = prod(shape, 0, j);
    mp.Q = shape[j];
    mp.B = prod(shape, j + 1, d);
    mp.P = (int32_t)dims[j];
    mp.M = F[j];
    mp.Mt = vp.mt;
    mp.rs = cols[j];
    mp.cs = 1;
    mp.out = vp.buf[which];
    TK_HIP(launch_mode_product(mp, cur_dt, TK_F64, fdt, st));
    shape[j] = dims[j];
    cur = vp.buf[which];
    cur_dt = TK_F64;
    which ^= 1;
  }
  if (cur_dt != TK_F64) {
    TK_HIP(launch_to_f64(cur, cur_dt, vp.buf[which], prod(shape, 0, d), st));
    cur = vp.buf[which];
  }
  ExpandResidual e{};
  e.T = static_cast<const double*>(cur);
  e.F = F[d - 1];
  e.X = nullptr;
  e.Xhat = out;
  e.partials = nullptr;
  e.resid2 = nullptr;
  e.A = prod(dims, 0, d - 1);
  e.n = dims[d - 1];
  e.c = cols[d - 1];
  e.accumulate = accumulate ? 1 : 0;
  TK_HIP(launch_expand_residual(e, fdt, fdt, st));
  return TK_OK;
}

// out[i][a] (+)= sum A[.., i, ..] B[.., a, ..] over all modes but k; A has
// dims[k] at mode k and B cols[k] (a_is_big: A's other modes are cols, else dims)
tk_status unfold_product(const void* A, int adt, const void* B, int bdt, int d, const int64_t* dims,
                         const int32_t* cols, int k, bool a_is_big, void* out, int out_dt,
                         bool accumulate, double* upart, hipStream_t st) {
  int64_t pre = 1, post = 1;
  for (int j = 0; j < d; ++j) {
    if (j == k) continue;
    const int64_t e = a_is_big ? cols[j] : dims[j];
    (j < k ? pre : post) *= e;
  }
  UnfoldGemm g{};
  g.A = A;
  g.B = B;
  g.out = out;
  g.partials = upart;
  g.pre = pre;
  g.post = post;
  g.n = (int32_t)dims[k];
  g.c = cols[k];
  g.splits = unfold_gemm_splits(dims[k], cols[k], pre * post);
  g.accumulate = accumulate ? 1 : 0;
  TK_HIP(launch_unfold_gemm(g, adt, bdt, out_dt, st));
  return TK_OK;
}


// ------------------------------------------------------------------ fused factor gradients
// FP32 tensors whose two trailing modes take a fused streaming pass: for
//   Fbar_k (+)= (Y x_{j != k} F_j^T)^(k) (C^(k))^T   (every mode k)
// the streaming pass of the core gives T = Y x_I F_I^T x_J F_J^T (the two
// trailing modes), from which the leading modes' gradients are small
// contractions; the trailing modes' gradients come from one more pass over Y
// (k_vjp_trail.hip) with K = C x_{j < d-2} F_j.  Y is read twice in all.
struct GradPlan {
  CorePlan cp;              // streaming pass of Y (cp.t32 = T) and its chain to a core
  double* buf[2] = {nullptr, nullptr};   // FP64 chain intermediates
  double* mt = nullptr;     // mode-product scratch
  double* upart = nullptr;  // unfolded-product partials
  float* K32 = nullptr;     // A x c_I x c_J
  float* partI = nullptr;
  float* partJ = nullptr;
  int nblocks = 0;
};

bool grads_fused_ok(int ydt, int d, const int64_t* dims, const int32_t* cols) {
  if (ydt != TK_F32 || d < 3) return false;
  const int kind = core_kind(ydt, d, dims, cols, false);
  if (kind != kCoreFused2 && kind != kCoreSlab2) return false;
  return vjp_trail_supported(dims[d - 2], dims[d - 1], cols[d - 2], cols[d - 1], prod(dims, 0, d - 2));
}

void plan_grads(Workspace& ws, int d, const int64_t* dims, const int32_t* cols, GradPlan& g) {
  plan_core(ws, TK_F32, d, dims, cols, g.cp, false);
  const int64_t A = prod(dims, 0, d - 2);
  const int64_t tsz = A * cols[d - 2] * cols[d - 1];   // |T| = |K|: every chain stays within it
  g.buf[0] = ws.take<double>((size_t)tsz);
  g.buf[1] = ws.take<double>((size_t)tsz);
  int64_t smax = 0, umax = 0, crest = 1;
  for (int k = 0; k < d; ++k) crest *= cols[k];
  for (int k = 0; k < d; ++k) {
    smax = std::max(smax, mode_product_scratch(cols[k], dims[k]));
    smax = std::max(smax, mode_product_scratch(dims[k], cols[k]));
    if (k < d - 2)
      umax = std::max(umax, (int64_t)unfold_gemm_splits(dims[k], cols[k], crest / cols[k]) * dims[k] *
                                cols[k]);
  }
  g.mt = ws.take<double>((size_t)smax);
  g.upart = ws.take<double>((size_t)std::max<int64_t>(umax, 1));
  g.K32 = ws.take<float>((size_t)tsz);
  g.nblocks = vjp_trail_blocks(A);
  g.partI = ws.take<float>((size_t)(g.nblocks * vjp_trail_rows_i(dims[d - 2]) * 32));
  g.partJ = ws.take<float>((size_t)(g.nblocks * vjp_trail_rows_j(dims[d - 1]) * 32));
}

// after run_core_pass(Y) has written T = g.cp.t32
tk_status run_grads(const void* Y, int d, const int64_t* dims, const void* const* F, const int32_t* cols,
                    const void* C, int cdt, void* const* Fbar, int fdt, bool accumulate, const GradPlan& g,
                    hipStream_t st) {
  const int I = d - 2, J = d - 1;
  int64_t shape[TK_MAX_ORDER];
  // K = C x_{j < d-2} F_j: FP64 intermediates, the last expansion into FP32
  if (Fbar[I] || Fbar[J]) {
    for (int j = 0; j < d; ++j) shape[j] = cols[j];
    const void* cur = C;
    int cur_dt = cdt;
    for (int j = 0; j < I; ++j) {
      const bool last = j == I - 1;
      ModeProduct mp{};
      mp.in = cur;
      mp.A = prod(shape, 0, j);
      mp.Q = shape[j];
      mp.B = prod(shape, j + 1, d);
      mp.P = (int32_t)dims[j];
      mp.M = F[j];
      mp.Mt = g.mt;
      mp.rs = cols[j];   // M[p][q] = F[p][q]
      mp.cs = 1;
      mp.out = last ? (void*)g.K32 : (void*)g.buf[j & 1];
      TK_HIP(launch_mode_product(mp, cur_dt, last ? TK_F32 : TK_F64, TK_F32, st));
      shape[j] = dims[j];
      cur = mp.out;
      cur_dt = last ? TK_F32 : TK_F64;
    }
    VjpTrail v{};
    v.X = static_cast<const float*>(Y);
    v.K = g.K32;
    v.FI = static_cast<const float*>(F[I]);
    v.FJ = static_cast<const float*>(F[J]);
    v.partI = g.partI;
    v.partJ = g.partJ;
    v.A = prod(dims, 0, I);
    v.nI = (int32_t)dims[I];
    v.nJ = (int32_t)dims[J];
    v.cI = cols[I];
    v.cJ = cols[J];
    v.nblocks = g.nblocks;
    TK_HIP(launch_vjp_trail(v, Fbar[I], Fbar[J], fdt, accumulate ? 1 : 0, st));
  }
  // leading modes: P_k = T x_{j < d-2, j != k} F_j^T (the largest reduction
  // first), then Fbar_k (+)= P_k^(k) (C^(k))^T
  for (int k = 0; k < I; ++k) {
    if (!Fbar[k]) continue;
    for (int j = 0; j < d; ++j) shape[j] = j < I ? dims[j] : cols[j];
    const void* cur = g.cp.t32;
    int cur_dt = TK_F32;
    bool used[TK_MAX_ORDER] = {};
    used[k] = true;
    int which = 0;
    for (int step = 0; step + 1 < I; ++step) {
      int best = -1;
      for (int j = I - 1; j >= 0; --j) {
        if (used[j]) continue;
        if (best < 0 || dims[j] * (int64_t)cols[best] > dims[best] * (int64_t)cols[j]) best = j;
      }
      used[best] = true;
      ModeProduct mp{};
      mp.in = cur;
      mp.A = prod(shape, 0, best);
      mp.Q = shape[best];
      mp.B = prod(shape, best + 1, d);
      mp.P = cols[best];
      mp.M = F[best];
      mp.Mt = g.mt;
      mp.rs = 1;   // M[p][q] = F[q][p]
      mp.cs = cols[best];
      mp.out = g.buf[which];
      TK_HIP(launch_mode_product(mp, cur_dt, TK_F64, TK_F32, st));
      shape[best] = cols[best];
      cur = g.buf[which];
      cur_dt = TK_F64;
      which ^= 1;
    }
    if (tk_status s = unfold_product(cur, cur_dt, C, cdt, d, dims, cols, k, true, Fbar[k], fdt,
                                     accumulate, g.upart, st)) return s;
  }
  return TK_OK;
}

// ------------------------------------------------------------------ batching form
// All tensors and modes of a batch: the descriptor tables are built once on
// the host and kept in the workspace; a run is a fixed launch sequence
// (sketch, QR, W step, streaming core, remaining modes) with no allocation,
// no host synchronisation and no memset, so it can be captured in a graph.
constexpr int kBatchWaveCap = 16384;              // schedule capacity (waves)
constexpr int64_t kBatchChunkMin = 32 << 10;     // smallest chunk the tuner tries (bytes)
constexpr int64_t kBatchResidChunk = 512 << 10;  // residual pass chunk (bytes)
constexpr int64_t kBatchChunkMax = 64 << 20;     // largest chunk a stored schedule may ask for

struct BatchPlanData {
  int count = 0;
  std::vector<SketchUnit> units;
  std::vector<QRMat> qr;
  std::vector<BatchTensor> tensors;
  std::vector<std::vector<BatchModeDesc>> steps;
  std::vector<int64_t> step_units, step_qmax;
  SketchUnit* d_units = nullptr;
  int32_t* d_block_unit = nullptr;
  std::vector<int32_t> block_unit;
  QRMat* d_qr = nullptr;
  BatchTensor* d_tensors = nullptr;
  BatchChunk* d_chunks = nullptr;
  int32_t* d_order = nullptr;
  int32_t* d_queue = nullptr;
  size_t chunk_cap = 0;
  std::vector<BatchModeDesc*> d_steps;
  SketchList sl{};
  BatchSlab bs{};
  int tg = 0, nbuf = 0;               // whole-slab pipeline form until tuned
  int64_t chunk_bytes = 128 << 10;
  // residual (when requested): expansion of each core over its leading
  // modes into the tensor's T, then the residual pass over its own schedule
  double* resid2 = nullptr;
  std::vector<std::vector<BatchModeDesc>> esteps;
  std::vector<int64_t> estep_units, estep_qmax;
  std::vector<BatchModeDesc*> d_esteps;
  std::vector<BatchChunk> rchunks;
  std::vector<int32_t> rorder, rtcb;
  BatchChunk* d_rchunks = nullptr;
  int32_t* d_rorder = nullptr;
  int32_t* d_rtcb = nullptr;
  int32_t* d_rqueue = nullptr;
  double* d_rpart = nullptr;
  BatchResid br{};
};

int64_t batch_chunk_slabs(const BatchTensor& t, int64_t chunk_bytes) {
  const int64_t sb = (int64_t)t.nI * t.nJ * 4;
  return std::max<int64_t>(1, chunk_bytes / sb);
}

// Chunks of consecutive slabs of every tensor, in tensor order, and the
// order in which the waves take them from the queue: largest first (cost =
// slab tiles, plus a start-up term per chunk), so the last chunks taken are
// the short ones and the waves finish together.
void batch_chunks(const std::vector<BatchTensor>& ts, int64_t chunk_bytes, std::vector<BatchChunk>& chunks,
                  std::vector<int32_t>& order) {
  chunks.clear();
  std::vector<int64_t> cost;
  for (int t = 0; t < (int)ts.size(); ++t) {
    const int64_t S = batch_chunk_slabs(ts[t], chunk_bytes);
    const int64_t tile_work = ceil_div(ts[t].nI, 16) * ceil_div(ts[t].nJ, 16);
    for (int64_t a0 = 0; a0 < ts[t].A; a0 += S) {
      BatchChunk c{};
      c.tensor = t;
      c.a0 = a0;
      c.a1 = std::min(ts[t].A, a0 + S);
      chunks.push_back(c);
      cost.push_back((c.a1 - c.a0) * tile_work + 4);
    }
  }
  order.resize(chunks.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
}

tk_status plan_batch(Workspace& ws, int count, const tk_tensor* X, const int32_t* ranks,
                     const tk_sketch* sk, void* const* U, void* const* G, int32_t* info, double* resid2,
                     BatchPlanData& P) {
  if (count < 1) return set_error(TK_EINVAL, "tucker_batch_plan_create: count = %d < 1", count);
  if (!X || !ranks || !sk || !U || !G)
    return set_error(TK_EINVAL, "tucker_batch_plan_create: a descriptor array is NULL");
  P = BatchPlanData{};
  P.count = count;
  int m0 = 0, max_order = 0;
  int64_t blocks = 0, outs = 0;
  for (int t = 0; t < count; ++t) {
    int64_t N;
    if (tk_status s = check_tensor(&X[t], "tucker_batch_plan_create", &N)) return s;
    const tk_tensor& x = X[t];
    const int d = x.order;
    if (x.dtype != TK_F32)
      return set_error(TK_EUNSUPPORTED, "tucker_batch_plan_create: tensor %d: the batch form takes FP32 tensors", t);
    if (d < 3) return set_error(TK_EUNSUPPORTED, "tucker_batch_plan_create: tensor %d: order %d < 3", t, d);
    if (x.dims[d - 2] > kBatchMaxN || x.dims[d - 1] > kBatchMaxN)
      return set_error(TK_EUNSUPPORTED, "tucker_batch_plan_create: tensor %d: trailing modes exceed %d", t, kBatchMaxN);
    if (N * 4 >= (int64_t(1) << 31))
      return set_error(TK_EUNSUPPORTED, "tucker_batch_plan_create: tensor %d: more than 2^29 entries", t);
    if (!G[t]) return set_error(TK_EINVAL, "tucker_batch_plan_create: G[%d] is NULL", t);
    for (int k = 0; k < d; ++k) {
      const int r = ranks[m0 + k];
      const tk_sketch& s = sk[m0 + k];
      const int64_t ncols = N / x.dims[k];
      if (tk_status e = check_sketch(s, x.dims[k], ncols, "tucker_batch_plan_create: sketch", m0 + k)) return e;
      if (r < 1 || r > s.ell)
        return set_error(TK_EINVAL, "tucker_batch_plan_create: rank %d of mode %d outside [1, ell = %d]", r, m0 + k, s.ell);
      const int rmax = k >= d - 2 ? kBatchMaxC : 32;
      if (r > rmax)
        return set_error(TK_EUNSUPPORTED, "tucker_batch_plan_create: rank %d of mode %d exceeds %d", r, m0 + k, rmax);
      if (!U[m0 + k]) return set_error(TK_EINVAL, "tucker_batch_plan_create: U[%d] is NULL", m0 + k);
    }
    m0 += d;
    max_order = std::max(max_order, d);
  }
  // sketches and their QR / W step
  m0 = 0;
  for (int t = 0; t < count; ++t) {
    const tk_tensor& x = X[t];
    const int d = x.order;
    for (int k = 0; k < d; ++k) {
      const tk_sketch& s = sk[m0 + k];
      const int64_t n = x.dims[k];
      double* Z = ws.take<double>((size_t)n * s.ell);
      float* Y = ws.take<float>((size_t)n * s.s);
      SketchUnit u;
      plan_unit(ws, u, x.data, prod(x.dims, 0, k), n, prod(x.dims, k + 1, d), s, Z, Y, blocks, outs);
      P.units.push_back(u);
      QRMat q;
      plan_qr(ws, q, Z, n, s.ell, true, Y, s.s, ranks[m0 + k], U[m0 + k], info ? info + m0 + k : nullptr);
      q.udtype = TK_F32;
      P.qr.push_back(q);
    }
    m0 += d;
  }
  // core: streaming pass per tensor, then the remaining modes step by step
  P.steps.assign(max_order - 2, {});
  P.resid2 = resid2;
  if (resid2) P.esteps.assign(max_order - 2, {});
  m0 = 0;
  for (int t = 0; t < count; ++t) {
    const tk_tensor& x = X[t];
    const int d = x.order;
    const int32_t* c = ranks + m0;
    BatchTensor bt{};
    bt.X = static_cast<const float*>(x.data);
    bt.FI = static_cast<const float*>(U[m0 + d - 2]);
    bt.FJ = static_cast<const float*>(U[m0 + d - 1]);
    bt.A = prod(x.dims, 0, d - 2);
    bt.nI = (int32_t)x.dims[d - 2];
    bt.nJ = (int32_t)x.dims[d - 1];
    bt.cI = c[d - 2];
    bt.cJ = c[d - 1];
    bt.T = ws.take<float>((size_t)bt.A * bt.cI * bt.cJ);
    int64_t shape[TK_MAX_ORDER];
    for (int k = 0; k < d; ++k) shape[k] = x.dims[k];
    shape[d - 2] = c[d - 2];
    shape[d - 1] = c[d - 1];
    // The leading modes are contracted first mode first (and expanded back
    // last mode first), so the steps that read or write the partial core T,
    // the largest, run with B = everything after mode 0: whole 128-column
    // blocks, where B = c_I c_J alone (often below 128) would leave lanes idle.
    int64_t mx = 1;
    {
      int64_t sh[TK_MAX_ORDER];
      for (int k = 0; k < d; ++k) sh[k] = shape[k];
      for (int k = 0; k < d - 3; ++k) {
        sh[k] = c[k];
        mx = std::max(mx, prod(sh, 0, d));
      }
    }
    float* buf[2] = {ws.take<float>((size_t)mx), ws.take<float>((size_t)mx)};
    const float* cur = bt.T;
    for (int k = 0; k < d - 2; ++k) {
      BatchModeDesc md{};
      md.in = cur;
      md.F = static_cast<const float*>(U[m0 + k]);
      md.A = prod(shape, 0, k);
      md.Q = shape[k];
      md.B = prod(shape, k + 1, d);
      md.P = c[k];
      md.out_slab = (int64_t)md.P * md.B;
      md.out = k == d - 3 ? static_cast<float*>(G[t]) : buf[k & 1];
      P.steps[k].push_back(md);
      shape[k] = c[k];
      cur = md.out;
    }
    if (resid2) {
      // T = G x_{d-3} U_{d-3} .. x_0 U_0: the projection's intermediate shapes
      // in reverse, so its two buffers serve
      for (int k = 0; k < d; ++k) shape[k] = c[k];
      const float* ecur = static_cast<const float*>(G[t]);
      for (int e = 0; e < d - 2; ++e) {
        const int k = d - 3 - e;
        const int64_t n = x.dims[k];
        float* out = k == 0 ? bt.T : buf[e & 1];
        const int64_t Bk = prod(shape, k + 1, d);
        for (int64_t p0 = 0; p0 < n; p0 += 32) {
          BatchModeDesc md{};
          md.in = ecur;
          md.F = static_cast<const float*>(U[m0 + k]) + p0 * c[k];
          md.out = out + p0 * Bk;
          md.A = prod(shape, 0, k);
          md.Q = c[k];
          md.B = Bk;
          md.P = (int32_t)std::min<int64_t>(32, n - p0);
          md.out_slab = n * Bk;
          md.ftrans = 1;
          P.esteps[e].push_back(md);
        }
        shape[k] = n;
        ecur = out;
      }
    }
    P.tensors.push_back(bt);
    m0 += d;
  }
  {
    int64_t qb = 0;
    for (auto& q : P.qr) {
      q.qty_begin = qb;
      qb += (int64_t)q.nrc * q.ncc;
    }
  }
  auto number_units = [](std::vector<std::vector<BatchModeDesc>>& steps, std::vector<int64_t>& units,
                         std::vector<int64_t>& qmax) {
    units.assign(steps.size(), 0);
    qmax.assign(steps.size(), 1);
    for (size_t s = 0; s < steps.size(); ++s)
      for (auto& md : steps[s]) {
        md.unit_begin = units[s];
        units[s] += batch_mode_units(md.A, md.B);
        qmax[s] = std::max(qmax[s], md.Q);
      }
  };
  number_units(P.steps, P.step_units, P.step_qmax);
  number_units(P.esteps, P.estep_units, P.estep_qmax);
  // device tables
  P.chunk_cap = 0;
  for (auto& bt : P.tensors) P.chunk_cap += (size_t)ceil_div(bt.A, batch_chunk_slabs(bt, kBatchChunkMin));
  P.d_units = ws.take<SketchUnit>(P.units.size());
  P.d_block_unit = ws.take<int32_t>((size_t)std::max<int64_t>(blocks, 1));
  P.d_qr = ws.take<QRMat>(P.qr.size());
  P.d_tensors = ws.take<BatchTensor>(P.tensors.size());
  P.d_chunks = ws.take<BatchChunk>(P.chunk_cap);
  P.d_order = ws.take<int32_t>(P.chunk_cap);
  P.d_queue = ws.take<int32_t>(1);
  for (auto& st : P.steps) P.d_steps.push_back(ws.take<BatchModeDesc>(st.size()));
  if (resid2) {
    for (auto& st : P.esteps) P.d_esteps.push_back(ws.take<BatchModeDesc>(st.size()));
    // chunks of 512 KB, handed out largest first from a queue to the
    // residual kernel's resident waves
    batch_chunks(P.tensors, kBatchResidChunk, P.rchunks, P.rorder);
    const int nrc = (int)P.rchunks.size();
    P.rtcb.assign(count + 1, nrc);
    for (int i = nrc - 1; i >= 0; --i) P.rtcb[P.rchunks[i].tensor] = i;
    for (int t = count - 1; t >= 0; --t) P.rtcb[t] = std::min(P.rtcb[t], P.rtcb[t + 1]);
    P.d_rchunks = ws.take<BatchChunk>(nrc);
    P.d_rorder = ws.take<int32_t>(nrc);
    P.d_rtcb = ws.take<int32_t>(P.rtcb.size());
    P.d_rqueue = ws.take<int32_t>(1);
    P.d_rpart = ws.take<double>(2 * (size_t)nrc);
    P.br.tensors = P.d_tensors;
    P.br.chunks = P.d_rchunks;
    P.br.order = P.d_rorder;
    P.br.tensor_chunk_begin = P.d_rtcb;
    P.br.partials = P.d_rpart;
    P.br.resid2 = resid2;
    P.br.queue = P.d_rqueue;
    P.br.nwaves = ws.base ? std::min(kBatchWaveCap, batch_resid_waves()) : 0;
    P.br.nchunks = nrc;
    P.br.count = count;
  }
  P.sl.u = P.d_units;
  P.sl.block_unit = P.d_block_unit;
  P.sl.count = (int32_t)P.units.size();
  P.sl.total_blocks = blocks;
  P.sl.total_out = outs;
  return TK_OK;
}

// chunk list of the streaming pass for a variant and chunk size (synchronous upload)
tk_status batch_set_schedule(BatchPlanData& P, int tg, int nbuf, int64_t chunk_bytes, hipStream_t st) {
  std::vector<BatchChunk> chunks;
  std::vector<int32_t> order;
  batch_chunks(P.tensors, std::max(chunk_bytes, kBatchChunkMin), chunks, order);
  if (chunks.size() > P.chunk_cap) return set_error(TK_EINVAL, "batch schedule exceeds its table");
  TK_HIP(hipMemcpyAsync(P.d_chunks, chunks.data(), chunks.size() * sizeof(BatchChunk), hipMemcpyHostToDevice, st));
  TK_HIP(hipMemcpyAsync(P.d_order, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
  TK_HIP(hipStreamSynchronize(st));
  P.tg = tg;
  P.nbuf = nbuf;
  P.chunk_bytes = chunk_bytes;
  P.bs.tensors = P.d_tensors;
  P.bs.chunks = P.d_chunks;
  P.bs.order = P.d_order;
  P.bs.queue = P.d_queue;
  P.bs.nchunks = (int32_t)chunks.size();
  P.bs.nwaves = std::min(kBatchWaveCap, batch_slab_waves(tg, nbuf));
  return TK_OK;
}

tk_status batch_upload(BatchPlanData& P, hipStream_t st) {
  TK_HIP(hipMemcpyAsync(P.d_units, P.units.data(), P.units.size() * sizeof(SketchUnit), hipMemcpyHostToDevice, st));
  P.block_unit.assign((size_t)P.sl.total_blocks, 0);
  for (size_t i = 0; i < P.units.size(); ++i) {
    const int64_t end = i + 1 < P.units.size() ? P.units[i + 1].block_begin : P.sl.total_blocks;
    for (int64_t bk = P.units[i].block_begin; bk < end; ++bk) P.block_unit[bk] = (int32_t)i;
  }
  if (!P.block_unit.empty())
    TK_HIP(hipMemcpyAsync(P.d_block_unit, P.block_unit.data(), P.block_unit.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, st));
  TK_HIP(hipMemcpyAsync(P.d_qr, P.qr.data(), P.qr.size() * sizeof(QRMat), hipMemcpyHostToDevice, st));
  TK_HIP(hipMemcpyAsync(P.d_tensors, P.tensors.data(), P.tensors.size() * sizeof(BatchTensor), hipMemcpyHostToDevice, st));
  for (size_t s = 0; s < P.steps.size(); ++s)
    TK_HIP(hipMemcpyAsync(P.d_steps[s], P.steps[s].data(), P.steps[s].size() * sizeof(BatchModeDesc),
                          hipMemcpyHostToDevice, st));
  if (P.resid2) {
    for (size_t s = 0; s < P.esteps.size(); ++s)
      TK_HIP(hipMemcpyAsync(P.d_esteps[s], P.esteps[s].data(), P.esteps[s].size() * sizeof(BatchModeDesc),
                            hipMemcpyHostToDevice, st));
    TK_HIP(hipMemcpyAsync(P.d_rchunks, P.rchunks.data(), P.rchunks.size() * sizeof(BatchChunk),
                          hipMemcpyHostToDevice, st));
    TK_HIP(hipMemcpyAsync(P.d_rorder, P.rorder.data(), P.rorder.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                          st));
    TK_HIP(hipMemcpyAsync(P.d_rtcb, P.rtcb.data(), P.rtcb.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
  }
  return batch_set_schedule(P, P.tg, P.nbuf, P.chunk_bytes, st);
}

tk_status batch_core(const BatchPlanData& P, hipStream_t st) {
  TK_HIP(profile_begin(st));
  TK_HIP(launch_batch_slab(P.bs, P.tg, P.nbuf, st));
  TK_HIP(profile_end(st));
  for (size_t s = 0; s < P.steps.size(); ++s) {
    BatchMode bm{};
    bm.descs = P.d_steps[s];
    bm.count = (int32_t)P.steps[s].size();
    TK_HIP(launch_batch_mode(bm, P.step_units[s], P.step_qmax[s], st));
  }
  return TK_OK;
}

tk_status batch_run(const BatchPlanData& P, hipStream_t st) {
  TK_HIP(launch_sketch_list(TK_F32, P.sl, st));
  QRList ql{};
  ql.m = P.d_qr;
  ql.count = (int32_t)P.qr.size();
  TK_HIP(launch_cholqr_list(ql, P.qr.data(), st));
  TK_HIP(launch_wstep_list(ql, P.qr.data(), TK_F32, TK_F32, st));
  if (tk_status s = batch_core(P, st)) return s;
  if (!P.resid2) return TK_OK;
  for (size_t s = 0; s < P.esteps.size(); ++s) {
    BatchMode bm{};
    bm.descs = P.d_esteps[s];
    bm.count = (int32_t)P.esteps[s].size();
    TK_HIP(launch_batch_mode(bm, P.estep_units[s], P.estep_qmax[s], st));
  }
  TK_HIP(launch_batch_resid(P.br, st));
  return TK_OK;
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" {

const char* tk_last_error(void) { return g_last_error.c_str(); }

void tk_profile_enable(int32_t on) { g_prof_on = on != 0; }

tk_status tk_profile_read(double* ms, int64_t* launches, int32_t reset) {
  clear_error();
  const ApiRange range_("tk_profile_read");
  double total = 0.0;
  const size_t pairs = g_prof_used / 2;
  for (size_t i = 0; i < pairs; ++i) {
    TK_HIP(hipEventSynchronize(g_prof_events[2 * i + 1]));
    float t = 0.0f;
    TK_HIP(hipEventElapsedTime(&t, g_prof_events[2 * i], g_prof_events[2 * i + 1]));
    total += t;
  }
  if (ms) *ms = total;
  if (launches) *launches = (int64_t)pairs;
  if (reset) g_prof_used = 0;
  return TK_OK;
}
const char* tk_version(void) { return "tkmi 0.1 (gfx950)"; }

tk_status tucker_draw_sketches(int32_t nunits, const int64_t* ncols, const int32_t* s, const int32_t* ell,
                               uint64_t seed, int64_t* const* idx, void* const* omega, int32_t omega_dtype,
                               void* stream) {
  clear_error();
  const ApiRange range_("tucker_draw_sketches");
  if (nunits < 1 || nunits > kMaxUnits)
    return set_error(TK_EINVAL, "tucker_draw_sketches: nunits %d outside [1, %d]", nunits, kMaxUnits);
  if (!ncols || !s || !ell || !idx || !omega)
    return set_error(TK_EINVAL, "tucker_draw_sketches: NULL array argument");
  if (omega_dtype != TK_F32 && omega_dtype != TK_F64)
    return set_error(TK_EINVAL, "tucker_draw_sketches: omega_dtype must be TK_F32 or TK_F64");
  DrawBatch b{};
  b.count = nunits;
  b.seed = seed;
  b.omega_dtype = omega_dtype;
  int smax = 1;
  for (int k = 0; k < nunits; ++k) {
    if (ncols[k] < 1 || s[k] < 0 || s[k] > ncols[k] || s[k] > kDrawMaxS || ell[k] < 1)
      return set_error(TK_EINVAL, "tucker_draw_sketches: unit %d: need 0 <= s <= min(ncols, %d), ell >= 1 "
                       "(ncols %lld, s %d, ell %d)", k, kDrawMaxS, (long long)ncols[k], s[k], ell[k]);
    if (s[k] > 0 && (!idx[k] || !omega[k]))
      return set_error(TK_EINVAL, "tucker_draw_sketches: unit %d: idx or omega is NULL", k);
    b.u[k] = DrawUnit{ncols[k], idx[k], omega[k], s[k], ell[k]};
    b.omega_begin[k + 1] = b.omega_begin[k] + (int64_t)s[k] * ell[k];
    smax = std::max(smax, (int)s[k]);
  }
  TK_HIP(launch_draw(b, smax, as_stream(stream)));
  return TK_OK;
}

int32_t tk_stream_read_blocks(void) { return (int32_t)stream_read_blocks(); }

tk_status tk_stream_read(const void* x, int64_t bytes, double* partials, int32_t npartials, void* stream) {
  clear_error();
  const ApiRange range_("tk_stream_read");
  if (!x || !partials || bytes < 0) return set_error(TK_EINVAL, "tk_stream_read: null buffer or negative size");
  const int32_t blocks = (int32_t)stream_read_blocks();
  if (npartials < blocks)
    return set_error(TK_EINVAL, "tk_stream_read: partials holds %d values, needs %d", npartials, blocks);
  TK_HIP(launch_stream_read(x, bytes, partials, blocks, as_stream(stream)));
  return TK_OK;
}

tk_status tucker_sketch_all_modes(const tk_tensor* X, const tk_sketch* sk, double* const* Z,
                                  void* const* Y, void* ws, size_t* ws_bytes, void* stream) {
  clear_error();
  const ApiRange range_("tucker_sketch_all_modes");
  int64_t N;
  if (tk_status s = check_tensor(X, "tucker_sketch_all_modes", &N)) return s;
  if (!sk || !Z) return set_error(TK_EINVAL, "tucker_sketch_all_modes: sk or Z is NULL");
  if (!ws_bytes) return set_error(TK_EINVAL, "tucker_sketch_all_modes: ws_bytes is NULL");
  const int d = X->order;
  for (int k = 0; k < d; ++k) {
    if (tk_status s = check_sketch(sk[k], X->dims[k], N / X->dims[k], "mode", k, kWideMaxEll)) return s;
    if (!Z[k]) return set_error(TK_EINVAL, "tucker_sketch_all_modes: Z[%d] is NULL", k);
  }
  Workspace w;
  w.base = static_cast<char*>(ws);
  SketchBatch b{};
  b.count = d;
  for (int k = 0; k < d; ++k)
    plan_unit(w, b.u[k], X->data, prod(X->dims, 0, k), X->dims[k], prod(X->dims, k + 1, d), sk[k],
              Z[k], Y ? Y[k] : nullptr, b.total_blocks, b.total_out);
  if (!ws) {
    *ws_bytes = w.off;
    return TK_OK;
  }
  if (*ws_bytes < w.off)
    return set_error(TK_EWORKSPACE, "tucker_sketch_all_modes: workspace %zu < required %zu",
                     *ws_bytes, w.off);
  TK_HIP(launch_sketch(X->dtype, b, as_stream(stream)));
  return TK_OK;
}

tk_status tucker_sketch_all_modes_noalloc(const tk_tensor* X, const tk_sketch* sk, double* const* Z,
                                          void* const* Y, void* stream) {
  const ApiRange range_("tucker_sketch_all_modes_noalloc");
  // the same validation, plan and kernels as tucker_sketch_all_modes, with
  // the fixed scratch array as the workspace: nothing is allocated
  size_t need = 0;
  if (tk_status s = tucker_sketch_all_modes(X, sk, Z, Y, nullptr, &need, stream)) return s;
  if (need > kNoAllocScratchBytes)
    return set_error(TK_EUNSUPPORTED,
                     "tucker_sketch_all_modes_noalloc: the call needs %zu bytes of scratch, above the "
                     "fixed %zu (use tucker_sketch_all_modes with a workspace)",
                     need, kNoAllocScratchBytes);
  char* base = nullptr;
  if (tk_status s = noalloc_scratch(&base)) return s;
  size_t have = kNoAllocScratchBytes;
  return tucker_sketch_all_modes(X, sk, Z, Y, base, &have, stream);
}

tk_status tucker_qr(int32_t nmat, const int64_t* m, const int32_t* ell, double* const* Z,
                    const void* const* Y, int32_t ydtype, const int64_t* s, const int32_t* r,
                    void* const* U, int32_t udtype, int32_t* info, void* ws, size_t* ws_bytes,
                    void* stream) {
  clear_error();
  const ApiRange range_("tucker_qr");
  if (nmat < 0) return set_error(TK_EINVAL, "tucker_qr: nmat < 0");
  if (!ws_bytes) return set_error(TK_EINVAL, "tucker_qr: ws_bytes is NULL");
  if (nmat > 0 && (!m || !ell || !Z)) return set_error(TK_EINVAL, "tucker_qr: m, ell or Z is NULL");
  if (Y) {
    if (!valid_dtype(ydtype)) return set_error(TK_EINVAL, "tucker_qr: unknown ydtype %d", ydtype);
    if (udtype != TK_F64 && udtype != TK_F32)
      return set_error(TK_EINVAL, "tucker_qr: udtype must be TK_F64 or TK_F32");
    if (nmat > 0 && (!s || !r || !U)) return set_error(TK_EINVAL, "tucker_qr: s, r or U is NULL");
  }
  for (int i = 0; i < nmat; ++i) {
    if (m[i] < 1) return set_error(TK_EINVAL, "tucker_qr: m[%d] < 1", i);
    if (ell[i] < 1 || ell[i] > m[i])
      return set_error(TK_EINVAL, "tucker_qr: ell[%d] = %d outside [1, m = %lld]", i, ell[i], (long long)m[i]);
    if (ell[i] > kWideMaxEll)
      return set_error(TK_EUNSUPPORTED, "tucker_qr: ell[%d] = %d > %d", i, ell[i], kWideMaxEll);
    if (!Z[i]) return set_error(TK_EINVAL, "tucker_qr: Z[%d] is NULL", i);
    if (Y) {
      if (!Y[i] || !U[i]) return set_error(TK_EINVAL, "tucker_qr: Y[%d] or U[%d] is NULL", i, i);
      if (s[i] < 1) return set_error(TK_EINVAL, "tucker_qr: s[%d] < 1", i);
      if (r[i] < 1 || r[i] > ell[i])
        return set_error(TK_EINVAL, "tucker_qr: r[%d] = %d outside [1, ell = %d]", i, r[i], ell[i]);
    }
  }
  Workspace w;
  w.base = static_cast<char*>(ws);
  // sketches up to kMaxEll wide share the batched one-workgroup kernels; wider
  // ones take the wide path, one matrix at a time
  std::vector<QRMat> mats;
  std::vector<WideQR> wide;
  for (int i = 0; i < nmat; ++i) {
    if (ell[i] > kMaxEll) {
      wide.emplace_back();
      plan_wide(w, wide.back(), Z[i], m[i], ell[i], Y != nullptr, Y ? Y[i] : nullptr, Y ? s[i] : 0,
                Y ? r[i] : 0, Y ? U[i] : nullptr, info ? info + i : nullptr);
    } else {
      mats.emplace_back();
      plan_qr(w, mats.back(), Z[i], m[i], ell[i], Y != nullptr, Y ? Y[i] : nullptr, Y ? s[i] : 0,
              Y ? r[i] : 0, Y ? U[i] : nullptr, info ? info + i : nullptr);
    }
  }
  if (!ws) {
    *ws_bytes = w.off;
    return TK_OK;
  }
  if (*ws_bytes < w.off)
    return set_error(TK_EWORKSPACE, "tucker_qr: workspace %zu < required %zu", *ws_bytes, w.off);
  hipStream_t st = as_stream(stream);
  // wide matrices next to narrow ones: the wide path runs on the side stream,
  // forked from and joined back into the caller's stream (the two touch
  // disjoint workspace, inputs and outputs)
  SideStream* side = nullptr;
  if (!wide.empty() && !mats.empty())
    if (tk_status e = side_stream(&side)) return e;
  if (!side) {
    for (WideQR& q : wide) {
      q.udtype = udtype;
      TK_HIP(launch_qr_wide(q, ydtype, Y != nullptr, st));
    }
    return run_qr(mats, ydtype, udtype, Y != nullptr, st);
  }
  std::lock_guard<std::mutex> lock(side->mu);
  TK_HIP(hipEventRecord(side->fork, st));
  TK_HIP(hipStreamWaitEvent(side->st, side->fork, 0));
  tk_status e = TK_OK;
  for (WideQR& q : wide) {
    q.udtype = udtype;
    if (hipError_t he = launch_qr_wide(q, ydtype, Y != nullptr, side->st)) {
      e = set_error(TK_EDEVICE, "tucker_qr: wide QR launch failed: %s", hipGetErrorString(he));
      break;
    }
  }
  if (e == TK_OK) e = run_qr(mats, ydtype, udtype, Y != nullptr, st);
  // joined on every path, so the caller's stream (possibly capturing) is
  // never left forked
  const hipError_t j1 = hipEventRecord(side->join, side->st);
  const hipError_t j2 = j1 == hipSuccess ? hipStreamWaitEvent(st, side->join, 0) : j1;
  if (e != TK_OK) return e;
  TK_HIP(j2);
  return TK_OK;
}

tk_status tucker_core(const tk_tensor* X, const void* const* F, const int32_t* cols, void* G,
                      void* ws, size_t* ws_bytes, void* stream) {
  clear_error();
  const ApiRange range_("tucker_core");
  int64_t N;
  if (tk_status s = check_tensor(X, "tucker_core", &N)) return s;
  if (tk_status s = check_factors(X->order, X->dims, F, cols, "tucker_core")) return s;
  if (!G) return set_error(TK_EINVAL, "tucker_core: G is NULL");
  if (!ws_bytes) return set_error(TK_EINVAL, "tucker_core: ws_bytes is NULL");
  Workspace w;
  w.base = static_cast<char*>(ws);
  CorePlan p;
  plan_core(w, X->dtype, X->order, X->dims, cols, p);
  if (!ws) {
    *ws_bytes = w.off;
    return TK_OK;
  }
  if (*ws_bytes < w.off)
    return set_error(TK_EWORKSPACE, "tucker_core: workspace %zu < required %zu", *ws_bytes, w.off);
  return run_core(X->data, X->dtype, X->order, X->dims, F, cols, G, factor_dtype(X->dtype), p,
                  as_stream(stream));
}

}  // extern "C"

namespace tk {
namespace {
// tucker_reconstruct, and with D = smul (*scale or 1) (Xref - X_hat) as one
// more optional output (D may be Xref itself: every entry is read before it
// is written, by the same thread)
tk_status reconstruct_impl(int32_t order, const int64_t* dims, int32_t fdtype, const void* G,
                           const void* const* F, const int32_t* cols, const tk_tensor* Xref,
                           void* Xhat, void* D, const double* scale, double smul, double* resid2,
                           void* ws, size_t* ws_bytes, void* stream) {
  if (order < 1 || order > TK_MAX_ORDER) return set_error(TK_EINVAL, "tucker_reconstruct: bad order %d", order);
  if (!dims) return set_error(TK_EINVAL, "tucker_reconstruct: dims is NULL");
  for (int k = 0; k < order; ++k)
    if (dims[k] < 1) return set_error(TK_EINVAL, "tucker_reconstruct: dims[%d] < 1", k);
  if (fdtype != TK_F64 && fdtype != TK_F32)
    return set_error(TK_EINVAL, "tucker_reconstruct: fdtype must be TK_F64 or TK_F32");
  if (!G) return set_error(TK_EINVAL, "tucker_reconstruct: G is NULL");
  if (tk_status s = check_factors(order, dims, F, cols, "tucker_reconstruct")) return s;
  if (!Xhat && !resid2 && !D) return set_error(TK_EINVAL, "tucker_reconstruct: neither Xhat nor resid2 given");
  if (resid2 && !Xref) return set_error(TK_EINVAL, "tucker_reconstruct: resid2 needs Xref");
  if (D && !Xref) return set_error(TK_EINVAL, "tucker_reconstruct: the scaled difference needs Xref");
  if (!ws_bytes) return set_error(TK_EINVAL, "tucker_reconstruct: ws_bytes is NULL");
  if (Xref) {
    int64_t N;
    if (tk_status s = check_tensor(Xref, "tucker_reconstruct(Xref)", &N)) return s;
    if (Xref->order != order) return set_error(TK_EINVAL, "tucker_reconstruct: Xref order mismatch");
    for (int k = 0; k < order; ++k)
      if (Xref->dims[k] != dims[k]) return set_error(TK_EINVAL, "tucker_reconstruct: Xref dims[%d] mismatch", k);
    if (factor_dtype(Xref->dtype) != fdtype)
      return set_error(TK_EINVAL, "tucker_reconstruct: fdtype does not match Xref's factor dtype");
  }
  // FP32 tensors of suitable shape: expand the leading modes (the last of them
  // into FP32), then one MFMA pass for the two trailing modes and the residual
  const bool fused = Xref && Xref->dtype == TK_F32 && fdtype == TK_F32 &&
                     resid2_supported(TK_F32, order, dims, cols);
  if (fused) {
    int64_t shape[TK_MAX_ORDER];
    for (int k = 0; k < order; ++k) shape[k] = cols[k];
    int64_t mx = 1;
    for (int k = 0; k < order - 2; ++k) {
      shape[k] = dims[k];
      mx = std::max(mx, prod(shape, 0, order));
    }
    Workspace w;
    w.base = static_cast<char*>(ws);
    double* buf[2] = {w.take<double>((size_t)mx), w.take<double>((size_t)mx)};
    float* T32 = w.take<float>((size_t)mx);
    int64_t smax = 0;
    for (int k = 0; k < order; ++k) smax = std::max(smax, mode_product_scratch(dims[k], cols[k]));
    double* mt = w.take<double>((size_t)smax);
    const int64_t A = prod(dims, 0, order - 2);
    double* partials = w.take<double>((size_t)2 * resid2_waves(A));
    if (!ws) {
      *ws_bytes = w.off;
      return TK_OK;
    }
    if (*ws_bytes < w.off)
      return set_error(TK_EWORKSPACE, "tucker_reconstruct: workspace %zu < required %zu", *ws_bytes, w.off);
    hipStream_t st = as_stream(stream);
    for (int k = 0; k < order; ++k) shape[k] = cols[k];
    const void* cur = G;
    int cur_dt = fdtype;
    for (int k = 0; k < order - 2; ++k) {
      const bool last = k == order - 3;
      ModeProduct mp{};
      mp.in = cur;
      mp.A = prod(shape, 0, k);
      mp.Q = shape[k];
      mp.B = prod(shape, k + 1, order);
      mp.P = (int32_t)dims[k];
      mp.M = F[k];
      mp.Mt = mt;
      mp.rs = cols[k];   // M[p][q] = F[p][q]
      mp.cs = 1;
      mp.out = last ? (void*)T32 : (void*)buf[k & 1];
      TK_HIP(launch_mode_product(mp, cur_dt, last ? TK_F32 : TK_F64, fdtype, st));
      shape[k] = dims[k];
      cur = mp.out;
      cur_dt = last ? TK_F32 : TK_F64;
    }
    ResidFused2 r{};
    r.X = static_cast<const float*>(Xref->data);
    r.T = T32;
    r.FI = static_cast<const float*>(F[order - 2]);
    r.FJ = static_cast<const float*>(F[order - 1]);
    r.Xhat = static_cast<float*>(Xhat);
    r.D = static_cast<float*>(D);
    r.scale = scale;
    r.smul = smul;
    r.partials = partials;
    r.resid2 = resid2;
    r.A = A;
    r.nI = (int32_t)dims[order - 2];
    r.nJ = (int32_t)dims[order - 1];
    r.cI = cols[order - 2];
    r.cJ = cols[order - 1];
    TK_HIP(profile_begin(st));
    TK_HIP(launch_resid2_f32(r, st));
    TK_HIP(profile_end(st));
    return TK_OK;
  }
  // small trailing modes (n <= 64, ranks <= 16), residual only, FP32 factors:
  // expand the leading modes (the last of them into FP32), then one MFMA pass
  // over X (BF16, FP16 or FP32) for the two trailing modes and the residual
  if (Xref && resid2 && !Xhat && !D && fdtype == TK_F32 &&
      resid_slab_supported(Xref->dtype, order, dims, cols)) {
    int64_t shape[TK_MAX_ORDER];
    for (int k = 0; k < order; ++k) shape[k] = cols[k];
    int64_t mx = 1;
    for (int k = 0; k < order - 2; ++k) {
      shape[k] = dims[k];
      mx = std::max(mx, prod(shape, 0, order));
    }
    Workspace w;
    w.base = static_cast<char*>(ws);
    double* buf[2] = {w.take<double>((size_t)mx), w.take<double>((size_t)mx)};
    float* T32 = w.take<float>((size_t)mx);
    int64_t smax = 0;
    for (int k = 0; k < order; ++k) smax = std::max(smax, mode_product_scratch(dims[k], cols[k]));
    double* mt = w.take<double>((size_t)smax);
    const int64_t A = prod(dims, 0, order - 2);
    double* partials = w.take<double>((size_t)2 * resid_slab_waves(A));
    if (!ws) {
      *ws_bytes = w.off;
      return TK_OK;
    }
    if (*ws_bytes < w.off)
      return set_error(TK_EWORKSPACE, "tucker_reconstruct: workspace %zu < required %zu", *ws_bytes, w.off);
    hipStream_t st = as_stream(stream);
    for (int k = 0; k < order; ++k) shape[k] = cols[k];
    const void* cur = G;
    int cur_dt = fdtype;
    for (int k = 0; k < order - 2; ++k) {
      const bool last = k == order - 3;
      ModeProduct mp{};
      mp.in = cur;
      mp.A = prod(shape, 0, k);
      mp.Q = shape[k];
      mp.B = prod(shape, k + 1, order);
      mp.P = (int32_t)dims[k];
      mp.M = F[k];
      mp.Mt = mt;
      mp.rs = cols[k];   // M[p][q] = F[p][q]
      mp.cs = 1;
      mp.out = last ? (void*)T32 : (void*)buf[k & 1];
      TK_HIP(launch_mode_product(mp, cur_dt, last ? TK_F32 : TK_F64, fdtype, st));
      shape[k] = dims[k];
      cur = mp.out;
      cur_dt = last ? TK_F32 : TK_F64;
    }
    ResidSlab r{};
    r.X = Xref->data;
    r.T = T32;
    r.FI = static_cast<const float*>(F[order - 2]);
    r.FJ = static_cast<const float*>(F[order - 1]);
    r.partials = partials;
    r.resid2 = resid2;
    r.A = A;
    r.nI = (int32_t)dims[order - 2];
    r.nJ = (int32_t)dims[order - 1];
    r.cI = cols[order - 2];
    r.cJ = cols[order - 1];
    TK_HIP(profile_begin(st));
    TK_HIP(launch_resid_slab(r, Xref->dtype, st));
    TK_HIP(profile_end(st));
    return TK_OK;
  }
  // FP32, last factor wider than 64 columns: expand modes 0 .. d-2 (the last
  // of them into FP32), the last mode on MFMA into X_hat (or a workspace
  // copy), then the residual over (X, X_hat) in one streaming pass
  const int64_t A_l = prod(dims, 0, order - 1);
  const bool mlast = fdtype == TK_F32 && order >= 2 && cols[order - 1] > 64 &&
                     (!Xref || Xref->dtype == TK_F32) &&
                     mode_last_mfma_supported(A_l, cols[order - 1], (int32_t)dims[order - 1]);
  if (mlast) {
    int64_t shape[TK_MAX_ORDER];
    for (int k = 0; k < order; ++k) shape[k] = cols[k];
    int64_t mx = 1;
    for (int k = 0; k + 2 < order; ++k) {   // FP64 outputs: every expansion but mode d-2's
      shape[k] = dims[k];
      mx = std::max(mx, prod(shape, 0, order));
    }
    const int64_t n_l = dims[order - 1];
    // X_hat goes to Xhat, else to a workspace buffer of a bounded number of
    // rows, reused chunk by chunk (never to D, which may be Xref itself)
    const int64_t rows = Xhat ? A_l : std::min<int64_t>(A_l, std::max<int64_t>(32, ((int64_t)64 << 20) / (n_l * 4)) / 32 * 32);
    const int64_t nchunk = ceil_div(A_l, rows);
    Workspace w;
    w.base = static_cast<char*>(ws);
    double* buf[2] = {w.take<double>((size_t)mx), w.take<double>((size_t)mx)};
    float* T32 = w.take<float>((size_t)(A_l * cols[order - 1]));
    float* Xh32 = Xhat ? static_cast<float*>(Xhat) : w.take<float>((size_t)(rows * n_l));
    int64_t smax = 0;
    for (int k = 0; k < order; ++k) smax = std::max(smax, mode_product_scratch(dims[k], cols[k]));
    double* mt = w.take<double>((size_t)smax);
    const int64_t nb = resid_pair_blocks(rows * n_l);
    double* partials = w.take<double>((size_t)(2 * nb * nchunk));
    if (!ws) {
      *ws_bytes = w.off;
      return TK_OK;
    }
    if (*ws_bytes < w.off)
      return set_error(TK_EWORKSPACE, "tucker_reconstruct: workspace %zu < required %zu", *ws_bytes, w.off);
    hipStream_t st = as_stream(stream);
    for (int k = 0; k < order; ++k) shape[k] = cols[k];
    const void* cur = G;
    int cur_dt = fdtype;
    for (int k = 0; k + 1 < order; ++k) {
      const bool to32 = k + 2 == order;
      ModeProduct mp{};
      mp.in = cur;
      mp.A = prod(shape, 0, k);
      mp.Q = shape[k];
      mp.B = prod(shape, k + 1, order);
      mp.P = (int32_t)dims[k];
      mp.M = F[k];
      mp.Mt = mt;
      mp.rs = cols[k];   // M[p][q] = F[p][q]
      mp.cs = 1;
      mp.out = to32 ? (void*)T32 : (void*)buf[k & 1];
      TK_HIP(launch_mode_product(mp, cur_dt, to32 ? TK_F32 : TK_F64, fdtype, st));
      shape[k] = dims[k];
      cur = mp.out;
      cur_dt = to32 ? TK_F32 : TK_F64;
    }
    const float* X32 = Xref ? static_cast<const float*>(Xref->data) : nullptr;
    TK_HIP(profile_begin(st));
    for (int64_t c = 0; c < nchunk; ++c) {
      const int64_t r0 = c * rows, nr = std::min<int64_t>(rows, A_l - r0);
      float* xh = Xhat ? Xh32 + r0 * n_l : Xh32;
      ModeMfma mm{};
      mm.in = T32 + r0 * cols[order - 1];
      mm.F = static_cast<const float*>(F[order - 1]);
      mm.A = nr;
      mm.Q = cols[order - 1];
      mm.B = 1;
      mm.P = (int32_t)n_l;
      mm.ftrans = 1;
      mm.out = xh;
      TK_HIP(launch_mode_last_mfma_f32(mm, TK_F32, st));
      if (X32 && (resid2 || D))
        TK_HIP(launch_resid_pair_f32(X32 + r0 * n_l, xh, nr * n_l, D ? static_cast<float*>(D) + r0 * n_l : nullptr,
                                     scale, smul, partials + 2 * nb * c, nullptr, st));
    }
    if (resid2) TK_HIP(launch_pair_sum(partials, nb * nchunk, resid2, st));
    TK_HIP(profile_end(st));
    return TK_OK;
  }
  // expand modes 0 .. d-2 into FP64 intermediates, the last one fused with the residual
  int64_t shape[TK_MAX_ORDER];
  for (int k = 0; k < order; ++k) shape[k] = cols[k];
  int64_t mx = prod(shape, 0, order);
  for (int k = 0; k < order - 1; ++k) {
    shape[k] = dims[k];
    mx = std::max(mx, prod(shape, 0, order));
  }
  Workspace w;
  w.base = static_cast<char*>(ws);
  double* buf[2] = {w.take<double>((size_t)mx), w.take<double>((size_t)mx)};
  int64_t smax = 0;
  for (int k = 0; k < order; ++k) smax = std::max(smax, mode_product_scratch(dims[k], cols[k]));
  double* mt = w.take<double>((size_t)smax);
  const int64_t A_last = prod(dims, 0, order - 1);
  const int64_t nb = expand_residual_blocks(A_last * dims[order - 1]);
  double* partials = w.take<double>((size_t)2 * nb);
  if (!ws) {
    *ws_bytes = w.off;
    return TK_OK;
  }
  if (*ws_bytes < w.off)
    return set_error(TK_EWORKSPACE, "tucker_reconstruct: workspace %zu < required %zu", *ws_bytes, w.off);
  hipStream_t st = as_stream(stream);
  for (int k = 0; k < order; ++k) shape[k] = cols[k];
  const void* cur = G;
  int cur_dt = fdtype;
  int which = 0;
  for (int k = 0; k < order - 1; ++k) {
    ModeProduct mp{};
    mp.in = cur;
    mp.A = prod(shape, 0, k);
    mp.Q = shape[k];
    mp.B = prod(shape, k + 1, order);
    mp.P = (int32_t)dims[k];
    mp.M = F[k];
    mp.Mt = mt;
    mp.rs = cols[k];   // M[p][q] = F[p][q]
    mp.cs = 1;
    mp.out = buf[which];
    TK_HIP(launch_mode_product(mp, cur_dt, TK_F64, fdtype, st));
    shape[k] = dims[k];
    cur = buf[which];
    cur_dt = TK_F64;
    which ^= 1;
  }
  if (order == 1 && fdtype != TK_F64) {
    // the last expansion reads an FP64 intermediate: widen the c_0 core values
    TK_HIP(launch_to_f64(G, fdtype, buf[0], cols[0], st));
    cur = buf[0];
  }
  ExpandResidual e{};
  e.T = static_cast<const double*>(cur);
  e.F = F[order - 1];
  e.X = Xref ? Xref->data : nullptr;
  e.Xhat = Xhat;
  e.D = D;
  e.scale = scale;
  e.smul = smul;
  e.partials = resid2 ? partials : nullptr;
  e.resid2 = resid2;
  e.A = A_last;
  e.n = dims[order - 1];
  e.c = cols[order - 1];
  TK_HIP(profile_begin(st));
  TK_HIP(launch_expand_residual(e, Xref ? Xref->dtype : fdtype, fdtype, st));
  TK_HIP(profile_end(st));
  return TK_OK;
}

}  // namespace
}  // namespace tk

extern "C" {

tk_status tucker_reconstruct(int32_t order, const int64_t* dims, int32_t fdtype, const void* G,
                             const void* const* F, const int32_t* cols, const tk_tensor* Xref,
                             void* Xhat, double* resid2, void* ws, size_t* ws_bytes,
                             void* stream) {
  clear_error();
  const ApiRange range_("tucker_reconstruct");
  return reconstruct_impl(order, dims, fdtype, G, F, cols, Xref, Xhat, nullptr, nullptr, 0.0, resid2, ws,
                          ws_bytes, stream);
}

// The tree must be the balanced heap tree of this order (left child = first
// ceil(|S|/2) modes of S), the one every H-Tucker entry point is built for.
tk_status check_ht_tree(const tk_tree* tree, int d, const char* name) {
  const int nn = 2 * d - 1;
  if (tree->num_nodes != nn)
    return set_error(TK_EINVAL, "%s: num_nodes %d != 2 order - 1", name, tree->num_nodes);
  if (!tree->left || !tree->right || !tree->first_mode || !tree->num_modes)
    return set_error(TK_EINVAL, "%s: tree arrays are NULL", name);
  // the expected balanced heap tree (left child = first ceil(|S|/2) modes)
  {
    std::vector<int> ef(1, 0), ec(1, d), el, er;
    size_t head = 0;
    el.assign(1, -1);
    er.assign(1, -1);
    while (head < ef.size()) {
      // breadth-first, children appended in order
      const size_t end = ef.size();
      std::vector<std::pair<int, int>> kids;
      for (size_t t = head; t < end; ++t) {
        if (ec[t] > 1) {
          const int cl = (ec[t] + 1) / 2;
          el[t] = (int)(end + kids.size());
          kids.push_back({ef[t], cl});
          er[t] = (int)(end + kids.size());
          kids.push_back({ef[t] + cl, ec[t] - cl});
        }
      }
      head = end;
      for (auto& kd : kids) {
        ef.push_back(kd.first);
        ec.push_back(kd.second);
        el.push_back(-1);
        er.push_back(-1);
      }
    }
    if ((int)ef.size() != nn) return set_error(TK_EINVAL, "%s: internal tree error", name);
    for (int t = 0; t < nn; ++t)
      if (tree->first_mode[t] != ef[t] || tree->num_modes[t] != ec[t] || tree->left[t] != el[t] ||
          tree->right[t] != er[t])
        return set_error(TK_EINVAL, "%s: node %d differs from the balanced heap tree", name, t);
  }
  return TK_OK;
}

tk_status htucker_decompose(const tk_tensor* X, const tk_tree* tree, const int32_t* rank,
                            const tk_sketch* sk, void* const* U, void* const* B, int32_t* info,
                            void* ws, size_t* ws_bytes, void* stream) {
  clear_error();
  const ApiRange range_("htucker_decompose");
  int64_t N;
  if (tk_status s = check_tensor(X, "htucker_decompose", &N)) return s;
  const int d = X->order;
  if (d < 2) return set_error(TK_EINVAL, "htucker_decompose: order must be >= 2");
  if (!tree || !rank || !sk || !U || !B || !ws_bytes)
    return set_error(TK_EINVAL, "htucker_decompose: NULL argument");
  const int nn = 2 * d - 1;
  if (tk_status s = check_ht_tree(tree, d, "htucker_decompose")) return s;
  std::vector<int64_t> nS(nn), nc(nn), A(nn), Bv(nn);
  for (int t = 0; t < nn; ++t) {
    const int f = tree->first_mode[t], c = tree->num_modes[t];
    A[t] = prod(X->dims, 0, f);
    nS[t] = prod(X->dims, f, f + c);
    Bv[t] = prod(X->dims, f + c, d);
    nc[t] = N / nS[t];
  }
  for (int t = 1; t < nn; ++t) {
    if (tk_status s = check_sketch(sk[t], nS[t], nc[t], "node", t)) return s;
    if (rank[t] < 1 || rank[t] > sk[t].ell)
      return set_error(TK_EINVAL, "htucker_decompose: rank[%d] = %d outside [1, ell = %d]", t, rank[t], sk[t].ell);
    if (!U[t]) return set_error(TK_EINVAL, "htucker_decompose: U[%d] is NULL", t);
    if (tree->left[t] >= 0 && !B[t]) return set_error(TK_EINVAL, "htucker_decompose: B[%d] is NULL", t);
  }
  if (!B[0]) return set_error(TK_EINVAL, "htucker_decompose: B[0] is NULL");
  for (int t = 0; t < nn; ++t) {
    if (tree->left[t] < 0) continue;
    const int l = tree->left[t], r = tree->right[t];
    if (rank[l] > kMaxEll || rank[r] > kMaxEll)
      return set_error(TK_EUNSUPPORTED, "htucker_decompose: child rank above %d", kMaxEll);
  }
  // bases and transfer tensors are small: they are produced in FP64 for every
  // tensor dtype, so storing them adds no error to the format
  const int fdt = TK_F64;
  Workspace w;
  w.base = static_cast<char*>(ws);
  // A dense node (every column sampled: idx NULL, s = n_notS) whose modes
  // are a prefix or a suffix of X's (the root's children) is sketched and
  // W-stepped by products with X itself: Z = X^(S) Omega and M = Q^T X^(S)
  // are mode products along X's first or last dimension, and the W step
  // starts from the Gram M M^T, so no copy of the unfolding is formed.
  // Other nodes gather their sampled columns.
  const bool xf = X->dtype == TK_F64 || X->dtype == TK_F32;
  std::vector<char> dense(nn, 0);
  for (int t = 1; t < nn; ++t)
    dense[t] = xf && sk[t].idx == nullptr && sk[t].s == nc[t] && (A[t] == 1 || Bv[t] == 1) && nc[t] > 1;
  const int odt = X->dtype == TK_F64 ? TK_F64 : TK_F32;   // Omega's dtype (the factor dtype)
  // sketches of every non-root node
  SketchBatch sb{};
  std::vector<double*> Z(nn, nullptr);
  std::vector<void*> Y(nn, nullptr);
  const size_t xs = dtype_size(X->dtype);
  for (int t = 1; t < nn; ++t) {
    Z[t] = w.take<double>((size_t)nS[t] * sk[t].ell);
    if (!dense[t]) Y[t] = w.take<char>((size_t)nS[t] * sk[t].s * xs);
  }
  for (int t = 1; t < nn; ++t)
    if (!dense[t])
      plan_unit(w, sb.u[sb.count++], X->data, A[t], nS[t], Bv[t], sk[t], Z[t], Y[t], sb.total_blocks,
                sb.total_out);
  std::vector<QRMat> mats(nn - 1);
  for (int t = 1; t < nn; ++t)
    plan_qr(w, mats[t - 1], Z[t], nS[t], sk[t].ell, true, Y[t], dense[t] ? kQRColChunk : sk[t].s, rank[t],
            U[t], info ? info + t : nullptr);
  // dense nodes: M (n_notS x ell values), a transposed copy, the unfolded
  // product's partials and the mode products' factor table
  std::vector<double*> Md(nn, nullptr), Mt(nn, nullptr);
  int64_t dmt = 1, dup = 1;
  for (int t = 1; t < nn; ++t) {
    if (!dense[t]) continue;
    const int ell = sk[t].ell;
    Md[t] = w.take<double>((size_t)nc[t] * ell);
    Mt[t] = w.take<double>((size_t)std::max<int64_t>(nc[t], nS[t]) * ell);
    dmt = std::max(dmt, mode_product_scratch(ell, nc[t]));
    dmt = std::max(dmt, mode_product_scratch(ell, nS[t]));
    dup = std::max<int64_t>(dup, (int64_t)unfold_gemm_splits(ell, ell, nc[t]) * ell * ell);
  }
  double* dense_mt = w.take<double>((size_t)dmt);
  double* dense_up = w.take<double>((size_t)dup);
  // partials of the first-dimension mode products (q split over up to 16 blocks)
  constexpr int kDenseSplit = 16;
  int64_t dpart = 1;
  for (int t = 1; t < nn; ++t)
    if (dense[t]) dpart = std::max<int64_t>(dpart, (int64_t)kDenseSplit * sk[t].ell * std::max(nc[t], nS[t]));
  double* dense_part = dpart > 1 ? w.take<double>((size_t)dpart) : nullptr;
  // both children of the root dense (a prefix and a suffix of X's modes): the
  // sketch products X Omega_l and Omega_r^T X share one read of X, and so do
  // the W-step products Q_l^T X and X Q_r
  const int L0 = tree->left[0], R0 = tree->right[0];
  const bool two_sided = dense[L0] && dense[R0] && A[L0] == 1 && Bv[R0] == 1 &&
                         twoside_supported(X->dtype, nS[L0], nS[R0], sk[L0].ell, sk[R0].ell);
  double* ts_part = two_sided ? w.take<double>((size_t)twoside_partials(nS[L0], nS[R0])) : nullptr;
  auto two_side = [&](const void* P1, int k1, const void* P2, int k2, int p_dt, double* o1, double* o2,
                      bool o2t) -> hipError_t {
    TwoSide x{};
    x.X = static_cast<const float*>(X->data);
    x.P1 = P1;
    x.P2 = P2;
    x.out1 = o1;
    x.out2 = o2;
    x.part1 = ts_part;
    x.n1 = nS[L0];
    x.n2 = nS[R0];
    x.k1 = k1;
    x.k2 = k2;
    x.out2_transposed = o2t ? 1 : 0;
    return launch_twoside(x, p_dt, as_stream(stream));
  };
  // transfers of internal non-root nodes
  std::vector<Transfer> tr;
  for (int t = 1; t < nn; ++t) {
    if (tree->left[t] < 0) continue;
    const int l = tree->left[t], r = tree->right[t];
    Transfer x{};
    x.US = U[t];
    x.Ul = U[l];
    x.Ur = U[r];
    x.Bout = B[t];
    x.nl = nS[l];
    x.nr = nS[r];
    x.rS = rank[t];
    x.rl = rank[l];
    x.rr = rank[r];
    x.V = w.take<double>((size_t)x.nl * x.rr * x.rS);
    x.Mt = w.take<double>((size_t)mode_product_scratch(x.rr, x.nr));
    tr.push_back(x);
  }
  // root: X viewed as (n_l, n_r): B_R = U_l^T X U_r
  const int L = tree->left[0], R = tree->right[0];
  const bool root_fused = root_pass_supported(X->dtype, nS[L], nS[R], rank[L], rank[R]);
  double* t1 = root_fused ? nullptr : w.take<double>((size_t)nS[L] * rank[R]);
  double* mt_root = root_fused ? nullptr
                               : w.take<double>((size_t)std::max(mode_product_scratch(rank[R], nS[R]),
                                                                 mode_product_scratch(rank[L], nS[L])));
  double* root_part = root_fused ? w.take<double>((size_t)root_pass_partials(nS[L], nS[R])) : nullptr;
  if (!ws) {
    *ws_bytes = w.off;
    return TK_OK;
  }
  if (*ws_bytes < w.off)
    return set_error(TK_EWORKSPACE, "htucker_decompose: workspace %zu < required %zu", *ws_bytes, w.off);
  hipStream_t st = as_stream(stream);
  // an order <= 16 tree has at most 30 non-root nodes: a single sketch launch
  if (sb.count > 0) TK_HIP(launch_sketch(X->dtype, sb, st));
  auto mode_x = [&](int64_t Aa, int64_t Qq, int64_t Bb, int P, const void* Mm, int m_dt, double* out,
                    const void* in, int in_dt) -> hipError_t {
    ModeProduct mp{};
    mp.in = in;
    mp.A = Aa;
    mp.Q = Qq;
    mp.B = Bb;
    mp.P = P;
    mp.M = Mm;
    mp.Mt = dense_mt;
    mp.rs = 1;
    mp.cs = P;           // M[p][q] = Mm[q * P + p]: an (Qq x P) row-major matrix used transposed
    mp.out = out;
    mp.part = dense_part;
    mp.qsplit_max = kDenseSplit;
    return launch_mode_product(mp, in_dt, TK_F64, m_dt, st);
  };
  if (two_sided)   // Z_l = X Omega_l; Z_r^T = Omega_r^T X, written transposed
    TK_HIP(two_side(sk[L0].omega, sk[L0].ell, sk[R0].omega, sk[R0].ell, odt, Z[L0], Z[R0], true));
  for (int t = 1; t < nn; ++t) {
    if (!dense[t] || (two_sided && (t == L0 || t == R0))) continue;
    const int ell = sk[t].ell;
    if (A[t] == 1) {     // prefix: X^(S) is X viewed n_S x n_notS, Z = X Omega
      TK_HIP(mode_x(nS[t], nc[t], 1, ell, sk[t].omega, odt, Z[t], X->data, X->dtype));
    } else {             // suffix: X^(S) = (X viewed n_notS x n_S)^T, Z^T = Omega^T X
      TK_HIP(mode_x(1, nc[t], nS[t], ell, sk[t].omega, odt, Mt[t], X->data, X->dtype));
      TK_HIP(launch_transpose_f64(Mt[t], Z[t], ell, nS[t], st));
    }
  }
  // CholeskyQR of every node; then the W step of the sampled nodes from their
  // gathered columns and of the dense ones from the Gram of Q^T X^(S)
  if (tk_status s = run_qr(mats, X->dtype, fdt, false, st)) return s;
  std::vector<QRMat> sparse_m, dense_m;
  for (int t = 1; t < nn; ++t) (dense[t] ? dense_m : sparse_m).push_back(mats[t - 1]);
  if (tk_status s = run_wstep(sparse_m, X->dtype, fdt, false, st)) return s;
  if (two_sided)   // M_l = Q_l^T X (ell_l x n_r) and M_r^T = X Q_r (n_l x ell_r)
    TK_HIP(two_side(mats[R0 - 1].Z, sk[R0].ell, mats[L0 - 1].Z, sk[L0].ell, TK_F64, Md[R0], Md[L0], false));
  for (int t = 1; t < nn; ++t) {
    if (!dense[t]) continue;
    const int ell = sk[t].ell;
    const QRMat& q = mats[t - 1];
    const bool done = two_sided && (t == L0 || t == R0);
    UnfoldGemm g{};
    if (A[t] == 1) {     // M = Q^T X^(S): ell x n_notS
      if (!done) TK_HIP(mode_x(1, nS[t], nc[t], ell, q.Z, TK_F64, Md[t], X->data, X->dtype));
      g.pre = 1;
      g.post = nc[t];
    } else {             // M^T = X_(n_notS x n_S) Q: n_notS x ell
      if (!done) TK_HIP(mode_x(nc[t], nS[t], 1, ell, q.Z, TK_F64, Md[t], X->data, X->dtype));
      g.pre = nc[t];
      g.post = 1;
    }
    g.A = Md[t];
    g.B = Md[t];
    g.out = q.cpart;
    g.partials = dense_up;
    g.n = ell;
    g.c = ell;
    g.splits = unfold_gemm_splits(ell, ell, nc[t]);
    g.accumulate = 0;
    TK_HIP(launch_unfold_gemm(g, TK_F64, TK_F64, TK_F64, st));
  }
  if (tk_status s = run_wstep(dense_m, X->dtype, fdt, true, st)) return s;
  for (const Transfer& x : tr) TK_HIP(launch_transfer(x, fdt, st));
  if (root_fused) {
    RootPass rp{};
    rp.X = static_cast<const float*>(X->data);
    rp.UL = static_cast<const double*>(U[L]);
    rp.UR = static_cast<const double*>(U[R]);
    rp.partials = root_part;
    rp.out = static_cast<double*>(B[0]);
    rp.nL = nS[L];
    rp.nR = nS[R];
    rp.rL = rank[L];
    rp.rR = rank[R];
    TK_HIP(launch_root_pass(rp, st));
  } else {
    ModeProduct mp{};
    mp.in = X->data;
    mp.A = nS[L];
    mp.Q = nS[R];
    mp.B = 1;
    mp.P = rank[R];
    mp.M = U[R];
    mp.Mt = mt_root;
    mp.rs = 1;
    mp.cs = rank[R];
    mp.out = t1;
    TK_HIP(profile_begin(st));
    TK_HIP(launch_mode_product(mp, X->dtype, TK_F64, fdt, st));
    TK_HIP(profile_end(st));
    ModeProduct m2{};
    m2.in = t1;
    m2.A = 1;
    m2.Q = nS[L];
    m2.B = rank[R];
    m2.P = rank[L];
    m2.M = U[L];
    m2.Mt = mt_root;
    m2.rs = 1;
    m2.cs = rank[L];
    m2.out = B[0];
    TK_HIP(launch_mode_product(m2, TK_F64, fdt, fdt, st));
  }
  return TK_OK;
}

// ------------------------------------------------------------------ H-Tucker format
// Shared checks and plan of the format's entry points: node sizes, the nested
// bases of every internal non-root node (U_S = C_S x_0 U_Sl x_1 U_Sr with
// C_S[j][k][i] = B_S[i][j][k], nestedness of Section 4) and their buffers.
struct HTFormat {
  int d = 0, nn = 0, L = 0, R = 0;
  std::vector<int64_t> nS;
  std::vector<double*> NB;      // nested bases (internal non-root nodes)
  double* C = nullptr;          // permuted transfer tensor
  double* E = nullptr;          // C x_0 U_l (and other n_l x r_r x r_S intermediates)
  double* Mt = nullptr;         // mode-product factor table
  int64_t mt_need = 0;
};

tk_status check_ht_format(int32_t order, const int64_t* dims, const tk_tree* tree, const int32_t* rank,
                          const void* const* U, const void* const* B, const char* name, HTFormat& f) {
  if (order < 2 || order > TK_MAX_ORDER)
    return set_error(TK_EINVAL, "%s: order %d outside [2, %d]", name, order, TK_MAX_ORDER);
  if (!dims || !tree || !rank || !U || !B) return set_error(TK_EINVAL, "%s: NULL argument", name);
  for (int k = 0; k < order; ++k)
    if (dims[k] < 1) return set_error(TK_EINVAL, "%s: dims[%d] < 1", name, k);
  if (tk_status s = check_ht_tree(tree, order, name)) return s;
  f.d = order;
  f.nn = 2 * order - 1;
  f.L = tree->left[0];
  f.R = tree->right[0];
  f.nS.assign(f.nn, 0);
  for (int t = 0; t < f.nn; ++t)
    f.nS[t] = prod(dims, tree->first_mode[t], tree->first_mode[t] + tree->num_modes[t]);
  for (int t = 1; t < f.nn; ++t) {
    if (rank[t] < 1) return set_error(TK_EINVAL, "%s: rank[%d] = %d < 1", name, t, rank[t]);
    if (tree->left[t] < 0 && !U[t]) return set_error(TK_EINVAL, "%s: U[%d] (leaf) is NULL", name, t);
    if (tree->left[t] >= 0 && !B[t]) return set_error(TK_EINVAL, "%s: B[%d] is NULL", name, t);
  }
  if (!B[0]) return set_error(TK_EINVAL, "%s: B[0] is NULL", name);
  if (!ht_expand_rpad(rank[f.R]))
    return set_error(TK_EUNSUPPORTED, "%s: rank of the root's right child %d above 64", name, rank[f.R]);
  return TK_OK;
}

void plan_ht_format(Workspace& w, const tk_tree* tree, const int32_t* rank, HTFormat& f) {
  f.NB.assign(f.nn, nullptr);
  int64_t cmax = 1, emax = 1;
  for (int t = 1; t < f.nn; ++t) {
    if (tree->left[t] < 0) continue;
    const int l = tree->left[t], r = tree->right[t];
    f.NB[t] = w.take<double>((size_t)f.nS[t] * rank[t]);
    cmax = std::max<int64_t>(cmax, (int64_t)rank[t] * rank[l] * rank[r]);
    emax = std::max<int64_t>(emax, f.nS[l] * rank[r] * rank[t]);
    f.mt_need = std::max(f.mt_need, mode_product_scratch(f.nS[l], rank[l]));
    f.mt_need = std::max(f.mt_need, mode_product_scratch(f.nS[r], rank[r]));
  }
  f.C = w.take<double>((size_t)cmax);
  f.E = w.take<double>((size_t)emax);
}

const double* ht_basis(const tk_tree* tree, const void* const* U, const HTFormat& f, int t) {
  return tree->left[t] < 0 ? static_cast<const double*>(U[t]) : f.NB[t];
}

// nested bases of every internal non-root node, children before parents
// (heap order: a child's index exceeds its parent's)
tk_status run_ht_bases(const tk_tree* tree, const int32_t* rank, const void* const* U,
                       const void* const* B, const HTFormat& f, hipStream_t st) {
  for (int t = f.nn - 1; t >= 1; --t) {
    if (tree->left[t] < 0) continue;
    const int l = tree->left[t], r = tree->right[t];
    TK_HIP(launch_permute_transfer(static_cast<const double*>(B[t]), f.C, rank[t], rank[l], rank[r], true, st));
    ModeProduct m1{};   // E = C x_0 U_l: (n_l, r_r, r_S)
    m1.in = f.C;
    m1.A = 1;
    m1.Q = rank[l];
    m1.B = (int64_t)rank[r] * rank[t];
    m1.P = (int32_t)f.nS[l];
    m1.M = ht_basis(tree, U, f, l);
    m1.Mt = f.Mt;
    m1.rs = rank[l];
    m1.cs = 1;
    m1.out = f.E;
    TK_HIP(launch_mode_product(m1, TK_F64, TK_F64, TK_F64, st));
    ModeProduct m2{};   // U_S = E x_1 U_r: (n_l, n_r, r_S) = U_S[(a n_r + b)][i]
    m2.in = f.E;
    m2.A = f.nS[l];
    m2.Q = rank[r];
    m2.B = rank[t];
    m2.P = (int32_t)f.nS[r];
    m2.M = ht_basis(tree, U, f, r);
    m2.Mt = f.Mt;
    m2.rs = rank[r];
    m2.cs = 1;
    m2.out = f.NB[t];
    TK_HIP(launch_mode_product(m2, TK_F64, TK_F64, TK_F64, st));
  }
  return TK_OK;
}

tk_status htucker_reconstruct(int32_t order, const int64_t* dims, const tk_tree* tree, const int32_t* rank,
                              const void* const* U, const void* const* B, const tk_tensor* Xref,
                              void* Xhat, int32_t xhat_dtype, double* resid2, void* ws, size_t* ws_bytes,
                              void* stream) {
  clear_error();
  const ApiRange range_("htucker_reconstruct");
  const char* nm = "htucker_reconstruct";
  HTFormat f;
  if (tk_status s = check_ht_format(order, dims, tree, rank, U, B, nm, f)) return s;
  if (!ws_bytes) return set_error(TK_EINVAL, "%s: ws_bytes is NULL", nm);
  if (!Xhat && !resid2) return set_error(TK_EINVAL, "%s: Xhat and resid2 are both NULL", nm);
  if (resid2 && !Xref) return set_error(TK_EINVAL, "%s: resid2 needs Xref", nm);
  if (Xhat && xhat_dtype != TK_F32 && xhat_dtype != TK_F64)
    return set_error(TK_EINVAL, "%s: xhat_dtype must be TK_F32 or TK_F64", nm);
  if (Xref) {
    int64_t N;
    if (tk_status s = check_tensor(Xref, nm, &N)) return s;
    if (Xref->order != order) return set_error(TK_EINVAL, "%s: Xref order %d != %d", nm, Xref->order, order);
    for (int k = 0; k < order; ++k)
      if (Xref->dims[k] != dims[k]) return set_error(TK_EINVAL, "%s: Xref dims[%d] differs", nm, k);
  }
  Workspace w;
  w.base = static_cast<char*>(ws);
  plan_ht_format(w, tree, rank, f);
  const int L = f.L, R = f.R;
  HTExpand e{};
  e.nL = f.nS[L];
  e.nR = f.nS[R];
  e.rr = rank[R];
  e.rpad = ht_expand_rpad(rank[R]);
  ht_expand_grid(e);
  double* T = w.take<double>((size_t)e.nL * e.rpad);
  double* part = resid2 ? w.take<double>((size_t)2 * e.ntile * e.groups) : nullptr;
  f.Mt = w.take<double>((size_t)std::max<int64_t>(1, f.mt_need));
  if (!ws) {
    *ws_bytes = w.off;
    return TK_OK;
  }
  if (*ws_bytes < w.off) return set_error(TK_EWORKSPACE, "%s: workspace %zu < required %zu", nm, *ws_bytes, w.off);
  hipStream_t st = as_stream(stream);
  if (tk_status s = run_ht_bases(tree, rank, U, B, f, st)) return s;
  // root: T = U_Rl B_R, then xhat = T U_Rr^T streamed against the reference
  TK_HIP(launch_ht_rowmat(ht_basis(tree, U, f, L), static_cast<const double*>(B[0]), T, e.nL, rank[L],
                          rank[R], e.rpad, st));
  e.T = T;
  e.UR = ht_basis(tree, U, f, R);
  e.X = Xref ? Xref->data : nullptr;
  e.Xh = Xhat;
  e.partials = part;
  e.resid2 = resid2;
  TK_HIP(profile_begin(st));
  TK_HIP(launch_ht_expand(e, Xref ? Xref->dtype : -1, Xhat ? xhat_dtype : -1, st));
  TK_HIP(profile_end(st));
  return TK_OK;
}

tk_status htucker_reconstruct_vjp(int32_t order, const int64_t* dims, const tk_tree* tree,
                                  const int32_t* rank, const void* const* U, const void* const* B,
                                  const void* H, int32_t h_dtype, void* const* Bbar, void* const* Ubar,
                                  void* ws, size_t* ws_bytes, void* stream) {
  clear_error();
  const ApiRange range_("htucker_reconstruct_vjp");
  const char* nm = "htucker_reconstruct_vjp";
  HTFormat f;
  if (tk_status s = check_ht_format(order, dims, tree, rank, U, B, nm, f)) return s;
  if (!ws_bytes || !H || !Bbar || !Ubar) return set_error(TK_EINVAL, "%s: NULL argument", nm);
  if (h_dtype != TK_F32 && h_dtype != TK_F64) return set_error(TK_EINVAL, "%s: h_dtype must be TK_F32 or TK_F64", nm);
  for (int t = 0; t < f.nn; ++t) {
    if (tree->left[t] >= 0 && !Bbar[t]) return set_error(TK_EINVAL, "%s: Bbar[%d] is NULL", nm, t);
    if (t > 0 && tree->left[t] < 0 && !Ubar[t]) return set_error(TK_EINVAL, "%s: Ubar[%d] is NULL", nm, t);
  }
  Workspace w;
  w.base = static_cast<char*>(ws);
  plan_ht_format(w, tree, rank, f);
  const int L = f.L, R = f.R;
  const int rl0 = rank[L], rr0 = rank[R];
  const int64_t nL = f.nS[L], nR = f.nS[R];
  // adjoints of the internal non-root bases; leaves write to Ubar
  std::vector<double*> UB(f.nn, nullptr);
  int64_t e2 = 1, up = 1;
  int64_t mt = f.mt_need;
  for (int t = 1; t < f.nn; ++t) {
    if (tree->left[t] < 0) continue;
    UB[t] = w.take<double>((size_t)f.nS[t] * rank[t]);
    const int l = tree->left[t], r = tree->right[t];
    const int64_t nl = f.nS[l], nr = f.nS[r];
    e2 = std::max<int64_t>(e2, (int64_t)rank[l] * nr * rank[t]);
    up = std::max<int64_t>(up, (int64_t)unfold_gemm_splits(nl, rank[l], nr * rank[t]) * nl * rank[l]);
    up = std::max<int64_t>(up, (int64_t)unfold_gemm_splits(nr, rank[r], nl * rank[t]) * nr * rank[r]);
    mt = std::max(mt, mode_product_scratch(rank[r], nr));
    mt = std::max(mt, mode_product_scratch(rank[l], nl));
  }
  mt = std::max(mt, mode_product_scratch(rr0, nR));
  mt = std::max(mt, mode_product_scratch(rl0, nL));
  mt = std::max(mt, mode_product_scratch(rl0, rr0));
  mt = std::max(mt, mode_product_scratch(nL, rl0));
  double* E2 = w.take<double>((size_t)e2);
  int64_t cb = 1;
  for (int t = 1; t < f.nn; ++t)
    if (tree->left[t] >= 0) cb = std::max<int64_t>(cb, (int64_t)rank[t] * rank[tree->left[t]] * rank[tree->right[t]]);
  double* Cbar2 = w.take<double>((size_t)cb);
  double* P1 = w.take<double>((size_t)nL * rr0);
  double* Qp = w.take<double>((size_t)rl0 * nR);
  double* W2 = w.take<double>((size_t)rr0 * nR);
  constexpr int kRootSplit = 16;
  double* rpart = w.take<double>((size_t)kRootSplit * rl0 * nR);
  mt = std::max(mt, mode_product_scratch(rr0, rl0));
  double* upart = w.take<double>((size_t)up);
  f.Mt = w.take<double>((size_t)std::max<int64_t>(1, mt));
  if (!ws) {
    *ws_bytes = w.off;
    return TK_OK;
  }
  if (*ws_bytes < w.off) return set_error(TK_EWORKSPACE, "%s: workspace %zu < required %zu", nm, *ws_bytes, w.off);
  hipStream_t st = as_stream(stream);
  if (tk_status s = run_ht_bases(tree, rank, U, B, f, st)) return s;
  auto adj = [&](int t) -> double* { return tree->left[t] < 0 ? static_cast<double*>(Ubar[t]) : UB[t]; };
  auto mode = [&](const void* in, int in_dt, int64_t A, int64_t Q, int64_t Bn, int64_t P, const void* M,
                  int rs, int cs, void* out, double* part = nullptr) -> hipError_t {
    ModeProduct m{};
    m.part = part;
    m.qsplit_max = part ? kRootSplit : 0;
    m.in = in;
    m.A = A;
    m.Q = Q;
    m.B = Bn;
    m.P = (int32_t)P;
    m.M = M;
    m.Mt = f.Mt;
    m.rs = rs;
    m.cs = cs;
    m.out = out;
    return launch_mode_product(m, in_dt, TK_F64, TK_F64, st);
  };
  auto ugemm = [&](const void* A, int adt, const void* Bm, int64_t pre, int64_t n, int64_t c, int64_t post,
                   void* out) -> hipError_t {
    UnfoldGemm g{};
    g.A = A;
    g.B = Bm;
    g.out = out;
    g.partials = upart;
    g.pre = pre;
    g.post = post;
    g.n = (int32_t)n;
    g.c = (int32_t)c;
    g.splits = unfold_gemm_splits(n, c, pre * post);
    g.accumulate = 0;
    return launch_unfold_gemm(g, adt, TK_F64, TK_F64, st);
  };
  const double* UL = ht_basis(tree, U, f, L);
  const double* UR = ht_basis(tree, U, f, R);
  // root, H viewed as n_l x n_r: P1 = H U_Rr; B_R_bar = U_Rl^T P1; U_Rl_bar = P1 B_R^T;
  // U_Rr_bar = H^T U_Rl B_R, contracting H first: Q' = U_Rl^T H (a
  // first-dimension product, its contraction split over blocks), then
  // (B_R^T Q')^T; each reads H once
  TK_HIP(mode(H, h_dtype, nL, nR, 1, rr0, UR, 1, rr0, P1));
  TK_HIP(mode(P1, TK_F64, 1, nL, rr0, rl0, UL, 1, rl0, Bbar[0]));
  TK_HIP(mode(P1, TK_F64, nL, rr0, 1, rl0, B[0], rr0, 1, adj(L)));
  TK_HIP(mode(H, h_dtype, 1, nL, nR, rl0, UL, 1, rl0, Qp, rpart));       // r_l x n_r
  TK_HIP(mode(Qp, TK_F64, 1, rl0, nR, rr0, B[0], 1, rr0, W2));           // r_r x n_r
  TK_HIP(launch_transpose_f64(W2, static_cast<double*>(adj(R)), rr0, nR, st));
  // internal nodes, parents before children: with H' = U_S_bar as (n_l, n_r, r_S)
  // and C = B_S permuted to (r_l, r_r, r_S):
  //   C_bar = H' x_0 U_l^T x_1 U_r^T,  U_l_bar = H'^(0) (C x_1 U_r)^(0)T,
  //   U_r_bar = H'^(1) (C x_0 U_l)^(1)T
  for (int t = 1; t < f.nn; ++t) {
    if (tree->left[t] < 0) continue;
    const int l = tree->left[t], r = tree->right[t];
    const int rS = rank[t], rl = rank[l], rr = rank[r];
    const int64_t nl = f.nS[l], nr = f.nS[r];
    const double* Ul = ht_basis(tree, U, f, l);
    const double* Ur = ht_basis(tree, U, f, r);
    const double* Hs = UB[t];
    TK_HIP(launch_permute_transfer(static_cast<const double*>(B[t]), f.C, rS, rl, rr, true, st));
    TK_HIP(mode(Hs, TK_F64, nl, nr, rS, rr, Ur, 1, rr, f.E));            // (n_l, r_r, r_S)
    TK_HIP(mode(f.E, TK_F64, 1, nl, (int64_t)rr * rS, rl, Ul, 1, rl, Cbar2));   // (r_l, r_r, r_S)
    TK_HIP(launch_permute_transfer(Cbar2, static_cast<double*>(Bbar[t]), rS, rl, rr, false, st));
    TK_HIP(mode(f.C, TK_F64, rl, rr, rS, nr, Ur, rr, 1, E2));            // (r_l, n_r, r_S)
    TK_HIP(ugemm(Hs, TK_F64, E2, 1, nl, rl, nr * rS, adj(l)));
    TK_HIP(mode(f.C, TK_F64, 1, rl, (int64_t)rr * rS, nl, Ul, rl, 1, f.E));   // (n_l, r_r, r_S)
    TK_HIP(ugemm(Hs, TK_F64, f.E, nl, nr, rr, rS, adj(r)));
  }
  return TK_OK;
}

tk_status tucker_core_vjp(const tk_tensor* X, const void* const* F, const int32_t* cols,
                          const void* Gbar, void* Xbar, void* const* Fbar, int32_t accumulate,
                          void* ws, size_t* ws_bytes, void* stream) {
  clear_error();
  const ApiRange range_("tucker_core_vjp");
  int64_t N;
  if (tk_status s = check_tensor(X, "tucker_core_vjp", &N)) return s;
  if (X->dtype != TK_F64 && X->dtype != TK_F32)
    return set_error(TK_EUNSUPPORTED, "tucker_core_vjp: tensor dtype must be F64 or F32");
  if (tk_status s = check_factors(X->order, X->dims, F, cols, "tucker_core_vjp")) return s;
  if (!Gbar) return set_error(TK_EINVAL, "tucker_core_vjp: Gbar is NULL");
  if (!ws_bytes) return set_error(TK_EINVAL, "tucker_core_vjp: ws_bytes is NULL");
  const int d = X->order;
  const int fdt = factor_dtype(X->dtype);
  bool any_f = false;
  for (int k = 0; Fbar && k < d; ++k) any_f |= Fbar[k] != nullptr;
  const bool fused = any_f && grads_fused_ok(X->dtype, d, X->dims, cols);
  Workspace w;
  w.base = static_cast<char*>(ws);
  VjpPlan vp;
  plan_vjp(w, d, X->dims, cols, vp, !fused);
  GradPlan gp;
  if (fused) plan_grads(w, d, X->dims, cols, gp);
  if (!ws) {
    *ws_bytes = w.off;
    return TK_OK;
  }
  if (*ws_bytes < w.off)
    return set_error(TK_EWORKSPACE, "tucker_core_vjp: workspace %zu < required %zu", *ws_bytes, w.off);
  hipStream_t st = as_stream(stream);
  // Xbar (+)= Gbar x_1 F_1 .. x_d F_d
  if (Xbar)
    if (tk_status s = expand_full(Gbar, fdt, d, X->dims, F, cols, Xbar, accumulate != 0, vp, st)) return s;
  // Fbar_k (+)= (X x_{j!=k} F_j^T)^(k) (Gbar^(k))^T
  if (fused) {
    if (tk_status s = run_core_pass(X->data, X->dtype, d, X->dims, F, cols, gp.cp, st)) return s;
    return run_grads(X->data, d, X->dims, F, cols, Gbar, fdt, Fbar, fdt, accumulate != 0, gp, st);
  }
  if (Fbar)
    for (int k = 0; k < d; ++k) {
      if (!Fbar[k]) continue;
      const void* P = nullptr;
      int pdt = 0;
      if (tk_status s = contract_all_but(X->data, X->dtype, d, X->dims, F, cols, k, vp, st, &P, &pdt)) return s;
      if (tk_status s = unfold_product(P, pdt, Gbar, fdt, d, X->dims, cols, k, true, Fbar[k], fdt,
                                       accumulate != 0, vp.upart, st)) return s;
    }
  return TK_OK;
}

tk_status tucker_reconstruct_vjp(int32_t order, const int64_t* dims, int32_t fdtype,
                                 const void* G, const void* const* F, const int32_t* cols,
                                 const void* H, void* Gbar, void* const* Fbar, void* ws,
                                 size_t* ws_bytes, void* stream) {
  clear_error();
  const ApiRange range_("tucker_reconstruct_vjp");
  if (order < 1 || order > TK_MAX_ORDER) return set_error(TK_EINVAL, "tucker_reconstruct_vjp: bad order %d", order);
  if (!dims) return set_error(TK_EINVAL, "tucker_reconstruct_vjp: dims is NULL");
  for (int k = 0; k < order; ++k)
    if (dims[k] < 1) return set_error(TK_EINVAL, "tucker_reconstruct_vjp: dims[%d] < 1", k);
  if (fdtype != TK_F64 && fdtype != TK_F32)
    return set_error(TK_EINVAL, "tucker_reconstruct_vjp: fdtype must be TK_F64 or TK_F32");
  if (!G || !H) return set_error(TK_EINVAL, "tucker_reconstruct_vjp: G or H is NULL");
  if (tk_status s = check_factors(order, dims, F, cols, "tucker_reconstruct_vjp")) return s;
  if (!ws_bytes) return set_error(TK_EINVAL, "tucker_reconstruct_vjp: ws_bytes is NULL");
  bool any_f = false;
  for (int k = 0; Fbar && k < order; ++k) any_f |= Fbar[k] != nullptr;
  const bool fused = grads_fused_ok(fdtype, order, dims, cols);
  Workspace w;
  w.base = static_cast<char*>(ws);
  VjpPlan vp;
  CorePlan cp;
  GradPlan gp;
  if (fused) {
    plan_grads(w, order, dims, cols, gp);
  } else {
    plan_vjp(w, order, dims, cols, vp);
    plan_core(w, fdtype, order, dims, cols, cp);
  }
  if (!ws) {
    *ws_bytes = w.off;
    return TK_OK;
  }
  if (*ws_bytes < w.off)
    return set_error(TK_EWORKSPACE, "tucker_reconstruct_vjp: workspace %zu < required %zu", *ws_bytes, w.off);
  hipStream_t st = as_stream(stream);
  if (fused) {
    // one streaming pass of H gives its partial core T: Gbar is T's remaining
    // contractions, and the factor gradients start from T as well
    if (tk_status s = run_core_pass(H, fdtype, order, dims, F, cols, gp.cp, st)) return s;
    if (Gbar)
      if (tk_status s = run_core_rest(H, fdtype, order, dims, F, cols, Gbar, fdtype, gp.cp, st)) return s;
    if (!any_f) return TK_OK;
    return run_grads(H, order, dims, F, cols, G, fdtype, Fbar, fdtype, false, gp, st);
  }
  // Gbar = H x_1 F_1^T .. x_d F_d^T (the core projection of H)
  if (Gbar)
    if (tk_status s = run_core(H, fdtype, order, dims, F, cols, Gbar, fdtype, cp, st)) return s;
  // Fbar_k = H^(k) ((G x_{j!=k} F_j)^(k))^T = (H x_{j!=k} F_j^T)^(k) (G^(k))^T:
  // contracting H first reads it once per mode through core-sized
  // intermediates (expanding G first would form an H-sized one per mode and
  // reread it for every row of Fbar_k)
  if (Fbar)
    for (int k = 0; k < order; ++k) {
      if (!Fbar[k]) continue;
      const void* P = nullptr;
      int pdt = 0;
      if (tk_status s = contract_all_but(H, fdtype, order, dims, F, cols, k, vp, st, &P, &pdt)) return s;
      if (tk_status s = unfold_product(P, pdt, G, fdtype, order, dims, cols, k, true, Fbar[k], fdtype,
                                       false, vp.upart, st)) return s;
    }
  return TK_OK;
}


tk_status tucker_projection_loss_vjp(const tk_tensor* X, const void* const* F, const int32_t* cols,
                                     const void* G, const double* lbar, void* Xbar, void* const* Fbar,
                                     void* ws, size_t* ws_bytes, void* stream) {
  clear_error();
  const ApiRange range_("tucker_projection_loss_vjp");
  int64_t N;
  if (tk_status s = check_tensor(X, "tucker_projection_loss_vjp", &N)) return s;
  if (X->dtype != TK_F64 && X->dtype != TK_F32)
    return set_error(TK_EUNSUPPORTED, "tucker_projection_loss_vjp: tensor dtype must be F64 or F32");
  if (tk_status s = check_factors(X->order, X->dims, F, cols, "tucker_projection_loss_vjp")) return s;
  if (!G) return set_error(TK_EINVAL, "tucker_projection_loss_vjp: G is NULL");
  if (!ws_bytes) return set_error(TK_EINVAL, "tucker_projection_loss_vjp: ws_bytes is NULL");
  const int d = X->order;
  const int fdt = X->dtype;
  const size_t esz = fdt == TK_F64 ? 8 : 4;
  int64_t gsz = 1;
  for (int k = 0; k < d; ++k) gsz *= cols[k];
  bool any_f = false;
  for (int k = 0; Fbar && k < d; ++k) any_f |= Fbar[k] != nullptr;
  if (!Xbar && !any_f) return set_error(TK_EINVAL, "tucker_projection_loss_vjp: no output requested");
  // own buffers: Gbar (the core of H) and, without Xbar, H itself; then one
  // region that every sub-step reuses in stream order
  Workspace w;
  w.base = static_cast<char*>(ws);
  void* Gb = w.take<char>((size_t)gsz * esz);
  void* Hb = Xbar ? Xbar : (void*)w.take<char>((size_t)N * esz);
  if (!ws) {
    // size query: the sub-steps' own queries check their pointers only for
    // being non-NULL and never dereference them
    Gb = reinterpret_cast<void*>(uintptr_t(256));
    if (!Hb) Hb = reinterpret_cast<void*>(uintptr_t(256));
  }
  const size_t sub_off = (w.off + 255) & ~size_t(255);
  tk_tensor Ht = *X;
  Ht.data = Hb;
  void* null_fb[TK_MAX_ORDER] = {};
  void* const* fb = Fbar ? Fbar : null_fb;
  size_t need[4] = {0, 0, 0, 0};
  if (tk_status s = reconstruct_impl(d, X->dims, fdt, G, F, cols, X, nullptr, Hb, lbar, -2.0, nullptr,
                                     nullptr, &need[0], stream)) return s;
  if (tk_status s = tucker_reconstruct_vjp(d, X->dims, fdt, G, F, cols, Hb, Gb, any_f ? fb : nullptr,
                                           nullptr, &need[1], stream)) return s;
  if (any_f)
    if (tk_status s = tucker_core_vjp(X, F, cols, Gb, nullptr, fb, 1, nullptr, &need[2], stream)) return s;
  if (Xbar)
    if (tk_status s = reconstruct_impl(d, X->dims, fdt, Gb, F, cols, &Ht, nullptr, Xbar, nullptr, -1.0,
                                       nullptr, nullptr, &need[3], stream)) return s;
  const size_t sub = std::max(std::max(need[0], need[1]), std::max(need[2], need[3]));
  const size_t total = sub_off + sub;
  if (!ws) {
    *ws_bytes = total;
    return TK_OK;
  }
  if (*ws_bytes < total)
    return set_error(TK_EWORKSPACE, "tucker_projection_loss_vjp: workspace %zu < required %zu", *ws_bytes, total);
  char* sw = static_cast<char*>(ws) + sub_off;
  size_t sb = sub;
  // H = dL/dX_hat = -2 lbar (X - X_hat), X_hat = G x_k F_k
  if (tk_status s = reconstruct_impl(d, X->dims, fdt, G, F, cols, X, nullptr, Hb, lbar, -2.0, nullptr, sw,
                                     &sb, stream)) return s;
  // through the reconstruction: Gbar = H x_k F_k^T, Fbar = its factor gradients
  sb = sub;
  if (tk_status s = tucker_reconstruct_vjp(d, X->dims, fdt, G, F, cols, Hb, Gb, any_f ? fb : nullptr, sw,
                                           &sb, stream)) return s;
  // through the core projection: Fbar += the factor gradients at Gbar
  sb = sub;
  if (any_f)
    if (tk_status s = tucker_core_vjp(X, F, cols, Gb, nullptr, fb, 1, sw, &sb, stream)) return s;
  // Xbar = Gbar x_k F_k + the direct term 2 lbar (X - X_hat) = Gbar x_k F_k - H
  // (in place: the pass reads H from Xbar and writes -(H - Gbar x_k F_k))
  sb = sub;
  if (Xbar)
    if (tk_status s = reconstruct_impl(d, X->dims, fdt, Gb, F, cols, &Ht, nullptr, Xbar, nullptr, -1.0,
                                       nullptr, sw, &sb, stream)) return s;
  return TK_OK;
}

struct tk_batch_plan {
  tk::BatchPlanData data;
  int device = 0;
};

tk_status tucker_batch_plan_create(int32_t count, const tk_tensor* X, const int32_t* ranks,
                                   const tk_sketch* sk, void* const* U, void* const* G, int32_t* info,
                                   double* resid2, void* ws, size_t* ws_bytes, void* stream,
                                   tk_batch_plan** plan) {
  clear_error();
  const ApiRange range_("tucker_batch_plan_create");
  if (!ws_bytes) return set_error(TK_EINVAL, "tucker_batch_plan_create: ws_bytes is NULL");
  Workspace w;
  w.base = static_cast<char*>(ws);
  BatchPlanData P;
  if (tk_status s = plan_batch(w, count, X, ranks, sk, U, G, info, resid2, P)) return s;
  if (!ws) {
    *ws_bytes = w.off;
    return TK_OK;
  }
  if (*ws_bytes < w.off)
    return set_error(TK_EWORKSPACE, "tucker_batch_plan_create: workspace %zu < required %zu", *ws_bytes, w.off);
  if (!plan) return set_error(TK_EINVAL, "tucker_batch_plan_create: plan is NULL");
  int dev = 0;
  TK_HIP(hipGetDevice(&dev));
  tk_batch_plan* p = new tk_batch_plan();
  p->data = std::move(P);
  p->device = dev;
  if (tk_status s = batch_upload(p->data, as_stream(stream))) {
    delete p;
    return s;
  }
  *plan = p;
  return TK_OK;
}

tk_status tucker_batch_run(const tk_batch_plan* plan, void* stream) {
  clear_error();
  const ApiRange range_("tucker_batch_run");
  if (!plan) return set_error(TK_EINVAL, "tucker_batch_run: plan is NULL");
  return batch_run(plan->data, as_stream(stream));
}

tk_status tucker_batch_autotune(tk_batch_plan* plan, void* stream, char* report, size_t report_bytes) {
  clear_error();
  const ApiRange range_("tucker_batch_autotune");
  if (!plan) return set_error(TK_EINVAL, "tucker_batch_autotune: plan is NULL");
  BatchPlanData& P = plan->data;
  hipStream_t st = as_stream(stream);
  // factors for the timed passes
  if (tk_status s = batch_run(P, st)) return s;
  const int variants[4][2] = {{0, 0}, {1, 2}, {2, 2}, {1, 3}};
  const int64_t chunk_sizes[3] = {kBatchChunkMin, 128 << 10, 512 << 10};
  hipEvent_t e0, e1;
  TK_HIP(hipEventCreate(&e0));
  TK_HIP(hipEventCreate(&e1));
  std::string rep;
  float best = 1e30f;
  int bv = 0, bc = 1;
  tk_status status = TK_OK;
  for (int v = 0; v < 4 && status == TK_OK; ++v)
    for (int c = 0; c < 3 && status == TK_OK; ++c) {
      if ((status = batch_set_schedule(P, variants[v][0], variants[v][1], chunk_sizes[c], st))) break;
      if ((status = batch_core(P, st))) break;   // warm-up
      if (hipEventRecord(e0, st) != hipSuccess) { status = set_error(TK_EDEVICE, "event record failed"); break; }
      for (int r = 0; r < 3 && status == TK_OK; ++r) status = batch_core(P, st);
      if (status) break;
      float ms = 0.0f;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        status = set_error(TK_EDEVICE, "event timing failed");
        break;
      }
      ms /= 3.0f;
      char line[160];
      snprintf(line, sizeof(line), "tiles/unit %d, buffers %d, chunk %lld KB: %.4f ms\n", variants[v][0],
               variants[v][1], (long long)(chunk_sizes[c] >> 10), ms);
      rep += line;
      if (ms < best) {
        best = ms;
        bv = v;
        bc = c;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status) return status;
  if (tk_status s = batch_set_schedule(P, variants[bv][0], variants[bv][1], chunk_sizes[bc], st)) return s;
  char line[160];
  snprintf(line, sizeof(line), "chosen: tiles/unit %d, buffers %d, chunk %lld KB\n", variants[bv][0],
           variants[bv][1], (long long)(chunk_sizes[bc] >> 10));
  rep += line;
  if (report && report_bytes) {
    strncpy(report, rep.c_str(), report_bytes - 1);
    report[report_bytes - 1] = 0;
  }
  return TK_OK;
}

tk_status tucker_batch_get_schedule(const tk_batch_plan* plan, int32_t* tiles_per_unit, int32_t* buffers,
                                    int64_t* chunk_bytes) {
  clear_error();
  const ApiRange range_("tucker_batch_get_schedule");
  if (!plan || !tiles_per_unit || !buffers || !chunk_bytes)
    return set_error(TK_EINVAL, "tucker_batch_get_schedule: NULL argument");
  *tiles_per_unit = plan->data.tg;
  *buffers = plan->data.nbuf;
  *chunk_bytes = plan->data.chunk_bytes;
  return TK_OK;
}

tk_status tucker_batch_set_schedule(tk_batch_plan* plan, int32_t tiles_per_unit, int32_t buffers,
                                    int64_t chunk_bytes, void* stream) {
  clear_error();
  const ApiRange range_("tucker_batch_set_schedule");
  if (!plan) return set_error(TK_EINVAL, "tucker_batch_set_schedule: plan is NULL");
  const bool variant = (tiles_per_unit == 0 && buffers == 0) || (tiles_per_unit == 1 && buffers == 2) ||
                       (tiles_per_unit == 2 && buffers == 2) || (tiles_per_unit == 1 && buffers == 3);
  if (!variant)
    return set_error(TK_EINVAL, "tucker_batch_set_schedule: no streaming-pass form with %d tiles per unit and %d "
                     "buffers", tiles_per_unit, buffers);
  if (chunk_bytes < kBatchChunkMin || chunk_bytes > kBatchChunkMax)
    return set_error(TK_EINVAL, "tucker_batch_set_schedule: chunk of %lld bytes outside [%lld, %lld]",
                     (long long)chunk_bytes, (long long)kBatchChunkMin, (long long)kBatchChunkMax);
  return batch_set_schedule(plan->data, tiles_per_unit, buffers, chunk_bytes, as_stream(stream));
}

void tucker_batch_plan_destroy(tk_batch_plan* plan) { delete plan; }

}  // extern "C"
