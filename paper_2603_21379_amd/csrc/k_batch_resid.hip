// Batching form of the reconstruction residual (Tucker format, Section 3;
// the error measure of Algorithm 1's experiments) for many FP32 tensors of
// uneven order and size in one launch:
//   X_hat_t[a] = F_I T_t[a] F_J^T            (n_I x n_J slabs of tensor t)
//   r2_t = sum (X_t - X_hat_t)^2,  x2_t = sum X_t^2
// where T_t[a] (c_I x c_J) is the core of tensor t expanded over its leading
// modes (done before this pass by the batched mode contraction), so X is read
// once and X_hat is never stored.
//
// The work is a list of chunks (consecutive slabs of one tensor), largest
// first, taken from a queue by the resident waves (the counter is cleared by
// a one-thread kernel before each pass, so runs can be replayed from a graph).  Per slab, on v_mfma_f32_16x16x4f32:
//  stage 1  P = T[a] F_J^T (c_I x n_J) into the wave's LDS table;
//  stage 2  the transposed tiles (F_I P)^T = P^T F_I^T, so register v of
//           lane l holds X_hat[16 it + l%16][16 jt + 4 (l/16) + v]: four
//           consecutive columns of one row, which meet X loaded as one
//           16-byte buffer load per tile (rows past n_I read zero from past
//           the slab; columns past n_J of the last column tile are masked).
// The tile counts are a template parameter chosen per chunk from the
// tensor's trailing sizes, so small tensors do not pay for the largest.
// Squares are summed in FP32 per lane and slab, then in FP64; each chunk
// writes one (r2, x2) pair and a second kernel sums a tensor's chunks in
// order, so the result does not depend on the schedule's timing.
#include "tk_kernels.hpp"

namespace tk {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kRsrcWord3 = 0x00020000;
constexpr int kPW = kBatchMaxN + 1;   // row stride of the P table (floats)

__device__ __forceinline__ floatx4 mma16(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Four consecutive entries of X in one load: 16 bytes of FP32 or 8 bytes of
// BF16 / FP16, widened to FP32.
template <typename TX> struct Quad;
template <> struct Quad<float> {
  typedef uintx4 raw;
  static __device__ __forceinline__ raw load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(uintx4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  }
  static __device__ __forceinline__ floatx4 widen(raw v) { return __builtin_bit_cast(floatx4, v); }
};
typedef unsigned int uintx2 __attribute__((ext_vector_type(2)));
template <> struct Quad<bf16> {
  typedef uintx2 raw;
  static __device__ __forceinline__ raw load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(uintx2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  }
  static __device__ __forceinline__ floatx4 widen(raw v) {
    return floatx4{__uint_as_float(v[0] << 16), __uint_as_float(v[0] & 0xFFFF0000u), __uint_as_float(v[1] << 16),
                   __uint_as_float(v[1] & 0xFFFF0000u)};
  }
};
template <> struct Quad<f16> {
  typedef uintx2 raw;
  static __device__ __forceinline__ raw load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(uintx2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  }
  static __device__ __forceinline__ floatx4 widen(raw v) {
    return floatx4{(float)__builtin_bit_cast(_Float16, (unsigned short)(v[0] & 0xFFFFu)),
                   (float)__builtin_bit_cast(_Float16, (unsigned short)(v[0] >> 16)),
                   (float)__builtin_bit_cast(_Float16, (unsigned short)(v[1] & 0xFFFFu)),
                   (float)__builtin_bit_cast(_Float16, (unsigned short)(v[1] >> 16))};
  }
};

// per wave: F_I and F_J of the chunk's tensor ([i][k], row stride 17) and the P table
constexpr int kFW = kBatchMaxC + 1;
constexpr int kWaveLds = 2 * kBatchMaxN * kFW + kBatchMaxC * kPW;   // floats

template <typename TX, int NT, int D>
__device__ __forceinline__ void resid_chunk(const BatchTensor& td, const TX* Xp, int64_t a0, int64_t a1, float* wl,
                                            int lane, double& r2, double& x2) {
  typedef typename Quad<TX>::raw raw;
  constexpr uint32_t kB = sizeof(TX);
  const int g = lane >> 4, l16 = lane & 15;
  const int nI = td.nI, nJ = td.nJ, cI = td.cI, cJ = td.cJ;
  const int nTI = (nI + 15) >> 4, nTJ = (nJ + 15) >> 4;
  float(*sFI)[kFW] = reinterpret_cast<float(*)[kFW]>(wl);
  float(*sFJ)[kFW] = reinterpret_cast<float(*)[kFW]>(wl + kBatchMaxN * kFW);
  float(*sP)[kPW] = reinterpret_cast<float(*)[kPW]>(wl + 2 * kBatchMaxN * kFW);
  // the factors of this tensor (zero past n and c); the previous chunk's
  // reads of these tables came first in this wave's program order
  for (int e = lane; e < 16 * NT * 16; e += 64) {
    const int i = e >> 4, k = e & 15;
    sFI[i][k] = (i < nI && k < cI) ? td.FI[i * cI + k] : 0.0f;
    sFJ[i][k] = (i < nJ && k < cJ) ? td.FJ[i * cJ + k] : 0.0f;
  }
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  const uint32_t rowb = (uint32_t)nJ * kB, slab_bytes = (uint32_t)(nI * nJ) * kB;
  // this lane's byte offset of tile (0, jt): row l%16, columns 16 jt + 4 (l/16) ..
  uint32_t coff[NT];
#pragma unroll
  for (int jt = 0; jt < NT; ++jt) {
    const int col = 16 * jt + 4 * g;
    coff[jt] = (jt < nTJ && col < nJ) ? (uint32_t)l16 * rowb + (uint32_t)col * kB : 0x80000000u;
  }
  uintx4 lastmask;
  {
    const int valid = nJ - (16 * (nTJ - 1) + 4 * g);
#pragma unroll
    for (int c = 0; c < 4; ++c) lastmask[c] = c < valid ? 0xFFFFFFFFu : 0u;
  }
  const int cIJ = cI * cJ;
  // T[a] as the stage-1 A operand: lane l gives T[a][l%16][4 ks + l/16]
  uint32_t toff[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int k = 4 * ks + g;
    toff[ks] = (l16 < cI && k < cJ) ? (uint32_t)(l16 * cJ + k) * 4u : 0x80000000u;
  }
  // the loads of one slab (X in the stage-2 layout, its T block); a slab
  // past the chunk gets empty ranges (every load reads zero, no traffic)
  auto issue = [&](int64_t a, raw (&xr)[NT][NT], float (&ta)[4]) {
    const bool live = a < a1;
    const char* xs = reinterpret_cast<const char*>(Xp) + (live ? a : a0) * (int64_t)slab_bytes;
#pragma unroll
    for (int it = 0; it < NT; ++it) {
      // one range per row tile (from its first row to the slab's end), so
      // the lane offsets are the same for every row tile
      const int rt = 16 * it * (int)rowb;
      const bool on = live && it < nTI;
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<char*>(xs) + (on ? rt : 0), (short)0, on ? (int)slab_bytes - rt : 0, kRsrcWord3);
#pragma unroll
      for (int jt = 0; jt < NT; ++jt) xr[it][jt] = Quad<TX>::load(rs, coff[jt]);
    }
    const __amdgpu_buffer_rsrc_t rt = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(td.T) + (live ? a : a0) * cIJ, (short)0, live ? cIJ * 4 : 0, kRsrcWord3);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) ta[ks] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rt, toff[ks], 0, 0));
  };
  // Rank steps, and for up to three tiles the tiles, past the tensor's
  // sizes multiply zeros (X reads zero there and the factor tables are
  // zero-padded), so those multiplies run without tests: a uniform branch per
  // step costs more than the MFMA it would skip.  From four tiles on, the
  // tile tests stay (they also keep the scheduler from hoisting operand
  // reads across tiles, which spills with a whole slab in registers).
  constexpr bool kSkip = NT >= 4;
  auto compute = [&](const raw (&xr)[NT][NT], const float (&ta)[4]) {
    // stage 1: P = T[a] F_J^T (B operand lane l: F_J[16 jt + l%16][4 ks + l/16])
#pragma unroll
    for (int jt = 0; jt < NT; ++jt) {
      if (kSkip && jt >= nTJ) continue;
      float fj[4];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) fj[ks] = sFJ[16 * jt + l16][4 * ks + g];
      floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) acc = mma16(ta[ks], fj[ks], acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) sP[4 * g + v][16 * jt + l16] = acc[v];
    }
    // ordered LDS accesses of one wave: the reads below see the writes
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    // stage 2 and the squares (A operand lane l: P[4 ks + l/16][16 jt + l%16])
    constexpr bool kKeepP = NT <= 4;
    float pv[kKeepP ? NT : 1][4];
    if constexpr (kKeepP) {
#pragma unroll
      for (int jt = 0; jt < NT; ++jt)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) pv[jt][ks] = sP[4 * ks + g][16 * jt + l16];
    }
    float r2t = 0.0f, x2t = 0.0f;
#pragma unroll
    for (int it = 0; it < NT; ++it) {
      if (kSkip && it >= nTI) continue;
      float fi[4];   // B operand lane l: F_I[16 it + l%16][4 ks + l/16]
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) fi[ks] = sFI[16 * it + l16][4 * ks + g];
#pragma unroll
      for (int jt = 0; jt < NT; ++jt) {
        if (kSkip && jt >= nTJ) continue;
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
          acc = mma16(kKeepP ? pv[kKeepP ? jt : 0][ks] : sP[4 * ks + g][16 * jt + l16], fi[ks], acc);
        const floatx4 x = __builtin_bit_cast(
            floatx4, __builtin_bit_cast(uintx4, Quad<TX>::widen(xr[it][jt])) & (jt == nTJ - 1 ? lastmask : ~uintx4{}));
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float d = x[v] - acc[v];
          r2t = fmaf(d, d, r2t);
          x2t = fmaf(x[v], x[v], x2t);
        }
      }
    }
    r2 += (double)r2t;
    x2 += (double)x2t;
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();   // this slab's reads of P precede the next slab's writes
  };
  // D slabs in flight: slot s of a group is multiplied while the loads of
  // the D - 1 slabs after it are pending.  Full groups carry no exit test
  // (one would leave skipped loads pending at the loop head and force a wait
  // for all of them); the tail multiplies the slabs still in flight.
  raw xr[D][NT][NT];
  float ta[D][4];
  int64_t next = a0;
#pragma unroll
  for (int s = 0; s < D - 1; ++s) issue(next++, xr[s], ta[s]);
  int64_t left = a1 - a0;
  for (; left >= D; left -= D) {
#pragma unroll
    for (int s = 0; s < D; ++s) {
      const int ls = (s + D - 1) % D;
      issue(next++, xr[ls], ta[ls]);
      __builtin_amdgcn_sched_barrier(0);
      compute(xr[s], ta[s]);
    }
  }
#pragma unroll
  for (int s = 0; s < D - 1; ++s)
    if (s < left) compute(xr[s], ta[s]);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_wave_barrier();   // the reads of the factor tables precede the next chunk's writes
}

__global__ __launch_bounds__(64 * kWaves, 2) void batch_resid_kernel(const BatchResid br) {
  extern __shared__ float lds[];
  float* wl = lds + (threadIdx.x >> 6) * kWaveLds;
  const int lane = threadIdx.x & 63;
  // chunks handed out by a queue in the plan's order (largest first): a wave
  // takes its next ticket when it starts a chunk, so the ticket's round trip
  // overlaps the chunk's work
  auto take = [&]() {
    int q = 0;
    if (lane == 0) q = atomicAdd(br.queue, 1);
    return __builtin_amdgcn_readfirstlane(q);
  };
  int q = take();
  while (q < br.nchunks) {
    const int qn = take();
    const int cid = wave_uniform(br.order[q]);
    const BatchChunk ch = wave_uniform(br.chunks[cid]);
    const BatchTensor td = wave_uniform(br.tensors[ch.tensor]);
    const int nt = (max(td.nI, td.nJ) + 15) >> 4;
    double r2 = 0.0, x2 = 0.0;
    switch (nt) {
      case 1: resid_chunk<float, 1, 8>(td, td.X, ch.a0, ch.a1, wl, lane, r2, x2); break;
      case 2: resid_chunk<float, 2, 6>(td, td.X, ch.a0, ch.a1, wl, lane, r2, x2); break;
      case 3: resid_chunk<float, 3, 3>(td, td.X, ch.a0, ch.a1, wl, lane, r2, x2); break;
      case 4: resid_chunk<float, 4, 2>(td, td.X, ch.a0, ch.a1, wl, lane, r2, x2); break;
      case 5: resid_chunk<float, 5, 1>(td, td.X, ch.a0, ch.a1, wl, lane, r2, x2); break;
      default: resid_chunk<float, 6, 1>(td, td.X, ch.a0, ch.a1, wl, lane, r2, x2); break;
    }
    for (int o = 32; o > 0; o >>= 1) {
      r2 += __shfl_xor(r2, o);
      x2 += __shfl_xor(x2, o);
    }
    if (lane == 0) {
      br.partials[2 * cid] = r2;
      br.partials[2 * cid + 1] = x2;
    }
    q = qn;
  }
}

__global__ void batch_queue_reset_kernel(int32_t* queue) { *queue = 0; }

// The same pass for one tensor whose trailing modes are at most 64 (the
// small-mode residual of the single-tensor path): chunks of equal slab
// counts taken round-robin by the resident waves (equal costs, so no queue);
// one (r2, x2) pair per wave, summed in wave order by the launcher's kernel.
template <typename TX>
__global__ __launch_bounds__(64 * kWaves, 2) void slab_resid_kernel(const ResidSlab p, int64_t chunk) {
  extern __shared__ float lds[];
  float* wl = lds + (threadIdx.x >> 6) * kWaveLds;
  const int lane = threadIdx.x & 63;
  const int gwave = __builtin_amdgcn_readfirstlane((int)blockIdx.x * kWaves + (int)(threadIdx.x >> 6));
  if (gwave >= p.nwaves) return;   // no workgroup barrier follows
  BatchTensor td{};
  td.FI = p.FI;
  td.FJ = p.FJ;
  td.T = const_cast<float*>(p.T);
  td.A = p.A;
  td.nI = p.nI;
  td.nJ = p.nJ;
  td.cI = p.cI;
  td.cJ = p.cJ;
  const TX* X = static_cast<const TX*>(p.X);
  const int nt = (max(p.nI, p.nJ) + 15) >> 4;
  const int64_t nch = (p.A + chunk - 1) / chunk;
  double r2 = 0.0, x2 = 0.0;
  for (int64_t c = gwave; c < nch; c += p.nwaves) {
    const int64_t a0 = c * chunk, a1 = min(p.A, a0 + chunk);
    switch (nt) {
      case 1: resid_chunk<TX, 1, 8>(td, X, a0, a1, wl, lane, r2, x2); break;
      case 2: resid_chunk<TX, 2, 6>(td, X, a0, a1, wl, lane, r2, x2); break;
      case 3: resid_chunk<TX, 3, 3>(td, X, a0, a1, wl, lane, r2, x2); break;
      default: resid_chunk<TX, 4, 2>(td, X, a0, a1, wl, lane, r2, x2); break;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    r2 += __shfl_xor(r2, o);
    x2 += __shfl_xor(x2, o);
  }
  if (lane == 0) {
    p.partials[2 * gwave] = r2;
    p.partials[2 * gwave + 1] = x2;
  }
}

// one thread per tensor: its chunks' pairs in chunk order
__global__ void batch_resid_sum_kernel(const double* partials, const int32_t* chunk_begin, int32_t count,
                                       double* resid2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  double r2 = 0.0, x2 = 0.0;
  for (int c = chunk_begin[t]; c < chunk_begin[t + 1]; ++c) {
    r2 += partials[2 * c];
    x2 += partials[2 * c + 1];
  }
  resid2[2 * t] = r2;
  resid2[2 * t + 1] = x2;
}

}  // namespace

int batch_resid_waves() {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_resid_kernel, 64 * kWaves,
                                                   kWaves * kWaveLds * sizeof(float)) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  return per_cu * cus * kWaves;
}

bool slab_resid_pipe_supported(int x_dtype, int64_t nI, int64_t nJ) {
  // two-byte entries are read four at a time as 8-byte loads: rows of an
  // even length keep every such load 4-byte aligned
  return nI <= 64 && nJ <= 64 && (x_dtype == TK_F32 || ((x_dtype == TK_BF16 || x_dtype == TK_F16) && nJ % 2 == 0));
}

hipError_t launch_slab_resid_pipe(const ResidSlab& pin, int x_dtype, int max_waves, hipStream_t st) {
  ResidSlab p = pin;
  const int64_t slab = (int64_t)p.nI * p.nJ * (x_dtype == TK_F32 ? 4 : 2);
  const int64_t chunk = std::max<int64_t>(1, (256 << 10) / slab);
  const int64_t nch = ceil_div(p.A, chunk);
  int per_cu = 0;
  const size_t lds = kWaves * kWaveLds * sizeof(float);
  hipError_t e = x_dtype == TK_F32
                     ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, slab_resid_kernel<float>, 64 * kWaves, lds)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, slab_resid_kernel<bf16>, 64 * kWaves, lds);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  // waves: resident ones, at most one per chunk, within the partials the caller sized
  p.nwaves = (int32_t)std::max<int64_t>(1, std::min<int64_t>({(int64_t)per_cu * cus * kWaves, nch, (int64_t)max_waves}));
  const dim3 grid((unsigned)ceil_div(p.nwaves, kWaves));
  switch (x_dtype) {
    case TK_F32: hipLaunchKernelGGL(slab_resid_kernel<float>, grid, dim3(64 * kWaves), lds, st, p, chunk); break;
    case TK_BF16: hipLaunchKernelGGL(slab_resid_kernel<bf16>, grid, dim3(64 * kWaves), lds, st, p, chunk); break;
    default: hipLaunchKernelGGL(slab_resid_kernel<f16>, grid, dim3(64 * kWaves), lds, st, p, chunk); break;
  }
  if (hipError_t e2 = hipGetLastError()) return e2;
  if (p.resid2) return launch_pair_sum(p.partials, p.nwaves, p.resid2, st);
  return hipSuccess;
}

hipError_t launch_batch_resid(const BatchResid& br, hipStream_t st) {
  if (br.count <= 0) return hipSuccess;
  if (br.nwaves > 0) {
    // a fill kernel, not a memset: the run may be captured in a graph
    hipLaunchKernelGGL(batch_queue_reset_kernel, dim3(1), dim3(1), 0, st, br.queue);
    hipLaunchKernelGGL(batch_resid_kernel, dim3((unsigned)ceil_div(br.nwaves, kWaves)), dim3(64 * kWaves),
                       kWaves * kWaveLds * sizeof(float), st, br);
    if (hipError_t e = hipGetLastError()) return e;
  }
  hipLaunchKernelGGL(batch_resid_sum_kernel, dim3((unsigned)ceil_div(br.count, 256)), dim3(256), 0, st,
                     br.partials, br.tensor_chunk_begin, br.count, br.resid2);
  return hipGetLastError();
}

}  // namespace tk
