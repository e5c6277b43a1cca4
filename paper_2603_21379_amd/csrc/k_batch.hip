// Batching form of the core projection (Algorithm 1, core step) for many
// FP32 tensors of uneven order and size in one launch per step.
//
// batch_slab_kernel: the streaming pass of every tensor, T[a] = F_I^T X[a] F_J
//   for the slabs X[a] of its two trailing modes (n <= 96, ranks <= 16), on
//   v_mfma_f32_16x16x4f32 exactly as the single-tensor small-mode pass.  The
//   work is a list of chunks (tensor, slab range) that the resident waves
//   take from a queue, largest first, so the waves finish together (the
//   counter is cleared by a one-thread kernel before each pass, so runs can
//   be replayed from a graph).  A wave keeps its tensor's F_J in registers
//   and F_I^T in its own LDS region, reloading both when its next chunk
//   belongs to another tensor.
//
// batch_mode_kernel: one remaining mode of every tensor that still has one,
//   out[a][p][b] = sum_q F[q][p] in[a][q][b], as the single-tensor MFMA mode
//   contraction; each descriptor's units are padded to whole workgroups so a
//   workgroup shares one F^T table.  The same kernel expands a core back over
//   a mode (F read transposed, 32 output rows per descriptor).
#include "tk_kernels.hpp"

namespace tk {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kRsrcWord3 = 0x00020000;
constexpr int NK = 6;      // 16-column chunks (n_J <= 96)
constexpr int NT = 6;      // 16-row tiles (n_I <= 96)

__device__ __forceinline__ floatx4 mma_f32(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int TG, int NBUF>
__global__ __launch_bounds__(256, 2) void batch_slab_kernel(const BatchSlab bs) {
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63, g = lane >> 4, l16 = lane & 15;
  const int wv = threadIdx.x >> 6;
  float* sA = lds + wv * (NT * 256);   // this wave's F_I^T table [t][v][lane]
  // chunks from the queue, largest first; the next ticket is taken when a
  // chunk starts, so its round trip overlaps the chunk
  auto take = [&]() {
    int q = 0;
    if (lane == 0) q = atomicAdd(bs.queue, 1);
    return __builtin_amdgcn_readfirstlane(q);
  };

  int cur_tensor = -1;
  float fj[NK][4];
  uintx4 lastmask;
  BatchTensor td{};
  int nT = 0, nK = 0;
  uint32_t lane_off = 0, tile_bytes = 0, slab_bytes = 0;

  int qt = take();
  while (qt < bs.nchunks) {
    const int qnext = take();
    const BatchChunk ch = wave_uniform(bs.chunks[wave_uniform(bs.order[qt])]);
    const int tid = ch.tensor;
    if (tid != cur_tensor) {
      cur_tensor = tid;
      td = wave_uniform(bs.tensors[tid]);
      nT = (td.nI + 15) / 16;
      nK = (td.nJ + 15) / 16;
#pragma unroll
      for (int kc = 0; kc < NK; ++kc)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int b = 16 * kc + 4 * g + c;
          fj[kc][c] = (b < td.nJ && l16 < td.cJ) ? td.FJ[b * td.cJ + l16] : 0.0f;
        }
      const int valid = td.nJ - ((nK - 1) * 16 + 4 * g);
#pragma unroll
      for (int w = 0; w < 4; ++w) lastmask[w] = w < valid ? 0xFFFFFFFFu : 0u;
      // the wave's own table: ordered LDS accesses of one wave need no barrier
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * t + 4 * g + v;
          sA[t * 256 + v * 64 + lane] = (i < td.nI && l16 < td.cI) ? td.FI[i * td.cI + l16] : 0.0f;
        }
      __builtin_amdgcn_wave_barrier();
      lane_off = (uint32_t)(l16 * td.nJ + 4 * g) * 4u;
      tile_bytes = (uint32_t)(16 * td.nJ) * 4u;
      slab_bytes = (uint32_t)td.nI * (uint32_t)td.nJ * 4u;
    }
    const int nG = (nT + TG - 1) / TG;
    const char* Xb = reinterpret_cast<const char*>(td.X);

    auto load_unit = [&](int64_t a, int grp, uintx4 (&buf)[TG][NK]) {
      const bool live = a >= 0;
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<char*>(Xb + (live ? a : 0) * (int64_t)slab_bytes), (short)0, live ? (int)slab_bytes : 0,
          kRsrcWord3);
      // the same TG NK loads in every unit (tiles past n_T and chunks past
      // n_K read zero from past the range): the waits before the multiplies
      // then count loads instead of waiting for all of them
#pragma unroll
      for (int tt = 0; tt < TG; ++tt) {
        const int t = grp * TG + tt;
        const uint32_t off = lane_off + t * tile_bytes;
#pragma unroll
        for (int kc = 0; kc < NK; ++kc) {
          const uint32_t o = (t < nT && kc < nK) ? off + kc * 64 : 0x80000000u;
          buf[tt][kc] = __builtin_bit_cast(uintx4, __builtin_amdgcn_raw_buffer_load_b128(rs, o, 0, 2));
        }
      }
    };
    floatx4 tacc = floatx4{};
    // Output staging: the partial cores of consecutive slabs are contiguous
    // (T + a c_I c_J), so runs of them collect in this wave's 4 KB LDS block
    // and are written as 16-byte pieces (four stores per 1024 values instead
    // of four per slab).  Needs c_I c_J divisible by 4 (16-byte alignment).
    const int cIJ = td.cI * td.cJ;
    const bool staged = (cIJ & 3) == 0;
    float* so = lds + kWaves * (NT * 256) + wv * 1024;
    int64_t sa0 = 0;
    int sn = 0;
    auto flush = [&]() {
      if (sn == 0) return;
      // ordered LDS accesses of one wave: the reads below see the writes
      __builtin_amdgcn_wave_barrier();
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      const int nf = sn * cIJ;
      const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(
          td.T + sa0 * cIJ, (short)0, nf * 4, kRsrcWord3);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int f = (u * 64 + lane) * 4;
        const floatx4 w = *reinterpret_cast<const floatx4*>(so + f);
        const uint32_t o = f < nf ? (uint32_t)(f * 4) : 0x80000000u;
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uintx4, w), ro, o, 0, kOutStorePolicy);
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      __builtin_amdgcn_wave_barrier();
      sn = 0;
    };
    auto compute_unit = [&](int64_t a, int grp, uintx4 (&buf)[TG][NK]) {
#pragma unroll
      for (int tt = 0; tt < TG; ++tt) {
        const int t = grp * TG + tt;
        if (t >= nT) continue;
        floatx4 acc = floatx4{};
#pragma unroll
        for (int kc = 0; kc < NK; ++kc) {
          if (kc >= nK) continue;
          uintx4 x = buf[tt][kc];
          if (kc == nK - 1) x &= lastmask;
          const floatx4 xf = __builtin_bit_cast(floatx4, x);
#pragma unroll
          for (int c = 0; c < 4; ++c) acc = mma_f32(xf[c], fj[kc][c], acc);
        }
        const float* A = sA + t * 256 + lane;
#pragma unroll
        for (int v = 0; v < 4; ++v) tacc = mma_f32(A[v * 64], acc[v], tacc);
      }
      if (grp != nG - 1) return;
      if (staged) {
        // slab complete: its c_I x c_J block goes to this wave's LDS block
        // after the previous slabs of the run; a full block is written out
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int jp = 4 * g + v;
          if (jp < td.cI && l16 < td.cJ) so[sn * cIJ + jp * td.cJ + l16] = tacc[v];
        }
        if (sn == 0) sa0 = a;
        sn = sn + 1;
        if ((sn + 1) * cIJ > 1024) flush();
      } else {
        const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(
            td.T + a * td.cI * td.cJ, (short)0, td.cI * td.cJ * 4, kRsrcWord3);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int jp = 4 * g + v;
          const uint32_t off = (jp < td.cI && l16 < td.cJ) ? (uint32_t)((jp * td.cJ + l16) * 4) : 0x80000000u;
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(tacc[v]), ro, off, 0, kOutStorePolicy);
        }
      }
      tacc = floatx4{};
    };

    // units (slab a, tile group) of this chunk through NBUF rotating buffers
    uintx4 buf[NBUF][TG][NK];
    int64_t ua[NBUF];
    int ug[NBUF];
    int64_t la = ch.a0;
    int lg = 0;
    auto advance = [&]() {
      if (la < 0) return;
      if (++lg >= nG) {
        lg = 0;
        la = la + 1 < ch.a1 ? la + 1 : -1;
      }
    };
    ua[0] = la;
    ug[0] = lg;
    load_unit(la, lg, buf[0]);
#pragma unroll
    for (int s = 1; s < NBUF - 1; ++s) {
      advance();
      ua[s] = la;
      ug[s] = lg;
      load_unit(la, lg, buf[s]);
    }
    // full groups of NBUF units with no exit test inside (one there would
    // leave loads of skipped units pending at the loop head and force a wait
    // for every load in flight); the tail multiplies the units in flight
    int left = (int)(ch.a1 - ch.a0) * nG;
    for (; left >= NBUF; left -= NBUF) {
#pragma unroll
      for (int s = 0; s < NBUF; ++s) {
        const int lb = (s + NBUF - 1) % NBUF;
        advance();
        ua[lb] = la;
        ug[lb] = lg;
        load_unit(la, lg, buf[lb]);
        __builtin_amdgcn_sched_barrier(0);
        compute_unit(ua[s], ug[s], buf[s]);
      }
    }
#pragma unroll
    for (int s = 0; s < NBUF - 1; ++s)
      if (s < left) compute_unit(ua[s], ug[s], buf[s]);
    flush();
    qt = qnext;
  }
}

__global__ void batch_slab_queue_reset_kernel(int32_t* queue) { *queue = 0; }

// Whole-slab form of the streaming pass: a wave keeps D slabs of a chunk in
// flight (X of a slab in registers as one 16-byte load per 16 x 16 tile:
// row 16 it + l%16, columns 16 jt + 4 (l/16) .. + 3), so small slabs put as
// many bytes in flight as large ones.  Per slab, on v_mfma_f32_16x16x4f32:
//   stage A  (X F_J) of row tile it: the four values of a load are the
//            A operands of four K steps (K index l/16 stands for column
//            16 jt + 4 (l/16) + c of step c), F_J[16 jt + 4 (l/16) + c][l%16]
//            the B operands;
//   stage B  T += F_I^T (X F_J): register v of the stage-A result (row
//            16 it + 4 (l/16) + v) is the B operand of K step v, with
//            F_I[16 it + 4 (l/16) + v][l%16] as the A operand.
// Columns past n_J of the last column tile hold the next row's values (or
// zero past the slab): they meet zero rows of F_J, so no mask is needed.
// The factor operands live in registers (reloaded per chunk); no LDS.
template <int NT, int D>
__device__ __forceinline__ void core_chunk(const BatchTensor& td, int64_t a0, int64_t a1, int lane, float* so) {
  const int g = lane >> 4, l16 = lane & 15;
  const int nI = td.nI, nJ = td.nJ, cI = td.cI, cJ = td.cJ;
  const int nTI = (nI + 15) >> 4, nTJ = (nJ + 15) >> 4;
  constexpr bool kSkip = NT >= 4;   // tile tests: see the residual pass
  float fj[NT][4], fi[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int r = 16 * t + 4 * g + c;
      fj[t][c] = (r < nJ && l16 < cJ) ? td.FJ[r * cJ + l16] : 0.0f;
      fi[t][c] = (r < nI && l16 < cI) ? td.FI[r * cI + l16] : 0.0f;
    }
  const uint32_t rowb = (uint32_t)nJ * 4u, slab_bytes = (uint32_t)(nI * nJ) * 4u;
  uint32_t coff[NT];
#pragma unroll
  for (int jt = 0; jt < NT; ++jt) {
    const int col = 16 * jt + 4 * g;
    coff[jt] = (jt < nTJ && col < nJ) ? (uint32_t)l16 * rowb + (uint32_t)col * 4u : 0x80000000u;
  }
  const int cIJ = cI * cJ;
  auto issue = [&](int64_t a, uintx4 (&xr)[NT][NT]) {
    const bool live = a < a1;
    const char* xs = reinterpret_cast<const char*>(td.X) + (live ? a : a0) * (int64_t)slab_bytes;
#pragma unroll
    for (int it = 0; it < NT; ++it) {
      // one range per row tile (from its first row to the slab's end)
      const int rt = 16 * it * (int)rowb;
      const bool on = live && it < nTI;
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<char*>(xs) + (on ? rt : 0), (short)0, on ? (int)slab_bytes - rt : 0, kRsrcWord3);
#pragma unroll
      for (int jt = 0; jt < NT; ++jt)
        xr[it][jt] = __builtin_bit_cast(uintx4, __builtin_amdgcn_raw_buffer_load_b128(rs, coff[jt], 0, 0));
    }
  };
  // Output staging: the partial cores of consecutive slabs are contiguous, so
  // runs of them collect in the wave's LDS block and leave as contiguous
  // stores: 16 bytes per lane when c_I c_J is a multiple of 4, else 4 bytes
  // per lane of consecutive floats (storing each tile entry in place filled
  // only part of each 64-byte segment for rows of c_J < 16 floats: 1.5x the
  // bytes of T in writes).
  constexpr int kStage = 1024;
  const bool quads = (cIJ & 3) == 0;
  int64_t sa0 = 0;
  int sn = 0;
  auto flush = [&]() {
    if (sn == 0) return;
    __builtin_amdgcn_wave_barrier();   // ordered LDS accesses of one wave: the reads see the writes
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    const int nf = sn * cIJ;
    const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(td.T + sa0 * cIJ, (short)0, nf * 4, kRsrcWord3);
    if (quads) {
#pragma unroll
      for (int u = 0; u < kStage / 256; ++u) {
        const int f = (u * 64 + lane) * 4;
        const floatx4 w = *reinterpret_cast<const floatx4*>(so + f);
        const uint32_t o = f < nf ? (uint32_t)(f * 4) : 0x80000000u;
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uintx4, w), ro, o, 0, kOutStorePolicy);
      }
    } else {
#pragma unroll 2
      for (int u = 0; u < kStage / 64; ++u) {
        const int f = u * 64 + lane;
        const uint32_t o = f < nf ? (uint32_t)(f * 4) : 0x80000000u;
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(so[f]), ro, o, 0, kOutStorePolicy);
      }
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();   // the reads precede the next run's writes
    sn = 0;
  };
  auto compute = [&](int64_t a, const uintx4 (&xr)[NT][NT]) {
    floatx4 tacc = floatx4{};
#pragma unroll
    for (int it = 0; it < NT; ++it) {
      if (kSkip && it >= nTI) continue;
      floatx4 acc = floatx4{};
#pragma unroll
      for (int jt = 0; jt < NT; ++jt) {
        if (kSkip && jt >= nTJ) continue;
        const floatx4 x = __builtin_bit_cast(floatx4, xr[it][jt]);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc = mma_f32(x[c], fj[jt][c], acc);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) tacc = mma_f32(fi[it][v], acc[v], tacc);
    }
    // the slab's c_I x c_J block after the run's previous ones in this
    // wave's LDS block; a full block goes out as contiguous stores
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int pr = 4 * g + v;
      if (pr < cI && l16 < cJ) so[sn * cIJ + pr * cJ + l16] = tacc[v];
    }
    if (sn == 0) sa0 = a;
    ++sn;
    if ((sn + 1) * cIJ > kStage) flush();
  };
  uintx4 xr[D][NT][NT];
  int64_t next = a0, cur = a0;
#pragma unroll
  for (int s = 0; s < D - 1; ++s) issue(next++, xr[s]);
  int64_t left = a1 - a0;
  for (; left >= D; left -= D) {
#pragma unroll
    for (int s = 0; s < D; ++s) {
      issue(next++, xr[(s + D - 1) % D]);
      __builtin_amdgcn_sched_barrier(0);
      compute(cur++, xr[s]);
    }
  }
#pragma unroll
  for (int s = 0; s < D - 1; ++s)
    if (s < left) compute(cur++, xr[s]);
  flush();
}

__global__ __launch_bounds__(256, 2) void batch_core_pipe_kernel(const BatchSlab bs) {
  __shared__ float sOut[kWaves][1024];   // each wave's output staging block
  const int lane = threadIdx.x & 63;
  float* so = sOut[threadIdx.x >> 6];
  auto take = [&]() {
    int q = 0;
    if (lane == 0) q = atomicAdd(bs.queue, 1);
    return __builtin_amdgcn_readfirstlane(q);
  };
  int qt = take();
  while (qt < bs.nchunks) {
    const int qnext = take();
    const BatchChunk ch = wave_uniform(bs.chunks[wave_uniform(bs.order[qt])]);
    const BatchTensor td = wave_uniform(bs.tensors[ch.tensor]);
    switch ((max(td.nI, td.nJ) + 15) >> 4) {
      case 1: core_chunk<1, 8>(td, ch.a0, ch.a1, lane, so); break;
      case 2: core_chunk<2, 6>(td, ch.a0, ch.a1, lane, so); break;
      case 3: core_chunk<3, 3>(td, ch.a0, ch.a1, lane, so); break;
      case 4: core_chunk<4, 2>(td, ch.a0, ch.a1, lane, so); break;
      case 5: core_chunk<5, 1>(td, ch.a0, ch.a1, lane, so); break;
      default: core_chunk<6, 1>(td, ch.a0, ch.a1, lane, so); break;
    }
    qt = qnext;
  }
}

// ---------------------------------------------------------------- remaining modes
constexpr int kCols = 128;
constexpr int kKB = 8;

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(256) void batch_mode_kernel(const BatchMode bm) {
  extern __shared__ float sF[];   // [Qp][32]
  const int64_t u0 = (int64_t)blockIdx.x * kWaves;
  // descriptor of this workgroup (unit ranges are padded to whole workgroups)
  int lo = 0, hi = bm.count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bm.descs[mid].unit_begin <= u0) lo = mid; else hi = mid - 1;
  }
  const BatchModeDesc m = wave_uniform(bm.descs[wave_uniform(lo)]);
  const int Qp = (int)((m.Q + 2 * kKB - 1) / (2 * kKB)) * 2 * kKB;
  for (int e = threadIdx.x; e < Qp * 32; e += blockDim.x) {
    const int q = e >> 5, p = e & 31;
    sF[e] = (q < m.Q && p < m.P) ? m.F[m.ftrans ? (int64_t)p * m.Q + q : (int64_t)q * m.P + p] : 0.0f;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, kh = lane >> 5, l32 = lane & 31;
  const int64_t nBb = (m.B + kCols - 1) / kCols;
  const int64_t unit = wave_uniform(u0 + (threadIdx.x >> 6) - m.unit_begin);
  if (unit >= m.A * nBb) return;  // no barrier follows
  const int64_t a = unit / nBb;
  const int64_t b0 = (unit - a * nBb) * kCols;
  const int64_t slab = m.Q * m.B;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(m.in + a * slab), (short)0, (int)(slab * 4), kRsrcWord3);
  const int64_t b = b0 + 4 * l32;
  const bool colok = b < m.B;
  const uint32_t rowb = (uint32_t)(m.B * 4);
  floatx16 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = floatx16{};
  auto load = [&](int q0, floatx4 (&buf)[kKB]) {
#pragma unroll
    for (int u = 0; u < kKB; ++u) {
      const int q = q0 + 2 * u + kh;
      const uint32_t off = (colok && q < m.Q) ? (uint32_t)q * rowb + (uint32_t)(b * 4) : 0x80000000u;
      buf[u] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
    }
  };
  auto compute = [&](int q0, const floatx4 (&buf)[kKB]) {
    const float* f = sF + (q0 + kh) * 32 + l32;
#pragma unroll
    for (int u = 0; u < kKB; ++u) {
      const float fv = f[u * 64];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = mfma32(fv, buf[u][c], acc[c]);
    }
  };
  // double buffered as the single-tensor mode contraction (loads past Q read
  // zero, so every step issues the next batch before multiplying)
  const int nb = Qp / (2 * kKB);
  floatx4 bufA[kKB], bufB[kKB];
  load(0, bufA);
  int bq = 0;
  for (; bq + 2 <= nb; bq += 2) {
    load((bq + 1) * 2 * kKB, bufB);
    __builtin_amdgcn_sched_barrier(0);
    compute(bq * 2 * kKB, bufA);
    load((bq + 2) * 2 * kKB, bufA);
    __builtin_amdgcn_sched_barrier(0);
    compute((bq + 1) * 2 * kKB, bufB);
  }
  if (bq < nb) compute(bq * 2 * kKB, bufA);
  if (!colok) return;
  float* out = m.out + a * m.out_slab;
  const int ncol = (int)min<int64_t>(4, m.B - b);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int p = 8 * (v >> 2) + 4 * kh + (v & 3);
    if (p >= m.P) continue;
    float* o = out + (int64_t)p * m.B + b;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < ncol) o[c] = acc[c][v];
  }
}

}  // namespace

// per wave: the F_I^T table and a 1024-value output staging block
size_t batch_slab_lds_bytes() { return (size_t)kWaves * (NT * 256 + 1024) * sizeof(float); }

int batch_slab_waves(int tg, int nbuf) {
  int per_cu = 0;
  const size_t lds = batch_slab_lds_bytes();
  hipError_t e = hipErrorInvalidValue;
  if (tg == 1 && nbuf == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_slab_kernel<1, 2>, 256, lds);
  if (tg == 2 && nbuf == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_slab_kernel<2, 2>, 256, lds);
  if (tg == 1 && nbuf == 3) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_slab_kernel<1, 3>, 256, lds);
  if (tg == 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_core_pipe_kernel, 256, 0);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  return per_cu * cus * kWaves;
}

hipError_t launch_batch_slab(const BatchSlab& bs, int tg, int nbuf, hipStream_t st) {
  if (bs.nwaves <= 0 || bs.nchunks <= 0) return hipSuccess;
  // a fill kernel, not a memset: the run may be captured in a graph
  hipLaunchKernelGGL(batch_slab_queue_reset_kernel, dim3(1), dim3(1), 0, st, bs.queue);
  const dim3 grid((unsigned)ceil_div(bs.nwaves, kWaves));
  const size_t lds = batch_slab_lds_bytes();
  if (tg == 0 && nbuf == 0) hipLaunchKernelGGL(batch_core_pipe_kernel, grid, dim3(256), 0, st, bs);
  else if (tg == 1 && nbuf == 2) hipLaunchKernelGGL((batch_slab_kernel<1, 2>), grid, dim3(256), lds, st, bs);
  else if (tg == 2 && nbuf == 2) hipLaunchKernelGGL((batch_slab_kernel<2, 2>), grid, dim3(256), lds, st, bs);
  else if (tg == 1 && nbuf == 3) hipLaunchKernelGGL((batch_slab_kernel<1, 3>), grid, dim3(256), lds, st, bs);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

int64_t batch_mode_units(int64_t A, int64_t B) {
  return ceil_div(A * ceil_div(B, kCols), kWaves) * kWaves;
}

size_t batch_mode_lds_bytes(int64_t Qmax) {
  return (size_t)((Qmax + 2 * kKB - 1) / (2 * kKB) * 2 * kKB) * 32 * sizeof(float);
}

hipError_t launch_batch_mode(const BatchMode& bm, int64_t total_units, int64_t Qmax, hipStream_t st) {
  if (total_units == 0 || bm.count == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_mode_kernel, dim3((unsigned)(total_units / kWaves)), dim3(256),
                     batch_mode_lds_bytes(Qmax), st, bm);
  return hipGetLastError();
}

}  // namespace tk
