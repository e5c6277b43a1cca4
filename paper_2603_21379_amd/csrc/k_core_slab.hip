// Streaming pass of the core projection (Algorithm 1, core step) for
// tensors whose trailing modes are small (n <= 128, ranks <= 16), on 16x16
// MFMA tiles:
//   T[a] = F_I^T X[a] F_J                    (two trailing modes), or
//   T3[r] = sum_h F_H[h] (x) F_I^T X[r,h] F_J  (three, accumulated over h)
// for BF16, FP16 and FP32 tensors.  The remaining modes are contracted
// afterwards from T (FP32).
//
// Precision form (BF16/FP16 tensors): X enters the MFMA as stored; every
// FP32 operand (the factors, and the stage-1 result D) enters as a hi + lo
// pair of 16-bit values, hi = round(x), lo = round(x - hi), so the products
// carry about 16 significant bits of the FP32 operand instead of 8 (BF16) or
// 11 (FP16); accumulation is FP32.  Stage 2 uses BF16 pairs whatever the
// tensor dtype (D may exceed the FP16 range).
//
// Stage 1, D[i][j] = sum_b X[a][i][b] F_J[b][j], one 16-row tile of i at a
// time (a "unit"): lane l loads 16 bytes of row 16 t + l%16,
//   16-bit: 8 values at columns 32 kc + 8 (l/16) .. +7, v_mfma_f32_16x16x32,
//   FP32:   4 values at columns 16 kc + 4 (l/16) .. +3, each component one
//           v_mfma_f32_16x16x4f32 (A = X[i][k], k <-> column 16 kc + 4 k + c),
// with F_J as the B operand from registers.
// Stage 2, T[j'][j] = sum_i F_I[i][j'] D[i][j]: the stage-1 accumulator (lane
// l holds D[16 t + 4 (l/16) + v][l%16]) is the B operand as it stands:
//   FP32: four K = 4 steps, K <-> rows 16 t + 4 k + v;
//   16-bit: the accumulators of tiles 2 tp and 2 tp + 1 form one K = 32 step,
//           K slots (l/16, v) <-> rows 32 tp + 4 (l/16) + v (v < 4) and
//           32 tp + 16 + 4 (l/16) + v - 4 (v >= 4);
// with F_I^T as the A operand, staged in LDS in that order.
//
// Rows past n_I load zero through the buffer range check (the descriptor
// spans one slab); columns past n_J are zeroed in registers and meet zero
// factor rows.  Waves are persistent over work items (slabs, or runs of n_H
// slabs when the third mode is accumulated), with NBUF units of loads in
// flight.
#include <stdlib.h>

#include <type_traits>

#include "tk_kernels.hpp"

namespace tk {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kRsrcWord3 = 0x00020000;
constexpr int kMaxC = 16;

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

// hi/lo split of eight FP32 values into BF16 vectors: hi = RNE(x) (one
// v_cvt_pk_bf16_f32 per pair), lo = RNE(x - hi)
__device__ __forceinline__ void split_bf16(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
  uintx4 h, l;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const floatx2 v = {x[2 * w], x[2 * w + 1]};
    const uint32_t hb = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
    const floatx2 r = {v[0] - __uint_as_float(hb << 16), v[1] - __uint_as_float(hb & 0xFFFF0000u)};
    h[w] = hb;
    l[w] = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf16x2));
  }
  hi = __builtin_bit_cast(bf16x8, h);
  lo = __builtin_bit_cast(bf16x8, l);
}

template <typename TX> struct Lp;
template <> struct Lp<bf16> {
  typedef bf16x8 vec;
  static __device__ __forceinline__ void split(const float (&x)[8], vec& hi, vec& lo) {
    split_bf16(x, hi, lo);
  }
  static __device__ __forceinline__ floatx4 mma(vec a, vec b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct Lp<f16> {
  typedef halfx8 vec;
  static __device__ __forceinline__ void split(const float (&x)[8], vec& hi, vec& lo) {
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const _Float16 h = (_Float16)x[v];
      hi[v] = h;
      lo[v] = (_Float16)(x[v] - (float)h);
    }
  }
  static __device__ __forceinline__ floatx4 mma(vec a, vec b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

__device__ __forceinline__ floatx4 mma_bf16(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mma_f32(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// TX: float, bf16 or f16.  NK: column chunks of stage 1 (32 columns for
// 16-bit, 16 for FP32), NT: row tiles (16 rows), both upper bounds of the
// runtime sizes.  H3: accumulate the third trailing mode.
// two workgroups per CU, except for the FP32 forms with the third mode and
// six or more K chunks, whose registers do not fit 256 (one, without spills)
template <typename TX, int NK, int NT, int TG, bool H3, int NBUF>
__global__ __launch_bounds__(256, (sizeof(TX) == 4 && H3 && NK >= 6) ? 1 : 2) void core_slab_kernel(
    const CoreSlab p) {
  constexpr bool kF32 = sizeof(TX) == 4;
  constexpr int kChunk = kF32 ? 16 : 32;      // columns per chunk
  constexpr int kPer = kF32 ? 4 : 8;          // values per lane per chunk
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63, g = lane >> 4, l16 = lane & 15;
  const int nT = (p.nI + 15) / 16;
  const int nK = (p.nJ + kChunk - 1) / kChunk;

  // F_I^T in the A-operand order of stage 2, per lane
  //   FP32:   sA[t][v][lane] = F_I[16 t + 4 g + v][l16]
  //   16-bit: sAh/sAl[tp][lane][8] (BF16 pairs), rows as in the header
  float* sA = lds;
  uint32_t* sAh = reinterpret_cast<uint32_t*>(lds);
  uint32_t* sAl = sAh + (NT / 2 + 1) * 64 * 4;
  if constexpr (kF32) {
    for (int e = threadIdx.x; e < NT * 4 * 64; e += blockDim.x) {
      const int t = e / 256, v = (e / 64) & 3, ln = e & 63;
      const int i = 16 * t + 4 * (ln >> 4) + v, j = ln & 15;
      sA[e] = (i < p.nI && j < p.cI) ? p.FI[i * p.cI + j] : 0.0f;
    }
  } else {
    for (int e = threadIdx.x; e < (NT / 2 + 1) * 64; e += blockDim.x) {
      const int tp = e / 64, ln = e & 63, gg = ln >> 4, j = ln & 15;
      float x[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int i = 32 * tp + (v < 4 ? 4 * gg + v : 16 + 4 * gg + v - 4);
        x[v] = (i < p.nI && j < p.cI) ? p.FI[i * p.cI + j] : 0.0f;
      }
      bf16x8 hi, lo;
      split_bf16(x, hi, lo);
      const uintx4 uh = __builtin_bit_cast(uintx4, hi), ul = __builtin_bit_cast(uintx4, lo);
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        sAh[e * 4 + w] = uh[w];
        sAl[e * 4 + w] = ul[w];
      }
    }
  }
  // F_H (n_H x c_H, rows padded to kMaxC) after the A tables
  float* sFH = lds + (kF32 ? NT * 256 : (NT / 2 + 1) * 64 * 4 * 2);
  if (H3)
    for (int e = threadIdx.x; e < p.nH * kMaxC; e += blockDim.x) {
      const int h = e / kMaxC, q = e % kMaxC;
      sFH[e] = q < p.cH ? p.FH[h * p.cH + q] : 0.0f;
    }
  __syncthreads();

  const int gwave = __builtin_amdgcn_readfirstlane((int)blockIdx.x * kWaves + (threadIdx.x >> 6));
  const int nwaves = p.nwaves;
  const int items = (int)p.items;
  if (gwave >= items) return;  // no barrier follows

  // F_J as the B operand of stage 1, in registers
  float fj32[NK][4];
  typename Lp<typename std::conditional<kF32, bf16, TX>::type>::vec fjh[NK], fjl[NK];
#pragma unroll
  for (int kc = 0; kc < NK; ++kc) {
    if constexpr (kF32) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int b = 16 * kc + 4 * g + c;
        fj32[kc][c] = (b < p.nJ && l16 < p.cJ) ? p.FJ[b * p.cJ + l16] : 0.0f;
      }
    } else {
      float x[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int b = 32 * kc + 8 * g + v;
        x[v] = (b < p.nJ && l16 < p.cJ) ? p.FJ[b * p.cJ + l16] : 0.0f;
      }
      Lp<typename std::conditional<kF32, bf16, TX>::type>::split(x, fjh[kc], fjl[kc]);
    }
  }
  // columns of the last chunk past n_J are cleared (dword masks: two 16-bit
  // values or one FP32 value per dword)
  uintx4 lastmask;
  {
    const int valid = p.nJ - ((nK - 1) * kChunk + kPer * g);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      if constexpr (kF32) {
        lastmask[w] = w < valid ? 0xFFFFFFFFu : 0u;
      } else {
        lastmask[w] = 2 * w + 1 < valid ? 0xFFFFFFFFu : (2 * w < valid ? 0x0000FFFFu : 0u);
      }
    }
  }

  const int nH = H3 ? p.nH : 1;
  const uint32_t slab_bytes = (uint32_t)p.nI * (uint32_t)p.nJ * (uint32_t)sizeof(TX);
  // lane part of every load offset (row l16 of a tile, column kPer g); tiles
  // add 16 rows, chunks an immediate; rows past n_I fall past the slab
  const uint32_t lane_off = (uint32_t)(l16 * p.nJ + kPer * g) * (uint32_t)sizeof(TX);
  const uint32_t tile_bytes = (uint32_t)(16 * p.nJ) * (uint32_t)sizeof(TX);
  const char* Xb = static_cast<const char*>(p.X);

  // one unit = TG tiles (group grp) of slab (item, h); item = -1 past the end
  const int nG = (nT + TG - 1) / TG;
  auto load_unit = [&](int item, int h, int grp, uintx4 (&buf)[TG][NK]) {
    item = __builtin_amdgcn_readfirstlane(item);
    h = __builtin_amdgcn_readfirstlane(h);
    grp = __builtin_amdgcn_readfirstlane(grp);
    const bool live = item >= 0;
    const int64_t slab = live ? (int64_t)item * nH + h : 0;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char*>(Xb + slab * slab_bytes), (short)0, live ? (int)slab_bytes : 0, kRsrcWord3);
    // every unit issues the same TG NK loads (tiles past n_T and chunks past
    // n_K read zero from past the range), so the waits before the multiplies
    // count loads instead of waiting for all of them
#pragma unroll
    for (int tt = 0; tt < TG; ++tt) {
      const int t = grp * TG + tt;
      const uint32_t off = lane_off + t * tile_bytes;
#pragma unroll
      for (int kc = 0; kc < NK; ++kc) {
        const uint32_t o = (t < nT && kc < nK) ? off + kc * kChunk * (uint32_t)sizeof(TX) : 0x80000000u;
        buf[tt][kc] = __builtin_bit_cast(uintx4, __builtin_amdgcn_raw_buffer_load_b128(rs, o, 0, 2));
      }
    }
  };

  floatx4 acc3[H3 ? kMaxC : 1];
#pragma unroll
  for (int q = 0; q < (H3 ? kMaxC : 1); ++q) acc3[q] = floatx4{};

  floatx4 tacc = floatx4{};
  auto compute_unit = [&](int item, int h, int grp, uintx4 (&buf)[TG][NK]) {
    floatx4 accE = floatx4{};
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
        if constexpr (kF32) {
          const floatx4 xf = __builtin_bit_cast(floatx4, x);
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) acc = mma_f32(xf[cc], fj32[kc][cc], acc);
        } else {
          typedef Lp<typename std::conditional<kF32, bf16, TX>::type> L;
          const typename L::vec xv = __builtin_bit_cast(typename L::vec, x);
          acc = L::mma(xv, fjh[kc], acc);
          acc = L::mma(xv, fjl[kc], acc);
        }
      }
      if constexpr (kF32) {
        const float* a = sA + t * 256 + lane;
#pragma unroll
        for (int v = 0; v < 4; ++v) tacc = mma_f32(a[v * 64], acc[v], tacc);
      } else {
        // tiles pair up into one K = 32 step (an odd last tile pairs with zero)
        const bool even = (tt & 1) == 0;
        if (even && t + 1 < nT) {
          accE = acc;
        } else {
          float d[8];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            d[v] = even ? acc[v] : accE[v];
            d[4 + v] = even ? 0.0f : acc[v];
          }
          bf16x8 dh, dl;
          split_bf16(d, dh, dl);
          const int tp = t >> 1;
          const bf16x8 ah = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uintx4*>(sAh + (tp * 64 + lane) * 4));
          const bf16x8 al = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uintx4*>(sAl + (tp * 64 + lane) * 4));
          tacc = mma_bf16(ah, dh, tacc);
          tacc = mma_bf16(al, dh, tacc);
          tacc = mma_bf16(ah, dl, tacc);
        }
      }
    }
    if (grp != nG - 1) return;
    // slab complete: lane holds T[j' = 4 g + v][j = l16]; lanes outside
    // (c_I, c_J) store past the range, which discards them
    uint32_t off[4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
      off[v] = (4 * g + v < p.cI && l16 < p.cJ) ? (uint32_t)(((4 * g + v) * p.cJ + l16) * 4) : 0x80000000u;
    if (H3) {
      const floatx4* fh = reinterpret_cast<const floatx4*>(sFH + h * kMaxC);
#pragma unroll
      for (int q4 = 0; q4 < kMaxC / 4; ++q4) {
        if (4 * q4 >= p.cH) continue;
        const floatx4 w = fh[q4];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc3[4 * q4 + r] += w[r] * tacc;
      }
      if (h == nH - 1) {
        // uniform: the plane stride is the scalar offset of the stores
        const int cIJ = __builtin_amdgcn_readfirstlane(p.cI * p.cJ);
        const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(
            p.T + (int64_t)item * p.cH * cIJ, (short)0, p.cH * cIJ * 4, kRsrcWord3);
        if ((cIJ & 3) == 0) {
          // the item's c_H x c_I x c_J block is contiguous: stage up to 1024
          // values of it in this wave's LDS block and write them as 16-byte
          // pieces (four stores per 1024 values instead of four per plane)
          float* so = sFH + p.nH * kMaxC + (threadIdx.x >> 6) * 1024;
          const int G = __builtin_amdgcn_readfirstlane(1024 / cIJ);
          for (int q0 = 0; q0 < p.cH; q0 += G) {
#pragma unroll
            for (int q = 0; q < kMaxC; ++q) {
              if (q < q0 || q >= q0 + G || q >= p.cH) continue;
#pragma unroll
              for (int v = 0; v < 4; ++v)
                if (off[v] != 0x80000000u) so[(q - q0) * cIJ + (off[v] >> 2)] = acc3[q][v];
            }
            // ordered LDS accesses of one wave: the reads below see the writes
            __builtin_amdgcn_wave_barrier();
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            const int nf = min(G, p.cH - q0) * cIJ;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int f = (u * 64 + lane) * 4;
              const floatx4 w = *reinterpret_cast<const floatx4*>(so + f);
              const uint32_t o = f < nf ? (uint32_t)((q0 * cIJ + f) * 4) : 0x80000000u;
              __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uintx4, w), ro, o, 0, kOutStorePolicy);
            }
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            __builtin_amdgcn_wave_barrier();
          }
#pragma unroll
          for (int q = 0; q < kMaxC; ++q) acc3[q] = floatx4{};
        } else {
#pragma unroll
          for (int q = 0; q < kMaxC; ++q) {
            if (q < p.cH) {
#pragma unroll
              for (int v = 0; v < 4; ++v)
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc3[q][v]), ro, off[v], q * cIJ * 4, kOutStorePolicy);
            }
            acc3[q] = floatx4{};
          }
        }
      }
    } else {
      const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(
          p.T + (int64_t)item * p.cI * p.cJ, (short)0, p.cI * p.cJ * 4, kRsrcWord3);
#pragma unroll
      for (int v = 0; v < 4; ++v) __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(tacc[v]), ro, off[v], 0, kOutStorePolicy);
    }
    tacc = floatx4{};
  };

  // NBUF units of loads rotate through the buffers: step s multiplies
  // buffer s after issuing the load of the unit NBUF - 1 ahead
  uintx4 buf[NBUF][TG][NK];
  int ci[NBUF], chh[NBUF], cg[NBUF];
  int li = gwave, lh = 0, lg = 0;
  auto advance = [&]() {
    if (li < 0) return;
    if (++lg >= nG) {
      lg = 0;
      if (++lh >= nH) {
        lh = 0;
        li = li + nwaves < items ? li + nwaves : -1;
      }
    }
  };
  ci[0] = li;
  chh[0] = lh;
  cg[0] = lg;
  load_unit(li, lh, lg, buf[0]);
#pragma unroll
  for (int s = 1; s < NBUF - 1; ++s) {
    advance();
    ci[s] = li;
    chh[s] = lh;
    cg[s] = lg;
    load_unit(li, lh, lg, buf[s]);
  }
  // the wave's units (items gwave, gwave + nwaves, ... times nH nG) run in
  // full groups of NBUF with no exit test inside (one there would leave the
  // loads of skipped units pending at the loop head and force a wait for
  // every load in flight); the tail multiplies the units already in flight
  int left = ((items - 1 - gwave) / nwaves + 1) * nH * nG;
  for (; left >= NBUF; left -= NBUF) {
#pragma unroll
    for (int s = 0; s < NBUF; ++s) {
      const int lb = (s + NBUF - 1) % NBUF;
      advance();
      ci[lb] = li;
      chh[lb] = lh;
      cg[lb] = lg;
      load_unit(li, lh, lg, buf[lb]);
      __builtin_amdgcn_sched_barrier(0);
      compute_unit(ci[s], chh[s], cg[s], buf[s]);
    }
  }
#pragma unroll
  for (int s = 0; s < NBUF - 1; ++s)
    if (s < left) compute_unit(ci[s], chh[s], cg[s], buf[s]);
}

template <typename TX, int NK, int NT, int TG, bool H3, int NBUF>
hipError_t launch_variant(CoreSlab p, size_t lds, hipStream_t st) {
  auto kern = core_slab_kernel<TX, NK, NT, TG, H3, NBUF>;
  // as many resident waves as the registers allow, persistent over the items
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(p.items, kWaves), (int64_t)per_cu * cus));
  p.nwaves = (int32_t)(blocks * kWaves);
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), lds, st, p);
  return hipGetLastError();
}

// TG tiles per unit keep one unit's loads at 32-48 registers
template <typename TX, int NK, int NT, bool H3>
hipError_t launch_depth(const CoreSlab& p, size_t lds, hipStream_t st) {
  constexpr int kTG0 = 12 / NK < 1 ? 1 : 12 / NK;
  constexpr int kTG1 = kTG0 > NT ? NT : kTG0;
  constexpr int TG = sizeof(TX) == 4 ? kTG1 : (kTG1 < 2 ? 2 : kTG1 & ~1);
  return launch_variant<TX, NK, NT, TG, H3, 2>(p, lds, st);   // two units of loads in flight
}

template <typename TX, int NK, int NT>
hipError_t launch_typed(const CoreSlab& p, bool h3, size_t lds, hipStream_t st) {
  // three modes: F_H and a 4 KB output staging block per wave
  if (h3) return launch_depth<TX, NK, NT, true>(p, lds + (size_t)p.nH * kMaxC * sizeof(float) + kWaves * 1024 * sizeof(float), st);
  return launch_depth<TX, NK, NT, false>(p, lds, st);
}

template <typename TX>
hipError_t launch_by_size(const CoreSlab& p, bool h3, hipStream_t st) {
  constexpr bool kF32 = sizeof(TX) == 4;
  const int nT = (p.nI + 15) / 16;
  const int nK = kF32 ? (p.nJ + 15) / 16 : (p.nJ + 31) / 32;
  // LDS of the stage-2 operand tables for NT tiles
  auto lds = [&](int NT) {
    return kF32 ? (size_t)NT * 256 * sizeof(float) : (size_t)(NT / 2 + 1) * 64 * 4 * 2 * sizeof(uint32_t);
  };
  if constexpr (kF32) {
    const int m = std::max(nT, nK);
    if (m <= 2) return launch_typed<TX, 2, 2>(p, h3, lds(2), st);
    if (m <= 4) return launch_typed<TX, 4, 4>(p, h3, lds(4), st);
    if (m <= 6) return launch_typed<TX, 6, 6>(p, h3, lds(6), st);
    return launch_typed<TX, 8, 8>(p, h3, lds(8), st);
  } else {
    if (nT <= 2 && nK <= 1) return launch_typed<TX, 1, 2>(p, h3, lds(2), st);
    if (nT <= 3 && nK <= 2) return launch_typed<TX, 2, 3>(p, h3, lds(3), st);
    if (nT <= 4 && nK <= 2) return launch_typed<TX, 2, 4>(p, h3, lds(4), st);
    return launch_typed<TX, 4, 8>(p, h3, lds(8), st);
  }
}

}  // namespace

bool slab_supported(int dtype, int64_t nI, int64_t nJ, int32_t cI, int32_t cJ) {
  if (dtype != TK_F32 && dtype != TK_BF16 && dtype != TK_F16) return false;
  if (nI < 1 || nJ < 1 || nI > 128 || nJ > 128 || cI > kMaxC || cJ > kMaxC) return false;
  // 16-bit rows must start on a dword boundary for the 16-byte loads
  return dtype == TK_F32 || nJ % 2 == 0;
}

hipError_t launch_core_slab(const CoreSlab& pin, int xdt, hipStream_t st) {
  if (pin.items == 0) return hipSuccess;
  CoreSlab p = pin;
  const bool h3 = p.FH != nullptr;
  if (!h3) p.nH = 1;
  switch (xdt) {
    case TK_F32: return launch_by_size<float>(p, h3, st);
    case TK_BF16: return launch_by_size<bf16>(p, h3, st);
    case TK_F16: return launch_by_size<f16>(p, h3, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace tk
