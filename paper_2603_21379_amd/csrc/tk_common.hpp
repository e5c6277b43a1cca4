// Internal definitions shared by the host layer and the kernels of libtkmi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "tkmi.h"

namespace tk {

// ------------------------------------------------------------------ element types
// BF16 is kept as raw bits: the upper half of an IEEE binary32 pattern.
struct bf16 {
  uint16_t u;
};
using f16 = _Float16;

__host__ __device__ __forceinline__ float to_float(float v) { return v; }
__host__ __device__ __forceinline__ float to_float(double v) { return (float)v; }
__host__ __device__ __forceinline__ float to_float(f16 v) { return (float)v; }
__device__ __forceinline__ float to_float(bf16 v) { return __uint_as_float(((uint32_t)v.u) << 16); }

__host__ __device__ __forceinline__ double to_double(double v) { return v; }
__host__ __device__ __forceinline__ double to_double(float v) { return (double)v; }
__host__ __device__ __forceinline__ double to_double(f16 v) { return (double)(float)v; }
__device__ __forceinline__ double to_double(bf16 v) { return (double)to_float(v); }

template <typename T> __device__ __forceinline__ T from_double(double v);
template <> __device__ __forceinline__ double from_double<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_double<float>(double v) { return (float)v; }

// factor dtype of a tensor dtype
inline int factor_dtype(int dt) { return dt == TK_F64 ? TK_F64 : TK_F32; }
inline size_t dtype_size(int dt) {
  switch (dt) {
    case TK_F64: return 8;
    case TK_F32: return 4;
    case TK_BF16: return 2;
    case TK_F16: return 2;
    default: return 0;
  }
}

// A value every lane of a wave holds (read from one address), passed word by
// word through v_readfirstlane so the compiler keeps it in scalar registers.
// Buffer descriptors and scalar offsets built from it then stay uniform;
// otherwise every buffer access is wrapped in a loop over distinct values.
template <typename T>
__device__ __forceinline__ T wave_uniform(const T& v) {
  static_assert(sizeof(T) % 4 == 0, "word-sized fields only");
  T out;
  const int* src = reinterpret_cast<const int*>(&v);
  int* dst = reinterpret_cast<int*>(&out);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
  return out;
}

// Cache policy (sc0 | sc1) of the small per-slab output stores of the
// streaming kernels: written through rather than held dirty in L2, so the
// write-back does not interleave with the read stream of X (measured on the
// 256^4 FP32 pass: ~0.17 ms of the ~0.5 ms the stores cost with the default
// policy).
constexpr int kOutStorePolicy = 0x11;

// ------------------------------------------------------------------ limits
constexpr int kMaxEll = 64;       // sketch width handled by the one-wave Jacobi solver
constexpr int kMaxCols = 192;     // factor columns per mode in the core / reconstruct
constexpr int kMaxUnits = 32;     // sketch units (modes or tree nodes) per launch

// ------------------------------------------------------------------ host error state
tk_status set_error(tk_status s, const char* fmt, ...);
void clear_error();

// Bump planner over a caller workspace.  Pass 1 (base == nullptr) only
// measures; pass 2 hands out aligned sub-buffers.
struct Workspace {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    size_t o = (off + 255) & ~size_t(255);
    off = o + count * sizeof(T);
    return base ? reinterpret_cast<T*>(base + o) : nullptr;
  }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Streaming-pass profiler (tk_profile_enable / tk_profile_read).
bool profiling();
hipError_t profile_begin(hipStream_t st);  // record the start event of one bracket
hipError_t profile_end(hipStream_t st);    // record its stop event

}  // namespace tk

#define TK_HIP(expr)                                                                  \
  do {                                                                                \
    hipError_t tk_e_ = (expr);                                                        \
    if (tk_e_ != hipSuccess)                                                          \
      return ::tk::set_error(TK_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(tk_e_)); \
  } while (0)

#define TK_LAUNCHED(what)                                                             \
  do {                                                                                \
    hipError_t tk_e_ = hipGetLastError();                                             \
    if (tk_e_ != hipSuccess)                                                          \
      return ::tk::set_error(TK_EDEVICE, "launch of %s failed: %s", what,            \
                             hipGetErrorString(tk_e_));                              \
  } while (0)
