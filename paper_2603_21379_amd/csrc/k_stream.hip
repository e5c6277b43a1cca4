// Read-only streaming reference for the measurement: one read of a device
// buffer with the access pattern of the streaming passes at their best (each
// 16-byte-per-lane load covers one contiguous 1 KB piece; persistent waves,
// two workgroups per CU, four loads in flight per wave), reduced to one
// checksum per workgroup so no load can be dropped.  The buffer is read as
// float4s; a tail of fewer than 16 bytes is not read.
#include "tk_kernels.hpp"

namespace tk {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void stream_read_kernel(const floatx4* __restrict__ x, int64_t n4,
                                                          double* partials) {
  __shared__ double red[256];
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (tid >> 6), nwaves = (int64_t)gridDim.x * 4;
  floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  // the wave's 4 KB blocks: 256 float4, four 1 KB loads
  const int64_t nblk = n4 / 256;
  for (int64_t b = wave; b < nblk; b += nwaves) {
    const floatx4* p = x + b * 256 + lane;
    floatx4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(p + 64 * u);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += v[u];
  }
  // the float4s past the last whole block
  for (int64_t i = nblk * 256 + wave * 64 + lane; i < n4; i += nwaves * 64) acc += x[i];
  red[tid] = (double)acc[0] + (double)acc[1] + (double)acc[2] + (double)acc[3];
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int i = 0; i < 256; ++i) s += red[i];
    partials[blockIdx.x] = s;
  }
}

}  // namespace

int stream_read_blocks() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  return 2 * cus;
}

hipError_t launch_stream_read(const void* x, int64_t bytes, double* partials, int32_t blocks, hipStream_t st) {
  const int64_t n4 = bytes / 16;
  if (n4 <= 0 || blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(stream_read_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                     static_cast<const floatx4*>(x), n4, partials);
  return hipGetLastError();
}

}  // namespace tk
