// Transfer tensors of the H-Tucker format (Section 4, transfer-tensor
// equation):  B_S(i,j,k) = <U_S(:,i), U_Sl(:,j) kron U_Sr(:,k)>, where row
// a*n_r + b of U_S pairs row a of U_Sl with row b of U_Sr.
//
// Two steps: V[a][k][i] = sum_b U_S[a n_r + b][i] U_Sr[b][k] (a mode product
// over the right child's rows, FP64), then B[i][j][k] = sum_a U_Sl[a][j] V[a][k][i].
#include "tk_kernels.hpp"

namespace tk {
namespace {

template <typename TF>
__global__ __launch_bounds__(256) void transfer_kernel(const Transfer t) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)t.rS * t.rl * t.rr;
  if (g >= total) return;
  const int k = (int)(g % t.rr);
  const int j = (int)((g / t.rr) % t.rl);
  const int i = (int)(g / ((int64_t)t.rr * t.rl));
  const TF* Ul = static_cast<const TF*>(t.Ul);
  double acc = 0.0;
  for (int64_t a = 0; a < t.nl; ++a)
    acc = fma(to_double(Ul[a * t.rl + j]), t.V[(a * t.rr + k) * t.rS + i], acc);
  static_cast<TF*>(t.Bout)[g] = from_double<TF>(acc);
}

}  // namespace

hipError_t launch_transfer(const Transfer& t, int f_dt, hipStream_t st) {
  // step 1: U_S viewed as (n_l, n_r, r_S); contract the n_r axis with U_Sr
  ModeProduct mp{};
  mp.in = t.US;
  mp.out = t.V;
  mp.M = t.Ur;
  mp.Mt = t.Mt;
  mp.A = t.nl;
  mp.Q = t.nr;
  mp.B = t.rS;
  mp.P = t.rr;
  mp.rs = 1;       // M[p = k][q = b] = Ur[b][k]
  mp.cs = t.rr;
  mp.accumulate = 0;
  hipError_t e = launch_mode_product(mp, f_dt, TK_F64, f_dt, st);
  if (e != hipSuccess) return e;
  const int64_t total = (int64_t)t.rS * t.rl * t.rr;
  if (f_dt == TK_F64)
    hipLaunchKernelGGL((transfer_kernel<double>), dim3((unsigned)ceil_div(total, 256)), dim3(256), 0,
                       st, t);
  else
    hipLaunchKernelGGL((transfer_kernel<float>), dim3((unsigned)ceil_div(total, 256)), dim3(256), 0,
                       st, t);
  return hipGetLastError();
}

}  // namespace tk
