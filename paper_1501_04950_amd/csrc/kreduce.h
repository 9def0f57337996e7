// Block reductions of doubles shared by the precision-independent kernels (kernels.hip)
// and the per-precision ones (kcommon.h).  The summation order is fixed, so a sum of
// the same partials gives the same bits in every kernel that takes it.
#pragma once

#include <hip/hip_runtime.h>

namespace dwa {

// wave64 butterfly sum (every lane ends with the total)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block sum: per-wave sums through LDS, added by thread 0 in wave order into *out_slot
__device__ __forceinline__ void block_sum_to(double v, double* out_slot) {
  __shared__ double wsum[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  if (lane == 0) wsum[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += wsum[i];
    *out_slot = t;
  }
}

// Sum of n partials, returned to every thread of the block (all threads must call it).
__device__ __forceinline__ double sum_partials_block(const double* part, int n) {
  // Thread k adds part[k], part[k + blockDim], ... in that order.  The loads of a group
  // of 8 are independent and go out together: the partials were just written by blocks
  // on every XCD, so each is a round trip to the Infinity Cache or HBM, and a loop that
  // waited for each in turn spent most of the time on them.
  constexpr int U = 8;
  double v = 0.0;
  for (int base = 0; base < n; base += U * blockDim.x) {
    double t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * int(blockDim.x) + int(threadIdx.x);
      t[u] = i < n ? part[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v += t[u];
  }
  __shared__ double res;
  block_sum_to(v, &res);
  __syncthreads();
  return res;
}

}  // namespace dwa
