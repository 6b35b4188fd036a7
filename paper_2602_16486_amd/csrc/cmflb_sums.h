// cmflb_sums.h -- the fixed-order FP64 sum of statistics rows shared by the
// single-lattice finalize (cmflb_kernels.hip) and the ensemble's per-replica
// reduction (cmflb_ensemble.hip).
#pragma once

#include "cmflb_internal.h"

namespace cmf {

// One 256-thread workgroup sums rows [lo, hi) of a [rows][kPartStride]
// array of block partials into out[0, kNAcc): thread t adds rows t, t + 256,
// ... in order, then a binary tree over the threads; the order depends on
// lo and hi only, so a replay gives the same bits.
__device__ __forceinline__ void block_sum_rows(const double *__restrict__ rows,
                                               int lo, int hi, double *out) {
  __shared__ double sh[256][kNAcc];
  const int tid = threadIdx.x;
  double s[kNAcc];
#pragma unroll
  for (int k = 0; k < kNAcc; ++k) s[k] = 0.0;
  for (int b = lo + tid; b < hi; b += 256)
#pragma unroll
    for (int k = 0; k < kNAcc; ++k) s[k] += rows[(int64_t)b * kPartStride + k];
#pragma unroll
  for (int k = 0; k < kNAcc; ++k) sh[tid][k] = s[k];
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (tid < h)
#pragma unroll
      for (int k = 0; k < kNAcc; ++k) sh[tid][k] += sh[tid + h][k];
    __syncthreads();
  }
  if (tid < kNAcc) out[tid] = sh[0][tid];
}

}  // namespace cmf
