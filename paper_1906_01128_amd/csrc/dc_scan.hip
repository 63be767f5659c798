// The leaves' 16-byte-chunk prefix, computed on the device after each upload.
//
// pre[l] is the sum over the leaves before l (in arena order) of
// ceil(bytes / 16), and pre[nl] the total: an exclusive prefix sum of a
// function of the size words the deep copy uploads anyway, so the prefix
// itself need not cross the host link (8 bytes per leaf less, about 62 MB for
// 7.7 M MD leaves). It is the sizing step of Algorithm 1 carried out for the
// leaves, whose chunk offsets the leaf tiles and the fused launch use to find
// the leaf holding each chunk.
//
// Three launches: every block of kScanLeaves leaves sums its chunks, one
// workgroup turns those sums into block offsets, and every block scans its
// leaves again from its offset. Within a workgroup: a prefix sum over each
// wavefront's 64 lanes in six shuffle steps, then over the four wave totals
// held in LDS.
#include <hip/hip_runtime.h>

#include "dc_internal.h"

namespace dc {

namespace {

__device__ __forceinline__ uint64_t leaf_chunks(const uint64_t* info, uint64_t l, uint64_t nl) {
  return l < nl ? ((info[l] & ((1ull << kLeafKindShift) - 1)) + kChunk - 1) / kChunk : 0;
}

// inclusive prefix sum over the 64 lanes of a wavefront
__device__ __forceinline__ uint64_t wave_scan(uint64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t o = __shfl_up((unsigned long long)v, (unsigned)d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// exclusive prefix sum over the kScanBlock threads of a workgroup; *total is their sum
__device__ __forceinline__ uint64_t block_scan(uint64_t v, uint64_t* wsum, uint64_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t inc = wave_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint64_t before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < (int)(kScanBlock / 64); k++) {
    if (k < w) before += wsum[k];
    all += wsum[k];
  }
  __syncthreads();  // wsum is written again by the next call
  *total = all;
  return before + inc - v;
}

__global__ void __launch_bounds__(kScanBlock) k_prefix_sums(const uint64_t* info, uint64_t nl, uint64_t* scan) {
  __shared__ uint64_t wsum[kScanBlock / 64];
  const uint64_t l0 = (uint64_t)blockIdx.x * kScanLeaves + (uint64_t)threadIdx.x * kScanPer;
  uint64_t v = 0;
#pragma unroll
  for (uint32_t k = 0; k < kScanPer; k++) v += leaf_chunks(info, l0 + k, nl);
  uint64_t total;
  block_scan(v, wsum, &total);
  if (threadIdx.x == 0) scan[blockIdx.x] = total;
}

// one workgroup: block sums -> block offsets, in rounds of kScanLeaves blocks
__global__ void __launch_bounds__(kScanBlock) k_prefix_offsets(uint64_t* scan, uint64_t nb, uint64_t* pre,
                                                               uint64_t nl) {
  __shared__ uint64_t wsum[kScanBlock / 64];
  uint64_t carry = 0;
  for (uint64_t b0 = 0; b0 < nb; b0 += kScanLeaves) {
    const uint64_t b = b0 + (uint64_t)threadIdx.x * kScanPer;
    uint64_t x[kScanPer], v = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanPer; k++) {
      x[k] = b + k < nb ? scan[b + k] : 0;
      v += x[k];
    }
    uint64_t total;
    uint64_t run = carry + block_scan(v, wsum, &total);
#pragma unroll
    for (uint32_t k = 0; k < kScanPer; k++) {
      if (b + k < nb) scan[b + k] = run;
      run += x[k];
    }
    carry += total;
  }
  if (threadIdx.x == 0) pre[nl] = carry;
}

__global__ void __launch_bounds__(kScanBlock) k_prefix_write(const uint64_t* info, uint64_t nl, const uint64_t* scan,
                                                             uint64_t* pre) {
  __shared__ uint64_t wsum[kScanBlock / 64];
  const uint64_t l0 = (uint64_t)blockIdx.x * kScanLeaves + (uint64_t)threadIdx.x * kScanPer;
  uint64_t x[kScanPer], v = 0;
#pragma unroll
  for (uint32_t k = 0; k < kScanPer; k++) {
    x[k] = leaf_chunks(info, l0 + k, nl);
    v += x[k];
  }
  uint64_t total;
  uint64_t run = scan[blockIdx.x] + block_scan(v, wsum, &total);
#pragma unroll
  for (uint32_t k = 0; k < kScanPer; k++) {
    if (l0 + k < nl) pre[l0 + k] = run;
    run += x[k];
  }
}

}  // namespace

hipError_t launch_leaf_prefix(const uint64_t* info, uint64_t nl, uint64_t* pre, uint64_t* scan, hipStream_t s) {
  const uint64_t nb = (nl + kScanLeaves - 1) / kScanLeaves;
  if (nb > 0xffffffffull) return hipErrorInvalidValue;
  if (nb) hipLaunchKernelGGL(k_prefix_sums, dim3((uint32_t)nb), dim3(kScanBlock), 0, s, info, nl, scan);
  hipLaunchKernelGGL(k_prefix_offsets, dim3(1), dim3(kScanBlock), 0, s, scan, nb, pre, nl);
  if (nb) hipLaunchKernelGGL(k_prefix_write, dim3((uint32_t)nb), dim3(kScanBlock), 0, s, info, nl, scan, pre);
  return hipGetLastError();
}

}  // namespace dc
