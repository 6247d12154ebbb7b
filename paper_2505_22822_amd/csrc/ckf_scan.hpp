// Device-wide scans of int arrays (sum or max) in three launches: block
// scans with block totals, one block over the totals, and the totals
// applied.  Results must fit in int; the totals are kept in long long.
#pragma once
#include <hip/hip_runtime.h>

namespace ckf {
namespace scan_detail {

constexpr int kScanBlock = 1024;

struct OpSum {
  __device__ static long long id() { return 0; }
  __device__ static long long f(long long a, long long b) { return a + b; }
};
struct OpMax {
  __device__ static long long id() { return -1; }
  __device__ static long long f(long long a, long long b) { return a > b ? a : b; }
};

// scan of n values in blocks of kScanBlock (inclusive or exclusive): per-block
// scans and block totals; then the totals scanned by one block; then applied
template <class Op, bool kIncl>
__global__ void __launch_bounds__(kScanBlock) k_scan_blocks(const int* __restrict__ in, long long n,
                                                              int* __restrict__ out, long long* __restrict__ sums) {
  __shared__ long long sh[kScanBlock];
  const long long i = (long long)blockIdx.x * kScanBlock + threadIdx.x;
  const long long v = i < n ? in[i] : Op::id();
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < kScanBlock; o <<= 1) {
    const long long t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : Op::id();
    __syncthreads();
    sh[threadIdx.x] = Op::f(sh[threadIdx.x], t);
    __syncthreads();
  }
  if (i < n) out[i] = (int)(kIncl ? sh[threadIdx.x] : (threadIdx.x ? sh[threadIdx.x - 1] : Op::id()));
  if (threadIdx.x == kScanBlock - 1) sums[blockIdx.x] = sh[threadIdx.x];
}

// one block: block totals -> exclusive block prefixes (serial over chunks); the grand total
template <class Op>
__global__ void __launch_bounds__(kScanBlock) k_scan_sums(long long nb, long long* __restrict__ sums,
                                                            int* __restrict__ total) {
  __shared__ long long sh[kScanBlock];
  long long base = Op::id();
  for (long long b0 = 0; b0 < nb; b0 += kScanBlock) {
    const long long b = b0 + threadIdx.x;
    const long long v = b < nb ? sums[b] : Op::id();
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kScanBlock; o <<= 1) {
      const long long t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : Op::id();
      __syncthreads();
      sh[threadIdx.x] = Op::f(sh[threadIdx.x], t);
      __syncthreads();
    }
    const long long prev = threadIdx.x ? sh[threadIdx.x - 1] : Op::id();
    if (b < nb) sums[b] = Op::f(base, prev);
    const long long chunk = sh[kScanBlock - 1];
    __syncthreads();
    base = Op::f(base, chunk);
  }
  if (threadIdx.x == 0 && total) *total = (int)base;
}

template <class Op>
__global__ void k_scan_apply(long long n, int* __restrict__ out, const long long* __restrict__ sums) {
  const long long i = (long long)blockIdx.x * kScanBlock + threadIdx.x;
  if (i < n) out[i] = (int)Op::f(sums[blockIdx.x], out[i]);
}

}  // namespace scan_detail

// out[i] = op(in[0..i]) (kIncl) or op(in[0..i-1]); *total = op(in[0..n-1])
// when total is not null.  sums: at least (n + 1023) / 1024 + 1 long longs.
template <class Op, bool kIncl>
inline void device_scan(const int* in, long long n, int* out, long long* sums, int* total, hipStream_t st) {
  const long long nb = (n + scan_detail::kScanBlock - 1) / scan_detail::kScanBlock;
  if (nb > 0)
    hipLaunchKernelGGL((scan_detail::k_scan_blocks<Op, kIncl>), dim3((unsigned)nb), dim3(scan_detail::kScanBlock), 0, st, in, n, out, sums);
  hipLaunchKernelGGL((scan_detail::k_scan_sums<Op>), dim3(1), dim3(scan_detail::kScanBlock), 0, st, nb, sums, total);
  if (nb > 0) hipLaunchKernelGGL((scan_detail::k_scan_apply<Op>), dim3((unsigned)nb), dim3(scan_detail::kScanBlock), 0, st, n, out, sums);
}

using scan_detail::OpMax;
using scan_detail::OpSum;

}  // namespace ckf
