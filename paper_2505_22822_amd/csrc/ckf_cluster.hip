// Cell clustering and measurement formation (paper section 2: connected
// component analysis of a sensor's activated cells; each cluster's weighted
// centroid and its error make a measurement, whose global position is a
// spacepoint).
//
// Cells arrive in readout order: grouped by (event, module) row, then by
// row c1 and column c0 inside a module.  Two cells touch when |dc0| <= 1 and
// |dc1| <= 1, so a cell's earlier neighbours lie in the rows c1 - 1 and c1,
// just before it in the order.  One lane takes one (event, module) row:
//   label   - union-find over the row's cells, each cell joined to the
//             touching cells found by scanning back while c1 >= its c1 - 1;
//             roots are the smaller index, so a cluster is named by its
//             first cell; clusters per row counted;
//   scan    - exclusive prefix sum of the counts: the measurements' row
//             offsets, the layout ckf_find reads;
//   measure - each cluster's charge-weighted mean of the cell centres (FP64
//             sums in readout order), pitch^2 / 12 variances, spacepoints.
// Rows hold a few cells each on average, so one lane per row keeps the
// union-find in private order with no atomics; the kernels stream the cells
// once or twice and are bound by memory and latency.
#include "ckf_device.hpp"
#include "ckf_kernels.hpp"

namespace ckf {

namespace {

constexpr int kClBlock = 256;
constexpr int kScanBlock = 1024;

__device__ __forceinline__ int cl_find(int* p, int x) {
  while (p[x] != x) {
    const int g = p[p[x]];
    p[x] = g;
    x = g;
  }
  return x;
}

__global__ void k_cl_clear(int* status) { *status = 0; }

__global__ void k_cl_label(CellsIn c, int* __restrict__ parent, int* __restrict__ counts, int* __restrict__ status) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long rows = (long long)c.n_events * c.n_surfaces;
  if (r >= rows) return;
  const int a = c.offsets[r], b = c.offsets[r + 1];
  if (a < 0 || b < a || (long long)b > c.n_cells) {
    atomicOr(status, CKF_CLUSTER_BAD_OFFSETS);
    counts[r] = 0;
    return;
  }
  int n_root = 0;
  for (int i = a; i < b; ++i) {
    parent[i] = i;
    const int x = c.c0[i], y = c.c1[i];
    if (i > a && (c.c1[i - 1] > y || (c.c1[i - 1] == y && c.c0[i - 1] >= x))) atomicOr(status, CKF_CLUSTER_UNSORTED);
    for (int j = i - 1; j >= a && c.c1[j] >= y - 1; --j) {
      if (abs(c.c0[j] - x) > 1) continue;
      const int ri = cl_find(parent, i), rj = cl_find(parent, j);
      if (ri != rj) parent[max(ri, rj)] = min(ri, rj);
    }
  }
  for (int i = a; i < b; ++i) {
    const int root = cl_find(parent, i);
    parent[i] = root;
    n_root += root == i ? 1 : 0;
  }
  counts[r] = n_root;
}

// exclusive scan of n ints in blocks of kScanBlock: per-block scans and sums
__global__ void __launch_bounds__(kScanBlock) k_scan_blocks(const int* __restrict__ in, long long n,
                                                              int* __restrict__ out, long long* __restrict__ sums) {
  __shared__ long long sh[kScanBlock];
  const long long i = (long long)blockIdx.x * kScanBlock + threadIdx.x;
  const long long v = i < n ? in[i] : 0;
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < kScanBlock; o <<= 1) {
    const long long t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < n) out[i] = (int)(sh[threadIdx.x] - v);
  if (threadIdx.x == kScanBlock - 1) sums[blockIdx.x] = sh[threadIdx.x];
}

// one block: block sums -> block offsets (serial over chunks), and the total
__global__ void __launch_bounds__(kScanBlock) k_scan_sums(long long nb, long long* __restrict__ sums,
                                                            int* __restrict__ total) {
  __shared__ long long sh[kScanBlock];
  long long base = 0;
  for (long long b0 = 0; b0 < nb; b0 += kScanBlock) {
    const long long b = b0 + threadIdx.x;
    const long long v = b < nb ? sums[b] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kScanBlock; o <<= 1) {
      const long long t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (b < nb) sums[b] = base + sh[threadIdx.x] - v;
    const long long chunk = sh[kScanBlock - 1];
    __syncthreads();
    base += chunk;
  }
  if (threadIdx.x == 0) *total = (int)base;
}

__global__ void k_scan_apply(long long n, int* __restrict__ out, const long long* __restrict__ sums) {
  const long long i = (long long)blockIdx.x * kScanBlock + threadIdx.x;
  if (i < n) out[i] += (int)sums[blockIdx.x];
}

__global__ void k_cl_measure(CellsIn c, GeomDev g, const float* __restrict__ pitch, const int* __restrict__ parent,
                             const int* __restrict__ moff, int* __restrict__ slot, double* __restrict__ acc,
                             float* __restrict__ loc, float* __restrict__ var, float* __restrict__ sp,
                             int* __restrict__ cell_cluster) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long rows = (long long)c.n_events * c.n_surfaces;
  if (r >= rows) return;
  const int a = c.offsets[r], b = c.offsets[r + 1];
  if (a < 0 || b < a || (long long)b > c.n_cells || a == b) return;
  const int s = (int)(r % c.n_surfaces);
  const int o0 = moff[r];
  int k = o0;
  for (int i = a; i < b; ++i)
    if (parent[i] == i) {
      slot[i] = k;
      acc[3ll * k] = acc[3ll * k + 1] = acc[3ll * k + 2] = 0.0;
      ++k;
    }
  Module M;
  load_module(g, s, M);
  const double p0 = pitch[2 * s], p1 = pitch[2 * s + 1], h0 = M.hw0, h1 = M.hw1;
  for (int i = a; i < b; ++i) {
    const int kk = slot[parent[i]];
    const double q = c.q[i];
    acc[3ll * kk] += q;
    acc[3ll * kk + 1] += q * ((c.c0[i] + 0.5) * p0 - h0);
    acc[3ll * kk + 2] += q * ((c.c1[i] + 0.5) * p1 - h1);
    if (cell_cluster) cell_cluster[i] = kk;
  }
  const float v0 = (float)(p0 * p0 / 12.0), v1 = (float)(p1 * p1 / 12.0);
  for (int m = o0; m < k; ++m) {
    const double w = acc[3ll * m];
    const double l0 = acc[3ll * m + 1] / w, l1 = acc[3ll * m + 2] / w;
    loc[2ll * m] = (float)l0;
    loc[2ll * m + 1] = (float)l1;
    var[2ll * m] = v0;
    var[2ll * m + 1] = v1;
    if (sp) {
      const float f0 = (float)l0, f1 = (float)l1;
#pragma unroll
      for (int d = 0; d < 3; ++d) sp[3ll * m + d] = M.c[d] + f0 * M.u[d] + f1 * M.v[d];
    }
  }
}

size_t al256c(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

size_t cluster_workspace_bytes(long long rows, long long n_cells) {
  const long long nb = (rows + kScanBlock - 1) / kScanBlock;
  return al256c((size_t)n_cells * 4) * 2 + al256c((size_t)n_cells * 24) + al256c((size_t)rows * 4) +
         al256c((size_t)(nb + 1) * 8) + 256;
}

hipError_t launch_cluster(const CellsIn& c, const GeomDev& g, const float* pitch, void* ws, int* moff, float* loc,
                          float* var, float* sp, int* cell_cluster, int* status, hipStream_t st) {
  const long long rows = (long long)c.n_events * c.n_surfaces;
  const long long nb = (rows + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(k_cl_clear, dim3(1), dim3(1), 0, st, status);  // a kernel, not a memset: capturable
  char* p = static_cast<char*>(ws);
  int* parent = reinterpret_cast<int*>(p);
  p += al256c((size_t)c.n_cells * 4);
  int* slot = reinterpret_cast<int*>(p);
  p += al256c((size_t)c.n_cells * 4);
  double* acc = reinterpret_cast<double*>(p);
  p += al256c((size_t)c.n_cells * 24);
  int* counts = reinterpret_cast<int*>(p);
  p += al256c((size_t)rows * 4);
  long long* sums = reinterpret_cast<long long*>(p);
  if (rows <= 0) {  // no rows: only the total (zero) of the offsets
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, st, 0ll, sums, moff);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)((rows + kClBlock - 1) / kClBlock)), block(kClBlock);
  hipLaunchKernelGGL(k_cl_label, grid, block, 0, st, c, parent, counts, status);
  hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(kScanBlock), 0, st, counts, rows, moff, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, st, nb, sums, moff + rows);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanBlock), 0, st, rows, moff, sums);
  hipLaunchKernelGGL(k_cl_measure, grid, block, 0, st, c, g, pitch, parent, moff, slot, acc, loc, var, sp,
                     cell_cluster);
  return hipGetLastError();
}

}  // namespace ckf
