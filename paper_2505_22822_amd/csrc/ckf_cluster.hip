// Cell clustering and measurement formation (paper section 2: connected
// component analysis of a sensor's activated cells; each cluster's weighted
// centroid and its error make a measurement, whose global position is a
// spacepoint).
//
// Cells arrive in readout order: grouped by (event, module) row, then by
// row c1 and column c0 inside a module.  Two cells touch when |dc0| <= 1 and
// |dc1| <= 1, so a cell's earlier neighbours lie in the rows c1 - 1 and c1,
// just before it in the order.  Everything runs one thread per cell (or per
// cluster), with no per-module serial work:
//   heads   - each (event, module) row marks its first cell; an inclusive
//             max-scan gives every cell its row;
//   link    - each cell scans back over the cells of its module while
//             c1 >= its c1 - 1 and joins the touching ones in a lock-free
//             union-find (compare-and-swap of the larger root onto the
//             smaller), so every cluster's root is its first cell;
//   flatten - every cell's root (read-only walk of the final forest) and
//             the root flags;
//   number  - an exclusive sum-scan of the root flags numbers the clusters in
//             readout order of their first cells: clusters come out grouped
//             by row, in the order the measurement layout needs, and a row's
//             measurement offset is the scan at its first cell;
//   label   - every cell's cluster number; each root notes its cluster's
//             first cell;
//   measure - per cluster: W = sum q, X = sum q (c + 1/2) over its cells in
//             FP64 and index order, then loc = pitch X / W - half length,
//             pitch^2 / 12 variances, the spacepoint.  The cluster's cells
//             follow its first cell in the module's row, and their c1 values
//             form an interval starting at the first cell's (a connected
//             set, first in readout order): the scan stops at the first cell
//             whose c1 is past the last member's c1 + 1.  No atomics, and the
//             additions happen in the same order as in a sequential pass.
#include <climits>

#include "ckf_device.hpp"
#include "ckf_kernels.hpp"
#include "ckf_scan.hpp"

namespace ckf {

namespace {

constexpr int kClBlock = 256;
constexpr int kScanBlock = scan_detail::kScanBlock;

__global__ void k_cl_clear(int* status) { *status = 0; }

__global__ void k_cl_init(long long n, int* __restrict__ head, int* __restrict__ parent) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  head[i] = -1;
  parent[i] = (int)i;
}

// each row marks its first cell with its row number; offsets checked
__global__ void k_cl_heads(CellsIn c, int* __restrict__ head, int* __restrict__ status) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long rows = (long long)c.n_events * c.n_surfaces;
  if (r >= rows) return;
  const int a = c.offsets[r], b = c.offsets[r + 1];
  if (a < 0 || b < a || (long long)b > c.n_cells) {
    atomicOr(status, CKF_CLUSTER_BAD_OFFSETS);
    return;
  }
  if (r == 0 && a != 0) atomicOr(status, CKF_CLUSTER_BAD_OFFSETS);
  if (a < b) head[a] = (int)r;
}

__device__ __forceinline__ int cl_find(int* p, int x) {
  int y = p[x];
  while (y != x) {  // parents only ever move to smaller indices: halving stays valid under races
    const int z = p[y];
    if (z != y) p[x] = z;
    x = y;
    y = z;
  }
  return x;
}

// joins the components of touching cells i and j: the larger root is hooked
// under the smaller one with compare-and-swap, retried on a lost race
__device__ __forceinline__ void link_pair(int* parent, int i, int j) {
  int ri = cl_find(parent, i), rj = cl_find(parent, j);
  while (ri != rj) {
    if (ri < rj) {
      const int t = ri;
      ri = rj;
      rj = t;
    }
    const int old = atomicCAS(&parent[ri], ri, rj);
    if (old == ri) break;
    ri = cl_find(parent, old);
    rj = cl_find(parent, rj);
  }
}

__global__ void k_cl_link(CellsIn c, const int* __restrict__ row, int* __restrict__ parent,
                          int* __restrict__ status) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.n_cells) return;
  const int r = row[i];
  if (r < 0) return;  // before the first row (bad offsets)
  const int x = c.c0[i], y = c.c1[i];
  const long long a = c.offsets[r];
  if (i > a && (c.c1[i - 1] > y || (c.c1[i - 1] == y && c.c0[i - 1] >= x))) atomicOr(status, CKF_CLUSTER_UNSORTED);
  // earlier cells of the module, newest first, while their row is c1 - 1 or
  // c1; their positions are loaded four at a time (loads in flight together)
  bool more = true;
  for (long long j0 = i - 1; more && j0 >= a; j0 -= 4) {
    int cy[4], cx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long j = j0 - u;
      cy[u] = j >= a ? c.c1[j] : INT_MIN;
      cx[u] = j >= a ? c.c0[j] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!more) break;
      if (cy[u] < y - 1) {  // also past the module's first cell (INT_MIN)
        more = false;
        break;
      }
      if (abs(cx[u] - x) <= 1) link_pair(parent, (int)i, (int)(j0 - u));
    }
  }
}

// every cell's root into a separate array: the forest is final, and it is
// only read here (a shortening store into it could land after another
// cell's and leave that cell pointing at an ancestor short of its root)
__global__ void k_cl_flatten(long long n, const int* __restrict__ parent, int* __restrict__ root,
                             int* __restrict__ is_root) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int x = (int)i, y = parent[x];
  while (y != x) {
    x = y;
    y = parent[x];
  }
  root[i] = x;
  is_root[i] = x == i ? 1 : 0;
}

// every cell's cluster number; the roots note their cluster's first cell
__global__ void k_cl_label(long long n, const int* __restrict__ row, const int* __restrict__ root,
                           const int* __restrict__ cid, int* __restrict__ first, int* __restrict__ cell_cluster) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = cid[root[i]];
  if (root[i] == i) first[k] = (int)i;
  if (cell_cluster) cell_cluster[i] = row[i] < 0 ? -1 : k;
}

__global__ void k_cl_measure(CellsIn c, GeomDev g, const float* __restrict__ pitch, const int* __restrict__ n_cl,
                             const int* __restrict__ first, const int* __restrict__ row,
                             const int* __restrict__ root, float* __restrict__ loc, float* __restrict__ var,
                             float* __restrict__ sp) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= *n_cl) return;
  const int f = first[k];
  const int rr = row[f];
  if (rr < 0) {  // a cell before the first row (bad offsets, flagged): no module
    loc[2 * k] = loc[2 * k + 1] = var[2 * k] = var[2 * k + 1] = NAN;
    if (sp) sp[3 * k] = sp[3 * k + 1] = sp[3 * k + 2] = NAN;
    return;
  }
  const int s = rr % c.n_surfaces;
  Module M;
  load_module(g, s, M);
  const double p0 = pitch[2 * s], p1 = pitch[2 * s + 1];
  // the cluster's cells: from its first cell to the end of its c1 interval
  // (the first cell at least, should flagged offsets have put it past its row's end)
  const long long end = max((long long)c.offsets[rr + 1], (long long)f + 1);
  double w = 0.0, x0 = 0.0, x1 = 0.0;
  int last = c.c1[f];
  bool more = true;
  for (long long j0 = f; more && j0 < end; j0 += 4) {  // four cells' loads in flight together
    int cy[4], cx[4], rt[4];
    float cq[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long j = j0 + u;
      const bool in = j < end;
      cy[u] = in ? c.c1[j] : INT_MAX;
      rt[u] = in ? root[j] : -1;
      cx[u] = in ? c.c0[j] : 0;
      cq[u] = in ? c.q[j] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!more) break;
      if (cy[u] > last + 1) {  // also past the row's end (INT_MAX)
        more = false;
        break;
      }
      if (rt[u] != f) continue;
      const double q = cq[u];
      w += q;
      x0 += q * ((double)cx[u] + 0.5);
      x1 += q * ((double)cy[u] + 0.5);
      last = cy[u];
    }
  }
  const double l0 = p0 * (x0 / w) - (double)M.hw0, l1 = p1 * (x1 / w) - (double)M.hw1;
  loc[2 * k] = (float)l0;
  loc[2 * k + 1] = (float)l1;
  var[2 * k] = (float)(p0 * p0 / 12.0);
  var[2 * k + 1] = (float)(p1 * p1 / 12.0);
  if (sp) {
    const float f0 = (float)l0, f1 = (float)l1;
#pragma unroll
    for (int d = 0; d < 3; ++d) sp[3 * k + d] = M.c[d] + f0 * M.u[d] + f1 * M.v[d];
  }
}

// a row's measurement offset: the cluster number at its first cell (the
// total past the last cell)
__global__ void k_cl_offsets(CellsIn c, const int* __restrict__ cid, const int* __restrict__ n_cl,
                             int* __restrict__ moff) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long rows = (long long)c.n_events * c.n_surfaces;
  if (r > rows) return;
  const long long a = r < rows ? c.offsets[r] : c.n_cells;
  moff[r] = (a >= 0 && a < c.n_cells) ? cid[a] : *n_cl;
}

size_t al256c(size_t b) { return (b + 255) & ~(size_t)255; }

struct ClWs {
  int *head, *row, *parent, *is_root, *cid, *first, *n_cl;
  long long* sums;
};

ClWs cl_view(void* ws, long long n) {
  char* p = static_cast<char*>(ws);
  ClWs w;
  int** ints[] = {&w.head, &w.row, &w.parent, &w.is_root, &w.cid, &w.first};
  for (int** q : ints) {
    *q = reinterpret_cast<int*>(p);
    p += al256c((size_t)n * 4);
  }
  w.n_cl = reinterpret_cast<int*>(p);
  p += 256;
  w.sums = reinterpret_cast<long long*>(p);
  return w;
}

}  // namespace

size_t cluster_workspace_bytes(long long rows, long long n_cells) {
  (void)rows;
  const long long n = n_cells > 0 ? n_cells : 1;
  const long long nb = (n + kScanBlock - 1) / kScanBlock;
  return 6 * al256c((size_t)n * 4) + 256 + al256c((size_t)(nb + 1) * 8) + 256;
}

hipError_t launch_cluster(const CellsIn& c, const GeomDev& g, const float* pitch, void* ws, int* moff, float* loc,
                          float* var, float* sp, int* cell_cluster, int* status, hipStream_t st) {
  const long long rows = (long long)c.n_events * c.n_surfaces;
  const long long n = c.n_cells;
  const ClWs w = cl_view(ws, n > 0 ? n : 1);
  hipLaunchKernelGGL(k_cl_clear, dim3(1), dim3(1), 0, st, status);  // a kernel, not a memset: capturable
  const auto blocks = [](long long m) { return dim3((unsigned)((m + kClBlock - 1) / kClBlock)); };
  if (n > 0) hipLaunchKernelGGL(k_cl_init, blocks(n), dim3(kClBlock), 0, st, n, w.head, w.parent);
  if (rows > 0) hipLaunchKernelGGL(k_cl_heads, blocks(rows), dim3(kClBlock), 0, st, c, w.head, status);
  device_scan<OpMax, true>(w.head, n, w.row, w.sums, nullptr, st);
  if (n > 0) {
    hipLaunchKernelGGL(k_cl_link, blocks(n), dim3(kClBlock), 0, st, c, w.row, w.parent, status);
    // the row heads are scanned already: their array takes the roots
    hipLaunchKernelGGL(k_cl_flatten, blocks(n), dim3(kClBlock), 0, st, n, w.parent, w.head, w.is_root);
  }
  device_scan<OpSum, false>(w.is_root, n, w.cid, w.sums, w.n_cl, st);
  if (n > 0) {
    hipLaunchKernelGGL(k_cl_label, blocks(n), dim3(kClBlock), 0, st, n, w.row, w.head, w.cid, w.first, cell_cluster);
    hipLaunchKernelGGL(k_cl_measure, blocks(n), dim3(kClBlock), 0, st, c, g, pitch, w.n_cl, w.first, w.row, w.head,
                       loc, var, sp);
  }
  hipLaunchKernelGGL(k_cl_offsets, blocks(rows + 1), dim3(kClBlock), 0, st, c, w.cid, w.n_cl, moff);
  return hipGetLastError();
}

}  // namespace ckf
