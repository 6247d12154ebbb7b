// gfx950 kernels of CKF track finding.
//
//  k_meas_rows,    per (event, module) row: measurements sorted by loc0 (ids
//  k_meas_scatter  kept) and the row's largest var0, for the exact chi2
//                  window of the search.
//  k_ckf           persistent kernel: each 64-lane workgroup pulls seeds from
//                  a global work queue into its slots and advances all their
//                  candidates step by step (navigate, RKN4 leg with Jacobian
//                  transport, chi2 search, Kalman update, branching), with
//                  wave ballot/scan compaction of the children into a
//                  per-workgroup candidate pool and per-seed pruning.
//  k_out_*         per-seed best track -> compacted CSR output (scan+gather).
//  k_propagate_batch, k_kf_update_batch: single-step component kernels.
#include "ckf_device.hpp"
#include "ckf_kernels.hpp"
#include "ckf_mlp.hpp"

namespace ckf {

// ---------------------------------------------------------------------------
// measurement preparation

// Pass 1, one thread per (event, module) row: validate the offsets (the
// rows must tile [0, n_meas) exactly, so every measurement gets a row), tag
// every measurement with its row, largest var0 of the row.
__global__ void k_meas_rows(int n_rows, long long n_meas, const int* __restrict__ offsets,
                            const float* __restrict__ var, int* row_of, float* maxv0, int* status) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n_rows) return;
  const int a = offsets[row], b = offsets[row + 1];
  if ((row == 0 && a != 0) || a > b || a < 0 || (long long)b > n_meas ||
      (row == n_rows - 1 && (long long)b != n_meas)) {
    atomicOr(status + CKF_STATUS_FLAGS, CKF_FLAG_BAD_OFFSETS);
    maxv0[row] = 0.f;
    return;
  }
  float mv = 0.f;
#pragma unroll 8  // eight independent loads in flight instead of one round trip per measurement
  for (int i = a; i < b; ++i) {
    row_of[i] = row;
    mv = fmaxf(mv, var[2 * i]);
  }
  maxv0[row] = mv;
}

// Sort key of a loc0: NaN sorts as +infinity (after every finite value), so
// that (key, index) is a strict total order and the ranks of a row are a
// permutation of it whatever the values.  Such a measurement never lies
// inside a chi2 window and its chi2 is never accepted.
__device__ __forceinline__ float loc0_key(float x) { return x != x ? INFINITY : x; }

// Pass 2, one thread per measurement: its rank by (loc0 key, id) inside its
// row is its sorted position (a stable segmented sort by loc0).  A
// workgroup's measurements lie in a few consecutive rows; their keys are
// read once into LDS and each thread ranks its measurement there (a row
// longer than the LDS span is ranked from memory).
constexpr int kScatterBlock = 256;
constexpr int kScatterSpan = 2304;  // keys of a workgroup's rows held in LDS

__global__ void __launch_bounds__(kScatterBlock) k_meas_scatter(long long n_meas, int n_rows,
                                                                const int* __restrict__ offsets,
                                                                const int* __restrict__ row_of,
                                                                const float* __restrict__ loc,
                                                                const float* __restrict__ var, float4* sorted,
                                                                float* key, int* id, const int* status) {
  __shared__ float s_key[kScatterSpan];
  if (status[CKF_STATUS_FLAGS] & CKF_FLAG_BAD_OFFSETS) return;  // (the same for the whole workgroup)
  const long long i0 = (long long)blockIdx.x * kScatterBlock;
  const long long i1 = min(i0 + kScatterBlock, n_meas);
  // the rows of the workgroup's measurements: [offsets[r0], offsets[r1 + 1])
  const int r0 = row_of[i0], r1 = row_of[i1 - 1];
  const long long s0 = offsets[r0], s1 = offsets[r1 + 1];
  const bool in_lds = s1 - s0 <= kScatterSpan;
  if (in_lds)
    for (long long j = s0 + threadIdx.x; j < s1; j += kScatterBlock) s_key[j - s0] = loc0_key(loc[2 * j]);
  __syncthreads();
  const long long i = i0 + threadIdx.x;
  if (i >= n_meas) return;
  const int row = row_of[i];
  if (row < 0 || row >= n_rows) return;  // (cannot happen once the offsets passed pass 1)
  const int a = offsets[row], b = offsets[row + 1];
  const float x = loc0_key(loc[2 * i]);
  int rank = 0;
  if (in_lds) {
    for (int j = a; j < b; ++j) {
      const float y = s_key[j - s0];
      rank += (y < x || (y == x && j < i)) ? 1 : 0;
    }
  } else {
#pragma unroll 8
    for (int j = a; j < b; ++j) {
      const float y = loc0_key(loc[2 * j]);
      rank += (y < x || (y == x && j < i)) ? 1 : 0;
    }
  }
  const int d = a + rank;
  sorted[d] = make_float4(x, loc[2 * i + 1], var[2 * i], var[2 * i + 1]);
  key[d] = x;
  id[d] = (int)i;
}

// ---------------------------------------------------------------------------
// per-call initialisation (a fill kernel, so the sequence can be captured)

__global__ void k_init(int n_seeds, int* res_node, int* res_nm, int* queue_head, unsigned long long* node_count,
                       int* status, long long* counters, int* n_tracks, int* offsets, int* seed_flags,
                       int* seed_cnt, int* seed_meas, int* seed_fill, unsigned long long* fin_count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_seeds) {
    res_node[i] = -1;
    res_nm[i] = 0;
    if (seed_flags) seed_flags[i] = 0;
    if (seed_cnt) {
      seed_cnt[i] = 0;
      seed_meas[i] = 0;
      seed_fill[i] = 0;
    }
  }
  if (i == 0) {
    for (int k = 0; k < kSeedQueues; ++k) queue_head[k] = 0;
    *node_count = 0ull;
    *fin_count = 0ull;
    *n_tracks = 0;
    offsets[0] = 0;
  }
  if (i < 8) status[i] = 0;
  if (counters && i < CKF_CNT_N) counters[i] = 0;
}

// ---------------------------------------------------------------------------
// candidate pool: structure-of-arrays per workgroup, two buffers (in/out)

struct Pool {
  char* base;  // records of kRecStride bytes: doubles, then ints, then floats
  int cap;
};

__device__ __forceinline__ Pool pool_at(char* base, int cap, int which) {
  Pool P;
  P.base = base + (size_t)which * cap * kRecStride;
  P.cap = cap;
  return P;
}

// Field k of record r: one per-lane base address, the field is an immediate
// offset from it.
__device__ __forceinline__ double& PDr(const Pool& P, int r, int k) {
  return reinterpret_cast<double*>(P.base + (size_t)r * kRecStride)[k];
}
__device__ __forceinline__ int& PIr(const Pool& P, int r, int k) {
  return reinterpret_cast<int*>(P.base + (size_t)r * kRecStride + PD_N * 8)[k];
}
__device__ __forceinline__ float& PFr(const Pool& P, int r, int k) {
  return reinterpret_cast<float*>(P.base + (size_t)r * kRecStride + PD_N * 8 + PI_N * 4)[k];
}

// Everything of a candidate except its covariance (loaded only when needed).
struct Light {
  double p[5];
  double chi2;
  int surf, node, nm, holes, nlist, root;
  unsigned long long mask;
  int list[kMaxList];
  float h, path;
};

__device__ __forceinline__ void load_cov(const Pool& P, int r, double* C) {
#pragma unroll
  for (int k = 0; k < 15; ++k) C[k] = PDr(P, r, PD_C + k);
}

// Store a record from its light part, with parameters/covariance/chi2/node/
// counts given separately (children differ from the parent only there).
__device__ __forceinline__ void store_rec(const Pool& P, int r, const Light& c, int slot, const double* p,
                                          const double* C, double chi2, int node, int nm, int holes) {
#pragma unroll
  for (int k = 0; k < 5; ++k) PDr(P, r, (PD_P + k)) = p[k];
#pragma unroll
  for (int k = 0; k < 15; ++k) PDr(P, r, (PD_C + k)) = C[k];
  PDr(P, r, PD_CHI2) = chi2;
  PIr(P, r, PI_SURF) = c.surf;
  PIr(P, r, PI_SLOT) = slot;
  PIr(P, r, PI_NODE) = node;
  PIr(P, r, PI_NMH) = nm | (holes << 16);
  PIr(P, r, PI_MASK_LO) = (int)(unsigned)(c.mask & 0xffffffffull);
  PIr(P, r, PI_MASK_HI) = (int)(unsigned)(c.mask >> 32);
#pragma unroll
  for (int k = 0; k < kMaxList; ++k) PIr(P, r, (PI_LIST + k)) = c.list[k];
  PIr(P, r, PI_NLIST) = c.nlist | (c.root << 8);
  PFr(P, r, PF_H) = c.h;
  PFr(P, r, PF_PATH) = c.path;
}

// ---------------------------------------------------------------------------
// wave helpers (64 lanes, one wave per workgroup)

__device__ __forceinline__ int lane_id() { return threadIdx.x; }

__device__ __forceinline__ int wave_excl_scan(int v, int& total) {
  const int lane = lane_id();
  int x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  total = __shfl(x, kWave - 1, kWave);
  return x - v;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v = max(v, __shfl_xor(v, d, kWave));
  return v;
}

__device__ __forceinline__ long long wave_sum64(long long v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Rank key: more measurements, smaller chi2 sum, fewer holes, then the
// measurement-id sequence in lexicographic order.  For equal lengths the
// histories are walked back together; the last difference met is the first
// in visiting order.  A shared ancestor ends the walk.
__device__ bool better(int nmA, double chiA, int hoA, int nodeA, int nmB, double chiB, int hoB, int nodeB,
                       const Node* nodes) {
  if (nmA != nmB) return nmA > nmB;
  if (chiA != chiB) return chiA < chiB;
  if (hoA != hoB) return hoA < hoB;
  int da = 0, db = 0;
  bool diff = false;
  for (int k = 0; k < nmA && nodeA >= 0 && nodeB >= 0 && nodeA != nodeB; ++k) {
    const int ma = nodes[nodeA].meas, mb = nodes[nodeB].meas;
    if (ma != mb) {
      da = ma;
      db = mb;
      diff = true;
    }
    nodeA = nodes[nodeA].parent;
    nodeB = nodes[nodeB].parent;
  }
  return diff && da < db;
}


// ---------------------------------------------------------------------------
// wave-cooperative module listing
//
// The lanes of a wave that need a listing have grid rows of very different
// lengths; listed one lane at a time, the wave walks its longest lane's rows
// (a quarter of the lanes busy on average).  Here the wave flattens all its
// lanes' rows into one sequence of grid entries and tests 64 entries per
// pass, each for the lane that owns it; passing modules go to the owner's
// slots in LDS and the owner keeps the kMaxList smallest (path, id).  The
// entries a lane tests are exactly those its own walk would test (the first
// kMaxCand in visiting order, counted in pairs), so the listing is the same.
constexpr int kListRows = 128;  // grid rows of one wave-wide listing
constexpr int kListRes = 6;     // passing modules kept per lane (more: the lane lists alone)

struct ListShared {
  int row_a[kListRows];        // first CSR entry of the row
  int row_pre[kListRows + 1];  // entries of the rows before it (exclusive scan)
  int row_own[kListRows];      // owning lane
  int res_n[kWave];            // passing modules per lane
  float res_s[kListRes][kWave];
  int res_m[kListRes][kWave];
};

// Called by all lanes of the wave together; lanes with want == false take
// part in the passes only.  Returns the number listed for this lane.
// `passes` (uniform) is the number of 64-entry passes the wave made.
template <bool kCount>
__device__ int list_wave(const GeomDev& g, ListShared& S, bool want, int l, V3 P, V3 T, V3 k, float s_base,
                         int exclude, float margin, int* list, int& n_tested, int& overflow, int& n_visited,
                         int& passes, int* tested_cnt) {
  const int lane = threadIdx.x;
  GridRange gr{0, -1, 0, -1};
  LayerRec Lr{};
  bool ok = false;
  if (want) {
    Lr = g.layers[l];
    ok = grid_range(Lr, P, T, gr);
  }
  int nr = (ok && gr.iw0 <= gr.iw1) ? gr.ip1 - gr.ip0 + 1 : 0;
  // lanes whose rows do not fit list alone afterwards
  int rtot;
  int rbase = wave_excl_scan(nr, rtot);
  bool alone = want && ok && rbase + nr > kListRows;
  if (alone) nr = 0;
  rbase = wave_excl_scan(nr, rtot);
  // this lane's rows: the entries its own walk visits (pairs started
  // before kMaxCand entries)
  int ovf = 0, vis = 0, before = 0;
  for (int j = 0; j < nr; ++j) {
    int a, b;
    grid_row(g, Lr, gr, gr.ip0 + j, a, b);
    const int n = b - a;
    const int take = before >= kMaxCand ? 0 : min(n, 2 * ((kMaxCand - before + 1) / 2));
    if (take < n) ovf = 1;
    vis += take;
    before += n;
    S.row_a[rbase + j] = a;
    S.row_pre[rbase + j] = take;  // counts for now, prefixes below
    S.row_own[rbase + j] = lane;
  }
  S.res_n[lane] = 0;
  __syncthreads();
  // exclusive prefix over the wave's rows (two rows per lane)
  {
    const int r0 = 2 * lane, r1 = 2 * lane + 1;
    const int c0 = r0 < rtot ? S.row_pre[r0] : 0, c1 = r1 < rtot ? S.row_pre[r1] : 0;
    int tot;
    const int e = wave_excl_scan(c0 + c1, tot);
    __syncthreads();
    if (r0 < rtot) S.row_pre[r0] = e;
    if (r1 < rtot) S.row_pre[r1] = e + c0;
    if (lane == 0) S.row_pre[rtot] = tot;
    __syncthreads();
  }
  const int total = S.row_pre[rtot];
  passes = (total + kWave - 1) / kWave;
  for (int c0 = 0; c0 < total; c0 += kWave) {
    const int c = c0 + lane;
    const bool act = c < total;
    int own = 0, q = 0;
    if (act) {  // the row holding entry c: the last row whose prefix is <= c
      int lo = 0, hi = rtot - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (S.row_pre[mid] <= c) lo = mid; else hi = mid - 1;
      }
      own = S.row_own[lo];
      q = S.row_a[lo] + (c - S.row_pre[lo]);
    }
    // the owner's trajectory (all lanes take part in the exchange)
    const V3 Po{__shfl(P.x, own), __shfl(P.y, own), __shfl(P.z, own)};
    const V3 To{__shfl(T.x, own), __shfl(T.y, own), __shfl(T.z, own)};
    const V3 ko{__shfl(k.x, own), __shfl(k.y, own), __shfl(k.z, own)};
    const float sbo = __shfl(s_base, own);
    const int exo = __shfl(exclude, own);
    if (act) {
      const int m = g.cell_mod[q];
      if (m != exo) {
        Module M;
        load_module(g, m, M);
        float cs;
        bool tested;
        if (list_probe(M, Po, To, ko, sbo, margin, cs, tested)) {
          const int slot = atomicAdd(&S.res_n[own], 1);
          if (slot < kListRes) {
            S.res_s[slot][own] = cs;
            S.res_m[slot][own] = m;
          }
        }
        if (kCount && tested) atomicAdd(&tested_cnt[own], 1);
      }
    }
  }
  __syncthreads();
  int nlist = 0;
  if (want && ok) {
    const int nres = S.res_n[lane];
    if (!alone && nres <= kListRes) {
      ListAcc acc;
      list_init(acc);
      for (int i = 0; i < nres; ++i) list_insert(acc, S.res_m[i][lane], S.res_s[i][lane]);
      nlist = list_out(acc, list);
      overflow |= ovf;
      n_visited += vis;
    } else {  // too many rows or passing modules for the shared slots
      int nt_seen = 0;  // (entries already tested in the passes were counted there)
      nlist = list_layer(g, l, P, T, k, s_base, exclude, margin, list, alone ? n_tested : nt_seen, overflow,
                         n_visited);
    }
  }
  if (want && !ok) {
#pragma unroll
    for (int q = 0; q < kMaxList; ++q) list[q] = -1;
  }
  __syncthreads();
  return nlist;
}

// ---------------------------------------------------------------------------
// wave-cooperative window scan
//
// Each crossing lane gates the measurements of its module inside its exact
// loc0 window [l, e) (found by two binary searches on the sorted row).  The
// windows differ in length from lane to lane, so the wave flattens them and
// gates 64 measurements per pass, each against its owning lane's predicted
// position and covariance; accepted ones go to the owner's slots in LDS and
// the owner keeps the smallest (chi2, id).  Every measurement of a window is
// gated exactly once, as in the lane's own scan, so the result is the same.
constexpr int kWinRes = 4;  // accepted measurements kept per lane (more: the lane scans alone)

struct WinShared {
  int pre[kWave + 1];  // measurements of the lanes before (exclusive scan)
  int start[kWave];    // first sorted position of the lane's window
  int res_n[kWave];
  double res_x2[kWinRes][kWave];
  int res_id[kWinRes][kWave];
  int res_pos[kWinRes][kWave];
};

// Insert an accepted measurement into a lane's kMaxBranch smallest (chi2, id).
__device__ __forceinline__ void acc_insert(double* acc_x2, int* acc_id, int* acc_pos, double cx, int cid, int cpos) {
#pragma unroll
  for (int k = 0; k < kMaxBranch; ++k) {
    const bool lt = cx < acc_x2[k] || (cx == acc_x2[k] && cid < acc_id[k]);
    if (lt) {
      const double tx = acc_x2[k];
      const int ti = acc_id[k], tp = acc_pos[k];
      acc_x2[k] = cx;
      acc_id[k] = cid;
      acc_pos[k] = cpos;
      cx = tx;
      cid = ti;
      cpos = tp;
    }
  }
}

// Called by all lanes together.  A lane with n > 0 owns the window of n
// sorted measurements from `start`, gated with (p0, p1) and the covariance
// entries (c00, c01, c11).  Returns the number accepted (all of them, not
// capped), or -1 when more than kWinRes were accepted (the lane then scans
// alone); acc_* receive the smallest.  `passes` (uniform): 64-entry passes.
__device__ int window_wave(WinShared& S, const Workspace& w, double chi2_max, int start, int n, double p0, double p1,
                           double c00, double c01, double c11, double* acc_x2, int* acc_id, int* acc_pos,
                           int& passes) {
  const int lane = threadIdx.x;
  int tot;
  const int e = wave_excl_scan(n, tot);
  S.pre[lane] = e;
  S.start[lane] = start;
  S.res_n[lane] = 0;
  if (lane == 0) S.pre[kWave] = tot;
  __syncthreads();
  passes = (tot + kWave - 1) / kWave;
  for (int c0 = 0; c0 < tot; c0 += kWave) {
    const int c = c0 + lane;
    const bool act = c < tot;
    int own = 0;
    if (act) {  // the last lane whose prefix is <= c
      int lo = 0, hi = kWave - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (S.pre[mid] <= c) lo = mid; else hi = mid - 1;
      }
      own = lo;
    }
    const double q0 = __shfl(p0, own), q1 = __shfl(p1, own);
    const double d00 = __shfl(c00, own), d01 = __shfl(c01, own), d11 = __shfl(c11, own);
    if (act) {
      const int i = S.start[own] + (c - S.pre[own]);
      const float4 ms = w.m_sorted[i];
      const double pq[2] = {q0, q1}, cq[6] = {d00, d01, 0.0, 0.0, 0.0, d11};
      const double x2 = chi2_of(pq, cq, (double)ms.x, (double)ms.y, (double)ms.z, (double)ms.w);
      if (x2 < chi2_max) {
        const int slot = atomicAdd(&S.res_n[own], 1);
        if (slot < kWinRes) {
          S.res_x2[slot][own] = x2;
          S.res_id[slot][own] = w.m_id[i];
          S.res_pos[slot][own] = i;
        }
      }
    }
  }
  __syncthreads();
  const int nres = S.res_n[lane];
  if (n > 0 && nres <= kWinRes)
    for (int k = 0; k < nres; ++k) acc_insert(acc_x2, acc_id, acc_pos, S.res_x2[k][lane], S.res_id[k][lane], S.res_pos[k][lane]);
  __syncthreads();
  return nres <= kWinRes ? nres : -1;
}

// tracks_per_seed = 0: append a finished candidate (seed, last node, counts,
// chi2) to the batch's list; beyond its capacity the flag is raised.
__device__ __forceinline__ void fin_append(const Workspace& w, int* status, int seed, int node, int nmh, double chi2) {
  const unsigned long long i = atomicAdd(w.fin_count, 1ull);
  if ((long long)i >= w.fin_cap) {
    atomicOr(status + CKF_STATUS_FLAGS, CKF_FLAG_FIN_CAPACITY);
    return;
  }
  w.fin_seed[i] = seed;
  w.fin_node[i] = node;
  w.fin_nmh[i] = nmh;
  w.fin_chi2[i] = chi2;
}

// C <- J C J^T on a pool record's covariance (J promoted to FP64), each new
// element stored as soon as it is formed; the three the gate needs are
// returned.  J's q/p row is the unit row (no energy loss along a leg), so
// its products are the covariance's own q/p row and column.
__device__ __forceinline__ void transport_cov_rec(const float J[5][5], const Pool& P, int r, double& c00, double& c01,
                                                  double& c11) {
  double C[15];
  load_cov(P, r, C);
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    double row[5];  // (J C)[i][:]
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < 5; ++l) s = fma((double)J[i][l], C[pk(l, k)], s);
      row[k] = i == 4 ? C[pk(4, k)] : s;  // (q/p row of J: the unit row)
    }
#pragma unroll
    for (int j = i; j < 5; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 5; ++k) s = fma(row[k], (double)J[j][k], s);
      if (j == 4) s = row[4];
      if (i == 0 && j == 0) c00 = s;
      if (i == 0 && j == 1) c01 = s;
      if (i == 1 && j == 1) c11 = s;
      PDr(P, r, PD_C + pk(i, j)) = s;
    }
  }
}

constexpr int kMaxSlots = 64;

// kCount: the instrumented variant that accumulates the work-unit counters
// (used once to measure the algorithmic work; the work is deterministic).
// kLearned: the learned-proposal form (network inference in the navigation).
// kMap: a field map (five tangent columns with field-gradient terms).
template <int kMinWaves, bool kCount, bool kLearned, bool kMap>
__global__ __launch_bounds__(kWave, kMinWaves) void k_ckf(CkfArgs A) {
  __shared__ int sh_seed[kMaxSlots], sh_event[kMaxSlots], sh_live[kMaxSlots], sh_step[kMaxSlots];
  __shared__ int sh_best_node[kMaxSlots], sh_best_nm[kMaxSlots], sh_best_holes[kMaxSlots];
  __shared__ double sh_best_chi2[kMaxSlots];
  __shared__ int sh_n_out, sh_bcast;
  __shared__ unsigned long long sh_node_base;
  __shared__ int sh_cnt[kCount ? CKF_CNT_N + 3 : 3][kWave];  // per-lane counters (kept out of registers)

  __shared__ LayerRec sh_layers[kMaxLayers];
  __shared__ int sh_order[3][kMaxLayers];
  __shared__ __align__(16) unsigned short sh_x[kLearned ? kWave * 8 : 1];  // network inputs (bf16), one row per lane
  // phase 4 work list: per output slot of a pass its parent lane and branch;
  // per parent lane its child count, node offset and accepted measurements
  // (the listing's LDS is only used during navigation: the two share space)
  __shared__ union {
    struct {
      int item[kWave * kMaxBranch];
      int kind[kWave], noff[kWave], surf[kWave];
      int acc_pos[kMaxBranch][kWave], acc_id[kMaxBranch][kWave];
      double acc_x2[kMaxBranch][kWave];
    } o;
    ListShared l;
    WinShared w;
    float lg[kLearned ? kWave * kLogitStride : 1];  // the network's logits (learned proposal)
  } sh_u;
  auto& sh_item = sh_u.o.item;
  auto& sh_kind = sh_u.o.kind;
  auto& sh_noff = sh_u.o.noff;
  auto& sh_surf = sh_u.o.surf;
  auto& sh_acc_pos = sh_u.o.acc_pos;
  auto& sh_acc_id = sh_u.o.acc_id;
  auto& sh_acc_x2 = sh_u.o.acc_x2;

  const CfgDev& cfg = A.cfg;
  const int lane = lane_id();
  // the per-layer navigation tables are small: keep them in LDS
  GeomDev g = A.g;
  if (lane < g.n_layers) sh_layers[lane] = A.g.layers[lane];
  if (lane < g.n_barrel) sh_order[0][lane] = A.g.barrel_order[lane];
  if (lane < g.n_disk_pos) sh_order[1][lane] = A.g.disk_pos[lane];
  if (lane < g.n_disk_neg) sh_order[2][lane] = A.g.disk_neg[lane];
  g.layers = sh_layers;
  g.barrel_order = sh_order[0];
  g.disk_pos = sh_order[1];
  g.disk_neg = sh_order[2];
  const int S = A.w.seeds_per_group;
  const int cap = A.w.pool_cap;
  const float margin = cfg.nav_margin;
  char* base = A.w.pools + (size_t)blockIdx.x * 2 * cap * kRecStride;
  const unsigned long long lt_mask = (1ull << lane) - 1ull;

  // Counter k of this lane.  Work counters (k < CKF_CNT_N) exist only in
  // the instrumented variant; the three status counters always exist.
  int* const cntp = &sh_cnt[0][lane];
  constexpr int kBad = CKF_CNT_N, kFailed = CKF_CNT_N + 1, kNavOvf = CKF_CNT_N + 2;
  constexpr int kStatusBase = kCount ? CKF_CNT_N : 0;
#define CNT_IDX(k) ((k) >= CKF_CNT_N ? (k) - CKF_CNT_N + kStatusBase : (k))
#define CNT_ADD(k, v)                                          \
  do {                                                         \
    if (kCount || (k) >= CKF_CNT_N) cntp[CNT_IDX(k) * kWave] += (v); \
  } while (0)
#define CNT_GET(k) cntp[CNT_IDX(k) * kWave]
#pragma unroll
  for (int k = 0; k < kStatusBase + 3; ++k) cntp[k * kWave] = 0;

  sh_seed[lane] = -1;
  sh_live[lane] = 0;
  __syncthreads();

  int cur = 0, n_in = 0;
  // invalid measurement offsets: search ranges cannot be trusted, do nothing
  bool queue_done = (((volatile int*)A.status)[CKF_STATUS_FLAGS] & CKF_FLAG_BAD_OFFSETS) != 0;
  // the part of the seed list taken from (this XCD's first), and how many
  // parts were found used up
  int part = blockIdx.x % kSeedQueues, parts_done = 0;
  for (;;) {
    if (((volatile int*)A.status)[CKF_STATUS_FLAGS] & CKF_FLAG_NODE_CAPACITY) break;
    const Pool Pin = pool_at(base, cap, cur), Pout = pool_at(base, cap, 1 - cur);

    // ---- admission: fill free seed slots from the work queue
    if (!queue_done) {
      const bool free_slot = lane < S && sh_seed[lane] < 0;
      const unsigned long long fm = __ballot(free_slot);
      const int nfree = __popcll(fm);
      if (nfree > 0) {
        if (lane == 0) sh_bcast = atomicAdd(A.w.queue_head + part, nfree);
        __syncthreads();
        const int start = sh_bcast;
        __syncthreads();
        const long long p0 = (long long)part * A.s.n / kSeedQueues, p1 = (long long)(part + 1) * A.s.n / kSeedQueues;
        const long long pos = p0 + start + __popcll(fm & lt_mask);
        if (p0 + start + nfree >= p1) {  // this part is used up: the next one
          part = (part + 1) % kSeedQueues;
          if (++parts_done == kSeedQueues) queue_done = true;
        }
        bool ok = free_slot && pos < p1;
        const int seed = ok ? (int)pos : 0;
        if (ok) {
          const int sf = A.s.surface[seed], ev = A.s.event[seed];
          bool good = sf >= 0 && sf < g.n_surfaces && ev >= 0 && ev < A.m.n_events;
          for (int k = 0; k < 5; ++k) good = good && isfinite(A.s.params[5 * seed + k]);
          for (int k = 0; k < 15; ++k) good = good && isfinite(A.s.cov[15 * seed + k]);
          good = good && A.s.params[5 * seed + 4] != 0.0;
          if (!good) {
            A.w.res_node[seed] = -1;
            A.w.res_nm[seed] = 0;
            CNT_ADD(kBad, 1);
            ok = false;
          }
        }
        const unsigned long long om = __ballot(ok);
        if (ok) {
          const int r = n_in + __popcll(om & lt_mask);
          sh_seed[lane] = seed;
          sh_event[lane] = A.s.event[seed];
          sh_live[lane] = 1;
          sh_step[lane] = 0;
          sh_best_node[lane] = -1;
          sh_best_nm[lane] = -1;
          sh_best_holes[lane] = 0;
          sh_best_chi2[lane] = 0.0;
          Light c;
          double p[5], C[15];
#pragma unroll
          for (int k = 0; k < 5; ++k) p[k] = A.s.params[5 * seed + k];
#pragma unroll
          for (int k = 0; k < 15; ++k) C[k] = A.s.cov[15 * seed + k];
          c.surf = A.s.surface[seed];
          c.mask = 0;  // the seed's own layer is marked at its first step (its module is loaded there)
#pragma unroll
          for (int k = 0; k < kMaxList; ++k) c.list[k] = -1;
          c.nlist = 0;
          c.root = 1;
          c.h = cfg.step_max;
          c.path = 0.f;
          store_rec(Pin, r, c, lane, p, C, 0.0, -1, 0, 0);
        }
        n_in += __popcll(om);
        __syncthreads();
      }
    }
    if (n_in == 0) {
      if (queue_done) break;
      continue;
    }

    // ---- one step of every live candidate
    const long long t_step = kCount ? clock64() : 0;
    sh_live[lane] = 0;
    if (lane == 0) sh_n_out = 0;
    __syncthreads();
    for (int b0 = 0; b0 < n_in; b0 += kWave) {
      const int r = b0 + lane;
      int slot = -1;
      if (r < n_in) slot = PIr(Pin, r, PI_SLOT);
      const bool act = slot >= 0;
      // outcome of this step: 0 nothing (dropped or idle), 1 the candidate
      // continues as it is, 2 it crossed a module (search), 3 it finished
      int outcome = 0;
      bool moved = false;
      float J[5][5];
      int c_list = 0, c_next = 0, c_land = 0, c_win = 0;  // loop iterations of this lane (instrumented run)
      int c_list_passes = 0, c_win_passes = 0;             // the wave's listing and window passes
      long long t_phase = kCount ? clock64() : 0;
      if (kCount && lane == 0) CNT_ADD(CKF_CNT_CHUNKS, 1);

      // ---- phase 1: navigation and the propagation leg (FP32); the changed
      // navigation state is written back into the candidate's own record.
      // Stage A: the next layer; then (learned form) the network for all
      // lanes together; stage B: module listing and the leg.
      double p[5];
      int surf = -1, nlist = 0, root = 0;
      unsigned long long mask = 0;
      int list[kMaxList];
      float h = 0.f, path = 0.f;
      Module Am;
      LegT<kMap ? 5 : 3> L;
      V3 uA, vA, origin, Pl, Tl;
      bool go = false, need_list = false;
      int lay = 0, excl = -1, nb_slot = -1, nb_row = -1;
      Window win{0, 0, 0.f, 0.f};
      float sb = 0.f;
      long long t_nav = 0;
      int prop[3] = {-1, -1, -1};
      bool confident = false;
      int pf_a = 0, pf_b = 0;  // the searched row's measurement range and largest var0 (loaded early)
      float pf_mv = 0.f;
      V3 kl{0.f, 0.f, 0.f};
      auto stage_a = [&]() {
        CNT_ADD(CKF_CNT_STEPS, 1);
#pragma unroll
        for (int k = 0; k < 5; ++k) p[k] = PDr(Pin, r, (PD_P + k));
        surf = PIr(Pin, r, PI_SURF);
        const int nlp = PIr(Pin, r, PI_NLIST);
        nlist = nlp & 0xff;
        root = nlp >> 8;
        mask = (unsigned long long)(unsigned)PIr(Pin, r, PI_MASK_LO) |
               ((unsigned long long)(unsigned)PIr(Pin, r, PI_MASK_HI) << 32);
#pragma unroll
        for (int k = 0; k < kMaxList; ++k) list[k] = PIr(Pin, r, (PI_LIST + k));
        h = PFr(Pin, r, PF_H);
        path = PFr(Pin, r, PF_PATH);
        if (kCount) t_nav = clock64();
        // the start module and the leg's initial free state are the same for
        // the seed's listing, the next-layer search and the leg itself
        load_module(g, surf, Am);
        leg_start(Am, p, L, uA, vA);
        origin = ld3(Am.c);
        if (root) mask |= 1ull << Am.layer;
        go = !root;
        // one listing call for both the seed's own layer and a newly found
        // layer, so that a wave holding both kinds of lanes lists once
        need_list = root;
        lay = Am.layer;
        excl = surf;
        Pl = origin + L.r;
        Tl = L.T;
        if (root) {
          outcome = 2;
        } else if (nlist == 0) {
          // learned: the module's neighbour-table entries, requested before
          // the next-layer search so that they arrive during it
          int nb_l[kMaxNext], nb_r[kMaxNext];
          if (kLearned) {
#pragma unroll
            for (int q = 0; q < kMaxNext; ++q) {
              nb_l[q] = g.nb_next[surf * kMaxNext + q];
              nb_r[q] = g.nb_row[surf * kMaxNext + q];
            }
          }
          const V3 Bf = field_at<kMap>(A.f, Pl);
          const Helix H = make_helix(Pl, L.T, L.lam, Bf);
          float sL;
          CNT_ADD(CKF_CNT_NAV, 1);
          const long long t_next = kCount ? clock64() : 0;
          V3 Pn, Tn;  // the crossing of the layer found (its point and direction)
          const int nl = next_layer(g, H, mask, cfg.path_max - path, sL, Pn, Tn, c_next);
          if (kCount) CNT_ADD(CKF_CNT_CYC_NEXT, (int)(clock64() - t_next));
          if (nl < 0) {
            outcome = 3;
            go = false;
          } else {
            mask |= 1ull << nl;
            Pl = Pn;
            Tl = Tn;
            need_list = true;
            lay = nl;
            excl = -1;
            sb = sL;
            if (kLearned) {
#pragma unroll
              for (int q = kMaxNext - 1; q >= 0; --q)  // the first slot holding layer nl
                if (nb_l[q] == nl) {
                  nb_slot = q;
                  nb_row = nb_r[q];
                }
              if (nb_slot >= 0 && !crossing_window(g.layers[nl], g.nb_anc[nb_row], Pl, win)) nb_slot = -1;
              if (nb_slot >= 0) {  // the network input goes to LDS now
                float f[7];
                mlp_features(g.layers[nl], nl, g.n_layers, win, Pl, Tl, L.lam, f);
                *reinterpret_cast<uint4*>(&sh_x[lane * 8]) =
                    make_uint4(cvt_pk_bf16(f[0], f[1]), cvt_pk_bf16(f[2], f[3]), cvt_pk_bf16(f[4], f[5]),
                               cvt_pk_bf16(f[6], 0.f));
              }
            }
          }
        }
        // the listing's curvature term at its base point
        if (need_list) kl = (kKappa * L.lam) * cross(Tl, field_at<kMap>(A.f, Pl));
      };
      // learned proposal: the network for every lane that found a next layer
      // listed in its module's neighbour table, 16 rows per MFMA pass
      auto proposal = [&]() {
        const unsigned long long wm = __ballot(nb_slot >= 0);
        if (wm) {
          if (nb_slot < 0) {
            *reinterpret_cast<uint4*>(&sh_x[lane * 8]) = make_uint4(0u, 0u, 0u, 0u);
          }
          __syncthreads();
          const int q4 = 4 * (lane >> 4);
          // the four 16-row blocks together: each weight tile is read once
          // per pass; the logits go to LDS, one row per lane
          {
            bf16x4 xb[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
              // features q4..q4+3 of the row (8-byte aligned; zero beyond the 8 stored)
              const int src = (16 * h + (lane & 15)) * 8 + q4;
              xb[h] = as_bf16x4(q4 < 8 ? *reinterpret_cast<const uint2*>(&sh_x[src]) : make_uint2(0u, 0u));
            }
            f32x4 out[4][2];
            mlp_blocks<4>(A.model, xb, lane, out);
            if (kCount && lane == 0) CNT_ADD(CKF_CNT_MLP_BLOCKS, 4);
#pragma unroll
            for (int h = 0; h < 4; ++h) logits_to_lds(out[h], h, lane, sh_u.lg);
          }
          __syncthreads();
          if (nb_slot >= 0) {
            CNT_ADD(CKF_CNT_MLP_ROWS, 1);
            RowTop rt;
            const float conf = row_top3_values(&sh_u.lg[lane * kLogitStride], cfg.topk, rt);
            confident = conf >= cfg.min_prob;
            if (confident) {
              int cls[3];
              row_top3_classes(rt, cls);
#pragma unroll
              for (int k = 0; k < 3; ++k)  // (a class outside 0..31 only if the logits were not finite)
                if (k < cfg.topk && cls[k] >= 0 && cls[k] < kNeighbours)
                  prop[k] = window_module(g, nb_row, win, cls[k]);
            }
          }
          __syncthreads();
        }
      };
      // stage B1: the learned proposal's listing (confident lanes); which
      // lanes still need the geometric listing
      bool want_geo = false;
      int nt = 0, ovf = 0;
      auto stage_b1 = [&]() {
        if (need_list) {
          bool listed = false;
          if (kLearned && confident) {
            // the proposed modules through the same listing test
            ListAcc acc;
            list_init(acc);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              if (prop[k] < 0) continue;
              Module Mp;
              load_module(g, prop[k], Mp);
              list_test(acc, prop[k], Mp, Pl, Tl, kl, sb, margin, nt);
            }
            const int np = list_out(acc, list);
            if (np > 0) {
              listed = true;
              nlist = np;
              CNT_ADD(CKF_CNT_PROPOSALS, 1);
              if (kCount) {  // audit against the geometric listing
                int full[kMaxList];
                int nt2 = 0, ovf2 = 0;
                int nv2 = 0;
                const int nf = list_layer(g, lay, Pl, Tl, kl, sb, excl, margin, full, nt2, ovf2, nv2);
                bool same = nf == np;
#pragma unroll
                for (int k = 0; k < kMaxList; ++k) same = same && full[k] == list[k];
                if (!same) {
                  CNT_ADD(CKF_CNT_PROPOSAL_MISS, 1);
                  if (A.seed_flags) A.seed_flags[sh_seed[slot]] = 1;
                }
              }
            }
          }
          want_geo = !listed;
        }
      };
      // the geometric listing, all lanes of the wave together
      auto listing = [&]() {
        int passes = 0;
        const int nl_geo = list_wave<kCount>(g, sh_u.l, act && want_geo, lay, Pl, Tl, kl, sb, excl, margin, list,
                                             nt, ovf, c_list, passes,
                                             kCount ? &sh_cnt[CNT_IDX(CKF_CNT_NAV_MODULES)][0] : nullptr);
        if (act && want_geo) nlist = nl_geo;
        if (kCount && lane == 0) c_list_passes += passes;
      };
      // stage B2: the leg to the next listed module.  The start state is
      // rebuilt from the record rather than kept in registers across the
      // network and the listing.
      auto stage_b2 = [&]() {
        if (root) {  // the searched row (the seed's own module), loaded ahead of the search
          const int row = sh_event[slot] * g.n_surfaces + surf;
          pf_a = A.m.offsets[row];
          pf_b = A.m.offsets[row + 1];
          pf_mv = A.w.row_maxvar0[row];
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) p[k] = PDr(Pin, r, (PD_P + k));
        load_module(g, surf, Am);
        leg_start(Am, p, L, uA, vA);
        origin = ld3(Am.c);
        if (need_list) {
          CNT_ADD(CKF_CNT_NAV_MODULES, nt);
          CNT_ADD(kNavOvf, ovf);
          if (!root && nlist == 0) {
            outcome = 1;  // the layer is crossed in a gap
            go = false;
          }
        }
        if (!root) {
          if (kCount) {  // navigation time of this lane (summed over lanes, divided later)
            const long long t = clock64();
            CNT_ADD(CKF_CNT_CYC_NAV, (int)(t - t_nav));
            t_nav = t;
          }
          if (go) {
            const int m = list[0];
#pragma unroll
            for (int k = 0; k < kMaxList - 1; ++k) list[k] = list[k + 1];
            list[kMaxList - 1] = -1;
            --nlist;
            Module Bm;
            load_module(g, m, Bm);
            {  // the row searched if the leg crosses m, loaded while the leg is propagated
              const int row = sh_event[slot] * g.n_surfaces + m;
              pf_a = A.m.offsets[row];
              pf_b = A.m.offsets[row + 1];
              pf_mv = A.w.row_maxvar0[row];
            }
            const V3 dB = ld3(Bm.c) - origin;
            LegStats ls{0, 0};
            CNT_ADD(CKF_CNT_LEGS, 1);
            bool good = land<kMap>(L, origin, dB, ld3(Bm.n), A.f, cfg, h, path, ls);
            CNT_ADD(CKF_CNT_RK_TRIALS, ls.trials);
            c_land = ls.trials + 1;
            CNT_ADD(CKF_CNT_RK_REJECTS, ls.rejects);
            if (good) {
              double pn[5];
              leg_end(L, uA, vA, Bm, dB, field_at<kMap>(A.f, origin + L.r), p[4], pn, J);
#pragma unroll
              for (int k = 0; k < 5; ++k) good = good && isfinite(pn[k]);
#pragma unroll
              for (int k = 0; k < 5; ++k) p[k] = pn[k];
            }
            if (!good) {
              CNT_ADD(kFailed, 1);  // dropped
            } else {
              moved = true;
              surf = m;
              outcome = (fabs(p[0]) <= (double)Bm.hw0 && fabs(p[1]) <= (double)Bm.hw1) ? 2 : 1;
            }
          }
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) PDr(Pin, r, (PD_P + k)) = p[k];
        PIr(Pin, r, PI_SURF) = surf;
        PIr(Pin, r, PI_NLIST) = nlist;  // root flag cleared
        PIr(Pin, r, PI_MASK_LO) = (int)(unsigned)(mask & 0xffffffffull);
        PIr(Pin, r, PI_MASK_HI) = (int)(unsigned)(mask >> 32);
#pragma unroll
        for (int k = 0; k < kMaxList; ++k) PIr(Pin, r, (PI_LIST + k)) = list[k];
        PFr(Pin, r, PF_H) = h;
        PFr(Pin, r, PF_PATH) = path;
      };
      if (act) stage_a();
      // the network runs with all lanes together between the stages
      if (kLearned) proposal();
      if (act) stage_b1();
      listing();
      if (act) stage_b2();

      if (kCount && lane == 0) {
        const long long t = clock64();
        CNT_ADD(CKF_CNT_CYC_LEG, (int)(t - t_phase));
        t_phase = t;
      }
      if (kCount) __syncthreads();
      // ---- phase 2: covariance transport (FP64), search and gate
      double acc_x2[kMaxBranch];
      int acc_id[kMaxBranch], acc_pos[kMaxBranch];
#pragma unroll
      for (int k = 0; k < kMaxBranch; ++k) {
        acc_x2[k] = INFINITY;
        acc_id[k] = 0x7fffffff;
        acc_pos[k] = 0;
      }
      int n_acc = 0;
      // phase 2a (per lane): the covariance transport, stored back into the
      // record, and the crossing lanes' exact loc0 windows
      int w_start = 0, w_n = 0, surf2 = -1;
      double g0 = 0.0, g1 = 0.0, k00 = 0.0, k01 = 0.0, k11 = 0.0;
      if (outcome == 1 || outcome == 2) {
        if (moved) {
          transport_cov_rec(J, Pin, r, k00, k01, k11);
        } else {
          k00 = PDr(Pin, r, PD_C + 0);
          k01 = PDr(Pin, r, PD_C + 1);
          k11 = PDr(Pin, r, PD_C + 5);
        }
        if (outcome == 2) {
          CNT_ADD(CKF_CNT_CROSSED, 1);
          g0 = PDr(Pin, r, PD_P + 0);
          g1 = PDr(Pin, r, PD_P + 1);
          surf2 = PIr(Pin, r, PI_SURF);
          const int a = pf_a, b = pf_b;  // the row of surf2 (the seed's module, or the leg's target)
          if (b > a) {
            const double wd = sqrt(cfg.chi2_max * (k00 + (double)pf_mv));
            const float lo = (float)(g0 - wd) - 1e-3f, hi = (float)(g0 + wd) + 1e-3f;
            // the first position with loc0 >= lo and the first with loc0 >
            // hi: two binary searches side by side, so that their loads are
            // in flight together
            int l = a, u = b, l2 = a, u2 = b;
            while (l < u || l2 < u2) {
              const int m1 = (l + u) >> 1, m2 = (l2 + u2) >> 1;
              const float k1 = l < u ? A.w.m_key[m1] : 0.f, k2 = l2 < u2 ? A.w.m_key[m2] : 0.f;
              if (l < u) {
                if (k1 < lo) l = m1 + 1; else u = m1;
              }
              if (l2 < u2) {
                if (k2 <= hi) l2 = m2 + 1; else u2 = m2;
              }
            }
            w_start = l;
            w_n = l2 - l;
            CNT_ADD(CKF_CNT_CHI2, w_n);
          }
        }
      }
      // phase 2b (the wave together): the windows' gates
      {
        int passes = 0;
        n_acc = window_wave(sh_u.w, A.w, cfg.chi2_max, w_start, w_n, g0, g1, k00, k01, k11, acc_x2, acc_id,
                            acc_pos, passes);
        if (kCount) {
          c_win = w_n;
          if (lane == 0) c_win_passes += passes;
        }
      }
      // phase 2c (per lane): a lane with more accepted measurements than the
      // shared slots scans its window alone; holes
      if (outcome == 2) {
        if (n_acc < 0) {
          n_acc = 0;
#pragma unroll
          for (int k = 0; k < kMaxBranch; ++k) {
            acc_x2[k] = INFINITY;
            acc_id[k] = 0x7fffffff;
            acc_pos[k] = 0;
          }
          for (int i = w_start; i < w_start + w_n; ++i) {
            const float4 ms = A.w.m_sorted[i];
            const double pq[2] = {g0, g1}, cq[6] = {k00, k01, 0.0, 0.0, 0.0, k11};
            const double x2 = chi2_of(pq, cq, (double)ms.x, (double)ms.y, (double)ms.z, (double)ms.w);
            if (x2 < cfg.chi2_max) {
              acc_insert(acc_x2, acc_id, acc_pos, x2, A.w.m_id[i], i);
              ++n_acc;
            }
          }
        }
        n_acc = min(n_acc, cfg.branches);
        if (n_acc == 0) {  // a hole
          CNT_ADD(CKF_CNT_HOLES, 1);
          const int nmh = PIr(Pin, r, PI_NMH) + (1 << 16);
          PIr(Pin, r, PI_NMH) = nmh;
          if (cfg.material) {
            double p[5], C[15];
#pragma unroll
            for (int k = 0; k < 5; ++k) p[k] = PDr(Pin, r, (PD_P + k));
            load_cov(Pin, r, C);
            Module M;
            load_module_ms(g, surf2, M);
            apply_ms(M, cfg.mass, p, C);
            CNT_ADD(CKF_CNT_MS, 1);
#pragma unroll
            for (int k = 0; k < 15; ++k) PDr(Pin, r, (PD_C + k)) = C[k];
          }
          outcome = (nmh >> 16) > cfg.max_holes ? 3 : 1;
        }
      } else {
        n_acc = 0;
      }

      if (kCount && lane == 0) {
        const long long t = clock64();
        CNT_ADD(CKF_CNT_CYC_SEARCH, (int)(t - t_phase));
        t_phase = t;
      }
      if (kCount) {  // loop divergence: lane iterations and the wave's longest lane
        CNT_ADD(CKF_CNT_LIST_LANE, c_list);
        CNT_ADD(CKF_CNT_NEXT_LANE, c_next);
        CNT_ADD(CKF_CNT_LAND_LANE, c_land);
        CNT_ADD(CKF_CNT_WIN_LANE, c_win);
        const int m1 = wave_max(c_next), m2 = wave_max(c_land);
        if (lane == 0) {
          CNT_ADD(CKF_CNT_LIST_WAVE, c_list_passes);
          CNT_ADD(CKF_CNT_NEXT_WAVE, m1);
          CNT_ADD(CKF_CNT_LAND_WAVE, m2);
          CNT_ADD(CKF_CNT_WIN_WAVE, c_win_passes);
        }
      }
      // ---- phase 3: slots for the outputs (wave scan) and history nodes
      const int n_out = outcome == 1 ? 1 : (outcome == 2 ? n_acc : 0);
      const int n_kf = outcome == 2 ? n_acc : 0;
      int tot_out;
      const int off = wave_excl_scan(n_out, tot_out);
      const int pos0 = sh_n_out + off;
      int tot_nodes;
      const int noff = wave_excl_scan(n_kf, tot_nodes);
      __syncthreads();
      if (lane == 0) {
        sh_n_out += tot_out;
        sh_node_base = tot_nodes > 0 ? atomicAdd(A.w.node_count, (unsigned long long)tot_nodes) : 0ull;
      }
      __syncthreads();

      // ---- phase 4: outputs, one output record per lane and round: the
      // parents' accepted measurements go through LDS, so a parent with
      // three children costs three lanes instead of three rounds of the wave
      sh_kind[lane] = act ? n_kf : 0;
      sh_noff[lane] = noff;
      sh_surf[lane] = surf2;
#pragma unroll
      for (int j = 0; j < kMaxBranch; ++j) {
        sh_acc_pos[j][lane] = acc_pos[j];
        sh_acc_id[j][lane] = acc_id[j];
        sh_acc_x2[j][lane] = acc_x2[j];
      }
      for (int j = 0; j < n_out; ++j) sh_item[off + j] = lane | (j << 8);
      __syncthreads();
      const int out_base = pos0 - off;  // this pass's first output slot (uniform)
      for (int c = lane; c < tot_out; c += kWave) {
        const int it = sh_item[c];
        const int src = it & 0xff, j = it >> 8;
        const int rs = b0 + src, q = out_base + c;
        const int nkf = sh_kind[src];
        const int pslot = PIr(Pin, rs, PI_SLOT);
        if (nkf == 0) {  // the record moves on unchanged: 14 16-byte words (records are 16-byte aligned)
          const float4* from = reinterpret_cast<const float4*>(Pin.base + (size_t)rs * kRecStride);
          float4* to = reinterpret_cast<float4*>(Pout.base + (size_t)q * kRecStride);
#pragma unroll
          for (int k = 0; k < (int)(kRecStride / 16); ++k) to[k] = from[k];
        } else {  // the Kalman-updated child for the parent's j-th accepted measurement
          const long long nd = (long long)sh_node_base + sh_noff[src];
          const bool room = nd + nkf <= A.w.node_cap;
          if (!room && j == 0) atomicOr(A.status + CKF_STATUS_FLAGS, CKF_FLAG_NODE_CAPACITY);
          // the parent's module (from its search) and its normal and
          // thickness for the scattering, requested with the parent's state
          const int surf = sh_surf[src];
          Module M;
          if (cfg.material) load_module_ms(g, surf, M);
          double p[5], C[15];
#pragma unroll
          for (int k = 0; k < 5; ++k) p[k] = PDr(Pin, rs, (PD_P + k));
          load_cov(Pin, rs, C);
          const int i = sh_acc_pos[j][src];
          double pc[5], Cc[15];
          const float4 ms = A.w.m_sorted[i];
          kf_update(p, C, (double)ms.x, (double)ms.y, (double)ms.z, (double)ms.w, pc, Cc);
          CNT_ADD(CKF_CNT_KF, 1);
          if (room) {
            Node* np = A.w.nodes + nd + j;
            np->parent = PIr(Pin, rs, PI_NODE);
            np->meas = sh_acc_id[j][src];
            np->surface = surf;
            np->pad = 0;
#pragma unroll
            for (int k = 0; k < 5; ++k) np->p[k] = pc[k];
#pragma unroll
            for (int k = 0; k < 15; ++k) np->cov[k] = Cc[k];
          }
          if (cfg.material) {
            apply_ms(M, cfg.mass, pc, Cc);
            CNT_ADD(CKF_CNT_MS, 1);
          }
#pragma unroll
          for (int k = 0; k < 5; ++k) PDr(Pout, q, (PD_P + k)) = pc[k];
#pragma unroll
          for (int k = 0; k < 15; ++k) PDr(Pout, q, (PD_C + k)) = Cc[k];
          PDr(Pout, q, PD_CHI2) = PDr(Pin, rs, PD_CHI2) + sh_acc_x2[j][src];
          PIr(Pout, q, PI_NODE) = room ? (int)(nd + j) : -1;
          PIr(Pout, q, PI_NMH) = PIr(Pin, rs, PI_NMH) + 1;
#pragma unroll
          for (int k = 0; k < PI_N; ++k)
            if (k != PI_NODE && k != PI_NMH) PIr(Pout, q, k) = PIr(Pin, rs, k);
#pragma unroll
          for (int k = 0; k < PF_N; ++k) PFr(Pout, q, k) = PFr(Pin, rs, k);
        }
        atomicAdd(&sh_live[pslot], 1);
      }
      // ---- finished candidates update their seed's best (one lane at a time)
      if (cfg.all_tracks) {  // every finished candidate is kept (no per-seed best)
        if (outcome == 3) {
          CNT_ADD(CKF_CNT_FINISHED, 1);
          const int nmh = PIr(Pin, r, PI_NMH);
          if ((nmh & 0xffff) >= cfg.min_meas)
            fin_append(A.w, A.status, sh_seed[slot], PIr(Pin, r, PI_NODE), nmh, PDr(Pin, r, PD_CHI2));
        }
      }
      // the finished records' counts are read by all their lanes at once;
      // the comparisons with the seed's best then go one lane at a time
      int f_nm = 0, f_ho = 0, f_nd = -1;
      double f_ch = 0.0;
      if (!cfg.all_tracks && outcome == 3) {
        CNT_ADD(CKF_CNT_FINISHED, 1);
        const int nmh = PIr(Pin, r, PI_NMH);
        f_nm = nmh & 0xffff;
        f_ho = nmh >> 16;
        f_nd = PIr(Pin, r, PI_NODE);
        f_ch = PDr(Pin, r, PD_CHI2);
      }
      unsigned long long fm = cfg.all_tracks ? 0ull : __ballot(outcome == 3 && f_nm >= cfg.min_meas);
      while (fm) {
        const int l = __ffsll((long long)fm) - 1;
        fm &= fm - 1;
        if (lane == l) {
          const int nm = f_nm, ho = f_ho, nd = f_nd;
          const double ch = f_ch;
          if (sh_best_node[slot] < 0 || better(nm, ch, ho, nd, sh_best_nm[slot], sh_best_chi2[slot],
                                               sh_best_holes[slot], sh_best_node[slot], A.w.nodes)) {
            sh_best_node[slot] = nd;
            sh_best_nm[slot] = nm;
            sh_best_chi2[slot] = ch;
            sh_best_holes[slot] = ho;
          }
        }
        __syncthreads();
      }
      if (kCount && lane == 0) CNT_ADD(CKF_CNT_CYC_OUT, (int)(clock64() - t_phase));
    }
    __syncthreads();
    const int n_out_total = sh_n_out;

    // ---- pruning: a seed keeps its max_live best candidates (rank key)
    {
      const bool over = lane < S && sh_seed[lane] >= 0 && sh_live[lane] > cfg.max_live;
      if (__ballot(over)) {
        if (over) {
          int kept = 0;
          for (int ra = 0; ra < n_out_total; ++ra) {
            if (PIr(Pout, ra, PI_SLOT) != lane && PIr(Pout, ra, PI_SLOT) != -2 - lane) continue;
            const int nmh_a = PIr(Pout, ra, PI_NMH);
            const double ch_a = PDr(Pout, ra, PD_CHI2);
            const int nd_a = PIr(Pout, ra, PI_NODE);
            int n_better = 0;
            for (int rb = 0; rb < n_out_total; ++rb) {
              if (rb == ra) continue;
              const int sb = PIr(Pout, rb, PI_SLOT);
              if (sb != lane && sb != -2 - lane) continue;
              const int nmh_b = PIr(Pout, rb, PI_NMH);
              if (better(nmh_b & 0xffff, PDr(Pout, rb, PD_CHI2), nmh_b >> 16, PIr(Pout, rb, PI_NODE),
                         nmh_a & 0xffff, ch_a, nmh_a >> 16, nd_a, A.w.nodes))
                ++n_better;
            }
            if (n_better >= cfg.max_live) {
              PIr(Pout, ra, PI_SLOT) = -2 - lane;  // pruned (still ranked by the others)
              CNT_ADD(CKF_CNT_PRUNED, 1);
            } else {
              ++kept;
            }
          }
          // pruned records become dead
          for (int ra = 0; ra < n_out_total; ++ra)
            if (PIr(Pout, ra, PI_SLOT) == -2 - lane) PIr(Pout, ra, PI_SLOT) = -1;
          sh_live[lane] = kept;
        }
      }
      __syncthreads();
    }

    // ---- step budget: the survivors of a seed's last step are finished
    {
      bool exhausted = false;
      if (lane < S && sh_seed[lane] >= 0) {
        sh_step[lane] += 1;
        exhausted = sh_step[lane] >= cfg.max_steps;
      }
      __syncthreads();
      if (__ballot(exhausted)) {
        for (int b0 = 0; b0 < n_out_total; b0 += kWave) {
          const int r = b0 + lane;
          bool f = false;
          int sl = -1, nm = 0, ho = 0, nd = -1;
          double ch = 0.0;
          if (r < n_out_total) {
            sl = PIr(Pout, r, PI_SLOT);
            if (sl >= 0 && sh_step[sl] >= cfg.max_steps) {
              f = true;
              const int nmh = PIr(Pout, r, PI_NMH);
              nm = nmh & 0xffff;
              ho = nmh >> 16;
              nd = PIr(Pout, r, PI_NODE);
              ch = PDr(Pout, r, PD_CHI2);
              PIr(Pout, r, PI_SLOT) = -1;
            }
          }
          if (cfg.all_tracks && f) {
            CNT_ADD(CKF_CNT_FINISHED, 1);
            if (nm >= cfg.min_meas) fin_append(A.w, A.status, sh_seed[sl], nd, nm | (ho << 16), ch);
          }
          unsigned long long fm = cfg.all_tracks ? 0ull : __ballot(f);
          while (fm) {
            const int l = __ffsll((long long)fm) - 1;
            fm &= fm - 1;
            if (lane == l) {
              CNT_ADD(CKF_CNT_FINISHED, 1);
              if (nm >= cfg.min_meas && (sh_best_node[sl] < 0 || better(nm, ch, ho, nd, sh_best_nm[sl],
                                                                          sh_best_chi2[sl], sh_best_holes[sl],
                                                                          sh_best_node[sl], A.w.nodes))) {
                sh_best_node[sl] = nd;
                sh_best_nm[sl] = nm;
                sh_best_chi2[sl] = ch;
                sh_best_holes[sl] = ho;
              }
            }
            __syncthreads();
          }
        }
        if (exhausted) sh_live[lane] = 0;
      }
      __syncthreads();
    }

    // ---- seeds without live candidates are done: publish their best
    if (lane < S && sh_seed[lane] >= 0 && sh_live[lane] == 0) {
      const int seed = sh_seed[lane];
      A.w.res_node[seed] = sh_best_node[lane];
      A.w.res_nm[seed] = sh_best_node[lane] >= 0 ? sh_best_nm[lane] : 0;
      A.w.res_holes[seed] = sh_best_holes[lane];
      A.w.res_chi2[seed] = sh_best_chi2[lane];
      sh_seed[lane] = -1;
    }
    __syncthreads();
    if (kCount && lane == 0) CNT_ADD(CKF_CNT_CYC_STEP, (int)(clock64() - t_step));
    cur = 1 - cur;
    n_in = n_out_total;
  }

  // ---- counters and status
  if (kCount && A.counters) {
#pragma unroll
    for (int k = 0; k < CKF_CNT_N; ++k) {
      const long long t = wave_sum64((long long)CNT_GET(k));
      if (lane == 0 && t) atomicAdd((unsigned long long*)(A.counters + k), (unsigned long long)t);
    }
  }
  const long long tb = wave_sum64(CNT_GET(kBad)), tf = wave_sum64(CNT_GET(kFailed)),
                  tn = wave_sum64(CNT_GET(kNavOvf));
  if (lane == 0) {
    if (tb) atomicAdd(A.status + CKF_STATUS_BAD_SEEDS, (int)tb);
    if (tf) atomicAdd(A.status + CKF_STATUS_FAILED_LEGS, (int)tf);
    if (tn) atomicAdd(A.status + CKF_STATUS_NAV_OVERFLOW, (int)tn);
  }
#undef CNT_ADD
#undef CNT_GET
#undef CNT_IDX
}

// ---------------------------------------------------------------------------
// output: per-seed best -> compacted CSR (block scan, scan of block sums,
// gather)

constexpr int kScanBlock = 256;

__device__ __forceinline__ void block_scan2(int a, int b, int& ea, int& eb, int& ta, int& tb) {
  __shared__ int sa[kScanBlock], sb[kScanBlock];
  const int t = threadIdx.x;
  sa[t] = a;
  sb[t] = b;
  __syncthreads();
  for (int d = 1; d < kScanBlock; d <<= 1) {
    const int xa = t >= d ? sa[t - d] : 0, xb = t >= d ? sb[t - d] : 0;
    __syncthreads();
    sa[t] += xa;
    sb[t] += xb;
    __syncthreads();
  }
  ea = sa[t] - a;
  eb = sb[t] - b;
  ta = sa[kScanBlock - 1];
  tb = sb[kScanBlock - 1];
  __syncthreads();
}

__global__ __launch_bounds__(kScanBlock) void k_out_count(int n, const int* res_node, const int* res_nm, int* bs_a,
                                                          int* bs_b) {
  const int s = blockIdx.x * kScanBlock + threadIdx.x;
  const int has = s < n && res_node[s] >= 0 ? 1 : 0;
  const int nm = has ? res_nm[s] : 0;
  int ea, eb, ta, tb;
  block_scan2(has, nm, ea, eb, ta, tb);
  if (threadIdx.x == 0) {
    bs_a[blockIdx.x] = ta;
    bs_b[blockIdx.x] = tb;
  }
}

__global__ __launch_bounds__(kScanBlock) void k_out_scan_blocks(int nb, int* bs_a, int* bs_b, int* status,
                                                                int* n_tracks, int cap_tracks, long long cap_meas,
                                                                int* offsets, const unsigned long long* node_count) {
  int carry_a = 0, carry_b = 0;
  for (int b0 = 0; b0 < nb; b0 += kScanBlock) {
    const int i = b0 + threadIdx.x;
    const int a = i < nb ? bs_a[i] : 0, b = i < nb ? bs_b[i] : 0;
    int ea, eb, ta, tb;
    block_scan2(a, b, ea, eb, ta, tb);
    if (i < nb) {
      bs_a[i] = carry_a + ea;
      bs_b[i] = carry_b + eb;
    }
    carry_a += ta;
    carry_b += tb;
  }
  if (threadIdx.x == 0) {
    const unsigned long long nc = *node_count;
    status[CKF_STATUS_NODES_NEEDED] = nc > 0x7fffffffull ? 0x7fffffff : (int)nc;
    status[CKF_STATUS_TRACKS] = carry_a;
    status[CKF_STATUS_MEAS_NEEDED] = carry_b;
    if (carry_a > cap_tracks || (long long)carry_b > cap_meas)
      atomicOr(status + CKF_STATUS_FLAGS, CKF_FLAG_OUT_CAPACITY);
    *n_tracks = min(carry_a, cap_tracks);
    if (carry_a <= cap_tracks) offsets[carry_a] = carry_b;
  }
}

// One thread per seed walks its best candidate's history backwards for the
// measurement list.  The tracks' parameter and covariance rows go through
// LDS and leave as one contiguous range per workgroup (coalesced stores).
__global__ __launch_bounds__(kScanBlock) void k_out_write(int n, const int* res_node, const int* res_nm,
                                                          const int* res_holes, const double* res_chi2,
                                                          const int* seed_event, const Node* nodes,
                                                          long long node_cap, const int* bs_a, const int* bs_b,
                                                          ckf_tracks out) {
  __shared__ double s_pc[kScanBlock * 20];  // per track of the workgroup: parameters (5), covariance (15)
  __shared__ int s_ok[kScanBlock];
  const int s = blockIdx.x * kScanBlock + threadIdx.x;
  const int has = s < n && res_node[s] >= 0 ? 1 : 0;
  const int nm = has ? res_nm[s] : 0;
  int ea, eb, ta, tb;
  block_scan2(has, nm, ea, eb, ta, tb);
  if (out.status[CKF_STATUS_FLAGS] & CKF_FLAG_NODE_CAPACITY) return;  // the same for the whole workgroup
  const int t0 = bs_a[blockIdx.x];
  const int t = t0 + ea;
  const long long mo = (long long)bs_b[blockIdx.x] + eb;
  int nd = has ? res_node[s] : -1;
  const bool ok = has && t < out.cap_tracks && mo + nm <= out.cap_meas && nd < node_cap;
  if (has) s_ok[ea] = ok ? 1 : 0;
  if (ok) {
    out.offsets[t] = (int)mo;
    const Node& last = nodes[nd];
#pragma unroll
    for (int k = 0; k < 5; ++k) s_pc[20 * ea + k] = last.p[k];
#pragma unroll
    for (int k = 0; k < 15; ++k) s_pc[20 * ea + 5 + k] = last.cov[k];
    out.last_surface[t] = last.surface;
    for (int k = nm - 1; k >= 0 && nd >= 0 && nd < node_cap; --k) {
      const Node& q = nodes[nd];
      out.meas[mo + k] = q.meas;
      if (out.meas_surface) out.meas_surface[mo + k] = q.surface;
      if (out.meas_params)
        for (int c = 0; c < 5; ++c) out.meas_params[5 * (mo + k) + c] = q.p[c];
      nd = q.parent;
    }
    out.chi2[t] = res_chi2[s];
    out.ndf[t] = 2 * nm - 5;
    out.holes[t] = res_holes[s];
    out.seed[t] = s;
    out.event[t] = seed_event[s];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 5 * ta; i += kScanBlock) {
    const int e = i / 5;
    if (s_ok[e]) out.params[5ll * t0 + i] = s_pc[20 * e + i % 5];
  }
  for (int i = threadIdx.x; i < 15 * ta; i += kScanBlock) {
    const int e = i / 15;
    if (s_ok[e]) out.cov[15ll * t0 + i] = s_pc[20 * e + 5 + i % 15];
  }
}

// ---------------------------------------------------------------------------
// output of every finished candidate (tracks_per_seed = 0): per-seed counts,
// the same block scans as above over (tracks, measurements) per seed, the
// records bucketed by seed, then one thread per seed orders its bucket by the
// rank key and writes its tracks.

__global__ void k_all_count(const Workspace w) {
  const long long n = min((long long)*w.fin_count, w.fin_cap);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    atomicAdd(&w.seed_cnt[w.fin_seed[i]], 1);
    atomicAdd(&w.seed_meas[w.fin_seed[i]], w.fin_nmh[i] & 0xffff);
  }
}

__global__ __launch_bounds__(kScanBlock) void k_all_block_sums(int n, const int* cnt, const int* meas, int* bs_a,
                                                               int* bs_b) {
  const int s = blockIdx.x * kScanBlock + threadIdx.x;
  int ea, eb, ta, tb;
  block_scan2(s < n ? cnt[s] : 0, s < n ? meas[s] : 0, ea, eb, ta, tb);
  if (threadIdx.x == 0) {
    bs_a[blockIdx.x] = ta;
    bs_b[blockIdx.x] = tb;
  }
}

// The seed's first track (block scan plus the scanned block sums) becomes
// its bucket cursor; each record then takes a slot in its seed's bucket.
__global__ __launch_bounds__(kScanBlock) void k_all_offsets(int n, const Workspace w, const int* bs_a) {
  const int s = blockIdx.x * kScanBlock + threadIdx.x;
  int ea, eb, ta, tb;
  block_scan2(s < n ? w.seed_cnt[s] : 0, 0, ea, eb, ta, tb);
  if (s < n) w.seed_fill[s] = bs_a[blockIdx.x] + ea;
}

__global__ void k_all_bucket(const Workspace w) {
  const long long n = min((long long)*w.fin_count, w.fin_cap);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    w.fin_order[atomicAdd(&w.seed_fill[w.fin_seed[i]], 1)] = (int)i;
}

__global__ __launch_bounds__(kScanBlock) void k_all_write(int n, const Workspace w, const int* seed_event,
                                                          const int* bs_a, const int* bs_b, ckf_tracks out) {
  const int s = blockIdx.x * kScanBlock + threadIdx.x;
  const int cnt = s < n ? w.seed_cnt[s] : 0, nms = s < n ? w.seed_meas[s] : 0;
  int ea, eb, ta, tb;
  block_scan2(cnt, nms, ea, eb, ta, tb);
  if (out.status[CKF_STATUS_FLAGS] & (CKF_FLAG_NODE_CAPACITY | CKF_FLAG_FIN_CAPACITY)) return;
  if (s >= n || cnt == 0) return;
  const int t0 = bs_a[blockIdx.x] + ea;
  long long mo = (long long)bs_b[blockIdx.x] + eb;
  if (t0 + cnt > out.cap_tracks || mo + nms > out.cap_meas) return;
  // the seed's bucket, ordered by the rank key (insertion sort: buckets are
  // small, and this is a mode for tests)
  int* b = w.fin_order + t0;
  for (int a = 1; a < cnt; ++a) {
    const int i = b[a];
    const int nm = w.fin_nmh[i] & 0xffff, ho = w.fin_nmh[i] >> 16, nd = w.fin_node[i];
    const double ch = w.fin_chi2[i];
    int j = a;
    while (j > 0) {
      const int o = b[j - 1];
      if (!better(nm, ch, ho, nd, w.fin_nmh[o] & 0xffff, w.fin_chi2[o], w.fin_nmh[o] >> 16, w.fin_node[o], w.nodes))
        break;
      b[j] = o;
      --j;
    }
    b[j] = i;
  }
  for (int k = 0; k < cnt; ++k) {
    const int t = t0 + k;
    const int i = b[k];
    const int nm = w.fin_nmh[i] & 0xffff;
    int nd = w.fin_node[i];
    out.offsets[t] = (int)mo;
    if (nd >= 0 && nd < w.node_cap) {
      const Node& last = w.nodes[nd];
#pragma unroll
      for (int c = 0; c < 5; ++c) out.params[5ll * t + c] = last.p[c];
#pragma unroll
      for (int c = 0; c < 15; ++c) out.cov[15ll * t + c] = last.cov[c];
      out.last_surface[t] = last.surface;
    } else {  // no measurement: nothing filtered
#pragma unroll
      for (int c = 0; c < 5; ++c) out.params[5ll * t + c] = NAN;
#pragma unroll
      for (int c = 0; c < 15; ++c) out.cov[15ll * t + c] = NAN;
      out.last_surface[t] = -1;
    }
    for (int q = nm - 1; q >= 0 && nd >= 0 && nd < w.node_cap; --q) {
      const Node& nn = w.nodes[nd];
      out.meas[mo + q] = nn.meas;
      if (out.meas_surface) out.meas_surface[mo + q] = nn.surface;
      if (out.meas_params)
        for (int c = 0; c < 5; ++c) out.meas_params[5 * (mo + q) + c] = nn.p[c];
      nd = nn.parent;
    }
    out.chi2[t] = w.fin_chi2[i];
    out.ndf[t] = 2 * nm - 5;
    out.holes[t] = w.fin_nmh[i] >> 16;
    out.seed[t] = s;
    out.event[t] = seed_event[s];
    mo += nm;
  }
}

// ---------------------------------------------------------------------------
// component kernels

template <bool kMap>
__global__ void __launch_bounds__(64) k_propagate_batch(GeomDev g, FieldDev F, CfgDev cfg, int n, const int* src, const double* p_in,
                                  const double* cov_in, const int* dst, double* p_out, double* cov_out, double* jac,
                                  double* path_out, int* ok_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = src[i], b = dst[i];
  if (a < 0 || a >= g.n_surfaces || b < 0 || b >= g.n_surfaces) {
    ok_out[i] = 0;
    return;
  }
  Module Am, Bm;
  load_module(g, a, Am);
  load_module(g, b, Bm);
  double p[5], C[15];
  for (int k = 0; k < 5; ++k) p[k] = p_in[5 * i + k];
  for (int k = 0; k < 15; ++k) C[k] = cov_in[15 * i + k];
  LegT<kMap ? 5 : 3> L;
  V3 uA, vA;
  leg_start(Am, p, L, uA, vA);
  const V3 origin = ld3(Am.c);
  const V3 dB = ld3(Bm.c) - origin;
  float h = cfg.step_max, path = 0.f;
  LegStats st{0, 0};
  const bool ok = land<kMap>(L, origin, dB, ld3(Bm.n), F, cfg, h, path, st);
  ok_out[i] = ok ? 1 : 0;
  if (!ok) return;
  double pn[5];
  float J[5][5];
  leg_end(L, uA, vA, Bm, dB, field_at<kMap>(F, origin + L.r), p[4], pn, J);
  transport_cov(J, C);
  for (int k = 0; k < 5; ++k) p_out[5 * i + k] = pn[k];
  for (int k = 0; k < 15; ++k) cov_out[15 * i + k] = C[k];
  if (jac)
    for (int r = 0; r < 5; ++r)
      for (int q = 0; q < 5; ++q) jac[25 * i + 5 * r + q] = (double)J[r][q];
  if (path_out) path_out[i] = (double)path;
}

__global__ void k_kf_update_batch(int n, const double* p_in, const double* cov_in, const float* meas,
                                  const float* var, double* p_out, double* cov_out, double* chi2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double p[5], C[15];
  for (int k = 0; k < 5; ++k) p[k] = p_in[5 * i + k];
  for (int k = 0; k < 15; ++k) C[k] = cov_in[15 * i + k];
  const double m0 = meas[2 * i], m1 = meas[2 * i + 1], v0 = var[2 * i], v1 = var[2 * i + 1];
  if (chi2) chi2[i] = chi2_of(p, C, m0, m1, v0, v1);
  double po[5], Co[15];
  kf_update(p, C, m0, m1, v0, v1, po, Co);
  for (int k = 0; k < 5; ++k) p_out[5 * i + k] = po[k];
  for (int k = 0; k < 15; ++k) cov_out[15 * i + k] = Co[k];
}

// ---------------------------------------------------------------------------
// host launchers

hipError_t launch_init(int n_seeds, const Workspace& w, const ckf_tracks& out, hipStream_t st) {
  const int n = n_seeds > 64 ? n_seeds : 64;
  const bool all = w.fin_cap > 0;
  hipLaunchKernelGGL(k_init, dim3((n + 255) / 256), dim3(256), 0, st, n_seeds, w.res_node, w.res_nm, w.queue_head,
                     w.node_count, out.status, reinterpret_cast<long long*>(out.counters), out.n_tracks, out.offsets,
                     out.seed_flags, all ? w.seed_cnt : nullptr, w.seed_meas, w.seed_fill, w.fin_count);
  return hipGetLastError();
}

hipError_t launch_meas_prepare(const MeasIn& m, const Workspace& w, int* status, hipStream_t st) {
  const int rows = m.n_events * m.n_surfaces;
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_meas_rows, dim3((rows + 255) / 256), dim3(256), 0, st, rows, (long long)m.n_meas, m.offsets,
                     m.var, w.row_of, w.row_maxvar0, status);
  if (m.n_meas > 0)
    hipLaunchKernelGGL(k_meas_scatter, dim3((unsigned)((m.n_meas + kScatterBlock - 1) / kScatterBlock)),
                       dim3(kScatterBlock), 0, st,
                       (long long)m.n_meas, rows, m.offsets, w.row_of, m.loc, m.var, w.m_sorted, w.m_key, w.m_id, status);
  return hipGetLastError();
}

hipError_t launch_ckf(const CkfArgs& a, int waves_per_simd, hipStream_t st) {
  const dim3 grid(a.w.grid), block(kWave);
  // Register budgets of 1, 2 and 3 waves per SIMD (the 3-wave builds spill;
  // the 2-wave builds are the fastest on the dense batch; 4 would spill much
  // more).  The learned form runs in a uniform field (the host rejects a map).
  const int w = waves_per_simd;
  if (a.f.map) {
    if (a.counters)
      hipLaunchKernelGGL((k_ckf<1, true, false, true>), grid, block, 0, st, a);
    else if (w >= 2)
      hipLaunchKernelGGL((k_ckf<2, false, false, true>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((k_ckf<1, false, false, true>), grid, block, 0, st, a);
  } else if (a.learned) {
    if (a.counters)
      hipLaunchKernelGGL((k_ckf<1, true, true, false>), grid, block, 0, st, a);
    else if (w >= 3)
      hipLaunchKernelGGL((k_ckf<3, false, true, false>), grid, block, 0, st, a);
    else if (w == 2)
      hipLaunchKernelGGL((k_ckf<2, false, true, false>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((k_ckf<1, false, true, false>), grid, block, 0, st, a);
  } else {
    if (a.counters)
      hipLaunchKernelGGL((k_ckf<1, true, false, false>), grid, block, 0, st, a);
    else if (w >= 3)
      hipLaunchKernelGGL((k_ckf<3, false, false, false>), grid, block, 0, st, a);
    else if (w == 2)
      hipLaunchKernelGGL((k_ckf<2, false, false, false>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((k_ckf<1, false, false, false>), grid, block, 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_output(int n_seeds, const Workspace& w, const int* seed_event, const ckf_tracks& out,
                         hipStream_t st) {
  const int nb = (n_seeds + kScanBlock - 1) / kScanBlock;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_out_count, dim3(nb), dim3(kScanBlock), 0, st, n_seeds, w.res_node, w.res_nm, w.scan_a,
                     w.scan_b);
  hipLaunchKernelGGL(k_out_scan_blocks, dim3(1), dim3(kScanBlock), 0, st, nb, w.scan_a, w.scan_b, out.status,
                     out.n_tracks, out.cap_tracks, (long long)out.cap_meas, out.offsets, w.node_count);
  hipLaunchKernelGGL(k_out_write, dim3(nb), dim3(kScanBlock), 0, st, n_seeds, w.res_node, w.res_nm, w.res_holes,
                     w.res_chi2, seed_event, w.nodes, w.node_cap, w.scan_a, w.scan_b, out);
  return hipGetLastError();
}

hipError_t launch_output_all(int n_seeds, const Workspace& w, const int* seed_event, const ckf_tracks& out,
                             hipStream_t st) {
  const int nb = (n_seeds + kScanBlock - 1) / kScanBlock;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_all_count, dim3(1024), dim3(256), 0, st, w);
  hipLaunchKernelGGL(k_all_block_sums, dim3(nb), dim3(kScanBlock), 0, st, n_seeds, w.seed_cnt, w.seed_meas,
                     w.scan_a, w.scan_b);
  hipLaunchKernelGGL(k_out_scan_blocks, dim3(1), dim3(kScanBlock), 0, st, nb, w.scan_a, w.scan_b, out.status,
                     out.n_tracks, out.cap_tracks, (long long)out.cap_meas, out.offsets, w.node_count);
  hipLaunchKernelGGL(k_all_offsets, dim3(nb), dim3(kScanBlock), 0, st, n_seeds, w, w.scan_a);
  hipLaunchKernelGGL(k_all_bucket, dim3(1024), dim3(256), 0, st, w);
  hipLaunchKernelGGL(k_all_write, dim3(nb), dim3(kScanBlock), 0, st, n_seeds, w, seed_event, w.scan_a, w.scan_b,
                     out);
  return hipGetLastError();
}

hipError_t launch_propagate(const GeomDev& g, const FieldDev& f, const CfgDev& c, int n, const int* src,
                            const double* p_in, const double* cov_in, const int* dst, double* p_out,
                            double* cov_out, double* jac, double* path, int* ok, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (f.map)
    hipLaunchKernelGGL(k_propagate_batch<true>, dim3((n + 63) / 64), dim3(64), 0, st, g, f, c, n, src, p_in, cov_in,
                       dst, p_out, cov_out, jac, path, ok);
  else
    hipLaunchKernelGGL(k_propagate_batch<false>, dim3((n + 63) / 64), dim3(64), 0, st, g, f, c, n, src, p_in, cov_in,
                       dst, p_out, cov_out, jac, path, ok);
  return hipGetLastError();
}

hipError_t launch_kf_update(int n, const double* p_in, const double* cov_in, const float* meas, const float* var,
                            double* p_out, double* cov_out, double* chi2, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kf_update_batch, dim3((n + 63) / 64), dim3(64), 0, st, n, p_in, cov_in, meas, var, p_out,
                     cov_out, chi2);
  return hipGetLastError();
}

}  // namespace ckf
