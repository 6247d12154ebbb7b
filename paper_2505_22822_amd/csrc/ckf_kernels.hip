// gfx950 kernels of CKF track finding.
//
//  k_meas_prepare  per (event, module) row: measurements sorted by loc0 (ids
//                  kept) and the row's largest var0, for the exact chi2
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

namespace ckf {

// ---------------------------------------------------------------------------
// measurement preparation

__global__ void k_meas_prepare(int n_rows, long long n_meas, const int* __restrict__ offsets,
                               const float* __restrict__ loc, const float* __restrict__ var, float* l0, float* l1,
                               float* v0, float* v1, int* id, float* maxv0, int* status) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n_rows) return;
  const int a = offsets[row], b = offsets[row + 1];
  if ((row == 0 && a != 0) || a > b || a < 0 || (long long)b > n_meas) {
    atomicOr(status + CKF_STATUS_FLAGS, CKF_FLAG_BAD_OFFSETS);
    maxv0[row] = 0.f;
    return;
  }
  float mv = 0.f;
  for (int i = a; i < b; ++i) {
    const float x = loc[2 * i];
    int j = i;
    while (j > a && l0[j - 1] > x) {
      l0[j] = l0[j - 1];
      l1[j] = l1[j - 1];
      v0[j] = v0[j - 1];
      v1[j] = v1[j - 1];
      id[j] = id[j - 1];
      --j;
    }
    l0[j] = x;
    l1[j] = loc[2 * i + 1];
    v0[j] = var[2 * i];
    v1[j] = var[2 * i + 1];
    id[j] = i;
    mv = fmaxf(mv, var[2 * i]);
  }
  maxv0[row] = mv;
}

// ---------------------------------------------------------------------------
// per-call initialisation (a fill kernel, so the sequence can be captured)

__global__ void k_init(int n_seeds, int* res_node, int* res_nm, int* queue_head, unsigned long long* node_count,
                       int* status, long long* counters, int* n_tracks, int* offsets) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_seeds) {
    res_node[i] = -1;
    res_nm[i] = 0;
  }
  if (i == 0) {
    *queue_head = 0;
    *node_count = 0ull;
    *n_tracks = 0;
    offsets[0] = 0;
  }
  if (i < 8) status[i] = 0;
  if (counters && i < CKF_CNT_N) counters[i] = 0;
}

// ---------------------------------------------------------------------------
// candidate pool records

struct Rec {
  double p[5];
  double C[15];
  double chi2;
  int surf, slot, node, nm, holes;
  unsigned long long mask;
  int list[kMaxList];
  int nlist;
  int root;
  float h, path;
};

struct Pool {
  double* d;
  int* i;
  float* f;
  int cap;
};

__device__ __forceinline__ Pool pool_at(char* base, int cap, int which) {
  char* p = base + (size_t)which * cap * kRecBytes;
  Pool P;
  P.d = reinterpret_cast<double*>(p);
  P.i = reinterpret_cast<int*>(p + (size_t)cap * PD_N * 8);
  P.f = reinterpret_cast<float*>(p + (size_t)cap * (PD_N * 8 + PI_N * 4));
  P.cap = cap;
  return P;
}

__device__ __forceinline__ void load_rec(const Pool& P, int r, Rec& c) {
  const int cap = P.cap;
#pragma unroll
  for (int k = 0; k < 5; ++k) c.p[k] = P.d[(PD_P + k) * cap + r];
#pragma unroll
  for (int k = 0; k < 15; ++k) c.C[k] = P.d[(PD_C + k) * cap + r];
  c.chi2 = P.d[PD_CHI2 * cap + r];
  c.surf = P.i[PI_SURF * cap + r];
  c.slot = P.i[PI_SLOT * cap + r];
  c.node = P.i[PI_NODE * cap + r];
  const int nmh = P.i[PI_NMH * cap + r];
  c.nm = nmh & 0xffff;
  c.holes = nmh >> 16;
  c.mask = (unsigned long long)(unsigned)P.i[PI_MASK_LO * cap + r] |
           ((unsigned long long)(unsigned)P.i[PI_MASK_HI * cap + r] << 32);
#pragma unroll
  for (int k = 0; k < kMaxList; ++k) c.list[k] = P.i[(PI_LIST + k) * cap + r];
  const int nl = P.i[PI_NLIST * cap + r];
  c.nlist = nl & 0xff;
  c.root = nl >> 8;
  c.h = P.f[PF_H * cap + r];
  c.path = P.f[PF_PATH * cap + r];
}

__device__ __forceinline__ void store_rec(const Pool& P, int r, const Rec& c) {
  const int cap = P.cap;
#pragma unroll
  for (int k = 0; k < 5; ++k) P.d[(PD_P + k) * cap + r] = c.p[k];
#pragma unroll
  for (int k = 0; k < 15; ++k) P.d[(PD_C + k) * cap + r] = c.C[k];
  P.d[PD_CHI2 * cap + r] = c.chi2;
  P.i[PI_SURF * cap + r] = c.surf;
  P.i[PI_SLOT * cap + r] = c.slot;
  P.i[PI_NODE * cap + r] = c.node;
  P.i[PI_NMH * cap + r] = c.nm | (c.holes << 16);
  P.i[PI_MASK_LO * cap + r] = (int)(unsigned)(c.mask & 0xffffffffull);
  P.i[PI_MASK_HI * cap + r] = (int)(unsigned)(c.mask >> 32);
#pragma unroll
  for (int k = 0; k < kMaxList; ++k) P.i[(PI_LIST + k) * cap + r] = c.list[k];
  P.i[PI_NLIST * cap + r] = c.nlist | (c.root << 8);
  P.f[PF_H * cap + r] = c.h;
  P.f[PF_PATH * cap + r] = c.path;
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

__device__ __forceinline__ long long wave_sum64(long long v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Rank key: more measurements, smaller chi2 sum, fewer holes, then the
// measurement-id sequence in lexicographic order (walk of the history).
__device__ bool better(int nmA, double chiA, int hoA, int nodeA, int nmB, double chiB, int hoB, int nodeB,
                       const Node* nodes) {
  if (nmA != nmB) return nmA > nmB;
  if (chiA != chiB) return chiA < chiB;
  if (hoA != hoB) return hoA < hoB;
  int ia[kMaxSteps], ib[kMaxSteps];
  int n = min(nmA, kMaxSteps);
  for (int k = n - 1; k >= 0; --k) {
    ia[k] = nodeA >= 0 ? nodes[nodeA].meas : -1;
    ib[k] = nodeB >= 0 ? nodes[nodeB].meas : -1;
    nodeA = nodeA >= 0 ? nodes[nodeA].parent : -1;
    nodeB = nodeB >= 0 ? nodes[nodeB].parent : -1;
  }
  for (int k = 0; k < n; ++k)
    if (ia[k] != ib[k]) return ia[k] < ib[k];
  return false;
}

struct Cnt {
  int v[CKF_CNT_N];
};

constexpr int kMaxSlots = 64;

__global__ __launch_bounds__(kWave) void k_ckf(CkfArgs A) {
  __shared__ int sh_seed[kMaxSlots], sh_event[kMaxSlots], sh_live[kMaxSlots], sh_step[kMaxSlots];
  __shared__ int sh_best_node[kMaxSlots], sh_best_nm[kMaxSlots], sh_best_holes[kMaxSlots];
  __shared__ double sh_best_chi2[kMaxSlots];
  __shared__ int sh_n_out, sh_bcast;
  __shared__ unsigned long long sh_node_base;

  const GeomDev& g = A.g;
  const CfgDev& cfg = A.cfg;
  const int lane = lane_id();
  const int S = A.w.seeds_per_group;
  const int cap = A.w.pool_cap;
  const float margin = cfg.nav_margin;
  char* base = A.w.pools + (size_t)blockIdx.x * 2 * cap * kRecBytes;
  const unsigned long long lt_mask = (1ull << lane) - 1ull;

  Cnt cnt;
#pragma unroll
  for (int k = 0; k < CKF_CNT_N; ++k) cnt.v[k] = 0;
  int bad_seeds = 0, failed_legs = 0, nav_ovf = 0;

  if (lane < kMaxSlots) {
    sh_seed[lane] = -1;
    sh_live[lane] = 0;
  }
  __syncthreads();

  int cur = 0, n_in = 0;
  // invalid measurement offsets: search ranges cannot be trusted, do nothing
  bool queue_done = (((volatile int*)A.status)[CKF_STATUS_FLAGS] & CKF_FLAG_BAD_OFFSETS) != 0;
  for (;;) {
    if (((volatile int*)A.status)[CKF_STATUS_FLAGS] & CKF_FLAG_NODE_CAPACITY) break;
    const Pool Pin = pool_at(base, cap, cur), Pout = pool_at(base, cap, 1 - cur);

    // ---- admission: fill free seed slots from the work queue
    if (!queue_done) {
      const bool free_slot = lane < S && sh_seed[lane] < 0;
      const unsigned long long fm = __ballot(free_slot);
      const int nfree = __popcll(fm);
      if (nfree > 0) {
        if (lane == 0) sh_bcast = atomicAdd(A.w.queue_head, nfree);
        __syncthreads();
        const int start = sh_bcast;
        __syncthreads();
        if (start + nfree >= A.s.n) queue_done = true;
        const int seed = start + __popcll(fm & lt_mask);
        bool ok = free_slot && seed < A.s.n;
        if (ok) {
          const int sf = A.s.surface[seed], ev = A.s.event[seed];
          bool good = sf >= 0 && sf < g.n_surfaces && ev >= 0 && ev < A.m.n_events;
          for (int k = 0; k < 5; ++k) good = good && isfinite(A.s.params[5 * seed + k]);
          for (int k = 0; k < 15; ++k) good = good && isfinite(A.s.cov[15 * seed + k]);
          good = good && A.s.params[5 * seed + 4] != 0.0;
          if (!good) {
            A.w.res_node[seed] = -1;
            A.w.res_nm[seed] = 0;
            ++bad_seeds;
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
          Rec c;
          for (int k = 0; k < 5; ++k) c.p[k] = A.s.params[5 * seed + k];
          for (int k = 0; k < 15; ++k) c.C[k] = A.s.cov[15 * seed + k];
          c.chi2 = 0.0;
          c.surf = A.s.surface[seed];
          c.slot = lane;
          c.node = -1;
          c.nm = 0;
          c.holes = 0;
          c.mask = 1ull << g.mod[c.surf].layer;
          for (int k = 0; k < kMaxList; ++k) c.list[k] = -1;
          c.nlist = 0;
          c.root = 1;
          c.h = cfg.step_max;
          c.path = 0.f;
          store_rec(Pin, r, c);
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
    if (lane < kMaxSlots) sh_live[lane] = 0;
    if (lane == 0) sh_n_out = 0;
    __syncthreads();
    for (int b0 = 0; b0 < n_in; b0 += kWave) {
      const int r = b0 + lane;
      Rec c;
      bool act = r < n_in;
      if (act) {
        load_rec(Pin, r, c);
        act = c.slot >= 0;
      }
      int n_out = 0, n_acc = 0;
      bool fin = false;
      double acc_chi2[kMaxBranch];
      int acc_pos[kMaxBranch];
      Module M;
      if (act) {
        ++cnt.v[CKF_CNT_STEPS];
        bool go = true, crossed = false;
        if (c.root) {
          c.root = 0;
          load_module(g, c.surf, M);
          Leg L;
          V3 uA, vA;
          leg_start(M, c.p, L, uA, vA);
          const V3 P = ld3(M.c) + L.r;
          const V3 k = (kKappa * L.lam) * cross(L.T, field_at(A.f, P));
          int nt = 0;
          c.nlist = list_layer(g, M.layer, P, L.T, k, 0.f, c.surf, margin, c.list, nt, nav_ovf);
          cnt.v[CKF_CNT_NAV_MODULES] += nt;
          crossed = true;
        } else {
          if (c.nlist == 0) {
            Module Cm;
            load_module(g, c.surf, Cm);
            Leg L;
            V3 uA, vA;
            leg_start(Cm, c.p, L, uA, vA);
            const V3 P = ld3(Cm.c) + L.r;
            const V3 Bf = field_at(A.f, P);
            const Helix H = make_helix(P, L.T, L.lam, Bf);
            float sL;
            ++cnt.v[CKF_CNT_NAV];
            const int nl = next_layer(g, H, c.mask, cfg.path_max - c.path, sL);
            if (nl < 0) {
              fin = true;
              go = false;
            } else {
              c.mask |= 1ull << nl;
              V3 Ps, Ts;
              helix_at(H, sL, Ps, Ts);
              const V3 ks = (kKappa * L.lam) * cross(Ts, Bf);
              int nt = 0;
              c.nlist = list_layer(g, nl, Ps, Ts, ks, sL, -1, margin, c.list, nt, nav_ovf);
              cnt.v[CKF_CNT_NAV_MODULES] += nt;
              if (c.nlist == 0) {
                n_out = 1;  // the layer is crossed in a gap
                go = false;
              }
            }
          }
          if (go) {
            const int m = c.list[0];
#pragma unroll
            for (int k = 0; k < kMaxList - 1; ++k) c.list[k] = c.list[k + 1];
            c.list[kMaxList - 1] = -1;
            --c.nlist;
            Module Am;
            load_module(g, c.surf, Am);
            load_module(g, m, M);
            Leg L;
            V3 uA, vA;
            leg_start(Am, c.p, L, uA, vA);
            const V3 origin = ld3(Am.c);
            const V3 dB = ld3(M.c) - origin;
            LegStats ls{0, 0};
            ++cnt.v[CKF_CNT_LEGS];
            const bool ok = land(L, origin, dB, ld3(M.n), A.f, cfg, c.h, c.path, ls);
            cnt.v[CKF_CNT_RK_TRIALS] += ls.trials;
            cnt.v[CKF_CNT_RK_REJECTS] += ls.rejects;
            double pn[5];
            float J[5][5];
            bool good = ok;
            if (ok) {
              leg_end(L, uA, vA, M, dB, field_at(A.f, origin + L.r), c.p[4], pn, J);
#pragma unroll
              for (int k = 0; k < 5; ++k) good = good && isfinite(pn[k]);
            }
            if (!good) {
              ++failed_legs;
              go = false;  // dropped
            } else {
              transport_cov(J, c.C);
#pragma unroll
              for (int k = 0; k < 5; ++k) c.p[k] = pn[k];
              c.surf = m;
              crossed = fabs(pn[0]) <= (double)M.hw0 && fabs(pn[1]) <= (double)M.hw1;
              if (!crossed) {
                n_out = 1;  // listed but not crossed
                go = false;
              }
            }
          }
        }
        if (go && crossed) {
          ++cnt.v[CKF_CNT_CROSSED];
          const int row = sh_event[c.slot] * g.n_surfaces + c.surf;
          const int a = A.m.offsets[row], b = A.m.offsets[row + 1];
          if (b > a) {
            const double wd = sqrt(cfg.chi2_max * (c.C[0] + (double)A.w.row_maxvar0[row]));
            const float lo = (float)(c.p[0] - wd) - 1e-3f, hi = (float)(c.p[0] + wd) + 1e-3f;
            int l = a, u = b;
            while (l < u) {  // first position with loc0 >= lo
              const int mid = (l + u) >> 1;
              if (A.w.m_loc0[mid] < lo) l = mid + 1; else u = mid;
            }
            for (int i = l; i < b && A.w.m_loc0[i] <= hi; ++i) {
              ++cnt.v[CKF_CNT_CHI2];
              const double x2 = chi2_of(c.p, c.C, (double)A.w.m_loc0[i], (double)A.w.m_loc1[i],
                                        (double)A.w.m_var0[i], (double)A.w.m_var1[i]);
              if (!(x2 < cfg.chi2_max)) continue;
              const int idi = A.w.m_id[i];
              int pos = n_acc;
              while (pos > 0 && (acc_chi2[pos - 1] > x2 ||
                                 (acc_chi2[pos - 1] == x2 && A.w.m_id[acc_pos[pos - 1]] > idi)))
                --pos;
              if (pos >= cfg.branches) continue;
              for (int q = min(n_acc, cfg.branches - 1); q > pos; --q) {
                acc_chi2[q] = acc_chi2[q - 1];
                acc_pos[q] = acc_pos[q - 1];
              }
              acc_chi2[pos] = x2;
              acc_pos[pos] = i;
              if (n_acc < cfg.branches) ++n_acc;
            }
          }
          if (n_acc == 0) {
            ++cnt.v[CKF_CNT_HOLES];
            ++c.holes;
            if (cfg.material) {
              apply_ms(M, cfg.mass, c.p, c.C);
              ++cnt.v[CKF_CNT_MS];
            }
            if (c.holes > cfg.max_holes) fin = true;
            else n_out = 1;
          } else {
            n_out = n_acc;
          }
        }
      }

      // ---- slots for the outputs (wave ballot/scan) and history nodes
      int tot_out;
      const int off = wave_excl_scan(n_out, tot_out);
      const int pos0 = sh_n_out + off;
      int tot_nodes;
      const int noff = wave_excl_scan(n_acc, tot_nodes);
      __syncthreads();
      if (lane == 0) {
        sh_n_out += tot_out;
        sh_node_base = tot_nodes > 0 ? atomicAdd(A.w.node_count, (unsigned long long)tot_nodes) : 0ull;
      }
      __syncthreads();
      const long long node0 = (long long)sh_node_base + noff;
      if (act && n_out > 0) {
        if (n_acc == 0) {
          store_rec(Pout, pos0, c);
          atomicAdd(&sh_live[c.slot], 1);
        } else {
          const bool room = node0 + n_acc <= A.w.node_cap;
          if (!room) atomicOr(A.status + CKF_STATUS_FLAGS, CKF_FLAG_NODE_CAPACITY);
          for (int j = 0; j < n_acc; ++j) {
            const int i = acc_pos[j];
            Rec ch = c;
            kf_update(ch.p, ch.C, (double)A.w.m_loc0[i], (double)A.w.m_loc1[i], (double)A.w.m_var0[i],
                      (double)A.w.m_var1[i]);
            ++cnt.v[CKF_CNT_KF];
            ch.nm = c.nm + 1;
            ch.chi2 = c.chi2 + acc_chi2[j];
            ch.node = room ? (int)(node0 + j) : -1;
            if (room) {
              Node* nd = A.w.nodes + node0 + j;
              nd->parent = c.node;
              nd->meas = A.w.m_id[i];
              nd->surface = c.surf;
              nd->pad = 0;
#pragma unroll
              for (int k = 0; k < 5; ++k) nd->p[k] = ch.p[k];
#pragma unroll
              for (int k = 0; k < 15; ++k) nd->cov[k] = ch.C[k];
            }
            if (cfg.material) {
              apply_ms(M, cfg.mass, ch.p, ch.C);
              ++cnt.v[CKF_CNT_MS];
            }
            store_rec(Pout, pos0 + j, ch);
            atomicAdd(&sh_live[c.slot], 1);
          }
        }
      }
      // ---- finished candidates update their seed's best (one lane at a time)
      unsigned long long fm = __ballot(act && fin);
      while (fm) {
        const int l = __ffsll((long long)fm) - 1;
        fm &= fm - 1;
        if (lane == l) {
          ++cnt.v[CKF_CNT_FINISHED];
          const int sl = c.slot;
          if (c.nm >= cfg.min_meas &&
              (sh_best_node[sl] < 0 || better(c.nm, c.chi2, c.holes, c.node, sh_best_nm[sl], sh_best_chi2[sl],
                                               sh_best_holes[sl], sh_best_node[sl], A.w.nodes))) {
            sh_best_node[sl] = c.node;
            sh_best_nm[sl] = c.nm;
            sh_best_chi2[sl] = c.chi2;
            sh_best_holes[sl] = c.holes;
          }
        }
        __syncthreads();
      }
    }
    __syncthreads();
    const int n_out_total = sh_n_out;

    // ---- pruning: a seed keeps its max_live best candidates (rank key)
    {
      const bool over = lane < S && sh_seed[lane] >= 0 && sh_live[lane] > cfg.max_live;
      if (__ballot(over)) {
        if (over) {
          int idx[kMaxSlots];
          int n = 0;
          for (int r = 0; r < n_out_total && n < kMaxSlots; ++r)
            if (Pout.i[PI_SLOT * cap + r] == lane) idx[n++] = r;
          for (int a = 0; a < n; ++a) {
            const int ra = idx[a];
            const int nmh_a = Pout.i[PI_NMH * cap + ra];
            const double ch_a = Pout.d[PD_CHI2 * cap + ra];
            const int nd_a = Pout.i[PI_NODE * cap + ra];
            int n_better = 0;
            for (int b = 0; b < n; ++b) {
              if (b == a) continue;
              const int rb = idx[b];
              const int nmh_b = Pout.i[PI_NMH * cap + rb];
              if (better(nmh_b & 0xffff, Pout.d[PD_CHI2 * cap + rb], nmh_b >> 16, Pout.i[PI_NODE * cap + rb],
                         nmh_a & 0xffff, ch_a, nmh_a >> 16, nd_a, A.w.nodes))
                ++n_better;
            }
            if (n_better >= cfg.max_live) {
              Pout.i[PI_SLOT * cap + ra] = -1;  // dead: skipped by the next step
              ++cnt.v[CKF_CNT_PRUNED];
            }
          }
          sh_live[lane] = min(n, cfg.max_live);
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
            sl = Pout.i[PI_SLOT * cap + r];
            if (sl >= 0 && sh_step[sl] >= cfg.max_steps) {
              f = true;
              const int nmh = Pout.i[PI_NMH * cap + r];
              nm = nmh & 0xffff;
              ho = nmh >> 16;
              nd = Pout.i[PI_NODE * cap + r];
              ch = Pout.d[PD_CHI2 * cap + r];
              Pout.i[PI_SLOT * cap + r] = -1;
            }
          }
          unsigned long long fm = __ballot(f);
          while (fm) {
            const int l = __ffsll((long long)fm) - 1;
            fm &= fm - 1;
            if (lane == l) {
              ++cnt.v[CKF_CNT_FINISHED];
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
    cur = 1 - cur;
    n_in = n_out_total;
  }

  // ---- counters and status
  if (A.counters) {
#pragma unroll
    for (int k = 0; k < CKF_CNT_N; ++k) {
      const long long t = wave_sum64((long long)cnt.v[k]);
      if (lane == 0 && t) atomicAdd((unsigned long long*)(A.counters + k), (unsigned long long)t);
    }
  }
  const long long tb = wave_sum64(bad_seeds), tf = wave_sum64(failed_legs), tn = wave_sum64(nav_ovf);
  if (lane == 0) {
    if (tb) atomicAdd(A.status + CKF_STATUS_BAD_SEEDS, (int)tb);
    if (tf) atomicAdd(A.status + CKF_STATUS_FAILED_LEGS, (int)tf);
    if (tn) atomicAdd(A.status + CKF_STATUS_NAV_OVERFLOW, (int)tn);
  }
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

__global__ __launch_bounds__(kScanBlock) void k_out_write(int n, const int* res_node, const int* res_nm,
                                                          const int* res_holes, const double* res_chi2,
                                                          const int* seed_event, const Node* nodes,
                                                          long long node_cap, const int* bs_a, const int* bs_b,
                                                          ckf_tracks out) {
  const int s = blockIdx.x * kScanBlock + threadIdx.x;
  const int has = s < n && res_node[s] >= 0 ? 1 : 0;
  const int nm = has ? res_nm[s] : 0;
  int ea, eb, ta, tb;
  block_scan2(has, nm, ea, eb, ta, tb);
  if (!has) return;
  if (out.status[CKF_STATUS_FLAGS] & CKF_FLAG_NODE_CAPACITY) return;
  const int t = bs_a[blockIdx.x] + ea;
  const long long mo = (long long)bs_b[blockIdx.x] + eb;
  if (t >= out.cap_tracks || mo + nm > out.cap_meas) return;
  out.offsets[t] = (int)mo;
  int nd = res_node[s];
  if (nd >= node_cap) return;
  const Node& last = nodes[nd];
  for (int k = 0; k < 5; ++k) out.params[5 * t + k] = last.p[k];
  for (int k = 0; k < 15; ++k) out.cov[15 * t + k] = last.cov[k];
  out.last_surface[t] = last.surface;
  for (int k = nm - 1; k >= 0 && nd >= 0 && nd < node_cap; --k) {
    out.meas[mo + k] = nodes[nd].meas;
    nd = nodes[nd].parent;
  }
  out.chi2[t] = res_chi2[s];
  out.ndf[t] = 2 * nm - 5;
  out.holes[t] = res_holes[s];
  out.seed[t] = s;
  out.event[t] = seed_event[s];
}

// ---------------------------------------------------------------------------
// component kernels

__global__ void k_propagate_batch(GeomDev g, FieldDev F, CfgDev cfg, int n, const int* src, const double* p_in,
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
  Leg L;
  V3 uA, vA;
  leg_start(Am, p, L, uA, vA);
  const V3 origin = ld3(Am.c);
  const V3 dB = ld3(Bm.c) - origin;
  float h = cfg.step_max, path = 0.f;
  LegStats st{0, 0};
  const bool ok = land(L, origin, dB, ld3(Bm.n), F, cfg, h, path, st);
  ok_out[i] = ok ? 1 : 0;
  if (!ok) return;
  double pn[5];
  float J[5][5];
  leg_end(L, uA, vA, Bm, dB, field_at(F, origin + L.r), p[4], pn, J);
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
  kf_update(p, C, m0, m1, v0, v1);
  for (int k = 0; k < 5; ++k) p_out[5 * i + k] = p[k];
  for (int k = 0; k < 15; ++k) cov_out[15 * i + k] = C[k];
}

// ---------------------------------------------------------------------------
// host launchers

hipError_t launch_init(int n_seeds, const Workspace& w, const ckf_tracks& out, hipStream_t st) {
  const int n = n_seeds > 64 ? n_seeds : 64;
  hipLaunchKernelGGL(k_init, dim3((n + 255) / 256), dim3(256), 0, st, n_seeds, w.res_node, w.res_nm, w.queue_head,
                     w.node_count, out.status, reinterpret_cast<long long*>(out.counters), out.n_tracks, out.offsets);
  return hipGetLastError();
}

hipError_t launch_meas_prepare(const MeasIn& m, const Workspace& w, int* status, hipStream_t st) {
  const int rows = m.n_events * m.n_surfaces;
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_meas_prepare, dim3((rows + 255) / 256), dim3(256), 0, st, rows, (long long)m.n_meas,
                     m.offsets, m.loc, m.var, w.m_loc0, w.m_loc1, w.m_var0, w.m_var1, w.m_id, w.row_maxvar0,
                     status);
  return hipGetLastError();
}

hipError_t launch_ckf(const CkfArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_ckf, dim3(a.w.grid), dim3(kWave), 0, st, a);
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

hipError_t launch_propagate(const GeomDev& g, const FieldDev& f, const CfgDev& c, int n, const int* src,
                            const double* p_in, const double* cov_in, const int* dst, double* p_out,
                            double* cov_out, double* jac, double* path, int* ok, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_propagate_batch, dim3((n + 63) / 64), dim3(64), 0, st, g, f, c, n, src, p_in, cov_in, dst,
                     p_out, cov_out, jac, path, ok);
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
