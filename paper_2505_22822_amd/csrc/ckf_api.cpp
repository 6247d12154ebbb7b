// Host runtime of the C ABI: validation, the navigation grid, workspace
// carving and kernel launches.  No allocation happens in ckf_find.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ckf.h"
#include "ckf_internal.hpp"
#include "ckf_kernels.hpp"

struct ckf_geometry {
  ckf::GeomDev dev;
  std::vector<void*> allocations;
  int device;
  int nb_rows = 0;  // rows of the neighbour table
};

struct ckf_field {
  ckf::FieldDev dev;
  void* map = nullptr;  // device copy of a field map
};

struct ckf_timer {
  hipEvent_t start, stop;
};

struct ckf_plan {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct ckf_model {
  void* buf = nullptr;  // packed fragments and biases (kModelBytes)
  int device = 0;
};

namespace {

thread_local std::string g_last_error;

ckf_status fail(ckf_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

ckf_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return CKF_ERR_DEVICE;
}

#define HIP_TRY(expr, what)                  \
  do {                                       \
    hipError_t e_ = (expr);                  \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

bool finite3(const float* p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

constexpr double kPi = 3.14159265358979323846;

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Boundary points of a module rectangle expanded by `pad`.
void rect_samples(const ckf::Module& M, double pad, std::vector<double>& xs) {
  xs.clear();
  const double a = M.hw0 + pad, b = M.hw1 + pad;
  const int k = 24;
  for (int e = 0; e < 4; ++e)
    for (int t = 0; t <= k; ++t) {
      const double f = -1.0 + 2.0 * t / k;
      double l0, l1;
      if (e == 0) { l0 = f * a; l1 = -b; }
      else if (e == 1) { l0 = a; l1 = f * b; }
      else if (e == 2) { l0 = -f * a; l1 = b; }
      else { l0 = -a; l1 = -f * b; }
      for (int d = 0; d < 3; ++d) xs.push_back(M.c[d] + l0 * M.u[d] + l1 * M.v[d]);
    }
}

struct HostGrid {
  std::vector<ckf::LayerRec> layers;
  std::vector<int> cell_off, cell_mod;
  std::vector<int> barrel, disk_pos, disk_neg;
};

ckf_status build_grid(const ckf_geometry_desc* d, const std::vector<ckf::Module>& mods, HostGrid& G) {
  const int L = d->n_layers;
  G.layers.resize(L);
  std::vector<std::vector<int>> members(L);
  for (int i = 0; i < d->n_surfaces; ++i) members[d->layer[i]].push_back(i);
  std::vector<std::vector<int>> cells;
  std::vector<double> xs;
  int cell_base = 0;
  for (int l = 0; l < L; ++l) {
    ckf::LayerRec& R = G.layers[l];
    R.type = d->layer_type[l];
    R.pos = d->layer_pos[l];
    R.lo = d->layer_lo[l];
    R.hi = d->layer_hi[l];
    // extents of the padded modules in (phi, w) and the layer depth
    double wlo = 1e30, whi = -1e30, depth = 0.0, rmax = 0.0;
    struct Ext {
      double plo, phi, wlo, whi;
    };
    std::vector<Ext> ext(members[l].size());
    for (size_t q = 0; q < members[l].size(); ++q) {
      const ckf::Module& M = mods[members[l][q]];
      rect_samples(M, ckf::kGridPad, xs);
      const double pc = std::atan2((double)M.c[1], (double)M.c[0]);
      double plo = 1e30, phi = -1e30, a = 1e30, b = -1e30;
      for (size_t k = 0; k < xs.size(); k += 3) {
        const double x = xs[k], y = xs[k + 1], z = xs[k + 2];
        const double r = std::sqrt(x * x + y * y);
        double dp = std::atan2(y, x) - pc;
        while (dp > kPi) dp -= 2 * kPi;
        while (dp < -kPi) dp += 2 * kPi;
        plo = std::min(plo, pc + dp);
        phi = std::max(phi, pc + dp);
        const double w = R.type == 0 ? z : r;
        a = std::min(a, w);
        b = std::max(b, w);
        depth = std::max(depth, R.type == 0 ? r - R.pos : std::fabs(z) - std::fabs((double)R.pos));
        rmax = std::max(rmax, r);
      }
      // the inner radius of a rectangle can lie inside an edge: sample densely above
      ext[q] = {plo, phi, a, b};
      wlo = std::min(wlo, a);
      whi = std::max(whi, b);
    }
    if (members[l].empty()) {
      wlo = R.lo;
      whi = R.hi;
    }
    R.depth = (float)(depth + 1.0);
    R.wlo = (float)wlo;
    R.whi = (float)whi;
    const double radius = R.type == 0 ? (double)R.pos : std::max(rmax, 1.0);
    R.nphi = std::max(1, std::min(4096, (int)std::lround(2 * kPi * radius / 20.0)));
    R.nw = std::max(1, std::min(4096, (int)std::lround((whi - wlo) / (R.type == 0 ? 60.0 : 30.0))));
    R.cell_base = cell_base;
    const int nc = R.nphi * R.nw;
    cells.resize(cell_base + nc);
    const double bph = 2 * kPi / R.nphi, bw = (whi - wlo) / R.nw;
    for (size_t q = 0; q < members[l].size(); ++q) {
      const Ext& e = ext[q];
      const int ip0 = (int)std::floor((e.plo + kPi) / bph), ip1 = (int)std::floor((e.phi + kPi) / bph);
      int iw0 = (int)std::floor((e.wlo - wlo) / bw), iw1 = (int)std::floor((e.whi - wlo) / bw);
      iw0 = std::max(0, iw0);
      iw1 = std::min(R.nw - 1, iw1);
      const int span = std::min(ip1 - ip0, R.nphi - 1);
      for (int ipr = ip0; ipr <= ip0 + span; ++ipr) {
        int ip = ipr % R.nphi;
        if (ip < 0) ip += R.nphi;
        for (int iw = iw0; iw <= iw1; ++iw) cells[cell_base + ip * R.nw + iw].push_back(members[l][q]);
      }
    }
    cell_base += nc;
    if (R.type == 0) G.barrel.push_back(l);
    else if (R.pos > 0) G.disk_pos.push_back(l);
    else G.disk_neg.push_back(l);
  }
  G.cell_off.assign(1, 0);
  for (auto& c : cells) {
    std::sort(c.begin(), c.end());
    G.cell_mod.insert(G.cell_mod.end(), c.begin(), c.end());
    G.cell_off.push_back((int)G.cell_mod.size());
  }
  auto by_pos = [&](int a, int b) {
    const float pa = std::fabs(G.layers[a].pos), pb = std::fabs(G.layers[b].pos);
    return pa < pb || (pa == pb && a < b);
  };
  std::sort(G.barrel.begin(), G.barrel.end(), by_pos);
  std::sort(G.disk_pos.begin(), G.disk_pos.end(), by_pos);
  std::sort(G.disk_neg.begin(), G.disk_neg.end(), by_pos);
  return CKF_OK;
}

template <class T>
ckf_status upload(ckf_geometry* g, const std::vector<T>& v, const T** out) {
  void* p = nullptr;
  const size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
  HIP_TRY(hipMalloc(&p, bytes), "hipMalloc(geometry)");
  g->allocations.push_back(p);
  if (!v.empty()) HIP_TRY(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy(geometry)");
  *out = static_cast<const T*>(p);
  return CKF_OK;
}

// Neighbour table of the learned proposal, in FP64 from the FP32 geometry.
// For module m: rays from the origin through its centre and corners
// (-,-), (+,-), (-,+), (+,+) in (loc0, loc1); each ray's next layer is the
// layer other than m's whose envelope it meets first, beyond the ray's
// point on m and within the envelope's extent.  The distinct next layers in
// ray order (at most kMaxNext) are kept, each with the anchor A where its
// first ray meets the envelope, the layer's module pitches there and the
// region of cells around A in the layer's curvilinear coordinates.
struct NbTable {
  std::vector<int> next, row, reg;
  std::vector<float4> anc;
};

double wrap_pi(double a) {
  a = std::fmod(a + kPi, 2.0 * kPi);
  if (a < 0) a += 2.0 * kPi;
  return a - kPi;
}

// curvilinear offset of point (x, y, z) from the anchor on layer L:
// barrels (R dphi, dz), disks (r dphi, dr) with r the point's radius
void layer_coords(const ckf_geometry_desc* d, int L, const double* X, const double* A, double& du, double& dv) {
  const double dphi = wrap_pi(std::atan2(X[1], X[0]) - std::atan2(A[1], A[0]));
  const double rX = std::hypot(X[0], X[1]);
  if (d->layer_type[L] == 0) {
    du = dphi * (double)d->layer_pos[L];
    dv = X[2] - A[2];
  } else {
    du = dphi * rX;
    dv = rX - std::hypot(A[0], A[1]);
  }
}

void build_neighbours(const ckf_geometry_desc* d, NbTable& T) {
  const int n = d->n_surfaces, nl = d->n_layers;
  T.next.assign((size_t)n * ckf::kMaxNext, -1);
  T.row.assign((size_t)n * ckf::kMaxNext, -1);
  T.reg.clear();
  T.anc.clear();
  std::vector<std::vector<int>> members(nl);
  for (int i = 0; i < n; ++i) members[d->layer[i]].push_back(i);
  std::vector<double> du, dv;
  for (int m = 0; m < n; ++m) {
    const float* c = d->center + 3 * m;
    const float* r = d->rot + 9 * m;
    const double h0 = d->half[2 * m], h1 = d->half[2 * m + 1];
    const double sgn[5][2] = {{0, 0}, {-1, -1}, {1, -1}, {-1, 1}, {1, 1}};
    int n_next = 0;
    for (int ray = 0; ray < 5 && n_next < ckf::kMaxNext; ++ray) {
      double q[3];
      for (int k = 0; k < 3; ++k)
        q[k] = ((double)c[k] + sgn[ray][0] * h0 * (double)r[k]) + sgn[ray][1] * h1 * (double)r[3 + k];
      const double tm = std::sqrt((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]);
      if (!(tm > 0)) continue;
      const double dvv[3] = {q[0] / tm, q[1] / tm, q[2] / tm};
      const double dperp = std::hypot(dvv[0], dvv[1]);
      int best = -1;
      double tbest = INFINITY;
      for (int L = 0; L < nl; ++L) {
        if (L == d->layer[m]) continue;
        const double pos = d->layer_pos[L], lo = d->layer_lo[L], hi = d->layer_hi[L];
        double t;
        if (d->layer_type[L] == 0) {
          if (!(dperp > 0)) continue;
          t = pos / dperp;
          const double z = t * dvv[2];
          if (!(z >= lo && z <= hi)) continue;
        } else {
          if (dvv[2] == 0) continue;
          t = pos / dvv[2];
          const double rr = t * dperp;
          if (!(t > 0 && rr >= lo && rr <= hi)) continue;
        }
        if (!(t > tm)) continue;
        if (t < tbest) {
          tbest = t;
          best = L;
        }
      }
      if (best < 0) continue;
      bool seen = false;
      for (int k = 0; k < n_next; ++k) seen = seen || T.next[(size_t)m * ckf::kMaxNext + k] == best;
      if (seen) continue;
      const double A[3] = {tbest * dvv[0], tbest * dvv[1], tbest * dvv[2]};
      // pitches from the module nearest to the anchor, then the cells
      const std::vector<int>& mem = members[best];
      du.resize(mem.size());
      dv.resize(mem.size());
      size_t a = 0;
      double d2best = INFINITY;
      for (size_t j = 0; j < mem.size(); ++j) {
        const double X[3] = {d->center[3 * mem[j]], d->center[3 * mem[j] + 1], d->center[3 * mem[j] + 2]};
        layer_coords(d, best, X, A, du[j], dv[j]);
        const double d2 = du[j] * du[j] + dv[j] * dv[j];
        if (d2 < d2best || (d2 == d2best && mem[j] < mem[a])) {
          d2best = d2;
          a = j;
        }
      }
      const int am = mem[a];
      double pu = INFINITY, pv = INFINITY;
      for (size_t j = 0; j < mem.size(); ++j) {
        const double ou = du[j] - du[a], ov = dv[j] - dv[a];
        if (std::fabs(ov) < d->half[2 * am + 1] && ou > 1e-3) pu = std::min(pu, ou);
      }
      if (!std::isfinite(pu)) pu = 2.0 * d->half[2 * am];
      for (size_t j = 0; j < mem.size(); ++j) {
        const double ou = du[j] - du[a], ov = dv[j] - dv[a];
        if (std::fabs(ou) < 0.5 * pu && ov > 1e-3) pv = std::min(pv, ov);
      }
      if (!std::isfinite(pv)) pv = 2.0 * d->half[2 * am + 1];
      const int row = (int)T.anc.size();
      std::vector<double> bestd(ckf::kRegCells, INFINITY);
      T.reg.resize((size_t)(row + 1) * ckf::kRegCells, -1);
      int* cells = T.reg.data() + (size_t)row * ckf::kRegCells;
      for (size_t j = 0; j < mem.size(); ++j) {
        const double iu = std::floor(du[j] / pu + 0.5), iv = std::floor(dv[j] / pv + 0.5);
        if (iu < ckf::kRegU0 || iu >= ckf::kRegU0 + ckf::kRegU || iv < ckf::kRegV0 || iv >= ckf::kRegV0 + ckf::kRegV)
          continue;
        const int k = (int)(iv - ckf::kRegV0) * ckf::kRegU + (int)(iu - ckf::kRegU0);
        const double eu = du[j] - iu * pu, ev = dv[j] - iv * pv;
        const double dist = eu * eu + ev * ev;
        if (dist < bestd[k] || (dist == bestd[k] && mem[j] < cells[k])) {
          bestd[k] = dist;
          cells[k] = mem[j];
        }
      }
      const double wA = d->layer_type[best] == 0 ? A[2] : std::hypot(A[0], A[1]);
      T.anc.push_back(make_float4((float)std::atan2(A[1], A[0]), (float)wA, (float)pu, (float)pv));
      T.next[(size_t)m * ckf::kMaxNext + n_next] = best;
      T.row[(size_t)m * ckf::kMaxNext + n_next] = row;
      ++n_next;
    }
  }
}

ckf_status check_config(const ckf_config* c) {
  if (!c) return fail(CKF_ERR_INVALID_ARGUMENT, "config is NULL");
  if (!(c->chi2_max > 0) || !(c->step_tol > 0) || !(c->step_max > 0) || !(c->land_tol > 0) || !(c->path_max > 0) ||
      !(c->nav_margin >= 0) || !(c->mass >= 0) || c->max_holes < 0 || c->min_meas < 0 || c->max_steps < 1 ||
      c->max_rk_steps < 1)
    return fail(CKF_ERR_INVALID_ARGUMENT, "config value out of range");
  if (c->branches_per_surface < 1 || c->branches_per_surface > ckf::kMaxBranch)
    return fail(CKF_ERR_NOT_SUPPORTED, "branches_per_surface must be 1..4 on the GPU");
  if (c->max_live_per_seed < 1 || c->max_live_per_seed * c->branches_per_surface > 64)
    return fail(CKF_ERR_NOT_SUPPORTED, "max_live_per_seed * branches_per_surface must be 1..64 on the GPU");
  if (c->max_steps > ckf::kMaxSteps) return fail(CKF_ERR_NOT_SUPPORTED, "max_steps must be <= 64");
  if (c->tracks_per_seed != 0 && c->tracks_per_seed != 1)
    return fail(CKF_ERR_NOT_SUPPORTED, "tracks_per_seed must be 1 (best) or 0 (all finished) on the GPU");
  if (c->nav_margin > ckf::kMaxNavMargin) return fail(CKF_ERR_NOT_SUPPORTED, "nav_margin must be <= 2 mm");
  if (!(c->learned_min_prob >= 0) || c->learned_topk < 1 || c->learned_topk > 3)
    return fail(CKF_ERR_INVALID_ARGUMENT, "learned_min_prob must be >= 0 and learned_topk 1..3");
  return CKF_OK;
}

ckf::CfgDev to_dev(const ckf_config* c) {
  ckf::CfgDev d;
  d.chi2_max = c->chi2_max;
  d.branches = c->branches_per_surface;
  d.max_live = c->max_live_per_seed;
  d.max_holes = c->max_holes;
  d.min_meas = c->min_meas;
  d.max_steps = c->max_steps;
  d.max_rk = c->max_rk_steps;
  d.step_tol = (float)c->step_tol;
  d.step_max = (float)c->step_max;
  d.land_tol = (float)c->land_tol;
  d.path_max = (float)c->path_max;
  d.nav_margin = (float)c->nav_margin;
  d.mass = c->mass;
  d.material = c->material_on != 0;
  d.min_prob = (float)c->learned_min_prob;
  d.topk = c->learned_topk;
  d.all_tracks = c->tracks_per_seed == 0;
  return d;
}

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
  return cus;
}

constexpr int kDefaultSeedsPerGroup = 48;
constexpr int kNodesPerSeed = 32;
constexpr int kFinPerSeed = 64;  // finished candidates kept per seed on average (tracks_per_seed = 0)

ckf::Launch resolve_launch(const ckf_config* c, const ckf_launch* l, int n_seeds) {
  ckf::Launch r;
  r.waves_per_simd = (l && l->waves_per_simd > 0) ? std::min(3, l->waves_per_simd) : 3;
  r.seeds_per_group = (l && l->seeds_per_group > 0) ? std::min(64, l->seeds_per_group) : kDefaultSeedsPerGroup;
  const int want = (n_seeds + r.seeds_per_group - 1) / r.seeds_per_group;
  // one workgroup per wave slot: 4 SIMDs per CU times the waves per SIMD
  const int dflt = device_cus() * 4 * r.waves_per_simd;
  r.grid = std::max(1, std::min((l && l->grid > 0) ? l->grid : dflt, std::max(1, want)));
  r.pool_cap = r.seeds_per_group * (c->max_live_per_seed * c->branches_per_surface + 1);
  r.nodes_per_seed = (l && l->nodes_per_seed > 0) ? l->nodes_per_seed : kNodesPerSeed;
  return r;
}

struct Layout {
  size_t off_sorted, off_key, off_id, off_rowof, off_maxv, off_nodes, off_nodecnt, off_queue, off_res_node,
      off_res_nm, off_res_holes, off_res_chi2, off_scan_a, off_scan_b, off_pools, off_fin_seed, off_fin_node,
      off_fin_nmh, off_fin_chi2, off_fin_count, off_seed_cnt, off_seed_meas, off_seed_fill, off_fin_order, total;
  long long node_cap, fin_cap;
};

Layout layout(const ckf::Launch& L, int n_events, int n_surfaces, int n_seeds, long long n_meas, bool all_tracks) {
  Layout o;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t r = at;
    at = align_up(at + std::max<size_t>(bytes, 1));
    return r;
  };
  const size_t nm = (size_t)std::max<long long>(n_meas, 1);
  const size_t rows = (size_t)std::max(1, n_events * n_surfaces);
  const size_t ns = (size_t)std::max(1, n_seeds);
  o.node_cap = (long long)ns * L.nodes_per_seed + 1024;
  o.off_sorted = take(nm * 16);
  o.off_key = take(nm * 4);
  o.off_id = take(nm * 4);
  o.off_rowof = take(nm * 4);
  o.off_maxv = take(rows * 4);
  o.off_nodes = take((size_t)o.node_cap * sizeof(ckf::Node));
  o.off_nodecnt = take(8);
  o.off_queue = take(ckf::kSeedQueues * 4);
  o.off_res_node = take(ns * 4);
  o.off_res_nm = take(ns * 4);
  o.off_res_holes = take(ns * 4);
  o.off_res_chi2 = take(ns * 8);
  const size_t nb = (ns + 255) / 256 + 1;
  o.off_scan_a = take(nb * 4);
  o.off_scan_b = take(nb * 4);
  o.off_pools = take((size_t)L.grid * 2 * L.pool_cap * ckf::kRecStride);
  // every finished candidate (tracks_per_seed = 0 only)
  o.fin_cap = all_tracks ? (long long)ns * kFinPerSeed + 1024 : 0;
  const size_t fc = (size_t)std::max<long long>(o.fin_cap, 1), sn = all_tracks ? ns : 1;
  o.off_fin_seed = take(fc * 4);
  o.off_fin_node = take(fc * 4);
  o.off_fin_nmh = take(fc * 4);
  o.off_fin_chi2 = take(fc * 8);
  o.off_fin_count = take(8);
  o.off_seed_cnt = take(sn * 4);
  o.off_seed_meas = take(sn * 4);
  o.off_seed_fill = take(sn * 4);
  o.off_fin_order = take(fc * 4);
  o.total = at;
  return o;
}

}  // namespace

extern "C" {

const char* ckf_status_string(ckf_status s) {
  switch (s) {
    case CKF_OK: return "ok";
    case CKF_ERR_INVALID_ARGUMENT: return "invalid argument";
    case CKF_ERR_UNSORTED_INPUT: return "unsorted input";
    case CKF_ERR_CAPACITY: return "capacity too small";
    case CKF_ERR_DEVICE: return "device error";
    case CKF_ERR_NOT_SUPPORTED: return "not supported";
    case CKF_ERR_NO_MODEL: return "no model";
  }
  return "unknown status";
}

const char* ckf_last_error(void) { return g_last_error.c_str(); }

void ckf_config_default(ckf_config* c) {
  if (!c) return;
  c->chi2_max = 15.0;
  c->branches_per_surface = 3;
  c->max_live_per_seed = 10;
  c->max_holes = 3;
  c->min_meas = 6;
  c->max_steps = 48;
  c->max_rk_steps = 100;
  c->step_tol = 1e-2;
  c->step_max = 200.0;
  c->land_tol = 1e-4;
  c->path_max = 4000.0;
  c->nav_margin = 1.0;
  c->mass = 0.1056583755;
  c->material_on = 1;
  c->tracks_per_seed = 1;
  c->learned_min_prob = 0.95;
  c->learned_topk = 3;
}

ckf_status ckf_geometry_create(const ckf_geometry_desc* d, ckf_geometry** out) {
  if (!d || !out) return fail(CKF_ERR_INVALID_ARGUMENT, "geometry_create: NULL argument");
  *out = nullptr;
  if (d->n_surfaces <= 0 || d->n_layers <= 0) return fail(CKF_ERR_INVALID_ARGUMENT, "geometry: empty");
  if (d->n_layers > ckf::kMaxLayers) return fail(CKF_ERR_NOT_SUPPORTED, "geometry: more than 64 layers");
  if (!d->center || !d->rot || !d->half || !d->thick || !d->layer || !d->layer_type || !d->layer_pos ||
      !d->layer_lo || !d->layer_hi)
    return fail(CKF_ERR_INVALID_ARGUMENT, "geometry: NULL array");
  for (int l = 0; l < d->n_layers; ++l) {
    if (d->layer_type[l] != 0 && d->layer_type[l] != 1) return fail(CKF_ERR_INVALID_ARGUMENT, "geometry: layer type");
    if (!std::isfinite(d->layer_pos[l]) || !(d->layer_lo[l] <= d->layer_hi[l]))
      return fail(CKF_ERR_INVALID_ARGUMENT, "geometry: layer envelope");
    if (d->layer_type[l] == 0 && !(d->layer_pos[l] > 0)) return fail(CKF_ERR_INVALID_ARGUMENT, "geometry: barrel radius");
  }
  std::vector<ckf::Module> mods(d->n_surfaces);
  for (int i = 0; i < d->n_surfaces; ++i) {
    const float* r = d->rot + 9 * i;
    if (!finite3(d->center + 3 * i) || !finite3(r) || !finite3(r + 3) || !finite3(r + 6) ||
        !(d->half[2 * i] > 0) || !(d->half[2 * i + 1] > 0) || !(d->thick[i] >= 0) || d->layer[i] < 0 ||
        d->layer[i] >= d->n_layers)
      return fail(CKF_ERR_INVALID_ARGUMENT, "geometry: bad module " + std::to_string(i));
    ckf::Module& M = mods[i];
    for (int k = 0; k < 3; ++k) {
      M.c[k] = d->center[3 * i + k];
      M.u[k] = r[k];
      M.v[k] = r[3 + k];
      M.n[k] = r[6 + k];
    }
    M.hw0 = d->half[2 * i];
    M.hw1 = d->half[2 * i + 1];
    M.thick = d->thick[i];
    M.layer = d->layer[i];
  }
  HostGrid G;
  ckf_status st = build_grid(d, mods, G);
  if (st != CKF_OK) return st;
  NbTable nb;
  build_neighbours(d, nb);
  int device = 0;
  const hipError_t ed = hipGetDevice(&device);
  if (ed != hipSuccess) return hip_fail(ed, "hipGetDevice");
  ckf_geometry* g = new ckf_geometry();
  g->device = device;
  auto cleanup = [&](ckf_status s) {
    for (void* p : g->allocations) (void)hipFree(p);
    delete g;
    return s;
  };
  const ckf::Module* dm;
  const ckf::LayerRec* dl;
  const int *co, *cm, *bo, *dp, *dn, *nn, *nr, *ng;
  const float4* na;
  if ((st = upload(g, mods, &dm)) != CKF_OK || (st = upload(g, G.layers, &dl)) != CKF_OK ||
      (st = upload(g, G.cell_off, &co)) != CKF_OK || (st = upload(g, G.cell_mod, &cm)) != CKF_OK ||
      (st = upload(g, G.barrel, &bo)) != CKF_OK || (st = upload(g, G.disk_pos, &dp)) != CKF_OK ||
      (st = upload(g, G.disk_neg, &dn)) != CKF_OK || (st = upload(g, nb.next, &nn)) != CKF_OK ||
      (st = upload(g, nb.row, &nr)) != CKF_OK || (st = upload(g, nb.anc, &na)) != CKF_OK ||
      (st = upload(g, nb.reg, &ng)) != CKF_OK)
    return cleanup(st);
  g->dev.nb_next = nn;
  g->dev.nb_row = nr;
  g->dev.nb_anc = na;
  g->dev.nb_reg = ng;
  g->nb_rows = (int)nb.anc.size();
  g->dev.n_surfaces = d->n_surfaces;
  g->dev.n_layers = d->n_layers;
  g->dev.mod = dm;
  g->dev.layers = dl;
  g->dev.cell_off = co;
  g->dev.cell_mod = cm;
  g->dev.barrel_order = bo;
  g->dev.disk_pos = dp;
  g->dev.disk_neg = dn;
  g->dev.n_barrel = (int)G.barrel.size();
  g->dev.n_disk_pos = (int)G.disk_pos.size();
  g->dev.n_disk_neg = (int)G.disk_neg.size();
  *out = g;
  return CKF_OK;
}

void ckf_geometry_destroy(ckf_geometry* g) {
  if (!g) return;
  for (void* p : g->allocations) (void)hipFree(p);
  delete g;
}

ckf_status ckf_field_create_uniform(float bx, float by, float bz, ckf_field** out) {
  if (!out) return fail(CKF_ERR_INVALID_ARGUMENT, "field_create: NULL out");
  if (!std::isfinite(bx) || !std::isfinite(by) || !std::isfinite(bz))
    return fail(CKF_ERR_INVALID_ARGUMENT, "field_create: non-finite field");
  ckf_field* f = new ckf_field();
  f->dev = {bx, by, bz};
  *out = f;
  return CKF_OK;
}

ckf_status ckf_field_create_rz(const float* values, int32_t nr, int32_t nz, float r0, float z0, float dr, float dz,
                               ckf_field** out) {
  if (!values || !out) return fail(CKF_ERR_INVALID_ARGUMENT, "field_create_rz: NULL argument");
  *out = nullptr;
  if (nr < 2 || nz < 2 || !(dr > 0) || !(dz > 0) || !std::isfinite(r0) || !std::isfinite(z0) ||
      (long long)nr * nz > (1ll << 28))
    return fail(CKF_ERR_INVALID_ARGUMENT, "field_create_rz: bad grid");
  // per (iz, ir): (B_r, B_z) at ir and at ir+1, so a cell row is one 16-byte load
  std::vector<float4> dev((size_t)nr * nz);
  for (int iz = 0; iz < nz; ++iz)
    for (int ir = 0; ir < nr; ++ir) {
      const int i1 = std::min(ir + 1, nr - 1);
      const float* a = values + ((size_t)iz * nr + ir) * 2;
      const float* b = values + ((size_t)iz * nr + i1) * 2;
      if (!std::isfinite(a[0]) || !std::isfinite(a[1])) return fail(CKF_ERR_INVALID_ARGUMENT, "field map: non-finite");
      dev[(size_t)iz * nr + ir] = make_float4(a[0], a[1], b[0], b[1]);
    }
  ckf_field* f = new ckf_field();
  const hipError_t e = hipMalloc(&f->map, dev.size() * sizeof(float4));
  if (e != hipSuccess) {
    delete f;
    return hip_fail(e, "hipMalloc(field map)");
  }
  const hipError_t e2 = hipMemcpy(f->map, dev.data(), dev.size() * sizeof(float4), hipMemcpyHostToDevice);
  if (e2 != hipSuccess) {
    (void)hipFree(f->map);
    delete f;
    return hip_fail(e2, "hipMemcpy(field map)");
  }
  f->dev.map = static_cast<const float4*>(f->map);
  f->dev.nr = nr;
  f->dev.nz = nz;
  f->dev.r0 = r0;
  f->dev.z0 = z0;
  f->dev.inv_dr = 1.0f / dr;
  f->dev.inv_dz = 1.0f / dz;
  *out = f;
  return CKF_OK;
}

void ckf_field_destroy(ckf_field* f) {
  if (!f) return;
  if (f->map) (void)hipFree(f->map);
  delete f;
}

ckf_status ckf_workspace_size(const ckf_geometry* g, const ckf_config* cfg, const ckf_launch* launch,
                              int32_t n_events, int32_t n_seeds, int64_t n_meas, size_t* bytes) {
  if (!g || !bytes) return fail(CKF_ERR_INVALID_ARGUMENT, "workspace_size: NULL argument");
  ckf_status st = check_config(cfg);
  if (st != CKF_OK) return st;
  if (n_events < 0 || n_seeds < 0 || n_meas < 0) return fail(CKF_ERR_INVALID_ARGUMENT, "workspace_size: negative size");
  if (n_meas > INT32_MAX) return fail(CKF_ERR_NOT_SUPPORTED, "more than 2^31 measurements");
  const ckf::Launch L = resolve_launch(cfg, launch, n_seeds);
  *bytes = layout(L, n_events, g->dev.n_surfaces, n_seeds, n_meas, cfg->tracks_per_seed == 0).total;
  return CKF_OK;
}

ckf_status ckf_find(const ckf_geometry* g, const ckf_field* f, const ckf_measurements* m, const ckf_seeds* s,
                    const ckf_config* cfg, const ckf_launch* launch, const ckf_model* model, void* workspace,
                    size_t workspace_bytes, ckf_tracks* out, void* stream) {
  if (!g || !f || !m || !s || !out) return fail(CKF_ERR_INVALID_ARGUMENT, "ckf_find: NULL argument");
  ckf_status st = check_config(cfg);
  if (st != CKF_OK) return st;
  if (m->n_surfaces != g->dev.n_surfaces) return fail(CKF_ERR_INVALID_ARGUMENT, "measurements: n_surfaces mismatch");
  if (m->n_events < 1 || m->n_meas < 0 || s->n_seeds < 0) return fail(CKF_ERR_INVALID_ARGUMENT, "bad batch sizes");
  if (m->n_meas > INT32_MAX) return fail(CKF_ERR_NOT_SUPPORTED, "more than 2^31 measurements");
  if ((long long)m->n_events * m->n_surfaces >= INT32_MAX) return fail(CKF_ERR_NOT_SUPPORTED, "too many rows");
  if (!m->offsets || (m->n_meas > 0 && (!m->loc || !m->var)))
    return fail(CKF_ERR_INVALID_ARGUMENT, "measurements: NULL array");
  if (s->n_seeds > 0 && (!s->event || !s->surface || !s->params || !s->cov))
    return fail(CKF_ERR_INVALID_ARGUMENT, "seeds: NULL array");
  if (!out->n_tracks || !out->offsets || !out->status || out->cap_tracks < 0 || out->cap_meas < 0)
    return fail(CKF_ERR_INVALID_ARGUMENT, "tracks: NULL array or negative capacity");
  if (out->cap_tracks > 0 && (!out->params || !out->cov || !out->chi2 || !out->ndf || !out->holes || !out->seed ||
                              !out->event || !out->last_surface))
    return fail(CKF_ERR_INVALID_ARGUMENT, "tracks: NULL array");
  if (out->cap_meas > 0 && !out->meas) return fail(CKF_ERR_INVALID_ARGUMENT, "tracks: NULL meas");
  if (!workspace) return fail(CKF_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (model && f->dev.map) return fail(CKF_ERR_NOT_SUPPORTED, "the learned proposal runs in a uniform field");
  const ckf::Launch L = resolve_launch(cfg, launch, s->n_seeds);
  const Layout o = layout(L, m->n_events, m->n_surfaces, s->n_seeds, m->n_meas, cfg->tracks_per_seed == 0);
  if (workspace_bytes < o.total)
    return fail(CKF_ERR_CAPACITY, "workspace too small: need " + std::to_string(o.total) + " bytes");
  char* ws = static_cast<char*>(workspace);
  ckf::Workspace w;
  w.m_sorted = reinterpret_cast<float4*>(ws + o.off_sorted);
  w.m_key = reinterpret_cast<float*>(ws + o.off_key);
  w.m_id = reinterpret_cast<int*>(ws + o.off_id);
  w.row_of = reinterpret_cast<int*>(ws + o.off_rowof);
  w.row_maxvar0 = reinterpret_cast<float*>(ws + o.off_maxv);
  w.nodes = reinterpret_cast<ckf::Node*>(ws + o.off_nodes);
  w.node_cap = o.node_cap;
  w.node_count = reinterpret_cast<unsigned long long*>(ws + o.off_nodecnt);
  w.queue_head = reinterpret_cast<int*>(ws + o.off_queue);
  w.res_node = reinterpret_cast<int*>(ws + o.off_res_node);
  w.res_nm = reinterpret_cast<int*>(ws + o.off_res_nm);
  w.res_holes = reinterpret_cast<int*>(ws + o.off_res_holes);
  w.res_chi2 = reinterpret_cast<double*>(ws + o.off_res_chi2);
  w.scan_a = reinterpret_cast<int*>(ws + o.off_scan_a);
  w.scan_b = reinterpret_cast<int*>(ws + o.off_scan_b);
  w.pools = ws + o.off_pools;
  w.fin_seed = reinterpret_cast<int*>(ws + o.off_fin_seed);
  w.fin_node = reinterpret_cast<int*>(ws + o.off_fin_node);
  w.fin_nmh = reinterpret_cast<int*>(ws + o.off_fin_nmh);
  w.fin_chi2 = reinterpret_cast<double*>(ws + o.off_fin_chi2);
  w.fin_count = reinterpret_cast<unsigned long long*>(ws + o.off_fin_count);
  w.fin_cap = o.fin_cap;
  w.seed_cnt = reinterpret_cast<int*>(ws + o.off_seed_cnt);
  w.seed_meas = reinterpret_cast<int*>(ws + o.off_seed_meas);
  w.seed_fill = reinterpret_cast<int*>(ws + o.off_seed_fill);
  w.fin_order = reinterpret_cast<int*>(ws + o.off_fin_order);
  w.pool_cap = L.pool_cap;
  w.seeds_per_group = L.seeds_per_group;
  w.grid = L.grid;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  ckf::MeasIn mi{m->n_events, m->n_surfaces, (long long)m->n_meas, m->offsets, m->loc, m->var};
  HIP_TRY(ckf::launch_init(s->n_seeds, w, *out, hs), "launch k_init");
  HIP_TRY(ckf::launch_meas_prepare(mi, w, out->status, hs), "launch k_meas_prepare");
  if (s->n_seeds > 0) {
    ckf::CkfArgs a;
    a.g = g->dev;
    a.f = f->dev;
    a.cfg = to_dev(cfg);
    a.m = mi;
    a.s = {s->n_seeds, s->event, s->surface, s->params, s->cov};
    a.w = w;
    a.status = out->status;
    a.counters = reinterpret_cast<long long*>(out->counters);
    a.learned = model != nullptr;
    a.model = model ? ckf::model_view(model->buf) : ckf::ModelDev{};
    a.seed_flags = out->seed_flags;
    if (launch && launch->timer) HIP_TRY(hipEventRecord(launch->timer->start, hs), "hipEventRecord");
    HIP_TRY(ckf::launch_ckf(a, L.waves_per_simd, hs), "launch k_ckf");
    if (launch && launch->timer) HIP_TRY(hipEventRecord(launch->timer->stop, hs), "hipEventRecord");
  }
  if (cfg->tracks_per_seed == 0)
    HIP_TRY(ckf::launch_output_all(s->n_seeds, w, s->event, *out, hs), "launch output (all finished)");
  else
    HIP_TRY(ckf::launch_output(s->n_seeds, w, s->event, *out, hs), "launch output");
  return CKF_OK;
}

ckf_status ckf_plan_create(const ckf_geometry* g, const ckf_field* f, const ckf_measurements* m,
                           const ckf_seeds* s, const ckf_config* cfg, const ckf_launch* launch,
                           const ckf_model* model, void* workspace, size_t workspace_bytes, ckf_tracks* out,
                           void* stream, ckf_plan** plan) {
  if (!plan) return fail(CKF_ERR_INVALID_ARGUMENT, "plan_create: NULL plan");
  *plan = nullptr;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  if (!hs) return fail(CKF_ERR_INVALID_ARGUMENT, "plan_create: capture needs a non-default stream");
  ckf_launch l{};
  if (launch) l = *launch;
  l.timer = nullptr;
  HIP_TRY(hipStreamBeginCapture(hs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  const ckf_status st = ckf_find(g, f, m, s, cfg, &l, model, workspace, workspace_bytes, out, stream);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(hs, &graph);
  if (st != CKF_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
  ckf_plan* p = new ckf_plan();
  p->graph = graph;
  const hipError_t ei = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(graph);
    delete p;
    return hip_fail(ei, "hipGraphInstantiate");
  }
  *plan = p;
  return CKF_OK;
}

ckf_status ckf_plan_launch(ckf_plan* plan, void* stream) {
  if (!plan || !plan->exec) return fail(CKF_ERR_INVALID_ARGUMENT, "plan_launch: NULL plan");
  HIP_TRY(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)), "hipGraphLaunch");
  return CKF_OK;
}

void ckf_plan_destroy(ckf_plan* plan) {
  if (!plan) return;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  delete plan;
}

ckf_status ckf_timer_create(ckf_timer** out) {
  if (!out) return fail(CKF_ERR_INVALID_ARGUMENT, "timer_create: NULL out");
  ckf_timer* t = new ckf_timer();
  hipError_t e = hipEventCreate(&t->start);
  if (e == hipSuccess) e = hipEventCreate(&t->stop);
  if (e != hipSuccess) {
    delete t;
    return hip_fail(e, "hipEventCreate");
  }
  *out = t;
  return CKF_OK;
}

void ckf_timer_destroy(ckf_timer* t) {
  if (!t) return;
  (void)hipEventDestroy(t->start);
  (void)hipEventDestroy(t->stop);
  delete t;
}

ckf_status ckf_timer_elapsed_ms(ckf_timer* t, float* ms) {
  if (!t || !ms) return fail(CKF_ERR_INVALID_ARGUMENT, "timer_elapsed: NULL argument");
  HIP_TRY(hipEventSynchronize(t->stop), "hipEventSynchronize");
  HIP_TRY(hipEventElapsedTime(ms, t->start, t->stop), "hipEventElapsedTime");
  return CKF_OK;
}

ckf_status ckf_propagate_batch(const ckf_geometry* g, const ckf_field* f, const ckf_config* cfg, int32_t n,
                               const int32_t* src, const double* p_in, const double* cov_in, const int32_t* dst,
                               double* p_out, double* cov_out, double* jac, double* path, int32_t* ok,
                               void* stream) {
  if (!g || !f || !cfg) return fail(CKF_ERR_INVALID_ARGUMENT, "propagate_batch: NULL argument");
  if (n < 0) return fail(CKF_ERR_INVALID_ARGUMENT, "propagate_batch: negative n");
  if (n > 0 && (!src || !p_in || !cov_in || !dst || !p_out || !cov_out || !ok))
    return fail(CKF_ERR_INVALID_ARGUMENT, "propagate_batch: NULL array");
  ckf_status st = check_config(cfg);
  if (st != CKF_OK) return st;
  HIP_TRY(ckf::launch_propagate(g->dev, f->dev, to_dev(cfg), n, src, p_in, cov_in, dst, p_out, cov_out, jac, path, ok,
                                static_cast<hipStream_t>(stream)),
          "launch k_propagate_batch");
  return CKF_OK;
}

ckf_status ckf_kf_update_batch(int32_t n, const double* p_in, const double* cov_in, const float* meas,
                               const float* var, double* p_out, double* cov_out, double* chi2, void* stream) {
  if (n < 0) return fail(CKF_ERR_INVALID_ARGUMENT, "kf_update_batch: negative n");
  if (n > 0 && (!p_in || !cov_in || !meas || !var || !p_out || !cov_out))
    return fail(CKF_ERR_INVALID_ARGUMENT, "kf_update_batch: NULL array");
  HIP_TRY(ckf::launch_kf_update(n, p_in, cov_in, meas, var, p_out, cov_out, chi2, static_cast<hipStream_t>(stream)),
          "launch k_kf_update_batch");
  return CKF_OK;
}

ckf_status ckf_geometry_neighbours(const ckf_geometry* g, int32_t* next_layers, float* anchors, int32_t* regions) {
  if (!g || !next_layers || !anchors || !regions)
    return fail(CKF_ERR_INVALID_ARGUMENT, "geometry_neighbours: NULL argument");
  const size_t n = (size_t)g->dev.n_surfaces * ckf::kMaxNext;
  std::vector<int> row(n);
  std::vector<float4> anc(std::max(1, g->nb_rows));
  std::vector<int> reg((size_t)std::max(1, g->nb_rows) * ckf::kRegCells);
  HIP_TRY(hipMemcpy(next_layers, g->dev.nb_next, n * sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy(neighbours)");
  HIP_TRY(hipMemcpy(row.data(), g->dev.nb_row, n * sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy(neighbours)");
  if (g->nb_rows > 0) {
    HIP_TRY(hipMemcpy(anc.data(), g->dev.nb_anc, (size_t)g->nb_rows * sizeof(float4), hipMemcpyDeviceToHost),
            "hipMemcpy(neighbours)");
    HIP_TRY(hipMemcpy(reg.data(), g->dev.nb_reg, (size_t)g->nb_rows * ckf::kRegCells * sizeof(int),
                      hipMemcpyDeviceToHost),
            "hipMemcpy(neighbours)");
  }
  for (size_t i = 0; i < n; ++i) {
    float* a = anchors + 4 * i;
    int32_t* r = regions + i * ckf::kRegCells;
    if (row[i] < 0) {
      a[0] = a[1] = a[2] = a[3] = 0.f;
      for (int k = 0; k < ckf::kRegCells; ++k) r[k] = -1;
      continue;
    }
    const float4 v = anc[row[i]];
    a[0] = v.x;
    a[1] = v.y;
    a[2] = v.z;
    a[3] = v.w;
    std::memcpy(r, reg.data() + (size_t)row[i] * ckf::kRegCells, ckf::kRegCells * sizeof(int));
  }
  return CKF_OK;
}

ckf_status ckf_model_create(const float* params, void* stream, ckf_model** out) {
  if (!params || !out) return fail(CKF_ERR_INVALID_ARGUMENT, "model_create: NULL argument");
  *out = nullptr;
  if (reinterpret_cast<uintptr_t>(params) % 16 != 0)
    return fail(CKF_ERR_INVALID_ARGUMENT, "model_create: params must be 16-byte aligned");
  int device = 0;
  const hipError_t ed = hipGetDevice(&device);
  if (ed != hipSuccess) return hip_fail(ed, "hipGetDevice");
  ckf_model* md = new ckf_model();
  md->device = device;
  const hipError_t e = hipMalloc(&md->buf, ckf::kModelBytes);
  if (e != hipSuccess) {
    delete md;
    return hip_fail(e, "hipMalloc(model)");
  }
  const hipError_t e2 = ckf::launch_model_pack(params, md->buf, static_cast<hipStream_t>(stream));
  if (e2 != hipSuccess) {
    (void)hipFree(md->buf);
    delete md;
    return hip_fail(e2, "launch k_model_pack");
  }
  *out = md;
  return CKF_OK;
}

ckf_status ckf_model_update(ckf_model* model, const float* params, void* stream) {
  if (!model || !params) return fail(CKF_ERR_INVALID_ARGUMENT, "model_update: NULL argument");
  if (reinterpret_cast<uintptr_t>(params) % 16 != 0)
    return fail(CKF_ERR_INVALID_ARGUMENT, "model_update: params must be 16-byte aligned");
  HIP_TRY(ckf::launch_model_pack(params, model->buf, static_cast<hipStream_t>(stream)), "launch k_model_pack");
  return CKF_OK;
}

void ckf_model_destroy(ckf_model* model) {
  if (!model) return;
  (void)hipFree(model->buf);
  delete model;
}

ckf_status ckf_mlp_forward(const ckf_model* model, const float* x, int64_t n, float* logits, void* stream) {
  if (!model || n < 0 || (n > 0 && (!x || !logits))) return fail(CKF_ERR_INVALID_ARGUMENT, "mlp_forward: bad argument");
  if (reinterpret_cast<uintptr_t>(logits) % 16 != 0)
    return fail(CKF_ERR_INVALID_ARGUMENT, "mlp_forward: logits must be 16-byte aligned");
  HIP_TRY(ckf::launch_mlp_forward(ckf::model_view(model->buf), x, n, logits, static_cast<hipStream_t>(stream)),
          "launch k_mlp_forward");
  return CKF_OK;
}

ckf_status ckf_mlp_workspace_size(int64_t n, size_t* bytes) {
  if (n < 1 || !bytes) return fail(CKF_ERR_INVALID_ARGUMENT, "mlp_workspace_size: bad argument");
  *bytes = ckf::mlp_workspace_bytes(n);
  return CKF_OK;
}

ckf_status ckf_mlp_grad(const float* params, const float* x, const int32_t* labels, const int32_t* rows, int64_t n,
                        void* workspace, size_t workspace_bytes, float* grad, float* loss, void* stream) {
  if (!params || !x || !labels || !workspace || !grad || !loss || n < 1)
    return fail(CKF_ERR_INVALID_ARGUMENT, "mlp_grad: bad argument");
  if (reinterpret_cast<uintptr_t>(params) % 16 != 0)
    return fail(CKF_ERR_INVALID_ARGUMENT, "mlp_grad: params must be 16-byte aligned");
  if (n > (int64_t)INT32_MAX * 64) return fail(CKF_ERR_NOT_SUPPORTED, "mlp_grad: batch too large");
  if (workspace_bytes < ckf::mlp_workspace_bytes(n)) return fail(CKF_ERR_CAPACITY, "mlp_grad: workspace too small");
  HIP_TRY(ckf::launch_mlp_grad(params, x, labels, rows, n, workspace, grad, loss, static_cast<hipStream_t>(stream)),
          "launch k_mlp_grad");
  return CKF_OK;
}

ckf_status ckf_mlp_adam(float* params, float* m, float* v, const float* grad, int32_t step, float lr, float beta1,
                        float beta2, float eps, void* stream) {
  if (!params || !m || !v || !grad || step < 1 || !(lr >= 0) || !(beta1 >= 0 && beta1 < 1) ||
      !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(CKF_ERR_INVALID_ARGUMENT, "mlp_adam: bad argument");
  HIP_TRY(ckf::launch_mlp_adam(params, m, v, grad, step, lr, beta1, beta2, eps, static_cast<hipStream_t>(stream)),
          "launch k_mlp_adam");
  return CKF_OK;
}

ckf_status ckf_fit_workspace_size(int64_t cap_meas, size_t* bytes) {
  if (cap_meas < 0 || !bytes) return fail(CKF_ERR_INVALID_ARGUMENT, "fit_workspace_size: bad argument");
  *bytes = ckf::fit_workspace_bytes(cap_meas);
  return CKF_OK;
}

ckf_status ckf_fit(const ckf_geometry* g, const ckf_field* f, const ckf_measurements* m, const ckf_seeds* s,
                   const ckf_config* cfg, const int32_t* n_tracks, int32_t cap_tracks, int64_t cap_meas,
                   const int32_t* offsets, const int32_t* meas, const int32_t* meas_surface, const int32_t* seed,
                   int32_t smoother, void* workspace, size_t workspace_bytes, double* params, double* cov,
                   double* chi2, int32_t* ok, void* stream) {
  if (!g || !f || !m || !s || !cfg) return fail(CKF_ERR_INVALID_ARGUMENT, "fit: NULL argument");
  if (cap_tracks < 0 || cap_meas < 0) return fail(CKF_ERR_INVALID_ARGUMENT, "fit: negative capacity");
  if (smoother != CKF_SMOOTHER_RTS && smoother != CKF_SMOOTHER_TWO_FILTER)
    return fail(CKF_ERR_INVALID_ARGUMENT, "fit: unknown smoother");
  if (m->n_surfaces != g->dev.n_surfaces) return fail(CKF_ERR_INVALID_ARGUMENT, "fit: n_surfaces differs from geometry");
  if (cap_tracks > 0 && (!n_tracks || !offsets || !seed || !chi2 || !ok))
    return fail(CKF_ERR_INVALID_ARGUMENT, "fit: NULL track array");
  if (cap_meas > 0 && (!meas || !meas_surface || !params || !cov))
    return fail(CKF_ERR_INVALID_ARGUMENT, "fit: NULL measurement array");
  if (cap_tracks > 0 && (!s->surface || !s->params || !s->cov || (m->n_meas > 0 && (!m->loc || !m->var))))
    return fail(CKF_ERR_INVALID_ARGUMENT, "fit: NULL seed or measurement input");
  ckf_status st = check_config(cfg);
  if (st != CKF_OK) return st;
  if (workspace_bytes < ckf::fit_workspace_bytes(cap_meas) || (cap_meas > 0 && !workspace))
    return fail(CKF_ERR_CAPACITY, "fit: workspace too small");
  const ckf::MeasIn mi{m->n_events, m->n_surfaces, (long long)m->n_meas, m->offsets, m->loc, m->var};
  const ckf::SeedsIn si{s->n_seeds, s->event, s->surface, s->params, s->cov};
  HIP_TRY(ckf::launch_fit(g->dev, f->dev, to_dev(cfg), mi, si, n_tracks, cap_tracks, cap_meas, offsets, meas,
                          meas_surface, seed, smoother == CKF_SMOOTHER_TWO_FILTER, workspace, params, cov, chi2, ok,
                          static_cast<hipStream_t>(stream)),
          "launch the fit");
  return CKF_OK;
}

ckf_status ckf_fit_noalloc(const ckf_geometry* g, const ckf_field* f, const ckf_measurements* m,
                           const ckf_seeds* s, const ckf_config* cfg, const int32_t* n_tracks, int32_t cap_tracks,
                           int64_t cap_meas, const int32_t* offsets, const int32_t* meas,
                           const int32_t* meas_surface, const int32_t* seed, int32_t smoother, double* params,
                           double* cov, double* chi2, int32_t* ok, void* stream) {
  if (cap_meas < 0) return fail(CKF_ERR_INVALID_ARGUMENT, "fit_noalloc: negative capacity");
  if (ckf::fit_workspace_bytes(cap_meas) > ckf_fit_noalloc_max_bytes())
    return fail(CKF_ERR_CAPACITY, "fit_noalloc: cap_meas " + std::to_string(cap_meas) + " exceeds the scratch limit of " +
                                      std::to_string(ckf_fit_noalloc_max_meas()) + " measurements");
  void* scratch = nullptr;
  size_t bytes = 0;
  HIP_TRY(ckf::fit_scratch(&scratch, &bytes), "hipGetSymbolAddress(fit scratch)");
  return ckf_fit(g, f, m, s, cfg, n_tracks, cap_tracks, cap_meas, offsets, meas, meas_surface, seed, smoother,
                 scratch, bytes, params, cov, chi2, ok, stream);
}

size_t ckf_fit_noalloc_max_bytes(void) { return size_t(64) << 20; }

int64_t ckf_fit_noalloc_max_meas(void) {
  // the largest capacity whose workspace fits (the size grows with it)
  int64_t lo = 0, hi = (int64_t)(ckf_fit_noalloc_max_bytes() / 4);
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (ckf::fit_workspace_bytes(mid) <= ckf_fit_noalloc_max_bytes()) lo = mid; else hi = mid - 1;
  }
  return lo;
}

ckf_status ckf_cluster_workspace_size(const ckf_cells* c, size_t* bytes) {
  if (!c || !bytes || c->n_events < 0 || c->n_surfaces < 0 || c->n_cells < 0)
    return fail(CKF_ERR_INVALID_ARGUMENT, "cluster_workspace_size: bad argument");
  *bytes = ckf::cluster_workspace_bytes((long long)c->n_events * c->n_surfaces, c->n_cells);
  return CKF_OK;
}

ckf_status ckf_cluster(const ckf_geometry* g, const ckf_cells* c, const float* pitch, void* workspace,
                       size_t workspace_bytes, int32_t* meas_offsets, float* loc, float* var, float* spacepoints,
                       int32_t* cell_cluster, int32_t* status, void* stream) {
  if (!g || !c || !pitch || !meas_offsets || !status) return fail(CKF_ERR_INVALID_ARGUMENT, "cluster: NULL argument");
  if (c->n_events < 0 || c->n_cells < 0) return fail(CKF_ERR_INVALID_ARGUMENT, "cluster: negative size");
  if (c->n_surfaces != g->dev.n_surfaces) return fail(CKF_ERR_INVALID_ARGUMENT, "cluster: n_surfaces differs from geometry");
  if (c->n_cells > INT32_MAX || (long long)c->n_events * c->n_surfaces >= INT32_MAX)
    return fail(CKF_ERR_NOT_SUPPORTED, "cluster: more than 2^31 - 1 cells or rows");
  if (c->n_events > 0 && !c->offsets) return fail(CKF_ERR_INVALID_ARGUMENT, "cluster: NULL offsets");
  if (c->n_cells > 0 && (!c->c0 || !c->c1 || !c->q || !loc || !var))
    return fail(CKF_ERR_INVALID_ARGUMENT, "cluster: NULL cell or output array");
  if (!workspace || workspace_bytes < ckf::cluster_workspace_bytes((long long)c->n_events * c->n_surfaces, c->n_cells))
    return fail(CKF_ERR_CAPACITY, "cluster: workspace too small");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const ckf::CellsIn ci{c->n_events, c->n_surfaces, c->n_cells, c->offsets, c->c0, c->c1, c->q};
  HIP_TRY(ckf::launch_cluster(ci, g->dev, pitch, workspace, meas_offsets, loc, var, spacepoints, cell_cluster, status,
                              hs),
          "launch the clustering");
  return CKF_OK;
}

ckf_status ckf_seed_workspace_size(int32_t n_events, int32_t n_surfaces, int64_t n_sp, int32_t n_layers,
                                   size_t* bytes) {
  if (!bytes || n_events < 0 || n_surfaces < 0 || n_sp < 0 || n_layers < 3 || n_layers > 8)
    return fail(CKF_ERR_INVALID_ARGUMENT, "seed_workspace_size: bad argument");
  *bytes = ckf::seed_workspace_bytes((long long)n_events * n_surfaces, n_sp, n_events, n_layers);
  return CKF_OK;
}

ckf_status ckf_seed_set_top_cap(int32_t cap, int32_t* cap_max) {
  const int mx = ckf::seed_top_cap_max();
  if (cap_max) *cap_max = mx;
  if (cap < 0 || cap > mx) return fail(CKF_ERR_INVALID_ARGUMENT, "seed_set_top_cap: cap outside [0, max]");
  ckf::seed_set_top_cap(cap);
  return CKF_OK;
}

ckf_status ckf_seed(const ckf_geometry* g, int32_t n_events, const int32_t* meas_offsets, int64_t n_sp,
                    const float* spacepoints, const float* loc, const int32_t* layers, int32_t n_layers, double bz,
                    void* workspace, size_t workspace_bytes, int64_t cap_seeds, int32_t* n_seeds,
                    int32_t* seed_event, int32_t* seed_surface, double* seed_params, double* seed_cov,
                    int32_t* seed_spacepoints, int64_t* counters, void* stream) {
  if (!g || !layers || !n_seeds || n_events < 0 || n_sp < 0 || cap_seeds < 0)
    return fail(CKF_ERR_INVALID_ARGUMENT, "seed: bad argument");
  if (n_layers < 3 || n_layers > 8) return fail(CKF_ERR_INVALID_ARGUMENT, "seed: 3 to 8 seeding layers");
  if (!(std::isfinite(bz) && bz != 0.0)) return fail(CKF_ERR_INVALID_ARGUMENT, "seed: bz must be finite and non-zero");
  if (n_sp > INT32_MAX || (long long)n_events * g->dev.n_surfaces >= INT32_MAX ||
      ckf::seed_bin_count(n_events, n_layers) >= INT32_MAX)
    return fail(CKF_ERR_NOT_SUPPORTED, "seed: too many spacepoints or rows");
  if (n_events > 0 && !meas_offsets) return fail(CKF_ERR_INVALID_ARGUMENT, "seed: NULL offsets");
  if (n_sp > 0 && (!spacepoints || !loc)) return fail(CKF_ERR_INVALID_ARGUMENT, "seed: NULL spacepoints");
  if (cap_seeds > 0 && (!seed_event || !seed_surface || !seed_params || !seed_cov))
    return fail(CKF_ERR_INVALID_ARGUMENT, "seed: NULL output");
  for (int q = 0; q < n_layers; ++q)
    if (layers[q] < 0 || layers[q] >= g->dev.n_layers) return fail(CKF_ERR_INVALID_ARGUMENT, "seed: bad layer id");
  if (!workspace || workspace_bytes < ckf::seed_workspace_bytes((long long)n_events * g->dev.n_surfaces, n_sp,
                                                                n_events, n_layers))
    return fail(CKF_ERR_CAPACITY, "seed: workspace too small");
  HIP_TRY(ckf::launch_seed(g->dev, n_events, g->dev.n_surfaces, meas_offsets, n_sp, spacepoints, loc, layers,
                           n_layers, bz, workspace, cap_seeds, n_seeds, seed_event, seed_surface, seed_params,
                           seed_cov, seed_spacepoints, reinterpret_cast<long long*>(counters),
                           static_cast<hipStream_t>(stream)),
          "launch the seeding");
  return CKF_OK;
}

ckf_status ckf_resolve_workspace_size(int32_t cap_tracks, int64_t n_meas, size_t* bytes) {
  if (cap_tracks < 0 || n_meas < 0 || !bytes) return fail(CKF_ERR_INVALID_ARGUMENT, "resolve_workspace_size: bad argument");
  *bytes = ckf::resolve_workspace_bytes(cap_tracks, n_meas);
  return CKF_OK;
}

ckf_status ckf_resolve(const int32_t* n_tracks, int32_t cap_tracks, int64_t cap_meas, const int32_t* offsets,
                       const int32_t* meas, int64_t n_meas, const double* chi2, const int32_t* ndf,
                       int32_t max_shared, int32_t max_rounds, void* workspace, size_t workspace_bytes, int32_t* keep,
                       int32_t* info, void* stream) {
  if (cap_tracks < 0 || cap_meas < 0 || n_meas < 0 || max_shared < 0)
    return fail(CKF_ERR_INVALID_ARGUMENT, "resolve: negative size or max_shared");
  if (max_rounds < 1 || max_rounds > 1024) return fail(CKF_ERR_INVALID_ARGUMENT, "resolve: max_rounds must be 1..1024");
  if (n_meas > INT32_MAX) return fail(CKF_ERR_NOT_SUPPORTED, "resolve: more than 2^31 - 1 measurements");
  if (cap_tracks > 0 && (!n_tracks || !offsets || !chi2 || !ndf || !keep || (cap_meas > 0 && !meas)))
    return fail(CKF_ERR_INVALID_ARGUMENT, "resolve: NULL array");
  if (!workspace || workspace_bytes < ckf::resolve_workspace_bytes(cap_tracks, n_meas))
    return fail(CKF_ERR_CAPACITY, "resolve: workspace too small");
  HIP_TRY(ckf::run_resolve(n_tracks, cap_tracks, cap_meas, offsets, meas, n_meas, chi2, ndf, max_shared, max_rounds,
                           workspace, keep, info, static_cast<hipStream_t>(stream)),
          "ambiguity resolution");
  return CKF_OK;
}

ckf_status ckf_capture_workspace_size(int32_t cap_tracks, size_t* bytes) {
  if (cap_tracks < 0 || !bytes) return fail(CKF_ERR_INVALID_ARGUMENT, "capture_workspace_size: bad argument");
  *bytes = ckf::capture_workspace_bytes(cap_tracks);
  return CKF_OK;
}

ckf_status ckf_capture_pairs(const ckf_geometry* g, const ckf_field* field, const int32_t* n_tracks,
                             int32_t cap_tracks, const int32_t* offsets, const int32_t* meas_surface,
                             const double* meas_params, int64_t cap_pairs, float* x, int32_t* label,
                             int32_t* track, int64_t* counts, void* workspace, size_t workspace_bytes,
                             void* stream) {
  if (!g || !field || !n_tracks || !offsets || !meas_surface || !meas_params || !counts || cap_tracks < 0 ||
      cap_pairs < 0 || (cap_pairs > 0 && (!x || !label)) || !workspace)
    return fail(CKF_ERR_INVALID_ARGUMENT, "capture_pairs: bad argument");
  if (workspace_bytes < ckf::capture_workspace_bytes(cap_tracks))
    return fail(CKF_ERR_CAPACITY, "capture_pairs: workspace too small");
  if (field->dev.map) return fail(CKF_ERR_NOT_SUPPORTED, "capture_pairs: uniform field only");
  HIP_TRY(ckf::launch_capture_pairs(g->dev, field->dev, n_tracks, cap_tracks, offsets, meas_surface, meas_params,
                                    cap_pairs, x, label, track, reinterpret_cast<long long*>(counts), workspace,
                                    static_cast<hipStream_t>(stream)),
          "launch the pair capture");
  return CKF_OK;
}

}  // extern "C"
