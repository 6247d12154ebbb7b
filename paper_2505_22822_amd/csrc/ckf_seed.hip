// Triplet seeding and helix parameter estimation (paper section 2: triplets
// of spacepoints that can approximately form a helix, and the track's
// position and momentum estimated at the first spacepoint with the helix
// model).
//
// Spacepoints are the measurements' global positions, in the measurement
// layout (rows of (event, module)).  The seeding layers are a list ordered
// outwards.  The kernels:
//   rows    - every spacepoint's row by a max-scan of row heads;
//   bin     - spacepoints of seeding layers keyed by (event, layer, phi bin,
//             z bin) and counted, each layer's radius range taken; a
//             sum-scan gives the bins' starts; a placement pass fills them
//             and copies the points in that order with their radius (order
//             inside a bin does not matter: a middle's candidates are all
//             tested and ranked by value and index);
//   triplet - one wave per spacepoint of an inner seeding layer (the
//             middle).  Candidates come from the same and the two
//             neighbouring phi bins (a bin is wider than the azimuth cut) and
//             from z windows: tops on higher layers within |cot| <= COT_MAX,
//             bottoms on lower layers within the beam-line cut at that
//             layer's radii.  The windows are bilinear in the radius and the
//             cut variable, so their corners bound them; they get a 1 mm
//             margin and only select candidates: every cut is then applied
//             as defined.  The middle's passing tops are bucketed by cot in
//             LDS, so a passing bottom visits only the buckets of its cot
//             window; the KEEP best by (d0, bottom, top) stay;
//   write   - a sum-scan of the per-middle counts places the seeds in middle
//             order; each gets its helix estimate at the bottom spacepoint.
// Every cut is computed in FP64 with the same operations in the same order
// as its definition, and the file is compiled without contraction into
// fused multiply-adds, so the decisions are the definition's to the bit.
#include "ckf_device.hpp"
#include <atomic>

#include "ckf_kernels.hpp"
#include "ckf_scan.hpp"

#pragma clang fp contract(off)

namespace ckf {

namespace {

constexpr int kSdBlock = 256;
constexpr int kNphi = 48;  // 0.1309 rad per bin, more than the azimuth cut
constexpr int kNz = 240;   // 5 mm bins over |z| < 600 mm (the edge bins take the rest)
constexpr double kZLo = -600.0, kZBin = 5.0, kZMargin = 1.0;
constexpr int kKeep = 2;
constexpr int kMaxSeedLayers = 8;
constexpr double kKappa64 = 2.99792458e-4;
constexpr double kCotMax = 3.0, kZ0Max = 200.0, kPtMin = 0.5, kD0Max = 1.0, kDcotBase = 0.01, kDcotMs = 0.007;
constexpr double kSigma[5] = {0.2, 0.6, 0.01, 0.01, 0.15};
constexpr double kTolMax = kDcotBase + kDcotMs * (1.0 + kCotMax * kCotMax);  // the largest cot tolerance
constexpr int kTriGrid = 1024;  // persistent workgroups of the triplet search: 4 per CU, a multiple of the 8 XCDs

struct SeedLayers {
  int n;
  int layer[kMaxSeedLayers];  // geometry layer id of seeding layer index i
};

__global__ void k_sd_heads(long long rows, const int* __restrict__ moff, long long n_sp, int* __restrict__ head) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int a = moff[r], b = moff[r + 1];
  if (a >= 0 && a < b && (long long)b <= n_sp) head[a] = (int)r;
}

__global__ void k_sd_fill(long long n, int* __restrict__ head, int* __restrict__ cnt, int nbins,
                          unsigned* __restrict__ rlim) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) head[i] = -1;
  if (i < nbins) cnt[i] = 0;
  if (rlim && i < kMaxSeedLayers) {
    rlim[2 * i] = 0x7f800000u;  // +inf: minimum radius of the layer's spacepoints
    rlim[2 * i + 1] = 0u;       // maximum
  }
}

__device__ __forceinline__ int z_bin(double z) {
  const double b = floor((z - kZLo) / kZBin);  // clamped before the conversion: NaN and inf map to bin 0
  return !(b >= 0.0) ? 0 : (b >= (double)kNz ? kNz - 1 : (int)b);
}

__device__ __forceinline__ int phi_bin(double x, double y) {
  const double pi = 3.14159265358979323846;
  int b = (int)floor((atan2(y, x) + pi) * (kNphi / (2.0 * pi)));
  return b < 0 ? 0 : (b >= kNphi ? kNphi - 1 : b);
}

// key of every spacepoint (-1: not on a seeding layer) and the bin counts
__global__ void __launch_bounds__(kSdBlock) k_sd_key(long long n, int n_surfaces, GeomDev g, SeedLayers sl,
                                                     const int* __restrict__ row, const float* __restrict__ xyz,
                                                     int* __restrict__ key, int* __restrict__ cnt,
                                                     unsigned* __restrict__ rlim) {
  // the layers' radius limits are reduced in the workgroup first: one global
  // atomic per layer and workgroup instead of one per spacepoint
  __shared__ unsigned s_lim[2 * kMaxSeedLayers];
  if (threadIdx.x < 2 * kMaxSeedLayers) s_lim[threadIdx.x] = (threadIdx.x & 1) ? 0u : 0x7f800000u;
  __syncthreads();
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = i < n ? row[i] : -1;
  int k = -1;
  if (r >= 0) {
    const int s = r % n_surfaces, e = r / n_surfaces;
    Module M;
    load_module(g, s, M);
    int li = -1;
    for (int q = 0; q < sl.n; ++q)
      if (sl.layer[q] == M.layer) li = q;
    if (li >= 0) {
      const double x = xyz[3 * i], y = xyz[3 * i + 1];
      k = ((e * sl.n + li) * kNphi + phi_bin(x, y)) * kNz + z_bin(xyz[3 * i + 2]);
      atomicAdd(&cnt[k], 1);
      const float r = (float)sqrt(x * x + y * y);  // radius bounds (positive floats order as their bits)
      atomicMin(&s_lim[2 * li], __float_as_uint(r));
      atomicMax(&s_lim[2 * li + 1], __float_as_uint(r));
    }
  }
  if (i < n) key[i] = k;
  __syncthreads();
  if (threadIdx.x < 2 * kMaxSeedLayers) {
    const unsigned v = s_lim[threadIdx.x];
    if (threadIdx.x & 1) {
      if (v != 0u) atomicMax(&rlim[threadIdx.x], v);
    } else if (v != 0x7f800000u) {
      atomicMin(&rlim[threadIdx.x], v);
    }
  }
}

// sorted copy of the binned spacepoints: (x, y, z, r) in float64, r as the
// doublet cuts compute it
__global__ void k_sd_place(long long n, const int* __restrict__ key, const int* __restrict__ start,
                           int* __restrict__ fill, const float* __restrict__ xyz, int* __restrict__ sorted,
                           double4* __restrict__ spt, int* __restrict__ count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  count[i] = 0;  // seeds per middle: set by the triplet search for middles only
  if (key[i] < 0) return;
  const int j = start[key[i]] + atomicAdd(&fill[key[i]], 1);
  sorted[j] = (int)i;
  const double x = xyz[3 * i], y = xyz[3 * i + 1];
  spt[j] = make_double4(x, y, (double)xyz[3 * i + 2], sqrt(x * x + y * y));
}

struct P3 {
  double x, y, z;
};

__device__ __forceinline__ P3 sp_at(const float* xyz, int i) {
  return P3{(double)xyz[3 * i], (double)xyz[3 * i + 1], (double)xyz[3 * i + 2]};
}

// doublet cuts for an inner point p and an outer point q with their radii
// rp, rq (see the oracle's definition: the same operations, in the same order)
__device__ __forceinline__ bool doublet(const P3& p, double rp, const P3& q, double rq, bool bottom, double tan_dphi,
                                        double& cot) {
  const double dr = rq - rp;
  if (!(dr > 0.0)) return false;
  cot = (q.z - p.z) / dr;
  if (!(fabs(cot) <= kCotMax)) return false;
  if (bottom && !(fabs(p.z - rp * cot) <= kZ0Max)) return false;
  const double dot = p.x * q.x + p.y * q.y;
  const double cross = p.x * q.y - p.y * q.x;
  return dot > 0.0 && fabs(cross) <= tan_dphi * dot;
}

__device__ __forceinline__ bool circle(const P3& a, const P3& b, const P3& c, double& ux, double& uy, double& R) {
  const double d = 2.0 * (a.x * (b.y - c.y) + b.x * (c.y - a.y) + c.x * (a.y - b.y));
  if (d == 0.0) return false;
  const double a2 = a.x * a.x + a.y * a.y, b2 = b.x * b.x + b.y * b.y, c2 = c.x * c.x + c.y * c.y;
  ux = (a2 * (b.y - c.y) + b2 * (c.y - a.y) + c2 * (a.y - b.y)) / d;
  uy = (a2 * (c.x - b.x) + b2 * (a.x - c.x) + c2 * (b.x - a.x)) / d;
  const double rx = a.x - ux, ry = a.y - uy;
  R = sqrt(rx * rx + ry * ry);
  return true;
}

struct Cand {
  double d0;
  int b, t;
};

__device__ __forceinline__ bool cand_less(const Cand& x, const Cand& y) {
  return x.d0 < y.d0 || (x.d0 == y.d0 && (x.b < y.b || (x.b == y.b && x.t < y.t)));
}

__device__ __forceinline__ void z_window(double a00, double a01, double a10, double a11, int& b0, int& b1) {
  const double lo = fmin(fmin(a00, a01), fmin(a10, a11)) - kZMargin;
  const double hi = fmax(fmax(a00, a01), fmax(a10, a11)) + kZMargin;
  b0 = z_bin(lo);
  b1 = z_bin(hi);
}

// One wave per middle spacepoint M (a persistent grid walks the binned
// spacepoints in sorted order, so the waves of one XCD work on neighbouring
// middles at the same time).  For M:
//   1. its tops: spacepoints of higher layers in M's and the two neighbouring
//      phi bins and in the z window of |cot| <= COT_MAX.  The lanes split
//      them; a first pass counts the ones passing the (M, T) doublet cuts per
//      cot bucket, a second pass (the same arithmetic, so the same results)
//      writes their (cot, index) into LDS in bucket order;
//   2. its bottoms, split over the lanes like the tops.  Bottoms passing the
//      (B, M) cuts enter a wave queue; each batch of 64 gives every lane one
//      bottom, which walks the tops of the buckets around cot_BM +- tol and
//      puts the (B, T) pairs within the cot cut into a second wave queue;
//      each batch of 64 pairs gets the circle and d0 cuts, one pair per lane.
//      So the expensive tests run on full waves;
//   3. each lane keeps its best KEEP by (d0, B, T); a wave reduction takes the
//      best KEEP of the middle.
// More passing tops than the LDS holds: each bottom then scans the tops of
// its z window directly (the same cuts, no buckets, no queues).
constexpr int kTriWaves = 4;          // waves per workgroup
constexpr int kTopCap = 608;          // passing tops of one middle held in LDS (at most)
constexpr int kRing = 128;            // capacity of each wave queue (a power of two >= 127)
constexpr double kCotBucket = 0.025;  // cot bucket width
constexpr int kNcot = 241;            // buckets over [-COT_MAX, COT_MAX] (cot = COT_MAX lands in the last)
constexpr int kNcotPad = 256;         // 4 per lane for the scan
constexpr double kCotMargin = 1e-9;   // widens a bucket window beyond rounding

__device__ __forceinline__ int cot_bucket(double c) {
  const double b = floor((c + kCotMax) / kCotBucket);
  return !(b >= 0.0) ? 0 : (b >= (double)kNcot ? kNcot - 1 : (int)b);
}

// LDS traffic of one wave ordered against its own later LDS accesses
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lanes_below(unsigned long long mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

__device__ __forceinline__ void keep_best(Cand (&best)[kKeep], const Cand& c) {
  if (!cand_less(c, best[kKeep - 1])) return;
  best[kKeep - 1] = c;
#pragma unroll
  for (int k = kKeep - 1; k > 0; --k)
    if (cand_less(best[k], best[k - 1])) {
      const Cand tmp = best[k];
      best[k] = best[k - 1];
      best[k - 1] = tmp;
    }
}

// triplet cuts of (B, M, T) past both doublets and the cot difference
__device__ __forceinline__ void try_triplet(const P3& B, int b, const P3& M, const double4& pt, int t, double rmin,
                                            Cand (&best)[kKeep]) {
  const P3 T{pt.x, pt.y, pt.z};
  double ux, uy, R;
  if (!circle(B, M, T, ux, uy, R)) return;  // collinear: no finite circle, the triplet fails
  if (!(R >= rmin)) return;
  const double d0 = fabs(sqrt(ux * ux + uy * uy) - R);
  if (!(d0 <= kD0Max)) return;
  keep_best(best, Cand{d0, b, t});
}

__global__ void __launch_bounds__(64 * kTriWaves) k_sd_triplets(
    long long nbins, SeedLayers sl, const int* __restrict__ key, const int* __restrict__ start,
    const int* __restrict__ cnt, const int* __restrict__ sorted, const double4* __restrict__ spt,
    const unsigned* __restrict__ rlim, double rmin, double tan_dphi, int top_cap, int* __restrict__ count,
    int2* __restrict__ best_out, unsigned long long* __restrict__ work) {
  __shared__ double s_ct[kTriWaves][kTopCap];
  __shared__ int s_j[kTriWaves][kTopCap];
  __shared__ int s_bs[kTriWaves][kNcotPad];
  __shared__ int s_bq[kTriWaves][kRing];
  __shared__ int2 s_pq[kTriWaves][kRing];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* ct_s = s_ct[w];
  int* j_s = s_j[w];
  int* bs = s_bs[w];
  int* bq = s_bq[w];
  int2* pq = s_pq[w];
  // XCD-aware numbering: workgroups are dealt round-robin to the 8 XCDs, so
  // consecutive logical waves are put on one XCD
  const int G = gridDim.x, xcd = blockIdx.x % 8, per = G / 8;
  const int lblock = (G % 8 == 0) ? xcd * per + blockIdx.x / 8 : blockIdx.x;
  const long long W = (long long)G * kTriWaves;
  const long long total = nbins > 0 ? (long long)start[nbins - 1] + cnt[nbins - 1] : 0;
  // this lane's work units: (M, T) and (B, M) doublet tests, (B, T) cot
  // comparisons, triplet (circle) tests
  unsigned n_mt = 0, n_bm = 0, n_cot = 0, n_tri = 0;
  for (long long j = (long long)lblock * kTriWaves + w; j < total; j += W) {
    const int m = sorted[j];
    const int km = key[m];
    const int bin_m = (km / kNz) % kNphi, li_m = (km / (kNz * kNphi)) % sl.n, e = km / (kNz * kNphi * sl.n);
    if (li_m == 0 || li_m == sl.n - 1) continue;
    const double4 pm = spt[j];
    const P3 M{pm.x, pm.y, pm.z};
    const double rM = pm.w;
    const auto range = [&](int layer, int dphi, int z0, int z1, int& j0, int& j1) {
      // consecutive z bins of one (event, layer, phi bin) are adjacent in the
      // sorted order: a z window is one range
      const int k0 = ((e * sl.n + layer) * kNphi + (bin_m + dphi + kNphi) % kNphi) * kNz;
      j0 = start[k0 + z0];
      j1 = start[k0 + z1] + cnt[k0 + z1];
    };
    // every top candidate of M through the (M, T) doublet cuts; place = false
    // counts the passing ones per bucket, place = true writes them in bucket
    // order (bs holds the buckets' starts then, and their ends afterwards)
    // A top of a triplet has |cot_MT| <= COT_MAX and, since the bottom's
    // doublet line meets z0 = z_M - r_M cot_BM within Z0_MAX and cot_MT is
    // within tol <= kTolMax of cot_BM, |z_M - r_M cot_MT| <= Z0_MAX + r_M
    // kTolMax: the cot window of the tops (1 mm of margin)
    const double zb = kZ0Max + kTolMax * rM + kZMargin;
    const double clo = fmax(-kCotMax, (M.z - zb) / rM), chi = fmin(kCotMax, (M.z + zb) / rM);
    const auto tops = [&](bool place) {
      int n = 0;
      for (int lt = li_m + 1; lt < sl.n; ++lt) {
        const double s0 = __uint_as_float(rlim[2 * lt]) - rM, s1 = __uint_as_float(rlim[2 * lt + 1]) - rM;
        if (!(s0 <= s1) || !(clo <= chi)) continue;
        int zt0, zt1;
        z_window(M.z + s0 * clo, M.z + s0 * chi, M.z + s1 * clo, M.z + s1 * chi, zt0, zt1);
        for (int dt = -1; dt <= 1; ++dt) {
          int j0, j1;
          range(lt, dt, zt0, zt1, j0, j1);
          for (int base = j0; base < j1; base += 64) {
            const int jt = base + lane;
            bool pass = false;
            double ct = 0.0;
            if (jt < j1) {
              const double4 pt = spt[jt];
              pass = doublet(M, rM, P3{pt.x, pt.y, pt.z}, pt.w, false, tan_dphi, ct);
              if (!place) ++n_mt;  // (the placing pass repeats the same tests)
            }
            if (pass) {
              if (!place) {
                atomicAdd(&bs[cot_bucket(ct)], 1);
              } else {
                const int pos = atomicAdd(&bs[cot_bucket(ct)], 1);
                ct_s[pos] = ct;
                j_s[pos] = jt;
              }
            }
            n += __popcll(__ballot(pass));
          }
        }
      }
      return n;
    };
    wave_sync();  // the previous middle's LDS reads are done
    // 1. tops: count per bucket, scan, place
    for (int q = lane; q < kNcotPad; q += 64) bs[q] = 0;
    wave_sync();
    const int n_top = tops(false);
    const bool in_lds = n_top <= top_cap;
    if (in_lds) {
      wave_sync();
      const int v0 = bs[4 * lane], v1 = bs[4 * lane + 1], v2 = bs[4 * lane + 2], v3 = bs[4 * lane + 3];
      const int sum = v0 + v1 + v2 + v3;
      int incl = sum;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
      }
      const int ex = incl - sum;
      bs[4 * lane] = ex;
      bs[4 * lane + 1] = ex + v0;
      bs[4 * lane + 2] = ex + v0 + v1;
      bs[4 * lane + 3] = ex + v0 + v1 + v2;
      wave_sync();
      tops(true);
      wave_sync();
    }
    Cand best[kKeep];
#pragma unroll
    for (int k = 0; k < kKeep; ++k) best[k] = Cand{INFINITY, -1, -1};
    // 2. bottoms
    int btail = 0, bhead = 0, ptail = 0, phead = 0;  // queue positions (the same in every lane)
    // up to 64 queued pairs, one per lane, through the circle and d0 cuts
    const auto run_pairs = [&]() {
      wave_sync();
      const int np = min(64, ptail - phead);
      if (lane < np) {
        ++n_tri;
        const int2 q = pq[(phead + lane) & (kRing - 1)];
        const double4 pb = spt[q.x];
        try_triplet(P3{pb.x, pb.y, pb.z}, sorted[q.x], M, spt[q.y], sorted[q.y], rmin, best);
      }
      phead += np;
      wave_sync();
    };
    // up to 64 queued bottoms, one per lane, walk their cot window
    const auto run_bottoms = [&]() {
      wave_sync();
      const int nb = min(64, btail - bhead);
      int p = 0, p1 = 0, jb = 0;
      double cb = 0.0, tol = 0.0;
      if (lane < nb) {
        jb = bq[(bhead + lane) & (kRing - 1)];
        const double4 pb = spt[jb];
        cb = (M.z - pb.z) / (rM - pb.w);  // cot of the (B, M) doublet, as its cut computed it
        tol = kDcotBase + kDcotMs * (1.0 + cb * cb);
        const int k0 = cot_bucket(cb - tol - kCotMargin), k1 = cot_bucket(cb + tol + kCotMargin);
        p = k0 > 0 ? bs[k0 - 1] : 0;
        p1 = bs[k1];
      }
      bhead += nb;
      while (__any(p < p1)) {
        bool hit = false;
        int jt = 0;
        if (p < p1) {
          ++n_cot;
          hit = fabs(cb - ct_s[p]) <= tol;
          jt = j_s[p];
          ++p;
        }
        const unsigned long long mask = __ballot(hit);
        if (hit) pq[(ptail + lanes_below(mask)) & (kRing - 1)] = make_int2(jb, jt);
        ptail += __popcll(mask);
        if (ptail - phead >= 64) run_pairs();
      }
    };
    for (int lb = 0; lb < li_m; ++lb) {
      // z_B = z0 + r_B (z_M - z0) / r_M for |z0| <= Z0_MAX, r_B in the layer's range
      const double r0 = __uint_as_float(rlim[2 * lb]), r1 = __uint_as_float(rlim[2 * lb + 1]);
      if (!(r0 <= r1)) continue;  // no spacepoints on that layer
      int zb0, zb1, zc0, zc1;
      z_window(-kZ0Max + r0 * (M.z + kZ0Max) / rM, kZ0Max + r0 * (M.z - kZ0Max) / rM,
               -kZ0Max + r1 * (M.z + kZ0Max) / rM, kZ0Max + r1 * (M.z - kZ0Max) / rM, zb0, zb1);
      // and |cot_BM| <= COT_MAX: z_B = z_M - (r_M - r_B) cot_BM
      z_window(M.z - kCotMax * (rM - r0), M.z + kCotMax * (rM - r0), M.z - kCotMax * (rM - r1),
               M.z + kCotMax * (rM - r1), zc0, zc1);
      zb0 = max(zb0, zc0);
      zb1 = min(zb1, zc1);
      if (zb0 > zb1) continue;
      for (int db = -1; db <= 1; ++db) {
        int j0, j1;
        range(lb, db, zb0, zb1, j0, j1);
        if (in_lds) {
          for (int base = j0; base < j1; base += 64) {
            const int jb = base + lane;
            bool pass = false;
            if (jb < j1) {
              const double4 pb = spt[jb];
              double cb;
              pass = doublet(P3{pb.x, pb.y, pb.z}, pb.w, M, rM, true, tan_dphi, cb);
              ++n_bm;
            }
            const unsigned long long mask = __ballot(pass);
            if (pass) bq[(btail + lanes_below(mask)) & (kRing - 1)] = jb;
            btail += __popcll(mask);
            if (btail - bhead >= 64) run_bottoms();
          }
          continue;
        }
        for (int jb = j0 + lane; jb < j1; jb += 64) {
          const double4 pb = spt[jb];
          const P3 B{pb.x, pb.y, pb.z};
          double cb;
          ++n_bm;
          if (!doublet(B, pb.w, M, rM, true, tan_dphi, cb)) continue;
          const int b = sorted[jb];
          const double tol = kDcotBase + kDcotMs * (1.0 + cb * cb);
          for (int lt = li_m + 1; lt < sl.n; ++lt) {
            // z_T = z_M + (r_T - r_M) cot_T for cot_T within tol of cot_BM
            const double s0 = __uint_as_float(rlim[2 * lt]) - rM, s1 = __uint_as_float(rlim[2 * lt + 1]) - rM;
            if (!(s0 <= s1)) continue;
            int zt0, zt1;
            z_window(M.z + s0 * (cb - tol), M.z + s0 * (cb + tol), M.z + s1 * (cb - tol), M.z + s1 * (cb + tol),
                     zt0, zt1);
            for (int dt = -1; dt <= 1; ++dt) {
              int t0, t1;
              range(lt, dt, zt0, zt1, t0, t1);
              for (int jt = t0; jt < t1; ++jt) {
                const double4 pt = spt[jt];
                double ct;
                ++n_mt;
                if (!doublet(M, rM, P3{pt.x, pt.y, pt.z}, pt.w, false, tan_dphi, ct)) continue;
                ++n_cot;
                if (!(fabs(cb - ct) <= tol)) continue;
                ++n_tri;
                try_triplet(B, b, M, pt, sorted[jt], rmin, best);
              }
            }
          }
        }
      }
    }
    if (in_lds) {
      if (btail > bhead) run_bottoms();  // the last, partial batch
      if (ptail > phead) run_pairs();    // fewer than 64 left after run_bottoms
    }
    // 3. the middle's best KEEP over the lanes: KEEP rounds of a butterfly
    //    minimum over the lanes' next unused candidate ((B, T) pairs are
    //    distinct across lanes: each bottom is visited once, and each of its
    //    tops once)
    int used = 0, c = 0;
#pragma unroll
    for (int k = 0; k < kKeep; ++k) {
      Cand head = Cand{INFINITY, -1, -1};
#pragma unroll
      for (int q = 0; q < kKeep; ++q)
        if (q == used) head = best[q];
      Cand x = head;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const Cand y{__shfl_xor(x.d0, off), __shfl_xor(x.b, off), __shfl_xor(x.t, off)};
        if (cand_less(y, x)) x = y;
      }
      if (x.b >= 0 && head.b == x.b && head.t == x.t) ++used;
      if (lane == 0) best_out[kKeep * (long long)m + k] = make_int2(x.b, x.t);
      c += x.b >= 0 ? 1 : 0;
    }
    if (lane == 0) count[m] = c;
  }
  if (work) {  // summed over the wave, then one atomic per unit
    unsigned long long u[4] = {n_mt, n_bm, n_cot, n_tri};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) u[q] += __shfl_xor(u[q], off);
      if (lane == 0 && u[q]) atomicAdd(work + q, u[q]);
    }
  }
}

__global__ void k_sd_clear(unsigned long long* work) {
  if (threadIdx.x < 4) work[threadIdx.x] = 0;
}

__global__ void k_sd_write(long long n, int n_surfaces, double bz, const int* __restrict__ row,
                           const float* __restrict__ xyz, const float* __restrict__ loc,
                           const int* __restrict__ count, const int* __restrict__ off,
                           const int2* __restrict__ best, long long cap, int* __restrict__ event,
                           int* __restrict__ surface, double* __restrict__ params, double* __restrict__ cov,
                           int* __restrict__ sp_ids) {
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n || count[m] == 0) return;
  const P3 M = sp_at(xyz, (int)m);
  for (int k = 0; k < count[m]; ++k) {
    const long long o = (long long)off[m] + k;
    if (o >= cap) return;
    const int b = best[kKeep * m + k].x, t = best[kKeep * m + k].y;
    const P3 B = sp_at(xyz, b), T = sp_at(xyz, t);
    double ux, uy, R;
    circle(B, M, T, ux, uy, R);
    const double rx = B.x - ux, ry = B.y - uy;
    double tx = -ry / R, ty = rx / R;
    if (tx * (M.x - B.x) + ty * (M.y - B.y) < 0.0) {
      tx = -tx;
      ty = -ty;
    }
    const double phi = atan2(ty, tx);
    const double cr = (M.x - B.x) * (T.y - M.y) - (M.y - B.y) * (T.x - M.x);
    const double q = ((cr < 0.0) == (bz > 0.0)) ? 1.0 : -1.0;
    const double cx = T.x - B.x, cy = T.y - B.y;
    const double chord = sqrt(cx * cx + cy * cy);
    const double s = 2.0 * R * asin(fmin(1.0, chord / (2.0 * R)));
    const double theta = atan2(s, T.z - B.z);
    const double qop = q * sin(theta) / (kKappa64 * fabs(bz) * R);
    const int rb = row[b];
    event[o] = rb / n_surfaces;
    surface[o] = rb % n_surfaces;
    double* p = params + 5 * o;
    p[0] = loc[2 * b];
    p[1] = loc[2 * b + 1];
    p[2] = phi;
    p[3] = theta;
    p[4] = qop;
    double* C = cov + 15 * o;
    for (int j = 0; j < 15; ++j) C[j] = 0.0;
    C[0] = kSigma[0] * kSigma[0];
    C[5] = kSigma[1] * kSigma[1];
    C[9] = kSigma[2] * kSigma[2];
    C[12] = kSigma[3] * kSigma[3];
    C[14] = (kSigma[4] * qop) * (kSigma[4] * qop);
    if (sp_ids) {
      sp_ids[3 * o] = b;
      sp_ids[3 * o + 1] = (int)m;
      sp_ids[3 * o + 2] = t;
    }
  }
}

size_t al256s(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

namespace {
std::atomic<int> g_top_cap{kTopCap};
}  // namespace

int seed_top_cap_max() { return kTopCap; }
long long seed_bin_count(int n_events, int n_layers) { return (long long)n_events * n_layers * kNphi * kNz; }
void seed_set_top_cap(int cap) { g_top_cap.store(cap); }

size_t seed_workspace_bytes(long long rows, long long n_sp, int n_events, int n_layers) {
  (void)rows;
  const long long n = n_sp > 0 ? n_sp : 1;
  const long long nbins = seed_bin_count(n_events, n_layers) + 1;
  const long long nb = (n > nbins ? n : nbins) / scan_detail::kScanBlock + 2;
  return 5 * al256s((size_t)n * 4) + al256s((size_t)n * 8 * kKeep) + al256s((size_t)n * 32) +
         3 * al256s((size_t)nbins * 4) + al256s((size_t)nb * 8) + 256 + 512;
}

hipError_t launch_seed(const GeomDev& g, int n_events, int n_surfaces, const int* moff, long long n_sp,
                       const float* xyz, const float* loc, const int* layers, int n_layers, double bz, void* ws,
                       long long cap, int* n_seeds, int* event, int* surface, double* params, double* cov,
                       int* sp_ids, long long* counters, hipStream_t st) {
  SeedLayers sl;
  sl.n = n_layers;
  for (int q = 0; q < kMaxSeedLayers; ++q) sl.layer[q] = q < n_layers ? layers[q] : -1;
  const long long rows = (long long)n_events * n_surfaces;
  const long long n = n_sp;
  const long long nbins = seed_bin_count(n_events, n_layers);
  char* p = static_cast<char*>(ws);
  const long long na = n > 0 ? n : 1;
  int* head = reinterpret_cast<int*>(p);
  p += al256s((size_t)na * 4);
  int* row = reinterpret_cast<int*>(p);
  p += al256s((size_t)na * 4);
  int* key = reinterpret_cast<int*>(p);
  p += al256s((size_t)na * 4);
  int* sorted = reinterpret_cast<int*>(p);
  p += al256s((size_t)na * 4);
  int* count = reinterpret_cast<int*>(p);
  p += al256s((size_t)na * 4);
  int2* best = reinterpret_cast<int2*>(p);
  p += al256s((size_t)na * 8 * kKeep);
  double4* spt = reinterpret_cast<double4*>(p);
  p += al256s((size_t)na * 32);
  int* cnt = reinterpret_cast<int*>(p);
  p += al256s((size_t)(nbins + 1) * 4);
  int* start = reinterpret_cast<int*>(p);
  p += al256s((size_t)(nbins + 1) * 4);
  int* fill = reinterpret_cast<int*>(p);
  p += al256s((size_t)(nbins + 1) * 4);
  unsigned* rlim = reinterpret_cast<unsigned*>(p);
  p += 256;
  long long* sums = reinterpret_cast<long long*>(p);
  const auto blocks = [](long long m) { return dim3((unsigned)((m + kSdBlock - 1) / kSdBlock)); };
  unsigned long long* work = reinterpret_cast<unsigned long long*>(counters);
  if (work) hipLaunchKernelGGL(k_sd_clear, dim3(1), dim3(64), 0, st, work);
  const long long nfill = n > nbins ? n : nbins;
  if (nfill > 0) {
    hipLaunchKernelGGL(k_sd_fill, blocks(nfill), dim3(kSdBlock), 0, st, n, head, cnt, (int)nbins, rlim);
    hipLaunchKernelGGL(k_sd_fill, blocks(nbins > 0 ? nbins : 1), dim3(kSdBlock), 0, st, 0ll, head, fill, (int)nbins,
                       (unsigned*)nullptr);
  }
  if (rows > 0) hipLaunchKernelGGL(k_sd_heads, blocks(rows), dim3(kSdBlock), 0, st, rows, moff, n, head);
  device_scan<OpMax, true>(head, n, row, sums, nullptr, st);
  if (n > 0)
    hipLaunchKernelGGL(k_sd_key, blocks(n), dim3(kSdBlock), 0, st, n, n_surfaces, g, sl, row, xyz, key, cnt, rlim);
  device_scan<OpSum, false>(cnt, nbins, start, sums, nullptr, st);
  if (n > 0) {
    hipLaunchKernelGGL(k_sd_place, blocks(n), dim3(kSdBlock), 0, st, n, key, start, fill, xyz, sorted, spt, count);
    const double rmin = kPtMin / (kKappa64 * fabs(bz));
    const double tan_dphi = tan(0.12);
    hipLaunchKernelGGL(k_sd_triplets, dim3(kTriGrid), dim3(64 * kTriWaves), 0, st, nbins, sl, key, start, cnt,
                       sorted, spt, rlim, rmin, tan_dphi, g_top_cap.load(), count, best, work);
  }
  device_scan<OpSum, false>(count, n, head, sums, n_seeds, st);  // head now holds the seed offsets
  if (n > 0)
    hipLaunchKernelGGL(k_sd_write, blocks(n), dim3(kSdBlock), 0, st, n, n_surfaces, bz, row, xyz, loc, count, head,
                       best, cap, event, surface, params, cov, sp_ids);
  return hipGetLastError();
}

}  // namespace ckf
