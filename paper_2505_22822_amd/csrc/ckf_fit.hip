// Kalman-filter fit of found tracks with a smoother (paper section 2: after
// track finding a Kalman-filter fit with the Rauch-Tung-Striebel smoother
// gives every measurement the information of the whole track; section 4:
// the optimal two-filter smoother as the stable alternative).
//
// One lane per track.  The forward filter starts from the track's seed and
// visits the surfaces of its measurements in order: an FP32 RKN4 leg with
// its tangent-column Jacobian (the search's stepper), FP64 covariance
// transport, FP64 gain-form update with the Joseph covariance, then the
// module's Highland scattering added at the updated state.  The smoother
// runs backwards over one workspace record per measurement, which holds what
// it reads: the predicted and filtered states, the filtered covariance and
// the leg's Jacobian (the predicted covariance is rebuilt from the record
// before it with the forward pass's own scattering and transport functions):
//   RTS:        A_k = C_k|k F^T C_k+1|k^-1 (a Cholesky solve, no inverse),
//               x_k|n = x_k|k + A_k (x_k+1|n - x_k+1|k),
//               C_k|n = C_k|k + A_k (C_k+1|n - C_k+1|k) A_k^T;
//   two-filter: Fraser and Potter's optimal smoother.  An independent
//               backward filter in information form (Y, y), started from
//               the last measurement's information alone, runs over the
//               model the forward pass linearised, in deviations from the
//               forward filtered states: d_k+1 = a + F (d_k + w_k), with
//               a = x_k+1|k - x_k+1|k+1 and w_k the scattering of module k.
//               A step back is Y <- F^T Y F, y <- F^T (y - Y a), then
//               (I + Y Q_k)^-1 on both (Q_k touches phi and theta only, so
//               a 2x2 solve); the smoothed state is the weighted mean
//               C = (C_f^-1 + Y)^-1, x = x_f + C y (two Cholesky
//               factorisations); each measurement then adds H^T V^-1 H
//               and H^T V^-1 (m - H x_f).
#include <mutex>

#include "ckf_device.hpp"
#include "ckf_kernels.hpp"

namespace ckf {

struct alignas(16) Rec {
  double pp[5];          // predicted state at the measurement
  double fp[5], fC[15];  // filtered
  float F[25];           // the leg into the measurement (row-major)
  float pad[1];
};
static_assert(sizeof(Rec) == 304, "fit record layout");

// Tracks are fitted in waves of 64 lanes, longest tracks first: a counting
// sort by measurement count (1 .. kFitMaxLen) deals them to waves, so that
// the lanes of a wave have (nearly) the same number of steps.  Wave w's
// records are maxlen_w blocks of 64 records: step j of lane l is record l of
// the wave's block j, kept by field (word k of lane l at word 64 k + l, the
// Jacobian's floats likewise after the 25 doubles), so the lanes' stores and
// loads of one field are contiguous.  With the tracks in descending order,
// 64 maxlen_w <= the measurements of wave w-1, so all waves need at most
// cap_meas / 64 + kFitMaxLen blocks.  Empty tracks are settled in the sort
// pass; a track of more than kFitMaxLen measurements is not fitted.
constexpr int kFitBlock = 64;
constexpr int kFitMaxLen = 64;  // the finder's step bound (kMaxSteps)
static_assert(kFitMaxLen == kMaxSteps, "fit length bound");

long long fit_blocks(long long cap_meas) { return cap_meas / kFitBlock + kFitMaxLen + 1; }
static size_t fit_al256(size_t b) { return (b + 255) & ~(size_t)255; }

// the workspace: record blocks, the sorted track order, the sort's counters
struct FitSort {
  int cnt[kFitMaxLen + 1];    // tracks per length
  int start[kFitMaxLen + 1];  // first sorted position of each length (longest first)
  int fill[kFitMaxLen + 1];
  unsigned long long total;   // measurements of the sorted tracks
  int n_sorted;               // tracks in the sorted order
  int bad;                    // the tracks' ranges overlap: nothing is fitted
};

size_t fit_workspace_bytes(long long cap_meas) {
  const long long cm = cap_meas > 0 ? cap_meas : 1;
  return fit_al256((size_t)fit_blocks(cap_meas) * kFitBlock * sizeof(Rec)) + fit_al256((size_t)cm * 4) +
         fit_al256(sizeof(FitSort));
}

// S is the stride between consecutive fields of a record (compile time, so
// that the field offsets are immediates).
template <int S>
struct RecAt {
  char* d;  // double field 0 of this record
  char* f;  // Jacobian element 0
  __device__ double& D(int k) const { return *reinterpret_cast<double*>(d + 8 * k * S); }
  __device__ float& F(int i) const { return *reinterpret_cast<float*>(f + 4 * i * S); }
};

struct WaveLayout {
  char* ws;
  long long base;  // the wave's first block
  int lane;
  // the record of this lane's j-th measurement
  __device__ RecAt<kFitBlock> blk(long long j) const {
    char* b = ws + (base + j) * (long long)(kFitBlock * sizeof(Rec));
    return RecAt<kFitBlock>{b + 8 * lane, b + 200 * kFitBlock + 4 * lane};
  }
};

// The fit's workspace for callers that cannot allocate: one file-scope
// device array per GPU, held until the process ends.  Every call on a GPU
// shares it (calls that overlap on one GPU race).  The length sort's
// counters are cleared by a fill kernel at the start of every call, and the
// forward pass writes each record before the smoother reads it.
constexpr size_t kFitScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kFitScratchBytes];

hipError_t fit_scratch(void** ptr, size_t* bytes) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    // the device address of this GPU's copy (the array's name is a host
    // stand-in, not a device address)
    e = hipGetSymbolAddress(&addr[dev], HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      addr[dev] = nullptr;
      return e;
    }
  }
  *ptr = addr[dev];
  *bytes = kFitScratchBytes;
  return hipSuccess;
}

namespace {

__device__ __forceinline__ void unpack5(const double* c, double M[5][5]) {
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = i; j < 5; ++j) M[i][j] = M[j][i] = c[pk(i, j)];
}

// Cholesky factor of a 5x5 SPD matrix (lower, in place of its lower part);
// false if not positive definite.
__device__ __forceinline__ bool chol5(double M[5][5]) {
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    double d = M[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= M[j][k] * M[j][k];
    if (!(d > 0.0)) return false;
    const double l = sqrt(d), il = 1.0 / l;
    M[j][j] = l;
#pragma unroll
    for (int i = j + 1; i < 5; ++i) {
      double s = M[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) s -= M[i][k] * M[j][k];
      M[i][j] = s * il;
    }
  }
  return true;
}

// X = (L L^T)^-1 B for the factor in L's lower part (B overwritten by X).
__device__ __forceinline__ void chol5_solve(const double L[5][5], double B[5][5]) {
#pragma unroll
  for (int c = 0; c < 5; ++c) {
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      double s = B[i][c];
#pragma unroll
      for (int k = 0; k < i; ++k) s -= L[i][k] * B[k][c];
      B[i][c] = s / L[i][i];
    }
#pragma unroll
    for (int i = 4; i >= 0; --i) {
      double s = B[i][c];
#pragma unroll
      for (int k = i + 1; k < 5; ++k) s -= L[k][i] * B[k][c];
      B[i][c] = s / L[i][i];
    }
  }
}

// One leg from module src to module dst: state and covariance replaced by
// the transported ones, J the bound-to-bound Jacobian.  False if it fails.
template <bool kMap>
__device__ bool fit_leg(const GeomDev& g, const FieldDev& F, const CfgDev& cfg, int src, int dst, double* p,
                        double* C, float J[5][5]) {
  Module Am, Bm;
  load_module(g, src, Am);
  load_module(g, dst, Bm);
  LegT<kMap ? 5 : 3> L;
  V3 uA, vA;
  leg_start(Am, p, L, uA, vA);
  const V3 origin = ld3(Am.c);
  const V3 dB = ld3(Bm.c) - origin;
  float h = cfg.step_max, path = 0.f;
  LegStats st{0, 0};
  if (!land<kMap>(L, origin, dB, ld3(Bm.n), F, cfg, h, path, st)) return false;
  double pn[5];
  leg_end(L, uA, vA, Bm, dB, field_at<kMap>(F, origin + L.r), p[4], pn, J);
  bool good = true;
#pragma unroll
  for (int k = 0; k < 5; ++k) good = good && isfinite(pn[k]);
  if (!good) return false;
  transport_cov(J, C);
#pragma unroll
  for (int k = 0; k < 5; ++k) p[k] = pn[k];
  return true;
}

__device__ __forceinline__ void fail_track(long long a, long long b, double* out_p, double* out_C, int* ok, int t,
                                           int code) {
  for (long long k = a; k < b; ++k) {
#pragma unroll
    for (int i = 0; i < 5; ++i) out_p[5 * k + i] = NAN;
#pragma unroll
    for (int i = 0; i < 15; ++i) out_C[15 * k + i] = NAN;
  }
  ok[t] = code;
}

__global__ void k_fit_sort_clear(FitSort* fs) {
  const int i = threadIdx.x;
  if (i <= kFitMaxLen) fs->cnt[i] = fs->fill[i] = 0;
  if (i == 0) {
    fs->total = 0ull;
    fs->n_sorted = 0;
    fs->bad = 0;
  }
}

constexpr int kSortBlock = 256;

// One thread per track: a CSR the fit cannot trust (ok -1, outputs
// untouched), an empty track (ok 1, or -1 for a seed out of range) and a
// track longer than kFitMaxLen (ok -1, NaN outputs) are settled here; the
// others are counted per length (a workgroup's histogram in LDS, then one
// global atomic per length it holds).
__global__ void __launch_bounds__(kSortBlock) k_fit_sort_count(
    const int* __restrict__ n_tracks_p, int cap_tracks, long long cap_meas, const int* __restrict__ off,
    const int* __restrict__ seed, SeedsIn s, int n_surfaces, FitSort* fs, double* __restrict__ out_p,
    double* __restrict__ out_C, double* __restrict__ chi2_out, int* __restrict__ ok) {
  __shared__ int h[kFitMaxLen + 1];
  __shared__ unsigned long long tot;
  const int i = threadIdx.x;
  if (i <= kFitMaxLen) h[i] = 0;
  if (i == 0) tot = 0ull;
  __syncthreads();
  const int t = blockIdx.x * kSortBlock + i;
  if (t < min(*n_tracks_p, cap_tracks)) {
    const long long a = off[t], b = off[t + 1];
    if (a < 0 || b > cap_meas || b < a) {  // the CSR itself cannot be trusted: touch nothing of it
      ok[t] = -1;
      chi2_out[t] = 0.0;
    } else if (b == a) {
      const int si = seed[t];
      ok[t] = si >= 0 && si < s.n && s.surface[si] >= 0 && s.surface[si] < n_surfaces ? 1 : -1;
      chi2_out[t] = 0.0;
    } else if (b - a > kFitMaxLen) {
      chi2_out[t] = 0.0;
      fail_track(a, b, out_p, out_C, ok, t, -1);
    } else {
      atomicAdd(&h[b - a], 1);
      atomicAdd(&tot, (unsigned long long)(b - a));
    }
  }
  __syncthreads();
  if (i <= kFitMaxLen && h[i] > 0) atomicAdd(&fs->cnt[i], h[i]);
  if (i == 0 && tot > 0) atomicAdd(&fs->total, tot);
}

// One thread: each length's first position in the order (longest first).
// Tracks whose ranges overlap (more measurements than the capacity) make
// the whole call unfittable.
__global__ void k_fit_sort_offsets(long long cap_meas, FitSort* fs) {
  if (threadIdx.x != 0) return;
  int pos = 0;
  for (int l = kFitMaxLen; l >= 1; --l) {
    fs->start[l] = pos;
    pos += fs->cnt[l];
  }
  fs->bad = fs->total > (unsigned long long)cap_meas ? 1 : 0;
  fs->n_sorted = fs->bad ? 0 : pos;
}

// Each sorted track's position: its length's start, the range its
// workgroup reserved for that length (one global atomic per length), its
// rank among the workgroup's tracks of that length (LDS atomics).
__global__ void __launch_bounds__(kSortBlock) k_fit_sort_place(const int* __restrict__ n_tracks_p, int cap_tracks,
                                                             long long cap_meas, const int* __restrict__ off,
                                                             FitSort* fs, int* __restrict__ order,
                                                             double* __restrict__ chi2_out, int* __restrict__ ok) {
  __shared__ int h[kFitMaxLen + 1], base[kFitMaxLen + 1];
  const int i = threadIdx.x;
  if (i <= kFitMaxLen) h[i] = 0;
  __syncthreads();
  const int t = blockIdx.x * kSortBlock + i;
  int l = 0, r = 0;
  if (t < min(*n_tracks_p, cap_tracks)) {
    const long long a = off[t], b = off[t + 1];
    if (a >= 0 && b <= cap_meas && b > a && b - a <= kFitMaxLen) {  // (the others were settled by the count pass)
      l = (int)(b - a);
      if (fs->bad) {
        ok[t] = -1;
        chi2_out[t] = 0.0;
        l = 0;
      } else {
        r = atomicAdd(&h[l], 1);
      }
    }
  }
  __syncthreads();
  if (i >= 1 && i <= kFitMaxLen && h[i] > 0) base[i] = atomicAdd(&fs->fill[i], h[i]);
  __syncthreads();
  if (l > 0) order[fs->start[l] + base[l] + r] = t;
}

// The first block of wave w: the blocks of the waves before it, each as many
// as its first (longest) track has measurements.
__device__ __forceinline__ long long wave_base(const FitSort* fs, int w) {
  long long base = 0;
  const long long end = (long long)w * kFitBlock;  // positions before the wave
  for (int l = kFitMaxLen; l >= 1; --l) {
    const long long p0 = fs->start[l], p1 = min(p0 + fs->cnt[l], end);
    if (p1 > p0)  // waves whose first position lies in [p0, p1)
      base += (long long)l * ((p1 + kFitBlock - 1) / kFitBlock - (p0 + kFitBlock - 1) / kFitBlock);
  }
  return base;
}

template <bool kMap, bool kTwo>
__global__ void __launch_bounds__(64) k_fit(GeomDev g, FieldDev F, CfgDev cfg, MeasIn m, SeedsIn s,
                                            const int* __restrict__ off, const int* __restrict__ meas,
                                            const int* __restrict__ msurf, const int* __restrict__ seed,
                                            void* __restrict__ ws_raw, const FitSort* __restrict__ fs,
                                            const int* __restrict__ order, long long n_blocks,
                                            double* __restrict__ out_p, double* __restrict__ out_C,
                                            double* __restrict__ chi2_out, int* __restrict__ ok) {
  const int lane = threadIdx.x;
  const int w = blockIdx.x, q = w * kFitBlock + lane;  // this lane's position in the sorted order
  const int n_sorted = fs->n_sorted;
  if (w * kFitBlock >= n_sorted) return;  // (the whole wave)
  // the wave's tracks, longest first: its first track's length is its blocks
  const int t = q < n_sorted ? order[q] : -1;
  const int longest = (int)(off[order[w * kFitBlock] + 1] - off[order[w * kFitBlock]]);
  const WaveLayout lay{static_cast<char*>(ws_raw), wave_base(fs, w), lane};
  if (t < 0) return;
  const long long a = off[t], b = off[t + 1];
  if (lay.base + longest > n_blocks) {  // (cannot happen: the sort's bound)
    fail_track(a, b, out_p, out_C, ok, t, -1);
    return;
  }
  const int si = seed[t];
  bool valid = si >= 0 && si < s.n && s.surface[si] >= 0 && s.surface[si] < g.n_surfaces;
  for (long long k = a; k < b && valid; ++k)
    valid = meas[k] >= 0 && meas[k] < m.n_meas && msurf[k] >= 0 && msurf[k] < g.n_surfaces;
  chi2_out[t] = 0.0;
  if (!valid) {
    fail_track(a, b, out_p, out_C, ok, t, -1);
    return;
  }
  // ---- forward filter
  double p[5], C[15];
#pragma unroll
  for (int i = 0; i < 5; ++i) p[i] = s.params[5ll * si + i];
#pragma unroll
  for (int i = 0; i < 15; ++i) C[i] = s.cov[15ll * si + i];
  int cur = s.surface[si];
  double chi2 = 0.0;
  for (long long k = a; k < b; ++k) {
    const int dst = msurf[k];
    // the measurement is loaded before the leg, so its loads are in flight
    // while the leg is propagated
    const int id = meas[k];
    const float lm0 = m.loc[2ll * id], lm1 = m.loc[2ll * id + 1], lv0 = m.var[2ll * id], lv1 = m.var[2ll * id + 1];
    float J[5][5];
    if (dst != cur) {
      if (!fit_leg<kMap>(g, F, cfg, cur, dst, p, C, J)) {
        fail_track(a, b, out_p, out_C, ok, t, 0);
        return;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) J[i][j] = i == j ? 1.f : 0.f;
    }
    const auto put_pred = [&](auto R) {
#pragma unroll
      for (int i = 0; i < 5; ++i) R.D(i) = p[i];
#pragma unroll
      for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) R.F(5 * i + j) = J[i][j];
    };
    put_pred(lay.blk(k - a));
    const double m0 = lm0, m1 = lm1, v0 = lv0, v1 = lv1;
    chi2 += chi2_of(p, C, m0, m1, v0, v1);
    double po[5], Co[15];
    kf_update(p, C, m0, m1, v0, v1, po, Co);
#pragma unroll
    for (int i = 0; i < 5; ++i) p[i] = po[i];
#pragma unroll
    for (int i = 0; i < 15; ++i) C[i] = Co[i];
    const auto put_filt = [&](auto R) {
#pragma unroll
      for (int i = 0; i < 5; ++i) R.D(5 + i) = po[i];
#pragma unroll
      for (int i = 0; i < 15; ++i) R.D(10 + i) = Co[i];
    };
    put_filt(lay.blk(k - a));
    if (cfg.material) {
      Module M;
      load_module(g, dst, M);
      apply_ms(M, cfg.mass, p, C);
    }
    cur = dst;
  }
  chi2_out[t] = chi2;
  // ---- the last measurement: smoothed = filtered
  double xs[5], Cs[15];
  {
    const auto get = [&](auto R) {
#pragma unroll
      for (int i = 0; i < 5; ++i) xs[i] = R.D(5 + i);
#pragma unroll
      for (int i = 0; i < 15; ++i) Cs[i] = R.D(10 + i);
    };
    get(lay.blk(b - 1 - a));
#pragma unroll
    for (int i = 0; i < 5; ++i) out_p[5 * (b - 1) + i] = xs[i];
#pragma unroll
    for (int i = 0; i < 15; ++i) out_C[15 * (b - 1) + i] = Cs[i];
  }
  if constexpr (!kTwo) {
    // ---- RTS
    // one step back from k+1 to k (records Rk, Rn); false if it fails
    const auto rts_step = [&](long long k, auto Rk, auto Rn) -> bool {
      // the prediction's covariance at k+1, as the forward pass made it:
      // the scattering of module k at the filtered state, then the leg
      // (none between two measurements of one module)
      double pC[15], kp[5];
#pragma unroll
      for (int i = 0; i < 15; ++i) pC[i] = Rk.D(10 + i);
#pragma unroll
      for (int i = 0; i < 5; ++i) kp[i] = Rk.D(5 + i);
      if (cfg.material) {
        Module M;
        load_module(g, msurf[k], M);
        apply_ms(M, cfg.mass, kp, pC);
      }
      if (msurf[k + 1] != msurf[k]) {
        float Fn[5][5];
#pragma unroll
        for (int i = 0; i < 5; ++i)
#pragma unroll
          for (int j = 0; j < 5; ++j) Fn[i][j] = Rn.F(5 * i + j);
        transport_cov(Fn, pC);
      }
      double fC[5][5], G[5][5], L[5][5];
      {
        double kfC[15];
#pragma unroll
        for (int i = 0; i < 15; ++i) kfC[i] = Rk.D(10 + i);
        unpack5(kfC, fC);
      }
      // G = F fC  (so A^T = pC^-1 G)
#pragma unroll
      for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          double acc = 0.0;
#pragma unroll
          for (int l = 0; l < 5; ++l) acc = fma((double)Rn.F(5 * i + l), fC[l][j], acc);
          G[i][j] = acc;
        }
      unpack5(pC, L);
      if (!chol5(L)) {
        return false;
      }
      chol5_solve(L, G);  // G now holds X = A^T
      double d[5];
#pragma unroll
      for (int i = 0; i < 5; ++i) d[i] = xs[i] - Rn.D(i);
      d[2] = wrap_phi(d[2]);
      double xn[5];
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        double acc = Rk.D(5 + i);
#pragma unroll
        for (int j = 0; j < 5; ++j) acc = fma(G[j][i], d[j], acc);
        xn[i] = acc;
      }
      xn[2] = wrap_phi(xn[2]);
      // C_k|n = fC + X^T (Cs - pC) X
      double D[5][5], E[5][5];
#pragma unroll
      for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = i; j < 5; ++j) D[i][j] = D[j][i] = Cs[pk(i, j)] - pC[pk(i, j)];
#pragma unroll
      for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          double acc = 0.0;
#pragma unroll
          for (int l = 0; l < 5; ++l) acc = fma(D[i][l], G[l][j], acc);
          E[i][j] = acc;
        }
#pragma unroll
      for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = i; j < 5; ++j) {
          double acc = fC[i][j];
#pragma unroll
          for (int l = 0; l < 5; ++l) acc = fma(G[l][i], E[l][j], acc);
          Cs[pk(i, j)] = acc;
        }
#pragma unroll
      for (int i = 0; i < 5; ++i) xs[i] = xn[i];
#pragma unroll
      for (int i = 0; i < 5; ++i) out_p[5 * k + i] = xs[i];
#pragma unroll
      for (int i = 0; i < 15; ++i) out_C[15 * k + i] = Cs[i];
      return true;
    };
    // the lanes step back in one index j (a lane starts at its own last
    // measurement), so that a block's fields are read together
    for (long long j = longest - 2; j >= 0; --j) {
      if (j > b - a - 2) continue;
      const long long k = a + j;
      if (!rts_step(k, lay.blk(j), lay.blk(j + 1))) {
        fail_track(a, b, out_p, out_C, ok, t, 0);
        return;
      }
    }
  } else {
    // ---- two-filter: the backward information filter, combined with the
    // forward filtered state at each measurement
    double Y[5][5], y[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      y[i] = 0.0;
#pragma unroll
      for (int j = 0; j < 5; ++j) Y[i][j] = 0.0;
    }
    auto add_meas = [&](long long k, const double* xf) {
      const int id = meas[k];
      const double v0 = m.var[2ll * id], v1 = m.var[2ll * id + 1];
      Y[0][0] += 1.0 / v0;
      Y[1][1] += 1.0 / v1;
      y[0] += ((double)m.loc[2ll * id] - xf[0]) / v0;
      y[1] += ((double)m.loc[2ll * id + 1] - xf[1]) / v1;
    };
    add_meas(b - 1, xs);  // (xs: the filtered state there)
    // one step back from k+1 to k (records Rk, Rn); false if it fails
    const auto tf_step = [&](long long k, auto Rk, auto Rn) -> bool {
      double kfp[5], kfC[15];
#pragma unroll
      for (int i = 0; i < 5; ++i) kfp[i] = Rk.D(5 + i);
#pragma unroll
      for (int i = 0; i < 15; ++i) kfC[i] = Rk.D(10 + i);
      // step back through d_k+1 = a + F (d_k + w_k): Yu = F^T Y F,
      // yu = F^T (y - Y a)
      double av[5], tv[5], YF[5][5], Yu[5][5], yu[5];
#pragma unroll
      for (int i = 0; i < 5; ++i) av[i] = Rn.D(i) - Rn.D(5 + i);
      av[2] = wrap_phi(av[2]);
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        double acc = y[i];
#pragma unroll
        for (int l = 0; l < 5; ++l) acc = fma(-Y[i][l], av[l], acc);
        tv[i] = acc;
      }
#pragma unroll
      for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          double acc = 0.0;
#pragma unroll
          for (int l = 0; l < 5; ++l) acc = fma(Y[i][l], (double)Rn.F(5 * l + j), acc);
          YF[i][j] = acc;
        }
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < 5; ++l) acc = fma((double)Rn.F(5 * l + i), tv[l], acc);
        yu[i] = acc;
#pragma unroll
        for (int j = i; j < 5; ++j) {
          double s = 0.0;
#pragma unroll
          for (int l = 0; l < 5; ++l) s = fma((double)Rn.F(5 * l + i), YF[l][j], s);
          Yu[i][j] = s;
        }
      }
#pragma unroll
      for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j) Yu[i][j] = Yu[j][i];
      // the scattering of module k at its filtered state: Q = diag(0, 0,
      // q2, q3, 0); (I + Yu Q)^-1 = I - Yu[:, S] G Q-rows with
      // G = (I2 + q Yu[S, S])^-1 q, S = {phi, theta}
      if (cfg.material) {
        double qc[15], qp[5];
#pragma unroll
        for (int i = 0; i < 15; ++i) qc[i] = 0.0;
#pragma unroll
        for (int i = 0; i < 5; ++i) qp[i] = kfp[i];
        Module M;
        load_module(g, msurf[k], M);
        apply_ms(M, cfg.mass, qp, qc);
        const double q2 = qc[pk(2, 2)], q3 = qc[pk(3, 3)];
        const double a00 = 1.0 + q2 * Yu[2][2], a01 = q2 * Yu[2][3], a10 = q3 * Yu[3][2], a11 = 1.0 + q3 * Yu[3][3];
        const double idet = 1.0 / (a00 * a11 - a01 * a10);
        // G = A^-1 diag(q2, q3)
        const double g00 = a11 * idet * q2, g01 = -a01 * idet * q3, g10 = -a10 * idet * q2, g11 = a00 * idet * q3;
        const double gs = 0.5 * (g01 + g10);
        double yn[5], Yn[5][5];
        const double ys2 = g00 * yu[2] + gs * yu[3], ys3 = gs * yu[2] + g11 * yu[3];
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          yn[i] = yu[i] - (Yu[i][2] * ys2 + Yu[i][3] * ys3);
          const double r2 = g00 * Yu[2][i] + gs * Yu[3][i], r3 = gs * Yu[2][i] + g11 * Yu[3][i];
#pragma unroll
          for (int j = 0; j < 5; ++j) Yn[j][i] = Yu[j][i] - (Yu[j][2] * r2 + Yu[j][3] * r3);
        }
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          y[i] = yn[i];
#pragma unroll
          for (int j = 0; j < 5; ++j) Y[i][j] = 0.5 * (Yn[i][j] + Yn[j][i]);
        }
      } else {
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          y[i] = yu[i];
#pragma unroll
          for (int j = 0; j < 5; ++j) Y[i][j] = Yu[i][j];
        }
      }
      // weighted mean: W = C_f^-1 + Y, C = W^-1, x = x_f + C y
      double Lf[5][5], W[5][5];
      unpack5(kfC, Lf);
      if (!chol5(Lf)) {
        return false;
      }
#pragma unroll
      for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) W[i][j] = i == j ? 1.0 : 0.0;
      chol5_solve(Lf, W);  // C_f^-1
      double Ws[5][5], Cm[5][5];
#pragma unroll
      for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          Ws[i][j] = 0.5 * (W[i][j] + W[j][i]) + Y[i][j];
          Cm[i][j] = i == j ? 1.0 : 0.0;
        }
      if (!chol5(Ws)) {
        return false;
      }
      chol5_solve(Ws, Cm);  // W^-1
#pragma unroll
      for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = i; j < 5; ++j) Cs[pk(i, j)] = 0.5 * (Cm[i][j] + Cm[j][i]);
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        double acc = kfp[i];
#pragma unroll
        for (int j = 0; j < 5; ++j) acc = fma(Cs[pk(min(i, j), max(i, j))], y[j], acc);
        xs[i] = acc;
      }
      xs[2] = wrap_phi(xs[2]);
#pragma unroll
      for (int i = 0; i < 5; ++i) out_p[5 * k + i] = xs[i];
#pragma unroll
      for (int i = 0; i < 15; ++i) out_C[15 * k + i] = Cs[i];
      // the backward filter takes measurement k
      add_meas(k, kfp);
      return true;
    };
    for (long long j = longest - 2; j >= 0; --j) {  // (one index j for all lanes, as for RTS)
      if (j > b - a - 2) continue;
      const long long k = a + j;
      if (!tf_step(k, lay.blk(j), lay.blk(j + 1))) {
        fail_track(a, b, out_p, out_C, ok, t, 0);
        return;
      }
    }
  }
  ok[t] = 1;
}

}  // namespace

hipError_t launch_fit(const GeomDev& g, const FieldDev& f, const CfgDev& cfg, const MeasIn& m, const SeedsIn& s,
                      const int* n_tracks, int cap_tracks, long long cap_meas, const int* off, const int* meas,
                      const int* msurf, const int* seed, bool two_filter, void* ws, double* out_p, double* out_C,
                      double* chi2, int* ok, hipStream_t st) {
  if (cap_tracks <= 0) return hipSuccess;
  const long long n_blocks = fit_blocks(cap_meas);
  char* p = static_cast<char*>(ws);
  char* rec = p;
  p += fit_al256((size_t)n_blocks * kFitBlock * sizeof(Rec));
  int* order = reinterpret_cast<int*>(p);
  p += fit_al256((size_t)(cap_meas > 0 ? cap_meas : 1) * 4);
  FitSort* fs = reinterpret_cast<FitSort*>(p);
  const dim3 tg((cap_tracks + kSortBlock - 1) / kSortBlock), tb(kSortBlock);
  hipLaunchKernelGGL(k_fit_sort_clear, dim3(1), dim3(128), 0, st, fs);
  hipLaunchKernelGGL(k_fit_sort_count, tg, tb, 0, st, n_tracks, cap_tracks, cap_meas, off, seed, s, g.n_surfaces, fs,
                     out_p, out_C, chi2, ok);
  hipLaunchKernelGGL(k_fit_sort_offsets, dim3(1), dim3(64), 0, st, cap_meas, fs);
  hipLaunchKernelGGL(k_fit_sort_place, tg, tb, 0, st, n_tracks, cap_tracks, cap_meas, off, fs, order, chi2, ok);
  const dim3 grid((cap_tracks + 63) / 64), block(64);
  if (f.map) {
    if (two_filter)
      hipLaunchKernelGGL((k_fit<true, true>), grid, block, 0, st, g, f, cfg, m, s, off, meas, msurf, seed, rec, fs,
                         order, n_blocks, out_p, out_C, chi2, ok);
    else
      hipLaunchKernelGGL((k_fit<true, false>), grid, block, 0, st, g, f, cfg, m, s, off, meas, msurf, seed, rec, fs,
                         order, n_blocks, out_p, out_C, chi2, ok);
  } else {
    if (two_filter)
      hipLaunchKernelGGL((k_fit<false, true>), grid, block, 0, st, g, f, cfg, m, s, off, meas, msurf, seed, rec, fs,
                         order, n_blocks, out_p, out_C, chi2, ok);
    else
      hipLaunchKernelGGL((k_fit<false, false>), grid, block, 0, st, g, f, cfg, m, s, off, meas, msurf, seed, rec, fs,
                         order, n_blocks, out_p, out_C, chi2, ok);
  }
  return hipGetLastError();
}

}  // namespace ckf
