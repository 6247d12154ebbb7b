// Greedy ambiguity resolution of found tracks by shared measurements (paper
// section 4: the stage after the CKF that removes duplicate and fake
// tracks).  The greedy removes, one at a time, the "bad" track (more than
// max_shared of its measurements held by other surviving tracks) with the
// largest key: share s/n, then chi2/ndf (FP32), then the track index.
//
// On the GPU the same result comes out of parallel rounds.  Removing a
// track only lowers the share of the tracks it shares measurements with,
// so a bad track whose key beats every bad track it shares a measurement
// with is removed by the greedy too, at a point where its key is still the
// same.  Each round therefore removes every such local maximum at once:
//   shared  - shared counts of live tracks, bad flags and keys; the bad
//             tracks clear the claim slots of their shared measurements;
//   claim_a - each bad track puts its (share, chi2/ndf) key into the slots
//             of its shared measurements (64-bit atomic max);
//   claim_b - where a track's key equals the slot's, its index goes into
//             the second slot (atomic max): ties go to the larger index;
//   decide  - a bad track that holds both slots of all its shared
//             measurements is marked for removal;
//   apply   - marked tracks die and release their measurements.
// The rounds run on the device with no host synchronisation (the call can be
// captured in a graph): a fixed number of rounds is launched, and once a
// "shared" pass finds no bad track every later kernel returns at once.  The
// bad-track count alternates between two words by round parity, so that a
// round reads the previous round's count while its own is being formed.  A
// last "shared" pass after the final round tells whether any bad track is
// left.
#include "ckf_device.hpp"
#include "ckf_kernels.hpp"

namespace ckf {

namespace {

constexpr int kResBlock = 256;

struct ResWs {
  int* use;                  // [n_meas] live tracks holding the measurement
  unsigned long long* slot_a;  // [n_meas]
  int* slot_b;               // [n_meas]
  unsigned long long* key;   // [cap_tracks]
  int* state;                // [cap_tracks] 1 live, 0 removed, -1 invalid; 2 marked this round (transient)
  int* bad;                  // [cap_tracks] 1 if bad this round
  int* n_bad;                // [2] bad tracks of the rounds of even / odd index
  int* rounds;               // [1] rounds that removed tracks
};

__device__ __forceinline__ bool track_range(const int* off, int t, long long cap_meas, long long& a, long long& b) {
  a = off[t];
  b = off[t + 1];
  return a >= 0 && b <= cap_meas && a <= b;
}

__global__ void k_res_init(long long n_meas, int cap_tracks, ResWs w) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_meas) w.use[i] = 0;
  if (i < cap_tracks) {
    w.state[i] = 0;
    w.bad[i] = 0;
  }
  if (i == 0) {
    w.n_bad[0] = w.n_bad[1] = 0;
    *w.rounds = 0;
  }
}

// every live track's measurements counted; tracks with ids out of range
// are invalid and take no part
__global__ void k_res_count(const int* __restrict__ n_tracks_p, int cap_tracks, long long cap_meas,
                            const int* __restrict__ off, const int* __restrict__ meas, long long n_meas, ResWs w) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int n_t = min(*n_tracks_p, cap_tracks);
  if (t >= n_t) return;
  long long a, b;
  bool ok = track_range(off, t, cap_meas, a, b);
  for (long long k = a; ok && k < b; ++k) ok = meas[k] >= 0 && meas[k] < n_meas;
  w.state[t] = ok ? 1 : -1;
  if (!ok) return;
  for (long long k = a; k < b; ++k) atomicAdd(&w.use[meas[k]], 1);
}

__device__ __forceinline__ unsigned long long share_key(int s, int n, double chi2, int ndf) {
  // s/n as floor(s 2^31 / n): exact order for n < 46341, equal for equal fractions
  const unsigned long long r = ((unsigned long long)s << 31) / (unsigned long long)n;
  float q = (float)chi2 / (float)(ndf > 1 ? ndf : 1);
  if (!(q >= 0.f)) q = 0.f;  // NaN or negative: lowest
  if (q > 3.0e38f) q = 3.0e38f;
  return (r << 31) | (unsigned long long)(__float_as_uint(q) & 0x7fffffffu);
}

__global__ void k_res_shared(const int* __restrict__ n_tracks_p, int cap_tracks, const int* __restrict__ off,
                             const int* __restrict__ meas, const double* __restrict__ chi2,
                             const int* __restrict__ ndf, int max_shared, ResWs w, int r) {
  if (r > 0 && w.n_bad[(r - 1) & 1] == 0) return;  // converged in an earlier round
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int n_t = min(*n_tracks_p, cap_tracks);
  if (t >= n_t) return;
  w.bad[t] = 0;
  if (w.state[t] != 1) return;
  const long long a = off[t], b = off[t + 1];
  int s = 0;
  for (long long k = a; k < b; ++k) s += w.use[meas[k]] > 1 ? 1 : 0;
  if (s <= max_shared) return;
  w.bad[t] = 1;
  w.key[t] = share_key(s, (int)(b - a), chi2[t], ndf[t]);
  atomicAdd(&w.n_bad[r & 1], 1);
  for (long long k = a; k < b; ++k) {
    const int m = meas[k];
    if (w.use[m] > 1) {
      w.slot_a[m] = 0ull;
      w.slot_b[m] = -1;
    }
  }
}

__global__ void k_res_claim_a(const int* __restrict__ n_tracks_p, int cap_tracks, const int* __restrict__ off,
                              const int* __restrict__ meas, ResWs w, int r) {
  if (w.n_bad[r & 1] == 0) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int n_t = min(*n_tracks_p, cap_tracks);
  if (t >= n_t || !w.bad[t]) return;
  const unsigned long long key = w.key[t];
  for (long long k = off[t]; k < off[t + 1]; ++k) {
    const int m = meas[k];
    if (w.use[m] > 1) atomicMax(&w.slot_a[m], key);
  }
}

__global__ void k_res_claim_b(const int* __restrict__ n_tracks_p, int cap_tracks, const int* __restrict__ off,
                              const int* __restrict__ meas, ResWs w, int r) {
  if (w.n_bad[r & 1] == 0) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int n_t = min(*n_tracks_p, cap_tracks);
  if (t >= n_t || !w.bad[t]) return;
  const unsigned long long key = w.key[t];
  for (long long k = off[t]; k < off[t + 1]; ++k) {
    const int m = meas[k];
    if (w.use[m] > 1 && w.slot_a[m] == key) atomicMax(&w.slot_b[m], t);
  }
}

__global__ void k_res_decide(const int* __restrict__ n_tracks_p, int cap_tracks, const int* __restrict__ off,
                             const int* __restrict__ meas, ResWs w, int r) {
  if (w.n_bad[r & 1] == 0) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) ++*w.rounds;
  const int n_t = min(*n_tracks_p, cap_tracks);
  if (t >= n_t || !w.bad[t]) return;
  const unsigned long long key = w.key[t];
  bool top = true;
  for (long long k = off[t]; top && k < off[t + 1]; ++k) {
    const int m = meas[k];
    if (w.use[m] > 1) top = w.slot_a[m] == key && w.slot_b[m] == t;
  }
  if (top) w.state[t] = 2;
}

__global__ void k_res_apply(const int* __restrict__ n_tracks_p, int cap_tracks, const int* __restrict__ off,
                            const int* __restrict__ meas, ResWs w, int r) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) w.n_bad[(r + 1) & 1] = 0;  // the next round's count (the previous round's is no longer read)
  if (w.n_bad[r & 1] == 0) return;
  const int n_t = min(*n_tracks_p, cap_tracks);
  if (t >= n_t) return;
  if (w.state[t] != 2) return;
  w.state[t] = 0;
  for (long long k = off[t]; k < off[t + 1]; ++k) atomicSub(&w.use[meas[k]], 1);
}

__global__ void k_res_out(const int* __restrict__ n_tracks_p, int cap_tracks, ResWs w, int* __restrict__ keep,
                          int* __restrict__ info, int r_last) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0 && info) {
    info[0] = *w.rounds;
    info[1] = w.n_bad[r_last & 1] == 0 ? 1 : 0;
  }
  if (t >= cap_tracks) return;
  const int n_t = min(*n_tracks_p, cap_tracks);
  keep[t] = t < n_t ? w.state[t] : 0;
}

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

ResWs res_view(void* ws, int cap_tracks, long long n_meas) {
  char* p = static_cast<char*>(ws);
  ResWs w;
  w.use = reinterpret_cast<int*>(p);
  p += al256((size_t)n_meas * 4);
  w.slot_a = reinterpret_cast<unsigned long long*>(p);
  p += al256((size_t)n_meas * 8);
  w.slot_b = reinterpret_cast<int*>(p);
  p += al256((size_t)n_meas * 4);
  w.key = reinterpret_cast<unsigned long long*>(p);
  p += al256((size_t)cap_tracks * 8);
  w.state = reinterpret_cast<int*>(p);
  p += al256((size_t)cap_tracks * 4);
  w.bad = reinterpret_cast<int*>(p);
  p += al256((size_t)cap_tracks * 4);
  w.n_bad = reinterpret_cast<int*>(p);
  w.rounds = w.n_bad + 2;
  return w;
}

}  // namespace

size_t resolve_workspace_bytes(int cap_tracks, long long n_meas) {
  return al256((size_t)n_meas * 4) + al256((size_t)n_meas * 8) + al256((size_t)n_meas * 4) +
         al256((size_t)cap_tracks * 8) + 2 * al256((size_t)cap_tracks * 4) + 256;  // last: n_bad[2], rounds
}

hipError_t run_resolve(const int* n_tracks, int cap_tracks, long long cap_meas, const int* off, const int* meas,
                       long long n_meas, const double* chi2, const int* ndf, int max_shared, int max_rounds, void* ws,
                       int* keep, int* info, hipStream_t st) {
  const ResWs w = res_view(ws, cap_tracks, n_meas);
  const long long n_init = n_meas > cap_tracks ? n_meas : (long long)cap_tracks;
  hipLaunchKernelGGL(k_res_init, dim3((unsigned)((n_init + kResBlock) / kResBlock)), dim3(kResBlock), 0, st, n_meas,
                     cap_tracks, w);
  if (cap_tracks <= 0) {  // nothing to resolve (the track arrays may be NULL): report 0 rounds, converged
    hipLaunchKernelGGL(k_res_out, dim3(1), dim3(kResBlock), 0, st, n_tracks, 0, w, keep, info, 0);
    return hipGetLastError();
  }
  const dim3 grid((cap_tracks + kResBlock - 1) / kResBlock), block(kResBlock);
  hipLaunchKernelGGL(k_res_count, grid, block, 0, st, n_tracks, cap_tracks, cap_meas, off, meas, n_meas, w);
  for (int r = 0; r < max_rounds; ++r) {
    hipLaunchKernelGGL(k_res_shared, grid, block, 0, st, n_tracks, cap_tracks, off, meas, chi2, ndf, max_shared, w, r);
    hipLaunchKernelGGL(k_res_claim_a, grid, block, 0, st, n_tracks, cap_tracks, off, meas, w, r);
    hipLaunchKernelGGL(k_res_claim_b, grid, block, 0, st, n_tracks, cap_tracks, off, meas, w, r);
    hipLaunchKernelGGL(k_res_decide, grid, block, 0, st, n_tracks, cap_tracks, off, meas, w, r);
    hipLaunchKernelGGL(k_res_apply, grid, block, 0, st, n_tracks, cap_tracks, off, meas, w, r);
  }
  // is any bad track left after the last round?
  hipLaunchKernelGGL(k_res_shared, grid, block, 0, st, n_tracks, cap_tracks, off, meas, chi2, ndf, max_shared, w,
                     max_rounds);
  hipLaunchKernelGGL(k_res_out, grid, block, 0, st, n_tracks, cap_tracks, w, keep, info, max_rounds);
  return hipGetLastError();
}

}  // namespace ckf
