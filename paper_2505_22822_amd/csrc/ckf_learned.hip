// Learned next-module proposal: network packing, evaluation, training
// (forward and backward on the bf16 matrix cores, Adam) and the capture of
// (state, module) training pairs from found tracks.
#include "ckf_device.hpp"
#include "ckf_kernels.hpp"
#include "ckf_mlp.hpp"

namespace ckf {

namespace {

// offsets of the FP32 parameter vector: W1 [64][7], b1, W2 [64][64], b2, W3 [32][64], b3
constexpr int kW1 = 0, kB1 = 448, kW2 = 512, kB2 = 4608, kW3 = 4672, kB3 = 6720, kNP = 6752;
static_assert(kNP == CKF_MLP_PARAMS, "parameter layout");

__device__ __forceinline__ unsigned pack2(float a, float b) {
  return (unsigned)bf16_bits(a) | ((unsigned)bf16_bits(b) << 16);
}

// Repack FP32 parameters into matrix-core fragments (one workgroup).
__global__ void k_model_pack(const float* __restrict__ P, uint2* __restrict__ out) {
  uint2* w1 = out;
  uint2* w2 = w1 + kModelW1;
  uint2* w3 = w2 + kModelW2;
  float* bias = reinterpret_cast<float*>(w3 + kModelW3);
  for (int t = threadIdx.x; t < kModelW1 + kModelW2 + kModelW3; t += blockDim.x) {
    const int lane = t & 63, f = t >> 6;
    const int i = lane & 15, q4 = 4 * (lane >> 4);
    float v[4];
    if (f < 4) {  // W1 tile (ob = f), inputs padded to 16
      for (int j = 0; j < 4; ++j) {
        const int col = q4 + j;
        v[j] = col < 7 ? P[kW1 + (16 * f + i) * 7 + col] : 0.f;
      }
      w1[lane * 4 + f] = make_uint2(pack2(v[0], v[1]), pack2(v[2], v[3]));
    } else if (f < 4 + 16) {
      const int g = f - 4, ob = g >> 2, kb = g & 3;
      for (int j = 0; j < 4; ++j) v[j] = P[kW2 + (16 * ob + i) * 64 + 16 * kb + q4 + j];
      w2[(ob * 64 + lane) * 4 + kb] = make_uint2(pack2(v[0], v[1]), pack2(v[2], v[3]));
    } else {
      const int g = f - 20, ob = g >> 2, kb = g & 3;
      for (int j = 0; j < 4; ++j) v[j] = P[kW3 + (16 * ob + i) * 64 + 16 * kb + q4 + j];
      w3[(ob * 64 + lane) * 4 + kb] = make_uint2(pack2(v[0], v[1]), pack2(v[2], v[3]));
    }
  }
  for (int t = threadIdx.x; t < 160; t += blockDim.x)
    bias[t] = t < 64 ? P[kB1 + t] : (t < 128 ? P[kB2 + t - 64] : P[kB3 + t - 128]);
}

// B operand of the network input for one 16-row block: this lane's four
// features 4*(l/16)..+3 of row `row` (zero beyond the 7 inputs or rows).
__device__ __forceinline__ bf16x4 input_frag(const float* x, long long row, long long n, int lane) {
  const int q4 = 4 * (lane >> 4);
  f32x4 v;
  v.x = v.y = v.z = v.w = 0.f;
  if (row < n) {
    const float* r = x + row * 7;
    v.x = q4 + 0 < 7 ? r[q4 + 0] : 0.f;
    v.y = q4 + 1 < 7 ? r[q4 + 1] : 0.f;
    v.z = q4 + 2 < 7 ? r[q4 + 2] : 0.f;
    v.w = q4 + 3 < 7 ? r[q4 + 3] : 0.f;
  }
  return pack_bf16(v);
}

// Logits of 64 rows per workgroup (one wave).
__global__ void __launch_bounds__(64) k_mlp_forward(ModelDev M, const float* __restrict__ x, long long n,
                                                    float* __restrict__ logits) {
  const int lane = threadIdx.x;
  const long long r0 = 64ll * blockIdx.x;
  const int i = lane & 15, q4 = 4 * (lane >> 4);
#pragma unroll 1
  for (int rb = 0; rb < 4; ++rb) {
    const long long row = r0 + 16 * rb + i;
    f32x4 out[1][2];
    const bf16x4 xb[1] = {input_frag(x, row, n, lane)};
    mlp_blocks<1>(M, xb, lane, out);
    if (row < n) {
#pragma unroll
      for (int ob = 0; ob < 2; ++ob)
        *reinterpret_cast<float4*>(logits + row * 32 + 16 * ob + q4) =
            make_float4(out[0][ob].x, out[0][ob].y, out[0][ob].z, out[0][ob].w);
    }
  }
}

// ---- training: one 64-row block per workgroup, everything staged in LDS

// C tile (rows 16*mb + 4*(l/16) + j, columns 16*nb + l%16) of sum_k A[m][k] B[k][n]
// with A(m, k) = A[m*am + k*ak] and B(k, n) = B[k*bk + n*bn], bf16 in LDS.
__device__ __forceinline__ f32x4 gemm_lds(const unsigned short* A, int am, int ak, const unsigned short* B, int bk,
                                          int bn, int mb, int nb, int K, f32x4 acc, int lane) {
  const int i = lane & 15, q4 = 4 * (lane >> 4);
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a, b;
    const int m = 16 * mb + i, nn = 16 * nb + i, k = k0 + q4;
    a.x = (short)A[m * am + (k + 0) * ak];
    a.y = (short)A[m * am + (k + 1) * ak];
    a.z = (short)A[m * am + (k + 2) * ak];
    a.w = (short)A[m * am + (k + 3) * ak];
    b.x = (short)B[(k + 0) * bk + nn * bn];
    b.y = (short)B[(k + 1) * bk + nn * bn];
    b.z = (short)B[(k + 2) * bk + nn * bn];
    b.w = (short)B[(k + 3) * bk + nn * bn];
    acc = mfma16(a, b, acc);
  }
  return acc;
}

__device__ __forceinline__ float sum16(float v) {  // over the 16 lanes of a row group
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 4);
  v += __shfl_xor(v, 8);
  return v;
}

__device__ __forceinline__ f32x4 zero4() {
  f32x4 z;
  z.x = z.y = z.z = z.w = 0.f;
  return z;
}

// Forward, softmax cross-entropy and backward of one 64-row block; writes the
// block's gradient sum (already divided by the batch size) and loss sum to
// partial[block][kNP + 1].
__global__ void __launch_bounds__(64) k_mlp_grad(const float* __restrict__ P, const float* __restrict__ x,
                                                 const int* __restrict__ labels, const int* __restrict__ rows,
                                                 long long n, float* __restrict__ partial) {
  __shared__ unsigned short Wb1[64 * 16], Wb2[64 * 64], Wb3[32 * 64];
  __shared__ unsigned short Xs[64 * 16];
  __shared__ unsigned short H1[64 * 64], H2[64 * 64], D3[32 * 64], D2[64 * 64];
  __shared__ float F[32 * 64];  // logits, then dZ3 (FP32); reused for dZ1 (bf16)
  unsigned short* D1 = reinterpret_cast<unsigned short*>(F);
  const int lane = threadIdx.x;
  const int i = lane & 15, q4 = 4 * (lane >> 4);
  const long long r0 = 64ll * blockIdx.x;
  const float inv_n = 1.0f / (float)n;
  float* out = partial + (long long)blockIdx.x * (kNP + 1);

  for (int t = lane; t < 64 * 16; t += 64) {
    const int o = t >> 4, c = t & 15;
    Wb1[t] = c < 7 ? bf16_bits(P[kW1 + o * 7 + c]) : 0;
  }
  for (int t = lane; t < 64 * 64; t += 64) Wb2[t] = bf16_bits(P[kW2 + t]);
  for (int t = lane; t < 32 * 64; t += 64) Wb3[t] = bf16_bits(P[kW3 + t]);
  const long long my_row = r0 + lane;
  const bool valid = my_row < n;
  long long src = valid ? (rows ? (long long)rows[my_row] : my_row) : 0;
  for (int c = 0; c < 16; ++c) Xs[lane * 16 + c] = (valid && c < 7) ? bf16_bits(x[src * 7 + c]) : 0;
  const int label = valid ? labels[src] : 0;
  __syncthreads();

  // forward: Z1^T = W1 X^T + b1, H1 = relu; Z2^T; H2; Z3^T (logits)
  for (int mb = 0; mb < 4; ++mb)
    for (int nb = 0; nb < 4; ++nb) {
      f32x4 acc = ld_f4(P + kB1 + 16 * mb + q4);
      acc = gemm_lds(Wb1, 16, 1, Xs, 1, 16, mb, nb, 16, acc, lane);
      const float a[4] = {acc.x, acc.y, acc.z, acc.w};
      for (int j = 0; j < 4; ++j) H1[(16 * mb + q4 + j) * 64 + 16 * nb + i] = bf16_bits(fmaxf(a[j], 0.f));
    }
  __syncthreads();
  for (int mb = 0; mb < 4; ++mb)
    for (int nb = 0; nb < 4; ++nb) {
      f32x4 acc = ld_f4(P + kB2 + 16 * mb + q4);
      acc = gemm_lds(Wb2, 64, 1, H1, 64, 1, mb, nb, 64, acc, lane);
      const float a[4] = {acc.x, acc.y, acc.z, acc.w};
      for (int j = 0; j < 4; ++j) H2[(16 * mb + q4 + j) * 64 + 16 * nb + i] = bf16_bits(fmaxf(a[j], 0.f));
    }
  __syncthreads();
  for (int mb = 0; mb < 2; ++mb)
    for (int nb = 0; nb < 4; ++nb) {
      f32x4 acc = ld_f4(P + kB3 + 16 * mb + q4);
      acc = gemm_lds(Wb3, 64, 1, H2, 64, 1, mb, nb, 64, acc, lane);
      const float a[4] = {acc.x, acc.y, acc.z, acc.w};
      for (int j = 0; j < 4; ++j) F[(16 * mb + q4 + j) * 64 + 16 * nb + i] = a[j];
    }
  __syncthreads();

  // softmax cross-entropy of this lane's row; dZ3 = (p - onehot) / n
  float loss = 0.f;
  {
    float mx = -INFINITY;
    for (int c = 0; c < 32; ++c) mx = fmaxf(mx, F[c * 64 + lane]);
    float s = 0.f;
    for (int c = 0; c < 32; ++c) s += expf(F[c * 64 + lane] - mx);
    const float lse = mx + logf(s);
    if (valid) loss = lse - F[label * 64 + lane];
    for (int c = 0; c < 32; ++c) {
      const float p = expf(F[c * 64 + lane] - lse);
      const float d = valid ? (p - (c == label ? 1.f : 0.f)) * inv_n : 0.f;
      F[c * 64 + lane] = d;
      D3[c * 64 + lane] = bf16_bits(d);
    }
  }
  for (int o = 32; o >= 1; o >>= 1) loss += __shfl_xor(loss, o);
  if (lane == 0) out[kNP] = loss;
  __syncthreads();
  if (lane < 32) {  // db3 from the FP32 dZ3
    float s = 0.f;
    for (int r = 0; r < 64; ++r) s += F[lane * 64 + r];
    out[kB3 + lane] = s;
  }
  // dW3[c][f] = sum_r dZ3[c][r] H2[f][r]
  for (int mb = 0; mb < 2; ++mb)
    for (int nb = 0; nb < 4; ++nb) {
      const f32x4 acc = gemm_lds(D3, 64, 1, H2, 1, 64, mb, nb, 64, zero4(), lane);
      const float a[4] = {acc.x, acc.y, acc.z, acc.w};
      for (int j = 0; j < 4; ++j) out[kW3 + (16 * mb + q4 + j) * 64 + 16 * nb + i] = a[j];
    }
  // dZ2^T = (W3^T dZ3^T) * [H2 > 0]; db2
  for (int mb = 0; mb < 4; ++mb) {
    float db[4] = {0.f, 0.f, 0.f, 0.f};
    for (int nb = 0; nb < 4; ++nb) {
      const f32x4 acc = gemm_lds(Wb3, 1, 64, D3, 64, 1, mb, nb, 32, zero4(), lane);
      const float a[4] = {acc.x, acc.y, acc.z, acc.w};
      for (int j = 0; j < 4; ++j) {
        const int idx = (16 * mb + q4 + j) * 64 + 16 * nb + i;
        const float d = (H2[idx] & 0x7fff) != 0 ? a[j] : 0.f;
        D2[idx] = bf16_bits(d);
        db[j] += sum16(d);
      }
    }
    if (i == 0)
      for (int j = 0; j < 4; ++j) out[kB2 + 16 * mb + q4 + j] = db[j];
  }
  __syncthreads();
  // dW2[f][g] = sum_r dZ2[f][r] H1[g][r]
  for (int mb = 0; mb < 4; ++mb)
    for (int nb = 0; nb < 4; ++nb) {
      const f32x4 acc = gemm_lds(D2, 64, 1, H1, 1, 64, mb, nb, 64, zero4(), lane);
      const float a[4] = {acc.x, acc.y, acc.z, acc.w};
      for (int j = 0; j < 4; ++j) out[kW2 + (16 * mb + q4 + j) * 64 + 16 * nb + i] = a[j];
    }
  // dZ1^T = (W2^T dZ2^T) * [H1 > 0]; db1
  for (int mb = 0; mb < 4; ++mb) {
    float db[4] = {0.f, 0.f, 0.f, 0.f};
    for (int nb = 0; nb < 4; ++nb) {
      const f32x4 acc = gemm_lds(Wb2, 1, 64, D2, 64, 1, mb, nb, 64, zero4(), lane);
      const float a[4] = {acc.x, acc.y, acc.z, acc.w};
      for (int j = 0; j < 4; ++j) {
        const int idx = (16 * mb + q4 + j) * 64 + 16 * nb + i;
        const float d = (H1[idx] & 0x7fff) != 0 ? a[j] : 0.f;
        D1[idx] = bf16_bits(d);
        db[j] += sum16(d);
      }
    }
    if (i == 0)
      for (int j = 0; j < 4; ++j) out[kB1 + 16 * mb + q4 + j] = db[j];
  }
  __syncthreads();
  // dW1[g][c] = sum_r dZ1[g][r] X[r][c]  (first 7 input columns)
  for (int mb = 0; mb < 4; ++mb) {
    const f32x4 acc = gemm_lds(D1, 64, 1, Xs, 16, 1, mb, 0, 64, zero4(), lane);
    const float a[4] = {acc.x, acc.y, acc.z, acc.w};
    if (i < 7)
      for (int j = 0; j < 4; ++j) out[kW1 + (16 * mb + q4 + j) * 7 + i] = a[j];
  }
}

// grad[p] = sum over blocks in block order; loss = summed loss / n.
__global__ void k_mlp_reduce(const float* __restrict__ partial, int n_blocks, long long n, float* __restrict__ grad,
                             float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kNP) return;
  float s = 0.f;
  for (int b = 0; b < n_blocks; ++b) s += partial[(long long)b * (kNP + 1) + p];
  if (p < kNP)
    grad[p] = s;
  else
    *loss = s / (float)n;
}

__global__ void k_mlp_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ g, int step, float lr, float b1, float b2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNP) return;
  const float gi = g[p];
  const float mi = b1 * m[p] + (1.f - b1) * gi;
  const float vi = b2 * v[p] + (1.f - b2) * gi * gi;
  m[p] = mi;
  v[p] = vi;
  const float mh = mi / (1.f - powf(b1, (float)step));
  const float vh = vi / (1.f - powf(b2, (float)step));
  P[p] -= lr * mh / (sqrtf(vh) + eps);
}

// ---- training pairs from found tracks (one workgroup of 1024 threads walks
// the tracks in chunks; a block scan places each chunk's pairs in track
// order)

constexpr int kCapBlock = 256;  // threads (tracks) per capture block

// Exclusive prefix sum of v over the kCapBlock threads of a block.
__device__ __forceinline__ int block_excl_scan(int v, int* sh_w, int& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh_w[w] = x;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kCapBlock / 64; ++k) {
    if (k < w) base += sh_w[k];
    tot += sh_w[k];
  }
  __syncthreads();
  total = tot;
  return base + x - v;
}

// The pairs of found track t: counted (write false: cnt pairs, drop
// dropped) or written from position o0 on (write true).
__device__ void capture_track(const GeomDev& g, const FieldDev& F, int t, const int* __restrict__ off,
                              const int* __restrict__ msurf, const double* __restrict__ mpar, bool write, long long o0,
                              long long cap_pairs, float* __restrict__ x, int* __restrict__ label,
                              int* __restrict__ track, int& cnt, int& drop) {
  int k = 0;
  for (int i = off[t]; i < off[t + 1] - 1; ++i) {
    const int m = msurf[i], m1 = msurf[i + 1];
    if (m < 0 || m >= g.n_surfaces || m1 < 0 || m1 >= g.n_surfaces) {
      ++drop;
      continue;
    }
    const int L = g.mod[m].layer, L2 = g.mod[m1].layer;
    if (L == L2) continue;
    int slot = -1;
    for (int s = 0; s < kMaxNext; ++s)
      if (slot < 0 && g.nb_next[m * kMaxNext + s] == L2) slot = s;
    // the local helix from the state on m to L2's envelope, as the navigation finds it
    bool have = false;
    V3 X = {0.f, 0.f, 0.f}, Tx = {0.f, 0.f, 0.f};
    Window w{0, 0, 0.f, 0.f};
    const LayerRec Lr = g.layers[L2];
    const int row = slot >= 0 ? g.nb_row[m * kMaxNext + slot] : -1;
    if (row >= 0) {
      Module M;
      load_module(g, m, M);
      const double* p = mpar + 5ll * i;
      float sp, cp, st, ct;
      sincosf((float)p[2], &sp, &cp);
      sincosf((float)p[3], &st, &ct);
      const V3 P = ld3(M.c) + (float)p[0] * ld3(M.u) + (float)p[1] * ld3(M.v);
      const V3 T = {cp * st, sp * st, ct};
      const Helix H = make_helix(P, T, (float)p[4], field_at<false>(F, P));
      float sc;
      const bool hit = Lr.type == 0 ? cross_cylinder(H, Lr.pos, sc) : cross_zplane(H, Lr.pos, sc);
      if (hit) {
        helix_at_nav(H, sc, X, Tx);
        have = crossing_window(Lr, g.nb_anc[row], X, w);
      }
    }
    // one pair per measurement of the track on L2 (overlaps give several)
    for (int j = i + 1; j < off[t + 1]; ++j) {
      const int m2 = msurf[j];
      if (m2 < 0 || m2 >= g.n_surfaces || g.mod[m2].layer != L2) break;
      int lab = -1;
      if (have) {
        const int* reg = g.nb_reg + (long long)row * kRegCells;
        for (int q = 0; q < kRegCells; ++q)
          if (lab < 0 && reg[q] == m2) {
            const int wu = (q % kRegU + kRegU0) - w.iu - kWinU0, wv = (q / kRegU + kRegV0) - w.iv - kWinV0;
            lab = (wu >= 0 && wu < kWinU && wv >= 0 && wv < kWinV) ? wv * kWinU + wu : -2;
          }
      }
      if (lab < 0) {
        ++drop;
        continue;
      }
      ++cnt;
      if (!write) continue;
      const long long o = o0 + k;
      ++k;
      if (o >= cap_pairs) continue;
      float f[7];
      mlp_features(Lr, L2, g.n_layers, w, X, Tx, (float)mpar[5ll * i + 4], f);
      for (int c = 0; c < 7; ++c) x[o * 7 + c] = f[c];
      label[o] = lab;
      if (track) track[o] = t;
    }
  }
}

// Pass 1: pairs of each track (kept for pass 3) and per-block sums of
// pairs and drops.
__global__ void __launch_bounds__(kCapBlock) k_capture_count(GeomDev g, FieldDev F, const int* __restrict__ n_tracks_p,
                                                             int cap_tracks, const int* __restrict__ off,
                                                             const int* __restrict__ msurf,
                                                             const double* __restrict__ mpar,
                                                             int* __restrict__ ws_cnt,
                                                             long long* __restrict__ ws_bsum) {
  __shared__ int sh_w[kCapBlock / 64];
  const int n_t = min(*n_tracks_p, cap_tracks);
  const int t = blockIdx.x * kCapBlock + threadIdx.x;
  int cnt = 0, drop = 0;
  if (t < n_t) capture_track(g, F, t, off, msurf, mpar, false, 0, 0, nullptr, nullptr, nullptr, cnt, drop);
  if (t < cap_tracks) ws_cnt[t] = cnt;
  int tc = 0, td = 0;
  (void)block_excl_scan(cnt, sh_w, tc);
  (void)block_excl_scan(drop, sh_w, td);
  if (threadIdx.x == 0) {
    ws_bsum[2 * blockIdx.x] = tc;
    ws_bsum[2 * blockIdx.x + 1] = td;
  }
}

// Pass 2 (one block): block offsets in track order and the totals.
__global__ void __launch_bounds__(kCapBlock) k_capture_offsets(int nb, const long long* __restrict__ ws_bsum,
                                                               long long* __restrict__ ws_boff,
                                                               long long* __restrict__ counts) {
  __shared__ long long sh_c[kCapBlock], sh_d[kCapBlock];
  long long base = 0, dropped = 0;
  for (int b0 = 0; b0 < nb; b0 += kCapBlock) {
    const int b = b0 + threadIdx.x;
    sh_c[threadIdx.x] = b < nb ? ws_bsum[2 * b] : 0;
    sh_d[threadIdx.x] = b < nb ? ws_bsum[2 * b + 1] : 0;
    __syncthreads();
    if (threadIdx.x == 0) {  // serial over one chunk: a few thousand blocks at most
      for (int k = 0; k < kCapBlock && b0 + k < nb; ++k) {
        const long long c = sh_c[k];
        ws_boff[b0 + k] = base;
        base += c;
        dropped += sh_d[k];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    counts[0] = base;
    counts[1] = dropped;
  }
}

// Pass 3: each track's pairs written at its block offset plus its position
// in the block.
__global__ void __launch_bounds__(kCapBlock) k_capture_write(GeomDev g, FieldDev F, const int* __restrict__ n_tracks_p,
                                                             int cap_tracks, const int* __restrict__ off,
                                                             const int* __restrict__ msurf,
                                                             const double* __restrict__ mpar,
                                                             const int* __restrict__ ws_cnt,
                                                             const long long* __restrict__ ws_boff, long long cap_pairs,
                                                             float* __restrict__ x, int* __restrict__ label,
                                                             int* __restrict__ track) {
  __shared__ int sh_w[kCapBlock / 64];
  const int n_t = min(*n_tracks_p, cap_tracks);
  const int t = blockIdx.x * kCapBlock + threadIdx.x;
  const int cnt = t < n_t ? ws_cnt[t] : 0;
  int tot = 0;
  const int pos = block_excl_scan(cnt, sh_w, tot);
  const long long o0 = ws_boff[blockIdx.x] + pos;
  if (t < n_t && cnt > 0 && o0 < cap_pairs) {
    int c = 0, d = 0;
    capture_track(g, F, t, off, msurf, mpar, true, o0, cap_pairs, x, label, track, c, d);
  }
}

}  // namespace

hipError_t launch_model_pack(const float* params, void* out, hipStream_t st) {
  hipLaunchKernelGGL(k_model_pack, dim3(1), dim3(256), 0, st, params, reinterpret_cast<uint2*>(out));
  return hipGetLastError();
}

ModelDev model_view(const void* buf) {
  ModelDev M;
  const uint2* b = reinterpret_cast<const uint2*>(buf);
  M.w1 = b;
  M.w2 = b + kModelW1;
  M.w3 = M.w2 + kModelW2;
  const float* bias = reinterpret_cast<const float*>(M.w3 + kModelW3);
  M.b1 = bias;
  M.b2 = bias + 64;
  M.b3 = bias + 128;
  return M;
}

hipError_t launch_mlp_forward(const ModelDev& M, const float* x, long long n, float* logits, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const long long blocks = (n + 63) / 64;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(64), 0, st, M, x, n, logits);
  return hipGetLastError();
}

size_t mlp_workspace_bytes(long long n) { return (size_t)((n + 63) / 64) * (kNP + 1) * sizeof(float); }

hipError_t launch_mlp_grad(const float* params, const float* x, const int* labels, const int* rows, long long n,
                           void* ws, float* grad, float* loss, hipStream_t st) {
  const int blocks = (int)((n + 63) / 64);
  float* partial = reinterpret_cast<float*>(ws);
  hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(64), 0, st, params, x, labels, rows, n, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kNP + 1 + 255) / 256), dim3(256), 0, st, partial, blocks, n, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* params, float* m, float* v, const float* grad, int step, float lr, float b1,
                           float b2, float eps, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((kNP + 255) / 256), dim3(256), 0, st, params, m, v, grad, step, lr, b1, b2,
                     eps);
  return hipGetLastError();
}

namespace {
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

size_t capture_workspace_bytes(int cap_tracks) {
  const size_t nb = (size_t)(cap_tracks + kCapBlock - 1) / kCapBlock;
  return align256((size_t)cap_tracks * sizeof(int)) + align256(nb * 2 * sizeof(long long)) +
         align256(nb * sizeof(long long));
}

hipError_t launch_capture_pairs(const GeomDev& g, const FieldDev& f, const int* n_tracks, int cap_tracks,
                                const int* off, const int* msurf, const double* mpar, long long cap_pairs, float* x,
                                int* label, int* track, long long* counts, void* ws, hipStream_t st) {
  const int nb = (cap_tracks + kCapBlock - 1) / kCapBlock;
  char* w = static_cast<char*>(ws);
  int* ws_cnt = reinterpret_cast<int*>(w);
  long long* ws_bsum = reinterpret_cast<long long*>(w + align256((size_t)cap_tracks * sizeof(int)));
  long long* ws_boff = reinterpret_cast<long long*>(reinterpret_cast<char*>(ws_bsum) +
                                                    align256((size_t)nb * 2 * sizeof(long long)));
  if (nb > 0) {
    hipLaunchKernelGGL(k_capture_count, dim3(nb), dim3(kCapBlock), 0, st, g, f, n_tracks, cap_tracks, off, msurf, mpar,
                       ws_cnt, ws_bsum);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_capture_offsets, dim3(1), dim3(kCapBlock), 0, st, nb, ws_bsum, ws_boff, counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nb == 0) return e;
  hipLaunchKernelGGL(k_capture_write, dim3(nb), dim3(kCapBlock), 0, st, g, f, n_tracks, cap_tracks, off, msurf, mpar,
                     ws_cnt, ws_boff, cap_pairs, x, label, track);
  return hipGetLastError();
}

}  // namespace ckf
