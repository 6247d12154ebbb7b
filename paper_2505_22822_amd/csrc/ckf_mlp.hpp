// The next-module network on the gfx950 matrix cores (device code shared by
// the track-finding kernel and the training kernels).
//
// The network runs transposed, features x rows: Z^T = W . X^T + b, so that
// one 16x16x16 bf16 MFMA (v_mfma_f32_16x16x16_bf16) takes a weight tile as
// its A operand and 16 rows' activations as its B operand.  With that
// operand order the 16x16 result tile of one layer (lane l: features
// 4*(l/16)+j of row l%16) is exactly the B operand of the next layer, so a
// 16-row block goes through all three layers in registers.
#pragma once
#include "ckf_device.hpp"

namespace ckf {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ unsigned short bf16_bits(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}


__device__ __forceinline__ bf16x4 pack_bf16(f32x4 v) {
  bf16x4 r;
  r.x = (short)bf16_bits(v.x);
  r.y = (short)bf16_bits(v.y);
  r.z = (short)bf16_bits(v.z);
  r.w = (short)bf16_bits(v.w);
  return r;
}

__device__ __forceinline__ bf16x4 relu_bf16(f32x4 v) {
  v.x = fmaxf(v.x, 0.f);
  v.y = fmaxf(v.y, 0.f);
  v.z = fmaxf(v.z, 0.f);
  v.w = fmaxf(v.w, 0.f);
  return pack_bf16(v);
}

__device__ __forceinline__ bf16x4 as_bf16x4(uint2 u) {
  bf16x4 r;
  r.x = (short)(u.x & 0xffffu);
  r.y = (short)(u.x >> 16);
  r.z = (short)(u.y & 0xffffu);
  r.w = (short)(u.y >> 16);
  return r;
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 ld_f4(const float* p) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  f32x4 r;
  r.x = v.x;
  r.y = v.y;
  r.z = v.z;
  r.w = v.w;
  return r;
}

// Logits of NB 16-row blocks at once: every weight tile is fetched once and
// applied to the NB blocks, which gives NB independent MFMA chains.  The
// operands of the next output tile (two 16-byte weight loads and the bias)
// are requested before the current tile's products, so each tile waits for
// at most one memory round trip, overlapped with the previous tile's work.
// xb[rb]: this lane's B operand of the input of rows 16*rb + l%16 of those
// blocks.  Must be called by all 64 lanes together.
struct TileOps {
  uint4 w01, w23;  // fragments kb = 0, 1 and 2, 3
  f32x4 b;
};

__device__ __forceinline__ TileOps tile_ops(const uint2* w, const float* b, int ob, int lane) {
  const uint4* p = reinterpret_cast<const uint4*>(w + (ob * 64 + lane) * 4);
  TileOps t;
  t.w01 = p[0];
  t.w23 = p[1];
  t.b = ld_f4(b + 16 * ob + 4 * (lane >> 4));
  return t;
}

__device__ __forceinline__ bf16x4 frag(const TileOps& t, int kb) {
  const uint4& u = kb < 2 ? t.w01 : t.w23;
  return as_bf16x4((kb & 1) ? make_uint2(u.z, u.w) : make_uint2(u.x, u.y));
}

template <int NB>
__device__ __forceinline__ void mlp_blocks(const ModelDev& M, const bf16x4 xb[NB], int lane, f32x4 out[NB][2]) {
  const int q4 = 4 * (lane >> 4);
  bf16x4 h1[NB][4], h2[NB][4];
  // layer 1: the lane's four W1 fragments (one per output tile) and biases
  const uint4* p1 = reinterpret_cast<const uint4*>(M.w1 + lane * 4);
  const uint4 w1a = p1[0], w1b = p1[1];
  f32x4 b1[4];
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) b1[ob] = ld_f4(M.b1 + 16 * ob + q4);
  TileOps nxt = tile_ops(M.w2, M.b2, 0, lane);
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    const uint4& u = ob < 2 ? w1a : w1b;
    const bf16x4 w = as_bf16x4((ob & 1) ? make_uint2(u.z, u.w) : make_uint2(u.x, u.y));
#pragma unroll
    for (int rb = 0; rb < NB; ++rb) h1[rb][ob] = relu_bf16(mfma16(w, xb[rb], b1[ob]));
  }
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    const TileOps cur = nxt;
    nxt = ob < 3 ? tile_ops(M.w2, M.b2, ob + 1, lane) : tile_ops(M.w3, M.b3, 0, lane);
    f32x4 acc[NB];
#pragma unroll
    for (int rb = 0; rb < NB; ++rb) acc[rb] = cur.b;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const bf16x4 w = frag(cur, kb);
#pragma unroll
      for (int rb = 0; rb < NB; ++rb) acc[rb] = mfma16(w, h1[rb][kb], acc[rb]);
    }
#pragma unroll
    for (int rb = 0; rb < NB; ++rb) h2[rb][ob] = relu_bf16(acc[rb]);
  }
#pragma unroll
  for (int ob = 0; ob < 2; ++ob) {
    const TileOps cur = nxt;
    if (ob == 0) nxt = tile_ops(M.w3, M.b3, 1, lane);
#pragma unroll
    for (int rb = 0; rb < NB; ++rb) out[rb][ob] = cur.b;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const bf16x4 w = frag(cur, kb);
#pragma unroll
      for (int rb = 0; rb < NB; ++rb) out[rb][ob] = mfma16(w, h2[rb][kb], out[rb][ob]);
    }
  }
}

// Proposal window of a crossing X of layer Lr's envelope, for a neighbour
// table row with anchor (phi_A, w_A, pitch u, pitch v): the centre cell
// (iu, iv) in the layer's curvilinear coordinates - (R dphi, dz) on a
// barrel, (r dphi, dr) on a disk - and X's fractional position in it.
// Returns false for a non-finite or far-away crossing.
struct Window {
  int iu, iv;
  float fu, fv;
};

__device__ __forceinline__ bool crossing_window(const LayerRec& Lr, float4 anc, V3 X, Window& w) {
  const float r = sqrtf(X.x * X.x + X.y * X.y);
  float dphi = atan2_as(X.y, X.x) - anc.x;
  if (dphi >= 3.14159265f) dphi -= 6.28318531f;
  if (dphi < -3.14159265f) dphi += 6.28318531f;
  const float du = Lr.type == 0 ? dphi * Lr.pos : dphi * r;
  const float dv = Lr.type == 0 ? X.z - anc.y : r - anc.y;
  const float qu = fdiv_fast(du, anc.z), qv = fdiv_fast(dv, anc.w);
  if (!(fabsf(qu) < 1000.f && fabsf(qv) < 1000.f)) return false;
  const float cu = floorf(qu + 0.5f), cv = floorf(qv + 0.5f);
  w.iu = (int)cu;
  w.iv = (int)cv;
  w.fu = qu - cu;
  w.fv = qv - cv;
  return true;
}

// Network input at a crossing X (direction T) of layer `L`: the fractional
// cell position, the direction in the layer frame (phi-hat, then z-hat and
// r-hat on barrels, r-hat and z-hat on disks), q/p, L / n_layers.
__device__ __forceinline__ void mlp_features(const LayerRec& Lr, int L, int n_layers, const Window& w, V3 X, V3 T,
                                             float qop, float x[7]) {
  const float r = sqrtf(X.x * X.x + X.y * X.y);
  const float ir = r > 0.f ? 1.0f / r : 0.f;
  const float tphi = (-X.y * T.x + X.x * T.y) * ir;
  const float tr = (X.x * T.x + X.y * T.y) * ir;
  x[0] = w.fu;
  x[1] = w.fv;
  x[2] = tphi;
  x[3] = Lr.type == 0 ? T.z : tr;
  x[4] = Lr.type == 0 ? tr : T.z;
  x[5] = qop;
  x[6] = (float)L / (float)n_layers;
}

// Module id of output k (0..31) of the window, or -1 (empty cell or outside
// the stored region).
__device__ __forceinline__ int window_module(const GeomDev& g, int row, const Window& w, int k) {
  const int cu = w.iu + kWinU0 + (k % kWinU), cv = w.iv + kWinV0 + k / kWinU;
  if (cu < kRegU0 || cu >= kRegU0 + kRegU || cv < kRegV0 || cv >= kRegV0 + kRegV) return -1;
  return g.nb_reg[(long long)row * kRegCells + (cv - kRegV0) * kRegU + (cu - kRegU0)];
}

// Sorted top-3 (value descending, class ascending) of (v, c) pairs.
struct Top3 {
  float v[3];
  int c[3];
};

__device__ __forceinline__ bool top_before(float va, int ca, float vb, int cb) {
  return va > vb || (va == vb && ca < cb);
}

__device__ __forceinline__ void top_insert(Top3& t, float v, int c) {
  if (!top_before(v, c, t.v[2], t.c[2])) return;
  if (top_before(v, c, t.v[1], t.c[1])) {
    t.v[2] = t.v[1];
    t.c[2] = t.c[1];
    if (top_before(v, c, t.v[0], t.c[0])) {
      t.v[1] = t.v[0];
      t.c[1] = t.c[0];
      t.v[0] = v;
      t.c[0] = c;
    } else {
      t.v[1] = v;
      t.c[1] = c;
    }
  } else {
    t.v[2] = v;
    t.c[2] = c;
  }
}

// Softmax statistics and the top-3 classes of each row of a block: the four
// lanes holding one row (l, l^16, l^32, l^48) all end with the same result.
// conf = summed probability of the first k (1..3) of the top three.
__device__ __forceinline__ void mlp_top3(const f32x4 out[2], int lane, int k, Top3& t, float& conf) {
  const int q4 = 4 * (lane >> 4);
  float vals[8];
#pragma unroll
  for (int ob = 0; ob < 2; ++ob) {
    vals[4 * ob + 0] = out[ob].x;
    vals[4 * ob + 1] = out[ob].y;
    vals[4 * ob + 2] = out[ob].z;
    vals[4 * ob + 3] = out[ob].w;
  }
  float mx = vals[0];
#pragma unroll
  for (int i = 1; i < 8; ++i) mx = fmaxf(mx, vals[i]);
  mx = fmaxf(mx, __shfl_xor(mx, 16));
  mx = fmaxf(mx, __shfl_xor(mx, 32));
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += __expf(vals[i] - mx);
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  t.v[0] = t.v[1] = t.v[2] = -INFINITY;
  t.c[0] = t.c[1] = t.c[2] = 1 << 20;
#pragma unroll
  for (int i = 0; i < 8; ++i) top_insert(t, vals[i], 16 * (i >> 2) + q4 + (i & 3));
#pragma unroll
  for (int x = 16; x <= 32; x <<= 1) {
    float ov[3];
    int oc[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      ov[j] = __shfl_xor(t.v[j], x);
      oc[j] = __shfl_xor(t.c[j], x);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) top_insert(t, ov[j], oc[j]);
  }
  float num = 0.f;
#pragma unroll
  for (int j = 0; j < 3; ++j)
    if (j < k) num += __expf(t.v[j] - mx);
  conf = num / s;
}

}  // namespace ckf
