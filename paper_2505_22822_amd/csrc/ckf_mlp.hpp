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

// four bfloat16 values from two words (element 0 in the low half of u.x)
__device__ __forceinline__ bf16x4 as_bf16x4(uint2 u) { return __builtin_bit_cast(bf16x4, u); }

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// two floats -> a packed bfloat16 pair (a in the low half), round to nearest
// even: one v_cvt_pk_bf16_f32 on gfx950; the same bits as bf16_bits for
// finite inputs
__device__ __forceinline__ unsigned cvt_pk_bf16(float a, float b) {
  const f32x2_t v = {a, b};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2_t));
}

// max(x, 0) on the bit pattern: a float with the sign bit set is a negative
// int, so one integer max gives 0 for it (-0 included) and x otherwise
__device__ __forceinline__ float relu_bits(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

__device__ __forceinline__ bf16x4 pack_bf16(f32x4 v) {
  return as_bf16x4(make_uint2(cvt_pk_bf16(v.x, v.y), cvt_pk_bf16(v.z, v.w)));
}

__device__ __forceinline__ bf16x4 relu_bf16(f32x4 v) {
  return as_bf16x4(make_uint2(cvt_pk_bf16(relu_bits(v.x), relu_bits(v.y)), cvt_pk_bf16(relu_bits(v.z), relu_bits(v.w))));
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


// Logits of one pass (up to 64 rows, row r = the lane that asked for it) in
// LDS, one row of 32 per lane: the result tiles of block rb land at rows
// 16 rb + l%16, classes 16 ob + 4 (l/16) .. +3.  The row stride keeps every
// 16-byte access aligned.
constexpr int kLogitStride = 36;

__device__ __forceinline__ void logits_to_lds(const f32x4 out[2], int rb, int lane, float* lg) {
  float* row = lg + (16 * rb + (lane & 15)) * kLogitStride + 4 * (lane >> 4);
#pragma unroll
  for (int ob = 0; ob < 2; ++ob) *reinterpret_cast<f32x4*>(row + 16 * ob) = out[ob];
}

// Softmax statistics of one row of 32 logits and its three largest values
// (with multiplicity, descending): each logit is inserted into the sorted
// three by a maximum and two medians (v_med3_f32), no branches.  conf =
// summed probability of the first k (1..3) of the three.  NaN logits (only
// from non-finite parameters) give a NaN confidence, which is never taken
// as confident.
struct RowTop {
  float v[32];
  float t[3];
};

__device__ __forceinline__ float row_top3_values(const float* row, int k, RowTop& r) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const f32x4 x = *reinterpret_cast<const f32x4*>(row + 4 * q);
    r.v[4 * q + 0] = x.x;
    r.v[4 * q + 1] = x.y;
    r.v[4 * q + 2] = x.z;
    r.v[4 * q + 3] = x.w;
  }
  float v0 = -INFINITY, v1 = -INFINITY, v2 = -INFINITY;
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    const float x = r.v[i];
    v2 = __builtin_amdgcn_fmed3f(v1, v2, x);
    v1 = __builtin_amdgcn_fmed3f(v0, v1, x);
    v0 = __builtin_amdgcn_fmed3f(v0, x, INFINITY);
  }
  r.t[0] = v0;
  r.t[1] = v1;
  r.t[2] = v2;
  // the row's maximum is v0
  const float l2e = 1.44269504f, m2 = v0 * l2e;
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 32; ++i) s += __builtin_amdgcn_exp2f(fmaf(r.v[i], l2e, -m2));
  float num = 0.f;
#pragma unroll
  for (int j = 0; j < 3; ++j)
    if (j < k) num += __builtin_amdgcn_exp2f(fmaf(r.t[j], l2e, -m2));
  return num / s;
}

// The classes of the three values in (value descending, class ascending)
// order: each is the smallest index holding its value that an earlier one
// has not taken.
__device__ __forceinline__ void row_top3_classes(const RowTop& r, int c[3]) {
  int c0 = 1 << 20, c1 = 1 << 20, c2 = 1 << 20;
#pragma unroll
  for (int i = 31; i >= 0; --i) {
    c0 = r.v[i] == r.t[0] ? i : c0;
    c1 = r.v[i] == r.t[1] ? i : c1;
    c2 = r.v[i] == r.t[2] ? i : c2;
  }
  if (r.t[1] == r.t[0] || r.t[2] == r.t[1]) {  // equal values: take the next free index
    c1 = c2 = 1 << 20;
#pragma unroll
    for (int i = 31; i >= 0; --i) c1 = (r.v[i] == r.t[1] && i != c0) ? i : c1;
#pragma unroll
    for (int i = 31; i >= 0; --i) c2 = (r.v[i] == r.t[2] && i != c0 && i != c1) ? i : c2;
  }
  c[0] = c0;
  c[1] = c1;
  c[2] = c2;
}

}  // namespace ckf
