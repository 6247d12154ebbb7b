// Device functions of the CKF hot path on gfx950.
//
// Precision split: propagation legs (state, tangent columns, navigation
// geometry) run in FP32 with positions relative to the leg's start module;
// bound parameters, covariances, chi2, the Kalman gain and the Joseph update
// are FP64.  Every decision compares FP64 quantities or FP32 geometry with
// the same thresholds as the documented readings.
#pragma once
#include <math.h>

#include "ckf_internal.hpp"

namespace ckf {

constexpr float kKappa = 2.99792458e-4f;  // GeV / (T mm)

struct V3 {
  float x, y, z;
};
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ float maxabs(V3 a) { return fmaxf(fabsf(a.x), fmaxf(fabsf(a.y), fabsf(a.z))); }
__device__ __forceinline__ V3 ld3(const float* p) { return {p[0], p[1], p[2]}; }

// a / b through the hardware reciprocal (about 1 ulp, instead of the
// correctly rounded division sequence) for FP32 geometry and step control
__device__ __forceinline__ float fdiv_fast(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// atan2 from the arctangent polynomial of Abramowitz and Stegun 4.4.49
// (|error| <= 2e-8 rad on [-1, 1]) after reducing to |x| <= 1 by octant;
// about 20 instructions against several times that for the library call.
__device__ __forceinline__ float atan2_as(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float t = mx > 0.f ? fdiv_fast(mn, mx) : 0.f;
  const float t2 = t * t;
  float p = 0.0028662257f;
  p = fmaf(p, t2, -0.0161657367f);
  p = fmaf(p, t2, 0.0429096138f);
  p = fmaf(p, t2, -0.0752896400f);
  p = fmaf(p, t2, 0.1065626393f);
  p = fmaf(p, t2, -0.1420889944f);
  p = fmaf(p, t2, 0.1999355085f);
  p = fmaf(p, t2, -0.3333314528f);
  float a = fmaf(p * t2, t, t);
  if (ay > ax) a = 1.57079632679f - a;
  if (x < 0.f) a = 3.14159265359f - a;
  return copysignf(a, y);
}

// Bilinear cell of the (r, z) map at p: the two rows and the fractions;
// cr / cz tell that the coordinate was clamped (no gradient along it).
struct MapCell {
  float4 lo, hi;  // rows iz and iz+1: (B_r, B_z) at ir and ir+1
  float fr, fz, r;
  bool cr, cz;
};

__device__ __forceinline__ void map_cell(const FieldDev& F, V3 p, MapCell& c) {
  c.r = sqrtf(p.x * p.x + p.y * p.y);
  float u = (c.r - F.r0) * F.inv_dr, w = (p.z - F.z0) * F.inv_dz;
  c.cr = c.cz = false;
  if (!(u > 0.f)) {  // also NaN
    u = 0.f;
    c.cr = true;
  } else if (u >= (float)(F.nr - 1)) {
    u = (float)(F.nr - 1);
    c.cr = true;
  }
  if (!(w > 0.f)) {
    w = 0.f;
    c.cz = true;
  } else if (w >= (float)(F.nz - 1)) {
    w = (float)(F.nz - 1);
    c.cz = true;
  }
  const int ir = min((int)u, F.nr - 2), iz = min((int)w, F.nz - 2);
  c.fr = u - (float)ir;
  c.fz = w - (float)iz;
  c.lo = F.map[iz * F.nr + ir];
  c.hi = F.map[(iz + 1) * F.nr + ir];
}

template <bool kMap>
__device__ __forceinline__ V3 field_at(const FieldDev& F, V3 p) {
  if (!kMap) return {F.bx, F.by, F.bz};
  MapCell c;
  map_cell(F, p, c);
  const float a = (1.f - c.fr) * (1.f - c.fz), b = c.fr * (1.f - c.fz), d = (1.f - c.fr) * c.fz, e = c.fr * c.fz;
  const float br = a * c.lo.x + b * c.lo.z + d * c.hi.x + e * c.hi.z;
  const float bz = a * c.lo.y + b * c.lo.w + d * c.hi.y + e * c.hi.w;
  const float ir = c.r > 0.f ? 1.0f / c.r : 0.f;
  return {br * p.x * ir, br * p.y * ir, bz};
}

// The map field and its gradient G[i][j] = dB_i/dx_j (of the interpolant).
__device__ __forceinline__ V3 field_grad(const FieldDev& F, V3 p, float G[3][3]) {
  MapCell c;
  map_cell(F, p, c);
  const float a = (1.f - c.fr) * (1.f - c.fz), b = c.fr * (1.f - c.fz), d = (1.f - c.fr) * c.fz, e = c.fr * c.fz;
  const float br = a * c.lo.x + b * c.lo.z + d * c.hi.x + e * c.hi.z;
  const float bz = a * c.lo.y + b * c.lo.w + d * c.hi.y + e * c.hi.w;
  const float inv_dr = F.inv_dr, inv_dz = F.inv_dz;
  const float brr = c.cr ? 0.f : ((1.f - c.fz) * (c.lo.z - c.lo.x) + c.fz * (c.hi.z - c.hi.x)) * inv_dr;
  const float bzr = c.cr ? 0.f : ((1.f - c.fz) * (c.lo.w - c.lo.y) + c.fz * (c.hi.w - c.hi.y)) * inv_dr;
  const float brz = c.cz ? 0.f : ((1.f - c.fr) * (c.hi.x - c.lo.x) + c.fr * (c.hi.z - c.lo.z)) * inv_dz;
  const float bzz = c.cz ? 0.f : ((1.f - c.fr) * (c.hi.y - c.lo.y) + c.fr * (c.hi.w - c.lo.w)) * inv_dz;
  const float ir = c.r > 0.f ? 1.0f / c.r : 0.f;
  const float cx = p.x * ir, sy = p.y * ir;
  G[0][0] = brr * cx * cx + br * sy * sy * ir;
  G[0][1] = brr * cx * sy - br * cx * sy * ir;
  G[0][2] = brz * cx;
  G[1][0] = G[0][1];
  G[1][1] = brr * sy * sy + br * cx * cx * ir;
  G[1][2] = brz * sy;
  G[2][0] = bzr * cx;
  G[2][1] = bzr * sy;
  G[2][2] = bzz;
  return {br * cx, br * sy, bz};
}

__device__ __forceinline__ V3 mat_vec(const float G[3][3], V3 d) {
  return {G[0][0] * d.x + G[0][1] * d.y + G[0][2] * d.z, G[1][0] * d.x + G[1][1] * d.y + G[1][2] * d.z,
          G[2][0] * d.x + G[2][1] * d.y + G[2][2] * d.z};
}

__device__ __forceinline__ void load_module(const GeomDev& g, int m, Module& M) {
  const float4* s = reinterpret_cast<const float4*>(g.mod + m);
  float4 a = s[0], b = s[1], c = s[2], d = s[3];
  M.c[0] = a.x; M.c[1] = a.y; M.c[2] = a.z; M.u[0] = a.w;
  M.u[1] = b.x; M.u[2] = b.y; M.v[0] = b.z; M.v[1] = b.w;
  M.v[2] = c.x; M.n[0] = c.y; M.n[1] = c.z; M.n[2] = c.w;
  M.hw0 = d.x; M.hw1 = d.y; M.thick = d.z; M.layer = __float_as_int(d.w);
}

// Only what the scattering reads (normal, thickness): two of the four loads.
__device__ __forceinline__ void load_module_ms(const GeomDev& g, int m, Module& M) {
  const float4* s = reinterpret_cast<const float4*>(g.mod + m);
  const float4 c = s[2], d = s[3];
  M.n[0] = c.y; M.n[1] = c.z; M.n[2] = c.w;
  M.thick = d.z;
}

// ---------------------------------------------------------------------------
// Propagation leg: free state relative to `origin` (the start module centre)
// plus tangent columns d(state)/d(bound start parameters).  In a uniform
// field the loc0/loc1 columns stay (u, 0, 0) and (v, 0, 0) along the whole
// leg, so NC = 3 columns (phi, theta, q/p) are carried; in a field map the
// force depends on position and all NC = 5 are.
template <int NC>
struct LegT {
  V3 r, T;
  float lam;
  V3 dr[NC], dT[NC];
};
using Leg = LegT<3>;

// One Nystrom RKN4 step of length h for r'' = kappa*lambda*(r' x B(r))
// (field sampled at start, midpoint and end).  The stages are evaluated
// first and give the error estimate h^2 * max|k1 - k2 - k3 + k4|; only an
// accepted step then advances the state and carries the tangent columns
// through the same stages, in place.
struct Stages {
  V3 k1, k2, k3, k4, T2, T3, T4;
  V3 B2, B4;  // field at the midpoint and the end (a map)
};

template <bool kMap, int NC>
__device__ __forceinline__ float rkn4_stages(const LegT<NC>& L, float h, V3 origin, const FieldDev& F, V3 B,
                                             Stages& S) {
  const float kl = kKappa * L.lam;
  const float h2 = 0.5f * h;
  S.k1 = kl * cross(L.T, B);
  S.B2 = kMap ? field_at<true>(F, origin + L.r + h2 * L.T + (0.125f * h * h) * S.k1) : B;
  S.T2 = L.T + h2 * S.k1;
  S.k2 = kl * cross(S.T2, S.B2);
  S.T3 = L.T + h2 * S.k2;
  S.k3 = kl * cross(S.T3, S.B2);
  S.B4 = kMap ? field_at<true>(F, origin + L.r + h * L.T + (0.5f * h * h) * S.k3) : B;
  S.T4 = L.T + h * S.k3;
  S.k4 = kl * cross(S.T4, S.B4);
  return h * h * maxabs(S.k1 - S.k2 - S.k3 + S.k4);
}

template <bool kMap, int NC>
__device__ __forceinline__ void rkn4_advance(LegT<NC>& L, float h, V3 origin, const FieldDev& F, V3 B,
                                             const Stages& S) {
  const float kl = kKappa * L.lam;
  const float h2 = 0.5f * h, h6 = h * (1.0f / 6.0f), hh6 = h * h * (1.0f / 6.0f);
  if (!kMap) {
    // d(kappa*lambda*(T x B)) = kappa*lambda*(dT x B) + kappa*dlambda*(T x B)
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const V3 dT = L.dT[j];
      V3 d1 = kl * cross(dT, B);
      if (j == NC - 1) d1 = d1 + kKappa * cross(L.T, B);
      const V3 dT2 = dT + h2 * d1;
      V3 d2 = kl * cross(dT2, B);
      if (j == NC - 1) d2 = d2 + kKappa * cross(S.T2, B);
      const V3 dT3 = dT + h2 * d2;
      V3 d3 = kl * cross(dT3, B);
      if (j == NC - 1) d3 = d3 + kKappa * cross(S.T3, B);
      const V3 dT4 = dT + h * d3;
      V3 d4 = kl * cross(dT4, B);
      if (j == NC - 1) d4 = d4 + kKappa * cross(S.T4, B);
      L.dr[j] = L.dr[j] + h * dT + hh6 * (d1 + d2 + d3);
      L.dT[j] = dT + h6 * (d1 + 2.0f * (d2 + d3) + d4);
    }
  } else {
    // plus kappa*lambda*(T x (dB/dr . d(stage point))) at each stage
    float G1[3][3], G2[3][3], G4[3][3];
    (void)field_grad(F, origin + L.r, G1);
    (void)field_grad(F, origin + L.r + h2 * L.T + (0.125f * h * h) * S.k1, G2);
    (void)field_grad(F, origin + L.r + h * L.T + (0.5f * h * h) * S.k3, G4);
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const V3 dr = L.dr[j], dT = L.dT[j];
      V3 d1 = kl * (cross(dT, B) + cross(L.T, mat_vec(G1, dr)));
      if (j == NC - 1) d1 = d1 + kKappa * cross(L.T, B);
      const V3 drm = dr + h2 * dT + (0.125f * h * h) * d1;
      const V3 dT2 = dT + h2 * d1;
      V3 d2 = kl * (cross(dT2, S.B2) + cross(S.T2, mat_vec(G2, drm)));
      if (j == NC - 1) d2 = d2 + kKappa * cross(S.T2, S.B2);
      const V3 dT3 = dT + h2 * d2;
      V3 d3 = kl * (cross(dT3, S.B2) + cross(S.T3, mat_vec(G2, drm)));
      if (j == NC - 1) d3 = d3 + kKappa * cross(S.T3, S.B2);
      const V3 dre = dr + h * dT + (0.5f * h * h) * d3;
      const V3 dT4 = dT + h * d3;
      V3 d4 = kl * (cross(dT4, S.B4) + cross(S.T4, mat_vec(G4, dre)));
      if (j == NC - 1) d4 = d4 + kKappa * cross(S.T4, S.B4);
      L.dr[j] = dr + h * dT + hh6 * (d1 + d2 + d3);
      L.dT[j] = dT + h6 * (d1 + 2.0f * (d2 + d3) + d4);
    }
  }
  L.r = L.r + h * L.T + hh6 * (S.k1 + S.k2 + S.k3);
  L.T = L.T + h6 * (S.k1 + 2.0f * (S.k2 + S.k3) + S.k4);
}

// Signed path to the plane (c, n) from r + d T + d^2 k / 2 (root nearest the
// straight-line one); NaN when the direction grazes the plane.
__device__ __forceinline__ float plane_distance(V3 r, V3 T, V3 k, V3 c, V3 n) {
  const float a = 0.5f * dot(n, k), b = dot(n, T), c0 = dot(n, r - c);
  if (fabsf(b) < 1e-9f) return __int_as_float(0x7fc00000);
  const float lin = fdiv_fast(-c0, b);
  const float disc = b * b - 4.0f * a * c0;
  if (disc < 0.0f) return lin;
  const float q = -0.5f * (b + copysignf(sqrtf(disc), b));
  if (q == 0.0f) return lin;
  return fdiv_fast(c0, q);
}

// ---------------------------------------------------------------------------
// Navigation: local helix about the field at the current point.

struct Helix {
  V3 p0, T0, bhat, tperp, w;
  float tpar, om, inv_om;
};

__device__ __forceinline__ Helix make_helix(V3 p, V3 T, float lam, V3 B) {
  Helix H;
  const float bm = sqrtf(dot(B, B));
  H.bhat = bm > 0.f ? (1.0f / bm) * B : V3{0.f, 0.f, 1.f};
  H.om = kKappa * lam * bm;
  H.inv_om = H.om != 0.f ? __builtin_amdgcn_rcpf(H.om) : 0.f;
  H.p0 = p;
  H.T0 = T;
  H.tpar = dot(T, H.bhat);
  H.tperp = T - H.tpar * H.bhat;
  H.w = cross(T, H.bhat);
  return H;
}

// (One accurate sine and cosine, of the half angle: sin a = 2 sh ch and
// cos a = 1 - 2 sh^2, and 1 - cos a = 2 sh^2 without cancellation.)
__device__ __forceinline__ void helix_at(const Helix& H, float s, V3& p, V3& T) {
  const float a = H.om * s;
  float S, Cc, sh, ch;
  sincosf(0.5f * a, &sh, &ch);
  const float sa = 2.0f * sh * ch, ca = 1.0f - 2.0f * sh * sh;
  if (fabsf(a) < 1e-3f) {
    S = s * (1.0f - a * a * (1.0f / 6.0f));
    Cc = s * (0.5f * a) * (1.0f - a * a * (1.0f / 12.0f));
  } else {
    S = sa * H.inv_om;
    Cc = 2.0f * sh * sh * H.inv_om;
  }
  p = H.p0 + (H.tpar * s) * H.bhat + S * H.tperp + Cc * H.w;
  T = H.tpar * H.bhat + ca * H.tperp + sa * H.w;
}

// The same point for navigation (layer envelopes, module listing with a
// millimetre margin): hardware sine and cosine of the half angle, whose
// absolute error of about 2e-7 moves the point by micrometres even at a
// 17 m bending radius.  Not used where a leg lands on a plane.
__device__ __forceinline__ void helix_at_nav(const Helix& H, float s, V3& p, V3& T) {
  const float a = H.om * s;
  const float sh = __sinf(0.5f * a), ch = __cosf(0.5f * a);
  const float sa = 2.0f * sh * ch, ca = 1.0f - 2.0f * sh * sh;
  float S, Cc;
  if (fabsf(a) < 1e-3f) {
    S = s * (1.0f - a * a * (1.0f / 6.0f));
    Cc = s * (0.5f * a) * (1.0f - a * a * (1.0f / 12.0f));
  } else {
    S = sa * H.inv_om;
    Cc = 2.0f * sh * sh * H.inv_om;
  }
  p = H.p0 + (H.tpar * s) * H.bhat + S * H.tperp + Cc * H.w;
  T = H.tpar * H.bhat + ca * H.tperp + sa * H.w;
}

// Signed path to the plane (c, n) along the local helix of (r, T, lam) in
// field B: three Newton steps from the second-order estimate; NaN when the
// direction grazes the plane.
__device__ __forceinline__ float helix_distance(V3 r, V3 T, float lam, V3 B, V3 c, V3 n) {
  const V3 k = (kKappa * lam) * cross(T, B);
  float s = plane_distance(r, T, k, c, n);
  if (!isfinite(s)) return s;
  const Helix H = make_helix(r, T, lam, B);
#pragma unroll
  for (int it = 0; it < 3; ++it) {
    V3 p, Ts;
    helix_at(H, s, p, Ts);
    const float fp = dot(n, Ts);
    if (fabsf(fp) < 1e-9f) return __int_as_float(0x7fc00000);
    s -= fdiv_fast(dot(n, p - c), fp);
  }
  return s;
}

struct LegStats {
  int trials, rejects;
};

// Adaptive RKN4 steps onto the plane (c, n) given relative to the origin.
template <bool kMap, int NC>
__device__ bool land(LegT<NC>& L, V3 origin, V3 c, V3 n, const FieldDev& F, const CfgDev& cfg, float& h_trial,
                     float& path, LegStats& st) {
  for (int it = 0; it < cfg.max_rk; ++it) {
    const V3 B = field_at<kMap>(F, origin + L.r);
    const float d = helix_distance(L.r, L.T, L.lam, B, c, n);
    if (!isfinite(d)) return false;
    if (fabsf(d) < cfg.land_tol) {
      L.r = L.r + d * L.T;
      L.T = rsqrtf(dot(L.T, L.T)) * L.T;
      path += fabsf(d);
      return true;
    }
    const bool limited = fabsf(d) < h_trial;
    const float h = copysignf(fminf(fabsf(d), h_trial), d);
    Stages S;
    const float err = rkn4_stages<kMap>(L, h, origin, F, B, S);
    ++st.trials;
    if (!(err <= cfg.step_tol)) {
      ++st.rejects;
      h_trial = fabsf(h) * fmaxf(0.25f, 0.9f * sqrtf(sqrtf(fdiv_fast(cfg.step_tol, err))));
      continue;
    }
    rkn4_advance<kMap>(L, h, origin, F, B, S);
    path += fabsf(h);
    const float grow = err > 0.0f ? fminf(4.0f, 0.9f * sqrtf(sqrtf(fdiv_fast(cfg.step_tol, err)))) : 4.0f;
    h_trial = limited ? fminf(cfg.step_max, fmaxf(h_trial, fabsf(h) * grow)) : fminf(cfg.step_max, fabsf(h) * grow);
  }
  return false;
}

// Bound parameters on module A -> leg start (relative to A's centre).
template <int NC>
__device__ __forceinline__ void leg_start(const Module& A, const double* p, LegT<NC>& L, V3& uA, V3& vA) {
  uA = ld3(A.u);
  vA = ld3(A.v);
  const float l0 = (float)p[0], l1 = (float)p[1];
  float sp, cp, st, ct;
  sincosf((float)p[2], &sp, &cp);
  sincosf((float)p[3], &st, &ct);
  L.r = l0 * uA + l1 * vA;
  L.T = {cp * st, sp * st, ct};
  L.lam = (float)p[4];
#pragma unroll
  for (int j = 0; j < NC; ++j) L.dr[j] = L.dT[j] = {0.f, 0.f, 0.f};
  if (NC == 5) {
    L.dr[0] = uA;
    L.dr[1] = vA;
  }
  L.dT[NC - 3] = {-sp * st, cp * st, 0.f};
  L.dT[NC - 2] = {cp * ct, sp * ct, -st};
}

// Landed free state -> bound parameters on module B and the bound-to-bound
// Jacobian with the path-length correction.  dB = B's centre relative to
// the leg origin; qop is the start's FP64 q/p (unchanged along the leg).
template <int NC>
__device__ __forceinline__ void leg_end(const LegT<NC>& L, V3 uA, V3 vA, const Module& Bm, V3 dB, V3 Bf, double qop,
                                        double* p, float J[5][5]) {
  const V3 uB = ld3(Bm.u), vB = ld3(Bm.v), nB = ld3(Bm.n);
  const V3 d = L.r - dB;
  const V3 T = L.T;
  const float st2 = T.x * T.x + T.y * T.y;
  const float st = sqrtf(st2);
  p[0] = (double)dot(uB, d);
  p[1] = (double)dot(vB, d);
  p[2] = (double)atan2_as(T.y, T.x);
  p[3] = (double)atan2_as(st, T.z);
  p[4] = qop;  // no energy loss: q/p keeps its FP64 value
  const V3 kend = (kKappa * L.lam) * cross(T, Bf);
  const float inT = fdiv_fast(1.0f, dot(nB, T));
  const float ist2 = fdiv_fast(1.0f, st2), ist = fdiv_fast(1.0f, st);
  V3 dr[5], dT[5];
  if (NC == 3) {
    dr[0] = uA;
    dT[0] = {0.f, 0.f, 0.f};
    dr[1] = vA;
    dT[1] = {0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    dr[j + 5 - NC] = L.dr[j];
    dT[j + 5 - NC] = L.dT[j];
  }
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const float ds = -dot(nB, dr[j]) * inT;
    const V3 drc = dr[j] + ds * T;
    const V3 dTc = dT[j] + ds * kend;
    J[0][j] = dot(uB, drc);
    J[1][j] = dot(vB, drc);
    J[2][j] = (T.x * dTc.y - T.y * dTc.x) * ist2;
    J[3][j] = -dTc.z * ist;
    J[4][j] = (j == 4) ? 1.0f : 0.0f;
  }
}

// ---------------------------------------------------------------------------
// FP64 covariance algebra on the packed upper triangle.

__device__ __forceinline__ int pk(int i, int j) {
  return i <= j ? i * 5 - (i * (i - 1)) / 2 + (j - i) : j * 5 - (j * (j - 1)) / 2 + (i - j);
}

// C <- J C J^T (J promoted to FP64), symmetric by construction.  J's q/p
// row is the unit row (a leg loses no energy), so its products are the
// covariance's own q/p row and column.
__device__ __forceinline__ void transport_cov(const float J[5][5], double* C) {
  double R[15];
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
      R[pk(i, j)] = s;
    }
  }
#pragma unroll
  for (int q = 0; q < 15; ++q) C[q] = R[q];
}

__device__ __forceinline__ double chi2_of(const double* p, const double* C, double m0, double m1, double v0,
                                          double v1) {
  const double r0 = m0 - p[0], r1 = m1 - p[1];
  const double s00 = C[0] + v0, s01 = C[1], s11 = C[5] + v1;
  const double det = s00 * s11 - s01 * s01;
  return (s11 * r0 * r0 - 2.0 * s01 * r0 * r1 + s00 * r1 * r1) / det;
}

__device__ __forceinline__ double wrap_phi(double phi) {
  const double pi = 3.14159265358979323846;
  if (phi > pi) phi -= 2.0 * pi;
  if (phi <= -pi) phi += 2.0 * pi;
  return phi;
}

// Gain-form Kalman update with the Joseph covariance, FP64, out of place:
// K = C H^T S^-1, p+ = p + K r and
// C+ = (I - K H) C (I - K H)^T + K V K^T evaluated element by element:
// C+_ij = C_ij - K0_i C_0j - K1_i C_1j - C_i0 K0_j - C_i1 K1_j
//         + K0_i g0_j + K1_i g1_j + v0 K0_i K0_j + v1 K1_i K1_j
// with g0 = C00 K0 + C01 K1 and g1 = C01 K0 + C11 K1 (symmetric as written).
__device__ __forceinline__ void kf_update(const double* p, const double* C, double m0, double m1, double v0,
                                          double v1, double* po, double* Co) {
  const double s00 = C[0] + v0, s01 = C[1], s11 = C[5] + v1;
  const double idet = 1.0 / (s00 * s11 - s01 * s01);
  const double i00 = s11 * idet, i01 = -s01 * idet, i11 = s00 * idet;
  const double r0 = m0 - p[0], r1 = m1 - p[1];
  double K0[5], K1[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const double c0 = C[pk(i, 0)], c1 = C[pk(i, 1)];
    K0[i] = c0 * i00 + c1 * i01;
    K1[i] = c0 * i01 + c1 * i11;
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) po[i] = p[i] + K0[i] * r0 + K1[i] * r1;
  po[2] = wrap_phi(po[2]);
  const double c00 = C[0], c01 = C[1], c11 = C[5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = i; j < 5; ++j) {
      const double g0 = c00 * K0[j] + c01 * K1[j], g1 = c01 * K0[j] + c11 * K1[j];
      double x = C[pk(i, j)] - K0[i] * C[pk(0, j)] - K1[i] * C[pk(1, j)] - C[pk(i, 0)] * K0[j] -
                 C[pk(i, 1)] * K1[j];
      x += K0[i] * g0 + K1[i] * g1 + v0 * K0[i] * K0[j] + v1 * K1[i] * K1[j];
      Co[pk(i, j)] = x;
    }
}

// Highland multiple scattering on module M (width in FP32, added in FP64).
__device__ __forceinline__ void apply_ms(const Module& M, double mass, const double* p, double* C) {
  if (!(M.thick > 0.0f)) return;
  float sp, cp, st, ct;
  sincosf((float)p[2], &sp, &cp);
  sincosf((float)p[3], &st, &ct);
  const float cosa = fabsf(M.n[0] * cp * st + M.n[1] * sp * st + M.n[2] * ct);
  const float x = fdiv_fast(M.thick, cosa);
  const float mom = __builtin_amdgcn_rcpf(fabsf((float)p[4]));
  const float m = (float)mass;
  const float beta = mom * __builtin_amdgcn_rsqf(mom * mom + m * m);
  const float th0 = fdiv_fast(0.0136f, beta * mom) * sqrtf(x) * (1.0f + 0.038f * logf(fdiv_fast(x, beta * beta)));
  const double t2 = (double)th0 * (double)th0;
  C[pk(2, 2)] += t2 / ((double)st * (double)st);
  C[pk(3, 3)] += t2;
}

__device__ bool cross_cylinder(const Helix& H, float R, float& s_out, V3& p_out, V3& T_out) {
  const float a = H.T0.x * H.T0.x + H.T0.y * H.T0.y;
  const float b = H.p0.x * H.T0.x + H.p0.y * H.T0.y;
  const float c = H.p0.x * H.p0.x + H.p0.y * H.p0.y - R * R;
  if (a < 1e-12f) return false;
  const float disc = b * b - a * c;
  if (disc < 0.f) return false;
  float s = fdiv_fast(-b + sqrtf(disc), a);
  if (!(s > 0.f)) return false;
  for (int it = 0; it < 20; ++it) {
    V3 p, T;
    helix_at_nav(H, s, p, T);
    const float g = p.x * p.x + p.y * p.y - R * R;
    const float gp = 2.0f * (p.x * T.x + p.y * T.y);
    if (!(gp > 0.f)) return false;
    const float ds = fdiv_fast(g, gp);
    s -= ds;
    if (fabsf(ds) < 1e-4f) break;
  }
  if (!(s > 0.f)) return false;
  V3 p, T;
  helix_at_nav(H, s, p, T);
  if (fabsf(sqrtf(p.x * p.x + p.y * p.y) - R) > 1e-3f) return false;
  s_out = s;
  p_out = p;
  T_out = T;
  return true;
}

__device__ __forceinline__ bool cross_cylinder(const Helix& H, float R, float& s_out) {
  V3 p, T;
  return cross_cylinder(H, R, s_out, p, T);
}

__device__ bool cross_zplane(const Helix& H, float Z, float& s_out) {
  if (fabsf(H.T0.z) < 1e-12f) return false;
  float s = fdiv_fast(Z - H.p0.z, H.T0.z);
  if (!(s > 0.f)) return false;
  for (int it = 0; it < 20; ++it) {
    V3 p, T;
    helix_at_nav(H, s, p, T);
    if (fabsf(T.z) < 1e-12f) return false;
    const float ds = fdiv_fast(p.z - Z, T.z);
    s -= ds;
    if (fabsf(ds) < 1e-4f) break;
  }
  if (!(s > 0.f)) return false;
  s_out = s;
  return true;
}

// Listing test: the second-order expansion P + d T + d^2 k / 2 (from the
// base point P at path s_base) meets the module plane within its half
// lengths plus the margin at positive total path.  The accumulator keeps the
// kMaxList smallest (path, id) in sorted order, each module once.
struct ListAcc {
  float ls[kMaxList];
  int lm[kMaxList];
};

__device__ __forceinline__ void list_init(ListAcc& a) {
#pragma unroll
  for (int q = 0; q < kMaxList; ++q) {
    a.ls[q] = INFINITY;
    a.lm[q] = -1;
  }
}

// The listing test of module m (record M) from the base point: true when the
// expansion meets its plane within the half lengths plus the margin at
// positive total path cs; `tested` is raised when the module passes the
// reach pre-filter.
__device__ __forceinline__ bool list_probe(const Module& M, V3 P, V3 T, V3 k, float s_base, float margin,
                                           float& cs, bool& tested) {
  const V3 c = ld3(M.c), nn = ld3(M.n);
  const float hd = sqrtf((M.hw0 + margin) * (M.hw0 + margin) + (M.hw1 + margin) * (M.hw1 + margin));
  const V3 dc = c - P;
  const float reach = hd + kReach;
  tested = false;
  if (dot(dc, dc) > reach * reach) return false;
  tested = true;
  const float qa = 0.5f * dot(nn, k), qb = dot(nn, T), c0 = dot(nn, P - c);
  if (fabsf(qb) < 1e-3f) return false;
  float d = fdiv_fast(-c0, qb);
  const float disc = qb * qb - 4.0f * qa * c0;
  if (disc >= 0.f) {
    const float qq = -0.5f * (qb + copysignf(sqrtf(disc), qb));
    if (qq != 0.f) d = fdiv_fast(c0, qq);
  }
  const V3 X = P + d * T + (0.5f * d * d) * k - c;
  const float l0 = dot(ld3(M.u), X), l1 = dot(ld3(M.v), X);
  if (fabsf(l0) > M.hw0 + margin || fabsf(l1) > M.hw1 + margin) return false;
  cs = s_base + d;
  return cs > 0.f;
}

// Insert a listed (path, module) into the accumulator: the kMaxList smallest
// (path, id) in order, each module once.  (A module met twice has the same
// path both times, so the result does not depend on the order of insertion.)
__device__ __forceinline__ void list_insert(ListAcc& a, int m, float cs) {
  if (a.lm[0] == m || a.lm[1] == m || a.lm[2] == m || a.lm[3] == m) return;
  int cm = m;
#pragma unroll
  for (int q = 0; q < kMaxList; ++q) {
    const bool lt = cs < a.ls[q] || (cs == a.ls[q] && cm < a.lm[q]);
    if (lt) {
      const float ts = a.ls[q];
      const int tm = a.lm[q];
      a.ls[q] = cs;
      a.lm[q] = cm;
      cs = ts;
      cm = tm;
    }
  }
}

__device__ __forceinline__ void list_test(ListAcc& a, int m, const Module& M, V3 P, V3 T, V3 k, float s_base,
                                          float margin, int& n_tested) {
  float cs;
  bool tested;
  const bool pass = list_probe(M, P, T, k, s_base, margin, cs, tested);
  n_tested += tested ? 1 : 0;
  if (pass) list_insert(a, m, cs);
}

__device__ __forceinline__ int list_out(const ListAcc& a, int* list) {
  int n = 0;
#pragma unroll
  for (int q = 0; q < kMaxList; ++q) {
    list[q] = a.lm[q];
    n += a.lm[q] >= 0 ? 1 : 0;
  }
  return n;
}

// The navigation grid's cells near the trajectory segment from P along T on
// layer Lr: phi rows ip0..ip1 (taken modulo nphi) and w cells iw0..iw1 of
// each row.  False when the segment's bounds are not finite (nothing is
// listed then); iw0 > iw1 means no cells.
struct GridRange {
  int ip0, ip1, iw0, iw1;
};

__device__ __forceinline__ bool grid_range(const LayerRec& Lr, V3 P, V3 T, GridRange& gr) {
  // segment of the trajectory that can reach the layer's modules
  float span;
  if (Lr.type == 0) {
    const float rp = sqrtf(P.x * P.x + P.y * P.y);
    const float vr = rp > 0.f ? fdiv_fast(P.x * T.x + P.y * T.y, rp) : 1.0f;
    span = fdiv_fast(Lr.depth, fmaxf(vr, 0.05f)) * 1.2f + 2.0f;
  } else {
    span = fdiv_fast(Lr.depth, fmaxf(fabsf(T.z), 0.05f)) * 1.2f + 2.0f;
  }
  span = fminf(span, 400.0f);
  const V3 Q = P + span * T;
  const float twopi = 6.28318530718f;
  float ph0 = atan2_as(P.y, P.x), ph1 = atan2_as(Q.y, Q.x);
  float w0 = Lr.type == 0 ? P.z : sqrtf(P.x * P.x + P.y * P.y);
  float w1 = Lr.type == 0 ? Q.z : sqrtf(Q.x * Q.x + Q.y * Q.y);
  float dph = ph1 - ph0;
  if (dph > 3.14159265f) dph -= twopi;
  if (dph < -3.14159265f) dph += twopi;
  const float phlo = fminf(ph0, ph0 + dph), phhi = fmaxf(ph0, ph0 + dph);
  const float wlo = fminf(w0, w1), whi = fmaxf(w0, w1);
  if (!(isfinite(phlo) && isfinite(phhi) && isfinite(wlo) && isfinite(whi))) return false;
  // bins per radian and per unit of w (the grid extents are padded, so
  // rounding of the bin edges cannot lose a module)
  const float iph = (float)Lr.nphi * (1.0f / twopi), iw = fdiv_fast((float)Lr.nw, Lr.whi - Lr.wlo);
  gr.ip0 = (int)floorf((phlo + 3.14159265f) * iph);
  gr.ip1 = (int)floorf((phhi + 3.14159265f) * iph);
  gr.iw0 = max((int)floorf((wlo - Lr.wlo) * iw), 0);
  gr.iw1 = min((int)floorf((whi - Lr.wlo) * iw), Lr.nw - 1);
  if (gr.ip1 - gr.ip0 >= Lr.nphi) {
    gr.ip0 = 0;
    gr.ip1 = Lr.nphi - 1;
  }
  return true;
}

// The CSR range of phi row ipr (modulo nphi) over the cells iw0..iw1: the
// cells of one row are adjacent in the grid's CSR.
__device__ __forceinline__ void grid_row(const GeomDev& g, const LayerRec& Lr, const GridRange& gr, int ipr, int& a,
                                         int& b) {
  int ip = ipr % Lr.nphi;
  if (ip < 0) ip += Lr.nphi;
  const int row = Lr.cell_base + ip * Lr.nw;
  a = g.cell_off[row + gr.iw0];
  b = g.cell_off[row + gr.iw1 + 1];
}

// Candidate modules of layer `l` near the trajectory segment from P along T
// (navigation grid lookup), each put through the listing test, at most
// kMaxCand grid entries in visiting order (rows by phi, entries in pairs).
// Returns the number listed (<= kMaxList, sorted by path then id).  One lane
// on its own; the search kernel lists a wave's lanes together (list_wave)
// and comes here only for the rare lane that does not fit that scheme.
__device__ int list_layer(const GeomDev& g, int l, V3 P, V3 T, V3 k, float s_base, int exclude, float margin,
                          int* list, int& n_tested, int& overflow, int& n_visited) {
  const LayerRec Lr = g.layers[l];
  GridRange gr;
  if (!grid_range(Lr, P, T, gr)) return 0;
  ListAcc acc;
  list_init(acc);
  int visited = 0;
  for (int ipr = gr.ip0; ipr <= gr.ip1 && gr.iw0 <= gr.iw1; ++ipr) {
    int a, b;
    grid_row(g, Lr, gr, ipr, a, b);
    // two candidates per round: their id and record loads are in flight together
    for (int q = a; q < b; q += 2) {
      if (visited >= kMaxCand) {
        overflow = 1;
        break;
      }
      visited += q + 1 < b ? 2 : 1;
      n_visited += q + 1 < b ? 2 : 1;
      const int m0 = g.cell_mod[q];
      const int m1 = q + 1 < b ? g.cell_mod[q + 1] : -1;
      Module M0, M1;
      load_module(g, m0, M0);
      if (m1 >= 0) load_module(g, m1, M1);
      if (m0 != exclude) list_test(acc, m0, M0, P, T, k, s_base, margin, n_tested);
      if (m1 >= 0 && m1 != exclude) list_test(acc, m1, M1, P, T, k, s_base, margin, n_tested);
    }
  }
  return list_out(acc, list);
}

// The next navigation layer from free state (p, T, lam) in global
// coordinates: the unvisited layer whose envelope the local helix meets
// first within its extent and the path budget, with the crossing's path,
// point and direction.  Returns -1 if none.
__device__ int next_layer(const GeomDev& g, const Helix& H, unsigned long long mask, float budget, float& s_best,
                          V3& p_best, V3& T_best, int& n_tried) {
  const float rperp = sqrtf(H.p0.x * H.p0.x + H.p0.y * H.p0.y);
  int best = -1;
  s_best = INFINITY;
  // With the field along z, z grows linearly along the path and the distance
  // from the axis by at most sin(theta) per unit path, so the crossing of
  // radius R lies at z beyond p0.z + cot(theta) (R - r): a barrel whose
  // extent that bound already overshoots (by more than kZSkip) is crossed
  // outside it, and its Newton solve can be skipped with the same outcome.
  constexpr float kZSkip = 1.0f;  // mm, far above the FP32 error of the bound
  const bool axial = H.bhat.x == 0.f && H.bhat.y == 0.f;
  const float sth = sqrtf(H.T0.x * H.T0.x + H.T0.y * H.T0.y);
  const float cot = sth > 0.f ? fdiv_fast(H.T0.z, sth) : 0.f;
  // barrels by radius: the first crossed within its extent is the nearest
  for (int q = 0; q < g.n_barrel; ++q) {
    const int l = g.barrel_order[q];
    if (mask & (1ull << l)) continue;
    const LayerRec Lr = g.layers[l];
    if (!(Lr.pos > rperp)) continue;
    if (axial && sth > 0.f) {
      const float zb = H.p0.z + cot * (Lr.pos - rperp);
      if (H.T0.z > 0.f ? zb > Lr.hi + kZSkip : zb < Lr.lo - kZSkip) continue;
    }
    ++n_tried;
    float s;
    V3 p, T;
    if (!cross_cylinder(H, Lr.pos, s, p, T)) continue;
    if (p.z < Lr.lo || p.z > Lr.hi) continue;
    if (s > budget) break;
    best = l;
    s_best = s;
    p_best = p;
    T_best = T;
    break;
  }
  // disks on the side the track moves to, by |z|
  const int nd = H.T0.z > 0.f ? g.n_disk_pos : g.n_disk_neg;
  const int* order = H.T0.z > 0.f ? g.disk_pos : g.disk_neg;
  for (int q = 0; q < nd; ++q) {
    const int l = order[q];
    if (mask & (1ull << l)) continue;
    const LayerRec Lr = g.layers[l];
    ++n_tried;
    float s;
    if (!cross_zplane(H, Lr.pos, s)) continue;
    if (s > s_best || s > budget) break;
    V3 p, T;
    helix_at_nav(H, s, p, T);
    const float r = sqrtf(p.x * p.x + p.y * p.y);
    if (r < Lr.lo || r > Lr.hi) continue;
    if (s < s_best || (s == s_best && l < best)) {
      best = l;
      s_best = s;
      p_best = p;
      T_best = T;
    }
    break;
  }
  return best;
}

}  // namespace ckf
