// FP64 CPU oracle of combinatorial-Kalman-filter (CKF) track finding.
//
// TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
// baseline of the benchmark; never by the GPU product path, with which it
// shares no code.  Built with -O2 -ffp-contract=off (no fused multiply-add,
// no fast-math) so that its rounding is plain IEEE-754 double.
//
// What it computes, in the paper's order (section 2):
//   * seeds are the initial track parameters of the CKF;
//   * parameters and covariances are propagated with the fourth-order
//     Runge-Kutta-Nystrom method (RKN4) and Jacobian transport;
//   * on each intersected module a Kalman-filter chi2 from the covariance and
//     the residual is computed for the measurements; a small enough chi2
//     attaches the measurement as a new branch;
//   * filtered parameters are most accurate at the last measurement, which is
//     what a found track reports;
//   * material effects assume muons (section 3): multiple scattering only.
// Matching of found patterns requires identical measurements (Table 1).
//
// Readings where the paper is silent (each is a documented choice shared by
// the GPU library, which implements it independently):
//   R-param  bound (loc0, loc1, phi, theta, q/p); free (r, T, q/p), |T| = 1.
//   R-rkn    textbook Nystrom RKN4 for r'' = kappa*lambda*(r' x B), field
//            sampled at the start, the shared midpoint and the end; error
//            estimate h^2 * max|k1-k2-k3+k4|; accept if <= step_tol; next
//            trial h * clamp(0.9 (tol/err)^(1/4)) within [0.25, 4].
//   R-land   each trial step is limited to the distance to the target plane
//            along the local helix (field at the current point; three Newton
//            steps from the second-order estimate r + dT + d^2 k/2); landed
//            when that distance is below land_tol, then moved onto the plane
//            along T.
//   R-jac    Jacobian by differentiating each RKN4 stage (tangent columns),
//            then free->bound with the path-length correction.
//   R-nav    the next navigation layer is the unvisited layer whose envelope
//            the local helix (field at the current point) meets first within
//            the envelope's extent; its modules whose centre lies within
//            their half diagonal (with margin) plus 30 mm of that crossing
//            are listed when the second-order expansion of the helix at the
//            crossing meets their plane within the half lengths plus
//            nav_margin; listed modules are visited in path order (at most
//            4); a visited module is crossed when the landed local position
//            is within its half lengths.  A seed starts with its own layer's
//            modules listed the same way from the seed position (overlaps).
//   R-gate   S = C[0:2,0:2] + V, chi2 = r^T S^-1 r, accept chi2 < chi2_max;
//            keep the branches_per_surface smallest (chi2, id).
//   R-kf     gain form, 2x2 innovation inverse, Joseph covariance.
//   R-ms     Highland width with the path x/X0/|cos(alpha)|, added to
//            Var(phi) (divided by sin^2 theta) and Var(theta) after the
//            update; no energy loss.
//   R-holes  a crossed module with no accepted measurement is a hole; no
//            "skip" branch is made when measurements are accepted.
//   R-prune  after each step, a seed keeps its max_live best live candidates
//            by the rank key (n_meas desc, chi2 asc, holes asc, ids lex asc).
//   R-out    best finished candidate per seed by the same key, reporting the
//            filtered state at its last measurement.
#include "oracle.h"

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

namespace {

constexpr double kKappa = 2.99792458e-4;  // GeV / (T mm): q/p[1/GeV] * B[T] -> curvature [1/mm]
constexpr double kReach = 30.0;           // mm: envelope-to-module reach of the candidate pre-filter
constexpr int kMaxList = 4;               // listed modules per layer
constexpr double kPi = 3.14159265358979323846;

struct V3 {
  double x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline double maxabs(V3 a) { return std::max(std::fabs(a.x), std::max(std::fabs(a.y), std::fabs(a.z))); }

struct Surface {
  V3 c, u, v, n;
  double hw0, hw1, thick;
  int layer;
};
struct Layer {
  int type;
  double pos, lo, hi;
};

struct Geometry {
  std::vector<Surface> s;
  std::vector<Layer> layers;
  std::vector<std::vector<int>> members;  // modules of each layer
};

Geometry load_geometry(const orc_geometry* g) {
  Geometry G;
  G.s.resize(g->n_surfaces);
  G.layers.resize(g->n_layers);
  G.members.resize(g->n_layers);
  for (int i = 0; i < g->n_surfaces; ++i) {
    Surface& S = G.s[i];
    const float* c = g->center + 3 * i;
    const float* r = g->rot + 9 * i;
    S.c = {c[0], c[1], c[2]};
    S.u = {r[0], r[1], r[2]};
    S.v = {r[3], r[4], r[5]};
    S.n = {r[6], r[7], r[8]};
    S.hw0 = g->half[2 * i];
    S.hw1 = g->half[2 * i + 1];
    S.thick = g->thick[i];
    S.layer = g->layer[i];
    G.members[S.layer].push_back(i);
  }
  for (int l = 0; l < g->n_layers; ++l)
    G.layers[l] = {g->layer_type[l], g->layer_pos[l], g->layer_lo[l], g->layer_hi[l]};
  return G;
}

// Field: uniform, or bilinear interpolation of an (r, z) map of (B_r, B_z)
// with coordinates clamped to the grid (the grid is the field's definition).
struct Field {
  V3 b{0, 0, 0};
  const float* map = nullptr;
  int nr = 0, nz = 0;
  double r0 = 0, z0 = 0, dr = 1, dz = 1;

  // cell, fractions and whether the coordinate was clamped
  void cell(double u, int n, int& i, double& f, bool& clamped) const {
    clamped = false;
    if (u <= 0) {
      u = 0;
      clamped = true;
    } else if (u >= n - 1) {
      u = n - 1;
      clamped = true;
    }
    i = std::min((int)std::floor(u), n - 2);
    f = u - i;
  }
  double node(int ir, int iz, int c) const { return map[((size_t)iz * nr + ir) * 2 + c]; }

  V3 at(V3 p) const {
    V3 B;
    double G[3][3];
    eval(p, B, G, false);
    return B;
  }
  // B at p and, if want_grad, G[i][j] = dB_i/dx_j (of the interpolant)
  void eval(V3 p, V3& B, double G[3][3], bool want_grad) const {
    if (!map) {
      B = b;
      if (want_grad)
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) G[i][j] = 0;
      return;
    }
    const double r = std::hypot(p.x, p.y);
    int ir, iz;
    double fr, fz;
    bool cr, cz;
    cell((r - r0) / dr, nr, ir, fr, cr);
    cell((p.z - z0) / dz, nz, iz, fz, cz);
    double v[2], vr[2], vz[2];
    for (int c = 0; c < 2; ++c) {
      const double a = node(ir, iz, c), bb = node(ir + 1, iz, c), cc = node(ir, iz + 1, c),
                   d = node(ir + 1, iz + 1, c);
      v[c] = (1 - fr) * (1 - fz) * a + fr * (1 - fz) * bb + (1 - fr) * fz * cc + fr * fz * d;
      vr[c] = cr ? 0.0 : ((1 - fz) * (bb - a) + fz * (d - cc)) / dr;
      vz[c] = cz ? 0.0 : ((1 - fr) * (cc - a) + fr * (d - bb)) / dz;
    }
    const double cx = r > 0 ? p.x / r : 0.0, sy = r > 0 ? p.y / r : 0.0;
    B = {v[0] * cx, v[0] * sy, v[1]};
    if (!want_grad) return;
    // chain rule through r = hypot(x, y): d(cx)/dx = sy^2/r, d(cx)/dy = -cx sy/r, ...
    const double ir_ = r > 0 ? 1.0 / r : 0.0;
    G[0][0] = vr[0] * cx * cx + v[0] * sy * sy * ir_;
    G[0][1] = vr[0] * cx * sy - v[0] * cx * sy * ir_;
    G[0][2] = vz[0] * cx;
    G[1][0] = vr[0] * cx * sy - v[0] * cx * sy * ir_;
    G[1][1] = vr[0] * sy * sy + v[0] * cx * cx * ir_;
    G[1][2] = vz[0] * sy;
    G[2][0] = vr[1] * cx;
    G[2][1] = vr[1] * sy;
    G[2][2] = vz[1];
  }
};

V3 mat_vec(const double G[3][3], V3 d) {
  return {G[0][0] * d.x + G[0][1] * d.y + G[0][2] * d.z, G[1][0] * d.x + G[1][1] * d.y + G[1][2] * d.z,
          G[2][0] * d.x + G[2][1] * d.y + G[2][2] * d.z};
}

Field load_field(const orc_field* f) {
  Field F;
  F.b = {f->b[0], f->b[1], f->b[2]};
  F.map = f->map;
  F.nr = f->nr;
  F.nz = f->nz;
  F.r0 = f->r0;
  F.z0 = f->z0;
  F.dr = f->dr;
  F.dz = f->dz;
  return F;
}

struct Cfg {
  double chi2_max, step_tol, step_max, land_tol, path_max, nav_margin, mass;
  int branches, max_live, max_holes, min_meas, max_steps, max_rk;
  bool material;
  int tracks_per_seed;
};

Cfg load_cfg(const orc_config* c) {
  Cfg k;
  k.chi2_max = c->chi2_max;
  k.step_tol = c->step_tol;
  k.step_max = c->step_max;
  k.land_tol = c->land_tol;
  k.path_max = c->path_max;
  k.nav_margin = c->nav_margin;
  k.mass = c->mass;
  k.branches = c->branches_per_surface;
  k.max_live = c->max_live_per_seed;
  k.max_holes = c->max_holes;
  k.min_meas = c->min_meas;
  k.max_steps = c->max_steps;
  k.max_rk = c->max_rk_steps;
  k.material = c->material_on != 0;
  k.tracks_per_seed = c->tracks_per_seed;
  return k;
}

struct Stats {
  int64_t steps = 0, navigations = 0, nav_modules = 0, legs = 0, legs_failed = 0, rk_trials = 0,
          rk_rejects = 0, chi2_evals = 0, kf_updates = 0, ms_updates = 0, crossed = 0, holes = 0,
          pruned = 0, finished = 0, mlp_rows = 0, proposals = 0, proposal_misses = 0;
  void add(const Stats& o) {
    steps += o.steps; navigations += o.navigations; nav_modules += o.nav_modules; legs += o.legs;
    legs_failed += o.legs_failed; rk_trials += o.rk_trials; rk_rejects += o.rk_rejects;
    chi2_evals += o.chi2_evals; kf_updates += o.kf_updates; ms_updates += o.ms_updates;
    crossed += o.crossed; holes += o.holes; pruned += o.pruned; finished += o.finished;
    mlp_rows += o.mlp_rows; proposals += o.proposals; proposal_misses += o.proposal_misses;
  }
};

// ---------------------------------------------------------------------------
// 5x5 matrices (row-major) and the packed upper triangle.

using M5 = std::array<double, 25>;

int packed_index(int i, int j) {
  if (i > j) std::swap(i, j);
  return i * 5 - i * (i - 1) / 2 + (j - i);
}
M5 unpack(const double* p) {
  M5 C{};
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) C[5 * i + j] = p[packed_index(i, j)];
  return C;
}
void pack(const M5& C, double* p) {
  for (int i = 0; i < 5; ++i)
    for (int j = i; j < 5; ++j) p[packed_index(i, j)] = C[5 * i + j];
}
M5 matmul(const M5& A, const M5& B) {
  M5 R{};
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      double s = 0;
      for (int k = 0; k < 5; ++k) s += A[5 * i + k] * B[5 * k + j];
      R[5 * i + j] = s;
    }
  return R;
}
M5 transpose(const M5& A) {
  M5 R{};
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) R[5 * j + i] = A[5 * i + j];
  return R;
}
// J C J^T, symmetrised.
M5 transport(const M5& J, const M5& C) {
  M5 R = matmul(matmul(J, C), transpose(J));
  for (int i = 0; i < 5; ++i)
    for (int j = i + 1; j < 5; ++j) {
      double a = 0.5 * (R[5 * i + j] + R[5 * j + i]);
      R[5 * i + j] = R[5 * j + i] = a;
    }
  return R;
}

double wrap_phi(double phi) {
  while (phi > kPi) phi -= 2 * kPi;
  while (phi <= -kPi) phi += 2 * kPi;
  return phi;
}

// ---------------------------------------------------------------------------
// Free state and tangent columns (derivatives w.r.t. the 5 bound parameters
// at the start of the transport).

struct Free {
  V3 r, T;
  double qop;
};
struct Tangent {
  V3 dr, dT;
  double dl;
};
using Tangents = std::array<Tangent, 5>;

V3 direction(double phi, double theta) {
  return {std::cos(phi) * std::sin(theta), std::sin(phi) * std::sin(theta), std::cos(theta)};
}

Free bound_to_free(const Surface& S, const double* p) {
  Free f;
  f.r = S.c + p[0] * S.u + p[1] * S.v;
  f.T = direction(p[2], p[3]);
  f.qop = p[4];
  return f;
}

// d(free)/d(bound) at the start surface: the initial tangent columns.
Tangents bound_to_free_jacobian(const Surface& S, const double* p) {
  double sp = std::sin(p[2]), cp = std::cos(p[2]), st = std::sin(p[3]), ct = std::cos(p[3]);
  Tangents J{};
  J[0] = {S.u, {0, 0, 0}, 0};
  J[1] = {S.v, {0, 0, 0}, 0};
  J[2] = {{0, 0, 0}, {-sp * st, cp * st, 0}, 0};
  J[3] = {{0, 0, 0}, {cp * ct, sp * ct, -st}, 0};
  J[4] = {{0, 0, 0}, {0, 0, 0}, 1};
  return J;
}

// One RKN4 step of length h for r'' = kappa*lambda*(r' x B(r)), with the
// tangent columns carried through the same stages.  Returns the error
// estimate h^2 * max|k1 - k2 - k3 + k4|.
double rkn4_step(const Field& F, const Free& f, const Tangents& J, double h, Free& fo, Tangents& Jo) {
  const double lam = f.qop;
  const V3 r = f.r, T = f.T;
  V3 B1, B2, B4;
  double G1[3][3], G2[3][3], G4[3][3];
  const bool grad = F.map != nullptr;  // a uniform field has no position derivative
  F.eval(r, B1, G1, grad);
  const V3 k1 = (kKappa * lam) * cross(T, B1);
  const V3 rm = r + (0.5 * h) * T + (h * h / 8.0) * k1;
  F.eval(rm, B2, G2, grad);
  const V3 T2 = T + (0.5 * h) * k1;
  const V3 k2 = (kKappa * lam) * cross(T2, B2);
  const V3 T3 = T + (0.5 * h) * k2;
  const V3 k3 = (kKappa * lam) * cross(T3, B2);
  const V3 re = r + h * T + (0.5 * h * h) * k3;
  F.eval(re, B4, G4, grad);
  const V3 T4 = T + h * k3;
  const V3 k4 = (kKappa * lam) * cross(T4, B4);
  fo.r = r + h * T + (h * h / 6.0) * (k1 + k2 + k3);
  fo.T = T + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4);
  fo.qop = lam;
  for (int j = 0; j < 5; ++j) {
    // d k = kappa (dl T x B + lam dT x B + lam T x (dB/dr . d(stage point)))
    const V3 dr = J[j].dr, dT = J[j].dT;
    const double dl = J[j].dl;
    V3 dk1 = kKappa * (dl * cross(T, B1) + lam * cross(dT, B1));
    if (grad) dk1 = dk1 + (kKappa * lam) * cross(T, mat_vec(G1, dr));
    const V3 drm = dr + (0.5 * h) * dT + (h * h / 8.0) * dk1;
    const V3 dT2 = dT + (0.5 * h) * dk1;
    V3 dk2 = kKappa * (dl * cross(T2, B2) + lam * cross(dT2, B2));
    if (grad) dk2 = dk2 + (kKappa * lam) * cross(T2, mat_vec(G2, drm));
    const V3 dT3 = dT + (0.5 * h) * dk2;
    V3 dk3 = kKappa * (dl * cross(T3, B2) + lam * cross(dT3, B2));
    if (grad) dk3 = dk3 + (kKappa * lam) * cross(T3, mat_vec(G2, drm));
    const V3 dre = dr + h * dT + (0.5 * h * h) * dk3;
    const V3 dT4 = dT + h * dk3;
    V3 dk4 = kKappa * (dl * cross(T4, B4) + lam * cross(dT4, B4));
    if (grad) dk4 = dk4 + (kKappa * lam) * cross(T4, mat_vec(G4, dre));
    Jo[j].dr = dr + h * dT + (h * h / 6.0) * (dk1 + dk2 + dk3);
    Jo[j].dT = dT + (h / 6.0) * (dk1 + 2.0 * dk2 + 2.0 * dk3 + dk4);
    Jo[j].dl = dl;
  }
  return h * h * maxabs(k1 - k2 - k3 + k4);
}

// Signed path to the plane (c, n) from the second-order expansion
// r + d T + d^2 k / 2; NaN when the direction grazes the plane.
double plane_distance(V3 r, V3 T, V3 k, V3 c, V3 n) {
  const double a = 0.5 * dot(n, k), b = dot(n, T), c0 = dot(n, r - c);
  if (std::fabs(b) < 1e-9) return NAN;
  const double lin = -c0 / b;
  const double disc = b * b - 4.0 * a * c0;
  if (disc < 0) return lin;
  const double q = -0.5 * (b + std::copysign(std::sqrt(disc), b));
  if (q == 0) return lin;
  return c0 / q;
}

// Local helix of a free state about the field at its position (exact
// trajectory in a uniform field).
struct Helix {
  V3 p0, T0, bhat, w;  // w = T0 x bhat
  double tpar;         // T0 . bhat
  V3 tperp;            // T0 - tpar bhat
  double om;           // kappa * q/p * |B|, turning rate about bhat
  double lam;
  V3 B;
  Helix(const Free& f, V3 B_) : p0(f.r), T0(f.T), lam(f.qop), B(B_) {
    const double bm = norm(B);
    bhat = bm > 0 ? (1.0 / bm) * B : V3{0, 0, 1};
    om = kKappa * f.qop * bm;
    tpar = dot(T0, bhat);
    tperp = T0 - tpar * bhat;
    w = cross(T0, bhat);
  }
  void at(double s, V3& p, V3& T) const {
    const double a = om * s;
    double S, Cc;  // sin(a)/om and (1-cos a)/om, stable for small a
    if (std::fabs(a) < 1e-4) {
      S = s * (1.0 - a * a / 6.0);
      Cc = s * (0.5 * a) * (1.0 - a * a / 12.0);
    } else {
      S = std::sin(a) / om;
      const double hs = std::sin(0.5 * a);
      Cc = 2.0 * hs * hs / om;
    }
    p = p0 + (tpar * s) * bhat + S * tperp + Cc * w;
    T = tpar * bhat + std::cos(a) * tperp + std::sin(a) * w;
  }
};

// Signed path to the plane (c, n) along the local helix: three Newton steps
// from the second-order estimate.  NaN when the direction grazes the plane.
double helix_distance(const Field& F, const Free& f, V3 c, V3 n) {
  const V3 k = (kKappa * f.qop) * cross(f.T, F.at(f.r));
  double s = plane_distance(f.r, f.T, k, c, n);
  if (!std::isfinite(s)) return s;
  const Helix H(f, F.at(f.r));
  for (int it = 0; it < 3; ++it) {
    V3 p, T;
    H.at(s, p, T);
    const double fp = dot(n, T);
    if (std::fabs(fp) < 1e-9) return NAN;
    s -= dot(n, p - c) / fp;
  }
  return s;
}

// Step onto the plane (c, n): RKN4 trials limited by the predicted distance,
// adaptive step size, landed below land_tol.  h_trial and path are updated.
bool land(const Field& F, const Cfg& cfg, V3 c, V3 n, Free& f, Tangents& J, double& h_trial,
          double& path, Stats& st) {
  for (int it = 0; it < cfg.max_rk; ++it) {
    const double d = helix_distance(F, f, c, n);
    if (!std::isfinite(d)) return false;
    if (std::fabs(d) < cfg.land_tol) {
      f.r = f.r + d * f.T;
      f.T = (1.0 / norm(f.T)) * f.T;
      path += std::fabs(d);
      return true;
    }
    const bool limited = std::fabs(d) < h_trial;
    const double h = std::copysign(std::min(std::fabs(d), h_trial), d);
    Free fo;
    Tangents Jo;
    const double err = rkn4_step(F, f, J, h, fo, Jo);
    ++st.rk_trials;
    if (!(err <= cfg.step_tol)) {
      ++st.rk_rejects;
      h_trial = std::fabs(h) * std::max(0.25, 0.9 * std::pow(cfg.step_tol / err, 0.25));
      continue;
    }
    f = fo;
    J = Jo;
    path += std::fabs(h);
    const double grow = err > 0 ? std::min(4.0, 0.9 * std::pow(cfg.step_tol / err, 0.25)) : 4.0;
    h_trial = limited ? std::min(cfg.step_max, std::max(h_trial, std::fabs(h) * grow))
                      : std::min(cfg.step_max, std::fabs(h) * grow);
  }
  return false;
}

// Free state on surface S -> bound parameters, and the bound-to-bound
// Jacobian from the tangent columns with the path-length correction
// (perturbed tracks are moved along the trajectory back onto the plane).
void free_to_bound(const Field& F, const Surface& S, const Free& f, const Tangents& J, double* p, M5& Jbb) {
  const V3 d = f.r - S.c;
  const V3 T = f.T;
  p[0] = dot(S.u, d);
  p[1] = dot(S.v, d);
  p[2] = std::atan2(T.y, T.x);
  const double sinth = std::sqrt(T.x * T.x + T.y * T.y);
  p[3] = std::atan2(sinth, T.z);
  p[4] = f.qop;
  const V3 kend = (kKappa * f.qop) * cross(T, F.at(f.r));
  const double nT = dot(S.n, T);
  for (int j = 0; j < 5; ++j) {
    const double ds = -dot(S.n, J[j].dr) / nT;
    const V3 drc = J[j].dr + ds * T;
    const V3 dTc = J[j].dT + ds * kend;
    Jbb[5 * 0 + j] = dot(S.u, drc);
    Jbb[5 * 1 + j] = dot(S.v, drc);
    Jbb[5 * 2 + j] = (T.x * dTc.y - T.y * dTc.x) / (sinth * sinth);
    Jbb[5 * 3 + j] = -dTc.z / sinth;
    Jbb[5 * 4 + j] = J[j].dl;
  }
}

// Bound state on src -> bound state on dst's plane with covariance transport.
bool propagate(const Geometry& G, const Field& F, const Cfg& cfg, int src, const double* p,
               const M5& C, int dst, double* po, M5& Co, M5* Jout, double& h_trial, double& path,
               Stats& st) {
  ++st.legs;
  Free f = bound_to_free(G.s[src], p);
  Tangents J = bound_to_free_jacobian(G.s[src], p);
  const Surface& D = G.s[dst];
  if (!land(F, cfg, D.c, D.n, f, J, h_trial, path, st)) {
    ++st.legs_failed;
    return false;
  }
  M5 Jbb{};
  free_to_bound(F, D, f, J, po, Jbb);
  for (int i = 0; i < 5; ++i)
    if (!std::isfinite(po[i])) {
      ++st.legs_failed;
      return false;
    }
  Co = transport(Jbb, C);
  if (Jout) *Jout = Jbb;
  return true;
}

// ---------------------------------------------------------------------------
// Kalman filter pieces.

// chi2 of a 2D measurement against the prediction (p, C).
double chi2_of(const double* p, const M5& C, double m0, double m1, double v0, double v1) {
  const double r0 = m0 - p[0], r1 = m1 - p[1];
  const double s00 = C[0] + v0, s01 = C[1], s11 = C[6] + v1;
  const double det = s00 * s11 - s01 * s01;
  return (s11 * r0 * r0 - 2.0 * s01 * r0 * r1 + s00 * r1 * r1) / det;
}

// Gain-form update with the Joseph covariance form.
double kf_update(const double* p, const M5& C, double m0, double m1, double v0, double v1,
                 double* po, M5& Co) {
  const double s00 = C[0] + v0, s01 = C[1], s11 = C[6] + v1;
  const double det = s00 * s11 - s01 * s01;
  const double i00 = s11 / det, i01 = -s01 / det, i11 = s00 / det;  // S^-1
  const double r0 = m0 - p[0], r1 = m1 - p[1];
  double K[5][2];
  for (int i = 0; i < 5; ++i) {
    K[i][0] = C[5 * i + 0] * i00 + C[5 * i + 1] * i01;
    K[i][1] = C[5 * i + 0] * i01 + C[5 * i + 1] * i11;
  }
  for (int i = 0; i < 5; ++i) po[i] = p[i] + K[i][0] * r0 + K[i][1] * r1;
  po[2] = wrap_phi(po[2]);
  M5 A{};  // I - K H
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) A[5 * i + j] = (i == j ? 1.0 : 0.0) - (j < 2 ? K[i][j] : 0.0);
  M5 R = matmul(matmul(A, C), transpose(A));
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) R[5 * i + j] += K[i][0] * v0 * K[j][0] + K[i][1] * v1 * K[j][1];
  for (int i = 0; i < 5; ++i)
    for (int j = i + 1; j < 5; ++j) {
      double a = 0.5 * (R[5 * i + j] + R[5 * j + i]);
      R[5 * i + j] = R[5 * j + i] = a;
    }
  Co = R;
  return i00 * r0 * r0 + 2.0 * i01 * r0 * r1 + i11 * r1 * r1;
}

// Multiple scattering in the module's material (Highland width).
void apply_ms(const Surface& S, double mass, const double* p, M5& C) {
  if (!(S.thick > 0)) return;
  const V3 T = direction(p[2], p[3]);
  const double cosa = std::fabs(dot(S.n, T));
  const double x = S.thick / cosa;
  const double mom = 1.0 / std::fabs(p[4]);
  const double beta = mom / std::sqrt(mom * mom + mass * mass);
  const double th0 = 0.0136 / (beta * mom) * std::sqrt(x) * (1.0 + 0.038 * std::log(x / (beta * beta)));
  const double sth = std::sin(p[3]);
  C[5 * 2 + 2] += th0 * th0 / (sth * sth);
  C[5 * 3 + 3] += th0 * th0;
}

// ---------------------------------------------------------------------------
// Navigation: local helix, layer envelopes, module listing.


// Smallest positive path to the cylinder r = R: straight-line root, then
// Newton on |p_perp(s)|^2 - R^2.  Returns false when there is none.
bool cross_cylinder(const Helix& H, double R, double& s_out) {
  const double a = H.T0.x * H.T0.x + H.T0.y * H.T0.y;
  const double b = H.p0.x * H.T0.x + H.p0.y * H.T0.y;
  const double c = H.p0.x * H.p0.x + H.p0.y * H.p0.y - R * R;
  if (a < 1e-12) return false;
  const double disc = b * b - a * c;
  if (disc < 0) return false;
  double s = (-b + std::sqrt(disc)) / a;
  if (!(s > 0)) return false;
  for (int it = 0; it < 20; ++it) {
    V3 p, T;
    H.at(s, p, T);
    const double g = p.x * p.x + p.y * p.y - R * R;
    const double gp = 2.0 * (p.x * T.x + p.y * T.y);
    if (!(gp > 0)) return false;
    const double ds = g / gp;
    s -= ds;
    if (std::fabs(ds) < 1e-6) break;
  }
  if (!(s > 0)) return false;
  V3 p, T;
  H.at(s, p, T);
  if (std::fabs(std::sqrt(p.x * p.x + p.y * p.y) - R) > 1e-3) return false;
  s_out = s;
  return true;
}

// Smallest positive path to the plane z = Z (Newton from the straight line).
bool cross_zplane(const Helix& H, double Z, double& s_out) {
  if (std::fabs(H.T0.z) < 1e-12) return false;
  double s = (Z - H.p0.z) / H.T0.z;
  if (!(s > 0)) return false;
  for (int it = 0; it < 20; ++it) {
    V3 p, T;
    H.at(s, p, T);
    if (std::fabs(T.z) < 1e-12) return false;
    const double ds = (p.z - Z) / T.z;
    s -= ds;
    if (std::fabs(ds) < 1e-6) break;
  }
  if (!(s > 0)) return false;
  s_out = s;
  return true;
}

struct Listed {
  double s;
  int id;
};

// The listing test of one module m from the trajectory point P (path
// s_base from the current state, direction T, curvature k): the second-order
// expansion P + d T + d^2 k / 2 meets its plane within the half lengths plus
// nav_margin at a positive total path.
void list_test(const Geometry& G, const Cfg& cfg, int m, V3 P, V3 T, V3 k, double s_base,
               std::vector<Listed>& cand, Stats& st) {
  const Surface& S = G.s[m];
  const double half_diag = std::sqrt((S.hw0 + cfg.nav_margin) * (S.hw0 + cfg.nav_margin) +
                                     (S.hw1 + cfg.nav_margin) * (S.hw1 + cfg.nav_margin));
  if (norm(S.c - P) > half_diag + kReach) return;
  ++st.nav_modules;
  const double a = 0.5 * dot(S.n, k), b = dot(S.n, T), c0 = dot(S.n, P - S.c);
  if (std::fabs(b) < 1e-3) return;
  double d = -c0 / b;
  const double disc = b * b - 4.0 * a * c0;
  if (disc >= 0) {
    const double q = -0.5 * (b + std::copysign(std::sqrt(disc), b));
    if (q != 0) d = c0 / q;
  }
  const V3 Q = P + d * T + (0.5 * d * d) * k;
  const double l0 = dot(S.u, Q - S.c), l1 = dot(S.v, Q - S.c);
  if (std::fabs(l0) > S.hw0 + cfg.nav_margin || std::fabs(l1) > S.hw1 + cfg.nav_margin) return;
  if (!(s_base + d > 0)) return;
  cand.push_back({s_base + d, m});
}

// The listed modules in path order (ties by id), at most 4.
void list_sorted(std::vector<Listed>& cand, std::vector<int>& list) {
  std::sort(cand.begin(), cand.end(), [](const Listed& x, const Listed& y) {
    return x.s < y.s || (x.s == y.s && x.id < y.id);
  });
  list.clear();
  for (size_t i = 0; i < cand.size() && (int)i < kMaxList; ++i) list.push_back(cand[i].id);
}

// Modules of `layer` that pass the listing test, in path order (at most 4).
void list_layer(const Geometry& G, const Cfg& cfg, int layer, V3 P, V3 T, V3 k, double s_base, int exclude,
                std::vector<int>& list, Stats& st) {
  std::vector<Listed> cand;
  for (int m : G.members[layer]) {
    if (m == exclude) continue;
    list_test(G, cfg, m, P, T, k, s_base, cand, st);
  }
  list_sorted(cand, list);
}

// ---------------------------------------------------------------------------
// The learned next-module proposal.  It is not in the paper: it replaces only
// the module lookup of the navigation (section 2, intersected modules) and
// keeps that lookup as its fallback.  Readings:
//   table    per module m, up to three next layers L', each with an anchor A
//            on L''s envelope, the module pitches (pu, pv) of L' there and a
//            region of 24 x 8 cells iu in [-12, 11], iv in [-4, 3] around A
//            holding module ids (an input here, built from the geometry by
//            the Python side of the oracle);
//   window   the navigation's own crossing X of L''s envelope, in the layer's
//            curvilinear coordinates around A - (R dphi, dz) on a barrel of
//            radius R, (r dphi, dr) on a disk with r the radius of X - divided
//            by the pitches; the rounded cell (floor(q + 1/2)) is the centre
//            of an 8 x 4 window iu in [-4, 3], iv in [-2, 1], outputs in
//            order (iv, iu); no window when |q| >= 1000;
//   input    X's fractional position in its cell (2), the direction at X in
//            the layer frame (phi-hat, then z-hat and r-hat on barrels, r-hat
//            and z-hat on disks), q/p, L' / number of layers;
//   network  7 -> 64 -> 64 -> 32 with ReLU; in the bfloat16 reading the
//            weights, the input and both hidden activations are rounded to
//            bfloat16 (through FP32, nearest, ties to even), sums and biases
//            stay wide;
//   use      softmax over the 32 outputs; the top k (probability descending,
//            index ascending) are summed; at or above min_prob their modules
//            (empty cells skipped) go through the listing test; when none
//            passes, or the sum is lower, the geometric lookup runs.
constexpr int kNIn = 7, kNH = 64, kNOut = 32;
constexpr int kMaxNext = 3;
constexpr int kWinU = 8, kWinV = 4, kWU0 = -4, kWV0 = -2;
constexpr int kRegU = 24, kRegV = 8, kRU0 = -12, kRV0 = -4, kRegCells = kRegU * kRegV;

// Causes by which a decision of the oracle can legitimately differ from one
// taken in FP32 with FP32 matrix-core sums (reported per seed, never used to
// decide anything):
constexpr int kNearConf = 1;  // summed probability within kConfEps of min_prob
constexpr int kNearBf16 = 2;  // one value near a bfloat16 rounding boundary decides the outcome
constexpr int kNearEdge = 4;  // crossing near a cell edge, and the neighbouring window decides otherwise
constexpr int kNearRank = 8;  // k-th and (k+1)-th probabilities within kConfEps (proposed set ambiguous)
constexpr double kConfEps = 1e-4;
constexpr double kEdgeEps = 5e-5;  // cell units
// how far an FP32 evaluation's network input can sit from the FP64 one:
// cell fractions, direction components, and q/p (relative)
constexpr double kInEps[kNIn] = {5e-5, 5e-5, 5e-6, 5e-6, 5e-6, 0.0, 1e-7};
constexpr double kQopRel = 1e-6;
constexpr double kSumRel = 1e-6;   // hidden pre-activations: relative to the sum of |terms|

double bf16_round(double v) {
  float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  u &= 0xffff0000u;
  std::memcpy(&f, &u, 4);
  return f;
}

struct Net {
  double W1[kNH][kNIn], b1[kNH], W2[kNH][kNH], b2[kNH], W3[kNOut][kNH], b3[kNOut];
};

Net load_net(const float* p, bool round) {
  Net n;
  auto w = [&](double v) { return round ? bf16_round(v) : v; };
  int o = 0;
  for (int i = 0; i < kNH; ++i)
    for (int j = 0; j < kNIn; ++j) n.W1[i][j] = w(p[o++]);
  for (int i = 0; i < kNH; ++i) n.b1[i] = p[o++];
  for (int i = 0; i < kNH; ++i)
    for (int j = 0; j < kNH; ++j) n.W2[i][j] = w(p[o++]);
  for (int i = 0; i < kNH; ++i) n.b2[i] = p[o++];
  for (int i = 0; i < kNOut; ++i)
    for (int j = 0; j < kNH; ++j) n.W3[i][j] = w(p[o++]);
  for (int i = 0; i < kNOut; ++i) n.b3[i] = p[o++];
  return n;
}

struct Learned {
  const int32_t* next;
  const int32_t* region;
  const double* anchor;
  Net net;
  double min_prob;
  int topk;
  bool bf16;
};

// Activations of one evaluation: pre-activations z, the sums of |terms|, and
// the (rounded) outputs h of the hidden layers.
struct Pass {
  double x[kNIn];
  double z1[kNH], a1[kNH], h1[kNH];
  double z2[kNH], a2[kNH], h2[kNH];
  double z3[kNOut];
};

double act(const Learned& L, double z) {
  const double r = z > 0 ? z : 0.0;
  return L.bf16 ? bf16_round(r) : r;
}

void layer2(const Learned& L, Pass& e) {
  for (int i = 0; i < kNH; ++i) {
    double z = 0, a = 0;
    for (int j = 0; j < kNH; ++j) {
      z += L.net.W2[i][j] * e.h1[j];
      a += std::fabs(L.net.W2[i][j] * e.h1[j]);
    }
    e.z2[i] = z + L.net.b2[i];
    e.a2[i] = a + std::fabs(L.net.b2[i]);
    e.h2[i] = act(L, e.z2[i]);
  }
}

void layer3(const Learned& L, Pass& e) {
  for (int i = 0; i < kNOut; ++i) {
    double z = 0;
    for (int j = 0; j < kNH; ++j) z += L.net.W3[i][j] * e.h2[j];
    e.z3[i] = z + L.net.b3[i];
  }
}

// Forward pass from the (already rounded) input e.x.
void forward(const Learned& L, Pass& e) {
  for (int i = 0; i < kNH; ++i) {
    double z = 0, a = 0;
    for (int j = 0; j < kNIn; ++j) {
      z += L.net.W1[i][j] * e.x[j];
      a += std::fabs(L.net.W1[i][j] * e.x[j]);
    }
    e.z1[i] = z + L.net.b1[i];
    e.a1[i] = a + std::fabs(L.net.b1[i]);
    e.h1[i] = act(L, e.z1[i]);
  }
  layer2(L, e);
  layer3(L, e);
}

// Softmax and the top k (probability descending, index ascending).
struct Ranked {
  int cls[kNOut];
  double p[kNOut];  // probabilities in ranked order
  double conf;
};

Ranked rank_outputs(const Learned& L, const double* z) {
  Ranked r;
  double mx = z[0];
  for (int i = 1; i < kNOut; ++i) mx = std::max(mx, z[i]);
  double e[kNOut], sum = 0;
  for (int i = 0; i < kNOut; ++i) {
    e[i] = std::exp(z[i] - mx);
    sum += e[i];
  }
  for (int i = 0; i < kNOut; ++i) r.cls[i] = i;
  std::stable_sort(r.cls, r.cls + kNOut, [&](int a, int b) { return e[a] > e[b]; });
  for (int i = 0; i < kNOut; ++i) r.p[i] = e[r.cls[i]] / sum;
  r.conf = 0;
  for (int i = 0; i < L.topk; ++i) r.conf += r.p[i];
  return r;
}

struct Window {
  int iu, iv;
  double fu, fv;
};

double wrap_pm_pi(double a) {  // into [-pi, pi)
  double w = std::fmod(a + kPi, 2 * kPi);
  if (w < 0) w += 2 * kPi;
  return w - kPi;
}

// The window cell of a crossing X of layer Lr for the anchor row anc
// (A x, y, z, pitch u, pitch v); false for a non-finite or far crossing.
bool window_of(const Layer& Lr, const double* anc, V3 X, Window& w, double& qu, double& qv) {
  const double dphi = wrap_pm_pi(std::atan2(X.y, X.x) - std::atan2(anc[1], anc[0]));
  const double rX = std::hypot(X.x, X.y);
  double du, dv;
  if (Lr.type == 0) {
    du = dphi * Lr.pos;
    dv = X.z - anc[2];
  } else {
    du = dphi * rX;
    dv = rX - std::hypot(anc[0], anc[1]);
  }
  qu = du / anc[3];
  qv = dv / anc[4];
  if (!(std::fabs(qu) < 1000.0 && std::fabs(qv) < 1000.0)) return false;
  const double cu = std::floor(qu + 0.5), cv = std::floor(qv + 0.5);
  w.iu = (int)cu;
  w.iv = (int)cv;
  w.fu = qu - cu;
  w.fv = qv - cv;
  return true;
}

// The network input at the crossing (unrounded).
void features(const Layer& Lr, int layer, int n_layers, const Window& w, V3 X, V3 T, double qop, double* x) {
  const double r = std::hypot(X.x, X.y);
  const V3 ph{-X.y / r, X.x / r, 0.0}, rh{X.x / r, X.y / r, 0.0};
  x[0] = w.fu;
  x[1] = w.fv;
  x[2] = dot(T, ph);
  x[3] = Lr.type == 0 ? T.z : dot(T, rh);
  x[4] = Lr.type == 0 ? dot(T, rh) : T.z;
  x[5] = qop;
  x[6] = (double)layer / (double)n_layers;
}

// Module id of window output c (empty cell or outside the region: -1).
int window_module(const int32_t* region, const Window& w, int c) {
  const int cu = w.iu + kWU0 + c % kWinU, cv = w.iv + kWV0 + c / kWinU;
  if (cu < kRU0 || cu >= kRU0 + kRegU || cv < kRV0 || cv >= kRV0 + kRegV) return -1;
  return region[(cv - kRV0) * kRegU + (cu - kRU0)];
}

// The outcome of a proposal: not confident, or the modules of the top k.
struct Decision {
  bool confident = false;
  std::vector<int> mods;  // in rank order, empty cells skipped
  bool operator==(const Decision& o) const {
    if (confident != o.confident) return false;
    if (!confident) return true;
    std::vector<int> a = mods, b = o.mods;
    std::sort(a.begin(), a.end());
    std::sort(b.begin(), b.end());
    return a == b;
  }
};

Decision decide(const Learned& L, const Pass& e, const int32_t* region, const Window& w, Ranked* out = nullptr) {
  const Ranked r = rank_outputs(L, e.z3);
  Decision d;
  d.confident = r.conf >= L.min_prob;
  if (d.confident)
    for (int i = 0; i < L.topk; ++i) {
      const int m = window_module(region, w, r.cls[i]);
      if (m >= 0) d.mods.push_back(m);
    }
  if (out) *out = r;
  return d;
}

// Network evaluation at a crossing: the decision, and (near != nullptr) the
// causes that could make an FP32 evaluation decide otherwise.
Decision evaluate(const Geometry& G, const Learned& L, int layer, const int32_t* region, const Window& w, V3 X,
                  V3 T, double qop, int* near, Ranked* ranked) {
  const Layer& Lr = G.layers[layer];
  double xr[kNIn];
  features(Lr, layer, (int)G.layers.size(), w, X, T, qop, xr);
  Pass e;
  for (int i = 0; i < kNIn; ++i) e.x[i] = L.bf16 ? bf16_round(xr[i]) : xr[i];
  forward(L, e);
  Ranked r;
  const Decision d = decide(L, e, region, w, &r);
  if (ranked) *ranked = r;
  if (!near) return d;
  if (std::fabs(r.conf - L.min_prob) < kConfEps) *near |= kNearConf;
  if (d.confident && r.p[L.topk - 1] - r.p[L.topk] < kConfEps) *near |= kNearRank;
  if (!L.bf16) return d;
  // one rounding at a time the other way: inputs, then hidden activations
  for (int i = 0; i < kNIn; ++i) {
    const double m = i == 5 ? kQopRel * std::fabs(xr[i]) : kInEps[i] * (i == 6 ? std::fabs(xr[i]) : 1.0);
    for (double v : {xr[i] - m, xr[i] + m}) {
      const double alt = bf16_round(v);
      if (alt == e.x[i]) continue;
      Pass f = e;
      f.x[i] = alt;
      forward(L, f);
      if (!(decide(L, f, region, w) == d)) *near |= kNearBf16;
    }
  }
  for (int j = 0; j < kNH; ++j) {
    const double m = kSumRel * e.a1[j];
    for (double v : {e.z1[j] - m, e.z1[j] + m}) {
      const double alt = act(L, v);
      if (alt == e.h1[j]) continue;
      Pass f = e;
      f.h1[j] = alt;
      layer2(L, f);
      layer3(L, f);
      if (!(decide(L, f, region, w) == d)) *near |= kNearBf16;
    }
  }
  for (int j = 0; j < kNH; ++j) {
    const double m = kSumRel * e.a2[j];
    for (double v : {e.z2[j] - m, e.z2[j] + m}) {
      const double alt = act(L, v);
      if (alt == e.h2[j]) continue;
      Pass f = e;
      f.h2[j] = alt;
      layer3(L, f);
      if (!(decide(L, f, region, w) == d)) *near |= kNearBf16;
    }
  }
  return d;
}

// The proposal for a navigation from module m to layer `layer`, crossing its
// envelope at X with direction T.  Returns false when the layer has no row
// in m's table or the crossing has no window (the network does not run).
bool propose(const Geometry& G, const Learned& L, int m, int layer, V3 X, V3 T, double qop, Decision& d,
             int* near, Stats& st) {
  int slot = -1;
  for (int q = 0; q < kMaxNext; ++q)
    if (slot < 0 && L.next[m * kMaxNext + q] == layer) slot = q;
  if (slot < 0) return false;
  const double* anc = L.anchor + ((size_t)m * kMaxNext + slot) * 5;
  const int32_t* region = L.region + ((size_t)m * kMaxNext + slot) * kRegCells;
  Window w;
  double qu, qv;
  if (!window_of(G.layers[layer], anc, X, w, qu, qv)) return false;
  ++st.mlp_rows;
  d = evaluate(G, L, layer, region, w, X, T, qop, near, nullptr);
  if (near && (0.5 - std::fabs(w.fu) < kEdgeEps || 0.5 - std::fabs(w.fv) < kEdgeEps)) {
    // the neighbouring centre cell an FP32 crossing could round to
    Window w2 = w;
    if (0.5 - std::fabs(w.fu) < kEdgeEps) {
      const int s = w.fu > 0 ? 1 : -1;
      w2.iu += s;
      w2.fu -= s;
    }
    if (0.5 - std::fabs(w.fv) < kEdgeEps) {
      const int s = w.fv > 0 ? 1 : -1;
      w2.iv += s;
      w2.fv -= s;
    }
    if (!(evaluate(G, L, layer, region, w2, X, T, qop, nullptr, nullptr) == d)) *near |= kNearEdge;
  }
  return true;
}

// Per-seed record of the learned navigation: causes of possible FP32
// disagreement, and whether a used proposal listed differently from the
// geometric lookup (then the seed may differ from the plain search).
struct LearnedTrace {
  int near = 0;
  bool differs = false;
};

// The next layer and its listed modules.  Returns the layer or -1.
int navigate(const Geometry& G, const Field& F, const Cfg& cfg, const Free& f, uint64_t mask,
             double path, std::vector<int>& list, Stats& st, const Learned* lrn = nullptr, int surface = -1,
             LearnedTrace* trace = nullptr) {
  ++st.navigations;
  const Helix H(f, F.at(f.r));
  const double rperp = std::sqrt(f.r.x * f.r.x + f.r.y * f.r.y);
  int best = -1;
  double sbest = INFINITY;
  for (int l = 0; l < (int)G.layers.size(); ++l) {
    if (mask & (uint64_t(1) << l)) continue;
    const Layer& L = G.layers[l];
    double s;
    V3 p, T;
    if (L.type == 0) {
      if (!(L.pos > rperp)) continue;
      if (!cross_cylinder(H, L.pos, s)) continue;
      H.at(s, p, T);
      if (p.z < L.lo || p.z > L.hi) continue;
    } else {
      if (!cross_zplane(H, L.pos, s)) continue;
      H.at(s, p, T);
      const double r = std::sqrt(p.x * p.x + p.y * p.y);
      if (r < L.lo || r > L.hi) continue;
    }
    if (path + s > cfg.path_max) continue;
    if (s < sbest) {
      sbest = s;
      best = l;
    }
  }
  list.clear();
  if (best < 0) return -1;
  V3 P, T;
  H.at(sbest, P, T);
  const V3 kk = (kKappa * f.qop) * cross(T, H.B);
  if (lrn && surface >= 0) {
    Decision d;
    if (propose(G, *lrn, surface, best, P, T, f.qop, d, trace ? &trace->near : nullptr, st) && d.confident) {
      std::vector<Listed> cand;
      for (int m : d.mods) list_test(G, cfg, m, P, T, kk, sbest, cand, st);
      list_sorted(cand, list);
      if (!list.empty()) {
        ++st.proposals;
        if (trace) {  // audit against the geometric lookup
          Stats scratch;
          std::vector<int> full;
          list_layer(G, cfg, best, P, T, kk, sbest, -1, full, scratch);
          if (full != list) {
            ++st.proposal_misses;
            trace->differs = true;
          }
        }
        return best;
      }
    }
  }
  list_layer(G, cfg, best, P, T, kk, sbest, -1, list, st);
  return best;
}

// ---------------------------------------------------------------------------
// The combinatorial Kalman filter.

struct Cand {
  int surface;
  double p[5];
  M5 C;
  int n_meas = 0, holes = 0;
  double chi2 = 0;
  std::vector<int> ids;
  std::vector<int> id_surface;              // module of each measurement
  std::vector<std::array<double, 5>> id_p;  // filtered parameters after each measurement
  int snap_surface = -1;
  double snap_p[5] = {0, 0, 0, 0, 0};
  M5 snap_C{};
  uint64_t mask = 0;
  std::vector<int> list;
  double h_trial = 0, path = 0;
  bool root = true;
};

// Rank key: more measurements, then smaller chi2 sum, fewer holes, then the
// measurement-id sequence in lexicographic order.  A total order on the
// distinct branches of one seed.
bool better(const Cand& a, const Cand& b) {
  if (a.n_meas != b.n_meas) return a.n_meas > b.n_meas;
  if (a.chi2 != b.chi2) return a.chi2 < b.chi2;
  if (a.holes != b.holes) return a.holes < b.holes;
  return std::lexicographical_compare(a.ids.begin(), a.ids.end(), b.ids.begin(), b.ids.end());
}

struct Event {
  const orc_measurements* m;
};

struct Accepted {
  double chi2;
  int id;
};

// One step of one candidate: search here if it is a fresh seed; otherwise
// navigate if its list is empty and visit the next listed module.  Surviving
// candidates go to `outs`, terminated ones to `fin`.
void step_candidate(const Geometry& G, const Field& F, const Cfg& cfg, const orc_measurements* M,
                    int event, Cand c, std::vector<Cand>& outs, std::vector<Cand>& fin, Stats& st,
                    const Learned* lrn, LearnedTrace* trace) {
  ++st.steps;
  if (c.root) {
    c.root = false;
  } else {
    if (c.list.empty()) {
      const Free f = bound_to_free(G.s[c.surface], c.p);
      const int L = navigate(G, F, cfg, f, c.mask, c.path, c.list, st, lrn, c.surface, trace);
      if (L < 0) {
        fin.push_back(std::move(c));
        return;
      }
      c.mask |= uint64_t(1) << L;
      if (c.list.empty()) {  // the layer is crossed in a gap
        outs.push_back(std::move(c));
        return;
      }
    }
    const int m = c.list.front();
    c.list.erase(c.list.begin());
    double po[5];
    M5 Co;
    if (!propagate(G, F, cfg, c.surface, c.p, c.C, m, po, Co, nullptr, c.h_trial, c.path, st)) return;
    c.surface = m;
    std::memcpy(c.p, po, sizeof po);
    c.C = Co;
    const Surface& S = G.s[m];
    if (!(std::fabs(c.p[0]) <= S.hw0 && std::fabs(c.p[1]) <= S.hw1)) {
      outs.push_back(std::move(c));  // listed but not crossed
      return;
    }
  }
  ++st.crossed;
  const Surface& S = G.s[c.surface];
  const int row = event * M->n_surfaces + c.surface;
  std::vector<Accepted> acc;
  for (int i = M->offsets[row]; i < M->offsets[row + 1]; ++i) {
    ++st.chi2_evals;
    const double x2 = chi2_of(c.p, c.C, M->loc[2 * i], M->loc[2 * i + 1], M->var[2 * i], M->var[2 * i + 1]);
    if (x2 < cfg.chi2_max) acc.push_back({x2, i});
  }
  std::sort(acc.begin(), acc.end(), [](const Accepted& a, const Accepted& b) {
    return a.chi2 < b.chi2 || (a.chi2 == b.chi2 && a.id < b.id);
  });
  if (cfg.branches > 0 && (int)acc.size() > cfg.branches) acc.resize(cfg.branches);
  if (acc.empty()) {
    ++st.holes;
    ++c.holes;
    if (cfg.material) {
      apply_ms(S, cfg.mass, c.p, c.C);
      ++st.ms_updates;
    }
    if (c.holes > cfg.max_holes)
      fin.push_back(std::move(c));
    else
      outs.push_back(std::move(c));
    return;
  }
  for (const Accepted& a : acc) {
    Cand ch = c;
    const int i = a.id;
    double po[5];
    M5 Co;
    kf_update(c.p, c.C, M->loc[2 * i], M->loc[2 * i + 1], M->var[2 * i], M->var[2 * i + 1], po, Co);
    ++st.kf_updates;
    std::memcpy(ch.p, po, sizeof po);
    ch.C = Co;
    ch.n_meas += 1;
    ch.chi2 += a.chi2;
    ch.ids.push_back(i);
    ch.id_surface.push_back(ch.surface);
    ch.id_p.push_back({po[0], po[1], po[2], po[3], po[4]});
    ch.snap_surface = ch.surface;
    std::memcpy(ch.snap_p, ch.p, sizeof ch.p);
    ch.snap_C = ch.C;
    if (cfg.material) {
      apply_ms(S, cfg.mass, ch.p, ch.C);
      ++st.ms_updates;
    }
    outs.push_back(std::move(ch));
  }
}

struct SeedResult {
  std::vector<Cand> tracks;  // best first
};

void find_seed(const Geometry& G, const Field& F, const Cfg& cfg, const orc_measurements* M,
               const orc_seeds* S, int k, SeedResult& res, Stats& st, const Learned* lrn = nullptr,
               LearnedTrace* trace = nullptr) {
  Cand root;
  root.surface = S->surface[k];
  std::memcpy(root.p, S->params + 5 * k, sizeof root.p);
  root.C = unpack(S->cov + 15 * k);
  root.mask = uint64_t(1) << G.s[root.surface].layer;
  root.h_trial = cfg.step_max;
  {  // overlapping modules of the seed's own layer still ahead of the seed
    const Free f = bound_to_free(G.s[root.surface], root.p);
    const V3 kk = (kKappa * f.qop) * cross(f.T, F.at(f.r));
    list_layer(G, cfg, G.s[root.surface].layer, f.r, f.T, kk, 0.0, root.surface, root.list, st);
  }
  const int event = S->event[k];
  std::vector<Cand> live{root}, finished;
  auto consider = [&](Cand& c) {
    ++st.finished;
    if (c.n_meas >= cfg.min_meas) finished.push_back(std::move(c));
  };
  for (int step = 0; step < cfg.max_steps && !live.empty(); ++step) {
    std::vector<Cand> outs, fin;
    for (Cand& c : live) step_candidate(G, F, cfg, M, event, std::move(c), outs, fin, st, lrn, trace);
    for (Cand& c : fin) consider(c);
    if (cfg.max_live > 0 && (int)outs.size() > cfg.max_live) {
      std::sort(outs.begin(), outs.end(), better);
      st.pruned += outs.size() - cfg.max_live;
      outs.resize(cfg.max_live);
    }
    live = std::move(outs);
  }
  for (Cand& c : live) consider(c);
  std::sort(finished.begin(), finished.end(), better);
  if (cfg.tracks_per_seed > 0 && (int)finished.size() > cfg.tracks_per_seed)
    finished.resize(cfg.tracks_per_seed);
  res.tracks = std::move(finished);
}

void to_stats(const Stats& s, orc_stats* o) {
  if (!o) return;
  o->steps = s.steps; o->navigations = s.navigations; o->nav_modules = s.nav_modules;
  o->legs = s.legs; o->legs_failed = s.legs_failed; o->rk_trials = s.rk_trials;
  o->rk_rejects = s.rk_rejects; o->chi2_evals = s.chi2_evals; o->kf_updates = s.kf_updates;
  o->ms_updates = s.ms_updates; o->crossed = s.crossed; o->holes = s.holes;
  o->pruned = s.pruned; o->finished = s.finished;
  o->mlp_rows = s.mlp_rows; o->proposals = s.proposals; o->proposal_misses = s.proposal_misses;
}

// Track finding for every seed, plain (lrn == nullptr) or with the learned
// proposal; traces (learned form only) are per seed.
int find_all(const orc_geometry* g, const orc_field* f, const orc_measurements* m, const orc_seeds* s,
             const orc_config* c, const Learned* lrn, int n_threads, orc_tracks* out, orc_stats* stats,
             int32_t* seed_near, int32_t* seed_differs) {
  if (!g || !f || !m || !s || !c || !out) return ORC_ERR_ARG;
  if (g->n_layers > 64 || m->n_surfaces != g->n_surfaces) return ORC_ERR_ARG;
  const Geometry G = load_geometry(g);
  const Field F = load_field(f);
  const Cfg cfg = load_cfg(c);
  const int n = s->n_seeds;
  std::vector<SeedResult> res(n);
  std::vector<LearnedTrace> traces(lrn ? n : 0);
  if (n_threads <= 0) n_threads = (int)std::max(1u, std::thread::hardware_concurrency());
  n_threads = std::max(1, std::min(n_threads, std::max(1, n)));
  std::vector<Stats> tstats(n_threads);
  std::atomic<int> next(0);
  auto work = [&](int t) {
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= n) break;
      find_seed(G, F, cfg, m, s, k, res[k], tstats[t], lrn, lrn ? &traces[k] : nullptr);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < n_threads; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto& th : pool) th.join();
  Stats total;
  for (auto& ts : tstats) total.add(ts);
  to_stats(total, stats);
  for (int k = 0; k < (lrn ? n : 0); ++k) {
    if (seed_near) seed_near[k] = traces[k].near;
    if (seed_differs) seed_differs[k] = traces[k].differs ? 1 : 0;
  }
  // Assemble the output in seed order.
  int nt = 0, nm = 0;
  for (int k = 0; k < n; ++k)
    for (const Cand& t : res[k].tracks) {
      ++nt;
      nm += (int)t.ids.size();
    }
  out->n_tracks = nt;
  out->n_meas_total = nm;
  if (nt > out->cap_tracks || nm > out->cap_meas) return ORC_ERR_CAPACITY;
  int it = 0, im = 0;
  out->offsets[0] = 0;
  for (int k = 0; k < n; ++k)
    for (const Cand& t : res[k].tracks) {
      for (size_t q = 0; q < t.ids.size(); ++q) {
        if (out->meas_surface) out->meas_surface[im] = t.id_surface[q];
        if (out->meas_params) std::memcpy(out->meas_params + 5 * im, t.id_p[q].data(), 5 * sizeof(double));
        out->meas[im++] = t.ids[q];
      }
      out->offsets[it + 1] = im;
      std::memcpy(out->params + 5 * it, t.snap_p, 5 * sizeof(double));
      pack(t.snap_C, out->cov + 15 * it);
      out->chi2[it] = t.chi2;
      out->ndf[it] = 2 * t.n_meas - 5;
      out->holes[it] = t.holes;
      out->seed[it] = k;
      out->event[it] = s->event[k];
      out->last_surface[it] = t.snap_surface;
      ++it;
    }
  return ORC_OK;
}

bool load_learned(const orc_geometry* g, const orc_learned* l, Learned& L) {
  if (!l || !l->next || !l->region || !l->anchor || !l->params) return false;
  if (l->topk < 1 || l->topk > 3) return false;
  L.next = l->next;
  L.region = l->region;
  L.anchor = l->anchor;
  L.bf16 = l->bf16 != 0;
  L.net = load_net(l->params, L.bf16);
  L.min_prob = l->min_prob;
  L.topk = l->topk;
  (void)g;
  return true;
}

}  // namespace

extern "C" int orc_field_eval(const orc_field* f, int32_t n, const double* p, double* B, double* G) {
  if (!f || !p || !B || n < 0) return ORC_ERR_ARG;
  const Field F = load_field(f);
  for (int i = 0; i < n; ++i) {
    V3 b;
    double g[3][3];
    F.eval({p[3 * i], p[3 * i + 1], p[3 * i + 2]}, b, g, G != nullptr);
    B[3 * i] = b.x;
    B[3 * i + 1] = b.y;
    B[3 * i + 2] = b.z;
    if (G)
      for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) G[9 * i + 3 * a + c] = g[a][c];
  }
  return ORC_OK;
}

extern "C" int orc_ckf_find(const orc_geometry* g, const orc_field* f, const orc_measurements* m,
                            const orc_seeds* s, const orc_config* c, int n_threads, orc_tracks* out,
                            orc_stats* stats) {
  return find_all(g, f, m, s, c, nullptr, n_threads, out, stats, nullptr, nullptr);
}

extern "C" int orc_ckf_find_learned(const orc_geometry* g, const orc_field* f, const orc_measurements* m,
                                    const orc_seeds* s, const orc_config* c, const orc_learned* l,
                                    int n_threads, orc_tracks* out, orc_stats* stats, int32_t* seed_near,
                                    int32_t* seed_differs) {
  Learned L;
  if (!load_learned(g, l, L)) return ORC_ERR_ARG;
  if (f && f->map) return ORC_ERR_ARG;  // the proposal is defined in the uniform field
  return find_all(g, f, m, s, c, &L, n_threads, out, stats, seed_near, seed_differs);
}

extern "C" int orc_mlp_forward(const float* params, int32_t bf16, int64_t n, const double* x, double* logits) {
  if (!params || n < 0 || (n > 0 && (!x || !logits))) return ORC_ERR_ARG;
  Learned L;
  L.bf16 = bf16 != 0;
  L.net = load_net(params, L.bf16);
  for (int64_t r = 0; r < n; ++r) {
    Pass e;
    for (int i = 0; i < kNIn; ++i) e.x[i] = L.bf16 ? bf16_round(x[r * kNIn + i]) : x[r * kNIn + i];
    forward(L, e);
    for (int i = 0; i < kNOut; ++i) logits[r * kNOut + i] = e.z3[i];
  }
  return ORC_OK;
}

extern "C" int orc_learned_propose(const orc_geometry* g, const orc_learned* l, int32_t surface, int32_t layer,
                                   const double* X, const double* T, double qop, int32_t* cell, double* feat,
                                   double* conf, int32_t* classes, int32_t* modules, int32_t* near) {
  Learned L;
  if (!g || !X || !T || !cell || !feat || !conf || !classes || !modules || !near) return ORC_ERR_ARG;
  if (!load_learned(g, l, L)) return ORC_ERR_ARG;
  if (surface < 0 || surface >= g->n_surfaces || layer < 0 || layer >= g->n_layers) return ORC_ERR_ARG;
  const Geometry G = load_geometry(g);
  int slot = -1;
  for (int q = 0; q < kMaxNext; ++q)
    if (slot < 0 && L.next[surface * kMaxNext + q] == layer) slot = q;
  if (slot < 0) return -1;
  const double* anc = L.anchor + ((size_t)surface * kMaxNext + slot) * 5;
  const int32_t* region = L.region + ((size_t)surface * kMaxNext + slot) * kRegCells;
  Window w;
  double qu, qv;
  const V3 Xv{X[0], X[1], X[2]}, Tv{T[0], T[1], T[2]};
  if (!window_of(G.layers[layer], anc, Xv, w, qu, qv)) return -1;
  cell[0] = w.iu;
  cell[1] = w.iv;
  features(G.layers[layer], layer, (int)G.layers.size(), w, Xv, Tv, qop, feat);
  Ranked r;
  int nr = 0;
  const Decision d = evaluate(G, L, layer, region, w, Xv, Tv, qop, &nr, &r);
  *near = nr;
  *conf = r.conf;
  for (int i = 0; i < 3; ++i) {
    classes[i] = r.cls[i];
    modules[i] = i < L.topk ? window_module(region, w, r.cls[i]) : -1;
  }
  return d.confident ? 1 : 0;
}

extern "C" int orc_propagate(const orc_geometry* g, const orc_field* f, const orc_config* c, int32_t src,
                             const double* p_in, const double* cov_in, int32_t dst, double* p_out,
                             double* cov_out, double* jac, double* path) {
  if (!g || !f || !c || !p_in || !cov_in || !p_out || !cov_out) return ORC_ERR_ARG;
  if (src < 0 || dst < 0 || src >= g->n_surfaces || dst >= g->n_surfaces) return ORC_ERR_ARG;
  const Geometry G = load_geometry(g);
  const Field F = load_field(f);
  const Cfg cfg = load_cfg(c);
  Stats st;
  M5 Co, J;
  double h = cfg.step_max, s = 0;
  if (!propagate(G, F, cfg, src, p_in, unpack(cov_in), dst, p_out, Co, &J, h, s, st)) return ORC_ERR_FAILED;
  pack(Co, cov_out);
  if (jac) std::memcpy(jac, J.data(), 25 * sizeof(double));
  if (path) *path = s;
  return ORC_OK;
}

extern "C" int orc_propagate_free(const orc_field* f, const orc_config* c, const double* fin,
                                  const double* cc, const double* nn, double* fout, double* path) {
  if (!f || !c || !fin || !cc || !nn || !fout) return ORC_ERR_ARG;
  const Field F = load_field(f);
  const Cfg cfg = load_cfg(c);
  Stats st;
  Free fr{{fin[0], fin[1], fin[2]}, {fin[3], fin[4], fin[5]}, fin[6]};
  Tangents J{};
  double h = cfg.step_max, s = 0;
  if (!land(F, cfg, {cc[0], cc[1], cc[2]}, {nn[0], nn[1], nn[2]}, fr, J, h, s, st)) return ORC_ERR_FAILED;
  const double o[7] = {fr.r.x, fr.r.y, fr.r.z, fr.T.x, fr.T.y, fr.T.z, fr.qop};
  std::memcpy(fout, o, sizeof o);
  if (path) *path = s;
  return ORC_OK;
}

extern "C" int orc_kf_update(const double* p_in, const double* cov_in, const double* meas,
                             const double* var, double* p_out, double* cov_out, double* chi2) {
  if (!p_in || !cov_in || !meas || !var || !p_out || !cov_out) return ORC_ERR_ARG;
  M5 Co;
  const double x2 = kf_update(p_in, unpack(cov_in), meas[0], meas[1], var[0], var[1], p_out, Co);
  pack(Co, cov_out);
  if (chi2) *chi2 = x2;
  return ORC_OK;
}

extern "C" int orc_trace(const orc_geometry* g, const orc_field* f, const orc_config* c, int32_t surface,
                         const double* params, int32_t cap, int32_t* visited, int32_t* crossed,
                         double* params_out) {
  if (!g || !f || !c || !params || !visited || !crossed) return -1;
  const Geometry G = load_geometry(g);
  const Field F = load_field(f);
  const Cfg cfg = load_cfg(c);
  Stats st;
  int cur = surface;
  double p[5];
  std::memcpy(p, params, sizeof p);
  M5 C{};
  for (int i = 0; i < 5; ++i) C[6 * i] = 1e-6;
  uint64_t mask = uint64_t(1) << G.s[cur].layer;
  std::vector<int> list;
  {
    const Free f0 = bound_to_free(G.s[cur], p);
    list_layer(G, cfg, G.s[cur].layer, f0.r, f0.T, (kKappa * f0.qop) * cross(f0.T, F.at(f0.r)), 0.0, cur,
               list, st);
  }
  double h = cfg.step_max, path = 0;
  int n = 0;
  for (int step = 0; step < cfg.max_steps && n < cap; ++step) {
    if (list.empty()) {
      const int L = navigate(G, F, cfg, bound_to_free(G.s[cur], p), mask, path, list, st);
      if (L < 0) break;
      mask |= uint64_t(1) << L;
      if (list.empty()) continue;
    }
    const int m = list.front();
    list.erase(list.begin());
    double po[5];
    M5 Co;
    if (!propagate(G, F, cfg, cur, p, C, m, po, Co, nullptr, h, path, st)) break;
    cur = m;
    std::memcpy(p, po, sizeof p);
    const Surface& S = G.s[m];
    visited[n] = m;
    crossed[n] = (std::fabs(p[0]) <= S.hw0 && std::fabs(p[1]) <= S.hw1) ? 1 : 0;
    if (params_out) std::memcpy(params_out + 5 * n, p, sizeof p);
    ++n;
  }
  return n;
}

extern "C" int orc_navigate(const orc_geometry* g, const orc_field* f, const orc_config* c, int32_t surface,
                            const double* params, uint64_t mask, double path, int32_t* list, int32_t* n_list) {
  if (!g || !f || !c || !params || !list || !n_list) return -2;
  const Geometry G = load_geometry(g);
  const Field F = load_field(f);
  const Cfg cfg = load_cfg(c);
  Stats st;
  std::vector<int> l;
  const int L = navigate(G, F, cfg, bound_to_free(G.s[surface], params), mask, path, l, st);
  *n_list = (int)l.size();
  for (size_t i = 0; i < l.size(); ++i) list[i] = l[i];
  return L;
}

extern "C" int orc_scatter(const orc_geometry* g, const orc_config* c, int32_t surface, const double* params,
                           double* cov) {
  if (!g || !c || !params || !cov) return ORC_ERR_ARG;
  const Geometry G = load_geometry(g);
  M5 C = unpack(cov);
  apply_ms(G.s[surface], c->mass, params, C);
  pack(C, cov);
  return ORC_OK;
}

extern "C" int orc_seed_list(const orc_geometry* g, const orc_field* f, const orc_config* c, int32_t surface,
                             const double* params, int32_t* list) {
  if (!g || !f || !c || !params || !list) return -1;
  const Geometry G = load_geometry(g);
  const Field F = load_field(f);
  const Cfg cfg = load_cfg(c);
  Stats st;
  const Free f0 = bound_to_free(G.s[surface], params);
  std::vector<int> l;
  list_layer(G, cfg, G.s[surface].layer, f0.r, f0.T, (kKappa * f0.qop) * cross(f0.T, F.at(f0.r)), 0.0, surface,
             l, st);
  for (size_t i = 0; i < l.size(); ++i) list[i] = l[i];
  return (int)l.size();
}
