/* FP64 CPU oracle of combinatorial-Kalman-filter track finding.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a plain, slow, obviously correct implementation of the same
 * method.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the GPU product path never does.  It shares no
 * code, header or constant with the GPU library.
 *
 * Method (paper, section 2): seeds are propagated with the fourth-order
 * Runge-Kutta-Nystrom method together with their covariance; on every
 * intersected module a chi2 from the covariance and the residual decides
 * whether a measurement is attached, each attached measurement making a new
 * branch; the filtered parameters at the last measurement are the most
 * accurate.  Material effects assume muons (section 3).  Every point the
 * paper leaves open is fixed by a documented reading; see oracle.cpp.
 *
 * Conventions: mm, GeV, tesla, unit charge.  Bound parameters on a module
 * are (loc0, loc1, phi, theta, q/p); free parameters (x, y, z, Tx, Ty, Tz,
 * q/p).  Covariances cross the interface as the packed upper triangle of the
 * 5x5 matrix, row-major: (00,01,02,03,04,11,12,13,14,22,23,24,33,34,44).
 * All arrays are host memory owned by the caller.
 */
#ifndef CKF_ORACLE_H
#define CKF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_geometry {
  int32_t n_surfaces;
  const float* center;      /* [n][3] */
  const float* rot;         /* [n][9] rows u (loc0 axis), v (loc1 axis), n (normal) */
  const float* half;        /* [n][2] half lengths along u, v */
  const float* thick;       /* [n] thickness in radiation lengths */
  const int32_t* layer;     /* [n] navigation layer of the module */
  int32_t n_layers;
  const int32_t* layer_type; /* [L] 0 barrel cylinder, 1 disk */
  const float* layer_pos;    /* [L] envelope radius (barrel) or signed z (disk) */
  const float* layer_lo;     /* [L] envelope extent: z_min (barrel), r_min (disk) */
  const float* layer_hi;     /* [L] z_max (barrel), r_max (disk) */
} orc_geometry;

/* Magnetic field, tesla: uniform b, or (map != NULL) a solenoidal map of
 * (B_r, B_z) on a regular (r, z) grid - node (ir, iz) at r0 + ir*dr,
 * z0 + iz*dz, values map[(iz*nr + ir)*2 + {0: B_r, 1: B_z}] - interpolated
 * bilinearly, coordinates clamped to the grid; B_x,y = B_r x,y / r. */
typedef struct orc_field {
  double b[3];
  const float* map;
  int32_t nr, nz;
  double r0, z0, dr, dz;
} orc_field;

typedef struct orc_measurements {
  int32_t n_events;
  int32_t n_surfaces;
  const int32_t* offsets;   /* [n_events*n_surfaces+1] rows of (event, surface) */
  const float* loc;         /* [n][2] local position */
  const float* var;         /* [n][2] variance of loc0, loc1 */
} orc_measurements;

typedef struct orc_seeds {
  int32_t n_seeds;
  const int32_t* event;     /* [k] */
  const int32_t* surface;   /* [k] module the parameters are bound to */
  const double* params;     /* [k][5] */
  const double* cov;        /* [k][15] packed upper triangle */
} orc_seeds;

typedef struct orc_config {
  double chi2_max;          /* gate: accept chi2 < chi2_max */
  int32_t branches_per_surface;  /* keep at most this many measurements per module; <=0: all */
  int32_t max_live_per_seed;     /* prune to this many live candidates per seed; <=0: no pruning */
  int32_t max_holes;        /* terminate when holes exceed this */
  int32_t min_meas;         /* finished candidates need this many measurements */
  int32_t max_steps;        /* step budget per seed */
  int32_t max_rk_steps;     /* RKN4 trials per leg before the leg fails */
  double step_tol;          /* mm, RKN4 error-estimate tolerance */
  double step_max;          /* mm, largest RKN4 step */
  double land_tol;          /* mm, distance to the target plane that counts as landed */
  double path_max;          /* mm, total path budget */
  double nav_margin;        /* mm, margin of the module-listing test */
  double mass;              /* GeV, particle hypothesis for scattering */
  int32_t material_on;      /* apply multiple scattering */
  int32_t tracks_per_seed;  /* 1: best finished candidate per seed; 0: all finished */
} orc_config;

typedef struct orc_tracks {
  int32_t cap_tracks;       /* in: capacity of the per-track arrays */
  int32_t cap_meas;         /* in: capacity of meas */
  int32_t n_tracks;         /* out */
  int32_t n_meas_total;     /* out (also set when capacity is short) */
  int32_t* offsets;         /* [cap_tracks+1] */
  int32_t* meas;            /* [cap_meas] measurement ids in visiting order */
  double* params;           /* [cap_tracks][5] filtered at the last measurement */
  double* cov;              /* [cap_tracks][15] */
  double* chi2;             /* [cap_tracks] */
  int32_t* ndf;
  int32_t* holes;
  int32_t* seed;
  int32_t* event;
  int32_t* last_surface;
  int32_t* meas_surface;    /* [cap_meas] or NULL: module of each measurement */
  double* meas_params;      /* [cap_meas][5] or NULL: filtered parameters after each measurement */
} orc_tracks;

typedef struct orc_stats {
  int64_t steps;            /* candidate steps */
  int64_t navigations;      /* next-layer searches */
  int64_t nav_modules;      /* modules put through the listing test */
  int64_t legs;             /* propagations to a module */
  int64_t legs_failed;
  int64_t rk_trials;        /* RKN4 steps attempted (accepted + rejected) */
  int64_t rk_rejects;
  int64_t chi2_evals;
  int64_t kf_updates;
  int64_t ms_updates;
  int64_t crossed;          /* visits that crossed their module */
  int64_t holes;
  int64_t pruned;
  int64_t finished;
  int64_t mlp_rows;         /* learned form: navigations that evaluated the network */
  int64_t proposals;        /* ... whose proposal was used (confident, non-empty listing) */
  int64_t proposal_misses;  /* ... used proposals listing differently from the geometric lookup */
} orc_stats;

/* The learned next-module proposal (not in the paper: it replaces only the
 * module lookup of the navigation and keeps that lookup as its fallback).
 * The neighbour table is an input: for module m, next[m][q] (q < 3, -1 pads)
 * is a next layer, anchor[m][q] = (A x, y, z, pitch u, pitch v) its anchor
 * point on that layer's envelope and pitches, region[m][q][iv*24 + iu] the
 * module id in cell (iu - 12, iv - 4) around the anchor (-1 empty).  The
 * network parameters are W1 [64][7], b1, W2 [64][64], b2, W3 [32][64], b3
 * (6752 FP32 values).  bf16 != 0 rounds weights, inputs and hidden
 * activations to bfloat16 where a bf16 matrix-core evaluation does. */
typedef struct orc_learned {
  const int32_t* next;      /* [n_surfaces][3] */
  const int32_t* region;    /* [n_surfaces][3][192] */
  const double* anchor;     /* [n_surfaces][3][5] */
  const float* params;      /* [6752] */
  double min_prob;          /* proposal used when its top-k probabilities sum to at least this */
  int32_t topk;             /* 1..3 modules proposed */
  int32_t bf16;
} orc_learned;

/* Causes (bits of seed_near) by which an FP32 evaluation of the proposal can
 * decide otherwise than this FP64 one. */
#define ORC_NEAR_CONF 1     /* summed probability within 1e-4 of the threshold */
#define ORC_NEAR_BF16 2     /* one value near a bfloat16 rounding boundary decides the outcome */
#define ORC_NEAR_EDGE 4     /* crossing within 5e-5 of a cell edge, the neighbouring window decides otherwise */
#define ORC_NEAR_RANK 8     /* k-th and (k+1)-th probabilities within 1e-4 */

/* Status codes. */
#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_CAPACITY 3
#define ORC_ERR_FAILED 7

/* The field (tesla) at n points p [n][3] (mm), and if G is not NULL its
 * gradient G [n][3][3] = dB_i/dx_j of the interpolant. */
int orc_field_eval(const orc_field* f, int32_t n, const double* p, double* B, double* G);

/* Track finding for every seed; n_threads <= 0 uses all hardware threads.
 * Output is ordered by seed index.  stats may be NULL. */
int orc_ckf_find(const orc_geometry* g, const orc_field* f, const orc_measurements* m,
                 const orc_seeds* s, const orc_config* cfg, int n_threads,
                 orc_tracks* out, orc_stats* stats);

/* Track finding with the learned proposal (uniform field only).  seed_near
 * (nullable, [n_seeds]) receives the OR of the ORC_NEAR_* causes met by any
 * network evaluation of the seed's candidates; seed_differs (nullable) 1 for
 * a seed one of whose used proposals listed differently from the geometric
 * lookup (every other seed finds exactly the plain search's tracks). */
int orc_ckf_find_learned(const orc_geometry* g, const orc_field* f, const orc_measurements* m,
                         const orc_seeds* s, const orc_config* cfg, const orc_learned* l, int n_threads,
                         orc_tracks* out, orc_stats* stats, int32_t* seed_near, int32_t* seed_differs);

/* Network logits [n][32] of inputs x [n][7]. */
int orc_mlp_forward(const float* params, int32_t bf16, int64_t n, const double* x, double* logits);

/* The proposal of one navigation from `surface` to `layer`, whose local
 * helix crosses the layer's envelope at X with direction T: returns -1 when
 * the network does not run (no table row, or no window), else 1 when the
 * proposal is used (confident) and 0 when not.  cell [2] the window's centre
 * cell, feat [7] the unrounded input, conf the summed top-k probability,
 * classes [3] the three most probable outputs, modules [3] the modules of
 * the top k (-1 for an empty cell or beyond k), near the ORC_NEAR_* causes. */
int orc_learned_propose(const orc_geometry* g, const orc_learned* l, int32_t surface, int32_t layer,
                        const double* X, const double* T, double qop, int32_t* cell, double* feat,
                        double* conf, int32_t* classes, int32_t* modules, int32_t* near);

/* Propagate bound parameters and covariance from module src to the plane of
 * module dst (no material, no bounds test).  jac (5x5 row-major, may be
 * NULL) is d(out)/d(in).  h_trial: in/out step-size hint (<=0: step_max).
 * Returns ORC_OK or ORC_ERR_FAILED. */
int orc_propagate(const orc_geometry* g, const orc_field* f, const orc_config* cfg,
                  int32_t src, const double* p_in, const double* cov_in, int32_t dst,
                  double* p_out, double* cov_out, double* jac, double* path);

/* Propagate a free state (x,y,z,Tx,Ty,Tz,q/p) onto the plane through c with
 * normal n; returns the landed free state and the path length. */
int orc_propagate_free(const orc_field* f, const orc_config* cfg, const double* free_in,
                       const double* c, const double* n, double* free_out, double* path);

/* One Kalman update (gain form, Joseph covariance) with a 2D measurement. */
int orc_kf_update(const double* p_in, const double* cov_in, const double* meas,
                  const double* var, double* p_out, double* cov_out, double* chi2);

/* Follow one track through the navigator without measurements or material:
 * visited modules in order, whether each was crossed, and the bound
 * parameters there.  Returns the number of visits written (<= cap). */
int orc_trace(const orc_geometry* g, const orc_field* f, const orc_config* cfg,
              int32_t surface, const double* params, int32_t cap,
              int32_t* visited, int32_t* crossed, double* params_out);

/* The navigator alone: from bound parameters on `surface` with visited-layer
 * mask and path so far, the next layer (returned, -1 if none) and its listed
 * modules in visiting order (at most 4, written to list, count to n_list). */
int orc_navigate(const orc_geometry* g, const orc_field* f, const orc_config* cfg, int32_t surface,
                 const double* params, uint64_t mask, double path, int32_t* list, int32_t* n_list);

/* The modules of the seed's own layer that a seed on `surface` visits after
 * its own (overlaps), in visiting order (at most 4); returns the count. */
int orc_seed_list(const orc_geometry* g, const orc_field* f, const orc_config* cfg, int32_t surface,
                  const double* params, int32_t* list);

/* Multiple-scattering covariance increment for bound parameters on a module
 * (adds to cov in place, packed upper triangle). */
int orc_scatter(const orc_geometry* g, const orc_config* cfg, int32_t surface, const double* params,
                double* cov);

#ifdef __cplusplus
}
#endif
#endif
