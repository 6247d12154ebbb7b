/* ckf.h - combinatorial Kalman filter (CKF) track finding on AMD Instinct
 * MI355X (gfx950).
 *
 * The operation (paper, section 2): seeds - initial track parameters on a
 * detector module - are propagated with the fourth-order Runge-Kutta-Nystrom
 * method together with their covariances through the detector in a
 * magnetic field; on every intersected module the Kalman filter computes a
 * chi2 from the covariance and the residual of each measurement, and every
 * measurement with a small enough chi2 starts a new branch.  The found track
 * is the pattern of measurements with its filtered parameters at the last
 * measurement.  Material effects assume muons (section 3).  The paper leaves
 * the step controller, navigation, gate, pruning and output rules open;
 * this library implements the documented readings listed in the design doc of
 * the source distribution (the same ones the test oracle implements).
 *
 * Units: mm, GeV, tesla, unit charge.  Bound parameters on a module are
 * (loc0, loc1, phi, theta, q/p).  A 5x5 covariance crosses the interface as
 * its packed upper triangle, row-major:
 *   (00,01,02,03,04,11,12,13,14,22,23,24,33,34,44).
 *
 * Memory: geometry and field are copied to the device once, when their
 * handles are created (paper, section 2: geometry and field are transferred
 * once).  Everything else - measurements, seeds, workspace, outputs - is
 * device memory owned by the caller (in practice PyTorch tensors) that must
 * outlive the stream work.  ckf_find allocates nothing and is asynchronous
 * on the caller's HIP stream.
 *
 * Errors: every entry point returns a ckf_status.  Argument and shape errors
 * are detected on the host before anything is enqueued; HIP errors map to
 * CKF_ERR_DEVICE with the message in ckf_last_error() (thread-local).
 * Conditions only the device can see (output or workspace capacity, bad
 * measurement offsets) are written to tracks->status after the stream work
 * completes; the caller synchronises and checks it.
 */
#ifndef CKF_H
#define CKF_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ckf_status {
  CKF_OK = 0,
  CKF_ERR_INVALID_ARGUMENT = 1,
  CKF_ERR_UNSORTED_INPUT = 2,
  CKF_ERR_CAPACITY = 3,
  CKF_ERR_DEVICE = 4,
  CKF_ERR_NOT_SUPPORTED = 5,
  CKF_ERR_NO_MODEL = 6
} ckf_status;

/* Device status words in ckf_tracks.status (int32[8]) after ckf_find. */
enum {
  CKF_STATUS_FLAGS = 0,       /* OR of the CKF_FLAG_* bits below */
  CKF_STATUS_NODES_NEEDED = 1, /* history nodes the batch needed */
  CKF_STATUS_TRACKS = 2,      /* tracks found (same as *n_tracks) */
  CKF_STATUS_MEAS_NEEDED = 3, /* measurement ids the output needed */
  CKF_STATUS_BAD_SEEDS = 4,   /* seeds skipped: bad surface/event or non-finite */
  CKF_STATUS_FAILED_LEGS = 5, /* propagations that did not land */
  CKF_STATUS_NAV_OVERFLOW = 6 /* navigation lookups that hit the candidate cap */
};
#define CKF_FLAG_NODE_CAPACITY 1  /* workspace history too small: retry larger */
#define CKF_FLAG_OUT_CAPACITY 2   /* output arrays too small: retry larger */
#define CKF_FLAG_BAD_OFFSETS 4    /* measurement offsets not non-decreasing */

typedef struct ckf_geometry ckf_geometry; /* opaque, device-resident */
typedef struct ckf_field ckf_field;       /* opaque, device-resident */
typedef struct ckf_timer ckf_timer;       /* opaque pair of HIP events */
typedef struct ckf_plan ckf_plan;         /* opaque captured ckf_find (hipGraph) */

/* Host description of a detector, copied by ckf_geometry_create.
 * Modules are planar rectangles: centre c, unit row vectors u (loc0 axis),
 * v (loc1 axis) and n = u x v (normal), half lengths along u and v.
 * Navigation layers: a barrel layer is the cylinder r = pos with
 * lo <= z <= hi; a disk layer the plane z = pos with lo <= r <= hi.  Every
 * module of a layer must lie on the far side of its envelope (r >= pos for
 * barrels, |z| >= |pos| for disks) and within its extent. */
typedef struct ckf_geometry_desc {
  int32_t n_surfaces;
  const float* center;       /* [n][3] */
  const float* rot;          /* [n][9] rows u, v, n */
  const float* half;         /* [n][2] */
  const float* thick;        /* [n] thickness in radiation lengths */
  const int32_t* layer;      /* [n] layer index, 0 <= layer < n_layers */
  int32_t n_layers;          /* at most 64 */
  const int32_t* layer_type; /* [L] 0 barrel, 1 disk */
  const float* layer_pos;    /* [L] */
  const float* layer_lo;     /* [L] */
  const float* layer_hi;     /* [L] */
} ckf_geometry_desc;

/* Algorithm configuration (all readings of points the paper leaves open). */
typedef struct ckf_config {
  double chi2_max;              /* accept chi2 < chi2_max (2 dof) */
  int32_t branches_per_surface; /* keep at most this many measurements per module (>= 1) */
  int32_t max_live_per_seed;    /* live candidates kept per seed after each step (>= 1) */
  int32_t max_holes;            /* terminate when holes exceed this */
  int32_t min_meas;             /* finished tracks need this many measurements */
  int32_t max_steps;            /* step budget per seed (<= 64) */
  int32_t max_rk_steps;         /* RKN4 trials per leg before the leg fails */
  double step_tol;              /* mm, RKN4 error-estimate tolerance */
  double step_max;              /* mm, largest RKN4 step */
  double land_tol;              /* mm, distance to the target plane that counts as landed */
  double path_max;              /* mm, total path budget */
  double nav_margin;            /* mm, margin of the module-listing test (<= 2) */
  double mass;                  /* GeV, particle hypothesis for scattering */
  int32_t material_on;          /* apply multiple scattering */
  int32_t tracks_per_seed;      /* must be 1: the best finished candidate per seed */
} ckf_config;

/* Measurements of one or more events, grouped by (event, surface): those of
 * event e on surface s are rows offsets[e*n_surfaces+s] .. offsets[..+1]-1.
 * A measurement's id is its row; found tracks report ids.  Device memory. */
typedef struct ckf_measurements {
  int32_t n_events;
  int32_t n_surfaces;        /* must equal the geometry's */
  int64_t n_meas;
  const int32_t* offsets;    /* [n_events*n_surfaces+1], non-decreasing, offsets[0] = 0 */
  const float* loc;          /* [n_meas][2] */
  const float* var;          /* [n_meas][2] variances of loc0, loc1 */
} ckf_measurements;

/* Seeds (device memory). */
typedef struct ckf_seeds {
  int32_t n_seeds;
  const int32_t* event;      /* [n] */
  const int32_t* surface;    /* [n] */
  const double* params;      /* [n][5] */
  const double* cov;         /* [n][15] packed */
} ckf_seeds;

/* Output (device memory, caller-allocated).  Tracks are ordered by seed
 * index, at most one per seed. */
typedef struct ckf_tracks {
  int32_t cap_tracks;        /* capacity of the per-track arrays (n_seeds suffices) */
  int64_t cap_meas;          /* capacity of meas */
  int32_t* n_tracks;         /* [1] */
  int32_t* offsets;          /* [cap_tracks+1] */
  int32_t* meas;             /* [cap_meas] measurement ids in visiting order */
  double* params;            /* [cap_tracks][5] filtered at the last measurement */
  double* cov;               /* [cap_tracks][15] */
  double* chi2;              /* [cap_tracks] sum of the accepted chi2 */
  int32_t* ndf;              /* [cap_tracks] 2*n_meas - 5 */
  int32_t* holes;            /* [cap_tracks] */
  int32_t* seed;             /* [cap_tracks] seed index */
  int32_t* event;            /* [cap_tracks] */
  int32_t* last_surface;     /* [cap_tracks] module of the last measurement */
  int32_t* status;           /* [8] CKF_STATUS_* words */
  int64_t* counters;         /* [24] or NULL: work-unit counters (CKF_CNT_*) */
} ckf_tracks;

/* Work-unit counters accumulated into tracks->counters when it is not NULL
 * (an instrumented kernel variant runs then; results are identical). */
enum {
  CKF_CNT_STEPS = 0,       /* candidate steps */
  CKF_CNT_NAV = 1,         /* next-layer searches */
  CKF_CNT_NAV_MODULES = 2, /* modules put through the listing test */
  CKF_CNT_LEGS = 3,        /* propagations to a module */
  CKF_CNT_RK_TRIALS = 4,   /* RKN4 steps attempted */
  CKF_CNT_CHI2 = 5,        /* chi2 evaluations */
  CKF_CNT_KF = 6,          /* Kalman updates */
  CKF_CNT_MS = 7,          /* scattering updates */
  CKF_CNT_CROSSED = 8,     /* visits that crossed their module */
  CKF_CNT_HOLES = 9,
  CKF_CNT_PRUNED = 10,
  CKF_CNT_FINISHED = 11,
  CKF_CNT_RK_REJECTS = 12,
  CKF_CNT_CYC_LEG = 13,    /* shader clocks per wave in the propagation leg (instrumented run) */
  CKF_CNT_CYC_SEARCH = 14, /* ... in covariance transport + search */
  CKF_CNT_CYC_OUT = 15,    /* ... in output slots, children, finishing */
  CKF_CNT_CYC_NAV = 16,    /* ... in navigation (next layer, module listing) */
  CKF_CNT_CYC_STEP = 17,   /* ... per whole step including admission, pruning, publishing */
  CKF_CNT_N = 24
};

/* Launch shape of ckf_find (chosen by the autotuner or the caller). */
typedef struct ckf_launch {
  int32_t grid;              /* persistent workgroups; 0 = device default */
  int32_t seeds_per_group;   /* concurrent seeds per 64-lane workgroup (1..64); 0 = default */
  int32_t nodes_per_seed;    /* history capacity per seed in the workspace; 0 = default (32) */
  ckf_timer* timer;          /* NULL, or events recorded around the track-finding kernel */
  int32_t waves_per_simd;    /* register budget of the kernel variant: 1 or 2 waves per SIMD (0 = 2) */
} ckf_launch;

/* Geometry: validates, builds the navigation grid on the host, uploads. */
ckf_status ckf_geometry_create(const ckf_geometry_desc* desc, ckf_geometry** out);
void ckf_geometry_destroy(ckf_geometry* g);

/* Uniform magnetic field (tesla). */
ckf_status ckf_field_create_uniform(float bx, float by, float bz, ckf_field** out);
void ckf_field_destroy(ckf_field* f);

/* The defaults of every configuration field (the readings documented in
 * the design doc). */
void ckf_config_default(ckf_config* cfg);

/* Workspace bytes ckf_find needs for this batch shape and launch. */
ckf_status ckf_workspace_size(const ckf_geometry* g, const ckf_config* cfg, const ckf_launch* launch,
                              int32_t n_events, int32_t n_seeds, int64_t n_meas, size_t* bytes);

/* Track finding for all seeds of a batch in one persistent launch.  stream
 * is a hipStream_t (NULL: the default stream).  launch may be NULL. */
ckf_status ckf_find(const ckf_geometry* g, const ckf_field* f, const ckf_measurements* m,
                    const ckf_seeds* s, const ckf_config* cfg, const ckf_launch* launch,
                    void* workspace, size_t workspace_bytes, ckf_tracks* out, void* stream);

/* Capture the whole ckf_find sequence for these arguments into a hipGraph
 * once (capture on `stream`, instantiation: allocates host-side graph
 * objects), so that repeated calls on the same buffers are one graph launch.
 * Every argument and buffer must stay valid and unchanged in address while
 * the plan is used; contents may change between launches.  The plan holds
 * no timer events (launch->timer is ignored). */
ckf_status ckf_plan_create(const ckf_geometry* g, const ckf_field* f, const ckf_measurements* m,
                           const ckf_seeds* s, const ckf_config* cfg, const ckf_launch* launch, void* workspace,
                           size_t workspace_bytes, ckf_tracks* out, void* stream, ckf_plan** plan);
/* Replay the captured sequence on `stream` (asynchronous, allocation-free). */
ckf_status ckf_plan_launch(ckf_plan* plan, void* stream);
void ckf_plan_destroy(ckf_plan* plan);

/* Component entry points (parity tests of single steps of the method). */

/* Propagate n bound states (device arrays) from module src[i] to the plane
 * of module dst[i]: parameters, transported covariance (FP64), bound-to-
 * bound Jacobian and path; ok[i] = 1 when the leg landed.  No material and
 * no bounds test. */
ckf_status ckf_propagate_batch(const ckf_geometry* g, const ckf_field* f, const ckf_config* cfg, int32_t n,
                               const int32_t* src, const double* p_in, const double* cov_in,
                               const int32_t* dst, double* p_out, double* cov_out, double* jac,
                               double* path, int32_t* ok, void* stream);

/* n independent Kalman updates (gain form, Joseph covariance, FP64) with
 * 2D measurements (device arrays). */
ckf_status ckf_kf_update_batch(int32_t n, const double* p_in, const double* cov_in, const float* meas,
                               const float* var, double* p_out, double* cov_out, double* chi2, void* stream);

/* A pair of HIP events that ckf_find records, on its stream, immediately
 * before and after the persistent track-finding kernel when the launch
 * names the timer.  Created once (it allocates driver events), reused. */
ckf_status ckf_timer_create(ckf_timer** out);
void ckf_timer_destroy(ckf_timer* t);
/* Milliseconds between the two events of the last recorded call; waits
 * for the second event. */
ckf_status ckf_timer_elapsed_ms(ckf_timer* t, float* ms);

const char* ckf_status_string(ckf_status s);
const char* ckf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
