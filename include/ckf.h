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
 * this library fixes them as stated at ckf_config and at each entry point
 * below (the test oracle implements the same readings independently).
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
#define CKF_FLAG_FIN_CAPACITY 8   /* tracks_per_seed = 0: more than 64 finished candidates per seed on
                                     average (the excess is lost; the output is incomplete) */
#define CKF_FLAG_BAD_OFFSETS 4    /* measurement offsets that do not tile [0, n_meas): offsets[0] != 0,
                                     a decreasing pair, or offsets[last] != n_meas (nothing is searched) */

typedef struct ckf_geometry ckf_geometry; /* opaque, device-resident */
typedef struct ckf_field ckf_field;       /* opaque, device-resident */
typedef struct ckf_timer ckf_timer;       /* opaque pair of HIP events */
typedef struct ckf_plan ckf_plan;         /* opaque captured ckf_find (hipGraph) */
typedef struct ckf_model ckf_model;       /* opaque next-module network packed for bf16 MFMA */

/* The learned next-module proposal (not in the paper: it replaces the
 * geometric module lookup of the navigation, section 2, by a small network
 * and keeps that lookup as its fallback).  For every module m the geometry
 * holds a neighbour table: the next layers a straight ray from the origin
 * through m's centre or corners meets (at most CKF_MAX_NEXT_LAYERS, in ray
 * order: centre, then corners (-,-), (+,-), (-,+), (+,+) in (loc0, loc1)),
 * and for each such layer L' the anchor A (where the first of those rays
 * that reaches L' meets its envelope), the module pitches (pu, pv) of L'
 * there, and a region of CKF_REGION_U x CKF_REGION_V cells around A in the
 * layer's curvilinear coordinates - (R dphi, dz) on a barrel of radius R,
 * (r dphi, dr) on a disk with r the point's own radius - each holding the
 * module of L' whose centre offset rounds to that cell (the nearest to the
 * cell centre when several do, ties by id).  A navigation that finds L'
 * centres a window of 8 x 4 cells (CKF_NEIGHBOURS) on the cell of its
 * local helix's crossing of L''s envelope; the network maps
 *   inputs (CKF_MLP_INPUTS): the crossing's fractional position in its cell
 *   (u, v), the direction there in the layer frame (phi-hat, then z-hat and
 *   r-hat on barrels, r-hat and z-hat on disks), q/p in 1/GeV, L' / number
 *   of layers;
 *   7 -> 64 -> 64 -> 32 with ReLU, bf16 weights and activations, FP32 sums,
 * to a softmax over the window's cells, in order (iv, iu) from (-2, -4).
 * Parameters cross the interface as one FP32 vector of CKF_MLP_PARAMS in
 * the order W1 [64][7], b1 [64], W2 [64][64], b2 [64], W3 [32][64], b3 [32]
 * (row-major, W[out][in]). */
#define CKF_MAX_NEXT_LAYERS 3
#define CKF_NEIGHBOURS 32
#define CKF_REGION_U 24
#define CKF_REGION_V 8
#define CKF_MLP_INPUTS 7
#define CKF_MLP_HIDDEN 64
#define CKF_MLP_OUTPUTS 32
#define CKF_MLP_PARAMS 6752

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
  int32_t tracks_per_seed;      /* 1: the best finished candidate per seed; 0: every finished candidate
                                   with at least min_meas measurements (ordered within a seed by the rank
                                   key), for tests; the workspace then holds up to 64 per seed */
  double learned_min_prob;      /* learned proposal: used when its top-k probabilities sum to at least this */
  int32_t learned_topk;         /* learned proposal: modules tested (1..3) */
} ckf_config;

/* Measurements of one or more events, grouped by (event, surface): those of
 * event e on surface s are rows offsets[e*n_surfaces+s] .. offsets[..+1]-1.
 * A measurement's id is its row; found tracks report ids.  Device memory.
 * Offsets that do not tile [0, n_meas) set CKF_FLAG_BAD_OFFSETS and nothing
 * is searched.  A measurement whose loc0 is NaN sorts after every finite one
 * of its module and is never accepted (its chi2 is not finite), as is one
 * with a NaN loc1 or variance. */
typedef struct ckf_measurements {
  int32_t n_events;
  int32_t n_surfaces;        /* must equal the geometry's */
  int64_t n_meas;
  const int32_t* offsets;    /* [n_events*n_surfaces+1], non-decreasing, offsets[0] = 0, last = n_meas */
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
 * index: at most one per seed, or with tracks_per_seed = 0 every finished
 * candidate of the seed in rank-key order (best first). */
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
  int64_t* counters;         /* [32] or NULL: work-unit counters (CKF_CNT_*) */
  int32_t* meas_surface;     /* [cap_meas] or NULL: module of each measurement */
  double* meas_params;       /* [cap_meas][5] or NULL: filtered parameters after each measurement */
  int32_t* seed_flags;       /* [n_seeds] or NULL: with counters and a model, 1 for a seed one of whose
                                candidates used a proposal whose listing differs from the geometric one
                                (those seeds may differ from the plain search; all others are identical);
                                cleared by ckf_find */
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
  CKF_CNT_CHUNKS = 18,     /* 64-lane passes over the candidate pools (instrumented run) */
  CKF_CNT_CYC_NEXT = 19,   /* shader clocks summed over lanes in the next-layer search */
  CKF_CNT_MLP_ROWS = 20,   /* navigations that evaluated the network */
  CKF_CNT_PROPOSALS = 21,  /* ... whose proposal was used (confident, non-empty listing) */
  CKF_CNT_PROPOSAL_MISS = 22, /* used proposals whose listing differs from the geometric one (audit) */
  CKF_CNT_MLP_BLOCKS = 23, /* 16-row network evaluations on the matrix cores */
  /* loop divergence (instrumented run): iterations summed over the lanes
   * that ran a loop, and the longest lane's iterations summed over the
   * wave's passes through it (their ratio / 64 is the loop's lane use) */
  CKF_CNT_LIST_LANE = 24,  /* grid entries visited by a module listing */
  CKF_CNT_LIST_WAVE = 25,  /* (the listing is wave-cooperative: its 64-entry passes) */
  CKF_CNT_NEXT_LANE = 26,  /* layer envelopes tried by a next-layer search */
  CKF_CNT_NEXT_WAVE = 27,
  CKF_CNT_LAND_LANE = 28,  /* landing iterations (RKN4 trials plus the final plane distance) of a leg */
  CKF_CNT_LAND_WAVE = 29,
  CKF_CNT_WIN_LANE = 30,   /* measurements read by a window scan */
  CKF_CNT_WIN_WAVE = 31,
  CKF_CNT_N = 32
};

/* Launch shape of ckf_find (chosen by the autotuner or the caller). */
typedef struct ckf_launch {
  int32_t grid;              /* persistent workgroups; 0 = device default */
  int32_t seeds_per_group;   /* concurrent seeds per 64-lane workgroup (1..64); 0 = default */
  int32_t nodes_per_seed;    /* history capacity per seed in the workspace; 0 = default (32) */
  ckf_timer* timer;          /* NULL, or events recorded around the track-finding kernel */
  int32_t waves_per_simd;    /* register budget of the kernel variant: 1, 2 or 3 waves per SIMD (0 = 3;
                                a field map uses at most 2) */
} ckf_launch;

/* Geometry: validates, builds the navigation grid on the host, uploads. */
ckf_status ckf_geometry_create(const ckf_geometry_desc* desc, ckf_geometry** out);
void ckf_geometry_destroy(ckf_geometry* g);

/* Uniform magnetic field (tesla). */
ckf_status ckf_field_create_uniform(float bx, float by, float bz, ckf_field** out);

/* A solenoidal field map (tesla) on a regular (r, z) grid: node (ir, iz) at
 * (r0 + ir*dr, z0 + iz*dz) holds values[(iz*nr + ir)*2 + {0: B_r, 1: B_z}]
 * (host memory, copied to the device once; nr, nz >= 2, dr, dz > 0).  The
 * field at a point is the bilinear interpolant in (r, z), coordinates
 * clamped to the grid, with B_x,y = B_r x,y / r; the transport Jacobian
 * includes the interpolant's gradient.  Not combined with the learned
 * proposal (ckf_find returns CKF_ERR_NOT_SUPPORTED). */
ckf_status ckf_field_create_rz(const float* values, int32_t nr, int32_t nz, float r0, float z0, float dr, float dz,
                               ckf_field** out);
void ckf_field_destroy(ckf_field* f);

/* The defaults of every configuration field: chi2_max 15, 3 branches per
 * module, 10 live candidates per seed, 3 holes, 6 measurements, 48 steps,
 * 100 RKN4 trials per leg, step tolerance 1e-2 mm, largest step 200 mm,
 * landing tolerance 1e-4 mm, path budget 4000 mm, listing margin 1 mm,
 * muon mass, scattering on, one track per seed, learned proposal used at a
 * summed top-3 probability of 0.95. */
void ckf_config_default(ckf_config* cfg);

/* Workspace bytes ckf_find needs for this batch shape and launch. */
ckf_status ckf_workspace_size(const ckf_geometry* g, const ckf_config* cfg, const ckf_launch* launch,
                              int32_t n_events, int32_t n_seeds, int64_t n_meas, size_t* bytes);

/* Track finding for all seeds of a batch in one persistent launch.  stream
 * is a hipStream_t (NULL: the default stream).  launch may be NULL.  model
 * NULL runs the plain geometric navigation; a model adds the learned
 * proposal: a navigation that finds a next layer listed for the current
 * module evaluates the network (one 16-row bf16 MFMA pass per 16 lanes) and,
 * when its top learned_topk probabilities sum to at least learned_min_prob,
 * lists among those modules only (same listing test); otherwise, or when
 * none of them passes, the geometric lookup runs. */
ckf_status ckf_find(const ckf_geometry* g, const ckf_field* f, const ckf_measurements* m,
                    const ckf_seeds* s, const ckf_config* cfg, const ckf_launch* launch, const ckf_model* model,
                    void* workspace, size_t workspace_bytes, ckf_tracks* out, void* stream);

/* Capture the whole ckf_find sequence for these arguments into a hipGraph
 * once (capture on `stream`, instantiation: allocates host-side graph
 * objects), so that repeated calls on the same buffers are one graph launch.
 * Every argument and buffer must stay valid and unchanged in address while
 * the plan is used; contents may change between launches.  The plan holds
 * no timer events (launch->timer is ignored). */
ckf_status ckf_plan_create(const ckf_geometry* g, const ckf_field* f, const ckf_measurements* m,
                           const ckf_seeds* s, const ckf_config* cfg, const ckf_launch* launch,
                           const ckf_model* model, void* workspace, size_t workspace_bytes, ckf_tracks* out,
                           void* stream, ckf_plan** plan);
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

/* ---- Learned proposal: neighbour table, network, training ---- */

/* Copy the geometry's neighbour table to host memory: next_layers
 * [n_surfaces][CKF_MAX_NEXT_LAYERS] (-1 pads), anchors
 * [n_surfaces][CKF_MAX_NEXT_LAYERS][4] = (phi_A, w_A, pu, pv) with w_A = z
 * on a barrel and r on a disk, and regions
 * [n_surfaces][CKF_MAX_NEXT_LAYERS][CKF_REGION_V * CKF_REGION_U] of module
 * ids, cell (iu, iv) for iu in [-12, 11], iv in [-4, 3] at
 * (iv + 4) * 24 + iu + 12 (-1 empty).  Synchronous. */
ckf_status ckf_geometry_neighbours(const ckf_geometry* g, int32_t* next_layers, float* anchors, int32_t* regions);

/* Pack CKF_MLP_PARAMS FP32 parameters (device memory, 16-byte aligned)
 * into a model for ckf_find (allocates ~15 KB of device memory; the packing
 * runs on `stream`).  ckf_model_update repacks new parameters into the same
 * model (allocation-free, asynchronous). */
ckf_status ckf_model_create(const float* params, void* stream, ckf_model** out);
ckf_status ckf_model_update(ckf_model* model, const float* params, void* stream);
void ckf_model_destroy(ckf_model* model);

/* Network logits [n][32] for inputs x [n][7] (device memory), evaluated
 * exactly as inside ckf_find (bf16 MFMA, FP32 sums). */
ckf_status ckf_mlp_forward(const ckf_model* model, const float* x, int64_t n, float* logits, void* stream);

/* Workspace bytes of ckf_mlp_grad for a batch of n rows. */
ckf_status ckf_mlp_workspace_size(int64_t n, size_t* bytes);

/* Mean softmax cross-entropy of a batch and its gradient with respect to
 * the FP32 parameters (forward and backward on bf16 MFMA with FP32 sums;
 * per-64-row partial gradients summed in a fixed order, so the result is
 * deterministic).  Row i of the batch is x[rows[i]], labels[rows[i]]
 * (rows NULL: row i).  grad [CKF_MLP_PARAMS] and loss [1] are written. */
ckf_status ckf_mlp_grad(const float* params, const float* x, const int32_t* labels, const int32_t* rows,
                        int64_t n, void* workspace, size_t workspace_bytes, float* grad, float* loss,
                        void* stream);

/* One Adam step (bias-corrected; step counts from 1) on FP32 parameters
 * with FP32 moments m, v (all CKF_MLP_PARAMS, device memory). */
ckf_status ckf_mlp_adam(float* params, float* m, float* v, const float* grad, int32_t step, float lr,
                        float beta1, float beta2, float eps, void* stream);

/* Kalman-filter fit of found tracks with a smoother (paper section 2: the
 * fit that follows track finding, with the Rauch-Tung-Striebel smoother;
 * section 4: the optimal two-filter smoother).  The forward filter starts
 * from each track's seed and visits the modules of its measurements in
 * order (the search's FP32 stepper and Jacobian, FP64 transport, gain-form
 * update with the Joseph covariance, then the module's scattering added at
 * the updated state).  The smoother gives every measurement the state
 * estimated from all of the track's measurements:
 *   CKF_SMOOTHER_RTS:        Rauch-Tung-Striebel gains over the forward pass;
 *   CKF_SMOOTHER_TWO_FILTER: Fraser and Potter's optimal smoother: an
 *                            independent backward information filter (no
 *                            prior, no forward information) over the model
 *                            the forward pass linearised, combined with the
 *                            forward filtered state by weight; equal to RTS
 *                            up to rounding.
 * Tracks (device memory, the layout ckf_find writes): n_tracks (device
 * int32, at most cap_tracks used), offsets [cap_tracks+1] into meas,
 * meas_surface [cap_meas] and seed [cap_tracks]; measurement ids index the
 * measurement arrays of m, seed ids the seeds of s.  Outputs (device,
 * caller-owned): params [cap_meas][5] and cov [cap_meas][15] smoothed at
 * each measurement (NaN for a track that failed), chi2 [cap_tracks] (sum of
 * the forward filter's chi2), ok [cap_tracks]: 1 fitted, 0 a leg failed or
 * a covariance lost positive definiteness, -1 ids out of range or a track
 * of more than 64 measurements (ckf_find's step bound; NaN outputs), -1
 * with the outputs untouched for offsets outside [0, cap_meas] or tracks
 * whose ranges overlap (more measurements in all than cap_meas: then no
 * track of the call is fitted).  The tracks are dealt to 64-lane waves
 * longest first, so a wave's lanes take about the same number of steps.
 * workspace: at least ckf_fit_workspace_size(cap_meas) bytes of device
 * memory (CKF_ERR_CAPACITY if smaller).  Asynchronous on `stream`;
 * allocates nothing. */
#define CKF_SMOOTHER_RTS 0
#define CKF_SMOOTHER_TWO_FILTER 1
ckf_status ckf_fit_workspace_size(int64_t cap_meas, size_t* bytes);
ckf_status ckf_fit(const ckf_geometry* g, const ckf_field* f, const ckf_measurements* m, const ckf_seeds* s,
                   const ckf_config* cfg, const int32_t* n_tracks, int32_t cap_tracks, int64_t cap_meas,
                   const int32_t* offsets, const int32_t* meas, const int32_t* meas_surface, const int32_t* seed,
                   int32_t smoother, void* workspace, size_t workspace_bytes, double* params, double* cov,
                   double* chi2, int32_t* ok, void* stream);

/* ckf_fit without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, outputs and errors as ckf_fit
 * minus the workspace: the fit's per-measurement records live in a fixed
 * device array of the library, ckf_fit_noalloc_max_bytes() = 64 MiB per GPU
 * (allocated when the library's code is loaded on a GPU and held until the
 * process ends), enough for ckf_fit_noalloc_max_meas() = 213,823
 * measurements; a larger cap_meas fails with CKF_ERR_CAPACITY and launches
 * nothing.  The call itself allocates nothing.  All calls on one GPU share
 * that array: calls that can overlap on one GPU (different streams, or
 * different host threads) race and must be ordered by the caller. */
ckf_status ckf_fit_noalloc(const ckf_geometry* g, const ckf_field* f, const ckf_measurements* m,
                           const ckf_seeds* s, const ckf_config* cfg, const int32_t* n_tracks, int32_t cap_tracks,
                           int64_t cap_meas, const int32_t* offsets, const int32_t* meas,
                           const int32_t* meas_surface, const int32_t* seed, int32_t smoother, double* params,
                           double* cov, double* chi2, int32_t* ok, void* stream);
size_t ckf_fit_noalloc_max_bytes(void);
int64_t ckf_fit_noalloc_max_meas(void);

/* Activated detector cells (device memory) in readout order: grouped by
 * (event, module) row like the measurements, then by row c1 and column c0
 * inside a module (strictly increasing (c1, c0) within a module). */
typedef struct ckf_cells {
  int32_t n_events;
  int32_t n_surfaces;        /* must equal the geometry's */
  int64_t n_cells;
  const int32_t* offsets;    /* [n_events*n_surfaces+1] */
  const int32_t* c0;         /* [n_cells] column */
  const int32_t* c1;         /* [n_cells] row */
  const float* q;            /* [n_cells] charge (> 0) */
} ckf_cells;

#define CKF_CLUSTER_BAD_OFFSETS 1 /* a row's offsets out of order or beyond n_cells (row skipped) */
#define CKF_CLUSTER_UNSORTED 2    /* cells of a module not in readout order (its clusters are not defined) */

/* Cell clustering and measurement formation (paper section 2: connected
 * component analysis of the activated cells, weighted centroids as
 * measurements, spacepoints in global coordinates).  Two cells of a module
 * are connected when |dc0| <= 1 and |dc1| <= 1; a cluster is a connected
 * component, named by its first cell in readout order, and a module's
 * clusters come out in that order.  Measurement: the charge-weighted mean of
 * the cell centres ((c + 1/2) pitch - half length, FP64 sums in readout
 * order, stored FP32), variances pitch^2 / 12.  pitch [n_surfaces][2]
 * (device) gives each module's cell size in mm.  Outputs (device,
 * caller-owned, sized for n_cells clusters at most): meas_offsets
 * [n_events*n_surfaces+1] (the layout of ckf_measurements), loc and var
 * [n_cells][2], spacepoints [n_cells][3] or NULL (centre + loc0 u + loc1 v),
 * cell_cluster [n_cells] or NULL (the measurement index of every cell),
 * status [1] (device, cleared by the call): CKF_CLUSTER_* bits.
 * workspace: at least ckf_cluster_workspace_size bytes (CKF_ERR_CAPACITY).
 * Asynchronous on `stream`; allocates nothing. */
ckf_status ckf_cluster_workspace_size(const ckf_cells* cells, size_t* bytes);
ckf_status ckf_cluster(const ckf_geometry* g, const ckf_cells* cells, const float* pitch, void* workspace,
                       size_t workspace_bytes, int32_t* meas_offsets, float* loc, float* var, float* spacepoints,
                       int32_t* cell_cluster, int32_t* status, void* stream);

/* Triplet seeding and helix parameter estimation (paper section 2: triplets
 * of spacepoints that can approximately form a helix; the track's position
 * and momentum estimated at the first spacepoint with the helix model).
 * Spacepoints in the measurement layout (ckf_cluster's output): rows of
 * (event, module) given by meas_offsets [n_events*n_surfaces+1], with
 * global positions spacepoints [n_sp][3] and local positions loc [n_sp][2]
 * (device).  layers [n_layers] (HOST array, 3 <= n_layers <= 8): the
 * seeding layers' geometry ids ordered outwards.  A triplet has its bottom,
 * middle and top on three seeding layers in that order, in one event.
 * Cuts (FP64, no fused operations): per doublet |dz/dr| <= 3, azimuth step
 * <= 0.12 rad, the bottom doublet's line within 200 mm of z = 0 at r = 0;
 * per triplet |cot_BM - cot_MT| <= 0.01 + 0.007 (1 + cot_BM^2), the
 * transverse circle's radius >= the helix radius of 0.5 GeV in bz and its
 * distance of closest approach to the beam line <= 1 mm.  Per middle
 * spacepoint at most the 2 best by (distance, bottom, top); seeds in order
 * of their middle spacepoint.  Seed on the bottom spacepoint's module:
 * (loc0, loc1) = its local position, phi = the circle's tangent there
 * towards the middle, theta from the transverse arc to the top and dz,
 * q/p = q sin(theta) / (kappa |bz| R); covariance diagonal (0.2 mm, 0.6 mm,
 * 10 mrad, 10 mrad, 15 % of q/p).  Outputs (device, caller-owned, cap_seeds
 * rows; seeds beyond the capacity are counted but not written): n_seeds
 * [1], seed_event, seed_surface, seed_params [cap][5], seed_cov [cap][15]
 * (the layout of ckf_seeds), seed_spacepoints [cap][3] (bottom, middle,
 * top) or NULL.  counters [4] (device) or NULL: set by the call to the work
 * units of the triplet search, CKF_SEED_CNT_* (for the algorithmic rate).
 * workspace: at least ckf_seed_workspace_size bytes (CKF_ERR_CAPACITY).
 * Asynchronous on `stream`; allocates nothing. */
ckf_status ckf_seed_workspace_size(int32_t n_events, int32_t n_surfaces, int64_t n_sp, int32_t n_layers,
                                   size_t* bytes);
ckf_status ckf_seed(const ckf_geometry* g, int32_t n_events, const int32_t* meas_offsets, int64_t n_sp,
                    const float* spacepoints, const float* loc, const int32_t* layers, int32_t n_layers, double bz,
                    void* workspace, size_t workspace_bytes, int64_t cap_seeds, int32_t* n_seeds,
                    int32_t* seed_event, int32_t* seed_surface, double* seed_params, double* seed_cov,
                    int32_t* seed_spacepoints, int64_t* counters, void* stream);

/* Work units of ckf_seed's triplet search (counters[k]).  A middle's tops
 * are counted once, though the on-chip path runs their test twice (to count
 * and then to place them). */
enum {
  CKF_SEED_CNT_MT = 0,  /* (middle, top) doublet tests */
  CKF_SEED_CNT_BM = 1,  /* (bottom, middle) doublet tests */
  CKF_SEED_CNT_COT = 2, /* (bottom, top) cot comparisons */
  CKF_SEED_CNT_TRI = 3, /* triplet tests (circle, radius, d0) */
  CKF_SEED_CNT_N = 4
};

/* Tuning of ckf_seed's triplet search (process-wide, for later calls).  The
 * search holds a middle spacepoint's tops that pass the doublet cuts in
 * on-chip memory, ordered by cot, and falls back to scanning each bottom's
 * window of tops directly when a middle has more than `cap` of them; both
 * ways give the same seeds.  cap in [0, *cap_max] (0: always scan); the
 * default is the maximum.  cap_max (host, out) or NULL: written in every
 * case.  A cap outside the range returns CKF_ERR_INVALID_ARGUMENT and keeps
 * the current setting.  Not synchronised with calls in flight on other
 * threads. */
ckf_status ckf_seed_set_top_cap(int32_t cap, int32_t* cap_max);

/* Greedy ambiguity resolution of found tracks by shared measurements (paper
 * section 4: the stage after track finding that removes duplicate and fake
 * tracks).  A measurement is shared when more than one surviving track holds
 * it; a surviving track is bad when more than max_shared of its
 * measurements are shared.  While a bad track exists, the bad track with the
 * largest shared fraction s/n is removed (ties: the larger chi2/ndf taken in
 * FP32, then the larger track index), and the shares are recounted.  The
 * result equals that sequential definition; the library reaches it in
 * parallel rounds that each remove every bad track whose key beats all bad
 * tracks it shares a measurement with.
 * Tracks (device memory, ckf_find's layout): n_tracks (device int32, at
 * most cap_tracks used), offsets [cap_tracks+1] into meas [cap_meas],
 * chi2 and ndf [cap_tracks]; measurement ids must lie in [0, n_meas).
 * keep [cap_tracks] (device) receives 1 kept, 0 removed, -1 for a track
 * whose offsets or ids are out of range (it takes no part).  The rounds run
 * on the device: max_rounds (1..1024) of them are launched, and once no bad
 * track is left the remaining ones return at once.  info (device int32[2],
 * or NULL) receives the rounds that removed tracks and 1 if no bad track is
 * left (0: max_rounds did not suffice and the result is a prefix of the
 * greedy; call again with a larger bound).  workspace: at least
 * ckf_resolve_workspace_size(cap_tracks, n_meas) bytes (CKF_ERR_CAPACITY if
 * smaller).  Asynchronous on `stream` with no host synchronisation, so it can
 * be captured in a graph; it allocates nothing.  n_meas above 2^31 - 1 gives
 * CKF_ERR_NOT_SUPPORTED. */
ckf_status ckf_resolve_workspace_size(int32_t cap_tracks, int64_t n_meas, size_t* bytes);
ckf_status ckf_resolve(const int32_t* n_tracks, int32_t cap_tracks, int64_t cap_meas, const int32_t* offsets,
                       const int32_t* meas, int64_t n_meas, const double* chi2, const int32_t* ndf,
                       int32_t max_shared, int32_t max_rounds, void* workspace, size_t workspace_bytes, int32_t* keep,
                       int32_t* info, void* stream);

/* Device workspace of ckf_capture_pairs for cap_tracks tracks: bytes it needs. */
ckf_status ckf_capture_workspace_size(int32_t cap_tracks, size_t* bytes);

/* Training pairs from found tracks (device memory): at every change of
 * layer between consecutive measurements of a track, the network input of
 * the state at the last measurement of the layer - through its local
 * helix's crossing of the next measurement's layer, in `field` - paired
 * with the position in the window around that crossing of the module of
 * each measurement the track has on that layer (overlapping modules give
 * several pairs with the same input).  A pair is dropped when that layer
 * is not listed for the module, the helix misses the envelope, or the
 * module is outside the window (or a module id is out of range).  Pairs are written in track
 * order, then measurement order, up to cap_pairs: x [cap][7], label [cap],
 * track [cap] (may be NULL).  counts [2] receives the number of pairs (also
 * beyond cap) and of dropped pairs.  n_tracks is a device int32 (as
 * ckf_find writes it); offsets, meas_surface and meas_params are a
 * ckf_find output (offsets within meas capacity).  workspace: device
 * memory of at least ckf_capture_workspace_size(cap_tracks) bytes
 * (CKF_ERR_CAPACITY if smaller), owned by the caller, free again when the
 * stream has passed the call.  Uniform field only (CKF_ERR_NOT_SUPPORTED
 * for a map). */
ckf_status ckf_capture_pairs(const ckf_geometry* g, const ckf_field* field, const int32_t* n_tracks,
                             int32_t cap_tracks, const int32_t* offsets, const int32_t* meas_surface,
                             const double* meas_params, int64_t cap_pairs, float* x, int32_t* label,
                             int32_t* track, int64_t* counts, void* workspace, size_t workspace_bytes,
                             void* stream);

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
