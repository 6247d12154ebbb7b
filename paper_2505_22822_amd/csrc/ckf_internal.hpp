// Internal layouts shared by the host runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ckf.h"

namespace ckf {

constexpr int kWave = 64;          // lanes per wavefront (one wave per workgroup)
constexpr int kMaxList = 4;        // listed modules per navigation layer
constexpr int kMaxBranch = 4;      // largest branches_per_surface supported
constexpr int kMaxCand = 96;       // grid cell entries visited per listing lookup
constexpr int kMaxLayers = 64;     // visited-layer mask width
constexpr int kMaxSteps = 64;      // largest max_steps (history walk buffer)
constexpr float kReach = 30.0f;    // mm, envelope-to-module reach of the candidate pre-filter
constexpr float kGridPad = 5.0f;   // mm, padding of module extents in the navigation grid
constexpr float kMaxNavMargin = 2.0f;
constexpr int kMaxNext = CKF_MAX_NEXT_LAYERS;  // next layers per module in the neighbour table
constexpr int kNeighbours = CKF_NEIGHBOURS;    // network outputs: the proposal window's cells
constexpr int kWinU = 8, kWinV = 4, kWinU0 = -4, kWinV0 = -2;          // window cells around the crossing
constexpr int kRegU = CKF_REGION_U, kRegV = CKF_REGION_V, kRegU0 = -12, kRegV0 = -4;  // stored region
constexpr int kRegCells = kRegU * kRegV;
static_assert(kWinU * kWinV == kNeighbours, "window size");

// Surface store: one 64-byte record per module (a lane reads one record per
// access; records of neighbouring modules share cache lines).
struct alignas(64) Module {
  float c[3];
  float u[3];
  float v[3];
  float n[3];
  float hw0, hw1, thick;
  int layer;
};
static_assert(sizeof(Module) == 64, "module record");
static_assert(kMaxList == 4 && kMaxBranch == 4, "list code is unrolled for 4 entries");

struct LayerRec {
  int type;        // 0 barrel, 1 disk
  float pos;       // envelope radius or signed z
  float lo, hi;    // envelope extent (z for barrels, r for disks)
  float depth;     // how far modules reach beyond the envelope (+ pad)
  int nphi, nw;    // grid bins in phi and in w (z or r)
  float wlo, whi;  // grid range in w
  int cell_base;   // first cell of this layer in the CSR
  int pad0, pad1;
};

struct GeomDev {
  int n_surfaces = 0, n_layers = 0;
  const Module* mod = nullptr;
  const LayerRec* layers = nullptr;
  const int* cell_off = nullptr;   // [n_cells + 1]
  const int* cell_mod = nullptr;
  const int* barrel_order = nullptr;  // barrel layers by radius
  const int* disk_pos = nullptr;      // z > 0 disks by |z|
  const int* disk_neg = nullptr;      // z < 0 disks by |z|
  int n_barrel = 0, n_disk_pos = 0, n_disk_neg = 0;
  // neighbour table of the learned proposal: per module the next layers and
  // their rows [n][kMaxNext] (-1 pads); per row the anchor and pitches
  // (phi_A, w_A, pitch u, pitch v) and the stored region of kRegCells
  // module ids (-1 empty), cell (iu, iv) at (iv - kRegV0) * kRegU + iu - kRegU0
  const int* nb_next = nullptr;
  const int* nb_row = nullptr;
  const float4* nb_anc = nullptr;
  const int* nb_reg = nullptr;
};

// Field: uniform (map == nullptr) or a solenoidal (r, z) map interpolated
// bilinearly with clamped coordinates.  map[iz*nr + ir] holds
// (B_r, B_z) at (ir, iz) and at (ir+1, iz), so one z row of a cell is one
// 16-byte load.
struct FieldDev {
  float bx = 0.f, by = 0.f, bz = 0.f;  // uniform field, tesla
  const float4* map = nullptr;
  int nr = 0, nz = 0;
  float r0 = 0.f, z0 = 0.f, inv_dr = 1.f, inv_dz = 1.f;
};

// Scalar configuration as the kernels use it.
struct CfgDev {
  double chi2_max;
  int branches, max_live, max_holes, min_meas, max_steps, max_rk;
  float step_tol, step_max, land_tol, path_max, nav_margin;
  double mass;
  int material;
  float min_prob;  // learned proposal: smallest summed probability of the top-k to use it
  int topk;        // learned proposal: modules tested per proposal
  int all_tracks;  // every finished candidate goes to the output (tracks_per_seed = 0)
};

// The next-module network packed for the bf16 matrix cores: weight tiles in
// the A-operand order of v_mfma_f32_16x16x16_bf16 (per 16x16 tile, lane l
// holds W[16*ob + l%16][16*kb + 4*(l/16) + j], j = 0..3), FP32 biases.  The
// four fragments a lane needs for one output tile are adjacent (32 bytes),
// so a tile's operands arrive with two 16-byte loads.
struct ModelDev {
  const uint2* w1 = nullptr;  // [64 lanes][4 ob]      (inputs padded 7 -> 16)
  const uint2* w2 = nullptr;  // [4 ob][64 lanes][4 kb]
  const uint2* w3 = nullptr;  // [2 ob][64 lanes][4 kb]
  const float* b1 = nullptr;  // [64]
  const float* b2 = nullptr;  // [64]
  const float* b3 = nullptr;  // [32]
};
constexpr int kModelW1 = 4 * 64, kModelW2 = 16 * 64, kModelW3 = 8 * 64;  // uint2 fragments
constexpr size_t kModelBytes = (size_t)(kModelW1 + kModelW2 + kModelW3) * 8 + 160 * 4;

// History node: written once per Kalman update (the filtered state there).
struct alignas(16) Node {
  int parent;
  int meas;
  int surface;
  int pad;
  double p[5];
  double cov[15];
};
static_assert(sizeof(Node) == 176, "node record");

// Candidate pool record (array of structs per workgroup): doubles, ints, floats.
enum PoolD { PD_P = 0, PD_C = 5, PD_CHI2 = 20, PD_N = 21 };
enum PoolI { PI_SURF = 0, PI_SLOT, PI_NODE, PI_NMH, PI_MASK_LO, PI_MASK_HI, PI_LIST, PI_NLIST = PI_LIST + kMaxList, PI_N };
enum PoolF { PF_H = 0, PF_PATH, PF_N };
constexpr size_t kRecBytes = PD_N * 8 + PI_N * 4 + PF_N * 4;
constexpr size_t kRecStride = (kRecBytes + 15) / 16 * 16;  // array-of-structs record stride

// The seed list is split into kSeedQueues equal parts, one per XCD: a
// workgroup takes seeds from the part of its own XCD (workgroups are dealt to
// the 8 XCDs round-robin by index) and, when that part is used up, from the
// next ones.  Seeds of one part are neighbours in the caller's order (for
// seeds listed by event, a few events), so each XCD's L2 holds the
// measurements of its own events.
constexpr int kSeedQueues = 8;

struct Workspace {
  // carved from the caller's workspace
  float4* m_sorted;  // (loc0, loc1, var0, var1) sorted by loc0 within each row
  float* m_key;      // the sorted loc0 keys alone (the window search reads 16 per cache line)
  int* m_id;         // caller's id of each sorted measurement
  int* row_of;
  float* row_maxvar0;
  Node* nodes;
  long long node_cap;
  unsigned long long* node_count;
  int* queue_head;  // kSeedQueues heads, one per part of the seed list
  int* res_node;
  int* res_nm;
  int* res_holes;
  double* res_chi2;
  int* scan_a;      // per-block sums for the output scan
  int* scan_b;
  // every finished candidate (tracks_per_seed = 0): seed, last node, counts
  // (n_meas | holes << 16), chi2; per-seed counts and the records by seed
  int* fin_seed;
  int* fin_node;
  int* fin_nmh;
  double* fin_chi2;
  unsigned long long* fin_count;
  long long fin_cap;
  int* seed_cnt;
  int* seed_meas;
  int* seed_fill;
  int* fin_order;
  char* pools;      // per-workgroup candidate pools
  int pool_cap;     // records per pool
  int seeds_per_group;
  int grid;
};

struct Launch {
  int grid;
  int seeds_per_group;
  int pool_cap;
  int nodes_per_seed;
  int waves_per_simd;
};

}  // namespace ckf
