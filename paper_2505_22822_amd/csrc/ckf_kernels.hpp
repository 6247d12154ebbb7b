// Kernel argument blocks and host-side launchers.
#pragma once
#include "ckf_internal.hpp"

namespace ckf {

struct MeasIn {
  int n_events, n_surfaces;
  long long n_meas;
  const int* offsets;
  const float* loc;
  const float* var;
};

struct SeedsIn {
  int n;
  const int* event;
  const int* surface;
  const double* params;
  const double* cov;
};

struct CellsIn {
  int n_events, n_surfaces;
  long long n_cells;
  const int* offsets;
  const int* c0;
  const int* c1;
  const float* q;
};

struct CkfArgs {
  GeomDev g;
  FieldDev f;
  CfgDev cfg;
  MeasIn m;
  SeedsIn s;
  Workspace w;
  int* status;
  long long* counters;
  bool learned;       // the learned-proposal form (model valid)
  ModelDev model;
  int* seed_flags;    // audit output of the instrumented learned form, or null
};

hipError_t launch_init(int n_seeds, const Workspace& w, const ckf_tracks& out, hipStream_t st);
hipError_t launch_meas_prepare(const MeasIn& m, const Workspace& w, int* status, hipStream_t st);
hipError_t launch_ckf(const CkfArgs& a, int waves_per_simd, hipStream_t st);
hipError_t launch_output(int n_seeds, const Workspace& w, const int* seed_event, const ckf_tracks& out,
                         hipStream_t st);
// tracks_per_seed = 0: every finished candidate, by seed, in rank-key order
hipError_t launch_output_all(int n_seeds, const Workspace& w, const int* seed_event, const ckf_tracks& out,
                             hipStream_t st);
hipError_t launch_propagate(const GeomDev& g, const FieldDev& f, const CfgDev& c, int n, const int* src,
                            const double* p_in, const double* cov_in, const int* dst, double* p_out,
                            double* cov_out, double* jac, double* path, int* ok, hipStream_t st);
hipError_t launch_model_pack(const float* params, void* out, hipStream_t st);
ModelDev model_view(const void* buf);
hipError_t launch_mlp_forward(const ModelDev& M, const float* x, long long n, float* logits, hipStream_t st);
size_t mlp_workspace_bytes(long long n);
hipError_t launch_mlp_grad(const float* params, const float* x, const int* labels, const int* rows, long long n,
                           void* ws, float* grad, float* loss, hipStream_t st);
hipError_t launch_mlp_adam(float* params, float* m, float* v, const float* grad, int step, float lr, float b1,
                           float b2, float eps, hipStream_t st);
size_t capture_workspace_bytes(int cap_tracks);
hipError_t launch_capture_pairs(const GeomDev& g, const FieldDev& f, const int* n_tracks, int cap_tracks, const int* off,
                                const int* msurf, const double* mpar, long long cap_pairs, float* x, int* label,
                                int* track, long long* counts, void* ws, hipStream_t st);
size_t fit_workspace_bytes(long long cap_meas);
constexpr int kMaxDevices = 64;
// Device address and size of this GPU's fit scratch array (looked up once per
// device, on the first call with that device current).
hipError_t fit_scratch(void** ptr, size_t* bytes);
size_t seed_workspace_bytes(long long rows, long long n_sp, int n_events, int n_layers);
int seed_top_cap_max();
long long seed_bin_count(int n_events, int n_layers);  // (event, layer, phi bin, z bin) bins
void seed_set_top_cap(int cap);
hipError_t launch_seed(const GeomDev& g, int n_events, int n_surfaces, const int* moff, long long n_sp,
                       const float* xyz, const float* loc, const int* layers, int n_layers, double bz, void* ws,
                       long long cap, int* n_seeds, int* event, int* surface, double* params, double* cov,
                       int* sp_ids, long long* counters, hipStream_t st);
size_t cluster_workspace_bytes(long long rows, long long n_cells);
hipError_t launch_cluster(const CellsIn& c, const GeomDev& g, const float* pitch, void* ws, int* moff, float* loc,
                          float* var, float* sp, int* cell_cluster, int* status, hipStream_t st);
size_t resolve_workspace_bytes(int cap_tracks, long long n_meas);
hipError_t run_resolve(const int* n_tracks, int cap_tracks, long long cap_meas, const int* off, const int* meas,
                       long long n_meas, const double* chi2, const int* ndf, int max_shared, int max_rounds, void* ws,
                       int* keep, int* info, hipStream_t st);
hipError_t launch_fit(const GeomDev& g, const FieldDev& f, const CfgDev& cfg, const MeasIn& m, const SeedsIn& s,
                      const int* n_tracks, int cap_tracks, long long cap_meas, const int* off, const int* meas,
                      const int* msurf, const int* seed, bool two_filter, void* ws, double* out_p, double* out_C,
                      double* chi2, int* ok, hipStream_t st);
hipError_t launch_kf_update(int n, const double* p_in, const double* cov_in, const float* meas, const float* var,
                            double* p_out, double* cov_out, double* chi2, hipStream_t st);

}  // namespace ckf
