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

struct CkfArgs {
  GeomDev g;
  FieldDev f;
  CfgDev cfg;
  MeasIn m;
  SeedsIn s;
  Workspace w;
  int* status;
  long long* counters;
};

hipError_t launch_init(int n_seeds, const Workspace& w, const ckf_tracks& out, hipStream_t st);
hipError_t launch_meas_prepare(const MeasIn& m, const Workspace& w, int* status, hipStream_t st);
hipError_t launch_ckf(const CkfArgs& a, int waves_per_simd, hipStream_t st);
hipError_t launch_output(int n_seeds, const Workspace& w, const int* seed_event, const ckf_tracks& out,
                         hipStream_t st);
hipError_t launch_propagate(const GeomDev& g, const FieldDev& f, const CfgDev& c, int n, const int* src,
                            const double* p_in, const double* cov_in, const int* dst, double* p_out,
                            double* cov_out, double* jac, double* path, int* ok, hipStream_t st);
hipError_t launch_kf_update(int n, const double* p_in, const double* cov_in, const float* meas, const float* var,
                            double* p_out, double* cov_out, double* chi2, hipStream_t st);

}  // namespace ckf
