// Kernel argument blocks and launchers (library-internal).
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace chimera {

constexpr int kEventBS = 512;   // threads per (event, lambda) workgroup
constexpr int kEventSPT = 12;   // samples per thread held in registers

struct EventArgs {
  const LamParams* P;
  const int* flag_mono;
  const int* flag_range;
  const double2* chi;
  const double2* inv;
  Geometry g;
  const double* gz64;
  const float* gz32;
  const double* nz64;
  const float* nz32;
  const int* ev_samp_off;   // [E+1]
  const double* dl;
  const double* lndl;
  const double* m1d;
  const double* m2d;
  const double* lnm1d;
  const double* lnm2d;
  const int* samp_row;      // catalogue row of each sample
  const double* samp_c;     // c_ir of each sample's pixel
  int E, B;
  double trunc;
  int nchunk, bc;           // lambda chunking of the XCD-aware block order
  double* lnI;              // [B][E]
};

struct SelArgs {
  const LamParams* P;
  const int* flag_mono;
  const int* flag_range;
  const double2* chi;
  const double2* inv;
  Geometry g;
  const double* ntot;
  const double* dl;
  const double* lndl;
  const double* m1d;
  const double* m2d;
  const double* lnm1d;
  const double* lnm2d;
  const double* ln_pdraw;
  long long n_det;
  long long n_total;
  int B;
  int nchunk;
  double* partial;          // [B][nchunk][2]
};

hipError_t launch_tables(const double* lam, int B, const Geometry& g, LamParams* P, double2* chi,
                         double2* inv, double* gz64, float* gz32, int* flag_mono,
                         int* flag_range, hipStream_t st);
hipError_t launch_events(const EventArgs& a, bool f32, hipStream_t st);
hipError_t launch_selection(const SelArgs& a, bool f32, double* ln_xi, double* neff,
                            hipStream_t st);
hipError_t launch_lnl_final(const LamParams* P, const int* flag_mono, const int* flag_range,
                            const double* lnI, const double* ln_xi, int E, int B, double* lnl,
                            hipStream_t st);
int event_max_samples();
int selection_chunks(long long n_det);

}  // namespace chimera
