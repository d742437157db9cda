// Kernel argument blocks and launchers (library-internal).
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace chimera {

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

// grouped event kernel (event_grouped.hip)
constexpr int kGroupBS = 1024;           // threads per (event, lambda) workgroup
constexpr int kGroupK = 8;               // samples per group (Horner chains per lane)
constexpr int kGroupFBytes64 = 96 * 1024;  // LDS for the staged F slice, FP64 path
constexpr int kGroupFBytes32 = 96 * 1024;  // ... FP32 path
constexpr int kGroupGCap = 2048;         // entries of the G_m table
constexpr int kGroupMaxPerEvent = kGroupBS;   // one group per thread
// samples of one event, kept as (z, w) in the F region during phase 1
constexpr int kGroupMaxSamples = kGroupFBytes64 / 16 < kGroupFBytes32 / 16 ? kGroupFBytes64 / 16 : kGroupFBytes32 / 16;

struct GroupedArgs {
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
  const int* ev_grp_off;    // [E+1] groups of each event
  const int* ev_samp_off;   // [E+1] samples of each event (group order)
  const int* ev_slot_off;   // [E+1] pixel slots of each event
  const int* slot_row;      // catalogue row of each pixel slot
  const int* grp_first;     // first sample of each group
  const int* grp_cnt;       // samples in the group (<= kGroupK)
  const int* grp_slot;      // pixel slot of the group, relative to its event
  const double* grp_c;      // c_ir of the group's pixel
  const double* dl;         // samples in group order
  const double* lndl;
  const double* m1d;
  const double* m2d;
  const double* lnm1d;
  const double* lnm2d;
  int E, B;
  double trunc;
  int nchunk, bc;
  int f_bytes, g_cap;
  double* lnI;
  unsigned long long* count;
};

hipError_t launch_events_grouped(const GroupedArgs& a, bool f32, int max_groups, hipStream_t st);

hipError_t launch_tables(const double* lam, int B, const Geometry& g, LamParams* P, double2* chi,
                         double2* inv, double* gz64, float* gz32, int* flag_mono,
                         int* flag_range, hipStream_t st);
hipError_t launch_selection(const SelArgs& a, bool f32, double* ln_xi, double* neff,
                            hipStream_t st);
hipError_t launch_lnl_final(const LamParams* P, const int* flag_mono, const int* flag_range,
                            const double* lnI, const double* ln_xi, int E, int B, double* lnl,
                            hipStream_t st);
int selection_chunks(long long n_det);

}  // namespace chimera
