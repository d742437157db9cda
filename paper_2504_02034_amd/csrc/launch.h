// Kernel argument blocks and launchers (library-internal).
#pragma once

#include <hip/hip_runtime.h>

#include "chimera.h"
#include "common.h"

namespace chimera {

#define CH_LAUNCH_CHECK()                        \
  do {                                           \
    hipError_t _e = hipGetLastError();           \
    if (_e != hipSuccess) return _e;             \
  } while (0)

// XCD-aware block order for the per-(item, lambda) kernels: the blocks of one
// item (event or work unit) at 32 consecutive lambdas land on one XCD (block
// id mod 8) back to back, so the item's data stay in that XCD's L2.
__device__ __forceinline__ bool decode_item_lambda(int n_items, int B, int& item, int& b) {
  const int bc = B < 32 ? B : 32;
  const int nchunk = (B + bc - 1) / bc;
  const int L = blockIdx.x;
  const int xcd = L & 7, s = L >> 3;
  const int u = (s / bc) * 8 + xcd;
  item = u / nchunk;
  b = (u % nchunk) * bc + (s % bc);
  return item < n_items && b < B;
}

inline long long item_lambda_blocks(int n_items, int B) {
  const int bc = B < 32 ? B : 32;
  const long long nchunk = (B + bc - 1) / bc;
  const long long units = (long long)n_items * nchunk;
  return ((units + 7) / 8) * 8 * bc;
}

struct SelArgs {
  const LamParams* P;
  const int* flag_mono;
  const int* flag_range;
  const double2* chi;
  const double2* inv;
  Geometry g;
  const double* ntot;       // [n_z], or [B][n_z] when ntot_stride = n_z (incompleteness)
  long long ntot_stride;
  const double2* mtab;      // [B][kMassPanels + 1] smoothed-edge tables (delta_m > 0)
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

// event kernels (event.hip)
constexpr int kZwBS = 256;               // k_event_zw: threads per (event, lambda)
constexpr int kSmBS = 256;               // k_event_smooth: one sample group per thread
constexpr int kGroupK = 8;               // samples per group (Horner chains per lane)
constexpr int kUnitGroups = kSmBS;       // groups per work unit (chunk of one event)
// LDS for the staged F slice: FP64 35.5 KB, FP32 36 KB; with the G_m table
// and the kernel's static arrays (< 512 B) four workgroups fit in a CU's
// 160 KB, as the registers allow
constexpr int kSmFBytes64 = 35 * 1024 + 512;
constexpr int kSmFBytes32 = 36 * 1024;
constexpr int sm_fbytes(bool f32) { return f32 ? kSmFBytes32 : kSmFBytes64; }
constexpr int kSmGCap = 512;             // entries of the G_m table
static_assert(4 * (kSmFBytes64 + kSmGCap * (int)sizeof(double) + 512) <= 160 * 1024, "LDS");
static_assert(4 * (kSmFBytes32 + kSmGCap * (int)sizeof(float) + 512) <= 160 * 1024, "LDS");
// per-sample gradient coefficients: z and c w (double), then d ln w / dp (9)
// and dz / dp (4) (double, or float in FP32 mode)
constexpr int kGradSampleFields = 15;
constexpr int kGradDerivFields = 13;
inline double grad_sample_bytes(bool f32) { return 16.0 + kGradDerivFields * (f32 ? 4.0 : 8.0); }
// every pixel row of an event needs a row of >= 2 slots in the F slice (the
// slice and G share the pool).  FP32 holds every accepted event; FP64 holds
// 2048 rows with a full G table, and a larger event whose rows and G do not
// fit takes the direct sums
static_assert(CHIMERA_MAX_EVENT_PIXELS * 2 * (int)sizeof(float) <= kSmFBytes32, "F slice too small");
static_assert(2048 * 2 * (int)sizeof(double) <= kSmFBytes64, "F slice too small");

struct EventArgs {
  const LamParams* P;
  const int* flag_mono;
  const int* flag_range;
  const double2* chi;
  const double2* inv;
  const double2* dtab;      // [B][n_t] (d_L^gw, dd_L^gw/dx) on the x nodes
  const double2* mtab;      // [B][kMassPanels + 1] smoothed-edge tables (delta_m > 0)
  double* wscale;           // [B][E] ln of the FP32 weights' scale (FP32 with delta_m), or null
  Geometry g;
  const double* gz64;
  const float* gz32;
  const double* nz64;
  const float* nz32;
  // incompleteness (null without it): 1 - P_compl per row, and the grid
  // factor times the completion density (the grid factor itself is then
  // scaled by f_R), F = n_r gz + (1 - P_r) gzb
  const double* mz64;
  const float* mz32;
  const double* gzb64;
  const float* gzb32;
  // event set
  const int* ev_samp_off;   // [E+1] samples of each event (group order)
  const int* ev_slot_off;   // [E+1] pixel slots of each event
  const int* ev_unit_off;   // [E+1] work units of each event
  const int* slot_row;      // catalogue row of each pixel slot
  const int* grp_first;     // first sample (absolute) of each group
  const int* grp_cnt;       // samples in the group (<= kGroupK)
  const int* grp_slot;      // pixel slot of the group, relative to its event
  const double* grp_c;      // c_ir of the group's pixel
  const int* unit_event;    // [U] event of each unit
  const int* unit_grp0;     // [U] first group (absolute) of each unit
  const int* unit_ngrp;     // [U] groups in each unit (<= kUnitGroups)
  const double* dl;         // samples in group order
  const double* lndl;
  const double* m1d;
  const double* m2d;
  const double* lnm1d;
  const double* lnm2d;
  int E, U, B;
  long long S;
  double trunc;
  // scratch
  double* zbuf;             // [B][S] redshift of each sample
  void* wbuf;               // [B][S] mass weight (double, or float in FP32 mode)
  double* hbuf;             // [B][E] bandwidth (<= 0: no weight in the event)
  double* part;             // [B][U] partial kernel sums
  double* lnI;              // [B][E]
  unsigned long long* count;  // pairs evaluated, while profiling (else null)
  long long* pcount;        // [B][U] pairs per (unit, lambda), summed into count
  // kernel options of Sect. 2.3
  int shape;                // kShapeGaussian / kShapeEpanechnikov
  int n_bins;               // 0, or bins per pixel slot
  int n_slots;              // pixel slots of the set
  const int* pix_off;       // [n_slots+1] samples of each slot in pix_idx
  const int* pix_idx;       // sample positions (group order) of each slot, by distance
  const double* slot_c;     // [n_slots] c_ir of each slot
  const int* slot_event;    // [n_slots] event of each slot
  // the 3D kernel: samples in a flat sky chart, pixel centres and areas, and
  // the (pixel, sample) points of each event, pixel-major
  const double* su;         // [S] chart coordinates of each sample (group order)
  const double* sv;
  const double* pu;         // [pixels] centre of each pixel in its event's chart
  const double* pv;
  const long long* virt_off;  // [E+1] first (pixel, sample) point of each event
  long long V;              // (pixel, sample) points of the set (0: not a 3D set)
  double* p3;               // [B][E][8] B_u, B_v, H_OO^-1 (uu, uv, vv), ln N2 norm
  double* z3;               // [B][V] z_j + B . dO of each point
  void* w3;                 // [B][V] w_j N2(dO; H_OO) (double, or float in FP32 mode)
  double* bz;               // [B][n_slots n_bins] bin centres
  void* bw;                 // [B][n_slots n_bins] bin weights (double, or float in FP32 mode)
};

enum : int { kShapeGaussian = 0, kShapeEpanechnikov = 1 };
constexpr double kEpanScale = 2.23606797749978969641;   // sqrt(5): support / bandwidth
constexpr int kEpBS = 256;               // k_event_epan: one pixel slot per wave, four per group
constexpr int kEpCap = 256;              // grid points of one staged prefix chunk per wave
constexpr int kBinBS = 256;              // k_event_bin: one pixel slot per wave

// The forward event kernels in order: k_event_zw on the samples (z, w, h);
// for a 3D set (a.V > 0) k_event_cov3d and k_event_expand3d, with `a`
// carrying the set's pixels as slots;
// with bins k_event_bin; then the smoothing kernel (Gaussian: over the
// samples, or over the bins with `kern` laid out on them) or k_event_epan
// (Epanechnikov, one partial per pixel slot: `kern` has U = n_slots and the
// slots as units), then k_event_final.  t0 / t1 bracket the dominant kernel.
hipError_t launch_events(const EventArgs& a, const EventArgs& kern, bool f32, hipStream_t st,
                         hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);

// static scratch of the allocation-free entry point (noalloc.hip): 256 MiB
// per device, lambda points run in chunks that fit it
constexpr size_t kStaticScratchBytes = size_t(256) << 20;
hipError_t static_scratch_address(void** ptr);

// lam rows of `stride` entries (kNlam, or kNlam + 1 with delta_m); mtab
// [B][kMassPanels + 1] when any point may carry delta_m > 0, else null
hipError_t launch_tables(const double* lam, int stride, int B, const Geometry& g, LamParams* P,
                         double2* mtab, double2* chi, double2* inv, double2* dtab, double* gz64,
                         float* gz32, int* flag_mono, int* flag_range, hipStream_t st);
hipError_t launch_selection(const SelArgs& a, bool f32, double* ln_xi, double* neff,
                            hipStream_t st);
hipError_t launch_lnl_final(const LamParams* P, const int* flag_mono, const int* flag_range,
                            const double* lnI, const double* ln_xi, const double* neff,
                            double neff_gate, int E, int B, double* lnl, hipStream_t st);
int selection_chunks(long long n_det);

// ---------------------------------------------------------------------------
// adjoint (grad.hip)
// ---------------------------------------------------------------------------
// Per-lambda constants of the mass-model derivatives.
struct GradParams {
  double pl_unit;          // 1 / int_mmin^mmax m^-alpha dm
  double tg_unit;          // 1 / (sigma sqrt(2 pi) Z)
  double dlnnpl_dalpha;    // d ln int m^-alpha dm / d alpha
  double dlnz_dmu, dlnz_dsigma;
};

struct GradArgs {
  const LamParams* P;
  GradParams* Q;            // written by the prepare kernel
  const int* flag_mono;
  const int* flag_range;
  const double2* chi;
  const double2* chio;      // [B][n_t] (dchi/dOm, its x-derivative)
  const double2* inv;
  const double2* dtab;
  Geometry g;
  const double* gz64;
  const float* gz32;
  double* gf64;             // [B][6][n_z] g dln g/dp, p = Om, Xi0, n, gamma, kappa, z_p
  float* gf32;
  const double* nz64;
  const float* nz32;
  // incomplete catalogue (null otherwise): the rows' 1 - P_compl and, per
  // lambda, the completion density v and (dv/dOm) g on the grid, f_R, df_R/dOm
  const double* mz64;
  const float* mz32;
  double* cv64;             // [B][2][n_z]
  float* cv32;
  double* cf;               // [B][2]
  const int* ev_samp_off;
  const int* samp_row;      // catalogue row of each sample
  const double* samp_c;     // c_ir of each sample's pixel
  const double* dl;
  const double* lndl;
  const double* m1d;
  const double* m2d;
  const double* lnm1d;
  const double* lnm2d;
  int E, B;
  double trunc;
  int shape;                // kShapeGaussian / kShapeEpanechnikov
  // binned data sets (bins > 0: bins per pixel slot): the slots' samples by
  // distance, each slot's row, and per (lambda, bin) the bin's point and
  // derivative coefficients in the layout of sc / sd (k_bin_grad)
  int bins;
  int n_slots;
  const int* ev_slot_off;   // [E+1]
  const int* slot_row;      // [n_slots]
  const int* pix_off;       // [n_slots+1]
  const int* pix_idx;       // sample positions of each slot, by distance
  double* bsc;              // [B][2][n_slots bins]
  void* bsd;                // [B][13][n_slots bins]
  double* hd;               // [B][E][10] h and d ln h/dp (written by the bandwidth kernel)
  double* sc;               // [B][2][S] z and c w of each sample (bandwidth kernel)
  void* sd;                 // [B][13][S] d ln w/dp, dz/dp: double, or float when f32
  int f32;
  long long S;              // samples of the event set
  double* lnI;              // [B][E]
  double* dlnI;             // [B][E][12]
};

struct SelGradArgs {
  const LamParams* P;
  const GradParams* Q;
  const int* flag_mono;
  const int* flag_range;
  const double2* chi;
  const double2* chio;
  const double2* inv;
  const double2* dtab;
  Geometry g;
  const double* ntot;       // [n_z], or [B][n_z] when ntot_stride = n_z (incompleteness)
  long long ntot_stride;
  const double* dntot_om;   // [B][n_z] d n_tot / d Om (incompleteness), or null
  const double* dl;
  const double* lndl;
  const double* m1d;
  const double* m2d;
  const double* lnm1d;
  const double* lnm2d;
  const double* ln_pdraw;
  long long n_det;
  int B;
  int nchunk;
  double* partial;          // [B][nchunk][13]: sum s, sum s dln s/dp
};

struct GradFinalArgs {
  const LamParams* P;
  const int* flag_mono;
  const int* flag_range;
  const double* partial;
  int nchunk;
  const double* lnI;
  const double* dlnI;
  int E;
  long long n_total;
  double neff_gate;         // > 0: ln L = -inf where N_eff <= neff_gate x E
  double* lnl;              // [B]
  double* grad;             // [B][12]
};

// The effective number of injections of Sect. 2.2 from sum s and sum s^2.
__host__ __device__ inline double neff_of(double s1, double s2, long long n_total) {
  const double dd = s2 - s1 * s1 / (double)n_total;
  return s1 > 0.0 ? (dd > 0.0 ? s1 * s1 / dd : INFINITY) : 0.0;
}

hipError_t launch_chi_om_table(const LamParams* P, int B, const Geometry& g, double2* chio,
                               hipStream_t st);
// With an incomplete catalogue (a.mz64 set) ntot / missing are the catalogue's
// n_tot and M(z), and sa.ntot / sa.dntot_om receive the per-lambda n_tot^eff
// and its Om derivative.
hipError_t launch_grad(const GradArgs& a, const SelGradArgs& sa, GradFinalArgs fa, bool f32,
                       hipStream_t st, const double* ntot = nullptr,
                       const double* missing = nullptr);
int selection_grad_chunks(long long n_det);

// ---------------------------------------------------------------------------
// catalogue density (catalog.hip)
// ---------------------------------------------------------------------------
struct CatalogGrid {
  int n_z;
  double z_lo, z_hi, dz;
};

struct CatalogArgs {
  const long long* off;     // [n_pix+1] galaxies of pixel p: [off[p], off[p+1])
  const double* mu;         // [n_gal] observed redshift, sorted by pixel
  const double* sig;        // [n_gal] redshift uncertainty
  double* norm;             // [n_gal] sum_k J_k V_k (written)
  CatalogGrid g;
  const double* vshape;     // [n_z] comoving volume element shape V_k
  long long n_gal, n_pix;
  double* rows_all;         // [n_pix][n_z] (written)
  const long long* rows_pix;// [n_rows] pixel of each catalogue row
  long long n_rows;
  double pixel_area;
  double* ntot;             // [n_z]
  double* nz64;             // [n_rows][n_z]
  float* nz32;
};

hipError_t launch_catalog(const CatalogArgs& c, hipStream_t st);
hipError_t launch_catalog_finish(const CatalogArgs& c, long long n_used, hipStream_t st);

// Single-1D event rows from the catalogue rows (catalog.hip).
struct FoldArgs {
  const int* pix_off;       // [n_ev+1] pixels of event e: [pix_off[e], pix_off[e+1])
  const int* row;           // [P] catalogue row of each pixel
  const double* s;          // [P] sky factor S_ir of each pixel
  int n_ev, n_z;
  const double* nz64;       // [n_rows][n_z] catalogue rows
  double* out64;            // [n_ev][n_z] (written)
  float* out32;             // [n_ev][n_z] (written)
  const double* mz64;       // [n_rows][n_z] 1 - P_compl (null: none)
  double* mout64;           // [n_ev][n_z] folded 1 - P_compl (written when mz64)
  float* mout32;
};

// Incompleteness (eqs. p-gal, p-miss, f-R) per lambda: the completion density
// v(z_g) = chi^2 / (E (4 pi / 3) chi(z_max)^3), f_R = sum_g tau_g (4 pi - M_g) v_g,
// n_tot^eff = f_R n_tot + M v into ntot_eff[B][n_z]; with gz64 (an event call)
// gzb = v gz and then gz *= f_R (both precisions).  One workgroup per lambda.
hipError_t launch_completion(const LamParams* P, const double2* chi, const Geometry& g, int B,
                             const double* ntot, const double* missing, double* ntot_eff,
                             double* gz64, float* gz32, double* gzb64, float* gzb32,
                             hipStream_t st);

hipError_t launch_fold_rows(const FoldArgs& f, hipStream_t st);

}  // namespace chimera
