// Host side of the C-ABI in include/chimera.h: argument checks, resident
// device data, per-call scratch (stream-ordered allocations) and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "chimera.h"
#include "launch.h"

using namespace chimera;

namespace {

thread_local std::string g_err;

// Device address of each GPU's copy of the static scratch (noalloc.hip),
// looked up once per device by chimera_create with that device current.
std::mutex g_static_mu;
std::map<int, void*> g_static_ptr;

chimera_status fail(chimera_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(e_ == hipErrorOutOfMemory ? CHIMERA_ENOMEM : CHIMERA_EDEVICE,         \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                   \
  } while (0)

template <class T>
hipError_t upload(T** dst, const T* src, size_t n) {
  *dst = nullptr;
  if (n == 0) return hipSuccess;
  hipError_t e = hipMalloc((void**)dst, n * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

bool finite_positive(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!(std::isfinite(v[i]) && v[i] > 0.0)) return false;
  return true;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Scratch is held per stream in power-of-two sizes (at least 1 MiB), so that
// calls of varying batch size on a stream reuse one block.
size_t pool_size(size_t bytes) {
  size_t a = size_t(1) << 20;
  while (a < bytes) a <<= 1;
  return a;
}

// Bump allocator over one device block.
struct Carve {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    T* p = reinterpret_cast<T*>(base + off);
    off += align_up(n * sizeof(T));
    return p;
  }
};

}  // namespace

struct chimera_events {
  int E = 0;
  int64_t n_samp = 0;
  int U = 0;
  int* ev_samp_off = nullptr;
  int* ev_slot_off = nullptr;
  int* ev_unit_off = nullptr;
  int* slot_row = nullptr;
  int *unit_event = nullptr, *unit_grp0 = nullptr, *unit_ngrp = nullptr;
  // per group
  int *grp_first = nullptr, *grp_cnt = nullptr, *grp_slot = nullptr;
  double* grp_c = nullptr;
  // samples in group order
  double *dl = nullptr, *lndl = nullptr, *m1d = nullptr, *m2d = nullptr;
  double *lnm1d = nullptr, *lnm2d = nullptr;
  int* samp_row = nullptr;      // catalogue row of each sample (adjoint)
  double* samp_c = nullptr;     // c_ir of each sample's pixel (adjoint)
  double dmin = 0.0, dmax = 0.0;
  int64_t rows_needed = 0;      // 1 + the largest catalogue row the set refers to
  // single-1D sets (eq. gw-kernel-single1d): one pseudo-pixel per event whose
  // row is the event's pixels' sky factors folded into the catalogue rows,
  // sum_p S_p n_{row_p}(z); folded at creation and again whenever the
  // catalogue is replaced.  slot_row / samp_row index these rows.
  bool single1d = false;
  int* fold_pix_off = nullptr;  // [E+1]
  int* fold_row = nullptr;      // [P] catalogue row of each pixel
  double* fold_s = nullptr;     // [P] sky factor of each pixel
  double* own64 = nullptr;      // [E][n_z]
  float* own32 = nullptr;
  double* ownm64 = nullptr;     // [E][n_z] the same fold of 1 - P_compl
  float* ownm32 = nullptr;
  // kernel options (chimera_set_event_kde, Sect. 2.3)
  int P = 0;                    // pixel slots
  int shape = 0, n_bins = 0;
  int* pix_off = nullptr;       // [P+1] samples of each slot in pix_idx
  int* pix_idx = nullptr;       // [n_samp] sample positions of each slot, by distance
  double* slot_c = nullptr;     // [P] c_ir of each slot
  int* slot_event = nullptr;    // [P] event of each slot
  // work layout over the bins: groups of <= kGroupK consecutive bins of a slot
  // the 3D kernel: the unique samples form one slot per event (the sample
  // transform and the bandwidth moments); the real pixels and the
  // (pixel, sample) points of the 1-D sums are below
  int64_t V = 0;                // (pixel, sample) points
  int Uv = 0;
  long long* virt_off = nullptr;  // [E+1]
  double *su = nullptr, *sv = nullptr;  // [n_samp] chart coordinates (group order)
  double *pu = nullptr, *pv = nullptr;  // [pixels] centres in the chart
  int *d3_slot_off = nullptr, *d3_slot_row = nullptr;
  int *v_ev_unit_off = nullptr, *v_unit_event = nullptr, *v_unit_grp0 = nullptr,
      *v_unit_ngrp = nullptr, *v_grp_first = nullptr, *v_grp_cnt = nullptr,
      *v_grp_slot = nullptr;
  double* v_grp_c = nullptr;
  std::vector<int> h_slot_off;   // host copies: slots of each event, c_ir of each slot
  std::vector<double> h_slot_c;
  int Ub = 0;
  int *b_ev_unit_off = nullptr, *b_unit_event = nullptr, *b_unit_grp0 = nullptr,
      *b_unit_ngrp = nullptr, *b_grp_first = nullptr, *b_grp_cnt = nullptr,
      *b_grp_slot = nullptr;
  double* b_grp_c = nullptr;
};

struct chimera_ctx {
  chimera_config cfg;
  std::mutex mu;
  int64_t n_rows = 0;
  double* nz64 = nullptr;
  float* nz32 = nullptr;
  double* ntot = nullptr;
  int64_t n_det = 0, n_inj_total = 0;
  double *inj_dl = nullptr, *inj_lndl = nullptr, *inj_m1d = nullptr, *inj_m2d = nullptr;
  double *inj_lnm1d = nullptr, *inj_lnm2d = nullptr, *inj_lnp = nullptr;
  double inj_dmin = 0.0, inj_dmax = 0.0;
  bool has_cat = false, has_inj = false;
  double neff_gate = 0.0;       // chimera_set_neff_gate
  std::atomic<int> nlam{CHIMERA_NLAM};  // lambda row width: +1 (delta_m) after chimera_set_mass_smoothing
  // incompleteness (chimera_set_completeness): 1 - P_compl per row, M(z)
  double* miss64 = nullptr;
  float* miss32 = nullptr;
  double* missing = nullptr;
  std::vector<chimera_events*> events;
  // per-stream scratch arenas (grown to the largest call on the stream; freed
  // by chimera_release_scratch or chimera_destroy).  A call holds its
  // stream's lock from taking the arena until its last enqueue (for host
  // calls until its results are back), so calls on one stream from several
  // host threads cannot interleave their use of the arena.
  struct Arena {
    void* p = nullptr;
    std::atomic<size_t> n{0};
    std::mutex mu;
  };
  std::map<hipStream_t, std::unique_ptr<Arena>> arenas;
  // diagnostics
  bool profile = false;
  unsigned long long* d_count = nullptr;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> marks;
};

namespace {

void free_bin_layout(chimera_events* ev) {
  dfree(ev->b_ev_unit_off); dfree(ev->b_unit_event); dfree(ev->b_unit_grp0);
  dfree(ev->b_unit_ngrp); dfree(ev->b_grp_first); dfree(ev->b_grp_cnt); dfree(ev->b_grp_slot);
  dfree(ev->b_grp_c);
  ev->b_ev_unit_off = ev->b_unit_event = ev->b_unit_grp0 = ev->b_unit_ngrp = nullptr;
  ev->b_grp_first = ev->b_grp_cnt = ev->b_grp_slot = nullptr;
  ev->b_grp_c = nullptr;
  ev->Ub = 0;
}

void free_events(chimera_events* ev) {
  dfree(ev->ev_samp_off); dfree(ev->ev_slot_off); dfree(ev->ev_unit_off); dfree(ev->slot_row);
  dfree(ev->unit_event); dfree(ev->unit_grp0); dfree(ev->unit_ngrp);
  dfree(ev->grp_first); dfree(ev->grp_cnt); dfree(ev->grp_slot); dfree(ev->grp_c);
  dfree(ev->dl); dfree(ev->lndl); dfree(ev->m1d); dfree(ev->m2d);
  dfree(ev->lnm1d); dfree(ev->lnm2d); dfree(ev->samp_row); dfree(ev->samp_c);
  dfree(ev->fold_pix_off); dfree(ev->fold_row); dfree(ev->fold_s);
  dfree(ev->own64); dfree(ev->own32); dfree(ev->ownm64); dfree(ev->ownm32);
  dfree(ev->pix_off); dfree(ev->pix_idx); dfree(ev->slot_c); dfree(ev->slot_event);
  dfree(ev->virt_off); dfree(ev->su); dfree(ev->sv); dfree(ev->pu); dfree(ev->pv);
  dfree(ev->d3_slot_off); dfree(ev->d3_slot_row);
  dfree(ev->v_ev_unit_off); dfree(ev->v_unit_event); dfree(ev->v_unit_grp0);
  dfree(ev->v_unit_ngrp); dfree(ev->v_grp_first); dfree(ev->v_grp_cnt); dfree(ev->v_grp_slot);
  dfree(ev->v_grp_c);
  free_bin_layout(ev);
  delete ev;
}

// The rows the kernels read for event set ev: its own folded rows for a
// single-1D set, else the catalogue's.
const double* rows64(const chimera_ctx* c, const chimera_events* ev) {
  return ev && ev->single1d ? ev->own64 : c->nz64;
}
const float* rows32(const chimera_ctx* c, const chimera_events* ev) {
  return ev && ev->single1d ? ev->own32 : c->nz32;
}
// 1 - P_compl rows for ev (null for a complete catalogue)
const double* miss64(const chimera_ctx* c, const chimera_events* ev) {
  if (!c->miss64) return nullptr;
  return ev && ev->single1d ? ev->ownm64 : c->miss64;
}
const float* miss32(const chimera_ctx* c, const chimera_events* ev) {
  if (!c->miss64) return nullptr;
  return ev && ev->single1d ? ev->ownm32 : c->miss32;
}

// Fold a single-1D set's rows from the current catalogue (and its
// completeness, if any) (ctx->mu held, device current); synchronous.
hipError_t fold_rows(const chimera_ctx* c, chimera_events* ev) {
  hipError_t e = hipSuccess;
  const size_t n = (size_t)ev->E * c->cfg.n_z;
  if (c->miss64 && !ev->ownm64) {
    e = hipMalloc((void**)&ev->ownm64, n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&ev->ownm32, n * sizeof(float));
    if (e != hipSuccess) return e;
  }
  FoldArgs f{ev->fold_pix_off, ev->fold_row, ev->fold_s, ev->E, c->cfg.n_z, c->nz64, ev->own64,
             ev->own32, c->miss64, ev->ownm64, ev->ownm32};
  e = launch_fold_rows(f, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return e;
}

void free_injections(chimera_ctx* c) {
  dfree(c->inj_dl); dfree(c->inj_lndl); dfree(c->inj_m1d); dfree(c->inj_m2d);
  dfree(c->inj_lnm1d); dfree(c->inj_lnm2d); dfree(c->inj_lnp);
  c->inj_dl = c->inj_lndl = c->inj_m1d = c->inj_m2d = nullptr;
  c->inj_lnm1d = c->inj_lnm2d = c->inj_lnp = nullptr;
  c->has_inj = false;
}

void free_completeness(chimera_ctx* c) {
  dfree(c->miss64); dfree(c->miss32); dfree(c->missing);
  c->miss64 = nullptr; c->miss32 = nullptr; c->missing = nullptr;
}

void free_catalog(chimera_ctx* c) {
  dfree(c->nz64); dfree(c->nz32); dfree(c->ntot);
  c->nz64 = nullptr; c->nz32 = nullptr; c->ntot = nullptr;
  c->has_cat = false;
  free_completeness(c);    // it belongs to the catalogue's rows
}

Geometry make_geometry(const chimera_ctx* c, double dmin, double dmax) {
  Geometry g;
  g.n_z = c->cfg.n_z;
  g.z_lo = c->cfg.z_lo;
  g.dz = (c->cfg.z_hi - c->cfg.z_lo) / (double)(c->cfg.n_z - 1);
  g.inv_dz = 1.0 / g.dz;
  g.n_t = c->cfg.n_tab;
  g.dx = std::log1p(c->cfg.z_tab_max) / (double)(g.n_t - 1);
  g.inv_dx = 1.0 / g.dx;
  g.n_u = c->cfg.n_tab;
  double ulo = std::log(dmin), uhi = std::log(dmax);
  if (uhi - ulo < 1e-6) {
    ulo -= 1e-3;
    uhi += 1e-3;
  }
  g.u_lo = ulo;
  g.du = (uhi - ulo) / (double)(g.n_u - 1);
  g.inv_du = 1.0 / g.du;
  return g;
}

struct Scratch {
  LamParams* P;
  double2* chi;
  double2* inv;
  double2* dtab;
  double* gz64;
  float* gz32;
  int* flag_mono;
  int* flag_range;
  double* partial;
  double* lam;
  double* lnI;
  double* ln_xi;
  double* neff;
  double* lnl;
  double* zbuf;
  void* wbuf;
  double* hbuf;
  double* part;
  long long* pcount;
  double* bz;
  void* bw;
  double* p3;
  double* z3;
  void* w3;
  double* ntot_eff;
  double* gzb64;
  float* gzb32;
  double2* mtab;
  double* wscale;
};

// Lay out (or size, when base is null) the scratch of one call.
size_t carve(Carve& cv, Scratch& s, const Geometry& g, int64_t B, int nchunk, bool need_lam,
             bool need_lnI, bool need_outs, const chimera_events* ev, bool f32,
             bool compl_ = false, int nlam = CHIMERA_NLAM) {
  const bool need_grid = ev != nullptr;
  const int E = ev ? ev->E : 0;
  const int64_t S = ev ? ev->n_samp : 0;
  // partial sums: one per work unit (samples or bins), or per event
  const int U = ev ? std::max(std::max(ev->U, ev->Ub), std::max(ev->P, ev->Uv)) : 0;
  const int64_t NB = ev && ev->n_bins ? (int64_t)ev->P * ev->n_bins : 0;
  const int64_t V = ev ? ev->V : 0;
  s.P = cv.take<LamParams>(B);
  s.chi = cv.take<double2>((size_t)B * g.n_t);
  s.inv = cv.take<double2>((size_t)B * g.n_u);
  s.dtab = need_grid ? cv.take<double2>((size_t)B * g.n_t) : nullptr;
  s.gz64 = need_grid ? cv.take<double>((size_t)B * g.n_z) : nullptr;
  s.gz32 = need_grid ? cv.take<float>((size_t)B * g.n_z) : nullptr;
  s.flag_mono = cv.take<int>(B);
  s.flag_range = cv.take<int>(B);
  s.partial = cv.take<double>((size_t)B * std::max(nchunk, 1) * 2);
  s.lam = need_lam ? cv.take<double>((size_t)B * nlam) : nullptr;
  s.mtab = nlam > CHIMERA_NLAM ? cv.take<double2>((size_t)B * (kMassPanels + 1)) : nullptr;
  s.wscale = nlam > CHIMERA_NLAM && f32 && S ? cv.take<double>((size_t)B * std::max(E, 1))
                                             : nullptr;
  s.lnI = need_lnI ? cv.take<double>((size_t)B * std::max(E, 1)) : nullptr;
  s.ln_xi = cv.take<double>(B);
  s.neff = cv.take<double>(B);
  s.lnl = need_outs ? cv.take<double>(B) : nullptr;
  s.zbuf = S ? cv.take<double>((size_t)B * S) : nullptr;
  s.wbuf = S ? (f32 ? (void*)cv.take<float>((size_t)B * S) : (void*)cv.take<double>((size_t)B * S))
             : nullptr;
  s.hbuf = S ? cv.take<double>((size_t)B * E) : nullptr;
  s.part = S ? cv.take<double>((size_t)B * std::max(U, 1)) : nullptr;
  s.pcount = S ? cv.take<long long>((size_t)B * std::max(U, 1)) : nullptr;
  s.bz = NB ? cv.take<double>((size_t)B * NB) : nullptr;
  s.bw = NB ? (f32 ? (void*)cv.take<float>((size_t)B * NB) : (void*)cv.take<double>((size_t)B * NB))
            : nullptr;
  s.ntot_eff = compl_ ? cv.take<double>((size_t)B * g.n_z) : nullptr;
  s.gzb64 = compl_ && need_grid ? cv.take<double>((size_t)B * g.n_z) : nullptr;
  s.gzb32 = compl_ && need_grid ? cv.take<float>((size_t)B * g.n_z) : nullptr;
  s.p3 = V ? cv.take<double>((size_t)B * E * 8) : nullptr;
  s.z3 = V ? cv.take<double>((size_t)B * V) : nullptr;
  s.w3 = V ? (f32 ? (void*)cv.take<float>((size_t)B * V) : (void*)cv.take<double>((size_t)B * V))
           : nullptr;
  return cv.off;
}

chimera_status check_common(chimera_ctx* ctx, const double* lam, int64_t B, int32_t prec,
                            int32_t mem) {
  if (!ctx) return fail(CHIMERA_EINVAL, "null context");
  if (!lam) return fail(CHIMERA_EINVAL, "null lambda pointer");
  if (B < 1 || B > (1 << 20)) return fail(CHIMERA_EINVAL, "batch size out of [1, 2^20]");
  if (prec != CHIMERA_FP64 && prec != CHIMERA_FP32) return fail(CHIMERA_EINVAL, "bad precision");
  if (mem != CHIMERA_HOST && mem != CHIMERA_DEVICE) return fail(CHIMERA_EINVAL, "bad mem kind");
  if (!ctx->has_inj) return fail(CHIMERA_ESTATE, "injections not set");
  if (!ctx->has_cat) return fail(CHIMERA_ESTATE, "catalogue not set");
  return CHIMERA_OK;
}

}  // namespace

extern "C" {

void chimera_default_config(chimera_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->n_z = 1000;
  cfg->z_lo = 0.0;
  cfg->z_hi = 1.6;
  cfg->n_tab = 8192;
  cfg->z_tab_max = 25.0;
  cfg->trunc_fp64 = 8.6;
  cfg->trunc_fp32 = 8.6;
  cfg->device = 0;
  cfg->hbm_budget = 0;
}

const char* chimera_last_error(void) { return g_err.c_str(); }

chimera_status chimera_create(const chimera_config* cfg, chimera_ctx** out) {
  if (!cfg || !out) return fail(CHIMERA_EINVAL, "null argument");
  *out = nullptr;
  if (cfg->n_z < 3 || !(cfg->z_hi > cfg->z_lo) || !(cfg->z_lo >= 0.0))
    return fail(CHIMERA_EINVAL, "grid needs n_z >= 3 and 0 <= z_lo < z_hi");
  if (cfg->n_tab < 256 || cfg->n_tab > 16 * 1024 + 1)
    return fail(CHIMERA_EINVAL, "n_tab must be in [256, 16385]");
  if (!(cfg->z_tab_max > cfg->z_hi)) return fail(CHIMERA_EINVAL, "z_tab_max must exceed z_hi");
  if (!(cfg->trunc_fp64 >= 8.6) || !(cfg->trunc_fp32 >= 3.0))
    return fail(CHIMERA_EINVAL, "trunc_fp64 must be >= 8.6 and trunc_fp32 >= 3");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (cfg->device < 0 || cfg->device >= ndev) return fail(CHIMERA_EINVAL, "no such device");
  HIP_TRY(hipSetDevice(cfg->device));
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr.count(cfg->device)) {
      void* p = nullptr;
      HIP_TRY(static_scratch_address(&p));
      g_static_ptr[cfg->device] = p;
    }
  }
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, cfg->device) == hipSuccess) {
    uint64_t thr = std::numeric_limits<uint64_t>::max();
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  auto* c = new chimera_ctx();
  c->cfg = *cfg;
  *out = c;
  return CHIMERA_OK;
}

void chimera_destroy(chimera_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->cfg.device);
  (void)hipDeviceSynchronize();
  for (auto& m : ctx->marks) {
    (void)hipEventDestroy(m.first);
    (void)hipEventDestroy(m.second);
  }
  dfree(ctx->d_count);
  for (auto& a : ctx->arenas) dfree(a.second->p);
  for (auto* e : ctx->events) free_events(e);
  free_catalog(ctx);
  free_injections(ctx);
  delete ctx;
}

namespace {

// A replacement catalogue must keep every row a resident event set refers to
// (call with ctx->mu held).
chimera_status check_resident_rows(const chimera_ctx* ctx, int64_t n_rows) {
  for (const auto* e : ctx->events)
    if (e->rows_needed > n_rows)
      return fail(CHIMERA_ERANGE, "a resident event set refers to catalogue rows past the new "
                                  "catalogue; release it first");
  return CHIMERA_OK;
}

// After a catalogue replacement: fold the rows of every resident single-1D
// set again (ctx->mu held).
chimera_status refold_all(chimera_ctx* ctx) {
  for (auto* e : ctx->events)
    if (e->single1d) {
      hipError_t er = fold_rows(ctx, e);
      if (er != hipSuccess)
        return fail(CHIMERA_EDEVICE, std::string("folding single-1D rows: ") + hipGetErrorString(er));
    }
  return CHIMERA_OK;
}

}  // namespace

chimera_status chimera_set_catalog(chimera_ctx* ctx, int64_t n_rows, const double* nz,
                                   const double* nz_tot) {
  if (!ctx || !nz_tot || (n_rows > 0 && !nz)) return fail(CHIMERA_EINVAL, "null argument");
  if (n_rows < 0) return fail(CHIMERA_EINVAL, "negative row count");
  const size_t nzn = (size_t)ctx->cfg.n_z;
  for (size_t i = 0; i < (size_t)n_rows * nzn; ++i)
    if (!(std::isfinite(nz[i]) && nz[i] >= 0.0)) return fail(CHIMERA_EINVAL, "nz must be finite, >= 0");
  for (size_t i = 0; i < nzn; ++i)
    if (!(std::isfinite(nz_tot[i]) && nz_tot[i] >= 0.0))
      return fail(CHIMERA_EINVAL, "nz_tot must be finite, >= 0");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (chimera_status st = check_resident_rows(ctx, n_rows); st != CHIMERA_OK) return st;
  HIP_TRY(hipSetDevice(ctx->cfg.device));
  HIP_TRY(hipDeviceSynchronize());
  free_catalog(ctx);
  std::vector<float> f32((size_t)n_rows * nzn);
  for (size_t i = 0; i < f32.size(); ++i) f32[i] = (float)nz[i];
  HIP_TRY(upload(&ctx->nz64, nz, (size_t)n_rows * nzn));
  HIP_TRY(upload(&ctx->nz32, f32.data(), f32.size()));
  HIP_TRY(upload(&ctx->ntot, nz_tot, nzn));
  ctx->n_rows = n_rows;
  ctx->has_cat = true;
  return refold_all(ctx);
}

chimera_status chimera_set_catalog_galaxies(chimera_ctx* ctx, int64_t n_pix, int64_t n_gal,
                                            const int64_t* gal_pix_off, const double* z_obs,
                                            const double* sigma_z, const double* vshape,
                                            double pixel_area, int64_t n_rows,
                                            const int64_t* rows_pix, int64_t* n_used) {
  if (!ctx || !gal_pix_off || !vshape || (n_gal > 0 && (!z_obs || !sigma_z)) ||
      (n_rows > 0 && !rows_pix))
    return fail(CHIMERA_EINVAL, "null argument");
  if (n_pix < 1 || n_gal < 0 || n_rows < 0) return fail(CHIMERA_EINVAL, "bad sizes");
  if (!(std::isfinite(pixel_area) && pixel_area > 0.0))
    return fail(CHIMERA_EINVAL, "pixel_area must be finite and > 0");
  if (gal_pix_off[0] != 0 || gal_pix_off[n_pix] != n_gal)
    return fail(CHIMERA_EINVAL, "gal_pix_off must run from 0 to n_gal");
  for (int64_t p = 0; p < n_pix; ++p)
    if (gal_pix_off[p + 1] < gal_pix_off[p])
      return fail(CHIMERA_EINVAL, "gal_pix_off must be non-decreasing");
  for (int64_t i = 0; i < n_gal; ++i)
    if (!std::isfinite(z_obs[i]) || !(std::isfinite(sigma_z[i]) && sigma_z[i] >= 0.0))
      return fail(CHIMERA_EINVAL, "z_obs must be finite and sigma_z finite, >= 0");
  const int nzn = ctx->cfg.n_z;
  for (int k = 0; k < nzn; ++k)
    if (!(std::isfinite(vshape[k]) && vshape[k] >= 0.0))
      return fail(CHIMERA_EINVAL, "vshape must be finite, >= 0");
  for (int64_t r = 0; r < n_rows; ++r)
    if (rows_pix[r] < 0 || rows_pix[r] >= n_pix)
      return fail(CHIMERA_ERANGE, "rows_pix refers past the pixels");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (chimera_status st = check_resident_rows(ctx, n_rows); st != CHIMERA_OK) return st;
  HIP_TRY(hipSetDevice(ctx->cfg.device));
  HIP_TRY(hipDeviceSynchronize());
  CatalogArgs c{};
  c.g.n_z = nzn;
  c.g.z_lo = ctx->cfg.z_lo;
  c.g.z_hi = ctx->cfg.z_hi;
  c.g.dz = (ctx->cfg.z_hi - ctx->cfg.z_lo) / (double)(nzn - 1);
  c.n_gal = n_gal;
  c.n_pix = n_pix;
  c.n_rows = n_rows;
  c.pixel_area = pixel_area;
  long long *off = nullptr, *rp = nullptr;
  double *mu = nullptr, *sig = nullptr, *vs = nullptr, *norm = nullptr, *rows_all = nullptr;
  double *nz64 = nullptr, *ntot = nullptr;
  float* nz32 = nullptr;
  auto cleanup = [&]() {
    dfree(off); dfree(rp); dfree(mu); dfree(sig); dfree(vs); dfree(norm); dfree(rows_all);
  };
  hipError_t e = hipSuccess;
  static_assert(sizeof(long long) == sizeof(int64_t), "int64 layout");
  if (e == hipSuccess) e = upload(&off, (const long long*)gal_pix_off, (size_t)n_pix + 1);
  if (e == hipSuccess && n_rows) e = upload(&rp, (const long long*)rows_pix, (size_t)n_rows);
  if (e == hipSuccess && n_gal) e = upload(&mu, z_obs, (size_t)n_gal);
  if (e == hipSuccess && n_gal) e = upload(&sig, sigma_z, (size_t)n_gal);
  if (e == hipSuccess) e = upload(&vs, vshape, (size_t)nzn);
  if (e == hipSuccess && n_gal) e = hipMalloc((void**)&norm, (size_t)n_gal * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&rows_all, (size_t)n_pix * nzn * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&nz64, std::max<size_t>(1, (size_t)n_rows * nzn) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&nz32, std::max<size_t>(1, (size_t)n_rows * nzn) * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&ntot, (size_t)nzn * sizeof(double));
  c.off = off; c.mu = mu; c.sig = sig; c.norm = norm; c.vshape = vs; c.rows_all = rows_all;
  c.rows_pix = rp; c.ntot = ntot; c.nz64 = nz64; c.nz32 = nz32;
  if (e == hipSuccess) e = launch_catalog(c, nullptr);
  int64_t used = 0;
  if (e == hipSuccess && n_gal) {
    std::vector<double> h((size_t)n_gal);
    e = hipMemcpy(h.data(), norm, (size_t)n_gal * sizeof(double), hipMemcpyDeviceToHost);
    for (double v : h) used += v > 0.0;
  }
  if (e == hipSuccess) e = launch_catalog_finish(c, used, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  cleanup();
  if (e != hipSuccess) {
    dfree(nz64); dfree(nz32); dfree(ntot);
    return fail(e == hipErrorOutOfMemory ? CHIMERA_ENOMEM : CHIMERA_EDEVICE,
                std::string("building the catalogue: ") + hipGetErrorString(e));
  }
  free_catalog(ctx);
  ctx->nz64 = nz64;
  ctx->nz32 = nz32;
  ctx->ntot = ntot;
  ctx->n_rows = n_rows;
  ctx->has_cat = true;
  if (n_used) *n_used = used;
  return refold_all(ctx);
}

chimera_status chimera_get_catalog(chimera_ctx* ctx, double* nz, double* nz_tot) {
  if (!ctx) return fail(CHIMERA_EINVAL, "null context");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (!ctx->has_cat) return fail(CHIMERA_ESTATE, "no catalogue set");
  HIP_TRY(hipSetDevice(ctx->cfg.device));
  HIP_TRY(hipDeviceSynchronize());
  const size_t nzn = (size_t)ctx->cfg.n_z;
  if (nz && ctx->n_rows)
    HIP_TRY(hipMemcpy(nz, ctx->nz64, (size_t)ctx->n_rows * nzn * sizeof(double),
                      hipMemcpyDeviceToHost));
  if (nz_tot) HIP_TRY(hipMemcpy(nz_tot, ctx->ntot, nzn * sizeof(double), hipMemcpyDeviceToHost));
  return CHIMERA_OK;
}

chimera_status chimera_set_injections(chimera_ctx* ctx, int64_t n_det, int64_t n_inj_total,
                                      const double* dl, const double* m1d, const double* m2d,
                                      const double* ln_pdraw) {
  if (!ctx) return fail(CHIMERA_EINVAL, "null context");
  if (n_det < 0 || n_inj_total < 1 || n_det > n_inj_total)
    return fail(CHIMERA_EINVAL, "need 0 <= n_det <= n_inj_total, n_inj_total >= 1");
  if (n_det > 0 && (!dl || !m1d || !m2d || !ln_pdraw)) return fail(CHIMERA_EINVAL, "null array");
  const size_t n = (size_t)n_det;
  if (!finite_positive(dl, n) || !finite_positive(m1d, n) || !finite_positive(m2d, n))
    return fail(CHIMERA_EINVAL, "injection distances and masses must be finite and > 0");
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(ln_pdraw[i])) return fail(CHIMERA_EINVAL, "ln_pdraw must be finite");
  std::vector<double> ld(n), l1(n), l2(n);
  double dmin = std::numeric_limits<double>::infinity(), dmax = 0.0;
  for (size_t i = 0; i < n; ++i) {
    ld[i] = std::log(dl[i]);
    l1[i] = std::log(m1d[i]);
    l2[i] = std::log(m2d[i]);
    dmin = std::min(dmin, dl[i]);
    dmax = std::max(dmax, dl[i]);
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->cfg.device));
  HIP_TRY(hipDeviceSynchronize());
  free_injections(ctx);
  HIP_TRY(upload(&ctx->inj_dl, dl, n));
  HIP_TRY(upload(&ctx->inj_lndl, ld.data(), n));
  HIP_TRY(upload(&ctx->inj_m1d, m1d, n));
  HIP_TRY(upload(&ctx->inj_m2d, m2d, n));
  HIP_TRY(upload(&ctx->inj_lnm1d, l1.data(), n));
  HIP_TRY(upload(&ctx->inj_lnm2d, l2.data(), n));
  HIP_TRY(upload(&ctx->inj_lnp, ln_pdraw, n));
  ctx->n_det = n_det;
  ctx->n_inj_total = n_inj_total;
  ctx->inj_dmin = n ? dmin : 1.0;
  ctx->inj_dmax = n ? dmax : 1.0;
  ctx->has_inj = true;
  return CHIMERA_OK;
}

namespace {

// Pixels of a single-1D set, folded into one row per event.
struct Fold {
  const int64_t* ev_pix_off;  // [n_ev+1]
  const int64_t* pix_row;     // [P] catalogue rows
  const double* s_ir;         // [P] sky factors
};

// Sky data of a 3D set.
struct Sky3 {
  const double* sky_u;        // [n_samp] chart coordinates of each sample (input order)
  const double* sky_v;
  const int64_t* ev_pix_off;  // [n_ev+1] the events' pixels
  const int64_t* pix_row;     // [P] catalogue rows
  const double* pix_u;        // [P] centres in the chart
  const double* pix_v;
  const double* pix_area;     // [P] areas
};

chimera_status build_events(chimera_ctx* ctx, int32_t n_ev, const int64_t* ev_pix_off,
                            const int64_t* pix_samp_off, const int64_t* pix_row,
                            const double* c_ir, const double* dl, const double* m1d,
                            const double* m2d, const Fold* fold, chimera_events** out,
                            const Sky3* sky = nullptr);

}  // namespace

chimera_status chimera_add_events(chimera_ctx* ctx, int32_t n_ev, const int64_t* ev_pix_off,
                                  const int64_t* pix_samp_off, const int64_t* pix_row,
                                  const double* c_ir, const double* dl, const double* m1d,
                                  const double* m2d, chimera_events** out) {
  if (!ctx || !out || !ev_pix_off || !pix_samp_off || !pix_row || !c_ir || !dl || !m1d || !m2d)
    return fail(CHIMERA_EINVAL, "null argument");
  *out = nullptr;
  if (n_ev < 1) return fail(CHIMERA_EINVAL, "need at least one event");
  if (!ctx->has_cat) return fail(CHIMERA_ESTATE, "set the catalogue before adding events");
  if (ev_pix_off[0] != 0) return fail(CHIMERA_EINVAL, "ev_pix_off[0] must be 0");
  for (int i = 0; i < n_ev; ++i) {
    if (ev_pix_off[i + 1] <= ev_pix_off[i])
      return fail(CHIMERA_EINVAL, "every event needs at least one pixel row");
    if (ev_pix_off[i + 1] - ev_pix_off[i] > CHIMERA_MAX_EVENT_PIXELS)
      return fail(CHIMERA_ERANGE, "an event has more pixel rows than CHIMERA_MAX_EVENT_PIXELS");
  }
  const int64_t P = ev_pix_off[n_ev];
  if (pix_samp_off[0] != 0) return fail(CHIMERA_EINVAL, "pix_samp_off[0] must be 0");
  for (int64_t p = 0; p < P; ++p) {
    if (pix_samp_off[p + 1] <= pix_samp_off[p])
      return fail(CHIMERA_EINVAL, "every pixel row needs at least one sample");
    if (pix_row[p] < 0 || pix_row[p] >= ctx->n_rows)
      return fail(CHIMERA_ERANGE, "pix_row refers past the catalogue");
    if (!(std::isfinite(c_ir[p]) && c_ir[p] > 0.0))
      return fail(CHIMERA_EINVAL, "c_ir must be finite and > 0");
  }
  const int64_t S = pix_samp_off[P];
  if (S > (int64_t)0x7fffffff) return fail(CHIMERA_ERANGE, "too many samples in one set");
  if (!finite_positive(dl, S) || !finite_positive(m1d, S) || !finite_positive(m2d, S))
    return fail(CHIMERA_EINVAL, "sample distances and masses must be finite and > 0");
  return build_events(ctx, n_ev, ev_pix_off, pix_samp_off, pix_row, c_ir, dl, m1d, m2d, nullptr,
                      out);
}

chimera_status chimera_add_events_single1d(chimera_ctx* ctx, int32_t n_ev,
                                           const int64_t* ev_samp_off, const double* dl,
                                           const double* m1d, const double* m2d,
                                           const int64_t* ev_pix_off, const int64_t* pix_row,
                                           const double* s_ir, chimera_events** out) {
  if (!ctx || !out || !ev_samp_off || !dl || !m1d || !m2d || !ev_pix_off || !pix_row || !s_ir)
    return fail(CHIMERA_EINVAL, "null argument");
  *out = nullptr;
  if (n_ev < 1) return fail(CHIMERA_EINVAL, "need at least one event");
  if (!ctx->has_cat) return fail(CHIMERA_ESTATE, "set the catalogue before adding events");
  if (ev_samp_off[0] != 0 || ev_pix_off[0] != 0)
    return fail(CHIMERA_EINVAL, "ev_samp_off[0] and ev_pix_off[0] must be 0");
  for (int i = 0; i < n_ev; ++i) {
    if (ev_samp_off[i + 1] <= ev_samp_off[i])
      return fail(CHIMERA_EINVAL, "every event needs at least one sample");
    if (ev_pix_off[i + 1] <= ev_pix_off[i])
      return fail(CHIMERA_EINVAL, "every event needs at least one pixel");
  }
  const int64_t P = ev_pix_off[n_ev];
  if (P > (int64_t)0x7fffffff) return fail(CHIMERA_ERANGE, "too many pixels in one set");
  for (int64_t p = 0; p < P; ++p) {
    if (pix_row[p] < 0 || pix_row[p] >= ctx->n_rows)
      return fail(CHIMERA_ERANGE, "pix_row refers past the catalogue");
    if (!(std::isfinite(s_ir[p]) && s_ir[p] > 0.0))
      return fail(CHIMERA_EINVAL, "s_ir must be finite and > 0");
  }
  const int64_t S = ev_samp_off[n_ev];
  if (S > (int64_t)0x7fffffff) return fail(CHIMERA_ERANGE, "too many samples in one set");
  if (!finite_positive(dl, S) || !finite_positive(m1d, S) || !finite_positive(m2d, S))
    return fail(CHIMERA_EINVAL, "sample distances and masses must be finite and > 0");
  // one pseudo-pixel per event over all its samples, c = 1/N_i (the KDE's
  // normalisation), row e = the event's folded row
  std::vector<int64_t> one(n_ev + 1), own_row(n_ev);
  std::vector<double> c(n_ev);
  for (int e = 0; e <= n_ev; ++e) one[e] = e;
  for (int e = 0; e < n_ev; ++e) {
    own_row[e] = e;
    c[e] = 1.0 / (double)(ev_samp_off[e + 1] - ev_samp_off[e]);
  }
  Fold f{ev_pix_off, pix_row, s_ir};
  return build_events(ctx, n_ev, one.data(), ev_samp_off, own_row.data(), c.data(), dl, m1d, m2d,
                      &f, out);
}

chimera_status chimera_add_events_3d(chimera_ctx* ctx, int32_t n_ev, const int64_t* ev_samp_off,
                                    const double* dl, const double* m1d, const double* m2d,
                                    const double* sky_u, const double* sky_v,
                                    const int64_t* ev_pix_off, const int64_t* pix_row,
                                    const double* pix_u, const double* pix_v,
                                    const double* pix_area, chimera_events** out) {
  if (!ctx || !out || !ev_samp_off || !dl || !m1d || !m2d || !sky_u || !sky_v || !ev_pix_off ||
      !pix_row || !pix_u || !pix_v || !pix_area)
    return fail(CHIMERA_EINVAL, "null argument");
  *out = nullptr;
  if (n_ev < 1) return fail(CHIMERA_EINVAL, "need at least one event");
  if (!ctx->has_cat) return fail(CHIMERA_ESTATE, "set the catalogue before adding events");
  if (ev_samp_off[0] != 0 || ev_pix_off[0] != 0)
    return fail(CHIMERA_EINVAL, "ev_samp_off[0] and ev_pix_off[0] must be 0");
  int64_t V = 0;
  for (int i = 0; i < n_ev; ++i) {
    const int64_t ns = ev_samp_off[i + 1] - ev_samp_off[i], np = ev_pix_off[i + 1] - ev_pix_off[i];
    if (ns < 1) return fail(CHIMERA_EINVAL, "every event needs at least one sample");
    if (np < 1) return fail(CHIMERA_EINVAL, "every event needs at least one pixel");
    if (np > CHIMERA_MAX_EVENT_PIXELS)
      return fail(CHIMERA_ERANGE, "an event has more pixels than CHIMERA_MAX_EVENT_PIXELS");
    V += ns * np;
  }
  if (V > (int64_t)0x7fffffff)
    return fail(CHIMERA_ERANGE, "samples x pixels of the set exceed 2^31 - 1");
  const int64_t P = ev_pix_off[n_ev];
  for (int64_t p = 0; p < P; ++p) {
    if (pix_row[p] < 0 || pix_row[p] >= ctx->n_rows)
      return fail(CHIMERA_ERANGE, "pix_row refers past the catalogue");
    if (!(std::isfinite(pix_u[p]) && std::isfinite(pix_v[p]) && std::isfinite(pix_area[p]) &&
          pix_area[p] > 0.0))
      return fail(CHIMERA_EINVAL, "pixel centres must be finite and areas finite and > 0");
  }
  const int64_t S = ev_samp_off[n_ev];
  if (S > (int64_t)0x7fffffff) return fail(CHIMERA_ERANGE, "too many samples in one set");
  if (!finite_positive(dl, S) || !finite_positive(m1d, S) || !finite_positive(m2d, S))
    return fail(CHIMERA_EINVAL, "sample distances and masses must be finite and > 0");
  for (int64_t j = 0; j < S; ++j)
    if (!(std::isfinite(sky_u[j]) && std::isfinite(sky_v[j])))
      return fail(CHIMERA_EINVAL, "sample sky coordinates must be finite");
  // the unique samples: one slot per event (row and c unused by the 3D sums)
  std::vector<int64_t> one(n_ev + 1), zero_row(n_ev, 0);
  std::vector<double> c(n_ev, 1.0);
  for (int e = 0; e <= n_ev; ++e) one[e] = e;
  Sky3 sky{sky_u, sky_v, ev_pix_off, pix_row, pix_u, pix_v, pix_area};
  return build_events(ctx, n_ev, one.data(), ev_samp_off, zero_row.data(), c.data(), dl, m1d, m2d,
                      nullptr, out, &sky);
}

namespace {

// The groups, work units and device copies of one event set (arguments
// checked by the caller).  fold != NULL makes a single-1D set: pix_row then
// indexes the set's own folded rows.  sky != NULL makes a 3D set: the
// samples form one slot per event and the (pixel, sample) layout is added.
chimera_status build_events(chimera_ctx* ctx, int32_t n_ev, const int64_t* ev_pix_off,
                            const int64_t* pix_samp_off, const int64_t* pix_row,
                            const double* c_ir, const double* dl, const double* m1d,
                            const double* m2d, const Fold* fold, chimera_events** out,
                            const Sky3* sky) {
  const int64_t P = ev_pix_off[n_ev];
  const int64_t S = pix_samp_off[P];
  // Groups: <= kGroupK samples of one pixel, consecutive in distance, spanning
  // at most kGroupSpread times the event's distance spread; the event's groups
  // are then ordered by mean distance (the same order in redshift for every
  // lambda, since d_L^gw is increasing).
  const double kGroupSpread = 0.6;
  const int kSpreadRun = 128;
  std::vector<int> ev_samp(n_ev + 1, 0), ev_slot(n_ev + 1), ev_unit(n_ev + 1, 0), srow(P);
  std::vector<int> u_event, u_grp0, u_ngrp;
  std::vector<int> gfirst, gcnt, gslot, gabs, ev_grp(n_ev + 1, 0);
  std::vector<int64_t> order;
  std::vector<double> gc;
  std::vector<double> odl, om1, om2, oc;
  std::vector<int> orow;
  odl.reserve(S); om1.reserve(S); om2.reserve(S); oc.reserve(S); orow.reserve(S);
  for (int64_t p = 0; p < P; ++p) srow[p] = (int)pix_row[p];
  for (int i = 0; i <= n_ev; ++i) ev_slot[i] = (int)ev_pix_off[i];
  struct G { double mean; int slot; std::vector<int64_t> idx; };
  for (int e = 0; e < n_ev; ++e) {
    const int64_t a0 = pix_samp_off[ev_pix_off[e]], a1 = pix_samp_off[ev_pix_off[e + 1]];
    double m = 0.0, m2 = 0.0;
    for (int64_t j = a0; j < a1; ++j) m += dl[j];
    m /= (double)(a1 - a0);
    for (int64_t j = a0; j < a1; ++j) m2 += (dl[j] - m) * (dl[j] - m);
    const double spread = kGroupSpread * std::sqrt(m2 / (double)std::max<int64_t>(a1 - a0, 1));
    std::vector<G> groups;
    for (int64_t p = ev_pix_off[e]; p < ev_pix_off[e + 1]; ++p) {
      std::vector<int64_t> idx;
      for (int64_t j = pix_samp_off[p]; j < pix_samp_off[p + 1]; ++j) idx.push_back(j);
      std::stable_sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return dl[x] < dl[y]; });
      size_t k = 0;
      while (k < idx.size()) {
        G g;
        g.slot = (int)(p - ev_pix_off[e]);
        const double d0 = dl[idx[k]];
        while (k < idx.size() && (int)g.idx.size() < kGroupK && dl[idx[k]] - d0 <= spread)
          g.idx.push_back(idx[k++]);
        double s = 0.0;
        for (auto j : g.idx) s += dl[j];
        g.mean = s / (double)g.idx.size();
        groups.push_back(std::move(g));
      }
    }
    std::stable_sort(groups.begin(), groups.end(), [](const G& x, const G& y) {
      return x.mean < y.mean || (x.mean == y.mean && x.slot < y.slot);
    });
    // work units: the event's groups in R nearly equal runs of <= kUnitGroups
    const int ng = (int)groups.size();
    const int R = (ng + kUnitGroups - 1) / kUnitGroups;
    const int gbase = (int)gfirst.size();
    for (int r = 0; r < R; ++r) {
      const int a = (int)((long long)ng * r / R), z = (int)((long long)ng * (r + 1) / R);
      u_event.push_back(e);
      u_grp0.push_back(gbase + a);
      u_ngrp.push_back(z - a);
    }
    ev_unit[e + 1] = (int)u_event.size();
    // within each unit, runs of kSpreadRun groups (neighbours in distance) are
    // ordered by their distance spread, so that the groups a wave takes have
    // edges of similar length
    for (int r = 0; r < R; ++r) {
      const int a = (int)((long long)ng * r / R), z = (int)((long long)ng * (r + 1) / R);
      for (int b0 = a; b0 < z; b0 += kSpreadRun) {
        const int b1 = std::min(b0 + kSpreadRun, z);
        std::stable_sort(groups.begin() + b0, groups.begin() + b1, [&](const G& x, const G& y) {
          return dl[x.idx.back()] - dl[x.idx.front()] < dl[y.idx.back()] - dl[y.idx.front()];
        });
      }
    }
    for (auto& g : groups) {
      gabs.push_back((int)(ev_pix_off[e] + g.slot));
      gfirst.push_back((int)odl.size());
      gcnt.push_back((int)g.idx.size());
      gslot.push_back(g.slot);
      gc.push_back(c_ir[ev_pix_off[e] + g.slot]);
      for (auto j : g.idx) {
        order.push_back(j);
        odl.push_back(dl[j]);
        om1.push_back(m1d[j]);
        om2.push_back(m2d[j]);
        oc.push_back(c_ir[ev_pix_off[e] + g.slot]);
        orow.push_back(srow[ev_pix_off[e] + g.slot]);
      }
    }
    ev_samp[e + 1] = (int)odl.size();
    ev_grp[e + 1] = (int)gfirst.size();
  }
  // each slot's samples (positions in group order) by distance, for the
  // binned data sets and the Epanechnikov sums
  std::vector<int> s_off(P + 1, 0), s_idx(S);
  for (size_t q = 0; q < gabs.size(); ++q) s_off[gabs[q] + 1] += gcnt[q];
  for (int64_t p = 0; p < P; ++p) s_off[p + 1] += s_off[p];
  {
    std::vector<int> fill(s_off.begin(), s_off.end() - 1);
    for (size_t q = 0; q < gabs.size(); ++q)
      for (int k = 0; k < gcnt[q]; ++k) s_idx[fill[gabs[q]]++] = gfirst[q] + k;
    for (int64_t p = 0; p < P; ++p)
      std::stable_sort(s_idx.begin() + s_off[p], s_idx.begin() + s_off[p + 1],
                       [&](int x, int y) { return odl[x] < odl[y]; });
  }
  std::vector<double> s_c(c_ir, c_ir + P);
  std::vector<int> s_ev(P);
  for (int i = 0; i < n_ev; ++i)
    for (int64_t p = ev_pix_off[i]; p < ev_pix_off[i + 1]; ++p) s_ev[p] = i;
  std::vector<double> ld(S), l1(S), l2(S);
  double dmin = std::numeric_limits<double>::infinity(), dmax = 0.0;
  for (int64_t j = 0; j < S; ++j) {
    ld[j] = std::log(odl[j]);
    l1[j] = std::log(om1[j]);
    l2[j] = std::log(om2[j]);
    dmin = std::min(dmin, odl[j]);
    dmax = std::max(dmax, odl[j]);
  }
  int64_t rows_needed = 0;
  std::vector<int> f_off, f_row;
  if (fold) {
    const int64_t FP = fold->ev_pix_off[n_ev];
    f_off.assign(fold->ev_pix_off, fold->ev_pix_off + n_ev + 1);
    f_row.resize(FP);
    for (int64_t p = 0; p < FP; ++p) {
      f_row[p] = (int)fold->pix_row[p];
      rows_needed = std::max(rows_needed, fold->pix_row[p] + 1);
    }
  } else if (sky) {
    for (int64_t p = 0; p < sky->ev_pix_off[n_ev]; ++p)
      rows_needed = std::max(rows_needed, sky->pix_row[p] + 1);
  } else {
    for (int64_t p = 0; p < P; ++p) rows_needed = std::max(rows_needed, pix_row[p] + 1);
  }
  // the 3D layout: per event, pixel-major (pixel, sample) points; groups are
  // the samples' groups repeated for every pixel, ordered group by group
  std::vector<long long> v_off;
  std::vector<double> su, sv, pu, pv;
  std::vector<int> d3_off, d3_row, veu, vue, vug0, vung, vgf, vgn, vgs;
  std::vector<double> vgc;
  if (sky) {
    const int64_t FP = sky->ev_pix_off[n_ev];
    su.resize(S);
    sv.resize(S);
    for (int64_t q = 0; q < S; ++q) {
      su[q] = sky->sky_u[order[q]];
      sv[q] = sky->sky_v[order[q]];
    }
    pu.assign(sky->pix_u, sky->pix_u + FP);
    pv.assign(sky->pix_v, sky->pix_v + FP);
    d3_off.assign(sky->ev_pix_off, sky->ev_pix_off + n_ev + 1);
    d3_row.assign(sky->pix_row, sky->pix_row + FP);
    v_off.assign(n_ev + 1, 0);
    veu.assign(n_ev + 1, 0);
    for (int e = 0; e < n_ev; ++e) {
      const int ns = ev_samp[e + 1] - ev_samp[e];
      const int p0 = d3_off[e], np = d3_off[e + 1] - p0;
      v_off[e + 1] = v_off[e] + (long long)ns * np;
      const int gbase = (int)vgf.size();
      for (int g = ev_grp[e]; g < ev_grp[e + 1]; ++g)
        for (int k = 0; k < np; ++k) {
          vgf.push_back((int)(v_off[e] + (long long)k * ns + (gfirst[g] - ev_samp[e])));
          vgn.push_back(gcnt[g]);
          vgs.push_back(k);
          vgc.push_back(sky->pix_area[p0 + k] / (double)ns);
        }
      const int ng = (int)vgf.size() - gbase;
      const int R = (ng + kUnitGroups - 1) / kUnitGroups;
      for (int u = 0; u < R; ++u) {
        const int a = (int)((long long)ng * u / R), z = (int)((long long)ng * (u + 1) / R);
        vue.push_back(e);
        vug0.push_back(gbase + a);
        vung.push_back(z - a);
      }
      veu[e + 1] = (int)vue.size();
    }
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (rows_needed > ctx->n_rows)   // the catalogue changed since the check above
    return fail(CHIMERA_ERANGE, "pix_row refers past the catalogue");
  HIP_TRY(hipSetDevice(ctx->cfg.device));
  auto* ev = new chimera_events();
  ev->E = n_ev;
  ev->n_samp = S;
  ev->U = (int)u_event.size();
  ev->dmin = dmin;
  ev->dmax = dmax;
  ev->rows_needed = rows_needed;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = upload(&ev->ev_unit_off, ev_unit.data(), ev_unit.size());
  if (e == hipSuccess) e = upload(&ev->unit_event, u_event.data(), u_event.size());
  if (e == hipSuccess) e = upload(&ev->unit_grp0, u_grp0.data(), u_grp0.size());
  if (e == hipSuccess) e = upload(&ev->unit_ngrp, u_ngrp.data(), u_ngrp.size());
  if (e == hipSuccess) e = upload(&ev->ev_samp_off, ev_samp.data(), ev_samp.size());
  if (e == hipSuccess) e = upload(&ev->ev_slot_off, ev_slot.data(), ev_slot.size());
  if (e == hipSuccess) e = upload(&ev->slot_row, srow.data(), srow.size());
  if (e == hipSuccess) e = upload(&ev->grp_first, gfirst.data(), gfirst.size());
  if (e == hipSuccess) e = upload(&ev->grp_cnt, gcnt.data(), gcnt.size());
  if (e == hipSuccess) e = upload(&ev->grp_slot, gslot.data(), gslot.size());
  if (e == hipSuccess) e = upload(&ev->grp_c, gc.data(), gc.size());
  if (e == hipSuccess) e = upload(&ev->dl, odl.data(), S);
  if (e == hipSuccess) e = upload(&ev->lndl, ld.data(), S);
  if (e == hipSuccess) e = upload(&ev->m1d, om1.data(), S);
  if (e == hipSuccess) e = upload(&ev->m2d, om2.data(), S);
  if (e == hipSuccess) e = upload(&ev->lnm1d, l1.data(), S);
  if (e == hipSuccess) e = upload(&ev->lnm2d, l2.data(), S);
  if (e == hipSuccess) e = upload(&ev->samp_row, orow.data(), S);
  if (e == hipSuccess) e = upload(&ev->samp_c, oc.data(), S);
  ev->P = (int)P;
  if (e == hipSuccess) e = upload(&ev->pix_off, s_off.data(), s_off.size());
  if (e == hipSuccess) e = upload(&ev->pix_idx, s_idx.data(), s_idx.size());
  if (e == hipSuccess) e = upload(&ev->slot_c, s_c.data(), s_c.size());
  if (e == hipSuccess) e = upload(&ev->slot_event, s_ev.data(), s_ev.size());
  // the bin layout of chimera_set_event_kde needs the slots' events
  ev->h_slot_off.assign(ev_slot.begin(), ev_slot.end());
  ev->h_slot_c = s_c;
  if (sky) {
    ev->V = v_off[n_ev];
    ev->Uv = (int)vue.size();
    if (e == hipSuccess) e = upload(&ev->virt_off, v_off.data(), v_off.size());
    if (e == hipSuccess) e = upload(&ev->su, su.data(), su.size());
    if (e == hipSuccess) e = upload(&ev->sv, sv.data(), sv.size());
    if (e == hipSuccess) e = upload(&ev->pu, pu.data(), pu.size());
    if (e == hipSuccess) e = upload(&ev->pv, pv.data(), pv.size());
    if (e == hipSuccess) e = upload(&ev->d3_slot_off, d3_off.data(), d3_off.size());
    if (e == hipSuccess) e = upload(&ev->d3_slot_row, d3_row.data(), d3_row.size());
    if (e == hipSuccess) e = upload(&ev->v_ev_unit_off, veu.data(), veu.size());
    if (e == hipSuccess) e = upload(&ev->v_unit_event, vue.data(), vue.size());
    if (e == hipSuccess) e = upload(&ev->v_unit_grp0, vug0.data(), vug0.size());
    if (e == hipSuccess) e = upload(&ev->v_unit_ngrp, vung.data(), vung.size());
    if (e == hipSuccess) e = upload(&ev->v_grp_first, vgf.data(), vgf.size());
    if (e == hipSuccess) e = upload(&ev->v_grp_cnt, vgn.data(), vgn.size());
    if (e == hipSuccess) e = upload(&ev->v_grp_slot, vgs.data(), vgs.size());
    if (e == hipSuccess) e = upload(&ev->v_grp_c, vgc.data(), vgc.size());
  }
  if (fold) {
    ev->single1d = true;
    const size_t rows = (size_t)n_ev * ctx->cfg.n_z;
    if (e == hipSuccess) e = upload(&ev->fold_pix_off, f_off.data(), f_off.size());
    if (e == hipSuccess) e = upload(&ev->fold_row, f_row.data(), f_row.size());
    if (e == hipSuccess) e = upload(&ev->fold_s, fold->s_ir, f_row.size());
    if (e == hipSuccess) e = hipMalloc((void**)&ev->own64, rows * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&ev->own32, rows * sizeof(float));
    if (e == hipSuccess) e = fold_rows(ctx, ev);
  }
  if (e != hipSuccess) {
    free_events(ev);
    return fail(e == hipErrorOutOfMemory ? CHIMERA_ENOMEM : CHIMERA_EDEVICE,
                std::string("uploading events: ") + hipGetErrorString(e));
  }
  ctx->events.push_back(ev);
  *out = ev;
  return CHIMERA_OK;
}

}  // namespace

chimera_status chimera_release_events(chimera_ctx* ctx, chimera_events* ev) {
  if (!ctx || !ev) return fail(CHIMERA_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = std::find(ctx->events.begin(), ctx->events.end(), ev);
  if (it == ctx->events.end()) return fail(CHIMERA_EINVAL, "unknown event set");
  HIP_TRY(hipSetDevice(ctx->cfg.device));
  HIP_TRY(hipDeviceSynchronize());
  ctx->events.erase(it);
  free_events(ev);
  return CHIMERA_OK;
}

chimera_status chimera_set_completeness(chimera_ctx* ctx, const double* p_compl,
                                       const double* missing) {
  if (!ctx) return fail(CHIMERA_EINVAL, "null context");
  const size_t nzn = (size_t)ctx->cfg.n_z;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (!ctx->has_cat) return fail(CHIMERA_ESTATE, "set the catalogue first");
  HIP_TRY(hipSetDevice(ctx->cfg.device));
  if (!p_compl) {
    HIP_TRY(hipDeviceSynchronize());
    free_completeness(ctx);
    return CHIMERA_OK;
  }
  if (!missing) return fail(CHIMERA_EINVAL, "null missing solid angle");
  const size_t n = (size_t)ctx->n_rows * nzn;
  for (size_t i = 0; i < n; ++i)
    if (!(p_compl[i] >= 0.0 && p_compl[i] <= 1.0))
      return fail(CHIMERA_EINVAL, "p_compl must lie in [0, 1]");
  for (size_t k = 0; k < nzn; ++k)
    if (!(missing[k] >= 0.0 && missing[k] <= 4.0 * M_PI))
      return fail(CHIMERA_EINVAL, "missing must lie in [0, 4 pi]");
  std::vector<double> m64(std::max<size_t>(n, 1), 0.0);
  std::vector<float> m32(std::max<size_t>(n, 1), 0.0f);
  for (size_t i = 0; i < n; ++i) {
    m64[i] = 1.0 - p_compl[i];
    m32[i] = (float)m64[i];
  }
  HIP_TRY(hipDeviceSynchronize());
  free_completeness(ctx);
  hipError_t e = upload(&ctx->miss64, m64.data(), std::max<size_t>(n, 1));
  if (e == hipSuccess) e = upload(&ctx->miss32, m32.data(), std::max<size_t>(n, 1));
  if (e == hipSuccess) e = upload(&ctx->missing, missing, nzn);
  if (e != hipSuccess) {
    free_completeness(ctx);
    return fail(e == hipErrorOutOfMemory ? CHIMERA_ENOMEM : CHIMERA_EDEVICE,
                std::string("uploading the completeness: ") + hipGetErrorString(e));
  }
  return refold_all(ctx);
}

chimera_status chimera_set_mass_smoothing(chimera_ctx* ctx, int32_t on) {
  if (!ctx) return fail(CHIMERA_EINVAL, "null context");
  if (on != 0 && on != 1) return fail(CHIMERA_EINVAL, "on must be 0 or 1");
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->nlam = on ? CHIMERA_NLAM + 1 : CHIMERA_NLAM;
  return CHIMERA_OK;
}

chimera_status chimera_lambda_width(chimera_ctx* ctx, int32_t* width) {
  if (!ctx || !width) return fail(CHIMERA_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  *width = ctx->nlam;
  return CHIMERA_OK;
}

chimera_status chimera_set_neff_gate(chimera_ctx* ctx, double factor) {
  if (!ctx) return fail(CHIMERA_EINVAL, "null context");
  if (!(std::isfinite(factor) && factor >= 0.0))
    return fail(CHIMERA_EINVAL, "the gate factor must be finite and >= 0");
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->neff_gate = factor;
  return CHIMERA_OK;
}

chimera_status chimera_set_event_kde(chimera_ctx* ctx, chimera_events* ev, int32_t shape,
                                     int32_t n_bins) {
  if (!ctx || !ev) return fail(CHIMERA_EINVAL, "null argument");
  if (shape != CHIMERA_KDE_GAUSSIAN && shape != CHIMERA_KDE_EPANECHNIKOV)
    return fail(CHIMERA_EINVAL, "unknown kernel shape");
  if (n_bins < 0 || n_bins > CHIMERA_MAX_BINS)
    return fail(CHIMERA_EINVAL, "n_bins out of [0, CHIMERA_MAX_BINS]");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (std::find(ctx->events.begin(), ctx->events.end(), ev) == ctx->events.end())
    return fail(CHIMERA_EINVAL, "unknown event set");
  if (ev->V && (shape != CHIMERA_KDE_GAUSSIAN || n_bins != 0))
    return fail(CHIMERA_EINVAL, "the 3D kernel is Gaussian on the samples");
  if ((int64_t)ev->P * n_bins > (int64_t)0x7fffffff)
    return fail(CHIMERA_ERANGE, "pixel slots x n_bins exceed 2^31 - 1");
  HIP_TRY(hipSetDevice(ctx->cfg.device));
  HIP_TRY(hipDeviceSynchronize());
  free_bin_layout(ev);
  ev->shape = CHIMERA_KDE_GAUSSIAN;
  ev->n_bins = 0;
  if (n_bins > 0) {
    // groups of <= kGroupK consecutive bins of one slot; within an event the
    // groups are ordered by their place in the slots' ranges (every slot's
    // first group, then every slot's second, ...), so that a work unit spans
    // a narrow redshift range, and cut into runs of <= kUnitGroups
    // bins per group: consecutive bins are (range / n_bins) apart, so groups
    // of n_bins / 4 bins (1..kGroupK) span about a quarter of a slot's range,
    // which keeps the groups' Horner factors within range in FP32
    const int bpg = std::max(1, std::min(kGroupK, n_bins / 4));
    const int gps = (n_bins + bpg - 1) / bpg;
    std::vector<int> eu(ev->E + 1, 0), ue, ug0, ung, gf, gn, gs;
    std::vector<double> gcv;
    for (int e = 0; e < ev->E; ++e) {
      const int so = ev->h_slot_off[e], ns = ev->h_slot_off[e + 1] - so;
      const int gbase = (int)gf.size();
      for (int q = 0; q < gps; ++q)
        for (int r = 0; r < ns; ++r) {
          gf.push_back((so + r) * n_bins + q * bpg);
          gn.push_back(std::min(bpg, n_bins - q * bpg));
          gs.push_back(r);
          gcv.push_back(ev->h_slot_c[so + r]);
        }
      const int ng = (int)gf.size() - gbase;
      const int R = (ng + kUnitGroups - 1) / kUnitGroups;
      for (int u = 0; u < R; ++u) {
        const int a = (int)((long long)ng * u / R), z = (int)((long long)ng * (u + 1) / R);
        ue.push_back(e);
        ug0.push_back(gbase + a);
        ung.push_back(z - a);
      }
      eu[e + 1] = (int)ue.size();
    }
    hipError_t er = hipSuccess;
    if (er == hipSuccess) er = upload(&ev->b_ev_unit_off, eu.data(), eu.size());
    if (er == hipSuccess) er = upload(&ev->b_unit_event, ue.data(), ue.size());
    if (er == hipSuccess) er = upload(&ev->b_unit_grp0, ug0.data(), ug0.size());
    if (er == hipSuccess) er = upload(&ev->b_unit_ngrp, ung.data(), ung.size());
    if (er == hipSuccess) er = upload(&ev->b_grp_first, gf.data(), gf.size());
    if (er == hipSuccess) er = upload(&ev->b_grp_cnt, gn.data(), gn.size());
    if (er == hipSuccess) er = upload(&ev->b_grp_slot, gs.data(), gs.size());
    if (er == hipSuccess) er = upload(&ev->b_grp_c, gcv.data(), gcv.size());
    if (er != hipSuccess) {
      free_bin_layout(ev);
      return fail(er == hipErrorOutOfMemory ? CHIMERA_ENOMEM : CHIMERA_EDEVICE,
                  std::string("uploading the bin layout: ") + hipGetErrorString(er));
    }
    ev->Ub = (int)ue.size();
  }
  ev->shape = shape;
  ev->n_bins = n_bins;
  return CHIMERA_OK;
}

// Largest per-sample scratch (z_j, w_j for every sample and lambda) of one
// launch sequence; a call over more lambda points runs in consecutive chunks.
constexpr double kSampleScratchCap = 8.0 * (1ull << 30);

int64_t lambda_chunk(const chimera_events* ev, int64_t B, bool f32) {
  if (!ev) return B;
  const double nb = ev->n_bins ? (double)ev->P * ev->n_bins : 0.0;
  const double per = ((double)ev->n_samp + nb + (double)ev->V) * (f32 ? 12.0 : 16.0) +
                     8.0 * (9.0 * ev->E + std::max(std::max(ev->U, ev->Ub), std::max(ev->P, ev->Uv)));
  const int64_t c = (int64_t)std::max(1.0, std::floor(kSampleScratchCap / per));
  return std::min(B, c);
}

// The arena of stream st (created empty on first use).
static chimera_ctx::Arena* arena_of(chimera_ctx* ctx, hipStream_t st) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto& a = ctx->arenas[st];
  if (!a) a.reset(new chimera_ctx::Arena());
  return a.get();
}

// The arena's block, at least `bytes` large (the caller holds ar->mu).  Work
// on one stream runs in order, so consecutive calls on it share the block; a
// block that has to grow is released in stream order (after the work that
// used it).
static hipError_t arena_reserve(chimera_ctx::Arena* ar, hipStream_t st, size_t bytes, void** out) {
  if (ar->n < bytes) {
    if (ar->p) {
      hipError_t e = hipFreeAsync(ar->p, st);
      if (e != hipSuccess) return e;
      ar->p = nullptr;
      ar->n = 0;
    }
    const size_t n = pool_size(bytes);
    hipError_t e = hipMallocAsync(&ar->p, n, st);
    if (e != hipSuccess) return e;
    ar->n = n;
  }
  *out = ar->p;
  return hipSuccess;
}

// One launch sequence.  ext (the static scratch, or NULL) replaces the
// stream's arena; then nothing is allocated (and no profiling events made).
static chimera_status run_chunk(chimera_ctx* ctx, const chimera_events* ev, const double* lam,
                                int64_t B, int32_t prec, double* lnl, double* lnI, double* ln_xi,
                                double* n_eff, int32_t mem, int nlam, void* hip_stream,
                                void* ext = nullptr) {
  hipStream_t st = (hipStream_t)hip_stream;
  HIP_TRY(hipSetDevice(ctx->cfg.device));
  const bool f32 = prec == CHIMERA_FP32;
  const bool host = mem == CHIMERA_HOST;
  const int E = ev ? ev->E : 0;
  double dmin = ctx->n_det ? ctx->inj_dmin : std::numeric_limits<double>::infinity();
  double dmax = ctx->n_det ? ctx->inj_dmax : 0.0;
  if (ev) {
    dmin = std::min(dmin, ev->dmin);
    dmax = std::max(dmax, ev->dmax);
  }
  if (!(dmax > 0.0)) dmin = dmax = 1.0;
  const Geometry g = make_geometry(ctx, dmin, dmax);
  const int nchunk = selection_chunks(ctx->n_det);
  Scratch s;
  Carve probe;
  const bool need_lnI = ev && (host || !lnI);
  const bool compl_ = ctx->miss64 != nullptr;
  const size_t bytes =
      carve(probe, s, g, B, nchunk, host, need_lnI, host, ev, f32, compl_, nlam);
  if (ctx->cfg.hbm_budget && pool_size(bytes) > ctx->cfg.hbm_budget)
    return fail(CHIMERA_ENOMEM, "call needs " + std::to_string(bytes) +
                                    " scratch bytes, over the context's hbm_budget");
  void* base = ext;
  std::unique_lock<std::mutex> stream_lock;
  if (!ext) {
    chimera_ctx::Arena* ar = arena_of(ctx, st);
    stream_lock = std::unique_lock<std::mutex>(ar->mu);
    HIP_TRY(arena_reserve(ar, st, bytes, &base));
  } else if (bytes > kStaticScratchBytes) {
    return fail(CHIMERA_ENOMEM, "launch needs " + std::to_string(bytes) +
                                    " scratch bytes, over the static scratch");
  }
  Carve cv;
  cv.base = (char*)base;
  carve(cv, s, g, B, nchunk, host, need_lnI, host, ev, f32, compl_, nlam);
  const double* lam_dev = lam;
  if (host) {
    HIP_TRY(hipMemcpyAsync(s.lam, lam, (size_t)B * nlam * sizeof(double),
                           hipMemcpyHostToDevice, st));
    lam_dev = s.lam;
  }
  double* lnI_dev = need_lnI ? s.lnI : lnI;
  double* lnxi_dev = (host || !ln_xi) ? s.ln_xi : ln_xi;
  // N_eff is always formed: the N_eff gate reads it
  double* neff_dev = host || !n_eff ? s.neff : n_eff;
  double* lnl_dev = host ? s.lnl : lnl;
  HIP_TRY(launch_tables(lam_dev, nlam, (int)B, g, s.P, s.mtab, s.chi, s.inv,
                        ev ? s.dtab : nullptr,
                        ev ? s.gz64 : nullptr,
                        ev ? s.gz32 : nullptr, s.flag_mono, s.flag_range, st));
  SelArgs sa;
  sa.P = s.P; sa.flag_mono = s.flag_mono; sa.flag_range = s.flag_range;
  if (compl_)
    HIP_TRY(launch_completion(s.P, s.chi, g, (int)B, ctx->ntot, ctx->missing, s.ntot_eff,
                              ev ? s.gz64 : nullptr, ev ? s.gz32 : nullptr, s.gzb64, s.gzb32, st));
  sa.chi = s.chi; sa.inv = s.inv; sa.g = g;
  sa.ntot = compl_ ? s.ntot_eff : ctx->ntot;
  sa.ntot_stride = compl_ ? g.n_z : 0;
  sa.mtab = s.mtab;
  sa.dl = ctx->inj_dl; sa.lndl = ctx->inj_lndl; sa.m1d = ctx->inj_m1d; sa.m2d = ctx->inj_m2d;
  sa.lnm1d = ctx->inj_lnm1d; sa.lnm2d = ctx->inj_lnm2d; sa.ln_pdraw = ctx->inj_lnp;
  sa.n_det = ctx->n_det; sa.n_total = ctx->n_inj_total; sa.B = (int)B; sa.nchunk = nchunk;
  sa.partial = s.partial;
  HIP_TRY(launch_selection(sa, f32, lnxi_dev, neff_dev, st));
  if (ev) {
    EventArgs a{};
    a.P = s.P; a.flag_mono = s.flag_mono; a.flag_range = s.flag_range;
    a.chi = s.chi; a.inv = s.inv; a.dtab = s.dtab; a.g = g; a.gz64 = s.gz64; a.gz32 = s.gz32;
    a.mtab = s.mtab;
    a.wscale = s.wscale;
    a.nz64 = rows64(ctx, ev); a.nz32 = rows32(ctx, ev);
    a.mz64 = miss64(ctx, ev); a.mz32 = miss32(ctx, ev);
    a.gzb64 = s.gzb64; a.gzb32 = s.gzb32;
    a.ev_samp_off = ev->ev_samp_off; a.ev_slot_off = ev->ev_slot_off;
    a.ev_unit_off = ev->ev_unit_off; a.slot_row = ev->slot_row;
    a.grp_first = ev->grp_first; a.grp_cnt = ev->grp_cnt; a.grp_slot = ev->grp_slot;
    a.grp_c = ev->grp_c;
    a.unit_event = ev->unit_event; a.unit_grp0 = ev->unit_grp0; a.unit_ngrp = ev->unit_ngrp;
    a.dl = ev->dl; a.lndl = ev->lndl; a.m1d = ev->m1d; a.m2d = ev->m2d;
    a.lnm1d = ev->lnm1d; a.lnm2d = ev->lnm2d;
    a.E = E; a.U = ev->U; a.B = (int)B; a.S = ev->n_samp;
    a.trunc = f32 ? ctx->cfg.trunc_fp32 : ctx->cfg.trunc_fp64;
    a.zbuf = s.zbuf; a.wbuf = s.wbuf; a.hbuf = s.hbuf; a.part = s.part; a.lnI = lnI_dev;
    a.count = nullptr;
    a.pcount = s.pcount;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (ctx->profile && !ext) {
      std::lock_guard<std::mutex> lk(ctx->mu);
      a.count = ctx->d_count;
      HIP_TRY(hipEventCreate(&t0));
      HIP_TRY(hipEventCreate(&t1));
    }
    a.shape = ev->shape; a.n_bins = ev->n_bins; a.n_slots = ev->P;
    a.pix_off = ev->pix_off; a.pix_idx = ev->pix_idx; a.slot_c = ev->slot_c;
    a.bz = s.bz; a.bw = s.bw;
    // the kernel-sum launch: over the samples, the bins, or one unit per event
    EventArgs k = a;
    a.slot_event = ev->slot_event;
    k.slot_event = ev->slot_event;
    a.V = ev->V;
    k.V = ev->V;
    if (ev->V) {
      // cov3d / expand3d read the real pixels as slots; the sums run over the points
      a.ev_slot_off = ev->d3_slot_off; a.slot_row = ev->d3_slot_row;
      a.su = ev->su; a.sv = ev->sv; a.pu = ev->pu; a.pv = ev->pv; a.virt_off = ev->virt_off;
      a.p3 = s.p3; a.z3 = s.z3; a.w3 = s.w3;
      k = a;
      k.zbuf = s.z3; k.wbuf = s.w3; k.S = ev->V;
      k.ev_unit_off = ev->v_ev_unit_off; k.U = ev->Uv;
      k.grp_first = ev->v_grp_first; k.grp_cnt = ev->v_grp_cnt; k.grp_slot = ev->v_grp_slot;
      k.grp_c = ev->v_grp_c;
      k.unit_event = ev->v_unit_event; k.unit_grp0 = ev->v_unit_grp0;
      k.unit_ngrp = ev->v_unit_ngrp;
    } else if (ev->shape == CHIMERA_KDE_EPANECHNIKOV) {
      k.U = ev->P;                          // one partial per pixel slot
      k.ev_unit_off = ev->ev_slot_off;
    } else if (ev->n_bins) {
      k.zbuf = s.bz; k.wbuf = s.bw; k.S = (long long)ev->P * ev->n_bins;
      k.ev_unit_off = ev->b_ev_unit_off; k.U = ev->Ub;
      k.grp_first = ev->b_grp_first; k.grp_cnt = ev->b_grp_cnt; k.grp_slot = ev->b_grp_slot;
      k.grp_c = ev->b_grp_c;
      k.unit_event = ev->b_unit_event; k.unit_grp0 = ev->b_unit_grp0;
      k.unit_ngrp = ev->b_unit_ngrp;
    }
    // t0 / t1 bracket the kernel sums (the dominant kernel) on stream st
    HIP_TRY(launch_events(a, k, f32, st, t0, t1));
    if (t0) {
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->marks.emplace_back(t0, t1);
    }
    HIP_TRY(launch_lnl_final(s.P, s.flag_mono, s.flag_range, lnI_dev, lnxi_dev, neff_dev,
                             ctx->neff_gate, E, (int)B,
                             lnl_dev, st));
  }
  if (host) {
    if (ev) HIP_TRY(hipMemcpyAsync(lnl, lnl_dev, B * sizeof(double), hipMemcpyDeviceToHost, st));
    if (ev && lnI)
      HIP_TRY(hipMemcpyAsync(lnI, lnI_dev, (size_t)B * E * sizeof(double), hipMemcpyDeviceToHost,
                             st));
    if (ln_xi)
      HIP_TRY(hipMemcpyAsync(ln_xi, lnxi_dev, B * sizeof(double), hipMemcpyDeviceToHost, st));
    if (n_eff)
      HIP_TRY(hipMemcpyAsync(n_eff, neff_dev, B * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  if (host) HIP_TRY(hipStreamSynchronize(st));
  return CHIMERA_OK;
}

static chimera_status run_batch(chimera_ctx* ctx, const chimera_events* ev, const double* lam,
                                int64_t B, int32_t prec, double* lnl, double* lnI, double* ln_xi,
                                double* n_eff, int32_t mem, void* hip_stream) {
  const int64_t Bc = lambda_chunk(ev, B, prec == CHIMERA_FP32);
  const int64_t E = ev ? ev->E : 0;
  const int nlam = ctx->nlam;
  for (int64_t c0 = 0; c0 < B; c0 += Bc) {
    const int64_t n = std::min(Bc, B - c0);
    chimera_status s =
        run_chunk(ctx, ev, lam + c0 * nlam, n, prec, lnl ? lnl + c0 : nullptr,
                  lnI ? lnI + c0 * E : nullptr, ln_xi ? ln_xi + c0 : nullptr,
                  n_eff ? n_eff + c0 : nullptr, mem, nlam, hip_stream);
    if (s != CHIMERA_OK) return s;
  }
  return CHIMERA_OK;
}

chimera_status chimera_scratch_bytes(chimera_ctx* ctx, const chimera_events* ev, int64_t B,
                                     int32_t prec, int32_t mem, size_t* bytes) {
  if (!ctx || !bytes) return fail(CHIMERA_EINVAL, "null argument");
  if (B < 1 || B > (1 << 20)) return fail(CHIMERA_EINVAL, "batch size out of [1, 2^20]");
  if (prec != CHIMERA_FP64 && prec != CHIMERA_FP32) return fail(CHIMERA_EINVAL, "bad precision");
  if (mem != CHIMERA_HOST && mem != CHIMERA_DEVICE) return fail(CHIMERA_EINVAL, "bad mem");
  const bool host = mem == CHIMERA_HOST;
  B = lambda_chunk(ev, B, prec == CHIMERA_FP32);
  double dmin = ev ? ev->dmin : 1.0, dmax = ev ? ev->dmax : 1.0;
  const Geometry g = make_geometry(ctx, dmin, dmax);
  Scratch s;
  Carve probe;
  // lnI is counted whenever there is an event set: a device call without an
  // lnI output keeps it in the scratch
  *bytes = pool_size(carve(probe, s, g, B, selection_chunks(ctx->n_det), host, ev != nullptr,
                           host, ev, prec == CHIMERA_FP32, ctx->miss64 != nullptr, ctx->nlam));
  return CHIMERA_OK;
}

chimera_status chimera_scratch_held(chimera_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return fail(CHIMERA_EINVAL, "null argument");
  std::vector<chimera_ctx::Arena*> all;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto& a : ctx->arenas) all.push_back(a.second.get());
  }
  size_t n = 0;
  for (auto* ar : all) {
    std::lock_guard<std::mutex> lk(ar->mu);
    n += ar->n;
  }
  *bytes = n;
  return CHIMERA_OK;
}

chimera_status chimera_release_scratch(chimera_ctx* ctx, void* hip_stream) {
  if (!ctx) return fail(CHIMERA_EINVAL, "null context");
  hipStream_t st = (hipStream_t)hip_stream;
  chimera_ctx::Arena* ar = arena_of(ctx, st);
  std::lock_guard<std::mutex> lk(ar->mu);
  HIP_TRY(hipSetDevice(ctx->cfg.device));
  if (ar->p) {
    HIP_TRY(hipFreeAsync(ar->p, st));
    HIP_TRY(hipStreamSynchronize(st));
    ar->p = nullptr;
    ar->n = 0;
  }
  // hand the freed block back to the device: keep only what the other
  // streams' arenas may still take from the pool
  size_t keep = 0;
  {
    std::lock_guard<std::mutex> lk2(ctx->mu);
    for (auto& a : ctx->arenas)
      if (a.second.get() != ar) keep += a.second->n;
  }
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, ctx->cfg.device) == hipSuccess)
    (void)hipMemPoolTrimTo(pool, keep);
  return CHIMERA_OK;
}

chimera_status chimera_lnl_batch(chimera_ctx* ctx, const chimera_events* ev, const double* lam,
                                 int64_t B, int32_t prec, double* lnl, double* lnI, int32_t mem,
                                 void* hip_stream) {
  chimera_status s = check_common(ctx, lam, B, prec, mem);
  if (s != CHIMERA_OK) return s;
  if (!ev) return fail(CHIMERA_EINVAL, "null event set");
  if (!lnl) return fail(CHIMERA_EINVAL, "null output");
  return run_batch(ctx, ev, lam, B, prec, lnl, lnI, nullptr, nullptr, mem, hip_stream);
}

// Scratch bytes of one device-mode launch sequence of B points.
static size_t device_launch_bytes(chimera_ctx* ctx, const chimera_events* ev, int64_t B,
                                  bool f32, bool have_lnI, int nlam) {
  double dmin = ctx->n_det ? ctx->inj_dmin : std::numeric_limits<double>::infinity();
  double dmax = ctx->n_det ? ctx->inj_dmax : 0.0;
  dmin = std::min(dmin, ev->dmin);
  dmax = std::max(dmax, ev->dmax);
  if (!(dmax > 0.0)) dmin = dmax = 1.0;
  const Geometry g = make_geometry(ctx, dmin, dmax);
  Scratch s;
  Carve probe;
  return carve(probe, s, g, B, selection_chunks(ctx->n_det), false, !have_lnI, false, ev, f32,
               ctx->miss64 != nullptr, nlam);
}

chimera_status chimera_lnl_batch_static(chimera_ctx* ctx, const chimera_events* ev,
                                        const double* lam, int64_t B, int32_t prec, double* lnl,
                                        double* lnI, void* hip_stream) {
  chimera_status s = check_common(ctx, lam, B, prec, CHIMERA_DEVICE);
  if (s != CHIMERA_OK) return s;
  if (!ev) return fail(CHIMERA_EINVAL, "null event set");
  if (!lnl) return fail(CHIMERA_EINVAL, "null output");
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    auto it = g_static_ptr.find(ctx->cfg.device);
    if (it == g_static_ptr.end()) return fail(CHIMERA_ESTATE, "static scratch not set up");
    base = it->second;
  }
  // the most lambda points per launch sequence that the static scratch holds
  const bool f32 = prec == CHIMERA_FP32;
  const int nlam = ctx->nlam;
  int64_t lo = 0, hi = B;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (device_launch_bytes(ctx, ev, mid, f32, lnI != nullptr, nlam) <= kStaticScratchBytes)
      lo = mid;
    else hi = mid - 1;
  }
  if (lo < 1)
    return fail(CHIMERA_ENOMEM,
                "one lambda point of this event set needs " +
                    std::to_string(device_launch_bytes(ctx, ev, 1, f32, lnI != nullptr, nlam)) +
                    " scratch bytes, more than the static scratch of " +
                    std::to_string(kStaticScratchBytes) + " (use chimera_lnl_batch)");
  const int64_t E = ev->E;
  for (int64_t c0 = 0; c0 < B; c0 += lo) {
    const int64_t n = std::min(lo, B - c0);
    chimera_status r = run_chunk(ctx, ev, lam + c0 * nlam, n, prec, lnl + c0,
                                 lnI ? lnI + c0 * E : nullptr, nullptr, nullptr, CHIMERA_DEVICE,
                                 nlam, hip_stream, base);
    if (r != CHIMERA_OK) return r;
  }
  return CHIMERA_OK;
}

chimera_status chimera_selection_xi(chimera_ctx* ctx, const double* lam, int64_t B, int32_t prec,
                                    double* ln_xi, double* n_eff, int32_t mem, void* hip_stream) {
  chimera_status s = check_common(ctx, lam, B, prec, mem);
  if (s != CHIMERA_OK) return s;
  if (!ln_xi) return fail(CHIMERA_EINVAL, "null output");
  return run_batch(ctx, nullptr, lam, B, prec, nullptr, nullptr, ln_xi, n_eff, mem, hip_stream);
}

// Lambda points per gradient launch sequence: the per-sample coefficients
// (120 bytes per sample and lambda, 68 in FP32) stay within 16 GiB.
constexpr double kGradScratchCap = 16.0 * (1ull << 30);

int64_t grad_lambda_chunk(const chimera_events* ev, int64_t B, bool f32) {
  const double nbp = ev->n_bins ? (double)ev->P * ev->n_bins : 0.0;   // binned sets' points
  const double per = ((double)ev->n_samp + nbp) * grad_sample_bytes(f32) + 8.0 * ev->E * 23.0;
  const int64_t c = (int64_t)std::max(1.0, std::floor(kGradScratchCap / per));
  return std::min(B, c);
}

// probe_bytes: only size the call's scratch (pool_size of its layout) and
// return, with no device work.
static chimera_status run_grad_chunk(chimera_ctx* ctx, const chimera_events* ev,
                                     const double* lam, int64_t B, int32_t prec, double* lnl,
                                     double* grad, int32_t mem, void* hip_stream,
                                     size_t* probe_bytes = nullptr) {
  hipStream_t st = (hipStream_t)hip_stream;
  HIP_TRY(hipSetDevice(ctx->cfg.device));
  const bool f32 = prec == CHIMERA_FP32;
  const bool host = mem == CHIMERA_HOST;
  const int E = ev->E;
  double dmin = ev->dmin, dmax = ev->dmax;
  if (ctx->n_det) {
    dmin = std::min(dmin, ctx->inj_dmin);
    dmax = std::max(dmax, ctx->inj_dmax);
  }
  const Geometry g = make_geometry(ctx, dmin, dmax);
  const int nchunk = selection_grad_chunks(ctx->n_det);
  const bool compl_ = ctx->miss64 != nullptr;
  double *ntot_eff = nullptr, *dntot = nullptr;
  auto lay = [&](Carve& cv, GradArgs& a, SelGradArgs& sa, GradFinalArgs& fa, double** lam_d,
                 LamParams** P, double2** chi, double2** inv, double2** dtab, double2** chio,
                 double** gz64, float** gz32, int** fm, int** fr) {
    *P = cv.take<LamParams>(B);
    a.Q = cv.take<GradParams>(B);
    *chi = cv.take<double2>((size_t)B * g.n_t);
    *chio = cv.take<double2>((size_t)B * g.n_t);
    *inv = cv.take<double2>((size_t)B * g.n_u);
    *dtab = cv.take<double2>((size_t)B * g.n_t);
    *gz64 = cv.take<double>((size_t)B * g.n_z);
    *gz32 = cv.take<float>((size_t)B * g.n_z);
    a.gf64 = cv.take<double>((size_t)B * 6 * g.n_z);
    a.gf32 = cv.take<float>((size_t)B * 6 * g.n_z);
    *fm = cv.take<int>(B);
    *fr = cv.take<int>(B);
    sa.partial = cv.take<double>((size_t)B * std::max(nchunk, 1) * (2 + CHIMERA_NGRAD));
    a.hd = cv.take<double>((size_t)B * E * 10);
    a.sc = cv.take<double>((size_t)B * 2 * ev->n_samp);
    a.sd = f32 ? (void*)cv.take<float>((size_t)B * kGradDerivFields * ev->n_samp)
               : (void*)cv.take<double>((size_t)B * kGradDerivFields * ev->n_samp);
    if (ev->n_bins) {
      const size_t NB = (size_t)ev->P * ev->n_bins;
      a.bsc = cv.take<double>((size_t)B * 2 * NB);
      a.bsd = f32 ? (void*)cv.take<float>((size_t)B * kGradDerivFields * NB)
                  : (void*)cv.take<double>((size_t)B * kGradDerivFields * NB);
    }
    a.lnI = cv.take<double>((size_t)B * E);
    a.dlnI = cv.take<double>((size_t)B * E * CHIMERA_NGRAD);
    *lam_d = host ? cv.take<double>((size_t)B * CHIMERA_NLAM) : nullptr;
    fa.lnl = host ? cv.take<double>(B) : lnl;
    fa.grad = host ? cv.take<double>((size_t)B * CHIMERA_NGRAD) : grad;
    if (compl_) {
      a.cv64 = cv.take<double>((size_t)B * 2 * g.n_z);
      a.cv32 = cv.take<float>((size_t)B * 2 * g.n_z);
      a.cf = cv.take<double>((size_t)B * 2);
      ntot_eff = cv.take<double>((size_t)B * g.n_z);
      dntot = cv.take<double>((size_t)B * g.n_z);
    }
  };
  GradArgs a{};
  SelGradArgs sa{};
  GradFinalArgs fa{};
  double* lam_d;
  LamParams* P;
  double2 *chi, *inv, *dtab, *chio;
  double* gz64;
  float* gz32;
  int *fm, *fr;
  Carve probe;
  lay(probe, a, sa, fa, &lam_d, &P, &chi, &inv, &dtab, &chio, &gz64, &gz32, &fm, &fr);
  const size_t bytes = probe.off;
  if (probe_bytes) {
    *probe_bytes = pool_size(bytes);
    return CHIMERA_OK;
  }
  if (ctx->cfg.hbm_budget && pool_size(bytes) > ctx->cfg.hbm_budget)
    return fail(CHIMERA_ENOMEM, "call needs " + std::to_string(bytes) +
                                    " scratch bytes, over the context's hbm_budget");
  void* base = nullptr;
  chimera_ctx::Arena* ar = arena_of(ctx, st);
  std::lock_guard<std::mutex> stream_lock(ar->mu);
  HIP_TRY(arena_reserve(ar, st, bytes, &base));
  Carve cv;
  cv.base = (char*)base;
  lay(cv, a, sa, fa, &lam_d, &P, &chi, &inv, &dtab, &chio, &gz64, &gz32, &fm, &fr);
  const double* lam_dev = lam;
  if (host) {
    HIP_TRY(hipMemcpyAsync(lam_d, lam, (size_t)B * CHIMERA_NLAM * sizeof(double),
                           hipMemcpyHostToDevice, st));
    lam_dev = lam_d;
  }
  HIP_TRY(launch_tables(lam_dev, CHIMERA_NLAM, (int)B, g, P, nullptr, chi, inv, dtab, gz64, gz32,
                        fm, fr, st));
  HIP_TRY(launch_chi_om_table(P, (int)B, g, chio, st));
  a.P = P; a.flag_mono = fm; a.flag_range = fr;
  a.chi = chi; a.chio = chio; a.inv = inv; a.dtab = dtab; a.g = g;
  a.gz64 = gz64; a.gz32 = gz32; a.nz64 = rows64(ctx, ev); a.nz32 = rows32(ctx, ev);
  a.mz64 = compl_ ? miss64(ctx, ev) : nullptr;
  a.mz32 = compl_ ? miss32(ctx, ev) : nullptr;
  a.ev_samp_off = ev->ev_samp_off; a.samp_row = ev->samp_row; a.samp_c = ev->samp_c;
  a.dl = ev->dl; a.lndl = ev->lndl; a.m1d = ev->m1d; a.m2d = ev->m2d;
  a.lnm1d = ev->lnm1d; a.lnm2d = ev->lnm2d;
  a.E = E; a.B = (int)B; a.S = ev->n_samp; a.f32 = f32 ? 1 : 0;
  a.trunc = f32 ? ctx->cfg.trunc_fp32 : ctx->cfg.trunc_fp64;
  a.shape = ev->shape;
  a.bins = ev->n_bins;
  a.n_slots = ev->P;
  a.ev_slot_off = ev->ev_slot_off; a.slot_row = ev->slot_row;
  a.pix_off = ev->pix_off; a.pix_idx = ev->pix_idx;
  sa.P = P; sa.Q = a.Q; sa.flag_mono = fm; sa.flag_range = fr;
  sa.chi = chi; sa.chio = chio; sa.inv = inv; sa.dtab = dtab; sa.g = g;
  sa.ntot = compl_ ? ntot_eff : ctx->ntot;
  sa.ntot_stride = compl_ ? g.n_z : 0;
  sa.dntot_om = compl_ ? dntot : nullptr;
  sa.dl = ctx->inj_dl; sa.lndl = ctx->inj_lndl; sa.m1d = ctx->inj_m1d; sa.m2d = ctx->inj_m2d;
  sa.lnm1d = ctx->inj_lnm1d; sa.lnm2d = ctx->inj_lnm2d; sa.ln_pdraw = ctx->inj_lnp;
  sa.n_det = ctx->n_det; sa.B = (int)B; sa.nchunk = nchunk;
  fa.P = P; fa.flag_mono = fm; fa.flag_range = fr; fa.partial = sa.partial; fa.nchunk = nchunk;
  fa.lnI = a.lnI; fa.dlnI = a.dlnI; fa.E = E; fa.n_total = ctx->n_inj_total;
  fa.neff_gate = ctx->neff_gate;
  HIP_TRY(launch_grad(a, sa, fa, f32, st, ctx->ntot, ctx->missing));
  if (host) {
    HIP_TRY(hipMemcpyAsync(lnl, fa.lnl, B * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(grad, fa.grad, (size_t)B * CHIMERA_NGRAD * sizeof(double),
                           hipMemcpyDeviceToHost, st));
  }
  if (host) HIP_TRY(hipStreamSynchronize(st));
  return CHIMERA_OK;
}

static chimera_status run_grad(chimera_ctx* ctx, const chimera_events* ev, const double* lam,
                               int64_t B, int32_t prec, double* lnl, double* grad, int32_t mem,
                               void* hip_stream) {
  const int64_t Bc = grad_lambda_chunk(ev, B, prec == CHIMERA_FP32);
  for (int64_t c0 = 0; c0 < B; c0 += Bc) {
    const int64_t n = std::min(Bc, B - c0);
    chimera_status s = run_grad_chunk(ctx, ev, lam + c0 * CHIMERA_NLAM, n, prec, lnl + c0,
                                      grad + c0 * CHIMERA_NGRAD, mem, hip_stream);
    if (s != CHIMERA_OK) return s;
  }
  return CHIMERA_OK;
}

chimera_status chimera_lnl_grad(chimera_ctx* ctx, const chimera_events* ev, const double* lam,
                                int64_t B, int32_t prec, double* lnl, double* grad, int32_t mem,
                                void* hip_stream) {
  chimera_status s = check_common(ctx, lam, B, prec, mem);
  if (s != CHIMERA_OK) return s;
  if (!ev) return fail(CHIMERA_EINVAL, "null event set");
  if (!lnl || !grad) return fail(CHIMERA_EINVAL, "null output");
  if (ev->V != 0)
    return fail(CHIMERA_EINVAL, "the adjoint takes the many-1D or single-1D kernels");
  if (ctx->nlam != CHIMERA_NLAM)
    return fail(CHIMERA_EINVAL, "the adjoint takes the unsmoothed mass model (no delta_m)");
  return run_grad(ctx, ev, lam, B, prec, lnl, grad, mem, hip_stream);
}

chimera_status chimera_grad_scratch_bytes(chimera_ctx* ctx, const chimera_events* ev, int64_t B,
                                          int32_t prec, int32_t mem, size_t* bytes) {
  if (!ctx || !ev || !bytes) return fail(CHIMERA_EINVAL, "null argument");
  if (B < 1 || B > (1 << 20)) return fail(CHIMERA_EINVAL, "batch size out of [1, 2^20]");
  if (prec != CHIMERA_FP64 && prec != CHIMERA_FP32) return fail(CHIMERA_EINVAL, "bad precision");
  if (mem != CHIMERA_HOST && mem != CHIMERA_DEVICE) return fail(CHIMERA_EINVAL, "bad mem");
  B = grad_lambda_chunk(ev, B, prec == CHIMERA_FP32);
  return run_grad_chunk(ctx, ev, nullptr, B, prec, nullptr, nullptr, mem, nullptr, bytes);
}

chimera_status chimera_profile_enable(chimera_ctx* ctx, int32_t on) {
  if (!ctx) return fail(CHIMERA_EINVAL, "null context");
  std::lock_guard<std::mutex> lk(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->cfg.device));
  if (on && !ctx->d_count) {
    HIP_TRY(hipMalloc((void**)&ctx->d_count, sizeof(unsigned long long)));
    HIP_TRY(hipMemset(ctx->d_count, 0, sizeof(unsigned long long)));
  }
  ctx->profile = on != 0;
  return CHIMERA_OK;
}

chimera_status chimera_profile_read(chimera_ctx* ctx, int64_t* n_launches, double* total_ms,
                                    int64_t* n_evals) {
  if (!ctx) return fail(CHIMERA_EINVAL, "null context");
  std::lock_guard<std::mutex> lk(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->cfg.device));
  double ms = 0.0;
  for (auto& m : ctx->marks) {
    HIP_TRY(hipEventSynchronize(m.second));
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, m.first, m.second));
    ms += t;
    (void)hipEventDestroy(m.first);
    (void)hipEventDestroy(m.second);
  }
  const int64_t n = (int64_t)ctx->marks.size();
  ctx->marks.clear();
  unsigned long long cnt = 0;
  if (ctx->d_count) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(&cnt, ctx->d_count, sizeof(cnt), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(ctx->d_count, 0, sizeof(cnt)));
  }
  if (n_launches) *n_launches = n;
  if (total_ms) *total_ms = ms;
  if (n_evals) *n_evals = (int64_t)cnt;
  return CHIMERA_OK;
}

}  // extern "C"
