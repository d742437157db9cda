/*
 * chimera.h -- C-ABI of the MI355X library that evaluates the hierarchical
 * standard-siren log-likelihood of Tagliazucchi et al. (2025),
 * arXiv:2504.02034, at batches of hyperparameter points lambda.
 *
 *   ln L(lambda) = sum_i ln I_i(lambda) - N_ev ln xi(lambda)        (eq. hyperlike)
 *
 * I_i is the many-1D kernel integral of event i (eq. like-integrals with the
 * KDE of eq. gw-kernel-many1d): for every sky pixel r of the event's region,
 *   I_i = sum_r c_ir sum_{j in r} w_j sum_g tau_g N(z_g; z_j, h_i) n_r(z_g) g(z_g),
 * where z_j solves d_L^gw(z) = d_j (eqs. dL-em and dL-mg, flat LCDM),
 * w_j = p(m1_j) p(m2_j | m1_j) of the source-frame masses m = m_det/(1+z_j)
 * (power law + Gaussian peak, Sect. 3.1), g(z) = psi(z) / [(1+z)^3 d d_L^gw/dz]
 * (eq. jacobian with the Madau-Dickinson rate psi), tau_g the trapezoid
 * weights of the uniform redshift grid, and h_i one Gaussian bandwidth per
 * (event, lambda) from Scott's rule with the Kish effective sample size
 * (the paper leaves the rule open).  xi is the injection estimator of
 * Sect. 2.2 (with 1/p_draw).
 *
 * Conventions
 *   units        distances in Mpc, H0 in km/s/Mpc, masses in solar masses
 *   lambda       row-major double [B][14]:
 *                H0, Om, Xi0, n, alpha, beta, mmin, mmax, mu_g, sigma_g,
 *                lambda_g, gamma, kappa, z_p
 *                ([B][15] with delta_m last once chimera_set_mass_smoothing
 *                is on; chimera_lambda_width gives the current width)
 *   gradient     row-major double [B][12], the same order without mmin, mmax
 *   ownership    the caller owns every array it passes; the library copies
 *                what it keeps (catalogue, events, injections) to the device
 *                and owns those copies until chimera_release_events /
 *                chimera_destroy
 *   mem          CHIMERA_HOST: lam and outputs are host pointers; the call
 *                returns when the outputs are written.
 *                CHIMERA_DEVICE: lam and outputs are device pointers on the
 *                context's device; the work is enqueued on hip_stream
 *                (a hipStream_t, NULL = the null stream) and the call returns
 *                without waiting.
 *   per-lambda   a lambda outside the domain (non-finite entry, H0 <= 0,
 *   results      Om outside (0,1], Xi0 <= 0, mmin <= 0, mmax <= mmin,
 *                sigma_g <= 0, lambda_g outside [0,1], z_p <= -1,
 *                delta_m < 0), or for
 *                which d_L^gw is not increasing on the distance table, gives
 *                lnl = -inf; one for which a resident distance exceeds
 *                d_L^gw(z_tab_max) gives lnl = NaN.  Neither is a call
 *                error: the other points of the batch are unaffected.
 *                An event with I_i = 0, or xi = 0, gives lnl = -inf.
 *   errors       every call returns a chimera_status; on failure the
 *                calling thread's chimera_last_error() describes it.
 *   threads      one context may be used from several host threads and
 *                streams at once for evaluation calls; chimera_set_* and
 *                chimera_add_events / chimera_release_events serialise on
 *                the context and must not race with evaluations that read
 *                the data they replace.
 */
#ifndef CHIMERA_H
#define CHIMERA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct chimera_ctx chimera_ctx;
typedef struct chimera_events chimera_events;

/* Largest number of pixel rows of one event.  The FP32 form stages every row
 * of such an event in the kernels' on-chip slice of the catalogue density;
 * FP64 does up to 2048 rows (more when the kernel windows are narrow) and
 * evaluates a larger event by direct sums (equal up to rounding). */
#define CHIMERA_MAX_EVENT_PIXELS 2560

typedef enum {
  CHIMERA_OK = 0,
  CHIMERA_EINVAL = -1,   /* bad argument (null pointer, size, layout) */
  CHIMERA_ENOMEM = -2,   /* device allocation failed or scratch > hbm_budget */
  CHIMERA_EDEVICE = -3,  /* HIP runtime error */
  CHIMERA_ERANGE = -4,   /* data outside what the context was configured for */
  CHIMERA_ESTATE = -5    /* catalogue / injections not set yet */
} chimera_status;

enum { CHIMERA_FP64 = 0, CHIMERA_FP32 = 1 };
enum { CHIMERA_HOST = 0, CHIMERA_DEVICE = 1 };

#define CHIMERA_NLAM 14
#define CHIMERA_NGRAD 12

/* 1-D kernel shapes of an event set (chimera_set_event_kde). */
enum { CHIMERA_KDE_GAUSSIAN = 0, CHIMERA_KDE_EPANECHNIKOV = 1 };
/* Largest number of bins per KDE data set. */
#define CHIMERA_MAX_BINS 4096

typedef struct {
  int32_t n_z;          /* redshift grid points (>= 3)                                */
  double z_lo, z_hi;    /* grid z_g = z_lo + g (z_hi - z_lo)/(n_z - 1)                 */
  int32_t n_tab;        /* nodes of the per-lambda distance tables (>= 256)           */
  double z_tab_max;     /* the tables cover z in [0, z_tab_max]                        */
  double trunc_fp64;    /* kernel support |z_g - z_j| <= T h in FP64 mode (>= 8.6)     */
  double trunc_fp32;    /* ... in FP32 mode (same quantity: keep it equal to trunc_fp64) */
  int32_t device;       /* HIP device ordinal                                          */
  size_t hbm_budget;    /* max scratch bytes one call may take; 0 = no limit           */
} chimera_config;

/* Fill cfg with defaults: n_z 1000 on [0, 1.6], n_tab 8192, z_tab_max 25,
 * trunc 8.6 in both precisions, device 0, no budget. */
void chimera_default_config(chimera_config* cfg);

/* Create a context on cfg->device.  Returns EINVAL for an inconsistent
 * config, EDEVICE if the device cannot be used. */
chimera_status chimera_create(const chimera_config* cfg, chimera_ctx** out);
void chimera_destroy(chimera_ctx* ctx);

/* Message of the calling thread's last failed call ("" if none). */
const char* chimera_last_error(void);

/* Galaxy-catalogue density on the grid (eq. p-cat, pre-computed once as in
 * Sect. 2.3 step b): nz is row-major [n_rows][n_z], n_r(z_g) per unit z per
 * steradian for each catalogue row that events refer to; nz_tot[n_z] is the
 * all-sky density n_tot(z_g) = pixel area x sum over all pixels, used by the
 * selection term.  Replaces any previous catalogue; returns ERANGE (and keeps
 * the current one) when a resident event set refers to a row at or past
 * n_rows — release such sets first. */
chimera_status chimera_set_catalog(chimera_ctx* ctx, int64_t n_rows, const double* nz,
                                   const double* nz_tot);

/* The catalogue density built on the device from the galaxies (the same
 * quantity as chimera_set_catalog's rows, eq. like-integrals' p_cat on the
 * grid): each galaxy's N(z; z_obs, sigma_z) truncated to 8 sigma_z is
 * projected on the grid's hat basis (half hats at the ends), weighted by
 * vshape[k] (the comoving volume element shape at node k) and normalised to
 * sum_k tau_k q_k = 1; then, over the n_used galaxies whose projection is not
 * zero, n_r(z_k) = sum_{gal in pixel} q_k / (n_used pixel_area) for the
 * pixels rows_pix[n_rows] (row r of the catalogue is pixel rows_pix[r]) and
 * n_tot(z_k) = sum_{all galaxies} q_k / n_used.
 *   gal_pix_off[n_pix+1]   galaxies of pixel p are [gal_pix_off[p], gal_pix_off[p+1])
 *   z_obs, sigma_z[n_gal]  sorted by pixel; sigma_z = 0 drops a galaxy
 *   vshape[n_z]            >= 0
 * Host arrays; synchronous.  Replaces any previous catalogue.  n_used may be
 * NULL.  Returns EINVAL on malformed input, ERANGE when a row names a pixel
 * past n_pix or when a resident event set refers to a row at or past n_rows
 * (the current catalogue is kept), ENOMEM when the device cannot hold
 * n_pix x n_z doubles. */
chimera_status chimera_set_catalog_galaxies(chimera_ctx* ctx, int64_t n_pix, int64_t n_gal,
                                            const int64_t* gal_pix_off, const double* z_obs,
                                            const double* sigma_z, const double* vshape,
                                            double pixel_area, int64_t n_rows,
                                            const int64_t* rows_pix, int64_t* n_used);

/* Copy the resident catalogue to the host: nz[n_rows][n_z] (FP64) and
 * nz_tot[n_z]; either may be NULL.  Synchronous.  ESTATE before a catalogue
 * is set. */
chimera_status chimera_get_catalog(chimera_ctx* ctx, double* nz, double* nz_tot);

/* Detected injections (Sect. 2.2): n_det draws with d_L, detector-frame
 * masses and ln p_draw (the draw density in (d_L, m1_det, m2_det)), out of
 * n_inj_total draws in all.  Distances must be > 0.  Replaces any previous set. */
chimera_status chimera_set_injections(chimera_ctx* ctx, int64_t n_det, int64_t n_inj_total,
                                      const double* dl, const double* m1d, const double* m2d,
                                      const double* ln_pdraw);

/* One resident event set in CSR layout (many-1D kernel, eq. gw-kernel-many1d):
 *   ev_pix_off[n_ev+1]      pixel rows of event i are [ev_pix_off[i], ev_pix_off[i+1])
 *   pix_samp_off[P+1]       samples of pixel row p are [pix_samp_off[p], pix_samp_off[p+1])
 *   pix_row[P]              catalogue row (index into nz) of pixel row p
 *   c_ir[P]                 sky factor / sample count of pixel row p (> 0)
 *   dl, m1d, m2d[n_samp]    samples, n_samp = pix_samp_off[P], ordered by
 *                           (event, pixel); within a pixel, ascending dl runs
 *                           fastest but any order is accepted
 * Every event must have at least one sample.  Distances > 0.  An event may
 * have at most CHIMERA_MAX_EVENT_PIXELS pixel rows.
 * Returns EINVAL on a malformed layout, ERANGE when a pixel row refers past
 * the catalogue or an event exceeds the largest size the kernels take. */
chimera_status chimera_add_events(chimera_ctx* ctx, int32_t n_ev, const int64_t* ev_pix_off,
                                  const int64_t* pix_samp_off, const int64_t* pix_row,
                                  const double* c_ir, const double* dl, const double* m1d,
                                  const double* m2d, chimera_events** out);

/* One resident event set for the single-1D kernel (eq. gw-kernel-single1d,
 * Sect. 2.3): each event's redshift KDE is one weighted KDE over all its
 * samples, KDE_i(z) = (1/N_i) sum_j w_j N(z; z_j, h_i), and its pixels enter
 * only through their sky factors,
 *   I_i = sum_r S_ir sum_g tau_g n_r(z_g) g(z_g) KDE_i(z_g).
 *   ev_samp_off[n_ev+1]   samples of event i are [ev_samp_off[i], ev_samp_off[i+1])
 *   dl, m1d, m2d[n_samp]  all N_i samples of each event (n_samp = ev_samp_off[n_ev]);
 *                         any order within an event
 *   ev_pix_off[n_ev+1]    pixels of event i are [ev_pix_off[i], ev_pix_off[i+1])
 *   pix_row[P]            catalogue row of each pixel
 *   s_ir[P]               sky factor S_ir of each pixel (> 0; with the many-1D
 *                         layout of the same region, S_ir = c_ir x N_ir)
 * The bandwidth h_i is taken over the same N_i samples.  The library folds
 * the sky factors into one row per event, sum_r S_ir n_r(z_g) (lambda does
 * not enter), at this call and again whenever the catalogue is replaced, and
 * then runs the many-1D kernels with one pseudo-pixel of c = 1/N_i per event:
 * every evaluation call (ln L, gradient, the allocation-free variant) takes
 * the returned set.  The set holds n_ev x n_z doubles and floats of rows.
 * There is no limit on an event's pixel count.  Host arrays; synchronous.
 * Returns EINVAL on a malformed layout, ERANGE when a pixel refers past the
 * catalogue, ESTATE before a catalogue is set. */
chimera_status chimera_add_events_single1d(chimera_ctx* ctx, int32_t n_ev,
                                           const int64_t* ev_samp_off, const double* dl,
                                           const double* m1d, const double* m2d,
                                           const int64_t* ev_pix_off, const int64_t* pix_row,
                                           const double* s_ir, chimera_events** out);

/* One resident event set for the 3D kernel (Sect. 2.2; kept in Sect. 2.3):
 * each event's kernel is one Gaussian KDE of its N_i samples in (z, u, v),
 * (u, v) the sample's position in a flat chart of the event's sky region
 * (e.g. gnomonic coordinates on the plane tangent at the samples' mean
 * direction, in radians), evaluated at each pixel centre:
 *   I_i = sum_k area_k sum_g tau_g n_k(z_g) g(z_g) (1/N_i) sum_j w_j N3(r; H_i),
 *   r = (z_g - z_j, u_k - u_j, v_k - v_j),
 * H_i = the weighted covariance of (z, u, v) x n_eff^(-2/7) at each lambda
 * (Scott's factor in three dimensions, Kish effective size).  The kernel
 * runs through the many-1D sums: per (pixel, sample) pair a point at
 * z_j + B dO (B = H_zO H_OO^-1) of weight w_j N2(dO; H_OO), all with the
 * conditional width s_i (s_i^2 = H_zz - B H_Oz); a pair counts when the sky
 * part of the quadratic form is <= T^2, a grid point when |z_g - z_j - B dO|
 * <= T s_i (T: the context's truncation).  An event whose H_i is not
 * positive definite, or whose weights vanish, has I_i = 0.
 *   ev_samp_off[n_ev+1]       samples of event i: [ev_samp_off[i], ev_samp_off[i+1])
 *   dl, m1d, m2d[n_samp]      every sample of each event
 *   sky_u, sky_v[n_samp]      their chart coordinates
 *   ev_pix_off[n_ev+1]        pixels of event i: [ev_pix_off[i], ev_pix_off[i+1])
 *   pix_row[P]                catalogue row of each pixel
 *   pix_u, pix_v[P]           pixel centres in the event's chart
 *   pix_area[P]               pixel areas [sr] (> 0)
 * An event may have at most CHIMERA_MAX_EVENT_PIXELS pixels, and the set
 * at most 2^31 - 1 (pixel, sample) pairs; the evaluation scratch holds a
 * redshift and a weight per pair and lambda point (calls run in chunks of
 * points as for chimera_lnl_batch).  chimera_lnl_grad and
 * chimera_set_event_kde (other than the defaults) refuse such a set.  Host
 * arrays; synchronous.  EINVAL on a malformed layout, ERANGE when a pixel
 * refers past the catalogue or a size limit is exceeded, ESTATE before a
 * catalogue is set. */
chimera_status chimera_add_events_3d(chimera_ctx* ctx, int32_t n_ev, const int64_t* ev_samp_off,
                                    const double* dl, const double* m1d, const double* m2d,
                                    const double* sky_u, const double* sky_v,
                                    const int64_t* ev_pix_off, const int64_t* pix_row,
                                    const double* pix_u, const double* pix_v,
                                    const double* pix_area, chimera_events** out);
chimera_status chimera_release_events(chimera_ctx* ctx, chimera_events* ev);

/* An incomplete catalogue (eqs. p-gal, p-miss, f-R): the galaxy density
 * becomes p_gal = f_R p_cat + (1 - f_R) p_miss with the missing galaxies
 * spread homogeneously in comoving volume up to the grid's end z_max:
 *   row r:   f_R n_r(z) + (1 - P_r(z)) v(z),
 *   n_tot:   f_R n_tot(z) + M(z) v(z),
 *   v(z) = (dV_c/dz per sr)(z) / V_c(z_max) = chi(z)^2 / (E(z) (4 pi/3) chi(z_max)^3),
 *   f_R = sum_g tau_g (4 pi - M(z_g)) v(z_g)   (eq. f-R on the grid),
 * at every lambda (v and f_R depend on Om).  p_compl[n_rows][n_z]: the
 * completeness P_compl of each catalogue row's pixel on the grid, in [0, 1];
 * missing[n_z]: M(z_g) = sum over all sky pixels of area x (1 - P_compl),
 * in [0, 4 pi] sr.  p_compl = NULL returns to a complete catalogue.  Applies
 * to later calls; replacing the catalogue clears it; resident single-1D
 * sets fold it as they fold the rows.  chimera_lnl_grad differentiates it
 * (f_R and v depend on Om).  Host arrays; synchronous.  ESTATE before a
 * catalogue is set, EINVAL for values out of range. */
chimera_status chimera_set_completeness(chimera_ctx* ctx, const double* p_compl,
                                       const double* missing);

/* The injection sum's stability check of Sect. 2.2 (reading: the effective
 * number of injections must exceed factor x the number of events of the
 * likelihood; the paper uses 5).  Once set, chimera_lnl_batch,
 * chimera_lnl_batch_static and chimera_lnl_grad give lnl = -inf (and a NaN
 * gradient) at every point whose ln L would be finite but whose N_eff <=
 * factor x n_ev of the event set.  factor = 0 (the default) turns the check
 * off.  EINVAL for a negative or non-finite factor.  Applies to later calls;
 * do not change it while calls are in flight. */
chimera_status chimera_set_neff_gate(chimera_ctx* ctx, double factor);

/* The smoothed lower edge of the mass model (Table 1's delta_m; the paper
 * takes the model's full form from the population literature).  on = 1:
 * every later call reads lambda rows of 15 doubles, delta_m >= 0 last; for
 * delta_m > 0 both p(m1) (power law + peak) and the power law of p(m2|m1)
 * are multiplied by
 *   S(m) = 0 for m <= mmin, 1 for m >= mmin + delta_m, and
 *   1 / (exp(delta_m/m' + delta_m/(m' - delta_m)) + 1) between, m' = m - mmin,
 * and normalised again on their supports: p(m1) by N1 = int p(m1) S dm,
 * p(m2|m1) by C(m1) = int_mmin^m1 m^beta S dm.  Per lambda a table on 4097
 * equal nodes of [mmin, min(mmax, mmin + delta_m)] holds C / (m^beta S) and
 * its derivative (Gauss-Legendre panels, sub-divided where S rises steeply;
 * cubic Hermite between the nodes), so the weights keep their relative
 * accuracy far down the edge; past the edge C is the table's end plus the
 * power law's closed form.  In FP32 mode an event's weights are formed as
 * logs and scaled by a per-(event, lambda) factor that ln I_i takes back,
 * so events whose weights all lie below FP32's range keep a finite ln I_i.
 * delta_m = 0 gives the unsmoothed model bitwise.  on = 0 returns to
 * 14-entry rows.
 * chimera_lnl_grad refuses a context with it on (EINVAL).  Applies to later
 * calls; do not change it while calls are in flight.  EINVAL for on not 0/1. */
chimera_status chimera_set_mass_smoothing(chimera_ctx* ctx, int32_t on);

/* The number of doubles per lambda row that calls on ctx read (14 or 15). */
chimera_status chimera_lambda_width(chimera_ctx* ctx, int32_t* width);

/* Kernel options of a resident event set (Sect. 2.3: the 1-D KDEs take a
 * Gaussian or an Epanechnikov kernel, and their data sets may be binned).
 *   shape   CHIMERA_KDE_GAUSSIAN (the default of every set) or
 *           CHIMERA_KDE_EPANECHNIKOV: K(z; z_j, h) = 3/(4 a h) (1 - u^2) for
 *           |u| <= 1, u = (z - z_j)/(a h), a = sqrt(5) (the kernel of
 *           variance h^2, so the bandwidth rule is unchanged); its support
 *           replaces the T h window
 *   n_bins  0 (the samples themselves) or 1..CHIMERA_MAX_BINS: at each
 *           lambda every KDE data set (a pixel's samples, or for a single-1D
 *           set the event's) is replaced by n_bins equal-width bins over its
 *           redshift range, each a point at the bin's centre carrying the
 *           summed weight of its samples (the largest redshift in the last
 *           bin; all samples at one redshift: one point there).  The
 *           bandwidth and the 1/N normalisation stay those of the samples.
 * Later evaluation calls on the set use the options, chimera_lnl_grad
 * included.  Synchronous; waits
 * for the device, so no call may be using the set.  EINVAL on a bad shape,
 * n_bins out of range or an unknown set; ERANGE when the set's pixel slots
 * times n_bins exceed 2^31 - 1. */
chimera_status chimera_set_event_kde(chimera_ctx* ctx, chimera_events* ev, int32_t shape,
                                     int32_t n_bins);

/* ln L at B points (eq. hyperlike).  prec: CHIMERA_FP64, or CHIMERA_FP32 for
 * FP32 bulk arithmetic (mass weights, kernel sums) with the distance tables,
 * the inversion, the bandwidth moments and every per-event and per-lambda sum
 * kept in FP64.  lnl[B]; lnI[B][n_ev] (ln I_i per point and event) may be NULL.
 * A call whose per-sample scratch (a redshift and a weight per sample and
 * point) would exceed 8 GiB runs as consecutive chunks of points on the same
 * stream; every point's result is independent of the chunking. */
chimera_status chimera_lnl_batch(chimera_ctx* ctx, const chimera_events* ev, const double* lam,
                                 int64_t B, int32_t prec, double* lnl, double* lnI, int32_t mem,
                                 void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * chimera_lnl_batch in device mode (lam, lnl and lnI are device pointers, the
 * work is enqueued on hip_stream) with its per-call scratch laid out in a
 * static array of 256 MiB per device that the library holds from its load
 * until the process ends, so the call allocates nothing.  Larger batches run
 * as consecutive launch sequences of the points that fit; results are the
 * same as chimera_lnl_batch's.  Every call on a device shares that device's
 * array: calls whose work overlaps on one device (other streams, other
 * contexts or threads) race and must be serialised by the caller (e.g. one
 * stream).  ENOMEM, with nothing enqueued, when one point of the event set
 * needs more scratch than the array holds (about 16 bytes per sample in FP64
 * and 12 in FP32, plus 0.4 MB); no profiling events are recorded. */
chimera_status chimera_lnl_batch_static(chimera_ctx* ctx, const chimera_events* ev,
                                        const double* lam, int64_t B, int32_t prec, double* lnl,
                                        double* lnI, void* hip_stream);

/* ln xi and the effective injection count N_eff (Sect. 2.2) at B points.
 * n_eff may be NULL. */
chimera_status chimera_selection_xi(chimera_ctx* ctx, const double* lam, int64_t B, int32_t prec,
                                    double* ln_xi, double* n_eff, int32_t mem, void* hip_stream);

/* Device scratch (bytes) that one launch sequence of chimera_lnl_batch uses
 * for B points of event set ev (NULL: the selection alone) in precision prec
 * and memory mode mem, rounded up to a power of two (with an event set, the
 * per-event ln I_i buffer is always counted).  The context keeps one scratch
 * block per stream, grown to the largest such size used on that stream and
 * reused by later calls on it (work on a stream runs in order); a call holds
 * its stream's block until its last launch is enqueued (a host call until its
 * results are back), so calls from several host threads on one stream run
 * one after the other.  For admission control by an HBM budget:
 * chimera_config's hbm_budget bounds one call; a scheduler of concurrent
 * calls on several streams bounds the sum of the blocks (chimera_scratch_held)
 * and frees idle ones (chimera_release_scratch).  For a chunked call (see
 * chimera_lnl_batch) this is one chunk's scratch. */
chimera_status chimera_scratch_bytes(chimera_ctx* ctx, const chimera_events* ev, int64_t B,
                                     int32_t prec, int32_t mem, size_t* bytes);

/* The same for chimera_lnl_grad: the stream's scratch block that a gradient
 * call over B points needs (one chunk's, for a chunked call: see
 * chimera_lnl_grad).  EINVAL for a null argument, B outside [1, 2^20], an
 * unknown precision or mem. */
chimera_status chimera_grad_scratch_bytes(chimera_ctx* ctx, const chimera_events* ev, int64_t B,
                                          int32_t prec, int32_t mem, size_t* bytes);

/* Bytes of the scratch blocks the context holds, summed over its streams. */
chimera_status chimera_scratch_held(chimera_ctx* ctx, size_t* bytes);

/* Free the scratch block of hip_stream (after the work enqueued on it) and
 * return the freed memory to the device, keeping in the stream-ordered pool
 * only what the context's other blocks add up to.  Synchronises hip_stream.
 * A later call on the stream allocates a new block. */
chimera_status chimera_release_scratch(chimera_ctx* ctx, void* hip_stream);

/* ln L and its gradient at B points (the adjoint of eq. hyperlike through
 * every step above: the redshift of each sample as an implicit function of
 * d_L^gw(z_j) = d_j, the mass weights, the bandwidth, the kernel sums, the
 * grid factor and the selection estimator).  lnl[B]; grad[B][12] =
 * d ln L / d(H0, Om, Xi0, n, alpha, beta, mu_g, sigma_g, lambda_g, gamma,
 * kappa, z_p); mmin and mmax are edges of the mass support and are not
 * differentiated.  The window edges |z_g - z_j| = T h are held fixed.  prec:
 * CHIMERA_FP64, or CHIMERA_FP32 for the per-sample window sums and the
 * stored per-sample derivatives in FP32 (the sample transform, bandwidth,
 * selection and every sum over samples, events and injections in FP64).  lnl
 * follows chimera_lnl_batch's rules; grad is NaN where lnl is not finite.
 * The per-lambda layout is the same as above.  Device scratch grows with 120
 * bytes per sample and point (68 in FP32); a call whose scratch would exceed
 * 16 GiB runs as consecutive chunks of points on the same stream, with the
 * same results.  With an incomplete catalogue (chimera_set_completeness) the
 * rows f_R n_r + (1 - P_r) v and n_tot^eff add their Om derivatives
 * (f_R' n_r + (1 - P_r) v', f_R' n_tot + M v', with d ln v / d Om =
 * 2 chi'/chi - E'/E - 3 chi'(z_max)/chi(z_max)).  A set with the
 * Epanechnikov kernel (chimera_set_event_kde, Sect. 2.3's compact option,
 * unbinned) is differentiated with k = 1 - u^2/W^2 on its support
 * |u| <= W = sqrt(5) h (dk/dz_j = 2u/W^2, h dk/dh = 2u^2/W^2; k vanishes on
 * the support's edge).  A binned set (n_bins > 0) is differentiated through
 * its bins: a bin's weight moves with its samples' weights (the samples'
 * bins held fixed) and its centre with the ends of the data set's redshift
 * range.  EINVAL for a 3D set or a context with the smoothed mass edge on. */
chimera_status chimera_lnl_grad(chimera_ctx* ctx, const chimera_events* ev, const double* lam,
                                int64_t B, int32_t prec, double* lnl, double* grad, int32_t mem,
                                void* hip_stream);

/* Diagnostics.  With profiling on, every chimera_lnl_batch call on this
 * context brackets its event kernel with HIP events recorded on the call's
 * stream, and the kernel counts the (sample, grid point) pairs it evaluates
 * (the windows |z_g - z_j| <= T h of samples with nonzero weight).
 * chimera_profile_read waits for the recorded events, returns the number of
 * event-kernel launches, their summed duration in milliseconds and the summed
 * evaluation count since the last read, and resets them. */
chimera_status chimera_profile_enable(chimera_ctx* ctx, int32_t on);
chimera_status chimera_profile_read(chimera_ctx* ctx, int64_t* n_launches, double* total_ms,
                                    int64_t* n_evals);

#ifdef __cplusplus
}
#endif

#endif /* CHIMERA_H */
