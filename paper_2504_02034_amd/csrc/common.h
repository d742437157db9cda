// Device-side types and helpers of the likelihood library (gfx950).
//
// Notation follows arXiv:2504.02034: d_L^em (eq. dL-em), Xi (eq. dL-mg),
// the detector-frame Jacobian (eq. jacobian), the PLP mass model and the
// Madau-Dickinson rate (Sect. 3.1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace chimera {

constexpr double kCkms = 299792.458;   // speed of light [km/s]
constexpr int kNlam = 14;            // lambda entries (15 with delta_m, chimera_set_mass_smoothing)
constexpr double kInvSqrt2Pi = 0.39894228040143267794;

// Flags of one lambda (bits).
enum : int { kFlagDomain = 1, kFlagNonMonotone = 2, kFlagRange = 4 };

// Per-lambda constants, computed once per call on the device.
struct LamParams {
  double h0, om, xi0, n, alpha, beta, mmin, mmax, mu, sigma, lg, gamma, kappa, zp;
  double dh;        // c / H0 [Mpc]
  double pl_coef;   // (1 - lambda_g) / int_mmin^mmax m^-alpha dm
  double tg_coef;   // lambda_g / (sigma sqrt(2 pi) Z), Z = peak mass in [mmin, mmax]
  double a2;        // 1 + beta
  double mmin_a2;   // mmin^(1 + beta)
  double ln_mmin, ln_mmax;
  double ln1zp;     // ln(1 + z_p)
  double inv_sigma;
  // smoothed lower mass edge (delta_m > 0; 0: none): S(m) multiplies p(m1)
  // and p(m2|m1), renormalised: 1/N1, Q = int_mmin^top m^beta S dm, the edge
  // mmin + delta_m and its log, top = min(mmax, edge), the table's node step
  double dm, sm_n1inv, sm_q, sm_edge, ln_edge, sm_top, sm_h;
  double sm_pl;     // edge^(1+beta) / (1+beta) (1 at beta = -1): the power law past the edge
  double sm_lnq, sm_lnn1inv;   // ln Q, ln(1/N1)
  int flag;         // kFlagDomain
  int pad;
};

// panels of the per-lambda node table of the smoothed edge on [mmin, top]
constexpr int kMassPanels = 4096;

// Geometry shared by all lambdas of one call.
struct Geometry {
  int n_z;          // redshift grid
  double z_lo, dz, inv_dz;
  int n_t;          // chi table: x_k = k dx, x = ln(1+z)
  double dx, inv_dx;
  int n_u;          // inverse table: u_m = u_lo + m du, u = ln d
  double u_lo, du, inv_du;
};

// Cubic Hermite on [0,1]: values y0, y1 and slopes (times the step) s0, s1.
__device__ __forceinline__ double hermite(double y0, double y1, double s0, double s1, double t) {
  const double d = y1 - y0;
  return y0 + t * (s0 + t * ((3.0 * d - 2.0 * s0 - s1) + t * (s0 + s1 - 2.0 * d)));
}

// chi(x) = int_0^z dz'/E from the per-lambda table of (chi_k, dchi/dx_k).
__device__ __forceinline__ double chi_at(const double2* __restrict__ tab, const Geometry& g,
                                         double x) {
  // clamp in floating point first: NaN and huge values map into the table
  const double q = x * g.inv_dx;
  const double p = fmin(fmax(q, 0.0), (double)(g.n_t - 1));
  int k = (int)p;
  k = k > g.n_t - 2 ? g.n_t - 2 : k;
  const double t = q - (double)k;
  const double2 a = tab[k], b = tab[k + 1];
  return hermite(a.x, b.x, a.y * g.dx, b.y * g.dx, t);
}

// d_L^gw(x) and dd_L^gw/dx from the per-lambda node table of (D_k, dD/dx_k):
// the cubic Hermite and the derivative of the same cubic.
__device__ __forceinline__ void dist_tab_at(const double2* __restrict__ tab, const Geometry& g,
                                            double x, double& D, double& Dx) {
  const double q = x * g.inv_dx;
  const double p = fmin(fmax(q, 0.0), (double)(g.n_t - 1));
  int k = (int)p;
  k = k > g.n_t - 2 ? g.n_t - 2 : k;
  const double t = q - (double)k;
  const double2 a = tab[k], b = tab[k + 1];
  const double s0 = a.y * g.dx, s1 = b.y * g.dx, d = b.x - a.x;
  const double c2 = 3.0 * d - 2.0 * s0 - s1, c3 = s0 + s1 - 2.0 * d;
  D = a.x + t * (s0 + t * (c2 + t * c3));
  Dx = (s0 + t * (2.0 * c2 + 3.0 * t * c3)) * g.inv_dx;
}

__device__ __forceinline__ double efunc_of_zp1(double om, double zp1) {
  return sqrt(om * zp1 * zp1 * zp1 + 1.0 - om);
}

// d_L^gw and its x-derivative at x = ln(1+z).  zp1 = e^x is passed in.
__device__ __forceinline__ void dist_at(const LamParams& P, const double2* __restrict__ tab,
                                        const Geometry& g, double x, double zp1, double& D,
                                        double& dDdx) {
  const double c = chi_at(tab, g, x);
  const double cp = zp1 / efunc_of_zp1(P.om, zp1);       // dchi/dx
  const double en = exp(-P.n * x);                        // (1+z)^-n
  const double xi = P.xi0 + (1.0 - P.xi0) * en;
  const double xi_x = -P.n * (1.0 - P.xi0) * en;
  D = P.dh * zp1 * c * xi;
  dDdx = P.dh * zp1 * (c * xi + cp * xi + c * xi_x);
}

// x = ln(1+z) solving d_L^gw(z) = d: per-lambda inverse table (Hermite in
// u = ln d), then `polish` Newton steps on d_L^gw from the chi table.
__device__ __forceinline__ double invert_x(const LamParams& P, const double2* __restrict__ chi,
                                           const double2* __restrict__ inv, const Geometry& g,
                                           double d, double lnd, int polish) {
  const double pos = (lnd - g.u_lo) * g.inv_du;
  int m = (int)fmin(fmax(pos, 0.0), (double)(g.n_u - 1));
  m = m > g.n_u - 2 ? g.n_u - 2 : m;
  const double t = pos - (double)m;
  const double2 a = inv[m], b = inv[m + 1];
  double x = hermite(a.x, b.x, a.y * g.du, b.y * g.du, t);
  for (int i = 0; i < polish; ++i) {
    double D, Dx;
    dist_at(P, chi, g, x, exp(x), D, Dx);
    x -= (D - d) / Dx;
  }
  return x;
}

// Redshift and mass weight of one sample (Sect. 2.1: z from d_L^gw; the
// masses in the source frame m = m_det / (1+z); eq. gw-kernel weight
// p(m1) p(m2|m1) with uniform PE priors).  FP64 path: inverse table + one
// Newton step on the d_L^gw node table, whose e^x update reuses the
// exponential; FP32 path: inverse table only and the mass model in FP32.
template <bool F32, bool SM = false, bool LOGW = false>
__device__ __forceinline__ void sample_zw(const LamParams& P, const double2* __restrict__ dtab,
                                          const double2* __restrict__ inv, const Geometry& g,
                                          double d, double lnd, double m1d, double m2d,
                                          double lnm1d, double lnm2d, double& z, double& w,
                                          const double2* __restrict__ mt);

// The smoothing of the lower mass edge: 0 at and below mmin, 1 from
// mmin + delta_m on, 1 / (exp(dm/m' + dm/(m' - dm)) + 1) between, m' = m - mmin.
__device__ __forceinline__ double smooth_edge(double m, double mmin, double dm) {
  const double mp = m - mmin;
  if (mp >= dm) return 1.0;
  if (!(mp > 0.0)) return 0.0;
  return 1.0 / (exp(dm / mp + dm / (mp - dm)) + 1.0);
}

// p(m1) p(m2|m1) with the smoothed edge: the unsmoothed mixture times
// S(m1) / N1, times m2^beta S(m2) over C(m1) = int_mmin^m1 m^beta S dm.  From
// the edge on, C = Q + the plain power law; below it C = R m1^beta S(m1), whose
// S(m1) cancels against p(m1)'s, with R(m1) the cubic Hermite of the
// per-lambda node table (R, dR/dm).  S(m2) = 1 / (1 + e^y) enters through one
// final division.  The masses, the exponent y and the table in FP64; in FP32
// mode the exponentials and the last products in FP32 (a weight whose e^y
// overflows FP32 is below FP32's range and gives 0).
template <bool F32>
__device__ __forceinline__ double mass_weight_smoothed(const LamParams& P,
                                                       const double2* __restrict__ mt, double m1,
                                                       double m2, double l1, double l2) {
  if (!(m1 >= P.mmin && m1 <= P.mmax && m2 >= P.mmin && m2 <= m1 && m1 > P.mmin)) return 0.0;
  using T = typename std::conditional<F32, float, double>::type;
  const double mp = m2 - P.mmin;
  T ey = (T)0;                                  // e^y of S(m2) = 1 / (1 + e^y)
  if (mp < P.dm) {
    if (!(mp > 0.0)) return 0.0;
    const double y = P.dm * (2.0 * mp - P.dm) / (mp * (mp - P.dm));
    ey = F32 ? __expf((float)y) : (T)exp(y);
    if (!(ey < (T)INFINITY)) return 0.0;
  }
  const bool past = m1 >= P.sm_edge;
  const T lead = (T)(past ? P.beta * l2 : P.beta * (l2 - l1));
  const T u = (T)((m1 - P.mu) * P.inv_sigma);
  const T al1 = (T)(P.alpha * l1);
  T num;
  if (F32)
    num = (T)P.pl_coef * __expf(lead - al1) + (T)P.tg_coef * __expf(lead - (T)0.5 * u * u);
  else
    num = (T)P.pl_coef * exp(lead - al1) + (T)P.tg_coef * exp(lead - (T)0.5 * u * u);
  T c;
  if (past) {
    const double d = l1 - P.ln_edge;
    c = (T)P.sm_q + (P.a2 == 0.0 ? (T)d
                                  : (T)P.sm_pl * (F32 ? expm1f((float)(P.a2 * d)) : (T)expm1(P.a2 * d)));
  } else {
    const double pos = (m1 - P.mmin) / P.sm_h;
    const int k = (int)fmin(fmax(pos, 0.0), (double)(kMassPanels - 1));
    const double t = pos - (double)k;
    const double2 a = mt[k], b = mt[k + 1];
    const double dd = b.x - a.x, s0 = a.y * P.sm_h, s1 = b.y * P.sm_h;
    const double r = a.x + t * (s0 + t * ((3.0 * dd - 2.0 * s0 - s1) + t * (s0 + s1 - 2.0 * dd)));
    if (!(r > 0.0)) return 0.0;
    c = (T)r;
    if (!(c > (T)0)) return 0.0;
  }
  return (double)(num * (T)P.sm_n1inv / (((T)1 + ey) * c));
}

// ln of the smoothed weight in FP32 (-inf for 0), so that an FP32 caller can
// scale an event's weights before they leave FP32's range.  Past the edge
// both the numerator and C carry the factor m1^-(1+beta), which keeps C near
// 1/(1+beta): C m1^-(1+beta) = Q m1^-(1+beta) - expm1(-(1+beta) d)/(1+beta).
__device__ __forceinline__ float lnw_smoothed32(const LamParams& P, const double2* __restrict__ mt,
                                                double m1, double m2, double l1, double l2) {
  if (!(m1 >= P.mmin && m1 <= P.mmax && m2 >= P.mmin && m2 <= m1 && m1 > P.mmin)) return -INFINITY;
  const double mp = m2 - P.mmin;
  float sp = 0.0f;                              // ln(1 + e^y) = -ln S(m2)
  if (mp < P.dm) {
    if (!(mp > 0.0)) return -INFINITY;
    const float y = (float)(P.dm * (2.0 * mp - P.dm) / (mp * (mp - P.dm)));
    sp = fmaxf(y, 0.0f) + log1pf(__expf(-fabsf(y)));
  }
  const bool past = m1 >= P.sm_edge;
  const float lead = (float)(past ? P.beta * l2 - P.a2 * l1 : P.beta * (l2 - l1));
  const float u = (float)((m1 - P.mu) * P.inv_sigma);
  const float al1 = (float)(P.alpha * l1);
  const float num = (float)P.pl_coef * __expf(lead - al1) + (float)P.tg_coef * __expf(lead - 0.5f * u * u);
  float c;
  if (past) {
    const float d = (float)(l1 - P.ln_edge), a2 = (float)P.a2;
    c = __expf((float)(P.sm_lnq - P.a2 * l1)) + (P.a2 == 0.0 ? d : -expm1f(-a2 * d) / a2);
  } else {
    const double pos = (m1 - P.mmin) / P.sm_h;
    const int k = (int)fmin(fmax(pos, 0.0), (double)(kMassPanels - 1));
    const double t = pos - (double)k;
    const double2 a = mt[k], b = mt[k + 1];
    const double dd = b.x - a.x, s0 = a.y * P.sm_h, s1 = b.y * P.sm_h;
    c = (float)(a.x + t * (s0 + t * ((3.0 * dd - 2.0 * s0 - s1) + t * (s0 + s1 - 2.0 * dd))));
  }
  if (!(num > 0.0f && c > 0.0f)) return -INFINITY;
  return __logf(num) - __logf(c) - sp + (float)P.sm_lnn1inv;
}

// p(m1) p(m2|m1) of the source-frame masses; 0 outside
// mmin <= m2 <= m1 <= mmax (and m1 > mmin).  l1, l2 = ln m1, ln m2.
// With a = 1 + beta the pairing term is p(m2|m1) = a m2^beta m1^-a /
// (1 - (mmin/m1)^a) (m2^-1 / ln(m1/mmin) at a = 0), so that
//   w = a [c_pl e^(beta l2 - (a + alpha) l1) + c_tg e^(beta l2 - a l1 - u^2/2)]
//       / (-expm1(a (ln mmin - l1)))
// with c_pl, c_tg the normalised power-law and peak coefficients of p(m1).
__device__ __forceinline__ double mass_weight64(const LamParams& P, double m1, double m2,
                                                double l1, double l2) {
  if (!(m1 >= P.mmin && m1 <= P.mmax && m2 >= P.mmin && m2 <= m1 && m1 > P.mmin)) return 0.0;
  const double lead = P.beta * l2 - P.a2 * l1;
  const double u = (m1 - P.mu) * P.inv_sigma;
  const double num = P.pl_coef * exp(lead - P.alpha * l1) + P.tg_coef * exp(lead - 0.5 * u * u);
  if (P.a2 == 0.0) return num / (l1 - P.ln_mmin);
  return P.a2 * num / -expm1(P.a2 * (P.ln_mmin - l1));
}

__device__ __forceinline__ float mass_weight32(const LamParams& P, double m1, double m2,
                                               double l1d, double l2d) {
  if (!(m1 >= P.mmin && m1 <= P.mmax && m2 >= P.mmin && m2 <= m1 && m1 > P.mmin)) return 0.0f;
  const float l1 = (float)l1d, l2 = (float)l2d;
  const float a2 = (float)P.a2;
  const float lead = (float)P.beta * l2 - a2 * l1;
  const float u = ((float)m1 - (float)P.mu) * (float)P.inv_sigma;
  const float num = (float)P.pl_coef * __expf(lead - (float)P.alpha * l1) +
                    (float)P.tg_coef * __expf(lead - 0.5f * u * u);
  if (P.a2 == 0.0) return num / (l1 - (float)P.ln_mmin);
  return a2 * num / -expm1f(a2 * ((float)P.ln_mmin - l1));
}

// SM: the point may carry the smoothed mass edge; LOGW (FP32, delta_m > 0):
// w is the weight's log from lnw_smoothed32
template <bool F32, bool SM, bool LOGW>
__device__ __forceinline__ void sample_zw(const LamParams& P, const double2* __restrict__ dtab,
                                          const double2* __restrict__ inv, const Geometry& g,
                                          double d, double lnd, double m1d, double m2d,
                                          double lnm1d, double lnm2d, double& z, double& w,
                                          const double2* __restrict__ mt) {
  double x = invert_x(P, nullptr, inv, g, d, lnd, 0);
  double zp1 = exp(x);
  if (!F32) {
    double D, Dx;
    dist_tab_at(dtab, g, x, D, Dx);
    const double dx = (D - d) / Dx;           // |dx| is at the inverse table's error
    x -= dx;
    zp1 *= 1.0 - dx + 0.5 * dx * dx;          // e^(x - dx)
  }
  z = zp1 - 1.0;
  const double r = 1.0 / zp1;
  const double m1 = m1d * r, m2 = m2d * r;
  const double l1 = lnm1d - x, l2 = lnm2d - x;
  if (LOGW) {
    w = (double)lnw_smoothed32(P, mt, m1, m2, l1, l2);
    return;
  }
  if (SM && P.dm > 0.0) {
    w = mass_weight_smoothed<F32>(P, mt, m1, m2, l1, l2);
    return;
  }
  w = F32 ? (double)mass_weight32(P, m1, m2, l1, l2) : mass_weight64(P, m1, m2, l1, l2);
}

// Madau-Dickinson psi at x = ln(1+z).
__device__ __forceinline__ double psi_of_x(const LamParams& P, double x) {
  return exp(P.gamma * x) / (1.0 + exp((P.gamma + P.kappa) * (x - P.ln1zp)));
}

}  // namespace chimera
