// HIP kernels (gfx950, wave64) of the many-1D standard-siren likelihood.
//
//   k_lam_prepare     per-lambda constants and domain checks (Table 1 layout)
//   k_mass_table      the smoothed lower mass edge's normalisations (Table 1's delta_m)
//   k_chi_table       chi(x) = int dz/E on x = ln(1+z) nodes, FP64 (eq. dL-em)
//   k_inverse_table   x(ln d) with d_L^gw(x) = d (eqs. dL-em, dL-mg)
//   k_grid_factor     tau_g psi(z_g) / [(1+z_g)^3 d d_L^gw/dz]   (eq. jacobian)
//   k_chi_om_table    dchi/dOm on the same nodes (gradient only)
//   (the per-(event, lambda) kernel sums are in event.hip, the adjoint in grad.hip)
//   k_selection       injection sums of s_j and s_j^2 (Sect. 2.2)
//   k_*_final         fixed-order reductions to ln xi, N_eff, ln L (eq. hyperlike)
//
// Every reduction runs in a fixed order that depends only on the launch
// shape, so each lambda's result is bitwise independent of the other points
// in its batch.
#include <math.h>

#include "common.h"
#include "launch.h"
#include "reduce.h"

namespace chimera {

// ---------------------------------------------------------------------------
// per-lambda constants
// ---------------------------------------------------------------------------
__device__ double ndtr_diff(double a, double b) {
  // Phi(b) - Phi(a), from the tail that does not cancel
  const double r = 0.70710678118654752440;
  return a > 0.0 ? 0.5 * (erfc(a * r) - erfc(b * r)) : 0.5 * (erfc(-b * r) - erfc(-a * r));
}

__global__ void k_lam_prepare(const double* __restrict__ lam, int stride, int B,
                              LamParams* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const double* l = lam + (size_t)b * stride;
  LamParams P;
  P.h0 = l[0]; P.om = l[1]; P.xi0 = l[2]; P.n = l[3]; P.alpha = l[4]; P.beta = l[5];
  P.mmin = l[6]; P.mmax = l[7]; P.mu = l[8]; P.sigma = l[9]; P.lg = l[10];
  P.gamma = l[11]; P.kappa = l[12]; P.zp = l[13];
  bool ok = true;
  for (int i = 0; i < kNlam; ++i) ok = ok && isfinite(l[i]);
  ok = ok && P.h0 > 0.0 && P.om > 0.0 && P.om <= 1.0 && P.xi0 > 0.0 && P.mmin > 0.0 &&
       P.mmax > P.mmin && P.sigma > 0.0 && P.lg >= 0.0 && P.lg <= 1.0 && P.zp > -1.0;
  P.flag = 0;
  P.pad = 0;
  P.dh = kCkms / P.h0;
  P.ln_mmin = log(P.mmin);
  P.ln_mmax = log(P.mmax);
  P.inv_sigma = 1.0 / P.sigma;
  P.ln1zp = log1p(P.zp);
  // int_mmin^mmax m^-alpha dm, stable for alpha -> 1
  const double a1 = 1.0 - P.alpha;
  const double lr = P.ln_mmax - P.ln_mmin;
  const double npl = (a1 == 0.0) ? lr : exp(a1 * P.ln_mmin) * expm1(a1 * lr) / a1;
  P.pl_coef = (1.0 - P.lg) / npl;
  const double zg = ndtr_diff((P.mmin - P.mu) / P.sigma, (P.mmax - P.mu) / P.sigma);
  ok = ok && zg > 0.0;
  P.tg_coef = P.lg / (P.sigma * 2.50662827463100050242 * zg);
  P.a2 = 1.0 + P.beta;
  P.mmin_a2 = exp(P.a2 * P.ln_mmin);
  // the smoothed lower edge (its constants come from k_mass_table)
  P.dm = stride > kNlam ? l[kNlam] : 0.0;
  ok = ok && isfinite(P.dm) && P.dm >= 0.0;
  P.sm_n1inv = 1.0; P.sm_q = 0.0; P.sm_h = 0.0;
  P.sm_top = fmin(P.mmax, P.mmin + P.dm);
  P.sm_edge = P.mmin + P.dm;
  P.ln_edge = log(P.sm_edge);
  P.sm_pl = P.a2 == 0.0 ? 1.0 : exp(P.a2 * P.ln_edge) / P.a2;
  if (!ok) P.flag = kFlagDomain;
  out[b] = P;
}

// ---------------------------------------------------------------------------
// smoothed-edge constants: one workgroup per lambda.  With f(m) = m^beta S(m)
// and C(m) = int_mmin^m f, the table holds R = C / f and dR/dm = 1 - R g'
// (g' = d ln f/dm) on kMassPanels + 1 equal nodes of [mmin, top],
// top = min(mmax, mmin + delta_m).  R stays smooth and representable where
// C and f underflow near mmin, so the weights keep their relative accuracy
// there.  Across a panel R(b) = R(a) f(a)/f(b) + int_a^b f/f(b): pass 1 (one
// panel per thread in turn, so the steep panels near mmin spread over the
// block) forms each panel's affine map with 8-point Gauss-Legendre on
// sub-panels sized to the steepness; pass 2 scans the maps in order.  It also
// gives Q = C(top) and N1 = int_mmin^top p(m1) S + int_top^mmax p(m1).
// ---------------------------------------------------------------------------
constexpr int kMassBS = 1024;

// 8-point Gauss-Legendre on [-1, 1]: the positive nodes and their weights
__constant__ double kGLx[4] = {0.18343464249564980494, 0.52553240991632898582,
                               0.79666647741362673959, 0.96028985649753623168};
__constant__ double kGLw[4] = {0.36268378337836198297, 0.31370664587788728734,
                               0.22238103445337447054, 0.10122853629037625915};

// y = dm/m' + dm/(m' - dm) of S = 1 / (1 + e^y), for 0 < m' < dm
__device__ __forceinline__ double smooth_exponent(double mp, double dm) {
  return dm * (2.0 * mp - dm) / (mp * (mp - dm));
}

// ln S(m) for 0 < m' = m - mmin < delta_m: -softplus(y)
__device__ __forceinline__ double ln_smooth(double mp, double dm) {
  const double y = smooth_exponent(mp, dm);
  return -(fmax(y, 0.0) + log1p(exp(-fabs(y))));
}

// ln f(m) = beta ln m + ln S(m), for m > mmin
__device__ __forceinline__ double ln_fm(const LamParams& P, double m) {
  const double mp = m - P.mmin;
  return P.beta * log(m) + (mp >= P.dm ? 0.0 : ln_smooth(mp, P.dm));
}

// g'(m) = d ln f/dm = beta/m + (1 - S) (dm/m'^2 + dm/(m' - dm)^2), for m > mmin
__device__ __forceinline__ double dln_fm(const LamParams& P, double m) {
  const double mp = m - P.mmin;
  if (mp >= P.dm) return P.beta / m;
  const double y = smooth_exponent(mp, P.dm);
  const double oms = 1.0 / (1.0 + exp(-y));
  const double q = mp - P.dm;
  return P.beta / m + (oms > 0.0 ? oms * (P.dm / (mp * mp) + P.dm / (q * q)) : 0.0);
}

__global__ __launch_bounds__(kMassBS) void k_mass_table(LamParams* __restrict__ Pv,
                                                        double2* __restrict__ mtab) {
  const int b = blockIdx.x;
  LamParams P = Pv[b];
  if (!(P.dm > 0.0) || P.flag) return;
  double2* tab = mtab + (size_t)b * (kMassPanels + 1);
  const double h = (P.sm_top - P.mmin) / (double)kMassPanels;
  const double* gx = kGLx;
  const double* gw = kGLw;
  auto node = [&](int k) { return k == kMassPanels ? P.sm_top : P.mmin + (double)k * h; };
  // the unsmoothed mixture p(m1) at m, ln m given
  auto mix = [&](double m, double lm) {
    const double u = (m - P.mu) * P.inv_sigma;
    return P.pl_coef * exp(-P.alpha * lm) + P.tg_coef * exp(-0.5 * u * u);
  };
  // pass 1: tab[k + 1] = (f(a)/f(b), int_a^b f/f(b)) of panel k = [a, b];
  // and the smoothed primary's mass below top
  double n1 = 0.0;
  for (int k = threadIdx.x; k < kMassPanels; k += kMassBS) {
    const double a = node(k), e = node(k + 1);
    const double lsb = e - P.mmin >= P.dm ? 0.0 : ln_smooth(e - P.mmin, P.dm);
    const double lb = P.beta * log(e) + lsb;
    const double ratio = k == 0 ? 0.0 : exp(ln_fm(P, a) - lb);
    // sub-panels resolve f's steep rise near mmin.  Where S(b) < 1e-100 no
    // weight that matters can use the node, and the recursion's factor
    // f(a)/f(b) < e^-14 there forgets the error within a panel or two, so
    // two sub-panels do.
    const double steep = k == 0 ? 1e300 : dln_fm(P, a) * (e - a);
    const double cap = lsb < -230.0 ? 2.0 : 32.0;
    const int nsub = (int)fmin(fmax(ceil(steep * 0.25), 1.0), cap);
    const double mid = 0.5 * (a + e), hp = 0.5 * (e - a);
    double acc = 0.0, sp = 0.0;
    if (nsub == 1) {
      // one set of nodes serves both integrals
#pragma unroll 2
      for (int q = 0; q < 8; ++q) {
        const double x = mid + (q & 1 ? hp : -hp) * gx[q >> 1];
        const double lx = log(x), mp = x - P.mmin;
        double ls = 0.0, sv = 1.0;
        if (mp < P.dm) {
          const double y = smooth_exponent(mp, P.dm);
          const double ex = exp(-fabs(y));
          ls = -(fmax(y, 0.0) + log1p(ex));
          sv = (y >= 0.0 ? ex : 1.0) / (1.0 + ex);
        }
        acc += gw[q >> 1] * exp(P.beta * lx + ls - lb);
        sp += gw[q >> 1] * mix(x, lx) * sv;
      }
      acc *= hp;
      sp *= hp;
    } else {
      const double w = (e - a) / (double)nsub, half = 0.5 * w;
      for (int j = 0; j < nsub; ++j) {
        const double mj = a + ((double)j + 0.5) * w;
        double sj = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          sj += gw[q] * (exp(ln_fm(P, mj - half * gx[q]) - lb) + exp(ln_fm(P, mj + half * gx[q]) - lb));
        acc += sj * half;
      }
#pragma unroll 2
      for (int q = 0; q < 8; ++q) {
        const double x = mid + (q & 1 ? hp : -hp) * gx[q >> 1];
        sp += gw[q >> 1] * mix(x, log(x)) * smooth_edge(x, P.mmin, P.dm);
      }
      sp *= hp;
    }
    tab[k + 1] = make_double2(ratio, acc);
    n1 += sp;
  }
  __syncthreads();
  // pass 2: compose the maps of this thread's panels, in order
  constexpr int per = kMassPanels / kMassBS;
  const int k0 = threadIdx.x * per;
  double A = 1.0, Bv = 0.0;          // R_end = A R_start + Bv
#pragma unroll
  for (int i = 0; i < per; ++i) {
    const double2 m = tab[k0 + i + 1];
    A *= m.x;
    Bv = m.x * Bv + m.y;
  }
  // inclusive scan of the maps (earlier threads first), then this thread's start
  constexpr int NW = kMassBS / 64;
  __shared__ double sA[NW], sB[NW], sN[NW];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double iA = A, iB = Bv;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double pA = __shfl_up(iA, o, 64), pB = __shfl_up(iB, o, 64);
    if (lane >= o) {
      iB = iA * pB + iB;
      iA = iA * pA;
    }
  }
  const double n1w = wave_sum(n1);
  if (lane == 63) { sA[wv] = iA; sB[wv] = iB; }
  if (lane == 0) sN[wv] = n1w;
  __syncthreads();
  // R at this thread's first node: the scan of all earlier maps applied to R(mmin) = 0
  double r0 = 0.0;
  for (int i = 0; i < wv; ++i) r0 = sA[i] * r0 + sB[i];
  const double eB = __shfl_up(iB, 1, 64), eA = __shfl_up(iA, 1, 64);
  if (lane > 0) r0 = eA * r0 + eB;
  double r = r0;
  if (threadIdx.x == 0) tab[0] = make_double2(0.0, 0.0);
#pragma unroll
  for (int i = 0; i < per; ++i) {
    const double2 m = tab[k0 + i + 1];
    r = m.x * r + m.y;
    const int k = k0 + i + 1;
    tab[k] = make_double2(r, 1.0 - r * dln_fm(P, node(k)));
  }
  if (threadIdx.x == kMassBS - 1) {
    double nb = 0.0;
    for (int i = 0; i < NW; ++i) nb += sN[i];
    // the unsmoothed mixture's mass on [top, mmax] in closed form
    double tail = 0.0;
    if (P.sm_top < P.mmax) {
      const double a1 = 1.0 - P.alpha, lt = log(P.sm_top), lr = P.ln_mmax - lt;
      const double pl = a1 == 0.0 ? lr : exp(a1 * lt) * expm1(a1 * lr) / a1;
      const double z = ndtr_diff((P.mmin - P.mu) / P.sigma, (P.mmax - P.mu) / P.sigma);
      tail = P.pl_coef * pl +
             P.lg * ndtr_diff((P.sm_top - P.mu) / P.sigma, (P.mmax - P.mu) / P.sigma) / z;
    }
    const double n1v = nb + tail;
    P.sm_h = h;
    P.sm_q = r * exp(ln_fm(P, P.sm_top));
    P.sm_n1inv = 1.0 / n1v;
    P.sm_lnq = log(P.sm_q);
    P.sm_lnn1inv = -log(n1v);
    if (!(P.sm_q > 0.0) || !(n1v > 0.0) || !isfinite(P.sm_q)) P.flag = kFlagDomain;
    Pv[b] = P;
  }
}

// ---------------------------------------------------------------------------
// chi table: one workgroup per lambda, block-wide scan of Gauss-Legendre
// panel integrals of dchi/dx = e^x / E(e^x).
// ---------------------------------------------------------------------------
constexpr int kTabBS = 1024;

__device__ __forceinline__ double dchi_dx(double om, double x) {
  const double zp1 = exp(x);
  return zp1 / efunc_of_zp1(om, zp1);
}

// d/dx of dchi/dOm = -1/2 int ((1+z)^3 - 1) / E^3 dz, in x = ln(1+z)
__device__ __forceinline__ double dchiom_dx(double om, double x) {
  const double zp1 = exp(x);
  const double e = efunc_of_zp1(om, zp1);
  return -0.5 * zp1 * (zp1 * zp1 * zp1 - 1.0) / (e * e * e);
}

// KIND 0: chi and the monotonicity flag of d_L^gw; KIND 1: dchi/dOm.
template <int KIND>
__global__ __launch_bounds__(kTabBS) void k_x_table(const LamParams* __restrict__ Pv, Geometry g,
                                                    double2* __restrict__ chi,
                                                    int* __restrict__ flag_mono) {
  auto fx = [](double om, double x) { return KIND == 0 ? dchi_dx(om, x) : dchiom_dx(om, x); };
  const int b = blockIdx.x;
  const LamParams P = Pv[b];
  double2* tab = chi + (size_t)b * g.n_t;
  __shared__ double wsum[kTabBS / 64 + 1];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  const int nint = g.n_t - 1;
  const int per = (nint + kTabBS - 1) / kTabBS;
  const int k0 = threadIdx.x * per;
  // 8-point Gauss-Legendre on [-1, 1]
  const double gx[4] = {0.18343464249564980494, 0.52553240991632898582, 0.79666647741362673959,
                        0.96028985649753623168};
  const double gw[4] = {0.36268378337836198297, 0.31370664587788728734, 0.22238103445337447054,
                        0.10122853629037625915};
  double local[16];
  double run = 0.0;
  for (int i = 0; i < per; ++i) {
    const int k = k0 + i;
    double s = 0.0;
    if (k < nint) {
      const double mid = ((double)k + 0.5) * g.dx, half = 0.5 * g.dx;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        s += gw[q] * (fx(P.om, mid - half * gx[q]) + fx(P.om, mid + half * gx[q]));
      s *= half;
    }
    run += s;
    if (i < 16) local[i] = run;
  }
  // exclusive scan of the per-thread totals (wave scan, then wave offsets)
  double incl = run;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int i = 0; i < kTabBS / 64; ++i) {
      const double t = wsum[i];
      wsum[i] = acc;
      acc += t;
    }
  }
  __syncthreads();
  const double base = wsum[w] + incl - run;
  if (threadIdx.x == 0) tab[0] = make_double2(0.0, fx(P.om, 0.0));
  int mybad = 0;
  for (int i = 0; i < per && i < 16; ++i) {
    const int k = k0 + i + 1;   // node index
    if (k <= nint) {
      const double x = (double)k * g.dx;
      const double c = base + local[i];
      const double cp = fx(P.om, x);
      tab[k] = make_double2(c, cp);
      if (KIND == 0) {
        const double en = exp(-P.n * x);
        const double xi = P.xi0 + (1.0 - P.xi0) * en;
        const double dd = c * xi + cp * xi - c * P.n * (1.0 - P.xi0) * en;
        if (!(dd > 0.0)) mybad = 1;
      }
    }
  }
  if (KIND == 0) {
    if (mybad) atomicOr(&bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) flag_mono[b] = bad ? kFlagNonMonotone : 0;
  }
}

// ---------------------------------------------------------------------------
// inverse table: x(u_m), u = ln d, and dx/du, one thread per (lambda, node)
// ---------------------------------------------------------------------------
__global__ void k_inverse_table(const LamParams* __restrict__ Pv, const double2* __restrict__ chi,
                                Geometry g, int B, double2* __restrict__ inv,
                                int* __restrict__ flag_range) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)B * g.n_u) return;
  const int b = (int)(id / g.n_u), m = (int)(id % g.n_u);
  const LamParams P = Pv[b];
  const double2* tab = chi + (size_t)b * g.n_t;
  const double d = exp(g.u_lo + (double)m * g.du);
  auto dnode = [&](int k) {
    const double x = (double)k * g.dx;
    return P.dh * exp(x) * tab[k].x * (P.xi0 + (1.0 - P.xi0) * exp(-P.n * x));
  };
  int lo = 0, hi = g.n_t - 1;
  const double dmax = dnode(hi);
  if (!(dmax >= d)) {   // beyond the table (or not finite)
    inv[id] = make_double2((double)hi * g.dx, 0.0);
    if (m == g.n_u - 1) flag_range[b] = kFlagRange;
    return;
  }
  if (m == g.n_u - 1) flag_range[b] = 0;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (dnode(mid) <= d) lo = mid; else hi = mid;
  }
  double xl = (double)lo * g.dx, xh = (double)hi * g.dx;
  const double dl0 = dnode(lo), dh0 = dnode(hi);
  double x = xl + (d - dl0) / (dh0 - dl0) * (xh - xl);
  double D = d, Dx = 1.0;
  for (int it = 0; it < 12; ++it) {
    dist_at(P, tab, g, x, exp(x), D, Dx);
    const double f = D - d;
    if (f < 0.0) xl = fmax(xl, x); else xh = fmin(xh, x);
    double xn = x - f / Dx;
    if (!(xn >= xl && xn <= xh)) xn = 0.5 * (xl + xh);
    if (xn == x) break;
    x = xn;
  }
  dist_at(P, tab, g, x, exp(x), D, Dx);
  inv[id] = make_double2(x, D / Dx);
}

// ---------------------------------------------------------------------------
// d_L^gw and dd_L^gw/dx on the nodes x_k = k dx (Hermite data for the Newton
// step of the sample transform)
// ---------------------------------------------------------------------------
__global__ void k_dist_table(const LamParams* __restrict__ Pv, const double2* __restrict__ chi,
                             Geometry g, int B, double2* __restrict__ dtab) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)B * g.n_t) return;
  const int b = (int)(id / g.n_t), k = (int)(id % g.n_t);
  const LamParams P = Pv[b];
  const double x = (double)k * g.dx;
  double D, Dx;
  dist_at(P, chi + (size_t)b * g.n_t, g, x, exp(x), D, Dx);
  dtab[id] = make_double2(D, Dx);
}

// ---------------------------------------------------------------------------
// grid factor tau_g psi / [(1+z)^3 D'(z)]  =  tau_g psi / [(1+z)^2 dD/dx]
// ---------------------------------------------------------------------------
__global__ void k_grid_factor(const LamParams* __restrict__ Pv, const double2* __restrict__ chi,
                              Geometry g, int B, double* __restrict__ gz64,
                              float* __restrict__ gz32) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)B * g.n_z) return;
  const int b = (int)(id / g.n_z), k = (int)(id % g.n_z);
  const LamParams P = Pv[b];
  const double z = g.z_lo + (double)k * g.dz;
  const double x = log1p(z);
  double D, Dx;
  dist_at(P, chi + (size_t)b * g.n_t, g, x, 1.0 + z, D, Dx);
  const double tau = (k == 0 || k == g.n_z - 1) ? 0.5 * g.dz : g.dz;
  const double zp1 = 1.0 + z;
  double v = tau * psi_of_x(P, x) / (zp1 * zp1 * Dx);
  if (!isfinite(v)) v = 0.0;
  gz64[id] = v;
  gz32[id] = (float)v;
}

// ---------------------------------------------------------------------------
// incompleteness: the homogeneous completion of eq. p-miss per lambda
// ---------------------------------------------------------------------------
constexpr int kCompBS = 256;
__global__ __launch_bounds__(kCompBS) void k_completion(const LamParams* __restrict__ Pv,
                                                        const double2* __restrict__ chi, Geometry g,
                                                        const double* __restrict__ ntot,
                                                        const double* __restrict__ missing,
                                                        double* __restrict__ ntot_eff,
                                                        double* __restrict__ gz64,
                                                        float* __restrict__ gz32,
                                                        double* __restrict__ gzb64,
                                                        float* __restrict__ gzb32) {
  const int b = blockIdx.x;
  __shared__ double red[kCompBS / 64 + 1];
  const LamParams P = Pv[b];
  const double2* tab = chi + (size_t)b * g.n_t;
  const double zmax = g.z_lo + (double)(g.n_z - 1) * g.dz;
  const double cm = chi_at(tab, g, log1p(zmax));
  const double norm = 1.0 / (4.0 * M_PI / 3.0 * cm * cm * cm);
  auto vol = [&](int k) {
    const double z = g.z_lo + (double)k * g.dz;
    const double c = chi_at(tab, g, log1p(z));
    return c * c / efunc_of_zp1(P.om, 1.0 + z) * norm;
  };
  double t = 0.0;
  for (int k = threadIdx.x; k < g.n_z; k += kCompBS) {
    const double tau = (k == 0 || k == g.n_z - 1) ? 0.5 * g.dz : g.dz;
    t += tau * (4.0 * M_PI - missing[k]) * vol(k);
  }
  const double fR = block_sum<kCompBS>(t, red);
  for (int k = threadIdx.x; k < g.n_z; k += kCompBS) {
    const double v = vol(k);
    const size_t i = (size_t)b * g.n_z + k;
    ntot_eff[i] = fR * ntot[k] + missing[k] * v;
    if (gz64) {
      const double gv = gz64[i];
      gz64[i] = fR * gv;
      gz32[i] = (float)(fR * gv);
      gzb64[i] = v * gv;
      gzb32[i] = (float)(v * gv);
    }
  }
}

hipError_t launch_completion(const LamParams* P, const double2* chi, const Geometry& g, int B,
                             const double* ntot, const double* missing, double* ntot_eff,
                             double* gz64, float* gz32, double* gzb64, float* gzb32,
                             hipStream_t st) {
  k_completion<<<B, kCompBS, 0, st>>>(P, chi, g, ntot, missing, ntot_eff, gz64, gz32, gzb64,
                                       gzb32);
  CH_LAUNCH_CHECK();
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// selection: partial sums of s_j and s_j^2 per (injection chunk, lambda)
// ---------------------------------------------------------------------------
constexpr int kSelBS = 256;
constexpr int kSelPer = 4;

// SM: the batch may carry the smoothed mass edge (a separate kernel keeps
// the plain one's registers)
template <bool F32, bool SM>
__device__ __forceinline__ void selection_sums(const SelArgs& a) {
  const int chunk = blockIdx.x, b = blockIdx.y;
  __shared__ double red[kSelBS / 64 + 1];
  const LamParams P = a.P[b];
  const int flag = P.flag | a.flag_mono[b] | a.flag_range[b];
  if (flag) {
    if (threadIdx.x == 0) {
      a.partial[((size_t)b * a.nchunk + chunk) * 2] = 0.0;
      a.partial[((size_t)b * a.nchunk + chunk) * 2 + 1] = 0.0;
    }
    return;
  }
  const double2* chi = a.chi + (size_t)b * a.g.n_t;
  const double2* inv = a.inv + (size_t)b * a.g.n_u;
  double s1 = 0.0, s2 = 0.0;
  for (int k = 0; k < kSelPer; ++k) {
    const long long j = (long long)chunk * kSelBS * kSelPer + k * kSelBS + threadIdx.x;
    if (j >= a.n_det) break;
    const double x = invert_x(P, chi, inv, a.g, a.dl[j], a.lndl[j], F32 ? 0 : 1);
    const double zp1 = exp(x);
    const double z = expm1(x);
    const double m1 = a.m1d[j] / zp1, m2 = a.m2d[j] / zp1;
    const double l1 = a.lnm1d[j] - x, l2 = a.lnm2d[j] - x;
    double w;
    if (SM && P.dm > 0.0) {
      w = mass_weight_smoothed<F32>(P, a.mtab + (size_t)b * (kMassPanels + 1), m1, m2, l1, l2);
    } else {
      w = F32 ? (double)mass_weight32(P, m1, m2, l1, l2) : mass_weight64(P, m1, m2, l1, l2);
    }
    if (w == 0.0) continue;
    // n_tot(z) by linear interpolation on the grid, 0 outside
    const double* ntot = a.ntot + (size_t)b * a.ntot_stride;
    const double pos = (z - a.g.z_lo) / a.g.dz;
    double nt = 0.0;
    if (pos >= 0.0 && pos <= (double)(a.g.n_z - 1)) {
      int kk = (int)pos;
      if (kk >= a.g.n_z - 1) {
        nt = ntot[a.g.n_z - 1];
      } else {
        const double t = pos - (double)kk;
        nt = ntot[kk] + t * (ntot[kk + 1] - ntot[kk]);
      }
    }
    if (nt == 0.0) continue;
    double D, Dx;
    dist_at(P, chi, a.g, x, zp1, D, Dx);
    const double s = w * nt * psi_of_x(P, x) / (zp1 * zp1 * Dx * exp(a.ln_pdraw[j]));
    s1 += s;
    s2 += s * s;
  }
  s1 = block_sum<kSelBS>(s1, red);
  s2 = block_sum<kSelBS>(s2, red);
  if (threadIdx.x == 0) {
    a.partial[((size_t)b * a.nchunk + chunk) * 2] = s1;
    a.partial[((size_t)b * a.nchunk + chunk) * 2 + 1] = s2;
  }
}

// Without a register target the FP32 kernel keeps ~40 copies of per-lambda
// constants in VGPRs (130: 3 waves per SIMD); at 5 waves it rematerialises
// them without spilling (-8 %; the FP64 kernel is faster at its own 4).
__global__ __launch_bounds__(kSelBS) __attribute__((amdgpu_waves_per_eu(5)))
void k_selection32(SelArgs a) { selection_sums<true, false>(a); }

__global__ __launch_bounds__(kSelBS) void k_selection64(SelArgs a) {
  selection_sums<false, false>(a);
}

template <bool F32>
__global__ __launch_bounds__(kSelBS) __attribute__((amdgpu_waves_per_eu(4)))
void k_selection_sm(SelArgs a) { selection_sums<F32, true>(a); }

__global__ void k_selection_final(SelArgs a, double* __restrict__ ln_xi,
                                  double* __restrict__ neff) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.B) return;
  const int flag = a.P[b].flag | a.flag_mono[b] | a.flag_range[b];
  double s1 = 0.0, s2 = 0.0;
  for (int c = 0; c < a.nchunk; ++c) {
    s1 += a.partial[((size_t)b * a.nchunk + c) * 2];
    s2 += a.partial[((size_t)b * a.nchunk + c) * 2 + 1];
  }
  const double xi = s1 / (double)a.n_total;
  double lx = xi > 0.0 ? log(xi) : -INFINITY;
  double ne = neff_of(s1, s2, a.n_total);
  if (flag) {
    lx = NAN;
    ne = NAN;
  }
  ln_xi[b] = lx;
  if (neff) neff[b] = ne;
}

// ln L_b = sum_i ln I_ib - E ln xi_b
constexpr int kFinBS = 256;
__global__ __launch_bounds__(kFinBS) void k_lnl_final(const LamParams* __restrict__ Pv,
                                                      const int* __restrict__ flag_mono,
                                                      const int* __restrict__ flag_range,
                                                      const double* __restrict__ lnI,
                                                      const double* __restrict__ ln_xi,
                                                      const double* __restrict__ neff,
                                                      double neff_gate, int E,
                                                      double* __restrict__ lnl) {
  const int b = blockIdx.x;
  __shared__ double red[kFinBS / 64 + 1];
  double s = 0.0;
  for (int i = threadIdx.x; i < E; i += kFinBS) s += lnI[(size_t)b * E + i];
  s = block_sum<kFinBS>(s, red);
  if (threadIdx.x == 0) {
    const int flag = Pv[b].flag | flag_mono[b] | flag_range[b];
    const double lx = ln_xi[b];
    double v;
    // a point outside the domain or with a non-monotone distance is -inf even
    // if its tables also ran out of range; out of range alone is NaN
    if (flag & (kFlagDomain | kFlagNonMonotone)) v = -INFINITY;
    else if (flag) v = NAN;
    else if (isnan(s) || isnan(lx)) v = NAN;
    else if (s == -INFINITY || lx == -INFINITY) v = -INFINITY;
    else v = s - (double)E * lx;
    // the injection sum's stability check of Sect. 2.2: N_eff > gate x N_ev
    if (neff_gate > 0.0 && isfinite(v) && !(neff[b] > neff_gate * (double)E)) v = -INFINITY;
    lnl[b] = v;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_tables(const double* lam, int stride, int B, const Geometry& g, LamParams* P,
                         double2* mtab, double2* chi, double2* inv, double2* dtab, double* gz64,
                         float* gz32, int* flag_mono, int* flag_range, hipStream_t st) {
  k_lam_prepare<<<(B + 63) / 64, 64, 0, st>>>(lam, stride, B, P);
  CH_LAUNCH_CHECK();
  if (mtab) {
    k_mass_table<<<B, kMassBS, 0, st>>>(P, mtab);
    CH_LAUNCH_CHECK();
  }
  k_x_table<0><<<B, kTabBS, 0, st>>>(P, g, chi, flag_mono);
  CH_LAUNCH_CHECK();
  const long long ni = (long long)B * g.n_u;
  k_inverse_table<<<(unsigned)((ni + 255) / 256), 256, 0, st>>>(P, chi, g, B, inv, flag_range);
  CH_LAUNCH_CHECK();
  if (dtab) {
    const long long nt = (long long)B * g.n_t;
    k_dist_table<<<(unsigned)((nt + 255) / 256), 256, 0, st>>>(P, chi, g, B, dtab);
    CH_LAUNCH_CHECK();
  }
  if (gz64) {
    const long long ng = (long long)B * g.n_z;
    k_grid_factor<<<(unsigned)((ng + 255) / 256), 256, 0, st>>>(P, chi, g, B, gz64, gz32);
    CH_LAUNCH_CHECK();
  }
  return hipSuccess;
}

hipError_t launch_chi_om_table(const LamParams* P, int B, const Geometry& g, double2* chio,
                               hipStream_t st) {
  k_x_table<1><<<B, kTabBS, 0, st>>>(P, g, chio, nullptr);
  CH_LAUNCH_CHECK();
  return hipSuccess;
}

int selection_chunks(long long n_det) {
  const long long per = (long long)kSelBS * kSelPer;
  return (int)((n_det + per - 1) / per);
}

hipError_t launch_selection(const SelArgs& a, bool f32, double* ln_xi, double* neff,
                            hipStream_t st) {
  if (a.nchunk > 0) {
    dim3 grid(a.nchunk, a.B);
    if (a.mtab) {
      if (f32) k_selection_sm<true><<<grid, kSelBS, 0, st>>>(a);
      else k_selection_sm<false><<<grid, kSelBS, 0, st>>>(a);
    } else {
      if (f32) k_selection32<<<grid, kSelBS, 0, st>>>(a);
      else k_selection64<<<grid, kSelBS, 0, st>>>(a);
    }
    CH_LAUNCH_CHECK();
  }
  k_selection_final<<<(a.B + 63) / 64, 64, 0, st>>>(a, ln_xi, neff);
  CH_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_lnl_final(const LamParams* P, const int* flag_mono, const int* flag_range,
                            const double* lnI, const double* ln_xi, const double* neff,
                            double neff_gate, int E, int B, double* lnl, hipStream_t st) {
  k_lnl_final<<<B, kFinBS, 0, st>>>(P, flag_mono, flag_range, lnI, ln_xi, neff, neff_gate, E, lnl);
  CH_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace chimera
