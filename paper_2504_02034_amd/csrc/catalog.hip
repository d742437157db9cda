// Catalogue density on the redshift grid, built on the device (the galaxy
// term p_cat of eq. like-integrals discretised on the grid, once per
// catalogue: Sect. 2.3 computes it before the inference).
//
// Each galaxy's redshift density N(z; z_obs, sigma), truncated to
// |z - z_obs| <= 8 sigma, is projected on the grid's hat basis,
//   J_k = int N(z) Lambda_k(z) dz     (half hats at the two ends),
// weighted by the comoving volume element at the node (a shape V_k given by
// the caller) and normalised per galaxy so that sum_k tau_k q_k = 1 with
// q_k = J_k V_k / tau_k.  Then, over the galaxies with a nonzero projection
// (n_used of them),
//   n_r(z_k) = sum_{gal in pixel r} q_k / (n_used * pixel area),
//   n_tot(z_k) = sum_{all galaxies} q_k / n_used.
//
// k_gal_norm       one thread per galaxy: sum_k J_k V_k
// k_pixel_rows     one workgroup per pixel, node-major (a thread per grid
//                  node sums the pixel's galaxies in their stored order), so
//                  every sum has a fixed order
// k_catalog_finish n_tot by fixed-order column sums; the rows of the pixels
//                  the events use, in FP64 and FP32
#include <math.h>

#include <algorithm>

#include "common.h"
#include "launch.h"

namespace chimera {

namespace {

constexpr double kSupport = 8.0;          // sigmas kept of each galaxy's Gaussian
constexpr double kInvSqrt2 = 0.70710678118654752440;

__device__ __forceinline__ double phi_diff(double al, double be) {
  // Phi(be) - Phi(al), al <= be, from the tail that does not cancel
  return al >= 0.0 ? 0.5 * (erfc(al * kInvSqrt2) - erfc(be * kInvSqrt2))
                   : 0.5 * (erfc(-be * kInvSqrt2) - erfc(-al * kInvSqrt2));
}

// int_a^b N(z; mu, s) sign (z - c) / dz dz over [a, b] clipped to the support
__device__ __forceinline__ double hat_segment(double a, double b, double c, double sign, double mu,
                                              double s, double dz) {
  const double a2 = fmax(a, mu - kSupport * s), b2 = fmin(b, mu + kSupport * s);
  if (!(b2 > a2)) return 0.0;
  const double al = (a2 - mu) / s, be = (b2 - mu) / s;
  const double cdf = phi_diff(al, be);
  const double pdf = (exp(-0.5 * al * al) - exp(-0.5 * be * be)) * kInvSqrt2Pi;
  return sign * (s * pdf + (mu - c) * cdf) / dz;
}

// J_k of one galaxy at node k
__device__ __forceinline__ double hat_node(int k, double mu, double s, const CatalogGrid& g) {
  const double zk = g.z_lo + (double)k * g.dz;
  const double lo = k > 0 ? zk - g.dz : zk;
  const double hi = k < g.n_z - 1 ? zk + g.dz : zk;
  const double rise = hat_segment(lo, zk, lo, 1.0, mu, s, g.dz);
  const double fall = hat_segment(zk, hi, hi, -1.0, mu, s, g.dz);
  return fmax(rise + fall, 0.0);
}

// nodes a galaxy can touch: [k_first, k_last] within the grid; empty when
// k_first > k_last
__device__ __forceinline__ void galaxy_nodes(double mu, double s, const CatalogGrid& g, int& k0,
                                             int& k1) {
  k0 = 1;
  k1 = 0;
  if (!(s > 0.0) || !(mu + kSupport * s >= g.z_lo) || !(mu - kSupport * s <= g.z_hi)) return;
  const double a = floor((mu - kSupport * s - g.z_lo) / g.dz) - 1.0;
  const double b = ceil((mu + kSupport * s - g.z_lo) / g.dz) + 1.0;
  k0 = (int)fmax(a, 0.0);
  k1 = (int)fmin(b, (double)(g.n_z - 1));
}

}  // namespace

__global__ void k_gal_norm(const double* __restrict__ mu, const double* __restrict__ sig,
                           long long n_gal, CatalogGrid g, const double* __restrict__ vshape,
                           double* __restrict__ norm) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_gal) return;
  const double m = mu[i], s = sig[i];
  int k0, k1;
  galaxy_nodes(m, s, g, k0, k1);
  double t = 0.0;
  for (int k = k0; k <= k1; ++k) t += hat_node(k, m, s, g) * vshape[k];
  norm[i] = t;
}

constexpr int kCatBS = 256;

// rows_all[p][k] = sum_{gal in p, norm > 0} J_k V_k / (tau_k norm)
__global__ __launch_bounds__(kCatBS) void k_pixel_rows(const long long* __restrict__ off,
                                                       const double* __restrict__ mu,
                                                       const double* __restrict__ sig,
                                                       const double* __restrict__ norm,
                                                       CatalogGrid g,
                                                       const double* __restrict__ vshape,
                                                       long long n_pix,
                                                       double* __restrict__ rows_all) {
  for (long long p = blockIdx.x; p < n_pix; p += gridDim.x) {
    const long long a = off[p], b = off[p + 1];
    double* row = rows_all + p * g.n_z;
    for (int k = threadIdx.x; k < g.n_z; k += kCatBS) {
      const double zk = g.z_lo + (double)k * g.dz;
      const double tau = (k == 0 || k == g.n_z - 1) ? 0.5 * g.dz : g.dz;
      double acc = 0.0;
      for (long long i = a; i < b; ++i) {
        const double m = mu[i], s = sig[i], nm = norm[i];
        if (!(nm > 0.0)) continue;
        // a galaxy touches the nodes within 8 sigma and one grid step of z_obs
        if (fabs(zk - m) > kSupport * s + 2.0 * g.dz) continue;
        acc += hat_node(k, m, s, g) * vshape[k] / (tau * nm);
      }
      row[k] = acc;
    }
  }
}

// n_tot and the used rows
__global__ void k_catalog_finish(const double* __restrict__ rows_all, long long n_pix,
                                 CatalogGrid g, const long long* __restrict__ rows_pix,
                                 long long n_rows, double inv_used, double inv_used_area,
                                 double* __restrict__ ntot, double* __restrict__ nz64,
                                 float* __restrict__ nz32) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < g.n_z) {
    double t = 0.0;
    for (long long p = 0; p < n_pix; ++p) t += rows_all[p * g.n_z + id];
    ntot[id] = t * inv_used;
  }
  if (id < n_rows * g.n_z) {
    const long long r = id / g.n_z, k = id % g.n_z;
    const double v = rows_all[rows_pix[r] * g.n_z + k] * inv_used_area;
    nz64[id] = v;
    nz32[id] = (float)v;
  }
}

hipError_t launch_catalog(const CatalogArgs& c, hipStream_t st) {
  if (c.n_gal > 0) {
    k_gal_norm<<<(unsigned)((c.n_gal + 255) / 256), 256, 0, st>>>(c.mu, c.sig, c.n_gal, c.g,
                                                                   c.vshape, c.norm);
    CH_LAUNCH_CHECK();
  }
  const long long blocks = c.n_pix < 65536 ? c.n_pix : 65536;
  if (blocks > 0) {
    k_pixel_rows<<<(unsigned)blocks, kCatBS, 0, st>>>(c.off, c.mu, c.sig, c.norm, c.g, c.vshape,
                                                      c.n_pix, c.rows_all);
    CH_LAUNCH_CHECK();
  }
  return hipSuccess;
}

hipError_t launch_catalog_finish(const CatalogArgs& c, long long n_used, hipStream_t st) {
  const long long n = std::max<long long>((long long)c.g.n_z, c.n_rows * c.g.n_z);
  const double inv_used = n_used > 0 ? 1.0 / (double)n_used : 0.0;
  k_catalog_finish<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
      c.rows_all, c.n_pix, c.g, c.rows_pix, c.n_rows, inv_used, inv_used / c.pixel_area, c.ntot,
      c.nz64, c.nz32);
  CH_LAUNCH_CHECK();
  return hipSuccess;
}

// Rows of a single-1D event set (eq. gw-kernel-single1d): the pixels' sky
// factors folded into one row per event, out[e][k] = sum_{p of e} s_p n_{row_p}(z_k),
// summed in the pixels' given order (and the same fold of 1 - P_compl when
// the catalogue is incomplete); a thread per (event, node).
__global__ void k_fold_rows(const int* __restrict__ pix_off, const int* __restrict__ row,
                            const double* __restrict__ s, long long n_ev, int n_z,
                            const double* __restrict__ nz64, double* __restrict__ out64,
                            float* __restrict__ out32, const double* __restrict__ mz64,
                            double* __restrict__ mout64, float* __restrict__ mout32) {
  const long long n = n_ev * n_z;
  for (long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x; id < n;
       id += (long long)gridDim.x * blockDim.x) {
    const long long e = id / n_z;
    const int k = (int)(id - e * n_z);
    double acc = 0.0, macc = 0.0;
    for (int p = pix_off[e]; p < pix_off[e + 1]; ++p) {
      acc += s[p] * nz64[(long long)row[p] * n_z + k];
      if (mz64) macc += s[p] * mz64[(long long)row[p] * n_z + k];
    }
    out64[id] = acc;
    out32[id] = (float)acc;
    if (mz64) {
      mout64[id] = macc;
      mout32[id] = (float)macc;
    }
  }
}

hipError_t launch_fold_rows(const FoldArgs& f, hipStream_t st) {
  const long long n = (long long)f.n_ev * f.n_z;
  if (n == 0) return hipSuccess;
  const long long blocks = std::min<long long>((n + 255) / 256, 1 << 16);
  k_fold_rows<<<(unsigned)blocks, 256, 0, st>>>(f.pix_off, f.row, f.s, f.n_ev, f.n_z, f.nz64,
                                                f.out64, f.out32, f.mz64, f.mout64, f.mout32);
  CH_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace chimera
