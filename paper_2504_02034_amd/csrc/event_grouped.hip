// Per-(event, lambda) kernel sums of the many-1D likelihood (eqs.
// like-integrals and gw-kernel-many1d), gfx950.
//
// One workgroup handles one event at one lambda:
//   1. every thread owns up to GT sample groups (<= K consecutive samples of
//      one pixel, pre-sorted on the host by distance, groups ordered by
//      distance so a wave's lanes sit close in redshift at every lambda);
//      it maps them to (z_j, w_j), and the workgroup reduces the weighted
//      moments to the event's bandwidth h;
//   2. the redshift window the event's kernels touch is cut into slices;
//      for each slice, F_r(z_g) = n_r(z_g) g(z_g) of every pixel of the event
//      is staged in LDS (one coalesced pass over the catalogue rows);
//   3. each lane evaluates its group's K Gaussian sums by Horner's rule in
//      rho_k = exp(dz delta_k / h^2): with the group's centre c and
//      G_m = exp(-m^2 dz^2 / 2h^2),
//        sum_g F_g N(z_g; z_k, h) = C_k rho_k^(lo-c) sum_g F_g G_(g-c) rho_k^(g-lo),
//      so one LDS read of F and one of G feed K fused multiply-adds; the
//      Horner chains continue from slice to slice (slices run downwards).
// Each sample's sum runs over exactly |z_g - z_j| <= T h: the chains of a
// group share the Horner steps where all of them are inside their windows
// and are masked one by one on the few edge points where they are not.
#include <math.h>

#include <type_traits>

#include "common.h"
#include "launch.h"
#include "reduce.h"

namespace chimera {

namespace {

__device__ __forceinline__ bool decode_block(const GroupedArgs& a, int& e, int& b) {
  const int L = blockIdx.x;
  const int xcd = L & 7, s = L >> 3;
  const int u = (s / a.bc) * 8 + xcd;     // (event, lambda-chunk) unit on this XCD
  e = u / a.nchunk;
  b = (u % a.nchunk) * a.bc + (s % a.bc);
  return e < a.E && b < a.B;
}

// acc_k <- acc_k rho_k + F_g G_(g-c) for g = hi down to lo (A: chain type,
// FT: staged F type, GT_: G table type).
template <class A, class FT, class GT_, int K>
__device__ __forceinline__ void horner_span(A (&acc)[K], const A (&rho)[K],
                                            const FT* __restrict__ F,
                                            const GT_* __restrict__ G, int hi, int lo) {
  int g = hi;
  for (; g - 3 >= lo; g -= 4) {
    const A a0 = (A)F[g] * (A)G[g];
    const A a1 = (A)F[g - 1] * (A)G[g - 1];
    const A a2 = (A)F[g - 2] * (A)G[g - 2];
    const A a3 = (A)F[g - 3] * (A)G[g - 3];
#pragma unroll
    for (int k = 0; k < K; ++k)
      acc[k] = fma(fma(fma(fma(acc[k], rho[k], a0), rho[k], a1), rho[k], a2), rho[k], a3);
  }
  for (; g >= lo; --g) {
    const A av = (A)F[g] * (A)G[g];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = fma(acc[k], rho[k], av);
  }
}

// The same step with chain k restricted to its own window [lo_k, hi_k]:
// before the window the chain stays 0, after it the chain is left as is.
template <class A, int K>
__device__ __forceinline__ void horner_masked(A (&acc)[K], const A (&rho)[K], const int (&lo_k)[K],
                                              const int (&hi_k)[K], const A* __restrict__ F,
                                              const A* __restrict__ G, int hi, int lo) {
  for (int g = hi; g >= lo; --g) {
    const A av = F[g] * G[g];
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (g >= lo_k[k]) acc[k] = fma(acc[k], rho[k], g <= hi_k[k] ? av : (A)0);
  }
}

}  // namespace

template <int BS, int K, int GT, bool F32>
__global__ __launch_bounds__(BS) void k_event_grouped(GroupedArgs a) {
  int e, b;
  if (!decode_block(a, e, b)) return;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[BS / 64 + 1];
  __shared__ double z_ref;

  const LamParams P = a.P[b];
  const int flag = P.flag | a.flag_mono[b] | a.flag_range[b];
  double* out = a.lnI + (size_t)b * a.E + e;
  if (flag) {
    if (threadIdx.x == 0) *out = (flag & (kFlagDomain | kFlagNonMonotone)) ? -INFINITY : NAN;
    return;
  }
  const double2* chi = a.chi + (size_t)b * a.g.n_t;
  const double2* inv = a.inv + (size_t)b * a.g.n_u;
  const int g0 = a.ev_grp_off[e];
  const int ng = a.ev_grp_off[e + 1] - g0;
  const int p0 = a.ev_slot_off[e];
  const int np = a.ev_slot_off[e + 1] - p0;
  const int polish = F32 ? 0 : 1;
  const double dz = a.g.dz;

  // ---- 1. redshifts, weights, moments -------------------------------------
  if (threadIdx.x == 0) {
    const int j = a.grp_first[g0];
    z_ref = expm1(invert_x(P, chi, inv, a.g, a.dl[j], a.lndl[j], polish));
  }
  __syncthreads();
  const double zref = z_ref;
  double zz[GT][K];
  double ww[GT][K];
  double W1 = 0.0, W2 = 0.0, S1 = 0.0, S2 = 0.0;
#pragma unroll
  for (int t = 0; t < GT; ++t) {
    const int gi = threadIdx.x + t * BS;
    const int first = gi < ng ? a.grp_first[g0 + gi] : 0;
    const int cnt = gi < ng ? a.grp_cnt[g0 + gi] : 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      zz[t][k] = 0.0;
      ww[t][k] = 0.0;
      if (k < cnt) {
        const int j = first + k;
        const double x = invert_x(P, chi, inv, a.g, a.dl[j], a.lndl[j], polish);
        const double zp1 = exp(x);
        const double z = expm1(x);
        const double m1 = a.m1d[j] / zp1, m2 = a.m2d[j] / zp1;
        const double l1 = a.lnm1d[j] - x, l2 = a.lnm2d[j] - x;
        const double w = F32 ? (double)mass_weight32(P, m1, m2, l1, l2)
                             : mass_weight64(P, m1, m2, l1, l2);
        zz[t][k] = z;
        ww[t][k] = w;
        const double d = z - zref;
        W1 += w;
        W2 += w * w;
        S1 += w * d;
        S2 += w * d * d;
      }
    }
  }
  W1 = block_sum<BS>(W1, red);
  W2 = block_sum<BS>(W2, red);
  S1 = block_sum<BS>(S1, red);
  S2 = block_sum<BS>(S2, red);
  if (!(W1 > 0.0)) {
    if (threadIdx.x == 0) *out = -INFINITY;
    return;
  }
  // bandwidth: Scott's rule, Kish effective size, unbiased weighted variance
  const double den = W1 * W1 - W2;
  double var = 0.0;
  if (!(den <= 1e-12 * W1 * W1)) var = (S2 - S1 * S1 / W1) / (W1 - W2 / W1);
  if (var < 0.0) var = 0.0;
  const double h = fmax(sqrt(var) * pow(W1 * W1 / W2, -0.2), 2.0 * dz);
  const double T = a.trunc;

  // ---- per-sample windows |z_g - z_j| <= T h, group windows ----------------
  // chain k of a group covers exactly its own window [lo_k, hi_k]; the group
  // runs Horner over [lo_G, hi_G] = union, masking per chain only on the
  // edges outside [L_int, H_int] = intersection.
  int klo[GT][K], khi[GT][K];
  int glo[GT], ghi[GT], gli[GT], ghi_i[GT], cc[GT];
  double lo_loc = 1e9, hi_loc = -1e9, mg_loc = 0.0;
#pragma unroll
  for (int t = 0; t < GT; ++t) {
    int lo_u = 1 << 30, hi_u = -(1 << 30), lo_i = -(1 << 30), hi_i = 1 << 30;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      klo[t][k] = 1;
      khi[t][k] = 0;
      if (ww[t][k] > 0.0) {
        const double lo_d = fmax(ceil((zz[t][k] - T * h - a.g.z_lo) / dz), 0.0);
        const double hi_d = fmin(floor((zz[t][k] + T * h - a.g.z_lo) / dz), (double)(a.g.n_z - 1));
        if (lo_d <= hi_d) {
          klo[t][k] = (int)lo_d;
          khi[t][k] = (int)hi_d;
          lo_u = min(lo_u, klo[t][k]);
          hi_u = max(hi_u, khi[t][k]);
          lo_i = max(lo_i, klo[t][k]);
          hi_i = min(hi_i, khi[t][k]);
        }
      }
    }
    glo[t] = lo_u;
    ghi[t] = hi_u;
    gli[t] = lo_i;
    ghi_i[t] = hi_i;
    cc[t] = 0;
    if (lo_u <= hi_u) {
      cc[t] = (lo_u + hi_u) >> 1;
      lo_loc = fmin(lo_loc, (double)lo_u);
      hi_loc = fmax(hi_loc, (double)hi_u);
      mg_loc = fmax(mg_loc, (double)max(hi_u - cc[t], cc[t] - lo_u));
    }
  }
  const int A_lo = (int)(-block_max<BS>(-lo_loc, red));
  const int A_hi = (int)block_max<BS>(hi_loc, red);
  const int M = (int)block_max<BS>(mg_loc, red);     // |g - c| <= M over every group window

  // ---- Horner chains: rho_k, exponent bound -----------------------------------
  const double inv_h2 = 1.0 / (h * h);
  double dmax_loc = 0.0;
#pragma unroll
  for (int t = 0; t < GT; ++t)
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (klo[t][k] <= khi[t][k])
        dmax_loc = fmax(dmax_loc, fabs(zz[t][k] - (a.g.z_lo + (double)cc[t] * dz)));
  const double dmax = block_max<BS>(dmax_loc, red);
  // |ln (rho^t G)| over a window is at most 2M dz |delta| / h^2 + delta^2 / 2h^2
  const double ebound = 2.0 * (double)M * dz * dmax * inv_h2 + 0.5 * dmax * dmax * inv_h2;
  // chains in the path's precision; FP32 chains need the bound well inside
  // the float range, FP64 chains inside the double range
  using CT = typename std::conditional<F32, float, double>::type;
  const bool horner_ok = ebound < (F32 ? 60.0 : 600.0);
  double total = 0.0;
  double npts = 0.0;

  // G_m = exp(-m^2 dz^2 / 2h^2), m in [-M, M], in LDS after the F slice
  const int esz = F32 ? 4 : 8;
  const int f_elems = a.f_bytes / esz;
  CT* Gt = (CT*)(smem + a.f_bytes);
  const int gcount = 2 * M + 1;
  const bool gtab = gcount <= a.g_cap;
  if (gtab) {
    for (int m = threadIdx.x; m < gcount; m += BS) {
      const double u = (double)(m - M) * dz;
      Gt[m] = (CT)exp(-0.5 * u * u * inv_h2);
    }
  }
  // slice length per pixel row (odd row stride spreads the LDS banks)
  int L = f_elems / (np > 0 ? np : 1) - 1;
  L = L < 1 ? 1 : L;
  const int Ls = L | 1;

  CT acc[GT][K], rho[GT][K];
#pragma unroll
  for (int t = 0; t < GT; ++t)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double delta = zz[t][k] - (a.g.z_lo + (double)cc[t] * dz);
      rho[t][k] = (CT)exp(dz * delta * inv_h2);
      acc[t][k] = (CT)0;
    }

  if (gtab && A_lo <= A_hi && horner_ok) {
    for (int s_hi = A_hi; s_hi >= A_lo; s_hi -= L) {
      const int s_lo = max(s_hi - L + 1, A_lo);
      const int len = s_hi - s_lo + 1;
      __syncthreads();   // the previous slice is consumed (and G is written)
      const double* gzb = a.gz64 + (size_t)b * a.g.n_z;
      for (int idx = threadIdx.x; idx < np * len; idx += BS) {
        const int p = idx / len, gg = s_lo + idx - p * len;
        const size_t src = (size_t)a.slot_row[p0 + p] * a.g.n_z + gg;
        if (F32) ((float*)smem)[p * Ls + (gg - s_lo)] = a.nz32[src] * a.gz32[(size_t)b * a.g.n_z + gg];
        else ((double*)smem)[p * Ls + (gg - s_lo)] = a.nz64[src] * gzb[gg];
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < GT; ++t) {
        const int gi = threadIdx.x + t * BS;
        if (gi >= ng || glo[t] > ghi[t]) continue;
        const int hi = min(ghi[t], s_hi), lo = max(glo[t], s_lo);
        if (lo > hi) continue;
        const CT* Fp = (const CT*)smem + a.grp_slot[g0 + gi] * Ls - s_lo;
        const CT* Gp = Gt + (M - cc[t]);
        if (gli[t] <= ghi_i[t]) {
          // upper edge (masked), shared bulk, lower edge (masked)
          horner_masked<CT, K>(acc[t], rho[t], klo[t], khi[t], Fp, Gp, hi, max(lo, ghi_i[t] + 1));
          horner_span<CT, CT, CT, K>(acc[t], rho[t], Fp, Gp, min(hi, ghi_i[t]), max(lo, gli[t]));
          horner_masked<CT, K>(acc[t], rho[t], klo[t], khi[t], Fp, Gp, min(hi, gli[t] - 1), lo);
        } else {
          horner_masked<CT, K>(acc[t], rho[t], klo[t], khi[t], Fp, Gp, hi, lo);
        }
      }
    }
    // prefactor C_k rho_k^(lo_k - c) and the sum over the event's samples
#pragma unroll
    for (int t = 0; t < GT; ++t) {
      const int gi = threadIdx.x + t * BS;
      if (gi >= ng || glo[t] > ghi[t]) continue;
      const double cir = a.grp_c[g0 + gi];
      const double zc = a.g.z_lo + (double)cc[t] * dz;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (klo[t][k] > khi[t][k]) continue;
        const double av = (double)acc[t][k];
        if (av == 0.0) continue;
        const double delta = zz[t][k] - zc;
        const double lg = -0.5 * delta * delta * inv_h2 + (double)(klo[t][k] - cc[t]) * dz * delta * inv_h2;
        total += cir * ww[t][k] * exp(lg) * av;
      }
    }
  } else if (A_lo <= A_hi) {
    // fallback (very wide windows): direct sums from the catalogue rows
    const double* gzb = a.gz64 + (size_t)b * a.g.n_z;
#pragma unroll
    for (int t = 0; t < GT; ++t) {
      const int gi = threadIdx.x + t * BS;
      if (gi >= ng) continue;
      const double cir = a.grp_c[g0 + gi];
      const size_t row = (size_t)a.slot_row[p0 + a.grp_slot[g0 + gi]] * a.g.n_z;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (klo[t][k] > khi[t][k]) continue;
        double sacc = 0.0;
        for (int g = klo[t][k]; g <= khi[t][k]; ++g) {
          const double u = (a.g.z_lo + (double)g * dz - zz[t][k]);
          sacc += exp(-0.5 * u * u * inv_h2) * a.nz64[row + g] * gzb[g];
        }
        total += cir * ww[t][k] * sacc;
      }
    }
  }
  if (a.count) {
    // the method's evaluations: grid points with |z_g - z_j| <= T h
#pragma unroll
    for (int t = 0; t < GT; ++t)
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (klo[t][k] <= khi[t][k]) npts += (double)(khi[t][k] - klo[t][k] + 1);
  }
  total = block_sum<BS>(total, red);
  if (a.count) {
    npts = block_sum<BS>(npts, red);
    if (threadIdx.x == 0) atomicAdd(a.count, (unsigned long long)npts);
  }
  if (threadIdx.x == 0) {
    const double I = total * kInvSqrt2Pi / h;
    *out = I > 0.0 ? log(I) : -INFINITY;
  }
}

hipError_t launch_events_grouped(const GroupedArgs& a0, bool f32, int max_groups, hipStream_t st) {
  GroupedArgs a = a0;
  a.bc = a.B < 32 ? a.B : 32;
  a.nchunk = (a.B + a.bc - 1) / a.bc;
  const long long units = (long long)a.E * a.nchunk;
  const long long blocks = ((units + 7) / 8) * 8 * a.bc;
  const int gt = (max_groups + kGroupBS - 1) / kGroupBS;
  a.f_bytes = f32 ? kGroupFBytes32 : kGroupFBytes64;
  a.g_cap = kGroupGCap;
  const size_t lds = (size_t)a.f_bytes + (size_t)a.g_cap * sizeof(double);
#define CH_GROUPED(GTV)                                                                          \
  do {                                                                                           \
    if (f32) {                                                                                   \
      auto kf = k_event_grouped<kGroupBS, kGroupK, GTV, true>;                                   \
      hipError_t e_ = hipFuncSetAttribute((const void*)kf,                                       \
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
      if (e_ != hipSuccess) return e_;                                                           \
      kf<<<(unsigned)blocks, kGroupBS, lds, st>>>(a);                                            \
    } else {                                                                                     \
      auto kf = k_event_grouped<kGroupBS, kGroupK, GTV, false>;                                  \
      hipError_t e_ = hipFuncSetAttribute((const void*)kf,                                       \
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
      if (e_ != hipSuccess) return e_;                                                           \
      kf<<<(unsigned)blocks, kGroupBS, lds, st>>>(a);                                            \
    }                                                                                            \
  } while (0)
  if (gt <= 1) CH_GROUPED(1);
  else return hipErrorInvalidValue;
#undef CH_GROUPED
  return hipGetLastError();
}

}  // namespace chimera
