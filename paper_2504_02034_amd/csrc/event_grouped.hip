// Per-(event, lambda) kernel sums of the many-1D likelihood (eqs.
// like-integrals and gw-kernel-many1d), gfx950.
//
// One workgroup handles one event at one lambda:
//   1. one sample per thread is mapped to (z_j, w_j), kept in LDS, and the
//      workgroup reduces the weighted moments to the event's bandwidth h;
//      then every thread takes one sample group (<= K consecutive samples of
//      one pixel, sorted on the host by distance; groups ordered by distance
//      so a wave's lanes sit close in redshift at every lambda);
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

template <int BS, int K, bool F32>
__global__ __launch_bounds__(BS) void k_event_grouped(GroupedArgs a) {
  int e, b;
  if (!decode_block(a, e, b)) return;
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NW = BS / 64 + 1;
  __shared__ double red[4 * NW];
  using CT = typename std::conditional<F32, float, double>::type;

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
  const int s0 = a.ev_samp_off[e];
  const int ns = a.ev_samp_off[e + 1] - s0;
  const double dz = a.g.dz;

  // ---- 1. one sample per thread: z_j, w_j into LDS (the F region), moments ----
  double* zs = (double*)smem;
  double* wsm = zs + ns;
  double m[3] = {0.0, 0.0, 0.0};     // W1, W2, sum w z
  for (int j = threadIdx.x; j < ns; j += BS) {
    const int q = s0 + j;
    double z, w;
    sample_zw<F32>(P, chi, inv, a.g, a.dl[q], a.lndl[q], a.m1d[q], a.m2d[q], a.lnm1d[q],
                   a.lnm2d[q], z, w);
    zs[j] = z;
    wsm[j] = w;
    m[0] += w;
    m[1] += w * w;
    m[2] += w * z;
  }
  block_reduce<BS, 3, false>(m, red);
  const double W1 = m[0], W2 = m[1];
  if (!(W1 > 0.0)) {
    if (threadIdx.x == 0) *out = -INFINITY;
    return;
  }
  // bandwidth: Scott's rule with the Kish effective size and the unbiased
  // weighted variance (second pass about the mean)
  const double mu = m[2] / W1;
  double v2[1] = {0.0};
  for (int j = threadIdx.x; j < ns; j += BS) {
    const double d = zs[j] - mu;
    v2[0] += wsm[j] * d * d;
  }
  block_reduce<BS, 1, false>(v2, red);
  double var = 0.0;
  if (!(W1 * W1 - W2 <= 1e-12 * W1 * W1)) var = v2[0] / (W1 - W2 / W1);
  const double h = fmax(sqrt(var) * pow(W1 * W1 / W2, -0.2), 2.0 * dz);
  const double T = a.trunc;
  const double inv_h2 = 1.0 / (h * h);

  // ---- 2. this thread's group: windows |z_g - z_k| <= T h, centre, chains ----
  // chain k covers exactly [lo_k, hi_k]; Horner runs over the union
  // [lo_u, hi_u] and masks chains only outside the intersection [lo_i, hi_i].
  const bool has = threadIdx.x < ng;
  const int gi = threadIdx.x;
  const int first = has ? a.grp_first[g0 + gi] - s0 : 0;
  const int cnt = has ? a.grp_cnt[g0 + gi] : 0;
  int klo[K], khi[K];
  double zk[K], wk[K];
  int lo_u = 1 << 30, hi_u = -(1 << 30), lo_i = -(1 << 30), hi_i = 1 << 30;
  double zsum = 0.0, zn = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    klo[k] = 1;
    khi[k] = 0;
    zk[k] = 0.0;
    wk[k] = 0.0;
    if (k < cnt) {
      zk[k] = zs[first + k];
      wk[k] = wsm[first + k];
      if (wk[k] > 0.0) {
        const double lo_d = fmax(ceil((zk[k] - T * h - a.g.z_lo) / dz), 0.0);
        const double hi_d = fmin(floor((zk[k] + T * h - a.g.z_lo) / dz), (double)(a.g.n_z - 1));
        if (lo_d <= hi_d) {
          klo[k] = (int)lo_d;
          khi[k] = (int)hi_d;
          lo_u = min(lo_u, klo[k]);
          hi_u = max(hi_u, khi[k]);
          lo_i = max(lo_i, klo[k]);
          hi_i = min(hi_i, khi[k]);
          zsum += zk[k];
          zn += 1.0;
        }
      }
    }
  }
  // centre: the grid point nearest the mean redshift of the group's chains
  int c = 0;
  double mloc = 0.0, dloc = 0.0;
  if (zn > 0.0) {
    const double cd = fmin(fmax(rint((zsum / zn - a.g.z_lo) / dz), -4.0 * a.g.n_z), 8.0 * a.g.n_z);
    c = (int)cd;
    mloc = (double)max(hi_u - c, c - lo_u);
    const double zc = a.g.z_lo + cd * dz;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (klo[k] <= khi[k]) dloc = fmax(dloc, fabs(zk[k] - zc));
  }
  double mx[4] = {lo_u <= hi_u ? -(double)lo_u : -1e9, lo_u <= hi_u ? (double)hi_u : -1e9, mloc,
                  dloc};
  block_reduce<BS, 4, true>(mx, red);     // also: every thread is done reading zs / wsm
  const int A_lo = (int)(-mx[0]);
  const int A_hi = (int)mx[1];
  const int M = (int)mx[2];               // |g - c| <= M over every group's union window
  const double dmax = mx[3];

  // Horner's partial sums are the kernel values times rho^(c - lo) / C: at
  // most exp(M dz |delta| / h^2 + delta^2 / 2h^2) away from the true values
  const double ebound = (double)M * dz * dmax * inv_h2 + 0.5 * dmax * dmax * inv_h2;
  const bool horner_ok = ebound < (F32 ? 60.0 : 600.0);
  const double zc = a.g.z_lo + (double)c * dz;
  const double cir = has ? a.grp_c[g0 + gi] : 0.0;
  CT acc[K], rho[K];
  double coef[K];                         // c_ir w_k C_k rho_k^(lo_k - c)
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double delta = zk[k] - zc;
    rho[k] = (CT)exp(dz * delta * inv_h2);
    acc[k] = (CT)0;
    coef[k] = 0.0;
    if (klo[k] <= khi[k])
      coef[k] = cir * wk[k] *
                exp(-0.5 * delta * delta * inv_h2 + (double)(klo[k] - c) * dz * delta * inv_h2);
  }
  double total = 0.0;

  // G_m = exp(-m^2 dz^2 / 2h^2), m in [-M, M], in LDS after the F slice
  const int f_elems = a.f_bytes / (int)sizeof(CT);
  CT* Gt = (CT*)(smem + a.f_bytes);
  const int gcount = 2 * M + 1;
  const bool gtab = gcount <= a.g_cap;
  if (gtab) {
    for (int q = threadIdx.x; q < gcount; q += BS) {
      const double u = (double)(q - M) * dz;
      Gt[q] = (CT)exp(-0.5 * u * u * inv_h2);
    }
  }
  // slice length per pixel row (odd row stride spreads the LDS banks)
  int L = f_elems / (np > 0 ? np : 1) - 1;
  L = L < 1 ? 1 : L;
  const int Ls = L | 1;

  if (gtab && A_lo <= A_hi && horner_ok) {
    const double* gzb = a.gz64 + (size_t)b * a.g.n_z;
    const float* gzf = a.gz32 + (size_t)b * a.g.n_z;
    for (int s_hi = A_hi; s_hi >= A_lo; s_hi -= L) {
      const int s_lo = max(s_hi - L + 1, A_lo);
      const int len = s_hi - s_lo + 1;
      __syncthreads();   // the previous slice is consumed (and G is written)
      // F_r(z_g) = n_r(z_g) g(z_g): several independent loads in flight per
      // thread before the LDS stores
      const int nst = np * len;
      constexpr int U = F32 ? 8 : 4;
      for (int i0 = threadIdx.x; i0 < nst; i0 += BS * U) {
        CT v[U];
        int dst[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int idx = i0 + u * BS;
          dst[u] = -1;
          v[u] = (CT)0;
          if (idx < nst) {
            const int p = idx / len, gg = s_lo + idx - p * len;
            const size_t src = (size_t)a.slot_row[p0 + p] * a.g.n_z + gg;
            dst[u] = p * Ls + (gg - s_lo);
            if (F32) v[u] = (CT)(a.nz32[src] * gzf[gg]);
            else v[u] = (CT)(a.nz64[src] * gzb[gg]);
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (dst[u] >= 0) ((CT*)smem)[dst[u]] = v[u];
      }
      __syncthreads();
      if (has && lo_u <= hi_u) {
        const int hi = min(hi_u, s_hi), lo = max(lo_u, s_lo);
        if (lo <= hi) {
          const CT* Fp = (const CT*)smem + a.grp_slot[g0 + gi] * Ls - s_lo;
          const CT* Gp = Gt + (M - c);
          if (lo_i <= hi_i) {
            // upper edge (masked), shared bulk, lower edge (masked)
            horner_masked<CT, K>(acc, rho, klo, khi, Fp, Gp, hi, max(lo, hi_i + 1));
            horner_span<CT, CT, CT, K>(acc, rho, Fp, Gp, min(hi, hi_i), max(lo, lo_i));
            horner_masked<CT, K>(acc, rho, klo, khi, Fp, Gp, min(hi, lo_i - 1), lo);
          } else {
            horner_masked<CT, K>(acc, rho, klo, khi, Fp, Gp, hi, lo);
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) total += coef[k] * (double)acc[k];
  } else if (A_lo <= A_hi && has) {
    // fallback (windows too wide for the tables or the chain range): direct
    // sums; z and w are still in LDS since no slice was staged
    const double* gzb = a.gz64 + (size_t)b * a.g.n_z;
    const size_t row = (size_t)a.slot_row[p0 + a.grp_slot[g0 + gi]] * a.g.n_z;
    for (int k = 0; k < cnt; ++k) {
      const double zj = zs[first + k], wj = wsm[first + k];
      if (!(wj > 0.0)) continue;
      const double lo_d = fmax(ceil((zj - T * h - a.g.z_lo) / dz), 0.0);
      const double hi_d = fmin(floor((zj + T * h - a.g.z_lo) / dz), (double)(a.g.n_z - 1));
      if (!(lo_d <= hi_d)) continue;
      double sacc = 0.0;
      for (int g = (int)lo_d; g <= (int)hi_d; ++g) {
        const double u = (a.g.z_lo + (double)g * dz - zj);
        sacc += exp(-0.5 * u * u * inv_h2) * a.nz64[row + g] * gzb[g];
      }
      total += cir * wj * sacc;
    }
  }
  double fin[2] = {total, 0.0};
  if (a.count) {
    // the method's evaluations: grid points with |z_g - z_j| <= T h
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (klo[k] <= khi[k]) fin[1] += (double)(khi[k] - klo[k] + 1);
  }
  block_reduce<BS, 2, false>(fin, red);
  if (threadIdx.x == 0) {
    if (a.count) atomicAdd(a.count, (unsigned long long)fin[1]);
    const double I = fin[0] * kInvSqrt2Pi / h;
    *out = I > 0.0 ? log(I) : -INFINITY;
  }
}

hipError_t launch_events_grouped(const GroupedArgs& a0, bool f32, int max_groups, hipStream_t st) {
  GroupedArgs a = a0;
  a.bc = a.B < 32 ? a.B : 32;
  a.nchunk = (a.B + a.bc - 1) / a.bc;
  const long long units = (long long)a.E * a.nchunk;
  const long long blocks = ((units + 7) / 8) * 8 * a.bc;
  if (max_groups > kGroupBS) return hipErrorInvalidValue;
  a.f_bytes = f32 ? kGroupFBytes32 : kGroupFBytes64;
  a.g_cap = kGroupGCap;
  const size_t lds = (size_t)a.f_bytes + (size_t)a.g_cap * (f32 ? sizeof(float) : sizeof(double));
  const void* kf = f32 ? (const void*)k_event_grouped<kGroupBS, kGroupK, true>
                       : (const void*)k_event_grouped<kGroupBS, kGroupK, false>;
  hipError_t err = hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  if (f32) k_event_grouped<kGroupBS, kGroupK, true><<<(unsigned)blocks, kGroupBS, lds, st>>>(a);
  else k_event_grouped<kGroupBS, kGroupK, false><<<(unsigned)blocks, kGroupBS, lds, st>>>(a);
  return hipGetLastError();
}

}  // namespace chimera
