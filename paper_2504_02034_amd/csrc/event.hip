// Per-(event, lambda) kernel sums of the many-1D likelihood (eqs.
// like-integrals and gw-kernel-many1d), gfx950.
//
// k_event_zw      one (event, lambda) per workgroup, one sample per thread:
//                 z_j from d_L^gw, w_j = p(m1) p(m2|m1) into scratch, and the
//                 event's bandwidth h (Scott's rule, Kish effective size,
//                 unbiased weighted variance by two passes about the mean).
// k_event_smooth  one work unit (<= 256 sample groups of one event, ordered by
//                 distance, so a narrow redshift range) at one lambda per
//                 workgroup:
//                   - every thread takes one group (<= K consecutive samples of
//                     one pixel); each sample's window |z_g - z_j| <= T h;
//                   - the unit's redshift range is cut into slices; for each
//                     slice F_r(z_g) = n_r(z_g) g(z_g) of every pixel of the
//                     event is staged in LDS;
//                   - each lane evaluates its group's K Gaussian sums by
//                     Horner's rule in rho_k = exp(dz delta_k / h^2) about the
//                     group's centre c, with G_m = exp(-m^2 dz^2 / 2h^2):
//                       sum_g F_g N(z_g; z_k, h)
//                         = C_k rho_k^(lo_k - c) sum_g F_g G_(g-c) rho_k^(g-lo_k),
//                     so one LDS read of F and one of G feed K fused
//                     multiply-adds; the chains continue from slice to slice
//                     and are masked one by one only on the few edge points
//                     where a sample's window and the group's differ;
//                   - the unit's partial sum of c_ir w_j A_j goes to scratch.
// k_event_final   per (event, lambda): the units' partial sums in a fixed
//                 order, I_i = sum / (h sqrt(2 pi)), ln I_i.
#include <math.h>

#include <type_traits>

#include "common.h"
#include "launch.h"
#include "reduce.h"

namespace chimera {

namespace {

// XCD-aware block order: the blocks of one item (event or unit) at 32
// consecutive lambdas land on one XCD (block id mod 8) back to back, so the
// item's data stay in that XCD's L2.
__device__ __forceinline__ bool decode_block(int n_items, int B, int& item, int& b) {
  const int bc = B < 32 ? B : 32;
  const int nchunk = (B + bc - 1) / bc;
  const int L = blockIdx.x;
  const int xcd = L & 7, s = L >> 3;
  const int u = (s / bc) * 8 + xcd;
  item = u / nchunk;
  b = (u % nchunk) * bc + (s % bc);
  return item < n_items && b < B;
}

long long grid_blocks(int n_items, int B) {
  const int bc = B < 32 ? B : 32;
  const long long nchunk = (B + bc - 1) / bc;
  const long long units = (long long)n_items * nchunk;
  return ((units + 7) / 8) * 8 * bc;
}

// acc_k <- acc_k rho_k + F_g G_(g-c) for g = hi down to lo (all chains inside
// their windows).
template <class A, int K>
__device__ __forceinline__ void horner_span(A (&acc)[K], const A (&rho)[K], const A* __restrict__ F,
                                            const A* __restrict__ G, int hi, int lo) {
  int g = hi;
  for (; g - 3 >= lo; g -= 4) {
    const A a0 = F[g] * G[g];
    const A a1 = F[g - 1] * G[g - 1];
    const A a2 = F[g - 2] * G[g - 2];
    const A a3 = F[g - 3] * G[g - 3];
#pragma unroll
    for (int k = 0; k < K; ++k)
      acc[k] = fma(fma(fma(fma(acc[k], rho[k], a0), rho[k], a1), rho[k], a2), rho[k], a3);
  }
  for (; g >= lo; --g) {
    const A av = F[g] * G[g];
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

// ---------------------------------------------------------------------------
template <bool F32>
__global__ __launch_bounds__(kZwBS) void k_event_zw(EventArgs a) {
  int e, b;
  if (!decode_block(a.E, a.B, e, b)) return;
  using CT = typename std::conditional<F32, float, double>::type;
  constexpr int NW = kZwBS / 64 + 1;
  __shared__ double red[3 * NW];
  const LamParams P = a.P[b];
  if (P.flag | a.flag_mono[b] | a.flag_range[b]) return;   // the final kernel reports it
  const double2* chi = a.chi + (size_t)b * a.g.n_t;
  const double2* inv = a.inv + (size_t)b * a.g.n_u;
  const int s0 = a.ev_samp_off[e];
  const int ns = a.ev_samp_off[e + 1] - s0;
  double* zb = a.zbuf + (size_t)b * a.S + s0;
  CT* wb = (CT*)a.wbuf + (size_t)b * a.S + s0;
  double m[3] = {0.0, 0.0, 0.0};   // W1, W2, sum w z
  for (int j = threadIdx.x; j < ns; j += kZwBS) {
    const int q = s0 + j;
    double z, w;
    sample_zw<F32>(P, chi, inv, a.g, a.dl[q], a.lndl[q], a.m1d[q], a.m2d[q], a.lnm1d[q],
                   a.lnm2d[q], z, w);
    const CT wc = (CT)w;
    zb[j] = z;
    wb[j] = wc;
    const double wd = (double)wc;
    m[0] += wd;
    m[1] += wd * wd;
    m[2] += wd * z;
  }
  block_reduce<kZwBS, 3, false>(m, red);
  const double W1 = m[0], W2 = m[1];
  if (!(W1 > 0.0)) {
    if (threadIdx.x == 0) a.hbuf[(size_t)b * a.E + e] = -1.0;
    return;
  }
  const double mu = m[2] / W1;
  double v[1] = {0.0};
  for (int j = threadIdx.x; j < ns; j += kZwBS) {   // this thread's own writes
    const double d = zb[j] - mu;
    v[0] += (double)wb[j] * d * d;
  }
  block_reduce<kZwBS, 1, false>(v, red);
  if (threadIdx.x == 0) {
    double var = 0.0;
    if (!(W1 * W1 - W2 <= 1e-12 * W1 * W1)) var = v[0] / (W1 - W2 / W1);
    a.hbuf[(size_t)b * a.E + e] = fmax(sqrt(var) * pow(W1 * W1 / W2, -0.2), 2.0 * a.g.dz);
  }
}

// ---------------------------------------------------------------------------
template <bool F32>
__global__ __launch_bounds__(kSmBS) void k_event_smooth(EventArgs a) {
  constexpr int K = kGroupK;
  constexpr int BS = kSmBS;
  int u, b;
  if (!decode_block(a.U, a.B, u, b)) return;
  using CT = typename std::conditional<F32, float, double>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NW = BS / 64 + 1;
  __shared__ double red[4 * NW];
  double* part = a.part + (size_t)b * a.U + u;
  const int e = a.unit_event[u];
  const LamParams P = a.P[b];
  const double h = a.hbuf[(size_t)b * a.E + e];
  if ((P.flag | a.flag_mono[b] | a.flag_range[b]) || !(h > 0.0)) {
    if (threadIdx.x == 0) *part = 0.0;
    return;
  }
  const int p0 = a.ev_slot_off[e];
  const int np = a.ev_slot_off[e + 1] - p0;
  const double dz = a.g.dz;
  const double T = a.trunc;
  const double inv_h2 = 1.0 / (h * h);
  const double* zb = a.zbuf + (size_t)b * a.S;
  const CT* wb = (const CT*)a.wbuf + (size_t)b * a.S;

  // ---- this thread's group: windows, union / intersection, centre -------------
  const bool has = threadIdx.x < a.unit_ngrp[u];
  const int gi = a.unit_grp0[u] + threadIdx.x;
  const int first = has ? a.grp_first[gi] : 0;
  const int cnt = has ? a.grp_cnt[gi] : 0;
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
      zk[k] = zb[first + k];
      wk[k] = (double)wb[first + k];
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
  int c = 0;
  double mloc = 0.0, dloc = 0.0;
  if (zn > 0.0) {
    const double cd = fmin(fmax(rint((zsum / zn - a.g.z_lo) / dz), -4.0 * a.g.n_z), 8.0 * a.g.n_z);
    c = (int)cd;
    mloc = (double)max(hi_u - c, c - lo_u);
    const double zc0 = a.g.z_lo + cd * dz;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (klo[k] <= khi[k]) dloc = fmax(dloc, fabs(zk[k] - zc0));
  }
  double mx[4] = {lo_u <= hi_u ? -(double)lo_u : -1e9, lo_u <= hi_u ? (double)hi_u : -1e9, mloc,
                  dloc};
  block_reduce<BS, 4, true>(mx, red);
  const int A_lo = (int)(-mx[0]);
  const int A_hi = (int)mx[1];
  const int M = (int)mx[2];              // |g - c| <= M over every group window of the unit
  const double dmax = mx[3];

  // Horner's partial sums are the kernel values times rho^(c - lo) / C: at
  // most exp(M dz |delta| / h^2 + delta^2 / 2h^2) away from the true values
  const double ebound = (double)M * dz * dmax * inv_h2 + 0.5 * dmax * dmax * inv_h2;
  const bool horner_ok = ebound < (F32 ? 60.0 : 600.0);
  const double zc = a.g.z_lo + (double)c * dz;
  const double cir = has ? a.grp_c[gi] : 0.0;
  CT acc[K], rho[K];
  double coef[K];                        // c_ir w_k C_k rho_k^(lo_k - c)
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double delta = zk[k] - zc;
    acc[k] = (CT)0;
    coef[k] = 0.0;
    if (klo[k] > khi[k]) {
      // a chain without a window (zero weight, or outside the grid) still runs
      // through the shared bulk; rho = 0 keeps it finite (the ratio of a
      // far-away sample would overflow) and coef = 0 drops it
      rho[k] = (CT)0;
    } else if (F32) {
      rho[k] = (CT)__expf((float)(dz * delta * inv_h2));
      coef[k] = cir * wk[k] *
                (double)__expf((float)(-0.5 * delta * delta * inv_h2 +
                                       (double)(klo[k] - c) * dz * delta * inv_h2));
    } else {
      rho[k] = (CT)exp(dz * delta * inv_h2);
      coef[k] = cir * wk[k] *
                exp(-0.5 * delta * delta * inv_h2 + (double)(klo[k] - c) * dz * delta * inv_h2);
    }
  }
  double total = 0.0, npts = 0.0;
  if (a.count) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (klo[k] <= khi[k]) npts += (double)(khi[k] - klo[k] + 1);
  }

  // G_m = exp(-m^2 dz^2 / 2h^2), m in [-M, M], in LDS after the F slice
  const int f_elems = kSmFBytes / (int)sizeof(CT);
  CT* Gt = (CT*)(smem + kSmFBytes);
  const int gcount = 2 * M + 1;
  const bool gtab = gcount <= kSmGCap;
  if (gtab) {
    for (int q = threadIdx.x; q < gcount; q += BS) {
      const double x = (double)(q - M) * dz;
      Gt[q] = (CT)exp(-0.5 * x * x * inv_h2);
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
      // F_r(z_g) = n_r(z_g) g(z_g); several independent loads in flight per
      // thread before the LDS stores
      const int nst = np * len;
      constexpr int UR = F32 ? 8 : 4;
      for (int i0 = threadIdx.x; i0 < nst; i0 += BS * UR) {
        CT v[UR];
        int dst[UR];
#pragma unroll
        for (int r = 0; r < UR; ++r) {
          const int idx = i0 + r * BS;
          dst[r] = -1;
          v[r] = (CT)0;
          if (idx < nst) {
            const int p = idx / len, gg = s_lo + idx - p * len;
            const size_t src = (size_t)a.slot_row[p0 + p] * a.g.n_z + gg;
            dst[r] = p * Ls + (gg - s_lo);
            if (F32) v[r] = (CT)(a.nz32[src] * gzf[gg]);
            else v[r] = (CT)(a.nz64[src] * gzb[gg]);
          }
        }
#pragma unroll
        for (int r = 0; r < UR; ++r)
          if (dst[r] >= 0) ((CT*)smem)[dst[r]] = v[r];
      }
      __syncthreads();
      if (has && lo_u <= hi_u) {
        const int hi = min(hi_u, s_hi), lo = max(lo_u, s_lo);
        if (lo <= hi) {
          const CT* Fp = (const CT*)smem + a.grp_slot[gi] * Ls - s_lo;
          const CT* Gp = Gt + (M - c);
          if (lo_i <= hi_i) {
            // upper edge (masked), shared bulk, lower edge (masked)
            horner_masked<CT, K>(acc, rho, klo, khi, Fp, Gp, hi, max(lo, hi_i + 1));
            horner_span<CT, K>(acc, rho, Fp, Gp, min(hi, hi_i), max(lo, lo_i));
            horner_masked<CT, K>(acc, rho, klo, khi, Fp, Gp, min(hi, lo_i - 1), lo);
          } else {
            horner_masked<CT, K>(acc, rho, klo, khi, Fp, Gp, hi, lo);
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (klo[k] <= khi[k]) total += coef[k] * (double)acc[k];
  } else if (A_lo <= A_hi && has) {
    // fallback (windows too wide for the tables or the chain range): direct sums
    const double* gzb = a.gz64 + (size_t)b * a.g.n_z;
    const size_t row = (size_t)a.slot_row[p0 + a.grp_slot[gi]] * a.g.n_z;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (klo[k] > khi[k]) continue;
      double sacc = 0.0;
      for (int g = klo[k]; g <= khi[k]; ++g) {
        const double x = (a.g.z_lo + (double)g * dz - zk[k]);
        sacc += exp(-0.5 * x * x * inv_h2) * a.nz64[row + g] * gzb[g];
      }
      total += cir * wk[k] * sacc;
    }
  }
  double fin[2] = {total, npts};
  block_reduce<BS, 2, false>(fin, red);
  if (threadIdx.x == 0) {
    *part = fin[0];
    if (a.count) atomicAdd(a.count, (unsigned long long)fin[1]);
  }
}

// ---------------------------------------------------------------------------
__global__ void k_event_final(EventArgs a) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)a.B * a.E) return;
  const int b = (int)(id / a.E), e = (int)(id % a.E);
  const int flag = a.P[b].flag | a.flag_mono[b] | a.flag_range[b];
  double out;
  if (flag) {
    out = (flag & (kFlagDomain | kFlagNonMonotone)) ? -INFINITY : NAN;
  } else {
    const double h = a.hbuf[(size_t)b * a.E + e];
    double s = 0.0;
    for (int u = a.ev_unit_off[e]; u < a.ev_unit_off[e + 1]; ++u) s += a.part[(size_t)b * a.U + u];
    const double I = h > 0.0 ? s * kInvSqrt2Pi / h : 0.0;
    out = I > 0.0 ? log(I) : -INFINITY;
  }
  a.lnI[(size_t)b * a.E + e] = out;
}

// ---------------------------------------------------------------------------
hipError_t launch_events(const EventArgs& a, bool f32, hipStream_t st, hipEvent_t t0,
                         hipEvent_t t1) {
  const long long bz = grid_blocks(a.E, a.B);
  const long long bs = grid_blocks(a.U, a.B);
  const size_t lds = (size_t)kSmFBytes + (size_t)kSmGCap * (f32 ? sizeof(float) : sizeof(double));
  hipError_t err;
  if (f32) {
    k_event_zw<true><<<(unsigned)bz, kZwBS, 0, st>>>(a);
    err = hipFuncSetAttribute((const void*)k_event_smooth<true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    if (t0 && (err = hipEventRecord(t0, st)) != hipSuccess) return err;
    k_event_smooth<true><<<(unsigned)bs, kSmBS, lds, st>>>(a);
    if (t1 && (err = hipEventRecord(t1, st)) != hipSuccess) return err;
  } else {
    k_event_zw<false><<<(unsigned)bz, kZwBS, 0, st>>>(a);
    err = hipFuncSetAttribute((const void*)k_event_smooth<false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    if (t0 && (err = hipEventRecord(t0, st)) != hipSuccess) return err;
    k_event_smooth<false><<<(unsigned)bs, kSmBS, lds, st>>>(a);
    if (t1 && (err = hipEventRecord(t1, st)) != hipSuccess) return err;
  }
  const long long nf = (long long)a.B * a.E;
  k_event_final<<<(unsigned)((nf + 255) / 256), 256, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace chimera
