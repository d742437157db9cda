// Per-(event, lambda) kernel sums of the many-1D likelihood (eqs.
// like-integrals and gw-kernel-many1d), gfx950.
//
// k_event_zw        one (event, lambda) per workgroup, one sample per thread:
//                   z_j from d_L^gw, w_j = p(m1) p(m2|m1) into scratch, and the
//                   event's bandwidth h (Scott's rule, Kish effective size,
//                   unbiased weighted variance from moments about a shift
//                   inside the data, one pass).
// k_event_smooth64  one work unit (<= 256 sample groups of one event, ordered
// k_event_smooth32  by distance, so a narrow redshift range) at one lambda per
//                   workgroup:
//                     - every thread takes one group (<= K consecutive samples
//                       of one pixel); each sample's window |z_g - z_j| <= T h;
//                     - the unit's redshift range is cut into slices; for each
//                       slice F_r(z_g) = n_r(z_g) g(z_g) of every pixel of the
//                       event is staged in LDS, one row segment per wave
//                       instruction;
//                     - each lane evaluates its group's K Gaussian sums by
//                       Horner's rule in rho_k = exp(dz delta_k / h^2) about the
//                       group's centre c, with G_m = exp(-m^2 dz^2 / 2h^2):
//                         sum_g F_g N(z_g; z_k, h)
//                           = C_k rho_k^(lo_k - c) sum_g F_g G_(g-c) rho_k^(g-lo_k),
//                       so one LDS read of F and one of G feed K fused
//                       multiply-adds; the chains continue from slice to slice
//                       and are masked one bound at a time only on the edge
//                       points where a sample's window and the group's differ;
//                     - the unit's partial sum of c_ir w_j A_j goes to scratch.
//                   Both run four workgroups per CU (the chain factors are
//                   formed after the sweep, which keeps the registers low).
// k_event_final     per (event, lambda): the units' partial sums in a fixed
//                   order, I_i = sum / (h sqrt(2 pi)), ln I_i.
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "common.h"
#include "launch.h"
#include "reduce.h"

namespace chimera {

namespace {

// acc_k <- acc_k rho_k + F_g G_(g-c) for g = hi down to lo (all chains inside
// their windows), eight grid points per iteration (then four, then one).
template <class A, int K>
__device__ __forceinline__ void horner_span(A (&acc)[K], const A (&rho)[K], const A* __restrict__ F,
                                            const A* __restrict__ G, int hi, int lo) {
  int g = hi;
  for (; g - 7 >= lo; g -= 8) {
    A av[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) av[i] = F[g - i] * G[g - i];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      A t = acc[k];
#pragma unroll
      for (int i = 0; i < 8; ++i) t = fma(t, rho[k], av[i]);
      acc[k] = t;
    }
  }
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

// Edge steps, where the group's windows differ.  Above the common part every
// chain has passed its lower bound, so only g <= hi_k is tested (a chain that
// has not entered its window is 0); below it every chain is inside its upper
// bound, so only g >= lo_k is tested (a chain past its window is left as is).
// Two grid points per iteration keep two pairs of LDS reads in flight.
template <class A, int K>
__device__ __forceinline__ void horner_upper(A (&acc)[K], const A (&rho)[K], const int (&hi_k)[K],
                                             const A* __restrict__ F, const A* __restrict__ G,
                                             int hi, int lo) {
  int g = hi;
  for (; g - 1 >= lo; g -= 2) {
    const A a0 = F[g] * G[g];
    const A a1 = F[g - 1] * G[g - 1];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      acc[k] = fma(acc[k], rho[k], g <= hi_k[k] ? a0 : (A)0);
      acc[k] = fma(acc[k], rho[k], g - 1 <= hi_k[k] ? a1 : (A)0);
    }
  }
  for (; g >= lo; --g) {
    const A av = F[g] * G[g];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = fma(acc[k], rho[k], g <= hi_k[k] ? av : (A)0);
  }
}

template <class A, int K>
__device__ __forceinline__ void horner_lower(A (&acc)[K], const A (&rho)[K], const int (&lo_k)[K],
                                             const A* __restrict__ F, const A* __restrict__ G,
                                             int hi, int lo) {
  int g = hi;
  for (; g - 1 >= lo; g -= 2) {
    const A a0 = F[g] * G[g];
    const A a1 = F[g - 1] * G[g - 1];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const A t0 = fma(acc[k], rho[k], a0);
      const A u0 = g >= lo_k[k] ? t0 : acc[k];
      const A t1 = fma(u0, rho[k], a1);
      acc[k] = g - 1 >= lo_k[k] ? t1 : u0;
    }
  }
  for (; g >= lo; --g) {
    const A av = F[g] * G[g];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const A t = fma(acc[k], rho[k], av);
      acc[k] = g >= lo_k[k] ? t : acc[k];
    }
  }
}

// Both bounds tested (groups whose windows have no common part).
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
// SM: the batch may carry the smoothed mass edge (a separate instance keeps
// the plain one's registers).  The smoothed edge can put an event's weights,
// or its sums, below FP32's range.  So in FP32 mode with delta_m > 0 the
// weights are formed as logs and stored as e^(ln w - L), L per (event,
// lambda): kLogHead32 above the largest log-weight L0 of the threads' first
// samples, so that weights up to e^(80 + kLogHead32) times those fit and
// ones more than e^(87 - kLogHead32) below them leave (they count only if
// every heavier sample's kernel sum is 0).  If a weight comes within e^18 of
// FP32's top, or all lie more than e^kLogHead32 below L0 (no first sample
// had weight), the event is transformed again with its largest weight at 1.
// L goes to wscale for k_event_final (0 elsewhere).
constexpr float kLogHead32 = 10.0f;

template <bool F32, bool SM>
__global__ __launch_bounds__(kZwBS) void k_event_zw(EventArgs a) {
  int e, b;
  if (!decode_item_lambda(a.E, a.B, e, b)) return;
  using CT = typename std::conditional<F32, float, double>::type;
  constexpr int NW = kZwBS / 64 + 1;
  __shared__ double red[4 * NW];
  const LamParams P = a.P[b];
  if (P.flag | a.flag_mono[b] | a.flag_range[b]) return;   // the final kernel reports it
  const double2* dtab = a.dtab + (size_t)b * a.g.n_t;
  const double2* inv = a.inv + (size_t)b * a.g.n_u;
  const double2* mt = a.mtab ? a.mtab + (size_t)b * (kMassPanels + 1) : nullptr;
  const int s0 = a.ev_samp_off[e];
  const int ns = a.ev_samp_off[e + 1] - s0;
  double* zb = a.zbuf + (size_t)b * a.S + s0;
  CT* wb = (CT*)a.wbuf + (size_t)b * a.S + s0;
  // weighted moments about a shift s near the data (the redshift of the
  // event's first sample from the inverse table, the same in every thread):
  // W1, W2, sum w (z - s), sum w (z - s)^2
  const double s = exp(invert_x(P, nullptr, inv, a.g, a.dl[s0], a.lndl[s0], 0)) - 1.0;
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  // software pipeline: the next sample's inputs are loaded while this one is
  // transformed (indices past the end read this event's first sample)
  auto in = [&](int j, double (&v)[6]) {
    const int q = s0 + (j < ns ? j : 0);
    v[0] = F32 ? 0.0 : a.dl[q];   // the FP32 transform uses ln d only
    v[1] = a.lndl[q]; v[2] = a.m1d[q];
    v[3] = a.m2d[q]; v[4] = a.lnm1d[q]; v[5] = a.lnm2d[q];
  };
  auto put = [&](int j, double z, CT wc) {
    zb[j] = z;
    wb[j] = wc;
    const double wd = (double)wc, t = z - s;
    m[0] += wd;
    m[1] += wd * wd;
    m[2] += wd * t;
    m[3] += wd * t * t;
  };
  double cur[6];
  in(threadIdx.x, cur);
  if constexpr (F32 && SM) {
    if (P.dm > 0.0) {
      auto lw_of = [&](const double (&v)[6], double& z) {
        double lw;
        sample_zw<true, true, true>(P, dtab, inv, a.g, v[0], v[1], v[2], v[3], v[4], v[5], z, lw,
                                    mt);
        return (float)lw;
      };
      double z0 = 0.0;
      const float l0 = threadIdx.x < ns ? lw_of(cur, z0) : -INFINITY;
      float L0 = (float)block_max<kZwBS>((double)l0, red);
      if (!(L0 > -INFINITY)) L0 = 0.0f;
      float L = L0 + kLogHead32;
      float top = l0 - L0;                      // the largest ln w - L0 seen
      if (threadIdx.x < ns) put(threadIdx.x, z0, __expf(fminf(l0 - L, 80.0f)));
      in(threadIdx.x + kZwBS, cur);
      for (int j = threadIdx.x + kZwBS; j < ns; j += kZwBS) {
        double nxt[6];
        in(j + kZwBS, nxt);
        double z;
        const float lw = lw_of(cur, z);
#pragma unroll
        for (int i = 0; i < 6; ++i) cur[i] = nxt[i];
        top = fmaxf(top, lw - L0);
        put(j, z, __expf(fminf(lw - L, 80.0f)));
      }
      const float M = (float)block_max<kZwBS>((double)top, red);
      if (M > -INFINITY && (M > 70.0f + kLogHead32 || M < -kLogHead32)) {
        // a weight near FP32's top, or all far below the first samples': again
        // with the largest weight at 1
        L = L0 + M;
#pragma unroll
        for (int i = 0; i < 4; ++i) m[i] = 0.0;
        for (int j = threadIdx.x; j < ns; j += kZwBS) {
          double v[6], z;
          in(j, v);
          const float lw = lw_of(v, z);
          put(j, z, __expf(lw - L));
        }
      }
      if (threadIdx.x == 0) a.wscale[(size_t)b * a.E + e] = (double)L;
    } else {
      if (threadIdx.x == 0) a.wscale[(size_t)b * a.E + e] = 0.0;
    }
  }
  if (!(F32 && SM) || !(P.dm > 0.0)) {
    for (int j = threadIdx.x; j < ns; j += kZwBS) {
      double nxt[6];
      in(j + kZwBS, nxt);
      double z, w;
      sample_zw<F32, SM>(P, dtab, inv, a.g, cur[0], cur[1], cur[2], cur[3], cur[4], cur[5], z, w,
                         mt);
#pragma unroll
      for (int i = 0; i < 6; ++i) cur[i] = nxt[i];
      put(j, z, (CT)w);
    }
  }
  block_reduce<kZwBS, 4, false>(m, red);
  const double W1 = m[0], W2 = m[1];
  if (!(W1 > 0.0)) {
    if (threadIdx.x == 0) a.hbuf[(size_t)b * a.E + e] = -1.0;
    return;
  }
  if (threadIdx.x == 0) {
    double var = 0.0;
    if (!(W1 * W1 - W2 <= 1e-12 * W1 * W1))
      var = fmax(m[3] - m[2] * (m[2] / W1), 0.0) / (W1 - W2 / W1);
    a.hbuf[(size_t)b * a.E + e] = fmax(sqrt(var) * pow(W1 * W1 / W2, -0.2), 2.0 * a.g.dz);
  }
}

// ---------------------------------------------------------------------------
template <bool F32, bool COMPL>
__device__ __forceinline__ void event_smooth(const EventArgs& a) {
  constexpr int K = kGroupK;
  constexpr int BS = kSmBS;
  int u, b;
  if (!decode_item_lambda(a.U, a.B, u, b)) return;
  using CT = typename std::conditional<F32, float, double>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NW = BS / 64 + 1;
  __shared__ double red[4 * NW];
  double* part = a.part + (size_t)b * a.U + u;
  const int e = a.unit_event[u];
  const LamParams P = a.P[b];
  const double h = a.hbuf[(size_t)b * a.E + e];
  if ((P.flag | a.flag_mono[b] | a.flag_range[b]) || !(h > 0.0)) {
    if (threadIdx.x == 0) {
      *part = 0.0;
      if (a.count) a.pcount[(size_t)b * a.U + u] = 0;
    }
    return;
  }
  const int p0 = a.ev_slot_off[e];
  const int np = a.ev_slot_off[e + 1] - p0;
  const double dz = a.g.dz;
  const double T = a.trunc;
  const double inv_h2 = 1.0 / (h * h);
  const double inv_dz = 1.0 / dz;
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
        const double lo_d = fmax(ceil((zk[k] - T * h - a.g.z_lo) * inv_dz), 0.0);
        const double hi_d = fmin(floor((zk[k] + T * h - a.g.z_lo) * inv_dz), (double)(a.g.n_z - 1));
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
  // Horner ratios rho_k = exp(dz (z_k - z_c) / h^2); a chain without a window
  // (zero weight, or outside the grid) still runs through the shared bulk:
  // rho = 0 keeps it finite (the ratio of a far-away sample would overflow)
  // and it is left out of the sum
  CT rho[K];
#pragma unroll
  for (int k = 0; k < K; ++k) rho[k] = (CT)0;
  int c = 0;
  double mloc = 0.0, dloc = 0.0;
  if (zn > 0.0) {
    const double cd = fmin(fmax(rint((zsum / zn - a.g.z_lo) * inv_dz), -4.0 * a.g.n_z), 8.0 * a.g.n_z);
    c = (int)cd;
    mloc = (double)max(hi_u - c, c - lo_u);
    const double zc0 = a.g.z_lo + cd * dz;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (klo[k] <= khi[k]) {
        const double delta = zk[k] - zc0;
        dloc = fmax(dloc, fabs(delta));
        rho[k] = F32 ? (CT)__expf((float)(dz * delta * inv_h2)) : (CT)exp(dz * delta * inv_h2);
      }
    }
  }
  // unit bounds, chain range and the largest |z_k - centre| (rounded up to
  // FP32 and compared as its bit pattern, which orders non-negative floats)
  float dl32 = (float)dloc;
  if ((double)dl32 < dloc) dl32 = __int_as_float(__float_as_int(dl32) + 1);
  __shared__ int redi[4 * (BS / 64)];
  int mx[4] = {lo_u <= hi_u ? -lo_u : -(1 << 30), lo_u <= hi_u ? hi_u : -(1 << 30), (int)mloc,
               __float_as_int(dl32)};
  block_max_i32<BS, 4>(mx, redi);
  const int A_lo = max(-mx[0], 0);
  const int A_hi = min(mx[1], a.g.n_z - 1);
  const int M = mx[2];                   // |g - c| <= M over every group window of the unit
  const double dmax = (double)__int_as_float(mx[3]);

  // Horner's partial sums are the kernel values times rho^(c - lo) / C: at
  // most exp(M dz |delta| / h^2 + delta^2 / 2h^2) away from the true values
  const double ebound = (double)M * dz * dmax * inv_h2 + 0.5 * dmax * dmax * inv_h2;
  const bool horner_ok = ebound < (F32 ? 60.0 : 600.0);
  const double zc = a.g.z_lo + (double)c * dz;
  const double cir = has ? a.grp_c[gi] : 0.0;
  // c_ir w_k C_k rho_k^(lo_k - c), the factor of chain k, formed after the
  // sweep from z_k and w_k read again, which keeps the registers low enough
  // for four waves per SIMD
  auto chain_coef = [&](int k, double zkk, double wkk) {
    const double delta = zkk - zc;
    const double x = -0.5 * delta * delta * inv_h2 + (double)(klo[k] - c) * dz * delta * inv_h2;
    return cir * wkk * (F32 ? (double)__expf((float)x) : exp(x));
  };
  CT acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = (CT)0;
  double total = 0.0, npts = 0.0;
  if (a.count) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (klo[k] <= khi[k]) npts += (double)(khi[k] - klo[k] + 1);
  }

  // G_m = exp(-m^2 dz^2 / 2h^2), m in [-M, M], and the F slice share the
  // workgroup's LDS: G takes its 2M + 1 entries at the end, the slice the
  // rest, as long as every pixel row of the event keeps two slots
  const int total_elems = (sm_fbytes(F32) + kSmGCap * (int)sizeof(CT)) / (int)sizeof(CT);
  const int gcount = 2 * M + 1;
  const int f_elems = total_elems - gcount;
  const bool gtab = gcount >= 1 && f_elems >= 2 * (np > 0 ? np : 1);
  CT* Gt = (CT*)smem + (gtab ? f_elems : 0);
  if (gtab) {
    for (int q = threadIdx.x; q < gcount; q += BS) {
      const double x = (double)(q - M) * dz;
      Gt[q] = (CT)exp(-0.5 * x * x * inv_h2);
    }
  }
  // Slice of the event's F rows in LDS, row stride Ls = L + 1 (odd: spreads the
  // banks).  L is a multiple of 64 when a row of 64 fits, so that one wave
  // stages one row segment per instruction (row base uniform per wave);
  // otherwise a power of two W < 64 and 64 / W rows per wave instruction.
  int L, lgW;
  {
    const int cap = max(f_elems / (np > 0 ? np : 1) - 1, 1);   // >= 1 whenever gtab
    if (cap >= 64) {
      L = cap & ~63;
      lgW = 6;
    } else {
      lgW = 31 - __clz(cap);
      L = 1 << lgW;
    }
  }
  const int Ls = L + 1;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr int NWV = BS / 64;

  if (gtab && A_lo <= A_hi && horner_ok) {
    const CT* gz = F32 ? (const CT*)(a.gz32 + (size_t)b * a.g.n_z)
                       : (const CT*)(a.gz64 + (size_t)b * a.g.n_z);
    const CT* nzt = F32 ? (const CT*)a.nz32 : (const CT*)a.nz64;
    // with incompleteness F = n_r gz + (1 - P_r) gzb (gz already carries f_R)
    const CT* gzc = COMPL ? (F32 ? (const CT*)(a.gzb32 + (size_t)b * a.g.n_z)
                                 : (const CT*)(a.gzb64 + (size_t)b * a.g.n_z))
                          : nullptr;
    const CT* mzt = COMPL ? (F32 ? (const CT*)a.mz32 : (const CT*)a.mz64) : nullptr;
    for (int s_hi = A_hi; s_hi >= A_lo; s_hi -= L) {
      const int s_lo = max(s_hi - L + 1, A_lo);
      const int len = s_hi - s_lo + 1;
      __syncthreads();   // the previous slice is consumed (and G is written)
      // F_r(z_g) = n_r(z_g) g(z_g); UR independent loads in flight per thread.
      // The batch's row indices are read first (one wait), then its UR row
      // segments are loaded together.
      constexpr int UR = (COMPL && !F32) ? 4 : 8;   // FP64 with the completion rows: 2 x 4 loads
      if (lgW == 6) {
        // a wave takes UR rows (uniform row index: scalar base address) and
        // sweeps the slice 64 points at a time
        for (int pb = wv; pb < np; pb += NWV * UR) {
          int rr[UR];
#pragma unroll
          for (int r = 0; r < UR; ++r) {
            const int p = pb + r * NWV;
            rr[r] = p < np ? a.slot_row[p0 + p] : 0;
          }
          const CT* rp[UR];
          const CT* mp[UR];
#pragma unroll
          for (int r = 0; r < UR; ++r) {
            const size_t off = (size_t)__builtin_amdgcn_readfirstlane(rr[r]) * a.g.n_z;
            rp[r] = nzt + off;
            mp[r] = COMPL ? mzt + off : nullptr;
          }
          for (int q0 = 0; q0 < len; q0 += 64) {
            const int q = q0 + lane;
            const bool qv = q < len;
            const int gg = s_lo + (qv ? q : 0);
            const CT gv = gz[gg];
            CT v[UR], mv[UR];
            // both rows' segments are loaded together (one wait)
#pragma unroll
            for (int r = 0; r < UR; ++r) {
              const bool ok = pb + r * NWV < np;
              v[r] = ok ? rp[r][gg] : (CT)0;
              if (COMPL) mv[r] = ok ? mp[r][gg] : (CT)0;
            }
            if (COMPL) {
              const CT gc = gzc[gg];
#pragma unroll
              for (int r = 0; r < UR; ++r) v[r] = v[r] * gv + mv[r] * gc;
            }
#pragma unroll
            for (int r = 0; r < UR; ++r) {
              const int p = pb + r * NWV;
              if (p < np && qv) ((CT*)smem)[p * Ls + q] = COMPL ? v[r] : v[r] * gv;
            }
          }
        }
      } else {
        const int RPW = 64 >> lgW;                 // rows per wave instruction
        const int q = lane & ((1 << lgW) - 1);
        const int sub = lane >> lgW;
        const bool qv = q < len;
        const int gg = s_lo + (qv ? q : 0);
        const CT gv = gz[gg];
        const CT gc = COMPL ? gzc[gg] : (CT)0;
        for (int pb = wv * RPW + sub; pb < np; pb += NWV * RPW * UR) {
          int rr[UR];
#pragma unroll
          for (int r = 0; r < UR; ++r) {
            const int p = pb + r * NWV * RPW;
            rr[r] = p < np ? a.slot_row[p0 + p] : 0;
          }
          CT v[UR], mv[UR];
#pragma unroll
          for (int r = 0; r < UR; ++r) {
            const int p = pb + r * NWV * RPW;
            v[r] = p < np ? nzt[(size_t)rr[r] * a.g.n_z + gg] : (CT)0;
            if (COMPL) mv[r] = p < np ? mzt[(size_t)rr[r] * a.g.n_z + gg] : (CT)0;
          }
          if (COMPL) {
#pragma unroll
            for (int r = 0; r < UR; ++r) v[r] = v[r] * gv + mv[r] * gc;
          }
#pragma unroll
          for (int r = 0; r < UR; ++r) {
            const int p = pb + r * NWV * RPW;
            if (p < np && qv) ((CT*)smem)[p * Ls + q] = COMPL ? v[r] : v[r] * gv;
          }
        }
      }
      __syncthreads();
      if (has && lo_u <= hi_u) {
        const int hi = min(hi_u, s_hi), lo = max(lo_u, s_lo);
        if (lo <= hi) {
          const CT* Fp = (const CT*)smem + a.grp_slot[gi] * Ls - s_lo;
          const CT* Gp = Gt + (M - c);
          if (lo_i <= hi_i) {
            // upper edge (masked), shared bulk, lower edge (masked)
            horner_upper<CT, K>(acc, rho, khi, Fp, Gp, hi, max(lo, hi_i + 1));
            horner_span<CT, K>(acc, rho, Fp, Gp, min(hi, hi_i), max(lo, lo_i));
            horner_lower<CT, K>(acc, rho, klo, Fp, Gp, min(hi, lo_i - 1), lo);
          } else {
            horner_masked<CT, K>(acc, rho, klo, khi, Fp, Gp, hi, lo);
          }
        }
      }
    }
    asm volatile("" ::: "memory");   // read z_k, w_k again
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (klo[k] <= khi[k]) {
        const double ck = chain_coef(k, zb[first + k], (double)wb[first + k]);
        total += ck * (double)acc[k];
      }
    }
  } else if (A_lo <= A_hi && has) {
    // fallback (windows too wide for the tables or the chain range): direct sums
    const double* gzb = a.gz64 + (size_t)b * a.g.n_z;
    const double* gzcb = COMPL ? a.gzb64 + (size_t)b * a.g.n_z : nullptr;
    const size_t row = (size_t)a.slot_row[p0 + a.grp_slot[gi]] * a.g.n_z;
    asm volatile("" ::: "memory");   // read z_k, w_k again
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (klo[k] > khi[k]) continue;
      const double zkk = zb[first + k];
      double sacc = 0.0;
      for (int g = klo[k]; g <= khi[k]; ++g) {
        const double x = (a.g.z_lo + (double)g * dz - zkk);
        const double F = COMPL ? a.nz64[row + g] * gzb[g] + a.mz64[row + g] * gzcb[g]
                               : a.nz64[row + g] * gzb[g];
        sacc += exp(-0.5 * x * x * inv_h2) * F;
      }
      total += cir * (double)wb[first + k] * sacc;
    }
  }
  double fin[1] = {total};
  block_reduce<BS, 1, false>(fin, red);
  if (threadIdx.x == 0) *part = fin[0];
  if (a.count) {   // profiling: the pairs this workgroup evaluated, summed after the kernel
    long long n = (long long)npts;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
    __shared__ long long redc[NWV];
    if (lane == 0) redc[wv] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long t = 0;
#pragma unroll
      for (int k = 0; k < NWV; ++k) t += redc[k];
      a.pcount[(size_t)b * a.U + u] = t;
    }
  }
}

__global__ __launch_bounds__(kSmBS) __attribute__((amdgpu_waves_per_eu(4)))
void k_event_smooth64(EventArgs a) { event_smooth<false, false>(a); }

__global__ __launch_bounds__(kSmBS) __attribute__((amdgpu_waves_per_eu(4)))
void k_event_smooth64c(EventArgs a) { event_smooth<false, true>(a); }

__global__ __launch_bounds__(kSmBS) __attribute__((amdgpu_waves_per_eu(4)))
void k_event_smooth32c(EventArgs a) { event_smooth<true, true>(a); }

__global__ __launch_bounds__(kSmBS) __attribute__((amdgpu_waves_per_eu(4)))
void k_event_smooth32(EventArgs a) { event_smooth<true, false>(a); }

// profiling: the pair counts of one launch into the context's counter
__global__ __launch_bounds__(256) void k_count_sum(const long long* __restrict__ pc, long long n,
                                                   unsigned long long* __restrict__ count) {
  long long t = 0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    t += pc[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  __shared__ long long r[4];
  if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(count, (unsigned long long)(r[0] + r[1] + r[2] + r[3]));
}

// ---------------------------------------------------------------------------
namespace {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Number of leading lanes (from lane 0) whose flag is set.
__device__ __forceinline__ int leading_set(bool f) {
  const unsigned long long m = __ballot(f);
  return (~m == 0ull) ? 64 : __builtin_ctzll(~m);
}

}  // namespace

// Binned data sets (Sect. 2.3): per pixel slot and lambda, n_bins equal-width
// bins over the slot's redshift range; a bin's point sits at its centre and
// carries the summed weight of its samples.  One wave per (slot, lambda)
// reads the slot's samples in distance order (pix_idx), which is redshift
// order since d_L^gw increases, 64 at a time: the bins along the lanes never
// decrease, so a segmented scan over the lanes sums each bin's run and its
// last lane adds the run to the bin's accumulator in LDS (runs that continue
// into the next 64 samples add in turn).  A fixed order, no atomics.
template <bool F32>
__global__ __launch_bounds__(kBinBS) void k_event_bin(EventArgs a) {
  using CT = typename std::conditional<F32, float, double>::type;
  constexpr int SPB = kBinBS / 64;                        // slots per workgroup
  extern __shared__ double bacc[];                        // [SPB][n_bins]
  int it, b;
  if (!decode_item_lambda((a.n_slots + SPB - 1) / SPB, a.B, it, b)) return;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int p = it * SPB + wv;
  const int lane = threadIdx.x & 63;
  if (p >= a.n_slots) return;
  if (a.P[b].flag | a.flag_mono[b] | a.flag_range[b]) return;
  const int j0 = a.pix_off[p], n = a.pix_off[p + 1] - j0;
  const int* idx = a.pix_idx + j0;
  const double* zb = a.zbuf + (size_t)b * a.S;
  const CT* wb = (const CT*)a.wbuf + (size_t)b * a.S;
  const int nb = a.n_bins;
  double* acc = bacc + (size_t)wv * nb;
  for (int q = lane; q < nb; q += 64) acc[q] = 0.0;
  const double zlo = zb[idx[0]], zhi = zb[idx[n - 1]];
  const double width = (zhi - zlo) / (double)nb;
  wave_sync();
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int j = c0 + lane;
    const bool valid = j < n;
    int bin = 1 << 30;
    double s = 0.0;
    if (valid) {
      const int q = idx[j];
      s = (double)wb[q];
      bin = 0;
      if (width > 0.0) {
        const double f = floor((zb[q] - zlo) / width);
        bin = f >= (double)(nb - 1) ? nb - 1 : (int)f;
      }
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double u = __shfl_up(s, o, 64);
      const int bu = __shfl_up(bin, o, 64);
      if (lane >= o && bu == bin) s += u;
    }
    const int bn = __shfl_down(bin, 1, 64);
    if (valid && (lane == 63 || bn != bin)) acc[bin] += s;
    wave_sync();
  }
  const size_t base = (size_t)b * a.n_slots * nb + (size_t)p * nb;
  for (int q = lane; q < nb; q += 64) {
    a.bz[base + q] = width > 0.0 ? zlo + ((double)q + 0.5) * width : zlo;
    ((CT*)a.bw)[base + q] = (CT)acc[q];
  }
}

// ---------------------------------------------------------------------------
// Epanechnikov kernel sums (Sect. 2.3's compact option): with
// K = 3/(4 a h) (1 - u^2), u = (z_g - z_j) / (a h), a = sqrt(5), and W = a h / dz,
//   sum_{|g - x_j| <= W} tau_g F(z_g) (1 - (g - x_j)^2 / W^2)
//     = S0 - (S2 - 2 d S1 + d^2 S0) / W^2,   S_m = sum tau F (g - m0)^m,
// d = x_j - m0, over the sample's window: each S_m is a difference of two
// prefix sums, so a point costs O(1) whatever its window.  One wave per
// (pixel slot, lambda) walks the slot's points (samples, or bins) in redshift
// order in chunks whose windows fit kEpCap grid points: it stages tau F over
// the chunk's range in LDS (the grid factor already carries tau), forms the
// three prefix sums in FP64 (per lane over a contiguous block, then a scan
// across lanes), and evaluates the chunk's points, loading the next points
// while it evaluates these.  The origin m0 is the chunk's middle point, which
// keeps (g - m0)^2 small against the window.  The slot's sum times c_ir is
// its partial; k_event_final adds an event's slots in order.
template <bool F32>
__global__ __launch_bounds__(kEpBS) void k_event_epan(EventArgs a) {
  using CT = typename std::conditional<F32, float, double>::type;
  constexpr int NWV = kEpBS / 64;
  constexpr int PER = kEpCap / 64;
  int it, b;
  if (!decode_item_lambda((a.n_slots + NWV - 1) / NWV, a.B, it, b)) return;
  __shared__ double q0[NWV][kEpCap], q1[NWV][kEpCap], q2[NWV][kEpCap];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int p = it * NWV + wv;
  if (p >= a.n_slots) return;
  const int e = a.slot_event[p];
  double* part = a.part + (size_t)b * a.n_slots + p;
  const LamParams P = a.P[b];
  const double h = a.hbuf[(size_t)b * a.E + e];
  if ((P.flag | a.flag_mono[b] | a.flag_range[b]) || !(h > 0.0)) {
    if (lane == 0) {
      *part = 0.0;
      if (a.count) a.pcount[(size_t)b * a.n_slots + p] = 0;
    }
    return;
  }
  const int nz = a.g.n_z;
  const double W = kEpanScale * h * a.g.inv_dz;
  const double inv_W2 = 1.0 / (W * W);
  const CT* gz = F32 ? (const CT*)(a.gz32 + (size_t)b * nz) : (const CT*)(a.gz64 + (size_t)b * nz);
  const CT* row = (F32 ? (const CT*)a.nz32 : (const CT*)a.nz64) + (size_t)a.slot_row[p] * nz;
  // tau F at node g (the grid factor carries tau; with incompleteness
  // F = n_r gz + (1 - P_r) gzb)
  const CT* mrow = a.mz64 ? (F32 ? (const CT*)a.mz32 : (const CT*)a.mz64) + (size_t)a.slot_row[p] * nz
                          : nullptr;
  const CT* gzc = a.mz64 ? (F32 ? (const CT*)(a.gzb32 + (size_t)b * nz)
                                : (const CT*)(a.gzb64 + (size_t)b * nz))
                         : nullptr;
  auto stage = [&](int g) {
    return mrow ? (double)(row[g] * gz[g] + mrow[g] * gzc[g]) : (double)(row[g] * gz[g]);
  };
  const bool binned = a.n_bins > 0;
  const double* zsrc = binned ? a.bz + (size_t)b * a.n_slots * a.n_bins : a.zbuf + (size_t)b * a.S;
  const CT* wsrc = binned ? (const CT*)a.bw + (size_t)b * a.n_slots * a.n_bins
                          : (const CT*)a.wbuf + (size_t)b * a.S;
  int j0, n;
  const int* idx = nullptr;
  if (binned) {
    j0 = p * a.n_bins;
    n = a.n_bins;
  } else {
    j0 = a.pix_off[p];
    n = a.pix_off[p + 1] - j0;
    idx = a.pix_idx + j0;
  }
  auto pos = [&](int j) { return idx ? idx[j] : j0 + j; };
  auto xat = [&](int j) { return (zsrc[pos(j)] - a.g.z_lo) * a.g.inv_dz; };
  double* Q0 = q0[wv];
  double* Q1 = q1[wv];
  double* Q2 = q2[wv];
  double acc = 0.0;
  long long npts = 0;
  // tau F over [glo, ghi] (at most kEpCap points) into LDS and its three
  // prefix sums about mid
  auto build_prefix = [&](int glo, int ghi, int mid) {
    const int L = ghi - glo + 1;
    wave_sync();                 // earlier prefix sums are read
    for (int q = lane; q < L; q += 64) Q0[q] = stage(glo + q);
    wave_sync();
    // per lane: a contiguous block of <= PER points
    const int per = (L + 63) >> 6;
    const int qa = min(lane * per, L), qb = min(qa + per, L);
    double f[PER];
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      f[i] = qa + i < qb ? Q0[qa + i] : 0.0;
      const double t = (double)(qa + i + glo - mid);
      t0 += f[i];
      t1 += f[i] * t;
      t2 += f[i] * t * t;
    }
    // exclusive scan of the lane totals across the wave (lane order)
    double c0 = t0, c1 = t1, c2 = t2;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double u0 = __shfl_up(c0, o, 64), u1 = __shfl_up(c1, o, 64), u2 = __shfl_up(c2, o, 64);
      if (lane >= o) {
        c0 += u0;
        c1 += u1;
        c2 += u2;
      }
    }
    c0 -= t0;
    c1 -= t1;
    c2 -= t2;
    wave_sync();                 // every lane has read its block of F
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (qa + i < qb) {
        const double t = (double)(qa + i + glo - mid);
        c0 += f[i];
        c1 += f[i] * t;
        c2 += f[i] * t * t;
        Q0[qa + i] = c0;
        Q1[qa + i] = c1;
        Q2[qa + i] = c2;
      }
    }
    wave_sync();
  };
  // one point's weight times its window sum, from the prefix sums
  auto eval = [&](double zk, double wk, int glo, int ghi, int mid) {
    if (!(wk > 0.0)) return;
    const double xk = (zk - a.g.z_lo) * a.g.inv_dz;
    const int lk = (int)fmax(ceil(xk - W), (double)glo);
    const int hk = (int)fmin(floor(xk + W), (double)ghi);
    if (lk > hk) return;
    const int qh = hk - glo, ql = lk - 1 - glo;
    const double S0 = Q0[qh] - (ql >= 0 ? Q0[ql] : 0.0);
    const double S1 = Q1[qh] - (ql >= 0 ? Q1[ql] : 0.0);
    const double S2 = Q2[qh] - (ql >= 0 ? Q2[ql] : 0.0);
    const double d = xk - (double)mid;
    const double A = S0 - (S2 - 2.0 * d * S1 + d * d * S0) * inv_W2;
    acc += wk * fmax(A, 0.0);
    npts += 1;
  };
  int j = 0;
  if (n <= 128) {
    // the common case: two points per lane in registers, loaded at once, and
    // (when their windows fit kEpCap points) one chunk
    double zr[2], wr[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int k = lane + 64 * r;
      zr[r] = 0.0;
      wr[r] = 0.0;
      if (k < n) {
        const int q = pos(k);
        zr[r] = zsrc[q];
        wr[r] = (double)wsrc[q];
      }
    }
    const double zfirst = __shfl(zr[0], 0, 64);
    const double zlast = __shfl(n > 64 ? zr[1] : zr[0], (n - 1) & 63, 64);
    const double lo0 = ceil((zfirst - a.g.z_lo) * a.g.inv_dz - W);
    const int glo = (int)fmax(lo0, 0.0);
    const int ghi = (int)fmin(floor((zlast - a.g.z_lo) * a.g.inv_dz + W), (double)(nz - 1));
    if (lo0 > (double)(nz - 1) || ghi < glo) {
      j = n;                     // no grid point in any window
    } else if (ghi - glo + 1 <= kEpCap) {
      const int mid = glo + ((ghi - glo + 1) >> 1);
      build_prefix(glo, ghi, mid);
#pragma unroll
      for (int r = 0; r < 2; ++r)
        if (lane + 64 * r < n) eval(zr[r], wr[r], glo, ghi, mid);
      j = n;
    }
  }
  while (j < n) {
    const double lo0 = ceil(xat(j) - W);
    if (lo0 > (double)(nz - 1)) break;                   // this point and the rest lie above the grid
    const int glo = (int)fmax(lo0, 0.0);
    const double cap_hi = (double)(glo + kEpCap - 1);
    // the chunk ends at the first point from j on whose window ends past
    // glo + kEpCap - 1 (the window ends rise with the point): a 64-way search
    auto fits = [&](int k) { return fmin(floor(xat(k) + W), (double)(nz - 1)) <= cap_hi; };
    int lo = j, hi = n;                                  // the end lies in [lo, hi]
    while (hi - lo > 64) {
      const int step = (hi - lo + 63) / 64;
      const int k = lo + lane * step;
      const int cnt = leading_set(k < hi && fits(k));
      if (cnt == 0) {
        hi = lo;
        break;
      }
      const int last_ok = lo + (cnt - 1) * step;
      hi = min(hi, last_ok + step);
      lo = last_ok + 1;
    }
    int j1 = lo;
    if (hi > lo) j1 = lo + leading_set(lo + lane < hi && fits(lo + lane));
    if (j1 == j) {
      // a window wider than a chunk: a direct sum, the wave across its points
      const double xj = xat(j);
      const int g0 = (int)fmax(ceil(xj - W), 0.0), g1 = (int)fmin(floor(xj + W), (double)(nz - 1));
      double t = 0.0;
      for (int g = g0 + lane; g <= g1; g += 64) {
        const double u = ((double)g - xj) / W;
        t += stage(g) * (1.0 - u * u);
      }
      t = wave_sum(t);
      if (lane == 0) {
        acc += (double)wsrc[pos(j)] * t;
        npts += 1;
      }
      ++j;
      continue;
    }
    const int ghi = (int)fmin(floor(xat(j1 - 1) + W), (double)(nz - 1));
    if (ghi < glo) {             // no grid point in any window of the chunk
      j = j1;
      continue;
    }
    const int mid = glo + ((ghi - glo + 1) >> 1);
    build_prefix(glo, ghi, mid);
    // the chunk's points, the next point's loads issued before this one's sums
    int k = j + lane;
    double zc = 0.0, wc = 0.0;
    if (k < j1) {
      const int q = pos(k);
      zc = zsrc[q];
      wc = (double)wsrc[q];
    }
    while (k < j1) {
      const int kn = k + 64;
      double zn = 0.0, wn = 0.0;
      if (kn < j1) {
        const int q = pos(kn);
        zn = zsrc[q];
        wn = (double)wsrc[q];
      }
      eval(zc, wc, glo, ghi, mid);
      k = kn;
      zc = zn;
      wc = wn;
    }
    j = j1;
  }
  const double st = wave_sum(acc);
  if (a.count) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) npts += __shfl_xor(npts, o, 64);
  }
  if (lane == 0) {
    *part = a.slot_c[p] * st;
    if (a.count) a.pcount[(size_t)b * a.n_slots + p] = npts;
  }
}

// ---------------------------------------------------------------------------
// The 3D kernel (Sect. 2.2): one Gaussian KDE of the event's samples in
// (z, u, v), (u, v) a flat sky chart, with bandwidth matrix H = weighted
// covariance x n_eff^(-2/7), evaluated at each pixel centre (u_k, v_k).  For
// a pixel offset dO = (u_k - u_j, v_k - v_j) the 3-D Gaussian factors as
//   N3 = N2(dO; H_OO) N(z_g; z_j + B dO, s),  B = H_zO H_OO^-1,
//   s^2 = H_zz - B H_Oz,
// so each (pixel, sample) pair is a point at z_j + B dO with weight
// w_j N2(dO; H_OO) in the pixel's 1-D sum, every point of the event with the
// one width s: the many-1D smoothing kernel then sums them unchanged.
//
// k_event_cov3d: per (event, lambda), the weighted moments of (z, u, v) about
// the first sample in one pass, then H, B, s and H_OO^-1 (hbuf takes s, or
// -1 when H is not positive definite or the weights vanish).
template <bool F32>
__global__ __launch_bounds__(kZwBS) void k_event_cov3d(EventArgs a) {
  using CT = typename std::conditional<F32, float, double>::type;
  constexpr int NW = kZwBS / 64 + 1;
  __shared__ double red[11 * NW];
  int e, b;
  if (!decode_item_lambda(a.E, a.B, e, b)) return;
  if (a.P[b].flag | a.flag_mono[b] | a.flag_range[b]) return;
  double* hp = a.hbuf + (size_t)b * a.E + e;
  if (!(*hp > 0.0)) return;                             // no weight in the event
  const int s0 = a.ev_samp_off[e], ns = a.ev_samp_off[e + 1] - s0;
  const double* zb = a.zbuf + (size_t)b * a.S + s0;
  const CT* wb = (const CT*)a.wbuf + (size_t)b * a.S + s0;
  const double* su = a.su + s0;
  const double* sv = a.sv + s0;
  const double z0 = zb[0], u0 = su[0], v0 = sv[0];
  double m[11];
#pragma unroll
  for (int i = 0; i < 11; ++i) m[i] = 0.0;
  for (int j = threadIdx.x; j < ns; j += kZwBS) {
    const double w = (double)wb[j];
    const double dz = zb[j] - z0, du = su[j] - u0, dv = sv[j] - v0;
    m[0] += w;
    m[1] += w * w;
    m[2] += w * dz;
    m[3] += w * du;
    m[4] += w * dv;
    m[5] += w * dz * dz;
    m[6] += w * du * du;
    m[7] += w * dv * dv;
    m[8] += w * dz * du;
    m[9] += w * dz * dv;
    m[10] += w * du * dv;
  }
  block_reduce<kZwBS, 11, false>(m, red);
  if (threadIdx.x != 0) return;
  const double W1 = m[0], W2 = m[1];
  double* p3 = a.p3 + ((size_t)b * a.E + e) * 8;
  if (!(W1 > 0.0) || W1 * W1 - W2 <= 1e-12 * W1 * W1) {
    *hp = -1.0;
    return;
  }
  const double mz = m[2] / W1, mu = m[3] / W1, mv = m[4] / W1;
  const double den = W1 - W2 / W1;
  const double f = pow(W1 * W1 / W2, -2.0 / 7.0) / den;
  const double Hzz = (m[5] - W1 * mz * mz) * f, Huu = (m[6] - W1 * mu * mu) * f;
  const double Hvv = (m[7] - W1 * mv * mv) * f, Hzu = (m[8] - W1 * mz * mu) * f;
  const double Hzv = (m[9] - W1 * mz * mv) * f, Huv = (m[10] - W1 * mu * mv) * f;
  const double det = Huu * Hvv - Huv * Huv;
  if (!(Hzz > 0.0 && det > 0.0)) {
    *hp = -1.0;
    return;
  }
  const double iuu = Hvv / det, iuv = -Huv / det, ivv = Huu / det;
  const double Bu = Hzu * iuu + Hzv * iuv, Bv = Hzu * iuv + Hzv * ivv;
  const double s2 = Hzz - (Bu * Hzu + Bv * Hzv);
  if (!(s2 > 0.0)) {
    *hp = -1.0;
    return;
  }
  p3[0] = Bu;
  p3[1] = Bv;
  p3[2] = iuu;
  p3[3] = iuv;
  p3[4] = ivv;
  p3[5] = -log(2.0 * M_PI * sqrt(det));
  *hp = sqrt(s2);
}

// k_event_expand3d: per (event, lambda), every (pixel, sample) point: its
// redshift z_j + B dO and weight w_j N2(dO; H_OO), 0 where the sky part of the
// quadratic form exceeds T^2; pixel-major, so each pixel's points follow the
// samples' group order (the groups of the 1-D sums stay consecutive).
template <bool F32>
__global__ __launch_bounds__(kZwBS) void k_event_expand3d(EventArgs a) {
  using CT = typename std::conditional<F32, float, double>::type;
  int e, b;
  if (!decode_item_lambda(a.E, a.B, e, b)) return;
  if (a.P[b].flag | a.flag_mono[b] | a.flag_range[b]) return;
  if (!(a.hbuf[(size_t)b * a.E + e] > 0.0)) return;
  const double* p3 = a.p3 + ((size_t)b * a.E + e) * 8;
  const double Bu = p3[0], Bv = p3[1], iuu = p3[2], iuv = p3[3], ivv = p3[4], lnn = p3[5];
  const double T2 = a.trunc * a.trunc;
  const int s0 = a.ev_samp_off[e], ns = a.ev_samp_off[e + 1] - s0;
  const int k0 = a.ev_slot_off[e], np = a.ev_slot_off[e + 1] - k0;
  const double* zb = a.zbuf + (size_t)b * a.S + s0;
  const CT* wb = (const CT*)a.wbuf + (size_t)b * a.S + s0;
  const double* su = a.su + s0;
  const double* sv = a.sv + s0;
  double* zo = a.z3 + (size_t)b * a.V + a.virt_off[e];
  CT* wo = (CT*)a.w3 + (size_t)b * a.V + a.virt_off[e];
  for (int k = 0; k < np; ++k) {
    const double uk = a.pu[k0 + k], vk = a.pv[k0 + k];
    for (int j = threadIdx.x; j < ns; j += kZwBS) {
      const double du = uk - su[j], dv = vk - sv[j];
      const double q = iuu * du * du + 2.0 * iuv * du * dv + ivv * dv * dv;
      const double w = q <= T2 ? (double)wb[j] * exp(lnn - 0.5 * q) : 0.0;
      zo[(size_t)k * ns + j] = zb[j] + Bu * du + Bv * dv;
      wo[(size_t)k * ns + j] = (CT)w;
    }
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
    const double norm = a.shape == kShapeEpanechnikov ? 0.75 / kEpanScale : kInvSqrt2Pi;
    const double I = h > 0.0 ? s * norm / h : 0.0;
    out = I > 0.0 ? log(I) + (a.wscale ? a.wscale[(size_t)b * a.E + e] : 0.0) : -INFINITY;
  }
  a.lnI[(size_t)b * a.E + e] = out;
}

// ---------------------------------------------------------------------------
hipError_t launch_events(const EventArgs& a, const EventArgs& kern, bool f32, hipStream_t st,
                         hipEvent_t t0, hipEvent_t t1) {
  const long long bz = item_lambda_blocks(a.E, a.B);
  hipError_t err;
  if (a.mtab) {
    if (f32) k_event_zw<true, true><<<(unsigned)bz, kZwBS, 0, st>>>(a);
    else k_event_zw<false, true><<<(unsigned)bz, kZwBS, 0, st>>>(a);
  } else {
    if (f32) k_event_zw<true, false><<<(unsigned)bz, kZwBS, 0, st>>>(a);
    else k_event_zw<false, false><<<(unsigned)bz, kZwBS, 0, st>>>(a);
  }
  if (a.V > 0) {
    if (f32) {
      k_event_cov3d<true><<<(unsigned)bz, kZwBS, 0, st>>>(a);
      k_event_expand3d<true><<<(unsigned)bz, kZwBS, 0, st>>>(a);
    } else {
      k_event_cov3d<false><<<(unsigned)bz, kZwBS, 0, st>>>(a);
      k_event_expand3d<false><<<(unsigned)bz, kZwBS, 0, st>>>(a);
    }
  }
  if (a.n_bins > 0) {
    const long long bb = item_lambda_blocks((a.n_slots + kBinBS / 64 - 1) / (kBinBS / 64), a.B);
    const size_t lds = (size_t)(kBinBS / 64) * a.n_bins * sizeof(double);
    const void* kb = f32 ? (const void*)k_event_bin<true> : (const void*)k_event_bin<false>;
    err = hipFuncSetAttribute(kb, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    if (f32) k_event_bin<true><<<(unsigned)bb, kBinBS, lds, st>>>(a);
    else k_event_bin<false><<<(unsigned)bb, kBinBS, lds, st>>>(a);
  }
  if (kern.shape == kShapeEpanechnikov) {
    const long long be = item_lambda_blocks((a.n_slots + kEpBS / 64 - 1) / (kEpBS / 64), a.B);
    if (t0 && (err = hipEventRecord(t0, st)) != hipSuccess) return err;
    if (f32) k_event_epan<true><<<(unsigned)be, kEpBS, 0, st>>>(kern);
    else k_event_epan<false><<<(unsigned)be, kEpBS, 0, st>>>(kern);
    if (t1 && (err = hipEventRecord(t1, st)) != hipSuccess) return err;
  } else {
    const long long bs = item_lambda_blocks(kern.U, kern.B);
    const size_t lds =
        (size_t)sm_fbytes(f32) + (size_t)kSmGCap * (f32 ? sizeof(float) : sizeof(double));
    const bool compl_ = kern.mz64 != nullptr;
    const void* smooth = compl_ ? (f32 ? (const void*)k_event_smooth32c : (const void*)k_event_smooth64c)
                                : (f32 ? (const void*)k_event_smooth32 : (const void*)k_event_smooth64);
    err = hipFuncSetAttribute(smooth, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    if (t0 && (err = hipEventRecord(t0, st)) != hipSuccess) return err;
    if (compl_) {
      if (f32) k_event_smooth32c<<<(unsigned)bs, kSmBS, lds, st>>>(kern);
      else k_event_smooth64c<<<(unsigned)bs, kSmBS, lds, st>>>(kern);
    } else {
      if (f32) k_event_smooth32<<<(unsigned)bs, kSmBS, lds, st>>>(kern);
      else k_event_smooth64<<<(unsigned)bs, kSmBS, lds, st>>>(kern);
    }
    if (t1 && (err = hipEventRecord(t1, st)) != hipSuccess) return err;
  }
  if (kern.count) {
    const long long nc = (long long)kern.B * kern.U;
    const unsigned blocks = (unsigned)std::min<long long>((nc + 4095) / 4096 + 1, 1024);
    k_count_sum<<<blocks, 256, 0, st>>>(kern.pcount, nc, kern.count);
  }
  const long long nf = (long long)kern.B * kern.E;
  k_event_final<<<(unsigned)((nf + 255) / 256), 256, 0, st>>>(kern);
  return hipGetLastError();
}

}  // namespace chimera
