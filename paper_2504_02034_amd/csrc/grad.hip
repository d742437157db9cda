// Adjoint of ln L (gradient with respect to the 12 differentiated parameters
// H0, Om, Xi0, n, alpha, beta, mu_g, sigma_g, lambda_g, gamma, kappa, z_p;
// mmin and mmax are hard edges of the mass model and are not differentiated).
//
// Chain rule, per event i with S_i = sum_r c_ir sum_j w_j A_j and
// I_i = S_i / (h sqrt(2 pi)):
//   d ln I_i / dp = (1/S_i) sum_j c_j w_j [ d ln w_j/dp A_j + dz_j/dp dA_j/dz_j
//                                          + dA_j/dh dh/dp + sum_g F_g K_jg d ln g/dp ]
//                   - d ln h / dp
// with dA/dz_j = sum F K (z_g - z_j) / h^2, dA/dh = sum F K (z_g - z_j)^2 / h^3
// (the window edges |z_g - z_j| = T h are not differentiated).  The redshift
// of a sample moves as dx_j/dp = -(dD/dp) / (dD/dx) (x = ln(1+z), implicit in
// d_L^gw(x_j) = d_j, eqs. dL-em and dL-mg).  The bandwidth derivative runs
// through the moments W1, W2, sum w (z - s), sum w (z - s)^2 (s: a shift).
// Selection: d ln xi / dp = sum_j s_j d ln s_j / dp / sum_j s_j.
//
// k_lam_grad_prepare  per-lambda normaliser derivatives of the mass model
// k_grid_grad         g(z_g) d ln g / dp on the grid for p = Om, Xi0, n,
//                     gamma, kappa, z_p (H0 enters g as a factor H0)
// k_event_bandwidth_grad  one (event, lambda) per workgroup: each sample's
//                     z, w and their derivatives (stored, structure of
//                     arrays), the bandwidth moments and their derivatives
//                     -> h, d ln h/dp
// k_event_grad        one (event, lambda) per workgroup, one sample per
//                     thread, from the stored coefficients: its window by the
//                     Gaussian ratio recurrence K_(g+1) = K_g r_g,
//                     r_(g+1) = r_g exp(-dz^2/h^2), or (EPAN) the
//                     Epanechnikov kernel's support with its polynomial
//                     k = 1 - u^2/W^2 per point
// k_bin_grad          binned sets: per (slot, lambda) each bin's point and
//                     derivative coefficients, from its samples'
// k_selection_grad    per (injection chunk, lambda) partial sums
// k_grad_final        ln L and d ln L / dp per lambda, fixed order
#include <math.h>

#include "common.h"
#include "launch.h"
#include "reduce.h"

namespace chimera {

namespace {

constexpr int kNG = CHIMERA_NGRAD;   // 12
constexpr int kNS = 9;               // parameters a sample depends on: H0, Om, Xi0, n, mass (5)
constexpr int kGradBS = 256;
constexpr int kSD = kGradDerivFields;
constexpr int kGradStageElems = 6144;   // LDS copy of g and g dln g/dp: 7 x span values
static_assert(kSD == kNS + 4 && kGradSampleFields == 2 + kSD, "per-sample coefficient layout");

__device__ __forceinline__ double phi_std(double t) {
  return 0.39894228040143267794 * exp(-0.5 * t * t);
}

// f(y) = y / (1 - e^-y) - 1, with its series near 0
__device__ __forceinline__ double f_pair(double y) {
  if (fabs(y) < 1e-5) return y * (0.5 + y / 12.0);
  return y / -expm1(-y) - 1.0;
}

// Per-sample redshift, weight and their derivatives.
struct SampleGrad {
  double x, zp1, w;
  double dx[4];      // dx/dp for H0, Om, Xi0, n
  double dlw[kNS];   // d ln w / dp (through z for the distance parameters)
};

// pieces of dD/dx = dh e^x (q + q'), q = chi Xi, q' = chi' Xi + chi Xi'
struct DistPieces {
  double chi, chio, chip, chiop, en, xi, xip, q, qp;
};

__device__ __forceinline__ DistPieces dist_pieces(const LamParams& P, const double2* chi,
                                                  const double2* chio, const Geometry& g,
                                                  double x, double zp1) {
  DistPieces d;
  const double e = efunc_of_zp1(P.om, zp1);
  d.chi = chi_at(chi, g, x);
  d.chio = chi_at(chio, g, x);
  d.chip = zp1 / e;
  d.chiop = -0.5 * zp1 * (zp1 * zp1 * zp1 - 1.0) / (e * e * e);
  d.en = exp(-P.n * x);
  d.xi = P.xi0 + (1.0 - P.xi0) * d.en;
  d.xip = -P.n * (1.0 - P.xi0) * d.en;
  d.q = d.chi * d.xi;
  d.qp = d.chip * d.xi + d.chi * d.xip;
  return d;
}

// d ln(dD/dx) / dp at fixed x for p = H0, Om, Xi0, n
__device__ __forceinline__ void dlnDx(const LamParams& P, const DistPieces& d, double x,
                                      double (&out)[4]) {
  const double inv = 1.0 / (d.q + d.qp);
  out[0] = -1.0 / P.h0;
  out[1] = (d.chio * d.xi + d.chiop * d.xi + d.chio * d.xip) * inv;
  const double xa = 1.0 - d.en, xap = P.n * d.en;                     // dXi, dXi'/dXi0
  out[2] = (d.chi * xa + d.chip * xa + d.chi * xap) * inv;
  const double xn = -(1.0 - P.xi0) * x * d.en;                        // dXi/dn
  const double xnp = -(1.0 - P.xi0) * d.en * (1.0 - P.n * x);         // dXi'/dn
  out[3] = (d.chi * xn + d.chip * xn + d.chi * xnp) * inv;
}

// d ln psi / d(gamma, kappa, z_p) at fixed x, and d ln psi / dx
__device__ __forceinline__ void dlnpsi(const LamParams& P, double x, double (&out)[3],
                                       double& ddx) {
  const double lr = x - P.ln1zp;
  const double r = exp((P.gamma + P.kappa) * lr);
  const double s = r / (1.0 + r);
  out[0] = x - s * lr;
  out[1] = -s * lr;
  out[2] = s * (P.gamma + P.kappa) / (1.0 + P.zp);
  ddx = P.gamma - s * (P.gamma + P.kappa);
}

__device__ __forceinline__ void sample_grad(const LamParams& P, const GradParams& Q,
                                            const double2* chi, const double2* chio,
                                            const double2* dtab, const double2* inv,
                                            const Geometry& g, double d, double lnd, double m1d,
                                            double m2d, double lnm1d, double lnm2d,
                                            SampleGrad& s, DistPieces& dp) {
  double x = invert_x(P, nullptr, inv, g, d, lnd, 0);
  double zp1 = exp(x);
  {
    double D, Dx;
    dist_tab_at(dtab, g, x, D, Dx);
    const double dxn = (D - d) / Dx;
    x -= dxn;
    zp1 *= 1.0 - dxn + 0.5 * dxn * dxn;
  }
  s.x = x;
  s.zp1 = zp1;
  dp = dist_pieces(P, chi, chio, g, x, zp1);
  const double dem = P.dh * zp1 * dp.chi;
  const double Dx = P.dh * zp1 * (dp.q + dp.qp);
  // -dD/dp / (dD/dx)
  s.dx[0] = (dem * dp.xi / P.h0) / Dx;
  s.dx[1] = -(P.dh * zp1 * dp.chio * dp.xi) / Dx;
  s.dx[2] = -(dem * (1.0 - dp.en)) / Dx;
  s.dx[3] = (dem * (1.0 - P.xi0) * x * dp.en) / Dx;
  const double r = 1.0 / zp1;
  const double m1 = m1d * r, m2 = m2d * r;
  const double l1 = lnm1d - x, l2 = lnm2d - x;
  s.w = mass_weight64(P, m1, m2, l1, l2);
#pragma unroll
  for (int k = 0; k < kNS; ++k) s.dlw[k] = 0.0;
  if (!(s.w > 0.0)) return;
  const double u = (m1 - P.mu) * P.inv_sigma;
  const double PL = Q.pl_unit * exp(-P.alpha * l1);
  const double TG = Q.tg_unit * exp(-0.5 * u * u);
  const double ip1 = 1.0 / ((1.0 - P.lg) * PL + P.lg * TG);
  s.dlw[4] = (1.0 - P.lg) * PL * (-l1 - Q.dlnnpl_dalpha) * ip1;
  const double L = l1 - P.ln_mmin;
  const double y = P.a2 * L;
  double pair_m1;                      // m1 d ln p(m2|m1) / d m1
  if (P.a2 == 0.0) {
    s.dlw[5] = l2 - P.ln_mmin - 0.5 * L;
    pair_m1 = -1.0 / L;
  } else {
    s.dlw[5] = l2 - P.ln_mmin - f_pair(y) / P.a2;
    pair_m1 = -P.a2 / -expm1(-y);
  }
  s.dlw[6] = P.lg * TG * (u * P.inv_sigma - Q.dlnz_dmu) * ip1;
  s.dlw[7] = P.lg * TG * ((u * u - 1.0) * P.inv_sigma - Q.dlnz_dsigma) * ip1;
  s.dlw[8] = (TG - PL) * ip1;
  const double m1_p1 = ((1.0 - P.lg) * PL * -P.alpha + P.lg * TG * (-u * m1 * P.inv_sigma)) * ip1;
  // m = m_det e^-x: d ln w / dx = -(m1 d/dm1 + m2 d/dm2) ln w
  const double dlw_dx = -(m1_p1 + pair_m1 + P.beta);
#pragma unroll
  for (int k = 0; k < 4; ++k) s.dlw[k] = dlw_dx * s.dx[k];
}

}  // namespace

// ---------------------------------------------------------------------------
__global__ void k_lam_grad_prepare(const LamParams* __restrict__ Pv, int B,
                                   GradParams* __restrict__ Qv) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const LamParams P = Pv[b];
  GradParams Q;
  // N_pl = int_mmin^mmax m^(a1-1) dm, a1 = 1 - alpha; d ln N_pl / d alpha =
  // -(ln mmin + f(a1 ln(mmax/mmin)) / a1)
  const double a1 = 1.0 - P.alpha;
  const double lr = P.ln_mmax - P.ln_mmin;
  const double npl = (a1 == 0.0) ? lr : exp(a1 * P.ln_mmin) * expm1(a1 * lr) / a1;
  Q.pl_unit = 1.0 / npl;
  Q.dlnnpl_dalpha = -(P.ln_mmin + (a1 == 0.0 ? 0.5 * lr : f_pair(a1 * lr) / a1));
  const double a = (P.mmin - P.mu) * P.inv_sigma, bb = (P.mmax - P.mu) * P.inv_sigma;
  const double r = 0.70710678118654752440;
  const double Z = a > 0.0 ? 0.5 * (erfc(a * r) - erfc(bb * r)) : 0.5 * (erfc(-bb * r) - erfc(-a * r));
  Q.tg_unit = 1.0 / (P.sigma * 2.50662827463100050242 * Z);
  Q.dlnz_dmu = (phi_std(a) - phi_std(bb)) * P.inv_sigma / Z;
  Q.dlnz_dsigma = (a * phi_std(a) - bb * phi_std(bb)) * P.inv_sigma / Z;
  Qv[b] = Q;
}

// g d ln g / dp on the grid, p = Om, Xi0, n, gamma, kappa, z_p: [B][6][n_z]
__global__ void k_grid_grad(const LamParams* __restrict__ Pv, const double2* __restrict__ chi,
                            const double2* __restrict__ chio, const double* __restrict__ gz64,
                            Geometry g, int B, double* __restrict__ gf64,
                            float* __restrict__ gf32) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)B * g.n_z) return;
  const int b = (int)(id / g.n_z), k = (int)(id % g.n_z);
  const LamParams P = Pv[b];
  const double z = g.z_lo + (double)k * g.dz;
  const double x = log1p(z);
  const DistPieces d = dist_pieces(P, chi + (size_t)b * g.n_t, chio + (size_t)b * g.n_t, g, x,
                                   1.0 + z);
  double dd[4], dpsi[3], unused;
  dlnDx(P, d, x, dd);
  dlnpsi(P, x, dpsi, unused);
  const double gv = gz64[id];
  const double f[6] = {-dd[1], -dd[2], -dd[3], dpsi[0], dpsi[1], dpsi[2]};
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    const double v = isfinite(gv * f[p]) ? gv * f[p] : 0.0;
    gf64[((size_t)b * 6 + p) * g.n_z + k] = v;
    gf32[((size_t)b * 6 + p) * g.n_z + k] = (float)v;
  }
}

// Incomplete catalogue (eqs. p-gal, p-miss, f-R): one workgroup per lambda.
// v = chi^2 / (E (4 pi/3) chi(z_max)^3) with d ln v / d Om = 2 chi'/chi -
// E'/E - 3 chi'(z_max)/chi(z_max), chi' = d chi / d Om (the chio table),
// E' = ((1+z)^3 - 1) / (2E); f_R = sum_g tau_g (4 pi - M) v and f_R' the same
// sum of v'.  Writes v and v' g on the grid, (f_R, f_R'), and n_tot^eff =
// f_R n_tot + M v with its Om derivative f_R' n_tot + M v'.
constexpr int kCompGradBS = 256;
__global__ __launch_bounds__(kCompGradBS) void k_completion_grad(GradArgs a,
                                                                 const double* __restrict__ ntot,
                                                                 const double* __restrict__ missing,
                                                                 double* __restrict__ ntot_eff,
                                                                 double* __restrict__ dntot) {
  const int b = blockIdx.x;
  __shared__ double red[kCompGradBS / 64 + 1];
  const LamParams P = a.P[b];
  const Geometry& g = a.g;
  const double2* chi = a.chi + (size_t)b * g.n_t;
  const double2* chio = a.chio + (size_t)b * g.n_t;
  const double zmax = g.z_lo + (double)(g.n_z - 1) * g.dz;
  const double xm = log1p(zmax);
  const double cm = chi_at(chi, g, xm), dcm = chi_at(chio, g, xm);
  const double norm = 1.0 / (4.0 * M_PI / 3.0 * cm * cm * cm);
  // v and v' at node k
  auto vol = [&](int k, double& dv) {
    const double z = g.z_lo + (double)k * g.dz;
    const double x = log1p(z);
    const double c = chi_at(chi, g, x);
    const double e = efunc_of_zp1(P.om, 1.0 + z);
    const double v = c * c / e * norm;
    const double zp3 = (1.0 + z) * (1.0 + z) * (1.0 + z);
    dv = c > 0.0 ? v * (2.0 * chi_at(chio, g, x) / c - (zp3 - 1.0) / (2.0 * e * e) - 3.0 * dcm / cm)
                 : 0.0;
    return v;
  };
  double t0 = 0.0, t1 = 0.0;
  for (int k = threadIdx.x; k < g.n_z; k += kCompGradBS) {
    const double tau = (k == 0 || k == g.n_z - 1) ? 0.5 * g.dz : g.dz;
    double dv;
    const double v = vol(k, dv);
    t0 += tau * (4.0 * M_PI - missing[k]) * v;
    t1 += tau * (4.0 * M_PI - missing[k]) * dv;
  }
  const double fR = block_sum<kCompGradBS>(t0, red);
  const double dfR = block_sum<kCompGradBS>(t1, red);
  if (threadIdx.x == 0) {
    a.cf[2 * b] = fR;
    a.cf[2 * b + 1] = dfR;
  }
  for (int k = threadIdx.x; k < g.n_z; k += kCompGradBS) {
    double dv;
    const double v = vol(k, dv);
    const size_t i = (size_t)b * g.n_z + k;
    ntot_eff[i] = fR * ntot[k] + missing[k] * v;
    dntot[i] = dfR * ntot[k] + missing[k] * dv;
    const size_t c0 = (size_t)b * 2 * g.n_z + k, c1 = c0 + g.n_z;
    const double dvg = dv * a.gz64[i];
    a.cv64[c0] = v;
    a.cv64[c1] = dvg;
    a.cv32[c0] = (float)v;
    a.cv32[c1] = (float)dvg;
  }
}

// ---------------------------------------------------------------------------
// Bandwidth and its derivatives, one (event, lambda) per workgroup: W1, W2,
// M1 = sum w (z - s), M2 = sum w (z - s)^2 (s: the event's first redshift)
// and their derivatives for the parameters a sample depends on.  Writes
// hd[b][e] = (h, d ln h / dp for those 9 parameters), h < 0 marking W1 = 0,
// and every sample's coefficients: sc[b][field][sample] = z, c w (0: no
// weight); sd[b][field][sample] = d ln w / dp (9), dz / dp (4 distance
// parameters), in FP32 when the window sums are.
__global__ __launch_bounds__(kGradBS) void k_event_bandwidth_grad(GradArgs a) {
  int e, b;
  if (!decode_item_lambda(a.E, a.B, e, b)) return;
  constexpr int NW = kGradBS / 64 + 1;
  __shared__ double red[40 * NW];
  __shared__ double shift;
  const LamParams P = a.P[b];
  double* hd = a.hd + ((size_t)b * a.E + e) * (1 + kNS);
  if (P.flag | a.flag_mono[b] | a.flag_range[b]) return;   // the final kernel reports it
  const GradParams Q = a.Q[b];
  const double2* chi = a.chi + (size_t)b * a.g.n_t;
  const double2* chio = a.chio + (size_t)b * a.g.n_t;
  const double2* dtab = a.dtab + (size_t)b * a.g.n_t;
  const double2* inv = a.inv + (size_t)b * a.g.n_u;
  const int s0 = a.ev_samp_off[e];
  const int ns = a.ev_samp_off[e + 1] - s0;
  SampleGrad sg;
  DistPieces dp;
  if (threadIdx.x == 0) {
    sample_grad(P, Q, chi, chio, dtab, inv, a.g, a.dl[s0], a.lndl[s0], a.m1d[s0], a.m2d[s0],
                a.lnm1d[s0], a.lnm2d[s0], sg, dp);
    shift = sg.zp1 - 1.0;
  }
  __syncthreads();
  const double zs = shift;
  double m[40];
#pragma unroll
  for (int i = 0; i < 40; ++i) m[i] = 0.0;
  // software pipeline: the next sample's inputs load while this one is
  // evaluated (indices past the end read this event's first sample)
  auto in = [&](int j, double (&v)[6]) {
    const int q = s0 + (j < ns ? j : 0);
    v[0] = a.dl[q]; v[1] = a.lndl[q]; v[2] = a.m1d[q];
    v[3] = a.m2d[q]; v[4] = a.lnm1d[q]; v[5] = a.lnm2d[q];
  };
  double cur[6];
  in(threadIdx.x, cur);
  for (int j = threadIdx.x; j < ns; j += kGradBS) {
    const int q = s0 + j;
    double nxt[6];
    in(j + kGradBS, nxt);
    sample_grad(P, Q, chi, chio, dtab, inv, a.g, cur[0], cur[1], cur[2], cur[3], cur[4], cur[5],
                sg, dp);
#pragma unroll
    for (int i = 0; i < 6; ++i) cur[i] = nxt[i];
    const double w = sg.w;
    double* sc = a.sc + (size_t)b * 2 * a.S + q;
    sc[0] = sg.zp1 - 1.0;
    sc[a.S] = w > 0.0 ? a.samp_c[q] * w : 0.0;
    if (a.f32) {
      float* sd = (float*)a.sd + (size_t)b * kSD * a.S + q;
#pragma unroll
      for (int p = 0; p < kNS; ++p) sd[(size_t)p * a.S] = (float)sg.dlw[p];
#pragma unroll
      for (int p = 0; p < 4; ++p) sd[(size_t)(kNS + p) * a.S] = (float)(sg.zp1 * sg.dx[p]);
    } else {
      double* sd = (double*)a.sd + (size_t)b * kSD * a.S + q;
#pragma unroll
      for (int p = 0; p < kNS; ++p) sd[(size_t)p * a.S] = sg.dlw[p];
#pragma unroll
      for (int p = 0; p < 4; ++p) sd[(size_t)(kNS + p) * a.S] = sg.zp1 * sg.dx[p];
    }
    if (!(w > 0.0)) continue;
    const double t = sg.zp1 - 1.0 - zs;
    m[0] += w;
    m[1] += w * w;
    m[2] += w * t;
    m[3] += w * t * t;
#pragma unroll
    for (int p = 0; p < kNS; ++p) {
      const double dw = w * sg.dlw[p];
      const double dzp = p < 4 ? sg.zp1 * sg.dx[p] : 0.0;
      m[4 + p] += dw;
      m[4 + kNS + p] += 2.0 * w * dw;
      m[4 + 2 * kNS + p] += dw * t + w * dzp;
      m[4 + 3 * kNS + p] += dw * t * t + 2.0 * w * t * dzp;
    }
  }
  block_reduce<kGradBS, 40, false>(m, red);
  if (threadIdx.x != 0) return;
  const double W1 = m[0], W2 = m[1], M1 = m[2], M2 = m[3];
  if (!(W1 > 0.0)) {
    hd[0] = -1.0;
    return;
  }
  const double mu = M1 / W1;
  const double den = W1 - W2 / W1;
  double var = 0.0, V = 0.0;
  const bool spread = !(W1 * W1 - W2 <= 1e-12 * W1 * W1);
  if (spread) {
    V = fmax(M2 - M1 * mu, 0.0);
    var = V / den;
  }
  const double raw = sqrt(var) * pow(W1 * W1 / W2, -0.2);
  hd[0] = fmax(raw, 2.0 * a.g.dz);
  const bool live = spread && V > 0.0 && raw >= 2.0 * a.g.dz;
  for (int p = 0; p < kNS; ++p) {
    double v = 0.0;
    if (live) {
      const double dW1 = m[4 + p], dW2 = m[4 + kNS + p];
      const double dM1 = m[4 + 2 * kNS + p], dM2 = m[4 + 3 * kNS + p];
      const double dV = dM2 - 2.0 * mu * dM1 + mu * mu * dW1;
      const double dden = dW1 - dW2 / W1 + W2 * dW1 / (W1 * W1);
      v = 0.5 * dV / V - 0.5 * dden / den - 0.2 * (2.0 * dW1 / W1 - dW2 / W2);
    }
    hd[1 + p] = v;
  }
}

// A sample's window sums: A = sum a, sum a m, sum a m^2 (a = n_r g K, m the
// grid offset from the grid point nearest the sample, exact in either
// precision, so u = m dz + delta) and six sum n_r K g dln g/dp, by the
// Gaussian ratio recurrence.  Grid point g of the grid factor is gz[g - off],
// of derivative p gf[p fstride + g - off] (the workgroup's LDS copy or the
// tables themselves); 4 points per iteration keep their loads in flight
// together.
template <class CT>
__device__ __forceinline__ void window_sums(const CT* __restrict__ nrow,
                                            const CT* __restrict__ gz,
                                            const CT* __restrict__ gf, int fstride, int off,
                                            int lo, int hi, CT m0, CT K, CT r, CT qr, CT& sA,
                                            CT& sB, CT& sC, CT (&sE)[6]) {
  int gi = lo;
  // FP32: the catalogue row one block ahead (the last block's start is read
  // again at the end, so every read stays inside [lo, hi]); FP64 has no
  // registers to spare for it
  constexpr bool PF = sizeof(CT) == 4;
  CT nx[4];
  if (PF && gi + 3 <= hi) {
#pragma unroll
    for (int i = 0; i < 4; ++i) nx[i] = nrow[gi + i];
  }
  for (; gi + 3 <= hi; gi += 4) {
    CT nv[4], gv[4], fv[6][4];
    const int gn = min(gi + 4, hi - 3);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (PF) {
        nv[i] = nx[i];
        nx[i] = nrow[gn + i];
      } else {
        nv[i] = nrow[gi + i];
      }
      gv[i] = gz[gi + i - off];
    }
#pragma unroll
    for (int p = 0; p < 6; ++p)
#pragma unroll
      for (int i = 0; i < 4; ++i) fv[p][i] = gf[p * fstride + gi + i - off];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const CT u = m0 + (CT)i;
      const CT bk = nv[i] * K;
      const CT av = bk * gv[i];
      sA += av;
      const CT t = av * u;
      sB += t;
      sC = fma(t, u, sC);
#pragma unroll
      for (int p = 0; p < 6; ++p) sE[p] = fma(bk, fv[p][i], sE[p]);
      K *= r;
      r *= qr;
    }
    m0 += (CT)4;
  }
  for (; gi <= hi; ++gi) {
    const CT u = m0;
    m0 += (CT)1;
    const CT bk = nrow[gi] * K;
    const CT av = bk * gz[gi - off];
    sA += av;
    const CT t = av * u;
    sB += t;
    sC = fma(t, u, sC);
#pragma unroll
    for (int p = 0; p < 6; ++p) sE[p] = fma(bk, gf[p * fstride + gi - off], sE[p]);
    K *= r;
    r *= qr;
  }
}

// The same sums with an incomplete catalogue: the row is f_R n_r + (1 - P_r) v
// (mrow = 1 - P_r, vz = v on the grid), so a and the six derivative sums take
// that row in place of n_r, and d/dOm adds the row's own derivative
// f_R' n_r g + (1 - P_r) v' g (dvg = v' g).  A separate function keeps the
// plain one's registers.
template <class CT>
__device__ __forceinline__ void window_sums_c(const CT* __restrict__ nrow,
                                              const CT* __restrict__ mrow,
                                              const CT* __restrict__ gz, const CT* __restrict__ gf,
                                              const CT* __restrict__ vz,
                                              const CT* __restrict__ dvg, CT fR, CT dfR,
                                              int fstride, int off, int lo, int hi, CT m0,
                                              CT K, CT r, CT qr, CT& sA, CT& sB, CT& sC,
                                              CT (&sE)[6]) {
  auto step = [&](CT n, CT m, CT gv, const CT (&fv)[6], CT v, CT dv, CT u) {
    const CT kn = n * K, km = m * K;
    const CT bk = fma(km, v, kn * fR);
    const CT av = bk * gv;
    sA += av;
    const CT t = av * u;
    sB += t;
    sC = fma(t, u, sC);
#pragma unroll
    for (int p = 0; p < 6; ++p) sE[p] = fma(bk, fv[p], sE[p]);
    sE[0] = fma(kn, dfR * gv, fma(km, dv, sE[0]));
    K *= r;
    r *= qr;
  };
  int gi = lo;
  for (; gi + 1 <= hi; gi += 2) {
    CT nv[2], mv[2], gv[2], fv[2][6], vv[2], dv[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      nv[i] = nrow[gi + i];
      mv[i] = mrow[gi + i];
      gv[i] = gz[gi + i - off];
      vv[i] = vz[gi + i - off];
      dv[i] = dvg[gi + i - off];
#pragma unroll
      for (int p = 0; p < 6; ++p) fv[i][p] = gf[p * fstride + gi + i - off];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
      step(nv[i], mv[i], gv[i], fv[i], vv[i], dv[i], m0 + (CT)i);
    m0 += (CT)2;
  }
  for (; gi <= hi; ++gi) {
    CT fv[6];
#pragma unroll
    for (int p = 0; p < 6; ++p) fv[p] = gf[p * fstride + gi - off];
    step(nrow[gi], mrow[gi], gz[gi - off], fv, vz[gi - off], dvg[gi - off], m0);
    m0 += (CT)1;
  }
}

// The window sums of the Epanechnikov kernel (Sect. 2.3's compact option,
// k = 1 - u^2 / W^2 on |u| <= W, W = sqrt(5) h): sA = sum a k, sB = sum a u,
// sC = sum a u^2 (a = r g with r the sample's row, n_r or, with COMPL, the
// completed row f_R n_r + (1 - P_r) v) and the six sum r k g dln g/dp (plus
// k (f_R' n_r g + (1 - P_r) v' g) for Om with COMPL), so that
// dA/dz_j = 2 sB / W^2 and h dA/dh = 2 sC / W^2.  u = m dz + delta with m
// exact; two points per iteration.
template <class CT, bool COMPL>
__device__ __forceinline__ void window_sums_epan(const CT* __restrict__ nrow,
                                                 const CT* __restrict__ mrow,
                                                 const CT* __restrict__ gz,
                                                 const CT* __restrict__ gf,
                                                 const CT* __restrict__ vz,
                                                 const CT* __restrict__ dvg, CT fR, CT dfR,
                                                 int fstride, int off, int lo, int hi, CT m0,
                                                 CT dzc, CT delta, CT invW2, CT& sA, CT& sB,
                                                 CT& sC, CT (&sE)[6]) {
  auto step = [&](int g, CT m) {
    const CT n = nrow[g];
    const CT gv = gz[g - off];
    CT rv = n;
    CT mr = (CT)0;
    if (COMPL) {
      mr = mrow[g];
      rv = fma(mr, vz[g - off], n * fR);
    }
    const CT u = fma(m, dzc, delta);
    const CT k = fma(-u * invW2, u, (CT)1);
    const CT av = rv * gv;
    sA = fma(av, k, sA);
    const CT t = av * u;
    sB += t;
    sC = fma(t, u, sC);
    const CT bk = rv * k;
#pragma unroll
    for (int p = 0; p < 6; ++p) sE[p] = fma(bk, gf[p * fstride + g - off], sE[p]);
    if (COMPL) sE[0] = fma(k, fma(n, dfR * gv, mr * dvg[g - off]), sE[0]);
  };
  int gi = lo;
  for (; gi + 1 <= hi; gi += 2) {
    step(gi, m0);
    step(gi + 1, m0 + (CT)1);
    m0 += (CT)2;
  }
  if (gi <= hi) step(gi, m0);
}

// Binned data sets (Sect. 2.3): each slot's n_bins equal-width bins over the
// redshift range of its samples, a point at each bin's centre carrying its
// samples' summed weight.  One wave per (slot, lambda): a bin's samples are
// a run of the slot's distance order (redshift order, as d_L^gw increases),
// with the forward pass's bin arithmetic; the bin's c W, its d ln W/dp = sum c w d ln w/dp / sum c w
// (the samples' bins held fixed) and its centre's dz/dp = (1 - f) dz_lo/dp +
// f dz_hi/dp (f = (k + 1/2) / n_bins; the range's ends are the first and last
// sample) go to bsc / bsd in the layout of the samples' sc / sd, so that
// k_event_grad sums the bins as it sums samples.
// Up to kBinScan bins per slot the sums come from one pass over the slot's
// samples, 64 at a time, lanes over samples: the bins along the lanes never
// decrease, so a segmented scan over the lanes sums each bin's run and the
// run's last lane adds it to the bin's LDS accumulators (as the forward
// binning kernel does); more bins take the binary searches below.
constexpr int kBinScan = 128;

__device__ __forceinline__ void wave_fence_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool F32>
__global__ __launch_bounds__(kGradBS) void k_bin_grad(GradArgs a) {
  using CT = typename std::conditional<F32, float, double>::type;
  constexpr int SPB = kGradBS / 64;
  __shared__ double bacc[SPB][kBinScan][1 + kNS];
  int it, b;
  if (!decode_item_lambda((a.n_slots + SPB - 1) / SPB, a.B, it, b)) return;
  const int wv = (int)(threadIdx.x >> 6);
  const int p = it * SPB + wv;
  const int lane = threadIdx.x & 63;
  if (p >= a.n_slots) return;
  if (a.P[b].flag | a.flag_mono[b] | a.flag_range[b]) return;
  const int nb = a.bins;
  const long long S = a.S, NB = (long long)a.n_slots * nb;
  const int j0 = a.pix_off[p], n = a.pix_off[p + 1] - j0;
  const int* idx = a.pix_idx + j0;
  const double* scb = a.sc + (size_t)b * 2 * S;
  const CT* sdb = (const CT*)a.sd + (size_t)b * kSD * S;
  double* bsc = a.bsc + (size_t)b * 2 * NB;
  CT* bsd = (CT*)a.bsd + (size_t)b * kSD * NB;
  const double zlo = n > 0 ? scb[idx[0]] : 0.0, zhi = n > 0 ? scb[idx[n - 1]] : 0.0;
  const double width = (zhi - zlo) / (double)nb;
  auto bin_of = [&](int j) {
    if (!(width > 0.0)) return 0;
    const double f = floor((scb[idx[j]] - zlo) / width);
    return f >= (double)(nb - 1) ? nb - 1 : (int)f;
  };
  auto first_at_least = [&](int k) {     // first position whose bin is >= k
    int lo = 0, hi = n;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (bin_of(mid) < k) lo = mid + 1;
      else hi = mid;
    }
    return lo;
  };
  const bool scan = nb <= kBinScan;
  double(*acc)[1 + kNS] = bacc[wv];
  if (scan) {
    for (int k = lane; k < nb; k += 64)
#pragma unroll
      for (int r = 0; r <= kNS; ++r) acc[k][r] = 0.0;
    wave_fence_barrier();
    for (int c0 = 0; c0 < n; c0 += 64) {
      const int j = c0 + lane;
      const bool valid = j < n;
      int bin = 1 << 30;
      double v[1 + kNS];
#pragma unroll
      for (int r = 0; r <= kNS; ++r) v[r] = 0.0;
      if (valid) {
        const int q = idx[j];
        bin = bin_of(j);
        v[0] = scb[S + q];
#pragma unroll
        for (int r = 0; r < kNS; ++r) v[1 + r] = v[0] * (double)sdb[(size_t)r * S + q];
      }
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int bu = __shfl_up(bin, o, 64);
        const bool same = lane >= o && bu == bin;
#pragma unroll
        for (int r = 0; r <= kNS; ++r) {
          const double u = __shfl_up(v[r], o, 64);
          if (same) v[r] += u;
        }
      }
      const int bn = __shfl_down(bin, 1, 64);
      if (valid && (lane == 63 || bn != bin))
#pragma unroll
        for (int r = 0; r <= kNS; ++r) acc[bin][r] += v[r];
      wave_fence_barrier();
    }
  }
  for (int k = lane; k < nb; k += 64) {
    double W = 0.0, D[kNS];
#pragma unroll
    for (int q = 0; q < kNS; ++q) D[q] = 0.0;
    if (scan) {
      W = acc[k][0];
#pragma unroll
      for (int r = 0; r < kNS; ++r) D[r] = acc[k][1 + r];
    } else {
      const int j1 = first_at_least(k), j2 = first_at_least(k + 1);
      for (int j = j1; j < j2; ++j) {
        const int q = idx[j];
        const double cw = scb[S + q];
        W += cw;
#pragma unroll
        for (int r = 0; r < kNS; ++r) D[r] += cw * (double)sdb[(size_t)r * S + q];
      }
    }
    const long long o = (long long)p * nb + k;
    bsc[o] = width > 0.0 ? zlo + ((double)k + 0.5) * width : zlo;
    bsc[NB + o] = W;
#pragma unroll
    for (int r = 0; r < kNS; ++r) bsd[(size_t)r * NB + o] = (CT)(W > 0.0 ? D[r] / W : 0.0);
    const double f = width > 0.0 ? ((double)k + 0.5) / (double)nb : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double dlo = n > 0 ? (double)sdb[(size_t)(kNS + r) * S + idx[0]] : 0.0;
      const double dhi = n > 0 ? (double)sdb[(size_t)(kNS + r) * S + idx[n - 1]] : 0.0;
      bsd[(size_t)(kNS + r) * NB + o] = (CT)((1.0 - f) * dlo + f * dhi);
    }
  }
}

// Kernel sums and their parameter contractions, one (event, lambda) per
// workgroup, one sample per thread, from the coefficients the bandwidth
// kernel stored.  The grid factor and its six derivatives over the union of
// the workgroup's windows are copied to LDS once (when they fit), so that
// each grid point reads only the sample's catalogue row from memory.
template <bool F32, bool COMPL, bool EPAN>
__global__ __launch_bounds__(kGradBS) void k_event_grad(GradArgs a) {
  int e, b;
  if (!decode_item_lambda(a.E, a.B, e, b)) return;
  using CT = typename std::conditional<F32, float, double>::type;
  constexpr int NW = kGradBS / 64 + 1;
  __shared__ double red[(1 + kNG) * NW];
  __shared__ int redi[2 * (kGradBS / 64)];
  extern __shared__ __align__(16) unsigned char gsm[];
  const LamParams P = a.P[b];
  double* lnI = a.lnI + (size_t)b * a.E + e;
  double* dlnI = a.dlnI + ((size_t)b * a.E + e) * kNG;
  if (P.flag | a.flag_mono[b] | a.flag_range[b]) {
    if (threadIdx.x == 0) *lnI = NAN;                 // the final kernel reports the flag
    return;
  }
  const double* hd = a.hd + ((size_t)b * a.E + e) * (1 + kNS);
  const double h = hd[0];
  if (!(h > 0.0)) {
    if (threadIdx.x == 0) {
      *lnI = -INFINITY;
      for (int p = 0; p < kNG; ++p) dlnI[p] = NAN;
    }
    return;
  }
  // the event's points: its samples, or its slots' bins (slot-major)
  const int s0 = a.bins ? a.ev_slot_off[e] * a.bins : a.ev_samp_off[e];
  const int ns = a.bins ? (a.ev_slot_off[e + 1] - a.ev_slot_off[e]) * a.bins
                        : a.ev_samp_off[e + 1] - s0;
  const double dz = a.g.dz, inv_h2 = 1.0 / (h * h);
  // the window's half-width in units of h: the Gaussian's truncation, or the
  // Epanechnikov kernel's support
  const double T = EPAN ? kEpanScale : a.trunc;
  const double W = kEpanScale * h;
  const CT qr = (CT)exp(-dz * dz * inv_h2);
  const CT* nzt = F32 ? (const CT*)a.nz32 : (const CT*)a.nz64;
  const CT* gzt = F32 ? (const CT*)(a.gz32 + (size_t)b * a.g.n_z)
                      : (const CT*)(a.gz64 + (size_t)b * a.g.n_z);
  const CT* gft = F32 ? (const CT*)(a.gf32 + (size_t)b * 6 * a.g.n_z)
                      : (const CT*)(a.gf64 + (size_t)b * 6 * a.g.n_z);
  // the completion parts (incomplete catalogue): v and v' g, f_R and f_R'
  const CT* mzt = COMPL ? (F32 ? (const CT*)a.mz32 : (const CT*)a.mz64) : nullptr;
  const CT* cvt = COMPL ? (F32 ? (const CT*)(a.cv32 + (size_t)b * 2 * a.g.n_z)
                               : (const CT*)(a.cv64 + (size_t)b * 2 * a.g.n_z))
                        : nullptr;
  const CT fR = COMPL ? (CT)a.cf[2 * b] : (CT)1, dfR = COMPL ? (CT)a.cf[2 * b + 1] : (CT)0;
  const int nz = a.g.n_z;
  const double* scb = a.sc + (size_t)b * 2 * a.S;
  const CT* sdb = (const CT*)a.sd + (size_t)b * kSD * a.S;
  // the union of the workgroup's windows
  int lo_b = 1 << 30, hi_b = -(1 << 30);
  for (int j = threadIdx.x; j < ns; j += kGradBS) {
    const int q = s0 + j;
    if (!(scb[a.S + q] > 0.0)) continue;
    const double z = scb[q];
    const double lo_d = fmax(ceil((z - T * h - a.g.z_lo) * a.g.inv_dz), 0.0);
    const double hi_d = fmin(floor((z + T * h - a.g.z_lo) * a.g.inv_dz), (double)(nz - 1));
    if (!(lo_d <= hi_d)) continue;
    lo_b = min(lo_b, (int)lo_d);
    hi_b = max(hi_b, (int)hi_d);
  }
  int mx[2] = {-lo_b, hi_b};
  block_max_i32<kGradBS, 2>(mx, redi);
  const int A_lo = max(-mx[0], 0), A_hi = min(mx[1], nz - 1);
  const int span = A_hi - A_lo + 1;
  CT* sg = reinterpret_cast<CT*>(gsm);
  CT* sgb = sg + 7 * span;                     // v and v' g after g and its derivatives
  const bool staged = span > 0 && (COMPL ? 9 : 7) * span <= kGradStageElems;
  if (staged) {
    for (int k = threadIdx.x; k < span; k += kGradBS) sg[k] = gzt[A_lo + k];
    for (int p = 0; p < 6; ++p)
      for (int k = threadIdx.x; k < span; k += kGradBS)
        sg[(1 + p) * span + k] = gft[(size_t)p * nz + A_lo + k];
    if (COMPL)
      for (int p = 0; p < 2; ++p)
        for (int k = threadIdx.x; k < span; k += kGradBS)
          sgb[p * span + k] = cvt[(size_t)p * nz + A_lo + k];
    __syncthreads();
  }
  double acc[1 + kNG];
#pragma unroll
  for (int i = 0; i <= kNG; ++i) acc[i] = 0.0;
  for (int j = threadIdx.x; j < ns; j += kGradBS) {
    const int q = s0 + j;
    const double cw = scb[a.S + q];
    if (!(cw > 0.0)) continue;
    const double z = scb[q];
    const double lo_d = fmax(ceil((z - T * h - a.g.z_lo) * a.g.inv_dz), 0.0);
    const double hi_d = fmin(floor((z + T * h - a.g.z_lo) * a.g.inv_dz), (double)(nz - 1));
    if (!(lo_d <= hi_d)) continue;
    const int lo = (int)lo_d, hi = (int)hi_d;
    const double u0 = a.g.z_lo + lo_d * dz - z;
    const CT K = EPAN ? (CT)0 : (CT)exp(-0.5 * u0 * u0 * inv_h2);
    const CT r = EPAN ? (CT)0 : (CT)exp(-(2.0 * u0 * dz + dz * dz) * 0.5 * inv_h2);
    // offsets from the grid point nearest the sample: u = m dz + delta
    const double gcd = rint((z - a.g.z_lo) * a.g.inv_dz);
    const double delta = a.g.z_lo + gcd * dz - z;
    const CT m0 = (CT)(lo_d - gcd);
    const int rq = a.bins ? a.slot_row[q / a.bins] : a.samp_row[q];
    const CT* nrow = nzt + (size_t)rq * nz;
    const CT* mrow = COMPL ? mzt + (size_t)rq * nz : nullptr;
    CT sA = 0, sB = 0, sC = 0, sE[6] = {0, 0, 0, 0, 0, 0};
    if (EPAN) {
      const CT invW2 = (CT)(1.0 / (W * W));
      if (staged)
        window_sums_epan<CT, COMPL>(nrow, mrow, sg, sg + span, sgb, sgb + span, fR, dfR, span,
                                    A_lo, lo, hi, m0, (CT)dz, (CT)delta, invW2, sA, sB, sC, sE);
      else
        window_sums_epan<CT, COMPL>(nrow, mrow, gzt, gft, cvt, COMPL ? cvt + nz : nullptr, fR,
                                    dfR, nz, 0, lo, hi, m0, (CT)dz, (CT)delta, invW2, sA, sB, sC,
                                    sE);
    } else if (COMPL) {
      if (staged)
        window_sums_c<CT>(nrow, mrow, sg, sg + span, sgb, sgb + span, fR, dfR, span, A_lo, lo, hi,
                          m0, K, r, qr, sA, sB, sC, sE);
      else
        window_sums_c<CT>(nrow, mrow, gzt, gft, cvt, cvt + nz, fR, dfR, nz, 0, lo, hi, m0, K, r,
                          qr, sA, sB, sC, sE);
    } else if (staged) {
      window_sums<CT>(nrow, sg, sg + span, span, A_lo, lo, hi, m0, K, r, qr, sA, sB, sC, sE);
    } else {
      window_sums<CT>(nrow, gzt, gft, nz, 0, lo, hi, m0, K, r, qr, sA, sB, sC, sE);
    }
    double A, Bz, Chh;
    if (EPAN) {
      // dA/dz_j = 2 sum a u / W^2, h dA/dh = 2 sum a u^2 / W^2
      const double iw2 = 2.0 / (W * W);
      A = (double)sA;
      Bz = (double)sB * iw2;
      Chh = (double)sC * iw2;
    } else {
      const double sm = (double)sB;
      A = (double)sA;
      Bz = (dz * sm + delta * A) * inv_h2;
      Chh = (dz * (dz * (double)sC + 2.0 * delta * sm) + delta * delta * A) * inv_h2;
    }
    acc[0] += cw * A;
    // distance parameters: weight, z-shift, bandwidth, grid factor (H0: g ~ H0)
    const double Eg[4] = {A / P.h0, (double)sE[0], (double)sE[1], (double)sE[2]};
#pragma unroll
    for (int p = 0; p < 4; ++p)
      acc[1 + p] += cw * ((double)sdb[(size_t)p * a.S + q] * A +
                          (double)sdb[(size_t)(kNS + p) * a.S + q] * Bz + Chh * hd[1 + p] + Eg[p]);
#pragma unroll
    for (int p = 4; p < kNS; ++p)
      acc[1 + p] += cw * ((double)sdb[(size_t)p * a.S + q] * A + Chh * hd[1 + p]);
#pragma unroll
    for (int p = 0; p < 3; ++p) acc[1 + kNS + p] += cw * (double)sE[3 + p];
  }
  block_reduce<kGradBS, 1 + kNG, false>(acc, red);
  if (threadIdx.x == 0) {
    const double S = acc[0];
    if (!(S > 0.0)) {
      *lnI = -INFINITY;
      for (int p = 0; p < kNG; ++p) dlnI[p] = NAN;
    } else {
      *lnI = log(S * (EPAN ? 0.75 / kEpanScale : kInvSqrt2Pi) / h);
      for (int p = 0; p < kNG; ++p) dlnI[p] = acc[1 + p] / S - (p < kNS ? hd[1 + p] : 0.0);
    }
  }
}

// ---------------------------------------------------------------------------
constexpr int kSelGradBS = 256;
constexpr int kSelGradPer = 4;

// FP64 in both modes: the selection sums are a small part of the work.
// Partials per chunk: sum s, the 12 sums s d ln s / dp, sum s^2 (N_eff).
constexpr int kSelParts = kNG + 2;
__global__ __launch_bounds__(kSelGradBS) void k_selection_grad(SelGradArgs a) {
  const int chunk = blockIdx.x, b = blockIdx.y;
  __shared__ double red[kSelParts * (kSelGradBS / 64 + 1)];
  double* part = a.partial + ((size_t)b * a.nchunk + chunk) * kSelParts;
  const LamParams P = a.P[b];
  if (P.flag | a.flag_mono[b] | a.flag_range[b]) {
    if (threadIdx.x == 0)
      for (int i = 0; i < kSelParts; ++i) part[i] = 0.0;
    return;
  }
  const GradParams Q = a.Q[b];
  const double2* chi = a.chi + (size_t)b * a.g.n_t;
  const double2* chio = a.chio + (size_t)b * a.g.n_t;
  const double2* dtab = a.dtab + (size_t)b * a.g.n_t;
  const double2* inv = a.inv + (size_t)b * a.g.n_u;
  double acc[kSelParts];
#pragma unroll
  for (int i = 0; i < kSelParts; ++i) acc[i] = 0.0;
  for (int k = 0; k < kSelGradPer; ++k) {
    const long long j = (long long)chunk * kSelGradBS * kSelGradPer + k * kSelGradBS + threadIdx.x;
    if (j >= a.n_det) break;
    SampleGrad sg;
    DistPieces d;
    sample_grad(P, Q, chi, chio, dtab, inv, a.g, a.dl[j], a.lndl[j], a.m1d[j], a.m2d[j],
                a.lnm1d[j], a.lnm2d[j], sg, d);
    if (!(sg.w > 0.0)) continue;
    const double w = sg.w;
    const double z = sg.zp1 - 1.0;
    const double pos = (z - a.g.z_lo) * a.g.inv_dz;
    if (!(pos >= 0.0 && pos <= (double)(a.g.n_z - 1))) continue;
    int kk = (int)pos;
    kk = kk > a.g.n_z - 2 ? a.g.n_z - 2 : kk;
    const double t = pos - (double)kk;
    const double* ntot = a.ntot + (size_t)b * a.ntot_stride;
    const double nt = ntot[kk] + t * (ntot[kk + 1] - ntot[kk]);
    if (!(nt > 0.0)) continue;
    const double slope = (ntot[kk + 1] - ntot[kk]) * a.g.inv_dz;   // dn_tot/dz
    const double x = sg.x, zp1 = sg.zp1;
    const double Dx = P.dh * zp1 * (d.q + d.qp);
    // second x-derivative of d_L^gw: dh e^x (q + 2 q' + q'')
    const double e2 = P.om * zp1 * zp1 * zp1 + 1.0 - P.om;
    const double chipp = d.chip * (1.0 - 1.5 * P.om * zp1 * zp1 * zp1 / e2);
    const double xipp = P.n * P.n * (1.0 - P.xi0) * d.en;
    const double qpp = chipp * d.xi + 2.0 * d.chip * d.xip + d.chi * xipp;
    const double Dxx = P.dh * zp1 * (d.q + 2.0 * d.qp + qpp);
    double dpsi[3], dlpsi_dx, dd[4];
    dlnpsi(P, x, dpsi, dlpsi_dx);
    dlnDx(P, d, x, dd);
    const double s = w * nt * psi_of_x(P, x) / (zp1 * zp1 * Dx * exp(a.ln_pdraw[j]));
    // d ln s / dx at fixed lambda (the weight's own z path is in dlw)
    const double dls_dx = zp1 * slope / nt + dlpsi_dx - 2.0 - Dxx / Dx;
    acc[0] += s;
    acc[1 + kNG] += s * s;
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[1 + p] += s * (sg.dlw[p] + dls_dx * sg.dx[p] - dd[p]);
    if (a.dntot_om) {          // n_tot^eff's own Om dependence (incompleteness)
      const double* dn = a.dntot_om + (size_t)b * a.g.n_z;
      acc[2] += s * (dn[kk] + t * (dn[kk + 1] - dn[kk])) / nt;
    }
#pragma unroll
    for (int p = 4; p < kNS; ++p) acc[1 + p] += s * sg.dlw[p];
#pragma unroll
    for (int p = 0; p < 3; ++p) acc[1 + kNS + p] += s * dpsi[p];
  }
  block_reduce<kSelGradBS, kSelParts, false>(acc, red);
  if (threadIdx.x == 0)
    for (int i = 0; i < kSelParts; ++i) part[i] = acc[i];
}

// ---------------------------------------------------------------------------
constexpr int kGFinBS = 256;

__global__ __launch_bounds__(kGFinBS) void k_grad_final(GradFinalArgs a) {
  const int b = blockIdx.x;
  __shared__ double red[kSelParts * (kGFinBS / 64 + 1)];
  const LamParams P = a.P[b];
  const int flag = P.flag | a.flag_mono[b] | a.flag_range[b];
  // selection: chunks in a fixed order
  double v[kSelParts];
#pragma unroll
  for (int i = 0; i < kSelParts; ++i) v[i] = 0.0;
  for (int c = threadIdx.x; c < a.nchunk; c += kGFinBS)
#pragma unroll
    for (int i = 0; i < kSelParts; ++i) v[i] += a.partial[((size_t)b * a.nchunk + c) * kSelParts + i];
  block_reduce<kGFinBS, kSelParts, false>(v, red);
  const double S1 = v[0], S2 = v[1 + kNG];
  // events
  double u[1 + kNG];
#pragma unroll
  for (int i = 0; i <= kNG; ++i) u[i] = 0.0;
  int bad = 0;
  for (int e = threadIdx.x; e < a.E; e += kGFinBS) {
    const double li = a.lnI[(size_t)b * a.E + e];
    if (!(li > -INFINITY) || isnan(li)) bad = 1;
    u[0] += li;
#pragma unroll
    for (int p = 0; p < kNG; ++p) u[1 + p] += a.dlnI[((size_t)b * a.E + e) * kNG + p];
  }
  u[0] += bad ? -INFINITY : 0.0;
  block_reduce<kGFinBS, 1 + kNG, false>(u, red);
  if (threadIdx.x == 0) {
    double* g = a.grad + (size_t)b * kNG;
    if (flag) {
      a.lnl[b] = (flag & (kFlagDomain | kFlagNonMonotone)) ? -INFINITY : NAN;
      for (int p = 0; p < kNG; ++p) g[p] = NAN;
      return;
    }
    double lnl = S1 > 0.0 ? u[0] - (double)a.E * log(S1 / (double)a.n_total) : -INFINITY;
    if (a.neff_gate > 0.0 && isfinite(lnl) &&
        !(neff_of(S1, S2, a.n_total) > a.neff_gate * (double)a.E))
      lnl = -INFINITY;
    a.lnl[b] = lnl;
    const bool ok = isfinite(lnl);
    for (int p = 0; p < kNG; ++p)
      g[p] = ok ? u[1 + p] - (double)a.E * v[1 + p] / S1 : NAN;
  }
}

// ---------------------------------------------------------------------------
hipError_t launch_grad(const GradArgs& a, const SelGradArgs& sa, GradFinalArgs fa, bool f32,
                       hipStream_t st, const double* ntot, const double* missing) {
  k_lam_grad_prepare<<<(a.B + 63) / 64, 64, 0, st>>>(a.P, a.B, a.Q);
  CH_LAUNCH_CHECK();
  const long long ng = (long long)a.B * a.g.n_z;
  k_grid_grad<<<(unsigned)((ng + 255) / 256), 256, 0, st>>>(a.P, a.chi, a.chio, a.gz64, a.g,
                                                             a.B, a.gf64, a.gf32);
  CH_LAUNCH_CHECK();
  if (a.mz64) {
    k_completion_grad<<<a.B, kCompGradBS, 0, st>>>(a, ntot, missing, const_cast<double*>(sa.ntot),
                                                   const_cast<double*>(sa.dntot_om));
    CH_LAUNCH_CHECK();
  }
  if (sa.nchunk > 0) {
    dim3 grid(sa.nchunk, sa.B);
    k_selection_grad<<<grid, kSelGradBS, 0, st>>>(sa);
    CH_LAUNCH_CHECK();
  }
  const long long nb = item_lambda_blocks(a.E, a.B);
  if (a.E > 0) {
    k_event_bandwidth_grad<<<(unsigned)nb, kGradBS, 0, st>>>(a);
    CH_LAUNCH_CHECK();
    // binned sets: the window sums run over the bins' points
    GradArgs ab = a;
    if (a.bins > 0) {
      const long long bbk = item_lambda_blocks((a.n_slots + kGradBS / 64 - 1) / (kGradBS / 64), a.B);
      if (f32) k_bin_grad<true><<<(unsigned)bbk, kGradBS, 0, st>>>(a);
      else k_bin_grad<false><<<(unsigned)bbk, kGradBS, 0, st>>>(a);
      CH_LAUNCH_CHECK();
      ab.sc = a.bsc;
      ab.sd = a.bsd;
      ab.S = (long long)a.n_slots * a.bins;
    }
    const size_t lds32 = kGradStageElems * sizeof(float), lds64 = kGradStageElems * sizeof(double);
    const bool ep = a.shape == kShapeEpanechnikov;
    if (a.mz64) {
      if (ep) {
        if (f32) k_event_grad<true, true, true><<<(unsigned)nb, kGradBS, lds32, st>>>(ab);
        else k_event_grad<false, true, true><<<(unsigned)nb, kGradBS, lds64, st>>>(ab);
      } else {
        if (f32) k_event_grad<true, true, false><<<(unsigned)nb, kGradBS, lds32, st>>>(ab);
        else k_event_grad<false, true, false><<<(unsigned)nb, kGradBS, lds64, st>>>(ab);
      }
    } else {
      if (ep) {
        if (f32) k_event_grad<true, false, true><<<(unsigned)nb, kGradBS, lds32, st>>>(ab);
        else k_event_grad<false, false, true><<<(unsigned)nb, kGradBS, lds64, st>>>(ab);
      } else {
        if (f32) k_event_grad<true, false, false><<<(unsigned)nb, kGradBS, lds32, st>>>(ab);
        else k_event_grad<false, false, false><<<(unsigned)nb, kGradBS, lds64, st>>>(ab);
      }
    }
    CH_LAUNCH_CHECK();
  }
  k_grad_final<<<a.B, kGFinBS, 0, st>>>(fa);
  CH_LAUNCH_CHECK();
  return hipSuccess;
}

int selection_grad_chunks(long long n_det) {
  const long long per = (long long)kSelGradBS * kSelGradPer;
  return (int)((n_det + per - 1) / per);
}

}  // namespace chimera
