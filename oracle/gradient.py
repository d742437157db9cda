"""d ln L / d lambda (TEST INFRASTRUCTURE; see package header).

Analytic chain rule through every step of likelihood.lnl, written out in the
redshift variable z, for the 12 parameters

    (H0, Om, Xi0, n, alpha, beta, mu_g, sigma_g, lambda_g, gamma, kappa, z_p);

mmin and mmax are hard edges of the mass model (ln L jumps when a sample
crosses them) and are held fixed.  Pieces:

* distances (eq. dL-em, eq. dL-mg): dD/dH0 = -D/H0;
  dD/dOm = (c/H0)(1+z) Xi dchi/dOm with dchi/dOm = -1/2 int_0^z ((1+z')^3-1)/E^3;
  dD/dXi0 = D_em (1 - (1+z)^-n); dD/dn = -D_em (1-Xi0)(1+z)^-n ln(1+z);
  a sample's redshift moves by dz/dp = -(dD/dp) / (dD/dz) (implicit function
  of D(z_j) = d_j);
* masses: w = p(m1) p(m2|m1) at m = m_det/(1+z): the direct derivatives in
  (alpha, beta, mu_g, sigma_g, lambda_g) and the path through z;
* bandwidth (Scott/Kish reading): ln h = 1/2 ln V - 1/2 ln(W1 - W2/W1)
  - 1/5 ln(W1^2/W2), differentiated through W1, W2 and V = sum w (z-mu)^2;
  0 where the 2 dz floor or the zero-variance branch is taken;
* kernel sums: dA/dz_j = sum F K (z_g - z_j)/h^2, dA/dh = sum F K (z_g-z_j)^2/h^3,
  and the grid factor g = psi / ((1+z)^3 D') differentiated on the grid;
  the window edges |z_g - z_j| = T h are not differentiated (their terms
  carry the kernel's value e^(-T^2/2) at the edge); the Epanechnikov kernel
  (Sect. 2.3's compact option) the same way with its polynomial k;
* selection: s_j = w n_tot psi / ((1+z)^3 D' p_draw) along the same chain,
  with n_tot linear between grid nodes;
* incomplete catalogue (eqs. p-gal, p-miss, f-R): the rows f_R n_r +
  (1 - P_r) v and n_tot^eff = f_R n_tot + M v depend on Om through the
  completion density v = chi^2 / (E (4 pi/3) chi(z_max)^3) and through
  f_R = sum_g tau_g (4 pi - M) v; d ln v / d Om = 2 chi'/chi - E'/E -
  3 chi'(z_max)/chi(z_max) with chi' = d chi / d Om and E' = ((1+z)^3 - 1)/(2E).

The lambda-only normalisation derivatives of the mass model: the power
law's by quadrature (scipy quad) of the differentiated density, the
truncated Gaussian's from d Phi / dt = phi.

Pins (tests/test_oracle_gradient.py): each piece against Richardson central
differences of the oracle function it differentiates; the whole gradient
against Richardson differences of likelihood.lnl on small inputs, also with
an incomplete catalogue; dlnL/dn = 0 exactly at Xi0 = 1 and dlnL/dXi0 = 0
exactly at n = 0.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate
from scipy.special import ndtr

from . import cosmology as cosmo
from . import likelihood as L
from .population import mass_weight, psi

# positions in the 14-entry lambda of the 12 differentiated parameters
GRAD_INDEX = (0, 1, 2, 3, 4, 5, 8, 9, 10, 11, 12, 13)
NG = len(GRAD_INDEX)
_H0, _OM, _XI0, _N, _ALPHA, _BETA, _MU, _SIG, _LG, _GAM, _KAP, _ZP = range(NG)


# ---------------------------------------------------------------------------
# distances
# ---------------------------------------------------------------------------
def _dchi_panel(a, b, om):
    t = 0.5 * (b - a)[..., None] * cosmo._GL_X + 0.5 * (a + b)[..., None]
    f = ((1.0 + t) ** 3 - 1.0) / cosmo.efunc(t, om) ** 3
    return 0.5 * (b - a) * np.sum(cosmo._GL_W * f, axis=-1)


_DCHI_CACHE: dict = {}


def dchi_dom(z, om):
    """d chi / d Om = -1/2 int_0^z ((1+z')^3 - 1) / E(z')^3 dz' (composite
    24-point Gauss-Legendre on the panels of chi)."""
    z = np.asarray(z, dtype=np.float64)
    key = float(om)
    if key not in _DCHI_CACHE:
        n = int(math.ceil(cosmo.Z_MAX / cosmo.PANEL)) + 2
        edges = cosmo.PANEL * np.arange(n + 1)
        _DCHI_CACHE[key] = np.concatenate([[0.0], np.cumsum(_dchi_panel(edges[:-1], edges[1:], om))])
        if len(_DCHI_CACHE) > 512:
            _DCHI_CACHE.pop(next(iter(_DCHI_CACHE)))
    pre = _DCHI_CACHE[key]
    k = np.clip(np.floor(z / cosmo.PANEL).astype(np.int64), 0, len(pre) - 2)
    return -0.5 * (pre[k] + _dchi_panel(cosmo.PANEL * k, z, om))


def distance_parts(z, lam):
    """D, dD/dz, d2D/dz2 and the parameter derivatives dD/dp, d(dD/dz)/dp for
    p = H0, Om, Xi0, n (arrays [4, len(z)])."""
    h0, om, xi0, n = lam[0], lam[1], lam[2], lam[3]
    z = np.asarray(z, dtype=np.float64)
    dh = cosmo.C_KM_S / h0
    zp1 = 1.0 + z
    E = cosmo.efunc(z, om)
    E_z = 1.5 * om * zp1 ** 2 / E
    chi = cosmo.chi(z, om)
    chi_z = 1.0 / E
    chi_zz = -E_z / E ** 2
    chi_om = dchi_dom(z, om)
    chi_z_om = -0.5 * (zp1 ** 3 - 1.0) / E ** 3
    pw = zp1 ** (-n)
    lz = np.log(zp1)
    Xi = xi0 + (1.0 - xi0) * pw
    Xi_z = -n * (1.0 - xi0) * pw / zp1
    Xi_zz = n * (n + 1.0) * (1.0 - xi0) * pw / zp1 ** 2
    D_em = dh * zp1 * chi
    D = D_em * Xi
    # D_z / dh = chi Xi + (1+z) chi_z Xi + (1+z) chi Xi_z
    Dz = dh * (chi * Xi + zp1 * chi_z * Xi + zp1 * chi * Xi_z)
    Dzz = dh * (2.0 * chi_z * Xi + 2.0 * chi * Xi_z + zp1 * chi_zz * Xi
                + 2.0 * zp1 * chi_z * Xi_z + zp1 * chi * Xi_zz)
    dD = np.empty((4,) + z.shape)
    dDz = np.empty((4,) + z.shape)
    # H0
    dD[0] = -D / h0
    dDz[0] = -Dz / h0
    # Om
    dD[1] = dh * zp1 * Xi * chi_om
    dDz[1] = dh * (chi_om * Xi + zp1 * chi_z_om * Xi + zp1 * chi_om * Xi_z)
    # Xi0: dXi/dXi0 = 1 - (1+z)^-n, dXi_z/dXi0 = n (1+z)^(-n-1)
    xa, xa_z = 1.0 - pw, n * pw / zp1
    dD[2] = D_em * xa
    dDz[2] = dh * (chi * xa + zp1 * chi_z * xa + zp1 * chi * xa_z)
    # n: dXi/dn = -(1-Xi0)(1+z)^-n ln(1+z), dXi_z/dn = -(1-Xi0)(1+z)^(-n-1)(1 - n ln(1+z))
    xn = -(1.0 - xi0) * pw * lz
    xn_z = -(1.0 - xi0) * pw / zp1 * (1.0 - n * lz)
    dD[3] = D_em * xn
    dDz[3] = dh * (chi * xn + zp1 * chi_z * xn + zp1 * chi * xn_z)
    return D, Dz, Dzz, dD, dDz


def dz_dparams(z, lam):
    """[12, len(z)]: dz_j/dp = -(dD/dp)/(dD/dz) for the distance parameters,
    0 for the population parameters."""
    _, Dz, _, dD, _ = distance_parts(z, lam)
    out = np.zeros((NG,) + np.shape(z))
    out[:4] = -dD / Dz
    return out


# ---------------------------------------------------------------------------
# masses
# ---------------------------------------------------------------------------
def _mass_norm_derivs(lam):
    """Normalisations of p(m1) and their parameter derivatives: the power law's
    by quadrature, the truncated peak's in closed form."""
    alpha, mmin, mmax, mu, sg = lam[4], lam[6], lam[7], lam[8], lam[9]
    opts = dict(epsabs=0.0, epsrel=1e-13, limit=200)
    npl = integrate.quad(lambda m: m ** (-alpha), mmin, mmax, **opts)[0]
    dnpl_da = integrate.quad(lambda m: -math.log(m) * m ** (-alpha), mmin, mmax, **opts)[0]
    a, b = (mmin - mu) / sg, (mmax - mu) / sg
    Z = ndtr(-a) - ndtr(-b) if a > 0 else ndtr(b) - ndtr(a)
    # Z = Phi(b) - Phi(a): dZ/dmu = (phi(a) - phi(b)) / sigma,
    # dZ/dsigma = (a phi(a) - b phi(b)) / sigma
    phi = lambda t: math.exp(-0.5 * t * t) / math.sqrt(2.0 * math.pi)  # noqa: E731
    dZ_dmu = (phi(a) - phi(b)) / sg
    dZ_ds = (a * phi(a) - b * phi(b)) / sg
    return npl, dnpl_da, Z, dZ_dmu, dZ_ds


def mass_log_derivs(m1, m2, lam):
    """For source-frame masses with w > 0: d ln w / d(alpha, beta, mu_g,
    sigma_g, lambda_g) [5, n] and m1 d ln w/dm1 + m2 d ln w/dm2 [n]."""
    alpha, beta, mmin, mu, sg, lg = lam[4], lam[5], lam[6], lam[8], lam[9], lam[10]
    m1 = np.asarray(m1, dtype=np.float64)
    m2 = np.asarray(m2, dtype=np.float64)
    npl, dnpl_da, Z, dZ_dmu, dZ_ds = _mass_norm_derivs(lam)
    PL = m1 ** (-alpha) / npl
    u = (m1 - mu) / sg
    TG = np.exp(-0.5 * u * u) / (sg * math.sqrt(2.0 * math.pi) * Z)
    p1 = (1.0 - lg) * PL + lg * TG
    d = np.zeros((5,) + m1.shape)
    d[0] = (1.0 - lg) * PL * (-np.log(m1) - dnpl_da / npl) / p1
    d[2] = lg * TG * (u / sg - dZ_dmu / Z) / p1
    d[3] = lg * TG * (-1.0 / sg + u * u / sg - dZ_ds / Z) / p1
    d[4] = (TG - PL) / p1
    # p(m2|m1) = m2^beta / n2, n2 = int_mmin^m1 m^beta dm
    a = 1.0 + beta
    l1, l2, lmin = np.log(m1), np.log(m2), math.log(mmin)
    if a == 0.0:
        n2 = l1 - lmin
        dn2 = 0.5 * (l1 ** 2 - lmin ** 2)
    else:
        n2 = (m1 ** a - mmin ** a) / a
        # int m^beta ln m dm = m^a (ln m / a - 1/a^2)
        dn2 = m1 ** a * (l1 / a - 1.0 / a ** 2) - mmin ** a * (lmin / a - 1.0 / a ** 2)
    d[1] = l2 - dn2 / n2
    # mass derivatives at fixed parameters
    dlp1_dm1 = ((1.0 - lg) * PL * (-alpha / m1) + lg * TG * (-u / sg)) / p1
    dl_dm1 = dlp1_dm1 - m1 ** beta / n2
    dl_dm2 = beta / m2
    return d, m1 * dl_dm1 + m2 * dl_dm2


def sample_log_weight_grad(z, m1d, m2d, lam):
    """(w, d ln w / dp [12, n] with the path through z, dz/dp [12, n]) where w > 0."""
    zp1 = 1.0 + z
    m1, m2 = m1d / zp1, m2d / zp1
    w = mass_weight(m1, m2, lam)
    dz = dz_dparams(z, lam)
    g = np.zeros((NG,) + np.shape(z))
    pos = w > 0
    if np.any(pos):
        dm, mdm = mass_log_derivs(m1[pos], m2[pos], lam)
        for k, p in enumerate((_ALPHA, _BETA, _MU, _SIG, _LG)):
            g[p, pos] = dm[k]
        dlw_dz = -mdm / zp1[pos]          # m = m_det/(1+z): d ln m / dz = -1/(1+z)
        g[:4, pos] = dlw_dz[None, :] * dz[:4, pos]
    return w, g, dz


# ---------------------------------------------------------------------------
# rate and grid factor
# ---------------------------------------------------------------------------
def psi_log_derivs(z, lam):
    """d ln psi / d(gamma, kappa, z_p) [3, n] and d ln psi / dz [n]."""
    gam, kap, zp = lam[11], lam[12], lam[13]
    zp1 = 1.0 + np.asarray(z, dtype=np.float64)
    lr = np.log(zp1 / (1.0 + zp))
    r = np.exp((gam + kap) * lr)
    s = r / (1.0 + r)
    d = np.stack([np.log(zp1) - s * lr, -s * lr, s * (gam + kap) / (1.0 + zp)])
    return d, gam / zp1 - s * (gam + kap) / zp1


def grid_factor_log_derivs(grid, lam):
    """d ln g / dp on the grid [12, n_z], g = psi / ((1+z)^3 dD/dz)."""
    _, Dz, _, _, dDz = distance_parts(grid, lam)
    out = np.zeros((NG, grid.size))
    out[:4] = -dDz / Dz
    dpsi, _ = psi_log_derivs(grid, lam)
    out[_GAM:] = dpsi
    return out


def completion_density_dom(z, om, z_max):
    """d v / d Om of likelihood.completion_density (0 at z = 0, where v = 0)."""
    z = np.asarray(z, dtype=np.float64)
    v = L.completion_density(z, om, z_max)
    ch = cosmo.chi(z, om)
    e = cosmo.efunc(z, om)
    dlv = (2.0 * dchi_dom(z, om) / np.where(ch > 0.0, ch, 1.0)
           - ((1.0 + z) ** 3 - 1.0) / (2.0 * e * e)
           - 3.0 * float(dchi_dom(np.array([z_max]), om)[0]) / float(cosmo.chi(z_max, om)))
    return np.where(ch > 0.0, v * dlv, 0.0)


def galaxy_density_dom(cat: L.Catalog, lam):
    """(d rows / d Om, d n_tot / d Om) of likelihood.galaxy_density with an
    incomplete catalogue: f_R' n_r + (1 - P_r) v' and f_R' n_tot + M v',
    f_R' = sum_g tau_g (4 pi - M) v'."""
    dv = completion_density_dom(cat.grid, lam[1], cat.grid[-1])
    df = float(np.sum(L.trapezoid(cat.grid) * (4.0 * math.pi - cat.missing) * dv))
    drows = {p: df * r + (1.0 - cat.p_compl[p]) * dv for p, r in cat.rows.items()}
    return drows, df * cat.n_tot + cat.missing * dv


# ---------------------------------------------------------------------------
# bandwidth
# ---------------------------------------------------------------------------
def bandwidth_grad(z, w, dlw, dz_p, dz_grid):
    """(h, d ln h / dp [12]) of the Scott/Kish rule; None when W1 = 0."""
    W1 = float(np.sum(w))
    if not W1 > 0:
        return None, None
    W2 = float(np.sum(w * w))
    mu = float(np.sum(w * z)) / W1
    h = L.bandwidth(z, w, dz_grid)
    dlnh = np.zeros(NG)
    if W1 * W1 - W2 <= 1e-12 * W1 * W1:
        return h, dlnh
    V = float(np.sum(w * (z - mu) ** 2))
    den = W1 - W2 / W1
    raw = math.sqrt(V / den) * (W1 * W1 / W2) ** (-0.2)
    if raw < 2.0 * dz_grid or V == 0.0:
        return h, dlnh
    dW1 = dlw @ w
    dW2 = dlw @ (2.0 * w * w)
    # sum w (z - mu) = 0 removes the d mu term
    dV = dlw @ (w * (z - mu) ** 2) + dz_p @ (2.0 * w * (z - mu))
    dden = dW1 - dW2 / W1 + W2 * dW1 / W1 ** 2
    dlnh = 0.5 * dV / V - 0.5 * dden / den - 0.2 * (2.0 * dW1 / W1 - dW2 / W2)
    return h, dlnh


# ---------------------------------------------------------------------------
# one event, selection, ln L
# ---------------------------------------------------------------------------
def binned_points(z, w, dlw, dz, n_bins):
    """The binned data set (likelihood.bin_samples) with its derivatives:
    (centres, weights, d weights / dp [NG, n_bins], d centres / dp [NG, n_bins]).
    The bins' edges follow the smallest and largest redshift, so a centre
    moves as (1 - f) dz_lo/dp + f dz_hi/dp with f = (k + 1/2) / n_bins; a
    bin's weight as the sum of its samples' w d ln w / dp (the samples' bins
    held fixed)."""
    centres, weights = L.bin_samples(z, w, n_bins)
    lo, hi = int(np.argmin(z)), int(np.argmax(z))
    width = (float(z[hi]) - float(z[lo])) / n_bins
    if width > 0.0:
        idx = np.minimum(np.floor((z - float(z[lo])) / width).astype(np.int64), n_bins - 1)
        f = (np.arange(n_bins) + 0.5) / n_bins
        dc = np.outer(dz[:, lo], 1.0 - f) + np.outer(dz[:, hi], f)
    else:
        idx = np.zeros(z.size, dtype=np.int64)
        dc = np.repeat(dz[:, lo:lo + 1], n_bins, axis=1)
    dW = np.zeros((dlw.shape[0], n_bins))
    for j, b in enumerate(idx):
        dW[:, b] += w[j] * dlw[:, j]
    return centres, weights, dW, dc


def event_grad(pix_z, pix_w, pix_dlw, pix_dz, pix_c, pix_rows, grid, tau, gz, dlng, T=None,
               pix_drows=None, shape="gaussian", n_bins=0):
    """(I_i, d ln I_i / dp [12]); pix_drows: d row / d Om of each pixel's row
    (an incomplete catalogue), or None.

    shape "epanechnikov" (the compact kernel of Sect. 2.3, scaled to variance
    h^2: 3 / (4 a h) (1 - u^2 / (a h)^2) on |u| <= a h, a = sqrt(5); T unused):
    with k = 1 - u^2 / (a h)^2 inside the support, dk/dz_j = 2 u / (a h)^2 and
    dk/dh = 2 u^2 / ((a h)^2 h); k vanishes on the support's edge, so grid
    points entering or leaving it add nothing to the derivative."""
    if shape not in ("gaussian", "epanechnikov"):
        raise ValueError(f"unknown kernel shape {shape!r}")
    dzg = grid[1] - grid[0]
    z = np.concatenate(pix_z)
    w = np.concatenate(pix_w)
    dlw = np.concatenate(pix_dlw, axis=1)
    dzp = np.concatenate(pix_dz, axis=1)
    h, dlnh = bandwidth_grad(z, w, dlw, dzp, dzg)
    if h is None:
        return 0.0, np.full(NG, np.nan)
    S = 0.0
    G = np.zeros(NG)
    drs = pix_drows if pix_drows is not None else [None] * len(pix_rows)
    for zr, wr, lw, zz, c, nr, dnr in zip(pix_z, pix_w, pix_dlw, pix_dz, pix_c, pix_rows, drs):
        if n_bins:
            # the bins stand in for the samples: a bin's w d ln w / dp is its
            # dW / dp, and its centre moves with the range's ends
            zr, wr, dW, dc = binned_points(zr, wr, lw, zz, n_bins)
            with np.errstate(divide="ignore", invalid="ignore"):
                lw = np.where(wr > 0, dW / np.where(wr > 0, wr, 1.0), 0.0)
            zz = dc
        f = tau * nr * gz
        u = grid[None, :] - zr[:, None]
        if shape == "epanechnikov":
            ah = L.EPAN_SCALE * h
            inside = np.abs(u) <= ah
            k = np.where(inside, 1.0 - (u / ah) ** 2, 0.0)
            fk = k * f[None, :]
            fi = np.where(inside, f[None, :], 0.0)
            A = fk.sum(axis=1)
            B = 2.0 * (fi * u).sum(axis=1) / ah ** 2              # dA/dz_j
            C = 2.0 * (fi * u * u).sum(axis=1) / (ah ** 2 * h)    # dA/dh
        else:
            k = np.exp(-0.5 * (u / h) ** 2)
            if T is not None:
                k = np.where(np.abs(u) <= T * h, k, 0.0)
            fk = k * f[None, :]
            A = fk.sum(axis=1)
            B = (fk * u).sum(axis=1) / h ** 2          # dA/dz_j
            C = (fk * u * u).sum(axis=1) / h ** 3      # dA/dh
        Eg = fk @ dlng.T                            # [n_j, 12]: sum F K dln g/dp
        S += c * float(wr @ A)
        G += c * (lw @ (wr * A) + zz @ (wr * B) + float(wr @ C) * h * dlnh + Eg.T @ wr)
        if dnr is not None:          # the row's own Om dependence
            G[_OM] += c * float(wr @ (k @ (tau * dnr * gz)))
    if not S > 0:
        return 0.0, np.full(NG, np.nan)
    if shape == "epanechnikov":
        I = S * 0.75 / (L.EPAN_SCALE * h)
    else:
        I = S / (h * math.sqrt(2.0 * math.pi))
    return I, G / S - dlnh


def selection_grad(inj: L.InjectionSet, cat: L.Catalog, lam):
    """(xi, d ln xi / dp [12])."""
    z = cosmo.invert_dl(inj.dl, lam[0], lam[1], lam[2], lam[3])
    w, dlw, dzp = sample_log_weight_grad(z, inj.m1d, inj.m2d, lam)
    grid = cat.grid
    _, n_tot, _ = L.galaxy_density(cat, lam)
    ntot = np.interp(z, grid, n_tot, left=0.0, right=0.0)
    # slope of the linear interpolation on the segment that holds z
    k = np.clip(np.searchsorted(grid, z, side="right") - 1, 0, grid.size - 2)
    slope = (n_tot[k + 1] - n_tot[k]) / (grid[k + 1] - grid[k])
    _, Dz, Dzz, _, dDz = distance_parts(z, lam)
    ps = psi(z, lam[11], lam[12], lam[13])
    s = w * ntot * ps / ((1.0 + z) ** 3 * Dz * np.exp(inj.ln_pdraw))
    S1 = float(np.sum(s))
    if not S1 > 0:
        return 0.0, np.full(NG, np.nan)
    pos = s > 0
    dpsi, dlpsi_dz = psi_log_derivs(z, lam)
    dls_dz = np.where(pos, slope / np.where(pos, ntot, 1.0), 0.0) + dlpsi_dz \
        - 3.0 / (1.0 + z) - Dzz / Dz
    dls = dlw + dls_dz[None, :] * dzp
    dls[:4] -= dDz / Dz
    dls[_GAM:] += dpsi
    if cat.p_compl is not None:        # n_tot^eff's own Om dependence
        _, dnt = galaxy_density_dom(cat, lam)
        dls[_OM] += np.where(pos, np.interp(z, grid, dnt, left=0.0, right=0.0)
                             / np.where(pos, ntot, 1.0), 0.0)
    return S1 / inj.n_total, (dls[:, pos] @ s[pos]) / S1


def lnl_grad(events, cat: L.Catalog, inj: L.InjectionSet, lam, T=None, kernel="many1d",
             shape="gaussian", n_bins=0):
    """dict(lnl, grad[12], lnI[E], dlnI[E, 12], ln_xi, dln_xi[12]).

    shape: the KDE kernel, "gaussian" or "epanechnikov" (see event_grad);
    n_bins > 0: the binned data sets (binned_points; the bandwidth stays the
    samples').

    kernel "single1d" (eq. gw-kernel-single1d): the sum over pixels of S_ir
    times the grid sum of n_r g KDE is, by linearity, the grid sum of
    (sum_r S_ir n_r) g KDE, i.e. one pixel holding all N_i samples with
    c = 1/N_i and that row; event_grad then applies unchanged.
    grad is NaN where lnl is not finite."""
    if kernel not in ("many1d", "single1d"):
        raise ValueError(f"unknown kernel {kernel!r}")
    if len(lam) > 14:
        raise NotImplementedError("the gradient of the smoothed mass model is not built")
    lam = np.asarray(lam, dtype=np.float64)
    E = len(events)
    out = {"lnl": -np.inf, "grad": np.full(NG, np.nan), "lnI": np.full(E, -np.inf),
           "dlnI": np.full((E, NG), np.nan), "ln_xi": np.nan, "dln_xi": np.full(NG, np.nan)}
    if not L.lambda_in_domain(lam):
        return out
    grid = cat.grid
    tau = L.trapezoid(grid)
    rows, _, _ = L.galaxy_density(cat, lam)
    drows = galaxy_density_dom(cat, lam)[0] if cat.p_compl is not None else None
    try:
        gz = L.grid_factor(grid, lam)
        dlng = grid_factor_log_derivs(grid, lam)
        xi, dlnxi = selection_grad(inj, cat, lam)
        per_event = []
        for ev in events:
            zs, ws, lws, zzs, cs, rs, drs = [], [], [], [], [], [], []
            if kernel == "single1d":
                dl, m1d, m2d = ev.all_samples()
                parts = [(dl, m1d, m2d, 1.0 / dl.size,
                          sum(px.sky() * rows[px.pix] for px in ev.pixels),
                          None if drows is None else
                          sum(px.sky() * drows[px.pix] for px in ev.pixels))]
            else:
                parts = [(px.dl, px.m1d, px.m2d, px.c, rows[px.pix],
                          None if drows is None else drows[px.pix]) for px in ev.pixels]
            for dl, m1d, m2d, c, row, drow in parts:
                z = cosmo.invert_dl(dl, lam[0], lam[1], lam[2], lam[3])
                if np.any(np.isnan(z)):
                    out["lnl"] = np.nan
                    return out
                w, lw, zz = sample_log_weight_grad(z, m1d, m2d, lam)
                zs.append(z); ws.append(w); lws.append(lw); zzs.append(zz)
                cs.append(c); rs.append(row); drs.append(drow)
            per_event.append(event_grad(zs, ws, lws, zzs, cs, rs, grid, tau, gz, dlng, T,
                                        drs if drows is not None else None, shape,
                                        n_bins))
    except cosmo.NonMonotone:
        return out
    out["ln_xi"] = math.log(xi) if xi > 0 else -np.inf
    out["dln_xi"] = dlnxi
    for i, (I, g) in enumerate(per_event):
        out["lnI"][i] = math.log(I) if I > 0 else -np.inf
        out["dlnI"][i] = g
    if np.all(np.isfinite(out["lnI"])) and xi > 0:
        out["lnl"] = float(np.sum(out["lnI"]) - E * math.log(xi))
        out["grad"] = out["dlnI"].sum(axis=0) - E * dlnxi
    return out


# ---------------------------------------------------------------------------
# Richardson-extrapolated central differences
# ---------------------------------------------------------------------------
def richardson(fun, lam, p_index, rel_step=1e-4, abs_floor=1e-6):
    """d fun / d lam[p_index]: central differences at steps h and h/2 combined
    as (4 D(h/2) - D(h)) / 3."""
    lam = np.asarray(lam, dtype=np.float64)
    h = max(abs(lam[p_index]) * rel_step, abs_floor)

    def central(step):
        lp, lm = lam.copy(), lam.copy()
        lp[p_index] += step
        lm[p_index] -= step
        return (fun(lp) - fun(lm)) / (2.0 * step)

    return (4.0 * central(0.5 * h) - central(h)) / 3.0
