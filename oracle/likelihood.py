"""ln L(lambda) for the many-1D galaxy-catalogue likelihood (TEST INFRASTRUCTURE).

Follows Sect. 2 of the paper:

eq. hyperlike   ln L = sum_i ln I_i - N_obs ln xi   (reading: no additive
                constant; the proportionality sign is taken as equality)
eq. like-integrals + eq. gw-kernel-many1d
                I_i = sum_{pixels r} c_ir sum_{j in r} w_j A_j,
                A_j = sum_g tau_g N(z_g; z_j, h_i) n_r(z_g) g(z_g),
                g(z) = psi(z) / [(1+z)^3 d d_L^gw/dz]   (eq. jacobian, with
                p_cbc = p_cat psi, complete catalogue f_R = 1)
                The KDE is (1/N_r) sum_j w_j N(z; z_j, h): not divided by
                sum w (reading), the 1/N_r sits in c_ir.
eqs. p-gal, p-miss, f-R (galaxy_density): with a completeness P_compl per
                pixel the rows and n_tot become those of
                p_gal = f_R p_cat + (1 - f_R) p_miss, homogeneous completion
                in comoving volume up to the grid's end (reading).
Sect. 2.2       xi = (1/N_inj) sum_{detected} s_j,
                s_j = p(m1,m2) n_tot(z_j) psi(z_j) / [(1+z_j)^3 D'(z_j) p_draw_j]
                (reading: the 1/p_draw of the cited estimators is restored;
                the sky integral of p_cat is n_tot since detection does not
                depend on the sky), N_eff as printed with sums over detected.

eq. gw-kernel-single1d (the single-1D kernel of Sect. 2.3)
                one weighted KDE per event over all its N_i samples (those
                outside the pixels of its region included),
                KDE(z) = (1/N_i) sum_j w_j N(z; z_j, h_i), h_i from the same
                N_i samples, times each pixel's 2-D sky factor S_ir:
                I_i = sum_r S_ir sum_g tau_g n_r(z_g) g(z_g) KDE(z_g)
                (same weights, bandwidth rule and window as many-1D).

The 3D kernel (Sect. 2.2, kept in Sect. 2.3; event_integral_3d) one Gaussian
                KDE of the event's N_i samples in (z, u, v), (u, v) a flat sky
                chart of the event (reading: the gnomonic plane at the samples'
                mean direction), evaluated at each region pixel's centre and
                integrated over the pixel as area x value; bandwidth matrix:
                weighted covariance x n_eff^(-2/7) (reading: Scott's rule in
                3-D, as scipy's gaussian_kde).

Kernel options of Sect. 2.3 (kernel_values, bin_samples): the Epanechnikov
                kernel in place of the Gaussian (reading: variance h^2, support
                sqrt(5) h), and binned data sets (reading: n_bins equal-width
                bins over each KDE's sample range, one point per bin at its
                centre with the bin's summed weight).

Bandwidth (the paper is silent; reading): one Gaussian bandwidth per
(event, lambda) from all of the event's in-region samples: Scott's rule with
the Kish effective size n_eff = W1^2/W2 and the unbiased weighted variance,
h = max(sigma * n_eff^(-1/5), 2 dz); sigma = 0 when W1^2 - W2 <= 1e-12 W1^2.
This is scipy.stats.gaussian_kde's weighted Scott rule (the pin).

Kernel support: T=None sums over the whole grid (the dense definition);
a finite T keeps grid points with |z_g - z_j| <= T h (the paper evaluates
the kernels only where samples are, Sect. 2.3).

Degenerate values: I_i = 0 or xi = 0 gives ln L = -inf; a lambda outside the
domain (H0 <= 0, Om outside (0,1], Xi0 <= 0, mmin >= mmax, sigma_g <= 0,
lambda_g outside [0,1], z_p <= -1, non-finite, or d_L^gw not increasing on
[0, 25]) gives -inf; a distance beyond d_L^gw(25) gives NaN.

Pins: tests/test_oracle_likelihood.py (KDE vs scipy gaussian_kde, grid
normalisation of the Gaussian, Gaussian-convolution closed form, constant
rescalings, permutations, distance-scaling identity, the analytic xi of a
draw density proportional to the population).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.special import ndtr

from . import cosmology as cosmo
from .population import mass_weight, psi


@dataclass
class Pixel:
    pix: int
    c: float
    dl: np.ndarray
    m1d: np.ndarray
    m2d: np.ndarray
    s: float = None           # sky factor S_ir (None: c x the pixel's sample count)
    uv: tuple = None          # centre in the event's flat sky chart (the 3D kernel)
    area: float = None        # pixel area [sr] (the 3D kernel)

    def sky(self) -> float:
        return self.s if self.s is not None else self.c * self.dl.size


@dataclass
class Event:
    pixels: list = field(default_factory=list)
    # every sample of the event, in and out of its pixels, as (dl, m1d, m2d);
    # None: the pixels' samples (the single-1D KDE is trained on these)
    samples: tuple = None
    # (u, v) of every sample in the event's flat sky chart, in the order of
    # `samples` (the 3D kernel)
    sky_uv: tuple = None

    def all_samples(self):
        if self.samples is not None:
            return self.samples
        return tuple(np.concatenate([getattr(px, a) for px in self.pixels])
                     for a in ("dl", "m1d", "m2d"))


@dataclass
class Catalog:
    grid: np.ndarray          # z_g, uniform
    rows: dict                # HEALPix id -> n_r(z_g)
    n_tot: np.ndarray
    # incompleteness (eqs. p-gal, p-miss, f-R); None: a complete catalogue
    p_compl: dict = None      # HEALPix id -> P_compl(z_g) of the pixel
    missing: np.ndarray = None  # M(z_g) = sum over all pixels of area x (1 - P_compl) [sr]


def completion_density(z, om, z_max):
    """v(z) = (dV_c/dz per steradian) / V_c(z_max): the homogeneous completion
    of eq. p-miss as a density in (z, Omega); H0 cancels, so
    v = chi(z)^2 / (E(z) (4 pi / 3) chi(z_max)^3)."""
    return (cosmo.chi(z, om) ** 2 / cosmo.efunc(z, om)
            / (4.0 * math.pi / 3.0 * float(cosmo.chi(z_max, om)) ** 3))


def galaxy_density(cat: Catalog, lam):
    """(rows, n_tot, f_R) of p_gal = f_R p_cat + (1 - f_R) p_miss (eqs. p-gal,
    p-miss, f-R) on the grid at lambda.  With P_compl per pixel and
    v = completion_density (z_max = the grid's end):
      (1 - f_R) p_miss = (1 - P_compl) v,
      f_R = int dz dOmega P_compl v = sum_g tau_g (4 pi - M(z_g)) v(z_g)
    (the trapezoid on the grid; reading), so a pixel's row becomes
    f_R n_r + (1 - P_r) v and the all-sky density f_R n_tot + M v (linear
    between nodes, as n_tot).  A complete catalogue gives the rows as they are."""
    if cat.p_compl is None:
        return cat.rows, cat.n_tot, 1.0
    v = completion_density(cat.grid, lam[1], cat.grid[-1])
    f_r = float(np.sum(trapezoid(cat.grid) * (4.0 * math.pi - cat.missing) * v))
    rows = {p: f_r * r + (1.0 - cat.p_compl[p]) * v for p, r in cat.rows.items()}
    return rows, f_r * cat.n_tot + cat.missing * v, f_r


@dataclass
class InjectionSet:
    dl: np.ndarray
    m1d: np.ndarray
    m2d: np.ndarray
    ln_pdraw: np.ndarray
    n_total: int


def trapezoid(grid):
    dz = grid[1] - grid[0]
    tau = np.full(grid.size, dz)
    tau[0] = tau[-1] = 0.5 * dz
    return tau


def lambda_in_domain(lam) -> bool:
    lam = np.asarray(lam, dtype=np.float64)
    if not np.all(np.isfinite(lam)):
        return False
    h0, om, xi0, _n, _a, _b, mmin, mmax, mu, sg, lg, _g, _k, zp = lam[:14]
    if not (h0 > 0 and 0 < om <= 1 and xi0 > 0 and 0 < mmin < mmax and sg > 0
            and 0 <= lg <= 1 and zp > -1):
        return False
    if lam.size > 14 and not lam[14] >= 0:      # delta_m (the smoothed mass edge)
        return False
    # reading: a Gaussian peak with no mass inside [mmin, mmax] cannot be normalised
    a, b = (mmin - mu) / sg, (mmax - mu) / sg
    return (ndtr(-a) - ndtr(-b) if a > 0 else ndtr(b) - ndtr(a)) > 0


def redshift_and_weight(dl, m1d, m2d, lam):
    """z_j from d_L^gw (Sect. 2.1), source masses m = m_det/(1+z), w = p(m1,m2)."""
    z = cosmo.invert_dl(dl, lam[0], lam[1], lam[2], lam[3])
    w = mass_weight(m1d / (1.0 + z), m2d / (1.0 + z), lam)
    return z, w


def bandwidth(z, w, dz):
    w1 = np.sum(w)
    if not w1 > 0:
        return None
    w2 = np.sum(w * w)
    mu = np.sum(w * z) / w1
    if w1 * w1 - w2 <= 1e-12 * w1 * w1:
        var = 0.0
    else:
        var = np.sum(w * (z - mu) ** 2) / (w1 - w2 / w1)
    neff = w1 * w1 / w2
    return max(math.sqrt(var) * neff ** (-0.2), 2.0 * dz)


def grid_factor(grid, lam):
    h0, om, xi0, n = lam[0], lam[1], lam[2], lam[3]
    return psi(grid, lam[11], lam[12], lam[13]) / (
        (1.0 + grid) ** 3 * cosmo.ddl_gw_dz(grid, h0, om, xi0, n))


EPAN_SCALE = math.sqrt(5.0)


def kernel_values(grid, z, h, shape="gaussian", T=None):
    """[len(z), len(grid)] kernel K(z_g; z_j, h), each integrating to 1 in z.

    "gaussian": N(z_g; z_j, h), kept where |z_g - z_j| <= T h when T is given.
    "epanechnikov" (the compact option of Sect. 2.3; reading: scaled to the
    variance h^2 so that the same bandwidth rule applies):
    3 / (4 a h) max(0, 1 - ((z_g - z_j) / (a h))^2), a = sqrt(5); T is unused
    (the kernel vanishes outside a h)."""
    diff = grid[None, :] - np.asarray(z)[:, None]
    if shape == "gaussian":
        k = np.exp(-0.5 * (diff / h) ** 2) / (h * math.sqrt(2.0 * math.pi))
        if T is not None:
            k = np.where(np.abs(diff) <= T * h, k, 0.0)
        return k
    if shape == "epanechnikov":
        ah = EPAN_SCALE * h
        return 0.75 / ah * np.maximum(0.0, 1.0 - (diff / ah) ** 2)
    raise ValueError(f"unknown kernel shape {shape!r}")


def support(h, shape, T):
    """Half-width of the kernel's support (None: the whole grid)."""
    if shape == "epanechnikov":
        return EPAN_SCALE * h
    return None if T is None else T * h


def grid_span(grid, z, reach):
    """The grid points within reach of some z (all points for reach None);
    only a saving: the kernel values outside are 0."""
    if reach is None:
        return slice(None)
    lo = np.searchsorted(grid, np.min(z) - reach, side="left")
    hi = np.searchsorted(grid, np.max(z) + reach, side="right")
    return slice(lo, hi)


def bin_samples(z, w, n_bins):
    """The binned data set of Sect. 2.3 (reading): n_bins equal-width bins
    spanning [min z, max z] of the samples (the largest in the last bin); each
    bin becomes one point at its centre carrying the summed weight of its
    samples (empty bins carry 0).  All samples at one redshift: one bin at
    that redshift holds the whole weight."""
    z = np.asarray(z, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    lo, hi = float(np.min(z)), float(np.max(z))
    width = (hi - lo) / n_bins
    if width > 0.0:
        idx = np.minimum(np.floor((z - lo) / width).astype(np.int64), n_bins - 1)
        centres = lo + (np.arange(n_bins) + 0.5) * width
    else:
        idx = np.zeros(z.size, dtype=np.int64)
        centres = np.full(n_bins, lo)
    weights = np.zeros(n_bins)
    for b, wj in zip(idx, w):          # in sample order: a plain, ordered sum
        weights[b] += wj
    return centres, weights


def event_integral(pixels_z, pixels_w, pixels_c, pixels_row, grid, tau, gz, T=None,
                   shape="gaussian", n_bins=0):
    """(I_i, h_i) of one event given its per-pixel (z, w, c, n_r).  shape:
    the 1-D kernel (kernel_values); n_bins > 0 replaces each pixel's samples
    by its binned data set (bin_samples) in the kernel sums, the bandwidth
    and the 1/N_r in c staying those of the samples."""
    dz = grid[1] - grid[0]
    z_all = np.concatenate(pixels_z)
    w_all = np.concatenate(pixels_w)
    h = bandwidth(z_all, w_all, dz)
    if h is None:
        return 0.0, float("nan")
    reach = support(h, shape, T)
    total = 0.0
    for zr, wr, c, nr in zip(pixels_z, pixels_w, pixels_c, pixels_row):
        if n_bins:
            zr, wr = bin_samples(zr, wr, n_bins)
        f = tau * nr * gz
        g = grid_span(grid, zr, reach)
        a = kernel_values(grid[g], zr, h, shape, T) @ f[g]
        total += c * float(wr @ a)
    return total, h


def event_integral_single1d(z_all, w_all, pixels_s, pixels_row, grid, tau, gz, T=None,
                            shape="gaussian", n_bins=0):
    """(I_i, h_i) of one event with the single-1D kernel (eq. gw-kernel-single1d):
    the event's one weighted redshift KDE over all its samples z_all (weights
    w_all; binned when n_bins > 0) on the grid, times each pixel's sky factor
    S_ir and catalogue row, summed over pixels."""
    dz = grid[1] - grid[0]
    h = bandwidth(z_all, w_all, dz)
    if h is None:
        return 0.0, float("nan")
    zk, wk = bin_samples(z_all, w_all, n_bins) if n_bins else (z_all, w_all)
    g = grid_span(grid, zk, support(h, shape, T))
    kde = np.zeros(grid.size)
    kde[g] = (wk @ kernel_values(grid[g], zk, h, shape, T)) / z_all.size
    total = 0.0
    for s_ir, nr in zip(pixels_s, pixels_row):
        total += s_ir * float(np.sum(tau * nr * gz * kde))
    return total, h


def kde3d_bandwidth(z, u, v, w):
    """The 3D kernel's bandwidth matrix: the weighted covariance of (z, u, v)
    (unbiased, W1 - W2/W1 in the denominator) times n_eff^(-2/7), Scott's
    factor in 3 dimensions with the Kish effective size (reading; the same
    rule as scipy.stats.gaussian_kde).  None when the weights vanish or the
    matrix is not positive definite."""
    W1 = float(np.sum(w))
    if not W1 > 0:
        return None
    W2 = float(np.sum(w * w))
    if W1 * W1 - W2 <= 1e-12 * W1 * W1:
        return None
    x = np.stack([z, u, v], axis=1)
    d = x - (w @ x) / W1
    cov = (d.T * w) @ d / (W1 - W2 / W1)
    H = cov * (W1 * W1 / W2) ** (-2.0 / 7.0)
    if not (H[0, 0] > 0 and np.linalg.det(H[1:, 1:]) > 0 and np.linalg.det(H) > 0):
        return None
    return H


def event_integral_3d(z, w, su, sv, pixels_uv, pixels_area, pixels_row, grid, tau, gz, T=None):
    """(I_i, s_i) of one event with the 3D kernel (the Gaussian KDE of the
    samples in (z, sky) evaluated at each pixel centre, Sect. 2.2-2.3):
    I_i = sum_k area_k sum_g tau_g n_k(z_g) g(z_g) (1/N) sum_j w_j N3(r_jgk; H),
    r = (z_g - z_j, u_k - u_j, v_k - v_j).  The kernel value is the full 3-D
    Gaussian; with finite T (reading) a pair (j, k) counts where the sky part
    of the quadratic form, dO^T H_OO^-1 dO, is <= T^2, and a grid point where
    |z_g - z_j - B dO| <= T s, with B = H_zO H_OO^-1 and s^2 = H_zz - B H_Oz
    the conditional mean shift and variance of z given the sky offset.  s_i
    is returned in the bandwidth's place."""
    H = kde3d_bandwidth(z, su, sv, w)
    if H is None:
        return 0.0, float("nan")
    Hinv = np.linalg.inv(H)
    norm = 1.0 / ((2.0 * math.pi) ** 1.5 * math.sqrt(np.linalg.det(H)))
    inv_oo = np.linalg.inv(H[1:, 1:])
    B = H[0, 1:] @ inv_oo
    s_cond = math.sqrt(H[0, 0] - B @ H[1:, 0])
    total = 0.0
    for (uk, vk), area, nr in zip(pixels_uv, pixels_area, pixels_row):
        do = np.stack([uk - su, vk - sv], axis=1)
        zc = z + do @ B
        keep = np.ones(z.size, dtype=bool)
        if T is not None:
            keep = np.einsum("ij,jk,ik->i", do, inv_oo, do) <= T * T
            if not keep.any():
                continue
            lo = np.searchsorted(grid, zc[keep].min() - T * s_cond, side="left")
            hi = np.searchsorted(grid, zc[keep].max() + T * s_cond, side="right")
            g = slice(lo, hi)
        else:
            g = slice(None)
        r0 = grid[g][None, :] - z[keep][:, None]
        r1 = do[keep, 0][:, None]
        r2 = do[keep, 1][:, None]
        q = (Hinv[0, 0] * r0 * r0 + Hinv[1, 1] * r1 * r1 + Hinv[2, 2] * r2 * r2
             + 2.0 * (Hinv[0, 1] * r0 * r1 + Hinv[0, 2] * r0 * r2 + Hinv[1, 2] * r1 * r2))
        k = norm * np.exp(-0.5 * q)
        if T is not None:
            k = np.where(np.abs(grid[g][None, :] - zc[keep][:, None]) <= T * s_cond, k, 0.0)
        kde = (w[keep] @ k) / z.size
        total += area * float(np.sum(tau[g] * nr[g] * gz[g] * kde))
    return total, s_cond


def selection(inj: InjectionSet, cat: Catalog, lam):
    """(xi, N_eff) by the injection estimator of Sect. 2.2."""
    z, w = redshift_and_weight(inj.dl, inj.m1d, inj.m2d, lam)
    ntot = np.interp(z, cat.grid, galaxy_density(cat, lam)[1], left=0.0, right=0.0)
    jac = (1.0 + z) ** 3 * cosmo.ddl_gw_dz(z, lam[0], lam[1], lam[2], lam[3])
    s = w * ntot * psi(z, lam[11], lam[12], lam[13]) / (jac * np.exp(inj.ln_pdraw))
    s1 = float(np.sum(s))
    s2 = float(np.sum(s * s))
    xi = s1 / inj.n_total
    den = s2 - s1 * s1 / inj.n_total
    neff = (s1 * s1 / den if den > 0 else np.inf) if s1 > 0 else 0.0
    return xi, neff, z


# -------------------------------------------------------------------------
# ln L for one lambda
# -------------------------------------------------------------------------
_WORK: dict = {}


def _event_worker(i):
    d = _WORK
    ev = d["events"][i]
    rs = [d["rows"][px.pix] for px in ev.pixels]
    opt = dict(shape=d["shape"], n_bins=d["n_bins"])
    if d["kernel"] == "3d":
        sl = d["slices"][i][0]
        su, sv = ev.sky_uv
        return event_integral_3d(d["z"][sl], d["w"][sl], su, sv, [px.uv for px in ev.pixels],
                                 [px.area for px in ev.pixels], rs, d["cat"].grid, d["tau"],
                                 d["gz"], d["T"])
    if d["kernel"] == "single1d":
        sl = d["slices"][i][0]
        return event_integral_single1d(d["z"][sl], d["w"][sl], [px.sky() for px in ev.pixels], rs,
                                       d["cat"].grid, d["tau"], d["gz"], d["T"], **opt)
    zs, ws, cs = [], [], []
    for px in ev.pixels:
        sl = d["slices"][i][len(zs)]
        zs.append(d["z"][sl]); ws.append(d["w"][sl]); cs.append(px.c)
    return event_integral(zs, ws, cs, rs, d["cat"].grid, d["tau"], d["gz"], d["T"], **opt)


def lnl(events, cat: Catalog, inj: InjectionSet, lam, T=None, workers: int = 1,
        event_subset=None, kernel: str = "many1d", shape: str = "gaussian", n_bins: int = 0,
        neff_gate: float = 0.0):
    """ln L and its parts at one lambda.

    kernel: "many1d" (eq. gw-kernel-many1d), "single1d" (eq.
    gw-kernel-single1d) or "3d" (event_integral_3d; h is then the
    conditional width s_i); shape: the 1-D kernel ("gaussian" or
    "epanechnikov", kernel_values); n_bins: 0, or the bins of each KDE's
    binned data set (bin_samples).  Returns dict(lnl, lnI[E] (NaN for events
    not in event_subset), h[E], ln_xi, neff).  With event_subset, lnl is the
    partial sum over those events minus len(subset) ln xi (used for sampled
    parity checks).  neff_gate > 0: the stability check of Sect. 2.2 (reading:
    a finite ln L becomes -inf unless N_eff > neff_gate x the number of events
    summed).
    """
    if kernel not in ("many1d", "single1d", "3d"):
        raise ValueError(f"unknown kernel {kernel!r}")
    if kernel == "3d" and (shape != "gaussian" or n_bins):
        raise ValueError("the 3D kernel is Gaussian on the samples")
    if shape not in ("gaussian", "epanechnikov"):
        raise ValueError(f"unknown kernel shape {shape!r}")
    if n_bins < 0:
        raise ValueError("n_bins must be >= 0")
    lam = np.asarray(lam, dtype=np.float64)
    E = len(events)
    sub = list(range(E)) if event_subset is None else list(event_subset)
    res = {"lnI": np.full(E, np.nan), "h": np.full(E, np.nan), "ln_xi": np.nan,
           "neff": np.nan, "lnl": -np.inf}
    if not lambda_in_domain(lam):
        return res
    # all samples of the selected events, inverted at once
    dls, m1s, m2s, slices = [], [], [], {}
    off = 0
    for i in sub:
        sl_i = []
        groups = ([events[i].all_samples()] if kernel in ("single1d", "3d") else
                  [(px.dl, px.m1d, px.m2d) for px in events[i].pixels])
        for dl, m1, m2 in groups:
            n = dl.size
            dls.append(dl); m1s.append(m1); m2s.append(m2)
            sl_i.append(slice(off, off + n))
            off += n
        slices[i] = sl_i
    try:
        z, w = redshift_and_weight(np.concatenate(dls), np.concatenate(m1s),
                                   np.concatenate(m2s), lam)
        xi, neff, zi = selection(inj, cat, lam)
    except cosmo.NonMonotone:
        return res
    if np.any(np.isnan(z)) or np.any(np.isnan(zi)):
        res["lnl"] = np.nan
        return res
    _WORK.update(events=events, slices=slices, z=z, w=w, cat=cat, tau=trapezoid(cat.grid),
                 gz=grid_factor(cat.grid, lam), T=T, kernel=kernel, shape=shape, n_bins=n_bins,
                 rows=galaxy_density(cat, lam)[0])
    if workers > 1 and len(sub) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            out = pool.map(_event_worker, sub, chunksize=max(1, len(sub) // (4 * workers)))
    else:
        out = [_event_worker(i) for i in sub]
    _WORK.clear()
    for i, (I, h) in zip(sub, out):
        res["lnI"][i] = math.log(I) if I > 0 else -np.inf
        res["h"][i] = h
    res["ln_xi"] = math.log(xi) if xi > 0 else -np.inf
    res["neff"] = neff
    lnI = res["lnI"][sub]
    if np.any(np.isneginf(lnI)) or xi <= 0:
        res["lnl"] = -np.inf
    else:
        res["lnl"] = float(np.sum(lnI) - len(sub) * math.log(xi))
        if neff_gate > 0 and not neff > neff_gate * len(sub):
            res["lnl"] = -np.inf
    return res
