"""Population model (TEST INFRASTRUCTURE; see package header).

Sect. 3.1 and Table 1: primary mass a power law of slope -alpha on
[m_low, m_high] plus a Gaussian peak (mu_g, sigma_g) of weight lambda_g;
secondary a power law of slope beta on [m_low, m1]; merger-rate evolution
psi(z) = (1+z)^gamma / (1 + ((1+z)/(1+z_p))^(gamma+kappa)).

Readings (the paper points to an external appendix for the full model):
* m_low = mmin, m_high = mmax; with a fifteenth entry delta_m > 0 in lambda
  the lower edge is smoothed (Table 1's delta_m): the mixture p(m1) and the
  power law of p(m2|m1) are multiplied by
  S(m) = 0 (m <= mmin), 1 (m >= mmin + delta_m),
  1 / (exp(delta_m/m' + delta_m/(m' - delta_m)) + 1) between (m' = m - mmin),
  and each is normalised again on its support (numerically); without it
  (or delta_m = 0) there is no smoothing;
* the Gaussian peak is truncated to [mmin, mmax] and renormalised there;
* p(m2|m1) is normalised on [mmin, m1] for each m1;
* every density is exactly 0 outside its support (edges inclusive);
* psi is used raw (any constant factor cancels between the events and xi).

Pins (tests/test_oracle_population.py): both densities integrate to 1
(scipy quad), the alpha=1 and beta=-1 limits are continuous, the peak
matches scipy.stats.truncnorm, psi(0)=1/(1+(1+z_p)^-(gamma+kappa)).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ndtr


def _pl_norm(slope_plus_one, lo, hi):
    """int_lo^hi m^(slope) dm with slope_plus_one = slope + 1 (log form at 0)."""
    if slope_plus_one == 0.0:
        return math.log(hi / lo)
    return (hi ** slope_plus_one - lo ** slope_plus_one) / slope_plus_one


def p_m1(m1, alpha, mmin, mmax, mu_g, sigma_g, lambda_g):
    """p(m1) = (1-lambda_g) PL(m1; -alpha) + lambda_g TG(m1; mu_g, sigma_g)."""
    m1 = np.asarray(m1, dtype=np.float64)
    inside = (m1 >= mmin) & (m1 <= mmax)
    mm = np.where(inside, m1, mmin)
    pl = mm ** (-alpha) / _pl_norm(1.0 - alpha, mmin, mmax)
    a, b = (mmin - mu_g) / sigma_g, (mmax - mu_g) / sigma_g
    # the peak's mass inside [mmin, mmax], from the tail that does not cancel
    z = ndtr(-a) - ndtr(-b) if a > 0 else ndtr(b) - ndtr(a)
    tg = np.exp(-0.5 * ((mm - mu_g) / sigma_g) ** 2) / (sigma_g * math.sqrt(2.0 * math.pi)) / z
    return np.where(inside, (1.0 - lambda_g) * pl + lambda_g * tg, 0.0)


def p_m2_given_m1(m2, m1, beta, mmin):
    """p(m2|m1) = m2^beta / int_mmin^m1 m^beta dm on [mmin, m1]."""
    m2 = np.asarray(m2, dtype=np.float64)
    m1 = np.asarray(m1, dtype=np.float64)
    inside = (m2 >= mmin) & (m2 <= m1) & (m1 > mmin)
    a = 1.0 + beta
    m1s = np.where(inside, m1, 2.0 * mmin)
    m2s = np.where(inside, m2, mmin)
    if a == 0.0:
        norm = np.log(m1s / mmin)
    else:
        norm = (m1s ** a - mmin ** a) / a
    return np.where(inside, m2s ** beta / norm, 0.0)


def smoothing(m, mmin, dm):
    """S(m; mmin, delta_m) of the smoothed lower mass edge."""
    m = np.asarray(m, dtype=np.float64)
    mp = m - mmin
    out = np.where(mp >= dm, 1.0, 0.0)
    mid = (mp > 0.0) & (mp < dm)
    if np.any(mid):
        x = mp[mid] if mp.ndim else mp
        with np.errstate(over="ignore"):
            sm = 1.0 / (np.exp(dm / x + dm / (x - dm)) + 1.0)
        if mp.ndim:
            out = out.copy()
            out[mid] = sm
        else:
            out = sm
    return out


def smoothed_constants(lam):
    """(N1, Q): N1 = int_mmin^mmax p(m1) S dm, the smoothed primary's
    normalisation, and Q = int_mmin^min(mmax, mmin + delta_m) m^beta S dm, the
    smoothed part of p(m2|m1)'s normalisation (scipy quad, epsrel 1e-13)."""
    from scipy.integrate import quad
    alpha, beta, mmin, mmax, mu_g, sigma_g, lambda_g, dm = (lam[4], lam[5], lam[6], lam[7],
                                                             lam[8], lam[9], lam[10], lam[14])
    top = min(mmax, mmin + dm)
    deficit = quad(lambda m: float(p_m1(m, alpha, mmin, mmax, mu_g, sigma_g, lambda_g))
                   * (1.0 - float(smoothing(m, mmin, dm))), mmin, top,
                   epsabs=0.0, epsrel=1e-13, limit=200)[0]
    q = quad(lambda m: m ** beta * float(smoothing(m, mmin, dm)), mmin, top,
             epsabs=0.0, epsrel=1e-13, limit=200)[0]
    return 1.0 - deficit, q


def p2_norm_smoothed(m1, beta, mmin, dm, q):
    """int_mmin^m1 m^beta S(m) dm: q plus the unsmoothed power law beyond
    mmin + delta_m, or a quadrature for m1 inside the smoothed range."""
    from scipy.integrate import quad
    m1 = np.asarray(m1, dtype=np.float64)
    edge = mmin + dm
    out = np.empty(m1.shape)
    for i, x in np.ndenumerate(m1):
        if x >= edge:
            out[i] = q + _pl_norm(1.0 + beta, edge, x)
        else:
            out[i] = quad(lambda m: m ** beta * float(smoothing(m, mmin, dm)), mmin, max(x, mmin),
                          epsabs=0.0, epsrel=1e-13, limit=200)[0]
    return out


def mass_weight(m1, m2, lam):
    """w = p(m1) p(m2|m1) with the PE prior pi = 1 (uniform priors, Sect. 3.2);
    smoothed lower edge when lambda carries delta_m > 0 (see the header)."""
    alpha, beta, mmin, mmax, mu_g, sigma_g, lambda_g = (lam[4], lam[5], lam[6], lam[7],
                                                         lam[8], lam[9], lam[10])
    dm = float(lam[14]) if len(lam) > 14 else 0.0
    if dm == 0.0:
        return (p_m1(m1, alpha, mmin, mmax, mu_g, sigma_g, lambda_g)
                * p_m2_given_m1(m2, m1, beta, mmin))
    m1 = np.asarray(m1, dtype=np.float64)
    m2 = np.asarray(m2, dtype=np.float64)
    n1, q = smoothed_constants(lam)
    p1 = p_m1(m1, alpha, mmin, mmax, mu_g, sigma_g, lambda_g) * smoothing(m1, mmin, dm) / n1
    inside = (m2 >= mmin) & (m2 <= m1) & (m1 > mmin) & (p1 > 0)
    w = np.zeros(np.broadcast(m1, m2).shape)
    if np.any(inside):
        m1i, m2i = np.broadcast_to(m1, w.shape)[inside], np.broadcast_to(m2, w.shape)[inside]
        w[inside] = (np.broadcast_to(p1, w.shape)[inside] * m2i ** beta * smoothing(m2i, mmin, dm)
                     / p2_norm_smoothed(m1i, beta, mmin, dm, q))
    return w


def psi(z, gamma, kappa, z_p):
    """Madau-Dickinson rate shape (Sect. 3.1)."""
    zp1 = 1.0 + np.asarray(z, dtype=np.float64)
    return zp1 ** gamma / (1.0 + (zp1 / (1.0 + z_p)) ** (gamma + kappa))
