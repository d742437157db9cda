"""Distances and their inversion (TEST INFRASTRUCTURE; see package header).

eq. dL-em : d_L^em(z) = (1+z) int_0^z c dz'/H(z'), flat geometry; the
            cosmology is flat LCDM (Table 1), so H = H0 E(z) with
            E(z) = sqrt(Om (1+z)^3 + 1 - Om) (reading: no radiation term).
eq. dL-mg : d_L^gw = d_L^em * Xi(z),  Xi = Xi0 + (1 - Xi0) (1+z)^-n.
eq. jacobian : the |d d_L / dz| of the detector-frame Jacobian is the
            derivative of d_L^gw (reading: the distance the GW measures).
Sect. 2.1 : the redshift of a sample is the z at which d_L^gw equals its
            measured distance.

chi(z) = int_0^z dz'/E(z') is computed by composite Gauss-Legendre
quadrature on fixed panels of width 0.05 (24 nodes each), which is exact
to rounding for this analytic integrand.

Pins (tests/test_oracle_cosmology.py): Einstein-de Sitter closed form
(Om=1), empty-universe limit (Om->0: chi=z), 30-digit mpmath quadrature,
closed-form derivative vs Richardson finite differences, Xi0=1 reducing
bit-exactly to GR, the paper's merger-count integral (Sect. 3.3, ~1.4e4/yr).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import roots_legendre

C_KM_S = 299792.458          # speed of light [km/s]; distances in Mpc, H0 in km/s/Mpc
Z_MAX = 25.0                 # inversion searches z in [0, Z_MAX]
PANEL = 0.05
_GL_X, _GL_W = roots_legendre(24)
_PANEL_CACHE: dict = {}


def efunc(z, om):
    return np.sqrt(om * (1.0 + z) ** 3 + 1.0 - om)


def _panel_integral(a, b, om):
    t = 0.5 * (b - a)[..., None] * _GL_X + 0.5 * (a + b)[..., None]
    return 0.5 * (b - a) * np.sum(_GL_W / efunc(t, om), axis=-1)


def _panel_prefix(om: float):
    key = float(om)
    if key not in _PANEL_CACHE:
        n = int(math.ceil(Z_MAX / PANEL)) + 2
        edges = PANEL * np.arange(n + 1)
        parts = _panel_integral(edges[:-1], edges[1:], om)
        _PANEL_CACHE[key] = np.concatenate([[0.0], np.cumsum(parts)])
        if len(_PANEL_CACHE) > 512:
            _PANEL_CACHE.pop(next(iter(_PANEL_CACHE)))
    return _PANEL_CACHE[key]


def chi(z, om):
    """int_0^z dz'/E(z') (dimensionless comoving distance)."""
    z = np.asarray(z, dtype=np.float64)
    pre = _panel_prefix(om)
    k = np.floor(z / PANEL).astype(np.int64)
    k = np.clip(k, 0, len(pre) - 2)
    a = PANEL * k
    return pre[k] + _panel_integral(a, z, om)


def xi(z, xi0, n):
    """Xi(z) of eq. dL-mg."""
    return xi0 + (1.0 - xi0) * (1.0 + np.asarray(z, dtype=np.float64)) ** (-n)


def dl_em(z, h0, om):
    z = np.asarray(z, dtype=np.float64)
    return (C_KM_S / h0) * (1.0 + z) * chi(z, om)


def dl_gw(z, h0, om, xi0, n):
    z = np.asarray(z, dtype=np.float64)
    return dl_em(z, h0, om) * xi(z, xi0, n)


def ddl_gw_dz(z, h0, om, xi0, n):
    """d d_L^gw / dz = (c/H0) [ (chi + (1+z)/E) Xi + (1+z) chi dXi/dz ]."""
    z = np.asarray(z, dtype=np.float64)
    c = chi(z, om)
    x = xi(z, xi0, n)
    dx = -n * (1.0 - xi0) * (1.0 + z) ** (-n - 1.0)
    return (C_KM_S / h0) * ((c + (1.0 + z) / efunc(z, om)) * x + (1.0 + z) * c * dx)


def comoving_volume_element(z, h0, om):
    """dV_c/dz over the full sky [Mpc^3]: 4 pi (c/H0)^3 chi^2 / E."""
    z = np.asarray(z, dtype=np.float64)
    dh = C_KM_S / h0
    return 4.0 * math.pi * dh ** 3 * chi(z, om) ** 2 / efunc(z, om)


class NonMonotone(Exception):
    pass


def invert_dl(d, h0, om, xi0, n, table_points: int = 20001, newton_steps: int = 6):
    """z such that d_L^gw(z) = d, searched on [0, Z_MAX].

    Bracket by a table of d_L^gw on a uniform z grid (np.searchsorted), then
    safeguarded Newton inside the bracket.  Raises NonMonotone if d_L^gw is not
    strictly increasing on [0, Z_MAX]; returns NaN where d exceeds d_L^gw(Z_MAX).
    """
    d = np.asarray(d, dtype=np.float64)
    zt = np.linspace(0.0, Z_MAX, table_points)
    dt = dl_gw(zt, h0, om, xi0, n)
    if np.any(ddl_gw_dz(zt, h0, om, xi0, n) <= 0.0) or np.any(np.diff(dt) <= 0.0):
        raise NonMonotone()
    k = np.searchsorted(dt, d, side="right") - 1
    out_of_range = (d > dt[-1]) | (d < 0)
    k = np.clip(k, 0, table_points - 2)
    lo, hi = zt[k], zt[k + 1]
    flo, fhi = dt[k] - d, dt[k + 1] - d
    z = lo + (hi - lo) * (-flo) / np.where(fhi - flo > 0, fhi - flo, 1.0)
    for _ in range(newton_steps):
        f = dl_gw(z, h0, om, xi0, n) - d
        fp = ddl_gw_dz(z, h0, om, xi0, n)
        # keep the bracket
        lo = np.where(f < 0, np.maximum(lo, z), lo)
        hi = np.where(f > 0, np.minimum(hi, z), hi)
        zn = z - f / fp
        bad = ~((zn >= lo) & (zn <= hi))
        z = np.where(bad, 0.5 * (lo + hi), zn)
    z = np.where(out_of_range, np.nan, z)
    return z
