"""Seeded synthetic inputs with the shapes of the paper's workloads.

This module is the *input generator* shared by the library's callers (bench,
server, tests) and by the test-side oracle.  It produces raw data only:

* a galaxy catalogue uniform in comoving volume, with spectroscopic or
  photometric redshift errors (Sect. 3.1 and the redshift-error models of
  Sect. 4), binned on a HEALPix RING sky pixelisation;
* GW events hosted by catalogue galaxies, with a power-law-plus-peak mass
  population and a Madau--Dickinson rate (Sect. 3.1), kept when a simple S/N
  proxy exceeds 20 (Sect. 3.3), each with Gaussian posterior samples of
  (d_L, m1_det, m2_det, sky position);
* injections drawn from a broad proposal with their stored draw density and
  a detected flag from the same S/N proxy (Sect. 2.2, injection estimator);
* batches of hyperparameter points lambda.

Nothing here evaluates the likelihood.  The distance--redshift relation used
to *place* synthetic events is a coarse cumulative trapezoid of its own
(good to ~1e-9), used for nothing else; the likelihood sides compute their
own distances from the paper's equations.

Sky pixelisation: HEALPix RING scheme of Gorski et al. (2005, ApJ 622, 759),
restated here from the geometry described in that paper (equal-area rings,
diamond-shaped equatorial pixels whose edges are lines of constant
phi*2N/pi +- 3/4 N cos(theta)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_KM_S = 299792.458

#: lambda layout, row-major [B][14] (Table 1 grouping: cosmology, MG, mass, rate)
LAMBDA_NAMES = ("H0", "Om", "Xi0", "n", "alpha", "beta", "mmin", "mmax",
                "mu_g", "sigma_g", "lambda_g", "gamma", "kappa", "z_p")
N_LAMBDA = len(LAMBDA_NAMES)
#: the 12 parameters the gradient is taken with respect to (mmin, mmax are hard edges)
GRAD_NAMES = ("H0", "Om", "Xi0", "n", "alpha", "beta", "mu_g", "sigma_g",
              "lambda_g", "gamma", "kappa", "z_p")
GRAD_COLUMNS = tuple(LAMBDA_NAMES.index(n) for n in GRAD_NAMES)

#: fiducial point of the synthetic populations
LAMBDA_TRUTH = np.array([70.0, 0.3, 1.0, 1.91, 3.4, 1.1, 5.0, 87.0,
                         34.0, 3.6, 0.04, 2.7, 3.0, 2.0])

SEED_ROOT = 250402034


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    n_events: int
    n_samples: int
    n_galaxies: int
    sigma_z0: float          # galaxy redshift error sigma = sigma_z0 * (1 + z)
    nside: int
    n_z: int
    z_lo: float
    z_hi: float
    n_inj: int
    batch: int
    seed_index: int
    xi0_truth: float = 1.0
    sky_sigma_deg: float = 2.0
    dl_frac: float = 0.1
    m_frac: float = 0.05
    cred: float = 0.9
    lam_kind: str = "prior"   # "truth" | "prior" | "jitter"

    def scaled(self, **kw) -> "Workload":
        d = dict(self.__dict__)
        d.update(kw)
        return Workload(**d)


WORKLOADS = {
    # 10 events x 1024 samples, 5e4 spec-z galaxies, nside 32, one lambda
    "fp64_10ev": Workload("fp64_10ev", 10, 1024, 50_000, 0.001, 32, 1000, 0.0, 1.6,
                          100_000, 1, 0, lam_kind="truth"),
    # 300 events x 5000 samples, 1e6 spec-z galaxies, nside 64, 256 lambda
    "precision_300ev": Workload("precision_300ev", 300, 5000, 1_000_000, 0.001, 64, 1000,
                                0.0, 1.6, 1_000_000, 256, 1),
    # 1000 events x 4096 samples, 1e7 photo-z galaxies, 2000-point grid, 128 lambda
    "photo_1000ev": Workload("photo_1000ev", 1000, 4096, 10_000_000, 0.05, 64, 2000,
                             0.0, 2.4, 5_000_000, 128, 2),
    # gradient workload: the 300-event data, 64 lambda with jittered population
    "grad_300ev": Workload("grad_300ev", 300, 5000, 1_000_000, 0.001, 64, 1000, 0.0, 1.6,
                           1_000_000, 64, 1, lam_kind="jitter"),
}


# --------------------------------------------------------------------------
# HEALPix RING pixelisation (Gorski et al. 2005)
# --------------------------------------------------------------------------
def nside_npix(nside: int) -> int:
    return 12 * nside * nside


def pixel_area(nside: int) -> float:
    return 4.0 * math.pi / nside_npix(nside)


def ang2pix_ring(nside: int, theta, phi) -> np.ndarray:
    """Pixel index (RING) of colatitude theta, longitude phi (radians)."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.mod(np.asarray(phi, dtype=np.float64), 2.0 * math.pi)
    z = np.cos(theta)
    za = np.abs(z)
    t = phi * (2.0 / math.pi)                     # longitude in base-pixel units, [0,4)
    t = np.where(t >= 4.0, 0.0, t)
    out = np.empty(z.shape, dtype=np.int64)
    n = np.int64(nside)

    eq = za <= 2.0 / 3.0
    if np.any(eq):
        te, ze = t[eq], z[eq]
        # diamond edges: floor of the two oblique coordinates
        a = n * (0.5 + te)
        b = 0.75 * n * ze
        up = np.floor(a - b).astype(np.int64)
        dn = np.floor(a + b).astype(np.int64)
        ring = n + 1 + up - dn                     # ring counted from z=2/3, 1..2n+1
        k = (up + dn - n + 1 - (ring & 1)) // 2
        k = np.mod(k, 4 * n)
        out[eq] = 2 * n * (n - 1) + 4 * n * (ring - 1) + k

    cap = ~eq
    if np.any(cap):
        tc, zc = t[cap], z[cap]
        frac = tc - np.floor(tc)
        s = n * np.sqrt(3.0 * (1.0 - np.abs(zc)))
        i1 = np.floor(frac * s).astype(np.int64)
        i2 = np.floor((1.0 - frac) * s).astype(np.int64)
        ring = i1 + i2 + 1                         # ring counted from the nearer pole
        k = np.mod(np.floor(tc * ring).astype(np.int64), 4 * ring)
        north = 2 * ring * (ring - 1) + k
        south = nside_npix(nside) - 2 * ring * (ring + 1) + k
        out[cap] = np.where(zc > 0, north, south)
    return out


def pix2ang_ring(nside: int, pix):
    """(theta, phi) of the centres of RING pixels."""
    p = np.asarray(pix, dtype=np.int64)
    n = np.int64(nside)
    npix = nside_npix(nside)
    ncap = 2 * n * (n - 1)
    theta = np.empty(p.shape)
    phi = np.empty(p.shape)

    north = p < ncap
    if np.any(north):
        q = p[north]
        ring = np.floor((1.0 + np.sqrt(1.0 + 2.0 * q)) / 2.0).astype(np.int64)
        k = q - 2 * ring * (ring - 1)
        theta[north] = np.arccos(1.0 - ring.astype(float) ** 2 / (3.0 * n * n))
        phi[north] = (k + 0.5) * math.pi / (2.0 * ring)

    south = p >= npix - ncap
    if np.any(south):
        q = npix - p[south]
        ring = np.floor((1.0 + np.sqrt(2.0 * q - 1.0)) / 2.0).astype(np.int64)
        k = p[south] - (npix - 2 * ring * (ring + 1))
        theta[south] = np.arccos(-(1.0 - ring.astype(float) ** 2 / (3.0 * n * n)))
        phi[south] = (k + 0.5) * math.pi / (2.0 * ring)

    eq = ~(north | south)
    if np.any(eq):
        q = p[eq] - ncap
        ring = q // (4 * n) + n                    # ring counted from the north pole
        k = q % (4 * n)
        theta[eq] = np.arccos(4.0 / 3.0 - 2.0 * ring / (3.0 * n))
        shift = np.where(((ring + n) & 1) == 1, 0.0, 0.5)
        phi[eq] = (k + shift) * math.pi / (2.0 * n)
    return theta, phi


def unit_vectors(theta, phi) -> np.ndarray:
    st = np.sin(theta)
    return np.stack([st * np.cos(phi), st * np.sin(phi), np.cos(theta)], axis=-1)


def vectors_to_angles(v):
    v = v / np.linalg.norm(v, axis=-1, keepdims=True)
    theta = np.arccos(np.clip(v[..., 2], -1.0, 1.0))
    phi = np.mod(np.arctan2(v[..., 1], v[..., 0]), 2.0 * math.pi)
    return theta, phi


def _tangent_basis(theta0, phi0):
    er = unit_vectors(theta0, phi0)
    ee = np.array([-math.sin(phi0), math.cos(phi0), 0.0])          # east
    en = np.cross(er, ee)                                            # north
    return er, ee, en


# --------------------------------------------------------------------------
# coarse cosmology for placing synthetic events (not the likelihood's)
# --------------------------------------------------------------------------
class _PlacementCosmology:
    def __init__(self, H0: float, Om: float, z_max: float = 3.0, n: int = 300_001):
        z = np.linspace(0.0, z_max, n)
        inv_e = 1.0 / np.sqrt(Om * (1 + z) ** 3 + 1 - Om)
        chi = np.concatenate([[0.0], np.cumsum(0.5 * (inv_e[1:] + inv_e[:-1]) * np.diff(z))])
        self.z, self.chi, self.inv_e, self.dh = z, chi, inv_e, C_KM_S / H0

    def dl_gw(self, z, xi0, n):
        chi = np.interp(z, self.z, self.chi)
        return self.dh * (1 + z) * chi * (xi0 + (1 - xi0) * (1 + z) ** (-n))

    def volume_weight(self, z):
        """shape of dV_c/dz (up to a constant)."""
        return np.interp(z, self.z, self.chi) ** 2 * np.interp(z, self.z, self.inv_e)


def _rate_shape(z, gamma, kappa, zp):
    return (1 + z) ** gamma / (1 + ((1 + z) / (1 + zp)) ** (gamma + kappa))


def _sample_plp_m1(rng, size, lam):
    alpha, mmin, mmax = lam[4], lam[6], lam[7]
    mu, sg, lg = lam[8], lam[9], lam[10]
    m = np.linspace(mmin, mmax, 200_001)
    pl = m ** (-alpha)
    pl /= np.trapezoid(pl, m)
    g = np.exp(-0.5 * ((m - mu) / sg) ** 2)
    g /= np.trapezoid(g, m)
    pdf = (1 - lg) * pl + lg * g
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(m))])
    cdf /= cdf[-1]
    return np.interp(rng.random(size), cdf, m)


def _sample_pl_m2(rng, m1, lam):
    beta, mmin = lam[5], lam[6]
    u = rng.random(m1.shape)
    a = 1.0 + beta
    lo = mmin ** a
    return (lo + u * (m1 ** a - lo)) ** (1.0 / a)


def _snr_shape(m1d, m2d, dl):
    mc = (m1d * m2d) ** 0.6 / (m1d + m2d) ** 0.2
    return (mc / 30.0) ** (5.0 / 6.0) * (1000.0 / dl)


_RHO0_CACHE: dict = {}


def snr_scale() -> float:
    """rho0 such that ~2.4% of population draws with z<1.3 at the fiducial point
    pass rho>20 (the paper's GR-scenario ratio 340 / 1.4e4, Sect. 3.3)."""
    if "rho0" in _RHO0_CACHE:
        return _RHO0_CACHE["rho0"]
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 999]))
    lam = LAMBDA_TRUTH
    cos = _PlacementCosmology(lam[0], lam[1])
    zz = np.linspace(0, 1.3, 20001)
    pdf = cos.volume_weight(zz) * _rate_shape(zz, lam[11], lam[12], lam[13]) / (1 + zz)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(zz))])
    cdf /= cdf[-1]
    n = 400_000
    z = np.interp(rng.random(n), cdf, zz)
    m1 = _sample_plp_m1(rng, n, lam)
    m2 = _sample_pl_m2(rng, m1, lam)
    dl = cos.dl_gw(z, lam[2], lam[3])
    r = _snr_shape(m1 * (1 + z), m2 * (1 + z), dl) * rng.random(n)
    rho0 = 20.0 / np.quantile(r, 1.0 - 0.024)
    _RHO0_CACHE["rho0"] = float(rho0)
    return float(rho0)


# --------------------------------------------------------------------------
# raw data containers
# --------------------------------------------------------------------------
@dataclass
class Catalog:
    z_obs: np.ndarray        # observed redshift per galaxy
    pix: np.ndarray          # RING pixel per galaxy
    sigma_z0: float          # sigma_z = sigma_z0 * (1 + z_obs)
    nside: int


@dataclass
class Events:
    offsets: np.ndarray      # [E+1] sample offsets
    dl: np.ndarray           # [S_tot] Mpc
    m1d: np.ndarray          # [S_tot] detector-frame primary mass
    m2d: np.ndarray
    theta: np.ndarray        # [S_tot] colatitude
    phi: np.ndarray
    pix: np.ndarray          # [S_tot] RING pixel
    nside: int
    truth: dict = field(default_factory=dict)

    @property
    def n_events(self) -> int:
        return len(self.offsets) - 1


@dataclass
class Injections:
    dl: np.ndarray
    m1d: np.ndarray
    m2d: np.ndarray
    ln_pdraw: np.ndarray
    n_total: int


def _rng(wl_seed: int, child: int):
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, wl_seed, child]))


def make_catalog(wl: Workload):
    """(Catalog, z_true, cos_theta, phi): the catalogue plus the true host values."""
    rng = _rng(wl.seed_index, 1)
    lam = LAMBDA_TRUTH
    cos = _PlacementCosmology(lam[0], lam[1])
    zz = np.linspace(0.0, 1.5, 30001)
    pdf = cos.volume_weight(zz)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(zz))])
    cdf /= cdf[-1]
    n = wl.n_galaxies
    z_true = np.interp(rng.random(n), cdf, zz)
    cos_theta = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    z_obs = z_true + wl.sigma_z0 * (1.0 + z_true) * rng.standard_normal(n)
    pix = ang2pix_ring(wl.nside, np.arccos(cos_theta), phi)
    return Catalog(z_obs=z_obs, pix=pix, sigma_z0=wl.sigma_z0, nside=wl.nside), z_true, cos_theta, phi


def make_events(wl: Workload, catalog_full=None, n_events: int | None = None,
                n_samples: int | None = None, child: int = 2) -> Events:
    """GW events hosted by catalogue galaxies, kept at S/N proxy > 20."""
    if catalog_full is None:
        catalog_full = make_catalog(wl)
    cat, z_true, cos_theta, phi = catalog_full
    n_ev = wl.n_events if n_events is None else n_events
    n_s = wl.n_samples if n_samples is None else n_samples
    rng = _rng(wl.seed_index, child)
    lam = LAMBDA_TRUTH.copy()
    lam[2] = wl.xi0_truth
    cos = _PlacementCosmology(lam[0], lam[1])
    rho0 = snr_scale()

    w = _rate_shape(z_true, lam[11], lam[12], lam[13]) / (1 + z_true)
    w = w / w.sum()
    hosts, m1s, m2s, dls = [], [], [], []
    have = 0
    while have < n_ev:
        k = max(4 * (n_ev - have) * 50, 1000)
        h = rng.choice(len(z_true), size=k, p=w)
        m1 = _sample_plp_m1(rng, k, lam)
        m2 = _sample_pl_m2(rng, m1, lam)
        z = z_true[h]
        dl = cos.dl_gw(z, lam[2], lam[3])
        rho = rho0 * _snr_shape(m1 * (1 + z), m2 * (1 + z), dl) * rng.random(k)
        keep = rho > 20.0
        hosts.append(h[keep]); m1s.append(m1[keep]); m2s.append(m2[keep]); dls.append(dl[keep])
        have += int(keep.sum())
    hosts = np.concatenate(hosts)[:n_ev]
    m1 = np.concatenate(m1s)[:n_ev]
    m2 = np.concatenate(m2s)[:n_ev]
    dl_true = np.concatenate(dls)[:n_ev]
    z_h = z_true[hosts]

    sig_sky = math.radians(wl.sky_sigma_deg)
    off = np.arange(n_ev + 1, dtype=np.int64) * n_s
    dl_all = np.empty(n_ev * n_s); m1_all = np.empty(n_ev * n_s); m2_all = np.empty(n_ev * n_s)
    th_all = np.empty(n_ev * n_s); ph_all = np.empty(n_ev * n_s)
    for e in range(n_ev):
        sl = slice(off[e], off[e + 1])
        # one scattered "observed" centre per event, samples around it
        d_c = dl_true[e] * (1.0 + wl.dl_frac * rng.standard_normal())
        d_c = max(d_c, 0.2 * dl_true[e])
        m1c = m1[e] * (1 + z_h[e]) * (1.0 + wl.m_frac * rng.standard_normal())
        m2c = m2[e] * (1 + z_h[e]) * (1.0 + wl.m_frac * rng.standard_normal())
        d = d_c * (1.0 + wl.dl_frac * rng.standard_normal(n_s))
        bad = d <= 0
        while np.any(bad):
            d[bad] = d_c * (1.0 + wl.dl_frac * rng.standard_normal(int(bad.sum())))
            bad = d <= 0
        a = np.abs(m1c * (1.0 + wl.m_frac * rng.standard_normal(n_s)))
        b = np.abs(m2c * (1.0 + wl.m_frac * rng.standard_normal(n_s)))
        dl_all[sl] = d
        m1_all[sl] = np.maximum(a, b)
        m2_all[sl] = np.minimum(a, b)
        # sky: tangent-plane Gaussian around a scattered centre
        th0, ph0 = math.acos(cos_theta[hosts[e]]), phi[hosts[e]]
        er, ee, en = _tangent_basis(th0, ph0)
        cx, cy = sig_sky * rng.standard_normal(2)
        c_vec = er + cx * ee + cy * en
        thc, phc = vectors_to_angles(c_vec)
        er, ee, en = _tangent_basis(float(thc), float(phc))
        xi = sig_sky * rng.standard_normal(n_s)
        eta = sig_sky * rng.standard_normal(n_s)
        v = er[None, :] + xi[:, None] * ee[None, :] + eta[:, None] * en[None, :]
        th_all[sl], ph_all[sl] = vectors_to_angles(v)
    pix = ang2pix_ring(wl.nside, th_all, ph_all)
    return Events(offsets=off, dl=dl_all, m1d=m1_all, m2d=m2_all, theta=th_all, phi=ph_all,
                  pix=pix, nside=wl.nside,
                  truth={"z": z_h, "dl": dl_true, "m1": m1, "m2": m2, "host": hosts})


INJ_DL = (1.0, 3.0e4)
INJ_M = (3.0, 400.0)


def make_injections(wl: Workload, n_inj: int | None = None, child: int = 3) -> Injections:
    """Broad proposal: d ~ U[1, 3e4] Mpc, m1d ~ logU[3, 400], m2d|m1d ~ U[3, m1d]."""
    n = wl.n_inj if n_inj is None else n_inj
    rng = _rng(wl.seed_index, child)
    rho0 = snr_scale()
    dl = rng.uniform(INJ_DL[0], INJ_DL[1], n)
    lm = rng.uniform(math.log(INJ_M[0]), math.log(INJ_M[1]), n)
    m1 = np.exp(lm)
    m2 = INJ_M[0] + rng.random(n) * (m1 - INJ_M[0])
    ln_p = (-math.log(INJ_DL[1] - INJ_DL[0]) - np.log(m1) - math.log(math.log(INJ_M[1] / INJ_M[0]))
            - np.log(np.maximum(m1 - INJ_M[0], 1e-300)))
    rho = rho0 * _snr_shape(m1, m2, dl) * rng.random(n)
    det = (rho > 20.0) & (m1 > INJ_M[0])
    return Injections(dl=dl[det].copy(), m1d=m1[det].copy(), m2d=m2[det].copy(),
                      ln_pdraw=ln_p[det].copy(), n_total=n)


def make_lambdas(wl: Workload, batch: int | None = None, child: int = 4) -> np.ndarray:
    b = wl.batch if batch is None else batch
    rng = _rng(wl.seed_index, child)
    lam = np.tile(LAMBDA_TRUTH, (b, 1))
    if wl.lam_kind == "truth":
        lam[:, 2] = wl.xi0_truth
        return lam
    lam[:, 0] = rng.uniform(20.0, 140.0, b)
    lam[:, 1] = rng.uniform(0.1, 0.5, b)
    lam[:, 2] = rng.uniform(0.3, 3.0, b)
    lam[:, 3] = rng.uniform(0.0, 10.0, b)
    if wl.lam_kind == "jitter":
        cols = [4, 5, 8, 9, 10, 11, 12, 13]
        lam[:, cols] *= rng.uniform(0.9, 1.1, (b, len(cols)))
    return lam


def z_grid(wl: Workload) -> np.ndarray:
    return np.linspace(wl.z_lo, wl.z_hi, wl.n_z)


def make_completeness(rows_pix, nside, grid, seed=7):
    """A synthetic catalogue completeness (input data for the incompleteness
    term): per HEALPix pixel a falling logistic P(z) = 1 / (1 + e^((z - z_c)/0.08))
    with z_c drawn in [0.5, 1.3] per pixel (the catalogue's magnitude limit
    reached at different depths across the sky).  Returns (P rows for
    rows_pix [n_rows][n_z], M(z) = sum over all 12 nside^2 pixels of
    area (1 - P) [n_z])."""
    npix = 12 * nside * nside
    rng = np.random.default_rng(np.random.SeedSequence([250402034, 99, seed]))
    zc = rng.uniform(0.5, 1.3, npix)
    area = pixel_area(nside)

    def p_of(z_c):
        return 1.0 / (1.0 + np.exp((grid[None, :] - np.asarray(z_c)[:, None]) / 0.08))

    missing = np.zeros(grid.size)
    for a in range(0, npix, 4096):
        missing += area * np.sum(1.0 - p_of(zc[a:a + 4096]), axis=0)
    return p_of(zc[np.asarray(rows_pix)]), missing
