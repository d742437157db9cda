"""Lambda-independent preprocessing: raw catalogue / posterior samples -> the
arrays the C-ABI library takes (``chimera_set_catalog``, ``chimera_add_events``).

The paper computes these once before inference (Sect. 2.3 steps a-c; the
many-1D kernel, eq. gw-kernel-many1d, reuses the pixelisation and the p_cat
grid, and its 2-D sky-KDE normalisation factors are independent of lambda).

* region (Sect. 2.3 step a; Fig. 1 caption): per event, pixels sorted by
  sample count (descending, ties by ascending pixel id) until >= cred of the
  samples are covered; samples outside the region are dropped;
* sky factor (eq. gw-kernel-many1d, second factor): S_ir = pixel area x 2-D
  Gaussian KDE of all the event's sky samples (tangent plane at their mean
  direction, Scott bandwidth) at the pixel centre; c_ir = S_ir / N_ir where
  N_ir is the pixel's sample count (the 1/N of the pixel's 1-D KDE);
* catalogue density (eq. p-cat): each galaxy's Gaussian N(z; z_obs, sigma),
  truncated at 8 sigma, is projected on the grid's linear-interpolation (hat)
  basis, multiplied by
  dV_c/dz at the node (frozen reference cosmology H0=70, Om=0.3) and
  normalised so that sum_k tau_k q_k = 1 (tau = trapezoid weights).
  n_r(z_k) = sum_{gal in r} q / (N_gal * pixel area); n_tot = area * sum_r n_r.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.special import ndtr, roots_legendre

from . import synth

REF_H0 = 70.0
REF_OM = 0.3
SUPPORT_SIGMAS = 8.0


@dataclass
class Prepared:
    """Arrays in the layout of the C-ABI (see include/chimera.h)."""
    n_z: int
    z_lo: float
    z_hi: float
    nz: np.ndarray            # [n_rows, n_z] float64 catalogue density rows
    row_pix: np.ndarray       # [n_rows] HEALPix id of each row
    nz_tot: np.ndarray        # [n_z]
    ev_pix_off: np.ndarray    # [E+1] int64
    pix_samp_off: np.ndarray  # [P+1] int64
    pix_row: np.ndarray       # [P] int64 catalogue row of each (event, pixel)
    pix_id: np.ndarray        # [P] HEALPix id of each (event, pixel)
    c_ir: np.ndarray          # [P] float64
    dl: np.ndarray            # [S] float64, sorted by (event, pixel, dl)
    m1d: np.ndarray
    m2d: np.ndarray
    s_ir: np.ndarray = None   # [P] float64 sky factor S_ir of each (event, pixel)

    @property
    def n_events(self) -> int:
        return len(self.ev_pix_off) - 1


@dataclass
class Single1D:
    """Arrays of chimera_add_events_single1d (eq. gw-kernel-single1d): every
    sample of each event (those outside its region included) and the
    region's pixels with their sky factors."""
    ev_samp_off: np.ndarray   # [E+1] int64
    dl: np.ndarray            # [S] float64, all samples of each event
    m1d: np.ndarray
    m2d: np.ndarray
    ev_pix_off: np.ndarray    # [E+1] int64
    pix_row: np.ndarray       # [P] int64 catalogue row
    s_ir: np.ndarray          # [P] float64

    @property
    def n_events(self) -> int:
        return len(self.ev_samp_off) - 1


def trapezoid_weights(n_z: int, z_lo: float, z_hi: float) -> np.ndarray:
    dz = (z_hi - z_lo) / (n_z - 1)
    tau = np.full(n_z, dz)
    tau[0] = tau[-1] = 0.5 * dz
    return tau


def _comoving_shape(z: np.ndarray) -> np.ndarray:
    """chi(z)^2 / E(z) at the reference cosmology (dV_c/dz up to a constant)."""
    x, w = roots_legendre(24)
    z = np.asarray(z, dtype=np.float64)
    # chi(z) = int_0^z dz'/E: composite Gauss-Legendre on panels of width <= 0.05
    chi = np.zeros_like(z)
    n_pan = np.maximum(1, np.ceil(z / 0.05)).astype(np.int64)
    for i in range(z.size):
        edges = np.linspace(0.0, z.flat[i], n_pan.flat[i] + 1)
        a, b = edges[:-1, None], edges[1:, None]
        t = 0.5 * (b - a) * x[None, :] + 0.5 * (a + b)
        f = 1.0 / np.sqrt(REF_OM * (1 + t) ** 3 + 1 - REF_OM)
        chi.flat[i] = np.sum(0.5 * (b - a) * f * w[None, :])
    e = np.sqrt(REF_OM * (1 + z) ** 3 + 1 - REF_OM)
    return chi ** 2 / e


def _phi_diff(al, be):
    """Phi(be) - Phi(al) for al <= be, from the tail that does not cancel."""
    return np.where(al >= 0.0, ndtr(-al) - ndtr(-be), ndtr(be) - ndtr(al))


def _hat_projection(mu, sig, z_lo, dz, n_z, k0, width):
    """J[g, m] = int N(z; mu_g, sig_g) Lambda_{k0_g+m}(z) dz over |z - mu_g| <= 8 sig_g."""
    k = k0[:, None] + np.arange(width)[None, :]          # node index
    valid = (k >= 0) & (k < n_z)
    # hat edges: node k-1, k, k+1 clipped to the grid (half hats at the ends)
    zk = z_lo + k * dz
    lo = np.where(k > 0, zk - dz, zk)
    hi = np.where(k < n_z - 1, zk + dz, zk)
    m = mu[:, None]
    s = sig[:, None]
    t_lo = m - SUPPORT_SIGMAS * s
    t_hi = m + SUPPORT_SIGMAS * s

    def seg(a, b, c, sign):
        # int_a^b N(z) * sign * (z - c)/dz dz on [a, b] clipped to the truncated support
        a2 = np.maximum(a, t_lo)
        b2 = np.minimum(b, t_hi)
        ok = b2 > a2
        al = np.where(ok, (a2 - m) / s, 0.0)
        be = np.where(ok, (b2 - m) / s, 0.0)
        cdf = _phi_diff(al, be)
        pdf = (np.exp(-0.5 * al * al) - np.exp(-0.5 * be * be)) / math.sqrt(2 * math.pi)
        return np.where(ok, sign * (s * pdf + (m - c) * cdf) / dz, 0.0)

    rise = seg(lo, zk, lo, 1.0)         # (z - z_{k-1})/dz on [z_{k-1}, z_k]
    fall = seg(zk, hi, hi, -1.0)        # (z_{k+1} - z)/dz on [z_k, z_{k+1}]
    # the node integrals are >= 0; rounding can leave values a few ulp below
    j = np.where(valid, np.maximum(rise + fall, 0.0), 0.0)
    return np.clip(k, 0, n_z - 1), j, valid


def catalog_density(cat: synth.Catalog, n_z: int, z_lo: float, z_hi: float,
                    rows_pix: np.ndarray, chunk: int = 200_000):
    """(nz[n_rows, n_z], nz_tot[n_z], n_gal_used) for the HEALPix pixels rows_pix."""
    dz = (z_hi - z_lo) / (n_z - 1)
    tau = trapezoid_weights(n_z, z_lo, z_hi)
    grid = z_lo + dz * np.arange(n_z)
    vshape = _comoving_shape(grid)
    area = synth.pixel_area(cat.nside)
    row_of_pix = {int(p): i for i, p in enumerate(rows_pix)}
    lut = np.full(synth.nside_npix(cat.nside), -1, dtype=np.int64)
    lut[np.asarray(rows_pix, dtype=np.int64)] = np.arange(len(rows_pix))
    n_rows = len(rows_pix)
    acc_rows = np.zeros(n_rows * n_z)
    acc_tot = np.zeros(n_z)
    n_used = 0
    for s0 in range(0, cat.z_obs.size, chunk):
        mu = cat.z_obs[s0:s0 + chunk]
        pix = cat.pix[s0:s0 + chunk]
        sig = cat.sigma_z0 * (1.0 + mu)
        keep = (mu + SUPPORT_SIGMAS * sig >= z_lo) & (mu - SUPPORT_SIGMAS * sig <= z_hi) & (sig > 0)
        mu, pix, sig = mu[keep], pix[keep], sig[keep]
        k0 = np.floor((mu - SUPPORT_SIGMAS * sig - z_lo) / dz).astype(np.int64) - 1
        width = int(np.max(np.ceil(2 * SUPPORT_SIGMAS * sig / dz))) + 4 if mu.size else 0
        if width == 0:
            continue
        kk, j, valid = _hat_projection(mu, sig, z_lo, dz, n_z, k0, width)
        q = np.where(valid, j / tau[kk] * vshape[kk], 0.0)
        norm = np.sum(np.where(valid, tau[kk] * q, 0.0), axis=1)
        good = norm > 0
        q = q[good] / norm[good, None]
        kk, valid, pix = kk[good], valid[good], pix[good]
        n_used += int(good.sum())
        acc_tot += np.bincount(kk[valid], weights=q[valid], minlength=n_z)
        r = lut[pix]
        sel = r >= 0
        if np.any(sel):
            idx = (r[sel, None] * n_z + kk[sel])[valid[sel]]
            acc_rows += np.bincount(idx, weights=q[sel][valid[sel]], minlength=n_rows * n_z)
    nz = acc_rows.reshape(n_rows, n_z) / (n_used * area)
    nz_tot = acc_tot / n_used
    del row_of_pix
    return nz, nz_tot, n_used


def _chart(theta, phi):
    """The event's flat sky chart: gnomonic coordinates on the plane tangent at
    the normalised mean of the samples' unit vectors (east, north axes)."""
    v = synth.unit_vectors(theta, phi)
    m = v.sum(axis=0)
    m /= np.linalg.norm(m)
    ph0 = math.atan2(m[1], m[0])
    east = np.array([-math.sin(ph0), math.cos(ph0), 0.0])
    north = np.cross(m, east)

    def proj(u):
        d = u @ m
        return np.stack([(u @ east) / d, (u @ north) / d], axis=-1)

    return proj, proj(v)


def _sky_factors(theta, phi, centres_theta, centres_phi, area):
    """area x 2-D Scott KDE of (theta, phi) samples at the centres (tangent plane)."""
    proj, x = _chart(theta, phi)
    c = proj(synth.unit_vectors(centres_theta, centres_phi))
    n = x.shape[0]
    cov = np.cov(x.T, bias=False) * n ** (-1.0 / 3.0)
    inv = np.linalg.inv(cov)
    norm = 1.0 / (2 * math.pi * math.sqrt(np.linalg.det(cov)))
    out = np.empty(c.shape[0])
    for i in range(c.shape[0]):
        d = x - c[i]
        q = np.einsum("ij,jk,ik->i", d, inv, d)
        out[i] = norm * np.mean(np.exp(-0.5 * q))
    return area * out


def prepare(cat: synth.Catalog, ev: synth.Events, n_z: int, z_lo: float, z_hi: float,
            cred: float = 0.9, with_catalog: bool = True) -> Prepared:
    """Build the C-ABI arrays for one event set against one catalogue.  With
    with_catalog=False the catalogue rows are left to the device builder
    (nz and nz_tot are None; see galaxy_arrays)."""
    area = synth.pixel_area(ev.nside)
    ev_pix_off = [0]
    samp_off = [0]
    pix_id, c_list, s_list, dl_l, m1_l, m2_l = [], [], [], [], [], []
    for e in range(ev.n_events):
        sl = slice(ev.offsets[e], ev.offsets[e + 1])
        pix = ev.pix[sl]
        n_s = pix.size
        uniq, cnt = np.unique(pix, return_counts=True)
        order = np.lexsort((uniq, -cnt))              # count desc, id asc
        cum = np.cumsum(cnt[order])
        n_take = int(np.searchsorted(cum >= cred * n_s, True)) + 1
        region = np.sort(uniq[order[:n_take]])
        th_c, ph_c = synth.pix2ang_ring(ev.nside, region)
        s_ir = _sky_factors(ev.theta[sl], ev.phi[sl], th_c, ph_c, area)
        dle, m1e, m2e = ev.dl[sl], ev.m1d[sl], ev.m2d[sl]
        for r, p in enumerate(region):
            idx = np.nonzero(pix == p)[0]
            idx = idx[np.argsort(dle[idx], kind="stable")]
            pix_id.append(int(p))
            c_list.append(s_ir[r] / idx.size)
            s_list.append(s_ir[r])
            dl_l.append(dle[idx]); m1_l.append(m1e[idx]); m2_l.append(m2e[idx])
            samp_off.append(samp_off[-1] + idx.size)
        ev_pix_off.append(len(pix_id))
    pix_id = np.asarray(pix_id, dtype=np.int64)
    rows_pix = np.unique(pix_id)
    pix_row = np.searchsorted(rows_pix, pix_id).astype(np.int64)
    nz, nz_tot = None, None
    if with_catalog:
        nz, nz_tot, _ = catalog_density(cat, n_z, z_lo, z_hi, rows_pix)
    return Prepared(n_z=n_z, z_lo=z_lo, z_hi=z_hi, nz=nz, row_pix=rows_pix, nz_tot=nz_tot,
                    ev_pix_off=np.asarray(ev_pix_off, dtype=np.int64),
                    pix_samp_off=np.asarray(samp_off, dtype=np.int64),
                    pix_row=pix_row, pix_id=pix_id, c_ir=np.asarray(c_list),
                    dl=np.concatenate(dl_l), m1d=np.concatenate(m1_l), m2d=np.concatenate(m2_l),
                    s_ir=np.asarray(s_list))


def subset(p: Prepared, events) -> Prepared:
    """The prepared arrays of the listed events (in that order), sharing the
    catalogue rows."""
    ev_off = [0]
    samp_off = [0]
    rows, ids, cs, ss, dls, m1s, m2s = [], [], [], [], [], [], []
    for e in events:
        for q in range(p.ev_pix_off[e], p.ev_pix_off[e + 1]):
            a, b = p.pix_samp_off[q], p.pix_samp_off[q + 1]
            rows.append(p.pix_row[q]); ids.append(p.pix_id[q]); cs.append(p.c_ir[q])
            ss.append(p.s_ir[q] if p.s_ir is not None else np.nan)
            dls.append(p.dl[a:b]); m1s.append(p.m1d[a:b]); m2s.append(p.m2d[a:b])
            samp_off.append(samp_off[-1] + (b - a))
        ev_off.append(len(rows))
    return Prepared(p.n_z, p.z_lo, p.z_hi, p.nz, p.row_pix, p.nz_tot,
                    np.asarray(ev_off, np.int64), np.asarray(samp_off, np.int64),
                    np.asarray(rows, np.int64), np.asarray(ids, np.int64),
                    np.asarray(cs, np.float64), np.concatenate(dls), np.concatenate(m1s),
                    np.concatenate(m2s), None if p.s_ir is None else np.asarray(ss, np.float64))


@dataclass
class ThreeD:
    """Arrays of chimera_add_events_3d: every sample of each event with its
    position in the event's flat sky chart, and the region's pixels with their
    centres in that chart and their areas."""
    ev_samp_off: np.ndarray   # [E+1] int64
    dl: np.ndarray            # [S]
    m1d: np.ndarray
    m2d: np.ndarray
    sky_u: np.ndarray         # [S] chart coordinates
    sky_v: np.ndarray
    ev_pix_off: np.ndarray    # [E+1] int64
    pix_row: np.ndarray       # [P] int64
    pix_u: np.ndarray         # [P]
    pix_v: np.ndarray
    pix_area: np.ndarray      # [P] sr

    @property
    def n_events(self) -> int:
        return len(self.ev_samp_off) - 1


def three_d(p: Prepared, ev: synth.Events, events=None) -> ThreeD:
    """The 3D-kernel arrays of the events p was prepared from (all of them, or
    the listed ones in that order)."""
    events = range(p.n_events) if events is None else list(events)
    area = synth.pixel_area(ev.nside)
    samp_off, pix_off = [0], [0]
    cols = {k: [] for k in ("dl", "m1d", "m2d", "su", "sv", "row", "pu", "pv")}
    for e in events:
        a, b = int(ev.offsets[e]), int(ev.offsets[e + 1])
        proj, x = _chart(ev.theta[a:b], ev.phi[a:b])
        q0, q1 = p.ev_pix_off[e], p.ev_pix_off[e + 1]
        th, ph = synth.pix2ang_ring(ev.nside, p.pix_id[q0:q1])
        c = proj(synth.unit_vectors(th, ph))
        cols["dl"].append(ev.dl[a:b]); cols["m1d"].append(ev.m1d[a:b]); cols["m2d"].append(ev.m2d[a:b])
        cols["su"].append(x[:, 0]); cols["sv"].append(x[:, 1])
        cols["row"].append(p.pix_row[q0:q1]); cols["pu"].append(c[:, 0]); cols["pv"].append(c[:, 1])
        samp_off.append(samp_off[-1] + (b - a))
        pix_off.append(pix_off[-1] + (q1 - q0))
    cat = {k: np.concatenate(v) for k, v in cols.items()}
    return ThreeD(np.asarray(samp_off, np.int64), cat["dl"], cat["m1d"], cat["m2d"], cat["su"],
                  cat["sv"], np.asarray(pix_off, np.int64), cat["row"].astype(np.int64), cat["pu"],
                  cat["pv"], np.full(cat["row"].size, area))


def single1d(p: Prepared, ev: synth.Events, events=None) -> Single1D:
    """The single-1D arrays of the events p was prepared from (all of them, or
    the listed ones in that order): the region, rows and sky factors of p,
    and every raw sample of each event."""
    events = range(p.n_events) if events is None else list(events)
    samp_off, pix_off = [0], [0]
    dls, m1s, m2s, rows, ss = [], [], [], [], []
    for e in events:
        a, b = int(ev.offsets[e]), int(ev.offsets[e + 1])
        dls.append(ev.dl[a:b]); m1s.append(ev.m1d[a:b]); m2s.append(ev.m2d[a:b])
        samp_off.append(samp_off[-1] + (b - a))
        q0, q1 = p.ev_pix_off[e], p.ev_pix_off[e + 1]
        rows.append(p.pix_row[q0:q1]); ss.append(p.s_ir[q0:q1])
        pix_off.append(pix_off[-1] + (q1 - q0))
    return Single1D(np.asarray(samp_off, np.int64), np.concatenate(dls), np.concatenate(m1s),
                    np.concatenate(m2s), np.asarray(pix_off, np.int64),
                    np.concatenate(rows).astype(np.int64), np.concatenate(ss).astype(np.float64))


def galaxy_arrays(cat: synth.Catalog, n_z: int, z_lo: float, z_hi: float):
    """Inputs of the device catalogue builder (chimera_set_catalog_galaxies):
    galaxies sorted by pixel with their pixel offsets, sigma_z = sigma0 (1 + z_obs),
    the comoving volume shape on the grid and the pixel area."""
    npix = synth.nside_npix(cat.nside)
    order = np.argsort(cat.pix, kind="stable")
    pix = cat.pix[order]
    off = np.searchsorted(pix, np.arange(npix + 1)).astype(np.int64)
    z = np.ascontiguousarray(cat.z_obs[order], dtype=np.float64)
    sig = cat.sigma_z0 * (1.0 + z)
    grid = z_lo + (z_hi - z_lo) / (n_z - 1) * np.arange(n_z)
    return off, z, sig, _comoving_shape(grid), synth.pixel_area(cat.nside)

