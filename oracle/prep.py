"""The lambda-independent pre-computation (TEST INFRASTRUCTURE; see header).

Sect. 2.3, steps a-c, and the many-1D kernel (eq. gw-kernel-many1d):
* region: the event's localisation area is divided in equal-area pixels;
  reading: pixels ordered by sample count (descending, ties by ascending
  pixel id) are taken until at least `cred` (0.9: the 90% area of Fig. 1)
  of the event's samples are covered; samples outside are dropped;
* sky factor: the 2-D KDE of all the event's sky samples at the pixel centre,
  times the pixel area (the d^2 Omega of eq. like-integrals over one pixel);
  reading: Gaussian KDE in the gnomonic tangent plane at the samples' mean
  direction, Scott bandwidth (covariance x S^(-1/3) in 2-D); c_ir = S_ir/N_ir;
* catalogue density (eq. p-cat): a sum over galaxies of the normalised
  N(z; z_obs, sigma_z) dV_c/dz, sigma_z = sigma_z0 (1 + z_obs) (Sect. 4).
  Reading for the grid: each galaxy's Gaussian is projected on the hat
  (linear-interpolation) basis of the grid, J_k = int N Lambda_k dz,
  computed here as the second difference of the Gaussian's second
  antiderivative G(z) = (z-mu) Phi(u) + sigma phi(u); the node value is
  J_k / tau_k x dV_c/dz(z_k) at the frozen reference cosmology (H0=70,
  Om=0.3; the paper fixes Om and H0 cancels), normalised to
  sum_k tau_k q_k = 1.  Galaxies whose Gaussian lies beyond 8 sigma of the
  grid are dropped.  n_r = sum_{gal in r} q / (N_gal * pixel area).

Pins: tests/test_oracle_prep.py (2-D KDE vs scipy.stats.gaussian_kde, hat
integrals vs scipy quad and their partition of unity, n normalisation).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ndtr

from . import cosmology as cosmo
from .likelihood import Catalog, Event, Pixel, trapezoid

REF_H0, REF_OM = 70.0, 0.3


def region(pix, cred=0.9):
    counts = {}
    for p in pix.tolist():
        counts[p] = counts.get(p, 0) + 1
    order = sorted(counts.items(), key=lambda kv: (-kv[1], kv[0]))
    taken, cum = [], 0
    for p, c in order:
        taken.append(p)
        cum += c
        if cum >= cred * pix.size:
            break
    return sorted(taken)


def _vec(theta, phi):
    return np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)], -1)


def tangent_plane(theta, phi, ref):
    """Gnomonic coordinates of (theta, phi) on the plane tangent at unit vector ref."""
    th0 = math.acos(max(-1.0, min(1.0, ref[2])))
    ph0 = math.atan2(ref[1], ref[0])
    e_r = np.array([math.sin(th0) * math.cos(ph0), math.sin(th0) * math.sin(ph0), math.cos(th0)])
    e_e = np.array([-math.sin(ph0), math.cos(ph0), 0.0])
    e_n = np.array([-math.cos(th0) * math.cos(ph0), -math.cos(th0) * math.sin(ph0), math.sin(th0)])
    u = _vec(theta, phi)
    return np.stack([(u @ e_e) / (u @ e_r), (u @ e_n) / (u @ e_r)], axis=-1)


def kde2d(x, at):
    """(1/S) sum_j N2(at; x_j, Sigma), Sigma = unbiased covariance x S^(-1/3)."""
    s = x.shape[0]
    d = x - x.mean(axis=0)
    cov = (d.T @ d) / (s - 1) * s ** (-1.0 / 3.0)
    det = cov[0, 0] * cov[1, 1] - cov[0, 1] * cov[1, 0]
    inv = np.array([[cov[1, 1], -cov[0, 1]], [-cov[1, 0], cov[0, 0]]]) / det
    out = np.empty(at.shape[0])
    for r in range(at.shape[0]):
        dd = x - at[r]
        q = inv[0, 0] * dd[:, 0] ** 2 + 2 * inv[0, 1] * dd[:, 0] * dd[:, 1] + inv[1, 1] * dd[:, 1] ** 2
        out[r] = np.sum(np.exp(-0.5 * q)) / (s * 2.0 * math.pi * math.sqrt(det))
    return out


def sky_factors(theta, phi, c_theta, c_phi, area):
    """S_ir = area x 2-D KDE of all the event's sky samples at the pixel centres."""
    v = _vec(theta, phi)
    mean = v.sum(axis=0)
    mean = mean / math.sqrt(float(mean @ mean))
    return area * kde2d(tangent_plane(theta, phi, mean), tangent_plane(c_theta, c_phi, mean))


def hat_integrals(mu, sig, grid):
    """J[k] = int N(z; mu, sig) Lambda_k(z) dz for all grid nodes k."""
    dz = grid[1] - grid[0]
    u = (grid - mu) / sig
    G = (grid - mu) * ndtr(u) + sig * np.exp(-0.5 * u * u) / math.sqrt(2 * math.pi)
    F = ndtr(u)
    j = np.empty(grid.size)
    j[1:-1] = (G[2:] - 2.0 * G[1:-1] + G[:-2]) / dz
    j[0] = (G[1] - G[0] - dz * F[0]) / dz
    j[-1] = (G[-2] - G[-1] + dz * F[-1]) / dz
    return j


def catalog(z_obs, pix, sigma_z0, grid, rows_pix, area, support=8.0, chunk=100_000):
    """Catalog(grid, rows{pix: n_r}, n_tot).

    Each galaxy touches the nodes within `support` sigma of its mean (plus one
    node each side); outside them its Gaussian is below e^-32 of the peak.
    Galaxies are processed in vectorised chunks; the arithmetic per galaxy
    is that of hat_integrals on the window extended by one node each side,
    so that the window's own end nodes are full hats unless they are the
    grid's ends.
    """
    tau = trapezoid(grid)
    vol = cosmo.comoving_volume_element(grid, REF_H0, REF_OM)
    dz = grid[1] - grid[0]
    n = grid.size
    want = {int(p): i for i, p in enumerate(rows_pix)}
    rows = np.zeros((len(want), n))
    tot = np.zeros(n)
    used = 0
    for s0 in range(0, z_obs.size, chunk):
        mu = z_obs[s0:s0 + chunk]
        px = pix[s0:s0 + chunk]
        sig = sigma_z0 * (1.0 + mu)
        ok = (sig > 0) & (mu + support * sig >= grid[0]) & (mu - support * sig <= grid[-1])
        mu, px, sig = mu[ok], px[ok], sig[ok]
        if mu.size == 0:
            continue
        lo = np.maximum(0, np.floor((mu - support * sig - grid[0]) / dz).astype(np.int64) - 1)
        hi = np.minimum(n, np.ceil((mu + support * sig - grid[0]) / dz).astype(np.int64) + 2)
        width = int(np.max(hi - lo))
        # node indices k = lo + m, m in [-1, width]; G evaluated on them
        m = np.arange(-1, width + 1)
        k = lo[:, None] + m[None, :]
        kc = np.clip(k, 0, n - 1)
        zk = grid[0] + dz * k
        u = (zk - mu[:, None]) / sig[:, None]
        G = (zk - mu[:, None]) * ndtr(u) + sig[:, None] * np.exp(-0.5 * u * u) / math.sqrt(2 * math.pi)
        F = ndtr(u)
        J = (G[:, 2:] - 2.0 * G[:, 1:-1] + G[:, :-2]) / dz       # interior hats at k = lo + [0, width)
        kk = k[:, 1:-1]
        first = kk == 0
        last = kk == n - 1
        J = np.where(first, (G[:, 2:] - G[:, 1:-1] - dz * F[:, 1:-1]) / dz, J)
        J = np.where(last, (G[:, :-2] - G[:, 1:-1] + dz * F[:, 1:-1]) / dz, J)
        inside = (kk >= lo[:, None]) & (kk < hi[:, None]) & (kk >= 0) & (kk < n)
        kkc = kc[:, 1:-1]
        q = np.where(inside, J / tau[kkc] * vol[kkc], 0.0)
        norm = np.sum(tau[kkc] * q, axis=1)
        good = norm > 0
        q = q[good] / norm[good, None]
        kkc, inside, px = kkc[good], inside[good], px[good]
        used += int(good.sum())
        tot += np.bincount(kkc[inside], weights=q[inside], minlength=n)
        r = np.array([want.get(int(p), -1) for p in px], dtype=np.int64)
        sel = (r >= 0)[:, None] & inside
        flat = (r[:, None] * n + kkc)[sel]
        rows += np.bincount(flat, weights=q[sel], minlength=rows.size).reshape(rows.shape)
    rows /= used * area
    return Catalog(grid=grid, rows={p: rows[i] for p, i in want.items()}, n_tot=tot / used)


def events(offsets, dl, m1d, m2d, theta, phi, pix, centres, area, cred=0.9):
    """List of likelihood.Event for raw per-event samples; centres(pix)->(theta, phi)."""
    out = []
    for e in range(len(offsets) - 1):
        sl = slice(offsets[e], offsets[e + 1])
        px = pix[sl]
        reg = region(px, cred)
        ct, cp = centres(np.asarray(reg, dtype=np.int64))
        s = sky_factors(theta[sl], phi[sl], ct, cp, area)
        ev = Event()
        for r, p in enumerate(reg):
            m = px == p
            ev.pixels.append(Pixel(pix=p, c=s[r] / int(m.sum()), dl=dl[sl][m], m1d=m1d[sl][m],
                                   m2d=m2d[sl][m]))
        out.append(ev)
    return out
