"""The lambda-independent pre-computation (TEST INFRASTRUCTURE; see header).

Sect. 2.3, steps a-c, and the many-1D kernel (eq. gw-kernel-many1d):
* region: the event's localisation area is divided in equal-area pixels;
  reading: pixels ordered by sample count (descending, ties by ascending
  pixel id) are taken until at least `cred` (0.9: the 90% area of Fig. 1)
  of the event's samples are covered; samples outside are dropped;
* flat sky chart (the 3D kernel): gnomonic coordinates on the plane tangent
  at the normalised mean of the samples' unit vectors (the plane of the sky
  factor below);
* sky factor: the 2-D KDE of all the event's sky samples at the pixel centre,
  times the pixel area (the d^2 Omega of eq. like-integrals over one pixel);
  reading: Gaussian KDE in the gnomonic tangent plane at the samples' mean
  direction, Scott bandwidth (covariance x S^(-1/3) in 2-D); c_ir = S_ir/N_ir;
* catalogue density (eq. p-cat): a sum over galaxies of the normalised
  N(z; z_obs, sigma_z) dV_c/dz, sigma_z = sigma_z0 (1 + z_obs) (Sect. 4).
  Reading for the grid: each galaxy's Gaussian, truncated at 8 sigma, is
  projected on the hat (linear-interpolation) basis of the grid,
  J_k = int N Lambda_k dz, from the antiderivative of (z - c) N(z); the node value is
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


def _segment(a, b, c, mu, sig):
    """int_a^b (z - c) N(z; mu, sig) dz, a <= b, with the antiderivative
    -sig phi(u) + (mu - c) Phi(u); the Phi difference is taken on the side of
    the Gaussian where it does not cancel."""
    al, be = (a - mu) / sig, (b - mu) / sig
    dphi = np.where(al >= 0.0, ndtr(-al) - ndtr(-be), ndtr(be) - ndtr(al))
    dpdf = (np.exp(-0.5 * al * al) - np.exp(-0.5 * be * be)) / math.sqrt(2.0 * math.pi)
    return sig * dpdf + (mu - c) * dphi


def hat_integrals(mu, sig, grid, support=8.0):
    """J[k] = int N(z; mu, sig) Lambda_k(z) dz over |z - mu| <= support sig.

    Lambda_k rises linearly on [z_{k-1}, z_k] and falls on [z_k, z_{k+1}]; at
    the grid's ends only one half exists.
    """
    dz = grid[1] - grid[0]
    lo_t, hi_t = mu - support * sig, mu + support * sig
    j = np.zeros(grid.size)
    for k in range(grid.size):
        tot = 0.0
        if k > 0:                                    # rising half: (z - z_{k-1}) / dz
            a, b = max(grid[k - 1], lo_t), min(grid[k], hi_t)
            if b > a:
                tot += _segment(a, b, grid[k - 1], mu, sig) / dz
        if k < grid.size - 1:                        # falling half: (z_{k+1} - z) / dz
            a, b = max(grid[k], lo_t), min(grid[k + 1], hi_t)
            if b > a:
                tot -= _segment(a, b, grid[k + 1], mu, sig) / dz
        j[k] = max(tot, 0.0)
    return j


def catalog(z_obs, pix, sigma_z0, grid, rows_pix, area, support=8.0):
    """Catalog(grid, rows{pix: n_r}, n_tot).

    Reading: each galaxy's Gaussian is truncated at `support` sigma (beyond it
    the density is below e^-32 of its peak); galaxies whose truncated Gaussian
    misses the grid are dropped.  Loops over galaxies; for each, the hat
    integrals of the nodes whose hats meet the truncated support.
    """
    tau = trapezoid(grid)
    vol = cosmo.comoving_volume_element(grid, REF_H0, REF_OM)
    dz = grid[1] - grid[0]
    n = grid.size
    want = {int(p): i for i, p in enumerate(rows_pix)}
    rows = np.zeros((len(want), n))
    tot = np.zeros(n)
    used = 0
    # vectorised over galaxies: every galaxy gets the same number of candidate
    # nodes around its mean; nodes whose hats miss the support integrate to 0
    sig_all = sigma_z0 * (1.0 + z_obs)
    width = int(np.ceil(2 * support * np.max(sig_all) / dz)) + 4
    for s0 in range(0, z_obs.size, 50_000):
        mu = z_obs[s0:s0 + 50_000]
        px = pix[s0:s0 + 50_000]
        sig = sig_all[s0:s0 + 50_000]
        k = np.floor((mu - support * sig - grid[0]) / dz).astype(np.int64)[:, None] - 1 \
            + np.arange(width)[None, :]
        inside = (k >= 0) & (k < n)
        kc = np.clip(k, 0, n - 1)
        zk = grid[kc]
        lo_t = (mu - support * sig)[:, None]
        hi_t = (mu + support * sig)[:, None]
        m, s = mu[:, None], sig[:, None]
        J = np.zeros(k.shape)
        # rising half
        prev = grid[np.clip(kc - 1, 0, n - 1)]
        a, b = np.maximum(prev, lo_t), np.minimum(zk, hi_t)
        ok = inside & (kc > 0) & (b > a)
        J += np.where(ok, _segment(np.where(ok, a, m), np.where(ok, b, m), prev, m, s) / dz, 0.0)
        # falling half
        nxt = grid[np.clip(kc + 1, 0, n - 1)]
        a, b = np.maximum(zk, lo_t), np.minimum(nxt, hi_t)
        ok = inside & (kc < n - 1) & (b > a)
        J -= np.where(ok, _segment(np.where(ok, a, m), np.where(ok, b, m), nxt, m, s) / dz, 0.0)
        J = np.maximum(J, 0.0)
        q = np.where(inside, J / tau[kc] * vol[kc], 0.0)
        norm = np.sum(tau[kc] * q, axis=1)
        good = norm > 0
        q, kc, inside, px = q[good] / norm[good, None], kc[good], inside[good], px[good]
        used += int(good.sum())
        tot += np.bincount(kc[inside], weights=q[inside], minlength=n)
        r = np.array([want.get(int(p), -1) for p in px], dtype=np.int64)
        sel = (r >= 0)[:, None] & inside
        flat = (r[:, None] * n + kc)[sel]
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
        mean = _vec(theta[sl], phi[sl]).sum(axis=0)
        mean = mean / math.sqrt(float(mean @ mean))
        suv = tangent_plane(theta[sl], phi[sl], mean)
        cuv = tangent_plane(ct, cp, mean)
        ev = Event(samples=(dl[sl], m1d[sl], m2d[sl]), sky_uv=(suv[:, 0], suv[:, 1]))
        for r, p in enumerate(reg):
            m = px == p
            ev.pixels.append(Pixel(pix=p, c=s[r] / int(m.sum()), dl=dl[sl][m], m1d=m1d[sl][m],
                                   m2d=m2d[sl][m], s=float(s[r]),
                                   uv=(float(cuv[r, 0]), float(cuv[r, 1])), area=area))
        out.append(ev)
    return out
