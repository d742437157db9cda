"""Brute force: ln L of tiny inputs (2 events, <= 8 samples, <= 3 pixels, a
20-point grid, 50 injections) evaluated at 30 significant digits with mpmath,
every step written out here from its definition (eq. dL-em and dL-mg with
adaptive quadrature and a bracketed root, the PLP mass model of Sect. 3.1,
the weighted Gaussian KDE of eq. gw-kernel-many1d, or the one per-event KDE
times the pixels' sky factors of eq. gw-kernel-single1d, summed over the grid, the
injection estimator of Sect. 2.2, eq. hyperlike); the oracle (dense, T = inf)
must agree to 1e-13."""
import mpmath as mp
import numpy as np
import pytest

import oracle

C = mp.mpf("299792.458")


def mp_lnl(events, grid, rows, n_tot, inj, lam, kernel="many1d", extra=None):
    mp.mp.dps = 30
    h0, om, xi0, n, alpha, beta, mmin, mmax, mu, sg, lg, gam, kap, zp = [mp.mpf(float(x)) for x in lam]

    def E(z):
        return mp.sqrt(om * (1 + z) ** 3 + 1 - om)

    chi_cache = {}

    def chi(z):
        key = mp.nstr(z, 40)
        if key not in chi_cache:
            chi_cache[key] = mp.quad(lambda t: 1 / E(t), [0, z])
        return chi_cache[key]

    def Xi(z):
        return xi0 + (1 - xi0) * (1 + z) ** (-n)

    def D(z):
        return C / h0 * (1 + z) * chi(z) * Xi(z)

    def Dz(z):
        # d/dz of (c/H0)(1+z) chi Xi, chi' = 1/E
        return C / h0 * ((chi(z) + (1 + z) / E(z)) * Xi(z)
                         + (1 + z) * chi(z) * (-n) * (1 - xi0) * (1 + z) ** (-n - 1))

    def z_of(d):
        d = mp.mpf(float(d))
        return mp.findroot(lambda z: D(z) - d, (mp.mpf(0), mp.mpf(25)), solver="anderson")

    npl = (mmax ** (1 - alpha) - mmin ** (1 - alpha)) / (1 - alpha)
    Z = mp.ncdf((mmax - mu) / sg) - mp.ncdf((mmin - mu) / sg)

    def p1(m):
        if m < mmin or m > mmax:
            return mp.mpf(0)
        return (1 - lg) * m ** (-alpha) / npl + lg * mp.npdf(m, mu, sg) / Z

    def p2(m2, m1):
        if m2 < mmin or m2 > m1 or m1 <= mmin:
            return mp.mpf(0)
        return m2 ** beta * (1 + beta) / (m1 ** (1 + beta) - mmin ** (1 + beta))

    def psi(z):
        return (1 + z) ** gam / (1 + ((1 + z) / (1 + zp)) ** (gam + kap))

    g = [mp.mpf(float(x)) for x in grid]
    dz = g[1] - g[0]
    tau = [dz / 2 if k in (0, len(g) - 1) else dz for k in range(len(g))]
    gfac = [psi(zg) / ((1 + zg) ** 3 * Dz(zg)) for zg in g]
    lnI = []
    for e, ev in enumerate(events):
        zs, ws, pix = [], [], []
        groups = list(enumerate((dl, m1d, m2d) for _c, _row, dl, m1d, m2d in ev))
        if kernel == "single1d" and extra is not None:
            groups.append((-1, extra[e]))      # samples outside every pixel
        for p, (dl, m1d, m2d) in groups:
            for d, a, b in zip(dl, m1d, m2d):
                z = z_of(d)
                zs.append(z)
                ws.append(p1(mp.mpf(float(a)) / (1 + z)) * p2(mp.mpf(float(b)) / (1 + z),
                                                              mp.mpf(float(a)) / (1 + z)))
                pix.append(p)
        W1 = mp.fsum(ws)
        W2 = mp.fsum(w * w for w in ws)
        mean = mp.fsum(w * z for w, z in zip(ws, zs)) / W1
        var = mp.fsum(w * (z - mean) ** 2 for w, z in zip(ws, zs)) / (W1 - W2 / W1)
        h = max(mp.sqrt(var) * (W1 * W1 / W2) ** mp.mpf("-0.2"), 2 * dz)
        total = mp.mpf(0)
        if kernel == "single1d":
            # eq. gw-kernel-single1d: one KDE over every sample of the event,
            # times the pixel's sky factor c_r N_r
            kde = [mp.fsum(w * mp.npdf(g[k], z, h) for z, w in zip(zs, ws)) / len(zs)
                   for k in range(len(g))]
            for p, (c, row, *_r) in enumerate(ev):
                n_p = sum(1 for q in pix if q == p)
                total += mp.mpf(float(c)) * n_p * mp.fsum(
                    tau[k] * mp.mpf(float(row[k])) * gfac[k] * kde[k] for k in range(len(g)))
        else:
            for p, (c, row, *_r) in enumerate(ev):
                for z, w, q in zip(zs, ws, pix):
                    if q != p:
                        continue
                    A = mp.fsum(tau[k] * mp.npdf(g[k], z, h) * mp.mpf(float(row[k])) * gfac[k]
                                for k in range(len(g)))
                    total += mp.mpf(float(c)) * w * A
        lnI.append(mp.log(total))
    s = []
    nt = [mp.mpf(float(x)) for x in n_tot]
    for d, a, b, lp in zip(inj["dl"], inj["m1d"], inj["m2d"], inj["lnp"]):
        z = z_of(d)
        w = p1(mp.mpf(float(a)) / (1 + z)) * p2(mp.mpf(float(b)) / (1 + z), mp.mpf(float(a)) / (1 + z))
        pos = (z - g[0]) / dz
        if pos < 0 or pos > len(g) - 1:
            continue
        k = min(int(mp.floor(pos)), len(g) - 2)
        t = pos - k
        ntz = nt[k] + t * (nt[k + 1] - nt[k])
        s.append(w * ntz * psi(z) / ((1 + z) ** 3 * Dz(z) * mp.exp(mp.mpf(float(lp)))))
    xi = mp.fsum(s) / inj["n_total"]
    return mp.fsum(lnI) - len(events) * mp.log(xi), [float(v) for v in lnI]


def tiny_inputs(seed):
    rng = np.random.default_rng(seed)
    grid = np.linspace(0.05, 1.9, 20)
    rows = [np.exp(-0.5 * ((grid - c) / 0.3) ** 2) + 0.1 for c in (0.6, 0.9, 1.3)]
    n_tot = np.mean(rows, axis=0)
    events = []
    for e, npx in enumerate((2, 3)):
        ev = []
        for p in range(npx):
            k = int(rng.integers(2, 4))
            dl = rng.uniform(2000.0, 12000.0, k)
            m1 = rng.uniform(15.0, 55.0, k)
            m2 = m1 * rng.uniform(0.5, 0.95, k)
            ev.append((float(rng.uniform(0.2, 1.0)), rows[(e + p) % 3], dl, m1, m2))
        events.append(ev)
    inj = {"dl": rng.uniform(500.0, 12000.0, 50), "m1d": rng.uniform(10.0, 120.0, 50),
           "lnp": rng.uniform(-14.0, -10.0, 50), "n_total": 400}
    inj["m2d"] = inj["m1d"] * rng.uniform(0.3, 1.0, 50)
    return events, grid, rows, n_tot, inj


@pytest.mark.parametrize("kernel", ["many1d", "single1d"])
@pytest.mark.parametrize("seed,lam", [
    (1, [70.0, 0.3, 1.0, 1.91, 3.4, 1.1, 5.0, 87.0, 34.0, 3.6, 0.04, 2.7, 3.0, 2.0]),
    (2, [62.0, 0.41, 1.6, 2.5, 2.2, -0.4, 6.0, 80.0, 30.0, 5.0, 0.3, 1.9, 2.6, 1.4]),
])
def test_oracle_matches_30_digit_brute_force(seed, lam, kernel):
    L = oracle.likelihood
    events, grid, rows, n_tot, inj = tiny_inputs(seed)
    o_events = []
    for ev in events:
        e = L.Event()
        for p, (c, row, dl, m1, m2) in enumerate(ev):
            e.pixels.append(L.Pixel(pix=next(i for i, r in enumerate(rows) if r is row), c=c,
                                    dl=dl, m1d=m1, m2d=m2))
        o_events.append(e)
    extra = None
    if kernel == "single1d":
        # two samples per event outside its pixels: they enter the single-1D
        # KDE and bandwidth, not the many-1D sums
        rng = np.random.default_rng(100 + seed)
        extra = []
        for e in o_events:
            m1 = rng.uniform(15.0, 55.0, 2)
            x = (rng.uniform(2000.0, 12000.0, 2), m1, m1 * rng.uniform(0.5, 0.95, 2))
            extra.append(x)
            e.samples = tuple(np.concatenate([getattr(px, a) for px in e.pixels] + [x[k]])
                              for k, a in enumerate(("dl", "m1d", "m2d")))
    cat = L.Catalog(grid=grid, rows={i: r for i, r in enumerate(rows)}, n_tot=n_tot)
    o_inj = L.InjectionSet(inj["dl"], inj["m1d"], inj["m2d"], inj["lnp"], inj["n_total"])
    ref = L.lnl(o_events, cat, o_inj, np.array(lam), kernel=kernel)
    if seed == 1:      # this case checks Scott's rule itself, not the 2 dz floor
        assert np.all(ref["h"] > 2.0 * (grid[1] - grid[0]))
    want, lnI = mp_lnl(events, grid, rows, n_tot, inj, lam, kernel=kernel, extra=extra)
    assert np.allclose(ref["lnI"], lnI, rtol=1e-13, atol=0.0)
    assert abs(ref["lnl"] - float(want)) <= 1e-13 * abs(float(want))
