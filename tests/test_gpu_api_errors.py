"""Error behaviour of the C-ABI as declared in include/chimera.h: argument
checks, call order, resident-data consistency and the HBM budget.  Small
handmade inputs; no parity claim (the results are only compared with
themselves)."""
import numpy as np
import pytest

from paper_2504_02034_amd import synth

pytestmark = pytest.mark.gpu

N_Z = 200


def catalog(n_rows):
    z = np.linspace(0.0, 1.6, N_Z)
    rows = np.stack([np.exp(-0.5 * ((z - c) / 0.2) ** 2) + 0.05 for c in np.linspace(0.3, 1.1, n_rows)])
    return rows, rows.mean(axis=0)


def events():
    """Two events: rows 0 and 1, and row 2."""
    rng = np.random.default_rng(3)
    ev_pix_off = np.array([0, 2, 3])
    pix_samp_off = np.array([0, 6, 10, 17])
    pix_row = np.array([0, 1, 2])
    c_ir = np.array([0.4, 0.7, 1.1])
    S = pix_samp_off[-1]
    dl = rng.uniform(1500.0, 4000.0, S)
    m1 = rng.uniform(20.0, 60.0, S)
    m2 = m1 * rng.uniform(0.5, 0.95, S)
    return ev_pix_off, pix_samp_off, pix_row, c_ir, dl, m1, m2


def injections():
    rng = np.random.default_rng(4)
    n = 200
    m1 = rng.uniform(10.0, 120.0, n)
    return (rng.uniform(500.0, 8000.0, n), m1, m1 * rng.uniform(0.3, 1.0, n),
            rng.uniform(-14.0, -10.0, n), 1000)


def context(chimera, **kw):
    ctx = chimera.Context(n_z=N_Z, z_lo=0.0, z_hi=1.6, **kw)
    rows, tot = catalog(3)
    ctx.set_catalog(rows, tot)
    ctx.set_injections(*injections())
    return ctx


def status(excinfo):
    return excinfo.value.status


@pytest.fixture(scope="module")
def chimera():
    from paper_2504_02034_amd import chimera as c
    return c


def test_batch_and_precision_arguments(chimera):
    ctx = context(chimera)
    es = ctx.add_events(*events())
    lam = synth.LAMBDA_TRUTH[None, :]
    assert np.isfinite(ctx.lnl(es, lam)[0])
    with pytest.raises(chimera.ChimeraError) as e:
        ctx.lnl(es, np.empty((0, 14)))
    assert status(e) == chimera.CHIMERA_EINVAL
    with pytest.raises(chimera.ChimeraError) as e:
        ctx.lnl(es, lam, prec=5)
    assert status(e) == chimera.CHIMERA_EINVAL
    with pytest.raises(chimera.ChimeraError) as e:
        ctx.lnl_grad(es, lam, prec=5)
    assert status(e) == chimera.CHIMERA_EINVAL
    ctx.close()


def test_call_order(chimera):
    ctx = chimera.Context(n_z=N_Z, z_lo=0.0, z_hi=1.6)
    with pytest.raises(chimera.ChimeraError) as e:
        ctx.add_events(*events())
    assert status(e) == chimera.CHIMERA_ESTATE
    rows, tot = catalog(3)
    ctx.set_catalog(rows, tot)
    es = ctx.add_events(*events())
    with pytest.raises(chimera.ChimeraError) as e:
        ctx.lnl(es, synth.LAMBDA_TRUTH[None, :])
    assert status(e) == chimera.CHIMERA_ESTATE
    ctx.close()


def test_event_set_checks(chimera):
    ctx = context(chimera)
    ev_pix_off, pix_samp_off, pix_row, c_ir, dl, m1, m2 = events()
    cases = [
        ((ev_pix_off, pix_samp_off, np.array([0, 1, 3]), c_ir, dl, m1, m2), chimera.CHIMERA_ERANGE),
        ((ev_pix_off, pix_samp_off, pix_row, c_ir, np.where(np.arange(dl.size) == 4, -1.0, dl), m1, m2),
         chimera.CHIMERA_EINVAL),
        ((ev_pix_off, pix_samp_off, pix_row, np.array([0.4, 0.0, 1.1]), dl, m1, m2),
         chimera.CHIMERA_EINVAL),
        ((np.array([0, 2, 2, 3]), pix_samp_off, pix_row, c_ir, dl, m1, m2), chimera.CHIMERA_EINVAL),
        ((ev_pix_off, np.array([0, 6, 6, 17]), pix_row, c_ir, dl, m1, m2), chimera.CHIMERA_EINVAL),
    ]
    for args, want in cases:
        with pytest.raises(chimera.ChimeraError) as e:
            ctx.add_events(*args)
        assert status(e) == want
    # one event over more pixel rows than an LDS slice can hold
    n = chimera.CHIMERA_MAX_EVENT_PIXELS + 1
    with pytest.raises(chimera.ChimeraError) as e:
        ctx.add_events(np.array([0, n]), np.arange(n + 1), np.zeros(n, np.int64), np.ones(n),
                       np.full(n, 2000.0), np.full(n, 40.0), np.full(n, 30.0))
    assert status(e) == chimera.CHIMERA_ERANGE
    ctx.close()


def test_smaller_catalogue_refused_while_events_refer_to_its_rows(chimera):
    ctx = context(chimera)
    es = ctx.add_events(*events())
    lam = synth.make_lambdas(synth.WORKLOADS["precision_300ev"])[:4]
    before = ctx.lnl(es, lam)
    rows, tot = catalog(2)                   # the event set uses row 2
    with pytest.raises(chimera.ChimeraError) as e:
        ctx.set_catalog(rows, tot)
    assert status(e) == chimera.CHIMERA_ERANGE
    gal_pix_off = np.array([0, 2, 3])
    with pytest.raises(chimera.ChimeraError) as e:
        ctx.set_catalog_galaxies(gal_pix_off, np.array([0.3, 0.5, 0.8]), np.full(3, 0.01),
                                 np.ones(N_Z), 1e-3, np.array([0, 1]))
    assert status(e) == chimera.CHIMERA_ERANGE
    # the resident catalogue is unchanged
    assert np.array_equal(ctx.lnl(es, lam), before, equal_nan=True)
    es.release()
    ctx.set_catalog(rows, tot)
    ctx.close()


def test_release_is_checked(chimera):
    ctx = context(chimera)
    es = ctx.add_events(*events())
    h = es.handle
    es.release()
    with pytest.raises(chimera.ChimeraError) as e:
        chimera.chimera_release_events(ctx.handle, h)
    assert status(e) == chimera.CHIMERA_EINVAL
    ctx.close()


def test_hbm_budget_bounds_a_call(chimera):
    ctx = context(chimera, hbm_budget=1 << 16)
    es = ctx.add_events(*events())
    with pytest.raises(chimera.ChimeraError) as e:
        ctx.lnl(es, synth.LAMBDA_TRUTH[None, :])
    assert status(e) == chimera.CHIMERA_ENOMEM
    with pytest.raises(chimera.ChimeraError) as e:
        ctx.lnl_grad(es, synth.LAMBDA_TRUTH[None, :])
    assert status(e) == chimera.CHIMERA_ENOMEM
    ctx.close()


def test_population_option_arguments(chimera):
    """chimera_set_completeness, chimera_set_mass_smoothing and
    chimera_lambda_width: null and out-of-range arguments, call order, and a
    replaced catalogue dropping the completeness."""
    import ctypes
    lib = chimera.lib
    assert lib.chimera_set_mass_smoothing(None, 1) == chimera.CHIMERA_EINVAL
    ctx0 = chimera.Context(n_z=N_Z, z_lo=0.0, z_hi=1.6)
    with pytest.raises(chimera.ChimeraError) as e:
        ctx0.set_completeness(np.full((3, N_Z), 0.5), np.zeros(N_Z))
    assert status(e) == chimera.CHIMERA_ESTATE
    assert lib.chimera_lambda_width(ctx0.handle, None) == chimera.CHIMERA_EINVAL
    w = ctypes.c_int32()
    assert lib.chimera_lambda_width(ctx0.handle, ctypes.byref(w)) == 0 and w.value == 14
    ctx0.close()
    ctx = context(chimera)
    es = ctx.add_events(*events())
    lam = synth.LAMBDA_TRUTH[None, :]
    plain = ctx.lnl(es, lam)
    p = np.full((3, N_Z), 0.5)
    for bad_p, bad_m in ((p, None), (p, np.full(N_Z, 13.0)), (p, np.full(N_Z, -0.1)),
                         (np.full((3, N_Z), -0.2), np.zeros(N_Z))):
        with pytest.raises(chimera.ChimeraError) as e:
            ctx.set_completeness(bad_p, bad_m)
        assert status(e) == chimera.CHIMERA_EINVAL
    assert np.array_equal(ctx.lnl(es, lam), plain)        # refused calls change nothing
    ctx.set_completeness(p, np.full(N_Z, 2.0 * np.pi))
    assert not np.array_equal(ctx.lnl(es, lam), plain)
    rows, tot = catalog(3)
    ctx.set_catalog(rows, tot)                             # a new catalogue is complete
    assert np.array_equal(ctx.lnl(es, lam), plain)
    ctx.set_mass_smoothing(True)
    assert ctx.lam_width == 15
    with pytest.raises(ValueError):
        ctx.lnl(es, lam)
    assert np.isfinite(ctx.lnl(es, np.append(synth.LAMBDA_TRUTH, 4.8)[None, :])[0])
    ctx.close()
