"""ctypes binding of libchimera.so (include/chimera.h), argument marshalling only.

Every step of the likelihood runs in the HIP library; this module converts
numpy arrays and torch tensors into pointers.  Importing it raises if the
library has not been built: there is no CPU fallback.

Functions keep the C names (chimera_create, chimera_lnl_batch, ...); the
classes Context / EventSet are thin owners of the opaque handles.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libchimera.so")

CHIMERA_OK, CHIMERA_EINVAL, CHIMERA_ENOMEM, CHIMERA_EDEVICE, CHIMERA_ERANGE, CHIMERA_ESTATE = (
    0, -1, -2, -3, -4, -5)
CHIMERA_FP64, CHIMERA_FP32 = 0, 1
CHIMERA_HOST, CHIMERA_DEVICE = 0, 1
CHIMERA_MAX_EVENT_PIXELS = 2560
CHIMERA_KDE_GAUSSIAN, CHIMERA_KDE_EPANECHNIKOV = 0, 1
CHIMERA_MAX_BINS = 4096
NLAM, NGRAD = 14, 12

_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ERANGE", -5: "ESTATE"}

#: every symbol include/chimera.h declares
EXPORTS = ("chimera_default_config", "chimera_create", "chimera_destroy", "chimera_last_error",
           "chimera_set_catalog", "chimera_set_catalog_galaxies", "chimera_get_catalog",
           "chimera_set_injections",
           "chimera_add_events", "chimera_add_events_single1d", "chimera_add_events_3d",
           "chimera_set_event_kde", "chimera_set_neff_gate", "chimera_set_completeness",
           "chimera_set_mass_smoothing", "chimera_lambda_width",
           "chimera_release_events", "chimera_lnl_batch", "chimera_lnl_batch_static",
           "chimera_selection_xi",
           "chimera_lnl_grad", "chimera_scratch_bytes", "chimera_grad_scratch_bytes",
           "chimera_scratch_held",
           "chimera_release_scratch", "chimera_profile_enable", "chimera_profile_read")


class ChimeraError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("n_z", ctypes.c_int32), ("z_lo", ctypes.c_double), ("z_hi", ctypes.c_double),
                ("n_tab", ctypes.c_int32), ("z_tab_max", ctypes.c_double),
                ("trunc_fp64", ctypes.c_double), ("trunc_fp32", ctypes.c_double),
                ("device", ctypes.c_int32), ("hbm_budget", ctypes.c_size_t)]


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(the likelihood has no CPU path)")
    # One HIP runtime per process: torch ships its own libamdhip64.so.7; when
    # it is loaded first, the library's dependency on that soname resolves to
    # the same copy, so device pointers and streams from torch are valid here.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "chimera_default_config": (None, [ctypes.POINTER(Config)]),
        "chimera_create": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(_P)]),
        "chimera_destroy": (None, [_P]),
        "chimera_last_error": (ctypes.c_char_p, []),
        "chimera_set_catalog": (ctypes.c_int, [_P, _I64, _P, _P]),
        "chimera_set_injections": (ctypes.c_int, [_P, _I64, _I64, _P, _P, _P, _P]),
        "chimera_get_catalog": (ctypes.c_int, [_P, _P, _P]),
        "chimera_set_catalog_galaxies": (ctypes.c_int, [_P, _I64, _I64, _P, _P, _P, _P,
                                                        ctypes.c_double, _I64, _P,
                                                        ctypes.POINTER(_I64)]),
        "chimera_add_events": (ctypes.c_int, [_P, _I32, _P, _P, _P, _P, _P, _P, _P,
                                              ctypes.POINTER(_P)]),
        "chimera_add_events_single1d": (ctypes.c_int, [_P, _I32, _P, _P, _P, _P, _P, _P, _P,
                                                       ctypes.POINTER(_P)]),
        "chimera_add_events_3d": (ctypes.c_int, [_P, _I32] + [_P] * 11 + [ctypes.POINTER(_P)]),
        "chimera_set_event_kde": (ctypes.c_int, [_P, _P, _I32, _I32]),
        "chimera_set_neff_gate": (ctypes.c_int, [_P, ctypes.c_double]),
        "chimera_set_mass_smoothing": (ctypes.c_int, [_P, _I32]),
        "chimera_lambda_width": (ctypes.c_int, [_P, ctypes.POINTER(_I32)]),
        "chimera_set_completeness": (ctypes.c_int, [_P, _P, _P]),
        "chimera_release_events": (ctypes.c_int, [_P, _P]),
        "chimera_lnl_batch": (ctypes.c_int, [_P, _P, _P, _I64, _I32, _P, _P, _I32, _P]),
        "chimera_lnl_batch_static": (ctypes.c_int, [_P, _P, _P, _I64, _I32, _P, _P, _P]),
        "chimera_selection_xi": (ctypes.c_int, [_P, _P, _I64, _I32, _P, _P, _I32, _P]),
        "chimera_lnl_grad": (ctypes.c_int, [_P, _P, _P, _I64, _I32, _P, _P, _I32, _P]),
        "chimera_scratch_bytes": (ctypes.c_int, [_P, _P, _I64, _I32, _I32,
                                                 ctypes.POINTER(ctypes.c_size_t)]),
        "chimera_grad_scratch_bytes": (ctypes.c_int, [_P, _P, _I64, _I32, _I32,
                                                      ctypes.POINTER(ctypes.c_size_t)]),
        "chimera_scratch_held": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
        "chimera_release_scratch": (ctypes.c_int, [_P, _P]),
        "chimera_profile_enable": (ctypes.c_int, [_P, _I32]),
        "chimera_profile_read": (ctypes.c_int, [_P, ctypes.POINTER(_I64),
                                                ctypes.POINTER(ctypes.c_double),
                                                ctypes.POINTER(_I64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def _check(status):
    if status != CHIMERA_OK:
        raise ChimeraError(status, lib.chimera_last_error().decode())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(_P)


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


# ---------------------------------------------------------------------------
# C names
# ---------------------------------------------------------------------------
def chimera_default_config() -> Config:
    c = Config()
    lib.chimera_default_config(ctypes.byref(c))
    return c


def chimera_create(cfg: Config):
    h = _P()
    _check(lib.chimera_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h


def chimera_destroy(h):
    lib.chimera_destroy(h)


def chimera_set_catalog(h, nz, nz_tot):
    nz, pnz = _host(nz, np.float64)
    nt, pnt = _host(nz_tot, np.float64)
    _check(lib.chimera_set_catalog(h, nz.shape[0] if nz.ndim == 2 else 0, pnz, pnt))


def chimera_set_catalog_galaxies(h, gal_pix_off, z_obs, sigma_z, vshape, pixel_area, rows_pix):
    """Device-built catalogue rows; returns the number of galaxies used."""
    o, po = _host(gal_pix_off, np.int64)
    z, pz = _host(z_obs, np.float64)
    sg, ps = _host(sigma_z, np.float64)
    v, pv = _host(vshape, np.float64)
    r, pr = _host(rows_pix, np.int64)
    used = _I64()
    _check(lib.chimera_set_catalog_galaxies(h, o.size - 1, z.size, po, pz, ps, pv,
                                            float(pixel_area), r.size, pr, ctypes.byref(used)))
    return used.value


def chimera_get_catalog(h, n_rows, n_z):
    """(nz [n_rows, n_z], nz_tot [n_z]) copied from the device."""
    nz = np.empty((n_rows, n_z))
    nt = np.empty(n_z)
    _check(lib.chimera_get_catalog(h, nz.ctypes.data_as(_P), nt.ctypes.data_as(_P)))
    return nz, nt


def chimera_set_injections(h, dl, m1d, m2d, ln_pdraw, n_inj_total):
    a = [_host(x, np.float64) for x in (dl, m1d, m2d, ln_pdraw)]
    _check(lib.chimera_set_injections(h, a[0][0].size, int(n_inj_total), *[p for _, p in a]))


def chimera_add_events(h, ev_pix_off, pix_samp_off, pix_row, c_ir, dl, m1d, m2d):
    o1, p1 = _host(ev_pix_off, np.int64)
    o2, p2 = _host(pix_samp_off, np.int64)
    o3, p3 = _host(pix_row, np.int64)
    rest = [_host(x, np.float64) for x in (c_ir, dl, m1d, m2d)]
    ev = _P()
    _check(lib.chimera_add_events(h, o1.size - 1, p1, p2, p3, *[p for _, p in rest],
                                  ctypes.byref(ev)))
    return ev


def chimera_add_events_single1d(h, ev_samp_off, dl, m1d, m2d, ev_pix_off, pix_row, s_ir):
    o1, p1 = _host(ev_samp_off, np.int64)
    samp = [_host(x, np.float64) for x in (dl, m1d, m2d)]
    o2, p2 = _host(ev_pix_off, np.int64)
    o3, p3 = _host(pix_row, np.int64)
    o4, p4 = _host(s_ir, np.float64)
    if o2.size != o1.size:
        raise ValueError("ev_samp_off and ev_pix_off must both have n_ev + 1 entries")
    ev = _P()
    _check(lib.chimera_add_events_single1d(h, o1.size - 1, p1, *[p for _, p in samp], p2, p3, p4,
                                           ctypes.byref(ev)))
    return ev


def chimera_add_events_3d(h, ev_samp_off, dl, m1d, m2d, sky_u, sky_v, ev_pix_off, pix_row,
                          pix_u, pix_v, pix_area):
    o1, p1 = _host(ev_samp_off, np.int64)
    samp = [_host(x, np.float64) for x in (dl, m1d, m2d, sky_u, sky_v)]
    o2, p2 = _host(ev_pix_off, np.int64)
    o3, p3 = _host(pix_row, np.int64)
    pix = [_host(x, np.float64) for x in (pix_u, pix_v, pix_area)]
    if o2.size != o1.size:
        raise ValueError("ev_samp_off and ev_pix_off must both have n_ev + 1 entries")
    ev = _P()
    _check(lib.chimera_add_events_3d(h, o1.size - 1, p1, *[p for _, p in samp], p2, p3,
                                     *[p for _, p in pix], ctypes.byref(ev)))
    return ev


def chimera_set_completeness(h, p_compl, missing):
    if p_compl is None:
        _check(lib.chimera_set_completeness(h, None, None))
        return
    a, pa = _host(p_compl, np.float64)
    m, pm = _host(missing, np.float64)
    _check(lib.chimera_set_completeness(h, pa, pm))


def chimera_set_neff_gate(h, factor):
    _check(lib.chimera_set_neff_gate(h, float(factor)))


def chimera_set_mass_smoothing(h, on):
    _check(lib.chimera_set_mass_smoothing(h, 1 if on else 0))


def chimera_lambda_width(h) -> int:
    w = _I32()
    _check(lib.chimera_lambda_width(h, ctypes.byref(w)))
    return w.value


def _check_lam(h, lam):
    """The library reads lambda rows of the context's width: refuse others."""
    w = chimera_lambda_width(h)
    if len(lam.shape) != 2 or lam.shape[1] != w:
        raise ValueError(f"lambda must be [B, {w}] for this context, got {tuple(lam.shape)}")


def chimera_set_event_kde(h, ev, shape, n_bins):
    _check(lib.chimera_set_event_kde(h, ev, int(shape), int(n_bins)))


def chimera_release_events(h, ev):
    _check(lib.chimera_release_events(h, ev))


def _stream_ptr(stream):
    if stream is None:
        import torch
        return _P(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return _P(stream)
    return _P(stream.cuda_stream)


def chimera_lnl_batch(h, ev, lam, prec=CHIMERA_FP64, lnl=None, lnI=None, n_ev=None, stream=None):
    """lam: numpy [B, width] (host call) or a torch tensor on the device (async
    call); width 14, or 15 with the smoothed mass edge."""
    if _is_torch(lam):
        import torch
        assert lam.is_cuda and lam.dtype == torch.float64 and lam.is_contiguous()
        _check_lam(h, lam)
        B = lam.shape[0]
        if lnl is None:
            lnl = torch.empty(B, dtype=torch.float64, device=lam.device)
        _check(lib.chimera_lnl_batch(h, ev, _P(lam.data_ptr()), B, prec, _P(lnl.data_ptr()),
                                     _P(lnI.data_ptr()) if lnI is not None else None,
                                     CHIMERA_DEVICE, _stream_ptr(stream)))
        return lnl
    lam, pl = _host(np.atleast_2d(lam), np.float64)
    _check_lam(h, lam)
    B = lam.shape[0]
    out = np.empty(B)
    lnI_arr = None
    if n_ev is not None:
        lnI_arr = np.empty((B, n_ev))
    _check(lib.chimera_lnl_batch(h, ev, pl, B, prec, out.ctypes.data_as(_P),
                                 lnI_arr.ctypes.data_as(_P) if lnI_arr is not None else None,
                                 CHIMERA_HOST, None))
    return (out, lnI_arr) if n_ev is not None else out


def chimera_lnl_batch_static(h, ev, lam, prec=CHIMERA_FP64, lnl=None, lnI=None, stream=None):
    """Device-mode ln L with the library's static scratch (no allocation in the
    call): lam, lnl (and lnI) are torch tensors on the device."""
    import torch
    assert lam.is_cuda and lam.dtype == torch.float64 and lam.is_contiguous()
    _check_lam(h, lam)
    B = lam.shape[0]
    if lnl is None:
        lnl = torch.empty(B, dtype=torch.float64, device=lam.device)
    _check(lib.chimera_lnl_batch_static(h, ev, _P(lam.data_ptr()), B, prec, _P(lnl.data_ptr()),
                                        _P(lnI.data_ptr()) if lnI is not None else None,
                                        _stream_ptr(stream)))
    return lnl


def chimera_selection_xi(h, lam, prec=CHIMERA_FP64, stream=None):
    if _is_torch(lam):
        import torch
        assert lam.is_cuda and lam.dtype == torch.float64 and lam.is_contiguous()
        _check_lam(h, lam)
        B = lam.shape[0]
        lx = torch.empty(B, dtype=torch.float64, device=lam.device)
        ne = torch.empty(B, dtype=torch.float64, device=lam.device)
        _check(lib.chimera_selection_xi(h, _P(lam.data_ptr()), B, prec, _P(lx.data_ptr()),
                                        _P(ne.data_ptr()), CHIMERA_DEVICE, _stream_ptr(stream)))
        return lx, ne
    lam, pl = _host(np.atleast_2d(lam), np.float64)
    _check_lam(h, lam)
    B = lam.shape[0]
    lx, ne = np.empty(B), np.empty(B)
    _check(lib.chimera_selection_xi(h, pl, B, prec, lx.ctypes.data_as(_P), ne.ctypes.data_as(_P),
                                    CHIMERA_HOST, None))
    return lx, ne


def chimera_lnl_grad(h, ev, lam, prec=CHIMERA_FP64, lnl=None, grad=None, stream=None):
    """(lnl [B], grad [B,12]); lam numpy [B,14] (host call) or a device tensor (async)."""
    if _is_torch(lam):
        import torch
        assert lam.is_cuda and lam.dtype == torch.float64 and lam.is_contiguous()
        _check_lam(h, lam)
        B = lam.shape[0]
        if lnl is None:
            lnl = torch.empty(B, dtype=torch.float64, device=lam.device)
        if grad is None:
            grad = torch.empty(B, NGRAD, dtype=torch.float64, device=lam.device)
        _check(lib.chimera_lnl_grad(h, ev, _P(lam.data_ptr()), B, prec, _P(lnl.data_ptr()),
                                    _P(grad.data_ptr()), CHIMERA_DEVICE, _stream_ptr(stream)))
        return lnl, grad
    lam, pl = _host(np.atleast_2d(lam), np.float64)
    _check_lam(h, lam)
    B = lam.shape[0]
    out, g = np.empty(B), np.empty((B, NGRAD))
    _check(lib.chimera_lnl_grad(h, ev, pl, B, prec, out.ctypes.data_as(_P), g.ctypes.data_as(_P),
                                CHIMERA_HOST, None))
    return out, g


def chimera_scratch_bytes(h, ev, B, prec=CHIMERA_FP64, mem=CHIMERA_DEVICE) -> int:
    out = ctypes.c_size_t()
    _check(lib.chimera_scratch_bytes(h, ev, int(B), prec, mem, ctypes.byref(out)))
    return out.value


def chimera_grad_scratch_bytes(h, ev, B, prec=CHIMERA_FP64, mem=CHIMERA_DEVICE) -> int:
    out = ctypes.c_size_t(0)
    _check(lib.chimera_grad_scratch_bytes(h, ev, int(B), prec, mem, ctypes.byref(out)))
    return out.value


def chimera_scratch_held(h) -> int:
    out = ctypes.c_size_t()
    _check(lib.chimera_scratch_held(h, ctypes.byref(out)))
    return out.value


def chimera_release_scratch(h, stream=None):
    _check(lib.chimera_release_scratch(h, _stream_ptr(stream)))


def chimera_profile_enable(h, on=True):
    _check(lib.chimera_profile_enable(h, 1 if on else 0))


def chimera_profile_read(h):
    """(event-kernel launches, their summed ms, summed (sample, grid point) evaluations)."""
    n, ms, ev = _I64(), ctypes.c_double(), _I64()
    _check(lib.chimera_profile_read(h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(ev)))
    return n.value, ms.value, ev.value


# ---------------------------------------------------------------------------
# owners
# ---------------------------------------------------------------------------
class EventSet:
    def __init__(self, ctx: "Context", handle, n_events: int):
        self.ctx, self.handle, self.n_events = ctx, handle, n_events

    def release(self):
        if self.handle is not None and self.ctx.handle is not None:
            chimera_release_events(self.ctx.handle, self.handle)
        self.handle = None


class Context:
    """Owns one chimera_ctx: resident catalogue, injections and event sets."""

    def __init__(self, n_z=1000, z_lo=0.0, z_hi=1.6, device=0, hbm_budget=0, **kw):
        cfg = chimera_default_config()
        cfg.n_z, cfg.z_lo, cfg.z_hi, cfg.device, cfg.hbm_budget = n_z, z_lo, z_hi, device, hbm_budget
        for k, v in kw.items():
            setattr(cfg, k, v)
        self.cfg = cfg
        self.handle = chimera_create(cfg)

    def close(self):
        if self.handle is not None:
            chimera_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_catalog(self, nz, nz_tot):
        chimera_set_catalog(self.handle, nz, nz_tot)

    def set_catalog_galaxies(self, gal_pix_off, z_obs, sigma_z, vshape, pixel_area, rows_pix):
        return chimera_set_catalog_galaxies(self.handle, gal_pix_off, z_obs, sigma_z, vshape,
                                            pixel_area, rows_pix)

    def get_catalog(self, n_rows):
        return chimera_get_catalog(self.handle, n_rows, self.cfg.n_z)

    def set_injections(self, dl, m1d, m2d, ln_pdraw, n_inj_total):
        chimera_set_injections(self.handle, dl, m1d, m2d, ln_pdraw, n_inj_total)

    def add_events(self, ev_pix_off, pix_samp_off, pix_row, c_ir, dl, m1d, m2d) -> EventSet:
        h = chimera_add_events(self.handle, ev_pix_off, pix_samp_off, pix_row, c_ir, dl, m1d, m2d)
        return EventSet(self, h, len(ev_pix_off) - 1)

    def add_prepared(self, p) -> EventSet:
        """Resident event set from prep.Prepared."""
        return self.add_events(p.ev_pix_off, p.pix_samp_off, p.pix_row, p.c_ir, p.dl, p.m1d, p.m2d)

    def add_events_single1d(self, ev_samp_off, dl, m1d, m2d, ev_pix_off, pix_row,
                            s_ir) -> EventSet:
        h = chimera_add_events_single1d(self.handle, ev_samp_off, dl, m1d, m2d, ev_pix_off,
                                        pix_row, s_ir)
        return EventSet(self, h, len(ev_samp_off) - 1)

    def set_completeness(self, p_compl, missing=None):
        """Incomplete catalogue: P_compl [n_rows][n_z] and M(z) [n_z]; None clears it."""
        chimera_set_completeness(self.handle, p_compl, missing)

    def set_neff_gate(self, factor):
        """ln L = -inf where N_eff <= factor x n_events (0: off)."""
        chimera_set_neff_gate(self.handle, factor)

    def set_mass_smoothing(self, on=True):
        """Lambda rows of 15 entries, delta_m (the smoothed lower mass edge) last."""
        chimera_set_mass_smoothing(self.handle, on)

    @property
    def lam_width(self) -> int:
        return chimera_lambda_width(self.handle)

    def set_event_kde(self, ev: EventSet, shape=None, n_bins=0):
        """Kernel options of an event set: shape CHIMERA_KDE_GAUSSIAN (default)
        or CHIMERA_KDE_EPANECHNIKOV, n_bins 0 (unbinned) or the bins per KDE."""
        chimera_set_event_kde(self.handle, ev.handle,
                              CHIMERA_KDE_GAUSSIAN if shape is None else shape, n_bins)

    def add_events_3d(self, ev_samp_off, dl, m1d, m2d, sky_u, sky_v, ev_pix_off, pix_row, pix_u,
                      pix_v, pix_area) -> EventSet:
        h = chimera_add_events_3d(self.handle, ev_samp_off, dl, m1d, m2d, sky_u, sky_v, ev_pix_off,
                                  pix_row, pix_u, pix_v, pix_area)
        return EventSet(self, h, len(ev_samp_off) - 1)

    def add_prepared_3d(self, t) -> EventSet:
        """Resident 3D event set from prep.ThreeD."""
        return self.add_events_3d(t.ev_samp_off, t.dl, t.m1d, t.m2d, t.sky_u, t.sky_v, t.ev_pix_off,
                                  t.pix_row, t.pix_u, t.pix_v, t.pix_area)

    def add_prepared_single1d(self, s) -> EventSet:
        """Resident single-1D event set from prep.Single1D."""
        return self.add_events_single1d(s.ev_samp_off, s.dl, s.m1d, s.m2d, s.ev_pix_off,
                                        s.pix_row, s.s_ir)

    def lnl(self, ev: EventSet, lam, prec=CHIMERA_FP64, with_lnI=False, lnl=None, lnI=None,
            stream=None):
        if _is_torch(lam):
            return chimera_lnl_batch(self.handle, ev.handle, lam, prec, lnl=lnl, lnI=lnI,
                                     stream=stream)
        return chimera_lnl_batch(self.handle, ev.handle, lam, prec,
                                 n_ev=ev.n_events if with_lnI else None)

    def selection(self, lam, prec=CHIMERA_FP64, stream=None):
        return chimera_selection_xi(self.handle, lam, prec, stream=stream)

    def scratch_bytes(self, ev: EventSet, B, prec=CHIMERA_FP64, mem=CHIMERA_DEVICE) -> int:
        return chimera_scratch_bytes(self.handle, ev.handle if ev is not None else None, B, prec,
                                     mem)

    def grad_scratch_bytes(self, ev: EventSet, B, prec=CHIMERA_FP64, mem=CHIMERA_DEVICE) -> int:
        return chimera_grad_scratch_bytes(self.handle, ev.handle, B, prec, mem)

    def scratch_held(self) -> int:
        return chimera_scratch_held(self.handle)

    def release_scratch(self, stream=None):
        chimera_release_scratch(self.handle, stream)

    def lnl_grad(self, ev: EventSet, lam, prec=CHIMERA_FP64, stream=None):
        """(ln L [B], d ln L / d(GRAD_NAMES) [B, 12])."""
        return chimera_lnl_grad(self.handle, ev.handle, lam, prec, stream=stream)


def context_from_prepared(p, inj, device=0, **kw) -> tuple:
    """(Context, EventSet) with the catalogue rows, injections and events of prep.Prepared."""
    ctx = Context(n_z=p.n_z, z_lo=p.z_lo, z_hi=p.z_hi, device=device, **kw)
    ctx.set_catalog(p.nz, p.nz_tot)
    ctx.set_injections(inj.dl, inj.m1d, inj.m2d, inj.ln_pdraw, inj.n_total)
    return ctx, ctx.add_prepared(p)
