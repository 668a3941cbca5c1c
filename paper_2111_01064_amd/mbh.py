"""Thin ctypes binding of libmbh (include/mbh.h): argument marshalling only.

Every function here forwards to the C entry point of the same name (without
the ``mbh_`` prefix); all computation happens in the HIP kernels of
``libmbh.so``.  PyTorch is used only for device memory and streams: device
arguments are ``torch`` CUDA tensors whose ``data_ptr()`` is passed through,
and the work is enqueued on ``torch.cuda.current_stream()``.

If ``libmbh.so`` has not been built this module raises on import: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmbh.so")

MBH_OK, MBH_EINVAL, MBH_ENOMEM, MBH_EBAND, MBH_EDEVICE, MBH_EAGAIN, MBH_ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
MODEL_IMR, MODEL_TF2 = 0, 1
MODE_22, MODE_33, MODE_44, MODE_21, MODE_32, MODE_43 = (1 << i for i in range(6))
MODES_ALL = 0x3F
FP64, MIXED = 0, 1
STAGE_SETUP, STAGE_MAIN, STAGE_FINISH = 1, 2, 3
NPARAM = 11

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                      "(the likelihoods have no CPU fallback)")
_L = ct.CDLL(LIB_PATH)


class MbhError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _L.mbh_last_error().decode()
        super().__init__(f"{where}: {_L.mbh_strerror(status).decode()} ({status}): {msg}")
        self.status = status


class _RefInfo(ct.Structure):
    _fields_ = [("model", ct.c_int32), ("n_chan", ct.c_int32), ("n_bins", ct.c_int32), ("modes", ct.c_uint32),
                ("k_lo", ct.c_int64), ("k_hi", ct.c_int64), ("lnL0", ct.c_double), ("dd", ct.c_double),
                ("dh0", ct.c_double), ("hh0", ct.c_double)]


class ServerConfig(ct.Structure):
    _fields_ = [("max_inflight", ct.c_int32), ("max_batch_walkers", ct.c_int32),
                ("hbm_budget_bytes", ct.c_size_t), ("prec", ct.c_int)]


class RequestSpec(ct.Structure):
    _fields_ = [("t_arrival_s", ct.c_double), ("ref_index", ct.c_int32), ("reserved", ct.c_int32),
                ("W", ct.c_int64), ("theta_row", ct.c_int64)]


class SamplerConfig(ct.Structure):
    _fields_ = [("n_temps", ct.c_int32), ("walkers_per_temp", ct.c_int32), ("stretch_a", ct.c_double),
                ("p_sky_all", ct.c_double), ("p_sky_lon", ct.c_double), ("p_sky_lat", ct.c_double),
                ("seed", ct.c_uint64), ("prec", ct.c_int), ("mixed_rungs", ct.c_int32)]


class Likelihood(ct.Structure):
    _fields_ = [("ref", ct.c_void_p), ("data", ct.c_void_p), ("modes", ct.c_uint32)]


class SamplerStop(ct.Structure):
    _fields_ = [("check_every", ct.c_int32), ("snr_stop", ct.c_double), ("lnl_tol", ct.c_double),
                ("lnl_checks", ct.c_int32), ("refresh_every", ct.c_int32), ("refresh_data", ct.c_void_p),
                ("max_iter", ct.c_int64)]


class SamplerReport(ct.Structure):
    _fields_ = [("iterations", ct.c_int64), ("reason", ct.c_int32), ("checks", ct.c_int32),
                ("refreshes", ct.c_int32), ("max_lnL", ct.c_double), ("best_snr", ct.c_double),
                ("seconds", ct.c_double)]


class ServerStats(ct.Structure):
    _fields_ = [("submitted", ct.c_uint64), ("completed", ct.c_uint64), ("batches", ct.c_uint64),
                ("walkers", ct.c_uint64), ("max_walkers_in_flight", ct.c_uint64),
                ("max_bytes_in_flight", ct.c_uint64), ("admission_waits", ct.c_uint64),
                ("host_build_s", ct.c_double), ("host_complete_s", ct.c_double)]


_vp, _dp, _i64, _u32, _i32, _d, _sz = ct.c_void_p, ct.POINTER(ct.c_double), ct.c_int64, ct.c_uint32, ct.c_int, ct.c_double, ct.c_size_t
_pp = ct.POINTER(ct.c_void_p)
_SIGS = {
    "mbh_create": [_i32, _sz, _pp],
    "mbh_destroy": [_vp],
    "mbh_memory_in_use": [_vp, ct.POINTER(ct.c_size_t)],
    "mbh_data_create": [_vp, _i32, _i64, _d, _d, _d, _vp, _vp, _vp, _pp],
    "mbh_data_release": [_vp],
    "mbh_data_inner_dd": [_vp, _dp],
    "mbh_tdi_to_aet_fd": [_vp, _i64, _d, _d, _vp, _d, _i64, _i64, _vp, _vp],
    "mbh_data_create_tdi": [_vp, _i64, _d, _d, _vp, _d, _i64, _i64, _vp, _d, _vp, _pp],
    "mbh_template_full": [_vp, _vp, _i32, _u32, _dp, _vp, _vp],
    "mbh_build_reference_coeffs": [_vp, _vp, _i32, _u32, _dp, _i32, _vp, _pp],
    "mbh_ref_release": [_vp],
    "mbh_ref_get_info": [_vp, ct.POINTER(_RefInfo)],
    "mbh_ref_export": [_vp, _dp, ct.POINTER(ct.c_int64), _dp, _dp, _dp, _dp, _dp],
    "mbh_build_reference_coeffs_pm": [_vp, _vp, _i32, _u32, _dp, ct.POINTER(ct.c_int32), _vp, _pp],
    "mbh_ref_pm_info": [_vp, ct.POINTER(ct.c_uint32), ct.POINTER(ct.c_int32)],
    "mbh_ref_pm_mode": [_vp, _i32, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32), _dp,
                        ct.POINTER(ct.c_int64), _dp, _dp, _dp, _dp, _dp],
    "mbh_ref_pm_pair": [_vp, _i32, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32), _dp,
                        ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32), _dp, _dp],
    "mbh_ref_refresh": [_vp, _vp, _vp, _vp, _vp, _i64, _vp],
    "mbh_ref_refresh_result": [_vp, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32)],
    "mbh_ref_refresh_prepare": [_vp, _vp],
    "mbh_loglike_heterodyned": [_vp, _vp, _vp, _i64, _i32, _vp, _vp, _vp],
    "mbh_loglike_heterodyned_noalloc": [_vp, _vp, _vp, _i64, _i32, _vp, _vp, _vp],
    "mbh_loglike_full": [_vp, _vp, _i32, _u32, _vp, _i64, _i32, _vp, _vp, _vp],
    "mbh_batch_create": [_vp, _i32, _pp, _pp, ct.POINTER(ct.c_int64), _pp, _pp, _i32, _pp],
    "mbh_batch_create_prec": [_vp, _i32, _pp, _pp, ct.POINTER(ct.c_int64), _pp, _pp, ct.POINTER(ct.c_int32), _pp],
    "mbh_batch_launch": [_vp, _vp],
    "mbh_batch_launch_stage": [_vp, _i32, _vp],
    "mbh_batch_launch_direct": [_vp, _vp],
    "mbh_batch_fp64_segments": [_vp, ct.POINTER(ct.c_uint64)],
    "mbh_batch_release": [_vp],
    "mbh_autotune_heterodyned": [_vp, _vp, _vp, _i64, _i32, ct.POINTER(ct.c_int)],
    "mbh_lanes_for": [_vp, _i32, _i32, _i32, ct.POINTER(ct.c_int)],
    "mbh_set_lanes": [_vp, _i32, _i32, _i32, _i32],
    "mbh_set_mixed_tolerance": [_vp, _d],
    "mbh_get_mixed_tolerance": [_vp, _dp],
    "mbh_set_full_shape": [_vp, _i32, _i32, _i32],
    "mbh_full_shape": [_vp, _i32, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int)],
    "mbh_autotune_full": [_vp, _vp, _i32, _u32, _vp, _i64, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int)],
    "mbh_autotune_save": [_vp, ct.c_char_p],
    "mbh_autotune_load": [_vp, ct.c_char_p],
    "mbh_server_create": [_vp, _i32, _pp, ct.POINTER(ServerConfig), _pp],
    "mbh_server_submit": [_vp, _i32, _dp, _i64, ct.POINTER(ct.c_uint64)],
    "mbh_server_wait": [_vp, ct.c_uint64, _i32, _dp, _dp, _i64, _dp],
    "mbh_server_refresh": [_vp, _i32, _vp, _dp, _dp, _i64, ct.POINTER(ct.c_uint64)],
    "mbh_server_replay": [_vp, ct.POINTER(RequestSpec), _i64, _dp, _i64, _dp, _dp, _dp, _dp],
    "mbh_server_get_stats": [_vp, ct.POINTER(ServerStats)],
    "mbh_sampler_create": [_vp, ct.POINTER(SamplerConfig), _dp, _dp, _dp, _pp],
    "mbh_sampler_destroy": [_vp],
    "mbh_sampler_set_walkers": [_vp, _dp, _dp, ct.POINTER(Likelihood), _vp],
    "mbh_sampler_step": [_vp, ct.POINTER(Likelihood), _i64, _vp],
    "mbh_sampler_step_served": [_vp, _vp, _i32, _i64, _vp, _dp],
    "mbh_sampler_propose": [_vp, _i32, _vp],
    "mbh_sampler_proposals": [_vp, _dp, _dp, ct.POINTER(ct.c_int32)],
    "mbh_sampler_accept": [_vp, _i32, _vp, _vp, _vp],
    "mbh_sampler_swap": [_vp, _vp],
    "mbh_sampler_get": [_vp, _dp, _dp, _dp, ct.POINTER(ct.c_int64)],
    "mbh_sampler_stats": [_vp, ct.POINTER(ct.c_uint64), ct.POINTER(ct.c_uint64), ct.POINTER(ct.c_uint64)],
    "mbh_sampler_run": [_vp, ct.POINTER(Likelihood), ct.POINTER(SamplerStop), _vp, ct.POINTER(SamplerReport)],
    "mbh_server_destroy": [_vp],
}
for _name, _args in _SIGS.items():
    _f = getattr(_L, _name)
    _f.argtypes = _args
    _f.restype = ct.c_int32
_L.mbh_last_error.restype = ct.c_char_p
_L.mbh_last_error.argtypes = []
_L.mbh_strerror.restype = ct.c_char_p
_L.mbh_strerror.argtypes = [ct.c_int32]


def _check(status: int, where: str):
    if status != MBH_OK:
        raise MbhError(status, where)


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _dev_ptr(t: torch.Tensor, dtype, shape=None) -> int:
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous CUDA tensor of {dtype}, got {t.dtype} on {t.device}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


def _host_theta(theta) -> np.ndarray:
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1))
    if th.size != NPARAM:
        raise ValueError("theta must have 11 entries")
    return th


# ------------------------------------------------------------------ handles
class Context:
    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = ct.c_void_p()
        _check(_L.mbh_create(device, hbm_budget_bytes, ct.byref(h)), "mbh_create")
        self.h = h
        self.device = device

    def memory_in_use(self) -> int:
        v = ct.c_size_t()
        _check(_L.mbh_memory_in_use(self.h, ct.byref(v)), "mbh_memory_in_use")
        return v.value

    def close(self):
        if getattr(self, "h", None):
            _L.mbh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Data:
    def __init__(self, ctx: Context, h, n_chan, n_f, f0, df, t_obs, keep):
        self.ctx, self.h = ctx, h
        self.n_chan, self.n_f, self.f0, self.df, self.t_obs = n_chan, n_f, f0, df, t_obs
        self._keep = keep

    def inner_dd(self) -> float:
        v = ct.c_double()
        _check(_L.mbh_data_inner_dd(self.h, ct.byref(v)), "mbh_data_inner_dd")
        return v.value

    def close(self):
        if getattr(self, "h", None):
            _L.mbh_data_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Reference:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h
        info = self.info
        self.n_bins, self.n_chan = info["n_bins"], info["n_chan"]

    @property
    def info(self) -> dict:
        """mbh_ref_get_info (waits for a pending refresh)."""
        info = _RefInfo()
        _check(_L.mbh_ref_get_info(self.h, ct.byref(info)), "mbh_ref_get_info")
        return {k: getattr(info, k) for k, _ in _RefInfo._fields_}

    def refresh(self, data: "Data", theta: torch.Tensor, lnL: torch.Tensor, stream=None):
        """mbh_ref_refresh: rebuild in place from the walker with the largest finite lnL (device tensors)."""
        W = theta.shape[0]
        _check(_L.mbh_ref_refresh(self.ctx.h, data.h, self.h, _dev_ptr(theta, torch.float64, (W, NPARAM)),
                                  _dev_ptr(lnL, torch.float64, (W,)), W, _stream(stream)), "mbh_ref_refresh")

    def prepare_refresh(self, stream=None):
        """mbh_ref_refresh_prepare: allocate the update buffers now."""
        _check(_L.mbh_ref_refresh_prepare(self.h, _stream(stream)), "mbh_ref_refresh_prepare")

    def refresh_result(self) -> dict:
        """mbh_ref_refresh_result: status, picked walker and refreshes committed."""
        st, pick, gen = ct.c_int32(), ct.c_int64(), ct.c_int32()
        _check(_L.mbh_ref_refresh_result(self.h, ct.byref(st), ct.byref(pick), ct.byref(gen)),
               "mbh_ref_refresh_result")
        return dict(status=st.value, pick=pick.value, generation=gen.value)

    def export(self) -> dict:
        nb, nc = self.n_bins, self.n_chan
        edges = np.zeros(nb + 1)
        kb = np.zeros(nb + 1, dtype=np.int64)
        A0, A1 = np.zeros((nc, nb, 2)), np.zeros((nc, nb, 2))
        B0, B1 = np.zeros((nc, nb)), np.zeros((nc, nb))
        h0 = np.zeros((nc, nb + 1, 2))
        P = lambda a: a.ctypes.data_as(_dp)
        _check(_L.mbh_ref_export(self.h, P(edges), kb.ctypes.data_as(ct.POINTER(ct.c_int64)), P(A0), P(A1),
                                 P(B0), P(B1), P(h0)), "mbh_ref_export")
        return dict(edges=edges, kb=kb, A0=A0[..., 0] + 1j * A0[..., 1], A1=A1[..., 0] + 1j * A1[..., 1],
                    B0=B0, B1=B1, h0_edges=h0[..., 0] + 1j * h0[..., 1])

    def pm_info(self) -> dict:
        """mbh_ref_pm_info: modes with bins (mask) and mode pairs with overlapping bands."""
        m, n = ct.c_uint32(), ct.c_int32()
        _check(_L.mbh_ref_pm_info(self.h, ct.byref(m), ct.byref(n)), "mbh_ref_pm_info")
        return dict(modes=m.value, n_pairs=n.value)

    def pm_mode(self, mode_index: int) -> dict:
        """mbh_ref_pm_mode: one mode's band, edges, bins and sums (complex arrays)."""
        lo, hi, nb = ct.c_int64(), ct.c_int64(), ct.c_int32()
        z = ct.POINTER(ct.c_double)()
        zi = ct.POINTER(ct.c_int64)()
        _check(_L.mbh_ref_pm_mode(self.h, mode_index, ct.byref(lo), ct.byref(hi), ct.byref(nb), z, zi, z, z, z, z, z),
               "mbh_ref_pm_mode")
        n = nb.value
        edges, kb = np.zeros(n + 1), np.zeros(n + 1, dtype=np.int64)
        a0, a1, b0, b1, h0 = np.zeros((3, n, 2)), np.zeros((3, n, 2)), np.zeros((3, n)), np.zeros((3, n)), np.zeros((3, n + 1, 2))
        P = lambda a: a.ctypes.data_as(_dp)
        _check(_L.mbh_ref_pm_mode(self.h, mode_index, None, None, None, P(edges),
                                  kb.ctypes.data_as(ct.POINTER(ct.c_int64)), P(a0), P(a1), P(b0), P(b1), P(h0)),
               "mbh_ref_pm_mode")
        c = lambda x: x[..., 0] + 1j * x[..., 1]
        return dict(k_lo=lo.value, k_hi=hi.value, edges=edges, kb=kb, Ares0=c(a0), Ares1=c(a1), B0=b0, B1=b1,
                    h0_edges=c(h0))

    def pm_pair(self, pair: int) -> dict:
        """mbh_ref_pm_pair: one mode pair's merged grid and cross sums."""
        ma, mb, nm = ct.c_int32(), ct.c_int32(), ct.c_int32()
        _check(_L.mbh_ref_pm_pair(self.h, pair, ct.byref(ma), ct.byref(mb), ct.byref(nm), None, None, None, None,
                                  None, None), "mbh_ref_pm_pair")
        n = nm.value
        edges, kb = np.zeros(n + 1), np.zeros(n + 1, dtype=np.int64)
        ba, bb = np.zeros(n, dtype=np.int32), np.zeros(n, dtype=np.int32)
        c0, c1 = np.zeros((3, n, 2)), np.zeros((3, n, 2))
        P = lambda a: a.ctypes.data_as(_dp)
        I32 = lambda a: a.ctypes.data_as(ct.POINTER(ct.c_int32))
        _check(_L.mbh_ref_pm_pair(self.h, pair, None, None, None, P(edges), kb.ctypes.data_as(ct.POINTER(ct.c_int64)),
                                  I32(ba), I32(bb), P(c0), P(c1)), "mbh_ref_pm_pair")
        c = lambda x: x[..., 0] + 1j * x[..., 1]
        return dict(mode_a=ma.value, mode_b=mb.value, edges=edges, kb=kb, bin_a=ba, bin_b=bb, C0=c(c0), C1=c(c1))

    def close(self):
        if getattr(self, "h", None):
            _L.mbh_ref_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ entry points
def data_create(ctx: Context, d: torch.Tensor, psd: torch.Tensor, f0: float, df: float, t_obs: float,
                stream=None) -> Data:
    """mbh_data_create: d complex128 [C][N] and psd float64 [C][N] on the device."""
    if d.dtype != torch.complex128:
        raise ValueError("d must be complex128")
    d = d.contiguous()
    dr = torch.view_as_real(d)
    C, N = d.shape
    h = ct.c_void_p()
    _check(_L.mbh_data_create(ctx.h, C, N, f0, df, t_obs, _dev_ptr(dr, torch.float64, (C, N, 2)),
                              _dev_ptr(psd, torch.float64, (C, N)), _stream(stream), ct.byref(h)),
           "mbh_data_create")
    return Data(ctx, h, C, N, f0, df, t_obs, keep=(d, psd))


def tdi_to_aet_fd(ctx: Context, xyz: torch.Tensor, dt: float, t0: float, k_first: int, n_freq: int,
                  alpha: float = 0.0, stream=None, out: torch.Tensor | None = None) -> torch.Tensor:
    """mbh_tdi_to_aet_fd: xyz float64 [3][N] on the device -> complex128 [3][n_freq]
    (into `out` when given)."""
    N = xyz.shape[1]
    if out is None:
        out = torch.empty((3, n_freq), dtype=torch.complex128, device=xyz.device)
    if out.dtype != torch.complex128:
        raise TypeError("out must be complex128")
    _check(_L.mbh_tdi_to_aet_fd(ctx.h, N, dt, t0, _dev_ptr(xyz, torch.float64, (3, N)), alpha, k_first, n_freq,
                                _dev_ptr(torch.view_as_real(out), torch.float64, (3, n_freq, 2)), _stream(stream)),
           "mbh_tdi_to_aet_fd")
    return out


def data_create_tdi(ctx: Context, xyz: torch.Tensor, dt: float, t0: float, k_first: int, n_freq: int,
                    psd: torch.Tensor, t_obs: float, alpha: float = 0.0, stream=None) -> Data:
    """mbh_data_create_tdi: data on f_k = k / (N dt), k = k_first.., from X, Y, Z series."""
    N = xyz.shape[1]
    h = ct.c_void_p()
    _check(_L.mbh_data_create_tdi(ctx.h, N, dt, t0, _dev_ptr(xyz, torch.float64, (3, N)), alpha, k_first, n_freq,
                                  _dev_ptr(psd, torch.float64, (3, n_freq)), t_obs, _stream(stream), ct.byref(h)),
           "mbh_data_create_tdi")
    T = N * dt
    return Data(ctx, h, 3, n_freq, k_first / T, 1.0 / T, t_obs, keep=(psd,))


def template_full(ctx: Context, data: Data, model: int, modes: int, theta, stream=None) -> torch.Tensor:
    """mbh_template_full: complex128 [C][N] template on the data grid."""
    th = _host_theta(theta)
    out = torch.empty((data.n_chan, data.n_f), dtype=torch.complex128, device=f"cuda:{ctx.device}")
    _check(_L.mbh_template_full(ctx.h, data.h, model, modes, th.ctypes.data_as(_dp),
                                torch.view_as_real(out).data_ptr(), _stream(stream)), "mbh_template_full")
    return out


def build_reference_coeffs(ctx: Context, data: Data, model: int, modes: int, theta0, n_bins: int,
                           stream=None) -> Reference:
    th = _host_theta(theta0)
    h = ct.c_void_p()
    _check(_L.mbh_build_reference_coeffs(ctx.h, data.h, model, modes, th.ctypes.data_as(_dp), n_bins,
                                         _stream(stream), ct.byref(h)), "mbh_build_reference_coeffs")
    return Reference(ctx, h)


def build_reference_coeffs_pm(ctx: Context, data: Data, model: int, modes: int, theta0, n_bins_mode,
                              stream=None) -> Reference:
    """mbh_build_reference_coeffs_pm: per-mode relative binning (n_bins_mode: 6 bin counts)."""
    th = _host_theta(theta0)
    nb = (ct.c_int32 * 6)(*[int(x) for x in n_bins_mode])
    h = ct.c_void_p()
    _check(_L.mbh_build_reference_coeffs_pm(ctx.h, data.h, model, modes, th.ctypes.data_as(_dp), nb,
                                            _stream(stream), ct.byref(h)), "mbh_build_reference_coeffs_pm")
    return Reference(ctx, h)


def loglike_heterodyned(ctx: Context, ref: Reference, theta: torch.Tensor, prec: int = FP64,
                        lnL: torch.Tensor | None = None, dh_hh: torch.Tensor | None = None, stream=None):
    W = theta.shape[0]
    tp = _dev_ptr(theta, torch.float64, (W, NPARAM))
    if lnL is None:
        lnL = torch.empty(W, dtype=torch.float64, device=theta.device)
    dp = _dev_ptr(dh_hh, torch.float64, (W, 2)) if dh_hh is not None else None
    _check(_L.mbh_loglike_heterodyned(ctx.h, ref.h, tp, W, prec, _dev_ptr(lnL, torch.float64, (W,)), dp,
                                      _stream(stream)), "mbh_loglike_heterodyned")
    return lnL


def loglike_heterodyned_noalloc(ctx: Context, ref: Reference, theta: torch.Tensor, lnL: torch.Tensor,
                                prec: int = FP64, dh_hh: torch.Tensor | None = None, stream=None):
    """mbh_loglike_heterodyned_noalloc: outputs are the caller's (no allocation
    here or in the library); calls on one GPU must not overlap."""
    W = theta.shape[0]
    tp = _dev_ptr(theta, torch.float64, (W, NPARAM))
    dp = _dev_ptr(dh_hh, torch.float64, (W, 2)) if dh_hh is not None else None
    _check(_L.mbh_loglike_heterodyned_noalloc(ctx.h, ref.h, tp, W, prec, _dev_ptr(lnL, torch.float64, (W,)), dp,
                                              _stream(stream)), "mbh_loglike_heterodyned_noalloc")
    return lnL


def loglike_full(ctx: Context, data: Data, model: int, modes: int, theta: torch.Tensor, prec: int = FP64,
                 lnL: torch.Tensor | None = None, dh_hh: torch.Tensor | None = None, stream=None):
    W = theta.shape[0]
    tp = _dev_ptr(theta, torch.float64, (W, NPARAM))
    if lnL is None:
        lnL = torch.empty(W, dtype=torch.float64, device=theta.device)
    dp = _dev_ptr(dh_hh, torch.float64, (W, 2)) if dh_hh is not None else None
    _check(_L.mbh_loglike_full(ctx.h, data.h, model, modes, tp, W, prec, _dev_ptr(lnL, torch.float64, (W,)), dp,
                               _stream(stream)), "mbh_loglike_full")
    return lnL


def lanes_for(ctx: Context, n_bins: int, n_modes: int, prec: int) -> int:
    v = ct.c_int()
    _check(_L.mbh_lanes_for(ctx.h, n_bins, n_modes, prec, ct.byref(v)), "mbh_lanes_for")
    return v.value


def set_lanes(ctx: Context, n_bins: int, n_modes: int, prec: int, lanes: int):
    _check(_L.mbh_set_lanes(ctx.h, n_bins, n_modes, prec, lanes), "mbh_set_lanes")


def set_mixed_tolerance(ctx: Context, tol: float):
    """Estimated-error tolerance of the mixed path (0: all FP64, inf: none)."""
    _check(_L.mbh_set_mixed_tolerance(ctx.h, float(tol)), "mbh_set_mixed_tolerance")


def mixed_tolerance(ctx: Context) -> float:
    v = ct.c_double()
    _check(_L.mbh_get_mixed_tolerance(ctx.h, ct.byref(v)), "mbh_get_mixed_tolerance")
    return v.value


def autotune_heterodyned(ctx: Context, ref: Reference, walkers, prec: int) -> int:
    """Time every mapping on ``walkers`` (a [W, 11] float64 CUDA tensor of
    representative walkers) or, if ``walkers`` is an int W, on W copies of a
    fixed parameter point; records and returns the fastest (0 = flattened)."""
    v = ct.c_int()
    if isinstance(walkers, int):
        ptr, W = None, walkers
    else:
        W = walkers.shape[0]
        ptr = _dev_ptr(walkers, torch.float64, (W, NPARAM))
    _check(_L.mbh_autotune_heterodyned(ctx.h, ref.h, ptr, W, prec, ct.byref(v)), "mbh_autotune_heterodyned")
    return v.value


def set_full_shape(ctx: Context, higher_modes: bool, kf: int, wpb_cap: int):
    """Full-grid tile: kf frequencies per thread, at most wpb_cap walkers per workgroup."""
    _check(_L.mbh_set_full_shape(ctx.h, int(bool(higher_modes)), kf, wpb_cap), "mbh_set_full_shape")


def full_shape(ctx: Context, higher_modes: bool) -> tuple[int, int]:
    kf, cap = ct.c_int(), ct.c_int()
    _check(_L.mbh_full_shape(ctx.h, int(bool(higher_modes)), ct.byref(kf), ct.byref(cap)), "mbh_full_shape")
    return kf.value, cap.value


def autotune_full(ctx: Context, data: Data, model: int, modes: int, theta: torch.Tensor) -> tuple[int, int]:
    """Time every full-grid tile on the walkers ``theta`` ([W, 11] float64,
    CUDA); records and returns the fastest (frequencies per thread, walkers
    per workgroup at most)."""
    W = theta.shape[0]
    kf, cap = ct.c_int(), ct.c_int()
    _check(_L.mbh_autotune_full(ctx.h, data.h, model, modes, _dev_ptr(theta, torch.float64, (W, NPARAM)), W,
                                ct.byref(kf), ct.byref(cap)), "mbh_autotune_full")
    return kf.value, cap.value


def autotune_save(ctx: Context, path: str):
    _check(_L.mbh_autotune_save(ctx.h, path.encode()), "mbh_autotune_save")


def autotune_load(ctx: Context, path: str):
    _check(_L.mbh_autotune_load(ctx.h, path.encode()), "mbh_autotune_load")


class Batch:
    """mbh_batch_*: one graph-captured launch over many items."""

    def __init__(self, ctx: Context, refs, thetas, lnLs, dh_hhs=None, prec: int = FP64, precs=None):
        """precs: one precision per item (mbh_batch_create_prec); else `prec` for every item."""
        n = len(refs)
        self.ctx = ctx
        arr = lambda xs: (ct.c_void_p * n)(*xs)
        Ws = (ct.c_int64 * n)(*[t.shape[0] for t in thetas])
        tp = arr([_dev_ptr(t, torch.float64, (t.shape[0], NPARAM)) for t in thetas])
        lp = arr([_dev_ptr(l, torch.float64, (t.shape[0],)) for l, t in zip(lnLs, thetas)])
        dp = None
        if dh_hhs is not None:
            dp = arr([_dev_ptr(x, torch.float64, (t.shape[0], 2)) if x is not None else None
                      for x, t in zip(dh_hhs, thetas)])
        h = ct.c_void_p()
        if precs is None:
            _check(_L.mbh_batch_create(ctx.h, n, arr([r.h for r in refs]), tp, Ws, lp, dp, prec, ct.byref(h)),
                   "mbh_batch_create")
        else:
            if len(precs) != n:
                raise ValueError("one precision per item")
            pv = (ct.c_int32 * n)(*precs)
            _check(_L.mbh_batch_create_prec(ctx.h, n, arr([r.h for r in refs]), tp, Ws, lp, dp, pv, ct.byref(h)),
                   "mbh_batch_create_prec")
        self.h = h
        self._keep = (refs, thetas, lnLs, dh_hhs)

    def launch(self, stream=None):
        _check(_L.mbh_batch_launch(self.h, _stream(stream)), "mbh_batch_launch")

    def launch_direct(self, stream=None):
        """The same work as launch(), as stream launches instead of a graph replay."""
        _check(_L.mbh_batch_launch_direct(self.h, _stream(stream)), "mbh_batch_launch_direct")

    def launch_stage(self, stage: int, stream=None):
        """STAGE_SETUP, STAGE_MAIN or STAGE_FINISH alone (for measurement)."""
        _check(_L.mbh_batch_launch_stage(self.h, stage, _stream(stream)), "mbh_batch_launch_stage")

    def fp64_segments(self) -> int:
        """Walker segments the mixed path computed in FP64 so far."""
        v = ct.c_uint64()
        _check(_L.mbh_batch_fp64_segments(self.h, ct.byref(v)), "mbh_batch_fp64_segments")
        return v.value

    def close(self):
        if getattr(self, "h", None):
            _L.mbh_batch_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """mbh_server_*: continuous-batching request server over resident references."""

    def __init__(self, ctx: Context, refs, max_inflight=2, max_batch_walkers=65536, hbm_budget_bytes=1 << 30,
                 prec: int = MIXED):
        cfg = ServerConfig(max_inflight, max_batch_walkers, hbm_budget_bytes, prec)
        n = len(refs)
        h = ct.c_void_p()
        _check(_L.mbh_server_create(ctx.h, n, (ct.c_void_p * n)(*[r.h for r in refs]), ct.byref(cfg),
                                    ct.byref(h)), "mbh_server_create")
        self.h, self.ctx, self._refs = h, ctx, refs
        self._W = {}  # walkers of each request not yet waited for

    def submit(self, ref_index: int, theta: np.ndarray) -> int:
        th = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1, NPARAM)
        rid = ct.c_uint64()
        _check(_L.mbh_server_submit(self.h, ref_index, th.ctypes.data_as(_dp), th.shape[0], ct.byref(rid)),
               "mbh_server_submit")
        self._W[rid.value] = th.shape[0]
        return rid.value

    def refresh(self, ref_index: int, data: "Data", theta: np.ndarray, lnL: np.ndarray) -> int:
        """mbh_server_refresh: queue a reference update (host population); wait() on its id returns no results."""
        th = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1, NPARAM)
        lv = np.ascontiguousarray(lnL, dtype=np.float64).reshape(-1)
        if lv.shape[0] != th.shape[0]:
            raise ValueError("theta and lnL sizes differ")
        rid = ct.c_uint64()
        _check(_L.mbh_server_refresh(self.h, ref_index, data.h, th.ctypes.data_as(_dp), lv.ctypes.data_as(_dp),
                                     th.shape[0], ct.byref(rid)), "mbh_server_refresh")
        self._W[rid.value] = 0
        return rid.value

    def wait(self, rid: int, W: int | None = None, timeout_ms: int = -1, want_dh_hh: bool = False):
        """mbh_server_wait; the buffers are sized from the request's own walker
        count (W, if given, must equal it)."""
        n = self._W.get(rid)
        if n is None:
            raise KeyError(f"unknown request {rid}")
        if W is not None and W != n:
            raise ValueError(f"request {rid} holds {n} walkers, not {W}")
        lnL = np.zeros(n)
        dh = np.zeros((n, 2)) if want_dh_hh else None
        lat = ct.c_double()
        st = _L.mbh_server_wait(self.h, rid, timeout_ms, lnL.ctypes.data_as(_dp),
                                dh.ctypes.data_as(_dp) if dh is not None else None, n, ct.byref(lat))
        if st == MBH_EAGAIN:
            return None
        if st in (MBH_OK, MBH_EDEVICE, MBH_ENOTFOUND):  # the library has forgotten the request
            del self._W[rid]
        _check(st, "mbh_server_wait")
        return (lnL, dh, lat.value) if want_dh_hh else (lnL, lat.value)

    def replay(self, t_arrival, ref_index, W, theta_row, theta: np.ndarray, want_lnL: bool = False):
        """mbh_server_replay: submit a request trace at its arrival times and
        collect it, all in native threads.  Returns a dict with per-request
        latency_s and submit_lag_s, wall_s and (want_lnL) the results in
        request order."""
        n = len(t_arrival)
        specs = (RequestSpec * n)()
        for i in range(n):
            specs[i] = RequestSpec(float(t_arrival[i]), int(ref_index[i]), 0, int(W[i]), int(theta_row[i]))
        th = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1, NPARAM)
        lat, lag = np.zeros(n), np.zeros(n)
        lnL = np.zeros(int(np.sum(W))) if want_lnL else None
        wall = ct.c_double()
        _check(_L.mbh_server_replay(self.h, specs, n, th.ctypes.data_as(_dp), th.shape[0], lat.ctypes.data_as(_dp),
                                    lag.ctypes.data_as(_dp), lnL.ctypes.data_as(_dp) if lnL is not None else None,
                                    ct.byref(wall)), "mbh_server_replay")
        out = dict(latency_s=lat, submit_lag_s=lag, wall_s=wall.value)
        if want_lnL:
            out["lnL"] = lnL
        return out

    def stats(self) -> dict:
        s = ServerStats()
        _check(_L.mbh_server_get_stats(self.h, ct.byref(s)), "mbh_server_get_stats")
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            _L.mbh_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


STOP_MAX_ITER, STOP_SNR, STOP_CONVERGED = 0, 1, 2


class Sampler:
    """mbh_sampler_*: tempered ensemble sampler on the device (Sec. 3)."""

    def __init__(self, ctx: Context, betas, walkers_per_temp: int, prior_lo, prior_hi, seed: int = 1,
                 stretch_a: float = 2.0, p_sky=(0.04, 0.03, 0.08), prec: int = FP64, mixed_rungs: int = 0):
        betas = np.ascontiguousarray(betas, dtype=np.float64)
        lo = np.ascontiguousarray(prior_lo, dtype=np.float64)
        hi = np.ascontiguousarray(prior_hi, dtype=np.float64)
        cfg = SamplerConfig(betas.size, walkers_per_temp, stretch_a, p_sky[0], p_sky[1], p_sky[2], seed, prec,
                            mixed_rungs)
        h = ct.c_void_p()
        _check(_L.mbh_sampler_create(ctx.h, ct.byref(cfg), betas.ctypes.data_as(_dp), lo.ctypes.data_as(_dp),
                                     hi.ctypes.data_as(_dp), ct.byref(h)), "mbh_sampler_create")
        self.h, self.ctx = h, ctx
        self.K, self.W = betas.size, walkers_per_temp

    @staticmethod
    def likelihood(ref: "Reference | None" = None, data: "Data | None" = None, modes: int = MODE_22) -> Likelihood:
        return Likelihood(ref.h if ref is not None else None, data.h if data is not None else None, modes)

    def set_walkers(self, x, like: Likelihood | None = None, lnL=None, stream=None):
        """Walkers in sampling coordinates and their lnL (given, or evaluated under `like`)."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.K * self.W, NPARAM)
        lv = None if lnL is None else np.ascontiguousarray(lnL, dtype=np.float64).reshape(self.K * self.W)
        _check(_L.mbh_sampler_set_walkers(self.h, x.ctypes.data_as(_dp), lv.ctypes.data_as(_dp) if lv is not None
                                          else None, ct.byref(like) if like is not None else None, _stream(stream)),
               "mbh_sampler_set_walkers")

    def step(self, like: Likelihood, n_iter: int = 1, stream=None):
        _check(_L.mbh_sampler_step(self.h, ct.byref(like), n_iter, _stream(stream)), "mbh_sampler_step")

    def step_served(self, server: "Server", ref_index: int, n_iter: int = 1, stream=None) -> np.ndarray:
        """mbh_sampler_step_served: iterations whose likelihood calls are requests
        to `server`; returns each request's latency in seconds ([2 n_iter])."""
        lat = np.zeros(2 * n_iter)
        _check(_L.mbh_sampler_step_served(self.h, server.h, ref_index, n_iter, _stream(stream),
                                          lat.ctypes.data_as(_dp)), "mbh_sampler_step_served")
        return lat

    def propose(self, half: int, stream=None):
        _check(_L.mbh_sampler_propose(self.h, half, _stream(stream)), "mbh_sampler_propose")

    def proposals(self):
        n = self.K * self.W // 2
        x, th, kind = np.zeros((n, NPARAM)), np.zeros((n, NPARAM)), np.zeros(n, dtype=np.int32)
        _check(_L.mbh_sampler_proposals(self.h, x.ctypes.data_as(_dp), th.ctypes.data_as(_dp),
                                        kind.ctypes.data_as(ct.POINTER(ct.c_int32))), "mbh_sampler_proposals")
        return x, th, kind

    def accept(self, half: int, lnL: torch.Tensor, dh_hh: torch.Tensor | None = None, stream=None):
        n = self.K * self.W // 2
        _check(_L.mbh_sampler_accept(self.h, half, _dev_ptr(lnL, torch.float64, (n,)),
                                     _dev_ptr(dh_hh, torch.float64, (n, 2)) if dh_hh is not None else None,
                                     _stream(stream)), "mbh_sampler_accept")

    def swap(self, stream=None):
        _check(_L.mbh_sampler_swap(self.h, _stream(stream)), "mbh_sampler_swap")

    def get(self):
        n = self.K * self.W
        x, l, dh = np.zeros((n, NPARAM)), np.zeros(n), np.zeros((n, 2))
        it = ct.c_int64()
        _check(_L.mbh_sampler_get(self.h, x.ctypes.data_as(_dp), l.ctypes.data_as(_dp), dh.ctypes.data_as(_dp),
                                  ct.byref(it)), "mbh_sampler_get")
        return dict(x=x, lnL=l, dh_hh=dh, iteration=it.value)

    def stats(self):
        acc, prop = np.zeros(self.K * 4, dtype=np.uint64), np.zeros(self.K * 4, dtype=np.uint64)
        sw = np.zeros(max(self.K - 1, 1), dtype=np.uint64)
        P = lambda a: a.ctypes.data_as(ct.POINTER(ct.c_uint64))
        _check(_L.mbh_sampler_stats(self.h, P(acc), P(prop), P(sw)), "mbh_sampler_stats")
        return dict(accepted=acc.reshape(self.K, 4), proposed=prop.reshape(self.K, 4), swaps=sw[: self.K - 1])

    def run(self, like: Likelihood, check_every=150, snr_stop=0.0, lnl_tol=1.0, lnl_checks=0, refresh_every=0,
            refresh_data: "Data | None" = None, max_iter=10000, stream=None) -> dict:
        stop = SamplerStop(check_every, snr_stop, lnl_tol, lnl_checks, refresh_every,
                           refresh_data.h if refresh_data is not None else None, max_iter)
        rep = SamplerReport()
        _check(_L.mbh_sampler_run(self.h, ct.byref(like), ct.byref(stop), _stream(stream), ct.byref(rep)),
               "mbh_sampler_run")
        return {k: getattr(rep, k) for k, _ in SamplerReport._fields_}

    def close(self):
        if getattr(self, "h", None):
            _L.mbh_sampler_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
