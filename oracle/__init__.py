"""Plain FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

ctypes wrapper around ``liboracle.so`` (built from ``mbh_oracle.c`` by
:func:`build`).  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the GPU library never does.

Parity status of each oracle function is listed in the module docstrings of
``tests/test_oracle_*.py``; every function here is pinned by at least one of
them (closed forms, invariants, brute force, a time-domain response check or
the paper's printed numbers).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mbh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODEL_IMR = 0
MODEL_TF2 = 1
MODE_22, MODE_33, MODE_44, MODE_21, MODE_32, MODE_43 = (1 << i for i in range(6))
ALL_MODES = 0x3F
NPARAM = 11
OK, EINVAL, EBAND = 0, -1, -3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
               "-shared", "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ct.CDLL(_LIB)
        dp = ct.POINTER(ct.c_double)
        lp = ct.POINTER(ct.c_int64)
        ip = ct.POINTER(ct.c_int)
        i64, u32, i32, d = ct.c_int64, ct.c_uint32, ct.c_int, ct.c_double
        L.oracle_sylm.argtypes = [i32, i32, d, d, dp, dp]
        L.oracle_mode.argtypes = [dp, i32, i32, i32, dp, dp, dp, dp, ip]
        L.oracle_fmax.argtypes = [dp]
        L.oracle_fmax.restype = d
        L.oracle_orbit.argtypes = [d, dp]
        L.oracle_link.argtypes = [i32, i32, d, dp, d, d, d, dp, dp, dp]
        L.oracle_tdi.argtypes = [d, d, d, d, d, dp, dp, dp]
        L.oracle_template.argtypes = [i32, u32, dp, i64, dp, d, dp]
        L.oracle_inner.argtypes = [i32, i64, dp, dp, dp, d]
        L.oracle_inner.restype = d
        L.oracle_loglike_full.argtypes = [i32, u32, i64, dp, i32, i64, d, d, d, dp, dp, dp, dp, dp]
        L.oracle_loglike_of.argtypes = [i32, i64, dp, dp, dp, d, dp, dp]
        L.oracle_loglike_of.restype = d
        L.oracle_reference.argtypes = [i32, u32, dp, i32, i64, d, d, d, dp, dp, i32, lp, lp, dp,
                                       lp, dp, dp, dp, dp, dp, dp, dp]
        L.oracle_bin_sums.argtypes = [i32, i64, d, d, dp, dp, dp, i32, dp, i64, i64, lp, dp, dp,
                                      dp, dp, dp]
        L.oracle_het_core.argtypes = [i32, i32, dp, dp, dp, dp, dp, d, dp, dp, dp, dp, dp]
        L.oracle_het_core_residual.argtypes = [i32, i32, dp, dp, dp, dp, dp, d, dp, dp, dp]
        L.oracle_loglike_het.argtypes = [i32, u32, i64, dp, i32, i32, dp, dp, dp, dp, dp, d, dp,
                                         d, dp, dp, dp]
        L.oracle_max_threads.restype = i32
        L.oracle_set_threads.argtypes = [i32]
        L.oracle_set_threads.restype = None
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def n_chan(model: int) -> int:
    return 1 if model == MODEL_TF2 else 3


def max_threads() -> int:
    return lib().oracle_max_threads()


def set_threads(n: int) -> None:
    """Threads of the walker loops (for timing; results do not depend on it)."""
    lib().oracle_set_threads(int(n))


def sylm(l: int, m: int, theta: float, phi: float) -> complex:
    re, im = ct.c_double(), ct.c_double()
    lib().oracle_sylm(l, m, theta, phi, ct.byref(re), ct.byref(im))
    return complex(re.value, im.value)


def mode(theta, l: int, m: int, f):
    """Amplitude, phase (without the t_ref shift), t_lm(f) and support flag."""
    th, f = _f64(theta), _f64(f)
    n = f.size
    amp, ph, tf = np.zeros(n), np.zeros(n), np.zeros(n)
    on = np.zeros(n, dtype=np.int32)
    rc = lib().oracle_mode(_p(th), l, m, n, _p(f), _p(amp), _p(ph), _p(tf),
                           on.ctypes.data_as(ct.POINTER(ct.c_int)))
    if rc != OK:
        raise ValueError("invalid parameters or mode")
    return amp, ph, tf, on.astype(bool)


def fmax(theta) -> float:
    return lib().oracle_fmax(_p(_f64(theta)))


def orbit(t: float) -> np.ndarray:
    p = np.zeros(9)
    lib().oracle_orbit(t, _p(p))
    return p.reshape(3, 3)


def link(i: int, j: int, f: float, p, lam, beta, psi, Kp: complex, Kc: complex) -> complex:
    p = _f64(p).reshape(9)
    kp = np.array([Kp.real, Kp.imag])
    kc = np.array([Kc.real, Kc.imag])
    y = np.zeros(2)
    lib().oracle_link(i, j, f, _p(p), lam, beta, psi, _p(kp), _p(kc), _p(y))
    return complex(y[0], y[1])


def tdi(f: float, t: float, lam, beta, psi, Kp: complex, Kc: complex) -> np.ndarray:
    """[X, Y, Z, A, E, T] transfer for one polarisation content."""
    kp = np.array([Kp.real, Kp.imag])
    kc = np.array([Kc.real, Kc.imag])
    out = np.zeros(12)
    lib().oracle_tdi(f, t, lam, beta, psi, _p(kp), _p(kc), _p(out))
    return out[0::2] + 1j * out[1::2]


def template(model: int, modes: int, theta, f, t_obs: float) -> np.ndarray:
    """Complex template [n_chan][n] on the frequencies f."""
    th, f = _f64(theta), _f64(f)
    nc = n_chan(model)
    h = np.zeros((nc, f.size, 2))
    rc = lib().oracle_template(model, modes, _p(th), f.size, _p(f), t_obs, _p(h))
    if rc != OK:
        raise ValueError("invalid parameters")
    return h[..., 0] + 1j * h[..., 1]


def _cplx_buf(z):
    z = np.asarray(z, dtype=np.complex128)
    out = np.empty(z.shape + (2,))
    out[..., 0] = z.real
    out[..., 1] = z.imag
    return out


def inner(a, b, psd, df: float) -> float:
    a, b, psd = np.atleast_2d(a), np.atleast_2d(b), _f64(np.atleast_2d(psd))
    A, B = _cplx_buf(a), _cplx_buf(b)
    return lib().oracle_inner(a.shape[0], a.shape[1], _p(A), _p(B), _p(psd), df)


def loglike_of(d, h, psd, df: float):
    """-1/2 <d-h|d-h>, <d|h>, <h|h> for explicit arrays."""
    d, h, psd = np.atleast_2d(d), np.atleast_2d(h), _f64(np.atleast_2d(psd))
    D, H = _cplx_buf(d), _cplx_buf(h)
    dh, hh = ct.c_double(), ct.c_double()
    v = lib().oracle_loglike_of(d.shape[0], d.shape[1], _p(D), _p(H), _p(psd), df,
                                ct.byref(dh), ct.byref(hh))
    return v, dh.value, hh.value


class Data:
    """Frequency-domain data on the uniform grid f_k = f0 + k df."""

    def __init__(self, d, psd, f0: float, df: float, t_obs: float):
        self.d = np.atleast_2d(np.asarray(d, dtype=np.complex128))
        self.psd = _f64(np.atleast_2d(psd))
        self.n_chan, self.n_f = self.d.shape
        self.f0, self.df, self.t_obs = float(f0), float(df), float(t_obs)
        self._dbuf = _cplx_buf(self.d)

    @property
    def freqs(self):
        return self.f0 + np.arange(self.n_f) * self.df


def loglike_full(model: int, modes: int, theta, data: Data):
    th = _f64(np.atleast_2d(theta))
    W = th.shape[0]
    lnL, dh, hh = np.zeros(W), np.zeros(W), np.zeros(W)
    rc = lib().oracle_loglike_full(model, modes, W, _p(th), data.n_chan, data.n_f, data.f0,
                                   data.df, data.t_obs, _p(data._dbuf), _p(data.psd),
                                   _p(lnL), _p(dh), _p(hh))
    if rc != OK:
        raise ValueError("oracle_loglike_full failed")
    return lnL, dh, hh


class Reference:
    """Heterodyne reference: band, edges, bin assignment and A0, A1, B0, B1 (+B2)."""

    def __init__(self, model: int, modes: int, theta0, data: Data, n_bins: int):
        self.model, self.modes, self.n_bins = model, modes, int(n_bins)
        self.theta0 = _f64(theta0)
        self.data = data
        nc, nb = data.n_chan, self.n_bins
        self.edges = np.zeros(nb + 1)
        self.kb = np.zeros(nb + 1, dtype=np.int64)
        self.A0 = np.zeros((nc, nb, 2))
        self.A1 = np.zeros((nc, nb, 2))
        self.B0 = np.zeros((nc, nb))
        self.B1 = np.zeros((nc, nb))
        self.B2 = np.zeros((nc, nb))
        self.h0_edges = np.zeros((nc, nb + 1, 2))
        klo, khi, dd = ct.c_int64(), ct.c_int64(), ct.c_double()
        lp = ct.POINTER(ct.c_int64)
        rc = lib().oracle_reference(model, modes, _p(self.theta0), nc, data.n_f, data.f0,
                                    data.df, data.t_obs, _p(data._dbuf), _p(data.psd), nb,
                                    ct.byref(klo), ct.byref(khi), _p(self.edges),
                                    self.kb.ctypes.data_as(lp), _p(self.A0), _p(self.A1),
                                    _p(self.B0), _p(self.B1), _p(self.B2), ct.byref(dd),
                                    _p(self.h0_edges))
        self.status = rc
        if rc == EINVAL:
            raise ValueError("invalid reference parameters")
        self.k_lo, self.k_hi, self.dd = klo.value, khi.value, dd.value

    @classmethod
    def from_edges(cls, data: Data, h0_grid, edges, lo: int, hi: int, h0_edges):
        """Reference with caller-chosen edges and an explicit h0 on the grid
        (used to test the binning identities)."""
        self = cls.__new__(cls)
        self.model, self.modes, self.data = None, None, data
        edges = _f64(edges)
        self.n_bins = edges.size - 1
        self.edges = edges
        nc, nb = data.n_chan, self.n_bins
        self.kb = np.zeros(nb + 1, dtype=np.int64)
        self.A0, self.A1 = np.zeros((nc, nb, 2)), np.zeros((nc, nb, 2))
        self.B0, self.B1, self.B2 = np.zeros((nc, nb)), np.zeros((nc, nb)), np.zeros((nc, nb))
        H0 = _cplx_buf(np.atleast_2d(h0_grid))
        lib().oracle_bin_sums(nc, data.n_f, data.f0, data.df, _p(data._dbuf), _p(data.psd),
                              _p(H0), nb, _p(edges), lo, hi,
                              self.kb.ctypes.data_as(ct.POINTER(ct.c_int64)), _p(self.A0),
                              _p(self.A1), _p(self.B0), _p(self.B1), _p(self.B2))
        self.h0_edges = _cplx_buf(np.atleast_2d(h0_edges))
        self.dd = inner(data.d, data.d, data.psd, data.df)
        self.k_lo, self.k_hi, self.status = lo, hi, OK
        return self

    @property
    def A0c(self):
        return self.A0[..., 0] + 1j * self.A0[..., 1]

    @property
    def A1c(self):
        return self.A1[..., 0] + 1j * self.A1[..., 1]

    @property
    def h0c(self):
        return self.h0_edges[..., 0] + 1j * self.h0_edges[..., 1]

    def core(self, h_edges, residual: bool = False):
        """Binned likelihood for a given template at the edges [n_chan][n_bins+1]."""
        H = _cplx_buf(np.atleast_2d(h_edges))
        lnL, dh, hh = ct.c_double(), ct.c_double(), ct.c_double()
        if residual:
            lib().oracle_het_core_residual(self.data.n_chan, self.n_bins, _p(self.edges),
                                           _p(self.A0), _p(self.A1), _p(self.B0), _p(self.B1),
                                           self.dd, _p(self.h0_edges), _p(H), ct.byref(lnL))
            return lnL.value
        lib().oracle_het_core(self.data.n_chan, self.n_bins, _p(self.edges), _p(self.A0),
                              _p(self.A1), _p(self.B0), _p(self.B1), self.dd,
                              _p(self.h0_edges), _p(H), ct.byref(lnL), ct.byref(dh),
                              ct.byref(hh))
        return lnL.value, dh.value, hh.value

    def loglike(self, theta):
        th = _f64(np.atleast_2d(theta))
        W = th.shape[0]
        lnL, dh, hh = np.zeros(W), np.zeros(W), np.zeros(W)
        rc = lib().oracle_loglike_het(self.model, self.modes, W, _p(th), self.data.n_chan,
                                      self.n_bins, _p(self.edges), _p(self.A0), _p(self.A1),
                                      _p(self.B0), _p(self.B1), self.dd, _p(self.h0_edges),
                                      self.data.t_obs, _p(lnL), _p(dh), _p(hh))
        if rc != OK:
            raise ValueError("oracle_loglike_het failed")
        return lnL, dh, hh


def best_walker(lnL) -> int:
    """Walker that the reference update of Sec. 3.2 (the reference becomes the
    highest-likelihood point of the population) moves to: the largest finite
    lnL, the lowest index among equal values; -1 if no value is finite."""
    v = np.asarray(lnL, dtype=np.float64).ravel()
    ok = np.isfinite(v)
    if not ok.any():
        return -1
    return int(np.flatnonzero(ok & (v == v[ok].max()))[0])


def refresh_reference(ref: Reference, walkers, lnL):
    """Sec. 3.2 reference update: (status, picked walker, new Reference with
    the same model, modes and bin count built at that walker, or None).
    status is EINVAL when no lnL is finite or the walker lies outside the
    model domain, EBAND when its template is empty on the grid or zero at an
    edge; the caller then keeps the old reference."""
    pick = best_walker(lnL)
    if pick < 0:
        return EINVAL, -1, None
    try:
        new = Reference(ref.model, ref.modes, np.asarray(walkers)[pick], ref.data, ref.n_bins)
    except ValueError:
        return EINVAL, pick, None
    if new.status != OK:
        return new.status, pick, None
    return OK, pick, new
