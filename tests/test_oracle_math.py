"""Pins of the oracle's building blocks against closed forms, textbook results
and independent time-domain constructions (CPU only).

oracle function          pinned by
-----------------------  ----------------------------------------------------
sylm                     closed forms of -2Y_lm (l=2 all m, (3,+-3), (3,+-2),
                         (4,+-4), (4,+-3)); sum rule; orthonormality
inner                    0PN chirp <h|h> closed forms (power-law PSD and the
                         chirp-case PSD via 2F1), midpoint-rule bound
template (chirp)         stationary-phase time t(f) = t_c - (5/256) Mc (pi Mc f)^(-8/3)
mode (IMR-lite)          eq. (tf) by numerical differentiation; 1.5PN spin-orbit
                         time-to-coalescence; Newtonian quadrupole amplitude;
                         higher-mode amplitudes from Fourier transforms of
                         time-domain PN modes (Blanchet's leading-order H_lm);
                         C1 phase / C0 amplitude at the transition; f_ref = argmax f^2 A22
orbit                    centroid = guiding centre, arm length, 60 deg inclination
link                     time-domain single-link Doppler of a monochromatic plane wave
tdi                      time-domain first-generation Michelson X; A,E,T orthogonality
"""
import math

import numpy as np
import pytest
from scipy.special import hyp2f1

import oracle as O
from paper_2111_01064_amd import inputs as I

MSUN_S = 4.925490947641267e-6
C_SI = 299792458.0
L_S = 2.5e9 / C_SI
R_S = 1.495978707e11 / C_SI


# ----------------------------------------------------------------- harmonics
def _closed_forms(th, ph):
    c, s = math.cos(th), math.sin(th)
    ch, sh = math.cos(th / 2), math.sin(th / 2)
    e = lambda m: complex(math.cos(m * ph), math.sin(m * ph))
    return {
        (2, 2): math.sqrt(5 / (64 * math.pi)) * (1 + c) ** 2 * e(2),
        (2, 1): math.sqrt(5 / (16 * math.pi)) * s * (1 + c) * e(1),
        (2, 0): math.sqrt(15 / (32 * math.pi)) * s * s,
        (2, -1): math.sqrt(5 / (16 * math.pi)) * s * (1 - c) * e(-1),
        (2, -2): math.sqrt(5 / (64 * math.pi)) * (1 - c) ** 2 * e(-2),
        (3, 3): -math.sqrt(21 / (2 * math.pi)) * ch ** 5 * sh * e(3),
        (3, -3): math.sqrt(21 / (2 * math.pi)) * ch * sh ** 5 * e(-3),
        (3, 2): math.sqrt(7 / math.pi) / 2 * ch ** 4 * (3 * c - 2) * e(2),
        (3, -2): math.sqrt(7 / (4 * math.pi)) * (2 + 3 * c) * sh ** 4 * e(-2),
        (4, 4): 3 * math.sqrt(7 / math.pi) * ch ** 6 * sh ** 2 * e(4),
        (4, -4): 3 * math.sqrt(7 / math.pi) * ch ** 2 * sh ** 6 * e(-4),
        (4, 3): -3 * math.sqrt(7 / (2 * math.pi)) * ch ** 5 * (2 * c - 1) * sh * e(3),
        (4, -3): 3 * math.sqrt(7 / (2 * math.pi)) * ch * (1 + 2 * c) * sh ** 5 * e(-3),
    }


@pytest.mark.parametrize("th,ph", [(0.3, 0.1), (1.2245, 2.0), (2.5, -0.7), (math.pi / 2, 0.0)])
def test_sylm_closed_forms(th, ph):
    for (l, m), ref in _closed_forms(th, ph).items():
        assert abs(O.sylm(l, m, th, ph) - ref) < 1e-14, (l, m)


@pytest.mark.parametrize("l", [2, 3, 4])
def test_sylm_sum_rule_and_orthonormality(l):
    for th in (0.1, 0.9, 2.2, 3.0):
        s = sum(abs(O.sylm(l, m, th, 0.4)) ** 2 for m in range(-l, l + 1))
        assert abs(s - (2 * l + 1) / (4 * math.pi)) < 1e-13
    x, w = np.polynomial.legendre.leggauss(40)
    th = np.arccos(x)
    for m in range(-l, l + 1):
        norm = 2 * math.pi * sum(wi * abs(O.sylm(l, m, t, 0.0)) ** 2 for t, wi in zip(th, w))
        assert abs(norm - 1.0) < 1e-12
        for l2 in range(max(2, abs(m)), 5):
            if l2 == l:
                continue
            ov = 2 * math.pi * sum(wi * (O.sylm(l, m, t, 0.0) * np.conj(O.sylm(l2, m, t, 0.0))).real
                                   for t, wi in zip(th, w))
            assert abs(ov) < 1e-12


# ----------------------------------------------------------------- inner product
def _chirp_amp_sq_over_s_integral(amp, s0, f0, a, b):
    G = lambda x: 0.375 * x ** (8 / 3) * hyp2f1(1.0, 2.0 / 3.0, 5.0 / 3.0, -(x / f0) ** 4)
    return 4.0 * amp ** 2 / (s0 * f0 ** 4) * (G(b) - G(a))


def _g(f, amp, s0, f0):
    return 4.0 * amp ** 2 / (s0 * f0 ** 4) * f ** (5 / 3) / (1 + (f / f0) ** 4)


def test_inner_chirp_psd_closed_form():
    g = I.grid_chirp()
    f = g.freqs
    th = np.array([3e5, 2.5e-21, 1e4, 0.4] + [0.0] * 7)
    h = O.template(O.MODEL_TF2, 0, th, f, g.t_obs)
    psd = I.psd_chirp(f)
    num = O.inner(h, h, psd, g.df)
    ref = _chirp_amp_sq_over_s_integral(th[1], 1e-40, 3e-3, f[0] - g.df / 2, f[-1] + g.df / 2)
    # midpoint rule: |sum - integral| <= df^2/24 * int |g''|
    ff = np.linspace(f[0] - g.df / 2, f[-1] + g.df / 2, 400001)
    gg = _g(ff, th[1], 1e-40, 3e-3)
    g2 = np.gradient(np.gradient(gg, ff), ff)
    bound = g.df ** 2 / 24 * np.trapezoid(np.abs(g2), ff)
    assert abs(num - ref) <= 1.2 * bound + 1e-12 * ref
    assert bound < 1e-3 * ref


def test_inner_power_law_closed_form():
    g = I.grid_chirp()
    f = g.freqs
    th = np.array([3e5, 1.0e-21, 1e4, 0.4] + [0.0] * 7)
    h = O.template(O.MODEL_TF2, 0, th, f, g.t_obs)
    s0, fr = 1e-40, 3e-3
    psd = I.psd_powerlaw(f, s0, fr, -4.0)
    num = O.inner(h, h, psd, g.df)
    a, b = f[0] - g.df / 2, f[-1] + g.df / 2
    ref = 4 * th[1] ** 2 / (s0 * fr ** 4) * 0.375 * (b ** (8 / 3) - a ** (8 / 3))
    # g = C f^(5/3): g'' = C (10/9) f^(-1/3) > 0, bound = df^2/24 [g'(b) - g'(a)]
    C = 4 * th[1] ** 2 / (s0 * fr ** 4)
    bound = g.df ** 2 / 24 * C * (5 / 3) * (b ** (2 / 3) - a ** (2 / 3))
    assert abs(num - ref) <= bound * 1.01 + 1e-13 * ref
    # and <a|b> is linear and symmetric
    h2 = 0.3 * h * np.exp(0.7j)
    assert abs(O.inner(h, h2, psd, g.df) - O.inner(h2, h, psd, g.df)) < 1e-12 * num
    assert abs(O.inner(h, 2 * h2, psd, g.df) - 2 * O.inner(h, h2, psd, g.df)) < 1e-12 * num


def test_chirp_stationary_phase_time():
    """t(f) = (1/2pi) d arg h / df must be the Newtonian time to coalescence."""
    Mc, tc = 4e5, 1e4
    th = np.array([Mc, 1.0, tc, 1.1] + [0.0] * 7)
    Mcs = Mc * MSUN_S
    for f in (2e-4, 1e-3, 5e-3, 2e-2):
        eps = f * 1e-6
        hs = O.template(O.MODEL_TF2, 0, th, np.array([f - eps, f + eps]), 1.0)[0]
        dphi = np.angle(hs[1] / hs[0])
        t_num = dphi / (2 * math.pi * 2 * eps)
        t_ref = tc - 5.0 / 256.0 * Mcs * (math.pi * Mcs * f) ** (-8 / 3)
        assert abs(t_num - t_ref) < 1e-5 * abs(t_ref - tc) + 1e-6


# ----------------------------------------------------------------- IMR-lite waveform
THETA = np.array([2.0e6, 0.45, 0.6, -0.3, 10.0, 0.7, 1.1, 3.5, 0.29, 0.8, 2.0e7])


def _fsets(th):
    M = th[0] * MSUN_S
    f1 = 0.018 / M
    return M, f1


@pytest.mark.parametrize("lm", [(2, 2), (3, 3), (4, 4), (2, 1), (3, 2), (4, 3)])
def test_time_frequency_is_phase_derivative(lm):
    """eq. (tf): t_lm(f) = t_ref - (1/2pi) d phi_lm / df."""
    l, m = lm
    M, f1 = _fsets(THETA)
    fs = np.array([1e-5, 1e-4, 0.3 * f1, 0.7 * f1, 1.3 * f1, 2.5 * f1, 3.3 * f1, 6 * f1]) * m / 2
    for f in fs:
        eps = f * 1e-6
        _, ph, _, _ = O.mode(THETA, l, m, np.array([f - eps, f + eps]))
        _, _, tf, _ = O.mode(THETA, l, m, np.array([f]))
        dphi = (ph[1] - ph[0]) / (2 * eps)
        t_num = THETA[10] - dphi / (2 * math.pi)
        assert abs(t_num - tf[0]) < 2e-7 * max(1.0, abs(THETA[10] - tf[0])), (f, t_num, tf[0])


def test_spin_orbit_time_to_coalescence():
    """Inspiral t(f) differences equal the textbook 1.5PN spin-orbit
    time-to-coalescence tau(v) = 5M/(256 eta v^8)[1 + (743/252 + 11 eta/3) v^2 - (8/5)(4 pi - beta) v^3]."""
    th = THETA
    M = th[0] * MSUN_S
    q = th[1]
    m1, m2 = 1 / (1 + q), q / (1 + q)
    eta = m1 * m2
    beta = ((113 * m1 ** 2 + 75 * eta) * th[2] + (113 * m2 ** 2 + 75 * eta) * th[3]) / 12

    def tau(f):
        v = (math.pi * M * f) ** (1 / 3)
        return 5 * M / (256 * eta * v ** 8) * (1 + (743 / 252 + 11 * eta / 3) * v ** 2
                                               - 1.6 * (4 * math.pi - beta) * v ** 3)

    fa, fb = 2e-5, 3e-4
    _, _, tf, _ = O.mode(th, 2, 2, np.array([fa, fb]))
    assert abs((tf[1] - tf[0]) - (tau(fa) - tau(fb))) < 1e-10 * abs(tau(fa) - tau(fb))


def test_newtonian_quadrupole_amplitude():
    """Face-on (2,2): K+ A22 = sqrt(5/24) pi^(-2/3) Mc^(5/6) f^(-7/6) / D_L."""
    th = THETA.copy()
    th[6] = 0.0
    M = th[0] * MSUN_S
    q = th[1]
    eta = q / (1 + q) ** 2
    Mc = eta ** 0.6 * M
    D = th[4] * 3.0856775814913673e25 / C_SI
    Kp = 0.5 * (O.sylm(2, 2, 0.0, 0.0) + np.conj(O.sylm(2, -2, 0.0, 0.0)))
    for f in (1e-5, 1e-4, 5e-4):
        a, _, _, _ = O.mode(th, 2, 2, np.array([f]))
        ref = math.sqrt(5 / 24) * math.pi ** (-2 / 3) * Mc ** (5 / 6) * f ** (-7 / 6) / D
        assert abs(abs(Kp) * a[0] / ref - 1) < 1e-12


# Leading-order magnitudes of the post-Newtonian mode amplitudes H_lm,
# relative to H_22 = 1 (Blanchet, Living Rev. Relativ. 17 (2014) 2, Sec. 9.5):
# h_lm(t) is proportional to x H_lm(x) e^{-i m Phi(t)}, x = (M omega)^(2/3),
# delta = (m1 - m2) / M.
def _pn_mode_magnitude(l, m, eta, delta, x):
    v = np.sqrt(x)
    return {(2, 2): np.ones_like(x),
            (3, 3): 0.75 * math.sqrt(15 / 14) * delta * v,
            (4, 4): 8 / 9 * math.sqrt(5 / 7) * (1 - 3 * eta) * x,
            (2, 1): delta * v / 3,
            (3, 2): math.sqrt(5 / 7) / 3 * (1 - 3 * eta) * x,
            (4, 3): 9 / (4 * math.sqrt(70)) * delta * (1 - 2 * eta) * x ** 1.5}[(l, m)]


def _fourier_amplitude_of_td_mode(l, m, M, eta, delta, x_s):
    """|int h_lm(t) e^{2 pi i f t} dt| by direct quadrature, for the Newtonian
    inspiral (dx/dt = 64 eta x^5 / (5 M), Phi = -x^(-5/2) / (32 eta)) at the
    frequency f = m omega / 2 pi whose stationary point has x = x_s.  A
    Gaussian window of width 4 / sqrt(m Phi'') about the stationary time keeps
    the integral finite; its effect on the magnitude is the same factor for
    every mode, so it cancels in ratios between modes."""
    phi2 = m * 96 / 5 * eta * x_s ** 5.5 / M ** 2
    sig = 4 / math.sqrt(phi2)
    tau_s = 5 * M / (256 * eta * x_s ** 4)
    t = np.linspace(-6 * sig, 6 * sig, 60001)
    x = (5 * M / (256 * eta * (tau_s - t))) ** 0.25
    f = m * x_s ** 1.5 / (2 * math.pi * M)
    ph = 2 * math.pi * f * t + (x ** -2.5 - x_s ** -2.5) * m / (32 * eta)
    h = x * _pn_mode_magnitude(l, m, eta, delta, x) * np.exp(1j * ph - t ** 2 / (2 * sig ** 2))
    return abs(np.trapezoid(h, t)), f


@pytest.mark.parametrize("q", [0.3, 0.8])
@pytest.mark.parametrize("lm", [(3, 3), (4, 4), (2, 1), (3, 2), (4, 3)])
def test_higher_mode_amplitude_ratio_from_time_domain_modes(q, lm):
    """A_lm(f) / A_22(2f/m) against the Fourier transform of time-domain
    post-Newtonian modes (leading-order H_lm, Newtonian phasing): fixes each
    mode's numerical prefactor, its power of v and the stationary-phase
    factor sqrt(2/m) that relates time-domain and Fourier amplitudes."""
    l, m = lm
    th = THETA.copy()
    th[0], th[1] = 3e5, q
    M = th[0] * MSUN_S
    eta, delta = q / (1 + q) ** 2, (1 - q) / (1 + q)
    for x_s in (1e-3, 3e-3):
        a22, f22 = _fourier_amplitude_of_td_mode(2, 2, M, eta, delta, x_s)
        alm, f = _fourier_amplitude_of_td_mode(l, m, M, eta, delta, x_s)
        assert abs(f22 - 2 * f / m) <= 1e-12 * f22
        want = alm / a22
        got = O.mode(th, l, m, np.array([f]))[0][0] / O.mode(th, 2, 2, np.array([f22]))[0][0]
        assert abs(got / want - 1) < 1e-5, (lm, q, x_s, got, want)


def test_transition_continuity_and_fmax():
    M, f1 = _fsets(THETA)
    eps = 1e-9 * f1
    a, p, t, _ = O.mode(THETA, 2, 2, np.array([f1 - eps, f1 + eps]))
    assert abs(a[1] / a[0] - 1) < 1e-7
    assert abs(p[1] - p[0]) < 1e-5
    assert abs(t[1] - t[0]) < 1e-3
    fm = O.fmax(THETA)
    fs = np.exp(np.linspace(math.log(0.5 * f1), math.log(0.2 / M), 200001))
    a, p, t, _ = O.mode(THETA, 2, 2, fs)
    k = np.argmax(fs ** 2 * a)
    assert abs(fs[k] / fm - 1) < 2e-4
    _, p, t, _ = O.mode(THETA, 2, 2, np.array([fm]))
    assert abs(t[0] - THETA[10]) < 1e-6
    assert abs(p[0]) < 1e-9


def test_support_mask():
    M, f1 = _fsets(THETA)
    for (l, m) in [(2, 2), (3, 3), (4, 4)]:
        fcut = m / 2 * 0.2 / M
        _, _, _, on = O.mode(THETA, l, m, np.array([0.99 * fcut, 1.01 * fcut]))
        assert on[0] and not on[1]
    # early inspiral before t = 0 is cut off
    _, _, tf, on = O.mode(THETA, 2, 2, np.array([1e-7, 1e-3]))
    assert tf[0] < 0 and not on[0] and on[1]


# ----------------------------------------------------------------- orbit and response
def test_orbit_geometry():
    e = L_S / (2 * math.sqrt(3) * R_S)
    for t in (0.0, 1.3e6, 7.7e6, 2.2e7):
        p = O.orbit(t)
        a = 2 * math.pi * t / I.YEAR_S
        c = p.mean(axis=0)
        assert np.allclose(c, [R_S * math.cos(a), R_S * math.sin(a), 0.0], atol=1e-12 * R_S)
        for i, j in ((0, 1), (1, 2), (2, 0)):
            arm = np.linalg.norm(p[i] - p[j])
            assert abs(arm / L_S - 1) < 3 * e
        nrm = np.cross(p[1] - p[0], p[2] - p[0])
        incl = math.degrees(math.acos(abs(nrm[2]) / np.linalg.norm(nrm)))
        assert abs(incl - 60.0) < 1.0
    assert np.allclose(O.orbit(1.0e6), O.orbit(1.0e6 + I.YEAR_S), atol=1e-9)


def _pol_basis(lam, beta, psi):
    k = -np.array([math.cos(beta) * math.cos(lam), math.cos(beta) * math.sin(lam), math.sin(beta)])
    u = np.array([math.sin(lam), -math.cos(lam), 0.0])
    v = np.array([-math.sin(beta) * math.cos(lam), -math.sin(beta) * math.sin(lam), math.cos(beta)])
    p = math.cos(psi) * u + math.sin(psi) * v
    q = -math.sin(psi) * u + math.cos(psi) * v
    return k, np.outer(p, p) - np.outer(q, q), np.outer(p, q) + np.outer(q, p)


def _td_link(i, j, t, f0, p, sky, Kp, Kc):
    """y_{i->j}(t) from the plane-wave metric at the retarded emission and
    reception events (frozen positions); h+(t) = Re[Kp e^{-2 pi i f0 t}], hx likewise."""
    k, ep, ec = sky
    n = p[j] - p[i]
    n /= np.linalg.norm(n)
    proj_p, proj_c = n @ ep @ n, n @ ec @ n

    def H(tt):
        z = np.exp(-2j * math.pi * f0 * tt)
        return proj_p * (Kp * z).real + proj_c * (Kc * z).real

    return (H(t - L_S - k @ p[i]) - H(t - k @ p[j])) / (2 * (1 - k @ n))


def _amplitude(y, t, f0):
    T = t[-1] - t[0] + (t[1] - t[0])
    return 2.0 / t.size * np.sum(y * np.exp(2j * math.pi * f0 * t)) * (t.size * (t[1] - t[0]) / T)


@pytest.mark.parametrize("f0", [1e-3, 1.7e-2, 0.045])
def test_link_matches_time_domain(f0):
    lam, beta, psi = 3.509, 0.293, 0.8
    sky = _pol_basis(lam, beta, psi)
    p = O.orbit(5.0e6)
    n_per, n_cyc = 64, 16
    t = np.arange(n_per * n_cyc) / (n_per * f0)
    for Kp, Kc in ((1.0 + 0j, 0j), (0j, 1.0 + 0j), (0.3 - 0.8j, 0.5 + 0.2j)):
        for i, j in ((0, 1), (1, 0), (2, 1), (0, 2)):
            y = _td_link(i, j, t, f0, p, sky, Kp, Kc)
            ref = _amplitude(y, t, f0)
            got = O.link(i, j, f0, p, lam, beta, psi, Kp, Kc)
            assert abs(got - ref) < 1e-9 * max(abs(ref), 1e-30) + 1e-14, (i, j, Kp, Kc)


def test_tdi_x_matches_time_domain_michelson():
    lam, beta, psi = 1.1, -0.6, 2.0
    sky = _pol_basis(lam, beta, psi)
    t_orb = 9.0e6
    p = O.orbit(t_orb)
    f0 = 7e-3
    Kp, Kc = 0.4 + 0.1j, -0.2 + 0.7j
    n_per, n_cyc = 64, 16
    t = np.arange(n_per * n_cyc) / (n_per * f0)
    y = lambda i, j, d: _td_link(i - 1, j - 1, t - d * L_S, f0, p, sky, Kp, Kc)
    X = (y(3, 1, 0) + y(1, 3, 1) + y(2, 1, 2) + y(1, 2, 3)) - (y(2, 1, 0) + y(1, 2, 1) + y(3, 1, 2) + y(1, 3, 3))
    ref = _amplitude(X, t, f0)
    got = O.tdi(f0, t_orb, lam, beta, psi, Kp, Kc)
    assert abs(got[0] - ref) < 1e-8 * abs(ref)


def test_aet_is_orthogonal_transform_and_t_suppressed():
    Kp, Kc = 0.7 + 0.2j, -0.1 + 0.5j
    for f in (1e-4, 3e-3, 2e-2):
        o = O.tdi(f, 3.3e6, 0.4, 0.9, 1.3, Kp, Kc)
        xyz = np.sum(np.abs(o[:3]) ** 2)
        aet = np.sum(np.abs(o[3:]) ** 2)
        assert abs(aet / xyz - 1) < 1e-12
    lo = O.tdi(1e-4, 3.3e6, 0.4, 0.9, 1.3, Kp, Kc)
    assert abs(lo[5]) < 1e-3 * max(abs(lo[3]), abs(lo[4]))
