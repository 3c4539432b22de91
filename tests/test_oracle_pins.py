"""Pins of the FP64 oracle against facts other than itself (CPU only).

Each test names what it checks against: closed forms of Eq. (1), library
routines (scipy quadrature and distributions, numpy interpolation), a
Gaussian toy population whose likelihood and selection function have closed
forms, 30-digit brute force on tiny inputs, exact invariances, and central
finite differences for the gradient.
"""
import copy
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest
import scipy.integrate as si
import scipy.stats as ss
import torch

from oracle import dsl_oracle as O
from paper_2605_23538_amd import synth
from tests import oracle_fixtures as F

T = lambda a: torch.tensor(a, dtype=torch.float64)
C = O.C_KMS
HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- Eq. (1)
@pytest.mark.parametrize("H0", [40.0, 70.0, 120.0])
def test_dl_closed_forms(H0):
    z = np.linspace(0.0, 2.0, 41)
    # Omega_m = 1 (Einstein-de Sitter): d_L = 2 c/H0 (1+z) (1 - (1+z)^-1/2)
    eds = 2 * C / H0 * (1 + z) * (1 - (1 + z) ** -0.5)
    got = O.dl_of_z(T(z), T(H0), T(1.0)).numpy()
    np.testing.assert_allclose(got, eds, rtol=1e-13, atol=1e-9)
    # Omega_m = 0 (pure Lambda): d_L = c/H0 z (1+z), dd_L/dz = c/H0 (1+2z)
    got0 = O.dl_of_z(T(z), T(H0), T(0.0)).numpy()
    np.testing.assert_allclose(got0, C / H0 * z * (1 + z), rtol=1e-13, atol=1e-9)
    np.testing.assert_allclose(O.ddl_dz(T(z), T(H0), T(0.0)).numpy(), C / H0 * (1 + 2 * z), rtol=1e-13)
    dEdS = 2 * C / H0 * (1 - 0.5 * (1 + z) ** -0.5)  # derivative of the EdS form
    np.testing.assert_allclose(O.ddl_dz(T(z), T(H0), T(1.0)).numpy(), dEdS, rtol=1e-13)


@pytest.mark.parametrize("Om", [0.1, 0.3, 0.5, 0.9])
def test_comoving_integral_vs_scipy(Om):
    for z in [0.01, 0.3, 1.0, 1.7, 2.0]:
        ref = si.quad(lambda x: 1 / math.sqrt(Om * (1 + x) ** 3 + 1 - Om), 0, z, epsabs=0, epsrel=2e-14)[0]
        got = float(O.comoving_integral(T(z), T(Om)))
        assert abs(got / ref - 1) < 5e-14


@pytest.mark.parametrize("Om", [0.0, 0.3, 1.0])
def test_z_of_dl_inverse(Om):
    H0 = 70.0
    dl = np.array([1.0, 50.0, 800.0, 1500.0, 4000.0, 10000.0])
    z, inside = O.z_of_dl(T(dl), T(H0), T(Om), 2.0)
    assert bool(inside.all())
    back = O.dl_of_z(z, T(H0), T(Om)).detach().numpy()
    np.testing.assert_allclose(back, dl, rtol=1e-14)
    if Om == 0.0:
        ref = [F.z_closed_om0(d, H0) for d in dl]
        np.testing.assert_allclose(z.detach().numpy(), ref, rtol=1e-14)
    # beyond d_L(z_max): outside the support
    big = float(O.dl_of_z(T(2.0), T(H0), T(Om))) * (1 + 1e-9)
    _, ins = O.z_of_dl(T([big]), T(H0), T(Om), 2.0)
    assert not bool(ins[0])


def test_dl_scales_inversely_with_H0():
    z = T(np.linspace(0.05, 2, 9))
    a = O.dl_of_z(z, T(50.0), T(0.3))
    b = O.dl_of_z(z, T(100.0), T(0.3))
    np.testing.assert_allclose((a / b).numpy(), 2.0, rtol=1e-15)


def test_dz_dH0_closed_form():
    """Implicit derivative dz/dH0 = (d_L/c) / D'(z) at fixed d_L (Omega_m = 0 closed form)."""
    H0 = T(70.0).requires_grad_(True)
    dl = T([1200.0])
    z, _ = O.z_of_dl(dl, H0, T(0.0), 2.0)
    g = torch.autograd.grad(z.sum(), H0)[0]
    u = 1200.0 * 70.0 / C
    dz_du = 1.0 / math.sqrt(1 + 4 * u)
    assert abs(float(g) / (dz_du * 1200.0 / C) - 1) < 1e-13


# ---------------------------------------------------------------- mass model
def _L(**kw):
    return O.Lam.of(T(synth.lam_vector(**kw)))


@pytest.mark.parametrize("kw", [dict(), dict(alpha=1.0), dict(alpha=7.0, lambda_g=0.1),
                                dict(mu_low=5.5, sigma_low=3.0, mmin=5.0)])
def test_p1_normalised_without_smoothing(kw):
    """delta_m = 0: p1 is a normalised mixture on [mmin, mmax] (scipy quad)."""
    L = _L(delta_m=0.0, **kw)
    f = lambda m: math.exp(float(O.log_p1(T([m]), L)[0]))
    lo, hi = float(L.mmin), float(L.mmax)
    pts = [float(L.mu_low), float(L.mu_high)]
    val = si.quad(f, lo, hi, points=[p for p in pts if lo < p < hi], epsabs=0, epsrel=1e-12, limit=400)[0]
    assert abs(val - 1) < 1e-10


def test_p1_components_vs_scipy():
    """Peak-only and power-law-only limits against scipy / closed forms."""
    m = np.linspace(4.7, 86.0, 50)
    L = _L(delta_m=0.0, lambda_g=1.0, lambda_low=1.0)
    ref = ss.truncnorm.logpdf(m, (4.6 - 9.7) / 0.7, (86.3 - 9.7) / 0.7, loc=9.7, scale=0.7)
    got = O.log_p1(T(m), L).numpy()
    ok = np.isfinite(ref)
    np.testing.assert_allclose(got[ok], ref[ok], rtol=1e-12, atol=1e-12)
    L = _L(delta_m=0.0, lambda_g=0.0)
    a, lo, hi = 2.9, 4.6, 86.3
    ref = np.log((a - 1) / (lo ** (1 - a) - hi ** (1 - a)) * m ** -a)
    np.testing.assert_allclose(O.log_p1(T(m), L).numpy(), ref, rtol=1e-13)


def test_smoothing_function():
    mmin, dm = 4.6, 4.8
    m = np.array([4.0, 4.6, 4.601, 5.5, 7.0, 9.39, 9.4, 20.0])
    got = np.exp(O.log_smoothing(T(m), T(mmin), T(dm)).numpy())
    ref = []
    for x in m:
        mp_ = x - mmin
        if mp_ <= 0:
            ref.append(0.0)
        elif mp_ >= dm:
            ref.append(1.0)
        else:
            y = dm / mp_ + dm / (mp_ - dm)
            ref.append(1.0 / (1.0 + math.exp(y)) if y < 700 else math.exp(-y))
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-300)


@pytest.mark.parametrize("kw", [dict(), dict(beta=-1.0), dict(beta=-3.5, delta_m=9.0, mmin=2.5),
                                dict(beta=6.0, delta_m=0.0)])
def test_p2_normalised(kw):
    """p2(. | m1) integrates to one over [mmin, m1], in and above the window."""
    L = _L(**kw)
    mmin, M = float(L.mmin), float(L.mmin + L.delta_m)
    for m1 in [mmin + 0.3 * max(float(L.delta_m), 0.5), M + 0.01, 0.5 * (M + 80), 80.0]:
        f = lambda m2: math.exp(float(O.log_p2(T([m2]), T([m1]), L)[0]))
        val = si.quad(f, mmin, m1, epsabs=0, epsrel=1e-12, limit=400,
                      points=[min(M, m1 - 1e-9)] if M < m1 else None)[0]
        assert abs(val - 1) < 1e-9, (m1, val)


def test_Z_delta_zero_closed_form():
    L = _L(delta_m=0.0, beta=1.7)
    m1 = np.array([5.0, 30.0, 80.0])
    s = 2.7
    ref = np.log((m1 ** s - 4.6 ** s) / s)
    np.testing.assert_allclose(O.log_Z(T(m1), L).numpy(), ref, rtol=1e-13)


def test_Z_window_vs_mpmath():
    """Window integral int_mmin^m1 m^beta S(m) dm against 30-digit tanh-sinh."""
    mp.mp.dps = 30
    for (mmin, dm, beta) in [(4.6, 4.8, 1.0), (2.0, 10.0, -4.0), (8.0, 2.0, 9.0)]:
        L = _L(mmin=mmin, delta_m=dm, beta=beta)

        def S(m):
            x = m - mmin
            if x <= 0:
                return mp.mpf(0)
            if x >= dm:
                return mp.mpf(1)
            return 1 / (1 + mp.e ** (dm / x + dm / (x - dm)))
        for t in [0.08, 0.3, 0.7, 1.0, 1.8]:
            m1 = mmin + t * dm
            ref = mp.quad(lambda m: m ** beta * S(m), [mmin, mmin + min(t, 1) * dm] + ([m1] if t > 1 else []))
            got = float(O.log_Z(T([m1]), L)[0])
            assert abs(got - float(mp.log(ref))) < 1e-12, (mmin, dm, beta, t)


# ---------------------------------------------------------------- rate, LOS
def test_rate_special_cases():
    z = T(np.linspace(0, 2, 11))
    L = _L(gamma=0.0, kappa=0.0)
    np.testing.assert_allclose(O.log_psi(z, L).numpy(), -math.log(2.0), rtol=1e-15)
    L = _L(gamma=2.7, kappa=2.9, z_p=1.0)
    # at z = z_p: (1+z)^gamma / 2
    assert abs(float(O.log_psi(T(1.0), L)) - (2.7 * math.log(2) - math.log(2))) < 1e-14
    # Madau-Dickinson shape at z = 0: 1 / (1 + (1+z_p)^-(gamma+kappa))
    assert abs(float(O.log_psi(T(0.0), L)) + math.log1p(2 ** -5.6)) < 1e-14


def test_los_interp_vs_numpy():
    rng = np.random.default_rng(0)
    tab = rng.random((3, 33))
    z = rng.uniform(0, 2, 200)
    rows = rng.integers(0, 3, 200)
    got = O.los_interp(T(tab), torch.from_numpy(rows), T(z), 2.0).numpy()
    zg = np.linspace(0, 2, 33)
    ref = np.array([np.interp(zz, zg, tab[r]) for zz, r in zip(z, rows)])
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-15)
    out = O.los_interp(T(tab), torch.tensor([0, 1]), T([-0.1, 2.0001]), 2.0).numpy()
    assert (out == 0).all()


# ---------------------------------------------------------------- Eq. (8)
def test_neff_invariants():
    seg = torch.zeros(5, dtype=torch.int64)
    lw = T([0.3] * 5)
    l1 = O.segment_lse(lw, seg, 1)
    l2 = O.segment_lse(2 * lw, seg, 1)
    assert abs(math.exp(2 * float(l1[0]) - float(l2[0])) - 5) < 1e-13
    lw = T([0.0, -math.inf, -math.inf])
    l1 = O.segment_lse(lw, torch.zeros(3, dtype=torch.int64), 1)
    l2 = O.segment_lse(2 * lw, torch.zeros(3, dtype=torch.int64), 1)
    assert abs(math.exp(2 * float(l1[0]) - float(l2[0])) - 1) < 1e-15
    rng = np.random.default_rng(1)
    for _ in range(20):
        x = rng.normal(0, 3, 17)
        l1 = float(O.segment_lse(T(x), torch.zeros(17, dtype=torch.int64), 1)[0])
        l2 = float(O.segment_lse(T(2 * x), torch.zeros(17, dtype=torch.int64), 1)[0])
        ne = math.exp(2 * l1 - l2)
        assert 1 - 1e-12 <= ne <= 17 + 1e-12


# ---------------------------------------------------------------- Gaussian toy
TOY_EVENTS = [(35.0 * 1.19, 2.0, 800.0), (31.0 * 1.4, 3.0, 1500.0), (50.0, 1.5, 2500.0)]


def test_gaussian_toy_event_likelihood():
    H0, mu, sigma = 70.0, 30.0, 3.0
    cat = F.make_toy_catalog(TOY_EVENTS, H0, mu, sigma)
    r = O.loglike(cat, F.toy_lambda(H0, mu, sigma))
    assert r["flags"] == 0
    n_s = cat.samples_per_event()
    for i, (x, s, d) in enumerate(TOY_EVENTS):
        truth = F.toy_event_truth(x, s, d, H0, mu, sigma)
        got = r["logL_event"][i] + math.log(n_s[i])
        assert abs(got - math.log(truth)) < 1e-11, (i, got, math.log(truth))


def test_gaussian_toy_selection_and_total():
    H0, mu, sigma = 55.0, 25.0, 2.5
    cat = F.make_toy_catalog(TOY_EVENTS[:2], H0, mu, sigma)
    r = O.loglike(cat, F.toy_lambda(H0, mu, sigma))
    # alpha = int_0^2 psi(z)/(1+z) dz = (1/2) ln 3 for a flat sky table
    assert abs(r["ln_alpha"] - math.log(0.5 * math.log(3.0))) < 1e-11
    n_s = cat.samples_per_event()
    truth = sum(math.log(F.toy_event_truth(x, s, d, H0, mu, sigma)) - math.log(n)
                for (x, s, d), n in zip(TOY_EVENTS[:2], n_s))
    truth -= 2 * math.log(0.5 * math.log(3.0))
    assert abs(r["logL"] - truth) < 1e-10


def test_monte_carlo_jacobian():
    """Injections drawn uniformly in detector space: mean weight -> int p_pop.

    No Jacobian is constructed here: draws are uniform in a box of
    (m1_det, m2_det, d_L) that covers the support, ln p_draw is the box
    density, and the estimate must reach int psi/(1+z) dz (within 5 sigma).
    """
    rng = np.random.default_rng(11)
    H0, Om, z_max = 70.0, 0.3, 2.0
    lam = synth.lam_vector(H0=H0, Om=Om, delta_m=0.0, gamma=0.0, kappa=0.0, mmin=5.0, mmax=60.0,
                           lambda_g=0.6, lambda_low=0.5, mu_low=12.0, sigma_low=2.0,
                           mu_high=35.0, sigma_high=4.0, alpha=2.3, beta=0.5)
    d_max = float(O.dl_of_z(T(z_max), T(H0), T(Om)))
    n = 1_000_000
    box = np.array([60 * 3.0, 60 * 3.0, d_max])
    m1 = rng.uniform(0, box[0], n)
    m2 = rng.uniform(0, box[1], n)
    dl = rng.uniform(0, box[2], n)
    lp = np.full(n, -np.log(box).sum())
    cat = synth.Catalog(
        event_pix_off=np.array([0, 1]), pix_samp_off=np.array([0, 1]), pix_los_row=np.zeros(1, np.int32),
        los=np.ones((1, 64), np.float32), sky_z=np.ones(64, np.float32), z_max=z_max,
        m1d=np.array([30.0]), m2d=np.array([20.0]), dl=np.array([1000.0]), ln_pi=np.array([0.0]),
        inj_m1d=m1, inj_m2d=m2, inj_dl=dl, inj_ln_pdraw=lp, n_draw=n)
    L = O.Lam.of(T(lam))
    lw = O.log_weights(T(m1), T(m2), T(dl), T(lp), T(np.ones((1, 64))), torch.zeros(n, dtype=torch.int64),
                       z_max, L).numpy()
    w = np.exp(lw)
    est, se = w.mean(), w.std() / math.sqrt(n)
    target = si.quad(lambda z: 0.5 / (1 + z), 0, z_max)[0]   # psi = 1/2 at gamma = kappa = 0
    assert abs(est - target) < 5 * se, (est, target, se)
    assert se / target < 0.03


# ---------------------------------------------------------------- brute force
def _mp_loglike(cat, lam, neff_min=2.0, flip=(), neff_out=None):
    """The definition evaluated with 30-digit mpmath (tanh-sinh, findroot); the
    gate decisions of the pixels in `flip` are inverted; neff_out collects every
    pixel's N_eff."""
    mp.mp.dps = 30
    H0, Om, a, b, mmin, mmax, dm, mul, sl, muh, sh, lg, ll, gam, kap, zp = [mp.mpf(float(x)) for x in lam]
    c = mp.mpf(C)
    Ez = lambda z: mp.sqrt(Om * (1 + z) ** 3 + 1 - Om)
    Iz = lambda z: mp.quad(lambda x: 1 / Ez(x), [0, z])
    zmax = mp.mpf(cat.z_max)
    Dmax = (1 + zmax) * Iz(zmax)

    def S(m):
        x = m - mmin
        if x <= 0:
            return mp.mpf(0)
        if x >= dm:
            return mp.mpf(1)
        return 1 / (1 + mp.e ** (dm / x + dm / (x - dm)))
    Ncdf = lambda x: (1 + mp.erf(x / mp.sqrt(2))) / 2
    def Nt(m, mu, s):
        return mp.npdf(m, mu, s) / (Ncdf((mmax - mu) / s) - Ncdf((mmin - mu) / s))
    Pn = (1 - a) / (mmax ** (1 - a) - mmin ** (1 - a))
    def p1(m):
        if m <= mmin or m > mmax:
            return mp.mpf(0)
        return S(m) * ((1 - lg) * Pn * m ** (-a) + lg * ll * Nt(m, mul, sl) + lg * (1 - ll) * Nt(m, muh, sh))
    def Z(m1):
        pts = [mmin, min(m1, mmin + dm)] + ([m1] if m1 > mmin + dm else [])
        return mp.quad(lambda m: m ** b * S(m), pts)
    def p2(m2, m1):
        if m2 > m1 or m2 <= mmin:
            return mp.mpf(0)
        return m2 ** b * S(m2) / Z(m1)
    def psi(z):
        return (1 + z) ** gam / (1 + ((1 + z) / (1 + zp)) ** (gam + kap))
    def weight(m1d, m2d, dl, lnp, tab):
        u = mp.mpf(float(dl)) * H0 / c
        if u > Dmax:
            return mp.mpf(0)
        z = mp.findroot(lambda zz: (1 + zz) * Iz(zz) - u, (mp.mpf(0), zmax), solver="anderson")
        nz = len(tab)
        x = z / zmax * (nz - 1)
        k = min(int(mp.floor(x)), nz - 2)
        f = x - k
        los = mp.mpf(float(tab[k])) * (1 - f) + mp.mpf(float(tab[k + 1])) * f
        m1 = mp.mpf(float(m1d)) / (1 + z)
        m2 = mp.mpf(float(m2d)) / (1 + z)
        jac = (1 + z) ** 2 * (c / H0) * (Iz(z) + (1 + z) / Ez(z))
        return los * psi(z) / (1 + z) * p1(m1) * p2(m2, m1) / jac * mp.e ** (-mp.mpf(float(lnp)))
    lnL_ev = []
    for e in range(cat.n_events):
        S1p, n_s = mp.mpf(0), 0
        for p in range(cat.event_pix_off[e], cat.event_pix_off[e + 1]):
            ws = [weight(cat.m1d[k], cat.m2d[k], cat.dl[k], cat.ln_pi[k], cat.los[cat.pix_los_row[p]])
                  for k in range(cat.pix_samp_off[p], cat.pix_samp_off[p + 1])]
            n_s += len(ws)
            s1, s2 = sum(ws), sum(w * w for w in ws)
            passes = s2 > 0 and s1 * s1 / s2 >= neff_min
            if neff_out is not None:
                neff_out.append(s1 * s1 / s2 if s2 > 0 else mp.mpf(0))
            if p in flip and s1 > 0:
                passes = not passes
            if passes:
                S1p += s1
        lnL_ev.append(mp.log(S1p / n_s))
    alpha = sum(weight(cat.inj_m1d[n], cat.inj_m2d[n], cat.inj_dl[n], cat.inj_ln_pdraw[n], cat.sky_z)
                for n in range(cat.n_inj)) / cat.n_draw
    return [float(x) for x in lnL_ev], float(mp.log(alpha)), float(sum(lnL_ev) - cat.n_events * mp.log(alpha))


@pytest.mark.parametrize("lam_kw,neff_min", [
    (dict(), 2.0),
    (dict(H0=45.0, Om=0.45, delta_m=8.0, beta=-2.0, z_p=0.5, gamma=5.0), 2.0),   # one event fails the gate
    (dict(H0=45.0, Om=0.45, delta_m=8.0, beta=-2.0, z_p=0.5, gamma=5.0), 1.2)])
def test_bruteforce_mpmath(lam_kw, neff_min):
    cat = F.tiny_catalog()
    lam = synth.lam_vector(**lam_kw)
    ev, la, tot = _mp_loglike(cat, lam, neff_min)
    r = O.loglike(cat, lam, neff_min=neff_min)
    np.testing.assert_allclose(r["logL_event"], ev, rtol=1e-12, atol=1e-12)
    assert abs(r["ln_alpha"] - la) < 1e-12
    np.testing.assert_allclose([r["logL"]], [tot], rtol=1e-12)


@pytest.mark.parametrize("flip", [[0], [1, 2], [3]])
def test_gate_flip_and_pixel_margins_bruteforce(flip):
    """The oracle's other-outcome hook (a path in another precision may decide
    a pixel near the N_eff threshold the other way) and its per-pixel gate
    margins, against the 30-digit definition with the same decisions inverted."""
    cat = F.tiny_catalog()
    lam = synth.lam_vector(H0=45.0, Om=0.45, delta_m=8.0, beta=-2.0, z_p=0.5, gamma=5.0)
    neff = []
    ev, la, tot = _mp_loglike(cat, lam, 2.0, flip=set(flip), neff_out=neff)
    r = O.loglike(cat, lam, gate_flip=flip, margins=True)
    np.testing.assert_allclose(r["logL_event"], ev, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose([r["logL"]], [tot], rtol=1e-12)
    base = O.loglike(cat, lam)
    assert not np.allclose(base["logL_event"], r["logL_event"], rtol=1e-9, atol=0)
    want = [abs(float(mp.log(n)) - math.log(2.0)) for n in neff]
    np.testing.assert_allclose(r["pixel_gate_margin"], want, rtol=1e-9, atol=1e-12)


def test_kde_gate_flip_of_the_failing_pixels_is_the_ungated_likelihood():
    """The KDE oracle's other-outcome hook: inverting the Eq. (8) decision of
    exactly the pixels that fail it passes every pixel with weight, which is
    the likelihood with the gate disabled (gate_mode 2); its per-pixel margins
    are |ln N_eff - ln 2| of those pixels."""
    cat = synth.make_catalog("c1", n_events=3, n_inj=400)
    lam = synth.lam_vector(H0=45.0, Om=0.45, delta_m=8.0, beta=-2.0)
    base = O.loglike_kde(cat, lam, margins=True)
    pm = base["pixel_gate_margin"]
    lneff = []
    failing = []
    for j in range(cat.n_pix):
        s0, s1 = int(cat.pix_samp_off[j]), int(cat.pix_samp_off[j + 1])
        if s1 == s0:
            continue
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a[s0:s1], dtype=np.float64))
        _, inside, lw = O.kde_log_weights(t(cat.m1d), t(cat.m2d), t(cat.dl), t(cat.ln_pi), cat.z_max, O.Lam.of(T(lam)))
        lw = lw[inside].numpy()
        if lw.size == 0 or not np.isfinite(lw).any():
            continue
        m = lw.max()
        ln = 2 * (m + math.log(np.exp(lw - m).sum())) - (2 * m + math.log(np.exp(2 * (lw - m)).sum()))
        lneff.append((j, ln))
        if ln < math.log(2.0):
            failing.append(j)
    assert failing, "the case must have pixels that fail the gate"
    for j, ln in lneff:
        assert abs(pm[j] - abs(ln - math.log(2.0))) < 1e-9
    flipped = O.loglike_kde(cat, lam, gate_flip=failing)
    ungated = O.loglike_kde(cat, lam, gate_mode=2)
    np.testing.assert_allclose(flipped["logL_event"], ungated["logL_event"], rtol=1e-12)
    assert not np.allclose(base["logL_event"], ungated["logL_event"], rtol=1e-9, atol=0)


# ---------------------------------------------------------------- invariances
def test_invariance_H0_distance_rescaling():
    """(d_L, H0) -> (s d_L, H0/s) leaves every redshift unchanged; the Jacobian
    scales by s in each event and in alpha alike, so ln L is unchanged."""
    cat = synth.make_catalog("c1", n_events=3, n_inj=3000)
    lam = synth.fiducial_lambda()
    r0 = O.loglike(cat, lam)
    s = 1.37
    cat2 = synth.Catalog(**{**cat.__dict__, "dl": cat.dl * s, "inj_dl": cat.inj_dl * s})
    lam2 = lam.copy()
    lam2[0] /= s
    r1 = O.loglike(cat2, lam2)
    assert abs(r1["logL"] - r0["logL"]) < 1e-9 * abs(r0["logL"])
    np.testing.assert_allclose(r1["logL_event"] + math.log(s), r0["logL_event"], rtol=1e-12)


def test_invariance_table_scaling_permutation_padding():
    cat = synth.make_catalog("c1", n_events=2, n_inj=2000)
    lam = synth.fiducial_lambda()
    r0 = O.loglike(cat, lam)
    # every pixel table x c1 shifts each ln L_i by ln c1 (gate is scale free)
    r1 = O.loglike(synth.Catalog(**{**cat.__dict__, "los": cat.los * 4.0}), lam)
    np.testing.assert_allclose(r1["logL_event"], r0["logL_event"] + math.log(4.0), rtol=1e-13)
    # sky table x c2 shifts ln alpha by ln c2
    r2 = O.loglike(synth.Catalog(**{**cat.__dict__, "sky_z": cat.sky_z * 2.0}), lam)
    assert abs(r2["logL"] - (r0["logL"] - cat.n_events * math.log(2.0))) < 1e-9
    # permuting samples inside a pixel
    p = np.arange(cat.n_samp)
    a, b = cat.pix_samp_off[3], cat.pix_samp_off[4]
    p[a:b] = p[a:b][::-1]
    cat3 = synth.Catalog(**{**cat.__dict__, "m1d": cat.m1d[p], "m2d": cat.m2d[p], "dl": cat.dl[p], "ln_pi": cat.ln_pi[p]})
    r3 = O.loglike(cat3, lam)
    assert abs(r3["logL"] - r0["logL"]) < 1e-10
    # an empty pixel (padding) contributes nothing
    pso = np.insert(cat.pix_samp_off, 2, cat.pix_samp_off[2])
    epo = cat.event_pix_off.copy()
    epo[1:] += 1
    cat4 = synth.Catalog(**{**cat.__dict__, "pix_samp_off": pso, "event_pix_off": epo,
                            "pix_los_row": np.insert(cat.pix_los_row, 2, 0)})
    r4 = O.loglike(cat4, lam)
    assert abs(r4["logL"] - r0["logL"]) < 1e-12


def test_invalid_lambda_and_no_pixel_flags():
    cat = F.tiny_catalog()
    bad = synth.lam_vector(mmin=90.0)
    r = O.loglike(cat, bad)
    assert r["flags"] & O.FLAG_INVALID_LAMBDA and r["logL"] == -math.inf
    r = O.loglike(cat, synth.fiducial_lambda(), neff_min=1e9)
    assert r["flags"] & O.FLAG_EVENT_NO_PIXEL and r["logL"] == -math.inf


def test_event_without_samples():
    """An event with no pixels, or with pixels holding no samples, has an empty
    Monte Carlo sum: ln L_i = -inf (not 0/0), flag 2, in both numerators; the
    other events keep exactly the values they have without it."""
    cat = F.tiny_catalog()
    lam = synth.fiducial_lambda()
    ref = O.loglike(cat, lam)
    ref_kde = O.loglike_kde(cat, lam)
    epo = np.asarray(cat.event_pix_off, np.int64)
    # event 0 without pixels, in front of the others
    no_pix = synth.Catalog(**{**cat.__dict__, "event_pix_off": np.concatenate([[0], epo])})
    # an extra last event with two empty pixels
    pso = np.asarray(cat.pix_samp_off, np.int64)
    empty_pix = synth.Catalog(**{**cat.__dict__, "event_pix_off": np.concatenate([epo, [epo[-1] + 2]]),
                                 "pix_samp_off": np.concatenate([pso, [pso[-1], pso[-1]]]),
                                 "pix_los_row": np.concatenate([cat.pix_los_row, [0, 0]]).astype(np.int32)})
    for c, i_empty, others in ((no_pix, 0, slice(1, None)), (empty_pix, cat.n_events, slice(0, -1))):
        for fn, r0 in ((O.loglike, ref), (O.loglike_kde, ref_kde)):
            r = fn(c, lam)
            assert r["flags"] == O.FLAG_EVENT_NO_PIXEL and r["logL"] == -math.inf
            assert r["logL_event"][i_empty] == -math.inf and r["neff_event"][i_empty] == 0.0
            np.testing.assert_array_equal(r["logL_event"][others], r0["logL_event"])


def test_table_ii_fixture():
    with open(os.path.join(HERE, "golden", "table_ii.json")) as f:
        g = json.load(f)
    for k, v in g["values"].items():
        if k in synth.TABLE_II:
            assert synth.TABLE_II[k] == v
    assert O.lambda_is_valid(synth.lam_vector(**g["values"]))


# ---------------------------------------------------------------- gradient
def test_gradient_vs_central_differences():
    cat = synth.make_catalog("c1", n_events=3, n_inj=2000)
    lam = synth.fiducial_lambda()
    r = O.loglike(cat, lam, grad=True, margins=True)
    g = r["grad"]
    assert np.all(np.isfinite(g))
    gn = np.linalg.norm(g)
    for p in range(16):
        h = 1e-6 * max(abs(lam[p]), 1.0)
        lp, lm = lam.copy(), lam.copy()
        lp[p] += h
        lm[p] -= h
        fd = (O.loglike(cat, lp)["logL"] - O.loglike(cat, lm)["logL"]) / (2 * h)
        assert abs(fd - g[p]) <= 2e-6 * gn + 1e-5 * abs(g[p]), (synth.LAMBDA_NAMES[p], fd, g[p])


def test_window_mean_is_one_half():
    """The logistic window S(m_min + t dm) averages to 1/2 over its width (30-digit
    quadrature), so the window integral is m_min^beta dm / 2 to first order in dm."""
    mp.mp.dps = 30
    f = lambda t: 1 / (1 + mp.e ** (1 / t + 1 / (t - 1)))
    assert abs(mp.quad(f, [0, 0.5, 1]) - mp.mpf(1) / 2) < mp.mpf(10) ** -25
    mmin, beta = 6.0, 2.5
    for dm in (1e-3, 1e-4):
        L = _L(mmin=mmin, delta_m=dm, beta=beta)
        zw = float(O._window_integral(T([mmin + dm]), L)[0])
        assert abs(zw / (0.5 * mmin ** beta * dm) - 1) < 2 * beta * dm / mmin


@pytest.mark.parametrize("beta", [1.0, 9.25])
def test_gradient_at_delta_m_zero(beta):
    """delta_m = 0 is the edge of its domain: d ln L / d delta_m there is the
    one-sided limit, checked against Richardson-extrapolated forward differences
    of ln L; the other entries against central differences."""
    cat = F.tiny_catalog()
    base = dict(delta_m=0.0, mmin=6.0, beta=beta)
    lam = synth.lam_vector(**base)
    r0 = O.loglike(cat, lam, grad=True)
    assert r0["flags"] == 0
    g = r0["grad"]
    gn = np.linalg.norm(g)
    f = lambda **kw: O.loglike(cat, synth.lam_vector(**{**base, **kw}))["logL"]
    D = lambda h: (f(delta_m=h) - r0["logL"]) / h
    h = 1e-4
    rich = 2 * D(h / 2) - D(h)
    assert abs(rich - g[6]) <= 1e-6 * max(abs(g[6]), 1e-2 * gn), (rich, g[6])
    for p in (0, 3, 4):
        hp = 1e-6 * max(abs(lam[p]), 1.0)
        name = synth.LAMBDA_NAMES[p]
        fd = (f(**{name: lam[p] + hp}) - f(**{name: lam[p] - hp})) / (2 * hp)
        assert abs(fd - g[p]) <= 2e-6 * gn + 1e-5 * abs(g[p]), (name, fd, g[p])


# ---------------------------------------------------------------- spectral sirens
def test_gaussian_toy_spectral():
    """Comoving-volume redshift prior, Omega_m = 0: I(z) = z, E = 1, so the prior
    is z^2; each toy event likelihood gains z_i^2 and alpha = (1/2) int z^2/(1+z) dz
    = (1/2) ln 3 over [0, 2]."""
    H0, mu, sigma = 70.0, 30.0, 3.0
    cat = F.make_toy_catalog(TOY_EVENTS, H0, mu, sigma)
    r = O.loglike(cat, F.toy_lambda(H0, mu, sigma), z_prior="comoving")
    n_s = cat.samples_per_event()
    for i, (x, s, d) in enumerate(TOY_EVENTS):
        z = F.z_closed_om0(d, H0)
        truth = F.toy_event_truth(x, s, d, H0, mu, sigma) * z * z
        assert abs(r["logL_event"][i] + math.log(n_s[i]) - math.log(truth)) < 1e-11
    assert abs(r["ln_alpha"] - math.log(0.5 * math.log(3.0))) < 1e-10


def test_comoving_prior_einstein_de_sitter():
    """Omega_m = 1: I = 2 (1 - (1+z)^-1/2), E = (1+z)^3/2 (closed forms)."""
    z = np.array([0.1, 0.5, 1.3])
    L = _L(Om=1.0)
    I = O.comoving_integral(T(z), L.Om).numpy()
    E = O.E_of_z(T(z), L.Om).numpy()
    ref = (2 * (1 - (1 + z) ** -0.5)) ** 2 / (1 + z) ** 1.5
    np.testing.assert_allclose(I ** 2 / E, ref, rtol=1e-13)


# ---------------------------------------------------------------- downsampling
def test_splitmix64_reference_values():
    """Published SplitMix64 test vector: seed 1234567 -> 6457827717110365317,
    3203168211198807973 (the generator's state advances by the golden gamma)."""
    g = 0x9E3779B97F4A7C15
    s1 = (1234567 + 0 * g) % 2 ** 64
    s2 = (1234567 + 1 * g) % 2 ** 64
    out = O.splitmix64(np.array([s1, s2], dtype=np.uint64))
    assert int(out[0]) == 6457827717110365317
    assert int(out[1]) == 3203168211198807973


def test_downsample_keeps_cap_per_pixel():
    cat = synth.make_catalog("c1", n_events=2, n_inj=100)
    ds = O.downsample(cat, 50, seed=7)
    counts = np.diff(ds.pix_samp_off)
    np.testing.assert_array_equal(counts, np.minimum(np.diff(cat.pix_samp_off), 50))
    # kept samples are a subset of each pixel, in their original order
    for j in range(cat.n_pix):
        a, b = cat.pix_samp_off[j], cat.pix_samp_off[j + 1]
        c, d = ds.pix_samp_off[j], ds.pix_samp_off[j + 1]
        src = cat.dl[a:b]
        got = ds.dl[c:d]
        pos = [int(np.flatnonzero(src == v)[0]) for v in got]
        assert pos == sorted(pos)
    # a different seed keeps a different subset
    ds2 = O.downsample(cat, 50, seed=8)
    assert not np.array_equal(ds.dl, ds2.dl)


def test_event_fp32_condition_bounds_input_perturbations():
    """The per-event sensitivities the parity tests allow for an FP32 evaluation
    of the inputs (d_L to 3.2e-7, masses to 6e-8, relative) bound the change of
    ln L_i and the relative change of N_eff,i under random perturbations of that
    size, and are not vacuous."""
    rng = np.random.default_rng(11)
    cat = synth.make_catalog("c1", n_events=3, n_inj=500)
    lam = synth.lam_vector(delta_m=0.5, mmin=7.0, beta=6.0, alpha=5.0)
    base = O.loglike(cat, lam, gate_mode=2, margins=True)
    cond = base["event_fp32_cond"]
    ncond = base["event_fp32_cond_neff"]
    assert np.all(cond > 0) and np.all(np.isfinite(cond))
    assert np.all(ncond > 0) and np.all(np.isfinite(ncond))
    worst = worst_n = 0.0
    for _ in range(3):
        c2 = copy.deepcopy(cat)
        c2.dl = cat.dl * (1 + 3.2e-7 * rng.choice([-1.0, 1.0], cat.n_samp))
        c2.m1d = cat.m1d * (1 + 6e-8 * rng.choice([-1.0, 1.0], cat.n_samp))
        c2.m2d = cat.m2d * (1 + 6e-8 * rng.choice([-1.0, 1.0], cat.n_samp))
        r = O.loglike(c2, lam, gate_mode=2)
        d = np.abs(r["logL_event"] - base["logL_event"])
        assert np.all(d <= cond * (1 + 1e-3)), (d, cond)
        worst = max(worst, float(np.max(d / cond)))
        dn = np.abs(np.log(r["neff_event"] / base["neff_event"]))
        assert np.all(dn <= ncond * (1 + 1e-3)), (dn, ncond)
        worst_n = max(worst_n, float(np.max(dn / ncond)))
    assert worst > 0.01 and worst_n > 0.01   # the bounds are not vacuous
