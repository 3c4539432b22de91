"""Hand-built catalogues used to pin the oracle (no GPU, no generator)."""
import math

import numpy as np

from paper_2605_23538_amd.synth import Catalog, lam_vector

C_KMS = 299792.458


def flat_table(n_z=64):
    return np.ones(n_z, dtype=np.float32)


def toy_lambda(H0=70.0, mu=30.0, sigma=3.0, z_max_note=None):
    """Single Gaussian peak, flat rate, Omega_m = 0 (closed-form distances)."""
    return lam_vector(H0=H0, Om=0.0, alpha=2.0, beta=0.0, mmin=2.0, mmax=200.0, delta_m=0.0,
                      mu_low=mu, sigma_low=sigma, mu_high=40.0, sigma_high=5.0,
                      lambda_g=1.0, lambda_low=1.0, gamma=0.0, kappa=0.0, z_p=1.0)


def z_closed_om0(dl, H0):
    """Omega_m = 0: d_L = (c/H0) z (1+z)  =>  z = (sqrt(1 + 4u) - 1)/2."""
    u = dl * H0 / C_KMS
    return 2.0 * u / (1.0 + math.sqrt(1.0 + 4.0 * u))


def toy_event_nodes(x, s, d_i, H0, mmin, n_gh=60, n_gl=2):
    """Quadrature nodes for one toy event.

    PE likelihood: N(x; m1_det, s^2) * delta(d_L - d_i), flat in m2_det.  The
    nodes and weights W satisfy sum_k g(theta_k) W_k ~= int N(m1_det; x, s^2)
    g(m1_det, m2_det, d_i) dm1_det dm2_det, so supplying ln pi_k = -ln W_k
    turns the sum of weights into the event's marginal likelihood.
    """
    t, wt = np.polynomial.hermite_e.hermegauss(n_gh)
    xg, wg = np.polynomial.legendre.leggauss(n_gl)
    z = z_closed_om0(d_i, H0)
    m1, m2, W = [], [], []
    for tk, wk in zip(t, wt):
        m1d = x + s * tk
        a, b = mmin * (1.0 + z), m1d
        if b <= a:              # p1 vanishes below m_min: the node contributes nothing
            continue
        for xl, wl in zip(xg, wg):
            m1.append(m1d)
            m2.append(0.5 * (b - a) * (xl + 1.0) + a)
            W.append(wk / math.sqrt(2 * math.pi) * 0.5 * (b - a) * wl)
    m1, m2, W = map(np.asarray, (m1, m2, W))
    return m1, m2, np.full_like(m1, d_i), -np.log(W)


def toy_event_truth(x, s, d_i, H0, mu, sigma):
    """Closed-form marginal likelihood of the toy event (source-frame integral).

    int N(x; m1 (1+z), s^2) delta(d_L(z) - d_i) N(m1; mu, sigma^2) p2 psi/(1+z) dm1 dm2 dz
    = psi / ((1+z) d_L'(z)) * N(x; mu (1+z), s^2 + sigma^2 (1+z)^2),
    psi = 1/2, d_L'(z) = (c/H0)(1 + 2z) for Omega_m = 0.
    """
    z = z_closed_om0(d_i, H0)
    a = 1.0 + z
    var = s * s + sigma * sigma * a * a
    gauss = math.exp(-0.5 * (x - mu * a) ** 2 / var) / math.sqrt(2 * math.pi * var)
    return 0.5 / (a * (C_KMS / H0) * (1.0 + 2.0 * z)) * gauss


def toy_injection_nodes(H0, mu, sigma, mmin, z_max, n_d=60, n_gh=40, n_gl=2):
    """Detector-frame quadrature nodes whose weights make sum(w) = alpha."""
    d_max = (C_KMS / H0) * z_max * (1.0 + z_max)
    xd, wd = np.polynomial.legendre.leggauss(n_d)
    t, wt = np.polynomial.hermite_e.hermegauss(n_gh)
    xg, wg = np.polynomial.legendre.leggauss(n_gl)
    m1, m2, dl, W = [], [], [], []
    for xdk, wdk in zip(xd, wd):
        d = 0.5 * d_max * (xdk + 1.0)
        Wd = 0.5 * d_max * wdk
        z = z_closed_om0(d, H0)
        mu_d, sg_d = mu * (1.0 + z), sigma * (1.0 + z)
        for tk, wk in zip(t, wt):
            m1d = mu_d + sg_d * tk
            W1 = wk * math.exp(0.5 * tk * tk) * sg_d
            a, b = mmin * (1.0 + z), m1d
            if b <= a:          # p1 vanishes below m_min: no contribution
                continue
            for xl, wl in zip(xg, wg):
                m1.append(m1d)
                m2.append(0.5 * (b - a) * (xl + 1.0) + a)
                dl.append(d)
                W.append(Wd * W1 * 0.5 * (b - a) * wl)
    m1, m2, dl, W = map(np.asarray, (m1, m2, dl, W))
    return m1, m2, dl, -np.log(W)


def make_toy_catalog(events, H0, mu, sigma, mmin=2.0, z_max=2.0, n_pix=3, n_z=64):
    """events: list of (x, s, d_i).  Samples split round-robin over n_pix pixels."""
    epo, pso, m1s, m2s, dls, lps = [0], [0], [], [], [], []
    for (x, s, d) in events:
        m1, m2, dl, lp = toy_event_nodes(x, s, d, H0, mmin)
        pix = np.arange(len(m1)) % n_pix
        order = np.argsort(pix, kind="stable")
        counts = np.bincount(pix, minlength=n_pix)
        m1s.append(m1[order]); m2s.append(m2[order]); dls.append(dl[order]); lps.append(lp[order])
        epo.append(epo[-1] + n_pix)
        pso.extend((pso[-1] + np.cumsum(counts)).tolist())
    im1, im2, idl, ilp = toy_injection_nodes(H0, mu, sigma, mmin, z_max)
    n_pix_tot = len(pso) - 1
    return Catalog(
        event_pix_off=np.asarray(epo, np.int64), pix_samp_off=np.asarray(pso, np.int64),
        pix_los_row=np.zeros(n_pix_tot, np.int32), los=flat_table(n_z)[None, :],
        sky_z=flat_table(n_z), z_max=z_max,
        m1d=np.concatenate(m1s), m2d=np.concatenate(m2s), dl=np.concatenate(dls),
        ln_pi=np.concatenate(lps), inj_m1d=im1, inj_m2d=im2, inj_dl=idl, inj_ln_pdraw=ilp,
        n_draw=1, name="gaussian-toy")


def tiny_catalog(seed=3, n_events=2, n_pix=2, per_pix=4, n_inj=6, n_z=16, z_max=2.0):
    """A few samples with structured LOS tables, for brute-force checks."""
    rng = np.random.default_rng(seed)
    epo = [0]
    pso = [0]
    for e in range(n_events):
        for p in range(n_pix):
            pso.append(pso[-1] + per_pix)
        epo.append(epo[-1] + n_pix)
    n_s = pso[-1]
    m1 = rng.uniform(15, 60, n_s)
    q = rng.uniform(0.35, 0.95, n_s)
    dl = rng.uniform(700, 2500, n_s)
    zg = np.linspace(0, z_max, n_z)
    los = np.stack([1.0 + 0.5 * np.sin(3 * zg + k) for k in range(n_events * n_pix)]).astype(np.float32)
    sky = (1.0 + 0.2 * zg).astype(np.float32)
    im1 = rng.uniform(10, 70, n_inj)
    iq = rng.uniform(0.3, 0.95, n_inj)
    idl = rng.uniform(300, 3000, n_inj)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    return Catalog(
        event_pix_off=np.asarray(epo, np.int64), pix_samp_off=np.asarray(pso, np.int64),
        pix_los_row=np.arange(n_events * n_pix, dtype=np.int32), los=los, sky_z=sky, z_max=z_max,
        m1d=f32(m1), m2d=f32(m1 * q), dl=f32(dl), ln_pi=f32(2 * np.log(dl)),
        inj_m1d=f32(im1), inj_m2d=f32(im1 * iq), inj_dl=f32(idl),
        inj_ln_pdraw=f32(-np.log(im1) * 2 + 2 * np.log(idl) - 20.0), n_draw=50, name="tiny")
