"""FP64 CPU oracle of the dark-siren hierarchical population log-likelihood.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the
benchmark's CPU-baseline leg may import this module; the product path never
does, and this module never imports the GPU path.  It is written to be plain
and slow: every step follows the paper's equations in their order, in float64,
with torch CPU tensors used as vectorised arrays and torch autograd used only
to differentiate the finished definition.

What is computed (paper, Sec. II A "Hierarchical Likelihood"):

* Eq. (1): d_L(z) = (1+z) c/H0 * I(z), I(z) = int_0^z dz'/E(z'),
  E(z) = sqrt(Om (1+z)^3 + 1 - Om) (flat LambdaCDM; I by 32-node
  Gauss-Legendre on [0, z], z(d_L) by bracketed Newton on that d_L);
* Eq. (7): per-sample weights  w = p_pop(z, m1, m2 | Lambda) / pi_PE, the
  population density being expressed in detector-frame variables, so it is
  divided by |d(m1_det, m2_det, d_L) / d(m1, m2, z)| = (1+z)^2 dd_L/dz;
  p_pop = p_LOS,j(z) psi(z)/(1+z) p1(m1) p2(m2|m1), p_LOS,j the pixel's
  redshift prior of Eq. (5);
* Eq. (8): per-pixel effective sample size (sum w)^2 / sum w^2; a pixel
  below the threshold contributes nothing (Sec. II A, after Eq. 8);
* Eq. (5) numerator: event likelihood = (1/N_samples) * sum over passing
  pixels of sum w (a Monte Carlo estimate of the double integral);
* Eq. (4)/(5) denominator: alpha = (1/N_draw) sum over detected injections of
  p_pop(z, m1, m2) with the sky-averaged redshift prior, divided by the same
  Jacobian and by the injection draw density;
* Eq. (3) with the scale-free rate prior of Sec. II A:
  ln L = sum_i ln L_i - N_det ln alpha.

Readings where the paper is silent:
* MultiPeak (power law + two Gaussian peaks + low-mass smoothing, cited in
  Appendix A): p1(m1) = S(m1) [(1-lg) P(m1) + lg ll N_T(m1; mu_l, s_l)
  + lg (1-ll) N_T(m1; mu_h, s_h)] on [mmin, mmax]; P the normalised power law
  m^-alpha, N_T Gaussians truncated to [mmin, mmax];
  S(m) = 1 / (1 + exp(dm/m' + dm/(m'-dm))), m' = m - mmin, 0 below mmin and 1
  above mmin + dm; p2(m2|m1) = m2^beta S(m2) / Z(m1) on [mmin, m1] with
  Z(m1) = int_mmin^m1 m^beta S(m) dm.  The global renormalisation of p1 after
  smoothing is a Lambda-only factor and cancels between numerator and
  alpha^N_det, so it is left out;
* Madau-Dickinson rate (cited in Appendix A): psi(z) = (1+z)^gamma /
  (1 + ((1+z)/(1+z_p))^(gamma+kappa)) without its constant prefactor;
* p_LOS,j: linear interpolation of the pixel's table on uniform nodes over
  [0, z_max], zero outside; samples with d_L > d_L(z_max) have zero weight;
* ties at the N_eff threshold pass; a pixel with no non-zero weight fails.
* spectral-siren mode (the paper's O5 mock analysis runs without a galaxy
  catalogue, Sec. III B): the redshift prior of every sample and injection is
  the comoving-volume shape dV_c/dz ∝ I(z)^2 / E(z) for the point's Omega_m
  instead of a table; its (c/H0)^3 factor and normalisation are Lambda-only
  and cancel between the events and alpha^N_det.

The paper's own numerator (loglike_kde; Eq. 6 inside Eq. 5, bandwidth rules of
Appendix D) replaces the per-sample sum of a pixel by the integral over a
redshift grid of a weighted Gaussian KDE of the samples' redshifts times the
pixel's redshift prior and psi(z)/(1+z).  Readings: the Eq. (7) weights of this
form carry the mass model, the Jacobian and the PE prior (the redshift prior
and the rate act on the grid, as the paper's per-component timing lists them);
the bandwidths use the unweighted in-support redshifts of the pixel (the
printed rules are unweighted), n their number, the sample standard deviation
with n - 1, quantiles by linear interpolation, the biweight scale as the
square root of the printed midvariance inside Scott's form; the grid is
KDE_GRID uniform nodes from max(0, min z - 5h) to min(z_max, max z + 5h)
integrated by the trapezoid rule; a zero bandwidth (one sample, equal
redshifts, zero MAD) takes the point-mass limit; Eq. (8) gates with the same
weights.

Parity status: the functional forms of the mass and rate models are readings
of cited, unprinted models, so agreement with the paper's own code is
"parity unpinned"; every function below is pinned by the tests in
tests/test_oracle_*.py against closed forms, library routines, brute-force
high-precision quadrature and a Gaussian toy likelihood.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

C_KMS = 299792.458
LN2 = math.log(2.0)
DT = torch.float64

_GL32 = np.polynomial.legendre.leggauss(32)
_GL64 = np.polynomial.legendre.leggauss(64)
GL32_X = torch.tensor(_GL32[0], dtype=DT)
GL32_W = torch.tensor(_GL32[1], dtype=DT)
GL64_X = torch.tensor(_GL64[0], dtype=DT)
GL64_W = torch.tensor(_GL64[1], dtype=DT)

FLAG_INVALID_LAMBDA = 1
FLAG_EVENT_NO_PIXEL = 2
FLAG_ALPHA_ZERO = 4
FLAG_NONFINITE = 8


# ---------------------------------------------------------------------------
# Hyperparameters
# ---------------------------------------------------------------------------
@dataclass
class Lam:
    H0: torch.Tensor
    Om: torch.Tensor
    alpha: torch.Tensor
    beta: torch.Tensor
    mmin: torch.Tensor
    mmax: torch.Tensor
    delta_m: torch.Tensor
    mu_low: torch.Tensor
    sigma_low: torch.Tensor
    mu_high: torch.Tensor
    sigma_high: torch.Tensor
    lambda_g: torch.Tensor
    lambda_low: torch.Tensor
    gamma: torch.Tensor
    kappa: torch.Tensor
    z_p: torch.Tensor

    @staticmethod
    def of(v: torch.Tensor) -> "Lam":
        return Lam(*[v[i] for i in range(16)])


def lambda_is_valid(lam) -> bool:
    """Domain of the model (flags bit 0 when violated)."""
    v = [float(x) for x in np.asarray(lam, dtype=np.float64)]
    H0, Om, alpha, beta, mmin, mmax, dm, mul, sl, muh, sh, lg, ll, gam, kap, zp = v
    if not all(math.isfinite(x) for x in v):
        return False
    return (H0 > 0 and 0.0 <= Om <= 1.0 and mmin > 0 and mmin < mmax and dm >= 0
            and sl > 0 and sh > 0 and 0.0 <= lg <= 1.0 and 0.0 <= ll <= 1.0 and zp > -1.0)


# ---------------------------------------------------------------------------
# Eq. (1): flat LambdaCDM distances
# ---------------------------------------------------------------------------
def E_of_z(z, Om):
    return torch.sqrt(Om * (1.0 + z) ** 3 + (1.0 - Om))


def comoving_integral(z, Om):
    """I(z) = int_0^z dz'/E(z'), 32-node Gauss-Legendre on [0, z]."""
    zz = z.unsqueeze(-1)
    t = 0.5 * zz * (GL32_X + 1.0)
    return 0.5 * z * (GL32_W / E_of_z(t, Om)).sum(-1)


def dl_of_z(z, H0, Om):
    """Luminosity distance in Mpc (Eq. 1)."""
    return (C_KMS / H0) * (1.0 + z) * comoving_integral(z, Om)


def ddl_dz(z, H0, Om):
    """d d_L / dz = (c/H0) [I(z) + (1+z)/E(z)]."""
    return (C_KMS / H0) * (comoving_integral(z, Om) + (1.0 + z) / E_of_z(z, Om))


def _solve_z(u, Om, z_max, iters=60):
    """Root of (1+z) I(z) = u on [0, z_max] (no autograd), bracketed Newton.

    The result is checked: |(1+z) I(z) - u| <= 1e-14 u for every element.
    """
    with torch.no_grad():
        Om = Om.detach() if torch.is_tensor(Om) else torch.tensor(Om, dtype=DT)
        lo = torch.zeros_like(u)
        hi = torch.full_like(u, z_max)
        z = torch.clamp(0.5 * (torch.sqrt(1.0 + 4.0 * u) - 1.0), 0.0, z_max)
        for _ in range(iters):
            I = comoving_integral(z, Om)
            E = E_of_z(z, Om)
            f = (1.0 + z) * I - u
            lo = torch.where(f <= 0, z, lo)
            hi = torch.where(f > 0, z, hi)
            zn = z - f / (I + (1.0 + z) / E)
            bad = (zn < lo) | (zn > hi) | ~torch.isfinite(zn)
            zn = torch.where(bad, 0.5 * (lo + hi), zn)
            step = torch.abs(zn - z)
            z = zn
            if bool((step <= 2e-15 * torch.clamp(z, min=1e-300)).all()):
                break
        res = torch.abs((1.0 + z) * comoving_integral(z, Om) - u)
        if u.numel():
            assert bool((res <= 1e-14 * torch.clamp(u, min=1e-300) + 1e-300).all()), float(res.max())
        return z


def z_of_dl(dl, H0, Om, z_max):
    """Redshift of each luminosity distance (Eq. 1 inverted) and its support.

    Returns (z, inside): z carries the exact first derivatives with respect to
    H0 and Om (implicit-function step around the detached root); inside is
    False where d_L > d_L(z_max).
    """
    u = dl * H0 / C_KMS                      # (1+z) I(z) = d_L H0 / c
    umax = (1.0 + z_max) * comoving_integral(torch.tensor(z_max, dtype=DT), Om.detach())
    inside = (u.detach() <= umax) & (u.detach() >= 0)
    u_safe = torch.where(inside, u, torch.zeros_like(u))
    z0 = _solve_z(u_safe.detach(), Om, z_max)
    D0 = (1.0 + z0) * comoving_integral(z0, Om)
    Dp0 = (comoving_integral(z0, Om) + (1.0 + z0) / E_of_z(z0, Om)).detach()
    z = z0 - (D0 - u_safe) / Dp0
    return z, inside


# ---------------------------------------------------------------------------
# Mass model (MultiPeak reading)
# ---------------------------------------------------------------------------
def log_smoothing(m, mmin, dm):
    """ln S(m): 0 above mmin+dm, -inf at or below mmin, logistic window between."""
    mp = m - mmin
    if float(torch.as_tensor(dm).detach()) <= 0.0:
        return torch.where(mp > 0, torch.zeros_like(m), torch.full_like(m, -math.inf))
    inside = (mp > 0) & (mp < dm)
    x = torch.where(inside, mp, 0.5 * dm + torch.zeros_like(mp))
    y = dm / x + dm / (x - dm)
    val = -torch.nn.functional.softplus(y)
    out = torch.where(inside, val, torch.zeros_like(val))
    return torch.where(mp <= 0, torch.full_like(out, -math.inf), out)


def log_powerlaw_norm(alpha, mmin, mmax):
    """ln of the normalisation of m^-alpha on [mmin, mmax]."""
    if abs(float(alpha.detach()) - 1.0) < 1e-12:
        return -torch.log(torch.log(mmax / mmin))
    a1 = 1.0 - alpha
    return torch.log(torch.abs(a1)) - torch.log(torch.abs(mmax ** a1 - mmin ** a1))


def log_truncnorm_norm(mu, sigma, mmin, mmax):
    """ln of 1 / (sigma sqrt(2 pi) [Phi(b) - Phi(a)])."""
    a = (mmin - mu) / sigma
    b = (mmax - mu) / sigma
    mass = torch.special.ndtr(b) - torch.special.ndtr(a)
    return -torch.log(sigma * math.sqrt(2 * math.pi)) - torch.log(mass)


def log_p1(m1, L: Lam):
    """ln p1(m1): smoothed power law + two truncated Gaussian peaks."""
    inside = (m1 <= L.mmax) & (m1 > L.mmin)
    ms = torch.where(inside, m1, 0.5 * (L.mmin + L.mmax) + torch.zeros_like(m1))
    lP = log_powerlaw_norm(L.alpha, L.mmin, L.mmax) - L.alpha * torch.log(ms)
    lNl = log_truncnorm_norm(L.mu_low, L.sigma_low, L.mmin, L.mmax) - 0.5 * ((ms - L.mu_low) / L.sigma_low) ** 2
    lNh = log_truncnorm_norm(L.mu_high, L.sigma_high, L.mmin, L.mmax) - 0.5 * ((ms - L.mu_high) / L.sigma_high) ** 2
    comps = torch.stack([torch.log(1.0 - L.lambda_g) + lP,
                         torch.log(L.lambda_g * L.lambda_low) + lNl,
                         torch.log(L.lambda_g * (1.0 - L.lambda_low)) + lNh], 0)
    lmix = torch.logsumexp(comps, 0)
    val = log_smoothing(ms, L.mmin, L.delta_m) + lmix
    return torch.where(inside, val, torch.full_like(val, -math.inf))


def _window_integral(upper, L: Lam):
    """int_mmin^upper m^beta S(m) dm for upper in [mmin, mmin+dm], 64-node GL."""
    t = 0.5 * (upper - L.mmin).unsqueeze(-1) * (GL64_X + 1.0) + L.mmin
    f = torch.exp(L.beta * torch.log(t) + log_smoothing(t, L.mmin, L.delta_m))
    return 0.5 * (upper - L.mmin) * (GL64_W * f).sum(-1)


def log_Z(m1, L: Lam):
    """ln Z(m1) = ln int_mmin^m1 m^beta S(m) dm (conditional-mass normaliser)."""
    s = L.beta + 1.0
    M = L.mmin + L.delta_m
    if float(L.delta_m.detach()) > 0.0:
        Zw = _window_integral(M.reshape(1), L)[0]
    else:
        # Zero width: the window integral is mmin^beta * delta_m / 2 to first
        # order (S(mmin + t dm) + S(mmin + (1-t) dm) = 1, so the window's mean
        # over its width is 1/2).  Its value here is 0; the first-order term
        # makes the derivative with respect to delta_m at the edge delta_m = 0
        # of its domain the one-sided limit from delta_m > 0.
        Zw = 0.5 * L.mmin ** L.beta * L.delta_m
    in_win = m1 < M
    up = torch.where(in_win, torch.clamp(m1, min=float(L.mmin.detach())), M + torch.zeros_like(m1))
    if float(L.delta_m.detach()) > 0.0:
        Zin = _window_integral(torch.where(in_win, up, L.mmin + 0.5 * L.delta_m + torch.zeros_like(up)), L)
    else:
        Zin = torch.zeros_like(m1)
    ma = torch.where(in_win, M + 1.0 + torch.zeros_like(m1), m1)
    if abs(float(s.detach())) < 1e-12:
        tail = torch.log(ma / M)
    else:
        tail = (ma ** s - M ** s) / s
    Z = torch.where(in_win, Zin, Zw + tail)
    return torch.log(Z)


def log_p2(m2, m1, L: Lam):
    """ln p2(m2 | m1) = beta ln m2 + ln S(m2) - ln Z(m1), support mmin < m2 <= m1."""
    ok = (m2 <= m1) & (m2 > L.mmin) & (m1 > L.mmin)
    m2s = torch.where(ok, m2, L.mmin + 1.0 + torch.zeros_like(m2))
    m1s = torch.where(ok, m1, L.mmin + 1.0 + torch.zeros_like(m1))
    val = L.beta * torch.log(m2s) + log_smoothing(m2s, L.mmin, L.delta_m) - log_Z(m1s, L)
    return torch.where(ok, val, torch.full_like(val, -math.inf))


# ---------------------------------------------------------------------------
# Redshift model
# ---------------------------------------------------------------------------
def log_psi(z, L: Lam):
    """ln psi(z) = gamma ln(1+z) - ln(1 + ((1+z)/(1+z_p))^(gamma+kappa))."""
    lz = torch.log1p(z)
    return L.gamma * lz - torch.nn.functional.softplus((L.gamma + L.kappa) * (lz - torch.log1p(L.z_p)))


def los_interp(tables, rows, z, z_max):
    """Linear interpolation of tables[rows] at z on uniform nodes over [0, z_max]."""
    n_z = tables.shape[1]
    dz = z_max / (n_z - 1)
    inside = (z >= 0) & (z <= z_max)
    x = torch.where(inside, z, torch.zeros_like(z)) / dz
    k = torch.clamp(torch.floor(x.detach()).to(torch.int64), 0, n_z - 2)
    f = x - k.to(DT)
    v0 = tables[rows, k]
    v1 = tables[rows, k + 1]
    val = v0 + f * (v1 - v0)
    return torch.where(inside, val, torch.zeros_like(val))


# ---------------------------------------------------------------------------
# Eq. (7): per-sample log weights
# ---------------------------------------------------------------------------
def log_weights(m1d, m2d, dl, ln_prior, tables, rows, z_max, L: Lam, margins=None, z_prior="los"):
    """ln w for detector-frame samples; -inf outside the model's support.

    ln_prior is ln pi_PE for posterior samples or ln p_draw for injections;
    tables[rows] is each sample's redshift prior (pixel table, or sky table),
    or, with z_prior="comoving", the comoving-volume shape I(z)^2 / E(z).
    """
    z, in_z = z_of_dl(dl, L.H0, L.Om, z_max)
    zs = torch.where(in_z, z, torch.full_like(z, 0.5 * z_max))
    opz = 1.0 + zs
    m1 = m1d / opz
    m2 = m2d / opz
    if z_prior == "comoving":
        los = comoving_integral(zs, L.Om) ** 2 / E_of_z(zs, L.Om)
    else:
        los = los_interp(tables, rows, zs, z_max)
    los_ok = los > 0
    l_los = torch.log(torch.where(los_ok, los, torch.ones_like(los)))
    l_rate = log_psi(zs, L) - torch.log(opz)
    l_mass = log_p1(m1, L) + log_p2(m2, m1, L)
    l_jac = 2.0 * torch.log(opz) + torch.log(ddl_dz(zs, L.H0, L.Om))
    lw = l_los + l_rate + l_mass - l_jac - ln_prior
    ok = in_z & los_ok & torch.isfinite(l_mass)
    if margins is not None:
        with torch.no_grad():
            u = dl * L.H0 / C_KMS
            umax = (1.0 + z_max) * comoving_integral(torch.tensor(z_max, dtype=DT), L.Om)
            r = torch.abs(u / umax - 1.0)
            r = torch.minimum(r, torch.abs(m1 / L.mmax - 1.0))
            if float(L.delta_m.detach()) == 0.0:
                r = torch.minimum(r, torch.abs(m2 / L.mmin - 1.0))
            margins.append(r)
    return torch.where(ok, lw, torch.full_like(lw, -math.inf))


# ---------------------------------------------------------------------------
# Eq. (8) and the reductions of Eq. (5)
# ---------------------------------------------------------------------------
def segment_lse(x, seg, n_seg):
    """log sum exp of x over segments (seg = segment id of each element)."""
    with torch.no_grad():
        mx = torch.full((n_seg,), -math.inf, dtype=DT).scatter_reduce(0, seg, x.detach(), "amax")
        mx = torch.where(torch.isfinite(mx), mx, torch.zeros_like(mx))
    s = torch.zeros(n_seg, dtype=DT).index_add(0, seg, torch.exp(x - mx[seg]))
    return torch.log(s) + mx


def lse_all(x):
    if x.numel() == 0:
        return torch.tensor(-math.inf, dtype=DT)
    return torch.logsumexp(x, 0)


@dataclass
class Options:
    neff_min: float = 2.0
    gate_mode: int = 0          # 0: per-pixel gate; 1: also per-event gate; 2: none
    z_prior: str = "los"        # "los" (pixel tables) or "comoving" (spectral sirens)
    gate_flip: Optional[np.ndarray] = None   # sorted pixel ids whose gate decision is inverted


def _block_tables(cat, pix):
    """The LOS rows of a block's pixels in float64, and each pixel's row in it
    (only the block's rows are converted, so the catalogue is streamed)."""
    uniq, inv = np.unique(np.asarray(cat.pix_los_row)[pix], return_inverse=True)
    return torch.from_numpy(np.asarray(cat.los[uniq], dtype=np.float64)), inv.astype(np.int64)


def _event_terms(cat, ev_ids, L: Lam, opt: Options, margin_out=None):
    """ln L_i, N_eff,i, pixel gate margins for a block of events."""
    p_lo = cat.event_pix_off[ev_ids]
    p_hi = cat.event_pix_off[ev_ids + 1]
    pix = np.concatenate([np.arange(a, b) for a, b in zip(p_lo, p_hi)]) if len(ev_ids) else np.zeros(0, np.int64)
    ev_of_pix = np.repeat(np.arange(len(ev_ids)), p_hi - p_lo)
    s_lo = cat.pix_samp_off[pix]
    s_hi = cat.pix_samp_off[pix + 1]
    samp = np.concatenate([np.arange(a, b) for a, b in zip(s_lo, s_hi)]) if len(pix) else np.zeros(0, np.int64)
    pix_of_samp = np.repeat(np.arange(len(pix)), s_hi - s_lo)
    tables, prow = _block_tables(cat, pix)
    rows = torch.from_numpy(prow)[torch.from_numpy(pix_of_samp)]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a[samp], dtype=np.float64))
    margins = [] if margin_out is not None else None
    m1d, m2d, dl = t(cat.m1d), t(cat.m2d), t(cat.dl)
    lw = log_weights(m1d, m2d, dl, t(cat.ln_pi), tables, rows, cat.z_max, L, margins, z_prior=opt.z_prior)
    if margin_out is not None:
        # each sample's ln w under a perturbation of its inputs at FP32 reach:
        # eps_dl = 3.2e-7 of d_L (FP32 redshifts are within 3.2e-7 of the FP64
        # ones), 6e-8 of each mass (FP32 rounding); first order in the inputs
        with torch.enable_grad():
            xs = [v.detach().clone().requires_grad_(True) for v in (m1d, m2d, dl)]
            L0 = Lam(*[getattr(L, f).detach() for f in L.__dataclass_fields__])
            lw2 = log_weights(*xs, t(cat.ln_pi), tables, rows, cat.z_max, L0, z_prior=opt.z_prior)
            ok2 = torch.isfinite(lw2)
            gr = torch.autograd.grad(torch.where(ok2, lw2, torch.zeros_like(lw2)).sum(), xs)
        cond = (3.2e-7 * torch.abs(dl * gr[2]) + 6e-8 * (torch.abs(m1d * gr[0]) + torch.abs(m2d * gr[1]))).detach()
        cond = torch.where(ok2, cond, torch.zeros_like(cond))
    seg = torch.from_numpy(pix_of_samp)
    n_p = len(pix)
    lS1 = segment_lse(lw, seg, n_p)
    lS2 = segment_lse(2.0 * lw, seg, n_p)
    lneff = 2.0 * lS1 - lS2
    finite = torch.isfinite(lS1)
    log_nmin = math.log(opt.neff_min) if opt.neff_min > 0 else -math.inf
    if opt.gate_mode == 2:
        passing = finite
    else:
        passing = finite & (lneff.detach() >= log_nmin)
        if opt.gate_flip is not None and len(opt.gate_flip):
            # the other outcome of the Eq. (8) test for the listed pixels: the
            # decisions a path in another precision may take near the threshold
            flip = torch.from_numpy(np.isin(pix, opt.gate_flip))
            passing = torch.where(flip, finite & ~passing, passing)
    ev_seg = torch.from_numpy(ev_of_pix)
    neg = torch.full_like(lS1, -math.inf)
    lS1p = torch.where(passing, lS1, neg)
    lS2p = torch.where(passing, lS2, neg)
    nE = len(ev_ids)
    # Segment LSE over passing pixels (pixels with -inf drop out).
    lE1 = segment_lse(lS1p, ev_seg, nE) if n_p else torch.full((nE,), -math.inf, dtype=DT)
    lE2 = segment_lse(lS2p, ev_seg, nE) if n_p else torch.full((nE,), -math.inf, dtype=DT)
    n_s = torch.from_numpy((s_hi - s_lo).astype(np.float64))
    ns_ev = torch.zeros(nE, dtype=DT).index_add(0, ev_seg, n_s) if n_p else torch.zeros(nE, dtype=DT)
    # An event without samples has an empty sum: L_i = 0 (the 1/N_s,i of Eq. 5
    # is read as 1/max(N_s,i, 1), as in loglike_kde).
    lnL = lE1 - torch.log(torch.clamp(ns_ev, min=1.0))
    neff_ev = torch.exp(2.0 * lE1.detach() - lE2.detach())
    neff_ev = torch.where(torch.isfinite(lE1.detach()), neff_ev, torch.zeros_like(neff_ev))
    if opt.gate_mode == 1:
        lnL = torch.where(neff_ev >= opt.neff_min, lnL, torch.full_like(lnL, -math.inf))
    if margin_out is not None:
        with torch.no_grad():
            gm = torch.abs(lneff - log_nmin)
            gm = torch.where(torch.isfinite(gm), gm, torch.full_like(gm, math.inf))
            ev_gate = torch.full((nE,), math.inf, dtype=DT).scatter_reduce(0, ev_seg, gm, "amin")
            sm = margins[0] if margins else torch.zeros(0, dtype=DT)
            smp = torch.full((n_p,), math.inf, dtype=DT).scatter_reduce(0, seg, sm, "amin")
            ev_samp = torch.full((nE,), math.inf, dtype=DT).scatter_reduce(0, ev_seg, smp, "amin")
            # per event: the weight-averaged sensitivity over its passing pixels
            wk = torch.exp(lw.detach() - lE1.detach()[ev_seg][seg])
            use = passing[seg] & torch.isfinite(wk)
            ev_cond = torch.zeros(nE, dtype=DT).index_add(0, ev_seg[seg], torch.where(use, wk * cond, torch.zeros_like(cond)))
            # and of ln N_eff,i = 2 ln S1 - ln S2: d ln N_eff / d ln w_k = 2 w_k/S1 - 2 w_k^2/S2
            wk2 = torch.exp(2.0 * lw.detach() - lE2.detach()[ev_seg][seg])
            ncond = torch.abs(2.0 * wk - 2.0 * wk2) * cond
            ev_ncond = torch.zeros(nE, dtype=DT).index_add(0, ev_seg[seg], torch.where(use, ncond, torch.zeros_like(cond)))
            margin_out.append((ev_gate.numpy(), ev_samp.numpy(), pix, gm.numpy(), ev_cond.numpy(), ev_ncond.numpy()))
    return lnL, neff_ev


def _selection_chunk(cat, sl, L: Lam, sky, margin_out=None, z_prior="los"):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a[sl], dtype=np.float64))
    n = sl.stop - sl.start
    rows = torch.zeros(n, dtype=torch.int64)
    margins = [] if margin_out is not None else None
    lw = log_weights(t(cat.inj_m1d), t(cat.inj_m2d), t(cat.inj_dl), t(cat.inj_ln_pdraw),
                     sky, rows, cat.z_max, L, margins, z_prior=z_prior)
    if margin_out is not None:
        margin_out.append(float(margins[0].min()) if n else math.inf)
    return lse_all(lw), lse_all(2.0 * lw)


def loglike(cat, lam, neff_min: float = 2.0, gate_mode: int = 0, grad: bool = False,
            event_block: int = 64, inj_chunk: int = 1 << 20, margins: bool = False, z_prior: str = "los",
            gate_flip=None):
    """Oracle log-likelihood of one hyperparameter point.

    Returns a dict with logL, logL_event[n_events], neff_event[n_events],
    neff_sel, flags and, when grad=True, grad[16] = d logL / d Lambda.  With
    margins=True it also reports, per event, the smallest |ln N_eff - ln N_min|
    over its pixels and the smallest relative distance of a sample to a
    support edge (d_L(z_max), m_max), for parity tests that must allow for
    decisions taken in another precision, and pixel_gate_margin[n_pix], that
    distance for every pixel (inf for a pixel without weight).  gate_flip (pixel
    ids) inverts the gate decision of those pixels, so such a test can evaluate
    the other outcome.  event_fp32_cond[n_events] bounds, to first order, how
    far ln L_i moves when every sample's d_L is perturbed by 3.2e-7 and its
    masses by 6e-8 (relative): the reach of an FP32 evaluation of the inputs;
    event_fp32_cond_neff[n_events] bounds the relative change of N_eff,i alike.
    """
    lam_np = np.asarray(lam, dtype=np.float64).reshape(16)
    nE = cat.n_events
    out = dict(logL=-math.inf, logL_event=np.full(nE, -math.inf), neff_event=np.zeros(nE),
               neff_sel=0.0, flags=0, grad=np.zeros(16))
    if not lambda_is_valid(lam_np):
        out["flags"] = FLAG_INVALID_LAMBDA
        return out
    flips = None if gate_flip is None else np.unique(np.asarray(gate_flip, dtype=np.int64))
    opt = Options(neff_min=neff_min, gate_mode=gate_mode, z_prior=z_prior, gate_flip=flips)
    lam_t = torch.tensor(lam_np, dtype=DT, requires_grad=grad)
    L = Lam.of(lam_t)
    sky = torch.from_numpy(np.asarray(cat.sky_z, dtype=np.float64)).reshape(1, -1)
    g_ev = torch.zeros(16, dtype=DT)
    lnL_ev = np.empty(nE)
    neff_ev = np.empty(nE)
    gate_m = np.empty(nE)
    samp_m = np.empty(nE)
    pix_m = np.full(cat.n_pix, math.inf) if margins else None
    ev_cond = np.zeros(nE)
    ev_ncond = np.zeros(nE)
    for b0 in range(0, nE, event_block):
        ids = np.arange(b0, min(nE, b0 + event_block))
        mo = [] if margins else None
        with torch.set_grad_enabled(grad):
            lnL_b, neff_b = _event_terms(cat, ids, L, opt, mo)
            if grad and torch.isfinite(lnL_b).all():
                g_ev += torch.autograd.grad(lnL_b.sum(), lam_t)[0]
        lnL_ev[ids] = lnL_b.detach().numpy()
        neff_ev[ids] = neff_b.numpy()
        if margins:
            gate_m[ids], samp_m[ids], pix_b, pm_b, ev_cond[ids], ev_ncond[ids] = mo[0]
            pix_m[pix_b] = pm_b
    # Selection term: alpha = (1/N_draw) sum_n w_n, merged over chunks.
    lc1, lc2, gc = [], [], []
    inj_margin = math.inf
    for c0 in range(0, cat.n_inj, inj_chunk):
        sl = slice(c0, min(cat.n_inj, c0 + inj_chunk))
        mo = [] if margins else None
        with torch.set_grad_enabled(grad):
            l1, l2 = _selection_chunk(cat, sl, L, sky, mo, z_prior=z_prior)
            if grad and torch.isfinite(l1):
                gc.append(torch.autograd.grad(l1, lam_t)[0])
            elif grad:
                gc.append(torch.zeros(16, dtype=DT))
        lc1.append(float(l1.detach()))
        lc2.append(float(l2.detach()))
        if margins:
            inj_margin = min(inj_margin, mo[0])
    l1 = torch.logsumexp(torch.tensor(lc1, dtype=DT), 0) if lc1 else torch.tensor(-math.inf, dtype=DT)
    l2 = torch.logsumexp(torch.tensor(lc2, dtype=DT), 0) if lc2 else torch.tensor(-math.inf, dtype=DT)
    ln_alpha = float(l1) - math.log(cat.n_draw)
    neff_sel = math.exp(2 * float(l1) - float(l2)) if math.isfinite(float(l1)) else 0.0
    flags = 0
    if not np.all(np.isfinite(lnL_ev)):
        flags |= FLAG_EVENT_NO_PIXEL
    if not math.isfinite(ln_alpha):
        flags |= FLAG_ALPHA_ZERO
    total = float(np.sum(lnL_ev)) - nE * ln_alpha if flags == 0 else -math.inf
    if flags == 0 and not math.isfinite(total):
        flags |= FLAG_NONFINITE
        total = -math.inf
    out.update(logL=total, logL_event=lnL_ev, neff_event=neff_ev, neff_sel=neff_sel, flags=flags,
               ln_alpha=ln_alpha)
    if grad and flags == 0:
        wts = torch.softmax(torch.tensor(lc1, dtype=DT), 0)
        g_sel = sum(w * g for w, g in zip(wts, gc))
        out["grad"] = (g_ev - nE * g_sel).numpy()
    if margins:
        out["gate_margin"] = gate_m
        out["sample_margin"] = samp_m
        out["inj_margin"] = inj_margin
        out["pixel_gate_margin"] = pix_m
        out["event_fp32_cond"] = ev_cond
        out["event_fp32_cond_neff"] = ev_ncond
    return out


# ---------------------------------------------------------------------------
# The paper's KDE numerator (Eq. 6 inside Eq. 5; bandwidths of Appendix D)
# ---------------------------------------------------------------------------
KDE_GRID = 256     # fiducial resolution of the redshift grid (Sec. III C)
KDE_TAU = 5.0      # the grid reaches this many bandwidths beyond the outermost sample


def kde_log_weights(m1d, m2d, dl, ln_prior, z_max, L: Lam):
    """Eq. (7) weights of the KDE form: the mass population over the PE prior
    expressed in (m1, m2, z), i.e. divided by the Jacobian (1+z)^2 dd_L/dz.
    The redshift prior and the rate enter on the grid.  Returns (z, inside, ln w)
    with ln w = -inf outside the mass support."""
    z, in_z = z_of_dl(dl, L.H0, L.Om, z_max)
    zs = torch.where(in_z, z, torch.full_like(z, 0.5 * z_max))
    opz = 1.0 + zs
    m1 = m1d / opz
    m2 = m2d / opz
    l_mass = log_p1(m1, L) + log_p2(m2, m1, L)
    l_jac = 2.0 * torch.log(opz) + torch.log(ddl_dz(zs, L.H0, L.Om))
    lw = l_mass - l_jac - ln_prior
    ok = in_z & torch.isfinite(l_mass)
    return zs, in_z, torch.where(ok, lw, torch.full_like(lw, -math.inf))


def _sorted(z):
    return torch.sort(z).values


def median(z):
    """Median with the average of the two middle values for even n."""
    s = _sorted(z)
    n = s.numel()
    return 0.5 * (s[(n - 1) // 2] + s[n // 2])


def quantile_linear(z, p):
    """Quantile at probability p by linear interpolation between order
    statistics at position p (n - 1)."""
    s = _sorted(z)
    n = s.numel()
    pos = p * (n - 1)
    a = min(int(math.floor(pos)), n - 1)
    b = min(a + 1, n - 1)
    f = pos - a
    return s[a] + f * (s[b] - s[a])


def sample_std(z):
    """Sample standard deviation (n - 1 in the denominator), computed about
    the first value so that equal values give exactly 0."""
    d = z - z[0].detach()
    d = d - torch.mean(d)
    return torch.sqrt(torch.sum(d * d) / (z.numel() - 1))


def bw_scott(z):
    """Appendix D, Scott's rule: h = 1.06 sigma n^(-1/5), sigma the sample
    standard deviation."""
    n = z.numel()
    if n < 2:
        return torch.zeros((), dtype=DT)
    return 1.06 * sample_std(z) * n ** -0.2


def bw_silverman(z):
    """Appendix D, Silverman's rule: h = 0.9 min(sigma, IQR/1.34) n^(-1/5)."""
    n = z.numel()
    if n < 2:
        return torch.zeros((), dtype=DT)
    iqr = quantile_linear(z, 0.75) - quantile_linear(z, 0.25)
    return 0.9 * torch.minimum(sample_std(z), iqr / 1.34) * n ** -0.2


def biweight_midvariance(z):
    """Appendix D, biweight midvariance about the median Q with u scaled by
    9 MAD; 0 when the MAD is 0."""
    n = z.numel()
    if n < 2:
        return torch.zeros((), dtype=DT)
    Q = median(z)
    mad = median(torch.abs(z - Q))
    if float(mad) == 0.0:
        return torch.zeros((), dtype=DT)
    u = (z - Q) / (9.0 * mad)
    inside = torch.abs(u.detach()) < 1.0
    d = torch.where(inside, z - Q, torch.zeros_like(z))
    uu = torch.where(inside, u * u, torch.zeros_like(u))
    num = n * torch.sum(d * d * (1.0 - uu) ** 4)
    den = torch.sum(torch.where(inside, (1.0 - uu) * (1.0 - 5.0 * uu), torch.zeros_like(uu))) ** 2
    return num / den


def bw_biweight(z):
    """Bandwidth from the biweight scale: Scott's form with sigma replaced by
    the square root of the biweight midvariance (Appendix D prints the
    midvariance itself, a squared scale)."""
    n = z.numel()
    v = biweight_midvariance(z)
    if float(v) <= 0.0:
        return torch.zeros((), dtype=DT)
    return 1.06 * torch.sqrt(v) * n ** -0.2


BANDWIDTHS = {"scott": bw_scott, "silverman": bw_silverman, "biweight": bw_biweight}


def kde_grid(z, h, z_max, n_grid=KDE_GRID, tau=KDE_TAU):
    """n_grid uniform nodes from max(0, min z - tau h) to min(z_max, max z + tau h)."""
    a = torch.clamp(torch.min(z) - tau * h, min=0.0)
    b = torch.clamp(torch.max(z) + tau * h, max=z_max)
    g = torch.arange(n_grid, dtype=DT) / (n_grid - 1)
    return a + g * (b - a)


def kde_pixel_integral(z, w, h, grid, v):
    """Trapezoid rule over the grid of f(z_g) v_g with the weighted Gaussian
    KDE f(z) = sum_k w_k N(z; z_k, h^2) (Eq. 6)."""
    x = (grid[:, None] - z[None, :]) / h
    K = torch.exp(-0.5 * x * x) / (h * math.sqrt(2.0 * math.pi))
    y = (K @ w) * v
    dz = grid[1] - grid[0]
    return dz * (torch.sum(y) - 0.5 * (y[0] + y[-1]))


def _pixel_kde_term(z, lw, h, table, z_max, L: Lam, n_grid):
    """ln of the pixel's integral of KDE x redshift prior x psi(z)/(1+z)."""
    mx = torch.max(lw.detach())
    w = torch.exp(lw - mx)
    if float(h) > 0.0:
        grid = kde_grid(z, h, z_max, n_grid)
        v = los_interp(table, torch.zeros(n_grid, dtype=torch.int64), grid, z_max) * \
            torch.exp(log_psi(grid, L) - torch.log1p(grid))
        T = kde_pixel_integral(z, w, h, grid, v)
    else:   # zero bandwidth: the kernel is a point mass at each sample
        v = los_interp(table, torch.zeros(z.numel(), dtype=torch.int64), z, z_max) * \
            torch.exp(log_psi(z, L) - torch.log1p(z))
        T = torch.sum(w * v)
    if float(T) <= 0.0:
        return torch.tensor(-math.inf, dtype=DT)
    return torch.log(T) + mx


def loglike_kde(cat, lam, bandwidth: str = "scott", n_grid: int = KDE_GRID, neff_min: float = 2.0,
                gate_mode: int = 0, grad: bool = False, margins: bool = False, gate_flip=None):
    """Oracle log-likelihood with the paper's KDE numerator.

    For every pixel j of event i: the in-support samples (d_L <= d_L(z_max))
    with their Eq. (7) weights w_k (kde_log_weights) form the KDE of Eq. (6)
    with the pixel's bandwidth h_j (Appendix D, from the samples' redshifts);
    T_j = integral over the grid of KDE(z) p_LOS,j(z) psi(z)/(1+z) (trapezoid
    rule on kde_grid); the pixel passes Eq. (8) on the same weights; and
    L_i = (1/N_s,i) sum_pass T_j.  The selection term is the Monte Carlo sum
    over injections, exactly as in loglike.  Pure-Python loop over pixels.
    margins and gate_flip as in loglike (pixel_gate_margin[n_pix]: the distance
    of each pixel's ln N_eff from ln N_min; gate_flip inverts those pixels'
    Eq. (8) decisions).
    """
    lam_np = np.asarray(lam, dtype=np.float64).reshape(16)
    nE = cat.n_events
    out = dict(logL=-math.inf, logL_event=np.full(nE, -math.inf), neff_event=np.zeros(nE),
               neff_sel=0.0, flags=0, grad=np.zeros(16))
    if not lambda_is_valid(lam_np):
        out["flags"] = FLAG_INVALID_LAMBDA
        return out
    bw = BANDWIDTHS[bandwidth]
    lam_t = torch.tensor(lam_np, dtype=DT, requires_grad=grad)
    L = Lam.of(lam_t)
    sky = torch.from_numpy(np.asarray(cat.sky_z, dtype=np.float64)).reshape(1, -1)
    log_nmin = math.log(neff_min) if neff_min > 0 else -math.inf
    lnL_ev = np.empty(nE)
    neff_ev = np.empty(nE)
    gate_m = np.full(nE, math.inf)
    samp_m = np.full(nE, math.inf)
    pix_m = np.full(cat.n_pix, math.inf)
    flips = set() if gate_flip is None else set(int(p) for p in np.asarray(gate_flip).reshape(-1))
    g_ev = torch.zeros(16, dtype=DT)
    umax = (1.0 + cat.z_max) * float(comoving_integral(torch.tensor(cat.z_max, dtype=DT), torch.tensor(lam_np[1])))
    with torch.set_grad_enabled(grad):
        for i in range(nE):
            lT, lS1, lS2, n_s = [], [], [], 0
            for j in range(int(cat.event_pix_off[i]), int(cat.event_pix_off[i + 1])):
                s0, s1 = int(cat.pix_samp_off[j]), int(cat.pix_samp_off[j + 1])
                n_s += s1 - s0
                if s1 == s0:
                    continue
                t = lambda a: torch.from_numpy(np.ascontiguousarray(a[s0:s1], dtype=np.float64))
                z, inside, lw = kde_log_weights(t(cat.m1d), t(cat.m2d), t(cat.dl), t(cat.ln_pi), cat.z_max, L)
                if margins:
                    u = t(cat.dl) * lam_np[0] / C_KMS
                    samp_m[i] = min(samp_m[i], float(torch.min(torch.abs(u / umax - 1.0))))
                z, lw = z[inside], lw[inside]
                if z.numel() == 0:
                    continue
                l1 = lse_all(lw)
                l2 = lse_all(2.0 * lw)
                lneff = float(2.0 * l1 - l2) if math.isfinite(float(l1)) else -math.inf
                if margins and math.isfinite(lneff):
                    gate_m[i] = min(gate_m[i], abs(lneff - log_nmin))
                    pix_m[j] = abs(lneff - log_nmin)
                passes = gate_mode == 2 or lneff >= log_nmin
                if gate_mode != 2 and j in flips:   # the other outcome of the Eq. (8) test
                    passes = not passes
                if not math.isfinite(float(l1)) or not passes:
                    continue
                h = bw(z)
                table = torch.from_numpy(np.asarray(cat.los[int(cat.pix_los_row[j])], dtype=np.float64))
                lT.append(_pixel_kde_term(z, lw, h, table.reshape(1, -1), cat.z_max, L, n_grid))
                lS1.append(l1)
                lS2.append(l2)
            if lT:
                lE = torch.logsumexp(torch.stack(lT), 0)
                e1 = float(torch.logsumexp(torch.stack(lS1), 0))
                e2 = float(torch.logsumexp(torch.stack(lS2), 0))
                neff = math.exp(2 * e1 - e2)
            else:
                lE = torch.tensor(-math.inf, dtype=DT)
                neff = 0.0
            lnL = lE - math.log(max(n_s, 1))
            if gate_mode == 1 and neff < neff_min:
                lnL = torch.tensor(-math.inf, dtype=DT)
            lnL_ev[i] = float(lnL)
            neff_ev[i] = neff
            if grad and math.isfinite(float(lnL)):
                g_ev += torch.autograd.grad(lnL, lam_t, allow_unused=True)[0]
    lc1, lc2, gc = [], [], []
    for c0 in range(0, cat.n_inj, 1 << 20):
        sl = slice(c0, min(cat.n_inj, c0 + (1 << 20)))
        with torch.set_grad_enabled(grad):
            l1, l2 = _selection_chunk(cat, sl, L, sky)
            if grad:
                gc.append(torch.autograd.grad(l1, lam_t)[0] if torch.isfinite(l1) else torch.zeros(16, dtype=DT))
        lc1.append(float(l1.detach()))
        lc2.append(float(l2.detach()))
    l1 = torch.logsumexp(torch.tensor(lc1, dtype=DT), 0)
    l2 = torch.logsumexp(torch.tensor(lc2, dtype=DT), 0)
    ln_alpha = float(l1) - math.log(cat.n_draw)
    neff_sel = math.exp(2 * float(l1) - float(l2)) if math.isfinite(float(l1)) else 0.0
    flags = 0
    if not np.all(np.isfinite(lnL_ev)):
        flags |= FLAG_EVENT_NO_PIXEL
    if not math.isfinite(ln_alpha):
        flags |= FLAG_ALPHA_ZERO
    total = float(np.sum(lnL_ev)) - nE * ln_alpha if flags == 0 else -math.inf
    if flags == 0 and not math.isfinite(total):
        flags |= FLAG_NONFINITE
        total = -math.inf
    out.update(logL=total, logL_event=lnL_ev, neff_event=neff_ev, neff_sel=neff_sel, flags=flags,
               ln_alpha=ln_alpha)
    if grad and flags == 0:
        wts = torch.softmax(torch.tensor(lc1, dtype=DT), 0)
        out["grad"] = (g_ev - nE * sum(w * g for w, g in zip(wts, gc))).numpy()
    if margins:
        out["gate_margin"] = gate_m
        out["sample_margin"] = samp_m
        out["pixel_gate_margin"] = pix_m
    return out


# ---------------------------------------------------------------------------
# Per-pixel random downsampling (Sec. II C, "Memory Reduction Strategies")
# ---------------------------------------------------------------------------
_U64 = np.uint64


def splitmix64(x):
    """SplitMix64 output function (Steele, Lea & Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=_U64) + _U64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> _U64(30))) * _U64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> _U64(27))) * _U64(0x94D049BB133111EB)
        return z ^ (z >> _U64(31))


def downsample(cat, cap, seed):
    """Keep at most `cap` samples per pixel: the ones with the smallest keys
    splitmix64(seed + splitmix64(pixel << 32 | k)) (ties by k), in order."""
    import dataclasses
    keep = []
    pso = [0]
    for j in range(cat.n_pix):
        s0, s1 = int(cat.pix_samp_off[j]), int(cat.pix_samp_off[j + 1])
        n = s1 - s0
        if n <= cap:
            idx = np.arange(n)
        else:
            k = np.arange(n, dtype=_U64)
            with np.errstate(over="ignore"):
                key = splitmix64(_U64(seed) + splitmix64((_U64(j) << _U64(32)) | k))
            idx = np.sort(np.lexsort((np.arange(n), key))[:cap])
        keep.append(s0 + idx)
        pso.append(pso[-1] + len(idx))
    sel = np.concatenate(keep) if keep else np.zeros(0, np.int64)
    return dataclasses.replace(cat, pix_samp_off=np.asarray(pso, np.int64), m1d=cat.m1d[sel], m2d=cat.m2d[sel],
                               dl=cat.dl[sel], ln_pi=cat.ln_pi[sel])


def loglike_batch(cat, lams, **kw):
    """Loop of loglike over a batch of hyperparameter points."""
    return [loglike(cat, lam, **kw) for lam in np.asarray(lams, dtype=np.float64).reshape(-1, 16)]
