"""Seeded synthetic catalogues for the dark-siren population likelihood.

This module only *generates inputs*: posterior samples, sky pixels with their
line-of-sight (LOS) redshift tables, detected injections and hyperparameter
points.  It holds none of the likelihood's arithmetic (no cosmology, no
population model, no reweighting), so both the FP64 oracle and the GPU path
can consume what it produces without sharing any of the method.

Stand-ins for the paper's data (Appendix A: O5 mock PE samples, GWTC-4.0
events, the GLADE+ K-band LOS priors and the public injection campaign), none
of which is available here:

* posterior samples, i.i.d. per event: m1_det ~ U(10, 80), q ~ U(0.3, 1),
  m2_det = q m1_det, d_L ~ LogNormal(ln 1500 Mpc, 0.3); the PE prior is
  pi ∝ d_L^2 (flat in detector-frame masses), so ln pi = 2 ln d_L;
* sky pixels: per event a Dirichlet(1) split of the samples over its pixels
  (the padded (event, pixel, sample) tensor of the paper's Sec. II B becomes
  CSR offsets, the flattened ragged layout its conclusions call for);
* one LOS table per pixel on n_z uniform nodes over [0, z_max]: half a mean
  of 20 Gaussian galaxy bumps (sigma 0.01, centres U(0.02, 1.5)) and half a
  smooth completion shape, normalised to unit integral; the completion shape
  is the comoving-volume element of an Omega_m = 1 universe,
  (1 - (1+z)^-1/2)^2 (1+z)^-3/2, which has a closed form;
* the sky-averaged table used by the selection term is that completion shape;
* injections: m1_det ~ LogUniform(5, 300), q ~ U(0.05, 1), d_L ∝ d_L^2 on
  (0, d_max], an orientation factor Theta ~ U(0.2, 1); detected when the toy
  SNR 8 (Mc_det / 20)^(5/6) (d_ref / d_L) Theta reaches 12 (the paper's SNR
  cut); ln p_draw is the analytic draw density in (m1_det, m2_det, d_L).

All stored sample values are float32-representable so the FP32 and FP64 GPU
paths and the FP64 oracle read identical numbers.  Every event and every
injection chunk has its own random stream, so any subset of a catalogue can be
regenerated alone (the full-size parity tests rely on this).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

# Hyperparameter layout shared by every interface of the library.
LAMBDA_NAMES = (
    "H0", "Om", "alpha", "beta", "mmin", "mmax", "delta_m",
    "mu_low", "sigma_low", "mu_high", "sigma_high", "lambda_g", "lambda_low",
    "gamma", "kappa", "z_p",
)
N_LAMBDA = len(LAMBDA_NAMES)
IDX = {n: i for i, n in enumerate(LAMBDA_NAMES)}

# Population values of the paper's Table II; the fiducial cosmology is
# H0 = 70, Omega_m = 0.3 (the benchmark point) instead of Table II's Planck values.
TABLE_II = dict(alpha=2.9, beta=1.0, mmin=4.6, mmax=86.3, delta_m=4.8,
                mu_low=9.7, sigma_low=0.7, mu_high=30.7, sigma_high=6.3,
                lambda_g=0.4, lambda_low=0.8, gamma=3.3, kappa=2.9, z_p=2.5)
FIDUCIAL = dict(H0=70.0, Om=0.3, **TABLE_II)

# Uniform prior box for batched draws (the paper prints none; H0 and Omega_m
# ranges are those of the batched workload definition).
PRIOR_BOUNDS = dict(
    H0=(20.0, 140.0), Om=(0.1, 0.5), alpha=(1.5, 12.0), beta=(-4.0, 12.0),
    mmin=(2.0, 10.0), mmax=(50.0, 200.0), delta_m=(0.0, 10.0),
    mu_low=(5.0, 20.0), sigma_low=(0.4, 10.0), mu_high=(20.0, 50.0),
    sigma_high=(0.4, 10.0), lambda_g=(0.0, 1.0), lambda_low=(0.0, 1.0),
    gamma=(0.0, 12.0), kappa=(0.0, 6.0), z_p=(0.0, 4.0),
)


def lam_vector(**kw) -> np.ndarray:
    """Hyperparameter vector in LAMBDA_NAMES order (float64[16])."""
    d = dict(FIDUCIAL)
    d.update(kw)
    return np.array([float(d[n]) for n in LAMBDA_NAMES], dtype=np.float64)


def fiducial_lambda() -> np.ndarray:
    return lam_vector()


def draw_lambdas(n: int, seed: int) -> np.ndarray:
    """n points uniform in PRIOR_BOUNDS, float64[n, 16]."""
    rng = np.random.default_rng([int(seed), 7, 0])
    lo = np.array([PRIOR_BOUNDS[k][0] for k in LAMBDA_NAMES])
    hi = np.array([PRIOR_BOUNDS[k][1] for k in LAMBDA_NAMES])
    return lo + (hi - lo) * rng.random((n, N_LAMBDA))


@dataclasses.dataclass
class Catalog:
    """CSR catalogue: events -> pixels -> samples, plus injections."""
    event_pix_off: np.ndarray   # int64[n_events + 1]
    pix_samp_off: np.ndarray    # int64[n_pix + 1]
    pix_los_row: np.ndarray     # int32[n_pix]
    los: np.ndarray             # float32[n_rows, n_z]
    sky_z: np.ndarray           # float32[n_z]
    z_max: float
    m1d: np.ndarray             # float64[n_samp]
    m2d: np.ndarray
    dl: np.ndarray              # Mpc
    ln_pi: np.ndarray
    inj_m1d: np.ndarray         # float64[n_inj]
    inj_m2d: np.ndarray
    inj_dl: np.ndarray
    inj_ln_pdraw: np.ndarray
    n_draw: int
    name: str = ""

    @property
    def n_events(self) -> int:
        return len(self.event_pix_off) - 1

    @property
    def n_pix(self) -> int:
        return len(self.pix_samp_off) - 1

    @property
    def n_samp(self) -> int:
        return len(self.m1d)

    @property
    def n_inj(self) -> int:
        return len(self.inj_m1d)

    @property
    def n_z(self) -> int:
        return self.los.shape[1]

    def samples_per_event(self) -> np.ndarray:
        return np.diff(self.pix_samp_off[self.event_pix_off])

    def nbytes(self) -> int:
        return sum(getattr(self, f.name).nbytes for f in dataclasses.fields(self)
                   if isinstance(getattr(self, f.name), np.ndarray))

    def save(self, path: str) -> None:
        arrays = {f.name: getattr(self, f.name) for f in dataclasses.fields(self)
                  if isinstance(getattr(self, f.name), np.ndarray)}
        np.savez(path, z_max=np.float64(self.z_max), n_draw=np.int64(self.n_draw),
                 name=np.str_(self.name), **arrays)

    @staticmethod
    def load(path: str) -> "Catalog":
        with np.load(path, allow_pickle=False) as f:
            kw = {k: f[k] for k in f.files}
        kw["z_max"] = float(kw["z_max"])
        kw["n_draw"] = int(kw["n_draw"])
        kw["name"] = str(kw["name"])
        return Catalog(**kw)

    def subset(self, events: Sequence[int], inj: Optional[slice] = None,
               n_draw: Optional[int] = None) -> "Catalog":
        """Catalogue restricted to the listed events (and an injection slice)."""
        events = np.asarray(events, dtype=np.int64)
        pix_lists, samp_lists, rows = [], [], []
        epo = [0]
        pso = [0]
        for e in events:
            p0, p1 = self.event_pix_off[e], self.event_pix_off[e + 1]
            for p in range(p0, p1):
                s0, s1 = self.pix_samp_off[p], self.pix_samp_off[p + 1]
                samp_lists.append(np.arange(s0, s1))
                pso.append(pso[-1] + (s1 - s0))
                rows.append(self.pix_los_row[p])
            epo.append(epo[-1] + (p1 - p0))
        sidx = np.concatenate(samp_lists) if samp_lists else np.zeros(0, np.int64)
        rows = np.asarray(rows, dtype=np.int64)
        uniq, inv = np.unique(rows, return_inverse=True)
        inj = inj if inj is not None else slice(0, self.n_inj)
        return Catalog(
            event_pix_off=np.asarray(epo, np.int64), pix_samp_off=np.asarray(pso, np.int64),
            pix_los_row=inv.astype(np.int32), los=self.los[uniq], sky_z=self.sky_z,
            z_max=self.z_max, m1d=self.m1d[sidx], m2d=self.m2d[sidx], dl=self.dl[sidx],
            ln_pi=self.ln_pi[sidx], inj_m1d=self.inj_m1d[inj], inj_m2d=self.inj_m2d[inj],
            inj_dl=self.inj_dl[inj], inj_ln_pdraw=self.inj_ln_pdraw[inj],
            n_draw=int(n_draw if n_draw is not None else self.n_draw), name=self.name + "-subset")


# --------------------------------------------------------------------------
# Workload shapes
# --------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Shape:
    name: str
    n_events: int
    samples: tuple          # ("fixed", n) | ("uniform", lo, hi)
    pixels: tuple           # ("fixed", n) | ("uniform", lo, hi) | ("loguniform", lo, hi)
    n_z: int
    n_inj: int
    z_max: float = 2.0
    inj_d_max: float = 6000.0
    inj_d_ref: float = 3000.0


SHAPES = {
    # 10 events x 2000 samples, 16 pixels of 512-node tables, 1e4 injections.
    "c1": Shape("c1", 10, ("fixed", 2000), ("fixed", 16), 512, 10_000),
    # GWTC-4-like: 140 events, U[2000, 20000] samples, 64-256 pixels, 2e6 inj.
    "c2": Shape("c2", 140, ("uniform", 2000, 20000), ("uniform", 64, 256), 1024, 2_000_000),
    # O5-like: 5000 events, U[1000, 8192] samples, 32-2048 pixels, 1e7 inj.
    "c4": Shape("c4", 5000, ("uniform", 1000, 8192), ("loguniform", 32, 2048), 1024, 10_000_000),
}
SHAPES["c3"] = dataclasses.replace(SHAPES["c1"], name="c3")
SHAPES["c5"] = dataclasses.replace(SHAPES["c1"], name="c5")

N_BUMPS = 20
BUMP_SIGMA = 0.01
BUMP_LO, BUMP_HI = 0.02, 1.5
INJ_CHUNK = 1 << 21          # draws per injection random stream


def _draw_count(rng, spec):
    kind = spec[0]
    if kind == "fixed":
        return int(spec[1])
    if kind == "uniform":
        return int(rng.integers(spec[1], spec[2] + 1))
    if kind == "loguniform":
        return int(min(spec[2], math.floor(math.exp(rng.uniform(math.log(spec[1]),
                                                                   math.log(spec[2] + 1))))))
    raise ValueError(spec)


def completion_shape(n_z: int, z_max: float) -> np.ndarray:
    """Closed-form comoving-volume shape of an Omega_m = 1 universe, unit integral."""
    z = np.linspace(0.0, z_max, n_z)
    x = 1.0 + z
    v = (1.0 - x ** -0.5) ** 2 * x ** -1.5
    dz = z_max / (n_z - 1)
    return v / (dz * (v.sum() - 0.5 * (v[0] + v[-1])))


def _event_rng(seed, i):
    return np.random.default_rng([int(seed), 1, int(i)])


def _gen_event(shape: Shape, seed: int, i: int):
    rng = _event_rng(seed, i)
    n_s = _draw_count(rng, shape.samples)
    n_p = _draw_count(rng, shape.pixels)
    probs = rng.dirichlet(np.ones(n_p))
    pix = rng.choice(n_p, size=n_s, p=probs)
    m1 = rng.uniform(10.0, 80.0, n_s)
    q = rng.uniform(0.3, 1.0, n_s)
    dl = rng.lognormal(math.log(1500.0), 0.3, n_s)
    centres = rng.uniform(BUMP_LO, BUMP_HI, (n_p, N_BUMPS))
    order = np.argsort(pix, kind="stable")
    counts = np.bincount(pix, minlength=n_p)
    m1f = m1[order].astype(np.float32)
    m2f = (m1[order] * q[order]).astype(np.float32)
    dlf = dl[order].astype(np.float32)
    return counts, m1f, m2f, dlf, centres


def _los_tables(centres: np.ndarray, n_z: int, z_max: float, base: np.ndarray) -> np.ndarray:
    """Rows of 0.5 * mean of Gaussian bumps + 0.5 * base, each of unit integral.

    Each bump is evaluated on the nodes within 6 sigma of its centre and added
    row by row in bump order (torch CPU kernels, parallel over rows); nodes
    outside [0, z_max] land in padding columns that are dropped.
    """
    import torch
    n_p = centres.shape[0]
    dz = z_max / (n_z - 1)
    half = int(math.ceil(6.0 * BUMP_SIGMA / dz)) + 1
    c = torch.from_numpy(np.ascontiguousarray(centres, dtype=np.float64))
    k0 = torch.round(c / dz).to(torch.int64)                     # [n_p, N_BUMPS]
    offs = torch.arange(-half, half + 1, dtype=torch.int64)
    offs_z = offs.to(torch.float64) * dz
    acc = torch.zeros((n_p, n_z + 2 * half), dtype=torch.float64)
    a = -0.5 / BUMP_SIGMA ** 2
    for b in range(N_BUMPS):
        d = (k0[:, b:b + 1].to(torch.float64) * dz - c[:, b:b + 1]) + offs_z[None, :]
        vals = torch.exp(d * d * a)
        acc.scatter_add_(1, k0[:, b:b + 1] + (offs + half)[None, :], vals)
    norm = 1.0 / (BUMP_SIGMA * math.sqrt(2 * math.pi))
    tab = (0.5 * norm / N_BUMPS) * acc[:, half:half + n_z] + 0.5 * torch.from_numpy(base)[None, :]
    integ = dz * (tab.sum(1) - 0.5 * (tab[:, 0] + tab[:, -1]))
    return (tab / integ[:, None]).to(torch.float32).numpy()


def _inj_chunk(shape: Shape, seed: int, c: int):
    rng = np.random.default_rng([int(seed), 2, int(c)])
    n = INJ_CHUNK
    lo, hi = math.log(5.0), math.log(300.0)
    m1 = np.exp(rng.uniform(lo, hi, n)).astype(np.float32).astype(np.float64)
    q = rng.uniform(0.05, 1.0, n)
    m2 = (m1 * q).astype(np.float32).astype(np.float64)
    dl = (shape.inj_d_max * rng.random(n) ** (1.0 / 3.0)).astype(np.float32).astype(np.float64)
    theta = rng.uniform(0.2, 1.0, n)
    mc = (m1 * m2) ** 0.6 / (m1 + m2) ** 0.2
    snr = 8.0 * (mc / 20.0) ** (5.0 / 6.0) * (shape.inj_d_ref / np.maximum(dl, 1e-3)) * theta
    det = np.flatnonzero(snr >= 12.0)
    # draw density: p(m1) p(q) / m1 p(d_L), with q = m2 / m1.
    ln_p = (-np.log(m1) - math.log(hi - lo) - math.log(0.95) - np.log(m1)
            + math.log(3.0) + 2.0 * np.log(dl) - 3.0 * math.log(shape.inj_d_max))
    return det, m1, m2, dl, ln_p


def make_injections(shape: Shape, seed: int, n_det: Optional[int] = None):
    n_det = shape.n_inj if n_det is None else n_det
    out = {k: [] for k in ("m1", "m2", "dl", "lp")}
    got, c, n_draw = 0, 0, 0
    while got < n_det:
        det, m1, m2, dl, lp = _inj_chunk(shape, seed, c)
        need = n_det - got
        if len(det) >= need:
            det = det[:need]
            n_draw += int(det[-1]) + 1
        else:
            n_draw += INJ_CHUNK
        for k, a in zip(("m1", "m2", "dl", "lp"), (m1, m2, dl, lp)):
            out[k].append(a[det])
        got += len(det)
        c += 1
    cat = {k: np.concatenate(v) for k, v in out.items()}
    cat["lp"] = cat["lp"].astype(np.float32).astype(np.float64)
    return cat["m1"], cat["m2"], cat["dl"], cat["lp"], n_draw


def make_catalog(config: str = "c1", seed: Optional[int] = None,
                 events: Optional[Sequence[int]] = None,
                 n_inj: Optional[int] = None, n_events: Optional[int] = None) -> Catalog:
    """Generate a seeded synthetic catalogue.

    config: one of SHAPES ("c1" .. "c5").  seed defaults to the config number.
    events: optional subset of event indices (same values as in the full
    catalogue).  n_inj / n_events override the shape's sizes.
    """
    shape = SHAPES[config]
    if seed is None:
        seed = int(config[1:])
    n_ev = shape.n_events if n_events is None else n_events
    ev_ids = np.arange(n_ev) if events is None else np.asarray(events, dtype=np.int64)
    base = completion_shape(shape.n_z, shape.z_max)
    epo, pso = [0], [0]
    m1s, m2s, dls, tabs = [], [], [], []
    pending_c, pending_rows = [], 0
    for i in ev_ids:
        counts, m1f, m2f, dlf, centres = _gen_event(shape, seed, int(i))
        epo.append(epo[-1] + len(counts))
        pso.extend((pso[-1] + np.cumsum(counts)).tolist())
        m1s.append(m1f)
        m2s.append(m2f)
        dls.append(dlf)
        pending_c.append(centres)
        pending_rows += len(counts)
        if pending_rows >= 20000:
            tabs.append(_los_tables(np.concatenate(pending_c), shape.n_z, shape.z_max, base))
            pending_c, pending_rows = [], 0
    if pending_c:
        tabs.append(_los_tables(np.concatenate(pending_c), shape.n_z, shape.z_max, base))
    los = np.concatenate(tabs) if tabs else np.zeros((0, shape.n_z), np.float32)
    m1d = np.concatenate(m1s).astype(np.float64)
    m2d = np.concatenate(m2s).astype(np.float64)
    dl = np.concatenate(dls).astype(np.float64)
    ln_pi = (2.0 * np.log(dl)).astype(np.float32).astype(np.float64)
    im1, im2, idl, ilp, n_draw = make_injections(shape, seed, n_inj)
    n_pix = len(pso) - 1
    return Catalog(
        event_pix_off=np.asarray(epo, np.int64), pix_samp_off=np.asarray(pso, np.int64),
        pix_los_row=np.arange(n_pix, dtype=np.int32), los=los,
        sky_z=base.astype(np.float32), z_max=shape.z_max,
        m1d=m1d, m2d=m2d, dl=dl, ln_pi=ln_pi,
        inj_m1d=im1, inj_m2d=im2, inj_dl=idl, inj_ln_pdraw=ilp, n_draw=n_draw,
        name=config)


def lambdas_for(config: str, B: Optional[int] = None, seed: Optional[int] = None) -> np.ndarray:
    """Hyperparameter batch of a workload: the fiducial point, or prior draws."""
    if config in ("c1", "c2"):
        return fiducial_lambda()[None, :].repeat(B or 1, 0)
    default_B = {"c3": 512, "c4": 64, "c5": 64}[config]
    return draw_lambdas(B or default_B, seed if seed is not None else int(config[1:]))
