"""GPU parity of the KDE numerator (Eq. 6 inside Eq. 5, Appendix D bandwidths)
against the oracle's loglike_kde, through the C ABI."""
import math

import numpy as np
import pytest

from tests.gpu_common import TOL_LOGL_FP32, TOL_LOGL_FP64, check_events, log, need_gpu, rel_close
from tests.test_gpu_edges import RAGGED, ragged_catalog

pytestmark = pytest.mark.gpu
BANDWIDTHS = ["scott", "silverman", "biweight"]


@pytest.fixture(scope="module")
def env():
    need_gpu()
    import torch
    from oracle import dsl_oracle as O
    from paper_2605_23538_amd import binding, synth
    return dict(torch=torch, O=O, binding=binding, synth=synth, c1=synth.make_catalog("c1"))


def _check(env, cat, lam, r, tol, **kw):
    O = env["O"]
    n_amb = 0
    for b in range(len(lam)):
        ref = O.loglike_kde(cat, lam[b], margins=True, **kw)
        assert int(r["flags"][b]) == ref["flags"], (b, int(r["flags"][b]), ref["flags"])
        n_amb += check_events(r["logL_event"][b].cpu().numpy(), r["neff_event"][b].cpu().numpy(), ref, tol)
        if not ref["flags"]:
            assert rel_close(float(r["logL"][b]), ref["logL"], tol), (b, float(r["logL"][b]), ref["logL"])
            assert abs(float(r["neff_sel"][b]) - ref["neff_sel"]) <= 1e-5 * ref["neff_sel"]
    return n_amb


def _run(env, cat, lam, precision="fp32", **kw):
    torch = env["torch"]
    lik = env["binding"].DarkSirenLikelihood(cat, precision=precision, numerator="kde", **kw)
    r = lik.loglike(torch.tensor(lam, device="cuda"), per_event=True)
    torch.cuda.synchronize()
    lik.close()
    return r


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("bandwidth", BANDWIDTHS)
def test_config1_kde(env, precision, bandwidth):
    """10 events x 2000 samples over 16 pixels each, 5 points (fiducial first)."""
    synth = env["synth"]
    log(f"[kde c1 {precision} {bandwidth}]")
    lam = synth.draw_lambdas(5, seed=31)
    lam[0] = synth.fiducial_lambda()
    r = _run(env, env["c1"], lam, precision, kde_bandwidth=bandwidth)
    tol = TOL_LOGL_FP32 if precision == "fp32" else TOL_LOGL_FP64
    assert _check(env, env["c1"], lam, r, tol, bandwidth=bandwidth) <= 1


@pytest.mark.parametrize("bandwidth", BANDWIDTHS)
@pytest.mark.parametrize("gate_mode", [0, 1, 2])
def test_ragged_pixels_kde(env, bandwidth, gate_mode):
    """Pixels of 0, 1, 2, 3, 7, 63, 64, 65, 130 and 200 samples: one-chunk and
    multi-chunk passes, zero bandwidths (single samples, without the gate)."""
    synth = env["synth"]
    log(f"[kde ragged {bandwidth} gate {gate_mode}]")
    cat = ragged_catalog(synth, RAGGED)
    lam = synth.draw_lambdas(4, seed=41)
    lam[0] = synth.fiducial_lambda()
    r = _run(env, cat, lam, kde_bandwidth=bandwidth, gate_mode=gate_mode)
    _check(env, cat, lam, r, TOL_LOGL_FP32, bandwidth=bandwidth, gate_mode=gate_mode)


def test_ragged_pixels_kde_fp64(env):
    """FP64 tiles of four points over ragged pixels: nine points, three tiles,
    the last holding one point."""
    synth = env["synth"]
    log("[kde ragged fp64 biweight]")
    cat = ragged_catalog(synth, RAGGED)
    lam = synth.draw_lambdas(9, seed=47)
    lam[0] = synth.fiducial_lambda()
    r = _run(env, cat, lam, "fp64", kde_bandwidth="biweight", gate_mode=2)
    _check(env, cat, lam, r, TOL_LOGL_FP64, bandwidth="biweight", gate_mode=2)


def test_downsampled_kde(env):
    """At most 40 samples per pixel kept at upload: the bandwidths and grids
    come from the kept samples (their d_L order is rebuilt after the cut)."""
    O, synth = env["O"], env["synth"]
    log("[kde downsampled 40/pixel]")
    ds = O.downsample(env["c1"], 40, seed=5)
    lam = synth.draw_lambdas(3, seed=53)
    lam[0] = synth.fiducial_lambda()
    r = _run(env, env["c1"], lam, max_samples_per_pixel=40, downsample_seed=5, gate_mode=2)
    _check(env, ds, lam, r, TOL_LOGL_FP32, gate_mode=2)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("B", [1, 2, 3])
@pytest.mark.parametrize("bandwidth", ["scott", "biweight"])
def test_fewer_points_than_rows(env, precision, B, bandwidth):
    """Batches of 1-3 points: the rows of a wavefront take different pixels of
    the ragged catalogue (0 to 200 samples side by side), with and without the
    gate."""
    synth = env["synth"]
    log(f"[kde B={B} {precision} {bandwidth}]")
    cat = ragged_catalog(synth, RAGGED)
    lam = synth.draw_lambdas(B, seed=59)
    lam[0] = synth.fiducial_lambda()
    tol = TOL_LOGL_FP32 if precision == "fp32" else TOL_LOGL_FP64
    for gate in (0, 2):
        r = _run(env, cat, lam, precision, kde_bandwidth=bandwidth, gate_mode=gate)
        _check(env, cat, lam, r, tol, bandwidth=bandwidth, gate_mode=gate)


@pytest.mark.parametrize("B", [4, 20, 64])
@pytest.mark.parametrize("bandwidth", BANDWIDTHS)
def test_point_tiles_ragged(env, B, bandwidth):
    """Batches take the tile kernel (4, 16 and 64 points per wavefront): pass A
    with the points side by side, the passing points packed into rows for the
    grid stage; ragged pixels (0 to 200 samples), every point against the
    oracle, with and without the gate."""
    synth = env["synth"]
    log(f"[kde tiles B={B} {bandwidth}]")
    cat = ragged_catalog(synth, RAGGED)
    lam = synth.draw_lambdas(B, seed=61)
    lam[0] = synth.fiducial_lambda()
    for gate in (0, 2):
        r = _run(env, cat, lam, kde_bandwidth=bandwidth, gate_mode=gate)
        _check(env, cat, lam, r, TOL_LOGL_FP32, bandwidth=bandwidth, gate_mode=gate)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("B", [1, 5])
@pytest.mark.parametrize("bandwidth", ["silverman", "biweight"])
def test_split_pixels(env, precision, B, bandwidth):
    """With fewer than four points, pixels above 256 samples are split for the
    grid stage (each part keeps the whole pixel's gate and bandwidth): sizes at
    and around the part size.  Batches (B = 5) walk whole pixels, largest first."""
    torch, synth = env["torch"], env["synth"]
    log(f"[kde split pixels B={B} {precision} {bandwidth}]")
    cat = ragged_catalog(synth, [[256, 257], [512, 3, 513], [1000]], n_inj=500)
    lam = synth.draw_lambdas(B, seed=73)
    lam[0] = synth.fiducial_lambda()
    tol = TOL_LOGL_FP32 if precision == "fp32" else TOL_LOGL_FP64
    for gate in (0, 2):
        lik = env["binding"].DarkSirenLikelihood(cat, precision=precision, numerator="kde",
                                                 kde_bandwidth=bandwidth, gate_mode=gate)
        r = lik.loglike(torch.tensor(lam, device="cuda"), per_event=True)
        torch.cuda.synchronize()
        # parts of 256: 1 + 2, 2 + 1 + 3, 4; whole pixels for batches
        assert lik.info("kde_units") == (13 if B < 4 else 6)
        lik.close()
        _check(env, cat, lam, r, tol, bandwidth=bandwidth, gate_mode=gate)


def test_large_pixels_unsplit(env):
    """With enough work per wavefront large pixels stay whole: 4096 points on a
    catalogue whose average work per wavefront exceeds twice its largest pixel
    (1000 samples), sampled against the oracle."""
    torch, O, synth, binding = env["torch"], env["O"], env["synth"], env["binding"]
    log("[kde large pixels, 4096 points, unsplit]")
    cat = ragged_catalog(synth, [[256, 257], [512, 3, 513], [1000]] + [[500, 500]] * 20, n_inj=500)
    lam = synth.draw_lambdas(4096, seed=79)
    lam[0] = synth.fiducial_lambda()
    lik = binding.DarkSirenLikelihood(cat, numerator="kde")
    r = lik.loglike(torch.tensor(lam, device="cuda"))
    torch.cuda.synchronize()
    assert lik.info("kde_units") == len(cat.pix_samp_off) - 1   # no pixel split
    for b in (0, 1, 2048, 4095):
        ref = O.loglike_kde(cat, lam[b], margins=True)
        assert int(r["flags"][b]) == ref["flags"], b
        if not ref["flags"]:
            assert rel_close(float(r["logL"][b]), ref["logL"], TOL_LOGL_FP32), (b, float(r["logL"][b]), ref["logL"])
    lik.close()


@pytest.mark.parametrize("n_grid", [2, 64, 300, 1024])
def test_grid_sizes(env, n_grid):
    """Grids below, at and above one node per lane, up to 16 nodes per lane."""
    synth = env["synth"]
    log(f"[kde grid {n_grid}]")
    cat = ragged_catalog(synth, RAGGED)
    lam = synth.fiducial_lambda()[None]
    r = _run(env, cat, lam, kde_grid=n_grid)
    _check(env, cat, lam, r, TOL_LOGL_FP32, n_grid=n_grid)


def test_batch_spans_two_tiles(env):
    """70 points: two point tiles, the second ragged."""
    torch, O, synth = env["torch"], env["O"], env["synth"]
    log("[kde B=70]")
    lam = synth.draw_lambdas(70, seed=43)
    r = _run(env, env["c1"], lam)
    for b in (0, 1, 63, 64, 69):
        ref = O.loglike_kde(env["c1"], lam[b], margins=True)
        assert int(r["flags"][b]) == ref["flags"]
        if not ref["flags"]:
            assert rel_close(float(r["logL"][b]), ref["logL"], TOL_LOGL_FP32), (b, float(r["logL"][b]), ref["logL"])


def test_full_size_pixels_subset(env):
    """Twelve events of the 140-event catalogue (pixels of tens to hundreds of
    samples, 1024-node tables), fiducial point, every bandwidth rule."""
    synth = env["synth"]
    cat = synth.make_catalog("c2").subset(np.arange(12), inj=slice(0, 200_000))
    lam = synth.fiducial_lambda()[None]
    for bw in BANDWIDTHS:
        log(f"[kde c2 subset {bw}]")
        r = _run(env, cat, lam, kde_bandwidth=bw)
        assert _check(env, cat, lam, r, TOL_LOGL_FP32, bandwidth=bw) <= 1


def test_kde_rejects_gradient_and_spectral(env):
    torch, binding = env["torch"], env["binding"]
    lam = torch.tensor(env["synth"].fiducial_lambda()[None], device="cuda")
    lik = binding.DarkSirenLikelihood(env["c1"], numerator="kde")
    with pytest.raises(binding.DSLError, match="no gradient"):
        lik.loglike_grad(lam)
    lik.set_option("z_prior", 1)
    with pytest.raises(binding.DSLError, match="z_prior"):
        lik.loglike(lam)
    lik.set_option("z_prior", 0)
    assert math.isfinite(float(lik.loglike(lam)["logL"][0]))
    lik.close()


def test_kde_deterministic_and_graph_replay(env):
    torch, binding = env["torch"], env["binding"]
    lam = torch.tensor(env["synth"].draw_lambdas(8, seed=5), device="cuda")
    lik = binding.DarkSirenLikelihood(env["c1"], numerator="kde", kde_bandwidth="biweight")
    lik.set_option("graph", 0)
    ref = lik.loglike(lam)["logL"].clone()
    lik.set_option("graph", 1)
    for _ in range(3):
        out = lik.loglike(lam)["logL"]
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    lik.close()


def test_kde_work_counters(env):
    """Grid-node counter = (pixel, point) pairs with a bandwidth > 0 (counted
    with the oracle's weights and bandwidth rule, no gate) x grid nodes; the
    kernel-term counter is a multiple of the grid size bounded by samples x
    points x nodes."""
    import torch as T_
    torch, synth, O = env["torch"], env["synth"], env["O"]
    cat = env["c1"]
    B, n_grid = 5, 256
    lam1 = synth.fiducial_lambda()
    L = O.Lam.of(T_.tensor(lam1, dtype=T_.float64))
    n_h = 0
    for j in range(len(cat.pix_samp_off) - 1):
        s0, s1 = int(cat.pix_samp_off[j]), int(cat.pix_samp_off[j + 1])
        if s1 == s0:
            continue
        t = lambda a: T_.from_numpy(np.ascontiguousarray(a[s0:s1], dtype=np.float64))
        z, inside, lw = O.kde_log_weights(t(cat.m1d), t(cat.m2d), t(cat.dl), t(cat.ln_pi), cat.z_max, L)
        z, lw = z[inside], lw[inside]
        if z.numel() and math.isfinite(float(O.lse_all(lw))) and float(O.BANDWIDTHS["scott"](z)) > 0:
            n_h += 1
    lam = torch.tensor(lam1[None].repeat(B, 0), device="cuda")
    lik = env["binding"].DarkSirenLikelihood(cat, numerator="kde", gate_mode=2)
    r = lik.loglike(lam)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(r["logL"].cpu().numpy()))
    log(f"  {n_h} pixels with a bandwidth, {lik.info('kde_nodes'):.0f} grid nodes")
    assert n_h > 0 and lik.info("kde_nodes") == n_h * B * n_grid
    ev = lik.info("kde_evals")
    assert ev % n_grid == 0 and 0 < ev <= cat.n_samp * B * n_grid
    lik.close()


def test_part_list_rebuilds_with_graphs(env):
    """One handle, graph replay on, batches that take different kernels (the
    row kernel with parts of 256 samples for one point, the tile kernel over
    whole pixels for 4096 points): every call equals an eager call of the same
    batch, bitwise."""
    torch, synth, binding = env["torch"], env["synth"], env["binding"]
    cat = ragged_catalog(synth, [[256, 257], [512, 3, 513], [1000]], n_inj=500)
    lams = {B: torch.tensor(synth.draw_lambdas(B, seed=83), device="cuda") for B in (1, 4096)}
    ref = {}
    for B, lam in lams.items():
        e = binding.DarkSirenLikelihood(cat, numerator="kde")
        e.set_option("graph", 0)
        ref[B] = e.loglike(lam)["logL"].clone()
        torch.cuda.synchronize()
        e.close()
    lik = binding.DarkSirenLikelihood(cat, numerator="kde")
    for B in (1, 4096, 1, 4096):
        out = lik.loglike(lams[B])["logL"]
        torch.cuda.synchronize()
        assert torch.equal(torch.nan_to_num(out, neginf=-1e300), torch.nan_to_num(ref[B], neginf=-1e300)), B
    lik.close()
