"""Edge cases, determinism and graph replay of the HIP path (through the C ABI)."""
import math

import numpy as np
import pytest

from tests.gpu_common import TOL_LOGL_FP32, check_events, check_grad, log, need_gpu, rel_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    need_gpu()
    import torch
    from oracle import dsl_oracle as O
    from paper_2605_23538_amd import binding, synth
    return dict(torch=torch, O=O, binding=binding, synth=synth)


def ragged_catalog(synth, sizes, n_inj=777, seed=0):
    """One event per entry of `sizes`, each a list of pixel sample counts."""
    rng = np.random.default_rng(seed)
    epo, pso = [0], [0]
    for ev in sizes:
        for n in ev:
            pso.append(pso[-1] + n)
        epo.append(epo[-1] + len(ev))
    n = pso[-1]
    m1 = rng.uniform(10, 80, n)
    q = rng.uniform(0.3, 1, n)
    dl = rng.lognormal(math.log(1500), 0.3, n)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    n_pix = len(pso) - 1
    zg = np.linspace(0, 2, 256)
    los = np.stack([1 + 0.8 * np.sin(7 * zg + k) ** 2 for k in range(n_pix)]).astype(np.float32)
    im1 = rng.uniform(8, 90, n_inj)
    iq = rng.uniform(0.2, 1, n_inj)
    idl = rng.uniform(100, 6000, n_inj)
    return synth.Catalog(
        event_pix_off=np.asarray(epo, np.int64), pix_samp_off=np.asarray(pso, np.int64),
        pix_los_row=np.arange(n_pix, dtype=np.int32), los=los, sky_z=np.ones(256, np.float32), z_max=2.0,
        m1d=f32(m1), m2d=f32(m1 * q), dl=f32(dl), ln_pi=f32(2 * np.log(dl)),
        inj_m1d=f32(im1), inj_m2d=f32(im1 * iq), inj_dl=f32(idl),
        inj_ln_pdraw=f32(-2 * np.log(im1) + 2 * np.log(idl) - 21.0), n_draw=5000)


RAGGED = [[1, 2, 63, 64, 65], [0, 130, 0, 7], [1], [200], [3, 3, 3, 3, 3, 3, 3]]


@pytest.mark.parametrize("precision,tile", [("fp32", 1), ("fp32", 4), ("fp32", 16), ("fp32", 64),
                                            ("fp64", 1), ("fp64", 4)])
@pytest.mark.parametrize("chunk", [64, 0])
def test_ragged_pixels_and_items(mods, precision, tile, chunk):
    """Pixels of 0, 1, 2, 63, 64, 65, 130, 200 samples; items split mid-event."""
    torch, O, synth = mods["torch"], mods["O"], mods["synth"]
    cat = ragged_catalog(synth, RAGGED)
    lik = mods["binding"].DarkSirenLikelihood(cat, precision=precision)
    lik.set_option("lambda_tile", tile)
    lik.set_option("chunk", chunk)
    lam = synth.draw_lambdas(5, seed=21)
    lam[0] = synth.fiducial_lambda()
    r = lik.loglike(torch.tensor(lam, device="cuda"), per_event=True)
    torch.cuda.synchronize()
    tol = TOL_LOGL_FP32 if precision == "fp32" else 1e-10
    for b in range(len(lam)):
        ref = O.loglike(cat, lam[b], margins=True)
        assert int(r["flags"][b]) == ref["flags"], (b, int(r["flags"][b]), ref["flags"])
        ev = r["logL_event"][b].cpu().numpy()
        check_events(ev, r["neff_event"][b].cpu().numpy(), ref, tol)
        if not ref["flags"]:
            assert rel_close(float(r["logL"][b]), ref["logL"], tol)
    lik.close()


def test_flags_invalid_lambda_and_failing_gate(mods):
    torch, O, synth = mods["torch"], mods["O"], mods["synth"]
    cat = ragged_catalog(synth, RAGGED)
    lik = mods["binding"].DarkSirenLikelihood(cat, precision="fp32")
    lam = np.stack([synth.fiducial_lambda()] * 6)
    lam[1, 4] = 100.0          # m_min > m_max
    lam[2, 1] = 1.5            # Omega_m > 1
    lam[3, 8] = -1.0           # sigma_low < 0
    lam[4, 11] = 1.2           # lambda_g > 1
    lam[5, 0] = float("nan")
    r = lik.loglike(torch.tensor(lam, device="cuda"))
    fl = r["flags"].cpu().numpy()
    lg = r["logL"].cpu().numpy()
    # the one-sample event cannot pass the N_eff >= 2 gate: flag 2, as in the oracle
    ref = O.loglike(cat, lam[0])
    assert fl[0] == ref["flags"] == 2 and lg[0] == -math.inf
    for b in range(1, 6):
        assert fl[b] & 1 and lg[b] == -math.inf
    # a gate nothing passes: every event flagged, ln L = -inf
    lik.set_option("neff_min", 1e9)
    r = lik.loglike(torch.tensor(lam[:1], device="cuda"), per_event=True)
    assert int(r["flags"][0]) & 2 and float(r["logL"][0]) == -math.inf
    assert np.all(np.isneginf(r["logL_event"][0].cpu().numpy()))
    # gate modes 0, 1 (event gate) and 2 (no gate) against the oracle
    for mode in (0, 1, 2):
        lik.set_option("neff_min", 2.0)
        lik.set_option("gate_mode", mode)
        r = lik.loglike(torch.tensor(lam[:1], device="cuda"), per_event=True)
        ref = O.loglike(cat, lam[0], gate_mode=mode, margins=True)
        assert int(r["flags"][0]) == ref["flags"]
        check_events(r["logL_event"][0].cpu().numpy(), r["neff_event"][0].cpu().numpy(), ref, TOL_LOGL_FP32)
    lik.close()


def test_bad_arguments_raise(mods):
    torch, synth, binding = mods["torch"], mods["synth"], mods["binding"]
    cat = ragged_catalog(synth, RAGGED)
    lik = binding.DarkSirenLikelihood(cat)
    lik.set_option("max_batch", 4)
    with pytest.raises(binding.DSLError):
        lik.loglike(torch.zeros(5, 16, dtype=torch.float64, device="cuda"))
    with pytest.raises(binding.DSLError):
        lik.set_option("lambda_tile", 3)
    with pytest.raises(binding.DSLError):
        lik.set_option("nonsense", 1)
    lik.close()


def test_determinism_and_graph_replay(mods):
    """Repeated calls are bitwise equal; graph replays (with eager work and
    synchronisations in between) equal the eager launch sequence."""
    torch, synth = mods["torch"], mods["synth"]
    cat = synth.make_catalog("c1", n_events=4, n_inj=5000)
    lik = mods["binding"].DarkSirenLikelihood(cat)
    lam = torch.tensor(synth.draw_lambdas(70, seed=9), device="cuda")
    lik.set_option("graph", 0)
    eager = lik.loglike_grad(lam)
    e_l, e_g = eager["logL"].clone(), eager["grad"].clone()
    lik.set_option("graph", 1)
    outs = []
    logL = torch.empty(70, dtype=torch.float64, device="cuda")
    for rep in range(4):
        r = lik.loglike_grad(lam)
        _ = (lam * 2).sum()            # unrelated eager work between replays
        torch.cuda.synchronize()
        outs.append((r["logL"].clone(), r["grad"].clone()))
    for l, g in outs:
        assert torch.equal(torch.nan_to_num(l, neginf=-1e300), torch.nan_to_num(e_l, neginf=-1e300))
        assert torch.equal(g, e_g)
    log("  4 graph replays bitwise equal to eager")
    lik.close()


def test_side_stream(mods):
    """Calls on a stream other than the current one (inputs prepared on the
    current stream just before) equal calls on the current stream, with and
    without graph replay."""
    torch, synth = mods["torch"], mods["synth"]
    cat = synth.make_catalog("c1", n_events=4, n_inj=5000)
    lik = mods["binding"].DarkSirenLikelihood(cat)
    lam0 = torch.tensor(synth.draw_lambdas(32, seed=5), device="cuda")
    ref = lik.loglike_grad(lam0)
    ref_f = lik.loglike(lam0)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    n = 0
    for graph in (0, 1):
        lik.set_option("graph", graph)
        for rep in range(3):
            lam = lam0 * 1.0   # written on the current stream right before the call
            r = lik.loglike_grad(lam, stream=side)
            f = lik.loglike(lam, stream=side)
            side.synchronize()
            for a, b in ((r["logL"], ref["logL"]), (f["logL"], ref_f["logL"])):
                assert torch.equal(torch.nan_to_num(a, neginf=-1e300), torch.nan_to_num(b, neginf=-1e300))
            assert torch.equal(r["grad"], ref["grad"])
            n += 1
    log(f"  {n} side-stream calls (graph off and on) equal current-stream calls")
    lik.close()


def test_graphs_after_workspace_growth(mods):
    """One handle, graph replay on, fixed output buffers per batch size, and
    batches that grow and shrink (workspace reallocations in between): every
    call equals an eager call of the same batch.  Captured graphs hold
    workspace addresses, so they must be dropped when a buffer moves."""
    import ctypes as C
    torch, synth = mods["torch"], mods["synth"]
    cat = synth.make_catalog("c1", n_events=4, n_inj=5000)
    eager = mods["binding"].DarkSirenLikelihood(cat)
    eager.set_option("graph", 0)
    lik = mods["binding"].DarkSirenLikelihood(cat)
    lib = lik.lib
    sizes = (16, 64, 130)
    lam = {B: torch.tensor(synth.draw_lambdas(B, seed=B), device="cuda") for B in sizes}
    out = {B: (torch.empty(B, dtype=torch.float64, device="cuda"), torch.empty(B, 16, dtype=torch.float64, device="cuda"))
           for B in sizes}
    ref = {}
    for B in sizes:
        r = eager.loglike_grad(lam[B])
        ref[B] = (r["logL"].clone(), r["grad"].clone())
    st = torch.cuda.current_stream().cuda_stream
    for B in (16, 64, 16, 130, 64, 16, 130):
        lo, go = out[B]
        rc = lib.dsl_loglike_grad(lik.h, C.c_void_p(lam[B].data_ptr()), B, C.c_void_p(lo.data_ptr()),
                                  C.c_void_p(go.data_ptr()), None, None, None, None, C.c_void_p(st))
        assert rc == 0, lib.dsl_last_error().decode()
        torch.cuda.synchronize()
        assert torch.equal(torch.nan_to_num(lo, neginf=-1e300), torch.nan_to_num(ref[B][0], neginf=-1e300)), B
        assert torch.equal(go, ref[B][1]), B
    log("  7 graph-mode calls over batches 16/64/130 equal eager calls")
    lik.close()
    eager.close()


def test_autograd_function(mods):
    torch, O, synth = mods["torch"], mods["O"], mods["synth"]
    cat = synth.make_catalog("c1", n_events=3, n_inj=3000)
    lik = mods["binding"].DarkSirenLikelihood(cat)
    lam = torch.tensor(synth.fiducial_lambda()[None].repeat(2, 0), device="cuda", requires_grad=True)
    out = lik(lam)
    (out * torch.tensor([1.0, 2.0], device="cuda", dtype=torch.float64)).sum().backward()
    ref = O.loglike(cat, synth.fiducial_lambda(), grad=True)
    g = lam.grad.cpu().numpy()
    np.testing.assert_allclose(g[0], ref["grad"], rtol=1e-4, atol=1e-6 * np.linalg.norm(ref["grad"]))
    np.testing.assert_allclose(g[1], 2 * ref["grad"], rtol=1e-4, atol=2e-6 * np.linalg.norm(ref["grad"]))
    # an input on the CPU: the value comes from the GPU, the gradient returns to the CPU
    lam_cpu = torch.tensor(synth.fiducial_lambda(), dtype=torch.float64, requires_grad=True)
    lik(lam_cpu).sum().backward()
    assert lam_cpu.grad.device.type == "cpu" and lam_cpu.grad.shape == (16,)
    np.testing.assert_allclose(lam_cpu.grad.numpy(), ref["grad"], rtol=1e-4, atol=1e-6 * np.linalg.norm(ref["grad"]))
    lik.close()


def test_autotune_and_cache(mods, tmp_path):
    """The autotuner's choice gives results at parity with the oracle, is
    written to and read back from its cache file (a second handle takes it
    without tuning and reproduces the first bitwise), leaves the caller's
    options as they were, and ignores a cache line it does not launch."""
    torch, O, synth, binding = mods["torch"], mods["O"], mods["synth"], mods["binding"]
    cat = synth.make_catalog("c1", n_events=4, n_inj=5000)
    lam_np = synth.draw_lambdas(16, seed=31)
    lam_np[0] = synth.fiducial_lambda()
    lam = torch.tensor(lam_np, device="cuda")
    cache = tmp_path / "tune.txt"
    a = binding.DarkSirenLikelihood(cat)
    a.set_option("graph", 0)
    a.autotune(16, grad=True, cache_path=str(cache))
    assert a.info("graph") == 0 and a.info("lambda_tile") == 0
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    key, gl, chunk, waves, wg = lines[0].split()
    ra = a.loglike_grad(lam)
    torch.cuda.synchronize()
    assert a.info("lambda_tile_used") == int(gl) and a.info("chunk") == int(chunk)
    log(f"  tuned: tile {gl}, chunk {chunk}, {waves} waves x {wg} per CU")
    for b in (0, 5):
        ref = O.loglike(cat, lam_np[b], grad=True)
        assert rel_close(float(ra["logL"][b]), ref["logL"], TOL_LOGL_FP32)
        check_grad(ra["grad"][b].cpu().numpy(), ref["grad"])
    # a second handle reads the entry (no new line) and reproduces the first
    b2 = binding.DarkSirenLikelihood(cat)
    b2.autotune(16, grad=True, cache_path=str(cache))
    assert len(cache.read_text().splitlines()) == 1
    rb = b2.loglike_grad(lam)
    torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(rb["logL"], neginf=-1e300), torch.nan_to_num(ra["logL"], neginf=-1e300))
    assert torch.equal(rb["grad"], ra["grad"])
    b2.close()
    # a line with a tile this library does not launch is ignored: the tuner runs again
    cache.write_text(f"{key} 3 {chunk} {waves} {wg}\n")
    c = binding.DarkSirenLikelihood(cat)
    c.set_option("lambda_tile", 4)
    c.autotune(16, grad=True, cache_path=str(cache))
    assert len(cache.read_text().splitlines()) == 2
    assert c.info("lambda_tile") == 4
    c.close()
    a.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_event_merge_paths(mods, precision):
    """Events spanning many work items are merged by one wavefront of the
    combine each (16-sample items: about 125 items per event, and several
    combine slices per point, merged by the last slice to finish); a few large
    items per event take the serial merge.  Both against the oracle, with
    gradient."""
    torch, O, synth = mods["torch"], mods["O"], mods["synth"]
    cat = synth.make_catalog("c1", n_events=4, n_inj=5000)
    lam = synth.draw_lambdas(5, seed=61)
    lam[0] = synth.fiducial_lambda()
    refs = [O.loglike(cat, lam[b], grad=True, margins=True) for b in range(len(lam))]
    tol = TOL_LOGL_FP32 if precision == "fp32" else 1e-10
    for chunk in (16, 4096):
        log(f"  [{precision} chunk {chunk}]")
        lik = mods["binding"].DarkSirenLikelihood(cat, precision=precision)
        lik.set_option("lambda_tile", 4)
        lik.set_option("chunk", chunk)
        r = lik.loglike_grad(torch.tensor(lam, device="cuda"), per_event=True)
        torch.cuda.synchronize()
        for b, ref in enumerate(refs):
            assert int(r["flags"][b]) == ref["flags"]
            check_events(r["logL_event"][b].cpu().numpy(), r["neff_event"][b].cpu().numpy(), ref, tol)
            if not ref["flags"]:
                assert rel_close(float(r["logL"][b]), ref["logL"], tol)
                check_grad(r["grad"][b].cpu().numpy(), ref["grad"])
        lik.close()


def test_combine_slice_merge_paths(mods):
    """The slices of a point are merged by the combine slice that finishes last
    in small grids (points x slices <= 64) and by a launch of their own in
    larger ones.  With 16-sample items the 10-event catalogue (20 000 samples,
    10 000 injections) gives the combine several slices per point, the same
    number at 2 and at 40 points, so the two points
    shared by a 2-point call (in-kernel merge) and a 40-point call (separate
    merge) must agree bitwise -- value, gradient and per-event terms -- and
    match the oracle."""
    torch, O, synth = mods["torch"], mods["O"], mods["synth"]
    cat = synth.make_catalog("c1")
    lam = synth.draw_lambdas(40, seed=83)
    lam[0] = synth.fiducial_lambda()
    out = {}
    for B in (2, 40):
        lik = mods["binding"].DarkSirenLikelihood(cat, precision="fp32")
        lik.set_option("lambda_tile", 4)
        lik.set_option("chunk", 16)
        r = lik.loglike_grad(torch.tensor(lam[:B], device="cuda"), per_event=True)
        torch.cuda.synchronize()
        n_items = int(lik.info("n_items"))
        assert n_items > 2 * 256 and (n_items + 255) // 256 <= 32   # 2..32 slices at both B
        out[B] = {k: r[k][:2].cpu().numpy() for k in ("logL", "grad", "logL_event", "neff_event", "flags")}
        lik.close()
    log(f"  {n_items} items")
    for k in out[2]:
        a, b = out[2][k], out[40][k]
        assert np.array_equal(a, b, equal_nan=True) if a.dtype.kind == "f" else np.array_equal(a, b), k
    for b in range(2):
        ref = O.loglike(cat, lam[b], grad=True, margins=True)
        assert int(out[2]["flags"][b]) == ref["flags"]
        check_events(out[2]["logL_event"][b], out[2]["neff_event"][b], ref, TOL_LOGL_FP32)
        if not ref["flags"]:
            assert rel_close(float(out[2]["logL"][b]), ref["logL"], TOL_LOGL_FP32)
            check_grad(out[2]["grad"][b], ref["grad"])


def test_degenerate_catalogues(mods):
    """An event with no pixels and an event whose pixels hold no samples (L_i = 0:
    flag 2, ln L = -inf), and injections all beyond z_max (alpha = 0: flag 4),
    with and without the gradient, against the oracle."""
    import dataclasses
    torch, O, synth = mods["torch"], mods["O"], mods["synth"]
    lam = synth.draw_lambdas(3, seed=67)
    lam[0] = synth.fiducial_lambda()
    base = ragged_catalog(synth, [[64, 65], [], [0, 0], [7]])
    far = dataclasses.replace(base, inj_dl=np.full_like(base.inj_dl, 1e6))
    for name, cat in (("empty events", base), ("alpha = 0", far)):
        log(f"  [{name}]")
        lik = mods["binding"].DarkSirenLikelihood(cat)
        lt = torch.tensor(lam, device="cuda")
        for grad in (False, True):
            r = lik.loglike_grad(lt, per_event=True) if grad else lik.loglike(lt, per_event=True)
            torch.cuda.synchronize()
            for b in range(len(lam)):
                ref = O.loglike(cat, lam[b], margins=True)
                assert int(r["flags"][b]) == ref["flags"] != 0, (name, b, int(r["flags"][b]), ref["flags"])
                assert float(r["logL"][b]) == -math.inf
                ev = r["logL_event"][b].cpu().numpy()
                assert np.array_equal(np.isneginf(ev), np.isneginf(ref["logL_event"]))
                check_events(ev, r["neff_event"][b].cpu().numpy(), ref, TOL_LOGL_FP32)
                if grad:
                    assert not r["grad"][b].any()
        lik.close()


def test_maximum_batch(mods):
    """B = max_batch (4096 points) with the gradient on a small catalogue:
    sampled points against the oracle, both ends of the batch included."""
    torch, O, synth = mods["torch"], mods["O"], mods["synth"]
    cat = synth.make_catalog("c1", n_events=3, n_inj=3000)
    B = 4096
    lam = synth.draw_lambdas(B, seed=71)
    lam[0] = synth.fiducial_lambda()
    lik = mods["binding"].DarkSirenLikelihood(cat)
    assert int(lik.info("max_batch")) == B
    r = lik.loglike_grad(torch.tensor(lam, device="cuda"))
    torch.cuda.synchronize()
    log(f"  tile {int(lik.info('lambda_tile_used'))}, {int(np.isfinite(r['logL'].cpu().numpy()).sum())} finite")
    for b in (0, 1, 63, 64, 2047, 4094, 4095):
        ref = O.loglike(cat, lam[b], grad=True)
        assert int(r["flags"][b]) == ref["flags"], b
        if not ref["flags"]:
            assert rel_close(float(r["logL"][b]), ref["logL"], TOL_LOGL_FP32), b
            check_grad(r["grad"][b].cpu().numpy(), ref["grad"])
    lik.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_delta_m_zero(mods, precision):
    """delta_m = 0, a window of zero width (a step at m_min): ln L, per-event
    values and the gradient against the oracle, whose delta_m entry there is
    the one-sided derivative; the KDE numerator's value as well."""
    torch, O, synth = mods["torch"], mods["O"], mods["synth"]
    cat = synth.make_catalog("c1", n_events=4, n_inj=5000)
    lam = np.stack([synth.lam_vector(delta_m=0.0),
                    synth.lam_vector(delta_m=0.0, mmin=6.0, beta=9.25, alpha=4.0),
                    synth.lam_vector(delta_m=0.0, H0=55.0, Om=0.4, beta=-1.5, mmin=3.0)])
    tol = TOL_LOGL_FP32 if precision == "fp32" else 1e-10
    lik = mods["binding"].DarkSirenLikelihood(cat, precision=precision)
    lt = torch.tensor(lam, device="cuda")
    r = lik.loglike_grad(lt, per_event=True)
    f = lik.loglike(lt)
    torch.cuda.synchronize()
    for b in range(len(lam)):
        ref = O.loglike(cat, lam[b], grad=True, margins=True)
        assert int(r["flags"][b]) == ref["flags"] == 0, (b, int(r["flags"][b]), ref["flags"])
        assert rel_close(float(r["logL"][b]), ref["logL"], tol), (b, float(r["logL"][b]), ref["logL"])
        # the adjoint takes the cell of samples next to a table node from their FP64
        # redshift; the forward sweep's FP32 cell differs there only by rounding
        assert rel_close(float(f["logL"][b]), float(r["logL"][b]), 1e-9)
        check_events(r["logL_event"][b].cpu().numpy(), r["neff_event"][b].cpu().numpy(), ref, tol)
        check_grad(r["grad"][b].cpu().numpy(), ref["grad"])
    lik.close()
    kde = mods["binding"].DarkSirenLikelihood(cat, precision=precision, numerator="kde")
    rk = kde.loglike(lt[:1], per_event=True)
    torch.cuda.synchronize()
    ref = O.loglike_kde(cat, lam[0], margins=True)
    assert int(rk["flags"][0]) == ref["flags"] == 0
    assert rel_close(float(rk["logL"][0]), ref["logL"], tol)
    kde.close()


def test_side_stream_alternating_batches(mods):
    """Calls on a non-blocking side stream, with no synchronisation between
    them, alternating batches of 1 and 64 points: each change of batch size
    rebuilds the work list for another item size while the previous call may
    still run.  Every result equals an eager call on the current stream, with
    graph replay off and on."""
    torch, synth = mods["torch"], mods["synth"]
    cat = synth.make_catalog("c2", n_events=30, n_inj=300_000)
    lam = synth.draw_lambdas(64, seed=83)
    lam[0] = synth.fiducial_lambda()
    lt = torch.tensor(lam, device="cuda")
    eager = mods["binding"].DarkSirenLikelihood(cat)
    eager.set_option("graph", 0)
    r64 = eager.loglike_grad(lt)
    ref64 = r64["logL"].clone(), r64["grad"].clone()
    ref1 = [eager.loglike(lt[i:i + 1])["logL"].clone() for i in range(4)]
    torch.cuda.synchronize()
    eager.close()
    lik = mods["binding"].DarkSirenLikelihood(cat)
    side = torch.cuda.Stream()
    same = lambda a, b: torch.equal(torch.nan_to_num(a, neginf=-1e300), torch.nan_to_num(b, neginf=-1e300))
    n = 0
    for graph in (0, 1):
        lik.set_option("graph", graph)
        outs = []
        for rep in range(3):
            for i in range(4):
                outs.append((i, lik.loglike(lt[i:i + 1], stream=side)))
                outs.append((None, lik.loglike_grad(lt, stream=side)))
        side.synchronize()
        for i, r in outs:
            if i is None:
                assert same(r["logL"], ref64[0]) and torch.equal(r["grad"], ref64[1]), graph
            else:
                assert same(r["logL"], ref1[i]), (graph, i)
            n += 1
    log(f"  {n} unsynchronised side-stream calls alternating B = 1 and 64 equal eager calls")
    lik.close()


def test_downsampling_device_bytes(mods):
    """A cap that binds (64 samples per pixel on a catalogue of about 125 per
    pixel): the handle holds (dropped samples) x (32-byte record + 4-byte order
    index) fewer bytes, apart from a shorter work list (its items cut the kept
    samples into runs), and the capped likelihood equals the oracle's on the
    catalogue downsampled by the same rule."""
    torch, O, synth = mods["torch"], mods["O"], mods["synth"]
    cat = synth.make_catalog("c1")
    full = mods["binding"].DarkSirenLikelihood(cat)
    capped = mods["binding"].DarkSirenLikelihood(cat, max_samples_per_pixel=64, downsample_seed=7)
    kept = int(capped.info("n_samp"))
    ds = O.downsample(cat, 64, seed=7)
    assert kept == ds.n_samp < cat.n_samp
    assert int(capped.info("n_samp_input")) == cat.n_samp
    drop = full.info("device_bytes") - capped.info("device_bytes")
    work = full.info("work_list_bytes") - capped.info("work_list_bytes")
    assert drop - work == (cat.n_samp - kept) * (32 + 4), (drop, work, cat.n_samp, kept)
    log(f"  kept {kept} of {cat.n_samp} samples; device bytes {full.info('device_bytes'):.0f} -> "
        f"{capped.info('device_bytes'):.0f}")
    lam = synth.fiducial_lambda()
    r = capped.loglike(torch.tensor(lam[None], device="cuda"), per_event=True)
    torch.cuda.synchronize()
    ref = O.loglike(ds, lam, margins=True)
    assert int(r["flags"][0]) == ref["flags"] == 0
    assert rel_close(float(r["logL"][0]), ref["logL"], TOL_LOGL_FP32)
    check_events(r["logL_event"][0].cpu().numpy(), r["neff_event"][0].cpu().numpy(), ref, TOL_LOGL_FP32)
    # after a call the footprint still differs by at least the dropped records
    full.loglike(torch.tensor(lam[None], device="cuda"))
    torch.cuda.synchronize()
    assert full.info("device_bytes") - capped.info("device_bytes") >= drop
    full.close()
    capped.close()
