"""The allocation-free gradient entry point against dsl_loglike_grad and the
oracle, through the C ABI: two calls in a row, the second with a smaller
batch, with no device memory taken by the handle in between."""
import math

import numpy as np
import pytest

from tests.gpu_common import TOL_LOGL_FP32, check_grad, log, need_gpu, rel_close, support_ambiguous

pytestmark = pytest.mark.gpu


def _outs(torch, B, n_events):
    f = lambda *shape: torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
    return dict(logL=f(B), grad=f(B, 16), logL_event=f(B, n_events), neff_event=f(B, n_events), neff_sel=f(B),
                flags=torch.full((B,), -1, dtype=torch.int32, device="cuda"))


def test_noalloc_matches_allocating_entry_point():
    need_gpu()
    import torch
    from oracle import dsl_oracle as O
    from paper_2605_23538_amd import binding, synth
    cat = synth.make_catalog("c1")
    lam = synth.draw_lambdas(24, seed=77)
    lam[0] = synth.fiducial_lambda()
    # a fresh handle for the allocation-free calls: nothing but the catalogue and
    # its work list is allocated before them, and nothing after
    lik = binding.DarkSirenLikelihood(cat, precision="fp32")
    ref_lik = binding.DarkSirenLikelihood(cat, precision="fp32")
    bytes0 = lik.info("device_bytes")
    for B in (24, 5):   # the second call is smaller
        log(f"[no-alloc gradient, c1 catalogue, B={B}]")
        lt = torch.tensor(lam[:B], device="cuda")
        out = lik.loglike_grad_noalloc(lt, _outs(torch, B, cat.n_events))
        ref = ref_lik.loglike_grad(lt, per_event=True)
        torch.cuda.synchronize()
        assert lik.info("device_bytes") == bytes0
        assert torch.equal(out["flags"], ref["flags"])
        # the same kernels, possibly another cut of the sums into work items:
        # equal to the parity bar (ln L to 1e-6, N_eff to 1e-5, gradient to 1e-4)
        for k, rtol in (("logL", TOL_LOGL_FP32), ("logL_event", TOL_LOGL_FP32), ("neff_event", 1e-5),
                        ("neff_sel", 1e-5)):
            a, r = out[k].cpu().numpy(), ref[k].cpu().numpy()
            fin = np.isfinite(r)
            assert np.array_equal(np.isfinite(a), fin), k
            assert np.all(a[~fin] == r[~fin]), k
            assert np.all(np.abs(a[fin] - r[fin]) <= rtol * np.maximum(1.0, np.abs(r[fin]))), k
        ga, gr_ref = out["grad"].cpu().numpy(), ref["grad"].cpu().numpy()
        for b in range(B):
            if math.isfinite(float(ref["logL"][b])):
                check_grad(ga[b], gr_ref[b])
            else:
                assert np.all(ga[b] == 0.0)
        lg = out["logL"].cpu().numpy()
        gr = out["grad"].cpu().numpy()
        for b in (0, 1, B - 1):
            o = O.loglike(cat, lam[b], grad=True, margins=True)
            if o["flags"]:
                assert lg[b] == -math.inf
                continue
            assert rel_close(float(lg[b]), o["logL"], TOL_LOGL_FP32)
            if not support_ambiguous(o):   # (point 23 has an injection at d_L(z_max))
                check_grad(gr[b], o["grad"])
    lik.close()
    ref_lik.close()


def test_noalloc_rejects_a_batch_beyond_the_scratch():
    """A workspace larger than the static scratch is refused with a clear error."""
    need_gpu()
    import torch
    from paper_2605_23538_amd import binding, synth
    cat = synth.make_catalog("c2")
    lik = binding.DarkSirenLikelihood(cat, precision="fp32")
    lik.set_option("max_batch", 4096)
    B = 4096
    lt = torch.tensor(synth.draw_lambdas(B, seed=3), device="cuda")
    bytes0 = lik.info("device_bytes")
    with pytest.raises(binding.DSLError, match="MiB scratch"):
        lik.loglike_grad_noalloc(lt, _outs(torch, B, cat.n_events))
    assert lik.info("device_bytes") == bytes0
    lik.close()
