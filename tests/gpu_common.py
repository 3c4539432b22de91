"""Helpers shared by the GPU tests (parity of the HIP path with the oracle)."""
import math
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2605_23538_amd", "libdsl.so")

# Relative tolerance on ln L of the FP32-bulk path (the accuracy the method must
# meet) and of the FP64 path, which is held far tighter than that bound.
TOL_LOGL_FP32 = 1e-6
TOL_LOGL_FP64 = 1e-10
# Gradient: |g - g_ref| <= 1e-4 max(|g_ref|, 1e-2 ||g_ref||) per component.
TOL_GRAD = 1e-4
# Decisions taken in another precision: events with a pixel whose N_eff lies
# within this relative distance of the threshold, or a sample within this
# relative distance of a support edge (d_L(z_max), m_max), are checked against
# both outcomes only through the total (see check_events).
GATE_MARGIN = 1e-5
SAMPLE_MARGIN = 1e-5


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(LIB):
        pytest.fail("libdsl.so is not built (run __graft_entry__.build())")


def log(msg):
    print(msg, flush=True)


def rel_close(a, b, rtol):
    if math.isinf(a) or math.isinf(b):
        return a == b
    return abs(a - b) <= rtol * max(1.0, abs(b))


def ambiguous_events(ref):
    gm = ref.get("gate_margin")
    sm = ref.get("sample_margin")
    if gm is None:
        return np.zeros(len(ref["logL_event"]), bool)
    return (gm < GATE_MARGIN) | (sm < SAMPLE_MARGIN)


def check_events(got_ev, got_neff, ref, rtol, neff_rtol=1e-5):
    """Per-event ln L_i and N_eff,i against the oracle; returns #ambiguous."""
    amb = ambiguous_events(ref)
    for i, (g, r) in enumerate(zip(got_ev, ref["logL_event"])):
        if amb[i]:
            continue
        assert rel_close(float(g), float(r), rtol), (i, g, r)
        rn = ref["neff_event"][i]
        assert abs(got_neff[i] - rn) <= neff_rtol * max(1.0, rn), (i, got_neff[i], rn)
    return int(amb.sum())


def check_grad(g, gr):
    g = np.asarray(g)
    gr = np.asarray(gr)
    tol = TOL_GRAD * np.maximum(np.abs(gr), 1e-2 * np.linalg.norm(gr))
    bad = np.abs(g - gr) > tol
    assert not bad.any(), (np.flatnonzero(bad), g[bad], gr[bad])
