"""Writes the expected values of the whole O5-like workload for chosen points.

The O5-like catalogue (5000 events, U[1000, 8192] samples each, 32-2048 pixels
of 1024-node redshift tables, 1e7 detected injections; the seeded generator of
paper_2605_23538_amd.synth) is evaluated by the FP64 oracle alone for points of
the benchmark's 64-point batch: every event's ln L_i and N_eff,i, ln alpha,
N_eff of the selection term, ln L and the 16-entry gradient (Sec. II A,
Eqs. 3-5, 7, 8), with the per-event margins of the gate and support decisions
and each event's sensitivity to its inputs at FP32 reach (event_fp32_cond for
ln L_i, event_fp32_cond_neff for the relative N_eff,i).

A pixel whose ln N_eff lies within AMB of ln N_min is a decision that a path
working in another precision may take the other way (Eq. 8).  For every event
holding such pixels the file also lists each combination of their outcomes
with the event's ln L_i and the change of the gradient it brings, so a parity
test can recognise the combination the other path took (by its ln L_i) and
compare the rest exactly.  Nothing here runs on a GPU or reads a GPU result.

    python tests/golden/make_c4_golden.py --points 0 1 --gate-modes 0 2

writes tests/golden/c4_point<b>_gate<g>.npz (load with numpy.load,
allow_pickle=False).
"""
import argparse
import itertools
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import dsl_oracle as O  # noqa: E402
from paper_2605_23538_amd import synth  # noqa: E402

AMB = 1e-4          # |ln N_eff - ln N_min| below which a pixel's gate decision is listed
MAX_AMB_PER_EVENT = 6


def gate_alternatives(cat, lam, pix_margin, gate_mode):
    """Rows (event, combination mask, ln L_i, gradient change) for the events
    with pixels near the gate threshold; mask bit k inverts the oracle's
    decision for the event's k-th such pixel."""
    ev, mask, lnl, dg, pix_list, pix_ev = [], [], [], [], [], []
    if gate_mode == 2:
        return (np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0), np.zeros((0, 16)),
                np.zeros(0, np.int64), np.zeros(0, np.int64))
    amb = np.flatnonzero(pix_margin < AMB)
    ev_of = np.searchsorted(cat.event_pix_off, amb, side="right") - 1
    for e in np.unique(ev_of):
        pids = amb[ev_of == e]
        if len(pids) > MAX_AMB_PER_EVENT:
            raise RuntimeError(f"event {e}: {len(pids)} pixels near the gate threshold")
        pix_list.extend(pids.tolist())
        pix_ev.extend([int(e)] * len(pids))
        sub = cat.subset([int(e)], inj=slice(0, 1))
        local = pids - int(cat.event_pix_off[e])
        base = None
        for bits in itertools.product((0, 1), repeat=len(pids)):
            m = sum(b << k for k, b in enumerate(bits))
            r = O.loglike(sub, lam, grad=True, gate_mode=gate_mode, gate_flip=local[np.array(bits, bool)])
            g = np.asarray(r["grad"], np.float64) if r["flags"] == 0 else np.full(16, np.nan)
            if m == 0:
                base = g
            ev.append(int(e))
            mask.append(m)
            lnl.append(float(r["logL_event"][0]))
            dg.append(g - base)
    return (np.asarray(ev, np.int64), np.asarray(mask, np.int64), np.asarray(lnl, np.float64),
            np.asarray(dg, np.float64).reshape(-1, 16), np.asarray(pix_list, np.int64),
            np.asarray(pix_ev, np.int64))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--points", type=int, nargs="+", default=[0, 1])
    ap.add_argument("--gate-modes", type=int, nargs="+", default=[0])
    ap.add_argument("--out", default=HERE)
    a = ap.parse_args()
    t0 = time.time()
    cat = synth.make_catalog("c4")
    lam = synth.lambdas_for("c4")
    print(f"c4 generated in {time.time() - t0:.0f} s: {cat.n_events} events, {cat.n_samp} samples, "
          f"{cat.n_inj} injections", flush=True)
    for b in a.points:
        for gm in a.gate_modes:
            t0 = time.time()
            r = O.loglike(cat, lam[b], grad=True, margins=True, gate_mode=gm)
            alt = gate_alternatives(cat, lam[b], r["pixel_gate_margin"], gm)
            path = os.path.join(a.out, f"c4_point{b}_gate{gm}.npz")
            np.savez_compressed(
                path, lam=lam[b], point=np.int64(b), gate_mode=np.int64(gm), neff_min=np.float64(2.0),
                logL=np.float64(r["logL"]), flags=np.int64(r["flags"]),
                ln_alpha=np.float64(r.get("ln_alpha", -np.inf)), neff_sel=np.float64(r["neff_sel"]),
                grad=np.asarray(r["grad"], np.float64), logL_event=np.asarray(r["logL_event"], np.float64),
                neff_event=np.asarray(r["neff_event"], np.float64),
                event_fp32_cond=np.asarray(r["event_fp32_cond"], np.float64),
                event_fp32_cond_neff=np.asarray(r["event_fp32_cond_neff"], np.float64),
                gate_margin=np.asarray(r["gate_margin"], np.float32),
                sample_margin=np.asarray(r["sample_margin"], np.float32),
                inj_margin=np.float64(r["inj_margin"]), amb_margin=np.float64(AMB),
                alt_event=alt[0], alt_mask=alt[1], alt_logL_event=alt[2], alt_dgrad=alt[3],
                amb_pixel=alt[4], amb_pixel_event=alt[5])
            print(f"point {b} gate {gm}: ln L {r['logL']!r} flags {r['flags']}, {len(alt[4])} pixels near the "
                  f"gate in {len(np.unique(alt[5]))} events, min sample margin {np.min(r['sample_margin']):.2e}, "
                  f"{time.time() - t0:.0f} s -> {os.path.basename(path)}", flush=True)


if __name__ == "__main__":
    main()
