"""Host-side checks of the C ABI (no GPU compute): the library loads, exports
every entry point include/dsl.h declares, and rejects malformed input before
touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from tests.gpu_common import LIB, ROOT

HEADER = os.path.join(ROOT, "include", "dsl.h")


def _lib():
    if not os.path.exists(LIB):
        pytest.skip("libdsl.so not built")
    from paper_2605_23538_amd import binding
    return binding, binding.load_library()


def test_exports_every_declared_symbol():
    binding, lib = _lib()
    src = open(HEADER).read()
    names = sorted(set(re.findall(r"\b(dsl_[a-z_]+)\s*\(", src)))
    assert "dsl_create" in names and "dsl_loglike_grad" in names
    for n in names:
        assert hasattr(lib, n), n
    assert lib.dsl_version().decode().startswith("dsl")


def test_header_layout_matches_binding():
    """The ctypes mirror of dsl_catalog_desc has the C field order."""
    binding, _ = _lib()
    src = open(HEADER).read()
    body = src[src.index("typedef struct dsl_catalog_desc"):src.index("} dsl_catalog_desc;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    c_fields = re.findall(r"\b(\w+);", body)
    assert [f for f, _ in binding.CatalogDesc._fields_] == c_fields


def _desc(binding, tables="f32", **over):
    """A valid one-event descriptor; `tables` gives the redshift-prior tables in
    float32 ("f32"), float64 ("f64"), both or neither."""
    epo = np.array([0, 2], np.int64)
    pso = np.array([0, 1, 3], np.int64)
    row = np.array([0, 0], np.int32)
    los = np.ones(8, np.float32)
    sky = np.ones(8, np.float32)
    s = np.array([30.0, 35.0, 40.0])
    keep = dict(epo=epo, pso=pso, row=row, los=los, sky=sky, los64=los.astype(np.float64),
                sky64=sky.astype(np.float64), m1=s, m2=s * 0.5, dl=s * 40, lp=s * 0,
                im1=s, im2=s * 0.5, idl=s * 40, ilp=s * 0)
    keep.update(over)
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    f32, f64 = tables in ("f32", "both"), tables in ("f64", "both")
    d = binding.CatalogDesc(n_events=1, event_pix_off=p(keep["epo"]), n_pix=2, pix_samp_off=p(keep["pso"]),
                            pix_los_row=p(keep["row"]), n_los_rows=1, n_z=8, z_max=2.0,
                            los=p(keep["los"]) if f32 else None, sky_z=p(keep["sky"]) if f32 else None,
                            los_f64=p(keep["los64"]) if f64 else None, sky_z_f64=p(keep["sky64"]) if f64 else None,
                            n_samp=3, m1d=p(keep["m1"]), m2d=p(keep["m2"]), dl=p(keep["dl"]),
                            ln_pi=p(keep["lp"]), n_inj=3, inj_m1d=p(keep["im1"]), inj_m2d=p(keep["im2"]),
                            inj_dl=p(keep["idl"]), inj_ln_pdraw=p(keep["ilp"]), n_draw=10, precision=1)
    return d, keep


@pytest.mark.parametrize("over,msg", [
    (dict(pso=np.array([0, 2, 1], np.int64)), "pix_samp_off"),
    (dict(row=np.array([0, 5], np.int32)), "pix_los_row"),
    (dict(m1=np.array([30.0, float("nan"), 40.0])), "finite"),
    (dict(dl=np.array([30.0, -1.0, 40.0])), "finite"),
    (dict(los=np.array([1, 1, 1, -1, 1, 1, 1, 1], np.float32)), "LOS"),
    (dict(ilp=np.array([0.0, float("inf"), 0.0])), "inj_ln_pdraw"),
    (dict(epo=np.array([0, 1], np.int64)), "event_pix_off"),
])
def test_create_rejects_malformed_catalogue(over, msg):
    binding, lib = _lib()
    d, keep = _desc(binding, **over)
    h = C.c_void_p()
    rc = lib.dsl_create(C.byref(d), C.byref(h))
    assert rc == 1 and not h.value
    assert msg in lib.dsl_last_error().decode()


@pytest.mark.parametrize("tables,over,msg", [
    ("both", {}, "exactly one"),
    ("none", {}, "exactly one"),
    ("f64", dict(los64=np.array([1, 1, 1, float("nan"), 1, 1, 1, 1])), "LOS"),
    ("f64", dict(sky64=np.array([1, 1, 1, 1, 1, 1, 1, -1.0])), "sky_z"),
])
def test_create_checks_table_precision_choice(tables, over, msg):
    """The tables come in float32 or in float64, never both; float64 tables are
    checked like float32 ones."""
    binding, lib = _lib()
    d, keep = _desc(binding, tables=tables, **over)
    h = C.c_void_p()
    assert lib.dsl_create(C.byref(d), C.byref(h)) == 1 and not h.value
    assert msg in lib.dsl_last_error().decode()


def test_null_arguments():
    binding, lib = _lib()
    h = C.c_void_p()
    assert lib.dsl_create(None, C.byref(h)) == 1
    assert lib.dsl_set_option(None, b"neff_min", 2.0) == 4
    assert lib.dsl_loglike(None, None, 1, None, None, None, None, None, None) == 4
    assert lib.dsl_get_timing(None, None, None, None) == 4
    lib.dsl_destroy(None)


@pytest.mark.parametrize("field,value,msg", [
    ("n_events", 0, "n_events"),
    ("n_inj", 0, "injection"),
    ("n_draw", 2, "n_draw"),
    ("n_z", 1, "n_z"),
    ("n_z", (1 << 24) + 1, "2^24"),
    ("n_events", 1 << 31, "too many events"),
    ("n_pix", 1 << 31, "too many pixels"),
    ("precision", 7, "precision"),
    ("max_samples_per_pixel", -1, "max_samples_per_pixel"),
])
def test_create_rejects_bad_sizes(field, value, msg):
    """Descriptor sizes out of range are rejected before anything is uploaded."""
    binding, lib = _lib()
    d, keep = _desc(binding)
    setattr(d, field, value)
    h = C.c_void_p()
    assert lib.dsl_create(C.byref(d), C.byref(h)) == 1 and not h.value
    assert msg in lib.dsl_last_error().decode()


def test_binding_requires_a_gpu():
    """No fallback: without a GPU the binding refuses to build a likelihood."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2605_23538_amd import binding, synth
    cat = synth.make_catalog("c1", n_events=2, n_inj=100)
    with pytest.raises(binding.DSLError, match="GPU"):
        binding.DarkSirenLikelihood(cat)


def test_bench_refuses_several_gpus():
    """bench.py runs on one GPU: --gpus 2 exits with a message before any GPU work."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]
