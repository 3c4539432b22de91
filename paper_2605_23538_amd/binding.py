"""ctypes binding of libdsl.so (the C ABI of include/dsl.h).

Argument marshalling only: every step of the likelihood runs in the HIP
kernels behind the ABI.  PyTorch provides device memory and the stream.
There is no CPU fallback: if the library or a GPU is missing this module
raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsl.so")

DSL_PRECISION_FP64 = 0
DSL_PRECISION_FP32 = 1
FLAG_INVALID_LAMBDA = 1
FLAG_EVENT_NO_PIXEL = 2
FLAG_ALPHA_ZERO = 4
FLAG_NONFINITE = 8


class DSLError(RuntimeError):
    pass


class CatalogDesc(C.Structure):
    _fields_ = [
        ("n_events", C.c_int64), ("event_pix_off", C.c_void_p),
        ("n_pix", C.c_int64), ("pix_samp_off", C.c_void_p), ("pix_los_row", C.c_void_p),
        ("n_los_rows", C.c_int64), ("n_z", C.c_int32), ("z_max", C.c_double),
        ("los", C.c_void_p), ("sky_z", C.c_void_p), ("los_f64", C.c_void_p), ("sky_z_f64", C.c_void_p),
        ("n_samp", C.c_int64), ("m1d", C.c_void_p), ("m2d", C.c_void_p), ("dl", C.c_void_p),
        ("ln_pi", C.c_void_p),
        ("n_inj", C.c_int64), ("inj_m1d", C.c_void_p), ("inj_m2d", C.c_void_p), ("inj_dl", C.c_void_p),
        ("inj_ln_pdraw", C.c_void_p), ("n_draw", C.c_int64), ("precision", C.c_int32),
        ("max_samples_per_pixel", C.c_int64), ("downsample_seed", C.c_uint64),
    ]


_lib = None


def load_library(path: Optional[str] = None):
    """Load libdsl.so and declare its entry points (raises if it is missing)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise DSLError(f"{p} not found: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(p)
    vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
    lib.dsl_create.argtypes = [C.POINTER(CatalogDesc), C.POINTER(vp)]
    lib.dsl_create.restype = i32
    lib.dsl_set_option.argtypes = [vp, C.c_char_p, dbl]
    lib.dsl_set_option.restype = i32
    lib.dsl_get_info.argtypes = [vp, C.c_char_p, C.POINTER(dbl)]
    lib.dsl_get_info.restype = i32
    lib.dsl_loglike.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp]
    lib.dsl_loglike.restype = i32
    lib.dsl_loglike_grad.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
    lib.dsl_loglike_grad.restype = i32
    lib.dsl_loglike_grad_noalloc.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
    lib.dsl_loglike_grad_noalloc.restype = i32
    lib.dsl_autotune.argtypes = [vp, i32, i32, C.c_char_p]
    lib.dsl_autotune.restype = i32
    lib.dsl_get_timing.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_float), C.POINTER(C.c_float)]
    lib.dsl_get_timing.restype = i32
    lib.dsl_destroy.argtypes = [vp]
    lib.dsl_destroy.restype = None
    lib.dsl_last_error.argtypes = []
    lib.dsl_last_error.restype = C.c_char_p
    lib.dsl_version.argtypes = []
    lib.dsl_version.restype = C.c_char_p
    if path is None:
        _lib = lib
    return lib


def _check(lib, rc, what):
    if rc != 0:
        raise DSLError(f"{what} failed (code {rc}): {lib.dsl_last_error().decode()}")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class DarkSirenLikelihood:
    """Handle on a catalogue resident on the current GPU.

    catalog: a paper_2605_23538_amd.synth.Catalog (or any object with the same
    CSR arrays).  precision: "fp32" (FP32 weights, FP64 sums) or "fp64".
    numerator: "mc" (per-sample sum over each pixel) or "kde" (the weighted
    Gaussian KDE in redshift of Eq. 6 integrated against the pixel's prior on
    a kde_grid-node grid, bandwidth rule kde_bandwidth; value only).
    """

    def __init__(self, catalog, precision: str = "fp32", neff_min: float = 2.0, gate_mode: int = 0,
                 device: Optional[int] = None, z_prior: str = "los", max_samples_per_pixel: int = 0,
                 downsample_seed: int = 0, numerator: str = "mc", kde_bandwidth: str = "scott",
                 kde_grid: int = 256):
        if not torch.cuda.is_available():
            raise DSLError("a GPU is required (the likelihood runs only in HIP kernels)")
        self.lib = load_library()
        self.device = torch.cuda.current_device() if device is None else int(device)
        prec = {"fp32": DSL_PRECISION_FP32, "fp64": DSL_PRECISION_FP64}[precision]
        self.precision = precision
        self.n_events = int(catalog.n_events)
        # redshift-prior tables go over in their own precision (float64 or float32);
        # the library converts them to the handle's
        tdt = np.float64 if np.asarray(catalog.los).dtype == np.float64 else np.float32
        sdt = np.float64 if np.asarray(catalog.sky_z).dtype == np.float64 else np.float32
        keep = dict(
            epo=_np(catalog.event_pix_off, np.int64), pso=_np(catalog.pix_samp_off, np.int64),
            row=_np(catalog.pix_los_row, np.int32), los=_np(catalog.los, tdt),
            sky=_np(catalog.sky_z, sdt), m1=_np(catalog.m1d, np.float64), m2=_np(catalog.m2d, np.float64),
            dl=_np(catalog.dl, np.float64), lp=_np(catalog.ln_pi, np.float64),
            im1=_np(catalog.inj_m1d, np.float64), im2=_np(catalog.inj_m2d, np.float64),
            idl=_np(catalog.inj_dl, np.float64), ilp=_np(catalog.inj_ln_pdraw, np.float64))
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        d = CatalogDesc(
            n_events=self.n_events, event_pix_off=p(keep["epo"]), n_pix=len(keep["pso"]) - 1,
            pix_samp_off=p(keep["pso"]), pix_los_row=p(keep["row"]), n_los_rows=keep["los"].shape[0],
            n_z=keep["los"].shape[1], z_max=float(catalog.z_max),
            los=p(keep["los"]) if tdt == np.float32 else None, sky_z=p(keep["sky"]) if sdt == np.float32 else None,
            los_f64=p(keep["los"]) if tdt == np.float64 else None,
            sky_z_f64=p(keep["sky"]) if sdt == np.float64 else None,
            n_samp=len(keep["m1"]), m1d=p(keep["m1"]), m2d=p(keep["m2"]), dl=p(keep["dl"]), ln_pi=p(keep["lp"]),
            n_inj=len(keep["im1"]), inj_m1d=p(keep["im1"]), inj_m2d=p(keep["im2"]), inj_dl=p(keep["idl"]),
            inj_ln_pdraw=p(keep["ilp"]), n_draw=int(catalog.n_draw), precision=prec,
            max_samples_per_pixel=int(max_samples_per_pixel), downsample_seed=int(downsample_seed))
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib, self.lib.dsl_create(C.byref(d), C.byref(h)), "dsl_create")
        self.h = h
        self.set_option("neff_min", neff_min)
        self.set_option("gate_mode", gate_mode)
        self.set_option("z_prior", {"los": 0, "comoving": 1}[z_prior])
        self.set_option("numerator", {"mc": 0, "kde": 1}[numerator])
        self.set_option("kde_bandwidth", {"scott": 0, "silverman": 1, "biweight": 2}[kde_bandwidth])
        self.set_option("kde_grid", kde_grid)

    # -- options / info
    def set_option(self, key: str, value: float):
        _check(self.lib, self.lib.dsl_set_option(self.h, key.encode(), float(value)), f"dsl_set_option({key})")

    def info(self, key: str) -> float:
        v = C.c_double()
        _check(self.lib, self.lib.dsl_get_info(self.h, key.encode(), C.byref(v)), f"dsl_get_info({key})")
        return v.value

    def autotune(self, B: int, grad: bool = False, cache_path: Optional[str] = None):
        with torch.cuda.device(self.device):
            _check(self.lib, self.lib.dsl_autotune(self.h, int(B), int(bool(grad)),
                                                   cache_path.encode() if cache_path else None), "dsl_autotune")

    def timing(self):
        a, b, c = C.c_float(), C.c_float(), C.c_float()
        _check(self.lib, self.lib.dsl_get_timing(self.h, C.byref(a), C.byref(b), C.byref(c)), "dsl_get_timing")
        return a.value, b.value, c.value

    # -- evaluation
    def _lam(self, lam: torch.Tensor) -> torch.Tensor:
        if lam.dim() == 1:
            lam = lam.unsqueeze(0)
        if lam.shape[-1] != 16:
            raise ValueError("lambda must have 16 columns")
        return lam.detach().to(device=f"cuda:{self.device}", dtype=torch.float64).contiguous()

    @staticmethod
    def _stream(stream, dev):
        """The launch stream.  A stream other than the current one first waits for
        the current stream, where the inputs and outputs were prepared; the
        caller synchronises with it before reading the results."""
        cur = torch.cuda.current_stream(dev)
        if stream is None or stream == cur:
            return cur, False
        stream.wait_stream(cur)
        return stream, True

    @staticmethod
    def _keep(tensors, stream):
        # the caching allocator must not reuse these blocks before `stream` is done
        for t in tensors:
            if t is not None:
                t.record_stream(stream)

    def loglike(self, lam: torch.Tensor, per_event: bool = False, stream=None):
        """ln L for a [B, 16] batch; dict of device tensors (written on `stream`,
        default the current stream)."""
        lam = self._lam(lam)
        B = lam.shape[0]
        dev = lam.device
        out = dict(logL=torch.empty(B, dtype=torch.float64, device=dev),
                   neff_sel=torch.empty(B, dtype=torch.float64, device=dev),
                   flags=torch.empty(B, dtype=torch.int32, device=dev))
        if per_event:
            out["logL_event"] = torch.empty(B, self.n_events, dtype=torch.float64, device=dev)
            out["neff_event"] = torch.empty(B, self.n_events, dtype=torch.float64, device=dev)
        s, side = self._stream(stream, dev)
        rc = self.lib.dsl_loglike(self.h, _ptr(lam), B, _ptr(out["logL"]), _ptr(out.get("logL_event")),
                                  _ptr(out.get("neff_event")), _ptr(out["neff_sel"]), _ptr(out["flags"]),
                                  C.c_void_p(s.cuda_stream))
        if side:
            self._keep([lam, *out.values()], s)
        _check(self.lib, rc, "dsl_loglike")
        return out

    def loglike_grad(self, lam: torch.Tensor, per_event: bool = False, stream=None):
        """ln L and d ln L / d Lambda [B, 16] (adjoint sweep); dict of device tensors
        (written on `stream`, default the current stream)."""
        lam = self._lam(lam)
        B = lam.shape[0]
        dev = lam.device
        out = dict(logL=torch.empty(B, dtype=torch.float64, device=dev),
                   grad=torch.empty(B, 16, dtype=torch.float64, device=dev),
                   neff_sel=torch.empty(B, dtype=torch.float64, device=dev),
                   flags=torch.empty(B, dtype=torch.int32, device=dev))
        if per_event:
            out["logL_event"] = torch.empty(B, self.n_events, dtype=torch.float64, device=dev)
            out["neff_event"] = torch.empty(B, self.n_events, dtype=torch.float64, device=dev)
        s, side = self._stream(stream, dev)
        rc = self.lib.dsl_loglike_grad(self.h, _ptr(lam), B, _ptr(out["logL"]), _ptr(out["grad"]),
                                       _ptr(out.get("logL_event")), _ptr(out.get("neff_event")),
                                       _ptr(out["neff_sel"]), _ptr(out["flags"]), C.c_void_p(s.cuda_stream))
        if side:
            self._keep([lam, *out.values()], s)
        _check(self.lib, rc, "dsl_loglike_grad")
        return out

    def loglike_grad_noalloc(self, lam: torch.Tensor, out: dict, stream=None):
        """loglike_grad into caller-provided device tensors `out` (logL [B], grad
        [B, 16]; optional logL_event / neff_event [B, n_events], neff_sel [B],
        flags [B] int32), through the entry point that allocates no device memory
        (its workspace is the library's static per-GPU scratch).  `lam` must be a
        contiguous float64 [B, 16] tensor on the handle's device."""
        if lam.dtype != torch.float64 or not lam.is_contiguous() or lam.dim() != 2 or lam.shape[1] != 16:
            raise ValueError("lam must be a contiguous float64 [B, 16] device tensor")
        B = lam.shape[0]
        dev = lam.device
        s, side = self._stream(stream, dev)
        rc = self.lib.dsl_loglike_grad_noalloc(
            self.h, _ptr(lam), B, _ptr(out["logL"]), _ptr(out["grad"]), _ptr(out.get("logL_event")),
            _ptr(out.get("neff_event")), _ptr(out.get("neff_sel")), _ptr(out.get("flags")),
            C.c_void_p(s.cuda_stream))
        if side:
            self._keep([lam, *out.values()], s)
        _check(self.lib, rc, "dsl_loglike_grad_noalloc")
        return out

    def __call__(self, lam: torch.Tensor) -> torch.Tensor:
        """Differentiable ln L (torch.autograd; the backward recomputes the weights)."""
        return LogLFunction.apply(lam, self)

    def close(self):
        if getattr(self, "h", None):
            self.lib.dsl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LogLFunction(torch.autograd.Function):
    """ln L(Lambda) with the hand-written adjoint as its backward."""

    @staticmethod
    def forward(ctx, lam, lik):
        ctx.lik = lik
        ctx.save_for_backward(lam)
        return lik.loglike(lam)["logL"]

    @staticmethod
    def backward(ctx, g):
        (lam,) = ctx.saved_tensors
        r = ctx.lik.loglike_grad(lam)
        grad = r["grad"] * g.to(device=r["grad"].device, dtype=r["grad"].dtype).reshape(-1)[:, None]
        if lam.dim() == 1:
            grad = grad[0]
        # the gradient goes back to the input's device and dtype (a CPU input is valid)
        return grad.to(device=lam.device, dtype=lam.dtype), None
