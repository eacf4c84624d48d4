"""Python binding of the gfx950 library ``libkx.so`` (argument marshalling only).

Every computation runs in the library's HIP kernels; this module only turns
numpy mechanism arrays into a ``kx_mech_desc``, torch device tensors into
pointers and torch streams into ``hipStream_t``.  There is no CPU fallback:
if the library has not been built, importing it raises.

torch is imported first so that the library binds to the HIP runtime torch
already loaded (both use the soname libamdhip64.so.7): device pointers and
streams are then shared.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkx.so")

KX_OK, KX_EINVAL, KX_ENOMEM, KX_EDEVICE, KX_EUNSUPPORTED, KX_EAGAIN = 0, -1, -2, -3, -4, -5
KX_FP64, KX_MIXED = 0, 1
PRECISION = {"fp64": KX_FP64, "mixed": KX_MIXED}


class KxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"kx error {code}: {msg}")
        self.code = code


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class _Desc(C.Structure):
    _fields_ = [
        ("n_species", C.c_int32), ("n_reactions", C.c_int32), ("n_elements", C.c_int32),
        ("elem_mass", _dp), ("composition", _ip), ("nasa_lo", _dp), ("nasa_hi", _dp),
        ("t_mid", _dp), ("rxn_type", _ip), ("reversible", _ip),
        ("reac_ptr", _ip), ("reac_sp", _ip), ("reac_nu", _ip),
        ("prod_ptr", _ip), ("prod_sp", _ip), ("prod_nu", _ip),
        ("A", _dp), ("beta", _dp), ("Ea", _dp), ("A0", _dp), ("beta0", _dp), ("Ea0", _dp),
        ("troe", _dp), ("eff_ptr", _ip), ("eff_sp", _ip), ("eff_val", _dp),
        ("eff_default", _dp), ("fit_order", C.c_int32), ("fit_L0", C.c_double),
        ("fit_h", C.c_double), ("diff_fit_kind", C.c_int32),
        ("visc_fit", _dp), ("cond_fit", _dp), ("diff_fit", _dp),
    ]


_F64_FIELDS = ["elem_mass", "nasa_lo", "nasa_hi", "t_mid", "A", "beta", "Ea", "A0", "beta0",
               "Ea0", "troe", "eff_val", "eff_default", "visc_fit", "cond_fit", "diff_fit"]
_I32_FIELDS = ["composition", "rxn_type", "reversible", "reac_ptr", "reac_sp", "reac_nu",
               "prod_ptr", "prod_sp", "prod_nu", "eff_ptr", "eff_sp"]

_lib = None


def lib():
    """Load libkx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2411_02640_amd.build`")
        L = C.CDLL(LIB_PATH, mode=C.RTLD_GLOBAL)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.kx_mech_create.argtypes = [C.POINTER(_Desc), C.c_int, C.POINTER(vp)]
        L.kx_mech_destroy.argtypes = [vp]
        L.kx_mech_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i64)]
        L.kx_production_rates.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.kx_production_rates_ex.argtypes = [vp, i64, vp, vp, vp, vp, i32, vp]
        L.kx_transport.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
        L.kx_transport_ex.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, i32, vp]
        L.kx_thermo.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
        L.kx_last_error.restype = C.c_char_p
        L.kx_version.restype = C.c_char_p
        for name in ("kx_mech_create", "kx_mech_destroy", "kx_mech_info", "kx_production_rates",
                     "kx_production_rates_ex", "kx_transport", "kx_transport_ex", "kx_thermo"):
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def check(code: int) -> None:
    if code != KX_OK:
        raise KxError(code, lib().kx_last_error().decode())


def version() -> str:
    return lib().kx_version().decode()


def make_desc(mech: dict):
    """Build a kx_mech_desc pointing at contiguous copies of the arrays.

    Returns (desc, keepalive); the arrays must outlive the create call only.
    """
    keep = {}
    d = _Desc()
    d.n_species = int(mech["n_species"])
    d.n_reactions = int(mech["n_reactions"])
    d.n_elements = int(mech["n_elements"])
    for k in _F64_FIELDS:
        a = np.ascontiguousarray(mech[k], dtype=np.float64)
        keep[k] = a
        setattr(d, k, a.ctypes.data_as(_dp))
    for k in _I32_FIELDS:
        a = np.ascontiguousarray(mech[k], dtype=np.int32)
        if a.size == 0:
            a = np.zeros(1, np.int32)
        keep[k] = a
        setattr(d, k, a.ctypes.data_as(_ip))
    d.fit_order = int(mech["fit_order"])
    d.fit_L0 = float(mech["fit_L0"])
    d.fit_h = float(mech["fit_h"])
    d.diff_fit_kind = int(mech["diff_fit_kind"])
    return d, keep


class Mechanism:
    """A mechanism resident on one GPU (wraps kx_mech_create / destroy)."""

    def __init__(self, mech: dict, device: int = 0):
        d, keep = make_desc(mech)
        h = C.c_void_p()
        check(lib().kx_mech_create(C.byref(d), int(device), C.byref(h)))
        del keep
        self.handle = h
        self.device = int(device)
        ns, nr, nb = C.c_int32(), C.c_int32(), C.c_int64()
        check(lib().kx_mech_info(h, C.byref(ns), C.byref(nr), C.byref(nb)))
        self.n_species, self.n_reactions, self.device_bytes = ns.value, nr.value, nb.value
        self.name = mech.get("name", "")

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            check(lib().kx_mech_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_ptr(stream, device):
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return C.c_void_p(stream.cuda_stream)


def _dev_tensor(t, device, shape, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.device.index != device:
        raise ValueError(f"{name} must be a torch tensor on cuda:{device}")
    if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be a contiguous float64 tensor of shape {shape}")
    return C.c_void_p(t.data_ptr())


def production_rates(mech: Mechanism, T, p, Y, out=None, precision: str = "fp64",
                     stream=None):
    """wdot[Ns, n] for device tensors T[n], p[n], Y[Ns, n] (enqueued on `stream`)."""
    n = T.shape[0]
    ns = mech.n_species
    dev = mech.device
    args = [_dev_tensor(T, dev, (n,), "T"), _dev_tensor(p, dev, (n,), "p"),
            _dev_tensor(Y, dev, (ns, n), "Y")]
    if out is None:
        out = torch.empty((ns, n), dtype=torch.float64, device=f"cuda:{dev}")
    w = _dev_tensor(out, dev, (ns, n), "out")
    check(lib().kx_production_rates_ex(mech.handle, n, *args, w, PRECISION[precision],
                                       _stream_ptr(stream, dev)))
    return out


def transport(mech: Mechanism, T, p, Y, out=None, precision: str = "fp64", stream=None):
    """(mu[n], lambda[n], Dmix[Ns, n]) for device tensors T, p, Y."""
    n = T.shape[0]
    ns = mech.n_species
    dev = mech.device
    args = [_dev_tensor(T, dev, (n,), "T"), _dev_tensor(p, dev, (n,), "p"),
            _dev_tensor(Y, dev, (ns, n), "Y")]
    if out is None:
        kw = dict(dtype=torch.float64, device=f"cuda:{dev}")
        out = (torch.empty(n, **kw), torch.empty(n, **kw), torch.empty((ns, n), **kw))
    mu, lam, Dm = out
    ptrs = [_dev_tensor(mu, dev, (n,), "mu"), _dev_tensor(lam, dev, (n,), "lambda"),
            _dev_tensor(Dm, dev, (ns, n), "Dmix")]
    check(lib().kx_transport_ex(mech.handle, n, *args, *ptrs, PRECISION[precision],
                                _stream_ptr(stream, dev)))
    return out


def thermo(mech: Mechanism, T, Y, stream=None):
    """(cp_k[Ns, n], h_k[Ns, n], cp_mix[n]) for device tensors T, Y."""
    n = T.shape[0]
    ns = mech.n_species
    dev = mech.device
    kw = dict(dtype=torch.float64, device=f"cuda:{dev}")
    cpk, hk, cp = torch.empty((ns, n), **kw), torch.empty((ns, n), **kw), torch.empty(n, **kw)
    check(lib().kx_thermo(mech.handle, n, _dev_tensor(T, dev, (n,), "T"),
                          _dev_tensor(Y, dev, (ns, n), "Y"), C.c_void_p(cpk.data_ptr()),
                          C.c_void_p(hk.data_ptr()), C.c_void_p(cp.data_ptr()),
                          _stream_ptr(stream, dev)))
    return cpk, hk, cp
