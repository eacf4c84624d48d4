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
# KX_LIBRARY names another build of the same library (the thread-sanitizer
# build of the host code, for instance); the default is the in-tree libkx.so.
LIB_PATH = os.environ.get("KX_LIBRARY") or os.path.join(HERE, "libkx.so")

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
        ("sri", _dp), ("chem_act", _ip), ("plog_ptr", _ip), ("plog_p", _dp),
        ("plog_A", _dp), ("plog_beta", _dp), ("plog_Ea", _dp),
        ("ord_ptr", _ip), ("ord_sp", _ip), ("ord_val", _dp), ("qss", _ip),
    ]


_F64_FIELDS = ["elem_mass", "nasa_lo", "nasa_hi", "t_mid", "A", "beta", "Ea", "A0", "beta0",
               "Ea0", "troe", "eff_val", "eff_default", "visc_fit", "cond_fit", "diff_fit"]
_I32_FIELDS = ["composition", "rxn_type", "reversible", "reac_ptr", "reac_sp", "reac_nu",
               "prod_ptr", "prod_sp", "prod_nu", "eff_ptr", "eff_sp"]

# Optional arrays of the further reaction forms (NULL when a mechanism has none).
_OPT_F64_FIELDS = ["sri", "plog_p", "plog_A", "plog_beta", "plog_Ea", "ord_val"]
_OPT_I32_FIELDS = ["chem_act", "plog_ptr", "ord_ptr", "ord_sp", "qss"]

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
        L.kx_jacobian.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.kx_qss_concentrations.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.kx_last_error.restype = C.c_char_p
        L.kx_version.restype = C.c_char_p
        for name in ("kx_mech_create", "kx_mech_destroy", "kx_mech_info", "kx_production_rates",
                     "kx_production_rates_ex", "kx_transport", "kx_transport_ex", "kx_thermo",
                     "kx_jacobian", "kx_qss_concentrations"):
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
    for k, dt, ptr in ([(k, np.float64, _dp) for k in _OPT_F64_FIELDS] +
                       [(k, np.int32, _ip) for k in _OPT_I32_FIELDS]):
        if mech.get(k) is None:
            setattr(d, k, None)
            continue
        a = np.ascontiguousarray(mech[k], dtype=dt)
        if a.size == 0:
            a = np.zeros(1, dt)
        keep[k] = a
        setattr(d, k, a.ctypes.data_as(ptr))
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
        q = mech.get("qss")
        self.n_qss = 0 if q is None else int(np.count_nonzero(q))

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


KX_DKJ_SYMMETRIC = 0x100


def transport(mech: Mechanism, T, p, Y, out=None, precision: str = "fp64", stream=None,
              symmetric: bool = False):
    """(mu[n], lambda[n], Dmix[Ns, n]) for device tensors T, p, Y.  symmetric:
    for tables of D_kj fits, evaluate each unordered pair once
    (KX_DKJ_SYMMETRIC)."""
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
    flag = PRECISION[precision] | (KX_DKJ_SYMMETRIC if symmetric else 0)
    check(lib().kx_transport_ex(mech.handle, n, *args, *ptrs, flag, _stream_ptr(stream, dev)))
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


def jacobian(mech: Mechanism, T, p, Y, out=None, stream=None):
    """jac[n, Ns, Ns] = d wdot_k / d C_j (1/s) at fixed T for device tensors T, p, Y."""
    n = T.shape[0]
    ns = mech.n_species
    dev = mech.device
    args = [_dev_tensor(T, dev, (n,), "T"), _dev_tensor(p, dev, (n,), "p"),
            _dev_tensor(Y, dev, (ns, n), "Y")]
    if out is None:
        out = torch.empty((n, ns, ns), dtype=torch.float64, device=f"cuda:{dev}")
    j = _dev_tensor(out, dev, (n, ns, ns), "out")
    check(lib().kx_jacobian(mech.handle, n, *args, j, _stream_ptr(stream, dev)))
    return out


def qss_concentrations(mech: Mechanism, T, p, Y, out=None, stream=None):
    """Cq[n_qss, n] (mol/cm^3): the concentrations of the mechanism's QSS
    species, in species order, for device tensors T, p, Y."""
    n = T.shape[0]
    ns, nq = mech.n_species, mech.n_qss
    dev = mech.device
    args = [_dev_tensor(T, dev, (n,), "T"), _dev_tensor(p, dev, (n,), "p"),
            _dev_tensor(Y, dev, (ns, n), "Y")]
    if out is None:
        out = torch.empty((max(nq, 1), n), dtype=torch.float64, device=f"cuda:{dev}")[:nq]
    c = _dev_tensor(out, dev, (nq, n), "out")
    check(lib().kx_qss_concentrations(mech.handle, n, *args, c, _stream_ptr(stream, dev)))
    return out


# --------------------------------------------------------------------------
# host-only mechanisms and the request server
# --------------------------------------------------------------------------
KX_OP_RATES, KX_OP_TRANSPORT = 1, 2
KX_SERVER_SIMULATE = 1
REQ_STATES = {0: "queued", 1: "admitted", 2: "running", 3: "done", 4: "cancelled", 5: "failed"}


class _Request(C.Structure):
    _fields_ = [("mech", C.c_void_p), ("ops", C.c_int32), ("precision", C.c_int32),
                ("n", C.c_int64), ("T", C.c_void_p), ("p", C.c_void_p), ("Y", C.c_void_p),
                ("arrival_s", C.c_double), ("inputs_ready", C.c_void_p)]


class _Result(C.Structure):
    _fields_ = [("state", C.c_int32), ("pad", C.c_int32), ("wdot", C.c_void_p),
                ("mu", C.c_void_p), ("lam", C.c_void_p), ("Dmix", C.c_void_p),
                ("t_arrival", C.c_double), ("t_admit", C.c_double), ("t_launch", C.c_double),
                ("t_done", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("submitted", "completed", "cancelled", "failed",
                                         "queued", "in_flight", "batches", "graph_launches",
                                         "arena_in_use", "arena_capacity",
                                         "resident_mechs", "resident_bytes")]


BATCH_MAX_ITEMS = 32


class _BatchItem(C.Structure):
    _fields_ = [("n", C.c_int64), ("T", C.c_void_p), ("p", C.c_void_p), ("Y", C.c_void_p),
                ("wdot", C.c_void_p), ("mu", C.c_void_p), ("lam", C.c_void_p),
                ("Dmix", C.c_void_p)]


def batch_noalloc(mech: Mechanism, items, transport: bool = False, precision: str = "fp64",
                  outs=None, stream=None):
    """kx_batch_noalloc: rates (and transport) of several point sets of one
    mechanism in one launch sequence that allocates nothing in the library.
    items: list of (T, p, Y) device tensors; outs: optional list of
    (wdot, mu, lambda, Dmix) tensors per item (the transport ones may be None
    without transport), allocated here by torch when not given.  Returns the
    list of output tuples."""
    L = lib()
    if not getattr(L, "_batch_ready", False):
        L.kx_batch_noalloc.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                       C.POINTER(_BatchItem), C.c_void_p]
        L.kx_batch_noalloc.restype = C.c_int32
        L._batch_ready = True
    ns = mech.n_species
    kw = dict(dtype=torch.float64, device=f"cuda:{mech.device}")
    arr = (_BatchItem * max(1, len(items)))()
    res = []
    for r, (T, p, Y) in enumerate(items):
        n = T.shape[0]
        if outs is not None:
            w, mu, lam, Dm = outs[r]
        else:
            w = torch.empty((ns, n), **kw)
            mu = lam = Dm = None
            if transport:
                mu, lam, Dm = torch.empty(n, **kw), torch.empty(n, **kw), torch.empty((ns, n), **kw)
        ptr = lambda t, shape, name: _dev_tensor(t, mech.device, shape, name).value
        arr[r].n = n
        arr[r].T = ptr(T, (n,), "T")
        arr[r].p = ptr(p, (n,), "p")
        arr[r].Y = ptr(Y, (ns, n), "Y")
        arr[r].wdot = ptr(w, (ns, n), "wdot")
        if transport:
            arr[r].mu = ptr(mu, (n,), "mu")
            arr[r].lam = ptr(lam, (n,), "lambda")
            arr[r].Dmix = ptr(Dm, (ns, n), "Dmix")
        res.append((w, mu, lam, Dm))
    ops = KX_OP_RATES | (KX_OP_TRANSPORT if transport else 0)
    check(L.kx_batch_noalloc(mech.handle, ops, PRECISION[precision], len(items), arr,
                             _stream_ptr(stream, mech.device)))
    return res


def _serve_lib():
    L = lib()
    if not getattr(L, "_serve_ready", False):
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.kx_mech_create_host.argtypes = [C.POINTER(_Desc), C.POINTER(vp)]
        L.kx_server_clock.restype = C.c_double
        L.kx_server_create.argtypes = [C.c_int, i64, i32, i32, C.POINTER(vp)]
        L.kx_server_destroy.argtypes = [vp]
        L.kx_server_add_mech.argtypes = [vp, vp]
        L.kx_submit.argtypes = [vp, C.POINTER(_Request), C.POINTER(i64)]
        L.kx_poll.argtypes = [vp, i64, C.POINTER(_Result)]
        L.kx_wait.argtypes = [vp, i64, C.c_double, C.POINTER(_Result)]
        L.kx_cancel.argtypes = [vp, i64]
        L.kx_result_copy.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.kx_release.argtypes = [vp, i64]
        L.kx_server_stats_get.argtypes = [vp, C.POINTER(_Stats)]
        for name in ("kx_mech_create_host", "kx_server_create", "kx_server_destroy",
                     "kx_server_add_mech", "kx_submit", "kx_poll", "kx_wait", "kx_cancel", "kx_result_copy",
                     "kx_release", "kx_server_stats_get"):
            getattr(L, name).restype = C.c_int32
        L._serve_ready = True
    return L


class HostMechanism(Mechanism):
    """Mechanism tables built without a device (kx_mech_create_host)."""

    def __init__(self, mech: dict):  # noqa: D401 - mirrors Mechanism
        L = _serve_lib()
        d, keep = make_desc(mech)
        h = C.c_void_p()
        check(L.kx_mech_create_host(C.byref(d), C.byref(h)))
        del keep
        self.handle = h
        self.device = -1
        ns, nr, nb = C.c_int32(), C.c_int32(), C.c_int64()
        check(L.kx_mech_info(h, C.byref(ns), C.byref(nr), C.byref(nb)))
        self.n_species, self.n_reactions, self.device_bytes = ns.value, nr.value, nb.value
        self.name = mech.get("name", "")


def clock() -> float:
    """The server's monotonic clock (seconds)."""
    return _serve_lib().kx_server_clock()


def _result_dict(r: _Result) -> dict:
    return {"state": REQ_STATES.get(r.state, r.state), "t_arrival": r.t_arrival,
            "t_admit": r.t_admit, "t_launch": r.t_launch, "t_done": r.t_done,
            "wdot": r.wdot, "mu": r.mu, "lambda": r.lam, "Dmix": r.Dmix}


class Server:
    """Continuous-batching request server (kx_server_*)."""

    def __init__(self, device: int = 0, hbm_budget: int = 8 << 30, max_slots: int = 64,
                 simulate: bool = False):
        L = _serve_lib()
        h = C.c_void_p()
        flags = KX_SERVER_SIMULATE if simulate else 0
        check(L.kx_server_create(int(device), int(hbm_budget), int(max_slots), flags,
                                 C.byref(h)))
        self.handle = h
        self.device = device
        self.simulate = simulate
        self._inputs = {}   # ticket -> (mech, tensors) kept alive until release
        self._meta = {}
        self._resident = {}  # handle value -> mechanism (kept alive with the server)

    def add_mech(self, mech: Mechanism) -> None:
        """Make a mechanism resident (kx_server_add_mech): its tables are copied
        into the server's HBM budget and its launch graphs captured."""
        if mech.handle.value in self._resident:
            return
        check(_serve_lib().kx_server_add_mech(self.handle, mech.handle))
        self._resident[mech.handle.value] = mech

    def submit(self, mech: Mechanism, T=None, p=None, Y=None, n: int | None = None,
               transport: bool = False, precision: str = "fp64",
               arrival: float | None = None, inputs_ready=None) -> int:
        """Queue a request.  A mechanism not yet resident is added first
        (add_mech).  inputs_ready: a torch.cuda.Event recorded after the work
        that writes T, p, Y (None: they are complete now)."""
        L = _serve_lib()
        self.add_mech(mech)
        r = _Request()
        r.mech = mech.handle.value
        r.ops = KX_OP_RATES | (KX_OP_TRANSPORT if transport else 0)
        r.precision = PRECISION[precision]
        if T is not None:
            n = T.shape[0]
            r.T = _dev_tensor(T, self.device, (n,), "T").value
            r.p = _dev_tensor(p, self.device, (n,), "p").value
            r.Y = _dev_tensor(Y, self.device, (mech.n_species, n), "Y").value
        r.n = int(n)
        r.arrival_s = -1.0 if arrival is None else float(arrival)
        r.inputs_ready = inputs_ready.cuda_event if inputs_ready is not None else None
        t = C.c_int64()
        check(L.kx_submit(self.handle, C.byref(r), C.byref(t)))
        self._inputs[t.value] = (mech, T, p, Y)
        self._meta[t.value] = (mech.n_species, int(n), transport)
        return t.value

    def poll(self, ticket: int) -> dict:
        res = _Result()
        check(_serve_lib().kx_poll(self.handle, ticket, C.byref(res)))
        return _result_dict(res)

    def wait(self, ticket: int, timeout: float = -1.0) -> dict:
        res = _Result()
        check(_serve_lib().kx_wait(self.handle, ticket, float(timeout), C.byref(res)))
        return _result_dict(res)

    def cancel(self, ticket: int) -> None:
        check(_serve_lib().kx_cancel(self.handle, ticket))

    def outputs(self, ticket: int, stream=None):
        """Copies of a done request's outputs: (wdot, mu, lambda, Dmix) tensors
        (the transport ones are None when not requested)."""
        ns, n, transport = self._meta[ticket]
        kw = dict(dtype=torch.float64, device=f"cuda:{self.device}")
        w = torch.empty((ns, n), **kw)
        mu = lam = Dm = None
        ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
        if transport:
            mu, lam, Dm = torch.empty(n, **kw), torch.empty(n, **kw), torch.empty((ns, n), **kw)
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        check(_serve_lib().kx_result_copy(self.handle, ticket, ptr(w), ptr(mu), ptr(lam),
                                          ptr(Dm), C.c_void_p(st.cuda_stream)))
        st.synchronize()  # the arena space may be reused as soon as it is released
        return w, mu, lam, Dm

    def copy_outputs(self, ticket: int, wdot, mu=None, lam=None, Dmix=None, stream=None):
        """Copy a done request's outputs into caller tensors (float64, contiguous,
        on this server's device or in pinned host memory; any may be None) and
        wait for the copies."""
        ns, n, transport = self._meta[ticket]
        shapes = ((wdot, (ns, n)), (mu, (n,)), (lam, (n,)), (Dmix, (ns, n)))
        for t, shape in shapes:
            if t is None:
                continue
            if t.dtype != torch.float64 or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"output tensor must be contiguous float64 of shape {shape}")
            if t.is_cuda:
                if t.device.index != self.device:
                    raise ValueError("output tensor on another device")
            elif not t.is_pinned():
                raise ValueError("host output tensors must be in pinned memory")
        ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        check(_serve_lib().kx_result_copy(self.handle, ticket, ptr(wdot),
                                          ptr(mu if transport else None),
                                          ptr(lam if transport else None),
                                          ptr(Dmix if transport else None),
                                          C.c_void_p(st.cuda_stream)))
        st.synchronize()

    def release(self, ticket: int) -> None:
        check(_serve_lib().kx_release(self.handle, ticket))
        self._inputs.pop(ticket, None)
        self._meta.pop(ticket, None)

    def stats(self) -> dict:
        st = _Stats()
        check(_serve_lib().kx_server_stats_get(self.handle, C.byref(st)))
        return {k: getattr(st, k) for k, _ in _Stats._fields_}

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            check(_serve_lib().kx_server_destroy(self.handle))
            self.handle = None
            self._inputs.clear()
            self._resident.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
