"""ctypes binding of libbqc.so (include/bqc.h).

Argument marshalling only: every step of the (T) computation runs in the HIP
kernels behind the C ABI.  Inputs may be numpy FP64 arrays (host; the
library uploads them) or torch FP64 tensors on a HIP device (passed as device
pointers on the current torch stream).  If the library is not built the
first call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbqc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bqc.h")

OK, PENDING, EINVAL, ENOMEM, EDEVICE, ENOTFOUND, ESHUTDOWN, ECANCELED = 0, 1, -1, -2, -3, -4, -5, -6
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp8": 3}

_dp = ctypes.POINTER(ctypes.c_double)


class TOpts(ctypes.Structure):
    # include/bqc.h: the four base options first, then the extensions
    _fields_ = [("precision", ctypes.c_int32), ("device", ctypes.c_int32),
                ("inputs_on_device", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("timing", ctypes.c_int32), ("formulation", ctypes.c_int32),
                ("triple_energies", _dp), ("triple_begin", ctypes.c_int64),
                ("triple_end", ctypes.c_int64), ("fock_ov", _dp)]


FORMULATIONS = {"occupied": 0, "virtual": 1}


class TStats(ctypes.Structure):
    # include/bqc.h: the six base statistics first, then the extensions
    _fields_ = [("queue_s", ctypes.c_double), ("upload_s", ctypes.c_double),
                ("gpu_s", ctypes.c_double), ("total_s", ctypes.c_double),
                ("flops", ctypes.c_double), ("footprint_bytes", ctypes.c_uint64),
                ("prepare_s", ctypes.c_double), ("gemm_s", ctypes.c_double),
                ("epilogue_s", ctypes.c_double), ("gemm_launches", ctypes.c_int32),
                ("epilogue_launches", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("n_triples", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Fragment(ctypes.Structure):
    """bqc_t_fragment"""
    _fields_ = [("nocc", ctypes.c_int32), ("nvir", ctypes.c_int32)] + \
               [(name, _dp) for name in ("eps_o", "eps_v", "t1", "t2", "ovvv", "ooov", "ovov")]


class ServerCfg(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("mem_budget_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_int32),
                ("direct_launch", ctypes.c_int32), ("no_grouping", ctypes.c_int32)]


class BqcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bqc error {code}: {msg}")
        self.code = code


_lib = None
_lock = threading.Lock()


def lib():
    """Load libbqc.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "python -m paper_2502_17963_amd.build")
            # One HIP runtime per process: torch's wheel ships its own
            # libamdhip64 (soname libamdhip64.so.7).  Loading torch first lets
            # the dynamic loader bind libbqc.so to that same runtime instead of
            # bringing in a second one, which torch could then not initialise.
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
            L = ctypes.CDLL(LIB_PATH)
            seven = [_dp] * 7
            L.bqc_t_energy.argtypes = [ctypes.c_int32, ctypes.c_int32, *seven, _dp]
            L.bqc_t_energy.restype = ctypes.c_int
            L.bqc_t_energy_ex.argtypes = [ctypes.c_int32, ctypes.c_int32, *seven,
                                          ctypes.POINTER(TOpts), _dp, ctypes.POINTER(TStats)]
            L.bqc_t_energy_ex.restype = ctypes.c_int
            L.bqc_t_energy_df.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, *([_dp] * 8),
                                          ctypes.POINTER(TOpts), _dp, ctypes.POINTER(TStats)]
            L.bqc_t_energy_df.restype = ctypes.c_int
            L.bqc_mp2_energy_df.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _dp, _dp, _dp,
                                            ctypes.POINTER(TOpts), _dp, ctypes.POINTER(TStats)]
            L.bqc_mp2_energy_df.restype = ctypes.c_int
            L.bqc_t_energy_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(Fragment), ctypes.POINTER(TOpts), _dp,
                                             ctypes.POINTER(TStats)]
            L.bqc_t_energy_batch.restype = ctypes.c_int
            L.bqc_t_batch_footprint.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                                ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
            L.bqc_t_batch_footprint.restype = ctypes.c_int64
            L.bqc_t_num_triples.argtypes = [ctypes.c_int32]
            L.bqc_t_num_triples.restype = ctypes.c_int64
            L.bqc_t_footprint.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
            L.bqc_t_footprint.restype = ctypes.c_int64
            L.bqc_t_footprint_ex.argtypes = [ctypes.c_int32] * 5
            L.bqc_t_footprint_ex.restype = ctypes.c_int64
            L.bqc_t_energy_noalloc.argtypes = [ctypes.c_int32, ctypes.c_int32, *seven,
                                               ctypes.POINTER(TOpts), _dp, ctypes.POINTER(TStats)]
            L.bqc_t_energy_noalloc.restype = ctypes.c_int
            L.bqc_t_noalloc_batch.argtypes = [ctypes.c_int32] * 5
            L.bqc_t_noalloc_batch.restype = ctypes.c_int64
            L.bqc_last_error.argtypes = []
            L.bqc_last_error.restype = ctypes.c_char_p
            L.bqc_version.argtypes = []
            L.bqc_version.restype = ctypes.c_int32
            L.bqc_hip_versions.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
            L.bqc_hip_versions.restype = ctypes.c_int
            if hasattr(L, "bqc_server_create"):
                L.bqc_server_create.argtypes = [ctypes.POINTER(ServerCfg), ctypes.POINTER(ctypes.c_void_p)]
                L.bqc_server_create.restype = ctypes.c_int
                L.bqc_server_destroy.argtypes = [ctypes.c_void_p]
                L.bqc_server_destroy.restype = ctypes.c_int
                L.bqc_t_submit.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, *seven,
                                           ctypes.POINTER(ctypes.c_uint64)]
                L.bqc_t_submit.restype = ctypes.c_int
                L.bqc_t_submit_ex.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, *seven,
                                              ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]
                L.bqc_t_submit_ex.restype = ctypes.c_int
                L.bqc_t_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, _dp, ctypes.POINTER(TStats)]
                L.bqc_t_poll.restype = ctypes.c_int
                L.bqc_t_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64, _dp, ctypes.POINTER(TStats)]
                L.bqc_t_wait.restype = ctypes.c_int
                L.bqc_t_cancel.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
                L.bqc_t_cancel.restype = ctypes.c_int
            _lib = L
        return _lib


def header_functions():
    """Names of the functions include/bqc.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\*?\s+\*?(bqc_[a-z0-9_]+)\s*\(", text, re.M)))


def last_error() -> str:
    return lib().bqc_last_error().decode()


def _check(rc):
    if rc != OK:
        raise BqcError(rc, last_error())


def runtime_versions() -> dict:
    """HIP version the library was compiled with and of the runtime the
    process has loaded (bqc_hip_versions)."""
    c, r = ctypes.c_int32(0), ctypes.c_int32(0)
    rc = lib().bqc_hip_versions(ctypes.byref(c), ctypes.byref(r))
    return {"compiled": c.value, "runtime": r.value if rc == OK else None,
            "match": rc == OK and c.value // 100000 == r.value // 100000}


def num_triples(nocc: int) -> int:
    return int(lib().bqc_t_num_triples(nocc))


def footprint(nocc: int, nvir: int, precision="fp64", formulation="occupied", fock=False) -> int:
    """Device bytes one solve holds (bqc_t_footprint_ex), -1 for invalid arguments."""
    if formulation not in FORMULATIONS:
        return -1
    return int(lib().bqc_t_footprint_ex(nocc, nvir, _prec(precision), FORMULATIONS[formulation], 1 if fock else 0))


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _torch_stream(tensor):
    """Stream handle for device inputs: torch's current stream.  torch's
    default stream has handle 0, which the ABI reads as "the library's own
    stream" (not ordered after torch's work), so that stream is synchronised
    here first."""
    import torch
    s = torch.cuda.current_stream(tensor.device)
    if s.cuda_stream == 0:
        s.synchronize()
    return s.cuda_stream


def _ptrs(arrays):
    """(pointers, on_device, keepalive) for numpy arrays or torch tensors."""
    first = arrays[0]
    if isinstance(first, np.ndarray):
        keep = [np.ascontiguousarray(a, dtype=np.float64) for a in arrays]
        return [k.ctypes.data_as(_dp) for k in keep], False, keep
    # torch tensors on a HIP device
    for a in arrays:
        if a.dtype.itemsize != 8 or not a.is_contiguous() or not a.is_cuda:
            raise ValueError("device inputs must be contiguous float64 tensors on a HIP device")
    return [ctypes.cast(ctypes.c_void_p(a.data_ptr()), _dp) for a in arrays], True, list(arrays)


def _solve_opts(arrays, precision, device, timing, stream, triple_range, fock_ov, formulation):
    """ctypes options of one solve: (pointers, opts, buffers to keep alive)."""
    if formulation not in FORMULATIONS:
        raise ValueError(f"formulation must be one of {sorted(FORMULATIONS)}")
    ptrs, on_dev, keep = _ptrs(arrays)
    opts = TOpts()
    opts.precision = _prec(precision)
    opts.device = device
    opts.inputs_on_device = 1 if on_dev else 0
    opts.timing = 1 if timing else 0
    opts.formulation = FORMULATIONS[formulation]
    if triple_range is not None:
        opts.triple_begin, opts.triple_end = int(triple_range[0]), int(triple_range[1])
    if fock_ov is not None:
        fp, f_dev, f_keep = _ptrs((fock_ov,))
        if f_dev != on_dev:
            raise ValueError("fock_ov must live where the other inputs live (host or device)")
        opts.fock_ov = fp[0]
        keep = list(keep) + list(f_keep)
    if stream is not None:
        opts.stream = ctypes.c_void_p(stream)
    elif on_dev:
        opts.stream = ctypes.c_void_p(_torch_stream(arrays[0]))
    return ptrs, opts, keep


def _finish(rc, e, st, etrip, ntrip, triple_energies, stats, timing):
    _check(rc)
    if not (triple_energies or stats or timing):
        return e.value
    extras = {}
    if triple_energies:
        extras["triples"] = etrip[:ntrip]
    extras["stats"] = st.as_dict()
    return e.value, extras


def t_energy(nocc, nvir, eps_o, eps_v, t1, t2, ovvv, ooov, ovov, precision="fp64",
             device=0, triple_energies=False, timing=False, stream=None, stats=False,
             triple_range=None, fock_ov=None, formulation="occupied"):
    """E_T through bqc_t_energy_ex.

    triple_range=(begin, end) solves only that share of the unique triples;
    fock_ov (f_ia, [nocc][nvir], on the same side as the other inputs) adds the
    f_ov term of a non-canonical reference; formulation="virtual" runs the
    loop over unique virtual triples (then "triples" below are those).
    Returns E_T, or (E_T, extras) when triple_energies or stats is requested;
    extras holds "triples" (numpy array in unique-triple order; with a range,
    entries outside it are zero) and/or "stats".
    """
    arrays = (eps_o, eps_v, t1, t2, ovvv, ooov, ovov)
    ptrs, opts, keep = _solve_opts(arrays, precision, device, timing, stream, triple_range, fock_ov,
                                   formulation)
    ntrip = num_triples(nvir if formulation == "virtual" else nocc)
    etrip = None
    if triple_energies:
        etrip = np.zeros(max(ntrip, 1))
        opts.triple_energies = etrip.ctypes.data_as(_dp)
    e = ctypes.c_double(0.0)
    st = TStats()
    rc = lib().bqc_t_energy_ex(nocc, nvir, *ptrs, ctypes.byref(opts), ctypes.byref(e), ctypes.byref(st))
    del keep
    return _finish(rc, e, st, etrip, ntrip, triple_energies, stats, timing)


def t_energy_noalloc(nocc, nvir, eps_o, eps_v, t1, t2, ovvv, ooov, ovov, precision="fp64", device=0,
                     triple_energies=False, stream=None, stats=False, triple_range=None, fock_ov=None,
                     formulation="occupied"):
    """E_T through bqc_t_energy_noalloc (device tensors only; the library's
    fixed device array is the workspace).  Arguments and results as
    t_energy."""
    arrays = (eps_o, eps_v, t1, t2, ovvv, ooov, ovov)
    ptrs, opts, keep = _solve_opts(arrays, precision, device, False, stream, triple_range, fock_ov,
                                   formulation)
    if not opts.inputs_on_device:
        raise ValueError("bqc_t_energy_noalloc takes device tensors")
    ntrip = num_triples(nvir if formulation == "virtual" else nocc)
    etrip = None
    if triple_energies:
        etrip = np.zeros(max(ntrip, 1))
        opts.triple_energies = etrip.ctypes.data_as(_dp)
    e = ctypes.c_double(0.0)
    st = TStats()
    rc = lib().bqc_t_energy_noalloc(nocc, nvir, *ptrs, ctypes.byref(opts), ctypes.byref(e), ctypes.byref(st))
    del keep
    return _finish(rc, e, st, etrip, ntrip, triple_energies, stats, False)


def noalloc_batch(nocc, nvir, precision="fp64", formulation="occupied", fock=False) -> int:
    """Triples per launch of bqc_t_energy_noalloc (0: does not fit its array)."""
    if formulation not in FORMULATIONS:
        return -1
    return int(lib().bqc_t_noalloc_batch(nocc, nvir, _prec(precision), FORMULATIONS[formulation],
                                         1 if fock else 0))


def t_energy_df(nocc, nvir, naux, eps_o, eps_v, t1, t2, b_ov, b_vv, ooov, ovov, precision="fp64",
                device=0, triple_energies=False, timing=False, stream=None, stats=False, triple_range=None,
                fock_ov=None, formulation="occupied"):
    """E_T through bqc_t_energy_df: (ia|bc) formed on the device from the
    density-fitting factors b_ov[naux][nocc][nvir] and b_vv[naux][nvir][nvir].
    Arguments and results as t_energy."""
    arrays = (eps_o, eps_v, t1, t2, b_ov, b_vv, ooov, ovov)
    ptrs, opts, keep = _solve_opts(arrays, precision, device, timing, stream, triple_range, fock_ov,
                                   formulation)
    ntrip = num_triples(nvir if formulation == "virtual" else nocc)
    etrip = None
    if triple_energies:
        etrip = np.zeros(max(ntrip, 1))
        opts.triple_energies = etrip.ctypes.data_as(_dp)
    e = ctypes.c_double(0.0)
    st = TStats()
    rc = lib().bqc_t_energy_df(nocc, nvir, naux, *ptrs, ctypes.byref(opts), ctypes.byref(e), ctypes.byref(st))
    del keep
    return _finish(rc, e, st, etrip, ntrip, triple_energies, stats, timing)


def mp2_energy_df(nocc, nvir, naux, eps_o, eps_v, b_ov, device=0, stream=None, stats=False,
                  pair_energies=False):
    """E_MP2 through bqc_mp2_energy_df (b_ov[naux][nocc][nvir]; FP64).
    Returns E_MP2, or (E_MP2, stats dict) with stats=True; with
    pair_energies=True, (E_MP2, extras) where extras["pairs"] holds e_ij for
    i <= j in lexicographic order and extras["stats"] the stats."""
    ptrs, on_dev, keep = _ptrs((eps_o, eps_v, b_ov))
    opts = TOpts()
    opts.device = device
    opts.inputs_on_device = 1 if on_dev else 0
    if stream is not None:
        opts.stream = ctypes.c_void_p(stream)
    elif on_dev:
        opts.stream = ctypes.c_void_p(_torch_stream(eps_o))
    pairs = None
    if pair_energies:
        pairs = np.zeros(max(nocc * (nocc + 1) // 2, 1))
        opts.triple_energies = pairs.ctypes.data_as(_dp)
    e = ctypes.c_double(0.0)
    st = TStats()
    rc = lib().bqc_mp2_energy_df(nocc, nvir, naux, *ptrs, ctypes.byref(opts), ctypes.byref(e), ctypes.byref(st))
    del keep
    _check(rc)
    if pair_energies:
        return e.value, {"pairs": pairs[:nocc * (nocc + 1) // 2], "stats": st.as_dict()}
    return (e.value, st.as_dict()) if stats else e.value


def t_energy_batch(fragments, precision="fp64", device=0, stream=None, stats=False):
    """E_T of several fragments through bqc_t_energy_batch.

    fragments: sequence of (nocc, nvir, eps_o, eps_v, t1, t2, ovvv, ooov, ovov),
    all host numpy arrays or all device tensors.  Returns the list of energies,
    or (energies, stats dict) with stats=True."""
    n = len(fragments)
    arr = (Fragment * max(n, 1))()
    keep = []
    on_dev = None
    for f, fr in enumerate(fragments):
        ptrs, dev, k = _ptrs(tuple(fr[2:9]))
        if on_dev is None:
            on_dev = dev
        elif dev != on_dev:
            raise ValueError("all fragments' inputs must live on the same side (host or device)")
        keep.append(k)
        arr[f].nocc, arr[f].nvir = int(fr[0]), int(fr[1])
        for name, p in zip(("eps_o", "eps_v", "t1", "t2", "ovvv", "ooov", "ovov"), ptrs):
            setattr(arr[f], name, p)
    opts = TOpts()
    opts.precision = _prec(precision)
    opts.device = device
    opts.inputs_on_device = 1 if on_dev else 0
    if stream is not None:
        opts.stream = ctypes.c_void_p(stream)
    elif on_dev:
        opts.stream = ctypes.c_void_p(_torch_stream(fragments[0][2]))
    e = (ctypes.c_double * max(n, 1))()
    st = TStats()
    rc = lib().bqc_t_energy_batch(n, arr, ctypes.byref(opts), e, ctypes.byref(st))
    del keep
    _check(rc)
    out = [e[f] for f in range(n)]
    return (out, st.as_dict()) if stats else out


def batch_footprint(shapes, precision="fp64") -> int:
    """bqc_t_batch_footprint for [(nocc, nvir), ...] (-1 for invalid arguments)."""
    n = len(shapes)
    o = (ctypes.c_int32 * max(n, 1))(*[s[0] for s in shapes])
    v = (ctypes.c_int32 * max(n, 1))(*[s[1] for s in shapes])
    return int(lib().bqc_t_batch_footprint(n, o, v, _prec(precision)))


def t_energy_plain(nocc, nvir, eps_o, eps_v, t1, t2, ovvv, ooov, ovov):
    """E_T through bqc_t_energy (host inputs, FP64, device 0)."""
    ptrs, on_dev, keep = _ptrs((eps_o, eps_v, t1, t2, ovvv, ooov, ovov))
    if on_dev:
        raise ValueError("bqc_t_energy takes host arrays")
    e = ctypes.c_double(0.0)
    rc = lib().bqc_t_energy(nocc, nvir, *ptrs, ctypes.byref(e))
    del keep
    _check(rc)
    return e.value


class Server:
    """bqc_server_* wrapper: continuous batching of independent (T) solves.

    Host input arrays are kept alive until the ticket reaches a terminal
    status (the C ABI borrows them until then).
    """

    def __init__(self, precision="fp64", device=0, mem_budget_bytes=0, max_inflight=0, graphs=True, grouping=True):
        cfg = ServerCfg()
        cfg.direct_launch = 0 if graphs else 1
        cfg.no_grouping = 0 if grouping else 1
        cfg.device = device
        cfg.precision = _prec(precision)
        cfg.mem_budget_bytes = int(mem_budget_bytes)
        cfg.max_inflight = int(max_inflight)
        self._h = ctypes.c_void_p()
        _check(lib().bqc_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))
        self._keep = {}

    def submit(self, nocc, nvir, eps_o, eps_v, t1, t2, ovvv, ooov, ovov) -> int:
        """Host numpy arrays (uploaded at admission) or device torch tensors
        (read in place; keep them unmodified until the ticket finishes)."""
        ptrs, on_dev, keep = _ptrs((eps_o, eps_v, t1, t2, ovvv, ooov, ovov))
        t = ctypes.c_uint64()
        if on_dev:
            import torch
            torch.cuda.current_stream(eps_o.device).synchronize()  # inputs complete before the server reads them
        _check(lib().bqc_t_submit_ex(self._h, nocc, nvir, *ptrs, 1 if on_dev else 0, ctypes.byref(t)))
        self._keep[t.value] = keep
        return t.value

    def _finish(self, fn, ticket):
        e = ctypes.c_double()
        st = TStats()
        rc = fn(self._h, ticket, ctypes.byref(e), ctypes.byref(st))
        if rc == PENDING:
            return None
        self._keep.pop(ticket, None)
        _check(rc)
        return e.value, st.as_dict()

    def poll(self, ticket):
        """None while pending, else (E_T, stats); raises BqcError on failure."""
        return self._finish(lib().bqc_t_poll, ticket)

    def wait(self, ticket):
        return self._finish(lib().bqc_t_wait, ticket)

    def cancel(self, ticket) -> bool:
        """bqc_t_cancel: True if the request was cancelled before it ran (or had
        already finished; its poll tells which), False if it is running."""
        rc = lib().bqc_t_cancel(self._h, ticket)
        if rc == PENDING:
            return False
        _check(rc)
        return True

    def close(self):
        if self._h:
            _check(lib().bqc_server_destroy(self._h))
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
