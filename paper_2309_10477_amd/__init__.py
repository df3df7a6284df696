"""Python binding of libheston (the MI355X Heston / Milstein Monte-Carlo library).

Argument marshalling only: every step of the path -- random numbers, Milstein
steps, payoffs, Greek samples and their cross-path sums -- runs in the HIP
kernels behind the C ABI declared in include/heston.h.  PyTorch provides device
memory (dump buffers, checkpoints) and the current HIP stream.

If libheston.so has not been built this module raises on import of the
library; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import operator
import os
import struct
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libheston.so")

EURO_CALL, EURO_PUT, ASIAN_CALL, ASIAN_PUT, GEO_ASIAN_CALL, GEO_ASIAN_PUT = 0, 1, 2, 3, 4, 5
FP64, FP32 = 0, 1
PHILOX, SOBOL_BRIDGE = 0, 1
(FULL_TRUNCATION, ABSORPTION, QE, EULER_FULL_TRUNCATION, EULER_ABSORPTION, PARTIAL_TRUNCATION,
 REFLECTION, EXACT) = 0, 1, 2, 3, 4, 5, 6, 7
EXACT_MAX_STEPS = 4096
GREEKS_PATHWISE, GREEKS_BUMP_FUSED, GREEKS_BUMP_PLAIN = 1, 2, 4
ABI_VERSION = 3
CONTROL_NONE, CONTROL_GEOMETRIC = 0, 1
CONTROL_MAX_FIXINGS = 8192
VALID_PRICE, VALID_PATHWISE, VALID_BUMPS, VALID_ADJOINT, VALID_CONTROL = 1, 2, 4, 8, 16
DUMP_WIDTH = 16
DUMP_FIELDS = ("S_T", "V_T", "Sbar", "pay", "pw_delta", "pw_rho", "pay_S0+", "pay_S0-",
               "pay_v0+", "pay_v0-", "pay_r+", "pay_r-", "pay_T+", "pay_T-", "x_T", "aux")
STATUS = {0: "OK", 1: "PENDING", -1: "INVALID_ARGUMENT", -2: "OUT_OF_MEMORY",
          -3: "OVER_BUDGET", -4: "DEVICE_ERROR", -5: "UNSUPPORTED", -6: "NOT_FOUND"}
PARAM_NAMES = ("S0", "K", "r", "T", "v0", "kappa", "theta", "sigma", "rho")
EST_NAMES = ("price", "delta", "gamma", "vega", "rho", "theta", "pw_delta", "pw_rho")


class HestonError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class CParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in PARAM_NAMES]


class CEst(ctypes.Structure):
    _fields_ = [("value", ctypes.c_double), ("std_err", ctypes.c_double)]


class CResult(ctypes.Structure):
    _fields_ = [(n, CEst) for n in EST_NAMES] + [("adj", CEst * 7),
        ("n_paths", ctypes.c_uint64), ("valid_mask", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32), ("device_ms", ctypes.c_double),
        ("cv_price", CEst), ("cv_beta", ctypes.c_double), ("cv_mean", ctypes.c_double),
        ("latency_ms", ctypes.c_double)]


class COpts(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("precision", ctypes.c_int32), ("rng", ctypes.c_int32),
        ("scheme", ctypes.c_int32), ("greeks", ctypes.c_uint32),
        ("qmc_replicates", ctypes.c_uint32),
        ("sobol_directions", ctypes.POINTER(ctypes.c_uint32)), ("sobol_dims", ctypes.c_uint32),
        ("fixing_steps", ctypes.POINTER(ctypes.c_uint32)), ("n_fixings", ctypes.c_uint32),
        ("bump_S0_rel", ctypes.c_double), ("bump_v0_rel", ctypes.c_double),
        ("bump_r_abs", ctypes.c_double), ("bump_T_abs", ctypes.c_double),
        ("control_variate", ctypes.c_int32), ("reserved", ctypes.c_uint32)]


class CRequest(ctypes.Structure):
    _fields_ = [("params", CParams), ("type", ctypes.c_int32), ("n_steps", ctypes.c_uint32),
                ("n_paths", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("want", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("se_target", ctypes.c_double)]


WANT_PATHWISE, WANT_ADJOINT = 1, 2


class CServerConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("precision", ctypes.c_int32),
                ("scheme", ctypes.c_int32), ("max_active", ctypes.c_uint32),
                ("max_steps", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("launch_path_steps", ctypes.c_uint64)]


class CServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "admitted", "completed", "queued",
                                               "active", "launches")] + \
        [(n, ctypes.c_double) for n in ("path_steps", "busy_ms", "p50_ms", "p99_ms", "mean_ms",
                                        "max_ms")] + \
        [(n, ctypes.c_uint64) for n in ("pool_bytes", "pool_free_bytes")]


class CBump(ctypes.Structure):
    _fields_ = [("param", ctypes.c_int32), ("relative", ctypes.c_int32), ("size", ctypes.c_double)]


_lib = None

# heston_param indices
P_S0, P_K, P_R, P_T, P_V0, P_KAPPA, P_THETA, P_SIGMA, P_RHO = range(9)
ADJOINT_PARAMS = ("S0", "v0", "r", "kappa", "theta", "sigma", "rho")


def lib():
    """The loaded libheston.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2309_10477_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, c = ctypes.POINTER, ctypes
    L.heston_default_opts.argtypes = [P(COpts)]
    L.heston_ctx_create.argtypes = [c.c_int, c.c_void_p, c.c_uint64, P(c.c_void_p)]
    L.heston_ctx_destroy.argtypes = [c.c_void_p]
    L.heston_price_greeks_ex.argtypes = [c.c_void_p, P(CParams), c.c_int, c.c_uint64, c.c_uint32,
                                         c.c_uint64, P(COpts), P(CResult)]
    L.heston_price_greeks.argtypes = [P(CParams), c.c_int, c.c_uint64, c.c_uint32, c.c_uint64,
                                      P(CResult)]
    L.heston_price_greeks_noalloc.argtypes = [P(CParams), c.c_int, c.c_uint64, c.c_uint32,
                                              c.c_uint64, P(COpts), c.c_void_p, P(CResult)]
    L.heston_dump_paths.argtypes = [c.c_void_p, P(CParams), c.c_int, c.c_uint64, c.c_uint32,
                                    c.c_uint64, P(COpts), c.c_uint64, c.c_uint64, c.c_void_p]
    L.heston_status_str.argtypes = [c.c_int]
    L.heston_status_str.restype = c.c_char_p
    L.heston_last_error.argtypes = []
    L.heston_last_error.restype = c.c_char_p
    L.heston_abi_version.restype = c.c_int
    if L.heston_abi_version() != ABI_VERSION:
        raise ImportError(f"{LIB_PATH} has ABI version {L.heston_abi_version()}, this binding "
                          f"expects {ABI_VERSION}; rebuild the library")
    L.heston_bump_revalue.argtypes = [c.c_void_p, P(CParams), c.c_int, c.c_uint64, c.c_uint32,
                                      c.c_uint64, P(COpts), P(CBump), c.c_uint32, P(CEst),
                                      P(CEst), P(CEst), P(c.c_double)]
    L.heston_adjoint_ckpt_bytes.argtypes = [c.c_uint64, c.c_uint32, c.c_uint32, c.c_int32]
    L.heston_adjoint_ckpt_bytes.restype = c.c_uint64
    L.heston_adjoint_forward.argtypes = [c.c_void_p, P(CParams), c.c_int, c.c_uint64, c.c_uint32,
                                         c.c_uint64, P(COpts), c.c_uint32, c.c_void_p,
                                         c.c_uint64, P(CEst), P(c.c_double)]
    L.heston_adjoint_backward.argtypes = [c.c_void_p, P(CParams), c.c_int, c.c_uint64,
                                          c.c_uint32, c.c_uint64, P(COpts), c.c_uint32,
                                          c.c_void_p, c.c_uint64, c.c_double, P(CEst),
                                          c.c_void_p, P(c.c_double)]
    L.heston_price_batch.argtypes = [c.c_void_p, P(CRequest), c.c_uint32, P(COpts), P(CResult),
                                     P(c.c_double)]
    L.heston_server_default_config.argtypes = [P(CServerConfig)]
    L.heston_server_create.argtypes = [c.c_void_p, P(CServerConfig), P(c.c_void_p)]
    L.heston_server_destroy.argtypes = [c.c_void_p]
    L.heston_submit.argtypes = [c.c_void_p, P(CRequest), P(c.c_uint64)]
    L.heston_poll.argtypes = [c.c_void_p, c.c_uint64, P(CResult)]
    L.heston_wait.argtypes = [c.c_void_p, c.c_uint64, c.c_double, P(CResult)]
    L.heston_server_get_stats.argtypes = [c.c_void_p, P(CServerStats)]
    _lib = L
    return L


def check(status: int):
    if status != 0:
        raise HestonError(status, lib().heston_last_error().decode())


def sobol_directions(dims: int) -> np.ndarray:
    """Joe-Kuo direction numbers [dims, 32] (uint32, columns >= 30 zero) from
    torch's SobolEngine state."""
    import torch
    st = torch.quasirandom.SobolEngine(dims, scramble=False).sobolstate.numpy()
    out = np.zeros((dims, 32), dtype=np.uint32)
    out[:, :st.shape[1]] = st.astype(np.uint32)
    return out


@dataclass
class Options:
    precision: int = FP64
    rng: int = PHILOX
    scheme: int = FULL_TRUNCATION
    greeks: int = GREEKS_PATHWISE | GREEKS_BUMP_FUSED
    qmc_replicates: int = 16
    fixings: tuple | None = None
    bump_S0_rel: float = 0.01
    bump_v0_rel: float = 0.01
    bump_r_abs: float = 1e-4
    bump_T_abs: float = 1.0 / 365.0
    control_variate: int = CONTROL_NONE


class _OptsHolder:
    """A COpts plus the host arrays it points to (kept alive for the call)."""

    _cache: dict = {}

    @classmethod
    def get(cls, o: Options, n_steps: int) -> "_OptsHolder":
        """The holder for these option values (built once per distinct set; the
        C library only reads it)."""
        fix = None if o.fixings is None else tuple(int(k) for k in o.fixings)
        key = (o.precision, o.rng, o.scheme, o.greeks, o.qmc_replicates, fix, o.bump_S0_rel,
               o.bump_v0_rel, o.bump_r_abs, o.bump_T_abs, o.control_variate,
               n_steps if o.rng == SOBOL_BRIDGE else 0)
        h = cls._cache.get(key)
        if h is None:
            if len(cls._cache) >= 64:
                cls._cache.clear()
            h = cls._cache[key] = cls(o, n_steps)
        return h

    def __init__(self, o: Options, n_steps: int):
        self.c = COpts()
        check(lib().heston_default_opts(ctypes.byref(self.c)))
        self.c.precision, self.c.rng, self.c.scheme = o.precision, o.rng, o.scheme
        self.c.greeks, self.c.qmc_replicates = o.greeks, o.qmc_replicates
        self.c.bump_S0_rel, self.c.bump_v0_rel = o.bump_S0_rel, o.bump_v0_rel
        self.c.bump_r_abs, self.c.bump_T_abs = o.bump_r_abs, o.bump_T_abs
        self.c.control_variate = o.control_variate
        self.fix = self.dirs = None
        if o.fixings is not None:
            self.fix = np.ascontiguousarray(o.fixings, dtype=np.uint32)
            self.c.fixing_steps = self.fix.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
            self.c.n_fixings = self.fix.size
        if o.rng == SOBOL_BRIDGE:
            self.dirs = _directions_cached(2 * n_steps)
            self.c.sobol_directions = self.dirs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
            self.c.sobol_dims = self.dirs.shape[0]


_dir_cache: dict = {}


def _directions_cached(dims: int) -> np.ndarray:
    if dims not in _dir_cache:
        _dir_cache[dims] = np.ascontiguousarray(sobol_directions(dims))
    return _dir_cache[dims]


_param_values = operator.itemgetter(*PARAM_NAMES)


def _cparams(params) -> CParams:
    if isinstance(params, dict):
        try:
            return CParams(*_param_values(params))
        except TypeError:  # values ctypes does not take as they are (e.g. numpy integers)
            return CParams(*(float(params[n]) for n in PARAM_NAMES))
    return CParams(*(float(getattr(params, n)) for n in PARAM_NAMES))


class Context:
    """A library context on one device, bound to a HIP stream (default: torch's
    current stream of that device)."""

    def __init__(self, device: int = 0, stream=None, hbm_budget_bytes: int = 0):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        handle = ctypes.c_void_p()
        ptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        check(lib().heston_ctx_create(device, ctypes.c_void_p(ptr), hbm_budget_bytes,
                                      ctypes.byref(handle)))
        self.handle = handle

    def close(self):
        if self.handle:
            check(lib().heston_ctx_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def price_greeks(self, params, opt_type: int, n_paths: int, n_steps: int, seed: int,
                     opts: Options | None = None) -> dict:
        """{estimator: (value, std_err)} plus 'device_ms', 'latency_ms' and 'n_paths'."""
        o = _OptsHolder.get(opts or Options(), n_steps)
        res = CResult()
        cp = _cparams(params)
        check(lib().heston_price_greeks_ex(self.handle, ctypes.byref(cp), opt_type, n_paths,
                                           n_steps, seed, ctypes.byref(o.c), ctypes.byref(res)))
        return _result_dict(res)

    def dump_paths(self, params, opt_type: int, n_paths: int, n_steps: int, seed: int,
                   first: int, count: int, opts: Options | None = None, out=None):
        """Per-path records [count, 16] (torch float64 tensor on the device)."""
        import torch
        if out is None:
            out = torch.empty((count, DUMP_WIDTH), dtype=torch.float64,
                              device=f"cuda:{self.device}")
        assert out.is_contiguous() and out.dtype == torch.float64 and out.numel() >= count * 16
        o = _OptsHolder(opts or Options(), n_steps)
        cp = _cparams(params)
        check(lib().heston_dump_paths(self.handle, ctypes.byref(cp), opt_type, n_paths, n_steps,
                                      seed, ctypes.byref(o.c), first, count,
                                      ctypes.c_void_p(out.data_ptr())))
        return out


    def bump_revalue(self, params, opt_type: int, n_paths: int, n_steps: int, seed: int,
                     bumps, opts: Options | None = None) -> dict:
        """Plain bump-and-revalue: bumps = [(param index, relative, size)].
        Returns {'price': (v, se), 'first': [(v, se)], 'second': [(v, se)], 'device_ms'}."""
        o = _OptsHolder(opts or Options(), n_steps)
        cb = (CBump * len(bumps))(*[CBump(int(a), int(r), float(h)) for a, r, h in bumps])
        price = CEst()
        first = (CEst * len(bumps))()
        second = (CEst * len(bumps))()
        ms = ctypes.c_double()
        cp = _cparams(params)
        check(lib().heston_bump_revalue(self.handle, ctypes.byref(cp), opt_type, n_paths, n_steps,
                                        seed, ctypes.byref(o.c), cb, len(bumps),
                                        ctypes.byref(price), first, second, ctypes.byref(ms)))
        return {"price": (price.value, price.std_err),
                "first": [(e.value, e.std_err) for e in first],
                "second": [(e.value, e.std_err) for e in second], "device_ms": ms.value}

    def adjoint_forward(self, params, opt_type: int, n_paths: int, n_steps: int, seed: int,
                        ckpt, every: int = 16, opts: Options | None = None):
        """Prices and fills the checkpoint tensor (uint8, on the device)."""
        o = _OptsHolder(opts or Options(greeks=GREEKS_PATHWISE), n_steps)
        price, ms = CEst(), ctypes.c_double()
        cp = _cparams(params)
        check(lib().heston_adjoint_forward(self.handle, ctypes.byref(cp), opt_type, n_paths,
                                           n_steps, seed, ctypes.byref(o.c), every,
                                           ctypes.c_void_p(ckpt.data_ptr()),
                                           ckpt.numel() * ckpt.element_size(),
                                           ctypes.byref(price), ctypes.byref(ms)))
        return (price.value, price.std_err), ms.value

    def adjoint_backward(self, params, opt_type: int, n_paths: int, n_steps: int, seed: int,
                         ckpt, every: int = 16, dprice: float = 1.0,
                         opts: Options | None = None, per_path=None):
        """[(value, se)] for d price / d (S0, v0, r, kappa, theta, sigma, rho), times dprice."""
        o = _OptsHolder(opts or Options(greeks=GREEKS_PATHWISE), n_steps)
        grads, ms = (CEst * 7)(), ctypes.c_double()
        cp = _cparams(params)
        pp = ctypes.c_void_p(per_path.data_ptr()) if per_path is not None else None
        if per_path is not None:
            assert per_path.is_contiguous() and per_path.numel() >= 8 * n_paths
        check(lib().heston_adjoint_backward(self.handle, ctypes.byref(cp), opt_type, n_paths,
                                            n_steps, seed, ctypes.byref(o.c), every,
                                            ctypes.c_void_p(ckpt.data_ptr()),
                                            ckpt.numel() * ckpt.element_size(), float(dprice),
                                            grads, pp, ctypes.byref(ms)))
        return [(g.value, g.std_err) for g in grads], ms.value


    def price_batch(self, requests, opts: Options | None = None):
        """requests: list of dicts with params (dict), type, n_steps, n_paths, seed,
        want (WANT_PATHWISE | WANT_ADJOINT).  Returns ([result dicts], device_ms)."""
        arr = (CRequest * len(requests))()
        for i, q in enumerate(requests):
            arr[i] = make_request(**q)
        out = (CResult * len(requests))()
        ms = ctypes.c_double()
        o = _OptsHolder(opts or Options(precision=FP32, greeks=GREEKS_PATHWISE), 1)
        check(lib().heston_price_batch(self.handle, arr, len(requests), ctypes.byref(o.c), out,
                                       ctypes.byref(ms)))
        return [_result_dict(r) for r in out], ms.value


def make_request(params, type, n_steps, n_paths, seed, want=1, se_target=0.0) -> CRequest:
    return CRequest(_cparams(params), int(type), int(n_steps), int(n_paths), int(seed),
                    int(want), 0, float(se_target))


def ckpt_bytes(n_paths: int, n_steps: int, every: int = 16, precision: int = FP32) -> int:
    return int(lib().heston_adjoint_ckpt_bytes(n_paths, n_steps, every, precision))


# heston_result as one record: 8 + 7 estimates (value, std_err), n_paths,
# valid_mask, reserved, device_ms, cv_price, cv_beta, cv_mean, latency_ms.
_RESULT = struct.Struct("<30dQIId2dddd")


def _result_dict(res: CResult) -> dict:
    v = _RESULT.unpack_from(bytes(res))
    out = dict(zip(EST_NAMES, zip(v[0:16:2], v[1:16:2])))
    out["adj"] = list(zip(v[16:30:2], v[17:30:2]))
    n_paths, mask, _, device_ms, cv_value, cv_se, cv_beta, cv_mean, latency_ms = v[30:]
    out["valid_mask"] = mask
    out["n_paths"] = n_paths
    out["device_ms"] = device_ms
    out["latency_ms"] = latency_ms
    if mask & VALID_CONTROL:
        out["cv_price"] = (cv_value, cv_se)
        out["cv_beta"] = cv_beta
        out["cv_mean"] = cv_mean
    return out


def price_greeks(params, opt_type: int, n_paths: int, n_steps: int, seed: int) -> dict:
    """heston_price_greeks: default context of the current device, default options."""
    res = CResult()
    cp = _cparams(params)
    check(lib().heston_price_greeks(ctypes.byref(cp), opt_type, n_paths, n_steps, seed,
                                    ctypes.byref(res)))
    return _result_dict(res)


def price_greeks_noalloc(params, opt_type: int, n_paths: int, n_steps: int, seed: int,
                         opts: Options | None = None, stream=None) -> dict:
    """heston_price_greeks_noalloc: no context and no allocation, on `stream`
    (a torch stream or a hipStream_t address; None: the current device's null
    stream)."""
    o = _OptsHolder(opts or Options(), n_steps)
    res = CResult()
    cp = _cparams(params)
    ptr = 0 if stream is None else (stream.cuda_stream if hasattr(stream, "cuda_stream")
                                    else int(stream))
    check(lib().heston_price_greeks_noalloc(ctypes.byref(cp), opt_type, n_paths, n_steps, seed,
                                            ctypes.byref(o.c), ctypes.c_void_p(ptr),
                                            ctypes.byref(res)))
    return _result_dict(res)


class Server:
    """Continuous-batching request loop of the library (heston_server_*): the
    engine runs natively; submit() returns a ticket at once."""

    def __init__(self, ctx: Context, precision: int = FP32, scheme: int = FULL_TRUNCATION,
                 max_active: int = 4096, max_steps: int = 2048, hbm_budget_bytes: int = 8 << 30,
                 launch_path_steps: int = 1 << 31):
        cfg = CServerConfig()
        check(lib().heston_server_default_config(ctypes.byref(cfg)))
        cfg.precision, cfg.scheme, cfg.max_active, cfg.max_steps = (precision, scheme,
                                                                    max_active, max_steps)
        cfg.hbm_budget_bytes, cfg.launch_path_steps = hbm_budget_bytes, launch_path_steps
        h = ctypes.c_void_p()
        check(lib().heston_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self.ctx = ctx

    def submit(self, **request) -> int:
        return self.submit_request(make_request(**request))

    def submit_request(self, q: CRequest) -> int:
        """Submits a request built by make_request (for callers that build
        their requests ahead of time)."""
        t = ctypes.c_uint64()
        check(lib().heston_submit(self.handle, ctypes.byref(q), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        res = CResult()
        st = lib().heston_poll(self.handle, ticket, ctypes.byref(res))
        if st == 1:
            return None
        check(st)
        return _result_dict(res)

    def wait(self, ticket: int, timeout_ms: float = 60_000.0):
        res = CResult()
        st = lib().heston_wait(self.handle, ticket, timeout_ms, ctypes.byref(res))
        if st == 1:
            return None
        check(st)
        return _result_dict(res)

    def stats(self) -> dict:
        st = CServerStats()
        check(lib().heston_server_get_stats(self.handle, ctypes.byref(st)))
        return {n: getattr(st, n) for n, _ in CServerStats._fields_}

    def close(self):
        if self.handle:
            check(lib().heston_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
