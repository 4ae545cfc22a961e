"""Python binding of libtlrqmc (ctypes): argument marshalling only.

Every step of the estimator runs in the library's HIP kernels; this module
converts numpy arrays to the C ABI of include/tlrqmc.h and back.  PyTorch
supplies the device memory (its caching allocator, through the allocator
callback) and the stream.  There is no fallback: if the shared library is
missing or no GPU is present, the calls raise.
"""

from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtlrqmc.so")

OK, WARN_RANKCAP, PENDING = 0, 1, 2
EINVAL, ENOTSPD, ENOMEM, EDEVICE, ENOTFOUND = -1, -2, -3, -4, -5
KERNEL_NAMES = ("init", "delta", "sweep", "zproj", "reduce")


class TLRQMCError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"tlrqmc error {status}: {message}")
        self.status = status


class Allocator(C.Structure):
    _fields_ = [("alloc", C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)),
                ("user", C.c_void_p)]


class Cov(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("sigma", C.c_void_p),
                ("ld", C.c_int64), ("xy", C.c_void_p), ("range", C.c_double),
                ("variance", C.c_double), ("nugget", C.c_double)]


class FactorInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int32), ("r", C.c_int32), ("k_tot", C.c_int64),
                ("k_max", C.c_int32), ("cap_hits", C.c_int32), ("diag_doubles", C.c_int64),
                ("uv_doubles", C.c_int64), ("device_bytes", C.c_int64), ("setup_seconds", C.c_double * 4),
                ("checksum", C.c_uint64), ("host_tiles", C.c_int64)]


class QmcOpts(C.Structure):
    _fields_ = [("n_samples", C.c_int64), ("n_shifts", C.c_int32), ("precision", C.c_int32),
                ("seed", C.c_uint64), ("logp_out", C.c_void_p), ("profile", C.c_int32),
                ("reserved", C.c_int32), ("chunk_samples", C.c_int64)]


class Result(C.Structure):
    _fields_ = [("log_p", C.c_double), ("p", C.c_double), ("std_err", C.c_double),
                ("rel_err", C.c_double), ("log_p_shift", C.c_double * 64), ("n_dead", C.c_int64),
                ("seconds", C.c_double), ("kernel_seconds", C.c_double * 5),
                ("kernel_busy_seconds", C.c_double * 5), ("kernel_launches", C.c_int64 * 5), ("n_shifts", C.c_int32), ("chunks", C.c_int32)]


class SkewNormalParams(C.Structure):
    _fields_ = [("xi", C.c_double), ("sigma1", C.c_double), ("beta1", C.c_double), ("sigma2", C.c_double),
                ("beta2", C.c_double)]


class SkewNormalResult(C.Structure):
    _fields_ = [("loglik", C.c_double), ("log_density", C.c_double), ("log_prob", C.c_double),
                ("log_prob_std_err", C.c_double), ("log_prob_rel_err", C.c_double), ("seconds", C.c_double * 3),
                ("prob", Result)]


class Request(C.Structure):
    _fields_ = [("n", C.c_int64), ("cov", Cov), ("a", C.c_void_p), ("b", C.c_void_p), ("nu", C.c_double),
                ("m", C.c_int32), ("max_rank", C.c_int32), ("tol", C.c_double), ("reorder", C.c_int32),
                ("reserved", C.c_int32), ("qmc", QmcOpts)]


class RequestInfo(C.Structure):
    _fields_ = [("t_submit", C.c_double), ("t_admit", C.c_double), ("t_ready", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double), ("reserved_bytes", C.c_int64),
                ("factor_bytes", C.c_int64), ("chunk_samples", C.c_int64), ("slots", C.c_int32),
                ("concurrency", C.c_int32), ("status", C.c_int32), ("reserved", C.c_int32),
                ("factor_checksum", C.c_uint64)]


class ServerInfo(C.Structure):
    _fields_ = [("budget_bytes", C.c_int64), ("reserved_bytes", C.c_int64), ("peak_reserved_bytes", C.c_int64),
                ("arena_in_use_bytes", C.c_int64), ("arena_peak_bytes", C.c_int64), ("steps", C.c_int64),
                ("launches", C.c_int64), ("slot_steps", C.c_int64), ("max_active_slots", C.c_int64),
                ("queued", C.c_int32), ("in_setup", C.c_int32), ("ready", C.c_int32), ("running", C.c_int32)]


_lib = None

# Exported names and argument types of the C ABI.
SIGNATURES = {
    "tlrqmc_ctx_create": (C.c_int, [C.c_int, C.c_void_p, C.POINTER(Allocator), C.POINTER(C.c_void_p)]),
    "tlrqmc_ctx_destroy": (None, [C.c_void_p]),
    "tlrqmc_last_error": (C.c_char_p, []),
    "tlrqmc_geometric_order": (C.c_int, [C.c_int64, C.POINTER(Cov), C.c_void_p]),
    "block_reorder": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(Cov), C.c_void_p, C.c_void_p, C.c_int,
                                C.c_void_p]),
    "tlr_factor": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(Cov), C.c_void_p, C.c_int, C.c_double, C.c_int,
                             C.POINTER(C.c_void_p)]),
    "tlr_factor_rbodr": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(Cov), C.c_void_p, C.c_void_p, C.c_int,
                                   C.c_double, C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "tlrqmc_factor_import": (C.c_int, [C.c_void_p, C.c_int64, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "tlrqmc_factor_stats": (C.c_int, [C.c_void_p, C.POINTER(FactorInfo)]),
    "tlrqmc_factor_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "tlrqmc_factor_free": (None, [C.c_void_p]),
    "mvn_prob": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(QmcOpts), C.POINTER(Result)]),
    "mvt_prob": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.POINTER(QmcOpts),
                           C.POINTER(Result)]),
    "tlrqmc_prob_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                      C.POINTER(QmcOpts), C.POINTER(Result)]),
    "tlrqmc_sample_logp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                     C.POINTER(QmcOpts), C.c_int32, C.c_int64, C.c_int64, C.c_void_p]),
    "tlrqmc_skewnormal_loglik": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.POINTER(SkewNormalParams),
                                           C.c_int, C.c_double, C.c_int, C.c_int, C.POINTER(QmcOpts),
                                           C.POINTER(SkewNormalResult), C.c_void_p, C.POINTER(C.c_void_p)]),
    "tlrqmc_server_create": (C.c_int, [C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)]),
    "tlrqmc_server_submit": (C.c_int, [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "tlrqmc_server_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int32, C.POINTER(Result), C.POINTER(RequestInfo)]),
    "tlrqmc_server_stats": (C.c_int, [C.c_void_p, C.POINTER(ServerInfo)]),
    "tlrqmc_server_destroy": (C.c_int, [C.c_void_p]),
}


def lib():
    """The loaded shared library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2003_11183_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int) -> int:
    if status < 0:
        raise TLRQMCError(status, lib().tlrqmc_last_error().decode())
    return status


def _ptr(a) -> int | None:
    return None if a is None else a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _cov(cov: dict, n: int | None = None) -> tuple[Cov, list]:
    """tlrqmc_cov from {'xy', 'beta'[, 'variance', 'nugget']} or {'sigma'},
    checked against the dimension n."""
    keep = []
    if "sigma" in cov:
        S = np.asfortranarray(cov["sigma"], dtype=np.float64)
        if S.ndim != 2 or S.shape[0] != S.shape[1] or (n is not None and S.shape[0] != n):
            raise ValueError(f"sigma must be {n} x {n}, got {S.shape}")
        keep.append(S)
        return Cov(0, 0, S.ctypes.data, S.shape[0], None, 0.0, 0.0, 0.0), keep
    xy = _f64(cov["xy"])
    if xy.ndim != 2 or xy.shape[1] != 2 or (n is not None and xy.shape[0] != n):
        raise ValueError(f"xy must be {n} x 2, got {xy.shape}")
    keep.append(xy)
    return Cov(1, 0, None, 0, xy.ctypes.data, float(cov["beta"]), float(cov.get("variance", 1.0)),
               float(cov.get("nugget", 0.0))), keep


class Context:
    """Library context on one device, using torch's stream and caching allocator."""

    def __init__(self, device: int = 0, use_torch_allocator: bool = True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU available: the TLR QMC library runs on the device only")
        self.device = device
        self._torch = torch
        stream = torch.cuda.current_stream(device)
        self.stream = stream
        alloc_p = None
        if use_torch_allocator:
            def _alloc(size, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(size), device, stream)
                except Exception:
                    return None

            def _free(ptr, user):
                torch.cuda.caching_allocator_delete(ptr)

            self._cb = Allocator(Allocator._fields_[0][1](_alloc), Allocator._fields_[1][1](_free), None)
            alloc_p = C.byref(self._cb)
        h = C.c_void_p()
        _check(lib().tlrqmc_ctx_create(device, C.c_void_p(stream.cuda_stream), alloc_p, C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().tlrqmc_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def geometric_order(xy) -> np.ndarray:
    n = len(xy)
    cv, keep = _cov({"xy": xy, "beta": 1.0})
    out = np.empty(n, dtype=np.int32)
    _check(lib().tlrqmc_geometric_order(n, C.byref(cv), out.ctypes.data))
    return out


def block_reorder(cov: dict, a, b, m: int, ctx: Context | None = None) -> np.ndarray:
    a, b = _f64(a), _f64(b)
    n = len(a)
    if len(b) != n:
        raise ValueError("a and b must have the same length")
    cv, keep = _cov(cov, n)
    out = np.empty(n, dtype=np.int32)
    _check(lib().block_reorder(ctx.handle if ctx else None, n, C.byref(cv), a.ctypes.data, b.ctypes.data,
                               int(m), out.ctypes.data))
    return out


def _tile_sizes(n: int, m: int) -> list[int]:
    r = (n + m - 1) // m
    return [min(m, n - i * m) for i in range(r)]


class Factor:
    """Device-resident TLR factor (owned by the library)."""

    def __init__(self, ctx: Context, handle: C.c_void_p, status: int = OK):
        self.ctx, self.handle, self.status = ctx, handle, status

    @classmethod
    def from_tiles(cls, ctx: Context, n: int, m: int, diag, ranks, U, V, perm=None) -> "Factor":
        sz = _tile_sizes(n, m)
        r = len(sz)
        d = np.concatenate([_f64(np.asarray(diag[i])).ravel() for i in range(r)])
        rk = np.ascontiguousarray(ranks, dtype=np.int32).reshape(r, r)
        us, vs = [], []
        for i in range(1, r):
            for j in range(i):
                if rk[i, j] > 0:
                    us.append(_f64(U[(i, j)]).reshape(sz[i], rk[i, j]).ravel())
                    vs.append(_f64(V[(i, j)]).reshape(sz[j], rk[i, j]).ravel())
        Ua = np.concatenate(us) if us else np.zeros(1)
        Va = np.concatenate(vs) if vs else np.zeros(1)
        p = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
        h = C.c_void_p()
        _check(lib().tlrqmc_factor_import(ctx.handle, n, m, _ptr(p), d.ctypes.data, rk.ctypes.data,
                                          Ua.ctypes.data, Va.ctypes.data, C.byref(h)))
        return cls(ctx, h)

    @classmethod
    def build(cls, ctx: Context, cov: dict, n: int, m: int, tol: float, max_rank: int = 0,
              perm=None) -> "Factor":
        cv, keep = _cov(cov, n)
        p = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
        if p is not None and p.shape != (n,):
            raise ValueError("perm must have n entries")
        h = C.c_void_p()
        st = _check(lib().tlr_factor(ctx.handle, n, C.byref(cv), _ptr(p), int(m), float(tol), int(max_rank),
                                     C.byref(h)))
        return cls(ctx, h, st)

    @classmethod
    def build_reordered(cls, ctx: Context, cov: dict, a, b, m: int, tol: float,
                        max_rank: int = 0) -> "Factor":
        """Factor with block reordering during the Cholesky factorization
        (tlr_factor_rbodr); its order is factor.perm."""
        a, b = _f64(a), _f64(b)
        n = len(a)
        if b.shape != (n,):
            raise ValueError("a and b must have the same length")
        cv, keep = _cov(cov, n)
        perm = np.empty(n, dtype=np.int32)
        h = C.c_void_p()
        st = _check(lib().tlr_factor_rbodr(ctx.handle, n, C.byref(cv), a.ctypes.data, b.ctypes.data, int(m),
                                           float(tol), int(max_rank), perm.ctypes.data, C.byref(h)))
        F = cls(ctx, h, st)
        F.perm = perm
        return F

    def stats(self) -> dict:
        inf = FactorInfo()
        _check(lib().tlrqmc_factor_stats(self.handle, C.byref(inf)))
        out = {k: getattr(inf, k) for k, _ in FactorInfo._fields_}
        out["setup_seconds"] = dict(zip(("cholesky", "download", "compress", "layout"), inf.setup_seconds))
        return out

    def export(self):
        """(perm, diag list, ranks, U dict, V dict) in the exchange layout."""
        st = self.stats()
        n, m, r = st["n"], st["m"], st["r"]
        sz = _tile_sizes(n, m)
        perm = np.empty(n, dtype=np.int32)
        d = np.empty(st["diag_doubles"])
        rk = np.empty((r, r), dtype=np.int32)
        _check(lib().tlrqmc_factor_export(self.handle, perm.ctypes.data, d.ctypes.data, rk.ctypes.data,
                                          None, None))
        nu_ = sum(sz[i] * int(rk[i, j]) for i in range(r) for j in range(i))
        nv_ = sum(sz[j] * int(rk[i, j]) for i in range(r) for j in range(i))
        Ua, Va = np.empty(max(nu_, 1)), np.empty(max(nv_, 1))
        _check(lib().tlrqmc_factor_export(self.handle, None, None, None, Ua.ctypes.data, Va.ctypes.data))
        diag, U, V = [], {}, {}
        o = 0
        for i in range(r):
            diag.append(d[o:o + sz[i] * sz[i]].reshape(sz[i], sz[i]).copy())
            o += sz[i] * sz[i]
        ou = ov = 0
        for i in range(1, r):
            for j in range(i):
                k = int(rk[i, j])
                U[(i, j)] = Ua[ou:ou + sz[i] * k].reshape(sz[i], k).copy()
                V[(i, j)] = Va[ov:ov + sz[j] * k].reshape(sz[j], k).copy()
                ou += sz[i] * k
                ov += sz[j] * k
        return perm, diag, rk, U, V

    def free(self):
        if self.handle:
            lib().tlrqmc_factor_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _opts(N, M, seed, precision, logp, profile, chunk):
    return QmcOpts(int(N), int(M), int(precision), int(seed) & 0xFFFFFFFFFFFFFFFF,
                   None if logp is None else logp.ctypes.data, int(bool(profile)), 0, int(chunk))


def _result(res: Result, status: int) -> dict:
    M = res.n_shifts
    out = dict(log_p=res.log_p, p=res.p, std_err=res.std_err, rel_err=res.rel_err,
               log_p_shift=np.array(res.log_p_shift[:M]), n_dead=res.n_dead, seconds=res.seconds,
               chunks=res.chunks, status=status)
    out["kernel_seconds"] = {KERNEL_NAMES[k]: res.kernel_seconds[k] for k in range(5)}
    out["kernel_busy_seconds"] = {KERNEL_NAMES[k]: res.kernel_busy_seconds[k] for k in range(5)}
    out["kernel_launches"] = {KERNEL_NAMES[k]: res.kernel_launches[k] for k in range(5)}
    return out


def probability(ctx: Context, factor: Factor, a, b, N: int, M: int, seed: int, nu: float = 0.0,
                precision: int = 0, return_logp: bool = False, profile: bool = False, chunk: int = 0):
    """mvn_prob (nu = 0) or mvt_prob (nu > 0); returns the result dict
    (with 'logp', M x N, when return_logp)."""
    a, b = _f64(a), _f64(b)
    n = factor.stats()["n"]
    if a.shape != (n,) or b.shape != (n,):
        raise ValueError(f"a and b must have {n} entries")
    logp = np.empty(int(N) * int(M)) if return_logp else None
    o = _opts(N, M, seed, precision, logp, profile, chunk)
    res = Result()
    if nu == 0:
        st = _check(lib().mvn_prob(ctx.handle, factor.handle, a.ctypes.data, b.ctypes.data, C.byref(o),
                                   C.byref(res)))
    else:
        st = _check(lib().mvt_prob(ctx.handle, factor.handle, a.ctypes.data, b.ctypes.data, float(nu),
                                   C.byref(o), C.byref(res)))
    out = _result(res, st)
    if return_logp:
        out["logp"] = logp.reshape(int(M), int(N))
    return out


def probability_noalloc(ctx: Context, factor: Factor, a, b, N: int, M: int, seed: int, nu: float = 0.0,
                        precision: int = 0, chunk: int = 0) -> dict:
    """tlrqmc_prob_noalloc: the estimate of probability() with every device
    buffer taken from the library's fixed scratch array (no allocation)."""
    a, b = _f64(a), _f64(b)
    n = factor.stats()["n"]
    if a.shape != (n,) or b.shape != (n,):
        raise ValueError(f"a and b must have {n} entries")
    o = _opts(N, M, seed, precision, None, False, chunk)
    res = Result()
    st = _check(lib().tlrqmc_prob_noalloc(ctx.handle, factor.handle, a.ctypes.data, b.ctypes.data, float(nu),
                                          C.byref(o), C.byref(res)))
    return _result(res, st)


def mvn_prob(ctx, factor, a, b, N, M, seed, **kw):
    return probability(ctx, factor, a, b, N, M, seed, 0.0, **kw)


def mvt_prob(ctx, factor, a, b, nu, N, M, seed, **kw):
    if not nu > 0:
        raise ValueError("nu must be > 0")
    return probability(ctx, factor, a, b, N, M, seed, nu, **kw)


def sample_logp(ctx: Context, factor: Factor, a, b, nu: float, N: int, M: int, seed: int, shift: int,
                k0: int, count: int, precision: int = 0, chunk: int = 0) -> np.ndarray:
    a, b = _f64(a), _f64(b)
    n = factor.stats()["n"]
    if a.shape != (n,) or b.shape != (n,):
        raise ValueError(f"a and b must have {n} entries")
    out = np.empty(int(count))
    o = _opts(N, M, seed, precision, None, False, chunk)
    _check(lib().tlrqmc_sample_logp(ctx.handle, factor.handle, a.ctypes.data, b.ctypes.data, float(nu),
                                    C.byref(o), int(shift), int(k0), int(count), out.ctypes.data))
    return out


def skewnormal_loglik(ctx: Context, xy, z, xi: float, sigma1: float, beta1: float, sigma2: float, beta2: float,
                      N: int, M: int, seed: int, m: int = 128, tol: float = 1e-5, max_rank: int = 0,
                      order: int = 0, precision: int = 0, return_factor: bool = False) -> dict:
    """Skew-normal log-likelihood (Eq. 6) of observations z at locations xy;
    order 0 = geometric, 2 = block reordering during the Cholesky factorization."""
    xy, z = _f64(xy), _f64(z)
    n = len(z)
    if xy.shape != (n, 2):
        raise ValueError(f"xy must be {n} x 2")
    prm = SkewNormalParams(float(xi), float(sigma1), float(beta1), float(sigma2), float(beta2))
    o = _opts(N, M, seed, precision, None, False, 0)
    res = SkewNormalResult()
    c = np.empty(n)
    h = C.c_void_p()
    st = _check(lib().tlrqmc_skewnormal_loglik(ctx.handle, n, xy.ctypes.data, z.ctypes.data, C.byref(prm), int(m),
                                               float(tol), int(max_rank), int(order), C.byref(o), C.byref(res),
                                               c.ctypes.data, C.byref(h) if return_factor else None))
    out = {"loglik": res.loglik, "log_density": res.log_density, "log_prob": res.log_prob,
           "log_prob_std_err": res.log_prob_std_err, "log_prob_rel_err": res.log_prob_rel_err,
           "seconds": {"linear_algebra": res.seconds[0], "factor": res.seconds[1], "estimate": res.seconds[2]},
           "c": c, "prob": _result(res.prob, st)}
    if return_factor:
        out["factor"] = Factor(ctx, h)
    return out


class Server:
    """Request server (continuous batching with footprint admission) on ctx's device.

    submit() copies the request and returns a ticket; result(ticket) waits
    for it and returns the result dict with an 'info' entry (timings in
    seconds since the server started, reservation, slots)."""

    def __init__(self, ctx: Context, budget_bytes: int):
        self.ctx = ctx
        h = C.c_void_p()
        _check(lib().tlrqmc_server_create(ctx.handle, int(budget_bytes), C.byref(h)))
        self.handle = h

    def submit(self, cov: dict, a, b, N: int, M: int, seed: int, nu: float = 0.0, m: int = 128,
               tol: float = 1e-5, max_rank: int = 0, reorder: bool = False, precision: int = 0) -> int:
        a, b = _f64(a), _f64(b)
        n = len(a)
        if b.shape != (n,):
            raise ValueError("a and b must have the same length")
        cv, keep = _cov(cov, n)
        req = Request(n, cv, a.ctypes.data, b.ctypes.data, float(nu), int(m), int(max_rank), float(tol),
                      int(bool(reorder)), 0, _opts(N, M, seed, precision, None, False, 0))
        t = C.c_uint64()
        _check(lib().tlrqmc_server_submit(self.handle, C.byref(req), C.byref(t)))
        return t.value

    def poll(self, ticket: int, wait_s: float = 0.0):
        """Result dict, or None while the request is pending (after waiting
        up to wait_s seconds; wait_s < 0 waits until it is done)."""
        res, inf = Result(), RequestInfo()
        wait_ms = -1 if wait_s < 0 else int(min(wait_s * 1e3, 2 ** 31 - 1))
        st = lib().tlrqmc_server_poll(self.handle, int(ticket), wait_ms, C.byref(res), C.byref(inf))
        if st == PENDING:
            return None
        _check(st)
        out = _result(res, st)
        out["info"] = {k: getattr(inf, k) for k, _ in RequestInfo._fields_}
        return out

    def result(self, ticket: int, timeout_s: float = -1.0):
        """Wait for a ticket's result (TimeoutError after timeout_s > 0 seconds)."""
        out = self.poll(ticket, timeout_s)
        if out is None:
            raise TimeoutError(f"request {ticket} not done after {timeout_s} s")
        return out

    def stats(self) -> dict:
        inf = ServerInfo()
        _check(lib().tlrqmc_server_stats(self.handle, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in ServerInfo._fields_}

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().tlrqmc_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def log_relative_gap(x: float, y: float) -> float:
    """|x - y| / max(|x|, |y|), with equal infinities counted as 0."""
    if x == y:
        return 0.0
    if math.isinf(x) or math.isinf(y):
        return math.inf
    return abs(x - y) / max(abs(x), abs(y), 1e-300)
