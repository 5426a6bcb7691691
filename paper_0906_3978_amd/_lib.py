"""ctypes binding of libwiener.so (include/wiener.h).

Argument marshalling only: every step of the reconstruction runs in the HIP
library.  numpy arrays are passed as host memory (WF_HOST); torch tensors on
the GPU as device memory (WF_DEVICE).  PyTorch supplies the device allocator
(its caching allocator, through the ABI's callbacks) and the stream.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwiener.so")

WF_OK, WF_EINVAL, WF_ESTATE, WF_ENOMEM, WF_EDEVICE, WF_ENOTCONV, WF_EOVERFLOW, WF_EBREAKDOWN = range(8)
STATUS_NAMES = ["WF_OK", "WF_EINVAL", "WF_ESTATE", "WF_ENOMEM", "WF_EDEVICE", "WF_ENOTCONV",
                "WF_EOVERFLOW", "WF_EBREAKDOWN"]
WF_HOST, WF_DEVICE = 0, 1
SCHEMES = {"ngp": 0, "cic": 1, "tsc": 2}
PRECISIONS = {"fp64": 0, "mixed": 1}
PRECONDS = {"none": 0, "prior": 1}

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class SolveOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("inner_tol", C.c_double), ("max_outer", C.c_int32), ("check_every", C.c_int32),
                ("precond", C.c_int32), ("err_tol", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iters_total", C.c_int32), ("outer_steps", C.c_int32),
                ("rel_res_recursive", C.c_double), ("rel_res_true", C.c_double),
                ("time_ms", C.c_double), ("model_bytes", C.c_double), ("nbar", C.c_double),
                ("status", C.c_int32), ("last_change", C.c_double), ("latency_ms", C.c_double),
                ("stagnated", C.c_int32)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["status_name"] = STATUS_NAMES[self.status] if 0 <= self.status < 8 else str(self.status)
        return d


class Request(C.Structure):
    _fields_ = [("n", C.c_int32), ("box_mpc", C.c_double), ("w", C.c_void_p),
                ("p_by_m2", C.c_void_p), ("xyz", C.c_void_p), ("n_gal", C.c_int64),
                ("scheme", C.c_int), ("supersample", C.c_int32), ("opts", SolveOpts)]


PROF_KINDS = 22
PROF_NAMES = ["zfwd_f32", "yfwd_f32", "xlam_f32", "yinv_f32", "zinv_f32", "update_f32",
              "zfwd_f64", "yfwd_f64", "xlam_f64", "yinv_f64", "zinv_f64", "update_f64",
              "deposit", "supersample",
              "sdir_f32", "sxinv_f32", "szw_f32", "sxfwd_f32",
              "sdir_f64", "sxinv_f64", "szw_f64", "sxfwd_f64"]


class Profile(C.Structure):
    _fields_ = [("launches", C.c_int64 * PROF_KINDS), ("skipped", C.c_int64 * PROF_KINDS),
                ("ms", C.c_double * PROF_KINDS), ("bytes", C.c_double * PROF_KINDS)]

    def as_dict(self):
        return {PROF_NAMES[k]: dict(launches=int(self.launches[k]), skipped=int(self.skipped[k]),
                                    ms=float(self.ms[k]), bytes=float(self.bytes[k]))
                for k in range(PROF_KINDS) if self.launches[k]}


class ServerStats(C.Structure):
    _fields_ = [("completed", C.c_int64), ("failed", C.c_int64), ("solves_per_s", C.c_double),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("peak_bytes", C.c_size_t),
                ("cohorts", C.c_int64), ("largest_cohort", C.c_int32)]


class WienerError(RuntimeError):
    def __init__(self, code, msg):
        self.code = code
        name = STATUS_NAMES[code] if 0 <= code < 8 else str(code)
        super().__init__(f"{name}: {msg}")


_LIB = None

# name -> (restype, argtypes)
_V, _P, _I32, _I64, _D, _SZ = C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
SIGNATURES = {
    "wf_abi_version": (C.c_int, []),
    "wf_status_str": (C.c_char_p, [C.c_int]),
    "wf_ctx_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, _V, ALLOC_FN, FREE_FN, _V]),
    "wf_ctx_destroy": (C.c_int, [_V]),
    "wf_last_error": (C.c_char_p, [_V]),
    "wf_set_grid": (C.c_int, [_V, _I32, _D]),
    "wf_set_mask": (C.c_int, [_V, _P, C.c_int]),
    "wf_set_power": (C.c_int, [_V, _P, _I64, C.c_int]),
    "wf_set_galaxies": (C.c_int, [_V, _P, _I64, C.c_int]),
    "wf_deposit": (C.c_int, [_V, C.c_int, _I32]),
    "wf_get_deposit": (C.c_int, [_V, _P, _P, _P, C.c_int]),
    "wf_set_rhs": (C.c_int, [_V, _P, _D, C.c_int]),
    "wf_apply_operator": (C.c_int, [_V, C.c_int, _P, _P, C.c_int]),
    "wf_forward_spectrum": (C.c_int, [_V, C.c_int, _P, _P, C.c_int]),
    "wf_solve": (C.c_int, [_V, C.POINTER(SolveOpts), _P, C.c_int, C.POINTER(SolveInfo)]),
    "wf_solve_begin": (C.c_int, [_V, C.POINTER(SolveOpts)]),
    "wf_solve_step": (C.c_int, [_V, _I32, C.POINTER(C.c_int32)]),
    "wf_snapshot_bytes": (_SZ, [_V]),
    "wf_solve_snapshot": (C.c_int, [_V, _P, _SZ]),
    "wf_solve_resume": (C.c_int, [_V, _P, _SZ]),
    "wf_solve_finish": (C.c_int, [_V, _P, C.c_int, C.POINTER(SolveInfo)]),
    "wf_solve_batch": (C.c_int, [_V, _I32, C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.c_int,
                                 _I32, C.POINTER(SolveOpts), C.POINTER(C.c_void_p), C.c_int,
                                 C.POINTER(SolveInfo)]),
    "wf_footprint_bytes": (_SZ, [_I32, _I32, C.c_int, _I32]),
    "wf_rsd_factor": (C.c_int, [_V, C.c_double, C.c_double, _P, C.c_int64, C.c_int]),
    "wf_fourier_filter": (C.c_int, [_V, _I32, C.c_double, C.c_double, C.c_double, _P, C.c_int64,
                                    _P, _P, C.c_int]),
    "wf_field_moments": (C.c_int, [_V, _P, _I32, _P, C.c_int]),
    "wf_field_moments_noalloc": (C.c_int, [_V, _P, _I32, _P]),
    "wf_compare_fields": (C.c_int, [_V, _P, _P, _I32, _P, C.c_int]),
    "wf_inverse_weighting": (C.c_int, [_V, C.c_int, _I32, _P, C.c_int]),
    "wf_jackknife_counts": (C.c_int, [_V, _D, C.c_uint64, C.c_int64, _I32, _P, C.c_int]),
    "wf_solve_sd": (C.c_int, [_V, C.POINTER(SolveOpts), _I32, _D, C.c_uint64, C.c_int64, _I32,
                              _P, _P, C.c_int, C.POINTER(SolveInfo)]),
    "wf_profile_enable": (C.c_int, [_V, _I32]),
    "wf_profile_read": (C.c_int, [_V, C.POINTER(Profile)]),
    "wf_server_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, _SZ, _I32, ALLOC_FN, FREE_FN, _V]),
    "wf_server_submit": (C.c_int, [_V, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "wf_server_poll": (C.c_int, [_V, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(SolveInfo)]),
    "wf_server_fetch": (C.c_int, [_V, C.c_uint64, _P]),
    "wf_server_cancel": (C.c_int, [_V, C.c_uint64]),
    "wf_server_stats_get": (C.c_int, [_V, C.POINTER(ServerStats)]),
    "wf_server_last_error": (C.c_char_p, [_V]),
    "wf_server_destroy": (C.c_int, [_V]),
}


def lib():
    """Loads libwiener.so; raises if it has not been built (no fallback)."""
    global _LIB
    if _LIB is None:
        # torch ships its own HIP runtime under the same soname; load it first
        # so that the process holds exactly one runtime whichever module the
        # caller imported first.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_0906_3978_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _ptr(a):
    """(pointer, mem) of a numpy array (host) or a torch GPU tensor (device)."""
    if a is None:
        return None, WF_HOST
    if isinstance(a, np.ndarray):
        if not a.flags.c_contiguous:
            raise ValueError("arrays must be C-contiguous")
        return a.ctypes.data, WF_HOST
    if hasattr(a, "data_ptr") and hasattr(a, "is_cuda"):
        if not a.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return a.data_ptr(), (WF_DEVICE if a.is_cuda else WF_HOST)
    raise TypeError(f"unsupported array type {type(a)}")


_DTYPES = {"f64": (np.float64, "float64"), "i64": (np.int64, "int64"),
           "i32": (np.int32, "int32")}


def _arg(a, kind, count, what, device=None):
    """(pointer, mem) of an array the library reads or writes as `count`
    elements of `kind` ("f64", "i64", "i32"): a numpy array, or a torch tensor
    (on `device` when it is a GPU tensor).  The library trusts the sizes its
    arguments imply, so a wrong dtype, size or device is refused here, before
    any call into it."""
    if a is None:
        return None, WF_HOST
    np_t, torch_name = _DTYPES[kind]
    if isinstance(a, np.ndarray):
        if a.dtype != np_t:
            raise TypeError(f"{what}: dtype {a.dtype}, expected {torch_name}")
        numel = a.size
    elif hasattr(a, "data_ptr") and hasattr(a, "is_cuda"):
        if str(a.dtype) != "torch." + torch_name:
            raise TypeError(f"{what}: dtype {a.dtype}, expected torch.{torch_name}")
        if a.is_cuda and device is not None and a.device.index != device:
            raise ValueError(f"{what}: tensor on cuda:{a.device.index}, the context is on "
                             f"cuda:{device}")
        numel = a.numel()
    else:
        raise TypeError(f"{what}: unsupported array type {type(a)}")
    if count is not None and numel != count:
        raise ValueError(f"{what}: {numel} elements, expected {count}")
    return _ptr(a)


def _torch_allocator(device):
    import torch

    def alloc(nbytes, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device)
        except Exception:  # out of memory: the library reports WF_ENOMEM
            return None

    def free(ptr, user):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except AttributeError:  # interpreter shutdown: torch is already torn down
            pass

    return ALLOC_FN(alloc), FREE_FN(free)


@dataclass
class Info:
    iters_total: int
    outer_steps: int
    rel_res_recursive: float
    rel_res_true: float
    time_ms: float
    model_bytes: float
    nbar: float
    status: int
    last_change: float
    latency_ms: float
    stagnated: int
    status_name: str


def _info(si):
    return Info(**si.as_dict())


def opts(precision="fp64", tol=1e-10, max_iter=10000, inner_tol=0.0, max_outer=0, check_every=0,
         precond="none", err_tol=0.0):
    return SolveOpts(PRECISIONS[precision], tol, max_iter, inner_tol, max_outer, check_every,
                     PRECONDS[precond], err_tol)


class Context:
    """One wf_ctx on a GPU.  Device memory comes from torch's caching allocator
    and work goes on torch's current stream unless told otherwise."""

    def __init__(self, device=0, stream=None, torch_allocator=True):
        L = lib()
        self._L = L
        self.device = device
        h = C.c_void_p()
        self._cbs = (ALLOC_FN(), FREE_FN())
        if torch_allocator:
            import torch
            torch.cuda.set_device(device)
            self._cbs = _torch_allocator(device)
            if stream is None:
                stream = torch.cuda.current_stream(device).cuda_stream
        self._check(L.wf_ctx_create(C.byref(h), device, stream, self._cbs[0], self._cbs[1], None), None)
        self._h = h
        self.n = None
        self.box = None

    def close(self):
        if getattr(self, "_h", None):
            self._L.wf_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, code, h="self", ok=(WF_OK,)):
        if code in ok:
            return code
        if h == "self":
            msg = self._L.wf_last_error(self._h)
            msg = msg.decode() if msg else ""
        else:
            msg = self._L.wf_status_str(code).decode()
        raise WienerError(code, msg)

    # ---- inputs ---------------------------------------------------------
    def set_grid(self, n, box):
        self._check(self._L.wf_set_grid(self._h, int(n), float(box)))
        self.n, self.box = int(n), float(box)

    def _m(self):
        if self.n is None:
            raise WienerError(2, "set_grid first")
        return self.n ** 3

    def set_mask(self, w):
        w = _as_f64(w)
        p, mem = _arg(w, "f64", self._m(), "mask", self.device)
        self._check(self._L.wf_set_mask(self._h, p, mem))

    def set_power(self, p_by_m2):
        a = _as_f64(p_by_m2)
        p, mem = _arg(a, "f64", None, "p_by_m2", self.device)
        self._check(self._L.wf_set_power(self._h, p, int(_numel(a)), mem))

    def set_galaxies(self, xyz):
        a = _as_f64(xyz)
        if _numel(a) % 3:
            raise ValueError("xyz: the element count must be a multiple of 3")
        p, mem = _arg(a, "f64", None, "xyz", self.device)
        self._check(self._L.wf_set_galaxies(self._h, p, int(_numel(a) // 3), mem))

    def deposit(self, scheme="cic", supersample=1):
        self._check(self._L.wf_deposit(self._h, SCHEMES[scheme], int(supersample)))

    def get_deposit(self, fine=True, n_obs=True, supersample=1):
        n = self.n
        nf = supersample * n
        g = np.empty((nf, nf, nf), dtype=np.int64) if fine else None
        o = np.empty((n, n, n), dtype=np.float64) if n_obs else None
        nb = C.c_double()
        self._check(self._L.wf_get_deposit(self._h, _ptr(g)[0], _ptr(o)[0], C.byref(nb), WF_HOST))
        return g, o, nb.value

    def set_rhs(self, b, nbar):
        b = _as_f64(b)
        p, mem = _arg(b, "f64", self._m(), "b", self.device)
        self._check(self._L.wf_set_rhs(self._h, p, float(nbar), mem))

    def apply_operator(self, v, precision="fp64"):
        v = np.ascontiguousarray(v, dtype=np.float64)
        _arg(v, "f64", self._m(), "v")
        out = np.empty_like(v)
        self._check(self._L.wf_apply_operator(self._h, PRECISIONS[precision], _ptr(v)[0],
                                              _ptr(out)[0], WF_HOST))
        return out

    def forward_spectrum(self, v, precision="fp64"):
        v = np.ascontiguousarray(v, dtype=np.float64)
        _arg(v, "f64", self._m(), "v")
        n = self.n
        out = np.empty((n, n, n // 2 + 1), dtype=np.complex128)
        self._check(self._L.wf_forward_spectrum(self._h, PRECISIONS[precision], _ptr(v)[0],
                                                out.ctypes.data, WF_HOST))
        return out

    # ---- after the solve (redshift space, filters, comparators) ---------
    def rsd_factor(self, beta, sigma_mpc, length=None):
        """<K D>_mu at k = (2 pi / L) sqrt(j), j < length (default 3 (n/2)^2 + 1)."""
        n = self.n
        length = length or 3 * (n // 2) ** 2 + 1
        out = np.empty(length, dtype=np.float64)
        self._check(self._L.wf_rsd_factor(self._h, float(beta), float(sigma_mpc), out.ctypes.data,
                                          length, WF_HOST))
        return out

    def fourier_filter(self, v, kind, a=0.0, b=0.0, c=1.0, table=None, out=None):
        """F^-1 diag(h) F v; kind "gauss" (a = r_S), "rsd_deconv" (a = beta,
        b = sigma, c = bias) or "table" (h by |m|^2)."""
        kinds = {"gauss": 0, "rsd_deconv": 1, "table": 2}
        m = self._m()
        p, mem = _arg(v, "f64", m, "v", self.device)
        if out is None:
            out = np.empty(v.shape, dtype=np.float64) if mem == WF_HOST else v.new_empty(v.shape)
        po, mo = _arg(out, "f64", m, "out", self.device)
        if mo != mem:
            raise ValueError("v and out must both be host arrays or both device tensors")
        tp, tl = (None, 0)
        if table is not None:
            table = _as_f64(table) if mem == WF_HOST else table
            tp, tm = _arg(table, "f64", None, "table", self.device)
            if tm != mem:
                raise ValueError("table must live where v does")
            tl = int(_numel(table))
        self._check(self._L.wf_fourier_filter(self._h, kinds[kind], float(a), float(b), float(c),
                                              tp, tl, p, po, mem))
        return out

    def field_moments(self, v, masked=False):
        """(count, mean, variance, skewness, excess kurtosis) over all cells or w > 0."""
        p, mem = _arg(v, "f64", self._m(), "v", self.device)
        out = np.empty(5, dtype=np.float64)
        self._check(self._L.wf_field_moments(self._h, p, int(bool(masked)), out.ctypes.data, mem))
        return tuple(float(x) for x in out)

    def field_moments_noalloc(self, v, masked=False):
        """field_moments of a device tensor through the allocation-free entry
        point (its partials in a static device array shared by every call on
        the GPU)."""
        p, mem = _arg(v, "f64", self._m(), "v", self.device)
        if mem != WF_DEVICE:
            raise ValueError("v must be a GPU tensor")
        out = np.empty(5, dtype=np.float64)
        self._check(self._L.wf_field_moments_noalloc(self._h, p, int(bool(masked)),
                                                     out.ctypes.data))
        return tuple(float(x) for x in out)

    def compare_fields(self, rec, truth, masked=False):
        """(r, D_Euc, D_KL) between a reconstruction and a reference field."""
        pr, mem = _arg(rec, "f64", self._m(), "rec", self.device)
        pt, mt = _arg(truth, "f64", self._m(), "truth", self.device)
        if mt != mem:
            raise ValueError("rec and truth must both be host arrays or both device tensors")
        out = np.empty(3, dtype=np.float64)
        self._check(self._L.wf_compare_fields(self._h, pr, pt, int(bool(masked)), out.ctypes.data,
                                              mem))
        return tuple(float(x) for x in out)

    def inverse_weighting(self, scheme="cic", supersample=2, out=None):
        """delta_IW from the galaxies of set_galaxies (1/w weights, deposit, low-pass)."""
        n = self.n
        if out is None:
            out = np.empty((n, n, n), dtype=np.float64)
        p, mem = _arg(out, "f64", self._m(), "out", self.device)
        self._check(self._L.wf_inverse_weighting(self._h, SCHEMES[scheme], int(supersample), p, mem))
        return out

    # ---- solves ---------------------------------------------------------
    def solve(self, out=None, allow=(WF_OK,), **kw):
        o = opts(**kw)
        n = self.n
        if out is None:
            out = np.empty((n, n, n), dtype=np.float64)
        p, mem = _arg(out, "f64", self._m(), "out", self.device)
        si = SolveInfo()
        code = self._L.wf_solve(self._h, C.byref(o), p, mem, C.byref(si))
        self._check(code, ok=allow)
        return out, _info(si)

    def solve_begin(self, **kw):
        o = opts(**kw)
        self._check(self._L.wf_solve_begin(self._h, C.byref(o)))

    def solve_step(self, iters):
        d = C.c_int32()
        self._check(self._L.wf_solve_step(self._h, int(iters), C.byref(d)))
        return bool(d.value)

    def snapshot(self):
        nb = self._L.wf_snapshot_bytes(self._h)
        buf = np.empty(nb, dtype=np.uint8)
        self._check(self._L.wf_solve_snapshot(self._h, buf.ctypes.data, nb))
        return buf

    def resume(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self._L.wf_solve_resume(self._h, buf.ctypes.data, buf.size))

    def solve_finish(self, allow=(WF_OK,)):
        n = self.n
        out = np.empty((n, n, n), dtype=np.float64)
        si = SolveInfo()
        self._check(self._L.wf_solve_finish(self._h, out.ctypes.data, WF_HOST, C.byref(si)), ok=allow)
        return out, _info(si)

    def profile_enable(self, on=True, every=1):
        """Event timing on or off; with every > 1 one launch in `every` of
        each kernel class is timed."""
        every = int(every)
        if every < 1:
            raise ValueError("every must be >= 1")
        self._check(self._L.wf_profile_enable(self._h, every if on else 0))

    def profile_read(self):
        pr = Profile()
        self._check(self._L.wf_profile_read(self._h, C.byref(pr)))
        return pr.as_dict()

    def solve_batch(self, catalogues, scheme="cic", supersample=2, outs=None,
                    allow=(WF_OK,), **kw):
        o = opts(**kw)
        nr = len(catalogues)
        cats = [_as_f64(c) for c in catalogues]
        n = self.n
        if outs is None:
            outs = [np.empty((n, n, n), dtype=np.float64) for _ in range(nr)]
        m = self._m()
        mem = _ptr(cats[0])[1] if nr else WF_HOST
        for i, c in enumerate(cats):
            if _numel(c) % 3:
                raise ValueError(f"catalogue {i}: the element count must be a multiple of 3")
            if _arg(c, "f64", None, f"catalogue {i}", self.device)[1] != mem:
                raise ValueError("catalogues must all be host arrays or all device tensors")
        if len(outs) != nr:
            raise ValueError(f"{len(outs)} outputs for {nr} catalogues")
        for i, x in enumerate(outs):
            if _arg(x, "f64", m, f"output {i}", self.device)[1] != mem:
                raise ValueError("outputs must live where the catalogues do")
        xp = (C.c_void_p * nr)(*[_ptr(c)[0] for c in cats])
        ng = (C.c_int64 * nr)(*[int(_numel(c) // 3) for c in cats])
        op = (C.c_void_p * nr)(*[_ptr(x)[0] for x in outs])
        infos = (SolveInfo * nr)()
        code = self._L.wf_solve_batch(self._h, nr, xp, ng, SCHEMES[scheme], int(supersample),
                                      C.byref(o), op, mem, infos)
        self._check(code, ok=allow)
        return outs, [_info(i) for i in infos]

    # ---- signal-dependent noise ------------------------------------------
    def jackknife_counts(self, alpha, seed, first=0, count=1, out=None):
        """Thinned counts N' of jackknife samples first .. first + count - 1
        (count x n^3 int32)."""
        n = self.n
        if out is None:
            out = np.empty((count, n, n, n), dtype=np.int32)
        p, mem = _arg(out, "i32", int(count) * self._m(), "out", self.device)
        self._check(self._L.wf_jackknife_counts(self._h, float(alpha), int(seed), int(first),
                                                int(count), p, mem))
        return out

    def solve_sd(self, kind="mean", alpha=0.0, seed=0, first=0, nsamples=1, mean_out=None,
                 samples_out=None, keep_samples=False, allow=(WF_OK,), **kw):
        """Signal-dependent noise reconstruction of the last deposit: kind
        "mean" (one solve) or "jackknife" (nsamples solves); returns the mean
        of the solutions, the solutions (if asked for) and the infos."""
        o = opts(**kw)
        n = self.n
        kinds = {"mean": 1, "jackknife": 2}
        if mean_out is None:
            mean_out = np.empty((n, n, n), dtype=np.float64)
        p, mem = _arg(mean_out, "f64", self._m(), "mean_out", self.device)
        if samples_out is None and keep_samples:
            samples_out = (np.empty((nsamples, n, n, n), dtype=np.float64) if mem == WF_HOST
                           else mean_out.new_empty((nsamples, n, n, n)))
        sp = None
        if samples_out is not None:
            sp, sm = _arg(samples_out, "f64", int(nsamples) * self._m(), "samples_out",
                          self.device)
            if sm != mem:
                raise ValueError("samples_out must live where mean_out does")
        infos = (SolveInfo * nsamples)()
        code = self._L.wf_solve_sd(self._h, C.byref(o), kinds[kind], float(alpha), int(seed),
                                   int(first), int(nsamples), p, sp, mem, infos)
        self._check(code, ok=allow)
        return mean_out, samples_out, [_info(i) for i in infos]


def footprint_bytes(n, supersample=2, precision="mixed", nrhs=1):
    return int(lib().wf_footprint_bytes(n, supersample, PRECISIONS[precision], nrhs))


def _as_f64(a):
    if isinstance(a, np.ndarray):
        return np.ascontiguousarray(a, dtype=np.float64)
    return a


def _numel(a):
    if isinstance(a, np.ndarray):
        return a.size
    return a.numel()


class Server:
    """Continuous-batching reconstruction server (wf_server_*).  Device memory
    for the whole budget is taken once (torch's caching allocator by default);
    requests are admitted into it as they fit."""

    def __init__(self, device=0, hbm_budget=8 << 30, max_active=8, torch_allocator=True):
        L = lib()
        self._L = L
        self._cbs = (ALLOC_FN(), FREE_FN())
        if torch_allocator:
            import torch
            torch.cuda.set_device(device)
            self._cbs = _torch_allocator(device)
        h = C.c_void_p()
        code = L.wf_server_create(C.byref(h), device, int(hbm_budget), int(max_active),
                                  self._cbs[0], self._cbs[1], None)
        if code != WF_OK:
            raise WienerError(code, L.wf_status_str(code).decode())
        self._h = h
        self._grid = {}   # ticket -> grid size of the request

    def _err(self, code):
        msg = self._L.wf_server_last_error(self._h)
        raise WienerError(code, msg.decode() if msg else "")

    def submit(self, n, box, w, p_by_m2, xyz, scheme="cic", supersample=2, **kw):
        n = int(n)
        w = np.ascontiguousarray(w, dtype=np.float64)
        p = np.ascontiguousarray(p_by_m2, dtype=np.float64)
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        if w.size != n ** 3:
            raise ValueError(f"w: {w.size} elements, expected {n ** 3}")
        if p.size != 3 * (n // 2) ** 2 + 1:
            raise ValueError(f"p_by_m2: {p.size} elements, expected {3 * (n // 2) ** 2 + 1}")
        if xyz.size % 3:
            raise ValueError("xyz: the element count must be a multiple of 3")
        xyz = xyz.reshape(-1, 3)
        req = Request(int(n), float(box), w.ctypes.data, p.ctypes.data,
                      xyz.ctypes.data if len(xyz) else None, len(xyz), SCHEMES[scheme],
                      int(supersample), opts(**kw))
        t = C.c_uint64()
        code = self._L.wf_server_submit(self._h, C.byref(req), C.byref(t))
        if code != WF_OK:
            self._err(code)
        self._grid[int(t.value)] = n
        return int(t.value)

    def poll(self, ticket):
        d = C.c_int32()
        si = SolveInfo()
        code = self._L.wf_server_poll(self._h, ticket, C.byref(d), C.byref(si))
        if code != WF_OK:
            self._err(code)
        return bool(d.value), (_info(si) if d.value else None)

    def fetch(self, ticket, n=None, allow=(WF_OK,)):
        """The result of a finished request (n^3 doubles, n the request's grid)."""
        g = self._grid.get(ticket)
        if g is None:
            raise ValueError(f"unknown ticket {ticket}")
        if n is not None and int(n) != g:
            raise ValueError(f"ticket {ticket} is a {g}^3 request, not {n}^3")
        done, _ = self.poll(ticket)
        if not done:
            raise WienerError(2, f"request {ticket} not finished")
        out = np.empty((g, g, g), dtype=np.float64)
        code = self._L.wf_server_fetch(self._h, ticket, out.ctypes.data)
        self._grid.pop(ticket, None)   # a finished ticket is released by the fetch
        if code not in allow:
            self._err(code)
        return out

    def wait(self, ticket, n, timeout=120.0, allow=(WF_OK,)):
        import time
        t0 = time.time()
        while True:
            done, info = self.poll(ticket)
            if done:
                return self.fetch(ticket, n, allow), info
            if time.time() - t0 > timeout:
                raise TimeoutError(f"request {ticket} not done after {timeout} s")
            time.sleep(0.0005)

    def cancel(self, ticket):
        code = self._L.wf_server_cancel(self._h, ticket)
        if code != WF_OK:
            self._err(code)

    def stats(self):
        st = ServerStats()
        self._L.wf_server_stats_get(self._h, C.byref(st))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self._L.wf_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
