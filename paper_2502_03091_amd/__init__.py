"""Python binding of libcrk.so, the chiral rank-k multigrid library for MI355X.

Argument marshalling only: every step of the setup and solve runs in the HIP
kernels of the shared library.  There is no CPU fallback; if the library is
missing or cannot be loaded every call raises.  PyTorch is used for device
memory and streams only (``*_dev`` calls take ``torch`` device tensors and the
current HIP stream).

Conventions are those of ``include/crk.h``: site index
s = x0 + L0*(x1 + L1*(x2 + L2*x3)), spinor component 3*spin + colour, host
fields complex128 ``[nrhs, V, 12]``, gauge complex128 ``[V, 4, 3, 3]``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcrk.so")

FORM_FP64, FORM_FP32, FORM_FP16S = 0, 1, 2
FORMS = {"fp64": 0, "fp32": 1, "fp16s": 2}

OK, EINVAL, ENOMEM, EHIP, ENOCONV, ESTATE, EBUSY, EINTERNAL = 0, -1, -2, -3, -4, -5, -6, -7
MAX_LEVELS = 3

GET_P, GET_SIGMA, GET_X, GET_YP, GET_YM, GET_VECTORS, GET_BLOCK_MAP, GET_DEVICE_ORDER = range(8)


class CrkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"crk error {code}: {msg}")
        self.code = code


class NoConvergence(CrkError):
    pass


class MGParams(C.Structure):
    _fields_ = [
        ("n_levels", C.c_int32),
        ("m_prime", C.c_int32 * MAX_LEVELS),
        ("k", C.c_int32 * MAX_LEVELS),
        ("block", (C.c_int32 * 4) * MAX_LEVELS),
        ("n_smooth", C.c_int32 * MAX_LEVELS),
        ("setup_form", C.c_int32),
        ("normalize", C.c_int32),
        ("seed", C.c_uint64),
        ("init_vectors", C.c_void_p * MAX_LEVELS),
        ("smooth_chunk", C.c_int32),
        ("svd_batch", C.c_int32),
        ("coarse_init", C.c_int32),
        ("smooth_defer", C.c_int32),
    ]


class SolveInfo(C.Structure):
    _fields_ = [
        ("tol", C.c_double),
        ("max_iter", C.c_int32),
        ("form", C.c_int32),
        ("restart", C.c_int32),
        ("tau", C.c_double),
        ("inner_maxit", C.c_int32),
        ("coarsest_maxit", C.c_int32),
        ("nu_post", C.c_int32),
        ("post_defer", C.c_int32),
        ("iters", C.c_int32),
        ("level_iters", C.c_int32 * MAX_LEVELS),
        ("true_rel_resid", C.c_double),
        ("seconds", C.c_double),
    ]

    def as_dict(self):
        return {
            "iters": self.iters,
            "level_iters": list(self.level_iters),
            "true_rel_resid": self.true_rel_resid,
            "seconds": self.seconds,
        }


class ServerParams(C.Structure):
    _fields_ = [
        ("hbm_budget_bytes", C.c_int64),
        ("slots_per_lane", C.c_int32),
        ("max_lanes", C.c_int32),
        ("idle_ms", C.c_int32),
        ("solve", SolveInfo),
    ]


class RequestInfo(C.Structure):
    _fields_ = [
        ("status", C.c_int32),
        ("lattice", C.c_int32),
        ("nrhs", C.c_int32),
        ("lane", C.c_int32),
        ("joined", C.c_int32),
        ("iters", C.c_int32),
        ("level_iters", C.c_int32 * MAX_LEVELS),
        ("true_rel_resid", C.c_double),
        ("t_submit", C.c_double),
        ("t_admit", C.c_double),
        ("t_done", C.c_double),
    ]

    def as_dict(self):
        return {k: (list(getattr(self, k)) if k == "level_iters" else getattr(self, k)) for k, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("submitted", "completed", "failed", "joins", "lanes_opened",
                                          "lanes_closed", "max_concurrent_lanes", "bytes_in_use", "peak_bytes",
                                          "budget_bytes")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it first (python -m paper_2502_03091_amd.build); "
            "there is no CPU fallback")
    # One HIP runtime per process: when PyTorch is installed its bundled HIP
    # runtime (same SONAME) must be loaded first, so the library shares it and
    # torch device memory and streams are valid in library calls.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "crk_version": (i32, []),
        "crk_last_error": (C.c_char_p, []),
        "crk_device_info": (i32, [C.c_char_p, i32, C.POINTER(i64), C.POINTER(i32)]),
        "crk_cached_memory_bytes": (i32, [C.POINTER(i64)]),
        "crk_release_cached_memory": (i32, []),
        "crk_create_lattice": (i32, [C.POINTER(i32), dbl, dbl, C.POINTER(vp)]),
        "crk_load_gauge": (i32, [vp, vp, i64]),
        "crk_lattice_set_clover": (i32, [vp, dbl]),
        "crk_dirac_apply": (i32, [vp, i32, vp, vp, i32]),
        "crk_dirac_apply_dev": (i32, [vp, i32, vp, vp, i32, vp]),
        "crk_dirac_apply_noalloc": (i32, [vp, i32, vp, vp, i32]),
        "crk_dirac_apply_noalloc_max_bytes": (i64, []),
        "crk_field_bytes": (i64, [vp, i32, i32]),
        "crk_field_import_dev": (i32, [vp, i32, vp, vp, i32, vp]),
        "crk_field_export_dev": (i32, [vp, i32, vp, vp, i32, vp]),
        "crk_lattice_get_map": (i32, [vp, i32, vp, i64]),
        "crk_lattice_destroy": (None, [vp]),
        "crk_mg_params_default": (None, [C.POINTER(MGParams)]),
        "crk_mg_setup": (i32, [vp, C.POINTER(MGParams), C.POINTER(vp)]),
        "crk_solve_info_default": (None, [C.POINTER(SolveInfo)]),
        "crk_mg_solve": (i32, [vp, vp, vp, i32, C.POINTER(SolveInfo)]),
        "crk_mg_solve_dev": (i32, [vp, vp, vp, i32, vp, C.POINTER(SolveInfo)]),
        "crk_mg_last_solve_rhs": (i32, [vp, C.POINTER(i32), C.POINTER(dbl), i32]),
        "crk_mg_last_solve_rhs_seconds": (i32, [vp, C.POINTER(dbl), i32]),
        "crk_mg_get": (i32, [vp, i32, i32, vp, i64]),
        "crk_mg_get_bytes": (i64, [vp, i32, i32]),
        "crk_mg_get_timing": (i32, [vp, i32, C.POINTER(dbl)]),
        "crk_mg_coarse_apply": (i32, [vp, i32, i32, vp, vp, i32]),
        "crk_mg_apply_dev": (i32, [vp, i32, i32, vp, vp, i32, vp]),
        "crk_mg_field_bytes": (i64, [vp, i32, i32, i32]),
        "crk_mg_restrict": (i32, [vp, i32, i32, vp, vp, i32]),
        "crk_mg_prolong": (i32, [vp, i32, i32, vp, vp, i32]),
        "crk_mg_footprint_bytes": (i64, [vp, i32, i32]),
        "crk_mg_destroy": (None, [vp]),
        "crk_server_params_default": (None, [C.POINTER(ServerParams)]),
        "crk_server_create": (i32, [C.POINTER(ServerParams), C.POINTER(vp)]),
        "crk_server_add": (i32, [vp, vp, C.POINTER(i32)]),
        "crk_server_submit": (i32, [vp, i32, vp, vp, i32, C.POINTER(C.c_uint64)]),
        "crk_server_wait": (i32, [vp, C.c_uint64, dbl, C.POINTER(RequestInfo)]),
        "crk_server_get_stats": (i32, [vp, C.POINTER(ServerStats)]),
        "crk_server_lane_bytes": (i64, [vp, i32]),
        "crk_server_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def lib():
    return _load()


def exported_symbols():
    """Names the binding expects the shared library to export."""
    return [
        "crk_version", "crk_last_error", "crk_device_info", "crk_cached_memory_bytes", "crk_release_cached_memory",
        "crk_create_lattice", "crk_load_gauge",
        "crk_lattice_set_clover",
        "crk_dirac_apply", "crk_dirac_apply_dev", "crk_dirac_apply_noalloc", "crk_dirac_apply_noalloc_max_bytes",
        "crk_field_bytes", "crk_field_import_dev",
        "crk_field_export_dev", "crk_lattice_get_map", "crk_lattice_destroy", "crk_mg_params_default",
        "crk_mg_setup", "crk_solve_info_default", "crk_mg_solve", "crk_mg_solve_dev",
        "crk_mg_last_solve_rhs", "crk_mg_last_solve_rhs_seconds", "crk_mg_get", "crk_mg_get_bytes", "crk_mg_get_timing",
        "crk_mg_coarse_apply", "crk_mg_apply_dev", "crk_mg_field_bytes", "crk_mg_restrict", "crk_mg_prolong",
        "crk_mg_footprint_bytes", "crk_mg_destroy",
    ]


def _check(rc, cls=CrkError):
    if rc != OK:
        msg = _load().crk_last_error().decode(errors="replace")
        if rc == ENOCONV:
            raise NoConvergence(rc, msg)
        raise cls(rc, msg)


def _cptr(a):
    return C.c_void_p(a.ctypes.data)


def _tptr(t):
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def device_info():
    name = C.create_string_buffer(64)
    hbm, ncu = C.c_int64(0), C.c_int32(0)
    _check(_load().crk_device_info(name, 64, C.byref(hbm), C.byref(ncu)))
    return {"arch": name.value.decode(), "hbm_bytes": hbm.value, "n_cu": ncu.value}


def cached_memory_bytes():
    """Device bytes the library holds for reuse on the current device (freed buffers kept for later requests)."""
    out = C.c_int64(0)
    _check(_load().crk_cached_memory_bytes(C.byref(out)))
    return out.value


def release_cached_memory():
    """Give the library's cached device buffers back to the HIP runtime (before large allocations elsewhere)."""
    _check(_load().crk_release_cached_memory())


def _as_c128(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    if shape is not None and a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a


class Lattice:
    """Periodic 4-D lattice with Wilson mass m0, temporal anisotropy xi and
    clover coefficient c_sw (0: the plain Wilson operator)."""

    def __init__(self, dims, m0, xi=1.0, c_sw=0.0):
        self.dims = [int(d) for d in dims]
        self.V = int(np.prod(self.dims))
        self.m0, self.xi, self.c_sw = float(m0), float(xi), float(c_sw)
        h = C.c_void_p()
        d = (C.c_int32 * 4)(*self.dims)
        _check(_load().crk_create_lattice(d, self.m0, self.xi, C.byref(h)))
        self._h = h
        if self.c_sw != 0.0:
            self.set_clover(self.c_sw)

    def set_clover(self, c_sw):
        self.c_sw = float(c_sw)
        _check(_load().crk_lattice_set_clover(self.handle, self.c_sw))

    def close(self):
        if getattr(self, "_h", None):
            _load().crk_lattice_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if not self._h:
            raise CrkError(ESTATE, "lattice closed")
        return self._h

    def load_gauge(self, U):
        U = _as_c128(U, (self.V, 4, 3, 3))
        _check(_load().crk_load_gauge(self.handle, _cptr(U), U.size * 2))

    def dirac_apply(self, psi, form=FORM_FP64):
        psi = _as_c128(psi)
        if psi.ndim == 2:
            psi = psi[None]
        assert psi.shape[1:] == (self.V, 12)
        out = np.empty_like(psi)
        _check(_load().crk_dirac_apply(self.handle, int(form), _cptr(psi), _cptr(out), psi.shape[0]))
        return out

    def dirac_apply_noalloc(self, psi, form=FORM_FP64):
        """As dirac_apply, staged through the library's fixed device scratch array
        (no device allocation; crk_dirac_apply_noalloc)."""
        psi = _as_c128(psi)
        if psi.ndim == 2:
            psi = psi[None]
        assert psi.shape[1:] == (self.V, 12)
        out = np.empty_like(psi)
        _check(_load().crk_dirac_apply_noalloc(self.handle, int(form), _cptr(psi), _cptr(out), psi.shape[0]))
        return out

    def field_bytes(self, form, nrhs):
        return int(_load().crk_field_bytes(self.handle, int(form), int(nrhs)))

    def dirac_apply_dev(self, inp, out, nrhs, form, stream=None):
        """Native-layout device tensors (see crk.h); stream-ordered."""
        _check(_load().crk_dirac_apply_dev(self.handle, int(form), _tptr(inp), _tptr(out), int(nrhs),
                                           _stream(stream)))

    def import_dev(self, host_layout, native, nrhs, form, stream=None):
        _check(_load().crk_field_import_dev(self.handle, int(form), _tptr(host_layout), _tptr(native),
                                            int(nrhs), _stream(stream)))

    def export_dev(self, native, host_layout, nrhs, form, stream=None):
        _check(_load().crk_field_export_dev(self.handle, int(form), _tptr(native), _tptr(host_layout),
                                            int(nrhs), _stream(stream)))

    def neighbor_map(self):
        out = np.empty((self.V, 8), dtype=np.int32)
        _check(_load().crk_lattice_get_map(self.handle, 0, _cptr(out), out.nbytes))
        return out


class Hierarchy:
    """Chiral rank-k multigrid hierarchy built on a Lattice (crk_mg_setup)."""

    def __init__(self, lattice, m_prime=(48,), k=(24,), block=((4, 4, 4, 4),), n_smooth=(20,),
                 setup_form=FORM_FP32, normalize=True, seed=0x2502030910, init_vectors=None, smooth_chunk=0,
                 svd_batch=0, coarse_init=False, smooth_defer=0):
        self.lattice = lattice
        p = MGParams()
        _load().crk_mg_params_default(C.byref(p))
        nsteps = len(m_prime)
        p.n_levels = nsteps + 1
        for l in range(nsteps):
            p.m_prime[l] = int(m_prime[l])
            p.k[l] = int(k[l])
            for mu in range(4):
                p.block[l][mu] = int(block[l][mu])
            p.n_smooth[l] = int(n_smooth[l])
        p.setup_form = int(setup_form)
        p.normalize = int(bool(normalize))
        p.seed = int(seed)
        p.smooth_chunk = int(smooth_chunk)
        p.svd_batch = int(svd_batch)
        p.coarse_init = int(bool(coarse_init))
        p.smooth_defer = int(smooth_defer)
        keep = []
        if init_vectors is not None:
            for l, v in enumerate(init_vectors):
                if v is None:
                    continue
                a = _as_c128(v)
                keep.append(a)
                p.init_vectors[l] = a.ctypes.data
        self.params = p
        h = C.c_void_p()
        _check(_load().crk_mg_setup(lattice.handle, C.byref(p), C.byref(h)))
        self._h = h
        self.n_levels = p.n_levels
        self.m_prime, self.k = list(m_prime), list(k)
        self.block = [list(b) for b in block]
        dims = list(lattice.dims)
        self.dims = [dims]
        self.ncomp = [12]
        for l in range(nsteps):
            dims = [d // b for d, b in zip(dims, self.block[l])]
            self.dims.append(dims)
            self.ncomp.append(2 * self.k[l])

    def close(self):
        if getattr(self, "_h", None):
            _load().crk_mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if not self._h:
            raise CrkError(ESTATE, "hierarchy closed")
        return self._h

    def volume(self, level):
        return int(np.prod(self.dims[level]))

    def get(self, level, what):
        n = int(_load().crk_mg_get_bytes(self.handle, level, what))
        if n < 0:
            raise CrkError(EINVAL, f"unknown quantity {what} at level {level}")
        if what in (GET_BLOCK_MAP, GET_DEVICE_ORDER):
            out = np.empty(n // 4, dtype=np.int32)
        elif what == GET_SIGMA:
            out = np.empty(n // 8, dtype=np.float64)
        else:
            out = np.empty(n // 16, dtype=np.complex128)
        _check(_load().crk_mg_get(self.handle, level, what, _cptr(out), n))
        return out

    def prolongator(self, level=0):
        """P blocks [d, 2, N_r, k] (rows h*l + c')."""
        k = self.k[level]
        d = self.volume(level + 1)
        return self.get(level, GET_P).reshape(d, 2, -1, k)

    def sigma(self, level=0):
        d = self.volume(level + 1)
        return self.get(level, GET_SIGMA).reshape(d, 2, -1)

    def coarse_links(self, level=0):
        """(X [Vc, N, N], Yp [4, Vc, N, N], Ym [4, Vc, N, N]) of level+1."""
        Vc, N = self.volume(level + 1), self.ncomp[level + 1]
        X = self.get(level, GET_X).reshape(Vc, N, N)
        Yp = self.get(level, GET_YP).reshape(4, Vc, N, N)
        Ym = self.get(level, GET_YM).reshape(4, Vc, N, N)
        return X, Yp, Ym

    def vectors(self, level=0):
        m = self.m_prime[level]
        return self.get(level, GET_VECTORS).reshape(m, self.volume(level), self.ncomp[level])

    def block_map(self, level=0):
        return self.get(level, GET_BLOCK_MAP).reshape(-1, 2)

    def timing(self, level=0):
        out = (C.c_double * 6)()
        _check(_load().crk_mg_get_timing(self.handle, level, out))
        keys = ["total", "smoother", "svd", "galerkin", "dslash_avg", "dslash_count"]
        return dict(zip(keys, list(out)))

    def coarse_apply(self, level, v, form=FORM_FP64):
        v = _as_c128(v)
        out = np.empty_like(v)
        _check(_load().crk_mg_coarse_apply(self.handle, level, int(form), _cptr(v), _cptr(out), v.shape[0]))
        return out

    def apply_dev(self, level, inp, out, nrhs, form, stream=None):
        """Operator of level `level` on device tensors in the hierarchy's own layout (see crk.h); stream-ordered."""
        _check(_load().crk_mg_apply_dev(self.handle, int(level), int(form), _tptr(inp), _tptr(out), int(nrhs),
                                        _stream(stream)))

    def field_bytes(self, level, form, nrhs):
        return int(_load().crk_mg_field_bytes(self.handle, int(level), int(form), int(nrhs)))

    def restrict(self, level, v, form=FORM_FP64):
        v = _as_c128(v)
        out = np.empty((v.shape[0], self.volume(level + 1), self.ncomp[level + 1]), dtype=np.complex128)
        _check(_load().crk_mg_restrict(self.handle, level, int(form), _cptr(v), _cptr(out), v.shape[0]))
        return out

    def prolong(self, level, vc, form=FORM_FP64):
        vc = _as_c128(vc)
        out = np.empty((vc.shape[0], self.volume(level), self.ncomp[level]), dtype=np.complex128)
        _check(_load().crk_mg_prolong(self.handle, level, int(form), _cptr(vc), _cptr(out), vc.shape[0]))
        return out

    @staticmethod
    def solve_params(**kw):
        info = SolveInfo()
        _load().crk_solve_info_default(C.byref(info))
        for k_, v_ in kw.items():
            if k_ == "form" and isinstance(v_, str):
                v_ = FORMS[v_]
            setattr(info, k_, v_)
        return info

    def solve(self, b, raise_on_noconv=True, **kw):
        """Host solve of D x = b, b complex128 [nrhs, V, 12]; returns (x, info dict)."""
        b = _as_c128(b)
        if b.ndim == 2:
            b = b[None]
        x = np.empty_like(b)
        info = self.solve_params(**kw)
        rc = _load().crk_mg_solve(self.handle, _cptr(b), _cptr(x), b.shape[0], C.byref(info))
        if rc != OK and (rc != ENOCONV or raise_on_noconv):
            _check(rc)
        d = info.as_dict()
        d["converged"] = rc == OK
        d["rhs"] = self.last_solve_rhs(b.shape[0])
        return x, d

    def solve_dev(self, b_dev, x_dev, nrhs, stream=None, raise_on_noconv=True, **kw):
        """Device solve on complex128 host-layout tensors [nrhs, V, 12] (as float64 views)."""
        info = self.solve_params(**kw)
        rc = _load().crk_mg_solve_dev(self.handle, _tptr(b_dev), _tptr(x_dev), int(nrhs), _stream(stream),
                                      C.byref(info))
        if rc != OK and (rc != ENOCONV or raise_on_noconv):
            _check(rc)
        d = info.as_dict()
        d["converged"] = rc == OK
        d["rhs"] = self.last_solve_rhs(int(nrhs))
        return d

    def last_solve_rhs(self, nrhs):
        it = (C.c_int32 * nrhs)()
        rr = (C.c_double * nrhs)()
        ts = (C.c_double * nrhs)()
        _check(_load().crk_mg_last_solve_rhs(self.handle, it, rr, nrhs))
        _check(_load().crk_mg_last_solve_rhs_seconds(self.handle, ts, nrhs))
        return {"iters": list(it), "true_rel_resid": list(rr), "seconds": list(ts)}

    def footprint_bytes(self, nrhs, form=FORM_FP32):
        return int(_load().crk_mg_footprint_bytes(self.handle, int(nrhs), int(form)))


class Server:
    """Continuously batched solve server over resident hierarchies (see crk.h).

    ``submit`` returns at once; the library's lane threads run the solves.  The
    host arrays of a request are kept alive here until ``wait`` returns.
    """

    def __init__(self, hbm_budget_bytes=0, slots_per_lane=12, max_lanes=4, idle_ms=200, **solve):
        p = ServerParams()
        _load().crk_server_params_default(C.byref(p))
        p.hbm_budget_bytes = int(hbm_budget_bytes)
        p.slots_per_lane = int(slots_per_lane)
        p.max_lanes = int(max_lanes)
        p.idle_ms = int(idle_ms)
        for k_, v_ in solve.items():
            if k_ == "form" and isinstance(v_, str):
                v_ = FORMS[v_]
            setattr(p.solve, k_, v_)
        h = C.c_void_p()
        _check(_load().crk_server_create(C.byref(p), C.byref(h)))
        self._h = h
        self._held = {}
        self._volumes = []

    @property
    def handle(self):
        if self._h is None:
            raise CrkError(EINVAL, "server is closed")
        return self._h

    def add(self, hierarchy):
        lid = C.c_int32()
        _check(_load().crk_server_add(self.handle, hierarchy.handle, C.byref(lid)))
        self._volumes.append(hierarchy.volume(0))
        return lid.value

    def submit(self, lattice, b):
        """Queue b (complex128 [nrhs, V, 12]); returns the request id."""
        b = _as_c128(b)
        if b.ndim == 2:
            b = b[None]
        if b.shape[1:] != (self._volumes[lattice], 12):
            raise CrkError(EINVAL, f"b has shape {b.shape}, lattice {lattice} needs [nrhs, {self._volumes[lattice]}, 12]")
        x = np.zeros_like(b)
        rid = C.c_uint64()
        _check(_load().crk_server_submit(self.handle, int(lattice), _cptr(b), _cptr(x), b.shape[0], C.byref(rid)))
        self._held[rid.value] = (b, x)
        return rid.value

    def wait(self, rid, timeout=-1.0, raise_on_noconv=True):
        """Block until request rid is done; returns (x, info dict).  None on timeout."""
        info = RequestInfo()
        rc = _load().crk_server_wait(self.handle, C.c_uint64(rid), float(timeout), C.byref(info))
        if rc == EBUSY:
            return None
        b, x = self._held.pop(rid)
        if rc != OK and (rc != ENOCONV or raise_on_noconv):
            _check(rc)
        d = info.as_dict()
        d["converged"] = rc == OK
        return x, d

    def lane_bytes(self, lattice):
        v = int(_load().crk_server_lane_bytes(self.handle, int(lattice)))
        if v < 0:
            _check(v)
        return v

    def stats(self):
        s = ServerStats()
        _check(_load().crk_server_get_stats(self.handle, C.byref(s)))
        return s.as_dict()

    def close(self):
        if self._h is not None:
            _load().crk_server_destroy(self._h)
            self._h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
