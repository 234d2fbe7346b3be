"""ctypes binding of libxc_mi355x.so, one Python function per C entry point
of include/xc.h (argument marshalling only: every step runs in the HIP
kernels of the library). PyTorch, when used, only provides device memory and
the stream.

The library must have been built (paper_2007_03143_amd/build.py); importing
this module without it raises ImportError.
"""
import ctypes
import os
from ctypes import (POINTER, Structure, byref, c_char_p, c_double, c_int,
                    c_longlong, c_size_t, c_ubyte, c_void_p)

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib",
                        "libxc_mi355x.so")

XC_OK = 0
XC_ERR_INVALID_ARG = -1
XC_ERR_UNSUPPORTED = -2
XC_ERR_NOMEM = -3
XC_ERR_DEVICE = -4
XC_ERR_STATE = -5
XC_ERR_BUSY = -6

XC_LDA_SVWN5 = 1
XC_GGA_PBE = 2
XC_MGGA_TPSS = 3
XC_FP64 = 0
XC_MIXED_FP32 = 1
XC_MIXED_BF16 = 2
XC_MIXED_FP32_V = 3

XC_PARTITION_SSF = 0
XC_PARTITION_BECKE = 1
PARTITIONS = {"ssf": XC_PARTITION_SSF, "becke": XC_PARTITION_BECKE}

FUNCTIONALS = {"lda": XC_LDA_SVWN5, "svwn5": XC_LDA_SVWN5, "pbe": XC_GGA_PBE,
               "tpss": XC_MGGA_TPSS}
PRECISIONS = {"fp64": XC_FP64, "fp32": XC_MIXED_FP32, "bf16": XC_MIXED_BF16,
              "fp32v": XC_MIXED_FP32_V}


class XcMolecule(Structure):
    _fields_ = [("natoms", c_int), ("xyz", POINTER(c_double)),
                ("mk_alpha", POINTER(c_double))]


class XcBasis(Structure):
    _fields_ = [("nshells", c_int), ("shell_atom", POINTER(c_int)),
                ("shell_L", POINTER(c_int)), ("shell_nprim", POINTER(c_int)),
                ("prim_alpha", POINTER(c_double)), ("prim_coef", POINTER(c_double)),
                ("shell_pure", POINTER(c_int))]


class XcGridSpec(Structure):
    _fields_ = [("n_rad", c_int), ("n_ang", c_int), ("ang_xyzw", POINTER(c_double)),
                ("ssf_a", c_double), ("screen_eta", c_double), ("batch_max", c_int),
                ("rho_thresh", c_double), ("atom_mask", POINTER(c_ubyte)),
                ("batch_merge", c_int), ("partition", c_int),
                ("becke_radius", POINTER(c_double))]


# device allocator callbacks: void* alloc(size_t bytes, void* user) and
# void free(void* ptr, void* user)
XC_ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_size_t, c_void_p)
XC_FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)


class XcDeviceOpts(Structure):
    _fields_ = [("stream", c_void_p), ("wave_bytes", c_size_t), ("alloc", XC_ALLOC_FN),
                ("free", XC_FREE_FN), ("alloc_user", c_void_p)]


class XcStats(Structure):
    _fields_ = [("n_points_nominal", c_longlong), ("n_points", c_longlong),
                ("n_batches", c_longlong), ("n_shell_entries", c_longlong),
                ("n_func_entries", c_longlong), ("max_nb", c_int), ("max_ng", c_int),
                ("sum_nb_ng", c_double), ("sum_nb2_ng", c_double),
                ("flops_contract", c_double), ("n_waves", c_int), ("built", c_int),
                ("persistent_bytes", c_size_t), ("wave_bytes", c_size_t),
                ("n_wide_waves", c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


PHASES = ["grid", "weights", "compact", "batch", "screen", "colloc", "density",
          "functional", "potential", "other"]


class XcTiming(Structure):
    _fields_ = [("ms", c_double * 10), ("launches", c_longlong * 10)]

    def as_dict(self):
        return {p: {"ms": self.ms[i], "launches": self.launches[i]}
                for i, p in enumerate(PHASES)}


class XcEngineOpts(Structure):
    _fields_ = [("stream", c_void_p), ("hbm_budget", c_size_t), ("wave_bytes", c_size_t),
                ("cache_phi", c_int)]


class XcEngineInfo(Structure):
    _fields_ = [("waiting", c_int), ("admitted", c_int), ("in_flight", c_int),
                ("bytes_used", c_size_t), ("budget", c_size_t), ("wave_bytes", c_size_t),
                ("steps", c_longlong), ("batches_launched", c_longlong),
                ("completed", c_longlong), ("colloc_batches", c_longlong),
                ("phi_cached", c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class XcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def _load():
    # PyTorch-ROCm carries its own HIP runtime (same soname as the system
    # one). Loading torch first makes this library bind to that runtime, so
    # the process holds one HIP runtime whichever module a caller imports
    # first; two runtimes in one process do not see the same devices.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "paper_2007_03143_amd/build.py (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.xc_strerror.restype = c_char_p
    lib.xc_strerror.argtypes = [c_int]
    lib.xc_last_error.restype = c_char_p
    lib.xc_last_error.argtypes = []
    lib.xc_abi_version.restype = c_int
    lib.xc_integrate.restype = c_int
    lib.xc_integrate.argtypes = [POINTER(XcMolecule), POINTER(XcBasis),
                                 POINTER(XcGridSpec), c_int, c_int,
                                 POINTER(c_double), c_int, POINTER(c_double),
                                 POINTER(c_double), POINTER(c_double)]
    lib.xc_context_create.restype = c_int
    lib.xc_context_create.argtypes = [POINTER(XcMolecule), POINTER(XcBasis),
                                      POINTER(XcGridSpec), POINTER(XcDeviceOpts),
                                      POINTER(c_void_p)]
    lib.xc_context_build_grid.restype = c_int
    lib.xc_context_build_grid.argtypes = [c_void_p]
    lib.xc_context_integrate.restype = c_int
    lib.xc_context_integrate.argtypes = [c_void_p, c_int, c_int, c_void_p, c_void_p,
                                         c_void_p]
    lib.xc_context_integrate_uks.restype = c_int
    lib.xc_context_integrate_uks.argtypes = [c_void_p, c_int, c_int, c_void_p, c_void_p,
                                             c_void_p, c_void_p, c_void_p]
    lib.xc_context_integrate_noalloc.restype = c_int
    lib.xc_context_integrate_noalloc.argtypes = [c_void_p, c_int, c_int, c_void_p,
                                                 c_void_p, c_void_p]
    lib.xc_context_stats.restype = c_int
    lib.xc_context_stats.argtypes = [c_void_p, POINTER(XcStats)]
    lib.xc_context_export_grid.restype = c_int
    lib.xc_context_export_grid.argtypes = [c_void_p, POINTER(c_double),
                                           POINTER(c_longlong)]
    lib.xc_context_export_batches.restype = c_int
    lib.xc_context_export_batches.argtypes = [c_void_p, POINTER(c_longlong),
                                              POINTER(c_double), POINTER(c_longlong),
                                              POINTER(c_int)]
    lib.xc_context_set_timing.restype = c_int
    lib.xc_context_set_timing.argtypes = [c_void_p, c_int]
    lib.xc_context_set_phi_cache.restype = c_int
    lib.xc_context_set_phi_cache.argtypes = [c_void_p, c_int]
    lib.xc_context_footprint.restype = c_int
    lib.xc_context_footprint.argtypes = [c_void_p, POINTER(c_size_t), POINTER(c_size_t)]
    lib.xc_context_timing.restype = c_int
    lib.xc_context_timing.argtypes = [c_void_p, POINTER(XcTiming)]
    lib.xc_context_destroy.restype = c_int
    lib.xc_context_destroy.argtypes = [c_void_p]
    lib.xc_engine_create.restype = c_int
    lib.xc_engine_create.argtypes = [POINTER(XcEngineOpts), POINTER(c_void_p)]
    lib.xc_engine_add_request.restype = c_int
    lib.xc_engine_add_request.argtypes = [c_void_p, POINTER(XcMolecule), POINTER(XcBasis),
                                          POINTER(XcGridSpec), c_int, c_int,
                                          POINTER(c_longlong)]
    lib.xc_engine_submit.restype = c_int
    lib.xc_engine_submit.argtypes = [c_void_p, c_longlong, c_void_p, c_void_p, c_void_p,
                                     POINTER(c_longlong)]
    lib.xc_engine_step.restype = c_int
    lib.xc_engine_step.argtypes = [c_void_p, POINTER(c_int)]
    lib.xc_engine_poll.restype = c_int
    lib.xc_engine_poll.argtypes = [c_void_p, c_longlong, POINTER(c_int)]
    lib.xc_engine_release.restype = c_int
    lib.xc_engine_release.argtypes = [c_void_p, c_longlong]
    lib.xc_engine_stats.restype = c_int
    lib.xc_engine_stats.argtypes = [c_void_p, POINTER(XcEngineInfo)]
    lib.xc_engine_destroy.restype = c_int
    lib.xc_engine_destroy.argtypes = [c_void_p]
    return lib


LIB = _load()


def _check(code):
    if code != XC_OK:
        raise XcError(code, LIB.xc_last_error().decode() or
                      LIB.xc_strerror(code).decode())


def _dptr(a):
    return a.ctypes.data_as(POINTER(c_double))


def _iptr(a):
    return a.ctypes.data_as(POINTER(c_int))


class _Inputs:
    """Keeps the numpy arrays behind the C structs alive."""

    def __init__(self, coords, mk_alpha, basis, grid):
        self.xyz = np.ascontiguousarray(coords, dtype=np.float64).reshape(-1, 3)
        self.alpha = np.ascontiguousarray(mk_alpha, dtype=np.float64)
        self.sa = np.ascontiguousarray(basis.shell_atom, dtype=np.int32)
        self.sl = np.ascontiguousarray(basis.shell_L, dtype=np.int32)
        self.sn = np.ascontiguousarray(basis.shell_nprim, dtype=np.int32)
        self.pa = np.ascontiguousarray(basis.prim_alpha, dtype=np.float64)
        self.pc = np.ascontiguousarray(basis.prim_coef, dtype=np.float64)
        sp = getattr(basis, "shell_pure", None)
        self.sp = None if sp is None else np.ascontiguousarray(sp, dtype=np.int32)
        self.ang = np.ascontiguousarray(grid["ang"], dtype=np.float64)
        m = grid.get("atom_mask")
        self.mask = None if m is None else np.ascontiguousarray(m, dtype=np.uint8)
        br = grid.get("becke_radius")
        self.brad = None if br is None else np.ascontiguousarray(br, dtype=np.float64)
        part = grid.get("partition", "ssf")
        part = PARTITIONS[part] if isinstance(part, str) else int(part)
        self.mol = XcMolecule(self.xyz.shape[0], _dptr(self.xyz), _dptr(self.alpha))
        self.basis = XcBasis(self.sa.shape[0], _iptr(self.sa), _iptr(self.sl),
                             _iptr(self.sn), _dptr(self.pa), _dptr(self.pc),
                             None if self.sp is None else _iptr(self.sp))
        self.grid = XcGridSpec(
            int(grid["n_rad"]), int(grid["n_ang"]), _dptr(self.ang),
            float(grid.get("ssf_a", 0.64)), float(grid.get("screen_eta", 1e-10)),
            int(grid.get("batch_max", 512)), float(grid.get("rho_thresh", 1e-15)),
            None if self.mask is None else self.mask.ctypes.data_as(POINTER(c_ubyte)),
            int(grid.get("batch_merge", 1)), part,
            None if self.brad is None else _dptr(self.brad))
        self.nbf = int(sum(2 * L + 1 if (self.sp is not None and self.sp[s] and L >= 2)
                           else (L + 1) * (L + 2) // 2 for s, L in enumerate(self.sl)))


def _code(table, v):
    return table[v] if isinstance(v, str) else int(v)


def xc_abi_version():
    return LIB.xc_abi_version()


def xc_strerror(code):
    return LIB.xc_strerror(code).decode()


def xc_integrate(coords, mk_alpha, basis, grid, functional, P, precision="fp64"):
    """One-shot integration with host arrays; returns (E_xc, N_e, V)."""
    inp = _Inputs(coords, mk_alpha, basis, grid)
    P = np.ascontiguousarray(P, dtype=np.float64)
    nbf = P.shape[0]
    V = np.empty((nbf, nbf))
    E = c_double()
    N = c_double()
    _check(LIB.xc_integrate(byref(inp.mol), byref(inp.basis), byref(inp.grid),
                            _code(FUNCTIONALS, functional), _code(PRECISIONS, precision),
                            _dptr(P), nbf, byref(E), byref(N), _dptr(V)))
    return E.value, N.value, V


def xc_context_create(coords, mk_alpha, basis, grid, stream=0, wave_bytes=0, alloc=None,
                      free=None):
    """alloc, free: XC_ALLOC_FN and XC_FREE_FN callback objects (the caller
    keeps them alive as long as the context), or None for hipMalloc."""
    inp = _Inputs(coords, mk_alpha, basis, grid)
    opts = XcDeviceOpts(c_void_p(int(stream)), int(wave_bytes))
    if alloc is not None:
        opts.alloc = alloc
    if free is not None:
        opts.free = free
    h = c_void_p()
    _check(LIB.xc_context_create(byref(inp.mol), byref(inp.basis), byref(inp.grid),
                                 byref(opts), byref(h)))
    return h, inp.nbf


def xc_context_build_grid(handle):
    _check(LIB.xc_context_build_grid(handle))


def xc_context_integrate(handle, functional, precision, d_P, d_V, d_EN):
    """Device pointers (ints); ordered on the context's stream."""
    _check(LIB.xc_context_integrate(handle, _code(FUNCTIONALS, functional),
                                    _code(PRECISIONS, precision), c_void_p(d_P),
                                    c_void_p(d_V), c_void_p(d_EN)))


def xc_context_integrate_uks(handle, functional, precision, d_Pa, d_Pb, d_Va, d_Vb, d_EN):
    """Spin-unrestricted integration; device pointers (ints)."""
    _check(LIB.xc_context_integrate_uks(handle, _code(FUNCTIONALS, functional),
                                        _code(PRECISIONS, precision), c_void_p(d_Pa),
                                        c_void_p(d_Pb), c_void_p(d_Va), c_void_p(d_Vb),
                                        c_void_p(d_EN)))


def xc_context_integrate_noalloc(handle, functional, precision, d_P, d_V, d_EN):
    """xc_context_integrate with the scratch in the library's static device
    array (no allocation); device pointers (ints)."""
    _check(LIB.xc_context_integrate_noalloc(handle, _code(FUNCTIONALS, functional),
                                            _code(PRECISIONS, precision), c_void_p(d_P),
                                            c_void_p(d_V), c_void_p(d_EN)))


STATIC_SCRATCH_BYTES = 64 << 20


def xc_context_stats(handle):
    s = XcStats()
    _check(LIB.xc_context_stats(handle, byref(s)))
    return s.as_dict()


def xc_context_export_grid(handle):
    st = xc_context_stats(handle)
    n = st["n_points"]
    xyzw = np.empty((n, 4))
    idx = np.empty(n, dtype=np.int64)
    _check(LIB.xc_context_export_grid(handle, _dptr(xyzw),
                                      idx.ctypes.data_as(POINTER(c_longlong))))
    return xyzw, idx


def xc_context_export_batches(handle):
    st = xc_context_stats(handle)
    nb = st["n_batches"]
    pp = np.empty(nb + 1, dtype=np.int64)
    bb = np.empty((nb, 6))
    sp = np.empty(nb + 1, dtype=np.int64)
    sh = np.empty(max(1, st["n_shell_entries"]), dtype=np.int32)
    _check(LIB.xc_context_export_batches(
        handle, pp.ctypes.data_as(POINTER(c_longlong)), _dptr(bb),
        sp.ctypes.data_as(POINTER(c_longlong)), _iptr(sh)))
    return pp, bb, sp, sh[:st["n_shell_entries"]]


def xc_context_set_timing(handle, enable):
    _check(LIB.xc_context_set_timing(handle, 1 if enable else 0))


def xc_context_set_phi_cache(handle, enable):
    _check(LIB.xc_context_set_phi_cache(handle, 1 if enable else 0))


def xc_context_footprint(handle):
    """(min_bytes, cached_bytes) of the context's integrations."""
    mn, al = c_size_t(), c_size_t()
    _check(LIB.xc_context_footprint(handle, byref(mn), byref(al)))
    return mn.value, al.value


def xc_context_timing(handle):
    t = XcTiming()
    _check(LIB.xc_context_timing(handle, byref(t)))
    return t.as_dict()


def xc_context_destroy(handle):
    _check(LIB.xc_context_destroy(handle))


def xc_engine_create(stream=0, hbm_budget=0, wave_bytes=0, cache_phi=True):
    h = c_void_p()
    opts = XcEngineOpts(c_void_p(int(stream)), int(hbm_budget), int(wave_bytes),
                        1 if cache_phi else 0)
    _check(LIB.xc_engine_create(byref(opts), byref(h)))
    return h


def xc_engine_add_request(handle, coords, mk_alpha, basis, grid, functional,
                          precision="fp64"):
    inp = _Inputs(coords, mk_alpha, basis, grid)
    rid = c_longlong()
    _check(LIB.xc_engine_add_request(handle, byref(inp.mol), byref(inp.basis),
                                     byref(inp.grid), _code(FUNCTIONALS, functional),
                                     _code(PRECISIONS, precision), byref(rid)))
    return rid.value, inp.nbf


def xc_engine_submit(handle, req_id, d_P, d_V, d_EN):
    t = c_longlong()
    _check(LIB.xc_engine_submit(handle, req_id, c_void_p(d_P), c_void_p(d_V),
                                c_void_p(d_EN), byref(t)))
    return t.value


def xc_engine_step(handle):
    n = c_int()
    _check(LIB.xc_engine_step(handle, byref(n)))
    return n.value


def xc_engine_poll(handle, ticket):
    d = c_int()
    _check(LIB.xc_engine_poll(handle, ticket, byref(d)))
    return bool(d.value)


def xc_engine_release(handle, req_id):
    _check(LIB.xc_engine_release(handle, req_id))


def xc_engine_stats(handle):
    s = XcEngineInfo()
    _check(LIB.xc_engine_stats(handle, byref(s)))
    return s.as_dict()


def xc_engine_destroy(handle):
    _check(LIB.xc_engine_destroy(handle))


class XcContext:
    """A device context whose P, V and E/N buffers are torch tensors on the
    current device, with launches ordered on torch's current stream."""

    def __init__(self, coords, mk_alpha, basis, grid, wave_bytes=0, stream=None,
                 allocator=None):
        """allocator: None (the library's hipMalloc), "torch" (torch's caching
        allocator on the context's stream) or a pair (alloc, free) of Python
        callables, alloc(nbytes) -> device address (0 on failure) and
        free(address)."""
        import torch
        self.torch = torch
        self.handle = None
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._alloc_cb = self._free_cb = None
        if allocator is not None:
            if allocator == "torch":
                dev, st = torch.cuda.current_device(), self.stream

                def py_alloc(n):
                    return torch.cuda.caching_allocator_alloc(n, dev, st)

                py_free = torch.cuda.caching_allocator_delete
            else:
                py_alloc, py_free = allocator

            def c_alloc(n, _user):
                try:
                    return int(py_alloc(int(n))) or None
                except Exception:
                    return None

            def c_free(p, _user):
                py_free(int(p))

            self._alloc_cb, self._free_cb = XC_ALLOC_FN(c_alloc), XC_FREE_FN(c_free)
        self.handle, self.nbf = xc_context_create(coords, mk_alpha, basis, grid,
                                                  self.stream.cuda_stream, wave_bytes,
                                                  self._alloc_cb, self._free_cb)
        self.V = torch.empty((self.nbf, self.nbf), dtype=torch.float64, device="cuda")
        self.EN = torch.empty(2, dtype=torch.float64, device="cuda")

    def build_grid(self):
        xc_context_build_grid(self.handle)

    def integrate(self, P, functional, precision="fp64"):
        """P: (nbf, nbf) float64 cuda tensor. Returns (V, EN) device tensors,
        valid once the stream has reached this point."""
        assert P.dtype == self.torch.float64 and P.is_cuda and P.is_contiguous()
        assert tuple(P.shape) == (self.nbf, self.nbf)
        xc_context_integrate(self.handle, functional, precision, P.data_ptr(),
                             self.V.data_ptr(), self.EN.data_ptr())
        return self.V, self.EN

    def integrate_uks(self, Pa, Pb, functional, precision="fp64"):
        """Spin-unrestricted: Pa, Pb (nbf, nbf) float64 cuda tensors. Returns
        (Va, Vb, EN) device tensors, valid once the stream reaches here."""
        for P in (Pa, Pb):
            assert P.dtype == self.torch.float64 and P.is_cuda and P.is_contiguous()
            assert tuple(P.shape) == (self.nbf, self.nbf)
        if not hasattr(self, "Vb"):
            self.Vb = self.torch.empty_like(self.V)
        xc_context_integrate_uks(self.handle, functional, precision, Pa.data_ptr(),
                                 Pb.data_ptr(), self.V.data_ptr(), self.Vb.data_ptr(),
                                 self.EN.data_ptr())
        return self.V, self.Vb, self.EN

    def stats(self):
        return xc_context_stats(self.handle)

    def export_grid(self):
        return xc_context_export_grid(self.handle)

    def set_timing(self, enable):
        xc_context_set_timing(self.handle, enable)

    def set_phi_cache(self, enable):
        xc_context_set_phi_cache(self.handle, enable)

    def footprint(self):
        return xc_context_footprint(self.handle)

    def timing(self):
        return xc_context_timing(self.handle)

    def export_batches(self):
        return xc_context_export_batches(self.handle)

    def close(self):
        if self.handle is not None:
            xc_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
