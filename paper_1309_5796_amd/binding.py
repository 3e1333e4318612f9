"""ctypes binding of libmmsd.so (argument marshalling only).

Every computation runs in the HIP library; this module converts NumPy arrays
to the C structs of ``include/mmsd.h`` and back.  PyTorch, when present, only
supplies device memory (through the allocator hooks) and the stream.

Loading fails loudly when the library is not built or no GPU is visible;
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmmsd.so")

OK, W_MAXEVALS, W_FLOOR = 0, 1, 2
E_INVALID, E_MESH, E_NOMEM, E_HIP, E_NONFINITE, E_BUSY, E_CANCELLED = -1, -2, -3, -4, -5, -6, -7
FP64, MIXED = 0, 1
EXCH, ANIS, ZEEM, DEMAG, ALL = 1, 2, 4, 8, 15
STEP_ADAPTIVE, STEP_ALTERNATE, STEP_BB1, STEP_BB2 = 0, 1, 2, 3
STOP_MAX_TORQUE, STOP_SUM_SQ = 0, 1
PRECOND_AUTO, PRECOND_JACOBI, PRECOND_AMG = 0, 1, 2
VC_FUSE_REST, VC_FOLD_SOLVE, VC_SLICE_ALL = 1, 2, 4
ASSEMBLE_HOST, ASSEMBLE_DEVICE = 0, 1

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class MeshC(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("xyz", C.POINTER(C.c_double)),
                ("n_tets", C.c_int64), ("tets", C.POINTER(C.c_int32)),
                ("tet_region", C.POINTER(C.c_int32)), ("dirichlet", C.POINTER(C.c_uint8)),
                ("shell", C.POINTER(C.c_double))]


class MaterialC(C.Structure):
    _fields_ = [("region", C.c_int32), ("Js_T", C.c_double), ("K1_Jm3", C.c_double),
                ("A_Jm", C.c_double), ("easy_axis", C.c_double * 3)]


class OptionsC(C.Structure):
    _fields_ = [("tol_torque", C.c_double), ("max_evals", C.c_int64), ("terms", C.c_int),
                ("nonmono_M", C.c_int), ("pcg_rtol", C.c_double), ("pcg_maxit", C.c_int),
                ("step_rule", C.c_int), ("refine_tol_T", C.c_double), ("precond", C.c_int),
                ("stop_rule", C.c_int)]


class ResultC(C.Structure):
    _fields_ = [("status", C.c_int), ("energy_J", C.c_double), ("e_exch_J", C.c_double),
                ("e_anis_J", C.c_double), ("e_zeem_J", C.c_double), ("e_demag_J", C.c_double),
                ("max_torque", C.c_double), ("sum_V_torque2", C.c_double), ("sum_torque2", C.c_double),
                ("m_avg", C.c_double * 3), ("iterations", C.c_int64), ("evals", C.c_int64),
                ("pcg_iters", C.c_int64), ("launches", C.c_int64), ("seconds", C.c_double)]


# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("mmsd_ctx_create", C.c_int, [C.c_int, C.c_void_p, ALLOC_FN, FREE_FN, C.c_void_p, C.POINTER(C.c_void_p)]),
    ("mmsd_ctx_destroy", C.c_int, [C.c_void_p]),
    ("mmsd_footprint", C.c_int, [C.POINTER(MeshC), C.c_int, C.POINTER(C.c_size_t)]),
    ("mmsd_set_vcycle", C.c_int, [C.c_void_p, C.c_int]),
    ("mmsd_set_assembly", C.c_int, [C.c_void_p, C.c_int]),
    ("mmsd_problem_create", C.c_int, [C.c_void_p, C.POINTER(MeshC), C.POINTER(MaterialC), C.c_int, C.c_int,
                                      C.POINTER(C.c_void_p)]),
    ("mmsd_problem_destroy", C.c_int, [C.c_void_p]),
    ("mmsd_problem_setup_times", C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    ("mmsd_n_magnetic", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("mmsd_n_potential", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("mmsd_problem_sizes", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("mmsd_set_material", C.c_int, [C.c_void_p, C.POINTER(MaterialC)]),
    ("mmsd_set_field", C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    ("mmsd_set_m", C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    ("mmsd_get_m", C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    ("mmsd_options_default", None, [C.POINTER(OptionsC)]),
    ("mmsd_minimize", C.c_int, [C.c_void_p, C.POINTER(OptionsC), C.POINTER(ResultC)]),
    ("mmsd_evaluate", C.c_int, [C.c_void_p, C.POINTER(OptionsC), C.POINTER(ResultC)]),
    ("mmsd_get_field", C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    ("mmsd_get_potential", C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    ("mmsd_hysteresis", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int64, C.POINTER(OptionsC),
                                  C.POINTER(ResultC), C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    ("mmsd_minimize_batch", C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(OptionsC), C.POINTER(ResultC)]),
    ("mmsd_get_state", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t)]),
    ("mmsd_set_state", C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    ("mmsd_timing_enable", C.c_int, [C.c_void_p, C.c_int]),
    ("mmsd_timing_read", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int]),
    ("mmsd_set_launch_config", C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    ("mmsd_copy_probe", C.c_int, [C.c_void_p, C.c_size_t, C.c_int, C.POINTER(C.c_double)]),
    ("mmsd_set_problem_launch", C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    ("mmsd_autotune", C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    ("mmsd_autotune_cache_get", C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
    ("mmsd_autotune_cache_put", C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    ("mmsd_assembly_export", C.c_int, [C.POINTER(MeshC), C.POINTER(MaterialC), C.c_int, C.POINTER(C.c_int64)]
     + [C.c_void_p] * 12),
    ("mmsd_assemble_device", C.c_int, [C.c_void_p, C.POINTER(MeshC), C.POINTER(MaterialC), C.c_int,
                                       C.POINTER(C.c_int64)] + [C.c_void_p] * 11),
    ("mmsd_assemble_device_noalloc", C.c_int, [C.c_void_p, C.POINTER(MeshC), C.POINTER(MaterialC), C.c_int,
                                               C.POINTER(C.c_int64)] + [C.c_void_p] * 11),
    ("mmsd_server_create", C.c_int, [C.c_void_p, C.c_size_t, C.c_int, C.POINTER(C.c_void_p)]),
    ("mmsd_submit", C.c_int, [C.c_void_p, C.POINTER(MeshC), C.POINTER(MaterialC), C.c_int, C.POINTER(C.c_double),
                              C.c_int, C.POINTER(C.c_double), C.POINTER(OptionsC), C.POINTER(C.c_uint64)]),
    ("mmsd_poll", C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(ResultC), C.POINTER(C.c_double)]),
    ("mmsd_cancel", C.c_int, [C.c_void_p, C.c_uint64]),
    ("mmsd_server_stats", C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    ("mmsd_server_destroy", C.c_int, [C.c_void_p]),
    ("mmsd_last_error", C.c_char_p, []),
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmmsd.so and declare its entry points (no device is touched)."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime and links it as libamdhip64.so;
        # loading torch first lets this library's libamdhip64.so.7 dependency
        # bind to that same runtime instead of starting a second one.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built: run `python -m paper_1309_5796_amd.build`")
        lib = C.CDLL(path)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class MMSDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mmsd error {code}: {msg}")
        self.code = code


def _check(rc: int) -> int:
    if rc < 0:
        raise MMSDError(rc, load_library().mmsd_last_error().decode())
    return rc


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class Result:
    status: int
    energy_J: float
    e_exch_J: float
    e_anis_J: float
    e_zeem_J: float
    e_demag_J: float
    max_torque: float
    sum_V_torque2: float
    sum_torque2: float
    m_avg: np.ndarray
    iterations: int
    evals: int
    pcg_iters: int
    launches: int
    seconds: float

    @staticmethod
    def from_c(r: ResultC) -> "Result":
        return Result(r.status, r.energy_J, r.e_exch_J, r.e_anis_J, r.e_zeem_J, r.e_demag_J,
                      r.max_torque, r.sum_V_torque2, r.sum_torque2, np.array(r.m_avg[:]),
                      r.iterations, r.evals, r.pcg_iters, r.launches, r.seconds)


def make_options(tol: float = 0.0, max_evals: int = 0, terms: int = 0, nonmono_M: int = 0,
                 pcg_rtol: float = 0.0, pcg_maxit: int = 0, step_rule: int = 0,
                 refine_tol_T: float = 0.0, precond: int = 0, stop_rule: int = 0) -> OptionsC:
    """Options struct; zero fields select the library defaults."""
    return OptionsC(tol, max_evals, terms, nonmono_M, pcg_rtol, pcg_maxit, step_rule, refine_tol_T, precond,
                    stop_rule)


class _TorchAllocator:
    """Device memory from PyTorch's caching allocator, handed to the library."""

    def __init__(self, device: int):
        import torch
        self.torch = torch
        self.device = device
        self.live = {}
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=f"cuda:{self.device}")
        except Exception:
            return None
        ptr = t.data_ptr()
        self.live[ptr] = t
        return ptr

    def _free(self, ptr, user):
        self.live.pop(ptr, None)


class Context:
    """A device, a stream and an allocator.  With torch=True (default when
    PyTorch sees a GPU) memory comes from torch and work goes on torch's
    current stream."""

    def __init__(self, device: int = 0, torch: Optional[bool] = None):
        lib = load_library()
        self._alloc = None
        stream = None
        if torch is None:
            try:
                import torch as _t
                torch = bool(_t.cuda.is_available())
            except Exception:
                torch = False
        if torch:
            import torch as _t
            self._alloc = _TorchAllocator(device)
            s = _t.cuda.current_stream(device).cuda_stream
            stream = C.c_void_p(s) if s else None
        h = C.c_void_p()
        if self._alloc:
            rc = lib.mmsd_ctx_create(device, stream, self._alloc.alloc_cb, self._alloc.free_cb, None, C.byref(h))
        else:
            rc = lib.mmsd_ctx_create(device, stream, ALLOC_FN(), FREE_FN(), None, C.byref(h))
        _check(rc)
        self.handle = h
        self.lib = lib
        self.device = device
        self._children = weakref.WeakSet()   # problems and servers to close first

    def set_launch_config(self, lanes_per_row: int = 0, max_blocks: int = 0):
        _check(self.lib.mmsd_set_launch_config(self.handle, lanes_per_row, max_blocks))

    def set_vcycle(self, flags: int):
        """V-cycle forms for problems created afterwards (VC_FUSE_REST, VC_FOLD_SOLVE, VC_SLICE_ALL)."""
        _check(self.lib.mmsd_set_vcycle(self.handle, flags))

    def set_assembly(self, where: int):
        """Where problems created afterwards assemble their operators (ASSEMBLE_HOST, ASSEMBLE_DEVICE)."""
        _check(self.lib.mmsd_set_assembly(self.handle, where))

    def autotune_cache(self) -> np.ndarray:
        """The autotuner's cache as an (n, 5) int32 array of records
        {precision, log2(N + 1), log2(N_t + 1), lanes, blocks}."""
        n = C.c_int()
        _check(self.lib.mmsd_autotune_cache_get(self.handle, None, 0, C.byref(n)))
        rec = np.zeros((n.value, 5), np.int32)
        if n.value:
            _check(self.lib.mmsd_autotune_cache_get(self.handle, rec.ctypes.data, n.value, C.byref(n)))
        return rec

    def put_autotune_cache(self, records):
        """Add records (as returned by autotune_cache) to this context's cache."""
        rec = np.ascontiguousarray(np.asarray(records, np.int32).reshape(-1, 5))
        _check(self.lib.mmsd_autotune_cache_put(self.handle, rec.ctypes.data if len(rec) else None, len(rec)))

    def timing(self, on: bool):
        _check(self.lib.mmsd_timing_enable(self.handle, 1 if on else 0))

    def timing_read(self, reset: bool = True):
        s = (C.c_double * 3)()
        _check(self.lib.mmsd_timing_read(self.handle, s, 1 if reset else 0))
        return dict(ms=s[0], launches=int(s[1]), bytes=s[2])

    def copy_probe(self, nbytes: int, reps: int = 10) -> float:
        """Mean milliseconds of a plain copy kernel of nbytes (counter calibration)."""
        ms = C.c_double()
        _check(self.lib.mmsd_copy_probe(self.handle, nbytes, reps, C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "handle", None):
            for ch in list(self._children):
                ch.close()
            self.lib.mmsd_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MeshArgs:
    """Contiguous arrays of a mesh kept alive while the C struct points at them."""

    def __init__(self, mesh, materials=None):
        self.xyz = np.ascontiguousarray(mesh.xyz, dtype=np.float64)
        self.tets = np.ascontiguousarray(mesh.tets, dtype=np.int32)
        self.region = np.ascontiguousarray(mesh.region, dtype=np.int32)
        d = getattr(mesh, "dirichlet", None)
        self.dir = None if d is None else np.ascontiguousarray(d, dtype=np.uint8)
        sh = getattr(mesh, "shell", None)
        self.shell = None if sh is None else np.ascontiguousarray(sh, dtype=np.float64)
        self.c = MeshC(self.xyz.shape[0], _dp(self.xyz), self.tets.shape[0],
                       self.tets.ctypes.data_as(C.POINTER(C.c_int32)),
                       self.region.ctypes.data_as(C.POINTER(C.c_int32)),
                       None if self.dir is None else self.dir.ctypes.data_as(C.POINTER(C.c_uint8)),
                       None if self.shell is None else _dp(self.shell))
        mats = materials if materials is not None else mesh.materials
        self.mats = (MaterialC * max(1, len(mats)))()
        for k, m in enumerate(mats):
            self.mats[k] = material_c(m)
        self.n_mats = len(mats)


def material_c(m) -> MaterialC:
    ax = np.asarray(m.axis, float)
    return MaterialC(int(m.region), float(m.Js), float(m.K1), float(m.A), (C.c_double * 3)(*ax))


def footprint(mesh, precision: int = FP64) -> int:
    a = MeshArgs(mesh)
    out = C.c_size_t()
    _check(load_library().mmsd_footprint(C.byref(a.c), precision, C.byref(out)))
    return int(out.value)


class Problem:
    def __init__(self, ctx: Context, mesh, materials=None, precision: int = FP64):
        self.ctx = ctx
        self.lib = ctx.lib
        a = MeshArgs(mesh, materials)
        h = C.c_void_p()
        _check(self.lib.mmsd_problem_create(ctx.handle, C.byref(a.c), a.mats, a.n_mats, precision, C.byref(h)))
        self.handle = h
        ctx._children.add(self)
        self.precision = precision
        self.n_nodes = a.xyz.shape[0]
        n = C.c_int64()
        _check(self.lib.mmsd_n_magnetic(h, C.byref(n)))
        self.N = int(n.value)
        _check(self.lib.mmsd_n_potential(h, C.byref(n)))
        self.Nt = int(n.value)

    def setup_times(self) -> dict:
        """Seconds of this problem's creation by stage."""
        t = (C.c_double * 4)()
        _check(self.lib.mmsd_problem_setup_times(self.handle, t))
        return dict(assembly=t[0], multigrid=t[1], device_build=t[2], total=t[3])

    def sizes(self) -> dict:
        """N, magnet-pattern entries, N_t and potential-matrix entries."""
        a = (C.c_int64 * 4)()
        _check(self.lib.mmsd_problem_sizes(self.handle, a))
        return dict(N=int(a[0]), nnz_magnet=int(a[1]), Nt=int(a[2]), nnz_potential=int(a[3]))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.mmsd_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_material(self, m):
        mc = material_c(m)
        _check(self.lib.mmsd_set_material(self.handle, C.byref(mc)))

    def set_field(self, b):
        b = np.ascontiguousarray(b, dtype=np.float64)
        _check(self.lib.mmsd_set_field(self.handle, _dp(b)))

    def set_m(self, m):
        m = np.ascontiguousarray(m, dtype=np.float64).reshape(self.N, 3)
        _check(self.lib.mmsd_set_m(self.handle, _dp(m)))

    def get_m(self) -> np.ndarray:
        out = np.empty((self.N, 3))
        _check(self.lib.mmsd_get_m(self.handle, _dp(out)))
        return out

    def minimize(self, **opts) -> Result:
        o = make_options(**opts)
        r = ResultC()
        _check(self.lib.mmsd_minimize(self.handle, C.byref(o), C.byref(r)))
        return Result.from_c(r)

    def evaluate(self, **opts) -> Result:
        o = make_options(**opts)
        r = ResultC()
        _check(self.lib.mmsd_evaluate(self.handle, C.byref(o), C.byref(r)))
        return Result.from_c(r)

    def get_field(self) -> np.ndarray:
        out = np.empty((self.N, 3))
        _check(self.lib.mmsd_get_field(self.handle, _dp(out)))
        return out

    def get_potential(self) -> np.ndarray:
        out = np.empty(self.n_nodes)
        _check(self.lib.mmsd_get_potential(self.handle, _dp(out)))
        return out

    def hysteresis(self, fields, **opts):
        f = np.ascontiguousarray(fields, dtype=np.float64).reshape(-1, 3)
        n = f.shape[0]
        res = (ResultC * n)()
        bsw = np.zeros(n)
        nsw = C.c_int64()
        o = make_options(**opts)
        _check(self.lib.mmsd_hysteresis(self.handle, _dp(f), n, C.byref(o), res, _dp(bsw), C.byref(nsw)))
        return [Result.from_c(r) for r in res], bsw[: nsw.value].copy()

    def set_launch(self, lanes_per_row: int, max_blocks: int):
        _check(self.lib.mmsd_set_problem_launch(self.handle, lanes_per_row, max_blocks))

    def autotune(self):
        """Pick lanes per row and block cap by timing; returns (lanes, blocks, us)."""
        lanes, blocks, us = C.c_int(), C.c_int(), C.c_double()
        _check(self.lib.mmsd_autotune(self.handle, C.byref(lanes), C.byref(blocks), C.byref(us)))
        return lanes.value, blocks.value, us.value

    def get_state(self) -> bytes:
        n = C.c_size_t()
        _check(self.lib.mmsd_get_state(self.handle, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(self.lib.mmsd_get_state(self.handle, buf, C.byref(n)))
        return buf.raw[: n.value]

    def set_state(self, state: bytes):
        buf = C.create_string_buffer(state, len(state))
        _check(self.lib.mmsd_set_state(self.handle, buf, len(state)))


def assembly_export(mesh, materials=None) -> dict:
    """Host-side assembly of a mesh (no device): the library's operators in
    its internal units (see mmsd_assembly_export in include/mmsd.h)."""
    lib = load_library()
    a = MeshArgs(mesh, materials)
    sizes = (C.c_int64 * 4)()
    null = [None] * 12
    _check(lib.mmsd_assembly_export(C.byref(a.c), a.mats, a.n_mats, sizes, *null))
    N, nnzM, Nt, nnzL = (int(x) for x in sizes)
    out = dict(mrp=np.empty(N + 1, np.int32), mci=np.empty(nnzM, np.int32), K=np.empty(nnzM),
               D1=np.empty(3 * nnzM), D2=np.empty(3 * nnzM), Q=np.empty(6 * N), V=np.empty(N),
               pot_global=np.empty(Nt, np.int32), lrp=np.empty(Nt + 1, np.int32), lci=np.empty(nnzL, np.int32),
               L=np.empty(nnzL), scalars=np.empty(4))
    order = ["mrp", "mci", "K", "D1", "D2", "Q", "V", "pot_global", "lrp", "lci", "L", "scalars"]
    ptrs = [out[k].ctypes.data_as(C.c_void_p) for k in order]
    _check(lib.mmsd_assembly_export(C.byref(a.c), a.mats, a.n_mats, sizes, *ptrs))
    out["D1"] = out["D1"].reshape(3, nnzM)
    out["D2"] = out["D2"].reshape(3, nnzM)
    out["Q"] = out["Q"].reshape(6, N)
    out.update(N=N, Nt=Nt)
    return out


def assemble_device(ctx: Context, mesh, materials=None, no_alloc: bool = False) -> dict:
    """The same operators as assembly_export, assembled by the device
    kernels into torch tensors on ctx's device (no scalars).  no_alloc uses
    mmsd_assemble_device_noalloc (temporaries in the library's fixed region)."""
    import torch
    lib = ctx.lib
    fn = lib.mmsd_assemble_device_noalloc if no_alloc else lib.mmsd_assemble_device
    a = MeshArgs(mesh, materials)
    sizes = (C.c_int64 * 4)()
    _check(fn(ctx.handle, C.byref(a.c), a.mats, a.n_mats, sizes, *([None] * 11)))
    N, nnzM, Nt, nnzL = (int(x) for x in sizes)
    dev = torch.device("cuda", ctx.device)
    i32, f64 = torch.int32, torch.float64
    out = dict(mrp=torch.empty(N + 1, dtype=i32, device=dev), mci=torch.empty(nnzM, dtype=i32, device=dev),
               K=torch.empty(nnzM, dtype=f64, device=dev), D1=torch.empty(3, nnzM, dtype=f64, device=dev),
               D2=torch.empty(3, nnzM, dtype=f64, device=dev), Q=torch.empty(6, N, dtype=f64, device=dev),
               V=torch.empty(N, dtype=f64, device=dev), pot_global=torch.empty(Nt, dtype=i32, device=dev),
               lrp=torch.empty(Nt + 1, dtype=i32, device=dev), lci=torch.empty(nnzL, dtype=i32, device=dev),
               L=torch.empty(nnzL, dtype=f64, device=dev))
    order = ["mrp", "mci", "K", "D1", "D2", "Q", "V", "pot_global", "lrp", "lci", "L"]
    # an empty tensor has no storage: give the library a valid one-element stand-in
    keep = [out[k] if out[k].numel() else torch.empty(1, dtype=out[k].dtype, device=dev) for k in order]
    _check(fn(ctx.handle, C.byref(a.c), a.mats, a.n_mats, sizes, *[C.c_void_p(t.data_ptr()) for t in keep]))
    out.update(N=N, Nt=Nt)
    return out


def minimize_batch(problems: Sequence[Problem], **opts) -> List[Result]:
    n = len(problems)
    hs = (C.c_void_p * n)(*[p.handle.value for p in problems])
    res = (ResultC * n)()
    o = make_options(**opts)
    _check(load_library().mmsd_minimize_batch(hs, n, C.byref(o), res))
    return [Result.from_c(r) for r in res]


class Server:
    """Continuous-batching server: submit minimizations, poll results."""

    def __init__(self, ctx: Context, hbm_budget: int, max_slots: int = 64):
        self.ctx = ctx
        self.lib = ctx.lib
        h = C.c_void_p()
        _check(self.lib.mmsd_server_create(ctx.handle, hbm_budget, max_slots, C.byref(h)))
        self.handle = h
        ctx._children.add(self)

    def submit(self, mesh, b_ext, precision: int = FP64, m0=None, materials=None, **opts) -> int:
        a = MeshArgs(mesh, materials)
        b = np.ascontiguousarray(b_ext, dtype=np.float64)
        m0a = None if m0 is None else np.ascontiguousarray(m0, dtype=np.float64)
        t = C.c_uint64()
        o = make_options(**opts)
        _check(self.lib.mmsd_submit(self.handle, C.byref(a.c), a.mats, a.n_mats, _dp(b), precision,
                                    None if m0a is None else _dp(m0a), C.byref(o), C.byref(t)))
        return int(t.value)

    def poll(self, ticket: int, n_magnetic: Optional[int] = None):
        """None while running; (Result, m or None) when done."""
        r = ResultC()
        m = None if n_magnetic is None else np.empty((n_magnetic, 3))
        rc = self.lib.mmsd_poll(self.handle, ticket, C.byref(r), None if m is None else _dp(m))
        if rc == E_BUSY:
            return None
        _check(rc)
        return Result.from_c(r), m

    def cancel(self, ticket: int):
        _check(self.lib.mmsd_cancel(self.handle, ticket))

    def stats(self) -> dict:
        s = (C.c_double * 9)()
        _check(self.lib.mmsd_server_stats(self.handle, s))
        keys = ["submitted", "completed", "resident", "queued", "bytes_resident", "launches", "node_evals",
                "setup_seconds", "loop_seconds"]
        return dict(zip(keys, s[:]))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.mmsd_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
