"""Thin ctypes binding of libesdg_swe.so (the C ABI in include/esdg_swe.h).

Argument marshalling only: every step of the RHS and the RK update runs in the HIP
kernels of the library.  PyTorch supplies the device workspace and the HIP stream.
The module raises at load time if the library is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

from .build import library_path

ESDG_OK, ESDG_EINVAL, ESDG_EMESH, ESDG_ENOMEM, ESDG_EDEVICE, ESDG_ENONPHYS, ESDG_ESTATE = 0, -1, -2, -3, -4, -5, -6
ESDG_FP64, ESDG_FP32, ESDG_FP32_BF16X3 = 0, 1, 2
ESDG_FLUX_EC, ESDG_FLUX_LF = 0, 1

PRECISIONS = {"fp64": ESDG_FP64, "fp32": ESDG_FP32, "bf16x3": ESDG_FP32_BF16X3}
FLUXES = {"ec": ESDG_FLUX_EC, "lf": ESDG_FLUX_LF}

EXPORTED = [
    "esdg_swe_init", "esdg_swe_bind", "esdg_swe_set_state", "esdg_swe_set_state_modal", "esdg_swe_get_state",
    "esdg_swe_state_device", "esdg_swe_rhs", "esdg_swe_rhs_noalloc", "esdg_swe_step", "esdg_swe_diagnostics", "esdg_swe_sync",
    "esdg_swe_query", "esdg_swe_launch_info", "esdg_swe_reference_level", "esdg_swe_last_error", "esdg_swe_destroy",
    "esdg_volume_kernel",
]


class esdg_swe_instance(C.Structure):
    _fields_ = [("N", C.c_int32), ("K", C.c_int32), ("xg", C.POINTER(C.c_double)), ("yg", C.POINTER(C.c_double)),
                ("b", C.POINTER(C.c_double)), ("Lx", C.c_double), ("Ly", C.c_double)]


class esdg_swe_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("flux", C.c_int32), ("g", C.c_double),
                ("use_graph", C.c_int32), ("elems_per_block", C.c_int32 * 6), ("matrix_cores", C.c_int32),
                ("fused_steps", C.c_int32), ("mass_inverse", C.c_int32), ("tile_shape", C.c_int32 * 6),
                ("scheme", C.c_int32)]


class esdg_swe_quadrature(C.Structure):
    _fields_ = [("vol_degree", C.c_int32), ("face_points", C.c_int32), ("nq", C.c_int32),
                ("rq", C.POINTER(C.c_double)), ("sq", C.POINTER(C.c_double)), ("wq", C.POINTER(C.c_double))]


FUSED = {False: 0, True: 1, "auto": 2}
MASS = {"stored": 0, "wadg": 1}      # inverse curved mass matrices: stored, or weight-adjusted
SCHEMES = {"modal": 0, "sbp": 1}     # modal ESDG (hybridized operators), or DG-SBP


def _per_degree(v):
    arr = (C.c_int32 * 6)()
    if isinstance(v, int):
        for N in range(1, 6):
            arr[N] = v
    elif v:
        for N, E in v.items():
            arr[int(N)] = int(E)
    return arr


def shape_code(rows: int, parts: int) -> int:
    """Tile shape of the residual phase as the ABI packs it: (rows << 4) | parts."""
    return (int(rows) << 4) | int(parts)


def make_options(precision: str, flux: str, g: float, use_graph: bool = True, epb=None,
                 matrix_cores: bool = False, fused="auto", mass: str = "stored",
                 scheme: str = "modal", shape=None) -> esdg_swe_options:
    """epb: None, an int (all degrees) or a mapping N -> elements per workgroup; shape: None,
    a packed tile shape (all degrees) or a mapping N -> packed shape (shape_code)."""
    return esdg_swe_options(PRECISIONS[precision], FLUXES[flux], float(g), int(use_graph), _per_degree(epb),
                            2 if matrix_cores else 1, FUSED[fused], MASS[mass], _per_degree(shape), SCHEMES[scheme])


def make_quadrature(spec, keep: list) -> esdg_swe_quadrature:
    """spec: None (default rules) or a mapping with optional keys vol_degree, face_points and
    rule = (r, s, w) (a caller's volume rule).  Arrays are appended to ``keep``, which must
    outlive the init call."""
    q = esdg_swe_quadrature()
    if not spec:
        return q
    q.vol_degree = int(spec.get("vol_degree", 0))
    q.face_points = int(spec.get("face_points", 0))
    rule = spec.get("rule")
    if rule is not None:
        r, s_, w = (np.ascontiguousarray(a, dtype=np.float64) for a in rule)
        keep += [r, s_, w]
        q.nq = int(w.size)
        q.rq, q.sq, q.wq = _dptr(r), _dptr(s_), _dptr(w)
    return q


class EsdgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"esdg status {status}: {msg}")
        self.status = status


_lib = None


def load_library(path: Optional[str] = None) -> C.CDLL:
    """Load libesdg_swe.so and declare its signatures (no GPU needed for loading).

    The in-tree build is used unless ``path`` or the ESDG_SWE_LIBRARY environment
    variable names another build of the same library."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or os.environ.get("ESDG_SWE_LIBRARY") or library_path()
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with `python -m paper_2005_02516_amd.build`")
    lib = C.CDLL(p)
    vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
    pdbl = C.POINTER(C.c_double)
    lib.esdg_swe_init.argtypes = [i32, C.POINTER(esdg_swe_instance), C.POINTER(esdg_swe_quadrature),
                                  C.POINTER(esdg_swe_options), C.POINTER(vp), C.POINTER(C.c_size_t)]
    lib.esdg_swe_bind.argtypes = [vp, vp, C.c_size_t, vp]
    lib.esdg_swe_set_state.argtypes = [vp, i32, pdbl]
    lib.esdg_swe_set_state_modal.argtypes = [vp, i32, pdbl]
    lib.esdg_swe_get_state.argtypes = [vp, i32, pdbl]
    lib.esdg_swe_state_device.argtypes = [vp, i32, C.POINTER(vp)]
    lib.esdg_swe_rhs.argtypes = [vp, i32, vp, vp]
    lib.esdg_swe_rhs_noalloc.argtypes = [vp, i32, vp, vp]
    lib.esdg_swe_step.argtypes = [vp, pdbl, i32]
    lib.esdg_swe_diagnostics.argtypes = [vp, pdbl]
    lib.esdg_swe_sync.argtypes = [vp]
    lib.esdg_swe_query.argtypes = [vp, i32, C.POINTER(i32)]
    lib.esdg_swe_reference_level.argtypes = [vp, i32, pdbl]
    lib.esdg_swe_last_error.argtypes = [vp]
    lib.esdg_swe_last_error.restype = C.c_char_p
    lib.esdg_swe_destroy.argtypes = [vp]
    lib.esdg_swe_destroy.restype = None
    lib.esdg_volume_kernel.argtypes = [i32, i32, vp, vp, vp, vp, i32, i32, C.c_double, vp]
    for name in EXPORTED:
        if name not in ("esdg_swe_last_error", "esdg_swe_destroy"):
            getattr(lib, name).restype = C.c_int32
    if path is None:
        _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class EsdgSwe:
    """One solver handle for n_inst instances, bound to a torch-allocated workspace."""

    def __init__(self, instances: Sequence, precision: str = "fp64", flux: str = "lf", g: float = 1.0,
                 elems_per_block=None, use_graph: bool = True, device: str = "cuda:0", stream=None,
                 tuned: bool = True, matrix_cores: Optional[bool] = None, fused: Optional[bool] = None,
                 mass: str = "stored", quadrature=None, scheme: str = "modal", tile_shape=None):
        """quadrature: None, one spec for every instance, or a list of specs (make_quadrature);
        scheme: "modal" (Section 2) or "sbp" (DG-SBP of Section 3, each spec with its rule)."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("EsdgSwe needs a GPU: the library has no CPU path")
        self.lib = load_library()
        self.torch = torch
        self.device = torch.device(device)
        self._keep = []
        arr = (esdg_swe_instance * len(instances))()
        for i, w in enumerate(instances):
            xg = np.ascontiguousarray(w.xg, dtype=np.float64)
            yg = np.ascontiguousarray(w.yg, dtype=np.float64)
            b = np.ascontiguousarray(w.b_nodes, dtype=np.float64)
            self._keep += [xg, yg, b]
            arr[i] = esdg_swe_instance(w.N, w.K, _dptr(xg), _dptr(yg), _dptr(b), w.Lx, w.Ly)
        if quadrature is None or isinstance(quadrature, dict):
            quadrature = [quadrature] * len(instances)
        qarr = (esdg_swe_quadrature * len(instances))()
        for i, spec in enumerate(quadrature):
            qarr[i] = make_quadrature(spec, self._keep)
        default_rules = scheme == "modal" and not any(quadrature)
        if matrix_cores is None:
            matrix_cores = os.environ.get("ESDG_SWE_MATRIX_CORES", "0") == "1"
        if not elems_per_block and tuned and default_rules:   # the tuning cache covers the default rules
            from .autotune import lookup_shapes
            elems_per_block, tuned_shape = lookup_shapes(precision, [(w.N, w.K) for w in instances],
                                                         valu=not matrix_cores)
            if tile_shape is None:
                tile_shape = tuned_shape
        if fused is None:       # one launch per step call when tiles can stay resident
            fused = {"0": False, "1": True}.get(os.environ.get("ESDG_SWE_FUSED", ""), "auto")
        self.elems_per_block = elems_per_block
        self.tile_shape = tile_shape
        opt = make_options(precision, flux, g, use_graph, elems_per_block, matrix_cores, fused, mass, scheme, tile_shape)
        self.mass = mass
        self.scheme = scheme
        h = C.c_void_p()
        nbytes = C.c_size_t()
        st = self.lib.esdg_swe_init(len(instances), arr, qarr, C.byref(opt), C.byref(h), C.byref(nbytes))
        if st != ESDG_OK:
            raise EsdgError(st, self.lib.esdg_swe_last_error(None).decode())
        self.h = h
        self.n_inst = len(instances)
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self._check(self.lib.esdg_swe_bind(self.h, C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                           C.c_void_p(self.stream.cuda_stream)))
        self.sizes = [self.query(i) for i in range(self.n_inst)]

    # -- helpers -------------------------------------------------------------------
    def _check(self, st: int):
        if st != ESDG_OK:
            raise EsdgError(st, self.lib.esdg_swe_last_error(self.h).decode())

    def launch_info(self):
        out = (C.c_int32 * 4)()
        self._check(self.lib.esdg_swe_launch_info(self.h, out))
        return dict(zip(["tiles", "resident_workgroups", "lds_bytes", "step_mode"], list(out)))

    def query(self, inst: int):
        out = (C.c_int32 * 6)()
        self._check(self.lib.esdg_swe_query(self.h, inst, out))
        return dict(zip(["N", "K", "Np", "Nq", "Nfq", "Nh"], list(out)))

    # -- C-ABI entry points (same names) ------------------------------------------
    def esdg_swe_set_state(self, inst: int, u_nodes: np.ndarray):
        """u_nodes: (h, hu, hv) at the geometry nodes, [3][K][(N+1)(N+2)/2]."""
        u = np.ascontiguousarray(u_nodes, dtype=np.float64)
        z = self.sizes[inst]
        assert u.shape == (3, z["K"], (z["N"] + 1) * (z["N"] + 2) // 2), u.shape
        self._check(self.lib.esdg_swe_set_state(self.h, inst, _dptr(u)))

    def esdg_swe_set_state_modal(self, inst: int, uh: np.ndarray):
        u = np.ascontiguousarray(uh, dtype=np.float64)
        z = self.sizes[inst]
        assert u.shape == (3, z["K"], z["Np"]), u.shape
        self._check(self.lib.esdg_swe_set_state_modal(self.h, inst, _dptr(u)))

    def esdg_swe_get_state(self, inst: int) -> np.ndarray:
        z = self.sizes[inst]
        out = np.empty((3, z["K"], z["Np"]), dtype=np.float64)
        self._check(self.lib.esdg_swe_get_state(self.h, inst, _dptr(out)))
        return out

    def esdg_swe_reference_level(self, inst: int) -> float:
        out = C.c_double()
        self._check(self.lib.esdg_swe_reference_level(self.h, inst, C.byref(out)))
        return out.value

    def esdg_swe_state_device(self, inst: int):
        """torch view of the instance state in the workspace ([3][K][Np] (eta, hu, hv), library precision)."""
        p = C.c_void_p()
        self._check(self.lib.esdg_swe_state_device(self.h, inst, C.byref(p)))
        z = self.sizes[inst]
        off = p.value - self.workspace.data_ptr()
        nbytes = 3 * z["K"] * z["Np"] * (8 if self.dtype == self.torch.float64 else 4)
        return self.workspace[off:off + nbytes].view(self.dtype).view(3, z["K"], z["Np"])

    def esdg_swe_rhs(self, inst: int, state, rhs):
        z = self.sizes[inst]
        for t in (state, rhs):
            assert t.is_cuda and t.dtype == self.dtype and t.is_contiguous() and tuple(t.shape) == (3, z["K"], z["Np"])
        self._check(self.lib.esdg_swe_rhs(self.h, inst, C.c_void_p(state.data_ptr()), C.c_void_p(rhs.data_ptr())))

    def esdg_swe_rhs_noalloc(self, inst: int, state, rhs):
        """esdg_swe_rhs with its scratch in the library's per-device array (no allocation)."""
        z = self.sizes[inst]
        for t in (state, rhs):
            assert t.is_cuda and t.dtype == self.dtype and t.is_contiguous() and tuple(t.shape) == (3, z["K"], z["Np"])
        self._check(self.lib.esdg_swe_rhs_noalloc(self.h, inst, C.c_void_p(state.data_ptr()),
                                                  C.c_void_p(rhs.data_ptr())))

    def esdg_swe_step(self, dt, nsteps: int):
        d = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (self.n_inst,)))
        self._check(self.lib.esdg_swe_step(self.h, _dptr(d), int(nsteps)))

    def esdg_swe_diagnostics(self) -> np.ndarray:
        out = np.empty((self.n_inst, 6), dtype=np.float64)
        self._check(self.lib.esdg_swe_diagnostics(self.h, _dptr(out)))
        return out

    def esdg_swe_sync(self):
        self._check(self.lib.esdg_swe_sync(self.h))

    # short aliases
    set_state = esdg_swe_set_state
    set_state_modal = esdg_swe_set_state_modal
    get_state = esdg_swe_get_state
    state_device = esdg_swe_state_device
    rhs = esdg_swe_rhs
    rhs_noalloc = esdg_swe_rhs_noalloc
    step = esdg_swe_step
    diagnostics = esdg_swe_diagnostics
    sync = esdg_swe_sync
    reference_level = esdg_swe_reference_level

    def close(self):
        if getattr(self, "h", None):
            self.stream.synchronize()
            self.lib.esdg_swe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


VOLUME_KINDS = {"traditional": 0, "entropy_stable": 1}


def esdg_volume_kernel(kind: str, QxT, QyT, u, r, g: float, stream=None) -> None:
    """The Section 5.4 volume term on the GPU (esdg_volume_kernel): torch tensors on the
    device, QxT/QyT [n][n] (transposed matrices), u and r [3][K][n], all float64 or all
    float32; asynchronous on ``stream`` (torch's current stream if None)."""
    import torch
    lib = load_library()
    ts = (QxT, QyT, u, r)
    if not all(t.is_cuda and t.is_contiguous() and t.dtype == u.dtype for t in ts):
        raise ValueError("QxT, QyT, u, r must be contiguous device tensors of one dtype")
    if u.dtype not in (torch.float64, torch.float32):
        raise ValueError("float64 or float32 only")
    n, K = int(u.shape[2]), int(u.shape[1])
    if tuple(QxT.shape) != (n, n) or tuple(QyT.shape) != (n, n) or tuple(r.shape) != tuple(u.shape) or u.shape[0] != 3:
        raise ValueError("shapes: QxT, QyT [n][n]; u, r [3][K][n]")
    st = stream if stream is not None else torch.cuda.current_stream(u.device)
    status = lib.esdg_volume_kernel(VOLUME_KINDS[kind], 0 if u.dtype == torch.float64 else 1,
                                    C.c_void_p(QxT.data_ptr()), C.c_void_p(QyT.data_ptr()), C.c_void_p(u.data_ptr()),
                                    C.c_void_p(r.data_ptr()), n, K, float(g), C.c_void_p(st.cuda_stream))
    if status != ESDG_OK:
        raise EsdgError(status, f"esdg_volume_kernel returned {status}")
