"""The C-ABI library loads, exports every symbol the header declares, and validates its
inputs at plan time (esdg_swe_init makes no device call, so this runs without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2005_02516_amd import binding
from paper_2005_02516_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    """Every function the headers under include/ declare (esdg_swe_* and esdg_volume_*)."""
    names = set()
    for f in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if f.endswith(".h"):
            text = open(os.path.join(ROOT, "include", f)).read()
            names |= set(re.findall(r"\b(esdg_(?:swe|volume)_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_symbols_exported():
    lib = binding.load_library()
    syms = header_symbols()
    assert len(syms) >= 14, syms
    for name in syms:
        assert hasattr(lib, name), name
    assert sorted(binding.EXPORTED) == syms


def _init(lib, w, precision=1, flux=1, g=1.0, epb=0, xg=None):
    xg = np.ascontiguousarray(w.xg if xg is None else xg)
    yg = np.ascontiguousarray(w.yg)
    b = np.ascontiguousarray(w.b_nodes)
    arr = (binding.esdg_swe_instance * 1)()
    arr[0] = binding.esdg_swe_instance(w.N, w.K, binding._dptr(xg), binding._dptr(yg), binding._dptr(b), w.Lx, w.Ly)
    opt = binding.make_options({0: "fp64", 1: "fp32"}.get(precision, "fp32") if precision in (0, 1) else "fp32",
                               {0: "ec", 1: "lf"}[flux], g, True, epb)
    if precision not in (0, 1):
        opt.precision = precision
    h = C.c_void_p()
    nb = C.c_size_t()
    st = lib.esdg_swe_init(1, arr, None, C.byref(opt), C.byref(h), C.byref(nb))
    return st, h, nb.value, lib.esdg_swe_last_error(None).decode()


def test_init_plans_without_device():
    lib = binding.load_library()
    for N in range(1, 6):
        w = wl.config2(n=3, N=N)
        st, h, nbytes, msg = _init(lib, w)
        assert st == binding.ESDG_OK, msg
        Np, Nh = (N + 1) * (N + 2) // 2, (N + 1) ** 2 + 3 * (N + 1)
        assert nbytes > 4 * w.K * (3 * 2 * Np + 4 * 3 * Nh)
        out = (C.c_int32 * 6)()
        assert lib.esdg_swe_query(h, 0, out) == 0
        assert list(out) == [N, w.K, Np, (N + 1) ** 2, 3 * (N + 1), Nh]
        lib.esdg_swe_destroy(h)


def test_init_rejects_bad_input():
    lib = binding.load_library()
    w = wl.config2(n=3, N=2)
    st, h, _, msg = _init(lib, w, g=-1.0)
    assert st == binding.ESDG_EINVAL
    st, h, _, msg = _init(lib, w, precision=7)
    assert st == binding.ESDG_EINVAL
    bad = w.xg.copy()
    bad[0] = bad[0][::-1].copy()            # a clockwise / folded element
    st, h, _, msg = _init(lib, w, xg=bad)
    assert st == binding.ESDG_EMESH and "Jacobian" in msg
    shifted = w.xg.copy()
    shifted[3] += 0.01                      # a hole in the mesh: faces no longer match
    st, h, _, msg = _init(lib, w, xg=shifted)
    assert st == binding.ESDG_EMESH and "partner" in msg


def test_calls_before_bind_fail_cleanly():
    lib = binding.load_library()
    w = wl.config2(n=2, N=1)
    st, h, _, msg = _init(lib, w)
    assert st == 0
    dt = np.array([1e-3])
    assert lib.esdg_swe_step(h, binding._dptr(dt), 1) == binding.ESDG_ESTATE
    u = np.ascontiguousarray(w.u_nodes)
    assert lib.esdg_swe_set_state(h, 0, binding._dptr(u)) == binding.ESDG_ESTATE
    assert lib.esdg_swe_rhs(h, 0, u.ctypes.data, u.ctypes.data) == binding.ESDG_ESTATE
    assert lib.esdg_swe_rhs_noalloc(h, 0, u.ctypes.data, u.ctypes.data) == binding.ESDG_ESTATE
    lib.esdg_swe_destroy(h)


def test_init_weight_adjusted_mass():
    """ESDG_MASS_WEIGHT_ADJUSTED plans without a device, stores Nq reals of w/J per element
    instead of the Np x Np inverse (smaller workspace), and an unknown mode is rejected."""
    lib = binding.load_library()
    w = wl.config2(n=3, N=5)
    sizes = {}
    for mass in ("stored", "wadg"):
        xg, yg, b = (np.ascontiguousarray(a) for a in (w.xg, w.yg, w.b_nodes))
        arr = (binding.esdg_swe_instance * 1)()
        arr[0] = binding.esdg_swe_instance(w.N, w.K, binding._dptr(xg), binding._dptr(yg), binding._dptr(b), w.Lx, w.Ly)
        opt = binding.make_options("fp32", "lf", 1.0, True, 0, mass=mass)
        h, nb = C.c_void_p(), C.c_size_t()
        assert lib.esdg_swe_init(1, arr, None, C.byref(opt), C.byref(h), C.byref(nb)) == binding.ESDG_OK
        sizes[mass] = nb.value
        lib.esdg_swe_destroy(h)
    Np, Nq = 21, 36
    assert sizes["stored"] - sizes["wadg"] >= 4 * w.K * (Np * Np - Nq)
    opt = binding.make_options("fp32", "lf", 1.0, True, 0)
    opt.mass_inverse = 2
    arr = (binding.esdg_swe_instance * 1)()
    arr[0] = binding.esdg_swe_instance(w.N, w.K, binding._dptr(xg), binding._dptr(yg), binding._dptr(b), w.Lx, w.Ly)
    h, nb = C.c_void_p(), C.c_size_t()
    assert lib.esdg_swe_init(1, arr, None, C.byref(opt), C.byref(h), C.byref(nb)) == binding.ESDG_EINVAL


def test_init_walls():
    """A closed basin (periods 0) plans with its boundary faces as reflective walls; the same
    mesh declared fully periodic is rejected (its boundary faces have no partner)."""
    lib = binding.load_library()
    w = wl.basin(n=3, N=3)
    for L, expect in ((0.0, binding.ESDG_OK), (2.0, binding.ESDG_EMESH)):
        xg, yg, b = (np.ascontiguousarray(a) for a in (w.xg, w.yg, w.b_nodes))
        arr = (binding.esdg_swe_instance * 1)()
        arr[0] = binding.esdg_swe_instance(w.N, w.K, binding._dptr(xg), binding._dptr(yg), binding._dptr(b), L, L)
        opt = binding.make_options("fp32", "lf", 1.0, True, 0)
        h, nb = C.c_void_p(), C.c_size_t()
        st = lib.esdg_swe_init(1, arr, None, C.byref(opt), C.byref(h), C.byref(nb))
        assert st == expect, lib.esdg_swe_last_error(None).decode()
        if st == binding.ESDG_OK:
            lib.esdg_swe_destroy(h)


def test_empty_and_out_of_range_inputs():
    """Empty inputs and sizes outside the documented ranges are rejected at the boundary,
    before any device call: no instances, an instance of 0 elements, degrees 0 and 6, more
    than 64 elements per workgroup; the volume-kernel entry point with 0 elements, 0 or 257
    nodes, or an unknown kind."""
    lib = binding.load_library()
    w = wl.config2(n=2, N=2)
    xg, yg, b = (np.ascontiguousarray(a) for a in (w.xg, w.yg, w.b_nodes))

    def init(N, K, n_inst=1, epb=0):
        arr = (binding.esdg_swe_instance * 1)()
        arr[0] = binding.esdg_swe_instance(N, K, binding._dptr(xg), binding._dptr(yg), binding._dptr(b), w.Lx, w.Ly)
        opt = binding.make_options("fp32", "lf", 1.0, True, epb)
        h, nb = C.c_void_p(), C.c_size_t()
        st = lib.esdg_swe_init(n_inst, arr, None, C.byref(opt), C.byref(h), C.byref(nb))
        if st == binding.ESDG_OK:
            lib.esdg_swe_destroy(h)
        return st

    assert init(2, w.K) == binding.ESDG_OK
    assert init(2, w.K, n_inst=0) == binding.ESDG_EINVAL
    assert init(2, 0) == binding.ESDG_EINVAL
    assert init(0, w.K) == binding.ESDG_EINVAL
    assert init(6, w.K) == binding.ESDG_EINVAL
    assert init(2, w.K, epb=65) == binding.ESDG_EINVAL
    dummy = C.c_void_p(16)                   # never dereferenced: the checks come first
    for kind, prec, n, K in ((0, binding.ESDG_FP32, 10, 0), (0, binding.ESDG_FP32, 0, 4),
                             (1, binding.ESDG_FP64, 257, 4), (2, binding.ESDG_FP32, 10, 4)):
        assert lib.esdg_volume_kernel(kind, prec, dummy, dummy, dummy, dummy, n, K, C.c_double(9.81), None) \
            == binding.ESDG_EINVAL, (kind, n, K)


def _init_quad(lib, w, quad, scheme="modal", precision="fp32"):
    keep = []
    xg, yg, b = (np.ascontiguousarray(a) for a in (w.xg, w.yg, w.b_nodes))
    arr = (binding.esdg_swe_instance * 1)()
    arr[0] = binding.esdg_swe_instance(w.N, w.K, binding._dptr(xg), binding._dptr(yg), binding._dptr(b), w.Lx, w.Ly)
    qarr = (binding.esdg_swe_quadrature * 1)()
    qarr[0] = binding.make_quadrature(quad, keep)
    opt = binding.make_options(precision, "lf", 1.0, True, 0, scheme=scheme)
    h = C.c_void_p()
    nb = C.c_size_t()
    st = lib.esdg_swe_init(1, arr, qarr, C.byref(opt), C.byref(h), C.byref(nb))
    out = (C.c_int32 * 6)()
    if st == 0:
        assert lib.esdg_swe_query(h, 0, out) == 0
        lib.esdg_swe_destroy(h)
    return st, lib.esdg_swe_last_error(None).decode(), list(out)


def test_init_quadrature_choices():
    """Section 2.1 quadrature at the boundary: the default rules, the Stroud rule with N+2
    points per direction and N+2 face points, a caller's rule (padded to the compiled node
    count), and the DG-SBP rules (Section 3.1) are accepted; the sizes follow."""
    from oracle import esdg_oracle as O
    from paper_2005_02516_amd import sbp_rules
    lib = binding.load_library()
    for N in (1, 3, 5):
        w = wl.config2(n=2, N=N)
        st, msg, out = _init_quad(lib, w, None)
        assert st == 0 and out[3] == (N + 1) ** 2 and out[4] == 3 * (N + 1), msg
        st, msg, out = _init_quad(lib, w, {"vol_degree": 2 * N + 2, "face_points": N + 2})
        assert st == 0 and out[3] == (N + 2) ** 2 and out[4] == 3 * (N + 2), msg
        st, msg, out = _init_quad(lib, w, {"face_points": N + 2})      # (N+1)^2 Stroud nodes, padded
        assert st == 0 and out[3] == (N + 2) ** 2, msg
        r, s, q = O.stroud_rule(N)
        st, msg, out = _init_quad(lib, w, {"rule": (s, r, q)})
        assert st == 0 and out[3] == (N + 1) ** 2, msg
    w = wl.config2(n=2, N=1)                     # the 3-point edge-midpoint rule (degree 2), padded to 4
    st, msg, out = _init_quad(lib, w, {"rule": ([0.0, 0.0, -1.0], [-1.0, 0.0, 0.0], [2 / 3] * 3)})
    assert st == 0 and out[3] == 4, msg
    st, msg, out = _init_quad(lib, w, {"rule": ([-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0], [2 / 3] * 3)})
    assert st == binding.ESDG_EINVAL, msg       # the vertex rule is exact only to degree 1
    for N in (1, 2, 3, 4):
        w = wl.config2(n=2, N=N)
        st, msg, out = _init_quad(lib, w, {"rule": sbp_rules.load(N)}, scheme="sbp")
        assert st == 0 and out[2] == out[3] == {1: 6, 2: 10, 3: 18, 4: 22}[N], msg


def test_init_quadrature_rejected():
    """Rules that fail Section 2.1's (or 3.1's) conditions are refused with ESDG_EINVAL."""
    from oracle import esdg_oracle as O
    from paper_2005_02516_amd import sbp_rules
    lib = binding.load_library()
    N = 2
    w = wl.config2(n=2, N=N)
    r, s, q = O.stroud_rule(N)
    bad = {
        "not exact": {"rule": (r, s, q * np.r_[1.01, np.ones(q.size - 1)])},
        "negative weight": {"rule": (np.r_[r, -0.5], np.r_[s, -0.5], np.r_[q, -1e-3])},
        "outside": {"rule": (np.r_[r, 0.5], np.r_[s, 0.5], np.r_[q, 0.0])},
        "degree above 2N+3": {"vol_degree": 2 * N + 4},
        "degree below 2N": {"vol_degree": 2 * N - 1},
        "face points": {"face_points": N + 3},
        "too many nodes": {"rule": O.stroud_rule(N, N + 3)},
        "(N+2)^2 nodes with N+1 face points": {"vol_degree": 2 * N + 2},
    }
    for name, quad in bad.items():
        st, msg, _ = _init_quad(lib, w, quad)
        assert st == binding.ESDG_EINVAL, (name, msg)
    # DG-SBP: the rule must contain the face nodes, have the compiled size, and N <= 4
    st, msg, _ = _init_quad(lib, w, {"rule": (r, s, q)}, scheme="sbp")
    assert st == binding.ESDG_EINVAL, msg
    st, msg, _ = _init_quad(lib, w, None, scheme="sbp")
    assert st == binding.ESDG_EINVAL, msg
    w5 = wl.config2(n=2, N=5)
    st, msg, _ = _init_quad(lib, w5, {"rule": sbp_rules.load(4)}, scheme="sbp")
    assert st == binding.ESDG_EINVAL, msg
    st, msg, _ = _init_quad(lib, w, {"rule": sbp_rules.load(N)}, scheme="sbp", precision="bf16x3")
    assert st == binding.ESDG_EINVAL, msg
