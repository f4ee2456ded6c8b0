"""Host logic of the tile-size autotuner (CPU): the committed cache is well formed, lookup
picks the entry of the nearest size class, mixed-degree fitting keeps the shared LDS within
its budget, and the tuner's LDS model agrees with the library's own limit (esdg_swe_init
rejects a tile size whose LDS exceeds 160 KiB, and plans without a device)."""
import ctypes as C
import json

import numpy as np
import pytest

from paper_2005_02516_amd import autotune as A
from paper_2005_02516_amd import binding
from paper_2005_02516_amd import workloads as wl


def _cache():
    with open(A.CACHE) as f:
        return json.load(f)["entries"]


def test_cache_entries_well_formed():
    for key, e in _cache().items():
        prec, nn, cls = key.split(":")
        N = int(nn[1:])
        assert prec in ("fp32", "fp64") and 1 <= N <= 5 and cls in ("S", "M", "L"), key
        assert A.size_class(e["K"]) == cls, key
        P = e.get("parts", A.default_shape(N, prec)[1])
        assert e["epb"] in A.CANDIDATES and A.lds_ok(N, e["epb"], prec, P), key
        if "rows" in e:                                          # the chosen (E, R, P) was timed
            assert (e["rows"], e["parts"]) in A.shapes(N, prec), key
            assert f'{e["epb"]}:{e["rows"]}:{e["parts"]}' in e["shape_us_per_stage"], key
        else:
            assert str(e["epb"]) in e["us_per_stage"], key          # the chosen size was timed


def test_lookup_size_classes():
    c = _cache()
    assert A.lookup("fp32", [(3, 8192)]) == {3: c["fp32:N3:S"]["epb"]}
    assert A.lookup("fp32", [(1, 65522)]) == {1: c["fp32:N1:M"]["epb"]}
    assert A.lookup("fp64", [(1, 65522)]) == {1: c["fp64:N1:M"]["epb"]}
    assert A.lookup("fp32", [(5, 524288)]) == {5: c["fp32:N5:L"]["epb"]}
    # no large-mesh class at N=4: the nearest one (M) serves it
    assert A.lookup("fp32", [(4, 524288)]) == {4: c["fp32:N4:M"]["epb"]}
    # the split-bf16 mode has the float LDS footprint
    assert A.lookup("bf16x3", [(5, 524288)]) == A.lookup("fp32", [(5, 524288)])
    # instances of one degree add up before the class is picked
    assert A.lookup("fp32", [(3, 20000), (3, 20000)]) == {3: c["fp32:N3:M"]["epb"]}


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_fit_mixed_budget(prec):
    word = 8 if prec == "fp64" else 4
    tuned = A.lookup(prec, [(2, 8192), (3, 8192), (4, 8192)])
    fitted = A.fit_mixed(prec, tuned)
    ref_max = max(A.ref_words(N) for N in fitted)
    P = {N: A.default_shape(N, prec)[1] for N in tuned}
    alone = max((A.ref_words(N) + A.tile_words(N, E, P[N])) * word + A.STATIC_LDS for N, E in tuned.items())
    budget = max(A.LDS_FOUR_PER_CU, alone)
    for N, E in fitted.items():
        assert E <= tuned[N] and (E == tuned[N] or E in A.CANDIDATES)
        assert E == 1 or (ref_max + A.tile_words(N, E, P[N])) * word + A.STATIC_LDS <= budget
        if E < tuned[N]:          # the largest candidate that fits
            bigger = min(c for c in A.CANDIDATES if c > E)
            assert (ref_max + A.tile_words(N, bigger, P[N])) * word + A.STATIC_LDS > budget
    assert A.fit_mixed(prec, {3: 8}) == {3: 8}


def test_parse_cases():
    assert A.parse_cases(None) == A.DEFAULT_CASES
    assert A.parse_cases("1:256,3:64") == [(1, 256), (3, 64)]
    with pytest.raises(ValueError):
        A.parse_cases("6:64")


def _init_status(lib, w, prec, E, shape=None):
    xg, yg, b = (np.ascontiguousarray(a) for a in (w.xg, w.yg, w.b_nodes))
    arr = (binding.esdg_swe_instance * 1)()
    arr[0] = binding.esdg_swe_instance(w.N, w.K, binding._dptr(xg), binding._dptr(yg), binding._dptr(b), w.Lx, w.Ly)
    opt = binding.make_options(prec, "lf", 1.0, True, {w.N: E}, shape={w.N: shape} if shape else None)
    h, nb = C.c_void_p(), C.c_size_t()
    st = lib.esdg_swe_init(1, arr, None, C.byref(opt), C.byref(h), C.byref(nb))
    if st == binding.ESDG_OK:
        lib.esdg_swe_destroy(h)
    return st


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_lds_model_matches_library_limit(prec):
    """The largest tile size the tuner's model fits in 160 KiB is the largest the library
    accepts (below the ABI's limit of 64 elements)."""
    lib = binding.load_library()
    word = 8 if prec == "fp64" else 4
    for N in range(1, 6):
        w = wl.config2(n=2, N=N)
        fits = [E for E in range(1, 65)
                if (A.ref_words(N) + A.tile_words(N, E, A.default_shape(N, prec)[1])) * word <= 160 * 1024]
        emax = max(fits)
        assert _init_status(lib, w, prec, emax) == binding.ESDG_OK, (N, emax)
        if emax < 64:
            assert _init_status(lib, w, prec, emax + 1) == binding.ESDG_EINVAL, (N, emax + 1)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_shapes_match_library(prec):
    """Every (R, P) the tuner searches is accepted by the library, other shapes are refused,
    and the LDS model with P column parts agrees with the library's 160 KiB limit."""
    lib = binding.load_library()
    word = 8 if prec == "fp64" else 4
    for N in range(1, 6):
        w = wl.config2(n=2, N=N)
        ok = A.shapes(N, prec)
        for R in (1, 2, 3):
            for P in (1, 2, 3, 4, 5):
                st = _init_status(lib, w, prec, 1, A.shape_code(R, P))
                assert (st == binding.ESDG_OK) == ((R, P) in ok), (N, R, P, st)
        for R, P in ok:
            fits = [E for E in range(1, 65) if (A.ref_words(N) + A.tile_words(N, E, P)) * word <= 160 * 1024]
            emax = max(fits)
            assert _init_status(lib, w, prec, emax, A.shape_code(R, P)) == binding.ESDG_OK, (N, R, P, emax)
            if emax < 64:
                assert _init_status(lib, w, prec, emax + 1, A.shape_code(R, P)) == binding.ESDG_EINVAL, (N, R, P)


def test_lookup_shapes_defaults_without_entry():
    e, shp = A.lookup_shapes("fp32", [(3, 8192)])
    assert e == A.lookup("fp32", [(3, 8192)])
    c = _cache()["fp32:N3:S"]
    if "rows" in c:
        assert shp == {3: A.shape_code(c["rows"], c["parts"])}
    else:
        assert shp is None


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_mixed_degrees_take_default_shape(prec):
    """A launch of several degrees uses the default tile shape and, per degree, the E timed
    fastest with it (then fitted to the shared LDS); so do the split-bf16 mode and
    matrix-core contractions on one degree."""
    c = _cache()
    sizes = [(2, 1 << 20), (3, 1 << 20), (4, 1 << 20)]
    e, shp = A.lookup_shapes(prec, sizes)
    assert shp is None
    best = {}
    for N in (2, 3, 4):
        ent = next(c[f"{prec}:N{N}:{cls}"] for cls in ("L", "M", "S") if f"{prec}:N{N}:{cls}" in c)
        t = ent["us_per_stage"]
        best[N] = int(min(t, key=lambda k: t[k])) if "rows" in ent else ent["epb"]
    assert e == A.fit_mixed(prec, best)
    for N in (1, 2, 3, 4, 5):
        assert A.lookup_shapes("bf16x3", [(N, 131072)])[1] is None
        assert A.lookup_shapes(prec, [(N, 131072)], valu=False)[1] is None
