"""Host-side checks of bench.py's bookkeeping (no GPU): the committed HBM counter summaries
are picked only for the kernel source, workload, launch mode and stages per launch they
were taken on."""
import importlib.util
import os
import types

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _summaries(b):
    out = []
    for path in b.TRAFFIC_FILES:
        if not os.path.exists(path):
            continue
        kv = {}
        with open(path) as fh:
            for line in fh:
                if "=" in line and not line.startswith("#"):
                    k, v = line.strip().split("=", 1)
                    kv[k] = v
        out.append((path, kv))
    return out


FIT_KEYS = ("fixed_fetch_bytes", "per_stage_fetch_bytes", "fixed_write_bytes", "per_stage_write_bytes")


def test_traffic_summaries_well_formed():
    """A summary gives the bytes of a launch of stages_per_launch stages, or (multi-stage
    launches) a fixed part and a per-stage part fitted over two stage counts."""
    b = _bench()
    found = _summaries(b)
    assert found, "no committed HBM counter summary"
    for path, kv in found:
        for key in ("kernel_source_sha256", "N", "K", "precision", "epb", "step_mode"):
            assert key in kv, (path, key)
        assert int(kv["step_mode"]) in (0, 1, 2)
        if "per_stage_fetch_bytes" in kv:
            assert all(k in kv for k in FIT_KEYS), path
            assert int(kv["step_mode"]) != 0, path
            assert all(int(kv[k]) > 0 for k in FIT_KEYS), path
        else:
            for key in ("stages_per_launch", "fetch_bytes", "write_bytes"):
                assert key in kv, (path, key)
            assert int(kv["fetch_bytes"]) > 0 and int(kv["write_bytes"]) > 0
            assert (int(kv["stages_per_launch"]) == 1) == (int(kv["step_mode"]) == 0)


def test_traffic_lookup_matches_only_its_configuration():
    b = _bench()
    for path, kv in _summaries(b):
        if kv["kernel_source_sha256"] != b.kernel_source_hash():
            continue  # taken on an older kernel source: never reported
        N, K, prec, epb = int(kv["N"]), int(kv["K"]), kv["precision"], int(kv["epb"])
        w = types.SimpleNamespace(N=N, K=K)
        other = "fp64" if prec == "fp32" else "fp32"
        mode = int(kv["step_mode"])
        if "per_stage_fetch_bytes" in kv:
            spl = 100
            want = round(int(kv["fixed_fetch_bytes"]) / spl + int(kv["per_stage_fetch_bytes"]))
            tr = b.measured_traffic(w, prec, epb, mode, spl)
            assert tr is not None and tr["fetch"] == want, path
            tr1000 = b.measured_traffic(w, prec, epb, mode, 1000)
            assert tr1000["fetch"] < tr["fetch"] and tr1000["write"] < tr["write"], path
        else:
            spl = int(kv["stages_per_launch"])
            tr = b.measured_traffic(w, prec, epb, mode, spl)
            assert tr is not None and tr["fetch"] == int(kv["fetch_bytes"]), path
            assert b.measured_traffic(w, prec, epb, mode, spl + 5) is None
        assert b.measured_traffic(w, other, epb, mode, spl) is None
        assert b.measured_traffic(w, prec, epb + 1, mode, spl) is None
        assert b.measured_traffic(w, prec, epb, (mode + 1) % 3, spl) is None or mode == 1
        assert b.measured_traffic(types.SimpleNamespace(N=N % 5 + 1, K=K), prec, epb, mode, spl) is None
