"""The no-allocation RHS entry point (esdg_swe_rhs_noalloc, for callers that cannot allocate
device memory) against esdg_swe_rhs, through the C ABI: the same kernels on the same
inputs, so the results must agree bitwise.  Two calls in a row, the second on a smaller
instance (the scratch array keeps the first call's contents), in FP32 and FP64; an
instance whose scratch need exceeds the array is refused before any launch."""
import numpy as np
import pytest

from paper_2005_02516_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _solver(w, precision):
    from paper_2005_02516_amd.binding import EsdgSwe
    s = EsdgSwe([w], precision=precision, flux="lf", g=w.g)
    s.set_state(0, w.u_nodes)
    return s


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_rhs_matches_rhs(precision):
    import torch
    print(f"no-alloc rhs, {precision}: config-2 recipe n=8 then n=3, N=3", flush=True)
    for n in (8, 3):                      # second call: smaller input
        w = wl.config2(n=n, N=3)
        s = _solver(w, precision)
        st = s.state_device(0)
        # a perturbed state, so that the evaluation does not sit at the initial projection
        x = (st + 1e-3 * torch.sin(torch.arange(st.numel(), device=st.device, dtype=st.dtype)).view_as(st)).contiguous()
        r_ref = torch.full_like(x, float("nan"))
        r_na = torch.full_like(x, float("nan"))
        s.rhs(0, x, r_ref)
        s.rhs_noalloc(0, x, r_na)
        s.sync()
        a, b = r_ref.cpu().numpy(), r_na.cpu().numpy()
        assert np.all(np.isfinite(a))
        np.testing.assert_array_equal(a, b)
        s.close()


def test_noalloc_rejects_oversize():
    import torch
    from paper_2005_02516_amd.binding import EsdgError, ESDG_EINVAL
    print("no-alloc rhs: oversize instance N=5, K=32768, fp64 (75 MB of scratch)", flush=True)
    w = wl.config2(n=128, N=5)
    s = _solver(w, "fp64")
    st = s.state_device(0)
    out = torch.empty_like(st)
    with pytest.raises(EsdgError) as e:
        s.rhs_noalloc(0, st, out)
    assert e.value.status == ESDG_EINVAL and "scratch" in str(e.value)
    s.close()
