"""fr_residual_noalloc, the residual for callers that cannot allocate: its
face data live in the library's fixed per-device array.  Checked through the
C ABI against fr_residual (the same kernels: bitwise equal) on two calls in a
row, the second with a smaller input (the coarser level), then the larger one
again over the array's leftover contents; a level whose face data exceed the
array is refused with FR_EINVAL and nothing launched."""
import numpy as np
import pytest

from paper_2202_09733_amd import capi
from paper_2202_09733_amd import workloads as W
from gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["vortical_16x16_p42", "tgv_8cubed_p32"])
def test_noalloc_residual_equals_fr_residual(case):
    require_gpu()
    announce("fr_residual_noalloc vs fr_residual: " + case)
    if case == "vortical_16x16_p42":
        wl = W.make_vortical_workload(n=(16, 16), dt_factor=1000.0)
    else:
        wl = W.make_tgv_workload(n=(8, 8, 8))
    fr = capi.FR.from_workload(wl)
    dq = fr.to_dev(wl.dq)
    q1 = fr.restrict(0, dq)
    r0 = fr.residual(0, dq).cpu().numpy()
    r1 = fr.residual(1, q1).cpu().numpy()
    a = fr.residual_noalloc(0, dq).cpu().numpy()
    b = fr.residual_noalloc(1, q1).cpu().numpy()     # smaller input
    c = fr.residual_noalloc(0, dq).cpu().numpy()     # over the smaller call's leftovers
    assert np.array_equal(a, r0) and np.array_equal(b, r1) and np.array_equal(c, r0)
    assert np.any(r0) and np.any(r1)


def test_noalloc_refuses_levels_beyond_the_scratch():
    require_gpu()
    announce("fr_residual_noalloc size limit")
    # 3D p = 3: 2 * 3 * 5 * 16 doubles (3840 bytes) per element -> 28^3 elements
    # need 84.3 MB > 64 MiB; the p = 1 level needs 21.1 MB
    wl = W.make_tgv_workload(n=(28, 28, 28), p0=3, p1=1)
    fr = capi.FR.from_workload(wl)
    dq = fr.to_dev(wl.dq)
    with pytest.raises(capi.FRError) as ex:
        fr.residual_noalloc(0, dq)
    assert ex.value.code == capi.FR_EINVAL
    # the coarser level fits, and the context still works
    q1 = fr.restrict(0, dq)
    assert np.array_equal(fr.residual_noalloc(1, q1).cpu().numpy(), fr.residual(1, q1).cpu().numpy())
