"""mm_energy_noalloc: the energies of mm_energy computed without any device
allocation (field buffer and reductions in the library's static scratch),
checked against mm_energy on the same plan and inputs, twice in a row with the
second input smaller, and against the plan's device bytes (unchanged by the
allocation-free call, grown by the first mm_energy)."""
import numpy as np
import pytest

from gpu_util import banner
from paper_2302_08843_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def mm():
    from paper_2302_08843_amd import mm as _mm

    _mm.lib()
    return _mm


def _case(mm, grid, prec, seed):
    d = (2e-9, 2.5e-9, 3e-9)
    plan = mm.Plan(grid, d, Ms=8e5, A=1.3e-11, Ku=4e4, alpha=0.5, prec=prec, ku_axis=(0.3, 0, 1),
                   Ku2=1e4, Kc1=2e4, kc_axes=((1, 1, 0), (0, 0, 1)))
    m = plan._v(W.random_unit_sphere(grid, seed))
    H = W.random_direction(seed + 1) * 2e4
    return plan, m, H


def test_noalloc_matches_mm_energy_twice_then_smaller(torch_cuda, mm):
    torch = torch_cuda
    runs = [((32, 24, 8), "fp64", 1), ((12, 10, 2), "fp32", 2)]
    plans = []
    for grid, prec, seed in runs:
        banner("energy_noalloc %s %s" % (grid, prec))
        plan, m, H = _case(mm, grid, prec, seed)
        before = plan.device_bytes()
        e_na = mm.mm_energy_noalloc(plan.handle, m, H, mm.MM_ALL, 0.0)
        torch.cuda.synchronize()
        assert plan.device_bytes() == before  # nothing allocated for the plan
        e_ref = plan.energy(m, H, mm.MM_ALL)
        assert plan.device_bytes() > before  # mm_energy allocates its work space
        # the same kernels and reduction order on the same inputs
        assert np.array_equal(e_na, e_ref), (grid, prec, e_na, e_ref)
        assert np.all(np.isfinite(e_na)) and e_na[0] != 0.0 and e_na[2] != 0.0
        plans.append((plan, m, H, e_ref))
    # the larger plan again after the smaller one: the scratch keeps the last
    # call's contents, which must not leak into the next result
    plan, m, H, e_ref = plans[0]
    for terms in (mm.MM_ALL, mm.MM_DEMAG | mm.MM_ZEEMAN):
        e_na = mm.mm_energy_noalloc(plan.handle, m, H, terms, 0.0)
        assert np.array_equal(e_na, plan.energy(m, H, terms))


def test_noalloc_rejects_plans_beyond_the_scratch(torch_cuda, mm):
    banner("energy_noalloc oversize")
    grid = (256, 256, 43)  # 2.82 M cells: 3N doubles exceed the 64 MiB scratch
    plan = mm.Plan(grid, (3e-9,) * 3, Ms=8e5, A=1.3e-11, prec="fp64")
    m = plan.empty()
    m.zero_()
    m[2] = 1.0
    with pytest.raises(mm.MMError) as ei:
        mm.mm_energy_noalloc(plan.handle, m, None, mm.MM_ALL, 0.0)
    assert ei.value.status == mm.MM_EINVAL and "maximum" in str(ei.value)
