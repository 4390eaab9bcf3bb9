"""A plan whose persistent buffers live in a caller-owned (torch) workspace
(mm_opts.workspace, sized by mm_plan_workspace_bytes) computes exactly what a
plan with its own allocations computes: the same kernels on the same data, so
fields and adaptive trajectories are bit-identical."""
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


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("grid", [(24, 18, 4), (33, 17, 1), (16, 1, 5)])
def test_workspace_plan_bit_identical(torch_cuda, mm, grid, prec):
    torch = torch_cuda
    banner("workspace %s %s" % (grid, prec))
    d = (2e-9, 2.5e-9, 3e-9)
    kw = dict(Ms=8e5, A=1.3e-11, Ku=3e4, alpha=0.5, prec=prec)
    H = np.array([2e4, -1e4, 5e3])
    code = mm.MM_FP32 if prec == "fp32" else mm.MM_FP64
    nbytes = mm.mm_plan_workspace_bytes(grid, code)
    ws = torch.full((nbytes,), 0xAB, dtype=torch.uint8, device="cuda")  # garbage on purpose
    a = mm.Plan(grid, d, **kw)
    b = mm.Plan(grid, d, workspace=ws, **kw)
    assert b.device_bytes() == nbytes
    m0 = W.random_unit_sphere(grid, 3)
    ha = a.heff(m0, H, mm.MM_ALL)
    hb = b.heff(m0, H, mm.MM_ALL)
    assert torch.equal(ha, hb)
    ma, mb = a._v(m0), b._v(m0)
    sa = a.llg_step(ma, H, mm.MM_ALL, rtol=1e-6, max_steps=15)
    sb = b.llg_step(mb, H, mm.MM_ALL, rtol=1e-6, max_steps=15)
    assert torch.equal(ma, mb) and sa == sb
    assert np.array_equal(a.energy(ma, H), b.energy(mb, H))
    b.close()
    del ws  # the workspace is the caller's: freeing it after the plan is fine
    torch.cuda.synchronize()


def test_workspace_rejected_when_small_or_misaligned(torch_cuda, mm):
    torch = torch_cuda
    grid, d = (20, 12, 3), (2e-9,) * 3
    nbytes = mm.mm_plan_workspace_bytes(grid, mm.MM_FP32)
    small = torch.empty((nbytes - 256,), dtype=torch.uint8, device="cuda")
    with pytest.raises(mm.MMError) as ei:
        mm.Plan(grid, d, Ms=8e5, prec="fp32", workspace=small)
    assert ei.value.status == mm.MM_EINVAL and "needed" in str(ei.value)
    big = torch.empty((nbytes + 1024,), dtype=torch.uint8, device="cuda")
    with pytest.raises(mm.MMError) as ei:
        mm.Plan(grid, d, Ms=8e5, prec="fp32", workspace=big[16:])
    assert ei.value.status == mm.MM_EINVAL and "aligned" in str(ei.value)
    with pytest.raises(mm.MMError) as ei:
        mm.Plan(grid, d, Ms=8e5, prec="fp32", workspace=big, layers=[1e-9, 2e-9, 1e-9])
    assert ei.value.status == mm.MM_EINVAL
