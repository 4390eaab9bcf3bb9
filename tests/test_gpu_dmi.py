"""GPU parity of the extended exchange stencil: per-cell exchange constants
with the harmonic-mean coupling (Sec. 4.2) and DMI of the interface, bulk and
D_2d types with uniform or per-cell strength and the averaged coupling of
Eq. D_avg (Sec. 4.3), fused into the x inverse / local pass.  The HIP library
through the C ABI against the CPU oracle on the same seeded inputs; bars as
for the other fields (relative L2 1e-12 in FP64, 2e-5 in FP32)."""
import numpy as np
import pytest

from gpu_util import TOL, banner, rel_l2, to_np
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


def _materials(grid, seed, vacuum=True):
    g = W.rng(seed)
    nx, ny, nz = grid
    Ms = g.uniform(4e5, 1.2e6, (nz, ny, nx))
    if vacuum:
        Ms[g.uniform(size=Ms.shape) < 0.15] = 0.0
    A = np.where(Ms > 0, g.uniform(5e-12, 2.5e-11, Ms.shape), 0.0)
    return Ms, A, g


GRIDS = [(37, 21, 5), (64, 48, 3), (9, 1, 1), (1, 7, 6)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("grid", GRIDS)
def test_per_cell_exchange_matches_oracle(torch_cuda, mm, orc, prec, grid):
    banner("per-cell A %s %s" % (prec, grid))
    d = (2e-9, 2.5e-9, 3e-9)
    Ms, A, _ = _materials(grid, 61)
    m = W.random_unit_sphere(grid, 62)
    H = np.array([1e4, -2e4, 3e4])
    plan = mm.Plan(grid, d, Ms=1.0, A=1.3e-11, Ku=2e4, alpha=0.2, prec=prec,
                   ku_axis=(0.0, 0.6, 0.8))
    plan.set_ms(Ms)
    plan.set_exchange(A)
    o = orc.Oracle(grid, d, Ms=Ms, A=A, Ku=2e4, eu=(0.0, 0.6, 0.8), alpha=0.2)
    o.set_field(H)
    mt = plan._t(m)
    for terms in (mm.MM_EXCH, mm.MM_ALL):
        e = rel_l2(to_np(plan.heff(mt, H, terms)), o.heff(m, 0.0, terms))
        print("  terms %d rel-L2 %.2e" % (terms, e))
        assert e <= TOL[prec], (terms, e)
    E, Er = plan.energy(mt, H, mm.MM_ALL), o.energy(m)
    assert abs(E[1] - Er[1]) <= (1e-12 if prec == "fp64" else 2e-5) * abs(Er[1])
    # NULL restores the plan's uniform A
    plan.set_exchange(None)
    o2 = orc.Oracle(grid, d, Ms=Ms, A=np.where(Ms > 0, 1.3e-11, 0.0))
    e = rel_l2(to_np(plan.heff(mt, H, mm.MM_EXCH)), o2.exchange(m))
    assert e <= TOL[prec], e


DMI_CASES = [("interface", "uniform"), ("bulk", "uniform"), ("d2d", "uniform"),
             ("interface", "percell"), ("bulk", "percell"), ("d2d", "percell"),
             ("interface", "mixed_sign"), ("bulk", "mixed_sign")]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind,dmode", DMI_CASES)
def test_dmi_matches_oracle(torch_cuda, mm, orc, prec, kind, dmode):
    grid = (33, 17, 4)
    banner("dmi %s %s %s %s" % (kind, dmode, prec, grid))
    d = (2e-9, 1.5e-9, 1e-9)
    Ms, A, g = _materials(grid, 71)
    m = W.random_unit_sphere(grid, 72)
    code = {"interface": (mm.MM_DMI_INTERFACE, orc.DMI_INTERFACE),
            "bulk": (mm.MM_DMI_BULK, orc.DMI_BULK), "d2d": (mm.MM_DMI_D2D, orc.DMI_D2D)}[kind]
    if dmode == "uniform":
        D = 3.5e-3
    elif dmode == "percell":
        D = g.uniform(1e-3, 5e-3, Ms.shape)
    else:
        D = g.uniform(-4e-3, 4e-3, Ms.shape)
    H = np.array([2e4, 1e4, -3e4])
    plan = mm.Plan(grid, d, Ms=1.0, A=1.2e-11, Ku=1e4, alpha=0.2, prec=prec)
    plan.set_ms(Ms)
    plan.set_dmi(D, code[0])
    o = orc.Oracle(grid, d, Ms=Ms, A=np.where(Ms > 0, 1.2e-11, 0.0), Ku=1e4, alpha=0.2)
    o.set_dmi(D, code[1])
    o.set_field(H)
    mt = plan._t(m)
    for terms in (mm.MM_DMI, mm.MM_EXCH | mm.MM_DMI, mm.MM_ALL):
        e = rel_l2(to_np(plan.heff(mt, H, terms)), o.heff(m, 0.0, terms))
        print("  terms %d rel-L2 %.2e" % (terms, e))
        assert e <= TOL[prec], (terms, e)
    E, Er = plan.energy(mt, H, mm.MM_ALL), o.energy(m)
    print("  E_dmi %.6e vs %.6e, total %.6e vs %.6e" % (E[5], Er[5], E[4], Er[4]))
    tol = 1e-12 if prec == "fp64" else 2e-5
    assert abs(E[5] - Er[5]) <= tol * abs(Er[5])
    assert abs(E[4] - Er[4]) <= tol * np.abs(Er[:4]).sum() + tol * abs(Er[5])
    # removing the term
    plan.set_dmi(0.0, code[0])
    assert np.abs(to_np(plan.heff(mt, H, mm.MM_DMI))).max() == 0.0


def test_dmi_with_per_cell_exchange_llg_matches_oracle(torch_cuda, mm, orc):
    """Time integration (Dormand-Prince, FP64) of a film with interface DMI,
    per-cell A and per-cell D against the oracle's integrator."""
    grid = (24, 20, 2)
    banner("dmi + per-cell A llg fp64 %s" % (grid,))
    d = (2e-9, 2e-9, 1e-9)
    Ms, A, g = _materials(grid, 81, vacuum=False)
    D = g.uniform(2e-3, 4e-3, Ms.shape)
    m0 = W.smooth_random(grid, 3.0, seed=82)
    H = W.mT(30.0) * np.array([0.0, 0.0, 1.0])
    alpha, t_end = 0.2, 4e-11
    plan = mm.Plan(grid, d, Ms=1.0, A=1e-11, Ku=5e4, alpha=alpha, prec="fp64")
    plan.set_ms(Ms)
    plan.set_exchange(A)
    plan.set_dmi(D, mm.MM_DMI_INTERFACE)
    o = orc.Oracle(grid, d, Ms=Ms, A=A, Ku=5e4, alpha=alpha)
    o.set_dmi(D, orc.DMI_INTERFACE)
    o.set_field(H)
    ref, t, _, st_o, _ = o.dp45(m0, rtol=1e-8, t_end=t_end)
    m = plan._t(m0)
    status, tt, _, st = plan.llg_step(m, H, mm.MM_ALL, rtol=1e-8, t_end=t_end)
    assert status == mm.MM_OK and tt == t_end
    e = rel_l2(to_np(m), ref)
    print("  %d/%d steps (gpu/oracle), rel-L2 vs oracle %.2e" % (st["accepted"], st_o["accepted"], e))
    assert e <= 1e-7


def test_extended_stencil_rejected_by_differentiation(torch_cuda, mm):
    grid = (8, 8, 2)
    banner("extended stencil vjp rejection")
    plan = mm.Plan(grid, (2e-9,) * 3, Ms=8e5, A=1e-11, prec="fp64")
    m = plan._t(W.random_unit_sphere(grid, 91))
    plan.set_dmi(2e-3, mm.MM_DMI_BULK)
    with pytest.raises(mm.MMError):
        plan.heff_vjp(m, m, mm.MM_ALL)
    # without the DMI bit the transposed operator is still available
    plan.heff_vjp(m, m, mm.MM_ALL & ~mm.MM_DMI)
    plan.set_dmi(0.0, mm.MM_DMI_BULK)
    plan.set_exchange(np.full((2, 8, 8), 1e-11))
    with pytest.raises(mm.MMError):
        plan.heff_vjp(m, m, mm.MM_ALL)
    plan.set_exchange(None)
    plan.heff_vjp(m, m, mm.MM_ALL)
    with pytest.raises(mm.MMError):
        plan.set_dmi(1e-3, 7)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_per_cell_ku_matches_oracle(torch_cuda, mm, orc, prec):
    """Per-cell first-order uniaxial constant (both signs) with per-cell Ms
    and vacuum, alone and with every other term; the density-form energy."""
    grid = (29, 13, 4)
    banner("per-cell Ku %s %s" % (prec, grid))
    d = (2e-9, 2e-9, 3e-9)
    Ms, A, g = _materials(grid, 101)
    Ku = g.uniform(-3e4, 6e4, Ms.shape)
    eu = np.array([0.48, 0.6, 0.64])
    m = W.random_unit_sphere(grid, 102)
    H = np.array([1e4, -1e4, 2e4])
    plan = mm.Plan(grid, d, Ms=1.0, A=1.2e-11, Ku=1e4, alpha=0.2, prec=prec, ku_axis=eu,
                   Ku2=5e3)
    plan.set_ms(Ms)
    plan.set_ku(Ku)
    o = orc.Oracle(grid, d, Ms=Ms, A=np.where(Ms > 0, 1.2e-11, 0.0), Ku=1e4, eu=eu / np.linalg.norm(eu),
                   alpha=0.2)
    o.set_anisotropy2(Ku2=5e3)
    o.set_ku(Ku)
    o.set_field(H)
    mt = plan._t(m)
    for terms in (mm.MM_ANIS, mm.MM_ALL):
        e = rel_l2(to_np(plan.heff(mt, H, terms)), o.heff(m, 0.0, terms))
        print("  terms %d rel-L2 %.2e" % (terms, e))
        assert e <= TOL[prec], (terms, e)
    E, Er = plan.energy(mt, H, mm.MM_ALL), o.energy(m)
    assert abs(E[2] - Er[2]) <= (1e-12 if prec == "fp64" else 2e-5) * abs(Er[2])
    plan2 = mm.Plan(grid, d, Ms=8e5, A=1.2e-11, Ku=1e4, prec=prec, ku_axis=eu)
    plan2.set_ku(Ku)
    m2 = plan2._t(m)
    with pytest.raises(mm.MMError):
        plan2.heff_vjp(m2, m2, mm.MM_ALL)
    plan2.set_ku(None)
    plan2.heff_vjp(m2, m2, mm.MM_ALL)
