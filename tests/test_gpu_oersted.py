"""GPU parity of the Oersted field (Sec. 4.5): the FFT convolution of a
current density with the cell-averaged Biot-Savart kernel (set up in
double-double from the antiderivative of Newell's f, singular current beyond
the near field), through the C ABI, against the oracle's direct sum; the
Oersted term in the effective field, the energy and an LLG integration."""
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


CASES = [((12, 10, 4), 20), ((33, 17, 5), 20), ((33, 17, 5), 2), ((20, 1, 3), 20),
         ((1, 9, 6), 20), ((16, 12, 1), 20), ((7, 1, 1), 20)]


def _current(grid, seed):
    nx, ny, nz = grid
    g = W.rng(seed)
    return g.standard_normal((3, nz, ny, nx)) * 1e11


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("grid,p", CASES)
def test_oersted_field_matches_oracle(torch_cuda, mm, orc, prec, grid, p):
    banner("oersted %s p=%d %s" % (grid, p, prec))
    d = (2e-9, 2.5e-9, 1.5e-9)
    j = _current(grid, 5)
    plan = mm.Plan(grid, d, Ms=8e5, A=1e-11, prec=prec, demag_p=p)
    o = orc.Oracle(grid, d, Ms=8e5, p=p)
    ref = o.oersted(j)
    got = to_np(plan.oersted(j))
    e = rel_l2(got, ref)
    print("  rel-L2 %.2e" % e)
    assert e <= TOL[prec], e
    # a second call reuses the kept kernel and gives the same result
    assert np.array_equal(to_np(plan.oersted(j)), got)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_oersted_term_and_energy(torch_cuda, mm, orc, prec):
    grid = (20, 14, 3)
    banner("oersted term %s %s" % (grid, prec))
    d = (2e-9, 2e-9, 2e-9)
    g = W.rng(8)
    Ms = g.uniform(4e5, 1.2e6, (3, 14, 20))
    Ms[g.uniform(size=Ms.shape) < 0.1] = 0.0
    j = _current(grid, 9)
    m = W.random_unit_sphere(grid, 10)
    H = np.array([1e4, 0, -2e4])
    f, t = 3e9, 0.11e-9
    plan = mm.Plan(grid, d, Ms=1.0, A=1.1e-11, prec=prec)
    plan.set_ms(Ms)
    plan.set_current(j, freq=f)
    o = orc.Oracle(grid, d, Ms=Ms, A=np.where(Ms > 0, 1.1e-11, 0.0))
    o.set_current(j, freq=f)
    o.set_field(H)
    mt = plan._t(m)
    for terms in (mm.MM_OERSTED, mm.MM_ALL):
        e = rel_l2(to_np(plan.heff(mt, H, terms, t)), o.heff(m, t, terms))
        print("  terms %d rel-L2 %.2e" % (terms, e))
        assert e <= TOL[prec], (terms, e)
    E, Er = plan.energy(mt, H, mm.MM_ALL, t), o.energy(m, t)
    assert abs(E[3] - Er[3]) <= (1e-12 if prec == "fp64" else 2e-5) * abs(Er[3])
    plan.set_current(None)
    assert np.abs(to_np(plan.heff(mt, H, mm.MM_OERSTED, t))).max() == 0.0


def test_oersted_llg_matches_oracle(torch_cuda, mm, orc):
    grid = (24, 16, 2)
    banner("oersted llg fp64 %s" % (grid,))
    d = (2.5e-9, 2.5e-9, 2e-9)
    # a current along x through a strip at the film's edge (an antenna)
    j = np.zeros((3, 2, 16, 24))
    j[0, :, 0:3, :] = 2e12
    m0 = W.smooth_random(grid, 3.0, seed=12)
    plan = mm.Plan(grid, d, Ms=8e5, A=1.3e-11, alpha=0.05, prec="fp64")
    plan.set_current(j, freq=5e9)
    o = orc.Oracle(grid, d, Ms=8e5, A=1.3e-11, alpha=0.05)
    o.set_current(j, freq=5e9)
    o.set_field((0, 0, 0))
    t_end = 2e-11
    ref, t, _, st_o, _ = o.dp45(m0, rtol=1e-8, t_end=t_end)
    m = plan._t(m0)
    status, tt, _, st = plan.llg_step(m, None, mm.MM_ALL, rtol=1e-8, t_end=t_end)
    assert status == mm.MM_OK and tt == t_end
    e = rel_l2(to_np(m), ref)
    print("  %d/%d steps (gpu/oracle), rel-L2 %.2e" % (st["accepted"], st_o["accepted"], e))
    assert e <= 1e-7


def test_oersted_rejected_for_layers(torch_cuda, mm):
    banner("oersted rejected for thin layers")
    plan = mm.Plan((8, 8, 2), (2e-9,) * 3, Ms=8e5, prec="fp64", layers=[1e-9, 2e-9])
    j = np.ones((3, 2, 8, 8))
    with pytest.raises(mm.MMError):
        plan.oersted(j)
    with pytest.raises(mm.MMError):
        plan.set_current(j)
