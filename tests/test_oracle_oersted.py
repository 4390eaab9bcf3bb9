"""Pins of the oracle's Oersted field (Sec. 4.5): the cell-averaged
Biot-Savart kernel G (h_t = sum_s j_s x G(X_t - X_s)) against the point
(singular) current at distance with the r^-2 approach, its antisymmetry and
vanishing self term, refinement consistency (the kernel of a cell twice as
long equals the averaged sum over its halves), the field of a finite straight
wire, and the Oersted term in the effective field and the Zeeman energy."""
import numpy as np
import pytest

from paper_2302_08843_amd import workloads as W

MU0 = 4e-7 * np.pi


def _point(d, I, J, K):
    D = np.array([I, J, K]) * np.array(d)
    return np.prod(d) / (4 * np.pi) * D / np.linalg.norm(D) ** 3


def test_point_current_limit(orc):
    d = (2e-9, 2.6e-9, 1.6e-9)
    errs = []
    for k in (1, 2, 4, 8):
        I, J, K = 3 * k, -2 * k, 1 * k
        g = orc.oersted_entry(d, I, J, K, p=-1)
        pt = _point(d, I, J, K)
        errs.append(np.abs(g - pt).max() / np.abs(pt).max())
    # O((cell / r)^2) approach: doubling the distance divides the error by ~4
    for a, b in zip(errs, errs[1:]):
        assert 3.0 < a / b < 5.0, errs
    assert errs[-1] < 5e-4
    # far field entries are the point current exactly
    assert np.allclose(orc.oersted_entry(d, 30, 1, 2, p=20), _point(d, 30, 1, 2), rtol=1e-15)


@pytest.mark.parametrize("I,J,K", [(1, 0, 0), (0, 1, 1), (2, -1, 3), (-1, -1, 1), (5, 2, -4)])
def test_antisymmetry_and_self(orc, I, J, K):
    d = (1e-9, 2e-9, 1.5e-9)
    g = orc.oersted_entry(d, I, J, K)
    # (to the long-double cancellation of the stencil, ~1e-15 at 5 cells)
    assert np.abs(g + orc.oersted_entry(d, -I, -J, -K)).max() <= 1e-13 * np.abs(g).max()
    # a component is odd along its own axis and even along the others
    gm = orc.oersted_entry(d, -I, J, K)
    assert abs(gm[0] + g[0]) <= 1e-13 * abs(g).max() and abs(gm[1] - g[1]) <= 1e-13 * abs(g).max()
    assert np.abs(orc.oersted_entry(d, 0, 0, 0)).max() < 1e-20


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("off", [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 1), (2, -1, 1), (3, 2, -2)])
def test_refinement_consistency(orc, axis, off):
    # a cell twice as long along `axis`: average over the two target halves
    # of the sum over the two source halves
    fine = [2e-9, 1.5e-9, 1e-9]
    coarse = list(fine)
    coarse[axis] *= 2
    gc = orc.oersted_entry(coarse, *off, p=-1)
    acc = np.zeros(3)
    for shift, w in ((-1, 1.0), (0, 2.0), (1, 1.0)):
        o = list(off)
        o[axis] = 2 * off[axis] + shift
        acc += w * orc.oersted_entry(fine, *o, p=-1)
    assert np.abs(gc - 0.5 * acc).max() < 1e-12 * max(np.abs(gc).max(), 1e-30) + 1e-25


def test_finite_straight_wire(orc):
    # one column of cells along z carrying j_z: away from the wire the field
    # approaches h_phi = I/(4 pi r) (sin th2 - sin th1) of a line current
    # the square cross-section and the cell averaging change a 2-D harmonic
    # field only at 4th order in cell / r, so within 1e-4 of the line current
    # already 5 cells away, with the cell-averaged kernel everywhere (p < 0)
    # and with the singular current beyond p = 20
    nx, nz = 41, 61
    d = (2e-9, 2e-9, 2e-9)
    j = np.zeros((3, nz, 1, nx))
    jz = 1e11
    j[2, :, 0, 0] = jz
    Icur = jz * d[0] * d[1]
    kc = nz // 2
    L1, L2 = -(kc + 0.5) * d[2], (nz - kc - 0.5) * d[2]
    for p in (-1, 20):
        h = orc.Oracle((nx, 1, nz), d, Ms=8e5, p=p).oersted(j)
        errs = []
        for i in (5, 10, 20):
            r = i * d[0]
            ref = Icur / (4 * np.pi * r) * (L2 / np.hypot(r, L2) - L1 / np.hypot(r, L1))
            assert abs(h[0, kc, 0, i]) < 1e-9 * ref and abs(h[2, kc, 0, i]) < 1e-9 * ref
            errs.append(abs(h[1, kc, 0, i] - ref) / ref)
        assert max(errs) < 1e-4, errs


def test_oersted_term_and_energy(orc):
    n, d = (5, 4, 3), (2e-9, 2.5e-9, 3e-9)
    g = W.rng(3)
    Ms = g.uniform(4e5, 1e6, (3, 4, 5))
    Ms[1, 2, 3] = 0.0
    j = g.standard_normal((3, 3, 4, 5)) * 1e11
    o = orc.Oracle(n, d, Ms=Ms, p=2)
    h_oe = o.oersted(j)
    f = 2e9
    o.set_current(j, freq=f)
    o.set_field((0, 0, 0), terms=orc.OERSTED)
    m = W.random_unit_sphere(n, 4)
    t = 0.13e-9
    s = np.sin(2 * np.pi * f * t)
    h = o.heff(m, t)
    assert np.allclose(h, s * h_oe * (Ms > 0)[None], rtol=1e-14, atol=0)
    # an applied field: E = -mu0 V sum Ms m . h, in the Zeeman slot
    V = d[0] * d[1] * d[2]
    E = o.energy(m, t)
    ref = -MU0 * V * (Ms[None] * m * h).sum()
    assert abs(E[3] - ref) < 1e-13 * abs(ref) and E[4] == E[3]
    o.set_current(None)
    assert np.abs(o.heff(m, t)).max() == 0.0


def test_oersted_at_matches_full_sum(orc):
    # the sampled direct sum (near table + singular current) equals the
    # full oracle field at every cell
    n, d = (9, 7, 5), (2e-9, 1.5e-9, 2.5e-9)
    j = W.rng(13).standard_normal((3, 5, 7, 9)) * 1e11
    for p in (2, 20):
        full = orc.Oracle(n, d, Ms=8e5, p=p).oersted(j).reshape(3, -1).T
        cells = np.arange(9 * 7 * 5)
        at = orc.oersted_at(n, d, j, cells, p=p)
        assert np.abs(at - full).max() <= 1e-13 * np.abs(full).max()
