"""Pins of the oracle's DMI term (Sec. 4.3, table of DMI types, Eq. D_avg)
and of per-cell exchange constants (Sec. 4.2): spiral and helix closed forms
of the central-difference stencil for each DMI type, derived from the DMI
vectors (e^dmi_x, e^dmi_y, e^dmi_z) and e^dmi_{-k} = -e^dmi_k; the edge cells
that ignore their missing neighbour; the equal-sign coupling average from a
two-cell chain; the Ms-weighted symmetry of the operator; dE/dm = -mu0 V Ms h;
and the continuum limit of the interface term, whose continuous form is
grad(m_z) - (div m) e_z."""
import numpy as np
import pytest

from paper_2302_08843_amd import workloads as W

MU0 = 4e-7 * np.pi


def _spiral(n, d, axis, q, comps):
    """m = cos(q s) e_a + sin(q s) e_b along grid axis `axis` (s = cell
    coordinate), comps = (a, b); returns m and the per-cell phase."""
    shape = [1, 1, 1]
    shape[2 - axis] = n[axis]
    phase = np.broadcast_to((q * np.arange(n[axis]) * d[axis]).reshape(shape),
                            (n[2], n[1], n[0]))
    m = np.zeros((3,) + phase.shape)
    m[comps[0]] = np.cos(phase)
    m[comps[1]] = np.sin(phase)
    return m


# (type, axis, components (a, b), sign s): interior h = s (2D/(mu0 Ms))
# (sin(q D)/D) m.  Each follows from sum_k e^dmi_k x (m_{i+k} - m_{i-k})/(2D):
#   interface (e_y, -e_x, 0):  x: e_y x (-sin, 0, cos) = (cos, 0, sin)   -> +1
#                              y: -e_x x (0, -sin, cos) = (0, cos, sin)  -> +1
#   bulk (e_x, e_y, e_z):      z: e_z x (-sin, cos, 0) = -(cos, sin, 0)  -> -1
#                              x: e_x x (0, -sin, cos) = -(0, cos, sin)  -> -1
#                              y: e_y x (cos-part)     = -(sin-, ...)    -> -1
#   D2d (-e_x, e_y, 0):        x: -e_x x (0, -sin, cos) = (0, cos, sin)  -> +1
#                              y: e_y x (-sin, 0, cos) = (cos, 0, sin)   -> +1
CASES = [
    ("DMI_INTERFACE", 0, (0, 2), +1),
    ("DMI_INTERFACE", 1, (1, 2), +1),
    ("DMI_BULK", 2, (0, 1), -1),
    ("DMI_BULK", 0, (1, 2), -1),
    ("DMI_BULK", 1, (2, 0), -1),
    ("DMI_D2D", 0, (1, 2), +1),
    ("DMI_D2D", 1, (0, 2), +1),
]


@pytest.mark.parametrize("kind,axis,comps,sign", CASES)
def test_dmi_spiral_closed_form(orc, kind, axis, comps, sign):
    # a one-dimensional chain along `axis` (single cells across, so no other
    # neighbours exist)
    n = [1, 1, 1]
    n[axis] = 20
    n = tuple(n)
    d = [2e-9, 3e-9, 2.5e-9]
    D, Ms = 3e-3, 6e5
    q = 0.4 / d[axis]
    o = orc.Oracle(n, d, Ms=Ms)
    o.set_dmi(D, getattr(orc, kind))
    m = _spiral(n, d, axis, q, comps)
    h = o.dmi(m).reshape(3, -1)
    m = m.reshape(3, -1)
    pre = 2 * D / (MU0 * Ms)
    expect = sign * pre * np.sin(q * d[axis]) / d[axis] * m
    assert np.abs(h[:, 1:-1] - expect[:, 1:-1]).max() < 1e-12 * pre / d[axis]
    # the end cells ignore their missing neighbour: h_0 = pre (e_k x m_1)/(2D)
    # with m_1 perpendicular to e_k, so |h_0| = pre / (2D)
    assert np.allclose(np.linalg.norm(h[:, 0]), pre / (2 * d[axis]), rtol=1e-13)
    assert np.allclose(np.linalg.norm(h[:, -1]), pre / (2 * d[axis]), rtol=1e-13)
    # linearity: cell 1's field is the sum of the contributions of m_0 and
    # m_2 alone, each of magnitude pre / (2D)
    m2 = np.zeros_like(m)
    m2[:, 2] = m[:, 2]
    h_plus = o.dmi(m2.reshape((3,) + o.shape)).reshape(3, -1)[:, 1]
    m0 = np.zeros_like(m)
    m0[:, 0] = m[:, 0]
    h_minus = o.dmi(m0.reshape((3,) + o.shape)).reshape(3, -1)[:, 1]
    assert np.allclose(h_plus + h_minus, h[:, 1], rtol=1e-14, atol=1e-9)
    assert np.allclose(np.linalg.norm(h_plus), pre / (2 * d[axis]), rtol=1e-13)


def test_dmi_two_cell_coupling_average(orc):
    # two cells along x, interface type: h_0 = (2/(mu0 Ms_0)) D~ (e_y x m_1)/(2 dx),
    # h_1 = (2/(mu0 Ms_1)) D~ (-e_y x m_0)/(2 dx), D~ the equal-sign average
    d = (2e-9, 2e-9, 2e-9)
    Ms = np.array([[[6e5, 9e5]]])
    D = np.array([[[1e-3, 3e-3]]])
    o = orc.Oracle((2, 1, 1), d, Ms=Ms)
    o.set_dmi(D, orc.DMI_INTERFACE)
    m = np.array([0.6, 0.0, 0.8, 0.0, 0.28, 0.96]).reshape(2, 3).T.reshape(3, 1, 1, 2)
    h = o.dmi(m)
    Dt = 2 * 1e-3 * 3e-3 / (1e-3 + 3e-3)  # 1.5e-3
    ey = np.array([0.0, 1.0, 0.0])
    h0 = 2 / (MU0 * 6e5) * Dt * np.cross(ey, m[:, 0, 0, 1]) / (2 * d[0])
    h1 = 2 / (MU0 * 9e5) * Dt * np.cross(-ey, m[:, 0, 0, 0]) / (2 * d[0])
    assert np.allclose(h[:, 0, 0, 0], h0, rtol=1e-14, atol=0)
    assert np.allclose(h[:, 0, 0, 1], h1, rtol=1e-14, atol=0)
    # a zero on one side switches the coupling off; equal values give D
    o.set_dmi(np.array([[[0.0, 3e-3]]]), orc.DMI_INTERFACE)
    assert np.abs(o.dmi(m)).max() == 0.0
    o.set_dmi(2e-3, orc.DMI_INTERFACE)
    h = o.dmi(m)
    assert np.allclose(h[:, 0, 0, 0], h0 * 2e-3 / Dt, rtol=1e-14, atol=0)


def test_dmi_opposite_sign_average_bounds(orc):
    # parity unpinned branch (opposite signs): only checked to be symmetric
    # in the two cells, to act as one scalar coupling, to take the printed
    # value, and to lie between -max|D| and 0
    d = (2e-9,) * 3
    m = W.random_unit_sphere((2, 1, 1), 5)
    Ds = [(2e-3, -1e-3), (-1e-3, 2e-3)]
    hs = []
    for pair in Ds:
        o = orc.Oracle((2, 1, 1), d, Ms=8e5)
        o.set_dmi(np.array(pair).reshape(1, 1, 2), orc.DMI_INTERFACE)
        hs.append(o.dmi(m))
    assert np.array_equal(hs[0], hs[1])
    o = orc.Oracle((2, 1, 1), d, Ms=8e5)
    o.set_dmi(1.0, orc.DMI_INTERFACE)
    unit = o.dmi(m)  # D~ = 1
    ratio = hs[0][np.abs(unit) > 0] / unit[np.abs(unit) > 0]
    assert np.allclose(ratio, ratio[0], rtol=1e-12)
    expect = -np.sqrt(np.sqrt(2e-3 * 1e-3) * abs(2e-3 - 1e-3) / 2)
    assert abs(ratio[0] - expect) < 1e-12 * abs(expect)
    assert -2e-3 < ratio[0] < 0


@pytest.mark.parametrize("kind", ["DMI_INTERFACE", "DMI_BULK", "DMI_D2D"])
def test_dmi_symmetric_in_ms_weighted_product(orc, kind):
    n = (5, 4, 3)
    g = W.rng(31)
    Ms = g.uniform(3e5, 1e6, (3, 4, 5))
    Ms[1, 2, 3] = 0.0
    D = g.uniform(-4e-3, 4e-3, (3, 4, 5))
    o = orc.Oracle(n, (1e-9, 2e-9, 3e-9), Ms=Ms)
    o.set_dmi(D, getattr(orc, kind))
    u = W.random_unit_sphere(n, 32)
    v = W.random_unit_sphere(n, 33)
    lhs = (Ms * (u * o.dmi(v)).sum(0)).sum()
    rhs = (Ms * (v * o.dmi(u)).sum(0)).sum()
    assert abs(lhs - rhs) < 1e-12 * np.abs(Ms * (u * o.dmi(v)).sum(0)).sum()


@pytest.mark.parametrize("kind", ["DMI_INTERFACE", "DMI_BULK", "DMI_D2D"])
def test_dmi_energy_gradient(orc, kind):
    # h = -(1/(mu0 V Ms)) dE/dm with E the DMI energy slot and the total
    n = (3, 3, 2)
    d = (2e-9, 3e-9, 2.5e-9)
    g = W.rng(41)
    Ms = g.uniform(4e5, 1e6, (2, 3, 3))
    D = g.uniform(1e-3, 4e-3, (2, 3, 3))
    o = orc.Oracle(n, d, Ms=Ms)
    o.set_dmi(D, getattr(orc, kind))
    o.set_field((0, 0, 0), terms=orc.DMI)
    m = W.random_unit_sphere(n, 42) * 0.9
    V = d[0] * d[1] * d[2]
    h = o.heff(m)
    assert np.array_equal(h, o.dmi(m))
    eps = 1e-6
    grad = np.zeros_like(m)
    for q in np.ndindex(m.shape):
        mp_, mm_ = m.copy(), m.copy()
        mp_[q] += eps
        mm_[q] -= eps
        grad[q] = (o.energy(mp_)[5] - o.energy(mm_)[5]) / (2 * eps)
    expect = -MU0 * V * Ms[None] * h
    assert np.abs(grad - expect).max() < 1e-7 * np.abs(expect).max()
    E = o.energy(m)
    assert E[4] == E[5] and E[0] == E[1] == E[2] == E[3] == 0.0


def test_interface_dmi_continuum_limit(orc):
    # smooth m on a fine grid: the stencil approaches (2D/(mu0 Ms))
    # (d_x m_z, d_y m_z, -d_x m_x - d_y m_y) with second-order error
    errs = []
    for nn in (16, 32):
        L = 40e-9
        dx = L / nn
        n = (nn, nn, 1)
        o = orc.Oracle(n, (dx, dx, 1e-9), Ms=8e5)
        D = 2e-3
        o.set_dmi(D, orc.DMI_INTERFACE)
        x = (np.arange(nn) * dx)[None, :]
        y = (np.arange(nn) * dx)[:, None]
        th = 0.7 * np.sin(2 * np.pi * x / L) * np.cos(np.pi * y / L) + 0.3
        ph = 2 * np.pi * y / L + np.pi * x / L
        mx, my, mz = np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)
        m = np.stack([mx, my, mz])[:, None]
        h = o.dmi(m)[:, 0]
        # analytic derivatives of the same functions
        dth_x = 0.7 * 2 * np.pi / L * np.cos(2 * np.pi * x / L) * np.cos(np.pi * y / L)
        dth_y = -0.7 * np.pi / L * np.sin(2 * np.pi * x / L) * np.sin(np.pi * y / L)
        dph_x, dph_y = np.pi / L, 2 * np.pi / L
        c, s = np.cos(th), np.sin(th)
        dmx_x = c * np.cos(ph) * dth_x - s * np.sin(ph) * dph_x
        dmy_y = c * np.sin(ph) * dth_y + s * np.cos(ph) * dph_y
        dmz_x, dmz_y = -s * dth_x, -s * dth_y
        pre = 2 * D / (MU0 * 8e5)
        ref = pre * np.stack([dmz_x + 0 * y, dmz_y + 0 * x, -dmx_x - dmy_y])
        inner = (slice(None), slice(2, -2), slice(2, -2))
        errs.append(np.abs(h[inner] - ref[inner]).max() / np.abs(ref[inner]).max())
    assert errs[1] < 0.3 * errs[0] and errs[1] < 0.02


def test_dmi_off_and_vacuum(orc):
    n = (6, 4, 2)
    Ms = np.full((2, 4, 6), 8e5)
    Ms[:, :, 3] = 0.0
    o = orc.Oracle(n, (2e-9,) * 3, Ms=Ms)
    m = W.random_unit_sphere(n, 51)
    assert np.abs(o.dmi(m)).max() == 0.0  # no D set
    o.set_dmi(3e-3, orc.DMI_BULK)
    h = o.dmi(m)
    assert np.abs(h[:, :, :, 3]).max() == 0.0
    # the vacuum column decouples the halves
    m2 = m.copy()
    m2[:, :, :, 4:] = W.random_unit_sphere(n, 52)[:, :, :, 4:]
    assert np.array_equal(o.dmi(m)[:, :, :, :3], o.dmi(m2)[:, :, :, :3])
    o.set_dmi(None)
    assert np.abs(o.dmi(m)).max() == 0.0


def test_per_cell_exchange_two_cell_series_coupling(orc):
    # two cells of exchange A0, A1: the coupling is that of the two half
    # cells in series, 1 / (dx/(2 A0) + dx/(2 A1)) per dx, i.e. the field on
    # cell 0 is (2/(mu0 Ms)) (2/dx^2) A0 A1/(A0 + A1) (m_1 - m_0)
    d = (2e-9, 3e-9, 3e-9)
    A0, A1, Ms = 1e-11, 3e-11, 8e5
    o = orc.Oracle((2, 1, 1), d, Ms=Ms, A=np.array([[[A0, A1]]]))
    m = np.array([0.6, 0.0, 0.8, 0.0, 0.28, 0.96]).reshape(2, 3).T.reshape(3, 1, 1, 2)
    h = o.exchange(m)
    series = 1.0 / (d[0] / (2 * A0) + d[0] / (2 * A1))  # per unit length: A~/dx
    expect = 2 / (MU0 * Ms) * (series / d[0]) * (m[:, 0, 0, 1] - m[:, 0, 0, 0])
    assert np.allclose(h[:, 0, 0, 0], expect, rtol=1e-14, atol=0)
