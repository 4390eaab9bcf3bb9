"""Pins of the oracle's thin-layer (non-equidistant) form of Sec. 4.4: the
cell-averaged tensor between cells of unequal height (equal-height limit,
additivity in the source, volume-weighted averaging over the target, the
trace identity for overlapping boxes, the dipole limit), the layered demag
field (equal layers reproduce the FFT convolution; mirror symmetries fix the
orientation of the unequal stencil), and the layered exchange and DMI
(textbook interlayer exchange energy, dE/dm = -mu0 V_k Ms h)."""
import numpy as np
import pytest

from paper_2302_08843_amd import workloads as W

MU0 = 4e-7 * np.pi


@pytest.mark.parametrize("I,J,K", [(0, 0, 0), (1, 0, 0), (0, 1, 1), (2, -1, 1), (-1, 3, -2),
                                   (4, 2, 3)])
def test_box_equal_height_limit(orc, I, J, K):
    dx, dy, dz = 2e-9, 3e-9, 1.5e-9
    ref = orc.newell((dx, dy, dz), I, J, K)
    got = orc.newell_box(dx, dy, I, J, K * dz, dz, dz)
    assert np.abs(got - ref).max() < 1e-12 * max(1e-3, np.abs(ref).max()), (got, ref)


@pytest.mark.parametrize("I,J,B", [(0, 0, 0.0), (1, 0, -1e-9), (0, 2, 2.5e-9), (3, -1, -4e-9)])
def test_box_additive_in_source(orc, I, J, B):
    # the field of a source of height c1 + c2 is the sum of the two stacked
    # sources' fields
    dx, dy, ct, c1, c2 = 2e-9, 2.5e-9, 1.2e-9, 0.7e-9, 1.6e-9
    whole = orc.newell_box(dx, dy, I, J, B, ct, c1 + c2)
    parts = orc.newell_box(dx, dy, I, J, B, ct, c1) + orc.newell_box(dx, dy, I, J, B + c1, ct, c2)
    assert np.abs(whole - parts).max() < 1e-12 * np.abs(whole).max()


@pytest.mark.parametrize("I,J,B", [(0, 0, 0.5e-9), (2, 1, -3e-9), (0, -1, 1.5e-9)])
def test_box_target_average(orc, I, J, B):
    # averaging over a target of height t1 + t2 is the height-weighted mean
    # of the averages over its two parts
    dx, dy, cs, t1, t2 = 2e-9, 2e-9, 1e-9, 0.8e-9, 1.7e-9
    whole = orc.newell_box(dx, dy, I, J, B, t1 + t2, cs)
    lower = orc.newell_box(dx, dy, I, J, B, t1, cs)
    upper = orc.newell_box(dx, dy, I, J, B - t1, t2, cs)
    mean = (t1 * lower + t2 * upper) / (t1 + t2)
    assert np.abs(whole - mean).max() < 1e-12 * np.abs(whole).max()


def test_box_trace_is_overlap_fraction(orc):
    # trace N = (volume of target & source) / (target volume): 1 for the
    # self term, cs/ct for a thinner source inside the target, 0 if disjoint
    dx, dy = 2e-9, 3e-9
    tr = lambda v: v[0] + v[1] + v[2]
    assert abs(tr(orc.newell_box(dx, dy, 0, 0, 0.0, 2e-9, 2e-9)) - 1.0) < 1e-14
    assert abs(tr(orc.newell_box(dx, dy, 0, 0, 0.5e-9, 2e-9, 0.6e-9)) - 0.3) < 1e-13
    assert abs(tr(orc.newell_box(dx, dy, 0, 0, 2e-9, 2e-9, 0.6e-9))) < 1e-13
    assert abs(tr(orc.newell_box(dx, dy, 1, 0, 0.0, 2e-9, 0.6e-9))) < 1e-13


def test_layer_entry_dipole_limit(orc):
    # far apart the near-field entry approaches the point dipole of the
    # source cell's moment at the centre offset
    dx, dy, dz = 2e-9, 2e-9, [1e-9, 3e-9]
    near = orc.layer_entry(dx, dy, dz, 0, 1, 25, 18, p=-1)
    far = orc.layer_entry(dx, dy, dz, 0, 1, 25, 18, p=0)
    assert np.abs(near - far).max() < 2e-3 * np.abs(far).max()


def _layered_problem(n, seed):
    g = W.rng(seed)
    nx, ny, nz = n
    m = W.random_unit_sphere(n, seed)
    Ms = g.uniform(4e5, 1.2e6, (nz, ny, nx))
    return m, Ms


def test_equal_layers_reproduce_fft_demag(orc):
    n, d = (7, 5, 4), (2e-9, 2.5e-9, 1.5e-9)
    m, Ms = _layered_problem(n, 3)
    o_eq = orc.Oracle(n, d, Ms=Ms, p=2)
    o_lay = orc.Oracle(n, d, Ms=Ms, p=2, layers=[d[2]] * n[2])
    ref = o_eq.demag(m)
    got = o_lay.demag(m)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("p", [20, 1])
def test_layered_demag_mirror_symmetries(orc, p):
    # reflecting the stack z -> -z (layers reversed, m_z negated) reflects the
    # field; the same for x -> -x.  Fixes the orientation of the unequal
    # stencil and of the odd components.
    n, d = (6, 4, 3), (2e-9, 2e-9, 1e-9)
    dz = [0.6e-9, 2.1e-9, 1.3e-9]
    m, Ms = _layered_problem(n, 5)
    h = orc.Oracle(n, d, Ms=Ms, p=p, layers=dz).demag(m)
    mz = m[:, ::-1].copy()
    mz[2] *= -1
    hz = orc.Oracle(n, d, Ms=Ms[::-1].copy(), p=p, layers=dz[::-1]).demag(mz)
    hz = hz[:, ::-1].copy()
    hz[2] *= -1
    assert np.abs(hz - h).max() < 1e-12 * np.abs(h).max()
    mx = m[:, :, :, ::-1].copy()
    mx[0] *= -1
    hx = orc.Oracle(n, d, Ms=Ms[:, :, ::-1].copy(), p=p, layers=dz).demag(mx)
    hx = hx[:, :, :, ::-1].copy()
    hx[0] *= -1
    assert np.abs(hx - h).max() < 1e-12 * np.abs(h).max()


def test_layered_demag_symmetric_in_volume_weighted_product(orc):
    # sum_t V_t Ms_t u_t . h(v)_t is symmetric in u, v (reciprocity of the
    # averaged tensor: V_t N^{ts} = V_s N^{st}^T)
    n, d = (5, 4, 3), (2e-9, 3e-9, 1e-9)
    dz = np.array([0.5e-9, 1.7e-9, 1.1e-9])
    g = W.rng(7)
    Ms = g.uniform(4e5, 1e6, (3, 4, 5))
    o = orc.Oracle(n, d, Ms=Ms, p=1, layers=dz)
    u = W.random_unit_sphere(n, 8)
    v = W.random_unit_sphere(n, 9)
    V = (d[0] * d[1] * dz)[:, None, None]
    lhs = (V * Ms * (u * o.demag(v)).sum(0)).sum()
    rhs = (V * Ms * (v * o.demag(u)).sum(0)).sum()
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_interlayer_exchange_energy_textbook(orc):
    # one column of layers: E_ex = A dx dy sum_k |m_{k+1} - m_k|^2 / delta_k
    # with delta_k the distance of the layer centres (A int |grad m|^2 with m
    # linear between the centres)
    n, d = (1, 1, 4), (3e-9, 2e-9, 1e-9)
    dz = np.array([0.8e-9, 2.0e-9, 1.1e-9, 0.5e-9])
    A = 1.3e-11
    o = orc.Oracle(n, d, Ms=8e5, A=A, layers=dz)
    o.set_field((0, 0, 0), terms=orc.EXCH)
    m = W.random_unit_sphere(n, 12)
    col = m[:, :, 0, 0]
    delta = 0.5 * (dz[1:] + dz[:-1])
    ref = A * d[0] * d[1] * (((col[:, 1:] - col[:, :-1]) ** 2).sum(0) / delta).sum()
    E = o.energy(m)
    assert abs(E[1] - ref) < 1e-13 * ref


@pytest.mark.parametrize("term", ["DEMAG", "EXCH", "DMI"])
def test_layered_energy_gradient(orc, term):
    # dE/dm_i = -mu0 V_k Ms_i h_i with the layer's own cell volume
    n, d = (3, 2, 3), (2e-9, 3e-9, 1e-9)
    dz = np.array([0.6e-9, 1.9e-9, 1.2e-9])
    g = W.rng(31)
    Ms = g.uniform(4e5, 1e6, (3, 2, 3))
    A = g.uniform(5e-12, 2e-11, (3, 2, 3))
    o = orc.Oracle(n, d, Ms=Ms, A=A, p=1, layers=dz)
    o.set_dmi(g.uniform(1e-3, 3e-3, (3, 2, 3)), orc.DMI_BULK)
    o.set_field((0, 0, 0), terms=getattr(orc, term))
    m = W.random_unit_sphere(n, 32) * 0.9
    h = o.heff(m)
    eps = 1e-6
    grad = np.zeros_like(m)
    for q in np.ndindex(m.shape):
        mp_, mm_ = m.copy(), m.copy()
        mp_[q] += eps
        mm_[q] -= eps
        grad[q] = (o.energy(mp_)[4] - o.energy(mm_)[4]) / (2 * eps)
    V = (d[0] * d[1] * dz)[None, :, None, None]
    expect = -MU0 * V * Ms[None] * h
    assert np.abs(grad - expect).max() < 1e-7 * np.abs(expect).max()


def test_equal_layers_reproduce_local_terms(orc):
    n, d = (5, 4, 3), (2e-9, 2e-9, 1.5e-9)
    m, Ms = _layered_problem(n, 41)
    A = 1.1e-11
    o_eq = orc.Oracle(n, d, Ms=Ms, A=A)
    o_lay = orc.Oracle(n, d, Ms=Ms, A=A, layers=[d[2]] * 3)
    for o in (o_eq, o_lay):
        o.set_dmi(2e-3, orc.DMI_BULK)
    assert np.abs(o_lay.exchange(m) - o_eq.exchange(m)).max() < 1e-12 * np.abs(o_eq.exchange(m)).max()
    assert np.abs(o_lay.dmi(m) - o_eq.dmi(m)).max() < 1e-12 * np.abs(o_eq.dmi(m)).max()
    E1, E2 = o_eq.energy(m), o_lay.energy(m)
    assert np.abs(E1 - E2).max() < 1e-12 * np.abs(E1).max()


def test_layer_demag_at_matches_full_sum(orc):
    n, d = (7, 6, 4), (2e-9, 2.5e-9, 1e-9)
    dz = [0.6e-9, 2.2e-9, 1.1e-9, 1.7e-9]
    m, Ms = _layered_problem(n, 61)
    for p in (1, 20):
        full = orc.Oracle(n, d, Ms=Ms, p=p, layers=dz).demag(m).reshape(3, -1).T
        at = orc.layer_demag_at(n, d, dz, m, np.arange(7 * 6 * 4), Ms=Ms, p=p)
        assert np.abs(at - full).max() <= 1e-13 * np.abs(full).max()


def test_no_demag_context_is_loud(orc):
    o = orc.Oracle((4, 3, 2), (2e-9,) * 3, Ms=8e5, A=1e-11, demag=False)
    m = W.random_unit_sphere((4, 3, 2), 3)
    assert np.isnan(o.demag(m)).all()
    ref = orc.Oracle((4, 3, 2), (2e-9,) * 3, Ms=8e5, A=1e-11).exchange(m)
    assert np.array_equal(o.exchange(m), ref)
