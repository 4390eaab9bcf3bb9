"""Pins of the oracle's local field terms (Sec. 4.1 anisotropy, Sec. 4.2
exchange, Zeeman) and of the energies (Sec. 4, Eq. linear_energy_discrete):
closed forms (spin spiral, uniform state, textbook energy densities), the
Ms-weighted symmetry of the exchange operator, and dE/dm = -mu0 V Ms h by
finite differences."""
import numpy as np
import pytest

from paper_2302_08843_amd import workloads as W

MU0 = 4e-7 * np.pi


def test_exchange_uniform_is_zero(orc):
    n = (7, 5, 3)
    o = orc.Oracle(n, (2e-9, 3e-9, 1e-9), Ms=8e5, A=1.3e-11)
    m = np.zeros((3, 3, 5, 7))
    m[:] = np.array([0.6, 0.0, 0.8])[:, None, None, None]
    assert np.abs(o.exchange(m)).max() == 0.0


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_exchange_spin_spiral_closed_form(orc, axis):
    # m = (cos q x, sin q x, 0) along one axis: interior h = (2A/(mu0 Ms))
    # (2 (cos(q D) - 1)/D^2) m, edge cell h = (2A/(mu0 Ms D^2)) (m_1 - m_0)
    n = [4, 4, 4]
    n[axis] = 24
    n = tuple(n)
    d = [2e-9, 3e-9, 2.5e-9]
    D = d[axis]
    Ms, A, q = 7e5, 1.1e-11, 0.3 / D
    o = orc.Oracle(n, d, Ms=Ms, A=A)
    coord = np.arange(n[axis]) * D
    shape = [1, 1, 1]
    shape[2 - axis] = n[axis]
    phase = np.broadcast_to((q * coord).reshape(shape), (n[2], n[1], n[0]))
    m = np.stack([np.cos(phase), np.sin(phase), np.zeros_like(phase)])
    h = o.exchange(m)
    pre = 2 * A / (MU0 * Ms)
    sl_int = [slice(None)] * 3
    sl_int[2 - axis] = slice(1, n[axis] - 1)
    expect = pre * 2 * (np.cos(q * D) - 1) / D ** 2 * m
    got = h[(slice(None),) + tuple(sl_int)]
    ref = expect[(slice(None),) + tuple(sl_int)]
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()
    sl0 = [slice(None)] * 3
    sl1 = [slice(None)] * 3
    sl0[2 - axis] = 0
    sl1[2 - axis] = 1
    edge = pre / D ** 2 * (m[(slice(None),) + tuple(sl1)] - m[(slice(None),) + tuple(sl0)])
    assert np.abs(h[(slice(None),) + tuple(sl0)] - edge).max() < 1e-13 * np.abs(edge).max()


def test_exchange_symmetric_in_ms_weighted_product(orc):
    n = (5, 4, 3)
    g = W.rng(3)
    Ms = g.uniform(3e5, 1e6, (3, 4, 5))
    A = g.uniform(5e-12, 2e-11, (3, 4, 5))
    o = orc.Oracle(n, (1e-9, 2e-9, 3e-9), Ms=Ms, A=A)
    u = W.random_unit_sphere(n, 4)
    v = W.random_unit_sphere(n, 5)
    lhs = (Ms * (u * o.exchange(v)).sum(0)).sum()
    rhs = (Ms * (v * o.exchange(u)).sum(0)).sum()
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_exchange_energy_textbook(orc):
    # homogeneous A: E_ex = A V sum_{neighbour pairs} |m_i - m_j|^2 / D^2
    n = (6, 5, 4)
    d = (2e-9, 3e-9, 2.5e-9)
    A = 1.3e-11
    o = orc.Oracle(n, d, Ms=8e5, A=A)
    o.set_field((0, 0, 0), terms=orc.EXCH)
    m = W.random_unit_sphere(n, 11)
    V = d[0] * d[1] * d[2]
    ref = 0.0
    for ax in range(3):
        diff = np.diff(m, axis=3 - ax)
        ref += A * V * (diff ** 2).sum() / d[ax] ** 2
    E = o.energy(m)
    assert abs(E[1] - ref) < 1e-12 * ref
    assert E[0] == 0.0 and E[2] == 0.0 and E[3] == 0.0


def test_anisotropy_and_zeeman_energy_textbook(orc):
    n = (4, 3, 2)
    d = (2e-9, 2e-9, 3e-9)
    g = W.rng(12)
    Ms = g.uniform(3e5, 1e6, (2, 3, 4))
    eu = np.array([1.0, 2.0, 2.0]) / 3.0
    Ku = 4.5e4
    H = np.array([1e4, -2e4, 5e3])
    o = orc.Oracle(n, d, Ms=Ms, Ku=Ku, eu=eu)
    o.set_field(H, terms=orc.ANIS | orc.ZEEMAN)
    m = W.random_unit_sphere(n, 13)
    V = d[0] * d[1] * d[2]
    em = np.einsum("a,a...->...", eu, m)
    E = o.energy(m)
    assert abs(E[2] - (-V * Ku * (em ** 2).sum())) < 1e-13 * abs(E[2])
    ez = -MU0 * V * (Ms * np.einsum("a,a...->...", H, m)).sum()
    assert abs(E[3] - ez) < 1e-13 * abs(ez)
    assert abs(E[4] - (E[2] + E[3])) < 1e-13 * abs(E[4])


def test_single_cube_demag_energy(orc):
    # one cubic cell: h = -Ms m / 3, E = mu0 V Ms^2 / 6
    d = 3e-9
    Ms = 8e5
    o = orc.Oracle((1, 1, 1), (d, d, d), Ms=Ms)
    o.set_field((0, 0, 0), terms=orc.DEMAG)
    m = np.array([0.36, 0.48, 0.8]).reshape(3, 1, 1, 1)
    assert np.allclose(o.demag(m), -Ms * m / 3, rtol=1e-15, atol=0)
    E = o.energy(m)
    assert abs(E[0] - MU0 * d ** 3 * Ms ** 2 / 6) < 1e-15 * E[0]


def test_vacuum_cells(orc):
    n = (6, 4, 2)
    Ms = np.full((2, 4, 6), 8e5)
    Ms[:, :, 3] = 0.0
    A = np.where(Ms > 0, 1.3e-11, 0.0)
    o = orc.Oracle(n, (2e-9,) * 3, Ms=Ms, A=A, Ku=1e4)
    o.set_field((1e3, 0, 0))
    m = W.random_unit_sphere(n, 9)
    h = o.heff(m)
    assert np.abs(h[:, :, :, 3]).max() == 0.0
    # the vacuum column decouples the two halves: exchange at x = 2 sees no
    # +x neighbour
    m2 = m.copy()
    m2[:, :, :, 4:] = W.random_unit_sphere(n, 10)[:, :, :, 4:]
    assert np.array_equal(o.exchange(m)[:, :, :, :3], o.exchange(m2)[:, :, :, :3])


@pytest.mark.parametrize("term", ["DEMAG", "EXCH", "ANIS", "ZEEMAN"])
def test_energy_gradient_is_minus_mu0_V_Ms_h(orc, term):
    # dE/dm_i = -mu0 V Ms_i h_i; pins the 1/2 of the linear terms, the
    # symmetry of the demag and exchange operators, and the Zeeman sign
    n = (3, 2, 2)
    d = (2e-9, 3e-9, 2.5e-9)
    g = W.rng(21)
    Ms = g.uniform(4e5, 1e6, (2, 2, 3))
    A = g.uniform(5e-12, 2e-11, (2, 2, 3))
    o = orc.Oracle(n, d, Ms=Ms, A=A, Ku=3e4, eu=(0.0, 0.6, 0.8), p=1)
    mask = getattr(orc, term)
    o.set_field((2e4, -1e4, 3e4), terms=mask)
    m = W.random_unit_sphere(n, 22) * 0.9
    V = d[0] * d[1] * d[2]
    h = o.heff(m)
    idx = np.argmax(np.isin(np.arange(5), [4]))  # total energy index
    eps = 1e-6
    grad = np.zeros_like(m)
    for q in np.ndindex(m.shape):
        mp_, mm_ = m.copy(), m.copy()
        mp_[q] += eps
        mm_[q] -= eps
        grad[q] = (o.energy(mp_)[idx] - o.energy(mm_)[idx]) / (2 * eps)
    expect = -MU0 * V * Ms[None] * h
    assert np.abs(grad - expect).max() < 1e-7 * np.abs(expect).max()


def _rotation(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 2] = -q[:, 2]
    return q


@pytest.mark.parametrize("which", ["Ku2", "Kc1", "Kc2", "all"])
def test_higher_anisotropy_energy_gradient(orc, which):
    """h = -(1 / (mu0 V Ms)) dE/dm for the second-order uniaxial and the cubic
    terms (central differences of the energy density sum; pins the factors 2
    and 4 and the signs of Sec. 4.3), with rotated cubic axes and per-cell Ms."""
    n, d = (4, 3, 2), (2e-9, 3e-9, 2.5e-9)
    g = np.random.default_rng(5)
    Ms = g.uniform(4e5, 1e6, (2, 3, 4))
    R = _rotation(3)
    k = dict(Ku2=3e4 if which in ("Ku2", "all") else 0.0, Kc1=-2e4 if which in ("Kc1", "all") else 0.0,
             Kc2=5e4 if which in ("Kc2", "all") else 0.0)
    o = orc.Oracle(n, d, Ms=Ms, Ku=1e4 if which == "all" else 0.0, eu=R[:, 2])
    o.set_anisotropy2(c1=R[:, 0], c2=R[:, 1], **k)
    o.set_field((0, 0, 0), terms=orc.ANIS)
    m = g.standard_normal((3, 2, 3, 4))
    h = o.anisotropy(m)
    V = np.prod(d)
    eps = 1e-6
    for idx in [(0, 0, 1, 2), (1, 1, 2, 3), (2, 0, 0, 0), (0, 1, 1, 1)]:
        mp, mm_ = m.copy(), m.copy()
        mp[idx] += eps
        mm_[idx] -= eps
        dE = (o.energy(mp)[2] - o.energy(mm_)[2]) / (2 * eps)
        expect = -MU0 * V * Ms[idx[1:]] * h[idx]
        assert abs(dE - expect) <= 1e-6 * abs(expect) + 1e-30, (idx, dE, expect)


def test_cubic_axes_and_covariance(orc):
    """Kc1 > 0: no field along a principal axis; Kc1 < 0: the body diagonal
    is a stationary point (field parallel to m); rotating the axes and m
    together rotates the field."""
    n, d = (1, 1, 1), (2e-9,) * 3
    R = _rotation(9)
    o = orc.Oracle(n, d, Ms=8e5)
    o.set_anisotropy2(Kc1=4e4, Kc2=1e4, c1=R[:, 0], c2=R[:, 1])
    h = o.anisotropy(R[:, 0].reshape(3, 1, 1, 1))
    assert np.abs(h).max() < 1e-9
    o.set_anisotropy2(Kc1=-4e4, Kc2=1e4, c1=R[:, 0], c2=R[:, 1])
    diag = (R[:, 0] + R[:, 1] + R[:, 2]) / np.sqrt(3)
    h = o.anisotropy(diag.reshape(3, 1, 1, 1)).ravel()
    assert np.linalg.norm(np.cross(diag, h)) < 1e-9 * np.linalg.norm(h)
    m = np.random.default_rng(2).standard_normal(3)
    o0 = orc.Oracle(n, d, Ms=8e5, Ku=2e4, eu=(0, 0, 1))
    o0.set_anisotropy2(Ku2=1e4, Kc1=3e4, Kc2=-2e4)
    o1 = orc.Oracle(n, d, Ms=8e5, Ku=2e4, eu=R[:, 2])
    o1.set_anisotropy2(Ku2=1e4, Kc1=3e4, Kc2=-2e4, c1=R[:, 0], c2=R[:, 1])
    h0 = o0.anisotropy(m.reshape(3, 1, 1, 1)).ravel()
    h1 = o1.anisotropy((R @ m).reshape(3, 1, 1, 1)).ravel()
    assert np.abs(h1 - R @ h0).max() <= 1e-12 * np.abs(h0).max()


def test_per_cell_uniaxial_constant(orc):
    """Per-cell Ku: the field and energy are the per-cell textbook forms
    h = 2 Ku_i/(mu0 Ms_i) e (e.m), E = -V sum Ku_i (e.m)^2; a uniform array
    equals the scalar; the energy gradient is -mu0 V Ms h."""
    n, d = (4, 3, 2), (2e-9, 2.5e-9, 3e-9)
    g = W.rng(71)
    Ms = g.uniform(4e5, 1e6, (2, 3, 4))
    Ku = g.uniform(-2e4, 5e4, (2, 3, 4))
    eu = np.array([2.0, 1.0, 2.0]) / 3.0
    o = orc.Oracle(n, d, Ms=Ms, Ku=1e4, eu=eu)
    o.set_ku(Ku)
    o.set_field((0, 0, 0), terms=orc.ANIS)
    m = W.random_unit_sphere(n, 72) * 0.9
    em = np.einsum("a,a...->...", eu, m)
    h = o.anisotropy(m)
    assert np.allclose(h, 2 * Ku / (MU0 * Ms) * em * eu[:, None, None, None], rtol=1e-14, atol=0)
    V = d[0] * d[1] * d[2]
    E = o.energy(m)
    assert abs(E[2] - (-V * (Ku * em ** 2).sum())) < 1e-13 * abs(E[2])
    eps = 1e-6
    grad = np.zeros_like(m)
    for q in np.ndindex(m.shape):
        mp_, mm_ = m.copy(), m.copy()
        mp_[q] += eps
        mm_[q] -= eps
        grad[q] = (o.energy(mp_)[4] - o.energy(mm_)[4]) / (2 * eps)
    assert np.abs(grad + MU0 * V * Ms[None] * h).max() < 1e-7 * np.abs(MU0 * V * Ms * h).max()
    o.set_ku(np.full((2, 3, 4), 3e4))
    ref = orc.Oracle(n, d, Ms=Ms, Ku=3e4, eu=eu).anisotropy(m)
    assert np.array_equal(o.anisotropy(m), ref)
