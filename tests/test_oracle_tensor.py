"""Pins of the oracle's demagnetisation kernel (Sec. 4.4: Newell near field,
point-dipole far field, Eq. dipole) against facts fixed by the mathematics:
the self term of a cube, trace identities, Aharoni's closed form for a
rectangular prism (J. Appl. Phys. 83, 3432 (1998)), the dipole limit and the
demag factors of a uniformly magnetised box."""
import mpmath as mp
import numpy as np
import pytest

mp.mp.dps = 40


def aharoni_dz(a, b, c):
    """Demag factor along c of a prism with semi-axes a, b, c (Aharoni 1998)."""
    a, b, c = mp.mpf(a), mp.mpf(b), mp.mpf(c)
    r = mp.sqrt(a * a + b * b + c * c)
    rab, rbc, rac = mp.sqrt(a * a + b * b), mp.sqrt(b * b + c * c), mp.sqrt(a * a + c * c)
    s = (b * b - c * c) / (2 * b * c) * mp.log((r - a) / (r + a))
    s += (a * a - c * c) / (2 * a * c) * mp.log((r - b) / (r + b))
    s += b / (2 * c) * mp.log((rab + a) / (rab - a))
    s += a / (2 * c) * mp.log((rab + b) / (rab - b))
    s += c / (2 * a) * mp.log((rbc - b) / (rbc + b))
    s += c / (2 * b) * mp.log((rac - a) / (rac + a))
    s += 2 * mp.atan(a * b / (c * r))
    s += (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
    s += (a * a + b * b - 2 * c * c) * r / (3 * a * b * c)
    s += c / (a * b) * (rac + rbc)
    s -= (rab ** 3 + rbc ** 3 + rac ** 3) / (3 * a * b * c)
    return s / mp.pi


def aharoni(a, b, c):
    """(Dx, Dy, Dz) of the prism with semi-axes a, b, c."""
    return (float(aharoni_dz(b, c, a)), float(aharoni_dz(c, a, b)), float(aharoni_dz(a, b, c)))


def test_aharoni_sum_rule():
    # pins the test's own closed form: the three factors of any prism sum to 1
    for abc in [(1, 1, 1), (1, 1, 0.5), (0.5, 1, 1.5), (3, 1, 0.2)]:
        assert abs(sum(aharoni(*abc)) - 1.0) < 1e-14
    assert abs(aharoni(1, 1, 1)[2] - 1.0 / 3.0) < 1e-15


def test_cube_self_term(orc):
    for d in (1.0, 2e-9, 5e-9):
        N = orc.newell((d, d, d), 0, 0, 0)
        assert np.allclose(N[:3], 1.0 / 3.0, rtol=0, atol=1e-15)
        assert np.allclose(N[3:], 0.0, atol=1e-15)
        K = orc.tensor_entry((d, d, d), 0, 0, 0, p=20)
        assert np.allclose(K[:3], -1.0 / 3.0, atol=1e-15)


@pytest.mark.parametrize("cell", [(2, 2, 1), (1, 2, 3), (3, 1, 1.5), (10, 10, 20), (4, 4, 1)])
def test_self_term_matches_aharoni(orc, cell):
    d = tuple(c * 1e-9 for c in cell)
    N = orc.newell(d, 0, 0, 0)
    D = aharoni(*(c / 2 for c in cell))
    assert np.allclose(N[:3], D, rtol=0, atol=2e-15), (N[:3], D)
    assert abs(N[:3].sum() - 1.0) < 2e-15


def test_trace_free_off_centre(orc):
    d = (2e-9, 3e-9, 1.5e-9)
    for off in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 1, 0), (5, 3, 1), (-3, 7, -2), (12, 0, 5)]:
        K = orc.tensor_entry(d, *off, p=20)
        # the kernel is dimensionless; long-double cancellation leaves ~1e-17
        assert abs(K[:3].sum()) < 1e-16, (off, K)
    # dipole part (beyond p) is trace free as well
    K = orc.tensor_entry(d, 25, 3, 1, p=20)
    assert abs(K[:3].sum()) < 1e-15 * np.abs(K).max()


def test_parity_and_symmetry(orc):
    d = (2e-9, 2.5e-9, 3e-9)
    for off in [(1, 2, 3), (4, 1, 2), (3, 5, 1), (22, 3, 2)]:
        I, J, K = off
        base = orc.tensor_entry(d, I, J, K)
        # diagonal components even in every axis
        for sx, sy, sz in [(-1, 1, 1), (1, -1, 1), (1, 1, -1), (-1, -1, -1)]:
            e = orc.tensor_entry(d, sx * I, sy * J, sz * K)
            assert np.allclose(e[:3], base[:3], rtol=1e-13, atol=0)
            # xy odd in x,y; xz odd in x,z; yz odd in y,z
            assert np.isclose(e[3], sx * sy * base[3], rtol=1e-13, atol=1e-30)
            assert np.isclose(e[4], sx * sz * base[4], rtol=1e-13, atol=1e-30)
            assert np.isclose(e[5], sy * sz * base[5], rtol=1e-13, atol=1e-30)


def test_newell_tends_to_dipole(orc):
    # For a cubic cell the relative Newell-dipole difference decays ~ r^-4
    # (the quadrupole correction vanishes by symmetry); along an axis the
    # ratio between 10 and 20 cells is close to 16.
    d = (1.0, 1.0, 1.0)
    rel = []
    for r in (10, 20):
        N = orc.newell(d, r, 0, 0)
        D = orc.dipole(d, r, 0, 0)
        rel.append(abs((N[0] + D[0]) / D[0]))
    assert 1e-5 < rel[0] < 1e-4
    assert 12.0 < rel[0] / rel[1] < 20.0
    # off-diagonal, off-axis offset: -N_xy close to the dipole value
    N = orc.newell(d, 10, 7, 3)
    D = orc.dipole(d, 10, 7, 3)
    assert abs((N[3] + D[3]) / D[3]) < 2e-5
    # far field switches to the dipole beyond p
    K = orc.tensor_entry(d, 21, 0, 0, p=20)
    assert np.allclose(K, orc.dipole(d, 21, 0, 0), rtol=0, atol=0)
    K = orc.tensor_entry(d, 20, 0, 0, p=20)
    assert np.allclose(K, -orc.newell(d, 20, 0, 0), rtol=0, atol=0)


@pytest.mark.parametrize("direct", [True, False])
def test_box_factors_all_newell(orc, direct):
    # With Newell everywhere the cell-averaged kernel is exact, so the mean
    # field of a uniformly magnetised box is -D Ms m with Aharoni's D.
    n = (8, 6, 3)
    d = (2e-9, 2e-9, 2e-9)
    o = orc.Oracle(n, d, Ms=1.0, p=-1, direct=direct)
    D = aharoni(n[0] * d[0] / 2, n[1] * d[1] / 2, n[2] * d[2] / 2)
    for a in range(3):
        m = np.zeros((3, n[2], n[1], n[0]))
        m[a] = 1.0
        h = o.demag(m)
        assert abs(h[a].mean() + D[a]) < 1e-13, (a, h[a].mean(), D[a])
        for b in range(3):
            if b != a:
                assert abs(h[b].mean()) < 1e-14


def test_uniform_cube_one_third(orc):
    # a cube of 4x4x4 cubic cells: body-averaged field = -Ms/3 exactly
    o = orc.Oracle((4, 4, 4), (1e-9,) * 3, Ms=1.0, p=-1)
    m = np.zeros((3, 4, 4, 4))
    m[2] = 1.0
    assert abs(o.demag(m)[2].mean() + 1.0 / 3.0) < 1e-14


def test_small_llg_box_with_dipole_far_field(orc):
    # 32x32x4 box of 2 nm cells, Newell within 20 cells, dipole beyond: the
    # far-field model error against Aharoni stays below 1e-5.
    n = (32, 32, 4)
    d = (2e-9,) * 3
    o = orc.Oracle(n, d, Ms=1.0, p=20)
    D = aharoni(32e-9, 32e-9, 4e-9)
    for a in range(3):
        m = np.zeros((3, 4, 32, 32))
        m[a] = 1.0
        dev = abs(-o.demag(m)[a].mean() - D[a])
        assert dev < 1e-5, (a, dev)


@pytest.mark.parametrize("p", [20, 2, -1])
def test_trace_invariant_field(orc, p):
    # sum_a h_a[m = e_a] = -Ms at every cell for any grid and any p (the kernel
    # is trace free off the centre and has trace -1 at the centre)
    n = (30, 5, 3)
    Ms = np.random.Generator(np.random.PCG64(5)).uniform(0.5, 2.0, (3, 5, 30))
    o = orc.Oracle(n, (1e-9, 2e-9, 1.5e-9), Ms=Ms, p=p)
    tot = np.zeros((3, 5, 30))
    for a in range(3):
        m = np.zeros((3, 3, 5, 30))
        m[a] = 1.0
        tot += o.demag(m)[a]
    assert np.abs(tot + Ms).max() < 1e-13 * Ms.max()
