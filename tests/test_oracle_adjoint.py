"""Pins of the oracle's differentiation tools (inverse design, Sec. 5.2): the
transposed field operator and the LLG vector-Jacobian product against the
forward operators (dot-product identities), Ms-gradients and the RK4 discrete
adjoint against central finite differences, the 4th order of RK4, and the
inverse-design sign pattern |x| < sqrt(2)|y| of the stray-field objective."""
import math

import numpy as np
import pytest

from paper_2302_08843_amd import workloads as W

MU0 = 4e-7 * np.pi
GAMMA = 2.21e5


def _problem(orc, n=(6, 5, 2), seed=1, Ku=3e4, p=2):
    g = W.rng(seed)
    nz, ny, nx = n[2], n[1], n[0]
    Ms = g.uniform(4e5, 1e6, (nz, ny, nx))
    A = g.uniform(5e-12, 2e-11, (nz, ny, nx))
    o = orc.Oracle(n, (2e-9, 3e-9, 2.5e-9), Ms=Ms, A=A, Ku=Ku, eu=(0.0, 0.6, 0.8), alpha=0.3, p=p)
    o.set_field((1e4, -2e4, 3e4))
    return o, Ms, g


@pytest.mark.parametrize("term", ["DEMAG", "EXCH", "ANIS"])
def test_field_transpose_dot_product(orc, term):
    o, Ms, g = _problem(orc)
    mask = getattr(orc, term)
    v = g.standard_normal((3,) + o.shape)
    w = g.standard_normal((3,) + o.shape)
    Hv = o.heff(v, 0.0, mask)
    HTw, _ = o.heff_vjp(v, w, mask)
    lhs, rhs = (w * Hv).sum(), (HTw * v).sum()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("term", ["DEMAG", "EXCH", "ANIS"])
def test_field_ms_gradient_finite_difference(orc, term):
    o, Ms, g = _problem(orc)
    mask = getattr(orc, term)
    m = W.random_unit_sphere(o.n, 3)
    w = g.standard_normal((3,) + o.shape)
    _, gms = o.heff_vjp(m, w, mask)
    for cell in [(0, 0, 0), (1, 2, 3), (0, 4, 5)]:
        eps = 1e-6 * Ms[cell]
        vals = []
        for sgn in (1, -1):
            Mp = Ms.copy()
            Mp[cell] += sgn * eps
            o.set_Ms(Mp)
            vals.append((w * o.heff(m, 0.0, mask)).sum())
        o.set_Ms(Ms)
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(fd - gms[cell]) <= 1e-6 * (abs(gms[cell]) + 1e-3 * np.abs(gms).max())


def test_llg_jvp_against_finite_differences(orc):
    o, Ms, g = _problem(orc)
    m = W.random_unit_sphere(o.n, 4)
    v = g.standard_normal((3,) + o.shape)
    eps = 1e-6
    fd = (o.llg_rhs(m + eps * v, o.heff(m + eps * v)) - o.llg_rhs(m - eps * v, o.heff(m - eps * v))) / (2 * eps)
    jv = o.llg_jvp(m, v)
    assert np.linalg.norm(fd - jv) <= 1e-7 * np.linalg.norm(jv)


def test_llg_vjp_dot_product_with_jvp(orc):
    o, Ms, g = _problem(orc)
    m = W.random_unit_sphere(o.n, 5)
    v = g.standard_normal((3,) + o.shape)
    w = g.standard_normal((3,) + o.shape)
    jv = o.llg_jvp(m, v)
    jtw, _ = o.llg_vjp(m, w)
    lhs, rhs = (w * jv).sum(), (jtw * v).sum()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_llg_ms_gradient_finite_difference(orc):
    o, Ms, g = _problem(orc)
    m = W.random_unit_sphere(o.n, 6)
    w = g.standard_normal((3,) + o.shape)
    _, gms = o.llg_vjp(m, w)
    for cell in [(0, 1, 1), (1, 4, 0), (1, 0, 5)]:
        eps = 1e-6 * Ms[cell]
        vals = []
        for sgn in (1, -1):
            Mp = Ms.copy()
            Mp[cell] += sgn * eps
            o.set_Ms(Mp)
            vals.append((w * o.llg_rhs(m, o.heff(m))).sum())
        o.set_Ms(Ms)
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(fd - gms[cell]) <= 1e-6 * abs(gms[cell])


def test_rk4_fourth_order(orc):
    H, alpha, th0 = 1e5, 0.1, 1.0
    o = orc.Oracle((1, 1, 1), (2e-9,) * 3, Ms=8e5, alpha=alpha)
    o.set_field((0, 0, H), terms=orc.DEMAG | orc.ZEEMAN)
    m0 = np.array([np.sin(th0), 0.0, np.cos(th0)]).reshape(3, 1, 1, 1)
    gp = GAMMA / (1 + alpha ** 2)
    T = 200e-12
    th = 2 * np.arctan(np.tan(th0 / 2) * np.exp(-alpha * gp * H * T))
    ref = np.array([np.sin(th) * np.cos(gp * H * T), np.sin(th) * np.sin(gp * H * T), np.cos(th)])
    errs = []
    for n in (20, 40, 80):
        m, _ = o.rk4(m0, T / n, n, np.ones((1, 1, 1)))
        errs.append(np.abs(m.ravel() - ref).max())
    assert 13 < errs[0] / errs[1] < 19 and 13 < errs[1] / errs[2] < 19, errs


def _adjoint_case(orc, n=(20, 16, 1)):
    g = W.rng(11)
    nx, ny, nz = n
    rho = g.uniform(0.5, 1.0, (nz, ny, nx))
    Ms0 = 8e5
    o = orc.Oracle(n, (5e-9,) * 3, Ms=rho * Ms0, A=1.3e-11, alpha=0.05)
    o.set_field((0, 0, 0), terms=orc.DEMAG | orc.EXCH | orc.ZEEMAN)
    strip = np.zeros((nz, ny, nx), np.uint8)
    strip[:, :, 2:4] = 1
    o.set_drive((0.0, W.mT(20.0), 0.0), 20e9, strip)
    region = np.zeros((nz, ny, nx), np.uint8)
    region[:, 6:10, 14:18] = 1
    m0 = np.zeros((3, nz, ny, nx))
    m0[0] = 1.0
    return o, rho * Ms0, m0, region, g


def test_rk4_adjoint_against_finite_differences(orc):
    o, Ms, m0, region, g = _adjoint_case(orc)
    dt, n = 1e-13, 40
    loss, gms, gm0 = o.rk4_adjoint(m0, dt, n, region)
    assert abs(loss - o.rk4(m0, dt, n, region)[1]) <= 1e-15
    # a seeded direction in Ms
    d = g.standard_normal(Ms.shape)
    eps = 1e-4
    vals = []
    for sgn in (1, -1):
        o.set_Ms(Ms * (1 + sgn * eps * d))
        vals.append(o.rk4(m0, dt, n, region)[1])
    o.set_Ms(Ms)
    fd = (vals[0] - vals[1]) / (2 * eps)
    ad = (gms * Ms * d).sum()
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
    # single cells, including the drive strip and the loss region
    for cell in [(0, 8, 15), (0, 3, 2), (0, 12, 9), (0, 0, 0), (0, 7, 16), (0, 15, 19), (0, 5, 3), (0, 9, 12)]:
        h = 1e-4 * Ms[cell]
        vals = []
        for sgn in (1, -1):
            Mp = Ms.copy()
            Mp[cell] += sgn * h
            o.set_Ms(Mp)
            vals.append(o.rk4(m0, dt, n, region)[1])
        o.set_Ms(Ms)
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - gms[cell]) <= 1e-6 * abs(gms).max(), (cell, fd, gms[cell])
    # initial-state gradient along a direction
    v = g.standard_normal(m0.shape)
    e2 = 1e-6
    lp = o.rk4(m0 + e2 * v, dt, n, region)[1]
    lm = o.rk4(m0 - e2 * v, dt, n, region)[1]
    assert abs((lp - lm) / (2 * e2) - (gm0 * v).sum()) <= 1e-6 * abs((gm0 * v).sum())


def test_inverse_design_sign_pattern(orc):
    # maximise h_y at the cell (50, 0, 0) of a 101 x 51 x 1 film of 5 nm
    # cells, Ms = 1, m = y: the gradient dJ/dm_y is the demag transpose of a
    # one-hot y cotangent; away from the target its sign follows the dipole
    # rule |x| < sqrt(2) |y| (Sec. 5.2)
    n = (101, 51, 1)
    o = orc.Oracle(n, (5e-9,) * 3, Ms=1.0)
    m = np.zeros((3, 1, 51, 101))
    m[1] = 1.0
    w = np.zeros_like(m)
    w[1, 0, 0, 50] = 1.0
    g, _ = o.heff_vjp(m, w, orc.DEMAG)
    gy = g[1, 0]
    checked = 0
    for j in range(51):
        for i in range(101):
            dx, dy = abs(i - 50), j
            r = math.hypot(dx, dy)
            if r < 6 or abs(dx - math.sqrt(2) * dy) < 0.15 * r:
                continue
            expect = 1.0 if dx < math.sqrt(2) * dy else -1.0
            assert np.sign(gy[j, i]) == expect, (i, j, gy[j, i])
            checked += 1
    assert checked > 3000


def test_field_transpose_with_vacuum_cells(orc):
    # vacuum targets carry no field, so the transpose ignores their cotangent
    o, Ms, g = _problem(orc)
    Ms2 = Ms.copy()
    Ms2[0, 1, 2] = Ms2[1, 3, 4] = 0.0
    o.set_Ms(Ms2)
    v = g.standard_normal((3,) + o.shape)
    w = g.standard_normal((3,) + o.shape)
    for mask in (orc.DEMAG, orc.ANIS, orc.DEMAG | orc.ANIS):
        lhs = (w * o.heff(v, 0.0, mask)).sum()
        rhs = (o.heff_vjp(v, w, mask)[0] * v).sum()
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
