"""Pins of the oracle's LLG right-hand side (Sec. 3, Eq. llg), its
Dormand-Prince integrator and the relaxation (Sec. 3): macrospin Larmor
precession and damped switching in closed form, the 5th order of the
propagated solution, the energy identities dE/dt = -mu0 V sum Ms
(alpha gamma/(1+alpha^2)) |m x h|^2 and energy conservation at alpha = 0,
|m| preservation, and the Stoner-Wohlfarth angle."""
import math

import numpy as np
import pytest

from paper_2302_08843_amd import workloads as W

MU0 = 4e-7 * np.pi
GAMMA = 2.21e5


def cell_vec(v):
    return np.asarray(v, float).reshape(3, 1, 1, 1)


def test_rhs_orthogonal_to_m(orc):
    n = (5, 4, 2)
    o = orc.Oracle(n, (2e-9,) * 3, Ms=8e5, alpha=0.3)
    m = W.random_unit_sphere(n, 1)
    h = W.random_unit_sphere(n, 2) * 1e5
    for precess in (True, False):
        dm = o.llg_rhs(m, h, precess=precess)
        assert np.abs((m * dm).sum(0)).max() < 1e-9 * np.abs(dm).max()
    # a field parallel to m exerts no torque
    assert np.abs(o.llg_rhs(m, 3.0 * m)).max() < 1e-14 * GAMMA * 3.0


def larmor(theta0, phi0, H, alpha, t):
    gp = GAMMA / (1 + alpha ** 2)
    th = 2 * np.arctan(np.tan(theta0 / 2) * np.exp(-alpha * gp * H * t))
    ph = phi0 + gp * H * t
    return np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])


def test_macrospin_larmor_closed_form(orc):
    # one cubic cell: its self demag field -Ms m/3 is parallel to m
    H, alpha, th0, ph0 = 1e5, 0.1, 1.0, 0.3
    o = orc.Oracle((1, 1, 1), (2e-9,) * 3, Ms=8e5, alpha=alpha)
    o.set_field((0, 0, H), terms=orc.DEMAG | orc.ZEEMAN)
    m0 = cell_vec(larmor(th0, ph0, H, alpha, 0.0))
    t_end = 200e-12
    m, t, dt, st, status = o.dp45(m0, rtol=1e-11, t_end=t_end)
    assert status == 0 and abs(t - t_end) < 1e-25
    assert np.abs(m.ravel() - larmor(th0, ph0, H, alpha, t_end)).max() < 1e-8


def test_damped_switching_closed_form(orc):
    # Ku along z, field antiparallel: theta' = a (H - HK cos th) sin th.  The
    # time to reach cos(theta) = u follows from partial fractions in u.
    Ms, Ku, alpha = 8e5, 5e4, 0.5
    HK = 2 * Ku / (MU0 * Ms)
    H = 1.5 * HK
    gp = GAMMA / (1 + alpha ** 2)
    Ap = HK ** 2 / (HK ** 2 - H ** 2)
    Bp = 1 / (2 * (H - HK))
    Cp = 1 / (2 * (H + HK))

    def F(u):
        return -(Ap / HK) * math.log(abs(H - HK * u)) - Bp * math.log(1 - u) + Cp * math.log(1 + u)

    th0 = 0.1
    u0 = math.cos(th0)
    o = orc.Oracle((1, 1, 1), (2e-9,) * 3, Ms=Ms, Ku=Ku, eu=(0, 0, 1), alpha=alpha)
    o.set_field((0, 0, -H), terms=orc.DEMAG | orc.ANIS | orc.ZEEMAN)
    m0 = cell_vec([math.sin(th0), 0.0, math.cos(th0)])
    for u in (0.5, 0.0, -0.9):
        t_u = -(F(u) - F(u0)) / (gp * alpha)
        m, t, _, _, status = o.dp45(m0, rtol=1e-12, t_end=t_u)
        assert status == 0
        assert abs(m[2].item() - u) < 1e-8, (u, m[2].item())


def test_dp45_fifth_order(orc):
    # fixed steps on the Larmor problem: halving dt divides the global error
    # by ~2^5
    H, alpha, th0, ph0 = 1e5, 0.1, 1.0, 0.3
    o = orc.Oracle((1, 1, 1), (2e-9,) * 3, Ms=8e5, alpha=alpha)
    o.set_field((0, 0, H), terms=orc.DEMAG | orc.ZEEMAN)
    m0 = cell_vec(larmor(th0, ph0, H, alpha, 0.0))
    t_end = 100e-12
    errs = []
    for dt in (10e-12, 5e-12, 2.5e-12):
        m, t, _, st, _ = o.dp45(m0, dt=dt, t_end=t_end, fixed=True)
        assert abs(t - t_end) < 1e-24
        errs.append(np.abs(m.ravel() - larmor(th0, ph0, H, alpha, t_end)).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 25 < r1 < 40 and 25 < r2 < 40, errs


def test_energy_dissipation_rate(orc):
    n = (4, 3, 2)
    d = (2e-9, 2e-9, 2.5e-9)
    alpha = 0.3
    o = orc.Oracle(n, d, Ms=8e5, A=1.3e-11, Ku=4e4, eu=(0, 0, 1), alpha=alpha)
    o.set_field((1e4, 2e4, -3e4))
    m0 = W.random_unit_sphere(n, 3)
    V = d[0] * d[1] * d[2]
    delta = 1e-14
    ms = [m0] + [o.dp45(m0, rtol=1e-13, t_end=q * delta)[0] for q in (1, 2, 3, 4)]
    E = [o.energy(x)[4] for x in ms]
    # fourth-order central difference at t = 2 delta
    dEdt = (-E[4] + 8 * E[3] - 8 * E[1] + E[0]) / (12 * delta)
    h = o.heff(ms[2])
    tq = np.cross(ms[2], h, axis=0)
    expect = -MU0 * V * (8e5 * alpha * GAMMA / (1 + alpha ** 2) * (tq ** 2).sum(0)).sum()
    assert abs(dEdt - expect) < 1e-6 * abs(expect)


def test_energy_conserved_without_damping(orc):
    n = (8, 8, 2)
    o = orc.Oracle(n, (2e-9,) * 3, Ms=8e5, A=1.3e-11, Ku=3e4, alpha=0.0)
    o.set_field((1e4, 0, 2e4))
    m0 = W.smooth_random(n, 2.0, 4)
    E0 = o.energy(m0)[4]
    m, t, _, st, status = o.dp45(m0, rtol=1e-8, max_steps=100)
    assert status == 0 and st["accepted"] == 100
    assert abs(o.energy(m)[4] - E0) < 1e-6 * abs(E0)


def test_norm_preserved_small_llg(orc):
    c = W.config_small_llg()
    o = orc.Oracle(c["n"], c["d"], Ms=c["Ms"], A=c["A"], alpha=c["alpha"])
    o.set_field(c["H"], terms=c["terms"])
    m, t, dt, st, status = o.dp45(c["m0"], rtol=c["rtol"], max_steps=c["steps"])
    assert status == 0 and st["accepted"] == 200
    # without renormalisation |m| drifts by at most ~ rtol per accepted step
    assert np.abs(np.sqrt((m ** 2).sum(0)) - 1).max() < c["steps"] * c["rtol"]


def test_relax_stoner_wohlfarth(orc):
    Ms, Ku = 8e5, 5e4
    HK = 2 * Ku / (MU0 * Ms)
    H, psi = 0.5 * HK, math.radians(30)
    o = orc.Oracle((1, 1, 1), (2e-9,) * 3, Ms=Ms, Ku=Ku, eu=(0, 0, 1))
    o.set_field((H * math.sin(psi), 0, H * math.cos(psi)), terms=orc.DEMAG | orc.ANIS | orc.ZEEMAN)
    m0 = cell_vec([math.sin(0.05), 0.0, math.cos(0.05)])
    # an explicit integrator stalls at a torque set by its error tolerance,
    # so the criterion is chosen above that floor
    m, st, status = o.relax(m0, tol=1e-8, max_steps=20000, rtol=1e-10)
    assert status == 0
    # dE/dtheta = 2 Ku cos th sin th + mu0 Ms H sin(th - psi) = 0 on (0, psi)
    lo, hi = 0.0, psi

    def g(th):
        return 2 * Ku * math.cos(th) * math.sin(th) + MU0 * Ms * H * math.sin(th - psi)

    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(lo) * g(mid) <= 0:
            hi = mid
        else:
            lo = mid
    th = math.atan2(m[0].item(), m[2].item())
    assert abs(th - lo) < 1e-7 and abs(m[1].item()) < 1e-12
    assert o.max_torque(m) < 1e-8


def test_relax_step_cap_reports_not_converged(orc):
    n = (8, 8, 1)
    o = orc.Oracle(n, (2e-9,) * 3, Ms=8e5, A=1.3e-11)
    m0 = W.random_unit_sphere(n, 2)
    m, st, status = o.relax(m0, tol=1e-9, max_steps=3)
    assert status == orc.ENOTCONV and st["accepted"] == 3


def test_overflowing_trial_step_is_rejected_not_fatal(orc):
    # a first step far beyond stability overflows the stages; the controller
    # rejects it (factor 0.2) and carries on; a NaN in the state is fatal
    n = (8, 8, 2)
    o = orc.Oracle(n, (2e-9,) * 3, Ms=8e5, A=1.3e-11, alpha=0.5)
    m0 = W.random_unit_sphere(n, 1)
    m, t, dt, st, status = o.dp45(m0, dt=1e-6, rtol=1e-6, max_steps=20)
    assert status == 0 and st["accepted"] == 20 and st["rejected"] >= 5
    assert np.all(np.isfinite(m)) and np.abs(np.sqrt((m ** 2).sum(0)) - 1).max() < 1e-3
    bad = m0.copy()
    bad[1, 0, 0, 0] = np.nan
    assert o.dp45(bad, dt=1e-13, max_steps=3)[4] == orc.ENONFINITE


def test_rkf45_fourth_order(orc):
    # the paper's default pair propagates the 4th-order solution: halving dt
    # divides the global error by ~2^4 (fixed steps, Larmor problem)
    H, alpha, th0, ph0 = 1e5, 0.1, 1.0, 0.3
    o = orc.Oracle((1, 1, 1), (2e-9,) * 3, Ms=8e5, alpha=alpha)
    o.set_field((0, 0, H), terms=orc.DEMAG | orc.ZEEMAN)
    m0 = cell_vec(larmor(th0, ph0, H, alpha, 0.0))
    t_end = 100e-12
    errs = []
    for dt in (10e-12, 5e-12, 2.5e-12):
        m, t, _, st, _ = o.rkf45(m0, dt=dt, t_end=t_end, fixed=True)
        assert abs(t - t_end) < 1e-24
        assert st["rhs_evals"] == 1 + 6 * st["accepted"]  # no first-same-as-last
        errs.append(np.abs(m.ravel() - larmor(th0, ph0, H, alpha, t_end)).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 13 < r1 < 20 and 13 < r2 < 20, errs


def test_rkf45_closed_forms(orc):
    # adaptive Fehlberg against the Larmor and damped-switching closed forms
    H, alpha, th0, ph0 = 1e5, 0.1, 1.0, 0.3
    o = orc.Oracle((1, 1, 1), (2e-9,) * 3, Ms=8e5, alpha=alpha)
    o.set_field((0, 0, H), terms=orc.DEMAG | orc.ZEEMAN)
    m0 = cell_vec(larmor(th0, ph0, H, alpha, 0.0))
    m, t, dt, st, status = o.rkf45(m0, rtol=1e-11, t_end=200e-12)
    assert status == 0
    assert np.abs(m.ravel() - larmor(th0, ph0, H, alpha, 200e-12)).max() < 1e-8
    # on a field-coupled grid Fehlberg converges, as rtol shrinks, to the
    # Dormand-Prince solution at rtol 1e-13
    c = W.config_small_llg()
    o2 = orc.Oracle(c["n"], c["d"], Ms=c["Ms"], A=c["A"], alpha=c["alpha"])
    o2.set_field(c["H"], terms=c["terms"])
    ref = o2.dp45(c["m0"], rtol=1e-13, t_end=1e-12)[0]
    e8 = np.abs(o2.rkf45(c["m0"], rtol=1e-8, t_end=1e-12)[0] - ref).max()
    e10 = np.abs(o2.rkf45(c["m0"], rtol=1e-10, t_end=1e-12)[0] - ref).max()
    assert e10 < 1e-7 and e10 < e8 / 10, (e8, e10)


def test_relax_second_order_uniaxial(orc):
    # Ku1, Ku2 along z and a transverse field H along x: the equilibrium
    # angle from z solves sin th (2 Ku1 + 4 Ku2 cos^2 th) = mu0 Ms H
    Ms, Ku1, Ku2 = 8e5, 3e4, 2e4
    H = 0.4 * (2 * Ku1 + 4 * Ku2) / (MU0 * Ms)
    o = orc.Oracle((1, 1, 1), (2e-9,) * 3, Ms=Ms, Ku=Ku1, eu=(0, 0, 1))
    o.set_anisotropy2(Ku2=Ku2)
    o.set_field((H, 0, 0), terms=orc.ANIS | orc.ZEEMAN)
    m0 = cell_vec([math.sin(0.05), 0.0, math.cos(0.05)])
    m, st, status = o.relax(m0, tol=1e-8, max_steps=20000, rtol=1e-10)
    assert status == 0
    lo, hi = 0.0, math.pi / 2

    def g(th):
        return math.sin(th) * (2 * Ku1 + 4 * Ku2 * math.cos(th) ** 2) - MU0 * Ms * H

    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(lo) * g(mid) <= 0:
            hi = mid
        else:
            lo = mid
    th = math.atan2(m[0].item(), m[2].item())
    assert abs(th - lo) < 1e-7, (th, lo)
