"""GPU tests of the serving form: the request server (mm_serve_*) runs
relaxations and time integrations with device-side step control replayed from
HIP graphs, admits requests by slots and device memory, and shares spectral
kernels per grid class.  Checked against the oracle (FP64), against the
host-controlled entry points, and for bit-identical results alone and in a
mix."""
import numpy as np
import pytest

from gpu_util import banner, rel_l2, to_np
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


def _drain(srv, n, limit_s=100.0):
    import time

    out, t0 = [], time.time()
    while len(out) < n:
        out += srv.poll()
        assert time.time() - t0 < limit_s, "server did not finish"
    return {c["tag"]: c for c in out}


def _req(seed, grid, cell=3e-9):
    g = W.rng(seed)
    d = g.standard_normal(3)
    d /= np.linalg.norm(d)
    return dict(grid=grid, cell=(cell, cell, cell), Ms=float(g.uniform(4e5, 1.4e6)),
                A=float(g.uniform(5e-12, 2e-11)), Ku=float(g.uniform(0.0, 5e4)),
                H=W.mT(float(g.uniform(10.0, 50.0))) * d,
                m0=W.smooth_random(grid, 4.0, seed=seed + 100))


def test_serve_relax_matches_oracle_fp64(torch_cuda, mm, orc):
    grid = (12, 10, 2)
    banner("serve relax fp64 vs oracle %s" % (grid,))
    r = _req(1, grid)
    srv = mm.Server(max_active=4, steps_per_launch=4, prec="fp64")
    m = torch_cuda.tensor(r["m0"], dtype=torch_cuda.float64, device="cuda").contiguous()
    tol = 1e-6
    srv.submit(m, grid, r["cell"], r["Ms"], r["A"], r["Ku"], h_ext=r["H"], tol=tol, rtol=1e-8,
               tag=7)
    c = _drain(srv, 1)[7]
    assert c["status"] == mm.MM_OK, c
    assert c["torque"] < tol
    o = orc.Oracle(grid, r["cell"], Ms=r["Ms"], A=r["A"], Ku=r["Ku"], alpha=1.0)
    o.set_field(r["H"])
    ref = o.relax(r["m0"], tol=tol, rtol=1e-8)[0]
    got = to_np(m)
    e = rel_l2(got, ref)
    print("  accepted %d rejected %d torque %.2e  rel-L2 vs oracle %.2e"
          % (c["accepted"], c["rejected"], c["torque"], e))
    assert e <= 1e-4
    # the relaxed state's torque measured independently by the oracle
    assert o.max_torque(got) < 2 * tol


def test_serve_relax_matches_host_controlled_relax(torch_cuda, mm):
    """FP32: the device-side controller against mm_relax's host-side one
    (same rules; the step-size factor may round differently, so the states
    agree to the relaxation tolerance rather than bitwise)."""
    grid = (32, 24, 1)
    banner("serve relax fp32 vs mm_relax %s" % (grid,))
    r = _req(2, grid)
    H = W.mT(60.0) * np.array([0.6, 0.0, 0.8])
    srv = mm.Server(max_active=2, steps_per_launch=8, prec="fp32")
    m = torch_cuda.tensor(r["m0"], dtype=torch_cuda.float32, device="cuda").contiguous()
    srv.submit(m, grid, r["cell"], r["Ms"], r["A"], r["Ku"], h_ext=H, tol=1e-4, rtol=1e-7,
               max_steps=20000, tag=1)
    c = _drain(srv, 1)[1]
    plan = mm.Plan(grid, r["cell"], Ms=r["Ms"], A=r["A"], Ku=r["Ku"], alpha=1.0, prec="fp32")
    mh = plan._t(r["m0"])
    status, st = plan.relax(mh, H, mm.MM_ALL, tol=1e-4, max_steps=20000, rtol=1e-7)
    e = rel_l2(to_np(m), to_np(mh))
    print("  server: %d steps torque %.2e | host: %d steps status %d | rel-L2 %.2e"
          % (c["accepted"], c["torque"], st["accepted"], status, e))
    assert status == mm.MM_OK and c["status"] == mm.MM_OK
    assert e <= 1e-3
    assert plan.max_torque(m, H) < 1e-4


def test_serve_integrate_matches_oracle(torch_cuda, mm, orc):
    grid = (16, 12, 2)
    banner("serve integrate fp64 vs oracle %s" % (grid,))
    r = _req(3, grid)
    alpha, t_end = 0.1, 5e-11
    srv = mm.Server(max_active=2, steps_per_launch=5, prec="fp64")
    m = torch_cuda.tensor(r["m0"], dtype=torch_cuda.float64, device="cuda").contiguous()
    srv.submit(m, grid, r["cell"], r["Ms"], r["A"], r["Ku"], alpha=alpha, h_ext=r["H"],
               kind=mm.MM_SERVE_INTEGRATE, rtol=1e-8, t_end=t_end, tag=3)
    c = _drain(srv, 1)[3]
    assert c["status"] == mm.MM_OK and c["t"] == t_end
    o = orc.Oracle(grid, r["cell"], Ms=r["Ms"], A=r["A"], Ku=r["Ku"], alpha=alpha)
    o.set_field(r["H"])
    ref, t, _, _, _ = o.dp45(r["m0"], rtol=1e-8, t_end=t_end)
    e = rel_l2(to_np(m), ref)
    print("  accepted %d rejected %d rel-L2 vs oracle %.2e" % (c["accepted"], c["rejected"], e))
    assert e <= 1e-7


@pytest.mark.parametrize("prec,rtol,bar", [("fp64", 1e-8, 1e-7), ("fp32", 1e-6, 1e-4)])
def test_serve_batched_integrations_match_oracle(torch_cuda, mm, orc, prec, rtol, bar):
    """Four time integrations of one grid class -- cell edges 2 to 3.5 nm (the
    class's one spectral kernel, rescaled), each with its own material, field
    and damping -- share one batch plan and every launch; each final state
    against the oracle's FP64 integration of that request alone (rtol 1e-8).
    Bars: FP64 10 rtol; FP32 (its own step sequence at rtol 1e-6, FP32
    fields) 1e-4, the FP32-against-FP64 trajectory bar."""
    grid = (16, 12, 2)
    banner("serve batched integrations %s vs oracle %s" % (prec, grid))
    t_end = 3e-11
    dt = torch_cuda.float64 if prec == "fp64" else torch_cuda.float32
    srv = mm.Server(max_active=2, steps_per_launch=5, prec=prec, batch=4)
    reqs, ms = [], {}
    for i in range(4):
        r = _req(70 + i, grid, cell=(2.0 + 0.5 * i) * 1e-9)
        r["alpha"] = 0.05 + 0.05 * i
        reqs.append(r)
        ms[i] = torch_cuda.tensor(r["m0"], dtype=dt, device="cuda").contiguous()
        srv.submit(ms[i], grid, r["cell"], r["Ms"], r["A"], r["Ku"], alpha=r["alpha"],
                   h_ext=r["H"], kind=mm.MM_SERVE_INTEGRATE, rtol=rtol, t_end=t_end, tag=i)
    comps = _drain(srv, 4)
    st = srv.stats()
    srv.close()
    assert st["max_batch"] == 4 and st["plans_created"] == 1, st
    for i, r in enumerate(reqs):
        c = comps[i]
        assert c["status"] == mm.MM_OK and c["t"] == t_end, c
        o = orc.Oracle(grid, r["cell"], Ms=r["Ms"], A=r["A"], Ku=r["Ku"], alpha=r["alpha"])
        o.set_field(r["H"])
        ref = o.dp45(r["m0"], rtol=1e-8, t_end=t_end)[0]
        e = rel_l2(to_np(ms[i]), ref)
        print("  request %d (cell %.1f nm, alpha %.2f): accepted %d rejected %d rel-L2 vs oracle %.2e"
              % (i, r["cell"][0] * 1e9, r["alpha"], c["accepted"], c["rejected"], e))
        assert e <= bar


def test_serve_batched_relaxations_match_oracle(torch_cuda, mm, orc):
    """Four FP64 relaxations of one grid class (cell edges 2 to 3.5 nm, own
    material and field) in one batch plan, each to its own torque criterion:
    every final state against the oracle's relaxation of that request alone,
    and its torque measured by the oracle."""
    grid = (12, 10, 2)
    banner("serve batched relaxations fp64 vs oracle %s" % (grid,))
    tol = 1e-6
    srv = mm.Server(max_active=2, steps_per_launch=4, prec="fp64", batch=4)
    reqs, ms = [], {}
    for i in range(4):
        r = _req(80 + i, grid, cell=(2.0 + 0.5 * i) * 1e-9)
        reqs.append(r)
        ms[i] = torch_cuda.tensor(r["m0"], dtype=torch_cuda.float64, device="cuda").contiguous()
        srv.submit(ms[i], grid, r["cell"], r["Ms"], r["A"], r["Ku"], h_ext=r["H"], tol=tol,
                   rtol=1e-8, tag=i)
    comps = _drain(srv, 4)
    st = srv.stats()
    srv.close()
    assert st["max_batch"] == 4 and st["plans_created"] == 1, st
    for i, r in enumerate(reqs):
        c = comps[i]
        assert c["status"] == mm.MM_OK and c["torque"] < tol, c
        o = orc.Oracle(grid, r["cell"], Ms=r["Ms"], A=r["A"], Ku=r["Ku"], alpha=1.0)
        o.set_field(r["H"])
        ref, st_o, status_o = o.relax(r["m0"], tol=tol, rtol=1e-8)
        got = to_np(ms[i])
        e = rel_l2(got, ref)
        print("  request %d (cell %.1f nm): accepted %d (oracle %d) torque %.2e rel-L2 vs oracle %.2e"
              % (i, r["cell"][0] * 1e9, c["accepted"], st_o["accepted"], c["torque"], e))
        assert status_o == 0
        # the same step path as the oracle: the states agree to rounding
        # accumulated over the steps; otherwise to the relaxation tolerance
        same = c["accepted"] == st_o["accepted"] and c["rejected"] == st_o["rejected"]
        assert e <= (1e-9 if same else 1e-4)
        assert o.max_torque(got) < 2 * tol


def test_serve_fp32_relaxation_converges_like_fp64(torch_cuda, mm):
    """Request 6 of the serving stream (128x128x2, 3 nm cells, tol 1e-5, rtol
    1e-7), whose FP32 torque levelled off at 1.5e-5 while the exchange
    stencil took the float-rounded state: with the split state the FP32
    server reaches the criterion within 2 % of the FP64 server's step count."""
    r = W.serving_requests(512, seed=0, rate=0.2)[6]
    banner("serve fp32 relaxation vs fp64 steps %s" % (r["n"],))
    steps = {}
    for prec, dt in (("fp64", torch_cuda.float64), ("fp32", torch_cuda.float32)):
        m = torch_cuda.tensor(W.smooth_random(r["n"], 8.0, seed=r["seed"]), dtype=dt,
                              device="cuda").contiguous()
        srv = mm.Server(max_active=2, steps_per_launch=8, prec=prec)
        srv.submit(m, r["n"], r["d"], r["Ms"], r["A"], r["Ku"], ku_axis=r["eu"], h_ext=r["H"],
                   tol=1e-5, rtol=1e-7, max_steps=20000, tag=0)
        c = _drain(srv, 1)[0]
        srv.close()
        print("  %s: status %d accepted %d rejected %d torque %.3g"
              % (prec, c["status"], c["accepted"], c["rejected"], c["torque"]))
        assert c["status"] == mm.MM_OK and c["torque"] < 1e-5, c
        steps[prec] = c["accepted"]
    assert abs(steps["fp32"] - steps["fp64"]) <= 0.02 * steps["fp64"], steps


def _mix(n):
    grids = [(16, 16, 1), (24, 8, 2), (32, 32, 1), (20, 12, 3)]
    reqs = []
    for i in range(n):
        r = _req(50 + i, grids[i % len(grids)], cell=(2.0 + 0.25 * (i % 5)) * 1e-9)
        r["tag"] = i
        reqs.append(r)
    return reqs


def _run(torch, mm, reqs, **kw):
    # a step cap keeps the test short: capped and converged requests alike
    # must give the same result alone and in the mix
    srv = mm.Server(prec="fp32", **kw)
    ms = {}
    for r in reqs:
        m = torch.tensor(r["m0"], dtype=torch.float32, device="cuda").contiguous()
        ms[r["tag"]] = m
        srv.submit(m, r["grid"], r["cell"], r["Ms"], r["A"], r["Ku"], h_ext=r["H"], tol=1e-4,
                   rtol=1e-7, max_steps=1200, tag=r["tag"])
    comps = _drain(srv, len(reqs))
    return srv, comps, {k: to_np(v) for k, v in ms.items()}


def test_serve_alone_and_in_mix_bit_identical(torch_cuda, mm):
    banner("serve alone vs mix, 16 requests")
    reqs = _mix(16)
    alone_m, alone_c = {}, {}
    for r in reqs:
        _, c, m = _run(torch_cuda, mm, [r], max_active=1)
        alone_m.update(m)
        alone_c.update(c)
    srv, mix_c, mix_m = _run(torch_cuda, mm, reqs, max_active=16, steps_per_launch=4)
    st = srv.stats()
    print("  stats", st)
    for r in reqs:
        k = r["tag"]
        assert mix_c[k]["status"] in (mm.MM_OK, mm.MM_ENOTCONV)
        assert np.array_equal(alone_m[k], mix_m[k]), k
        for f in ("status", "accepted", "rejected", "rhs_evals", "torque"):
            assert alone_c[k][f] == mix_c[k][f], (k, f)
    # four grid classes, five cell sizes each: one resident kernel per class;
    # the requests of a class share launches
    assert st["tensors_built"] == 4
    assert st["max_batch"] >= 2


@pytest.mark.parametrize("batch", [1, 8])
def test_serve_plan_reuse_bit_identical(torch_cuda, mm, batch):
    """Later requests of a class run on resident plans (cell size, material and
    field rewritten, state and controller prepared afresh): with batch = 1 a
    finished request's plan is kept idle and taken over by the next request
    of its class, with batch = 8 a finished request's slot in a running group
    is refilled.  Eight requests of two classes through two streams: plans are
    reused, and every result is bit-identical to a run on a fresh server."""
    banner("serve plan reuse, 8 requests of two classes, 2 streams, batch %d" % batch)
    reqs = []
    for i in range(8):
        grid = (24, 16, 1) if i % 2 == 0 else (16, 8, 2)
        r = _req(70 + i, grid, cell=(2.0 + 0.5 * i) * 1e-9)
        r["tag"] = i
        reqs.append(r)
    alone_m, alone_c = {}, {}
    for r in reqs:
        srv1, c, m = _run(torch_cuda, mm, [r], max_active=1, batch=batch)
        assert srv1.stats()["plans_reused"] == 0
        alone_m.update(m)
        alone_c.update(c)
    srv, cs, ms = _run(torch_cuda, mm, reqs, max_active=2, steps_per_launch=4, batch=batch)
    st = srv.stats()
    print("  stats", st)
    for r in reqs:
        k = r["tag"]
        assert cs[k]["status"] in (mm.MM_OK, mm.MM_ENOTCONV)
        assert np.array_equal(alone_m[k], ms[k]), k
        for f in ("status", "accepted", "rejected", "rhs_evals", "torque"):
            assert alone_c[k][f] == cs[k][f], (k, f)
    assert st["plans_reused"] > 0
    assert st["plans_created"] + st["plans_reused"] == len(reqs)
    assert st["tensors_built"] == 2


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_serve_shared_launches_bit_identical(torch_cuda, mm, prec):
    """Requests of one group run in shared launches (batch plan, request index
    in every kernel's grid, one graph for the group), joining and leaving the
    batch as slots free up: six requests through four slots give results
    bit-identical to a server that runs every request on a plan of its own
    (batch = 1, the single-request kernels)."""
    banner("serve shared launches vs single-request plans, %s" % prec)
    dt = torch_cuda.float32 if prec == "fp32" else torch_cuda.float64
    reqs = []
    for i in range(6):
        r = _req(90 + i, (20, 12, 2), cell=(2.0 + 0.4 * i) * 1e-9)
        r["tag"] = i
        reqs.append(r)
    res = {}
    for batch in (1, 4):
        srv = mm.Server(max_active=2, steps_per_launch=4, prec=prec, batch=batch)
        ms = {}
        for r in reqs:
            m = torch_cuda.tensor(r["m0"], dtype=dt, device="cuda").contiguous()
            ms[r["tag"]] = m
            srv.submit(m, r["grid"], r["cell"], r["Ms"], r["A"], r["Ku"], h_ext=r["H"], tol=1e-4,
                       rtol=1e-7, max_steps=600, tag=r["tag"])
        comps = _drain(srv, len(reqs))
        st = srv.stats()
        print("  batch %d stats %s" % (batch, st))
        res[batch] = (comps, {k: to_np(v) for k, v in ms.items()}, st)
    for r in reqs:
        k = r["tag"]
        c1, c4 = res[1][0][k], res[4][0][k]
        assert c4["status"] in (mm.MM_OK, mm.MM_ENOTCONV)
        assert np.array_equal(res[1][1][k], res[4][1][k]), k
        for f in ("status", "accepted", "rejected", "rhs_evals", "torque"):
            assert c1[f] == c4[f], (k, f)
    # four requests shared one group's launches; the other two started a
    # second group on the second stream; fewer graph launches in all
    assert res[1][2]["max_batch"] == 1
    assert res[4][2]["max_batch"] == 4
    assert res[4][2]["plans_created"] <= 2
    assert res[4][2]["plans_created"] + res[4][2]["plans_reused"] == len(reqs)
    assert res[4][2]["graph_launches"] < res[1][2]["graph_launches"]


def test_serve_admission_by_memory_budget(torch_cuda, mm):
    banner("serve admission under a memory budget")
    reqs = _mix(8)
    # room for the four resident kernels (about 0.23 MB) and a few plans
    # (0.11 - 0.36 MB per request) at a time; groups shrink to fit
    budget = 800 * 1024
    srv, comps, _ = _run(torch_cuda, mm, reqs, max_active=8, budget=budget)
    st = srv.stats()
    print("  stats", st)
    assert all(c["status"] in (mm.MM_OK, mm.MM_ENOTCONV) for c in comps.values())
    assert st["bytes_peak"] <= budget
    assert st["waited_memory"] > 0
    assert st["completed"] == 8


def test_serve_rejects_oversized_and_invalid(torch_cuda, mm):
    banner("serve oversized / invalid requests")
    srv = mm.Server(max_active=2, budget=1 << 20, prec="fp32")
    grid = (128, 128, 2)
    m = torch_cuda.zeros((3, 2, 128, 128), dtype=torch_cuda.float32, device="cuda")
    m[0] = 1.0
    srv.submit(m, grid, (3e-9,) * 3, 8e5, 1e-11, tag=11)
    c = _drain(srv, 1)[11]
    assert c["status"] == mm.MM_ENOMEM
    with pytest.raises(mm.MMError):
        srv.submit(m, grid, (3e-9, 3e-9, -1.0), 8e5, 1e-11, tag=12)
    with pytest.raises(mm.MMError):
        srv.submit(m, grid, (3e-9,) * 3, 8e5, 1e-11, tol=0.0, tag=13)


def test_serve_step_cap_reports_not_converged(torch_cuda, mm):
    banner("serve step cap")
    r = _req(9, (16, 16, 1))
    srv = mm.Server(max_active=1, steps_per_launch=8, prec="fp32")
    m = torch_cuda.tensor(r["m0"], dtype=torch_cuda.float32, device="cuda").contiguous()
    srv.submit(m, r["grid"], r["cell"], r["Ms"], r["A"], r["Ku"], h_ext=r["H"], tol=1e-12,
               rtol=1e-5, max_steps=13, tag=5)
    c = _drain(srv, 1)[5]
    assert c["status"] == mm.MM_ENOTCONV
    assert c["accepted"] == 13
