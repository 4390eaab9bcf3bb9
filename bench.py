"""Benchmark of the micromagnetic hot path on one MI355X.

Workload (default): the 512 x 512 x 64 grid of 4 nm cells (16.7 M cells,
padded FFT 1024 x 1024 x 128), Ms 1e6 A/m, A 1.5e-11 J/m, alpha 0.02, Ku 0,
H 0 (demag + exchange), seeded Voronoi vortex domains.  One step is one
accepted adaptive Dormand-Prince step in FP32 (six effective-field + LLG
right-hand-side evaluations through the FFT passes, whose x forward pass also
forms each stage input, the error norm in FP64 and the host controller).  `value` is effective-field
evaluations x cells per second over the timed steps.  Inputs are resident in
HBM before timing starts.

The JSON line also carries: the same steps in FP64, effective-field-only
throughput (FP32 and FP64), the roofline of the dominant kernel (the z pass
with the spectral product) from HIP-event timing of every launch inside the
timed region, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Heff evals×cells/s at 16.7M cells FP32 vs FP64; p50/p99 batched solve latency"
HBM_PEAK_GBS = 8000.0


def pass_bytes(grid, prec):
    """Algorithmic HBM bytes per launch of each pass (the traffic model: every
    array a pass must read or write, once)."""
    nx, ny, nz = grid
    P = [1 if n == 1 else 1 << (2 * n - 2).bit_length() for n in grid]
    Px, Py, Pz = P
    hx = Px // 2 + 1 if Px > 1 else 1
    w = 4 if prec == "fp32" else 8
    N = nx * ny * nz
    S1 = 3 * hx * ny * nz * 2 * w
    S2 = 3 * hx * Py * nz * 2 * w
    K = 6 * hx * (Py // 2 + 1) * (Pz // 2 + 1) * w
    m = 3 * N * w
    return {"x_fwd": m + S1, "y_fwd": S1 + S2, "mid": 2 * S2 + K, "y_inv": S2 + S1,
            "x_inv_local": S1 + m + m}


def measured_traffic(grid):
    """HBM bytes per launch of the z pass (FETCH_SIZE + WRITE_SIZE, each scaled
    by a 1 GiB copy) from the committed rocprofv3 counter summary -- only if
    the kernel sources are the ones it was measured on and the grid is its
    grid; else None."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "mid_512x512x64_fp32_hbm_traffic.json")
    if tuple(grid) != (512, 512, 64) or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for fn in rec["sources"]:
        with open(os.path.join(ROOT, fn), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec.get("source_sha256") or "read_bytes" not in rec:
        return None
    return rec["read_bytes"] + rec["write_bytes"]


def run_steps(mm, plan, m, cfg, steps, warmup, rtol, profile=False, method=0):
    import torch

    H = cfg["H"]
    t, dt = 0.0, -1.0
    if warmup:
        _, t, dt, st = plan.llg_step(m, H, cfg["terms"], t, dt, rtol=rtol, max_steps=warmup,
                                     method=method)
    torch.cuda.synchronize()
    if profile:
        plan.profile(True)
    t0 = time.perf_counter()
    _, t, dt, st = plan.llg_step(m, H, cfg["terms"], t, dt, rtol=rtol, max_steps=steps,
                                 method=method)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = plan.profile_read() if profile else None
    if profile:
        plan.profile(False)
    return wall, st, prof


def heff_only(mm, plan, m, cfg, iters, profile=False):
    """Seconds per effective-field evaluation and, with profile, the per-pass
    HIP-event times of the same evaluations."""
    import torch

    out = plan.empty()
    for _ in range(3):
        plan.heff(m, cfg["H"], cfg["terms"], out=out)
    torch.cuda.synchronize()
    if profile:
        plan.profile(True)
    t0 = time.perf_counter()
    for _ in range(iters):
        plan.heff(m, cfg["H"], cfg["terms"], out=out)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / iters
    prof = plan.profile_read() if profile else None
    if profile:
        plan.profile(False)
    return wall, prof


# Dormand-Prince stage inputs: non-zero a_sj per stage s = 2..7, so the x
# forward pass of stage s reads that many derivative vectors beside y.
DP45_STAGE_K = (1, 2, 3, 4, 5, 5)


def step_bytes(grid, prec):
    """Algorithmic bytes per launch of the kernels of a Dormand-Prince step,
    averaged over its six stages: the x forward pass with the stage input
    formed in its load (y, the k_j of non-zero a_sj, the stage input written;
    the last stage also writes the partial error), the x inverse + local pass
    (the last stage also reads the partial error and y for the error norm),
    and the error norm as a kernel of its own where it runs (y, y1 and the
    six k_j of non-zero b_j - b*_j)."""
    pb = pass_bytes(grid, prec)
    w = 4 if prec == "fp32" else 8
    m = 3 * grid[0] * grid[1] * grid[2] * w
    ns = len(DP45_STAGE_K)
    out = dict(pb)
    out["x_fwd_stage"] = pb["x_fwd"] + m + m * sum(DP45_STAGE_K) / ns + m / ns
    out["x_inv_local"] = pb["x_inv_local"] + 2 * m / ns
    out["rk"] = 8 * m
    return out


def extended_stencil(mm, plan, m, cfg, iters):
    """Field evaluation with per-cell exchange constants and per-cell
    interface DMI (the extended stencil of the x inverse / local pass) on the
    same plan and state; the uniform-A kernel is timed beside it."""
    import torch

    nx, ny, nz = plan.grid
    g = np.random.Generator(np.random.PCG64(5))
    A = cfg["A"] * g.uniform(0.5, 1.5, (nz, ny, nx))
    D = g.uniform(2e-3, 4e-3, (nz, ny, nx))
    out = plan.empty()
    res = {}
    for name, on in (("plain", False), ("extended", True)):
        if on:
            plan.set_exchange(A)
            plan.set_dmi(D, mm.MM_DMI_INTERFACE)
        terms = cfg["terms"] | (mm.MM_DMI if on else 0)
        for _ in range(3):
            plan.heff(m, cfg["H"], terms, out=out)
        torch.cuda.synchronize()
        plan.profile(True)
        t0 = time.perf_counter()
        for _ in range(iters):
            plan.heff(m, cfg["H"], terms, out=out)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / iters
        ms, n = plan.profile_read()["x_inv_local"]
        plan.profile(False)
        res[name] = (wall, 1e3 * ms / n)
    plan.set_exchange(None)
    plan.set_dmi(0.0, mm.MM_DMI_INTERFACE)
    N = nx * ny * nz
    ext_bytes = pass_bytes(plan.grid, "fp32")["x_inv_local"] + 2 * N * 4
    return {"heff_ms": 1e3 * res["extended"][0], "heff_plain_ms": 1e3 * res["plain"][0],
            "x_inv_local_us": res["extended"][1], "x_inv_local_plain_us": res["plain"][1],
            "model_bytes": ext_bytes, "GBs": ext_bytes / (res["extended"][1] * 1e-6) / 1e9,
            "terms": "demag + per-cell exchange + per-cell interface DMI"}


def zdense_bytes(grid, prec):
    """Algorithmic HBM bytes per launch of the dense layer-coupling pass: the
    kernel spectra of the nz (nz + 1) / 2 unordered layer pairs, 6 (Py/2+1) Hx
    reals each, and the y-transformed spectrum 3 nz Py Hx complex read and
    written."""
    nx, ny, nz = grid
    Px = 1 if nx == 1 else 1 << (2 * nx - 2).bit_length()
    Py = 1 if ny == 1 else 1 << (2 * ny - 2).bit_length()
    hx = Px // 2 + 1 if Px > 1 else 1
    w = 4 if prec == "fp32" else 8
    return 6 * nz * (nz + 1) // 2 * (Py // 2 + 1) * hx * w + 2 * 3 * nz * Py * hx * 2 * w


def layers(mm, W, iters):
    """Field evaluation of the thin-layer form (unequal heights, dense layer
    coupling) on 512 x 512 x 8, FP32, beside the equidistant plan of the same
    grid (zero-padded 3-D convolution)."""
    import torch

    cfg = W.config_layers()
    grid = cfg["n"]
    out = {}
    for name, lay in (("layers", cfg["dz"]), ("equidistant", None)):
        plan = mm.Plan(grid, cfg["d"], Ms=cfg["Ms"], A=cfg["A"], alpha=cfg["alpha"], prec="fp32",
                       layers=lay)
        m = plan._t(cfg["m0"])
        h = plan.empty()
        for _ in range(3):
            plan.heff(m, None, cfg["terms"], out=h)
        torch.cuda.synchronize()
        plan.profile(True)
        t0 = time.perf_counter()
        for _ in range(iters):
            plan.heff(m, None, cfg["terms"], out=h)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / iters
        prof = plan.profile_read()
        plan.profile(False)
        out[name] = (wall, {k: 1e3 * v[0] / v[1] for k, v in prof.items() if v[1]})
        del plan, m, h
        torch.cuda.empty_cache()
    zb = zdense_bytes(grid, "fp32")
    zus = out["layers"][1]["mid"]
    return {"grid": list(grid), "dz_nm": [round(v * 1e9, 4) for v in cfg["dz"]],
            "heff_ms": 1e3 * out["layers"][0], "passes_us": out["layers"][1],
            "zdense_us": zus, "zdense_model_bytes": zb, "zdense_GBs": zb / (zus * 1e-6) / 1e9,
            "equidistant_heff_ms": 1e3 * out["equidistant"][0],
            "equidistant_passes_us": out["equidistant"][1]}


def oersted_bytes(grid):
    """Algorithmic HBM bytes of one FP32 Oersted field evaluation: the demag
    pass chain (x, y forward; z forward + cross product with the 3-component
    kernel octant + z inverse; y, x inverse) reading the current density and
    writing the field."""
    nx, ny, nz = grid
    P = [1 if n == 1 else 1 << (2 * n - 2).bit_length() for n in grid]
    hx = P[0] // 2 + 1 if P[0] > 1 else 1
    N = nx * ny * nz
    s1, s2 = 3 * nz * ny * hx * 8, 3 * nz * P[1] * hx * 8
    g = 3 * (P[2] // 2 + 1) * (P[1] // 2 + 1) * hx * 4
    return (12 * N + s1) + (s1 + s2) + (2 * s2 + g) + (s2 + s1) + (s1 + 24 * N)


def oersted(mm, plan, cfg, iters):
    """Oersted field of a current density on the benchmark grid, FP32: kernel
    set-up once, then repeated evaluations (the cost of updating the field
    of a time-varying current every step)."""
    import torch

    nx, ny, nz = plan.grid
    g = np.random.Generator(np.random.PCG64(7))
    j = plan._t(g.standard_normal((3, nz, ny, nx)) * 1e11)
    out = plan.empty()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.oersted(j, out=out)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(iters):
        plan.oersted(j, out=out)
    torch.cuda.synchronize()
    call = (time.perf_counter() - t0) / iters
    b = oersted_bytes(plan.grid)
    return {"first_call_s": setup, "call_ms": 1e3 * call, "model_bytes": b,
            "GBs": b / call / 1e9}


def _serve_once(mm, reqs, states, arrivals, opts):
    """Run the request server over `reqs` (start states already in HBM) with
    the given arrival offsets (s); returns completions, makespan and stats."""
    import torch

    srv = mm.Server(budget=opts["budget"], max_active=opts["max_active"],
                    steps_per_launch=opts["steps_per_launch"], prec="fp32",
                    batch=opts.get("batch", 8))
    # resident kernels and plans for every grid class before the clock starts
    seen = set()
    for r in reqs:
        if r["n"] in seen:
            continue
        seen.add(r["n"])
        warm = states[reqs.index(r)].clone()
        srv.submit(warm, r["n"], r["d"], r["Ms"], r["A"], r["Ku"], ku_axis=r["eu"], h_ext=r["H"],
                   tol=opts["tol"], rtol=opts["rtol"], max_steps=0, tag=-1 - len(seen))
    warm_done = 0
    while warm_done < len(seen):
        warm_done += len(srv.poll())
    ms = [m.clone() for m in states]
    torch.cuda.synchronize()
    t0 = srv.clock()
    done, i, n = {}, 0, len(reqs)
    while len(done) < n:
        now = srv.clock() - t0
        while i < n and arrivals[i] <= now:
            r = reqs[i]
            srv.submit(ms[i], r["n"], r["d"], r["Ms"], r["A"], r["Ku"], ku_axis=r["eu"],
                       h_ext=r["H"], tol=opts["tol"], rtol=opts["rtol"],
                       max_steps=opts["max_steps"], tag=i)
            i += 1
        for c in srv.poll():
            done[c["tag"]] = c
            if len(done) % 32 == 0:
                print("[bench] serving: %d/%d requests done" % (len(done), n), file=sys.stderr,
                      flush=True)
    st = srv.stats()
    srv.close()
    return done, t0, st


def serving(mm, W, nreq, opts):
    """Serving on the relaxation request stream (grids 64x64x1, 128x128x2,
    256x64x4, 256x256x8; seeded material, field and smooth start per request)
    at the stream's parameters: torque criterion 1e-5, step cap
    opts["max_steps"], Poisson arrivals at opts["rate"] per second (seeded).
    Only the first `nreq` requests of the 512-request stream are served.
    Latency = completion - scheduled arrival on the host monotonic clock;
    p50/p99 over all requests and over the converged ones, capped requests
    counted separately."""
    import torch

    reqs = W.serving_requests(512, seed=0, rate=opts["rate"])[:nreq]
    states = [torch.tensor(W.smooth_random(r["n"], 8.0, seed=r["seed"]), dtype=torch.float32,
                           device="cuda").contiguous() for r in reqs]
    torch.cuda.synchronize()
    arrivals = [r["arrival"] - reqs[0]["arrival"] for r in reqs]
    print("[bench] serving: %d requests, Poisson arrivals at %.2f/s, cap %d steps" %
          (nreq, opts["rate"], opts["max_steps"]), file=sys.stderr, flush=True)
    done, t0, st = _serve_once(mm, reqs, states, arrivals, opts)
    lat = np.array([done[k]["t_done"] - (t0 + arrivals[k]) for k in range(nreq)])
    conv = [k for k in range(nreq) if done[k]["status"] == mm.MM_OK]
    last = max(c["t_done"] for c in done.values())
    per = {}
    for cls in W.SERVING_GRIDS:
        idx = [k for k in range(nreq) if reqs[k]["n"] == cls]
        if idx:
            lc = lat[idx]
            per["%dx%dx%d" % cls] = {"n": len(idx), "p50_s": float(np.percentile(lc, 50)),
                                     "p99_s": float(np.percentile(lc, 99)),
                                     "converged": sum(done[k]["status"] == mm.MM_OK for k in idx),
                                     "mean_accepted": float(np.mean([done[k]["accepted"]
                                                                     for k in idx]))}
    steps = [done[k]["accepted"] for k in range(nreq)]
    capped = [k for k in range(nreq) if done[k]["status"] == mm.MM_ENOTCONV]
    return {
        "requests": nreq, "stream": "first %d of the 512-request stream" % nreq,
        "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
        "converged_p50_s": float(np.percentile(lat[conv], 50)) if conv else None,
        "converged_p99_s": float(np.percentile(lat[conv], 99)) if conv else None,
        "solves_per_s": nreq / (last - t0), "arrival_rate": opts["rate"],
        "converged": len(conv), "capped": len(capped),
        "capped_final_torque": [float(done[k]["torque"]) for k in capped],
        "mean_accepted_steps": float(np.mean(steps)), "per_class": per,
        "tol": opts["tol"], "rtol": opts["rtol"], "max_steps": opts["max_steps"],
        "max_active": opts["max_active"], "steps_per_launch": opts["steps_per_launch"],
        "hbm_budget_bytes": st["budget"], "hbm_peak_bytes": st["bytes_peak"],
        "waited_memory": st["waited_memory"], "waited_slot": st["waited_slot"],
        "graph_launches": st["graph_launches"], "plans_created": st["plans_created"],
        "plans_reused": st["plans_reused"], "batch": opts.get("batch", 8),
        "max_batch": st["max_batch"],
    }


def serving_shared_launches(mm, W, count=32, grids=((64, 64, 1), (128, 128, 2))):
    """Shared launches on small requests: `count` relaxations of one small
    grid class (seeded material, field and smooth start; tol 1e-5, rtol 1e-7,
    cap 2,000 steps) submitted at once, served with groups of up to 8 requests
    per launch and with one request per plan; makespan and request-steps
    (accepted + rejected) per second.  The trajectories are identical."""
    import torch

    out = {}
    for grid in grids:
        g = W.rng(7)
        reqs = []
        for i in range(count):
            d = g.standard_normal(3)
            d /= np.linalg.norm(d)
            reqs.append(dict(cell=float(g.uniform(2e-9, 5e-9)), Ms=float(g.uniform(4e5, 1.4e6)),
                             A=float(g.uniform(5e-12, 2e-11)), Ku=float(g.uniform(0.0, 5e4)),
                             H=W.mT(float(g.uniform(0.0, 50.0))) * d,
                             m0=W.smooth_random(grid, 8.0, seed=1000 + i)))
        row = {}
        for batch in (8, 1):
            states = [torch.tensor(r["m0"], dtype=torch.float32, device="cuda").contiguous()
                      for r in reqs]
            torch.cuda.synchronize()
            srv = mm.Server(budget=8 << 30, max_active=16, steps_per_launch=8, prec="fp32",
                            batch=batch)
            t0 = srv.clock()
            for i, r in enumerate(reqs):
                c = r["cell"]
                srv.submit(states[i], grid, (c, c, c), r["Ms"], r["A"], r["Ku"], h_ext=r["H"],
                           tol=1e-5, rtol=1e-7, max_steps=2000, tag=i)
            done = {}
            while len(done) < count:
                for c in srv.poll():
                    done[c["tag"]] = c
                time.sleep(0.0005)
            T = max(c["t_done"] for c in done.values()) - t0
            steps = sum(c["accepted"] + c["rejected"] for c in done.values())
            st = srv.stats()
            row["batch%d" % batch] = {"makespan_s": T, "request_steps_per_s": steps / T,
                                      "graph_launches": st["graph_launches"],
                                      "max_batch": st["max_batch"], "request_steps": steps}
            srv.close()
        row["speedup"] = row["batch8"]["request_steps_per_s"] / row["batch1"]["request_steps_per_s"]
        out["%dx%dx%d" % grid] = row
    out["requests"] = count
    return out


def throughput_c2(mm, W, iters):
    """Single-field throughput on the 256 x 256 x 16 grid (1,048,576 cells of
    3 nm, padded 512 x 512 x 32): Ms and A drawn per run (seeds 0, 1, 2), Ku
    5e4 along z, smooth random start; `iters` repeated field evaluations per
    run in FP32 and FP64, median over the runs.  Every pass buffer fits the
    256 MB Infinity Cache here, so the roofline fractions are cache-assisted."""
    import torch

    out = {}
    for prec in ("fp32", "fp64"):
        walls, passes = [], None
        for seed in (0, 1, 2):
            c = W.config_throughput(seed=seed)
            plan = mm.Plan(c["n"], c["d"], Ms=c["Ms"], A=c["A"], Ku=c["Ku"], alpha=0.5, prec=prec)
            m = plan._t(c["m0"])
            h = plan.empty()
            for _ in range(10):
                plan.heff(m, c["H"], c["terms"], out=h)
            torch.cuda.synchronize()
            plan.profile(seed == 0)
            t0 = time.perf_counter()
            for _ in range(iters):
                plan.heff(m, c["H"], c["terms"], out=h)
            torch.cuda.synchronize()
            walls.append((time.perf_counter() - t0) / iters)
            if seed == 0:
                pr = plan.profile_read()
                plan.profile(False)
                pb = pass_bytes(c["n"], prec)
                passes = {k: {"avg_us": 1e3 * v[0] / v[1], "GBs": pb[k] / (v[0] / 1e3 / v[1]) / 1e9}
                          for k, v in pr.items() if v[1] and k in pb}
            del plan, m, h
        N = 256 * 256 * 16
        wall = float(np.median(walls))
        byt = sum(pass_bytes((256, 256, 16), prec).values())
        out[prec] = {"cell_evals_per_s": N / wall, "ms": 1e3 * wall, "model_bytes": byt,
                     "GBs": byt / wall / 1e9, "roofline_frac_cache_assisted": byt / wall / 1e9 /
                     HBM_PEAK_GBS, "passes": passes, "runs": [1e3 * w for w in walls]}
        torch.cuda.empty_cache()
    out["fp32_over_fp64"] = out["fp32"]["cell_evals_per_s"] / out["fp64"]["cell_evals_per_s"]
    out["iters"] = iters
    return out


def differentiation(mm, W):
    """The design case (128 x 128 x 1 film, per-cell density, 500 RK4 steps of
    0.1 ps with checkpoints every 50, time-averaged region m_z): forward and
    discrete-adjoint wall time on the GPU in FP32 and FP64, the memory of the
    checkpoints and the relative L2 difference of the FP32 gradient from the
    FP64 one."""
    import torch

    c = W.config_adjoint()
    res, grads = {}, {}
    for prec in ("fp32", "fp64"):
        plan = mm.Plan(c["n"], c["d"], Ms=1.0, A=c["A"], alpha=c["alpha"], prec=prec)
        plan.set_ms(c["Ms0"] * c["rho"])
        plan.set_drive(c["drive_amp"], c["drive_freq"], c["strip"])
        for rep in range(2):  # the first pair allocates the work space
            m = plan._t(c["m0"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            loss, ck = plan.rk4(m, c["dt"], c["steps"], c["region"], None, mm.MM_ALL, 0.0,
                                c["checkpoint_every"])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, gms, _ = plan.rk4_adjoint(ck, c["dt"], c["steps"], c["region"], None, mm.MM_ALL,
                                         0.0, c["checkpoint_every"], want_m0=False)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
        grads[prec] = gms.double().cpu().numpy() * c["Ms0"]  # dL/drho
        res[prec] = {"forward_s": t1 - t0, "backward_s": t2 - t1, "loss": loss,
                     "checkpoint_bytes": ck.numel() * ck.element_size()}
        del plan
    g32, g64 = grads["fp32"], grads["fp64"]
    res["grad_rel_l2_fp32_vs_fp64"] = float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))
    res["case"] = "128x128x1, 500 RK4 steps of 0.1 ps, checkpoints every 50"
    return res


def copy_bandwidth():
    """Measured device-to-device copy rate (1 GiB read + 1 GiB written per
    copy, torch copy kernel, HIP events): the attainable HBM rate beside the
    8 TB/s nominal peak."""
    import torch

    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / 10
    del a, b
    torch.cuda.empty_cache()
    return {"GBs": 2 * (1 << 30) / t / 1e9, "bytes_per_copy": 2 * (1 << 30),
            "frac_of_nominal": 2 * (1 << 30) / t / 1e9 / HBM_PEAK_GBS}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline():
    """The CPU oracle (plain FP64 C, OpenMP over FFT lines) on the
    single-field throughput grid (256 x 256 x 16, padded 512 x 512 x 32; Ms, A
    of seed 0, Ku 5e4, smooth start): effective-field evaluations on all the
    host threads, then on one."""
    import oracle
    from paper_2302_08843_amd import workloads as W

    c = W.config_throughput(seed=0)
    o = oracle.Oracle(c["n"], c["d"], Ms=c["Ms"], A=c["A"], Ku=c["Ku"], alpha=0.5)
    o.set_field(c["H"], terms=c["terms"])
    N = int(np.prod(c["n"]))
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    rates = {}
    for threads, budget, cap in ((cores, 8.0, 10), (1, 10.0, 2)):
        oracle.set_threads(threads)
        o.heff(c["m0"])  # first touch
        evals, t0 = 0, time.perf_counter()
        while True:
            o.heff(c["m0"])
            evals += 1
            el = time.perf_counter() - t0
            if el > budget or evals >= cap:
                break
        rates[threads] = (N * evals / el, evals, oracle.num_threads())
    oracle.set_threads(cores)
    allc = rates[cores]
    return {"value": allc[0], "unit": "cell-evals/s", "cores": allc[2], "kind": "oracle",
            "sample": "FP64 oracle effective field (FFT demag + exchange + anisotropy + Zeeman) "
                      "on the 256x256x16 throughput grid (padded 512x512x32), %d evaluations on "
                      "%d threads; cells x evaluations per second" % (allc[1], allc[2]),
            "one_core": {"value": rates[1][0], "evals": rates[1][1], "cores": 1},
            "cpu_model": _cpu_model(), "host_threads": cores}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--grid", type=str, default="512,512,64")
    ap.add_argument("--heff-iters", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-layers", dest="layers", action="store_false",
                    help="skip the thin-layer field evaluation")
    ap.add_argument("--no-oersted", dest="oersted", action="store_false",
                    help="skip the Oersted field evaluation")
    ap.add_argument("--layers-only", action="store_true",
                    help="only the thin-layer field evaluation (profiling its kernels alone)")
    ap.add_argument("--serve-requests", type=int, default=8,
                    help="requests of the serving sample, a prefix of the stream (0: skip)")
    ap.add_argument("--serve-max-steps", type=int, default=50000)
    ap.add_argument("--serve-rate", type=float, default=0.2,
                    help="Poisson arrival rate of the serving stream (requests/s)")
    ap.add_argument("--c2-iters", type=int, default=1000)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the C2 throughput, differentiation and copy measurements")
    ap.add_argument("--serve-budget-mib", type=int, default=1024)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB read + 1 GiB write kernel (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(a z-slab decomposition is designed, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2302_08843_amd import mm
    from paper_2302_08843_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calib_copy:
        # torch.mul(a, 1, out=b): reads 1 GiB, writes 1 GiB; HBM counters of
        # this kernel calibrate FETCH_SIZE / WRITE_SIZE
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        print("[bench] calibration copy: 3 x (1 GiB read + 1 GiB write)", file=sys.stderr,
              flush=True)
        del a, b
    if args.layers_only:
        print(json.dumps({"layers_fp32": layers(mm, W, args.heff_iters)}), flush=True)
        return
    grid = tuple(int(v) for v in args.grid.split(","))
    cfg = W.config_large(n=grid)
    N = int(np.prod(grid))
    res = {}
    for prec in (["fp32"] if args.no_fp64 else ["fp32", "fp64"]):
        print("[bench] %s plan %s" % (prec, grid), file=sys.stderr, flush=True)
        plan = mm.Plan(grid, cfg["d"], Ms=cfg["Ms"], A=cfg["A"], Ku=cfg["Ku"], alpha=cfg["alpha"],
                       prec=prec)
        m = plan._t(cfg["m0"])
        wall, st, prof = run_steps(mm, plan, m, cfg, args.steps, args.warmup, args.rtol,
                                   profile=(prec == "fp32"))
        print("[bench] %s %d steps in %.3f s (%d evals)" % (prec, st["accepted"], wall,
                                                            st["rhs_evals"]),
              file=sys.stderr, flush=True)
        th, hprof = heff_only(mm, plan, plan._t(cfg["m0"]), cfg, args.heff_iters,
                              profile=(prec == "fp32"))
        res[prec] = dict(wall=wall, stats=st, prof=prof, heff_s=th, heff_prof=hprof,
                         device_bytes=plan.device_bytes())
        if prec == "fp32":
            # the paper's default pair, same steps from the same start
            m = plan._t(cfg["m0"])
            wall_f, st_f, _ = run_steps(mm, plan, m, cfg, args.steps, args.warmup, args.rtol,
                                        method=mm.MM_RKF45)
            res["rkf45"] = dict(wall=wall_f, stats=st_f)
            print("[bench] extended stencil (per-cell A + DMI)", file=sys.stderr, flush=True)
            res["ext"] = extended_stencil(mm, plan, plan._t(cfg["m0"]), cfg, args.heff_iters)
            if args.oersted:
                print("[bench] Oersted field", file=sys.stderr, flush=True)
                res["oe"] = oersted(mm, plan, cfg, 10)
        del plan, m
        torch.cuda.empty_cache()

    r32 = res["fp32"]
    evals = r32["stats"]["rhs_evals"]
    value = evals * N / r32["wall"]
    prof = r32["prof"]
    pb = pass_bytes(grid, "fp32")
    mid_ms, mid_n = prof["mid"]
    mid_avg_s = mid_ms / 1e3 / mid_n
    achieved = pb["mid"] / mid_avg_s / 1e9
    # the passes of a plain effective-field evaluation, each against its own
    # byte model; then the kernels of the timed steps, where the x forward
    # pass also forms the stage input
    passes = {}
    hprof = r32["heff_prof"]
    for k in ("x_fwd", "y_fwd", "mid", "y_inv", "x_inv_local"):
        ms, n = hprof[k]
        if n:
            gbs = pb[k] / (ms / 1e3 / n) / 1e9
            passes[k] = {"avg_us": 1e3 * ms / n, "launches": n, "model_bytes": pb[k],
                         "GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
    sb = step_bytes(grid, "fp32")
    step_k = {}
    for k, name in (("x_fwd", "x_fwd_stage"), ("y_fwd", "y_fwd"), ("mid", "mid"),
                    ("y_inv", "y_inv"), ("x_inv_local", "x_inv_local"), ("rk", "rk")):
        ms, n = prof[k]
        if n:
            gbs = sb[name] / (ms / 1e3 / n) / 1e9
            step_k[name] = {"avg_us": 1e3 * ms / n, "launches": n, "model_bytes": sb[name],
                            "GBs": gbs, "frac": gbs / HBM_PEAK_GBS,
                            "ms_per_step": ms / max(1, r32["stats"]["accepted"])}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r32["wall"] / max(1, r32["stats"]["accepted"]),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "large_512x512x64 adaptive Dormand-Prince steps, FP32 bulk, "
                               "demag + exchange, vortex-domain start",
                   "grid": list(grid), "cells": N, "cell_m": list(cfg["d"]), "rtol": args.rtol,
                   "rhs_evals": evals, "rejected": r32["stats"]["rejected"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(grid),
                     "kernel": "k_mid_w<float,128,2,...> (z forward + spectral product + z inverse)",
                     "bytes_per_launch": pb["mid"], "avg_us": mid_avg_s * 1e6},
        "passes_fp32": passes,
        "step_kernels_fp32": step_k,
        "heff_only": {"fp32_cell_evals_per_s": N / r32["heff_s"], "fp32_ms": 1e3 * r32["heff_s"]},
        "serving": None,
    }
    if args.serve_requests > 0:
        out["serving"] = serving(mm, W, args.serve_requests,
                                 dict(budget=args.serve_budget_mib << 20, max_active=16,
                                      steps_per_launch=8, tol=1e-5, rtol=1e-7,
                                      max_steps=args.serve_max_steps, rate=args.serve_rate))
    if not args.no_extras:
        print("[bench] copy bandwidth", file=sys.stderr, flush=True)
        out["copy_bandwidth"] = copy_bandwidth()
        print("[bench] 256x256x16 throughput", file=sys.stderr, flush=True)
        out["throughput_256x256x16"] = throughput_c2(mm, W, args.c2_iters)
        print("[bench] differentiation case", file=sys.stderr, flush=True)
        out["differentiation"] = differentiation(mm, W)
        print("[bench] serving: shared launches on small requests", file=sys.stderr, flush=True)
        out["serving_shared_launches"] = serving_shared_launches(mm, W)
    if "rkf45" in res:
        rf = res["rkf45"]
        out["rkf45_fp32"] = {"value": rf["stats"]["rhs_evals"] * N / rf["wall"],
                             "ms_per_step": 1e3 * rf["wall"] / max(1, rf["stats"]["accepted"]),
                             "rhs_evals": rf["stats"]["rhs_evals"],
                             "rejected": rf["stats"]["rejected"]}
    if "ext" in res:
        out["extended_stencil_fp32"] = res["ext"]
    if "oe" in res:
        out["oersted_fp32"] = res["oe"]
    if args.layers:
        print("[bench] thin layers 512x512x8", file=sys.stderr, flush=True)
        out["layers_fp32"] = layers(mm, W, args.heff_iters)
    if "fp64" in res:
        r64 = res["fp64"]
        out["fp64"] = {"value": r64["stats"]["rhs_evals"] * N / r64["wall"],
                       "ms_per_step": 1e3 * r64["wall"] / max(1, r64["stats"]["accepted"]),
                       "rhs_evals": r64["stats"]["rhs_evals"]}
        out["heff_only"]["fp64_cell_evals_per_s"] = N / r64["heff_s"]
        out["heff_only"]["fp64_ms"] = 1e3 * r64["heff_s"]
        out["fp32_over_fp64"] = value / out["fp64"]["value"]
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
