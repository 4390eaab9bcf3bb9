"""The C-ABI library loads on a machine without a GPU, exports every entry
point declared in include/mm.h, and rejects invalid arguments before touching
the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    from paper_2302_08843_amd import mm

    assert declared_functions() == sorted(mm.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_2302_08843_amd import mm

    L = mm.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_invalid_arguments_rejected_without_device():
    from paper_2302_08843_amd import mm

    L = mm.lib()
    o = mm.mm_opts_default()
    assert o.prec == mm.MM_FP64 and o.demag_p == 20 and list(o.ku_axis) == [0.0, 0.0, 1.0]
    bad = [
        ((0, 4, 4), (1e-9,) * 3, 8e5, 1e-11, 0, 0.5),
        ((513, 4, 4), (1e-9,) * 3, 8e5, 1e-11, 0, 0.5),
        ((4, 4, 4), (1e-9, 0.0, 1e-9), 8e5, 1e-11, 0, 0.5),
        ((4, 4, 4), (1e-9,) * 3, -1.0, 1e-11, 0, 0.5),
        ((4, 4, 4), (1e-9,) * 3, 8e5, -1e-11, 0, 0.5),
        ((4, 4, 4), (1e-9,) * 3, 8e5, 1e-11, 0, -0.5),
        ((4, 4, 4), (1e-9,) * 3, float("nan"), 1e-11, 0, 0.5),
    ]
    for args in bad:
        with pytest.raises(mm.MMError) as ei:
            mm.mm_plan_create(*args, opts=o)
        assert ei.value.status == mm.MM_EINVAL
    o.ku_axis[0] = o.ku_axis[1] = o.ku_axis[2] = 0.0
    with pytest.raises(mm.MMError):
        mm.mm_plan_create((4, 4, 4), (1e-9,) * 3, 8e5, 1e-11, 0, 0.5, opts=o)
    # null handles
    assert L.mm_heff(None, None, None, 15, 0.0, None) == mm.MM_EINVAL
    assert L.mm_energy(None, None, None, 15, 0.0, None) == mm.MM_EINVAL
    L.mm_plan_destroy(None)


def test_serve_options_and_rejections_without_device():
    """Serving options: the defaults the header documents (the binding's
    structure carries every field, batch included), and options out of range
    rejected before the device is touched."""
    from paper_2302_08843_amd import mm

    o = mm.mm_serve_opts_default()
    assert (o.hbm_budget, o.max_active, o.steps_per_launch, o.prec, o.demag_p, o.batch) == \
        (0, 16, 8, mm.MM_FP32, 20, 8)
    for field, val in (("batch", 0), ("batch", 65), ("max_active", 0), ("steps_per_launch", 65)):
        b = mm.mm_serve_opts_default()
        setattr(b, field, val)
        with pytest.raises(mm.MMError) as ei:
            mm.mm_serve_create(b)
        assert ei.value.status == mm.MM_EINVAL, field
    assert [f for f, _ in mm.mm_serve_stats._fields_][-1] == "max_batch"


def test_next_row_entry_points_reject_invalid_arguments_without_device():
    """Per-cell exchange, DMI, the Oersted field and thin layers: invalid
    handles, types and heights are refused before any device work."""
    from paper_2302_08843_amd import mm

    L = mm.lib()
    assert L.mm_set_exchange(None, None) == mm.MM_EINVAL
    assert L.mm_set_dmi(None, mm.MM_DMI_BULK, 1e-3, None) == mm.MM_EINVAL
    assert L.mm_oersted(None, None, None) == mm.MM_EINVAL
    assert L.mm_set_current(None, None, 0.0) == mm.MM_EINVAL
    o = mm.mm_opts_default()
    assert not o.dz_layers and o.ku2 == o.kc1 == o.kc2 == 0.0
    for heights in ([1e-9, -1e-9, 1e-9], [1e-9, float("nan"), 1e-9], [1e-9] * 17):
        arr = (C.c_double * len(heights))(*heights)
        o.dz_layers = C.cast(arr, C.POINTER(C.c_double))
        with pytest.raises(mm.MMError) as ei:
            mm.mm_plan_create((4, 4, len(heights)), (1e-9,) * 3, 8e5, 1e-11, 0, 0.5, opts=o)
        assert ei.value.status == mm.MM_EINVAL
    assert mm.MM_ALL == (mm.MM_DEMAG | mm.MM_EXCH | mm.MM_ANIS | mm.MM_ZEEMAN | mm.MM_DMI |
                         mm.MM_OERSTED)


def test_binding_rejects_bad_tensors_before_any_call(monkeypatch):
    """Every tensor handed to the library is checked against its plan (dtype,
    shape, contiguity, device) before the call: a mismatch raises ValueError
    and never reaches the C ABI (which would otherwise read or write 3N values
    of the plan's precision through the raw pointer)."""
    import numpy as np
    import torch

    from paper_2302_08843_amd import mm

    calls = []

    class Spy:
        def __getattr__(self, name):
            def f(*a):
                calls.append(name)
                return mm.MM_OK
            return f

    monkeypatch.setattr(mm, "_lib", Spy())
    fake = mm.C.c_void_p(0x1000)
    monkeypatch.setitem(mm._PLANS, fake.value, ((5, 4, 3), "float32", 0))
    good = torch.zeros((3, 3, 4, 5), dtype=torch.float32)  # right dtype/shape, CPU memory
    cases = [
        (torch.zeros((3, 3, 4, 5), dtype=torch.float64), "dtype"),
        (torch.zeros((3, 60), dtype=torch.float32), "shape"),
        (torch.zeros((3, 3, 4, 6), dtype=torch.float32), "shape"),
        (torch.zeros((3, 3, 5, 4), dtype=torch.float32).transpose(2, 3), "contiguous"),
        (good, "cuda:0"),
        (np.zeros((3, 3, 4, 5), np.float32), "torch tensor"),
    ]
    for bad, word in cases:
        # the tensor under test is the first one each call validates
        for call in (lambda t: mm.mm_heff(fake, t, None, mm.MM_ALL, 0.0, good),
                     lambda t: mm.mm_oersted(fake, t, good),
                     lambda t: mm.mm_llg_step(fake, t, None, mm.MM_ALL, 0.0, 0.0,
                                              mm.mm_step_opts()),
                     lambda t: mm.mm_llg_rhs_vjp(fake, t, None, mm.MM_ALL, 0.0, good, good, None)):
            with pytest.raises(ValueError) as ei:
                call(bad)
            assert word in str(ei.value), (word, str(ei.value))
    # per-cell fields: (nz, ny, nx); checkpoints: (ceil(n / every), 3, nz, ny, nx)
    with pytest.raises(ValueError, match="shape"):
        mm.mm_set_ms(fake, torch.zeros((3, 4, 6), dtype=torch.float32))
    with pytest.raises(ValueError, match="dtype"):
        mm.mm_set_drive(fake, (1, 0, 0), 1e9, torch.zeros((3, 4, 5), dtype=torch.float32))
    with pytest.raises(ValueError, match="needed"):  # 10 steps, every 4: 3 checkpoints
        mm._ckpt(fake, torch.zeros((2, 3, 3, 4, 5), dtype=torch.float32), 10, 4, "ckpt")
    with pytest.raises(ValueError, match="shape"):
        mm._ckpt(fake, torch.zeros((3, 3, 3, 5, 4), dtype=torch.float32), 10, 4, "ckpt")
    with pytest.raises(ValueError, match="ckpt is required"):
        mm.mm_rk4_adjoint(fake, None, None, mm.MM_ALL, 0.0, 1e-13, 10, None, 4, None, None)
    with pytest.raises(ValueError, match="unknown plan"):
        mm.mm_heff(mm.C.c_void_p(0x2000), good, None, mm.MM_ALL, 0.0, good)
    assert calls == [], calls


def _workspace_model(grid, prec):
    """Bytes of the plan buffers written out from their definitions: padded
    extents P = next power of two >= 2n - 1 (1 for n = 1), x bins Hx = Px/2 + 1
    rounded up to 128 bytes of reals, the folded real kernel 6 (Pz/2+1)(Py/2+1)
    Hx, spectra 3 nz ny Hx and (when Py, Pz > 1) 3 nz Py Hx complex, Lmax
    twiddles, 8192 + 8 reduction doubles, 10 vectors of 3N, the 120-byte
    controller and 2 ny nz doubles of error-norm partials, each rounded up to
    256 bytes."""
    def pad(n):
        p = 1
        while n > 1 and p < 2 * n - 1:
            p *= 2
        return p
    es = 4 if prec == 0 else 8
    nx, ny, nz = grid
    Px, Py, Pz = pad(nx), pad(ny), pad(nz)
    Hx = Px // 2 + 1 if Px > 1 else 1
    al = 32 if prec == 0 else 16
    Hx = -(-Hx // al) * al
    up = lambda b: -(-b // 256) * 256
    parts = [6 * (Pz // 2 + 1) * (Py // 2 + 1) * Hx * es, 3 * nz * ny * Hx * 2 * es]
    if Py > 1 and Pz > 1:
        parts.append(3 * nz * Py * Hx * 2 * es)
    parts += [max(Px, Py, Pz) * 2 * es, 8 * 8192, 8 * 8, 10 * 3 * nx * ny * nz * es, 120,
              2 * 8 * ny * nz]
    return sum(up(b) for b in parts)


def test_workspace_size_query():
    """mm_plan_workspace_bytes (host only): the plan's persistent buffers for a
    caller-owned workspace, against the layout written out independently."""
    from paper_2302_08843_amd import mm

    for grid in [(512, 512, 64), (256, 256, 16), (32, 32, 4), (64, 64, 1), (7, 1, 1), (1, 1, 1),
                 (101, 51, 1), (3, 5, 300)]:
        for prec in (mm.MM_FP32, mm.MM_FP64):
            assert mm.mm_plan_workspace_bytes(grid, prec) == _workspace_model(grid, prec), (grid, prec)
    assert mm.mm_plan_workspace_bytes((0, 4, 4), mm.MM_FP32) == 0
    assert mm.mm_plan_workspace_bytes((513, 4, 4), mm.MM_FP32) == 0
    assert mm.mm_plan_workspace_bytes((4, 4, 4), 7) == 0
    # the large benchmark grid: kernel 410.5 MB + spectra 1.22 GB + RK 2.01 GB (FP32)
    assert abs(mm.mm_plan_workspace_bytes((512, 512, 64), mm.MM_FP32) / 1e9 - 3.70) < 0.05
