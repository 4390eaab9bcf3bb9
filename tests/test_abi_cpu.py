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
