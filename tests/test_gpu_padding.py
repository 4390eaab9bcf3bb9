"""Zero padding, kernel placement and crop (Sec. 4.4, Eq. convolution) checked
against the oracle entry by entry:

* the resident folded spectrum (mm_debug_spectrum) equals the real part of the
  FFT of the oracle's kernel placed in the padded grid by the padding rule
  (offsets |I| <= n-1 at I mod P, zero elsewhere), scaled by 1/(Px Py Pz), at
  every kept bin of the octant;
* a single source at a corner cell of an odd grid: the field at every cell is
  K(x - c) Ms m_c from the oracle's tensor entries -- the largest offsets
  (opposite corner) sit on the edge of the placement, so too small a padding
  would alias the far side back in and a shifted pack or crop would move the
  whole field."""
import numpy as np
import pytest

from gpu_util import banner, rel_l2, to_np

pytestmark = pytest.mark.gpu

GRIDS = [((5, 3, 2), (2e-9, 3e-9, 2.5e-9)), ((7, 6, 3), (1e-9, 1e-9, 1e-9)),
         ((9, 1, 5), (2e-9, 2e-9, 1e-9)), ((3, 5, 1), (3e-9, 2e-9, 4e-9)),
         ((17, 9, 6), (2e-9, 2e-9, 3e-9))]


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


def _placed(orc, grid, cell, p):
    """The oracle's real-space kernel (6 components) in the padded grid."""
    P = [orc.padded(n) for n in grid]
    K = np.zeros((6, P[2], P[1], P[0]))
    nx, ny, nz = grid
    for I in range(-(nx - 1), nx):
        for J in range(-(ny - 1), ny):
            for Kk in range(-(nz - 1), nz):
                K[:, Kk % P[2], J % P[1], I % P[0]] = orc.tensor_entry(cell, I, J, Kk, p)
    return P, K


@pytest.mark.parametrize("grid,cell", GRIDS)
def test_resident_spectrum_entries(torch_cuda, mm, orc, grid, cell):
    banner("spectrum %s" % (grid,))
    plan = mm.Plan(grid, cell, Ms=1.0, prec="fp64")
    P, K = _placed(orc, grid, cell, 20)
    Px, Py, Pz = P
    hx = Px // 2 + 1 if Px > 1 else 1
    F = np.fft.fftn(K, axes=(1, 2, 3))
    # scale of the whole tensor (components that vanish by symmetry, such as
    # xy and yz on a single row, are rounding noise on both sides)
    scale = np.abs(F.real).max() / (Px * Py * Pz)
    for s in range(6):
        # K has definite parity along every axis, so its transform is real
        assert np.abs(F[s].imag).max() / (Px * Py * Pz) <= 1e-13 * scale
        ref = F[s].real[: Pz // 2 + 1, : Py // 2 + 1, :hx] / (Px * Py * Pz)
        got = to_np(plan.debug_spectrum(s))
        assert got.shape == ref.shape
        # FFT rounding of both sides (~1e-14 of the scale here); a misplaced
        # entry or a wrong fold would be off by O(1) of the scale
        assert np.abs(got - ref).max() <= 2e-13 * scale, (s, np.abs(got - ref).max() / scale)


@pytest.mark.parametrize("grid,cell", GRIDS)
def test_corner_source_pack_and_crop(torch_cuda, mm, orc, grid, cell):
    nx, ny, nz = grid
    Ms = 8e5
    plan = mm.Plan(grid, cell, Ms=Ms, prec="fp64")
    for corner in ((0, 0, 0), (nx - 1, ny - 1, nz - 1)):
        banner("corner source %s %s" % (grid, corner))
        m = np.zeros((3, nz, ny, nx))
        mc = np.array([0.6, -0.48, 0.64])
        m[:, corner[2], corner[1], corner[0]] = mc
        h = to_np(plan.heff(m, None, mm.MM_DEMAG))
        ref = np.zeros_like(h)
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    xx, yy, zz, xy, xz, yz = orc.tensor_entry(cell, i - corner[0], j - corner[1],
                                                              k - corner[2], 20)
                    Kc = np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])
                    ref[:, k, j, i] = Ms * Kc @ mc
        assert rel_l2(h, ref) <= 1e-12, rel_l2(h, ref)
        # the farthest cell (the opposite corner) on its own: FFT rounding is
        # relative to the field's scale, while an aliased (too small) padding
        # would add about the far field itself there
        o = (nx - 1 - corner[0], ny - 1 - corner[1], nz - 1 - corner[2])
        far = ref[:, o[2], o[1], o[0]]
        err = np.abs(h[:, o[2], o[1], o[0]] - far).max()
        assert err <= 1e-12 * np.abs(ref).max() and err <= 1e-4 * np.abs(far).max(), (err, far)
