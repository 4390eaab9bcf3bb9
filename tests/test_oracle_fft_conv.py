"""Pins of the oracle's FFT and zero-padded FFT convolution (Sec. 4.4, discrete
convolution h_i = sum_j N_{i-j} M_j): the radix-2 FFT against the naive DFT
(the definition), the padding rule, and the FFT convolution against the
O(N^2) direct sum."""
import numpy as np
import pytest

from paper_2302_08843_amd import workloads as W


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft_matches_naive_dft(orc, n, sign):
    g = W.rng(n)
    x = g.standard_normal(n) + 1j * g.standard_normal(n)
    X = orc.fft1d(x, sign)
    R = orc.dft1d(x, sign)
    assert np.linalg.norm(X - R) <= 1e-14 * np.linalg.norm(R) + 1e-300


def test_naive_dft_delta_and_constant(orc):
    # definition checks: a delta transforms to a unit-modulus phase ramp, a
    # constant to a delta
    n = 12
    x = np.zeros(n, complex)
    x[3] = 1.0
    X = orc.dft1d(x, -1)
    assert np.allclose(X, np.exp(-2j * np.pi * 3 * np.arange(n) / n), atol=1e-15)
    X = orc.dft1d(np.ones(n), -1)
    assert abs(X[0] - n) < 1e-13 and np.abs(X[1:]).max() < 1e-13


def test_padding_rule(orc):
    cases = {1: 1, 2: 4, 3: 8, 4: 8, 5: 16, 32: 64, 51: 128, 64: 128, 101: 256, 256: 512, 512: 1024}
    for n, p in cases.items():
        assert orc.padded(n) == p


@pytest.mark.parametrize("n", [(5, 3, 2), (8, 8, 4), (7, 1, 1), (1, 1, 5), (6, 5, 1), (1, 9, 3), (16, 12, 3)])
def test_fft_conv_matches_direct_sum(orc, n):
    g = W.rng(sum(n))
    nx, ny, nz = n
    Ms = g.uniform(0.2, 1.5, (nz, ny, nx)) * 1e6
    Ms[g.uniform(size=Ms.shape) < 0.15] = 0.0  # vacuum cells
    m = W.random_unit_sphere(n, 7)
    d = (2e-9, 3e-9, 2.5e-9)
    a = orc.Oracle(n, d, Ms=Ms, p=3, direct=True).demag(m)
    b = orc.Oracle(n, d, Ms=Ms, p=3, direct=False).demag(m)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a)


def test_fft_conv_matches_direct_sum_small_llg_grid(orc):
    c = W.config_small_llg()
    a = orc.Oracle(c["n"], c["d"], Ms=c["Ms"], direct=True).demag(c["m0"])
    b = orc.Oracle(c["n"], c["d"], Ms=c["Ms"], direct=False).demag(c["m0"])
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a)


def test_demag_linear_and_symmetric(orc):
    # the convolution operator is symmetric: <u, K v> = <v, K u> (K_ab = K_ba,
    # K(-r) = K(r)); with Ms = 1 this is the plain inner product
    n = (6, 5, 3)
    o = orc.Oracle(n, (1e-9, 2e-9, 3e-9), Ms=1.0)
    u = W.random_unit_sphere(n, 1)
    v = W.random_unit_sphere(n, 2)
    lhs = (u * o.demag(v)).sum()
    rhs = (v * o.demag(u)).sum()
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    w = o.demag(2.0 * u - 0.5 * v)
    assert np.allclose(w, 2.0 * o.demag(u) - 0.5 * o.demag(v), rtol=0, atol=1e-13)


@pytest.mark.parametrize("grid,p", [((9, 7, 5), 2), ((12, 5, 1), 3), ((6, 6, 6), 20), ((1, 11, 4), 1)])
def test_demag_at_equals_convolution(orc, grid, p):
    """The direct sum at selected cells (used on grids too large for the FFT
    path) agrees with the FFT convolution and the O(N^2) direct path at every
    cell, near/far split included, with per-cell Ms and vacuum cells."""
    g = np.random.default_rng(7)
    nx, ny, nz = grid
    d = (2e-9, 3e-9, 2.5e-9)
    Ms = g.uniform(3e5, 1e6, (nz, ny, nx))
    Ms[g.uniform(size=Ms.shape) < 0.2] = 0.0
    m = g.standard_normal((3, nz, ny, nx))
    o = orc.Oracle(grid, d, Ms=Ms, p=p)
    od = orc.Oracle(grid, d, Ms=Ms, p=p, direct=True)
    ref = o.demag(m)
    ref_direct = od.demag(m)
    N = nx * ny * nz
    got = orc.demag_at(grid, d, m, np.arange(N), Ms=Ms, p=p)
    got = got.T.reshape(3, nz, ny, nx)
    scale = np.abs(ref).max()
    assert np.abs(got - ref_direct).max() <= 1e-13 * scale
    assert np.abs(got - ref).max() <= 1e-12 * scale
