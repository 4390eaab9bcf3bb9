"""Seeded synthetic inputs for the micromagnetic hot path.

This module only draws random numbers and shapes them into magnetisation
fields and material parameters; it holds none of the method's arithmetic
(no field term, no integrator), so both the GPU tests and the CPU oracle
tests take their inputs from here.  Every generator uses numpy's PCG64 with an
explicit seed.

Arrays are float64, shape (3, nz, ny, nx): component-major, x fastest -- the
layout the library takes on device (``v[c*N + i + nx*(j + ny*k)]``).

The paper measures on "different system sizes N" with unstated shapes and
uses a random unit-sphere start (``RandomUnitSphere``) and a vortex template
(Sec. 2 listing); the configurations below stand in for those workloads.
"""
from __future__ import annotations

import numpy as np

MU0 = 4.0e-7 * np.pi


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _normalise(v: np.ndarray) -> np.ndarray:
    n = np.sqrt((v * v).sum(axis=0, keepdims=True))
    n[n == 0] = 1.0
    return v / n


def random_unit_sphere(n, seed: int) -> np.ndarray:
    """i.i.d. Gaussian 3-vectors per cell, normalised to unit length."""
    nx, ny, nz = n
    return _normalise(rng(seed).standard_normal((3, nz, ny, nx)))


def random_direction(seed: int) -> np.ndarray:
    v = rng(seed).standard_normal(3)
    return v / np.linalg.norm(v)


def smooth_random(n, ell: float, seed: int) -> np.ndarray:
    """Gaussian white noise per component, low-passed by exp(-2 pi^2 ell^2 |k|^2)
    on the periodic n-grid (k in cycles per cell, i.e. a Gaussian of standard
    deviation ell cells in real space), then normalised per cell."""
    nx, ny, nz = n
    w = rng(seed).standard_normal((3, nz, ny, nx))
    kz = np.fft.fftfreq(nz)[:, None, None]
    ky = np.fft.fftfreq(ny)[None, :, None]
    kx = np.fft.fftfreq(nx)[None, None, :]
    filt = np.exp(-2.0 * np.pi ** 2 * ell ** 2 * (kx ** 2 + ky ** 2 + kz ** 2))
    out = np.empty_like(w)
    for c in range(3):
        out[c] = np.real(np.fft.ifftn(np.fft.fftn(w[c]) * filt))
    return _normalise(out)


def vortex_domains(n, d, ndomains: int = 16, seed: int = 0, core: float = 5e-9) -> np.ndarray:
    """Voronoi vortex domains: ndomains seeded in-plane centres; each cell
    takes its nearest centre and the vortex template of the paper's Sec. 2
    listing, (c (y-yc)/r, -c (x-xc)/r, p core/r) normalised, with a seeded
    chirality c and polarity p per domain; (0, 0, p) at the centre.  Identical
    in every layer."""
    nx, ny, nz = n
    g = rng(seed)
    cx = g.uniform(0, nx, ndomains)
    cy = g.uniform(0, ny, ndomains)
    chir = g.choice([-1.0, 1.0], ndomains)
    pol = g.choice([-1.0, 1.0], ndomains)
    x = (np.arange(nx) + 0.5)[None, :]
    y = (np.arange(ny) + 0.5)[:, None]
    dist = (x[None] - cx[:, None, None]) ** 2 + (y[None] - cy[:, None, None]) ** 2
    owner = np.argmin(dist, axis=0)
    dx = (x - cx[owner]) * d[0]
    dy = (y - cy[owner]) * d[1]
    r = np.sqrt(dx ** 2 + dy ** 2)
    v = np.stack([chir[owner] * dy, -chir[owner] * dx, pol[owner] * core * np.ones_like(r)])
    v = _normalise(v)
    v[:, r == 0] = np.stack([np.zeros_like(pol[owner]), np.zeros_like(pol[owner]), pol[owner]])[:, r == 0]
    return np.ascontiguousarray(np.broadcast_to(v[:, None], (3, nz, ny, nx)).copy())


def mT(b_mT: float) -> float:
    """Field given as mu0*H in mT -> H in A/m."""
    return b_mT * 1e-3 / MU0


# --------------------------------------------------------------------------
# Workload configurations
# --------------------------------------------------------------------------

def config_small_llg():
    """FP64 LLG parity case: 32x32x4 cells of 2 nm, Ms 8e5, A 1.3e-11, Ku 0,
    alpha 0.5, exchange + demag + Zeeman (10 mT along a seeded direction),
    random unit-sphere start, 200 adaptive steps at rtol 1e-6."""
    n = (32, 32, 4)
    return dict(name="llg_32x32x4", n=n, d=(2e-9, 2e-9, 2e-9), Ms=8e5, A=1.3e-11, Ku=0.0,
                eu=(0.0, 0.0, 1.0), alpha=0.5, H=mT(10.0) * random_direction(1),
                m0=random_unit_sphere(n, 0), steps=200, rtol=1e-6, terms=1 | 2 | 8)


def config_throughput(seed: int = 0, n=(256, 256, 16)):
    """Single-field throughput case: 256x256x16 cubic 3 nm cells, Ms and A
    drawn per run, Ku 5e4 along z, smooth random m (8-cell correlation)."""
    g = rng(1000 + seed)
    Ms = float(g.uniform(4e5, 1.4e6))
    A = float(g.uniform(5e-12, 2e-11))
    return dict(name="heff_%dx%dx%d" % n, n=n, d=(3e-9, 3e-9, 3e-9), Ms=Ms, A=A, Ku=5e4,
                eu=(0.0, 0.0, 1.0), alpha=0.5, H=np.zeros(3), m0=smooth_random(n, 8.0, seed),
                terms=15)


def config_large(n=(512, 512, 64), seed: int = 0):
    """Large-grid case: 512x512x64 cells of 4 nm (16.7 M cells, padded FFT
    1024x1024x128), Ms 1e6, A 1.5e-11, alpha 0.02, Ku 0, H 0, vortex domains."""
    d = (4e-9, 4e-9, 4e-9)
    return dict(name="large_%dx%dx%d" % n, n=n, d=d, Ms=1e6, A=1.5e-11, Ku=0.0,
                eu=(0.0, 0.0, 1.0), alpha=0.02, H=np.zeros(3), m0=vortex_domains(n, d, 16, seed),
                terms=1 | 2)


def config_layers(n=(512, 512, 8), seed: int = 0):
    """Thin-layer case (the non-equidistant form of Sec. 4.4): 512x512 cells
    of 4 nm laterally, 8 layers of heights drawn from U[0.5, 4] nm (a
    multilayer stack with thin spacers), Ms 1e6, A 1.5e-11, alpha 0.02,
    vortex domains."""
    d = (4e-9, 4e-9, 4e-9)
    dz = rng(seed + 1).uniform(0.5e-9, 4e-9, n[2])
    return dict(name="layers_%dx%dx%d" % n, n=n, d=d, dz=dz, Ms=1e6, A=1.5e-11, Ku=0.0,
                eu=(0.0, 0.0, 1.0), alpha=0.02, H=np.zeros(3), m0=vortex_domains(n, d, 16, seed),
                terms=1 | 2)


SERVING_GRIDS = [(64, 64, 1), (128, 128, 2), (256, 64, 4), (256, 256, 8)]


def serving_requests(count: int = 512, seed: int = 0, rate: float = 1.0):
    """Relaxation requests with Poisson arrivals (rate per second): grid drawn
    from SERVING_GRIDS, cubic cell 2-5 nm, Ms in [4e5, 1.4e6], A in
    [5e-12, 2e-11], Ku in [0, 5e4] along z, |B| in [0, 50] mT in a uniform
    random direction, smooth random start (8-cell correlation)."""
    g = rng(seed)
    arrivals = np.cumsum(g.exponential(1.0 / rate, count))
    reqs = []
    for r in range(count):
        n = SERVING_GRIDS[int(g.integers(0, len(SERVING_GRIDS)))]
        c = float(g.uniform(2e-9, 5e-9))
        dirv = g.standard_normal(3)
        dirv /= np.linalg.norm(dirv)
        reqs.append(dict(id=r, arrival=float(arrivals[r]), n=n, d=(c, c, c),
                         Ms=float(g.uniform(4e5, 1.4e6)), A=float(g.uniform(5e-12, 2e-11)),
                         Ku=float(g.uniform(0.0, 5e4)), eu=(0.0, 0.0, 1.0),
                         H=mT(float(g.uniform(0.0, 50.0))) * dirv, seed=int(g.integers(0, 2 ** 31))))
    return reqs


def config_adjoint(seed: int = 0, n=(128, 128, 1)):
    """Differentiation case: 128x128x1 film of 5 nm cells, per-cell density
    rho in [0.5, 1] (Ms = rho * 8e5), A 1.3e-11, alpha 0.05, m0 = x, a 20 mT
    20 GHz drive along y on the strip 16 <= i < 20, 500 RK4 steps of 0.1 ps,
    loss = time average of mean m_z over 96 <= i < 112, 56 <= j < 72."""
    nx, ny, nz = n
    rho = rng(seed).uniform(0.5, 1.0, (nz, ny, nx))
    m0 = np.zeros((3, nz, ny, nx))
    m0[0] = 1.0
    strip = np.zeros((nz, ny, nx), np.uint8)
    strip[:, :, 16:20] = 1
    region = np.zeros((nz, ny, nx), bool)
    region[:, 56:72, 96:112] = True
    return dict(name="adjoint_%dx%dx%d" % n, n=n, d=(5e-9, 5e-9, 5e-9), Ms0=8e5, rho=rho,
                A=1.3e-11, alpha=0.05, m0=m0, drive_amp=np.array([0.0, mT(20.0), 0.0]),
                drive_freq=20e9, strip=strip, region=region, steps=500, dt=1e-13,
                checkpoint_every=50)
