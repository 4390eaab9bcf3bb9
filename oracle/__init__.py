"""CPU oracle for the micromagnetic hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library
(``paper_2302_08843_amd``) never imports, links or calls it; the two share no
source.  The C implementation lives in ``mmref.c`` (plain FP64 with a
long-double Newell tensor) and is loaded here with ctypes.

Arrays crossing this wrapper are float64, C-contiguous, shape ``(3, nz, ny, nx)``
(component-major, x fastest), the same cell order the paper's grid uses
(Sec. 2, cell centre x0 + (i dx, j dy, k dz)).

Parity status per function (what pins it) is documented in each docstring and
in the oracle tests under ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mmref.c")
_LIB = os.path.join(_HERE, "liboracle.so")

DEMAG, EXCH, ANIS, ZEEMAN, DMI, OERSTED = 1, 2, 4, 8, 16, 32
ALL = DEMAG | EXCH | ANIS | ZEEMAN | DMI | OERSTED
DMI_INTERFACE, DMI_BULK, DMI_D2D = 0, 1, 2
MU0 = 4.0e-7 * np.pi
GAMMA = 2.21e5

OK, ENONFINITE, EDTMIN, ENOTCONV = 0, -4, -5, -6


def build(force: bool = True) -> str:
    """Compile mmref.c into liboracle.so with gcc (no -ffast-math; x87 long
    double for the tensor)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


class _Stats(C.Structure):
    _fields_ = [("accepted", C.c_long), ("rejected", C.c_long), ("rhs_evals", C.c_long),
                ("t", C.c_double), ("dt", C.c_double), ("err_last", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.or_newell.argtypes = [dp, C.c_long, C.c_long, C.c_long, dp]
        L.or_dipole.argtypes = [dp, C.c_long, C.c_long, C.c_long, dp]
        L.or_tensor_entry.argtypes = [dp, C.c_long, C.c_long, C.c_long, C.c_int, dp]
        L.or_demag_at.argtypes = [C.POINTER(C.c_long), dp, C.c_int, C.c_void_p, C.c_double, dp,
                                  C.c_long, C.POINTER(C.c_long), dp]
        L.or_demag_at.restype = C.c_int
        L.or_fft1d.argtypes = [C.c_long, C.c_void_p, C.c_int]
        L.or_dft1d.argtypes = [C.c_long, C.c_void_p, C.c_void_p, C.c_int]
        L.or_padded.argtypes = [C.c_long]
        L.or_padded.restype = C.c_long
        L.or_create.argtypes = [C.POINTER(C.c_long), dp, C.c_int, dp, dp, C.c_double, dp,
                                C.c_double, C.c_int]
        L.or_create.restype = C.c_void_p
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_set_field.argtypes = [C.c_void_p, dp, C.c_uint]
        L.or_set_drive.argtypes = [C.c_void_p, dp, C.c_double, C.c_void_p]
        L.or_set_Ms.argtypes = [C.c_void_p, dp]
        L.or_set_anisotropy2.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, dp, dp]
        L.or_set_dmi.argtypes = [C.c_void_p, C.c_void_p, C.c_int]
        L.or_set_layers.argtypes = [C.c_void_p, C.c_void_p]
        L.or_set_ku.argtypes = [C.c_void_p, C.c_void_p]
        L.or_oersted_entry.argtypes = [dp, C.c_long, C.c_long, C.c_long, C.c_int, dp]
        L.or_oersted.argtypes = [C.c_void_p, dp, dp]
        L.or_oersted.restype = C.c_int
        L.or_set_current.argtypes = [C.c_void_p, C.c_void_p, C.c_double]
        L.or_set_current.restype = C.c_int
        L.or_oersted_at.argtypes = [C.POINTER(C.c_long), dp, C.c_int, dp, C.c_long,
                                    C.POINTER(C.c_long), dp]
        L.or_oersted_at.restype = C.c_int
        L.or_layer_demag_at.argtypes = [C.POINTER(C.c_long), dp, dp, C.c_int, C.c_void_p,
                                        C.c_double, dp, C.c_long, C.POINTER(C.c_long), dp]
        L.or_layer_demag_at.restype = C.c_int
        L.or_newell_box.argtypes = [C.c_double, C.c_double, C.c_long, C.c_long, C.c_double,
                                    C.c_double, C.c_double, dp]
        L.or_layer_entry.argtypes = [C.c_double, C.c_double, dp, C.c_long, C.c_long, C.c_long,
                                     C.c_long, C.c_int, dp]
        for name in ("or_demag", "or_exchange", "or_anisotropy", "or_dmi"):
            getattr(L, name).argtypes = [C.c_void_p, dp, dp]
        L.or_zeeman.argtypes = [C.c_void_p, C.c_double, dp]
        L.or_heff.argtypes = [C.c_void_p, dp, C.c_double, C.c_uint, dp]
        L.or_llg_rhs.argtypes = [C.c_void_p, dp, dp, C.c_double, C.c_int, dp]
        L.or_energy.argtypes = [C.c_void_p, dp, C.c_double, dp]
        L.or_dp45.argtypes = [C.c_void_p, dp, dp, dp, C.c_double, C.c_double, C.c_double,
                              C.c_long, C.c_int, C.c_int, C.c_double, C.c_int,
                              C.POINTER(_Stats), C.c_double]
        L.or_dp45.restype = C.c_int
        L.or_rk_adaptive.argtypes = [C.c_void_p, C.c_int, dp, dp, dp, C.c_double, C.c_double,
                                     C.c_double, C.c_long, C.c_int, C.c_int, C.c_double, C.c_int,
                                     C.POINTER(_Stats), C.c_double]
        L.or_rk_adaptive.restype = C.c_int
        L.or_relax.argtypes = [C.c_void_p, dp, C.c_double, C.c_long, C.c_double, C.POINTER(_Stats)]
        L.or_relax.restype = C.c_int
        L.or_max_torque.argtypes = [C.c_void_p, dp, C.c_double]
        L.or_max_torque.restype = C.c_double
        L.or_num_threads.restype = C.c_int
        L.or_set_threads.argtypes = [C.c_int]
        L.or_set_threads.restype = None
        L.or_heff_vjp.argtypes = [C.c_void_p, dp, dp, C.c_uint, dp, dp]
        L.or_llg_jvp.argtypes = [C.c_void_p, dp, dp, C.c_double, dp]
        L.or_llg_vjp.argtypes = [C.c_void_p, dp, C.c_double, dp, dp, dp]
        L.or_rk4.argtypes = [C.c_void_p, dp, C.c_double, C.c_double, C.c_long, C.c_void_p]
        L.or_rk4.restype = C.c_double
        L.or_rk4_adjoint.argtypes = [C.c_void_p, dp, C.c_double, C.c_double, C.c_long, C.c_void_p,
                                     dp, dp]
        L.or_rk4_adjoint.restype = C.c_double
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _d3(v) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(3))


def newell(d, I, J, K) -> np.ndarray:
    """Newell's cell-averaged tensor N (self term +1/3 for a cube), order
    xx, yy, zz, xy, xz, yz.  Pinned: cube self term, trace, Aharoni, dipole
    limit."""
    out = np.zeros(6)
    lib().or_newell(_dp(_d3(d)), int(I), int(J), int(K), _dp(out))
    return out


def dipole(d, I, J, K) -> np.ndarray:
    """Point-dipole kernel of Eq. (dipole) (positive sign, multiplies M)."""
    out = np.zeros(6)
    lib().or_dipole(_dp(_d3(d)), int(I), int(J), int(K), _dp(out))
    return out


def tensor_entry(d, I, J, K, p=20) -> np.ndarray:
    """Demag kernel K (h = K M): -Newell within Chebyshev index distance p,
    dipole beyond (Sec. 4.4)."""
    out = np.zeros(6)
    lib().or_tensor_entry(_dp(_d3(d)), int(I), int(J), int(K), int(p), _dp(out))
    return out


def demag_at(n, d, m, cells, Ms=1.0, p=20) -> np.ndarray:
    """Demag field at the given linear cell indices by direct summation over
    every source cell (no padded grid): shape (len(cells), 3).  Ms is a
    scalar or an (nz, ny, nx) array; m is (3, nz, ny, nx)."""
    nn = (C.c_long * 3)(*[int(v) for v in n])
    m = np.ascontiguousarray(np.asarray(m, dtype=np.float64))
    cl = np.ascontiguousarray(np.asarray(cells, dtype=np.int64))
    out = np.zeros((len(cl), 3))
    if np.ndim(Ms) == 0:
        ms_ptr, ms0 = None, float(Ms)
    else:
        msa = np.ascontiguousarray(np.asarray(Ms, dtype=np.float64))
        ms_ptr, ms0 = msa.ctypes.data, 0.0
    rc = lib().or_demag_at(nn, _dp(_d3(d)), int(p), ms_ptr, ms0, _dp(m), len(cl),
                           cl.ctypes.data_as(C.POINTER(C.c_long)), _dp(out))
    if rc != 0:
        raise ValueError("or_demag_at needs p >= 0")
    return out


def newell_box(dx, dy, I, J, Bz, ct, cs) -> np.ndarray:
    """Newell tensor between a target cell of height ct and a source cell of
    height cs whose bottom is Bz above the target's bottom, laterally offset by
    (I dx, J dy) (source minus target).  Order xx, yy, zz, xy, xz, yz."""
    out = np.zeros(6)
    lib().or_newell_box(float(dx), float(dy), int(I), int(J), float(Bz), float(ct), float(cs),
                        _dp(out))
    return out


def layer_entry(dx, dy, dz, t, s, I, J, p=20) -> np.ndarray:
    """Layered demag kernel K^{ts}(I, J) (h_t = sum K M_s; I = i_t - i_s) for
    layer heights dz stacked from 0."""
    zb = np.concatenate([[0.0], np.cumsum(np.asarray(dz, dtype=np.float64))])
    out = np.zeros(6)
    lib().or_layer_entry(float(dx), float(dy), _dp(zb), int(t), int(s), int(I), int(J), int(p),
                         _dp(out))
    return out


def oersted_entry(d, I, J, K, p=20) -> np.ndarray:
    """Oersted kernel G (h_t = sum_s j_s x G(X_t - X_s)) for the cell offset
    (I, J, K) (target minus source): the cell-averaged Biot-Savart vector
    within Chebyshev index distance p, the singular current beyond."""
    out = np.zeros(3)
    lib().or_oersted_entry(_dp(_d3(d)), int(I), int(J), int(K), int(p), _dp(out))
    return out


def oersted_at(n, d, j, cells, p=20) -> np.ndarray:
    """Oersted field of the current density j ((3, nz, ny, nx)) at the given
    linear cell indices by direct summation over every source cell: shape
    (len(cells), 3)."""
    nn = (C.c_long * 3)(*[int(v) for v in n])
    j = np.ascontiguousarray(np.asarray(j, dtype=np.float64))
    cl = np.ascontiguousarray(np.asarray(cells, dtype=np.int64))
    out = np.zeros((len(cl), 3))
    if lib().or_oersted_at(nn, _dp(_d3(d)), int(p), _dp(j), len(cl),
                           cl.ctypes.data_as(C.POINTER(C.c_long)), _dp(out)) != 0:
        raise ValueError("or_oersted_at needs p >= 0")
    return out


def layer_demag_at(n, d, dz, m, cells, Ms=1.0, p=20) -> np.ndarray:
    """Demag field of thin layers of heights dz at the given linear cell
    indices by direct summation: shape (len(cells), 3)."""
    nn = (C.c_long * 3)(*[int(v) for v in n])
    m = np.ascontiguousarray(np.asarray(m, dtype=np.float64))
    dzl = np.ascontiguousarray(np.asarray(dz, dtype=np.float64))
    cl = np.ascontiguousarray(np.asarray(cells, dtype=np.int64))
    out = np.zeros((len(cl), 3))
    if np.ndim(Ms) == 0:
        ms_ptr, ms0 = None, float(Ms)
    else:
        msa = np.ascontiguousarray(np.asarray(Ms, dtype=np.float64))
        ms_ptr, ms0 = msa.ctypes.data, 0.0
    if lib().or_layer_demag_at(nn, _dp(_d3(d)), _dp(dzl), int(p), ms_ptr, ms0, _dp(m), len(cl),
                               cl.ctypes.data_as(C.POINTER(C.c_long)), _dp(out)) != 0:
        raise ValueError("or_layer_demag_at needs p >= 0")
    return out


def padded(n: int) -> int:
    """Zero-padding extent: 1 for n == 1, else next power of two >= 2n-1."""
    return int(lib().or_padded(int(n)))


def fft1d(x, sign=-1) -> np.ndarray:
    """Radix-2 FFT (unnormalised); pinned by dft1d."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.complex128).copy())
    lib().or_fft1d(a.size, a.ctypes.data, int(sign))
    return a


def dft1d(x, sign=-1) -> np.ndarray:
    """Naive DFT with long-double accumulation (the definition)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    out = np.zeros_like(a)
    lib().or_dft1d(a.size, a.ctypes.data, out.ctypes.data, int(sign))
    return out


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_threads(n: int) -> None:
    """Threads of the following oracle calls (timing only)."""
    lib().or_set_threads(int(n))


class Oracle:
    """One problem: grid n = (nx, ny, nz), cell d (m), material, demag kernel.

    Ms and A may be scalars or per-cell arrays of shape (nz, ny, nx).  p is the
    Newell near-field radius in cells (p < 0: Newell everywhere).  direct=True
    evaluates demag as the O(N^2) direct sum instead of the FFT convolution.
    """

    def __init__(self, n, d, Ms, A=0.0, Ku=0.0, eu=(0, 0, 1), alpha=0.5, p=20, direct=False,
                 layers=None, demag=True):
        self.n = tuple(int(v) for v in n)
        self.d = tuple(float(v) for v in d)
        nx, ny, nz = self.n
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.Ms = np.ascontiguousarray(np.broadcast_to(np.asarray(Ms, np.float64), self.shape).copy())
        self.A = np.ascontiguousarray(np.broadcast_to(np.asarray(A, np.float64), self.shape).copy())
        self.alpha = float(alpha)
        self.V = self.d[0] * self.d[1] * self.d[2]
        nn = (C.c_long * 3)(*self.n)
        # demag=False: no demag kernel (local terms only; the demag field reads NaN)
        mode = 2 if not demag else int(bool(direct))
        self._c = lib().or_create(nn, _dp(_d3(self.d)), int(p), _dp(self.Ms), _dp(self.A),
                                  float(Ku), _dp(_d3(eu)), self.alpha, mode)
        self.Hext = np.zeros(3)
        self.terms = ALL
        self.layers = None
        if layers is not None:
            self.set_layers(layers)

    def set_ku(self, Ku):
        """Per-cell first-order uniaxial constant (scalar or (nz, ny, nx));
        None restores the uniform Ku."""
        if Ku is None:
            lib().or_set_ku(self._c, None)
            return
        self.Kuc = np.ascontiguousarray(np.broadcast_to(np.asarray(Ku, np.float64), self.shape).copy())
        lib().or_set_ku(self._c, self.Kuc.ctypes.data)

    def set_layers(self, dz):
        """Thin layers of heights dz[0..nz) (the non-equidistant case of
        Sec. 4.4); None restores equal layers of height d[2]."""
        if dz is None:
            self.layers = None
            lib().or_set_layers(self._c, None)
            return
        self.layers = np.ascontiguousarray(np.asarray(dz, dtype=np.float64).reshape(self.n[2]))
        lib().or_set_layers(self._c, self.layers.ctypes.data)

    def __del__(self):
        if getattr(self, "_c", None):
            lib().or_destroy(self._c)
            self._c = None

    def _m(self, m) -> np.ndarray:
        a = np.ascontiguousarray(np.asarray(m, dtype=np.float64))
        assert a.shape == (3,) + self.shape, a.shape
        return a

    def set_field(self, H, terms=ALL):
        """Uniform external field H (A/m) and the term mask used by heff /
        rhs / dp45 / relax / energy."""
        self.Hext = _d3(H)
        self.terms = int(terms)
        lib().or_set_field(self._c, _dp(self.Hext), self.terms)

    def set_drive(self, amp, freq, mask):
        """Add H += mask * amp * sin(2 pi freq t) to the Zeeman term."""
        mk = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(self.shape))
        lib().or_set_drive(self._c, _dp(_d3(amp)), float(freq), mk.ctypes.data)

    def set_anisotropy2(self, Ku2=0.0, Kc1=0.0, Kc2=0.0, c1=(1, 0, 0), c2=(0, 1, 0)):
        """Second-order uniaxial (Ku2, along the Ku axis) and cubic (Kc1, Kc2,
        principal axes c1, c2, c1 x c2) anisotropy (Sec. 4.3)."""
        lib().or_set_anisotropy2(self._c, float(Ku2), float(Kc1), float(Kc2), _dp(_d3(c1)),
                                 _dp(_d3(c2)))

    def set_dmi(self, D, kind=DMI_INTERFACE):
        """DMI strength D (J/m^2, scalar or per-cell) of one of the tabulated
        types (Sec. 4.3): DMI_INTERFACE, DMI_BULK or DMI_D2D.  D=None removes
        the term."""
        if D is None:
            lib().or_set_dmi(self._c, None, 0)
            return
        self.D = np.ascontiguousarray(np.broadcast_to(np.asarray(D, np.float64), self.shape).copy())
        lib().or_set_dmi(self._c, self.D.ctypes.data, int(kind))

    def set_Ms(self, Ms):
        self.Ms = np.ascontiguousarray(np.broadcast_to(np.asarray(Ms, np.float64), self.shape).copy())
        lib().or_set_Ms(self._c, _dp(self.Ms))

    def _field(self, name, m):
        m = self._m(m)
        h = np.zeros_like(m)
        getattr(lib(), name)(self._c, _dp(m), _dp(h))
        return h

    def demag(self, m):
        """h_dem = sum_j K_{i-j} Ms_j m_j (Sec. 4.4)."""
        return self._field("or_demag", m)

    def exchange(self, m):
        """Harmonic-mean exchange field (Sec. 4.2)."""
        return self._field("or_exchange", m)

    def anisotropy(self, m):
        """First-order uniaxial anisotropy field (Sec. 4.1)."""
        return self._field("or_anisotropy", m)

    def oersted(self, j):
        """Oersted field (Sec. 4.5) of the current density j (A/m^2,
        (3, nz, ny, nx)) at every cell, by direct summation."""
        j = self._m(j)
        h = np.zeros_like(j)
        if lib().or_oersted(self._c, _dp(j), _dp(h)) != 0:
            raise ValueError("the Oersted field needs equal layers")
        return h

    def set_current(self, j, freq=0.0):
        """Current density for the OERSTED term: its field, times
        sin(2 pi freq t) if freq != 0, joins the effective field on magnetic
        cells (and the Zeeman energy).  None removes it."""
        if j is None:
            lib().or_set_current(self._c, None, 0.0)
            return
        self._j = self._m(j).copy()
        if lib().or_set_current(self._c, self._j.ctypes.data, float(freq)) != 0:
            raise ValueError("the Oersted field needs equal layers")

    def dmi(self, m):
        """DMI field by central differences with the averaged coupling D~
        (Sec. 4.3, Eq. D_avg); missing and vacuum neighbours are ignored."""
        return self._field("or_dmi", m)

    def zeeman(self, t=0.0):
        h = np.zeros((3,) + self.shape)
        lib().or_zeeman(self._c, float(t), _dp(h))
        return h

    def heff(self, m, t=0.0, terms=None):
        m = self._m(m)
        h = np.zeros_like(m)
        lib().or_heff(self._c, _dp(m), float(t), int(self.terms if terms is None else terms), _dp(h))
        return h

    def llg_rhs(self, m, h, alpha=None, precess=True):
        """Eq. (llg) right-hand side."""
        m = self._m(m)
        h = self._m(h)
        dm = np.zeros_like(m)
        lib().or_llg_rhs(self._c, _dp(m), _dp(h), float(self.alpha if alpha is None else alpha),
                         int(bool(precess)), _dp(dm))
        return dm

    def energy(self, m, t=0.0) -> np.ndarray:
        """[E_demag, E_exchange, E_anisotropy, E_zeeman, E_total, E_dmi] in J
        (the total includes the DMI energy)."""
        m = self._m(m)
        E = np.zeros(6)
        lib().or_energy(self._c, _dp(m), float(t), _dp(E))
        return E

    def dp45(self, m, t=0.0, dt=-1.0, rtol=1e-6, atol=None, t_end=np.inf, max_steps=1 << 40,
             renorm=False, precess=True, alpha=None, fixed=False, torque_tol=0.0, method=0):
        """Adaptive embedded Runge-Kutta integration (method 0: Dormand-Prince
        5(4), 1: Runge-Kutta-Fehlberg 4(5)); returns (m, t, dt, stats, status)."""
        y = self._m(m).copy()
        tt = C.c_double(t)
        dd = C.c_double(dt)
        st = _Stats()
        status = lib().or_rk_adaptive(self._c, int(method), _dp(y), C.byref(tt), C.byref(dd),
                                      float(rtol), float(rtol if atol is None else atol),
                                      float(t_end), int(max_steps), int(bool(renorm)),
                                      int(bool(precess)),
                                      float(self.alpha if alpha is None else alpha),
                                      int(bool(fixed)), C.byref(st), float(torque_tol))
        stats = dict(accepted=st.accepted, rejected=st.rejected, rhs_evals=st.rhs_evals,
                     t=st.t, dt=st.dt, err_last=st.err_last)
        return y, tt.value, dd.value, stats, status

    def rkf45(self, m, **kw):
        """Runge-Kutta-Fehlberg 4(5), the paper's default integrator (Sec. 3)."""
        return self.dp45(m, method=1, **kw)

    def relax(self, m, tol=1e-5, max_steps=50000, rtol=1e-4):
        """Precession-free alpha = 1 relaxation (Sec. 3) until the maximum
        torque |m x h|/Ms < tol; returns (m, stats, status)."""
        y = self._m(m).copy()
        st = _Stats()
        status = lib().or_relax(self._c, _dp(y), float(tol), int(max_steps), float(rtol), C.byref(st))
        stats = dict(accepted=st.accepted, rejected=st.rejected, rhs_evals=st.rhs_evals,
                     t=st.t, dt=st.dt, err_last=st.err_last)
        return y, stats, status

    def max_torque(self, m, t=0.0) -> float:
        return float(lib().or_max_torque(self._c, _dp(self._m(m)), float(t)))

    # ------------------------------------------------------------------
    # differentiation (inverse design, Sec. 5.2)
    # ------------------------------------------------------------------
    def heff_vjp(self, m, w, terms=DEMAG | EXCH | ANIS):
        """(H^T w, d(w.h)/dMs) for the linear field terms in `terms`."""
        m, w = self._m(m), self._m(w)
        gm = np.zeros_like(m)
        gms = np.zeros(self.shape)
        lib().or_heff_vjp(self._c, _dp(m), _dp(w), int(terms), _dp(gm), _dp(gms))
        return gm, gms

    def llg_jvp(self, m, v, t=0.0):
        """Exact Jacobian-vector product of the LLG right-hand side."""
        m, v = self._m(m), self._m(v)
        out = np.zeros_like(m)
        lib().or_llg_jvp(self._c, _dp(m), _dp(v), float(t), _dp(out))
        return out

    def llg_vjp(self, m, w, t=0.0):
        """(J^T w, d(w.f)/dMs) of the LLG right-hand side at (m, t)."""
        m, w = self._m(m), self._m(w)
        gm = np.zeros_like(m)
        gms = np.zeros(self.shape)
        lib().or_llg_vjp(self._c, _dp(m), float(t), _dp(w), _dp(gm), _dp(gms))
        return gm, gms

    def rk4(self, m0, dt, nsteps, region, t0=0.0):
        """Classical RK4; returns (m, loss) with loss = time average of the
        region mean of m_z over the nsteps steps."""
        m = self._m(m0).copy()
        reg = np.ascontiguousarray(np.asarray(region, dtype=np.uint8).reshape(self.shape))
        loss = lib().or_rk4(self._c, _dp(m), float(t0), float(dt), int(nsteps), reg.ctypes.data)
        return m, loss

    def rk4_adjoint(self, m0, dt, nsteps, region, t0=0.0):
        """(loss, dloss/dMs per cell, dloss/dm0) by the discrete adjoint."""
        m0 = self._m(m0)
        reg = np.ascontiguousarray(np.asarray(region, dtype=np.uint8).reshape(self.shape))
        gms = np.zeros(self.shape)
        gm0 = np.zeros_like(m0)
        loss = lib().or_rk4_adjoint(self._c, _dp(m0), float(t0), float(dt), int(nsteps),
                                    reg.ctypes.data, _dp(gms), _dp(gm0))
        return loss, gms, gm0
