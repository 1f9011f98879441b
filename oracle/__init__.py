"""FP64 CPU oracle of the synchrotron sightline march -- test infrastructure.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never touches it, and it shares no code with that path.

The arithmetic lives in ``sync_oracle.c`` (plain C, FP64, no fast-math); this
module is ctypes marshalling plus ``build()``.  Each C function cites the
passage of Diao et al. (arXiv:2410.01136) it follows.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sync_oracle.c")
_LIB = os.path.join(_HERE, "libsync_oracle.so")
_LIB_SAN = os.path.join(_HERE, "libsync_oracle_san.so")
# SYNC_ORACLE_LIB names another build of the same source to load instead (the
# sanitized one: its process must preload the clang ASan runtime)
_LIB_OVERRIDE = os.environ.get("SYNC_ORACLE_LIB")

MODEL16, GRID, SPHERE, WMAP = 0, 1, 2, 4
NPARAM = 16
SPEC_POWER, SPEC_BROKEN = 0, 1
MAX_FREQ = 16


def build(quiet: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math); with sanitize,
    a second copy with clang under AddressSanitizer and UndefinedBehaviorSanitizer."""
    if sanitize:
        clang = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang")
        out = _LIB_SAN
        cmd = [clang, "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-fno-omit-frame-pointer", "-shared-libsan", "-o", out + ".tmp", _SRC, "-lm"]
    else:
        out = _LIB
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
               "-o", out + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True, capture_output=quiet)
    os.replace(out + ".tmp", out)
    return out


class _Geom(ctypes.Structure):
    _fields_ = [("nside", ctypes.c_int32), ("n_steps", ctypes.c_int32),
                ("r_obs", ctypes.c_double * 3), ("r_max", ctypes.c_double),
                ("box_lo", ctypes.c_double * 3), ("box_hi", ctypes.c_double * 3),
                ("n_freq", ctypes.c_int32), ("freq_hz", ctypes.c_double * MAX_FREQ)]


class _Field(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("theta", ctypes.c_double * NPARAM),
                ("grid_n", ctypes.c_int32 * 3), ("grid_lo", ctypes.c_double * 3),
                ("grid_hi", ctypes.c_double * 3),
                ("grid_bn", ctypes.c_void_p), ("grid_c", ctypes.c_void_p),
                ("te_k", ctypes.c_double), ("grid_alpha", ctypes.c_void_p),
                ("spectrum", ctypes.c_int32), ("alpha_hi", ctypes.c_double),
                ("gamma_break", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _LIB_OVERRIDE:
        lib = ctypes.CDLL(_LIB_OVERRIDE)
    else:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    gp, fp = ctypes.POINTER(_Geom), ctypes.POINTER(_Field)
    lib.or_forward.argtypes = [gp, fp, dp]
    lib.or_forward_pixels.argtypes = [gp, fp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
                                      dp, dp]
    lib.or_adjoint.argtypes = [gp, fp, dp, dp, dp, dp]
    lib.or_pix2zphi_ring.argtypes = [ctypes.c_int32, ctypes.c_int64, dp, dp]
    lib.or_zphi2pix_ring.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double]
    lib.or_zphi2pix_ring.restype = ctypes.c_int64
    lib.or_path_length.argtypes = [gp, dp]
    lib.or_path_length.restype = ctypes.c_double
    for name in ("or_j_I", "or_j_P"):
        getattr(lib, name).argtypes = [ctypes.c_double] * 4
        getattr(lib, name).restype = ctypes.c_double
    lib.or_digamma.argtypes = [ctypes.c_double]
    lib.or_digamma.restype = ctypes.c_double
    lib.or_k_rm.restype = ctypes.c_double
    lib.or_rj.argtypes = [ctypes.c_double]
    lib.or_rj.restype = ctypes.c_double
    lib.or_kff.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.or_kff.restype = ctypes.c_double
    lib.or_fields.argtypes = [fp, dp, dp, dp, dp]
    lib.or_sample_model16.argtypes = [dp, ctypes.POINTER(ctypes.c_int32), dp, dp,
                                      ctypes.c_void_p, ctypes.c_void_p]
    lib.or_num_threads.restype = ctypes.c_int
    lib.or_sample_field.argtypes = [fp, ctypes.POINTER(ctypes.c_int32), dp, dp, ctypes.c_void_p,
                                    ctypes.c_void_p]
    lib.or_set_num_threads.argtypes = [ctypes.c_int]
    for name in ("or_gamma_upper",):
        getattr(lib, name).argtypes = [ctypes.c_double] * 2
        getattr(lib, name).restype = ctypes.c_double
    for name in ("or_synch_F", "or_synch_G", "or_moment_F", "or_moment_G"):
        getattr(lib, name).argtypes = [ctypes.c_double]
        getattr(lib, name).restype = ctypes.c_double
    lib.or_moment_tails.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp]
    lib.or_j_broken.argtypes = [ctypes.c_double] * 6 + [dp]
    lib.or_dj_broken.argtypes = [ctypes.c_double] * 6 + [dp, dp]
    lib.or_midpoints.argtypes = [gp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, dp]
    lib.or_forward_tabulated.argtypes = [gp, ctypes.c_double, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.c_int64, dp, dp]
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_geom(nside, n_steps, freqs_hz, r_obs=(-8.5, 0.0, 0.0), r_max=math.inf,
              box_lo=(-math.inf,) * 3, box_hi=(math.inf,) * 3) -> _Geom:
    g = _Geom()
    g.nside, g.n_steps = int(nside), int(n_steps)
    g.r_obs[:] = [float(v) for v in r_obs]
    g.r_max = float(r_max)
    g.box_lo[:] = [float(v) for v in box_lo]
    g.box_hi[:] = [float(v) for v in box_hi]
    freqs = [float(v) for v in freqs_hz]
    if not 1 <= len(freqs) <= MAX_FREQ:
        raise ValueError("1..16 frequencies")
    g.n_freq = len(freqs)
    g.freq_hz[:len(freqs)] = freqs
    return g


class Field:
    """Field description; keeps the grid arrays alive while in use."""

    def __init__(self, kind, theta, grid_bn=None, grid_c=None, grid_lo=None, grid_hi=None,
                 te_k=0.0, grid_alpha=None, broken=None):
        self.s = _Field()
        self.s.kind = int(kind)
        self.s.te_k = float(te_k)  # > 0: free-free emission and absorption at T_e [K]
        if broken is not None:  # (alpha_hi, gamma_break): broken power law, theta[12] below
            self.s.spectrum = SPEC_BROKEN
            self.s.alpha_hi, self.s.gamma_break = float(broken[0]), float(broken[1])
        th = np.asarray(theta, dtype=np.float64)
        if th.shape != (NPARAM,):
            raise ValueError("theta must have 16 entries")
        self.s.theta[:] = th.tolist()
        self.grid_bn = self.grid_c = None
        if kind == GRID:
            self.grid_bn = np.ascontiguousarray(grid_bn, dtype=np.float32)
            if self.grid_bn.ndim != 4 or self.grid_bn.shape[3] != 4:
                raise ValueError("grid_bn must be [nz][ny][nx][4]")
            nz, ny, nx, _ = self.grid_bn.shape
            self.s.grid_n[:] = [nx, ny, nz]
            self.s.grid_lo[:] = [float(v) for v in grid_lo]
            self.s.grid_hi[:] = [float(v) for v in grid_hi]
            self.s.grid_bn = self.grid_bn.ctypes.data
            if grid_c is not None:
                self.grid_c = np.ascontiguousarray(grid_c, dtype=np.float32)
                if self.grid_c.shape != (nz, ny, nx):
                    raise ValueError("grid_c must be [nz][ny][nx]")
                self.s.grid_c = self.grid_c.ctypes.data
            self.grid_alpha = None
            if grid_alpha is not None:  # spectral index per node (theta[12] unused)
                self.grid_alpha = np.ascontiguousarray(grid_alpha, dtype=np.float32)
                if self.grid_alpha.shape != (nz, ny, nx):
                    raise ValueError("grid_alpha must be [nz][ny][nx]")
                self.s.grid_alpha = self.grid_alpha.ctypes.data


def forward(geom: _Geom, field: Field) -> np.ndarray:
    """Full RING map [n_freq][3][npix] of (T_I, T_Q, T_U) in K, FP64."""
    lib = _load()
    npix = 12 * geom.nside ** 2
    maps = np.zeros((geom.n_freq, 3, npix), dtype=np.float64)
    if lib.or_forward(ctypes.byref(geom), ctypes.byref(field.s), _dptr(maps)) != 0:
        raise ValueError("oracle rejected the geometry or field")
    return maps


def forward_pixels(geom: _Geom, field: Field, pix, want_phi=False):
    """Selected pixels: [n][n_freq][3] in K (and the end Faraday depth)."""
    lib = _load()
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    out = np.zeros((pix.size, geom.n_freq, 3), dtype=np.float64)
    phi = np.zeros(pix.size, dtype=np.float64)
    rc = lib.or_forward_pixels(ctypes.byref(geom), ctypes.byref(field.s),
                               pix.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), pix.size,
                               _dptr(out), _dptr(phi))
    if rc != 0:
        raise ValueError("oracle rejected the request")
    return (out, phi) if want_phi else out


def adjoint(geom: _Geom, field: Field, dmaps, want_grid=False):
    """Gradient of sum(dmaps * maps): (dtheta, dgrid_bn, dgrid_c); dtheta has 16
    entries, or 18 for a broken spectrum (then [12] is the index below the break,
    [16] the index above it, [17] ln gamma_break)."""
    lib = _load()
    dm = np.ascontiguousarray(dmaps, dtype=np.float64)
    npix = 12 * geom.nside ** 2
    if dm.shape != (geom.n_freq, 3, npix):
        raise ValueError("dmaps must be [n_freq][3][npix]")
    dth = np.zeros(NPARAM + 2 if field.s.spectrum == SPEC_BROKEN else NPARAM)
    gbn = gc = None
    nul = ctypes.POINTER(ctypes.c_double)()
    if want_grid and field.s.kind == GRID:
        nz, ny, nx, _ = field.grid_bn.shape
        gbn = np.zeros((nz, ny, nx, 4))
        gc = np.zeros((nz, ny, nx)) if field.grid_c is not None else None
    rc = lib.or_adjoint(ctypes.byref(geom), ctypes.byref(field.s), _dptr(dm), _dptr(dth),
                        _dptr(gbn) if gbn is not None else nul,
                        _dptr(gc) if gc is not None else nul)
    if rc != 0:
        raise ValueError("oracle rejected the request")
    return dth, gbn, gc


def sample_model16(theta, n_xyz, lo, hi):
    """Analytic 16-parameter model on a node-centred grid: (bn [nz][ny][nx][4], c)."""
    lib = _load()
    nx, ny, nz = (int(v) for v in n_xyz)
    bn = np.zeros((nz, ny, nx, 4), dtype=np.float32)
    c = np.zeros((nz, ny, nx), dtype=np.float32)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    n = (ctypes.c_int32 * 3)(nx, ny, nz)
    lo_a = np.ascontiguousarray(lo, dtype=np.float64)
    hi_a = np.ascontiguousarray(hi, dtype=np.float64)
    if lib.or_sample_model16(_dptr(th), n, _dptr(lo_a), _dptr(hi_a), bn.ctypes.data,
                             c.ctypes.data) != 0:
        raise ValueError("bad grid shape")
    return bn, c


def sample_field(field: Field, n_xyz, lo, hi):
    """Any field kind on a node-centred grid: (bn [nz][ny][nx][4], c [nz][ny][nx])."""
    lib = _load()
    nx, ny, nz = (int(v) for v in n_xyz)
    bn = np.zeros((nz, ny, nx, 4), dtype=np.float32)
    c = np.zeros((nz, ny, nx), dtype=np.float32)
    n = (ctypes.c_int32 * 3)(nx, ny, nz)
    lo_a = np.ascontiguousarray(lo, dtype=np.float64)
    hi_a = np.ascontiguousarray(hi, dtype=np.float64)
    if lib.or_sample_field(ctypes.byref(field.s), n, _dptr(lo_a), _dptr(hi_a), bn.ctypes.data,
                           c.ctypes.data) != 0:
        raise ValueError("bad grid shape")
    return bn, c


def pix2zphi(nside: int, p: int):
    lib = _load()
    z, phi = ctypes.c_double(), ctypes.c_double()
    lib.or_pix2zphi_ring(int(nside), int(p), ctypes.byref(z), ctypes.byref(phi))
    return z.value, phi.value


def zphi2pix(nside: int, z: float, phi: float) -> int:
    return int(_load().or_zphi2pix_ring(int(nside), float(z), float(phi)))


def fields_at(field: Field, r):
    lib = _load()
    r = np.ascontiguousarray(r, dtype=np.float64)
    B = np.zeros(3)
    ne, n0 = ctypes.c_double(), ctypes.c_double()
    lib.or_fields(ctypes.byref(field.s), _dptr(r), _dptr(B),
                  ctypes.cast(ctypes.byref(ne), ctypes.POINTER(ctypes.c_double)),
                  ctypes.cast(ctypes.byref(n0), ctypes.POINTER(ctypes.c_double)))
    return B, ne.value, n0.value


def path_length(geom: _Geom, nhat) -> float:
    n = np.ascontiguousarray(nhat, dtype=np.float64)
    return _load().or_path_length(ctypes.byref(geom), _dptr(n))


def j_I(alpha, nu, bt_gauss, n0):
    return _load().or_j_I(alpha, nu, bt_gauss, n0)


def j_P(alpha, nu, bt_gauss, n0):
    return _load().or_j_P(alpha, nu, bt_gauss, n0)


def gamma_upper(a, y):
    """Upper incomplete gamma function Gamma(a, y) (not regularised)."""
    return _load().or_gamma_upper(a, y)


def synch_F(x):
    """F(x) = x int_x^inf K_5/3(z) dz."""
    return _load().or_synch_F(x)


def synch_G(x):
    """G(x) = x K_2/3(x)."""
    return _load().or_synch_G(x)


def moment_F(mu):
    return _load().or_moment_F(mu)


def moment_G(mu):
    return _load().or_moment_G(mu)


def moment_tails(alpha, xb):
    """Shares (tF, tG) of the x-moments of order (alpha - 3) / 2 of F and G
    above xb."""
    a, b = ctypes.c_double(), ctypes.c_double()
    _load().or_moment_tails(alpha, xb, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def j_broken(a1, a2, gamma_break, nu, bt_gauss, n0):
    """(j_I, j_P, dj_I/dbt, dj_P/dbt) of the broken power-law spectrum."""
    out = np.zeros(4)
    _load().or_j_broken(a1, a2, gamma_break, nu, bt_gauss, n0, _dptr(out))
    return out


def dj_broken(a1, a2, gamma_break, nu, bt_gauss, n0):
    """d(j_I, j_P)/d(a1, a2, ln gamma_break): two arrays of 3."""
    dI, dP = np.zeros(3), np.zeros(3)
    _load().or_dj_broken(a1, a2, gamma_break, nu, bt_gauss, n0, _dptr(dI), _dptr(dP))
    return dI, dP


def digamma(x):
    return _load().or_digamma(x)


def k_rm():
    return _load().or_k_rm()


def rayleigh_jeans(nu):
    return _load().or_rj(nu)


def kff(nu, te_k):
    """Free-free optical depth per pc per (n_e / cm^-3)^2."""
    return _load().or_kff(nu, te_k)


def num_threads():
    return _load().or_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (n >= 1)."""
    _load().or_set_num_threads(int(n))


def midpoints(geom: _Geom, pix) -> np.ndarray:
    """Sightline midpoints [n][n_steps][3] (kpc) of the given pixels."""
    lib = _load()
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    out = np.zeros((pix.size, geom.n_steps, 3))
    if lib.or_midpoints(ctypes.byref(geom), pix.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                        pix.size, _dptr(out)) != 0:
        raise ValueError("oracle rejected the request")
    return out


def forward_tabulated(geom: _Geom, alpha: float, pix, fields) -> np.ndarray:
    """The march over given field samples fields[n][n_steps][5] -> [n][n_freq][3] (K)."""
    lib = _load()
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    fl = np.ascontiguousarray(fields, dtype=np.float64)
    if fl.shape != (pix.size, geom.n_steps, 5):
        raise ValueError("fields must be [n_pix][n_steps][5]")
    out = np.zeros((pix.size, geom.n_freq, 3))
    if lib.or_forward_tabulated(ctypes.byref(geom), float(alpha),
                                pix.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), pix.size,
                                _dptr(fl), _dptr(out)) != 0:
        raise ValueError("oracle rejected the request")
    return out
