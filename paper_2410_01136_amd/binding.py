"""Thin Python binding of libsynmarch.so (the C ABI in include/synmarch.h).

Argument marshalling only: every step of the march runs in the HIP kernels.
PyTorch supplies device memory and the current stream.  If the library is
missing the import of this module fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# SYNMARCH_LIB names another build of the same sources to load instead (the
# host-sanitized one: its process must preload the clang ASan runtime)
LIB_PATH = os.environ.get("SYNMARCH_LIB") or os.path.join(_HERE, "libsynmarch.so")

SYN_OK, SYN_EINVAL, SYN_EUNSUPPORTED, SYN_ENOMEM, SYN_EHIP, SYN_EWORKSPACE = 0, -1, -2, -3, -4, -5
FIELD_MODEL16, FIELD_GRID, FIELD_SPHERE, FIELD_MLP, FIELD_WMAP = 0, 1, 2, 3, 4
KERNEL_FORWARD, KERNEL_ADJOINT, KERNEL_BATCH = 0, 1, 2
SPEC_POWER_LAW, SPEC_BROKEN = 0, 1
NPARAM, MAX_FREQ = 16, 16

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "(or python -m paper_2410_01136_amd._build); there is no CPU fallback")
_lib = ctypes.CDLL(LIB_PATH)


class SynGeom(ctypes.Structure):
    _fields_ = [("nside", ctypes.c_int32), ("n_steps", ctypes.c_int32),
                ("r_obs_kpc", ctypes.c_double * 3), ("r_max_kpc", ctypes.c_double),
                ("box_lo_kpc", ctypes.c_double * 3), ("box_hi_kpc", ctypes.c_double * 3),
                ("n_freq", ctypes.c_int32), ("freq_hz", ctypes.c_double * MAX_FREQ)]


class SynField(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("theta", ctypes.c_double * NPARAM),
                ("grid_n", ctypes.c_int32 * 3), ("grid_lo_kpc", ctypes.c_double * 3),
                ("grid_hi_kpc", ctypes.c_double * 3), ("grid_bn", ctypes.c_void_p),
                ("grid_c", ctypes.c_void_p), ("mlp", ctypes.c_void_p),
                ("te_k", ctypes.c_double), ("grid_alpha", ctypes.c_void_p),
                ("spectrum", ctypes.c_int32), ("alpha_hi", ctypes.c_double),
                ("gamma_break", ctypes.c_double), ("spectrum_table", ctypes.c_void_p)]


class SynBatchDesc(ctypes.Structure):
    _fields_ = [("n_sets", ctypes.c_int32), ("nside", ctypes.POINTER(ctypes.c_int32)),
                ("theta", ctypes.POINTER(ctypes.c_double)), ("geom", SynGeom),
                ("use_graph", ctypes.c_int32), ("kind", ctypes.c_int32)]


_vp, _i32, _i64, _sz, _dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, \
    ctypes.POINTER(ctypes.c_double)
_G, _F = ctypes.POINTER(SynGeom), ctypes.POINTER(SynField)


def _sig(name, res, args):
    fn = getattr(_lib, name)
    fn.restype = res
    fn.argtypes = args
    return fn


syn_version = _sig("syn_version", _i32, [])
syn_last_error = _sig("syn_last_error", ctypes.c_char_p, [])
syn_workspace_bytes = _sig("syn_workspace_bytes", _sz, [_G, _F, _i32])
syn_forward = _sig("syn_forward", _i32, [_G, _F, _vp, _vp, _sz, _vp])
syn_adjoint = _sig("syn_adjoint", _i32, [_G, _F, _vp, _vp, _sz, _vp, _vp, _vp, _vp])
syn_spectrum_table_bytes = _sig("syn_spectrum_table_bytes", _sz, [])
syn_spectrum_table = _sig("syn_spectrum_table", _i32,
                          [ctypes.c_double, ctypes.c_double, _vp, _sz, _vp])
syn_spectrum_table_host = _sig("syn_spectrum_table_host", _i32,
                               [ctypes.c_double, ctypes.c_double, _vp, _sz])
syn_chi2_workspace_bytes = _sig("syn_chi2_workspace_bytes", _sz, [_i64, _i32])
syn_chi2 = _sig("syn_chi2", _i32, [_i64, _i32, _vp, _vp, _dp, _vp, _vp, _vp, _sz, _vp])
syn_chi2_cotangent = _sig("syn_chi2_cotangent", _i32, [_i64, _i32, _vp, _vp, _dp, _vp, _vp, _vp])
syn_sample_model16 = _sig("syn_sample_model16", _i32,
                          [_dp, ctypes.POINTER(_i32), _dp, _dp, _vp, _vp, _vp])
syn_eval_fields = _sig("syn_eval_fields", _i32, [_F, _i64, _vp, _vp, _vp])
syn_mlp_packed_bytes = _sig("syn_mlp_packed_bytes", _sz, [])
syn_mlp_pack = _sig("syn_mlp_pack", _i32, [_vp] * 8)
syn_batch_create = _sig("syn_batch_create", _i32,
                        [ctypes.POINTER(SynBatchDesc), ctypes.POINTER(_vp)])
syn_batch_total_pixels = _sig("syn_batch_total_pixels", _i64, [_vp])
syn_batch_offset = _sig("syn_batch_offset", _i64, [_vp, _i32])
syn_batch_run = _sig("syn_batch_run", _i32, [_vp, _vp, _dp, _vp, _vp, _vp, _vp, _vp])
syn_batch_set_theta = _sig("syn_batch_set_theta", _i32, [_vp, _dp, _vp])
syn_batch_destroy = _sig("syn_batch_destroy", None, [_vp])
syn_set_lanes_per_ray = _sig("syn_set_lanes_per_ray", _i32, [_i32, _i32, _i32])
syn_get_lanes_per_ray = _sig("syn_get_lanes_per_ray", _i32, [_i32, _i32, _i64])
syn_set_grid_addressing = _sig("syn_set_grid_addressing", _i32, [_i32])
syn_adam_step = _sig("syn_adam_step", _i32, [_i64, _i32, ctypes.c_uint32, _vp, _vp, _vp, _vp,
                                             _i32, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, _vp])
syn_get_grid_addressing = _sig("syn_get_grid_addressing", _i32, [])
syn_autotune_load = _sig("syn_autotune_load", _i32, [ctypes.c_char_p])
syn_autotune_clear = _sig("syn_autotune_clear", None, [])
syn_autotune_entries = _sig("syn_autotune_entries", _i32, [])
syn_autotune_lookup = _sig("syn_autotune_lookup", _i32, [_i32, _i32, _i64, _i32, _i32,
                                                         ctypes.POINTER(_i32), ctypes.POINTER(_i32)])
syn_build_id = _sig("syn_build_id", ctypes.c_char_p, [])
syn_host_nest_pixel = _sig("syn_host_nest_pixel", _i32,
                           [_i32, _i64, ctypes.POINTER(_i64), _dp, _dp])


class SynError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = syn_last_error().decode(errors="replace")
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != SYN_OK:
        raise SynError(status, where)


def _stream(stream=None) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _dev_f32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    return t


# --------------------------------------------------------------------------- descriptors

def make_geom(nside: int, n_steps: int, freqs_hz: Sequence[float], r_obs=(-8.5, 0.0, 0.0),
              r_max: float = math.inf, box_lo=(-math.inf,) * 3, box_hi=(math.inf,) * 3) -> SynGeom:
    g = SynGeom()
    g.nside, g.n_steps = int(nside), int(n_steps)
    g.r_obs_kpc[:] = [float(v) for v in r_obs]
    g.r_max_kpc = float(r_max)
    g.box_lo_kpc[:] = [float(v) for v in box_lo]
    g.box_hi_kpc[:] = [float(v) for v in box_hi]
    fr = [float(v) for v in freqs_hz]
    if not 1 <= len(fr) <= MAX_FREQ:
        raise ValueError("1..16 frequencies")
    g.n_freq = len(fr)
    g.freq_hz[:len(fr)] = fr
    return g


def geom_from(g) -> SynGeom:
    """SynGeom from any object with nside, n_steps, freqs_hz, r_obs, r_max, box_lo, box_hi."""
    return make_geom(g.nside, g.n_steps, g.freqs_hz, g.r_obs, g.r_max, g.box_lo, g.box_hi)


_spectrum_tables = {}


def spectrum_table(alpha_lo: float, alpha_hi: float, device=None, stream=None) -> torch.Tensor:
    """The device table of a broken power law with indices (alpha_lo, alpha_hi),
    built once per device and pair by syn_spectrum_table and kept here."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    key = (dev.index, float(alpha_lo), float(alpha_hi))
    t = _spectrum_tables.get(key)
    if t is None:
        nb = int(syn_spectrum_table_bytes())
        t = torch.empty((nb + 3) // 4, dtype=torch.float32, device=dev)
        check(syn_spectrum_table(float(alpha_lo), float(alpha_hi), t.data_ptr(), nb, _stream(stream)),
              "syn_spectrum_table")
        _spectrum_tables[key] = t
    return t


class Field:
    """A syn_field plus the tensors it points to (kept alive here).

    broken = (alpha_hi, gamma_break) selects the broken power-law CR spectrum
    (theta[12] the index below the break); its table comes from
    spectrum_table()."""

    def __init__(self, kind: int, theta, grid_bn: Optional[torch.Tensor] = None,
                 grid_c: Optional[torch.Tensor] = None, lo=None, hi=None,
                 mlp: Optional[torch.Tensor] = None, te_k: float = 0.0,
                 grid_alpha: Optional[torch.Tensor] = None, broken=None):
        self.s = SynField()
        self.s.kind = int(kind)
        self.s.te_k = float(te_k)  # > 0: free-free emission and absorption at T_e [K]
        self.grid_alpha = grid_alpha  # CR spectral index per node (GRID fields)
        th = np.asarray(theta, dtype=np.float64).reshape(-1)
        if th.size != NPARAM:
            raise ValueError("theta must have 16 entries")
        self.s.theta[:] = th.tolist()
        self.broken, self.spec_table = broken, None
        if broken is not None:
            self.s.spectrum = SPEC_BROKEN
            self.s.alpha_hi, self.s.gamma_break = float(broken[0]), float(broken[1])
            self.spec_table = spectrum_table(float(th[12]), float(broken[0]))
            self.s.spectrum_table = self.spec_table.data_ptr()
        self.grid_bn, self.grid_c, self.mlp = grid_bn, grid_c, mlp
        if grid_bn is not None:
            _dev_f32(grid_bn, "grid_bn")
            if grid_bn.dim() != 4 or grid_bn.shape[3] != 4:
                raise ValueError("grid_bn must be [nz][ny][nx][4]")
            nz, ny, nx, _ = grid_bn.shape
            self.s.grid_n[:] = [nx, ny, nz]
            self.s.grid_bn = grid_bn.data_ptr()
            if grid_c is not None:
                _dev_f32(grid_c, "grid_c")
                if tuple(grid_c.shape) != (nz, ny, nx):
                    raise ValueError("grid_c must be [nz][ny][nx]")
                self.s.grid_c = grid_c.data_ptr()
            if grid_alpha is not None:
                _dev_f32(grid_alpha, "grid_alpha")
                if tuple(grid_alpha.shape) != (nz, ny, nx):
                    raise ValueError("grid_alpha must be [nz][ny][nx]")
                self.s.grid_alpha = grid_alpha.data_ptr()
        if lo is not None:
            self.s.grid_lo_kpc[:] = [float(v) for v in lo]
            self.s.grid_hi_kpc[:] = [float(v) for v in hi]
        if mlp is not None:
            self.s.mlp = mlp.data_ptr()

    @property
    def theta(self) -> np.ndarray:
        return np.array(self.s.theta[:], dtype=np.float64)

    def with_theta(self, theta) -> "Field":
        return Field(self.s.kind, theta, self.grid_bn, self.grid_c,
                     self.s.grid_lo_kpc[:], self.s.grid_hi_kpc[:], self.mlp, self.s.te_k,
                     self.grid_alpha, self.broken)

    def with_te(self, te_k: float) -> "Field":
        """The same field with free-free emission and absorption at T_e = te_k [K]."""
        return Field(self.s.kind, self.theta, self.grid_bn, self.grid_c,
                     self.s.grid_lo_kpc[:], self.s.grid_hi_kpc[:], self.mlp, te_k,
                     self.grid_alpha, self.broken)

    def with_broken(self, broken) -> "Field":
        """The same field with a broken power-law spectrum (alpha_hi, gamma_break),
        or None for one power law."""
        return Field(self.s.kind, self.theta, self.grid_bn, self.grid_c,
                     self.s.grid_lo_kpc[:], self.s.grid_hi_kpc[:], self.mlp, self.s.te_k,
                     self.grid_alpha, broken)


def model16(theta) -> Field:
    return Field(FIELD_MODEL16, theta)


def grid(theta, grid_bn: torch.Tensor, grid_c: Optional[torch.Tensor], lo, hi,
         grid_alpha: Optional[torch.Tensor] = None) -> Field:
    return Field(FIELD_GRID, theta, grid_bn, grid_c, lo, hi, grid_alpha=grid_alpha)


def sphere(theta) -> Field:
    return Field(FIELD_SPHERE, theta)


def wmap(theta) -> Field:
    """The WMAP field and cosmic-ray density of Sec. 3.1 (theta as inputs.wmap_theta)."""
    return Field(FIELD_WMAP, theta)


# --------------------------------------------------------------------------- calls

def workspace_bytes(geom: SynGeom, field: Field, with_adjoint: bool = True) -> int:
    return int(syn_workspace_bytes(ctypes.byref(geom), ctypes.byref(field.s), int(with_adjoint)))


def alloc_workspace(geom: SynGeom, field: Field, device="cuda") -> torch.Tensor:
    n = workspace_bytes(geom, field, True)
    if n == 0:
        check(SYN_EINVAL, "syn_workspace_bytes")
    return torch.empty((n + 7) // 8, dtype=torch.float64, device=device)


def forward(geom: SynGeom, field: Field, maps: Optional[torch.Tensor] = None,
            ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Maps [n_freq][3][npix] (float32, K) of the march on the current device."""
    npix = 12 * geom.nside ** 2
    if maps is None:
        maps = torch.empty((geom.n_freq, 3, npix), dtype=torch.float32, device="cuda")
    _dev_f32(maps, "maps")
    if maps.numel() != geom.n_freq * 3 * npix:
        raise ValueError("maps has the wrong size")
    wsb = 0 if ws is None else ws.numel() * ws.element_size()
    check(syn_forward(ctypes.byref(geom), ctypes.byref(field.s), maps.data_ptr(), _ptr(ws), wsb,
                      _stream(stream)), "syn_forward")
    return maps


def adjoint(geom: SynGeom, field: Field, dmaps: torch.Tensor, ws: torch.Tensor,
            want_theta: bool = True, dgrid_bn: Optional[torch.Tensor] = None,
            dgrid_c: Optional[torch.Tensor] = None, stream=None):
    """dL/dtheta (float64 [16] on device, or None); grid gradients ADDED in place.
    With a broken power-law spectrum dtheta has 18 entries: [12] the index below
    the break, [16] the index above it, [17] ln gamma_break."""
    _dev_f32(dmaps, "dmaps")
    nth = NPARAM + 2 if field.s.spectrum == SPEC_BROKEN else NPARAM
    dth = torch.empty(nth, dtype=torch.float64, device=dmaps.device) if want_theta else None
    if dgrid_bn is not None:
        _dev_f32(dgrid_bn, "dgrid_bn")
    if dgrid_c is not None:
        _dev_f32(dgrid_c, "dgrid_c")
    check(syn_adjoint(ctypes.byref(geom), ctypes.byref(field.s), dmaps.data_ptr(), ws.data_ptr(),
                      ws.numel() * ws.element_size(), _ptr(dth), _ptr(dgrid_bn), _ptr(dgrid_c),
                      _stream(stream)), "syn_adjoint")
    return dth


def chi2(maps: torch.Tensor, target: torch.Tensor, inv_sigma2, want_grad: bool = True,
         stream=None):
    """(chi2 as a device float64 [1] tensor, dchi2/dmaps or None)."""
    _dev_f32(maps, "maps")
    _dev_f32(target, "target")
    if maps.shape != target.shape:
        raise ValueError("maps and target differ in shape")
    n_maps = int(np.prod(maps.shape[:-1]))
    n_pix = int(maps.shape[-1])
    inv = np.ascontiguousarray(np.broadcast_to(np.asarray(inv_sigma2, dtype=np.float64).reshape(-1),
                                               (n_maps,)))
    out = torch.empty(1, dtype=torch.float64, device=maps.device)
    dm = torch.empty_like(maps) if want_grad else None
    nws = syn_chi2_workspace_bytes(n_pix, n_maps)
    ws = torch.empty((nws + 7) // 8, dtype=torch.float64, device=maps.device)
    check(syn_chi2(n_pix, n_maps, maps.data_ptr(), target.data_ptr(),
                   inv.ctypes.data_as(_dp), _ptr(dm), out.data_ptr(), ws.data_ptr(), nws,
                   _stream(stream)), "syn_chi2")
    return out, dm


def chi2_cotangent(maps: torch.Tensor, target: torch.Tensor, inv_sigma2, chi2_out: torch.Tensor,
                   dmaps_out: Optional[torch.Tensor] = None, stream=None) -> None:
    """chi2 into chi2_out (device float64 [1]) and dchi2/dmaps into dmaps_out,
    through the entry point that allocates nothing (static device scratch)."""
    _dev_f32(maps, "maps")
    _dev_f32(target, "target")
    if maps.shape != target.shape:
        raise ValueError("maps and target differ in shape")
    if dmaps_out is not None:
        _dev_f32(dmaps_out, "dmaps_out")
        if dmaps_out.shape != maps.shape:
            raise ValueError("dmaps_out differs from maps in shape")
    if chi2_out.dtype != torch.float64 or not chi2_out.is_cuda or chi2_out.numel() < 1:
        raise ValueError("chi2_out must be a device float64 tensor")
    n_maps = int(np.prod(maps.shape[:-1]))
    n_pix = int(maps.shape[-1])
    inv = np.ascontiguousarray(np.broadcast_to(np.asarray(inv_sigma2, dtype=np.float64).reshape(-1),
                                               (n_maps,)))
    check(syn_chi2_cotangent(n_pix, n_maps, maps.data_ptr(), target.data_ptr(),
                             inv.ctypes.data_as(_dp), _ptr(dmaps_out), chi2_out.data_ptr(),
                             _stream(stream)), "syn_chi2_cotangent")


def sample_model16(theta, n_xyz, lo, hi, device="cuda", stream=None):
    """Analytic model on grid nodes: (bn [nz][ny][nx][4], c [nz][ny][nx]) float32."""
    nx, ny, nz = (int(v) for v in n_xyz)
    bn = torch.empty((nz, ny, nx, 4), dtype=torch.float32, device=device)
    c = torch.empty((nz, ny, nx), dtype=torch.float32, device=device)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    n = (_i32 * 3)(nx, ny, nz)
    lo_a = np.ascontiguousarray(lo, dtype=np.float64)
    hi_a = np.ascontiguousarray(hi, dtype=np.float64)
    check(syn_sample_model16(th.ctypes.data_as(_dp), n, lo_a.ctypes.data_as(_dp),
                             hi_a.ctypes.data_as(_dp), bn.data_ptr(), c.data_ptr(),
                             _stream(stream)), "syn_sample_model16")
    return bn, c


def eval_fields(field: Field, xyz: torch.Tensor, stream=None) -> torch.Tensor:
    _dev_f32(xyz, "xyz")
    n = xyz.numel() // 3
    out = torch.empty((n, 5), dtype=torch.float32, device=xyz.device)
    check(syn_eval_fields(ctypes.byref(field.s), n, xyz.data_ptr(), out.data_ptr(),
                          _stream(stream)), "syn_eval_fields")
    return out


def adam_step(params, grads, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8, period: int = 1, mask: int = 1) -> None:
    """syn_adam_step on contiguous FP32 CUDA tensors of equal size (in place)."""
    import torch
    for x in (params, grads, m, v):
        if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
            raise ValueError("adam_step needs contiguous float32 CUDA tensors")
        if x.numel() != params.numel():
            raise ValueError("adam_step tensors differ in size")
    check(syn_adam_step(params.numel(), period, mask, params.data_ptr(), grads.data_ptr(),
                        m.data_ptr(), v.data_ptr(), t, lr, beta1, beta2, eps, _stream()),
          "syn_adam_step")


def set_grid_addressing(mode: int) -> None:
    """0: automatic, 1: 64-bit addresses per lane, 2: buffer reads per lane,
    3: buffer reads shared through LDS (2 and 3 where the grid allows)."""
    check(syn_set_grid_addressing(mode), "syn_set_grid_addressing")


def get_grid_addressing() -> int:
    return int(syn_get_grid_addressing())


def set_lanes_per_ray(kernel: int, kind: int, lanes: int) -> None:
    check(syn_set_lanes_per_ray(kernel, kind, lanes), "syn_set_lanes_per_ray")


def get_lanes_per_ray(kernel: int, kind: int, npix: int) -> int:
    return int(syn_get_lanes_per_ray(kernel, kind, npix))


def host_nest_pixel(nside: int, q: int) -> Tuple[int, float, float]:
    ring, z, phi = _i64(), ctypes.c_double(), ctypes.c_double()
    check(syn_host_nest_pixel(nside, q, ctypes.byref(ring), ctypes.byref(z), ctypes.byref(phi)),
          "syn_host_nest_pixel")
    return ring.value, z.value, phi.value


# --------------------------------------------------------------------------- autograd

class SynMarchFn(torch.autograd.Function):
    """maps = march(theta, grid_bn, grid_c) with a hand-written HIP adjoint.

    theta: float64 [16] (any device; the gradient comes back on its device);
    grid_bn / grid_c: the grid tensors of a GRID field (or None).
    """

    @staticmethod
    def forward(ctx, theta, grid_bn, grid_c, geom: SynGeom, field: Field):
        fld = field.with_theta(theta.detach().cpu().numpy())
        ws = alloc_workspace(geom, fld)
        maps = forward(geom, fld, ws=ws)
        ctx.geom, ctx.field, ctx.ws = geom, fld, ws
        ctx.theta_device = theta.device
        ctx.mark_non_differentiable()
        return maps

    @staticmethod
    def backward(ctx, dmaps):
        dmaps = dmaps.contiguous().to(torch.float32)
        need_th = ctx.needs_input_grad[0]
        need_bn = ctx.needs_input_grad[1]
        need_c = ctx.needs_input_grad[2]
        dbn = torch.zeros_like(ctx.field.grid_bn) if need_bn else None
        dc = torch.zeros_like(ctx.field.grid_c) if need_c else None
        dth = adjoint(ctx.geom, ctx.field, dmaps, ctx.ws, want_theta=need_th, dgrid_bn=dbn,
                      dgrid_c=dc)
        if dth is not None:
            # (a broken spectrum's two parameters after theta are not inputs here)
            dth = dth[:NPARAM].to(ctx.theta_device)
        return dth, dbn, dc, None, None


def march(theta: torch.Tensor, geom: SynGeom, field: Field) -> torch.Tensor:
    """Differentiable maps: gradients flow to theta and to the field's grid tensors."""
    return SynMarchFn.apply(theta, field.grid_bn, field.grid_c, geom, field)
