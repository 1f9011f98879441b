"""Launch-shape autotuner for the march kernels.

The tunables are S, the number of lanes that share a sightline (1, 4, 8, 16
or 64; the batch kernels 1, 4, 16 or 64): larger S gives more parallelism for
small maps (few sightlines) and, for the grid adjoint, a wavefront count that
fills the chip in whole rounds; smaller S fewer scan instructions and more
register reuse for large maps; and, for
gridded forwards, the grid read path (per-lane buffer reads or cells shared
through LDS).  The tuner times each candidate with HIP events on the workload
at hand and applies the fastest through syn_set_lanes_per_ray.  Results are
cached in a JSON file keyed by device, the library's build id (a hash of its
sources) and workload shape (environment variable SYNMARCH_TUNE_CACHE,
default ~/.cache/synmarch/tune.json); a missing or unreadable cache falls back
to the built-in choice.  load() hands the cache to the library
(syn_autotune_load), which then applies the tuned shapes by itself to every
call of a matching shape, with no Python in the loop.
"""
from __future__ import annotations

import json
import os
from typing import Callable, Dict, Iterable, Optional

import torch

from . import binding as sm

CANDIDATES = (1, 4, 8, 16, 64)  # lanes per sightline of the forward and reverse marches
BATCH_CANDIDATES = (1, 4, 16, 64)  # the persistent many-set kernels
# grid read modes tried for gridded forwards (syn_set_grid_addressing):
# 2 = per-lane buffer reads, 3 = cell reads shared through LDS
GRID_MODES = (2, 3)


def cache_path() -> str:
    return os.environ.get("SYNMARCH_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "synmarch", "tune.json"))


def source_hash() -> str:
    """The loaded library's build id (hash of the sources it was built from)."""
    return sm.syn_build_id().decode()


def load(path: Optional[str] = None) -> int:
    """Hands the cache to the library (syn_autotune_load); returns the number of
    entries it kept (those tuned on this build).  Raises SynError when the file
    is missing or malformed; the library's table is then unchanged."""
    p = path or cache_path()
    sm.check(sm.syn_autotune_load(p.encode()), "syn_autotune_load")
    return int(sm.syn_autotune_entries())


def _key(kernel: int, kind: int, npix: int, n_steps: int, n_freq: int) -> str:
    dev = torch.cuda.get_device_name(torch.cuda.current_device()) if torch.cuda.is_available() else "cpu"
    return f"{dev}|{source_hash()}|k{kernel}|f{kind}|p{npix}|n{n_steps}|q{n_freq}"


def _kernel_of(key: str) -> Optional[int]:
    for part in key.split("|"):
        if len(part) > 1 and part[0] == "k" and part[1:].isdigit():
            return int(part[1:])
    return None


def _lane_count(v, kernel: Optional[int]) -> bool:
    allowed = BATCH_CANDIDATES if kernel == sm.KERNEL_BATCH else CANDIDATES
    return isinstance(v, int) and not isinstance(v, bool) and v in allowed


def _valid(v, kernel: Optional[int] = None) -> bool:
    # a lane count, or [lane count, grid read mode]
    if _lane_count(v, kernel):
        return True
    return (isinstance(v, list) and len(v) == 2 and _lane_count(v[0], kernel)
            and isinstance(v[1], int) and not isinstance(v[1], bool) and v[1] in GRID_MODES)


def load_cache(path: Optional[str] = None) -> Dict[str, object]:
    """The cache as a dict of valid entries; {} (the built-in shapes) when the
    file is missing, unreadable or not a JSON object."""
    path = path or cache_path()
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError, TypeError):
        return {}
    if not isinstance(d, dict):
        return {}
    return {k: v for k, v in d.items() if isinstance(k, str) and _valid(v, _kernel_of(k))}


def save_cache(d: Dict[str, int], path: Optional[str] = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_candidate(run: Callable[[], None], reps: int = 5) -> float:
    """Median milliseconds of `run` over `reps` timed calls after one warm-up."""
    run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def tune(kernel: int, kind: int, shape, run: Callable[[], None],
         candidates: Iterable[int] = CANDIDATES, reps: int = 5, use_cache: bool = True,
         write_cache: bool = True, grid_modes: Optional[Iterable[int]] = None,
         prepare: Optional[Callable[[], None]] = None) -> Dict[str, object]:
    """Times `run` for every lane count (and, given grid_modes, every grid read
    mode) and applies the fastest.  `prepare`, if given, runs untimed after each
    candidate is applied (e.g. the forward whose stored state the timed
    reverse pass reads).

    shape: (npix, n_steps, n_freq) of the workload, for the cache key.
    Returns {"lanes": best S, "grid_mode": best mode or None, "ms": {label: ms},
    "cached": bool}.
    """
    modes = list(grid_modes) if grid_modes is not None else [None]
    key = _key(kernel, kind, *shape) + ("|g" if grid_modes is not None else "")
    cache = load_cache() if use_cache else {}

    def apply(S, mode):
        sm.set_lanes_per_ray(kernel, kind, S)
        if mode is not None:
            sm.set_grid_addressing(mode)

    if key in cache:
        v = cache[key]
        S, mode = (v, None) if isinstance(v, int) else (v[0], v[1])
        apply(S, mode)
        if prepare is not None:
            prepare()
        return {"lanes": S, "grid_mode": mode, "ms": {}, "cached": True}
    ms = {}
    for mode in modes:
        for S in candidates:
            apply(S, mode)
            if prepare is not None:
                prepare()
            ms[(S, mode)] = time_candidate(run, reps)
    best = min(ms, key=ms.get)
    apply(*best)
    if prepare is not None:
        prepare()
    if write_cache:
        cache = load_cache()
        cache[key] = best[0] if best[1] is None else [best[0], best[1]]
        try:
            save_cache(cache)
        except OSError:
            pass
    label = {(S if m is None else f"{S}/mode{m}"): round(t, 4) for (S, m), t in ms.items()}
    return {"lanes": best[0], "grid_mode": best[1], "ms": label, "cached": False}


def tune_forward(geom, field, maps=None, ws=None, **kw):
    npix = 12 * geom.nside ** 2
    if maps is None:
        maps = torch.empty((geom.n_freq, 3, npix), dtype=torch.float32, device="cuda")
    if field.s.kind == sm.FIELD_GRID and "grid_modes" not in kw:
        kw["grid_modes"] = GRID_MODES
    return tune(sm.KERNEL_FORWARD, field.s.kind, (npix, geom.n_steps, geom.n_freq),
                lambda: sm.forward(geom, field, maps=maps, ws=ws), **kw)


def tune_adjoint(geom, field, dmaps, ws, want_theta=True, dgrid_bn=None, dgrid_c=None, **kw):
    """Tunes the reverse pass.  The pass reads the sums the forward stored at the
    ends of its pieces, laid out for the lane count in force when the forward
    ran: each candidate gets its own workspace and forward (untimed), and the
    forward is rerun into `ws` for the winner when `ws` has room for its
    pieces (else the caller allocates a new workspace and reruns it)."""
    npix = 12 * geom.nside ** 2
    shape = (npix, geom.n_steps, geom.n_freq)
    state = {}

    def prepare():
        w = sm.alloc_workspace(geom, field)
        sm.forward(geom, field, ws=w)
        state["ws"] = w

    res = tune(sm.KERNEL_ADJOINT, field.s.kind, shape,
               lambda: sm.adjoint(geom, field, dmaps, state["ws"], want_theta=want_theta,
                                  dgrid_bn=dgrid_bn, dgrid_c=dgrid_c), prepare=prepare, **kw)
    if ws is not None and ws.numel() * ws.element_size() >= sm.workspace_bytes(geom, field, True):
        sm.forward(geom, field, ws=ws)
    return res


def make_batch(thetas, nsides, geom, use_graph=True, kind=None):
    """Creates a batch plan (ctypes handle) for MODEL16 (default) or WMAP
    parameter sets."""
    import ctypes
    import numpy as np
    desc = sm.SynBatchDesc()
    ns = np.ascontiguousarray(nsides, dtype=np.int32)
    th = np.ascontiguousarray(thetas, dtype=np.float64)
    desc.n_sets = int(ns.size)
    desc.nside = ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    desc.theta = th.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    desc.geom = geom
    desc.use_graph = int(use_graph)
    desc.kind = sm.FIELD_MODEL16 if kind is None else int(kind)
    plan = ctypes.c_void_p()
    sm.check(sm.syn_batch_create(ctypes.byref(desc), ctypes.byref(plan)), "syn_batch_create")
    return plan


def tune_batch(thetas, nsides, geom, target, inv_sigma2, candidates: Iterable[int] = BATCH_CANDIDATES,
               reps: int = 3, **kw):
    """Tunes the lane count of the persistent many-set kernels (plans are
    rebuilt per candidate, since a plan fixes its launch shape)."""
    import numpy as np
    total = int(sum(12 * int(n) ** 2 for n in nsides))
    inv = np.ascontiguousarray(inv_sigma2, dtype=np.float64)
    maps = torch.empty((3, total), dtype=torch.float32, device="cuda")
    dmaps = torch.empty_like(maps)
    chi2 = torch.empty(len(nsides), dtype=torch.float64, device="cuda")
    dth = torch.empty((len(nsides), 16), dtype=torch.float64, device="cuda")
    plans = {}

    def runner():
        cur = sm.get_lanes_per_ray(sm.KERNEL_BATCH, sm.FIELD_MODEL16, total)
        if cur not in plans:
            plans[cur] = make_batch(thetas, nsides, geom)

        def run():
            sm.check(sm.syn_batch_run(plans[cur], target.data_ptr(), inv.ctypes.data_as(sm._dp),
                                      maps.data_ptr(), dmaps.data_ptr(), chi2.data_ptr(),
                                      dth.data_ptr(), sm._stream()), "syn_batch_run")
        run()

    try:
        return tune(sm.KERNEL_BATCH, sm.FIELD_MODEL16, (total, geom.n_steps, 1), runner,
                    candidates=candidates, reps=reps, **kw)
    finally:
        torch.cuda.synchronize()
        for p in plans.values():
            sm.syn_batch_destroy(p)
