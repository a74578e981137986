"""Run-time tile choices of the V-cycle passes: the library's autotuner
(fmg_autotune_vcycle) and a JSON cache of its results, keyed by device name, dimension,
level size and precision, so that later processes apply a measured choice without timing
again.  The choices change speed only: every choice gives the same bits."""
from __future__ import annotations

import ctypes as C
import json
import os

from . import _ffi, lib

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "fmgeig", "tuning.json")


FIELDS = ("vpass3d_variant", "vpass3d_min_n", "vpass3d_one_pass", "vtile3d", "vpass2d_wide_min_n", "vbottom2d_max_n")
N3D = 4   # the first N3D fields are the 3D choices, the rest the 2D ones


def get() -> dict:
    t = _ffi.fmg_tuning()
    if lib().fmg_get_tuning(C.byref(t)) != 0:
        raise RuntimeError(lib().fmg_last_error().decode())
    return {k: getattr(t, k) for k in FIELDS}


def apply(choice: dict):
    """Set the given fields; the others keep their current values."""
    t = _ffi.fmg_tuning()
    cur = get()
    for k in FIELDS:
        setattr(t, k, int(choice.get(k, cur[k])))
    if lib().fmg_set_tuning(C.byref(t)) != 0:
        raise RuntimeError(lib().fmg_last_error().decode())


def _key(dim, n, precision):
    import torch
    return f"{torch.cuda.get_device_name()}|dim={dim}|n={n}|{precision}"


def autotune(dim: int, n: int, precision: str = "fp64", cache: str | None = DEFAULT_CACHE, apply_result=True,
             refresh=False, stream=None) -> dict:
    """The tuning for V-cycles on a level of n cells per side (the fields of this dimension):
    from the cache when it holds this device and problem class (unless refresh), else
    measured by the library's autotuner and stored.  Applied to the library unless
    apply_result is False."""
    key = _key(dim, n, precision)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
    choice = None if refresh else table.get(key)
    if choice is None:
        from . import _stream
        t = _ffi.fmg_tuning()
        prec = _ffi.FMG_MIXED if precision == "mixed" else _ffi.FMG_FP64
        if lib().fmg_autotune_vcycle(dim, n, prec, _stream(stream), C.byref(t)) != 0:
            raise RuntimeError(lib().fmg_last_error().decode())
        keys = FIELDS[:N3D] if dim == 3 else FIELDS[N3D:]
        choice = {k: getattr(t, k) for k in keys}
        if cache:
            table[key] = choice
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
    if apply_result:
        apply(choice)
    return choice
