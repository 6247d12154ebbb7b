"""Launch-shape autotuner for ckf_find.

Times the persistent kernel (HIP events recorded by the library around it)
for a set of launch shapes - persistent workgroups, concurrent seeds per
64-lane workgroup, register variant - on the caller's actual batch, checks
that every shape finds exactly the same tracks, and caches the fastest
shape in a JSON file keyed by device, geometry size, batch-size class and
configuration.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import Finder, KernelTimer, _abi, launch

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ckf_mi355x", "autotune.json")


def _key(batch, cfg, device_name, learned):
    c = {name: getattr(cfg, name) for name, _ in _abi.Config._fields_}
    h = hashlib.sha1(json.dumps(c, sort_keys=True).encode()).hexdigest()[:12]
    seeds_class = int(2 ** round(np.log2(max(1, batch.n_seeds))))
    form = "learned" if learned else "plain"
    return f"{device_name}|surf={batch.n_surfaces}|seeds~{seeds_class}|cfg={h}|{form}"


def candidates(n_cus: int):
    for waves in (3, 2, 1):
        for spg in (16, 24, 32, 48, 64):
            for per_cu in (4 * waves, 8 * waves):
                yield dict(grid=n_cus * per_cu, seeds_per_group=spg, waves_per_simd=waves)


def tune(geometry, field, batch, cfg=None, shapes=None, reps=3, cache_path=DEFAULT_CACHE, use_cache=True,
         verbose=False, model=None):
    """Return (best launch dict, table of (shape, median kernel ms)).  With a
    model the learned form is tuned (its timing depends on the model, so a
    cached entry is only a starting point: pass use_cache=False to retune)."""
    import torch
    props = torch.cuda.get_device_properties(batch.loc.device)
    key = _key(batch, cfg if cfg is not None else _default_cfg(), props.name, model is not None)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        return cache[key]["best"], cache[key]["table"]
    shapes = list(shapes) if shapes is not None else list(candidates(props.multi_processor_count))
    timer = KernelTimer()
    table, ref = [], None
    for sh in shapes:
        f = Finder(geometry, field, batch, cfg,
                   launch(sh["grid"], sh["seeds_per_group"], 0, timer, sh["waves_per_simd"]), counters=False,
                   model=model)
        f.enqueue()  # warm-up
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            f.enqueue()
            ms.append(timer.elapsed_ms())
        r = f.result()
        if ref is None:
            ref = r
        elif not (np.array_equal(r["offsets"], ref["offsets"]) and np.array_equal(r["meas"], ref["meas"])
                  and np.array_equal(r["params"], ref["params"])):
            raise RuntimeError(f"launch shape {sh} changed the found tracks")
        table.append((sh, float(np.median(ms))))
        if verbose:
            print(f"# autotune {sh}: {np.median(ms):.3f} ms", flush=True)
        del f
    best = min(table, key=lambda t: t[1])[0]
    if cache_path:
        cache[key] = dict(best=best, table=table, when=time.time())
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path + ".tmp", "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(cache_path + ".tmp", cache_path)
    return best, table


def _default_cfg():
    from . import config
    return config()
