"""Tuner for the persistent step kernel: for every grid side present in a
population, times each compiled (workgroup size, exchange variant)
configuration on the live population and keeps the fastest.  Results are
cached in a JSON file keyed by (device name, side, population bucket)."""
import json
import os
import time

import torch

from . import api


def _bucket(count):
    b = 1
    while b < count:
        b *= 2
    return b


def tune(pop, steps=200, cache_path=None, verbose=False):
    """Tunes `pop` in place (it must be built); returns {side: (block, variant, seconds)}.
    The population is reset to its build state afterwards."""
    dev_name = torch.cuda.get_device_name(pop.device)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        cache = json.load(open(cache_path))
    counts = {}
    for n in pop.sides:
        counts[n] = counts.get(n, 0) + 1
    result = {}
    for n, cnt in sorted(counts.items()):
        key = "%s|n=%d|R<=%d%s" % (dev_name, n, _bucket(cnt), "|dash" if pop.dashpots else "")
        if key in cache:
            b, v, t = cache[key]
            pop.set_persist_variant(n, b, v)
            result[n] = (b, v, t)
            continue
        best = None
        for b, v in api.persist_configs(n):
            if bool(v & 16) != pop.dashpots:
                continue  # kernels for the other spring model
            pop.set_persist_variant(n, b, v)
            pop.reset()
            pop.step(20)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pop.step(steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if verbose:
                print("side %d block %d variant %d: %.4f s" % (n, b, v, dt), flush=True)
            if best is None or dt < best[2]:
                best = (b, v, dt)
        pop.set_persist_variant(n, best[0], best[1])
        result[n] = best
        cache[key] = list(best)
    pop.reset()
    if cache_path:
        tmp = cache_path + ".tmp"
        json.dump(cache, open(tmp, "w"), indent=1)
        os.replace(tmp, cache_path)
    return result
