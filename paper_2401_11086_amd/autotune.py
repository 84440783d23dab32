"""Launch autotuner: picks lbsmrt_set_launch's mode, work-group size and lanes per node
by timing a few steps of the caller's own lattice, and caches the choice in a JSON file
keyed by device, velocity set, order, precision, collision form, problem-size bucket and a
digest of the domain geometry (shapes and boundary types), so that a choice made for shock
tubes is never replayed on periodic domains of the same size.  autotune() tunes the population
step (lbsmrt_step), autotune_moment_state() the moment-state step (lbsmrt_step_moment_state:
direct or captured launches, one or eight lanes per node on line domains); the launch setting is
one per context, so the last call's choice holds for both forms."""
import hashlib
import json
import math
import os

import torch

CANDIDATES = [(mode, block, lpn) for lpn in (1, 2, 4, 8, 16) for mode in ("direct", "graph", "persistent")
              for block in (64, 128, 256) if not (lpn == 16 and mode == "persistent")]


def _candidates(lat):
    """More than one lane per node exists for shock contexts with FP64 contractions only."""
    shock = any(int(d.get("bc_x", 0)) != 0 for d in lat.domains)
    split_ok = shock and lat.precision == "fp64_contract"
    return [c for c in CANDIDATES if c[2] == 1 or split_ok]


def _cache_path():
    return os.environ.get("LBSMRT_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "lbsmrt", "autotune.json"))


def _geometry_digest(lat):
    """Short digest of every domain's (nx, ny, nz, bc_x), in order."""
    h = hashlib.sha256()
    for d in lat.domains:
        h.update(f"{int(d['nx'])},{int(d.get('ny', 1))},{int(d.get('nz', 1))},{int(d.get('bc_x', 0))};".encode())
    return h.hexdigest()[:16]


def _key(lat, form_suffix=""):
    props = torch.cuda.get_device_properties(lat.device)
    arch = getattr(props, "gcnArchName", props.name)
    bucket = int(round(math.log2(max(lat.n_nodes, 1))))
    shock = int(any(int(d.get("bc_x", 0)) != 0 for d in lat.domains))
    form = "rebuilt" if lat.regularized else "additive"
    return (f"{arch}|Q{lat.Q}|N{lat.N}|{lat.precision}|{form}|nodes2^{bucket}|dom{len(lat.domains)}"
            f"|shock{shock}|geom{_geometry_digest(lat)}|lpn{form_suffix}")


def _time(lat, fa, fb, steps):
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lat.step(fa, fb, 2)
    torch.cuda.synchronize()
    ev0.record()
    lat.step(fa, fb, steps)
    ev1.record()
    torch.cuda.synchronize()
    lat.sync()
    return ev0.elapsed_time(ev1) / steps


def autotune(lat, fa, fb, steps=20, graph_steps=32, use_cache=True):
    """Time every candidate on (fa, fb) (their contents are advanced), apply the fastest,
    and return {'mode', 'block', 'lanes_per_node', 'ms_per_step', 'trials'}."""
    path = _cache_path()
    key = _key(lat)
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        best = cache[key]
        try:
            lat.set_launch(best["mode"], best["block"], graph_steps, best["lanes_per_node"])
            return dict(best, cached=True)
        except Exception:
            pass   # a stale or foreign entry: tune again and overwrite it
    trials = []
    for mode, block, lpn in _candidates(lat):
        try:
            lat.set_launch(mode, block, graph_steps, lpn)
        except Exception:
            continue
        trials.append((mode, block, lpn, _time(lat, fa, fb, steps)))
    mode, block, lpn, ms = min(trials, key=lambda t: t[3])
    lat.set_launch(mode, block, graph_steps, lpn)
    best = {"mode": mode, "block": block, "lanes_per_node": lpn, "ms_per_step": round(ms, 5)}
    if use_cache:
        cache[key] = best
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
        except OSError:
            pass
    return dict(best, trials=[{"mode": m, "block": b, "lanes_per_node": k, "ms": round(t, 5)}
                              for m, b, k, t in trials], cached=False)


def _time_ms(lat, ma, mb, work, steps):
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lat.step_moment_state(ma, mb, work, 2)
    torch.cuda.synchronize()
    ev0.record()
    lat.step_moment_state(ma, mb, work, steps)
    ev1.record()
    torch.cuda.synchronize()
    lat.sync()
    return ev0.elapsed_time(ev1) / steps


def autotune_moment_state(lat, ma, mb, work, steps=40, graph_steps=32, use_cache=True):
    """Time the moment-state step's candidates on (ma, mb) (advanced in place): direct or
    graph-captured launches, and on line domains one or eight lanes per node where the context
    allows more than one; apply the fastest and return it as autotune() does."""
    path = _cache_path()
    key = _key(lat, "|moment_state")
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        best = cache[key]
        try:
            lat.set_launch(best["mode"], 0, graph_steps, best["lanes_per_node"])
            return dict(best, cached=True)
        except Exception:
            pass
    lines = all(int(d.get("ny", 1)) == 1 and int(d.get("nz", 1)) == 1 for d in lat.domains)
    lanes = (1, 8) if lines and any(c[2] > 1 for c in _candidates(lat)) else (1,)
    trials = []
    for mode in ("direct", "graph"):
        for lpn in lanes:
            try:
                lat.set_launch(mode, 0, graph_steps, lpn)
            except Exception:
                continue
            trials.append((mode, lpn, _time_ms(lat, ma, mb, work, steps)))
    mode, lpn, ms = min(trials, key=lambda t: t[2])
    lat.set_launch(mode, 0, graph_steps, lpn)
    best = {"mode": mode, "lanes_per_node": lpn, "ms_per_step": round(ms, 5)}
    if use_cache:
        cache[key] = best
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
        except OSError:
            pass
    return dict(best, trials=[{"mode": m, "lanes_per_node": k, "ms": round(t, 5)} for m, k, t in trials],
                cached=False)
