"""Launch-shape autotuner.

The recursion kernels take their work decomposition from the library's launch keys (march
segments, XCD split, segment direction, store kind, block cap, chunks per thread, batch waves,
steps per pass, chunk groups of 2D blocked passes, two-step passes on 3D lattices).
The best values depend on the operator class, the lattice shape, R and the precision, so this
module times candidates on the caller's own operators and keeps the fastest.

The time of one recursion step is measured as the difference of two solves of K and 2K steps
(so start vectors, reductions and moments cancel; one Hamiltonian runs kpm_moments, several one
batched solve), each taken as the minimum of a few
repeats on the current stream with device events.  The keys are tuned one at a time, each over
its candidate list with the others held at their best value so far (coordinate descent, two
passes); a change is kept only if it is at least `min_gain` faster.  Only launch keys change:
the moments are identical for every candidate, up to the order in which the rounding errors of
the dot products are summed.

Results are cached in a JSON file keyed by the shape class (operator kinds, sizes, R, vector kind,
precision), so later runs of the same shape apply them without timing:

    best = tune(hams, R=16, vec=VEC_PHASE)
    with launch_settings(**best["settings"]):
        mus = moments_batched(hams, M, R, VEC_PHASE, seeds)
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, List, Optional, Sequence

from . import Hamiltonian, get_launch, launch_settings, moments, moments_batched

CANDIDATES: Dict[str, List[int]] = {
    "march_items": [128, 256, 512, 1024, 2048, 4096],
    "xcd_split": [0, 1, 2, 3],
    "alternate": [0, 1],
    "streaming": [0, 1, 2],
    "max_blocks": [512, 1024, 2048, 4096, 8192],
    "elems_per_thread": [1, 2, 4],
    "wave_mib": [0, 128, 192, 224, 256],
    "tblock": [-1, 0, 1, 3, 4, 5],
    "tb_group": [0, 4, 8, 16],
    "tb3": [-1, 0, 1],
}
LATTICE_KEYS = ["march_items", "xcd_split", "alternate", "streaming", "max_blocks", "tblock", "tb_group", "tb3"]
FLAT_KEYS = ["elems_per_thread", "max_blocks"]


def default_cache_path() -> str:
    return os.environ.get("KPM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "kpm_tune.json"))


def shape_key(hams: Sequence[Hamiltonian], R, vec: int) -> str:
    """Shape class of a (batched) solve: operator kinds and sizes, R, vector kind, precision."""
    Rs = [int(R)] * len(hams) if isinstance(R, int) else [int(x) for x in R]
    parts = []
    for h, r in zip(hams, Rs):
        op = h.op
        if hasattr(op, "row_ptr"):
            parts.append(f"csr{op.n}x{len(op.col)}{'c' if op.val_im is not None else 'r'}")
        else:
            L = "x".join(str(int(x)) for x in op.L[:op.dim])
            parts.append(f"d{op.dim}{'s' if op.hop else 'r'}{L}")
        parts[-1] += f"R{r}"
    counts = {}
    for p in parts:
        counts[p] = counts.get(p, 0) + 1
    body = ",".join(f"{p}*{n}" if n > 1 else p for p, n in sorted(counts.items()))
    if len(body) > 160:
        body = f"{len(counts)}shapes:" + hashlib.sha1(body.encode()).hexdigest()[:16]
    return f"p{hams[0].prec}v{vec}n{len(hams)}:" + body


def _keys_for(hams: Sequence[Hamiltonian]) -> List[str]:
    lattice = any(not hasattr(h.op, "row_ptr") for h in hams)
    csr = any(hasattr(h.op, "row_ptr") for h in hams)
    keys = list(LATTICE_KEYS) if lattice else []
    if csr:
        keys += [k for k in FLAT_KEYS if k not in keys]
    if len(hams) > 1:
        keys.append("wave_mib")
    return keys


def time_step(hams: Sequence[Hamiltonian], R, vec: int, steps: int = 16, repeats: int = 3) -> float:
    """Seconds per recursion step of the solve of `hams` (one Hamiltonian: kpm_moments; several: one
    batched solve) under the current launch keys."""
    import torch
    stream = torch.cuda.current_stream()

    def run(K: int) -> float:
        best = float("inf")
        for _ in range(repeats):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            if len(hams) == 1:     # a single solve runs the single-solve path (kpm_moments)
                moments(hams[0], 2 * K, R if isinstance(R, int) else R[0], vec, 1, 0)
            else:
                moments_batched(hams, 2 * K, R, vec, [1] * len(hams), list(range(len(hams))))
            e1.record(stream)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e-3)
        return best

    run(steps)                         # warm-up: allocations, first launches
    return max(run(2 * steps) - run(steps), 1e-9) / steps


def tune(hams: Sequence[Hamiltonian], R, vec: int, keys: Optional[Sequence[str]] = None, steps: int = 16,
         passes: int = 2, min_gain: float = 0.01, cache: Optional[str] = None, use_cache: bool = True,
         log=None) -> dict:
    """Tune the launch keys for the batched solve of `hams` (one Hamiltonian = a single solve).
    Returns {"key", "settings", "seconds_per_step", "default_seconds_per_step", "trials"}; the
    settings are also stored in the cache file unless cache is ""."""
    cache = default_cache_path() if cache is None else cache
    key = shape_key(hams, R, vec)
    if cache and use_cache and os.path.exists(cache):
        with open(cache) as f:
            stored = json.load(f)
        if key in stored:
            return dict(stored[key], key=key, cached=True)
    keys = list(keys) if keys is not None else _keys_for(hams)
    base = get_launch()
    current = {k: base[k] for k in keys}
    trials = []

    def measure(settings) -> float:
        with launch_settings(**settings):
            t = time_step(hams, R, vec, steps)
        trials.append((dict(settings), t))
        if log:
            log(f"tune: {settings} -> {t * 1e6:.2f} us/step")
        return t

    with launch_settings(**current):
        time_step(hams, R, vec, steps, repeats=1)     # first-use costs stay out of the comparison
    t_default = measure(current)
    t_best = t_default
    for _ in range(passes):
        changed = False
        for k in keys:
            for v in CANDIDATES[k]:
                if v == current[k]:
                    continue
                trial = dict(current, **{k: v})
                t = measure(trial)
                if t < t_best * (1.0 - min_gain):
                    t_best, current, changed = t, trial, True
        if not changed:
            break
    out = {"settings": current, "seconds_per_step": t_best, "default_seconds_per_step": t_default,
           "trials": len(trials)}
    if cache:
        stored = {}
        if os.path.exists(cache):
            with open(cache) as f:
                stored = json.load(f)
        stored[key] = out
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(stored, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(out, key=key, cached=False)


def _main():
    import argparse
    import sys

    import torch

    from . import F32, F64, gershgorin, scale_from_bounds
    from . import workloads as wl
    ap = argparse.ArgumentParser(description="Tune launch keys for one of the standard workloads.")
    ap.add_argument("--workload", default="config2", choices=["config1", "config2", "config3", "config4"])
    ap.add_argument("--prec", default="f32", choices=["f32", "f64"])
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--cache", default="", help="JSON cache file ('' = do not store)")
    args = ap.parse_args()
    cfg = getattr(wl, args.workload)()
    ops = cfg["lattices"] if "lattices" in cfg else [cfg["lattice"]]
    prec = F32 if args.prec == "f32" else F64
    hams = []
    for op in ops:
        lo, hi = gershgorin(op)
        a, b = scale_from_bounds(lo, hi, 0.01)
        hams.append(Hamiltonian(op, a, b, prec))
    log = lambda m: print(m, file=sys.stderr, flush=True)
    res = tune(hams, cfg["R"], cfg["vec"], steps=args.steps, cache=args.cache, use_cache=False, log=log)
    torch.cuda.synchronize()
    print(json.dumps(res))


if __name__ == "__main__":
    _main()
