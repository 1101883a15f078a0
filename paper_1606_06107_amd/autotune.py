"""Autotuner of launch shapes: times every compiled tile shape of the
per-step kernel, and block / superstep choices of the batched launch, with
HIP events on the caller's stream, and keeps the fastest.  Results are
cached in memory and, if LBMX_AUTOTUNE_CACHE names a JSON file, on disk,
keyed by (kernel, lattice, dtype, shape, device architecture).  Every shape
gives bitwise-identical results (no cross-node arithmetic depends on it), so
tuning changes speed only."""
from __future__ import annotations

import json
import os

import torch

from ._lib import LBM_EUNSUPPORTED, LbmError

TILES = {1: [(64, 1), (128, 1), (256, 1), (512, 1), (1024, 1)],
         2: [(64, 4), (32, 8), (128, 2), (256, 1), (64, 8), (32, 16), (16, 16), (64, 2)],
         3: [(64, 1), (32, 2), (16, 4)]}

_mem: dict = {}


def _arch():
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _path():
    return os.environ.get("LBMX_AUTOTUNE_CACHE")


def _load():
    p = _path()
    if p and os.path.exists(p):
        with open(p) as fh:
            _mem.update(json.load(fh))


def _store():
    p = _path()
    if p:
        with open(p, "w") as fh:
            json.dump(_mem, fh, indent=1, sort_keys=True)


def _time_calls(fn, reps, stream):
    """Median over `reps` calls of fn() (ms), each bracketed by its own
    events; the first call (graph recording, caches) is not timed."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def tune_sim(sim, steps=20, reps=5, finalists=3, force=False):
    """Pick the fastest tile of the per-step kernel for this Sim.

    A first pass times every compiled tile (median of `reps` calls of
    step(steps)); a second pass times the `finalists` fastest again,
    interleaved call by call so that drift of the clock or the memory
    affects them alike, and picks the smallest median.  Advances the Sim.
    Returns (tile, table) with table = {"all": {tile: ms per step},
    "finalists": {...}}."""
    _load()
    key = (f"step|D{sim.D}|lat{sim.lattice}|{sim.dtype}|{'x'.join(map(str, sim.shape))}|ip{sim._inplace}"
           f"|blk{sim._blocked}|{_arch()}")
    if key in _mem and not force:
        t = tuple(_mem[key]["best"])
        sim.set_tile(*t)
        return t, _mem[key]["table"]
    r1 = {}
    for t in TILES[sim.D]:
        try:
            sim.set_tile(*t)
        except LbmError as e:  # not available for this sim (e.g. blocked 3-D order)
            if e.status != LBM_EUNSUPPORTED:
                raise
            continue
        r1["x".join(map(str, t))] = _time_calls(lambda: sim.step(steps), reps, sim.stream) / steps
    fin = sorted(r1, key=r1.get)[:max(1, finalists)]
    runs = {k: [] for k in fin}
    for k in fin:  # record every finalist's graph before timing any
        sim.set_tile(*[int(v) for v in k.split("x")])
        sim.prepare(steps)
    for _ in range(reps):
        for k in fin:
            sim.set_tile(*[int(v) for v in k.split("x")])
            sim.prepare(steps)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record(sim.stream)
            sim.step(steps)
            b.record(sim.stream)
            torch.cuda.synchronize()
            runs[k].append(a.elapsed_time(b) / steps)
    r2 = {k: sorted(v)[len(v) // 2] for k, v in runs.items()}
    best = min(r2, key=r2.get)
    bt = tuple(int(v) for v in best.split("x"))
    sim.set_tile(*bt)
    table = {"all": {k: round(v, 5) for k, v in r1.items()}, "finalists": {k: round(v, 5) for k, v in r2.items()}}
    _mem[key] = {"best": list(bt), "table": table}
    _store()
    return bt, table


def tune_batch(make_batch, init_args, blocks=(512, 1024), supersteps=(16, 24, 32), force=False, key_extra=""):
    """make_batch(block, superstep) -> a Batch; each candidate is stepped once
    (graph capture), re-initialised from init_args = (rho, u, T) and timed on
    its second step.  Returns ((block, superstep), table)."""
    _load()
    key = f"batch|{key_extra}|{_arch()}"
    if key in _mem and not force:
        return tuple(_mem[key]["best"]), _mem[key]["table"]
    table = {}
    for blk in blocks:
        for sup in supersteps:
            b = make_batch(blk, sup)
            b.init(*init_args)
            b.step()
            b.init(*init_args)
            a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record(b.stream)
            b.step()
            e.record(b.stream)
            torch.cuda.synchronize()
            table[f"{blk}/{sup}"] = a.elapsed_time(e)
            del b
    best = min(table, key=table.get)
    bb = tuple(int(v) for v in best.split("/"))
    _mem[key] = {"best": list(bb), "table": table}
    _store()
    return bb, table
