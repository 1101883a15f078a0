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


def _time(fn, reps, stream):
    fn()  # warm-up (graph capture, caches)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune_sim(sim, steps=20, reps=3, force=False):
    """Pick the fastest tile of the per-step kernel for this Sim (advances it
    by (len(tiles) * (reps + 1)) * steps steps).  Returns (tile, table)."""
    _load()
    key = (f"step|D{sim.D}|lat{sim.lattice}|{sim.dtype}|{'x'.join(map(str, sim.shape))}|ip{sim._inplace}"
           f"|blk{sim._blocked}|{_arch()}")
    if key in _mem and not force:
        t = tuple(_mem[key]["best"])
        sim.set_tile(*t)
        return t, _mem[key]["table"]
    table = {}
    for t in TILES[sim.D]:
        try:
            sim.set_tile(*t)
        except LbmError as e:  # not available for this sim (e.g. blocked 3-D order)
            if e.status != LBM_EUNSUPPORTED:
                raise
            continue
        table["x".join(map(str, t))] = _time(lambda: sim.step(steps), reps, sim.stream) / steps
    best = min(table, key=table.get)
    bt = tuple(int(v) for v in best.split("x"))
    sim.set_tile(*bt)
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
