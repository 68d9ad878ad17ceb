"""Autotuner for the launch shapes of the MD step.

The paper tunes its task granularity (subnodes per core) by timing a few
steps for increasing subnode counts, doubling until the elapsed time stops
dropping (Sec. 3.3).  The GPU counterpart here tunes, per workload, by
timing a short graphed run of the real step for each candidate:

  * list form: global-index full list or tile-local full list;
  * tile-local lists: workgroup size (MD_TUNE_TILE_THREADS), staged
    capacity (MD_TUNE_TILE_SLOTS: less LDS, more workgroups per CU), rows per tile
    (1 x 1, 2 x 1 or 2 x 2 in y x z) and cells per tile along x, the last
    swept the paper's way -- from the fewest (largest) tiles that fit (chosen
    per replica in a batch: tile_cells None), make tiles smaller (more of
    them, the same width for every replica) while the time keeps dropping;
  * neighbour-gather batch (MD_TUNE_PAIR_BATCH);
  * on tile lists, the fused force + integrator call or the split calls
    (when the factory takes ``fuse``).

Results are cached as JSON keyed by the device name and a coarse workload
signature (atom count bucket, mean atoms per cell, replicas, types), so a
later run of a similar workload reuses the choice.  Tuning only changes
speed; every candidate computes the same forces (full lists: bitwise for a
fixed candidate, and within round-off across candidates).
"""
from __future__ import annotations

import inspect
import json
import math
import os
import time

import numpy as np
import torch

from . import _abi as abi

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2109_10876_amd",
                             "tune.json")


def signature(natoms, box, rc, skin, ntypes):
    """Coarse workload key: log2 bucket of the total atom count, mean atoms
    per cell of edge rc + skin (to 0.5), replica-count bucket, type count."""
    natoms = np.asarray(natoms, dtype=np.float64).ravel()
    box = np.asarray(box, dtype=np.float64).reshape(-1, 3)
    rl = rc + skin
    cells = np.prod(np.maximum(1.0, np.floor(box / rl)), axis=1)
    nu = float(np.max(natoms / cells))
    dev = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
    return (f"{dev}|N2^{int(round(math.log2(natoms.sum())))}|nu{round(2 * nu) / 2}"
            f"|R2^{int(round(math.log2(len(natoms))))}|t{ntypes}|rl{rl:.3f}")


def _apply(lib, cand):
    lib.md_tune_set(abi.MD_TUNE_PAIR_BATCH, int(cand.get("batch", 4)))
    lib.md_tune_set(abi.MD_TUNE_TILE_THREADS, int(cand.get("tile_threads", 256)))
    lib.md_tune_set(abi.MD_TUNE_TILE_SLOTS, int(cand.get("tile_slots", 0)))


def _time(make, cand, steps, warmup):
    """ms per graphed step of a system built for ``cand``."""
    lib = abi.load()
    _apply(lib, cand)
    extra = {"fuse": cand["fuse"]} if "fuse" in cand else {}
    s = make(mode=cand["mode"], tile_cells=cand.get("tile_cells"),
             tile_rows=tuple(cand.get("tile_rows", (1, 1))), **extra)
    s.setup()
    s.run_checked(warmup, k=min(25, max(1, warmup)))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(4):
        # a run whose list overflowed is discarded and timed again from its start
        cp = s.checkpoint()
        ev0.record()
        s.run_graphed(steps, k=min(25, steps))
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        if not s.overflowed():
            break
        s.restore(cp)
    status = s.ensure_list()
    tc = s.tile_cells
    del s
    torch.cuda.empty_cache()
    return ms, status, tc


def tune(make, key, steps=40, warmup=10, cache=DEFAULT_CACHE, retune=False, log=None):
    """Pick the fastest candidate for ``make(mode=..., tile_cells=...,
    tile_rows=...[, fuse=...])`` (a factory returning an MDSystem) and
    remember it under ``key``.

    Returns (best candidate dict, list of (candidate, ms) trials)."""
    table = {}
    if cache and os.path.exists(cache):
        try:
            with open(cache) as fh:
                table = json.load(fh)
        except (OSError, ValueError):
            table = {}
    if not retune and key in table:
        return table[key]["best"], table[key].get("trials", [])
    trials = []

    def run(c):
        t0 = time.perf_counter()
        try:
            ms, status, tc = _time(make, c, steps, warmup)
        except (RuntimeError, abi.MDError) as exc:
            # a candidate the workload cannot use (e.g. a single-cell tile
            # that overflows the staging capacity): skipped
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            if log:
                log(f"autotune {json.dumps(c)} -> not usable ({exc})")
            return math.inf
        if c["mode"] == "tile":
            # the automatic width stays automatic (per replica in a batch);
            # its largest value starts the sweep below
            c = dict(c, tile_cells_max=tc) if c.get("tile_cells") is None else c
        trials.append((c, ms))
        if log:
            log(f"autotune {json.dumps(c)} -> {ms:.4f} ms/step ({time.perf_counter() - t0:.1f} s)")
        return ms

    for batch in (2, 4, 8):
        run({"mode": "full", "batch": batch})
    for tb, slots, rows in ((256, 0, [1, 1]), (256, 0, [2, 2]), (256, 2048, [2, 1]),
                            (256, 2048, [2, 2]), (256, 1536, [2, 2]), (128, 0, [2, 2])):
        # cells per tile: the largest that fits (automatic), then smaller ones
        # while that helps; mirrors the paper's grow-until-no-gain sweep
        base = {"mode": "tile", "batch": 4, "tile_threads": tb, "tile_slots": slots,
                "tile_rows": rows}
        best_ms = run(dict(base, tile_cells=None))
        if math.isinf(best_ms):
            continue
        m = trials[-1][0]["tile_cells_max"]
        while m and m > 2:
            m = max(2, m - max(1, m // 4))
            ms = run(dict(base, tile_cells=m))
            if ms >= best_ms:
                break
            best_ms = ms
    best = dict(min(trials, key=lambda t: t[1])[0])
    if best["mode"] == "tile":
        # 16 entries per pass against 8: within a percent of each other on
        # a liquid, so each is timed twice, interleaved, and the better
        # trial of either decides
        alt = dict(best, batch=8)
        for cand in (alt, best, alt):
            run(dict(cand))
        best = dict(min(trials, key=lambda t: t[1])[0])
        # the fused force + integrator call against the split calls (for a
        # factory that takes ``fuse``): with a thermostat the fused kernel
        # also draws the noise, which pays on some workloads and not others
        if "fuse" in inspect.signature(make).parameters:
            run(dict(best, fuse=False))
            best = dict(min(trials, key=lambda t: t[1])[0])
    _apply(abi.load(), best)
    if cache:
        table[key] = {"best": best, "trials": trials}
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        with open(cache, "w") as fh:
            json.dump(table, fh, indent=1)
    return best, trials


def apply(cand):
    """Set the process-wide knobs of a tuned candidate."""
    _apply(abi.load(), cand)
