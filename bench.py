"""Benchmark: NVE velocity-Verlet MD of a 1,048,576-atom Lennard-Jones fluid
on one MI355X through libmd.

Workload: FCC 64^3 x 4 sites at density 0.8442, Maxwell velocities at T = 1.0,
rc = 2.5, skin = 0.3, dt = 0.005, energy-shifted LJ, full Verlet list
(the list form and launch shape chosen by the autotuner, untimed, unless
--mode names one).
One step = Integrate1 + skin test + (gated) re-sort and list build + forces
with energy and virial + Integrate2 with kinetic energy -- every kernel of
the path, nothing skipped.  Both pair-arithmetic precisions are run on the
same inputs: FP32-mixed (the headline value) and FP64.

Prints ONE JSON line.  Usage: python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, published
# MI355X vector peak, FMA counted as 2 flops: 256 CUs x 4 SIMDs x 16 lanes x
# 2 x 2.4 GHz.  FP64 runs at this rate, and so does FP32 issued one value per
# lane (the 157.3 TFLOP/s FP32 figure needs packed two-wide FP32, which this
# code does not use).
VALU_PEAK_TFLOPS = 78.6
# Algorithmic flops of the method's pair work, each unordered pair once (a
# half list with Newton's third law, Sec. 2.1.2): every half-list entry pays
# the displacement (3), r^2 (5) and the cutoff test (1); every pair inside rc
# the LJ terms: 1/r^2 (1), q^3 (2), w = q^3 (A q^3 - B) (3), fr = w q (1),
# force accumulation (6), energy (5) and virial (2).
FLOPS_PER_ENTRY = 9
FLOPS_PER_PAIR_IN_RC = 20
# Algorithmic HBM bytes of one force evaluation per atom (the half-list
# minimum): 4 B per half-list entry (int32 index), the count (4), own FP64
# position (24) and FP64 force write (24), neighbour positions being cache-
# or LDS-resident after the spatial sort.  Fused with the integrator: also
# the velocity read and write, the build-time position read and the next
# position write (4 x 24 B).
BYTES_PER_HALF_ENTRY = 4
BYTES_PER_ATOM_FORCE = 52
BYTES_PER_ATOM_VV_FUSED = 96
# Velocity-Verlet work per atom when fused into the force kernel: two half
# kicks (2 x 6), kinetic energy (8), drift (6), displacement from the build
# positions and its running maximum (9), and the step factor (1).
FLOPS_PER_ATOM_VV = 36

# Memory bytes per pair-kernel launch on this workload from rocprofv3
# FETCH_SIZE and WRITE_SIZE (FETCH x 2.0, WRITE x 1.0: the factors a plain
# 512 MiB device copy needs to read back its true size), valid only for the
# kernel source they were taken on (profiles/k_tile_lj_lj1m_hbm_counters.md).
# Keyed by list form ("_fused": the force kernel with the integrator fused
# in); each entry: source hash of the kernel's files and, per pair batch of
# the launch (8 takes 16 entries per pass), calibrated bytes per launch for
# the FP32-mixed and FP64 paths.
COUNTED_TRAFFIC = {
    "tile_fused": {"src_sha256_16": "cdb2de62444cf33d",
                   "bytes_per_launch": {"4": {"mixed": 420400571, "fp64": 421723454},
                                        "8": {"mixed": 439971407, "fp64": 442008382}}},
    "tile": {"src_sha256_16": "cdb2de62444cf33d",
             "bytes_per_launch": {"4": {"mixed": 317826611, "fp64": 319613777},
                                  "8": {"mixed": 336739664, "fp64": 339324424}}},
}

FORCE_KERNEL_SOURCES = {
    "full": ("md_forces.hip", "md_pair.hpp", "md_common.hpp"),
    "tile": ("md_tile.hip", "md_tile.hpp", "md_pair.hpp", "md_philox.hpp", "md_common.hpp"),
}


def force_kernel_src_hash(mode):
    import hashlib
    h = hashlib.sha256()
    for f in FORCE_KERNEL_SOURCES.get(mode, ()):
        with open(os.path.join(ROOT, "paper_2109_10876_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def s_max(times, accelerated, factor):
    """The paper's ideal-speedup model (Sec. 4.1, Eq. vec-perf-model): the
    run time over the run time with the sections named in ``accelerated`` sped
    up ``factor``-fold and the rest unchanged; ``times`` maps section names to
    times."""
    total = sum(times.values())
    fast = sum(t for k, t in times.items() if k in accelerated)
    return total / (total - fast + fast / factor)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def pairs_within_rc(s):
    """Unordered pairs within rc at the current positions: a full list of
    radius rc (skin 0) built by libmd itself from the current state
    (measurement only, outside the timed region)."""
    from paper_2109_10876_amd import MDSystem
    t = MDSystem(s.h_atom_off[1:] - s.h_atom_off[:-1], s.h_box, s.positions(),
                 s.velocities(), rc=s.rc, skin=0.0, dt=s.dt, shift=s.shift, mode="full")
    t.setup()
    t.ensure_list()
    n = int(t.count.sum().item()) // 2
    del t
    return n


def graph_length(steps, cap=50):
    """Steps per captured graph for a run of ``steps`` steps: the first step's
    head runs eagerly, so up to steps - 1 repeated steps are replayed; an even
    number (the fused call alternates two position buffers), at most cap."""
    return max(2, min(cap, (steps - 1) // 2 * 2))


def warm_graph(s, k):
    """Launch a freshly captured graph once, outside any timed region, and
    return to the state before it: the first launch of a HIP graph also
    uploads it (about 0.5 ms for 50 steps of this workload), a one-time
    cost that would otherwise land inside the first timed replay."""
    for _ in range(2):
        cp = s.checkpoint()
        s.run_graphed(k + 1, k=k)
        s.restore(cp)
        if s._graph is not None:
            return
        s.capture(k)   # the list grew (an overflow): the graph was dropped


def time_path(cfg, prec, steps, warmup, tuned):
    import torch
    from paper_2109_10876_amd import MDSystem, autotune
    autotune.apply(tuned)
    graph_k = graph_length(steps)
    s = MDSystem(cfg.natoms, cfg.box, cfg.pos, cfg.vel, rc=cfg.rc, skin=cfg.skin, dt=cfg.dt,
                 shift=cfg.shift, mode=tuned["mode"], prec=prec,
                 tile_cells=tuned.get("tile_cells"),
                 tile_rows=tuple(tuned.get("tile_rows", (1, 1))))
    s.setup()
    s.capture(graph_k)
    warm_graph(s, graph_k)
    if warmup:
        s.run_checked(warmup, k=graph_k)
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for attempt in range(4):
        # a timed run whose list overflowed is discarded: back to its start
        # (the list grows) and timed again
        cp = s.checkpoint()
        e_start = float(s.energy[0]) + float(s.ke[0])
        torch.cuda.synchronize()
        t0.record(stream)
        s.run_graphed(steps, k=graph_k)
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        if not s.overflowed():
            break
        log(f"[{prec}] list overflow during the timed run; regrow and repeat")
        s.restore(cp)
        s.capture(graph_k)
        warm_graph(s, graph_k)
    else:
        raise RuntimeError("list overflow persisted")
    s.ensure_list()
    e_end = float(s.energy[0]) + float(s.ke[0])
    drift = {"steps": steps, "e_total_start": e_start, "e_total_end": e_end,
             "per_atom": (e_end - e_start) / s.N,
             "rel": (e_end - e_start) / abs(e_start)}
    replays = (steps - 1) // graph_k
    graphed = {"graph_steps": graph_k, "replays": replays,
               "eager_steps": steps - replays * graph_k}
    # dominant kernel: the pair-force kernel of the step (fused with the
    # integrator on pure-LJ tile runs), timed by libmd itself with HIP events
    # around each of its launches on their stream, over nrep eager steps of
    # the same configuration right after the timed region
    import ctypes
    from paper_2109_10876_amd import _abi
    lib = _abi.load()
    nrep = 50
    torch.cuda.synchronize()
    assert lib.md_kernel_timing_start(nrep) == 0
    s.run(nrep + 1, check_every=nrep + 1)
    f_ms, n_timed = ctypes.c_double(), ctypes.c_int32()
    assert lib.md_kernel_timing_read(ctypes.byref(f_ms), ctypes.byref(n_timed)) == 0
    assert n_timed.value == nrep, n_timed.value
    f_ms = f_ms.value
    s.ensure_list()
    sections = time_sections(s, ms / steps, f_ms)
    mean_k = float(s.count.double().mean().item())
    npairs = pairs_within_rc(s)
    snap = (s.positions(), s.velocities())
    return s, ms, f_ms, mean_k, npairs, snap, bool(s.fuse), sections, drift, graphed


def time_sections(s, step_ms, pair_ms, nsteps=200, nrep=10):
    """Step time split into the paper's sections (Sec. 4: Pair, Neigh,
    Resort, Integrate, Other), outside the timed region: the rebuild interval
    from the gate over nsteps eager steps, the list build and the re-sort
    timed ungated (every replica rebuilds) and amortised over that interval,
    the pair kernel from the library's events (fused runs integrate inside
    it), Other the remainder (finalisers, gated no-op launches, launch gaps)."""
    import torch
    rebuilds = 0
    cp = s.checkpoint()
    s._head()
    for _ in range(nsteps):
        s._body()
        rebuilds += int(s.step_gate.max().item() > 0)
    s._tail()
    if s.overflowed():
        s.restore(cp)   # the count stands; the state goes back to a valid list
    s.ensure_list()
    interval = nsteps / max(rebuilds, 1)

    def timed(fn):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(nrep):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / nrep

    sort_ms = timed(lambda: s.sort(gated=False))
    build_ms = timed(lambda: s.build(gated=False))
    s.ensure_list()
    neigh, resort = build_ms / interval, sort_ms / interval
    other = step_ms - pair_ms - neigh - resort
    return {"rebuild_interval_steps": interval,
            "pair_us": pair_ms * 1e3, "integrate_us": 0.0 if s.fuse else None,
            "neigh_us": neigh * 1e3, "resort_us": resort * 1e3, "other_us": other * 1e3,
            "per_rebuild_us": {"neigh": build_ms * 1e3, "resort": sort_ms * 1e3},
            "note": ("integrate runs inside the pair kernel" if s.fuse
                     else "integrate is part of other")}


def time_workload(name, steps, warmup=10):
    """Throughput of one of the other workloads (FP32-mixed, graphed steps):
    the polymer melts (purely repulsive LJ + FENE + Langevin: linear chains,
    and the paper's rings with the cosine angle term), the LJ slab
    and the LJ sphere in vacuum (Langevin) and the batch of uneven replicas
    (NVE), plus, for the batch,
    one force + adjoint evaluation of a force-matching loss."""
    import torch
    import md_inputs
    from paper_2109_10876_amd import MDSystem
    from paper_2109_10876_amd import autotune
    cfg = md_inputs.CONFIGS[name]()
    lang = {"kg_melt": (0.5, 1.0, 3), "ring_melt": (0.5, 1.0, 7), "lj_slab": (1.0, 0.85, 4),
            "lj_sphere": (1.0, 0.1, 6)}.get(name)
    ntypes = int(np.atleast_2d(np.asarray(cfg.eps)).shape[0])

    def make(mode="full", tile_cells=None, tile_rows=(1, 1), fuse=True):
        return MDSystem(cfg.natoms, cfg.box, cfg.pos, cfg.vel, cfg.types, cfg.eps, cfg.sig,
                        cfg.mass, rc=cfg.rc, skin=cfg.skin, dt=cfg.dt, shift=cfg.shift,
                        bonds=cfg.bonds, angles=cfg.angles, langevin=lang, prec="mixed",
                        mode=mode, tile_cells=tile_cells, tile_rows=tile_rows, fuse=fuse)
    from paper_2109_10876_amd import _abi
    if ntypes <= _abi.MD_TILE_MAX_TYPES:
        # list form and launch shape from the autotuner (untimed)
        key = autotune.signature(cfg.natoms, cfg.box, cfg.rc, cfg.skin, ntypes)
        tuned, _ = autotune.tune(make, key, steps=30, warmup=5, cache=None)
    else:
        tuned = {"mode": "full", "batch": 4}
    autotune.apply(tuned)
    s = make(tuned["mode"], tuned.get("tile_cells"), tuple(tuned.get("tile_rows", (1, 1))),
             tuned.get("fuse", True))
    s.setup()
    gk = graph_length(steps, cap=25)
    s.capture(gk)
    warm_graph(s, gk)
    s.run_checked(warmup, k=gk)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(4):
        # a timed run whose list overflowed is discarded and timed again
        cp = s.checkpoint()
        ev0.record()
        s.run_graphed(steps, k=gk)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        if not s.overflowed():
            break
        s.restore(cp)
        s.capture(gk)
    st = s.ensure_list()
    out = {"N": s.N, "R": s.R, "steps": steps, "ms_per_step": ms / steps, "launch": tuned,
           "atom_steps_per_s": s.N * steps / (ms * 1e-3), "status": st,
           "mean_list_entries": float(s.count.double().mean().item())}
    if name == "replicas":
        # one force + adjoint evaluation of a force-matching loss, on the
        # tuned list and on a global-index full list; the faster is reported
        def force_vjp_ms(sy):
            gf = [torch.randn(sy.N, dtype=torch.float64, device=sy.dev) for _ in range(3)]
            gE = torch.randn(sy.R, dtype=torch.float64, device=sy.dev)
            gx = torch.empty(3 * sy.N, dtype=torch.float64, device=sy.dev)
            ge = torch.empty(sy.ntypes ** 2, dtype=torch.float64, device=sy.dev)
            gs = torch.empty(sy.ntypes ** 2, dtype=torch.float64, device=sy.dev)
            torch.cuda.synchronize()
            ev0.record()
            for _ in range(20):
                sy.forces()
                sy.vjp(*gf, gE, gx, ge, gs)
            ev1.record()
            torch.cuda.synchronize()
            return ev0.elapsed_time(ev1) / 20
        per_list = {}
        if tuned["mode"] != "half":
            per_list[tuned["mode"]] = force_vjp_ms(s)
        if tuned["mode"] != "full":
            del s
            torch.cuda.empty_cache()
            autotune.apply({"mode": "full", "batch": 4})
            s = make("full")
            s.setup()
            s.ensure_list()
            per_list["full"] = force_vjp_ms(s)
        best = min(per_list, key=per_list.get)
        t = per_list[best]
        out["force_plus_vjp_ms"] = t
        out["force_plus_vjp_list"] = best
        out["force_plus_vjp_ms_by_list"] = per_list
        out["force_plus_vjp_atoms_per_s"] = s.N / (t * 1e-3)
    del s
    torch.cuda.empty_cache()
    return out


def host_cpu():
    """CPU model and logical CPU count of this host (for the baseline's record)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def oracle_leg(pos, vel, box, rc, skin, dt, samples=3):
    """The FP64 oracle as it stands, timed on this host's cores on the given
    state: single-threaded (liborc.so) and on all usable threads (the
    timing-only liborc_omp.so, same per-pair arithmetic).  One sample is the
    time of a 1-step run minus that of a 0-step run (each starts with one
    force evaluation), i.e. one step: Integrate1, skin test, pair search and
    forces within rc, Integrate2.  Also returns the 1-step result, the
    reference of the per-result errors."""
    import oracle
    oracle.build()
    cpu = host_cpu()
    threads = max(1, min(int(os.environ.get("OMP_NUM_THREADS", cpu["usable_cpus"])),
                         cpu["usable_cpus"]))
    os.environ["OMP_NUM_THREADS"] = str(threads)
    legs, ref1 = {}, None
    for name, omp in (("single", False), ("all_cores", True)):
        per = []
        for _ in range(samples):
            t = time.perf_counter()
            oracle.md_run(pos, vel, box, rc, skin, dt, 0, omp=omp)
            t0 = time.perf_counter() - t
            t = time.perf_counter()
            r1 = oracle.md_run(pos, vel, box, rc, skin, dt, 1, omp=omp)
            per.append(max(time.perf_counter() - t - t0, 1e-9))
            if not omp:
                ref1 = r1
        med = float(np.median(per))
        legs[name] = {"value": pos.shape[0] / med, "unit": "atom-steps/s",
                      "cores": 1 if not omp else threads, "s_per_step": per,
                      "s_per_step_median": med}
    return legs, cpu, ref1


def per_result_errors(cfg, tuned, pos, vel, ref1, steps_window):
    """Error of each result of the FP32-mixed path on one thermalised state
    (the mixed run's final positions and velocities): potential energy E,
    virial W and forces against the FP64 GPU path and the FP64 oracle, and
    kinetic energy and positions after one step against both.  E and W of the
    oracle come from its cell-list force evaluation of all atoms; its forces
    are sampled with the O(N) single-atom loop."""
    import torch
    import oracle
    from paper_2109_10876_amd import MDSystem, autotune
    autotune.apply(tuned)
    box = cfg.box[0]
    res = {}
    for prec in ("mixed", "fp64"):
        s = MDSystem(cfg.natoms, cfg.box, pos, vel, rc=cfg.rc, skin=cfg.skin, dt=cfg.dt,
                     shift=cfg.shift, mode=tuned["mode"], prec=prec,
                     tile_cells=tuned.get("tile_cells"),
                     tile_rows=tuple(tuned.get("tile_rows", (1, 1))))
        s.setup()
        s.ensure_list()
        r = {"E": float(s.energy[0]), "W": float(s.virial[0]), "F": s.forces_np()}
        s.run(1, check_every=1)
        s.ensure_list()
        r["KE1"] = float(s.ke[0])
        r["pos1"] = s.positions()
        res[prec] = r
        del s
        torch.cuda.empty_cache()
    f_o, e_o, w_o = oracle.lj_forces(pos, cfg.box[0], cfg.rc, shift=cfg.shift)
    m, d = res["mixed"], res["fp64"]
    rel = lambda a, b: abs(a - b) / abs(b)
    nrm = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    out = {
        "state": f"the mixed run's state after its {steps_window} timed steps and the "
                 f"measurement steps that follow them (thermalised)",
        "vs_oracle": {
            "E_rel": rel(m["E"], e_o), "W_rel": rel(m["W"], w_o), "F_rel": nrm(m["F"], f_o),
            "KE_1step_rel": rel(m["KE1"], ref1["ekin"][-1]),
            "pos_1step_max_abs": float(np.abs(m["pos1"] - ref1["pos"]).max()),
        },
        "vs_fp64_gpu": {
            "E_rel": rel(m["E"], d["E"]), "W_rel": rel(m["W"], d["W"]),
            "F_rel": nrm(m["F"], d["F"]), "KE_1step_rel": rel(m["KE1"], d["KE1"]),
            "pos_1step_max_abs": float(np.abs(m["pos1"] - d["pos1"]).max()),
        },
        "fp64_gpu_vs_oracle": {
            "E_rel": rel(d["E"], e_o), "W_rel": rel(d["W"], w_o), "F_rel": nrm(d["F"], f_o),
            "KE_1step_rel": rel(d["KE1"], ref1["ekin"][-1]),
            "pos_1step_max_abs": float(np.abs(d["pos1"] - ref1["pos"]).max()),
        },
        "bounds": {"F_rel": 1e-5, "E_rel": 1e-6, "W_rel": 1e-6},
    }
    return out


def copy_probe_gbs(nbytes=512 << 20, reps=5):
    """HBM bandwidth a plain streaming kernel reaches on this GPU: libmd's
    copy probe over nbytes, bytes read + written per launch over the mean
    launch time (HIP events on the launch stream)."""
    import ctypes
    import torch
    from paper_2109_10876_amd import _abi
    lib = _abi.load()
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    for _ in range(2):
        assert lib.md_copy_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                 nbytes, sp) == 0
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        assert lib.md_copy_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                 nbytes, sp) == 0
        b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    assert torch.equal(src, dst)
    mean = float(np.mean(ms))
    out = {"bytes_each_way": nbytes, "launches": reps, "ms_mean": mean,
           "gbs": 2 * nbytes / (mean * 1e-3) / 1e9}
    del src, dst
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--mode", default="auto", choices=["auto", "full", "half", "tile"],
                    help="list form; auto = chosen by the autotuner (untimed)")
    ap.add_argument("--tile-cells", type=int, default=None,
                    help="tile lists: cells per tile along x (default: largest that fits)")
    ap.add_argument("--tile-rows", type=int, nargs=2, default=[2, 2], metavar=("PY", "PZ"),
                    help="tile lists: rows per tile along y and z")
    ap.add_argument("--tile-threads", type=int, default=256, choices=[64, 128, 256])
    ap.add_argument("--tile-slots", type=int, default=2048, choices=[0, 1536, 2048, 3072],
                    help="tile lists: staged capacity of the 256-thread shape")
    ap.add_argument("--batch", type=int, default=4, choices=[1, 2, 4, 8],
                    help="neighbour gathers issued together")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle leg (CPU baseline and per-result errors)")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the melt / slab / replica-batch throughput lines")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run libmd's 512 MiB streaming copy probe (the calibration "
                         "kernel for HBM byte counters), print its bandwidth and exit")
    ap.add_argument("--workload", default=None,
                    choices=["kg_melt", "ring_melt", "lj_slab", "lj_sphere", "replicas"],
                    help="only time this secondary workload (autotuned, graphed, "
                         "--steps steps) and print its JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(spatial decomposition across GPUs is described, not implemented)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import md_inputs
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload:
        out = time_workload(args.workload, args.steps, warmup=args.warmup)
        print(json.dumps({"workload": args.workload, **out}), flush=True)
        return
    if args.copy_probe:
        print(json.dumps(copy_probe_gbs()), flush=True)
        return
    copy = copy_probe_gbs()
    log(f"copy probe: {json.dumps(copy)}")
    cfg = md_inputs.CONFIGS["lj1m"]()
    from paper_2109_10876_amd import MDSystem, autotune
    if args.mode == "auto":
        def make(mode, tile_cells, tile_rows=(1, 1)):
            return MDSystem(cfg.natoms, cfg.box, cfg.pos, cfg.vel, rc=cfg.rc, skin=cfg.skin,
                            dt=cfg.dt, shift=cfg.shift, mode=mode, prec="mixed",
                            tile_cells=tile_cells, tile_rows=tile_rows)
        key = autotune.signature(cfg.natoms, cfg.box, cfg.rc, cfg.skin, 1)
        tuned, _ = autotune.tune(make, key, steps=40, warmup=10, cache=None, log=log)
    else:
        tuned = {"mode": args.mode, "batch": args.batch, "tile_threads": args.tile_threads,
                 "tile_slots": args.tile_slots, "tile_cells": args.tile_cells,
                 "tile_rows": list(args.tile_rows)}
    log(f"configuration: {json.dumps(tuned)}")
    out, snaps = {}, {}
    for prec in ("mixed", "fp64"):
        log(f"[{prec}] timing {args.steps} steps after {args.warmup} warm-up steps")
        s, ms, f_ms, mean_k, npairs, snap, fused, sections, drift, graphed = time_path(
            cfg, prec, args.steps, args.warmup, tuned)
        snaps[prec] = snap
        n = s.N
        k_half = mean_k / 2.0 if tuned["mode"] != "half" else mean_k
        # algorithmic bytes of one launch (the half-list minimum, each
        # unordered pair once) and the bytes of the list form this run uses
        vv_b = BYTES_PER_ATOM_VV_FUSED if fused else 0
        bytes_min = n * (BYTES_PER_HALF_ENTRY * k_half + BYTES_PER_ATOM_FORCE + vv_b)
        ebytes = 2.0 if tuned["mode"] == "tile" else 4.0
        bytes_own = n * (ebytes * mean_k + BYTES_PER_ATOM_FORCE + vv_b)
        gbs = bytes_min / (f_ms * 1e-3) / 1e9
        # the method's flops, each unordered pair once
        flops_launch = (n * k_half * FLOPS_PER_ENTRY + npairs * FLOPS_PER_PAIR_IN_RC
                        + (n * FLOPS_PER_ATOM_VV if fused else 0))
        tfs = flops_launch / (f_ms * 1e-3) / 1e12
        traffic = traffic_bytes = None
        counted = COUNTED_TRAFFIC.get(tuned["mode"] + ("_fused" if fused else ""))
        per_batch = counted["bytes_per_launch"].get(str(tuned.get("batch", 4))) if counted else None
        if per_batch and force_kernel_src_hash(tuned["mode"]) == counted["src_sha256_16"]:
            traffic_bytes = per_batch[prec]
            traffic = traffic_bytes / (f_ms * 1e-3) / 1e9
        if fused:
            kernel = "md_lj_forces_vv (k_tile_lj fused with velocity-Verlet)"
        else:
            kernel = "md_lj_forces (%s)" % ("k_tile_lj" if tuned["mode"] == "tile" else "k_lj")
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
                "frac_of_copy_probe": gbs / copy["gbs"], "copy_probe_gbs": copy["gbs"],
                "target_frac_of_copy_probe": 0.6,
                "bytes_per_launch": bytes_min,
                "bytes_per_atom": bytes_min / n,
                "bytes_formula": "N x (4 K_half + 52 + 96 if fused), K_half = half-list "
                                 "entries per atom = full-list mean / 2",
                "own_list_bytes_per_launch": bytes_own,
                "own_list_frac": bytes_own / (f_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "traffic_unit": "GB/s", "traffic_bytes_per_launch": traffic_bytes,
                "kernel": kernel, "kernel_ms": f_ms,
                "alu_view": {"achieved": tfs, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": tfs / VALU_PEAK_TFLOPS, "flops_per_launch": flops_launch,
                             "count": "the method's work: each unordered pair once"}}
        out[prec] = {
            "ms_per_step": ms / args.steps,
            "atom_steps_per_s": n * args.steps / (ms * 1e-3),
            "pair_evals_per_s": npairs * args.steps / (ms * 1e-3),
            "pairs_within_rc": npairs,
            "mean_list_entries": mean_k,
            "forces_kernel_ms": f_ms,
            "roofline": roof,
            "drift": drift,
            "graph": graphed,
        }
        # Amdahl-style bound in the spirit of the paper's S_max (Sec. 4.1):
        # the step if the pair kernel ran at the copy-probe bandwidth on its
        # algorithmic bytes, every other section unchanged
        step_us = ms / args.steps * 1e3
        pair_min_us = bytes_min / (copy["gbs"] * 1e9) * 1e6
        sections["s_max_pair_at_copy_bw"] = s_max(
            {"pair": sections["pair_us"], "rest": step_us - sections["pair_us"]}, ("pair",),
            sections["pair_us"] / pair_min_us)
        sections["pair_at_copy_bw_us"] = pair_min_us
        out[prec]["sections"] = sections
        log(f"[{prec}] {json.dumps(out[prec])}")
        del s
        torch.cuda.empty_cache()
    m = out["mixed"]
    line = {
        "metric": "atom-steps/s and pair-evals/s, FP32-mixed vs FP64 path, at force err <=1e-5 rel",
        "value": m["atom_steps_per_s"],
        "unit": "atom-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": "LJ fluid FCC 64^3x4 N=1048576 rho=0.8442 T=1.0 rc=2.5 "
                               "skin=0.3 dt=0.005 NVE", "N": cfg.n, "launch": tuned},
        "pair_evals_per_s": m["pair_evals_per_s"],
        "forces_kernel_ms": m["forces_kernel_ms"],
        "force_err_rel": None,
        "roofline": m["roofline"],
        "copy_probe": copy,
        "sections": m["sections"],
        "graph": m["graph"],
        "drift": {"mixed": m["drift"], "fp64": out["fp64"]["drift"]},
        "err": None,
        "fp64": {k: out["fp64"][k] for k in ("atom_steps_per_s", "pair_evals_per_s",
                                             "ms_per_step", "forces_kernel_ms",
                                             "roofline", "sections")},
        "cpu_baseline": None,
    }
    if not args.no_other:
        other = {}
        for name, steps in (("kg_melt", 300), ("ring_melt", 300), ("lj_slab", 300),
                            ("lj_sphere", 100),
                            ("replicas", 200)):
            log(f"[{name}] timing {steps} steps")
            try:
                other[name] = time_workload(name, steps)
            except Exception as exc:   # a secondary workload never hides the headline
                other[name] = {"error": repr(exc)}
            log(f"[{name}] {json.dumps(other[name])}")
        line["workloads"] = other
    if not args.no_cpu:
        # the oracle leg on the mixed run's final (thermalised) state: CPU
        # timing on one core and on all cores, then the error of every
        # result of the mixed path against the oracle and the FP64 GPU path
        pos, vel = snaps["mixed"]
        log("oracle leg: CPU timing (1 core, all cores) on the final state")
        legs, cpu, ref1 = oracle_leg(pos, vel, cfg.box[0], cfg.rc, cfg.skin, cfg.dt)
        one = legs["single"]
        line["cpu_baseline"] = {
            "value": one["value"], "unit": "atom-steps/s", "cores": one["cores"],
            "kind": "oracle",
            "sample": (f"3 samples of one NVE step of the full {cfg.n}-atom system from the "
                       f"mixed run's final state, each a 1-step minus a 0-step oracle run; "
                       f"median {one['s_per_step_median']:.2f} s/step on 1 core, "
                       f"{legs['all_cores']['s_per_step_median']:.2f} s/step on "
                       f"{legs['all_cores']['cores']} threads"),
            "legs": legs, "host": cpu}
        log("per-result errors of the mixed path")
        err = per_result_errors(cfg, tuned, pos, vel, ref1, args.steps)
        line["err"] = err
        line["force_err_rel"] = err["vs_oracle"]["F_rel"]
        line["fp64"]["force_err_rel"] = err["fp64_gpu_vs_oracle"]["F_rel"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
