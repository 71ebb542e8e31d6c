"""Throughput of the PIC hot path on one MI355X.

Workload: the warm uniform plasma, 2048 x 2048 cells, dx = dy = 0.1,
dt = 0.07, periodic, 16 electrons per cell (67,108,864 particles), u_th = 0.05
with drift u_x = 0.2, tiles of 32 x 32 cells, strict sort every step, FP32
particles with an int32 packed cell index + FP32 in-cell offsets.  Synthetic,
seeded, resident in HBM before the timed region.

A timed step is one full PIC step through the C ABI (pic_step): push +
deposit, then the strict in-place re-sort and the Yee field advance (with the
fold of the tile currents into J) side by side on two streams, joined before
the call returns.  `value` counts particle pushes over the whole step.

Prints ONE JSON line.  The push kernel's duration comes from HIP events that
libpic records around it on its launching stream during the timed region;
the other kernels' split from a few extra steps timed the same way.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-pushes/sec (push+deposit+sort), 1 MI355X; % of HBM roofline"
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
BYTES_PARTICLE = 22          # tile-relative cell (2) + x, y (8) + ux, uy, uz (12)


# The thesis's whole-run figures (500 steps, field solve and overheads
# included, 500^2 decks of 25 M particles, FP32), as pushes/s = particles x
# steps / time (Table 5.4): other hardware and a different workload, context only.
PAPER_CONTEXT = {
    "source": "thesis Table 5.4, warm deck, whole run",
    "serial_cpu_xeon_gold_5218_1core_pushes_per_s": 10.8e6,
    "openmp_2x_xeon_gold_5218_32t_pushes_per_s": 292e6,
    "opencl_radeon_instinct_mi25_pushes_per_s": 2372e6,
    "fpga_arria10_4lane_pushes_per_s": 60.8e6,
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def push_bytes(n_particles, n_tiles, tile, leavers, n_species=1, halo=1):
    """Algorithmic HBM bytes of one push + deposit launch of pic_step: every
    particle read and written once, each tile's E/B halo ((T+2H)^2 cells x 6
    fields, H the halo pad: 1, the sort cadence, or 2 for the quadratic
    shape) read once, each tile's current halo ((T+2H+1)^2 nodes x 3)
    written once, the B half step of the tile's T^2 cells (3 floats each)
    written once, the tile_offset pair and the count record (32 ints) per
    tile and species, and one 4-byte entry per leaver (the leavers' 32-byte
    records are not counted)."""
    return (2 * BYTES_PARTICLE * n_particles
            + n_tiles * (tile + 2 * halo) ** 2 * 6 * 4
            + n_tiles * (tile + 2 * halo + 1) ** 2 * 3 * 4
            + n_tiles * tile * tile * 3 * 4
            + n_species * n_tiles * (8 + 32 * 4)
            + 4 * leavers)


def step_bytes(n_particles, n_tiles, tile, nx, ny, leavers, movers, n_species=1, motion=False, halo=1):
    """Algorithmic HBM bytes of one whole pic_step: the push (push_bytes),
    the hole fill it does for the last sort (per mover: its hole slot and its
    32-byte staged record), the field half (the E step: E read and written,
    the half-step B read, J written, the tile current halos read; the second
    B half step: the half-step B and E read, B written: 21 plane passes) and
    the sort (per tile: nine count-record entries and the offsets; per leaver
    entry 4 B; per mover its 32-byte record read, its staging record written
    and its hole slot).  With motion=True the sort is the motion-class
    counting pass instead (per tile its class counts and offsets; per
    particle its 2-byte cell read to count, then its 22 bytes read and
    written into the staging arrays) and there is no hole fill: the push
    reads the staging arrays, the same bytes as the particle arrays.  halo:
    the push's halo pad (2 for the quadratic shape)."""
    plane = 4 * nx * ny
    field = 21 * plane + n_tiles * (tile + 2 * halo + 1) ** 2 * 3 * 4
    sort = n_species * n_tiles * (9 * 4 + 8) + 4 * leavers + movers * (32 + 32 + 4)
    fill = movers * (4 + 32)
    if motion:
        sort = n_species * n_tiles * (9 * 4 + 8) + (2 * BYTES_PARTICLE + 2) * n_particles
        fill = 0
    return push_bytes(n_particles, n_tiles, tile, leavers, n_species, halo) + fill + field + sort


def cpu_baseline(w, st, T, budget_s=10.0, max_steps=8):
    """The oracle (serial FP64 C) on a bounded sample of the same workload:
    the first 8,388,608 particles (the lower eighth of the grid), full-size
    fields, push + deposit + canonical sort per step, until ~budget_s."""
    import oracle
    s = w.species[0]
    M = min(8 * 1024 * 1024, st["ix"].size)
    sp = oracle.OracleSpecies(s.qm, s.q, *(st[k][:M] for k in ("ix", "iy", "x", "y", "ux", "uy", "uz")))
    sim = oracle.OracleSim(w.nx, w.ny, w.dx, w.dy, w.dt, [sp])
    steps, t_hot = 0, 0.0
    while steps < max_steps and (steps == 0 or t_hot < budget_s):
        t0 = time.perf_counter()
        sim.push_deposit()
        sim.sort(T)
        t_hot += time.perf_counter() - t0
        sim.field_advance()
        steps += 1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": M * steps / t_hot, "unit": "particle-pushes/s", "cores": 1, "kind": "oracle",
            "host_cores": os.cpu_count(), "cpu_model": model,
            "sample": f"first {M} particles (tiles 0-{M // (T * T * s.n_ppc) - 1}, tile {T}) of the "
                      f"{w.nx}x{w.ny} workload, {steps} steps of push+deposit+sort, serial FP64 C "
                      f"(field advance untimed)",
            "seconds": t_hot}


def cpu_baseline_openmp(w, st, T, steps=3):
    """The oracle's OpenMP driver (Sec. 4.2.1's CPU scheme: an OpenMP loop over
    tiles, a private current per thread; the canonical sort split over
    threads) on the WHOLE workload, on every host core it is given
    (OMP_NUM_THREADS); push + deposit + sort timed per step, the median of
    `steps` steps (the field advance untimed)."""
    import oracle
    s = w.species[0]
    sp = oracle.OracleSpecies(s.qm, s.q, *(st[k] for k in ("ix", "iy", "x", "y", "ux", "uy", "uz")))
    sim = oracle.OracleOmpSim(w.nx, w.ny, w.dx, w.dy, w.dt, [sp], T)
    times = []
    for _ in range(steps):
        t0 = time.perf_counter()
        sim.push_deposit()
        sim.sort()
        times.append(time.perf_counter() - t0)
        sim.field_advance()
    n = sp.n
    med = float(np.median(times))
    return {"value": n / med, "unit": "particle-pushes/s", "cores": oracle.omp_threads(), "kind": "oracle-openmp",
            "sample": f"all {n} particles of the {w.nx}x{w.ny} workload, median of {steps} steps of "
                      f"push+deposit+sort (FP64, OpenMP over {T}x{T} tiles, private current per thread)",
            "step_s": times}


def stream_probe(n=1 << 26, launches=20):
    """The push's particle stream without its arithmetic (pic_probe_stream):
    one 16-bit and five float arrays of n values read and written back in
    place, with and without the non-temporal hint, event-timed; and a plain
    device copy of the same bytes.  Returns achieved GB/s (44 n bytes per
    launch)."""
    import torch

    from paper_2501_14795_amd import _lib
    nb = 2 * BYTES_PARTICLE * n
    arrays = [torch.zeros(n, dtype=torch.int16, device="cuda")]
    arrays += [torch.zeros(n, dtype=torch.float32, device="cuda") for _ in range(5)]
    ptrs = [a.data_ptr() for a in arrays]
    s = torch.cuda.current_stream().cuda_stream
    out = {"elements": n, "bytes_per_launch": nb}
    for name, nt in (("soa_rw_nontemporal", True), ("soa_rw", False)):
        for _ in range(3):
            _lib.pic_probe_stream(ptrs, n, nt, s)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(launches):
            _lib.pic_probe_stream(ptrs, n, nt, s)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / launches
        out[name + "_gbs"] = nb / (ms * 1e-3) / 1e9
    src = torch.ones(BYTES_PARTICLE * n // 2, dtype=torch.int16, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(launches):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    out["copy_gbs"] = nb / (e0.elapsed_time(e1) / launches * 1e-3) / 1e9
    del arrays, src, dst
    torch.cuda.empty_cache()
    return out


def batched_comparison(n_sims=256, steps=20, tune_sims=32):
    """The batched workload (256 independent simulations, grids 32..256
    cells, 8..64 ppc): the autotuner times its candidates on the first
    tune_sims members and the three fastest again on the whole batch, then the
    full batch runs as
    captured-graph replays, as direct batched launches, and one simulation per
    launch sequence (pic_step on each member in turn, the same cadence), all
    on the same members and data."""
    import torch

    import pic_workloads as pw
    from paper_2501_14795_amd import Batch, _lib
    from paper_2501_14795_amd.tune import autotune_batch, time_batch

    specs = pw.batched_members(n_sims, 4)

    def build(tile, subset=None):
        out = []
        for m in (specs if subset is None else specs[:subset]):
            st = pw.species_state(m["nx"], m["ny"], tile, m["spec"], m["seed"])
            out.append({"nx": m["nx"], "ny": m["ny"], "dx": m["dx"], "dy": m["dy"], "dt": m["dt"],
                        "species": [(m["spec"].qm, m["spec"].q, st)]})
        return out

    t0 = time.perf_counter()
    (tile, reps, every, ppl, motion), tuning, refined = autotune_batch(lambda T: build(T, tune_sims),
                                                                       refine_members=lambda T: build(T))
    log(f"autotuned tile {tile} replicas {reps} sort_every {every} particles/lane {ppl} motion sort {motion} in "
        f"{time.perf_counter() - t0:.1f}s: {tuning}")
    members = build(tile)
    n = sum(m["species"][0][2]["ix"].size for m in members)
    b = Batch(members, tile=tile, j_replicas=reps, sort_every=every, ppl=ppl, motion_sort=motion)
    del members
    direct = time_batch(b, steps)
    # one simulation per launch sequence, on the same members
    s = b.stream.cuda_stream
    steps = -(-steps // every) * every   # whole cadence cycles
    for _ in range(every):
        for m in b.members:
            _lib.pic_step(m.handle, s)
    b.stream.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for m in b.members:
            _lib.pic_step(m.handle, s)
    b.sync()
    b.stream.synchronize()
    per_sim = (time.perf_counter() - t0) / steps
    # the batched push alone, event-timed in direct batched steps: its
    # algorithmic bytes (every member's push bytes, as for one simulation)
    # over its average duration
    m0 = b[0]
    m0.set_timing(["push"])
    b.step(steps)
    b.stream.synchronize()
    kt = m0.timing()["push"]
    m0.set_timing(False)
    push_ms = kt[0] / max(kt[1], 1)
    bytes_push = 0
    for m in b.members:
        d = m.diag(_lib.PIC_DIAG_COUNTS)
        bytes_push += push_bytes(m.buf.cfg.species[0].n, m.n_tiles, tile, d.leavers[0], halo=every)
    b.capture()
    graph = time_batch(b, steps)
    rc = b.check()
    b.close()
    if rc != 0:
        raise SystemExit(f"device error in the batched run: {_lib.strerror(rc)}")
    return {
        "workload": f"{n_sims} simulations, grids 32..256 cells, 8..64 ppc (seed 4)",
        "particles": n, "steps": steps, "tile": tile, "j_replicas": reps, "sort_every": every,
        "particles_per_lane": ppl, "sort": "motion-class" if motion else "in-place",
        "autotune_ms_per_step": {f"T{k[0]}_R{k[1]}_S{k[2]}_P{k[3]}{'_M' if k[4] else ''}": v * 1e3
                                 for k, v in tuning.items()},
        "autotune_refined_ms_per_step": {f"T{k[0]}_R{k[1]}_S{k[2]}_P{k[3]}{'_M' if k[4] else ''}": v * 1e3
                                         for k, v in refined.items()},
        "graph_pushes_per_s": n / graph, "direct_pushes_per_s": n / direct,
        "per_sim_launch_pushes_per_s": n / per_sim,
        "graph_ms_per_step": graph * 1e3, "direct_ms_per_step": direct * 1e3,
        "per_sim_launch_ms_per_step": per_sim * 1e3,
        "speedup_vs_per_sim_launch": per_sim / graph,
        "roofline": {"bound": "hbm", "kernel": "k_push_batch", "avg_launch_ms": push_ms,
                     "algorithmic_bytes_per_launch": bytes_push,
                     "achieved": bytes_push / (push_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": bytes_push / (push_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }


def filter_measurement(w, launches=20):
    """One binomial current-filter pass over the workload's grid (three FP32
    planes in, three out: 24 B per node), event-timed on a particle-free
    simulation of the same grid with one filter pass per step."""
    import numpy as np

    from paper_2501_14795_amd import Sim
    empty = {k: np.zeros(0, np.int32 if k in ("ix", "iy") else np.float32)
             for k in ("ix", "iy", "x", "y", "ux", "uy", "uz")}
    sim = Sim(w.nx, w.ny, w.dx, w.dy, w.dt, w.tile, [(-1.0, -1.0, empty)], j_filter=1)
    for _ in range(3):
        sim.push_deposit()
        sim.sort()
    sim.set_timing(["filter"])
    for _ in range(launches):
        sim.push_deposit()
        sim.sort()
    kt = sim.timing()
    sim.set_timing(False)
    sim.close()
    ms = kt["filter"][0] / max(kt["filter"][1], 1)
    nbytes = 24 * w.nx * w.ny
    return {"kernel": "k_binomial_f", "grid": f"{w.nx}x{w.ny}", "pass_ms": ms, "bytes_per_pass": nbytes,
            "achieved": nbytes / (ms * 1e-3) / 1e9, "unit": "GB/s", "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def variant_measurement(w, T, steps=20, warmup=3, **options):
    """The same workload and step with a library option (the Esirkepov
    deposit, the full re-sort, ...): whole-step rate and the event-timed
    kernel durations per step."""
    import torch

    import pic_workloads as pw
    from paper_2501_14795_amd import Sim
    states = pw.workload_state(w, tile=T)
    n = sum(s["ix"].size for s in states)
    sim = Sim(w.nx, w.ny, w.dx, w.dy, w.dt, T, [(s.qm, s.q, st) for s, st in zip(w.species, states)], **options)
    del states
    for _ in range(warmup):
        sim.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sim.step()
    sim.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # per-kernel split from as many extra, event-timed steps
    sim.set_timing(True)
    for _ in range(steps):
        sim.step()
    torch.cuda.synchronize()
    kt = sim.timing()
    sim.set_timing(False)
    rc = sim.check()
    sim.close()
    if rc != 0:
        raise SystemExit(f"device error in the {options} measurement")
    return {"workload": w.name, "tile": T, "options": options, "steps": steps,
            "pushes_per_s": n * steps / elapsed, "ms_per_step": elapsed * 1e3 / steps,
            "kernel_ms_per_step": {k: v[0] / steps for k, v in kt.items()}}


def window_measurement(w, T, moves=20, warmup=3, n_columns=4):
    """The moving-window step on the same workload: after each full step the
    window moves one cell (pic_move_window) and a new column of plasma of the
    workload's species, ppc and temperature comes in (pre-drawn, resident in
    HBM, cycled over n_columns draws).  pic_move_window synchronises, so the
    window call is wall-timed on its own; the steps between are not counted."""
    import torch

    import pic_workloads as pw
    from paper_2501_14795_amd import Sim, _lib
    states = pw.workload_state(w, tile=T)
    n = [st["ix"].size for st in states]
    col_n = [int(np.ceil(k / w.nx)) * 2 for k in n]
    sim = Sim(w.nx, w.ny, w.dx, w.dy, w.dt, T, [(s.qm, s.q, st) for s, st in zip(w.species, states)],
              moving_window=True, capacity=[k + c for k, c in zip(n, col_n)])
    del states
    cols = []
    for c in range(n_columns):
        per = []
        for k, spec in enumerate(w.species):
            st = pw.species_state(T, w.ny, T, spec, w.seed + 1000 + c, k, cell_box=(T - 1, T, 0, w.ny))
            st["ix"] = st["ix"] + (w.nx - T)
            per.append(sim.upload_particles(st))
        cols.append(per)
    times = []
    for i in range(warmup + moves):
        sim.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.move_window(cols[i % n_columns])
        if i >= warmup:
            times.append(time.perf_counter() - t0)
    counts = sim.counts()
    d = sim.diag(_lib.PIC_DIAG_COUNTS)   # of the last move
    removed, movers = list(d.leavers)[:len(w.species)], list(d.movers)[:len(w.species)]
    rc = sim.check()
    sim.close()
    if rc != 0:
        raise SystemExit("device error in the moving-window measurement")
    ms = 1e3 * sum(times) / len(times)
    return {"workload": w.name, "moves": moves, "window_ms": ms, "window_ms_min": 1e3 * min(times),
            "new_per_move": [int(t["cell"].numel()) for t in cols[0]],
            "last_move": {"removed": removed, "moved_by_sort": movers}, "particles_after": counts}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--tile", type=int, default=0, help="tile edge (default: the workload's)")
    ap.add_argument("--replicas", type=int, default=0)
    ap.add_argument("--workload", default="warm2048")
    ap.add_argument("--j-float", action="store_true", help="FP32-atomic LDS current instead of fixed point")
    ap.add_argument("--j-filter", type=int, default=0, help="binomial current filter passes in the timed step")
    ap.add_argument("--esirkepov", action="store_true", help="Esirkepov deposit instead of split Villasenor-Buneman")
    ap.add_argument("--quadratic", action="store_true",
                    help="the quadratic particle shape (gather and Esirkepov deposit) in the timed step")
    ap.add_argument("--motion-sort", action="store_true",
                    help="the motion-class sort instead of the in-place one in the timed step")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the short measurements of the filter pass and of the Esirkepov deposit")

    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-mode comparison")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (a known-size "
                         "reference kernel for the HBM byte counters of a profiling run)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "push_traffic.json"),
                    help="HBM traffic of the push kernel measured by rocprofv3 PMC runs (optional)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is "
              f"not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch

    import pic_workloads as pw
    from paper_2501_14795_amd import Sim, _lib

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = pw.WORKLOADS[args.workload]
    T = args.tile or w.tile
    t0 = time.perf_counter()
    states = pw.workload_state(w, tile=T)
    n = sum(s["ix"].size for s in states)
    log(f"generated {n} particles in {time.perf_counter() - t0:.1f}s")

    cpu = None
    if not args.no_cpu_baseline and len(states) == 1:
        cpu = cpu_baseline(w, states[0], T)
        log(f"cpu baseline {cpu['value'] / 1e6:.2f} M push/s over {cpu['seconds']:.1f}s")
        cpu["openmp"] = cpu_baseline_openmp(w, states[0], T)
        log(f"cpu baseline (OpenMP, {cpu['openmp']['cores']} threads) {cpu['openmp']['value'] / 1e6:.1f} M push/s, "
            f"steps {cpu['openmp']['step_s']}")
    probe = stream_probe()
    log(f"stream probe: {probe}")

    sim = Sim(w.nx, w.ny, w.dx, w.dy, w.dt, T, [(s.qm, s.q, st) for s, st in zip(w.species, states)],
              j_replicas=args.replicas, j_float=args.j_float, j_filter=args.j_filter, esirkepov=args.esirkepov,
              motion_sort=args.motion_sort, quadratic=args.quadratic)
    del states
    log("initialised")
    for _ in range(args.warmup):
        sim.step()
    rc = sim.check()
    if rc != 0:
        raise SystemExit(f"device error after warmup: {_lib.strerror(rc)}")

    # the timed region: HIP events around the push kernel only (each event
    # pair adds a little time to a step), on the stream it is launched on
    torch.cuda.synchronize()
    sim.set_timing(["push"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sim.step()
    sim.sync()   # the last sort's hole fill (the next push would do it) inside the timed region
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt_push = sim.timing()["push"]
    sim.set_timing(False)
    rc = sim.check()
    if rc != 0:
        raise SystemExit(f"device error in the timed region: {_lib.strerror(rc)}")
    d = sim.diag(_lib.PIC_DIAG_COUNTS | _lib.PIC_DIAG_ENERGY)
    leavers = sum(d.leavers[k] for k in range(len(w.species)))
    movers = sum(d.movers[k] for k in range(len(w.species)))
    # per-kernel split: a short extra run with every kernel event-timed
    split_steps = min(args.steps, 20)
    sim.set_timing(True)
    for _ in range(split_steps):
        sim.step()
    torch.cuda.synchronize()
    kt = sim.timing()
    sim.set_timing(False)

    ms_step = elapsed * 1e3 / args.steps
    value = n * args.steps / elapsed
    push_ms = kt_push[0] / max(kt_push[1], 1)
    halo = 2 if args.quadratic else 1
    pb = push_bytes(n, sim.n_tiles, T, leavers, len(w.species), halo)
    achieved = pb / (push_ms * 1e-3) / 1e9
    sb = step_bytes(n, sim.n_tiles, T, w.nx, w.ny, leavers, movers, len(w.species), motion=args.motion_sort,
                    halo=halo)
    step_gbs = sb / (ms_step * 1e-3) / 1e9
    hot_ms = sum(kt[k][0] for k in ("push", "j_reduce", "sort_scan", "sort_plan", "sort_scatter")) / split_steps

    traffic = None
    # the counters were taken on the default push (split Villasenor-Buneman
    # deposit, fixed-point current, in-place sort, no filter)
    default_push = not (args.esirkepov or args.j_float or args.motion_sort or args.j_filter or args.replicas > 1 or
                        args.quadratic)
    if default_push and os.path.exists(args.traffic_json):
        try:
            tj = json.load(open(args.traffic_json))
            if tj.get("workload") == w.name and tj.get("tile") == T and tj.get("kernel_source_sha") == \
                    _kernel_sha():
                traffic = tj.get("bytes_per_launch")
        except Exception:
            traffic = None

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "dx": w.dx, "dt": w.dt,
                   "particles": n, "ppc": sum(s.n_ppc for s in w.species), "tile": T,
                   "j_accumulation": "fp32-atomic" if args.j_float else "int64-fixed-point",
                   "j_replicas": args.replicas or ((4 if T < 32 else 2) if args.j_float else 1),
                   "sort_every": 1, "j_filter": args.j_filter,
                   "deposit": ("esirkepov-quadratic" if args.quadratic else
                               "esirkepov" if args.esirkepov else "villasenor-buneman-split"),
                   "sort": "motion-class" if args.motion_sort else "in-place",
                   "step": "push+deposit+sort+field_advance"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_source": None if traffic is None else
                     "rocprofv3 FETCH_SIZE/WRITE_SIZE passes of this kernel source (profiles/push_traffic.json)",
                     "kernel": "k_push_deposit", "algorithmic_bytes_per_launch": pb,
                     "avg_launch_ms": push_ms,
                     "probe_gbs": probe["soa_rw_nontemporal_gbs"],
                     "frac_of_probe": achieved / probe["soa_rw_nontemporal_gbs"],
                     "probe": probe,
                     # the whole step (push, hole fill, field half, sort) against the same peak
                     "step": {"algorithmic_bytes": sb, "achieved": step_gbs, "frac": step_gbs / HBM_PEAK_GBS,
                              "frac_of_probe": step_gbs / probe["soa_rw_nontemporal_gbs"]}},
        "hot_path": {
            "ms_per_step": hot_ms,
            "pushes_per_s": n / (hot_ms * 1e-3),
            "kernel_ms_per_step": {k: v[0] / split_steps for k, v in kt.items()},
            "split_steps": split_steps,
            "leavers_per_step": leavers, "movers_per_step": movers,
        },
        "energy": {"u_e": d.u_e, "u_b": d.u_b, "u_k": d.u_k[0]},
        "paper_context": PAPER_CONTEXT,
        "cpu_baseline": None if cpu is None else {k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample",
                                                                     "host_cores", "cpu_model", "openmp")},
    }
    sim.close()
    del sim
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not args.no_variants:
        out["filter_pass"] = filter_measurement(w)
        log(f"filter pass: {out['filter_pass']}")
        if not args.esirkepov:
            out["esirkepov"] = variant_measurement(w, T, esirkepov=True)
            log(f"esirkepov: {out['esirkepov']}")
        if not args.quadratic:
            out["quadratic"] = variant_measurement(w, T, quadratic=True)
            log(f"quadratic shape: {out['quadratic']}")
        out["motion_sort"] = variant_measurement(w, T, motion_sort=True)
        log(f"motion-class sort: {out['motion_sort']}")
        for ppl in (1, 4):
            out[f"particles_per_lane_{ppl}"] = variant_measurement(w, T, ppl=ppl)
            log(f"{ppl} particle(s) per lane: {out[f'particles_per_lane_{ppl}']}")
        out["moving_window"] = window_measurement(w, T)
        log(f"moving window: {out['moving_window']}")
    if not args.no_batched:
        out["batched"] = batched_comparison()
        log(f"batched: {out['batched']}")
    print(json.dumps(out), flush=True)


def _kernel_sha():
    """Hash of what the push kernel's translation unit is compiled from:
    k_push.hip, the definitions it shares (pic_push.h) and the fold it
    includes (pic_fold.h); pic_internal.h adds only launcher declarations and
    other kernels' structures to them."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2501_14795_amd", "csrc")
    for name in ("k_push.hip", "pic_push.h", "pic_fold.h"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
