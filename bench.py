"""Benchmark: EAM atom-steps/s of the MI355X force loop (one JSON line).

Default workload: bcc Fe, 80^3 cells with 1% random vacancies (N = 1,013,760),
600 K, neighbour list rebuilt every 10 steps.  A step is one pass of the whole
hot path: (scheduled) cell sort + list build, density pass with embedding,
force pass with velocity-Verlet update, and - on the last step of each
md_step call - the energy/virial reductions; the `energy_every_step` leg
reduces energies and the virial on every step.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload bcc1m]

`value` is the FP64 rate (the paper's precision).  The mixed-precision rate
(FP32 pair terms, FP64 accumulation and integration), gated on its force
error against the FP64 path, is reported beside it with its own roofline.
Inputs are seeded and synthetic and already resident in HBM when the timed
region starts.
"""
from __future__ import annotations

import argparse
import copy
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "EAM atom-steps/s: mixed vs FP64 (force err ≤1e-5), batched vs one-by-one"
HBM_PEAK_GBS = 8000.0

# HBM bytes of one launch of the force kernel on bcc1m, per precision and
# evaluator (the autotuner may pick either for FP64: FP64 knot sums or FP64
# tables, four records in flight; mixed: tables, eight), from two rocprofv3
# --pmc passes (FETCH_SIZE, WRITE_SIZE; KiB per dispatch, mean of 185
# dispatches), each scaled by the reading for a plain 1 GiB device copy
# (FETCH_SIZE reads 524,300 KiB -> x2.0; WRITE_SIZE reads 1,048,576 KiB ->
# x1.0); and the VALU instructions per wavefront of the same kernels
# (SQ_INSTS_VALU / SQ_WAVES: a wave carries 64 atoms, so this is also the
# lane-operations per atom of one launch).  Valid only for the kernel sources
# they were taken with (hash below); after any change the bench reports null
# until the counters are taken again.
_COUNTED = {"fetch_scale": 2.0, "write_scale": 1.0, "sources_sha256_16": "9f245d71b74f2274", "workload": "bcc1m",
            "kernel": "k_force"}
FORCE_TRAFFIC = {  # (precision, evaluator) -> counters of the step's force kernel (velocity-Verlet variant)
    ("fp64", 1): {"fetch_kib": 103008, "write_kib": 55440, "valu_per_wave": 2055.9, **_COUNTED},
    ("fp64", 0): {"fetch_kib": 102167, "write_kib": 55440, "valu_per_wave": 1444.4, **_COUNTED},
    ("mixed", 0): {"fetch_kib": 115742, "write_kib": 71280, "valu_per_wave": 1619.5, **_COUNTED},
}
# Lane-operation issue peak of the vector ALUs: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz (FP64 and unpacked FP32 issue at the same rate; packed FP32 is off).
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
FORCE_SOURCES = ["paper_1107_2619_amd/csrc/kernels.hip", "paper_1107_2619_amd/csrc/kernels_brick.hip",
                 "paper_1107_2619_amd/csrc/md_device.h", "paper_1107_2619_amd/csrc/md_internal.h"]
# The paper's own timings (section "Parallel benchmarks"), quoted as context
# only: they are FP64 runs of a Fortran 95 / OpenMP code on other hardware and
# are never used as a ratio.
PAPER_CONTEXT = {
    "hardware": "4 x quad-core Intel Xeon E7310, 1.6 GHz, 16 GB shared memory, up to 16 OpenMP threads",
    "precision": "FP64 (full 64-bit precision)",
    "code": "MOLDY, Fortran 95 + OpenMP (2011)",
    "workload": "bcc Fe, 15-spline iron potential, 300 K, Parrinello-Rahman at 0.1 GPa, dt 1 fs, 1000 steps, "
                "no neighbour-list update during the run",
    "runtime_per_atom": "about 0.013 at 16 threads for the smallest systems, levelling off near 0.092 from "
                        "32k atoms up (the unit is not recoverable from the text; no rate is derived from it)",
    "weak_scaling": "16 threads with ~18.4k atoms each take 1.4x the one-thread time of 18,432 atoms",
    "neighbour_list": "a full list update costs about twice a force evaluation (serial list routine)",
}


def force_sources_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in FORCE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def force_kernel_bytes_per_atom(nbar: float) -> float:
    """Algorithmic HBM bytes of one force-pass launch per atom: read x and F'_i
    (32), read and write v (48), write the drifted x (24), and the neighbour
    list counted once per unordered pair as a 32-bit index (2 n_bar)."""
    return 32.0 + 48.0 + 24.0 + 2.0 * nbar


def step_bytes_per_atom(nbar: float, k: int) -> float:
    """Algorithmic bytes of a whole step per atom (both passes plus the list
    build amortised over the rebuild period k)."""
    return 136.0 + 4.0 * nbar + (56.0 + 2.0 * nbar) / k


def roofline_for(r, prec, nbar, n, k, workload, copy_gbs):
    """HBM roofline of the force kernel of one precision's timed run: the
    algorithmic bytes per launch (force_kernel_bytes_per_atom x N) over the
    kernel's mean duration (HIP events on its launch stream), against the
    MI355X peak; traffic from committed FETCH/WRITE counters when they were
    taken on these kernel sources, else null."""
    force_us = r["force_kernel_us"]
    fbytes = force_kernel_bytes_per_atom(nbar) * n
    achieved = fbytes / (force_us * 1e-6) / 1e9
    kernel = "k_brick_force" if r["autotuned"].get("kernel") == 0 else "k_force"
    t = FORCE_TRAFFIC.get((prec, r["autotuned"].get("evaluator")))
    valid = (t is not None and workload == t["workload"] and kernel == t["kernel"]
             and force_sources_hash() == t["sources_sha256_16"])
    traffic_bytes = 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) if valid else None
    alu = None
    if valid:
        lane_ops = t["valu_per_wave"] * n / (force_us * 1e-6)
        alu = {"achieved": lane_ops / 1e12, "peak": VALU_PEAK_LANE_OPS / 1e12, "unit": "T lane-ops/s",
               "frac": lane_ops / VALU_PEAK_LANE_OPS, "valu_instr_per_wave": t["valu_per_wave"]}
    step_b = step_bytes_per_atom(nbar, k)
    return {
        "bound": "hbm",
        "kernel": f"{kernel} ({prec}: force pass + velocity Verlet)",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic_bytes / (force_us * 1e-6) / 1e9 if valid else None,
        "traffic_bytes_per_launch": traffic_bytes,
        "algorithmic_bytes_per_launch": fbytes,
        "bytes_per_atom": force_kernel_bytes_per_atom(nbar),
        "force_kernel_us": force_us,
        "step_bytes_per_atom": step_b,
        "step_frac": step_b * r["value"] / 1e9 / HBM_PEAK_GBS,
        "measured_copy_GBs": copy_gbs,
        "alu": alu,
    }


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def timed_steps(sim, steps):
    """Milliseconds of one md_step(steps) call between HIP events on the
    caller's stream (barriers on both sides), and the wall time."""
    import torch

    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    sim.step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1), time.perf_counter() - wall0


AUTO_GRAPH_STEPS = 16  # steps per captured graph with automatic rebuilds (a library constant)


def run_precision(md, system, precision, steps, warmup, timing, nbr_mode="full", tune=None, nvt=None,
                  integrator="verlet", energy_every=0, energy_ring=0):
    """A warmed-up timed run.  tune: options to apply (e.g. an autotuner's
    choice); graph replay is used unless per-kernel timing is requested.
    nvt: (targets [R] K, thermostat masses [R] eV fs^2) for a Nose-Hoover run.
    energy_every: reduce energies every that many steps into a ring of
    energy_ring entries.  The timed call continues from the last warm-up
    call (no reload and no force pass at its entry)."""
    kw = {} if nvt is None else {"nh_temperature": nvt[0], "nh_mass": nvt[1]}
    kw["integrator"] = integrator
    sim = md.Simulation(system, precision=precision, want_e_atom=False, nbr_mode=nbr_mode,
                        energy_ring=energy_ring, **kw)
    for opt, val in (tune or {}).items():
        sim.set_option(opt, val)
    if energy_every:
        sim.set_option(md.MD_OPT_ENERGY_EVERY, energy_every)
    if not timing:
        sim.set_option(md.MD_OPT_USE_GRAPH, 1)
        # two warm-up calls long enough to capture the graphs of both ping-pong
        # states a call can start in (a graph spans two rebuild periods), each a
        # whole number of graph spans, so that the timed call starts on a span
        # boundary and replays its steps from the graphs
        auto = bool((tune or {}).get(md.MD_OPT_AUTO_REBUILD, 0))
        span = AUTO_GRAPH_STEPS if auto else 2 * system.rebuild_every
        calls = [span * -(-max(warmup, 2 * span + 2) // span)] * 2
    else:
        calls = [warmup]
    sim.set_option(md.MD_OPT_TIMING, 1 if timing else 0)
    for w in calls:
        sim.step(w)
        sim.energy()
    if timing:
        sim.kernel_times(reset=True)
    builds0 = sim.get_option(md.MD_OPT_N_BUILDS)
    ms, wall = timed_steps(sim, steps)
    en = sim.energy()
    sim.timed_builds = sim.get_option(md.MD_OPT_N_BUILDS) - builds0
    kt = sim.kernel_times(reset=True) if timing else None
    sim.warmup_steps = sum(calls)
    return sim, ms, wall, en, kt


def choice_options(md, ch):
    """The md_set_option settings of an autotuner choice."""
    return {md.MD_OPT_KERNEL: ch["kernel"], md.MD_OPT_BRICK_DIMS: ch["brick_dims"] if ch["kernel"] == 0 else 0,
            md.MD_OPT_LANES_PER_ATOM: ch["lanes"], md.MD_OPT_BRICK_BLOCK: ch["block"],
            md.MD_OPT_EVALUATOR: ch["evaluator"], md.MD_OPT_NEIGHBOUR_CHUNK: ch.get("nchunk", 4)}


def tune_options(md, system, precision):
    """md_autotune on the workload; returns the options it chose."""
    sim = md.Simulation(system, precision=precision, want_e_atom=False)
    ch = sim.autotune(trials=3)
    log(f"autotune {precision}: {ch}")
    del sim
    return choice_options(md, ch), ch


def nvt_vs_nve(md, system, name, steps, warmup, ch, precision="mixed", tau_fs=100.0):
    """A batched workload with a Nose-Hoover thermostat per replica (target:
    the replica's initial temperature; Q = g k_B T tau^2) timed beside the
    same run without it, with the same kernel settings: atom-steps/s of both."""
    opts = choice_options(md, ch)
    targets, q = nh_masses(system, tau_fs)
    sim, ms_nve, _, _, _ = run_precision(md, system, precision, steps, warmup, timing=False, tune=opts)
    del sim
    sim, ms_nvt, _, _, _ = run_precision(md, system, precision, steps, warmup, timing=False, tune=opts,
                                         nvt=(targets, q))
    del sim
    nve = system.n_atoms * steps / (ms_nve * 1e-3)
    nvt = system.n_atoms * steps / (ms_nvt * 1e-3)
    log(f"{name} NVT: {nvt:.3e} atom-steps/s, NVE {nve:.3e} ({ms_nvt / ms_nve - 1.0:+.1%})")
    return {"workload": name, "n_replicas": system.n_replicas, "n_atoms": system.n_atoms, "precision": precision,
            "steps": steps, "tau_fs": tau_fs, "nvt": nvt, "nve": nve, "overhead": ms_nvt / ms_nve - 1.0,
            "nvt_ms_per_step": ms_nvt / steps}


def batched_vs_one_by_one(md, system, name, steps, warmup, precision="mixed"):
    """The replicas of a batched workload run (a) together, one launch per
    kernel per step, autotuned, with graph replay, and (b) one by one through
    the single-system path with the same kernel settings and their own graphs.
    atom-steps/s of both."""
    log(f"{name}: {system.n_replicas} replicas, {system.n_atoms} atoms, {precision}")
    opts, ch = tune_options(md, system, precision)
    sim, ms, _, en, _ = run_precision(md, system, precision, steps, warmup, timing=False, tune=opts)
    batched = system.n_atoms * steps / (ms * 1e-3)
    del sim
    total_ms = 0.0
    for r in range(system.n_replicas):
        sub = system.replica(r)
        if sub.n_atoms == 0:
            continue
        s1, ms1, _, _, _ = run_precision(md, sub, precision, steps, warmup, timing=False, tune=opts)
        total_ms += ms1
        del s1
    one = system.n_atoms * steps / (total_ms * 1e-3)
    log(f"{name}: batched {batched:.3e}, one-by-one {one:.3e} atom-steps/s")
    return {
        "workload": name,
        "n_replicas": system.n_replicas,
        "n_atoms": system.n_atoms,
        "precision": precision,
        "steps": steps,
        "batched": batched,
        "one_by_one": one,
        "speedup": batched / one,
        "batched_ms_per_step": ms / steps,
        "autotuned": {k: v for k, v in ch.items()},
        "pe_per_atom_eV": float(np.sum(en.pe) / system.n_atoms),
    }


def auto_rebuild_leg(md, system, name, steps, warmup, skins, precision, fixed=None):
    """Automatic rebuilds (a rebuild of a replica whenever one of its atoms
    moved more than skin/2, checked every step) at several skins, each
    autotuned with the option on, beside the workload's fixed update period
    (`fixed`: its atom-steps/s at its own skin and period)."""
    runs = []
    for skin in skins:
        s2 = copy.copy(system)
        s2.skin = skin
        sim = md.Simulation(s2, precision=precision, want_e_atom=False)
        sim.set_option(md.MD_OPT_AUTO_REBUILD, 1)
        ch = sim.autotune(trials=3)
        del sim
        opts = {**choice_options(md, ch), md.MD_OPT_AUTO_REBUILD: 1}
        sim, ms, _, en, _ = run_precision(md, s2, precision, steps, warmup, timing=False, tune=opts)
        rate = system.n_atoms * steps / (ms * 1e-3)
        runs.append({"skin": skin, "value": rate, "ms_per_step": ms / steps, "builds": sim.timed_builds,
                     "steps_per_build": steps / max(sim.timed_builds, 1), "autotuned": ch,
                     "temperature_K_mean": float(np.mean(en.temperature))})
        log(f"{name} auto rebuild {precision} skin {skin}: {rate:.3e} atom-steps/s, {sim.timed_builds} builds "
            f"in {steps} steps")
        del sim
    best = max(runs, key=lambda r: r["value"])
    out = {"workload": name, "n_atoms": system.n_atoms, "n_replicas": system.n_replicas, "precision": precision,
           "steps": steps, "runs": runs, "best_skin": best["skin"], "best": best["value"],
           "fixed_period": {"skin": system.skin, "rebuild_every": system.rebuild_every, "value": fixed}}
    if fixed:
        out["best_vs_fixed"] = best["value"] / fixed
    return out


def nh_masses(system, tau_fs):
    """Thermostat mass per replica, Q = g k_B T tau^2 (g as in the temperature)."""
    from paper_1107_2619_amd.inputs import KB_EV

    targets = np.asarray(system.temperature, np.float64)
    n = np.diff(system.atom_offset)
    n_mobile = np.array([int((system.rigid[a:b] == 0).sum()) for a, b in zip(system.atom_offset[:-1],
                                                                            system.atom_offset[1:])])
    dof = np.where(n_mobile < n, 3 * n_mobile, np.maximum(3 * n_mobile - 3, 1))
    return targets, dof * KB_EV * np.maximum(targets, 1.0) * tau_fs**2


def diffusion_leg(md, system, name, steps, warmup, sample_every, precision="mixed", tau_fs=100.0):
    """The self-diffusion workload ("Self-diffusion in iron"): every replica
    thermostatted at its own temperature, the mean square displacement
    sampled every `sample_every` steps inside the timed region (each sample
    synchronises), then the md_msd call on its own."""
    import torch

    log(f"{name}: {system.n_replicas} replicas, {system.n_atoms} atoms, {precision}, NVT, "
        f"MSD every {sample_every} steps")
    opts, ch = tune_options(md, system, precision)
    targets, q = nh_masses(system, tau_fs)
    sim = md.Simulation(system, precision=precision, want_e_atom=False, nh_temperature=targets, nh_mass=q)
    for opt, val in opts.items():
        sim.set_option(opt, val)
    sim.set_option(md.MD_OPT_USE_GRAPH, 1)
    for _ in range(2):
        sim.step(max(warmup, 4 * system.rebuild_every + 2))
    sim.msd_origin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    samples = []
    for _ in range(steps // sample_every):
        sim.step(sample_every)
        samples.append(sim.msd()[0][:, 0])
    elapsed = time.perf_counter() - t0
    n_steps = sample_every * (steps // sample_every)
    t1 = time.perf_counter()
    for _ in range(50):
        sim.msd()
    msd_call_us = (time.perf_counter() - t1) / 50 * 1e6
    en = sim.energy()
    last = samples[-1]
    by_t = {}
    for t in np.unique(targets):
        sel = targets == t
        by_t[f"{t:.0f}"] = {"msd_A2": float(last[sel].mean()), "temperature_K": float(en.temperature[sel].mean())}
    value = system.n_atoms * n_steps / elapsed
    log(f"{name}: {value:.3e} atom-steps/s with MSD sampling, md_msd call {msd_call_us:.1f} us")
    del sim
    return {"workload": name, "n_replicas": system.n_replicas, "n_atoms": system.n_atoms, "precision": precision,
            "steps": n_steps, "sample_every": sample_every, "tau_fs": tau_fs, "value": value,
            "ms_per_step": elapsed * 1e3 / n_steps, "msd_call_us": msd_call_us, "autotuned": ch,
            "by_temperature_after_run": by_t}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="bcc1m")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--piston-steps", type=int, default=100, help="steps of the 2.88 M-atom piston slab (0 = skip)")
    ap.add_argument("--batched", default="fec256,liquid4096",
                    help="comma-separated batched workloads to run together and one by one ('' = none)")
    ap.add_argument("--batched-steps", type=int, default=100)
    ap.add_argument("--half-steps", type=int, default=100, help="steps of the half-list + atomics comparison")
    ap.add_argument("--nvt-steps", type=int, default=100,
                    help="steps of the batched Nose-Hoover run beside its NVE twin (0 = skip)")
    ap.add_argument("--repeats", type=int, default=5,
                    help="further timed runs of the main workload for a median (reported beside value)")
    ap.add_argument("--pr-steps", type=int, default=200,
                    help="steps of the main crystal under the barostat beside a fixed box (0 = skip)")
    ap.add_argument("--large-steps", type=int, default=200,
                    help="steps of the 4.15 M-atom crystal (beyond the last-level cache; 0 = skip)")
    ap.add_argument("--gear-steps", type=int, default=100,
                    help="steps of the Gear predictor-corrector on the main workload (0 = skip)")
    ap.add_argument("--evaluator-steps", type=int, default=100,
                    help="steps of the table versus explicit evaluation comparison (0 = skip)")
    ap.add_argument("--diffusion-steps", type=int, default=1000,
                    help="steps of the vacancy self-diffusion workload with MSD sampling (0 = skip)")
    ap.add_argument("--energy-steps", type=int, default=200,
                    help="steps of the leg that reduces energies and the virial every step (0 = skip)")
    ap.add_argument("--auto-steps", type=int, default=100,
                    help="steps of each automatic-rebuild run (batched workloads and the headline; 0 = skip)")
    ap.add_argument("--auto-skins", default="0.3,0.4,0.5",
                    help="skins of the automatic-rebuild runs of the batched workloads")
    ap.add_argument("--small-steps", type=int, default=100,
                    help="steps of the 2000-atom FP64 configuration (0 = skip)")
    ap.add_argument("--copy-gbs-mib", type=int, default=1024,
                    help="size of the device copy whose bandwidth is reported beside the roofline (0 = skip)")
    ap.add_argument("--nchunk", type=int, choices=[2, 4, 8], default=4,
                    help="with --kernel global: neighbour records in flight per thread")
    ap.add_argument("--nchunk-mixed", type=int, choices=[2, 4, 8], default=0,
                    help="with --kernel global: the same for the mixed leg (0: as --nchunk)")
    ap.add_argument("--fp64-evaluator", type=int, choices=[0, 1], default=0,
                    help="with --kernel global or brick: the FP64 leg's evaluator (0 tables, 1 knot sums)")
    ap.add_argument("--kernel", choices=["auto", "global", "brick"], default="auto",
                    help="main workload: autotuned configuration, or the global-gather or LDS-brick kernels with tables")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run plain device-to-device copies of this size (for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    from paper_1107_2619_amd import inputs

    # batched workloads first, while no GPU context exists (the liquid
    # generator may use a process pool)
    batched_sys = {}
    for w in [w for w in args.batched.split(",") if w]:
        t = time.perf_counter()
        kw = {"workers": min(16, os.cpu_count() or 1)} if w == "liquid4096" else {}
        batched_sys[w] = inputs.workload(w, **kw)
        log(f"built {w} in {time.perf_counter() - t:.1f} s")
    piston = inputs.workload("fcc_piston") if args.piston_steps > 0 else None
    vacancy = inputs.workload("vacancy192") if args.diffusion_steps > 0 else None

    import torch

    from paper_1107_2619_amd import md

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.copy_calibration_mib > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counter readings
        # calibrate the counters of the force kernel
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {nbytes} bytes")
        del src, dst
    # a plain device-to-device copy: the HBM bandwidth this GPU reaches
    copy_gbs = None
    if args.copy_gbs_mib > 0:
        nbytes = args.copy_gbs_mib << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        copy_gbs = 5 * 2 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9
        log(f"device copy: {copy_gbs:.0f} GB/s (read + write)")
        del src, dst
    log(f"building workload {args.workload}")
    system = inputs.workload(args.workload)
    n = system.n_atoms

    results = {}
    tuned = {}
    for prec in ("fp64", "mixed"):
        if args.kernel in ("global", "brick"):  # fixed configuration (counter passes compare the same kernels)
            ch = {"kernel": 1 if args.kernel == "global" else 0, "brick_dims": 444, "lanes": 1, "block": 1024,
                  "evaluator": args.fp64_evaluator if prec == "fp64" else 0,
                  "nchunk": args.nchunk if prec == "fp64" else (args.nchunk_mixed or args.nchunk), "step_us": None}
            opts = choice_options(md, ch)
            log(f"{prec}: {args.kernel} kernels, {'knot sums' if ch['evaluator'] else 'tables'} (no autotune)")
        else:
            opts, ch = tune_options(md, system, prec)
        tuned[prec] = ch
        log(f"{prec}: warmup 2 x {args.warmup}, timed {args.steps} steps")
        sim, ms, wall, en, _ = run_precision(md, system, prec, args.steps, args.warmup, timing=False, tune=opts)
        log(f"{prec}: {ms / args.steps * 1e3:.1f} us/step  (wall {wall:.3f} s)")
        repeats = [timed_steps(sim, args.steps)[0] for _ in range(args.repeats)]
        # a second timed pass with per-kernel HIP events for the roofline
        sim_t, ms_t, _, _, kt = run_precision(md, system, prec, args.steps, args.warmup, timing=True, tune=opts)
        results[prec] = {"sim": sim, "ms": ms, "ms_timed": ms_t, "en": en, "kt": kt, "warmup_run": sim.warmup_steps,
                         "repeats": repeats}
        del sim_t

    rec_ms = {prec: results[prec]["ms"] / args.steps for prec in ("fp64", "mixed")}

    # the Parrinello-Rahman barostat on the same crystal (zero pressure, box
    # period ~1 ps), beside the same run with a fixed box; both with a 0.5 A skin,
    # which leaves the barostat's displacement and strain guards room at 600 K
    barostat = None
    if args.pr_steps > 0:
        opts_pr = choice_options(md, tuned["mixed"])
        opts_pr[md.MD_OPT_KERNEL] = 1
        rates = {}
        # the same crystal in the cell [a, b, c + a] (the cube's periodic
        # system with non-orthogonal edges): held fixed, and under the
        # full-matrix barostat with a 0.2 GPa xy shear stress
        h_skew = np.diag(system.box[0]) @ np.array([[1.0, 0.0, 1.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
        shear = np.zeros((3, 3))
        shear[0, 1] = shear[1, 0] = 0.2
        legs = (("fixed_box", {}), ("barostat", {"pr_pressure_gpa": [0.0], "pr_mass": [2.0e7]}),
                ("sheared_cell_fixed", {"box_matrix": h_skew}),
                ("barostat_box_matrix", {"box_matrix": h_skew, "pr_pressure_gpa": [0.0], "pr_mass": [2.0e7],
                                         "pr_stress_gpa": shear}))
        for label, kw in legs:
            sim_b = md.Simulation(system, precision="mixed", want_e_atom=False, skin=0.5, **kw)
            for opt, val in opts_pr.items():
                sim_b.set_option(opt, val)
            sim_b.set_option(md.MD_OPT_USE_GRAPH, 1)
            for _ in range(2):
                sim_b.step(max(args.warmup, 4 * system.rebuild_every + 2))
                sim_b.energy()
            ms_b, _ = timed_steps(sim_b, args.pr_steps)
            e_b = sim_b.energy()
            rates[label] = {"value": n * args.pr_steps / (ms_b * 1e-3), "ms_per_step": ms_b / args.pr_steps,
                            "box_A": [float(x) for x in e_b.box[0]], "pressure_gpa": float(e_b.pressure_gpa[0])}
            if "box_matrix" in kw:
                rates[label]["h_A"] = e_b.h[0].tolist()
            del sim_b
        fixed_ms = rates["fixed_box"]["ms_per_step"]
        barostat = {"workload": f"{args.workload} with a 0.5 A skin", "precision": "mixed", "steps": args.pr_steps,
                    "pressure_gpa": 0.0, "box_mass_eV_fs2_per_A2": 2.0e7, "shear_stress_xy_gpa": 0.2, **rates,
                    "overhead": rates["barostat"]["ms_per_step"] / fixed_ms - 1.0,
                    "overhead_sheared_cell": rates["sheared_cell_fixed"]["ms_per_step"] / fixed_ms - 1.0,
                    "overhead_box_matrix": rates["barostat_box_matrix"]["ms_per_step"] / fixed_ms - 1.0}
        log(f"barostat: {rates['barostat']['value']:.3e} atom-steps/s, fixed box {rates['fixed_box']['value']:.3e} "
            f"({barostat['overhead']:+.1%}); sheared cell {rates['sheared_cell_fixed']['value']:.3e} "
            f"({barostat['overhead_sheared_cell']:+.1%}), full-matrix barostat "
            f"{rates['barostat_box_matrix']['value']:.3e} ({barostat['overhead_box_matrix']:+.1%})")

    # the same crystal four times larger, beyond the 256 MB last-level cache
    size_sweep = []
    if args.large_steps > 0:
        big = inputs.workload("bcc4m")
        for prec in ("fp64", "mixed"):
            opts_b, ch_b = tune_options(md, big, prec)
            sim_b, ms_b, _, _, _ = run_precision(md, big, prec, args.large_steps, args.warmup, timing=False,
                                                 tune=opts_b)
            size_sweep.append({"workload": "bcc4m: bcc Fe 128^3 cells, 1% vacancies, 600 K, rebuild every 10",
                               "n_atoms": big.n_atoms, "precision": prec, "steps": args.large_steps,
                               "value": big.n_atoms * args.large_steps / (ms_b * 1e-3),
                               "ms_per_step": ms_b / args.large_steps, "autotuned": ch_b})
            log(f"bcc4m {prec}: {ms_b / args.large_steps * 1e3:.1f} us/step")
            del sim_b
        del big

    # the half-list + FP64-atomics variant on the same workload (comparison)
    half = {}
    if args.half_steps > 0:
        for prec in ("fp64", "mixed"):
            sim_h, ms_h, _, _, _ = run_precision(md, system, prec, args.half_steps, args.warmup, timing=False,
                                                 nbr_mode="half", tune={md.MD_OPT_KERNEL: 1})
            half[prec] = {"value": n * args.half_steps / (ms_h * 1e-3), "ms_per_step": ms_h / args.half_steps}
            log(f"half list {prec}: {ms_h / args.half_steps * 1e3:.1f} us/step")
            del sim_h

    # the paper's lookup-table versus explicit-evaluation comparison ("Parallel
    # benchmarks"): the exact local-polynomial tables against the term-by-term
    # knot sums, each precision with its autotuned kernel settings
    evaluator = {}
    if args.evaluator_steps > 0:
        for prec in ("fp64",):  # the term-by-term knot sums are FP64 only
            opts = choice_options(md, tuned[prec])
            rates = {}
            for ev, label in ((0, "table"), (1, "explicit")):
                sim_e, ms_e, _, _, _ = run_precision(md, system, prec, args.evaluator_steps, args.warmup,
                                                     timing=False, tune={**opts, md.MD_OPT_EVALUATOR: ev})
                rates[label] = n * args.evaluator_steps / (ms_e * 1e-3)
                del sim_e
            rates["table_speedup"] = rates["table"] / rates["explicit"]
            evaluator[prec] = rates
            log(f"evaluator {prec}: table {rates['table']:.3e}, explicit {rates['explicit']:.3e} atom-steps/s")

    # the same comparison with the paper's own benchmark potential, an iron
    # potential of 15 cubic splines (13 pair + 2 density knots): at the paper's
    # size for it (31,250 atoms) and on this workload's crystal; the kernel
    # options are those tuned above
    evaluator_fe15 = {}
    if args.evaluator_steps > 0:
        w15 = {"bcc31250_fe15": inputs.workload("bcc31250_fe15")}
        if args.workload in ("bcc1m", "bcc4m"):
            s15 = copy.copy(system)
            s15.potential = inputs.perturbed_potential("fe15_fs", 3)
            # sigma of a 10 fs displacement at 600 K: 0.032 A per axis with this
            # potential; a 0.5 A skin keeps the guard at 7.9 sigma
            s15.skin = 0.5
            s15.max_neighbours = 64  # the 4.76 A shell reaches into 4.6 A when hot
            w15[args.workload + "_fe15"] = s15
        for wname, s15 in w15.items():
            per = {"n_atoms": s15.n_atoms, "skin": s15.skin}
            for prec in ("fp64",):
                opts = choice_options(md, tuned[prec])
                rates = {}
                for ev, label in ((0, "table"), (1, "explicit")):
                    sim_e, ms_e, _, _, _ = run_precision(md, s15, prec, args.evaluator_steps, args.warmup,
                                                         timing=False, tune={**opts, md.MD_OPT_EVALUATOR: ev})
                    rates[label] = s15.n_atoms * args.evaluator_steps / (ms_e * 1e-3)
                    del sim_e
                rates["table_speedup"] = rates["table"] / rates["explicit"]
                per[prec] = rates
                log(f"evaluator {wname} {prec}: table {rates['table']:.3e}, explicit {rates['explicit']:.3e}")
            evaluator_fe15[wname] = per

    # the third-order Gear predictor-corrector on the same workload ("Time
    # integration"), each precision with its autotuned kernel settings
    gear = {}
    if args.gear_steps > 0:
        for prec in ("fp64", "mixed"):
            sim_g, ms_g, _, _, _ = run_precision(md, system, prec, args.gear_steps, args.warmup, timing=False,
                                                 tune=choice_options(md, tuned[prec]), integrator="gear3")
            gear[prec] = {"value": n * args.gear_steps / (ms_g * 1e-3), "ms_per_step": ms_g / args.gear_steps,
                          "vs_verlet": (ms_g / args.gear_steps) / rec_ms[prec]}
            log(f"gear {prec}: {ms_g / args.gear_steps * 1e3:.1f} us/step")
            del sim_g

    batched = [batched_vs_one_by_one(md, system_b, w, args.batched_steps, args.warmup)
               for w, system_b in batched_sys.items()]
    nvt_rec = None
    if "fec256" in batched_sys and args.nvt_steps > 0:
        ch_fec = next(b["autotuned"] for b in batched if b["workload"] == "fec256")
        nvt_rec = nvt_vs_nve(md, batched_sys["fec256"], "fec256", args.nvt_steps, args.warmup, ch_fec)
    if "liquid4096" in batched_sys:  # cfg5 also compares FP64 with mixed
        batched.append(batched_vs_one_by_one(md, batched_sys["liquid4096"], "liquid4096", args.batched_steps,
                                             args.warmup, precision="fp64"))

    # automatic rebuilds on the batched workloads at smaller skins than their
    # fixed periods need, and on the headline workload at its own skin (FP64)
    auto_rec = []
    if args.auto_steps > 0:
        skins = [float(x) for x in args.auto_skins.split(",") if x]
        for w, system_b in batched_sys.items():
            fixed = next((b["batched"] for b in batched if b["workload"] == w and b["precision"] == "mixed"), None)
            auto_rec.append(auto_rebuild_leg(md, system_b, w, args.auto_steps, args.warmup, skins, "mixed", fixed))
        auto_rec.append(auto_rebuild_leg(md, system, args.workload, args.auto_steps, args.warmup, [system.skin],
                                         "fp64", n * args.steps / (results["fp64"]["ms"] * 1e-3)))

    diffusion = None
    if vacancy is not None:
        diffusion = diffusion_leg(md, vacancy, "vacancy192", args.diffusion_steps, args.warmup, 100)

    # the free-surface piston slab (2.88 M atoms, mixed)
    piston_rec = None
    if piston is not None:
        opts_p, ch_p = tune_options(md, piston, "mixed")
        sim_p, ms_p, _, en_p, _ = run_precision(md, piston, "mixed", args.piston_steps, args.warmup, timing=False,
                                                tune=opts_p)
        piston_rec = {"workload": "fcc_piston: fcc Cu-like 60x60x200 cells, free z, rigid piston at 1 km/s, "
                                  f"dt {piston.dt_fs} fs", "n_atoms": piston.n_atoms, "precision": "mixed",
                      "steps": args.piston_steps, "value": piston.n_atoms * args.piston_steps / (ms_p * 1e-3),
                      "ms_per_step": ms_p / args.piston_steps, "autotuned": ch_p,
                      "piston_work_eV": float(en_p.piston_work[0])}
        log(f"piston: {ms_p / args.piston_steps * 1e3:.1f} us/step")
        del sim_p

    # mixed-vs-FP64 force error on one shared state (the FP64 run's final state)
    ref_sim = results["fp64"]["sim"]
    pos, vel = ref_sim.positions(), ref_sim.velocities()
    ref_sim.eam_forces(want_energy=True)
    f64 = ref_sim.forces()
    mix_sim = results["mixed"]["sim"]
    mix_sim.set_state(pos, vel)
    mix_sim.build_neighbours()
    mix_sim.eam_forces(want_energy=True)
    fmix = mix_sim.forces()
    mix_err = float(np.max(np.linalg.norm(fmix - f64, axis=1)) / np.sqrt(np.mean(np.sum(f64**2, 1))))
    log(f"mixed vs fp64 force error {mix_err:.3e}")

    # neighbour statistics for the byte model
    counts, _ = ref_sim.neighbours()
    nbar = float(counts.mean())

    rec = {}
    for prec in ("fp64", "mixed"):
        r = results[prec]
        ms_step = r["ms"] / args.steps
        kt = r["kt"]
        f_ms, f_n = kt["force"]
        d_ms, d_n = kt["density"]
        b_ms, b_n = kt["build"]
        rec[prec] = {
            "value": n * args.steps / (r["ms"] * 1e-3),
            "ms_per_step": ms_step,
            "force_kernel_us": 1e3 * f_ms / f_n,
            "density_kernel_us": 1e3 * d_ms / d_n,
            "build_us_per_rebuild": 1e3 * b_ms / max(b_n, 1),
            "timing_overhead_frac": r["ms_timed"] / r["ms"] - 1.0,
            "temperature_K": float(r["en"].temperature[0]),
            "autotuned": tuned[prec],
            "graph_replay": True,
            "warmup_steps_run": r["warmup_run"],
            "repeat_ms_per_step": [x / args.steps for x in r["repeats"]],
            "median_value": (n * args.steps / (float(np.median(r["repeats"])) * 1e-3)) if r["repeats"] else None,
        }
        rec[prec]["roofline"] = roofline_for(rec[prec], prec, nbar, n, system.rebuild_every, args.workload,
                                             copy_gbs)
    gate_ok = mix_err <= 1e-5
    rec["mixed"]["gate"] = {"force_err_vs_fp64": mix_err, "bound": 1e-5, "ok": gate_ok}
    rec["mixed"]["speedup_vs_fp64"] = rec["mixed"]["value"] / rec["fp64"]["value"]
    head = rec["fp64"]
    roofline = head["roofline"]

    # energies, virial and pressure reduced on every step (device ring), the
    # same workload and kernel settings as the headline, both precisions
    every_step = {}
    if args.energy_steps > 0:
        for prec in ("fp64", "mixed"):
            sim_e, ms_e, _, _, _ = run_precision(md, system, prec, args.energy_steps, args.warmup, timing=False,
                                                 tune=choice_options(md, tuned[prec]), energy_every=1,
                                                 energy_ring=args.energy_steps + 1024)
            hist = sim_e.energy_history(max_entries=args.energy_steps + 1024)
            every_step[prec] = {
                "value": n * args.energy_steps / (ms_e * 1e-3), "ms_per_step": ms_e / args.energy_steps,
                "vs_energy_at_call_end": (ms_e / args.energy_steps) / rec[prec]["ms_per_step"],
                "entries_read": len(hist),
                "pe_last_eV_per_atom": float(hist[-1].pe[0] / n) if hist else None,
                "pressure_last_gpa": float(hist[-1].pressure_gpa[0]) if hist else None,
            }
            log(f"energies every step {prec}: {ms_e / args.energy_steps * 1e3:.1f} us/step")
            del sim_e

    # the small configuration: 2000-atom bcc Fe, FP64, 100 velocity-Verlet steps
    small_rec = None
    if args.small_steps > 0:
        small = inputs.workload("bcc2000")
        opts_s, ch_s = tune_options(md, small, "fp64")
        sim_s, ms_s, _, en_s, _ = run_precision(md, small, "fp64", args.small_steps, args.warmup, timing=False,
                                                tune=opts_s)
        small_rec = {"workload": "bcc2000: bcc Fe 10^3 cells, 300 K, dt 1 fs, rebuild every 10",
                     "n_atoms": small.n_atoms, "precision": "fp64", "steps": args.small_steps,
                     "value": small.n_atoms * args.small_steps / (ms_s * 1e-3),
                     "ms_per_step": ms_s / args.small_steps, "autotuned": ch_s}
        log(f"bcc2000 fp64: {ms_s / args.small_steps * 1e3:.1f} us/step")
        del sim_s

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(system, ref_sim, pos, f64, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: bcc Fe 80^3 cells, 1% vacancies, N={n}, 600 K, "
                         if args.workload == "bcc1m" else
                         f"{args.workload}: {system.n_replicas} replica(s), N={n}, ")
                        + f"rebuild every {system.rebuild_every}, dt {system.dt_fs} fs",
            "n_atoms": n,
            "mean_neighbours": nbar,
            "precision": "fp64",
            "parallelism": "single GPU",
        },
        "mixed_force_err_vs_fp64": mix_err,
        "fp64": rec["fp64"],
        "mixed": rec["mixed"],
        "energy_every_step": every_step,
        "small_config": small_rec,
        "paper_context": PAPER_CONTEXT,
        "larger_system": size_sweep,
        "barostat": barostat,
        "half_list_atomics": half,
        "table_vs_explicit": evaluator,
        "table_vs_explicit_fe15": evaluator_fe15,
        "gear_predictor_corrector": gear,
        "batched_vs_one_by_one": batched,
        "auto_rebuild": auto_rec,
        "nvt_batched": nvt_rec,
        "diffusion": diffusion,
        "piston_slab": piston_rec,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def cpu_baseline(system, sim, pos, f_gpu, seconds):
    """The FP64 oracle as it stands, on a bounded sample of atoms of the same
    state: brute-force forces of S sampled atoms over all N atoms (each needs
    the densities of its neighbours, also by brute force).  Also a full-size
    parity check of the GPU FP64 forces at those atoms."""
    import oracle

    pot = oracle.Potential(system.potential)
    rng = np.random.default_rng(77)
    probe = rng.choice(system.n_atoms, 16, replace=False)
    t = time.perf_counter()
    oracle.forces_sampled(pos, system.species, system.box[0], system.periodic[0], pot, probe)
    per_atom = (time.perf_counter() - t) / len(probe)
    s = int(max(16, min(4096, seconds / max(per_atom, 1e-6))))
    sample = rng.choice(system.n_atoms, s, replace=False)
    log(f"cpu baseline: {s} sampled atoms (~{per_atom * s:.1f} s)")
    t = time.perf_counter()
    ref = oracle.forces_sampled(pos, system.species, system.box[0], system.periodic[0], pot, sample)
    dt = time.perf_counter() - t
    fr = f_gpu[sample]
    err = float(np.max(np.linalg.norm(fr - ref.f, axis=1)) / np.sqrt(np.mean(np.sum(ref.f**2, 1))))
    # the whole 2000-atom crystal for 100 velocity-Verlet steps, as the oracle runs it
    from paper_1107_2619_amd import inputs

    small = inputs.workload("bcc2000")
    t = time.perf_counter()
    oracle.run_verlet(small.pos, small.vel, small.species, small.box[0], small.periodic[0],
                      oracle.Potential(small.potential), small.dt_fs, 100)
    small_rate = small.n_atoms * 100 / (time.perf_counter() - t)
    log(f"cpu baseline: bcc2000 x 100 steps at {small_rate:.3e} atom-steps/s")
    # the same crystal on one thread (30 steps), and a 16,000-atom crystal (20^3 cells) for 3 steps
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    t = time.perf_counter()
    oracle.run_verlet(small.pos, small.vel, small.species, small.box[0], small.periodic[0],
                      oracle.Potential(small.potential), small.dt_fs, 30)
    one_rate = small.n_atoms * 30 / (time.perf_counter() - t)
    oracle.set_num_threads(threads)
    big = inputs.bcc_fe(20, a=2.87, temperature=600.0, seed=2)
    t = time.perf_counter()
    oracle.run_verlet(big.pos, big.vel, big.species, big.box[0], big.periodic[0], oracle.Potential(big.potential),
                      big.dt_fs, 3)
    big_rate = big.n_atoms * 3 / (time.perf_counter() - t)
    log(f"cpu baseline: bcc2000 on one thread {one_rate:.3e}, bcc16000 x 3 steps {big_rate:.3e} atom-steps/s")
    return {
        "value": s / dt,
        "unit": "atom-steps/s",
        "cores": oracle.num_threads(),
        "cpu_model": cpu_model(),
        "logical_cpus": os.cpu_count(),
        "kind": "oracle",
        "sample": f"forces of {s} random atoms of the same {system.n_atoms}-atom state, brute force O(N) each "
                  f"(O(N^2) algorithm), FP64, OpenMP; {dt:.1f} s",
        "gpu_fp64_force_err_on_sample": err,
        "bcc2000_100_steps": {"value": small_rate, "unit": "atom-steps/s",
                              "note": "2000-atom bcc Fe, 100 velocity-Verlet steps, whole run, O(N^2) per step"},
        "bcc2000_30_steps_one_thread": {"value": one_rate, "unit": "atom-steps/s", "cores": 1},
        "bcc16000_3_steps": {"value": big_rate, "unit": "atom-steps/s",
                             "note": "16,000-atom bcc Fe (20^3 cells), 3 velocity-Verlet steps, O(N^2) per step"},
    }


if __name__ == "__main__":
    main()
