"""Benchmark of the aspherical PIC particle loop on one MI355X.

A step is one full PIC step of the library (particle push with gather, boundary
tests and deposit for both species; Maxwellian injection; periodic cell sort;
charge density, FP64 multigrid Poisson solve and nodal gradient; grain force).
`value` is particle-steps per second over the timed steps (resident particles of
both species pushed per step, summed, divided by the wall time between two
device synchronisations), inputs resident in HBM before timing starts.

Headline workload: c4, the batched ensemble of 64 grains in one context (the
FP32 batched form, autotuned launch schedule, graph-captured steps).  Beside it
the line carries the plain FP64 path on the same ensemble (`fp64`,
`speedup_fp32_vs_fp64`), the single-grain workloads c3 (FP32 and FP64) and c5,
the Boltzmann-electron and conservative field-solve modes on c3, and the
oracle's rate on a bounded sample of the headline workload (`cpu_baseline`).

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
[--no-fp64] [--no-cpu-baseline] [--no-c3] [--no-c5] [--no-boltzmann]
[--no-conservative]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_PER_PARTICLE = {"fp32": 48, "fp64": 80}   # read + write of the particle state
TRAFFIC_FILES = {"c4": os.path.join(ROOT, "profiles", "k_push_split_c4_traffic.md"),
                 "c3": os.path.join(ROOT, "profiles", "k_push_split_c3_traffic.md")}
KERNEL_SOURCE = os.path.join(ROOT, "paper_2307_11107_amd", "csrc", "particles.hip")
COPY_BYTES = 1 << 30           # calibration copy: 1 GiB read + 1 GiB written


def copy_calibration():
    """A plain device copy of known size, outside the timed region: its first
    run lets a hardware-counter run of this script scale its byte counters;
    five more, timed with events, give the read-plus-write rate this GPU
    sustains for a plain stream (GB/s of bytes read and written)."""
    import torch
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(5):
        y.copy_(x)
    b.record()
    b.synchronize()
    gbs = 5 * 2 * COPY_BYTES / (a.elapsed_time(b) * 1e-3) / 1e9
    del x, y
    return gbs


def measured_traffic(particles_per_launch, workload):
    """HBM bytes per push launch from the committed counter summary, if it was
    taken on the current kernel source and this workload (else None)."""
    if workload not in TRAFFIC_FILES:
        return None
    import hashlib
    try:
        text = open(TRAFFIC_FILES[workload]).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    digest = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if vals.get("kernel_source_sha256") != digest or "hbm_bytes_per_particle_step" not in vals:
        return None
    return float(vals["hbm_bytes_per_particle_step"]) * particles_per_launch


def grain_cfgs(grains, boltzmann=False):
    import paper_2307_11107_amd as apic
    cfgs = []
    for w in grains:
        ions = apic.species(1.0, w["mi"], w["Ti"], 1.0, 0.0, 0.0, w["n_macro"])
        sp = [ions] if boltzmann else [apic.species(-1.0, 1.0, 1.0, 1.0, 0.0, 0.0, w["n_macro"]), ions]
        cfgs.append(apic.grain_cfg(w["alpha"], w["n1"], w["n2"], sp, x1_out=w["x1_out"], wce=w["wce"],
                                   kappa=w["kappa"], phi_grain=-2.5, phi_out=0.0, dt=w["dt"], seed=w["seed"]))
    return cfgs


TUNING_STEPS_MAX = 96


def run_gpu(grains, precision, steps, warmup, stream, autotune=False, boltzmann=False, conservative=False):
    """Loads every grain; with the autotuner, steps until the schedule is
    chosen (untimed, whatever `warmup` is, so that no timed step runs a tuning
    candidate); then runs `warmup` steps and times `steps` steps between device
    synchronisations."""
    import torch
    import paper_2307_11107_amd as apic
    prec = apic.APIC_FP32_SPLIT if precision == "fp32" else apic.APIC_FP64
    ns = 1 if boltzmann else 2
    ctx = apic.apic_init(grain_cfgs(grains, boltzmann), apic.opts(precision=prec, inject=True, stream=stream,
                                                                  autotune=autotune, boltzmann_electrons=boltzmann,
                                                                  conservative_poisson=conservative))
    try:
        for g in range(len(grains)):
            for s in range(ns):
                apic.apic_inject(ctx, g, s)
        tuning_steps = 0
        while autotune and not apic.apic_schedule(ctx)["tuned"] and tuning_steps < TUNING_STEPS_MAX:
            apic.apic_step(ctx, 1)
            tuning_steps += 1
        apic.apic_step(ctx, warmup)
        torch.cuda.synchronize()
        t0 = [apic.apic_tallies(ctx, g, ns, w["n2"]) for g, w in enumerate(grains)]
        apic.apic_set_profiling(ctx, True)
        torch.cuda.synchronize()
        start = time.perf_counter()
        apic.apic_step(ctx, steps)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - start
        tm = apic.apic_timing(ctx)
        t1 = [apic.apic_tallies(ctx, g, ns, w["n2"]) for g, w in enumerate(grains)]
        sched = apic.apic_schedule(ctx)
    finally:
        apic.apic_free(ctx)
    pushed = int(sum(sum(b["particle_steps"]) - sum(a["particle_steps"]) for a, b in zip(t0, t1)))
    balance = all(int(t["injected"][s]) == int(t["absorbed"][s] + t["escaped"][s] + t["resident"][s])
                  for t in t1 for s in range(ns))
    return {"elapsed": elapsed, "particle_steps": pushed, "timing": tm, "balance_exact": balance,
            "schedule": sched, "tuning_steps": tuning_steps}


def _cpu_grain(args):
    w, n_sample, steps = args
    os.environ["OMP_NUM_THREADS"] = "1"
    return cpu_baseline(w, n_sample, steps)


def cpu_baseline_grains(grains, n_sample, steps, procs):
    """The oracle on several grains of the ensemble at once, one process per
    grain (the grains are independent simulations), all timing their steps
    concurrently: the sum of the processes' particle-step rates."""
    import multiprocessing as mp
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(procs) as pool:
        res = pool.map(_cpu_grain, [(g, n_sample, steps) for g in grains])
    wall = time.perf_counter() - t0
    return sum(rate for rate, _ in res), wall, sum(secs for _, secs in res)


def cpu_baseline(w, n_sample, steps):
    """The FP64 oracle on a bounded sample of the workload (same geometry, field
    solve and step; fewer macro-particles)."""
    from oracle.pic import Config, Simulation, Species
    cfg = Config(alpha=w["alpha"], n1=w["n1"], n2=w["n2"], x1_out=w["x1_out"], wce=w["wce"],
                 kappa=w["kappa"], dt=w["dt"], seed=w["seed"],
                 species=[Species(q=-1.0, m=1.0, n_macro=n_sample),
                          Species(q=1.0, m=w["mi"], T=w["Ti"], n_macro=n_sample)])
    sim = Simulation(cfg)
    sim.load(0)
    sim.load(1)
    sim.initialize_field()
    t0 = time.perf_counter()
    pushed = 0
    for _ in range(steps):
        pushed += sim.resident(0) + sim.resident(1)
        sim.step()
    dt = time.perf_counter() - t0
    return pushed / dt, dt


def push_summary(r, precision):
    """Average push launch time and algorithmic GB/s of a run."""
    tm = r["timing"]
    avg_ms = tm["push_ms"] / max(tm["push_launches"], 1)
    per_launch = r["particle_steps"] / max(tm["push_launches"], 1)
    gbs = BYTES_PER_PARTICLE[precision] * per_launch / (avg_ms * 1e-3) / 1e9
    return avg_ms, per_launch, gbs


def breakdown(r):
    tm = r["timing"]
    return {k: tm[k] / max(tm["steps"], 1) for k in ("push_ms", "inject_ms", "sort_ms", "field_ms")}


def secondary(r, precision, steps, workload, unit="particle-steps/s"):
    avg, _, gbs = push_summary(r, precision)
    tm = r["timing"]
    return {"workload": workload, "value": r["particle_steps"] / r["elapsed"], "unit": unit,
            "ms_per_step": 1e3 * r["elapsed"] / steps, "push_avg_launch_ms": avg, "push_GBps": gbs,
            "push_frac_of_hbm_peak": gbs / HBM_PEAK_GBS, "breakdown_ms_per_step": breakdown(r),
            "mg_cycles_per_step": tm["mg_cycles"] / max(tm["steps"], 1), "balance_exact": r["balance_exact"]}


def describe(name, w):
    return (f"{name}: alpha={w['alpha']}, wce/wpe={w['wce']}, grid {w['n1']}x{w['n2']}, x1_out={w['x1_out']}, "
            f"lambdaD/R0={w['kappa']}, mi/me={w['mi']}, Ti/Te={w['Ti']}, {w['n_macro']:.0e} macro-particles per "
            f"species, Maxwellian flux injection, dt={w['dt']}/wpe")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000)
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--cpu-procs", type=int, default=16)
    ap.add_argument("--no-c3", action="store_true")
    ap.add_argument("--c3-steps", type=int, default=50)
    ap.add_argument("--c3-warmup", type=int, default=10)
    ap.add_argument("--no-c5", action="store_true")
    ap.add_argument("--no-boltzmann", action="store_true")
    ap.add_argument("--no-conservative", action="store_true")
    ap.add_argument("--c5-steps", type=int, default=20)
    ap.add_argument("--c5-warmup", type=int, default=6)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the particle loop of this build runs on a single MI355X "
              "(multi-GPU sharding is a design note only); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from synthetic_inputs import WORKLOADS, ensemble_c4
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    copy_gbs = copy_calibration()

    # headline: the c4 ensemble, FP32 split, autotuned (the tuner's steps are
    # part of the warm-up)
    ens = ensemble_c4()
    n_ens = sum(g["n_macro"] for g in ens)
    r32 = run_gpu(ens, "fp32", args.steps, args.warmup, stream, autotune=True)
    value = r32["particle_steps"] / r32["elapsed"]
    push_avg_ms, per_launch, achieved = push_summary(r32, "fp32")
    tm = r32["timing"]
    out = {
        "metric": "particle-steps/s (push+gather+deposit) on 1 MI355X, FP32 vs FP64; % HBM peak",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r32["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"c4: batched ensemble of {len(ens)} grains in one context (alpha U[0,0.2], "
                               f"wce/wpe in {{0,0.5,1}}, lambdaD/R0 U[0.5,5], grids 128x128..512x256, x1_out=-0.1, "
                               f"mi/me=1836, Te=Ti, {n_ens:.3g} macro-particles per species in total, log-uniform "
                               f"1e6-2e7 per grain, Maxwellian flux injection, dt=0.05/wpe); FP32 split "
                               f"push/gather/deposit in one persistent launch, autotuned schedule, graph-captured "
                               f"steps, FP64 multigrid Poisson and tallies",
                   "grains": len(ens), "particles_per_species_total": n_ens},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(per_launch, "c4"),
                     "kernel": "k_push_split (FP32 split push+gather+deposit, all grains and species in one launch)",
                     "avg_launch_ms": push_avg_ms, "algorithmic_bytes_per_particle": BYTES_PER_PARTICLE["fp32"],
                     "particles_per_launch": per_launch,
                     # a plain 1 GiB device copy on the same GPU, read plus written bytes per second
                     "copy_GBps": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "breakdown_ms_per_step": breakdown(r32),
        "mg_cycles_per_step": tm["mg_cycles"] / max(tm["steps"], 1),
        "schedule": r32["schedule"],
        # untimed steps the autotuner took to choose the schedule, before the warmup
        "tuning_steps": r32["tuning_steps"],
        "balance_exact": r32["balance_exact"],
    }
    if not args.no_fp64:
        r64 = run_gpu(ens, "fp64", args.steps, args.warmup, stream, autotune=True)
        avg64, _, gb64 = push_summary(r64, "fp64")
        v64 = r64["particle_steps"] / r64["elapsed"]
        out["fp64"] = {"value": v64, "ms_per_step": 1e3 * r64["elapsed"] / args.steps, "push_avg_launch_ms": avg64,
                       "push_GBps": gb64, "breakdown_ms_per_step": breakdown(r64),
                       "balance_exact": r64["balance_exact"]}
        out["speedup_fp32_vs_fp64"] = value / v64
    if not args.no_c3:
        w = WORKLOADS["c3"]
        r3 = run_gpu([w], "fp32", args.c3_steps, args.c3_warmup, stream)
        out["c3"] = secondary(r3, "fp32", args.c3_steps, describe("c3", w) + "; FP32 split")
        out["c3"]["push_traffic"] = measured_traffic(push_summary(r3, "fp32")[1], "c3")
        if not args.no_fp64:
            r3d = run_gpu([w], "fp64", args.c3_steps, args.c3_warmup, stream)
            out["c3"]["fp64"] = secondary(r3d, "fp64", args.c3_steps, describe("c3", w) + "; FP64 plain")
            out["c3"]["speedup_fp32_vs_fp64"] = out["c3"]["value"] / out["c3"]["fp64"]["value"]
    if not args.no_c5:
        # the largest single grain (2048 x 1024 cells, 2e8 macro-particles per
        # species): the push at four times the c3 state
        w5 = WORKLOADS["c5"]
        r5 = run_gpu([w5], "fp32", args.c5_steps, args.c5_warmup, stream)
        out["c5"] = secondary(r5, "fp32", args.c5_steps, describe("c5", w5) + "; FP32 split, FP64 multigrid")
    w = WORKLOADS["c3"]
    if not args.no_boltzmann:
        # the c3 grain and ions with Boltzmann electrons (not moved; the field
        # solve is the Newton-multigrid one)
        rb = run_gpu([w], "fp32", args.c3_steps, args.c3_warmup, stream, boltzmann=True)
        out["boltzmann_electrons"] = secondary(
            rb, "fp32", args.c3_steps, f"c3 grain and ions ({w['n_macro']:.0e} macro-particles), electrons "
            f"n0 exp(phi) (not moved), FP32 split, FP64 Newton-multigrid Poisson", unit="ion particle-steps/s")
    if not args.no_conservative:
        rc = run_gpu([w], "fp32", args.c3_steps, args.c3_warmup, stream, conservative=True)
        out["conservative_poisson"] = secondary(
            rc, "fp32", args.c3_steps, "c3, FP32 split, field solve on the conservative (bilinear finite-element) form")
    if not args.no_cpu_baseline:
        # the grains are independent: the oracle runs the first `procs` grains
        # of the ensemble at once, one process (one thread) each
        procs = max(1, min(args.cpu_procs, len(os.sched_getaffinity(0)), len(ens)))
        rate, wall, cpu = cpu_baseline_grains([dict(g) for g in ens[:procs]], args.cpu_sample, args.cpu_steps, procs)
        out["cpu_baseline"] = {"value": rate, "unit": "particle-steps/s", "cores": procs, "kind": "oracle",
                               "sample": f"grains 0-{procs - 1} of the c4 ensemble, one process and thread each, "
                                         f"{args.cpu_sample:.0e} macro-particles per species per grain, "
                                         f"{args.cpu_steps} full steps timed in each process while all run ({wall:.1f} s "
                                         f"wall, {cpu:.1f} s of CPU time in the timed steps); the sum of the "
                                         f"processes' rates; numpy oracle"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
