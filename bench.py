"""Benchmark of the aspherical PIC particle loop on one MI355X.

A step is one full PIC step of the library (particle push with gather, boundary
tests and deposit for both species; Maxwellian injection; periodic cell sort;
charge density, FP64 multigrid Poisson solve and nodal gradient; grain force).
`value` is particle-steps per second over the timed steps (resident particles of
both species pushed per step, summed, divided by the wall time between two
device synchronisations), inputs resident in HBM before timing starts.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
[--workload c3] [--no-fp64] [--no-cpu-baseline] [--no-ensemble]

Beside the headline workload the line carries the plain FP64 path on the same
workload (`fp64`), the 64-grain ensemble in one context (`ensemble`), and the
oracle's rate on a bounded sample (`cpu_baseline`).
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_push_split_c3_traffic.md")
TRAFFIC_WORKLOAD = "c3"
KERNEL_SOURCE = os.path.join(ROOT, "paper_2307_11107_amd", "csrc", "particles.hip")
COPY_BYTES = 1 << 30           # calibration copy: 1 GiB read + 1 GiB written


def copy_calibration():
    """A plain device copy of known size, run once outside the timed region so
    that a hardware-counter run of this script can scale its byte counters."""
    import torch
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    del x, y


def measured_traffic(particles_per_launch, workload):
    """HBM bytes per push launch from the committed counter summary, if it was
    taken on the current kernel source and this workload (else None)."""
    if workload != TRAFFIC_WORKLOAD:
        return None
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
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


def run_gpu(grains, precision, steps, warmup, stream, autotune=False, boltzmann=False, conservative=False):
    """Loads every grain, runs `warmup` steps (the autotuner's steps among
    them), then times `steps` steps between device synchronisations."""
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
            "schedule": sched}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000)
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--ensemble-steps", type=int, default=16)
    ap.add_argument("--ensemble-warmup", type=int, default=30)
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
    w = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    copy_calibration()

    r32 = run_gpu([w], "fp32", args.steps, args.warmup, stream)
    value = r32["particle_steps"] / r32["elapsed"]
    tm = r32["timing"]
    push_avg_ms = tm["push_ms"] / max(tm["push_launches"], 1)
    per_launch = r32["particle_steps"] / max(tm["push_launches"], 1)
    achieved = BYTES_PER_PARTICLE["fp32"] * per_launch / (push_avg_ms * 1e-3) / 1e9
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
        "config": {"workload": f"{args.workload}: alpha={w['alpha']}, wce/wpe={w['wce']}, grid {w['n1']}x{w['n2']}, "
                               f"x1_out={w['x1_out']}, lambdaD/R0={w['kappa']}, mi/me={w['mi']}, Ti/Te={w['Ti']}, "
                               f"{w['n_macro']:.0e} macro-particles per species, Maxwellian flux injection, "
                               f"dt={w['dt']}/wpe; FP32 split push/gather/deposit, FP64 multigrid Poisson and tallies",
                   "particles_per_species": w["n_macro"], "grid": [w["n1"], w["n2"]]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(per_launch, args.workload),
                     "kernel": "k_push_split (FP32 split push+gather+deposit, all species in one launch)", "avg_launch_ms": push_avg_ms,
                     "algorithmic_bytes_per_particle": BYTES_PER_PARTICLE["fp32"]},
        "breakdown_ms_per_step": {k: tm[k] / max(tm["steps"], 1) for k in ("push_ms", "inject_ms", "sort_ms", "field_ms")},
        "mg_cycles_per_step": tm["mg_cycles"] / max(tm["steps"], 1),
        "balance_exact": r32["balance_exact"],
    }
    if not args.no_fp64:
        r64 = run_gpu([w], "fp64", args.steps, args.warmup, stream)
        v64 = r64["particle_steps"] / r64["elapsed"]
        t64 = r64["timing"]
        a64 = t64["push_ms"] / max(t64["push_launches"], 1)
        out["fp64"] = {"value": v64, "ms_per_step": 1e3 * r64["elapsed"] / args.steps,
                       "push_avg_launch_ms": a64,
                       "push_GBps": BYTES_PER_PARTICLE["fp64"] * r64["particle_steps"] / max(t64["push_launches"], 1)
                       / (a64 * 1e-3) / 1e9}
        out["speedup_fp32_vs_fp64"] = value / v64
    if not args.no_ensemble:
        ens = ensemble_c4()
        re = run_gpu(ens, "fp32", args.ensemble_steps, args.ensemble_warmup, stream, autotune=True)
        te = re["timing"]
        pe = te["push_ms"] / max(te["push_launches"], 1)
        ve = re["particle_steps"] / re["elapsed"]
        gbe = BYTES_PER_PARTICLE["fp32"] * re["particle_steps"] / max(te["push_launches"], 1) / (pe * 1e-3) / 1e9
        out["ensemble"] = {
            "workload": f"c4: {len(ens)} grains in one context (alpha U[0,0.2], wce/wpe in {{0,0.5,1}}, "
                        f"lambdaD/R0 U[0.5,5], grids 128x128..512x256, "
                        f"{sum(g['n_macro'] for g in ens):.3g} macro-particles per species in total, "
                        f"log-uniform 1e6-2e7 per grain), FP32 split, autotuned schedule, graph-captured steps",
            "value": ve, "unit": "particle-steps/s", "ms_per_step": 1e3 * re["elapsed"] / args.ensemble_steps,
            "push_avg_launch_ms": pe, "push_GBps": gbe, "push_frac_of_hbm_peak": gbe / HBM_PEAK_GBS,
            "breakdown_ms_per_step": {k: te[k] / max(te["steps"], 1)
                                      for k in ("push_ms", "inject_ms", "sort_ms", "field_ms")},
            "mg_cycles_per_step": te["mg_cycles"] / max(te["steps"], 1),
            "schedule": re["schedule"], "balance_exact": re["balance_exact"]}
    if not args.no_c5 and args.workload != "c5":
        # the largest single grain (2048 x 1024 cells, 2e8 macro-particles per
        # species): the push at four times the c3 state
        w5 = WORKLOADS["c5"]
        r5 = run_gpu([w5], "fp32", args.c5_steps, args.c5_warmup, stream)
        t5 = r5["timing"]
        p5 = t5["push_ms"] / max(t5["push_launches"], 1)
        gb5 = BYTES_PER_PARTICLE["fp32"] * r5["particle_steps"] / max(t5["push_launches"], 1) / (p5 * 1e-3) / 1e9
        out["c5"] = {
            "workload": f"c5: alpha={w5['alpha']}, wce/wpe={w5['wce']}, grid {w5['n1']}x{w5['n2']}, "
                        f"x1_out={w5['x1_out']}, lambdaD/R0={w5['kappa']}, {w5['n_macro']:.0e} macro-particles "
                        f"per species, FP32 split, FP64 multigrid",
            "value": r5["particle_steps"] / r5["elapsed"], "unit": "particle-steps/s",
            "ms_per_step": 1e3 * r5["elapsed"] / args.c5_steps,
            "push_avg_launch_ms": p5, "push_GBps": gb5, "push_frac_of_hbm_peak": gb5 / HBM_PEAK_GBS,
            "breakdown_ms_per_step": {k: t5[k] / max(t5["steps"], 1)
                                      for k in ("push_ms", "inject_ms", "sort_ms", "field_ms")},
            "mg_cycles_per_step": t5["mg_cycles"] / max(t5["steps"], 1),
            "balance_exact": r5["balance_exact"]}
    if not args.no_boltzmann:
        # the same grain and ions with Boltzmann electrons (not moved; the
        # field solve is the Newton-multigrid one)
        rb = run_gpu([w], "fp32", args.steps, args.warmup, stream, boltzmann=True)
        tb = rb["timing"]
        pb = tb["push_ms"] / max(tb["push_launches"], 1)
        gbb = BYTES_PER_PARTICLE["fp32"] * rb["particle_steps"] / max(tb["push_launches"], 1) / (pb * 1e-3) / 1e9
        out["boltzmann_electrons"] = {
            "workload": f"{args.workload} grain and ions ({w['n_macro']:.0e} macro-particles), electrons "
                        f"n0 exp(phi) (not moved), FP32 split, FP64 Newton-multigrid Poisson",
            "value": rb["particle_steps"] / rb["elapsed"], "unit": "ion particle-steps/s",
            "ms_per_step": 1e3 * rb["elapsed"] / args.steps, "push_avg_launch_ms": pb, "push_GBps": gbb,
            "push_frac_of_hbm_peak": gbb / HBM_PEAK_GBS,
            "breakdown_ms_per_step": {k: tb[k] / max(tb["steps"], 1)
                                      for k in ("push_ms", "inject_ms", "sort_ms", "field_ms")},
            "mg_cycles_per_step": tb["mg_cycles"] / max(tb["steps"], 1),
            "balance_exact": rb["balance_exact"]}
    if not args.no_conservative:
        # the same workload with the conservative (finite-element) field solve
        rc = run_gpu([w], "fp32", args.steps, args.warmup, stream, conservative=True)
        tc = rc["timing"]
        out["conservative_poisson"] = {
            "workload": f"{args.workload}, FP32 split, field solve on the conservative (bilinear finite-element) form",
            "value": rc["particle_steps"] / rc["elapsed"], "unit": "particle-steps/s",
            "ms_per_step": 1e3 * rc["elapsed"] / args.steps,
            "breakdown_ms_per_step": {k: tc[k] / max(tc["steps"], 1)
                                      for k in ("push_ms", "inject_ms", "sort_ms", "field_ms")},
            "mg_cycles_per_step": tc["mg_cycles"] / max(tc["steps"], 1),
            "balance_exact": rc["balance_exact"]}
    if not args.no_cpu_baseline:
        rate, secs = cpu_baseline(w, args.cpu_sample, args.cpu_steps)
        out["cpu_baseline"] = {"value": rate, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"{args.workload} geometry, grid and field solve with "
                                         f"{args.cpu_sample:.0e} macro-particles per species, {args.cpu_steps} full "
                                         f"steps ({secs:.1f} s of CPU time; numpy oracle, one thread)"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
