"""Throughput of the speed-limited PIC/MCC step on one MI355X.

Workload: the batched Paschen sweep -- 64 independent argon gaps (d = 1 cm,
pd log-spaced from 0.1 to 100 Torr cm, quarter-mean-free-path cells clamped
to 128..4096, 1e4..2e6 target markers each, about 2.5e7 in all), FP32
particles with FP64 Poisson solves and population totals, every instance
advanced by the same launch pair.  A step is one pass of push, null-collision
MCC (elastic, excitation, ionization with spawn; ion charge exchange),
ion-induced secondary emission, population control, deposit and the Poisson
solve over every instance.  Markers start from the seeded state (uniform in
the first cell, kT_e = 1 eV) and are resident in HBM before timing starts.
The seeds take about EVOLVE = 200 steps to spread over their gaps, so when
the warmup is shorter the sweep first takes EVOLVE - W untimed steps (the
line's config names them): the timed steps always see the evolved sweep,
whatever W is.  The plain leg takes the same steps before its timing.

Prints one JSON line:
  value       particle-steps/s = sum over timed steps and instances of the
              markers entering the step, over the wall time of the steps,
              replayed from the captured HIP graph (16 steps per graph;
              captured before the timed region), in the launch shape the
              autotuner picks on a separate copy of the workload
  roofline    particle kernel: 56 algorithmic bytes per marker-step (28-byte
              record read + 28-byte record written) over its average
              HIP-event duration, against 8 TB/s, from the same number of
              steps launched one by one right after the timed ones; traffic
              is the committed counter summary's HBM bytes per marker-step
              times the markers of one of these launches
  plain       the same instances stepped one handle at a time (n_inst = 1)
  cpu_baseline the FP64 oracle on a bounded sample of the same instances

  configs     (--all-configs) the other workloads, each timed on its own:
              the plain FP64 gap (1 cm, 64 cells, 1e4 seeds), the 512-cell
              2 cm gap (1e6 seeds), the 4096-cell 5 cm gap (1e7 seeds, cell
              sort every 16 steps) and the 256-instance bisection round

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-plain]
       [--no-cpu] [--scale S] [--pic] [--all-configs]
       python bench.py --copy-calibration   (plain device copy of 1 GiB,
       for scaling HBM counters)
"""

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_MARKER_STEP = 56.0      # 28-byte FP32 record in + out
EVOLVE = 200                      # steps for the seeded sweep to spread over its gaps
HBM_PEAK_GBS = 8000.0             # MI355X HBM3E
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_gen_c4_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2103_12194_amd", "csrc", f)
                  for f in ("slpic_kernels.hip", "slpic_internal.hpp")]


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per particle-kernel launch and per marker-step from the
    committed counter summary, or None when the kernel sources changed
    since the counters were taken."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    m = re.search(r"kernel source sha256/16: ([0-9a-f]+)", text)
    b = re.search(r"HBM bytes per launch: ([0-9.eE+]+)", text)
    pm = re.search(r"HBM bytes per marker-step: ([0-9.eE+]+)", text)
    if not (m and b and pm) or m.group(1) != kernel_source_hash():
        return None
    return float(b.group(1)), float(pm.group(1))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--scale", type=float, default=1.0,
                    help="marker-count scale of the sweep (1 = full size)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--pic", action="store_true",
                    help="also compare SLPIC with plain PIC on one gap")
    ap.add_argument("--all-configs", action="store_true",
                    help="also time the single-gap and bisection-round workloads")
    ap.add_argument("--evolve", type=int, default=None,
                    help="untimed steps before the warmup (default: max(0, %d - warmup)); "
                         "e.g. 20000 times the sweep with its glow developed" % EVOLVE)
    return ap.parse_args()


def copy_calibration():
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n,
                      "launches": 3}), flush=True)


def workload(scale):
    import synth
    from synth import configs
    xs = synth.argon_like()
    w = configs.c4(xs.sigma_total_max(), precision=32)
    if scale != 1.0:
        w = configs.scaled(w, scale)
    return w, xs


def history_total(sim, first, n):
    total = 0
    for k in range(sim.n_inst):
        total += int(sim.history(first, n, inst=k)["n_in"].sum())
    return total


def time_steps(sim, steps, profile):
    import torch
    if profile:
        sim.profile(True)
    s0 = sim.steps_done()
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = sim.kernel_times() if profile else None
    if profile:
        sim.profile(False)
    return s0, t1 - t0, kt


def plain_leg(w, xs, steps, warmup):
    """Each instance in a handle of its own, stepped alone, with the Philox
    stream it has in the batch: it repeats the batched run draw for draw."""
    import dataclasses
    import paper_2103_12194_amd as slpic
    ps, secs = 0, 0.0
    for k, inst in enumerate(w.instances):
        sim = slpic.Sim([dataclasses.replace(inst, stream=k)], w.run, xs)
        sim.step(warmup)
        s0, dt, _ = time_steps(sim, steps, profile=False)
        ps += history_total(sim, s0, steps)
        secs += dt
        sim.close()
        del sim
    return ps, secs


def host_cpu():
    """Logical CPUs the process may use and the CPU model of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"logical_cpus": os.cpu_count(), "usable_cpus": usable, "model": model}


def cpu_leg(w, xs, budget_s):
    """The oracle on a sample: every 8th instance of the sweep with markers
    scaled so one step stays well under a second, each stepped from its
    seeded state on a host thread of its own (the oracle releases the
    interpreter while it steps) for the time budget.  Returns the aggregate
    rate, the sample description and the number of threads."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    from synth import configs
    sample = w.instances[::8]
    threads = max(1, min(len(sample), os.cpu_count() or 1, 16))

    def one(k):
        inst = sample[k]
        scale = min(1.0, 20000.0 / max(inst.n_seed, 1))
        small = configs.scaled(configs.Workload("s", w.run, [inst], 1), scale).instances[0]
        sim = oracle.Sim(small, w.run, xs, instance_index=8 * k)
        t0 = time.perf_counter()
        ps = n = 0
        while time.perf_counter() - t0 < budget_s:
            sim.step(1)
            ps += int(sim.stats()["n_in"])
            n += 1
        return ps, n

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(one, range(len(sample))))
    secs = time.perf_counter() - t0
    ps = sum(r[0] for r in res)
    steps = sum(r[1] for r in res)
    desc = (f"every 8th instance of the sweep ({len(sample)} instances) with "
            f"at most 2e4 seeded markers each, FP64, each stepped from its "
            f"seeded state on its own host thread for {budget_s:.0f} s "
            f"({steps} steps in all)")
    return ps / secs, desc, threads


def pic_leg(xs):
    """SLPIC against plain PIC (v_limit = +inf, beta == 1, the PIC step of
    Sec. IV) on the C1 gap in FP32, each from the same seeded state over the
    same simulated time, one ion crossing time (Sec. IV), with graph replay:
    the Table I comparison of steps and wall time on this GPU."""
    import math
    import paper_2103_12194_amd as slpic
    from paper_2103_12194_amd import breakdown as bd
    from synth import configs
    w = configs.c1(precision=32)
    base = w.instances[0]
    t_c = bd.crossing_time(base.d, base.V)
    out = {"gap": "C1: d=1 cm, p=1 Torr, V=300 V, 64 cells, 1e4 seeded electrons, FP32",
           "simulated_s": t_c}
    for name, v_limit in (("slpic", 0.0), ("pic", math.inf)):
        inst = configs.replace(base, v_limit=v_limit)
        sim = slpic.Sim([inst], w.run, xs)
        steps = int(math.ceil(t_c / sim.scalars()["dt"]))
        sim.use_graph(True)
        s0, secs, _ = time_steps(sim, steps, profile=False)
        out[name] = {"dt_s": sim.scalars()["dt"], "steps": steps, "wall_s": secs,
                     "electrons_at_end": sim.count(0), "ions_at_end": sim.count(1)}
        sim.close()
    out["step_ratio"] = out["pic"]["steps"] / out["slpic"]["steps"]
    out["speedup"] = out["pic"]["wall_s"] / out["slpic"]["wall_s"]
    print(f"# pic leg: {out['pic']['steps']} PIC steps in {out['pic']['wall_s']:.2f} s, "
          f"{out['slpic']['steps']} SLPIC steps in {out['slpic']['wall_s']:.3f} s",
          file=sys.stderr, flush=True)
    return out


def size_class(inst):
    """Size class of an instance: marker target (<= 1e5, <= 1e6, above)
    times cells (<= 1024, above)."""
    m = 0 if inst.n_target <= 1e5 else (1 if inst.n_target <= 1e6 else 2)
    return 2 * m + (0 if inst.cells <= 1024 else 1)


def tuned_shape(w, xs, trial_steps=2):
    """Launch shape the autotuner picks for a workload, on a handle of its
    own (its trial steps advance that handle only): (grid, waves per SIMD,
    work distribution)."""
    import paper_2103_12194_amd as slpic
    sim = slpic.Sim(w.instances, w.run, xs)
    sim.autotune(trial_steps)
    shape = sim.launch_shape() + (sim.work_distribution(),)
    sim.close()
    return shape


def apply_shape(sim, shape):
    sim.set_launch_shape(shape[0], shape[1])
    sim.set_work_distribution(shape[2])


def per_class_leg(w, xs, warm, steps):
    """The bisection round split into one handle per size class, each with
    its autotuned launch shape, every instance on its batch index's Philox
    stream (so each repeats its draws in the single handle): the classes'
    steps are enqueued on their handles' own streams and run concurrently."""
    import dataclasses
    import torch
    import paper_2103_12194_amd as slpic
    from synth import configs
    groups = {}
    for k, inst in enumerate(w.instances):
        groups.setdefault(size_class(inst), []).append(dataclasses.replace(inst, stream=k))
    sims, shapes = [], {}
    for c, insts in sorted(groups.items()):
        sub = configs.Workload(f"class {c}", w.run, insts, w.steps)
        shape = tuned_shape(sub, xs)
        sim = slpic.Sim(insts, w.run, xs)
        apply_shape(sim, shape)
        sim.step(warm)
        sims.append(sim)
        shapes[str(c)] = {"instances": len(insts), "grid": shape[0], "waves_per_simd": shape[1],
                          "claimed_runs": shape[2]}
    for sim in sims:
        sim.sync()
    torch.cuda.synchronize()
    s0 = [sim.steps_done() for sim in sims]
    t0 = time.perf_counter()
    for sim in sims:
        sim.step(steps)
    for sim in sims:
        sim.sync()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    ps = sum(history_total(sim, a, steps) for sim, a in zip(sims, s0))
    for sim in sims:
        sim.close()
    return {"value": ps / secs, "unit": "particle-steps/s", "ms_per_step": secs * 1e3 / steps,
            "classes": shapes}


def configs_leg(xs):
    """Throughput of the other workloads, each from its seeded state after a
    warmup that lets its population settle: (name, workload, warmup,
    timed steps)."""
    import paper_2103_12194_amd as slpic
    from synth import configs
    legs = [("C1 plain FP64 gap", configs.c1(), 200, 400),
            ("C2 512-cell gap, 300 V", configs.c2(300.0), 200, 200),
            ("C3 4096-cell gap, sort every 16 steps", configs.c3(), 2048, 64),
            ("C5 256-instance bisection round", configs.c5(xs.sigma_total_max()), 100, 50)]
    out = {}
    for name, w, warm, steps in legs:
        sim = slpic.Sim(w.instances, w.run, xs)
        sim.step(warm)
        sim.sync()
        s0, secs, (gen_ms, tail_ms, nk) = time_steps(sim, steps, profile=True)
        ps = history_total(sim, s0, steps)
        bytes_per = 2.0 * (4 + 3 * 8 + 8 + 8) if w.run.precision == 64 else BYTES_PER_MARKER_STEP
        achieved = bytes_per * ps / nk / (gen_ms / nk * 1e-3) / 1e9
        out[name] = {"value": ps / secs, "unit": "particle-steps/s", "n_inst": len(w.instances),
                     "dtype": "f64" if w.run.precision == 64 else "f32",
                     "warmup": warm, "steps": steps, "ms_per_step": secs * 1e3 / steps,
                     "kernel_ms": gen_ms / nk, "tail_kernel_ms": tail_ms / nk,
                     "markers_per_step": ps / steps, "bytes_per_marker_step": bytes_per,
                     "achieved_GBs": round(achieved, 1),
                     "frac": round(achieved / HBM_PEAK_GBS, 4)}
        print(f"# {name}: {ps / secs:.3e} particle-steps/s, particle kernel "
              f"{gen_ms / nk:.3f} ms, {ps / steps:.3e} markers/step", file=sys.stderr, flush=True)
        sim.close()
        del sim
        if name.startswith("C5"):
            pc = per_class_leg(w, xs, warm, steps)
            out[name]["per_size_class_autotuned"] = pc
            print(f"# {name}, one handle per size class, autotuned: {pc['value']:.3e} "
                  f"particle-steps/s {pc['classes']}", file=sys.stderr, flush=True)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              f"(instances of a sweep are independent and would be spread "
              f"over GPUs by a launcher, which this package does not include)",
              file=sys.stderr)
        return 2
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        return 1
    if args.copy_calibration:
        copy_calibration()
        return 0
    import paper_2103_12194_amd as slpic
    if not os.path.exists(slpic.LIB):
        slpic.build()
    w, xs = workload(args.scale)
    print(f"# {w.name}: {len(w.instances)} instances, "
          f"{sum(i.n_target for i in w.instances):.3e} target markers", file=sys.stderr, flush=True)

    # launch shape: autotuned on a copy of the workload, so that the timed
    # handle takes exactly the warmup steps asked for
    shape = tuned_shape(w, xs)
    print(f"# autotuned launch shape: grid {shape[0]}, {shape[1]} waves per SIMD, "
          f"{'claimed runs' if shape[2] else 'equal shares'}", file=sys.stderr, flush=True)
    sim = slpic.Sim(w.instances, w.run, xs)
    default_shape = sim.launch_shape() + (sim.work_distribution(),)
    apply_shape(sim, shape)
    # untimed steps that let the seeds spread over their gaps, then the warmup
    evolve = max(0, EVOLVE - args.warmup) if args.evolve is None else max(0, args.evolve)
    sim.step(evolve)
    sim.step(args.warmup)
    sim.sync()
    print(f"# {evolve} evolution steps and {args.warmup} warmup steps done", file=sys.stderr,
          flush=True)
    # the timed steps: graph replay (captured here, outside the timed region)
    sim.use_graph(True)
    s0, secs, _ = time_steps(sim, args.steps, profile=False)
    ps = history_total(sim, s0, args.steps)
    value = ps / secs
    sim.use_graph(False)
    # kernel durations: the same number of steps launched one by one with
    # HIP events around each kernel on the handle's stream
    e0, esecs, (gen_ms, tail_ms, nk) = time_steps(sim, args.steps, profile=True)
    eps_ = history_total(sim, e0, args.steps)
    print(f"# timed {args.steps} steps (graph): {secs * 1e3 / args.steps:.3f} ms/step; "
          f"then {args.steps} eager steps: {esecs * 1e3 / args.steps:.3f} ms/step, "
          f"particle kernel {gen_ms / nk:.3f} ms, tail {tail_ms / nk:.3f} ms",
          file=sys.stderr, flush=True)
    eager = {"value": eps_ / esecs, "ms_per_step": esecs * 1e3 / args.steps}

    per_launch = BYTES_PER_MARKER_STEP * eps_ / nk
    achieved = per_launch / (gen_ms / nk * 1e-3) / 1e9
    tr = measured_traffic()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if tr is None else tr[1] * eps_ / nk,
                "traffic_per_marker_step": None if tr is None else tr[1],
                "traffic_source": "profiles/k_gen_c4_traffic.txt (rocprofv3 FETCH_SIZE + "
                                  "WRITE_SIZE per marker-step, scaled to this launch)",
                "kernel": "k_gen (particle kernel)",
                "bytes_per_launch": per_launch,
                "kernel_ms": gen_ms / nk, "tail_kernel_ms": tail_ms / nk}
    n_markers = ps / args.steps
    sim.close()
    del sim

    plain = None
    if not args.no_plain:
        pps, psecs = plain_leg(w, xs, args.steps, evolve + args.warmup)
        plain = {"value": pps / psecs, "unit": "particle-steps/s",
                 "ms_per_step_all_instances": psecs * 1e3 / args.steps,
                 "batched_over_plain": value / (pps / psecs)}
        print(f"# plain leg: {plain['value']:.3e} particle-steps/s", file=sys.stderr, flush=True)

    pic = pic_leg(xs) if args.pic else None
    others = configs_leg(xs) if args.all_configs else None

    cpu = None
    if not args.no_cpu:
        rate, desc, threads = cpu_leg(w, xs, args.cpu_seconds)
        cpu = {"value": rate, "unit": "particle-steps/s", "cores": threads,
               "threads": threads, "host": host_cpu(),
               "kind": "oracle", "sample": desc}

    line = {
        "metric": "particle-steps/s (push+MCC+deposit); batched FP32 vs plain at fixed V_b error",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": secs * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched Paschen sweep: 64 argon gaps, d=1 cm, "
                               "pd 0.1-100 Torr cm log-spaced, 128-4096 cells, "
                               "1e4-2e6 target markers each; FP32 particles, "
                               "FP64 Poisson and totals; one launch pair per step",
                   "n_inst": len(w.instances), "marker_scale": args.scale,
                   "markers_per_step": n_markers, "parallelism": "none (1 GPU)",
                   "initial_state": "seeded in each gap's first cell (1 eV Maxwellian)",
                   "untimed_steps_before_warmup": evolve},
        "roofline": roofline, "plain": plain, "eager": eager,
        "launch_shape": {"grid": shape[0], "waves_per_simd": shape[1],
                         "claimed_runs": shape[2], "autotuned": True,
                         "default": {"grid": default_shape[0],
                                     "waves_per_simd": default_shape[1],
                                     "claimed_runs": default_shape[2]}},
        "cpu_baseline": cpu,
    }
    if pic is not None:
        line["pic"] = pic
    if others is not None:
        line["configs"] = others
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
