"""Benchmark of the batched collision step on one MI355X.

Workload: 65,536 cells with lognormal particle counts clipped to [16, 4096]
(about 2.15e7 electrons and ions, mass ratio 100), N97, moment correction
on, inputs resident in HBM.  The headline is the FP32-kinematics step
(FP64 state, sums and correction) run as one HIP graph replay per step; the
plain FP64 step on the same inputs is reported beside it.  The kernel of
each cell-size bucket is then timed alone (HIP events on the stream it runs
on) and the slowest one is set against the HBM roofline.  Prints ONE JSON
line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--autotune]
  python bench.py --copy-calibration MIB   (reference copy for the byte counters)
  python bench.py --paper-test1            (the paper's Test 1 cases: one JSON line each)
  python bench.py --paper-test2            (the paper's Test 2 cases: one JSON line each)
  python bench.py --paper-test3            (the paper's Test 3 cases: one JSON line each)
  python bench.py --paper-test3-curve      (T3b and T3c relaxed to equilibrium, sampled)
  python bench.py --nxn                    (N x N against order-N pairing, one JSON line each)
  python bench.py --rebin                  (incremental re-binning after a push, one JSON line each)
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic HBM bytes per particle and step (sorted entry): w read 8,
# v read 24, v write 24, and 8 for the cell and species ids a particle
# carries (here implied by the offsets, whose per-group entries are < 0.1 %)
BYTES_PER_PARTICLE_STEP = 64
BYTES_MOVED = 56  # what the sorted kernel itself reads and writes per particle
# the unsorted entry: the sorted step plus binning (ids in, permutation out:
# 12 B) and the payload moved each way (w, v gathered: 32 + 32 B; v
# scattered back: 24 + 24 B) and the permutation read twice (8 B): 150 B
BYTES_UNSORTED = 150
BYTES_BIN = 12  # binning alone: cell and species ids read, permutation written
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "collide_c3_hbm_traffic.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "collide_c3_valu.txt")
RELAX_FILE = os.path.join(ROOT, "tests", "golden", "c3_4096_relaxation_oracle.txt")
# MI355X: 256 CUs of 4 SIMDs at 2.4 GHz; a wave64 VALU instruction holds a
# SIMD for 4 cycles (16 lanes), so 6.14e11 wave instructions/s; FP64 vector
# peak 78.6 TFLOP/s
VALU_PEAK_WINST = 256 * 4 * 2.4e9 / 4
FP64_PEAK_TFLOPS = 78.6
BUCKET_CAP = [128, 256, 512, 1024, 2048, 4096, 32768]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cells", type=int, default=65536)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--autotune", action="store_true",
                    help="time the candidate variants per bucket instead of the built-in table")
    ap.add_argument("--only", choices=["fp32", "fp64"], default=None)
    ap.add_argument("--quick", action="store_true",
                    help="only the plan timings (for profiling runs): no autotuned plan, "
                         "per-call, unsorted, copy-ceiling or relaxation legs")
    ap.add_argument("--paper-test1", action="store_true",
                    help="only time the paper's Test 1 cases (SI units, 180 cells, FP64) and exit")
    ap.add_argument("--paper-test2", action="store_true",
                    help="only time the paper's Test 2 cases (SI units, 180 cells, FP64) and exit")
    ap.add_argument("--rebin", action="store_true",
                    help="only time incremental re-binning (mcc_rebin) against binning from "
                         "scratch on the 65,536-cell population after a push, and exit")
    ap.add_argument("--nxn", action="store_true",
                    help="only time the N x N pairing (Sec. 3.1) against order-N on 1024 cells "
                         "of 256 electrons + 256 ions, and exit")
    ap.add_argument("--hard-sphere", action="store_true",
                    help="only time the hard-sphere process against N97 (both FP64) on the "
                         "65,536-cell population, and exit")
    ap.add_argument("--paper-test3-curve", action="store_true",
                    help="relax the paper's T3b and T3c to equilibrium (1.1e6 steps each), "
                         "sampling T_e and T_i, and exit")
    ap.add_argument("--paper-test3", action="store_true",
                    help="only time the paper's Test 3 cases (SI units, 1600 cells, FP64) and exit")
    ap.add_argument("--unsorted", action="store_true",
                    help="only time the unsorted entry (mcc_collide on the 65,536-cell population "
                         "in random order, FP32 kinematics) and mcc_bin alone, and exit")
    ap.add_argument("--configs", action="store_true",
                    help="only time the other named workloads at their full sizes (FP64 and "
                         "FP32 plans; tangent and adjoint steps of the differentiated one) and "
                         "exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB three times (the "
                         "reference reading for the HBM byte counters) and exit")
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def copy_calibration(mib):
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": n * 8, "copies": 3}), flush=True)


def kernel_source_hash():
    """sha256 over the code the collide kernels are built from (their
    instantiation units, the headers they include and the public header;
    comments aside): counters taken from other code do not describe the
    kernels that run now."""
    from paper_2407_19151_amd import profile_summary
    return profile_summary.source_hash()


def read_traffic():
    """Per-launch HBM bytes of each collide kernel from the committed
    rocprofv3 counter summary, if it was taken from the current sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    table, src, ff, wf = {}, None, None, None
    for line in open(TRAFFIC_FILE):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "source_sha256":
            src = f[1]
        elif f[0] == "fetch_factor":
            ff = float(f[1])
        elif f[0] == "write_factor":
            wf = float(f[1])
        elif f[0] == "kernel":
            # kernel <mode> <tpc>x<cap> L<layout> fetch_kib <F> write_kib <W>
            table[(f[1], f[2], f[3])] = (float(f[5]), float(f[7]))
    if src != kernel_source_hash() or ff is None or wf is None:
        return None
    return {k: (fk * 1024 * ff + wk * 1024 * wf) for k, (fk, wk) in table.items()}


def read_valu():
    """Per-launch VALU wave instructions and FP64 operations of each collide
    kernel from the committed rocprofv3 counter summary, if it was taken
    from the current sources: {(mode, tpcxcap, L<layout>): (valu, fp64_flops)}."""
    if not os.path.exists(VALU_FILE):
        return None
    table, src = {}, None
    for line in open(VALU_FILE):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "source_sha256":
            src = f[1]
        elif f[0] == "kernel":
            # kernel <mode> <tpc>x<cap> L<layout> valu <V> fp64_flops <F> ...
            table[(f[1], f[2], f[3])] = (float(f[5]), float(f[7]))
    if src != kernel_source_hash():
        return None
    return table


def events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_plan(plan, steps, warmup, first_step=1000):
    import torch
    plan.run(first_step, warmup)
    torch.cuda.synchronize()
    e0, e1 = events()
    t0 = time.perf_counter()
    e0.record()
    plan.run(first_step + warmup, steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def time_buckets(plan, buckets, steps, first_step=5000):
    """Average duration of each bucket's kernel, launched alone `steps` times
    on the current stream (the one the plan launches on) between two events."""
    import torch
    out = {}
    for b in buckets:
        plan.run_bucket(b, first_step)  # warm-up
        torch.cuda.synchronize()
        e0, e1 = events()
        e0.record()
        for k in range(steps):
            plan.run_bucket(b, first_step + 1 + k)
        e1.record()
        torch.cuda.synchronize()
        out[b] = e0.elapsed_time(e1) / steps
    return out


def bucket_particles(wl):
    sizes = np.diff(wl.offsets[::wl.n_species])
    b = np.searchsorted(np.asarray(BUCKET_CAP), sizes, side="left")
    return {int(k): int(sizes[b == k].sum()) for k in np.unique(b)}


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return os.cpu_count() or 1, model


def cpu_baseline(seconds):
    """The oracle on a bounded sample of the same workload: one thread, then
    every host core (its cell loop in OpenMP threads; the same result bit for
    bit)."""
    import oracle
    from paper_2407_19151_amd import workloads as W
    nproc, model = host_cpu()
    out = {}
    for threads in (1, nproc):
        sub = W.config3(n_cells=2048, seed_data=3)
        pc = sub.particle_collisions_per_step()
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        steps = 0
        while True:
            oracle.run_workload(sub, steps=1, first_step=steps)
            steps += 1
            if time.perf_counter() - t0 > seconds / 2:
                break
        dt = time.perf_counter() - t0
        out[threads] = (pc * steps / dt, steps, sub.n)
    # the other workloads, on every core: whole at their full sizes except the
    # relativistic beam (its first 1024 of 16384 cells, rates scaled per
    # particle); each for about a second
    configs = {}
    oracle.set_threads(nproc)
    for name, make in (("config1", W.config1), ("config2_n97", lambda: W.config2(method=W.N97)),
                       ("config2_ta77", lambda: W.config2(method=W.TA77)),
                       ("config4_relativistic_1024_cells", lambda: W.config4(n_cells=1024)),
                       ("config5", W.config5)):
        wl = make()
        pc = wl.particle_collisions_per_step()
        t0 = time.perf_counter()
        steps = 0
        while True:
            st = oracle.run_workload(wl, steps=1, first_step=steps)
            steps += 1
            if time.perf_counter() - t0 > 1.0:
                break
        dt = time.perf_counter() - t0
        configs[name] = dict(particles=wl.n, steps=steps,
                             particle_collisions_per_s=pc * steps / dt,
                             particle_steps_per_s=wl.n * steps / dt,
                             pairs_per_s=st["pairs"] * steps / dt)
    oracle.set_threads(1)
    v1, s1, n1 = out[1]
    va, sa, _ = out[nproc]
    return dict(value=va, unit="particle-collisions/s", cores=nproc, kind="oracle",
                sample="%d steps (%d threads) and %d steps (1 thread) of the first 2048 cells "
                       "of the same recipe (%d particles, N97, FP64, correction on)"
                       % (sa, nproc, s1, n1),
                one_thread=v1, nproc=nproc, cpu=model, configs=configs)


def copy_ceiling():
    """Device-to-device copy of 1 GiB (float64), the best of 5, in GB/s
    (bytes read plus bytes written)."""
    import torch
    n = (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    best = 1e30
    for _ in range(6):
        e0, e1 = events()
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n * 8 / (best * 1e-3) / 1e9


def relaxation_rate_error(ctx):
    """The FP32-kinematics and FP64 steps against the oracle over 200 steps
    of 4096 cells of the same recipe: the relaxation rate of T_e - T_i (slope
    of its logarithm against the step) and the largest temperature
    deviation.  The oracle's trajectory is the committed reference written
    by tests/golden/make_c3_relaxation_reference.py."""
    import torch
    from paper_2407_19151_amd import autodiff, native, runner
    from paper_2407_19151_amd import workloads as W
    ref = np.loadtxt(RELAX_FILE)
    steps = int(ref[-1, 0])
    wl = W.config3(n_cells=4096)
    out = {}

    def rate(T):
        return -np.polyfit(np.arange(T.shape[0]), np.log(T[:, 0] - T[:, 1]), 1)[0]

    r_or = rate(ref[:, 1:3])
    for mode, prec in (("fp32", native.MCC_FP32_KINEMATICS), ("fp64", native.MCC_FP64)):
        dw = runner.DeviceWorkload(wl)
        plan = runner.make_plan(ctx, dw, params=runner.params_for(wl, precision=prec),
                                autotune=False)
        v = torch.stack([dw.vx, dw.vy, dw.vz])
        T = [autodiff.species_temperatures(wl, v)]
        for k in range(steps):
            plan.run(k, 1)
            T.append(autodiff.species_temperatures(wl, torch.stack([dw.vx, dw.vy, dw.vz])))
        plan.close()
        T = torch.stack(T).cpu().numpy()
        out[mode] = dict(rate_rel_err=abs(rate(T) / r_or - 1.0),
                         max_T_rel_dev=float(np.abs(T / ref[:, 1:3] - 1.0).max()))
    return dict(cells=wl.n_cells, particles=wl.n, steps=steps, oracle_rate_per_step=r_or,
                **out)


def unsorted_entry(ctx, wl_sorted, mode, steps, warmup):
    """mcc_collide (particles in any order) on the same population in random
    order, and mcc_bin alone on its ids."""
    import torch
    from paper_2407_19151_amd import native, runner
    wl = wl_sorted.unsorted(seed=77)
    dw = runner.DeviceWorkload(wl)
    prec = native.MCC_FP32_KINEMATICS if mode == "fp32" else native.MCC_FP64
    params = runner.params_for(wl, precision=prec)
    for k in range(warmup):
        runner.collide_unsorted(ctx, dw, k, params=params)
    torch.cuda.synchronize()
    e0, e1 = events()
    e0.record()
    for k in range(steps):
        runner.collide_unsorted(ctx, dw, warmup + k, params=params)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    for _ in range(warmup):
        ctx.bin(dw.cells, dw.species, wl.n_cells, wl.n_species)
    torch.cuda.synchronize()
    e0, e1 = events()
    e0.record()
    for _ in range(steps):
        ctx.bin(dw.cells, dw.species, wl.n_cells, wl.n_species)
    e1.record()
    torch.cuda.synchronize()
    bms = e0.elapsed_time(e1) / steps
    assert ctx.device_error() == 0
    del dw
    torch.cuda.empty_cache()
    gbs = BYTES_UNSORTED * wl.n / (ms * 1e-3) / 1e9
    bgbs = BYTES_BIN * wl.n / (bms * 1e-3) / 1e9
    return {"ms_per_step": ms, "value": wl.particle_collisions_per_step() / (ms * 1e-3),
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "bytes_per_particle_step": BYTES_UNSORTED},
            "bin_ms": bms,
            "bin_roofline": {"bound": "hbm", "achieved": bgbs, "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": bgbs / HBM_PEAK_GBS,
                             "bytes_per_particle": BYTES_BIN}}


def per_call_sorted(ctx, wl, mode, steps, warmup):
    """mcc_collide_sorted called once per step (no plan: the work lists and
    the weights' data are rebuilt every call)."""
    import torch
    from paper_2407_19151_amd import native, runner
    dw = runner.DeviceWorkload(wl)
    prec = native.MCC_FP32_KINEMATICS if mode == "fp32" else native.MCC_FP64
    params = runner.params_for(wl, precision=prec)
    for k in range(warmup):
        runner.collide_sorted(ctx, dw, k, params=params, with_stats=False)
    torch.cuda.synchronize()
    e0, e1 = events()
    e0.record()
    for k in range(steps):
        runner.collide_sorted(ctx, dw, warmup + k, params=params, with_stats=False)
    e1.record()
    torch.cuda.synchronize()
    del dw
    torch.cuda.empty_cache()
    return e0.elapsed_time(e1) / steps


def config_scale(ctx, steps=10, warmup=2):
    """The other named workloads at their full sizes, timed as the headline
    is (plan, one HIP graph per step, inputs resident in HBM): per-step time,
    particle-collisions per second and the step's algorithmic HBM fraction
    (64 B per particle), in FP64 and, where the kinematics allow it, FP32.
    The differentiated workload also times one tangent (forward-mode) step
    and one adjoint (reverse-mode) step through the C ABI."""
    import torch
    from paper_2407_19151_amd import native, runner
    from paper_2407_19151_amd import workloads as W
    f64, f32 = native.MCC_FP64, native.MCC_FP32_KINEMATICS
    cases = [("config1", W.config1, (("fp64", f64), ("fp32", f32))),
             ("config2_n97", lambda: W.config2(method=W.N97), (("fp64", f64), ("fp32", f32))),
             ("config2_ta77", lambda: W.config2(method=W.TA77), (("fp64", f64), ("fp32", f32))),
             ("config4_relativistic", W.config4, (("fp64", f64),)),
             ("config5", W.config5, (("fp64", f64), ("fp32", f32)))]
    out = {}
    for name, make, precs in cases:
        wl = make()
        pcs = wl.particle_collisions_per_step()
        entry = {"workload": wl.name, "cells": wl.n_cells, "particles": wl.n,
                 "particle_collisions_per_step": pcs}
        for pname, prec in precs:
            dw = runner.DeviceWorkload(wl)
            plan = runner.make_plan(ctx, dw, params=runner.params_for(wl, precision=prec),
                                    autotune=False)
            ms, _ = time_plan(plan, steps, warmup)
            plan.close()
            entry[pname] = {"ms_per_step": ms, "particle_collisions_per_s": pcs / (ms * 1e-3),
                            "step_hbm_frac": BYTES_PER_PARTICLE_STEP * wl.n / (ms * 1e-3) / 1e9
                            / HBM_PEAK_GBS}
            del dw
        if name == "config5":
            for pname, prec in (("fp64", f64), ("fp32", f32)):
                dw = runner.DeviceWorkload(wl)
                params = runner.params_for(wl, precision=prec)
                v = torch.stack([dw.vx, dw.vy, dw.vz]).contiguous()
                g = torch.randn(3, wl.n, dtype=torch.float64, device="cuda")
                gl = torch.zeros(1, dtype=torch.float64, device="cuda")
                for k in range(warmup):
                    runner.collide_adjoint(ctx, dw, v, g, k, g_lnl=gl, params=params)
                torch.cuda.synchronize()
                e0, e1 = events()
                e0.record()
                for k in range(steps):
                    runner.collide_adjoint(ctx, dw, v, g, warmup + k, g_lnl=gl, params=params)
                e1.record()
                torch.cuda.synchronize()
                entry[pname]["adjoint_ms_per_step"] = e0.elapsed_time(e1) / steps
                if prec == f64:
                    t = torch.randn(3, wl.n, dtype=torch.float64, device="cuda")
                    for k in range(warmup):
                        runner.collide_sorted_jvp(ctx, dw, t, k, update_primal=False)
                    torch.cuda.synchronize()
                    e0, e1 = events()
                    e0.record()
                    for k in range(steps):
                        runner.collide_sorted_jvp(ctx, dw, t, warmup + k, update_primal=False)
                    e1.record()
                    torch.cuda.synchronize()
                    entry[pname]["tangent_ms_per_step"] = e0.elapsed_time(e1) / steps
                del dw
        assert ctx.device_error() == 0
        out[name] = entry
        log("%s: %s" % (name, {k: round(v["ms_per_step"], 4) for k, v in entry.items()
                               if isinstance(v, dict)}))
        torch.cuda.empty_cache()
    return out


def paper_tests(which, steps, warmup):
    """Step time and throughput of each case of the paper's Test 1, 2 or 3
    (a plan, graph replays)."""
    import torch
    from paper_2407_19151_amd import native, runner
    from paper_2407_19151_amd import workloads as W
    ctx = native.Context(0)
    cases, make = {1: (W.PAPER_T1_CASES, W.paper_test1), 2: (W.PAPER_T2_CASES, W.paper_test2),
                   3: (W.PAPER_T3_CASES, W.paper_test3)}[which]
    for case in sorted(cases):
        wl = make(case)
        corr = int((wl.extra or {}).get("moment_correction", True))
        dw = runner.DeviceWorkload(wl)
        plan = runner.make_plan(ctx, dw, params=runner.params_for(wl, moment_correction=corr),
                                autotune=False)
        ms, _ = time_plan(plan, steps, warmup, first_step=0)
        desc = json.loads(plan.describe())
        plan.close()
        b = [x for x in desc["buckets"] if x["cells"]][0]
        print(json.dumps({"workload": wl.name, "ms_per_step": ms,
                          "particle_collisions_per_s": wl.particle_collisions_per_step() / (ms * 1e-3),
                          "variant": "%dx%d layout %d" % (b["tpc"], b["cap"], b["layout"]),
                          "moment_correction": bool(corr), "steps": steps, "dtype": "f64"}), flush=True)
        del dw
        torch.cuda.empty_cache()


def nxn_bench(steps, warmup):
    """N x N and duplicity pairing against order-N on the same workload (1024
    cells of 256 electrons + 256 ions, three collisions): step time and
    binary pair scatters per second."""
    import torch
    from paper_2407_19151_amd import native, runner
    from paper_2407_19151_amd import workloads as W
    ctx = native.Context(0)
    wl = W.config5()
    names = {0: "order_n", 1: "nxn", 2: "duplicity"}
    for pairing, prec in ((1, native.MCC_FP64), (1, native.MCC_FP32_KINEMATICS),
                          (0, native.MCC_FP64), (0, native.MCC_FP32_KINEMATICS),
                          (2, native.MCC_FP64)):
        dw = runner.DeviceWorkload(wl)
        plan = runner.make_plan(ctx, dw, params=runner.params_for(wl, pairing=pairing,
                                                                  precision=prec),
                                autotune=False)
        ms, _ = time_plan(plan, steps, warmup, first_step=0)
        plan.close()
        runner.collide_sorted(ctx, dw, 0, params=runner.params_for(wl, pairing=pairing,
                                                                   precision=prec))
        pairs = native.read_stats(dw.stats)["pairs"]
        print(json.dumps({"workload": wl.name, "pairing": names[pairing],
                          "dtype": "f32 kinematics" if prec else "f64", "ms_per_step": ms,
                          "pairs_per_step": int(pairs),
                          "pair_scatters_per_s": pairs / (ms * 1e-3), "steps": steps}),
              flush=True)
        del dw
        torch.cuda.empty_cache()


def hard_sphere_bench(steps, warmup):
    """The hard-sphere process (about 5 % collision probability per particle
    and collision) against N97 Coulomb scattering, both FP64, on the
    65,536-cell population: step time, particle-collisions per second, and
    the duration of each size bucket's kernel with its algorithmic HBM rate
    (64 B per particle)."""
    import torch
    from paper_2407_19151_amd import native, runner
    from paper_2407_19151_amd import workloads as W
    ctx = native.Context(0)
    base = W.config3()
    per_bucket_n = bucket_particles(base)
    for wl in (W.hard_sphere(base), base):
        dw = runner.DeviceWorkload(wl)
        plan = runner.make_plan(ctx, dw, params=runner.params_for(wl), autotune=False)
        ms, _ = time_plan(plan, steps, warmup)
        bms = time_buckets(plan, sorted(per_bucket_n), steps)
        plan.close()
        assert ctx.device_error() == 0
        dom = max(bms, key=lambda b: bms[b])
        print(json.dumps({
            "workload": wl.name, "method": "hard_sphere" if wl.method == W.HARD_SPHERE else "n97",
            "dtype": "f64", "ms_per_step": ms,
            "particle_collisions_per_s": wl.particle_collisions_per_step() / (ms * 1e-3),
            "bucket_ms": {str(b): round(v, 4) for b, v in bms.items()},
            "dominant_bucket": dom, "dominant_ms": bms[dom],
            "dominant_frac_of_8TBs": BYTES_PER_PARTICLE_STEP * per_bucket_n[dom]
            / (bms[dom] * 1e-3) / 8e12,
            "steps": steps}), flush=True)
        del dw
        torch.cuda.empty_cache()


def rebin_bench(steps, warmup):
    """mcc_rebin on the 65,536-cell population after a push that moves a
    fraction of the particles to a neighbouring cell (10 % of those jump
    anywhere), against mcc_bin on the same new keys.  Roofline: the
    operation's least HBM traffic, 4 B of new cell id read and 4 B of
    permutation written per particle, plus 64 B when w, vx, vy, vz are moved
    (read and written once)."""
    import numpy as np
    import torch
    from paper_2407_19151_amd import native
    from paper_2407_19151_amd import workloads as W
    ctx = native.Context(0)
    wl = W.config3()
    n = wl.n
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    off = dev(wl.offsets)
    sp = dev(wl.species.astype(np.int32))
    pay = [dev(a) for a in (wl.w, wl.vx, wl.vy, wl.vz)]
    pay_out = [torch.empty_like(t) for t in pay]
    rng = np.random.default_rng(5)
    cell = wl.cells.astype(np.int32)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = events()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    for frac in (0.01, 0.05):
        new = cell.copy()
        mv = rng.uniform(size=n) < frac
        step = np.where(rng.uniform(size=n) < 0.5, -1, 1)
        new[mv] = (cell[mv] + step[mv]) % wl.n_cells
        far = mv & (rng.uniform(size=n) < 0.1)
        new[far] = rng.integers(0, wl.n_cells, size=int(far.sum()))
        cn = dev(new.astype(np.int32))
        t_keys = timed(lambda: ctx.rebin(off, cn, wl.n_cells, wl.n_species))
        t_pay = timed(lambda: ctx.rebin(off, cn, wl.n_cells, wl.n_species, *pay))
        t_out = timed(lambda: ctx.rebin_out(off, cn, wl.n_cells, wl.n_species, *pay, *pay_out))
        t_bin = timed(lambda: ctx.bin(cn, sp, wl.n_cells, wl.n_species))
        assert ctx.device_error() == 0
        print(json.dumps({
            "workload": "65536-cell population (%d particles), %.0f %% moved" % (n, 100 * frac),
            "rebin_ms": t_keys, "rebin_with_payload_ms": t_pay,
            "rebin_out_of_place_ms": t_out, "bin_from_scratch_ms": t_bin,
            "speedup_vs_bin": t_bin / t_keys,
            "roofline": {"bound": "hbm", "unit": "GB/s", "peak": 8000.0,
                         "keys": {"bytes_per_particle": 8, "achieved": 8 * n / t_keys / 1e6,
                                  "frac": 8 * n / t_keys / 1e6 / 8000.0},
                         "with_payload": {"bytes_per_particle": 72,
                                          "achieved": 72 * n / t_pay / 1e6,
                                          "frac": 72 * n / t_pay / 1e6 / 8000.0},
                         "out_of_place": {"bytes_per_particle": 72,
                                          "achieved": 72 * n / t_out / 1e6,
                                          "frac": 72 * n / t_out / 1e6 / 8000.0}},
            "steps": steps}), flush=True)


def paper_test3_curve(total=1_100_000, every=50_000):
    """T3b and T3c (N_e = N_i = 512, w_e = 6 w_i, without and with the
    correction) stepped to equilibrium; one JSON line per sample with the
    species temperatures and the momentum and energy drift."""
    import numpy as np
    import torch
    from paper_2407_19151_amd import native, runner
    from paper_2407_19151_amd import workloads as W
    ctx = native.Context(0)
    for case in ("T3c", "T3b"):
        wl = W.paper_test3(case)
        corr = int(wl.extra["moment_correction"])
        m = wl.mass[wl.species] * wl.w
        v0 = wl.velocities()
        p0 = (m * v0).sum(1)
        e0 = (0.5 * m * (v0 * v0).sum(0)).sum()
        ps = (m * np.linalg.norm(v0, axis=0)).sum()
        dw = runner.DeviceWorkload(wl)
        plan = runner.make_plan(ctx, dw, params=runner.params_for(wl, moment_correction=corr),
                                autotune=False)
        te, ti = W.species_temperatures(wl, v0)
        print(json.dumps({"case": case, "step": 0, "t_fs": 0.0, "T_e": te, "T_i": ti}),
              flush=True)
        t0 = time.perf_counter()
        for k in range(every, total + 1, every):
            plan.run(k - every, every)
            torch.cuda.synchronize()
            v = dw.velocities()
            te, ti = W.species_temperatures(wl, v)
            print(json.dumps({"case": case, "step": k, "t_fs": k * wl.dt * 1e15, "T_e": te,
                              "T_i": ti,
                              "rel_dP": float(np.abs((m * v).sum(1) - p0).max() / ps),
                              "rel_dE": float(abs((0.5 * m * (v * v).sum(0)).sum() - e0) / e0),
                              "wall_s": time.perf_counter() - t0}), flush=True)
        plan.close()
        del dw
        torch.cuda.empty_cache()


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.paper_test3_curve:
        paper_test3_curve()
        return
    if args.nxn:
        nxn_bench(args.steps, args.warmup)
        return
    if args.unsorted:
        from paper_2407_19151_amd import native
        from paper_2407_19151_amd import workloads as W
        print(json.dumps(unsorted_entry(native.Context(0), W.config3(), "fp32", args.steps,
                                        args.warmup)), flush=True)
        return
    if args.configs:
        from paper_2407_19151_amd import native
        print(json.dumps(config_scale(native.Context(0), args.steps, args.warmup)), flush=True)
        return
    if args.rebin:
        rebin_bench(args.steps, args.warmup)
        return
    if args.hard_sphere:
        hard_sphere_bench(args.steps, args.warmup)
        return
    if args.paper_test1 or args.paper_test2 or args.paper_test3:
        paper_tests(1 if args.paper_test1 else 2 if args.paper_test2 else 3, args.steps, args.warmup)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path here (cells shard "
              "by range with no exchange; the design notes describe it)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2407_19151_amd import native, runner
    from paper_2407_19151_amd import workloads as W

    wl = W.config3(n_cells=args.cells)
    log("workload: %d cells, %d particles" % (wl.n_cells, wl.n))
    pcs = wl.particle_collisions_per_step()
    per_bucket_n = bucket_particles(wl)
    ctx = native.Context(0)
    out = {}
    modes = ["fp32", "fp64"] if args.only is None else [args.only]
    tuned_ms = None
    for mode in modes:
        dw = runner.DeviceWorkload(wl)
        prec = native.MCC_FP32_KINEMATICS if mode == "fp32" else native.MCC_FP64
        plan = runner.make_plan(ctx, dw, params=runner.params_for(wl, precision=prec),
                                autotune=args.autotune)
        log("%s plan built" % mode)
        ms, wall = time_plan(plan, args.steps, args.warmup)
        log("%s timed: %.3f ms/step" % (mode, ms))
        desc = json.loads(plan.describe())
        bms = time_buckets(plan, sorted(per_bucket_n), args.steps)
        log("%s per-bucket kernel ms: %s" % (mode, {b: round(v, 4) for b, v in bms.items()}))
        plan.close()
        if mode == modes[0] and not args.autotune and not args.quick:
            tplan = runner.make_plan(ctx, dw, params=runner.params_for(wl, precision=prec),
                                     autotune=True)
            tuned_ms, _ = time_plan(tplan, args.steps, args.warmup)
            tuned_desc = json.loads(tplan.describe())
            tplan.close()
            log("%s autotuned plan: %.3f ms/step" % (mode, tuned_ms))
        assert ctx.device_error() == 0
        gbs = BYTES_PER_PARTICLE_STEP * wl.n / (ms * 1e-3) / 1e9
        out[mode] = dict(ms=ms, wall=wall, gbs=gbs, value=pcs / (ms * 1e-3), plan=desc,
                         bucket_ms=bms)
        del dw
        torch.cuda.empty_cache()
    head_mode = "fp32" if "fp32" in out else "fp64"
    head = out[head_mode]
    # dominant kernel: the bucket kernel with the longest launch
    dom = max(head["bucket_ms"], key=lambda b: head["bucket_ms"][b])
    dom_ms = head["bucket_ms"][dom]
    bd = head["plan"]["buckets"][dom]
    kname = "collide_kernel<%d, %d, %s, false, %d, false, false, 0>" % (
        bd["tpc"], bd["cap"], "float" if head_mode == "fp32" else "double", bd["layout"])
    alg_bytes = BYTES_PER_PARTICLE_STEP * per_bucket_n[dom]
    achieved = alg_bytes / (dom_ms * 1e-3) / 1e9
    traffic = read_traffic()
    valu = read_valu()
    tkey = (head_mode, "%dx%d" % (bd["tpc"], bd["cap"]), "L%d" % bd["layout"])
    res = {
        "metric": "particle-collisions/s per step + HBM roofline fraction, plain FP64 vs FP32+fix",
        "value": head["value"],
        "unit": "particle-collisions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head_mode == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "65536 cells, lognormal(ln 200, 1) counts clipped to [16, 4096], "
                               "electrons + ions (m_i/m_e = 100), N97, moment correction, "
                               "batched HIP-graph step",
                   "cells": wl.n_cells, "particles": wl.n,
                   "particle_collisions_per_step": pcs,
                   "mode": ("fp32 kinematics + fp64 correction" if head_mode == "fp32"
                            else "fp64"),
                   "variants": "autotuned" if args.autotune else "built-in table"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (traffic.get(tkey) if traffic else None),
                     "kernel": kname, "bucket_max_cell": BUCKET_CAP[dom],
                     "bucket_particles": per_bucket_n[dom], "launch_ms": dom_ms,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "bytes_per_particle_step": BYTES_PER_PARTICLE_STEP,
                     # the same on the 56 B the sorted kernel itself moves
                     # (w in, v in and out: the ids are implied by the offsets)
                     "frac_bytes_moved": achieved * BYTES_MOVED / BYTES_PER_PARTICLE_STEP
                     / HBM_PEAK_GBS},
        "valu_roofline": (
            {"bound": "valu", "achieved": valu[tkey][0] / (dom_ms * 1e-3),
             "peak": VALU_PEAK_WINST, "unit": "wave-instructions/s",
             "frac": valu[tkey][0] / (dom_ms * 1e-3) / VALU_PEAK_WINST,
             "valu_per_launch": valu[tkey][0]}
            if valu and tkey in valu else None),
        "step_hbm_frac": head["gbs"] / HBM_PEAK_GBS,
        "bucket_launch_ms": {str(BUCKET_CAP[b]): v for b, v in head["bucket_ms"].items()},
    }
    if "fp64" in out and "fp32" in out:
        o64 = out["fp64"]
        res["plain_fp64"] = {"value": o64["value"], "ms_per_step": o64["ms"],
                             "step_hbm_frac": o64["gbs"] / HBM_PEAK_GBS}
        if valu:
            # FP64 operations of the plain FP64 step (every bucket kernel, from
            # the counters) over its step time, against the FP64 vector peak
            f64 = 0.0
            for b, bdsc in enumerate(o64["plan"]["buckets"]):
                if bdsc["cells"] == 0:
                    continue
                k = ("fp64", "%dx%d" % (bdsc["tpc"], bdsc["cap"]), "L%d" % bdsc["layout"])
                f64 += valu[k][1] if k in valu else float("nan")
            tf = f64 / (o64["ms"] * 1e-3) / 1e12
            res["plain_fp64"]["fp64_valu"] = {"achieved_tflops": tf, "peak": FP64_PEAK_TFLOPS,
                                              "frac": tf / FP64_PEAK_TFLOPS}
    if tuned_ms is not None:
        res["autotuned_plan"] = {"mode": modes[0], "ms_per_step": tuned_ms,
                                 "value": pcs / (tuned_ms * 1e-3), "plan": tuned_desc}
    if not args.quick:
        log("per-call sorted step (no plan)")
        pc_ms = per_call_sorted(ctx, wl, head_mode, args.steps, args.warmup)
        res["per_call_sorted"] = {"mode": head_mode, "ms_per_step": pc_ms,
                                  "value": pcs / (pc_ms * 1e-3)}
        log("unsorted entry and binning")
        res["unsorted_entry"] = dict(unsorted_entry(ctx, wl, head_mode, args.steps, args.warmup),
                                     mode=head_mode)
        log("copy ceiling")
        res["copy_ceiling_gbs"] = copy_ceiling()
        log("relaxation-rate error against the oracle")
        res["relaxation_vs_oracle"] = relaxation_rate_error(ctx)
        log("the other workloads at full size")
        res["config_scale"] = config_scale(ctx)
    res["plans"] = {m: o["plan"] for m, o in out.items()}
    if not args.no_cpu:
        log("timing the CPU oracle on a sample")
        res["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
