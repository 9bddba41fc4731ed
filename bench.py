#!/usr/bin/env python3
"""Benchmark of the SPH Runge-Kutta stage on one MI355X.

Workload: the 2+1D boost-invariant viscous BSQ event of 40,000 particles
(200 x 200 lattice at 0.08 fm, h = 0.24 fm, 150 seeded Gaussian hot spots,
rhoB = 0.05 s, rhoQ = 0.02 s, eta/s = 0.08, zeta/s Gaussian peak 0.02 at
0.17 GeV, 64 x 32^3 synthetic massless-gas EoS table, Heun steps of
dt = 0.005 fm/c from tau = 0.6 fm/c).  One step is one pass of the whole hot
path: binning, both Heun stages (density sums, EoS inversion, gradient sums,
local equations of motion, update).  Inputs are resident on the GPU before
the timed region; the event is re-initialised (outside the timed region)
after the warm-up.

Reported: particle-steps/s for FP32-Kahan pair sums (value) and FP64; the
roofline of the dominant kernel from HIP-event timings on the simulation's
stream; the FP64 CPU oracle timed on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6      # vector FP64: 256 CU x 128 flop/clk x 2.4 GHz
FP32_PEAK_TFLOPS = 157.3     # vector FP32, published figure: needs packed (two-wide) FP32 instructions
# The build disables packed FP32, so the vector ALU peak of these kernels is
# one wave64 instruction per clock per CU (4 SIMDs x 16 lanes), i.e. 2 flop x
# 64 lanes x 256 CU x 2.4 GHz for FP32 FMA, the same as FP64.
VALU_PEAK_TFLOPS = 78.6
VALU_ISSUE_PER_S = 256 * 2.4e9   # wave64 vector instructions per second, whole chip

METRIC = "SPH particle-steps/s (FP64 vs FP32-Kahan) + p50/p99 event latency, 1 GPU"

# binning skin of the 2+1D event, in units of h (a performance setting: a
# larger skin rebins less often and keeps the cached neighbour rows longer,
# at the price of more candidates; measured best between 0.2 h and 0.3 h)
HEADLINE_SKIN_H = 0.25


GROUPS = ["binning", "density_sums", "eos_inversion", "gradient_sums", "eom_update"]

# sources that the stage kernels are compiled from; the measured HBM traffic of
# a kernel is reported only while these are unchanged since the counters were read
KERNEL_SOURCES = ["common.h", "sph_device.h", "pair_device.h", "eos_device.h", "eom_device.h", "stage.hip"]
# counter summaries per workload key: profiles/<group>_<key>_traffic.txt
WL_2D, WL_3D = "lumpy2d_40k", "lumpy3d_1p2M"
def traffic_file(group, key=WL_2D):
    return f"{group}_{key}_traffic.txt"
# kernel-name prefixes of the groups in the counter output
GROUP_KERNELS = {"density_sums": "void ccake::k_density<", "eos_inversion": "void ccake::k_eos<",
                 "gradient_sums": "void ccake::k_grad<", "eom_update": "void ccake::k_eom<"}


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2511_22852_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_summary(group, key=WL_2D):
    """The committed counter summary of the group's kernel on a workload
    (key: value), or None when there is none or the kernel sources changed
    since."""
    path = os.path.join(ROOT, "profiles", traffic_file(group, key)) if group in GROUP_KERNELS else None
    if not path or not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_digest") != kernel_source_digest():
        return None
    return kv


def measured_traffic(group, key=WL_2D):
    """HBM bytes per launch of the group's kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE per dispatch, each divided by what the
    counter reads per byte of a plain device copy), or None."""
    kv = counter_summary(group, key)
    if kv is None:
        return None
    fetch = float(kv["fetch_kib_per_dispatch"]) * 1024 / float(kv["copy_fetch_factor"])
    write = float(kv["write_kib_per_dispatch"]) * 1024 / float(kv["copy_write_factor"])
    return fetch + write


def summarize_counters(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_mib, out_dir, command,
                       sq_dir=None, key=WL_2D):
    """Write one traffic file per kernel group from rocprofv3 --pmc output:
    mean FETCH_SIZE and WRITE_SIZE (KiB) per dispatch of the group's kernel,
    and the factors that the same counters read per KiB actually moved by a
    plain copy of copy_mib MiB (read copy_mib, write copy_mib).  With sq_dir
    (a run with SQ_INSTS_VALU and SQ_WAVES), also the vector-ALU instructions
    (per wave, summed over waves) per dispatch."""
    import csv
    import glob

    def means(d, counter):
        acc = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r.get("Counter_Name") == counter:
                    acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}

    kib = copy_mib * 1024.0
    cf = [v for k, v in means(copy_fetch_dir, "FETCH_SIZE").items() if "k_copy" in k]
    cw = [v for k, v in means(copy_write_dir, "WRITE_SIZE").items() if "k_copy" in k]
    if len(cf) != 1 or len(cw) != 1:
        raise SystemExit("copy calibration dispatch not found")
    f_factor, w_factor = cf[0][0] / kib, cw[0][0] / kib
    fetch, write = means(fetch_dir, "FETCH_SIZE"), means(write_dir, "WRITE_SIZE")
    valu = means(sq_dir, "SQ_INSTS_VALU") if sq_dir else {}
    digest = kernel_source_digest()
    for g, prefix in GROUP_KERNELS.items():
        fk = [(k, v) for k, v in fetch.items() if k.startswith(prefix)]
        wk = [(k, v) for k, v in write.items() if k.startswith(prefix)]
        if len(fk) != 1 or len(wk) != 1:
            raise SystemExit(f"{g}: expected one kernel instance, found {[k for k, _ in fk]}")
        (kname, (fm, fn)), (_, (wm, wn)) = fk[0], wk[0]
        path = os.path.join(out_dir, traffic_file(g, key))
        what = ("40,000-particle 2+1D" if key == WL_2D else "1,228,800-particle 3+1D")
        with open(path, "w") as fh:
            fh.write(f"# HBM traffic of {kname.split('(')[0]} on the {what} viscous BSQ lumpy\n"
                     f"# event (mixed precision), from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs of the\n"
                     f"# native driver; KiB per dispatch (mean over {fn} and {wn} dispatches), scaled by what\n"
                     f"# the counters read per KiB of a {copy_mib} MiB device copy.  Commands:\n")
            for line in command.strip().splitlines():
                fh.write(f"#   {line}\n")
            fh.write(f"kernel: {kname.split('(')[0]}\n")
            fh.write(f"fetch_kib_per_dispatch: {fm:.1f}\nwrite_kib_per_dispatch: {wm:.1f}\n")
            fh.write(f"copy_fetch_factor: {f_factor:.4f}\ncopy_write_factor: {w_factor:.4f}\n")
            fh.write(f"hbm_bytes_per_dispatch: {fm * 1024 / f_factor + wm * 1024 / w_factor:.0f}\n")
            vk = [v for k, v in valu.items() if k.startswith(prefix)]
            if len(vk) == 1:
                fh.write(f"valu_wave_instructions_per_dispatch: {vk[0][0]:.0f}\n")
            fh.write(f"source_digest: {digest}\n")
        print(path)


def algorithmic_model(dim, viscous, ncharge, mixed, smoothed=True):
    """Per kernel of one Heun stage: compulsory HBM bytes per particle (each
    array the kernel must touch, read or written once; neighbour data reused
    on chip is not counted) and flops per accepted neighbour pair.  Bytes:
    density sums read positions (and S, N for smoothed densities) and the
    cell index, and write the six sums; the EoS pass reads the sums, the state
    it needs and the warm start, and writes thermodynamics, the neighbour
    record and the new warm start; the gradient pass reads positions, the
    record and sigma*, and writes its sums; the update reads the sums, the
    thermodynamics and two state copies and writes one.  The compensation
    flops of the FP32 (Kahan) sums are overhead of the precision pattern, not
    work of the method: they are kept apart (comp_flops) and left out of the
    roofline figure, like the pair test of rejected candidates."""
    nP = (6 if dim == 3 else 4) if viscous else 0
    state = 2 * dim + 1 + ncharge + (1 + nP if viscous else 0)
    rec = 1 + (dim * dim if viscous else 0) + 2 * dim
    recb = 4 if mixed else 8
    nth = 6 + (5 if viscous else 0)
    ngs = dim + dim * dim + 1
    dens_in = dim + ((1 + ncharge) if smoothed else 0)
    # compensated (Kahan) additions of the FP32 form: 3 more flops per term
    kd = 3 * (1 + ((1 + ncharge) if smoothed else 0)) if mixed else 0
    kg = 3 * (dim + dim * dim + 1) if mixed else 0
    return {
        "density_sums": dict(bytes=8 * dens_in + 4 + 8 * 6,
                             pair_flops=5 + 1 + 1 + 7 + 1 + (2 * (1 + ncharge) if smoothed else 0),
                             comp_flops=kd),
        "eos_inversion": dict(bytes=8 * 5 + 8 * (state - dim) + 8 * 8 * 2 + 8 * nth + recb * rec, pair_flops=0,
                              comp_flops=0),
        "gradient_sums": dict(bytes=8 * dim + 4 + recb * rec + 8 + 8 * ngs,
                              pair_flops=5 + 1 + 1 + 5 + 1 + dim + 1 + 2 * dim + 4 * dim * dim + 3 * dim
                              + ((4 * dim * dim + dim) if viscous else 0),
                              comp_flops=kg),
        "eom_update": dict(bytes=8 * ngs + 8 * nth + 8 * state * 3, pair_flops=0, comp_flops=0),
    }


def kernel_roofline(model, name, n, nnb, ms, launches, k, traffic_key=WL_2D):
    """Roofline of one stage kernel: algorithmic bytes (n particles x the
    model's bytes per particle) and flops (accepted pairs x flops per pair)
    per launch against the launch's average duration from the dispatch
    events; the binding roof is whichever of bytes / 8 TB/s and flops / the
    vector-ALU peak takes longer."""
    avg_s = ms[k] / launches[k] / 1e3
    nbytes = n * model[name]["bytes"]
    flops = n * nnb * model[name]["pair_flops"]
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    t_alu = flops / (VALU_PEAK_TFLOPS * 1e12)
    if t_hbm >= t_alu:
        r = dict(bound="hbm", achieved=nbytes / avg_s / 1e9, peak=HBM_PEAK_GBS, unit="GB/s")
    else:
        r = dict(bound="alu", achieved=flops / avg_s / 1e12, peak=VALU_PEAK_TFLOPS, unit="TFLOP/s")
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = measured_traffic(name, traffic_key)
    r["kernel"] = name
    r["avg_launch_us"] = avg_s * 1e6
    r["algorithmic_bytes_per_launch"] = nbytes
    r["algorithmic_flops_per_launch"] = flops
    r["compensation_flops_per_launch"] = n * nnb * model[name]["comp_flops"]
    # issued vector-ALU instructions (counters) against the issue rate
    cs = counter_summary(name, traffic_key)
    if cs and "valu_wave_instructions_per_dispatch" in cs:
        r["valu_issue_frac"] = float(cs["valu_wave_instructions_per_dispatch"]) / (avg_s * VALU_ISSUE_PER_S)
    return r


def rooflines(model, n, nnb, ms, launches, traffic_key=WL_2D):
    """(the dominant stage kernel's roofline, every stage kernel's)."""
    k = max(range(1, len(GROUPS)), key=lambda i: ms[i])
    roof = kernel_roofline(model, GROUPS[k], n, nnb, ms, launches, k, traffic_key)
    roof_all = {GROUPS[i]: {key: v for key, v in kernel_roofline(model, GROUPS[i], n, nnb, ms, launches, i,
                                                                 traffic_key).items() if key != "kernel"}
                for i in range(1, len(GROUPS))}
    return roof, roof_all


def run_gpu(B, I, w, eos, precision, steps, warmup, diffusion=False):
    import torch
    cfg = B.config(dim=2, hyperbolic=True, viscous=True, precision=precision, ncharge=3, h=w.h,
                   eta_over_s=0.08, zeta_peak=0.02, zeta_Tpeak_GeV=0.17, zeta_width_GeV=0.02,
                   diffusion=diffusion, skin=HEADLINE_SKIN_H * w.h)
    sim = B.Sim(cfg, eos, w.n)
    sim.init_particles(w.t0, w.xi, w.u, w.dens_kind, w.dens)
    if warmup:
        sim.step(w.dt, warmup)
        sim.check()
    sim.init_particles(w.t0, w.xi, w.u, w.dens_kind, w.dens)
    nnb = float(sim.read(B.AUX_NNB).mean())
    torch.cuda.synchronize()
    sim.synchronize()
    t0 = time.perf_counter()
    sim.step(w.dt, steps)
    sim.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sim.check()
    tot, cnt = sim.totals()
    # kernel durations: the same steps again, kernels bracketed by HIP events
    sim.init_particles(w.t0, w.xi, w.u, w.dens_kind, w.dens)
    sim.set_profiling(True)
    sim.step(w.dt, steps)
    ms, launches = sim.kernel_times()
    sim.set_profiling(False)
    sim.check()
    nnb_win = window_neighbours(B, w, sim, steps)
    sim.close()
    return dict(elapsed=elapsed, nnb=nnb, nnb_window=nnb_win, ms=ms, launches=launches, totals=tot.tolist(),
                backup=cnt.backup, newton_iters=cnt.newton_iters, newton_hist=list(cnt.newton_hist))


def window_neighbours(B, w, sim, steps, samples=10):
    """Mean neighbour count over the timed window (the flops of the pair
    kernels scale with it, and it grows as the flow compresses parts of the
    event): the same steps once more, sampled at the start of each of
    `samples` equal chunks."""
    sim.init_particles(w.t0, w.xi, w.u, w.dens_kind, w.dens)
    samples = max(1, min(samples, steps))
    vals, done = [], 0
    for i in range(samples):
        vals.append(float(sim.read(B.AUX_NNB).mean()))
        k = (steps * (i + 1)) // samples - done
        if k > 0:
            sim.step(w.dt, k)
            done += k
    sim.check()
    return sum(vals) / len(vals)


def run_3d(B, w, eos, precision, steps, warmup, sources=None):
    """Throughput of a 3+1D hyperbolic viscous BSQ event (same transport and
    EoS as the headline run): warm-up steps, re-initialisation, then timed
    steps of the whole path."""
    import torch
    cfg = B.config(dim=3, hyperbolic=True, viscous=True, precision=precision, ncharge=3, h=w.h,
                   eta_over_s=0.08, zeta_peak=0.02, zeta_Tpeak_GeV=0.17, zeta_width_GeV=0.02)
    sim = B.Sim(cfg, eos, w.n)
    if sources:
        sim.set_sources(sources)
    sim.init_particles(w.t0, w.xi, w.u, w.dens_kind, w.dens)
    if warmup:
        sim.step(w.dt, warmup)
        sim.check()
    sim.init_particles(w.t0, w.xi, w.u, w.dens_kind, w.dens)
    nnb = float(sim.read(B.AUX_NNB).mean())
    torch.cuda.synchronize()
    sim.synchronize()
    t0 = time.perf_counter()
    sim.step(w.dt, steps)
    sim.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sim.check()
    # kernel durations: the same steps again, kernels bracketed by HIP events
    sim.init_particles(w.t0, w.xi, w.u, w.dens_kind, w.dens)
    sim.set_profiling(True)
    sim.step(w.dt, steps)
    ms, launches = sim.kernel_times()
    sim.set_profiling(False)
    sim.check()
    nnb_win = window_neighbours(B, w, sim, steps, samples=5)
    sim.close()
    model = algorithmic_model(3, True, 3, precision == B.MIXED)
    roof, roof_all = rooflines(model, w.n, nnb_win, ms, launches, WL_3D)
    return dict(particle_steps_per_s=w.n * steps / elapsed, ms_per_step=elapsed / steps * 1e3, steps=steps,
                particles=w.n, mean_neighbours=nnb, mean_neighbours_window=nnb_win,
                tau_window_fm=[w.t0, w.t0 + steps * w.dt],
                kernel_ms_per_step=[m / steps for m in ms], roofline=roof, roofline_by_kernel=roof_all)


def run_serving(B, I, eos, events, steps, precision, rate=None, max_particles=4_000_000, max_events=256):
    """Continuous batching of the given events through the server.  rate None:
    all submitted at once (capacity); otherwise Poisson arrivals at that rate
    (events/s), submitted in real time.  max_events = 1 runs the events one
    after another on the same arrival trace (the sequential baseline, queueing
    included).  Returns latencies and throughput."""
    cfg = B.config(dim=2, hyperbolic=True, viscous=True, precision=precision, ncharge=3, h=events[0].h,
                   eta_over_s=0.08, zeta_peak=0.02, zeta_Tpeak_GeV=0.17, zeta_width_GeV=0.02,
                   skin=HEADLINE_SKIN_H * events[0].h)
    srv = B.Server(cfg, eos, budget_bytes=64 << 30, max_particles=max_particles, max_events=max_events,
                   dt=events[0].dt)
    arrivals = [0.0] * len(events) if rate is None else list(I.poisson_arrivals(len(events), rate))
    results = []
    start = time.perf_counter()
    for k, (w, ta) in enumerate(zip(events, arrivals)):
        delay = ta - (time.perf_counter() - start)
        if delay > 0:
            time.sleep(delay)
        srv.submit(w.t0, w.t0 + steps * w.dt, w.xi, w.u, w.dens_kind, w.dens, tag=k)
        results += srv.poll(256)
    srv.drain()
    results += srv.poll(1024)
    st = srv.stats()
    srv.close()
    # an event whose evolution fails (sticky status: non-finite update, EoS
    # without a root) is still stepped to its end time and returned with
    # that status; it is reported here, and its latency counts like any other
    failed = [dict(tag=int(r["tag"]), status=int(r["status"])) for r in results if r["status"] != 0]
    lat = sorted(r["t_finish"] - r["t_submit"] for r in results)
    first = min(r["t_submit"] for r in results)
    last = max(r["t_finish"] for r in results)
    span = last - first
    import numpy as np
    return dict(events=len(results), makespan_s=span, events_per_s=len(results) / span,
                particle_steps_per_s=st["particle_steps"] / span,
                p50_latency_s=float(np.percentile(lat, 50)), p99_latency_s=float(np.percentile(lat, 99)),
                mean_resident_particles=st["particle_steps"] / max(st["steps"], 1), failed_events=failed)


def cpu_baseline_run(I, w, min_seconds):
    """The FP64 oracle on the same event, Heun steps from the initial state
    until at least min_seconds of wall time; OpenMP over particles."""
    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    cols, lo, hi = I.massless_gas_table()
    prm = O.params(dim=2, hyperbolic=True, viscous=True, ncharge=3, h=w.h, eta_over_s=0.08,
                   zeta_peak=0.02, zeta_Tpeak_GeV=0.17, zeta_width_GeV=0.02, use_cells=1, nthreads=threads)
    eos = O.eos_table(cols, lo, hi)
    y = O.init(prm, eos, w.t0, w.xi, w.u, w.dens_kind, w.dens)
    t = w.t0
    steps = 0
    t0 = time.perf_counter()
    while True:
        y, _, _ = O.heun_step(prm, eos, t, w.dt, y)
        t += w.dt
        steps += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    el = time.perf_counter() - t0
    return dict(value=w.n * steps / el, unit="particle-steps/s", cores=threads, kind="oracle",
                sample=f"{w.n}-particle lumpy viscous BSQ event, {steps} FP64 Heun steps from the initial "
                       f"state in {el:.1f} s (uniform-grid neighbour search, OpenMP over particles)")


def copy_calibration(mib):
    """One device-to-device copy of a known size: the HBM byte counters of this
    dispatch (read mib MiB, write mib MiB) calibrate those of the SPH kernels."""
    import torch
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n}))


def write_inputs(path, three_d=False):
    """The headline workload (or the 1.2 M-particle 3+1D event), mixed
    precision, in the native driver's file format (see
    paper_2511_22852_amd/csrc/ccake_bench.cpp)."""
    import struct
    import numpy as np
    from paper_2511_22852_amd import binding as B
    from paper_2511_22852_amd import inputs as I
    w = I.lumpy_3d_workload() if three_d else I.lumpy_2d_workload()
    cols, lo, hi = I.massless_gas_table()
    cfg = B.config(dim=3 if three_d else 2, hyperbolic=True, viscous=True, precision=B.MIXED, ncharge=3, h=w.h,
                   eta_over_s=0.08, zeta_peak=0.02, zeta_Tpeak_GeV=0.17, zeta_width_GeV=0.02,
                   skin=None if three_d else HEADLINE_SKIN_H * w.h)
    with open(path, "wb") as f:
        f.write(b"CCAKEBN1")
        f.write(bytes(cfg))
        f.write(struct.pack("<qddii", w.n, w.t0, w.dt, w.dens_kind, 0))
        f.write(struct.pack("<4i", *cols.shape[1:]))
        f.write(np.asarray(lo, dtype="<f8").tobytes() + np.asarray(hi, dtype="<f8").tobytes())
        for a in (cols, w.xi, w.u, w.dens):
            f.write(np.ascontiguousarray(a, dtype="<f8").tobytes())
    print(json.dumps({"workload_file": path, "particles": w.n}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1480, help="timed Heun steps (1480 = tau 0.6 -> 8 fm/c)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-events", type=int, default=256, help="serving load: events (0 = skip)")
    ap.add_argument("--no-c1b", action="store_true",
                    help="skip the event with ten times smaller charge fractions (rhoB = 0.005 s, rhoQ = 0.002 s)")
    ap.add_argument("--serve-steps", type=int, default=1480,
                    help="Heun steps per served event (1480 = tau 0.6 -> 8 fm/c)")
    ap.add_argument("--steps-3d", type=int, default=10,
                    help="timed steps of each 3+1D configuration (0 = skip them)")
    ap.add_argument("--no-offline", action="store_true", help="skip the offline-inverter run of the event")
    ap.add_argument("--no-diffusion", action="store_true", help="skip the BSQ-diffusion run of the event")
    ap.add_argument("--only-3d", action="store_true",
                    help="only time the 1.2 M-particle 3+1D event in mixed precision (profiling runs)")
    ap.add_argument("--precision", choices=["both", "mixed", "fp64"], default="both",
                    help="which precisions to run (counter-collection passes use one)")
    ap.add_argument("--write-inputs", metavar="PATH",
                    help="only write the headline workload (with --only-3d: the 1.2 M-particle 3+1D "
                         "event), mixed precision, for the native driver paper_2511_22852_amd/ccake_bench "
                         "and exit")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                    help="FETCH WRITE COPY_FETCH COPY_WRITE MIB [SQ]: only write profiles/*_traffic.txt from "
                         "rocprofv3 --pmc output directories of the native driver (FETCH_SIZE, WRITE_SIZE), of "
                         "its --copy MIB calibration and optionally of an SQ_INSTS_VALU run, and exit")
    ap.add_argument("--counter-key", default=WL_2D, choices=[WL_2D, WL_3D],
                    help="with --summarize-counters: the workload the counters were read on")
    ap.add_argument("--counter-command", default="",
                    help="with --summarize-counters: the commands that produced the counters (recorded)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run one device-to-device copy of MIB MiB (reference kernel for the HBM "
                         "byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU decomposition is a design "
              "note, not a measured path.", file=sys.stderr)
        sys.exit(2)
    if args.summarize_counters:
        if len(args.summarize_counters) not in (5, 6):
            ap.error("--summarize-counters takes FETCH WRITE COPY_FETCH COPY_WRITE MIB [SQ]")
        fd, wd, cfd, cwd, mib = args.summarize_counters[:5]
        sq = args.summarize_counters[5] if len(args.summarize_counters) == 6 else None
        summarize_counters(fd, wd, cfd, cwd, int(mib), os.path.join(ROOT, "profiles"), args.counter_command, sq,
                           key=args.counter_key)
        return
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.write_inputs:
        write_inputs(args.write_inputs, args.only_3d)
        return

    from paper_2511_22852_amd import binding as B
    from paper_2511_22852_amd import inputs as I

    cols, lo, hi = I.massless_gas_table()
    eos = B.Eos.table(cols, lo, hi)
    if args.only_3d:
        r = run_3d(B, I.lumpy_3d_workload(), eos, B.MIXED, args.steps_3d, 2)
        print(json.dumps({"lumpy_3d_viscous_bsq_1.2M_mixed": r}))
        return
    w = I.lumpy_2d_workload()
    res = {}
    for name, prec in (("fp64", B.FP64), ("mixed", B.MIXED)):
        if args.precision not in ("both", name):
            continue
        res[name] = run_gpu(B, I, w, eos, prec, args.steps, args.warmup)
        print(f"[bench] {name}: {args.steps} steps in {res[name]['elapsed']:.3f} s", file=sys.stderr, flush=True)
    if args.precision != "both":
        print(json.dumps({k: dict(ms_per_step=v["elapsed"] / args.steps * 1e3) for k, v in res.items()}))
        return

    head = res["mixed"]
    value = w.n * args.steps / head["elapsed"]
    value64 = w.n * args.steps / res["fp64"]["elapsed"]
    model = algorithmic_model(2, True, 3, True)

    # roofline of each stage kernel of the headline (mixed) run; the
    # dominant one (largest time) is the reported roofline
    roof, roof_all = rooflines(model, w.n, head["nnb_window"], head["ms"], head["launches"])

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["elapsed"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (Kahan) pair sums, f64 state/EoS/update",
        "data": "synthetic",
        "config": {"workload": "lumpy_2d_viscous_bsq_40k", "particles": w.n, "h_fm": w.h, "dt_fm": w.dt,
                   "tau0_fm": w.t0, "eos": "massless-gas table 64x32x32x32 + analytic backup",
                   "precision": "mixed", "mean_neighbours": head["nnb"],
                   "mean_neighbours_window": head["nnb_window"], "skin_h": HEADLINE_SKIN_H,
                   "tau_window_fm": [w.t0, w.t0 + args.steps * w.dt]},
        "fp64": {"value": value64, "ms_per_step": res["fp64"]["elapsed"] / args.steps * 1e3},
        "mixed_over_fp64": value / value64,
        "kernel_ms_per_step": {"mixed": [m / args.steps for m in head["ms"]],
                               "fp64": [m / args.steps for m in res["fp64"]["ms"]],
                               "groups": GROUPS},
        # counters of one evaluation at the final state (every particle inverted once)
        "eos_backup_fraction_final_state": head["backup"] / w.n,
        "eos_mean_newton_iterations_final_state": head["newton_iters"] / w.n,
        "eos_newton_iteration_histogram_final_state": head["newton_hist"],
        "roofline": roof,
        "roofline_by_kernel": roof_all,
    }
    if not args.no_offline:
        # the offline inverter (the paper's GPU path) on the same event: the
        # (s, n) inversions of the stages interpolate a table on a grid in s
        # (evenly spaced inside decades) and n_q / s
        grid = dict(decade_lo=-2, decade_hi=3, per_decade=36, nx=(11, 7, 9), x_lo=(0.0, -0.03, -0.02),
                    x_hi=(0.1, 0.03, 0.06))
        eos_off = B.Eos.table(cols, lo, hi)
        t0 = time.perf_counter()
        eos_off.build_inverted(3, **grid)
        build_s = time.perf_counter() - t0
        r = run_gpu(B, I, w, eos_off, B.MIXED, args.steps, args.warmup)
        out["offline_eos_mixed"] = {
            "value": w.n * args.steps / r["elapsed"], "ms_per_step": r["elapsed"] / args.steps * 1e3,
            "eos_inversion_ms_per_step": r["ms"][2] / args.steps,
            "online_eos_inversion_ms_per_step": head["ms"][2] / args.steps,
            "table": f"s: 10^-2..10^3 fm^-3, {grid['per_decade']} per decade; n/s (B, S, Q): {grid['nx']} nodes",
            "build_seconds": build_s,
            "eos_mean_newton_iterations_final_state": r["newton_iters"] / w.n,
        }
        print(f"[bench] offline EoS: {out['offline_eos_mixed']['ms_per_step']:.4f} ms/step", file=sys.stderr,
              flush=True)
        eos_off.close()
    if not args.no_diffusion:
        # the same event with BSQ charge diffusion (the paper's full kappa/T^2
        # matrix, tau_J = 0.2/T): currents in the state, their pair sums and
        # relaxation in every stage
        try:
            r = run_gpu(B, I, w, eos, B.MIXED, args.steps, args.warmup, diffusion=True)
            out["bsq_diffusion_mixed"] = {
                "value": w.n * args.steps / r["elapsed"], "ms_per_step": r["elapsed"] / args.steps * 1e3,
                "kernel_ms_per_step": [m / args.steps for m in r["ms"]],
                "kappa_over_T2": "paper's full BSQ matrix", "tauJ": "0.2/T",
            }
            print(f"[bench] BSQ diffusion: {out['bsq_diffusion_mixed']['ms_per_step']:.4f} ms/step", file=sys.stderr,
                  flush=True)
        except B.CcakeError as err:
            out["bsq_diffusion_mixed"] = {"error": str(err)}
    if not args.no_c1b:
        # the same event with rhoB = 0.005 s, rhoQ = 0.002 s (mu_B / T about
        # 0.47): the table answers nearly every inversion
        w1b = I.lumpy_2d_workload(rhoB=0.005, rhoQ=0.002)
        c1b = {}
        for name, prec in (("mixed", B.MIXED), ("fp64", B.FP64)):
            r = run_gpu(B, I, w1b, eos, prec, args.steps, args.warmup)
            c1b[name] = {"value": w1b.n * args.steps / r["elapsed"], "ms_per_step": r["elapsed"] / args.steps * 1e3,
                         "kernel_ms_per_step": [m / args.steps for m in r["ms"]],
                         "eos_backup_fraction_final_state": r["backup"] / w1b.n,
                         "eos_mean_newton_iterations_final_state": r["newton_iters"] / w1b.n}
            print(f"[bench] c1b {name}: {c1b[name]['ms_per_step']:.4f} ms/step", file=sys.stderr, flush=True)
        out["lumpy_2d_viscous_bsq_40k_low_charge"] = dict(
            workload="the headline event with rhoB = 0.005 s, rhoQ = 0.002 s", **c1b)
    if args.steps_3d > 0:
        w2 = I.lumpy_3d_workload()
        other = {}
        for name, prec in (("fp64", B.FP64), ("mixed", B.MIXED)):
            other[f"lumpy_3d_viscous_bsq_1.2M_{name}"] = run_3d(B, w2, eos, prec, args.steps_3d, 2)
            print(f"[bench] 3D 1.2M {name}: {other[f'lumpy_3d_viscous_bsq_1.2M_{name}']['ms_per_step']:.2f} ms/step",
                  file=sys.stderr, flush=True)
        del w2
        w4 = I.lumpy_3d_source_workload()
        other["lumpy_3d_viscous_bsq_4M_jets_mixed"] = run_3d(B, w4, eos, B.MIXED, args.steps_3d, 2,
                                                             sources=I.jet_sources())
        print(f"[bench] 3D 4M jets: {other['lumpy_3d_viscous_bsq_4M_jets_mixed']['ms_per_step']:.2f} ms/step",
              file=sys.stderr, flush=True)
        out["other_configs"] = other
    if args.serve_events > 0:
        import numpy as np
        specs = I.serving_events(args.serve_events)
        events = [I.serving_event(s) for s in specs]
        steps = args.serve_steps
        # capacity from a burst of the first events submitted together, as
        # particle-steps/s; the arrival rate is 70% of it for the whole set
        burst = events[:min(len(events), 24)]
        cap = run_serving(B, I, eos, burst, steps, B.MIXED)
        mean_n = float(np.mean([e.n for e in events]))
        rate = 0.7 * cap["particle_steps_per_s"] / (mean_n * steps)
        print(f"[bench] serving: capacity {cap['particle_steps_per_s']:.3e} particle-steps/s, rate {rate:.2f} ev/s",
              file=sys.stderr, flush=True)
        load = run_serving(B, I, eos, events, steps, B.MIXED, rate=rate)
        print(f"[bench] serving: p50 {load['p50_latency_s']:.3f} s, p99 {load['p99_latency_s']:.3f} s, "
              f"failed events {load['failed_events']}", file=sys.stderr, flush=True)
        seq = run_serving(B, I, eos, events, steps, B.FP64, rate=rate, max_events=1)
        print(f"[bench] FP64 sequential: p50 {seq['p50_latency_s']:.3f} s, p99 {seq['p99_latency_s']:.3f} s, "
              f"failed events {seq['failed_events']}", file=sys.stderr, flush=True)
        out["serving"] = {
            "workload": f"{len(events)} lumpy viscous BSQ events, N ~ U[5000, 80000] (total "
                        f"{sum(e.n for e in events)} particles), {steps} Heun steps each "
                        f"(tau {events[0].t0:g} -> {events[0].t0 + steps * events[0].dt:g} fm/c), mixed precision, "
                        f"Poisson arrivals at 70% of the measured capacity",
            "capacity_particle_steps_per_s": cap["particle_steps_per_s"],
            "capacity_burst_events": len(burst),
            "poisson_rate_events_per_s": rate,
            "events_per_s": load["events_per_s"],
            "particle_steps_per_s": load["particle_steps_per_s"],
            "p50_latency_s": load["p50_latency_s"],
            "p99_latency_s": load["p99_latency_s"],
            "mean_resident_particles": load["mean_resident_particles"],
            "capacity_failed_events": cap["failed_events"],
            "failed_events": load["failed_events"],
            "failed_events_note": "events (tag = index in the set) returned with a non-zero status (3: a "
                                  "non-finite particle update); "
                                  "the evolution runs to tau = 8 fm/c with no freeze-out, and the dilute edge "
                                  "of some events (T of a few MeV) becomes unstable late in the run",
            "fp64_sequential": {k: v for k, v in seq.items() if k != "mean_resident_particles"},
            "fp64_sequential_note": "the same events and arrival trace, FP64, one event on the GPU at a time "
                                    "(a server with one event slot), latencies measured live",
        }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_run(I, w, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
