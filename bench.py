#!/usr/bin/env python3
"""Throughput benchmark of the XZZX simulated-annealing decoder on one MI355X.

A step is one pass of the whole decoder (greedy references, annealing of
every chain, per-syndrome reduction and recovery) over one batch of freshly
sampled syndromes already resident in HBM.  Default workload: rotated XZZX
d = 11, eta = 100, p in {0.10, 0.15, 0.20, 0.25} (one syndrome group per p,
all four in one persistent launch), 32 replicas (128 chains) per syndrome,
2000 sweeps of a geometric beta schedule 0.05 -> 10.

Prints one JSON line: flip attempts/s (value), decodes/s, the annealing
kernel's share of the ALU roofline (timed with HIP events on its own stream),
a CPU-oracle baseline on a bounded sample, and the plain one-launch-per-
syndrome form on the same GPU.
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

# Algorithmic integer lane-operations per flip attempt:
#   random draw: a quarter of a Philox4x32-10 block = 2.5 rounds x (2 widening
#   32x32 multiplies + 2 three-input XORs) = 10;
#   move: 8-bit pattern of the generator's four 2-bit codes (3), energy-table
#   index (1), acceptance compares (2), energy update (1), flip of the two row
#   words (2) = 9;  total 19.
OPS_PER_ATTEMPT = 19
# MI355X int32 vector issue peak from its unit counts and clock: 256 CUs x 4
# SIMDs x 32 lanes per clock (a wave64 instruction every two clocks) x 2.4 GHz
# = 78.6 T lane-ops/s, the lane rate of the published 157.3 TFLOP/s fp32
# vector figure (an FMA counts two).  bench.py --peaks measures it.
ALU_PEAK_OPS = 256 * 128 * 2.4e9
# LDS bytes a flip attempt reads in the packed-row kernels specialised to d:
# the generator's (shape, pattern) -> entry offset lookup (2 B) and the
# 12 bytes of its (dE, threshold, always-accept) entry.
LDS_BYTES_PER_ATTEMPT = 14
# MI355X LDS read peak from its unit counts and clock: 256 CUs x 64 banks x
# 4 bytes per clock x 2.4 GHz = 157.3 TB/s, the rate of 128-bit reads
# (bench.py --peaks measures 1.3-1.4e14 B/s for them; 32- and 64-bit reads
# move half as many bytes per clock).
LDS_PEAK_BYTES = 256 * 256 * 2.4e9


def kernel_source_sha256(kernel=""):
    """Digest of the sources a kernel is built from, in name order: its
    translation units and every header they include, transitively.  The
    annealing kernels specialised to a distance come from the xzzx_static_*
    units (k_anneal_rows_d<D>), xzzx_planar.hip (k_anneal_planar_d<D>),
    xzzx_ladder_rows*.hip (k_anneal_ladder_rows_d<D>) and
    xzzx_ladder_planar.hip (k_anneal_ladder_planar_d<D>); any other kernel
    is digested with every device source."""
    import glob
    import hashlib
    import re

    csrc = os.path.join(ROOT, "paper_2509_17837_amd", "csrc")
    units = {
        "k_anneal_rows_d": "xzzx_static_*.hip",
        "k_anneal_planar_d": "xzzx_planar.hip",
        "k_anneal_ladder_rows_d": "xzzx_ladder_rows*.hip",
        "k_anneal_ladder_planar_d": "xzzx_ladder_planar.hip",
    }
    pattern = next((g for k, g in units.items() if kernel.startswith(k)), "*.hip")
    todo = glob.glob(os.path.join(csrc, pattern))
    files = set()
    while todo:
        f = os.path.realpath(todo.pop())
        if f in files:
            continue
        files.add(f)
        for inc in re.findall(r'^#include "([^"]+)"', open(f).read(), re.M):
            todo.append(os.path.join(os.path.dirname(f), inc))
    h = hashlib.sha256()
    for f in sorted(files, key=os.path.basename):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def profile_values(kernel, workload, batch):
    """Key = value lines of the committed counter summary of an annealing
    kernel on a workload (HBM traffic from FETCH_SIZE + WRITE_SIZE
    calibrated against a copy of known size, LDS bank-conflict cycles per
    wave-step), or {} when the summary is for another kernel source, kernel or
    workload."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.md")
    if not os.path.exists(path):
        return {}
    kv = {}
    for line in open(path):
        if " = " in line:
            k, v = line.split(" = ", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_sha256(kernel) or kv.get("workload") != f"{workload} batch {batch}":
        return {}
    return kv


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="d11_bias100")
    ap.add_argument("--batch", type=int, default=2048, help="syndromes per group per step")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline workload only (no d31_large, mixed_d5_21 and serving lines)")
    ap.add_argument("--peaks", action="store_true",
                    help="measure the int32 VALU issue rate and the LDS read bandwidth (microbenchmarks) and exit")
    ap.add_argument("--cpu-one-core-seconds", type=float, default=6.0)
    ap.add_argument("--plain-syndromes", type=int, default=32)
    ap.add_argument("--eager", action="store_true", help="no hipGraph capture")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-knob autotuner")
    ap.add_argument("--serve", action="store_true", help="serving-loop benchmark (Poisson arrivals)")
    ap.add_argument("--rates", default="1e3,3e3,1e4,3e4,1e5")
    ap.add_argument("--requests", type=int, default=20000, help="most requests per arrival rate (--serve)")
    ap.add_argument("--serve-seconds", type=float, default=3.0,
                    help="arrival window per rate (--serve): min(--requests, rate x this) requests")
    ap.add_argument("--slice", type=int, default=250,
                    help="sweeps per serving slice of the costliest resident request (--serve)")
    ap.add_argument("--lanes", type=int, default=0,
                    help="most lanes per chain the server may use (--serve; 0: library default, 1: plan kernels)")
    ap.add_argument("--waves", type=int, default=0, help="wave budget per serving slice (--serve; 0: default)")
    ap.add_argument("--slots", type=int, default=32768, help="resident requests at most (--serve)")
    ap.add_argument("--lds-budget", type=int, default=0,
                    help="LDS bytes the resident requests' tasks may take (--serve; 0: library default)")
    ap.add_argument("--by-distance", action="store_true",
                    help="annealing rate of the default kernel for each odd d in --distances")
    ap.add_argument("--distances", default="11,13,15,17,21,25,29,31")
    ap.add_argument("--order", choices=["colour", "site"], default="colour",
                    help="Metropolis step order: colour-class sweeps, or random-site steps (Alg. 3 as printed)")
    ap.add_argument("--ladder", default="",
                    help="replica exchange instead of annealing: 'K,beta_lo,beta_hi' (levels per ladder; n_rep of the "
                         "workload must be a multiple of K)")
    ap.add_argument("--paper-trends", action="store_true",
                    help="logical error rates of the paper's set-up against N_SA and N_beta (planar, 1:eta:1)")
    ap.add_argument("--trend-d", type=int, default=9)
    ap.add_argument("--trend-p", type=float, default=0.15)
    ap.add_argument("--trend-etas", default="1,5,10")
    ap.add_argument("--trend-samples", type=int, default=20000)
    ap.add_argument("--trend-nsa", default="1,2,3,5,10,20,50,100")
    ap.add_argument("--trend-nbeta", default="0,5,10,20,50,100")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this decoder shards by syndrome with no communication, "
              "and multi-GPU runs are not part of this build (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    if args.peaks:
        print(json.dumps({"mode": "peaks", **measure_peaks(full=True)}), flush=True)
        return
    if args.serve:
        return serve_bench(args)
    if args.by_distance:
        return distance_bench(args)
    if args.paper_trends:
        return trends_bench(args)
    run = run_batch(args, args.workload, args.batch, args.steps, args.warmup, tune=not args.no_tune,
                    order=args.order, ladder=args.ladder)
    wl, R, sweeps = run["wl"], run["R"], run["sweeps"]
    peaks = measure_peaks()
    result = {
        "metric": "stabilizer-flip attempts/s",
        "value": run["value"],
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": describe(run),
            "name": args.workload,
            "step_order": "random-site (Alg. 3)" if args.order == "site" else "colour-class sweeps",
            "replica_exchange": (f"ladders of {args.ladder.split(',')[0]} levels, beta "
                                 f"{args.ladder.split(',')[1]} -> {args.ladder.split(',')[2]} (schedule unused)")
                                if args.ladder else None,
            "syndromes_per_step": run["syndromes_step"],
            "attempts_per_step": run["attempts_step"],
            "graphs": run["graphs"],
            "autotuned": run["tuned"],
            "seeds": run["seeds"],
        },
        "decodes_per_s": run["decodes"],
        "decodes_per_s_anneal_only": run["syndromes_step"] / run["anneal_s"],
        "stage_ms": run["stage_ms"],
        "roofline": roofline(run, peaks, args.workload, args.batch),
        "peaks_measured": peaks,
        "logical_error_rate": run["ler"],
    }
    if not args.no_plain:
        result["plain_form"] = plain_form(args, run)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(args, run)
    if not args.no_extras and args.workload == "d11_bias100" and not args.order == "site" and not args.ladder:
        result["d31_large"] = extra_batch(args, "d31_large", 1024, peaks)
        result["mixed_d5_21"] = extra_batch(args, "mixed_d5_21", 2048, peaks)
        result["serving"] = serve_extra(args, peaks)
    print(json.dumps(result), flush=True)


def describe(run):
    wl, conv = run["wl"], run["conv"]
    return (f"{wl.get('layout', 'rotated')} XZZX d={','.join(str(d) for d in wl['d'])}, "
            f"{'p_x:p_y:p_z = 1:eta:1' if conv else 'p_y = p eta/(eta+1)'}, eta={wl['eta']}, p={wl['p']}, "
            f"{run['R']} replicas ({4 * run['R']} chains)/syndrome, {run['sweeps']} sweeps {wl['schedule'][0]} "
            f"{wl['schedule'][1]}->{wl['schedule'][2]}")


def run_batch(args, name, B, steps, warm, tune=True, order="colour", ladder=""):
    """Time `steps` decode steps of workload `name` after `warm` untimed ones:
    one group per (d, p, eta) of B syndromes, all groups in one call, each
    stage captured in a hipGraph (unless --eager) and launched on torch's
    current stream; fresh syndromes every step, resident in HBM before the
    timed region."""
    import torch

    from paper_2509_17837_amd import _lib as X
    from paper_2509_17837_amd import decoder as D
    from paper_2509_17837_amd import inputs

    wl = inputs.WORKLOADS[name]
    seeds = inputs.seeds(name)
    sched_kind = inputs.SCHEDULE_KIND[wl["schedule"][0]]
    sweeps = wl["sweeps"]
    R = wl["n_rep"]
    dev = torch.device("cuda:0")
    specs = [(d, p, eta) for d in wl["d"] for p in wl["p"] for eta in wl["eta"]]
    layout, conv = inputs.layout_of(wl), inputs.convention_of(wl)
    plans, lats = [], {}
    beta = D.schedule(sched_kind, wl["schedule"][1], wl["schedule"][2], sweeps)
    for d, p, eta in specs:
        if d not in lats:
            lats[d] = D.Lattice(layout, d)
        w, wg = D.weights(p, D.noise(p, eta, conv))
        plans.append(D.Plan(lats[d], w, wg, beta))
        if order == "site":
            plans[-1].set_order(X.ORDER_RANDOM_SITE)
        if ladder:
            k, blo, bhi = ladder.split(",")
            plans[-1].set_ladder(int(k), float(blo), float(bhi))
    ng = len(plans)
    tuned = {}
    if tune:
        for (d, p, eta), plan in zip(specs, plans):
            # probe at the launch's real size (all groups share one launch)
            tuned[f"d{d}_p{p}_eta{eta:g}"] = plan.autotune(R, n_syn=B * ng, probe_sweeps=10)

    syn_all, uid_all, err_all = [], [], []
    for k in range(steps + warm):
        row_s, row_u, row_e = [], [], []
        for gi, ((d, p, eta), plan) in enumerate(zip(specs, plans)):
            # errors keyed by the sample seed and each syndrome's uid
            err = inputs.sample_errors(B, plan.nq, inputs.channel(p, eta, conv), seeds["sample"],
                                       uid0=(k * ng + gi) * B)
            row_s.append(D.syndrome(plan, torch.from_numpy(err).to(dev)))
            row_u.append(torch.from_numpy(inputs.sample_uids(B, (k * ng + gi) * B).view(np.int32)).to(dev))
            row_e.append(err)
        syn_all.append(row_s)
        uid_all.append(row_u)
        err_all.append(row_e)
    torch.cuda.synchronize()

    syn_buf = [torch.empty_like(syn_all[0][g]) for g in range(ng)]
    uid_buf = [torch.empty_like(uid_all[0][g]) for g in range(ng)]
    groups, outs = [], []
    for g in range(ng):
        grp, o = D.make_group(plans[g], R, uid_buf[g], syn=syn_buf[g], want_extra=False)
        groups.append(grp)
        outs.append(o)
    gs, as_ = seeds["greedy"], seeds["anneal"]
    stage_flags = [X.STAGE_GREEDY, X.STAGE_ANNEAL, X.STAGE_FINISH]
    ws = D.workspace(groups)
    graphs = None
    if not args.eager:
        cap = torch.cuda.Stream()
        graphs = [D.Graph(groups, gs, as_, X.GREEDY_RANDOM, f, stream=cap, ws=ws) for f in stage_flags]
        torch.cuda.synchronize()
    cur = torch.cuda.current_stream()

    def run_step(k, ev=None):
        for g in range(ng):
            syn_buf[g].copy_(syn_all[k][g], non_blocking=True)
            uid_buf[g].copy_(uid_all[k][g], non_blocking=True)
        for si, f in enumerate(stage_flags):
            if ev is not None:
                ev[si].record(cur)
            if graphs is not None:
                graphs[si].launch(cur)
            else:
                D.decode_groups(groups, gs, as_, X.GREEDY_RANDOM, f, ws=ws)
        if ev is not None:
            ev[3].record(cur)

    for k in range(warm):
        run_step(k)
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        run_step(warm + k, events[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stage_ms = [float(np.mean([events[k][i].elapsed_time(events[k][i + 1]) for k in range(steps)])) for i in range(3)]
    attempts_step = sum(B * 4 * R * sweeps * plan.nstab for plan in plans)

    # logical error rate of the last timed batch: [C_true * recovery] != I
    last = warm + steps - 1
    ler = {}
    for g, (d, p, eta) in enumerate(specs):
        fails = logical_failures(lats[d], err_all[last][g], outs[g].recovery.cpu().numpy())
        ler[f"d{d}_p{p}_eta{eta:g}"] = float(fails.mean())

    kinds = {pl.info()["kernel"] for pl in plans}
    if kinds == {X.KERNEL_SITE}:
        kernel_name = "k_anneal_site"
    elif kinds == {X.KERNEL_LADDER} and layout == X.PLANAR and len(set(wl["d"])) == 1 and wl["d"][0] <= 15:
        kernel_name = f"k_anneal_ladder_planar_d{wl['d'][0]}"   # ladders on planar packed rows specialised to d
    elif kinds == {X.KERNEL_LADDER} and len(set(wl["d"])) == 1 and wl["d"][0] <= 31 and (4 * R) % 64 == 0:
        kernel_name = f"k_anneal_ladder_rows_d{wl['d'][0]}"     # ladders on packed rows specialised to d
    elif kinds == {X.KERNEL_LADDER}:
        kernel_name = "k_anneal_ladder"
    elif kinds == {X.KERNEL_ROWS} and layout == X.PLANAR and len(set(wl["d"])) == 1:
        kernel_name = f"k_anneal_planar_d{wl['d'][0]}"   # planar packed rows specialised to d
    elif kinds == {X.KERNEL_ROWS} and len(set(wl["d"])) == 1 and (4 * R) % 64 == 0:
        kernel_name = f"k_anneal_rows_d{wl['d'][0]}"   # packed rows specialised to d
    elif kinds == {X.KERNEL_ROWS} and (4 * R) % 64 == 0:
        kernel_name = "k_anneal_rows_d<D>"   # one specialised launch per distance, run concurrently
    elif kinds <= {X.KERNEL_ROWS, X.KERNEL_ROWS_GENERIC}:
        kernel_name = "k_anneal_rows"
    else:
        kernel_name = "k_anneal"
    return dict(wl=wl, seeds=seeds, specs=specs, plans=plans, lats=lats, layout=layout, conv=conv, R=R,
                sweeps=sweeps, B=B, ng=ng, tuned=tuned, graphs=graphs is not None, stage_ms=dict(
                    greedy=stage_ms[0], anneal=stage_ms[1], finish=stage_ms[2]),
                anneal_s=stage_ms[1] / 1e3, attempts_step=attempts_step, syndromes_step=B * ng,
                value=steps * attempts_step / elapsed, decodes=steps * B * ng / elapsed,
                ms_per_step=1e3 * elapsed / steps, ler=ler, kernel=kernel_name, outs=outs,
                syn_last=syn_all[last], uid_last=uid_all[last], gs=gs, as_=as_, order=order, ladder=ladder)


def measure_peaks(full=False):
    """The two device limits, measured by the library's microbenchmarks: int32
    VALU lane-ops/s (v_xor_b32, v_add_u32, v_bitop3_b32; v_mad_u64_u32 apart)
    and conflict-free LDS read bytes/s, with eight wavefronts per SIMD (and
    four, with full)."""
    from paper_2509_17837_amd import decoder as D

    out = {}
    waves = (8, 4) if full else (8,)
    for wv in waves:
        sfx = "" if wv == 8 else f"_w{wv}"
        simple = [D.probe_valu(k, wv, 4000) for k in (0, 1, 2)]
        out["valu_xor_ops" + sfx] = simple[0]
        out["valu_add_ops" + sfx] = simple[1]
        out["valu_bitop3_ops" + sfx] = simple[2]
        out["valu_mad_u64_ops" + sfx] = D.probe_valu(3, wv, 2000)
        for b in ((4, 8, 16) if full else (16,)):
            out[f"lds_b{8 * b}_bytes" + sfx] = D.probe_lds(b, wv, 4000)
    out["valu_simple_ops"] = max(out["valu_xor_ops"], out["valu_add_ops"], out["valu_bitop3_ops"])
    out["lds_bytes"] = out["lds_b128_bytes"]
    out["note"] = ("lane-ops/s and bytes/s over all CUs at the clock the device ran; peaks from unit counts: "
                   f"VALU {ALU_PEAK_OPS:.4g} lane-ops/s, LDS {LDS_PEAK_BYTES:.4g} B/s")
    return out


def roofline(run, peaks, workload, batch):
    """The annealing kernel against both limits that can bind it: int32 VALU
    issue (19 algorithmic lane-ops per attempt) and LDS reads (14 bytes per
    attempt), each against the peak from unit counts and clock and against the
    measured one; `bound` names the side with the larger fraction."""
    attempts, t = run["attempts_step"], run["anneal_s"]
    alu = OPS_PER_ATTEMPT * attempts / t
    lds = LDS_BYTES_PER_ATTEMPT * attempts / t
    kv = profile_values(run["kernel"], workload, batch)
    traffic = int(kv["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in kv else None
    sides = {
        "alu": {"achieved": alu / 1e12, "peak": ALU_PEAK_OPS / 1e12, "unit": "Tops/s (int32 lane-ops)",
                "frac": alu / ALU_PEAK_OPS, "peak_measured": peaks["valu_simple_ops"] / 1e12,
                "frac_of_measured": alu / peaks["valu_simple_ops"], "ops_per_attempt": OPS_PER_ATTEMPT,
                "valu_busy_frac": float(kv["valu_busy_frac"]) if "valu_busy_frac" in kv else None},
        "lds": {"achieved": lds / 1e12, "peak": LDS_PEAK_BYTES / 1e12, "unit": "TB/s (LDS reads)",
                "frac": lds / LDS_PEAK_BYTES, "peak_measured": peaks["lds_bytes"] / 1e12,
                "frac_of_measured": lds / peaks["lds_bytes"], "bytes_per_attempt": LDS_BYTES_PER_ATTEMPT,
                "bank_conflict_cycles_per_wave_step": (float(kv["lds_bank_conflict_cycles_per_wave_step"])
                                                       if "lds_bank_conflict_cycles_per_wave_step" in kv else None),
                "lds_busy_frac": float(kv["lds_busy_frac"]) if "lds_busy_frac" in kv else None},
    }
    bound = "alu" if sides["alu"]["frac"] >= sides["lds"]["frac"] else "lds"
    top = sides[bound]
    return {"bound": bound, "kernel": run["kernel"], "achieved": top["achieved"], "peak": top["peak"],
            "unit": top["unit"], "frac": top["frac"], "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "anneal_ms_per_launch": 1e3 * t, "alu": sides["alu"], "lds": sides["lds"]}


def plain_form(args, run):
    """One annealing launch per syndrome (no persistence, no graph) on the
    first syndromes of the last timed batch; same results required."""
    import torch

    from paper_2509_17837_amd import _lib as X
    from paper_2509_17837_amd import decoder as D

    n = min(args.plain_syndromes, run["B"])
    R, gs, as_ = run["R"], run["gs"], run["as_"]
    pg, po = D.make_group(run["plans"][0], R, run["uid_last"][0][:n].contiguous(),
                          syn=run["syn_last"][0][:n].contiguous(), want_extra=False)
    pws = D.workspace([pg])
    D.decode_groups([pg], gs, as_, X.GREEDY_RANDOM, X.STAGE_GREEDY, ws=pws)
    torch.cuda.synchronize()
    cur = torch.cuda.current_stream()
    ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ea.record(cur)
    D.decode_groups([pg], gs, as_, X.GREEDY_RANDOM, X.STAGE_ANNEAL | X.FLAG_PLAIN, ws=pws)
    eb.record(cur)
    torch.cuda.synchronize()
    plain_s = ea.elapsed_time(eb) / 1e3
    D.decode_groups([pg], gs, as_, X.GREEDY_RANDOM, X.STAGE_FINISH, ws=pws)
    torch.cuda.synchronize()
    o0 = run["outs"][0]
    same = bool(torch.equal(po.recovery, o0.recovery[:n]) and torch.equal(po.e_best, o0.e_best[:n]))
    rate = n * 4 * R * run["sweeps"] * run["plans"][0].nstab / plain_s
    return {"value": rate, "unit": "attempts/s", "syndromes": n,
            "batched_over_plain": (run["attempts_step"] / run["anneal_s"]) / rate, "same_results_as_batched": same}


def host_cpu():
    """(usable threads, model name) of the host."""
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return threads, model


def cpu_baseline(args, run):
    """Time the oracle (plain C, one syndrome per thread) on bounded samples
    of the last timed batch: on every usable host thread, and on one; the
    samples are checked against the GPU results."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O
    from paper_2509_17837_amd import inputs

    threads, model = host_cpu()
    wl, specs, plans, R, sweeps = run["wl"], run["specs"], run["plans"], run["R"], run["sweeps"]
    ng = len(specs)
    sched = wl["schedule"]
    obeta = O.schedule(inputs.SCHEDULE_KIND[sched[0]], sched[1], sched[2], sweeps)
    owts = [O.weights(p, O.noise(p, eta, run["conv"])) for (_, p, eta) in specs]
    syn = [s.cpu().numpy() for s in run["syn_last"]]
    uid = [u.cpu().numpy().view(np.uint32) for u in run["uid_last"]]
    outs = run["outs"]

    def one(job):
        g, i = job
        lat = O.Lattice(run["layout"], specs[g][0])
        if run["ladder"]:
            k, blo, bhi = run["ladder"].split(",")
            return lat.decode(owts[g][0], owts[g][1], syn[g][i], int(uid[g][i]), R, obeta, run["gs"], run["as_"],
                              order=O.ORDER_LADDER, ladder=(int(k), float(blo), float(bhi)))
        return lat.decode(owts[g][0], owts[g][1], syn[g][i], int(uid[g][i]), R, obeta, run["gs"], run["as_"],
                          order=O.ORDER_RANDOM_SITE if run["order"] == "site" else O.ORDER_COLOUR)

    def check(jobs, res):
        ok = 0
        for (g, i), r in zip(jobs, res):
            ok += int(outs[g].e_best[i].item() == r["e_best"] and outs[g].cls[i].item() == r["cls"] and
                      np.array_equal(outs[g].recovery[i].cpu().numpy(), r["recovery"]))
        return ok

    # one core: syndromes in turn until the time is spent
    jobs1, res1 = [], []
    t = time.perf_counter()
    while time.perf_counter() - t < args.cpu_one_core_seconds or not jobs1:
        job = (len(jobs1) % ng, len(jobs1) // ng)
        jobs1.append(job)
        res1.append(one(job))
    wall1 = time.perf_counter() - t
    per = wall1 / len(jobs1)
    # every thread: a sample sized to about --cpu-seconds
    n = max(threads, int(args.cpu_seconds * threads / max(per, 1e-6)))
    n = min(n, 4 * len(syn[0]))
    jobs = [((i + len(jobs1)) % ng, (i + len(jobs1)) // ng) for i in range(n)]
    t = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(one, jobs))
    wall = time.perf_counter() - t
    attempts = sum(4 * R * sweeps * plans[g].nstab for g, _ in jobs)
    attempts1 = sum(4 * R * sweeps * plans[g].nstab for g, _ in jobs1)
    return {
        "value": attempts / wall,
        "unit": "attempts/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{n} syndromes of the last timed batch (groups round-robin), full decode "
                  f"({R} replicas, {sweeps} sweeps), {wall:.1f} s wall on {threads} threads; "
                  f"{len(jobs1)} more on one thread, {wall1:.1f} s",
        "decodes_per_s": n / wall,
        "one_core": {"value": attempts1 / wall1, "decodes_per_s": len(jobs1) / wall1},
        "host": {"threads": threads, "nproc": os.cpu_count(), "model": model},
        "bitexact_with_gpu": f"{check(jobs, res) + check(jobs1, res1)}/{n + len(jobs1)}",
    }


def extra_batch(args, name, batch, peaks):
    """Another workload of the metric in the headline's launch configuration
    (one step after a warm-up; no autotuning, every group on its plan's
    default kernel), with its roofline and the oracle's decode of one
    syndrome per group (its chains spread over the host threads) compared
    bit for bit."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O
    from paper_2509_17837_amd import inputs

    run = run_batch(args, name, batch, 2, 1, tune=False)
    rl = roofline(run, peaks, name, batch)
    wl, specs = run["wl"], run["specs"]
    sched = wl["schedule"]
    obeta = O.schedule(inputs.SCHEDULE_KIND[sched[0]], sched[1], sched[2], run["sweeps"])
    threads, _ = host_cpu()
    ok, t0 = 0, time.perf_counter()
    with ThreadPoolExecutor(threads) as pool:
        for g, (d, p, eta) in enumerate(specs):
            w, wg = O.weights(p, O.noise(p, eta, run["conv"]))
            syn = run["syn_last"][g][0].cpu().numpy()
            uid = int(run["uid_last"][g][0].cpu().numpy().view(np.uint32))
            r = O.decode_by_chain(run["layout"], d, w, wg, syn, uid, run["R"], obeta, run["gs"], run["as_"], pool)
            o = run["outs"][g]
            ok += int(o.e_best[0].item() == r["e_best"] and o.cls[0].item() == r["cls"] and
                      np.array_equal(o.recovery[0].cpu().numpy(), r["recovery"]))
    print(f"[bench] {name}: {run['value']:.4g} attempts/s, oracle check {ok}/{len(specs)} "
          f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    return {"value": run["value"], "unit": "attempts/s", "decodes_per_s": run["decodes"],
            "decodes_per_s_anneal_only": run["syndromes_step"] / run["anneal_s"], "steps": 2, "warmup": 1,
            "ms_per_step": run["ms_per_step"], "workload": describe(run), "syndromes_per_step": run["syndromes_step"],
            "stage_ms": run["stage_ms"], "roofline": rl, "logical_error_rate": run["ler"],
            "oracle_bitexact": f"{ok}/{len(specs)} syndromes (first of each group of the last step: "
                               "E_best, P*, recovery)"}


def distance_bench(args):
    """Annealing-stage rate by lattice distance: rotated lattice, p = 0.15,
    eta = 10, 16 replicas (one 64-chain task per syndrome), 200 sweeps
    geometric 0.05->10, enough syndromes for several tasks per wavefront
    slot; the greedy stage runs once, untimed."""
    import torch

    from paper_2509_17837_amd import _lib as X
    from paper_2509_17837_amd import decoder as D
    from paper_2509_17837_amd import inputs

    p, eta, R, sweeps = 0.15, 10.0, 16, 200
    beta = D.schedule(inputs.SCHEDULE_KIND["geometric"], 0.05, 10.0, sweeps)
    kernels = {X.KERNEL_ROWS: "rows", X.KERNEL_ROWS_GENERIC: "rows_generic", X.KERNEL_BYTES: "bytes"}
    rows = []
    for d in [int(x) for x in args.distances.split(",")]:
        lat = D.Lattice(X.ROTATED, d)
        w, wg = D.weights(p, D.noise(p, eta))
        plan = D.Plan(lat, w, wg, beta)
        n_syn = 32768 if d <= 21 else 16384
        err = inputs.sample_errors(n_syn, lat.nq, inputs.channel(p, eta), 1100 + d)
        syn = D.syndrome(plan, torch.from_numpy(np.ascontiguousarray(err)).cuda())
        uid = torch.from_numpy(inputs.sample_uids(n_syn).view(np.int32)).cuda()
        g, _ = D.make_group(plan, R, uid, syn=syn)
        ws = D.decode_groups([g], 1, 2, flags=X.STAGE_GREEDY)
        times = []
        for _ in range(args.warmup + args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            D.decode_groups([g], 1, 2, flags=X.STAGE_ANNEAL, ws=ws)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times[args.warmup:]))
        attempts = n_syn * 4 * R * sweeps * lat.nstab
        rows.append({"d": d, "syndromes": n_syn, "anneal_ms": ms, "attempts_per_s": attempts / ms * 1e3,
                     "kernel": kernels.get(plan.info()["kernel"], "?")})
        print(f"[by-distance] d={d}: {ms:.2f} ms, {attempts / ms * 1e3:.4g} attempts/s ({rows[-1]['kernel']})",
              file=sys.stderr, flush=True)
    print(json.dumps({"metric": "stabilizer-flip attempts/s by distance (annealing stage)", "unit": "attempts/s",
                      "n_gpus": 1, "dtype": "int32", "data": "synthetic",
                      "config": {"workload": f"rotated XZZX, p={p}, eta={eta}, {R} replicas, {sweeps} sweeps "
                                             f"geometric 0.05->10"},
                      "distances": rows}), flush=True)


def logical_failures(lat, err, rec):
    """Rows i where err[i] * rec[i] is a non-trivial logical operator, i.e.
    anticommutes with L_X or L_Z (both have the syndrome of err[i])."""
    lx, lz = lat.logicals()
    e = np.bitwise_xor(err, rec).astype(np.int64)
    ex, ez = (e >> 1) & 1, e & 1

    def symp(L):
        L = L.astype(np.int64)
        return (ex @ (L & 1) + ez @ ((L >> 1) & 1)) & 1

    return (symp(lx) | symp(lz)).astype(bool)


def trends_bench(args):
    """Logical error rates of the paper's own set-up (Sec. V): planar layout,
    p_x:p_y:p_z = 1:eta:1, log schedule 0.9 beta_N -> beta_N (Eqs. 23-24).
      * P_L against N_SA at N_beta = 100 with randomized greedy references
        (Alg. 6), and the greedy-matching decoder (Alg. 5) alone (Figs. 6-8);
      * P_L against N_beta at N_SA = 10 for the three reference constructions
        of Sec. V.C: boundary, greedy (same), greedy (different) (Figs. 9-11,
        which plot the ratio to an exact decoder; P_L itself is reported here).
    Every rate is over the same seeded syndromes, so two settings can also be
    compared pair by pair: `better`/`worse` count syndromes that one setting
    decodes and the other does not (each check lists `better` and `worse`
    for the setting the paper finds better)."""
    import torch

    from paper_2509_17837_amd import _lib as X
    from paper_2509_17837_amd import decoder as D
    from paper_2509_17837_amd import inputs

    d, p, n = args.trend_d, args.trend_p, args.trend_samples
    etas = [float(x) for x in args.trend_etas.split(",")]
    nsas = [int(x) for x in args.trend_nsa.split(",")]
    nbetas = [int(x) for x in args.trend_nbeta.split(",")]
    dev = torch.device("cuda:0")
    lat = D.Lattice(X.PLANAR, d)
    gs, as_ = 0x7E4D0000 + d, 0xA11E7E4D0000 + d
    t_start = time.perf_counter()

    def rate(fail):
        m = float(fail.mean())
        return [m, float(np.sqrt(max(m * (1 - m), 1e-300) / len(fail)))]

    def paired(fa, fb):
        """Failure arrays of settings a (the one the paper finds better) and b:
        syndromes only a decodes (better) and only b decodes (worse)."""
        return {"better": int(np.count_nonzero(~fa & fb)), "worse": int(np.count_nonzero(fa & ~fb))}

    out = {"mode": "paper_trends", "data": "synthetic",
           "config": {"layout": "planar", "d": d, "p": p, "etas": etas, "channel": "p_x:p_y:p_z = 1:eta:1",
                      "schedule": "paper_log 0.9 -> 1.0 (units of beta_N)", "syndromes": n},
           "p_l_vs_n_sa": {}, "greedy_decoder": {}, "p_l_vs_n_beta": {}, "checks": {}}
    for eta in etas:
        key = f"eta{eta:g}"
        w, wg = D.weights(p, D.noise(p, eta, X.BIAS_PAPER))
        err = inputs.sample_errors(n, lat.nq, inputs.channel(p, eta, 1), 4242, stream=int(eta * 10))
        uid = torch.from_numpy(inputs.sample_uids(n).view(np.int32)).to(dev)
        plans = {nb: D.Plan(lat, w, wg, D.schedule(X.SCHED_PAPER_LOG, 0.9, 1.0, nb)) for nb in set(nbetas) | {100}}
        syn = D.syndrome(plans[100], torch.from_numpy(err).to(dev))
        # greedy-matching decoder: the reference of Alg. 5 is the recovery
        refs, _ = D.greedy_init(plans[100], syn, uid, 1, gs, X.GREEDY_SAME)
        f_greedy = logical_failures(lat, err, refs[:, 0].cpu().numpy())
        out["greedy_decoder"][key] = rate(f_greedy)
        fails = {}
        for nsa in nsas:
            o = D.decode(plans[100], syn, uid, nsa, gs, as_, X.GREEDY_RANDOM)
            fails[nsa] = logical_failures(lat, err, o.recovery.cpu().numpy())
        out["p_l_vs_n_sa"][key] = {str(k): rate(v) for k, v in fails.items()}
        byinit = {}
        for mname, mode in (("boundary", X.GREEDY_BOUNDARY), ("greedy_same", X.GREEDY_SAME),
                            ("greedy_different", X.GREEDY_RANDOM)):
            byinit[mname] = {}
            for nb in nbetas:
                o = D.decode(plans[nb], syn, uid, 10, gs, as_, mode)
                byinit[mname][nb] = logical_failures(lat, err, o.recovery.cpu().numpy())
        out["p_l_vs_n_beta"][key] = {m: {str(nb): rate(f) for nb, f in v.items()} for m, v in byinit.items()}
        # step order: the literal random-site chain against colour-class sweeps
        site_plan = D.Plan(lat, w, wg, D.schedule(X.SCHED_PAPER_LOG, 0.9, 1.0, 100))
        site_plan.set_order(X.ORDER_RANDOM_SITE)
        o = D.decode(site_plan, syn, uid, 10, gs, as_, X.GREEDY_RANDOM)
        f_site = logical_failures(lat, err, o.recovery.cpu().numpy())
        out.setdefault("step_order_n_sa10", {})[key] = {"colour": rate(fails[10]) if 10 in fails else None,
                                                        "random_site": rate(f_site)}
        # replica exchange against annealing at equal work: 8 replicas x 4
        # cosets x 100 sweeps; ladders of K levels at fixed beta 0.9 .. 1.0
        f_sa8 = logical_failures(lat, err, D.decode(plans[100], syn, uid, 8, gs, as_).recovery.cpu().numpy())
        lad = {"anneal_log_0.9_1.0": rate(f_sa8)}
        lad_checks = {}
        for K, blo in ((1, 0.9), (2, 0.9), (4, 0.9), (8, 0.9), (8, 0.3)):
            lp = D.Plan(lat, w, wg, D.schedule(X.SCHED_PAPER_LOG, 0.9, 1.0, 100))
            lp.set_ladder(K, blo, 1.0)
            f_l = logical_failures(lat, err, D.decode(lp, syn, uid, 8, gs, as_).recovery.cpu().numpy())
            lad[f"ladder_K{K}_{blo}_1.0"] = rate(f_l)
            lad_checks[f"ladder_K{K}_{blo}_1.0_vs_anneal"] = paired(f_l, f_sa8)
        out.setdefault("replica_exchange_n_rep8", {})[key] = lad
        # pair-by-pair comparisons behind the paper's statements
        ks = sorted(fails)
        out["checks"][key] = {
            "n_sa_steps": {f"{a}->{b}": paired(fails[b], fails[a]) for a, b in zip(ks, ks[1:])},
            "sa_vs_greedy": {str(k): paired(fails[k], f_greedy) for k in ks},
            "different_vs_same": {str(nb): paired(byinit["greedy_different"][nb], byinit["greedy_same"][nb])
                                  for nb in nbetas},
            "same_vs_boundary": {str(nb): paired(byinit["greedy_same"][nb], byinit["boundary"][nb])
                                 for nb in nbetas},
        }
        if 10 in fails:
            out["checks"][key]["colour_vs_random_site"] = paired(fails[10], f_site)
        out["checks"][key].update(lad_checks)
        print(f"[trends] eta={eta:g} greedy {out['greedy_decoder'][key][0]:.4f} "
              + " ".join(f"N_SA={k}:{fails[k].mean():.4f}" for k in ks), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    out["seconds"] = time.perf_counter() - t_start
    print(json.dumps(out), flush=True)


def serve_setup(args):
    """Plans and pre-sampled requests of the serving workload (d and eta drawn
    uniformly per request, syndromes computed by the library's kernel)."""
    import torch

    from paper_2509_17837_amd import _lib as X
    from paper_2509_17837_amd import decoder as D
    from paper_2509_17837_amd import inputs

    name = "serving_d7_25"
    wl = inputs.WORKLOADS[name]
    seeds = inputs.seeds(name)
    kind = inputs.SCHEDULE_KIND[wl["schedule"][0]]
    beta = D.schedule(kind, wl["schedule"][1], wl["schedule"][2], wl["sweeps"])
    R = wl["n_rep"]
    specs = [(d, eta) for d in wl["d"] for eta in wl["eta"]]
    plans, lats = [], {}
    p = wl["p"][0]
    for d, eta in specs:
        if d not in lats:
            lats[d] = D.Lattice(X.ROTATED, d)
        w, wg = D.weights(p, D.noise(p, eta))
        plans.append(D.Plan(lats[d], w, wg, beta))
    n = max(int(args.requests), 1)
    rng = np.random.default_rng([seeds["sample"], 11])
    pick = rng.integers(0, len(specs), size=n)
    reqs = []
    for i in range(n):
        d, eta = specs[pick[i]]
        err = inputs.sample_errors(1, d * d, inputs.channel(p, eta), seeds["sample"], uid0=7_000_000 + i)[0]
        reqs.append((int(pick[i]), err))
    syns = [None] * n
    for k in range(len(specs)):   # one syndrome launch per (d, eta)
        idx = [i for i in range(n) if reqs[i][0] == k]
        if idx:
            s = D.syndrome(plans[k], torch.from_numpy(np.stack([reqs[i][1] for i in idx])).cuda()).cpu().numpy()
            for j, i in enumerate(idx):
                syns[i] = s[j]
    torch.cuda.synchronize()
    attempts = [4 * R * wl["sweeps"] * plans[k].nstab for k, _ in reqs]
    return dict(name=name, wl=wl, seeds=seeds, R=R, specs=specs, plans=plans, p=p, reqs=reqs, syns=syns,
                attempts=attempts)


def serve_rate(args, S, rate, seconds, keep=()):
    """Poisson arrivals at `rate` over `seconds` (at most --requests requests)
    submitted while earlier ones run; returns the server's statistics and the
    results of the requests listed in `keep`."""
    from paper_2509_17837_amd import decoder as D
    from paper_2509_17837_amd import inputs

    n_rate = max(1, min(len(S["reqs"]), int(rate * seconds)))
    arr = inputs.poisson_arrivals(rate, n_rate, S["seeds"]["sample"] + int(rate))
    srv = D.Server(max_slots=args.slots, max_rep=S["R"], max_qubits=max(d * d for d in S["wl"]["d"]),
                   sweeps_per_slice=args.slice, greedy_seed=S["seeds"]["greedy"], anneal_seed=S["seeds"]["anneal"],
                   max_lanes_per_chain=args.lanes, max_waves=args.waves, lds_budget_bytes=args.lds_budget)
    t0 = time.perf_counter()
    tickets = []
    i = 0
    # every request whose arrival time has passed goes in one submission, so
    # the Python loop keeps up with the offered rate
    while i < n_rate:
        now = time.perf_counter() - t0
        if now < arr[i]:
            if arr[i] - now > 2e-4:
                time.sleep((arr[i] - now) * 0.5)
            continue
        j = i + 1
        while j < n_rate and arr[j] <= now:
            j += 1
        ks = [S["reqs"][m][0] for m in range(i, j)]
        tickets += srv.submit_many([S["plans"][k] for k in ks], S["syns"][i:j], range(7_000_000 + i, 7_000_000 + j),
                                   S["R"])
        i = j
    srv.drain()
    wall = time.perf_counter() - t0
    st = srv.stats()
    kept = {}
    for i, t in enumerate(tickets):
        r = srv.poll(t)
        if i in keep:
            kept[i] = r
    srv.close()
    row = {"rate_per_s": rate, "requests": n_rate,
           "p50_latency_ms": 1e3 * st["p50_latency_s"], "p99_latency_ms": 1e3 * st["p99_latency_s"],
           "mean_latency_ms": 1e3 * st["mean_latency_s"],
           "decodes_per_s": st["decodes_per_s"], "attempts_per_s": st["attempts_per_s"],
           "offered_attempts_per_s": rate * float(np.mean(S["attempts"][:n_rate])),
           "slices": st["slices"], "wall_s": wall}
    print(f"[serve] rate {rate:g}/s: p50 {row['p50_latency_ms']:.2f} ms, p99 {row['p99_latency_ms']:.2f} ms, "
          f"{st['decodes_per_s']:.0f} decodes/s", file=sys.stderr, flush=True)
    return row, kept


def serve_extra(args, peaks):
    """The serving workload's latency and throughput for the headline line:
    p50/p99 at 10^3 and 10^4 requests/s, and the saturation rate with
    2 x 10^5 requests/s offered; 24 requests of the 10^4 run compared bit for
    bit with the oracle."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O

    import copy

    a = copy.copy(args)
    a.requests = max(args.requests, 100000)
    S = serve_setup(a)
    keep = tuple(range(0, 2400, 100))
    rows = {}
    # 2 s of arrivals at 10^3 and 10^4 per second; saturation: 10^5 requests
    # offered at 2 x 10^5 per second, so the steady state outlasts the ramps
    for rate, secs in ((1e3, 2.0), (1e4, 2.0), (2e5, 0.5)):
        rows[rate], kept = serve_rate(a, S, rate, secs, keep if rate == 1e4 else ())
        if rate == 1e4:
            check = kept
    p, R, wl, seeds = S["p"], S["R"], S["wl"], S["seeds"]
    beta = O.schedule(O.SCHED_GEOMETRIC, wl["schedule"][1], wl["schedule"][2], wl["sweeps"])

    def oracle(i):
        k, _ = S["reqs"][i]
        d, eta = S["specs"][k]
        w, wg = O.weights(p, O.noise(p, eta))
        return O.Lattice(O.ROTATED, d).decode(w, wg, S["syns"][i], 7_000_000 + i, R, beta, seeds["greedy"],
                                              seeds["anneal"])

    threads, _ = host_cpu()
    with ThreadPoolExecutor(threads) as pool:
        refs = dict(zip(check, pool.map(oracle, list(check))))
    ok = sum(int(check[i]["e_best"] == refs[i]["e_best"] and check[i]["cls"] == refs[i]["cls"] and
                 np.array_equal(check[i]["recovery"], refs[i]["recovery"])) for i in check)
    sat = rows[2e5]
    return {
        "workload": (f"single-syndrome requests, rotated XZZX d in {wl['d']}, eta in {wl['eta']}, p={p}, {R} replicas, "
                     f"{wl['sweeps']} sweeps geometric 0.05->10, Poisson arrivals"),
        "p50_ms_at_1e3": rows[1e3]["p50_latency_ms"], "p99_ms_at_1e3": rows[1e3]["p99_latency_ms"],
        "p50_ms_at_1e4": rows[1e4]["p50_latency_ms"], "p99_ms_at_1e4": rows[1e4]["p99_latency_ms"],
        "saturation_decodes_per_s": sat["decodes_per_s"], "saturation_attempts_per_s": sat["attempts_per_s"],
        "saturation_alu_frac": sat["attempts_per_s"] * OPS_PER_ATTEMPT / ALU_PEAK_OPS,
        "rates": list(rows.values()),
        "sweeps_per_slice": args.slice, "max_slots": args.slots,
        "oracle_bitexact": f"{ok}/{len(check)} requests of the 10^4/s run (E_best, P*, recovery)",
    }


def serve_bench(args):
    """Serving loop under Poisson arrivals: requests of the serving workload
    (d and eta drawn uniformly per request) are submitted at their arrival
    times while earlier ones run; reports p50/p99 latency and throughput per
    arrival rate."""
    S = serve_setup(args)
    out = [serve_rate(args, S, float(rate), args.serve_seconds)[0] for rate in args.rates.split(",")]
    wl, R = S["wl"], S["R"]
    result = {
        "metric": "decode latency p50/p99 (serving, continuous batching)",
        "value": out[0]["p99_latency_ms"],
        "unit": "ms (p99 at the lowest rate)",
        "n_gpus": 1,
        "higher_is_better": False,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"single-syndrome requests, rotated XZZX d in {wl['d']}, eta in {wl['eta']}, "
                               f"p={S['p']}, {R} replicas, {wl['sweeps']} sweeps geometric 0.05->10, Poisson arrivals",
                   "name": S["name"], "sweeps_per_slice": args.slice, "max_slots": args.slots,
                   "max_lanes_per_chain": args.lanes,
                   "max_waves": args.waves, "seeds": S["seeds"]},
        "rates": out,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
