#!/usr/bin/env python3
"""Benchmark of the GCB greedy RBF hot path on one MI355X.

One step = the whole hot path over one synthetic input: the GCB greedy
selection (partition and staging, group sweeps, argmax, FP64 inverse-factor
appends, FP64 all-node certificate) on the 80,000-node wing at m = 107, then
the volume deformation (Eq. 6) of 3,000,000 graded volume points.  Inputs are
resident in HBM before the timed region.

Prints ONE JSON line: metric, value (pair-evals/s over greedy + volume), the
roofline of the dominant kernel, and the FP64 CPU oracle timed on the host
cores as a baseline.
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

FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector (256 CU x 64 lanes x 2 flop x 2.4 GHz)
FLOPS_PER_PAIR = 21            # canonical: 3 sub, 5 for r^2, 1 sqrt, 1 clamp, 5 for phi, 3 FMA (x2)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="wing", choices=["wing", "small", "wing-large"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-volume", type=int, default=3_000_000,
                    help="volume points in the oracle's timed sample")
    ap.add_argument("--modes", type=int, default=64,
                    help="also time Eq. 6 for this many deformation modes on the wing supports (0: skip)")
    ap.add_argument("--surfaces", type=int, default=32,
                    help="also time this many uneven independent surfaces, batched vs one at a time (0: skip)")
    ap.add_argument("--requests", type=int, default=250,
                    help="also replay a Poisson stream of this many deformation requests (20 req/s), served "
                         "with continuous batching and resident meshes vs one at a time (0: skip)")
    ap.add_argument("--warmup-requests", type=int, default=25,
                    help="requests at the start of the stream left out of the latency percentiles")
    ap.add_argument("--saturation-rate", type=float, default=80.0,
                    help="also replay the stream at this arrival rate (req/s), above one-at-a-time capacity (0: skip)")
    ap.add_argument("--m-sweep", default="1,5,10,20,40,80,107,160",
                    help="also select the wing at these group counts m (the paper's m-sweep, free Nc; '' skips)")
    ap.add_argument("--no-host-buffers", dest="host_buffers", action="store_false",
                    help="skip the PCIe-inclusive step with host inputs and output")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="before timing, one device-to-device copy of this many MiB (the known-size "
                         "kernel that scales FETCH_SIZE / WRITE_SIZE counter readings)")
    return ap.parse_args()


def kernel_source_hash(kernel_src: str) -> str:
    """sha256 prefix of the volume kernel's sources (the kernel file and its device header)."""
    import hashlib
    h = hashlib.sha256()
    for f in (kernel_src, os.path.join(os.path.dirname(kernel_src), "gcb_device.h")):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def profile_values(name: str, kernel_src: str, keys: tuple) -> dict | None:
    """`key: value` lines of a committed rocprofv3 summary under profiles/, or None when
    the kernel source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        text = open(path).read()
    except OSError:
        return None
    vals = {k.strip(): v.strip() for k, v in (l.split(":", 1) for l in text.splitlines()
                                              if l.startswith(keys + ("kernel_source_sha256_prefix:",)))}
    if vals.get("kernel_source_sha256_prefix", "") != kernel_source_hash(kernel_src):
        return None
    return vals


def measured_traffic(kernel_src: str) -> float | None:
    """Per-launch HBM bytes of the volume sweep (FETCH_SIZE + WRITE_SIZE, calibrated)."""
    vals = profile_values("volume_wing80k_traffic.md", kernel_src, ("traffic_bytes_per_launch:",))
    return float(vals["traffic_bytes_per_launch"]) if vals else None


def measured_valu(kernel_src: str) -> dict | None:
    """Issue slots per pair, the op-mix ceiling and VALUBusy of the volume sweep, and VALUBusy of the
    greedy's three kernels."""
    vals = profile_values("volume_wing80k_valu.md", kernel_src,
                          ("issue_slots_per_pair:", "op_mix_ceiling_frac:", "valu_busy_pct:",
                           "greedy_valu_busy_pct:"))
    if not vals:
        return None
    greedy = {}
    for item in vals.get("greedy_valu_busy_pct", "").split(","):
        if item.strip():
            k, v = item.split()
            greedy[k] = float(v)
    return {"issue_slots_per_pair": float(vals["issue_slots_per_pair"]),
            "op_mix_ceiling_frac": float(vals["op_mix_ceiling_frac"]),
            "valu_busy_pct": float(vals["valu_busy_pct"]), "greedy_valu_busy_pct": greedy}


def kl_divergence(xyz: np.ndarray, s1, s2) -> float:
    """KL(S1 || S2) between two support sets of the same boundary (Section 4.1, the KL
    equation): sum over boundary nodes i of d1_i log(d1_i / d2_i), with dk_i the distance
    from node i to the nearest node of Sk.  A node of either set has a zero distance, which
    makes its term 0 log 0 or x log(x / 0); such terms are left out of the sum."""
    from scipy.spatial import cKDTree
    d1, _ = cKDTree(xyz[np.asarray(s1)]).query(xyz)
    d2, _ = cKDTree(xyz[np.asarray(s2)]).query(xyz)
    ok = (d1 > 0.0) & (d2 > 0.0)
    return float(np.sum(d1[ok] * np.log(d1[ok] / d2[ok])))


def problem(name):
    import synth
    if name == "small":
        return synth.config_small_ellipsoid()
    if name == "wing-large":
        return synth.config_wing_large()
    return synth.config_wing()


def host_cpu() -> dict:
    """Model name and usable core count of the host the oracle runs on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"model": model, "cpu_count": os.cpu_count(), "usable_cores": usable}


def cpu_baseline(p, nv_sample, nv_single=300_000):
    """The FP64 oracle as it stands, on all host cores: full greedy + a volume sample, with the
    greedy (t1 + t2) and volume (t3) phases timed apart; then one thread on the same greedy and a
    smaller volume sample.  Returns the baseline record and the oracle's all-core results
    (support set, sampled displacements)."""
    import oracle
    threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    r = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed, nthreads=threads)
    t1 = time.perf_counter()
    vol = p.volume[:nv_sample]
    ref = oracle.interpolate(p.xyz[r.S], r.W, p.radius, vol, nthreads=threads)
    t2 = time.perf_counter()
    pg = r.pairs_group + r.pairs_append
    pv = vol.shape[0] * r.nc
    rec = {"value": (pg + pv) / (t2 - t0), "unit": "pair-evals/s", "cores": threads, "kind": "oracle",
           "sample": f"full greedy (Nb={p.nb}, m={p.m}, Nc={r.nc}, {r.iterations} iterations, {t1 - t0:.2f} s) "
                     f"+ Eq. 6 at {vol.shape[0]} volume points ({t2 - t1:.2f} s)",
           "seconds": t2 - t0,
           "phases": {"greedy": {"seconds": t1 - t0, "pair_evals_per_s": pg / (t1 - t0)},
                      "volume": {"seconds": t2 - t1, "pair_evals_per_s": pv / (t2 - t1)}},
           "host": host_cpu()}
    if nv_single > 0:
        s0 = time.perf_counter()
        r1 = oracle.select(p.xyz, p.disp, p.radius, p.m, p.tol_abs, seed=p.seed, nthreads=1)
        s1 = time.perf_counter()
        vol1 = p.volume[:min(nv_single, p.volume.shape[0])]
        oracle.interpolate(p.xyz[r1.S], r1.W, p.radius, vol1, nthreads=1)
        s2 = time.perf_counter()
        pg1 = r1.pairs_group + r1.pairs_append
        pv1 = vol1.shape[0] * r1.nc
        rec["single_thread"] = {"value": (pg1 + pv1) / (s2 - s0), "cores": 1,
                                "sample": f"full greedy + Eq. 6 at {vol1.shape[0]} volume points",
                                "phases": {"greedy": {"seconds": s1 - s0, "pair_evals_per_s": pg1 / (s1 - s0)},
                                           "volume": {"seconds": s2 - s1, "pair_evals_per_s": pv1 / (s2 - s1)}}}
    return rec, r, ref


def certify_sequence(ctx, p, S_gpu) -> dict:
    """Follow-mode replay of the context's last selection by the oracle: every iteration's group, its
    argmax within tau = 1e-9 max|d| of the oracle's own maximum, and every append decision; continuing from
    the GPU's choices, so a legitimate near-tie divergence is certified rather than counted as an error."""
    import oracle
    log = ctx.get_log()
    tau = 1e-9 * p.max_disp
    bad, reason, gap = oracle.validate(p.xyz, p.disp, p.radius, p.m, p.tol_abs, S_gpu[:3], log.group, log.node,
                                       log.appended, tau, seed=p.seed, nthreads=os.cpu_count() or 1)
    return {"certified": bad < 0, "first_bad_iteration": bad, "reason": reason, "max_gap_rel_max_d": gap / p.max_disp,
            "tau_rel_max_d": 1e-9, "iterations": int(len(log.group))}


def multi_surface(count, dev, vs_oracle=False):
    """Uneven independent surfaces (Nb log-uniform in [1e3, 5e4], Nv = 25 Nb), each selected and
    deformed: one context at a time vs one batch (shared launches); with vs_oracle, the batch's
    support sets, certificates and sampled displacements against the FP64 oracle."""
    import torch
    import synth
    import paper_2004_04817_amd as gcb
    probs = synth.config_multi_surface(count, with_volume=True)
    vols = [torch.from_numpy(q.volume).to(dev) for q in probs]
    samples = [q.volume[:: max(1, q.volume.shape[0] // 2000)] for q in probs] if vs_oracle else None
    for q in probs:
        q.volume = None
    ctxs = []
    for q in probs:
        c = gcb.Context(0)
        c.set_boundary(torch.from_numpy(q.xyz).to(dev), torch.from_numpy(q.disp).to(dev))
        c.set_params(q.radius, q.m, q.tol_abs, seed=q.seed)
        ctxs.append(c)
    outs = [torch.empty_like(v) for v in vols]

    def one_at_a_time():
        infos = []
        for c, v, o in zip(ctxs, vols, outs):
            infos.append(c.select())
            c.deform(v, out=o)
        return infos

    # tile shapes of the batched launches picked by the autotuner on this device and workload
    from paper_2004_04817_amd import autotune
    best, times = autotune.tune_batch(ctxs)
    batch = gcb.Batch(0)
    batch.set_layout(*best)

    def batched():
        infos = batch.select(ctxs)
        batch.deform(ctxs, vols, outs)
        return infos

    res = {}
    for name, fn in (("one_at_a_time", one_at_a_time), ("batched", batched)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        pairs = sum(i["pairs_group"] + i["pairs_append"] + v.shape[0] * i["nc"] for i, v in zip(infos, vols))
        res[name] = {"ms": 1e3 * dt, "pair_evals_per_s": pairs / dt,
                     "iterations_max": max(i["iterations"] for i in infos),
                     "iterations_sum": sum(i["iterations"] for i in infos),
                     "all_converged": all(bool(i["converged"]) for i in infos)}
    res["speedup"] = res["one_at_a_time"]["ms"] / res["batched"]["ms"]
    if vs_oracle:
        import oracle
        same, cert, verr = 0, 0.0, 0.0
        for q, c, o, smp in zip(probs, ctxs, outs, samples):
            r = oracle.select(q.xyz, q.disp, q.radius, q.m, q.tol_abs, seed=q.seed, nthreads=16)
            S, _ = c.get_support()
            same += int(list(S) == list(r.S))
            cert = max(cert, abs(c.certify()[0] - r.final_max_err) / max(r.final_max_err, 1e-300))
            step = max(1, o.shape[0] // 2000)
            ref = oracle.interpolate(q.xyz[r.S], r.W, q.radius, smp, nthreads=16)
            verr = max(verr, float(np.abs(o[::step].cpu().numpy() - ref).max()) / q.max_disp)
        res["vs_oracle"] = {"same_support_sets": same, "surfaces": count,
                            "certificate_rel_diff_max": cert, "volume_max_err_rel_max_d": verr,
                            "volume_points_compared_per_surface": "about 2,000 (every k-th point)"}
    res["autotune"] = {"chosen": {"sweep_targets_per_lane": best[0], "factor_chunks_per_wave": best[1]},
                       "select_ms": {f"tpl{c[0]}_rpw{c[1]}": 1e3 * t for c, t in times.items()},
                       "note": "0 = automatic (narrow layouts below 4 running surfaces, wide above)"}
    res.update({"surfaces": count, "nb_sum": sum(q.nb for q in probs), "nv_sum": sum(v.shape[0] for v in vols),
                "precision": "fp64"})
    batch.close()
    for c in ctxs:
        c.close()
    return res


def serving_section(n_requests, dev, warmup_requests=25, rate=20.0, sat_rate=0.0):
    """Poisson stream (sizes of the uneven batch, 20 % repeats with new fields),
    latency arrival -> output complete: served (continuous batching, resident
    meshes, warm starts) vs plain FP64 one at a time (FIFO)."""
    import synth
    import paper_2004_04817_amd as gcb
    from paper_2004_04817_amd import serving
    stream = synth.config_requests(n_requests, rate=rate, repeat_p=0.2)
    items = serving.materialise(stream)
    max_nv = 25 * max(i[1].nb for i in items)
    pool = serving.volume_pool(max_nv, dev)
    res = {"requests": n_requests, "warmup_requests": warmup_requests, "rate_per_s": rate, "repeat_p": 0.2,
           "nv_per_nb": 25, "precision": "fp64"}
    modes = (("served", dict(max_active=32, flags=gcb.GCB_SERVE_BATCH | gcb.GCB_SERVE_CACHE)),
             ("one_at_a_time", dict(max_active=1, flags=0)))
    for name, kw in modes:
        with gcb.Server(0, hbm_budget=64 << 30, **kw) as srv:
            served = serving.replay(srv, items, pool, nv_per_nb=25, iterations=48)
            res[name] = serving.latency_summary(served, skip=warmup_requests)
    if sat_rate > 0:
        # the same requests arriving faster than one-at-a-time service can keep up with
        scale = rate / sat_rate
        fast = [(type(i[0])(i[0].t * scale, i[0].key, i[0].nb, i[0].field_seed),) + tuple(i[1:]) for i in items]
        sat = {"rate_per_s": sat_rate}
        for name, kw in modes:
            with gcb.Server(0, hbm_budget=64 << 30, **kw) as srv:
                served = serving.replay(srv, fast, pool, nv_per_nb=25, iterations=48)
                sat[name] = serving.latency_summary(served, skip=warmup_requests)
        res["saturation"] = sat
    del pool
    return res


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; use --gpus 1"}))
        sys.exit(2)
    import torch
    import paper_2004_04817_amd as gcb

    p = problem(a.config)
    dev = torch.device("cuda:0")
    xyz = torch.from_numpy(p.xyz).to(dev)
    disp = torch.from_numpy(p.disp).to(dev)
    vol = torch.from_numpy(p.volume).to(dev)
    out = torch.empty_like(vol)
    nv = vol.shape[0]
    ctx = gcb.Context(0)
    ctx.set_boundary(xyz, disp)
    ctx.set_params(p.radius, p.m, p.tol_abs, seed=p.seed)
    stream = torch.cuda.current_stream(dev)
    if a.calib_copy_mb > 0:
        src = torch.empty(a.calib_copy_mb << 17, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        info = ctx.select()
        ctx.deform(vol, out=out)
        return info

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    step_ms, vol_ms, infos = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        ts = time.perf_counter()
        info = step()
        torch.cuda.synchronize()
        step_ms.append(1e3 * (time.perf_counter() - ts))
        # HIP events the library records on its stream around the volume kernels (host latency excluded)
        vol_ms.append(ctx.deform_time())
        infos.append(info)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    info = infos[-1]
    nc = info["nc"]
    pairs_greedy = info["pairs_group"] + info["pairs_append"]
    pairs_volume = nv * nc
    value = a.steps * (pairs_greedy + pairs_volume) / total
    vol_avg_ms = float(np.mean(vol_ms))
    achieved = FLOPS_PER_PAIR * pairs_volume / (vol_avg_ms * 1e-3) / 1e12
    rec = {
        "metric": "RBF pair-evals/s (greedy+volume); deform latency p50/p99 vs plain FP64 GPU",
        "value": value,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * total / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": p.name + f"+volume{nv}", "nb": p.nb, "nv": nv, "m": p.m, "radius": p.radius,
                   "tol_abs": p.tol_abs, "tol_rel": p.tol_rel, "nc": nc, "iterations": info["iterations"],
                   "precision": "fp64", "parallelism": "single-gpu"},
        "phases_ms": {"select": float(np.mean([i["ms_select"] for i in infos])), "volume": vol_avg_ms},
        "phase_pair_evals_per_s": {
            "greedy": pairs_greedy / (1e-3 * float(np.mean([i["ms_select"] for i in infos]))),
            "volume": pairs_volume / (1e-3 * vol_avg_ms)},
        "pairs": {"group": info["pairs_group"], "append": info["pairs_append"], "volume": pairs_volume,
                  "certificate": info["pairs_cert"]},
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "accuracy": {"final_max_err": info["final_max_err"], "final_rms_err": info["final_rms_err"],
                     "converged": bool(info["converged"])},
        "roofline": {"kernel": "k_volume64<double,double>", "bound": "alu", "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": (measured_traffic(os.path.join(ROOT, "paper_2004_04817_amd", "csrc",
                                                               "gcb_kernels.hip")) if a.config == "wing" else None),
                     "flops_per_pair": FLOPS_PER_PAIR, "pairs_per_launch": pairs_volume,
                     "launch_ms": vol_avg_ms},
    }
    valu = measured_valu(os.path.join(ROOT, "paper_2004_04817_amd", "csrc", "gcb_kernels.hip"))
    greedy_busy = valu.pop("greedy_valu_busy_pct") if valu else None
    if valu and a.config == "wing":
        # the instruction mix caps the fraction of peak: 21 flops per pair over 2 flops per issue slot
        valu["frac_of_op_mix_ceiling"] = (achieved / FP64_PEAK_TFLOPS) / valu["op_mix_ceiling_frac"]
        rec["roofline"]["instruction_mix"] = valu
    # the greedy phase: one iteration is three dependent launches; the VALUs are nearly idle in them
    rec["greedy_iteration"] = {"bound": "latency", "kernels_per_iteration": 3,
                               "us_per_iteration": 1e3 * rec["phases_ms"]["select"] / info["iterations"],
                               "valu_busy_pct": greedy_busy if a.config == "wing" else None}
    # dense FP64 refactorisation of the selected support system (blocked Cholesky + triangular inverse, MFMA)
    drift, rinfo = ctx.refactor()        # against the incrementally grown factor
    _, rinfo = ctx.refactor()            # timed again with warm caches
    rflops = 2.0 * nc ** 3 / 3.0
    rec["refactor"] = {"nc": nc, "ms": rinfo["ms_select"], "drift": drift,
                       "tflops": rflops / (rinfo["ms_select"] * 1e-3) / 1e12,
                       "flops": "Nc^3/3 (Cholesky) + Nc^3/3 (triangular inverse)"}
    ctx.set_params(p.radius, p.m, p.tol_abs, seed=p.seed)
    ctx.select()
    # Eq. (6) in FP32 (GCB_PREC_FP32_EVAL) on the same supports: time and error against the FP64 output
    ctx.set_params(p.radius, p.m, p.tol_abs, seed=p.seed, precision=gcb.GCB_PREC_FP32_EVAL)
    ctx.select()
    out32 = torch.empty_like(vol)
    ctx.deform(vol, out=out32)
    ts = []
    for _ in range(3):
        ctx.deform(vol, out=out32)
        torch.cuda.synchronize()
        ts.append(ctx.deform_time())
    ms32 = float(np.mean(ts))
    err32 = float((out32 - out).abs().max().item()) / p.max_disp
    rec["volume_fp32_eval"] = {"ms": ms32, "pair_evals_per_s": pairs_volume / (ms32 * 1e-3),
                               "speedup_vs_fp64": vol_avg_ms / ms32, "max_err_vs_fp64_rel_max_d": err32,
                               "meets_1e-6_max_d": err32 <= 1e-6}
    del out32
    ctx.set_params(p.radius, p.m, p.tol_abs, seed=p.seed)
    ctx.select()
    if a.host_buffers:
        # the same step with the inputs and the output in host memory (pageable numpy arrays): boundary copied in,
        # selection, volume points copied in and displacements copied out; never the headline value
        hctx = gcb.Context(0)
        hout = np.empty_like(p.volume)
        hs = []
        for r in range(3):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            hctx.set_boundary(p.xyz, p.disp)
            hctx.set_params(p.radius, p.m, p.tol_abs, seed=p.seed)
            hinfo = hctx.select()
            hctx.deform(p.volume, out=hout)
            torch.cuda.synchronize()
            if r > 0:
                hs.append(time.perf_counter() - ts)
        hsec = float(np.mean(hs))
        rec["host_buffers"] = {"ms_per_step": 1e3 * hsec,
                               "pair_evals_per_s": (hinfo["pairs_group"] + hinfo["pairs_append"] + nv * nc) / hsec,
                               "bytes_in": int(p.xyz.nbytes + p.disp.nbytes + p.volume.nbytes),
                               "bytes_out": int(hout.nbytes),
                               "what": "PCIe-inclusive step: host boundary and volume in, host displacements out"}
        hctx.close()
        del hout
    if a.modes > 0 and a.config == "wing":
        import synth
        modes = torch.from_numpy(synth.config_modes(p, a.modes)).to(dev)
        mout = torch.empty((nv, 3 * a.modes), dtype=torch.float64, device=dev)
        ctx.deform_multi(modes, vol, out=mout)   # warm-up
        ts = []
        for _ in range(2):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.deform_multi(modes, vol, out=mout)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.mean(ts))
        rhs = 3 * a.modes
        flops = (2.0 * rhs + 15.0) * nv * nc   # matrix-core FMAs + the phi evaluation per pair
        mvs = None
        if not a.no_cpu_baseline:
            # sampled points of the 192-column output against the oracle's solve on the same support set
            import oracle
            S_m, _ = ctx.get_support()
            mh = modes.cpu().numpy()
            Wo = oracle.solve_on_support(p.xyz, S_m, p.radius, mh)
            step = max(1, nv // 20000)
            ref = oracle.interpolate(p.xyz[S_m], Wo, p.radius, p.volume[::step], nthreads=16)
            got = mout[::step].cpu().numpy()
            scale = float(np.abs(mh).max())
            mvs = {"points_compared": int(ref.shape[0]), "max_err_rel_max_mode": float(np.abs(got - ref).max()) / scale,
                   "rms_err_rel_max_mode": float(np.sqrt(np.mean((got - ref) ** 2))) / scale}
        # each mode's interpolation error at all nb boundary nodes (Eq. 3 holds only on S: the support set was
        # selected for the benchmark field, so no tolerance is claimed for the modes)
        bout = torch.empty((p.nb, rhs), dtype=torch.float64, device=dev)
        ctx.deform_multi(modes, xyz, out=bout)
        e = torch.linalg.vector_norm((bout - modes).reshape(p.nb, a.modes, 3), dim=2).max(dim=0).values
        peak = torch.linalg.vector_norm(modes.reshape(p.nb, a.modes, 3), dim=2).max(dim=0).values
        rel = (e / peak).cpu().numpy()
        all_node = {"max_err_rel_max_mode": {"min": float(rel.min()), "median": float(np.median(rel)),
                                             "max": float(rel.max())}, "nodes": p.nb}
        del bout
        rec["modes"] = {"k_modes": a.modes, "rhs": rhs, "nv": nv, "nc": nc, "ms": ms, "vs_oracle": mvs,
                        "all_node_error": all_node,
                        "pair_evals_per_s": nv * nc / (ms * 1e-3),
                        "roofline": {"kernel": "k_volume_multi<double,double> (+ weight TRMMs)", "bound": "mfma",
                                     "achieved": flops / (ms * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
                                     "unit": "TFLOP/s", "frac": flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS}}
        del mout, modes
    if a.m_sweep and a.config == "wing":
        # GCB group count m against the traditional greedy (m = 1), free Nc, same E* (Tables 3 and 6 protocol)
        rows = []
        for m in [int(x) for x in a.m_sweep.split(",")]:
            ctx.set_params(p.radius, m, p.tol_abs, seed=p.seed)
            ctx.select()
            inf = ctx.select()
            rows.append({"m": m, "nc": inf["nc"], "iterations": inf["iterations"], "select_ms": inf["ms_select"],
                         "pairs_greedy": inf["pairs_group"] + inf["pairs_append"],
                         "converged": bool(inf["converged"])})
        base = next((r["select_ms"] for r in rows if r["m"] == 1), None)
        for r in rows:
            r["speedup_vs_m1"] = base / r["select_ms"] if base else None
        # fixed Nc (Tables 2 and 5 protocol): E* = 0, every m selects exactly Nc^max supports
        nc_fixed = 1100
        fixed, sets = [], {}
        for m in [int(x) for x in a.m_sweep.split(",")]:
            ctx.set_params(p.radius, m, 0.0, nc_max=nc_fixed, seed=p.seed)
            ctx.select()
            inf = ctx.select()
            sets[m] = ctx.get_support()[0]
            fixed.append({"m": m, "nc": inf["nc"], "iterations": inf["iterations"], "select_ms": inf["ms_select"],
                          "final_max_err_rel": inf["final_max_err"] / p.max_disp})
        fbase = next((r["select_ms"] for r in fixed if r["m"] == 1), None)
        for r in fixed:
            r["speedup_vs_m1"] = fbase / r["select_ms"] if fbase else None
        # distribution of the support nodes against the traditional greedy's (Table 4 analog): KL(m = 1 || m),
        # and two seeded random sets of the same size
        kl = None
        if 1 in sets:
            kl = {f"m{m}": kl_divergence(p.xyz, sets[1], S) for m, S in sets.items() if m != 1}
            for r_id in (1, 2):
                rnd = np.random.default_rng(1000 + r_id).choice(p.nb, size=nc_fixed, replace=False)
                kl[f"random{r_id}"] = kl_divergence(p.xyz, sets[1], rnd)
        # error history of the benchmark selection (all-node max and RMS every m iterations; Figs. 4-7 analog)
        ctx.set_params(p.radius, p.m, p.tol_abs, seed=p.seed, monitor_every=p.m)
        ctx.select()
        it_h, mx_h, rm_h = ctx.get_monitor()
        log_h = ctx.get_log()
        nc_at = np.cumsum(log_h.appended.astype(np.int64)) + 3
        pick = np.unique(np.linspace(0, len(it_h) - 1, 8).astype(int)) if len(it_h) else []
        history = [{"iteration": int(it_h[i]), "nc": int(nc_at[it_h[i] - 1]), "max_err_rel": float(mx_h[i] / p.max_disp),
                    "rms_err_rel": float(rm_h[i] / p.max_disp)} for i in pick]
        rec["m_sweep"] = {"free_nc": rows, "fixed_nc": {"nc": nc_fixed, "rows": fixed, "kl_vs_m1": kl},
                          "history_m107": history}
        ctx.set_params(p.radius, p.m, p.tol_abs, seed=p.seed)
        ctx.select()
    if a.surfaces > 0:
        rec["multi_surface"] = multi_surface(a.surfaces, dev, vs_oracle=not a.no_cpu_baseline)
    if a.requests > 0:
        rec["serving"] = serving_section(a.requests, dev, warmup_requests=a.warmup_requests,
                                         sat_rate=a.saturation_rate)
        rec["latency_ms"] = {"p50": rec["serving"]["served"]["p50_ms"], "p99": rec["serving"]["served"]["p99_ms"],
                             "p50_one_at_a_time_fp64": rec["serving"]["one_at_a_time"]["p50_ms"],
                             "p99_one_at_a_time_fp64": rec["serving"]["one_at_a_time"]["p99_ms"],
                             "what": "deformation request latency, arrival to output complete"}
    if not a.no_cpu_baseline:
        base, r_orc, ref = cpu_baseline(p, min(a.cpu_sample_volume, nv))
        rec["cpu_baseline"] = base
        # the benchmark's own outputs against the FP64 oracle (same inputs)
        S_gpu, _ = ctx.get_support()
        o = out[: ref.shape[0]].cpu().numpy()
        err = np.sqrt(((o - ref) ** 2).sum(axis=1))
        S_orc = np.asarray(r_orc.S)
        k = min(len(S_gpu), len(S_orc))
        diff = np.nonzero(np.asarray(S_gpu[:k]) != S_orc[:k])[0]
        rec["accuracy"]["vs_oracle"] = {
            "same_support_sequence": bool(np.array_equal(S_gpu, S_orc)),
            "identical_prefix": int(diff[0]) if diff.size else k,
            "nc_gpu": int(len(S_gpu)), "nc_oracle": int(len(S_orc)),
            "gpu_sequence_certified": certify_sequence(ctx, p, S_gpu),
            "volume_points_compared": int(ref.shape[0]),
            "volume_max_err_rel_max_d": float(err.max() / p.max_disp),
            "volume_rms_err_rel_max_d": float(np.sqrt((err ** 2).mean()) / p.max_disp),
            "oracle_final_max_err": r_orc.final_max_err}
    print(json.dumps(rec), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
