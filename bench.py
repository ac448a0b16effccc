"""Benchmark: converged pixel retrievals per second at 284 bands on one MI355X.

Workload (default): the clustered-fire scene, 1,234 cross-track x 2,048 lines =
2,527,232 pixels x 284 bands float32 radiance (3 % fire pixels in smoothed
blobs, the rest f = 0 background), synthetic and seeded.  One step = scene
setup (band resampling) + warm-start network inference (BF16 matrix cores)
+ Levenberg-Marquardt retrieval of every pixel from the network's start
with fallback to the default start (FP32 forward model / Jacobian /
reductions, FP64 damped solves), radiance already resident in HBM.  The
network is trained once for the scene's atmosphere before the timed steps
(its time is reported, not included).  The plain LM from the default start
is run and reported beside it.

Prints one JSON line (see the keys below).  --gpus N > 1 is refused: this
build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Roofline of the dominant kernel: FP32 vector ALU.  MI355X's published FP32
# vector peak is 157.3 TFLOP/s = 78.6e12 FMA lanes/s (256 CUs x 4 SIMDs x 32
# lanes x 2.4 GHz).  Instructions are weighted by their issue cost in FMA
# equivalents as measured on this GPU by ff_valu_rates (bench.py --workload
# valu-rates; profiles/valu_rates_mi355x.md): a 32-bit FMA or other simple
# FP32 op 1, exp2 3.29, rcp 3.33, an FP64 FMA/add/mul 1.92, a float<->double
# conversion 1.68.  (The same run measures a 32-bit FMA at 60.7e12 lanes/s
# without packed instructions, 77 % of the published peak.)
PEAK_FMA32 = 256 * 4 * 32 * 2.4e9
MEASURED_FMA32 = 60.7e12
UNIT_FMA = "T FP32-FMA-equivalent lane-ops/s"
OP_FMA = "issue cost in 32-bit FMA equivalents (measured: exp2 3.29, rcp 3.33, FP64 op 1.92, conversion 1.68)"
W_EXP2, W_RCP, W_F64, W_CVT = 3.29, 3.33, 1.92, 1.68
HBM_PEAK = 8.0e12
# MI355X's published FP32 vector peak in flops (an FMA is 2)
PEAK_FP32_PUBLISHED = 157.3e12

# HBM bytes per launch of the retrieval kernel on this workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; each scaled by what the
# counter reads for a 1 GiB device copy: x2.000 and x1.000), recorded in
# profiles/lm_kernel_fp32_q32_clustered_fire_2p53M.md.  They describe the
# kernel sources with the SHA-1 below; any other source reports null.
TRAFFIC_SOURCES = ("paper_2608_07580_amd/csrc/lm.hip", "paper_2608_07580_amd/csrc/solve.hpp",
                   "paper_2608_07580_amd/csrc/physics.hpp", "paper_2608_07580_amd/csrc/ff_internal.hpp")
TRAFFIC_SHA1 = "aaabbb54cc282686ea010bf61436005a3b6c5981"
TRAFFIC_BYTES = {"plain": 85.49e9, "warm": 83.74e9}


def measured_traffic(leg: str):
    import hashlib
    h = hashlib.sha1()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return TRAFFIC_BYTES[leg] if h.hexdigest() == TRAFFIC_SHA1 else None


# Issue cost of one Planck node (x = a u, 2^x - 1, three FMAs and one product
# for the three quadrature sums, the exponential and the reciprocal) and of
# the FP64 residual per band and pixel (ten FP64 operations for rho, 1 - S rho,
# the Newton step of the reciprocal, the solar term, the residual and
# F += r^2, four conversions and the reciprocal seed, less the FP32 solar
# term's 5), in 32-bit FMA equivalents.
NODE_W = 7 + W_EXP2 + W_RCP
RESIDUAL64_W = 10 * W_F64 + 4 * W_CVT + W_RCP - 5


def nodes_evaluated(n_quad: int) -> int:
    """Nodes of the Q-node Gauss-Hermite rule the FP32 lognormal sums
    evaluate: the coldest nodes, whose weights are below 2^-32 of the largest,
    contribute less than the sums' FP32 rounding and are left out (5 of 32,
    2 of 24)."""
    return n_quad - {32: 5, 24: 2}.get(n_quad, 0)


# Issue cost the one-component kernel does not spend per band when the
# scene's spherical albedo S is 0 on every band (1 - S rho is then exactly 1):
# in FP32 the reflectance, 1 - S rho, its reciprocal and the two products by
# it (5); in FP64 1 - S rho, the two Newton FMAs, the two conversions around
# the FP32 seed and the seed.
S0_SAVED_W = 5 + 3 * W_F64 + 2 * W_CVT + W_RCP


def slots_per_eval(n_bands: int, n_quad: int, model: int = 1, s_zero: bool = False) -> float:
    """Issue cost, in 32-bit FMA equivalents, of one model + Jacobian +
    reduction evaluation of one pixel: NODE_W per (band, evaluated node) and component;
    per band and component 5 for the scaling (one of them the reciprocal of
    1 - S rho, counted as simple here), plus 19 (n = 5) / 49 (n = 8) for the
    solar term, basis, residual and the J^T J, J^T r, r.r accumulations, and
    the FP64 residual's RESIDUAL64_W; less S0_SAVED_W for the one-component
    model on a scene with S = 0 on every band (s_zero)."""
    if model == 4:
        # one component; the endmember surface: 5 FMAs for rho and 5 basis
        # products where the linear surface has 2 and 2 (25), the n = 8
        # accumulations (45), and four more FP64 FMAs for the FP64 reflectance
        return n_bands * (NODE_W * nodes_evaluated(n_quad) + 5 + 25 + 45 + RESIDUAL64_W + 4 * W_F64 + 4)
    comps = 1 if model == 1 else 2
    per_band = comps * (NODE_W * nodes_evaluated(n_quad) + 5) + (19 + 21 if model == 1 else 49 + 45) + RESIDUAL64_W
    if s_zero and model == 1:
        per_band -= S0_SAVED_W
    return n_bands * per_band


def flops_per_eval(n_bands: int, n_quad: int, s_zero: bool = False) -> int:
    """Floating-point operations of one evaluation of the one-component model
    (FMA = 2, exp2 and rcp = 1 each): per (band, evaluated node) x = a u (1), 2^x (1),
    - 1 (1), rcp (1), three FMAs and q q + q (8), x (...) (1) = 13; per band
    72 for the reflectance, the basis, the FP64 solar term and residual and
    the J^T J, J^T r, r.r accumulations (58 when S = 0 on every band: the
    FP32 reflectance, 1 - S rho twice, the two reciprocals, the Newton step
    and the two products by the reciprocal are not needed)."""
    return n_bands * (13 * nodes_evaluated(n_quad) + (58 if s_zero else 72))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(args, dev):
    import torch
    import paper_2608_07580_amd as ff
    import scenegen
    atm = scenegen.make_atmosphere(1, 0)
    t0 = time.time()
    states, fire = scenegen.config1_states(args.lines, args.cross, scene=0)
    P = states.shape[0]
    scene = ff.Scene(atm)
    B = scene.n_bands
    lt = torch.empty((P, B), dtype=torch.float32, device=dev)
    chunk = 1 << 18
    for s in range(0, P, chunk):
        st = torch.tensor(states[s:s + chunk], dtype=torch.float32, device=dev)
        lt[s:s + chunk] = ff.forward(scene, st, 1)
    noise = scenegen.noise_normals(1, 0, P, B)
    rad = torch.empty_like(lt)
    for s in range(0, P, chunk):
        n = torch.from_numpy(noise[s:s + chunk]).to(dev)
        rad[s:s + chunk] = lt[s:s + chunk] * (1.0 + n / args.snr)
    del lt
    torch.cuda.synchronize()
    log(f"workload: {P} px x {B} bands, {fire.sum()} fire px, built in {time.time() - t0:.1f}s")
    return atm, scene, states, fire, noise, rad


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


PARITY_KEYS = ("both", "same_min", "same_frac", "t_n", "dT_max", "dT_p99", "f_n", "df_max", "drrr_max_same",
               "dT_over_tol", "df_over_tol", "cov_sd_rel_max", "cov_corr_max", "cov_n", "determined",
               "loss_worse_determined", "dchi2_max_determined", "flat", "flat_worse_0.001", "flat_better_0.001",
               "flat_worse_0.1", "flat_better_0.1", "flat_worse_1", "flat_better_1")


def cpu_baseline(args, atm, rad, states, gpu_legs):
    """The FP64 oracle on a seeded subsample of the same scene, on this host,
    fed the GPU's own float32 radiance rows (the same input both retrieve);
    the GPU legs' results on the same pixels are compared with it under the
    tests' parity gate."""
    import torch
    import oracle
    import scenegen
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _helpers import parity_report
    P = states.shape[0]
    idx = scenegen.subsample(1, 0, P, args.cpu_sample)
    tab = oracle.band_tables(atm)
    lobs = rad[torch.from_numpy(idx).to(rad.device)].cpu().numpy()
    lo, hi, x0 = scenegen.default_prior(1)
    cores = len(os.sched_getaffinity(0))
    t0 = time.time()
    r = oracle.retrieve(tab, lobs, 1, lo, hi, x0, nthreads=cores)
    dt = time.time() - t0
    conv = int(r.converged.sum())
    parity = {}
    for name, res in gpu_legs.items():
        rep = parity_report({k: v[idx] for k, v in res.items() if v is not None}, r, 1, tab, lobs)
        parity[name] = {k: rep[k] for k in PARITY_KEYS if k in rep}
        parity[name]["gpu_converged"] = int(((res["status"][idx] & 7) != 0).sum())
    return {"value": conv / dt, "unit": "converged retrievals/s", "cores": cores, "cpu": cpu_model(),
            "kind": "oracle",
            "sample": f"seeded uniform subsample of {len(idx)} of the {P} scene pixels "
                      f"({int((states[idx, 0] > 0).sum())} fire), the GPU's own float32 radiance rows, "
                      f"FP64 LM from the default start, {dt:.1f} s wall, {conv} converged, "
                      f"mean {r.iters.mean():.1f} iterations",
            "gpu_vs_oracle": parity}


def train_network(args, atm, dev):
    """Warm-start network for this scene's atmosphere, trained on spectra the
    forward model generates (one-time setup per atmosphere, not timed)."""
    import torch
    import paper_2608_07580_amd as ff
    sc = ff.Scene(atm)
    prior = ff.default_prior(1)
    net = ff.WarmStart(seed=args.seed)
    torch.cuda.synchronize()
    t0 = time.time()
    nrad, _ = ff.generate(sc, prior, args.seed + 1000, 0, 16384, bg_fraction=args.bg_fraction)
    net.fit_normalization(nrad)
    hist = net.train(sc, prior, steps=args.train_steps, batch=args.train_batch, seed=args.seed,
                     bg_fraction=args.bg_fraction, lr=1e-3, lr_final=1e-5)
    torch.cuda.synchronize()
    dt = time.time() - t0
    h = hist.cpu().numpy()
    info = {"train_s": dt, "samples": args.train_steps * args.train_batch, "steps": args.train_steps,
            "batch": args.train_batch, "bg_fraction": args.bg_fraction,
            "loss_first": float(h[:20].mean()), "loss_last": float(h[-50:].mean())}
    sc.close()
    log(f"network trained on {info['samples']} spectra in {dt:.2f}s, loss {info['loss_first']:.4g} -> "
        f"{info['loss_last']:.4g}")
    return net, info


def run_leg(args, atm, rad, stream, net):
    """Warmup + timed steps of one path; returns timing and outputs."""
    import torch
    import paper_2608_07580_amd as ff
    P = rad.shape[0]
    prior = ff.default_prior(1)
    opts = ff.default_options(n_quad=args.n_quad)
    tuned = None
    if not args.no_tune:
        # launch shape from the tuner's table (tuned on this batch on a miss)
        sc = ff.Scene(atm)
        z0 = net.infer_routed(sc, rad, stream=stream)[0] if net is not None else None
        with torch.cuda.stream(stream):
            opts, tms = ff.tune([sc], [rad], prior, z0s=None if z0 is None else [z0], options=opts,
                                cache_path=args.tune_cache, retune=args.retune, stream=stream)
        torch.cuda.synchronize()
        sc.close()
        del z0
        tuned = {"lanes_per_pixel": opts.lanes_per_pixel, "block_size": opts.block_size,
                 "blocks_per_cu": opts.blocks_per_cu, "schedule": opts.schedule, "tuned_ms": tms}
        log(f"tuned launch: {tuned}")
    outs = ff.allocate_outputs(P, 1, rad.device)
    evals = torch.zeros(1, dtype=torch.int64, device=rad.device)
    live = []      # scene tables must outlive the asynchronous launches that read them
    lm_events = []

    def step(timed):
        sc = ff.Scene(atm)
        z0 = net.infer_routed(sc, rad, stream=stream)[0] if net is not None else None
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ff.retrieve(sc, rad, prior, z0=z0, options=opts, outputs=outs, evals=evals, stream=stream)
        b.record(stream)
        if timed:
            lm_events.append((a, b))
        live.append((sc, z0))

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step(False)
        torch.cuda.synchronize()
        evals.zero_()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.time()
        ev0.record(stream)
        for _ in range(args.steps):
            step(True)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.time() - t0
    for sc, _ in live:
        sc.close()
    ms = ev0.elapsed_time(ev1) / args.steps
    lm_ms = sum(a.elapsed_time(b) for a, b in lm_events) / len(lm_events)
    res = outs.numpy()
    st = res["status"].astype(np.int64)
    conv = int(((st & ff.ST_CONVERGED) != 0).sum())
    it = res["iters"]
    leg = {"converged": conv, "pixels": P, "converged_per_s": conv / (ms * 1e-3), "ms_per_step": ms,
           "lm_kernel_ms": lm_ms, "wall_s_per_step": wall / args.steps,
           "evals_per_pixel": int(evals.item()) / args.steps / P,
           "mean_iters": float(it.mean()), "p99_iters": float(np.percentile(it, 99)),
           "max_iters": int(it.max()), "launch": tuned}
    if net is not None:
        leg["fallback_rate"] = float(((st & ff.ST_USED_FALLBACK) != 0).mean())
    return leg, res, int(evals.item()) / args.steps


def run_valu_rates(args):
    """ff_valu_rates on this GPU: each instruction's sustained lane rate and
    its weight in issue slots (the 32-bit FMA rate is one slot)."""
    import torch
    import paper_2608_07580_amd as ff
    torch.cuda.init()
    rates = ff.valu_rates()
    fma = rates["fma_f32"]
    out = {"workload": "valu-rates", "lane_ops_per_s": rates,
           "slots": {k: fma / v for k, v in rates.items()},
           "fma_f32_frac_of_published_peak": fma / PEAK_FMA32,
           "published_fma_lanes_per_s": PEAK_FMA32}
    print(json.dumps(out), flush=True)


def make_ragged_workload(args, dev):
    """Sixteen scenes of log-uniform size on four atmospheres; the four
    smallest are 15 x 15 footprint averages of a finer truth.  Radiance by the
    library's FP32 forward model, noise sigma = L / SNR from a seeded device
    generator."""
    import torch
    import paper_2608_07580_amd as ff
    import scenegen
    t0 = time.time()
    layout = scenegen.config4_layout()
    atms = [scenegen.make_atmosphere(4, a) for a in range(scenegen.RAGGED_ATMOSPHERES)]
    scenes = [ff.Scene(a) for a in atms]
    gen = torch.Generator(device=dev)
    gen.manual_seed(4)
    rads, fires = [], []
    chunk = 1 << 18
    for spec in layout:
        sc = scenes[spec["atmosphere"]]
        B, P, b = sc.n_bands, spec["pixels"], spec["block"]
        states, mask = scenegen.config4_states(spec)
        rad = torch.empty((P, B), dtype=torch.float32, device=dev)
        if b == 1:
            for s0 in range(0, P, chunk):
                st = torch.tensor(states[s0:s0 + chunk], dtype=torch.float32, device=dev)
                rad[s0:s0 + chunk] = ff.forward(sc, st, 1)
            fire = mask
        else:
            rows, cols = spec["rows"], spec["cols"]
            fc = cols * b
            g = max(1, (1 << 20) // (b * fc))            # coarse rows per strip
            for r0 in range(0, rows, g):
                r1 = min(rows, r0 + g)
                st = torch.tensor(states[r0 * b * fc:r1 * b * fc], dtype=torch.float32, device=dev)
                L = ff.forward(sc, st, 1).view(r1 - r0, b, cols, b, B).mean(dim=(1, 3))
                rad[r0 * cols:r1 * cols] = L.reshape(-1, B)
            fire = mask.reshape(rows, b, cols, b).any(axis=(1, 3)).ravel()
        for s0 in range(0, P, chunk):
            n = torch.randn((min(chunk, P - s0), B), generator=gen, device=dev, dtype=torch.float32)
            rad[s0:s0 + chunk].mul_(1.0 + n / args.snr)
        rads.append(rad)
        fires.append(fire)
    torch.cuda.synchronize()
    log(f"ragged workload: {len(layout)} scenes, {sum(s['pixels'] for s in layout)} px, built in "
        f"{time.time() - t0:.1f}s")
    return layout, atms, scenes, rads, fires


def run_ragged(args):
    import torch
    import paper_2608_07580_amd as ff
    dev = torch.device("cuda:0")
    ff.lib()
    layout, atms, scenes, rads, fires = make_ragged_workload(args, dev)
    sc = [scenes[s["atmosphere"]] for s in layout]
    P_tot = sum(r.shape[0] for r in rads)
    B = rads[0].shape[1]
    prior = ff.default_prior(1)
    base = ff.default_options(n_quad=args.n_quad)
    nets, train_s = [], 0.0
    for atm in atms:
        net, info = train_network(args, atm, dev)
        nets.append(net)
        train_s += info["train_s"]
    net_of = [nets[s["atmosphere"]] for s in layout]
    stream = torch.cuda.Stream(device=dev)

    def tuned(scs, rs, ns):
        with torch.cuda.stream(stream):
            z0s = None if ns is None else [n.infer_routed(s_, r, stream=stream)[0] for n, s_, r in zip(ns, scs, rs)]
            opts, _ = ff.tune(scs, rs, prior, z0s=z0s, options=base,
                              cache_path=None if args.no_tune else args.tune_cache, retune=args.retune, stream=stream)
        torch.cuda.synchronize()
        return opts

    def time_graph(pipe, evals):
        for _ in range(args.warmup):
            pipe.launch()
        torch.cuda.synchronize()
        evals.zero_()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.steps):
            pipe.launch(stream)
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / args.steps, int(evals.item()) / args.steps

    legs = {}
    for name, ns in (("warm", net_of), ("plain", None)):
        opts = tuned(sc, rads, ns) if not args.no_tune else base
        evals = torch.zeros(1, dtype=torch.int64, device=dev)
        pipe = ff.Pipeline(sc, rads, prior, net=ns, options=opts, evals=evals, stream=stream,
                           route=None if ns is None else ff.HFDI_THRESHOLD)
        ms, ev = time_graph(pipe, evals)
        conv = [int(((o.status.cpu().numpy() & ff.ST_CONVERGED) != 0).sum()) for o in pipe.outputs]
        it = np.concatenate([o.iters.cpu().numpy() for o in pipe.outputs])
        st = np.concatenate([o.status.cpu().numpy() for o in pipe.outputs])
        legs[name] = {"graph_ms_per_step": ms, "converged": sum(conv), "converged_per_s": sum(conv) / (ms * 1e-3),
                      "evals_per_pixel": ev / P_tot, "mean_iters": float(it.mean()),
                      "p99_iters": float(np.percentile(it, 99)), "converged_by_scene": conv,
                      "fallback_rate": float(((st & ff.ST_USED_FALLBACK) != 0).mean()),
                      "launch": {"lanes_per_pixel": opts.lanes_per_pixel, "block_size": opts.block_size,
                                 "blocks_per_cu": opts.blocks_per_cu, "schedule": opts.schedule},
                      "evals": ev}
        pipe.close()
        log(f"{name}: {ms:.1f} ms per batch, {sum(conv) / (ms * 1e-3):.4g} converged/s")
    # the same warm batch launched eagerly (no graph)
    opts_w = tuned(sc, rads, net_of) if not args.no_tune else base
    outs = [ff.allocate_outputs(r.shape[0], 1, dev) for r in rads]
    with torch.cuda.stream(stream):
        for rep in range(args.warmup + args.steps):
            if rep == args.warmup:
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
            z0s = [n.infer_routed(s_, r, stream=stream)[0] for n, s_, r in zip(net_of, sc, rads)]
            ff.retrieve_batch(sc, rads, prior, z0s=z0s, options=opts_w, outputs=outs, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    eager_ms = a.elapsed_time(b) / args.steps
    # each scene alone (network + LM, tuned for its size): latency
    per_scene = []
    for spec, s1, r, n in zip(layout, sc, rads, net_of):
        o1 = tuned([s1], [r], [n])
        pipe = ff.Pipeline([s1], [r], prior, net=[n], options=o1, stream=stream, route=ff.HFDI_THRESHOLD)
        for _ in range(2):
            pipe.launch()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        pipe.launch(stream)
        b.record(stream)
        torch.cuda.synchronize()
        per_scene.append({"scene": spec["scene"], "pixels": spec["pixels"], "block": spec["block"],
                          "latency_ms": a.elapsed_time(b), "lanes_per_pixel": o1.lanes_per_pixel})
        pipe.close()
    seq_ms = sum(p["latency_ms"] for p in per_scene)
    w = legs["warm"]
    spe = slots_per_eval(B, args.n_quad, s_zero=all(not np.any(a.s_sph) for a in atms))
    achieved = w["evals"] * spe / (w["graph_ms_per_step"] * 1e-3)
    line = {
        "metric": "converged pixel retrievals/sec @284 bands, plain LM vs NN warm start, % roofline",
        "value": w["converged_per_s"], "unit": "converged retrievals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": w["graph_ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"ragged batch of {len(layout)} scenes ({P_tot} px x {B} bands, sizes "
                               f"log-uniform in [10k, 2.5M], 4 scenes 15x15 footprint averages of a finer "
                               f"truth), network warm start per atmosphere + LM, one graph launch per batch",
                   "pixels": P_tot, "scenes": len(layout), "bands": B, "n_quad": args.n_quad},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FMA32 / 1e12, "unit": UNIT_FMA,
                     "frac": achieved / PEAK_FMA32, "traffic": None,
                     "kernel": "whole graph (network + lm_kernel)", "kernel_ms": w["graph_ms_per_step"],
                     "op": OP_FMA, "ops_per_eval": spe,
                     "evals_per_launch": w["evals"]},
        "warm_start": w, "plain_lm": legs["plain"],
        "eager_batch_ms": eager_ms, "sequential_scene_sum_ms": seq_ms, "per_scene": per_scene,
        "train_s_total": train_s,
    }
    print(json.dumps(line), flush=True)


def run_precision(args):
    """Precision variants on the two-component stress set (8-parameter
    state, 1e-5 <= f <= 1e-3): FP32 bulk with FP32 or FP64 accumulation and
    the all-FP64 path, each timed on the GPU and compared output by output
    with the FP64 oracle on a seeded subsample."""
    import torch
    import oracle
    import paper_2608_07580_amd as ff
    import scenegen
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _helpers import parity_report
    dev = torch.device("cuda:0")
    ff.lib()
    P = args.precision_pixels
    X = scenegen.config2_states(P)
    atm = scenegen.make_atmosphere(2, 0)
    sc = ff.Scene(atm)
    B = sc.n_bands
    t0 = time.time()
    L = torch.empty((P, B), dtype=torch.float64, device=dev)
    chunk = 1 << 16
    for s0 in range(0, P, chunk):
        L[s0:s0 + chunk] = ff.forward(sc, torch.tensor(X[s0:s0 + chunk], dtype=torch.float64, device=dev), 2)
    noise = torch.from_numpy(scenegen.noise_normals(2, 0, P, B)).to(dev)
    rad = (L * (1.0 + noise.double() / args.snr)).float().contiguous()
    del L, noise
    torch.cuda.synchronize()
    log(f"precision workload: {P} px, built in {time.time() - t0:.1f}s")
    prior = ff.default_prior(2)
    variants = {"fp32": dict(precision=ff.PRECISION_FP32, accumulate=ff.ACCUMULATE_FP32),
                "fp32_fp64acc": dict(precision=ff.PRECISION_FP32, accumulate=ff.ACCUMULATE_FP64),
                "fp64": dict(precision=ff.PRECISION_FP64)}
    idx = scenegen.subsample(2, 0, P, args.cpu_sample)
    lobs = rad[idx].cpu().numpy()
    tab = oracle.band_tables(atm)
    lo, hi, x0 = scenegen.default_prior(2)
    t0 = time.time()
    ref = oracle.retrieve(tab, lobs, 2, lo, hi, x0, nthreads=len(os.sched_getaffinity(0)))
    t_oracle = time.time() - t0
    stream = torch.cuda.Stream(device=dev)
    names = ("f", "eta", "m_s", "s_s", "m_h", "s_h", "rho0", "rho1")
    report = {}
    for name, kw in variants.items():
        opts = ff.default_options(n_quad=args.n_quad, **kw)
        if not args.no_tune:
            with torch.cuda.stream(stream):
                opts, _ = ff.tune([sc], [rad], prior, options=opts, cache_path=args.tune_cache, retune=args.retune, stream=stream)
            torch.cuda.synchronize()
        outs = ff.allocate_outputs(P, 2, dev, state_f64=kw["precision"] == ff.PRECISION_FP64)
        evals = torch.zeros(1, dtype=torch.int64, device=dev)
        with torch.cuda.stream(stream):
            for rep in range(args.warmup + args.steps):
                if rep == args.warmup:
                    torch.cuda.synchronize()
                    evals.zero_()
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                ff.retrieve(sc, rad, prior, options=opts, outputs=outs, evals=evals, stream=stream)
            b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.steps
        res = outs.numpy()
        if res["state_f64"] is not None:
            res["state"] = res["state_f64"]
        conv = (res["status"] & ff.ST_CONVERGED) != 0
        sub = {k: v[idx] for k, v in res.items() if v is not None}
        rep = parity_report(sub, ref, model=2)
        both, same = rep["both_mask"], rep["same_mask"]
        errs = {}
        for j, nm in enumerate(names):
            d = np.abs(sub["state"][:, j] - ref.state[:, j])
            errs[nm] = {"same_min_max": float(d[same].max()) if same.any() else None,
                        "same_min_p99": float(np.percentile(d[same], 99)) if same.any() else None,
                        "both_conv_median": float(np.median(d[both])) if both.any() else None}
        for j, nm in enumerate(("E[T]", "sd[T]")):
            d = np.abs(sub["moments"][:, j] - ref.moments[:, j])
            errs[nm] = {"same_min_max": float(d[same].max()) if same.any() else None,
                        "same_min_p99": float(np.percentile(d[same], 99)) if same.any() else None,
                        "both_conv_median": float(np.median(d[both])) if both.any() else None}
        d = np.abs(sub["rrr"] - ref.rrr)
        errs["rrr"] = {"both_conv_max": float(d[both].max()), "same_min_max": float(d[same].max()) if same.any() else None}
        report[name] = {"ms_per_step": ms, "converged": int(conv.sum()), "converged_per_s": int(conv.sum()) / (ms * 1e-3),
                        "evals_per_pixel": int(evals.item()) / args.steps / P,
                        "launch": {"lanes_per_pixel": opts.lanes_per_pixel, "block_size": opts.block_size},
                        "vs_oracle": {k: v for k, v in rep.items() if not k.endswith("_mask")}, "errors": errs}
        log(f"{name}: {ms:.1f} ms, {int(conv.sum())} converged, same minimum {rep['same_frac']:.4f}")
    line = {"metric": "precision variants on the two-component stress set: time and error per output vs the FP64 oracle",
            "config": {"workload": f"two-component (smouldering + flaming lognormal) stress set, {P} px x {B} bands, "
                                   f"1e-5 <= f <= 1e-3, SNR {args.snr:g}", "pixels": P, "n_state": 8,
                       "oracle_sample": len(idx), "oracle_s": t_oracle,
                       "oracle_converged": int(ref.converged.sum())},
            "variants": report}
    print(json.dumps(line), flush=True)


def adam_slots_per_pixel(lam, stages, n_bands: int, n_quad: int) -> int:
    """Issue cost, in 32-bit FMA equivalents, of one pixel's staged-Adam solve
    (one component): per step and band inside the union of the free
    variables' windows, the thermal quadrature (NODE_W per node + 5), 19 for the solar term, basis and
    residual, and 12 for the windowed gradient sums (7 products into the
    per-variable sums, 5 window selects); then one full evaluation with the
    normal equations for the outputs (slots_per_eval)."""
    per_band = NODE_W * nodes_evaluated(n_quad) + 5 + 19 + 12
    total = 0
    for st in stages:
        lo = min(st["window"][j][0] for j in st["free"])
        hi = max(st["window"][j][1] for j in st["free"])
        nb = int(((lam >= lo) & (lam <= hi)).sum())
        total += st["steps"] * nb * per_band
    return total + slots_per_eval(n_bands, n_quad)


def run_solvers(args):
    """The paper's own solver against LM on the clustered-fire scene: the
    two-stage Adam schedule of Sec. 2.5 (130 fixed steps) and the plain LM
    from the same default start, each timed on the GPU, with accuracy against
    the true states and, on a seeded subsample, the FP64 oracle's staged Adam
    and LM for the same statistics."""
    import torch
    import oracle
    import paper_2608_07580_amd as ff
    import scenegen
    dev = torch.device("cuda:0")
    ff.lib()
    atm, scene, states, fire, noise, rad = make_workload(args, dev)
    P, B = rad.shape
    prior = ff.default_prior(1)
    stream = torch.cuda.Stream(device=dev)
    lam = scene.band_tables()[:, 0]

    def accuracy(state, moments, rrr, X):
        f = X[:, 0] > 1e-3
        eT = np.abs(moments[f, 0] - X[f, 1])
        ef = np.abs(state[:, 0] - X[:, 0])
        return {"fire_px": int(f.sum()), "dT_fire_median_K": float(np.median(eT)),
                "dT_fire_p90_K": float(np.percentile(eT, 90)), "df_median": float(np.median(ef)),
                "df_p90": float(np.percentile(ef, 90)), "rrr_median": float(np.median(rrr)),
                "rrr_p90": float(np.percentile(rrr, 90))}

    def timed(launch):
        with torch.cuda.stream(stream):
            for _ in range(args.warmup):
                launch()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(args.steps):
                launch()
            b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / args.steps

    # LM from the default start, tuned launch shape
    opts = ff.default_options(n_quad=args.n_quad)
    if not args.no_tune:
        with torch.cuda.stream(stream):
            opts, _ = ff.tune([scene], [rad], prior, options=opts, cache_path=args.tune_cache, retune=args.retune, stream=stream)
        torch.cuda.synchronize()
    out_lm = ff.allocate_outputs(P, 1, dev)
    ms_lm = timed(lambda: ff.retrieve(scene, rad, prior, options=opts, outputs=out_lm, stream=stream))
    r_lm = out_lm.numpy()
    conv = (r_lm["status"] & ff.ST_CONVERGED) != 0
    log(f"LM: {ms_lm:.1f} ms, {int(conv.sum())} converged")

    # LM stopped after a few iterations: the budget at which it matches the
    # accuracy of the paper's schedule
    lm_budget = []
    for mi in args.lm_budgets:
        o2 = ff.default_options(n_quad=args.n_quad, max_iter=mi, lanes_per_pixel=opts.lanes_per_pixel,
                                block_size=opts.block_size, blocks_per_cu=opts.blocks_per_cu,
                                schedule=opts.schedule)
        out2 = ff.allocate_outputs(P, 1, dev)
        ms2 = timed(lambda: ff.retrieve(scene, rad, prior, options=o2, outputs=out2, stream=stream))
        r2 = out2.numpy()
        lm_budget.append({"max_iter": mi, "ms_per_step": ms2,
                          "accuracy": accuracy(r2["state"], r2["moments"], r2["rrr"], states)})
        log(f"LM max_iter {mi}: {ms2:.1f} ms")
        del out2

    # the paper's staged Adam
    aopt = ff.adam_options(prior, n_quad=args.n_quad, lanes_per_pixel=args.adam_lpp)
    stages = [dict(steps=aopt.stage[k].steps, lr=aopt.stage[k].lr,
                   free=[j for j in range(5) if (aopt.stage[k].free_mask >> j) & 1],
                   window={j: (aopt.stage[k].window_lo_nm[j], aopt.stage[k].window_hi_nm[j]) for j in range(5)})
              for k in range(aopt.n_stages)]
    out_ad = ff.allocate_outputs(P, 1, dev)
    ms_ad = timed(lambda: ff.adam_retrieve(scene, rad, prior, options=aopt, outputs=out_ad, stream=stream))
    r_ad = out_ad.numpy()
    log(f"Adam: {ms_ad:.1f} ms")
    spp = adam_slots_per_pixel(lam, stages, B, args.n_quad)
    achieved = P * spp / (ms_ad * 1e-3)

    # oracle on a seeded subsample: both solvers, same statistics
    idx = scenegen.subsample(1, 0, P, args.solver_sample)
    tab = oracle.band_tables(atm)
    lobs = rad[torch.from_numpy(idx).to(dev)].cpu().numpy()
    lo, hi, x0 = scenegen.default_prior(1)
    cores = len(os.sched_getaffinity(0))
    t0 = time.time()
    o_lm = oracle.retrieve(tab, lobs, 1, lo, hi, x0, nthreads=cores)
    t_olm = time.time() - t0
    t0 = time.time()
    o_ad = oracle.adam_retrieve(tab, lobs, 1, lo, hi, x0, oracle.paper_stages(1, lo, hi, x0), nthreads=cores)
    t_oad = time.time() - t0
    X = states
    line = {
        "metric": "the paper's two-stage Adam vs LM on the clustered-fire scene: solved pixels/s and accuracy",
        "config": {"workload": f"clustered-fire scene {args.cross} x {args.lines} px x {B} bands, 3% fire, "
                               f"SNR {args.snr:g}; both solvers from the default start",
                   "pixels": P, "bands": B, "n_quad": args.n_quad},
        "lm": {"ms_per_step": ms_lm, "pixels_per_s": P / (ms_lm * 1e-3), "converged": int(conv.sum()),
               "launch": {"lanes_per_pixel": opts.lanes_per_pixel, "block_size": opts.block_size},
               "accuracy": accuracy(r_lm["state"], r_lm["moments"], r_lm["rrr"], X),
               "stopped_early": lm_budget},
        "adam": {"ms_per_step": ms_ad, "pixels_per_s": P / (ms_ad * 1e-3), "steps_per_pixel": 130,
                 "lanes_per_pixel": args.adam_lpp,
                 "accuracy": accuracy(r_ad["state"], r_ad["moments"], r_ad["rrr"], X),
                 "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FMA32 / 1e12,
                              "unit": UNIT_FMA, "frac": achieved / PEAK_FMA32, "kernel": "adam_kernel",
                              "ops_per_pixel": spp}},
        "oracle_sample": {"pixels": len(idx), "cores": cores, "lm_s": t_olm, "adam_s": t_oad,
                          "lm": accuracy(o_lm.state, o_lm.moments, o_lm.rrr, X[idx]),
                          "adam": accuracy(o_ad.state, o_ad.moments, o_ad.rrr, X[idx]),
                          "gpu_lm": accuracy(r_lm["state"][idx], r_lm["moments"][idx], r_lm["rrr"][idx], X[idx]),
                          "gpu_adam": accuracy(r_ad["state"][idx], r_ad["moments"][idx], r_ad["rrr"][idx], X[idx])},
    }
    print(json.dumps(line), flush=True)


# Grid nodes whose Planck ratios the scene tabulates (the FP32 32-node grid):
# the ratio is then read, not evaluated per pixel.
GRID_TABLE_NODES = 32


def grid_slots_per_eval(n_bands: int, n_nodes: int, model: int = 3) -> int:
    """Algorithmic VALU slots of one evaluation of the Gaussian-mixture model
    on the temperature grid, in 32-bit FMA equivalents: per (band, node) 7 per
    component for its weight product and the three centred sums, plus one
    Planck ratio shared by the two components (x = a2/T, exp2, minus 1, rcp)
    unless the scene tabulates the grid's ratios (n_nodes == GRID_TABLE_NODES:
    they do not depend on the pixel); per band 25 for the scaling, solar term,
    basis and residual and 45 for the J^T J, J^T r, r.r accumulations (n = 8),
    and the FP64 residual's RESIDUAL64_W.  The full model (endmember surface,
    n = 11) adds 6 for the five-term reflectance and basis, accumulates 78,
    and forms the FP64 reflectance with four more FP64 FMAs."""
    per_band = 25 + 45 if model == 3 else 25 + 6 + 78 + 4 * W_F64
    ratio = 0 if n_nodes == GRID_TABLE_NODES else 2 + W_EXP2 + W_RCP
    return n_bands * (n_nodes * (ratio + 2 * 7) + per_band + RESIDUAL64_W)


def run_paper_model(args, model: int = 3):
    """The paper's thermal form (two Gaussians on a [350, 2200] K grid, Sec.
    2.2) on a 262,144-pixel two-component set: LM (tuned launch) and the
    paper's staged Adam, timed, with E[T] accuracy against the truth and the
    FP64 oracle's LM on a seeded subsample.  model 5: the paper's full
    forward model, the same thermal term over the five-endmember simplex
    surface (Sec. 2.4), with path reflectance and spherical albedo."""
    import torch
    import oracle
    import paper_2608_07580_amd as ff
    import scenegen
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _helpers import parity_report
    dev = torch.device("cuda:0")
    ff.lib()
    P = args.precision_pixels
    lib = None
    if model == ff.MODEL_FULL:
        X = scenegen.draw_states_full(scenegen.rng_for(5, 0, scenegen.STREAM_PARAMS), P)
        atm = scenegen.make_atmosphere(5, 0, rho_atm=0.01, s_sph=0.1)
        lib = scenegen.endmember_library(atm.hr_lambda_nm)
        sc = ff.Scene(atm).set_endmembers(atm.hr_lambda_nm, lib)
    else:
        X = scenegen.config5_states(P)
        atm = scenegen.make_atmosphere(5, 0)
        sc = ff.Scene(atm)
    B = sc.n_bands
    L = torch.empty((P, B), dtype=torch.float64, device=dev)
    for s0 in range(0, P, 1 << 16):
        L[s0:s0 + (1 << 16)] = ff.forward(sc, torch.tensor(X[s0:s0 + (1 << 16)], dtype=torch.float64, device=dev),
                                          model)
    noise = torch.from_numpy(scenegen.noise_normals(5, 0, P, B)).to(dev)
    rad = (L * (1.0 + noise.double() / args.snr)).float().contiguous()
    del L, noise
    torch.cuda.synchronize()
    prior = ff.default_prior(model)
    stream = torch.cuda.Stream(device=dev)
    opts = ff.default_options(n_quad=args.n_quad, max_iter=args.grid_max_iter)
    if not args.no_tune:
        with torch.cuda.stream(stream):
            opts, _ = ff.tune([sc], [rad], prior, options=opts, cache_path=args.tune_cache, retune=args.retune, stream=stream)
        torch.cuda.synchronize()

    def timed(launch):
        with torch.cuda.stream(stream):
            for _ in range(args.warmup):
                launch()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(args.steps):
                launch()
            b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / args.steps

    et_true, _ = oracle.mixture_moments(X[:, 1], X[:, 4], X[:, 5], X[:, 2], X[:, 3])
    strong = X[:, 0] >= 1e-2

    def acc(r):
        d = np.abs(r["moments"][:, 0] - et_true)
        a = {"dT_median_K": float(np.median(d)), "dT_median_strong_K": float(np.median(d[strong])),
             "rrr_median": float(np.nanmedian(r["rrr"]))}
        if lib is not None:
            fr = r["state"][:, 6:]
            a.update({"fraction_mae": float(np.nanmean(np.abs(fr - X[:, 6:]))),
                      "max_simplex_sum_error": float(np.nanmax(np.abs(fr.sum(axis=1) - 1.0))),
                      "min_fraction": float(np.nanmin(fr))})
        return a

    out = ff.allocate_outputs(P, model, dev)
    evals = torch.zeros(1, dtype=torch.int64, device=dev)
    ms_lm = timed(lambda: ff.retrieve(sc, rad, prior, options=opts, outputs=out, evals=evals, stream=stream))
    r_lm = out.numpy()
    ev = int(evals.item()) / (args.steps + args.warmup)
    conv = int(((r_lm["status"].astype(np.int64) & ff.ST_CONVERGED) != 0).sum())
    spe = grid_slots_per_eval(B, args.n_quad, model)
    achieved = ev * spe / (ms_lm * 1e-3)
    aopt = ff.adam_options(prior, n_quad=args.n_quad)
    out_a = ff.allocate_outputs(P, model, dev)
    ms_ad = timed(lambda: ff.adam_retrieve(sc, rad, prior, options=aopt, outputs=out_a, stream=stream))
    r_ad = out_a.numpy()
    idx = scenegen.subsample(5, 0, P, args.solver_sample)
    tab = oracle.band_tables(atm, lib)
    lo, hi, x0 = scenegen.default_prior(model)
    t0 = time.time()
    ref = oracle.retrieve(tab, rad[torch.from_numpy(idx).to(dev)].cpu().numpy(), model, lo, hi, x0,
                          opts=oracle.LMOptions(max_iter=args.grid_max_iter), nthreads=len(os.sched_getaffinity(0)))
    t_or = time.time() - t0
    rep = parity_report({k: v[idx] for k, v in r_lm.items() if v is not None}, ref, model=model)
    what = ("the paper's full forward model (Gaussian mixture on the grid over the 5-endmember simplex surface)"
            if lib is not None else "the paper's Gaussian-mixture thermal model")
    surface = ", 5-endmember simplex surface, rho_atm 0.01, S 0.1" if lib is not None else ""
    line = {
        "metric": f"{what}: LM and staged Adam retrievals per second",
        "config": {"workload": f"two-Gaussian mixture on a {args.n_quad}-node [350, 2200] K grid{surface}, "
                               f"{P} px x {B} bands, 1e-4 <= f <= 0.1, SNR {args.snr:g}", "pixels": P,
                   "nodes": args.n_quad, "max_iter": args.grid_max_iter},
        "lm": {"ms_per_step": ms_lm, "converged": conv, "converged_per_s": conv / (ms_lm * 1e-3),
               "evals_per_pixel": ev / P, "accuracy": acc(r_lm),
               "launch": {"lanes_per_pixel": opts.lanes_per_pixel, "block_size": opts.block_size},
               "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FMA32 / 1e12, "unit": UNIT_FMA,
                            "frac": achieved / PEAK_FMA32, "kernel": "lm_kernel", "ops_per_eval": spe}},
        "adam": {"ms_per_step": ms_ad, "pixels_per_s": P / (ms_ad * 1e-3), "accuracy": acc(r_ad)},
        "oracle_sample": {"pixels": len(idx), "s": t_or, "converged": int(ref.converged.sum()),
                          "gpu_lm_vs_oracle": {k: v for k, v in rep.items() if not k.endswith("_mask")}},
    }
    print(json.dumps(line), flush=True)


def run_endmember(args):
    """The endmember surface (Sec. 2.2 with the library of Sec. 2.4: five
    spectra, fractions on the unit simplex) under one lognormal fire
    component, on a 262,144-pixel set with path reflectance and spherical
    albedo: the simplex-constrained LM (tuned launch) and the paper's
    staged Adam with its projection, timed, with E[T] and fraction accuracy
    against the truth and the FP64 oracle's LM on a seeded subsample."""
    import torch
    import oracle
    import paper_2608_07580_amd as ff
    import scenegen
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _helpers import parity_report
    dev = torch.device("cuda:0")
    ff.lib()
    P = args.precision_pixels
    model = ff.MODEL_ENDMEMBER_1
    X = scenegen.draw_states_endmember1(scenegen.rng_for(6, 0, scenegen.STREAM_PARAMS), P)
    atm = scenegen.make_atmosphere(6, 0, rho_atm=0.02, s_sph=0.1)
    lib = scenegen.endmember_library(atm.hr_lambda_nm)
    sc = ff.Scene(atm).set_endmembers(atm.hr_lambda_nm, lib)
    B = sc.n_bands
    L = torch.empty((P, B), dtype=torch.float64, device=dev)
    for s0 in range(0, P, 1 << 16):
        L[s0:s0 + (1 << 16)] = ff.forward(sc, torch.tensor(X[s0:s0 + (1 << 16)], dtype=torch.float64, device=dev),
                                          model)
    noise = torch.from_numpy(scenegen.noise_normals(6, 0, P, B)).to(dev)
    rad = (L * (1.0 + noise.double() / args.snr)).float().contiguous()
    del L, noise
    torch.cuda.synchronize()
    prior = ff.default_prior(model)
    stream = torch.cuda.Stream(device=dev)
    opts = ff.default_options(n_quad=args.n_quad, max_iter=args.grid_max_iter)
    if not args.no_tune:
        with torch.cuda.stream(stream):
            opts, _ = ff.tune([sc], [rad], prior, options=opts, cache_path=args.tune_cache, retune=args.retune, stream=stream)
        torch.cuda.synchronize()

    def timed(launch):
        with torch.cuda.stream(stream):
            for _ in range(args.warmup):
                launch()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(args.steps):
                launch()
            b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / args.steps

    strong = X[:, 0] >= 1e-2

    def acc(r):
        d = np.abs(r["moments"][:, 0] - X[:, 1])
        fr = r["state"][:, 3:]
        return {"dT_median_K": float(np.nanmedian(d)), "dT_median_strong_K": float(np.nanmedian(d[strong])),
                "fraction_mae": float(np.nanmean(np.abs(fr - X[:, 3:]))),
                "max_simplex_sum_error": float(np.nanmax(np.abs(fr.sum(axis=1) - 1.0))),
                "min_fraction": float(np.nanmin(fr)), "rrr_median": float(np.nanmedian(r["rrr"]))}

    out = ff.allocate_outputs(P, model, dev)
    evals = torch.zeros(1, dtype=torch.int64, device=dev)
    ms_lm = timed(lambda: ff.retrieve(sc, rad, prior, options=opts, outputs=out, evals=evals, stream=stream))
    r_lm = out.numpy()
    ev = int(evals.item()) / (args.steps + args.warmup)
    conv = int(((r_lm["status"].astype(np.int64) & ff.ST_CONVERGED) != 0).sum())
    spe = slots_per_eval(B, args.n_quad, model)
    achieved = ev * spe / (ms_lm * 1e-3)
    aopt = ff.adam_options(prior, n_quad=args.n_quad)
    out_a = ff.allocate_outputs(P, model, dev)
    ms_ad = timed(lambda: ff.adam_retrieve(sc, rad, prior, options=aopt, outputs=out_a, stream=stream))
    r_ad = out_a.numpy()
    idx = scenegen.subsample(6, 0, P, args.solver_sample)
    tab = oracle.band_tables(atm, lib)
    lo, hi, x0 = scenegen.default_prior(model)
    t0 = time.time()
    ref = oracle.retrieve(tab, rad[torch.from_numpy(idx).to(dev)].cpu().numpy(), model, lo, hi, x0,
                          opts=oracle.LMOptions(max_iter=args.grid_max_iter), nthreads=len(os.sched_getaffinity(0)))
    t_or = time.time() - t0
    rep = parity_report({k: v[idx] for k, v in r_lm.items() if v is not None}, ref, model=model)
    line = {
        "metric": "endmember surface on the unit simplex: LM and staged Adam retrievals per second",
        "config": {"workload": f"one lognormal fire component over a 5-endmember simplex surface, {P} px x {B} "
                               f"bands, rho_atm 0.02, S 0.1, 1e-4 <= f <= 0.3, Dirichlet(0.7) fractions, "
                               f"SNR {args.snr:g}", "pixels": P, "max_iter": args.grid_max_iter},
        "lm": {"ms_per_step": ms_lm, "converged": conv, "converged_per_s": conv / (ms_lm * 1e-3),
               "evals_per_pixel": ev / P, "accuracy": acc(r_lm),
               "launch": {"lanes_per_pixel": opts.lanes_per_pixel, "block_size": opts.block_size},
               "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FMA32 / 1e12, "unit": UNIT_FMA,
                            "frac": achieved / PEAK_FMA32, "kernel": "lm_kernel", "ops_per_eval": spe}},
        "adam": {"ms_per_step": ms_ad, "pixels_per_s": P / (ms_ad * 1e-3), "accuracy": acc(r_ad)},
        "oracle_sample": {"pixels": len(idx), "s": t_or, "converged": int(ref.converged.sum()),
                          "gpu_lm_vs_oracle": {k: v for k, v in rep.items() if not k.endswith("_mask")}},
    }
    print(json.dumps(line), flush=True)


def run_coarsening(args):
    """The paper's resolution-rescaling analysis on the clustered-fire scene:
    12 x 12 block means of the fine radiance, LM at both resolutions, and the
    Quantile Error Curve of every coarse fire pixel against the fine
    retrievals in its footprint (empirical and Gaussian-mixture).  Times each
    stage; reports the mean curves."""
    import torch
    import paper_2608_07580_amd as ff
    dev = torch.device("cuda:0")
    ff.lib()
    atm, scene, states, fire, noise, rad = make_workload(args, dev)
    P, B = rad.shape
    rows, cols, b = args.lines, args.cross, args.block
    prior = ff.default_prior(1)
    stream = torch.cuda.Stream(device=dev)
    opts = ff.default_options(n_quad=args.n_quad)
    if not args.no_tune:
        with torch.cuda.stream(stream):
            opts, _ = ff.tune([scene], [rad], prior, options=opts, cache_path=args.tune_cache, retune=args.retune, stream=stream)
        torch.cuda.synchronize()
    K = (rows // b) * (cols // b)
    fine = ff.allocate_outputs(P, 1, dev)
    coarse = ff.allocate_outputs(K, 1, dev)
    ev = []

    def step():
        e = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        e[0].record(stream)
        crad = ff.block_mean(rad, rows, cols, b, stream=stream)
        e[1].record(stream)
        ff.retrieve(scene, rad, prior, options=opts, outputs=fine, stream=stream)
        e[2].record(stream)
        ff.retrieve(scene, crad, prior, options=opts, outputs=coarse, stream=stream)
        e[3].record(stream)
        out = ff.qec(fine, coarse, rows, cols, b, stream=stream)
        e[4].record(stream)
        ev.append(e)
        return out

    with torch.cuda.stream(stream):
        for _ in range(args.warmup + args.steps):
            emp, mix, n_used = step()
    torch.cuda.synchronize()
    ev = ev[args.warmup:]
    stage = [sum(e[i].elapsed_time(e[i + 1]) for e in ev) / len(ev) for i in range(4)]
    emp, mix, n_used = emp.cpu().numpy(), mix.cpu().numpy(), n_used.cpu().numpy()
    ok = np.isfinite(emp[:, 0])
    f, c = fine.numpy(), coarse.numpy()
    # mean fine E[T] of the footprint against the coarse E[T]
    R, C = rows // b, cols // b
    d = []
    for k in np.nonzero(ok)[0]:
        r0, c0 = divmod(int(k), C)
        idx = ((r0 * b + np.arange(b))[:, None] * cols + (c0 * b + np.arange(b))[None, :]).ravel()
        sel = idx[((f["status"][idx].astype(np.int64) & ff.ST_CONVERGED) != 0) & (f["state"][idx, 0] >= 1e-4)
                  & np.isfinite(f["moments"][idx, 1]) & (f["moments"][idx, 1] > 0)]
        d.append(c["moments"][k, 0] - f["moments"][sel, 0].mean())
    d = np.array(d)
    line = {
        "metric": "resolution rescaling: QEC of coarse (12 x 12 block-mean) posteriors against fine retrievals",
        "config": {"workload": f"clustered-fire scene {cols} x {rows} px x {B} bands, 3% fire, SNR {args.snr:g}; "
                               f"{b} x {b} block means -> {C} x {R} coarse px", "fine_pixels": P,
                   "coarse_pixels": K, "block": b, "levels": list(ff.QEC_LEVELS), "f_min": 1e-4, "min_fine": 5},
        "ms": {"block_mean": stage[0], "fine_lm": stage[1], "coarse_lm": stage[2], "qec": stage[3],
               "total": sum(stage)},
        "coarse_evaluated": int(ok.sum()),
        "fine_used_mean": float(n_used[ok].mean()) if ok.any() else None,
        "qec_empirical_mean_K": [float(v) for v in emp[ok].mean(0)],
        "qec_mixture_mean_K": [float(v) for v in mix[ok].mean(0)],
        "qec_empirical_mean_abs_K": float(np.abs(emp[ok].mean(0)).mean()),
        "qec_mixture_mean_abs_K": float(np.abs(mix[ok].mean(0)).mean()),
        "coarse_minus_fine_mean_ET": {"mae_K": float(np.abs(d).mean()), "bias_K": float(d.mean())},
        "block_mean_hbm": {"bytes": P * B * 4 + K * B * 4, "GB_per_s": (P * B * 4 + K * B * 4) / (stage[0] * 1e-3) / 1e9,
                           "frac_of_8TBs": (P * B * 4 + K * B * 4) / (stage[0] * 1e-3) / HBM_PEAK},
    }
    print(json.dumps(line), flush=True)


def run_front_end(args):
    """The paper's candidate selection in front of the retrieval: the HFDI
    pre-filter (Sec. 2.1, threshold -0.1) builds the candidate list on the
    device and LM solves only the listed pixels (the count never leaves the
    device).  Timed per step: HFDI + listed LM.  The warm leg adds the
    learned start on the candidates only: HFDI, the count read back, the
    network on the listed rows (ff_mlp_infer_listed), LM on the listed rows
    from those starts with fallback."""
    import torch
    import paper_2608_07580_amd as ff
    dev = torch.device("cuda:0")
    ff.lib()
    atm, scene, states, fire, noise, rad = make_workload(args, dev)
    P, B = rad.shape
    prior = ff.default_prior(1)
    stream = torch.cuda.Stream(device=dev)
    # launch shape for the candidate set: tuned on the gathered candidate rows
    with torch.cuda.stream(stream):
        idx, cnt, _ = ff.hfdi_candidates(scene, rad, args.hfdi_threshold, with_index_values=False, stream=stream)
    torch.cuda.synchronize()
    n = int(cnt.item())
    opts = ff.default_options(n_quad=args.n_quad)
    if not args.no_tune and n > 0:
        sub = rad[idx[:n]].contiguous()
        with torch.cuda.stream(stream):
            opts, _ = ff.tune([scene], [sub], prior, options=opts, cache_path=args.tune_cache, retune=args.retune, stream=stream)
        torch.cuda.synchronize()
        del sub
    out = ff.allocate_outputs(P, 1, dev)
    evals = torch.zeros(1, dtype=torch.int64, device=dev)
    ev = []

    def step(timed):
        a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        a.record(stream)
        ix, ct, _ = ff.hfdi_candidates(scene, rad, args.hfdi_threshold, with_index_values=False, stream=stream)
        b.record(stream)
        ff.retrieve_listed(scene, rad, ix, ct, prior, options=opts, outputs=out, evals=evals, stream=stream)
        c.record(stream)
        if timed:
            ev.append((a, b, c))
        return ix, ct

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step(False)
        torch.cuda.synchronize()
        evals.zero_()
        for _ in range(args.steps):
            ix, ct = step(True)
    torch.cuda.synchronize()
    hfdi_ms = sum(a.elapsed_time(b) for a, b, c in ev) / len(ev)
    lm_ms = sum(b.elapsed_time(c) for a, b, c in ev) / len(ev)
    ms = hfdi_ms + lm_ms
    n = int(ct.item())
    cands = ix[:n].cpu().numpy()
    r = out.numpy()
    conv = int(((r["status"][cands].astype(np.int64) & ff.ST_CONVERGED) != 0).sum())
    plain_evals = int(evals.item()) / args.steps / max(n, 1)
    fire_idx = np.nonzero(fire)[0]

    # warm leg: the network on the candidates only, LM from its starts
    net, info = train_network(args, atm, dev)
    z0 = torch.empty((P, ff.N_STATE[1]), dtype=torch.float32, device=dev)
    wout = ff.allocate_outputs(P, 1, dev)
    wopts = ff.default_options(n_quad=args.n_quad)
    if not args.no_tune and n > 0:
        sub = rad[idx[:n]].contiguous()
        with torch.cuda.stream(stream):
            zs = net.infer(sub, stream=stream)
            wopts, _ = ff.tune([scene], [sub], prior, z0s=[zs], options=wopts, cache_path=args.tune_cache,
                               retune=args.retune, stream=stream)
        torch.cuda.synchronize()
        del sub, zs
    wev = []

    def warm_step(timed):
        t0 = time.perf_counter()
        a, b, c, d = (torch.cuda.Event(enable_timing=True) for _ in range(4))
        a.record(stream)
        ix, ct, _ = ff.hfdi_candidates(scene, rad, args.hfdi_threshold, with_index_values=False, stream=stream)
        b.record(stream)
        m = int(ct.item())                      # the one host round trip: the inference grid needs the count
        net.infer_listed(rad, ix, m, z0=z0, stream=stream)
        c.record(stream)
        ff.retrieve_listed(scene, rad, ix, ct, prior, z0=z0, options=wopts, outputs=wout, evals=evals,
                           stream=stream)
        d.record(stream)
        stream.synchronize()
        if timed:
            wev.append((a, b, c, d, time.perf_counter() - t0))

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            warm_step(False)
        torch.cuda.synchronize()
        evals.zero_()
        for _ in range(args.steps):
            warm_step(True)
    torch.cuda.synchronize()
    w_hfdi = sum(a.elapsed_time(b) for a, b, c, d, t in wev) / len(wev)
    w_net = sum(b.elapsed_time(c) for a, b, c, d, t in wev) / len(wev)
    w_lm = sum(c.elapsed_time(d) for a, b, c, d, t in wev) / len(wev)
    w_wall = sum(t for a, b, c, d, t in wev) / len(wev) * 1e3
    wr = wout.numpy()
    wst = wr["status"][cands].astype(np.int64)
    wconv = int(((wst & ff.ST_CONVERGED) != 0).sum())
    isf = fire[cands]
    warm = {"ms_per_step": w_hfdi + w_net + w_lm, "wall_ms_per_step": w_wall, "hfdi_ms": w_hfdi,
            "network_ms": w_net, "lm_ms": w_lm, "converged_candidates": wconv,
            "converged_per_s": wconv / ((w_hfdi + w_net + w_lm) * 1e-3),
            "mean_iters": float(wr["iters"][cands].mean()), "mean_iters_fire": float(wr["iters"][cands][isf].mean()),
            "evals_per_candidate": int(evals.item()) / args.steps / max(n, 1),
            "fallback_rate": float(((wst & ff.ST_USED_FALLBACK) != 0).mean()),
            "launch": {"lanes_per_pixel": wopts.lanes_per_pixel, "block_size": wopts.block_size,
                       "blocks_per_cu": wopts.blocks_per_cu, "schedule": wopts.schedule},
            "train_s": info["train_s"]}
    log(f"front end, warm: HFDI {w_hfdi:.3f} + network {w_net:.3f} + LM {w_lm:.3f} ms "
        f"(wall {w_wall:.3f} ms), {wconv} of {n} converge, iterations {warm['mean_iters']:.2f} "
        f"against {float(r['iters'][cands].mean()):.2f}")
    line = {
        "metric": "HFDI front end + LM on the candidates: scene pixels/s and converged candidates/s",
        "config": {"workload": f"clustered-fire scene {args.cross} x {args.lines} px x {B} bands, 3% fire, "
                               f"SNR {args.snr:g}; HFDI >= {args.hfdi_threshold:g} (Sec. 2.1), plain LM on the "
                               f"candidates", "pixels": P, "bands": B},
        "candidates": n, "fire_pixels": int(fire.sum()),
        "fire_recall": float(np.isin(fire_idx, cands).mean()),
        "background_candidates": int((~fire[cands]).sum()),
        "ms_per_step": ms, "hfdi_ms": hfdi_ms, "lm_ms": lm_ms,
        "scene_pixels_per_s": P / (ms * 1e-3), "converged_candidates": conv,
        "converged_per_s": conv / (ms * 1e-3), "evals_per_candidate": plain_evals,
        "mean_iters": float(r["iters"][cands].mean()), "mean_iters_fire": float(r["iters"][cands][isf].mean()),
        "launch": {"lanes_per_pixel": opts.lanes_per_pixel, "block_size": opts.block_size,
                   "blocks_per_cu": opts.blocks_per_cu, "schedule": opts.schedule},
        "warm_start": warm,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lines", type=int, default=2048)
    ap.add_argument("--cross", type=int, default=1234)
    ap.add_argument("--snr", type=float, default=300.0)
    ap.add_argument("--n-quad", type=int, default=32)
    ap.add_argument("--start", choices=("warm", "plain"), default="plain",
                    help="path whose throughput is the headline value (both are run): plain = the "
                         "configuration's plain LM from the default start; warm = network + LM with fallback")
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--train-batch", type=int, default=2048)
    ap.add_argument("--bg-fraction", type=float, default=0.3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=65536)
    ap.add_argument("--no-tune", action="store_true", help="default launch shape instead of the tuner's")
    ap.add_argument("--grid-max-iter", type=int, default=200, help="paper-model workload: LM iteration cap")
    ap.add_argument("--block", type=int, default=12, help="coarsening workload: block side")
    ap.add_argument("--workload", choices=("clustered-fire", "ragged", "precision", "solvers", "front-end",
                                           "paper-model", "full-model", "endmember-surface", "coarsening",
                                           "valu-rates"),
                    default="clustered-fire",
                    help="clustered-fire: the 2.53M-pixel scene (headline); ragged: 16-scene batch; "
                         "precision: FP32/FP64 variants on the two-component stress set; "
                         "solvers: the paper's two-stage Adam vs LM on the clustered-fire scene; "
                         "front-end: HFDI candidate selection + LM on the candidates; "
                         "paper-model: the paper's two-Gaussian grid thermal model, LM and staged Adam; "
                         "endmember-surface: the 5-endmember simplex surface, LM and staged Adam; "
                         "full-model: the paper's full forward model (grid mixture over the endmember surface); "
                         "coarsening: 12 x 12 block means, LM at both resolutions, Quantile Error Curves")
    ap.add_argument("--adam-lpp", type=int, default=1, help="lanes per pixel of the Adam kernel")
    ap.add_argument("--hfdi-threshold", type=float, default=-0.1, help="front-end workload: HFDI threshold")
    ap.add_argument("--solver-sample", type=int, default=4096, help="oracle subsample of the solvers workload")
    ap.add_argument("--lm-budgets", type=int, nargs="*", default=[1, 2, 3, 5],
                    help="solvers workload: LM iteration caps timed beside the full LM")
    ap.add_argument("--precision-pixels", type=int, default=262144)
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2608_07580_amd", "tuning.json"),
                    help="autotuner table (read, and written on a miss)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--retune", action="store_true",
                    help="time the launch-shape candidates again and overwrite the tuner table's entries")
    ap.add_argument("--tune-quadrature", action="store_true",
                    help="also run the tuner's quadrature-order choice on the scene and report it "
                         "(the headline keeps --n-quad)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the library runs on one GPU per process and this benchmark on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "valu-rates":
        run_valu_rates(args)
        return
    if args.workload == "ragged":
        run_ragged(args)
        return
    if args.workload == "solvers":
        run_solvers(args)
        return
    if args.workload == "front-end":
        run_front_end(args)
        return
    if args.workload == "paper-model":
        run_paper_model(args)
        return
    if args.workload == "coarsening":
        run_coarsening(args)
        return
    if args.workload == "endmember-surface":
        run_endmember(args)
        return
    if args.workload == "full-model":
        run_paper_model(args, model=5)
        return
    if args.workload == "precision":
        if args.cpu_sample == 65536:
            args.cpu_sample = 8192
        run_precision(args)
        return

    import torch
    import paper_2608_07580_amd as ff
    dev = torch.device("cuda:0")
    ff.lib()
    atm, scene, states, fire, noise, rad = make_workload(args, dev)
    P, B = rad.shape
    stream = torch.cuda.Stream(device=dev)

    plain, res_plain, ev_plain = run_leg(args, atm, rad, stream, None)
    log(f"plain LM: {plain['converged_per_s']:.4g} converged/s, {plain['ms_per_step']:.1f} ms/step, "
        f"{plain['mean_iters']:.2f} iters")
    net, train_info = train_network(args, atm, dev)
    warm, res_warm, ev_warm = run_leg(args, atm, rad, stream, net)
    log(f"warm LM: {warm['converged_per_s']:.4g} converged/s, {warm['ms_per_step']:.1f} ms/step, "
        f"{warm['mean_iters']:.2f} iters, fallback {warm['fallback_rate']:.4f}")
    warm.update(train_info)
    # temperature of the warm-started fits against the plain fits: fire pixels
    # both converge on with f >= 1e-4 in both
    both = ((res_plain["status"] & ff.ST_CONVERGED) != 0) & ((res_warm["status"] & ff.ST_CONVERGED) != 0)
    fok = both & fire & (res_plain["state"][:, 0] >= 1e-4) & (res_warm["state"][:, 0] >= 1e-4)
    dT = np.abs(res_warm["moments"][:, 0] - res_plain["moments"][:, 0])[fok]
    warm["dT_vs_plain_K"] = {"pixels": int(fok.sum()), "median": float(np.median(dT)),
                             "p99": float(np.percentile(dT, 99)), "max": float(dT.max())}
    # the radiance hand-over from host memory, timed apart from the step (the
    # boundary takes device buffers): pinned host copy of the scene -> device
    head_ms = (warm if args.start == "warm" else plain)["ms_per_step"]
    # (skipped in counter runs, whose calibration copy must be the only copy)
    h2d_info = None
    if not args.copy_calibration:
        host = torch.empty(rad.shape, dtype=rad.dtype, pin_memory=True)
        host.copy_(rad)
        torch.cuda.synchronize()
        h2d = []
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(stream):
                e0.record(stream)
                rad.copy_(host, non_blocking=True)
                e1.record(stream)
            torch.cuda.synchronize()
            h2d.append(e0.elapsed_time(e1))
        del host
        h2d_ms = min(h2d)
        h2d_info = {"ms": h2d_ms, "GB_per_s": rad.numel() * 4 / (h2d_ms * 1e-3) / 1e9, "host_memory": "pinned",
                    "step_ms_with_h2d": head_ms + h2d_ms}
        log(f"radiance host -> device: {h2d_ms:.1f} ms ({h2d_info['GB_per_s']:.1f} GB/s, pinned)")
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    head, ev_head = (warm, ev_warm) if args.start == "warm" else (plain, ev_plain)
    s_zero = not np.any(atm.s_sph)
    spe = slots_per_eval(B, args.n_quad, s_zero=s_zero)
    achieved = ev_head * spe / (head["lm_kernel_ms"] * 1e-3)
    fpe = flops_per_eval(B, args.n_quad, s_zero=s_zero)
    flops = ev_head * fpe / (head["lm_kernel_ms"] * 1e-3)
    start_desc = ("network warm start (trained per atmosphere, not timed) + LM with fallback"
                  if args.start == "warm" else "default start (plain LM)")
    line = {
        "metric": "converged pixel retrievals/sec @284 bands, plain LM vs NN warm start, % roofline",
        "value": head["converged_per_s"], "unit": "converged retrievals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"clustered-fire scene {args.cross} x {args.lines} px x {B} bands, "
                               f"3% fire, SNR {args.snr:g}; {start_desc}",
                   "pixels": P, "bands": B, "n_quad": args.n_quad, "precision": "fp32-bulk/fp64-solve",
                   "start": args.start},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FMA32 / 1e12,
                     "unit": UNIT_FMA, "frac": achieved / PEAK_FMA32,
                     "traffic": measured_traffic(args.start),
                     "traffic_unit": "HBM bytes per launch (calibrated TCC FETCH_SIZE + WRITE_SIZE)",
                     "kernel": "lm_kernel", "kernel_ms": head["lm_kernel_ms"],
                     "op": OP_FMA,
                     "ops_per_eval": spe, "evals_per_launch": ev_head,
                     "frac_of_measured_fma_rate": achieved / MEASURED_FMA32,
                     "flops_per_eval": fpe, "achieved_TFLOPs": flops / 1e12,
                     "frac_published": flops / PEAK_FP32_PUBLISHED,
                     "peak_published_TFLOPs": PEAK_FP32_PUBLISHED / 1e12},
        "plain_lm": plain,
        "warm_start": warm,
        "h2d": h2d_info,
    }
    if args.tune_quadrature:
        # the tuner's quadrature dimension on this scene (plain start), reported
        # beside the headline, which keeps the configuration's 32 nodes
        with torch.cuda.stream(stream):
            _, rep = ff.tune_quadrature([scene], [rad], ff.default_prior(1),
                                        options=ff.default_options(n_quad=args.n_quad),
                                        cache_path=args.tune_cache, stream=stream)
        torch.cuda.synchronize()
        line["quadrature_choice"] = rep
        log(f"quadrature choice: {rep}")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args, atm, rad, states, {"plain": res_plain, "warm": res_warm})
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
