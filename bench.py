#!/usr/bin/env python3
"""Benchmark of the LM/PCG hot path on one MI355X.

One step = one Levenberg-Marquardt iteration on one image subset: build the
gradient cache (projection, binning, depth sort, forward render, cache fill,
b = -J^T F), the Jacobi diagonal, Algorithm 1 with n_iters PCG iterations
(n_iters + 1 applications of J^T J), the subset combination, one J
product for ||J delta||^2, the line search on 30% of the views, the
trust-region ratio and the update (paper section 3.2).  Inputs (scene,
cameras, targets) are resident in HBM before the timed region.  `value`
counts the n_iters + 1 J^T J applications per iteration over the whole
iteration's time.

Default workload: 1,000,000 Gaussians, SH degree 3 (59 parameters each), 32
views at 1024x640 in one subset, float32 cache, 8 Jacobi-PCG iterations per
LM step, lambda = 1e-2.  Targets are renders of the perturbed scene plus
pixel noise (synthetic stand-ins for the paper's captured images).

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "J^TJ·p applies/s + HBM GB/s; LM-iter ms, bf16/batched/learned vs plain"
# The paper's own timings of this path, quoted with the hardware it names
# (context only: other hardware, other scenes, precision not stated)
PAPER_CONTEXT = {
    "per_kernel_profile": {
        "hardware": "NVIDIA RTX 3090", "workload": "MipNeRF360 garden, one image, one PCG iteration",
        "source": "supplement, detailed runtime analysis (kernel profile table)",
        "ms": {"buildCache": 35.97, "sortCacheByGaussians": 5.04, "diagJTJ": 41.60, "sortX": 4.45, "applyJ": 10.98,
               "applyJT": 7.50},
        "JtJp_ms": 22.93},
    "end_to_end_s": {
        "hardware": "NVIDIA A100", "source": "results, quantitative comparison table (3DGS and 3DGS + LM)",
        "MipNeRF360": {"3DGS": 1271, "3DGS+LM": 972}, "Tanks&Temples": {"3DGS": 736, "3DGS+LM": 663},
        "Deep Blending": {"3DGS": 1222, "3DGS+LM": 951}},
}
HBM_PEAK_GBPS = 8000.0


def traffic_file(dtype: str) -> str:
    """Committed rocprofv3 counter summary of the fused pass for one cache type."""
    return os.path.join(ROOT, "profiles", f"apply_tile_JtJ_paper_{dtype}_traffic.txt")

# the tile pass and the wave sums it uses
APPLY_SRC = [os.path.join(ROOT, "paper_2409_12892_amd", "csrc", f) for f in ("products.h", "wave.h")]


def apply_src_sha() -> str:
    h = hashlib.sha256()
    for f in APPLY_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


class OneCam:
    """Cameras-like wrapper of a single camera dict (for the oracle)."""

    def __init__(self, cam):
        self.cam = cam
        self.V = 1

    def view(self, v):
        return self.cam


def apply_tile_alg_bytes(info: dict, weighted: bool = False) -> int:
    """Algorithmic HBM bytes of one fused J^T J tile-pass launch: every cached
    pair once (T, dC/dalpha x3 in the cache dtype + the pixel byte), per
    segment its staged splat (6 floats), pair offset and gv index (2 x 4 B),
    its tangent coefficients (9 floats, read) and moments (9 floats,
    written), per tile its offsets, view and ||Jp||^2 partial; with residual
    weights, 3 floats per pixel."""
    wb = 4 if info["cache_dtype"] == 0 else 2
    return int(info["n_pairs"] * (4 * wb + 1) + info["n_segments"] * (24 + 8 + 36 + 36) + info["n_tiles"] * 28
               + (12 * info["n_pixels"] if weighted else 0))


def read_traffic(alg_bytes: int, tile: str, dtype: str):
    """HBM traffic per launch from the committed rocprofv3 counter summary of
    this cache type, or None when it is absent or was taken on a different
    kernel source or tile shape."""
    path = traffic_file(dtype)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    src = apply_src_sha()
    if kv.get("apply_src_sha256") != src or kv.get("tile") != tile or kv.get("cache_dtype") != dtype:
        return None
    try:
        return int(float(kv["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


COPY_BYTES = 4 * 1024 * 1024 * 1024   # well beyond the 256 MB Infinity Cache


def summarize_pmc(fetch_dir: str, write_dir: str, command: str, tile: str, dtype: str, last: int = 9) -> dict:
    """HBM traffic of the fused J^T J tile pass from two rocprofv3 --pmc runs
    of `bench.py --copy-calibration` (one with FETCH_SIZE, one with
    WRITE_SIZE).  Each counter is summed over its instances per dispatch and
    averaged over the dispatches of the kernel.  The 4 GiB device copies of
    the same run (16 times the Infinity Cache) give the scale of each counter
    (true bytes / counted bytes); the 4 GiB reductions (a streaming read of
    known size) cross-check the FETCH_SIZE scale.  Writes the summary that
    read_traffic() reads for this cache type."""
    import csv
    import glob

    def per_dispatch(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            rows += list(csv.DictReader(open(f)))
        disp = {}
        for r in rows:
            if r["Counter_Name"] != counter:
                continue
            key = (int(r["Dispatch_Id"]), r["Kernel_Name"])
            disp[key] = disp.get(key, 0.0) + float(r["Counter_Value"])
        return sorted(disp.items())

    def mean(vals):
        return (sum(vals) / len(vals), len(vals)) if vals else (None, 0)

    res = {}
    for tag, d, ctr in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        disp = per_dispatch(d, ctr)
        # the timed step's products: the kernel's last `last` dispatches (the
        # autotuner's candidate shapes come before them)
        a, na = mean([v for (_, name), v in disp if "k_apply_tile<3," in name][-last:])
        # the calibration copies and reductions are the run's last three of each
        cp, nc = mean([v for (_, name), v in disp if "copyBuffer" in name][-3:])
        rd, nr = mean([v for (_, name), v in disp if "reduce_kernel" in name][-3:])
        if a is None or cp is None:
            raise SystemExit(f"{ctr}: apply dispatches {na}, copy dispatches {nc} in {d}")
        scale = COPY_BYTES / (cp * 1024.0)
        res[tag] = dict(kib_per_launch=a, launches=na, copy_kib=cp, copy_launches=nc, scale=scale,
                        read_kib=rd, read_launches=nr, bytes_per_launch=a * 1024.0 * scale)
    total = res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"]
    src = apply_src_sha()
    gib = COPY_BYTES / 2**30
    with open(traffic_file(dtype), "w") as f:
        f.write(f"# HBM traffic of k_apply_tile<J^T J fused, {dtype} cache> at the paper workload, {tile} tiles\n")
        f.write(f"# command: {command}\n")
        for tag in ("fetch", "write"):
            r = res[tag]
            f.write(f"# {tag}: {r['kib_per_launch']:.1f} KiB counted per launch over {r['launches']} launches; "
                    f"{gib:g} GiB copy counted {r['copy_kib']:.1f} KiB -> scale {r['scale']:.3f}")
            if r["read_kib"] is not None:
                f.write(f"; {gib:g} GiB streaming read (reduction) counted {r['read_kib']:.1f} KiB")
            f.write("\n")
        f.write(f"apply_src_sha256={src}\n")
        f.write(f"tile={tile}\n")
        f.write(f"cache_dtype={dtype}\n")
        f.write(f"fetch_bytes_per_launch={res['fetch']['bytes_per_launch']:.0f}\n")
        f.write(f"write_bytes_per_launch={res['write']['bytes_per_launch']:.0f}\n")
        f.write(f"traffic_bytes_per_launch={total:.0f}\n")
    return res


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _oracle_view_worker(task):
    """One view of an oracle workload in a child process: the explicit float64
    Jacobian's build and its J^T J p (SciPy CSR, one thread)."""
    name, v, reps = task
    from oracle import jacobian
    from paper_2409_12892_amd import scenegen as sg
    d = sg.config_scene(name)
    sc = d["scene"]
    cams = d["cams"][0].subset([v])
    t0 = time.perf_counter()
    J = jacobian.Jacobian(sc.x, cams, sc.sh_degree)
    t_build = time.perf_counter() - t0
    p = np.random.default_rng(0).normal(size=J.P * J.N)
    J.apply_JtJ(p)
    t1 = time.perf_counter()
    for _ in range(reps):
        J.apply_JtJ(p)
    return t_build, (time.perf_counter() - t1) / reps, J.n_pairs


def oracle_config_timing(name: str, reps: int = 3) -> dict:
    """The oracle on a whole small workload (every view), on one core (views
    one after another in this process) and on all cores (one view per child
    process, the views at once).  J^T J p of the subset is the sum over views,
    so the parallel apply time is the slowest view's."""
    import multiprocessing as mp
    from paper_2409_12892_amd import scenegen as sg
    V = sg.CONFIGS[name]["subsets"][0][0]
    t0 = time.perf_counter()
    one = [_oracle_view_worker((name, v, reps)) for v in range(V)]
    t_one = time.perf_counter() - t0
    procs = min(V, cpu_cores())
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(procs) as pool:
        par = pool.map(_oracle_view_worker, [(name, v, reps) for v in range(V)])
    t_par = time.perf_counter() - t0
    apply_one = sum(r[1] for r in one)
    apply_par = max(r[1] for r in par)
    pairs = sum(r[2] for r in one)
    return {"pairs": pairs, "one_core": {"build_s": round(sum(r[0] for r in one), 3),
                                         "apply_ms": round(apply_one * 1e3, 2),
                                         "applies_per_s": round(1.0 / apply_one, 3), "wall_s": round(t_one, 2)},
            "all_cores": {"processes": procs, "build_s": round(max(r[0] for r in par), 3),
                          "apply_ms": round(apply_par * 1e3, 2), "applies_per_s": round(1.0 / apply_par, 3),
                          "wall_s": round(t_par, 2)}}


def cpu_baseline(scene, cams, n_pairs_per_apply: int, tile: int = 16, crop: int = 64, reps: int = 3,
                 configs=("tiny", "precision")) -> dict:
    """The FP64 oracle, as it stands, on a bounded sample of the same
    workload: a crop x crop pixel window at the centre of view 0 (all
    Gaussians whose tile rectangle touches it).  Times the oracle's explicit
    Jacobian build and its J^T J p (SciPy CSR, float64, one thread), and
    scales the pair rate to applies/s of the full workload.  Beside it, the
    oracle on the whole tiny and precision workloads, on one core and on all
    cores (one view per process)."""
    from oracle import forward, jacobian
    cam = dict(cams.view(0))
    x0 = (cam["W"] // 2 - crop // 2) // tile * tile
    y0 = (cam["H"] // 2 - crop // 2) // tile * tile
    cc = dict(cam, cx=np.float32(cam["cx"] - x0), cy=np.float32(cam["cy"] - y0), W=crop, H=crop)
    x64 = scene.x.astype(np.float64)
    t0 = time.perf_counter()
    pr = forward.project(x64, cc, scene.sh_degree)
    bn = forward.bin_view(pr["y"], pr["z"], pr["radius"], pr["visible"], crop, crop, tile, tile)
    sel = np.unique(bn["values"])
    J = jacobian.Jacobian(x64[:, sel], OneCam(cc), scene.sh_degree, tile, tile)
    t_build = time.perf_counter() - t0
    p = np.random.default_rng(0).normal(size=J.P * J.N)
    J.apply_JtJ(p)
    t1 = time.perf_counter()
    for _ in range(reps):
        J.apply_JtJ(p)
    t_apply = (time.perf_counter() - t1) / reps
    pairs = J.n_pairs
    rate = pairs / t_apply
    out = dict(value=rate / n_pairs_per_apply, unit="applies/s", cores=1, kind="oracle",
               sample=(f"view 0, {crop}x{crop} centre crop ({(crop // tile) ** 2} tiles), {len(sel)} Gaussians, "
                       f"{pairs} pairs; J^T J p with the explicit float64 J (SciPy CSR, single thread) "
                       f"= {t_apply * 1e3:.1f} ms, i.e. {rate / 1e6:.2f} M pairs/s, scaled to the "
                       f"{n_pairs_per_apply} pairs of one full apply; oracle build of the sample "
                       f"{t_build:.1f} s"),
               pairs_per_s=rate, sample_build_s=t_build, sample_apply_ms=t_apply * 1e3,
               cpu_model=cpu_model(), cores_available=cpu_cores())
    out["configs"] = {}
    for name in configs:
        log(f"cpu baseline: oracle on the whole {name} workload")
        out["configs"][name] = oracle_config_timing(name)
    return out


def bench_batching(args, B, sg, torch) -> dict:
    """The PCG phase of one LM iteration over the four uneven image subsets
    of the batching workload (1.5M Gaussians, SH 3; 16 x 512x384, 24 x
    800x600, 32 x 1024x640, 48 x 1280x720): every subset's cache resident
    (compact builds), the tile shape of each autotuned, then Algorithm 1 with
    n_iters iterations for all subsets plus eq. combine-pcg, timed once as one
    batched call replaying a captured iteration and once as four sequential
    calls launched iteration by iteration, and once as one batched call in
    the persistent PCG kernel."""
    cfg = dict(sg.CONFIGS["batching"])
    d = sg.config_scene("batching", N=args.N)
    scene = d["scene"]
    dev = torch.device("cuda:0")
    x = torch.from_numpy(scene.x).to(dev)
    x_star = torch.from_numpy(d["x_star"]).to(dev)
    lam, n_iters, floor = float(cfg["lam"]), int(cfg["n_iters"]), 1e-2
    subs = []
    for i, cams in enumerate(d["cams"]):
        V, W, H = cfg["subsets"][i]
        noise = torch.from_numpy(np.concatenate([n.ravel() for n in d["noise"][i]])).to(dev)
        target = B.lm_render(x_star, scene.sh_degree, cams)
        target.add_(noise)
        del noise
        t0 = time.perf_counter()
        tile, scores = B.lm_autotune_tile(x, scene.sh_degree, cams, target, cache_dtype=args.cache_dtype,
                                          n_products=n_iters + 2)
        t1 = time.perf_counter()
        cache, b, _ = B.lm_build_cache(x, scene.sh_degree, cams, target, tile=tile, cache_dtype=args.cache_dtype,
                                       compact=True)
        M = B.lm_jacobi_diag(cache)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        del target
        inf = cache.info()
        log(f"subset {i}: {V} views {W}x{H}, tile {tile[0]}x{tile[1]} (autotune {t1 - t0:.1f} s), "
            f"{inf['n_pairs']} pairs, build + diagonal {1e3 * (t2 - t1):.0f} ms")
        subs.append(dict(cache=cache, b=b, M=M, tile=tile, scores=scores, info=inf, views=(V, W, H)))
    del x_star
    caches = [s_["cache"] for s_ in subs]
    bs, Ms = [s_["b"] for s_ in subs], [s_["M"] for s_ in subs]

    def batched():
        B.lm_pcg_use_graph(1)
        deltas, st = B.lm_pcg_solve(caches, bs, Ms, lam, n_iters, diag_floor=floor)
        return B.lm_combine_subsets(deltas, Ms), deltas, st

    def persistent():
        B.lm_pcg_use_graph(3)
        deltas, st = B.lm_pcg_solve(caches, bs, Ms, lam, n_iters, diag_floor=floor)
        return B.lm_combine_subsets(deltas, Ms), deltas, st

    def sequential():
        B.lm_pcg_use_graph(0)
        deltas, st = [], []
        for c_, b_, M_ in zip(caches, bs, Ms):
            dl, s1 = B.lm_pcg_solve([c_], [b_], [M_], lam, n_iters, diag_floor=floor)
            deltas += dl
            st += s1
        return B.lm_combine_subsets(deltas, Ms), deltas, st

    res = {}
    for name, fn in (("sequential", sequential), ("batched", batched), ("persistent", persistent)):
        fn()
        torch.cuda.synchronize()
        B.lm_profile_read()
        B.lm_profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out, deltas, st = fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        B.lm_profile_enable(False)
        prof = B.lm_profile_read()
        res[name] = dict(ms=(t1 - t0) * 1e3 / args.steps, out=out, deltas=deltas, iters=[s_["iters"] for s_ in st],
                         kernels={k: round(v[1] / args.steps, 3) for k, v in sorted(prof.items())})
        log(f"{name}: {res[name]['ms']:.1f} ms per PCG phase")
    B.lm_pcg_use_graph(2)
    diff = max(float((a_ - b_).norm() / max(b_.norm(), 1e-30))
               for a_, b_ in zip(res["batched"]["deltas"], res["sequential"]["deltas"]))
    comb = float((res["batched"]["out"] - res["sequential"]["out"]).norm() / max(res["sequential"]["out"].norm(), 1e-30))
    comb_p = float((res["persistent"]["out"] - res["sequential"]["out"]).norm()
                   / max(res["sequential"]["out"].norm(), 1e-30))
    pairs = sum(s_["info"]["n_pairs"] for s_ in subs)
    out = {
        "metric": "PCG phase ms, 4 uneven subsets: batched with graph replay vs sequential",
        "value": round(res["batched"]["ms"], 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": round(res["batched"]["ms"], 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.cache_dtype,
        "data": "synthetic",
        "config": {
            "workload": (f"batching: {scene.N} Gaussians SH{scene.sh_degree}, subsets "
                         + ", ".join(f"{V}x{W}x{H}" for V, W, H in cfg["subsets"])
                         + f", {args.cache_dtype} cache, {n_iters} PCG iterations + combine"),
            "N": scene.N, "subsets": cfg["subsets"], "pcg_iters": n_iters, "lambda": lam, "diag_floor": floor,
        },
        "sequential_ms": round(res["sequential"]["ms"], 3),
        "speedup": round(res["sequential"]["ms"] / res["batched"]["ms"], 3),
        "persistent_ms": round(res["persistent"]["ms"], 3),
        "rel_diff_batched_vs_sequential": {"deltas_max": diff, "combined": comb},
        "rel_diff_persistent_vs_sequential": {"combined": comb_p},
        "pcg_iters": res["batched"]["iters"],
        "subsets": [dict(views=s_["views"], tile=f"{s_['tile'][0]}x{s_['tile'][1]}", n_pairs=s_["info"]["n_pairs"],
                         n_tiles=s_["info"]["n_tiles"], cache_bytes=s_["info"]["cache_bytes"],
                         device_bytes=s_["info"]["device_bytes"],
                         autotune=[dict(tile=f"{c['tile'][0]}x{c['tile'][1]}", build_ms=round(c["build_ms"], 2),
                                        apply_ms=round(c["apply_ms"], 3)) for c in s_["scores"]])
                    for s_ in subs],
        "n_pairs_total": pairs,
        "device_bytes_total": sum(s_["info"]["device_bytes"] for s_ in subs),
        "kernels_ms_per_phase": {k: v["kernels"] for k, v in res.items()},
    }
    for s_ in subs:
        s_["cache"].destroy()
    return out


TRAIN_RUNS = 20          # seeded runs of the paper-scale plain-method workload
TRAIN_SAMPLES = 65536    # observed Gaussians drawn per run
TRAIN_STEPS = 600        # Adam steps
# target: the row-sum scaling unshrunk (at the learned-preconditioner workload
# the exact targets take 22 PCG iterations unshrunk, 26 shrunk by 1/2 and 33
# as per-parameter means alone, against 26 for Jacobi)
TRAIN_SHRINK = 1.0


def train_learned_mlp(args, B, sg, torch, lam, floor):
    """The perceptron of the learned preconditioner, trained on the GPU on
    20 seeded runs of the paper-scale plain-method workload (1,000,000
    Gaussians, SH degree 3, 32 views 1024x640; seeds 1000..1019; targets
    rendered from the perturbed parameters plus pixel noise; the scenes are
    drawn on host threads while the GPU processes the previous run): per
    run the bfloat16 cache (the deployed cache type), the Jacobi diagonal,
    the features and the exact targets (each Gaussian's block rows summed
    over the views in float64; the unshrunk row-sum scaling, TRAIN_SHRINK)
    of TRAIN_SAMPLES observed Gaussians drawn per run (seeded), then
    TRAIN_STEPS Adam steps on all runs' samples."""
    import concurrent.futures as cf
    dev = torch.device("cuda:0")
    feats, ts, masks = [], [], []
    gen = torch.Generator(device="cpu")
    gen.manual_seed(2024)
    n_obs = []
    t_data = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=min(8, max(1, (os.cpu_count() or 2) // 2))) as ex:
        futs = [ex.submit(sg.config_scene, "paper", seed=1000 + r) for r in range(TRAIN_RUNS)]
        for r in range(TRAIN_RUNS):
            d = futs[r].result()
            futs[r] = None
            sc, cams = d["scene"], d["cams"][0]
            x = torch.from_numpy(sc.x).to(dev)
            target = B.lm_render(torch.from_numpy(d["x_star"]).to(dev), sc.sh_degree, cams)
            target.add_(torch.from_numpy(np.concatenate([n.ravel() for n in d["noise"][0]])).to(dev))
            del d
            cache, _, _ = B.lm_build_cache(x, sc.sh_degree, cams, target, tile=(8, 32), cache_dtype="bf16",
                                           want_b=False)
            M = B.lm_jacobi_diag(cache)
            f = B.lm_precond_features(cache, x, M)
            t, m = B.lm_precond_targets(cache, lam, floor, shrink=TRAIN_SHRINK)
            cache.destroy()
            obs = torch.nonzero(m[0] > 0).flatten().cpu()
            n_obs.append(int(obs.numel()))
            pick = obs[torch.randperm(obs.numel(), generator=gen)[:TRAIN_SAMPLES]].to(dev)
            feats.append(f[:, pick])
            ts.append(t[:, pick])
            masks.append(m[:, pick])
            del x, target, M, f, t, m
    data_s = time.perf_counter() - t_data
    feat, t, mask = torch.cat(feats, 1).contiguous(), torch.cat(ts, 1).contiguous(), torch.cat(masks, 1).contiguous()
    n_samples = int(feat.shape[1])
    log(f"training data: {TRAIN_RUNS} runs, {n_samples} Gaussians ({data_s:.1f} s)")
    P = t.shape[0]
    trainer = B.MlpTrainer(B.mlp_init(P, seed=3), lr=3e-3)
    loss0, _ = trainer.step(feat, t, mask, lr=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(TRAIN_STEPS):
        trainer.step(feat, t, mask)
    torch.cuda.synchronize()
    train_ms = (time.perf_counter() - t0) * 1e3 / TRAIN_STEPS
    loss1, _ = trainer.step(feat, t, mask, lr=0.0)
    log(f"training: loss {loss0.item():.4f} -> {loss1.item():.4f}, {train_ms:.3f} ms per Adam step "
        f"({n_samples} samples)")
    del feat, t, mask, feats, ts, masks
    torch.cuda.empty_cache()
    return trainer, dict(runs=TRAIN_RUNS, workload="1000000 Gaussians SH3, 32 views 1024x640, bf16 cache",
                         observed_per_run=n_obs, samples=n_samples, data_s=round(data_s, 1), steps=TRAIN_STEPS,
                         ms_per_step=round(train_ms, 3), loss_first=round(loss0.item(), 5),
                         loss_last=round(loss1.item(), 5))


# parameter groups (rows of x): mean, log-scale, quaternion, opacity, SH
# degree-0 colour, SH degrees 1-3
PARAM_GROUPS = (("mean", 0, 3), ("log_scale", 3, 6), ("quaternion", 6, 10), ("opacity", 10, 11),
                ("sh_dc", 11, 14), ("sh_rest", 14, 59))


def bench_learned(args, B, sg, torch) -> dict:
    """The learned diagonal preconditioner at the learned-preconditioner
    workload, one subset at full size (3M Gaussians, SH 3, 40 views
    1280x720, bfloat16 cache; the workload's four subsets would not leave
    room for the build transients).  The perceptron is trained on the GPU on
    20 seeded runs of the paper-scale workload (train_learned_mlp); then, on the workload
    subset, Algorithm 1 runs to a relative residual of 1e-2 with the Jacobi,
    the learned and the exact-target scalings (shrink 1/2, unshrunk, and the
    per-parameter means alone), with constant rescalings of each parameter
    group, and with the block-Jacobi preconditioner."""
    cfg = dict(sg.CONFIGS["learned"])
    lam, floor, tol, max_it = float(cfg["lam"]), 1e-2, 1e-2, 200
    dev = torch.device("cuda:0")

    def subset(N, views, seed):
        d = sg.config_scene("learned", N=N, subsets=[views], seed=seed)
        sc, cams = d["scene"], d["cams"][0]
        x = torch.from_numpy(sc.x).to(dev)
        noise = torch.from_numpy(np.concatenate([n.ravel() for n in d["noise"][0]])).to(dev)
        target = B.lm_render(torch.from_numpy(d["x_star"]).to(dev), sc.sh_degree, cams)
        target.add_(noise)
        del noise
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cache, b, _ = B.lm_build_cache(x, sc.sh_degree, cams, target, cache_dtype=args.cache_dtype, compact=True)
        M = B.lm_jacobi_diag(cache)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        del target
        return dict(scene=sc, x=x, cache=cache, b=b, M=M, build_ms=(t1 - t0) * 1e3)

    trainer, training = train_learned_mlp(args, B, sg, torch, lam, floor)
    P = sg.n_params(int(cfg["deg"]))

    V, W, H = cfg["subsets"][0]
    log(f"workload subset: {cfg['N']} Gaussians, {V} views {W}x{H}")
    ws = subset(int(cfg["N"]), (V, W, H), int(cfg["seed"]))
    info = ws["cache"].info()
    log(f"built: {info['n_pairs']} pairs, {ws['build_ms']:.0f} ms with the diagonal")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        f = B.lm_precond_features(ws["cache"], ws["x"], ws["M"])
        _, scale, nf = B.lm_mlp_forward(trainer.w, f, P, want_s=False)
    torch.cuda.synchronize()
    pre_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    def exact_scale(shrink):
        tt, mm = B.lm_precond_targets(ws["cache"], lam, floor, shrink=shrink)
        out = torch.where(mm > 0, torch.exp(tt), torch.ones_like(tt))
        del tt, mm
        return out

    def solve(sc_, timed=True):
        kw = dict(scales=None if sc_ is None else [sc_], diag_floor=floor)
        if timed:
            B.lm_pcg_solve([ws["cache"]], [ws["b"]], [ws["M"]], lam, max_it, tol, B.TOL_RELATIVE, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = B.lm_pcg_solve([ws["cache"]], [ws["b"]], [ws["M"]], lam, max_it, tol, B.TOL_RELATIVE, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        return dict(iters=int(st[0]["iters"]), ms=round(ms, 2), rel_res=float(np.sqrt(st[0]["history"][-1])))

    res = {}
    for name, mk in (("jacobi", lambda: None), ("learned", lambda: scale),
                     ("exact_target", lambda: exact_scale(0.5)), ("exact_target_unshrunk", lambda: exact_scale(1.0)),
                     ("exact_target_means_only", lambda: exact_scale(0.0))):
        res[name] = solve(mk())
        log(f"{name}: {res[name]['iters']} iterations, {res[name]['ms']:.1f} ms")
    # constant rescalings of whole parameter groups against Jacobi (how far
    # any per-parameter-type diagonal can move the iteration count)
    groups = {}
    for gname, g0, g1 in PARAM_GROUPS:
        for f in (0.5, 2.0):
            sc_ = torch.ones(P, int(cfg["N"]), device=dev)
            sc_[g0:g1] = f
            r = solve(sc_, timed=False)
            groups[f"{gname}_x{f:g}"] = r["iters"]
            del sc_
    log(f"group rescalings (iterations; Jacobi {res['jacobi']['iters']}): {groups}")
    # block-Jacobi (exact per-Gaussian damped blocks): factorisation timed on
    # its own (a call that recomputes the factors and synchronises), then the
    # solve with the factors kept
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, n_bj_fallback = B.lm_block_precond_apply(ws["cache"], ws["b"], lam, floor, count_fallback=True)
    factor_ms = (time.perf_counter() - t0) * 1e3
    B.lm_pcg_solve([ws["cache"]], [ws["b"]], [ws["M"]], lam, max_it, tol, B.TOL_RELATIVE, diag_floor=floor,
                   block=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = B.lm_pcg_solve([ws["cache"]], [ws["b"]], [ws["M"]], lam, max_it, tol, B.TOL_RELATIVE,
                           diag_floor=floor, block=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    res["block_jacobi"] = dict(iters=int(st[0]["iters"]), ms=round(ms, 2), factor_ms=round(factor_ms, 2),
                               rel_res=float(np.sqrt(st[0]["history"][-1])), n_fallback=n_bj_fallback)
    log(f"block_jacobi: {res['block_jacobi']['iters']} iterations, {ms:.1f} ms + factors {factor_ms:.1f} ms")
    ws["cache"].destroy()
    j, l_ = res["jacobi"], res["learned"]
    return {
        "metric": "PCG to relative residual 1e-2: ms (iterations), learned vs Jacobi preconditioner",
        "value": round(l_["ms"] + pre_ms, 2),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": round(l_["ms"] + pre_ms, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.cache_dtype,
        "data": "synthetic",
        "config": {"workload": (f"learned preconditioner: {cfg['N']} Gaussians SH3, one subset of {V} views "
                                f"{W}x{H} (of the workload's four), {args.cache_dtype} cache"),
                   "N": int(cfg["N"]), "views": V, "width": W, "height": H, "lambda": lam, "diag_floor": floor,
                   "tol_relative": tol},
        "jacobi": j, "learned": l_, "exact_target": res["exact_target"],
        "exact_target_unshrunk": res["exact_target_unshrunk"],
        "exact_target_means_only": res["exact_target_means_only"], "group_rescalings_iters": groups,
        "block_jacobi": res["block_jacobi"],
        "features_and_forward_ms": round(pre_ms, 3),
        "speedup_vs_jacobi": round(j["ms"] / (l_["ms"] + pre_ms), 3),
        "training": training,
        "n_pairs": info["n_pairs"], "build_and_diag_ms": round(ws["build_ms"], 1),
        "n_fallback": int(nf.item()),
    }


def bench_thin(args, B, sg, torch) -> dict:
    """The thinned cache (paper section 4.4): bytes and fused J^T J tile-pass
    time at the paper workload (float32: full cache and windows of 8 and 32)
    and at one subset of the learned-preconditioner workload (3M Gaussians,
    40 views 1280x720: the full bfloat16 cache against float32 thinned caches
    with windows of 8 and 32), 8x32 tiles; each tile pass timed over
    `--steps` products after one untimed product."""
    dev = torch.device("cuda:0")
    out = []
    for name, subsets, variants in (("paper", None, (("f32", 0), ("f32", 8), ("f32", 32))),
                                    ("learned", [(40, 1280, 720)], (("bf16", 0), ("f32", 8), ("f32", 32)))):
        d = sg.config_scene(name, subsets=subsets)
        sc, cams = d["scene"], d["cams"][0]
        x = torch.from_numpy(sc.x).to(dev)
        target = B.lm_render(torch.from_numpy(d["x_star"]).to(dev), sc.sh_degree, cams)
        target.add_(torch.from_numpy(np.concatenate([n.ravel() for n in d["noise"][0]])).to(dev))
        del d
        p = torch.full_like(x, 0.01)
        for dt, K in variants:
            cache, b, _ = B.lm_build_cache(x, sc.sh_degree, cams, target, tile=(8, 32), cache_dtype=dt, thin_window=K)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cache, b, _ = B.lm_build_cache(x, sc.sh_degree, cams, target, tile=(8, 32), cache_dtype=dt, thin_window=K,
                                           cache=cache, b=b)
            torch.cuda.synchronize()
            build_ms = (time.perf_counter() - t0) * 1e3
            B.lm_apply_JtJ(cache, p)
            torch.cuda.synchronize()
            B.lm_profile_read()
            B.lm_profile_enable(True)
            for _ in range(args.steps):
                B.lm_apply_JtJ(cache, p)
            torch.cuda.synchronize()
            prof = B.lm_profile_read()
            B.lm_profile_enable(False)
            n, tms = prof.get("apply_tile_JtJ", (0, 0.0))
            info = cache.info()
            r = dict(workload=name, cache_dtype=dt, thin_window=K, n_pairs=info["n_pairs"],
                     cache_bytes=info["cache_bytes"], device_bytes=info["device_bytes"],
                     cache_bytes_per_pair=round(info["cache_bytes"] / max(info["n_pairs"], 1), 3),
                     build_ms=round(build_ms, 1), tile_pass_ms=round(tms / max(n, 1), 3),
                     product_ms=round(sum(v[1] for v in prof.values()) / max(args.steps, 1), 3))
            log(f"{name} {dt} K={K}: {r['cache_bytes'] / 1e9:.2f} GB cache ({r['cache_bytes_per_pair']} B/pair), "
                f"tile pass {r['tile_pass_ms']} ms, build {r['build_ms']} ms")
            out.append(r)
            cache.destroy()
            del b
            torch.cuda.empty_cache()
        del x, target, p
        torch.cuda.empty_cache()
    return {"metric": "thinned cache: bytes and J^T J tile-pass ms against the full cache", "value": None,
            "unit": "ms", "n_gpus": 1, "steps": args.steps, "data": "synthetic", "results": out}


def bench_deploy(args, B, sg, torch, brief: bool = False) -> dict:
    """One LM step's solve phase at the learned-preconditioner workload
    (3M Gaussians, SH 3, four subsets of 40 views 1280x720), to a relative
    residual of 1e-2 in each subset, in two forms:
      plain: float32 caches, one subset at a time in one reused cache
             (build, Jacobi diagonal, Algorithm 1 with Jacobi), then
             eq. combine-pcg;
      full:  bfloat16 compact caches sharing one scratch handle for the
             build transients, subsets held together in groups of
             --deploy-group (default: all four; the builds' transients are
             released before the diagonals, and each cache is trimmed to
             what PCG reads), the learned scaling, one batched
             graph-replayed Algorithm 1 per group, then eq. combine-pcg;
      full_thin: the same with float32 thinned caches (--deploy-thin) and
             the persistent PCG kernel;
      bf16_learned_sequential: bfloat16 and the learned scaling, one subset
             at a time in one reused cache.
    brief: the plain and full forms only (the comparison that the default
    bench line carries).
    The cache handles persist from the warm-up run into the timed run (as in
    an LM loop), and the library's memory comes from PyTorch's caching
    allocator (--deploy-alloc torch, the default), so the transients that a
    compact build releases serve the next build; the perceptron is trained
    first, outside the timed regions."""
    cfg = dict(sg.CONFIGS["learned"])
    lam, floor, tol, max_it = float(cfg["lam"]), 1e-2, 1e-2, 80
    dev = torch.device("cuda:0")
    trainer, training = train_learned_mlp(args, B, sg, torch, lam, floor)
    if args.deploy_alloc == "torch":
        B.use_torch_allocator()
    log("workload: 3000000 Gaussians, 4 subsets of 40 views 1280x720")
    d = sg.config_scene("learned")
    sc = d["scene"]
    P, N = sc.P, sc.N
    x = torch.from_numpy(sc.x).to(dev)
    x_star = torch.from_numpy(d["x_star"]).to(dev)
    targets = []
    for i, cams in enumerate(d["cams"]):
        tg = B.lm_render(x_star, sc.sh_degree, cams)
        tg.add_(torch.from_numpy(np.concatenate([n.ravel() for n in d["noise"][i]])).to(dev))
        targets.append(tg)
    del x_star, d["noise"]
    torch.cuda.synchronize()
    tile = tuple(int(v) for v in (args.tile if args.tile != "auto" else "8x32").split("x"))

    group = max(1, min(4, int(args.deploy_group)))
    phases = {}

    def mark(name, t0):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        phases[name] = phases.get(name, 0.0) + (t1 - t0) * 1e3
        return t1

    # cache handles live across the warm-up and the timed run, as in an LM
    # loop: the timed run allocates nothing new
    plain_h = [None]
    full_h = [None] * group + [B.Cache()]          # the last one: scratch of the compact builds

    def sequential(dtype, learned, tag):
        deltas, Ms, its = [], [], []
        cache = plain_h[0]
        for i, cams in enumerate(d["cams"]):
            t0 = time.perf_counter()
            cache, b, _ = B.lm_build_cache(x, sc.sh_degree, cams, targets[i], tile=tile, cache_dtype=dtype,
                                           cache=cache)
            M = B.lm_jacobi_diag(cache)
            scales = None
            if learned:
                f = B.lm_precond_features(cache, x, M)
                _, scale, _ = B.lm_mlp_forward(trainer.w, f, P, want_s=False)
                scales = [scale]
                del f
            t0 = mark(f"{tag}_build_diag", t0)
            dl, st = B.lm_pcg_solve([cache], [b], [M], lam, max_it, tol, B.TOL_RELATIVE, scales=scales,
                                    diag_floor=floor)
            mark(f"{tag}_pcg", t0)
            deltas.append(dl[0])
            Ms.append(M)
            its.append(int(st[0]["iters"]))
            del b
        out = B.lm_combine_subsets(deltas, Ms)
        torch.cuda.synchronize()
        plain_h[0] = cache
        mem_tables[tag] = dict(subset=cache.memory())
        return out, its, cache.info()["device_bytes"]

    def full_form(dtype, grp, thin, handles, tag, mode):
        """Compact caches held grp at a time (sharing the last handle as the
        scratch of their build transients), the learned scaling, one batched
        Algorithm 1 per group in PCG launch mode `mode`, then eq. combine-pcg."""
        deltas, Ms_all, its, mem = [], [], [], 0
        B.lm_pcg_use_graph(mode)
        for g0 in range(0, 4, grp):
            caches, bs, Ms, scales = [], [], [], []
            t0 = time.perf_counter()
            for k, i in enumerate(range(g0, min(4, g0 + grp))):
                cache, b, _ = B.lm_build_cache(x, sc.sh_degree, d["cams"][i], targets[i], tile=tile,
                                               cache_dtype=dtype, compact=True, cache=handles[k],
                                               scratch=handles[grp], thin_window=thin)
                handles[k] = cache
                caches.append(cache)
                bs.append(b)
            mem_tables[tag] = dict(subset_built=caches[0].memory(), scratch=handles[grp].memory())
            if g0 + grp >= 4:
                # the last group's builds are done: their transients go back
                # (to the allocator's pool) before the diagonals' Gram values
                handles[grp].destroy()
                handles[grp] = B.Cache()
            for cache in caches:
                M = B.lm_jacobi_diag(cache)
                f = B.lm_precond_features(cache, x, M)
                _, scale, _ = B.lm_mlp_forward(trainer.w, f, P, want_s=False)
                cache.trim()                     # the Gram values: not read by PCG
                Ms.append(M)
                scales.append(scale)
                del f
            t0 = mark(f"{tag}_build_diag_scale", t0)
            dl, st = B.lm_pcg_solve(caches, bs, Ms, lam, max_it, tol, B.TOL_RELATIVE, scales=scales,
                                    diag_floor=floor)
            mark(f"{tag}_pcg", t0)
            deltas += dl
            Ms_all += Ms
            its += [int(s_["iters"]) for s_ in st]
            mem = max(mem, sum(c.info()["device_bytes"] for c in caches))
            mem_tables[tag]["subset_solved"] = caches[0].memory()
            del bs, scales
        B.lm_pcg_use_graph(2)
        out = B.lm_combine_subsets(deltas, Ms_all)
        torch.cuda.synchronize()
        return out, its, mem

    thin_k = int(args.deploy_thin)
    thin_h = [None] * 4 + [B.Cache()]
    mem_tables = {}            # device bytes per buffer: one subset's cache (and the scratch handle)

    res = {}
    forms = [("plain", lambda: sequential("f32", False, "plain"))]
    if not brief:
        forms.append(("bf16_learned_sequential", lambda: sequential("bf16", True, "seq")))
    forms.append(("full", lambda: full_form("bf16", group, 0, full_h, "full", 2)))
    if thin_k > 0 and not brief:
        forms.append(("full_thin", lambda: full_form("f32", 4, thin_k, thin_h, "thin", 3)))
    for name, fn in forms:
        # warm-up: allocations and code objects; the memory it freed stays in
        # the caching allocator's pool for the timed run, as in an LM loop
        fn()
        torch.cuda.synchronize()
        phases.clear()
        t0 = time.perf_counter()
        r = fn()
        ms = (time.perf_counter() - t0) * 1e3
        res[name] = dict(ms=round(ms, 1), pcg_iters=r[1], cache_device_bytes=int(r[2]),
                         phases_ms={k: round(v, 1) for k, v in phases.items()})
        res[name]["delta"] = r[0]
        log(f"{name}: {ms:.1f} ms, PCG iterations {r[1]}, phases {res[name]['phases_ms']}")
        hl = full_h if name == "full" else (thin_h if name == "full_thin" else plain_h)
        for k, h in enumerate(hl):
            if h is not None:
                h.destroy()
            hl[k] = None
        torch.cuda.empty_cache()
    dp, df = res["plain"].pop("delta"), res["full"].pop("delta")
    if "bf16_learned_sequential" in res:
        res["bf16_learned_sequential"].pop("delta")
    dt = res["full_thin"].pop("delta") if "full_thin" in res else None
    if args.deploy_alloc == "torch":
        B.use_torch_allocator(False)
    diff = float(torch.linalg.vector_norm(df - dp) / torch.linalg.vector_norm(dp))
    diff_thin = None if dt is None else float(torch.linalg.vector_norm(dt - dp) / torch.linalg.vector_norm(dp))
    return {
        "metric": "LM solve phase to relative residual 1e-2 in every subset: ms, full form vs plain",
        "value": res["full"]["ms"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": res["full"]["ms"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": (f"learned preconditioner deployment: {N} Gaussians SH3, 4 subsets of 40 views "
                                f"1280x720; plain = float32, sequential subsets, Jacobi; full = bfloat16, subsets "
                                f"resident in groups of {group}, batched graph-replayed PCG, learned scaling"),
                   "N": N, "subsets": 4, "views": 40, "width": 1280, "height": 720, "lambda": lam,
                   "diag_floor": floor, "tol_relative": tol, "tile": f"{tile[0]}x{tile[1]}", "group": group,
                   "allocator": args.deploy_alloc},
        "plain": res["plain"], "full": res["full"], "bf16_learned_sequential": res.get("bf16_learned_sequential"),
        "full_thin": res.get("full_thin"),
        "speedup_full_vs_plain": round(res["plain"]["ms"] / res["full"]["ms"], 3),
        "speedup_full_thin_vs_plain": (round(res["plain"]["ms"] / res["full_thin"]["ms"], 3)
                                       if "full_thin" in res else None),
        "device_memory_per_buffer": mem_tables,
        "combined_direction_rel_diff": diff,
        "combined_direction_rel_diff_thin": diff_thin,
        "training": training,
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="paper")
    ap.add_argument("--cache-dtype", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--tile", default="auto",
                    help="tile shape WxH, or auto: lm_autotune_tile on the workload before the timed region")
    ap.add_argument("--N", type=int, default=None, help="override the number of Gaussians")
    ap.add_argument("--views", type=int, default=None, help="override the views of the subset")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--deploy-alloc", default="torch", choices=["hip", "torch"],
                    help="device memory of --config deploy: hipMalloc, or PyTorch's caching allocator")
    ap.add_argument("--deploy-thin", type=int, default=32,
                    help="--config deploy: also run the full form with thinned caches (this window; 0: not), "
                         "all four subsets resident, persistent-kernel PCG")
    ap.add_argument("--deploy-sub", type=int, default=1,
                    help="paper workload: after the timed steps, also run the plain-vs-full solve-phase "
                         "comparison of --config deploy (plain and full forms) and attach it as `deploy`")
    ap.add_argument("--deploy-group", type=int, default=4,
                    help="subsets held and solved together by the full form of --config deploy")
    ap.add_argument("--precond", default="jacobi", choices=["jacobi", "block"],
                    help="Jacobi (Algorithm 1) or the per-Gaussian block-Jacobi preconditioner")
    ap.add_argument("--objective", default="l2", choices=["l2", "l1_ssim"],
                    help="least-squares RGB residuals (the configured workload) or the paper's square-root "
                         "L1 / SSIM residuals")
    ap.add_argument("--thin", type=int, default=0,
                    help="thinned cache: blend state of every K-th contributor per pixel (0: full cache)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, copy 4 GiB device to device and sum 4 GiB three times "
                         "each (the reference kernels for rocprofv3 byte counters)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the traffic summary from two rocprofv3 --pmc output folders and exit")
    ap.add_argument("--pmc-command", default="", help="command line recorded in the traffic summary")
    ap.add_argument("--pmc-tile", default="", help="tile shape of the counted runs, recorded in the summary")
    args = ap.parse_args()
    if args.summarize_pmc:
        res = summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.pmc_command, args.pmc_tile,
                            args.cache_dtype)
        print(json.dumps(res))
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU layout (one image subset per GPU, one all-reduce of the weighted "
              "mean) is not run.", file=sys.stderr)
        return 2

    import torch

    from paper_2409_12892_amd import binding as B
    from paper_2409_12892_amd import scenegen as sg

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 3
    B.load()
    if args.config == "batching":
        print(json.dumps(bench_batching(args, B, sg, torch)), flush=True)
        return 0
    if args.config == "learned":
        print(json.dumps(bench_learned(args, B, sg, torch)), flush=True)
        return 0
    if args.config == "deploy":
        print(json.dumps(bench_deploy(args, B, sg, torch)), flush=True)
        return 0
    if args.config == "thin":
        print(json.dumps(bench_thin(args, B, sg, torch)), flush=True)
        return 0
    cfg = dict(sg.CONFIGS[args.config])
    subsets = cfg["subsets"][:1]
    if args.views is not None:
        subsets = [(args.views, subsets[0][1], subsets[0][2])]
    log(f"generating scene: config={args.config} N={args.N or cfg['N']} subsets={subsets}")
    d = sg.config_scene(args.config, N=args.N, subsets=subsets)
    scene, cams = d["scene"], d["cams"][0]
    V, W, H = subsets[0]
    dev = torch.device("cuda:0")
    x = torch.from_numpy(scene.x).to(dev)
    x_star = torch.from_numpy(d["x_star"]).to(dev)
    noise = torch.from_numpy(np.concatenate([n.ravel() for n in d["noise"][0]])).to(dev)
    target = B.lm_render(x_star, scene.sh_degree, cams)      # targets: 16x16 binning whatever the tile
    target.add_(noise)
    del x_star, noise
    torch.cuda.synchronize()
    lam, n_iters = float(cfg["lam"]), int(cfg["n_iters"])
    log(f"inputs resident: N={scene.N} P={scene.P} views={V} {W}x{H}")
    tile_scores = None
    if args.tile == "auto":
        (tw, th), sc_ = B.lm_autotune_tile(x, scene.sh_degree, cams, target, cache_dtype=args.cache_dtype,
                                          n_products=n_iters + 2, thin_window=args.thin)
        tile_scores = [dict(tile=f"{c['tile'][0]}x{c['tile'][1]}", build_ms=round(c["build_ms"], 2),
                            apply_ms=round(c["apply_ms"], 3)) for c in sc_]
        log(f"autotuned tile {tw}x{th}: " + ", ".join(f"{c['tile']} {c['build_ms']:.0f}/{c['apply_ms']:.1f} ms"
                                                       for c in tile_scores))
    else:
        tw, th = (int(v) for v in args.tile.split("x"))

    from paper_2409_12892_amd.lm_loop import LMConfig, LMSolver
    solver = LMSolver(x, scene.sh_degree, cams, target,
                      LMConfig(lam=lam, n_iters=n_iters, tile=(tw, th), cache_dtype=args.cache_dtype,
                               objective=args.objective, precond=args.precond, thin_window=args.thin))

    def show(tag, rec):
        log(f"{tag}: E {rec['E0']:.4g} -> {rec['E1']:.4g} gamma {rec['gamma']:g} rho {rec['rho']:.3g} "
            f"{'accepted' if rec['accepted'] else 'rejected'} lambda {rec['lam']:.3g} -> {rec['lam_next']:.3g}")

    # the configured workload is an LM run of `lm_steps` iterations from the
    # initial scene (the paper's second stage: 5 LM iterations): the bench
    # repeats such runs, every iteration a full one, restarting from the
    # initial parameters after each run
    lm_run = int(cfg.get("lm_steps", 0))
    x_init = x.clone()
    n_done = [0]

    def lm_step():
        if lm_run and n_done[0] and n_done[0] % lm_run == 0:
            solver.restart(x_init)
        n_done[0] += 1
        return solver.iteration()

    for i in range(args.warmup):
        show(f"warmup step {i + 1}/{args.warmup}", lm_step())
    torch.cuda.synchronize()
    B.lm_profile_read()
    B.lm_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        show(f"timed step {i + 1}/{args.steps}", lm_step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    B.lm_profile_enable(False)
    prof = B.lm_profile_read()
    if args.copy_calibration:
        src_buf = torch.empty(COPY_BYTES // 4, device=dev)
        dst_buf = torch.empty_like(src_buf)
        src_buf.fill_(1.0)
        for _ in range(3):
            dst_buf.copy_(src_buf)
        for _ in range(3):
            dst_buf.sum()
        torch.cuda.synchronize()
        del src_buf, dst_buf
    info = solver.cache.info()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    applies = (n_iters + 1) * args.steps   # the J^T J products of Algorithm 1 (the ratio's J delta is J only)
    value = applies / (t1 - t0)

    launches, tot_ms = prof.get("apply_tile_JtJ", (0, 0.0))
    apply_ms = tot_ms / max(launches, 1)
    alg = apply_tile_alg_bytes(info, weighted=args.objective != "l2")
    achieved = alg / (apply_ms * 1e-3) / 1e9
    # the counter summary covers the least-squares (unweighted) pass
    traffic = read_traffic(alg, f"{tw}x{th}", args.cache_dtype) if args.objective == "l2" else None
    full_apply_ms = sum(prof.get(k, (0, 0.0))[1] for k in ("tangent", "apply_tile_JtJ", "chain", "pcg_vector")) \
        / max(launches, 1)
    log(f"steps done: {ms_per_step:.1f} ms/step, apply tile pass {apply_ms:.3f} ms, {achieved:.0f} GB/s")

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.cache_dtype,
        "data": "synthetic",
        "config": {
            "workload": (f"LM iteration, {'plain method' if args.objective == 'l2' else 'square-root L1/SSIM objective'}: "
                         f"{scene.N} Gaussians SH{scene.sh_degree}, {V} views "
                         f"{W}x{H} in one subset, {args.cache_dtype} cache, {n_iters} {'Jacobi' if args.precond == 'jacobi' else 'block-Jacobi'}-PCG iterations"
                         + (f", LM runs of {lm_run} iterations from the initial scene" if lm_run else "")),
            "objective": args.objective, "precond": args.precond,
            "N": scene.N, "P": scene.P, "views": V, "width": W, "height": H, "tile": f"{tw}x{th}",
            "tile_autotune": tile_scores,
            "cache_dtype": args.cache_dtype, "pcg_iters": n_iters, "lambda": lam,
            "diag_floor": solver.cfg.diag_floor, "line_search_views": int(len(solver.ls_idx)),
            "lm_run_length": lm_run,
        },
        "roofline": {
            "kernel": "k_apply_tile<J^T J fused>",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "alg_bytes_per_launch": alg,
            "avg_launch_ms": round(apply_ms, 4),
        },
        "lm_iter_ms": round(ms_per_step, 3),
        "apply_JtJ_ms": round(full_apply_ms, 4),
        "apply_JtJ_per_s": round(1e3 / full_apply_ms, 2) if full_apply_ms > 0 else None,
        "kernels_ms_per_step": {k: round(v[1] / args.steps, 3) for k, v in sorted(prof.items())},
        "kernel_launches": {k: v[0] for k, v in sorted(prof.items())},
        "cache": {k: info[k] for k in ("n_keys", "n_pairs", "n_segments", "n_gv", "n_tiles", "cache_bytes",
                                        "device_bytes")},
        "lm_steps": [{k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}
                     for r in solver.history],
        "paper_context": PAPER_CONTEXT,
    }
    if args.cpu_baseline:
        log("cpu baseline: oracle on a bounded crop of view 0")
        try:
            out["cpu_baseline"] = cpu_baseline(scene, cams, info["n_pairs"], tile=16)
        except Exception as e:  # the GPU result stands even if the CPU sample fails
            out["cpu_baseline"] = {"value": None, "error": repr(e)}
        log("cpu baseline done")
    solver.close()
    if args.deploy_sub and args.config == "paper":
        # the second comparison: BF16 + batched + learned solve phase against
        # the plain float32 Jacobi form at the learned-preconditioner workload
        del solver, x, target, x_init
        torch.cuda.empty_cache()
        log("deploy comparison: plain and full forms at the learned-preconditioner workload")
        try:
            dep = bench_deploy(args, B, sg, torch, brief=True)
            out["deploy"] = {k: dep[k] for k in ("metric", "value", "unit", "config", "plain", "full",
                                                "speedup_full_vs_plain", "combined_direction_rel_diff",
                                                "training")}
        except Exception as e:  # the headline line stands even if the comparison fails
            out["deploy"] = {"value": None, "error": repr(e)}
        log("deploy comparison done")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
