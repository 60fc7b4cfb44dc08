"""Benchmark of the EOD-ABE hot path on one MI355X.

One step = one eodabe_factor call (Alg. 1 basis extraction + Alg. 2 closing
steps, returning rank, U, D, V^T) on a synthetic input already resident in
HBM.  Prints one JSON line (see the keys below).  Only one GPU is used:
``--gpus`` above 1 exits with a message.

Workloads (``--workload``):
  image4096      4096 x 4096 FP32 image-like matrix in [0, 255] (64 Gaussian
                 blobs + 32 cosine modes), pixel noise std 0.05, tol 1e-3
                 (default; the low-rank reading of the 4096^2 image case).
  image4096_n05  same image with noise std 0.5 as written (rank ~ 0.75 n).
  hsi262144      262144 x 200 FP32 hyperspectral-shaped matrix, tol 1e-2.
  lowrank512     512 x 512 FP64 exact rank 20 + 1e-12 noise, tol 1e-8.
  tiles1024      1024 FP32 tiles, sides uniform in [64, 1024], exact-rank
                 content 5..80 + N(0, 1e-4) noise, tol 1e-4: one step is one
                 eodabe_factor_batched call over all tiles, compared with
                 1024 sequential eodabe_factor calls on the same tiles.
  learned4096    six 4096 x 4096 FP32 matrices U diag(s) V^T + noise with
                 geometric singular-value decay over ranks 96..416, tol 1e-4:
                 one step factors all six with the learned warm start
                 (paper_2506_22713_amd/predictor.ckpt), compared with the
                 plain loop on the same matrices.

With the default workload the line's config also carries ``end_to_end``
(the whole factorization against the HBM and MFMA roofs) and
``subresults``: the other configurations (the 4096^2 rank sweep 95..416,
the hyperspectral matrix in FP32 and the FP16 form, the image as written,
the 512^2 FP64 matrix, colour images, complex input, the hyperspectral KNN,
the 1024 tiles batched against sequential), each measured briefly on the
GPU; the cpu_baseline leg adds the oracle's ranks beside them.
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

METRIC = "EOD-ABE matrices/s + HBM GB/s at fixed rel. error, plain FP32 vs BF16/batched"
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_workload(name: str):
    import workloads as W
    if name == "image4096":
        return W.image(0, 4096, 0.05), 1e-3, 32, "f32", dict(noise_std=0.05)
    if name == "image4096_n05":
        return W.image(0, 4096, 0.5), 1e-3, 32, "f32", dict(noise_std=0.5)
    if name == "hsi262144":
        return W.hyperspectral(0), 1e-2, 16, "f32", dict(noise_std=1e-3)
    if name == "lowrank512":
        return W.lowrank_haar(0), 1e-8, 32, "f64", dict(noise_std=1e-12)
    raise SystemExit(f"unknown workload {name}")


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/traffic_<workload>.txt), or None when there is none or the
    kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in ("paper_2506_22713_amd/csrc/eodabe_kernels.hpp", "paper_2506_22713_amd/csrc/eodabe_tiles.hpp",
              "paper_2506_22713_amd/csrc/eodabe_mlp.hpp", "paper_2506_22713_amd/csrc/eodabe_apps.hpp",
              "paper_2506_22713_amd/csrc/eodabe.hip"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    fields, kernels = {}, {}
    for line in open(path):
        if line.startswith("#") or ":" not in line:
            continue
        if line.startswith("kernel "):
            name = line.split()[1]
            kernels[name] = float(line.rsplit("bytes", 1)[1])
        else:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_sources_sha256") != h.hexdigest():
        return None
    return kernels.get(kernel)


def cpu_baseline(A64: np.ndarray, tol: float, block: int, budget_s: float):
    """Time the oracle (as it stands) on whole factorizations of the same
    matrix, repeating until about budget_s seconds of CPU work."""
    import oracle.eodabe_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    O.eod_abe(A64[:256, :256], tol, k=block)            # warm the BLAS threads
    times, res = [], None
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        res = O.eod_abe(A64, tol, k=block, q=0, seed=0)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start >= budget_s or len(times) >= 200:
            break
    med = float(np.median(times))
    return dict(value=1.0 / med, unit="matrices/s", cores=int(cores), kind="oracle",
                sample=f"{len(times)} whole factorizations of the same {A64.shape[0]}x{A64.shape[1]} "
                       f"matrix (FP64 NumPy oracle), median {med * 1e3:.1f} ms"), res


def cpu_baseline_tiles(tiles, tol, blocks, budget_s):
    """Oracle (as it stands) on the tiles in order until about budget_s
    seconds of CPU work: matrices/s over the tiles it finished."""
    import oracle.eodabe_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    done, t0 = 0, time.perf_counter()
    for T, b in zip(tiles, blocks):
        O.eod_abe(T.astype(np.float64), tol, k=int(b), q=0, seed=0)
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return dict(value=done / el, unit="matrices/s", cores=int(cores), kind="oracle",
                sample=f"the first {done} of the {len(tiles)} tiles (LPT-independent order), "
                       f"FP64 NumPy oracle, {el:.1f} s")


def run_learned(args):
    """Warm-started factorizations (trained predictor) against the plain loop
    on the same 4096^2 matrices: matrices/s, sketch passes per solve,
    fallback rate, rank agreement and the equal-error check."""
    import torch
    import paper_2506_22713_amd as E
    from paper_2506_22713_amd import predictor as PR
    import workloads as W
    tol, b, n = 1e-4, args.block or 32, 4096
    ranks_in = [96, 160, 224, 288, 352, 416]
    log("generating", len(ranks_in), "matrices")
    mats = []
    for k, r in enumerate(ranks_in):
        sig = W.spectrum_sigma("geom", r, 3.0)
        noise = 1e-7 * float(np.sqrt((sig ** 2).sum()) / n)
        mats.append(W.spectrum_torch(1000 + k, n, n, sig, noise, dtype=torch.float32))
    pred = PR.Predictor.load(os.path.join(ROOT, "paper_2506_22713_amd", "predictor.ckpt"))
    cp, cl = E.Context(block=b, seed=0), E.Context(block=b, seed=0)
    pred.attach(cl, margin=0.1)
    wsp, wsl = cp.workspace(n, n, n), cl.workspace(n, n, n)
    out_p = [E.alloc_outputs(A, n) for A in mats]
    out_l = [E.alloc_outputs(A, n) for A in mats]

    def run(ctx, ws, outs, steps, record=False):
        res = []
        for _ in range(steps):
            for i, A in enumerate(mats):
                f = E.factor(A, tol, ctx=ctx, ws=ws, out=outs[i])
                if record:
                    res.append((f, ctx.last_prediction()))
        return res
    log("warmup", args.warmup)
    run(cp, wsp, out_p, max(args.warmup, 1))
    run(cl, wsl, out_l, max(args.warmup, 1))
    res = {}
    for name, ctx, ws, outs in (("plain", cp, wsp, out_p), ("learned", cl, wsl, out_l)):
        log("timed", name, args.steps)
        ctx.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = run(ctx, ws, outs, args.steps, record=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        sk = ctx.profile_read(E.PROF_SKETCH)
        ctx.profile(False)
        res[name] = dict(ms_per_step=el * 1e3 / args.steps, passes=sk[1] / (args.steps * len(mats)),
                         sketch_ms=sk[0] / args.steps, last=rec[-len(mats):])
    agree, excess, fb, d0s = 0, 0.0, 0, []
    for (fp, _), (fl, pl), A in zip(res["plain"]["last"], res["learned"]["last"], mats):
        A64 = A.double()
        nA = torch.linalg.norm(A64)
        ep = float(torch.linalg.norm(A64 - fp.U.double() @ fp.D.double() @ fp.Vt.double()) / nA)
        el = float(torch.linalg.norm(A64 - fl.U.double() @ fl.D.double() @ fl.Vt.double()) / nA)
        agree += int(fp.rank == fl.rank)
        excess = max(excess, el - ep)
        fb += int(pl[3] == 2)
        d0s.append(int(pl[0]))
    ms_l, ms_p = res["learned"]["ms_per_step"], res["plain"]["ms_per_step"]
    line = {
        "metric": METRIC,
        "value": round(len(mats) * 1e3 / ms_l, 2),
        "unit": "matrices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_l, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": dict(workload="learned4096", m=n, n=n, tol=tol, block=b, matrices=len(mats),
                       content_ranks=ranks_in, ranks=[int(f.rank) for f, _ in res["learned"]["last"]],
                       predicted_d0=d0s, fallback_rate=fb / len(mats),
                       sketch_passes_per_solve=dict(learned=res["learned"]["passes"], plain=res["plain"]["passes"]),
                       plain=dict(ms_per_step=round(ms_p, 4), matrices_per_s=round(len(mats) * 1e3 / ms_p, 2)),
                       speedup_vs_plain=round(ms_p / ms_l, 4), rank_agree=agree, max_relerr_excess=excess,
                       sketch_ms_per_step=dict(learned=round(res["learned"]["sketch_ms"], 4),
                                               plain=round(res["plain"]["sketch_ms"], 4))),
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def run_tiles(args):
    """Batched persistent launch over 1024 uneven tiles against 1024
    sequential single-matrix calls on the same tiles (same seed, tol and
    block width per tile)."""
    import torch
    import paper_2506_22713_amd as E
    import workloads as W
    tol, seed = 1e-4, 0
    log("generating 1024 tiles")
    tiles = W.tiles(0, count=1024)
    dev = [torch.from_numpy(np.ascontiguousarray(T)).cuda() for T in tiles]
    ctx = E.Context(block=args.block or 32, seed=seed)
    bt = E.Batch(ctx, dev)
    torch.cuda.synchronize()
    chosen = None
    if not args.no_tune:
        log("autotune")
        chosen = [int(x) for x in bt.tune(tol)]
    log("warmup", args.warmup)
    for _ in range(args.warmup):
        bt.run(tol)
    log("timed", args.steps)
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bt.run(tol)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    tot_ms, launches, by = ctx.profile_read(E.PROF_TILES)
    ctx.profile(False)
    ranks_b, status_b, blocks = bt.ranks.copy(), bt.status.copy(), bt.blocks.copy()
    if args.copy_calib:
        # one plain device copy of 64 MiB: its FETCH_SIZE / WRITE_SIZE under
        # rocprofv3 --pmc calibrate the counters of k_tiles
        src = torch.ones(16 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {src.numel() * 4} bytes read and written")
        del src, dst
    if args.skip_sequential:
        # counter runs only: the batched launches without the sequential comparison
        log(f"batched only: {ms_per_step:.3f} ms per batch; sequential comparison skipped")
        return

    # sequential plain calls, one context per block width in use
    log("sequential plain calls")
    ctxs = {int(b): E.Context(block=int(b), seed=seed) for b in set(blocks.tolist())}
    wss = {}
    for b, c in ctxs.items():
        need = max(c.workspace_size(A.shape[0], A.shape[1], min(A.shape)) for A in dev)
        wss[b] = torch.empty(need, dtype=torch.uint8, device="cuda")
    outs = [E.alloc_outputs(A, min(A.shape)) for A in dev]
    seq = [None] * len(dev)
    for t, A in enumerate(dev):                          # warm every path once
        b = int(blocks[t])
        seq[t] = E.factor(A, tol, ctx=ctxs[b], ws=wss[b], out=outs[t])
    passes = 2
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(passes):
        for t, A in enumerate(dev):
            b = int(blocks[t])
            seq[t] = E.factor(A, tol, ctx=ctxs[b], ws=wss[b], out=outs[t])
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1e3 / passes

    # equal-error check (same tiles, seed, tol and block width)
    log("errors")
    agree, excess, e_b_all, e_s_all = 0, 0.0, [], []
    for t, A in enumerate(dev):
        A64 = A.double()
        nA = torch.linalg.norm(A64)
        U, D, Vt, r, st = bt.result(t)
        eb = float(torch.linalg.norm(A64 - U.double() @ D.double() @ Vt.double()) / nA)
        f = seq[t]
        es = float(torch.linalg.norm(A64 - f.U.double() @ f.D.double() @ f.Vt.double()) / nA)
        agree += int(r == f.rank)
        excess = max(excess, eb - es)
        e_b_all.append(eb)
        e_s_all.append(es)

    avg_ms = tot_ms / max(launches, 1)
    per_launch = by / max(launches, 1)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    # the committed counters were taken with block 32 for every tile: they
    # describe this launch only when the autotuner is off
    traffic = measured_traffic("tiles1024", "k_tiles") if args.no_tune else None
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=round(achieved / PEAK_HBM_GBS, 4), traffic=None if traffic is None else int(traffic),
                    kernel="persistent tile kernel (k_tiles, with its descriptor/result copies)",
                    avg_us=round(avg_ms * 1e3, 2), launches=int(launches), bytes_per_launch=int(per_launch))
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline_tiles(tiles, tol, blocks, args.cpu_budget)
    elems = int(sum(T.size for T in tiles))
    hist = np.bincount(np.minimum(ranks_b // 16, 8), minlength=9).tolist()
    line = {
        "metric": METRIC,
        "value": round(len(tiles) * 1e3 / ms_per_step, 1),
        "unit": "matrices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": dict(workload="tiles1024", tiles=len(tiles), elements=elems, tol=tol, sides="U[64,1024]",
                       content_rank="U[5,80]", noise_std=1e-4, block_default=args.block or 32,
                       tuned_blocks=chosen, blocks_per_tile_mean=float(np.mean(bt.blocks)),
                       rank_hist_by16=hist, status_counts=np.bincount(status_b.clip(0), minlength=4).tolist(),
                       sequential=dict(ms_per_pass=round(ms_seq, 3),
                                       matrices_per_s=round(len(tiles) * 1e3 / ms_seq, 1)),
                       speedup_vs_sequential=round(ms_seq / ms_per_step, 2),
                       rank_agree=agree, max_relerr_excess=excess,
                       relerr_mean=float(np.mean(e_b_all)), relerr_seq_mean=float(np.mean(e_s_all))),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def host_cpu():
    """Host cores and CPU model (for the CPU baselines)."""
    model = "unknown"
    try:
        for l in open("/proc/cpuinfo"):
            if l.startswith("model name"):
                model = l.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(nproc=os.cpu_count(), model=model)


def algorithmic_work(m, n, r, J, b, s):
    """Bytes and flops one solve must move / perform (q = 0): J passes over
    A for the sketches and one for C = Q^T A, the basis traffic of the
    block re-orthogonalisation and the outputs; flops of the sketches, the
    projection, the BCGS2 and CholeskyQR2 products and the closing."""
    by = (J + 1) * m * n * s + 2 * m * r * r * 4 / b + 6 * (m + n) * r * 4
    fl = 2 * m * n * J * b + 2 * m * n * r + 4 * m * b * b * J * (J - 1) + 6 * m * b * b * J + 6 * n * r * r + 2 * m * r * r
    return by, fl


def solve_stats(E, torch, A, tol, ctx, steps, warmup=1):
    """Time whole factorizations of one resident matrix; rank, blocks,
    relative error (FP64 on the device) and ms per solve."""
    m, n = A.shape
    rc = min(m, n)
    ws = ctx.workspace(m, n, rc)
    out = E.alloc_outputs(A, rc)
    for _ in range(warmup):
        f = E.factor(A, tol, ctx=ctx, ws=ws, out=out)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        f = E.factor(A, tol, ctx=ctx, ws=ws, out=out)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    A64 = A.double()
    rel = float(torch.linalg.norm(A64 - f.U.double() @ f.D.double() @ f.Vt.double()) / torch.linalg.norm(A64))
    del ws, out
    return dict(rank=int(f.rank), blocks=int(f.blocks), ms_per_solve=round(ms, 4), relerr=rel,
                flags=int(f.flags))


def timed_calls(torch, fn, steps):
    """(ms per call, last result) of `steps` calls after one warm-up call,
    bracketed by device synchronisations."""
    res = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, res


def subresults(args, E, torch):
    """The other configurations of the benchmark set, each measured briefly
    on the GPU after the headline.  Returns the results and the list of
    (result dict, FP64 host matrix, tol, block) whose oracle rank the
    cpu_baseline leg adds where the oracle finishes in seconds."""
    import workloads as W
    out, checks = {}, []
    t_all = time.perf_counter()

    log("sub: 4096^2 rank sweep")
    sweep = []
    for k, r in enumerate([96, 160, 288, 416]):
        sig = W.spectrum_sigma("geom", r, 3.0)
        noise = 1e-7 * float(np.sqrt((sig ** 2).sum()) / 4096)
        A = W.spectrum_torch(1000 + k, 4096, 4096, sig, noise, dtype=torch.float32)
        st = solve_stats(E, torch, A, 1e-4, E.Context(block=32, seed=0), steps=5)
        st["content_rank"] = r
        if r <= 160:
            checks.append((st, A.double().cpu().numpy(), 1e-4, 32, False))
        by, fl = algorithmic_work(4096, 4096, st["rank"], st["blocks"], 32, 4)
        st["tflops"] = round(fl / (st["ms_per_solve"] * 1e-3) / 1e12, 3)
        st["hbm_frac_end_to_end"] = round(by / (st["ms_per_solve"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
        sweep.append(st)
        del A
    out["rank_sweep_4096_tol1e-4"] = sweep

    log("sub: hyperspectral 262144 x 200")
    H = W.hyperspectral(0)
    Ht = torch.from_numpy(H).cuda()
    hs = {}
    for name, code in (("fp32", E.SKETCH_NATIVE), ("fp16_form", E.SKETCH_F16)):
        ctx = E.Context(block=16, seed=0, sketch=code)
        st = solve_stats(E, torch, Ht, 1e-2, ctx, steps=50)
        ctx.profile(True)                     # the sketch rate, from its own short run:
        solve_stats(E, torch, Ht, 1e-2, ctx, steps=5, warmup=0)   # events between kernels slow the solve
        tot, n_l, by = ctx.profile_read(E.PROF_SKETCH)
        ctx.profile(False)
        if n_l:
            st["sketch_GBs"] = round(by / (tot * 1e-3) / 1e9, 1)
            st["sketch_hbm_frac"] = round(by / (tot * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
        hs[name] = st
    checks.append((hs, H.astype(np.float64), 1e-2, 16, True))
    out["hsi262144_tol1e-2"] = hs
    del Ht

    log("sub: image 4096^2 as written (noise std 0.5)")
    A = torch.from_numpy(W.image(0, 4096, 0.5)).cuda()
    st = solve_stats(E, torch, A, 1e-3, E.Context(block=32, seed=0), steps=1)
    st["note"] = "rank ~ 0.75 n: the noise floor exceeds tol (oracle not run: minutes on the host)"
    out["image4096_n05_tol1e-3"] = st
    del A

    log("sub: lowrank 512^2 FP64")
    L = W.lowrank_haar(0)
    st = solve_stats(E, torch, torch.from_numpy(L).cuda(), 1e-8, E.Context(block=32, seed=0, dtype=torch.float64),
                     steps=20)
    checks.append((st, L, 1e-8, 32, True))
    out["lowrank512_fp64_tol1e-8"] = st

    log("sub: colour images (one factorization per channel, fused reconstruction and criteria)")
    for h in (1024, 4096):
        img = torch.from_numpy(W.rgb_image(0, h, h, noise_std=0.05)).cuda()
        ctx = E.Context(block=32, seed=0)
        ms, ci = timed_calls(torch, lambda: E.compress_image(img, 1e-3, ctx), 3 if h > 1024 else 10)
        inf = ci.info
        out[f"rgb{h}_tol1e-3"] = dict(ms_per_image=round(ms, 4), megapixels_per_s=round(h * h / (ms * 1e3), 1),
                                      ranks=[int(inf.rank[c]) for c in range(3)], relerr=inf.relerr,
                                      psnr=round(inf.psnr, 3), ssim=round(inf.ssim, 6),
                                      reduction=round(inf.reduction, 4))
        del img, ci

    log("sub: complex input")
    for name, cdt in (("complex64", torch.complex64), ("complex128", torch.complex128)):
        Ac = torch.from_numpy(W.lowrank_complex(0, m=2048, n=2048, r=40, noise_std=1e-9, decades=2.0)).to(
            device="cuda", dtype=cdt)
        rdt = torch.float32 if cdt == torch.complex64 else torch.float64
        ctx = E.Context(block=16, seed=0, dtype=rdt)
        ms, fc = timed_calls(torch, lambda: E.factor_complex(Ac, 1e-4, ctx), 10)
        A64 = Ac.to(torch.complex128)
        rel = float(torch.linalg.norm(A64 - fc.U.to(torch.complex128) @ fc.D.to(torch.complex128)
                                      @ fc.Vt.to(torch.complex128)) / torch.linalg.norm(A64))
        out[f"{name}_2048_r40_tol1e-4"] = dict(ms_per_solve=round(ms, 4), rank=int(fc.rank), blocks=int(fc.blocks),
                                               relerr=rel)
        del Ac, A64, fc

    log("sub: hyperspectral features and 10-fold KNN (21025 pixels)")
    Hl, lab, fold = W.hyperspectral_labelled(0)
    Hd = torch.from_numpy(Hl).cuda()
    labd, foldd = torch.from_numpy(lab).cuda(), torch.from_numpy(fold).cuda()
    fh = E.factor(Hd, 1e-2, block=16, seed=0)
    F = E.features(fh).contiguous()
    ms_knn, res = timed_calls(torch, lambda: E.knn_cv(F, labd, foldd, 5, 15), 5)
    out["hsi21025_knn5_tol1e-2"] = dict(features=int(fh.rank), ms_knn=round(ms_knn, 3), oa=res[2],
                                        pairs_per_s=round(21025 * 21025 / (ms_knn * 1e-3), 1))
    del Hd, labd, foldd, F, fh

    log("sub: 1024 tiles, batched vs sequential")
    tiles = W.tiles(0, count=1024)
    dev = [torch.from_numpy(np.ascontiguousarray(T)).cuda() for T in tiles]
    ctx = E.Context(block=32, seed=0)
    bt = E.Batch(ctx, dev)
    bt.run(1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        bt.run(1e-4)
    torch.cuda.synchronize()
    ms_b = (time.perf_counter() - t0) * 1e3 / 3
    ranks_b = bt.ranks.copy()
    ws = torch.empty(max(ctx.workspace_size(A.shape[0], A.shape[1], min(A.shape)) for A in dev),
                     dtype=torch.uint8, device="cuda")
    outs = [E.alloc_outputs(A, min(A.shape)) for A in dev]
    fs = [E.factor(A, 1e-4, ctx=ctx, ws=ws, out=o) for A, o in zip(dev, outs)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fs = [E.factor(A, 1e-4, ctx=ctx, ws=ws, out=o) for A, o in zip(dev, outs)]
    torch.cuda.synchronize()
    ms_s = (time.perf_counter() - t0) * 1e3
    out["tiles1024_tol1e-4"] = dict(batched_ms=round(ms_b, 3), batched_matrices_per_s=round(1024e3 / ms_b, 1),
                                    sequential_ms=round(ms_s, 2), sequential_matrices_per_s=round(1024e3 / ms_s, 1),
                                    speedup=round(ms_s / ms_b, 2),
                                    rank_agree=int(sum(int(f.rank) == int(r) for f, r in zip(fs, ranks_b))))
    del dev, bt, ws, outs, fs
    out["seconds"] = round(time.perf_counter() - t_all, 1)
    return out, checks


def cpu_baseline_oracle_checks(checks):
    """Part of the cpu_baseline leg: the oracle's rank (and RelErr) on the
    sub-configurations' matrices, written beside the GPU's results."""
    import oracle.eodabe_oracle as O
    for st, A64, tol, k, want_err in checks:
        ref = O.eod_abe(A64, tol, k=k, seed=0)
        st["oracle_rank"] = int(ref.rank)
        if want_err:
            st["oracle_relerr"] = float(O.rel_err(A64, ref.U, ref.D, ref.V))


def cpu_baseline_one_thread(A64, tol, block, budget_s):
    """The oracle with its BLAS limited to one thread, on the same matrix."""
    import oracle.eodabe_oracle as O
    try:
        from threadpoolctl import threadpool_limits
    except Exception:
        return None
    times = []
    with threadpool_limits(limits=1):
        t_start = time.perf_counter()
        while True:
            t0 = time.perf_counter()
            O.eod_abe(A64, tol, k=block, q=0, seed=0)
            times.append(time.perf_counter() - t0)
            if time.perf_counter() - t_start >= budget_s or len(times) >= 50:
                break
    med = float(np.median(times))
    return dict(value=1.0 / med, unit="matrices/s", cores=1, kind="oracle",
                sample=f"{len(times)} whole factorizations, one BLAS thread, median {med * 1e3:.1f} ms")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 300 for one matrix per step, 50 for tiles1024 and learned4096)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default 20 for one matrix per step, 5 for tiles1024 and learned4096)")
    ap.add_argument("--workload", default="image4096")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sketch", default="native", choices=["native", "f16", "bf16"],
                    help="precision of the sketches after the second block (FP32 data only)")
    ap.add_argument("--block", type=int, default=0, help="block width b (0: the workload's default)")
    ap.add_argument("--no-tune", action="store_true", help="tiles1024: skip the block-width autotuner")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one plain device copy of A (64 MiB for tiles1024; counter calibration under a profiler)")
    ap.add_argument("--no-subresults", action="store_true",
                    help="headline only (no other configurations; for profiler runs)")
    ap.add_argument("--skip-sequential", action="store_true",
                    help="tiles1024 under a counter profiler: time the batched launches only, print no JSON line")
    args = ap.parse_args()
    many = args.workload in ("tiles1024", "learned4096")      # steps of many matrices each
    if args.steps is None:
        args.steps = 50 if many else 300
    if args.warmup is None:
        args.warmup = 5 if many else 20
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the EOD-ABE library here runs on a single GPU", file=sys.stderr)
        sys.exit(2)

    if args.workload == "tiles1024":
        run_tiles(args)
        return
    if args.workload == "learned4096":
        run_learned(args)
        return

    import torch
    import paper_2506_22713_amd as E

    log("generating", args.workload)
    A_np, tol, block, dt, extra = make_workload(args.workload)
    if args.block:
        block = args.block
    sketch_code = {"native": E.SKETCH_NATIVE, "f16": E.SKETCH_F16, "bf16": E.SKETCH_BF16}[args.sketch]
    tdt = torch.float32 if dt == "f32" else torch.float64
    m, n = A_np.shape
    A = torch.from_numpy(np.ascontiguousarray(A_np)).to(device="cuda", dtype=tdt)
    ctx = E.Context(block=block, seed=0, dtype=tdt, sketch=sketch_code)
    rc = min(m, n)
    ws = ctx.workspace(m, n, rc)
    out = E.alloc_outputs(A, rc)
    torch.cuda.synchronize()

    log("warmup", args.warmup)
    for _ in range(args.warmup):
        f = E.factor(A, tol, ctx=ctx, ws=ws, out=out)
    torch.cuda.synchronize()

    log("timed", args.steps)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    ranks = []
    for _ in range(args.steps):
        f = E.factor(A, tol, ctx=ctx, ws=ws, out=out)
        ranks.append(f.rank)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    ms_wall = wall * 1e3 / args.steps
    # Kernel durations: the same K steps again with HIP events riding on the
    # sketch and projection dispatches.  Those events cost about 9 us per
    # timed launch, so the throughput above comes from the steps without them.
    log("timed with kernel events", args.steps)
    ctx.profile(True)
    ev2, ev3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev2.record(stream)
    for _ in range(args.steps):
        f = E.factor(A, tol, ctx=ctx, ws=ws, out=out)
        ranks.append(f.rank)
    ev3.record(stream)
    torch.cuda.synchronize()
    ms_per_step_ev = ev2.elapsed_time(ev3) / args.steps
    prof = {k: ctx.profile_read(k) for k in (E.PROF_SKETCH, E.PROF_PROJECT)}
    ctx.profile(False)
    if args.copy_calib:
        # one copy of exactly A's bytes: its FETCH_SIZE / WRITE_SIZE under
        # rocprofv3 --pmc calibrate the counters of the factorization kernels
        dst = torch.empty_like(A)
        dst.copy_(A)
        torch.cuda.synchronize()
        log(f"copy calibration: {A.numel() * A.element_size()} bytes read and written")
        del dst

    # correctness of the timed result (the same call each step)
    A64 = A.double()
    rel = float(torch.linalg.norm(A64 - f.U.double() @ f.D.double() @ f.Vt.double()) /
                torch.linalg.norm(A64))
    log(f"rank {f.rank} blocks {f.blocks} relerr {rel:.4e} ms/step {ms_per_step:.3f} (wall {ms_wall:.3f})")

    # roofline of the dominant pass over A (the larger accumulated time of
    # the sketch and the projection, the HBM-bound streaming kernels); the
    # latency-bound small kernels are reported end to end below
    # the sketch runs as k_sketch_rows (16-row tiles, no partials) when the
    # matrix has >= 4081 rows, its sketch would be split along K and b <= 32;
    # otherwise as k_sketch (K-split partials, folded by k_fold_parts)
    sk_rows = 4081 <= max(m, n) <= 32768 and min(m, n) >= 512 and block <= 32 and args.sketch == "native"
    names = {E.PROF_SKETCH: "sketch Y = A*Omega_j (%s)" % ("k_sketch_rows" if sk_rows else "k_sketch"),
             E.PROF_PROJECT: "projection C = Q^T A (k_gemm_nn)"}
    kernel_id = {E.PROF_SKETCH: "k_sketch_rows" if sk_rows else "k_sketch", E.PROF_PROJECT: "k_gemm_nn"}
    kind = max(prof, key=lambda k: prof[k][0])
    tot_ms, launches, by = prof[kind]
    avg_ms = tot_ms / max(launches, 1)
    per_launch_bytes = by / max(launches, 1)
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic = measured_traffic(args.workload, kernel_id[kind])
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=round(achieved / PEAK_HBM_GBS, 4),
                    traffic=None if traffic is None else int(traffic),
                    kernel=names[kind], avg_us=round(avg_ms * 1e3, 2), launches=int(launches),
                    bytes_per_launch=int(per_launch_bytes))
    others = {names[k]: dict(avg_us=round(prof[k][0] / max(prof[k][1], 1) * 1e3, 2),
                             launches=int(prof[k][1]),
                             GBs=round(prof[k][2] / max(prof[k][0], 1e-12) / 1e6, 1))
              for k in prof}

    roofline["scope"] = "dominant pass over A (sketch or projection)"
    s_el = 4 if dt == "f32" else 8
    by_e2e, fl_e2e = algorithmic_work(m, n, int(f.rank), int(f.blocks), block, s_el)
    peak_fl = PEAK_FP32_TFLOPS if dt == "f32" else 78.6
    end_to_end = dict(bytes=int(by_e2e), flops=int(fl_e2e),
                      achieved_GBs=round(by_e2e / (ms_per_step * 1e-3) / 1e9, 1),
                      hbm_frac=round(by_e2e / (ms_per_step * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                      tflops=round(fl_e2e / (ms_per_step * 1e-3) / 1e12, 3),
                      mfma_frac=round(fl_e2e / (ms_per_step * 1e-3) / 1e12 / peak_fl, 4),
                      roofline_frac=round(max(by_e2e / (PEAK_HBM_GBS * 1e9), fl_e2e / (peak_fl * 1e12))
                                          / (ms_per_step * 1e-3), 4))

    subs, checks = None, []
    if not args.no_subresults and args.workload == "image4096" and args.sketch == "native" and not args.block:
        subs, checks = subresults(args, E, torch)

    cpu = None
    orc = {}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu, res = cpu_baseline(A_np.astype(np.float64), tol, block, args.cpu_budget)
        import oracle.eodabe_oracle as O
        orc = dict(oracle_rank=int(res.rank),
                   oracle_relerr=float(O.rel_err(A_np.astype(np.float64), res.U, res.D, res.V)))
        cpu.update(host_cpu())
        log("cpu baseline, one thread")
        one = cpu_baseline_one_thread(A_np.astype(np.float64), tol, block, min(args.cpu_budget, 10.0))
        if one:
            cpu["one_thread"] = one
        if checks:
            log("cpu baseline leg: oracle ranks of the sub-configurations")
            cpu_baseline_oracle_checks(checks)

    line = {
        "metric": METRIC,
        "value": round(1e3 / ms_per_step, 2),
        "unit": "matrices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt,
        "data": "synthetic",
        "config": dict(workload=args.workload, m=m, n=n, tol=tol, block=block, power_iters=0,
                       sketch=args.sketch,
                       rank=int(f.rank), blocks=int(f.blocks), relerr=rel,
                       ranks_constant=len(set(ranks)) == 1, ms_wall_per_step=round(ms_wall, 4),
                       ms_per_step_with_kernel_events=round(ms_per_step_ev, 4),
                       kernels=others, end_to_end=end_to_end, **extra, **orc,
                       subresults=subs),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
