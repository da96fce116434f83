"""Benchmark of the banded Gaussian-loss hot path on one MI355X.

One step = one pass of the whole fused forward + backward unit over the batch:
  loss_b = log det Q_b - y_b^T Q_b^{-1} y_b + tr(Q_b^{-1} S_b)   (per problem)
  forward: Cholesky, log-determinant, forward solve, subset inverse;
  backward: Algorithm 4, the solve sensitivity, the log-determinant
  sensitivity and Algorithm 2 -> dloss/dQ (stored band), dloss/dy.
Workload (default): 16 Matérn-5/2 state-space precisions (state dimension 3,
so k = 5) on a regular grid of 10^6 inputs each (N = 3e6 rows per problem),
lengthscales 1 + b/16, y ~ N(0, I), S a diagonally dominant symmetric band.

Prints ONE JSON line on stdout; diagnostics go to stderr.
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

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_per_row(k: int, prec: int):
    """Algorithmic bytes per row of each kernel kind (what the kernel must read
    and write from HBM, nothing re-read).  w_b: one band record, w_v: one
    vector entry."""
    wb = 8 * (k + 1) if prec == 0 else 4 * (k + 1) + 8
    wv = 8 if prec == 0 else 4
    return {
        "f1_summary": wb + wv,            # Q, y
        "f1_replay": 2 * wb + 2 * wv,     # Q, y -> L, z
        "f2_summary": wb + wv,            # L, z
        "f2_replay": 2 * wb + 2 * wv,     # L, z -> Sigma, ybar
        "b1_summary": 2 * wb,             # L, S
        "b1_replay": 4 * wb,              # L, Sigma, S -> Lbar
        "b2_summary": 2 * wb + 2 * wv,    # L, Lbar, ybar, z
        "b2_replay": 3 * wb + 2 * wv,     # L, Lbar, ybar, z -> Qbar
        "unit": 11 * wb + 4 * wv,         # the loss unit's algorithmic traffic per row
    }


def make_c3(nbatch: int, n_in: int):
    from paper_1902_10078_amd import inputs
    Qs, ys, Ss = [], [], []
    for b in range(nbatch):
        Q, y, S, _ = inputs.config3_problem(b, n_in=n_in, nbatch=16)
        Qs.append(Q)
        ys.append(y)
        Ss.append(S)
    return Qs, ys, Ss, [5] * nbatch


def cpu_baseline(Qs, ys, Ss, ks, nsample: int):
    """The FP64 oracle, OpenMP across problems, on the first nsample problems."""
    import oracle
    ns = [q.shape[0] for q in Qs[:nsample]]
    Qf = np.concatenate([q.ravel() for q in Qs[:nsample]])
    yf = np.concatenate(ys[:nsample])
    Sf = np.concatenate([s.ravel() for s in Ss[:nsample]])
    t0 = time.perf_counter()
    parts, _, _, info, threads = oracle.gauss_loss_batch(ns, ks[:nsample], Qf, yf, Sf)
    dt = time.perf_counter() - t0
    rows = sum(ns)
    return dict(value=rows / dt, unit="band-rows/s", cores=int(threads), kind="oracle",
                sample=f"{nsample} of the batch's problems ({rows} rows), FP64 C oracle, "
                       f"OpenMP across problems, {dt:.2f} s wall"), parts


def traffic_profile_path(prec: str, nbatch: int, n_in: int) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_matern52_b{nbatch}_nin{n_in}_{prec}.txt")


def measured_traffic(slot: str, args, rows: int):
    """HBM bytes per launch of `slot` from the committed rocprofv3 counter
    summary of this workload, or None when there is none, it covers another
    workload, or the kernels have changed since it was taken."""
    from paper_1902_10078_amd import profsum
    path = traffic_profile_path(args.prec, args.batch, args.n_in)
    tr, meta = profsum.read_traffic(path)
    if slot not in tr or meta.get("source_hash") != profsum.source_hash():
        return None
    if int(meta.get("rows_per_launch", -1)) != rows:
        return None
    return round(tr[slot])


def copy_probe(torch, mib: int):
    """A plain copy of a known number of bytes: the reference reading for the
    HBM byte counters (it reads and writes exactly mib MiB each)."""
    dev = torch.device("cuda", 0)
    nbytes = mib << 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    reps = 5
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps(dict(copy_bytes=nbytes, launches=reps + 1, avg_ms=ms,
                          gbs=2 * nbytes / (ms / 1e3) / 1e9)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", choices=["f64", "mixed"], default="f64")
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--n-in", type=int, default=1_000_000)
    ap.add_argument("--target-chunks", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--kernels-json", default="")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (a known-size kernel "
                         "that calibrates HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        log("bench.py measures one GPU: this build has no multi-GPU path (the batch shards "
            "by whole problems across GPUs with no exchange; see the design notes). Use --gpus 1.")
        sys.exit(2)

    import torch
    if args.copy_probe:
        copy_probe(torch, args.copy_probe)
        return
    from paper_1902_10078_amd import bandops as bo

    prec = bo.F64 if args.prec == "f64" else bo.MIXED
    t0 = time.perf_counter()
    Qs, ys, Ss, ks = make_c3(args.batch, args.n_in)
    log(f"inputs: {len(Qs)} problems x {Qs[0].shape[0]} rows, k=5 ({time.perf_counter() - t0:.1f} s)")
    ns = [q.shape[0] for q in Qs]
    rows = sum(ns)

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    vdt = torch.float64 if prec == bo.F64 else torch.float32

    def upload(arrs, dt):
        return torch.from_numpy(np.concatenate([a.ravel() for a in arrs])).to(dev, dt)

    Qt = upload(Qs, vdt)
    St = upload(Ss, vdt)
    yt = upload(ys, vdt)
    E, N = Qt.numel(), yt.numel()
    bufs = {nm: torch.zeros(E, dtype=vdt, device=dev) for nm in ("L", "Sig", "Lbar", "Qbar")}
    z = torch.zeros(N, dtype=vdt, device=dev)
    ybar = torch.zeros(N, dtype=vdt, device=dev)
    parts = torch.zeros((len(ns), 3), dtype=torch.float64, device=dev)
    info = torch.zeros(len(ns), dtype=torch.int32, device=dev)
    kw = dict(Q=Qt, y=yt, S=St, z=z, x=ybar, parts=parts, info=info, **bufs)
    if prec == bo.MIXED:
        diag = lambda arrs: torch.from_numpy(np.concatenate([a[:, 0] for a in arrs])).to(dev)
        kw.update(Qd=diag(Qs), Sd=diag(Ss),
                  **{nm: torch.zeros(N, dtype=torch.float64, device=dev)
                     for nm in ("Ld", "Sigd", "Lbard", "Qbard")})
    plan = bo.Plan(ns, ks, target_chunks=args.target_chunks, device=dev)
    io = plan.io(**kw)
    log(f"plan: {plan.stats}, workspace {plan.ws.numel() / 2**20:.1f} MiB")

    def step():
        plan.gauss_loss(prec, io)

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    assert int(info.max().item()) == 0, "Cholesky failed on the benchmark inputs"

    use_graph = not args.no_graph
    if use_graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                step()
        torch.cuda.current_stream().wait_stream(s)
        run = g.replay
        run()
        torch.cuda.synchronize()
    else:
        run = step

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    value = rows / (ms / 1e3)
    log(f"timed: {args.steps} steps, {ms:.3f} ms/step, {value:.4e} band-rows/s")

    # per-kernel durations (events on the launch stream, eager run)
    bo.profile_enable(True)
    nprof = 3
    for _ in range(nprof):
        step()
    prof = bo.profile_read()
    bo.profile_enable(False)
    bpr = bytes_per_row(5, prec)
    kern = {}
    for name, (tms, cnt) in prof.items():
        avg = tms / cnt
        entry = dict(avg_ms=avg, launches_per_step=cnt / nprof)
        if name in bpr:
            entry["alg_bytes_per_launch"] = bpr[name] * rows
            entry["gbs"] = bpr[name] * rows / (avg / 1e3) / 1e9
        kern[name] = entry
        log(f"  {name:20s} {avg:8.3f} ms x{cnt / nprof:.0f}"
            + (f"  {entry['gbs']:8.1f} GB/s" if "gbs" in entry else ""))
    dom = max((k_ for k_ in kern if "gbs" in kern[k_]), key=lambda k_: kern[k_]["avg_ms"])
    d = kern[dom]
    roof = dict(bound="hbm", kernel=dom, achieved=round(d["gbs"], 2), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(d["gbs"] / HBM_PEAK_GBS, 4), traffic=measured_traffic(dom, args, rows),
                bytes_per_row=bpr[dom], rows_per_launch=rows)
    unit_gbs = bpr["unit"] * rows / (ms / 1e3) / 1e9
    if args.kernels_json:
        with open(args.kernels_json, "w") as f:
            json.dump(dict(kernels=kern, ms_per_step=ms, rows=rows), f, indent=1)

    # the plain FP64 one-matrix-per-launch form: per-problem plans, host loop, no graph
    vs_plain = None
    if not args.no_plain:
        plains = []
        for p in range(len(ns)):
            pl = bo.Plan([ns[p]], [5], device=dev)
            o, v, sz = plan.boff[p], plan.voff[p], ns[p] * 6
            sl = lambda t, a, b_: t[a:a + b_]
            kw64 = {}
            for nm, t in kw.items():
                if nm in ("parts",):
                    kw64[nm] = t[p]
                elif nm == "info":
                    kw64[nm] = t[p:p + 1]
                elif nm in ("Qd", "Sd", "Ld", "Sigd", "Lbard", "Qbard", "y", "z", "x"):
                    kw64[nm] = sl(t, v, ns[p])
                else:
                    kw64[nm] = sl(t, o, sz)
            plains.append((pl, pl.io(**kw64)))

        def plain_step():
            for pl, pio in plains:
                pl.gauss_loss(prec, pio)

        if prec == bo.F64:
            plain_step()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(max(args.steps // 4, 2)):
                plain_step()
            e1.record()
            torch.cuda.synchronize()
            ms_plain = e0.elapsed_time(e1) / max(args.steps // 4, 2)
            vs_plain = ms_plain / ms
            log(f"plain FP64 one-matrix-per-launch: {ms_plain:.3f} ms/step -> batched is {vs_plain:.2f}x")

    out = {
        "metric": "band-rows/s fwd+bwd (Cholesky+solve+subset-inverse), % HBM roofline, vs FP64 plain",
        "value": value,
        "unit": "band-rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == bo.F64 else "f64 (f32 band storage, f64 diagonals)",
        "data": "synthetic",
        "config": {"workload": f"matern52_ssm_batch{len(ns)}_rows{ns[0]}_k5_gauss_loss_fwd_bwd",
                   "batch": len(ns), "rows_per_problem": ns[0], "k": 5,
                   "storage": args.prec, "graph": use_graph, "chunks": plan.stats["nchunk"]},
        "roofline": roof,
        "unit_hbm_frac": round(unit_gbs / HBM_PEAK_GBS, 4),
        "vs_fp64_plain": vs_plain,
    }
    if not args.no_cpu:
        cb, cparts = cpu_baseline(Qs, ys, Ss, ks, min(args.cpu_sample, len(Qs)))
        gp = parts.cpu().numpy()[: len(cparts)]
        cb["max_rel_diff_loss_parts_vs_gpu"] = float(np.max(np.abs(gp - cparts) / np.abs(cparts)))
        out["cpu_baseline"] = cb
        log(f"cpu baseline: {cb}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
