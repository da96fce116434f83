"""Benchmark of the banded Gaussian-model hot path on one MI355X.

Default workload (the headline): one step = the fused forward + backward loss
unit over a batch,
  loss_b = log det Q_b - y_b^T Q_b^{-1} y_b + tr(Q_b^{-1} S_b)   (per problem)
  forward: Cholesky, log-determinant, forward solve, subset inverse;
  backward: Algorithm 4, the solve sensitivity, the log-determinant
  sensitivity and Algorithm 2 -> dloss/dQ (stored band), dloss/dy,
on 16 Matérn-5/2 state-space precisions (state dimension 3, so k = 5) on a
regular grid of 10^6 inputs each (N = 3e6 rows per problem), lengthscales
1 + b/16, y ~ N(0, I), S a diagonally dominant symmetric band.

Other workloads (--workload):
  uneven_forward   4096 problems, n log-uniform in [256, 65536], k in
                   {1,3,5,11}: the forward list (Cholesky, logdet, L^{-1} y,
                   L^{-T} L^{-1} y, band of Q^{-1}) in one plan, mixed format
                   by default;
  matern32_forward one Matérn-3/2 precision of 1e5 jittered inputs (N = 2e5,
                   k = 3), lengthscale 10: the same forward list, FP64.
  wide_loss        8 wide block-banded problems (n = 2e5, k = 64, Q = D +
                   band(B B^T)): loss = log det Q + tr(Q^{-1} W) forward and
                   backward on 64 x 64 blocks (FP32 MFMA products, FP64 pivots).
  vi_kl            16 KL terms KL(q || p) of Algorithm 7 (n = 1e6, k = 5) with
                   their gradients in L_q, L_p, m_q, m_p;
  solve_band_mat   one matrix solve with a banded right-hand side (Algorithm
                   5; n = 1.6e7, k = 5, R with 2 lower and 5 upper diagonals)
                   and its reverse mode;
  marglik          16 log marginal likelihoods with partial observations
                   (Algorithm 8) on the Matérn-5/2 priors of the loss
                   workload, 80% of the inputs' function values observed,
                   with the gradients in Q, b and tau2;
  natgp_co2        1024 GP regressions in banded natural parameters
                   (Algorithm 10) on CO2-shaped state-space priors (3082
                   weekly inputs, Matérn-3/2 trend + two quasi-periodic
                   harmonics: 18492 rows, k = 11), one per lengthscale
                   setting of a grid, with the gradients in both precisions
                   and the prior natural mean;
  whiten_hmc       one gradient evaluation of a whitened HMC target
                   (Algorithm 6) on the 16 Matérn-5/2 precisions of the loss
                   workload: F = L^{-T} v, then vbar and Qbar from a given
                   Fbar (the likelihood's gradient, synthetic);
  graph_whiten     the same gradient evaluation on graph GMRFs: a 3 x 333334
                   road strip in its reverse Cuthill-McKee order (host,
                   once), 16 edge-precision settings assembled into bands from
                   CSR each step, and the band gradients gathered back to the
                   CSR values.

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
METRIC = "band-rows/s fwd+bwd (Cholesky+solve+subset-inverse), % HBM roofline, vs FP64 plain"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def record_bytes(k: int, prec: int):
    """(w_b, w_v): bytes of one band record and of one vector entry."""
    return (8 * (k + 1), 8) if prec == 0 else (4 * (k + 1) + 8, 4)


def bytes_per_row(k: int, prec: int, forward_only: bool = False):
    """Algorithmic bytes per row of each kernel kind (what the kernel must read
    and write from HBM, nothing re-read).  w_b: one band record, w_v: one
    vector entry."""
    wb, wv = record_bytes(k, prec)
    if forward_only:
        return {
            "f1_summary": wb + wv,            # Q, y
            "f1_replay": 2 * wb + 2 * wv,     # Q, y -> L, z
            "f2_replay": 2 * wb + 2 * wv,     # L, z -> Sigma, x
            "unit": 4 * wb + 4 * wv,          # the forward list's traffic per row
        }
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


def vi_bytes_per_row(k: int, prec: int):
    """Algorithmic bytes per row of the KL term's kernels (Algorithm 7)."""
    wb, wv = record_bytes(k, prec)
    return {"vi_pre": 2 * wb + 8 + 3 * wv,          # L_p, diag L_q, m_q, m_p -> Q_p / 2, v
            "chunk_product": wb,                     # L_q
            "f2_summary": wb,                        # L_q
            "f2_replay": 3 * wb,                     # L_q, Q_p / 2 -> Sigma
            "b1_summary": 2 * wb,                    # L_q, Q_p / 2
            "b1_replay": 4 * wb,                     # L_q, Sigma, Q_p / 2 -> Lqbar
            "vi_post": 3 * wb + 4 * wv,              # L_p, Sigma, m_q, m_p, v -> Lpbar, mpbar
            "vi_neg": 2 * wv,                        # mpbar -> mqbar
            "unit": 5 * wb + 4 * wv}                 # inputs L_q, L_p, m_q, m_p; outputs Sigma and the gradients


def ml_bytes_per_row(k: int, prec: int):
    """Algorithmic bytes per row of the marginal likelihood's kernels
    (Algorithm 8 and its reverse mode): two forward lists (on Q without a
    right-hand side, on Q1 with b) and the row kernels around them."""
    wb, wv = record_bytes(k, prec)
    return {"chunk_product": 0,                      # chunk scans only (written by the F1 replays)
            "f1_summary": 2 * wb + 2 * wv,           # Q; Q, mask, b (Q1 = Q + mask / tau2 as read)
            "f1_replay": 4 * wb + 3 * wv,            # Q -> L_Q; Q, mask, b -> L, z
            "f2_replay": 4 * wb + 2 * wv,            # L_Q -> I(L_Q); L, z -> Sigma, x
            "ml_post": 3 * wb + 4 * wv,              # Sigma, I(L_Q), x, mask, b -> Qbar, bbar
            "unit": 4 * wb + 4 * wv}                 # Q, mask, b in; L, Sigma, x, Qbar, bbar out


def ng_bytes_per_row(k: int, prec: int):
    """Algorithmic bytes per row of the natural-parameter GP regression's
    kernels (Algorithm 10 and its reverse mode): two forward lists with a
    right-hand side each and the row kernels around them."""
    wb, wv = record_bytes(k, prec)
    return {"ng_pre": 3 * wb + 3 * wv,               # Lam_pr, Lam_lik, eta_pr, eta_lik -> Lam_po, eta_po
            "f1_summary": 2 * wb + 2 * wv,           # Lam_pr, eta_pr; Lam_po, eta_po
            "f1_replay": 4 * wb + 4 * wv,            # -> C_pr, z_pr; C_po, z_po
            "f2_summary": 2 * wb + 2 * wv,           # C, z of both lists
            "f2_replay": 4 * wb + 4 * wv,            # C, z -> Sigma, mu of both lists
            "ng_post": 4 * wb + 2 * wv,              # Sigma_po, Sigma_pr, mu_po, mu_pr -> Lprbar, Llikbar
            "ng_neg": 3 * wv,                        # mu_po, mu_pr -> etaprbar
            "unit": 6 * wb + 5 * wv}                 # 2 bands + 2 vectors in; L, Sigma, 2 band grads, x, etaprbar out


def wh_bytes_per_row(k: int, prec: int):
    """Algorithmic bytes per row of the whitened sample and its reverse mode
    (Algorithm 6; Table 1, Algorithm 2): every summary is its own kernel."""
    wb, wv = record_bytes(k, prec)
    return {"f1_summary": wb,                       # Q
            "f1_replay": 2 * wb,                    # Q -> L
            "f2_summary": wb + wv,                  # L, v
            "f2_replay": wb + 2 * wv,               # L, v -> F
            "chunk_product": wb,                    # L (only when the backward does not reuse them)
            "fs_summary": wb + wv,                  # L, Fbar
            "fs_replay": wb + 2 * wv,               # L, Fbar -> vbar
            "b2_summary": wb + 2 * wv,              # L, F, vbar
            "b2_replay": 2 * wb + 2 * wv,           # L, F, vbar -> Qbar
            "unit": 3 * wb + 5 * wv}                # Q, v, Fbar in; L, F, vbar, Qbar out


def alg5_bytes_per_row(k: int, lr: int, u: int):
    """Algorithmic bytes per row of the matrix solve with a banded right-hand
    side (Algorithm 5) and its reverse mode, FP64."""
    wl, wr, wo = 8 * (k + 1), 8 * (lr + u + 1), 8 * (k + u + 1)
    return {"solve_mat": wl + wr + wo,          # L, R -> O
            "solve_mat_g": wl + 2 * wo + wr,    # L, Obar -> G = L^{-T} Obar, Rbar
            "solve_mat_out": 2 * wo + wl,       # G, O -> Lbar
            "unit": wl + wr + 2 * wo + wr + wl}  # L, R, Obar in; O, Rbar, Lbar out


def wide_bytes_per_row():
    """Algorithmic bytes per row of the wide passes' replays (mixed storage,
    k = 64); the chunk summaries re-read inputs and are not counted."""
    wb, _ = record_bytes(64, 1)
    return {"wide_f1": 2 * wb,      # Q -> L
            "wide_f2": 2 * wb,      # W -> Sigma (trace term)
            "wide_b1": 4 * wb,      # L, Sigma, W -> Lbar
            "wide_b2": 3 * wb,      # L, Lbar -> Qbar
            "unit": 11 * wb}


# Algorithmic flops per row of the wide loss unit: 9 k (k + 1) (Cholesky
# k(k+1)/2 multiply-adds, Takahashi k(k+1), Algorithm 4 2k(k+1), Algorithm 2
# k(k+1), two flops each), k = 64.
WIDE_FLOP_PER_ROW = 9 * 64 * 65
FP32_MFMA_PEAK_TFLOPS = 157.3


def batch_bytes(ns, ks, prec, forward_only, vi=False, ml=False, ng=False, wh=False):
    """Algorithmic bytes of one step of each kernel kind over the batch."""
    tot = {}
    for n, k in zip(ns, ks):
        per = (vi_bytes_per_row(k, prec) if vi else ml_bytes_per_row(k, prec) if ml
               else ng_bytes_per_row(k, prec) if ng else wh_bytes_per_row(k, prec) if wh
               else bytes_per_row(k, prec, forward_only))
        for nm, b in per.items():
            tot[nm] = tot.get(nm, 0) + b * n
    return tot


def traffic_profile_path(workload: str, prec: str, nbatch: int, n_in: int) -> str:
    if workload == "matern52_loss":
        return os.path.join(ROOT, "profiles", f"traffic_matern52_b{nbatch}_nin{n_in}_{prec}.txt")
    return os.path.join(ROOT, "profiles", f"traffic_{workload}_{prec}.txt")


def measured_traffic(slot: str, path: str, rows: int):
    """HBM bytes per launch of `slot` from the committed rocprofv3 counter
    summary of this workload, or None when there is none, it covers another
    workload, or the kernels have changed since it was taken."""
    import profsum
    tr, meta = profsum.read_traffic(path)
    if slot not in tr or meta.get("source_hash") != profsum.source_hash(meta.get("hash_sources")):
        return None
    if int(meta.get("rows_per_launch", -1)) != rows:
        return None
    return round(tr[slot])


def copy_gbs(torch, mib: int):
    """Measured rate of a plain device copy of mib MiB (read + write bytes per
    second, GB/s): the bandwidth these streaming kernels can actually reach,
    reported beside the 8 TB/s peak."""
    dev = torch.device("cuda", 0)
    nbytes = mib << 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    reps = 10
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms / 1e3) / 1e9


def host_info(threads_used: int):
    """Host CPU facts for the CPU baseline: logical CPUs the process may run
    on, the OpenMP threads the oracle used, and the CPU model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return dict(cores=int(threads_used), host_cpus_available=avail, host_cpus_total=os.cpu_count(),
                omp_num_threads=os.environ.get("OMP_NUM_THREADS"), cpu_model=model)


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


# ------------------------------------------------------------------ workloads

class Workload:
    """Inputs resident on the device, a plan over the batch, and the step."""

    def __init__(self, bo, torch, dev, ns, ks, prec, host_inputs, forward_only, target_chunks=0, keep=False):
        """keep: the loss unit keeps L, Sigma and Lbar in the plan's workspace
        (interleaved by chunk) instead of writing them to caller arrays."""
        self.bo, self.torch, self.dev = bo, torch, dev
        self.ns, self.ks, self.prec = ns, ks, prec
        self.forward_only = forward_only
        vdt = torch.float64 if prec == bo.F64 else torch.float32
        Qs, ys, Ss = host_inputs

        def upload(arrs, dt):
            return torch.from_numpy(np.concatenate([a.ravel() for a in arrs])).to(dev, dt)

        def diag(arrs):
            return torch.from_numpy(np.concatenate([a[:, 0] for a in arrs])).to(dev)

        Qt, yt = upload(Qs, vdt), upload(ys, vdt)
        E, N = Qt.numel(), yt.numel()
        nprob = len(ns)
        kw = dict(Q=Qt, y=yt, z=torch.zeros(N, dtype=vdt, device=dev), x=torch.zeros(N, dtype=vdt, device=dev),
                  info=torch.zeros(nprob, dtype=torch.int32, device=dev))
        names = ("L", "Sig") if forward_only else (("Qbar",) if keep else ("L", "Sig", "Lbar", "Qbar"))
        if keep:
            del kw["z"]   # an intermediate of the loss unit: kept in the workspace
        for nm in names:
            kw[nm] = torch.zeros(E, dtype=vdt, device=dev)
        if forward_only:
            kw["logdet"] = torch.zeros(nprob, dtype=torch.float64, device=dev)
        else:
            kw["S"] = upload(Ss, vdt)
            kw["parts"] = torch.zeros((nprob, 3), dtype=torch.float64, device=dev)
        if prec == bo.MIXED:
            kw["Qd"] = diag(Qs)
            if not forward_only:
                kw["Sd"] = diag(Ss)
            for nm in names:
                kw[nm + "d"] = torch.zeros(N, dtype=torch.float64, device=dev)
        self.kw = kw
        self.set_schedule(target_chunks)

    def set_schedule(self, target_chunks: int):
        """(Re)build the plan for a target chunk count (0: the library default)."""
        self.plan = self.bo.Plan(self.ns, self.ks, target_chunks=target_chunks, device=self.dev)
        self.io = self.plan.io(**self.kw)

    def step(self):
        if self.forward_only:
            self.plan.forward(self.prec, self.io)
        else:
            self.plan.gauss_loss(self.prec, self.io)

    def plain_steps(self):
        """The plain FP64 form: one plan per matrix, launched from a host loop,
        no graph (on the FP64 inputs)."""
        bo = self.bo
        out = []
        for p in range(len(self.ns)):
            n, k = self.ns[p], self.ks[p]
            pl = bo.Plan([n], [k], device=self.dev)
            o, v, sz = self.plan.boff[p], self.plan.voff[p], n * (k + 1)
            kw = {}
            for nm, t in self.kw.items():
                if nm == "parts":
                    kw[nm] = t[p]
                elif nm in ("info", "logdet"):
                    kw[nm] = t[p:p + 1]
                elif nm in ("y", "z", "x") or nm.endswith("d"):
                    kw[nm] = t[v:v + n]
                else:
                    kw[nm] = t[o:o + sz]
            out.append((pl, pl.io(**kw)))

        def run():
            for pl, pio in out:
                if self.forward_only:
                    pl.forward(bo.F64, pio)
                else:
                    pl.gauss_loss(bo.F64, pio)
        return run


def make_matern52(args):
    from paper_1902_10078_amd import inputs
    Qs, ys, Ss = [], [], []
    for b in range(args.batch):
        Q, y, S, _ = inputs.config3_problem(b, n_in=args.n_in, nbatch=16)
        Qs.append(Q)
        ys.append(y)
        Ss.append(S)
    return [q.shape[0] for q in Qs], [5] * args.batch, (Qs, ys, Ss)


def make_uneven(args, bo, torch, dev):
    """The uneven batch; Q_b = band(L_b L_b^T) is formed on the device with
    the library's banded product (input construction, untimed)."""
    from paper_1902_10078_amd import inputs
    ns, ks = inputs.config2_shapes(nprob=args.nprob)
    ns, ks = [int(v) for v in ns], [int(v) for v in ks]
    Ls, ys = inputs.config2_factors(2, ns, ks)
    Qs = []
    for L, k in zip(Ls, ks):
        Lb = bo.band_from(torch.from_numpy(L).to(dev), k)
        Qs.append(bo.bo_gbmm(Lb, Lb, 0, 1, k, 0).band.cpu().numpy())
    return ns, ks, (Qs, ys, None)


def make_matern32(args):
    from paper_1902_10078_amd import inputs
    Q, y, _, _ = inputs.config1_inputs(seed=1, n_in=args.n_in32, ell=args.ell)
    return [Q.shape[0]], [3], ([Q], [y], None)


class VIWorkload:
    """The KL term of the variational objective over a batch (inputs resident
    on the device): L_q, L_p, m_q, m_p in, I(L_q), the four gradients and the
    parts out."""

    def __init__(self, bo, torch, dev, ns, ks, prec, host_inputs, target_chunks=0):
        self.bo, self.torch, self.dev = bo, torch, dev
        self.ns, self.ks, self.prec = ns, ks, prec
        Lqs, Lps, mqs, mps = host_inputs
        vdt = torch.float64 if prec == bo.F64 else torch.float32
        up = lambda arrs: torch.from_numpy(np.concatenate([a.ravel() for a in arrs])).to(dev, vdt)
        diag = lambda arrs: torch.from_numpy(np.concatenate([a[:, 0] for a in arrs])).to(dev)
        kw = dict(Lq=up(Lqs), Lp=up(Lps), mq=up(mqs), mp=up(mps))
        E, N = kw["Lq"].numel(), kw["mq"].numel()
        for nm in ("Sig", "Lqbar", "Lpbar"):
            kw[nm] = torch.zeros(E, dtype=vdt, device=dev)
        for nm in ("mqbar", "mpbar"):
            kw[nm] = torch.zeros(N, dtype=vdt, device=dev)
        kw["parts"] = torch.zeros((len(ns), 4), dtype=torch.float64, device=dev)
        if prec == bo.MIXED:
            kw["Lqd"], kw["Lpd"] = diag(Lqs), diag(Lps)
            for nm in ("Sigd", "Lqbard", "Lpbard"):
                kw[nm] = torch.zeros(N, dtype=torch.float64, device=dev)
        self.kw = kw
        self.set_schedule(target_chunks)

    def set_schedule(self, target_chunks: int):
        self.plan = self.bo.Plan(self.ns, self.ks, target_chunks=target_chunks, device=self.dev)
        self.io = self.plan.kl_io(**self.kw)

    def step(self):
        self.plan.vi_kl(self.prec, self.io)

    def plain_steps(self):
        """The plain FP64 form: one plan per matrix, host loop, no graph."""
        bo = self.bo
        out = []
        for p in range(len(self.ns)):
            n, k = self.ns[p], self.ks[p]
            pl = bo.Plan([n], [k], device=self.dev)
            o, v, sz = self.plan.boff[p], self.plan.voff[p], n * (k + 1)
            kw = {}
            for nm, t in self.kw.items():
                if nm == "parts":
                    kw[nm] = t[p]
                elif nm in ("mq", "mp", "mqbar", "mpbar") or nm.endswith("d"):
                    kw[nm] = t[v:v + n]
                else:
                    kw[nm] = t[o:o + sz]
            out.append((pl, pl.kl_io(**kw)))

        def run():
            for pl, pio in out:
                pl.vi_kl(bo.F64, pio)
        return run


def make_vi(args):
    """L_q, L_p lower bands (diagonal U[1,2], off-diagonal N(0, 0.3^2)) and
    normal means: the variational and prior factors of Algorithm 7."""
    from paper_1902_10078_amd import inputs
    Lqs, Lps, mqs, mps = [], [], [], []
    for b in range(args.batch):
        rng = np.random.default_rng(7000 + b)
        Lqs.append(inputs.random_lower_band(args.n_vi, 5, rng))
        Lps.append(inputs.random_lower_band(args.n_vi, 5, rng))
        mqs.append(rng.normal(size=args.n_vi))
        mps.append(rng.normal(size=args.n_vi))
    return [args.n_vi] * args.batch, [5] * args.batch, (Lqs, Lps, mqs, mps)


class MLWorkload:
    """The log marginal likelihood with partial observations over a batch
    (inputs resident on the device): Q, mask, b, tau2 in; L, Sigma, x, Qbar,
    bbar, tau2bar, the parts and info out."""

    def __init__(self, bo, torch, dev, ns, ks, prec, host_inputs, target_chunks=0):
        self.bo, self.torch, self.dev = bo, torch, dev
        self.ns, self.ks, self.prec = ns, ks, prec
        Qs, masks, bs, tau2 = host_inputs
        vdt = torch.float64 if prec == bo.F64 else torch.float32
        up = lambda arrs: torch.from_numpy(np.concatenate([a.ravel() for a in arrs])).to(dev, vdt)
        kw = dict(Q=up(Qs), mask=up(masks), b=up(bs),
                  tau2=torch.tensor(np.asarray(tau2, dtype=np.float64), device=dev))
        E, N, P = kw["Q"].numel(), kw["b"].numel(), len(ns)
        for nm in ("L", "Sig", "Qbar"):
            kw[nm] = torch.zeros(E, dtype=vdt, device=dev)
        for nm in ("x", "bbar"):
            kw[nm] = torch.zeros(N, dtype=vdt, device=dev)
        kw["tau2bar"] = torch.zeros(P, dtype=torch.float64, device=dev)
        kw["parts"] = torch.zeros((P, 4), dtype=torch.float64, device=dev)
        kw["info"] = torch.zeros(P, dtype=torch.int32, device=dev)
        if prec == bo.MIXED:
            kw["Qd"] = torch.from_numpy(np.concatenate([a[:, 0] for a in Qs])).to(dev)
            for nm in ("Ld", "Sigd", "Qbard"):
                kw[nm] = torch.zeros(N, dtype=torch.float64, device=dev)
        self.kw = kw
        self.set_schedule(target_chunks)

    def set_schedule(self, target_chunks: int):
        self.plan = self.bo.Plan(self.ns, self.ks, target_chunks=target_chunks, device=self.dev)
        self.io = self.plan.ml_io(**self.kw)

    def step(self):
        self.plan.marglik(self.prec, self.io)

    def plain_steps(self):
        """The plain FP64 form: one plan per matrix, host loop, no graph."""
        bo = self.bo
        out = []
        for p in range(len(self.ns)):
            n, k = self.ns[p], self.ks[p]
            pl = bo.Plan([n], [k], device=self.dev)
            o, v, sz = self.plan.boff[p], self.plan.voff[p], n * (k + 1)
            kw = {}
            for nm, t in self.kw.items():
                if nm in ("parts", "tau2", "tau2bar", "info"):
                    kw[nm] = t[p:p + 1]
                elif nm in ("mask", "b", "x", "bbar") or nm.endswith("d"):
                    kw[nm] = t[v:v + n]
                else:
                    kw[nm] = t[o:o + sz]
            out.append((pl, pl.ml_io(**kw)))

        def run():
            for pl, pio in out:
                pl.marglik(bo.F64, pio)
        return run


def make_ml(args):
    """The Matérn-5/2 prior precisions of the loss workload with each input's
    function value observed with probability 0.8, noise variance 0.1."""
    from paper_1902_10078_amd import inputs
    Qs, masks, bs, t2 = [], [], [], []
    for b in range(args.batch):
        Q, mask, y, tau2 = inputs.config5_marglik(b, n_in=args.n_in, nbatch=16)
        Qs.append(Q)
        masks.append(mask)
        bs.append(y)
        t2.append(tau2)
    return [q.shape[0] for q in Qs], [5] * args.batch, (Qs, masks, bs, t2)


class NGWorkload:
    """GP regression with banded natural parameters over a batch (inputs
    resident on the device): Lam_pr, eta_pr, Lam_lik, eta_lik in; L, Sigma, x,
    the three gradients, the parts and info out."""

    def __init__(self, bo, torch, dev, ns, ks, prec, host_inputs, target_chunks=0):
        self.bo, self.torch, self.dev = bo, torch, dev
        self.ns, self.ks, self.prec = ns, ks, prec
        vdt = torch.float64 if prec == bo.F64 else torch.float32
        up = lambda key: torch.from_numpy(np.concatenate([p[key].ravel() for p in host_inputs])).to(dev, vdt)
        kw = dict(Lpr=up("Lam_pr"), etapr=up("eta_pr"), Llik=up("Lam_lik"), etalik=up("eta_lik"))
        E, N, P = kw["Lpr"].numel(), kw["etapr"].numel(), len(ns)
        for nm in ("L", "Sig", "Lprbar", "Llikbar"):
            kw[nm] = torch.zeros(E, dtype=vdt, device=dev)
        for nm in ("x", "etaprbar"):
            kw[nm] = torch.zeros(N, dtype=vdt, device=dev)
        kw["parts"] = torch.zeros((P, 5), dtype=torch.float64, device=dev)
        kw["info"] = torch.zeros(P, dtype=torch.int32, device=dev)
        if prec == bo.MIXED:
            dg = lambda key: torch.from_numpy(np.concatenate([p[key][:, 0] for p in host_inputs])).to(dev)
            kw["Lprd"], kw["Llikd"] = dg("Lam_pr"), dg("Lam_lik")
            for nm in ("Ld", "Sigd", "Lprbard", "Llikbard"):
                kw[nm] = torch.zeros(N, dtype=torch.float64, device=dev)
        self.kw = kw
        self.set_schedule(target_chunks)

    def set_schedule(self, target_chunks: int):
        self.plan = self.bo.Plan(self.ns, self.ks, target_chunks=target_chunks, device=self.dev)
        self.io = self.plan.ng_io(**self.kw)

    def step(self):
        self.plan.natgp(self.prec, self.io)

    def plain_steps(self):
        """The plain FP64 form: one plan per matrix, host loop, no graph."""
        bo = self.bo
        out = []
        for p in range(len(self.ns)):
            n, k = self.ns[p], self.ks[p]
            pl = bo.Plan([n], [k], device=self.dev)
            o, v, sz = self.plan.boff[p], self.plan.voff[p], n * (k + 1)
            kw = {}
            for nm, t in self.kw.items():
                if nm in ("parts", "info"):
                    kw[nm] = t[p:p + 1]
                elif nm in ("etapr", "etalik", "x", "etaprbar") or nm.endswith("d"):
                    kw[nm] = t[v:v + n]
                else:
                    kw[nm] = t[o:o + sz]
            out.append((pl, pl.ng_io(**kw)))

        def run():
            for pl, pio in out:
                pl.natgp(bo.F64, pio)
        return run


def make_ng(args):
    """CO2-shaped regression problems (weekly inputs, 3082 weeks, Matérn-3/2
    trend plus two quasi-periodic harmonics: d = 6, k = 11), one per
    hyper-parameter setting of a grid over the two lengthscales."""
    from paper_1902_10078_amd import inputs
    probs = []
    for b in range(args.nng):
        g = int(round(args.nng ** 0.5))
        ell_s = 1.0 + 2.0 * (b % g) / g
        ell_q = 0.5 + (b // g) / g
        probs.append(inputs.co2_natgp(args.t_ng, seed=600 + b, J=2, ell_s=ell_s, ell_q=ell_q))
    return [p["Lam_pr"].shape[0] for p in probs], [p["k"] for p in probs], probs


class WHWorkload:
    """One gradient evaluation of a whitened HMC target over a batch (inputs
    resident on the device): F = L^{-T} v with L = C(Q), then the reverse mode
    from a given Fbar (the likelihood's gradient, here synthetic)."""

    def __init__(self, bo, torch, dev, ns, ks, prec, host_inputs, target_chunks=0):
        self.bo, self.torch, self.dev = bo, torch, dev
        self.ns, self.ks, self.prec = ns, ks, prec
        Qs, vs, Fbs = host_inputs
        vdt = torch.float64 if prec == bo.F64 else torch.float32
        up = lambda arrs: torch.from_numpy(np.concatenate([a.ravel() for a in arrs])).to(dev, vdt)
        kw = dict(Q=up(Qs), v=up(vs), Fbar=up(Fbs))
        E, N, P = kw["Q"].numel(), kw["v"].numel(), len(ns)
        for nm in ("L", "Qbar"):
            kw[nm] = torch.zeros(E, dtype=vdt, device=dev)
        for nm in ("F", "vbar"):
            kw[nm] = torch.zeros(N, dtype=vdt, device=dev)
        kw["logdet"] = torch.zeros(P, dtype=torch.float64, device=dev)
        kw["info"] = torch.zeros(P, dtype=torch.int32, device=dev)
        if prec == bo.MIXED:
            kw["Qd"] = torch.from_numpy(np.concatenate([a[:, 0] for a in Qs])).to(dev)
            for nm in ("Ld", "Qbard"):
                kw[nm] = torch.zeros(N, dtype=torch.float64, device=dev)
        self.kw = kw
        self.set_schedule(target_chunks)

    def set_schedule(self, target_chunks: int):
        self.plan = self.bo.Plan(self.ns, self.ks, target_chunks=target_chunks, device=self.dev)
        self.io = self.plan.wh_io(reuse=True, **self.kw)   # backward right after forward

    def step(self):
        self.plan.whiten(self.prec, self.io)
        self.plan.whiten_bwd(self.prec, self.io)

    def plain_steps(self):
        """The plain FP64 form: one plan per matrix, host loop, no graph."""
        bo = self.bo
        out = []
        for p in range(len(self.ns)):
            n, k = self.ns[p], self.ks[p]
            pl = bo.Plan([n], [k], device=self.dev)
            o, v, sz = self.plan.boff[p], self.plan.voff[p], n * (k + 1)
            kw = {}
            for nm, t in self.kw.items():
                if nm in ("logdet", "info"):
                    kw[nm] = t[p:p + 1]
                elif nm in ("v", "Fbar", "F", "vbar") or nm.endswith("d"):
                    kw[nm] = t[v:v + n]
                else:
                    kw[nm] = t[o:o + sz]
            out.append((pl, pl.wh_io(**kw)))

        def run():
            for pl, pio in out:
                pl.whiten(bo.F64, pio)
                pl.whiten_bwd(bo.F64, pio)
        return run


def make_wh(args):
    """The Matérn-5/2 precisions of the loss workload with v, Fbar ~ N(0, I)
    (per-problem substreams of seed 8)."""
    from paper_1902_10078_amd import inputs
    Qs, vs, Fbs = [], [], []
    for b in range(args.batch):
        Q, _, _, _ = inputs.config3_problem(b, n_in=args.n_in, nbatch=16)
        rng = np.random.default_rng(np.random.SeedSequence([8, b]))
        Qs.append(Q)
        vs.append(rng.normal(size=Q.shape[0]))
        Fbs.append(rng.normal(size=Q.shape[0]))
    return [q.shape[0] for q in Qs], [5] * args.batch, (Qs, vs, Fbs)


class GraphWorkload:
    """Gradient evaluations of a whitened HMC target on graph GMRFs: one road
    graph in its reverse Cuthill-McKee order (computed once, on the host), one
    precision per lengthscale setting.  A step assembles every band from the
    CSR values, runs the whitened sample and its reverse mode over the batch,
    and gathers the band gradients back to the CSR values."""

    def __init__(self, bo, torch, dev, host_inputs, prec, target_chunks=0):
        self.bo, self.prec = bo, prec
        g = host_inputs
        n, k, nb = g["n"], g["k"], len(g["vals"])
        self.n, self.k, self.nb = n, k, nb
        i64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64)).to(dev)
        self.ip, self.ix = i64(g["pindptr"]), i64(g["pindices"])
        self.vals = torch.from_numpy(np.concatenate([v[g["map"]] for v in g["vals"]])).to(dev)
        vdt = torch.float64 if prec == bo.F64 else torch.float32
        E, N = nb * n * (k + 1), nb * n
        kw = dict(Q=torch.zeros(E, dtype=vdt, device=dev), L=torch.zeros(E, dtype=vdt, device=dev),
                  Qbar=torch.zeros(E, dtype=vdt, device=dev),
                  v=torch.from_numpy(np.concatenate(g["v"])).to(dev, vdt),
                  Fbar=torch.from_numpy(np.concatenate(g["Fbar"])).to(dev, vdt),
                  F=torch.zeros(N, dtype=vdt, device=dev), vbar=torch.zeros(N, dtype=vdt, device=dev),
                  logdet=torch.zeros(nb, dtype=torch.float64, device=dev),
                  info=torch.zeros(nb, dtype=torch.int32, device=dev))
        if prec == bo.MIXED:
            for nm in ("Qd", "Ld", "Qbard"):
                kw[nm] = torch.zeros(N, dtype=torch.float64, device=dev)
        self.kw = kw
        self.gvals = torch.zeros_like(self.vals)
        self.dropped = torch.zeros(1, dtype=torch.int64, device=dev)
        self.plan = bo.Plan([n] * nb, [k] * nb, target_chunks=target_chunks, device=dev)
        self.io = self.plan.wh_io(reuse=True, **kw)   # backward right after forward

    def step(self):
        bo, p, kw = self.bo, self.prec, self.kw
        bo.csr_to_band(p, self.ip, self.ix, self.vals, self.k, kw["Q"], kw.get("Qd"), self.dropped, nsets=self.nb)
        self.plan.whiten(p, self.io)
        self.plan.whiten_bwd(p, self.io)
        bo.band_to_csr_grad(p, self.ip, self.ix, self.k, kw["Qbar"], kw.get("Qbard"), self.gvals, nsets=self.nb)


def make_graph(args, bo):
    """A W = 3 by L road strip (10^6 junctions by default) in its reverse
    Cuthill-McKee order (the library's host ordering and permuted pattern,
    timed together; the values are then laid out in the new order), Matérn-1/2 edge
    precisions for 16 lengthscales ell_b = 2 + b/8, v and Fbar ~ N(0, I) in the
    new order."""
    from paper_1902_10078_amd import inputs
    n, ip, ix, ln = inputs.road_graph(3, args.graph_len, seed=9)
    qip, qix, vals = inputs.graph_gmrf_csr(n, ip, ix, ln, ell=[2.0 + b / 8.0 for b in range(16)])
    t0 = time.perf_counter()
    perm, iperm, bw = bo.rcm(qip, qix)
    pip, pix, mp = bo.csr_permute(qip, qix, perm, iperm)
    rcm_ms = (time.perf_counter() - t0) * 1e3
    vs, Fbs = [], []
    for b in range(16):
        rng = np.random.default_rng(np.random.SeedSequence([10, b]))
        vs.append(rng.normal(size=n))
        Fbs.append(rng.normal(size=n))
    return dict(n=n, k=bw, indptr=qip, indices=qix, perm=perm, iperm=iperm, vals=vals, v=vs, Fbar=Fbs,
                pindptr=pip, pindices=pix, map=mp, rcm_ms=rcm_ms, nnz=int(qip[-1]))


def graph_bytes_per_row(k: int, prec: int, nnz_per_row: float):
    """Algorithmic bytes per row of the graph workload's kernels."""
    wb, wv = record_bytes(k, prec)
    csr = 8 + 16 * nnz_per_row          # indptr, column indices and values
    per = wh_bytes_per_row(k, prec)
    per["csr_to_band"] = csr + wb                       # CSR in band order -> band
    per["band_to_csr"] = 8 + 16 * nnz_per_row + wb      # indptr, indices, band gradient -> CSR gradient
    per["unit"] = per["unit"] + 2 * csr
    return per


class Alg5Workload:
    """One matrix: O = band of L^{-1} R (Algorithm 5) and the reverse mode
    (Table 1, solve matrix-matrix) from a fixed Obar; every output and the
    workspace allocated once, the step only launches."""

    def __init__(self, bo, torch, dev, host_inputs, k, lr, u):
        import ctypes
        L, R, Ob = host_inputs
        n = L.shape[0]
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        self.bo, self.k, self.lr, self.u = bo, k, lr, u
        self.t = dict(L=f(L), R=f(R), Obar=f(Ob))
        self.bands = dict(L=bo.Band(self.t["L"], k), R=bo.Band(self.t["R"], lr, u), Obar=bo.Band(self.t["Obar"], k, u),
                          O=bo.new_band(n, k, u, device=dev), Rbar=bo.new_band(n, lr, u, device=dev),
                          Lbar=bo.new_band(n, k, 0, device=dev))
        self.c = {nm: b.c() for nm, b in self.bands.items()}
        self.ws = torch.empty(max(int(bo.lib().bo_solve_band_mat_workspace(n, k, u)), 256), dtype=torch.uint8,
                              device=dev)
        self.kw = dict(O=self.bands["O"].band)
        self.ref = ctypes.byref

    def step(self):
        bo, c, r = self.bo, self.c, self.ref
        bo._check(bo.lib().bo_solve_band_mat(bo.F64, r(c["L"]), r(c["R"]), r(c["O"]), bo._stream()),
                  "bo_solve_band_mat")
        bo._check(bo.lib().bo_solve_band_mat_bwd(bo.F64, r(c["L"]), r(c["O"]), r(c["Obar"]), r(c["Rbar"]),
                                                 r(c["Lbar"]), bo._ptr(self.ws), self.ws.numel(), bo._stream()),
                  "bo_solve_band_mat_bwd")


def make_alg5(args):
    """L a lower band (diagonal U[1,2], off-diagonals N(0, 0.3^2)), R and
    Obar general bands with N(0,1) entries, seed 5."""
    from paper_1902_10078_amd import inputs
    n, k, lr, u = args.n_alg5, 5, 2, 5
    rng = np.random.default_rng(5)
    L = inputs.random_lower_band(n, k, rng)
    R = rng.normal(size=(n, lr + u + 1))
    Ob = rng.normal(size=(n, k + u + 1))
    for s_ in range(lr + u + 1):   # slots past the matrix edges are zero
        i = np.arange(n) - u + s_
        R[(i < 0) | (i >= n), s_] = 0.0
    for s_ in range(k + u + 1):
        i = np.arange(n) - u + s_
        Ob[(i < 0) | (i >= n), s_] = 0.0
    return [n], [k], (L, R, Ob), (k, lr, u)


class WideWorkload:
    """The wide block-banded batch on the device (mixed storage)."""

    def __init__(self, bo, torch, dev, ns, host_inputs):
        Qs, _, Ws = host_inputs
        self.plan = bo.WidePlan(ns, device=dev)
        f32 = lambda arrs: torch.from_numpy(np.concatenate([a.ravel() for a in arrs])).to(dev, torch.float32)
        f64 = lambda arrs: torch.from_numpy(np.concatenate([a[:, 0] for a in arrs])).to(dev)
        E, N = self.plan.band_elems, self.plan.rows
        kw = dict(Q=f32(Qs), Qd=f64(Qs), S=f32(Ws), Sd=f64(Ws),
                  parts=torch.zeros((len(ns), 3), dtype=torch.float64, device=dev),
                  info=torch.zeros(len(ns), dtype=torch.int32, device=dev))
        for nm in ("L", "Sig", "Lbar", "Qbar"):
            kw[nm] = torch.zeros(E, dtype=torch.float32, device=dev)
            kw[nm + "d"] = torch.zeros(N, dtype=torch.float64, device=dev)
        self.kw = kw
        self.io = self.plan.io(**kw)
        self.stats = {"nprob": len(ns), "blocks": sum((n + 63) // 64 for n in ns)}

    def step(self):
        self.plan.gauss_loss(self.io)


def make_wide(args, bo, torch, dev):
    """Q = D + band(B B^T) and W likewise (another seed), formed on the device
    with the library's banded product (input construction, untimed), then
    stored in the mixed format."""
    from paper_1902_10078_amd import inputs

    def build(b, seed):
        B, D = inputs.config4_factors(b, seed=seed, n=args.n_wide)
        Bb = bo.band_from(torch.from_numpy(B).to(dev), 64)
        Q = bo.bo_gbmm(Bb, Bb, 0, 1, 64, 0).band.cpu().numpy()
        Q[:, 0] += D
        Qr = Q.astype(np.float32).astype(np.float64)
        Qr[:, 0] = Q[:, 0]
        return Qr

    ns = [args.n_wide] * args.nwide
    Qs = [build(b, 4) for b in range(args.nwide)]
    Ws = [build(b, 5) for b in range(args.nwide)]
    ys = [np.zeros(n) for n in ns]
    return ns, [64] * len(ns), (Qs, ys, Ws)


def cpu_baseline_alg5(host_inputs, widths, rows: int):
    """The FP64 oracle (Algorithm 5 and its reverse mode, single-threaded:
    one sequential sweep per column family) on the first `rows` rows."""
    import oracle
    L, R, Ob = host_inputs
    k, lr, u = widths
    Ls, Rs, Obs = L[:rows].copy(), R[:rows].copy(), Ob[:rows].copy()
    for s_ in range(lr + u + 1):
        Rs[np.arange(rows) - u + s_ >= rows, s_] = 0.0
    for s_ in range(k + u + 1):
        Obs[np.arange(rows) - u + s_ >= rows, s_] = 0.0
    t0 = time.perf_counter()
    O = oracle.solve_band_mat(Ls, k, Rs, lr, u)
    oracle.solve_band_mat_bwd(Ls, k, O, Obs, lr, u)
    dt = time.perf_counter() - t0
    return dict(value=rows / dt, unit="band-rows/s", kind="oracle", **host_info(1),
                sample=f"the first {rows} rows of the matrix, FP64 C oracle (forward and reverse), "
                       f"one thread, {dt:.2f} s wall"), O


def cpu_baseline_ng(host_inputs, ns, nsample: int):
    """The FP64 oracle (Algorithm 10 and its reverse mode), one thread, problem
    after problem, on the first `nsample` problems."""
    import oracle
    idx = list(range(min(nsample, len(ns))))
    t0 = time.perf_counter()
    ref = np.array([oracle.natgp(host_inputs[i]["Lam_pr"], host_inputs[i]["eta_pr"], host_inputs[i]["Lam_lik"],
                                 host_inputs[i]["eta_lik"], host_inputs[i]["k"])["parts"] for i in idx])
    dt = time.perf_counter() - t0
    rows = sum(ns[i] for i in idx)
    return dict(value=rows / dt, unit="band-rows/s", kind="oracle", **host_info(1),
                sample=f"{len(idx)} of the workload's {len(ns)} problems ({rows} rows), FP64 C oracle "
                       f"(forward and reverse), one thread, {dt:.2f} s wall"), ref


def cpu_baseline_wh(host_inputs, ns, ks, nsample: int):
    """The FP64 oracle (Algorithm 6 and its reverse mode), one thread, problem
    after problem, on the first `nsample` problems; returns the log-determinants."""
    import oracle
    Qs, vs, Fbs = host_inputs
    idx = list(range(min(nsample, len(ns))))
    t0 = time.perf_counter()
    ref = []
    for i in idx:
        L, F, _ = oracle.whiten(Qs[i], ks[i], vs[i])
        oracle.whiten_bwd(L, ks[i], F, Fbs[i])
        ref.append(oracle.logdet(L, ks[i]))
    dt = time.perf_counter() - t0
    rows = sum(ns[i] for i in idx)
    return dict(value=rows / dt, unit="band-rows/s", kind="oracle", **host_info(1),
                sample=f"{len(idx)} of the workload's {len(ns)} problems ({rows} rows), FP64 C oracle "
                       f"(forward and reverse), one thread, {dt:.2f} s wall"), np.array(ref)


def cpu_baseline_ml(host_inputs, ns, ks, nsample: int):
    """The FP64 oracle (Algorithm 8 and its reverse mode), one thread, problem
    after problem, on the first `nsample` problems."""
    import oracle
    Qs, masks, bs, t2 = host_inputs
    idx = list(range(min(nsample, len(ns))))
    t0 = time.perf_counter()
    ref = np.array([oracle.marglik(Qs[i], ks[i], masks[i], bs[i], t2[i])["parts"] for i in idx])
    dt = time.perf_counter() - t0
    rows = sum(ns[i] for i in idx)
    return dict(value=rows / dt, unit="band-rows/s", kind="oracle", **host_info(1),
                sample=f"{len(idx)} of the workload's {len(ns)} problems ({rows} rows), FP64 C oracle "
                       f"(forward and reverse), one thread, {dt:.2f} s wall"), ref


def cpu_baseline(host_inputs, ns, ks, nsample: int, vi: bool = False):
    """The FP64 oracle as it stands, OpenMP across problems, on a bounded
    sample of the workload's problems."""
    import oracle
    idx = list(range(min(nsample, len(ns))))
    sn, sk = [ns[i] for i in idx], [ks[i] for i in idx]
    if vi:
        cat = lambda arrs: np.concatenate([arrs[i].ravel() for i in idx])
        Lqs, Lps, mqs, mps = host_inputs
        t0 = time.perf_counter()
        parts, _, _, _, _, threads = oracle.vi_kl_batch(sn, sk, cat(Lqs), cat(Lps), cat(mqs), cat(mps))
        dt = time.perf_counter() - t0
        rows = sum(sn)
        used = min(threads, len(idx))
        return dict(value=rows / dt, unit="band-rows/s", kind="oracle", **host_info(used),
                    sample=f"{len(idx)} of the workload's {len(ns)} problems ({rows} rows), FP64 C oracle, "
                           f"OpenMP across problems ({threads} threads, {used} busy), {dt:.2f} s wall"), parts
    Qs, ys, Ss = host_inputs
    Qf = np.concatenate([Qs[i].ravel() for i in idx])
    yf = np.concatenate([ys[i] for i in idx])
    t0 = time.perf_counter()
    full = None
    if Ss is not None:
        Sf = np.concatenate([Ss[i].ravel() for i in idx])
        ref, _, _, _, threads = oracle.gauss_loss_batch(sn, sk, Qf, yf, Sf)
    else:
        Lr, zr, xr, Sr, ref, _, threads = oracle.forward_batch(sn, sk, Qf, yf)
        full = dict(L=Lr, z=zr, x=xr, Sig=Sr, logdet=ref)
    dt = time.perf_counter() - t0
    rows = sum(sn)
    # OpenMP runs one problem per thread: the threads in use are at most the problems
    used = min(threads, len(idx))
    cb = dict(value=rows / dt, unit="band-rows/s", kind="oracle", **host_info(used),
              sample=f"{len(idx)} of the workload's {len(ns)} problems ({rows} rows), FP64 C oracle, "
                     f"OpenMP across problems ({threads} threads, {used} busy), {dt:.2f} s wall")
    if full is not None:
        cb["_full"] = full
    return cb, ref


def forward_output_errors(bo, kw, prec, ns, ks, full):
    """Per-output error of the forward list on the oracle's sample (the first
    problems of the batch): max |gpu - oracle| / max |oracle| for L, z, x and
    Sigma, and the largest relative log-det error.  Mixed bands are compared
    with their FP64 diagonals in slot 0."""
    m = len(full["logdet"])
    sn, sk = np.asarray(ns[:m], dtype=np.int64), np.asarray(ks[:m], dtype=np.int64)
    E, N = int(np.sum(sn * (sk + 1))), int(np.sum(sn))
    boff = np.concatenate([[0], np.cumsum(sn * (sk + 1))[:-1]])
    pos = np.concatenate([boff[b] + np.arange(sn[b]) * (sk[b] + 1) for b in range(m)]) if N else np.zeros(0, int)

    def band(nm):
        g = kw[nm][:E].double().cpu().numpy()
        if prec == bo.MIXED:
            g[pos] = kw[nm + "d"][:N].cpu().numpy()
        return g

    def rel(g, r):
        den = np.max(np.abs(r)) if r.size else 0.0
        return float(np.max(np.abs(g - r)) / den) if den > 0 else 0.0

    ld = kw["logdet"][:m].cpu().numpy()
    return {"L": rel(band("L"), full["L"]), "Sig": rel(band("Sig"), full["Sig"]),
            "z": rel(kw["z"][:N].double().cpu().numpy(), full["z"]),
            "x": rel(kw["x"][:N].double().cpu().numpy(), full["x"]),
            "logdet": float(np.max(np.abs(ld - full["logdet"]) / np.maximum(np.abs(full["logdet"]), 1e-300)))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["matern52_loss", "uneven_forward", "matern32_forward", "wide_loss",
                                           "vi_kl", "solve_band_mat", "marglik", "natgp_co2", "whiten_hmc", "graph_whiten"],
                    default="matern52_loss")
    ap.add_argument("--prec", choices=["f64", "mixed"], default=None,
                    help="storage format (default: f64; mixed for uneven_forward)")
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--n-in", type=int, default=1_000_000)
    ap.add_argument("--nprob", type=int, default=4096)
    ap.add_argument("--n-in32", type=int, default=100_000)
    ap.add_argument("--ell", type=float, default=10.0)
    ap.add_argument("--nwide", type=int, default=8)
    ap.add_argument("--n-wide", type=int, default=200_000)
    ap.add_argument("--n-vi", type=int, default=1_000_000, help="rows per problem of the KL batch")
    ap.add_argument("--nng", type=int, default=1024, help="problems of the natural-parameter GP batch")
    ap.add_argument("--t-ng", type=int, default=3082, help="weeks (inputs) per natural-parameter GP problem")
    ap.add_argument("--graph-len", type=int, default=333_334, help="length of the road strip (3 x len junctions)")
    ap.add_argument("--n-alg5", type=int, default=16_000_000, help="rows of the Algorithm 5 matrix")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="problems timed on the CPU oracle (default: the whole batch for the loss workload, 8 for the KL batch, "
                         "256 for the uneven batch, the whole batch for the marginal-likelihood, "
                         "natural-parameter, whitened and graph batches, 1 otherwise)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--caller-arrays", action="store_true",
                    help="loss unit: write L, Sigma and Lbar to caller arrays (default: keep them in the workspace)")
    ap.add_argument("--kernels-json", default="")
    ap.add_argument("--target-chunks", type=int, default=0, help="plan chunk target (0: library default)")
    ap.add_argument("--autotune", action="store_true",
                    help="measure a few chunk targets first and time the fastest")
    ap.add_argument("--tune-cache", default="", help="JSON cache for --autotune results")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (a known-size kernel "
                         "that calibrates HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        log("bench.py measures one GPU: the library has no multi-GPU path (a batch would shard by whole "
            "problems across GPUs, with no exchange between them). Use --gpus 1.")
        sys.exit(2)

    import torch
    if args.copy_probe:
        copy_probe(torch, args.copy_probe)
        return
    from paper_1902_10078_amd import bandops as bo

    if args.prec is None:
        args.prec = "mixed" if args.workload in ("uneven_forward", "wide_loss") else "f64"
    if args.workload == "wide_loss" and args.prec != "mixed":
        sys.exit("wide_loss runs in the mixed format only")
    prec = bo.F64 if args.prec == "f64" else bo.MIXED
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    t0 = time.perf_counter()
    forward_only = args.workload in ("uneven_forward", "matern32_forward")
    wide = args.workload == "wide_loss"
    vi = args.workload == "vi_kl"
    ml = args.workload == "marglik"
    ng = args.workload == "natgp_co2"
    wh = args.workload == "whiten_hmc"
    gr = args.workload == "graph_whiten"
    alg5 = args.workload == "solve_band_mat"
    if args.workload == "matern52_loss":
        ns, ks, host_inputs = make_matern52(args)
        cfg = {"workload": f"matern52_ssm_batch{len(ns)}_rows{ns[0]}_k5_gauss_loss_fwd_bwd",
               "batch": len(ns), "rows_per_problem": ns[0], "k": 5}
        nsample = args.cpu_sample or len(ns)   # the whole batch, one problem per OpenMP thread
    elif args.workload == "uneven_forward":
        ns, ks, host_inputs = make_uneven(args, bo, torch, dev)
        cfg = {"workload": f"uneven_batch{len(ns)}_n256-65536_k1-3-5-11_forward",
               "batch": len(ns), "rows": sum(ns), "k": "1,3,5,11"}
        nsample = args.cpu_sample or len(ns)   # the whole batch, OpenMP across problems
    elif alg5:
        ns, ks, host_inputs, widths = make_alg5(args)
        cfg = {"workload": f"solve_band_mat_rows{ns[0]}_k5_R2-5_fwd_bwd", "batch": 1,
               "rows_per_problem": ns[0], "k": 5, "R_lower": 2, "R_upper": 5}
        nsample = 0
    elif ml:
        ns, ks, host_inputs = make_ml(args)
        cfg = {"workload": f"marglik_matern52_batch{len(ns)}_rows{ns[0]}_k5_obs0.8_fwd_bwd",
               "batch": len(ns), "rows_per_problem": ns[0], "k": 5}
        nsample = args.cpu_sample or len(ns)   # the whole batch: about 10 s of one core
    elif gr:
        host_inputs = make_graph(args, bo)
        ns, ks = [host_inputs["n"]] * 16, [host_inputs["k"]] * 16
        if host_inputs["k"] > 12:
            sys.exit(f"graph bandwidth {host_inputs['k']} after ordering exceeds the compiled widths")
        cfg = {"workload": f"graph_whiten_road3x{args.graph_len}_rcm_batch16_k{host_inputs['k']}_fwd_bwd",
               "batch": 16, "rows_per_problem": host_inputs["n"], "k": host_inputs["k"],
               "nnz": host_inputs["nnz"], "rcm_host_ms": round(host_inputs["rcm_ms"], 1)}
        nsample = args.cpu_sample or 16   # the whole batch: a few seconds of one core
    elif wh:
        ns, ks, host_inputs = make_wh(args)
        cfg = {"workload": f"whiten_hmc_matern52_batch{len(ns)}_rows{ns[0]}_k5_fwd_bwd",
               "batch": len(ns), "rows_per_problem": ns[0], "k": 5}
        nsample = args.cpu_sample or 16
    elif ng:
        ns, ks, host_inputs = make_ng(args)
        cfg = {"workload": f"natgp_co2_batch{len(ns)}_weeks{args.t_ng}_rows{ns[0]}_k11_fwd_bwd",
               "batch": len(ns), "rows_per_problem": ns[0], "k": 11}
        nsample = args.cpu_sample or len(ns)   # the whole batch: a few seconds of one core
        # At k = 11 every chunk's replays are one lane's serial work; 65536
        # chunks (64 per problem) fill one round of resident waves (4 per CU
        # on 256 CUs) exactly, measured best against 32768, 72704, 98304,
        # 131072 and 196608 (also with the summaries and scans on quads).
        if not args.target_chunks and not args.autotune:
            args.target_chunks = 65536
    elif vi:
        ns, ks, host_inputs = make_vi(args)
        cfg = {"workload": f"vi_kl_batch{len(ns)}_rows{ns[0]}_k5_fwd_bwd",
               "batch": len(ns), "rows_per_problem": ns[0], "k": 5}
        nsample = args.cpu_sample or 8
    elif wide:
        ns, ks, host_inputs = make_wide(args, bo, torch, dev)
        cfg = {"workload": f"wide_blockband_batch{len(ns)}_rows{ns[0]}_k64_loss_fwd_bwd",
               "batch": len(ns), "rows_per_problem": ns[0], "k": 64}
        nsample = args.cpu_sample or 1
    else:
        ns, ks, host_inputs = make_matern32(args)
        cfg = {"workload": f"matern32_ssm_rows{ns[0]}_k3_ell{args.ell:g}_forward",
               "batch": 1, "rows_per_problem": ns[0], "k": 3}
        nsample = args.cpu_sample or 1
    rows = sum(ns)
    log(f"inputs: {len(ns)} problems, {rows} rows ({time.perf_counter() - t0:.1f} s)")

    if gr:
        W = GraphWorkload(bo, torch, dev, host_inputs, prec, args.target_chunks)
    elif wide:
        W = WideWorkload(bo, torch, dev, ns, host_inputs)
        log(f"wide plan: {W.stats}, workspace {W.plan.ws.numel() / 2**20:.1f} MiB")
    elif alg5:
        W = Alg5Workload(bo, torch, dev, host_inputs, *widths)
    else:
        if vi:
            W = VIWorkload(bo, torch, dev, ns, ks, prec, host_inputs, args.target_chunks)
        elif ml:
            W = MLWorkload(bo, torch, dev, ns, ks, prec, host_inputs, args.target_chunks)
        elif ng:
            W = NGWorkload(bo, torch, dev, ns, ks, prec, host_inputs, args.target_chunks)
        elif wh:
            W = WHWorkload(bo, torch, dev, ns, ks, prec, host_inputs, args.target_chunks)
        else:
            keep = not forward_only and prec == bo.F64 and not args.caller_arrays
            W = Workload(bo, torch, dev, ns, ks, prec, host_inputs, forward_only, args.target_chunks, keep=keep)
            if not forward_only:
                cfg.update(intermediates="workspace, interleaved by chunk" if keep else "caller arrays")
        if args.autotune:
            from paper_1902_10078_amd import autotune

            def make_step(t):
                W.set_schedule(t)
                return W.step
            tuned = autotune.tune(ns, ks, make_step, args.workload, prec,
                                  cache_path=args.tune_cache or None)
            W.set_schedule(tuned["target_chunks"])
            log(f"autotune: {tuned}")
        log(f"plan: {W.plan.stats}, workspace {W.plan.ws.numel() / 2**20:.1f} MiB")
    for _ in range(max(args.warmup, 1)):
        W.step()
    torch.cuda.synchronize()
    if "info" in W.kw:
        assert int(W.kw["info"].max().item()) == 0, "Cholesky failed on the benchmark inputs"
    elif alg5:
        assert bool(torch.isfinite(W.kw["O"]).all()), "non-finite solve on the benchmark inputs"
    else:
        assert bool(torch.isfinite(W.kw["parts"]).all()), "non-finite KL on the benchmark inputs"

    use_graph = not args.no_graph
    if use_graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                W.step()
        torch.cuda.current_stream().wait_stream(s)
        run = g.replay
        run()
        torch.cuda.synchronize()
    else:
        run = W.step

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
        W.step()
    prof = bo.profile_read()
    bo.profile_enable(False)
    if wide:
        bb = {nm: b * rows for nm, b in wide_bytes_per_row().items()}
    elif alg5:
        bb = {nm: b * rows for nm, b in alg5_bytes_per_row(*widths).items()}
    elif gr:
        bb = {nm: b * rows for nm, b in graph_bytes_per_row(ks[0], prec, host_inputs["nnz"] / ns[0]).items()}
    else:
        bb = batch_bytes(ns, ks, prec, forward_only, vi, ml, ng, wh)
    kern = {}
    for name, (tms, cnt) in prof.items():
        entry = dict(avg_ms=tms / cnt, launches_per_step=cnt / nprof, ms_per_step=tms / nprof)
        if name in bb:
            entry["alg_bytes_per_step"] = bb[name]
            entry["gbs"] = bb[name] / (tms / nprof / 1e3) / 1e9
        kern[name] = entry
        log(f"  {name:20s} {tms / nprof:8.3f} ms/step x{cnt / nprof:.0f}"
            + (f"  {entry['gbs']:8.1f} GB/s" if "gbs" in entry else ""))
    dom = max((k_ for k_ in kern if "gbs" in kern[k_]), key=lambda k_: kern[k_]["ms_per_step"])
    d = kern[dom]
    path = traffic_profile_path(args.workload, args.prec, args.batch, args.n_in)
    # per launch: every launch of the marginal likelihood's kernels covers all rows
    whole = d["launches_per_step"] == 1 or ml or ng
    roof = dict(bound="hbm", kernel=dom, achieved=round(d["gbs"], 2), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(d["gbs"] / HBM_PEAK_GBS, 4),
                traffic=measured_traffic(dom, path, rows) if whole else None,
                bytes_per_step=bb[dom], launches_per_step=d["launches_per_step"], rows=rows)
    unit_gbs = bb["unit"] / (ms / 1e3) / 1e9
    copy_rate = copy_gbs(torch, 1024)
    log(f"plain 1 GiB device copy: {copy_rate:.1f} GB/s (read + write)")
    if wide:
        tf = WIDE_FLOP_PER_ROW * rows / (ms / 1e3) / 1e12
        roof["mfma"] = dict(bound="mfma", achieved=round(tf, 3), peak=FP32_MFMA_PEAK_TFLOPS, unit="TFLOP/s",
                            frac=round(tf / FP32_MFMA_PEAK_TFLOPS, 5), flop_per_step=WIDE_FLOP_PER_ROW * rows,
                            note="algorithmic flops of the whole unit over the step time")
    if args.kernels_json:
        with open(args.kernels_json, "w") as f:
            json.dump(dict(kernels=kern, ms_per_step=ms, rows=rows), f, indent=1)

    # the plain FP64 one-matrix-per-launch form: per-problem plans, host loop, no graph
    vs_plain = None
    if not args.no_plain and not wide and not alg5 and not gr:
        if prec == bo.F64:
            W64 = W
        elif vi:
            W64 = VIWorkload(bo, torch, dev, ns, ks, bo.F64, host_inputs)
        elif ml:
            W64 = MLWorkload(bo, torch, dev, ns, ks, bo.F64, host_inputs)
        elif ng:
            W64 = NGWorkload(bo, torch, dev, ns, ks, bo.F64, host_inputs)
        elif wh:
            W64 = WHWorkload(bo, torch, dev, ns, ks, bo.F64, host_inputs)
        else:
            W64 = Workload(bo, torch, dev, ns, ks, bo.F64, host_inputs, forward_only)
        plain_step = W64.plain_steps()
        plain_step()
        torch.cuda.synchronize()
        reps = max(args.steps // 4, 2)
        e0.record()
        for _ in range(reps):
            plain_step()
        e1.record()
        torch.cuda.synchronize()
        ms_plain = e0.elapsed_time(e1) / reps
        vs_plain = ms_plain / ms
        log(f"plain FP64 one-matrix-per-launch: {ms_plain:.3f} ms/step -> batched is {vs_plain:.2f}x")

    cfg.update(storage=args.prec, graph=use_graph)
    if wide:
        cfg.update(blocks=W.stats["blocks"])
    elif alg5 or gr:
        pass
    else:
        cfg.update(chunks=W.plan.stats["nchunk"])
        if args.autotune:
            cfg.update(schedule={"target_chunks": tuned["target_chunks"],
                                 "candidates_ms": {str(k): round(v, 3) for k, v in tuned["ms"].items()}})
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "band-rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if (wide or prec != bo.F64) else "f64",
        "data": "synthetic",
        "config": cfg,
        "roofline": roof,
        "unit_hbm_frac": round(unit_gbs / HBM_PEAK_GBS, 4),
        "copy_gbs": round(copy_rate, 1),
        "unit_frac_of_copy": round(unit_gbs / copy_rate, 4),
        "dominant_frac_of_copy": round(d["gbs"] / copy_rate, 4),
        "vs_fp64_plain": vs_plain,
    }
    if not args.no_cpu and alg5:
        cb, ref = cpu_baseline_alg5(host_inputs, widths, rows=min(2_000_000, rows))
        got = W.kw["O"].cpu().numpy()[: ref.shape[0] - 12]   # rows whose band lies inside the sample
        cb["max_rel_diff_vs_gpu"] = float(np.max(np.abs(got - ref[: got.shape[0]])) / np.max(np.abs(ref)))
        out["cpu_baseline"] = cb
        log(f"cpu baseline: {cb}")
    elif not args.no_cpu and gr:
        import oracle
        g = host_inputs
        idx = list(range(min(nsample, 16)))
        t0 = time.perf_counter()
        ref = []
        for b in idx:
            B, _ = oracle.csr_to_band(g["n"], g["indptr"], g["indices"], g["vals"][b], g["perm"], g["k"])
            L, F, _ = oracle.whiten(B, g["k"], g["v"][b])
            oracle.whiten_bwd(L, g["k"], F, g["Fbar"][b])
            ref.append(oracle.logdet(L, g["k"]))
        dt = time.perf_counter() - t0
        rws = len(idx) * g["n"]
        cb = dict(value=rws / dt, unit="band-rows/s", kind="oracle", **host_info(1),
                  sample=f"{len(idx)} of the workload's 16 problems ({rws} rows), FP64 oracle (band assembly, "
                         f"whitened sample and its reverse mode), one thread, {dt:.2f} s wall")
        gp = W.kw["logdet"].cpu().numpy()[: len(ref)]
        cb["max_rel_diff_vs_gpu"] = float(np.max(np.abs(gp - np.array(ref)) / np.abs(np.array(ref))))
        out["cpu_baseline"] = cb
        log(f"cpu baseline: {cb}")
    elif not args.no_cpu and wh:
        cb, ref = cpu_baseline_wh(host_inputs, ns, ks, nsample)
        gp = W.kw["logdet"].cpu().numpy()[: len(ref)]
        cb["max_rel_diff_vs_gpu"] = float(np.max(np.abs(gp - ref) / np.maximum(np.abs(ref), 1e-300)))
        out["cpu_baseline"] = cb
        log(f"cpu baseline: {cb}")
    elif not args.no_cpu and ng:
        cb, ref = cpu_baseline_ng(host_inputs, ns, nsample)
        gp = W.kw["parts"].cpu().numpy()[: len(ref)]
        cb["max_rel_diff_vs_gpu"] = float(np.max(np.abs(gp - ref) / np.maximum(np.abs(ref), 1e-300)))
        out["cpu_baseline"] = cb
        log(f"cpu baseline: {cb}")
    elif not args.no_cpu and ml:
        cb, ref = cpu_baseline_ml(host_inputs, ns, ks, nsample)
        gp = W.kw["parts"].cpu().numpy()[: len(ref)]
        cb["max_rel_diff_vs_gpu"] = float(np.max(np.abs(gp - ref) / np.maximum(np.abs(ref), 1e-300)))
        out["cpu_baseline"] = cb
        log(f"cpu baseline: {cb}")
    elif not args.no_cpu:
        cb, ref = cpu_baseline(host_inputs, ns, ks, nsample, vi)
        src = W.kw["logdet"] if forward_only else W.kw["parts"]
        gp = src.cpu().numpy()[: len(ref)]
        cb["max_rel_diff_vs_gpu"] = float(np.max(np.abs(gp - ref) / np.maximum(np.abs(ref), 1e-300)))
        full = cb.pop("_full", None)
        if full is not None and forward_only:
            out["rel_err_vs_oracle"] = dict(forward_output_errors(bo, W.kw, prec, ns, ks, full),
                                            sample=f"the first {len(ref)} problems")
        out["cpu_baseline"] = cb
        log(f"cpu baseline: {cb}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
