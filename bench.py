"""Benchmark: lambda-solves/s of sketch-preconditioned Tikhonov least squares.

One step = the whole hot path for one batch: sketch A once, build every
preconditioner, run preconditioned LSQR for all lambdas (and all problems).
The default workload is the tall kappa(A) = 1e8 problem (m = 200000,
n = 2000, N = 32, lambda in [1e-8, 1e-1], SRHT sketch of size 4n, Cholesky
route).  --workload selects the others:

  over_svd      m=2000 n=100 N=10, Haar factors, SRHT s=4n, plain FP64
  over_gauss    (default) as above, mixed batched with FP64 fallback
  under_scaled  m=2000 n=200000 N=32, A_ij = G_ij / j in FP32, BF16 Gaussian
                sketch s=4m, mixed batched (Algorithm 2)
  lowsd         m=100000 n=10000 N=16, sigma_i = exp(-i/200), FP32 A, BF16
                Gaussian sketch s = 2 ceil(sd), low-rank route (Algorithm 3)
  ragged        256 problems m~U[5000,50000] n~U[100,1000] N=8 (2048 solves),
                FP32 A, BF16 sketches s=4n_p, mixed batched

A and b are resident on the GPU before timing starts.

value = (number of solves within 1e-8 relative error of the CPU FP64 oracle)
/ (seconds per step) for the batched solve; every solve is checked: the
oracle's direct solve for every problem, or, where that takes minutes (the
low-rank workload), an a-posteriori bound (gradient in extended precision,
inverted with the generator's planted factors).  config.mode names what ran:
a mixed-mode call whose every lambda needed FP64 products is f64_batched.
The timed steps run as a user runs them (the solve loop replays captured
graphs); then --prof-steps more steps run with HIP events around every
launch on the library's stream, which give the kernel durations behind
roofline (the dominant kernel family's algorithmic bytes per launch over its
average launch time).  Beside the timed mode, the plain FP64 per-lambda loop
and batched FP64 are timed (events) at an LSQR tolerance whose forward error
meets the FP64 target 1e-10, each with its own error against the oracle.
cpu_baseline: the oracle's direct QR solve, timed on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
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

METRIC = "λ-solves/s to 1e-8 rel err: mixed batched vs plain FP64; HBM GB/s"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFS = 2500.0   # MI355X dense BF16 matrix peak
FP64_PEAK_TFS = 78.6     # MI355X FP64 matrix (and vector) peak
FP32_PEAK_TFS = 157.3    # MI355X FP32 matrix peak
TOL_ERR = 1e-8
FAMILIES = ("sketch", "gram", "chol", "trinv", "lowrank", "lr_qr", "lr_sweep", "lr_q", "gemm_n",
            "gemm_t", "trmv", "trmv_t", "lr_apply", "vec", "residual")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def generate(name, W, dev):
    """The problems of one named workload."""
    gens = {"over_svd": lambda: [W.over_svd()], "over_gauss": lambda: [W.over_gauss()],
            "under_scaled": lambda: [W.under_scaled()], "lowsd": lambda: [W.lowsd(device=dev)],
            "ragged": lambda: W.ragged()}
    if name not in gens:
        raise SystemExit(f"unknown workload {name}")
    return gens[name]()


def workload_cfg(name, tik, plist):
    """Settings (embedding, sketch precision, route, mode, description, check) of a workload."""
    if name == "over_svd":
        return dict(embed=tik.SRHT, sdt=tik.F64, route=tik.ROUTE_CHOL, mode="f64",
                    desc="tall Haar SVD, sigma logspaced 1..1e-6: m=2000 n=100 N=10 lambda 1e-6..1, "
                         "SRHT s=400, Cholesky route", check="full")
    if name == "over_gauss":
        return dict(embed=tik.SRHT, sdt=tik.F64, route=tik.ROUTE_CHOL, mode="auto",
                    desc="tall Gaussian, sigma logspaced 1..1e-8: m=200000 n=2000 N=32 lambda "
                         "1e-8..1e-1, SRHT s=8000, Cholesky route", check="full")
    if name == "under_scaled":
        return dict(embed=tik.GAUSS, sdt=tik.BF16, route=tik.ROUTE_CHOL, mode="auto",
                    desc="wide A_ij = G_ij / j (FP32): m=2000 n=200000 N=32 lambda 1e-6..1, BF16 "
                         "Gaussian s=8000, Cholesky route (Algorithm 2)", check="full")
    if name == "lowsd":
        return dict(embed=tik.GAUSS, sdt=tik.BF16, route=tik.ROUTE_LOWRANK, mode="auto",
                    desc=f"tall U diag(exp(-i/200)) V^T (FP32): m=100000 n=10000 N=16 lambda "
                         f"1e-4..1e-1, BF16 Gaussian s={plist[0].s}, low-rank route (Algorithm 3)",
                    check="certify")
    if name == "ragged":
        return dict(embed=tik.GAUSS, sdt=tik.BF16, route=tik.ROUTE_CHOL, mode="auto",
                    desc="256 tall Gaussian problems, sigma logspaced 1..1e-6 (FP32): m~U[5000,50000] "
                         "n~U[100,1000] N=8 lambda 1e-6..1e-1, BF16 Gaussian s=4n_p, Cholesky route",
                    check="full")
    raise SystemExit(f"unknown workload {name}")


def build_workload(name, tik, W, dev):
    """(problems, settings) of one named workload."""
    plist = generate(name, W, dev)
    return plist, workload_cfg(name, tik, plist)


SAVED_FIELDS = ("A", "b", "lams", "sigma", "U", "V", "x0")


def save_workload(path, plist):
    """Problems as .npy files (array fields) plus meta.json (the scalar settings)."""
    os.makedirs(path, exist_ok=True)
    meta = []
    for k, p in enumerate(plist):
        d = {"name": p.name, "s": p.s, "embed": p.embed, "route": p.route, "tol": p.tol,
             "seed": p.seed, "alpha": p.alpha, "arrays": []}
        for f in SAVED_FIELDS:
            v = getattr(p, f)
            if v is not None:
                np.save(os.path.join(path, f"{k}_{f}.npy"), v, allow_pickle=False)
                d["arrays"].append(f)
        meta.append(d)
    with open(os.path.join(path, "meta.json"), "w") as fh:
        json.dump(meta, fh)


def load_workload(path, name, tik, W):
    """Problems written by save_workload (arrays memory-mapped), with the workload's settings."""
    with open(os.path.join(path, "meta.json")) as fh:
        meta = json.load(fh)
    plist = []
    for k, d in enumerate(meta):
        arrs = {f: np.load(os.path.join(path, f"{k}_{f}.npy"), mmap_mode="r", allow_pickle=False)
                for f in d["arrays"]}
        plist.append(W.Problem(d["name"], arrs["A"], np.asarray(arrs["b"]), np.asarray(arrs["lams"]), d["s"],
                               d["embed"], d["route"], d["tol"], d["seed"], sigma=arrs.get("sigma"),
                               U=arrs.get("U"), V=arrs.get("V"), x0=arrs.get("x0"), alpha=d["alpha"]))
    return plist, workload_cfg(name, tik, plist)


MAXIT = 300
F64_TARGET = 1e-10          # forward error the FP64 path is held to
# LSQR tolerance per workload at which the FP64 legs reach F64_TARGET
F64_TOL = {"over_svd": 1e-12, "over_gauss": 1e-13, "under_scaled": 1e-12, "lowsd": 1e-12,
           "ragged": 1e-12}
FAMILY_KERNEL = {"gemm_n": "k_gemm_n", "gemm_t": "k_gemm_t", "trmv": "k_trmv<", "trmv_t": "k_trmv_t<",
                 "lr_apply": "k_lr_"}


def cpu_model():
    """The host CPU's model name (Linux), for the CPU baseline's record."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def measured_traffic(workload, family):
    """HBM bytes per launch of the family's kernel from the committed rocprofv3 counter record
    (profiles/traffic.json: FETCH_SIZE and WRITE_SIZE, scaled by a device-copy calibration),
    or None when there is none or the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))[workload]
        h = hashlib.sha256()
        for src in rec["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
        if h.hexdigest() != rec["source_sha256"]:
            return None
        key = FAMILY_KERNEL.get(family)
        bpd = rec["bytes_per_dispatch"]
        if family == "gemm_n":
            # one A W launch of the family is k_gemm_n_mfma<TA, TC, NC, 0, RT> (every
            # row block), or, where the last round is split into column pieces,
            # k_gemm_n_mfma<TA, TC, NC, 3, RT> (the row blocks and the pieces) and
            # their sum (k_gemm_n_tail_fin<TC>)
            best = None
            for k, v in bpd.items():
                if "k_gemm_n_mfma<" not in k:
                    continue
                args = k.split("k_gemm_n_mfma<", 1)[1].split(">", 1)[0].split(",")
                if len(args) != 5 or args[3].strip() not in ("0", "3"):
                    continue
                tot = v
                if args[3].strip() == "3":
                    tot += max([w for kk, w in bpd.items()
                                if "k_gemm_n_tail_fin<" + args[1].strip() + ">" in kk] or [0])
                best = tot if best is None else max(best, tot)
            return int(best) if best is not None else None
        vals = [v for k, v in bpd.items() if key and key in k]
        return int(max(vals)) if vals else None
    except (OSError, KeyError, ValueError):
        return None


def pick_mode(tik, pr, cfg, svec, lams, alpha, want):
    """(mode, LSQR tol) of the timed batched solve: mixed where the library offers it."""
    mode = tik.F64_BATCHED
    if want in ("auto", "mixed"):
        try:
            sk = tik.sketch(pr, cfg["embed"], svec, 0, sketch_dtype=cfg["sdt"])
            pc = tik.precond(sk, lams, cfg["route"], alpha)
            tik.Solver(pr, pc, tik.MIXED_BATCHED)
            mode = tik.MIXED_BATCHED
            del sk, pc
        except tik.TikError as e:
            if want == "mixed":
                raise
            log("mixed mode unavailable, timing FP64 batched:", e)
    return mode, (1e-11 if mode == tik.F64_BATCHED else 1e-8)


def run_study(args, tik, W, torch) -> int:
    """Embedding study of Section 4.2 (the comparison of Fig. 3) on the paper's kind of
    matrix: for each embedding (SRHT, Gaussian, sparse with 1 or 8 nonzeros per column)
    and sketch size on the Cholesky route, and for the low-rank route, the condition
    number of the preconditioned matrix B R^{-1} per lambda, the LSQR iterations and the
    time of each stage; unpreconditioned LSQR beside it.  kappa(B R^{-1}) is measured
    from the downloaded preconditioner: W = A R^{-1} on the GPU, then the eigenvalues of
    W^T W + lam R^{-T} R^{-1} on the host (well conditioned: the preconditioned Gram)."""
    import math
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    p = W.decay50(m=args.study_m, n=args.study_n, N=args.study_N)
    log(f"generated the {p.m} x {p.n} study matrix in {time.perf_counter() - t0:.1f}s")
    pr = tik.Problems.from_numpy([p.A], [p.b], device=dev)
    A_d = torch.from_numpy(np.ascontiguousarray(p.A)).to(dev)
    n = p.n
    lams = p.lams
    sd = np.array([float(np.sum(1.0 / (1.0 + lam / p.sigma ** 2))) for lam in lams])
    sdm = int(math.ceil(sd.max()))
    cases = [("chol", "srht", 1, s) for s in (2 * n, 4 * n, 10 * n)]
    cases += [("chol", "gauss", 1, s) for s in (2 * n, 4 * n)]
    cases += [("chol", "sparse", 1, s) for s in (4 * n, 10 * n)]
    cases += [("chol", "sparse", 8, 2 * n)]
    cases += [("lowrank", "gauss", 1, min(n, 2 * sdm)), ("lowrank", "srht", 1, min(n, 10 * sdm))]
    embeds = {"srht": tik.SRHT, "gauss": tik.GAUSS, "sparse": tik.SPARSE}
    rows = []

    def kappa_of(Rinv, lam):
        R_d = torch.from_numpy(Rinv).to(dev)
        Wm = A_d @ R_d
        G = (Wm.T @ Wm + lam * (R_d.T @ R_d)).cpu().numpy()
        ev = np.linalg.eigvalsh(0.5 * (G + G.T))
        return float(math.sqrt(ev[-1] / ev[0])) if ev[0] > 0 else float("inf")

    # one untimed pass of each kind first: module loading and first-call setup
    for route, emb in (("chol", "srht"), ("chol", "gauss"), ("chol", "sparse"), ("lowrank", "gauss")):
        sk = tik.sketch(pr, embeds[emb], [min(n, 2 * sdm) if route == "lowrank" else 2 * n], 1)
        pc = tik.precond(sk, lams, tik.ROUTE_CHOL if route == "chol" else tik.ROUTE_LOWRANK, 2.0)
        tik.lsqr_batch(pr, pc, tik.F64_BATCHED, args.study_tol, 2000)
    torch.cuda.synchronize()
    for route, emb, zeta, s in cases:
        tik.set_option("sparse_nnz", zeta)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        torch.cuda.synchronize()
        ev[0].record()
        sk = tik.sketch(pr, embeds[emb], [s], 1)
        ev[1].record()
        rt = tik.ROUTE_CHOL if route == "chol" else tik.ROUTE_LOWRANK
        pc = tik.precond(sk, lams, rt, 2.0)
        ev[2].record()
        res = tik.lsqr_batch(pr, pc, tik.F64_BATCHED, args.study_tol, 2000)
        ev[3].record()
        torch.cuda.synchronize()
        its = res.iters.cpu().numpy()[0].tolist()
        kap = []
        for i, lam in enumerate(lams):
            if route == "chol":
                Rinv = pc.data(0, i)
            else:
                V = pc.data(0, i)
                sig = pc.sigma(0)[:V.shape[1]]
                Sd = 1.0 - 1.0 / np.sqrt(1.0 + sig ** 2 / lam)
                Rinv = (np.eye(n) - (V * Sd[None, :]) @ V.T) / math.sqrt(lam)
            kap.append(round(kappa_of(Rinv, lam), 3))
        row = {"route": route, "embedding": emb if emb != "sparse" else f"sparse{zeta}", "s": s,
               "s_over_n": round(s / n, 2), "kappa_BRinv": kap, "iters": its,
               "status_ok": bool(np.all(res.status.cpu().numpy() <= 1)),
               "ranks": [pc.rank(0, i) for i in range(len(lams))] if route == "lowrank" else None,
               "ms": {"sketch": round(ev[0].elapsed_time(ev[1]), 3), "precond": round(ev[1].elapsed_time(ev[2]), 3),
                      "solve": round(ev[2].elapsed_time(ev[3]), 3)}}
        rows.append(row)
        log(f"{route:8s} {row['embedding']:8s} s={s:6d} kappa max {max(kap):9.3f} iters max {max(its):4d} "
            f"ms {row['ms']}")
        del sk, pc, res
    tik.set_option("sparse_nnz", 1)
    # unpreconditioned LSQR (scipy, on the host) for a few lambdas, capped
    none = None
    if args.study_none:
        from scipy.sparse.linalg import lsqr
        kB = [float(math.sqrt((p.sigma[0] ** 2 + lam) / (p.sigma[-1] ** 2 + lam))) for lam in lams]
        pick = [0, len(lams) // 2, len(lams) - 1]
        it_none = {}
        for i in pick:
            lam = float(lams[i])
            out = lsqr(p.A, p.b, damp=math.sqrt(lam), atol=args.study_tol, btol=args.study_tol,
                       iter_lim=args.study_none)
            it_none[f"{lam:.1e}"] = int(out[2])
        none = {"kappa_B": [round(k, 3) for k in kB], "iters_at": it_none, "iter_cap": args.study_none}
        log(f"unpreconditioned: iterations {it_none} (cap {args.study_none})")
    line = {"study": "embedding", "matrix": f"A = U diag(logspace(0, -50, {n})) V^T, {p.m} x {n}, FP64",
            "lambdas": [float(v) for v in lams], "sd": [round(float(v), 1) for v in sd],
            "tol": args.study_tol, "cases": rows, "unpreconditioned": none}
    print(json.dumps(line), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="over_gauss",
                    choices=["over_svd", "over_gauss", "under_scaled", "lowsd", "ragged"])
    ap.add_argument("--mode", default=None, choices=["auto", "mixed", "f64"])
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--alt-steps", type=int, default=1,
                    help="steps of batched FP64 on the same input at the FP64 legs' tolerance")
    ap.add_argument("--no-oracle", action="store_true", help="skip the oracle (profiling runs)")
    ap.add_argument("--calibrate-copy", type=float, default=0.0,
                    help="GiB: also run one plain device copy of this size (HBM counter calibration)")
    ap.add_argument("--prof-steps", type=int, default=2,
                    help="steps run after the timed ones with per-launch events on (kernel durations)")
    ap.add_argument("--graph-chunk", type=int, default=None,
                    help="LSQR iterations per graph-captured chunk (library option; 0: no graphs)")
    ap.add_argument("--f64-tol", type=float, default=None,
                    help="LSQR tolerance of the FP64 legs (default: one that reaches 1e-10)")
    ap.add_argument("--save-inputs", default=None, metavar="DIR",
                    help="generate the workload, write it to DIR as .npy files and exit (lets a "
                         "profiled run load inputs made by an unprofiled process)")
    ap.add_argument("--load-inputs", default=None, metavar="DIR",
                    help="load the workload from DIR (written by --save-inputs) instead of generating it")
    ap.add_argument("--study", default=None, choices=["embedding"],
                    help="run the embedding study (Section 4.2) instead of the benchmark")
    ap.add_argument("--study-m", type=int, default=50000)
    ap.add_argument("--study-n", type=int, default=1000)
    ap.add_argument("--study-N", type=int, default=16)
    ap.add_argument("--study-tol", type=float, default=1e-10)
    ap.add_argument("--study-none", type=int, default=1000,
                    help="iteration cap of the unpreconditioned LSQR runs (0: skip them)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding of "
              "this path (rows or columns of A per GPU, one all-reduce per product) is not built",
              file=sys.stderr)
        return 2

    import torch
    import workloads as W
    from paper_2203_07329_amd import tik

    if args.study:
        return run_study(args, tik, W, torch)
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.graph_chunk is not None:
        tik.set_option("graph_chunk", args.graph_chunk)
    t0 = time.perf_counter()
    if args.load_inputs:
        plist, cfg = load_workload(args.load_inputs, args.workload, tik, W)
        log(f"loaded {len(plist)} problem(s) from {args.load_inputs} in {time.perf_counter() - t0:.1f}s")
    else:
        plist, cfg = build_workload(args.workload, tik, W, "cuda:0")
        log(f"generated {len(plist)} problem(s), {sum(p.m * p.n for p in plist) / 1e6:.0f} M entries "
            f"in {time.perf_counter() - t0:.1f}s")
    if args.save_inputs:
        save_workload(args.save_inputs, plist)
        log(f"saved to {args.save_inputs}")
        return 0
    pr = tik.Problems.from_numpy([p.A for p in plist], [p.b for p in plist], device=dev)
    torch.cuda.synchronize()
    svec = [p.s for p in plist]
    lams = np.stack([p.lams for p in plist])
    nsolve = int(lams.size)
    alpha = plist[0].alpha

    def one_step(m_, tol, marks=None):
        """sketch, preconditioners, batched solve; `marks` collects an event after each stage."""
        def mark():
            if marks is not None:
                e = torch.cuda.Event(enable_timing=True)
                e.record()
                marks.append(e)
        mark()
        sk = tik.sketch(pr, cfg["embed"], svec, 0, sketch_dtype=cfg["sdt"])
        mark()
        pc = tik.precond(sk, lams, cfg["route"], alpha)
        mark()
        out = tik.Solver(pr, pc, m_)(tol, maxit)
        mark()
        return out

    mode, tol = pick_mode(tik, pr, cfg, svec, lams, alpha, args.mode or cfg["mode"])
    dtype = "f32+f64" if mode == tik.MIXED_BATCHED else "f64"
    maxit = MAXIT
    # FP64 legs at a tolerance whose forward error meets the FP64 target of 1e-10:
    # x = R^{-1} y amplifies the error of y along R's small singular directions
    f64_tol = args.f64_tol or F64_TOL.get(args.workload, 1e-13)

    def timed(m_, tol_, steps):
        """Mean ms per step of `steps` whole steps, between events on the current stream."""
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(steps):
            out = one_step(m_, tol_)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps, out

    # ---- warmup
    for _ in range(args.warmup):
        one_step(mode, tol)
    torch.cuda.synchronize()
    log("warmup done")

    # ---- timed steps (no per-launch events: the solve loop replays captured graphs)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    w0 = time.perf_counter()
    marks = []
    for _ in range(args.steps):
        res = one_step(mode, tol, marks)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = ev0.elapsed_time(ev1) / args.steps
    launch_shape = tik.last_tiles()    # the product launch shape of the last solve group timed
    n32, n64 = tik.lsqr_info()
    # ---- profiled steps: the same steps with HIP events around every launch on the
    # library's stream (each iteration then launched directly), for kernel durations
    tik.prof_reset()
    tik.prof_enable(True)
    torch.cuda.synchronize()
    for _ in range(args.prof_steps):
        one_step(mode, tol)
    torch.cuda.synchronize()
    tik.prof_enable(False)
    # wall time of each stage on the caller's stream, per step
    stage_ms = {k: 0.0 for k in ("sketch", "precond", "solve")}
    for st in range(args.steps):
        e = marks[4 * st:4 * st + 4]
        for j, k in enumerate(("sketch", "precond", "solve")):
            stage_ms[k] += e[j].elapsed_time(e[j + 1]) / args.steps
    log(f"timed {args.steps} steps: {ms_step:.2f} ms/step")
    fam = {}
    npf = max(1, args.prof_steps)
    for f in FAMILIES:
        ms, n = tik.prof_query(f)
        if n:
            fam[f] = (ms / npf, n // npf, ms / n)
    if mode == tik.MIXED_BATCHED:
        dtype = "f32+f64" if n32 > 0 else "f64"
    # what ran: a mixed call whose every lambda needed FP64 products is batched FP64
    ran = "mixed_batched" if (mode == tik.MIXED_BATCHED and n32 > 0) else "f64_batched"
    # ---- L-curve of the timed step's solutions (Section 4.3): both norms in FP64 on
    # the GPU (one pass over each A), the corner on the host; outside the timed region
    lc = None
    if lams.shape[1] >= 3:
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        xn_d, rn_d = tik.lcurve(pr, res.X)
        b.record()
        torch.cuda.synchronize()
        xn_h, rn_h = xn_d.cpu().numpy(), rn_d.cpu().numpy()
        corners = [tik.lcurve_corner(lams[k], xn_h[k], rn_h[k])[0] for k in range(len(plist))]
        lc = {"ms": round(a.elapsed_time(b), 3), "corner_index": corners[0],
              "corner_lambda": float(lams[0][corners[0]])}
        if len(plist) > 1:
            lc["corner_index_p50"] = float(np.percentile(corners, 50))
    Xs = [res.x_numpy(k) for k in range(len(plist))]
    iters = res.iters.cpu().numpy()
    status = res.status.cpu().numpy()
    if args.calibrate_copy > 0:
        nel = int(args.calibrate_copy * (1 << 30)) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nel * 8} bytes read, {nel * 8} bytes written")
        del src, dst

    # ---- plain FP64 per-lambda loop
    plain = None
    if args.plain_steps > 0:
        plain_ms, rp = timed(tik.PLAIN_F64_PER_LAMBDA, f64_tol, args.plain_steps)
        plain = {"ms_per_step": plain_ms, "X": [rp.x_numpy(k) for k in range(len(plist))],
                 "iters": rp.iters.cpu().numpy(), "tol": f64_tol}
        log(f"plain per-lambda (tol {f64_tol:g}): {plain_ms:.1f} ms/step")

    # ---- batched FP64 on the same input, beside a mixed-mode line (FP32-stored A
    # is read at the same bytes per pass in both modes)
    alt = None
    if args.alt_steps > 0:
        one_step(tik.F64_BATCHED, f64_tol)
        alt_ms, ra = timed(tik.F64_BATCHED, f64_tol, args.alt_steps)
        alt = {"ms_per_step": alt_ms, "X": [ra.x_numpy(k) for k in range(len(plist))],
               "iters": ra.iters.cpu().numpy(), "tol": f64_tol}
        log(f"batched FP64 on the same input (tol {f64_tol:g}): {alt_ms:.1f} ms/step")

    # ---- oracle (timed: the CPU baseline) and accuracy
    n_ok = None
    err_max = None
    cpu = None
    checked = None
    if not args.no_oracle:
        import oracle
        try:
            from threadpoolctl import threadpool_info
            cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [os.cpu_count()])
        except Exception:  # pragma: no cover
            cores = os.cpu_count()
        if cfg["check"] == "certify":
            p = plist[0]
            c0 = time.perf_counter()
            bound = oracle.certify_planted(p.A, p.b, p.lams, Xs[0], p.sigma, p.V)
            tcert = time.perf_counter() - c0
            errs = [bound]
            pl_errs = [oracle.certify_planted(p.A, p.b, p.lams, plain["X"][0], p.sigma, p.V)] \
                if plain is not None else None
            al_errs = [oracle.certify_planted(p.A, p.b, p.lams, alt["X"][0], p.sigma, p.V)] \
                if alt is not None else None
            checked = f"all {nsolve} solves by an a-posteriori bound ({tcert:.1f} s on the host)"
        else:
            idx = list(range(len(plist)))
            c0 = time.perf_counter()
            Xo = {}
            for k in idx:
                Xo[k] = oracle.solve(plist[k].A, plist[k].b, plist[k].lams)
                if len(idx) > 1 and (k + 1) % 32 == 0:
                    log(f"oracle: {k + 1} of {len(idx)} problems solved ({time.perf_counter() - c0:.0f} s)")
            tcpu = time.perf_counter() - c0
            errs = [oracle.rel_err(Xs[k], Xo[k]) for k in idx]
            pl_errs = [oracle.rel_err(plain["X"][k], Xo[k]) for k in idx] if plain is not None else None
            al_errs = [oracle.rel_err(alt["X"][k], Xo[k]) for k in idx] if alt is not None else None
            nsamp = sum(plist[k].lams.size for k in idx)
            what = (f"Householder QR of A once plus per-lambda QR solves, {len(idx)} problem(s), "
                    f"{nsamp} solves ({tcpu:.1f} s)")
            cpu = {"value": round(nsamp / tcpu, 4), "unit": "λ-solves/s", "cores": int(cores),
                   "kind": "oracle", "cpu": cpu_model(),
                   "sample": "full workload: " + what}
            checked = f"{len(idx)} of {len(plist)} problems against the oracle's direct solve"
        allerr = np.concatenate([np.ravel(e) for e in errs])
        err_max = float(allerr.max())
        n_ok = int(np.sum(allerr <= TOL_ERR))          # every solve is checked
        for other, oe in ((plain, pl_errs), (alt, al_errs)):
            if other is not None and oe is not None:
                pe = np.concatenate([np.ravel(e) for e in oe])
                other["n_ok"] = int(np.sum(pe <= TOL_ERR))
                other["n_ok_f64"] = int(np.sum(pe <= F64_TARGET))
                other["max_rel_err"] = float(pe.max())
    value = (n_ok if n_ok is not None else 0) / (ms_step / 1000.0)

    # ---- roofline of the dominant kernel family with known algorithmic bytes
    ab = 8 if plist[0].A.dtype == np.float64 else 4
    vb = 4 if (mode == tik.MIXED_BATCHED and n32 > 0) else 8
    N = lams.shape[1]
    a_bytes = sum(p.m * p.n * ab for p in plist)
    long_short = sum((p.m + p.n) for p in plist)
    kmin = [min(p.m, p.n) for p in plist]
    per_launch = {
        # one pass over every A, plus the N-wide vectors on both sides of it
        "gemm_n": a_bytes + N * long_short * vb * 2,
        "gemm_t": a_bytes + N * long_short * vb,
    }
    if cfg["route"] == tik.ROUTE_CHOL:
        # upper triangles of the N inverses of every problem, FP64
        per_launch["trmv"] = per_launch["trmv_t"] = sum(N * k * k * 4 for k in kmin)
    else:
        # V (k x s) read twice per application: projection and expansion
        per_launch["lr_apply"] = sum(2 * k * p.s * 8 for k, p in zip(kmin, plist))
    # algorithmic flops per launch of the products: 2 m n N per problem (one product over A)
    flops_launch = {"gemm_n": sum(2.0 * p.m * p.n * N for p in plist),
                    "gemm_t": sum(2.0 * p.m * p.n * N for p in plist)}
    known = {k: v for k, v in fam.items() if k in per_launch}
    dom = max(known.items(), key=lambda kv: kv[1][0]) if known else None
    roof = None
    if dom:
        name, (ms_ps, launches, avg_ms) = dom
        ach = per_launch[name] / (avg_ms / 1000.0) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(args.workload, name),
                "kernel": name, "avg_launch_ms": round(avg_ms, 4),
                "algorithmic_bytes_per_launch": int(per_launch[name])}
        if name in flops_launch:
            # the same launches against the matrix-core peak of their arithmetic
            pk = FP64_PEAK_TFS if (vb == 8) else FP32_PEAK_TFS
            tf = flops_launch[name] / (avg_ms / 1000.0) / 1e12
            roof["matrix_core"] = {"achieved": round(tf, 2), "peak": pk, "unit": "TFLOP/s",
                                   "frac": round(tf / pk, 4), "flops_per_launch": flops_launch[name]}
        # one whole LSQR iteration (batched FP64 loop) against the bound of a single fused
        # pass: max(A once plus the preconditioner's bytes at 8 TB/s, both products' flops
        # at the matrix-core peak)
        if ran == "f64_batched" and fam.get("gemm_n", (0, 0, 0))[1] > 0:
            loop = [f for f in ("gemm_n", "gemm_t", "trmv", "trmv_t", "lr_apply", "vec") if f in fam]
            it_ms = sum(fam[f][0] for f in loop) / fam["gemm_n"][1]
            bytes_it = a_bytes + sum(per_launch.get(f, 0) for f in ("trmv", "trmv_t", "lr_apply"))
            flops_it = 2.0 * flops_launch["gemm_n"]
            pk = FP64_PEAK_TFS
            bound_ms = max(bytes_it / (HBM_PEAK_GBS * 1e9), flops_it / (pk * 1e12)) * 1e3
            roof["iteration"] = {"ms": round(it_ms, 4), "bound_ms": round(bound_ms, 4),
                                 "frac": round(bound_ms / it_ms, 4), "families": loop,
                                 "bytes": int(bytes_it), "flops": flops_it}

    # ---- per-problem latency of a batch, measured: one more (untimed) step with the
    # library recording, on the device's constant-rate clock, when each (problem,
    # lambda) solve stopped; a problem is done when its last lambda stops.  Its
    # preconditioner is ready when the batched sketch and preconditioner stages end
    # (events around them in the same step).  The mixed refinement is not timed per
    # lambda, so a mixed-mode workload is measured on its batched FP64 solve.
    latency, latency_mode = None, None
    if len(plist) > 1:
        lat_mode = mode if mode != tik.MIXED_BATCHED else tik.F64_BATCHED
        tik.set_option("record_times", 1)
        try:
            lm = []
            one_step(lat_mode, tol if lat_mode == mode else f64_tol, lm)
            torch.cuda.synchronize()
            tms = tik.lsqr_times(len(plist), lams.shape[1])
        finally:
            tik.set_option("record_times", 0)
        ready = lm[0].elapsed_time(lm[2])
        lat = ready + np.nanmax(tms, axis=1)
        latency = [round(float(np.percentile(lat, 50)), 2), round(float(np.percentile(lat, 99)), 2)]
        latency_mode = {tik.F64_BATCHED: "f64_batched", tik.MIXED_BATCHED: "mixed_batched"}[lat_mode]
        log(f"per-problem latency ({latency_mode}): p50 {latency[0]} ms, p99 {latency[1]} ms "
            f"(ready at {ready:.1f} ms, solve loop {np.nanmax(tms):.1f} ms)")

    # ---- matrix-core use of the BF16 Gaussian sketch product (2 s m n flops per
    # problem over the "sketch" family's time: the product and its split-K reduction)
    sketch_mfma = None
    if cfg["embed"] == tik.GAUSS and cfg["sdt"] == tik.BF16 and "sketch" in fam:
        flops = sum(2.0 * p.s * p.m * p.n for p in plist)
        sk_ms = fam["sketch"][0]
        if sk_ms > 0:
            tf = flops / (sk_ms / 1000.0) / 1e12
            sketch_mfma = {"bound": "mfma", "dtype": "bf16", "achieved": round(tf, 1),
                           "peak": BF16_PEAK_TFS, "unit": "TFLOP/s", "frac": round(tf / BF16_PEAK_TFS, 4),
                           "ms_per_step": round(sk_ms, 3), "flops": flops}
            # a batch's per-problem sketches run on several streams at once, which stretches each
            # launch: the stage's wall time gives the rate the whole GPU delivers
            if stage_ms["sketch"] > 0:
                sketch_mfma["stage_tflops"] = round(flops / (stage_ms["sketch"] / 1000.0) / 1e12, 1)

    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "λ-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": cfg["desc"], "mode": ran,
                   "requested_mode": {tik.F64_BATCHED: "f64_batched", tik.MIXED_BATCHED: "mixed_batched"}[mode],
                   "tol": tol, "solves": nsolve, "graph_chunk": tik.get_option("graph_chunk")},
        "roofline": roof,
        "launch_shape": launch_shape,
        "sketch_mfma": sketch_mfma,
        "cpu_baseline": cpu,
        "solves_ok": n_ok,
        "checked": checked,
        "lambdas_fp32_refined": n32,
        "lambdas_fp64": n64,
        "max_rel_err": err_max,
        "iters_max": int(iters.max()),
        "iters_p50_p99": [float(np.percentile(iters.max(axis=1), 50)),
                          float(np.percentile(iters.max(axis=1), 99))] if len(plist) > 1 else None,
        "latency_p50_p99_ms": latency,
        "latency_measured_on": latency_mode,
        "stage_ms_per_step": {k: round(v, 3) for k, v in stage_ms.items()},
        "status_ok": bool(np.all(status <= 1)),
        "phases_ms_per_step": {k: round(v[0], 3) for k, v in fam.items()},
        "launches_per_step": {k: v[1] for k, v in fam.items()},
        "wall_s_timed": round(wall, 3),
        "lcurve": lc,
    }
    # the FP64 legs: value counts solves within 1e-8 (the metric), value_f64 those
    # within the FP64 target 1e-10 that their tolerance is chosen for
    if plain is not None:
        sec = plain["ms_per_step"] / 1000.0
        pv = plain.get("n_ok", 0) / sec
        line["plain_f64_per_lambda"] = {"value": round(pv, 3), "value_f64": round(plain.get("n_ok_f64", 0) / sec, 3),
                                        "ms_per_step": round(plain["ms_per_step"], 2), "tol": plain["tol"],
                                        "max_rel_err": plain.get("max_rel_err"),
                                        "iters_max": int(plain["iters"].max())}
        line["speedup_vs_plain"] = round(value / pv, 2) if pv > 0 else None
    if alt is not None:
        sec = alt["ms_per_step"] / 1000.0
        av = alt.get("n_ok", 0) / sec
        line["f64_batched"] = {"value": round(av, 3), "value_f64": round(alt.get("n_ok_f64", 0) / sec, 3),
                               "ms_per_step": round(alt["ms_per_step"], 2), "tol": alt["tol"],
                               "solves_ok": alt.get("n_ok"), "solves_ok_f64": alt.get("n_ok_f64"),
                               "max_rel_err": alt.get("max_rel_err"), "iters_max": int(alt["iters"].max())}
        if plain is not None and plain.get("n_ok_f64"):
            pf = plain["n_ok_f64"] / (plain["ms_per_step"] / 1000.0)
            line["f64_batched_vs_plain_at_1e-10"] = round(line["f64_batched"]["value_f64"] / pf, 2)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
