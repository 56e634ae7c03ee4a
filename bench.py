"""Benchmark: time-step solves per second of MGRIT with p-multigrid spatial solves, run to a 1e-10
relative MGRIT residual, on one MI355X.

Workload (synthetic, seeded): the 2D heat equation on the unit square, kappa 1, T 0.1, N_t 1024,
h 2^-6, B-spline degrees p = 3, 4 and 5 batched as three instances of one solver handle, source
8 random sin-sin modes (seed 2107), u0 = 0, MGRIT m 8 with levels 1024 -> 128 -> 16 -> 2, ILUT
(tau 1e-12, fill = nnz of A), exact p = 1 solve, spatial tolerance 1e-12.  One step = one full
MGRIT solve of all three instances from the zero initial iterate to the 1e-10 residual.

Variants: plain FP64 V-cycles; FP32 V-cycles inside FP64 iterative refinement; "tuned":
FP32-refined with the autotuned LDS placement, the HIP-graph-captured iteration and coarse-level
spatial solves to 1e-4 (level 0 stays at 1e-12); and that with the learned warm start.
`value` is the fastest variant (all reach the same 1e-10 residual).  The network of the learned
variant is trained first (not timed) on sequential solver trajectories of other sources.  The
dominant kernel's roofline uses HIP events the library records around each of its launches on
the solve stream (around each captured iteration in graph mode).  The CPU baseline times the
oracle (single thread) on a bounded sample.

--c4: the learned-warm-start measurement at p = 3, h 2^-6, N_t 4096: a network trained on 64
sequential trajectories (sources seeded 0..63), then sequential solves of four unseen sources
(seeds 1000..1003) with the zero, previous-step and learned guesses (V-cycles and time).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-step solves/s at 1e-10 MGRIT residual: FP64 vs FP32-refined+learned"
WORKLOAD = ["heat-p3-h64-Nt1024", "heat-p4-h64-Nt1024", "heat-p5-h64-Nt1024"]
HBM_PEAK_GBS = 8000.0
RHS_PER_BATCH = 128  # level-0 F-sweep width (N_t / m)


def make(precision: int, guess: int = 2, autotune: int = 0, graph: int = 0, coarse_tol: float = 0.0,
         lds_mask: int = 0):
    import paper_2107_05337_amd as pm
    from paper_2107_05337_amd import workloads as W

    cfgs = [W.config(n) for n in WORKLOAD]
    insts = [c["instances"][0] for c in cfgs]
    probs = [pm.problem(d["p"], d["n"], d["Nt"], d["kappa"], d["T"], d["domain"]) for d in insts]
    mo = pm.default_mgrit_opts(cfactor=8, max_levels=12, coarsest_max=8, tol=1e-10, use_graph=graph)
    so = pm.default_solver_opts(precision=precision, guess=guess, autotune=autotune, coarse_tol=coarse_tol,
                                lds_mask=lds_mask)
    S = pm.Solver(probs, mo, so, device=0)
    for i, d in enumerate(insts):
        S.set_source(i, d["src"], d["tkind"])
    return S, insts


def train_network(n_src: int = 4, epochs: int = 8, batch: int = 64, lr: float = 2e-3):
    """Warm-start network for the benchmark's degrees: sequential FP64 trajectories of n_src other
    sources per degree (seeds 0..n_src-1) at the benchmark's h and N_t, then Adam training."""
    import paper_2107_05337_amd as pm
    from paper_2107_05337_amd import workloads as W

    t0 = time.perf_counter()
    base = [W.config(n)["instances"][0] for n in WORKLOAD]
    probs, srcs = [], []
    for d in base:
        for k in range(n_src):
            probs.append(pm.problem(d["p"], d["n"], d["Nt"], d["kappa"], d["T"], d["domain"]))
            srcs.append(W.random_modes(k))
    T = pm.Solver(probs, pm.default_mgrit_opts(), pm.default_solver_opts(guess=1), device=0)
    for i, src in enumerate(srcs):
        T.set_source(i, src, 0)
    U, _ = T.solve_sequential()
    t1 = time.perf_counter()
    T.net_load(W.net_init(0).astype("float32"))
    st = T.net_train(U, epochs=epochs, batch=batch, lr=lr, seed=1)
    theta = T.net_save()
    T.close()
    del U
    info = dict(trajectories=len(probs), samples=len(probs) * base[0]["Nt"], epochs=epochs, batch=batch,
                data_s=round(t1 - t0, 2), train_s=round(st["seconds"], 2), loss_first=st["loss_first"],
                loss_last=st["loss_last"], adam_steps=st["adam_steps"])
    return theta, info


def unit_bytes(S, inst: int, precision: int) -> float:
    """Algorithmic bytes of one V-cycle on one right-hand side: the vector traffic
    of an unfused V-cycle, 26 n_dof + 6 n_dof1 words, plus the matrices one V-cycle streams
    (A three times, the ILUT factors L and U twice, P twice, the p = 1 fast-diagonalisation data
    twice) amortised over the 128 right-hand sides of a level-0 F-sweep."""
    nd, _, _ = S.dims(inst)
    p = S.problems[inst]
    n1 = p.n_elems - 1
    nd1 = n1 * n1
    w = 8 if precision == 0 else 4          # V-cycle word size
    mw = 12 if precision == 0 else 8        # V-cycle matrix bytes per non-zero (value + index)
    nnzA = S.host_matrix("A", inst).nnz
    nnzL = S.host_matrix("L", inst).nnz
    nnzU = S.host_matrix("U", inst).nnz
    nnzP = S.host_matrix("P", inst).nnz
    vec = (6 * nd) * 8 + (20 * nd + 6 * nd1) * w   # outer FP64 residual / update + V-cycle vectors
    mat = 12 * nnzA + mw * (2 * nnzA + 2 * (nnzL + nnzU) + 2 * nnzP) + 8 * 4 * n1 * n1
    return vec + mat / RHS_PER_BATCH


def run_variant(precision: int, steps: int, warmup: int, guess: int = 2, autotune: int = 0, graph: int = 0,
                coarse_tol: float = 0.0, theta=None, lds_mask: int = 0):
    import torch

    S, insts = make(precision, guess, autotune, graph, coarse_tol, lds_mask)
    if theta is not None:
        S.net_load(theta)
    outs = S.alloc_trajectories()
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        S.solve_mgrit(outs, stream)
    S.profile(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(steps):
        _, st = S.solve_mgrit(outs, stream)
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = S.profile(0)
    nsteps_total = sum(d["Nt"] for d in insts)
    sec_per_step = (t1 - t0) / steps
    ub = [unit_bytes(S, i, precision) for i in range(len(insts))]
    w = [S.dims(i)[0] for i in range(len(insts))]
    ubar = sum(a * b for a, b in zip(ub, w)) / sum(w)
    res = dict(value=nsteps_total / sec_per_step, ms_per_step=1e3 * sec_per_step,
               mgrit_iters=stats[-1]["mgrit_iters"], vcycles_per_solve=stats[-1]["vcycles"],
               phi_calls=stats[-1]["phi_calls"], kernel_ms=prof["ms"], launches=prof["launches"],
               unit_bytes=ubar, units=prof["vcycles"], lds_masks=[S.group_info(i)["lds_mask"] for i in range(S.n)],
               lds_masks_wide=[S.group_info(i)["lds_mask_wide"] for i in range(S.n)])
    final = [o.clone() for o in outs]
    S.close()
    return res, final


def cpu_baseline(iters: int):
    """Oracle MGRIT (plain C, one thread) on the p = 3 instance, one iteration timed (two
    FCF-relaxations with their residuals and one coarse cycle), scaled to a full solve."""
    import numpy as np

    import oracle as O
    from paper_2107_05337_amd import workloads as W

    d = W.config(WORKLOAD[0])["instances"][0]
    P = O.Problem(d["p"], d["n"], d["domain"])
    F = P.load_vector(d["src"])
    t0 = time.perf_counter()
    r = P.mgrit(d["kappa"], d["T"], d["Nt"], F, d["tkind"], np.zeros(P.ndof), m=8, max_iter=1)
    dt = time.perf_counter() - t0
    # a full solve = (iters + 1) FCF sweeps and iters coarse cycles ~ (iters + 1) / 2 of this sample
    est = dt * (iters + 1) / 2.0
    return dict(value=d["Nt"] / est, unit="time-step solves/s", cores=1, kind="oracle",
                sample=f"oracle MGRIT on {WORKLOAD[0]} (single thread), max_iter=1 timed {dt:.1f} s, "
                       f"scaled by (iters+1)/2 with iters={iters} to a full 1e-10 solve (p=3 is the cheapest "
                       f"instance of the workload, so this over-states the oracle's rate on it); "
                       f"return code {r['rc']} = stopped at max_iter, as the sample intends")


def traffic_for(kernel_src_hash: str):
    path = os.path.join(ROOT, "profiles", "phi_kernel_heat-h64-Nt1024_counters.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("kernel_src_sha1") != kernel_src_hash:
        return None
    return rec


def copy_calibration(mib: int = 512, reps: int = 4):
    """A plain device copy of known size, for scaling rocprofv3's FETCH_SIZE / WRITE_SIZE counters
    (each dispatch reads and writes exactly `mib` MiB)."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_dispatch": n * 4, "dispatches": reps}))


def c4_learned(n_train: int = 64, epochs: int = 4, batch: int = 128, lr: float = 2e-3):
    """Learned warm start at p = 3, h 2^-6, N_t 4096 (sequential stepping)."""
    import numpy as np
    import torch

    import paper_2107_05337_amd as pm
    from paper_2107_05337_amd import workloads as W

    d = W.config("heat-p3-h64-Nt4096")["instances"][0]
    mk = lambda n, g: pm.Solver([pm.problem(d["p"], d["n"], d["Nt"], d["kappa"], d["T"], d["domain"])] * n,
                                pm.default_mgrit_opts(), pm.default_solver_opts(guess=g), device=0)
    t0 = time.perf_counter()
    T = mk(n_train, 1)
    for i in range(n_train):
        T.set_source(i, W.random_modes(i), 0)
    U, st = T.solve_sequential()
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    T.net_load(W.net_init(0).astype(np.float32))
    tr = T.net_train(U, epochs=epochs, batch=batch, lr=lr, seed=1)
    theta = T.net_save()
    T.close()
    del U
    torch.cuda.empty_cache()
    res = {}
    ref = None
    for g, name in ((0, "zero"), (1, "previous"), (3, "learned")):
        S = mk(4, g)
        for i in range(4):
            S.set_source(i, W.random_modes(1000 + i), 0)
        if g == 3:
            S.net_load(theta)
        outs = S.alloc_trajectories()
        S.solve_sequential(outs)  # warm-up
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, sts = S.solve_sequential(outs)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        if ref is None:
            ref = [o.clone() for o in outs]
        diff = max(float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) for a, b in zip(outs, ref))
        res[name] = dict(vcycles=sts["vcycles"], solves=sts["phi_calls"], seconds=round(dt, 3),
                         vcycles_per_solve=round(sts["vcycles"] / sts["phi_calls"], 3), rel_diff_vs_zero=diff)
        S.close()
    return {"experiment": "learned warm start, sequential implicit Euler, p=3 h=2^-6 N_t=4096",
            "training": dict(trajectories=n_train, samples=n_train * d["Nt"], data_s=round(t_data, 2),
                             epochs=epochs, batch=batch, adam_steps=tr["adam_steps"], train_s=round(tr["seconds"], 2),
                             loss_first=tr["loss_first"], loss_last=tr["loss_last"]),
            "evaluation": "4 unseen sources (seeds 1000..1003), one handle, spatial tol 1e-12", "guesses": res}


NET_MACS_PER_PIXEL = 9 * (3 * 32 + 32 * 32 + 32 * 32 + 32 * 1)
BF16_PEAK_TFLOPS = 2500.0


def net_bench(nb: int = 256, G: int = 67, reps: int = 20):
    """Throughput of the warm-start network kernels on a batch of nb samples of a G x G grid:
    inference and loss gradient (forward + backward), HIP-event timed on the current stream."""
    import numpy as np
    import torch

    import paper_2107_05337_amd as pm
    from paper_2107_05337_amd import workloads as W

    S = pm.Solver([pm.problem(3, G - 3, 8)], pm.default_mgrit_opts(), pm.default_solver_opts(), device=0)
    S.net_load(W.net_init(0).astype(np.float32))
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn((nb, 3, G, G), generator=g, device="cuda")
    t = torch.randn((nb, G, G), generator=g, device="cuda")
    y = torch.empty((nb, G, G), device="cuda")
    fwd = 2.0 * NET_MACS_PER_PIXEL * G * G * nb
    out = {}
    for name, fn, flops in (("forward", lambda: S.net_forward(x, y), fwd),
                            ("forward+backward", lambda: S.net_grad(x, t), 3.0 * fwd)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = dict(ms=round(ms, 4), tflops=round(flops / ms * 1e-9, 2),
                         frac_bf16_peak=round(flops / ms * 1e-9 / BF16_PEAK_TFLOPS, 5))
    S.close()
    return {"experiment": "warm-start network kernels", "batch": nb, "grid": G,
            "flop_per_sample_forward": 2 * NET_MACS_PER_PIXEL * G * G, "peak_tflops_bf16": BF16_PEAK_TFLOPS,
            "note": "forward+backward counted as 3x forward (the first layer's input gradient is not formed); "
                    "net_grad also copies the gradient to the host",
            "results": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--variants", default="fp64,fp64+tuned,fp32,fp32+tuned,fp32+learned")
    ap.add_argument("--c4", action="store_true", help="run the learned-warm-start measurement instead")
    ap.add_argument("--net", action="store_true", help="time the network kernels instead")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 512 MiB device copy (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.c4:
        print(json.dumps(c4_learned()))
        return
    if args.net:
        print(json.dumps(net_bench()))
        return
    specs = {"fp64": dict(precision=0), "fp64+tuned": dict(precision=0, autotune=1, graph=1, coarse_tol=1e-4),
             "fp32": dict(precision=1),
             "fp32+tuned": dict(precision=1, autotune=1, graph=1, coarse_tol=1e-4),
             "fp32+learned": dict(precision=1, guess=3, autotune=1, graph=1, coarse_tol=1e-4)}
    variants = {}
    finals = {}
    for v in args.variants.split(","):
        kw = dict(specs[v])
        if kw.get("guess") == 3:
            theta, tinfo = train_network()
            print(f"# network: {tinfo}", file=sys.stderr, flush=True)
            kw["theta"] = theta
        res, fin = run_variant(steps=args.steps, warmup=args.warmup, **kw)
        res["coarse_tol"] = kw.get("coarse_tol", 0.0) or 1e-12
        if kw.get("guess") == 3:
            res["training"] = tinfo
        variants[v] = res
        finals[v] = fin
        print(f"# {v}: {res['value']:.1f} time-step solves/s, {res['ms_per_step']:.1f} ms/step, "
              f"iters {res['mgrit_iters']}, V-cycles {res['vcycles_per_solve']}", file=sys.stderr, flush=True)
    if "fp64" in finals:
        den = sum(float(torch.linalg.norm(b)) ** 2 for b in finals["fp64"])
        for v in finals:
            if v != "fp64":
                num = sum(float(torch.linalg.norm(a - b)) ** 2 for a, b in zip(finals[v], finals["fp64"]))
                variants[v]["rel_diff_vs_fp64"] = (num / den) ** 0.5
    head = max(variants, key=lambda k: variants[k]["value"])
    b = variants[head]
    achieved = b["units"] * b["unit_bytes"] / (b["kernel_ms"] * 1e-3) / 1e9
    src = open(os.path.join(ROOT, "paper_2107_05337_amd", "csrc", "phi_kernels.hip"), "rb").read()
    tr = traffic_for(hashlib.sha1(src).hexdigest())
    traffic = None
    f64 = head.startswith("fp64")
    if tr is not None and tr.get("precision") == ("fp64" if f64 else "fp32"):
        traffic = tr.get("hbm_bytes_per_launch")
    roof = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic,
            "kernel": f"phi_kernel<{'double' if f64 else 'float'}>",
            "avg_launch_ms": round(b["kernel_ms"] / max(b["launches"], 1), 4),
            "bytes_per_unit": round(b["unit_bytes"])}
    out = {"metric": METRIC, "value": round(b["value"], 3), "unit": "time-step solves/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(b["ms_per_step"], 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if f64 else "f32-vcycle-in-f64-refinement", "data": "synthetic",
           "config": {"workload": "heat-h64-Nt1024-p3,p4,p5 (3 instances batched)", "variant": head,
                      "N_t": 1024, "h": "2^-6", "p": [3, 4, 5], "m": 8, "levels": [1024, 128, 16, 2],
                      "mgrit_tol": 1e-10, "spatial_tol": 1e-12},
           "roofline": roof, "variants": variants}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(variants.get("fp64", b)["mgrit_iters"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
