#!/usr/bin/env python3
"""Time-to-s-eigenpairs of A X = B X Lambda on one MI355X (variant KI:
Cholesky, Lanczos on C = U^-T A U^-1 with TRSV/SYMV/TRSV per step and full
re-orthogonalisation, Ritz vectors, back-solve, FP64 check).

One step = restore B (the solve overwrites it with U, a device-to-device
copy) + one gsyeig_solve on a known-spectrum instance already resident in
HBM.  Prints ONE JSON line on stdout; progress goes to stderr.

  python bench.py [--steps K] [--warmup W] [--config 1]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CONFIGS = {
    0: dict(n=512, s=10, law="spaced", label="known-spectrum pencil n=512 s=10, FP64 single-vector KI"),
    1: dict(n=16384, s=100, law="spaced", label="known-spectrum pencil n=16384 s=100, FP64 single-vector KI"),
    2: dict(n=32768, s=200, law="clustered", prec="mixed",
            label="known-spectrum pencil n=32768 s=200, clustered spectrum, mixed FP32 sweeps + FP64 refinement"),
    3: dict(n=65536, s=800, law="spaced", prec="mixed", block=32,
            label="known-spectrum pencil n=65536 s=800 with eigenvectors Y = I - 2 Q Q^T (Q orthonormal, rank 256) "
                  "+ 1-D FEM pencil (inverse pencil), block Lanczos, mixed FP32 block products + FP64 refinement"),
    4: dict(n=0, s=0, law="spaced", label="batched known-spectrum pencils, n ~ U{256..4096}, s = ceil(0.05 n)"),
}
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def measured_traffic(kernel, n, prec):
    """HBM bytes per launch of `kernel` from a committed counter summary under
    profiles/ (two calibrated rocprofv3 --pmc passes), or None when there is
    none for this size or the kernel's sources changed since it was taken."""
    import glob
    import hashlib
    import re

    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for m in re.finditer(r"<!-- traffic (.*?) -->", open(f).read()):
            kv = dict(item.split("=", 1) for item in m.group(1).split())
            if kv.get("kernel") != kernel or int(kv.get("n", -1)) != n or kv.get("prec") != prec:
                continue
            h = hashlib.sha256()
            srcs = [os.path.join(ROOT, src) for src in kv["sources"].split(",")]
            if not all(os.path.exists(f) for f in srcs):
                continue  # the measured kernel's sources are gone: its counters no longer apply
            for f in srcs:
                h.update(open(f, "rb").read())
            if h.hexdigest()[:16] == kv.get("sha256_16"):
                return float(kv["bytes_per_launch"])
    return None


def sweep_kernels(kind, block=512):
    """(KI1 kernel, KI3 kernel) of sweep kind `kind` (gsyeig_set_trsv_sweep:
    0 both work queues, 1 both one workgroup per tile, 2 per-tile KI1 and
    queue KI3, 3 the reverse); block 64 runs the 64-row chains."""
    if block == 64:
        return "k_trsv_n", "k_trsv_t"
    return ("k_trsvq_n" if kind in (0, 3) else "k_trsv_w_n"), ("k_trsvq_t" if kind in (0, 2) else "k_trsv_w_t")


def sweep_traffic(kind, block, n, prec):
    """Mean measured HBM bytes per launch of the two sweep kernels (None if
    either has no current counter summary)."""
    a, b = sweep_kernels(kind, block)
    ta, tb = measured_traffic(a, n, prec), measured_traffic(b, n, prec)
    return None if ta is None or tb is None else 0.5 * (ta + tb)


def cpu_baseline(n_target, law="spaced", sizes=(768, 1024, 1536, 2048)):
    """The oracle (plain C, FP64) on a bounded sample: full solves of the same
    generator at a few sizes (s = ceil(0.006 n), the config's ratio), a
    least-squares fit of log t = log c + e log n over them, extrapolated to
    n_target.  Every stage is O(n^3), so e should come out close to 3; the
    fitted exponent is reported with the sample."""
    import gen
    import numpy as np
    import oracle

    oracle.lib()
    ts = []
    for n in sizes:
        s = max(1, math.ceil(0.006 * n))
        d = gen.known_spectrum(n, law, seed=gen.BASE_SEED, stream=(1, 0, 99, n))
        t0 = time.perf_counter()
        oracle.gsyeig(d["A"], d["B"], s)
        ts.append(time.perf_counter() - t0)
    e, logc = np.polyfit(np.log(np.array(sizes, dtype=float)), np.log(np.array(ts)), 1)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    pts = ", ".join(f"n={n}: {t:.2f} s" for n, t in zip(sizes, ts))
    return {"value": float(math.exp(logc) * n_target ** e), "unit": "s", "cores": threads, "kind": "oracle",
            "extrapolated": True,
            "sample": f"full oracle solves of the same generator ({pts}); fit t = c n^e gives e = {e:.2f}, "
                      f"extrapolated to n={n_target}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=1, choices=sorted(CONFIGS))
    ap.add_argument("--profile-every", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--instances", type=int, default=512, help="instances for --config 4")
    ap.add_argument("--streams", type=int, default=16, help="worker streams for --config 4")
    ap.add_argument("--n", type=int, default=0, help="override n (exploration; the config label then says so)")
    ap.add_argument("--s", type=int, default=0, help="override s")
    ap.add_argument("--no-fp64-compare", action="store_true", help="--config 2: skip the FP64 solve")
    ap.add_argument("--block", type=int, default=0,
                    help="Lanczos block size (--config 3: default 32; --config 2/4: default 1, single-vector)")
    ap.add_argument("--prec", type=int, default=-1,
                    help="--config 4: 0 = FP64, 1 = mixed (default: mixed, the configuration's precision)")
    ap.add_argument("--no-loop", action="store_true", help="--config 4: skip the loop of single FP64 solves")
    ap.add_argument("--refine-inner", type=int, default=0, help="MINRES steps per refinement round (0 = default)")
    ap.add_argument("--basis", type=int, default=0, help="--config 3: basis size before a restart (0 = auto)")
    ap.add_argument("--acc32", type=int, default=0, help="--config 3: 1 = FP32 accumulation in block products")
    ap.add_argument("--no-fem", action="store_true", help="--config 3: skip the FEM pencil")
    ap.add_argument("--fem-only", action="store_true", help="--config 3: only the FEM pencil")
    ap.add_argument("--fem-prec", type=int, default=1, help="--config 3: FEM pencil precision (0 FP64, 1 mixed)")
    ap.add_argument("--eta-tol", type=float, default=0.0, help="refinement target (0 = library default)")
    ap.add_argument("--reorth", type=int, default=-1,
                    help="re-orthogonalisation: 0 twice, 1 second pass when needed, 2 partial (-1 = default)")
    ap.add_argument("--variant", choices=["ki", "ke"], default="ki",
                    help="configs 0/1: the timed variant (KI: implicit operator, the default; KE: explicit C)")
    ap.add_argument("--no-ke", action="store_true", help="configs 0/1: skip the KE solve timed beside KI")
    ap.add_argument("--no-autotune", action="store_true",
                    help="configs 0/1: keep the library's default kernel choices (no gsyeig_autotune)")
    ap.add_argument("--tune-cache", default="", help="JSON cache file for gsyeig_autotune")
    ap.add_argument("--no-config2", action="store_true",
                    help="config 1: skip the mixed-vs-FP64 comparison on the n = 32768 clustered pencil")
    ap.add_argument("--trsv-sweep", type=int, default=-1,
                    help="super-block sweep kernels (gsyeig_set_trsv_sweep): 0 work queue, 1 one workgroup per tile")
    ap.add_argument("--sweep-s", default="",
                    help="comma-separated s values: time the variants (--sweep-variants) against s on the config's "
                         "input (the shape of the paper's Figs. 1-2); one JSON line per point, no headline line")
    ap.add_argument("--sweep-variants", default="ki,ke,td", help="variants of --sweep-s")
    ap.add_argument("--gemm-only", action="store_true",
                    help="run only GS2 (form C) and GS1 at the config's n (FP64), for MFMA counter passes; no JSON")
    ap.add_argument("--trsv-only", action="store_true",
                    help="run only KI1/KI3 at the config's n on a random factor, plus a device copy of n^2 doubles "
                         "(the fixed-size reference kernel for hardware byte counters); prints timings, no JSON")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only: the solver runs on a single MI355X "
              f"(requested --gpus {args.gpus}, WORLD_SIZE {world}); multi-GPU runs are not part of this build.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_1111_6374_amd as gs

    cfg = dict(CONFIGS[args.config])
    if args.trsv_only:
        return trsv_only(args, cfg)
    if args.gemm_only:
        return gemm_only(args, cfg)
    if args.n or args.s:
        cfg["n"] = args.n or cfg["n"]
        cfg["s"] = args.s or cfg["s"]
        cfg["label"] += f" (reduced to n={cfg['n']} s={cfg['s']})"
    if args.sweep_s:
        return bench_sweep(args, cfg)
    if args.config == 4:
        return bench_batched(args, cfg)
    if args.config == 2:
        return bench_mixed(args, cfg)
    if args.config == 3:
        return bench_block(args, cfg)
    n, s = cfg["n"], cfg["s"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"generating n={n} s={s} law={cfg['law']}")
    t0 = time.perf_counter()
    inst = gen.known_spectrum_device(n, cfg["law"], seed=gen.BASE_SEED + args.config,
                                     stream=(args.config, 0, 0), device=dev, keep_factors=False)
    A, B0 = inst["A"], inst["B"]
    lam_true = np.sort(inst["lam"])[:s]
    B = torch.empty_like(B0)
    torch.cuda.synchronize()
    log(f"generated in {time.perf_counter() - t0:.1f} s")

    solver = gs.Solver()
    tuning = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        rc, tu = gs.gsyeig_autotune(solver.ctx, n, gs.GSYEIG_FP64, args.tune_cache or None)
        if rc:
            raise gs.GsyeigError("gsyeig_autotune", rc)
        tuning = tu.as_dict()
        log(f"autotune ({time.perf_counter() - t0:.1f} s): {tuning}")
    if args.trsv_sweep >= 0:
        rc = gs.gsyeig_set_trsv_sweep(solver.ctx, args.trsv_sweep)
        if rc:
            raise gs.GsyeigError("gsyeig_set_trsv_sweep", rc)
    kind = args.trsv_sweep if args.trsv_sweep >= 0 else (tuning["trsv_sweep"] if tuning else 0)
    kblock = tuning["trsv_block"] if tuning and args.trsv_sweep < 0 else 512
    opts = gs.gsyeig_opts_default()
    opts.profile_every = args.profile_every
    if args.reorth >= 0:
        opts.reorth = args.reorth
    if args.block > 1:
        opts.block = args.block
    opts.variant = gs.GSYEIG_KE if args.variant == "ke" else gs.GSYEIG_KI
    if args.variant == "ke":
        cfg["label"] = cfg["label"].replace("single-vector KI", "single-vector KE (explicit C)")
    Lam = torch.empty(s, dtype=torch.float64, device=dev)
    X = torch.empty(s, n, dtype=torch.float64, device=dev)

    def step(o=opts):
        B.copy_(B0)
        rc, info = gs.gsyeig_solve(solver.ctx, n, s, A, n, B, n, o, Lam, X, n)
        if rc:
            raise gs.GsyeigError("gsyeig_solve", rc)
        return info

    for w in range(args.warmup):
        info = step()
        log(f"warmup {w}: {info.t_total_ms:.1f} ms, steps={info.steps}, reorth_steps={info.reorth_steps}")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        infos.append(step())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    for k, inf in enumerate(infos):
        log(f"step {k}: total {inf.t_total_ms:.1f} ms (GS1 {inf.t_gs1_ms:.1f}, GS2 {inf.t_gs2_ms:.1f}, "
            f"loop {inf.t_ki_ms:.1f}, KI5 {inf.t_ki5_ms:.1f}, BT1 {inf.t_bt1_ms:.1f}, check {inf.t_check_ms:.1f}) "
            f"m={inf.steps}")

    # parity against the generator's known spectrum and the device FP64 check
    lam = Lam.cpu().numpy()
    e_lam = float(np.max(np.abs(lam - lam_true)) / np.max(np.abs(inst["lam"])))
    last = infos[-1]

    # the other variant on the same input, timed beside the headline one
    other = None
    if not args.no_ke and opts.block == 1:
        o2 = gs.gsyeig_opts_default()
        o2.profile_every = args.profile_every
        o2.reorth = opts.reorth
        o2.variant = gs.GSYEIG_KI if opts.variant == gs.GSYEIG_KE else gs.GSYEIG_KE
        name = "KI" if o2.variant == gs.GSYEIG_KI else "KE"
        step(o2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        oi = [step(o2) for _ in range(2)]
        torch.cuda.synchronize()
        t_other = (time.perf_counter() - t0) / 2
        lam2 = Lam.cpu().numpy()
        i2 = oi[-1]
        sm = sum(i.prof_samples for i in oi)
        other = {"variant": name, "time_s": t_other, "steps": int(i2.steps),
                 "stages_ms": {"gs1": i2.t_gs1_ms, "gs2": i2.t_gs2_ms, "loop": i2.t_ki_ms, "ki5": i2.t_ki5_ms,
                               "bt1": i2.t_bt1_ms, "check": i2.t_check_ms},
                 "op_ms_per_step": i2.t_ki_ms / max(i2.steps, 1),
                 "symv_ms": sum(i.t_ki2_ms_sum for i in oi) / max(sm, 1),
                 "e_lambda_vs_known": float(np.max(np.abs(lam2 - lam_true)) / np.max(np.abs(inst["lam"]))),
                 "eta_max": i2.eta_max}
        log(f"{name} beside: {t_other * 1e3:.1f} ms per solve (GS2 {i2.t_gs2_ms:.1f} ms, loop {i2.t_ki_ms:.1f} ms, "
            f"m={i2.steps}), eta={i2.eta_max:.2e}")

    # dominant kernels: sampled per-launch durations inside the timed solves
    samples = sum(i.prof_samples for i in infos)
    t1 = sum(i.t_ki1_ms_sum for i in infos) / max(samples, 1)
    t2 = sum(i.t_ki2_ms_sum for i in infos) / max(samples, 1)
    t3 = sum(i.t_ki3_ms_sum for i in infos) / max(samples, 1)
    tri_bytes = 8.0 * n * (n + 1) / 2
    vec_bytes = 8.0 * 2 * n
    trsv_ms = 0.5 * (t1 + t3)
    trsv_gbs = (tri_bytes + vec_bytes) / (trsv_ms * 1e-3) / 1e9 if trsv_ms > 0 else None
    symv_gbs = (tri_bytes + vec_bytes) / (t2 * 1e-3) / 1e9 if t2 > 0 else None

    ke = opts.variant == gs.GSYEIG_KE
    if ke:  # the dominant kernel of KE is the SYMV with the explicit C (full read of the tile triangle)
        sy_ms = t2
        sy_gbs = (tri_bytes + vec_bytes) / (sy_ms * 1e-3) / 1e9 if sy_ms > 0 else None
    out = {
        "metric": "time-to-s-eigenpairs",
        "value": ms_per_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["label"], "n": n, "s": s, "spectrum": cfg["law"], "prec": "fp64",
                   "block": int(opts.block), "lanczos_steps": int(last.steps), "reorth": int(opts.reorth),
                   "reorth_steps": int(last.reorth_steps), "parallelism": "single-gpu"},
        "roofline": ({"bound": "hbm", "achieved": sy_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": (sy_gbs / HBM_PEAK_GBS) if sy_gbs else None,
                      "traffic": measured_traffic("k_symv_tiles_q", n, "fp64"),
                      "kernel": "k_symv_tiles_q + k_symv_reduce (KE's SYMV with C; traffic: the tile pass)",
                      "avg_launch_ms": sy_ms,
                      "algorithmic_bytes_per_launch": tri_bytes + vec_bytes} if ke else
                     {"bound": "hbm", "achieved": trsv_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": (trsv_gbs / HBM_PEAK_GBS) if trsv_gbs else None,
                      "traffic": sweep_traffic(kind, kblock, n, "fp64"),
                      "kernel": "%s/%s (KI1/KI3, mean of the two)" % sweep_kernels(kind, kblock),
                      "avg_launch_ms": trsv_ms, "algorithmic_bytes_per_launch": tri_bytes + vec_bytes}),
        "kernels": ({"symv_ms": t2, "symv_GBs": symv_gbs, "samples": samples} if ke else
                    {"ki1": sweep_kernels(kind, kblock)[0], "ki1_ms": t1, "ki3": sweep_kernels(kind, kblock)[1],
                     "ki3_ms": t3, "trsv_ms": trsv_ms, "trsv_GBs": trsv_gbs, "symv_tile_pass_ms": t2,
                     "symv_tile_pass_GBs": symv_gbs, "samples": samples,
                     "note": "KI2 is timed as its tile pass; its reduction runs inside KI3 (trsv_ms)"}),
        "stages_ms": {"gs1": last.t_gs1_ms, "gs2": last.t_gs2_ms, "loop": last.t_ki_ms, "ki5": last.t_ki5_ms,
                      "bt1": last.t_bt1_ms, "check": last.t_check_ms, "total": last.t_total_ms},
        "parity": {"e_lambda_vs_known": e_lam, "eta_max": last.eta_max, "omega": last.omega,
                   "rho_F": last.rho_f, "pass": bool(e_lam <= 1e-10 and last.eta_max <= 1e-10)},
    }
    out["config"]["variant"] = "KE" if ke else "KI"
    if other:
        out["beside"] = other
    if tuning:
        out["tuning"] = tuning
    solver.close()
    if args.config == 1 and not args.no_config2 and not (args.n or args.s):
        del A, B0, B, X, inst
        torch.cuda.empty_cache()
        out["config2"] = config2_comparison(args)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(n)
    print(json.dumps(out), flush=True)


def config2_comparison(args):
    """The metric's comparison, measured once each inside the default run:
    the mixed-precision solve (FP32 sweeps + FP64 refinement) against the
    plain FP64 solve of the same pencil, n = 32768, s = 200, clustered law
    (80 % U[0,1], 20 % U[1,10]); device draws (a different seeded instance
    of the same law than --config 2's host draws).  Time-to-s-eigenpairs
    from the first kernel to the verified pairs, inputs resident in HBM."""
    import numpy as np
    import torch

    import gen
    import paper_1111_6374_amd as gs

    cfg = CONFIGS[2]
    n, s = cfg["n"], cfg["s"]
    dev = torch.device("cuda:0")
    log(f"config 2 comparison: generating n={n} s={s} law={cfg['law']} (device draws)")
    t0 = time.perf_counter()
    inst = gen.known_spectrum_device(n, cfg["law"], seed=gen.BASE_SEED + 2, stream=(2, 1, 0), device=dev,
                                     keep_factors=False, rng_kind="torch")
    A, B0 = inst["A"], inst["B"]
    lam_true = np.sort(inst["lam"])[:s]
    scale = np.max(np.abs(inst["lam"]))
    B = torch.empty_like(B0)
    torch.cuda.synchronize()
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    Lam = torch.empty(s, dtype=torch.float64, device=dev)
    X = torch.empty(s, n, dtype=torch.float64, device=dev)
    res = {"workload": f"known-spectrum pencil n={n} s={s}, clustered spectrum (device draws)", "n": n, "s": s}
    with gs.Solver() as sv:
        for name, prec in (("mixed", gs.GSYEIG_MIXED), ("fp64", gs.GSYEIG_FP64)):
            rc, tu = gs.gsyeig_autotune(sv.ctx, n, prec, args.tune_cache or None)
            if rc:
                raise gs.GsyeigError("gsyeig_autotune", rc)
            o = gs.gsyeig_opts_default()
            o.prec = prec
            o.profile_every = args.profile_every
            B.copy_(B0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, inf = gs.gsyeig_solve(sv.ctx, n, s, A, n, B, n, o, Lam, X, n)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if rc:
                raise gs.GsyeigError("gsyeig_solve", rc)
            e_lam = float(np.max(np.abs(Lam.cpu().numpy() - lam_true)) / scale)
            sm = max(inf.prof_samples, 1)
            k1, k2, k3 = inf.t_ki1_ms_sum / sm, inf.t_ki2_ms_sum / sm, inf.t_ki3_ms_sum / sm
            esz = 4.0 if prec == gs.GSYEIG_MIXED else 8.0
            tri = esz * n * (n + 1) / 2 + 16.0 * n
            res[name] = {"time_s": dt, "steps": int(inf.steps), "reorth_steps": int(inf.reorth_steps),
                         "e_lambda_vs_known": e_lam, "eta_max": inf.eta_max, "omega": inf.omega,
                         "stages_ms": {"gs1": inf.t_gs1_ms, "loop": inf.t_ki_ms, "ki5": inf.t_ki5_ms,
                                       "bt1": inf.t_bt1_ms, "refine": inf.t_refine_ms, "check": inf.t_check_ms},
                         "sweeps_ms": {"ki1": k1, "ki2_tile_pass": k2, "ki3": k3},
                         "trsv_hbm_frac": (tri / (0.5 * (k1 + k3) * 1e-3) / 1e9 / HBM_PEAK_GBS) if k1 + k3 > 0
                         else None,
                         "tuning": tu.as_dict()}
            log(f"config 2 {name}: {dt:.2f} s, m={inf.steps}, e_lam={e_lam:.1e}, eta={inf.eta_max:.1e}, "
                f"KI1 {k1:.3f} ms KI3 {k3:.3f} ms")
    res["speedup_mixed_vs_fp64"] = res["fp64"]["time_s"] / res["mixed"]["time_s"]
    res["pass"] = bool(all(res[k]["e_lambda_vs_known"] <= 1e-10 and res[k]["eta_max"] <= 1e-10
                           for k in ("mixed", "fp64")))
    return res


def bench_sweep(args, cfg):
    """Time-to-s-eigenpairs against s for variants KI, KE and TD on one input
    (the known-spectrum pencil of the configuration, FP64): the paper's
    Figs. 1-2 plot the same quantity for its MD and DFT problems, where the
    Krylov variants win for s up to a few per cent of n (Sec. 6).  Each point
    is the median of --steps solves after one untimed solve of the same
    variant and s."""
    import numpy as np
    import torch

    import gen
    import paper_1111_6374_amd as gs

    n = cfg["n"]
    svals = [int(v) for v in args.sweep_s.split(",") if v]
    names = [v.strip().upper() for v in args.sweep_variants.split(",") if v.strip()]
    code = {"KI": gs.GSYEIG_KI, "KE": gs.GSYEIG_KE, "TD": gs.GSYEIG_TD}
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"generating n={n} law={cfg['law']}")
    inst = gen.known_spectrum_device(n, cfg["law"], seed=gen.BASE_SEED + args.config,
                                     stream=(args.config, 0, 0), device=dev, keep_factors=False)
    A, B0 = inst["A"], inst["B"]
    lam_sorted = np.sort(inst["lam"])
    scale = np.max(np.abs(inst["lam"]))
    B = torch.empty_like(B0)
    solver = gs.Solver()
    rows = []
    for s_ in svals:
        Lam = torch.empty(s_, dtype=torch.float64, device=dev)
        X = torch.empty(s_, n, dtype=torch.float64, device=dev)
        for name in names:
            o = gs.gsyeig_opts_default()
            o.variant = code[name]
            times, info = [], None
            for k in range(1 + max(1, args.steps)):
                B.copy_(B0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rc, info = gs.gsyeig_solve(solver.ctx, n, s_, A, n, B, n, o, Lam, X, n)
                torch.cuda.synchronize()
                if rc:
                    raise gs.GsyeigError("gsyeig_solve", rc)
                if k > 0:
                    times.append(time.perf_counter() - t0)
            e_lam = float(np.max(np.abs(Lam.cpu().numpy() - lam_sorted[:s_])) / scale)
            row = {"n": n, "s": s_, "s_over_n": s_ / n, "variant": name, "time_s": float(np.median(times)),
                   "steps": int(info.steps), "gs1_ms": info.t_gs1_ms, "gs2_ms": info.t_gs2_ms,
                   "loop_ms": info.t_ki_ms, "ki5_ms": info.t_ki5_ms, "bt1_ms": info.t_bt1_ms,
                   "e_lambda": e_lam, "eta_max": info.eta_max}
            rows.append(row)
            log(f"s={s_} ({100 * s_ / n:.2f} %) {name}: {row['time_s']:.3f} s (GS2 {info.t_gs2_ms:.0f} ms, "
                f"loop/TD {info.t_ki_ms:.0f} ms, m={info.steps}) e_lam={e_lam:.1e} eta={info.eta_max:.1e}")
            print(json.dumps(row), flush=True)
    solver.close()
    return rows


def trsv_only(args, cfg):
    """KI1 and KI3 alone (no eigen-solve, no QR): the workload of the byte-
    counter passes.  Also one device copy of n^2 FP64 values, whose read and
    written bytes are known exactly, to calibrate the counters.  For the mixed
    configuration the factor is stored FP32 and the FP32-matrix sweeps run."""
    import torch

    import paper_1111_6374_amd as gs

    n = args.n or cfg["n"]
    lp = cfg.get("prec") == "mixed"
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(6374)
    U = torch.triu(torch.randn(n, n, generator=g, device=dev, dtype=torch.float64) / math.sqrt(n), 1)
    U.diagonal().copy_(1.0 + torch.rand(n, generator=g, device=dev, dtype=torch.float64))
    U32 = U.float() if lp else None
    b = torch.randn(n, generator=g, device=dev, dtype=torch.float64)
    x = torch.empty_like(b)
    C = torch.empty_like(U)
    with gs.Solver() as sv:
        if args.trsv_sweep >= 0:
            gs.gsyeig_set_trsv_sweep(sv.ctx, args.trsv_sweep)
        for trans in (0, 1):
            for _ in range(max(1, args.steps)):
                if lp:
                    rc = gs.gsyeig_trsv_lp(sv.ctx, n, U32, n, trans, b, x)
                else:
                    rc = gs.gsyeig_trsv(sv.ctx, n, U, n, trans, b, x)
                if rc:
                    raise gs.GsyeigError("gsyeig_trsv_lp" if lp else "gsyeig_trsv", rc)
        # the whole operator of the Lanczos loop (KI1, KI2's tile pass, KI3
        # summing KI2's partials) on a symmetric A
        A = torch.randn(n, n, generator=g, device=dev, dtype=torch.float64)
        A = A + A.t()
        A32 = A.float() if lp else None
        for _ in range(max(1, args.steps)):
            rc = (gs.gsyeig_apply_op_lp(sv.ctx, n, A32, n, U32, n, b, x) if lp else
                  gs.gsyeig_apply_op(sv.ctx, n, A, n, U, n, b, x))
            if rc:
                raise gs.GsyeigError("gsyeig_apply_op", rc)
        del A, A32
        C.copy_(U)  # reads and writes 8 n^2 bytes
        torch.cuda.synchronize()
    log(f"trsv-only n={n} ({'FP32' if lp else 'FP64'} factor): {2 * max(1, args.steps)} solves, "
        f"{max(1, args.steps)} operator applications and one copy of {8 * n * n} bytes done")


def gemm_only(args, cfg):
    """The matrix-core products alone, for hardware counter passes: GS2
    (C = U^-T A U^-1, two block solves with n right-hand sides) and one GS1
    (Cholesky) at the config's n, FP64."""
    import torch

    import paper_1111_6374_amd as gs

    n = args.n or cfg["n"]
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(6374)
    U = torch.triu(torch.randn(n, n, generator=g, device=dev, dtype=torch.float64) / math.sqrt(n), 1)
    U.diagonal().copy_(1.0 + torch.rand(n, generator=g, device=dev, dtype=torch.float64))
    A = torch.randn(n, n, generator=g, device=dev, dtype=torch.float64)
    A = A + A.t()
    C = torch.empty_like(A)
    with gs.Solver() as sv:
        for _ in range(max(1, args.steps)):
            rc = gs.gsyeig_form_c(sv.ctx, n, A, n, U, n, C, n)
            if rc:
                raise gs.GsyeigError("gsyeig_form_c", rc)
        B = torch.matmul(U.t().contiguous(), U)
        rc = gs.gsyeig_potrf(sv.ctx, n, B, n)
        if rc:
            raise gs.GsyeigError("gsyeig_potrf", rc)
        torch.cuda.synchronize()
    log(f"gemm-only n={n}: {max(1, args.steps)} GS2 and one GS1 done")


def bench_block(args, cfg):
    """Block Lanczos in mixed precision on the known-spectrum pencil (the timed
    workload) and on the 1-D FEM pencil through the inverse pencil (checked
    against its closed form, timed once)."""
    import numpy as np
    import torch

    import gen
    import paper_1111_6374_amd as gs

    n, s = cfg["n"], cfg["s"]
    blk = args.block or cfg["block"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.fem_only:
        return bench_fem(args, cfg, blk)
    t0 = time.perf_counter()
    if n * n >= 2**31:  # row-blocked assembly with Y = I - 2 Q Q^T (no dense n x n QR)
        log(f"generating n={n} s={s} law={cfg['law']} (device draws, row-blocked, Y = I - 2QQ^T)")
        inst = gen.known_spectrum_device_blocked(n, cfg["law"], seed=gen.BASE_SEED + 3, stream=(3, 0, 0),
                                                 device=dev)
    else:
        log(f"generating n={n} s={s} law={cfg['law']} (device draws)")
        inst = gen.known_spectrum_device(n, cfg["law"], seed=gen.BASE_SEED + 3, stream=(3, 0, 0), device=dev,
                                         keep_factors=False, rng_kind="torch")
    A, B0 = inst["A"], inst["B"]
    lam_true = np.sort(inst["lam"])[:s]
    B = torch.empty_like(B0)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    solver = gs.Solver()
    Lam = torch.empty(s, dtype=torch.float64, device=dev)
    X = torch.empty(s, n, dtype=torch.float64, device=dev)

    def opts(**kw):
        o = gs.gsyeig_opts_default()
        o.prec = gs.GSYEIG_MIXED
        o.block = blk
        o.basis = args.basis
        o.block_acc32 = args.acc32
        o.profile_every = args.profile_every
        if args.eta_tol > 0:
            o.eta_tol = args.eta_tol
        if args.refine_inner > 0:
            o.refine_inner = args.refine_inner
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def run(Am, Bm, Bsrc, o):
        if Bsrc is not None:
            gen.copy_rows(Bm, Bsrc)
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc, info = gs.gsyeig_solve(solver.ctx, n, s, Am, n, Bm, n, o, Lam, X, n)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        if rc:
            raise gs.GsyeigError("gsyeig_solve", rc)
        return dt, info

    def show(tag, dt, inf):
        log(f"{tag}: {dt:.2f} s (GS1 {inf.t_gs1_ms:.0f} ms, KI {inf.t_ki_ms:.0f} [projected solves "
            f"{inf.t_rr_ms:.0f} in {inf.rr_count}], KI5 {inf.t_ki5_ms:.0f}, BT1 {inf.t_bt1_ms:.0f}, refine "
            f"{inf.t_refine_ms:.0f}, check {inf.t_check_ms:.0f}) ops={inf.steps} restarts={inf.restarts} "
            f"basis={inf.basis} kept={inf.kept} eta={inf.eta_max:.2e} eta1={inf.eta_phase1:.2e} "
            f"rounds={inf.refine_iters} cluster_fallbacks={inf.cluster_fallbacks} (reason {inf.fallback_reason})")

    for w in range(args.warmup):
        dt, inf = run(A, B, B0, opts())
        show("warmup", dt, inf)
    times, infos = [], []
    for k in range(args.steps):
        dt, inf = run(A, B, B0, opts())
        show(f"step {k}", dt, inf)
        times.append(dt)
        infos.append(inf)
    lam_b = Lam.cpu().numpy()
    mx = float(np.max(np.abs(inst["lam"])))
    e_lam = float(np.max(np.abs(lam_b - lam_true)) / mx)
    value = sum(times) / len(times)
    last = infos[-1]
    samples = sum(i.prof_samples for i in infos)
    t1 = sum(i.t_ki1_ms_sum for i in infos) / max(samples, 1)
    t2 = sum(i.t_ki2_ms_sum for i in infos) / max(samples, 1)
    t3 = sum(i.t_ki3_ms_sum for i in infos) / max(samples, 1)
    # one block application: two triangular block solves (n^2 b flops each)
    # and the symmetric product on the full A~ (2 n^2 b)
    flops = 4.0 * n * n * blk
    t_app = t1 + t2 + t3
    tf = flops / (t_app * 1e-3) / 1e12 if t_app > 0 else None
    peak = 157.3 if args.acc32 else 78.6
    del A, B, B0, inst
    torch.cuda.empty_cache()
    solver.close()
    fem = None if args.no_fem else bench_fem(args, cfg, blk, emit=False)
    out = {
        "metric": "time-to-s-eigenpairs", "value": value, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * value, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": cfg["label"], "n": n, "s": s, "spectrum": cfg["law"], "prec": "mixed",
                   "block": blk, "block_products": "fp32-acc" if args.acc32 else "fp64-acc",
                   "operator_applications": int(last.steps), "restarts": int(last.restarts),
                   "basis": int(last.basis), "kept": int(last.kept), "refine_rounds": int(last.refine_iters),
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "achieved": tf, "peak": peak, "unit": "TFLOP/s",
                     "frac": (tf / peak) if tf else None, "traffic": None,
                     "kernel": "k_gemm (block operator: TRSM, SYMM, TRSM)", "avg_launch_ms": t_app,
                     "algorithmic_flops_per_application": flops},
        "kernels": {"trsm_n_ms": t1, "symm_ms": t2, "trsm_t_ms": t3, "samples": samples},
        "stages_ms": {"gs1": last.t_gs1_ms, "ki_loop": last.t_ki_ms, "projected_solves": last.t_rr_ms,
                      "ki5": last.t_ki5_ms, "bt1": last.t_bt1_ms, "refine": last.t_refine_ms,
                      "check": last.t_check_ms, "total": last.t_total_ms},
        "parity": {"e_lambda_vs_known": e_lam, "eta_max": last.eta_max, "omega": last.omega, "rho_F": last.rho_f,
                   "pass": bool(e_lam <= 1e-10 and last.eta_max <= 1e-10)},
        "fem_inverse_pencil": fem,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, cfg["law"])
    print(json.dumps(out), flush=True)


def bench_fem(args, cfg, blk, emit=True):
    """The 1-D FEM pencil (stiffness, mass) of order n through the inverse
    pencil with block Lanczos, against its closed-form eigenvalues."""
    import numpy as np
    import torch

    import gen
    import paper_1111_6374_amd as gs

    n, s = cfg["n"], cfg["s"]
    dev = torch.device("cuda:0")
    K, M = gen.fem_pencil_device(n, dev)
    lam_ref, _ = gen.fem_eigs(n, s)
    o = gs.gsyeig_opts_default()
    o.prec = args.fem_prec
    o.block = blk
    o.basis = args.basis
    o.block_acc32 = args.acc32
    o.invert = 1
    if args.eta_tol > 0:
        o.eta_tol = args.eta_tol
    Lam = torch.empty(s, dtype=torch.float64, device=dev)
    X = torch.empty(s, n, dtype=torch.float64, device=dev)
    with gs.Solver() as sv:
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc, inf = gs.gsyeig_solve(sv.ctx, n, s, K, n, M, n, o, Lam, X, n)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
    if rc:
        raise gs.GsyeigError("gsyeig_solve", rc)
    lam = Lam.cpu().numpy()
    rel = np.abs(lam - lam_ref) / lam_ref
    j = int(np.argmax(rel))
    # the same errors as seen by the inverse pencil: |d mu| / ||C||, mu = 1/lambda
    dmu = np.abs(1.0 / lam - 1.0 / lam_ref) * lam_ref[0]
    log(f"fem (inverse pencil, prec {args.fem_prec}): {dt:.2f} s (GS1 {inf.t_gs1_ms:.0f} ms, KI {inf.t_ki_ms:.0f} "
        f"[projected solves {inf.t_rr_ms:.0f} in {inf.rr_count}], refine {inf.t_refine_ms:.0f}, check "
        f"{inf.t_check_ms:.0f}) ops={inf.steps} max rel err {rel[j]:.2e} at mode {j + 1} "
        f"(rel err mode 1 {rel[0]:.2e}, mode {s} {rel[-1]:.2e}), max |dmu|/||C|| {dmu.max():.2e}, "
        f"eta={inf.eta_max:.2e} rounds={inf.refine_iters}")
    out = {"time_s": dt, "prec": "mixed" if args.fem_prec else "fp64", "operator_applications": int(inf.steps),
           "restarts": int(inf.restarts), "max_rel_err_vs_closed_form": float(rel[j]), "worst_mode": j + 1,
           "max_abs_dmu_over_normC": float(dmu.max()), "eta_max": inf.eta_max, "omega": inf.omega,
           "refine_rounds": int(inf.refine_iters)}
    del K, M
    if emit:
        print(json.dumps({"fem_inverse_pencil": out, "n": n, "s": s, "block": blk}), flush=True)
    return out


def bench_mixed(args, cfg):
    """Mixed precision (FP32 sweeps + FP64 refinement) on the clustered
    known-spectrum pencil, with the plain FP64 solve of the same input timed
    beside it on the same GPU."""
    import numpy as np
    import torch

    import gen
    import paper_1111_6374_amd as gs

    n, s = cfg["n"], cfg["s"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"generating n={n} s={s} law={cfg['law']}")
    t0 = time.perf_counter()
    inst = gen.known_spectrum_device(n, cfg["law"], seed=gen.BASE_SEED + 2, stream=(2, 0, 0), device=dev,
                                     keep_factors=False)
    A, B0 = inst["A"], inst["B"]
    lam_true = np.sort(inst["lam"])[:s]
    B = torch.empty_like(B0)
    torch.cuda.synchronize()
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    solver = gs.Solver()
    Lam = torch.empty(s, dtype=torch.float64, device=dev)
    X = torch.empty(s, n, dtype=torch.float64, device=dev)
    kind, kblock, tunings, tuned_for = 0, 512, {}, [None]

    def tune(prec):
        # the sweep kernels of this precision: autotuned unless pinned by --trsv-sweep
        nonlocal kind, kblock
        if tuned_for[0] == prec:
            return
        tuned_for[0] = prec
        if args.trsv_sweep >= 0:
            rc = gs.gsyeig_set_trsv_sweep(solver.ctx, args.trsv_sweep)
            if rc:
                raise gs.GsyeigError("gsyeig_set_trsv_sweep", rc)
            kind, kblock = args.trsv_sweep, 512
        elif not args.no_autotune:
            rc, tu = gs.gsyeig_autotune(solver.ctx, n, prec, args.tune_cache or None)
            if rc:
                raise gs.GsyeigError("gsyeig_autotune", rc)
            tunings["mixed" if prec == gs.GSYEIG_MIXED else "fp64"] = tu.as_dict()
            kind, kblock = tu.trsv_sweep, tu.trsv_block

    def run(prec):
        tune(prec)
        o = gs.gsyeig_opts_default()
        o.prec = prec
        o.profile_every = args.profile_every
        if args.block > 1:
            o.block = args.block
        if args.reorth >= 0:
            o.reorth = args.reorth
        if args.refine_inner > 0:
            o.refine_inner = args.refine_inner
        B.copy_(B0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc, info = gs.gsyeig_solve(solver.ctx, n, s, A, n, B, n, o, Lam, X, n)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        if rc:
            raise gs.GsyeigError("gsyeig_solve", rc)
        return dt, info

    def show(tag, dt, inf):
        log(f"{tag}: {dt:.2f} s (GS1 {inf.t_gs1_ms:.0f} ms, KI {inf.t_ki_ms:.0f}, KI5 {inf.t_ki5_ms:.0f}, "
            f"BT1 {inf.t_bt1_ms:.0f}, refine {inf.t_refine_ms:.0f}, check {inf.t_check_ms:.0f}) m={inf.steps} "
            f"eta={inf.eta_max:.2e} eta1={inf.eta_phase1:.2e} rounds={inf.refine_iters} "
            f"block_ops={inf.block_applies}x{inf.block_cols}")

    for w in range(args.warmup):
        dt, inf = run(gs.GSYEIG_MIXED)
        show("warmup mixed", dt, inf)
    times, infos = [], []
    for k in range(args.steps):
        dt, inf = run(gs.GSYEIG_MIXED)
        show(f"step {k} mixed", dt, inf)
        times.append(dt)
        infos.append(inf)
    lam_mixed = Lam.cpu().numpy()
    mx = float(np.max(np.abs(inst["lam"])))
    e_lam = float(np.max(np.abs(lam_mixed - lam_true)) / mx)
    value = sum(times) / len(times)
    last = infos[-1]
    kind_m, kblock_m = kind, kblock  # the mixed solves' sweeps (the FP64 comparison may retune)
    fp64 = None
    if not args.no_fp64_compare:
        dt64, inf64 = run(gs.GSYEIG_FP64)
        show("fp64", dt64, inf64)
        lam64 = Lam.cpu().numpy()
        fp64 = {"time_s": dt64, "lanczos_steps": int(inf64.steps), "eta_max": inf64.eta_max,
                "e_lambda_vs_known": float(np.max(np.abs(lam64 - lam_true)) / mx),
                "lambda_diff_vs_mixed": float(np.max(np.abs(lam64 - lam_mixed)) / mx),
                "stages_ms": {"gs1": inf64.t_gs1_ms, "ki_loop": inf64.t_ki_ms, "ki5": inf64.t_ki5_ms,
                              "bt1": inf64.t_bt1_ms, "check": inf64.t_check_ms},
                "speedup_of_mixed": dt64 / value}
    samples = sum(i.prof_samples for i in infos)
    t1 = sum(i.t_ki1_ms_sum for i in infos) / max(samples, 1)
    t2 = sum(i.t_ki2_ms_sum for i in infos) / max(samples, 1)
    t3 = sum(i.t_ki3_ms_sum for i in infos) / max(samples, 1)
    tri32 = 4.0 * n * (n + 1) / 2
    vec = 8.0 * 2 * n
    trsv_ms = 0.5 * (t1 + t3)
    trsv_gbs = (tri32 + vec) / (trsv_ms * 1e-3) / 1e9 if trsv_ms > 0 else None
    symv_gbs = (tri32 + vec) / (t2 * 1e-3) / 1e9 if t2 > 0 else None
    out = {
        "metric": "time-to-s-eigenpairs", "value": value, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * value, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": cfg["label"], "n": n, "s": s, "spectrum": cfg["law"], "prec": "mixed",
                   "block": 1, "lanczos_steps": int(last.steps), "reorth_steps": int(last.reorth_steps),
                   "refine_rounds": int(last.refine_iters),
                   "block_cols": int(last.block_cols), "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": trsv_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (trsv_gbs / HBM_PEAK_GBS) if trsv_gbs else None,
                     "traffic": sweep_traffic(kind_m, kblock_m, n, "fp32"),
                     "kernel": "%s/%s on FP32 W (KI1/KI3, mean of the two)" % sweep_kernels(kind_m, kblock_m),
                     "avg_launch_ms": trsv_ms,
                     "algorithmic_bytes_per_launch": tri32 + vec},
        "kernels": {"ki1": sweep_kernels(kind_m, kblock_m)[0], "ki1_ms": t1, "ki3": sweep_kernels(kind_m, kblock_m)[1],
                    "ki3_ms": t3, "trsv_ms": trsv_ms, "trsv_GBs": trsv_gbs, "symv_ms": t2, "symv_GBs": symv_gbs,
                    "samples": samples},
        "stages_ms": {"gs1": last.t_gs1_ms, "ki_loop": last.t_ki_ms, "ki5": last.t_ki5_ms, "bt1": last.t_bt1_ms,
                      "refine": last.t_refine_ms, "check": last.t_check_ms, "total": last.t_total_ms},
        "refinement": {"eta_after_first_rr": last.eta_phase1, "rounds": int(last.refine_iters),
                       "fp32_block_applications": int(last.block_applies), "block_cols": int(last.block_cols)},
        "parity": {"e_lambda_vs_known": e_lam, "eta_max": last.eta_max, "omega": last.omega, "rho_F": last.rho_f,
                   "pass": bool(e_lam <= 1e-10 and last.eta_max <= 1e-10)},
        "fp64_same_input": fp64,
    }
    if tunings:
        out["tuning"] = tunings
    solver.close()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(n, cfg["law"])
    print(json.dumps(out), flush=True)


def bench_batched(args, cfg):
    """Many uneven instances: the batched entry point vs a loop of single solves."""
    import numpy as np
    import torch

    import gen
    import paper_1111_6374_amd as gs

    dev = torch.device("cuda:0")
    g = gen.rng(gen.BASE_SEED + 4, 0)
    sizes = [int(v) for v in g.integers(256, 4097, size=args.instances)]
    ss = [int(math.ceil(0.05 * n)) for n in sizes]
    log(f"generating {len(sizes)} instances, sum n^3 = {sum(n**3 for n in sizes):.3e}")
    t0 = time.perf_counter()
    A, B0, lam_true = [], [], []
    for i, n in enumerate(sizes):
        d = gen.known_spectrum_device(n, "spaced", seed=gen.BASE_SEED + 4, stream=(4, i), device=dev,
                                      keep_factors=False, rng_kind="torch")
        A.append(d["A"])
        B0.append(d["B"])
        lam_true.append(np.sort(d["lam"])[: ss[i]])
    B = [torch.empty_like(b) for b in B0]
    Lam = [torch.empty(s, dtype=torch.float64, device=dev) for s in ss]
    X = [torch.empty(s, n, dtype=torch.float64, device=dev) for s, n in zip(ss, sizes)]
    torch.cuda.synchronize()
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    solver = gs.Solver()

    def restore():
        for b, b0 in zip(B, B0):
            b.copy_(b0)
        torch.cuda.synchronize()

    prec = gs.GSYEIG_MIXED if args.prec != 0 else gs.GSYEIG_FP64
    o = gs.gsyeig_opts_default()
    o.prec = prec
    if args.block > 1:
        o.block = args.block
    if args.reorth >= 0:
        o.reorth = args.reorth

    def batched():
        restore()
        t = time.perf_counter()
        rc, status, infos = gs.gsyeig_solve_batched(solver.ctx, sizes, ss, A, sizes, B, sizes, o, Lam, X,
                                                    sizes, nstreams=args.streams)
        torch.cuda.synchronize()
        if rc:
            raise gs.GsyeigError("gsyeig_solve_batched", rc)
        return time.perf_counter() - t, infos

    for w in range(args.warmup):
        dt, _ = batched()
        log(f"warmup batched: {dt:.2f} s")
    times = []
    for k in range(args.steps):
        dt, infos = batched()
        times.append(dt)
        log(f"step {k}: batched {dt:.2f} s")
    e_lam = max(float(np.max(np.abs(L.cpu().numpy() - lt))) for L, lt in zip(Lam, lam_true))
    eta = max(i.eta_max for i in infos)
    # the batched driver in the other precision, and with every instance a
    # gsyeig_solve on the worker streams (batch_mode 1), same instances
    t_other = t_mode1 = None
    if not args.no_loop:
        o.prec = gs.GSYEIG_FP64 if prec == gs.GSYEIG_MIXED else gs.GSYEIG_MIXED
        t_other, _ = batched()
        log(f"batched, {'FP64' if o.prec == gs.GSYEIG_FP64 else 'mixed'}: {t_other:.2f} s")
        o.prec = prec
        o.batch_mode = 1
        t_mode1, _ = batched()
        log(f"batched, every instance a gsyeig_solve on {args.streams} streams: {t_mode1:.2f} s")
        o.batch_mode = 0
    # reference: the same instances as a loop of single-instance plain FP64 solves
    t_loop = None
    if not args.no_loop:
        restore()
        t = time.perf_counter()
        for i, n in enumerate(sizes):
            rc, _ = gs.gsyeig_solve(solver.ctx, n, ss[i], A[i], n, B[i], n, None, Lam[i], X[i], n)
            if rc:
                raise gs.GsyeigError("gsyeig_solve", rc)
        torch.cuda.synchronize()
        t_loop = time.perf_counter() - t
        log(f"loop of single FP64 solves: {t_loop:.2f} s")
    value = sum(times) / len(times)
    out = {
        "metric": "time-to-s-eigenpairs",
        "value": value, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * value, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == gs.GSYEIG_MIXED else "f64", "data": "synthetic",
        "config": {"workload": cfg["label"], "instances": len(sizes), "sum_n": sum(sizes),
                   "streams": args.streams, "prec": "mixed" if prec == gs.GSYEIG_MIXED else "fp64",
                   "batch_mode": "one launch for the Lanczos phase of every instance (n <= 4096)",
                   "block": max(1, args.block), "parallelism": "single-gpu"},
        "loop_of_single_fp64_solves_s": t_loop, "batched_speedup": (t_loop / value) if t_loop else None,
        ("batched_fp64_s" if prec == gs.GSYEIG_MIXED else "batched_mixed_s"): t_other,
        "batched_per_instance_solves_s": t_mode1,
        "lanczos_one_launch_ms_sum": float(sum(i.t_ki_ms for i in infos)),
        "lanczos_steps_total": int(sum(i.steps for i in infos)),
        # bytes the Lanczos operator reads and writes per step, summed over the
        # steps: A's upper triangle and U's twice (n (n + 1) / 2 elements each,
        # FP32 mixed / FP64), the 64 x 64 FP64 diagonal-block inverses twice
        # (64 n doubles each time) and the product's row-sum scratch written
        # and read once (16 n doubles each way)
        "lanczos_operator_bytes": float(sum(i.steps * (3 * n * (n + 1) // 2 * (4 if prec == gs.GSYEIG_MIXED else 8)
                                                       + 2 * 64 * n * 8 + 2 * 16 * n * 8)
                                            for i, n in zip(infos, sizes))),
        "parity": {"e_lambda_vs_known": e_lam, "eta_max": eta, "pass": bool(e_lam <= 1e-10 and eta <= 1e-10)},
    }
    solver.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
