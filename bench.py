"""Benchmark: whole-solve throughput of the HZ-GHSVD path on one MI355X.

A "step" is one complete ghsvd_solve of the n = 1024 pencil (F 1536 x 1024
with J = diag(+1 x1152, -1 x384), G 2048 x 1024 = U diag(s) W^* with s
log-uniform in [1e-8, 1], so cond(G^* G) = 1e16; complex128): input checks,
one-time reduction (hyperbolic QR of F, QR of G), the sweep stages of the
chosen path (default: Level-2 blocked FP64 sweeps until a sweep has no big
transformation), and the outputs lambda, X.  Inputs are resident in HBM
before the timed region.  Prints one JSON line.

Beside the timed path it reports:
  * per sweep-kernel kind, the mean launch time measured with HIP events on
    the launch stream over the timed region, and its roofline;
  * the error of lambda against the stored oracle eigenvalues of this pencil;
  * the other paths on the same pencil (plain FP64 pointwise; mixed FP32 ->
    FP64), with their times and errors;
  * the CPU oracle on a bounded sample (reduction + one sweep, extrapolated);
  * the full GHSVD (Phase 4: U, V, Sigma_F, Sigma_G, X = Z^{-1}) of the swept
    square factors, timed alone, with the relative errors (7.1).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|mixed]
                    [--variant blocked|pointwise] [--no-compare] [--no-cpu-baseline]
                    [--no-full]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GHSVD pencils/s + pair-updates/s, mixed+batched vs plain FP64, rel err<=1e-12"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_MFMA_PEAK_TF = 78.6       # dense FP64 matrix
FP32_MFMA_PEAK_TF = 157.3      # dense FP32 matrix
FP64_VALU_PEAK_TF = 78.6       # FP64 vector
GOLDEN = os.path.join(ROOT, "tests", "golden", "workload2_lambda.json")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def pair_bytes(visited, transformed, mr, pr, n, fp32=False):
    """Algorithmic HBM bytes of the pointwise pair kernel: a transformed pair
    reads and writes two columns of F, G and Z' (64 (m_r + p_r + n) bytes in
    complex128), a skipped pair only reads its F and G columns
    (32 (m_r + p_r) bytes).  Complex64 halves both."""
    b = transformed * 64.0 * (mr + pr + n) + (visited - transformed) * 32.0 * (mr + pr)
    return b / 2 if fp32 else b


def block_width_for(n):
    """The block width the library picks for a pencil of order n."""
    return 16 if n >= 512 else 8


def kernel_rooflines(times, info_sum, mr, pr, n, w, nbp, fp32_blocked=False):
    """Per-kind roofline over the timed region.  times[kind] = (ms, timed, launches)."""
    out = {}
    c = 2 * w
    for kind, (ms, timed, launches) in times.items():
        if timed == 0 or launches == 0:
            continue
        mean_s = ms / timed * 1e-3
        rec = {"mean_us": mean_s * 1e6, "launches": launches, "timed_launches": timed,
               "total_ms_est": mean_s * launches * 1e3}
        if kind in ("pair64", "pair32"):
            vis, tr = info_sum["pw_visited"], info_sum["pw_transformed"]
            if kind == "pair32":  # FP32 pair stage counters are not separated; skip
                continue
            b = pair_bytes(vis, tr, mr, pr, n) / launches
            rec.update(bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS,
                       achieved=b / mean_s / 1e9, units_per_launch=vis / launches,
                       work_per_launch=b, work_unit="bytes")
        elif kind in ("gram", "update"):
            bsz = 8 if fp32_blocked else 16
            if kind == "gram":
                flops = 4.0 * c * c * (mr + pr) * nbp           # Hermitian Grams: 8 c^2 rows / 2
                byts = c * bsz * (mr + pr) * nbp                # block columns read once
            else:
                flops = 8.0 * c * c * (mr + pr + n) * nbp       # three complex GEMMs
                byts = 2.0 * c * bsz * (mr + pr + n) * nbp      # block columns read + written
            peak_tf = FP32_MFMA_PEAK_TF if fp32_blocked else FP64_MFMA_PEAK_TF
            t_mfma = flops / (peak_tf * 1e12)
            t_hbm = byts / (HBM_PEAK_GBS * 1e9)
            if t_hbm >= t_mfma:
                rec.update(bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS,
                           achieved=byts / mean_s / 1e9, work_per_launch=byts, work_unit="bytes")
            else:
                rec.update(bound="mfma", unit="TFLOP/s", peak=peak_tf,
                           achieved=flops / mean_s / 1e12, work_per_launch=flops,
                           work_unit="flops")
            rec["units_per_launch"] = nbp
        elif kind == "inner":
            # two-sided 2x2-block updates of H^ and S^ (128 flops each) and the
            # accumulation into Z^ (64 flops), (c/2)^2 blocks per inner step,
            # c - 1 inner steps per block pair
            flops = 320.0 * (c * c / 4.0) * (c - 1) * nbp
            rec.update(bound="alu", unit="TFLOP/s", peak=FP64_VALU_PEAK_TF,
                       achieved=flops / mean_s / 1e12, work_per_launch=flops, work_unit="flops",
                       units_per_launch=nbp, us_per_inner_step=mean_s * 1e6 / (c - 1))
        rec["frac"] = rec["achieved"] / rec["peak"]
        rec["traffic"] = stored_traffic(kind)
        out[kind] = rec
    return out


KERNEL_NAMES = {"pair64": "k_pair<double> (pointwise FP64 pair kernel)",
                "gram": "k_blk_gram (block-pivot Grams, MFMA)",
                "inner": "k_blk_inner (inner 2x2 sweep of a block pivot, LDS)",
                "update": "k_blk_update (block-column update, MFMA)"}


def stored_traffic(kind):
    """HBM bytes per launch from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE, each scaled by what the counter reads for a plain copy), or
    None when a source of the kernel changed since the counters were taken."""
    try:
        with open(TRAFFIC) as f:
            t = json.load(f).get(kind)
    except (OSError, ValueError):
        return None
    if not t:
        return None
    h = hashlib.sha256()
    try:
        for src in t["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
    except OSError:
        return None
    return t["bytes_per_launch"] if h.hexdigest() == t["sha256"] else None


def lambda_errors(lam):
    with open(GOLDEN) as f:
        ref = np.asarray(json.load(f)["lambda"], dtype=np.float64)
    e = np.abs(lam - ref) / np.abs(ref)
    return float(e.max()), float(np.median(e))


def cpu_baseline(P, oracle_sweeps):
    """The CPU oracle on a bounded sample of the same workload: the full
    reduction (hyperbolic QR + QR) plus one round-robin sweep on the square
    factors, extrapolated to the oracle's own sweep count on this pencil."""
    from oracle import oracle as O
    o = O.Oracle()
    t0 = time.perf_counter()
    st, Fsq, Jsq, Gsq, perm, n2 = o.reduce(P.F, P.J, P.G)
    t_red = time.perf_counter() - t0
    t0 = time.perf_counter()
    o.hz_run(Fsq, Jsq, Gsq, order=1, max_sweeps=1)
    t_sw = time.perf_counter() - t0
    total = t_red + oracle_sweeps * t_sw
    return {"value": 1.0 / total, "unit": "pencils/s", "cores": 1, "kind": "oracle",
            "sample": (f"one pencil: reduction ({t_red:.1f} s) + 1 square sweep ({t_sw:.1f} s) "
                       f"measured single-threaded; total extrapolated to {oracle_sweeps} sweeps "
                       f"(the oracle's count on this pencil) = {total:.0f} s/pencil")}


def full_leg(ghsvd, F, J, G, reps=3):
    """The full GHSVD of the pencil (Phase 4): the reduction, the row split
    by the signature, blocked FP64 sweeps in place on the square factors, then
    ghsvd_full, timed alone (median of `reps` calls), with the relative errors
    (7.1) of the decomposition of the square factors."""
    import torch
    Fsq, Jsq, Gsq, perm, n2 = ghsvd.reduce(F, J, G)
    n = Fsq.shape[1]
    order = torch.cat([torch.nonzero(Jsq > 0).flatten(), torch.nonzero(Jsq < 0).flatten()])
    n_plus = int((Jsq > 0).sum().item())
    # column-major copies: F0, G0 keep the square factors for the errors,
    # Fw, Gw, Zw are swept in place
    F0 = Fsq[order, :].t().contiguous().t()
    G0 = Gsq.t().clone().t()
    Fw = F0.t().clone().t()
    Gw = G0.t().clone().t()
    Zw = torch.eye(n, dtype=torch.complex128, device=F.device).t()
    rc, done, cnt = ghsvd.block_sweeps(Fw, n_plus, Gw, Zw, 60, block_width=16)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U, V, sf, sg, X = ghsvd.full(Fw, n_plus, Gw, Zw)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    eF = (torch.linalg.norm(F0 - (U * sf[None, :]) @ X) / torch.linalg.norm(F0)).item()
    eG = (torch.linalg.norm(G0 - (V * sg[None, :]) @ X) / torch.linalg.norm(G0)).item()
    return {"ms": 1000.0 * sorted(ts)[len(ts) // 2], "sweeps": done, "sweep_status": rc,
            "errors_7_1": {"F": eF, "G": eG}}


def run_path(ghsvd, F, J, G, P, kw, steps, warmup, profile_every=0):
    import torch
    dev = F.device
    opt = ghsvd.options(**kw)
    work = torch.empty(ghsvd.workspace_size(P.m, P.n, P.p, opt), dtype=torch.uint8, device=dev)
    lam = torch.empty(P.n, dtype=torch.float64, device=dev)
    X = ghsvd.fortran_empty(P.n, P.n, device=dev)
    torch.cuda.synchronize()
    for _ in range(warmup):
        ghsvd.solve(F, J, G, work=work, out=(lam, X), **kw)
    torch.cuda.synchronize()
    if profile_every:
        ghsvd.profile_enable(profile_every)
        for k in ghsvd.PROF_KINDS:
            ghsvd.profile_read(k)  # clear
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, _, info = ghsvd.solve(F, J, G, work=work, out=(lam, X), **kw)
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    times = {}
    if profile_every:
        times = {k: ghsvd.profile_read(k) for k in ghsvd.PROF_KINDS}
        ghsvd.profile_enable(0)
    return dt, infos, lam.cpu().numpy(), times


def batched_workload(args, ghsvd, synth, torch, dev):
    """The batch of 64 k-point pencils (n_k uniform in [300, 900], F 1.5 n_k x n_k
    with a 3:1 signature, G 2 n_k x n_k with s log-uniform in [1e-6, 1]) in one
    ghsvd_solve_batched call per step, after an untimed launch-tuning call."""
    sizes = synth.workload_sizes(4)
    Ps = [synth.workload_pencil(4, k) for k in range(len(sizes))]
    Fs = [ghsvd.to_device_fortran(P.F, dev) for P in Ps]
    Gs = [ghsvd.to_device_fortran(P.G, dev) for P in Ps]
    Js = [torch.from_numpy(P.J).to(dev) for P in Ps]
    tuned = {}
    for var in ("blocked", "pointwise"):
        w, wpp, trials = ghsvd.autotune(Fs, Js, Gs, variant=var)
        tuned[var] = {"block_width": w, "waves_per_pair": wpp, "trial_ms": trials}
    paths = {}
    lams = {}
    for prec, var in (("fp64", "blocked"), ("mixed", "blocked"), ("fp64", "pointwise")):
        kw = dict(precision=prec, variant=var, max_sweeps=args.max_sweeps,
                  block_width=args.block_width)
        for _ in range(args.warmup):
            ghsvd.solve_batched(Fs, Js, Gs, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            lam, X, infos, rc = ghsvd.solve_batched(Fs, Js, Gs, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        lams[f"{prec}-{var}"] = [l.cpu().numpy() for l in lam]
        paths[f"{prec}-{var}"] = {
            "pencils_per_s": len(Ps) * args.steps / dt, "ms_per_batch": 1000.0 * dt / args.steps,
            "status": rc, "max_sweeps_fp64": max(i["sweeps_fp64"] for i in infos),
            "max_sweeps_fp32": max(i["sweeps_fp32"] for i in infos),
            "pair_updates_per_s": sum(i["pairs_visited"] for i in infos) * args.steps / dt}
    ref = lams["fp64-blocked"]
    for key in ("mixed-blocked", "fp64-pointwise"):
        e = max(float(np.max(np.abs(a - b) / np.abs(b))) for a, b in zip(lams[key], ref))
        paths[key]["max_rel_diff_vs_fp64_blocked"] = e
    best = max(paths, key=lambda k: paths[k]["pencils_per_s"])
    rec = {
        "metric": METRIC, "value": paths[best]["pencils_per_s"], "unit": "pencils/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": paths[best]["ms_per_batch"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if best.startswith("fp64") else "f32+f64",
        "data": "synthetic",
        "config": {"workload": ("64 k-point pencils, n_k uniform in [300,900], F ceil(1.5 n_k) x n_k "
                                "Gaussian, J 3:1, G 2 n_k x n_k = U diag(s) W^*, s log-uniform "
                                f"[1e-6,1], complex128, one batched call; best path {best}"),
                   "batch": len(Ps), "n_min": int(min(sizes)), "n_max": int(max(sizes))},
        "paths": paths, "tuned": tuned,
    }
    print(json.dumps(rec), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def prime(ghsvd, synth, torch, dev, kw):
    """One small untimed solve on the path, so that the timed runs start warm."""
    P = synth.workload_pencil(1)
    ghsvd.solve(ghsvd.to_device_fortran(P.F, dev), torch.from_numpy(P.J).to(dev),
                ghsvd.to_device_fortran(P.G, dev), check=False, **kw)
    torch.cuda.synchronize()


def time_paths(args, ghsvd, synth, torch, dev, pencils, paths_wanted):
    """Times each (precision, variant) path on a list of (F, J, G) device
    pencils in one batched call per step; returns per-path records and lambdas."""
    Fs = [q[0] for q in pencils]
    Js = [q[1] for q in pencils]
    Gs = [q[2] for q in pencils]
    paths, lams = {}, {}
    for prec, var in paths_wanted:
        kw = dict(precision=prec, variant=var, max_sweeps=args.max_sweeps,
                  block_width=args.block_width)
        prime(ghsvd, synth, torch, dev, kw)
        for _ in range(args.warmup):
            ghsvd.solve_batched(Fs, Js, Gs, **kw)
        torch.cuda.synchronize()
        log(f"timing {prec}-{var}")
        t0 = time.perf_counter()
        for _ in range(args.steps):
            lam, X, infos, rc = ghsvd.solve_batched(Fs, Js, Gs, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        key = f"{prec}-{var}"
        lams[key] = [l.cpu().numpy() for l in lam]
        del X
        paths[key] = {
            "pencils_per_s": len(Fs) * args.steps / dt, "ms_per_batch": 1000.0 * dt / args.steps,
            "status": rc, "max_sweeps_fp64": max(i["sweeps_fp64"] for i in infos),
            "max_sweeps_fp32": max(i["sweeps_fp32"] for i in infos),
            "pair_updates_per_s": sum(i["pairs_visited"] for i in infos) * args.steps / dt}
        log(f"{key}: {paths[key]['ms_per_batch']:.1f} ms, status {rc}")
    ref = lams.get("fp64-blocked")
    if ref is not None:
        for key in lams:
            if key != "fp64-blocked":
                paths[key]["max_rel_diff_vs_fp64_blocked"] = max(
                    float(np.max(np.abs(a - b) / np.abs(b))) for a, b in zip(lams[key], ref))
    return paths


def large_workload(args, ghsvd, synth, torch, dev):
    """Workload 3 (one n=4096 pencil, F 6144 x 4096 with a 3:1 signature, G
    8192 x 4096 with s log-uniform in [1e-5, 1], plus the same pencil under
    J = I) or workload 5 (16 pencils, n_k uniform in [2000, 6000], F 1.5 n_k x
    n_k with a 4:1 signature, G 2 n_k x n_k, s in [1e-6, 1]) on the blocked
    paths (and the pointwise FP64 path for workload 3).  Workload 5's Haar QRs
    run on the device (same draws as the host recipe)."""
    W = args.workload
    sizes = synth.workload_sizes(W)
    pencils = []
    for k in range(len(sizes)):
        if W == 3:
            P = synth.workload_pencil(3, k)
            pencils.append((ghsvd.to_device_fortran(P.F, dev), torch.from_numpy(P.J).to(dev),
                            ghsvd.to_device_fortran(P.G, dev)))
        else:
            F, J, G, _ = synth.workload_pencil_device(5, k, dev)
            pencils.append((F, J, G))
        log(f"pencil {k}: n={sizes[k]} built")
    torch.cuda.synchronize()
    want = [("fp64", "blocked"), ("mixed", "blocked")]
    if W == 3 and not args.no_compare:
        want.append(("fp64", "pointwise"))
    paths = time_paths(args, ghsvd, synth, torch, dev, pencils, want)
    extra = {}
    if W == 3:
        ones = [(F, torch.ones_like(J), G) for F, J, G in pencils]
        extra["j_identity"] = time_paths(args, ghsvd, synth, torch, dev, ones,
                                         [("fp64", "blocked"), ("mixed", "blocked")])
    best = max(paths, key=lambda k: paths[k]["pencils_per_s"])
    desc = {3: ("one pencil n=4096: F 6144x4096 Gaussian, J 4608(+)/1536(-), G 8192x4096 = "
                "U diag(s) W^*, s log-uniform [1e-5,1] (cond S = 1e10), complex128; plus the "
                "same pencil under J = I"),
            5: ("16 pencils, n_k uniform in [2000,6000], F ceil(1.5 n_k) x n_k Gaussian, J 4:1, "
                "G 2 n_k x n_k = U diag(s) W^*, s log-uniform [1e-6,1], complex128, one batched "
                "call")}[W]
    rec = {
        "metric": METRIC, "value": paths[best]["pencils_per_s"], "unit": "pencils/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": paths[best]["ms_per_batch"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if best.startswith("fp64") else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{desc}; best path {best}", "batch": len(sizes),
                   "n_min": int(min(sizes)), "n_max": int(max(sizes))},
        "paths": paths, **extra,
    }
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--variant", default="blocked", choices=["pointwise", "blocked"])
    ap.add_argument("--inner", default="cross", choices=["cross", "full", "fb"],
                    help="blocked inner level: one sweep per block pivot in the cross or full "
                         "round-robin ordering (BO), or sweeps to convergence (FB, at most 30; "
                         "the inner kernel's roofline counts one sweep per launch)")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reduce", action="store_true",
                    help="sweep the tall factors directly, without the one-time reduction")
    ap.add_argument("--no-full", action="store_true",
                    help="skip the full-GHSVD leg (Phase 4 timing and the errors (7.1))")
    ap.add_argument("--profile-every", type=int, default=4)
    ap.add_argument("--max-sweeps", type=int, default=0)
    ap.add_argument("--block-width", type=int, default=0, choices=[0, 8, 16, 32],
                    help="blocked variant's block width (0: the library's choice)")
    ap.add_argument("--workload", type=int, default=2, choices=[2, 3, 4, 5],
                    help="2: the single n=1024 pencil (default); 3: one n=4096 pencil; "
                         "4: the batch of 64 pencils; 5: the batch of 16 large pencils")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe:
        # A plain copy of known size: reads and writes copy_probe bytes once.
        src = torch.ones(args.copy_probe // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "copies": 3}), flush=True)
        return

    from paper_1907_08560_amd import ghsvd, synth

    dev = torch.device("cuda:0")
    if args.workload == 4:
        batched_workload(args, ghsvd, synth, torch, dev)
        return
    if args.workload in (3, 5):
        large_workload(args, ghsvd, synth, torch, dev)
        return
    P = synth.workload_pencil(2)
    F = ghsvd.to_device_fortran(P.F, dev)
    G = ghsvd.to_device_fortran(P.G, dev)
    J = torch.from_numpy(P.J).to(dev)
    kw = dict(precision=args.precision, variant=args.variant, max_sweeps=args.max_sweeps,
              block_width=args.block_width, reduce=not args.no_reduce, inner_order=args.inner)

    dt, infos, lam, times = run_path(ghsvd, F, J, G, P, kw, args.steps, args.warmup,
                                     args.profile_every)
    ms_per_step = 1000.0 * dt / args.steps
    info = infos[-1]
    isum = {k: sum(i[k] for i in infos) for k in ("pairs_visited", "pw_visited", "pw_transformed")}
    mr, pr, n = info["m_r"], info["p_r"], P.n
    w = args.block_width or block_width_for(n)
    nb = -(-n // w)
    nb += nb & 1
    kr = kernel_rooflines(times, isum, mr, pr, n, w, nb // 2,
                          fp32_blocked=args.precision == "mixed")
    dom = max(kr, key=lambda k: kr[k]["total_ms_est"]) if kr else None
    err_max, err_med = lambda_errors(lam)

    rec = {
        "metric": METRIC,
        "value": args.steps / dt,
        "unit": "pencils/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": ("one LAPW-shaped pencil n=1024: F 1536x1024 Gaussian, J 1152(+)/384(-), "
                         "G 2048x1024 = U diag(s) W^*, s log-uniform [1e-8,1] (cond S = 1e16), "
                         f"complex128; {'no reduction (tall factors)' if args.no_reduce else 'reduction'}"
                         f" + {args.variant} {args.precision} sweeps"),
            "n": n, "m": P.m, "p": P.p, "batch": 1,
            "precision": args.precision, "variant": args.variant, "reduce": not args.no_reduce,
            "inner": args.inner,
        },
        "pair_updates_per_s": isum["pairs_visited"] / dt,
        "sweeps_fp64": info["sweeps_fp64"],
        "sweeps_fp32": info["sweeps_fp32"],
        "sweeps_blocked": info["sweeps_blocked"],
        "status": info["status"],
        "lambda_rel_err_vs_oracle": {"max": err_max, "median": err_med},
    }
    if dom is not None:
        d = kr[dom]
        rec["roofline"] = {
            "bound": d["bound"], "kernel": KERNEL_NAMES.get(dom, dom),
            "achieved": d["achieved"], "peak": d["peak"], "unit": d["unit"], "frac": d["frac"],
            "traffic": stored_traffic(dom),
            "mean_launch_us": d["mean_us"], "work_per_launch": d["work_per_launch"],
            "work_unit": d["work_unit"], "timed_launches": d["timed_launches"],
            "launches": d["launches"],
        }
        rec["kernels"] = kr
    if not args.no_compare:
        comp = {}
        for prec, var in (("fp64", "pointwise"), ("mixed", "blocked"), ("fp64", "blocked")):
            if prec == args.precision and var == args.variant:
                continue
            ckw = dict(precision=prec, variant=var, max_sweeps=args.max_sweeps,
                       block_width=args.block_width)
            cdt, cinf, clam, _ = run_path(ghsvd, F, J, G, P, ckw, 2, 1)
            emax, emed = lambda_errors(clam)
            comp[f"{prec}-{var}"] = {"ms_per_pencil": 1000.0 * cdt / 2,
                                     "pencils_per_s": 2 / cdt,
                                     "sweeps_fp32": cinf[-1]["sweeps_fp32"],
                                     "sweeps_fp64": cinf[-1]["sweeps_fp64"],
                                     "status": cinf[-1]["status"],
                                     "lambda_rel_err_vs_oracle": {"max": emax, "median": emed}}
        rec["compare"] = comp
    if not args.no_full:
        rec["full_ghsvd"] = full_leg(ghsvd, F, J, G)
    if not args.no_cpu_baseline:
        with open(GOLDEN) as f:
            osw = json.load(f)["sweeps"]
        rec["cpu_baseline"] = cpu_baseline(P, osw)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
