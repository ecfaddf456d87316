"""Benchmark: batched throughput of the HZ-GHSVD path on one MI355X.

Default (the headline): a "step" is one ghsvd_solve_batched call on 64
k-point pencils of uneven order (n_k uniform in [300, 900]; F ceil(1.5 n_k) x
n_k Gaussian with a 3:1 signature; G 2 n_k x n_k = U diag(s) W^* with s
log-uniform in [1e-6, 1], so cond(G^* G) <= 1e12; complex128): input checks,
one-time reduction of every pencil (hyperbolic QR of F, QR of G), complex
FP32 blocked warm-up sweeps, the hand-off to FP64, FP64 blocked sweeps to
convergence, and the outputs lambda, X.  Inputs are resident in HBM before
the timed region.  `value` is pencils/s of that mixed-precision path.  Prints
one JSON line.

Beside it the line reports:
  * the plain FP64 blocked and FP64 pointwise paths on the same batch (ms per
    batch, sweeps, the largest lambda difference from FP64 blocked);
  * every path's lambda error against the stored oracle eigenvalues;
  * per kernel kind (FP32 and FP64 Gram, inner sweep, update; the reduction's
    column step), the mean launch time measured with HIP events on the launch
    stream over the timed region, and its roofline; `roofline` is the
    dominant kernel of the headline path;
  * the CPU oracle on a bounded sample of the batch, in a process pool;
  * the single n = 1024 pencil at cond(S) = 1e16 (FP64 and mixed blocked, and
    the full GHSVD of its swept factors with the errors (7.1));
  * Phase 1 (ZHEBPJ of the atom blocks and the assembly of F~, J~, G~) on the
    A1- and B1-shaped atom sets, with the product kernel's MFMA roofline;
  * the explicit-formation route (Section 4.5) against the HZ solve on
    well-conditioned pencils of order 1024 and 2048.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 4|2|3|5]
                    [--block-width 0|8|16|32] [--inner cross|full|fb]
                    [--no-compare] [--no-cpu-baseline] [--no-workload2] [--no-full]
                    [--no-phase1] [--no-fast]

--workload 2 times single solves of the n = 1024 pencil on one path
(--precision, --variant); 3 and 5 time the large pencils on the blocked paths.
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
FP32_VALU_PEAK_TF = 157.3      # FP32 vector
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


KERNEL_NAMES = {"pair64": "k_pair<double> (pointwise FP64 pair kernel)",
                "gram": "k_blk_gram<double> (block-pivot Grams, MFMA)",
                "inner": "k_blk_inner (inner 2x2 sweep of a block pivot, LDS; FP64 stage)",
                "update": "k_blk_update<double> (block-column update, MFMA)",
                "gram32": "k_blk_gram<float> (block-pivot Grams, FP32 MFMA)",
                "inner32": "k_blk_inner (inner 2x2 sweep of a block pivot, LDS; FP32 stage)",
                "update32": "k_blk_update<float> (block-column update, FP32 MFMA)",
                "reduce": "one-time reduction column step (k_jqr_cross, k_jqr_cross2, k_jqr_step)"}


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


GOLDEN4 = os.path.join(ROOT, "tests", "golden", "workload4_lambda.json")


def golden_batch(path, Ps):
    """Stored oracle eigenvalues of a batch, by pencil (None where the stored
    input fingerprint does not match)."""
    try:
        with open(path) as f:
            recs = {r["k"]: r for r in json.load(f)["pencils"]}
    except (OSError, ValueError, KeyError):
        return None, None
    lams, sweeps = [], []
    for k, P in enumerate(Ps):
        r = recs.get(k)
        ok = r is not None and r["n"] == P.n and abs(
            r["fingerprint"][0] - float(np.abs(P.F).sum())) <= 1e-9 * r["fingerprint"][0]
        if ok:
            lam = np.asarray([float(v) for v in r["lambda"]])
            kap = np.asarray(r.get("kappa_h", np.ones_like(lam)), dtype=np.float64)
            # the parity tests' gate: 1e-10, plus the cancellation in h_j of an
            # eigenvalue near zero (kappa_j = ||F x_j||^2 / |lambda_j|)
            lams.append((lam, 1e-10 + 4.0 * np.sqrt(float(P.m) * P.n) * 2.0 ** -52 * kap))
        else:
            lams.append(None)
        sweeps.append(r["sweeps"] if ok else None)
    return lams, sweeps


def batch_errors(lams, ref):
    """max and median over all eigenvalues of all pencils of |lam - ref| / |ref|,
    and the largest ratio of that error to the parity tests' per-eigenvalue gate."""
    es, rs = [], []
    for a, r in zip(lams, ref):
        if r is None:
            continue
        e = np.abs(a - r[0]) / np.abs(r[0])
        es.append(e)
        rs.append(e / r[1])
    if not es:
        return None
    e = np.concatenate(es)
    return {"max": float(e.max()), "median": float(np.median(e)), "pencils": len(es),
            "max_over_gate": float(np.concatenate(rs).max())}


def block_schedule(n, w):
    """Blocks (rounded up to even), block pairs per step and block steps per sweep."""
    nb = -(-n // w)
    nb += nb & 1
    return nb, nb // 2, nb - 1


def batch_rooflines(times, infos, w, inner_order, steps, fp32_blocked=True):
    """Per-kind roofline of a batched path over the timed region (`steps`
    solves).  The algorithmic work of a kind is counted from each pencil's
    block schedule and its sweep counts (info): every block pair of every
    block step of a sweep (the update kernel skips a pair only when its inner
    sweep transformed nothing, which the sweep counters show to be rare), in
    the precision of the stage.  Per launch it is that total over all launches
    of the kind (pencils that have retired or have fewer block steps idle in a
    launch), divided by the sampled mean launch time."""
    c = 2 * w
    tot = {}
    for inf in infos:
        n = inf["n"]
        mr, pr = inf["m_r"], inf["p_r"]
        nb, nbp, bsteps = block_schedule(n, w)
        # sweeps_blocked counts the blocked sweeps of both stages
        s32 = inf["sweeps_fp32"] if fp32_blocked else 0
        for kind32, sweeps in ((True, s32), (False, inf["sweeps_blocked"] - s32)):
            if sweeps <= 0:
                continue
            bsz = 8 if kind32 else 16
            pairs = sweeps * bsteps * nbp
            sfx = "32" if kind32 else ""
            g = tot.setdefault("gram" + sfx, [0.0, 0.0])
            g[0] += pairs * c * bsz * (mr + pr)                 # block columns read once
            g[1] += pairs * 4.0 * c * c * (mr + pr)             # Hermitian Grams
            u = tot.setdefault("update" + sfx, [0.0, 0.0])
            u[0] += pairs * 2.0 * c * bsz * (mr + pr + n)       # block columns read + written
            u[1] += pairs * 8.0 * c * c * (mr + pr + n)         # three complex GEMMs
            # inner: two-sided 2x2-block updates of H^, S^ (128 flops each) and
            # the accumulation into Z^ (64 flops) for (c/2)^2 blocks per inner
            # step; 2w - 1 inner steps at block step 0 and w at the others in
            # the cross ordering, 2w - 1 at every step in the full one
            later = w if inner_order == "cross" else c - 1
            isteps = sweeps * nbp * ((c - 1) + (bsteps - 1) * later)
            i = tot.setdefault("inner" + sfx, [0.0, 0.0])
            i[1] += isteps * 320.0 * (c * c / 4.0)
        if inf.get("pw_visited"):
            r = tot.setdefault("pair64", [0.0, 0.0])
            r[0] += pair_bytes(inf["pw_visited"], inf["pw_transformed"], mr, pr, n)
        if inf.get("reduced"):
            m, p = inf["m"], inf["p"]
            t = np.arange(n, dtype=np.float64)
            r = tot.setdefault("reduce", [0.0, 0.0])
            # one read and one write of the trailing columns of F and G per column step
            r[0] += float(np.sum(32.0 * (m + p - 2 * t) * (n - t)))
    out = {}
    for kind, (ms, timed, launches) in times.items():
        if timed == 0 or launches == 0 or kind not in tot:
            continue
        mean_s = ms / timed * 1e-3
        byts, flops = (v * steps / launches for v in tot[kind])
        rec = {"mean_us": mean_s * 1e6, "launches": launches, "timed_launches": timed,
               "total_ms_est": mean_s * launches * 1e3}
        fp32 = kind.endswith("32")
        peak_tf = FP32_MFMA_PEAK_TF if fp32 else FP64_MFMA_PEAK_TF
        if kind.startswith("inner"):
            rec.update(bound="alu", unit="TFLOP/s", peak=FP32_VALU_PEAK_TF if fp32 else
                       FP64_VALU_PEAK_TF, achieved=flops / mean_s / 1e12,
                       work_per_launch=flops, work_unit="flops",
                       note="latency-bound inner sweep; reported as time, ALU fraction for context")
        elif kind == "reduce" or byts / (HBM_PEAK_GBS * 1e9) >= flops / (peak_tf * 1e12):
            rec.update(bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS,
                       achieved=byts / mean_s / 1e9, work_per_launch=byts, work_unit="bytes")
        else:
            rec.update(bound="mfma", unit="TFLOP/s", peak=peak_tf,
                       achieved=flops / mean_s / 1e12, work_per_launch=flops, work_unit="flops")
        rec["frac"] = rec["achieved"] / rec["peak"]
        rec["traffic"] = stored_traffic(kind)
        out[kind] = rec
    return out


def time_batch(ghsvd, torch, Fs, Js, Gs, kw, steps, warmup, profile_every=0):
    """Times `steps` batched solves after `warmup` untimed ones; returns (seconds,
    infos of the last solve, lambdas of the last solve, per-kind kernel times)."""
    for _ in range(warmup):
        ghsvd.solve_batched(Fs, Js, Gs, **kw)
    torch.cuda.synchronize()
    if profile_every:
        ghsvd.profile_enable(profile_every)
        for k in ghsvd.PROF_KINDS:
            ghsvd.profile_read(k)  # clear
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        lam, X, infos, rc = ghsvd.solve_batched(Fs, Js, Gs, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    times = {}
    if profile_every:
        times = {k: ghsvd.profile_read(k) for k in ghsvd.PROF_KINDS}
        ghsvd.profile_enable(0)
    lams = [l.cpu().numpy() for l in lam]
    del X
    return dt, infos, lams, times, rc


def _oracle_sample(job):
    """One pencil of the CPU baseline's sample: the oracle's reduction and one
    round-robin sweep of the square factors, in CPU seconds."""
    number, k = job
    from oracle import oracle as O
    from paper_1907_08560_amd import synth
    P = synth.workload_pencil(number, k)
    o = O.Oracle()
    t0 = time.process_time()
    st, Fsq, Jsq, Gsq, perm, n2 = o.reduce(P.F, P.J, P.G)
    t_red = time.process_time() - t0
    t0 = time.process_time()
    o.hz_run(Fsq, Jsq, Gsq, order=1, max_sweeps=1)
    t_sw = time.process_time() - t0
    return k, P.n, t_red, t_sw


def cpu_baseline_batched(sizes, oracle_sweeps, cores):
    """The CPU oracle on a bounded sample of the batch, in a process pool of
    `cores` workers (one serial oracle process per core): for each of the
    first `cores` pencils, the reduction and one square sweep, each pencil's
    time extrapolated to its own oracle sweep count; the batch's throughput
    is the pool's, cores / mean per-pencil time (the sample's mean scaled by
    the batch's mean n^3 over the sample's)."""
    import multiprocessing as mp
    jobs = [(4, k) for k in range(min(cores, len(sizes)))]
    # one thread per worker (the workers' numpy draws the inputs; the oracle
    # itself is serial), set before the workers start
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(len(jobs)) as pool:
        res = pool.map(_oracle_sample, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    per = []
    for k, n, t_red, t_sw in res:
        sw = oracle_sweeps[k] if oracle_sweeps and oracle_sweeps[k] else 28
        per.append(t_red + sw * t_sw)
    n3 = np.asarray(sizes, dtype=np.float64) ** 3
    scale = n3.mean() / n3[: len(per)].mean()
    mean_pencil = float(np.mean(per)) * scale
    cpu_s = sum(r[2] + r[3] for r in res)
    return {"value": cores / mean_pencil, "unit": "pencils/s", "cores": cores, "kind": "oracle",
            "host_cpu_count": os.cpu_count(),
            "sample": (f"{len(jobs)} of the {len(sizes)} pencils, one serial oracle process per "
                       f"core: reduction + 1 round-robin sweep each ({cpu_s:.0f} CPU-s, {wall:.1f} s "
                       f"wall), each pencil extrapolated to its own oracle sweep count "
                       f"(mean {mean_pencil:.0f} CPU-s per pencil at the batch's mean n^3); "
                       f"value = cores / that")}


def workload2_leg(args, ghsvd, synth, torch, dev):
    """The single n = 1024 pencil at cond(S) = 1e16: FP64 and mixed blocked
    solves (3 each), errors against its stored oracle eigenvalues, and the
    full GHSVD of its swept square factors."""
    P = synth.workload_pencil(2)
    F = ghsvd.to_device_fortran(P.F, dev)
    G = ghsvd.to_device_fortran(P.G, dev)
    J = torch.from_numpy(P.J).to(dev)
    out = {}
    for prec in ("fp64", "mixed"):
        kw = dict(precision=prec, variant="blocked", max_sweeps=args.max_sweeps)
        dt, infos, lam, _ = run_path(ghsvd, F, J, G, P, kw, 3, 1)
        emax, emed = lambda_errors(lam)
        out[f"{prec}-blocked"] = {"ms_per_pencil": 1000.0 * dt / 3, "pencils_per_s": 3 / dt,
                                  "sweeps_fp32": infos[-1]["sweeps_fp32"],
                                  "sweeps_fp64": infos[-1]["sweeps_fp64"],
                                  "status": infos[-1]["status"],
                                  "lambda_rel_err_vs_oracle": {"max": emax, "median": emed}}
        log(f"workload 2 {prec}-blocked: {out[f'{prec}-blocked']['ms_per_pencil']:.1f} ms")
    if not args.no_full:
        out["full_ghsvd"] = full_leg(ghsvd, F, J, G)
    return out


def phase1_leg(ghsvd, synth, torch, dev, reps=3):
    """Phase 1 (Section 4) on the A1- and B1-shaped atom sets: the whole
    ghsvd_phase1 call and ZHEBPJ alone (median of `reps` after one warm-up,
    HIP events on the launch stream), the product kernel's FP64 MFMA
    roofline (8 r^2 n flops per atom, r = 2 N_L), and eq. (4.2) checked on
    the first and last atom: F~_a^* J~_a F~_a = H_a^* T_a H_a."""
    out = {}
    for name, cfg in synth.PHASE1_SETS.items():
        T, H, U = synth.phase1_set(cfg["seed"], cfg["atoms"], cfg["kind"], cfg["nl"], cfg["n"])
        r, na, n = 2 * cfg["nl"], cfg["atoms"], cfg["n"]
        Td = ghsvd.atoms_to_device(T, dev)
        Hd = ghsvd.to_device_fortran(H, dev)
        Ud = torch.from_numpy(np.ascontiguousarray(U.T)).to(dev)

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                res = fn()
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            return float(np.median(ts)), res

        t_all, (F, J, G, stats) = timed(lambda: ghsvd.phase1(Td, Hd, Ud))
        t_bpj, _ = timed(lambda: ghsvd.hebpj_batched(Td))
        t_apply = max(t_all - t_bpj, 1e-6)
        flops = 8.0 * r * r * n * na
        errs = []
        for a in (0, na - 1):
            Ha = H[a * r:(a + 1) * r]
            ref = Ha.conj().T @ (T[:, :, a] @ Ha)
            Fa = F[a * r:(a + 1) * r].cpu().numpy()
            Ja = J[a * r:(a + 1) * r].cpu().numpy().astype(np.float64)
            got = Fa.conj().T @ (Ja[:, None] * Fa)
            errs.append(float(np.abs(got - ref).max() / np.abs(ref).max()))
        out[name] = {
            "atoms": na, "n_l": cfg["nl"], "n": n, "m": r * na,
            "ms": t_all, "ms_hebpj": t_bpj, "ms_product_and_g": t_apply,
            "atoms_per_s": na / (t_all / 1000.0),
            "product_roofline": {"bound": "mfma", "achieved": flops / (t_apply * 1e-3) / 1e12,
                                 "peak": 78.6, "unit": "TFLOP/s",
                                 "frac": flops / (t_apply * 1e-3) / 1e12 / 78.6,
                                 "hbm_bytes": 3.0 * r * na * n * 16,
                                 "note": "time = whole call minus ZHEBPJ alone"},
            "status_ok": bool((stats[:, 0] >= 0).all().item()),
            "eq_4_2_rel_err_sampled": max(errs)}
        log(f"phase 1 {name}: {t_all:.2f} ms (ZHEBPJ {t_bpj:.2f} ms)")
        del T, H, Td, Hd, F, G
        torch.cuda.empty_cache()
    return out


def fast_leg(ghsvd, synth, torch, dev, reps=3):
    """The explicit-formation route (Section 4.5) against the implicit HZ
    solve on well-conditioned pencils of the workload-2 shape (F 1.5n x n,
    J 3:1, G 2n x n, s log-uniform in [0.1, 1], so cond(S) <= 1e2), n = 1024
    and 2048: median wall time of `reps` calls each (inputs resident), the
    route's Jacobi sweeps, and the largest relative lambda difference."""
    out = {}
    for n in (1024, 2048):
        m = synth.rows_for(n, 1.5)
        P = synth.random_pencil(3000 + n, n, m, int(round(0.75 * m)), 2 * n, 0.1)
        F = ghsvd.to_device_fortran(P.F, dev)
        G = ghsvd.to_device_fortran(P.G, dev)
        J = torch.from_numpy(P.J).to(dev)

        def timed(fn):
            res = fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                res = fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            return 1000.0 * float(np.median(ts)), res

        t_fast, (lf, _, inf) = timed(lambda: ghsvd.solve_fast(F, J, G, cond_max=1e4))
        rec = {"n": n, "m": P.m, "p": P.p, "fast_ms": t_fast, "fast_path": inf["path"],
               "fast_sweeps": inf["sweeps"], "cond_est": inf["cond_est"]}
        for prec in ("fp64", "mixed"):
            t_hz, (lh, _, ih) = timed(lambda: ghsvd.solve(F, J, G, precision=prec,
                                                          variant="blocked"))
            rec[f"hz_{prec}_ms"] = t_hz
            rec[f"hz_{prec}_sweeps"] = ih["sweeps_fp64"] + ih["sweeps_fp32"]
            if prec == "fp64":
                a, b = lf.cpu().numpy(), lh.cpu().numpy()
                rec["max_rel_diff_fast_vs_hz"] = float(np.max(np.abs(a - b) / np.abs(b)))
        rec["speedup_vs_hz_fp64"] = rec["hz_fp64_ms"] / t_fast
        out[f"n{n}"] = rec
        log(f"fast route n={n}: {t_fast:.1f} ms ({inf['sweeps']} sweeps) vs HZ "
            f"{rec['hz_fp64_ms']:.1f} ms")
    return out


def batched_workload(args, ghsvd, synth, torch, dev):
    """The headline: 64 k-point pencils (n_k uniform in [300, 900], F
    ceil(1.5 n_k) x n_k with a 3:1 signature, G 2 n_k x n_k with s
    log-uniform in [1e-6, 1]) in one ghsvd_solve_batched call per step.  The
    timed path is mixed precision (FP32 blocked warm-up, FP64 blocked finish);
    the plain FP64 blocked and FP64 pointwise paths are timed on the same
    batch beside it, after an untimed launch-tuning call."""
    sizes = synth.workload_sizes(4)
    Ps = [synth.workload_pencil(4, k) for k in range(len(sizes))]
    Fs = [ghsvd.to_device_fortran(P.F, dev) for P in Ps]
    Gs = [ghsvd.to_device_fortran(P.G, dev) for P in Ps]
    Js = [torch.from_numpy(P.J).to(dev) for P in Ps]
    log(f"{len(Ps)} pencils built, n in [{min(sizes)}, {max(sizes)}]")
    ref, oracle_sweeps = golden_batch(GOLDEN4, Ps)
    w, wpp, trials = ghsvd.autotune(Fs, Js, Gs, variant="blocked")
    if args.block_width:
        w = args.block_width
    tuned = {"block_width": w, "waves_per_pair": wpp, "trial_ms": trials}
    log(f"tuned: w={w}, waves per pair {wpp}")
    inner = args.inner
    kw = dict(variant="blocked", max_sweeps=args.max_sweeps, block_width=w, waves_per_pair=wpp,
              inner_order=inner)
    prime(ghsvd, synth, torch, dev, dict(kw, precision="mixed"))
    paths, kern, lams = {}, {}, {}
    plan = [("mixed", "blocked", args.steps, args.warmup),
            ("fp64", "blocked", max(3, args.steps // 4), 1)]
    if not args.no_compare:
        plan.append(("fp64", "pointwise", 2, 0))
    for prec, var, steps, warm in plan:
        pkw = dict(kw, precision=prec, variant=var)
        log(f"timing {prec}-{var}: {steps} steps after {warm} warm-up")
        dt, infos, lam, times, rc = time_batch(ghsvd, torch, Fs, Js, Gs, pkw, steps, warm,
                                               args.profile_every if var == "blocked" else 0)
        key = f"{prec}-{var}"
        lams[key] = lam
        for inf, P in zip(infos, Ps):
            inf.update(n=P.n, m=P.m, p=P.p, reduced=P.m > P.n or P.p > P.n)
        rec = {"pencils_per_s": len(Ps) * steps / dt, "ms_per_batch": 1000.0 * dt / steps,
               "steps": steps, "warmup": warm, "status": rc,
               "max_sweeps_fp32": max(i["sweeps_fp32"] for i in infos),
               "max_sweeps_fp64": max(i["sweeps_fp64"] for i in infos),
               "mean_sweeps_fp32": float(np.mean([i["sweeps_fp32"] for i in infos])),
               "mean_sweeps_fp64": float(np.mean([i["sweeps_fp64"] for i in infos])),
               "pair_updates_per_s": sum(i["pairs_visited"] for i in infos) * steps / dt}
        if ref is not None:
            rec["lambda_rel_err_vs_oracle"] = batch_errors(lam, ref)
        paths[key] = rec
        if times:
            kern[key] = batch_rooflines(times, infos, w, inner, steps, fp32_blocked=var == "blocked")
        log(f"{key}: {rec['ms_per_batch']:.1f} ms per batch, status {rc}")
    for key in paths:
        if key != "fp64-blocked":
            paths[key]["max_rel_diff_vs_fp64_blocked"] = max(
                float(np.max(np.abs(a - b) / np.abs(b))) for a, b in zip(lams[key],
                                                                         lams["fp64-blocked"]))
    head = paths["mixed-blocked"]
    rec = {
        "metric": METRIC, "value": head["pencils_per_s"], "unit": "pencils/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_batch"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": ("64 k-point pencils, n_k uniform in [300,900], F ceil(1.5 n_k) x "
                                "n_k Gaussian, J 3:1, G 2 n_k x n_k = U diag(s) W^*, s "
                                "log-uniform [1e-6,1] (cond S <= 1e12), complex128, one batched "
                                "call per step: reduction + FP32 blocked warm-up + FP64 blocked "
                                "finish + lambda, X"),
                   "batch": len(Ps), "n_min": int(min(sizes)), "n_max": int(max(sizes)),
                   "precision": "mixed", "variant": "blocked", "inner": inner,
                   "block_width": w, "waves_per_pair": wpp},
        "pair_updates_per_s": head["pair_updates_per_s"],
        "lambda_rel_err_vs_oracle": head.get("lambda_rel_err_vs_oracle"),
        "vs_fp64_blocked": head["pencils_per_s"] / paths["fp64-blocked"]["pencils_per_s"],
        "paths": paths, "tuned": tuned,
    }
    km = kern.get("mixed-blocked", {})
    # the dominant single kernel ("reduce" brackets the three or four
    # launches of a reduction column step and is reported in `kernels`)
    single = [k for k in km if k != "reduce"]
    if single:
        dom = max(single, key=lambda k: km[k]["total_ms_est"])
        d = km[dom]
        rec["roofline"] = {
            "bound": d["bound"], "kernel": KERNEL_NAMES.get(dom, dom),
            "achieved": d["achieved"], "peak": d["peak"], "unit": d["unit"], "frac": d["frac"],
            "traffic": d["traffic"], "mean_launch_us": d["mean_us"],
            "work_per_launch": d["work_per_launch"], "work_unit": d["work_unit"],
            "timed_launches": d["timed_launches"], "launches": d["launches"]}
    rec["kernels"] = kern
    if not args.no_workload2:
        rec["workload2"] = workload2_leg(args, ghsvd, synth, torch, dev)
    if not args.no_phase1:
        rec["phase1"] = phase1_leg(ghsvd, synth, torch, dev)
    if not args.no_fast:
        rec["explicit_formation"] = fast_leg(ghsvd, synth, torch, dev)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        rec["cpu_baseline"] = cpu_baseline_batched(sizes, oracle_sweeps,
                                                   min(16, os.cpu_count() or 1))
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
    ap.add_argument("--inner", default="cross",
                    choices=["cross", "full", "fb", "full_jqr", "fb_jqr", "ml_bo", "ml_fb"],
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
    ap.add_argument("--workload", type=int, default=4, choices=[2, 3, 4, 5],
                    help="4: the batch of 64 pencils (default, the headline); 2: the single "
                         "n=1024 pencil; 3: one n=4096 pencil; 5: the batch of 16 large pencils")
    ap.add_argument("--no-workload2", action="store_true",
                    help="workload 4: skip the single-pencil n=1024 leg")
    ap.add_argument("--no-phase1", action="store_true",
                    help="workload 4: skip the Phase 1 leg (A1- and B1-shaped atom sets)")
    ap.add_argument("--phase1-only", action="store_true",
                    help="only run the Phase 1 leg and print its record")
    ap.add_argument("--no-fast", action="store_true",
                    help="workload 4: skip the explicit-formation leg")
    ap.add_argument("--fast-only", action="store_true",
                    help="only run the explicit-formation leg and print its record")
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
    if args.phase1_only:
        print(json.dumps({"phase1": phase1_leg(ghsvd, synth, torch, dev)}), flush=True)
        return
    if args.fast_only:
        print(json.dumps({"explicit_formation": fast_leg(ghsvd, synth, torch, dev)}), flush=True)
        return
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
    n = P.n
    w = args.block_width or block_width_for(n)
    info.update(n=n, m=P.m, p=P.p, reduced=not args.no_reduce and (P.m > n or P.p > n))
    kr = batch_rooflines(times, [info], w, args.inner, args.steps,
                         fp32_blocked=args.variant == "blocked")
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
