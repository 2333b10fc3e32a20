"""Benchmark of the IETI-DP hot path on one MI355X.

A step is one time-to-solution (TTS): ieti_factor (local factorisations and
coarse setup on the GPU) followed by ieti_solve (right-hand side, PCG on the
multipliers to rtol 1e-8 with the Dirichlet preconditioner, recovery of the
solution).  Host assembly and the upload to HBM happen before the timed
region.  The default workload is ``cube64``: 4x4x4 patches, p=3, 8 elements
per patch and direction (123,201 DOFs), 16 uneven subdomains, reluctivity
1 or 1e-3, random trigonometric source, plain FP64.

Prints one JSON line (rank 0): value = solves per second (1 / TTS).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6

WORKLOADS = {
    "cube64": "cube64: 4x4x4 patches, p=3, n_el=8, 16 uneven subdomains (1-8 patches), nu in {1,1e-3}, "
              "trig J, FP64, rtol 1e-8",
    "cube8": "cube8: 2x2x2 patches, p=2, n_el=4, 8 subdomains, nu=1, manufactured polynomial A, FP64",
    "cube256": "cube256: 8x8x4 patches, p=2, n_el=6, 64 uneven subdomains, nu log-uniform [1e-3,1], trig J, FP64",
    "ring576": "ring576: NURBS annulus 48x3x4 patches, p=2, n_el=5, 48 sector subdomains, coil current, FP64",
    "stream256": "stream256: 256 independent box problems in batches",
}


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "cube64_hbm_traffic_pmc.md")
# the per-launch traffic depends on the kernels and on the factorisation's task lists
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_2501_04340_amd", "csrc", "device", "kernels.hip"),
                   os.path.join(ROOT, "paper_2501_04340_amd", "csrc", "host", "plan.cpp")]


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` ("k_update_multi", "k_gemv_sym<double>"
    or "k_gemv<double>") on `workload` from the committed PMC summary, or None
    when the summary holds no figure for that kernel on that workload, or when
    the kernel source or the task-list builder changed since the counters were
    taken."""
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
        sha = sources_sha256()
    except OSError:
        return None
    pat = (r"traffic_per_launch " + re.escape(kernel)
           + r": workload=(\S+) .*total_bytes=(\d+) sources_sha256=([0-9a-f]+)")
    for m in re.finditer(pat, text):
        if m.group(1) == workload and m.group(3) == sha:
            return float(m.group(2))
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(prob, iters, budget_s=20.0):
    """Time the CPU oracle on a bounded sample of the same workload.

    Sample: the oracle's setup (SuperLU factorisations of K_rr and K_VV, the
    n_gp coarse solves and the right-hand-side solve) and its per-iteration
    local work (one K_rr solve for the operator, one K_VV solve for the
    preconditioner) for whole subdomains taken in index order until the
    budget is used.  The time of the full solve is extrapolated to all
    subdomains with cost ~ n_r^2 for the setup and ~ n_r^(4/3) per
    iteration (nested-dissection sparse Cholesky in 3D), times the GPU run's
    PCG iteration count.  Host assembly is excluded as on the GPU side.
    """
    from threadpoolctl import threadpool_limits

    from oracle.ietidp import LocalProblem
    from oracle.space import Space
    from oracle.topology import build_topology
    import scipy.sparse as sp

    space = Space(prob)
    topo = build_topology(space)
    n_r = np.array([len(r) for r in topo.sub_r], dtype=np.float64)
    ed = space.element_data(0)
    setup_t, iter_t, used = {}, {}, []
    t_start = time.perf_counter()
    with threadpool_limits(limits=1):
        for k in range(topo.n_sub):
            if time.perf_counter() - t_start > budget_s and used:
                break
            pats = np.flatnonzero(prob.patch_to_sub == k)
            Kk = None
            jk = np.zeros(space.n_edges)
            for q in pats:
                K, j = space.assemble_patch(int(q), True, ed=ed)
                g = space.patch_local_edges(int(q))
                r, c = np.nonzero(K)
                M = sp.csr_matrix((prob.nu[q] * K[r, c], (g[r], g[c])), shape=(space.n_edges, space.n_edges))
                Kk = M if Kk is None else Kk + M
                np.add.at(jk, g, j)
            t0 = time.perf_counter()
            L = LocalProblem(k, Kk, jk, topo.sub_r[k], topo.sub_p[k], topo.sub_I[k], topo.gp_index, topo.m_r,
                             topo.mult)
            KrpC = L.K_rp @ L.C
            for c in range(KrpC.shape[1]):
                L.solve(KrpC[:, c])
            L.solve(L.j_r)
            t1 = time.perf_counter()
            u = np.random.default_rng(k).standard_normal(len(L.r))
            reps = 3
            for _ in range(reps):
                L.solve(u)
                if len(L.I):
                    L.schur_I(u[L.I])
            t2 = time.perf_counter()
            setup_t[k] = t1 - t0
            iter_t[k] = (t2 - t1) / reps
            used.append(k)
    ks = np.array(used)
    c_setup = np.sum([setup_t[k] for k in used]) / np.sum(n_r[ks] ** 2)
    c_iter = np.sum([iter_t[k] for k in used]) / np.sum(n_r[ks] ** (4.0 / 3.0))
    tts = c_setup * np.sum(n_r ** 2) + iters * c_iter * np.sum(n_r ** (4.0 / 3.0))
    return {
        "value": 1.0 / tts,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle setup + {iters} PCG iterations of local solves measured on subdomains {used} "
                   f"({len(used)}/{topo.n_sub}, {time.perf_counter() - t_start:.1f}s of CPU), extrapolated to "
                   f"all subdomains with n_r^2 (setup) and n_r^(4/3) (per iteration); est. TTS {tts:.1f}s"),
    }


def ring_warm_start(args):
    """ring576: train the warm-start network on 512 solver-generated solves,
    then time 64 held-out draws cold and warm, plain FP64 and mixed."""
    import torch

    from paper_2501_04340_amd import Solver
    from paper_2501_04340_amd.ietidp import PREC_FP64, PREC_MIXED
    from paper_2501_04340_amd.warmstart import RingWarmStart
    from workloads import configs

    torch.cuda.set_device(0)
    fkw = {} if args.gemv_variant is None else {"gemv_variant": args.gemv_variant}
    prob = configs.ring576()
    t0 = time.perf_counter()
    S = Solver(prob)
    log(f"host assembly {time.perf_counter() - t0:.1f}s sizes {S.sizes()}")
    W = RingWarmStart(S, prob, window=2, hidden=args.nn_hidden, layers=2)

    def draw(i):
        nu, cur = configs.ring_coefficients(configs.ring_sample_seed(i))
        return nu, configs.ring_load_scale(cur)

    n_train, n_test = args.ring_train, args.ring_test
    t0 = time.perf_counter()
    X, Cc, T, gst = W.generate([draw(i) for i in range(n_train)], rtol=1e-10, log=log)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    losses = W.fit(X, Cc, T, epochs=args.nn_epochs, lr=args.nn_lr, batch=256, seed=0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"data {t_gen:.1f}s, training {t_train:.1f}s, loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    W.attach()
    variants = {"plain_cold": (PREC_FP64, False), "plain_warm": (PREC_FP64, True),
                "mixed_cold": (PREC_MIXED, False), "mixed_warm": (PREC_MIXED, True)}
    res = {k: {"tts_ms": [], "iters": [], "r0": [], "fallback": 0, "applies": 0, "pcg_s": 0.0} for k in variants}
    lam_err = []
    for i in range(n_train, n_train + n_test):
        nu, scale = draw(i)
        S.set_coefficients(nu, scale)
        lam_ref = None
        for name, (prec, warm) in variants.items():
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            S.factor(precision=prec, **fkw)
            _, st = S.solve(rtol=args.rtol, warm_start=warm)
            torch.cuda.synchronize()
            r = res[name]
            r["tts_ms"].append((time.perf_counter() - t1) * 1e3)
            r["iters"].append(st["iters"])
            r["r0"].append(st["rel_residual0"])
            r["fallback"] += int(st["warm_start"] == -1)
            r["applies"] += st["f_applies"]
            r["pcg_s"] += st["t_pcg_s"]
            lam = S.lambda_()
            if lam_ref is None:
                lam_ref = lam
            else:
                lam_err.append(float(np.linalg.norm(lam - lam_ref) / np.linalg.norm(lam_ref)))
        if (i - n_train + 1) % 16 == 0:
            log(f"held-out {i - n_train + 1}/{n_test}: " + ", ".join(
                f"{k} {np.median(v['tts_ms']):.1f}ms/{np.mean(v['iters']):.1f}it" for k, v in res.items()))
    S.factor(precision=PREC_FP64, **fkw)
    summ = {}
    for k, v in res.items():
        summ[k] = {"tts_ms_p50": float(np.median(v["tts_ms"])), "tts_ms_p99": float(np.percentile(v["tts_ms"], 99)),
                   "pcg_iters_mean": float(np.mean(v["iters"])), "rel_residual0_median": float(np.median(v["r0"])),
                   "fallbacks": v["fallback"], "f_applies_per_s": v["applies"] / v["pcg_s"] if v["pcg_s"] else None}
    base = summ["plain_cold"]["tts_ms_p50"]
    for k in summ:
        summ[k]["speedup_vs_plain_cold"] = base / summ[k]["tts_ms_p50"]
    ms = summ["mixed_warm"]["tts_ms_p50"]
    out = {
        "metric": "IETI-DP time-to-solution and F·λ applies/s at rtol 1e-8, mixed+warm vs plain FP64",
        "value": 1e3 / ms, "unit": "solves/s", "n_gpus": 1, "steps": n_test, "warmup": 0, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS["ring576"], "variant": "mixed + warm start, held-out draws",
                   "n_g": S.n_global, "n_sub": S.n_sub, "m_r": S.m_r, "n_gp": S.n_gp, "rtol": args.rtol},
        "variants": summ,
        "warm_start": {"train_solves": n_train, "held_out": n_test, "data_s": t_gen, "train_s": t_train,
                       "epochs": args.nn_epochs, "hidden": args.nn_hidden, "params": W.net.n_params,
                       "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
                       "loss_curve": [float(x) for x in losses[:: max(1, len(losses) // 20)]],
                       "lambda_rel_diff_vs_plain_cold_max": max(lam_err) if lam_err else None},
    }
    print(json.dumps(out), flush=True)


def stream_batches(args):
    """stream256: independent box problems, each solved alone (plain FP64,
    one handle per problem) and in batches (one handle and one set of
    launches per chunk, plain FP64 and mixed).  Host assembly is untimed."""
    import concurrent.futures

    import torch

    from paper_2501_04340_amd import Solver
    from paper_2501_04340_amd.ietidp import GEMV_SYM, PREC_FP64, PREC_MIXED
    from workloads import configs

    torch.cuda.set_device(0)
    fkw = {} if args.gemv_variant is None else {"gemv_variant": args.gemv_variant}
    n, chunk = args.stream_count, args.stream_chunk
    lat_single, lat_bplain, lat_bmixed = [], [], []
    t_single = t_bplain = t_bmixed = 0.0
    iters_single, iters_batch, resid = [], [], []
    roof = None
    max_diff = 0.0
    n_g_total = 0
    t_host = 0.0
    for c0 in range(0, n, chunk):
        ids = list(range(c0, min(n, c0 + chunk)))
        th = time.perf_counter()
        probs = [configs.stream_problem(i) for i in ids]
        with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
            singles = list(ex.map(Solver, probs))
        t_host += time.perf_counter() - th
        # each problem alone, plain FP64 (first factor autotunes; one warm-up solve)
        outs = []
        for S in singles:
            S.factor(**fkw)
            S.solve(rtol=args.rtol)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.factor(**fkw)
            a, st = S.solve(rtol=args.rtol)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            lat_single.append(dt * 1e3)
            t_single += dt
            iters_single.append(st["iters"])
            outs.append(a)
            n_g_total += S.n_global
        kts = [S.kernel_times() for S in singles]  # interface-block bytes per application, both layouts
        B = Solver.batch_of(singles)
        for S in singles:
            S.close()
        for prec, lat in ((PREC_FP64, lat_bplain), (PREC_MIXED, lat_bmixed)):
            B.factor(precision=prec, **fkw)
            B.solve(rtol=args.rtol, maxit=3000)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.factor(precision=prec, **fkw)
            a, st = B.solve(rtol=args.rtol, maxit=3000)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            lat.extend([dt * 1e3] * len(ids))
            info = B.batch_info()
            resid.extend(b["rel_residual"] for b in info)
            if prec == PREC_FP64:
                t_bplain += dt
                iters_batch.extend(b["iters"] for b in info)
                for ai, ao in zip(B.split(a), outs):
                    max_diff = max(max_diff, float(np.abs(ai - ao).max() / max(np.abs(ao).max(), 1e-300)))
            else:
                t_bmixed += dt
        if roof is None:
            # a finished problem's GEMV tasks are skipped, so the bytes of the
            # profiled solve are sum_p bytes_p * (2 iters_p + 1): one
            # preconditioner application to start, two applications per iteration
            B.factor(**fkw)
            B.set_profiling(True)
            B.solve(rtol=args.rtol, maxit=3000)
            kt = B.kernel_times()
            B.set_profiling(False)
            its = [b["iters"] for b in B.batch_info()]
            bsym = int(B.gemv_tuning()[0][0]) == GEMV_SYM
            bytes_p = [k["gemv_bytes_lower" if bsym else "gemv_bytes_full"] for k in kts]
            total_bytes = float(sum(bp * (2 * it + 1) for bp, it in zip(bytes_p, its)))
            ach = total_bytes / (kt["gemv_ms"] * 1e-3) / 1e9
            kname = "k_gemv_sym<double>" if bsym else "k_gemv<double>"
            shape = "autotuned shape" if args.gemv_variant is None else "pinned shape"
            roof = {"kernel": f"{kname} ({shape}), one batch of "
                              f"{len(ids)} problems", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
                    "avg_launch_ms": kt["gemv_ms"] / max(kt["gemv_launches"], 1),
                    "bytes_all_problems_active": kt["gemv_bytes"],
                    "bytes_over_solve": total_bytes, "launches": kt["gemv_launches"]}
        B.close()
        log(f"problems {ids[0]}..{ids[-1]}: alone {np.sum(lat_single[-len(ids):]):.0f} ms total, batch plain "
            f"{lat_bplain[-1]:.0f} ms, batch mixed {lat_bmixed[-1]:.0f} ms (host {t_host:.0f}s so far)")

    def summ(lat, total):
        return {"solves_per_s": n / total, "latency_ms_p50": float(np.percentile(lat, 50)),
                "latency_ms_p99": float(np.percentile(lat, 99))}

    out = {
        "metric": "IETI-DP time-to-solution and F·λ applies/s at rtol 1e-8, mixed+warm vs plain FP64",
        "value": n / t_bmixed, "unit": "solves/s", "n_gpus": 1, "steps": n, "warmup": 1,
        "ms_per_step": t_bmixed * 1e3 / n, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"stream256: {n} independent box problems (2^a x 2^b x 2^c patches, p in {{2,3}}, "
                               f"4-6 elements, nu in [1e-3,1]), batches of {chunk}, rtol {args.rtol}",
                   "variant": "batched mixed precision (no warm start: no network is trained for this stream)",
                   "n_g_total": n_g_total},
        "variants": {"single_plain_fp64": summ(lat_single, t_single), "batch_plain_fp64": summ(lat_bplain, t_bplain),
                     "batch_mixed": summ(lat_bmixed, t_bmixed)},
        "speedup_batch_mixed_vs_single_plain": t_single / t_bmixed,
        "pcg_iters": {"single_mean": float(np.mean(iters_single)), "batch_max_mean": float(np.mean(iters_batch))},
        "max_rel_residual": float(np.max(resid)),
        "batch_vs_single_max_rel_diff": max_diff,
        "host_assembly_s": t_host,
        "roofline": roof,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cube64", choices=sorted(WORKLOADS))
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 3 device-to-device copies of MIB MiB (HBM counter calibration) and exit")
    ap.add_argument("--stream-count", type=int, default=256)
    ap.add_argument("--stream-chunk", type=int, default=32)
    ap.add_argument("--ring-train", type=int, default=512)
    ap.add_argument("--ring-test", type=int, default=64)
    ap.add_argument("--nn-epochs", type=int, default=300)
    ap.add_argument("--nn-hidden", type=int, default=256)
    ap.add_argument("--nn-lr", type=float, default=1e-3)
    ap.add_argument("--gemv-variant", type=int, default=None, metavar="V",
                    help="force the interface GEMV launch shape (0-11 row streaming, 12 symmetric) instead of "
                         "the autotuner's choice; for profiled runs, where tracing adds a cost to every launch "
                         "and so favours shapes with fewer launches")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested); the multi-GPU sharding "
              "of the subdomains is a design, not a measured path.", flush=True)
        sys.exit(2)

    import torch

    from paper_2501_04340_amd import Solver
    from paper_2501_04340_amd.ietidp import GEMV_SYM
    from workloads import configs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20)
        x = torch.ones(n, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": n, "launches": 3}), flush=True)
        return
    if args.workload == "ring576":
        return ring_warm_start(args)
    if args.workload == "stream256":
        return stream_batches(args)
    torch.cuda.set_device(0)
    prob = configs.make_config(args.workload)
    t0 = time.perf_counter()
    S = Solver(prob)
    fkw = {} if args.gemv_variant is None else {"gemv_variant": args.gemv_variant}
    log(f"host assembly {time.perf_counter() - t0:.1f}s sizes {S.sizes()}")
    info = S.plan_info()
    # the solution stays in HBM (a device buffer), as the inputs do
    a_dev = torch.empty(S.n_edges, dtype=torch.float64, device="cuda")
    for w in range(args.warmup):
        S.factor(**fkw)
        st = S.solve_device(a_dev.data_ptr(), rtol=args.rtol)
        log(f"warmup {w}: iters {st['iters']} factor {st['t_factor_s'] * 1e3:.1f}ms solve {st['t_solve_s'] * 1e3:.1f}ms")
    torch.cuda.synchronize()
    stats, step_ms = [], []
    t_begin = time.perf_counter()
    for k in range(args.steps):
        t_k = time.perf_counter()
        S.factor(**fkw)
        st = S.solve_device(a_dev.data_ptr(), rtol=args.rtol)  # returns after a stream synchronisation
        step_ms.append((time.perf_counter() - t_k) * 1e3)
        stats.append(st)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    # kernel durations: one more step with launch events on every GEMV and
    # update launch (direct launches; the timed steps replay a hipGraph)
    S.set_profiling(True)
    S.factor(**fkw)
    S.solve(rtol=args.rtol)
    kt = S.kernel_times()
    S.set_profiling(False)
    # condition number of the preconditioned interface operator (Section 4)
    # from the recorded PCG coefficients of one more (untimed) solve
    S.record_pcg(4000)
    S.solve(rtol=args.rtol)
    lo, hi = S.condition()
    S.record_pcg(0)
    ms_per_step = (t_end - t_begin) * 1e3 / args.steps
    iters = int(np.median([s["iters"] for s in stats]))
    applies = sum(s["f_applies"] for s in stats)
    pcg_s = sum(s["t_pcg_s"] for s in stats)
    factor_ms = float(np.median([s["t_factor_s"] for s in stats])) * 1e3
    solve_ms = float(np.median([s["t_solve_s"] for s in stats])) * 1e3
    log(f"timed: {ms_per_step:.2f} ms/step, iters {iters}, factor {factor_ms:.2f} ms, solve {solve_ms:.2f} ms, "
        f"kernels {kt}")
    # roofline of the dominant kernel (largest total time per step): the
    # factorisation's tile update (FP64 MFMA) or the interface GEMV (HBM)
    chosen, tune_ms = S.gemv_tuning()
    sym = int(chosen[0]) == GEMV_SYM
    gemv_name = "k_gemv_sym<double>" if sym else "k_gemv<double>"
    gemv_ms = kt["gemv_ms"] / max(kt["gemv_launches"], 1)
    gemv_ach = kt["gemv_bytes"] / (gemv_ms * 1e-3) / 1e9
    roof_gemv = {"kernel": gemv_name, "bound": "hbm", "achieved": gemv_ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": gemv_ach / HBM_PEAK_GBS, "traffic": measured_traffic(gemv_name, args.workload),
                 "avg_launch_ms": gemv_ms, "bytes_per_launch": kt["gemv_bytes"],
                 "launches_per_step": kt["gemv_launches"], "ms_per_step": kt["gemv_ms"]}
    flops_per_task = 2.0 * 64 ** 3
    upd_avg = kt["update_ms"] / max(kt["update_launches"], 1)
    upd_flops = kt["update_tasks"] / max(kt["update_launches"], 1) * flops_per_task
    upd_ach = upd_flops / (upd_avg * 1e-3) / 1e12
    roof_upd = {"kernel": "k_update_multi", "bound": "mfma", "achieved": upd_ach, "peak": FP64_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": upd_ach / FP64_MFMA_PEAK_TFLOPS, "traffic": measured_traffic("k_update_multi", args.workload),
                "avg_launch_ms": upd_avg, "flops_per_launch": upd_flops,
                "launches_per_step": kt["update_launches"], "ms_per_step": kt["update_ms"]}
    roof = dict(roof_gemv if kt["gemv_ms"] >= kt["update_ms"] else roof_upd)
    roof["other"] = roof_upd if roof["kernel"] == gemv_name else roof_gemv
    log(f"GEMV autotuner (FP64 blocks): chosen shape {chosen[0]}, ms per shape {np.round(tune_ms[0], 4).tolist()}")
    # mixed-precision variant of the same step (FP32-stored interface blocks in
    # the inner PCG, outer refinement on the FP64 residual)
    from paper_2501_04340_amd.ietidp import PREC_FP64, PREC_MIXED
    S.factor(precision=PREC_MIXED, **fkw)
    S.solve(rtol=args.rtol)
    torch.cuda.synchronize()
    mstats = []
    t0m = time.perf_counter()
    for k in range(args.steps):
        S.factor(precision=PREC_MIXED, **fkw)
        st_m = S.solve_device(a_dev.data_ptr(), rtol=args.rtol)
        mstats.append(st_m)
    torch.cuda.synchronize()
    ms_mixed = (time.perf_counter() - t0m) * 1e3 / args.steps
    chosen32, tune_ms32 = S.gemv_tuning()
    S.set_profiling(True)
    S.factor(precision=PREC_MIXED, **fkw)
    _, st_mp = S.solve(rtol=args.rtol)
    kt_m = S.kernel_times()
    S.set_profiling(False)
    log(f"mixed, profiled solve (direct launches): pcg {st_mp['t_pcg_s'] * 1e3:.2f} ms, {kt_m['gemv_launches']:.0f} "
        f"GEMV launches taking {kt_m['gemv_ms']:.2f} ms")
    # rho-scaled preconditioner (stiffness diagonal), plain and mixed
    from paper_2501_04340_amd.ietidp import SCALE_STIFFNESS
    scaled = {}
    for tag, prec in (("plain_fp64_rho_scaling", PREC_FP64), ("mixed_rho_scaling", PREC_MIXED)):
        S.factor(precision=prec, scaling=SCALE_STIFFNESS, **fkw)
        S.solve(rtol=args.rtol)
        torch.cuda.synchronize()
        t0s = time.perf_counter()
        for k in range(args.steps):
            S.factor(precision=prec, scaling=SCALE_STIFFNESS, **fkw)
            st_s = S.solve_device(a_dev.data_ptr(), rtol=args.rtol)
        torch.cuda.synchronize()
        ms_s = (time.perf_counter() - t0s) * 1e3 / args.steps
        scaled[tag] = {"tts_ms": ms_s, "pcg_iters": int(st_s["iters"]), "rel_residual_fp64": float(st_s["rel_residual"]),
                       "speedup_vs_plain": ms_per_step / ms_s}
        log(f"{tag}: {ms_s:.2f} ms/step, iters {st_s['iters']}")
    S.factor(precision=PREC_FP64, **fkw)
    mfac = float(np.median([x["t_factor_s"] for x in mstats])) * 1e3
    msol = float(np.median([x["t_solve_s"] for x in mstats])) * 1e3
    mpcg = float(np.median([x["t_pcg_s"] for x in mstats])) * 1e3
    log(f"mixed: {ms_mixed:.2f} ms/step (factor {mfac:.2f}, solve {msol:.2f}, pcg {mpcg:.2f}), iters "
        f"{mstats[-1]['iters']}, outer {mstats[-1]['outer_iters']}, rel residual {mstats[-1]['rel_residual']:.2e}; "
        f"plain pcg {float(np.median([x['t_pcg_s'] for x in stats])) * 1e3:.2f}")
    out = {
        "metric": "IETI-DP time-to-solution and F·λ applies/s at rtol 1e-8, mixed+warm vs plain FP64",
        "value": 1e3 / ms_per_step,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "variant": "plain FP64", "n_g": S.n_global,
                   "n_sub": S.n_sub, "m_r": S.m_r, "n_gp": S.n_gp, "rtol": args.rtol},
        "tts_ms": ms_per_step,
        "tts_ms_median": float(np.median(step_ms)),
        "factor_ms": factor_ms,
        "solve_ms": solve_ms,
        "pcg_iters": iters,
        "kappa_lanczos": hi / lo,
        "f_applies_per_s": applies / pcg_s if pcg_s > 0 else None,
        "rel_residual": float(stats[-1]["rel_residual"]),
        "factor_tflops": info["flops"] / (factor_ms * 1e-3) / 1e12,
        "roofline": roof,
        "gemv_autotune": {"fp64_shape": int(chosen[0]), "fp64_ms": [float(x) for x in tune_ms[0]],
                          "fp32_shape": int(chosen32[1]), "fp32_ms": [float(x) for x in tune_ms32[1]]},
        "variants": {
            "plain_fp64": {"tts_ms": ms_per_step, "pcg_iters": iters},
            "mixed_fp32_blocks_fp64_refinement": {
                "tts_ms": ms_mixed, "factor_ms": mfac, "solve_ms": msol, "pcg_ms": mpcg,
                "pcg_iters": int(mstats[-1]["iters"]),
                "outer_iters": int(mstats[-1]["outer_iters"]),
                "rel_residual_fp64": float(mstats[-1]["rel_residual"]),
                "speedup_vs_plain": ms_per_step / ms_mixed},
            **scaled,
        },
    }
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(prob, iters, args.cpu_budget)
        log(f"cpu baseline {time.perf_counter() - t0:.1f}s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
