"""Benchmark of the IETI-DP hot path on one MI355X.

A time-to-solution (TTS) is ieti_factor (local factorisations and coarse
setup on the GPU) followed by ieti_solve (right-hand side, PCG on the
multipliers to rtol 1e-8 with the Dirichlet preconditioner, recovery of the
solution).  Host assembly and the upload to HBM happen before the timed
region.

The default workload is ``stream256``: 256 independent box problems
(2^a x 2^b x 2^c patches, p in {2, 3}, 4-6 elements, random reluctivity and
source), solved in batches of 64 problems per handle, batched mixed
precision against batched plain FP64 and each problem alone; a step is one
pass over the whole stream and value = problems solved per second.
``--workload cube64`` (and cube8, cube256, ring576) time single problems:
a step is one TTS, value = 1 / TTS.

Prints one JSON line (rank 0).
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


# PMC traffic summaries (rocprofv3 FETCH_SIZE / WRITE_SIZE passes) by workload
TRAFFIC_PROFILES = [os.path.join(ROOT, "profiles", "stream256_batch64_hbm_traffic_pmc.md"),
                    os.path.join(ROOT, "profiles", "cube64_hbm_traffic_pmc.md"),
                    os.path.join(ROOT, "profiles", "cube256_hbm_traffic_pmc.md")]
# the per-launch traffic depends on the kernels and on the factorisation's task lists
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_2501_04340_amd", "csrc", "device", "kernels.hip"),
                   os.path.join(ROOT, "paper_2501_04340_amd", "csrc", "device", "kernels.hpp"),
                   os.path.join(ROOT, "paper_2501_04340_amd", "csrc", "host", "plan.cpp")]


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload, params=None):
    """HBM bytes per launch of `kernel` ("k_update_multi", "k_gemv_sym<double>",
    "k_gemv_sym<float>" or "k_gemv<double>") on `workload` from the committed
    PMC summaries, or None when they hold no figure for that kernel on that
    workload, when the kernel source or the task-list builder changed since
    the counters were taken, or (for the tile update, whose launches are the
    deferred-update groups) when the counters were taken with other schedule
    parameters than `params` = (defer, defer_tail, update_wgs)."""
    import re
    try:
        sha = sources_sha256()
    except OSError:
        return None
    text = ""
    for f in TRAFFIC_PROFILES:
        try:
            text += open(f).read() + "\n"
        except OSError:
            pass
    pat = r"traffic_per_launch " + re.escape(kernel) + r": (.*)"
    for m in re.finditer(pat, text):
        fields = dict(kv.split("=", 1) for kv in m.group(1).split() if "=" in kv)
        if fields.get("workload") != workload or fields.get("sources_sha256") != sha:
            continue
        if kernel.startswith("k_update") and (params is None or fields.get("params")
                                              != ",".join(str(int(x)) for x in params)):
            continue
        return float(fields["total_bytes"])
    return None


def factor_summary(info, factor_s):
    """The factorisation's rate against the FP64 matrix peak, counted three
    ways: the 64x64 tile products it executes (padding and tile-level fill
    included), and the scalar Cholesky work sum_j c_j^2 in the same
    elimination order, of K_rr alone (the method's local factorisations) and
    with the augmented trailing rows that yield the explicit interface
    blocks."""
    out = {"factor_ms": factor_s * 1e3, "tile_flops": info["flops"],
           "scalar_flops_krr": info["flops_scalar_rr"], "scalar_flops_augmented": info["flops_scalar_aug"]}
    for key, f in (("tile", info["flops"]), ("scalar_krr", info["flops_scalar_rr"]),
                   ("scalar_augmented", info["flops_scalar_aug"])):
        tf = f / factor_s / 1e12 if factor_s > 0 else 0.0
        out[f"{key}_tflops"] = tf
        out[f"{key}_frac_fp64_mfma"] = tf / FP64_MFMA_PEAK_TFLOPS
    return out


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
    res = {k: {"tts_ms": [], "iters": [], "r0": [], "fallback": 0, "applies": 0, "pcg_s": 0.0, "factor_ms": [],
               "solve_ms": []} for k in variants}
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
            r["factor_ms"].append(st["t_factor_s"] * 1e3)
            r["solve_ms"].append(st["t_solve_s"] * 1e3)
            lam = S.lambda_()
            if lam_ref is None:
                lam_ref = lam
            else:
                lam_err.append(float(np.linalg.norm(lam - lam_ref) / np.linalg.norm(lam_ref)))
        if (i - n_train + 1) % 16 == 0:
            log(f"held-out {i - n_train + 1}/{n_test}: " + ", ".join(
                f"{k} {np.median(v['tts_ms']):.1f}ms/{np.mean(v['iters']):.1f}it" for k, v in res.items()))
    S.factor(precision=PREC_FP64, **fkw)
    chosen, tune_ms = S.gemv_tuning()
    summ = {}
    for k, v in res.items():
        summ[k] = {"tts_ms_p50": float(np.median(v["tts_ms"])), "tts_ms_p99": float(np.percentile(v["tts_ms"], 99)),
                   "pcg_iters_mean": float(np.mean(v["iters"])), "rel_residual0_median": float(np.median(v["r0"])),
                   "fallbacks": v["fallback"], "f_applies_per_s": v["applies"] / v["pcg_s"] if v["pcg_s"] else None,
                   "factor_ms_p50": float(np.median(v["factor_ms"])), "solve_ms_p50": float(np.median(v["solve_ms"]))}
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
        "gemv_autotune": {"fp64_shape": int(chosen[0]), "fp64_ms": [float(x) for x in tune_ms[0]],
                          "fp32_shape": int(chosen[1]), "fp32_ms": [float(x) for x in tune_ms[1]]},
        "warm_start": {"train_solves": n_train, "held_out": n_test, "data_s": t_gen, "train_s": t_train,
                       "epochs": args.nn_epochs, "hidden": args.nn_hidden, "params": W.net.n_params,
                       "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
                       "loss_curve": [float(x) for x in losses[:: max(1, len(losses) // 20)]],
                       "lambda_rel_diff_vs_plain_cold_max": max(lam_err) if lam_err else None},
    }
    print(json.dumps(out), flush=True)


def _oracle_stream_task(i, rtol):
    """One whole stream problem on one core with the oracle (runs in a pool
    worker): assembly and topology untimed, then the timed reference IETI-DP
    (SuperLU local factorisations, coarse problem, right-hand side, PCG to
    rtol, recovery), then the untimed monolithic direct solve that serves
    as the reference for the B errors."""
    from threadpoolctl import threadpool_limits

    from oracle.post import b_error
    from oracle.run import OracleRun
    from workloads import configs

    with threadpool_limits(limits=1):
        O = OracleRun(configs.stream_problem(i))
        t0 = time.perf_counter()
        D = O.ieti
        lam, info = D.pcg(rtol=rtol, maxit=5000)
        a = D.recover(lam)
        t = time.perf_counter() - t0
        a_ref = O.monolithic()
        e_self = b_error(O.space, a, a_ref=a_ref)[1]
    return i, t, int(info["iters"]), a_ref, float(e_self)


def stream_oracle_baseline(n, rtol, budget_s, max_edges):
    """cpu_baseline of the stream: the oracle on whole problems, one problem
    per task in a pool of min(os.cpu_count(), 16) single-threaded workers.
    The sample is the stream's problems in index order whose coefficient
    vector has at most ``max_edges`` entries, submitted until ``budget_s``
    of wall time have passed (the larger problems are left out, so the
    rate is an upper bound for the oracle on the whole stream).  Runs
    before the GPU is touched (the pool forks)."""
    import multiprocessing as mp

    from oracle.space import Space
    from workloads import configs

    sample = [i for i in range(n) if Space(configs.stream_problem(i)).n_edges <= max_edges]
    workers = max(1, min(os.cpu_count() or 1, 16))
    ctx = mp.get_context("fork")
    res, pending = {}, []
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        nxt = 0
        while nxt < len(sample) or pending:
            while nxt < len(sample) and len(pending) < workers and time.perf_counter() - t0 < budget_s:
                pending.append(pool.apply_async(_oracle_stream_task, (sample[nxt], rtol)))
                nxt += 1
            if nxt < len(sample) and time.perf_counter() - t0 >= budget_s:
                nxt = len(sample)
            done = [r for r in pending if r.ready()]
            for r in done:
                i, t, it, a_ref, e_self = r.get()
                res[i] = {"t": t, "iters": it, "a_ref": a_ref, "e_self": e_self}
                pending.remove(r)
            if not done:
                time.sleep(0.05)
    wall = time.perf_counter() - t0
    ids = sorted(res)
    if not ids:
        return None, {}
    t_sum = float(sum(res[i]["t"] for i in ids))
    # one core alone (no other worker running): the first sampled problem again
    _, t1, _, _, _ = _oracle_stream_task(ids[0], rtol)
    base = {
        "value": workers * len(ids) / t_sum, "unit": "solves/s", "cores": workers, "kind": "oracle",
        "sample": (f"{len(ids)} whole stream problems {ids[0]}..{ids[-1]} (those with <= {max_edges} coefficients, "
                   f"index order, {wall:.1f}s wall over {workers} single-threaded workers): oracle IETI-DP setup + "
                   f"PCG to rtol {rtol:g} + recovery, {t_sum:.1f}s of CPU in total; value = workers x problems / "
                   f"summed solve time (host assembly excluded, as on the GPU)"),
        "solve_s_mean": t_sum / len(ids),
        "value_1core": 1.0 / t1,
        "sample_1core": f"problem {ids[0]} alone on one core: {t1:.2f}s",
    }
    return base, res


def stream_batches(args):
    """stream256: 256 independent box problems (configuration 5), solved in
    batches (one handle and one set of launches per chunk of problems),
    mixed precision and plain FP64, and each problem alone (plain FP64).
    A step is one pass over the whole stream; each chunk's timed region
    starts with its inputs resident in HBM and ends with the chunk's
    solutions in HBM.  Host assembly and upload are untimed."""
    import concurrent.futures

    n, chunk = args.stream_count, args.stream_chunk
    base, oracle_res = (None, {})
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        base, oracle_res = stream_oracle_baseline(n, args.rtol, args.cpu_budget, args.cpu_max_edges)
        log(f"cpu baseline {time.perf_counter() - t0:.1f}s over {len(oracle_res)} problems")

    import torch

    from oracle.post import b_error
    from oracle.space import Space
    from paper_2501_04340_amd import Solver
    from paper_2501_04340_amd.ietidp import GEMV_SYM, PREC_FP64, PREC_MIXED
    from workloads import configs

    torch.cuda.set_device(0)
    fkw = {} if args.gemv_variant is None else {"gemv_variant": args.gemv_variant}
    K, W = args.steps, args.warmup
    variants = {"batch_mixed": PREC_MIXED, "batch_plain_fp64": PREC_FP64}
    passes = {"batch_mixed": K, "batch_plain_fp64": min(K, 5)}
    t_var = {k: 0.0 for k in variants}
    lat = {k: [] for k in variants}
    pcg_s = {k: 0.0 for k in variants}
    pcg_bytes = {k: 0.0 for k in variants}
    fac_s = {k: 0.0 for k in variants}
    plan_sum = {"flops": 0.0, "flops_scalar_rr": 0.0, "flops_scalar_aug": 0.0}
    applies = {k: 0 for k in variants}
    lat_single, t_single = [], 0.0
    iters = {k: [] for k in variants}
    outer = []
    resid = {k: [] for k in variants}
    a_sample = {}
    roof = None
    kprof = None
    n_g_total, t_host = 0, 0.0
    ftune = None
    pinned = tuple(int(x) for x in args.factor_params.split(",")) if args.factor_params else None
    for c0 in range(0, n, chunk):
        ids = list(range(c0, min(n, c0 + chunk)))
        th = time.perf_counter()
        probs = [configs.stream_problem(i) for i in ids]
        with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
            singles = list(ex.map(Solver, probs))
        t_host += time.perf_counter() - th
        log(f"problems {ids[0]}..{ids[-1]}: assembled")
        n_g_total += sum(S.n_global for S in singles)
        # each problem alone (plain FP64): one untimed factor + solve, then a timed one
        buf = torch.empty(max(S.n_edges for S in singles), dtype=torch.float64, device="cuda")
        for S in ([] if args.no_single else singles):
            S.factor(**fkw)
            S.solve_device(buf.data_ptr(), rtol=args.rtol)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.factor(**fkw)
            S.solve_device(buf.data_ptr(), rtol=args.rtol)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            lat_single.append(dt * 1e3)
            t_single += dt
        del buf
        if pinned is None and ftune is None and not args.no_factor_tune:
            # the factorisation autotuner runs once, on a batch of (at most) the
            # first 32 problems; every batch then uses its choice
            nt = min(32, len(singles))
            Bt = Solver.batch_of(singles[:nt])
            Bt.factor(precision=PREC_MIXED, tune=True, **fkw)
            prm, flog = Bt.factor_tuning()
            Bt.close()
            ftune = {"params": list(prm), "tuned_on_problems": [ids[0], ids[nt - 1]],
                     "log_defer_tail_wgs_ms": [[float(x) for x in r] for r in flog]}
            log(f"factorisation autotuner: defer {prm[0]}, tail {prm[1]}, update workgroups {prm[2]}")
        B = Solver.batch_of(singles)
        for S in singles:
            S.close()
        log(f"problems {ids[0]}..{ids[-1]}: batch handle built")
        if pinned is not None:
            B.set_factor_params(*pinned)
            ftune = {"params": list(pinned), "pinned": True}
        elif ftune is not None:
            B.set_factor_params(*ftune["params"])
        info = B.batch_info()
        pinfo = B.plan_info()
        for key in plan_sum:
            plan_sum[key] += pinfo[key]
        a_dev = torch.empty(B.n_edges, dtype=torch.float64, device="cuda")
        for name, prec in variants.items():
            # the headline variant runs W warm-up and K timed passes, the
            # comparison one warm-up and min(K, 5) timed passes
            head = name == "batch_mixed"
            for _ in range(W if head else 1):
                B.factor(precision=prec, **fkw)
                B.solve_device(a_dev.data_ptr(), rtol=args.rtol, maxit=3000)
            for _ in range(K if head else min(K, 5)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                B.factor(precision=prec, **fkw)
                st = B.solve_device(a_dev.data_ptr(), rtol=args.rtol, maxit=3000)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                t_var[name] += dt
                lat[name].extend([dt * 1e3] * len(ids))
                pcg_s[name] += st["t_pcg_s"]
                pcg_bytes[name] += st["pcg_bytes"]
                fac_s[name] += st["t_factor_s"]
                applies[name] += st["f_applies"]
            log(f"problems {ids[0]}..{ids[-1]}: {name} timed")
            ps = [B.problem_stats(p) for p in range(len(ids))]
            iters[name].extend(x["iters"] for x in ps)
            resid[name].extend(x["rel_residual"] for x in ps)
            if name == "batch_mixed":
                outer.extend(x["outer_iters"] for x in ps)
                a_host = a_dev.cpu().numpy()
                for p, i in enumerate(ids):
                    if i in oracle_res:
                        b0 = info[p]["edge_base"]
                        a_sample[i] = a_host[b0:b0 + info[p]["n_edges"]].copy()
        if kprof is None:
            # kernel durations: one more headline pass with launch events on every
            # GEMV and tile-update launch (direct launches, no graph replay)
            B.factor(precision=PREC_MIXED, **fkw)
            B.set_profiling(True)
            B.factor(precision=PREC_MIXED, **fkw)
            B.solve_device(a_dev.data_ptr(), rtol=args.rtol, maxit=3000)
            kt = B.kernel_times()
            B.set_profiling(False)
            ps = [B.problem_stats(p) for p in range(len(ids))]
            chosen = B.gemv_tuning()[0]
            kprof = {"kt": kt, "ps": ps, "chosen": chosen, "ids": (ids[0], ids[-1]), "plan": B.plan_info(),
                     "params": B.factor_tuning()[0]}
        B.close()
        del a_dev
        log(f"problems {ids[0]}..{ids[-1]}: alone {np.sum(lat_single[-len(ids):]) if lat_single else 0:.0f} ms, batch mixed "
            f"{lat['batch_mixed'][-1]:.0f} ms, batch plain {lat['batch_plain_fp64'][-1]:.0f} ms "
            f"(host assembly {t_host:.0f}s so far)")

    # roofline of the dominant kernel of the headline pass (largest total time)
    kt, ps = kprof["kt"], kprof["ps"]
    # the PMC summary's figures are per launch of one batch: keyed by its problems
    batch_key = f"stream256[{kprof['ids'][0]}..{kprof['ids'][1]}]"
    def gemv_roof(fp32):
        s_b = 4.0 if fp32 else 8.0
        nb = sum((x["f_applies"][fp32] + x["m_applies"][fp32]) * x["block_entries"] * s_b for x in ps)
        ms = kt["gemv32_ms" if fp32 else "gemv_ms"]
        nl = kt["gemv32_launches" if fp32 else "gemv_launches"]
        sym = int(kprof["chosen"][fp32]) == GEMV_SYM
        name = ("k_gemv_sym" if sym else "k_gemv") + ("<float>" if fp32 else "<double>")
        ach = nb / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        return {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic(name, batch_key),
                "avg_launch_ms": ms / max(nl, 1), "launches": nl, "total_ms": ms,
                "alg_bytes_per_launch": nb / max(nl, 1)}
    upd_avg = kt["update_ms"] / max(kt["update_launches"], 1)
    upd_flops = kt["update_tasks"] / max(kt["update_launches"], 1) * 2.0 * 64 ** 3
    upd_ach = upd_flops / (upd_avg * 1e-3) / 1e12 if upd_avg > 0 else 0.0
    roof_upd = {"kernel": "k_update_multi", "bound": "mfma", "achieved": upd_ach, "peak": FP64_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": upd_ach / FP64_MFMA_PEAK_TFLOPS,
                "traffic": measured_traffic("k_update_multi", batch_key, kprof["params"]), "avg_launch_ms": upd_avg,
                "launches": kt["update_launches"], "total_ms": kt["update_ms"],
                "flops_per_launch": upd_flops, "flops_counted": "64x64x64 tile products (2 T^3 each)"}
    cands = [gemv_roof(1), gemv_roof(0), roof_upd]
    cands.sort(key=lambda r: -r["total_ms"])
    roof = dict(cands[0])
    roof["kernel"] += f", one batch of problems {kprof['ids'][0]}..{kprof['ids'][1]}"
    roof["others"] = cands[1:]

    def summ(name):
        return {"solves_per_s": n * passes[name] / t_var[name], "ms_per_pass": t_var[name] * 1e3 / passes[name],
                "timed_passes": passes[name],
                "latency_ms_p50": float(np.percentile(lat[name], 50)),
                "latency_ms_p99": float(np.percentile(lat[name], 99)),
                "pcg_iters_mean": float(np.mean(iters[name])), "max_rel_residual_fp64": float(np.max(resid[name])),
                "f_applies_per_s": applies[name] / pcg_s[name] if pcg_s[name] else None,
                "solve_phase": {"alg_bytes": pcg_bytes[name], "pcg_s": pcg_s[name],
                                "achieved_GBs": pcg_bytes[name] / pcg_s[name] / 1e9 if pcg_s[name] else None,
                                "frac_of_hbm_peak": (pcg_bytes[name] / pcg_s[name] / 1e9 / HBM_PEAK_GBS
                                                     if pcg_s[name] else None)}}
    vs = {k: summ(k) for k in variants}
    if lat_single:
        vs["single_plain_fp64"] = {"solves_per_s": n / t_single,
                                   "latency_ms_p50": float(np.percentile(lat_single, 50)),
                                   "latency_ms_p99": float(np.percentile(lat_single, 99)), "passes": 1}
    # B error of the headline's solutions against the oracle's direct solves
    errs = {}
    for i, a in a_sample.items():
        errs[i] = float(b_error(Space(configs.stream_problem(i)), a, a_ref=oracle_res[i]["a_ref"])[1])
    b_err = None
    if errs:
        ev = np.array(list(errs.values()))
        b_err = {"max": float(ev.max()), "median": float(np.median(ev)), "problems": len(ev),
                 "oracle_ieti_vs_direct_max": float(max(oracle_res[i]["e_self"] for i in errs)),
                 "what": "relative B-field L2 error of the batched mixed solutions (rtol "
                         f"{args.rtol:g}) against the oracle's direct solve of the same problem"}
    ms_step = t_var["batch_mixed"] * 1e3 / K
    out = {
        "metric": "IETI-DP time-to-solution and F·λ applies/s at rtol 1e-8, mixed+warm vs plain FP64",
        "value": n * K / t_var["batch_mixed"], "unit": "solves/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"stream256 (configuration 5): {n} independent box problems (2^a x 2^b x 2^c "
                               f"patches, a,b,c in {{1,2,3}}, p in {{2,3}}, 4-6 elements, nu log-uniform in "
                               f"[1e-3,1], trigonometric J), batches of {chunk}, rtol {args.rtol:g}",
                   "variant": ("batched mixed precision: FP64 factorisation, coarse problem, recurrences and "
                               "outer refinement; FP32-stored interface blocks in the inner PCG; lambda_0 = 0 "
                               "(no warm-start network for this stream: every problem has its own random source)"),
                   "step": "one pass over all problems (each chunk timed with its inputs resident in HBM)",
                   "n_g_total": n_g_total},
        "variants": vs,
        "speedup_batch_mixed_vs_batch_plain": vs["batch_mixed"]["solves_per_s"] / vs["batch_plain_fp64"]["solves_per_s"],
        "speedup_batch_mixed_vs_single_plain": (t_single * K) / t_var["batch_mixed"] if lat_single else None,
        "mixed_outer_iters_mean": float(np.mean(outer)) if outer else None,
        "factorisation": factor_summary(plan_sum, fac_s["batch_mixed"] / K),
        "factor_autotune": ftune,
        "b_error_vs_oracle": b_err,
        "host_assembly_s": t_host,
        "roofline": roof,
    }
    if base is not None:
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 3 on stream256, else 20)")
    ap.add_argument("--warmup", type=int, default=None, help="warm-up steps (default 1 on stream256, else 2)")
    ap.add_argument("--workload", default="stream256", choices=sorted(WORKLOADS))
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0,
                    help="seconds of oracle work in the cpu_baseline leg (wall time of the worker pool on stream256)")
    ap.add_argument("--cpu-max-edges", type=int, default=25000,
                    help="stream256 cpu_baseline: largest problem (coefficients) the oracle sample takes")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 3 device-to-device copies of MIB MiB (HBM counter calibration) and exit")
    ap.add_argument("--stream-count", type=int, default=256)
    ap.add_argument("--stream-chunk", type=int, default=64,
                    help="stream256: problems per batch handle (64: the host-side plan of a batch takes about "
                         "1 GB per problem, so the whole stream of 256 in one handle does not fit host memory)")
    ap.add_argument("--ring-train", type=int, default=512)
    ap.add_argument("--ring-test", type=int, default=64)
    ap.add_argument("--nn-epochs", type=int, default=300)
    ap.add_argument("--nn-hidden", type=int, default=256)
    ap.add_argument("--nn-lr", type=float, default=1e-3)
    ap.add_argument("--no-factor-tune", action="store_true",
                    help="keep the default factorisation parameters (no autotuning of the update schedule)")
    ap.add_argument("--factor-params", default=None, metavar="D,DT,W",
                    help="pin the factorisation parameters (deferral thresholds, update workgroups) instead of "
                         "autotuning them, e.g. for profiled runs")
    ap.add_argument("--no-single", action="store_true",
                    help="stream256: skip the each-problem-alone comparison (profiled runs of the batches)")
    ap.add_argument("--gemv-variant", type=int, default=None, metavar="V",
                    help="force the interface GEMV launch shape (0-11 row streaming, 12 symmetric) instead of "
                         "the autotuner's choice; for profiled runs, where tracing adds a cost to every launch "
                         "and so favours shapes with fewer launches")
    args = ap.parse_args()
    stream = args.workload == "stream256"
    if args.steps is None:
        args.steps = 3 if stream else 20
    if args.warmup is None:
        args.warmup = 1 if stream else 2
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested); the multi-GPU sharding "
              "of the subdomains is a design, not a measured path.", flush=True)
        sys.exit(2)

    if stream and not args.copy_calibration:
        # the oracle's worker pool forks before anything touches the GPU
        return stream_batches(args)

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
    torch.cuda.set_device(0)
    prob = configs.make_config(args.workload)
    t0 = time.perf_counter()
    S = Solver(prob)
    fkw = {} if args.gemv_variant is None else {"gemv_variant": args.gemv_variant}
    log(f"host assembly {time.perf_counter() - t0:.1f}s sizes {S.sizes()}")
    info = S.plan_info()
    # the solution stays in HBM (a device buffer), as the inputs do
    a_dev = torch.empty(S.n_edges, dtype=torch.float64, device="cuda")
    if args.factor_params:
        S.set_factor_params(*(int(x) for x in args.factor_params.split(",")))
    elif not args.no_factor_tune:
        S.factor(tune=True, **fkw)  # the factorisation autotuner; its choice is kept by the handle
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
    # algorithmic bytes: every symmetric interface block's lower triangle once,
    # sum_k n_I (n_I + 1) / 2 entries; the kernel reads whole lower 64x64 tiles
    # inside n_I (read_bytes_per_launch)
    gemv_ach = kt["gemv_bytes_alg"] / (gemv_ms * 1e-3) / 1e9
    roof_gemv = {"kernel": gemv_name, "bound": "hbm", "achieved": gemv_ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": gemv_ach / HBM_PEAK_GBS, "traffic": measured_traffic(gemv_name, args.workload),
                 "avg_launch_ms": gemv_ms, "bytes_per_launch": kt["gemv_bytes_alg"],
                 "read_bytes_per_launch": kt["gemv_bytes"],
                 "launches_per_step": kt["gemv_launches"], "ms_per_step": kt["gemv_ms"]}
    flops_per_task = 2.0 * 64 ** 3
    upd_avg = kt["update_ms"] / max(kt["update_launches"], 1)
    upd_flops = kt["update_tasks"] / max(kt["update_launches"], 1) * flops_per_task
    upd_ach = upd_flops / (upd_avg * 1e-3) / 1e12
    roof_upd = {"kernel": "k_update_multi", "bound": "mfma", "achieved": upd_ach, "peak": FP64_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": upd_ach / FP64_MFMA_PEAK_TFLOPS, "traffic": measured_traffic("k_update_multi", args.workload, S.factor_tuning()[0]),
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
        "factor_tflops": S.plan_info()["flops"] / (factor_ms * 1e-3) / 1e12,
        "factorisation": factor_summary(S.plan_info(), factor_ms * 1e-3),
        "factor_autotune": {"params": list(S.factor_tuning()[0]),
                            "log_defer_tail_wgs_ms": S.factor_tuning()[1].tolist()},
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
