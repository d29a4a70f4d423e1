"""Throughput of the PEPS-VMC hot path on one MI355X.

One step = one pass of the whole path over one batch of spin configurations:
top-down and bottom-up boundary-MPS sweeps (apply + QR/SVD truncation), the
single- and two-row sandwiches, every J1/J2 spin-flip ratio, the local energy,
and the energy gradient dE/dA of the Monte Carlo estimator (log-derivatives of
every site contracted with 2(E - <E>)/B).

Headline workload: 16x16 open J1-J2 lattice (J2/J1 = 0.5), D = 6, Dc = 36, 1024
samples (one per Markov chain, seeded S^z = 0 configurations), site tensors N(0,1)
normalised per site; every contraction and factorisation in float64 (the paper's
arithmetic).  Inputs are resident in HBM before the timed region.  Beside it the
line reports the same workload with float32 and bfloat16 contractions (with their
errors against the float64 results), the plain path (batch 1, float64), the 8x8
workload, a 24x24 subset, and the oracle on the host cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload NAME] [--prec f64]
                    [--no-legs] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2516.6}   # dense MFMA TFLOP/s
T_START = time.time()
# wall-clock budget of one run: a leg (below) starts only if its estimated cost still
# fits, so a default run stays within a few minutes whatever the step time
BUDGET_S = float(os.environ.get("BENCH_BUDGET_S", "480"))


def _log(msg: str) -> None:
    print(f"[bench {time.time() - T_START:7.1f} s] {msg}", file=sys.stderr, flush=True)


def _fits(seconds: float) -> bool:
    return time.time() - T_START + seconds < BUDGET_S


def _oracle_worker(args):
    from threadpoolctl import threadpool_limits

    import oracle as O
    from paper_1806_03761_amd.workloads import make_workload
    name, lo, hi, sweeps = args
    with threadpool_limits(limits=1):
        lat, A, S, _ = make_workload(name, hi)
        for b in range(lo, hi):
            O.full_path_one(A, lat, S[b], sweeps)
    return hi - lo


def start_cpu_baseline(name: str, per_proc: int, sweeps: int = 0):
    """Start the FP64 oracle (amplitude + local energy + log-derivatives, one sample at a
    time per process, numpy single-threaded) on up to 16 host cores over the first samples
    of the workload; returns a handle for finish_cpu_baseline."""
    import multiprocessing as mp
    procs = max(1, min(16, os.cpu_count() or 1))
    tasks = [(name, k * per_proc, (k + 1) * per_proc, sweeps) for k in range(procs)]
    pool = mp.get_context("spawn").Pool(procs)
    pool.map(_oracle_worker, [(name, 0, 0, sweeps)] * procs)   # imports warmed up
    t0 = time.perf_counter()
    res = pool.map_async(_oracle_worker, tasks)
    return pool, res, t0, procs, per_proc


def finish_cpu_baseline(h, name):
    pool, res, t0, procs, per_proc = h
    done = sum(res.get())
    dt = time.perf_counter() - t0
    pool.close()
    pool.join()
    return {"value": done / dt, "unit": "samples/s", "cores": procs, "kind": "oracle",
            "sample": f"the first {done} configurations of the {name} workload, {per_proc} per "
                      f"process, {procs} processes, numpy single-threaded, run during the warm-up "
                      f"steps; wall {dt:.1f} s"}


# HBM traffic per launch of the contraction GEMMs, from two rocprofv3 --pmc passes
# (FETCH_SIZE, WRITE_SIZE, KiB per dispatch) over one evaluation, each scaled by what the
# same counter reads for a 256 MiB device copy (FETCH_SIZE reads half of the copied bytes:
# factor 2.0; WRITE_SIZE all: 1.0).  Valid only for the kernel sources they were measured
# on (hash below) and the workload, arithmetic and batch named; otherwise null.
TRAFFIC = {"sources": "d2c823b1675075b6",
           "bytes_per_launch": {("8x8_D4_Dc16", "f64", 4096, "gemm"): 166.4e6}}


def _sources_hash() -> str:
    import hashlib
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_1806_03761_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".cpp", ".h")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


CLASSES = ("gemm", "fused", "qr", "svd")
CLASS_NAMES = {"svd": "truncation step (Q application, Gram matrix, tridiagonalisation, bisection, "
                      "eigenvectors, subspace refinement)",
               "qr": "blocked Householder QR (register panels + 32-reflector WY GEMMs)",
               "gemm": "k_mgemm contraction GEMMs (apply, sandwiches, environments)",
               "fused": "fused sandwich steps (k_pair_mfma / k_row_step)"}


def _read(peps, classes):
    out = {}
    for cls in classes:
        kms, n, fl = peps.profile_read(cls)
        by = peps.profile_bytes(cls)
        out[cls] = {"ms_total": kms, "launches": n, "avg_us": 1e3 * kms / max(n, 1),
                    "tflops": fl / max(kms, 1e-12) / 1e9, "flops": fl, "bytes": by,
                    "gbps": by / max(kms, 1e-12) / 1e6}
    return out


HBM_PEAK_GBPS = 8000.0


def _roofline(timed, peak_tflops):
    """The binding roof of a kernel class from its algorithmic flops and bytes: HBM when the
    arithmetic intensity is below the ridge point peak_flops / peak_bandwidth, else the
    matrix cores; both views are kept."""
    ridge = peak_tflops * 1e12 / (HBM_PEAK_GBPS * 1e9)
    ai = timed["flops"] / timed["bytes"] if timed["bytes"] > 0 else float("inf")
    mfma = {"achieved": timed["tflops"], "peak": peak_tflops, "unit": "TFLOP/s",
            "frac": timed["tflops"] / peak_tflops}
    hbm = {"achieved": timed["gbps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
           "frac": timed["gbps"] / HBM_PEAK_GBPS} if timed["bytes"] > 0 else None
    if hbm is not None and ai < ridge:
        return dict(bound="hbm", **hbm, arithmetic_intensity=ai, ridge=ridge, mfma_view=mfma,
                    algorithmic_bytes_per_launch=timed["bytes"] / max(timed["launches"], 1))
    return dict(bound="mfma", **mfma, arithmetic_intensity=ai, ridge=ridge, hbm_view=hbm)


def _rel_errors(x, ref, floor=1.0):
    import numpy as np
    x, ref = np.asarray(x, np.float64), np.asarray(ref, np.float64)
    e = np.abs(x - ref) / np.maximum(floor, np.abs(ref))
    return {"median": float(np.median(e)), "p99": float(np.quantile(e, 0.99)), "max": float(e.max())}


def run_mixed(args, peps, torch):
    """The uneven persistent batch: every lattice's tiles autotuned at its own batch, then
    the whole launch sequence of the three jobs captured once and replayed per step."""
    from paper_1806_03761_amd.workloads import MIXED_BATCH, make_workload
    dev = torch.device("cuda:0")
    peps.set_workspace_limit(200 << 30)
    peps.set_truncation(args.truncation_sweeps)
    jobs, total = [], 0
    tuned = {}
    for name, B in MIXED_BATCH:
        lat, A, S, _ = make_workload(name, B)
        Ad, Sd = torch.from_numpy(A).to(dev), torch.from_numpy(S).to(dev)
        # the D = 8 lattice keeps the heuristic tiles: its tuning pass (every candidate tile
        # on every GEMM shape of a 410-sample evaluation) takes minutes by itself
        if args.no_tune or lat.D >= 8:
            n = "heuristic tiles"
        else:
            n = peps.autotune(Ad, Sd, lat, "f32")
        tuned[name] = n
        _log(f"{name}: batch {B}, GEMM tiles tuned: {n}")
        jobs.append({"A": Ad, "S": Sd, "lat": lat, "grad_mode": 3})
        total += B
    outs = None
    for k in range(max(args.warmup, 1)):
        outs = peps.eval_jobs(jobs, "f32", graph=True, outputs=outs)
        torch.cuda.synchronize()
        _log(f"warm-up step {k + 1}")
    t0 = time.perf_counter()
    for k in range(args.steps):
        outs = peps.eval_jobs(jobs, "f32", graph=True, outputs=outs)
        torch.cuda.synchronize()
        _log(f"timed step {k + 1}")
    dt = time.perf_counter() - t0
    flags = sum(int((o[4] != 0).sum().item()) for o in outs)
    res = {"metric": "samples/sec (amplitude+E_loc+grad) & contraction MFMA util, batched vs plain",
           "value": total * args.steps / dt, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
           "warmup": max(args.warmup, 1), "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "uneven batch in one captured graph: " +
                                  ", ".join(f"{n} x {B}" for n, B in MIXED_BATCH) +
                                  "; float32 contraction GEMMs, float64 QR/SVD; amplitude + local energy + dE/dA",
                      "batch": total, "autotuned_gemm_shapes": tuned,
                      "truncation": ("canonical SVD" if args.truncation_sweeps == 0 else
                                     f"variational, {args.truncation_sweeps} sweeps (float64)")},
           "flagged_samples": flags, "run_wall_s": time.time() - T_START}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="16x16_D6_Dc36")
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16"])
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--no-legs", action="store_true", help="headline only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the GEMM tile autotuner")
    ap.add_argument("--truncation-sweeps", type=int, default=0,
                    help="boundary truncation of the timed workload: 0 = canonical SVD (the default "
                         "path), n > 0 = variational compression with n sweeps")
    ap.add_argument("--mixed", action="store_true",
                    help="only the uneven batch: 2048 samples over 8x8 (D 4, Dc 16), 12x12 (D 6, Dc 36) "
                         "and 16x16 (D 8, Dc 64) at 50/30/20, float32 contractions, one captured graph")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 256 MiB device-to-device copy (3 times): the reference "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on one GPU only (the path is data-parallel over samples; "
              "multi-GPU sharding is described in the design notes, not run)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        # the reference kernel of the traffic counters, and the bandwidth a plain device
        # copy reaches (read + write bytes over event time, 20 copies after 3 untimed)
        n = 256 * 2 ** 20 // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 20
        print(json.dumps({"copy_calibration_bytes_per_launch": 8 * n,
                          "copy_read_plus_write_GBps": 2 * 8 * n / (ms * 1e-3) / 1e9}), flush=True)
        return

    from paper_1806_03761_amd import peps

    if args.mixed:
        return run_mixed(args, peps, torch)
    from paper_1806_03761_amd.workloads import WORKLOADS, make_workload

    name = args.workload
    lat, A, S, _ = make_workload(name, args.batch)
    B = S.shape[0]
    dev = torch.device("cuda:0")
    peps.set_workspace_limit(200 << 30)
    Ad = torch.from_numpy(A).to(dev)
    Sd = torch.from_numpy(S).to(dev)
    N, D4 = lat.N, lat.D ** 4
    grad = torch.empty((N, 2, D4), dtype=torch.float64, device=dev)
    peps.set_truncation(args.truncation_sweeps)

    def step(prec=args.prec, Ax=Ad, Sx=Sd, latx=lat, out=grad):
        return peps.evaluate(Ax, Sx, latx, prec, grad_mode=3, out=out)

    tuned = 0
    if not args.no_tune:
        tuned = peps.autotune(Ad, Sd, lat, args.prec)     # untimed: picks GEMM tiles by measurement
    _log(f"{name}: batch {B}, {tuned} GEMM shapes tuned")
    cpu_h = None
    if not args.no_cpu_baseline:
        cpu_h = start_cpu_baseline(name, 1, args.truncation_sweeps)
    # warm-up steps with every kernel class bracketed by HIP events: the per-class
    # breakdown, and which class dominates
    peps.profile_enable(CLASSES)
    for k in range(max(args.warmup, 1)):
        step()
        torch.cuda.synchronize()
        _log(f"warm-up step {k + 1}")
    kern = _read(peps, CLASSES)
    # the roofline kernel: the contraction kernel family with the most time (the MFMA GEMMs,
    # or the fused sandwich steps where those replace them); the factorisation classes are
    # reported beside it
    dom = "gemm" if kern["gemm"]["ms_total"] >= kern["fused"]["ms_total"] else "fused"
    cpu = finish_cpu_baseline(cpu_h, name) if cpu_h else None
    _log("cpu baseline done" if cpu else "no cpu baseline")
    # progress lines in the timed region only for slow steps (the host runs ahead of the
    # GPU, so a line marks an enqueue, not a completion; it adds no synchronisation)
    dt_step_log = 1 if kern and sum(v["ms_total"] for v in kern.values()) > 2000 * max(args.warmup, 1) else 0
    # timed region: only the dominant class is bracketed by events (on the library's
    # stream), which keeps the instrumentation out of the throughput
    peps.profile_enable((dom,))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        res_f64 = step()
        if dt_step_log and (k + 1) % dt_step_log == 0:
            _log(f"timed step {k + 1} enqueued")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _log(f"timed region {dt:.1f} s")
    timed = _read(peps, (dom,))[dom]
    peps.profile_enable(())
    ms = dt * 1e3 / args.steps
    value = B * args.steps / dt

    res = {
        "metric": "samples/sec (amplitude+E_loc+grad) & contraction MFMA util, batched vs plain",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"{lat.Lx}x{lat.Ly} open J1-J2 (J2/J1={lat.J2}), D={lat.D}, Dc={lat.Dc}, "
                               f"{B} samples, {args.prec} contractions and f64 QR/SVD; amplitude + "
                               f"local energy + dE/dA",
                   "lattice": [lat.Lx, lat.Ly], "D": lat.D, "Dc": lat.Dc, "batch": B,
                   "gemm_precision": args.prec, "factorisation_precision": "f64",
                   "truncation": ("canonical SVD" if args.truncation_sweeps == 0 else
                                  f"variational, {args.truncation_sweeps} sweeps"),
                   "autotuned_gemm_shapes": tuned},
    }
    peak = MI355X_PEAK["f64" if args.prec == "f64" else "f32"]
    traffic = None
    if TRAFFIC["sources"] == _sources_hash():
        traffic = TRAFFIC["bytes_per_launch"].get((name, args.prec, B, dom))
    res["roofline"] = dict({"kernel": CLASS_NAMES[dom], "class": dom}, **_roofline(timed, peak),
                           traffic=traffic, avg_launch_us=timed["avg_us"], launches=timed["launches"],
                           share_of_kernel_time=kern[dom]["ms_total"] / max(sum(v["ms_total"] for v in kern.values()), 1e-9))
    # every class against the dtype's matrix-core peak (the factorisations against fp64)
    res["kernels_warmup"] = {k: dict(v, frac_of_peak=v["tflops"] / (MI355X_PEAK["f64"] if k in ("svd", "qr") else peak))
                             for k, v in kern.items()}
    if not args.no_legs and args.truncation_sweeps == 0:
        la0, sg0, e0, g0, fl0 = (t.detach().cpu().numpy() for t in res_f64)
        legs = {}
        step_s = ms / 1e3
        # variational boundary compression (one sweep) in place of the SVD truncation on
        # the same batch: throughput, the class breakdown (the flops move from the float64
        # factorisations onto the GEMMs) and how far its results are from the SVD ones
        # (two different approximations of W, so a difference, not an error)
        vname = f"{name}_variational_1sweep"
        if _fits(4.0 * step_s + 20.0):
            _log(f"leg {vname}")
            peps.set_truncation(1)
            try:
                gv = torch.empty_like(grad)
                if not args.no_tune:
                    peps.autotune(Ad, Sd, lat, args.prec)
                step(out=gv)
                torch.cuda.synchronize()
                peps.profile_enable(CLASSES)
                t1 = time.perf_counter()
                rv = step(out=gv)
                torch.cuda.synchronize()
                dv = time.perf_counter() - t1
                kv = _read(peps, CLASSES)
                peps.profile_enable(())
            finally:
                peps.set_truncation(0)
            lav, sgv, ev, ggv, flv = (t.detach().cpu().numpy() for t in rv)
            ok = (fl0 == 0) & (flv == 0)
            legs[vname] = {"samples_per_s": B / dv, "ms_per_step": dv * 1e3, "sweeps": 1,
                           "kernels": {k: {"ms_total": v["ms_total"], "tflops": v["tflops"]} for k, v in kv.items()},
                           "gemm_frac_of_f64_peak": kv["gemm"]["tflops"] / MI355X_PEAK["f64"],
                           "diff_log_amp_vs_svd": _rel_errors(lav[ok], la0[ok]),
                           "diff_e_loc_vs_svd": _rel_errors(ev[ok], e0[ok]),
                           "sign_differences_vs_svd": int((sgv[ok] != sg0[ok]).sum())}
        else:
            legs[vname] = {"skipped": "time budget of the run"}
        # 24x24, D = 8, Dc = 64 with variational compression: 128 of its 512 samples
        if _fits(60.0):
            _log("leg 24x24_D8_Dc64_variational_1sweep")
            lat6, A6, S6, _ = make_workload("24x24_D8_Dc64", 128)
            A6d, S6d = torch.from_numpy(A6).to(dev), torch.from_numpy(S6).to(dev)
            g6 = torch.empty((lat6.N, 2, lat6.D ** 4), dtype=torch.float64, device=dev)
            peps.set_truncation(1)
            try:
                step("f64", A6d, S6d, lat6, g6)
                torch.cuda.synchronize()
                peps.profile_enable(CLASSES)
                t1 = time.perf_counter()
                r6 = step("f64", A6d, S6d, lat6, g6)
                torch.cuda.synchronize()
                d6 = time.perf_counter() - t1
                k6 = _read(peps, CLASSES)
                peps.profile_enable(())
            finally:
                peps.set_truncation(0)
            legs["24x24_D8_Dc64_variational_1sweep"] = {
                "samples_per_s": S6.shape[0] / d6, "ms_per_step": d6 * 1e3, "batch": int(S6.shape[0]),
                "flagged": int((r6[4] != 0).sum().item()),
                "kernels": {k: {"ms_total": v["ms_total"], "tflops": v["tflops"]} for k, v in k6.items()},
                "sample": "the first 128 of the 512 configurations, f64, heuristic GEMM tiles; amplitude + "
                          "local energy + dE/dA"}
            del A6d, S6d, g6, r6
        else:
            legs["24x24_D8_Dc64_variational_1sweep"] = {"skipped": "time budget of the run"}
        # the Dc ∝ D regime (D = 16, Dc = 32) on 16x16, variational compression, 64 samples
        if _fits(60.0):
            _log("leg 16x16_D16_Dc32_variational_1sweep")
            lat5, A5, S5, _ = make_workload("16x16_D16_Dc32")
            A5d, S5d = torch.from_numpy(A5).to(dev), torch.from_numpy(S5).to(dev)
            g5 = torch.empty((lat5.N, 2, lat5.D ** 4), dtype=torch.float64, device=dev)
            peps.set_truncation(1)
            try:
                step("f64", A5d, S5d, lat5, g5)
                torch.cuda.synchronize()
                peps.profile_enable(CLASSES)
                t1 = time.perf_counter()
                r5 = step("f64", A5d, S5d, lat5, g5)
                torch.cuda.synchronize()
                d5 = time.perf_counter() - t1
                k5 = _read(peps, CLASSES)
                peps.profile_enable(())
            finally:
                peps.set_truncation(0)
            legs["16x16_D16_Dc32_variational_1sweep"] = {
                "samples_per_s": S5.shape[0] / d5, "ms_per_step": d5 * 1e3, "batch": int(S5.shape[0]),
                "flagged": int((r5[4] != 0).sum().item()),
                "kernels": {k: {"ms_total": v["ms_total"], "tflops": v["tflops"]} for k, v in k5.items()},
                "sample": "the 16x16_D16_Dc32 workload (64 configurations, Frobenius-normalised Gaussian tensors), f64, heuristic GEMM tiles"}
            del A5d, S5d, g5, r5
        else:
            legs["16x16_D16_Dc32_variational_1sweep"] = {"skipped": "time budget of the run"}
        # the same workload with narrower contraction arithmetic: throughput and the error
        # of every result against the float64 results above (which match the oracle to
        # 1e-10 on the tested subsets)
        for pr in ("f32", "bf16"):
            if pr == args.prec:
                continue
            if not _fits(2.2 * step_s):
                legs[pr] = {"skipped": "time budget of the run"}
                continue
            _log(f"leg {pr}")
            g1 = torch.empty_like(grad)
            step(pr, out=g1)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r1 = step(pr, out=g1)
            torch.cuda.synchronize()
            d1 = time.perf_counter() - t1
            la1, sg1, e1, gg1, fl1 = (t.detach().cpu().numpy() for t in r1)
            ok = (fl0 == 0) & (fl1 == 0)
            legs[pr] = {"samples_per_s": B / d1, "ms_per_step": d1 * 1e3,
                        "err_log_amp_vs_f64": _rel_errors(la1[ok], la0[ok]),
                        "sign_mismatches": int((sg1[ok] != sg0[ok]).sum()),
                        "err_e_loc_vs_f64": _rel_errors(e1[ok], e0[ok]),
                        "err_grad_rel_l2_vs_f64": float(np.linalg.norm(gg1 - g0) / np.linalg.norm(g0))}
        # plain path: the same library at batch 1, float64, one sample at a time
        nplain = 2
        if _fits(20.0):
            _log("leg plain")
            peps.evaluate(Ad, Sd[0:1], lat, "f64", grad_mode=1)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for b in range(nplain):
                peps.evaluate(Ad, Sd[b:b + 1], lat, "f64", grad_mode=1)
            torch.cuda.synchronize()
            legs["plain"] = {"value": nplain / (time.perf_counter() - t1), "unit": "samples/s",
                             "sample": f"{nplain} samples one at a time, f64, batch 1"}
        else:
            legs["plain"] = {"skipped": "time budget of the run"}
        # the 8x8, D = 4, Dc = 16 workload (4096 samples), float64 and float32
        lat2, A2, S2, _ = make_workload("8x8_D4_Dc16")
        A2d, S2d = torch.from_numpy(A2).to(dev), torch.from_numpy(S2).to(dev)
        g2 = torch.empty((lat2.N, 2, lat2.D ** 4), dtype=torch.float64, device=dev)
        r2 = {}
        for pr in ("f64", "f32"):
            if not _fits(15.0):
                legs["8x8_D4_Dc16_" + pr] = {"skipped": "time budget of the run"}
                continue
            _log(f"leg 8x8_D4_Dc16 {pr}")
            peps.autotune(A2d, S2d, lat2, pr)
            step(pr, A2d, S2d, lat2, g2)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(5):
                rr = step(pr, A2d, S2d, lat2, g2)
            torch.cuda.synchronize()
            legs["8x8_D4_Dc16_" + pr] = {"samples_per_s": 5 * S2.shape[0] / (time.perf_counter() - t1),
                                         "batch": int(S2.shape[0])}
            r2[pr] = [t.detach().cpu().numpy() for t in rr]
        for pr in ("f32",):
            if "f64" not in r2 or pr not in r2:
                continue
            # against float64 over the whole 4096-sample batch (float64 matches the oracle
            # to 1e-10 / 1e-9 on the tested subsets); E_loc relative to max(1, |E|)
            la0, sg0, e0, gg0, fl0 = r2["f64"]
            la1, sg1, e1, gg1, fl1 = r2[pr]
            ok = (fl0 == 0) & (fl1 == 0)
            le = _rel_errors(e1[ok], e0[ok])
            legs["8x8_D4_Dc16_" + pr].update({
                "err_log_amp_vs_f64": _rel_errors(la1[ok], la0[ok]),
                "sign_mismatches": int((sg1[ok] != sg0[ok]).sum()),
                "err_e_loc_vs_f64": le,
                "e_loc_above_1e-4": int((np.abs(e1[ok] - e0[ok]) / np.maximum(1.0, np.abs(e0[ok])) > 1e-4).sum()),
                "err_grad_rel_l2_vs_f64": float(np.linalg.norm(gg1 - gg0) / np.linalg.norm(gg0))})
        del A2d, S2d, g2
        # 24x24, D = 8, Dc = 64: one step over the first 2 of its 512 samples
        if _fits(150.0):
            _log("leg 24x24_D8_Dc64 f64")
            lat4, A4, S4, _ = make_workload("24x24_D8_Dc64", 2)
            A4d, S4d = torch.from_numpy(A4).to(dev), torch.from_numpy(S4).to(dev)
            g4 = torch.empty((lat4.N, 2, lat4.D ** 4), dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            step("f64", A4d, S4d, lat4, g4)
            torch.cuda.synchronize()
            legs["24x24_D8_Dc64_f64"] = {"samples_per_s": S4.shape[0] / (time.perf_counter() - t1),
                                         "sample": "first 2 of the 512 configurations, one step, f64 (includes "
                                                   "first-use workspace set-up)"}
            del A4d, S4d, g4
        else:
            legs["24x24_D8_Dc64_f64"] = {"skipped": "time budget of the run"}
        res["legs"] = legs
    if cpu:
        res["cpu_baseline"] = cpu
    res["run_wall_s"] = time.time() - T_START
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
