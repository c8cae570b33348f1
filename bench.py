"""Benchmark: D-BiCGStab time to a 1e-8 residual per source, and Dslash HBM bandwidth, on one MI355X.

Workload (one step): 16^4 Wilson lattice, links exp(0.6 i Q) (seed 102), kappa = 0.995 kappa_c,
D-BiCGStab(20) on 12 Z2-noise sources batched in one call, FP32 inner iterations with 12-real
links and FP64 reliable updates, deflated with the 20 GMRES-DR(60,20) eigenvectors of a point
source.  kappa_c and the GMRES-DR eigenvectors are computed once on the GPU before timing.
Also reported (outside the timed steps): plain FP64 single-right-hand-side D-BiCGStab time per
source, undeflated FP64 BiCGStab, the GMRES-DR time, a Dslash bandwidth sweep on 24^3 x 48, and
the CPU oracle on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--quick]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dslash HBM GB/s; D-BiCGStab time-to-1e-8/source (mixed+batched vs FP64 plain)"
HBM_PEAK_GBS = 8000.0
# FETCH_SIZE / WRITE_SIZE summary of the FP32 batched Dslash on this workload, and the kernel
# sources it was measured with: the traffic figure is reported only while they are unchanged.
COUNTERS = os.path.join(ROOT, "profiles", "dslash_f32_batched_16x16x16x16_nrhs12_counters.md")
KERNEL_SOURCES = ("paper_0710_1988_amd/csrc/dslash.hip", "paper_0710_1988_amd/csrc/kernels.h",
                  "paper_0710_1988_amd/csrc/common.h")


def kernel_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic():
    """Scaled FETCH_SIZE + WRITE_SIZE bytes per FP32 Dslash launch from the committed counter
    summary, or None when the summary is missing or the kernel sources changed since."""
    try:
        txt = open(COUNTERS).read()
    except OSError:
        return None, "no counter summary"
    m_t = re.search(r"^DSLASH_F32_TRAFFIC_BYTES_PER_LAUNCH = (\d+)", txt, re.M)
    m_h = re.search(r"^KERNEL_SOURCE_SHA256 = ([0-9a-f]{64})", txt, re.M)
    if not (m_t and m_h):
        return None, "counter summary incomplete"
    if m_h.group(1) != kernel_digest():
        return None, "kernel sources changed since the counters were taken"
    return float(m_t.group(1)), "profiles/" + os.path.basename(COUNTERS)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(U, L, kappa, b, mv_per_source):
    """The oracle, as written, timed on the host on a bounded sample: FP64 BiCGStab iterations
    on one source of the same 16^4 problem, scaled by the GPU's FP64 MVP count per source."""
    from threadpoolctl import threadpool_limits

    from oracle import solvers as S
    from oracle import wilson as W
    lat = W.Lattice(L)
    A = W.operator(U, lat, kappa)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        n_mv = 0
        while time.perf_counter() - t0 < 12.0:
            _, info = S.bicgstab(A, b.reshape(-1), tol=1e-30, max_mv=20)
            n_mv += info["matvecs"]
        dt = time.perf_counter() - t0
    per_mv = dt / n_mv
    return dict(value=per_mv * mv_per_source * 1e3, unit="ms/source", cores=1, kind="oracle",
                sample=f"{n_mv} MVPs of oracle FP64 BiCGStab (numpy, 1 thread) on one 16^4 source in "
                       f"{dt:.1f} s = {per_mv * 1e3:.1f} ms/MVP, scaled by the GPU FP64 solve's "
                       f"{mv_per_source:.0f} MVPs/source; host has {os.cpu_count()} logical CPUs")


def dslash_sweep(dbq, torch):
    """Pure Dslash kernel bandwidth (HIP events around each launch) beyond the 256 MB MALL."""
    import synth
    out = {}
    L = (24, 24, 24, 48)
    U = torch.from_numpy(synth.gauge_field(L, 0.6, 105)).cuda()
    for prec, nrhs, kind in (("fp64", 1, 0), ("mixed", 1, 1), ("mixed", 12, 1)):
        psi = torch.from_numpy(synth.z2_sources(L, nrhs, 1105)).cuda()
        dbq.wilson_apply(L, U, psi, 0.13, 0.0, False, prec)
        torch.cuda.synchronize()
        dbq.reset_timing()
        dbq.set_timing(True)
        for _ in range(5):
            dbq.wilson_apply(L, U, psi, 0.13, 0.0, False, prec)
        torch.cuda.synchronize()
        ms, n, by = dbq.kernel_time(kind)
        dbq.set_timing(False)
        out[f"{prec}_24x24x24x48_nrhs{nrhs}"] = dict(
            GBps=round(by / (ms * 1e-3) / 1e9, 1), us_per_launch=round(ms / n * 1e3, 1),
            MB_per_launch=round(by / n / 1e6, 1))
        del psi
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="skip the FP64 comparisons and sweep")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 256 MiB with a plain device copy (a known-size reference "
                         "for hardware byte counters)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the solve of "
              "independent sources would shard over GPUs with no communication; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_0710_1988_amd as dbq
    import synth
    if not torch.cuda.is_available():
        print("no GPU", file=sys.stderr)
        sys.exit(1)
    dev = "cuda:0"
    if a.calibrate_copy:
        src = torch.ones(1 << 26, dtype=torch.float32, device=dev)  # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 268435456 bytes read, 268435456 bytes written")
        del src, dst
    L = (16, 16, 16, 16)
    Vol = int(np.prod(L))
    nrhs, m, k, tol = 12, 60, 20, 1e-8
    Uh = synth.gauge_field(L, 0.6, 102)
    U = torch.from_numpy(Uh).to(dev)

    # ---- setup (untimed): kappa_c, GMRES-DR eigenvectors
    t = time.perf_counter()
    kc, lam, res, st = dbq.kappa_critical(L, U, m=48, k=16, tol=1e-10)
    t_kc = time.perf_counter() - t
    kappa = 0.995 * kc
    log(f"kappa_c = {kc:.8f} (lambda_max Re {lam.real:.6f}, resid {res:.1e}, {t_kc:.1f} s)")
    b0 = torch.from_numpy(synth.point_source(L)).to(dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    x0, V, theta, gst = dbq.gmresdr_first_rhs(L, U, b0, kappa, m, k, tol=tol)
    torch.cuda.synchronize()
    t_gd = time.perf_counter() - t
    log(f"GMRES-DR({m},{k}): {gst['matvecs']} MVPs, {gst['iterations']} cycles, status "
        f"{gst['status_name']}, {t_gd:.2f} s, k_out {V.shape[0]}")
    Bh = synth.z2_sources(L, nrhs, 1102)
    B = torch.from_numpy(Bh).to(dev)
    prob = dict(L=L, links=U, kappa=kappa, B=B, V=V)

    # ---- timed: mixed precision, all sources batched in one call
    for _ in range(a.warmup):
        dbq.dbicgstab_solve([prob], tol=tol, prec="mixed")
    torch.cuda.synchronize()
    dbq.reset_timing()
    dbq.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for _ in range(a.steps):
        X, stats, status = dbq.dbicgstab_solve([prob], tol=tol, prec="mixed")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dbq.set_timing(False)
    ms32, n32, by32 = dbq.kernel_time(1)
    ms64, n64, by64 = dbq.kernel_time(0)
    ms_step = (t1 - t0) * 1e3 / a.steps
    worst = max(s["rel_true_resid"] for s in stats)
    ok = all(s["status"] == 0 for s in stats)
    mv_mixed = float(np.mean([s["matvecs"] for s in stats]))
    log(f"mixed batched: {ms_step:.1f} ms/step, {ms_step / nrhs:.2f} ms/source, worst true resid "
        f"{worst:.2e}, all converged {ok}, MVPs/source {mv_mixed:.0f}")
    avg_us = ms32 / max(n32, 1) * 1e3
    ach = by32 / max(n32, 1) / (avg_us * 1e-6) / 1e9 if n32 else 0.0
    traffic, traffic_src = counter_traffic()
    out = {
        "metric": METRIC,
        "value": round(ms_step / nrhs, 4),
        "unit": "ms/source",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "16^4 Wilson, links exp(0.6iQ) seed 102, kappa=0.995 kappa_c, "
                               "D-BiCGStab(20) on 12 Z2 sources (seed 1102) batched, tol 1e-8, "
                               "FP32 inner / FP64 reliable updates, deflation from GMRES-DR(60,20)",
                   "lattice": list(L), "nrhs": nrhs, "k": int(V.shape[0]), "kappa": kappa,
                   "kappa_c": kc},
        "sources_per_s": round(nrhs / (ms_step * 1e-3), 2),
        "worst_rel_true_resid": worst,
        "all_converged": ok,
        "mvps_per_source": mv_mixed,
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "traffic_source": traffic_src,
                     "kernel": "k_dslash<float> (FP32 12-real links, 12 rhs per launch; "
                               "working set MALL-resident at 16^4)",
                     "avg_launch_us": round(avg_us, 2), "launches": n32,
                     "algorithmic_MB_per_launch": round(by32 / max(n32, 1) / 1e6, 2)},
        "fp64_dslash_in_step": {"launches": n64,
                                "avg_launch_us": round(ms64 / max(n64, 1) * 1e3, 2)},
        "setup": {"kappa_c_s": round(t_kc, 3), "gmresdr_s": round(t_gd, 3),
                  "gmresdr_mvps": gst["matvecs"], "gmresdr_status": gst["status_name"],
                  "gmresdr_ms_amortized_per_source": round(t_gd * 1e3 / nrhs, 3)},
    }
    mv64 = None
    if not a.quick:
        # FP64 plain single-rhs D-BiCGStab (the comparison point), two sources one at a time
        tt = []
        mvs = []
        for j in range(2):
            pj = dict(prob, B=B[j:j + 1])
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, sj, _ = dbq.dbicgstab_solve([pj], tol=tol, prec="fp64")
            torch.cuda.synchronize()
            tt.append(time.perf_counter() - t)
            mvs.append(sj[0]["matvecs"])
        mv64 = float(np.mean(mvs))
        fp64_ms = float(np.mean(tt)) * 1e3
        # undeflated FP64 BiCGStab, one source
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, su, _ = dbq.dbicgstab_solve([dict(L=L, links=U, kappa=kappa, B=B[:1])], tol=tol,
                                       prec="fp64")
        torch.cuda.synchronize()
        und_ms = (time.perf_counter() - t) * 1e3
        out["fp64_single_rhs_ms_per_source"] = round(fp64_ms, 3)
        out["fp64_single_rhs_mvps_per_source"] = mv64
        out["speedup_vs_fp64_single_rhs"] = round(fp64_ms / (ms_step / nrhs), 2)
        out["bicgstab_fp64_undeflated_ms_per_source"] = round(und_ms, 3)
        out["bicgstab_fp64_undeflated_mvps"] = su[0]["matvecs"]
        log(f"FP64 single-rhs: {fp64_ms:.1f} ms/source ({mv64:.0f} MVPs); undeflated "
            f"{und_ms:.1f} ms ({su[0]['matvecs']} MVPs)")
        del X
        out["dslash_24x24x24x48"] = dslash_sweep(dbq, torch)
        log(f"dslash sweep: {out['dslash_24x24x24x48']}")
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(Uh, L, kappa, Bh[0], mv64 or mv_mixed)
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
