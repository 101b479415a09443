"""Benchmark of the periodic-box pair sweep on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload headline|pk|bk|...]

Default (headline) workload: the largest single-GPU configuration, a
2^24-point weighted Thomas catalogue (2^20 parents, 16 children each,
sigma = 1 Mpc/h, weights uniform in [0.5, 1.5]) in a 1000 Mpc/h periodic box
with R0 = 15 Mpc/h.  One step is the whole hot path on device-resident
positions: the power spectrum (ell = 0, 2, 4, 60 log k-bins over 2-20 h/Mpc)
and the bispectrum (ell = 0..4, 16 log k-bins over 2-20 h/Mpc, the DDR^II term
from f_rand = 3 uniform randoms that the library draws on the device from a
seed), both in the mixed form: cell lists, pair enumeration, pair weights,
harmonic sums, Gram contraction, C-term sweep, merges and normalisation.

Beside it: the same step in the FP64 form (`fp64_form`), the 2e6-point power
spectrum (`pk_config2`, the mixed and table forms) and the FP64 brute-force
oracle on the host cores over a fixed subset of the same workload's
primaries (`cpu_baseline`).  Other workloads (--workload) time single
calls: the bispectrum (bk, bk5, their analytic-DDR^II forms), the 2^24-point
power spectrum (pk5), the 64-box batch (batch) and the survey-geometry power
spectrum (survey).

Prints one JSON line.  `value` is pair-weights per second: ordered pairs
inside R0 x n_k x n_ell for P plus (data-data + random-data ordered pairs)
x n_k x (ell_max+1)^2 for B, per second of the whole step.  `roofline` refers
to the dominant kernel, the bispectrum sweep k_bk_quad: its algorithmic
FLOPs per launch (bk_flops_per_pair, without the C sums in the mixed form,
which the C-term histogram sweep takes) over its average duration measured
with HIP events on the library's stream, against the chip's 157.3 TFLOP/s
FP32 vector peak (the kernel computes mostly in FP64, which issues at half
that rate; `frac_fp64` is the fraction of the 78.6 TFLOP/s FP64 peak).
`traffic` is read from the committed rocprofv3 counter summary of that
kernel when its sources are unchanged since the counters were taken, else
null.
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

METRIC = "pair-weights/s (P_ℓ & B_ℓ) + boxes/s, mixed vs FP64 GPU at ≤1e-6 rel err"
# FP32 vector peak: 256 CUs x 128 FP32 FMA per clock x 2 flop x 2.4 GHz.  Non-packed
# FP32 FMAs issue at this rate on gfx950 (twice the FP64 rate, 78.6 TFLOP/s).
PEAK_VALU_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
SWEEP_SOURCES = ["paper_2005_01739_amd/csrc/pk.hip", "paper_2005_01739_amd/csrc/specfun.h",
                 "paper_2005_01739_amd/csrc/coeffs.h"]
BK_SOURCES = ["paper_2005_01739_amd/csrc/bk.hip", "paper_2005_01739_amd/csrc/specfun.h",
              "paper_2005_01739_amd/csrc/coeffs.h", "paper_2005_01739_amd/csrc/fmac_dpp.h"]
PROFILE = os.path.join(ROOT, "profiles", "k_pk_far_mixed_thomas_2e6.md")
BK_PROFILE = os.path.join(ROOT, "profiles", "k_bk_quad_mixed_thomas_2p24.md")
BK3_PROFILE = os.path.join(ROOT, "profiles", "k_bk_quad_mixed_thomas_5e5.md")


def sweep_source_hash(sources=SWEEP_SOURCES) -> str:
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pktab_flops_per_pair(n_ell: int) -> float:
    """Algorithmic FP64 FLOPs per unordered pair of the table form: the
    separation and r^2 (8), sqrt, window and mu (16), the Legendre
    polynomials (3 per multipole above 0), the six Lagrange weights (25) and
    two multiplies per (multipole, node) (12 per multipole)."""
    return 49.0 + 3.0 * (n_ell - 1) + 12.0 * n_ell


def pk_flops_per_pair(n_k: int, n_ell: int) -> float:
    """Algorithmic FLOPs per unordered pair for the power-spectrum weights."""
    return 40.0 + 80.0 * (n_k + 1) + 5.0 * n_k * n_ell


def bk_flops_per_pair(n_k: int, ell_max: int, with_c: bool = True) -> float:
    """Algorithmic FLOPs per ordered pair for the bispectrum weights: the special
    functions at n_k+1 edges (60 shared + 10 per multipole per edge), the real
    harmonics (6 per y_lm), the A_lm sums (2 n_k (l_max+1)^2) and, when the fused
    kernel sums them (FP64 form, random primaries), the C^ab_l sums over a <= b
    (2 (l_max+1) n_k (n_k+1)/2).  The mixed form takes the data primaries' C from
    the separate C-term pair histogram."""
    n_l = ell_max + 1
    c_term = n_l * n_k * (n_k + 1) if with_c else 0.0
    return 40.0 + (60.0 + 10.0 * n_l) * (n_k + 1) + 6.0 * n_l * n_l + 2.0 * n_k * n_l * n_l + c_term


def traffic_from_profile(profile=PROFILE, sources=SWEEP_SOURCES):
    """HBM bytes per sweep launch from the committed counter summary, or None."""
    if not os.path.exists(profile):
        return None
    txt = open(profile).read()
    m = re.search(r"<!-- traffic-json (\{.*?\}) -->", txt, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("source_hash") != sweep_source_hash(sources):
        return None
    return d.get("bytes_per_launch")


def table_form(hp, pos, wl, steps: int, warmup: int):
    """The same workload in the table form (HIPSTER_TABLE): time per call
    over `steps` calls after `warmup`, and its largest relative deviation
    from the FP64 form over every output bin, measured here."""
    import torch
    kw = dict(box=wl.box, r0=wl.r0, k_edges=wl.k_edges_p, ell_max=wl.ell_max_p)
    for _ in range(warmup):
        hp.pk_ell(pos, precision="table", **kw)
    torch.cuda.synchronize()
    sweep_ms, pairs = 0.0, 0
    t0 = time.perf_counter()
    for _ in range(steps):
        got, info = hp.pk_ell(pos, precision="table", return_diag=True, **kw)
        sweep_ms += info["ms_sweep"]
        pairs = info["n_pairs"]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ref, rinfo = hp.pk_ell(pos, precision="fp64", return_diag=True, **kw)
    n_k, n_ell = len(wl.k_edges_p) - 1, wl.ell_max_p // 2 + 1
    return {"precision": "table", "value": pairs * n_k * n_ell / dt, "unit": "pair-weights/s",
            "ms_per_step": dt * 1e3, "avg_sweep_ms": sweep_ms / steps, "table_nodes": info["table_nodes"],
            "pair_count_equals_fp64": bool(pairs == rinfo["n_pairs"]),
            "max_rel_err_vs_fp64": float(np.max(np.abs(got - ref) / np.abs(ref)))}


def host_cores():
    """Threads this process may run on, and the CPU model."""
    threads = os.cpu_count() or 1
    try:
        threads = len(os.sched_getaffinity(0))
    except Exception:
        pass
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return threads, model


def cpu_baseline(wl, n_primaries: int = 16384, seed: int = 0):
    """Time the FP64 oracle on a fixed subset of primaries (every secondary)."""
    import oracle
    rng = np.random.default_rng(seed)
    mask = np.zeros(wl.n, np.uint8)
    mask[rng.choice(wl.n, n_primaries, replace=False)] = 1
    threads, _ = host_cores()
    t0 = time.perf_counter()
    ref = oracle.pk_ell(wl.pos, wl.weights, wl.box, wl.r0, wl.k_edges_p, wl.ell_max_p,
                        primary_mask=mask, nthreads=threads)
    dt = time.perf_counter() - t0
    n_k = len(wl.k_edges_p) - 1
    n_ell = wl.ell_max_p // 2 + 1
    pw = ref["n_pairs"] * n_k * n_ell
    return {"value": pw / dt, "unit": "pair-weights/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_primaries} random primaries of the {wl.n}-point catalogue against all "
                      f"{wl.n} secondaries ({ref['n_pairs']} ordered pairs, {dt:.1f} s)"}


def cpu_baseline_headline(wl, n_pk: int, n_bk: int, f_rand: float, seed: int, rseed: int = 0):
    """The FP64 oracle on the host cores over a fixed subset of the headline
    workload's primaries: P on n_pk data primaries, B on n_bk data and
    f_rand n_bk random primaries (the library's drawn catalogue, regenerated
    here by the oracle), every secondary; pair-weights per second of the
    two calls together, in the headline's units."""
    import oracle
    threads, model = host_cores()
    rng = np.random.default_rng(rseed)
    mp = np.zeros(wl.n, np.uint8)
    mp[rng.choice(wl.n, n_pk, replace=False)] = 1
    mb = np.zeros(wl.n, np.uint8)
    mb[rng.choice(wl.n, n_bk, replace=False)] = 1
    n_r = int(round(f_rand * wl.n))
    rpos = oracle.philox_randoms(n_r, wl.box, seed)
    mr = np.zeros(n_r, np.uint8)
    mr[rng.choice(n_r, int(round(f_rand * n_bk)), replace=False)] = 1
    t0 = time.perf_counter()
    rp = oracle.pk_ell(wl.pos, wl.weights, wl.box, wl.r0, wl.k_edges_p, wl.ell_max_p, primary_mask=mp,
                       nthreads=threads)
    t1 = time.perf_counter()
    rb = oracle.bk_ell(wl.pos, wl.weights, rpos, None, wl.box, wl.r0, wl.k_edges_b, wl.ell_max_b, mask_d=mb,
                       mask_r=mr, nthreads=threads)
    t2 = time.perf_counter()
    n_kp, n_lp = len(wl.k_edges_p) - 1, wl.ell_max_p // 2 + 1
    n_kb, n_lb = len(wl.k_edges_b) - 1, wl.ell_max_b + 1
    pw = rp["n_pairs"] * n_kp * n_lp + (rb["n_pairs_dd"] + rb["n_pairs_rd"]) * n_kb * n_lb * n_lb
    return {"value": pw / (t2 - t0), "unit": "pair-weights/s", "cores": threads, "kind": "oracle",
            "cpu_model": model, "nproc": os.cpu_count(),
            "sample": (f"P: {n_pk} random primaries of the {wl.n}-point catalogue against every secondary "
                       f"({rp['n_pairs']} ordered pairs, {t1 - t0:.1f} s); B: {n_bk} data and "
                       f"{int(round(f_rand * n_bk))} random primaries ({rb['n_pairs_dd']} + {rb['n_pairs_rd']} "
                       f"ordered pairs, {t2 - t1:.1f} s)")}


def headline(args, hp, torch, synthetic):
    """The whole hot path on the largest single-GPU configuration: P and B of
    the 2^24-point weighted box per step (see the module docstring)."""
    wl = synthetic.workload(5)
    f_rand, seed = wl.f_rand, wl.seed
    pos = torch.from_numpy(wl.pos).cuda()
    w = torch.from_numpy(wl.weights).cuda()
    n_kp, n_lp = len(wl.k_edges_p) - 1, wl.ell_max_p // 2 + 1
    n_kb, n_lb = len(wl.k_edges_b) - 1, wl.ell_max_b + 1
    ctx = hp.Context(0, torch.cuda.current_stream().cuda_stream)

    def step(prec):
        _, ip = hp.pk_ell(pos, w, box=wl.box, r0=wl.r0, k_edges=wl.k_edges_p, ell_max=wl.ell_max_p,
                          precision=prec, return_diag=True, ctx=ctx)
        _, ib = hp.bk_ell(pos, w, box=wl.box, r0=wl.r0, k_edges=wl.k_edges_b, ell_max=wl.ell_max_b,
                          precision=prec, f_rand=f_rand, seed=seed, return_diag=True, ctx=ctx)
        return ip, ib

    def timed(prec, steps, warmup):
        for _ in range(warmup):
            step(prec)
        torch.cuda.synchronize()
        acc = {"bk_sweep_ms": 0.0, "bk_launches": 0, "pk_sweep_ms": 0.0, "pk_far_ms": 0.0, "pk_launches": 0,
               "pk_ms": 0.0, "bk_ms": 0.0, "bk_cterm_ms": 0.0}
        t0 = time.perf_counter()
        for _ in range(steps):
            ip, ib = step(prec)
            acc["bk_sweep_ms"] += ib["ms_sweep"]
            acc["bk_launches"] += ib["sweep_launches"]
            acc["bk_ms"] += ib["ms_total"]
            acc["bk_cterm_ms"] += ib["ms_cterm"]
            acc["pk_sweep_ms"] += ip["ms_sweep"]
            acc["pk_far_ms"] += ip["ms_sweep_far"]
            acc["pk_launches"] += ip["sweep_launches"]
            acc["pk_ms"] += ip["ms_total"]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        pw_p = ip["n_pairs"] * n_kp * n_lp
        pw_b = (ib["n_pairs"] + ib["n_pairs_rand"]) * n_kb * n_lb * n_lb
        return dt, ip, ib, acc, pw_p, pw_b

    dt, ip, ib, acc, pw_p, pw_b = timed("mixed", args.steps, args.warmup)
    steps = args.steps
    # dominant kernel: the bispectrum sweep, two launches per step (data and
    # random primaries); the mixed form's C sums are the histogram sweep's
    launches_per_step = acc["bk_launches"] / steps
    bk_flops = (ib["n_pairs"] + ib["n_pairs_rand"]) * bk_flops_per_pair(n_kb, wl.ell_max_b, with_c=False)
    flops_per_launch = bk_flops / launches_per_step
    avg_launch_ms = acc["bk_sweep_ms"] / max(acc["bk_launches"], 1)
    achieved = flops_per_launch / (avg_launch_ms * 1e-3) / 1e12
    # every bispectrum kernel of the step (sweep + C-term histogram), against
    # the full per-pair model with the C sums
    bk_full = (ib["n_pairs"] + ib["n_pairs_rand"]) * bk_flops_per_pair(n_kb, wl.ell_max_b, with_c=True)
    bk_kernels_ms = (acc["bk_sweep_ms"] + acc["bk_cterm_ms"]) / steps
    whole_b = bk_full / (bk_kernels_ms * 1e-3) / 1e12
    pk_per_pair = pk_flops_per_pair(n_kp, n_lp)
    pk_far_ms = acc["pk_far_ms"] / steps
    out = {"metric": METRIC, "value": (pw_p + pw_b) / dt, "unit": "pair-weights/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
           "config": {"workload": wl.name, "n_points": wl.n, "box": wl.box, "r0": wl.r0, "weights": "U[0.5, 1.5]",
                      "pk": {"n_k": n_kp, "ells": [0, 2, 4], "k_range": [2.0, 20.0], "bins": "log"},
                      "bk": {"n_k": n_kb, "ell_max": wl.ell_max_b, "k_range": [2.0, 20.0], "bins": "log",
                             "f_rand": f_rand, "n_randoms": int(ib["n_rand"]), "randoms": "drawn on the device"},
                      "precision": "mixed"},
           "roofline": {"bound": "alu", "kernel": "k_bk_quad", "achieved": achieved, "peak": PEAK_VALU_TFLOPS,
                        "unit": "TFLOP/s", "frac": achieved / PEAK_VALU_TFLOPS,
                        "frac_fp64": achieved / PEAK_FP64_TFLOPS,
                        "traffic": traffic_from_profile(BK_PROFILE, BK_SOURCES),
                        "flops_per_launch": flops_per_launch, "avg_launch_ms": avg_launch_ms,
                        "pairs_per_launch": (ib["n_pairs"] + ib["n_pairs_rand"]) / launches_per_step,
                        "whole_bispectrum": {"kernels": "k_bk_quad + C-term histogram sweep",
                                             "flops_per_step": bk_full, "kernel_ms_per_step": bk_kernels_ms,
                                             "achieved": whole_b, "frac": whole_b / PEAK_VALU_TFLOPS}},
           "parts": {"pk": {"pair_weights": pw_p, "ordered_pairs": ip["n_pairs"], "ms": acc["pk_ms"] / steps,
                            "sweep_ms": acc["pk_sweep_ms"] / steps,
                            "far_kernel": {"ms": pk_far_ms, "pairs": ip["n_pairs_far"],
                                           "frac": (ip["n_pairs_far"] * pk_per_pair / (pk_far_ms * 1e-3) / 1e12
                                                    / PEAK_VALU_TFLOPS) if pk_far_ms > 0 else None}},
                     "bk": {"pair_weights": pw_b, "ordered_pairs_dd": ib["n_pairs"],
                            "ordered_pairs_rd": ib["n_pairs_rand"], "ms": acc["bk_ms"] / steps,
                            "sweep_ms": acc["bk_sweep_ms"] / steps, "cterm_ms": acc["bk_cterm_ms"] / steps}}}
    if not args.no_fp64_form:
        dt64, ip64, ib64, acc64, pwp64, pwb64 = timed("fp64", 1, 1)
        out["fp64_form"] = {"value": (pwp64 + pwb64) / dt64, "unit": "pair-weights/s", "ms_per_step": dt64 * 1e3,
                            "pk_ms": acc64["pk_ms"], "bk_ms": acc64["bk_ms"],
                            "pair_counts_equal": bool(ip64["n_pairs"] == ip["n_pairs"]
                                                      and ib64["n_pairs"] == ib["n_pairs"]
                                                      and ib64["n_pairs_rand"] == ib["n_pairs_rand"]),
                            "mixed_speedup": dt64 / dt}
    if not args.no_config2:
        wl2 = synthetic.workload(2)
        pos2 = torch.from_numpy(wl2.pos).cuda()
        nk2, nl2 = len(wl2.k_edges_p) - 1, wl2.ell_max_p // 2 + 1
        kw2 = dict(box=wl2.box, r0=wl2.r0, k_edges=wl2.k_edges_p, ell_max=wl2.ell_max_p, return_diag=True, ctx=ctx)
        for _ in range(2):
            hp.pk_ell(pos2, **kw2)
        torch.cuda.synchronize()
        n2, far2, fms2 = 10, 0, 0.0
        t0 = time.perf_counter()
        for _ in range(n2):
            _, i2 = hp.pk_ell(pos2, **kw2)
            fms2 += i2["ms_sweep_far"]
            far2 = i2["n_pairs_far"]
        torch.cuda.synchronize()
        dt2 = (time.perf_counter() - t0) / n2
        far_ach = far2 * pk_flops_per_pair(nk2, nl2) / (fms2 / n2 * 1e-3) / 1e12
        out["pk_config2"] = {"workload": wl2.name, "value": i2["n_pairs"] * nk2 * nl2 / dt2, "unit": "pair-weights/s",
                             "ms_per_step": dt2 * 1e3,
                             "roofline": {"kernel": "k_pk_far", "achieved": far_ach,
                                          "frac": far_ach / PEAK_VALU_TFLOPS, "avg_launch_ms": fms2 / n2,
                                          "traffic": traffic_from_profile()},
                             "table_form": table_form(hp, pos2, wl2, 10, 2)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_headline(wl, args.cpu_pk_primaries, args.cpu_bk_primaries, f_rand, seed)
    print(json.dumps(out), flush=True)


def calibrate_copy(nbytes: int = 1 << 30):
    """A plain device copy of known size, for scaling rocprofv3 byte counters."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": nbytes}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "pk", "pk-fp64", "pk-table", "bk", "bk-fp64", "pk5", "bk5", "batch", "survey", "survey-fp64", "survey-table",
                             "bk-analytic", "bk-analytic-fp64", "bk5-analytic", "cov", "batch-analytic", "bk-aniso"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-table-form", action="store_true",
                    help="pk workload: leave out the table-form measurement (for profiling the mixed path alone)")
    ap.add_argument("--cpu-primaries", type=int, default=16384)
    ap.add_argument("--cpu-pk-primaries", type=int, default=2048, help="headline: oracle P sample")
    ap.add_argument("--cpu-bk-primaries", type=int, default=512, help="headline: oracle B sample (data primaries)")
    ap.add_argument("--no-fp64-form", action="store_true", help="headline: leave out the FP64-form step")
    ap.add_argument("--no-config2", action="store_true", help="headline: leave out the 2e6-point power spectrum")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--scale", type=float, default=0.1,
                    help="batch workload: fraction of each box's N (pairs scale as its square)")
    ap.add_argument("--split", type=int, default=1,
                    help="batch workload: run the 64 boxes as this many batch calls of about equal work")
    ap.add_argument("--device-randoms", action="store_true",
                    help="batch workload: randoms drawn by the library (f_rand, seed) instead of given")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the pair sweep of one box is measured on one device and the multi-GPU sharding is a "
              "design note, not a measured path.", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return

    import torch
    import paper_2005_01739_amd as hp
    import synthetic

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.synchronize()
    if args.workload == "headline":
        headline(args, hp, torch, synthetic)
        return

    if args.workload in ("pk", "pk-fp64", "pk5", "pk-table"):
        wl = synthetic.workload(5 if args.workload == "pk5" else 2)
        prec = {"pk-fp64": "fp64", "pk-table": "table"}.get(args.workload, "mixed")
        pos = torch.from_numpy(wl.pos).cuda()
        w = None if wl.weights is None else torch.from_numpy(wl.weights).cuda()
        n_k, n_ell = len(wl.k_edges_p) - 1, wl.ell_max_p // 2 + 1

        def step():
            return hp.pk_ell(pos, w, box=wl.box, r0=wl.r0, k_edges=wl.k_edges_p, ell_max=wl.ell_max_p,
                             precision=prec, return_diag=True)
        units_per_pair = n_k * n_ell
        cfg = {"workload": wl.name, "n_points": wl.n, "box": wl.box, "r0": wl.r0, "n_k": n_k,
               "ells": list(range(0, wl.ell_max_p + 1, 2)), "k_range": [float(wl.k_edges_p[0]), float(wl.k_edges_p[-1])],
               "precision": prec, "weights": wl.weights is not None}
    elif args.workload in ("survey", "survey-fp64", "survey-table"):
        sv = synthetic.survey()
        prec = {"survey-fp64": "fp64", "survey-table": "table"}.get(args.workload, "mixed")
        pos = torch.from_numpy(sv.pos).cuda()
        rnd = torch.from_numpy(sv.randoms).cuda()
        n_k, n_ell = len(sv.k_edges) - 1, sv.ell_max // 2 + 1

        def step():
            out, info = hp.pk_survey(pos, None, rnd, volume=sv.volume, r0=sv.r0, k_edges=sv.k_edges,
                                     ell_max=sv.ell_max, precision=prec, return_diag=True)
            info = dict(info)
            info["n_pairs_rand"] = info["n_pairs_rand"] + info["n_pairs_rr"]
            return out, info
        units_per_pair = n_k * n_ell
        cfg = {"workload": sv.name, "n_points": sv.n, "n_randoms": int(sv.randoms.shape[0]), "volume": sv.volume,
               "r0": sv.r0, "n_k": n_k, "ells": list(range(0, sv.ell_max + 1, 2)),
               "k_range": [float(sv.k_edges[0]), float(sv.k_edges[-1])], "precision": prec,
               "estimator": "DD - 2DR + RR, pair-midpoint line of sight"}
    elif args.workload in ("bk", "bk-fp64", "bk5"):
        wl = synthetic.workload(5 if args.workload == "bk5" else 3)
        prec = "fp64" if args.workload == "bk-fp64" else "mixed"
        pos = torch.from_numpy(wl.pos).cuda()
        w = None if wl.weights is None else torch.from_numpy(wl.weights).cuda()
        n_k = len(wl.k_edges_b) - 1

        def step():
            # f_rand = 3 randoms drawn by the library on the device from the seed
            return hp.bk_ell(pos, w, box=wl.box, r0=wl.r0, k_edges=wl.k_edges_b, ell_max=wl.ell_max_b,
                             precision=prec, f_rand=wl.f_rand, seed=wl.seed, return_diag=True)
        units_per_pair = n_k * (wl.ell_max_b + 1) ** 2
        cfg = {"workload": wl.name, "n_points": wl.n, "n_randoms": int(round(wl.f_rand * wl.n)), "box": wl.box,
               "r0": wl.r0, "n_k": n_k, "ell_max": wl.ell_max_b, "precision": prec, "randoms": "drawn on the device"}
    elif args.workload == "bk-aniso":
        # the anisotropic bispectrum (l1 <= l2 <= 4, m <= l1: 35 combinations)
        # of the 5e5-point clustered box, 3N randoms drawn on the device
        wl = synthetic.workload(3)
        prec = "mixed"
        pos = torch.from_numpy(wl.pos).cuda()
        w = None
        n_k = len(wl.k_edges_b) - 1
        lmax_a = 4

        def step():
            out, info = hp.bk_aniso(pos, box=wl.box, r0=wl.r0, k_edges=wl.k_edges_b, ell_max=lmax_a,
                                    f_rand=wl.f_rand, seed=wl.seed, return_diag=True)
            info = dict(info)
            info["sweep_launches"] = 2
            return out, info
        units_per_pair = n_k * (lmax_a + 1) ** 2
        cfg = {"workload": wl.name + "_anisotropic", "n_points": wl.n, "n_randoms": int(round(wl.f_rand * wl.n)),
               "box": wl.box, "r0": wl.r0, "n_k": n_k, "ell_max": lmax_a, "n_combinations": 35,
               "precision": prec, "randoms": "drawn on the device", "line_of_sight": "z"}
    elif args.workload == "cov":
        # theory side: Gaussian covariance of the headline power spectrum's
        # binning (40 log bins over 1-10 h/Mpc, R0 = 25, l = 0, 2, 4) on a
        # 9600-node p quadrature over [0, 40] with a model power spectrum
        wl = synthetic.workload(2)
        k = wl.k_edges_p
        gx, gw = np.polynomial.legendre.leggauss(16)
        e = np.linspace(0.0, 40.0, 601)
        mid, half = 0.5 * (e[:-1] + e[1:]), 0.5 * (e[1:] - e[:-1])
        p = (mid[:, None] + half[:, None] * gx).ravel()
        wp = (half[:, None] * gw).ravel()
        pk = np.array([2e4 / (1 + (p / 0.1) ** 2), -4e3 / (1 + (p / 0.15) ** 2), 8e2 / (1 + (p / 0.2) ** 2)])
        V = wl.box ** 3
        ctx = hp.Context(0)
        n_k, n_ell = len(k) - 1, 3

        def step():
            t = time.perf_counter()
            hp.cov_gauss(wl.r0, V, k, 4, p, wp, pk, ctx=ctx)
            ms = (time.perf_counter() - t) * 1e3
            return None, {"ms_sweep": ms, "sweep_launches": 1, "n_pairs": 0}
        for _ in range(args.warmup):
            step()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        dt = (time.perf_counter() - t0) / args.steps
        # the dominant kernel's algorithmic work: omega's contraction, 2 FLOP per
        # (l, p node, bin, r node); the r node count follows the library's rule
        hmax = min(0.25 * wl.r0, 8.0 / max(p.max(), k[-1]))
        n_r = 16 * sum(max(1, int(np.ceil(d / hmax))) for d in (0.5 * wl.r0, 0.25 * wl.r0, 0.25 * wl.r0))
        flops = 2.0 * n_ell * p.size * n_k * n_r
        out = {"metric": METRIC, "value": 1.0 / dt, "unit": "covariances/s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "f64", "data": "synthetic",
               "config": {"workload": "cov_gauss_40bins_l024", "r0": wl.r0, "n_k": n_k, "ells": [0, 2, 4],
                          "p_nodes": int(p.size), "r_nodes": int(n_r)},
               "omega_flops": flops}
        print(json.dumps(out), flush=True)
        return
    elif args.workload in ("bk-analytic", "bk-analytic-fp64", "bk5-analytic"):
        wl = synthetic.workload(5 if args.workload == "bk5-analytic" else 3)
        prec = "fp64" if args.workload == "bk-analytic-fp64" else "mixed"
        pos = torch.from_numpy(wl.pos).cuda()
        w = None if wl.weights is None else torch.from_numpy(wl.weights).cuda()
        n_k = len(wl.k_edges_b) - 1
        n_tables = (wl.ell_max_b + 1) * n_k * (n_k + 1) // 2

        def step():
            out, info = hp.bk_ell_analytic(pos, w, box=wl.box, r0=wl.r0, k_edges=wl.k_edges_b,
                                           ell_max=wl.ell_max_b, precision=prec, return_diag=True)
            info = dict(info, sweep_launches=1, n_pairs_rand=0)
            return out, info
        units_per_pair = n_k * (wl.ell_max_b + 1) ** 2
        cfg = {"workload": wl.name + "_analytic_ddr2", "n_points": wl.n, "n_randoms": 0, "box": wl.box,
               "r0": wl.r0, "n_k": n_k, "ell_max": wl.ell_max_b, "precision": prec,
               "ddr2": "E^II kernel table + pair sweep to 2 R0 (no randoms)"}
    else:
        boxes = synthetic.batch_boxes(64, args.scale)
        analytic = args.workload == "batch-analytic"
        specs, work = [], []
        for b in boxes:
            pos = torch.from_numpy(b.pos).cuda()
            pk = dict(pk_edges=b.k_edges_p, pk_ell_max=b.ell_max_p)
            bk = dict(bk_edges=b.k_edges_b, bk_ell_max=b.ell_max_b)
            if analytic:
                bk["bk_eii_nodes"] = 0  # DDR^II from the E^II kernel, default table, no randoms
            elif args.device_randoms:
                bk["f_rand"], bk["seed"] = b.f_rand, b.seed  # drawn by the library on the device
            else:
                bk["randoms"] = torch.from_numpy(b.randoms()).cuda()
            # expected ordered pairs inside R0 (Poisson part)
            pairs = b.n * b.n / b.box ** 3 * 4.18879 * b.r0 ** 3
            if args.split > 1:
                # a box's P and B as two units of work (a P pair costs about a
                # quarter of a B pair visit)
                specs += [dict(pos=pos, box=b.box, r0=b.r0, **pk), dict(pos=pos, box=b.box, r0=b.r0, **bk)]
                work += [0.125 * pairs, pairs * (1.0 if analytic else 1.0 + b.f_rand)]
            else:
                specs.append(dict(pos=pos, box=b.box, r0=b.r0, **pk, **bk))
                work.append(pairs * (1.0 if analytic else 1.0 + b.f_rand))
        prec = "mixed"
        nkp, nkb = len(boxes[0].k_edges_p) - 1, len(boxes[0].k_edges_b) - 1
        print(f"batch inputs on the device: {len(boxes)} boxes ({len(specs)} P/B specs), "
              f"{sum(b.n for b in boxes)} points",
              file=sys.stderr, flush=True)
        # --split K: the 64 boxes' P and B as K batch calls of about equal
        # expected work (greedy, dearest first), each call's end printed as it
        # happens
        parts = [[] for _ in range(max(1, args.split))]
        load = [0.0] * len(parts)
        for i in sorted(range(len(specs)), key=lambda i: -work[i]):
            k = min(range(len(parts)), key=lambda k: load[k])
            parts[k].append(i)
            load[k] += work[i]
        parts = [sorted(p) for p in parts if p]

        def step():
            outs, info = [], {}
            for k, part in enumerate(parts):
                t = time.perf_counter()
                o, inf = hp.batch([specs[i] for i in part], precision=prec, return_diag=True)
                outs += o
                for key, v in inf.items():
                    info[key] = info.get(key, 0) + v if isinstance(v, (int, float)) else v
                if len(parts) > 1:
                    print(f"batch call {k + 1}/{len(parts)}: {len(part)} units, {time.perf_counter() - t:.1f} s",
                          file=sys.stderr, flush=True)
            info["n_pairs"] = sum(o["n_pairs"] for o, sp in zip(outs, [specs[i] for p in parts for i in p])
                                  if "pk_edges" in sp)
            return outs, info
        units_per_pair = None
        cfg = {"workload": "batch_64_boxes" + ("_analytic_ddr2" if analytic else ""), "n_boxes": 64,
               "scale": args.scale, "n_points_total": int(sum(b.n for b in boxes)),
               "pk": {"n_k": nkp, "ells": [0, 2, 4]}, "bk": {"n_k": nkb, "ell_max": boxes[0].ell_max_b},
               "randoms_per_point": 0 if analytic else 3,
               "randoms": None if analytic else ("drawn on the device" if args.device_randoms else "given"),
               "batch_calls": len(parts), "precision": prec}

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sweep_ms, far_ms, launches, pairs, pairs_r, far_pairs = 0.0, 0.0, 0, 0, 0, 0
    ddr2_ms, table_ms, pairs_2r0 = 0.0, 0.0, 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, info = step()
        sweep_ms += info["ms_sweep"]
        far_ms += info.get("ms_sweep_far", 0.0)
        launches += info["sweep_launches"]
        pairs = info["n_pairs"]
        pairs_r = info.get("n_pairs_rand", 0)
        far_pairs = info.get("n_pairs_far", 0)
        ddr2_ms += info.get("ms_ddr2", 0.0)
        table_ms += info.get("ms_eii_table", 0.0)
        pairs_2r0 = info.get("n_pairs_2r0", 0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt * 1e3 / args.steps
    if args.workload in ("bk-analytic", "bk-analytic-fp64", "bk5-analytic"):
        # DD pairs inside R0 carry n_k (l_max+1)^2 weights (the a_lm sums); each
        # (pair, image) inside 2 R0 carries one interpolated kernel value per
        # (l, a <= b) table
        # the rate in its own unit: DD pair-weights of the randoms-free
        # estimator per second of the whole call (the 2 R0 stage's (pair, image)
        # terms are reported beside it, per second of that stage)
        value = pairs * units_per_pair / (dt / args.steps)
        avg_launch_ms = sweep_ms / max(launches, 1)
        flops = pairs * bk_flops_per_pair(n_k, wl.ell_max_b, with_c=prec == "fp64") / (launches / args.steps)
        achieved = flops / (avg_launch_ms * 1e-3) / 1e12
        # the table depends on (R0, bins) only: built in the warm-up, reused by the
        # context in the timed steps; its cold build time is reported beside
        _, cold = hp.bk_ell_analytic(pos, w, box=wl.box, r0=wl.r0, k_edges=wl.k_edges_b, ell_max=wl.ell_max_b,
                                     precision=prec, ctx=hp.Context(0), return_diag=True)
        out = {"metric": METRIC, "value": value, "unit": "DD pair-weights/s (analytic DDR^II)", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32" if prec == "mixed" else "f64",
               "data": "synthetic", "config": cfg,
               "ddr2_terms_per_s": pairs_2r0 * n_tables / (ddr2_ms / args.steps * 1e-3) if ddr2_ms > 0 else None,
               "roofline": {"bound": "alu", "kernel": "k_bk_quad", "achieved": achieved, "peak": PEAK_VALU_TFLOPS,
                            "unit": "TFLOP/s", "frac": achieved / PEAK_VALU_TFLOPS,
                            "frac_fp64": achieved / PEAK_FP64_TFLOPS, "traffic": None, "flops_per_launch": flops,
                            "avg_launch_ms": avg_launch_ms},
               "pairs_per_step": pairs, "pairs_2r0_per_step": pairs_2r0, "n_tables": n_tables,
               "avg_ddr2_ms": ddr2_ms / args.steps, "table_ms_in_steps": table_ms / args.steps,
               "table_ms_cold": cold["ms_eii_table"], "eii_nodes": cold["eii_nodes"],
               "ms_per_step_with_cold_table": ms_step + cold["ms_eii_table"]}
        print(json.dumps(out), flush=True)
        return
    if args.workload in ("batch", "batch-analytic"):
        value = 64 / (dt / args.steps)
        out = {"metric": METRIC, "value": value, "unit": "boxes/s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic", "config": cfg,
               "pk_pairs_per_step": pairs, "avg_sweep_ms": sweep_ms / args.steps}
        print(json.dumps(out), flush=True)
        return
    value = (pairs + pairs_r) * units_per_pair / (dt / args.steps)

    out = {"metric": METRIC, "value": value, "unit": "pair-weights/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64+f32" if prec == "mixed" else "f64", "data": "synthetic",
           "config": cfg}
    if prec == "table":
        out["dtype"] = "f64+i64"
    avg_launch_ms = sweep_ms / max(launches, 1)
    if args.workload in ("pk-table", "survey-table"):
        # histogram-sweep launches (one per pair set); their algorithmic FP64
        # work per unordered pair inside R0 (pktab_flops_per_pair), against
        # the FP64 vector peak: the kernel is bound by LDS atomics and
        # pair-finding latency, not by this arithmetic
        flops = ((pairs + pairs_r) / 2.0) * pktab_flops_per_pair(n_ell) / (launches / args.steps)
        avg_launch_ms = sweep_ms / max(launches, 1)
        achieved = flops / (avg_launch_ms * 1e-3) / 1e12
        out["roofline"] = {"bound": "alu", "kernel": "k_ddr2_hist<kHistPk>", "achieved": achieved,
                           "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                           "traffic": None, "flops_per_launch": flops, "avg_launch_ms": avg_launch_ms}
    elif args.workload in ("pk", "pk-fp64", "pk5", "survey", "survey-fp64"):
        unordered = (pairs + pairs_r) / 2.0
        per_pair = pk_flops_per_pair(n_k, n_ell)
        flops = unordered * per_pair / (launches / args.steps)
        achieved = flops / (avg_launch_ms * 1e-3) / 1e12
        sweep = {"kernels": "k_pk_sweep + k_pk_far", "achieved": achieved, "frac": achieved / PEAK_VALU_TFLOPS,
                 "frac_fp64": achieved / PEAK_FP64_TFLOPS,
                 "flops_per_launch": flops, "avg_launch_ms": avg_launch_ms}
        if far_pairs > 0 and far_ms > 0.0:
            # the dominant kernel: the far-pair kernel, timed on its own
            far_flops = far_pairs * per_pair / (launches / args.steps)
            far_avg = far_ms / max(launches, 1)
            far_ach = far_flops / (far_avg * 1e-3) / 1e12
            out["roofline"] = {"bound": "alu", "kernel": "k_pk_far", "achieved": far_ach, "peak": PEAK_VALU_TFLOPS,
                               "unit": "TFLOP/s", "frac": far_ach / PEAK_VALU_TFLOPS,
                               "frac_fp64": far_ach / PEAK_FP64_TFLOPS,
                               "traffic": traffic_from_profile() if args.workload == "pk" else None,
                               "flops_per_launch": far_flops, "avg_launch_ms": far_avg,
                               "pairs_per_launch": far_pairs / (launches / args.steps), "whole_sweep": sweep}
        else:
            out["roofline"] = {"bound": "alu", "kernel": "k_pk_sweep", "achieved": achieved,
                               "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_VALU_TFLOPS,
                               "frac_fp64": achieved / PEAK_FP64_TFLOPS,
                               "traffic": None, "flops_per_launch": flops, "avg_launch_ms": avg_launch_ms}
    else:
        # both primary catalogues, per launch (data primaries, then random primaries)
        lm = lmax_a if args.workload == "bk-aniso" else wl.ell_max_b
        flops = ((pairs + pairs_r) * bk_flops_per_pair(n_k, lm, with_c=prec == "fp64")
                 / (launches / args.steps))
        achieved = flops / (avg_launch_ms * 1e-3) / 1e12
        kname = "k_bk_quad (anisotropic contraction)" if args.workload == "bk-aniso" else "k_bk_quad"
        out["roofline"] = {"bound": "alu", "kernel": kname, "achieved": achieved, "peak": PEAK_VALU_TFLOPS,
                           "unit": "TFLOP/s", "frac": achieved / PEAK_VALU_TFLOPS,
                           "frac_fp64": achieved / PEAK_FP64_TFLOPS,
                           "traffic": (traffic_from_profile(BK3_PROFILE, BK_SOURCES)
                                       if args.workload == "bk" and prec == "mixed" else None),
                           "flops_per_launch": flops, "avg_launch_ms": avg_launch_ms}
    out["pairs_per_step"] = pairs + pairs_r
    if args.workload == "pk" and not args.no_table_form:
        out["table_form"] = table_form(hp, pos, wl, args.steps, args.warmup)
    if not args.no_cpu_baseline and args.workload == "pk":
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_primaries)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
