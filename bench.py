"""Benchmark of the periodic-box pair sweep on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload pk|bk|pk5|bk5|batch|survey]

Default workload: the mixed-precision power spectrum of a 2,000,000-point
Thomas cluster catalogue (10 children per parent, sigma = 2 Mpc/h, extra
N(0, 4 Mpc/h) line-of-sight displacement) in a 1000 Mpc/h periodic box,
R0 = 25 Mpc/h, ell = 0, 2, 4, 40 log-spaced k-bins over 1-10 h/Mpc.  One step
is one full hipster_pk_ell call on device-resident positions: cell list,
pair enumeration, pair-weight sweep, merge and normalisation.

Other workloads: the bispectrum (bk, bk5), the 2^24-point box (pk5), the
64-box batch (batch) and the survey-geometry power spectrum (survey: 1e6 Thomas
points and 3e6 randoms in a 1000 Mpc/h cube 1000-2000 Mpc/h from the observer,
DD - 2DR + RR with the pair-midpoint line of sight; pairs are the ordered DD,
DR + RD and RR pairs).

Prints one JSON line.  `value` is pair-weights per second (ordered pairs
inside R0 x n_k x n_ell, per second of the whole step).  `roofline` refers to
the dominant kernel: for the mixed power spectrum the far-pair sweep kernel
k_pk_far (pairs with every edge on the large-argument side, about 90% of the
pairs), otherwise the whole pair-weight sweep; algorithmic FLOPs per launch
(the per-pair model 40 + 80 (n_k+1) + 5 n_k n_ell per unordered pair, times
the pairs that launch sweeps) over its average duration measured with HIP
events on the library's stream, against the chip's 157.3 TFLOP/s FP32 vector
peak (the kernels compute mostly in FP64, which issues at half that rate;
`frac_fp64` gives the fraction of the 78.6 TFLOP/s FP64 vector peak).
`roofline.whole_sweep` gives the same figures for both sweep kernels
together.  `traffic` is read from the committed rocprofv3 counter summary of
that kernel when the kernel's sources are unchanged since the counters were
taken, else null.
`cpu_baseline` times the FP64 brute-force oracle on the host cores over a
fixed subset of primaries of the same catalogue.
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
PROFILE = os.path.join(ROOT, "profiles", "k_pk_far_mixed_thomas_2e6.md")


def sweep_source_hash() -> str:
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
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


def traffic_from_profile():
    """HBM bytes per sweep launch from the committed counter summary, or None."""
    if not os.path.exists(PROFILE):
        return None
    txt = open(PROFILE).read()
    m = re.search(r"<!-- traffic-json (\{.*?\}) -->", txt, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("source_hash") != sweep_source_hash():
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


def cpu_baseline(wl, n_primaries: int = 16384, seed: int = 0):
    """Time the FP64 oracle on a fixed subset of primaries (every secondary)."""
    import oracle
    rng = np.random.default_rng(seed)
    mask = np.zeros(wl.n, np.uint8)
    mask[rng.choice(wl.n, n_primaries, replace=False)] = 1
    threads = os.cpu_count() or 1
    try:
        threads = len(os.sched_getaffinity(0))
    except Exception:
        pass
    threads = min(threads, 16)
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="pk",
                    choices=["pk", "pk-fp64", "pk-table", "bk", "bk-fp64", "pk5", "bk5", "batch", "survey", "survey-fp64", "survey-table",
                             "bk-analytic", "bk-analytic-fp64", "bk5-analytic", "cov", "batch-analytic"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-table-form", action="store_true",
                    help="pk workload: leave out the table-form measurement (for profiling the mixed path alone)")
    ap.add_argument("--cpu-primaries", type=int, default=16384)
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--scale", type=float, default=0.1,
                    help="batch workload: fraction of each box's N (pairs scale as its square)")
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
        rnd = torch.from_numpy(wl.randoms()).cuda()
        n_k = len(wl.k_edges_b) - 1

        def step():
            return hp.bk_ell(pos, w, rnd, box=wl.box, r0=wl.r0, k_edges=wl.k_edges_b, ell_max=wl.ell_max_b,
                             precision=prec, return_diag=True)
        units_per_pair = n_k * (wl.ell_max_b + 1) ** 2
        cfg = {"workload": wl.name, "n_points": wl.n, "n_randoms": int(rnd.shape[0]), "box": wl.box, "r0": wl.r0,
               "n_k": n_k, "ell_max": wl.ell_max_b, "precision": prec}
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
        specs = []
        for b in boxes:
            pos = torch.from_numpy(b.pos).cuda()
            spec = dict(pos=pos, box=b.box, r0=b.r0, pk_edges=b.k_edges_p, pk_ell_max=b.ell_max_p,
                        bk_edges=b.k_edges_b, bk_ell_max=b.ell_max_b)
            if analytic:
                spec["bk_eii_nodes"] = 0  # DDR^II from the E^II kernel, default table, no randoms
            else:
                spec["randoms"] = torch.from_numpy(b.randoms()).cuda()
            specs.append(spec)
        prec = "mixed"
        nkp, nkb = len(boxes[0].k_edges_p) - 1, len(boxes[0].k_edges_b) - 1

        def step():
            outs, info = hp.batch(specs, precision=prec, return_diag=True)
            info["n_pairs"] = sum(o["n_pairs"] for o in outs)
            return outs, info
        units_per_pair = None
        cfg = {"workload": "batch_64_boxes" + ("_analytic_ddr2" if analytic else ""), "n_boxes": 64,
               "scale": args.scale, "n_points_total": int(sum(b.n for b in boxes)),
               "pk": {"n_k": nkp, "ells": [0, 2, 4]}, "bk": {"n_k": nkb, "ell_max": boxes[0].ell_max_b},
               "randoms_per_point": 0 if analytic else 3, "precision": prec}

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
        value = (pairs * units_per_pair + pairs_2r0 * n_tables) / (dt / args.steps)
        avg_launch_ms = sweep_ms / max(launches, 1)
        flops = pairs * bk_flops_per_pair(n_k, wl.ell_max_b, with_c=prec == "fp64") / (launches / args.steps)
        achieved = flops / (avg_launch_ms * 1e-3) / 1e12
        # the table depends on (R0, bins) only: built in the warm-up, reused by the
        # context in the timed steps; its cold build time is reported beside
        _, cold = hp.bk_ell_analytic(pos, w, box=wl.box, r0=wl.r0, k_edges=wl.k_edges_b, ell_max=wl.ell_max_b,
                                     precision=prec, ctx=hp.Context(0), return_diag=True)
        out = {"metric": METRIC, "value": value, "unit": "pair-weights/s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "f64+f32" if prec == "mixed" else "f64", "data": "synthetic",
               "config": cfg,
               "roofline": {"bound": "alu", "kernel": "k_bk_fused", "achieved": achieved, "peak": PEAK_VALU_TFLOPS,
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
        flops = (pairs * bk_flops_per_pair(n_k, wl.ell_max_b, with_c=prec == "fp64")
                 + pairs_r * bk_flops_per_pair(n_k, wl.ell_max_b)) / (launches / args.steps)
        achieved = flops / (avg_launch_ms * 1e-3) / 1e12
        out["roofline"] = {"bound": "alu", "kernel": "k_bk_fused", "achieved": achieved, "peak": PEAK_VALU_TFLOPS,
                           "unit": "TFLOP/s", "frac": achieved / PEAK_VALU_TFLOPS,
                           "frac_fp64": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                           "flops_per_launch": flops, "avg_launch_ms": avg_launch_ms}
    out["pairs_per_step"] = pairs + pairs_r
    if args.workload == "pk" and not args.no_table_form:
        out["table_form"] = table_form(hp, pos, wl, args.steps, args.warmup)
    if not args.no_cpu_baseline and args.workload == "pk":
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_primaries)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
