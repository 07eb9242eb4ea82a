"""Benchmark of the SPAI-smoothed multigrid hot path on one MI355X.

One step = one FP64 V(1,1) solve to ||r_k|| <= 1e-10 ||r_0|| of each of the
two fixed-size Poisson workloads (2D N=4096, 4095^2 unknowns, M9 smoother;
3D N=256, 255^3 unknowns, M7 smoother), from the same seeded initial guess,
with inputs resident in HBM.  The headline value is fine-grid unknowns per
second per V-cycle over the pair: sum(unknowns x cycles) / sum(solve time).

Also reported: per-workload rates, the roofline of the dominant kernel (the
fine-level fused residual + smoother sweep, timed live with HIP events on the
launch stream), the time to 1e-10 of the 3D N=512 noisy problem in FP64 and
with FP32 / FP16 V-cycles inside FP64 refinement, and the CPU oracle timed on
a bounded sample of the same workloads (single thread).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
       [--no-mixed] [--workloads a,b]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes of one fine-level fused smoother sweep per point in FP64:
# read u and b, write the new iterate
SMOOTH_BYTES_PER_PT = 24.0

WORKLOADS = {"poisson2d_n4096": (2, 4096), "poisson3d_n256": (3, 256)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--workloads", default="poisson2d_n4096,poisson3d_n256")
    ap.add_argument("--tol", type=float, default=1e-10)
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                          "(the multi-GPU decomposition is a design, not code)"}))
        sys.exit(2)
    import torch

    from paper_2206_05543_amd import M7, M9
    from paper_2206_05543_amd._lib import Multigrid
    from paper_2206_05543_amd.workloads import workload

    torch.cuda.init()
    stream = torch.cuda.current_stream()
    names = [w for w in a.workloads.split(",") if w]
    probs = {}
    for name in names:
        d, N = WORKLOADS[name]
        p = workload(name)
        mg = Multigrid(N, d, M9 if d == 2 else M7, max_cycles=100, timing=1)
        probs[name] = dict(d=d, N=N, mg=mg, b=torch.from_numpy(p["b"]).cuda(),
                           u0=torch.from_numpy(p["u0"]).cuda(),
                           u=torch.empty_like(torch.from_numpy(p["u0"])).cuda())
        print(f"[bench] loaded {name}", file=sys.stderr, flush=True)

    def step():
        out = {}
        for name, P in probs.items():
            P["u"].copy_(P["u0"])
            st = P["mg"].solve(P["b"], P["u"], tol=a.tol)
            if st["code"] != 0:
                raise RuntimeError(f"{name}: solve failed {st}")
            out[name] = st
        return out

    for i in range(a.warmup):
        step()
        print(f"[bench] warmup {i + 1}/{a.warmup}", file=sys.stderr, flush=True)
    for P in probs.values():
        P["mg"].reset_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per = {n: {"cycles": 0, "ms": 0.0} for n in probs}
    for i in range(a.steps):
        res = step()
        for n, st in res.items():
            per[n]["cycles"] += st["cycles"]
            per[n]["ms"] += st["elapsed_ms"]
        print(f"[bench] step {i + 1}/{a.steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    total_uc = 0.0
    details = {}
    smooth_stats = {}
    for n, P in probs.items():
        pts = (P["N"] - 1) ** P["d"]
        uc = pts * per[n]["cycles"]
        total_uc += uc
        ms, cnt = P["mg"].timing("smooth", 0)
        avg_us = ms / cnt * 1e3 if cnt else float("nan")
        gbs = SMOOTH_BYTES_PER_PT * pts / (avg_us * 1e-6) / 1e9 if cnt else float("nan")
        smooth_stats[n] = (avg_us, gbs, ms)
        details[n] = {
            "unknowns": pts,
            "cycles_per_solve": per[n]["cycles"] / a.steps,
            "solve_ms": per[n]["ms"] / a.steps,
            "unknowns_per_s_per_cycle": uc / (per[n]["ms"] * 1e-3),
            "fine_smooth_us": avg_us,
            "fine_smooth_GBps": gbs,
        }
    value = total_uc / wall
    dom = max(smooth_stats, key=lambda n: smooth_stats[n][2])
    avg_us, gbs, _ = smooth_stats[dom]

    line = {
        "metric": "fine-grid unknowns/s per V-cycle",
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": wall / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded sine-mode right-hand sides, U[-1,1] initial guess",
        "config": {"workload": "+".join(names), "tol": a.tol, "cycle": "V(1,1)",
                   "smoothers": {"2D": "M9 (Theorem 3.1)", "3D": "M7 (Theorem 3.2)"}},
        "per_workload": details,
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": f"fine-level fused residual+SPAI smoother ({dom})",
                     "avg_launch_us": avg_us,
                     "algorithmic_bytes_per_launch": SMOOTH_BYTES_PER_PT *
                     (probs[dom]["N"] - 1) ** probs[dom]["d"]},
    }
    for P in probs.values():
        P["mg"].close()
    del probs
    torch.cuda.empty_cache()

    if not a.no_mixed:
        line["mixed_precision"] = mixed(a.tol)
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


def mixed(tol):
    """Time to tol of the 3D N=512 noisy problem: FP64 V-cycles vs FP32 and
    FP16 V-cycles inside FP64 refinement (same GPU, same input)."""
    import torch

    from paper_2206_05543_amd import M7
    from paper_2206_05543_amd._lib import Multigrid
    from paper_2206_05543_amd.workloads import workload

    print("[bench] mixed precision: generating 3D N=512 input", file=sys.stderr, flush=True)
    p = workload("poisson3d_n512_noisy")
    b = torch.from_numpy(p["b"]).cuda()
    u0 = torch.from_numpy(p["u0"]).cuda()
    del p
    out = {"workload": "poisson3d_n512_noisy", "unknowns": 511 ** 3}
    ref = None
    for prec in ("fp64", "fp32_ir", "fp16_ir"):
        mg = Multigrid(512, 3, M7, precision=prec, max_cycles=100)
        u = u0.clone()
        mg.solve(b, u, tol=tol)  # warm-up
        times = []
        for _ in range(3):
            u.copy_(u0)
            st = mg.solve(b, u, tol=tol)
            times.append(st["elapsed_ms"])
        rk = mg.residual_norm(b, u)
        rec = {"time_ms": min(times), "cycles": st["cycles"], "code": st["code"],
               "rel_residual": rk / st["r0"]}
        if prec == "fp64":
            ref = u.clone()
        else:
            rec["rel_diff_vs_fp64"] = float((u - ref).norm() / ref.norm())
        out[prec] = rec
        mg.close()
        print(f"[bench] mixed {prec}: {rec}", file=sys.stderr, flush=True)
    out["speedup_fp32_ir"] = out["fp64"]["time_ms"] / out["fp32_ir"]["time_ms"]
    out["speedup_fp16_ir"] = out["fp64"]["time_ms"] / out["fp16_ir"]["time_ms"]
    return out


def cpu_baseline():
    """The CPU oracle (plain FP64 loops, one thread) on a bounded sample: two
    consecutive V(1,1) cycles of each workload of the step."""
    import oracle as O
    from paper_2206_05543_amd import M7, M9
    from paper_2206_05543_amd.workloads import workload

    O.lib()
    total_uc, total_s = 0.0, 0.0
    for name, (d, N) in WORKLOADS.items():
        p = workload(name)
        c = np.array(M9 if d == 2 else M7)
        t = time.perf_counter()
        u = O.vcycle(d, N, c, p["u0"], p["b"])
        O.vcycle(d, N, c, u, p["b"])
        total_s += time.perf_counter() - t
        total_uc += 2 * (N - 1) ** d
        print(f"[bench] cpu oracle {name}: {time.perf_counter() - t:.1f} s", file=sys.stderr,
              flush=True)
    return {"value": total_uc / total_s, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": "two V(1,1) cycles of 2D N=4096 and two of 3D N=256 "
                      f"({total_s:.1f} s single-threaded)"}


if __name__ == "__main__":
    main()
