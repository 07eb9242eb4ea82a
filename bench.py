"""Benchmark of the SPAI-smoothed multigrid hot path on one MI355X.

One step = one FP64 V(1,1) solve to ||r_k|| <= 1e-10 ||r_0|| of each of the
two fixed-size Poisson workloads (2D N=4096, 4095^2 unknowns, M9 smoother;
3D N=256, 255^3 unknowns, M7 smoother), from the same seeded initial guess,
with inputs resident in HBM.  The headline value is fine-grid unknowns per
second per V-cycle over the pair: sum(unknowns x cycles) / sum(solve time).

Also reported: per-workload rates, the roofline of the dominant kernel (of
the fine-level kernels timed live with HIP events on the launch stream, the
one with the largest total time), per-level kernel times and GB/s (extra solves after the timed
region, every launch timed), the time to 1e-10 of the 3D N=512 noisy problem in FP64 and
with FP32 / FP16 V-cycles inside FP64 refinement, forward and backward times
of the two gradient workloads, and the CPU oracle timed on
a bounded sample of the same workloads (all host threads, and one thread).

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
# algorithmic bytes per fine point of the two fine-level kernels in FP64:
# read u and b, write the new iterate, and once per coarse node (8 / 2^d
# bytes per fine point) write the coarse right-hand side (the pre-smoother
# fused with the restriction) or read the coarse correction (the
# post-smoother)
SWEEP_KINDS = ("smooth_restrict", "post_pre_restrict", "smooth_correct")  # timed if timed
SWEEP_NAMES = {"smooth_restrict": "fine-level fused residual + SPAI pre-smoother + "
                                  "residual + full-weighting restriction",
               "post_pre_restrict": "fine-level fused coarse correction + SPAI post-smoother + "
                                    "next cycle's SPAI pre-smoother + residual + "
                                    "full-weighting restriction",
               "smooth_correct": "fine-level fused residual + SPAI post-smoother with the "
                                 "coarse correction"}


def launches_per_solve(kind, d, run):
    """Launches of a fine-level fused kernel in one FP64 solve that ran `run`
    cycles (pre-smoothers): 2D solves chain the cycles, so the first cycle's
    pre-smoother is the only `smooth_restrict` and every later one is fused
    with the previous post-smoother; 3D solves run one of each per cycle."""
    if d == 2:
        return 1.0 if kind == "smooth_restrict" else (run - 1.0 if kind == "post_pre_restrict"
                                                      else 0.0)
    return run if kind in ("smooth_restrict", "smooth_correct") else 0.0


def sweep_bytes_per_pt(kind, d):
    c = 8.0 / 2 ** d
    # the chained kernel reads u1, b and the coarse correction and writes
    # u_{k+1}, the next u1 and the coarse right-hand side
    return 32.0 + 2 * c if kind == "post_pre_restrict" else 24.0 + c


# HBM traffic of these sweeps, per launch, from rocprofv3 --pmc runs of this
# benchmark (FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch), each scaled
# by what the same counter reads for the benchmark's own device copy of the
# initial guess (a plain copy of known size in the same process): FETCH_SIZE
# reads half the copied bytes, WRITE_SIZE all of them.  The summaries and
# commands are in profiles/hbm_counters_fp64_sweeps.md.  Valid for the
# kernels and launch shapes they were taken on; set to None when those change.
PMC = {
    ("poisson3d_n256", "smooth_restrict"): (142654, 146079),
    ("poisson3d_n256", "smooth_correct"): (144893, 144825),
    ("poisson2d_n4096", "smooth_restrict"): (143194, 165892),
    ("poisson2d_n4096", "post_pre_restrict"): (159426, 301422),
    # the refinement solves' fine-level sweeps at 3D N=512, per storage
    # precision (profiles/hbm_counters_lowprec_sweeps.md)
    ("poisson3d_n512_noisy:fp16_ir", "smooth_correct"): (290990, 333261),
    ("poisson3d_n512_noisy:fp16_ir", "smooth_restrict"): (276448, 301305),
    ("poisson3d_n512_noisy:fp16_ir", "zero_smooth_restrict"): (138316, 293086),
    ("poisson3d_n512_noisy:fp32_ir", "smooth_correct"): (591048, 579097),
    ("poisson3d_n512_noisy:fp32_ir", "smooth_restrict"): (767053, 655203),
    ("poisson3d_n512_noisy:fp32_ir", "zero_smooth_restrict"): (276358, 586599),
}
PMC_COPY = {  # copy bytes, FETCH_SIZE KiB, WRITE_SIZE KiB of the same run
    "poisson3d_n256": (255 ** 3 * 8, 64782, 129542),
    "poisson2d_n4096": (4095 ** 2 * 8, 65516, 131008),
    "poisson3d_n512_noisy:fp16_ir": (511 ** 3 * 8, 521234, 1042444),
    "poisson3d_n512_noisy:fp32_ir": (511 ** 3 * 8, 521234, 1042444),
}


def hbm_traffic(name, kind):
    """Measured HBM bytes per launch of a fine-level sweep (None if unmeasured)."""
    if (name, kind) not in PMC or name not in PMC_COPY:
        return None
    fetch, write = PMC[(name, kind)]
    cbytes, cfetch, cwrite = PMC_COPY[name]
    return fetch * (cbytes / (cfetch * 1024.0)) * 1024.0 + write * (cbytes / (cwrite * 1024.0)) * 1024.0

WORKLOADS = {"poisson2d_n4096": (2, 4096), "poisson3d_n256": (3, 256)}

# algorithmic FP64 bytes per fine point of a level, per timed kernel kind
# (the tail is reported by time only)
LEVEL_KINDS = ("smooth", "smooth_zero", "restrict", "smooth_restrict", "post_pre_restrict",
               "zero_smooth_restrict", "smooth_correct", "prolong", "tail")


def level_bytes_per_pt(kind, d):
    c = 8.0 / 2 ** d  # one coarse value per 2^d fine points
    return {"smooth": 24.0, "smooth_zero": 16.0, "restrict": 16.0 + c,
            "smooth_restrict": 24.0 + c, "post_pre_restrict": 32.0 + 2 * c,
            "zero_smooth_restrict": 16.0 + c,
            "smooth_correct": 24.0 + c,
            "prolong": 16.0 + c}.get(kind)


def per_level(probs, tol, solves=2):
    """Per-level kernel times and algorithmic GB/s (fraction of 8 TB/s) from
    the library's HIP events on every launch (timing mode 2), over extra
    solves run after the timed region."""
    from paper_2206_05543_amd._lib import OPT_TIMING
    out = {}
    for name, P in probs.items():
        mg, d, N = P["mg"], P["d"], P["N"]
        mg.set_option(OPT_TIMING, 2)
        mg.reset_timing()
        for _ in range(solves):
            P["u"].copy_(P["u0"])
            mg.solve(P["b"], P["u"], tol=tol)
        rows = []
        for lev in range(mg.num_levels):
            n = (N >> lev) - 1
            pts = n ** d
            for kind in LEVEL_KINDS:
                ms, cnt = mg.timing(kind, lev)
                if not cnt:
                    continue
                avg_us = ms / cnt * 1e3
                r = {"level": lev, "n": n, "kind": kind, "launches_per_solve": cnt / solves,
                     "avg_us": avg_us}
                bpp = level_bytes_per_pt(kind, d)
                if bpp is not None:
                    gbs = bpp * pts / (avg_us * 1e-6) / 1e9
                    r["GBps"] = gbs
                    r["frac_of_peak"] = gbs / HBM_PEAK_GBS
                rows.append(r)
        mg.set_option(OPT_TIMING, 1)
        out[name] = rows
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-examples", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    # only the gradient workloads' forward/backward timing (for kernel traces)
    ap.add_argument("--adjoint-only", action="store_true")
    ap.add_argument("--workloads", default="poisson2d_n4096,poisson3d_n256")
    ap.add_argument("--tol", type=float, default=1e-10)
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 "
                          "(the multi-GPU decomposition is a design, not code)"}))
        sys.exit(2)
    import torch

    from paper_2206_05543_amd import M7, M9
    from paper_2206_05543_amd._lib import Multigrid
    from paper_2206_05543_amd.workloads import workload

    torch.cuda.init()
    if a.adjoint_only:
        print(json.dumps({"adjoint": adjoint()}), flush=True)
        return
    stream = torch.cuda.current_stream()
    names = [w for w in a.workloads.split(",") if w]
    probs = {}
    for name in names:
        d, N = WORKLOADS[name]
        p = workload(name)
        # timing mode 3: one event pair per solve, around the second launch
        # of the fine level's fused pre-smoother kernel (an event after a
        # large kernel idles the GPU ~5 us, so timing every cycle would cost
        # ~4% of the measured throughput)
        mg = Multigrid(N, d, M9 if d == 2 else M7, max_cycles=100, timing=3)
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
    per = {n: {"cycles": 0, "run": 0, "ms": 0.0} for n in probs}
    for i in range(a.steps):
        res = step()
        for n, st in res.items():
            per[n]["cycles"] += st["cycles"]
            per[n]["run"] += st["cycles_run"]
            per[n]["ms"] += st["elapsed_ms"]
        print(f"[bench] step {i + 1}/{a.steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    total_uc = 0.0
    details = {}
    sweeps = {}  # (workload, kind) -> (avg us, algorithmic GB/s, us per solve, bytes)
    for n, P in probs.items():
        pts = (P["N"] - 1) ** P["d"]
        uc = pts * per[n]["cycles"]
        total_uc += uc
        details[n] = {
            "unknowns": pts,
            "cycles_per_solve": per[n]["cycles"] / a.steps,
            "solve_ms": per[n]["ms"] / a.steps,
            "unknowns_per_s_per_cycle": uc / (per[n]["ms"] * 1e-3),
        }
        for kind in SWEEP_KINDS:
            ms, cnt = P["mg"].timing(kind, 0)
            if not cnt:
                continue
            avg_us = ms / cnt * 1e3
            byt = sweep_bytes_per_pt(kind, P["d"]) * pts
            gbs = byt / (avg_us * 1e-6) / 1e9
            per_solve = launches_per_solve(kind, P["d"], per[n]["run"] / a.steps)
            sweeps[(n, kind)] = (avg_us, gbs, avg_us * per_solve, byt)
            details[n][f"fine_{kind}_us"] = avg_us
            details[n][f"fine_{kind}_GBps"] = gbs
    value = total_uc / wall
    # the dominant kernel: the fine-level sweep with the largest time per solve
    dom = max(sweeps, key=lambda k: sweeps[k][2])
    avg_us, gbs, _, byt = sweeps[dom]
    traffic = hbm_traffic(*dom)

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
                     "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": SWEEP_NAMES[dom[1]] + f" ({dom[0]})",
                     "avg_launch_us": avg_us,
                     "algorithmic_bytes_per_launch": byt,
                     "traffic_GBps": traffic / (avg_us * 1e-6) / 1e9 if traffic else None},
    }
    line["per_level"] = per_level(probs, a.tol)
    for P in probs.values():
        P["mg"].close()
    del probs
    torch.cuda.empty_cache()

    if not a.no_mixed:
        line["mixed_precision"] = mixed(a.tol)
        line["roofline_lowprec"] = lowprec_roofline(line["mixed_precision"])
    if not a.no_adjoint:
        line["adjoint"] = adjoint()
    if not a.no_examples:
        line["paper_examples"] = paper_examples(a.tol)
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


def closed_form_sine_solution(N, modes, weights, device):
    """The exact discrete solution of A_h u = sum_m w_m phi_m on the 3D grid:
    every sine mode phi_m is an eigenvector of A_h with eigenvalue
    4 N^2 sum_a sin^2(k_a pi / (2 N)), so u = sum_m w_m phi_m / lambda_m."""
    import torch
    x = torch.arange(1, N, dtype=torch.float64, device=device) / N
    u = torch.zeros((N - 1,) * 3, dtype=torch.float64, device=device)
    for kk, w in zip(modes, weights):
        lam = 4.0 * N * N * sum(np.sin(int(k) * np.pi / (2 * N)) ** 2 for k in kk)
        sx, sy, sz = (torch.sin(int(k) * np.pi * x) for k in kk)
        u += (float(w) / lam) * sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    return u


def mixed_oracle_anchored(tol, N=64):
    """The same three solves on the same recipe at 3D N=64, where the oracle
    solves to 1e-14: each GPU result's relative error against that solution."""
    import torch

    import oracle as O
    from paper_2206_05543_amd import M7
    from paper_2206_05543_amd._lib import Multigrid
    from paper_2206_05543_amd.workloads import WORKLOADS, poisson_problem

    kw = dict(WORKLOADS["poisson3d_n512_noisy"])
    kw.update(N=N)
    p = poisson_problem(**kw)
    ref, k, _ = O.solve(3, N, np.array(M7), p["u0"], p["b"], tol=1e-14, maxc=200)
    out = {"N": N, "oracle_cycles_to_1e-14": k}
    for prec in ("fp64", "fp32_ir", "fp16_ir"):
        with Multigrid(N, 3, M7, precision=prec) as mg:
            u = torch.from_numpy(p["u0"].copy()).cuda()
            st = mg.solve(torch.from_numpy(p["b"]).cuda(), u, tol=tol)
        got = u.cpu().numpy()
        out[prec] = {"code": st["code"], "cycles": st["cycles"],
                     "rel_error_vs_oracle": float(np.linalg.norm(got - ref) / np.linalg.norm(ref))}
    return out


# the fine-level kernels of the refinement solves, and their algorithmic bytes
# per fine node with storage of sb bytes: the pre-smoother + residual +
# restriction (read u, b; write u1, b_c), the post-smoother with the fused
# correction (read u1, b, e_c; write u), the zero-guess pre-smoother +
# restriction (read b; write e, b_c) and the FP64 refinement step (read u, b
# in FP64 and e; write u in FP64 and the scaled right-hand side; its first
# step, with no correction yet, moves less, so its average overstates the
# bytes slightly)
LOWPREC_KINDS = ("smooth_restrict", "smooth_correct", "zero_smooth_restrict", "ir_step")
LOWPREC_NAMES = {"smooth_restrict": "k_sr3d (pre-smoother + residual + restriction)",
                 "smooth_correct": "k_smooth3d PRO (post-smoother + fused correction)",
                 "zero_smooth_restrict": "k_zrestrict3d (zero-guess pre-smoother + restriction)",
                 "ir_step": "k_ir3d (FP64 refinement step)"}
STORAGE_BYTES = {"fp64": 8, "fp32_ir": 4, "fp16_ir": 2}


def lowprec_bytes_per_pt(kind, sb):
    return {"smooth_restrict": 3 * sb + sb / 8.0, "smooth_correct": 3 * sb + sb / 8.0,
            "zero_smooth_restrict": 2 * sb + sb / 8.0, "ir_step": 24.0 + 2 * sb}[kind]


def fine_kernel_rates(mg, b, u, u0, tol, sb, pts):
    """One more solve with every launch timed (its own dispatch timestamps):
    per fine-level kernel kind, launches per solve, average time and
    algorithmic GB/s."""
    from paper_2206_05543_amd._lib import OPT_TIMING
    mg.set_option(OPT_TIMING, 2)
    mg.reset_timing()
    u.copy_(u0)
    mg.solve(b, u, tol=tol)
    mg.set_option(OPT_TIMING, 0)
    rows = {}
    for kind in LOWPREC_KINDS:
        ms, cnt = mg.timing(kind, 0)
        if not cnt:
            continue
        avg_us = ms / cnt * 1e3
        gbs = lowprec_bytes_per_pt(kind, sb) * pts / (avg_us * 1e-6) / 1e9
        rows[kind] = {"kernel": LOWPREC_NAMES[kind], "launches_per_solve": cnt,
                      "avg_us": avg_us, "bytes_per_pt": lowprec_bytes_per_pt(kind, sb),
                      "GBps": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS}
    return rows


def lowprec_roofline(mixed_out):
    """The FP16-storage solve's storage-precision sweep with the largest time
    per solve, as a roofline entry (algorithmic bytes over its average
    launch time)."""
    rows = mixed_out.get("fp16_ir", {}).get("fine_kernels", {})
    sweeps = {k: v for k, v in rows.items() if k != "ir_step"}
    if not sweeps:
        return None
    kind = max(sweeps, key=lambda k: sweeps[k]["avg_us"] * sweeps[k]["launches_per_solve"])
    r = sweeps[kind]
    return {"bound": "hbm", "achieved": r["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": r["frac_of_peak"], "traffic": hbm_traffic("poisson3d_n512_noisy:fp16_ir", kind),
            "kernel": r["kernel"] + ", FP16 storage, FP32 arithmetic (poisson3d_n512_noisy)",
            "avg_launch_us": r["avg_us"],
            "algorithmic_bytes_per_launch": r["bytes_per_pt"] * 511 ** 3}


def mixed(tol):
    """Time to tol of the 3D N=512 noisy problem: FP64 V-cycles vs FP32 and
    FP16 V-cycles inside FP64 refinement (same GPU, same input).  Each result
    is also measured against a tightly converged FP64 solve, against the
    closed-form discrete solution of the sine part of b, and by the CPU
    oracle's own residual of it."""
    import torch

    import oracle as O
    from paper_2206_05543_amd import M7
    from paper_2206_05543_amd._lib import Multigrid
    from paper_2206_05543_amd.workloads import workload

    print("[bench] mixed precision: generating 3D N=512 input", file=sys.stderr, flush=True)
    p = workload("poisson3d_n512_noisy")
    b_host = p["b"]
    b = torch.from_numpy(b_host).cuda()
    u0 = torch.from_numpy(p["u0"]).cuda()
    out = {"workload": "poisson3d_n512_noisy", "unknowns": 511 ** 3}
    # reference solution: FP64 cycles run until the residual stops falling
    # (a 1e-10 reduction relative to the random initial guess pins the
    # solution only to about 1e-3, so the solves are compared against this)
    mg = Multigrid(512, 3, M7, max_cycles=40)
    ref = u0.clone()
    st = mg.solve(b, ref, tol=1e-14)
    out["reference"] = {"cycles": st["cycles"], "code": st["code"],
                        "rel_residual": st["rk"] / st["r0"],
                        "rel_residual_vs_b": st["rk"] / st["b_norm"]}
    ref_norm = float(ref.norm())
    mg.close()
    # the sine part's exact discrete solution; the noise part of b (1e-3)
    # adds A^-1 noise, which bounds how close any solution can come to it
    ucf = closed_form_sine_solution(512, p["modes"], p["weights"], "cuda")
    ucf_norm = float(ucf.norm())
    out["reference"]["rel_diff_vs_closed_form_sine"] = float((ref - ucf).norm()) / ucf_norm
    b_norm = float(np.linalg.norm(b_host))
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
        uh = u.cpu().numpy()
        r_or = O.norm2(O.residual(3, 512, uh, b_host))
        del uh
        rec = {"time_ms": min(times), "cycles": st["cycles"], "code": st["code"],
               "rel_residual": rk / st["r0"],
               "oracle_rel_residual": r_or / st["r0"],
               "oracle_residual_vs_b": r_or / b_norm,
               "rel_error_vs_reference": float((u - ref).norm()) / ref_norm,
               "rel_error_vs_closed_form_sine": float((u - ucf).norm()) / ucf_norm}
        rec["fine_kernels"] = fine_kernel_rates(mg, b, u, u0, tol, STORAGE_BYTES[prec], 511 ** 3)
        out[prec] = rec
        mg.close()
        print(f"[bench] mixed {prec}: {rec}", file=sys.stderr, flush=True)
    out["speedup_fp32_ir"] = out["fp64"]["time_ms"] / out["fp32_ir"]["time_ms"]
    out["speedup_fp16_ir"] = out["fp64"]["time_ms"] / out["fp16_ir"]["time_ms"]
    del ucf, ref, u, b, u0
    torch.cuda.empty_cache()
    out["oracle_anchored"] = mixed_oracle_anchored(tol)
    return out


# FP64 bytes per fine point that the adjoint cycle's fine-level kernels read
# and write (mg_vcycle_adjoint): the forward recomputation's pre-smoother +
# restriction with the residual r1 kept (read u, b; write t, r1, b_c) and
# post-smoother with the fused correction and r3 kept (read t, b, e_c; write
# u_out, r3); the reverse pass's two smoothing sweeps (read ubar, r, bbar;
# write ubar', bbar), the restriction of ubar (read a fine field, write a
# coarse one) and the update with the interpolated bbar_c (read ubar, bbar,
# bbar_c; write ubar', bbar); the fused pre-smoother reads an FP32
# checkpoint as stored (4 instead of 8 bytes of u).  c is one coarse value per
# 2^d fine points.
def adjoint_bytes_per_pt(d, ckpt="fp64"):
    c = 8.0 / 2 ** d
    forward = (32 + c) + (32 + c)
    reverse = 40 + (8 + c) + (32 + c) + 40
    return forward + reverse - (4.0 if ckpt == "fp32" else 0.0)


ADJOINT_CASES = (("errors2d_n1024_b16", 2, 1024, 16, 3, "fp64"),
                 ("errors3d_n256_b4", 3, 256, 4, 2, "fp32"))


def adjoint(reps=3):
    """Forward + backward of the k-cycle loss L = sum ||V^K(e0, 0; c)||^2
    through the autograd wrapper on the two gradient workloads: 2D N=1024,
    batch 16, K = 3, FP64 checkpoints; 3D N=256, batch 4, K = 2, FP32
    checkpoints.  Best of `reps` after a warm-up, timed with events on the
    current stream."""
    import torch

    from paper_2206_05543_amd import M7, M9
    from paper_2206_05543_amd._lib import Multigrid
    from paper_2206_05543_amd.autograd import kcycles
    from paper_2206_05543_amd.workloads import workload

    out = {}
    for name, d, N, batch, K, ck in ADJOINT_CASES:
        w = workload(name)
        e0 = torch.from_numpy(w["e0"]).cuda()
        b = torch.zeros_like(e0)
        c0 = M9 if d == 2 else M7
        ckd = torch.float64 if ck == "fp64" else torch.float32
        mg = Multigrid(N, d, c0, batch=batch)
        best_f, best_b = float("inf"), float("inf")
        for it in range(reps + 1):
            cp = torch.tensor(c0, dtype=torch.float32, requires_grad=True)
            torch.cuda.synchronize()
            e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e1.record()
            u = kcycles(mg, cp, b, e0, K, ckd)
            L = (u * u).sum()
            e2.record()
            L.backward()
            e3.record()
            torch.cuda.synchronize()
            if it > 0:
                best_f = min(best_f, e1.elapsed_time(e2))
                best_b = min(best_b, e2.elapsed_time(e3))
        mg.close()
        pts = (N - 1) ** d * batch
        byt = adjoint_bytes_per_pt(d, ck) * pts * K
        out[name] = {"d": d, "N": N, "batch": batch, "cycles": K, "checkpoints": ck,
                     "forward_ms": best_f, "backward_ms": best_b,
                     "backward_over_forward": best_b / best_f,
                     "fine_unknowns_per_s_fwd_bwd": pts * K / ((best_f + best_b) * 1e-3),
                     "adjoint_fine_bytes_per_pt_per_cycle": adjoint_bytes_per_pt(d, ck),
                     "adjoint_fine_GBps": byt / (best_b * 1e-3) / 1e9,
                     "adjoint_frac_of_peak": byt / (best_b * 1e-3) / 1e9 / HBM_PEAK_GBS}
        print(f"[bench] adjoint {name}: {out[name]}", file=sys.stderr, flush=True)
        del e0, b, u, L
        torch.cuda.empty_cache()
    return out


EXAMPLE_SIZES = ((1, 4096), (2, 4096), (3, 512))


def paper_examples(tol):
    """Section 4's smoother and cycle comparison on its analytic problems:
    Examples 1 and 2 at 2D N=4096, Example 3 at 3D N=512 (the paper's
    134-million-unknown case), every smoother under V(1,1) and W(1,0) from a
    U(0,1) initial guess to a tol residual reduction.  Per case: cycles, the
    observed rate (||r_k||/||r_0||)^(1/k), GPU time to solution (best of two
    after a warm-up) and the maximum error against the exact solution."""
    import torch

    from paper_2206_05543_amd import SMOOTHERS
    from paper_2206_05543_amd._lib import Multigrid
    from paper_2206_05543_amd.workloads import example_problem

    out = {}
    for ex, N in EXAMPLE_SIZES:
        print(f"[bench] example {ex}: generating N={N} input", file=sys.stderr, flush=True)
        p = example_problem(ex, N)
        d = p["d"]
        b = torch.from_numpy(p["b"]).cuda()
        u0 = torch.from_numpy(p["u0"]).cuda()
        uex = torch.from_numpy(p["u"]).cuda()
        del p
        rec = {"d": d, "N": N, "unknowns": (N - 1) ** d}
        for name, c in SMOOTHERS[d].items():
            for cyc, key in (("V11", "V"), ("W10", "W")):
                mg = Multigrid(N, d, c, cycle=cyc, max_cycles=200)
                u = u0.clone()
                mg.solve(b, u, tol=tol)  # warm-up
                times = []
                for _ in range(2):
                    u.copy_(u0)
                    st = mg.solve(b, u, tol=tol)
                    times.append(st["elapsed_ms"])
                mg.close()
                k = st["cycles"]
                r = {"cycles": k, "rho_hat": (st["rk"] / st["r0"]) ** (1.0 / k) if k else None,
                     "time_ms": min(times), "code": st["code"],
                     "max_error": float((u - uex).abs().max())}
                rec[f"{name}_{key}"] = r
                print(f"[bench] example {ex} {name} {key}: {r}", file=sys.stderr, flush=True)
        out[f"example{ex}"] = rec
        del b, u0, uex, u
        torch.cuda.empty_cache()
    out["paper_context"] = ("Example 3 at N=512 with M7 and V-cycles: about 200 s in serial "
                            "MATLAB on an i9-10900X (Section 4)")
    return out


CPU_CYCLES = 5


def host_cpu():
    """The host's CPU model (from /proc/cpuinfo), logical CPUs and the CPUs
    this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0))}


def cpu_baseline():
    """The CPU oracle (plain FP64 loops) on a bounded sample: CPU_CYCLES
    consecutive V(1,1) cycles of each workload of the step, once with the
    OpenMP build on every thread OMP_NUM_THREADS allows (the value) and once
    single-threaded (the checker build; bit-identical results)."""
    import oracle as O
    from paper_2206_05543_amd import M7, M9
    from paper_2206_05543_amd.workloads import workload

    O.lib()
    O.lib_omp()
    legs = {}
    for parallel in (True, False):
        total_uc, total_s = 0.0, 0.0
        for name, (d, N) in WORKLOADS.items():
            p = workload(name)
            c = np.array(M9 if d == 2 else M7)
            t = time.perf_counter()
            u = p["u0"]
            for _ in range(CPU_CYCLES):
                u = O.vcycle(d, N, c, u, p["b"], parallel=parallel)
            total_s += time.perf_counter() - t
            total_uc += CPU_CYCLES * (N - 1) ** d
            print(f"[bench] cpu oracle {name} ({O.num_threads(parallel)} threads): "
                  f"{time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
        legs[parallel] = (total_uc / total_s, total_s, O.num_threads(parallel))
    rate, secs, threads = legs[True]
    rate1, secs1, _ = legs[False]
    return {"value": rate, "unit": "unknowns/s", "cores": threads, "kind": "oracle",
            "sample": f"{CPU_CYCLES} consecutive V(1,1) cycles of 2D N=4096 and {CPU_CYCLES} "
                      f"of 3D N=256 from the benchmark's initial guesses ({secs:.1f} s on "
                      f"{threads} threads; {secs1:.1f} s single-threaded)",
            "single_thread": {"value": rate1, "cores": 1},
            "host": host_cpu()}


if __name__ == "__main__":
    main()
