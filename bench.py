"""Benchmark: CG voxel-iterations/s and Newton step time at 256^3, FP32-split and FP64.

Workload: 256^3 periodic Voronoi polycrystal (512 grains, seeded), rotated-cubic Saint
Venant-Kirchhoff grains (C11, C12, C44) = (1.7, 1.2, 0.75), full stress control with P11
cycled 0 -> +0.02 -> 0 -> -0.02 -> 0 over 40 increments (paper tolerances: Newton 1e-6,
CG 1e-8).  A step is one load increment: the shift of the prescribed means, then Newton
(constitutive update, FP64 residual, CG on G*(K:dF), Newton update) to convergence.

value = N * (CG iterations in the timed increments) / (wall time of those increments), the
whole-job throughput with every input resident in HBM.  Prints ONE JSON line on stdout;
progress goes to stderr.  The default run (2 warm-up + 38 timed increments) covers the whole
40-increment cycle, both stress-free crossings included; more increments than that cycle the
periodic history again.  An increment that fails is recorded in the JSON (status, message)
and stays in the timed region.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CG operator voxel-iters/s + Newton step time at 256^3, FP64 vs FP32-split"
PEAK_HBM_GBS = 8000.0
CG_FORCING = 1e-5
# the timed region brackets every PROFILE_EVERY-th launch of the dominant kernel with HIP
# events (each bracketed launch leaves the GPU idle for a few microseconds); a uniform sample
PROFILE_EVERY = 4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def op_bytes(name, N, Nh, w, svk=True, update_p=True):
    """Algorithmic HBM bytes of one launch of an operator pass (w = bytes of a real)."""
    spec = 9 * Nh * 2 * w  # the 9-component half spectrum
    field = 9 * N * w
    if "yfwd" in name or "yinv" in name or "xproj" in name:
        return 2 * spec
    if "zfwd" in name:
        state = (9 if svk else 12) * N * w + (2 * N if svk else 0)  # SVK: H = F - I (no scale plane), phase
        # CG step: r, p, x in; x, p out (x += alpha p of the previous step, p = r + beta p)
        return field * (5 if update_p else 1) + state + spec
    if "zinv" in name:  # CG step: spectrum, r in; r out (r -= alpha Ap)
        return spec + 2 * field
    return None


def csrc_hash():
    """Hash of the kernel sources: measured counters only count for the code they measured."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1901_06531_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, shape):
    """HBM bytes per launch from the committed counter runs (256^3 polycrystal), or None for
    another grid or if the kernels changed since."""
    if tuple(shape) != (256, 256, 256):
        return None
    path = os.path.join(ROOT, "profiles", "polycrystal256_hbm_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except OSError:
        return None
    if d.get("csrc_sha256_16") != csrc_hash() or kernel not in d["kernels"]:
        return None
    k = d["kernels"][kernel]
    return k["read_bytes"] + k["write_bytes"]


def steady_launches(samples):
    """The launches of a kernel record within 10% of its median launch: the steady CG
    iterations.  Left out (and counted): launches queued after a solve had stopped, which exit
    at once, and the first iteration of each solve, which moves fewer bytes."""
    ms = np.asarray(samples, dtype=np.float64)
    med = float(np.median(ms))
    keep = ms[(ms >= 0.9 * med) & (ms <= 1.1 * med)]
    return keep, int(np.sum(ms < 0.2 * med)), int(len(ms) - len(keep) - np.sum(ms < 0.2 * med))


def cycled_history(target, total):
    """The periodic load history repeated until it holds `total` increments."""
    reps = -(-total // len(target))
    return np.tile(target, (reps, 1))[:max(total, len(target))]


def run_gpu(w, precision, steps, warmup, profile):
    from paper_1901_06531_amd import ghom

    s = ghom.Solver(w["shape"], precision=precision)
    s.setup(w)
    s.set_history(cycled_history(w["target"], steps + warmup))
    gauge = s.control()[1]
    xproj = {"f64": s.get_option(ghom.OPT_XPROJ_F64), "f32": s.get_option(ghom.OPT_XPROJ_F32)}
    schedule = s.schedule()
    # both precisions stop CG at max(1e-8, 1e-5 |b|): the float32 CG needs the relative
    # floor, and the float64 run uses the same rule so that the two are compared fairly
    s.set_tolerances(w["newton_tol"], w["cg_tol"], CG_FORCING)
    # warm-up: every launch timed, to find the operator pass with the largest share; the
    # timed region then brackets only every PROFILE_EVERY-th launch of that kernel with events
    # (each timed launch costs a few microseconds)
    if profile and warmup:
        s.profile_reset()
        s.set_profiling(True)
    failures = []

    def one(k, what):
        info = s.step(check=False)
        if info["status"] != 0:
            failures.append({"increment": k, "phase": what, "status": info["status"], "error": info["error"],
                             "newton_iters": info["newton_iters"], "cg_iters": info["cg_iters_total"]})
            log("  %s increment %d FAILED: %s" % (what, k, info["error"]))
            if info["status"] != ghom.STATUS_CODE["ENOTCONVERGED"]:
                # the increment was not advanced (ESINGULAR, EDOMAIN): retry it in halves
                try:
                    info2 = s.step_adaptive(max_cuts=8, grow_below=2)
                except ghom.GhomError as ex:
                    failures[-1]["recovered_by"] = "nothing: step_adaptive failed too (%s)" % ex
                    info["stuck"] = True
                    return info
                failures[-1]["recovered_by"] = "step_adaptive: %d substeps, %d cuts" % (info2["substeps"],
                                                                                       info2["cuts"])
                for key in ("newton_iters", "cg_iters_total", "t_cg_ms", "t_total_ms", "cg_stalls"):
                    info[key] += info2[key]
        log("  %s increment %d: newton %d cg %d stalls %d  %.1f ms" % (
            what, k, info["newton_iters"], info["cg_iters_total"], info["cg_stalls"], info["t_total_ms"]))
        return info

    for i in range(warmup):
        if one(i + 1, "warmup").get("stuck"):
            raise RuntimeError("warm-up increment %d could not be advanced: %s" % (i + 1, failures[-1]))
    warm_prof = {}
    warm_steady = {}
    if profile and warmup:
        warm_prof = s.profile()
        op = {k: v for k, v in warm_prof.items() if k.startswith("op_")}
        for k in op:
            keep, _, _ = steady_launches(s.profile_samples(k))
            warm_steady[k] = float(keep.mean())
        s.set_profiling_filter(max(op, key=lambda k: op[k][1]) if op else None)
        s.set_option(ghom.OPT_PROFILE_EVERY, PROFILE_EVERY)
    import torch
    torch.cuda.synchronize()
    if profile:
        s.profile_reset()
        s.set_profiling(True)
    infos = []
    t0 = time.perf_counter()
    for i in range(steps):
        infos.append(one(warmup + i + 1, "timed"))
        if infos[-1].get("stuck"):
            break  # the same increment would fail again; the partial region is reported
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = s.profile() if profile else {}
    samples = {k: s.profile_samples(k) for k in prof} if profile else {}
    F, P = s.averages()
    s.close()
    if warm_prof:
        log("kernel times (warm-up, every launch timed, steady launches): " + ", ".join(
            "%s %.3f ms" % (k, v) for k, v in sorted(warm_steady.items())))
    cg = sum(i["cg_iters_total"] for i in infos)
    newton = sum(i["newton_iters"] for i in infos)
    N = int(np.prod(w["shape"]))
    return {
        "voxel_iters_per_s": N * cg / wall,
        "ms_per_increment": 1e3 * wall / len(infos),
        "increments_timed": len(infos),
        "newton_step_ms": 1e3 * wall / max(newton, 1),
        "cg_ms_per_iter": sum(i["t_cg_ms"] for i in infos) / max(cg, 1),
        "cg_iters": cg,
        "newton_iters": newton,
        "cg_stalls": sum(i["cg_stalls"] for i in infos),
        "cg_breakdowns": sum(i["cg_breakdowns"] for i in infos),
        "newton_per_increment": [i["newton_iters"] for i in infos],
        "cg_per_increment": [i["cg_iters_total"] for i in infos],
        "failures": failures,
        "rotation_gauge_axis": gauge,
        "F11": float(F[0]),
        "P11": float(P[0]),
        "xproj_variant": xproj,
        "schedule": schedule,
        "pass_ms_steady": {k: round(v, 4) for k, v in sorted(warm_steady.items())},
    }, (prof, samples)


def run_batch(steps, warmup, sample_per_size=2):
    """The batched workload: 64 RVEs (16 each of 32^3, 48^3, 64^3, 96^3) x 6 load cases = 384
    problems advanced together (FP32-split), one increment per step; beside it a sample of the
    same problems run one at a time through single-problem contexts."""
    from paper_1901_06531_amd import ghom, synth

    t0 = time.perf_counter()
    ws = synth.workload_batch()
    log("batch workload: %d problems, %.1f M voxels, built in %.1f s" % (
        len(ws), sum(int(np.prod(w["shape"])) for w in ws) / 1e6, time.perf_counter() - t0))
    import torch
    t0 = time.perf_counter()
    b = ghom.Batch(ws, precision=ghom.FP32_SPLIT)
    b.set_tolerances(1e-6, 1e-8, CG_FORCING)
    log("batch created in %.1f s (%d launch groups)" % (time.perf_counter() - t0, b.num_classes()))
    schedules = b.schedules()
    for sch in schedules:
        log("  schedule: " + sch)
    for i in range(warmup):
        t0 = time.perf_counter()
        b.step()
        log("  batch warmup increment %d: %.1f ms" % (i + 1, 1e3 * (time.perf_counter() - t0)))
    torch.cuda.synchronize()
    vox_its = 0
    t0 = time.perf_counter()
    for i in range(steps):
        infos = b.step()
        vox_its += sum(int(np.prod(w["shape"])) * inf["cg_iters_total"] for w, inf in zip(ws, infos))
        log("  batch timed increment %d: max newton %d, CG iterations %d..%d" % (
            warmup + i + 1, max(x["newton_iters"] for x in infos), min(x["cg_iters_total"] for x in infos),
            max(x["cg_iters_total"] for x in infos)))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.close()
    # the same kind of problems one at a time (sample: the first load case of the first
    # `sample_per_size` RVEs of every size), same precision and tolerances
    seen = {}
    sample = []
    for w in ws:
        n = w["shape"][0]
        if w["name"].endswith("uniaxial_x") and seen.get(n, 0) < sample_per_size:
            seen[n] = seen.get(n, 0) + 1
            sample.append(w)
    s_vox = 0
    s_wall = 0.0
    for w in sample:
        with ghom.Solver(w["shape"], precision=ghom.FP32_SPLIT) as s:
            s.setup(w)
            s.set_tolerances(1e-6, 1e-8, CG_FORCING)
            for _ in range(warmup):
                s.step()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(steps):
                inf = s.step()
                s_vox += int(np.prod(w["shape"])) * inf["cg_iters_total"]
            torch.cuda.synchronize()
            s_wall += time.perf_counter() - t1
    return {"problems": len(ws), "launch_groups": len(schedules), "schedules": schedules, "increments_timed": steps,
            "voxel_iters_per_s": round(vox_its / wall, 1), "ms_per_increment": round(1e3 * wall / steps, 1),
            "one_at_a_time_voxel_iters_per_s": round(s_vox / s_wall, 1),
            "one_at_a_time_sample": "%d problems (%d per grid size), same increments" % (len(sample), sample_per_size)}


def _oracle_cg_rate(w, seconds):
    """Voxel-iterations/s of the oracle's CG iterations (first Newton solve of increment 1) on
    workload w, over about `seconds` of CPU work (at least 3 iterations)."""
    from oracle import ghom_oracle as go

    o = go.Oracle(w["shape"])
    o.set_material_svk(w["phase"], w["C"])
    o.set_control(w["mask"])
    o.set_history(w["target"])
    o.set_tolerances(w["newton_tol"], w["cg_tol"], 0.0, 50, 1)
    Pbar = np.where(w["mask"] > 0, w["target"][0], 0.0)
    P = o.stress()
    b = o.residual(P, Pbar)
    t0 = time.perf_counter()
    its = 0
    while True:
        try:
            o.conjugate_gradient(b)
        except go.NotConvergedError:
            pass
        its += 1
        if (time.perf_counter() - t0 > seconds and its >= 3) or its >= 200:
            break
    dt = time.perf_counter() - t0
    N = int(np.prod(w["shape"]))
    return N * its / dt, its, dt


def _oracle_newton_step(w):
    """Wall time of one oracle Newton iteration at the start of increment 1 (constitutive
    update, FP64 residual, CG solve at the bench's forcing, update) on workload w, with its CG
    count."""
    from oracle import ghom_oracle as go

    o = go.Oracle(w["shape"])
    o.set_material_svk(w["phase"], w["C"])
    o.set_control(w["mask"])
    o.set_history(w["target"])
    o.set_tolerances(w["newton_tol"], w["cg_tol"], CG_FORCING, 1, 5000)
    Pbar = np.where(o.mask > 0, w["target"][0], 0.0)
    t0 = time.perf_counter()
    b = o.residual(o.stress(), Pbar)
    dF, its = o.conjugate_gradient(b)
    o.F = o.F + dF
    go.Oracle.newton_criterion(dF, o.F.reshape(9, -1).mean(axis=1))
    return time.perf_counter() - t0, its


def _oracle_operator_s(w):
    """Wall time of one oracle operator application A(v) = G*(K : v) on workload w at F = I
    (v seeded random): the work of one CG iteration at the benchmark's own grid."""
    from oracle import ghom_oracle as go

    o = go.Oracle(w["shape"])
    o.set_material_svk(w["phase"], w["C"])
    o.set_control(w["mask"])
    F = np.zeros((9,) + tuple(w["shape"]))
    F[[0, 4, 8]] = 1.0
    v = np.random.default_rng(0).standard_normal((9,) + tuple(w["shape"]))
    t0 = time.perf_counter()
    o.apply_operator(v, F)
    return time.perf_counter() - t0


def cpu_baseline(grid, seconds=15.0):
    """The FP64 oracle timed on this host (its transforms on every core): CG iterations at
    the 128^3 and 16^3 instances of the benchmark's generator, one Newton step at 64^3, and
    one operator application at the benchmark's grid."""
    from oracle import ghom_oracle as go
    from paper_1901_06531_amd import synth

    big = max(16, grid // 2)
    rate, its, dt = _oracle_cg_rate(synth.workload_polycrystal(n=big), seconds)
    rate16, its16, dt16 = _oracle_cg_rate(synth.workload_polycrystal(n=16, ngrains=64), 1.0)
    nt, nits = _oracle_newton_step(synth.workload_polycrystal(n=64))
    op_s = _oracle_operator_s(synth.workload_polycrystal(n=grid))
    return {"value": rate, "unit": "voxel-iters/s", "cores": go.WORKERS, "kind": "oracle",
            "sample": "%d CG iteration(s) of the oracle's first Newton solve on the %d^3 instance of the "
                      "benchmark's polycrystal generator (%.1f s)" % (its, big, dt),
            "cg_voxel_iters_per_s_16": rate16,
            "newton_step_s_64": round(nt, 3),
            "operator_s_%d" % grid: round(op_s, 3),
            "newton_step_sample": "one oracle Newton iteration (constitutive update, FP64 residual, CG solve of "
                                  "%d iterations at forcing 1e-5, update) at the start of increment 1 on the 64^3 "
                                  "instance" % nits}


def run_paper_example(n, nsteps, precision_name):
    """The three control types of the particle example (Sec. 3.1) on one geometry: (1)
    mixed (F11 ramp, transverse stresses zero), (2) full stress control ramping to case
    (1)'s end stress, (3) full strain control ramping to case (1)'s end deformation
    gradient.  Per increment: Newton and CG iterations and time (the paper's Fig. 3a and
    3c); at the end: how far the three end states are apart (rotation invariants)."""
    from paper_1901_06531_amd import ghom, synth

    prec = ghom.FP64 if precision_name == "fp64" else ghom.FP32_SPLIT
    w1 = synth.workload_paper_particles(n=n, nsteps=nsteps)

    def run(w):
        with ghom.Solver(w["shape"], precision=prec) as s:
            s.setup(w)
            s.set_tolerances(w["newton_tol"], w["cg_tol"], CG_FORCING if prec == ghom.FP32_SPLIT else 0.0)
            recs = []
            for k in range(len(w["target"])):
                info = s.step()
                F, P = s.averages()
                recs.append((info, F, P))
            Ff = s.field(ghom.FIELD_F)
        return recs, Ff

    cases = {}
    log("case (1): mixed control")
    r1, F1 = run(w1)
    F_end, P_end = r1[-1][1], r1[-1][2]
    w2 = dict(w1, mask=synth.mask_full_stress(), target=synth.history_stress_ramp(P_end, nsteps))
    log("case (2): full stress control")
    r2, F2 = run(w2)
    w3 = dict(w1, mask=synth.mask_full_strain(), target=synth.history_strain_ramp(F_end, nsteps))
    log("case (3): full strain control")
    r3, F3 = run(w3)

    def cbar(F9):
        F = np.asarray(F9).reshape(3, 3)
        return F.T @ F

    def ftf(Ff):
        G = Ff.reshape(3, 3, -1)
        return np.einsum("kin,kjn->ijn", G, G)

    C1 = ftf(F1)
    for name, recs, Ff in (("1_mixed", r1, F1), ("2_stress", r2, F2), ("3_strain", r3, F3)):
        cases[name] = {
            "cg_per_increment": [r[0]["cg_iters_total"] for r in recs],
            "newton_per_increment": [r[0]["newton_iters"] for r in recs],
            "ms_per_increment": [round(r[0]["t_total_ms"], 2) for r in recs],
            "total_cg": int(sum(r[0]["cg_iters_total"] for r in recs)),
            "total_ms": round(sum(r[0]["t_total_ms"] for r in recs), 1),
            "P_mid": [round(v, 8) for v in recs[len(recs) // 2 - 1][2]],
            "end_P_diff_vs_1": float(np.max(np.abs(recs[-1][2] - P_end))),
            "end_Cbar_diff_vs_1": float(np.max(np.abs(cbar(recs[-1][1]) - cbar(F_end)))),
            "end_voxel_FtF_diff_vs_1": float(np.max(np.abs(ftf(Ff) - C1))),
        }
    t3 = cases["3_strain"]["total_ms"]
    for c in cases.values():
        c["time_vs_case3"] = round(c["total_ms"] / t3, 3)
    return {"paper_example": {"grid": [n, n, n], "increments": nsteps, "precision": precision_name,
                              "newton_tol": w1["newton_tol"], "cg_tol": w1["cg_tol"], "cases": cases}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=38)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 384-problem workload")
    ap.add_argument("--paper-example", action="store_true",
                    help="only run the three control types of the particle example (Sec. 3.1) and print their "
                         "iteration counts, times and end-state differences")
    ap.add_argument("--paper-example-precision", default="fp64", choices=["fp64", "split"])
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (5 times): the reference for HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.paper_example:
        print(json.dumps(run_paper_example(64, 100, args.paper_example_precision)), flush=True)
        return

    if args.copy_calibration:
        import torch
        n = 1 << 28  # 2^28 float32 = 1 GiB read + 1 GiB written per copy
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 5
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "ms": 1e3 * dt,
                          "GBps_read_plus_write": 8 * n / dt / 1e9}), flush=True)
        return

    from paper_1901_06531_amd import ghom, synth

    t0 = time.perf_counter()
    w = synth.workload_polycrystal(n=args.grid)
    N = int(np.prod(w["shape"]))
    log("workload %s built in %.1f s" % (w["name"], time.perf_counter() - t0))

    log("FP32-split run")
    split, (prof, samples) = run_gpu(w, ghom.FP32_SPLIT, args.steps, args.warmup, profile=True)
    fp64 = None
    if not args.no_fp64:
        log("FP64 run")
        fp64, _ = run_gpu(w, ghom.FP64, args.steps, args.warmup, profile=False)

    # roofline of the dominant operator kernel, from the HIP-event timings of the timed region
    nzh = w["shape"][2] // 2
    Nh = w["shape"][0] * w["shape"][1] * nzh
    op = {k: v for k, v in prof.items() if k.startswith("op_")}
    roof = None
    if op:
        name = max(op, key=lambda k: op[k][1])
        launches, ms = op[name]
        wbytes = 4 if name.endswith("f32") else 8
        per_launch = op_bytes(name, N, Nh, wbytes)
        keep, noop, other = steady_launches(samples[name])
        avg_ms = float(keep.mean())
        achieved = per_launch / (avg_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(name, w["shape"]),
                "kernel": name,
                "avg_ms": round(avg_ms, 4), "bytes_per_launch": per_launch,
                "launches": {"sampled_every": PROFILE_EVERY, "steady": int(len(keep)), "noop": noop,
                             "other": other, "all_avg_ms": round(ms / launches, 4)}}
        log("kernel times (timed region): " + ", ".join("%s %.3f ms x%d" % (k, v[1] / v[0], v[0])
                                                        for k, v in sorted(op.items())))

    batch = None
    if not args.no_batch:
        log("batched workload")
        batch = run_batch(1, 1)

    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        # the oracle takes about a minute per CG iteration at 256^3: time it on the
        # 128^3 instance of the same generator (same grain count, seeds and loading)
        cpu = cpu_baseline(args.grid)

    out = {
        "metric": METRIC,
        "value": round(split["voxel_iters_per_s"], 1),
        "unit": "voxel-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(split["ms_per_increment"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64-split",
        "data": "synthetic",
        "config": {"workload": w["name"], "grid": list(w["shape"]), "grains": 512, "material": "svk-cubic",
                   "control": "full stress, P11 triangle +-0.02 over 40 increments (cycled)",
                   "increments": [args.warmup + 1, args.warmup + args.steps],
                   "step": "one load increment", "precision": "fp32-split",
                   "newton_tol": w["newton_tol"], "cg_tol": w["cg_tol"], "cg_forcing": CG_FORCING},
        "newton_step_ms": round(split["newton_step_ms"], 3),
        "cg_ms_per_iter": round(split["cg_ms_per_iter"], 4),
        # the rate inside the CG loops alone (operator, update and reductions; no Newton level)
        "cg_loop_voxel_iters_per_s": round(N / (split["cg_ms_per_iter"] * 1e-3), 1),
        "cg_iters": split["cg_iters"],
        "newton_iters": split["newton_iters"],
        "newton_per_increment": split["newton_per_increment"],
        "cg_per_increment": split["cg_per_increment"],
        "cg_stalls": split["cg_stalls"],
        "cg_breakdowns": split["cg_breakdowns"],
        "failures": split["failures"],
        "rotation_gauge_axis": split["rotation_gauge_axis"],
        "xproj_variant": split["xproj_variant"],
        "schedule": split["schedule"],
        "pass_ms_steady": split["pass_ms_steady"],
        "fp64": None if fp64 is None else {
            "value": round(fp64["voxel_iters_per_s"], 1), "ms_per_step": round(fp64["ms_per_increment"], 3),
            "newton_step_ms": round(fp64["newton_step_ms"], 3), "cg_ms_per_iter": round(fp64["cg_ms_per_iter"], 4),
            "cg_loop_voxel_iters_per_s": round(N / (fp64["cg_ms_per_iter"] * 1e-3), 1),
            "cg_iters": fp64["cg_iters"], "newton_iters": fp64["newton_iters"],
            "cg_stalls": fp64["cg_stalls"], "failures": fp64["failures"],
            "split_vs_fp64_F11_diff": abs(fp64["F11"] - split["F11"])},
        "batch": batch,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
