"""Benchmark: DDA solves per second on one MI355X.

Workload (default): the 64^3 filled cube, 262,144 dipoles, m = 1.5 + 0.02i,
size parameter x = 10, one plane wave along +z polarised along x, LDR
polarisabilities, FFT grid 128^3.  One step = the whole hot path for this
target: interaction spectrum (tensor first column + pruned DFTs), the
QMR_sym solve to a true FP64 residual of 1e-6 in mixed precision (FP32 FFT
passes and Krylov vectors, FP64 residuals, refinement and inner products),
and the cross sections.  Inputs are resident in HBM before timing starts.

Besides the headline, the line carries (outside the timed region):
  roofline            the whole FP32 matrix-vector product of the headline
                      workload against the 3-pass byte model B3 (HIP events
                      around every product), with the dominant z kernel's own
                      fraction as a separate key;
  batched_orientations  the 96^3 ellipsoid with 128 right-hand sides in one
                      mixed solve: solves/s, the FP64 single-RHS path on the
                      same GPU, and the largest relative error of C_ext, C_abs
                      and C_sca over all 128 against an FP64 solve to 1e-12;
  matvec_rates        FP32 and FP64 products of the 128^3 sphere (one RHS) and
                      of the 128-RHS ellipsoid batch against B3 (working sets
                      larger than the 256 MB Infinity Cache).

Prints ONE JSON line (see the keys below).  ``--gpus N`` with N > 1 exits:
the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DDA solves/sec at 1e-6 residual (mixed vs FP64); matvec HBM GB/s vs peak"
HBM_PEAK_GBPS = 8000.0


def pass_bytes(K, J, P, Kpp, Jpp, Kh, Jh, Ph, nd, b, jacobi):
    """Algorithmic HBM bytes of one launch of each matrix-vector pass, one
    right-hand side, b bytes per complex value."""
    grid_y = 3 * K * Jpp * P      # y-transformed array, complex values
    grid_xy = 3 * Kpp * Jpp * P   # x- and y-transformed array
    spec = 6 * Kh * Jh * Ph
    idx = 8 * ((K + 31) // 32) * J * P  # bit-fielded occupancy: (bits, base) per 32 sites of a row
    diag = nd * b * (1 if jacobi else 1)
    return {
        "y_forward": 3 * nd * b + idx + grid_y * b + (diag if jacobi else 0),
        "x_forward": (grid_y + grid_xy) * b,
        "z_product": (2 * grid_xy + spec) * b,
        "x_inverse": (grid_xy + grid_y) * b,
        "y_inverse": grid_y * b + idx + 3 * nd * b + diag + 3 * nd * b,
        # fused xy-plane passes: the y-transformed array never reaches HBM
        "xy_forward": 3 * nd * b + idx + (diag if jacobi else 0) + grid_xy * b,
        "xy_inverse": grid_xy * b + idx + 3 * nd * b + diag + 3 * nd * b,
    }


def kernel_source_sha1():
    import hashlib
    h = hashlib.sha1()
    for f in ["fft_fast.hpp", "fft_core.hpp", "kernels_fft.hpp", "fft_reg.hpp"]:
        with open(os.path.join(ROOT, "paper_0908_0863_amd", "csrc", f), "rb") as fh:
            h.update(hashlib.sha1(fh.read()).hexdigest().encode())
    return h.hexdigest()[:16]


def measured_traffic(pass_name, workload, schedule):
    """HBM bytes per launch of an FP32 pass ("matvec": the whole product) from
    the committed rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE,
    copy-calibrated), or None when the summary is missing, was taken with
    another schedule, or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_matvec_fp32_{workload}.txt")
    if not os.path.exists(path):
        return None
    key = "pass matvec_total" if pass_name == "matvec" else f"pass {pass_name}"
    sha = sched = None
    for line in open(path):
        if line.startswith("source_sha1:"):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith("schedule:"):
            sched = int(line.split(":", 1)[1])
        elif line.startswith(key + " ") and sha == kernel_source_sha1() and sched == schedule:
            return int(line.split()[-1])
    return None


def tuned_schedule(tune_file, K, J, P, prec):
    """The schedule the autotuner recorded for a single-RHS product of this
    lattice in this precision (the low 4 bits of the plan), or None."""
    if not os.path.exists(tune_file):
        return None
    for ln in open(tune_file):
        if ln.startswith(f"mv {K}x{J}x{P} ") and f" nrhs 1 {prec} = " in ln:
            return int(ln.rsplit("=", 1)[1]) & 15
    return None


def b3_bytes(K, J, P, Jpp, Kh, Jh, Ph, nd, b, nrhs=1):
    """Minimal 3-pass data motion of one matrix-vector product (y pass, fused
    xz-plane pass, inverse y pass): b [9 N_d + 12 K J'' P + 6 K_h J_h P_h] per
    right-hand side, the spectrum read once for all right-hand sides."""
    return b * (nrhs * (9 * nd + 12 * K * Jpp * P) + 6 * Kh * Jh * Ph)


def matvec_rates(lib, name, nrhs=1, reps=10, precisions=("fp32", "fp64")):
    """Whole matrix-vector products of a workload (Jacobi form, LDR S of its
    first orientations, tuned schedule), each bracketed by HIP events on the
    launch stream: average time, and B3 bytes / time against the HBM peak."""
    import numpy as np
    import torch

    from paper_0908_0863_amd import dda, inputs
    w = inputs.workload(name)
    t = dda.Target(lib, w["K"], w["J"], w["P"], w["kd"])
    nd = t.set_occupancy(w["occ"])
    t.set_permittivity(w["m"] ** 2, "ldr")
    t.build_spectrum()
    i = t.info()
    out = {"workload": f"{name}: {w['K']}^3 lattice, {nd} dipoles, FFT grid {i['Kpp']}x{i['Jpp']}x{i['Ppp']}, "
                       f"{nrhs} right-hand side(s)", "nrhs": nrhs}
    for prec in precisions:
        dt = torch.complex64 if prec == "fp32" else torch.complex128
        b = 8 if prec == "fp32" else 16
        x = torch.from_numpy(inputs.complex_gaussian(0, (nrhs, 3, nd)).astype(np.complex64)).to("cuda", dt)
        y = torch.empty_like(x)
        Sv = [0.1 * (r % 4) for r in range(nrhs)]  # LDR factors in their range; timing does not depend on them
        for _ in range(3):
            t.matvec(x, S=Sv, jacobi=True, out=y)  # tunes the schedule on the first call
        torch.cuda.synchronize()
        lib.profile(True)
        lib.profile_reset()
        for _ in range(reps):
            t.matvec(x, S=Sv, jacobi=True, out=y)
        prof = lib.profile_read()
        lib.profile(2)  # the whole products alone, no events between their passes
        lib.profile_reset()
        for _ in range(reps):
            t.matvec(x, S=Sv, jacobi=True, out=y)
        ms, n = lib.profile_read()[("matvec", prec)]
        lib.profile(False)
        us = ms / n * 1e3
        b3 = b3_bytes(w["K"], w["J"], w["P"], i["Jpp"], i["Kh"], i["Jh"], i["Ph"], nd, b, nrhs)
        out[prec] = {"us": round(us, 2), "B3_bytes": b3, "gbps_B3": round(b3 / us / 1e3, 1),
                     "frac_B3": round(b3 / us / 1e3 / HBM_PEAK_GBPS, 4),
                     "passes_us": {p: round(prof[(p, prec)][0] / prof[(p, prec)][1] * 1e3, 2)
                                   for p in dda.PASS_NAMES if p != "matvec" and prof[(p, prec)][1]}}
        del x, y
    t.close()
    torch.cuda.empty_cache()
    return out


def cpu_baseline(w, nd, matvecs_per_solve, budget_s=12.0):
    """The CPU oracle (dense O(N_d^2) FP64 matvec, OpenMP over rows) timed on a
    bounded sample of rows of the same matrix, extrapolated to the matvecs one
    FP64 solve of this workload needs."""
    import numpy as np

    import oracle as ora
    from paper_0908_0863_amd import inputs

    sites = ora.sites_of(w["occ"])
    eps = w["m"] ** 2
    ainv = ora.alpha_inv(np.full(nd, eps), w["kd"], "ldr", 0.0)
    x = inputs.complex_gaussian(0, (3, nd))
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        pass
    cores = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))
    # grow the row sample until one run takes about budget_s (the first call
    # also pays the thread pool's start-up, so a single calibration undershoots)
    rows, t = 32, 0.0
    for _ in range(6):
        sel = np.linspace(0, nd - 1, rows).astype(np.int64)
        t0 = time.perf_counter()
        ora.dense_matvec(sites, w["kd"], ainv, x, rows=sel, nthreads=cores)
        t = time.perf_counter() - t0
        if t >= 0.5 * budget_s or rows >= nd:
            break
        rows = int(min(nd, max(2 * rows, rows * budget_s / max(t, 1e-4))))
    t_matvec = t * nd / rows
    t_solve = t_matvec * matvecs_per_solve
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"dense FP64 matvec on {rows} of {nd} rows ({t:.1f} s), extrapolated to a full matvec "
                      f"({t_matvec:.1f} s) x {matvecs_per_solve} matvecs per FP64 QMR_sym solve"}


def _line(metric, value, unit, args, el, steps, dtype, config, **extra):
    res = {"metric": metric, "value": round(value, 3), "unit": unit, "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": round(el / steps * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}
    res.update(extra)
    print(json.dumps(res), flush=True)


def batch_rhs_summary(lib, name, n, steps, warmup, tol, inner_tol, fp64_ref=True):
    """All orientations of one target in a single multi-right-hand-side mixed
    solve (the spectrum is shared): solves/s; the FP64 single-RHS path on a
    subset of the same right-hand sides (extrapolated); and the largest
    relative error of each cross section over all right-hand sides against one
    FP64 solve to 1e-12."""
    import numpy as np
    import torch

    from paper_0908_0863_amd import dda, inputs
    w = inputs.workload(name)
    t = dda.Target(lib, w["K"], w["J"], w["P"], w["kd"])
    nd = t.set_occupancy(w["occ"])
    t.set_permittivity(w["m"] ** 2, "ldr")
    n = n if n > 0 else len(w["khat"])
    khat = np.array(w["khat"][:n])
    ehat = np.array(w["ehat"][:n], np.complex128)
    kw = dict(solver="qmr_sym", tol=tol, inner_tol=inner_tol, check_every=16, use_graph=True)
    t.build_spectrum()
    for _ in range(max(1, warmup)):
        t.solve(khat=khat, ehat=ehat, precision="mixed", **kw)
    torch.cuda.synchronize()
    steps = max(1, steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        t.build_spectrum()
        Pm, im = t.solve(khat=khat, ehat=ehat, precision="mixed", **kw)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    E = t.incident_field(khat, ehat)
    cm = t.cross_sections(E, Pm)  # S of the solve, derived by the library from khat/ehat
    del Pm
    # FP64 single-RHS path on the first right-hand sides
    m64 = min(n, 16)
    t.solve(khat=khat[:1], ehat=ehat[:1], precision="fp64", **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for r in range(m64):
        t.solve(khat=khat[r:r + 1], ehat=ehat[r:r + 1], precision="fp64", **kw)
    torch.cuda.synchronize()
    e64 = time.perf_counter() - t1
    value = n * steps / el
    out = dict(workload=f"{name}: {w['K']}x{w['J']}x{w['P']} lattice, {nd} dipoles, {n} right-hand sides "
                        f"(orientations x polarisations) in one mixed solve, QMR_sym to {tol:g}",
               nrhs=n, nd=nd, solves_per_s=round(value, 3), seconds_per_batch=round(el / steps, 3),
               iterations_max=max(i["iterations"] for i in im), outer_max=max(i["outer_iterations"] for i in im),
               rel_residual_max=max(i["rel_residual"] for i in im),
               fp64_single_rhs_solves_per_s=round(m64 / e64, 3),
               fp64_single_rhs_sample=f"{m64} of {n} right-hand sides solved one by one in FP64 to {tol:g}, "
                                      f"rate extrapolated to all",
               speedup_vs_fp64_single=round(value / (m64 / e64), 3))
    if fp64_ref:
        t2 = time.perf_counter()
        Pr, ir = t.solve(khat=khat, ehat=ehat, precision="fp64", **dict(kw, tol=1e-12))
        cr = t.cross_sections(E, Pr)
        torch.cuda.synchronize()
        del Pr
        errs = [float(np.max(np.abs(cm[c] - cr[c]) / np.abs(cr[c]))) for c in range(3)]
        out["cross_section_max_rel_err_vs_fp64_1e-12"] = {"cext": errs[0], "cabs": errs[1], "csca": errs[2],
                                                           "over": f"all {n} right-hand sides",
                                                           "reference_solve_s": round(time.perf_counter() - t2, 2)}
        if max(errs) > 1e-6:
            # the residual at which every cross section is within 1e-6 of FP64,
            # and the throughput there (same batched mixed solve, timed once)
            tol2 = tol / 5
            t.solve(khat=khat[:1], ehat=ehat[:1], precision="mixed", **dict(kw, tol=tol2))  # tunes nothing new
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            P2, i2 = t.solve(khat=khat, ehat=ehat, precision="mixed", **dict(kw, tol=tol2))
            torch.cuda.synchronize()
            e3 = time.perf_counter() - t3
            c2 = t.cross_sections(E, P2)
            del P2
            errs2 = [float(np.max(np.abs(c2[c] - cr[c]) / np.abs(cr[c]))) for c in range(3)]
            t4 = time.perf_counter()
            for r in range(m64):
                t.solve(khat=khat[r:r + 1], ehat=ehat[r:r + 1], precision="fp64", **dict(kw, tol=tol2))
            torch.cuda.synchronize()
            f64b = m64 / (time.perf_counter() - t4)
            out["at_tighter_residual"] = {"tol": tol2, "solves_per_s": round(n / e3, 3),
                                          "fp64_single_rhs_solves_per_s": round(f64b, 3),
                                          "speedup_vs_fp64_single": round(n / e3 / f64b, 3),
                                          "rel_residual_max": max(i["rel_residual"] for i in i2),
                                          "cross_section_max_rel_err_vs_fp64_1e-12":
                                              {"cext": errs2[0], "cabs": errs2[1], "csca": errs2[2]}}
    t.close()
    torch.cuda.empty_cache()
    return out


def bench_batch_rhs(args):
    from paper_0908_0863_amd import dda
    lib = dda.Library(0)
    name = args.workload if args.workload != "cube64" else "ellipsoid96"
    t0 = time.perf_counter()
    r = batch_rhs_summary(lib, name, args.nrhs, min(args.steps, 3), args.warmup, args.tol, args.inner_tol,
                          fp64_ref=not args.no_fp64)
    steps = max(1, min(args.steps, 3))
    _line("DDA solves/sec at 1e-6 residual, batched right-hand sides (mixed)", r["solves_per_s"], "solves/s", args,
          r["seconds_per_batch"] * steps, steps, "f32+f64", {"workload": r["workload"], "nrhs": r["nrhs"],
                                                            "nd": r["nd"]},
          **{k: v for k, v in r.items() if k not in ("workload", "nrhs", "nd", "solves_per_s")},
          wall_s=round(time.perf_counter() - t0, 1))


def bench_batch_targets(args):
    """40 seeded aggregates (2 polarisations along +z each) through the
    multi-target batch solve, against the same items solved one after another."""
    import numpy as np
    import torch

    from paper_0908_0863_amd import dda, inputs
    aggs = inputs.aggregates(4, 40)
    kd = 2 * np.pi / 25
    lib = dda.Library(0)
    zh, xh, yh = [0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]
    items, nds = [], []
    tb0 = time.perf_counter()
    for a in aggs:
        L = a["L"]
        t = dda.Target(lib, L, L, L, kd)
        nds.append(t.set_occupancy(a["occ"]))
        t.set_permittivity(a["m"] ** 2, "ldr")
        t.build_spectrum()
        items.append(dict(target=t, khat=[zh, zh], ehat=[xh, yh]))
    torch.cuda.synchronize()
    t_spec = time.perf_counter() - tb0
    kw = dict(solver="qmr_sym", precision="mixed", tol=args.tol, inner_tol=args.inner_tol, check_every=16,
              use_graph=True)
    lib.batch_solve(items, nworkers=args.workers, **kw)  # warm-up: tuning, workspaces, graphs
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 3))
    t0 = time.perf_counter()
    for _ in range(steps):
        res = lib.batch_solve(items, nworkers=args.workers, **kw)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    t1 = time.perf_counter()
    lib.batch_solve(items, nworkers=1, **kw)
    torch.cuda.synchronize()
    e1 = time.perf_counter() - t1
    nrhs = 2 * len(items)
    value = nrhs * steps / el
    _line("DDA solves/sec at 1e-6 residual, multi-target batch (mixed)", value, "solves/s", args, el, steps,
          "f32+f64", {"workload": f"40 seeded aggregates of 20..200 touching spheres (radius 4 d), lattices "
                                  f"{min(a['L'] for a in aggs)}..{max(a['L'] for a in aggs)}^3, {min(nds)}..{max(nds)} "
                                  f"dipoles, kd = 2 pi / 25, 2 polarisations along +z, QMR_sym to {args.tol:g}",
                      "targets": len(items), "nrhs": nrhs},
          workers=args.workers or 4, one_worker_solves_per_s=round(nrhs / e1, 3),
          speedup_vs_one_worker=round(value / (nrhs / e1), 3), spectrum_build_s=round(t_spec, 3),
          iterations_max=max(i["iterations"] for _, inf in res for i in inf))


def bench_paper200(args):
    """The paper's benchmark solve (Sec. 6, Table 3): 200^3 sphere, N_d =
    4,188,896, lambda = 3.175 um, a_eff = 0.5 um, m = 1.63631 + 0.372i,
    polarisation x, FP64, tol 1e-10, zero initial guess, Point-Jacobi.  The
    paper's times (NEMO, 2x dual-core Opteron 275; serial / OpenMP on 4
    cores) are quoted as context."""
    import torch

    from paper_0908_0863_amd import dda, inputs
    w = inputs.workload("sphere200")
    lib = dda.Library(0)
    t = dda.Target(lib, 200, 200, 200, w["kd"])
    nd = t.set_occupancy(w["occ"])
    t.set_permittivity(w["m"] ** 2, "ldr")
    torch.cuda.synchronize()
    # padded lengths chosen by timing FP64 products (planning by measurement)
    t0 = time.perf_counter()
    pads = t.tune_padding(1, "fp64")
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    t0 = time.perf_counter()
    t.build_spectrum()
    torch.cuda.synchronize()
    t_spec = time.perf_counter() - t0
    # Table 3: scheme (SV) -> iterations, serial and OpenMP-4 seconds on NEMO
    paper = {("bicg", 0): (21, 1439.7, 404.3), ("bicg_sym", 0): (21, 741.5, 212.7),
             ("bicgstab", 0): (12, 846.6, 234.7), ("cgs", 0): (13, 911.3, 257.4),
             ("mlbicgstab", 1): (12, 836.0, 238.9), ("mlbicgstab", 2): (8, 811.7, 246.2),
             ("mlbicgstab", 3): (6, 842.9, 266.2), ("qmr", 0): (22, 3704.6, 1055.1),
             ("qmr_sym", 0): (21, 759.6, 216.7), ("rbicgstab", 1): (14, 996.3, 284.5),
             ("rbicgstab", 2): (7, 990.5, 285.2), ("rbicgstab", 3): (4, 851.1, 242.2),
             ("tfqmr", 0): (13, 1850.3, 524.7)}
    out = {}
    for (solver, sv), (ni, ser, omp) in paper.items():
        kw = dict(khat=w["khat"], ehat=w["ehat"], solver=solver, solver_param=sv, precision="fp64", tol=1e-10,
                  check_every=4, use_graph=True)
        t.solve(**kw)  # tuning, workspaces, graph
        torch.cuda.synchronize()
        steps = max(1, min(args.steps, 5))
        t1 = time.perf_counter()
        for _ in range(steps):
            P, info = t.solve(**kw)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t1) / steps
        key = solver + (f"({sv})" if sv else "")
        out[key] = dict(iterations=info[0]["iterations"], seconds=round(el, 4), paper_iterations=ni,
                        paper_serial_s=ser, paper_openmp4_s=omp, speedup_vs_openmp4=round(omp / el, 1))
    total = sum(v["seconds"] for v in out.values())
    _line("Table 3 benchmark solves/sec (200^3 sphere, FP64, tol 1e-10)", len(out) / total, "solves/s", args,
          total, len(out), "f64", {"workload": f"sphere200: 200^3 lattice, {nd} dipoles, m=1.63631+0.372i, "
                                               f"kd={w['kd']:.6f}, FFT grid {pads[0]}x{pads[1]}x{pads[2]} (tuned), "
                                               f"tol 1e-10, Jacobi"},
          solvers=out, spectrum_build_s=round(t_spec, 4), padding_tune_s=round(t_plan, 3),
          paper_spectrum_build_s={"serial": 13.4, "openmp4": 3.8})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cube64")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--inner-tol", type=float, default=0.0,
                    help="FP32 inner-solve tolerance (default: 5e-5 for the single-RHS line, 1e-4 for the batch modes)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--tune-file", default=None,
                    help="autotuner record to read and extend (default: a fresh one per run); a profiled run "
                         "given the file of an earlier run uses the same plans")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline only: skip the 128^3 / 96^3 x 128 keys (matvec_rates, batched_orientations)")
    ap.add_argument("--fp64", action="store_true", help="--profile-matvec: FP64 vectors")
    ap.add_argument("--schedule", type=int, default=-1, help="--profile-matvec: force a matvec schedule (-1: tuned)")
    ap.add_argument("--composition", type=int, default=0,
                    help="--profile-matvec: seeded random composition of this many materials per dipole and "
                         "direction (bit-fielded diagonal) instead of one permittivity")
    ap.add_argument("--iso-random", action="store_true",
                    help="--profile-matvec: seeded random isotropic permittivity per dipole (per-dipole diagonal)")
    ap.add_argument("--profile-matvec", type=int, default=0,
                    help="only run this many FP32 matrix-vector products (for rocprofv3 counter runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates the HBM byte counters)")
    ap.add_argument("--mode", choices=["single", "batch-rhs", "batch-targets", "paper200"], default="single",
                    help="single: one right-hand side of --workload (the headline line); batch-rhs: all "
                         "orientations of --workload in one multi-RHS solve; batch-targets: 40 seeded "
                         "aggregates through the multi-target batch solve; paper200: the paper's Table 3 "
                         "benchmark solve (200^3 sphere, FP64, tol 1e-10) with the schemes of its Table 3")
    ap.add_argument("--nrhs", type=int, default=0,
                    help="batch-rhs: right-hand sides (default: all); --profile-matvec: right-hand sides (default 1)")
    ap.add_argument("--workers", type=int, default=0, help="batch-targets: host workers (default 4)")
    args = ap.parse_args()
    if args.inner_tol <= 0:
        args.inner_tol = 5e-5 if args.mode == "single" else 1e-4
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is described in DESIGN.md but not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0908_0863_amd import dda, inputs

    torch.cuda.set_device(0)
    if args.copy_probe:
        n = 1 << 27  # complex64 elements: 1 GiB
        a = torch.ones(n, dtype=torch.complex64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 5}))
        return
    if args.mode == "batch-targets":
        return bench_batch_targets(args)
    if args.mode == "batch-rhs":
        return bench_batch_rhs(args)
    if args.mode == "paper200":
        return bench_paper200(args)
    w = inputs.workload(args.workload)
    K, J, P = w["K"], w["J"], w["P"]
    import tempfile
    tune_file = args.tune_file or os.path.join(tempfile.mkdtemp(prefix="dda_tune_"), "tune.txt")
    lib = dda.Library(0, tune_cache=tune_file)
    t = dda.Target(lib, K, J, P, w["kd"])
    nd = t.set_occupancy(w["occ"])
    eps = w["m"] ** 2
    t.set_permittivity(eps, "ldr")
    khat = np.array(w["khat"][:1])
    ehat = np.array(w["ehat"][:1], np.complex128)
    E = t.incident_field(khat, ehat)
    info = t.info()

    if args.profile_matvec:
        # only products (for rocprofv3 counter and trace runs): --nrhs right-hand sides
        rng = np.random.default_rng(7)
        if args.composition:
            mats = eps + 0.05 * np.arange(args.composition)
            t.set_composition(mats, rng.integers(0, args.composition, (3, nd)), "ldr")
        elif args.iso_random:
            t.set_permittivity(eps + 0.05 * rng.random(nd), "ldr")
        if args.schedule >= 0:
            t.set_option(dda.DDA_OPT_SCHEDULE, args.schedule)
        t.build_spectrum()
        nr = max(1, args.nrhs)
        x = torch.from_numpy(inputs.complex_gaussian(0, (nr, 3, nd), np.complex64)).cuda()
        if args.fp64:
            x = x.to(torch.complex128)
        y = torch.empty_like(x)
        Sz = [0.0] * nr
        t.matvec(x, S=Sz, jacobi=True, out=y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.profile_matvec):
            t.matvec(x, S=Sz, jacobi=True, out=y)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / args.profile_matvec
        print(json.dumps({"workload": args.workload, "nrhs": nr, "dtype": str(x.dtype), "matvec_us": el * 1e6,
                          "count": args.profile_matvec, "tuned_schedules": open(tune_file).read().split("\n")
                          if os.path.exists(tune_file) else []}))
        return

    def step(precision):
        t.build_spectrum()
        P_, inf = t.solve(khat=khat, ehat=ehat, solver="qmr_sym", precision=precision, tol=args.tol,
                          inner_tol=args.inner_tol, check_every=16, use_graph=not profiling[0])
        ce, ca, cs = t.cross_sections(E, P_)  # S of the solve (derived by the library from khat/ehat)
        return P_, inf, (ce[0], ca[0], cs[0])

    profiling = [False]
    # reference cross sections: FP64 solve to 1e-12
    t.build_spectrum()
    Pref, infref = t.solve(khat=khat, ehat=ehat, solver="qmr_sym", precision="fp64", tol=1e-12)
    cref = [c[0] for c in t.cross_sections(E, Pref)]
    del Pref

    for _ in range(args.warmup):
        step("mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Pm, infm, cm = step("mixed")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    value = args.steps / el
    # the same steps again with every matrix-vector pass, and every whole
    # product, bracketed by HIP events on its stream (eager launches: events
    # are not captured)
    profiling[0] = True
    lib.profile(True)
    lib.profile_reset()
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(args.steps):
        step("mixed")
    torch.cuda.synchronize()
    el_prof = time.perf_counter() - tp0
    prof = lib.profile_read()
    # and once more with events around the whole products only, so that no
    # event record sits between two passes of the product being timed
    lib.profile(2)
    lib.profile_reset()
    for _ in range(args.steps):
        step("mixed")
    prof_mv = lib.profile_read()
    # and the same product on its own (dda_matvec: this target, its tuned
    # FP32 schedule, the solve's orientation factor, Jacobi form), without
    # the QMR_sym step that the solve fuses into its y-forward pass
    S_solve = t.orientation_factors(1)
    xs = torch.from_numpy(inputs.complex_gaussian(11, (1, 3, nd)).astype(np.complex64)).cuda()
    ys = torch.empty_like(xs)
    for _ in range(3):
        t.matvec(xs, S=S_solve, jacobi=True, out=ys)
    lib.profile_reset()
    n_alone = 200
    for _ in range(n_alone):
        t.matvec(xs, S=S_solve, jacobi=True, out=ys)
    prof_alone = lib.profile_read()
    del xs, ys
    lib.profile(False)
    profiling[0] = False

    # plain FP64 single-RHS GPU path on the same right-hand side
    fp64 = None
    if not args.no_fp64:
        step("fp64")
        torch.cuda.synchronize()
        k64 = max(1, args.steps // 2)
        t1 = time.perf_counter()
        for _ in range(k64):
            P64, inf64, c64 = step("fp64")
        torch.cuda.synchronize()
        e64 = time.perf_counter() - t1
        fp64 = dict(solves_per_s=k64 / e64, iterations=inf64[0]["iterations"], matvecs=inf64[0]["matvecs"],
                    rel_residual=inf64[0]["rel_residual"],
                    cross_section_rel_err=[abs(c64[i] - cref[i]) / abs(cref[i]) for i in range(3)])

    bpe = {pr: pass_bytes(K, J, P, info["Kpp"], info["Jpp"], info["Kh"], info["Jh"], info["Ph"], nd,
                          8 if pr == "fp32" else 16, True) for pr in ("fp32", "fp64")}
    passes = {f"{k[0]}_{k[1]}": dict(avg_us=round(v[0] / v[1] * 1e3, 2), launches=v[1],
                                     **({"gbps": round(bpe[k[1]][k[0]] / (v[0] / v[1] / 1e3) / 1e9, 1)}
                                        if k[0] in bpe[k[1]] else {}))
              for k, v in prof.items() if v[1] > 0}
    # roofline: the whole FP32 product (every pass and the gaps between them,
    # HIP events on the launch stream) against the 3-pass byte model B3
    mv_ms, mv_n = prof_alone[("matvec", "fp32")]
    mv_s = mv_ms / mv_n / 1e3
    sv_ms, sv_n = prof_mv[("matvec", "fp32")]
    sv_s = sv_ms / sv_n / 1e3
    b3 = b3_bytes(K, J, P, info["Jpp"], info["Kh"], info["Jh"], info["Ph"], nd, 8)
    achieved = b3 / mv_s / 1e9
    sched32 = tuned_schedule(tune_file, K, J, P, "fp32")
    pass_sum_s = sum(prof[(p, "fp32")][0] / prof[(p, "fp32")][1] for p in dda.PASS_NAMES
                     if p != "matvec" and prof[(p, "fp32")][1]) / 1e3
    # the z pass (z DFT, product, inverse z DFT) on its own bytes, and the
    # longest FP32 pass of the product
    zname = "z_product"
    zms, zn = prof[(zname, "fp32")]
    lname, lms, ln = max(((p, *prof[(p, "fp32")]) for p in dda.PASS_NAMES
                          if p != "matvec" and prof[(p, "fp32")][1]), key=lambda a: a[1] / a[2])
    z_s = zms / zn / 1e3
    z_ach = bpe["fp32"][zname] / z_s / 1e9

    res = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64 (FP32 FFT passes and Krylov vectors; FP64 residual, refinement, inner products)",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {K}x{J}x{P} lattice, {nd} dipoles, m={w['m']}, "
                               f"kd={w['kd']:.5f}, FFT grid {info['Kpp']}x{info['Jpp']}x{info['Ppp']}, "
                               f"QMR_sym to {args.tol:g} true FP64 residual, 1 RHS",
                   "solver": "qmr_sym", "precision": "mixed", "tol": args.tol, "inner_tol": args.inner_tol,
                   "nrhs": 1, "nd": nd},
        "roofline": {"bound": "hbm", "kernel": "FP32 matrix-vector product (all passes)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": measured_traffic("matvec", args.workload, sched32),
                     "schedule": sched32,
                     "bytes": "B3 = 8 [9 N_d + 12 K J'' P + 6 K_h J_h P_h] per product (3-pass model)",
                     "bytes_per_launch": b3, "avg_launch_us": round(mv_s * 1e6, 2), "launches": mv_n,
                     "pass_kernels_sum_us": round(pass_sum_s * 1e6, 2),
                     "timed": f"HIP events around each of {mv_n} products of the headline target on its own "
                              f"(dda_matvec, tuned FP32 schedule, Jacobi form, the solve's S; nothing between "
                              f"the passes), eager launches",
                     "in_solve": {"avg_launch_us": round(sv_s * 1e6, 2), "launches": sv_n,
                                  "frac_B3": round(b3 / sv_s / 1e9 / HBM_PEAK_GBPS, 4),
                                  "note": f"the products inside {args.steps} repeated timed steps; their "
                                          f"y-forward pass also runs the fused QMR_sym step (its vector "
                                          f"traffic is not in B3); passes timed one by one in another "
                                          f"{args.steps} steps ({el_prof / args.steps * 1e3:.2f} ms/step)"},
                     "z_kernel": {"pass": zname, "achieved": round(z_ach, 1),
                                  "frac": round(z_ach / HBM_PEAK_GBPS, 4), "avg_launch_us": round(z_s * 1e6, 2),
                                  "bytes_per_launch": bpe["fp32"][zname],
                                  "traffic": measured_traffic(zname, args.workload, sched32)},
                     "longest_pass": {"pass": lname, "avg_launch_us": round(lms / ln * 1e3, 2)}},
        "solve": {"iterations": infm[0]["iterations"], "outer_iterations": infm[0]["outer_iterations"],
                  "matvecs": infm[0]["matvecs"], "rel_residual": infm[0]["rel_residual"],
                  "cross_sections": {"cext": cm[0], "cabs": cm[1], "csca": cm[2]},
                  "cross_section_rel_err_vs_fp64_1e-12": [abs(cm[i] - cref[i]) / abs(cref[i]) for i in range(3)]},
        "fp64_single_rhs": fp64,
        "mixed_vs_fp64_speedup": round(value / fp64["solves_per_s"], 3) if fp64 else None,
        "passes": passes,
        "tuned_schedules": [ln.strip() for ln in open(tune_file)] if os.path.exists(tune_file) else [],
    }
    t.close()
    torch.cuda.empty_cache()
    if not args.no_extra:
        # larger-than-cache working sets: the 128^3 sphere, the 128-RHS ellipsoid batch
        res["matvec_rates"] = {"sphere128": matvec_rates(lib, "sphere128", 1),
                               "ellipsoid96_x128": matvec_rates(lib, "ellipsoid96", 128, reps=3,
                                                                precisions=("fp32",))}
        res["batched_orientations"] = batch_rhs_summary(lib, "ellipsoid96", 128, 1, 1, args.tol, 1e-4,
                                                        fp64_ref=not args.no_fp64)
    if not args.no_cpu:
        mv = fp64["matvecs"] if fp64 else infref[0]["matvecs"]
        res["cpu_baseline"] = cpu_baseline(w, nd, mv)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
