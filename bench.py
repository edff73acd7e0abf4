#!/usr/bin/env python3
"""Throughput of the FFT + Thomas Poisson solve on one MI355X.

Metric: grid points solved per second (Mpts/s) at 512^3, periodic x,y /
Neumann z, source = discrete divergence of a seeded Gaussian velocity field
(workload div_ppn), in double precision; the float solve wrapped in double
iterative refinement is timed beside it.  One step = one complete solve
(x forward transform, z march with the y transforms and z solves, x inverse
transform, reductions) of one right-hand side already resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload div_ppn]

Prints one JSON line on stdout; progress goes to stderr.  The per-kernel
durations come from HIP events the library records on the solve's stream
during the timed steps.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpts/s per solve at 512^3 (FP64 vs FP32+refine @1e-12); % peak HBM BW"
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, published peak
GROUPS = ("x_forward", "z_march", "x_inverse", "other")
KERNEL_NAMES = {"x_forward": "k_xfwd", "z_march": "k_zpipe", "x_inverse": "k_xinv"}   # k_zmarch when ny > 1024
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
# sources whose changes can change the kernels' traffic (the plan code lays out
# the tables the z march reads)
SOURCES = [os.path.join(ROOT, "paper_1909_05423_amd", "csrc", n)
           for n in ("pp_device.hpp", "pp_kernels.hpp", "xdir.hip", "zmarch.hip", "zpcr.hip", "plan.cpp")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for p in SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(plan_shape, batch, slots, elem_in, elem_spec):
    """Bytes each kernel must move through HBM per launch (one pass over its
    input and output), as a dict keyed by kernel group."""
    nz, ny, nx = plan_shape
    n = nx * ny * nz * batch
    spec = slots * ny * nz * batch * elem_spec     # spectral array S (complex)
    return {
        "x_forward": n * elem_in + spec,           # read f, write S
        "z_march": 4 * spec,                       # read+write S upward, read+write S downward
        "x_inverse": spec + n * elem_in,           # read S, write u
    }


def refined_bytes(plan_shape, batch, slots, corrections):
    """Algorithmic bytes of one refined solve with the given number of
    corrections (rows up to 512: the first correction's residual fused into its
    x transform), per kernel group: the first solve reads f (8 B/pt), writes
    float spectra, marches them (read + write up and down) and writes the float
    first solution u0; the first correction reads f and u0, marches, and reads
    u0 to write u (8 B/pt); later corrections read and write u itself."""
    nz, ny, nx = plan_shape
    n = nx * ny * nz * batch
    spec = slots * ny * nz * batch * 8             # float spectra
    xf = (n * 8 + spec) + (n * 8 + n * 4 + spec)
    zm = 2 * 4 * spec
    xi = (spec + n * 4) + (spec + n * 4 + n * 8)
    for _ in range(max(0, corrections - 1)):
        xf += n * 8 + n * 8 + n * 4 + n * 4 + spec  # residual (f, u in; float r out) + x transform of r
        zm += 4 * spec
        xi += spec + 2 * n * 8
    return {"x_forward": xf, "z_march": zm, "x_inverse": xi}


def traffic_for(group, workload, dtype):
    """HBM bytes per launch measured by rocprofv3 (FETCH_SIZE + WRITE_SIZE,
    scaled by the copy-kernel calibration), if taken on the current kernels."""
    try:
        with open(TRAFFIC_FILE) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    if data.get("kernel_source_hash") != kernel_source_hash():
        return None
    entry = data.get("entries", {}).get(f"{workload}/{dtype}/{group}")
    return None if entry is None else entry.get("bytes_per_launch")


def time_solves(plan, f, u, steps, warmup, lib, faces=None):
    import ctypes
    import torch
    kw = {} if faces is None else {"faces": faces}
    for _ in range(warmup):
        plan.solve(f, u, **kw)
    torch.cuda.synchronize()
    lib.pp_plan_set_timing(plan._handle, 1)
    lib.pp_plan_kernel_times(plan._handle, None, None, 1)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        plan.solve(f, u, **kw)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = (ctypes.c_double * 4)()
    cnt = (ctypes.c_int * 4)()
    lib.pp_plan_kernel_times(plan._handle, ms, cnt, 1)
    lib.pp_plan_set_timing(plan._handle, 0)
    per = {}
    for g, name in enumerate(GROUPS):
        per[name] = dict(total_ms=ms[g], launches=cnt[g], avg_ms=(ms[g] / cnt[g] if cnt[g] else None))
    return start.elapsed_time(end) / steps, wall, per


def roofline_block(per, abytes, workload, dtype, ny):
    best = None
    for g in ("x_forward", "z_march", "x_inverse"):
        k = per[g]
        if k["launches"] and (best is None or k["total_ms"] > per[best]["total_ms"]):
            best = g
    k = per[best]
    achieved = abytes[best] / (k["avg_ms"] * 1e-3) / 1e9
    traffic = traffic_for(best, workload, dtype)
    name = KERNEL_NAMES[best]
    if best == "z_march" and ny > 1024:
        name = "k_zmarch"
    return dict(bound="hbm", kernel=name, achieved=round(achieved, 1), peak=PEAK_HBM_GBS,
                unit="GB/s", frac=round(achieved / PEAK_HBM_GBS, 4), traffic=traffic,
                bytes_per_launch=abytes[best], avg_launch_ms=round(k["avg_ms"], 5))


def device_copy_bandwidth(lib, reps=10):
    """Read + write bandwidth of a 1 GiB device-to-device copy: the library's
    streaming copy (pp_stream_copy: 16-byte non-temporal loads and stores,
    persistent grid), the practical ceiling for a kernel that streams its
    input once and its output once; and torch's copy_ beside it."""
    import ctypes
    import torch
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").normal_()
    b = torch.empty_like(a)
    nbytes = a.numel() * a.element_size()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def own():
        st = lib.pp_stream_copy(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), nbytes, stream)
        if st != 0:
            raise RuntimeError(f"pp_stream_copy: {st}")

    out = {}
    for name, fn in (("stream_copy", own), ("torch_copy", lambda: b.copy_(a))):
        fn()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        for _ in range(reps):
            fn()
        end.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(end) / reps
        out[name] = 2 * nbytes / (ms * 1e-3) / 1e9
    if not torch.equal(a, b):
        raise RuntimeError("device copy check failed")
    del a, b
    return out


def zsolver_sweep(lib, warmup, steps=10, bc="PPPPNN"):
    """The paper's comparison of the tridiagonal solvers (section "Comparison of
    Tridiagonal Solvers"): 64 x 64 x nz grids, nz = 2^n - 1 up to 4095, the
    whole f64 solve timed with the fused Thomas march (its automatic layout,
    and forced segmented), PCR and CR-P (the last two with the y transforms
    as separate passes).  Seeded N(0,1) source."""
    import numpy as np
    import torch
    from paper_1909_05423_amd import Plan
    rows = []
    for nz in (255, 511, 1023, 2047, 4095):
        shape = (nz, 64, 64)
        h = (1 / 64, 1 / 64, 1 / nz)
        f = torch.from_numpy(np.random.default_rng(nz).standard_normal((1,) + shape)).to("cuda")
        u = torch.empty_like(f)
        row = {"nz": nz}
        ref = None
        for key in ("thomas", "thomas_segmented", "pcr", "cr"):
            if key == "thomas_segmented":   # forced: the automatic choice keeps the zero mode's column whole
                plan = Plan(shape, bc, h, dtype="f64", zsplit="seg")
            else:
                plan = Plan(shape, bc, h, dtype="f64", zsolver=key)
            ms, _, _ = time_solves(plan, f, u, steps, warmup, lib)
            row[f"{key}_ms"] = round(ms, 4)
            if ref is None:
                ref = u.clone()
            else:
                row[f"{key}_max_rel_diff_vs_thomas"] = float((u - ref).abs().max() / ref.abs().max())
            del plan
        rows.append(row)
        log(f"64 x 64 x {nz}: Thomas {row['thomas_ms']:.3f} ms (segmented {row['thomas_segmented_ms']:.3f} ms), "
            f"PCR {row['pcr_ms']:.3f} ms, CR-P {row['cr_ms']:.3f} ms")
        del f, u, ref
    return {"shape": "64 x 64 x nz", "bc": bc, "dtype": "f64", "rows": rows}


def cpu_baseline(workload_name, min_seconds=10.0, max_reps=8):
    """The oracle, timed on this host, on the same recipe on a 512 x 512 x 32
    slab of the 512^3 grid, repeated until about min_seconds of CPU work have
    run.  The oracle's transforms are direct sums over whole 512-long x and y
    lines, so their cost per point is that of the full grid; the z solves cost
    the same per point at any nz."""
    import numpy as np
    import oracle
    import workloads
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    full = workloads.WORKLOADS[workload_name]["shape"]
    shape = (min(32, full[0]), full[1], full[2])
    wl = workloads.make(workload_name, shape=shape, batch=1)
    reps, dt = 0, 0.0
    while reps < max_reps and (reps == 0 or dt < min_seconds):
        t0 = time.perf_counter()
        u = oracle.solve(wl["f"][0], wl["bc"], wl["h"])
        dt += time.perf_counter() - t0
        reps += 1
        del u
    pts = float(np.prod(shape)) * reps
    return dict(value=round(pts / dt / 1e6, 3), unit="Mpts/s", cores=int(threads), kind="oracle",
                sample=f"{reps} oracle solves of the {workload_name} recipe on a {shape[2]} x {shape[1]} x "
                       f"{shape[0]} slab (x, y lines as at full size; {dt:.1f} s wall in total, float64 numpy, "
                       f"BLAS threads {threads})")


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="div_ppn")
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--skip-refined", action="store_true")
    ap.add_argument("--skip-fp32", action="store_true", help="skip timing the plain float solve")
    ap.add_argument("--skip-faces", action="store_true", help="skip timing the solve with face values")
    ap.add_argument("--skip-periodic-z", action="store_true", help="skip timing the periodic-z solve")
    ap.add_argument("--skip-pcr", action="store_true", help="skip timing the PCR and CR-P z solvers")
    ap.add_argument("--skip-sweep", action="store_true",
                    help="skip the z-solver comparison on 64 x 64 x nz grids (the paper's sweep)")
    ap.add_argument("--skip-check", action="store_true", help="skip the host-side backward-error check")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (torch copy_) three times, as the reference "
                         "kernel of known size for hardware traffic counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solver has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads
    from paper_1909_05423_amd import Plan, _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1909_05423_amd import build
        log("library not built; building")
        build.build()
    lib = _lib.load()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")

    log(f"generating workload {args.workload}")
    wl = workloads.make(args.workload)
    shape, bc, h, batch = wl["shape"], wl["bc"], wl["h"], wl["batch"]
    npts = float(np.prod(shape)) * batch
    f = torch.from_numpy(wl["f"]).to("cuda")
    f_host = wl.pop("f")
    u = torch.empty_like(f)

    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").normal_()
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 1 GiB device copies done")
        del a, b
    copies = device_copy_bandwidth(lib)
    copy_gbs = copies["stream_copy"]
    log(f"device copy (1 GiB read + 1 GiB write): {copy_gbs:.0f} GB/s streaming kernel, "
        f"{copies['torch_copy']:.0f} GB/s torch copy_")

    log(f"plan f64 {shape} {bc} batch {batch}")
    plan = Plan(shape, bc, h, dtype="f64", batch=batch)
    ms, wall, per = time_solves(plan, f, u, args.steps, args.warmup, lib)
    log(f"f64: {ms:.3f} ms/solve, {npts / ms / 1e3:.0f} Mpts/s")
    slots = (shape[2] + 1) // 2
    ab64 = algorithmic_bytes(shape, batch, slots, 8, 16)
    kern = {g: dict(per[g]) for g in GROUPS}
    for g in ab64:
        if per[g]["avg_ms"]:
            kern[g]["algorithmic_GBs"] = round(ab64[g] / (per[g]["avg_ms"] * 1e-3) / 1e9, 1)
    total_bytes = sum(ab64.values())
    result = {
        "metric": METRIC,
        "value": round(npts / ms / 1e3, 1),
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "shape_zyx": list(shape), "bc": bc, "batch": batch,
                   "h": list(h)},
        "roofline": roofline_block(per, ab64, args.workload, "f64", shape[1]),
        "device_copy_GBs": round(copy_gbs, 1),
        "torch_copy_GBs": round(copies["torch_copy"], 1),
        "solve_hbm_GBs": round(total_bytes / (ms * 1e-3) / 1e9, 1),
        "solve_hbm_frac": round(total_bytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        "kernels": kern,
    }

    # correctness of the timed result (outside the timed region): normwise backward error
    if not args.skip_check:
        import oracle
        u64 = u.cpu().numpy()
        fp = f_host - f_host.mean(axis=(1, 2, 3), keepdims=True) if oracle.is_singular(bc) else f_host
        eta = max(oracle.backward_error(fp[b], u64[b], bc, h) for b in range(batch))
        result["f64_backward_error"] = float(eta)
        log(f"f64 backward error {eta:.2e}")

    if not args.skip_faces:
        # the same solve with non-homogeneous data on every non-periodic face
        # (Dirichlet values / Neumann fluxes drawn N(0,1), seeded), through pp_solve_bc
        gen = torch.Generator(device="cuda").manual_seed(5)
        faces = []
        for i in range(6):
            if bc[i] == "P":
                faces.append(None)
                continue
            faces.append(torch.randn(plan.face_shape(i), generator=gen, device="cuda", dtype=torch.float64))
        uf = torch.empty_like(f)
        ms_fc, _, per_fc = time_solves(plan, f, uf, args.steps, args.warmup, lib, faces=faces)
        result["faces"] = {
            "value": round(npts / ms_fc / 1e3, 1), "unit": "Mpts/s", "ms_per_step": round(ms_fc, 4),
            "faces": [bc[i] for i in range(6) if faces[i] is not None],
            "kernels": {g: dict(per_fc[g]) for g in GROUPS},
        }
        log(f"f64 with face values: {ms_fc:.3f} ms/solve")
        del faces, uf

    if not args.skip_periodic_z and bc[4:6] != "PP":
        # the same source with the z faces made periodic (cyclic z-systems)
        bcp = bc[:4] + "PP"
        plan_p = Plan(shape, bcp, h, dtype="f64", batch=batch)
        up = torch.empty_like(f)
        ms_p, _, per_p = time_solves(plan_p, f, up, args.steps, args.warmup, lib)
        result["periodic_z"] = {
            "bc": bcp, "value": round(npts / ms_p / 1e3, 1), "unit": "Mpts/s", "ms_per_step": round(ms_p, 4),
            "kernels": {g: dict(per_p[g]) for g in GROUPS},
        }
        log(f"f64 with periodic z ({bcp}): {ms_p:.3f} ms/solve")
        del plan_p, up

    if not args.skip_pcr and shape[0] <= 512 and shape[1] <= 512 and bc[4:6] != "PP":
        # the same solve with the z-systems by parallel cyclic reduction and by
        # cyclic reduction (y transforms as separate passes), for comparison
        # with the fused march
        for key in ("pcr", "cr"):
            plan_c = Plan(shape, bc, h, dtype="f64", batch=batch, zsolver=key)
            uc = torch.empty_like(f)
            ms_c, _, per_c = time_solves(plan_c, f, uc, args.steps, args.warmup, lib)
            result[key] = {
                "value": round(npts / ms_c / 1e3, 1), "unit": "Mpts/s", "ms_per_step": round(ms_c, 4),
                "max_rel_diff_vs_thomas": float((uc - u).abs().max() / u.abs().max()),
                "kernels": {g: dict(per_c[g]) for g in GROUPS},
            }
            log(f"f64 with {key.upper()} z solver: {ms_c:.3f} ms/solve")
            del plan_c, uc

    if not args.skip_sweep:
        result["zsolver_sweep"] = zsolver_sweep(lib, args.warmup)

    if not args.skip_refined:
        plan_r = Plan(shape, bc, h, dtype="f32_refined", batch=batch)
        ur = torch.empty_like(f)
        ms_r, _, per_r = time_solves(plan_r, f, ur, max(3, args.steps // 2), 2, lib)
        its, _, rel = plan_r.last_info()
        diff = float((ur - u).abs().max() / u.abs().max())
        kern_r = {g: dict(per_r[g]) for g in GROUPS}
        abr = refined_bytes(shape, batch, slots, its)
        for g in abr:
            if per_r[g]["total_ms"]:
                # bytes of all launches of the group over their total time
                kern_r[g]["algorithmic_GBs"] = round(abr[g] * per_r[g]["launches"] / (its + 1)
                                                     / (per_r[g]["total_ms"] * 1e-3) / 1e9, 1)
        result["fp32_refined"] = {
            "value": round(npts / ms_r / 1e3, 1), "unit": "Mpts/s", "ms_per_step": round(ms_r, 4),
            "refinement_steps": its, "last_rel_correction": rel, "max_rel_diff_vs_f64": diff,
            "bytes_per_point": round(sum(abr.values()) / npts, 2),
            "kernels": kern_r,
        }
        log(f"f32+refine: {ms_r:.3f} ms/solve, {its} corrections, diff vs f64 {diff:.2e}")
        del plan_r, ur

    if not args.skip_fp32:
        # the plain float solve (float source, arithmetic and spectra)
        plan_s = Plan(shape, bc, h, dtype="f32", batch=batch)
        fs = f.float()
        us = torch.empty_like(fs)
        ms_s, _, per_s = time_solves(plan_s, fs, us, args.steps, args.warmup, lib)
        ab32 = algorithmic_bytes(shape, batch, slots, 4, 8)
        kern_s = {g: dict(per_s[g]) for g in GROUPS}
        for g in ab32:
            if per_s[g]["avg_ms"]:
                kern_s[g]["algorithmic_GBs"] = round(ab32[g] / (per_s[g]["avg_ms"] * 1e-3) / 1e9, 1)
        result["fp32"] = {
            "value": round(npts / ms_s / 1e3, 1), "unit": "Mpts/s", "ms_per_step": round(ms_s, 4),
            "max_rel_diff_vs_f64": float((us.double() - u).abs().max() / u.abs().max()),
            "solve_hbm_GBs": round(sum(ab32.values()) / (ms_s * 1e-3) / 1e9, 1),
            "kernels": kern_s,
        }
        log(f"f32: {ms_s:.3f} ms/solve")
        del plan_s, fs, us

    if not args.skip_cpu_baseline:
        log("timing the oracle on a slab of the full grid")
        result["cpu_baseline"] = cpu_baseline(args.workload)
    result["context"] = {"paper_single_gpu_512cubed_Mpts_s": {"V100": 4.09, "K40": 1.56},
                         "note": "paper's multi-GPU code path on one GPU, boundary conditions unstated"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
