"""Benchmark of the hierarchical view-factor radiosity path on one MI355X.

Workload ``c3`` (default): 64 convex cavities (icospheres, ellipsoids,
closed cylinders; 2k-35k facets, 696,072 in all) solved together as one
block-diagonal system.  Low-rank factors are stored in BF16 (near field in
FP32) with an FP32 copy of the factors for the FP64 refinement residual.
One step = one batched radiosity solve of all 64 cavities (radiosity J and
facet flux q of eq. (12), one right-hand side each) with the H-matrices
resident in HBM, assembled once before the timed region as the paper reuses
its matrix over all Newton iterations and time steps.  ``value`` counts
solves (cavity right-hand sides) per second.  Beside it, on the same GPU and
cavities: the plain FP32 H-solve (per-cavity FP32 GMRES, one cavity at a
time, FP32 factors) and the batched FP32 solve.

Workload ``c2``: the 20,176-facet jittered cylinder, plain FP32 H-solve.

Prints ONE JSON line on stdout (progress goes to stderr).

Workload ``fe``: the finite-element coupling (Sec. 3.1-3.4), implicit Euler
steps of a conducting 20,480-facet ellipsoid shell with cavity radiation.

Workload ``hlu``: the hierarchical block LU (Sec. 5.1-5.2) of four
geometries up to a 4,992-facet cylinder, factor and solve times beside a
GMRES solve of the same system.

Workload ``open``: the 13-sphere spiral at 37,440 facets as an open cavity
(isolated facets, fully pivoted ACA, the ambient exchange of eq. (35)) with
the headline's solver.

Default (``--workload all``): the ``c3`` record is the headline; the ``c4``
transient, ``c5`` serving, ``fe`` coupling, ``hlu`` and ``open`` records ride
along on the same JSON line (keys ``c4_transient``, ``c5_serving``,
``fe_coupling``, ``block_lu`` and ``open_spiral``), each with its own value,
roofline or latency figures and oracle baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload all|c3|c2|c4|c5|fe|hlu|open]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "H-matvec % HBM peak; radiosity solves/s vs plain FP32 H-solve at 1e-6 rel err"
RTOL = 1e-7            # residual target; with cond(C) ~ 5 a solve error below 1e-6
IR_INNER = 2e-4        # inner tolerance of each refinement step (2 outer steps on the 64-cavity batch)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count()


def _best_of(fn, reps=3):
    """Runs fn once as a warm-up, then `reps` times; the shortest time and the
    last result."""
    fn()
    best, out = 1e30, None
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        best = min(best, time.perf_counter() - t0)
    return best, out


def cpu_baseline_dense(samples, sizes):
    """The oracle (numpy/scipy FP64) timed on sample cavities of the workload,
    each component after a warm-up as the best of three: dense centroid-rule
    F (eq. (10)), LU of the reflection system with g = F C^-1 eps, and J and
    q of eq. (12) for one right-hand side.  Each component of the largest
    sample is scaled to every cavity by its order (assembly and the
    triangular solves by n^2, the factorisation by n^3).  Returns solves per
    second for one right-hand side per cavity of the whole workload."""
    from oracle import geometry, radiosity, viewfactor
    parts = []
    for cav in samples:
        c, nrm, area = geometry.facets_from_triangles(cav.v, cav.tri)
        t_asm, F = _best_of(lambda: viewfactor.view_factor_matrix(c, nrm, area))
        t_lu, rad = _best_of(lambda: radiosity.DenseRadiosity(F, cav.eps))
        t_sol, _ = _best_of(lambda: rad.flux(cav.T[:, 0], rad.radiosity(cav.T[:, 0])))
        parts.append({"cavity": cav.name, "n": int(area.size), "assembly_s": t_asm, "lu_and_g_s": t_lu,
                      "solve_and_flux_s": t_sol, "solves_per_s": 1.0 / (t_asm + t_lu + t_sol)})
        del F, rad
    ref = max(parts, key=lambda p: p["n"])
    ns = ref["n"]
    total = sum(ref["assembly_s"] * (n / ns) ** 2 + ref["lu_and_g_s"] * (n / ns) ** 3
                + ref["solve_and_flux_s"] * (n / ns) ** 2 for n in sizes)
    return {"value": len(sizes) / total if total > 0 else None, "unit": "solves/s", "cores": _blas_threads(),
            "kind": "oracle",
            "sample": "dense FP64 oracle on %s (warm-up, then best of 3 per component: assembly, LU + g, J + q); "
                      "the %d-facet cavity's components scaled to the %d cavities (assembly and solves "
                      "x(n/%d)^2, LU x(n/%d)^3)" % (", ".join(p["cavity"] for p in parts), ns, len(sizes), ns, ns),
            "components": parts, "seconds_per_step": total}


def roofline(prof, bytes_total_lim=1 << 30):
    k1 = (prof["bytes_phase1"] / 1e6) / prof["ms_phase1"] if prof["ms_phase1"] > 0 else 0.0
    k2 = (prof["bytes_phase2"] / 1e6) / prof["ms_phase2"]
    dom = "k_phase2" if prof["ms_phase2"] >= prof["ms_phase1"] else "k_phase1"
    ach = k2 if dom == "k_phase2" else k1
    tot = (prof["bytes_phase1"] + prof["bytes_phase2"]) / 1e6 / prof["ms_total"]
    return {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None,
            "bytes_per_launch": prof["bytes_phase2"] if dom == "k_phase2" else prof["bytes_phase1"],
            "ms_per_launch": prof["ms_phase2"] if dom == "k_phase2" else prof["ms_phase1"],
            "phase1_GBps": k1, "phase2_GBps": k2,
            "matvec_ms": prof["ms_total"], "matvec_GBps": tot, "matvec_frac": tot / HBM_PEAK_GBS}


KERNEL_SOURCES = ("paper_2305_06891_amd/csrc/matvec.hip", "paper_2305_06891_amd/csrc/dev_common.hpp",
                  "paper_2305_06891_amd/csrc/hm_internal.hpp")
COUNTERS = os.path.join(ROOT, "profiles", "hmatvec_c3_batch_hbm_counters.md")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE summary (calibrated against a plain copy kernel), or None when
    the kernel sources changed since those counters were taken."""
    import hashlib
    try:
        txt = open(COUNTERS).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, s), "rb").read())
    if ("`%s`" % h.hexdigest()[:16]) not in txt:
        return None
    for line in txt.splitlines():
        if line.startswith("traffic_bytes %s:" % kernel):
            return int(line.split(":")[1])
    return None


def copy_ceiling_gbps():
    """Streaming copy b = 1.0 * a of 1 GiB (torch elementwise kernel): bytes
    read + written per second, best of 5 (HIP events)."""
    import torch
    a = torch.ones(256 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    best = 1e30
    for _ in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.mul(a, 1.0, out=b)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return 2 * a.numel() * 4 / 1e6 / best


def base_record(args, value, ms, dtype, config):
    return {"metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def run_c3(args):
    import torch
    from paper_2305_06891_amd import hm
    from workloads import configs

    dev = torch.device("cuda:0")
    cavs = configs.c3_batch()
    sizes = [c.n for c in cavs]
    ctx = hm.Context(0)
    t0 = time.perf_counter()
    trees = []
    for cav in cavs:
        c, nrm, area = hm.hm_facets_from_triangles(cav.v, cav.tri, orient=1)
        trees.append(hm.hm_build_cluster_tree(ctx, c, nrm, area, cav.leaf, cav.eta))
    t_tree = time.perf_counter() - t0
    t0 = time.perf_counter()
    # the batched configuration: all cavities in one assembly call (shared ACA
    # launches, one product split tuned on the batch)
    rc = args.recompress
    Mx = hm.hm_assemble_hmatrix_batched(ctx, trees, [cav.aca_tol for cav in cavs], 256, hm.HM_BF16, hm.HM_F32,
                                        keep_f32_copy=1, autotune=1, recompress=rc, lowrank_rounding=1)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    # the plain configuration: one cavity per call, each tuned alone (the
    # same H-matrix approximation: recompressed as well)
    t0 = time.perf_counter()
    M32 = [hm.hm_assemble_hmatrix(ctx, t, cav.aca_tol, 256, hm.HM_F32, hm.HM_F32, autotune=1, recompress=rc)
           for t, cav in zip(trees, cavs)]
    torch.cuda.synchronize()
    t_asm32 = time.perf_counter() - t0
    stx = [m.stats() for m in Mx]
    ent_d = sum(s["entries_dense"] for s in stx)
    ent_l = sum(s["entries_lowrank"] for s in stx)
    log("c3: %d cavities, %d facets; tree %.2fs; mixed batched assembly %.2fs, fp32 one-by-one assembly %.2fs; "
        "entries dense %d "
        "low-rank %d; device bytes mixed %.2f GB fp32 %.2f GB"
        % (len(cavs), sum(sizes), t_tree, t_asm, t_asm32, ent_d, ent_l,
           sum(s["bytes_device"] for s in stx) / 1e9, sum(m.stats()["bytes_device"] for m in M32) / 1e9))
    eps = [torch.as_tensor(c.eps, device=dev) for c in cavs]
    T = [torch.as_tensor(c.T[:, 0], device=dev) for c in cavs]
    J = [torch.empty_like(t) for t in T]
    q = [torch.empty_like(t) for t in T]

    # --- headline: batched mixed-precision solve (BF16 factors + FP64 refinement)
    pmx = hm.solve_params(rtol=RTOL, restart=30, max_iter=400, mixed_precision=1, ir_inner_rtol=IR_INNER, want_q=1)
    for _ in range(args.warmup):
        hm.hm_solve_radiosity_batched(ctx, Mx, eps, T, hm.SIGMA, pmx, J, q)
    torch.cuda.synchronize()
    step_s = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, _, infos = hm.hm_solve_radiosity_batched(ctx, Mx, eps, T, hm.SIGMA, pmx, J, q)
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / args.steps
    value = len(cavs) * args.steps / dt
    i0 = infos[0]
    worst = max(i["rel_residual"] for i in infos)
    log("batched mixed: %.2f ms/step = %.1f solves/s (median %.2f ms, p90 %.2f ms over %d); outer %d inner %d "
        "matvecs %d worst residual %.2e" % (ms, value, 1e3 * np.median(step_s), 1e3 * np.percentile(step_s, 90),
                                            len(step_s), i0["outer_iters"], i0["iters"], i0["matvecs"], worst))

    # --- batched FP32 (batching gain without the precision gain)
    p32 = hm.solve_params(rtol=RTOL, restart=30, max_iter=400, want_q=1, vec_dtype=hm.HM_F32)
    hm.hm_solve_radiosity_batched(ctx, M32, eps, T, hm.SIGMA, p32, J, q)
    torch.cuda.synchronize()
    nb = max(1, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(nb):
        _, _, infb = hm.hm_solve_radiosity_batched(ctx, M32, eps, T, hm.SIGMA, p32, J, q)
    torch.cuda.synchronize()
    rate_b32 = len(cavs) * nb / (time.perf_counter() - t0)
    log("batched fp32: %.1f solves/s, iters %d" % (rate_b32, infb[0]["iters"]))

    # --- plain FP32 H-solve: one cavity at a time
    for m, e, t, j, qq in zip(M32, eps, T, J, q):
        hm.hm_solve_radiosity(ctx, m, e, t, hm.SIGMA, p32, j, qq)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it_plain = []
    for m, e, t, j, qq in zip(M32, eps, T, J, q):
        _, _, inf = hm.hm_solve_radiosity(ctx, m, e, t, hm.SIGMA, p32, j, qq)
        it_plain.append(inf["iters"])
    torch.cuda.synchronize()
    rate_plain = len(cavs) / (time.perf_counter() - t0)
    log("plain fp32: %.1f solves/s, iters %d..%d" % (rate_plain, min(it_plain), max(it_plain)))

    # --- roofline of the batched product (the inner BF16 product and the FP32 one)
    prof = hm.hm_hmatvec_profile(ctx, Mx, 1, hm.HM_F32, reps=20, flush_bytes=0)
    prof_hi = hm.hm_hmatvec_profile(ctx, Mx, 1, hm.HM_F64, use_f32_copy=True, reps=10, flush_bytes=0)
    prof32 = hm.hm_hmatvec_profile(ctx, M32, 1, hm.HM_F32, reps=10, flush_bytes=0)
    rf = roofline(prof)
    rf["traffic"] = measured_traffic("k_phase2<float, bf16, float, 1, 4>" if rf["kernel"] == "k_phase2"
                                     else "k_phase1<bf16, float, 1, 4>")
    ceil = copy_ceiling_gbps()
    rf["copy_ceiling_GBps"] = ceil
    rf["frac_of_copy_ceiling"] = rf["achieved"] / ceil
    log("profile bf16", prof, "\nprofile hi", prof_hi, "\nprofile fp32", prof32, "\ncopy ceiling %.0f GB/s" % ceil)
    out = base_record(args, value, ms, "f32+f64", {
        "workload": "c3_64_cavities_%d_facets" % sum(sizes), "cavities": len(cavs), "facets": sum(sizes),
        "facets_min": min(sizes), "facets_max": max(sizes), "leaf": 64, "eta": 1.5, "aca_tol": 1e-6,
        "recompression": "truncated svd at aca_tol" if rc else "none",
        "storage": "bf16 low-rank factors (dithered rounding), fp32 near field, fp32 factor copy for the residual",
        "ir_inner_rtol": IR_INNER,
        "solver": "batched gmres(30) fp32 inside fp64 iterative refinement", "rtol": RTOL, "nrhs": 1})
    out["timing"] = {"reps": len(step_s), "median_ms": 1e3 * float(np.median(step_s)),
                     "p90_ms": 1e3 * float(np.percentile(step_s, 90)), "min_ms": 1e3 * float(np.min(step_s)),
                     "median_solves_per_s": len(cavs) / float(np.median(step_s))}
    out["roofline"] = rf
    out["roofline_fp64_residual_product"] = roofline(prof_hi)
    out["roofline_fp32_product"] = roofline(prof32)
    out["plain_fp32"] = {"value": rate_plain, "unit": "solves/s", "iters_min": min(it_plain),
                         "iters_max": max(it_plain)}
    out["batched_fp32"] = {"value": rate_b32, "unit": "solves/s", "iters": infb[0]["iters"]}
    out["speedup_vs_plain_fp32"] = value / rate_plain
    out["speedup_vs_batched_fp32"] = value / rate_b32
    out["solve"] = {"outer_iters": i0["outer_iters"], "inner_iters": i0["iters"], "matvecs": i0["matvecs"],
                    "worst_rel_residual": worst}
    out["matrix"] = {"entries_dense": ent_d, "entries_lowrank": ent_l,
                     "bytes_device_mixed": sum(s["bytes_device"] for s in stx),
                     "n_fallback": sum(s["n_fallback"] for s in stx), "max_rank": max(s["max_rank"] for s in stx)}
    out["tuning"] = Mx[0].tuning()  # one choice for the whole batch
    out["assembly_s"] = {"mixed_batched": t_asm, "fp32_one_by_one": t_asm32, "trees": t_tree}

    # --- the same batch with a BF16 near field too (FP32 copies for the
    # residual): fewer bytes per inner product, at a lower share of HBM peak
    del M32
    Mb = hm.hm_assemble_hmatrix_batched(ctx, trees, [cav.aca_tol for cav in cavs], 256, hm.HM_BF16, hm.HM_BF16,
                                        keep_f32_copy=1, autotune=1, recompress=rc, lowrank_rounding=1)
    for _ in range(args.warmup):
        hm.hm_solve_radiosity_batched(ctx, Mb, eps, T, hm.SIGMA, pmx, J, q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, infm = hm.hm_solve_radiosity_batched(ctx, Mb, eps, T, hm.SIGMA, pmx, J, q)
    torch.cuda.synchronize()
    rate_bn = len(cavs) * args.steps / (time.perf_counter() - t0)
    profb = hm.hm_hmatvec_profile(ctx, Mb, 1, hm.HM_F32, reps=20, flush_bytes=0)
    rb = roofline(profb)
    log("batched mixed, bf16 near field: %.1f solves/s; outer %d inner %d; product %s"
        % (rate_bn, infm[0]["outer_iters"], infm[0]["iters"], profb))
    out["bf16_near_field"] = {"value": rate_bn, "unit": "solves/s", "outer_iters": infm[0]["outer_iters"],
                              "inner_iters": infm[0]["iters"],
                              "worst_rel_residual": max(i["rel_residual"] for i in infm),
                              "matvec_ms": rb["matvec_ms"], "matvec_GBps": rb["matvec_GBps"],
                              "matvec_frac": rb["matvec_frac"]}
    del Mb
    # context: BF16 factors rounded to nearest even (errors of near-equal
    # entries add up coherently; refinement needs a third outer step)
    Me = hm.hm_assemble_hmatrix_batched(ctx, trees, [cav.aca_tol for cav in cavs], 256, hm.HM_BF16, hm.HM_F32,
                                        keep_f32_copy=1, autotune=1, recompress=rc, lowrank_rounding=0)
    for _ in range(args.warmup):
        hm.hm_solve_radiosity_batched(ctx, Me, eps, T, hm.SIGMA, pmx, J, q)
    torch.cuda.synchronize()
    ne = max(1, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(ne):
        _, _, infe = hm.hm_solve_radiosity_batched(ctx, Me, eps, T, hm.SIGMA, pmx, J, q)
    torch.cuda.synchronize()
    rate_e = len(cavs) * ne / (time.perf_counter() - t0)
    out["nearest_even_rounding"] = {"value": rate_e, "unit": "solves/s",
                                    "outer_iters": max(i["outer_iters"] for i in infe),
                                    "worst_rel_residual": max(i["rel_residual"] for i in infe)}
    log("batched mixed, nearest-even bf16 rounding: %.1f solves/s, outer %d"
        % (rate_e, out["nearest_even_rounding"]["outer_iters"]))
    del Me
    if rc:
        # context: the same batch with the ACA crosses as they are
        del Mx
        Mn = hm.hm_assemble_hmatrix_batched(ctx, trees, [cav.aca_tol for cav in cavs], 256, hm.HM_BF16,
                                            hm.HM_F32, keep_f32_copy=1, autotune=1, recompress=0, lowrank_rounding=1)
        for _ in range(args.warmup):
            hm.hm_solve_radiosity_batched(ctx, Mn, eps, T, hm.SIGMA, pmx, J, q)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nn = max(1, args.steps // 2)
        for _ in range(nn):
            hm.hm_solve_radiosity_batched(ctx, Mn, eps, T, hm.SIGMA, pmx, J, q)
        torch.cuda.synchronize()
        rate_n = len(cavs) * nn / (time.perf_counter() - t0)
        profn = roofline(hm.hm_hmatvec_profile(ctx, Mn, 1, hm.HM_F32, reps=10, flush_bytes=0))
        stn = [m.stats() for m in Mn]
        out["without_recompression"] = {"value": rate_n, "unit": "solves/s",
                                        "entries_lowrank": sum(x["entries_lowrank"] for x in stn),
                                        "bytes_device_mixed": sum(x["bytes_device"] for x in stn),
                                        "matvec_ms": profn["matvec_ms"], "matvec_frac": profn["matvec_frac"]}
        log("batched mixed without recompression: %.1f solves/s, product %.3f ms" % (rate_n, profn["matvec_ms"]))
        del Mn
    if not args.no_cpu_baseline:
        samples = [min(cavs, key=lambda c: abs(c.n - t)) for t in (2000, 5000)]
        out["cpu_baseline"] = cpu_baseline_dense(samples, sizes)
    return out


def run_kernels_only(args):
    """Only product kernels and calibration kernels, for profiler runs.

    c3: the 64-cavity batch (assembled with its autotuning), 20 batched
    products with FP32 vectors on the BF16 factors and 10 with FP64 vectors
    on the FP32 factor copy; then 5 elementwise copies of 1 GiB (b = 1.0 * a:
    a streaming kernel of known size that calibrates the HBM byte counters)
    and 5 FP64 elementwise products of 2^26 entries (c = a * b: a kernel of
    known FP64 operation count that calibrates the VALU flop counters).
    c4: the 200,000-facet ellipsoid (FP32), 10 products with 16 right-hand
    sides and FP32 vectors (matrix cores), 10 with 16 and FP64 vectors
    (matrix cores, FP64 sums) and 10 with one."""
    import torch
    from paper_2305_06891_amd import hm
    from workloads import configs

    ctx = hm.Context(0)
    if args.workload == "c4":
        cav = configs.c4_ellipsoid()
        c, nrm, area = hm.hm_facets_from_triangles(cav.v, cav.tri, orient=1)
        t = hm.hm_build_cluster_tree(ctx, c, nrm, area, cav.leaf, cav.eta)
        # the product's work split tuned on 16-column products (the transient's width)
        M = hm.hm_assemble_hmatrix(ctx, t, cav.aca_tol, 256, hm.HM_F32, hm.HM_F32, autotune=16,
                                   recompress=args.recompress)
        torch.cuda.synchronize()
        p16 = hm.hm_hmatvec_profile(ctx, M, 16, hm.HM_F32, reps=10, flush_bytes=0)
        log("16-rhs product x10:", p16)
        p16d = hm.hm_hmatvec_profile(ctx, M, 16, hm.HM_F64, reps=10, flush_bytes=0)
        log("16-rhs fp64 product x10:", p16d)
        p1 = hm.hm_hmatvec_profile(ctx, M, 1, hm.HM_F32, reps=10, flush_bytes=0)
        log("1-rhs product x10:", p1)
        return {"kernels_only": True, "roofline": roofline(p16), "roofline_fp64_16rhs": roofline(p16d),
                "roofline_1rhs": roofline(p1)}
    cavs = configs.c3_batch()
    trees = []
    for cav in cavs:
        c, nrm, area = hm.hm_facets_from_triangles(cav.v, cav.tri, orient=1)
        trees.append(hm.hm_build_cluster_tree(ctx, c, nrm, area, cav.leaf, cav.eta))
    Mx = hm.hm_assemble_hmatrix_batched(ctx, trees, [cav.aca_tol for cav in cavs], 256, hm.HM_BF16, hm.HM_F32,
                                        keep_f32_copy=1, autotune=1, recompress=args.recompress, lowrank_rounding=1)
    torch.cuda.synchronize()
    ev = sum(m.stats()["entries_dense"] for m in Mx)
    log("assembled %d cavities (%d near-field entries)" % (len(Mx), ev))
    prof = hm.hm_hmatvec_profile(ctx, Mx, 1, hm.HM_F32, reps=20, flush_bytes=0)
    log("bf16 product x20:", prof)
    prof_hi = hm.hm_hmatvec_profile(ctx, Mx, 1, hm.HM_F64, use_f32_copy=True, reps=10, flush_bytes=0)
    log("fp32-copy product, fp64 vectors x10:", prof_hi)
    a = torch.ones(256 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    log("copied 5 x %d bytes" % (a.numel() * 4))
    del a, b
    x = torch.full((1 << 26,), 1.5, dtype=torch.float64, device="cuda")
    y = torch.full_like(x, 0.5)
    z = torch.empty_like(x)
    for _ in range(5):
        torch.mul(x, y, out=z)
    torch.cuda.synchronize()
    log("multiplied 5 x %d doubles" % x.numel())
    return {"kernels_only": True, "roofline": roofline(prof), "roofline_fp64_residual_product": roofline(prof_hi),
            "copy_bytes": 1 << 30, "fp64_muls": x.numel()}


def run_c4(args):
    """200,000-facet (4, 2, 1) ellipsoid, 16 scenarios: one step = one
    backward-Euler step of all 16 (diagonal Newton on the lumped balance,
    each iteration a 16-right-hand-side FP32 solve plus an FP64 flux)."""
    import torch
    from paper_2305_06891_amd import hm
    from workloads import configs

    cav = configs.c4_ellipsoid()
    ctx = hm.Context(0)
    t0 = time.perf_counter()
    c, nrm, area = hm.hm_facets_from_triangles(cav.v, cav.tri, orient=1)
    tree = hm.hm_build_cluster_tree(ctx, c, nrm, area, cav.leaf, cav.eta)
    t_tree = time.perf_counter() - t0
    t0 = time.perf_counter()
    # the product's work split tuned on 16-column products (the transient's width)
    M = hm.hm_assemble_hmatrix(ctx, tree, cav.aca_tol, 256, hm.HM_F32, hm.HM_F32, autotune=16,
                               recompress=args.recompress)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    st = M.stats()
    log("c4: matrix", st, "tree %.2fs assembly %.2fs" % (t_tree, t_asm))
    steps = args.c4_steps
    eps = torch.as_tensor(cav.eps, device="cuda")
    T = torch.as_tensor(np.asfortranarray(cav.T), device="cuda")
    src = torch.as_tensor(np.asfortranarray(cav.extra["source"]), device="cuda")
    sp = hm.solve_params(rtol=RTOL, restart=30, max_iter=400, want_q=1, vec_dtype=hm.HM_F32)
    kw = dict(mc=cav.extra["mc"], dt=cav.extra["dt"], newton_rtol=1e-9, params=sp)
    hm.hm_transient_run(ctx, M, eps, T, src, steps=max(1, args.warmup), **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = hm.hm_transient_run(ctx, M, eps, T, src, steps=steps, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    solves = info["newton_total"] * T.shape[1]
    log("c4: %d steps in %.3f s: newton %d (max %d), matvecs %d, residual %.1e"
        % (steps, dt, info["newton_total"], info["newton_max"], info["matvecs"], info["max_rel_residual"]))
    prof = hm.hm_hmatvec_profile(ctx, M, 16, hm.HM_F32, reps=10, flush_bytes=0)
    prof1 = hm.hm_hmatvec_profile(ctx, M, 1, hm.HM_F32, reps=10, flush_bytes=0)
    profd = hm.hm_hmatvec_profile(ctx, M, 16, hm.HM_F64, reps=10, flush_bytes=0)
    log("profile 16 rhs", prof, "\nprofile 16 rhs fp64", profd, "\nprofile 1 rhs", prof1)
    out = base_record(args, solves / dt, 1e3 * dt / steps, "f32+f64", {
        "workload": "c4_ellipsoid_200000_16_scenarios", "facets": cav.n, "scenarios": int(T.shape[1]),
        "leaf": cav.leaf, "eta": cav.eta, "aca_tol": cav.aca_tol, "storage": "fp32",
        "recompression": "truncated svd at aca_tol" if args.recompress else "none",
        "solver": "backward Euler, diagonal Newton; 16-rhs products on the matrix cores: gmres(30) fp32, flux fp64",
        "rtol": RTOL, "newton_rtol": 1e-9, "mc": cav.extra["mc"], "dt": cav.extra["dt"]})
    out["roofline"] = roofline(prof)
    out["roofline_fp64_16rhs"] = roofline(profd)
    out["roofline_1rhs"] = roofline(prof1)
    out["steps"] = steps
    out["steps_per_s"] = steps / dt
    out["transient"] = {k: info[k] for k in ("steps_done", "newton_total", "newton_max", "matvecs",
                                             "max_rel_residual")}
    out["matrix"] = {k: st[k] for k in ("bytes_device", "entries_dense", "entries_lowrank", "max_rank",
                                        "n_dense_blocks", "n_lowrank_blocks", "n_fallback")}
    out["assembly_s"] = t_asm
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_transient(cav.n, info["newton_total"] / max(1, steps))
    return out


def cpu_baseline_serving(samples, cavity_sizes, request_sizes):
    """The oracle serving the same request stream: per cavity id, dense F and
    LU once (then kept, as the server keeps its H-matrices); per right-hand
    side, J and q.  Components timed as in cpu_baseline_dense on sample
    cavities and scaled from the largest by n^2 / n^3.  cavity_sizes: facets
    of every id the stream uses; request_sizes: (facets, right-hand sides) of
    every request.  Returns right-hand sides solved per second."""
    base = cpu_baseline_dense(samples, [])
    ref = max(base["components"], key=lambda p: p["n"])
    ns = ref["n"]
    t_setup = sum(ref["assembly_s"] * (n / ns) ** 2 + ref["lu_and_g_s"] * (n / ns) ** 3 for n in cavity_sizes)
    t_solve = sum(r * ref["solve_and_flux_s"] * (n / ns) ** 2 for n, r in request_sizes)
    rhs = sum(r for _, r in request_sizes)
    return {"value": rhs / (t_setup + t_solve), "unit": "solves/s", "cores": base["cores"], "kind": "oracle",
            "sample": "dense FP64 oracle on %s (warm-up, then best of 3 per component); the %d-facet cavity's "
                      "assembly + LU scaled to each of the %d cavity ids the stream uses (x(n/%d)^2, x(n/%d)^3) "
                      "and its J + q to each of the %d right-hand sides (x(n/%d)^2)"
                      % (", ".join(p["cavity"] for p in base["components"]), ns, len(cavity_sizes), ns, ns, rhs, ns),
            "components": base["components"], "seconds": t_setup + t_solve}


def cpu_baseline_transient(n, newton_per_step):
    """The oracle's transient (dense F, LU, diagonal Newton, 16 scenarios)
    timed on the 4,500-facet member of the same ellipsoid family, scaled to n
    facets: assembly x(n/ns)^2 and LU x(n/ns)^3 once, each Newton iteration
    (16-right-hand-side triangular solves and products, O(n^2)) x(n/ns)^2.
    Returns radiosity solves (right-hand sides) per second over 10 steps."""
    from oracle import geometry, radiosity, transient, viewfactor
    from workloads import configs
    cav = configs.c4_ellipsoid(nu=15, scenarios=16)
    c, nrm, area = geometry.facets_from_triangles(cav.v, cav.tri)
    ns = cav.n
    t0 = time.perf_counter()
    F = viewfactor.view_factor_matrix(c, nrm, area)
    t_asm = time.perf_counter() - t0
    t0 = time.perf_counter()
    rad = radiosity.DenseRadiosity(F, cav.eps)
    t_lu = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, it, _ = transient.newton_step(rad, cav.T, cav.extra["source"], cav.extra["mc"], cav.extra["dt"], tol=1e-9)
    t_step = time.perf_counter() - t0
    per_it = t_step / max(1, it)
    r2, r3 = (n / ns) ** 2, (n / ns) ** 3
    steps = 10
    total = t_asm * r2 + t_lu * r3 + steps * newton_per_step * per_it * r2
    return {"value": steps * newton_per_step * 16 / total, "unit": "solves/s", "cores": _blas_threads(),
            "kind": "oracle",
            "sample": "dense FP64 oracle transient on the %d-facet ellipsoid (assembly %.2f s, LU + g %.2f s, "
                      "one Newton iteration of 16 scenarios %.3f s) scaled to %d facets and 10 steps of %.1f "
                      "Newton iterations" % (ns, t_asm, t_lu, per_it, n, newton_per_step),
            "seconds_per_step": total / steps}


def cpu_baseline_fe(n_facets, n_nodes):
    """The oracle's finite-element step (dense F, R_bar from a dense solve
    with C, dense S, Newton with the exact dense Jacobian) on the 2,000-facet
    member of the same shell family, each part after a warm-up as the best of
    three, scaled to the workload: F x(n/ns)^2, R_bar x(n/ns)^3, S and the
    Newton solves x(nn/nns)^3."""
    from oracle import fe, geometry, viewfactor
    from workloads import configs
    cav = configs.fe_shell(nu=10)
    c, nrm, area = geometry.facets_from_triangles(cav.v, cav.tri)
    ns, nns = cav.n, cav.v.shape[0]
    x = cav.extra
    t_f, F = _best_of(lambda: viewfactor.view_factor_matrix(c, nrm, area))
    t_r, Rb = _best_of(lambda: fe.exchange_matrix(F, cav.eps, area))
    M, K, P = fe.surface_p1(cav.v, cav.tri, x["conductance"], x["capacity"])
    fN = fe.nodal_load(cav.tri, area, x["source"], nns)

    def step():
        S = fe.cavity_operator(P, Rb)
        return fe.newton_step(cav.T[:, 0], x["dt"], M, K, S, fN, tol=1e-10)

    t_s, _ = _best_of(step)
    total = t_f * (n_facets / ns) ** 2 + t_r * (n_facets / ns) ** 3 + t_s * (n_nodes / nns) ** 3
    return {"value": 1.0 / total, "unit": "steps/s", "cores": _blas_threads(), "kind": "oracle",
            "sample": "dense FP64 oracle finite-element step on the %d-facet shell (F %.2f s, R_bar %.2f s, S and "
                      "Newton %.2f s) scaled to %d facets and %d nodes" % (ns, t_f, t_r, t_s, n_facets, n_nodes)}


def run_fe(args):
    """Finite-element coupling (Sec. 3.1-3.4): implicit Euler steps of the
    conducting ellipsoid shell (20,480 facets, 10,242 nodes) with cavity
    radiation, FP64 H-matrix (leaf 64, eta 1.5, ACA 1e-6), Newton-Krylov with
    the sparse part as preconditioner; every step starts from the seeded
    temperatures (the same work each time)."""
    import torch
    from paper_2305_06891_amd import hm
    from workloads import configs

    cav = configs.fe_shell()
    x = cav.extra
    ctx = hm.Context(0)
    c, nrm, area = hm.hm_facets_from_triangles(cav.v, cav.tri, orient=1)
    tree = hm.hm_build_cluster_tree(ctx, c, nrm, area, cav.leaf, cav.eta)
    M = hm.hm_assemble_hmatrix(ctx, tree, cav.aca_tol, 256, hm.HM_F64, hm.HM_F64, recompress=args.recompress)
    dev = torch.device("cuda:0")
    eps = torch.as_tensor(cav.eps, device=dev)
    p = hm.fe_params(x["conductance"], x["capacity"], x["dt"], newton_rtol=1e-10, krylov_rtol=1e-8, pc_rtol=1e-10,
                     solve=hm.solve_params(rtol=1e-12, restart=30, max_iter=600))
    obj = hm.hm_fe_create(ctx, M, cav.v, cav.tri, eps, p)
    T0 = torch.as_tensor(np.ascontiguousarray(cav.T[:, 0]), device=dev)
    src = torch.as_tensor(x["source"], device=dev)
    T1, info = obj.step(T0, src)  # warm-up
    torch.cuda.synchronize()
    steps = 3
    t0 = time.perf_counter()
    for _ in range(steps):
        T1, info = obj.step(T0, src)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    # the heat content changes only by the sources (any size): sum_N (M (T1 - T0))_N / dt = sum_i A_i f_i
    q_load = obj.cavity_load(T1)
    torch.cuda.synchronize()
    a = np.asarray(area)
    nodes = cav.v.shape[0]
    out = {"metric": "finite-element implicit Euler steps/s (conduction + cavity radiation)", "value": 1.0 / sec,
           "unit": "steps/s", "ms_per_step": 1e3 * sec, "steps": steps, "dtype": "f64",
           "config": {"workload": cav.name, "facets": cav.n, "nodes": nodes, "leaf": cav.leaf, "eta": cav.eta,
                      "aca_tol": cav.aca_tol, "conductance": x["conductance"], "capacity": x["capacity"],
                      "dt": x["dt"], "newton_rtol": 1e-10, "cavity_solve_rtol": 1e-12},
           "step": info,
           "ms_per_cavity_solve_upper_bound": 1e3 * sec / max(1, info["cavity_solves"]),
           "radiation_load_sum_rel": float(abs(q_load.sum().item()) / torch.linalg.norm(q_load).item()),
           "source_power_W": float((a * x["source"]).sum())}
    log("fe: %.1f ms/step; %s" % (1e3 * sec, info))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_fe(cav.n, nodes)
    obj.close()
    return out


def run_hlu(args):
    """Hierarchical block LU (Sec. 5.1) and its substitutions (Sec. 5.2),
    FP64, eps_rel 1e-6: factor and solve times of four geometries, the
    largest being a 4,992-facet cylinder (leaf 64), beside the time of a
    GMRES solve of the same system on the H-matvec; value = factorisations
    per second of the cylinder.  The oracle's block LU (plain numpy) is
    timed on the 1,280-facet ellipsoid, the same case as the first row."""
    import torch
    from paper_2305_06891_amd import hm
    from workloads import configs, meshes

    ctx = hm.Context(0)
    dev = torch.device("cuda:0")
    cases = []
    v, f = meshes.ellipsoid(8, (3.0, 2.0, 1.0))
    cases.append(("ellipsoid_1280", v, meshes.inward(f), 32, 0))
    sp = configs.fibonacci_spiral(nu=3)
    cases.append(("spiral_13_spheres_%d" % sp.n, sp.v, sp.tri, 32, 1))
    v, f = meshes.ellipsoid(12, (3.0, 2.0, 1.0))
    cases.append(("ellipsoid_2880", v, meshes.inward(f), 32, 0))
    v, f = meshes.cylinder_for_count(5000, seed=3)
    cases.append(("cylinder_%d" % f.shape[0], v, meshes.inward(f), 64, 0))
    rows = []
    warm = True
    for name, v, f, leaf, pivot in cases:
        n = f.shape[0]
        eps_h = np.random.default_rng(1).uniform(0.1, 0.9, n)
        eps = torch.as_tensor(eps_h, device=dev)
        c, nrm, area = hm.hm_facets_from_triangles(v, f, orient=1)
        tree = hm.hm_build_cluster_tree(ctx, c, nrm, area, leaf, 1.5)
        if warm:  # first launches of every kernel
            hm.hm_hlu_factor(ctx, tree, eps, aca_tol=1e-6, aca_pivot=pivot)
            warm = False
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        LU = hm.hm_hlu_factor(ctx, tree, eps, aca_tol=1e-6, aca_pivot=pivot)
        torch.cuda.synchronize()
        t_f = time.perf_counter() - t0
        st = LU.stats()
        b = torch.ones(n, dtype=torch.float64, device=dev)
        LU.solve(b)
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            LU.solve(b)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        # the same system by GMRES on the FP64 H-matvec (assembled at the same tolerance)
        M = hm.hm_assemble_hmatrix(ctx, tree, 1e-6, 256, hm.HM_F64, hm.HM_F64, aca_pivot=pivot)
        T = torch.as_tensor(np.full(n, 800.0), device=dev)
        p = hm.solve_params(rtol=1e-10, want_q=0)
        hm.hm_solve_radiosity(ctx, M, eps, T, params=p)
        torch.cuda.synchronize()
        tg = []
        for _ in range(5):
            t0 = time.perf_counter()
            hm.hm_solve_radiosity(ctx, M, eps, T, params=p)
            torch.cuda.synchronize()
            tg.append(time.perf_counter() - t0)
        rows.append({"case": name, "n": n, "leaf": leaf, "full_pivot_aca": pivot, "factor_s": t_f,
                     "solve_ms": 1e3 * float(np.median(ts)), "entries": st["entries"], "dense_entries": n * n,
                     "max_rank": st["max_rank"], "gmres_solve_ms": 1e3 * float(np.median(tg))})
        log("hlu: %s n %d factor %.2f s, solve %.2f ms, entries %d (dense %d), GMRES %.2f ms"
            % (name, n, t_f, rows[-1]["solve_ms"], st["entries"], n * n, rows[-1]["gmres_solve_ms"]))
        del LU, M
    cyl = rows[-1]
    out = {"metric": "block-LU factorisations/s (FP64, eps_rel 1e-6)", "value": 1.0 / cyl["factor_s"],
           "unit": "factorisations/s", "dtype": "f64",
           "config": {"workload": cyl["case"], "facets": cyl["n"], "leaf": 64, "eta": 1.5, "eps_rel": 1e-6},
           "cases": rows}
    if not args.no_cpu_baseline:
        from oracle import geometry, hlu as ohlu
        v, f = meshes.ellipsoid(8, (3.0, 2.0, 1.0))
        f = meshes.inward(f)
        eps_h = np.random.default_rng(1).uniform(0.1, 0.9, f.shape[0])
        cg, ng, ag = geometry.facets_from_triangles(v, f)

        def factor():
            root, _ = ohlu.build_reflection(cg, ng, ag, eps_h, 32, 1.5, 1e-6)
            ohlu.factorize(root, 1e-6)

        t_o, _ = _best_of(factor, reps=2)
        out["cpu_baseline"] = {"value": 1.0 / t_o, "unit": "factorisations/s", "cores": _blas_threads(),
                               "kind": "oracle",
                               "sample": "the oracle's block LU (assembly of the blocks + factorisation) of the "
                                         "1,280-facet ellipsoid, warm-up then best of 2; the GPU factors it in "
                                         "%.2f s" % rows[0]["factor_s"]}
    return out


def run_c5(args):
    """Serving: a stream of radiosity-solve requests on 256 cavity ids
    (1k-100k facets, Zipf 1.1 over ids, 1-8 right-hand sides), BF16 factors
    + FP64 refinement to a residual of 1e-7, resident H-matrices admitted by
    a 64 GB budget, continuous batching.  First a closed-loop burst (all
    requests at once, after a warm-up that assembles the popular cavities)
    measures the saturation rate; then Poisson arrivals at 0.5, 0.8 and 0.95
    of it give the latency percentiles.  value = right-hand sides solved per
    second at saturation."""
    import torch
    from paper_2305_06891_amd import hm
    from workloads import configs

    nreq = args.c5_requests
    seed = 5999
    budget_gb = args.c5_budget_gb
    ctx = hm.Context(0)
    p = hm.solve_params(rtol=RTOL, restart=30, max_iter=400, mixed_precision=1, ir_inner_rtol=IR_INNER, want_q=1)
    srv = hm.Server(ctx, hbm_budget_bytes=int(budget_gb * (1 << 30)), max_active=64, max_rhs_per_slot=8, params=p)
    # the request streams (arrival order, ids, nrhs) of every phase
    _, ids_all, nrhs_all = configs.c5_requests(nreq * 5, 1.0, seed=seed)
    t0 = time.perf_counter()
    sizes = {}
    for cid in range(256):
        cav = configs.c5_cavity(cid)
        c, nrm, area = hm.hm_facets_from_triangles(cav.v, cav.tri, orient=1)
        tree = hm.hm_build_cluster_tree(ctx, c, nrm, area, cav.leaf, cav.eta)
        srv.register_cavity(cid, tree, cav.eps, aca_tol=cav.aca_tol, lowrank_dtype=hm.HM_BF16,
                            dense_dtype=hm.HM_F32, keep_f32_copy=1, lowrank_rounding=1)
        sizes[cid] = cav.n
    log("c5: registered %d cavity ids (%d-%d facets) in %.1f s" % (len(sizes), min(sizes.values()),
                                                                    max(sizes.values()), time.perf_counter() - t0))

    def temps(k):
        cid, nr = int(ids_all[k]), int(nrhs_all[k])
        return cid, configs.request_temperatures(sizes[cid], nr, seed, k)

    seen = set()  # cavity ids requested so far (first requests on an id find it cold)

    def run_phase(first, count, arrivals):
        """Submit requests first..first+count-1 at the given arrival offsets
        (None: all at once); returns (elapsed s, latencies s, rhs, statuses,
        cold flags: the request was the first on its cavity id, whose
        H-matrix is assembled on arrival)."""
        reqs = [temps(first + k) for k in range(count)]
        lat, rhs, sts, cold = [], 0, [], []
        pending = {}
        t_start = time.perf_counter()
        i = 0
        while i < count or pending:
            now = time.perf_counter() - t_start
            while i < count and (arrivals is None or arrivals[i] <= now):
                cid, T = reqs[i]
                tk, shape = srv.submit(cid, T)
                pending[tk] = (shape, cid not in seen)
                seen.add(cid)
                i += 1
            for tk in list(pending):
                shape, c = pending[tk]
                r = srv.poll(tk, shape)
                if r is not None:
                    lat.append(r[2]["latency"])
                    rhs += shape[1]
                    sts.append(r[2]["rel_residual"])
                    cold.append(c)
                    del pending[tk]
            time.sleep(0.0002)
        return time.perf_counter() - t_start, np.array(lat), rhs, sts, np.array(cold, dtype=bool)

    # warm-up: assembles the cavities of the first requests
    t_w, _, _, _, _ = run_phase(0, nreq // 2, None)
    st0 = srv.stats()
    log("c5: warm-up %d requests in %.1f s; %s" % (nreq // 2, t_w, st0))
    el, lat, rhs, res, _ = run_phase(nreq // 2, nreq, None)
    sat_req = nreq / el
    sat_rhs = rhs / el
    log("c5: saturation %.1f requests/s, %.1f solves/s (p50 %.1f ms, p99 %.1f ms; worst residual %.1e)"
        % (sat_req, sat_rhs, 1e3 * np.percentile(lat, 50), 1e3 * np.percentile(lat, 99), max(res)))
    loads = []
    first = nreq // 2 + nreq
    for frac in (0.5, 0.8, 0.95):
        rate = frac * sat_req
        gaps = np.random.default_rng([seed, int(1000 * frac)]).exponential(1.0 / rate, nreq)
        el, lat, rhs, res, cold = run_phase(first, nreq, np.cumsum(gaps))
        first += nreq
        warm = lat[~cold]
        loads.append({"load": frac, "offered_req_per_s": rate, "achieved_req_per_s": nreq / el,
                      "solves_per_s": rhs / el, "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                      "p99_ms": 1e3 * float(np.percentile(lat, 99)), "worst_rel_residual": float(max(res)),
                      # requests on cavities already requested (resident) and first requests on a new id
                      "resident_p50_ms": 1e3 * float(np.percentile(warm, 50)) if warm.size else None,
                      "resident_p99_ms": 1e3 * float(np.percentile(warm, 99)) if warm.size else None,
                      "cold_requests": int(cold.sum()),
                      "cold_p50_ms": 1e3 * float(np.percentile(lat[cold], 50)) if cold.any() else None})
        log("c5: load %.2f: %s" % (frac, loads[-1]))
    st = srv.stats()
    srv.close()
    log("c5: server stats %s" % st)
    out = base_record(args, sat_rhs, 1e3 / sat_req, "f32+f64", {
        "workload": "c5_serving_256_ids", "cavity_ids": 256, "ids_used": len(sizes), "zipf_s": 1.1,
        "facets_range": [min(sizes.values()), max(sizes.values())], "rhs_per_request": "1-8",
        "hbm_budget_gb": budget_gb, "storage": "bf16 low-rank factors, fp32 near field, fp32 factor copy",
        "solver": "continuous batching, fp64 refinement rounds with batched fp32 gmres", "rtol": RTOL,
        "requests_per_phase": nreq})
    out["unit"] = "solves/s"
    out["saturation"] = {"req_per_s": sat_req, "solves_per_s": sat_rhs}
    out["latency"] = loads
    out["server"] = st
    if not args.no_cpu_baseline:
        reqs = [(sizes[int(ids_all[k])], int(nrhs_all[k])) for k in range(len(ids_all))]
        used = sorted(set(int(i) for i in ids_all))
        samples = [configs.c5_cavity(c) for c in (3, 0)]  # 2,000 and 5,120 facets
        for cav in samples:
            cav.T = configs.request_temperatures(cav.n, 1, seed, 0)
        out["cpu_baseline"] = cpu_baseline_serving(samples, [sizes[c] for c in used], reqs)
    return out


def run_c2(args):
    import torch
    from paper_2305_06891_amd import hm
    from workloads import configs

    dev = torch.device("cuda:0")
    cav = configs.c2_cylinder()
    n = cav.n
    ctx = hm.Context(0)
    t0 = time.perf_counter()
    c, nrm, area = hm.hm_facets_from_triangles(cav.v, cav.tri, orient=1)
    tree = hm.hm_build_cluster_tree(ctx, c, nrm, area, cav.leaf, cav.eta)
    t_tree = time.perf_counter() - t0
    t0 = time.perf_counter()
    M = hm.hm_assemble_hmatrix(ctx, tree, cav.aca_tol, 256, hm.HM_F32, hm.HM_F32, autotune=1)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    st = M.stats()
    log("matrix", st, "tree %.2fs assembly %.2fs" % (t_tree, t_asm), "tuning", M.tuning())
    eps = torch.as_tensor(cav.eps, device=dev)
    T = torch.as_tensor(cav.T[:, 0], device=dev)
    p = hm.solve_params(rtol=RTOL, restart=30, max_iter=300, want_q=1, vec_dtype=hm.HM_F32)
    J = torch.empty_like(T)
    q = torch.empty_like(T)
    for _ in range(args.warmup):
        hm.hm_solve_radiosity(ctx, M, eps, T, hm.SIGMA, p, J, q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, info = hm.hm_solve_radiosity(ctx, M, eps, T, hm.SIGMA, p, J, q)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / args.steps
    log("solve: %.3f ms/step, iters %d, matvecs %d, rel residual %.2e" %
        (ms, info["iters"], info["matvecs"], info["rel_residual"]))
    # the 300 MB product fits the 256 MB last-level cache in part: flush it
    prof = hm.hm_hmatvec_profile(ctx, M, 1, hm.HM_F32, reps=20, flush_bytes=512 << 20)
    log("profile", prof)
    out = base_record(args, args.steps / dt, ms, "f32", {
        "workload": cav.name, "facets": n, "leaf": cav.leaf, "eta": cav.eta, "aca_tol": cav.aca_tol,
        "storage": "fp32", "solver": "plain FP32 H-solve, gmres(30) fp32 vectors, fp64 dots", "rtol": RTOL,
        "nrhs": 1})
    out["roofline"] = roofline(prof)
    out["matrix"] = {k: st[k] for k in ("bytes_device", "entries_dense", "entries_lowrank", "max_rank",
                                        "n_dense_blocks", "n_lowrank_blocks", "n_fallback")}
    out["tuning"] = M.tuning()
    out["assembly_s"] = t_asm
    out["solve"] = {"iters": info["iters"], "matvecs": info["matvecs"], "rel_residual": info["rel_residual"]}
    if not args.no_cpu_baseline:
        from workloads import meshes
        from workloads.configs import Cavity
        v, f = meshes.cylinder_for_count(5000, seed=1)
        rng = np.random.default_rng(2)
        nf = f.shape[0]
        sample = Cavity("cylinder_%d" % nf, v, meshes.inward(f), rng.uniform(0.1, 0.9, nf),
                        rng.uniform(300, 1500, (nf, 1)))
        out["cpu_baseline"] = cpu_baseline_dense(sample, [n])
    return out


def run_open(args):
    """The 13-sphere spiral of Sec. 6 at its finest mesh level (frequency-12
    spheres, 37,440 facets) as an open, non-convex cavity: isolated facets
    (zero rows of F), fully pivoted ACA at 1e-6 (partial pivoting misses
    parts of this geometry's blocks), recompressed crosses, BF16 factors
    with an FP32 copy, and the ambient exchange of eq. (35) in the flux.
    One step is one radiosity solve (J and q, one right-hand side) with the
    headline's solver: FP32 GMRES on the BF16 factors inside FP64
    refinement to a residual of 1e-7.  Parity of the same settings against
    the dense oracle is tested on the 9,360-facet member of the family."""
    import torch
    from paper_2305_06891_amd import hm
    from workloads import configs

    dev = torch.device("cuda:0")
    cav = configs.fibonacci_spiral(nu=12)
    n = cav.n
    T_amb = cav.extra["T_amb"]
    ctx = hm.Context(0)
    t0 = time.perf_counter()
    c, nrm, area = hm.hm_facets_from_triangles(cav.v, cav.tri, orient=1)
    tree = hm.hm_build_cluster_tree(ctx, c, nrm, area, 64, 1.5)
    t_tree = time.perf_counter() - t0
    t0 = time.perf_counter()
    M = hm.hm_assemble_hmatrix(ctx, tree, 1e-6, 256, hm.HM_BF16, hm.HM_F32, keep_f32_copy=1, autotune=1,
                               recompress=1, aca_pivot=1, lowrank_rounding=1)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    st = M.stats()
    log("open spiral: %d facets, matrix %s, tree %.2fs assembly %.2fs" % (n, st, t_tree, t_asm))
    eps = torch.as_tensor(cav.eps, device=dev)
    T = torch.as_tensor(cav.T[:, 0], device=dev)
    p = hm.solve_params(rtol=RTOL, restart=30, max_iter=400, mixed_precision=1, ir_inner_rtol=IR_INNER, want_q=1,
                        open_cavity=1, ambient_temperature=T_amb)
    J = torch.empty_like(T)
    q = torch.empty_like(T)
    for _ in range(args.warmup):
        hm.hm_solve_radiosity(ctx, M, eps, T, hm.SIGMA, p, J, q)
    torch.cuda.synchronize()
    times = []
    info = None
    for _ in range(args.steps):
        t0 = time.perf_counter()
        _, _, info = hm.hm_solve_radiosity(ctx, M, eps, T, hm.SIGMA, p, J, q)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    total = sum(times)
    ms = 1e3 * total / len(times)
    log("open spiral solve: %.3f ms/step (median %.3f), outer %d inner %d, rel residual %.2e" %
        (ms, 1e3 * float(np.median(times)), info["outer_iters"], info["iters"], info["rel_residual"]))
    prof = hm.hm_hmatvec_profile(ctx, M, 1, hm.HM_F32, reps=20, flush_bytes=512 << 20)
    out = base_record(args, len(times) / total, ms, "f32+f64", {
        "workload": "open_spiral_%d" % n, "facets": n, "spheres": 13, "leaf": 64, "eta": 1.5, "aca_tol": 1e-6,
        "aca": "full pivoting", "recompression": "truncated svd at aca_tol",
        "storage": "bf16 low-rank factors (dithered rounding), fp32 near field, fp32 factor copy for the residual",
        "solver": "gmres(30) fp32 inside fp64 iterative refinement", "rtol": RTOL, "ir_inner_rtol": IR_INNER,
        "open_cavity": True, "ambient_temperature_K": T_amb, "nrhs": 1})
    out["metric"] = "open-cavity radiosity solves/s (13-sphere spiral, ambient exchange)"
    out["timing"] = {"reps": len(times), "median_ms": 1e3 * float(np.median(times)),
                     "p90_ms": 1e3 * float(np.percentile(times, 90))}
    out["roofline"] = roofline(prof)
    out["matrix"] = {k: st[k] for k in ("bytes_device", "entries_dense", "entries_lowrank", "max_rank",
                                        "n_dense_blocks", "n_lowrank_blocks", "n_fallback")}
    out["assembly_s"] = {"trees": t_tree, "full_pivot_aca_and_recompression": t_asm}
    out["solve"] = {"outer_iters": info["outer_iters"], "inner_iters": info["iters"], "matvecs": info["matvecs"],
                    "rel_residual": info["rel_residual"]}
    if not args.no_cpu_baseline:
        sample = configs.fibonacci_spiral(nu=5)
        out["cpu_baseline"] = cpu_baseline_dense([sample], [n])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50, help="timed batched solves of the 64-cavity workload")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="all", choices=["all", "c3", "c2", "c4", "c5", "fe", "hlu", "open"],
                    help="all: the 64-cavity batch (the headline record) with the transient and serving "
                         "records attached to the same line")
    ap.add_argument("--recompress", type=int, default=1, choices=[0, 1],
                    help="truncated-SVD recompression of the ACA crosses (c3, c4)")
    ap.add_argument("--c4-steps", type=int, default=20, help="timed backward-Euler steps of the transient")
    ap.add_argument("--c5-requests", type=int, default=1500, help="requests per serving phase")
    ap.add_argument("--c5-budget-gb", type=float, default=48.0,
                    help="device budget of the server (resident H-matrices + solve buffers)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernels-only", action="store_true",
                    help="profiling aid: only the batched product kernels and a calibration copy, no solves")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the multi-GPU path (row clusters sharded by stored bytes with an "
              "all-gather of x per product, or whole cavities per GPU) is a design, not built here",
              file=sys.stderr)
        sys.exit(2)
    if args.kernels_only:
        out = run_kernels_only(args)
    elif args.workload == "all":
        out = run_c3(args)
        import gc
        gc.collect()
        out["c4_transient"] = run_c4(args)
        gc.collect()
        out["c5_serving"] = run_c5(args)
        gc.collect()
        out["fe_coupling"] = run_fe(args)
        gc.collect()
        out["block_lu"] = run_hlu(args)
        gc.collect()
        out["open_spiral"] = run_open(args)
    else:
        out = {"c3": run_c3, "c2": run_c2, "c4": run_c4, "c5": run_c5, "fe": run_fe,
               "hlu": run_hlu, "open": run_open}[args.workload](args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
