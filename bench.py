"""Benchmark of the multiple-scattering hot path on one MI355X.

Default line (the batched multi-right-hand-side workload, the largest that the
headline metric is quoted on): M = 1000 disks, radii U[0.3, 1] placed by seeded
rejection in [0,150]^2 with edge gap 0.1, k = 10, N_p = ceil(k a_p) + 10
(34,932 complex128 unknowns), 256 incidence angles.

One step = one operator apply A = D^-1 L on all 256 columns (the metric's
complex unknown.RHS matvecs), inputs resident in HBM: input scale, forward
transforms and per-frequency FP64-MFMA products of the well-separated pairs
(circulant-embedded form), the close pairs on the MFMA work queue, output pass.
value = N_tot * R / (mean step time).  Also printed: the phase times of the
timed applies (HIP events on the launch stream), the roofline of the dominant
kernel (the per-frequency products), time-to-1e-8 of the whole 256-column
solve (tables + right-hand sides + s-step GMRES(30), s = 15), the direct form's
apply time, the one-RHS workload's step (tables + GMRES(50) to 1e-8 + far
field), and the CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu-baseline] [--no-solve]
    python bench.py --workload one_rhs | uneven | differentiation | dort | formulations |
                               nearfield | penetrable      (documentation runs)
    python bench.py --workload multi_rhs_block [--block-sizes 16,8] [--sstep-sizes 15,10]
                               (the 256-column solve by lockstep, block and s-step GMRES)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_apply_one_rhs_traffic.txt")
SOLVE_SSTEP = 15   # Newton vectors per block of the 256-column solve
APPLY_SRC = [os.path.join(ROOT, "paper_1409_8186_amd", "csrc", f)
             for f in ("matvec.hip", "common.h", "tables.hip")]
CIRC_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_circ_gemm_multi_rhs_traffic.txt")
CIRC_SRC = [os.path.join(ROOT, "paper_1409_8186_amd", "csrc", f)
            for f in ("circulant.hip", "common.h")]


def measured_peaks(achieved, kind="fp64_fma"):
    """The same rate against what this device reaches on a plain loop of the
    dominant instruction (FP64 FMA or FP64 MFMA), and its copy bandwidth."""
    from paper_1409_8186_amd import probe
    peak = probe(kind)
    return {"peak_measured": peak, "frac_of_measured": achieved / peak,
            "peak_measured_kind": kind + " loop (mudiff_probe)",
            "copy_GBps_measured": probe("copy", 1 << 30)}


def apply_source_sha(files=None):
    """Digest of the sources that define a kernel and its data (default: the
    one-RHS apply)."""
    h = hashlib.sha256()
    for f in files or APPLY_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def algorithmic_flops(n_modes, R=1):
    """8 real flops per complex MAC over every ordered pair: 8 R sum_{p != q} n_p n_q."""
    n = [2 * int(N) + 1 for N in n_modes]
    s = sum(n)
    return 8.0 * R * (s * s - sum(x * x for x in n))


def algorithmic_bytes(n_modes, R=1):
    """Operator data: one H_nu(k b_pq) vector (nu = 0..N_p+N_q) per unordered pair,
    the diagonal factors, and x, y once: 16 B per complex, 8 B per real."""
    N = [int(x) for x in n_modes]
    M = len(N)
    pair = 0
    for p in range(M):
        for q in range(p + 1, M):
            pair += N[p] + N[q] + 1
    ntot = sum(2 * x + 1 for x in N)
    return 16.0 * pair + ntot * (8 + 16) + 2 * 16.0 * R * ntot


def traffic_per_launch(path=TRAFFIC_FILE, files=None):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or None
    if absent or taken on a different revision of the kernel source."""
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    sha = apply_source_sha(files)
    m = re.search(r"source_sha256_16:\s*([0-9a-f]+)", txt)
    f = re.search(r"fetch_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    w = re.search(r"write_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not (m and f and w) or m.group(1) != sha:
        return None
    return float(f.group(1)) + float(w.group(1))


def circ_traffic_per_launch(tile):
    """HBM bytes per launch of the per-frequency product variant `tile`
    (rows, cols, kstep, buffers) from the committed counter summary, or None if
    absent, not measured for that variant, or taken on another source revision."""
    if not os.path.exists(CIRC_TRAFFIC_FILE):
        return None
    txt = open(CIRC_TRAFFIC_FILE).read()
    m = re.search(r"source_sha256_16[^:]*:\s*([0-9a-f]+)", txt)
    if not m or m.group(1) != apply_source_sha(CIRC_SRC):
        return None
    pat = r"variant %dx%d K%d stages %d threads %d products %d .*bytes_per_launch (\d+)" % tuple(tile)
    v = re.search(pat, txt)
    return float(v.group(1)) if v else None


def _blas_threads():
    from threadpoolctl import threadpool_info
    return int(max([d.get("num_threads", 1) for d in threadpool_info()] + [1]))


def cpu_baseline(cl, n_iter_gpu):
    """The oracle on the host: dense assembly of the preconditioned EFIE matrix,
    then oracle GMRES iterations (dense ZGEMV + modified Gram-Schmidt); the
    whole-step rate is extrapolated to the GPU run's iteration count."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import farfield, operator, rhs, solve
    t0 = time.perf_counter()
    L = operator.efie_matrix(cl.centers, cl.radii, cl.n_modes, cl.k)
    D = operator.efie_diagonal(cl.radii, cl.n_modes, cl.k)
    A = operator.preconditioned(L, D)
    del L
    t_asm = time.perf_counter() - t0
    U = rhs.planewave(cl.centers, cl.radii, cl.n_modes, cl.k, cl.betas)[0]
    f = -U / D
    n_sample = 30
    t0 = time.perf_counter()
    x, flag, relres, it, _ = solve.gmres(lambda v: A @ v, f, 50, 1e-30, n_sample)
    t_it = (time.perf_counter() - t0) / it
    t0 = time.perf_counter()
    farfield.farfield(cl.centers, cl.radii, cl.n_modes, cl.k, cl.thetas, x)
    t_ff = time.perf_counter() - t0
    n_app = n_iter_gpu + math.ceil(n_iter_gpu / 50)
    t_step = t_asm + n_app * t_it + t_ff
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    return {
        "value": cl.n_tot * n_app / t_step, "unit": "complex unknown·RHS matvecs/s",
        "cores": int(threads), "kind": "oracle",
        "sample": (f"dense assembly ({t_asm:.1f} s) + {it} oracle GMRES(50) iterations "
                   f"({t_it * 1e3:.1f} ms each: dense ZGEMV + MGS) + far field ({t_ff:.2f} s), "
                   f"extrapolated to the GPU run's {n_iter_gpu} iterations "
                   f"({n_app} applies): oracle step {t_step:.0f} s"),
        "time_to_1e8_s_extrapolated": t_asm + n_app * t_it,
    }


def _segmented_gmres(P, betas, restart, tol, label, seg_cycles=1, max_segments=200, block=0):
    """GMRES(restart) to tol in segments of seg_cycles restart cycles, each
    warm-started from the last (a segment boundary falls on a restart, so the
    iterates are those of one continuous run); progress goes to stderr."""
    import torch
    rho, its, t0 = None, None, time.perf_counter()
    for seg in range(max_segments):
        rho, flag, relres, iters, _ = P.gmres(betas=betas, restart=restart, tol=tol,
                                              maxit=restart * seg_cycles, x0=rho, block=block)
        it = iters.cpu()
        its = it if its is None else its + it
        n_un = int((flag != 0).sum())
        print(f"[{label}] segment {seg}: {time.perf_counter() - t0:.2f} s, unconverged columns "
              f"{n_un}, max relres {float(relres.max()):.2e}", file=sys.stderr, flush=True)
        if n_un == 0:
            break
    torch.cuda.synchronize()
    return rho, flag, its, time.perf_counter() - t0


def embed_len(n_modes):
    """Embedding length of an instance: L_min = 2 (N' + N'') + 1 over its two
    largest orders, or the shortest 2^i 3^j >= L_min (fast transforms) when that
    is at most 128 and at most 1.2 L_min."""
    n = sorted((int(v) for v in n_modes), reverse=True)
    lmin = 2 * (n[0] + n[1]) + 1
    smooth = min(2 ** i * 3 ** j for i in range(9) for j in range(6) if 2 ** i * 3 ** j >= lmin)
    return smooth if smooth <= 128 and 5 * smooth <= 6 * lmin else lmin


def circ_split(insts, R):
    """Work of one batched apply in the form the library runs it: for the
    instances in the circulant form (far-pair work >= half of the direct form's,
    the library's rule), the per-frequency products, 8 R L_b per well-separated
    ordered pair (L_b the embedding length the tables pick, embed_len), and
    their minimal bytes (the
    matrices T_f, 16 L_b M_b^2, and the transformed panels in and out,
    2 x 16 R L_b M_b); and the direct form's 8 R n_p n_q for all other pairs.
    Returns (product flops, product bytes, direct flops, instances in form)."""
    import numpy as np
    prod = direct = pbytes = 0.0
    n_in = 0
    for c in insts:
        N = np.asarray(c.n_modes, dtype=np.int64)
        n = 2 * N + 1
        d = np.hypot(c.centers[:, None, 0] - c.centers[None, :, 0],
                     c.centers[:, None, 1] - c.centers[None, :, 1])
        near = c.k * d < (N[:, None] + N[None, :])
        np.fill_diagonal(near, False)
        w = np.outer(n, n).astype(float)
        np.fill_diagonal(w, 0.0)
        far = ~near
        np.fill_diagonal(far, False)
        L = embed_len(N) if len(N) > 1 else 0
        if L > 0 and (w * far).sum() >= 0.5 * w.sum():
            n_in += 1
            prod += 8.0 * R * L * far.sum()
            pbytes += 16.0 * L * len(N) ** 2 + 2 * 16.0 * R * L * len(N)
            direct += 8.0 * R * (w * near).sum()
        else:
            direct += 8.0 * R * w.sum()
    return prod, pbytes, direct, n_in


def block_workload(base, args):
    """The multi-RHS workload (1,000 disks, 256 incidences) solved to 1e-8 with
    GMRES(30) by lockstep batched GMRES, by block GMRES for each block size in
    --block-sizes and by s-step GMRES for each size in --sstep-sizes (the
    circulant-form apply in every case): time, steps, and the agreement of the
    solutions with lockstep's."""
    import numpy as np
    import torch

    import synth
    from paper_1409_8186_amd import Problem
    cl = synth.multi_rhs()
    R = len(cl.betas)
    betas = cl.betas[None, :]
    P = Problem.from_cluster(cl, circulant=True)
    x = torch.randn(R * cl.n_tot, dtype=torch.complex128, device="cuda")
    P.matvec(x, R=R, op=1)  # forms and tiles timed outside the solves
    torch.cuda.synchronize()
    runs, ref = [], None
    for sb in [0] + [int(v) for v in args.block_sizes.split(",") if v]:
        label = "lockstep" if sb == 0 else f"block {sb}"
        rho, flag, its, t_s = _segmented_gmres(P, betas, 30, 1e-8, label, seg_cycles=10, block=sb)
        r = {"solver": label, "time_s": t_s, "steps_max": int(its.max()), "steps_min": int(its.min()),
             "all_converged": bool((flag == 0).all()), "apply_ms": None}
        if ref is None:
            ref = rho
        else:
            d = (rho - ref).reshape(R, -1)
            r["max_rel_diff_vs_lockstep"] = float((d.norm(dim=1) / ref.reshape(R, -1).norm(dim=1)).max())
        runs.append(r)
        print(f"[bench] {label}: {t_s:.1f} s, steps <= {r['steps_max']}", file=sys.stderr, flush=True)
        del rho
    for ss in [int(v) for v in args.sstep_sizes.split(",") if v]:
        label = f"s-step {ss}"
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rho, flag, _, its, _ = P.gmres(betas=betas, restart=30, tol=1e-8, maxit=20000, sstep=ss)
        torch.cuda.synchronize()
        t_s = time.perf_counter() - t0
        d = (rho - ref).reshape(R, -1)
        runs.append({"solver": label, "time_s": t_s, "steps_max": int(its.max()),
                     "steps_min": int(its.min()), "all_converged": bool((flag == 0).all()),
                     "max_rel_diff_vs_lockstep": float((d.norm(dim=1) / ref.reshape(R, -1).norm(dim=1)).max())})
        print(f"[bench] {label}: {t_s:.1f} s, steps <= {int(its.max())}", file=sys.stderr, flush=True)
        del rho
    t_lock = runs[0]["time_s"]
    best = min(runs, key=lambda r: r["time_s"])
    out = dict(base)
    out.update({"metric": "time-to-1e-8 GMRES solve (all 256 columns)", "value": best["time_s"],
                "unit": "s", "higher_is_better": False, "ms_per_step": best["time_s"] * 1e3,
                "config": {"workload": "multi_rhs, GMRES variants: M=1000 disks, k=10, N_p=ceil(10a)+10, "
                                       "256 incidences, GMRES(30) to 1e-8, lockstep, block GMRES "
                                       "(blocks of consecutive incidences) and s-step GMRES, "
                                       "circulant-form apply",
                           "n_unknowns": cl.n_tot, "R": R, "fastest": best["solver"]},
                "runs": runs,
                "speedup_vs_lockstep": {r["solver"]: t_lock / r["time_s"] for r in runs[1:]}})
    return out


def other_workload(args):
    """Documentation runs of the batched and differentiation workloads: the
    batched apply (phases timed by HIP events) against the FP64 MFMA roofline,
    the batched solve or gradient, the same work one instance at a time on a
    sample, and the oracle on a bounded sample."""
    import numpy as np
    import torch

    import synth
    from paper_1409_8186_amd import Problem
    base = {"n_gpus": 1, "steps": 1, "warmup": 1, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "complex128 (f64)",
            "data": "synthetic (seeded disk clusters)"}

    def apply_roofline(P, R, insts, reps=5):
        n = sum(c.n_tot for c in insts)
        x = torch.randn(R * n, dtype=torch.complex128, device="cuda")
        y = P.empty(R)
        P.matvec(x, R=R, op=1, out=y)       # first call of this R times the forms and tiles
        torch.cuda.synchronize()
        P.profile_begin(reps)
        t0 = time.perf_counter()
        for _ in range(reps):
            P.matvec(x, R=R, op=1, out=y)
        torch.cuda.synchronize()
        t_app = (time.perf_counter() - t0) / reps
        ph = P.profile_end()
        k = ph.pop("applies")
        ph = {key: v / k for key, v in ph.items()}
        cfg = P.apply_config(R)
        prod, pbytes, direct, n_in = circ_split(insts, R)
        if cfg["kind"] == "circulant":
            flops, kt = prod, ph["frequency_products"] / 1e3
            kname = "k_circ_gemm (per-frequency products), tile %s" % (P.circulant_tile(R),)
        else:
            flops, kt = sum(algorithmic_flops(c.n_modes, R) for c in insts), ph["mfma_or_lane"] / 1e3
            pbytes = 0.0
            kname = "k_apply_mfma (direct Toeplitz tiles)"
        # the bound is whichever of the minimal HBM traffic and the FP64 MFMA work
        # takes longer at peak (few right-hand sides: the matrices T_f dominate)
        if pbytes / (PEAK_HBM_GBS * 1e9) > flops / (PEAK_FP64_MFMA_TFLOPS * 1e12):
            r = {"bound": "hbm", "achieved": pbytes / kt / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                 "frac": pbytes / kt / 1e9 / PEAK_HBM_GBS, "algorithmic_bytes_per_launch": pbytes,
                 "flops_TFLOPs": flops / kt / 1e12}
        else:
            r = {"bound": "mfma", "achieved": flops / kt / 1e12, "peak": PEAK_FP64_MFMA_TFLOPS,
                 "unit": "TFLOP/s", "frac": flops / kt / 1e12 / PEAK_FP64_MFMA_TFLOPS}
            r.update(measured_peaks(flops / kt / 1e12, "fp64_mfma"))
        r.update({"traffic": None, "kernel": kname, "kernel_ms": kt * 1e3, "apply": cfg,
                  "algorithmic_flops_per_launch": flops, "instances_in_circulant_form": n_in,
                  "direct_flops_of_close_pairs": direct})
        return t_app, ph, r

    if args.workload == "uneven":
        insts = synth.uneven_instances()
        R = 8
        betas = np.stack([c.betas for c in insts])
        P = Problem.from_clusters(insts, circulant=True)
        n = sum(c.n_tot for c in insts)
        t_app, ph, roof = apply_roofline(P, R, insts, reps=5)
        rho, flag, its, t_s = _segmented_gmres(P, betas, 300, 1e-8, "uneven batched")
        it = its.numpy().reshape(len(insts), R)
        # the same solves one instance at a time, on a seeded sample
        rng = np.random.default_rng(11)
        sample = sorted(rng.choice(len(insts), 16, replace=False).tolist())
        t1 = 0.0
        for b in sample:
            Pb = Problem.from_cluster(insts[b], circulant=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Pb.gmres(betas=betas[b:b + 1], restart=300, tol=1e-8, maxit=20000)
            torch.cuda.synchronize()
            t1 += time.perf_counter() - t0
            Pb.close()
        per_inst_single = t1 / len(sample)
        # the oracle: dense assembly + LU solve of the 8 incidences, same sample
        from oracle import operator as oop, rhs as orhs, solve as osol
        c0 = time.perf_counter()
        for b in sample:
            c = insts[b]
            L = oop.efie_matrix(c.centers, c.radii, c.n_modes, c.k)
            osol.efie_solve_lu(L, orhs.planewave(c.centers, c.radii, c.n_modes, c.k, c.betas))
        t_cpu = (time.perf_counter() - c0) / len(sample) * len(insts)
        return {**base, "metric": "time-to-1e-8 GMRES solve (all instances)", "value": t_s,
                "unit": "s", "higher_is_better": False, "ms_per_step": t_s * 1e3,
                "config": {"workload": "uneven: 512 seeded instances, M~U{10..200}, k~U[1,20], "
                                       "N_p=ceil(k a)+8, R=8, GMRES(300) to 1e-8, all instances "
                                       "in each launch", "unknowns_x_rhs": n * R,
                           "iters_min": int(it.min()), "iters_max": int(it.max()),
                           "all_converged": bool((flag == 0).all())},
                "apply_ms": t_app * 1e3, "apply_rate": n * R / t_app, "phases_ms": ph,
                "roofline": roof,
                "one_at_a_time": {"sample_instances": len(sample),
                                  "mean_s_per_instance": per_inst_single,
                                  "extrapolated_s_all": per_inst_single * len(insts),
                                  "batched_speedup": per_inst_single * len(insts) / t_s},
                "cpu_baseline": {"value": t_cpu, "unit": "s (all instances)", "cores": _blas_threads(),
                                 "kind": "oracle",
                                 "sample": f"oracle dense assembly + LU solve (8 incidences) of the "
                                           f"same {len(sample)} seeded instances, extrapolated by "
                                           f"count to all {len(insts)}"}}
    if args.workload == "multi_rhs_block":
        return block_workload(base, args)
    if args.workload == "dort":
        return dort_workload(base)
    if args.workload == "formulations":
        return formulations_workload(base)
    if args.workload == "nearfield":
        return nearfield_workload(base)
    if args.workload == "penetrable":
        return penetrable_workload(base)
    pairs = synth.differentiation()
    bases = [b for b, _ in pairs]
    betas = np.stack([b.betas for b in bases])
    th = bases[0].thetas
    # targets: far fields of the perturbed geometries (computed on the device)
    tgt_cls = [t for _, t in pairs]
    PT = Problem.from_clusters(tgt_cls)
    rho_t, fl, _, _, _ = PT.gmres(betas=betas, restart=50, tol=1e-10, maxit=20000)
    target = PT.farfield(rho_t, th, R=betas.shape[1]).reshape(betas.shape[0], -1)
    PT.close()

    from paper_1409_8186_amd import _lib as L
    gflags = (L.SSTEP | L.sstep_size(args.grad_sstep)) if args.grad_sstep > 0 else 0

    def step(idx):
        P = Problem.from_clusters([bases[i] for i in idx], circulant=True)
        out = P.grad(betas[idx], th, target[idx].reshape(-1), restart=50, tol=1e-8, maxit=20000,
                     flags=gflags)
        P.close()
        return out
    allidx = list(range(len(bases)))
    step(allidx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step(allidx)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    t1 = 0.0
    for i in range(4):                      # one configuration at a time, sample of 4
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        step([i])
        torch.cuda.synchronize()
        t1 += time.perf_counter() - s0
    P = Problem.from_clusters(bases, circulant=True)
    t_app, ph, roof = apply_roofline(P, betas.shape[1], bases, reps=5)
    # the oracle adjoint gradient of one configuration (dense LU, 64 forward and
    # 64 adjoint solves, chain rule over every factor)
    from oracle import gradient as ograd
    c0 = time.perf_counter()
    ograd.misfit_grad(bases[0].centers, bases[0].radii, bases[0].n_modes, bases[0].k, bases[0].betas,
                      th, target[0].cpu().numpy().reshape(len(bases[0].betas), -1))
    t_cpu = time.perf_counter() - c0
    return {**base, "metric": "adjoint grads/s", "value": len(bases) / t, "unit": "gradients/s",
            "ms_per_step": t * 1e3,
            "config": {"workload": "differentiation: 32 configs, M=100, a~U[0.4,0.8], [0,40]^2, "
                                   "k=8, N_p=ceil(8a)+8, 64 incidences x 64 receivers, forward + "
                                   "adjoint GMRES(50) to 1e-8, gradient w.r.t. 200 center "
                                   "coordinates, 100 radii and k per config",
                       "configs_per_step": len(bases),
                       "solver": (f"s-step GMRES(50), s = {args.grad_sstep}" if args.grad_sstep > 0
                                  else "lockstep GMRES(50)")},
            "apply_ms": t_app * 1e3, "phases_ms": ph,
            "roofline": roof,
            "one_at_a_time": {"sample_configs": 4, "grads_per_s": 4 / t1,
                              "batched_speedup": (len(bases) / t) / (4 / t1)},
            "cpu_baseline": {"value": 1.0 / t_cpu, "unit": "gradients/s", "cores": _blas_threads(),
                             "kind": "oracle",
                             "sample": "oracle adjoint gradient of the first configuration "
                                       f"(dense LU, 64 forward + 64 adjoint solves): {t_cpu:.1f} s"}}


def dort_workload(base):
    """The time-reversal experiment of the paper's Example III (sound-soft): far-field
    mirror matrix F (batched GMRES over the 512 incidences + far field at the 512
    opposite directions), T = conj(F)^T F, its eigen-decomposition, and the
    Herglotz waves of the three leading eigenvectors on a 201 x 201 grid."""
    import numpy as np
    import torch

    import synth
    from paper_1409_8186_amd import Problem, herglotz, tro, tro_eigh
    n_alpha = 512
    cl = synth.dort_example(n_alpha)
    g = np.linspace(-30.0, 30.0, 201)
    grid = np.stack(np.meshgrid(g, g, indexing="ij"), axis=-1).reshape(-1, 2)
    grid_d = torch.tensor(grid, device="cuda")
    al_d = torch.tensor(2.0 * np.pi * np.arange(n_alpha) / n_alpha, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def run():
        t = {}
        s0 = time.perf_counter()
        P = Problem.from_cluster(cl)
        X, flag, relres, iters = P.mirror_farfield(n_alpha, restart=30, tol=1e-12, maxit=2000)
        torch.cuda.synchronize()
        t["farfield_matrix_s"] = time.perf_counter() - s0
        s1 = time.perf_counter()
        T = tro(X)
        torch.cuda.synchronize()
        t["tro_s"] = time.perf_counter() - s1
        s2 = time.perf_counter()
        w, ev, sweeps = tro_eigh(X, tol=1e-13)
        torch.cuda.synchronize()
        t["eigh_s"] = time.perf_counter() - s2
        s3 = time.perf_counter()
        u = herglotz(al_d, ev[:3].contiguous(), cl.k, grid_d)
        torch.cuda.synchronize()
        t["herglotz_s"] = time.perf_counter() - s3
        t["total_s"] = time.perf_counter() - s0
        P.close()
        return t, w, sweeps, int(flag.max()), int(iters.max()), u
    run()
    t, w, sweeps, fmax, itmax, u = run()
    w = w.cpu().numpy()
    # the Jacobi rounds: 128 blocks of 4 columns, 127 rounds a sweep; per launch,
    # 64 workgroups each read and rewrite 8 columns of F (512 complex) and 8 rows
    # of V (512 complex)
    n_blocks = (n_alpha + 3) // 4 + ((n_alpha + 3) // 4) % 2
    launches = sweeps * (n_blocks - 1)
    bytes_round = (n_blocks // 2) * 8 * 2 * (n_alpha + n_alpha) * 16
    # the oracle on the host: dense LU solve, T, LAPACK eigh, Herglotz sums
    from oracle import dort as odort
    c0 = time.perf_counter()
    F = odort.farfield_matrix(cl.centers, cl.radii, cl.n_modes, cl.k, n_alpha)
    wo, Vo = odort.eig_desc(odort.time_reversal(F))
    for j in range(3):
        odort.herglotz(n_alpha, Vo[:, j], cl.k, grid)
    t_cpu = time.perf_counter() - c0
    out = {**base, "metric": "time per DORT experiment", "value": t["total_s"], "unit": "s",
           "higher_is_better": False, "ms_per_step": t["total_s"] * 1e3,
           "config": {"workload": "dort: Example III sound-soft, 3 disks (0,20),(10,-10),(-10,-20), "
                                  "a=0.02,0.01,0.005, k=2pi, N_p=4, 512 mirror cells, GMRES(30) "
                                  "to 1e-12 for 512 incidences, T, one-sided Jacobi eigh (tol "
                                  "1e-13), 3 Herglotz waves on a 201x201 grid over [-30,30]^2",
                      "gmres_iters_max": itmax, "all_converged": fmax == 0,
                      "jacobi_sweeps": sweeps,
                      "eigenvalues_top4": [float(x) for x in w[:4]]},
           "phases_s": t,
           "roofline": {"bound": "hbm", "kernel": "k_jacobi_block_round<2, 256> (one-sided Jacobi round over blocks of 4 columns)",
                        "achieved": bytes_round * launches / t["eigh_s"] / 1e9,
                        "peak": 8000.0, "unit": "GB/s",
                        "frac": bytes_round * launches / t["eigh_s"] / 1e9 / 8000.0,
                        "traffic": None,
                        "note": "includes launch gaps and the per-sweep host check; "
                                "the 8 MB of F and V stay in the last-level cache"},
           "cpu_baseline": {"value": t_cpu, "unit": "s", "cores": _blas_threads(),
                            "kind": "oracle", "sample": "the whole experiment (LU solve, T, "
                            "LAPACK eigh, 3 Herglotz waves)"}}
    return out


def formulations_workload(base):
    """The one-RHS geometry (M=400, N_p=12, k=2 pi, beta=pi/4) solved by every
    formulation (GMRES(50) to 1e-8, single-scattering preconditioner): time,
    iterations, agreement of the far fields (sound-soft forms against the
    EFIE, sound-hard forms against each other), and the one-RHS apply with the
    operator tables."""
    import numpy as np
    import torch

    import synth
    from paper_1409_8186_amd import Problem
    cl = synth.one_rhs()
    th = torch.tensor(cl.thetas, device="cuda")
    beta = [[math.pi / 4]]
    P = Problem.from_cluster(cl)
    res, far = {}, {}
    for name in Problem.FORMULATIONS:
        if name == "efie":
            P.set_operator(None)
        else:
            P.set_operator(name)
        P.gmres(betas=beta, restart=50, tol=1e-8, maxit=20000, graph=True)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rho, flag, relres, iters, _ = P.gmres(betas=beta, restart=50, tol=1e-8, maxit=20000,
                                              graph=True)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        far[name] = P.farfield(rho, th).cpu().numpy()[0]
        x = torch.randn(cl.n_tot, dtype=torch.complex128, device="cuda")
        y = P.empty(1)
        P.matvec(x, op=1, out=y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            P.matvec(x, op=1, out=y)
        e1.record()
        e1.synchronize()
        res[name] = {"solve_s": t, "iters": int(iters[0]), "flag": int(flag[0]),
                     "relres": float(relres[0]), "apply_us": e0.elapsed_time(e1) / 20 * 1e3}
    P.set_operator(None)

    def dev(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))
    for name in ("mfie", "cfie", "bwie"):
        res[name]["farfield_rel_diff_vs_efie"] = dev(far[name], far["efie"])
    res["neumann_dl"]["farfield_rel_diff_vs_neumann_sl"] = dev(far["neumann_dl"], far["neumann_sl"])
    flops = algorithmic_flops(cl.n_modes, 1)
    t_app = res["cfie"]["apply_us"] * 1e-6
    # the oracle: dense CFIE assembly, LU solve and far field on the first 200 disks
    from oracle import operators as oops
    c0 = time.perf_counter()
    oops.solve_farfield("cfie", cl.centers[:200], cl.radii[:200], cl.n_modes[:200], cl.k,
                        [math.pi / 4], cl.thetas, alpha=0.5, eta=1j * cl.k)
    t_cpu = time.perf_counter() - c0
    return {**base, "metric": "time-to-1e-8 GMRES solve per formulation", "value": res["cfie"]["solve_s"],
            "unit": "s (CFIE)", "higher_is_better": False, "ms_per_step": res["cfie"]["solve_s"] * 1e3,
            "config": {"workload": "formulations: one_rhs geometry (M=400, a=0.5, N_p=12, k=2pi, "
                                   "beta=pi/4), GMRES(50) to 1e-8 with graph replay; CFIE alpha=1/2, "
                                   "eta=ik; BWIE eta=ik",
                       "n_unknowns": cl.n_tot},
            "formulations": res,
            "roofline": {"bound": "alu", "kernel": "operator apply with operator tables, one RHS: "
                                                   "k_apply_lane<12, true> + k_apply_finish (CFIE)",
                         "achieved": flops / t_app / 1e12, "peak": PEAK_FP64_VECTOR_TFLOPS,
                         "unit": "TFLOP/s", "frac": flops / t_app / 1e12 / PEAK_FP64_VECTOR_TFLOPS,
                         "traffic": None},
            "cpu_baseline": {"value": t_cpu, "unit": "s per solve", "cores": _blas_threads(),
                             "kind": "oracle",
                             "sample": "dense CFIE assembly + LU solve + far field of the first 200 "
                                       "disks (5,000 unknowns), not the 400-disk solve"}}


def nearfield_workload(base):
    """Total field of the one-RHS solve on a 1000 x 1000 grid over [-5, 65]^2
    (1e6 points x 400 disks), after GMRES(50) to 1e-8."""
    import numpy as np
    import torch

    import synth
    from paper_1409_8186_amd import Problem
    cl = synth.one_rhs()
    P = Problem.from_cluster(cl)
    rho, flag, _, _, _ = P.gmres(betas=[[math.pi / 4]], restart=50, tol=1e-8, maxit=20000, graph=True)
    g = np.linspace(-5.0, 65.0, 1000)
    pts = torch.tensor(np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2), device="cuda")
    P.nearfield(rho, pts, betas=[[math.pi / 4]])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 3
    for _ in range(reps):
        u = P.nearfield(rho, pts, betas=[[math.pi / 4]])
    e1.record()
    e1.synchronize()
    t = e0.elapsed_time(e1) / reps / 1e3
    n_pairs = pts.shape[0] * cl.M
    # per (point, disk): the mode sum, 2N+1 complex MACs, the H_m and phase
    # recurrences (N complex updates each); H_0, H_1 not counted
    N = int(cl.n_modes[0])
    flops_pair = 8 * (2 * N + 1) + 2 * 8 * N
    # the oracle on a sample of 2000 points
    from oracle import nearfield as onf
    sample = pts[:2000].cpu().numpy()
    c0 = time.perf_counter()
    onf.total_field(cl.centers, cl.radii, cl.n_modes, cl.k, rho.cpu().numpy()[None, :], sample,
                    [math.pi / 4])
    t_cpu = (time.perf_counter() - c0) * pts.shape[0] / len(sample)
    return {**base, "metric": "near-field points x disks per second", "value": n_pairs / t,
            "unit": "point-disk evaluations/s", "ms_per_step": t * 1e3,
            "config": {"workload": "nearfield: one_rhs geometry (M=400, N_p=12, k=2pi), total field "
                                   "on a 1000x1000 grid over [-5,65]^2 after GMRES(50) to 1e-8",
                       "points": int(pts.shape[0]), "disks": cl.M,
                       "max_abs_total_field": float(u.abs().max())},
           "roofline": {"bound": "alu", "kernel": "k_nearfield",
                        "achieved": n_pairs * flops_pair / t / 1e12, "peak": PEAK_FP64_VECTOR_TFLOPS,
                        "unit": "TFLOP/s",
                        "frac": n_pairs * flops_pair / t / 1e12 / PEAK_FP64_VECTOR_TFLOPS,
                        "traffic": None,
                        "note": "counts the mode sums and recurrences only; the H_0, H_1 "
                                "evaluation per (point, disk) is not counted"},
           "cpu_baseline": {"value": n_pairs / t_cpu, "unit": "point-disk evaluations/s",
                            "cores": _blas_threads(), "kind": "oracle",
                            "sample": "oracle total field on 2000 of the grid points, extrapolated"}}


def penetrable_workload(base):
    """Penetrable lattice (400 unit disks, k+ = 1, k- = 2, point source at the
    origin): one step = tables + penetrable tables, GMRES(50) to 1e-8 with the
    point-source right-hand side, far field at 720 angles, total field on a
    400 x 400 grid over [-33, 33]^2."""
    import numpy as np
    import torch

    import synth
    from paper_1409_8186_amd import Problem
    cl = synth.penetrable_example()
    k_int = 2.0
    src = [[[0.0, 0.0]]]
    th = torch.tensor(cl.thetas, device="cuda")
    g = np.linspace(-33.0, 33.0, 400)
    pts = torch.tensor(np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2), device="cuda")
    info = {}

    def step():
        P = Problem.from_cluster(cl)
        P.set_penetrable(k_int)
        rho, flag, relres, iters, _ = P.gmres(sources=src, restart=50, tol=1e-8, maxit=20000, graph=True)
        a = P.farfield(rho, th)
        u = P.nearfield(rho, pts, sources=src)
        info.update(P=P, rho=rho, flag=flag, relres=relres, iters=iters, a=a, u=u)

    step()
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    P = info["P"]
    x = torch.randn(cl.n_tot, dtype=torch.complex128, device="cuda")
    y = P.empty(1)
    P.matvec(x, op=1, out=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        P.matvec(x, op=1, out=y)
    e1.record()
    e1.synchronize()
    t_app = e0.elapsed_time(e1) / 20 / 1e3
    flops = algorithmic_flops(cl.n_modes, 1)
    a = info["a"].cpu().numpy()[0]
    rcs = 10 * np.log10(2 * np.pi * np.abs(a) ** 2)
    out = {**base, "metric": "penetrable point-source step time", "value": t, "unit": "s",
           "higher_is_better": False, "ms_per_step": t * 1e3, "steps": reps,
           "config": {"workload": "penetrable: 400 unit disks on a 21x21 lattice of spacing 3 minus "
                                  "the middle row and column, k+=1, k-=2, mu=1, N_p=8, point source "
                                  "at the origin; GMRES(50) to 1e-8 with graph replay, far field at "
                                  "720 angles, total field on 400x400 points",
                      "n_unknowns": cl.n_tot},
           "iterations": int(info["iters"][0]), "flag": int(info["flag"][0]),
           "relres": float(info["relres"][0]), "rcs_db_min_max": [float(rcs.min()), float(rcs.max())],
           "max_abs_total_field": float(info["u"].abs().max()),
           "apply_us": t_app * 1e6,
           "roofline": {"bound": "alu", "kernel": "operator apply with the penetrable tables, one RHS: "
                                                  "k_apply_lane<8, true> + k_apply_finish",
                        "achieved": flops / t_app / 1e12, "peak": PEAK_FP64_VECTOR_TFLOPS,
                        "unit": "TFLOP/s", "frac": flops / t_app / 1e12 / PEAK_FP64_VECTOR_TFLOPS,
                        "traffic": None}}
    # the oracle's dense 2x2 block solve on a 14 x 14 sub-lattice (196 disks)
    from oracle import penetrable as opn, pointsource as ops_
    sub = synth.penetrable_example(half=7)
    c0 = time.perf_counter()
    U = ops_.point_source(sub.centers, sub.radii, sub.n_modes, sub.k, [[0.0, 0.0]])
    dU = ops_.point_source_dn(sub.centers, sub.radii, sub.n_modes, sub.k, [[0.0, 0.0]])
    opn.solve_coefficients(sub.centers, sub.radii, sub.n_modes, sub.k, np.full(sub.M, k_int), U, dU)
    t_cpu = time.perf_counter() - c0
    out["cpu_baseline"] = {"value": t_cpu, "unit": "s per solve", "cores": _blas_threads(), "kind": "oracle",
                           "sample": f"dense block-system solve of a 196-disk sub-lattice "
                                     f"({2 * sub.n_tot} unknowns), not the 400-disk step"}
    return out


def cpu_baseline_multi(cl, R, t_budget=10.0):
    """The oracle on the host for the 256-column apply: dense rows of L (oracle
    row blocks of whole disks) times the 256 input columns (ZGEMM), on the first
    disks until about t_budget seconds of assembly; the apply time is
    extrapolated to all disks by the share of unknowns covered."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import operator
    rng = np.random.default_rng(3)
    X = rng.normal(size=(R, cl.n_tot)) + 1j * rng.normal(size=(R, cl.n_tot))
    blocks, t_asm, rows = [], 0.0, 0
    for p in range(cl.M):
        t0 = time.perf_counter()
        blocks.append(operator.efie_row_block(cl.centers, cl.radii, cl.n_modes, cl.k, p))
        t_asm += time.perf_counter() - t0
        rows += blocks[-1].shape[0]
        if t_asm >= t_budget:
            break
    Lrows = np.concatenate(blocks)
    del blocks
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        Lrows @ X.T
        ts.append(time.perf_counter() - t0)
    t_mm = sorted(ts)[1]
    scale = cl.n_tot / rows
    t_apply = t_mm * scale
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    return {"value": cl.n_tot * R / t_apply, "unit": "complex unknown·RHS matvecs/s",
            "cores": int(threads), "kind": "oracle",
            "sample": (f"oracle dense rows of the first {p + 1} disks ({rows} of "
                       f"{cl.n_tot} unknowns; assembly {t_asm:.1f} s) times the {R} columns "
                       f"(ZGEMM, median of 3: {t_mm:.3f} s), extrapolated by unknowns to the "
                       f"whole apply: {t_apply:.2f} s; dense assembly of the whole operator "
                       f"extrapolated: {t_asm * scale:.0f} s"),
            "apply_s_extrapolated": t_apply, "assembly_s_extrapolated": t_asm * scale}


def one_rhs_step(args, n_steps, n_warm, with_cpu):
    """The one-RHS workload: tables + GMRES(50) to 1e-8 + far field per step."""
    import torch

    import synth
    from paper_1409_8186_amd import Problem
    cl = synth.one_rhs()
    beta = [[math.pi / 4]]
    th = torch.tensor(cl.thetas, device="cuda")
    info = {}

    def step():
        P = Problem.from_cluster(cl)                          # geometry + tables
        rho, flag, relres, iters, _ = P.gmres(betas=beta, restart=50, tol=1e-8, maxit=20000,
                                              graph=args.graph)
        a = P.farfield(rho, th)                              # far field, 720 angles
        info["P"], info["iters"], info["flag"], info["relres"], info["a"] = P, iters, flag, relres, a
        return P

    for _ in range(n_warm):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_steps):
        step()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / n_steps
    iters = int(info["iters"][0])
    flag = int(info["flag"][0])
    assert flag == 0, f"GMRES did not converge (flag {flag})"
    n_app = iters + math.ceil(iters / 50)           # Arnoldi applies + one residual per cycle
    P = info["P"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.gmres(betas=beta, restart=50, tol=1e-8, maxit=20000, graph=args.graph)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    x = torch.randn(cl.n_tot, dtype=torch.complex128, device="cuda")
    y = P.empty(1)
    for _ in range(5):
        P.matvec(x, op=1, out=y)
    n_rep = 200
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(n_rep):
        P.matvec(x, op=1, out=y)
    ev1.record()
    ev1.synchronize()
    t_apply = ev0.elapsed_time(ev1) / 1e3 / n_rep      # lane kernel + output pass
    P.profile_begin(n_rep)
    for _ in range(n_rep):
        P.matvec(x, op=1, out=y)
    ph = P.profile_end()
    t_lane = ph["mfma_or_lane"] / 1e3 / ph["applies"]
    flops = algorithmic_flops(cl.n_modes)
    achieved = flops / t_lane / 1e12
    out = {"metric": "complex unknown·RHS matvecs/s", "value": cl.n_tot * n_app / t_step,
           "unit": "complex unknown·RHS matvecs/s", "steps": n_steps, "warmup": n_warm,
           "ms_per_step": t_step * 1e3,
           "config": {"workload": "one_rhs: M=400 disks a=0.5 in [0,60]^2 gap 0.2, k=2pi, N_p=12 "
                                  "(10,000 unknowns), beta=pi/4, GMRES(50) to 1e-8, far field 720 "
                                  "angles; one step = tables + solve + far field",
                      "n_unknowns": cl.n_tot, "R": 1, "gmres_iters": iters,
                      "operator_applies_per_step": n_app, "graph": bool(args.graph)},
           "time_to_1e8_ms": t_solve * 1e3, "apply_us": t_apply * 1e6,
           "apply_rate": cl.n_tot / t_apply,
           "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS,
                        "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR_TFLOPS,
                        "traffic": traffic_per_launch(),
                        "kernel": "k_apply_lane<12, false> (one lane per ordered pair)",
                        "kernel_us": t_lane * 1e6,
                        "source_sha256_16": apply_source_sha(),
                        "algorithmic_flops_per_launch": flops,
                        "algorithmic_bytes_per_launch": algorithmic_bytes(cl.n_modes)}}
    if with_cpu:
        out["roofline"].update(measured_peaks(achieved))
        out["cpu_baseline"] = cpu_baseline(cl, iters)
    return out


def headline(args):
    """The default line: the 256-column apply of the multi-RHS workload."""
    import numpy as np
    import torch

    import synth
    from paper_1409_8186_amd import Problem
    cl = synth.multi_rhs()
    R = len(cl.betas)
    t0 = time.perf_counter()
    P = Problem.from_cluster(cl, circulant=True)
    torch.cuda.synchronize()
    t_tables = time.perf_counter() - t0
    x = torch.randn(R * cl.n_tot, dtype=torch.complex128, device="cuda")
    y = P.empty(R)
    P.matvec(x, R=R, op=1, out=y)           # first apply of this R times the candidate forms
    for _ in range(args.warmup):
        P.matvec(x, R=R, op=1, out=y)
    torch.cuda.synchronize()
    P.profile_begin(args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        P.matvec(x, R=R, op=1, out=y)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    ph = P.profile_end()
    n = ph.pop("applies")
    phases_ms = {k: v / n for k, v in ph.items()}
    cfg = P.apply_config(R)
    info = P.circulant_info()
    tile = P.circulant_tile(R)
    circ = cfg["kind"] == "circulant"
    if circ:
        kern_s = phases_ms["frequency_products"] / 1e3
        flops = 8.0 * R * info["L_max"] * info["far_pairs"]
        kname = (f"k_circ_gemm (per-frequency products T_f Z_f, tile {tile[0]}x{tile[1]} "
                 f"K{tile[2]}, staging depth {tile[3]}, {tile[4]} threads, {tile[5]} real "
                 f"products per complex product)")
        traffic = circ_traffic_per_launch(tile)
        sha = apply_source_sha(CIRC_SRC)
    else:
        kern_s = phases_ms["mfma_or_lane"] / 1e3
        flops = algorithmic_flops(cl.n_modes, R)
        kname = "k_apply_mfma (direct Toeplitz tiles on the MFMA work queue)"
        traffic, sha = None, apply_source_sha()
    achieved = flops / kern_s / 1e12
    out = {"metric": "complex unknown·RHS matvecs/s", "value": cl.n_tot * R / t_step,
           "unit": "complex unknown·RHS matvecs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": t_step * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "complex128 (f64)",
           "data": "synthetic (seeded disk cluster)",
           "config": {"workload": "multi_rhs: M=1000 disks, a~U[0.3,1] in [0,150]^2 gap 0.1, k=10, "
                                  "N_p=ceil(10a)+10 (34,932 unknowns), 256 incidences; one step = "
                                  "one operator apply A = D^-1 L on all 256 columns",
                      "n_unknowns": cl.n_tot, "R": R, "apply": cfg,
                      "pairs": info, "product_tile": list(tile)},
           "phases_ms": phases_ms, "tables_s": t_tables,
           "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_MFMA_TFLOPS,
                        "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_MFMA_TFLOPS,
                        "traffic": traffic, "kernel": kname, "kernel_ms": kern_s * 1e3,
                        "algorithmic_flops_per_launch": flops,
                        "flops_note": ("8 R L per well-separated ordered pair (the products of "
                                       "the circulant form; the zero entries of T_f for the "
                                       "diagonal and the close pairs are not counted); a "
                                       "complex multiply-add counts 8 flops in either product "
                                       "form, and in Gauss's three-product form the matrix "
                                       "cores execute 6 of them" if circ
                                       else "8 R n_p n_q per ordered pair"),
                        "matrix_core_flops_per_launch": (flops * (6.0 if circ and tile[5] == 3 else 8.0)
                                                         / 8.0),
                        "source_sha256_16": sha}}
    out["roofline"].update(measured_peaks(achieved, "fp64_mfma"))
    # the same apply in the direct form (every pair as Toeplitz tiles on MFMA)
    P.set_circulant(R, 0)
    P.matvec(x, R=R, op=1, out=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        P.matvec(x, R=R, op=1, out=y)
    e1.record()
    e1.synchronize()
    out["direct_form_apply_ms"] = e0.elapsed_time(e1) / 3
    P.set_circulant(R, -1)
    print(f"[bench] apply {t_step * 1e3:.3f} ms; direct form {out['direct_form_apply_ms']:.1f} ms",
          file=sys.stderr, flush=True)
    if args.solve:
        # time-to-1e-8: tables, right-hand sides and the lockstep solve of all 256 columns
        P.close()
        del P
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P = Problem.from_cluster(cl, circulant=True)
        rho, flag, relres, iters, _ = P.gmres(betas=cl.betas[None, :], restart=30, tol=1e-8,
                                              maxit=20000, sstep=SOLVE_SSTEP)
        torch.cuda.synchronize()
        out["time_to_1e8_s"] = time.perf_counter() - t0
        out["solve"] = {"what": "tables + plane-wave right-hand sides + s-step GMRES(30) "
                                f"(s = {SOLVE_SSTEP}: a first one-vector cycle, then Newton bases "
                                "with its Ritz shifts), x0 = 0, all 256 columns to 1e-8 (the first "
                                "apply times the forms)",
                        "gmres_iters_max": int(iters.max()), "gmres_iters_min": int(iters.min()),
                        "all_converged": bool((flag == 0).all()),
                        "relres_max": float(relres.max()),
                        "apply_form": P.apply_config(R)["kind"]}
        print(f"[bench] 256-column solve {out['time_to_1e8_s']:.1f} s", file=sys.stderr, flush=True)
        P.close()
        del P, rho
        torch.cuda.empty_cache()
    one = one_rhs_step(args, 3, 1, False)
    out["one_rhs"] = {k: one[k] for k in ("value", "ms_per_step", "time_to_1e8_ms", "apply_us",
                                          "apply_rate", "roofline")}
    out["one_rhs"]["config"] = one["config"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_multi(cl, R)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", dest="graph", action="store_true", default=True,
                    help="replay each GMRES restart cycle as a captured HIP graph (default)")
    ap.add_argument("--no-graph", dest="graph", action="store_false",
                    help="enqueue every GMRES kernel from the host")
    ap.add_argument("--no-solve", dest="solve", action="store_false", default=True,
                    help="skip the 256-column time-to-1e-8 solve of the default line")
    ap.add_argument("--kernel-only", type=int, default=0, metavar="REPS",
                    help="profiling mode: build the tables, run REPS operator applies of the "
                         "selected workload (multi_rhs: 256 columns; one_rhs: one), exit")
    ap.add_argument("--workload", default="multi_rhs",
                    choices=["multi_rhs", "multi_rhs_block", "one_rhs", "uneven", "differentiation", "dort",
                             "formulations", "nearfield", "penetrable"],
                    help="multi_rhs (default bench line) or a documentation run of another workload")
    ap.add_argument("--grad-sstep", type=int, default=10, metavar="S",
                    help="differentiation workload: s-step size of the gradient's solves (0: one-vector)")
    ap.add_argument("--sstep-sizes", default="15,10", metavar="S,S,...",
                    help="multi_rhs_block workload: s-step sizes to run next to lockstep")
    ap.add_argument("--block-sizes", default="16,8", metavar="S,S,...",
                    help="multi_rhs_block: block sizes of the block GMRES solves")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="profiling mode: one device-to-device copy of BYTES (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path is a single-GPU build "
              "(see the sharding notes in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1409_8186_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1409_8186_amd.build import build
        build()
    from paper_1409_8186_amd import Problem

    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.ones(args.copy_probe // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8, "launches": 3}), flush=True)
        return
    if args.kernel_only:
        if args.workload == "one_rhs":
            cl, R, P = synth.one_rhs(), 1, None
            P = Problem.from_cluster(cl)
        else:
            cl = synth.multi_rhs()
            R = len(cl.betas)
            P = Problem.from_cluster(cl, circulant=True)
        x = torch.randn(R * cl.n_tot, dtype=torch.complex128, device="cuda")
        y = P.empty(R)
        P.matvec(x, R=R, op=1, out=y)
        for _ in range(args.kernel_only):
            P.matvec(x, R=R, op=1, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"applies": args.kernel_only, "apply": P.apply_config(R)}), flush=True)
        return
    if args.workload == "multi_rhs":
        print(json.dumps(headline(args)), flush=True)
        return
    if args.workload == "one_rhs":
        out = one_rhs_step(args, args.steps, args.warmup, not args.no_cpu_baseline)
        out.update({"n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                    "dtype": "complex128 (f64)", "data": "synthetic (seeded disk cluster)"})
        print(json.dumps(out), flush=True)
        return
    print(json.dumps(other_workload(args)), flush=True)


if __name__ == "__main__":
    main()
