#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

A step is one V-cycle x = MG_L(0, b) (Alg. gmg) of the 3-D Q4 SIPG problem on
32^3 uniform cells of the unit cube (4,096,000 DoFs, FP64): on each of the two
finer levels 2 pre- and 2 post-smoothing sweeps of the additive vertex-patch
Schwarz smoother (omega = 0.5, fast-diagonalisation local solves, matrix-free
residual), restriction and prolongation, and the LU solve of the 64,000-DoF
coarse problem (8^3 cells; factors stored by slabs of cells, the exact zeros
of the dense factors left out and the blocks between slabs kept in the
low-rank form their face coupling gives them).  Setup (1-D eigenproblems, coarse LU) is
outside the timed region; b is resident in HBM.

value = fine-level DoFs processed per second = N / (time per V-cycle).
Per-kernel rooflines are measured live with events on the launch stream.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--no-mixed] [--no-batched] [--no-mult]
    python bench.py --profile-only | --profile-mixed PREC | --profile-batched | --profile-distorted
                    | --calibrate-copy   (for rocprofv3)

The JSON line also carries the smoother rooflines, the 48^3 Q7
mixed-precision CG comparison, the 64-mesh batched sweep, the multiplicative
smoothers with GMRES, the surrogate smoother on a distorted mesh, and the CPU
oracle baseline.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from synthetic import CONFIGS, random_vector, uniform_widths  # noqa: E402
from paper_1910_11239_amd import workmodel as wm  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def _events_time(fn, reps, warm=True):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if warm:
        fn()  # first call outside the timed region (kernel code objects load lazily)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps  # ms


def measured_traffic(kernel):
    """HBM bytes per call of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by the copy calibration), or
    None when the kernel's source has changed since the counters were taken."""
    import hashlib
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(tpath):
        return None
    rec = json.load(open(tpath)).get(kernel)
    if not rec:
        return None
    h = hashlib.sha256()
    for rel in rec["sources"]:
        src = os.path.join(ROOT, rel)
        if not os.path.exists(src):
            return None
        h.update(open(src, "rb").read())
    if h.hexdigest() != rec["sha256"]:
        return None
    return rec["bytes_per_call"]


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def mixed_errors_vs_oracle(solutions):
    """The exact discrete solution of the 48^3 Q7 problem from the oracle's
    global fast diagonalisation (host FP64), and each precision's CG solution's
    relative 2-norm and max-norm error against it."""
    from oracle.mesh import uniform_mesh
    from oracle import onedim
    cfg = CONFIGS["mixed_3d_q7"]
    m = uniform_mesh(cfg["dim"], cfg["k"], cfg["m"], gamma_hat=cfg["gamma_hat"])
    t = time.perf_counter()
    xs = onedim.global_fastdiag_solve(m, random_vector(m.ndofs, cfg["seed_b"]))
    dt = time.perf_counter() - t
    n2, ninf = float(np.linalg.norm(xs)), float(np.abs(xs).max())
    errs = {prec: {"rel_2": float(np.linalg.norm(x - xs)) / n2, "rel_max": float(np.abs(x - xs).max()) / ninf}
            for prec, x in solutions.items()}
    return {"by_precision": errs, "oracle_seconds": dt,
            "oracle": "onedim.global_fastdiag_solve: (S x S x S) diag(1/Lambda) (S x S x S)^T of the global 1-D "
                      "SIPG matrices (384 x 384 per axis), FP64 on the host"}


def cpu_baseline(cfg):
    """The oracle (plain FP64 numpy/scipy: sparse quadrature matrix, dense-LU
    patch solves) on the same workload reduced to 8^3 fine cells (64,000 DoFs;
    3 levels 8^3/4^3/2^3, Q4, omega 0.5, 2/2 sweeps): one residual, one
    smoother sweep and one V-cycle, each with one BLAS thread and with all the
    host's threads; setup excluded.  value = V-cycle DoFs/s, all threads."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle.mesh import uniform_mesh
    from oracle import multigrid
    fine = uniform_mesh(3, cfg["k"], 8, gamma_hat=cfg["gamma_hat"])
    nl = cfg["nlevels"]
    h = multigrid.Hierarchy(fine, nl, "vertex", [0.0] + [cfg["omega"]] * (nl - 1),
                            m_pre=cfg["m_pre"], m_post=cfg["m_post"])
    b = random_vector(fine.ndofs, cfg["seed_b"])
    x = random_vector(fine.ndofs, cfg["seed_x"])
    A = h.A[-1]

    def med(fn, reps):
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))

    threads_all = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    timings = {}
    for label, limit in (("1_thread", 1), ("all_threads", None)):
        with threadpool_limits(limit):
            timings[label] = {
                "residual_s": med(lambda: b - A @ x, 5),
                "sweep_s": med(lambda: h.smooth(nl - 1, x.copy(), b), 3),
                "vcycle_s": med(lambda: h.vcycle(np.zeros_like(b), b), 3),
            }
    for v in timings.values():
        for key in list(v):
            v[key.replace("_s", "_dofs_per_s")] = fine.ndofs / v[key]
    return {"value": fine.ndofs / timings["all_threads"]["vcycle_s"], "unit": "DoFs/s", "cores": int(threads_all),
            "kind": "oracle", "cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count(),
            "timings": timings,
            "sample": "oracle residual (x5), smoother sweep (x3) and V-cycle (x3, the value) on the same workload "
                      "reduced to 8^3 fine cells (64,000 DoFs), medians, 1 thread and all threads, setup excluded"}


def mixed_vs_fp64(steps_hint=1):
    """3-D Q7 on 48^3 cells (56,623,104 DoFs): FP64 CG preconditioned by one
    V-cycle (5 levels 48^3..3^3, vertex patches, omega = 2^-3, 2+2 sweeps,
    dense LU on 13,824 coarse DoFs) to ||r|| <= 1e-10 ||b||, with the smoother
    contractions in FP64, FP32, FP16-MFMA and BF16-MFMA.  Times are
    time-to-solution (setup excluded); rel_diff_vs_f64 = ||x_prec - x_f64|| / ||x_f64||; the
    error against the oracle's exact solution is added by the cpu_baseline leg."""
    import torch
    import paper_1910_11239_amd as fts
    cfg = CONFIGS["mixed_3d_q7"]
    dim, k, m, nl = cfg["dim"], cfg["k"], cfg["m"], cfg["nlevels"]
    omegas = [0.0] + [cfg["omega"]] * (nl - 1)
    t0 = time.perf_counter()
    hier = fts.Hierarchy(dim, k, uniform_widths(dim, m), nl, "vertex", omegas, cfg["gamma_hat"],
                         cfg["m_pre"], cfg["m_post"])
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    N = hier.ndofs
    b = torch.as_tensor(random_vector(N, cfg["seed_b"])).cuda()
    ws = torch.empty((int(fts.lib().fts_pcg_ws_bytes(hier._h)) + 7) // 8, dtype=torch.float64, device="cuda")
    out, sol = {}, {}
    fine, eg = hier.levels[-1], hier.eigs[-1]
    r = torch.as_tensor(random_vector(N, 5)).cuda()
    xa = torch.zeros_like(r)
    rr = torch.empty_like(r)
    patch_flops = wm.smoother_flops(dim, k, (m,) * dim, "vertex")
    apply_bytes = wm.patch_apply_bytes(dim, k, (m,) * dim)
    res_bytes = wm.residual_bytes(dim, k, (m,) * dim)
    t_res = _events_time(lambda: fine.residual(b, xa, rr), 5)
    for prec in ("f64", "f32", "f16", "bf16"):
        x = torch.zeros(N, dtype=torch.float64, device="cuda")
        hier.pcg(b, x, rtol=cfg["rtol"], maxit=3, prec=prec, ws=ws)  # warm-up
        x.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        it, rel, _ = hier.pcg(b, x, rtol=cfg["rtol"], maxit=400, prec=prec, ws=ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        t_apply = _events_time(lambda: fts.schwarz_apply(fine, eg, cfg["omega"], r, xa, prec=prec), 3)
        # one smoothing step as the V-cycle runs it: r = b - A x (FP64; stored
        # in FP32 for the 16-bit owner tiles), then the local solves
        sweep_ms = _events_time(lambda: fts.schwarz_smooth(fine, eg, cfg["omega"], b, xa, 1, prec=prec, ws=rr), 5)
        sol[prec] = x
        out[prec] = {"iterations": it, "seconds": dt, "final_relres": rel,
                     "patch_apply_ms": t_apply,
                     "patch_apply_tflops": patch_flops / (t_apply * 1e-3) / 1e12,
                     "patch_apply_hbm_gbs": apply_bytes / (t_apply * 1e-3) / 1e9,
                     "sweep_ms": sweep_ms,
                     "sweep_dofs_per_s": N / (sweep_ms * 1e-3),
                     "sweep_hbm_gbs": (res_bytes + apply_bytes) / (sweep_ms * 1e-3) / 1e9}
    for prec in out:
        out[prec]["rel_diff_vs_f64"] = float(torch.linalg.norm(sol[prec] - sol["f64"]) /
                                             torch.linalg.norm(sol["f64"]))
        out[prec]["speedup_vs_f64"] = out["f64"]["seconds"] / out[prec]["seconds"]
    host_sol = {prec: v.cpu().numpy() for prec, v in sol.items()}
    del hier, sol
    torch.cuda.empty_cache()
    return {"workload": "mixed_3d_q7: 3-D DG Q7, 48^3 cells (56,623,104 DoFs), CG to 1e-10 with a 5-level "
                        "vertex-patch V-cycle (omega 0.125, 2+2 sweeps, dense LU on 13,824 DoFs)",
            "setup_s": setup_s, "residual_ms": t_res,
            "algorithmic_bytes": {"residual": res_bytes, "patch_apply": apply_bytes,
                                  "note": "residual reads x, b and writes r (24 B/DoF); the patch apply reads r "
                                          "and reads and writes x (24 B/DoF); a sweep is both (48 B/DoF, counted "
                                          "with an FP64 r for every precision)"},
            "error_vs_oracle": "filled in by the cpu_baseline leg: each precision's ||x - x_oracle|| / "
                               "||x_oracle|| against the exact discrete solution (oracle global fast "
                               "diagonalisation on the host); also asserted by "
                               "tests/test_gpu_parity.py::test_mixed_3d_q7_cg_error_vs_oracle",
            "by_precision": out}, host_sol


def batched_workload():
    """64 independent 3-D meshes (k ~ U{2..9}, m ~ U{8..24} cells per axis,
    per-slab widths log-uniform in [0.25, 4]): one sweep = FP64 residual + FP32
    local solves in one persistent launch + batched gather, after autotuning
    the persistent launch shape."""
    import torch
    import paper_1910_11239_amd as fts
    from synthetic import batched_meshes
    specs = batched_meshes()
    t0 = time.perf_counter()
    batch = fts.Batch([(k, w, 1.0) for k, w in specs])
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    N = batch.ndofs
    b = torch.as_tensor(random_vector(N, 0)).cuda()
    x = torch.zeros(N, dtype=torch.float64, device="cuda")
    r = torch.empty_like(x)
    batch.residual(b, x, r)
    report = batch.autotune(r, prec="f32")
    flops = sum(wm.smoother_flops(3, k, tuple(len(a) for a in w), "vertex") for k, w in specs)
    t_apply = _events_time(lambda: batch.apply(0.125, r, x, prec="f32"), 5)
    t_res = _events_time(lambda: batch.residual(b, x, r), 5)
    ws = torch.empty_like(x)
    t_sweep = _events_time(lambda: batch.smooth(0.125, b, x, 1, prec="f32", ws=ws), 5)
    del batch
    torch.cuda.empty_cache()
    return {"workload": "batched: 64 meshes, k ~ U{2..9}, m ~ U{8..24}^3, widths log-uniform [0.25, 4] per slab",
            "dofs": N, "degrees": sorted({k for k, _ in specs}), "setup_s": setup_s,
            "sweep_ms": t_sweep, "sweep_dofs_per_s": N / (t_sweep * 1e-3),
            "apply_ms": t_apply, "apply_fp32_tflops": flops / (t_apply * 1e-3) / 1e12,
            "residual_ms": t_res, "launch": report.strip().splitlines()[-1]}


def distorted_workload():
    """Sec. 4: the 3-D distorted cube (8^3 cells with interior vertices moved
    by 25 % of the local edge length in random directions, refined twice to
    32^3 cells), Q3, gamma_hat = 4: one sweep of the additive cell smoother
    with Cartesian surrogate local solvers = matrix-free mapped SIPG residual
    + per-cell fast-diagonalisation solves; then the V-cycle and CG of the
    multigrid on the three nested distorted levels (Sec. 4 with Alg. gmg)."""
    import torch
    import paper_1910_11239_amd as fts
    from synthetic import distorted_vertices
    ms, V = distorted_vertices(3, 8, 2, 0.25, 0)
    lv = fts.MappedLevel(3, 3, ms, V, 4.0)
    N = lv.ndofs
    b = torch.as_tensor(random_vector(N, 0)).cuda()
    x = torch.as_tensor(random_vector(N, 1)).cuda()
    r = torch.empty_like(x)
    ws = torch.empty_like(x)
    t_res = _events_time(lambda: lv.residual(b, x, r), 5)
    t_apply = _events_time(lambda: lv.schwarz_apply(0.5, r, x), 5)
    t_sweep = _events_time(lambda: lv.schwarz_smooth(0.5, b, x, 1, ws), 5)
    del lv
    # multigrid on the three nested distorted levels 8^3, 16^3, 32^3 (the
    # paper's 3-D damping for Q3, omega 0.55), CG to 1e-8 from x = 0
    levels = [distorted_vertices(3, 8, lev, 0.25, 0)[1] for lev in range(2)] + [V]
    mg = {}
    for steps in (1, 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = fts.MappedHierarchy(3, 3, (8, 8, 8), levels, 4.0, [0.0, 0.55, 0.55], steps, steps)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        t_vc = _events_time(lambda: h.vcycle(b, x), 5)
        xs = torch.zeros_like(b)
        h.pcg(b, xs, rtol=1e-8, maxit=300)  # warm-up solve
        xs.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, rel, _ = h.pcg(b, xs, rtol=1e-8, maxit=300)
        torch.cuda.synchronize()
        mg[f"ACS_{steps}"] = {"setup_s": setup_s, "vcycle_ms": t_vc, "cg_iterations": it, "cg_relres": rel,
                              "cg_seconds": time.perf_counter() - t0}
        del h
    torch.cuda.empty_cache()
    return {"workload": "distorted cube: 8^3 cells, interior vertices moved by 0.25 h_v, refined twice to 32^3 "
                        "mapped cells, Q3 (2,097,152 DoFs), gamma_hat 4, omega 0.5",
            "dofs": N, "residual_ms": t_res, "surrogate_apply_ms": t_apply, "sweep_ms": t_sweep,
            "sweep_dofs_per_s": N / (t_sweep * 1e-3),
            "residual_gbs": wm.residual_bytes(3, 3, ms) / (t_res * 1e-3) / 1e9,
            "multigrid": {"levels": "8^3, 16^3, 32^3 mapped cells, omega 0.55, ACS_m = m pre- and post-smoothing "
                                    "steps, CG to 1e-8, uniform random right-hand side", **mg}}


def multiplicative_workload():
    """Multiplicative smoothers on the 3-D Q4 32^3 mesh (4,096,000 DoFs):
    one sweep of the vertex-patch smoother with 2^(d+1) = 16 colors and of the
    red-black cell smoother (a residual before every color, Alg. multsmoother),
    and time-to-solution at a relative residual of 1e-8 (the paper's
    criterion) of GMRES preconditioned by the V-cycle with the multiplicative
    vertex-patch smoother (omega 1, 1+1 sweeps, 3 levels) next to PCG with the
    additive one (omega 2^-3, 1+1 sweeps).  Setup excluded."""
    import torch
    import paper_1910_11239_amd as fts
    cfg = CONFIGS["avs_3d_q4"]
    dim, k, m, nl = cfg["dim"], cfg["k"], cfg["m"], cfg["nlevels"]
    widths = uniform_widths(dim, m)
    out = {"workload": "3-D SIPG Q4, 32^3 uniform cells (4,096,000 DoFs), FP64"}
    lv = fts.Level(dim, k, widths, cfg["gamma_hat"])
    N = lv.ndofs
    b = torch.as_tensor(random_vector(N, cfg["seed_b"])).cuda()
    x = torch.zeros(N, dtype=torch.float64, device="cuda")
    ws = torch.empty(N, dtype=torch.float64, device="cuda")
    for kind, ncol in (("vertex", 16), ("cell", 2)):
        eg = fts.Eigs(lv, kind)
        fn = lambda: fts.schwarz_smooth_mult(lv, eg, 1.0, b, x, nsweeps=1, ws=ws)
        fn()
        t = _events_time(fn, 5)
        out[f"{kind}_sweep"] = {"colors": ncol, "ms": t, "dofs_per_s": N / (t * 1e-3)}
        del eg
    del lv
    torch.cuda.empty_cache()
    solve = {}
    for name, smoother, omega, method in (("gmres_multiplicative_vertex", "multiplicative", 1.0, "gmres"),
                                          ("pcg_additive_vertex", "additive", 0.125, "pcg")):
        h = fts.Hierarchy(dim, k, widths, nl, "vertex", [0.0] + [omega] * (nl - 1), cfg["gamma_hat"], 1, 1)
        h.set_smoother(smoother)
        xs = torch.zeros(N, dtype=torch.float64, device="cuda")
        run = (lambda: h.gmres(b, xs, rtol=1e-8, restart=30, maxit=300)) if method == "gmres" else \
              (lambda: h.pcg(b, xs, rtol=1e-8, maxit=300))
        run()  # warm-up
        xs.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, relres, _ = run()
        torch.cuda.synchronize()
        solve[name] = {"iterations": it, "final_relres": relres, "seconds": time.perf_counter() - t0}
        del h
        torch.cuda.empty_cache()
    out["time_to_1e-8"] = solve
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the 48^3 Q7 mixed-precision CG comparison")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-mesh batched sweep")
    ap.add_argument("--no-mult", action="store_true", help="skip the multiplicative-smoother measurements")
    ap.add_argument("--no-distorted", action="store_true", help="skip the distorted-mesh surrogate smoother and multigrid")
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup + steps of the V-cycle only (for rocprofv3)")
    ap.add_argument("--profile-mixed", choices=["f64", "f32", "f16", "bf16"],
                    help="run warmup + steps V-cycles of the 48^3 Q7 CG preconditioner at this contraction "
                         "precision only (for rocprofv3)")
    ap.add_argument("--profile-distorted", action="store_true",
                    help="only the distorted-mesh multigrid V-cycle (ACS_1), warmup + steps times (for rocprofv3)")
    ap.add_argument("--profile-batched", action="store_true",
                    help="run the 64-mesh batched smoother only: 3 x (FP32 patch apply + gathers, FP64 residual) "
                         "at 256 threads x 1,024 workgroups x chunks of 4 (for rocprofv3)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 1 GiB FP64 buffer on the device --steps times (reference kernel of known "
                         "traffic for the rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the smoother and V-cycle are single-GPU kernels "
              "(a multi-GPU halo exchange is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        n = 1 << 27  # 2^27 doubles = 1 GiB
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "copies": args.steps}))
        return
    import paper_1910_11239_amd as fts
    if args.profile_distorted:
        from synthetic import distorted_vertices
        levels = [distorted_vertices(3, 8, lev, 0.25, 0)[1] for lev in range(3)]
        hd = fts.MappedHierarchy(3, 3, (8, 8, 8), levels, 4.0, [0.0, 0.55, 0.55], 1, 1)
        bd = torch.as_tensor(random_vector(hd.ndofs, 0)).cuda()
        xd = torch.zeros_like(bd)
        for _ in range(args.warmup + args.steps):
            xd.zero_()
            hd.vcycle(bd, xd)
        torch.cuda.synchronize()
        print(json.dumps({"distorted_dofs": hd.ndofs, "vcycles": args.warmup + args.steps}))
        return

    if args.profile_batched:
        from synthetic import batched_meshes
        batch = fts.Batch([(k, w, 1.0) for k, w in batched_meshes()])
        nb = batch.ndofs
        bb = torch.as_tensor(random_vector(nb, 0)).cuda()
        xb = torch.zeros(nb, dtype=torch.float64, device="cuda")
        rb = torch.empty_like(xb)
        batch.residual(bb, xb, rb)
        batch.set_launch(256, 1024, 4)
        for _ in range(3):
            batch.apply(0.125, rb, xb, prec="f32")
            batch.residual(bb, xb, rb)
        torch.cuda.synchronize()
        print(json.dumps({"batched_dofs": nb}))
        return

    if args.profile_mixed:
        c3 = CONFIGS["mixed_3d_q7"]
        nl3 = c3["nlevels"]
        h3 = fts.Hierarchy(3, c3["k"], uniform_widths(3, c3["m"]), nl3, "vertex", [0.0] + [c3["omega"]] * (nl3 - 1),
                           c3["gamma_hat"], c3["m_pre"], c3["m_post"])
        b3 = torch.as_tensor(random_vector(h3.ndofs, c3["seed_b"])).cuda()
        x3 = torch.zeros_like(b3)
        for _ in range(args.warmup):
            x3.zero_()
            h3.vcycle(b3, x3, prec=args.profile_mixed)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        for _ in range(args.steps):
            x3.zero_()
            h3.vcycle(b3, x3, prec=args.profile_mixed)
        torch.cuda.synchronize()
        print(json.dumps({"prec": args.profile_mixed, "ms_per_vcycle": (time.perf_counter() - t3) / args.steps * 1e3}))
        return

    cfg = CONFIGS["avs_3d_q4"]
    dim, k, m, nl = cfg["dim"], cfg["k"], cfg["m"], cfg["nlevels"]
    omegas = [0.0] + [cfg["omega"]] * (nl - 1)
    widths = uniform_widths(dim, m)
    t0 = time.perf_counter()
    hier = fts.Hierarchy(dim, k, widths, nl, "vertex", omegas, cfg["gamma_hat"], cfg["m_pre"], cfg["m_post"])
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    N = hier.ndofs
    b = torch.as_tensor(random_vector(N, cfg["seed_b"])).cuda()
    x = torch.zeros(N, dtype=torch.float64, device="cuda")

    def step():
        x.zero_()
        hier.vcycle(b, x)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ms = _events_time(step, args.steps, warm=False)
    if args.profile_only:
        print(json.dumps({"ms_per_step": ms}))
        return

    # live per-kernel measurements on the launch stream (same launch configs as in the step)
    fine, eg = hier.levels[-1], hier.eigs[-1]
    r = torch.empty_like(x)
    xs = torch.as_tensor(random_vector(N, cfg["seed_x"])).cuda()
    reps = max(10, args.steps)
    t_res = _events_time(lambda: fine.residual(b, xs, r), reps)
    t_patch = _events_time(lambda: fts.schwarz_apply(fine, eg, cfg["omega"], r, xs), reps)
    n0 = hier.levels[0].ndofs
    b0 = torch.as_tensor(random_vector(n0, 3)).cuda()
    x0 = torch.zeros(n0, dtype=torch.float64, device="cuda")
    t_coarse = _events_time(lambda: hier.coarse_solve(b0, x0), max(5, args.steps // 2))

    ncells = (m,) * dim
    patch_flops = wm.smoother_flops(dim, k, ncells, "vertex")
    res_bytes = wm.residual_bytes(dim, k, ncells)
    # coarse factors: nb slabs of B unknowns; the diagonal blocks are read in
    # full (lower half forward, upper half backward), the low-rank factors of
    # the blocks between slabs in their nonzero parts
    m0 = m // 2 ** (nl - 1)
    B0 = (k + 1) ** dim * m0 ** (dim - 1)
    nb0 = m0
    coarse_bytes = float(wm.coarse_solve_bytes(dim, k, (m0,) * dim))
    sweeps_fine = cfg["m_pre"] + cfg["m_post"]
    kernels = {
        "vertex_patch_apply_fp64": {
            "kernel": "k_schwarz_zrun<5,double> (runs of 4 patches along z) + k_patch_gather", "bound": "alu",
            "achieved": patch_flops / (t_patch * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "ms_per_call": t_patch, "calls_per_step": sweeps_fine,
            "algorithmic": f"{patch_flops:.4g} flop per call (4d n^(d+1) + 2 n^d per patch, n = 10, 29,791 patches; "
                           "the even-odd form executes about half of the 4d n^(d+1) at mirror-symmetric patches)"},
        "residual_fp64": {
            "kernel": "k_operator<3,5,residual>", "bound": "hbm",
            "achieved": res_bytes / (t_res * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "ms_per_call": t_res, "calls_per_step": sweeps_fine + 1,
            "algorithmic": f"{res_bytes:.4g} bytes per call (read x, b, write r)"},
        "coarse_lu_solve": {
            "kernel": f"k_slab_mv ({2 * (2 * nb0 - 1)} launches) + k_lr_expand / k_lr_reduce "
                      f"({2 * (nb0 - 1)} launches)", "bound": "hbm",
            "achieved": coarse_bytes / (t_coarse * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "ms_per_call": t_coarse, "calls_per_step": 1,
            "algorithmic": f"{coarse_bytes:.4g} bytes per call (slab-blocked LU factors of the {n0}-DoF "
                           f"coarse matrix, {nb0} slabs of {B0}: diagonal blocks 8 nb B^2, blocks between slabs "
                           "in low-rank form)"},
    }
    for v in kernels.values():
        v["frac"] = v["achieved"] / v["peak"]
        v["ms_per_step"] = v["ms_per_call"] * v["calls_per_step"]
    dom_name = max(kernels, key=lambda n: kernels[n]["ms_per_step"])
    dom = kernels[dom_name]
    traffic = measured_traffic(dom_name)
    roofline = {"bound": dom["bound"], "achieved": round(dom["achieved"], 3), "peak": dom["peak"],
                "unit": dom["unit"], "frac": round(dom["frac"], 4), "traffic": traffic, "kernel": dom_name}

    sweep_ms = t_res + t_patch
    out = {
        "metric": "smoother DoFs/s + HBM GB/s (3D vertex patch); mixed vs FP64 at 1e-10 residual",
        "value": N / (ms * 1e-3),
        "unit": "DoFs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "avs_3d_q4: 3-D SIPG Poisson, DG Q4, 32^3 uniform cells (4,096,000 DoFs), "
                               "V-cycle 32^3/16^3/8^3, vertex-patch additive Schwarz omega 0.5, 2 pre/post "
                               "sweeps, dense LU on 64,000 coarse DoFs; b uniform[-1,1] seed 0",
                   "global_batch": 1, "dofs": N, "parallelism": "single GPU"},
        "roofline": roofline,
        "kernels": {n: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for n, v in kernels.items()},
        "smoother_sweep": {"dofs_per_s": N / (sweep_ms * 1e-3), "ms": sweep_ms,
                           "algorithmic_hbm_gbs": wm.smoother_sweep_bytes(dim, k, ncells) / (sweep_ms * 1e-3) / 1e9},
        "setup_s": setup_s,
    }
    del hier
    torch.cuda.empty_cache()
    apply_bytes = wm.patch_apply_bytes(dim, k, ncells)
    smoother = {
        "avs_3d_q4_fp64_patch_apply": {
            "kernel": kernels["vertex_patch_apply_fp64"]["kernel"], "bound": "alu",
            "achieved": round(patch_flops / (t_patch * 1e-3) / 1e12, 3), "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(patch_flops / (t_patch * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
            "hbm_gbs": round(apply_bytes / (t_patch * 1e-3) / 1e9, 1),
            "hbm_frac": round(apply_bytes / (t_patch * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("avs_3d_q4_fp64_patch_apply"),
            "algorithmic": f"{patch_flops:.4g} flop and {apply_bytes:.4g} bytes (read r, read and write x) per call"},
    }
    out["smoother_roofline"] = smoother
    mixed_solutions = None
    if not args.no_mixed:
        out["mixed_vs_fp64"], mixed_solutions = mixed_vs_fp64()
        mx = out["mixed_vs_fp64"]
        for prec in ("f16", "bf16"):
            bp = mx["by_precision"][prec]
            smoother[f"mixed_3d_q7_{prec}_sweep"] = {
                "kernel": "k_operator (FP64 residual, stored FP32) + k_schwarz_mfma_tile (16-bit MFMA owner tiles)",
                "bound": "hbm",
                "achieved": round(bp["sweep_hbm_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(bp["sweep_hbm_gbs"] / HBM_PEAK_GBS, 4),
                "apply_hbm_gbs": round(bp["patch_apply_hbm_gbs"], 1),
                "apply_frac": round(bp["patch_apply_hbm_gbs"] / HBM_PEAK_GBS, 4),
                "ms": bp["sweep_ms"], "dofs_per_s": bp["sweep_dofs_per_s"],
                "traffic": measured_traffic(f"mixed_3d_q7_{prec}_sweep"),
                "algorithmic": "48 B/DoF per sweep: residual 24 (read x, b, write r) + apply 24 (read r, "
                               "read and write x), 56,623,104 DoFs"}
    if not args.no_batched:
        out["batched"] = batched_workload()
    if not args.no_mult:
        out["multiplicative"] = multiplicative_workload()
    if not args.no_distorted:
        out["distorted"] = distorted_workload()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg)
        if mixed_solutions is not None:
            out["mixed_vs_fp64"]["error_vs_oracle"] = mixed_errors_vs_oracle(mixed_solutions)
            del mixed_solutions
    print(json.dumps(out))


if __name__ == "__main__":
    main()
