"""Benchmark: matrix-free phase-field Jacobian on one MI355X.

Workload (default): Sneddon-type mesh, 1024 x 1024 base cells + 3 local
refinement levels in the band |x| < 2, |y| < 0.5, Q2 (20.5 M unknowns), FP64.

Reported (one JSON line on stdout):
  value        GDoF/s of the leaf Jacobian vmult (N_dof / time per call, HIP
               events on the launch stream, inputs resident in HBM)
  ms_per_step  one Newton / primal-dual active set iteration (Alg. 2:
               residual, active set, multigrid setup, GMRES with the block
               V-cycle, line search), FP64, the first K iterations of a load step
  load_step    the whole load step to convergence (active set unchanged and
               |R~| <= 1e-7), FP64 and mixed precision (FP32 V-cycle with
               Chebyshev degree 4 and a coarse CG): seconds, Newton steps,
               GMRES iterations, final residual, TCV against Sneddon's value,
               and the mixed solution's difference from the FP64 one
  roofline     algorithmic bytes of one vmult / its duration vs 8 TB/s HBM
  cpu_baseline the FP64 oracle's assembled-Jacobian SpMV (median of 20 calls,
               one host thread) on a smaller mesh of the same family; the
               assembly time is reported apart
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "vmult_traffic.json")
KERNEL_SOURCES = ["paper_2404_03265_amd/csrc/tile_kernel.hpp", "paper_2404_03265_amd/csrc/cell.hpp",
                  "paper_2404_03265_amd/csrc/mesh.cpp", "paper_2404_03265_amd/csrc/mesh.hpp"]


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, path: str = TRAFFIC_FILE):
    """HBM bytes per vmult from the committed counter summary, or None when
    there is none for the workload or the kernel sources have changed since
    the counters were taken (their hash differs)."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        tr = json.load(fh)
    w = tr.get("workloads", {}).get(workload)
    if tr.get("kernel_hash") != kernel_hash() or w is None:
        return None
    return w.get("bytes_per_launch")


def algorithmic_bytes(n_nodes: int, n_cells: int, degree: int) -> int:
    """Bytes one vmult must move: src and dst (3 comps, 8 B each), the state
    (u_x, u_y, phi, phit: 4 x 8 B per node) and an int32 dof map per cell."""
    return 16 * 3 * n_nodes + 32 * n_nodes + 4 * (degree + 1) ** 2 * n_cells


def tcv_sneddon(spec) -> float:
    """Sneddon's crack volume 2 pi p l0^2 / E' (plane strain E' = E / (1 - nu^2), l0 = 1)."""
    import math
    return 2.0 * math.pi * spec.pressure / (spec.E / (1.0 - spec.nu ** 2))


def cod_sneddon(spec, x: float) -> float:
    """Sneddon's opening 4 p l0 / E' (1 - x^2 / l0^2)^(1/2) for |x| < l0 (l0 = 1), the
    total jump whose integral over x is the crack volume 2 pi p l0^2 / E'."""
    import math
    ep = spec.E / (1.0 - spec.nu ** 2)
    return 4.0 * spec.pressure / ep * math.sqrt(max(0.0, 1.0 - x * x)) if abs(x) < 1.0 else 0.0


def make_state(g, spec, seed=0, random=True):
    import numpy as np
    import torch

    import inputs
    X, Y = g.coords()
    fl = g.flags()
    ux, uy, phi = inputs.sneddon_state(X, Y, g.M, spec.degree, seed=seed, random=random)
    d = (fl & 1) != 0
    U = np.concatenate([np.where(d, 0.0, ux), np.where(d, 0.0, uy), phi])
    return (torch.tensor(U, device="cuda"), torch.tensor(phi, device="cuda"), X, Y)


def time_calls(fn, reps, warm=5):
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps   # ms


def median_call(fn, reps, warm=5):
    """Median duration of single calls (events around each call), ms."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = sorted(a.elapsed_time(b) for a, b in ev)
    return t[len(t) // 2]


def cpu_baseline(sample_base=512, sample_local=3, degree=2, reps=20, warm=2):
    """The oracle as it stands, on one host thread: assemble the masked
    Jacobian J~ as a CSR matrix (timed, reported apart), then time the product
    J~ src itself, the operation the GPU vmult replaces: the median of `reps`
    calls after `warm` untimed ones. The sample mesh is the same Sneddon
    family at a smaller size (512^2 + 3 local levels, Q2, 5.1 M unknowns),
    since assembling the benchmark mesh's Jacobian takes minutes and tens of
    GB; the rate is per unknown, so it compares across sizes."""
    import numpy as np

    import inputs
    from oracle.assemble import LeafProblem, Params
    from oracle.mesh import Mesh
    spec = inputs.WorkloadSpec(name="sample", n_base=sample_base, n_local=sample_local, degree=degree)
    m = Mesh(sample_base, sample_local, degree)
    lp = LeafProblem(m, Params(E=spec.E, nu=spec.nu, Gc=spec.Gc, pressure=spec.pressure,
                               kappa=spec.kappa, ell=spec.ell))
    ux, uy, phi = inputs.sneddon_state(m.NX, m.NY, m.M, m.p, seed=0)
    U = lp.distribute(np.concatenate([ux, uy, phi]))
    act = inputs.bernoulli_mask(m.NX, m.NY, 2, 0.1) & ~m.hanging
    src = inputs.random_vector(m.NX, m.NY, 1)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):      # the reported core count: BLAS pinned to one thread
        t0 = time.perf_counter()
        J = lp.masked_operator(U, phi, act)
        t_asm = time.perf_counter() - t0
        y = None
        for _ in range(warm):
            y = J @ src
        ts = []
        for _ in range(reps):
            t1 = time.perf_counter()
            y = J @ src
            ts.append(time.perf_counter() - t1)
    t_med = sorted(ts)[len(ts) // 2]
    n_dof = 3 * m.n_nodes
    return {
        "value": n_dof / t_med / 1e9,
        "unit": "GDoF/s",
        "cores": 1,     # SciPy's CSR product runs on one thread (BLAS limited to one as well)
        "kind": "oracle",
        "sample": (f"the oracle's assembled masked Jacobian times a vector (SciPy CSR, {J.nnz} nonzeros), "
                   f"median of {reps} calls after {warm} warm-ups: {t_med * 1e3:.1f} ms for {n_dof} unknowns "
                   f"on sneddon {sample_base}x{sample_base} + {sample_local} local levels, Q{degree} (the same "
                   f"family as the benchmark workload, about a quarter of its size)"),
        "assembly_seconds": t_asm,
        "spmv_ms_median": t_med * 1e3,
        "host_cpus": os.cpu_count(),
        "_check": float(abs(y).sum()),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sneddon_1024x1024_L3_Q2")
    ap.add_argument("--vmult-reps", type=int, default=50)
    ap.add_argument("--tile", type=int, nargs=2, default=(0, 0),
                    help="owned cells per tile (x, y); 0 0 = library default")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--scenario", choices=("none", "diff", "quasistatic", "table2"), default="none",
                    help="diff: 16-vector vmult / vmult_T batch and the adjoint crack-volume gradient "
                         "checked by central differences (use with sneddon_512x512_L3_Q2); "
                         "quasistatic: pressure increments p = 1e-3 k with the active set carried, "
                         "FP32 V-cycle, adjoint at the last step (use with sneddon_2048x2048_L4_Q2); "
                         "table2: the paper's mesh family (Q1, 40 x 40 base, 0-8 local levels), one "
                         "load step each")
    ap.add_argument("--increments", type=int, default=10)
    ap.add_argument("--table2-kappa", default="1e-10", help="table2: a value, or 'paper' for 1e-12 h")
    ap.add_argument("--table2-local-max", type=int, default=8)
    ap.add_argument("--extrapolate", action="store_true",
                    help="quasistatic: phi~ extrapolated from the last two load steps (from the third increment)")
    ap.add_argument("--no-newton", action="store_true")
    ap.add_argument("--no-load-step", action="store_true",
                    help="time the Newton steps only, not the whole load step (for profiler runs)")
    ap.add_argument("--newton-modes", default="fp64,mixed,mixed_cheb3,gc_fp64,gc_mixed,tri_fp64",
                    help="comma-separated subset of fp64,mixed,mixed_cheb3")
    ap.add_argument("--profile-pass", action="store_true",
                    help="only a few vmults and one plain device copy of the same vector "
                         "(for hardware counter runs)")
    args = ap.parse_args()
    if args.scenario != "none":
        args.no_newton = True
        args.no_cpu_baseline = True
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import inputs
    from paper_2404_03265_amd import PhaseFieldSolver, SolverParams

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    spec = inputs.WORKLOADS[args.workload]
    sp_ = SolverParams(E=spec.E, nu=spec.nu, Gc=spec.Gc, pressure=spec.pressure, kappa=spec.kappa,
                       ell=spec.ell)
    t0 = time.time()
    # both multigrid hierarchies: local smoothing (Sec. 3.2) and global
    # coarsening (modes gc_*)
    want_gc = not args.no_newton and any(m.startswith("gc_") for m in args.newton_modes.split(","))
    g = PhaseFieldSolver(spec.n_base, spec.n_local, spec.degree, coarse=spec.coarse, band=spec.band,
                         tile=tuple(args.tile), params=sp_, mg_global=want_gc)
    n_tiles, n_rec, _ = g.tile_stats()
    log(f"{spec.name}: {3 * g.n} unknowns, {g.n_levels} levels, {n_tiles} tiles, "
        f"built in {time.time() - t0:.1f}s")
    n_dof = 3 * g.n

    # ---- vmult at a random state, active set from the rule ----------------
    U, phi, X, Y = make_state(g, spec, random=True)
    g.set_state(U, phi, phi, None, setup_mg=False)
    src = torch.tensor(inputs.random_vector(X, Y, 1), device="cuda")
    dst = torch.empty_like(src)
    if args.profile_pass:
        for _ in range(3):
            g.vmult(src, dst)
        calib = torch.empty_like(src)
        calib.copy_(src)      # plain copy of 3n doubles: counter calibration
        torch.cuda.synchronize()
        print(json.dumps({"profile_pass": spec.name, "copy_bytes": 2 * src.numel() * 8}), flush=True)
        return
    ms_vmult = time_calls(lambda: g.vmult(src, dst), args.vmult_reps)
    med_vmult = median_call(lambda: g.vmult(src, dst), args.vmult_reps)
    gdofs = n_dof / (ms_vmult * 1e-3) / 1e9
    n_cells_leaf = n_rec          # one cell record per leaf cell
    algo = algorithmic_bytes(g.n, n_cells_leaf, spec.degree)
    achieved = algo / (ms_vmult * 1e-3) / 1e9
    log(f"vmult {ms_vmult * 1e3:.1f} us -> {gdofs:.2f} GDoF/s, {achieved:.0f} GB/s algorithmic")
    traffic = load_traffic(spec.name)

    # ---- load-step solves (Alg. 2 loop), FP64 and mixed precision ----------
    extra = {}
    ms_step = None
    if not args.no_newton:
        from paper_2404_03265_amd.autograd import solve_load_step
        U0, phi0, _, _ = make_state(g, spec, random=False)
        Uw = U0.clone()
        solve = {}
        # FP64: Chebyshev degree 3 smoothing and coarse Chebyshev; mixed: the
        # whole V-cycle in FP32 with Chebyshev degree 4 and a coarse CG (30
        # steps); residual, GMRES and line search stay FP64 in both
        # "mixed_cheb3": the FP32 V-cycle with the FP64 configuration's smoother
        # and coarse solve, isolating the effect of the precision
        # gc_fp64 / gc_mixed: the same two configurations with the
        # global-coarsening hierarchy in place of local smoothing
        modes = {"fp64": dict(vcycle_fp32=0, cheb_degree=3, coarse_mode=0, coarse_its=30, mg_kind=0, prec_kind=0),
                 "mixed": dict(vcycle_fp32=1, cheb_degree=4, coarse_mode=1, coarse_its=30, mg_kind=0, prec_kind=0),
                 "mixed_cheb3": dict(vcycle_fp32=1, cheb_degree=3, coarse_mode=0, coarse_its=30, mg_kind=0,
                                     prec_kind=0),
                 "gc_fp64": dict(vcycle_fp32=0, cheb_degree=3, coarse_mode=0, coarse_its=30, mg_kind=1,
                                 prec_kind=0),
                 "gc_mixed": dict(vcycle_fp32=1, cheb_degree=4, coarse_mode=1, coarse_its=30, mg_kind=1,
                                  prec_kind=0),
                 # the block-triangular preconditioner (keeps the coupling block)
                 "tri_fp64": dict(vcycle_fp32=0, cheb_degree=3, coarse_mode=0, coarse_its=30, mg_kind=0,
                                  prec_kind=1)}
        modes = {k: v for k, v in modes.items() if k in args.newton_modes.split(",")}
        U_ref = None
        tcv_ref = None
        newton = {}
        for mode, cfg in modes.items():
            for k, v in cfg.items():
                setattr(sp_, k, v)
            g.set_params(sp_)
            # the timed step: one Newton / active-set iteration (Alg. 2: residual,
            # active set, multigrid setup, GMRES with the V-cycle, line search),
            # the first K iterations of the load step from its start
            act = torch.zeros(g.n, dtype=torch.uint8, device="cuda")
            Uw.copy_(U0)
            for _ in range(args.warmup):
                g.newton_step(Uw, phi0, phi0, act)
            Uw.copy_(U0)
            act.zero_()
            torch.cuda.synchronize()
            t_a = time.perf_counter()
            its, t_setup, t_solve = [], 0.0, 0.0
            for _ in range(args.steps):
                info, _ = g.newton_step(Uw, phi0, phi0, act)
                its.append(info["gmres_iterations"])
                t_setup += info["setup_seconds"]
                t_solve += info["solve_seconds"]
            torch.cuda.synchronize()
            t_b = time.perf_counter()
            newton[mode] = {"ms_per_newton_step": (t_b - t_a) / args.steps * 1e3, "gmres_iterations": its,
                            # multigrid setup (level states, diagonals, eigenvalue estimates) and the
                            # GMRES solve per step; the solve time per GMRES iteration (V-cycle,
                            # vmult, orthogonalisation)
                            "setup_ms": t_setup / args.steps * 1e3, "solve_ms": t_solve / args.steps * 1e3,
                            "ms_per_gmres_iteration": t_solve / max(sum(its), 1) * 1e3,
                            "level_nodes": list(g.level_nodes)}
            log(f"{mode}: Newton step {newton[mode]['ms_per_newton_step']:.1f} ms (gmres {its}; setup "
                f"{newton[mode]['setup_ms']:.1f} ms, {newton[mode]['ms_per_gmres_iteration']:.2f} ms per GMRES "
                f"iteration)")
            if args.no_load_step:
                continue
            # the whole load step to convergence (active set unchanged and
            # |R~| <= 1e-7), once
            Uw.copy_(U0)
            torch.cuda.synchronize()
            t_a = time.perf_counter()
            act, infos = solve_load_step(g, Uw, phi0, phi0, tol=1e-7, max_steps=400)
            torch.cuda.synchronize()
            t_b = time.perf_counter()
            tcv = g.tcv(Uw)
            conv = bool(infos[-1]["active_changed"] == 0 and infos[-1]["residual_before"] <= 1e-7)
            gm = [i["gmres_iterations"] for i in infos]
            solve[mode] = {
                "seconds": t_b - t_a,
                "converged": conv,
                "newton_steps": len(infos),
                "gmres_iterations_total": int(sum(gm)),
                "gmres_iterations_first_last": [gm[0], gm[-1]],
                "final_residual": infos[-1]["residual_before"],
                "n_active": infos[-1]["n_active"],
                "tcv": tcv,
                "tcv_rel_error_vs_sneddon": abs(tcv - tcv_sneddon(spec)) / tcv_sneddon(spec),
                "seconds_per_newton_step": (t_b - t_a) / len(infos),
                "settings": cfg,
            }
            if U_ref is None:
                U_ref, tcv_ref = Uw.clone(), tcv
            else:
                # error of the other configurations' load step against the FP64 one
                solve[mode]["rel_diff_U_vs_fp64"] = float(torch.linalg.norm(Uw - U_ref) / torch.linalg.norm(U_ref))
                solve[mode]["rel_diff_tcv_vs_fp64"] = abs(tcv - tcv_ref) / abs(tcv_ref)
            log(f"{mode}: load step "
                f"{solve[mode]['seconds']:.2f} s, {len(infos)} Newton steps (converged {conv}), "
                f"{solve[mode]['gmres_iterations_total']} GMRES iterations, final |R~| "
                f"{solve[mode]['final_residual']:.2e}, TCV {tcv:.6e} "
                f"({100 * solve[mode]['tcv_rel_error_vs_sneddon']:.2f} % from Sneddon's value)")
        if "fp64" not in newton:
            raise SystemExit("--newton-modes must include fp64 (the reported step)")
        ms_step = newton["fp64"]["ms_per_newton_step"]
        # V-cycle times at the state left by the last solve
        vsrc = torch.tensor(inputs.random_vector(X, Y, 3), device="cuda")
        vdst = torch.empty_like(vsrc)
        vc = {}
        for mode, cfg in modes.items():
            for k, v in cfg.items():
                setattr(sp_, k, v)
            g.set_params(sp_)
            g.set_state(Uw, phi0, phi0, None, setup_mg=True)
            vc[mode] = time_calls(lambda: g.vcycle(vsrc, fp32=bool(cfg["vcycle_fp32"]), out=vdst), 5, warm=2)
        extra = {"newton_step": newton, "load_step": solve, "vcycle_ms": vc}
    if ms_step is None:
        ms_step = ms_vmult

    out = {
        # value: the first quantity (vmult GDoF/s); the second (seconds per
        # Newton solve, FP64 against mixed precision) is in "load_step"
        "metric": "GDoF/s of matrix-free Jacobian vmult; s per Newton solve, FP64 vs mixed",
        "value": gdofs,
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": spec.name, "unknowns": n_dof, "degree": spec.degree,
                   "step": "one Newton / primal-dual active set iteration of the load step from its "
                           "start (residual, active set, MG setup, GMRES(30) with the block V-cycle, "
                           "line search), FP64, local-smoothing V-cycle; the global-coarsening V-cycle "
                           "is timed beside it (modes gc_*)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"leaf vmult = tile_kernel<{spec.degree}, double, MODE_J> + shared_fixup",
                     "algorithmic_bytes": algo, "vmult_us": ms_vmult * 1e3,
                     "vmult_us_median": med_vmult * 1e3,
                     # beside the required figures: the algorithmic fraction at the
                     # median call time, and the measured HBM traffic (counters) as
                     # a rate at the mean and median times
                     "frac_at_median": algo / (med_vmult * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic_gbs": traffic / (ms_vmult * 1e-3) / 1e9 if traffic else None,
                     "traffic_frac_at_median": (traffic / (med_vmult * 1e-3) / 1e9 / HBM_PEAK_GBS
                                                if traffic else None)},
    }
    out.update(extra)
    if args.scenario == "diff":
        out["scenario"] = scenario_diff(g, spec, sp_, log)
    elif args.scenario == "quasistatic":
        out["scenario"] = scenario_quasistatic(g, spec, sp_, args.increments, log, args.extrapolate)
    elif args.scenario == "table2":
        out["scenario"] = scenario_table2(log, args.table2_local_max, args.table2_kappa)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb = cpu_baseline()
        cb.pop("_check", None)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def solve_frozen(solver, U, phi_old, phi_tilde, active, tol=1e-10, max_steps=20):
    """Newton iterations with the active set held fixed (phi = phi_old on it):
    residual, GMRES with the V-cycle, hanging distribution; the re-solves of
    the finite-difference check of the adjoint. U is updated in place;
    returns the final masked residual norm."""
    import torch
    for _ in range(max_steps):
        solver.set_state(U, phi_old, phi_tilde, active, setup_mg=True)
        R = solver.residual(U, masked=True)
        r = float(torch.linalg.norm(R))
        if r <= tol:
            return r
        dU, info, rc = solver.gmres(R, tol=max(1e-3 * r, 1e-2 * tol))
        solver.distribute(dU, 3)
        U += dU
    solver.set_state(U, phi_old, phi_tilde, active, setup_mg=False)
    return float(torch.linalg.norm(solver.residual(U, masked=True)))


def scenario_diff(g, spec, sp_, log):
    """Differentiation form: a converged load step, 16 seeded vectors through
    vmult and vmult_T (batched), the adjoint gradient of TCV with respect to
    (Gc, E, p) by a transposed GMRES solve, and central differences with
    relative step 1e-6 of TCV from re-solves with the active set frozen."""
    import numpy as np
    import torch

    import inputs
    from paper_2404_03265_amd.autograd import adjoint_tcv_gradient, solve_load_step
    X, Y = g.coords()
    U, phi0, _, _ = make_state(g, spec, random=False)
    for k, v in dict(vcycle_fp32=0, cheb_degree=3, coarse_mode=0, coarse_its=30,
                     gmres_rtol=1e-10, gmres_atol=1e-14).items():
        setattr(sp_, k, v)
    g.set_params(sp_)
    t0 = time.perf_counter()
    active, infos = solve_load_step(g, U, phi0, phi0, tol=1e-11, max_steps=400)
    t_solve = time.perf_counter() - t0
    g.set_state(U, phi0, phi0, active, setup_mg=True)
    n_dof = 3 * g.n
    V = torch.tensor(np.concatenate([inputs.random_vector(X, Y, 100 + i) for i in range(16)]), device="cuda")
    W = torch.empty_like(V)
    ms_fwd = time_calls(lambda: [g.vmult(V[i * n_dof:(i + 1) * n_dof], W[i * n_dof:(i + 1) * n_dof])
                                 for i in range(16)], 5, warm=2)
    ms_T = time_calls(lambda: g.vmult_T(V, batch=16, out=W), 5, warm=2)
    # transpose identity on the batch: z^T (J v) = (J^T z)^T v
    Jv = torch.empty_like(V)
    for i in range(16):
        g.vmult(V[i * n_dof:(i + 1) * n_dof], Jv[i * n_dof:(i + 1) * n_dof])
    JTv = g.vmult_T(V, batch=16)
    z = V[:n_dof]
    worst = 0.0
    for i in range(16):
        v = V[i * n_dof:(i + 1) * n_dof]
        a = float(torch.dot(z, Jv[i * n_dof:(i + 1) * n_dof]))
        b = float(torch.dot(JTv[:n_dof], v))
        worst = max(worst, abs(a - b) / max(abs(a), 1e-300))
    t0 = time.perf_counter()
    tcv, grad, _, ginfo = adjoint_tcv_gradient(g, U, phi0, phi0, active)
    t_adj = time.perf_counter() - t0
    grad = grad.cpu().numpy()
    names = ("Gc", "E", "pressure")
    fd = {}
    err = {}
    for h in (1e-6, 1e-4):
        fd[h] = []
        for k, name in enumerate(names):
            base = getattr(sp_, name)
            vals = []
            for sgn in (1.0, -1.0):
                setattr(sp_, name, base * (1.0 + sgn * h))
                g.set_params(sp_)
                Ut = U.clone()
                solve_frozen(g, Ut, phi0, phi0, active, tol=1e-13)
                vals.append(g.tcv(Ut))
            setattr(sp_, name, base)
            g.set_params(sp_)
            fd[h].append((vals[0] - vals[1]) / (2.0 * h * base))
        # difference in units of TCV / theta (a zero derivative stays meaningful)
        err[h] = [abs(grad[k] - fd[h][k]) * getattr(sp_, names[k]) / abs(tcv) for k in range(3)]
    log(f"diff: load step {t_solve:.2f} s, vmult x16 {ms_fwd:.2f} ms, vmult_T batch 16 {ms_T:.2f} ms, "
        f"adjoint {t_adj:.2f} s, grad {grad}, fd(1e-6) {fd[1e-6]}, err {err[1e-6]}, fd(1e-4) {fd[1e-4]}, "
        f"err {err[1e-4]}")
    return {
        "name": "diff", "workload": spec.name, "load_step_seconds": t_solve, "newton_steps": len(infos),
        "vmult_16_ms": ms_fwd, "vmult_T_batch16_ms": ms_T,
        "vmult_T_gdofs_per_vector": 16 * n_dof / (ms_T * 1e-3) / 1e9,
        "transpose_identity_worst_rel": worst,
        "tcv": tcv, "adjoint_seconds": t_adj, "adjoint_gmres_iterations": ginfo["iterations"],
        "grad_Gc_E_p": [float(x) for x in grad],
        "fd_h1e-6_Gc_E_p": [float(x) for x in fd[1e-6]], "fd_h1e-4_Gc_E_p": [float(x) for x in fd[1e-4]],
        "err_vs_fd_h1e-6": [float(x) for x in err[1e-6]], "err_vs_fd_h1e-4": [float(x) for x in err[1e-4]],
        "err_units": "|adjoint - central difference| * theta / TCV",
    }


def scenario_quasistatic(g, spec, sp_, increments, log, extrapolate=False):
    """Pressure increments p = 1e-3 k (k = 1..K): each load step solved by
    Newton / active set iterations from the previous solution, phi_old the
    previous step's phase field, phi~ = phi_old or (extrapolate) the linear
    extrapolation from the last two steps, active set carried over; FP32
    V-cycle (Chebyshev 4, coarse CG), FP64 outer loop; adjoint gradient of
    TCV at the last step."""
    import torch

    from paper_2404_03265_amd.autograd import adjoint_tcv_gradient, solve_load_path
    U, phi0, _, _ = make_state(g, spec, random=False)
    for k, v in dict(vcycle_fp32=1, cheb_degree=4, coarse_mode=1, coarse_its=30).items():
        setattr(sp_, k, v)
    g.set_params(sp_)
    pressures = [1e-3 * k for k in range(1, increments + 1)]
    steps = []
    clock = {"t": time.perf_counter()}

    def progress(k, j, info):
        if j % 10 == 0:
            log(f"  increment {k + 1}: {j} Newton steps, |R~| {info['residual_before']:.2e}, "
                f"{info['n_active']} active")

    def record(k, phi_tilde, infos):
        torch.cuda.synchronize()
        now = time.perf_counter()
        dt, clock["t"] = now - clock["t"], now
        tcv = g.tcv(U)
        steps.append({"pressure": pressures[k], "seconds": dt, "newton_steps": len(infos),
                      "gmres_iterations": [i["gmres_iterations"] for i in infos],
                      "final_residual": infos[-1]["residual_before"], "n_active": infos[-1]["n_active"],
                      "tcv": tcv})
        log(f"increment {k + 1}: p={pressures[k]:.0e} {dt:.2f} s, {len(infos)} Newton steps, "
            f"gmres {steps[-1]['gmres_iterations']}, |R~| {steps[-1]['final_residual']:.2e}, TCV {tcv:.6e}")
        clock["t"] = time.perf_counter()

    torch.cuda.synchronize()
    t_all = time.perf_counter()
    clock["t"] = t_all
    active, out = solve_load_path(g, U, phi0, pressures, extrapolate=extrapolate, tol=1e-7,
                                  progress=progress, done=record)
    total = time.perf_counter() - t_all
    phi_old = out[-1][2]
    phi_tilde = out[-1][0]
    t0 = time.perf_counter()
    tcv, grad, _, ginfo = adjoint_tcv_gradient(g, U, phi_old, phi_tilde, active)
    t_adj = time.perf_counter() - t0
    log(f"adjoint at the last step: {t_adj:.2f} s, {ginfo['iterations']} GMRES iterations, grad {grad.tolist()}")
    return {"name": "quasistatic", "workload": spec.name, "extrapolated_phi_tilde": bool(extrapolate),
            "increments": steps, "total_seconds": total,
            "adjoint_seconds": t_adj, "adjoint_gmres_iterations": ginfo["iterations"],
            "grad_Gc_E_p": [float(x) for x in grad.tolist()]}


def scenario_table2(log, local_max=8, kappa="1e-10"):
    """The Sneddon test on the paper's mesh family (Sec. 4, Tables 1 and 2): Q1
    on a 40 x 40 base mesh (a 10 x 10 coarse grid with 2 global refinements)
    and 0..local_max local refinements of the cells with centres in |x| < 3,
    |y| < 1 (unknown counts within 10 % of Table 2's); l = 2h with h the
    finest cell diagonal, p = 1e-3, Newton tolerance 1e-7 (Table 1); kappa =
    1e-10 (the workloads' value) or, with kappa="paper", 1e-12 h (Table 1).
    Per mesh, one load step from its start in the FP64 configuration (at most
    100 Newton steps): unknowns, TCV error against Sneddon's value, Newton
    steps, mean and largest GMRES iterations per Newton step, GPU wall time."""
    import math

    import torch

    import inputs
    from paper_2404_03265_amd import PhaseFieldSolver, SolverParams
    from paper_2404_03265_amd.autograd import solve_load_step
    rows = []
    for L in range(local_max + 1):
        base = inputs.WorkloadSpec(name="", n_base=40, n_local=L, degree=1)
        h = math.sqrt(2.0) * base.finest_edge
        kap = 1e-12 * h if kappa == "paper" else float(kappa)
        spec = inputs.WorkloadSpec(name=f"sneddon_40x40_L{L}_Q1", n_base=40, n_local=L, degree=1,
                                   kappa=kap, coarse=10, band=(3.0, 1.0))
        sp = SolverParams(E=spec.E, nu=spec.nu, Gc=spec.Gc, pressure=spec.pressure, kappa=spec.kappa,
                          ell=spec.ell)
        g = PhaseFieldSolver(spec.n_base, spec.n_local, spec.degree, coarse=spec.coarse, band=spec.band, params=sp)
        U, phi0, _, _ = make_state(g, spec, random=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        def progress(j, info, L=L):
            if j % 10 == 0:
                log(f"  table2 L={L}: {j} Newton steps, |R~| {info['residual_before']:.2e}, "
                    f"GMRES {info['gmres_iterations']}")
        act, infos = solve_load_step(g, U, phi0, phi0, tol=1e-7, max_steps=100, progress=progress)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tcv = g.tcv(U)
        gm = [i["gmres_iterations"] for i in infos]
        ref = tcv_sneddon(spec)
        # COD(x) (Sec. 4) across the crack against Sneddon's opening
        xs = [-0.75, -0.5, -0.25, 0.0, 0.25, 0.5, 0.75]
        cod = [float(v) for v in g.cod(U, xs)]
        cod_ref = [cod_sneddon(spec, x) for x in xs]
        row = {"local_levels": L, "h": h, "kappa": kap, "unknowns": 3 * g.n, "tcv": tcv,
               "tcv_error": abs(tcv - ref) / ref, "cod_x": xs, "cod": cod, "cod_ref": cod_ref,
               "cod_error_x0": abs(cod[3] - cod_ref[3]) / cod_ref[3], "newton_steps": len(infos),
               "converged": bool(infos[-1]["active_changed"] == 0 and infos[-1]["residual_before"] <= 1e-7),
               "mean_gmres": sum(gm) / len(gm), "max_gmres": max(gm), "seconds": dt}
        rows.append(row)
        log(f"table2 L={L}: h {h:.4f}, {row['unknowns']} unknowns, TCV error {100 * row['tcv_error']:.2f} %, "
            f"COD(0) error {100 * row['cod_error_x0']:.2f} %, "
            f"{len(infos)} Newton steps, GMRES mean {row['mean_gmres']:.2f} max {row['max_gmres']}, {dt:.2f} s")
        g.close()
        del g
    return {"name": "table2", "kappa": kappa, "rows": rows}


if __name__ == "__main__":
    main()
