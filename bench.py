"""Benchmark: FMG Stokes solve at discretisation accuracy on one MI355X.

Workload (one step = one full FMG solve, Alg. fmg of the paper): P2-P1
Taylor-Hood Stokes on the unit cube split into 6 Kuhn macro-tetrahedra,
refinement level 5 (32 intervals per macro edge, 859,812 DoFs including the
Dirichlet velocity DoFs), analytic cube solution of the paper (Sec. 5.1.1),
FMG(1, 3, 0, 1, A_f, 3) from coarsest level 1 -- the least-work tuple of the
paper's 768-tuple search space (Sec. 5.1) that solves to discretisation
accuracy, gamma_u and gamma_p <= 2 (eq. gamma), on this mesh and ordering.
float64, inputs resident in HBM.

Printed JSON line: value = DoF / s of the whole solve; roofline of the
dominant kernel family of the step (HIP-event timed, algorithmic bytes);
accuracy of the result (gamma_u, gamma_p against a float64 solve converged to
1e-12 on the GPU, errors of eq. error); two cheaper tuples with their
rates and gammas; the M_L reading of the Schur scaling; the relative error of
eq. relative-error on a seeded Fourier forcing; the operator apply's HBM
roofline at the largest throughput size (P2-P1, 48 tets, level 7); and the
CPU oracle timed on the same workload on one and on all host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
       python bench.py --mode {apply,dc,learned,sweep,c3,umesh}

--mode umesh: the cube benchmark exactly as the paper configures it (Sec.
5.1.1): P1-P1 PSPG on the unit cube split into 24 tetrahedra, level 6
(4.29e6 DoFs), on the library's unstructured (per-cell) path, with the
paper's three P1-P1 tuples of Tab. fmg-table.
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
# FMG tuples (nu_pre, nu_post, nu_inc, kappa, A_hat, xi): the headline is the
# least-work tuple of the 768-tuple search space (Sec. 5.1) whose solution
# meets gamma_u, gamma_p <= 2 (eq. gamma) on this workload, and also the one of
# least GPU time among them; the others are the least-work and the least-time
# tuples under the loosest bounds of Tab. fmg-table (2, 10) and the paper's own
# tuple for those bounds.
HEADLINE = (1, 3, 0, 1, 0, 3)
ALTERNATIVES = [((0, 1, 3, 1, 0, 3), "least work with gamma_u <= 2, gamma_p <= 10"),
                ((1, 3, 0, 1, 0, 2), "least GPU time with gamma_u <= 2, gamma_p <= 10"),
                ((0, 2, 1, 1, 0, 3), "the paper's P2-P1 tuple for gamma bounds (2, 10)")]
# HBM traffic of one launch of a kernel family from rocprofv3 counters
# (FETCH_SIZE x 2 + WRITE_SIZE, per dispatch, the calibration factor of a plain
# copy applied); valid for the kernel code the summary names.
TRAFFIC = {
    "gs_edge_colour": {"bytes_per_launch": 3.0e6,
                       "source": "profiles/fmg_p2p1_level5_cube.md: FETCH_SIZE x 2 + WRITE_SIZE per k_gs_edge "
                                 "dispatch, weighted with the solve's launch mix over levels 3-5"},
}
APPLY_TRAFFIC = {"f64": 10.81e9, "f32": 4.66e9}   # profiles/apply_p2p1_48tets_level7.md
# algorithmic bytes per work unit (float64 words), see the design doc
WORDS = {
    "apply_p2": 6.25,        # y = calA x per P2 site
    "gs_colour": 9.0,        # per updated site: u read + u write + f read (3 components)
}


def _tname(s):
    return f"({s[0]},{s[1]},{s[2]},{s[3]},{'A_f' if s[4] == 0 else 'A_s'},{s[5]})"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--level", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-apply-roofline", action="store_true")
    ap.add_argument("--mode", choices=["fmg", "apply", "learned", "dc", "sweep", "c3", "umesh"], default="fmg",
                    help="apply: only the operator-apply roofline (for counter runs); learned: the "
                         "learned coarse-solve workload (pairs, GPU training, held-out evaluation)")
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--hidden", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=100)
    ap.add_argument("--test-seeds", type=int, default=1000)
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--sweep-out", default=None, help="sweep: write every row of the study to this JSON file")
    ap.add_argument("--profile", action="store_true",
                    help="profiler runs: setup, the timed headline solves and a 1 GiB calibration copy only")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2010_13513_amd import hhg, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    L, lmin = args.level, 1
    prob = W.paper_cube()

    ctx = hhg.hhg_ctx_create(0, stream.cuda_stream)
    if args.mode == "umesh":
        res = bench_umesh(torch, hhg, dev, stream, ctx, args)
        print(json.dumps(res), flush=True)
        hhg.hhg_ctx_destroy(ctx)
        return
    if args.mode == "dc":
        res = bench_dc(torch, hhg, ctx, level=args.level if args.level != 5 else 7)
        print(json.dumps(res), flush=True)
        hhg.hhg_ctx_destroy(ctx)
        return
    if args.mode == "c3":
        res = bench_c3(torch, hhg, dev, stream, ctx, levels=(5, 6, 7))
        print(json.dumps(res), flush=True)
        hhg.hhg_ctx_destroy(ctx)
        return
    if args.mode == "sweep":
        res = bench_sweep(torch, hhg, ctx, args)
        print(json.dumps(res), flush=True)
        hhg.hhg_ctx_destroy(ctx)
        return
    if args.mode == "learned":
        res = bench_learned(torch, hhg, ctx, args)
        print(json.dumps(res), flush=True)
        hhg.hhg_ctx_destroy(ctx)
        return
    if args.mode == "apply":
        res = bench_apply(torch, hhg, dev, stream, ctx, reps=args.apply_reps)
        # plain copy of a known size (calibration of the HBM byte counters)
        n = 1 << 27
        a = torch.ones(n, dtype=torch.float64, device=dev)
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {n * 8} bytes read, {n * 8} bytes written per launch")
        print(json.dumps({"apply_roofline": res}), flush=True)
        hhg.hhg_ctx_destroy(ctx)
        return
    mesh = hhg.hhg_mesh_cube(ctx, 0)
    H = hhg.hhg_hier_create(mesh, hhg.HHG_P2P1, lmin, L, hhg.HHG_SCHUR_SD)
    Hml = hhg.hhg_hier_create(mesh, hhg.HHG_P2P1, lmin, L, hhg.HHG_SCHUR_ML)    # the M_L reading of S_hat
    Ev = hhg.hhg_hier_create(mesh, hhg.HHG_P2P1, L, L + 1, hhg.HHG_SCHUR_SD)   # error evaluation only
    hhg.hhg_mesh_destroy(mesh)

    def lattice_fields(level, fn_u, fn_p=None):
        N = 2 ** level
        g = np.arange(2 * N + 1) / (2.0 * N)
        Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
        u = fn_u(X.ravel(), Y.ravel(), Z.ravel())
        gp = np.arange(N + 1) / float(N)
        Zp, Yp, Xp = np.meshgrid(gp, gp, gp, indexing="ij")
        p = np.zeros(Xp.size) if fn_p is None else fn_p(Xp.ravel(), Yp.ravel(), Zp.ravel())
        return np.concatenate([u[0], u[1], u[2], p])

    def upload(hier, level, arr):
        _, _, vw, _ = hhg.hhg_vec_layout(hier, level)
        dst = torch.zeros(vw, dtype=torch.float64, device=dev)
        hhg.hhg_vec_from_lattice(hier, level, torch.from_numpy(arr).to(dev), dst)
        return dst

    def rhs_levels(problem):
        out = []
        for l in range(lmin, L + 1):
            f_nod = upload(H, l, lattice_fields(l, problem.f))
            b = torch.zeros_like(f_nod)
            hhg.hhg_rhs(H, l, f_nod, b)
            out.append(b)
        return out

    # ---- inputs (setup, not timed): right-hand sides of every level, boundary data
    bs = rhs_levels(prob)
    x0 = upload(H, L, lattice_fields(L, prob.u))      # boundary data (interior ignored)
    v0 = torch.from_numpy(W.normal_vector(W.SEED_BASE + 1000, (2 ** L + 1) ** 3)).to(dev)
    omega_inv = hhg.hhg_estimate_omega(H, L, v0, 100)
    x = torch.zeros_like(x0)
    N = 2 ** L
    dofs = 3 * (2 * N + 1) ** 3 + (N + 1) ** 3
    log(f"[bench] workload P2-P1 L={L} dofs={dofs} omega_inv={omega_inv:.6f}")

    # ---- accuracy: eq. error on level L+1, gamma against a converged solve
    xs_fine = upload(Ev, L + 1, lattice_fields(L + 1, prob.u, prob.p))

    def errors(xL):
        e = torch.zeros_like(xs_fine)
        hhg.hhg_prolong_add(Ev, L, xL, e)
        e -= xs_fine
        hhg.hhg_project_mean_zero(Ev, L + 1, e)
        me = torch.empty_like(e)
        hhg.hhg_apply(Ev, L + 1, hhg.HHG_OP_MASS, e, me)
        du, dp = hhg.hhg_dots(Ev, L + 1, e, me)
        return float(np.sqrt(du)), float(np.sqrt(dp))

    if args.profile:
        prm = hhg.solver_params(*HEADLINE, omega_inv)
        for q in range(args.warmup + args.steps):
            x.copy_(x0)
            hhg.hhg_fmg_solve(H, x, bs, prm, want_stats=False)
        torch.cuda.synchronize()
        n = 1 << 27
        a = torch.ones(n, dtype=torch.float64, device=dev)
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] profile run: {args.warmup + args.steps} FMG{_tname(HEADLINE)} solves; calibration copy "
            f"{n * 8} bytes read and written per launch")
        for hh in (Ev, Hml, H):
            hhg.hhg_hier_destroy(hh)
        hhg.hhg_ctx_destroy(ctx)
        return
    xd = x0.clone()
    st = hhg.hhg_fmg_solve(H, xd, bs, hhg.solver_params(3, 3, 0, 1, hhg.HHG_GS_FWD, 3, omega_inv, rtol=1e-12,
                                                        max_cycles=200))
    eud, epd = errors(xd)
    log(f"[bench] discrete solution ({st.cycles} cycles, rel res {st.rel_res:.1e}): errors u {eud:.4e} p {epd:.4e}")

    def run_tuple(s, steps, warmup, hier=H, om=omega_inv):
        """Time `steps` graph-replayed FMG solves of tuple s; gamma of the result."""
        prm = hhg.solver_params(*s, om)

        def step():
            x.copy_(x0)
            hhg.hhg_fmg_solve(hier, x, bs, prm, want_stats=False)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        eu, ep = errors(x)
        xw = x0.clone()
        wu = hhg.hhg_fmg_solve(hier, xw, bs, prm).work_units
        return ms, eu, ep, wu, step

    ms_step, eu, ep, wu, step = run_tuple(HEADLINE, args.steps, args.warmup)
    value = dofs / (ms_step * 1e-3)
    gamma_u, gamma_p = eu / eud, ep / epd
    log(f"[bench] FMG{_tname(HEADLINE)} ({wu:.2f} WU): {args.steps} steps {ms_step:.3f} ms/step, {value:.3e} DoF/s, "
        f"gamma_u {gamma_u:.3f} gamma_p {gamma_p:.3f}")
    alternatives = []
    for s_alt, why in ALTERNATIVES:
        ms_a, eu_a, ep_a, wu_a, _ = run_tuple(s_alt, max(5, args.steps // 2), 2)
        alternatives.append({"fmg": _tname(s_alt), "why": why, "work_units": round(wu_a, 3),
                             "ms_per_solve": round(ms_a, 4), "dofs_per_s": dofs / (ms_a * 1e-3),
                             "gamma_u": round(eu_a / eud, 4), "gamma_p": round(ep_a / epd, 4)})
        log(f"[bench] FMG{_tname(s_alt)} ({why}): {ms_a:.3f} ms, {dofs / (ms_a * 1e-3):.3e} DoF/s, "
            f"gamma ({eu_a / eud:.3f}, {ep_a / epd:.3f})")

    # ---- the M_L reading of S_hat (eq. omega-eigenvalue-problem) with the headline tuple
    om_ml = hhg.hhg_estimate_omega(Hml, L, v0, 100)
    ms_ml, eu_ml, ep_ml, _, _ = run_tuple(HEADLINE, 5, 2, hier=Hml, om=om_ml)
    schur_ml = {"omega_inv": om_ml, "gamma_u": round(eu_ml / eud, 4), "gamma_p": round(ep_ml / epd, 4),
                "ms_per_solve": round(ms_ml, 4)}
    log(f"[bench] M_L reading: omega_inv {om_ml:.4f}, gamma ({eu_ml / eud:.3f}, {ep_ml / epd:.3f})")

    # ---- eq. relative-error on the seeded Fourier forcing (u = 0 on the boundary)
    fprob = W.fourier_forcing(W.SEED_BASE + 2000)
    bsf = rhs_levels(fprob)
    xf0 = torch.zeros_like(x0)
    xref = xf0.clone()
    stf = hhg.hhg_fmg_solve(H, xref, bsf, hhg.solver_params(3, 3, 0, 1, hhg.HHG_GS_FWD, 3, omega_inv, rtol=1e-12,
                                                            max_cycles=200))
    xt = xf0.clone()
    hhg.hhg_fmg_solve(H, xt, bsf, hhg.solver_params(*HEADLINE, omega_inv))

    def mnorm2(v):
        mv = torch.empty_like(v)
        hhg.hhg_apply(H, L, hhg.HHG_OP_MASS, v, mv)
        return hhg.hhg_dots(H, L, v, mv)
    du, dp = mnorm2(xt - xref)
    ru, rp = mnorm2(xref)
    delta = {"forcing": "8 Fourier modes, k in {-4..4}^3, N(0,1)/|k|^2 amplitudes, u = 0 on the boundary",
             "delta_u": float(np.sqrt(du / ru)), "delta_p": float(np.sqrt(dp / rp)),
             "reference": f"FMG + V(3,3) cycles to rel. residual {stf.rel_res:.1e}"}
    log(f"[bench] relative error (Fourier forcing): delta_u {delta['delta_u']:.3e} delta_p {delta['delta_p']:.3e}")

    # ---- roofline of the dominant kernel family (HIP events on the solve stream)
    fams = {hhg.KF_APPLY: "apply_residual", hhg.KF_PROW_BND: "boundary_pressure_rows",
            hhg.KF_GS_VERTEX: "gs_vertex_colour", hhg.KF_GS_EDGE: "gs_edge_colour", hhg.KF_PSTEP: "uzawa_pressure_step",
            hhg.KF_RESTRICT: "restrict", hhg.KF_PROLONG: "prolong", hhg.KF_COARSE: "coarse_gemv",
            hhg.KF_REDUCE: "reductions", hhg.KF_OTHER: "other", hhg.KF_SMALL: "small_level_vcycle"}
    rsteps = max(2, min(args.steps, 5))
    hhg.hhg_timer_start(sum(1 << f for f in fams))
    for _ in range(rsteps):
        step()
    torch.cuda.synchronize()
    per_fam = {}
    for f, name in fams.items():
        ms, n, units = hhg.hhg_timer_read(f)
        per_fam[name] = (ms / rsteps, n // rsteps, units / rsteps)
    hhg.hhg_timer_start(0)
    dom = max(("gs_edge_colour", "gs_vertex_colour", "apply_residual"), key=lambda k: per_fam[k][0])
    ms_d, n_d, units_d = per_fam[dom]
    words = WORDS["gs_colour"] if dom.startswith("gs_") else WORDS["apply_p2"]
    bytes_launch = units_d / max(n_d, 1) * words * 8
    avg_ms = ms_d / max(n_d, 1)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    log("[bench] kernel families per step: " + ", ".join(
        f"{k} {v[0]:.3f} ms/{v[1]}" for k, v in sorted(per_fam.items(), key=lambda kv: -kv[1][0])))
    traffic = TRAFFIC.get(dom)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic["bytes_per_launch"] if traffic else None,
                "avg_launch_us": round(avg_ms * 1e3, 3), "bytes_per_launch": int(bytes_launch),
                "launches_per_step": n_d, "share_of_step": round(ms_d / ms_step, 3),
                "timing": ("HIP events stamped by each launch's dispatch packet (kernel start to end)"
                           if dom.startswith("gs_") else "HIP events recorded around each launch")}
    if traffic:
        roofline["traffic_source"] = traffic["source"]

    # ---- P1-P1: a solve at discretisation accuracy within 10 work units
    p1_solved = bench_p1_solved(torch, hhg, ctx, stream, steps=max(5, args.steps // 2))

    # ---- operator-apply HBM roofline at the throughput size (48 tets, level 7)
    apply_roofline = None
    if not args.no_apply_roofline:
        apply_roofline = bench_apply(torch, hhg, dev, stream, ctx)

    out = {
        "metric": "FMG Stokes DoF/s at discretization accuracy; operator-apply HBM GB/s vs peak",
        "value": value, "unit": "DoF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"P2-P1 Taylor-Hood Stokes, unit cube, 6 Kuhn macro-tets, level {L} "
                               f"({dofs} DoFs), paper cube solution, FMG{_tname(HEADLINE)} from level 1 "
                               "(least work with gamma_u, gamma_p <= 2 over the 768-tuple search space)",
                   "dofs": dofs, "level": L, "fmg": _tname(HEADLINE), "omega_inv": omega_inv, "schur": "SD",
                   "work_units": round(wu, 3), "gamma_u": round(gamma_u, 4), "gamma_p": round(gamma_p, 4),
                   "err_u": eu, "err_p": ep, "disc_err_u": eud, "disc_err_p": epd},
        "alternatives": alternatives,
        "schur_ml": schur_ml,
        "relative_error": delta,
        "p1p1_solved": p1_solved,
        "roofline": roofline,
    }
    if apply_roofline:
        out["apply_roofline"] = apply_roofline
    hhg.hhg_hier_destroy(Ev)
    hhg.hhg_hier_destroy(Hml)
    hhg.hhg_hier_destroy(H)
    hhg.hhg_ctx_destroy(ctx)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(L, omega_inv)
    print(json.dumps(out), flush=True)


# The least-work tuple of the 768-tuple search space whose P1-P1 level-6
# result meets gamma_u, gamma_p <= 2 (the sweep's Tab. fmg-table row (2, 2))
P1_SOLVED = (1, 0, 1, 1, 0, 3)


def bench_p1_solved(torch, hhg, ctx, stream, steps=10, warmup=2, L=6):
    """P1-P1 PSPG, 6 Kuhn macro-tets, level 6 (1,098,500 DoFs), paper cube
    solution, coarsest level 0: FMG with P1_SOLVED (graph-replayed), its work
    units and gammas (eq. gamma against a solve converged to 1e-12)."""
    from paper_2010_13513_amd import study, workloads as W
    from paper_2010_13513_amd.problem import Problem
    prob = W.paper_cube()
    P = Problem(torch, ctx, hhg.HHG_P1P1, 0, L)
    try:
        v0 = torch.from_numpy(W.normal_vector(W.SEED_BASE + 1000, (2 ** L + 1) ** 3)).to(P.dev)
        om = hhg.hhg_estimate_omega(P.h, L, v0, 100)
        bs = P.rhs(prob)
        x0 = P.boundary(prob)
        gev = study.GammaEvaluator(torch, P, prob)
        try:
            xd, _ = study.discrete_solution(P, bs, x0, om)
            ed = gev.errors(xd)
            prm = hhg.solver_params(*P1_SOLVED, om)
            x = torch.empty_like(x0)

            def step():
                x.copy_(x0)
                hhg.hhg_fmg_solve(P.h, x, bs, prm, want_stats=False)
            for _ in range(warmup):
                step()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                step()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            eu, ep = gev.errors(x)
            wu = hhg.hhg_fmg_solve(P.h, x0.clone(), bs, prm).work_units
            dofs = P.dofs(L)
            res = {"workload": f"P1-P1 PSPG Stokes, unit cube, 6 Kuhn macro-tets, level {L} ({dofs} DoFs), paper "
                               "cube solution, coarsest level 0",
                   "fmg": _tname(P1_SOLVED), "work_units": round(wu, 3), "omega_inv": om,
                   "gamma_u": round(eu / ed[0], 4), "gamma_p": round(ep / ed[1], 4), "ms_per_solve": round(ms, 4),
                   "dofs_per_s": dofs / (ms * 1e-3)}
            log(f"[bench] P1-P1 level {L} FMG{_tname(P1_SOLVED)} ({wu:.2f} WU): {ms:.3f} ms, "
                f"{res['dofs_per_s']:.3e} DoF/s, gamma ({res['gamma_u']:.3f}, {res['gamma_p']:.3f})")
            return res
        finally:
            gev.close()
    finally:
        P.close()


def bench_apply(torch, hhg, dev, stream, ctx, level=7, reps=20):
    """y = calA x, P2-P1 on the 48-tet cube at the given macro level
    (N = 2^(level+1) intervals), float64 and float32, N(0,1) input."""
    res = {}
    mesh = hhg.hhg_mesh_cube(ctx, 1)
    H = hhg.hhg_hier_create(mesh, hhg.HHG_P2P1, level - 1, level, hhg.HHG_SCHUR_SD)
    hhg.hhg_mesh_destroy(mesh)
    try:
        N, nn, vw, lw = hhg.hhg_vec_layout(H, level)
        sites = (2 * N + 1) ** 3
        g = torch.Generator(device=dev).manual_seed(13513 + 3000)
        lat = torch.randn(lw, generator=g, dtype=torch.float64, device=dev)
        for prec, dt, name in ((hhg.HHG_F64, torch.float64, "f64"), (hhg.HHG_F32, torch.float32, "f32")):
            x = torch.zeros(vw, dtype=dt, device=dev)
            hhg.hhg_vec_from_lattice(H, level, lat, x, prec)
            y = torch.empty_like(x)
            for _ in range(3):
                hhg.hhg_apply(H, level, hhg.HHG_OP_FULL, x, y, prec)
            hhg.hhg_timer_start(1 << hhg.KF_APPLY)
            for _ in range(reps):
                hhg.hhg_apply(H, level, hhg.HHG_OP_FULL, x, y, prec)
            torch.cuda.synchronize()
            ms, n, _ = hhg.hhg_timer_read(hhg.KF_APPLY)
            hhg.hhg_timer_start(0)
            avg = ms / n
            b = sites * 6.25 * (8 if prec == hhg.HHG_F64 else 4)
            gbs = b / (avg * 1e-3) / 1e9
            res[name] = {"achieved": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4), "avg_launch_ms": round(avg, 4),
                         "bytes_per_launch": int(b), "traffic": APPLY_TRAFFIC[name] if level == 7 else None}
            del x, y
        res.update({"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "workload": f"P2-P1 apply, 48 macro-tets, level {level} ({sites} P2 sites)"})
        log(f"[bench] apply roofline: {res}")
    finally:
        hhg.hhg_hier_destroy(H)
    return res


# algorithmic words per unit (P2 site / P1 node) of the throughput kernels:
# each vector word touched once (apply: x in, y out; residual: + b; one Uzawa
# iteration with xi fused velocity sweeps; restriction / prolong-add per fine
# site)
C3_WORDS = {
    2: {"apply": 6.25, "residual": 9.375, "uzawa_xi1": 9.125 + 3.375, "uzawa_xi3": 3 * 9.125 + 3.375,
        "restrict": 3.125 * 9 / 8, "prolong_add": 6.6},
    1: {"apply": 8.0, "residual": 12.0, "uzawa_xi1": 10.0 + 6.0, "uzawa_xi3": 30.0 + 6.0,
        "restrict": 4.5, "prolong_add": 8.5},
}


def bench_c3(torch, hhg, dev, stream, ctx, levels=(5, 6, 7), reps=5):
    """Operator and smoother throughput on the 48-tet cube (one Bey step of
    the Kuhn cube) at macro levels 5..7 (N = 64..256), P1-P1 and P2-P1,
    float64 and float32, seeded N(0,1) inputs: time per call (torch events on
    the library's stream) and algorithmic GB/s of apply, residual, one Uzawa
    iteration (A_f, xi = 1 and 3), restriction and prolong-add."""
    rows = []
    for disc, vo, name in ((hhg.HHG_P1P1, 1, "P1-P1"), (hhg.HHG_P2P1, 2, "P2-P1")):
        for level in levels:
            mesh = hhg.hhg_mesh_cube(ctx, 1)
            H = hhg.hhg_hier_create(mesh, disc, level - 1, level, hhg.HHG_SCHUR_SD)
            hhg.hhg_mesh_destroy(mesh)
            try:
                N, nn, vw, lw = hhg.hhg_vec_layout(H, level)
                Nc, _, vwc, lwc = hhg.hhg_vec_layout(H, level - 1)
                sites = (vo * N + 1) ** 3
                g = torch.Generator(device=dev).manual_seed(13513 + 3000 + level)
                lat = torch.randn(lw, generator=g, dtype=torch.float64, device=dev)
                latb = torch.randn(lw, generator=g, dtype=torch.float64, device=dev)
                latc = torch.randn(lwc, generator=g, dtype=torch.float64, device=dev)
                for prec, dt, pname in ((hhg.HHG_F64, torch.float64, "f64"), (hhg.HHG_F32, torch.float32, "f32")):
                    x = torch.zeros(vw, dtype=dt, device=dev)
                    b = torch.zeros_like(x)
                    y = torch.empty_like(x)
                    xc = torch.zeros(vwc, dtype=dt, device=dev)
                    hhg.hhg_vec_from_lattice(H, level, lat, x, prec)
                    hhg.hhg_vec_from_lattice(H, level, latb, b, prec)
                    hhg.hhg_vec_from_lattice(H, level - 1, latc, xc, prec)
                    calls = {
                        "apply": lambda: hhg.hhg_apply(H, level, hhg.HHG_OP_FULL, x, y, prec),
                        "residual": lambda: hhg.hhg_residual(H, level, x, b, y, prec),
                        "uzawa_xi1": lambda: hhg.hhg_smooth(H, level, x, b, 1, hhg.HHG_GS_FWD, 1, 2.0, prec),
                        "uzawa_xi3": lambda: hhg.hhg_smooth(H, level, x, b, 1, hhg.HHG_GS_FWD, 3, 2.0, prec),
                        "restrict": lambda: hhg.hhg_restrict(H, level, x, xc, prec),
                        "prolong_add": lambda: hhg.hhg_prolong_add(H, level - 1, xc, y, prec),
                    }
                    for kname, fn in calls.items():
                        fn()
                        torch.cuda.synchronize()
                        ts = []
                        for _ in range(reps):           # median of per-call times
                            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                            e0.record(stream)
                            fn()
                            e1.record(stream)
                            torch.cuda.synchronize()
                            ts.append(e0.elapsed_time(e1))
                        ms = float(np.median(ts))
                        nbytes = sites * C3_WORDS[vo][kname] * (8 if prec == hhg.HHG_F64 else 4)
                        gbs = nbytes / (ms * 1e-3) / 1e9
                        rows.append({"disc": name, "level": level, "N": N, "sites": sites, "prec": pname,
                                     "kernel": kname, "ms": round(ms, 4), "alg_bytes": int(nbytes),
                                     "GB_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)})
                        log(f"[c3] {name} L{level} {pname} {kname}: {ms:.4f} ms, {gbs:.0f} GB/s "
                            f"({100 * gbs / HBM_PEAK_GBS:.1f} %)")
                    del x, b, y, xc
                    # hhg_smooth reads x back each time; values drift, which does not change the work
            finally:
                torch.cuda.synchronize()
                hhg.hhg_hier_destroy(H)
    return {"mode": "c3", "workload": "48 macro-tets (one Bey step of the Kuhn cube), N(0,1) inputs, "
                                      "algorithmic words per site: apply 6.25 / 8, residual 9.375 / 12, Uzawa 9.125 xi + 3.375 / "
                                      "10 xi + 6 (P2-P1 / P1-P1), transfers per fine site", "rows": rows}


def bench_learned(torch, hhg, ctx, args, L=6, lmin=2):
    """Learned coarse solve on P1-P1 PSPG, 6 macro-tets, level 6, coarsest
    N = 4 (206 unknowns): pairs from plain V(3,3) solves over log-normal
    viscosity seeds, GPU training, held-out pair errors, V-cycle rates (exact
    / network / relaxation only) and the time of a solve with a new viscosity
    (plain: pseudo-inverse rebuilt; network: none) at equal tolerance."""
    from paper_2010_13513_amd import learned
    from paper_2010_13513_amd.problem import Problem
    P = Problem(torch, ctx, hhg.HHG_P1P1, lmin, L)
    v33 = (3, 3, 0, 1, hhg.HHG_GS_FWD, 1)
    # omega^{-1} by power iteration (eq. omega-eigenvalue-problem) for the
    # first training field, used for every field
    P.set_viscosity(learned.W.lognormal_viscosity(learned.TRAIN_BASE))
    v0 = torch.from_numpy(W_normal(P, L)).to(P.dev)
    om = hhg.hhg_estimate_omega(P.h, L, v0, 100)
    log(f"[learned] omega_inv {om:.4f}")
    # pairs: the first 16 coarse-grid visits (FMG, then V(3,3) cycles) of a
    # plain solve per training field
    prm_pairs = hhg.solver_params(*v33, om, extra_cycles=12)
    out = {"mode": "learned", "workload": f"P1-P1 PSPG, 6 Kuhn macro-tets, level {L} ({P.dofs(L)} DoFs), "
                                          f"coarsest level {lmin} (N=4, 206 unknowns), log-normal viscosity "
                                          f"1:100, Fourier forcing, V(3,3)"}
    m = None
    try:
        t0 = time.perf_counter()
        F, T, used = learned.collect_pairs(P, [learned.TRAIN_BASE + s for s in range(100000)], prm_pairs, args.pairs,
                                           per_seed=16, log=log)
        out["pairs"] = {"n": int(F.shape[0]), "seeds": used, "seconds": round(time.perf_counter() - t0, 2)}
        log(f"[learned] {F.shape[0]} pairs from {used} seeds in {out['pairs']['seconds']} s")
        hhg.hhg_timer_start(1 << hhg.KF_MLP)
        t0 = time.perf_counter()
        m, hist = learned.train(ctx, F, T, hidden=args.hidden, batch=256, epochs=args.epochs, lr=1e-3,
                                lr_final=1e-4, stages=4, log=log)
        t_train = time.perf_counter() - t0
        ms, n, flops = hhg.hhg_timer_read(hhg.KF_MLP)
        hhg.hhg_timer_start(0)
        tf = flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        out["train"] = {"hidden": args.hidden, "epochs": args.epochs, "batch": 256, "seconds": round(t_train, 2),
                        "loss_history": [round(h, 6) for h in hist]}
        out["mlp_roofline"] = {"bound": "mfma", "kernel": "k_gemm_bf16", "achieved": round(tf, 2),
                               "peak": 2500.0, "unit": "TFLOP/s", "frac": round(tf / 2500.0, 5),
                               "avg_launch_us": round(1e3 * ms / max(n, 1), 2), "launches": n, "traffic": None}
        log(f"[learned] training {t_train:.1f} s; MLP GEMMs {n} launches, {tf:.2f} TFLOP/s")
        # held-out pairs: the coarse visits of FMG + one cycle on every held-out seed
        prm_fmg = hhg.solver_params(*v33, om, extra_cycles=1)
        t0 = time.perf_counter()
        Fh, Th, used_h = learned.collect_pairs(P, [learned.TEST_BASE + s for s in range(args.test_seeds)], prm_fmg,
                                               8 * args.test_seeds, log=log)
        eh = learned.pair_errors(P, m, Fh, Th)
        et = learned.pair_errors(P, m, F[:4096], T[:4096])
        out["pair_error"] = {"held_out_seeds": used_h, "held_out_pairs": int(Fh.shape[0]),
                             "held_out_median": round(float(np.median(eh)), 4),
                             "held_out_p90": round(float(np.percentile(eh, 90)), 4),
                             "train_median": round(float(np.median(et)), 4),
                             "seconds": round(time.perf_counter() - t0, 2)}
        log(f"[learned] pair errors {out['pair_error']}")
        # V(3,3) convergence rates on held-out fields
        prm0 = hhg.solver_params(*v33, om)
        prms = hhg.solver_params(*v33, om, coarse_smooth=2)
        rates = {"exact": [], "network": [], "relax_only": []}
        for s in range(10):
            seed = learned.TEST_BASE + 5000 + s
            rates["exact"].append(float(np.mean(learned.cycle_rates(P, seed, prm0, 12)[2:])))
            rates["relax_only"].append(float(np.mean(learned.cycle_rates(P, seed, prms, 12)[2:])))
            hhg.hhg_hier_set_mlp(P.h, m, 1.0, 0.0)
            rates["network"].append(float(np.mean(learned.cycle_rates(P, seed, prm0, 12)[2:])))
            hhg.hhg_hier_set_mlp(P.h, None)
        out["vcycle_rate_mean"] = {k: round(float(np.mean(v)), 4) for k, v in rates.items()}
        log(f"[learned] V(3,3) rates {out['vcycle_rate_mean']}")
        # a solve per new viscosity to rtol 1e-8: setup (viscosity on every
        # level, plain: + pseudo-inverse) + FMG and cycles
        rho = float(np.max(rates["exact"]))    # monitor: plain rate of the worst held-out field
        res = {"plain": [], "network": []}
        prm_solve = hhg.solver_params(*v33, om, rtol=1e-8, max_cycles=200)
        for s in range(10):
            seed = learned.TEST_BASE + 6000 + s
            xs = {}
            for mode in ("plain", "network"):
                if mode == "network":
                    hhg.hhg_hier_set_mlp(P.h, m, rho, 0.5)
                nu = learned.W.lognormal_viscosity(seed)
                prob = learned.W.fourier_forcing(learned.forcing_seed(seed))
                nus = {l: torch.from_numpy(nu(*P.p1_nodes(l))).to(P.dev) for l in range(lmin, L + 1)}
                bs = P.rhs(prob)
                x = P.boundary(prob)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for l in range(lmin, L + 1):
                    hhg.hhg_set_viscosity(P.h, l, nus[l])
                t1 = time.perf_counter()
                st = hhg.hhg_fmg_solve(P.h, x, bs, prm_solve, check=False)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                res[mode].append((t1 - t0, t2 - t1, st.cycles, st.fallbacks, st.rel_res))
                xs[mode] = x
                if mode == "network":
                    hhg.hhg_hier_set_mlp(P.h, None)
            d = ((xs["network"] - xs["plain"]).abs().max() / xs["plain"].abs().max()).item()
            res.setdefault("max_rel_diff", []).append(d)
        summ = {}
        for mode in ("plain", "network"):
            a = np.array(res[mode])
            summ[mode] = {"setup_ms": round(1e3 * float(np.median(a[:, 0])), 3),
                          "solve_ms": round(1e3 * float(np.median(a[:, 1])), 3),
                          "total_ms": round(1e3 * float(np.median(a[:, 0] + a[:, 1])), 3),
                          "cycles_median": float(np.median(a[:, 2])), "fallbacks": int(a[:, 3].sum()),
                          "max_rel_res": float(a[:, 4].max())}
        summ["max_rel_diff_network_vs_plain"] = float(max(res["max_rel_diff"]))
        out["new_viscosity_solve"] = summ
        log(f"[learned] per new viscosity: {summ}")
    finally:
        if m is not None:
            hhg.hhg_hier_set_mlp(P.h, None)
            hhg.hhg_mlp_destroy(m)
        P.close()
    return out


def bench_dc(torch, hhg, ctx, level=7, lmin=1):
    """Mixed precision: P2-P1 Taylor-Hood, 6 macro-tets, the given level,
    Gaussian-bump viscosity 1:100, Fourier forcing, u = 0 on the boundary.
    Defect correction in float64 to ||r|| <= 1e-12 ||b|| around one V(3,3)
    cycle per correction, inner cycles in float64, in float32, and in float32
    with bfloat16 storage on the levels <= 3; reports times, cycles and
    ||x - x64||_M / ||x64||_M."""
    from paper_2010_13513_amd import workloads as W
    from paper_2010_13513_amd.problem import Problem
    P = Problem(torch, ctx, hhg.HHG_P2P1, lmin, level)
    N = P.N(level)
    out = {"mode": "dc", "workload": f"P2-P1 Taylor-Hood, 6 Kuhn macro-tets, level {level} ({P.dofs(level)} DoFs), "
                                     f"Gaussian-bump viscosity 1:100, Fourier forcing, V(3,3) inner cycles (A_f, xi=3)"}
    try:
        t0 = time.perf_counter()
        P.set_viscosity(W.gaussian_bump_viscosity(W.SEED_BASE + 4000, N_ref=N))
        prob = W.fourier_forcing(W.SEED_BASE + 4001)
        b = P.rhs(prob)[-1]
        x0 = P.boundary(prob)
        v0 = torch.from_numpy(W.normal_vector(W.SEED_BASE + 4002, (N + 1) ** 3)).to(P.dev)
        om = hhg.hhg_estimate_omega(P.h, level, v0, 100)
        torch.cuda.synchronize()
        out["setup_s"] = round(time.perf_counter() - t0, 2)
        out["omega_inv"] = om
        log(f"[dc] level {level}: {P.dofs(level)} DoFs, omega_inv {om:.4f}, setup {out['setup_s']} s")
        # V(3,3) with A_f and xi = 3 Gauss-Seidel sweeps per Uzawa step: every
        # P2-P1 tuple of Tab. fmg-table with A_f uses xi = 3 (xi = 1 diverges here)
        prm = hhg.solver_params(3, 3, 0, 1, hhg.HHG_GS_FWD, 3, om)
        nbf = max(0, min(3, level) - lmin + 1)             # bfloat16 storage on levels <= 3
        out["bf16_levels"] = f"{lmin}..{lmin + nbf - 1}"
        xs = {}
        for name, prec, nb in (("f64", hhg.HHG_F64, 0), ("f32", hhg.HHG_F32, 0), ("f32_bf16", hhg.HHG_F32, nbf)):
            hhg.hhg_hier_set_bf16_levels(P.h, nb)
            x = x0.clone()                                  # warm-up solve (allocations, code paths)
            hhg.hhg_dc_solve(P.h, x, b, prm, prec, 1, 1e-12, 200, check=False)
            x = x0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = hhg.hhg_dc_solve(P.h, x, b, prm, prec, 1, 1e-12, 200, check=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            xs[name] = x
            out[name] = {"seconds": round(dt, 4), "cycles": st.cycles, "rel_res": st.rel_res,
                         "converged": bool(st.rel_res <= 1e-12),
                         "ms_per_cycle": round(1e3 * dt / max(st.cycles, 1), 3),
                         "dofs_per_s": P.dofs(level) / dt}
            log(f"[dc] inner {name}: {st.cycles} cycles, rel res {st.rel_res:.2e}, {dt:.3f} s")
        hhg.hhg_hier_set_bf16_levels(P.h, 0)
        mx = torch.empty_like(xs["f64"])
        hhg.hhg_apply(P.h, level, hhg.HHG_OP_MASS, xs["f64"], mx)
        xu, xp = hhg.hhg_dots(P.h, level, xs["f64"], mx)
        for name in ("f32", "f32_bf16"):
            e = xs[name] - xs["f64"]
            hhg.hhg_project_mean_zero(P.h, level, e)
            me = torch.empty_like(e)
            hhg.hhg_apply(P.h, level, hhg.HHG_OP_MASS, e, me)
            eu, ep = hhg.hhg_dots(P.h, level, e, me)
            out[name]["rel_diff_M"] = {"u": float(np.sqrt(eu / xu)), "p": float(np.sqrt(ep / xp))}
            # a speed-up is only "at equal final float64 error" if both arms
            # reached the tolerance
            ok = out[name]["converged"] and out["f64"]["converged"]
            out[name]["speedup_vs_f64"] = round(out["f64"]["seconds"] / out[name]["seconds"], 3) if ok else None
            log(f"[dc] {name}: ||x - x64||_M / ||x64||_M u {out[name]['rel_diff_M']['u']:.2e}, "
                f"p {out[name]['rel_diff_M']['p']:.2e}; rel res {out[name]['rel_res']:.2e} "
                f"(f64 {out['f64']['rel_res']:.2e}); speed-up {out[name]['speedup_vs_f64']}")
        out["speedup_f32_vs_f64"] = out["f32"]["speedup_vs_f64"]
    finally:
        P.close()
    return out


def bench_sweep(torch, hhg, ctx, args):
    """The paper's parameter study (Sec. 5.1): all 768 tuples of the search
    space S with GPU FMG on the 6-tet cube, paper cube solution, P1-P1 level 6
    (coarsest 0) and P2-P1 level 5 (coarsest 1); gamma of eq. gamma against
    the discrete solution; the synthetic Tab. fmg-table and the least-error-
    for-work envelopes."""
    from paper_2010_13513_amd import study, workloads as W
    from paper_2010_13513_amd.problem import Problem
    prob = W.paper_cube()
    out = {"mode": "sweep", "problem": "paper cube solution (Sec. 5.1.1), 6 Kuhn macro-tets, Dirichlet",
           "schur": "SD", "ordering": "multicolour"}
    allrows = {}
    for disc, name, lmin, L in ((hhg.HHG_P1P1, "P1-P1", 0, 6), (hhg.HHG_P2P1, "P2-P1", 1, 5)):
        P = Problem(torch, ctx, disc, lmin, L)
        try:
            v0 = torch.from_numpy(W.normal_vector(W.SEED_BASE + 1000, (2 ** L + 1) ** 3)).to(P.dev)
            om = hhg.hhg_estimate_omega(P.h, L, v0, 100)
            log(f"[sweep] {name} level {L} ({P.dofs(L)} DoFs): omega_inv {om:.6f}")
            t0 = time.perf_counter()
            rows, ed = study.run(torch, P, prob, om, study.search_space(), log=log)
            el = time.perf_counter() - t0
            tab = study.best_under_bounds(rows)
            env_u = study.min_error_for_work(rows, "gamma_u")
            env_p = study.min_error_for_work(rows, "gamma_p")
            for t in tab:
                b = t["best"]
                log(f"[sweep] {name} bounds {t['bounds']}: " +
                    (f"{b['name']} WU {b['wu']:.2f} gamma ({b['gamma_u']:.3f}, {b['gamma_p']:.3f})" if b else "none"))
            out[name] = {"level": L, "dofs": P.dofs(L), "omega_inv": om, "disc_errors": ed, "seconds": round(el, 2),
                         "tuples": len(rows), "table": tab, "envelope_gamma_u": env_u, "envelope_gamma_p": env_p,
                         "solve_ms_median": round(1e3 * float(np.median([r["seconds"] for r in rows])), 3)}
            allrows[name] = rows
        finally:
            P.close()
    if args.sweep_out:
        with open(args.sweep_out, "w") as f:
            json.dump(allrows, f)
    return out


# Tab. fmg-table, P1-P1 rows (24-tetrahedron cube, L = 6): tuple, bounds
# (gamma_u_hat, gamma_p_hat), the paper's work units and gammas
PAPER_P1_TUPLES = [((2, 3, 2, 1, 1, 1), (1.1, 2.0), 10.77, 1.10, 1.51),
                   ((3, 1, 3, 1, 1, 1), (1.1, 5.0), 9.55, 1.10, 2.91),
                   ((1, 0, 2, 1, 1, 1), (2.0, 10.0), 3.97, 1.62, 8.52)]
UMESH_HEADLINE = PAPER_P1_TUPLES[0][0]


def bench_umesh(torch, hhg, dev, stream, ctx, args, L=6):
    """FMG on the paper's cube benchmark configuration on the unstructured
    path: the unit cube as 24 tetrahedra (workloads.cube24, 15 vertices),
    P1-P1 PSPG, levels 0..L (L = 6: 1,073,409 nodes, 4,293,636 DoFs with the
    Dirichlet ones), the paper's analytic cube solution, omega^{-1} from 100
    power iterations on level L, Schur diagonal SD.  Step = one FMG solve of
    the paper's first P1-P1 tuple of Tab. fmg-table (graph-replayed); the
    other two tuples and their gammas (eq. gamma: errors of eq. error on
    level L + 1 against a solve converged to 1e-12) next to the paper's."""
    from paper_2010_13513_amd import workloads as W
    xyz, tets = W.cube24()
    prob = W.paper_cube()
    mesh = hhg.hhg_mesh_create(ctx, xyz, tets)
    H = hhg.hhg_hier_create(mesh, hhg.HHG_P1P1, 0, L, hhg.HHG_SCHUR_SD)
    Ev = hhg.hhg_hier_create(mesh, hhg.HHG_P1P1, L, L + 1, hhg.HHG_SCHUR_SD)   # error evaluation only
    hhg.hhg_mesh_destroy(mesh)

    def upload(hier, level, arr):
        _, _, vw, _ = hhg.hhg_vec_layout(hier, level)
        dst = torch.zeros(vw, dtype=torch.float64, device=dev)
        hhg.hhg_vec_from_lattice(hier, level, torch.from_numpy(np.ascontiguousarray(arr)).to(dev), dst)
        return dst

    def download(hier, level, vec):
        _, _, _, lw = hhg.hhg_vec_layout(hier, level)
        out = torch.empty(lw, dtype=torch.float64, device=dev)
        hhg.hhg_vec_to_lattice(hier, level, vec, out)
        return out.cpu().numpy()

    # node positions (canonical order): host tables up to level L, level L+1
    # by prolongation of the coordinate fields (exact for linear fields)
    pos = {l: hhg.hhg_query_umesh(xyz, tets, l)["pos"] for l in range(0, L + 1)}
    nn_f = hhg.hhg_vec_layout(Ev, L + 1)[1]
    fine = []
    for d in range(3):
        e = upload(Ev, L + 1, np.zeros(4 * nn_f))
        hhg.hhg_prolong_add(Ev, L, upload(Ev, L, np.concatenate([pos[L][:, d]] * 4)), e)
        fine.append(download(Ev, L + 1, e)[:nn_f])
    pos[L + 1] = np.stack(fine, axis=1)

    def fields(level, fn_u, fn_p=None):
        P = pos[level]
        u = fn_u(P[:, 0], P[:, 1], P[:, 2])
        p = np.zeros(P.shape[0]) if fn_p is None else fn_p(P[:, 0], P[:, 1], P[:, 2])
        return np.concatenate([u[0], u[1], u[2], p])

    bs = []
    for l in range(0, L + 1):
        f_nod = upload(H, l, fields(l, prob.f))
        b = torch.zeros_like(f_nod)
        hhg.hhg_rhs(H, l, f_nod, b)
        bs.append(b)
    x0 = upload(H, L, fields(L, prob.u))
    nn = pos[L].shape[0]
    dofs = 4 * nn
    v0 = torch.from_numpy(W.normal_vector(W.SEED_BASE + 8000, nn)).to(dev)
    omega_inv = hhg.hhg_estimate_omega(H, L, v0, 100)
    log(f"[umesh] cube24 P1-P1 L={L}: {nn} nodes, {dofs} DoFs, omega_inv {omega_inv:.6f}")
    xs_fine = upload(Ev, L + 1, fields(L + 1, prob.u, prob.p))

    def errors(xL):
        e = torch.zeros_like(xs_fine)
        hhg.hhg_prolong_add(Ev, L, xL, e)
        e -= xs_fine
        hhg.hhg_project_mean_zero(Ev, L + 1, e)
        me = torch.empty_like(e)
        hhg.hhg_apply(Ev, L + 1, hhg.HHG_OP_MASS, e, me)
        du, dp = hhg.hhg_dots(Ev, L + 1, e, me)
        return float(np.sqrt(du)), float(np.sqrt(dp))

    xd = x0.clone()
    st = hhg.hhg_fmg_solve(H, xd, bs, hhg.solver_params(3, 3, 0, 1, hhg.HHG_GS_SYM, 1, omega_inv, rtol=1e-12,
                                                        max_cycles=200))
    eud, epd = errors(xd)
    log(f"[umesh] discrete solution ({st.cycles} cycles, rel res {st.rel_res:.1e}): errors u {eud:.4e} p {epd:.4e}")
    x = torch.zeros_like(x0)

    def run_tuple(s, steps, warmup):
        prm = hhg.solver_params(*s, omega_inv)

        def step():
            x.copy_(x0)
            hhg.hhg_fmg_solve(H, x, bs, prm, want_stats=False)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        eu, ep = errors(x)
        wu = hhg.hhg_fmg_solve(H, x0.clone(), bs, prm).work_units
        return ms, eu / eud, ep / epd, wu, step

    rows = []
    step = None
    for s_t, bounds, w_p, gu_p, gp_p in PAPER_P1_TUPLES:
        steps = args.steps if s_t == UMESH_HEADLINE else max(5, args.steps // 2)
        ms, gu, gp, wu, st_fn = run_tuple(s_t, steps, args.warmup)
        if s_t == UMESH_HEADLINE:
            step, ms_step, g_head, wu_head = st_fn, ms, (gu, gp), wu
        rows.append({"fmg": _tname(s_t), "bounds": list(bounds), "work_units": round(wu, 3),
                     "ms_per_solve": round(ms, 4), "dofs_per_s": dofs / (ms * 1e-3),
                     "gamma_u": round(gu, 4), "gamma_p": round(gp, 4),
                     "paper": {"work_units": w_p, "gamma_u": gu_p, "gamma_p": gp_p}})
        log(f"[umesh] FMG{_tname(s_t)}: {ms:.3f} ms, {dofs / (ms * 1e-3):.3e} DoF/s, {wu:.2f} WU, "
            f"gamma ({gu:.3f}, {gp:.3f}); paper {w_p} WU, ({gu_p}, {gp_p})")
    value = dofs / (ms_step * 1e-3)

    # kernel families of one headline step
    fams = {hhg.KF_APPLY: "cell_interior_rows", hhg.KF_IFACE: "interface_nodes",
            hhg.KF_GS_VERTEX: "gs_interior_colour", hhg.KF_PSTEP: "uzawa_pressure_step",
            hhg.KF_RESTRICT: "restrict", hhg.KF_PROLONG: "prolong", hhg.KF_COARSE: "coarse_gemv",
            hhg.KF_REDUCE: "reductions", hhg.KF_OTHER: "other", hhg.KF_SMALL: "one_workgroup_smoothing"}
    rsteps = max(2, min(args.steps, 5))
    hhg.hhg_timer_start(sum(1 << f for f in fams))
    for _ in range(rsteps):
        step()
    torch.cuda.synchronize()
    per_fam = {}
    for f, name in fams.items():
        ms, n, units = hhg.hhg_timer_read(f)
        per_fam[name] = (ms / rsteps, n // rsteps, units / rsteps)
    hhg.hhg_timer_start(0)
    log("[umesh] kernel families per step: " + ", ".join(
        f"{k} {v[0]:.3f} ms/{v[1]}" for k, v in sorted(per_fam.items(), key=lambda kv: -kv[1][0])))
    dom = max(("gs_interior_colour", "cell_interior_rows"), key=lambda k: per_fam[k][0])
    ms_d, n_d, units_d = per_fam[dom]
    words = 10.0 if dom == "gs_interior_colour" else 8.0
    bytes_launch = units_d / max(n_d, 1) * words * 8
    avg_ms = ms_d / max(n_d, 1)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_launch_us": round(avg_ms * 1e3, 3), "bytes_per_launch": int(bytes_launch),
                "launches_per_step": n_d, "share_of_step": round(ms_d / ms_step, 3),
                "timing": "HIP events recorded around each launch",
                "families_ms_per_step": {k: round(v[0], 4) for k, v in per_fam.items()}}

    # apply roofline at level L + 1 (8.5e6 nodes): interior rows of y = calA x
    nn7 = hhg.hhg_vec_layout(Ev, L + 1)[1]
    xa = upload(Ev, L + 1, W.normal_vector(W.SEED_BASE + 8001, 4 * nn7))
    ya = torch.empty_like(xa)
    for _ in range(3):
        hhg.hhg_apply(Ev, L + 1, hhg.HHG_OP_FULL, xa, ya)
    hhg.hhg_timer_start((1 << hhg.KF_APPLY) | (1 << hhg.KF_IFACE))
    for _ in range(args.apply_reps):
        hhg.hhg_apply(Ev, L + 1, hhg.HHG_OP_FULL, xa, ya)
    torch.cuda.synchronize()
    ms_a, n_a, units_a = hhg.hhg_timer_read(hhg.KF_APPLY)
    ms_i, n_i, units_i = hhg.hhg_timer_read(hhg.KF_IFACE)
    hhg.hhg_timer_start(0)
    b_a = units_a / n_a * 64.0
    gbs = b_a / (ms_a / n_a * 1e-3) / 1e9
    apply_roofline = {"bound": "hbm", "kernel": "cell_interior_rows", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "avg_launch_ms": round(ms_a / n_a, 4),
                      "bytes_per_launch": int(b_a), "interface_ms": round(ms_i / max(n_i, 1), 4),
                      "interface_nodes": int(units_i / max(n_i, 1)),
                      "workload": f"y = calA x, 24-tetrahedron cube, level {L + 1} ({nn7} nodes), float64"}
    log(f"[umesh] apply roofline: {apply_roofline}")
    out = {
        "metric": "FMG Stokes DoF/s at discretization accuracy; operator-apply HBM GB/s vs peak",
        "value": value, "unit": "DoF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"P1-P1 PSPG Stokes, unit cube split into 24 tetrahedra (the cube benchmark's "
                               f"partition, unstructured path), level {L} ({dofs} DoFs), paper cube solution, "
                               f"FMG{_tname(UMESH_HEADLINE)} from level 0 (the paper's tuple for bounds (1.1, 2))",
                   "dofs": dofs, "level": L, "omega_inv": omega_inv, "schur": "SD",
                   "work_units": round(wu_head, 3), "gamma_u": round(g_head[0], 4), "gamma_p": round(g_head[1], 4),
                   "disc_err_u": eud, "disc_err_p": epd},
        "paper_tuples": rows,
        "roofline": roofline,
        "apply_roofline": apply_roofline,
    }
    hhg.hhg_hier_destroy(Ev)
    hhg.hhg_hier_destroy(H)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_umesh(omega_inv)
    return out


def _oracle_umesh_worker(args):
    """Oracle FMG solves of the 24-tetrahedron cube workload at a small level
    for about budget_s seconds (setup not timed).  Returns (solves, s, dofs)."""
    Ls, omega_inv, budget_s = args
    from oracle import multigrid as mg, umesh
    from paper_2010_13513_amd import workloads as W
    prob = W.paper_cube()
    H = umesh.hierarchy(*W.cube24(), 0, Ls, schur="sd")
    bs = {l: H.rhs(l, prob) for l in range(0, Ls + 1)}
    s = UMESH_HEADLINE
    prm = mg.Params(s[0], s[1], s[2], s[3], "f" if s[4] == 0 else "s", s[5], omega_inv)
    n, t0 = 0, time.perf_counter()
    while True:
        H.fmg(prob, prm, b=bs)
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 200:
            break
    return n, el, H.S[Ls].n


def cpu_baseline_umesh(omega_inv, Ls=4, budget_s=12.0):
    """The oracle (as it stands) on the same FMG tuple and mesh at level Ls
    (the whole oracle hierarchy of level 6 does not fit a bounded sample),
    one single-threaded process; DoF/s of level Ls."""
    import multiprocessing as mp
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    ctx = mp.get_context("spawn")
    with ctx.Pool(1) as pool:
        n, el, dofs = pool.map(_oracle_umesh_worker, [(Ls, omega_inv, budget_s)])[0]
    v = dofs * n / el
    log(f"[umesh] cpu oracle: {n} FMG solves of level {Ls} ({dofs} DoFs) in {el:.1f} s -> {v:.3e} DoF/s")
    return {"value": v, "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} complete FMG{_tname(UMESH_HEADLINE)} solves of the same mesh at level {Ls} "
                      f"({dofs} DoFs; setup excluded) in one single-threaded numpy/scipy float64 process"}


def W_normal(P, level):
    from paper_2010_13513_amd import workloads as W
    return W.normal_vector(W.SEED_BASE + 5000 + 1, (P.N(level) + 1) ** 3)


def _oracle_worker(args):
    """One host process: build the oracle hierarchy (not timed), then time
    complete FMG solves for about budget_s seconds.  Returns (solves, s)."""
    L, omega_inv, s, budget_s = args
    from oracle import multigrid as mg
    from paper_2010_13513_amd import workloads as W
    prob = W.paper_cube()
    H = mg.Hierarchy(2, 1, L, schur="sd")
    bs = {l: H.rhs(l, prob) for l in range(1, L + 1)}
    prm = mg.Params(s[0], s[1], s[2], s[3], "f" if s[4] == 0 else "s", s[5], omega_inv)
    n, t0 = 0, time.perf_counter()
    while True:
        H.fmg(prob, prm, b=bs)
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 200:
            break
    return n, el


def cpu_baseline(L, omega_inv, budget_s=12.0):
    """The float64 oracle (numpy / scipy, as it stands) on the headline FMG
    workload: first one process alone, then one process per host core (up to
    16, the machine's CPU share) each solving independently; value = the
    all-core throughput (solves x DoFs / wall time), setup excluded."""
    import multiprocessing as mp
    N = 2 ** L
    dofs = 3 * (2 * N + 1) ** 3 + (N + 1) ** 3
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(16, cores))
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"          # one thread per oracle process (children inherit this)
    ctx = mp.get_context("spawn")
    with ctx.Pool(1) as pool:
        n1, el1 = pool.map(_oracle_worker, [(L, omega_inv, HEADLINE, budget_s)])[0]
    single = dofs * n1 / el1
    log(f"[bench] cpu oracle, 1 process: {n1} FMG solves in {el1:.1f} s -> {single:.3e} DoF/s")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(L, omega_inv, HEADLINE, budget_s)] * cores)
    wall = time.perf_counter() - t0
    tot = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    v = dofs * tot / busy
    log(f"[bench] cpu oracle, {cores} processes: {tot} FMG solves, longest timed run {busy:.1f} s "
        f"(wall {wall:.1f} s incl. setup) -> {v:.3e} DoF/s")
    return {"value": v, "unit": "DoF/s", "cores": cores, "kind": "oracle",
            "single_core_value": single, "nproc": os.cpu_count(),
            "sample": f"{tot} complete FMG{_tname(HEADLINE)} solves of the same level-{L} workload "
                      f"(setup excluded) in {cores} independent single-threaded numpy/scipy float64 processes, "
                      f"about {budget_s:.0f} s each; single process alone: {n1} solves"}


if __name__ == "__main__":
    main()
