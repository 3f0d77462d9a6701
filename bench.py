"""Benchmark: FMG Stokes solve at discretisation accuracy on one MI355X.

Workload (one step = one full FMG solve, Alg. fmg of the paper): P2-P1
Taylor-Hood Stokes on the unit cube split into 6 Kuhn macro-tetrahedra,
refinement level 5 (32 intervals per macro edge, 859,812 DoFs including the
Dirichlet velocity DoFs), analytic cube solution of the paper (Sec. 5.1.1),
FMG(0, 2, 1, 1, A_f, 3) from coarsest level 1 -- the paper's cheapest P2-P1
tuple of Tab. fmg-table (8.11 work units).  float64, inputs resident in HBM.

Printed JSON line: value = DoF / s of the whole solve; roofline of the
dominant kernel family of the step (HIP-event timed, algorithmic bytes);
accuracy of the result (gamma_u, gamma_p of eq. gamma against a float64
solve converged to 1e-12 on the GPU, errors of eq. error); the operator
apply's HBM roofline at the largest throughput size (P2-P1, 48 tets, level
7); and the CPU oracle timed on the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
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
# algorithmic bytes per work unit (float64 words), see the design doc
WORDS = {
    "apply_p2": 6.25,        # y = calA x per P2 site
    "gs_colour": 9.0,        # per updated site: u read + u write + f read (3 components)
}


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
    ap.add_argument("--mode", choices=["fmg", "apply"], default="fmg",
                    help="apply: only the operator-apply roofline (for counter runs)")
    ap.add_argument("--apply-reps", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is "
              "not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2010_13513_amd import hhg, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    L, lmin = args.level, 1
    s = (0, 2, 1, 1, hhg.HHG_GS_FWD, 3)
    prob = W.paper_cube()

    ctx = hhg.hhg_ctx_create(0, stream.cuda_stream)
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
    H = hhg.hhg_hier_create(ctx, hhg.HHG_P2P1, 0, lmin, L, hhg.HHG_SCHUR_SD)
    Ev = hhg.hhg_hier_create(ctx, hhg.HHG_P2P1, 0, L, L + 1, hhg.HHG_SCHUR_SD)   # error evaluation only

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

    # ---- inputs (setup, not timed): right-hand sides of every level, boundary data
    bs = []
    for l in range(lmin, L + 1):
        f_nod = upload(H, l, lattice_fields(l, prob.f))
        b = torch.zeros_like(f_nod)
        hhg.hhg_rhs(H, l, f_nod, b)
        bs.append(b)
    x0 = upload(H, L, lattice_fields(L, prob.u))      # boundary data (interior ignored)
    v0 = torch.from_numpy(W.normal_vector(W.SEED_BASE + 1000, (2 ** L + 1) ** 3)).to(dev)
    omega_inv = hhg.hhg_estimate_omega(H, L, v0, 100)
    prm = hhg.solver_params(*s, omega_inv)
    x = torch.zeros_like(x0)
    N = 2 ** L
    dofs = 3 * (2 * N + 1) ** 3 + (N + 1) ** 3
    log(f"[bench] workload P2-P1 L={L} dofs={dofs} omega_inv={omega_inv:.6f}")

    def step():
        x.copy_(x0)
        hhg.hhg_fmg_solve(H, x, bs, prm, want_stats=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_step = e0.elapsed_time(e1) / args.steps
    value = dofs / (ms_step * 1e-3)
    log(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step (wall {1e3 * t_wall / args.steps:.3f}), "
        f"{value:.3e} DoF/s")

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

    step()
    torch.cuda.synchronize()
    eu, ep = errors(x)
    xd = x0.clone()
    st = hhg.hhg_fmg_solve(H, xd, bs, hhg.solver_params(3, 3, 0, 1, hhg.HHG_GS_FWD, 3, omega_inv, rtol=1e-12,
                                                        max_cycles=200))
    eud, epd = errors(xd)
    gamma_u, gamma_p = eu / eud, ep / epd
    log(f"[bench] errors u {eu:.4e} p {ep:.4e}; discrete ({st.cycles} cycles, rel res {st.rel_res:.1e}) "
        f"u {eud:.4e} p {epd:.4e}; gamma_u {gamma_u:.3f} gamma_p {gamma_p:.3f}")

    # ---- roofline of the dominant kernel family (HIP events on the solve stream)
    fams = {hhg.KF_APPLY: "apply_residual", hhg.KF_PROW_BND: "boundary_pressure_rows",
            hhg.KF_GS_VERTEX: "gs_vertex_colour", hhg.KF_GS_EDGE: "gs_edge_colour", hhg.KF_PSTEP: "uzawa_pressure_step",
            hhg.KF_RESTRICT: "restrict", hhg.KF_PROLONG: "prolong", hhg.KF_COARSE: "coarse_gemv",
            hhg.KF_REDUCE: "reductions", hhg.KF_OTHER: "other"}
    rsteps = max(2, min(args.steps, 5))
    hhg.hhg_timer_start((1 << len(fams)) - 1)
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
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_launch_us": round(avg_ms * 1e3, 3), "bytes_per_launch": int(bytes_launch),
                "launches_per_step": n_d, "share_of_step": round(ms_d / ms_step, 3)}

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
                               f"({dofs} DoFs), paper cube solution, FMG(0,2,1,1,A_f,3) from level 1",
                   "dofs": dofs, "level": L, "fmg": "0,2,1,1,A_f,3", "omega_inv": omega_inv,
                   "work_units": 8.11, "gamma_u": round(gamma_u, 4), "gamma_p": round(gamma_p, 4),
                   "err_u": eu, "err_p": ep},
        "roofline": roofline,
    }
    if apply_roofline:
        out["apply_roofline"] = apply_roofline
    hhg.hhg_hier_destroy(Ev)
    hhg.hhg_hier_destroy(H)
    hhg.hhg_ctx_destroy(ctx)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(L, omega_inv)
    print(json.dumps(out), flush=True)


def bench_apply(torch, hhg, dev, stream, ctx, level=7, reps=20):
    """y = calA x, P2-P1 on the 48-tet cube at the given macro level
    (N = 2^(level+1) intervals), float64 and float32, N(0,1) input."""
    res = {}
    H = hhg.hhg_hier_create(ctx, hhg.HHG_P2P1, 1, level - 1, level, hhg.HHG_SCHUR_SD)
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
                         "bytes_per_launch": int(b)}
            del x, y
        res.update({"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "workload": f"P2-P1 apply, 48 macro-tets, level {level} ({sites} P2 sites)"})
        log(f"[bench] apply roofline: {res}")
    finally:
        hhg.hhg_hier_destroy(H)
    return res


def cpu_baseline(L, omega_inv, budget_s=15.0):
    """The float64 oracle on the same FMG workload, host cores (scipy sparse,
    one thread), repeated for about budget_s seconds; setup excluded."""
    from oracle import multigrid as mg
    from paper_2010_13513_amd import workloads as W
    prob = W.paper_cube()
    H = mg.Hierarchy(2, 1, L, schur="sd")
    bs = {l: H.rhs(l, prob) for l in range(1, L + 1)}
    prm = mg.Params(0, 2, 1, 1, "f", 3, omega_inv)
    n, t0 = 0, time.perf_counter()
    while True:
        H.fmg(prob, prm, b=bs)
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 50:
            break
    N = 2 ** L
    dofs = 3 * (2 * N + 1) ** 3 + (N + 1) ** 3
    v = dofs * n / el
    log(f"[bench] cpu oracle: {n} FMG solves in {el:.1f} s -> {v:.3e} DoF/s")
    return {"value": v, "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} complete FMG solves of the same level-{L} workload (setup excluded), "
                      "numpy/scipy float64, single thread"}


if __name__ == "__main__":
    main()
