"""Benchmark: Vanka-GMG-FGMRES on one MI355X.

One step = the whole hot path on the resident hierarchy: build every cell
inverse and the coarse inverse, then flexible GMRES with the V(2,2) Vanka
multigrid preconditioner to relative residual 1e-8.  The reported value is
Vanka cell-sweeps per second over the whole step (sweeps on all smoothed
levels, divided by the wall time of the step including the inverse build).

Default workload: the 3d channel [0,2.5]x[0,0.41]^2, 128x24x24 Q2/P1disc
cells, 4 levels, dG(1) in time (170 local DoFs per cell), Oseen at a seeded
divergence-free convection field, nu = 1e-3, tau = 0.01, seeded N(0,1)
right-hand side; FP64-stored inverses timed, FP32-stored inverses as the
second leg.  The 2d channel 512x128, 6 levels, dG(2) (tau = 0.005) is timed
the same way and reported as "secondary_workload".
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from types import SimpleNamespace

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the 3d precision workload (FP64- vs FP32-stored 170 x 170 cell inverses) is
# the largest single-GPU workload; the 2d dG(2) channel is reported beside it
DEFAULT_WORKLOAD = "3d-128x24x24-dG1"
SECONDARY_WORKLOAD = "2d-512x128-dG2"
# counter-measured HBM bytes per launch (profiles/), one record per workload
TRAFFIC_RECORDS = {
    "2d-512x128-dG2": os.path.join(ROOT, "profiles", "traffic_2d512x128_dG2.json"),
    "3d-128x24x24-dG1": os.path.join(ROOT, "profiles", "traffic_3d128x24x24_dG1.json"),
    "batched-256-2d-dG1": os.path.join(ROOT, "profiles", "traffic_batched256_2d_dG1.json"),
}


def measured_traffic(workload: str, kernel: str, launches_per_level):
    """HBM bytes per launch from the counter record in profiles/ (bytes per
    launch on each level), averaged over the given launches per level, or
    None when there is no record for this workload and kernel, a level is
    missing, or the kernel source changed since the counters were taken."""
    import hashlib
    if workload not in TRAFFIC_RECORDS:
        return None
    try:
        rec = json.load(open(TRAFFIC_RECORDS[workload]))
    except (OSError, ValueError):
        return None
    if rec.get("workload") != workload or kernel not in rec:
        return None
    src = os.path.join(ROOT, rec["kernel_source"])
    try:
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    if sha != rec.get("kernel_source_sha256"):
        return None
    per = rec[kernel]["bytes_per_launch_by_level"]
    tot = n = 0
    for g, cnt in launches_per_level.items():
        if cnt == 0:
            continue
        if str(g) not in per:
            return None
        tot += cnt * per[str(g)]
        n += cnt
    return int(tot / n) if n else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD,
                    choices=["2d-512x128-dG2", "2d-16x4-dG1", "3d-128x24x24-dG1",
                             "batched-256-2d-dG1"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--nu1", type=int, default=2)
    ap.add_argument("--nu2", type=int, default=2)
    ap.add_argument("--omega", type=float, default=0.7)
    ap.add_argument("--coarse-algo", default="auto", choices=["auto", "panels", "slabs", "tournament"])
    ap.add_argument("--coarse-overlap", type=int, default=1, choices=[0, 1],
                    help="coarse factorisation concurrent with the cell inverses (1) or before (0)")
    ap.add_argument("--inverse-cus", type=int, default=None,
                    help="compute units the 3d complex cell-inverse kernel may hold beside the "
                         "coarse factorisation (0: no cap; default: the library's)")
    ap.add_argument("--coarse-lookahead", type=int, default=1, choices=[0, 1],
                    help="look-ahead updates in the complex-pivot coarse chain (1) or not (0)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--shapes", default=None,
                    help='launch shapes instead of the autotuner\'s, as JSON {"level": [residual '
                         'shape, sweep workgroups(, transfer shapes of P and P^T)], ...} (levels '
                         'not named keep the defaults)')
    ap.add_argument("--no-kron", action="store_true",
                    help="residual from the stored blocks instead of the spatial factors")
    ap.add_argument("--no-graph-leg", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 2d dG(2) workload that the default run reports beside the 3d one")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the measured copy and FP64 GEMM reference rates")
    ap.add_argument("--nu-sweep", action="store_true",
                    help="instead of the timing line: FGMRES iterations of the batched "
                         "instances against viscosity, undamped and damped smoother")
    ap.add_argument("--newton", action="store_true",
                    help="instead of the Oseen solve: the linear solve of a Newton step of the "
                         "Navier-Stokes system (256x64, 5 levels, dG(1), Jacobian at the iterate "
                         "after one Newton step from rest: full time blocks)")
    ap.add_argument("--gradient", action="store_true",
                    help="instead of the solve: one gradient of the outflow loss with respect "
                         "to every cell viscosity and the inflow amplitude per step (256x64, "
                         "5 levels, dG(1), per-cell viscosity)")
    return ap.parse_args()


WORKLOADS = {
    # name: (dim, finest cells, levels, k, tau, nu, seed, description,
    #        CPU-baseline sample: (finest cells, levels) of the same operator)
    "2d-512x128-dG2": (2, (512, 128), 6, 2, 0.005, 1e-3, 1002,
                       "2d channel 512x128 Q2/P1disc x dG(2), 6 levels, Oseen nu=1e-3, tau=0.005",
                       ((256, 64), 5)),
    "2d-16x4-dG1": (2, (16, 4), 2, 1, 0.01, 1e-3, 1001,
                    "2d channel 16x4 Q2/P1disc x dG(1), 2 levels, Oseen nu=1e-3, tau=0.01",
                    ((16, 4), 2)),
    "3d-128x24x24-dG1": (3, (128, 24, 24), 4, 1, 0.01, 1e-3, 1003,
                         "3d channel 128x24x24 Q2/P1disc x dG(1), 4 levels, Oseen nu=1e-3, tau=0.01",
                         ((48, 12, 12), 3)),
}
# 256 independent 2d dG(1) instances (finest 32x8 .. 128x32, nu in [5e-4, 5e-3],
# seeds 2000 + j), one batch, FP32-stored inverses, FP64 FGMRES
BATCHED = "batched-256-2d-dG1"
N_BATCH = 256


def sweep_bytes(L, b, inv_bytes, zero_init_fraction):
    """Algorithmic bytes of one cell-sweep launch on a level: stored inverse
    rows, cell DoF lists, owner lists and offsets, one read of the residual and
    one read + write of the iterate (write only for a zero initial iterate)."""
    n_st = L.n_sdofs * b
    n_owned = L.n_sdofs                       # each spatial DoF is owned by one cell
    idx = L.cell_sdofs.size * 4 + (L.n_cells + 1) * 4 + n_owned + L.n_cells * 8
    vec = n_st * 8 + n_st * 8 * (2.0 - zero_init_fraction)
    return inv_bytes + idx + vec


def residual_bytes(L, b, kron=False, n_mass=None):
    """Algorithmic bytes of one level residual: blocks (or the spatial factor
    values of each block: (m, a) where the mass entry m is nonzero, a alone
    elsewhere; n_mass = number of blocks with m != 0), columns, row
    pointers, x, r and y once each."""
    nnzb = int(L.col.shape[0])
    n_st = L.n_sdofs * b
    vec = 3 * n_st * 8
    if not kron:
        return nnzb * (b * b * 8 + 4) + (L.n_sdofs + 1) * 4 + vec
    if n_mass is None:     # one list of (m, a) pairs
        return nnzb * (16 + 4) + (L.n_sdofs + 1) * 4 + vec
    n1 = int(n_mass)
    return n1 * (16 + 4) + (nnzb - n1) * (8 + 4) + 2 * (L.n_sdofs + 1) * 4 + vec


def cpu_baseline(workload, nu1, nu2, omega):
    """The FP64 oracle on a bounded sample of the same workload, full step
    (all inverses + FGMRES to 1e-8) per instance, one thread; reported in
    cell-sweeps per second.  Single hierarchies: the same channel, operator
    and degree on a smaller mesh (the sample field of the workload); the
    batch: its first eight instances."""
    from threadpoolctl import threadpool_limits

    import oracle
    from stgen.problem import batched_instance, make_problem
    if workload == BATCHED:
        probs = [batched_instance(j) for j in range(8)]
        what = ("the batch's first 8 instances (" +
                ", ".join("x".join(map(str, p.meta["n_fine"])) for p in probs) + " cells)")
    else:
        dim, n, G, k, tau, nu, seed, _, (n_s, G_s) = WORKLOADS[workload]
        probs = [make_problem(dim, n_s, G_s, k, tau, nu, seed)]
        what = f"{'x'.join(map(str, n_s))} cells, {G_s} levels, same operator"
    sweeps = 0
    its = []
    with threadpool_limits(1):
        t0 = time.perf_counter()
        for p in probs:
            ol = oracle.prepare_levels(p.levels, p.b)
            oracle.build_inverses(ol)
            cinv = oracle.coarse_inverse(ol[0])
            _, info = oracle.fgmres(lambda v: ol[-1].J @ v, p.rhs,
                                    lambda v: oracle.vcycle(ol, v, nu1, nu2, omega, coarse_inv=cinv),
                                    restart=30, rtol=1e-8)
            sweeps += info["iters"] * (nu1 + nu2) * sum(L.n_cells for L in p.levels[1:])
            its.append(info["iters"])
        dt = time.perf_counter() - t0
    return dict(value=sweeps / dt, unit="cell-sweeps/s", cores=1, kind="oracle",
                sample=f"{what}; full step {dt:.1f} s, FGMRES iterations {its}, 1 thread",
                seconds=dt, iters=its)


def load_workload(name):
    """Hierarchies (a list, one per instance), dim, k, right-hand sides,
    description, and whether the step stores the inverses in FP32."""
    from stgen.problem import batched_instance, make_problem
    if name == BATCHED:
        probs = [batched_instance(j) for j in range(N_BATCH)]
        desc = ("256 independent 2d channels Q2/P1disc x dG(1), finest 32x8/64x16/96x24/128x32, "
                "3-5 levels, Oseen nu in [5e-4, 5e-3], tau=0.01, one batch")
        return probs, 2, 1, desc, True
    dim, n, G, k, tau, nu, seed, desc, _ = WORKLOADS[name]
    return [make_problem(dim, n, G, k, tau, nu, seed)], dim, k, desc, False


def packed_members(probs):
    """Per packed level g (finest aligned): [(level object, smoothed?)]."""
    D = max(len(p.levels) for p in probs)
    out = []
    for g in range(D):
        mem = []
        for p in probs:
            l = g - (D - len(p.levels))
            if l >= 0:
                mem.append((p.levels[l], l > 0))
        out.append(mem)
    return out


def nu_sweep(args):
    """Iterations to 1e-8 of the 256 batched instances (each its own seeded
    viscosity) with the undamped (omega = 1) and damped (omega = 0.7)
    smoother, grouped by viscosity and finest grid."""
    import torch

    import paper_2107_10561_amd as stv
    from stgen.problem import batched_instance
    probs = [batched_instance(j) for j in range(N_BATCH)]
    s = stv.Solver(0)
    s.set_batch([p.levels for p in probs], 2, 1)
    s.build_cell_inverses(fp32=False)
    rhs = torch.from_numpy(np.concatenate([p.rhs for p in probs])).to("cuda:0")
    nus = np.array([p.nu for p in probs])
    edges = np.geomspace(5e-4, 5e-3, 5)
    out = {}
    for omega in (1.0, 0.7):
        x = torch.zeros_like(rhs)
        info = s.gmres_solve(rhs, x, restart=30, max_it=1000, rtol=1e-8, nu1=args.nu1,
                             nu2=args.nu2, omega=omega, raise_on_noconv=False)
        its = np.array([s.instance_info(i)["iters"] for i in range(N_BATCH)])
        conv = np.array([s.instance_info(i)["converged"] for i in range(N_BATCH)])
        rows = []
        for a, b_ in zip(edges[:-1], edges[1:]):
            for size in ((32, 8), (64, 16), (96, 24), (128, 32)):
                sel = (nus >= a) & (nus <= b_) & np.array([p.meta["n_fine"] == size for p in probs])
                if sel.any():
                    rows.append(dict(nu=[float(a), float(b_)], finest="x".join(map(str, size)),
                                     instances=int(sel.sum()), mean_iters=round(float(its[sel].mean()), 2),
                                     max_iters=int(its[sel].max())))
        out[f"omega={omega}"] = dict(all_converged=bool(conv.all()), max_iters=int(its.max()),
                                     mean_iters=round(float(its.mean()), 2), table=rows)
        print(f"[nu-sweep] omega {omega}: mean {its.mean():.2f} max {its.max()} "
              f"converged {conv.all()} ({info['iters']} lockstep steps)", file=sys.stderr, flush=True)
    print(json.dumps({"nu_sweep": out, "cycle": f"V({args.nu1},{args.nu2})", "instances": N_BATCH,
                      "data": "synthetic"}), flush=True)


def gradient_cpu_baseline(n_fine, G, reps=1):
    """The oracle's gradient on a bounded sample of the differentiation
    workload: forward and adjoint FGMRES(30) with the oracle's Vanka-GMG (of J
    and of J^T) to 1e-8, then the cellwise contractions; one thread."""
    from threadpoolctl import threadpool_limits

    import oracle
    from oracle import adjoint as oadj
    from stgen import adjoint as gadj
    p = gadj.make_differentiation_problem(n_fine, G, 1, 0.01, 3000)
    m = p.levels[-1].mesh
    refs, ptr, idx, w = gadj.nu_derivative_refs(m)
    tw = gadj.time_weights(p.k, p.tau)
    F0, in_cells, Fc = gadj.inflow_rhs_parts(m, p.k, p.tau)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        for _ in range(reps):
            ol = oracle.build_inverses(oracle.prepare_levels(p.levels, p.b))
            olt = oadj.transpose_levels(ol)
            ci, cit = oracle.coarse_inverse(ol[0]), oracle.coarse_inverse(olt[0])
            x, fi = oracle.fgmres(lambda v: ol[-1].J @ v, p.rhs,
                                  lambda v: oracle.vcycle(ol, v, 2, 2, 0.7, coarse_inv=ci),
                                  restart=30, rtol=1e-8)
            lam, ai = oracle.fgmres(lambda v: olt[-1].J @ v, p.loss,
                                    lambda v: oracle.vcycle(olt, v, 2, 2, 0.7, coarse_inv=cit),
                                    restart=30, rtol=1e-8)
            csd = m.cell_sdofs()
            g = -oadj.cell_contraction(lam, x, csd, p.b, refs, ptr, idx, w, tw)
            g[in_cells] += oadj.cell_dot(lam, in_cells, csd, p.b, Fc)
        dt = (time.perf_counter() - t0) / reps
    sweeps = (fi["iters"] + ai["iters"]) * 4 * sum(L.n_cells for L in p.levels[1:])
    return dict(value=round(1.0 / dt, 4), unit="gradients/s", cores=1, kind="oracle",
                cell_sweeps_per_s=round(sweeps / dt, 1),
                sample=f"{n_fine[0]}x{n_fine[1]} cells, {G} levels, dG(1), same loss and "
                       f"viscosity field law ({fi['iters']} + {ai['iters']} FGMRES iterations); "
                       f"{dt:.1f} s per gradient, 1 thread")


def gradient_bench(args):
    """One step = the gradient of the outflow loss L = q . x with respect to
    every cell viscosity and the inflow amplitude: the cell inverses (all
    rows), FGMRES on J x = b, FGMRES on J^T lam = q with the stored inverses
    read transposed, and the cellwise contractions, on the resident
    hierarchy (assembly and upload of the operator are input, outside)."""
    import torch

    import paper_2107_10561_amd as stv
    from stgen import adjoint as gadj
    n_fine, G = (256, 64), 5
    t0 = time.time()
    p = gadj.make_differentiation_problem(n_fine, G, 1, 0.01, 3000)
    m = p.levels[-1].mesh
    refs, ptr, idx, w = gadj.nu_derivative_refs(m)
    tw = gadj.time_weights(p.k, p.tau)
    F0, in_cells, Fc = gadj.inflow_rhs_parts(m, p.k, p.tau)
    print(f"[bench] generated the differentiation workload in {time.time() - t0:.1f} s",
          file=sys.stderr, flush=True)
    s = stv.Solver(0)
    s.set_hierarchy(p.levels, p.dim, p.k)
    dev = torch.device("cuda", 0)
    b = torch.from_numpy(p.rhs).to(dev)
    q = torch.from_numpy(p.loss).to(dev)
    x = torch.zeros_like(b)
    lam = torch.zeros_like(b)
    nc = m.n_cells
    grad = torch.empty(nc, dtype=torch.float64, device=dev)
    fcf = Fc.reshape(len(in_cells), -1)
    cells_smoothed = sum(L.n_cells for L in p.levels[1:])

    def step(fp32):
        s.build_cell_inverses(fp32=fp32, full=True)
        fi = s.gmres_solve(b, x, restart=30, max_it=1000, rtol=1e-8)
        ai = s.gmres_solve_transposed(q, lam, restart=30, max_it=1000, rtol=1e-8)
        # dL/dnu_c = -lam_c^T (W (x) K_c) x_c + U lam_c^T F_c (U = 1), one device pass
        s.cell_gradient(G - 1, lam, x, refs, ptr, idx, w, tw, -1.0, in_cells, fcf, 1.0, grad)
        return fi, ai

    def leg(fp32):
        for _ in range(args.warmup):
            step(fp32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sweeps = 0
        for _ in range(args.steps):
            fi, ai = step(fp32)
            sweeps += (fi["iters"] + ai["iters"]) * cells_smoothed * (args.nu1 + args.nu2)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        g = grad.cpu().numpy()
        return dict(ms_per_step=round(1e3 * el / args.steps, 3),
                    gradients_per_s=round(args.steps / el, 3),
                    cell_sweeps_per_s=round(sweeps / el, 1), forward_iters=fi["iters"],
                    adjoint_iters=ai["iters"], forward_relres=fi["true_relres"],
                    adjoint_relres=ai["true_relres"], max_abs_grad=float(np.abs(g).max()),
                    loss=float((q * x).sum()))

    r64 = leg(False)
    r32 = None if args.no_fp32 else leg(True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = gradient_cpu_baseline((128, 32), 4)
    print(json.dumps({
        "metric": "gradient of the outflow loss w.r.t. every cell viscosity and the inflow "
                  "amplitude (forward + adjoint Vanka-GMG-FGMRES to 1e-8)",
        "value": r64["gradients_per_s"], "unit": "gradients/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2d channel 256x64 Q2/P1disc x dG(1), 5 levels, per-cell "
                               "viscosity 1e-3 exp(0.3 z), tau=0.01, outflow-flux loss",
                   "cells_finest": nc, "levels": G, "parallelism": "single GPU"},
        "fp64": r64, "fp32_inverses": r32,
        "cpu_baseline": cpu}), flush=True)


def newton_system(n_fine, G):
    """The Newton problem, its data and the iterate after one Newton step
    from rest (solved directly on the host: input generation)."""
    import scipy.sparse as sps
    import scipy.sparse.linalg as sla

    from stgen.newton import NewtonProblem
    P = NewtonProblem(2, n_fine, G, 1, 0.01, 1e-3)
    F = P.data(0.0, np.zeros(P.fine.mesh.n_sdofs))
    u = np.zeros(P.fine.mesh.n_sdofs * P.b)
    L = P.hierarchy(u)[-1]
    n = L["n_sdofs"] * P.b
    J0 = sps.bsr_matrix((np.asarray(L["val"]).reshape(-1, P.b, P.b), L["col"], L["rowptr"]),
                        shape=(n, n))
    u = u - sla.spsolve(J0.tocsc(), P.residual(u, F))
    return P, F, u


def newton_cpu_baseline(n_fine, G):
    """The oracle's Vanka-GMG FGMRES(30) on the Newton Jacobian of a bounded
    sample (cell inverses, coarse inverse and the solve to 1e-8), one thread."""
    from threadpoolctl import threadpool_limits

    import oracle
    P, F, u = newton_system(n_fine, G)
    H = P.hierarchy(u)
    R = P.residual(u, F)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        ol = oracle.build_inverses(oracle.prepare_levels(H, P.b))
        ci = oracle.coarse_inverse(ol[0])
        _, info = oracle.fgmres(lambda v: ol[-1].J @ v, -R,
                                lambda v: oracle.vcycle(ol, v, 2, 2, 0.7, coarse_inv=ci),
                                restart=30, rtol=1e-8)
        dt = time.perf_counter() - t0
    sweeps = info["iters"] * 4 * sum(int(np.asarray(L["cell_sdofs"]).shape[0]) for L in H[1:])
    return dict(value=round(sweeps / dt, 1), unit="cell-sweeps/s", cores=1, kind="oracle",
                sample=f"{n_fine[0]}x{n_fine[1]} cells, {G} levels, dG(1), Newton Jacobian at "
                       f"the same kind of iterate ({info['iters']} FGMRES iterations); "
                       f"{dt:.1f} s per solve, 1 thread")


def newton_bench(args):
    """One step = the linear solve of a Newton step: all cell inverses and the
    coarse inverse of the Jacobian hierarchy J(u) (full time blocks: the
    convection term is integrated exactly in time at a time-dependent
    iterate), then FGMRES(30) + V(2,2) on J(u) du = -R(u) to 1e-8."""
    import torch

    import paper_2107_10561_amd as stv
    n_fine, G = (256, 64), 5
    t0 = time.time()
    P, F, u = newton_system(n_fine, G)
    H = P.hierarchy(u)
    R = P.residual(u, F)
    print(f"[bench] Newton system at the first iterate in {time.time() - t0:.1f} s",
          file=sys.stderr, flush=True)
    s = stv.Solver(0)
    s.set_hierarchy(H, 2, 1)
    rhs = torch.from_numpy(-R).to("cuda:0")
    du = torch.zeros_like(rhs)
    cells = sum(int(np.asarray(L["cell_sdofs"]).shape[0]) for L in H[1:])

    top = s.n_levels - 1
    Lt = H[top]
    fine = SimpleNamespace(n_sdofs=int(Lt["n_sdofs"]), cell_sdofs=np.asarray(Lt["cell_sdofs"]),
                           n_cells=int(np.asarray(Lt["cell_sdofs"]).shape[0]))
    zi = 1.0 / (args.nu1 + args.nu2) if args.nu1 > 0 else 0.0

    def leg(fp32):
        for _ in range(args.warmup):
            s.build_cell_inverses(fp32=fp32)
            s.gmres_solve(rhs, du, restart=30, max_it=1000, rtol=1e-8)
        # the finest-level sweep launches of the timed steps are stamped by the
        # kernels' own start/end records (no event records between launches)
        s.set_timing(True, classes=["sweep"], levels=[top])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sweeps = 0
        for _ in range(args.steps):
            s.build_cell_inverses(fp32=fp32)
            info = s.gmres_solve(rhs, du, restart=30, max_it=1000, rtol=1e-8)
            sweeps += info["iters"] * cells * (args.nu1 + args.nu2)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        n_sw, ms_sw = s.kernel_stats("sweep", top)
        s.set_timing(False)
        byt = sweep_bytes(fine, P.b, s.level_info(top)["inverse_bytes"], zi)
        gbs = byt / (ms_sw / n_sw / 1e3) / 1e9 if n_sw else 0.0
        r1 = P.residual(u + du.cpu().numpy(), F)
        return dict(ms_per_step=round(1e3 * el / args.steps, 3),
                    cell_sweeps_per_s=round(sweeps / el, 1), iters=info["iters"],
                    true_relres=info["true_relres"],
                    newton_residual_before=float(np.linalg.norm(R) / np.linalg.norm(F)),
                    newton_residual_after=float(np.linalg.norm(r1) / np.linalg.norm(F)),
                    roofline_sweep=dict(
                        bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(gbs / HBM_PEAK_GBS, 4), bytes_per_launch=int(byt),
                        avg_launch_ms=round(ms_sw / max(n_sw, 1), 5), launches=n_sw,
                        kernel=f"Vanka cell sweep on the full-row store (k_vanka), finest "
                               f"level ({top}), {'FP32' if fp32 else 'FP64'} store"))

    r64 = leg(False)
    r32 = None if args.no_fp32 else leg(True)
    roof = r64.pop("roofline_sweep")
    cpu = None if args.no_cpu_baseline else newton_cpu_baseline((128, 32), 4)
    print(json.dumps({
        "metric": "Newton-step linear solve: GMG-GMRES time to rel. residual 1e-8; Vanka "
                  "cell-sweeps/s", "value": r64["cell_sweeps_per_s"], "unit": "cell-sweeps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2d channel 256x64 Q2/P1disc x dG(1), 5 levels, Navier-Stokes "
                               "Newton Jacobian, nu=1e-3, tau=0.01, parabolic inflow ramp",
                   "cells_finest": n_fine[0] * n_fine[1], "levels": G,
                   "parallelism": "single GPU"},
        "roofline": dict(roof, traffic=None), "fp64": r64, "fp32_inverses": r32,
        "cpu_baseline": cpu}), flush=True)


FP64_PEAK_TFLOPS = 78.6


def inverse_flops_per_cell(dim, k, n_ls, dec, cx=False):
    """Flops of the Gauss-Jordan inversion(s) one cell's build runs: 2 n^3 for
    an explicit inverse of order n.  The time-decoupled build (2d levels with
    spatial factors) inverts one block of order n_ls per real eigenvalue of the
    time matrix and the real form (order 2 n_ls) of one block per complex
    pair instead of the whole J_T of order (k+1) n_ls; the complex build (3d
    dG(1) levels with spatial factors) inverts the complex block of order n_ls
    in complex arithmetic, 8 n_ls^3 real flops."""
    b = k + 1
    if cx:
        return 8 * n_ls ** 3
    if dec:
        n_pairs = b // 2
        n_real = b - 2 * n_pairs
        return n_real * 2 * n_ls ** 3 + n_pairs * 2 * (2 * n_ls) ** 3
    return 2 * (b * n_ls) ** 3


def coarse_flops(k, n_s, kron):
    """Flops of the coarse Gauss-Jordan inverse: 2 N^3 for the whole matrix of
    order N = (k+1) n_s; with spatial factors the eliminated matrices are the
    real forms (order 2 n_s) of the pair blocks, and of the real eigenvalues'
    blocks padded into the same launches (one real-form block per two real
    eigenvalues, rounded up)."""
    b = k + 1
    if not kron:
        return 2 * (b * n_s) ** 3
    n_pairs = b // 2
    n_real = b - 2 * n_pairs
    blocks = n_pairs + (n_real + 1) // 2
    return blocks * 2 * (2 * n_s) ** 3


def measured_peaks():
    """A plain copy (1 GiB read + 1 GiB written, torch's copy kernel) and a
    plain FP64 GEMM (8192^3, the vendor BLAS through torch) on this GPU."""
    import torch
    dev = torch.device("cuda", 0)
    n = 1 << 27
    x = torch.empty(n, dtype=torch.float64, device=dev).normal_()
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    reps = 10
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * 8 * n * reps / (a.elapsed_time(b) / 1e3) / 1e9
    del x, y
    m = 8192
    A = torch.randn(m, m, dtype=torch.float64, device=dev)
    B = torch.randn(m, m, dtype=torch.float64, device=dev)
    C = A @ B
    torch.cuda.synchronize()
    a.record()
    reps = 5
    for _ in range(reps):
        C = A @ B
    b.record()
    torch.cuda.synchronize()
    dgemm = 2 * m ** 3 * reps / (a.elapsed_time(b) / 1e3) / 1e12
    del A, B, C
    torch.cuda.empty_cache()
    return dict(copy_GBps=round(copy_gbs, 1), dgemm_TFLOPs=round(dgemm, 2),
                copy="torch copy_ of 1 GiB float64, read + write bytes",
                dgemm="torch float64 matmul 8192 x 8192 x 8192")


def run_workload(args, name, legs=True):
    """Set up one workload (resident hierarchy, spatial factors, autotuned
    shapes), time args.steps steps after args.warmup untimed ones, and return
    the measurements: throughput, phase split, rooflines of the sweep, the
    residual and the inverse build, and (legs) the other storage precision of
    the inverses and the graph-replay step."""
    import torch

    import paper_2107_10561_amd as stv

    t0 = time.time()
    probs, dim, k, desc, primary_fp32 = load_workload(name)
    b = k + 1
    print(f"[bench] generated {desc} in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    s = stv.Solver(0)
    s.set_coarse_algorithm(args.coarse_algo)
    s.set_coarse_overlap(bool(args.coarse_overlap))
    s.set_coarse_lookahead(bool(args.coarse_lookahead))
    if args.inverse_cus is not None:
        s.set_inverse_cus(args.inverse_cus)
    t0 = time.time()
    if len(probs) == 1:
        s.set_hierarchy(probs[0].levels, dim, k)
    else:
        s.set_batch([p.levels for p in probs], dim, k)
    t_set = time.time() - t0
    G = s.n_levels
    members = packed_members(probs)
    kron = not args.no_kron
    n_mass = {}
    if kron:
        from stgen import fe
        from stgen.problem import spatial_factors
        t0 = time.time()
        _, w, C, _ = fe.time_matrices(k)
        tw = probs[0].tau * np.asarray(w, dtype=np.float64)
        for g in range(G):
            parts = [spatial_factors(L) for L, _ in members[g]]
            s.set_kron_factors(g, np.concatenate([m_ for m_, _ in parts]),
                               np.concatenate([a_ for _, a_ in parts]), np.asarray(C), tw)
            n_mass[g] = [int(np.count_nonzero(m_)) for m_, _ in parts]
        print(f"[bench] spatial factors of every level in {time.time() - t0:.1f} s",
              file=sys.stderr, flush=True)
    rhs_h = np.concatenate([p.rhs for p in probs])
    rhs = torch.from_numpy(rhs_h).to("cuda:0")
    x = torch.zeros_like(rhs)
    mg = dict(nu1=args.nu1, nu2=args.nu2, omega=args.omega)
    cells_smoothed = [sum(L.n_cells for L in p.levels[1:]) for p in probs]

    def step(fp32, out=None):
        s.build_cell_inverses(fp32=fp32)
        return s.gmres_solve(rhs, x if out is None else out, restart=30, max_it=1000, rtol=1e-8,
                             **mg)

    def useful_sweeps():
        return sum(s.instance_info(i)["iters"] * c for i, c in enumerate(cells_smoothed)) * \
            (args.nu1 + args.nu2)

    shapes = None
    if args.shapes:
        shapes = {str(g): list(v) for g, v in json.loads(args.shapes).items()}
        for g, v in shapes.items():
            s.set_launch(int(g), int(v[0]), int(v[1]))
            if len(v) >= 4:
                s.transfer_shapes(int(g), int(v[2]), int(v[3]))
        print(f"[bench] launch shapes set: {shapes}", file=sys.stderr, flush=True)
    elif not args.no_autotune:
        s.build_cell_inverses(fp32=primary_fp32)
        t0 = time.time()
        # per level: residual shape, sweep workgroups, transfer shapes (P, P^T)
        shapes = {str(g): list(v) + list(s.transfer_shapes(g))
                  for g, v in s.autotune().items() if g > 0}
        print(f"[bench] autotuned launch shapes in {time.time() - t0:.2f} s: {shapes}",
              file=sys.stderr, flush=True)
    for i in range(args.warmup):
        info = step(primary_fp32)
        print(f"[bench] warmup {i}: iters {info['iters']} relres {info['true_relres']:.2e}",
              file=sys.stderr, flush=True)
    # inside the timed region only the two roofline classes are timed, by the
    # kernels' own start/end stamps (no event records between launches)
    s.set_timing(True, classes=["sweep", "residual"], levels=[G - 1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    t_inv = t_gm = 0.0
    total_sweeps = 0
    for i in range(args.steps):
        a = time.perf_counter()
        s.build_cell_inverses(fp32=primary_fp32)
        torch.cuda.synchronize()
        m = time.perf_counter()
        infos.append(s.gmres_solve(rhs, x, restart=30, max_it=1000, rtol=1e-8, **mg))
        torch.cuda.synchronize()
        e = time.perf_counter()
        total_sweeps += useful_sweeps()
        t_inv += m - a
        t_gm += e - m
        print(f"[bench] step {i}: inv {1e3 * (m - a):.2f} ms gmres {1e3 * (e - m):.2f} ms "
              f"iters {infos[-1]['iters']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = total_sweeps / elapsed

    top = G - 1
    zi = 1.0 / (args.nu1 + args.nu2) if args.nu1 > 0 else 0.0
    inv_b = {g: s.level_info(g)["inverse_bytes"] for g in range(G)}

    def sweep_bytes_packed(g):
        return inv_b[g] + sum(sweep_bytes(L, b, 0, zi) for L, sm in members[g] if sm)

    def residual_bytes_packed(g):
        # the split lists (shapes 7..12) stream a alone where m = 0
        split = kron and shapes is not None and shapes.get(str(g), [0])[0] >= 7
        nm = n_mass.get(g) if split else None
        nm = nm or [None] * len(members[g])
        return sum(residual_bytes(L, b, kron, q) for (L, _), q in zip(members[g], nm))

    def roofline(cls, bytes_of, kernel, traffic_key):
        """The finest level's launches of the kernel in the timed region: the
        only launches timed there (by their own start/end stamps), the bulk
        of the kernel's bytes."""
        n_f, ms_f = s.kernel_stats(cls, top)
        gbs_f = bytes_of(top) / (ms_f / n_f / 1e3) / 1e9 if n_f else 0.0
        return dict(bound="hbm", achieved=round(gbs_f, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(gbs_f / HBM_PEAK_GBS, 4),
                    traffic=measured_traffic(name, traffic_key, {top: n_f}),
                    kernel=kernel + f", finest level ({top})",
                    bytes_per_launch=int(bytes_of(top)), avg_launch_ms=round(ms_f / max(n_f, 1), 5),
                    launches=n_f)

    def all_levels(cls, bytes_of):
        """Every smoothed level, from the instrumented step."""
        tb = tms = 0.0
        tn = 0
        for g in range(1, G):
            n_g, ms_g = s.kernel_stats(cls, g)
            tb += n_g * bytes_of(g)
            tms += ms_g
            tn += n_g
        gbs = tb / (tms / 1e3) / 1e9 if tms > 0 else 0.0
        return dict(achieved=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4),
                    bytes_per_launch=int(tb / max(tn, 1)), avg_launch_ms=round(tms / max(tn, 1), 5),
                    launches=tn)

    kname_res = ("level residual from spatial factors (k_spmv_kron)" if kron
                 else "block-sparse level residual (k_spmv_rows)")
    # with spatial factors the library stores the owned rows of 2d cell
    # problems (n_loc = 21, B <= 3) time-decoupled and sweeps with k_vanka_dec
    # (one row per owned spatial DoF), and those of 3d dG(1) levels (one complex
    # pair: k_inverse_cx) as complex rows swept by k_vanka_cx
    dec = kron and dim == 2 and 2 <= b <= 3
    cx = kron and dim == 3 and b == 2
    if dec:
        roof_sweep = roofline("sweep", sweep_bytes_packed,
                              "Vanka cell sweep on time-decoupled inverses (k_vanka_dec)",
                              "k_vanka_dec")
    elif cx:
        roof_sweep = roofline("sweep", sweep_bytes_packed,
                              "Vanka cell sweep on complex time-decoupled inverses (k_vanka_cx)",
                              "k_vanka_cx")
    else:
        roof_sweep = roofline("sweep", sweep_bytes_packed, "Vanka cell sweep (k_vanka)", "k_vanka")
    split_top = kron and shapes is not None and shapes.get(str(top), [0])[0] >= 7
    if split_top:
        kname_res = "level residual from spatial factors, split lists (k_spmv_kron)"
    roof_res = roofline("residual", residual_bytes_packed, kname_res,
                        ("k_spmv_kron_split" if split_top else "k_spmv_kron") if kron
                        else "k_spmv")
    # time per kernel class (and both kernels over every level) from one more
    # step with every class and level timed, outside the timed region: the
    # event records around the classes that are not stamped by their launch
    # slow the step down
    s.set_timing(True)
    step(primary_fp32)
    torch.cuda.synchronize()
    breakdown = {cls: round(s.kernel_stats(cls)[1], 3) for cls in stv.KERNEL_CLASSES}
    roof_sweep["all_levels_instrumented_step"] = all_levels("sweep", sweep_bytes_packed)
    roof_res["all_levels_instrumented_step"] = all_levels("residual", residual_bytes_packed)
    # the inverse build against the FP64 matrix peak: cell inverses of every
    # smoothed level (one launch class on the caller's stream) and the coarse
    # chain (its own stream, concurrent with them)
    inv_flops = 0
    for g in range(1, G):
        for L, sm in members[g]:
            if sm:
                inv_flops += L.n_cells * inverse_flops_per_cell(dim, k, L.cell_sdofs.shape[1], dec,
                                                                cx=cx)
    crs_flops = sum(coarse_flops(k, p.levels[0].n_sdofs, kron) for p in probs)
    n_inv, ms_inv = s.kernel_stats("inverse")
    n_crs, ms_crs = s.kernel_stats("coarse_factor")

    def flop_roof(fl, ms, kernel, launches):
        tf = fl / (ms / 1e3) / 1e12 if ms > 0 else 0.0
        return dict(bound="mfma", achieved=round(tf, 3), peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(tf / FP64_PEAK_TFLOPS, 4), flops_per_build=int(fl),
                    ms_per_build=round(ms, 3), launches=launches, kernel=kernel)
    inv_roof = dict(
        cell_inverses=flop_roof(inv_flops, ms_inv, "cell inverses, every smoothed level "
                                "(k_inverse_cx)" if cx else "cell inverses, every smoothed level "
                                "(k_inverse_wave / k_inverse_mfma)", n_inv),
        coarse=flop_roof(crs_flops, ms_crs, "coarse Gauss-Jordan inverse chain "
                         "(k_gj_tour_cx / k_gj_slab_update and helpers)", n_crs),
        concurrent="the coarse chain runs on a second stream beside the cell inverses; "
                   "each class's time includes the contention")
    s.set_timing(False)
    res = dict(workload=desc, value=round(value, 1), unit="cell-sweeps/s",
               ms_per_step=round(ms_per_step, 3),
               t_inv_ms=round(1e3 * t_inv / args.steps, 3),
               t_gmres_ms=round(1e3 * t_gm / args.steps, 3), t_set_hierarchy_s=round(t_set, 3),
               gmres_iters=infos[-1]["iters"], true_relres=infos[-1]["true_relres"],
               cell_sweeps_per_step=useful_sweeps(), kernel_ms_per_step=breakdown,
               roofline=roof_sweep, roofline_residual=roof_res, inverse_roofline=inv_roof,
               launch_shapes=shapes, residual_from_spatial_factors=kron,
               config={"workload": desc, "instances": len(probs),
                       "cells_finest": int(sum(p.levels[-1].n_cells for p in probs)),
                       "levels": G,
                       "spacetime_dofs_finest": int(sum(p.levels[-1].n_sdofs for p in probs) * b),
                       "k": k, "cycle": f"V({args.nu1},{args.nu2})", "omega": args.omega,
                       "restart": 30, "rtol": 1e-8, "parallelism": "single GPU"},
               primary_fp32=primary_fp32)
    if legs and not args.no_fp32:
        # the other storage precision of the inverses, same solve; the two
        # solutions are compared (equal accuracy: both reach the same true
        # residual; their difference is within the solve tolerance)
        alt = not primary_fp32
        x_alt = torch.zeros_like(x)
        step(alt, x_alt)
        torch.cuda.synchronize()
        # the leg's own finest-level sweep launches are stamped as in the
        # timed region, for the roofline of the other storage precision
        s.set_timing(True, classes=["sweep"], levels=[top])
        torch.cuda.synchronize()
        a = time.perf_counter()
        reps = max(1, min(3, args.steps))
        for _ in range(reps):
            inf_alt = step(alt, x_alt)
        torch.cuda.synchronize()
        t_alt = (time.perf_counter() - a) / reps
        n_f, ms_f = s.kernel_stats("sweep", top)
        inv_b_alt = s.level_info(top)["inverse_bytes"]
        s.set_timing(False)
        b_alt = inv_b_alt + sum(sweep_bytes(L, b, 0, zi) for L, sm in members[top] if sm)
        gbs_alt = b_alt / (ms_f / n_f / 1e3) / 1e9 if n_f else 0.0
        diff = float(torch.linalg.vector_norm(x_alt - x) / torch.linalg.vector_norm(x))
        res["fp64_inverses" if primary_fp32 else "fp32_inverses"] = dict(
            ms_per_step=round(1e3 * t_alt, 3), iters=inf_alt["iters"],
            true_relres=inf_alt["true_relres"],
            rel_diff_to_primary_solution=diff,
            inverse_bytes_finest=inv_b_alt,
            speedup_vs_primary=round(ms_per_step / (1e3 * t_alt), 4),
            roofline_sweep=dict(bound="hbm", achieved=round(gbs_alt, 1), peak=HBM_PEAK_GBS,
                                unit="GB/s", frac=round(gbs_alt / HBM_PEAK_GBS, 4),
                                bytes_per_launch=int(b_alt),
                                avg_launch_ms=round(ms_f / max(n_f, 1), 5), launches=n_f,
                                kernel=roof_sweep["kernel"].replace("inverses (", "inverses, "
                                                                    "other precision (")))
        print(f"[bench] {'fp32' if alt else 'fp64'} step {1e3 * t_alt:.2f} ms "
              f"iters {inf_alt['iters']}", file=sys.stderr, flush=True)
    if legs and not args.no_graph_leg:
        # the same step with the V-cycle replayed from a captured HIP graph
        s.set_graph(True)
        step(primary_fp32)
        torch.cuda.synchronize()
        a = time.perf_counter()
        reps = max(1, min(3, args.steps))
        for _ in range(reps):
            inf_g = step(primary_fp32)
        torch.cuda.synchronize()
        t_g = (time.perf_counter() - a) / reps
        s.set_graph(False)
        res["graph_replay"] = dict(ms_per_step=round(1e3 * t_g, 3), iters=inf_g["iters"],
                                   true_relres=inf_g["true_relres"])
        print(f"[bench] graph step {1e3 * t_g:.2f} ms iters {inf_g['iters']}", file=sys.stderr,
              flush=True)
    s.close()
    del s, rhs, x
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.newton:
        if args.gpus != 1:
            print("bench.py runs on one GPU only.", file=sys.stderr)
            sys.exit(2)
        newton_bench(args)
        return
    if args.nu_sweep:
        nu_sweep(args)
        return
    if args.gradient:
        if args.gpus != 1:
            print("bench.py runs on one GPU only.", file=sys.stderr)
            sys.exit(2)
        gradient_bench(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "sharding is a design note, not a measured path.", file=sys.stderr)
        sys.exit(2)

    main_res = run_workload(args, args.workload)
    secondary = None
    if args.workload == DEFAULT_WORKLOAD and not args.no_secondary:
        print(f"[bench] secondary workload {SECONDARY_WORKLOAD}", file=sys.stderr, flush=True)
        sec = run_workload(args, SECONDARY_WORKLOAD)
        secondary = {k_: v for k_, v in sec.items() if k_ not in ("primary_fp32",)}
    peaks = None
    if not args.no_peaks:
        peaks = measured_peaks()
        peaks["sweep_frac_of_copy"] = round(main_res["roofline"]["achieved"] / peaks["copy_GBps"], 4)
        peaks["cell_inverses_frac_of_dgemm"] = round(
            main_res["inverse_roofline"]["cell_inverses"]["achieved"] / peaks["dgemm_TFLOPs"], 4)
        peaks["coarse_frac_of_dgemm"] = round(
            main_res["inverse_roofline"]["coarse"]["achieved"] / peaks["dgemm_TFLOPs"], 4)
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cb = cpu_baseline(args.workload, args.nu1, args.nu2, args.omega)
        cpu = {k_: (round(v, 3) if isinstance(v, float) else v) for k_, v in cb.items()
               if k_ in ("value", "unit", "cores", "kind", "sample")}

    r = main_res
    out = {
        "metric": "GMG-GMRES time to rel. residual 1e-8; Vanka cell-sweeps/s + HBM GB/s, FP64 vs FP32",
        "value": r["value"],
        "unit": "cell-sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64, inverses stored f32" if r["primary_fp32"] else "f64",
        "data": "synthetic",
        "config": r["config"],
        "time_to_solution_ms": r["ms_per_step"],
        "t_inv_ms": r["t_inv_ms"],
        "t_gmres_ms": r["t_gmres_ms"],
        "t_set_hierarchy_s": r["t_set_hierarchy_s"],
        "gmres_iters": r["gmres_iters"],
        "true_relres": r["true_relres"],
        "cell_sweeps_per_step": r["cell_sweeps_per_step"],
        "kernel_ms_per_step": r["kernel_ms_per_step"],
        "kernel_ms_per_step_from": "one extra step after the timed region, every class timed",
        "roofline": r["roofline"],
        "roofline_residual": r["roofline_residual"],
        "inverse_roofline": r["inverse_roofline"],
        "measured_peaks": peaks,
        ("fp64_inverses" if r["primary_fp32"] else "fp32_inverses"):
            r.get("fp64_inverses" if r["primary_fp32"] else "fp32_inverses"),
        "graph_replay": r.get("graph_replay"),
        "launch_shapes": r["launch_shapes"],
        "residual_from_spatial_factors": r["residual_from_spatial_factors"],
        "secondary_workload": secondary,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
