"""Throughput benchmark of the hot path on one MI355X.

Workload (the constant-coefficient Cartesian case): u_tt = Laplace(u) on the periodic
unit square, 256 x 256 elements of 16 x 16 GD cells (N + 1 = 17 nodes per direction),
degree p = 5, upwind flux (xi = c = 1), simultaneous-diagonalisation local solves,
classical RK4 with dt = 0.15 h (h = 1/4096; CFL 0.5 is outside RK4's stability
region for the upwind flux at p = 5), initial data a seeded superposition of 8
Fourier modes (|k| <= 16, amplitude N(0,1)/|k|^2), v0 = 0.  One "step" is one full
RK4 step (4 fused stage kernels) over all 18,939,904 DOF per field.

Printed: ONE JSON line.  `value` = DOF-updates/s in FP64 (nx*ny*(N+1)^2 * steps /
time; inputs resident in HBM).  Also reported: the FP32-storage mode, the error of
both against the exact solution, the roofline of the stage kernel (algorithmic HBM
bytes per launch / measured average launch time), the variable-coefficient mapped PCG
workload in FP64 and in mixed precision (`pcg`) with the IC(0) baseline solves of its
element systems (`pcg.ic0_baseline`), the same grid as the headline with
Dirichlet walls (`walls`), box elements in 3D (`fdm3d`), the learned preconditioner
(`learned`),
the 64-problem batch (`batch`) and the FP64 CPU oracle timed on a bounded sample on the
host (`cpu_baseline`).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # MI355X HBM3E, B/s
# HBM bytes per launch of the FP64 stage kernel k_stage<double,*,17,4> on the workload
# below, from rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB per dispatch, mean over the 4 stage
# variants), scaled by a plain device copy's reading of the same counters (x2.0 read,
# x1.0 write); the summary with its commands is profiles/fdm_stage_256x256_N16_p5_fp64.md.
# Set to None whenever that kernel changes until the counters are taken again.
FDM_STAGE_TRAFFIC = (318921.1 * 2.0 + 469083.7) * 1024.0
# The same for one RK stage of the PCG path on the 128 x 128, N = 12, p = 5 mapped workload:
# the sum over its four launches (k_pcg_lift, k_pcg_solve_w0<0,13,5>, k_pcg_solve_w0<1,13,5>,
# k_pcg_update; profiles/pcg_stage_128x128_N12_p5_fp64.md).
PCG_STAGE_TRAFFIC = ((112150.3 + 1236712.2 + 1213141.7 + 117189.7) * 2.0
                     + (44032.0 + 44561.2 + 22544.0 + 128789.4)) * 1024.0


def _workload(n=256, N=16, p=5, seed=2, cfl=0.15):
    from paper_2105_01722_amd import inputs
    X, Y = inputs.node_coords(n, n, N)
    modes = inputs.fourier_modes(seed)
    U0 = inputs.fourier_field(modes, X, Y)
    return dict(n=n, N=N, p=p, modes=modes, X=X, Y=Y, U0=U0, dt=cfl / (n * N))


def _time_gpu(w, precision, steps, warmup):
    import torch
    from paper_2105_01722_amd import gdw
    n, N, p = w["n"], w["N"], w["p"]
    s = gdw.Solver(n, n, N, p, c2=1.0, flux="upwind", xi=1.0, precision=precision)
    U0 = torch.from_numpy(w["U0"]).cuda()
    s.set_state(U0, torch.zeros_like(U0))
    stream = torch.cuda.current_stream()
    if warmup:
        s.run(w["dt"], warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.run(w["dt"], steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    U, V = s.get_state()
    st = s.stats()
    s.close()
    T = w["dt"] * (steps + warmup)
    Ue, Ve = _fourier_exact_uv(w["modes"], w["X"], w["Y"], T)
    Uh, Vh = U.cpu().numpy(), V.cpu().numpy()
    err = {"u": float(np.linalg.norm(Uh - Ue) / np.linalg.norm(Ue)),
           "v": float(np.linalg.norm(Vh - Ve) / np.linalg.norm(Ve)),
           "u_max": float(np.abs(Uh - Ue).max() / np.abs(Ue).max()),
           "v_max": float(np.abs(Vh - Ve).max() / np.abs(Ve).max())}
    return ms, err, st


def _fourier_exact_uv(modes, X, Y, t):
    """u and v = u_t of the exact solution from the Fourier data with v0 = 0 (c = 1)."""
    U = np.zeros_like(X)
    V = np.zeros_like(X)
    for kx, ky, a, th in modes:
        wk = 2 * np.pi * np.hypot(kx, ky)
        ph = np.cos(2 * np.pi * (kx * X + ky * Y) + th)
        U += a * np.cos(wk * t) * ph
        V -= a * wk * np.sin(wk * t) * ph
    return U, V


def _time_walls(steps, warmup, n=256, N=16, p=5, cfl=0.15, k=4, l=3):
    """The headline grid with Dirichlet walls on all four sides: u0 = sin(k pi x)
    sin(l pi y), v0 = 0, whose exact solution is cos(pi sqrt(k^2 + l^2) t) u0."""
    import torch
    from paper_2105_01722_amd import gdw, inputs
    X, Y = inputs.node_coords(n, n, N)
    U0n = np.sin(k * np.pi * X) * np.sin(l * np.pi * Y)
    dt = cfl / (n * N)
    s = gdw.Solver(n, n, N, p, c2=1.0, flux="upwind", xi=1.0, bc=("dirichlet",) * 4)
    U0 = torch.from_numpy(U0n).cuda()
    s.set_state(U0, torch.zeros_like(U0))
    stream = torch.cuda.current_stream()
    if warmup:
        s.run(dt, warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.run(dt, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    U, _ = s.get_state()
    s.stats()
    s.close()
    T = dt * (steps + warmup)
    exact = np.cos(np.pi * np.hypot(k, l) * T) * U0n
    err = float(np.linalg.norm(U.cpu().numpy() - exact) / np.linalg.norm(exact))
    ndof = n * n * (N + 1) ** 2
    return {"workload": "256x256 elements, N=16, p=5, upwind, Dirichlet walls on all sides, "
                        "u0 = sin(%d pi x) sin(%d pi y), v0 = 0, RK4 dt = 0.15 h" % (k, l),
            "ms_per_step": ms / steps, "value": ndof * steps / (ms * 1e-3),
            "unit": "DOF-updates/s", "dtype": "f64", "rel_err_vs_exact": err}


def _time_3d(steps, warmup, n=48, N=8, p=3, cfl=0.12, seed=2, precision="fp64"):
    """Box elements in 3D: the periodic unit cube, n^3 elements of N^3 GD cells, degree p,
    upwind flux, RK4 with dt = 0.12 h (the largest stable value on the dense spectrum is
    0.17 h), initial data 8 seeded 3D Fourier modes (|k| <= 8, amplitude N(0,1)/|k|^2),
    v0 = 0; the error against the exact standing-wave solution is taken on every 5th
    element in each direction."""
    import torch
    from paper_2105_01722_amd import gdw, inputs
    X, Y, Z = inputs.node_coords3(n, n, n, N)
    modes = inputs.fourier_modes3(seed)
    U0 = torch.from_numpy(inputs.fourier_field3(modes, X, Y, Z)).cuda()
    dt = cfl / (n * N)
    s = gdw.Solver(n, n, N, p, nz=n, flux="upwind", xi=1.0, precision=precision)
    s.set_state(U0, torch.zeros_like(U0))
    del U0
    stream = torch.cuda.current_stream()
    if warmup:
        s.run(dt, warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.run(dt, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    U, V = s.get_state()
    s.stats()
    s.close()
    sl = (slice(None, None, 5),) * 3
    T = dt * (steps + warmup)
    Xs, Ys, Zs = X[sl], Y[sl], Z[sl]
    Ue = inputs.fourier_field3(modes, Xs, Ys, Zs, t=T)
    Ve = inputs.fourier_field3(modes, Xs, Ys, Zs, t=T, deriv=True)
    Uh, Vh = U[sl].cpu().numpy(), V[sl].cpu().numpy()
    ndof = n ** 3 * (N + 1) ** 3
    launches = 4 * steps
    alg = 32 * 8 * ndof / 4          # survey count per launch: 32 s per DOF-update
    return {"workload": "3D periodic unit cube, %d^3 box elements, N=%d, p=%d, upwind, RK4 dt = "
                        "%.2f h, 8 seeded 3D Fourier modes" % (n, N, p, cfl),
            "dof_per_field": ndof, "steps": steps, "ms_per_step": ms / steps,
            "value": ndof * steps / (ms * 1e-3), "unit": "DOF-updates/s",
            "dtype": "f64" if precision == "fp64" else "f32 increments / f64 register",
            "rel_err_vs_exact": float(np.linalg.norm(Uh - Ue) / np.linalg.norm(Ue)),
            "rel_err_v_vs_exact": float(np.linalg.norm(Vh - Ve) / np.linalg.norm(Ve)),
            "roofline": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK / 1e9,
                         "achieved": alg / (ms * 1e-3 / launches) / 1e9,
                         "frac": alg / (ms * 1e-3 / launches) / HBM_PEAK,
                         "alg_bytes_per_launch": alg, "alg_bytes_per_dof_update": 256,
                         "avg_launch_us": ms * 1e3 / launches,
                         "kernel": "k_stage3<double,*,9,2> (4 stage variants)"}}


def _pcg_workload(n=128, N=12, p=5, grf_seed=3, mode_seed=2):
    """Variable c^2 = 1 + 0.5 g (g: clipped smooth periodic random field, length 0.1) on
    the mapped mesh X = x + 0.05 s, Y = y + 0.05 s, s = sin(2 pi x) sin(2 pi y)."""
    from paper_2105_01722_amd import inputs
    X, Y = inputs.node_coords(n, n, N)
    c2 = inputs.c2_field(grf_seed, X, Y)
    Xm, Ym = inputs.mapped_coords(X, Y)
    U0 = inputs.fourier_field(inputs.fourier_modes(mode_seed), Xm, Ym)
    return dict(n=n, N=N, p=p, X=Xm, Y=Ym, c2=c2, U0=U0, dt=0.1 / (n * N))


def _pcg_flops_per_step(st, nel, N, p):
    """Algorithmic FP64 flops of one RK4 step of the PCG path: per element solve,
    (iterations + 1) x (one full-stencil matvec + one preconditioner application),
    plus the -S_K U product; lifts and traces are not counted."""
    n1 = N + 1
    w = sum(min(k + p, N) - max(k - p, 0) + 1 for k in range(n1))
    nnz = w * w
    pre = 4 * 2 * n1 ** 3
    per_stage = nel * ((st["mean_it_S"] + 1) * (2 * nnz + pre) + 2 * nnz
                       + (st["mean_it_M"] + 1) * (2 * nnz + pre))
    return 4 * per_stage


def _pcg_alg_bytes_per_dof_update(N, p, s=8):
    """Algorithmic HBM bytes per DOF-update of the PCG path: the 32 s of the RK4 state plus,
    per stage, the symmetric halves of S_K and M_J read once (s bytes per entry)."""
    n1 = N + 1
    nnz_sym = 0
    for i in range(n1 * n1):
        ix, iy = i % n1, i // n1
        for j in range(i, n1 * n1):
            jx, jy = j % n1, j // n1
            # rows i, j couple when their windows overlap in both directions
            if abs(ix - jx) <= p and abs(iy - jy) <= p and _gd_couple(ix, jx, N, p) \
                    and _gd_couple(iy, jy, N, p):
                nnz_sym += 1
    return 32 * s + 4 * s * 2 * nnz_sym / (n1 * n1)


def _gd_couple(i, j, N, p):
    """Whether 1D GD nodes i and j share a cell window (their mass entry is non-zero)."""
    lo = lambda k: min(max(k - (p - 1) // 2, 0), N - p)
    return any(lo(k) <= i <= lo(k) + p and lo(k) <= j <= lo(k) + p for k in range(N))


def _time_pcg(w, steps, warmup, rtol=1e-12, precision="fp64"):
    import torch
    from paper_2105_01722_amd import gdw
    n, N, p = w["n"], w["N"], w["p"]
    s = gdw.Solver(n, n, N, p, flux="upwind", xi=1.0, solver="pcg", coeff_variable=True,
                   mapped=True, pcg_rtol=rtol, precision=precision)
    s.set_coeff(w["c2"], w["X"], w["Y"])
    U0 = torch.from_numpy(w["U0"]).cuda()
    s.set_state(U0, torch.zeros_like(U0))
    if warmup:
        s.run(w["dt"], warmup)
    torch.cuda.synchronize()
    st0 = s.stats()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.run(w["dt"], steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    st = s.stats()
    U, V = s.get_state()
    U, V = U.cpu().numpy(), V.cpu().numpy()
    s.close()
    # iteration means of the timed steps only
    tot = st["solves"]
    prev = st0["solves"]
    mS = (st["mean_it_S"] * tot - st0["mean_it_S"] * prev) / (tot - prev)
    mM = (st["mean_it_M"] * tot - st0["mean_it_M"] * prev) / (tot - prev)
    mR = (st["mean_refine"] * tot - st0["mean_refine"] * prev) / (tot - prev)
    return ms, {"mean_it_S": mS, "mean_it_M": mM, "max_it_S": st["max_it_S"],
                "max_it_M": st["max_it_M"], "mean_refine": mR}, (U, V)


def _ic0_section(w, reps=2, seed=21, rtol=1e-12):
    """IC(0) baseline (Sec. 7.1's preconditioner) on the PCG workload's element systems: one
    IC(0)-PCG solve of every element's S_hat and M_J system from x = 0 for a seeded random
    right-hand side (N(0, 1) entries).  The entry point factors and solves in one synchronous
    call; the time is the host clock around the last of `reps` calls (the first one
    allocates the context's workspace, which the later ones reuse)."""
    import time
    import torch
    from paper_2105_01722_amd import gdw
    n, N, p = w["n"], w["N"], w["p"]
    s = gdw.Solver(n, n, N, p, flux="upwind", xi=1.0, solver="pcg", coeff_variable=True,
                   mapped=True, pcg_rtol=rtol)
    s.set_coeff(w["c2"], w["X"], w["Y"])
    b = torch.from_numpy(np.random.default_rng(seed).standard_normal((n * n, (N + 1) ** 2))).cuda()
    res = {"rhs": "seeded N(0, 1) entries, x0 = 0, rtol %g" % rtol}
    for op, name in ((0, "S_hat"), (1, "M_J")):
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, its = s.ic0_solve(op, b, rtol=rtol, maxit=500)
            t1 = time.perf_counter()
        its = its.cpu().numpy()
        res[name] = {"ms_all_elements": (t1 - t0) * 1e3, "mean_it": float(its.mean()),
                     "max_it": int(its.max())}
    s.close()
    return res


def _learned_section(steps, epochs=60, n_train=20000, seed_train=5000, seed_test=6):
    """Learned correction of the tensor-product preconditioner on the 256 x 256 Cartesian
    variable-coefficient workload (N=12, p=5, upwind, rtol 1e-10): train on the solver's
    own data from another coefficient field (n_train random elements), then compare PCG
    iterations and time with the plain preconditioner and with the exact modal
    diagonal itself (the analytic control)."""
    import time as _t
    import torch
    from paper_2105_01722_amd import gdw, inputs
    n, N, p = 256, 12, 5
    K = (N + 1) ** 2 - 1
    X, Y = inputs.node_coords(n, n, N)
    # training data from the solver's own assembled operators
    tr = gdw.Solver(n, n, N, p, flux="upwind", solver="pcg", coeff_variable=True)
    tr.set_coeff(inputs.c2_field(seed_train, X, Y))
    smp, tgt = tr.precond_data()
    tr.close()
    perm = torch.from_numpy(np.random.default_rng(7).permutation(n * n)[:n_train]).cuda()
    xs, ys = smp[perm].contiguous(), tgt[perm].contiguous()
    net = gdw.Mlp(64, 128, K, seed=11, max_batch=4096)
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    losses = net.train(xs, ys, epochs=epochs, batch=256, lr=1e-3)
    train_s = _t.perf_counter() - t0
    c2 = inputs.c2_field(seed_test, X, Y)
    U0 = torch.from_numpy(inputs.fourier_field(inputs.fourier_modes(2), X, Y)).cuda()
    V0 = torch.zeros_like(U0)
    dt = 0.1 / (n * N)
    res = {}
    ref = None
    for mode in ("plain", "learned", "exact_diag"):
        s = gdw.Solver(n, n, N, p, flux="upwind", solver="pcg", coeff_variable=True, pcg_rtol=1e-10)
        s.set_coeff(c2)
        if mode == "learned":
            s.set_precond_mlp(net)
        elif mode == "exact_diag":
            _, t = s.precond_data()
            s.set_precond_log(t)
        s.set_state(U0, V0)
        s.run(dt, 1)
        torch.cuda.synchronize()
        st0 = s.stats()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        s.run(dt, steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        st = s.stats()
        U, _ = s.get_state()
        s.close()
        Uh = U.cpu().numpy()
        if ref is None:
            ref = Uh
        tot, prev = st["solves"], st0["solves"]
        res[mode] = {"ms_per_step": ms / steps,
                     "mean_it_S": (st["mean_it_S"] * tot - st0["mean_it_S"] * prev) / (tot - prev),
                     "mean_it_M": (st["mean_it_M"] * tot - st0["mean_it_M"] * prev) / (tot - prev),
                     "rel_diff_vs_plain": float(np.linalg.norm(Uh - ref) / np.linalg.norm(ref))}
    net.close()
    return {"workload": "256x256 Cartesian elements, N=12, p=5, c^2 = 1 + 0.5 g (clipped smooth "
                        "random field), upwind, PCG rtol 1e-10, RK4 dt = 0.1 h",
            "train": {"elements": n_train, "epochs": epochs, "batch": 256, "seconds": train_s,
                      "loss_first": float(losses[0]), "loss_last": float(losses[-1])},
            "steps": steps, **res}


# Time steps of the batched workload, as fractions of the cell width: about two thirds
# of the largest RK4-stable value measured on the dense spectrum (upwind; Cartesian
# constant c and the mapped variable-c^2 mesh respectively).
BATCH_CFL_CONST = {3: 0.2, 5: 0.15, 7: 0.1}
BATCH_CFL_VAR = {3: 0.12, 5: 0.09, 7: 0.06}


def _batch_section(steps, seed=4, n_prob=64):
    """Independent problems of uneven size and degree advanced together (one captured
    graph launch per step): constant-coefficient problems in FP32 storage, variable
    ones (mapped mesh, c^2 = 1 + 0.5 g) with FP64 PCG at rtol 1e-12."""
    import torch
    from paper_2105_01722_amd import gdw, inputs
    specs = inputs.batch_specs(seed, n_prob)
    probs, dts, kinds = [], [], []
    for sp in specs:
        n, N, p = sp["n"], sp["N"], sp["p"]
        if sp["variable"]:
            probs.append(dict(nx=n, ny=n, N=N, p=p, flux="upwind", solver="pcg",
                              coeff_variable=True, mapped=True, pcg_rtol=1e-12))
            dts.append(BATCH_CFL_VAR[p] / (n * N))
        else:
            probs.append(dict(nx=n, ny=n, N=N, p=p, flux="upwind", precision="fp32"))
            dts.append(BATCH_CFL_CONST[p] / (n * N))
        kinds.append(sp)
    b = gdw.Batch(probs)
    dof = []
    for i, (kw, sp) in enumerate(zip(probs, specs)):
        n, N = kw["nx"], kw["N"]
        X, Y = inputs.node_coords(n, n, N)
        if sp["variable"]:
            c2 = inputs.c2_field(sp["grf_seed"], X, Y)
            X, Y = inputs.mapped_coords(X, Y)
            b.problems[i].set_coeff(c2, X, Y)
        U0 = inputs.fourier_field(inputs.fourier_modes(sp["mode_seed"]), X, Y)
        b.problems[i].set_state(U0, np.zeros_like(U0))
        dof.append(n * n * (N + 1) ** 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.tune(dts)
    tune_s = time.perf_counter() - t0
    b.run(dts, 1)                                   # warm-up (graph build)
    torch.cuda.synchronize()
    b.run(dts, steps)
    st = np.array(b.step_times())
    total_ms = float(st.sum())
    its = [b.problems[i].stats() for i in range(len(probs)) if probs[i].get("solver") == "pcg"]
    # each problem alone, one step through gdw_run on the same context
    solo = []
    stream = torch.cuda.current_stream()
    for i in range(len(probs)):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.problems[i].run(dts[i], 1)
        e1.record(stream)
        torch.cuda.synchronize()
        solo.append(e0.elapsed_time(e1))
    plan = b.plan().split("candidates:")[0].strip().splitlines()
    b.close()
    tot_dof = int(sum(dof))
    return {
        "workload": "%d independent periodic problems: n ~ U{16..128}^2 elements, N ~ U{8,12,16}, "
                    "p ~ U{3,5,7} (seed %d); even-numbered: c = 1 Cartesian, FP32 storage; "
                    "odd-numbered: mapped mesh, c^2 = 1 + 0.5 g, FP64 PCG rtol 1e-12; upwind; "
                    "dt = CFL h per problem" % (n_prob, seed),
        "problems": len(probs), "dof_total": tot_dof, "steps": steps,
        "value": tot_dof * steps / (total_ms * 1e-3), "unit": "DOF-updates/s",
        "step_ms_p50": float(np.percentile(st, 50)), "step_ms_p99": float(np.percentile(st, 99)),
        "step_ms_min": float(st.min()), "step_ms_max": float(st.max()),
        "solo_sum_ms_per_step": float(sum(solo)),
        "speedup_vs_solo_sequence": float(sum(solo) / (total_ms / steps)),
        "pcg_mean_it_S": float(np.mean([s["mean_it_S"] for s in its])) if its else None,
        "pcg_mean_it_M": float(np.mean([s["mean_it_M"] for s in its])) if its else None,
        "tune_seconds": tune_s,
        "plan": plan,
        "per_problem": [
            {"n": probs[i]["nx"], "N": probs[i]["N"], "p": probs[i]["p"],
             "kind": "pcg-f64" if probs[i].get("solver") == "pcg" else "fdm-f32",
             "dof": dof[i], "solo_ms_per_step": round(solo[i], 4),
             "solo_dof_updates_per_s": dof[i] / (solo[i] * 1e-3)}
            for i in range(len(probs))],
    }


def _physical_cores():
    """Physical cores of the host from lscpu (distinct (core, socket) pairs), or None."""
    import subprocess
    try:
        out = subprocess.run(["lscpu", "-p=Core,Socket"], capture_output=True, text=True,
                             timeout=10).stdout
        pairs = {ln.strip() for ln in out.splitlines() if ln and not ln.startswith("#")}
        return len(pairs) or None
    except Exception:
        return None


def _cpu_baseline(w, n_patch=32, steps=10):
    """The FP64 oracle, as it is, on a bounded sample: a 32 x 32-element periodic patch
    of the same element type (N = 16, p = 5, upwind) for 10 RK4 steps, timed with the
    BLAS thread pool at the cores this process may use (the physical cores lscpu reports,
    capped by the CPU affinity and OMP_NUM_THREADS) and again with one thread."""
    from oracle import dg2d
    from paper_2105_01722_amd import inputs
    from threadpoolctl import threadpool_limits
    phys = _physical_cores()
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cap = [c for c in (phys, avail, int(os.environ.get("OMP_NUM_THREADS", "0")) or None) if c]
    threads = max(1, min(cap)) if cap else 1
    N, p = w["N"], w["p"]
    prob = dg2d.CartProblem(nx=n_patch, ny=n_patch, N=N, p=p, flux="upwind")
    ops = dg2d.CartOps(prob)
    X, Y = inputs.node_coords(n_patch, n_patch, N)
    U = inputs.fourier_field(w["modes"], X, Y)
    V = np.zeros_like(U)
    dofs = n_patch * n_patch * (N + 1) ** 2 * steps
    res = {}
    for nt in (threads, 1):
        with threadpool_limits(limits=nt):
            t0 = time.perf_counter()
            dg2d.run(U, V, ops, w["dt"], steps)
            res[nt] = time.perf_counter() - t0
    return {"value": dofs / res[threads], "unit": "DOF-updates/s", "cores": int(threads),
            "kind": "oracle",
            "sample": "%dx%d-element periodic patch, N=%d, p=%d, upwind, %d RK4 steps, FP64 "
                      "(numpy/scipy dense Cholesky element solves, BLAS threads = cores)"
                      % (n_patch, n_patch, N, p, steps),
            "seconds": res[threads], "physical_cores_lscpu": phys, "cpu_affinity": avail,
            "value_1_thread": dofs / res[1], "seconds_1_thread": res[1]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)   # the headline workload: 100 RK4 steps
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 storage mode")
    ap.add_argument("--no-walls", action="store_true", help="skip the Dirichlet-wall run")
    ap.add_argument("--no-pcg", action="store_true", help="skip the variable-coefficient PCG workload")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D box-element workload")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner section")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-problems section")
    ap.add_argument("--batch-only", action="store_true",
                    help="profiling aid: run only the batched-problems section")
    ap.add_argument("--ic0-only", action="store_true",
                    help="only the IC(0) baseline solves on the PCG workload")
    ap.add_argument("--pcg-only", action="store_true",
                    help="profiling aid: run only the PCG workload (prints its section only)")
    ap.add_argument("--pcg-steps", type=int, default=5, help="timed RK4 steps of the PCG workload")
    ap.add_argument("--pcg-precision", default="fp64", choices=["fp64", "mixed", "pc32"],
                    help="precision of the PCG solves under --pcg-only")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB, 5 times (HBM counter "
                         "calibration under rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "repeats": 5}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only; the library has no multi-GPU path "
              "(the element grid would shard by blocks with one face-trace exchange per "
              "RK stage)", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.batch_only:
        print(json.dumps({"batch": _batch_section(max(1, min(args.steps, 5)))}))
        return
    if args.ic0_only:
        print(json.dumps({"ic0": _ic0_section(_pcg_workload())}))
        return
    if args.pcg_only:
        pw = _pcg_workload()
        ms, its, _ = _time_pcg(pw, max(1, args.pcg_steps), 1, precision=args.pcg_precision)
        print(json.dumps({"pcg_ms_per_step": ms / max(1, args.pcg_steps), **its}))
        return
    w = _workload()
    n, N = w["n"], w["N"]
    ndof = n * n * (N + 1) ** 2
    print("bench: workload ready, %d DOF per field" % ndof, file=sys.stderr, flush=True)
    ms64, err64, st = _time_gpu(w, "fp64", args.steps, args.warmup)
    print("bench: fp64 %.3f ms/step" % (ms64 / args.steps), file=sys.stderr, flush=True)
    value = ndof * args.steps / (ms64 * 1e-3)
    launches = 4 * args.steps
    # Algorithmic HBM bytes per DOF-update: 32 s (s = 8 B), the three-register classical
    # RK4 count (16 field accesses per DOF, field and step).  The stage kernels need only
    # 24 s (the y / Y / accumulator form with 12 accesses), reported beside it.
    alg_bytes_step = 32 * 8 * ndof
    kern_bytes_step = 24 * 8 * ndof
    achieved = alg_bytes_step * args.steps / (ms64 * 1e-3)
    achieved_kern = kern_bytes_step * args.steps / (ms64 * 1e-3)
    out = {
        "metric": "DOF-updates/s per time step + mean PCG iters; FP64 plain vs mixed/learned @ fixed err",
        "value": value, "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms64 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2D wave, periodic unit square, 256x256 Cartesian elements, "
                               "16x16 GD cells (N+1=17), p=5, upwind, FDM mass solve, RK4 dt=0.15h, "
                               "8 seeded Fourier modes",
                   "elements": n * n, "N": N, "p": w["p"], "dof_per_field": ndof,
                   "parallelism": "single GPU"},
        "rel_err_vs_exact": err64["u"], "rel_err_v_vs_exact": err64["v"],
        "max_rel_err_vs_exact": err64["u_max"],
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK,
                     "traffic": FDM_STAGE_TRAFFIC,
                     "traffic_unit": "HBM bytes per launch (counters, copy-calibrated)",
                     "kernel": "k_stage<double,*,17,4,false> (4 stage variants)",
                     "avg_launch_us": ms64 * 1e3 / launches,
                     "alg_bytes_per_launch": alg_bytes_step / 4,
                     "alg_bytes_per_dof_update": 32 * 8,
                     "kernel_bytes_per_launch": kern_bytes_step / 4,
                     "kernel_bytes_per_dof_update": 24 * 8,
                     "achieved_kernel_bytes": achieved_kern / 1e9,
                     "frac_kernel_bytes": achieved_kern / HBM_PEAK},
    }
    if not args.no_fp32:
        ms32, err32, _ = _time_gpu(w, "fp32", args.steps, args.warmup)
        print("bench: fp32 %.3f ms/step" % (ms32 / args.steps), file=sys.stderr, flush=True)
        # FP32 storage of the stage increments around the FP64 register y: 72 B per DOF,
        # field and step (see the stage kernel), 144 B per DOF-update
        out["fp32"] = {"value": ndof * args.steps / (ms32 * 1e-3), "ms_per_step": ms32 / args.steps,
                       "speedup_vs_fp64": ms64 / ms32,
                       "rel_err_vs_exact": err32["u"], "rel_err_v_vs_exact": err32["v"],
                       "max_rel_err_vs_exact": err32["u_max"],
                       "max_rel_err_v_vs_exact": err32["v_max"],
                       "bytes_per_dof_update": 144,
                       "roofline_frac": 144 * ndof * args.steps / (ms32 * 1e-3) / HBM_PEAK,
                       "note": "stage increments and traces stored in FP32, y accumulated and "
                               "the right-hand side evaluated in FP64"}
    if not args.no_walls:
        out["walls"] = _time_walls(args.steps, args.warmup)
        out["walls"]["ms_vs_periodic"] = out["walls"]["ms_per_step"] / (ms64 / args.steps)
        print("bench: walls %.3f ms/step" % out["walls"]["ms_per_step"], file=sys.stderr,
              flush=True)
    if not args.no_3d:
        out["fdm3d"] = _time_3d(args.steps, args.warmup)
        out["fdm3d"]["fp32"] = _time_3d(args.steps, args.warmup, precision="fp32")
        for k in ("workload", "dof_per_field", "steps", "roofline", "unit"):
            out["fdm3d"]["fp32"].pop(k)
        print("bench: 3d %.3f ms/step (fp32 %.3f)" % (out["fdm3d"]["ms_per_step"],
                                                      out["fdm3d"]["fp32"]["ms_per_step"]),
              file=sys.stderr, flush=True)
    if not args.no_pcg:
        pw = _pcg_workload()
        pn, pN = pw["n"], pw["N"]
        pdof = pn * pn * (pN + 1) ** 2
        ksteps = max(1, min(args.steps, args.pcg_steps))
        ms, its, st64 = _time_pcg(pw, ksteps, 1)
        print("bench: pcg fp64 %.3f ms/step" % (ms / ksteps), file=sys.stderr, flush=True)
        msm, itm, stm = _time_pcg(pw, ksteps, 1, precision="mixed")
        print("bench: pcg mixed %.3f ms/step" % (msm / ksteps), file=sys.stderr, flush=True)
        dmix = max(float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(stm, st64))
        msp, itp, stp = _time_pcg(pw, ksteps, 1, precision="pc32")
        print("bench: pcg pc32 %.3f ms/step" % (msp / ksteps), file=sys.stderr, flush=True)
        dpc = max(float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(stp, st64))
        ic0r = _ic0_section(pw)
        print("bench: pcg ic0 baseline S %.1f its %.1f ms, M %.1f its %.1f ms"
              % (ic0r["S_hat"]["mean_it"], ic0r["S_hat"]["ms_all_elements"],
                 ic0r["M_J"]["mean_it"], ic0r["M_J"]["ms_all_elements"]), file=sys.stderr,
              flush=True)
        flops = _pcg_flops_per_step(its, pn * pn, pN, pw["p"]) * ksteps / (ms * 1e-3)
        pbytes = _pcg_alg_bytes_per_dof_update(pN, pw["p"])
        pach = pbytes * pdof * ksteps / (ms * 1e-3)
        out["pcg"] = {
            "workload": "128x128 mapped elements (X = x + 0.05 sin(2 pi x) sin(2 pi y), same for Y), "
                        "N=12, p=5, c^2 = 1 + 0.5 g (clipped smooth random field, length 0.1), upwind, "
                        "PCG rtol 1e-12, RK4 dt = 0.1 h",
            "dof_per_field": pdof, "steps": ksteps, "ms_per_step": ms / ksteps,
            "value": pdof * ksteps / (ms * 1e-3), "unit": "DOF-updates/s", "dtype": "f64",
            "mean_it_S": its["mean_it_S"], "mean_it_M": its["mean_it_M"],
            "max_it_S": its["max_it_S"], "max_it_M": its["max_it_M"],
            "roofline": {"bound": "hbm", "achieved": pach / 1e9, "peak": HBM_PEAK / 1e9,
                         "unit": "GB/s", "frac": pach / HBM_PEAK,
                         "traffic": PCG_STAGE_TRAFFIC,
                         "traffic_unit": "HBM bytes per RK stage (counters, copy-calibrated)",
                         "alg_bytes_per_dof_update": pbytes,
                         "alg_bytes_per_stage": pbytes * pdof / 4,
                         "avg_stage_us": ms * 1e3 / (4 * ksteps),
                         "alu_achieved_tflops": flops / 1e12, "alu_frac_fp64": flops / 78.6e12,
                         "kernel": "RK stage of 4 launches: k_pcg_lift, k_pcg_solve_w0<0,13,5> "
                                   "(S_hat), k_pcg_solve_w0<1,13,5> (M_J), k_pcg_update"},
            "mixed": {"ms_per_step": msm / ksteps, "value": pdof * ksteps / (msm * 1e-3),
                      "speedup_vs_fp64": ms / msm, "mean_it_S": itm["mean_it_S"],
                      "mean_it_M": itm["mean_it_M"], "mean_refine_sweeps": itm["mean_refine"],
                      "rel_diff_vs_fp64_state": dmix,
                      "note": "FP32 operator for the inner CG iterations, FP64 residual refinement "
                              "to the same rtol; same final tolerance as the FP64 path"},
            "mixed_pc32": {"ms_per_step": msp / ksteps, "value": pdof * ksteps / (msp * 1e-3),
                           "speedup_vs_fp64": ms / msp, "mean_it_S": itp["mean_it_S"],
                           "mean_it_M": itp["mean_it_M"], "rel_diff_vs_fp64_state": dpc,
                           "note": "preconditioner transforms on the FP32 matrix cores inside the "
                                   "FP64 recurrence (operator products, residuals and the stop "
                                   "test FP64); same rtol as the FP64 path"},
            "ic0_baseline": ic0r,
        }
    if not args.no_learned:
        out["learned"] = _learned_section(max(1, min(args.steps, 3)))
        print("bench: learned section done", file=sys.stderr, flush=True)
    if not args.no_batch:
        out["batch"] = _batch_section(max(1, min(args.steps, 5)))
        print("bench: batch section done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = _cpu_baseline(w)
        print("bench: cpu baseline done", file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
