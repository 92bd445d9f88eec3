#!/usr/bin/env python3
"""Benchmark: quasi-static load steps of the 2048 x 2048 AT1 notched square.

A "step" is one load step: set the next load, run ORAM (over-relaxed
alternate minimisation: elastic PCG with multigrid, damage box-QP active set,
relaxation) and its composition with reduced-space Newton (Algorithm 3) to
the stop test, commit alpha_prev.  The workload is the 2048^2 plane-strain
unit square with a seeded edge notch (height and length drawn from
U[0.1, 0.4]), ell = 4h, k_ell = 1e-6, loads t = 0.1 k, k = 1..20.  W warm-up
load steps run first on a separate instance, which is then discarded; a
fresh instance then runs load steps 1..K, all timed (HIP-synchronised on
both sides); value = K / seconds.  The default K = 20 is the whole load
path: elastic loading, crack initiation (t = 1.0), stable growth, the
unstable propagation through the specimen (t = 1.5, thousands of ORAM
sweeps) and the separated body.

Also reported: PCG DOF-iterations per second, per-step latency (p50/p99),
the same steps in mixed precision (with its distance to the FP64 result),
the roofline of the dominant kernel (algorithmic bytes per launch over its
mean duration, measured with HIP events on the solver's stream) with its
measured HBM traffic, and the CPU oracle on the same load steps at a small
size.  Optional samples (--omega-sweep, --with-serve, --with-surfing,
--with-tshock, --with-deflation) add the other workloads to the same line.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "load steps/s + PCG DOF/s (FP64 vs mixed) at 2048² AT1; p50/p99 step latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(n_sample, steps, model="AT1"):
    """The oracle (assembled sparse FE, exact LU solves, exact box-QP active
    set, exact-LU reduced Newton) on the same recipe and the same load steps
    as the GPU leg, ORAM-N at omega = 1 with the same switch and stop
    tolerances, at n_sample^2: its own load steps/s at that size, with no
    extrapolation to the GPU's size."""
    from oracle import am, problems
    from paper_1511_08463_amd import workloads
    S = workloads.CONFIG2_SOLVER
    p, notch, loads, _ = workloads.config2(model, 1.0, seed=0, n=n_sample)
    P = problems.tension_2d(n_sample, n_sample, **workloads.oracle_kwargs(p))
    st = am.initial_state(P, notch.astype(bool))
    sweeps = 0
    t0 = time.perf_counter()
    for t in loads[:steps]:
        o = am.solve_load_step(P, st, t, omega=1.0, newton_on=True, switch_tol=S["switch_tol"],
                               final_tol=S["final_tol"], max_am=20000)
        sweeps += o["sweeps"]
    dt = time.perf_counter() - t0
    threads = os.environ.get("OMP_NUM_THREADS", "unset")
    return {
        "value": steps / dt,
        "unit": f"load steps/s at {n_sample}x{n_sample}",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle ORAM-N (omega=1, switch ||Phi||2<{S['switch_tol']:g}, stop ||Phi||2<"
                   f"{S['final_tol']:g}, exact LU "
                   f"solves) over load steps 1..{steps} (t=0.1..{0.1 * steps:.1f}, through crack "
                   f"initiation and the unstable propagation) of the same recipe at "
                   f"{n_sample}x{n_sample} cells: {sweeps} sweeps in {dt:.2f} s; not scaled to the "
                   f"GPU's size. SciPy SuperLU and sparse matvec are single-threaded; host "
                   f"cpu_count={os.cpu_count()}, affinity={len(os.sched_getaffinity(0))}, "
                   f"OMP_NUM_THREADS={threads}"),
        "seconds": dt,
    }


def serve(args):
    """The served stream (config 5): first --instances requests of the seeded
    Poisson stream, admitted under a device memory budget, run concurrently."""
    import numpy as np
    from paper_1511_08463_amd import serving, workloads
    reqs = [serving.Request(r["rid"], r["params"], r["notch"], r["loads"], r["arrival"])
            for r in workloads.config5(n_instances=args.instances, solver=args.serve_solver)]
    budget = int(args.budget_gb * 1e9)
    log(f"[serve] {len(reqs)} requests, budget {args.budget_gb} GB, {args.workers} workers, "
        f"GPU_MAX_HW_QUEUES={os.environ.get('GPU_MAX_HW_QUEUES', 'default')}")
    def progress(done, total, t):
        if done % 16 == 0 or done == total:
            log(f"[serve] {done}/{total} requests finished at {t:.1f} s")

    # a sample of the stream (the first two requests of each side up to 512)
    # is re-run alone afterwards and compared bit for bit with its result in
    # the mix
    sample, seen = [], {}
    for r in reqs:
        n = r.params["nx"]
        if n <= 512 and seen.get(n, 0) < 2:
            seen[n] = seen.get(n, 0) + 1
            sample.append(r)
    keep = {r.rid for r in sample} if args.serve_check else set()
    svc = serving.Service(budget, max_slots=args.slots, workers=args.workers, keep_state=keep,
                          progress=progress)
    summary, results = svc.run(reqs)
    log(f"[serve] {summary}")
    if args.serve_check:
        equal = []
        for r in sample:
            alone, _ = serving.run_alone(r)
            same = all(np.array_equal(a, b) for a, b in zip(alone, results[r.rid].state))
            equal.append(same)
            log(f"[serve] rid {r.rid} n={r.params['nx']} steps={len(r.loads)} alone == mixed: {same}")
        summary["alone_equal"] = f"{sum(equal)}/{len(equal)}"
        summary["alone_checked"] = [dict(rid=r.rid, n=r.params["nx"]) for r in sample]
    return summary


def thermal(args):
    """Config 3: the 128x128x32 thermal-shock slab, FP64 or mixed, AM load steps."""
    import torch
    from paper_1511_08463_amd import fracture, workloads
    p, loads = workloads.config3(dt_max_factor=args.dt_factor)
    prec = fracture.FRACTURE_MIXED if args.precision == "mixed" else fracture.FRACTURE_FP64
    if args.thermal_newton:
        # ORAM-N with the benchmark's inexact sweeps and stop test
        S = dict(workloads.CONFIG2_SOLVER, max_am=5000)
        params = fracture.make_params(**p, **S, precision=prec)
    else:
        params = fracture.make_params(**p, am_tol=args.am_tol, pcg_rtol=args.pcg_rtol, max_am=2000,
                                      vi_cg_rtol=args.vi_cg_rtol, newton=0, precision=prec)
    solver = fracture.Fracture(params, None, device="cuda:0")
    log(f"[thermal] 128x128x32 Kuhn, {args.precision}, DT_c={workloads.thermal_dtc(p):.3f}")
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, t in enumerate(loads[: args.warmup + args.steps]):
        solver.set_load(t)
        st = solver.solve_step(raise_on_error=False)
        if st["code"] != fracture.FRACTURE_OK:
            log(f"[thermal] step {k + 1} DT={t:.3f} failed: {st}")
            raise fracture.FractureError(st["code"], "fracture_solve_step")
        stats.append(st)
        el, su = solver.energy()
        log(f"[thermal] step {k + 1} DT={t:.3f} sweeps={st['sweeps']} pcg={st['pcg_iters']} "
            f"vi={st['vi_iters']} vi_cg={st['vi_cg_iters']} newton={st['newton_iters']} "
            f"minres={st['minres_iters']} ms={st['ms_total']:.1f} (pcg {st['ms_pcg']:.1f}, "
            f"vi {st['ms_vi']:.1f}, newton {st['ms_newton']:.1f}) E_el={el:.4e} E_s={su:.4e}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rl = {}
    for name, kid in (("smooth", fracture.FRACTURE_KERNEL_SMOOTH), ("apply", fracture.FRACTURE_KERNEL_APPLY)):
        ms, nbytes = fracture.fracture_time_kernel(solver.h, kid, args.kernel_reps)
        rl[name] = {"us": ms * 1e3, "gbs": nbytes / (ms * 1e-3) / 1e9}
        log(f"[thermal] kernel {name}: {ms * 1e3:.1f} us, {rl[name]['gbs']:.0f} GB/s")
    solver.close()
    n = args.warmup + args.steps
    algo = ("ORAM-N (omega=1, the 2048^2 benchmark's inexact sweeps, stop ||Phi||2<"
            f"{workloads.CONFIG2_SOLVER['final_tol']:g})" if args.thermal_newton
            else f"AM to ||dalpha||inf<{args.am_tol:g}")
    return {"workload": "128x128x32 hexes x 6 Kuhn tetrahedra, AT1, ell=4h, thermal eigenstrain "
                        f"-DT exp(-x/0.05) I, DT_k=(k/15) {args.dt_factor:g} DT_c, k=1..{n}, {algo}",
            "precision": args.precision, "load_steps": n, "seconds": dt, "load_steps_per_s": n / dt,
            "sweeps": sum(s["sweeps"] for s in stats), "pcg_iters": sum(s["pcg_iters"] for s in stats),
            "newton_iters": sum(s["newton_iters"] for s in stats), "kernels": rl}


KERNELS = ("smooth", "apply", "vi_eval", "helm", "copy")
LIVE_CAP = 16384  # finest-level Chebyshev steps timed (every fifth, from the start of the timed region)


def roofline(live, dom, traffic, rl):
    """The dominant kernel, the finest-level Chebyshev step k_col2d<SMOOTH>
    (k_col_prol_smooth2d for the first post-smoothing step of a V-cycle):
    its launches inside the timed region (live HIP events; algorithmic bytes
    of each launch summed), with the back-to-back measurement of the 88 B/node
    form alongside."""
    out = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    if live:
        out.update({
            "kernel": (f"k_col2d<SMOOTH>: the finest-level Chebyshev steps of the V-cycles in the "
                       f"timed region (every fifth: {live['launches']} launches, "
                       f"{live['bytes'] / 1e6:.1f} MB "
                       f"algorithmic per launch on average: coefficients 8 B, b, x_in, a distinct "
                       f"d_in, x_out, d_out 16 B each per node, and 16 B per coarse node of the "
                       f"coarse correction for the first post-smoothing step, which carries the "
                       f"prolongation)"),
            "achieved": live["gbs"], "frac": live["gbs"] / HBM_PEAK_GBS,
            "avg_us": live["us"], "launches": live["launches"], "bytes_per_launch": live["bytes"],
            "traffic": traffic,
            "traffic_gbs": traffic / (live["us"] * 1e-6) / 1e9 if traffic else None,
        })
    else:
        out.update({"kernel": "k_col2d<SMOOTH> (finest-level Chebyshev step, 88 B/node)",
                    "achieved": dom["gbs"], "frac": dom["gbs"] / HBM_PEAK_GBS, "traffic": None,
                    "traffic_gbs": None})
    out["back_to_back_88B"] = {"us": round(dom["us"], 2), "gbs": round(dom["gbs"], 1)}
    out["per_kernel_gbs"] = {k: round(v["gbs"], 1) for k, v in rl.items()}
    out["per_kernel_us"] = {k: round(v["us"], 2) for k, v in rl.items()}
    return out


def time_kernels(solver, reps):
    """Mean duration of each hot kernel over back-to-back launches, timed with
    HIP events on the solver's stream, and its algorithmic bytes."""
    from paper_1511_08463_amd import fracture
    ids = {"smooth": fracture.FRACTURE_KERNEL_SMOOTH, "apply": fracture.FRACTURE_KERNEL_APPLY,
           "vi_eval": fracture.FRACTURE_KERNEL_VI_EVAL, "helm": fracture.FRACTURE_KERNEL_HELM,
           "copy": fracture.FRACTURE_KERNEL_COPY}
    rl = {}
    for name in KERNELS:
        ms, nbytes = fracture.fracture_time_kernel(solver.h, ids[name], reps)
        rl[name] = {"us": ms * 1e3, "bytes": nbytes, "gbs": nbytes / (ms * 1e-3) / 1e9}
        log(f"[bench] kernel {name}: {ms * 1e3:.1f} us/launch, {nbytes / 1e6:.1f} MB -> "
            f"{rl[name]['gbs']:.0f} GB/s")
    return rl


# HBM bytes per launch of the finest-level Chebyshev step at 2048^2, averaged
# over its launches inside the V-cycles of load steps 1-3 (the mix of the
# timed region: two steps with x given, one from zero, one that also applies
# the prolongation), from rocprofv3 FETCH_SIZE and WRITE_SIZE of the headline leg,
# each scaled by the factor that maps the same counter on the plain copy
# kernel to its known bytes.  Valid only for the sources they were taken on
# (sha256 over the files below: the kernels and the host code that sets each
# launch's operands).
TRAFFIC = {
    # profiles/hbm_traffic_2048_at1.md: mean over the 570 launches of the
    # warm-up step and load steps 1-3, FETCH x 1.9994 + WRITE x 1.0000
    "bytes": 292202601,
    "source_sha256": "e9ebf4d73ceb724703b657af7fce4c05a3d8f54eec082acb96888c5374fed235",
}
TRAFFIC_SOURCES = ("paper_1511_08463_amd/csrc/common.h", "paper_1511_08463_amd/csrc/ops2d.h",
                   "paper_1511_08463_amd/csrc/kernels2d.hip", "paper_1511_08463_amd/csrc/solver.hip")


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    if TRAFFIC is None or TRAFFIC["source_sha256"] != kernel_source_sha():
        return None
    return TRAFFIC["bytes"]


def surfing(args):
    """The surfing slab (Sec. 4.1) at ell = --surf-ell, h = ell/4, ORAM-N:
    load steps/s over t = 0.1 .. 0.8 and the dissipation rate against
    Griffith's Gc v."""
    import numpy as np
    import torch
    from paper_1511_08463_amd import fracture, workloads
    p, notch, loads = workloads.surfing(args.surf_ell, steps=9)
    params = fracture.make_params(**p, newton=args.newton, max_am=args.max_am,
                                  pcg_rtol=args.pcg_rtol, omega=args.omega,
                                  omega_auto=1 if args.omega_auto else 0, am_tol=args.am_tol,
                                  newton_forcing_mode=args.forcing_mode,
                                  pcg_reduction=args.pcg_reduction,
                                  precision=fracture.FRACTURE_MIXED if args.precision == "mixed"
                                  else fracture.FRACTURE_FP64)
    solver = fracture.Fracture(params, notch, device="cuda:0")
    nx, ny = p["nx"], p["ny"]
    x = np.arange(nx + 1) * (2.0 / nx)
    log(f"[surfing] {nx}x{ny} cells, ell={args.surf_ell}, {args.precision}, omega={args.omega}, "
        f"newton={args.newton}")
    surf, tips, stats = [], [], []
    torch.cuda.synchronize()
    t_start = None
    for k, t in enumerate(loads):
        if k == 1:
            torch.cuda.synchronize()
            t_start = time.perf_counter()
        solver.set_load(t)
        st = solver.solve_step()
        stats.append(st)
        surf.append(solver.energy()[1])
        a = solver.state()[1].reshape(ny + 1, nx + 1)[ny // 2]
        tips.append(float(x[a > 0.5].max()))
        log(f"[surfing] t={t:.1f} sweeps={st['sweeps']} pcg={st['pcg_iters']} newton={st['newton_iters']} "
            f"minres={st['minres_iters']} ms={st['ms_total']:.1f} Es={surf[-1]:.5f} tip={tips[-1]:.4f}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t_start
    solver.close()
    ts = np.array(loads)
    late = ts >= 0.3 - 1e-12
    rate = float(np.polyfit(ts[late], np.array(surf)[late], 1)[0])
    return {"workload": (f"surfing slab [0,2]x[0,1] (Sec. 4.1), {nx}x{ny} cells (h = ell/4), AT1, "
                         f"ell={args.surf_ell}, plane stress, K_I = sqrt(Gc E), v = 1, L_c = 0.05; "
                         f"{'ORAM-N' if args.newton else 'ORAM'} omega="
                         f"{('auto <= %g' % args.omega) if args.omega_auto else args.omega}, "
                         f"t = 0.1..0.8 timed after t = 0"),
            "precision": args.precision, "omega": args.omega, "load_steps": len(loads) - 1, "seconds": dt,
            "load_steps_per_s": (len(loads) - 1) / dt,
            "sweeps": sum(s["sweeps"] for s in stats[1:]),
            "newton_iters": sum(s["newton_iters"] for s in stats[1:]),
            "dissipation_rate": rate, "griffith_rate": 1.0, "tips": tips}


def tshock(args, ratios=(2.0, 4.0, 8.0, 16.0), omegas=(0.8, 1.0, 1.2, 1.4, 1.6, 1.8)):
    """The 2D thermal shock (Sec. 4.3) on the paper's 40 x 10 slab, ell = 1,
    --tshock-n x --tshock-n/4 cells: plain ORAM sweeps over the evolution
    tau = 0.1 .. --tshock-tau in steps of 0.1, for each shock intensity
    DT/DT_c and over-relaxation factor (the experiment of Table 3)."""
    import torch
    from paper_1511_08463_amd import fracture, workloads
    nx = args.tshock_n
    ny = nx // 4
    nsteps = int(round(args.tshock_tau / 0.1))
    taus = [round(0.1 * k, 10) for k in range(1, nsteps + 1)]
    rows = {}
    for ratio in ratios:
        row = {}
        for om in omegas:
            p = workloads.tshock(nx, ny, 40.0, 10.0, ratio=ratio, omega=om)
            params = fracture.make_params(**p, newton=0, am_tol=args.am_tol,
                                          max_am=args.tshock_max_am, pcg_rtol=args.pcg_rtol)
            solver = fracture.Fracture(params, None, device="cuda:0")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sweeps, ok = 0, True
            for tau in taus:
                solver.set_load(tau)
                try:
                    st = solver.solve_step()
                except fracture.FractureError as e:
                    # sweep limit of a step: reported, and the evolution stops there
                    log(f"[tshock] DT/DT_c={ratio:g} omega={om:g} tau={tau:g}: {e}")
                    ok = False
                    break
                sweeps += st["sweeps"]
                ok = ok and st["converged"]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            amax = float(solver.state()[1].max())
            solver.close()
            log(f"[tshock] DT/DT_c={ratio:g} omega={om:g}: {sweeps} sweeps, {dt:.2f} s, "
                f"converged={ok}, max alpha {amax:.3f}")
            row[f"{om:g}"] = {"sweeps": sweeps, "seconds": round(dt, 3), "converged": ok}
        base = row["1"]["sweeps"] if "1" in row and row["1"]["converged"] else None
        best = min((v["sweeps"] for v in row.values() if v["converged"]), default=None)
        row["reduction_vs_omega1"] = round(1.0 - best / base, 4) if base and best else None
        rows[f"{ratio:g}"] = row
    return {"workload": (f"2D thermal shock (Sec. 4.3): slab 40 x 10, ell = 1, {nx}x{ny} cells "
                         f"(h = ell/{nx / 40:g}), AT1, plane strain, nu = 0.3, erfc eigenstrain, "
                         f"u_x = 0 laterally, u_y = 0 on top; plain ORAM to ||dalpha||inf < "
                         f"{args.am_tol:g}, tau = 0.1..{args.tshock_tau:g} in steps of 0.1; "
                         f"sweeps summed over the evolution"),
            "sweeps": rows}


def deflation(args):
    """Crack-aware deflation of the elastic CG (Sec. 3.1) on a broken
    specimen: the --n x --n tension square, AT1 damage profile (ell = 4h)
    across the mid-line, alpha_prev = alpha, one plain ORAM load step at
    t = 0.5 from u = 0, with and without deflation."""
    import numpy as np
    import torch
    from paper_1511_08463_amd import fracture, workloads
    n = args.n
    p = workloads.tension(n, 4.0 / n, args.model)
    y = np.repeat(np.arange(n + 1) / n, n + 1)
    alpha = np.clip(1.0 - np.abs(y - 0.5) / (8.0 / n), 0.0, 1.0) ** 2
    out, states = {}, {}
    for dfl in (0, 1):
        params = fracture.make_params(**p, newton=0, am_tol=args.am_tol, pcg_rtol=args.pcg_rtol,
                                      vi_cg_rtol=args.vi_cg_rtol, max_am=args.max_am, deflate=dfl)
        solver = fracture.Fracture(params, None, device="cuda:0")
        solver.set_state(u=np.zeros(2 * alpha.size), alpha=alpha, alpha_prev=alpha)
        solver.set_load(0.5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = solver.solve_step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        nf = solver.fragments()[0] if dfl else None
        states[dfl] = solver.state()[0]
        solver.close()
        out["deflated" if dfl else "plain"] = {
            "sweeps": st["sweeps"], "pcg_iters": st["pcg_iters"], "ms_pcg": round(st["ms_pcg"], 2),
            "seconds": round(dt, 3), "fragments": nf, "converged": st["converged"]}
        log(f"[deflation] deflate={dfl}: {st['sweeps']} sweeps, {st['pcg_iters']} PCG iterations, "
            f"PCG {st['ms_pcg']:.1f} ms, step {dt:.2f} s, fragments {nf}")
    d = np.linalg.norm(states[1] - states[0]) / np.linalg.norm(states[0])
    out["rel_l2_u_deflated_vs_plain"] = float(d)
    out["workload"] = (f"{n}x{n} tension square, {args.model}, ell = 4h, damage profile "
                       f"(1 - |y - 1/2| / 2 ell)^2 across the mid-line (two fragments), "
                       f"alpha_prev = alpha, one ORAM load step t = 0.5 from u = 0 to "
                       f"||dalpha||inf < {args.am_tol:g}, PCG rtol {args.pcg_rtol:g}")
    return out


def shard(args):
    """One GPU's share of a slab decomposition of the --n x --n square over R
    GPUs: the --n x --n/R slab with the same h, ell = 4h and tension strain,
    alpha = 0.  One ORAM load step from u = 0 (a full elastic PCG solve to
    --pcg-rtol, then the damage step) per R; reports the PCG's time per
    iteration and the back-to-back finest-level Chebyshev step on the slab.
    Halo exchanges and all-reduces are not part of it (one GPU)."""
    import torch
    from paper_1511_08463_amd import fracture, workloads
    n = args.n
    rows = []
    for r in (1, 2, 4, 8):
        if n % r or (n // r) % 16:
            continue
        ny = n // r
        p = dict(workloads.tension(n, 4.0 / n, args.model), ny=ny, ly=ny / n)
        params = fracture.make_params(**p, newton=0, am_tol=args.am_tol, pcg_rtol=args.pcg_rtol,
                                      vi_cg_rtol=args.vi_cg_rtol, max_am=args.max_am,
                                      cheb_degree=args.cheb_degree,
                                      use_graphs=0 if args.no_graphs else 1)
        solver = fracture.Fracture(params, None, device="cuda:0")
        solver.set_load(0.1 * ny / n)              # the headline's first strain, u_y = 0.1 at y = 1
        torch.cuda.synchronize()
        st = solver.solve_step()
        torch.cuda.synchronize()
        ms, nbytes = fracture.fracture_time_kernel(solver.h, fracture.FRACTURE_KERNEL_SMOOTH,
                                                   args.kernel_reps)
        solver.close()
        dofs = 2 * (n + 1) * (ny + 1)
        it_ms = st["ms_pcg"] / max(st["pcg_iters"], 1)
        rows.append({"gpus": r, "slab": f"{n}x{ny}", "dofs": dofs, "pcg_iters": st["pcg_iters"],
                     "pcg_ms_per_iter": round(it_ms, 4),
                     "dof_iter_per_s": round(dofs / (it_ms * 1e-3), 1),
                     "smooth_us": round(ms * 1e3, 2),
                     "smooth_gbs": round(nbytes / (ms * 1e-3) / 1e9, 1)})
        log(f"[shard] {n}x{ny} ({r} GPUs): {st['pcg_iters']} PCG iterations, "
            f"{it_ms:.3f} ms each ({rows[-1]['dof_iter_per_s'] / 1e9:.2f} G DOF-it/s), "
            f"Chebyshev step {ms * 1e3:.1f} us ({rows[-1]['smooth_gbs']:.0f} GB/s)")
    return {"workload": (f"{n} x {n}/R slabs of the {n}^2 square (h = 1/{n}, ell = 4h, "
                         f"{args.model}, alpha = 0), one ORAM load step from u = 0, PCG rtol "
                         f"{args.pcg_rtol:g}; no halo exchange or all-reduce"),
            "slabs": rows}


def parse_args(argv=None):
    from paper_1511_08463_amd.workloads import CONFIG2_SOLVER as S
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed load steps: steps 1..K of the 20-step load path")
    ap.add_argument("--warmup", type=int, default=1,
                    help="untimed load steps run first on a separate instance that is then discarded")
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--model", default="AT1")
    ap.add_argument("--omega", type=float, default=1.0)
    ap.add_argument("--omega-auto", action="store_true",
                    help="per-step omega from the measured AM convergence factor (cap: --omega)")
    ap.add_argument("--am-tol", type=float, default=S["am_tol"])
    ap.add_argument("--max-am", type=int, default=S["max_am"], help="sweep limit per load step")
    ap.add_argument("--pcg-rtol", type=float, default=S["pcg_rtol"])
    ap.add_argument("--newton", type=int, default=S["newton"], help="ORAM-N (1) or ORAM alone (0)")
    ap.add_argument("--switch-tol", type=float, default=S["switch_tol"])
    ap.add_argument("--final-tol", type=float, default=S["final_tol"])
    ap.add_argument("--minres-rtol", type=float, default=S["minres_rtol"])
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--newton-vcycles", type=int, default=S["newton_vcycles"],
                    help="V-cycles per action of A^-1 in the Newton block preconditioner")
    ap.add_argument("--no-graphs", action="store_true", help="launch eagerly (no HIP graph replay)")
    ap.add_argument("--cheb-degree", type=int, default=S["cheb_degree"], help="Chebyshev steps per V-cycle side")
    ap.add_argument("--newton-precond", type=int, default=S["newton_precond"],
                    help="0: symmetric block preconditioner (paper), 1: block diagonal")
    ap.add_argument("--newton-forcing", type=float, default=S["newton_forcing"],
                    help="adaptive Newton forcing factor (0: fixed --minres-rtol)")
    ap.add_argument("--vi-cg-rtol", type=float, default=S["vi_cg_rtol"],
                    help="relative tolerance of the damage CG inside the active-set method")
    ap.add_argument("--pcg-reduction", type=float, default=S["pcg_reduction"],
                    help="ORAM-N: elastic solves of ORAM sweeps stop at this reduction of the warm-start residual")
    ap.add_argument("--vi-reduction", type=float, default=S["vi_reduction"],
                    help="ORAM-N: damage solves of ORAM sweeps stop at this reduction of their starting max |Phi|")
    ap.add_argument("--forcing-mode", type=int, default=S["newton_forcing_mode"],
                    help="1: Eisenstat-Walker forcing terms; 0: the final-tolerance target")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--cpu-n", type=int, default=32,
                    help="mesh of the oracle's CPU baseline (same recipe and load steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--mixed-budget", type=float, default=300.0,
                    help="skip the mixed leg when the FP64 leg took longer than this (s), so the "
                         "default run stays within minutes")
    ap.add_argument("--snap-step", type=int, default=9,
                    help="load step whose state the mixed leg is also compared at (9: t = 0.9, "
                         "before initiation); 0 for none")
    ap.add_argument("--deflate", action="store_true",
                    help="deflate the elastic CG of the headline legs by the fragments' rigid modes")
    # optional samples of the other workloads in the same JSON line
    ap.add_argument("--omega-sweep", action="store_true",
                    help="also time the same steps at omega = 1.4 and 1.8")
    ap.add_argument("--with-serve", action="store_true", help="also run the served-stream sample")
    ap.add_argument("--with-surfing", action="store_true", help="also run the surfing sample")
    ap.add_argument("--with-tshock", action="store_true", help="also run the thermal shock sample")
    ap.add_argument("--with-deflation", action="store_true", help="also run the deflation sample")
    # one workload alone
    ap.add_argument("--serve", action="store_true", help="run only the served stream")
    ap.add_argument("--thermal", action="store_true", help="run only the 3D thermal slab (config 3)")
    ap.add_argument("--dt-factor", type=float, default=16.0, help="thermal ramp end in units of DT_c")
    ap.add_argument("--thermal-newton", action="store_true",
                    help="thermal slab by ORAM-N (default: alternate minimisation)")
    ap.add_argument("--surfing", action="store_true", help="run only the surfing slab (Sec. 4.1)")
    ap.add_argument("--surf-ell", type=float, default=1.0 / 128)
    ap.add_argument("--tshock", action="store_true",
                    help="run only the 2D thermal shock omega sweep (Sec. 4.3, Table 3)")
    ap.add_argument("--tshock-n", type=int, default=256, help="thermal shock cells along the slab")
    ap.add_argument("--tshock-tau", type=float, default=2.0, help="last tau of the thermal shock")
    ap.add_argument("--tshock-max-am", type=int, default=20000, help="sweep limit per thermal shock step")
    ap.add_argument("--deflation", action="store_true",
                    help="run only the deflated vs plain elastic CG comparison")
    ap.add_argument("--shard", action="store_true",
                    help="run only the per-GPU slabs of a 1/2/4/8-GPU row decomposition")
    ap.add_argument("--kernels-only", action="store_true",
                    help="time the hot kernels only (no solve), e.g. under hardware counters")
    ap.add_argument("--instances", type=int, default=256, help="served stream: requests run")
    ap.add_argument("--serve-solver", choices=("am", "oramn"), default="oramn",
                    help="served stream: ORAM-N with the benchmark's inexact sweeps (default) or "
                         "alternate minimisation")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="served stream: hardware queues of the process (GPU_MAX_HW_QUEUES, at most "
                         "32), so that the instances' streams do not share four queues")
    ap.add_argument("--budget-gb", type=float, default=4.0)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--no-serve-check", dest="serve_check", action="store_false",
                    help="served stream: skip re-running a sample alone for the bitwise check")
    ap.add_argument("--slots", type=int, default=32)
    ap.add_argument("--dry-run", action="store_true",
                    help="validate the arguments, print the plan as JSON and exit (no GPU)")
    return ap.parse_args(argv)


NSTEPS = 20   # the load path of the workload: t = 0.1 k, k = 1..20


def plan(args):
    """Validated run plan, or (None, message) for an invalid request."""
    if args.gpus != 1:
        return None, ("the benchmark runs on one GPU only; --gpus must be 1 "
                      "(the multi-GPU decomposition is designed, not implemented)")
    if not 1 <= args.steps <= NSTEPS:
        return None, f"--steps must be in 1..{NSTEPS} (the load path has {NSTEPS} steps)"
    if args.warmup < 0:
        return None, "--warmup must be >= 0"
    return {"timed_steps": list(range(1, args.steps + 1)),
            "warmup_steps": list(range(1, min(args.warmup, NSTEPS) + 1)),
            "warmup_instance": "separate, discarded before the timed instance is created",
            "legs": (["fp64" if args.precision == "fp64" else "mixed"]
                     + (["mixed"] if args.precision == "fp64" and not args.no_mixed else [])
                     + (["omega 1.4", "omega 1.8"] if args.omega_sweep else [])
                     + (["serve"] if args.with_serve else []) + (["surfing"] if args.with_surfing else [])
                     + (["tshock"] if args.with_tshock else [])
                     + (["deflation"] if args.with_deflation else [])
                     + ([] if args.no_cpu_baseline else [f"cpu_baseline {args.cpu_n}^2"]))}, None


def pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=float), q)) if len(v) else None


def main():
    args = parse_args()
    pl, err = plan(args)
    if pl is None:
        print(json.dumps({"error": err}), flush=True)
        sys.exit(2)
    if args.dry_run:
        print(json.dumps({"plan": pl}), flush=True)
        return
    if args.serve or args.with_serve:
        # read by the HIP runtime when it initialises (no device call has been made yet)
        os.environ["GPU_MAX_HW_QUEUES"] = str(max(1, min(args.hw_queues, 32)))

    import numpy as np
    import torch
    from paper_1511_08463_amd import fracture, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.serve:
        summary = serve(args)
        print(json.dumps({"serving": summary}), flush=True)
        return
    if args.thermal:
        print(json.dumps({"thermal": thermal(args)}), flush=True)
        return
    if args.surfing:
        print(json.dumps({"surfing": surfing(args)}), flush=True)
        return
    if args.tshock:
        print(json.dumps({"tshock": tshock(args)}), flush=True)
        return
    if args.deflation:
        print(json.dumps({"deflation": deflation(args)}), flush=True)
        return
    if args.shard:
        print(json.dumps({"shard": shard(args)}), flush=True)
        return
    p, notch, loads, (y0, a) = workloads.config2(args.model, args.omega, seed=0, n=args.n)

    def make_solver(precision, omega=None):
        pp = dict(p, omega=args.omega if omega is None else omega)
        params = fracture.make_params(**pp, am_tol=args.am_tol, pcg_rtol=args.pcg_rtol,
                                      vi_cg_rtol=args.vi_cg_rtol, max_am=args.max_am, newton=args.newton,
                                      switch_tol=args.switch_tol, final_tol=args.final_tol,
                                      minres_rtol=args.minres_rtol,
                                      newton_vcycles=args.newton_vcycles,
                                      newton_forcing=args.newton_forcing,
                                      newton_forcing_mode=args.forcing_mode,
                                      pcg_reduction=args.pcg_reduction,
                                      vi_reduction=args.vi_reduction,
                                      cheb_degree=args.cheb_degree,
                                      newton_precond=args.newton_precond,
                                      omega_auto=1 if args.omega_auto else 0,
                                      deflate=1 if args.deflate and precision != "mixed" else 0,
                                      use_graphs=0 if args.no_graphs else 1,
                                      precision=fracture.FRACTURE_MIXED if precision == "mixed"
                                      else fracture.FRACTURE_FP64)
        return fracture.Fracture(params, notch, device=dev)

    if args.kernels_only:
        # the hot kernels alone (no solve), for hardware-counter runs
        solver = make_solver(args.precision)
        solver.set_load(loads[0])
        rl = time_kernels(solver, args.kernel_reps)
        solver.close()
        print(json.dumps({"kernels": rl}), flush=True)
        return

    free_dofs = 2 * (args.n + 1) ** 2 - (args.n + 1) * 2 - 1

    def leg(precision, omega=None, live=False):
        """W untimed load steps on a discarded instance, then load steps
        1..K of a fresh instance, timed.  live: time the finest-level
        Chebyshev steps of the timed region with HIP events on the solver's
        stream (the roofline's kernel)."""
        om = args.omega if omega is None else omega
        log(f"[bench] {precision} {args.n}^2 {args.model} omega={om} notch y0={y0:.4f} "
            f"a={a:.4f} warmup={args.warmup} (discarded instance) steps={args.steps}")
        last = [time.perf_counter()]

        def monitor(sweep, da, phi):
            # progress every few seconds
            now = time.perf_counter()
            if now - last[0] > 10.0:
                last[0] = now
                log(f"[bench]   ... sweep/newton {sweep} dalpha={da:.2e} phi={phi:.2e}")

        def run(solver, k, tag):
            solver.set_load(loads[k])
            st = solver.solve_step()
            log(f"[bench] {precision} {tag} step {k + 1} t={loads[k]:.2f} sweeps={st['sweeps']} "
                f"pcg={st['pcg_iters']} vi={st['vi_iters']} vi_cg={st['vi_cg_iters']} "
                f"newton={st['newton_iters']} minres={st['minres_iters']} "
                f"fails={st['newton_failures']} dalpha={st['dalpha_inf']:.2e} phi={st['phi_l2']:.2e} "
                f"ms={st['ms_total']:.1f} (pcg {st['ms_pcg']:.1f}, vi {st['ms_vi']:.1f}, "
                f"newton {st['ms_newton']:.1f})")
            return st

        if args.warmup:
            warm = make_solver(precision, om)
            warm.set_monitor(monitor)
            for k in range(min(args.warmup, NSTEPS)):
                run(warm, k, "warm-up")
            torch.cuda.synchronize()
            warm.close()
            del warm
        solver = make_solver(precision, om)
        solver.set_monitor(monitor)
        if live:
            fracture.fracture_kernel_timing(solver.h, fracture.FRACTURE_KERNEL_SMOOTH, LIVE_CAP)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats, snap, paused, step_s = [], None, 0.0, []
        for k in range(args.steps):
            ts = time.perf_counter()
            stats.append(run(solver, k, "timed"))
            step_s.append(time.perf_counter() - ts)
            if k + 1 == args.snap_step:
                # the state before crack initiation, copied out untimed
                torch.cuda.synchronize()
                tp = time.perf_counter()
                snap = solver.state()
                paused += time.perf_counter() - tp
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0 - paused
        live_stats = None
        if live:
            n_l, ms_l, b_l = fracture.fracture_kernel_timing_read(solver.h)
            fracture.fracture_kernel_timing(solver.h, fracture.FRACTURE_KERNEL_SMOOTH, 0)
            if n_l > 0:
                live_stats = {"launches": n_l, "us": 1e3 * ms_l / n_l, "bytes": b_l / n_l,
                              "gbs": b_l / (ms_l * 1e-3) / 1e9}
                log(f"[bench] live finest-level Chebyshev steps: {n_l} launches, "
                    f"{live_stats['us']:.1f} us, {live_stats['bytes'] / 1e6:.1f} MB -> "
                    f"{live_stats['gbs']:.0f} GB/s")
        pcg_iters = sum(s["pcg_iters"] for s in stats)
        pcg_s = sum(s["ms_pcg"] for s in stats) / 1e3
        step_ms = [round(s["ms_total"], 2) for s in stats]
        res = {
            "value": args.steps / elapsed,
            "ms_per_step": 1e3 * elapsed / args.steps,
            "seconds": elapsed,
            "pcg_dof_iter_per_s": free_dofs * pcg_iters / pcg_s if pcg_s > 0 else None,
            "sweeps": sum(s["sweeps"] for s in stats),
            "pcg_iters": pcg_iters,
            "vi_cg_iters": sum(s["vi_cg_iters"] for s in stats),
            "newton_iters": sum(s["newton_iters"] for s in stats),
            "minres_iters": sum(s["minres_iters"] for s in stats),
            "step_ms": step_ms,
            "step_sweeps": [s["sweeps"] for s in stats],
            "p50_step_ms": pct(step_ms, 50), "p99_step_ms": pct(step_ms, 99),
            "live": live_stats,
        }
        state = solver.state()
        energy = solver.energy()
        return solver, res, (state, snap), energy

    solver, res, (state64, snap64), energy64 = leg(args.precision, live=True)
    rl = time_kernels(solver, args.kernel_reps)
    solver.close()
    dom = rl["smooth"]
    traffic = recorded_traffic()
    precision_note = ("f64" if args.precision == "fp64" else "f32 operator and multigrid inside f64 refinement")
    out = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "load steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": precision_note,
        "data": "synthetic",
        "config": {
            "workload": (f"{args.n}x{args.n} plane-strain unit square, P1 right-diagonal triangles, "
                         f"{args.model}, ell=4h, k_ell=1e-6, seeded edge notch (y0={y0:.4f}, a={a:.4f}), "
                         f"tension load steps t=0.1k, k=1..{args.steps} of {NSTEPS} all timed "
                         f"(elastic loading, crack initiation, stable growth, the unstable "
                         f"propagation through the specimen and the separated body); "
                         + (f"ORAM omega={args.omega} switching to reduced-space Newton at ||Phi||2<{args.switch_tol:g}, "
                            f"stop ||Phi||2<{args.final_tol:g}, MINRES forcing "
                            + ((("Eisenstat-Walker, " if args.forcing_mode == 1 else "")
                                + f"target {args.newton_forcing:g} final_tol/||Phi||, floor {args.minres_rtol:g}")
                               if args.newton_forcing > 0 else f"{args.minres_rtol:g}")
                            + f", {args.newton_vcycles} V-cycle(s) per A^-1"
                            if args.newton else
                            f"ORAM omega={args.omega} to ||dalpha||inf<{args.am_tol:g}")
                         + f", PCG rtol {args.pcg_rtol:g}"
                         + (f" (ORAM sweeps: or {args.pcg_reduction:g} x warm-start residual; damage "
                            f"solve to {args.vi_reduction:g} x its starting max |Phi|)"
                            if args.newton and args.pcg_reduction > 0 else "")
                         + f"; {args.warmup} warm-up load step(s) on a separate, discarded instance"),
            "precision": args.precision,
            "newton": bool(args.newton),
            "deflate": bool(args.deflate),
        },
        "seconds": res["seconds"],
        "pcg_dof_iter_per_s": res["pcg_dof_iter_per_s"],
        "sweeps": res["sweeps"],
        "pcg_iters": res["pcg_iters"],
        "vi_cg_iters": res["vi_cg_iters"],
        "newton_iters": res["newton_iters"],
        "minres_iters": res["minres_iters"],
        "step_ms": res["step_ms"],
        "step_sweeps": res["step_sweeps"],
        "p50_step_ms": res["p50_step_ms"],
        "p99_step_ms": res["p99_step_ms"],
        "final_energy": {"elastic": energy64[0], "surface": energy64[1]},
        "roofline": roofline(res["live"], dom, traffic, rl),
    }
    if args.omega_sweep and args.precision == "fp64":
        # the other over-relaxation factors of the workload, same load steps
        out["omega_sweep"] = {}
        for om in (1.4, 1.8):
            if om == args.omega:
                continue
            s_om, r_om, (st_om, _), e_om = leg(args.precision, omega=om)
            s_om.close()
            o_om = {k: r_om[k] for k in ("value", "ms_per_step", "sweeps", "pcg_iters",
                                         "newton_iters", "minres_iters", "step_sweeps")}
            # the converged end state against omega's: the same crack?
            a1, a0 = st_om[1], state64[1]
            o_om["final_energy"] = {"elastic": e_om[0], "surface": e_om[1]}
            o_om["rel_surface_energy_vs_omega"] = abs(e_om[1] - energy64[1]) / abs(energy64[1])
            o_om["iou_crack_vs_omega"] = float(np.sum((a1 > 0.5) & (a0 > 0.5)) /
                                               max(np.sum((a1 > 0.5) | (a0 > 0.5)), 1))
            out["omega_sweep"][f"{om:g}"] = o_om
    if not args.no_mixed and args.precision == "fp64":
        if res["seconds"] > args.mixed_budget:
            out["mixed"] = {"skipped": f"the FP64 leg took {res['seconds']:.0f} s > --mixed-budget "
                                       f"{args.mixed_budget:g} s"}
        else:
            # the same load steps with the float32 operator and multigrid inside
            # float64 refinement, against the float64 run just made
            s32, r32, (state32, snap32), energy32 = leg("mixed")
            s32.close()
            rel = lambda a_, b_: float(np.linalg.norm(a_ - b_) / max(np.linalg.norm(b_), 1e-300))
            out["mixed"] = {
                "value": r32["value"], "unit": "load steps/s", "ms_per_step": r32["ms_per_step"],
                "pcg_dof_iter_per_s": r32["pcg_dof_iter_per_s"], "pcg_iters": r32["pcg_iters"],
                "sweeps": r32["sweeps"], "step_sweeps": r32["step_sweeps"],
                "minres_iters": r32["minres_iters"], "speedup_vs_fp64": r32["value"] / res["value"],
                "p50_step_ms": r32["p50_step_ms"], "p99_step_ms": r32["p99_step_ms"],
                "rel_l2_u_vs_fp64": rel(state32[0], state64[0]),
                "rel_l2_alpha_vs_fp64": rel(state32[1], state64[1]),
                "rel_energy_vs_fp64": abs(sum(energy32) - sum(energy64)) / abs(sum(energy64)),
                "rel_surface_energy_vs_fp64": abs(energy32[1] - energy64[1]) / abs(energy64[1]),
                "iou_crack_vs_fp64": float(np.sum((state32[1] > 0.5) & (state64[1] > 0.5))
                                           / max(np.sum((state32[1] > 0.5) | (state64[1] > 0.5)), 1)),
            }
            if snap32 is not None and snap64 is not None:
                # before initiation the two runs track one solution branch; at
                # initiation each may select a different one (the crack path is a
                # bifurcation), so the distance after it is not a rounding measure
                out["mixed"][f"rel_l2_u_vs_fp64_t{loads[args.snap_step - 1]:.1f}"] = rel(snap32[0], snap64[0])
                out["mixed"][f"rel_l2_alpha_vs_fp64_t{loads[args.snap_step - 1]:.1f}"] = rel(snap32[1],
                                                                                          snap64[1])
    if args.with_serve:
        sv = serve(args)
        out["serving"] = {k: sv[k] for k in ("instances", "steps", "wall_s", "steps_per_s",
                                             "instances_per_s", "p50_ms", "p99_ms",
                                             "failed_steps", "peak_used_bytes")}
        out["serving"]["workload"] = (f"first {args.instances} requests of the seeded config-5 stream "
                                      f"(n in 64..1024, ell in [0.01,0.05], h=ell/4, 10-30 steps, "
                                      f"Poisson 50/s), mixed precision, budget {args.budget_gb} GB, "
                                      f"{args.workers} workers, {args.hw_queues} hardware queues")
    if args.with_surfing:
        # the surfing slab at ell = 1/64, ORAM-N with the automatic
        # over-relaxation factor (cap 1.9)
        sargs = argparse.Namespace(**vars(args))
        sargs.surf_ell, sargs.omega, sargs.precision, sargs.newton = 1.0 / 64, 1.9, "fp64", 1
        sargs.omega_auto = True
        sargs.forcing_mode = 0
        sargs.max_am = 5000
        out["surfing"] = surfing(sargs)
    if args.with_tshock:
        # the 2D thermal shock at DT = 4 DT_c, plain ORAM at omega = 1 and at
        # the paper's best over-relaxation 1.6
        out["tshock"] = tshock(args, ratios=(4.0,), omegas=(1.0, 1.6))
    if args.with_deflation:
        out["deflation"] = deflation(args)
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline (oracle, {args.cpu_n}^2, load steps 1..{args.steps}) ...")
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, args.steps, args.model)
        log(f"[bench] cpu baseline {out['cpu_baseline']['seconds']:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
