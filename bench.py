"""Throughput of the DGSEM right-hand side on one MI355X.

Workload (default): the 3D compressible Navier-Stokes Taylor-Green vortex,
Mach 0.1, Re 1600, Pr 0.72, 32^3 periodic hexahedra, N = 3 (2,097,152 nodes,
10,485,760 DOF), FP64; entropy-conservative flux differencing, Rusanov
faces, BR1 viscous terms.  A step is one SSPRK3 step (three right-hand-side
evaluations fused with the stage updates, replayed from a HIP graph), so

    GDOF-RHS/s = 3 * DOF * steps / seconds / 1e9.

The headline is the median of 5 timed runs of --steps steps each.  Prints
one JSON line (see the keys below).  The oracle (NumPy) is timed on the same
32^3 state for the cpu_baseline entry, on one core and on all usable cores.
"""
import argparse
import hashlib
import json
import math

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDOF-RHS/s (FP64, N=3/4) on 1 MI355X; thermo time, surrogate vs plain Newton"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def rhs_bytes_per_launch(nelem, nn, nvar, dim, n1, stage_base=True):
    """Algorithmic HBM bytes of one fused k_rhs launch (every datum once).

    per node: state u (nvar) and stage base u0 (nvar, stages 2 and 3) read,
    next stage (nvar) written, element-local viscous divergence (dim+1) read;
    per element: the neighbours' face viscous fluxes (2 dim faces x (dim+1) x
    n1^(dim-1) face nodes), dim*dim+1 affine geometry doubles and 2*dim int32
    neighbour indices.
    """
    nf = n1 ** (dim - 1)
    per_node = nvar + (nvar if stage_base else 0) + nvar + (dim + 1)
    per_elem = 2 * dim * (dim + 1) * nf * 8 + (dim * dim + 1) * 8 + 2 * dim * 4
    return nelem * nn * per_node * 8 + nelem * per_elem


def grad_bytes_per_launch(nelem, nn, nvar, dim, n1):
    """k_grad: state read; local viscous divergence and face fluxes written."""
    nf = n1 ** (dim - 1)
    return nelem * nn * (nvar + dim + 1) * 8 + nelem * (2 * dim * (dim + 1) * nf * 8 + (dim * dim + 1) * 8 + 2 * dim * 4)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rhs_worker(n, reps, barrier, out):
    """One process of the all-cores leg: builds the oracle for the n^3 TGV
    state, waits for every process to be ready, then times `reps` right-hand
    sides single-threaded and puts the seconds into `out`."""
    from threadpoolctl import threadpool_limits
    from paper_2511_17551_amd import workloads as W
    from oracle.dgsem import Operator
    case = W.case_c2(n=n)
    with threadpool_limits(limits=1):
        op = Operator(case.cfg, case.mesh)
        barrier.wait()
        t0 = time.perf_counter()
        for _ in range(reps):
            op.rhs(case.u0)
        out.put(time.perf_counter() - t0)


def cpu_baseline(n=32, budget_s=10.0, max_procs=16):
    """The oracle (NumPy FP64) on the headline state, timed on this host's
    cores before the GPU is touched: one process on one thread (right-hand
    sides until ~budget_s), then one single-threaded process per usable core
    (at most max_procs, the host share of one GPU), each evaluating one full
    right-hand side of its own copy of the state, wall time of the slowest.
    Returns the all-cores throughput as the value, the one-core figure beside
    it, the core counts and the CPU model."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from paper_2511_17551_amd import workloads as W
    from oracle.dgsem import Operator
    case = W.case_c2(n=n)
    dof = case.u0.size
    with threadpool_limits(limits=1):
        op = Operator(case.cfg, case.mesh)
        t0 = time.perf_counter()
        k = 0
        while True:
            op.rhs(case.u0)
            k += 1
            el1 = time.perf_counter() - t0
            if el1 > budget_s or k >= 10:
                break
    del op
    one = dof * k / el1 / 1e9
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    procs = max(1, min(usable, max_procs))
    ctx = mp.get_context("fork")   # the GPU is not initialised yet: plain fork, no exec
    barrier, q = ctx.Barrier(procs), ctx.Queue()
    ps = [ctx.Process(target=_oracle_rhs_worker, args=(n, 1, barrier, q)) for _ in range(procs)]
    for p in ps:
        p.start()
    secs = [q.get() for _ in ps]
    for p in ps:
        p.join()
    elp = max(secs)   # all processes ran concurrently from the barrier on
    allc = dof * procs / elp / 1e9
    return dict(value=allc, unit="GDOF-RHS/s", cores=procs, kind="oracle",
                one_core=dict(value=one, unit="GDOF-RHS/s", cores=1, rhs=k, seconds=round(el1, 2)),
                nproc=os.cpu_count(), usable_cores=usable, cpu_model=_cpu_model(),
                sample="the %d^3 N=3 Navier-Stokes TGV state (%d DOF), NumPy FP64: one thread, "
                       "%d right-hand sides in %.1f s; then %d single-threaded processes started together, "
                       "one right-hand side each, the slowest %.1f s" % (n, dof, k, el1, procs, elp))


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "k_rhs_traffic.json")


def kernel_source_hash():
    """SHA-1 of the code the right-hand-side kernel is compiled from: its
    sources with // comments, trailing blanks and empty lines removed (a
    comment edit does not make the recorded traffic stale)."""
    h = hashlib.sha1()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2511_17551_amd", "csrc")
    for f in ("k_rhs.h", "physics.h", "dgx_internal.h"):
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode("utf-8") + b"\n")
    return h.hexdigest()


ORDER_NAMES = {0: "round_robin", 1: "xcd_contiguous", 2: "work_list",
               4: "round_robin+alt_tiling", 5: "xcd_contiguous+alt_tiling", 6: "work_list+alt_tiling"}


def recorded_traffic(workload, order, epb=None):
    """HBM bytes per k_rhs launch (FETCH_SIZE + WRITE_SIZE per dispatch, each
    divided by its copy-kernel calibration factor) of this workload under this
    workgroup numbering and elements per workgroup, from the committed
    counter summary; None when no record matches or it was taken on other
    kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        recs = json.load(fh).get("records", [])
    sha = kernel_source_hash()
    for rec in recs:
        if rec.get("workload") == workload and rec.get("order") == ORDER_NAMES[order] \
                and rec.get("source_sha1") == sha \
                and (epb is None or rec.get("elements_per_workgroup") == epb):
            return float(rec["traffic_bytes_per_launch"])
    return None


def thermo_leg(torch, W, dgx, snapshots=16, steps_per_snap=20, epochs=16, reps=5):
    """Per-node T(e): surrogate-guided vs plain Newton on solver-generated states.

    States: a reacting run of the impulsively started Mach-8 cylinder O-grid
    (64 x 128, N = 3, positivity limiter, CFL 0.2), each step Strang-split
    (chemistry over dt/2, one frozen-mixture SSPRK3 step, chemistry over
    dt/2), snapshots every 20 steps -> 16 x 131072 = 2,097,152 states.
    Labels: the plain solve's converged T.  The chemistry call is timed on
    the run's last state (its dt/2) and on the hot, partly dissociated
    cylinder state (same mesh, dt = 1e-9 s).
    The surrogate is trained on the same set (Adam, batch 4096), then both
    solves are timed (HIP events, same stream, same 1e-10 tolerance).
    """
    probe = W.case_c4(lambda rs, T: 0 * T, lambda rs, T: 1 + 0 * T, nr=4, nth=8)
    pctx = dgx.dgx_create(probe.cfg, probe.species, probe.reactions)
    energy, cv = dgx.mixture_energy_fns(pctx)
    c = W.case_c4(energy, cv)
    hot = W.case_c4(energy, cv, hot=True)
    dgx.dgx_destroy(pctx)   # the energy functions use it: only after the cases are built
    c.cfg["eq"] = W.EQ_EULER_MIX
    s = dgx.Solver(c)
    u = torch.from_numpy(c.u0).to("cuda")
    dt = dgx.dgx_max_dt(s.ctx, u, 0.2)
    snaps = []
    for _ in range(snapshots):
        for _ in range(steps_per_snap):
            dgx.dgx_chem_step(s.ctx, u, 0.5 * dt, stats=False)
            s.ssprk3(u, dt, 1)
            dgx.dgx_chem_step(s.ctx, u, 0.5 * dt, stats=False)
        snaps.append(u.reshape(u.shape[0], -1).clone())
    s.check()
    e0, e1 = _events(torch)

    def time_chem(ctx, src, cdt):
        """Chemistry over cdt on fresh copies of src: (stats, ms)."""
        uc = src.clone()
        st = dgx.dgx_chem_step(ctx, uc, cdt)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            uc.copy_(src)
            dgx.dgx_chem_step(ctx, uc, cdt, stats=False)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        e0.record()
        for _ in range(reps):
            uc.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        return st, ms - e0.elapsed_time(e1) / reps

    def chem_summary(st, cdt, ms):
        return dict(nodes=int(st["nodes"]), dt=cdt, ms=round(ms, 4),
                    iters_mean=round(st["iters_total"] / st["nodes"], 3), iters_max=int(st["iters_max"]),
                    wave_max_mean=round(st["iters_wave_max_mean"], 3),
                    substeps_max=int(st["substeps_max"]),
                    extra_substeps=int(st["substeps_total"] - st["nodes"]))

    run_st, run_ms = time_chem(s.ctx, u, 0.5 * dt)
    s.check()
    # the chemistry step on the hot cylinder state
    hot.cfg["eq"] = W.EQ_EULER_MIX
    sh = dgx.Solver(hot)
    uh = torch.from_numpy(hot.u0).to("cuda")
    chem_dt = 1e-9
    chem_stats, chem_ms = time_chem(sh.ctx, uh, chem_dt)
    sh.check()
    sh.close()
    del uh
    states = torch.cat(snaps, 1).contiguous()
    del snaps
    n = states.shape[1]
    T = torch.empty(n, dtype=torch.float64, device="cuda")
    st_plain = dgx.dgx_thermo(s.ctx, states, T, nstates=n)
    t0 = time.perf_counter()
    dgx.dgx_surrogate_init(s.ctx, states, T, seed=41)
    losses = dgx.dgx_surrogate_train(s.ctx, states, T, epochs=epochs, batch=4096, lr=2e-3, seed=42)
    train_s = time.perf_counter() - t0
    Ts = torch.empty_like(T)
    st_sur = dgx.dgx_thermo(s.ctx, states, Ts, nstates=n, guess=dgx.GUESS_SURROGATE)
    # relative agreement of the converged temperatures, over states above 1 K:
    # in the near-vacuum wake of the impulsive start the positivity limiter
    # leaves thermal energies at the rounding level of the formation
    # energies (T ~ 1e-11 K), where T is determined only to that level
    phys = T > 1.0
    maxrel = float(((Ts - T).abs() / T)[phys].max())
    near_vacuum = int((~phys).sum())
    Tg = torch.empty_like(T)
    res = {}
    for name, guess in (("plain", dgx.GUESS_FREESTREAM), ("surrogate", dgx.GUESS_SURROGATE)):
        dgx.dgx_thermo(s.ctx, states, Ts, nstates=n, guess=guess, stats=False)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            dgx.dgx_thermo(s.ctx, states, Ts, nstates=n, guess=guess, stats=False)
        e1.record()
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / reps
    dgx.dgx_surrogate_predict(s.ctx, states, Tg)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dgx.dgx_surrogate_predict(s.ctx, states, Tg)
    e1.record()
    torch.cuda.synchronize()
    infer_ms = e0.elapsed_time(e1) / reps
    guess_err = float(((Tg - T).abs() / T).median())
    # the disturbed states only (|T - T_inf| > 1% T_inf): shock layer and wake
    sel = ((T - c.cfg["T_guess"]).abs() > 0.01 * c.cfg["T_guess"]).nonzero().flatten()
    sub = states[:, sel].contiguous()
    nsub = sub.shape[1]
    Tsub = torch.empty(nsub, dtype=torch.float64, device="cuda")
    sp_sub = dgx.dgx_thermo(s.ctx, sub, Tsub, nstates=nsub)
    ss_sub = dgx.dgx_thermo(s.ctx, sub, Tsub, nstates=nsub, guess=dgx.GUESS_SURROGATE)
    sub_ms = {}
    for name, guess in (("plain", dgx.GUESS_FREESTREAM), ("surrogate", dgx.GUESS_SURROGATE)):
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            dgx.dgx_thermo(s.ctx, sub, Tsub, nstates=nsub, guess=guess, stats=False)
        e1.record()
        torch.cuda.synchronize()
        sub_ms[name] = e0.elapsed_time(e1) / reps
    s.check()
    s.close()
    return dict(states=n, T_min=float(T.min()), T_max=float(T.max()),
                plain_ms=round(res["plain"], 4), surrogate_ms=round(res["surrogate"], 4),
                speedup=round(res["plain"] / res["surrogate"], 3), surrogate_inference_ms=round(infer_ms, 4),
                iters_mean_plain=round(st_plain["iters_total"] / n, 3),
                iters_mean_surrogate=round(st_sur["iters_total"] / n, 3),
                wave_max_mean_plain=round(st_plain["iters_wave_max_mean"], 3),
                wave_max_mean_surrogate=round(st_sur["iters_wave_max_mean"], 3),
                max_rel_T_diff=maxrel, near_vacuum_states=near_vacuum, median_rel_guess_err=guess_err,
                disturbed=dict(states=int(nsub), plain_ms=round(sub_ms["plain"], 4),
                               surrogate_ms=round(sub_ms["surrogate"], 4),
                               speedup=round(sub_ms["plain"] / sub_ms["surrogate"], 3),
                               iters_mean_plain=round(sp_sub["iters_total"] / nsub, 3),
                               iters_mean_surrogate=round(ss_sub["iters_total"] / nsub, 3),
                               wave_max_mean_plain=round(sp_sub["iters_wave_max_mean"], 3),
                               wave_max_mean_surrogate=round(ss_sub["iters_wave_max_mean"], 3)),
                train_epochs=epochs, train_s=round(train_s, 2), loss_first=float(losses[0]),
                loss_last=float(losses[-1]), tol=1e-10,
                chemistry=dict(hot_state=chem_summary(chem_stats, chem_dt, chem_ms),
                               reacting_run=chem_summary(run_st, 0.5 * dt, run_ms),
                               strang_steps=snapshots * steps_per_snap))


def c3_bytes_per_launch(nelem, nn, nvar, dim, stage_base=True):
    """Algorithmic HBM bytes of one fused k_rhs launch on curved mixture
    elements: per node the state (nvar) and its temperature read, the stage
    base u0 (nvar) read, the next stage (nvar) written, the nodal metric terms
    Ja (dim x dim) and J read; per element the blending factor and 2*dim int32
    neighbour indices.  (Subcell normals, read by shocked elements only, are
    not counted.)"""
    per_node = nvar + 1 + (nvar if stage_base else 0) + nvar + dim * dim + 1
    return nelem * nn * per_node * 8 + nelem * (8 + 2 * dim * 4)


def c3_leg(torch, W, dgx, reps=20, order=-1, epb=0):
    """The curvilinear 24^3 N = 4 frozen 5-species Mach-3 shock case:
    back-to-back right-hand sides on the shock state (each: T(e) Newton per
    node, modal indicator, fused RHS with subcell FV in the shocked elements),
    GDOF-RHS/s and the k_rhs roofline of its stage-form launch."""
    probe = W.case_c4(lambda rs, T: 0 * T, lambda rs, T: 1 + 0 * T, nr=4, nth=8)
    pctx = dgx.dgx_create(probe.cfg, probe.species, probe.reactions)
    energy, cv = dgx.mixture_energy_fns(pctx)
    c = W.case_c3(energy, cv)
    dgx.dgx_destroy(pctx)   # the energy functions use it: only after the case is built
    nvar, nelem, nn = c.u0.shape
    s = dgx.Solver(c)
    u = torch.from_numpy(c.u0).to("cuda")
    du = torch.empty_like(u)
    if epb > 0:
        dgx.dgx_set_launch(s.ctx, epb)   # fixed launch shape (profiling runs)
    else:
        epb, tune = dgx.dgx_autotune(s.ctx, u, reps=5)
    if order >= 0:
        dgx.dgx_set_launch(s.ctx, epb, order)
    _, used_order = dgx.dgx_get_launch(s.ctx)
    for _ in range(2):
        dgx.dgx_rhs(s.ctx, u, 0.0, du)
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record()
    for _ in range(reps):
        dgx.dgx_rhs(s.ctx, u, 0.0, du)
    e1.record()
    torch.cuda.synchronize()
    s.check()
    ms_rhs = e0.elapsed_time(e1) / reps
    alpha = dgx.dgx_last_alpha(s.ctx, nelem)
    shocked = int((alpha > 0).sum()) if alpha is not None else 0
    kt = dgx.dgx_kernel_times(s.ctx, u, reps=10)
    s.close()
    rb = c3_bytes_per_launch(nelem, nn, nvar, 3)
    k_ms = kt["k_rhs"]
    achieved = rb / (k_ms * 1e-3) / 1e9
    return dict(workload="curved24_N4_air5_mach3_shock_rhs", elements=nelem, N=4, nodes=nelem * nn,
                dof=int(c.u0.size), value=round(c.u0.size / (ms_rhs * 1e-3) / 1e9, 3),
                unit="GDOF-RHS/s", ms_per_rhs=round(ms_rhs, 5), elements_per_workgroup=epb,
                workgroup_order=ORDER_NAMES[used_order], shocked_elements=shocked, kernel_ms={k: round(v, 5) for k, v in kt.items()},
                roofline=dict(bound="hbm", kernel="k_rhs", achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                              unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4), bytes_per_launch=rb,
                              traffic=recorded_traffic("curved24_N4_air5_mach3_shock", used_order, epb)))


def euler_bytes_per_launch(nelem, nn, nvar):
    """Algorithmic HBM bytes of one fused k_rhs launch for the perfect-gas
    Euler equations on affine elements: per node u, u0 read and the next stage
    written; per element the affine geometry and 2*dim int32 neighbours."""
    return nelem * nn * 3 * nvar * 8 + nelem * (10 * 8 + 6 * 4)


def flux_leg(torch, W, dgx, reps=20):
    """The 32^3 N=3 Taylor-Green state under the 3D Euler equations with each
    built volume / surface flux pair: back-to-back right-hand sides and the
    k_rhs time of its stage-form launch (HIP events)."""
    variants = [("ranocha_rusanov", W.VF_RANOCHA, W.SF_RUSANOV),
                ("kennedy_gruber_rusanov", W.VF_KENNEDY_GRUBER, W.SF_RUSANOV),
                ("pirozzoli_rusanov", W.VF_PIROZZOLI, W.SF_RUSANOV),
                ("central_rusanov", W.VF_CENTRAL, W.SF_RUSANOV),
                ("ranocha_hll", W.VF_RANOCHA, W.SF_HLL),
                ("ranocha_hllc", W.VF_RANOCHA, W.SF_HLLC)]
    out = {}
    for name, vf, sf in variants:
        c = W.case_c2(eq=W.EQ_EULER)
        c.cfg = dict(c.cfg, volume_flux=vf, surface_flux=sf)
        nvar, nelem, nn = c.u0.shape
        s = dgx.Solver(c)
        u = torch.from_numpy(c.u0).to("cuda")
        du = torch.empty_like(u)
        epb, _ = dgx.dgx_autotune(s.ctx, u, reps=5)
        for _ in range(2):
            dgx.dgx_rhs(s.ctx, u, 0.0, du)
        torch.cuda.synchronize()
        e0, e1 = _events(torch)
        e0.record()
        for _ in range(reps):
            dgx.dgx_rhs(s.ctx, u, 0.0, du)
        e1.record()
        torch.cuda.synchronize()
        s.check()
        ms = e0.elapsed_time(e1) / reps
        kt = dgx.dgx_kernel_times(s.ctx, u, reps=10)
        s.close()
        rb = euler_bytes_per_launch(nelem, nn, nvar)
        out[name] = dict(value=round(c.u0.size / (ms * 1e-3) / 1e9, 3), unit="GDOF-RHS/s", ms_per_rhs=round(ms, 5),
                         k_rhs_ms=round(kt["k_rhs"], 5), elements_per_workgroup=epb,
                         roofline_frac=round(rb / (kt["k_rhs"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
    return dict(workload="tgv3d_euler_32cube_N3_rhs", bytes_per_launch=euler_bytes_per_launch(32768, 64, 5),
                variants=out)


def _rhs_rate(torch, dgx, case, reps=10, tune_reps=3):
    """Autotuned back-to-back right-hand sides of a case: (GDOF-RHS/s,
    ms per RHS, per-kernel ms, elements per workgroup)."""
    s = dgx.Solver(case)
    u = torch.from_numpy(case.u0).to("cuda")
    du = torch.empty_like(u)
    epb, _ = dgx.dgx_autotune(s.ctx, u, reps=tune_reps)
    for _ in range(2):
        dgx.dgx_rhs(s.ctx, u, 0.0, du)
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record()
    for _ in range(reps):
        dgx.dgx_rhs(s.ctx, u, 0.0, du)
    e1.record()
    torch.cuda.synchronize()
    s.check()
    ms = e0.elapsed_time(e1) / reps
    kt = dgx.dgx_kernel_times(s.ctx, u, reps=5)
    s.close()
    return round(case.u0.size / (ms * 1e-3) / 1e9, 3), round(ms, 5), {k: round(v, 5) for k, v in kt.items()}, epb


def mixture_flux_leg(torch, W, dgx):
    """The curved 24^3 N = 4 5-species shock with every volume / surface flux
    built for the mixture: right-hand-side throughput and the k_rhs roofline
    fraction (the c3 leg's algorithmic bytes)."""
    probe = W.case_c4(lambda rs, T: 0 * T, lambda rs, T: 1 + 0 * T, nr=4, nth=8)
    pctx = dgx.dgx_create(probe.cfg, probe.species, probe.reactions)
    energy, cv = dgx.mixture_energy_fns(pctx)
    base = W.case_c3(energy, cv)
    dgx.dgx_destroy(pctx)
    nvar, nelem, nn = base.u0.shape
    rb = c3_bytes_per_launch(nelem, nn, nvar, 3)
    out = {}
    for name, vf, sf in (("kennedy_gruber_rusanov", W.VF_KENNEDY_GRUBER, W.SF_RUSANOV),
                         ("pirozzoli_rusanov", W.VF_PIROZZOLI, W.SF_RUSANOV),
                         ("central_rusanov", W.VF_CENTRAL, W.SF_RUSANOV),
                         ("entropy_conservative_rusanov", W.VF_RANOCHA, W.SF_RUSANOV),
                         ("ducros_hll", W.VF_DUCROS, W.SF_HLL),
                         ("ducros_hllc", W.VF_DUCROS, W.SF_HLLC)):
        c = W.Case(base.name, dict(base.cfg, volume_flux=vf, surface_flux=sf), base.mesh, base.u0,
                   species=base.species)
        v, ms, kt, epb = _rhs_rate(torch, dgx, c)
        out[name] = dict(value=v, unit="GDOF-RHS/s", ms_per_rhs=ms, kernel_ms=kt, elements_per_workgroup=epb,
                         roofline_frac=round(rb / (kt["k_rhs"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
    return dict(workload="curved24_N4_air5_mach3_shock_rhs", bytes_per_launch=rb, variants=out)


def ns_leg(torch, W, dgx):
    """Navier-Stokes beyond the periodic affine TGV: the curved periodic 24^3
    mesh at N = 3 and 4, and the wall channel on the 2:1 octree mesh (16^3
    base, one level inside r = 0.3, isothermal walls, viscous mortars).
    Right-hand-side throughput; for the curved kernels the k_rhs roofline
    fraction on per node u 5 + u0 5 + out 5 + local viscous part 4 +
    nodal metric terms 10 doubles."""
    out = {}
    for name, make in (("curved_periodic_24cube_N3", lambda: W.curved_periodic_case(n=24, N=3, eq=W.EQ_NS, mu=1e-3)),
                       ("curved_periodic_24cube_N4", lambda: W.curved_periodic_case(n=24, N=4, eq=W.EQ_NS, mu=1e-3)),
                       ("wall_channel_octree16", lambda: W.wall_channel_case(N=3, base=16, radii=(0.3,), T_hi=1.6,
                                                                             mu=1e-3))):
        c = make()
        nvar, nelem, nn = c.u0.shape
        v, ms, kt, epb = _rhs_rate(torch, dgx, c)
        rec = dict(value=v, unit="GDOF-RHS/s", ms_per_rhs=ms, kernel_ms=kt, elements=nelem,
                   mortars=int(len(c.mesh.mortars)), boundary_faces=int(len(c.mesh.bfaces)), elements_per_workgroup=epb)
        if name.startswith("curved"):
            rb = nelem * nn * 29 * 8
            rec["roofline_frac"] = round(rb / (kt["k_rhs"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        out[name] = rec
    return out


def amr_leg(torch, W, dgx, cycles=3, steps=10):
    """Dynamic AMR: a Gaussian density pulse (width 0.1) carried across the
    periodic unit cube on an octree of 16^3 level-0 cells, levels 0-2
    (Loehner's estimate of the density, thresholds 0.01 / 0.03: at this
    resolution the pulse's estimate peaks near 0.045).  Per cycle: the indicator (GPU), the
    plan (host), the transfer and mesh upload, then `steps` SSPRK3 steps;
    the right-hand-side throughput on the final mesh."""
    import time as _t
    base = 16
    leaves = np.array([(0, i, j, k) for k in range(base) for j in range(base) for i in range(base)], np.int32)
    c0 = W.case_amr(base=4, radii=(0.4,), centre=(0.5, 0.5, 0.5))
    s = dgx.Solver(c0)
    order = s.set_octree(base, leaves)
    N = 3
    xi = W._mesh_nodes(N)

    def coords(order):
        n1 = N + 1
        node = np.arange(n1 ** 3)
        idx = [node % n1, (node // n1) % n1, node // (n1 * n1)]
        x = np.empty((3, len(order), n1 ** 3))
        for e, (L, i, j, k) in enumerate(order):
            h = 1.0 / (base * 2 ** L)
            for d, cc in enumerate((i, j, k)):
                x[d, e] = h * (cc + 0.5 * (xi[idx[d]] + 1.0))
        return x
    u = torch.from_numpy(W.blob_state(coords(order))).to("cuda")
    ctrl = dict(base_level=0, med_level=1, max_level=2, med_threshold=0.01, max_threshold=0.03)
    recs = []
    for cyc in range(cycles):
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        ind = s.amr_indicator(u, 0, 0)
        torch.cuda.synchronize()
        t1 = _t.perf_counter()
        ind_h = ind.cpu().numpy()
        n_new = dgx.dgx_amr_plan(s.ctx, ind_h, ctrl)
        t2 = _t.perf_counter()
        un = torch.empty((u.shape[0], n_new, u.shape[2]), dtype=u.dtype, device=u.device)
        dgx.dgx_amr_apply(s.ctx, u, un)
        torch.cuda.synchronize()
        t3 = _t.perf_counter()
        u = un
        dt = dgx.dgx_max_dt(s.ctx, u, 0.5)
        s.ssprk3(u, dt, steps)
        torch.cuda.synchronize()
        s.check()
        lv = np.bincount(s.octree()[:, 0], minlength=3)
        recs.append(dict(elements=int(n_new), levels=[int(v) for v in lv], indicator_ms=round((t1 - t0) * 1e3, 3),
                         plan_ms=round((t2 - t1) * 1e3, 3), transfer_and_mesh_ms=round((t3 - t2) * 1e3, 3)))
    du = torch.empty_like(u)
    e0, e1 = _events(torch)
    for _ in range(2):
        dgx.dgx_rhs(s.ctx, u, 0.0, du)
    e0.record()
    for _ in range(10):
        dgx.dgx_rhs(s.ctx, u, 0.0, du)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    s.close()
    return dict(workload="octree16_blob_loehner_levels0-2_thresholds0.01-0.03", cycles=recs, final_elements=int(u.shape[1]),
                rhs_GDOF_RHS_s=round(u.numel() / (ms * 1e-3) / 1e9, 3), ms_per_rhs=round(ms, 5))


def c4_leg(torch, W, dgx, reps=20):
    """The 2D reacting 5-species cylinder (64 x 128 O-grid, N = 3, 17
    Arrhenius reactions): back-to-back right-hand sides on the hot, partly
    dissociated state (each: T(e) Newton per node, modal indicator, fused RHS
    with the species sources)."""
    probe = W.case_c4(lambda rs, T: 0 * T, lambda rs, T: 1 + 0 * T, nr=4, nth=8)
    pctx = dgx.dgx_create(probe.cfg, probe.species, probe.reactions)
    energy, cv = dgx.mixture_energy_fns(pctx)
    c = W.case_c4(energy, cv, hot=True)
    dgx.dgx_destroy(pctx)   # the energy functions use it: only after the case is built
    nvar, nelem, nn = c.u0.shape
    s = dgx.Solver(c)
    u = torch.from_numpy(c.u0).to("cuda")
    du = torch.empty_like(u)
    epb, _ = dgx.dgx_autotune(s.ctx, u, reps=5)
    for _ in range(2):
        dgx.dgx_rhs(s.ctx, u, 0.0, du)
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record()
    for _ in range(reps):
        dgx.dgx_rhs(s.ctx, u, 0.0, du)
    e1.record()
    torch.cuda.synchronize()
    s.check()
    ms_rhs = e0.elapsed_time(e1) / reps
    kt = dgx.dgx_kernel_times(s.ctx, u, reps=10)
    s.close()
    return dict(workload="cylinder64x128_N3_air5_17reactions_hot_rhs", elements=nelem, N=3, nodes=nelem * nn,
                dof=int(c.u0.size), value=round(c.u0.size / (ms_rhs * 1e-3) / 1e9, 3), unit="GDOF-RHS/s",
                ms_per_rhs=round(ms_rhs, 5), elements_per_workgroup=epb,
                kernel_ms={k: round(v, 5) for k, v in kt.items()})


def batch_leg(torch, W, dgx, reps=10):
    """The AMR density wave + 16 vortex-tube cases: one launch per stage for
    everything vs one context / launch sequence per case."""
    c = W.case_c5()
    s = dgx.Solver(c)
    u = torch.from_numpy(c.u0).to("cuda")
    dt = dgx.dgx_max_dt(s.ctx, u, 0.3)
    epb, _ = dgx.dgx_autotune(s.ctx, u, reps=5)
    _, form = dgx.dgx_get_launch(s.ctx)
    s.ssprk3(u, dt, 3)
    e0, e1 = _events(torch)
    # the median of three repeats of 30 steps
    rep_ms = []
    for _ in range(3):
        torch.cuda.synchronize()
        e0.record()
        s.ssprk3(u, dt, 30)
        e1.record()
        torch.cuda.synchronize()
        rep_ms.append(e0.elapsed_time(e1) / 30)
    ms_batched = float(np.median(rep_ms))
    s.check()
    s.close()
    dof = c.u0.size
    offs = c.mesh.case_offsets
    amr = W.case_amr()
    cases = [amr]
    for n in c.extra["sizes"]:
        x, faces, u0 = W.vortex_tube_case(n)
        m = W.Mesh(3, 3, x, faces, np.zeros((0, 3), np.int32), np.zeros((0, 7), np.int32),
                   np.zeros(0, np.int32), np.zeros((0, 5)))
        cases.append(W.Case("tube", W.base_cfg(3, 3, W.EQ_EULER), m, u0))
    solvers, states = [], []
    for cc in cases:
        sc = dgx.Solver(cc)
        uc = torch.from_numpy(cc.u0).to("cuda")
        dgx.dgx_set_launch(sc.ctx, epb) if epb * 64 <= 512 else None
        sc.ssprk3(uc, dt, 2)
        solvers.append(sc)
        states.append(uc)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        for sc, uc in zip(solvers, states):
            sc.ssprk3(uc, dt, 1)
    e1.record()
    torch.cuda.synchronize()
    ms_sep = e0.elapsed_time(e1) / reps
    for sc in solvers:
        sc.check()
        sc.close()
    return dict(elements=int(c.mesh.nelem), amr_elements=int(c.extra["amr_elements"]),
                mortars=int(len(c.mesh.mortars)), cases=len(offs) - 1, dof=int(dof),
                batched_ms_per_step=round(ms_batched, 4), batched_repeat_ms=[round(r, 4) for r in rep_ms],
                separate_ms_per_step=round(ms_sep, 4),
                batched_GDOF_RHS_s=round(3 * dof / (ms_batched * 1e-3) / 1e9, 3),
                separate_GDOF_RHS_s=round(3 * dof / (ms_sep * 1e-3) / 1e9, 3),
                elements_per_workgroup=epb, launch_form=ORDER_NAMES[form])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs of --steps steps each (at least this many, more when --steps is "
                         "small: enough that all repeats together last about 0.5 s, at most 50); the "
                         "median is reported")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the mixture legs (curved N=4 shock, reacting cylinder)")
    ap.add_argument("--no-thermo", action="store_true", help="skip the surrogate vs plain T(e) leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched AMR + cases leg")
    ap.add_argument("--no-fluxes", action="store_true",
                    help="skip the leg that times each built volume / surface flux on the TGV (Euler)")
    ap.add_argument("--no-widened", action="store_true",
                    help="skip the legs of the mixture flux variants, Navier-Stokes on curved / wall / "
                         "mortar meshes and dynamic AMR")
    ap.add_argument("--epb", type=int, default=0,
                    help="elements per workgroup to use instead of autotuning (profiling runs)")
    ap.add_argument("--c3-epb", type=int, default=0,
                    help="elements per workgroup of the curved-shock leg instead of autotuning (profiling runs)")
    ap.add_argument("--order", type=int, default=-1, choices=(-1, 0, 1, 2, 4, 5, 6),
                    help="launch form of the headline and curved-shock legs instead of the autotuner's "
                         "(0 round-robin over the XCDs, 1 XCD-contiguous, 2 work-list queue; +4 the "
                         "alternative LDS tiling; profiling runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB read + 1 GiB write kernel (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X; how the "
              "path would shard across GPUs is described, not implemented", file=sys.stderr)
        sys.exit(2)

    # the oracle on the host cores first, while no process has touched the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline()

    import torch
    from paper_2511_17551_amd import workloads as W
    from paper_2511_17551_amd import dgx

    case = W.case_c2()
    nvar, nelem, nn = case.u0.shape
    dof = case.u0.size
    solver = dgx.Solver(case)
    u = torch.from_numpy(case.u0).to("cuda")
    dt = dgx.dgx_max_dt(solver.ctx, u, 0.5)
    if args.epb > 0:
        dgx.dgx_set_launch(solver.ctx, args.epb)
        epb, tune_ms = args.epb, {}
    else:
        epb, tune_ms = dgx.dgx_autotune(solver.ctx, u, reps=20)
    if args.order >= 0:
        dgx.dgx_set_launch(solver.ctx, epb, args.order)
    _, order = dgx.dgx_get_launch(solver.ctx)
    if args.copy_probe:
        # counter calibration: kernels of known traffic on 1 GiB buffers
        # (larger than the 256 MB Infinity Cache)
        cx = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        cy = torch.empty_like(cx)
        for _ in range(3):
            torch.mul(cx, 1.0, out=cy)   # elementwise kernel
            cy.copy_(cx)                 # runtime copy kernel
            cx.sum()                     # reduction (reads only)
        torch.cuda.synchronize()
        del cx, cy
    solver.ssprk3(u, dt, max(args.warmup, 1))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    # timed runs of exactly `steps` steps each (200 steps take ~0.11 s),
    # each bracketed by device synchronisation; the median run is the
    # headline
    reps_ms, walls = [], []
    # number of repeats: at least --repeats, and enough that the repeats
    # together last about 0.5 s (a 20-step repeat lasts ~11 ms), estimated
    # from one untimed repeat
    t0 = time.perf_counter()
    solver.ssprk3(u, dt, args.steps)
    torch.cuda.synchronize()
    est = time.perf_counter() - t0
    nrep = min(50, max(args.repeats, int(math.ceil(0.5 / max(est, 1e-6)))))
    for _ in range(max(1, nrep)):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        t0.record(stream)
        solver.ssprk3(u, dt, args.steps)
        t1.record(stream)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - wall0)
        reps_ms.append(t0.elapsed_time(t1))
    solver.check()
    ms = float(np.median(reps_ms))
    wall = float(np.median(walls))
    ms_per_step = ms / args.steps
    value = 3.0 * dof / (ms_per_step * 1e-3) / 1e9

    # per-kernel durations (HIP events on the launch stream, same fused stage form)
    kt = dgx.dgx_kernel_times(solver.ctx, u, reps=20)
    k_rhs_ms = kt["k_rhs"]
    rb = rhs_bytes_per_launch(nelem, nn, nvar, 3, 4)
    gb = grad_bytes_per_launch(nelem, nn, nvar, 3, 4)
    achieved = rb / (k_rhs_ms * 1e-3) / 1e9
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=recorded_traffic("tgv3d_ns_32cube_N3", order, epb),
                kernel="k_rhs", kernel_ms=round(k_rhs_ms, 5), bytes_per_launch=rb,
                other_kernels={k: round(v, 5) for k, v in kt.items() if k != "k_rhs"},
                k_grad_GBs=round(gb / (kt.get("k_grad", float("nan")) * 1e-3) / 1e9, 1))
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GDOF-RHS/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "tgv3d_ns_32cube_N3_ssprk3", "elements": nelem, "N": 3, "nodes": nelem * nn,
                   "dof": dof, "rhs_per_step": 3, "dt": dt, "wall_s": round(wall, 4),
                   "repeats": len(reps_ms), "repeat_ms_per_step": [round(r / args.steps, 5) for r in reps_ms],
                   "elements_per_workgroup": epb, "workgroup_order": ORDER_NAMES[order], "autotune_ms": {str(k): round(v, 5) for k, v in tune_ms.items()}},
        "roofline": roof,
    }
    solver.close()
    if not args.no_thermo:
        out["thermo"] = thermo_leg(torch, W, dgx)
    if not args.no_batch:
        out["batch"] = batch_leg(torch, W, dgx)
    if not args.no_c3:
        out["c3"] = c3_leg(torch, W, dgx, order=args.order, epb=args.c3_epb)
        out["c4"] = c4_leg(torch, W, dgx)
    if not args.no_fluxes:
        out["fluxes"] = flux_leg(torch, W, dgx)
    if not args.no_widened:
        out["mixture_fluxes"] = mixture_flux_leg(torch, W, dgx)
        out["ns"] = ns_leg(torch, W, dgx)
        out["amr"] = amr_leg(torch, W, dgx)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
