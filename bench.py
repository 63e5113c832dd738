"""Throughput of the DGSEM right-hand side on one MI355X.

Workload (default): the 3D compressible Navier-Stokes Taylor-Green vortex,
Mach 0.1, Re 1600, Pr 0.72, 32^3 periodic hexahedra, N = 3 (2,097,152 nodes,
10,485,760 DOF), FP64; entropy-conservative flux differencing, Rusanov
faces, BR1 viscous terms.  A step is one SSPRK3 step (three right-hand-side
evaluations fused with the stage updates, replayed from a HIP graph), so

    GDOF-RHS/s = 3 * DOF * steps / seconds / 1e9.

Prints one JSON line (see the keys below).  The oracle (NumPy, one thread)
is timed on the same 32^3 state for the cpu_baseline entry.
"""
import argparse
import json
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


def cpu_baseline(case, budget_s=20.0):
    """Oracle right-hand sides on the same state, one thread, ~budget_s."""
    from threadpoolctl import threadpool_limits
    from oracle.dgsem import Operator
    with threadpool_limits(limits=1):
        op = Operator(case.cfg, case.mesh)
        t0 = time.perf_counter()
        n = 0
        while True:
            op.rhs(case.u0)
            n += 1
            el = time.perf_counter() - t0
            if el > budget_s or n >= 10:
                break
    dof = case.u0.size
    return dict(value=dof * n / el / 1e9, unit="GDOF-RHS/s", cores=1, kind="oracle",
                sample="%d full right-hand sides of the 32^3 N=3 TGV state (%.1f s, NumPy FP64, 1 thread)"
                % (n, el))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 84 MB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs on a single MI355X "
              "(multi-GPU sharding is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_17551_amd import workloads as W
    from paper_2511_17551_amd import dgx

    case = W.case_c2()
    nvar, nelem, nn = case.u0.shape
    dof = case.u0.size
    solver = dgx.Solver(case)
    u = torch.from_numpy(case.u0).to("cuda")
    dt = dgx.dgx_max_dt(solver.ctx, u, 0.5)
    epb, tune_ms = dgx.dgx_autotune(solver.ctx, u, reps=10)
    if args.copy_probe:
        tmp = torch.empty_like(u)
        for _ in range(5):
            tmp.copy_(u)
        torch.cuda.synchronize()
        del tmp
    solver.ssprk3(u, dt, max(args.warmup, 1))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    solver.ssprk3(u, dt, args.steps)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    solver.check()
    ms = t0.elapsed_time(t1)
    ms_per_step = ms / args.steps
    value = 3.0 * dof / (ms_per_step * 1e-3) / 1e9

    # per-kernel durations (HIP events on the launch stream, same fused stage form)
    kt = dgx.dgx_kernel_times(solver.ctx, u, reps=20)
    k_rhs_ms = kt["k_rhs"]
    rb = rhs_bytes_per_launch(nelem, nn, nvar, 3, 4)
    gb = grad_bytes_per_launch(nelem, nn, nvar, 3, 4)
    achieved = rb / (k_rhs_ms * 1e-3) / 1e9
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
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
                   "elements_per_workgroup": epb, "autotune_ms": {str(k): round(v, 5) for k, v in tune_ms.items()}},
        "roofline": roof,
    }
    solver.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
