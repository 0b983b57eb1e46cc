#!/usr/bin/env python
"""Benchmark of the matrix-free Q2 heat operator on one MI355X.

Workload (the heat operator at scale): unit cube, 64^3 uniform hexahedral
cells, Q2 (3x3x3 Gauss points), 129^3 = 2,146,689 nodes, liquid sphere of
radius 0.3 at the center with phi = tanh(d/(2 eps)), eps = 2h, properties
blended by H = (1+phi)/2 (rho c_p 5e6 / 5e3 J/m^3K, k 30 / 0.3 W/mK),
dt = 1e-3, homogeneous Dirichlet faces.  Inputs are synthetic and resident
in device memory before timing starts.

One step = 100 operator applies y = A x (x ~ U[-1,1], seed 0) + one
Jacobi-preconditioned CG solve to 1e-10 relative residual with b = A T_I,
T_I the nodal interpolant of sin(pi x) sin(pi y) sin(pi z).

value      = applied DoFs per second over the timed applies (100 per step),
             whole-apply time (output clearing + kernel) from HIP events.
roofline   = the apply kernel alone (start/stop events attached to the
             kernel's own dispatch inside the library, on every 20th apply
             of the timed steps), algorithmic flops and bytes per launch.
cpu_baseline = the CPU oracle (assembled CSR, OpenMP) on the same workload.
mg_vs_cg   = FP32-multigrid-preconditioned FP64 flexible CG vs FP64 Jacobi-CG,
             both to 1e-8, on 128^3 cells (257^3 nodes): the hierarchy of the
             level rule and the configured six-level one.
oseen, heat_convection, heat_sources, three_phase, gradient,
transport_velocity = the other operators, the interface-flux right-hand
             side, the three-phase coefficients with the Tanasawa penalty and
             Darcy damping (and one Picard step), the adjoint step, and the
             level-set transport velocity.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of one heat apply in the FP64 level-set mode:
#   flops per cell, counted from the sum-factorized algorithm:
#     2 fields x 3 interpolation passes x 9 lines x 10 flops      = 540
#     coefficients, 27 Gauss points x 10 flops                      = 270
#     mass term, 27 products                                        =  27
#     gradient: 3 directions x 9 lines x 33 flops                   = 891
#     3 transposed interpolation passes x 9 lines x 9 flops         = 243
#     sums of the 27 cell results into nodes                        =  27
#   bytes per node: read x, read phi, write y, 8 bytes each        =  24
FLOPS_PER_CELL = 1998
BYTES_PER_NODE = 24
# With the convective term (heat operator given a velocity field), per cell:
#   3 velocity components x 3 interpolation passes x 9 lines x 10 flops = 810
#   u.grad T: 3 directions x 9 lines x (12 derivative + 9 products)    = 567
#   rc W (alpha_m T + alpha_c u.grad T), 27 points x 3 flops           =  81
# and per node 48 bytes: x, phi, the 3 velocity components and y.
FLOPS_PER_CELL_CONV = FLOPS_PER_CELL + 810 + 567 + 81
BYTES_PER_NODE_CONV = 48
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
METRIC = "Q2 operator-apply DoFs/s + HBM GB/s; FP32-MG vs FP64 CG time to 1e-8 resid"

# HBM traffic of the apply kernel, from hardware counters (FETCH_SIZE and
# WRITE_SIZE, one profiler pass each, scaled by what the same counters read for
# a copy kernel of known size).  The summary records a hash of the sources the
# kernel is built from; once they change, the figure no longer describes the
# kernel and traffic is reported as null.
APPLY_KERNEL = "heat_apply_kernel<double, 0, 0, false, 0, true, 4>"  # level set, equal cell edges
CALIB_KERNEL = "neg_kernel"
CALIB_BYTES = 8 << 26  # 2^26 doubles read and 2^26 written by the calibration copy
KERNEL_SOURCES = ["paper_2501_18781_amd/csrc/heat.hip", "paper_2501_18781_amd/csrc/brick.hpp",
                  "paper_2501_18781_amd/csrc/mf_common.hpp", "paper_2501_18781_amd/csrc/kernels.hpp"]
TRAFFIC_SUMMARY = "profiles/heat_apply_64cells_hbm_traffic.txt"


def parse():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--cells", type=int, default=64, help="cells per direction of the timed workload")
    p.add_argument("--applies", type=int, default=100)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-mg", action="store_true")
    p.add_argument("--no-cold", action="store_true")
    p.add_argument("--mg-cells", type=int, default=128)
    p.add_argument("--no-oseen", action="store_true")
    p.add_argument("--no-grad", action="store_true")
    p.add_argument("--no-conv", action="store_true")
    p.add_argument("--no-sources", action="store_true")
    p.add_argument("--no-three-phase", action="store_true")
    p.add_argument("--no-transport", action="store_true")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run a plain 512 MiB device copy first (reference for HBM byte counters)")
    p.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                   help="write the HBM traffic summary from two rocprofv3 --pmc output folders and exit")
    p.add_argument("--command", default="", help="profiled command line, recorded in the summary")
    p.add_argument("--kernel", default=APPLY_KERNEL,
                   help="kernel name (substring) the counter summaries describe")
    p.add_argument("--algorithmic-bytes", type=float, default=0.0,
                   help="algorithmic bytes per launch of --kernel, for the traffic summary")
    p.add_argument("--title", default="", help="first line of a counter summary")
    p.add_argument("--summarize-sq", nargs="+", metavar="DIR",
                   help="write the SQ counter summary of --kernel from rocprofv3 --pmc output folders and exit")
    p.add_argument("--summarize-trace", metavar="DIR",
                   help="write the kernel statistics of a rocprofv3 --kernel-trace --stats folder and exit")
    p.add_argument("--summarize-traffic-table", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                   help="write the per-kernel HBM traffic table from two rocprofv3 --pmc output folders and exit")
    p.add_argument("--profile-leg", default="",
                   help="run only this supplementary leg (oseen, heat_convection, heat_sources, three_phase, "
                        "gradient, transport_velocity, mg_vs_cg) and print its JSON, for profiler runs")
    return p.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _counter_means(folder, counter, kernel=APPLY_KERNEL):
    """Mean counter value per dispatch of the kernel and of the calibration copy."""
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {folder}")
    vals = {kernel: [], CALIB_KERNEL: []}
    for f in files:
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            for k in vals:
                if k in r["Kernel_Name"] and (k != CALIB_KERNEL or int(r["Grid_Size"]) >= (1 << 24)):
                    vals[k].append(float(r["Counter_Value"]))
    for k, v in vals.items():
        if not v:
            raise SystemExit(f"no {counter} rows for {k} in {folder}")
    return {k: sum(v) / len(v) for k, v in vals.items()}, {k: len(v) for k, v in vals.items()}


def summarize_counters(fetch_dir, write_dir, command, kernel=APPLY_KERNEL, alg_bytes=0.0, title=""):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the kernel, scaled so
    that the calibration copy reads as its true 512 MiB each way."""
    f, nf = _counter_means(fetch_dir, "FETCH_SIZE", kernel)
    w, nw = _counter_means(write_dir, "WRITE_SIZE", kernel)
    sf = CALIB_BYTES / (f[CALIB_KERNEL] * 1024.0)
    sw = CALIB_BYTES / (w[CALIB_KERNEL] * 1024.0)
    fetch_b = f[kernel] * 1024.0 * sf
    write_b = w[kernel] * 1024.0 * sw
    heat = kernel == APPLY_KERNEL
    alg = alg_bytes or (BYTES_PER_NODE * 129 ** 3 if heat else 0.0)
    lines = [
        title or "HBM traffic of the FP64 heat apply kernel, 64^3 cells (2,146,689 nodes)",
        f"command: {command}",
        f"kernel: {kernel} ({nf[kernel]} dispatches counted for FETCH_SIZE, {nw[kernel]} for WRITE_SIZE)",
        f"calibration: {CALIB_KERNEL} over 2^26 doubles ({CALIB_BYTES} bytes read, {CALIB_BYTES} written)",
        f"calibration FETCH_SIZE KiB: {f[CALIB_KERNEL]:.1f} (scale {sf:.4f})",
        f"calibration WRITE_SIZE KiB: {w[CALIB_KERNEL]:.1f} (scale {sw:.4f})",
        f"kernel FETCH_SIZE KiB per dispatch: {f[kernel]:.1f}",
        f"kernel WRITE_SIZE KiB per dispatch: {w[kernel]:.1f}",
        f"fetch_bytes_per_launch: {fetch_b:.0f}",
        f"write_bytes_per_launch: {write_b:.0f}",
        f"traffic_bytes_per_launch: {fetch_b + write_b:.0f}",
        f"algorithmic_bytes_per_launch: {alg:.0f}",
    ]
    if alg:
        lines.append(f"traffic / algorithmic: {(fetch_b + write_b) / alg:.3f}")
    if heat:
        lines.append(f"source_hash: {kernel_source_hash()}")
    return "\n".join(lines) + "\n"


def summarize_traffic_table(fetch_dir, write_dir, command, title=""):
    """FETCH_SIZE and WRITE_SIZE per dispatch of every kernel (by name and
    grid size) in two rocprofv3 --pmc folders, scaled like summarize_counters
    by the calibration copy."""
    def means(folder, counter):
        files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
        acc, calib = {}, []
        for f in files:
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter:
                    continue
                name = r["Kernel_Name"]
                if CALIB_KERNEL in name and int(r["Grid_Size"]) >= (1 << 24):
                    calib.append(float(r["Counter_Value"]))
                    continue
                short = name[5:] if name.startswith("void ") else name
                short = short[:short.index(">(") + 1] if ">(" in short else short.split("(")[0]
                acc.setdefault((short, int(r["Grid_Size"])), []).append(float(r["Counter_Value"]))
        if not calib:
            raise SystemExit(f"no calibration rows for {counter} in {folder}")
        scale = CALIB_BYTES / (sum(calib) / len(calib) * 1024.0)
        return {k: (sum(v) / len(v) * 1024.0 * scale, len(v)) for k, v in acc.items()}, scale
    f, sf = means(fetch_dir, "FETCH_SIZE")
    w, sw = means(write_dir, "WRITE_SIZE")
    rows = sorted(set(f) & set(w), key=lambda k: -(f[k][0] + w[k][0]) * f[k][1])
    lines = [title or "HBM traffic per dispatch", f"command: {command}",
             f"calibration: {CALIB_KERNEL} over 2^26 doubles; FETCH_SIZE scale {sf:.4f}, WRITE_SIZE scale {sw:.4f}", "",
             " dispatches  grid size   fetch MB   write MB  kernel"]
    for k in rows[:40]:
        lines.append(f"{f[k][1]:11d} {k[1]:10d} {f[k][0] / 1e6:10.2f} {w[k][0] / 1e6:10.2f}  {k[0]}")
    return "\n".join(lines) + "\n"


SQ_ORDER = ["SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_ACTIVE_INST_ANY", "SQ_WAIT_INST_ANY", "SQ_WAIT_ANY",
            "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS",
            "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_MISC"]


def summarize_sq(dirs, kernel, command, title=""):
    """Mean per-dispatch SQ counters of the kernel from rocprofv3 --pmc folders,
    with the shares of each wavefront's cycles they imply."""
    vals, ndisp = {}, 0
    for d in dirs:
        for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            acc = {}
            for r in csv.DictReader(open(fn)):
                if kernel in r["Kernel_Name"]:
                    acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
            for k, v in acc.items():
                vals[k] = sum(v) / len(v)
                ndisp = max(ndisp, len(v))
    lines = [title or f"SQ counters of {kernel}", f"command: {command}", f"kernel: {kernel} ({ndisp} dispatches averaged)",
             "", "per launch (summed over the device)            value"]
    for k in SQ_ORDER:
        if k in vals:
            lines.append(f"  {k:<40s} {vals[k]:>14.0f}")
    wc, nw = vals.get("SQ_WAVE_CYCLES"), vals.get("SQ_WAVES")
    if wc and nw:
        lines += ["", "derived, per wavefront (share of its wave cycles):"]
        for k, label in [("SQ_ACTIVE_INST_ANY", "issuing an instruction"), ("SQ_WAIT_INST_ANY", "waiting for the next issue"),
                         ("SQ_WAIT_ANY", "waiting on memory counters"), ("SQ_ACTIVE_INST_VALU", "VALU issue"),
                         ("SQ_ACTIVE_INST_LDS", "LDS issue")]:
            if k in vals:
                lines.append(f"  {label:<34s} {vals[k] / wc:7.1%}")
        for k, label in [("SQ_INSTS_VALU", "VALU"), ("SQ_INSTS_SALU", "SALU"), ("SQ_INSTS_LDS", "LDS"),
                         ("SQ_INSTS_VMEM_RD", "vector memory read"), ("SQ_INSTS_VMEM_WR", "vector memory write")]:
            if k in vals:
                lines.append(f"  {label + ' instructions per wavefront':<48s} {vals[k] / nw:8.0f}")
    return "\n".join(lines) + "\n"


def summarize_trace(folder, command, title=""):
    """Per-kernel statistics (calls, average, min, max, share) of a rocprofv3
    --kernel-trace --stats folder, the kernels sorted by total time."""
    files = glob.glob(os.path.join(folder, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no kernel_stats.csv under {folder}")
    rows = list(csv.DictReader(open(files[0])))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [title or "Kernel statistics", f"command: {command}", "",
             " calls    avg us    min us    max us  % time  kernel"]
    for r in rows[:40]:
        name = r["Name"]
        name = name[5:] if name.startswith("void ") else name
        name = name.split("(")[0] if "<" not in name.split("(")[0] else name[:name.index(">(") + 1] if ">(" in name else name
        lines.append(f"{int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:9.1f} {float(r['MinNs']) / 1e3:9.1f} "
                     f"{float(r['MaxNs']) / 1e3:9.1f} {float(r['Percentage']):6.1f}%  {name}")
    return "\n".join(lines) + "\n"


def measured_traffic():
    """Scaled counter bytes per launch from the committed summary, or None if
    the summary is missing or was taken from other kernel sources."""
    path = os.path.join(ROOT, TRAFFIC_SUMMARY)
    if not os.path.exists(path):
        return None
    fields = dict(l.split(": ", 1) for l in open(path).read().splitlines() if ": " in l)
    if fields.get("source_hash", "").strip() != kernel_source_hash():
        return None
    return float(fields["traffic_bytes_per_launch"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu():
    """Model name and logical CPU count of the host, from /proc/cpuinfo and lscpu."""
    import subprocess
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        lscpu = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        fields = {l.split(":", 1)[0].strip(): l.split(":", 1)[1].strip() for l in lscpu.splitlines() if ":" in l}
        lscpu = {k: fields[k] for k in ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket",
                                         "Socket(s)", "L3") if k in fields}
    except Exception:
        lscpu = {}
    return {"model": model, "nproc": os.cpu_count(), "lscpu": lscpu}


def cpu_baseline(wl, x, b_T, min_spmv_s=5.0, max_spmv=3000):
    """The oracle as it is (assembled CSR + OpenMP SpMV, numpy Krylov loops):
      heat 64^3: assembly, CSR SpMVs until min_spmv_s seconds have passed (at
        most max_spmv), one Jacobi-CG solve to 1e-10 (b = A T_I);
      Oseen 48^3: assembly, GMRES(30) with 3x3 point-block Jacobi to 1e-8 on
        b = A x_ref (x_ref ~ U[-1,1], seed 1);
      gradient 32^3: assembled-matrix adjoint gradient of the one-step
        misfit with respect to k_q, rc_q and phi (delta-form and adjoint
        Jacobi-CG to 1e-14).
    value = heat SpMV DoFs/s."""
    import numpy as np

    import oracle as O
    from paper_2501_18781_amd import workloads as W

    t0 = time.perf_counter()
    A = O.heat_matrix(wl.mesh, wl.params, phi=wl.phi)
    t_asm = time.perf_counter() - t0
    y = O.spmv(A, x)
    t0 = time.perf_counter()
    nspmv = 0
    while nspmv < max_spmv and (time.perf_counter() - t0) < min_spmv_s:
        y = O.spmv(A, x)
        nspmv += 1
    t_spmv = time.perf_counter() - t0
    b = O.spmv(A, b_T)
    t0 = time.perf_counter()
    r = O.jacobi_cg(A, b, 1e-10)
    t_cg = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    del A, y
    out = {
        "value": nspmv * wl.mesh.n_nodes / t_spmv,
        "unit": "DoFs/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{wl.mesh.n[0]}^3 heat operator: CSR assembly by full Gauss quadrature ({t_asm:.1f} s), "
                   f"{nspmv} CSR SpMVs ({t_spmv:.2f} s), Jacobi-CG to 1e-10 ({r.iters} it, {t_cg:.2f} s); "
                   f"value = SpMV DoFs/s; also Oseen 48^3 GMRES(30) and the 32^3 adjoint gradient"),
        "assembly_s": t_asm,
        "cg_s": t_cg,
        "cg_iters": r.iters,
        "host": host_cpu(),
    }
    log(f"[bench] CPU heat: {out['value']:.3g} DoFs/s, CG {r.iters} it {t_cg:.2f} s")
    # Oseen 48^3, GMRES(30) with point-block Jacobi to 1e-8
    ow = W.oseen_wavy_workload(48)
    t0 = time.perf_counter()
    B = O.oseen_matrix(ow.mesh, ow.params, ow.phi, ow.u0)
    t_oasm = time.perf_counter() - t0
    xr = W.uniform(1, 3 * ow.mesh.n_nodes)
    bo = O.spmv(B, xr)
    t0 = time.perf_counter()
    pc = O.block_jacobi(B, ow.mesh.n_nodes)
    ro = O.gmres(B, bo, pc, 30, 1e-8)
    t_gm = time.perf_counter() - t0
    out["oseen_gmres30_block_jacobi"] = {"cells": 48, "assembly_s": t_oasm, "solve_s": t_gm, "iters": ro.iters,
                                         "rel_res": ro.rel_res, "converged": bool(ro.converged),
                                         "rel_err_vs_x_ref": float(np.linalg.norm(ro.x - xr) / np.linalg.norm(xr))}
    log(f"[bench] CPU Oseen 48^3: assembly {t_oasm:.1f} s, GMRES(30) {ro.iters} it {t_gm:.1f} s")
    del B, pc
    # assembled-adjoint gradient on 32^3 cells
    gw = W.heat_sphere_workload(32, W.ALL_FACES)
    t0 = time.perf_counter()
    m, p = gw.mesh, gw.params
    kq, rcq = O.heat_qp_coeffs(m, p, gw.phi)
    Told = W.manufactured_T(m)
    free = ~O.constrained_mask(m)
    Told[~free] = 0.0
    Ag = O.heat_matrix(m, p, kq=kq, rcq=rcq)
    K = O.heat_matrix(m, p, kq=kq, rcq=rcq, alpha_m=0.0)
    dT = O.jacobi_cg(Ag, -(K @ Told) * free, 1e-14).x
    lam = O.jacobi_cg(Ag, 2.0 * (dT - 0.999 * dT) * free, 1e-14).x
    O.heat_grad(m, p, Told + dT, Told, lam, phi=gw.phi, dT=dT)
    t_gr = time.perf_counter() - t0
    out["gradient_32"] = {"cells": 32, "s": t_gr,
                          "what": "assembly, delta-form CG, adjoint CG, gradients w.r.t. k_q, rc_q, phi"}
    log(f"[bench] CPU adjoint gradient 32^3: {t_gr:.2f} s")
    return out


def main():
    args = parse()
    if args.summarize_counters:
        sys.stdout.write(summarize_counters(*args.summarize_counters, args.command, args.kernel,
                                            args.algorithmic_bytes, args.title))
        return
    if args.summarize_sq:
        sys.stdout.write(summarize_sq(args.summarize_sq, args.kernel, args.command, args.title))
        return
    if args.summarize_trace:
        sys.stdout.write(summarize_trace(args.summarize_trace, args.command, args.title))
        return
    if args.summarize_traffic_table:
        sys.stdout.write(summarize_traffic_table(*args.summarize_traffic_table, args.command, args.title))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the path has no multi-GPU code (the kernels run on one GPU); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2501_18781_amd import mf
    from paper_2501_18781_amd import workloads as W

    torch.cuda.set_device(0)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    legs = {"mg_vs_cg": lambda: mg_vs_cg(args.mg_cells, dev), "oseen": lambda: oseen_bench(dev),
            "heat_convection": lambda: heat_conv_bench(dev), "heat_sources": lambda: heat_sources_bench(dev),
            "three_phase": lambda: three_phase_bench(dev), "gradient": lambda: grad_bench(dev),
            "transport_velocity": lambda: transport_bench(dev)}
    if args.copy_calibration:
        # 2^26 doubles: FETCH_SIZE and WRITE_SIZE of this copy should read 512 MiB each
        src = torch.ones(1 << 26, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if args.profile_leg:
        print(json.dumps({args.profile_leg: legs[args.profile_leg]()}), flush=True)
        return
    n = args.cells
    wl = W.heat_sphere_workload(n, W.ALL_FACES)
    nn, nc = wl.mesh.n_nodes, wl.mesh.n_cells
    log(f"[bench] heat {n}^3 cells, {nn} nodes")
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
    x_np = W.uniform(0, nn)
    x = dev(x_np)
    y = torch.empty(nn, dtype=torch.float64, device="cuda")
    b = torch.empty_like(y)
    mf.operator_apply(op, dev(W.manufactured_T(wl.mesh)), b)
    xs = torch.empty_like(y)
    s = torch.cuda.current_stream()

    # Every SAMPLE-th apply of a timed step carries start/stop events attached
    # to the kernel's own dispatch (the roofline's kernel time); events on
    # every launch would add about 5 us to each whole apply.
    # The sample sits mid-way through each group of SAMPLE applies, away from
    # the step's CG solve.
    SAMPLE = 20
    phase = min(SAMPLE // 2, args.applies - 1)

    def step(ev, timed=False):
        ev[0].record(s)
        for i in range(args.applies):
            sample = timed and i % SAMPLE == phase
            if sample:
                ctx.timing_enable(True)
            mf.operator_apply(op, x, y)
            if sample:
                ctx.timing_enable(False)
        ev[1].record(s)
        info = mf.cg_solve(op, b, xs, 1e-10, 1000)
        ev[2].record(s)
        return info

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(max(args.steps, args.warmup, 1))]
    for i in range(args.warmup):
        step(ev[i])
    torch.cuda.synchronize()
    log("[bench] warmup done")
    ctx.timing_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step(ev[i], timed=True) for i in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel_ms, launches = ctx.timing_read(reset=True)
    apply_ms = sum(e[0].elapsed_time(e[1]) for e in ev[:args.steps])
    per_step_us = [e[0].elapsed_time(e[1]) * 1e3 / args.applies for e in ev[:args.steps]]
    cg_ms = sum(e[1].elapsed_time(e[2]) for e in ev[:args.steps]) / args.steps
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = args.steps * args.applies * nn / (apply_ms * 1e-3)
    k_s = kernel_ms * 1e-3 / launches
    flops = FLOPS_PER_CELL * nc
    bytes_ = BYTES_PER_NODE * nn
    tflops = flops / k_s / 1e12
    gbs = bytes_ / k_s / 1e9
    frac_alu, frac_hbm = tflops / PEAK_FP64_TFLOPS, gbs / PEAK_HBM_GBS
    if frac_alu >= frac_hbm:
        roof = {"bound": "alu", "achieved": tflops, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": frac_alu}
    else:
        roof = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": frac_hbm}
    traffic = measured_traffic() if n == 64 else None
    roof["traffic"] = traffic
    roof["kernel"] = "heat_apply_kernel<double, levelset>"
    roof["kernel_us"] = k_s * 1e6
    roof["flops_per_launch"] = flops
    roof["bytes_per_launch"] = bytes_
    roof["hbm_frac"] = frac_hbm
    roof["fp64_frac"] = frac_alu
    # attainable-bandwidth reference: a streaming copy (torch.neg) of 512 MiB
    src = torch.ones(1 << 26, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(s)
    for _ in range(10):
        torch.neg(src, out=dst)
    c1.record(s)
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * src.numel() * 8 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst
    roof["copy_gbs"] = copy_gbs
    roof["hbm_frac_vs_copy"] = gbs / copy_gbs
    roof["whole_apply_us"] = apply_ms / args.steps / args.applies * 1e3
    log(f"[bench] apply kernel {k_s * 1e6:.1f} us: {tflops:.2f} TFLOP/s ({frac_alu:.1%} FP64), "
        f"{gbs:.0f} GB/s ({frac_hbm:.1%} HBM); whole apply {apply_ms / args.steps / args.applies * 1e3:.1f} us")
    info = infos[-1]
    log(f"[bench] CG {info.iters} iterations, {cg_ms:.2f} ms, true rel. residual {info.rel_res:.2e}")

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "DoFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"heat operator, Q2, {n}^3 cells ({nn} nodes), sphere r=0.3 tanh level set, "
                               f"eps=2h, rc 5e6/5e3, k 30/0.3, dt=1e-3, Dirichlet; 100 applies + Jacobi-CG to 1e-10",
                   "cells": n, "nodes": nn, "applies_per_step": args.applies},
        "roofline": roof,
        "cg": {"iters": info.iters, "ms": cg_ms, "rel_res": info.rel_res, "converged": bool(info.converged)},
        # the spread of the timed steps (value above is their total)
        "apply_steps": {"whole_apply_us": per_step_us, "median_us": sorted(per_step_us)[len(per_step_us) // 2]},
    }

    if not args.no_cold:
        # HBM-resident figure: rotate through 8 independent (x, phi, y) sets
        # (412 MB in total at 64^3) so that no apply finds its data in the
        # 256 MB last-level cache.
        sets = []
        for k in range(8):
            phik = dev(wl.phi)
            sets.append((mf.heat_operator(ctx, wl.params, phi=phik), dev(np.roll(x_np, k)), torch.empty_like(y)))
        for o, xx, yy in sets:
            mf.operator_apply(o, xx, yy)
        torch.cuda.synchronize()
        ctx.timing_enable(True)
        ctx.timing_read(reset=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for i in range(args.applies):
            o, xx, yy = sets[i % 8]
            mf.operator_apply(o, xx, yy)
        e1.record(s)
        torch.cuda.synchronize()
        kms, kl = ctx.timing_read(reset=True)
        ctx.timing_enable(False)
        kc = kms * 1e-3 / kl
        result["apply_cold"] = {"dofs_per_s": args.applies * nn / (e0.elapsed_time(e1) * 1e-3),
                                "kernel_us": kc * 1e6, "gbs": bytes_ / kc / 1e9, "tflops": flops / kc / 1e12,
                                "note": "8 rotating buffer sets, 412 MB, larger than the last-level cache"}
        log(f"[bench] cold apply kernel {kc * 1e6:.1f} us ({bytes_ / kc / 1e9:.0f} GB/s)")
        del sets

    del ctx, op
    for flag, key in [(args.no_mg, "mg_vs_cg"), (args.no_oseen, "oseen"), (args.no_conv, "heat_convection"),
                      (args.no_sources, "heat_sources"), (args.no_three_phase, "three_phase"),
                      (args.no_grad, "gradient"), (args.no_transport, "transport_velocity")]:
        if flag:
            continue
        try:
            result[key] = legs[key]()
        except Exception as e:  # reported, never silently replaced
            result[key] = {"error": f"{type(e).__name__}: {e}"}

    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        result["cpu_baseline"] = cpu_baseline(wl, x_np, W.manufactured_T(wl.mesh))
    print(json.dumps(result), flush=True)


def mg_vs_cg(n, dev):
    """Time to 1e-8 relative residual on n^3 cells: FP32-multigrid flexible CG
    vs FP64 Jacobi-CG.  Two hierarchies:
      fcg_fp32_mg             the level rule (coarsening stops where the mass
                              term dominates the diagonal, that level smoothed
                              by Chebyshev(2); Chebyshev(1) on the levels with
                              a coarse correction, 4^3 coarse level by FP64 CG);
      fcg_fp32_mg_configured  six levels to 4^3, Chebyshev(4), FP64 CG coarse."""
    import numpy as np
    import torch

    from paper_2501_18781_amd import mf
    from paper_2501_18781_amd import workloads as W

    out = {"cells": n, "rtol": 1e-8}
    regimes = [("dt=1e-3", W.HeatParams()),
               ("dt=1 (mass and conduction comparable, supplementary)", W.HeatParams(dt=1.0)),
               ("dt=1e3 (conduction-dominated, supplementary)", W.HeatParams(dt=1e3))]
    hierarchies = [("fcg_fp32_mg", mf.MGConfig(coarse_cells=4, degree=1, auto_levels=True, smooth_degree=2)),
                   ("fcg_fp32_mg_configured", mf.MGConfig(coarse_cells=4, degree=4))]
    for label, params in regimes:
        wl = W.heat_sphere_workload(n, W.ALL_FACES, params)
        log(f"[bench] mg vs cg {n}^3 {label}")
        ctx = mf.Context(wl.mesh)
        op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
        b = torch.empty(wl.mesh.n_nodes, dtype=torch.float64, device="cuda")
        mf.operator_apply(op, dev(W.manufactured_T(wl.mesh)), b)
        xc = torch.empty_like(b)
        xm = torch.empty_like(b)
        mf.cg_solve(op, b, xc, 1e-8, 5000)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ic = mf.cg_solve(op, b, xc, 1e-8, 5000)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t0
        entry = {"cg_fp64_jacobi": {"ms": tc * 1e3, "iters": ic.iters, "rel_res": ic.rel_res}}
        msg = f"[bench]   CG {ic.iters} it {tc * 1e3:.1f} ms"
        for key, cfg in hierarchies:
            t0 = time.perf_counter()
            mg = mf.Multigrid(op, cfg)
            torch.cuda.synchronize()
            tsetup = time.perf_counter() - t0
            mf.mg_cg_solve(mg, b, xm, 1e-8, 300)  # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            im = mf.mg_cg_solve(mg, b, xm, 1e-8, 300)
            torch.cuda.synchronize()
            tm = time.perf_counter() - t0
            err = float(torch.linalg.norm(xm - xc) / torch.linalg.norm(xc))
            entry[key] = {"ms": tm * 1e3, "iters": im.iters, "rel_res": im.rel_res, "setup_ms": tsetup * 1e3,
                          "levels": [{"cells": c, "degree": d} for c, d, _, _ in mg.levels()],
                          "speedup": tc / tm, "rel_diff_vs_cg": err}
            msg += f" | {key} {im.iters} it {tm * 1e3:.1f} ms ({mg.n_levels} levels, {tc / tm:.2f}x)"
            mg.close()
        entry["speedup"] = entry["fcg_fp32_mg"]["speedup"]
        entry["rel_diff_vs_cg"] = entry["fcg_fp32_mg"]["rel_diff_vs_cg"]
        out[label] = entry
        log(msg)
        del op, ctx
    return out


def oseen_bench(dev, applies=50):
    """Linearized momentum operator on 48^3 cells (3 x 912,673 velocity DoFs):
    apply throughput, and GMRES(30) with 3x3 point-block Jacobi to 1e-8 on
    b = A x_ref (x_ref ~ U[-1,1], seed 1)."""
    import torch

    from paper_2501_18781_amd import mf
    from paper_2501_18781_amd import workloads as W

    wl = W.oseen_wavy_workload(48)
    nd = 3 * wl.mesh.n_nodes
    log(f"[bench] oseen 48^3: {nd} velocity DoFs")
    ctx = mf.Context(wl.mesh)
    op = mf.oseen_operator(ctx, wl.params, dev(wl.phi), dev(wl.u0))
    xr = dev(W.uniform(1, nd))
    b = torch.empty_like(xr)
    # algorithmic bytes per velocity DoF: x, y, u0 (8 B each) and phi (8 B per 3 DoFs);
    # operation estimate per velocity DoF: about 390 flops (interpolations of
    # x, u0 and phi, the quadrature-point operator, the transposed integration)
    bpd, fpd = 24 + 8 / 3, 390.0
    out = {"cells": 48, "velocity_dofs": nd, "bytes_per_dof": bpd, "flops_per_dof_estimate": fpd}
    for label, fn in [("apply", mf.operator_apply), ("apply_transpose", mf.operator_apply_transpose)]:
        whole, kt = _time_applies(ctx, fn, op, xr, b, applies)
        out[label] = {"us": whole * 1e6, "dofs_per_s": nd / whole, "algorithmic_gbs": nd * bpd / whole / 1e9,
                      "kernel_us": kt * 1e6, "kernel_algorithmic_gbs": nd * bpd / kt / 1e9,
                      "kernel_tflops_estimate": nd * fpd / kt / 1e12,
                      "hbm_frac": nd * bpd / kt / (PEAK_HBM_GBS * 1e9),
                      "fp64_frac_estimate": nd * fpd / kt / (PEAK_FP64_TFLOPS * 1e12)}
    mf.operator_apply(op, xr, b)
    x = torch.empty_like(b)
    mf.gmres_solve(op, b, x, 1e-8, 3000, precond=mf.MF_PC_BLOCK_JACOBI, restart=30)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = mf.gmres_solve(op, b, x, 1e-8, 3000, precond=mf.MF_PC_BLOCK_JACOBI, restart=30)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    err = float(torch.linalg.norm(x - xr) / torch.linalg.norm(xr))
    out["gmres30_block_jacobi"] = {"ms": t * 1e3, "iters": info.iters, "rel_res": info.rel_res,
                                   "converged": bool(info.converged), "rel_err_vs_x_ref": err}
    log(f"[bench]   apply {out['apply']['us']:.1f} us (kernel {out['apply']['kernel_us']:.1f}), transpose "
        f"{out['apply_transpose']['us']:.1f} us; GMRES(30) {info.iters} it {t * 1e3:.1f} ms, err {err:.1e}")
    return out


def heat_conv_bench(dev, applies=50):
    """Heat operator with the convective term on the 64^3 heat mesh (2,146,689
    nodes) with the Taylor-Green velocity (peak 1 m/s): apply and transpose
    throughput (kernel alone and whole apply), and Jacobi-GMRES(30) to 1e-8 on
    b = A x_ref (x_ref ~ U[-1,1], seed 0)."""
    import torch

    from paper_2501_18781_amd import mf
    from paper_2501_18781_amd import workloads as W

    n = 64
    wl = W.heat_conv_workload(n, W.ALL_FACES)
    nn = wl.mesh.n_nodes
    log(f"[bench] heat with convection {n}^3: {nn} nodes")
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi), u0=dev(wl.u0))
    xr = dev(W.uniform(0, nn))
    b = torch.empty_like(xr)
    flops, bytes_ = FLOPS_PER_CELL_CONV * n ** 3, BYTES_PER_NODE_CONV * nn
    out = {"cells": n, "nodes": nn, "flops_per_cell": FLOPS_PER_CELL_CONV, "bytes_per_node": BYTES_PER_NODE_CONV}
    for label, fn in [("apply", mf.operator_apply), ("apply_transpose", mf.operator_apply_transpose)]:
        whole, kt = _time_applies(ctx, fn, op, xr, b, applies)
        out[label] = {"us": whole * 1e6, "dofs_per_s": nn / whole, "kernel_us": kt * 1e6,
                      "kernel_algorithmic_gbs": bytes_ / kt / 1e9, "kernel_tflops": flops / kt / 1e12,
                      "hbm_frac": bytes_ / kt / 1e9 / PEAK_HBM_GBS, "fp64_frac": flops / kt / 1e12 / PEAK_FP64_TFLOPS}
    mf.operator_apply(op, xr, b)
    x = torch.empty_like(b)
    mf.gmres_solve(op, b, x, 1e-8, 3000, precond=mf.MF_PC_JACOBI, restart=30)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = mf.gmres_solve(op, b, x, 1e-8, 3000, precond=mf.MF_PC_JACOBI, restart=30)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    err = float(torch.linalg.norm(x - xr) / torch.linalg.norm(xr))
    out["gmres30_jacobi"] = {"ms": t * 1e3, "iters": info.iters, "rel_res": info.rel_res,
                             "converged": bool(info.converged), "rel_err_vs_x_ref": err}
    log(f"[bench]   apply {out['apply']['us']:.1f} us (kernel {out['apply']['kernel_us']:.1f}), transpose "
        f"{out['apply_transpose']['us']:.1f} us; GMRES(30) {info.iters} it {t * 1e3:.1f} ms, err {err:.1e}")
    return out


def heat_sources_bench(dev, reps=50):
    """Right-hand side of the interface heat fluxes (evaporative cooling and the
    laser heat flux) on the 64^3 heat mesh: sphere level set, temperature
    around the boiling point, beam along -z.  Whole assembly (kernel + shared
    node combine), HIP events; 24 algorithmic bytes per node (phi, T, b)."""
    import torch

    from paper_2501_18781_amd import mf
    from paper_2501_18781_amd import workloads as W

    n = 64
    wl = W.heat_source_workload(n, W.ALL_FACES)
    nn = wl.mesh.n_nodes
    log(f"[bench] interface heat sources {n}^3: {nn} nodes")
    ctx = mf.Context(wl.mesh)
    op = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
    T = dev(wl.T)
    b = torch.empty_like(T)
    t = _time_calls(lambda: mf.heat_source_rhs(op, wl.sources, T, b), reps)
    out = {"cells": n, "nodes": nn, "us": t * 1e6, "dofs_per_s": nn / t, "algorithmic_gbs": 24 * nn / t / 1e9,
           "terms": "evaporative cooling (Tanasawa, local T) + Gaussian laser flux"}
    log(f"[bench]   assembly {t * 1e6:.1f} us ({24 * nn / t / 1e9:.0f} GB/s algorithmic)")
    return out


def _warm(call, ms=30.0):
    """Run call() back to back for at least `ms` milliseconds of wall time, so
    that the timed calls that follow see the GPU at its steady clocks."""
    import torch
    t0 = time.perf_counter()
    while True:
        for _ in range(5):
            call()
        torch.cuda.synchronize()
        if (time.perf_counter() - t0) * 1e3 >= ms:
            return


def _time_calls(call, n, batches=5):
    """Median over `batches` batches of n back-to-back calls (HIP events on
    the current stream) of the time per call in seconds, after a warm-up."""
    import torch
    _warm(call)
    s = torch.cuda.current_stream()
    per = []
    for _ in range(batches):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(n):
            call()
        e1.record(s)
        torch.cuda.synchronize()
        per.append(e0.elapsed_time(e1) * 1e-3 / n)
    return sorted(per)[len(per) // 2]


def _time_applies(ctx, fn, op, x, y, applies):
    """Whole-apply and apply-kernel time (seconds per apply) of `applies`
    back-to-back calls each, after a warm-up: the whole applies without
    kernel events (they would add about 5 us to each), then the kernel alone
    with start/stop events attached to its dispatch."""
    import torch
    whole = _time_calls(lambda: fn(op, x, y), applies)
    ctx.timing_enable(True)
    ctx.timing_read(reset=True)
    for _ in range(applies):
        fn(op, x, y)
    torch.cuda.synchronize()
    kms, kl = ctx.timing_read(reset=True)
    ctx.timing_enable(False)
    return whole, kms * 1e-3 / kl


def three_phase_bench(dev, applies=50, beta=2.0e9):
    """Three-phase coefficients at a frozen temperature crossing the melting
    range (T = 1800 K + 600 K z):
      heat, 64^3 cells with the sphere level set and the Tanasawa penalty
      (beta = 2e9): apply (32 algorithmic bytes per node: x, phi, T, y),
      Jacobi-CG to 1e-8 on b = A x_ref next to the two-phase operator's, and one
      Picard step (dt = 1e-3, evaporation + laser + penalty right-hand side,
      update 1e-10);
      Oseen, 48^3 cells with the wavy-plane level set and Darcy damping:
      apply and transpose (3 x 8 + 8/3 + 8/3 bytes per velocity DoF)."""
    import dataclasses

    import torch

    from paper_2501_18781_amd import mf, picard
    from paper_2501_18781_amd import workloads as W

    n = 64
    wl = W.heat_sphere_workload(n, W.ALL_FACES)
    nn = wl.mesh.n_nodes
    log(f"[bench] three-phase heat {n}^3: {nn} nodes")
    ctx = mf.Context(wl.mesh)
    p = dataclasses.replace(wl.params, penalty=beta)
    Tc = dev(W.melt_temperature(wl.mesh))
    op = mf.heat_operator(ctx, p, phi=dev(wl.phi), T_coef=Tc)
    op2 = mf.heat_operator(ctx, wl.params, phi=dev(wl.phi))
    xr = dev(W.uniform(0, nn))
    b = torch.empty_like(xr)
    out = {"heat": {"cells": n, "nodes": nn, "bytes_per_node": 32, "penalty": beta}}
    for label, fn in [("apply", mf.operator_apply)]:
        whole, kt = _time_applies(ctx, fn, op, xr, b, applies)
        out["heat"][label] = {"us": whole * 1e6, "dofs_per_s": nn / whole, "kernel_us": kt * 1e6,
                              "kernel_algorithmic_gbs": 32 * nn / kt / 1e9,
                              "hbm_frac": 32 * nn / kt / 1e9 / PEAK_HBM_GBS}
    x = torch.empty_like(xr)
    for label, o in [("cg_jacobi", op), ("cg_jacobi_two_phase", op2)]:
        mf.operator_apply(o, xr, b)
        mf.cg_solve(o, b, x, 1e-8, 5000)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = mf.cg_solve(o, b, x, 1e-8, 5000)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out["heat"][label] = {"ms": t * 1e3, "iters": info.iters, "rel_res": info.rel_res,
                              "converged": bool(info.converged)}
    sp = dataclasses.replace(W.heat_source_workload(n, W.ALL_FACES).sources, terms=7)
    T_old = dev(W.melt_temperature(wl.mesh))
    picard.heat_step(ctx, p, dev(wl.phi), T_old, sources=sp, tol=1e-10, maxit=10)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = picard.heat_step(ctx, p, dev(wl.phi), T_old, sources=sp, tol=1e-10, maxit=10)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out["heat"]["picard_step"] = {"ms": t * 1e3, "iterations": res.iterations, "converged": res.converged,
                                  "cg_iterations": res.cg_iterations}
    h = out["heat"]
    log(f"[bench]   apply {h['apply']['us']:.1f} us (kernel {h['apply']['kernel_us']:.1f}); CG "
        f"{h['cg_jacobi']['iters']} it {h['cg_jacobi']['ms']:.1f} ms (two-phase {h['cg_jacobi_two_phase']['iters']} it "
        f"{h['cg_jacobi_two_phase']['ms']:.1f} ms); Picard {res.iterations} it {t * 1e3:.1f} ms")

    wo = W.oseen_wavy_workload(48)
    nd = 3 * wo.mesh.n_nodes
    log(f"[bench] three-phase oseen 48^3: {nd} velocity DoFs")
    octx = mf.Context(wo.mesh)
    oop = mf.oseen_operator(octx, wo.params, dev(wo.phi), dev(wo.u0), T_coef=dev(W.melt_temperature(wo.mesh)))
    xo = dev(W.uniform(1, nd))
    bo = torch.empty_like(xo)
    bpd = 24 + 16 / 3
    out["oseen"] = {"cells": 48, "velocity_dofs": nd, "bytes_per_dof": bpd}
    for label, fn in [("apply", mf.operator_apply), ("apply_transpose", mf.operator_apply_transpose)]:
        whole, kt = _time_applies(octx, fn, oop, xo, bo, applies)
        out["oseen"][label] = {"us": whole * 1e6, "dofs_per_s": nd / whole, "kernel_us": kt * 1e6,
                               "kernel_algorithmic_gbs": bpd * nd / kt / 1e9}
    log(f"[bench]   oseen apply {out['oseen']['apply']['us']:.1f} us, transpose "
        f"{out['oseen']['apply_transpose']['us']:.1f} us")
    return out


def grad_bench(dev, reps=5):
    """One differentiable implicit heat step on 32^3 cells: forward (delta-form
    Jacobi-CG to 1e-14) and backward (adjoint CG + gradient kernel), with
    respect to the level set and to the quadrature-point coefficients."""
    import torch

    from paper_2501_18781_amd import mf
    from paper_2501_18781_amd import workloads as W
    from paper_2501_18781_amd.autograd import HeatStep, heat_step

    wl = W.heat_sphere_workload(32, W.ALL_FACES)
    ctx = mf.Context(wl.mesh)
    step = HeatStep(ctx, wl.params)
    Told = dev(W.manufactured_T(wl.mesh))
    tgt = Told * 0.999
    nq = ctx.n_cells * 27
    kq = torch.empty(nq, dtype=torch.float64, device="cuda")
    rcq = torch.empty_like(kq)
    mf.heat_qp_coeffs(step.operator(phi=dev(wl.phi)), kq, rcq)
    out = {"cells": 32, "nodes": wl.mesh.n_nodes, "quad_points": nq}
    for label, make in [("wrt_phi", lambda: {"phi": dev(wl.phi).requires_grad_(True)}),
                        ("wrt_k_rc", lambda: {"k_q": kq.clone().requires_grad_(True),
                                              "rc_q": rcq.clone().requires_grad_(True)})]:
        times = []
        for _ in range(reps + 1):
            kw = make()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            T, _ = heat_step(step, Told, **kw)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            torch.sum((T - tgt) ** 2).backward()
            torch.cuda.synchronize()
            times.append((t1 - t0, time.perf_counter() - t1))
        fw = sorted(t[0] for t in times[1:])[reps // 2]
        bw = sorted(t[1] for t in times[1:])[reps // 2]
        out[label] = {"forward_ms": fw * 1e3, "backward_ms": bw * 1e3}
        log(f"[bench]   gradient {label}: forward {fw * 1e3:.2f} ms, backward {bw * 1e3:.2f} ms")
    return out


# Algorithmic bytes per node of the transport velocity: read phi, T and the
# three velocity components, write the three components of u_Gamma.
BYTES_PER_NODE_TRANSPORT = 8 * 8


def transport_bench(dev, reps=50):
    """Level-set transport velocity on the 64^3 mesh (2,146,689 nodes): the
    liquid sphere with the sine Heaviside, Taylor-Green velocity, temperature
    around the boiling point.  Whole call (distance pass + velocity pass),
    HIP events, both variants; 64 algorithmic bytes per node."""
    import torch

    from paper_2501_18781_amd import mf
    from paper_2501_18781_amd import workloads as W

    wl = W.transport_workload(64)
    nn = wl.mesh.n_nodes
    log(f"[bench] transport velocity 64^3: {nn} nodes")
    ctx = mf.Context(wl.mesh)
    phi, u, T = dev(wl.phi), dev(wl.u), dev(wl.T)
    ug = torch.empty_like(u)
    out = {"cells": 64, "nodes": nn, "bytes_per_node": BYTES_PER_NODE_TRANSPORT}
    for variant, label in [(mf.MF_TRANSPORT_LOCAL, "local"), (mf.MF_TRANSPORT_LIQUID_EXTENSION, "liquid_extension")]:
        t = _time_calls(lambda: mf.transport_velocity(ctx, variant, wl.params, wl.sources, phi, u, T, ug), reps)
        gbs = BYTES_PER_NODE_TRANSPORT * nn / t / 1e9
        out[label] = {"us": t * 1e6, "nodes_per_s": nn / t, "algorithmic_gbs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS}
        log(f"[bench]   {label}: {t * 1e6:.1f} us ({gbs:.0f} GB/s algorithmic)")
    return out


if __name__ == "__main__":
    main()
