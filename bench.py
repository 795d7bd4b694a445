"""Throughput of the space-time HDG + lAIR-FGMRES hot path on one MI355X.

Headline workload (all at once, 2+1-D): the space-time cube [0,1]^3 split
into 96^3 cubes -> 5,308,416 tets (x1-reflected Kuhn split), p = 1 (b = 3,
31,795,200 free facet DOFs), a = (1, 0.5), nu = 1e-4, smooth solution plus a
tanh front of width 1e-2 (data from the manufactured solution).  The system
is assembled once; one step is AIR setup (block AIR on level 0, the facet
blocks as the points of the coarsening; scalar lAIR below) + FGMRES(100) to
relative residual 1e-8 (F, F, C Jacobi post-sweeps), the metric's
"setup+solve", on the assembled system resident in HBM.  The same step with
scalar AIR on every level is recorded beside it.

value = free DOFs / step time with the FP64 cycle; the FP32-cycle figure
sits beside it.  The roofline entry is the tagged kernel with the largest
total time in the timed FP64 steps: its algorithmic bytes (counted by the
library per launch) over its average launch duration, measured with HIP
events on the stream it runs on.  Secondary records: the 64-slab
slab-by-slab march (2+1-D rotating hill, 64x64 quads, p = 2) and the
differentiation form on the mapped 48^3 mesh.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# kernels timed with HIP events inside the library (ah_profile_*)
PROFILE_TAGS = ["element", "spmv0", "relax0_f", "relax0_c", "relax0_f_f32", "relax0_c_f32", "relax1_f", "relax1_c",
                "relax1_f_f32", "relax1_c_f32", "restrict0", "restrict0_f32", "rap0", "arnoldi_dot",
                "arnoldi_update"]
METRIC = "DOF/s to 1e-8 rel. residual (setup+solve), FP32 vs FP64 V-cycle; HBM GB/s"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--c3-n", type=int, default=96, help="cubes per side of the headline space-time mesh")
    ap.add_argument("--c3-nu", type=float, default=1e-4)
    ap.add_argument("--scalar-air", action="store_true",
                    help="headline with scalar AIR on level 0 instead of block AIR (the scalar figures are "
                         "recorded beside the block ones either way)")
    ap.add_argument("--no-alt-air", action="store_true",
                    help="skip the record of the other level-0 coarsening (scalar AIR, or block AIR with --scalar-air)")
    ap.add_argument("--no-c3-variants", action="store_true",
                    help="skip BiCGSTAB, ordered relaxations and nu = 0, 1e-2 on the headline mesh")
    ap.add_argument("--no-march", action="store_true", help="skip the slab-by-slab march record")
    ap.add_argument("--march-steps", type=int, default=3, help="timed passes of the slab march")
    ap.add_argument("--extras", action="store_true",
                    help="also the march's BiCGSTAB, distance-two lAIR, Section 4 thresholds, all-at-once, "
                         "internal-layer, ordered-relaxation and slab-0 adjoint records")
    ap.add_argument("--cpu-n", type=int, default=24, help="mesh of the oracle's CPU baseline sample")
    ap.add_argument("--n", type=int, default=64, help="quads per side of the march's spatial mesh")
    ap.add_argument("--slabs", type=int, default=64)
    ap.add_argument("--p", type=int, default=2)
    ap.add_argument("--nu", type=float, default=1e-4)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--solve-alone", type=int, default=0, metavar="N",
                    help="only time N FGMRES solves of slab 0 with nothing else on the GPU")
    ap.add_argument("--relax", type=int, default=0,
                    help="with --solve-alone: relaxation (0 F,F,C Jacobi; 2, 3 ordered Gauss-Seidel)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the C5 (48^3 mapped, adjoint) workload")
    ap.add_argument("--builders", type=int, default=1,
                    help="builder threads (streams) of the pipelined march")
    ap.add_argument("--no-sequential", action="store_true",
                    help="skip the sequential pass that gives the stage split")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB 10 times (HBM counter calibration)")
    ap.add_argument("--profile-summary", default=None, metavar="DIR",
                    help="only summarize the rocprofv3 CSV output found under DIR")
    ap.add_argument("--grid", type=int, default=0,
                    help="with --profile-summary: keep only dispatches of this grid size in counters")
    ap.add_argument("--traffic", nargs=7, default=None,
                    metavar=("TAG", "KERNEL_SUBSTR", "GRID", "FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR",
                             "COPY_WRITE_DIR"),
                    help="only print the HBM traffic record of one kernel from rocprofv3 --pmc FETCH_SIZE / "
                         "WRITE_SIZE runs of the bench and of --copy-probe")
    return ap.parse_args()


def _find(d, suffix):
    import glob
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    return hits[0] if hits else None


def profile_summary(d, grid=0, top=25):
    """Compact text summary of rocprofv3 --output-format csv results."""
    import csv
    from collections import defaultdict

    def key(row, *names):
        for n in names:
            if n in row:
                return row[n]
        return None
    ks = _find(d, "kernel_stats.csv")
    if ks:
        rows = list(csv.DictReader(open(ks)))
        tot = sum(float(key(r, "TotalDurationNs")) for r in rows)
        print("kernel stats: %s (total %.3f ms)" % (os.path.basename(ks), tot / 1e6))
        print("%-12s %8s %12s %10s  %s" % ("total_ms", "calls", "avg_us", "pct", "kernel"))
        for r in sorted(rows, key=lambda r: -float(key(r, "TotalDurationNs")))[:top]:
            print("%-12.3f %8s %12.2f %9.2f%%  %s" % (float(key(r, "TotalDurationNs")) / 1e6, key(r, "Calls"),
                                                       float(key(r, "AverageNs")) / 1e3,
                                                       float(key(r, "Percentage")), key(r, "Name")[:110]))
    kt = _find(d, "kernel_trace.csv")
    if kt:
        rows = list(csv.DictReader(open(kt)))
        ev = []
        for r in rows:
            t0 = int(key(r, "Start_Timestamp"))
            t1 = int(key(r, "End_Timestamp"))
            g = int(float(key(r, "Grid_Size", "Grid_Size_X") or 0))
            ev.append((t0, t1, key(r, "Kernel_Name"), g))
        ev.sort()
        if ev:
            # GPU busy time (union of dispatch intervals) over the second half
            # of the trace, which with --warmup 1 --steps 1 is the timed step
            lo = ev[0][0] + (max(e[1] for e in ev) - ev[0][0]) // 2
            busy, cur0, cur1 = 0, None, None
            for t0, t1, _, _ in ev:
                if t1 <= lo:
                    continue
                t0 = max(t0, lo)
                if cur1 is None or t0 > cur1:
                    if cur1 is not None:
                        busy += cur1 - cur0
                    cur0, cur1 = t0, t1
                else:
                    cur1 = max(cur1, t1)
            if cur1 is not None:
                busy += cur1 - cur0
            span = max(e[1] for e in ev) - lo
            print("kernel trace: %d dispatches; second half of the trace: %.3f ms span, GPU busy %.1f%%"
                  % (len(ev), span / 1e6, 100.0 * busy / max(span, 1)))
        acc = defaultdict(lambda: [0, 0])
        for t0, t1, name, g in ev:
            a = acc[(name, g)]
            a[0] += 1
            a[1] += t1 - t0
        print("%-12s %8s %12s %10s  %s" % ("total_ms", "calls", "avg_us", "grid", "kernel (by grid size)"))
        for (name, g), (n, tot) in sorted(acc.items(), key=lambda t: -t[1][1])[:top]:
            if grid and g != grid:
                continue
            print("%-12.3f %8d %12.2f %10d  %s" % (tot / 1e6, n, tot / n / 1e3, g, name[:100]))
    api = _find(d, "hip_api_stats.csv")
    if api:
        rows = list(csv.DictReader(open(api)))
        print("HIP API stats: %s" % os.path.basename(api))
        for r in sorted(rows, key=lambda r: -float(key(r, "TotalDurationNs")))[:top]:
            print("%-12.3f %8s %12.2f  %s" % (float(key(r, "TotalDurationNs")) / 1e6, key(r, "Calls"),
                                              float(key(r, "AverageNs")) / 1e3, key(r, "Name")))
    cc = _find(d, "counter_collection.csv")
    if cc:
        acc = defaultdict(lambda: [0, 0.0])
        for r in csv.DictReader(open(cc)):
            g = int(float(key(r, "Grid_Size", "Grid_Size_X") or 0))
            if grid and g != grid:
                continue
            name = key(r, "Kernel_Name")
            cn = key(r, "Counter_Name")
            a = acc[(name, cn, g)]
            a[0] += 1
            a[1] += float(key(r, "Counter_Value"))
        print("counters: %s%s" % (os.path.basename(cc), " (grid %d)" % grid if grid else ""))
        print("%-14s %8s %16s %10s  %s" % ("counter", "disp", "mean_per_disp", "grid", "kernel"))
        for (name, cn, g), (n, v) in sorted(acc.items(), key=lambda t: -t[1][1])[:top]:
            print("%-14s %8d %16.1f %10d  %s" % (cn, n, v / n, g, name[:100]))


KERNEL_SOURCES = {"element": "paper_2010_11130_amd/csrc/assemble.hip",
                  "spmv0": "paper_2010_11130_amd/csrc/solve.hip",
                  "relax0_f": "paper_2010_11130_amd/csrc/solve.hip",
                  "relax0_c": "paper_2010_11130_amd/csrc/solve.hip",
                  "relax0_f_f32": "paper_2010_11130_amd/csrc/solve.hip",
                  "relax0_c_f32": "paper_2010_11130_amd/csrc/solve.hip",
                  "relax1_f": "paper_2010_11130_amd/csrc/solve.hip",
                  "relax1_c": "paper_2010_11130_amd/csrc/solve.hip",
                  "relax1_f_f32": "paper_2010_11130_amd/csrc/solve.hip",
                  "relax1_c_f32": "paper_2010_11130_amd/csrc/solve.hip",
                  "restrict0": "paper_2010_11130_amd/csrc/solve.hip",
                  "restrict0_f32": "paper_2010_11130_amd/csrc/solve.hip",
                  "arnoldi_dot": "paper_2010_11130_amd/csrc/solve.hip",
                  "arnoldi_update": "paper_2010_11130_amd/csrc/solve.hip",
                  "rap0": "paper_2010_11130_amd/csrc/setup.hip"}
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic.json")


def _sha256(path):
    import hashlib
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), path), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _counter_mean(d, counter, substr, grid):
    """Mean per-dispatch value of ``counter`` over dispatches of kernels whose
    name contains ``substr`` (and of grid size ``grid`` if nonzero)."""
    import csv
    cc = _find(d, "counter_collection.csv")
    tot, n = 0.0, 0
    for r in csv.DictReader(open(cc)):
        if r.get("Counter_Name") != counter or substr not in r.get("Kernel_Name", ""):
            continue
        g = int(float(r.get("Grid_Size") or r.get("Grid_Size_X") or 0))
        if grid and g != grid:
            continue
        tot += float(r["Counter_Value"])
        n += 1
    return tot / n if n else None, n


def traffic_record(tag, substr, grid, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir):
    """HBM bytes per dispatch of one kernel: FETCH_SIZE and WRITE_SIZE (KiB
    per dispatch) scaled by what the same counters read for a plain device
    copy of known size (``--copy-probe``).  ``tag`` is "workload:tag"."""
    grid = int(grid)
    fk, nf = _counter_mean(fetch_dir, "FETCH_SIZE", substr, grid)
    wk, nw = _counter_mean(write_dir, "WRITE_SIZE", substr, grid)
    cf, _ = _counter_mean(copy_fetch_dir, "FETCH_SIZE", "copyBuffer", 0)
    cw, _ = _counter_mean(copy_write_dir, "WRITE_SIZE", "copyBuffer", 0)
    probe = 1024 * (1 << 20)          # bytes read and written by one --copy-probe 1024 launch
    f_fac = probe / (cf * 1024.0)
    w_fac = probe / (cw * 1024.0)
    rec = {"tag": tag, "kernel_substr": substr, "grid": grid, "dispatches": [nf, nw],
           "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk,
           "copy_probe_fetch_kib": cf, "copy_probe_write_kib": cw,
           "fetch_factor": f_fac, "write_factor": w_fac,
           "bytes_per_launch": fk * 1024.0 * f_fac + wk * 1024.0 * w_fac,
           "source": KERNEL_SOURCES[tag.split(":")[-1]],
           "source_sha256": _sha256(KERNEL_SOURCES[tag.split(":")[-1]])}
    print(json.dumps(rec))


def measured_traffic(tag):
    """Counter-measured HBM bytes per launch of ``tag`` ("workload:tag"), or
    None when no record exists or the kernel's source changed since it was
    taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            recs = json.load(f)
    except (OSError, ValueError):
        return None
    rec = recs.get(tag)
    if not rec or rec.get("source_sha256") != _sha256(rec["source"]):
        return None
    return rec["bytes_per_launch"]


def copy_probe(mib):
    """A plain device-to-device copy of known size, for scaling the FETCH_SIZE /
    WRITE_SIZE counters of the profiled kernels."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 10}))


def copy_bandwidth(mib=1024, reps=20):
    """Achieved bandwidth of a plain device-to-device copy (bytes read plus
    written per second), the practical ceiling to set beside the nominal HBM
    peak."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    return 2.0 * n * 8 / t / 1e9


def workload_inputs(v, c, prob, p, f_q=None):
    """Host mesh topology and boundary kinds, then the device inputs of
    hdg_assemble: quadrature points, boundary data (g_D on Dirichlet facets,
    u(t0) on the initial plane, 0 on the final plane), vertex velocity and
    source values."""
    import numpy as np
    import torch
    from paper_2010_11130_amd import Mesh
    from workloads import boundary_kinds
    m = Mesh(v, c)
    fv, _ = m.facets()
    bf = m.boundary_facets()
    isb = np.zeros(m.nf, dtype=bool)
    isb[bf] = True
    kinds = boundary_kinds(v, fv, isb)
    m.set_bc(kinds)
    xe, xb = m.quad_points(p)
    t = v[fv[bf]][:, :, 0]
    bot = torch.as_tensor(np.all(np.abs(t - v[:, 0].min()) <= 1e-12, axis=1), device="cuda")[:, None]
    kb = torch.as_tensor(kinds[bf], device="cuda")[:, None]
    g = torch.where(kb == 1, prob.g_dirichlet(xb),
                    torch.where(bot, prob.g_neumann(xb, True), prob.g_neumann(xb, False))).contiguous()
    a = torch.as_tensor(np.ascontiguousarray(prob.a_vertices(v)), device="cuda")
    if f_q is None:
        f_q = prob.f(xe).contiguous()
    elif f_q is False:
        f_q = None
    return m, xe, g, a, f_q


def c3_inputs(n, nu):
    """Mesh, device inputs and the assembled C3 system (96^3 Kuhn cubes of
    the space-time cube, p = 1, a = (1, 0.5), smooth solution plus a tanh
    front), with the assembly time."""
    import torch
    from paper_2010_11130_amd import System
    from workloads import kuhn_cube_mesh
    from workloads.problems import SmoothPlusFront
    v, c = kuhn_cube_mesh(n)
    m, xe, g, a, _ = workload_inputs(v, c, SmoothPlusFront(nu), 1, f_q=False)
    f = SmoothPlusFront(nu).f(xe).contiguous()
    t = []
    s = None
    for _ in range(2):
        del s
        s = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = System(m, 1, nu, a, f, g, keep=False)
        torch.cuda.synchronize()
        t.append(time.perf_counter() - t0)
    return {"mesh": m, "xe": xe, "g": g, "a": a, "f": f, "system": s, "assemble_ms": 1e3 * t[-1],
            "tets": c.shape[0]}


def setup_solve_steps(s, steps, warmup, tol, precision=0, profile=False, method=0, **air):
    """``warmup`` untimed, then ``steps`` timed passes of lAIR setup + Krylov
    solve on the assembled system ``s`` (each pass builds its own hierarchy
    and solver workspace); with ``profile`` the library's per-kernel HIP
    events are on during the timed passes."""
    import torch
    from paper_2010_11130_amd import Hierarchy, lib
    kw = dict(air)
    kw["fp32_cycle"] = 1 if precision else 0
    for _ in range(warmup):
        h = Hierarchy(s, **kw)
        h.solve(tol=tol, precision=precision, method=method)
        del h
    if profile:
        lib().ah_profile_reset()
        lib().ah_profile_enable(1)
    torch.cuda.synchronize()
    setup, solve, iters = [], [], []
    x = info = h = None
    T0 = time.perf_counter()
    for _ in range(steps):
        del h, x
        t0 = time.perf_counter()
        h = Hierarchy(s, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, info = h.solve(tol=tol, precision=precision, method=method)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        setup.append(1e3 * (t1 - t0))
        solve.append(1e3 * (t2 - t1))
        iters.append(info["iters"])
    T = (time.perf_counter() - T0) / steps
    prof = None
    if profile:
        lib().ah_profile_enable(0)
        prof = profile_totals(PROFILE_TAGS)
        lib().ah_profile_reset()
    med = lambda v: sorted(v)[len(v) // 2]
    rec = {"value": s.n / T, "ms_per_step": 1e3 * T, "setup_ms_median": med(setup), "solve_ms_median": med(solve),
           "iters": iters[-1], "converged": info["converged"], "true_relres": info["true_relres"],
           "levels": h.info["levels"], "op_complexity": h.info["op_complexity"]}
    if air.get("relax", 0) >= 2:
        rec["flow_order_levels"] = h.flow_levels()[1]
    return rec, prof, x


def setup_warm_solve(s, tol, precision=0, method=0, **air):
    """lAIR setup, a first solve (which also allocates the solver workspace
    from the stream-ordered pool; after many differently sized objects the
    pool may map new memory for it) and a second, timed solve on the same
    hierarchy: setup + warm solve."""
    import torch
    from paper_2010_11130_amd import Hierarchy
    kw = dict(air)
    kw["fp32_cycle"] = 1 if precision else 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = Hierarchy(s, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    h.solve(tol=tol, precision=precision, method=method)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    x, info = h.solve(tol=tol, precision=precision, method=method)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    rec = {"value": s.n / ((t1 - t0) + (t3 - t2)), "setup_ms": 1e3 * (t1 - t0), "solve_ms": 1e3 * (t3 - t2),
           "first_solve_ms": 1e3 * (t2 - t1), "iters": info["iters"], "converged": info["converged"],
           "true_relres": info["true_relres"], "levels": h.info["levels"]}
    if air.get("relax", 0) >= 2:
        rec["flow_order_levels"] = h.flow_levels()[1]
    del h
    return rec, x


def c3_variants(c3, tol, x64, air):
    """Setup + warm solve of other settings on the same 96^3 workload, with
    the headline's level-0 coarsening ``air``: strength threshold 0.5 (also
    with 0.25 for the restriction neighbourhoods, FP64 and FP32 cycle), the
    Section 4 thresholds (0.2 for the coarsening, 0.3 for the restriction),
    BiCGSTAB (the paper's Krylov method), the ordered Gauss-Seidel
    relaxations of Lemma 3.1 (relax 2: all points in flow order; relax 3: F
    points then all points, the Section 4 schedule), FP64 and FP32 cycles,
    and relax 2 with the other coarsening; the same mesh at nu = 0 and
    nu = 1e-2, both coarsenings."""
    import torch
    from paper_2010_11130_amd import System
    from workloads.problems import SmoothPlusFront
    s = c3["system"]
    other = {} if air else {"block_air": 1}
    oname = "scalar" if air else "block"
    out = {}
    for key, prec, kw in (("theta_0.5", 0, {"theta": 0.5}),
                          ("theta_0.5_theta_r_0.25", 0, {"theta": 0.5, "theta_r": 0.25}),
                          ("theta_0.5_theta_r_0.25_fp32_cycle", 1, {"theta": 0.5, "theta_r": 0.25}),
                          ("section4_theta_0.2_theta_r_0.3", 0, {"theta": 0.2, "theta_r": 0.3}),
                          ("bicgstab", 0, {"method": 1}),
                          ("ordered_relax2", 0, {"relax": 2}), ("ordered_relax2_fp32_cycle", 1, {"relax": 2}),
                          ("ordered_relax3", 0, {"relax": 3}),
                          (oname + "_ordered_relax2", 0, dict(other, relax=2))):
        kw = dict(air, **kw) if not key.startswith(oname) else kw
        r, x = setup_warm_solve(s, tol, prec, **kw)
        r["rel_diff_vs_headline_fp64"] = (torch.linalg.norm(x - x64) / torch.linalg.norm(x64)).item()
        out[key] = r
        del x
    # nu = 1e-2: scalar AIR at theta 0.25 does not converge in 1000 iterations
    v12 = ((("jacobi", air), ("scalar_jacobi_theta_0.1", {"theta": 0.1})) if air else
           (("jacobi_theta_0.1", {"theta": 0.1}), ("block_jacobi", other)))
    for nu, variants in ((0.0, (("jacobi", air), (oname + "_jacobi", other), ("ordered_relax2", dict(air, relax=2)))),
                         (1e-2, v12)):
        prob = SmoothPlusFront(nu)
        f = prob.f(c3["xe"]).contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sn = System(c3["mesh"], 1, nu, c3["a"], f, c3["g"], keep=False)
        torch.cuda.synchronize()
        rec = {"assemble_ms": 1e3 * (time.perf_counter() - t0)}
        for key, kw in variants:
            r, x = setup_warm_solve(sn, tol, 0, **kw)
            rec[key] = r
            del x
        out["nu=%g" % nu] = rec
        del sn
    return out


def c4_record(args):
    """The precision form on the C2 slab shapes (64 slabs of 342,528 DOFs,
    p = 2, rotating hill) at nu = 0 and 1e-4: the pipelined march with the
    FP64 and the FP32 cycle, FGMRES iterations per slab, and the FP32-cycle
    solution's difference from the FP64 one on the last slab (the FP64 slab
    solve matches the FP64 oracle in the full-slab tests)."""
    import torch
    out = {}
    for nu in (0.0, 1e-4):
        march = March(args.n, args.slabs, args.p, nu)
        march.builders = args.builders
        rec = {}
        last = {}
        for prec in (0, 1):
            march.step(prec, args.tol)
            torch.cuda.synchronize()
            its = []
            t0 = time.perf_counter()
            for _ in range(args.march_steps):
                lam, _ = march.step(prec, args.tol, iters=its)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.march_steps
            last[prec] = lam
            rec["fp64" if prec == 0 else "fp32_cycle"] = {
                "value": args.slabs * lam.numel() / dt, "ms_per_step": 1e3 * dt,
                "fgmres_iters_per_slab": {"min": min(its), "max": max(its), "mean": sum(its) / len(its)}}
        rec["fp32_cycle"]["rel_diff_vs_fp64_last_slab"] = (torch.linalg.norm(last[1] - last[0]) /
                                                           torch.linalg.norm(last[0])).item()
        rec["fp32_cycle"]["speedup_vs_fp64"] = rec["fp64"]["ms_per_step"] / rec["fp32_cycle"]["ms_per_step"]
        out["nu=%g" % nu] = rec
        del march
    return out


def c1_record(n=16, p=1, nu=1e-4, tol=1e-10, steps=20):
    """The C1 problem (1+1D, (0,1)^2 as n x n quads -> 2 n^2 triangles, p = 1,
    a = 1, manufactured u = sin 2 pi (x - t) e^-t, 1,536 free DOFs at n = 16):
    assembly, then setup + solve to 1e-10 timed over ``steps`` passes, FP64
    and FP32 cycles.  Latency bound (a few thousand unknowns): no roofline
    claim."""
    import torch
    from paper_2010_11130_amd import System
    from workloads import square_tri_mesh
    from workloads.problems import C1Advection1D
    prob = C1Advection1D(nu)
    v, c = square_tri_mesh(n)
    m, xe, g, a, f = workload_inputs(v, c, prob, p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = System(m, p, nu, a, f, g, keep=False)
    torch.cuda.synchronize()
    out = {"mesh": "%dx%d quads -> %d triangles" % (n, n, c.shape[0]), "p": p, "free_dofs": s.n,
           "assemble_ms": 1e3 * (time.perf_counter() - t0)}
    for prec in (0, 1):
        r, _, x = setup_solve_steps(s, steps, 2, tol, prec)
        out["fp64" if prec == 0 else "fp32_cycle"] = {k: r[k] for k in ("value", "ms_per_step", "setup_ms_median",
                                                                        "solve_ms_median", "iters", "levels")}
        del x
    return out


def c5_adjoint(tol):
    """The C5 workload: the 48^3 Kuhn mesh mapped by the time-dependent
    domain map (663,552 tets, p = 2, 7.9M free DOFs), 256 Gaussian sources,
    nu = 1e-3: assembly with the element data kept, lAIR setup with the
    transposed operators, the forward FGMRES solve, the adjoint solve of the
    misfit J = |Lambda|^2 / 2 and the gradients with respect to the source
    values and nu; FP64 and FP32 cycles, and with strength threshold 0.5
    for the coarsening (also with 0.25 for the restriction neighbourhoods):
    the facet couplings are diffusion-dominated here (tau = nu alpha / h_K
    exceeds |a|)."""
    import torch
    from paper_2010_11130_amd import System, Hierarchy, source_gauss
    from workloads import kuhn_cube_mesh, map_vertices_c5
    from workloads.problems import GaussianSources, c5_sources
    centers, _, c0 = c5_sources(256)
    prob = GaussianSources(1e-3, centers, c0)
    v, c = kuhn_cube_mesh(48)
    v = map_vertices_c5(v)
    m, xe, g, a, _ = workload_inputs(v, c, prob, 2, f_q=False)
    f = source_gauss(xe.reshape(-1, 3), centers, prob.width, c0).reshape(xe.shape[:-1]).contiguous()
    out = {"mesh": "48^3 Kuhn cubes mapped, 663552 tets", "p": 2, "nu": 1e-3}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = System(m, 2, prob.nu, a, f, g, keep=True)
    torch.cuda.synchronize()
    out["assemble_ms"] = 1e3 * (time.perf_counter() - t0)
    out["free_dofs"] = s.n
    for prec, theta, theta_r, key in ((0, 0.25, 0.0, "fp64"), (1, 0.25, 0.0, "fp32_cycle"),
                                      (0, 0.5, 0.0, "fp64_theta_0.5"),
                                      (0, 0.5, 0.25, "fp64_theta_0.5_theta_r_0.25"),
                                      (1, 0.5, 0.25, "fp32_cycle_theta_0.5_theta_r_0.25")):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        h = Hierarchy(s, adjoint=1, fp32_cycle=prec, theta=theta, theta_r=theta_r)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        # a first forward and adjoint solve allocate the FGMRES basis
        x, _ = h.solve(tol=tol, precision=prec)
        h.solve_adjoint(x, tol=tol, precision=prec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, fi = h.solve(tol=tol, precision=prec)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        lam, ai = h.solve_adjoint(x, tol=tol, precision=prec)
        torch.cuda.synchronize()
        td = time.perf_counter()
        s.grad(x, lam)
        torch.cuda.synchronize()
        te = time.perf_counter()
        out[key] = {
            "setup_ms": 1e3 * (tb - ta), "forward_ms": 1e3 * (tc - t1), "adjoint_ms": 1e3 * (td - tc),
            "gradient_ms": 1e3 * (te - td), "first_forward_and_adjoint_ms": 1e3 * (t1 - tb),
            "forward_iters": fi["iters"], "adjoint_iters": ai["iters"],
            "converged": fi["converged"] and ai["converged"],
            "dofs_per_s_setup_forward_adjoint": s.n / ((tb - ta) + (td - t1))}
        del h, x, lam
    return out


class March:
    """Device-resident inputs of the slab march and one step of it."""

    def __init__(self, n, slabs, p, nu):
        import numpy as np
        import torch
        from paper_2010_11130_amd import Mesh
        from workloads import slab_prism_tet_mesh, boundary_kinds
        from workloads.problems import slab_hill
        self.np, self.torch = np, torch
        self.dt = 1.0 / slabs
        self.slabs, self.p = slabs, p
        self.prob = slab_hill(nu)
        v, c = slab_prism_tet_mesh(n, self.dt)
        self.vert, self.cell = v, c
        m = Mesh(v, c)
        fv, _ = m.facets()
        bf = m.boundary_facets()
        isb = np.zeros(m.nf, dtype=bool)
        isb[bf] = True
        kinds = boundary_kinds(v, fv, isb)
        m.set_bc(kinds)
        self.mesh = m
        _, xb = m.quad_points(p)
        tb = v[fv[bf]][:, :, 0]
        bot = torch.as_tensor(np.all(np.abs(tb) <= 1e-12, axis=1), device="cuda")[:, None]
        kb = torch.as_tensor(kinds[bf], device="cuda")[:, None]
        g = []
        for k in range(slabs):
            x = xb.clone()
            x[..., 0] += k * self.dt
            u = self.prob.u(x)
            g.append(torch.where(kb == 1, u, torch.where(bot, u, torch.zeros_like(u))))
        self.g = torch.stack(g).contiguous()
        self.a = torch.as_tensor(self.prob.a(v), device="cuda").contiguous()
        self.nu = nu
        self.builders = 1
        torch.cuda.synchronize()

    def step(self, precision, tol, pipelined=True, stages=None, method=0, iters=None, air_extra=None):
        """One pass of the march over all slabs: per slab assembly, lAIR
        setup, the Krylov solve to ``tol`` (FGMRES, or BiCGSTAB with
        method=1) and reconstruction of u_h."""
        from paper_2010_11130_amd import SlabMarch
        out = {}

        def keep_u(k, s, h, x, info):
            out["U"] = s.reconstruct(x)
            if iters is not None:
                iters.append(info["iters"])

        air_kw = {"fp32_cycle": 1 if precision else 0}
        air_kw.update(air_extra or {})
        m = SlabMarch(self.mesh, self.p, self.nu, self.a, air_kw=air_kw,
                      solve_kw={"tol": tol, "precision": precision, "method": method}, builders=self.builders)
        s, x, info = m.run([self.g[k] for k in range(self.slabs)], pipelined=pipelined, on_slab=keep_u,
                           stages=stages)
        self.torch.cuda.synchronize()
        self.wait_s = getattr(self, "wait_s", 0.0) + getattr(m, "wait_s", 0.0)
        return x, out["U"]


def profile_totals(tags):
    import ctypes as C
    from paper_2010_11130_amd import lib
    out = {}
    for t in tags:
        n, ms, by = C.c_int64(), C.c_double(), C.c_double()
        lib().ah_profile_read(t.encode(), C.byref(n), C.byref(ms), C.byref(by))
        if n.value:
            out[t] = {"launches": n.value, "total_ms": ms.value, "bytes": by.value,
                      "avg_us": 1e3 * ms.value / n.value,
                      "gbs": by.value / (ms.value * 1e-3) / 1e9 if ms.value > 0 else 0.0}
    return out


def run_timed(march, precision, steps, warmup, tol, sequential=True):
    """Pipelined march: ``warmup`` untimed passes, then ``steps`` timed ones
    with the library's per-kernel HIP-event timing on.  Then one sequential
    pass for the stage split (assembly / setup / solve)."""
    import torch
    from paper_2010_11130_amd import lib
    for _ in range(warmup):
        march.step(precision, tol)
    lib().ah_profile_reset()
    lib().ah_profile_enable(1)
    torch.cuda.synchronize()
    march.wait_s = 0.0
    t0 = time.perf_counter()
    last = None
    for _ in range(steps):
        last = march.step(precision, tol)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # time the solving thread spent waiting for the builder, per step
    march.wait_ms_per_step = 1e3 * march.wait_s / steps
    lib().ah_profile_enable(0)
    prof = profile_totals(PROFILE_TAGS)
    lib().ah_profile_reset()
    if not sequential:
        return (t1 - t0) / steps, None, None, prof, last
    stages = []
    t2 = time.perf_counter()
    march.step(precision, tol, pipelined=False, stages=stages)
    t3 = time.perf_counter()
    return (t1 - t0) / steps, stages, t3 - t2, prof, last


def all_at_once(args, U_march_last):
    """The stacked slabs as one space-time system (Section 2.2): assembly,
    lAIR setup, FGMRES to the same tolerance and reconstruction, timed after
    the mesh and boundary data are on the device (one warm-up run)."""
    import numpy as np
    import torch
    from paper_2010_11130_amd import Mesh, System, Hierarchy
    from workloads import stacked_prism_tet_mesh, boundary_kinds
    from workloads.problems import slab_hill
    prob = slab_hill(args.nu)
    v, c = stacked_prism_tet_mesh(args.n, args.slabs, T=1.0)
    m = Mesh(v, c)
    fv, _ = m.facets()
    bf = m.boundary_facets()
    isb = np.zeros(m.nf, dtype=bool)
    isb[bf] = True
    kinds = boundary_kinds(v, fv, isb)
    m.set_bc(kinds)
    _, xb = m.quad_points(args.p)
    tb = v[fv[bf]][:, :, 0]
    bot = torch.as_tensor(np.all(np.abs(tb) <= 1e-12, axis=1), device="cuda")[:, None]
    kb = torch.as_tensor(kinds[bf], device="cuda")[:, None]
    u = prob.u(xb)
    g = torch.where(kb == 1, u, torch.where(bot, u, torch.zeros_like(u))).contiguous()
    a = torch.as_tensor(prob.a(v), device="cuda").contiguous()
    res = None
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = System(m, args.p, args.nu, a, None, g)
        h = Hierarchy(s)
        x, info = h.solve(tol=args.tol)
        U = s.reconstruct(x)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        res = (s, h, x, info, U, t)
    s, h, x, info, U, t = res
    ne_slab = 6 * args.n * args.n
    Ul = U[(args.slabs - 1) * ne_slab:]
    diff = (torch.linalg.norm(Ul - U_march_last) / torch.linalg.norm(U_march_last)).item()
    # the same system with BiCGSTAB (the paper's Krylov method): no growing
    # orthogonalisation basis
    bres = None
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sb = System(m, args.p, args.nu, a, None, g)
        hb = Hierarchy(sb)
        xb_, infob = hb.solve(tol=args.tol, method=1)
        sb.reconstruct(xb_)
        torch.cuda.synchronize()
        bres = (sb, infob, time.perf_counter() - t0)
        del hb
    sb, infob, tb_ = bres
    return {"value": s.n / t, "unit": "DOF/s", "ms": 1e3 * t, "free_dofs": s.n, "iters": info["iters"],
            "levels": h.info["levels"], "last_slab_rel_diff_vs_march": diff,
            "bicgstab": {"value": sb.n / tb_, "ms": 1e3 * tb_, "steps": infob["iters"]}}


def solve_alone(march, repeats, tol, precision=0, relax=0):
    """Slab 0 of the march assembled and set up once, then ``repeats``
    FGMRES solves (V-cycle in FP64, or FP32 with ``precision=1``) with nothing
    else on the GPU: the solve's kernels without the builder's competition
    (per-kernel HIP-event averages included); ``relax`` selects the
    relaxation (2, 3: ordered Gauss-Seidel on level 0)."""
    import torch
    from paper_2010_11130_amd import System, Hierarchy, lib
    s = System(march.mesh, march.p, march.nu, march.a, None, march.g[0])
    h = Hierarchy(s, fp32_cycle=1 if precision else 0, relax=relax)
    for _ in range(3):
        h.solve(tol=tol, precision=precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = 0
    for _ in range(repeats):
        _, info = h.solve(tol=tol, precision=precision)
        its += info["iters"]
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    # a second pass with the per-kernel HIP events on
    lib().ah_profile_reset()
    lib().ah_profile_enable(1)
    for _ in range(repeats):
        h.solve(tol=tol, precision=precision)
    torch.cuda.synchronize()
    lib().ah_profile_enable(0)
    prof = profile_totals(PROFILE_TAGS + ["gs0", "gs0_f"])
    lib().ah_profile_reset()
    return {"free_dofs": s.n, "repeats": repeats, "ms_per_solve": 1e3 * t / repeats,
            "us_per_iteration": 1e6 * t / its, "iters": its // repeats, "kernels": prof}


def internal_layer(n=48, p=1, tol=1e-8, air=None):
    """The moving internal layer of Section 4.2 (nu = 0, discontinuous exact
    solution) on the uniform n^3 Kuhn mesh of the space-time unit cube, all
    at once: assembly, lAIR setup (parameters ``air``), FGMRES and
    reconstruction, timed after one warm-up run with the mesh and boundary
    data on the device."""
    import numpy as np
    import torch
    from paper_2010_11130_amd import Mesh, System, Hierarchy
    from workloads import kuhn_cube_mesh, boundary_kinds
    from workloads.problems import MovingInternalLayer
    prob = MovingInternalLayer()
    v, c = kuhn_cube_mesh(n)
    m = Mesh(v, c)
    fv, _ = m.facets()
    bf = m.boundary_facets()
    isb = np.zeros(m.nf, dtype=bool)
    isb[bf] = True
    kinds = boundary_kinds(v, fv, isb)
    m.set_bc(kinds)
    _, xb = m.quad_points(p)
    kb = torch.as_tensor(kinds[bf], device="cuda")[:, None]
    # Dirichlet: the exact solution; initial plane: u(0) = 0; final plane: 0
    g = torch.where(kb == 1, prob.u(xb), torch.zeros_like(xb[..., 0])).contiguous()
    a = torch.as_tensor(prob.a(v), device="cuda").contiguous()
    res = None
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = System(m, p, 0.0, a, None, g)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        h = Hierarchy(s, **(air or {}))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        x, info = h.solve(tol=tol)
        s.reconstruct(x)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        res = (s, h, info, t3 - t0, t1 - t0, t2 - t1, t3 - t2)
    s, h, info, t, ta, tsu, tso = res
    out = {"value": s.n / t, "unit": "DOF/s", "ms": 1e3 * t, "mesh": "%d^3 Kuhn cubes, %d tets" % (n, 6 * n ** 3),
           "p": p, "free_dofs": s.n, "iters": info["iters"], "levels": h.info["levels"],
           "op_complexity": h.info["op_complexity"],
           "stages_ms": {"assemble": 1e3 * ta, "setup": 1e3 * tsu, "solve_and_reconstruct": 1e3 * tso}}
    if air and air.get("relax", 0) >= 2:
        _, rounds, breaks = h.flow_levels()
        out["flow_order"] = {"rounds": rounds, "cycle_breaks": breaks}
    return out


def adjoint_slab(march, tol, repeats=3):
    """The differentiation form on slab 0 of the march: lAIR setup with the
    transposed operators, the forward FGMRES solve, the adjoint solve
    S^T lam = dJ/dLambda of the misfit J = |Lambda|^2 / 2 with the transposed
    cycle, and the gradients dJ/df (at the element quadrature points) and
    dJ/dnu; FP64 and FP32 cycles."""
    import torch
    from paper_2010_11130_amd import System, Hierarchy
    s = System(march.mesh, march.p, march.nu, march.a, None, march.g[0])
    out = {"free_dofs": s.n}
    for prec in (0, 1):
        Hierarchy(s, adjoint=1, fp32_cycle=prec).solve(tol=tol, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = Hierarchy(s, adjoint=1, fp32_cycle=prec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tf = ta = tg = 0.0
        for _ in range(repeats):
            ta0 = time.perf_counter()
            x, fi = h.solve(tol=tol, precision=prec)
            torch.cuda.synchronize()
            ta1 = time.perf_counter()
            lam, ai = h.solve_adjoint(x, tol=tol, precision=prec)
            torch.cuda.synchronize()
            ta2 = time.perf_counter()
            s.grad(x, lam)
            torch.cuda.synchronize()
            ta3 = time.perf_counter()
            tf, ta, tg = tf + ta1 - ta0, ta + ta2 - ta1, tg + ta3 - ta2
        out["fp64" if prec == 0 else "fp32_cycle"] = {
            "setup_ms": 1e3 * (t1 - t0), "forward_ms": 1e3 * tf / repeats, "adjoint_ms": 1e3 * ta / repeats,
            "gradient_ms": 1e3 * tg / repeats, "forward_iters": fi["iters"], "adjoint_iters": ai["iters"],
            "adjoint_converged": ai["converged"]}
    return out


def ordered_slab(s, relax, tol, repeats=3):
    """lAIR setup and FGMRES solves of one assembled slab with the given
    relaxation (0: F,F,C Jacobi; 2, 3: ordered Gauss-Seidel on level 0),
    plus the per-sweep time of the ordered sweeps from the HIP events."""
    import torch
    from paper_2010_11130_amd import Hierarchy, lib
    Hierarchy(s, relax=relax).solve(tol=tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = Hierarchy(s, relax=relax)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    its = 0
    for _ in range(repeats):
        _, info = h.solve(tol=tol)
        its += info["iters"]
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out = {"iters": its // repeats, "setup_ms": 1e3 * (t1 - t0), "solve_ms": 1e3 * (t2 - t1) / repeats,
           "dofs_per_s_setup_solve": s.n / ((t1 - t0) + (t2 - t1) / repeats)}
    if relax >= 2:
        _, rounds, breaks = h.flow_levels()
        out["flow_order"] = {"rounds": rounds, "cycle_breaks": breaks}
        lib().ah_profile_reset()
        lib().ah_profile_enable(1)
        h.solve(tol=tol)
        torch.cuda.synchronize()
        lib().ah_profile_enable(0)
        out["sweeps"] = profile_totals(["gs0", "gs0_f"])
        for v in out["sweeps"].values():
            v["us_per_level"] = v["avg_us"] / rounds
        lib().ah_profile_reset()
    return out


def ordered_relaxation(args, march):
    """Ordered Gauss-Seidel in the flow order of Lemma 3.1 against F,F,C
    Jacobi: the moving internal layer (nu = 0: one ordered sweep inverts level
    0) all at once, and slab 0 of the march."""
    from paper_2010_11130_amd import System
    out = {}
    for relax in (2, 3):
        out["internal_layer_relax%d" % relax] = internal_layer(tol=args.tol, air={"relax": relax})
    s0 = System(march.mesh, args.p, args.nu, march.a, None, march.g[0])
    for relax in (0, 2, 3):
        out["slab0_relax%d" % relax] = ordered_slab(s0, relax, args.tol)
    return out


def element_flops(D, p):
    """Algorithmic FP64 flops of one space-time element (the element kernel):
    the quadrature sums of A, B, C, the diagonal facet blocks of D and F
    (Section 2.3, conical-product rule with p+2 points per direction), the
    LU of A, the solves A^-1 [B | F | I] and the Schur complement
    D - C A^-1 B with C A^-1 F (Section 2.5).  Counted per entry and
    quadrature point as multiply + add pairs; basis tabulation excluded."""
    from math import comb
    nu = comb(p + D, D)
    b = comb(p + D - 1, D - 1)
    nl = (D + 1) * b
    nq = (p + 2) ** D
    nqf = (p + 2) ** (D - 1)
    vol = nq * (2 * (D - 1) * (D + 1) + 2 * D * D)          # velocity and J^-T a per point
    vol += nq * nu * (2 * D + 2 * D * (D - 1))               # advective derivative, spatial gradient
    vol += nu * nu * nq * (2 * (D - 1) + 5)                  # A: advection + diffusion
    vol += nu * nq * 3                                       # F
    fac = (D + 1) * nqf * (9 * nu * nu + 7 * nu * b * 2 + 3 * b * b)   # A, B, C, D facet terms
    cond = 2 * nu ** 3 // 3 + (nl + 1 + nu) * 2 * nu * nu + (nl * nl + nl) * 2 * nu
    return vol + fac + cond


def roofline(prof, workload, p, D, ne):
    """Roofline entry of the tagged kernel with the largest total time: the
    element kernel against FP64 vector peak (flops above), the sparse and
    Arnoldi kernels against HBM bandwidth (algorithmic bytes counted by the
    library per launch)."""
    name = max(prof, key=lambda k: prof[k]["total_ms"])
    k = prof[name]
    sec = k["avg_us"] * 1e-6
    traffic = measured_traffic("%s:%s" % (workload, name))
    if name == "element":
        flops = element_flops(D, p) * ne
        ach = flops / sec / 1e12
        return {"kernel": name, "bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / FP64_PEAK_TFLOPS, "traffic": traffic, "flops_per_launch": flops,
                "avg_launch_us": k["avg_us"]}
    ach = k["bytes"] / k["launches"] / sec / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
            "bytes_per_launch": k["bytes"] / k["launches"], "avg_launch_us": k["avg_us"],
            "launches": k["launches"]}


def cpu_baseline(n=24, nu=1e-4, tol=1e-8, block_air=True):
    """The oracle (plain FP64 numpy/scipy) on a bounded sample of the
    headline workload's mesh family: the n^3 Kuhn mesh of the same problem,
    p = 1, the headline's level-0 coarsening.  value = free DOFs / (AIR
    setup + FGMRES) as in the headline, with the BLAS thread pools held at
    one thread (the oracle's sparse products and loops run on one core
    anyway); ``all_cores`` repeats setup + FGMRES on the same system with
    the pools left at their default size (the thread count they report).
    Assembly timed apart."""
    from workloads import kuhn_cube_mesh
    from workloads.problems import SmoothPlusFront
    from oracle.drivers import setup_problem
    from oracle import air, krylov
    try:
        import threadpoolctl
    except Exception:
        threadpoolctl = None

    def setup_solve(s):
        t1 = time.perf_counter()
        H = air.setup(s.Shat, block_air=block_air, block=s.b)
        t2 = time.perf_counter()
        x, info = krylov.fgmres(s.Shat, s.Hhat, lambda r: air.vcycle(H, r), tol=tol)
        t3 = time.perf_counter()
        return t2 - t1, t3 - t2, info["iters"]

    limiter = threadpoolctl.threadpool_limits(limits=1) if threadpoolctl else None
    v, c = kuhn_cube_mesh(n)
    t0 = time.perf_counter()
    s = setup_problem(v, c, SmoothPlusFront(nu), 1)
    ta = time.perf_counter() - t0
    ts, tf, it = setup_solve(s)
    if limiter is not None:
        limiter.unregister()
    threads = max([p.get("num_threads", 1) for p in threadpoolctl.threadpool_info()] or [1]) if threadpoolctl else None
    ts_all, tf_all, it_all = setup_solve(s)
    return {"value": s.n / (ts + tf), "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "sample": "%d^3 Kuhn mesh of the headline problem (p=1, nu=%g, %d free DOFs, 1/%d of the headline's): "
                      "%s setup %.1f s + FGMRES to %g %.1f s (%d iterations), one thread; assembly %.1f s apart"
                      % (n, nu, s.n, round(31795200 / s.n), "block AIR" if block_air else "lAIR", ts, tol,
                         tf, it, ta),
            "all_cores": {"value": s.n / (ts_all + tf_all), "unit": "DOF/s", "threads": threads,
                          "setup_s": ts_all, "fgmres_s": tf_all, "iters": it_all,
                          "note": "the same setup + FGMRES with the BLAS pools at their default size; the sparse "
                                  "products and Python loops stay on one core"}}


def march_record(args):
    """The slab-by-slab march (secondary record): pipelined FP64 and FP32-cycle
    marches, the sequential stage split, and the slab solved alone; with
    ``--extras`` the other march and slab-0 records."""
    import torch
    march = March(args.n, args.slabs, args.p, args.nu)
    march.builders = args.builders
    seq = not args.no_sequential
    steps, warmup = args.march_steps, 1
    t64, stages64, tseq64, prof64, last64 = run_timed(march, 0, steps, warmup, args.tol, seq)
    ndof_slab = last64[0].numel()
    total = ndof_slab * args.slabs

    def split(stages, tseq):
        if stages is None:
            return {}
        st = {k: 1e3 * sum(x[k] for x in stages) for k in ("assemble", "setup", "solve")}
        iters = [x["iters"] for x in stages]
        return {"stages_ms_per_step": st,
                "sequential_march": {"dofs_per_s": total / tseq, "ms_per_step": 1e3 * tseq},
                "setup_solve_dofs_per_s": total / (1e-3 * (st["setup"] + st["solve"])),
                "fgmres_iters_per_slab": {"min": min(iters), "max": max(iters), "mean": sum(iters) / len(iters)}}

    out = {"value": total / t64, "unit": "DOF/s", "ms_per_step": 1e3 * t64, "steps": steps,
           "workload": "slab-by-slab 2+1D rotating Gaussian hill: %dx%d quads -> %d tets/slab, %d slabs dt=1/%d, "
                       "p=%d, nu=%g, lAIR-FGMRES to %g per slab; per slab assembly + lAIR setup + solve + "
                       "reconstruction, the next slab's assembly and setup overlapped with the current solve on a "
                       "second stream" % (args.n, args.n, 6 * args.n * args.n, args.slabs, args.slabs, args.p,
                                          args.nu, args.tol),
           "free_dofs_per_slab": ndof_slab, "total_free_dofs": total, "kernels": prof64,
           "build_wait_ms_per_step": march.wait_ms_per_step}
    if stages64:
        out["levels"] = stages64[0]["levels"]
        out["op_complexity"] = stages64[0]["op_complexity"]
    out.update(split(stages64, tseq64))
    alone64 = None
    if not args.no_fp32:
        t32, stages32, tseq32, prof32, last32 = run_timed(march, 1, steps, warmup, args.tol, seq)
        err = (torch.linalg.norm(last32[0] - last64[0]) / torch.linalg.norm(last64[0])).item()
        out["fp32_cycle"] = {"value": total / t32, "ms_per_step": 1e3 * t32, "speedup_vs_fp64": t64 / t32,
                             "last_slab_rel_diff_vs_fp64": err, "kernels": prof32,
                             "build_wait_ms_per_step": march.wait_ms_per_step}
        out["fp32_cycle"].update(split(stages32, tseq32))
        a64 = alone64 = solve_alone(march, 10, args.tol, 0)
        a32 = solve_alone(march, 10, args.tol, 1)
        out["fp32_cycle"]["solve_alone"] = {
            "fp64_ms_per_solve": a64["ms_per_solve"], "fp32_ms_per_solve": a32["ms_per_solve"],
            "fp64_us_per_iteration": a64["us_per_iteration"], "fp32_us_per_iteration": a32["us_per_iteration"],
            "iters": [a64["iters"], a32["iters"]], "speedup_vs_fp64": a64["ms_per_solve"] / a32["ms_per_solve"]}
    if prof64:
        # the slab's level-0 operator (about 84 MB) stays in the 256 MB
        # Infinity Cache: a cache-resident figure, not an HBM one
        rf = roofline(prof64, "c2", args.p, march.vert.shape[1], march.cell.shape[0])
        rf["note"] = "cache-resident working set (level-0 operator about 84 MB < 256 MB Infinity Cache)"
        k = (alone64 or {}).get("kernels", {}).get(rf["kernel"])
        if k:
            ach = k["bytes"] / k["launches"] / (k["avg_us"] * 1e-6) / 1e9
            rf["alone"] = {"avg_launch_us": k["avg_us"], "achieved": ach, "frac": ach / HBM_PEAK_GBS}
        out["roofline"] = rf
    if args.extras:
        from paper_2010_11130_amd import System, Hierarchy
        march.step(0, args.tol, method=1)
        its = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            its.clear()
            march.step(0, args.tol, method=1, iters=its)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / steps
        out["bicgstab"] = {"value": total / tb, "ms_per_step": 1e3 * tb,
                           "steps_per_slab": {"min": min(its), "max": max(its), "mean": sum(its) / len(its)}}
        s0 = System(march.mesh, args.p, args.nu, march.a, None, march.g[0], block_scale=False)
        x0, i0 = Hierarchy(s0).solve(tol=args.tol, maxit=100)
        out["no_block_inverse_slab0"] = {"converged": i0["converged"], "iters": i0["iters"],
                                         "relres": i0["true_relres"]}
        for key, extra in (("lair_distance2", {"lair_distance": 2}),
                           ("paper_thresholds", {"theta": 0.2, "theta_r": 0.3})):
            march.step(0, args.tol, air_extra=extra)
            its = []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                its.clear()
                march.step(0, args.tol, iters=its, air_extra=extra)
            torch.cuda.synchronize()
            td = (time.perf_counter() - t0) / steps
            out[key] = {"value": total / td, "ms_per_step": 1e3 * td, "params": extra,
                        "iters_per_slab": {"min": min(its), "max": max(its), "mean": sum(its) / len(its)}}
        out["all_at_once"] = all_at_once(args, last64[1])
        out["internal_layer"] = internal_layer(tol=args.tol)
        out["ordered_relaxation"] = ordered_relaxation(args, march)
        out["adjoint_slab0"] = adjoint_slab(march, args.tol)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only (--gpus %d requested): the path has no "
              "multi-GPU sharding" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.profile_summary:
        profile_summary(args.profile_summary, args.grid)
        return
    if args.traffic:
        traffic_record(*args.traffic)
        return
    import torch
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    from paper_2010_11130_amd import lib
    lib()
    if not torch.cuda.is_available():
        print("bench.py: no HIP device", file=sys.stderr)
        sys.exit(1)
    if args.solve_alone:
        march = March(args.n, args.slabs, args.p, args.nu)
        print(json.dumps({"solve_alone": solve_alone(march, args.solve_alone, args.tol, relax=args.relax)}))
        return
    log = (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True))
    # headline: the C3 workload, setup + solve on the assembled system
    c3 = c3_inputs(args.c3_n, args.c3_nu)
    s = c3["system"]
    log("bench: C3 %d^3 assembled, %d free DOFs, %.1f ms" % (args.c3_n, s.n, c3["assemble_ms"]))
    air = {} if args.scalar_air else {"block_air": 1}
    r64, prof64, x64 = setup_solve_steps(s, args.steps, args.warmup, args.tol, 0, profile=True, **air)
    log("bench: FP64 %.1f ms/step, %d iterations" % (r64["ms_per_step"], r64["iters"]))
    level0 = ("scalar lAIR on every level" if args.scalar_air else
              "block AIR on level 0 (facet blocks as the points of strength, PMIS and one-point P; lAIR over "
              "all rows of the strong F blocks), scalar lAIR below")
    out = {
        "metric": METRIC, "value": r64["value"], "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r64["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "all-at-once 2+1D space-time cube: %d^3 Kuhn cubes -> %d tets, p=1 (b=3), "
                               "a=(1,0.5), nu=%g, smooth solution + tanh front of width 1e-2; one step = AIR setup "
                               "(%s; theta 0.25, PMIS, one-point P, distance-1 lAIR) + FGMRES(100) to %g with F,F,C "
                               "Jacobi post-sweeps, on the assembled system in HBM"
                               % (args.c3_n, c3["tets"], args.c3_nu, level0, args.tol),
                   "free_dofs": s.n, "tol": args.tol, "block_air": not args.scalar_air},
        "fp64": r64, "assemble_ms": c3["assemble_ms"],
        "end_to_end_dofs_per_s": s.n / (1e-3 * (c3["assemble_ms"] + r64["ms_per_step"])),
        "kernels": prof64,
    }
    if not args.no_fp32:
        r32, prof32, x32 = setup_solve_steps(s, args.steps, args.warmup, args.tol, 1, profile=True, **air)
        log("bench: FP32 cycle %.1f ms/step, %d iterations" % (r32["ms_per_step"], r32["iters"]))
        r32["speedup_vs_fp64"] = r64["ms_per_step"] / r32["ms_per_step"]
        r32["rel_diff_vs_fp64"] = (torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64)).item()
        r32["kernels"] = prof32
        out["fp32_cycle"] = r32
        del x32
    # the other level-0 coarsening on the same system, same timing
    other = {"block_air": 1} if args.scalar_air else {}
    rec = {}
    for prec in (() if args.no_alt_air else (0,) if args.no_fp32 else (0, 1)):
        r, _, x = setup_solve_steps(s, args.steps, args.warmup, args.tol, prec, **other)
        r["rel_diff_vs_headline_fp64"] = (torch.linalg.norm(x - x64) / torch.linalg.norm(x64)).item()
        rec["fp64" if prec == 0 else "fp32_cycle"] = r
        del x
    if rec:
        out["block_air" if args.scalar_air else "scalar_air"] = rec
        log("bench: %s done" % ("block AIR" if args.scalar_air else "scalar AIR"))
    if prof64:
        rf = roofline(prof64, "c3", 1, 3, c3["tets"])
        cb = copy_bandwidth()
        rf["copy_gbs"] = cb
        rf["frac_of_copy"] = rf["achieved"] / cb
        out["roofline"] = rf
    if not args.no_c3_variants:
        out["c3_variants"] = c3_variants(c3, args.tol, x64, air)
        log("bench: C3 variants done")
    del x64, s, c3
    # the library's cached blocks of the C3 objects go back to the device
    # (outside any timed region), so the next records start from free memory
    from paper_2010_11130_amd import pool_trim
    torch.cuda.empty_cache()
    pool_trim()
    if not args.no_march:
        out["slab_march"] = march_record(args)
        log("bench: march done")
        pool_trim()
        out["c4_precision"] = c4_record(args)
        log("bench: C4 done")
        pool_trim()
    if not args.no_large:
        out["c5_adjoint"] = c5_adjoint(args.tol)
        log("bench: C5 done")
        pool_trim()
    out["c1"] = c1_record()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, args.c3_nu, args.tol, not args.scalar_air)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
