"""Throughput benchmark: Whittle-Matern field samples per second on one MI355X.

Workload (default, the largest configuration of the measured metric): unit sphere as six cube-face
patches, degree-3 B-splines, 256 x 256 elements per patch (399,386 unknowns); kappa = 30, beta = 2.3
split into two integer solves plus the sinc rule for 0.3 with h = 0.4 and 61 nodes; 32 independent
white-noise loads (seeds 0..31); the multigrid V-cycle and its operator in FP32, the outer CG in FP64,
every shifted system to relative residual 1e-6.

One step = one call of the sampler over the 32 loads, loads already resident in device memory:
integer solves, the batch of 61 x 32 shifted systems, and the quadrature sum.  After the timed steps
the field error of two of the timed samples is measured against the FP64 path (rtol 1e-11) in the
M-norm, and the derivative d loss / d kappa (loss over 1000 seeded surface points, adjoint solves) is
timed on the same workload (gradients_per_s).

Prints one JSON line.  The roofline entry is for the dominant kernel, the Chebyshev smoothing step
on the finest level (the stencil operator fused with the smoother's update), timed with HIP events
stamped by the runtime around every launch, on extra steps run after the timed ones; a second entry
covers the FP64 operator application of the outer CG.  The CPU baseline is the FP64 oracle (sparse
LU, one thread) on one load; for meshes above 64 x 64 elements per patch its per-system cost is
measured at two coarser levels of the same workload and extrapolated (stated in the line).

--load sqrtm replaces the element-wise noise factor by the paper's own load f = sqrt(M) y (Sec. 3.3,
Khat shifted mass solves per sample, bounds estimated by the library on every call), computed inside
every step.
"""
import argparse
import collections
import csv
import hashlib
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CONFIGS = {
    # name: (perturbed, p, level, kappa, beta, h, k, nsamp, precision, rtol)
    "c2": (False, 2, 6, 10.0, 1.6, 0.4, 20, 64, 0, 1e-10),
    "c2-mixed": (False, 2, 6, 10.0, 1.6, 0.4, 20, 64, 1, 1e-10),
    "c1": (False, 2, 2, 4.0, 0.75, 0.4, 15, 1, 0, 1e-13),
    "c5": (False, 3, 8, 30.0, 2.3, 0.4, 30, 32, 1, 1e-6),
    "c4": (False, 3, 6, 8.0, 0.8, 0.4, 20, 16, 1, 1e-7),
    "c5-grad": (False, 3, 8, 30.0, 2.3, 0.4, 30, 32, 1, 1e-7),
    # NURBS multi-patch surface: the 4 x 4 patch torus R = 2, r = 1 (biquadratic rational Bezier
    # patches, four at every corner), 32 x 32 elements per patch
    "torus": ("torus", 2, 5, 10.0, 1.6, 0.4, 20, 64, 0, 1e-10),
}
# configs whose step also computes d loss / d kappa by the adjoint (loss over 1000 seeded points)
GRADIENT_CONFIGS = {"c4", "c5-grad"}
# relative residual of the forward and adjoint solves of a gradient: at 1e-6 the mixed-precision
# d loss / d kappa deviates from the FP64 adjoint by up to 1.4e-6 (degree 3, 64 x 64 mesh, four
# samples), at 1e-7 by 2.5e-8, inside the 1e-6 stated for gradients
GRAD_RTOL = 1e-7


# several sampling requests solved together (one call of the batched sampler per step): every
# combination of degree, level and kappa is one request; sample s goes to request s mod (number of
# requests), with white-noise seed s
BATCH_CONFIGS = {
    "c3": dict(perturbed=True, degrees=(2, 3), levels=(5, 6, 7), kappas=(5.0, 10.0, 20.0), beta=0.9, h=0.4, k=20,
               nsamp=256, precision=1, rtol=1e-6),
    "c3-fp64": dict(perturbed=True, degrees=(2, 3), levels=(5, 6, 7), kappas=(5.0, 10.0, 20.0), beta=0.9, h=0.4,
                    k=20, nsamp=256, precision=0, rtol=1e-6),
}


def accurate_nodes(beta, kappa, level, h, eps=1e-6):
    """(k_minus, k_plus) of the tolerance-driven node set at step h: each tail of the sinc sum for
    beta' = beta - floor(beta) is cut where its terms, relative to the exact power, fall below eps
    for the extreme eigenvalues of the discrete operator (lambda from kappa^2 up to
    kappa^2 + l (l + 1) with l = sqrt(6) 2^level, the largest degree a mesh of 2^level elements
    per patch side resolves).  Large t: terms ~ t^-beta', cut at t^-beta' = eps lambda_max^-beta';
    small t: terms ~ t^(1-beta') / kappa^2, cut at (t / kappa^2)^(1-beta') = eps."""
    bf = beta - math.floor(beta)
    lmax = math.sqrt(6.0) * 2 ** level
    lam_max = kappa * kappa + lmax * (lmax + 1.0)
    y_lo = (math.log(eps) - bf * math.log(lam_max)) / (2.0 * bf)
    y_hi = -(math.log(eps) + (1.0 - bf) * math.log(kappa * kappa)) / (2.0 * (1.0 - bf))
    return math.ceil(-y_lo / h), math.ceil(y_hi / h)


def batch_workload_name(bc, nreq, nodes_desc=None):
    surf = "perturbed sphere" if bc["perturbed"] else "unit sphere"
    lv = "/".join(f"{2**l}x{2**l}" for l in bc["levels"])
    return (f"{surf}, 6 patches, degrees {bc['degrees']}, {lv} elements/patch, kappa in {bc['kappas']}, "
            f"beta={bc['beta']:g} ({nodes_desc or str(2*bc['k']+1) + ' sinc nodes'}, h={bc['h']:g}); {bc['nsamp']} samples over {nreq} "
            f"requests in one batched call; {'FP64' if bc['precision'] == 0 else 'FP32 V-cycle / FP64 CG'} MG-PCG "
            f"to rel. residual {bc['rtol']:g}")


def workload_name(cfg, km=None, kp=None):
    pert, p, lev, kappa, beta, h, k, nsamp, prec, rtol = cfg
    n1 = 2 ** lev + p
    nint = math.floor(beta)
    if pert == "torus":
        N, surf, npatch = 16 * (n1 - 1) ** 2, "NURBS torus R=2 r=1", 16
    else:
        N, npatch = 6 * (n1 - 2) ** 2 + 12 * (n1 - 2) + 8, 6
        surf = "perturbed sphere" if pert else "unit sphere"
    return (f"{surf}, {npatch} patches, degree {p}, {2**lev}x{2**lev} elements/patch ({N} DOF); kappa={kappa:g}, "
            f"beta={beta:g} ({nint} integer solve(s) + "
            f"{(2*k+1) if km is None else f'{km+kp+1} (k = -{km}..{kp}, tolerance 1e-6)'} sinc nodes, h={h:g}); "
            f"{nsamp} samples; "
            f"{'FP64' if prec == 0 else 'FP32 V-cycle / FP64 CG (FP32 search direction)'} MG-PCG to rel. residual {rtol:g}")


KERNEL_SOURCES = [os.path.join(ROOT, "paper_2605_24882_amd", "csrc", f) for f in ("k_fused.hip", "k_stencil.h")]


def traffic_file(config):
    return os.path.join(ROOT, "profiles", f"traffic_stencil_{config}.json")


def source_sha():
    """SHA-256 of the stencil kernels' sources (the traffic counters are valid only for these)."""
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _stencil_kind(name, p, kind, vt):
    """Whether a kernel name is the finest-level operator launch of `kind`: "outer" (EPI_STORE with the
    inner product, FP64) or "smoother" (EPI_CHEB in type vt), in the combined-stencil kernel
    k_stencil<T, P, TY, KIND, DOT, MODE> or the separate-stencil kernel k_apply_fused<T, P, TY, KIND, DOT>."""
    for k in ("k_stencil", "k_apply_fused"):
        pre = f"void gf::{k}<{vt}, {p}, "
        if not name.startswith(pre):
            continue
        args = [a.strip() for a in name[len(pre):].rstrip(">").split(",")]  # TY, KIND, DOT[, MODE]
        if len(args) < 3:
            return False
        return (args[1], args[2]) == ("0", "1") if kind == "outer" else args[1] == "1"
    return False


def _kernel_rows(path, p, kind, value_key, last=None):
    # `path`: a CSV file or its rows
    """values of every launch of the stencil kernel with epilogue `kind` ("outer": EPI_STORE with the
    inner product, FP64; "smoother": EPI_CHEB in the V-cycle's precision, FP32 when no FP64 smoothing
    step was launched) at the finest level (the largest grid of that kernel), in dispatch order; with
    `last`, only the last that many of them (the launches of the event-timed step, which ends the run)."""
    rows = list(csv.DictReader(open(path))) if isinstance(path, str) else list(path)
    if rows and "Dispatch_Id" in rows[0]:
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    has_double_smoother = any(_stencil_kind(r["Kernel_Name"].split("(")[0], p, "smoother", "double") for r in rows)
    vt = "double" if kind == "outer" or has_double_smoother else "float"
    out = []
    for r in rows:
        name = r["Kernel_Name"].split("(")[0]
        if _stencil_kind(name, p, kind, vt):
            grid = int(r.get("Grid_Size") or r.get("Grid_Size_X"))
            v = value_key(r)
            if v is not None:
                out.append((grid, v))
    big = max(g for g, _ in out)
    vals = [v for g, v in out if g == big]
    return (vals[-last:] if last else vals), big


def _events(path):
    """launch counts, algorithmic bytes and event-timed durations per launch of the two operator
    kinds from a bench.py JSON line (its event-timed step is the last part of the run)"""
    if not path:
        return None
    with open(path) as f:
        d = json.loads(f.read().strip().splitlines()[-1])
    return {"smoother": d["roofline"], "outer": d["roofline_outer_operator"]}


READ_REQ = {"TCC_EA0_RDREQ_32B_sum": 32, "TCC_EA0_RDREQ_64B_sum": 64, "TCC_EA0_RDREQ_128B_sum": 128}


def _dispatch_counters(path):
    """rows of a rocprofv3 counter CSV merged per dispatch: {dispatch id: row with a "counters" dict}"""
    out = {}
    for r in csv.DictReader(open(path)):
        d = out.setdefault(int(r["Dispatch_Id"]), dict(r, counters={}))
        d["counters"][r["Counter_Name"]] = float(r["Counter_Value"])
    return [out[k] for k in sorted(out)]


def _read_bytes(counters):
    """bytes an L2 channel fetched from memory, from the request counts by size"""
    return sum(counters[n] * b for n, b in READ_REQ.items())


def pmc_summary(fetch_csv, write_csv, config, probe_mib, events=None):
    """Per-launch HBM traffic of the finest-level smoothing launches and of the outer operator from
    two counter runs, KiB per dispatch.  Reads: either FETCH_SIZE, scaled by what it reads for the
    plain elementwise probe kernel (dst = -src over probe_mib MiB, which reads and writes exactly that
    many bytes), or the memory read requests of the L2 by size (TCC_EA0_RDREQ_{32B,64B,128B}_sum: bytes
    counted directly; the probe is then a check).  Writes: WRITE_SIZE, scaled by the probe.  With
    `events` (the JSON line of a run with the same launch sequence), only the launches of the
    event-timed step are averaged and set against their algorithmic bytes."""
    p = CONFIGS[config][1]
    known_kib = probe_mib * 1024.0
    out = {"config": config, "kernel_source_sha256": source_sha(), "probe_mib": probe_mib}
    for key, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = _dispatch_counters(path)
        by_req = key == "fetch" and all(n in rows[0]["counters"] for n in READ_REQ)
        if by_req:
            val = lambda r: _read_bytes(r["counters"]) / 1024.0
            out["fetch_counters"] = "TCC_EA0_RDREQ_32B/64B/128B (request counts x size)"
        else:
            name = "FETCH_SIZE" if key == "fetch" else "WRITE_SIZE"
            val = lambda r, name=name: r["counters"][name]
            out[f"{key}_counters"] = name
        probe = [r for r in rows if "neg_kernel" in r["Kernel_Name"]]
        if not probe:
            raise SystemExit(f"{path}: no probe kernel dispatch")
        # the copy probe runs before the workload; a later elementwise kernel of another size (the
        # stream probe of a run without --copy-probe-mib) has another grid and is left out
        pv = [val(r) for r in probe if r["Grid_Size"] == probe[0]["Grid_Size"]]
        factor = 1.0 if by_req else known_kib / (sum(pv) / len(pv))
        out[f"{key}_probe_kib"] = sum(pv) / len(pv)
        out[f"{key}_factor"] = round(factor, 4)
        for kind in ("smoother", "outer"):
            e = out.setdefault(kind, {})
            vals, grid = _kernel_rows(rows, p, kind, val, last=events[kind]["launches"] if events else None)
            e[f"{key}_kib_per_launch"] = sum(vals) / len(vals)
            e[f"{key}_launches"] = len(vals)
            e[f"{key}_grid"] = grid
            e[f"{key}_bytes_per_launch"] = sum(vals) / len(vals) * 1024.0 * factor
    for kind in ("smoother", "outer"):
        e = out[kind]
        e["traffic_bytes_per_launch"] = e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]
        if events:
            e["algorithmic_bytes_per_launch"] = events[kind]["bytes_per_launch"]
            e["traffic_over_algorithmic"] = round(e["traffic_bytes_per_launch"] / events[kind]["bytes_per_launch"], 4)
    return out


def counter_summary(csvs, config):
    """Markdown table: every counter of the given rocprofv3 --pmc runs, averaged per launch, for the
    finest-level smoothing step and the outer operator."""
    p = CONFIGS[config][1]
    table = {}
    for path in csvs:
        names = sorted({r["Counter_Name"] for r in csv.DictReader(open(path))})
        for n in names:
            for kind in ("smoother", "outer"):
                vals, _ = _kernel_rows(path, p, kind,
                                       lambda r, n=n: float(r["Counter_Value"]) if r["Counter_Name"] == n else None)
                vals = [v for v in vals if v is not None]
                table.setdefault(n, {})[kind] = (sum(vals) / len(vals), len(vals)) if vals else (float("nan"), 0)
    lines = ["| counter | smoothing step, per launch | outer operator, per launch |", "|---|---:|---:|"]
    for n in sorted(table):
        sm, ou = table[n]["smoother"], table[n]["outer"]
        lines.append(f"| {n} | {sm[0]:.4g} ({sm[1]} launches) | {ou[0]:.4g} ({ou[1]} launches) |")
    return "\n".join(lines)


def trace_summary(trace_csv, p, top=25, events=None):
    """Text summary of a rocprofv3 kernel trace: time per kernel and grid, and the two operator kinds;
    with `events` (the JSON line the traced run printed) also the trace's average over the launches of
    the event-timed step (the last launches of each kind) beside the events' average."""
    rows = list(csv.DictReader(open(trace_csv)))
    agg = collections.defaultdict(list)
    for r in rows:
        g = (int(r["Grid_Size_X"]), int(r["Grid_Size_Y"]), int(r["Grid_Size_Z"]))
        agg[(r["Kernel_Name"].split("(")[0], g)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    tot = sum(sum(v) for v in agg.values())
    lines = [f"total kernel time {tot / 1e3:.2f} ms over {len(rows)} dispatches", "",
             "| ms | % | calls | avg us | kernel | grid |", "|---:|---:|---:|---:|---|---|"]
    for (k, g), v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:top]:
        lines.append(f"| {sum(v) / 1e3:.2f} | {100 * sum(v) / tot:.1f} | {len(v)} | {sum(v) / len(v):.2f} | `{k}` | {g[0]} |")
    d = {}
    # the smoothing step runs in the V-cycle's precision (float in mixed mode), the outer operator in
    # double
    has_double_smoother = any(_stencil_kind(r["Kernel_Name"].split("(")[0], p, "smoother", "double") for r in rows)
    for kind in ("smoother", "outer"):
        ts = []
        vt = "double" if kind == "outer" or has_double_smoother else "float"
        for r in rows:
            name = r["Kernel_Name"].split("(")[0]
            if _stencil_kind(name, p, kind, vt):
                ts.append((int(r["Start_Timestamp"]), int(r["Grid_Size_X"]),
                           (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
        big = max(g for _, g, _ in ts)
        d[kind] = [x for _, g, x in sorted(ts) if g == big]
        lines += ["", f"{kind} ({'finest-level Chebyshev smoothing step' if kind == 'smoother' else 'outer CG operator'}, "
                      f"grid {big}): {len(d[kind])} launches, avg {sum(d[kind]) / len(d[kind]):.2f} us"]
        if events:
            n = events[kind]["launches"]
            tail = d[kind][-n:]
            ev = events[kind]["avg_launch_us"]
            tr = sum(tail) / len(tail)
            lines.append(f"  event-timed step: last {n} launches, trace avg {tr:.2f} us, events avg {ev:.2f} us "
                         f"(ratio {ev / tr:.4f}); algorithmic {events[kind]['bytes_per_launch']:.4e} B per launch "
                         f"-> {events[kind]['bytes_per_launch'] / tr / 1e3:.1f} GB/s by the trace")
    return "\n".join(lines), d


def one_at_a_time(g, sp, b, cfg, kw, nodes_timed=6):
    """The same shifted systems solved one per call (gf_solve_shifted with one system, FP64, same
    solver and tolerance) on the GPU: the unbatched reference the batched sampler is measured against.

    Bounded sample: for load 0, its integer-chain system (shift kappa^2) and `nodes_timed` of the node
    systems (evenly spaced in k), each with load 0 as right-hand side; per sample, the chain systems
    and all nodes at the measured average (multigrid plans are built before timing, as the batched
    path's are cached)."""
    import torch
    pert, p, lev, kappa, beta, h, k, nsamp, prec, rtol = cfg
    n = math.floor(beta)
    bf = beta - n
    t = [math.exp(-2.0 * kk * h) for kk in range(-k, k + 1)]
    pick = [round(i * (len(t) - 1) / (nodes_timed - 1)) for i in range(nodes_timed)] if bf > 0 else []
    shifts = ([kappa * kappa] if n > 0 else []) + [kappa * kappa + t[i] for i in pick]
    b0 = b[0:1].contiguous()
    for sg in shifts:  # plans
        sp.solve_shifted(sg, b0, precision=0, rtol=rtol, max_iter=kw["max_iter"])
    torch.cuda.synchronize()
    times = []
    for sg in shifts:
        t0 = time.perf_counter()
        sp.solve_shifted(sg, b0, precision=0, rtol=rtol, max_iter=kw["max_iter"])
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    chain = times[0] if n > 0 else 0.0
    node = sum(times[1:] if n > 0 else times) / max(1, len(pick))
    per_sample = n * chain + (len(t) * node if bf > 0 else 0.0)
    return {"value": round(1.0 / per_sample, 3), "unit": "samples/s", "dtype": "f64",
            "sample": (f"load 0: {'its chain system and ' if n > 0 else ''}{len(pick)} of the {len(t)} node systems, "
                       f"one system per call; per sample {n} chain system(s) at {chain * 1e3:.1f} ms and {len(t)} "
                       f"node systems at {node * 1e3:.1f} ms on average")}


def stream_probe(torch, mib=1024, reps=10):
    """Achieved bandwidth of a plain streaming kernel on this GPU (dst = -src over `mib` MiB of FP64:
    reads and writes that many bytes), as context for the roofline fraction of the stencil kernels."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.neg(src, out=dst)
    e1.record()
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    gbs = 2.0 * n * 8 / (us * 1e-6) / 1e9
    del src, dst
    return {"kernel": f"dst = -src, {mib} MiB FP64 each way", "avg_launch_us": round(us, 2),
            "achieved": round(gbs, 1), "unit": "GB/s", "frac_of_peak": round(gbs / 8000.0, 4)}


def cpu_model():
    """(model name, logical CPUs) of the host."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, os.cpu_count()


_POOL = {}  # the matrices and load of the pool's node solves (inherited by the forked workers)


def _pool_node_solve(i):
    """one sinc-node system of the pooled oracle run: the oracle's own node solve (SuperLU
    factorisation + solve) on one thread; returns its duration"""
    from threadpoolctl import threadpool_limits
    from oracle import fractional
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        fractional.node_solutions(_POOL["M"], _POOL["S"], _POOL["sig"][i:i + 1], _POOL["r"])
        return time.perf_counter() - t0


def _oracle_pool_rate(pert, p, lev, kappa, beta, h, k, cores):
    """The oracle on one load at one level: its integer chain on one thread, then `cores` of its node
    solves (evenly spaced in k) run by `cores` forked worker processes at once.  Returns the unknowns,
    the chain time, the node count and the wall time of the pooled node solves."""
    import multiprocessing

    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import assembly, fractional, noise
    from paper_2605_24882_amd import inputs
    n, bf = fractional.split_plain(beta)
    if pert == "torus":
        from oracle import geometry
        d = assembly.Discretisation(p, lev, geometry.NurbsSurface(*inputs.torus_patches(2.0, 1.0)))
    else:
        d = assembly.Discretisation(p, lev, pert)
    b = noise.load(d, inputs.noise_vectors([0], inputs.noise_length(p, lev, 16 if pert == "torus" else 6)))
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ws = fractional.integer_chain(d.M, d.S, kappa, n, b)
        chain = time.perf_counter() - t0
    r = b if n == 0 else np.stack([d.M @ w for w in ws[-1]])
    sigma, _, _ = fractional.nodes(kappa, bf, h, k, k)
    pick = np.linspace(0, len(sigma) - 1, cores).round().astype(int)
    _POOL.update(M=d.M, S=d.S, r=r, sig=sigma[pick])
    with multiprocessing.get_context("fork").Pool(cores) as pool:
        t0 = time.perf_counter()
        single = pool.map(_pool_node_solve, range(cores), chunksize=1)
        wall = time.perf_counter() - t0
    _POOL.clear()
    return dict(N=d.N, n=n, chain=chain, nodes=len(sigma) if bf > 0 else 0, wall=wall,
                single=sum(single) / len(single))


def cpu_baseline(cfg):
    """The oracle (sparse LU, FP64) on the first load of the workload, its node solves spread over a
    pool of worker processes (one per core of the host's share, one thread each).

    Bounded sample.  Per level measured: the integer chain of the load on one thread, then as many node
    solves as there are workers, all at once (evenly spaced in k).  Every node solve is one SuperLU
    factorisation plus a solve; the pool's wall time gives the core-seconds one node solve costs with
    every core busy, t = wall x cores / solves (memory contention included).  A sample costs its
    chain plus its nodes, in node-solve units c = nodes + chain time / single-solve time, so the pool
    completes cores / (c t) samples per second.  Up to 64 x 64 elements per patch the workload's level
    is measured; finer meshes (one factorisation alone would take minutes) at the two levels three and
    two below, t extrapolated to the workload's unknowns by the power law of those two levels."""
    pert, p, lev, kappa, beta, h, k, nsamp, prec, rtol = cfg
    model, ncpu = cpu_model()
    cores = max(1, min(16, ncpu or 1))
    levels = [lev] if lev <= 6 else [lev - 3, lev - 2]
    ms = [_oracle_pool_rate(pert, p, lv, kappa, beta, h, k, cores) for lv in levels]
    t_eff = [m["wall"] for m in ms]  # core-seconds per node solve with every core busy (cores solves, cores workers)
    m = ms[-1]
    if lev <= 6:
        t = t_eff[0]
        extra = ""
    else:
        n1 = 2 ** lev + p
        N = 6 * (n1 - 2) ** 2 + 12 * (n1 - 2) + 8
        expo = math.log(t_eff[1] / t_eff[0]) / math.log(ms[1]["N"] / ms[0]["N"])
        t = t_eff[1] * (N / ms[1]["N"]) ** expo
        extra = (f"; {t_eff[0]:.3f} s and {t_eff[1]:.2f} s per node solve at levels {levels[0]} and {levels[1]} "
                 f"({ms[0]['N']} and {ms[1]['N']} unknowns), extrapolated as N^{expo:.2f} to {N} unknowns: {t:.0f} s")
    c = m["nodes"] + m["chain"] / m["single"]
    value = cores / (c * t)
    sample = (f"1 of the {nsamp} loads (seed 0) at level{'s' if len(levels) > 1 else ''} "
              f"{' and '.join(str(v) for v in levels)}: its {m['n']} integer solve(s) on one thread "
              f"({m['chain']:.2f} s), then {cores} of its {m['nodes']} node solves at once in {cores} worker "
              f"processes ({m['wall']:.2f} s wall; {m['single']:.2f} s per solve): {t:.2f} core-s per node "
              f"solve with every core busy{extra}; {c:.1f} node-solve units per sample; assembly excluded")
    return {"value": value, "unit": "samples/s", "cores": cores, "kind": "oracle", "sample": sample,
            "host_cpu": model, "host_logical_cpus": ncpu}


def cpu_baseline_child(config):
    """cpu_baseline in a child process that never touches the GPU (its worker pool forks it)"""
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--config", config, "--cpu-baseline-only"],
                       capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"cpu baseline failed:\n{r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c5", choices=sorted(CONFIGS) + sorted(BATCH_CONFIGS))
    ap.add_argument("--apply-kind", type=int, default=0)
    ap.add_argument("--cheb", type=int, default=0)
    ap.add_argument("--precond", choices=("vcycle", "bpx"), default="vcycle",
                    help="multigrid preconditioner: the V-cycle or the additive BPX form")
    ap.add_argument("--split", choices=("plain", "improved"), default="plain",
                    help="split of beta: plain n + beta', or the improved split (the rule applied twice)")
    ap.add_argument("--load", choices=("factor", "sqrtm"), default="factor",
                    help="white-noise load: element-wise factor (default) or sqrt(M) y inside every step")
    ap.add_argument("--khat", type=int, default=16, help="square-root rule size for --load sqrtm")
    ap.add_argument("--nodes", choices=("fixed", "accurate"), default="fixed",
                    help="sinc nodes: the workload's symmetric K, or the tolerance-driven set (1e-6) per request")
    ap.add_argument("--mg-levels", type=int, default=0,
                    help="levels of the multigrid hierarchy (0: the library's choice, all levels down to 0)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="time the oracle's bounded sample of the workload on the host (no GPU), print it as JSON")
    ap.add_argument("--no-gradient", action="store_true",
                    help="skip the d loss / d kappa timing that follows the sampling steps")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the field error of two timed samples against the FP64 path")
    ap.add_argument("--no-one-at-a-time", action="store_true",
                    help="skip the one-system-per-call FP64 GPU reference timing")
    ap.add_argument("--apply-shape", default="",
                    help="fix the operator launch shape 'TY,TX' instead of autotuning it (profiling runs)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the per-launch traffic of the outer operator from two rocprofv3 counter runs "
                         "(made with --copy-probe-mib) as JSON to stdout, then exit")
    ap.add_argument("--counter-summary", nargs="+", metavar="COUNTER_CSV",
                    help="print the per-launch averages of every counter in these --pmc runs and exit")
    ap.add_argument("--trace-summary", metavar="KERNEL_TRACE_CSV",
                    help="print a summary of a rocprofv3 kernel trace of this benchmark, then exit")
    ap.add_argument("--events-json", metavar="BENCH_JSON",
                    help="with --trace-summary / --pmc-summary: the JSON line of a run of this benchmark with the same "
                         "launch sequence; restricts the averages to the launches of its event-timed step")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the timed steps, stream this many MiB through a plain elementwise kernel "
                         "(dst = -src: reads and writes exactly that many bytes; the known-size reference for "
                         "the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline(CONFIGS[args.config])))
        return
    if args.pmc_summary:
        print(json.dumps(pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.config,
                                     args.copy_probe_mib or 512, _events(args.events_json)), indent=1))
        return
    if args.counter_summary:
        print(counter_summary(args.counter_summary, args.config))
        return
    if args.trace_summary:
        print(trace_summary(args.trace_summary, CONFIGS[args.config][1], events=_events(args.events_json))[0])
        return
    if args.apply_shape:
        os.environ["GF_APPLY_SHAPE"] = args.apply_shape
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (samples are independent: "
              f"several GPUs would each solve their own samples, with no communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2605_24882_amd import gfield as g
    from paper_2605_24882_amd import inputs

    ctx = g.Context(0)
    t0 = time.perf_counter()
    if args.config in BATCH_CONFIGS:
        bc = BATCH_CONFIGS[args.config]
        pert, prec, rtol, nsamp, p = bc["perturbed"], bc["precision"], bc["rtol"], bc["nsamp"], max(bc["degrees"])
        geo = g.Geometry(ctx, pert)
        spaces = {(dg, lv): g.Space(ctx, geo, dg, lv, mg_levels=args.mg_levels) for dg in bc["degrees"]
                  for lv in bc["levels"]}
        space_s = time.perf_counter() - t0
        combos = [(dg, lv, kp) for dg in bc["degrees"] for lv in bc["levels"] for kp in bc["kappas"]]
        reqs = []
        for i, (dg, lv, kp) in enumerate(combos):
            sp = spaces[(dg, lv)]
            seeds = [s_ for s_ in range(nsamp) if s_ % len(combos) == i]
            z = torch.from_numpy(inputs.noise_vectors(seeds, sp.noise_length)).cuda()
            km_, kp_ = (accurate_nodes(bc["beta"], kp, lv, bc["h"]) if args.nodes == "accurate"
                        else (bc["k"], bc["k"]))
            reqs.append(dict(space=sp, kappa=kp, beta=bc["beta"], b=sp.white_noise(z), h=bc["h"],
                             k_minus=km_, k_plus=kp_,
                             split=g.GF_SPLIT_IMPROVED if args.split == "improved" else g.GF_SPLIT_PLAIN))
            del z
        kw = dict(precision=prec, rtol=rtol, max_iter=2000, cheb_degree=args.cheb, apply_kind=args.apply_kind,
                  preconditioner=g.GF_PRECOND_BPX if args.precond == "bpx" else g.GF_PRECOND_VCYCLE)

        def step(flags=0):
            return g.sample_batch(ctx, reqs, flags=flags, **kw)
        workload = batch_workload_name(
            bc, len(combos), None if args.nodes == "fixed" else
            f"{min(r['k_minus'] + r['k_plus'] + 1 for r in reqs)}..{max(r['k_minus'] + r['k_plus'] + 1 for r in reqs)}"
            f" sinc nodes per request (tolerance 1e-6)")
    else:
        cfg = CONFIGS[args.config]
        pert, p, lev, kappa, beta, h, k, nsamp, prec, rtol = cfg
        if pert == "torus":
            geo = g.Geometry.nurbs(ctx, *inputs.torus_patches(2.0, 1.0))
        else:
            geo = g.Geometry(ctx, pert)
        sp = g.Space(ctx, geo, p, lev, mg_levels=args.mg_levels)
        space_s = time.perf_counter() - t0
        if args.load == "sqrtm":
            y = torch.from_numpy(inputs.noise_vectors(range(nsamp), sp.ndofs)).cuda()
            b = None
        else:
            z = torch.from_numpy(inputs.noise_vectors(range(nsamp), sp.noise_length)).cuda()
            b = sp.white_noise(z)
            del z
        km, kp = accurate_nodes(beta, kappa, lev, h) if args.nodes == "accurate" else (k, k)
        kw = dict(h=h, k_minus=km, k_plus=kp, precision=prec, rtol=rtol, max_iter=1000, cheb_degree=args.cheb,
                  apply_kind=args.apply_kind,
                  split=g.GF_SPLIT_IMPROVED if args.split == "improved" else g.GF_SPLIT_PLAIN,
                  preconditioner=g.GF_PRECOND_BPX if args.precond == "bpx" else g.GF_PRECOND_VCYCLE)

        grad_step = None
        if pert != "torus" and args.load == "factor":
            pts, yv = inputs.sphere_points_and_targets(1000, seed=7)
            patch, stp = geo.locate(pts)
            yt = torch.from_numpy(yv).cuda()

            kwg = dict(kw)
            kwg["rtol"] = min(kw["rtol"], GRAD_RTOL)

            def grad_step(flags=0):
                """forward samples and d loss / d kappa per sample (loss over 1000 seeded points)"""
                u, tape, st1 = sp.sample_tape(kappa, beta, b, flags=flags, **kwg)
                vals = sp.eval(patch, stp, u)
                gk, st2 = tape.grad_kappa(sp.eval_adjoint(patch, stp, vals - yt[None, :]))
                tape.close()
                st = dict(st1)
                for key in ("apply_ms", "apply_launches", "apply_bytes", "smooth_ms", "smooth_launches",
                            "smooth_bytes", "n_systems"):
                    st[key] = st1[key] + st2[key]
                st["max_iters"] = max(st1["max_iters"], st2["max_iters"])
                st["max_rel_resid"] = max(st1["max_rel_resid"], st2["max_rel_resid"])
                return gk, st
        if args.config in GRADIENT_CONFIGS:
            step = grad_step
            workload = workload_name(cfg, *((km, kp) if args.nodes == "accurate" else ())) + "; plus d loss/d kappa by adjoint solves (loss over 1000 points)"
        elif args.load == "sqrtm":
            def step(flags=0):
                f, st0 = sp.sqrt_mass(y, khat=args.khat, rtol=rtol, flags=flags & ~g.GF_FLAG_TIME_APPLY)
                u, st = sp.sample(kappa, beta, f, flags=flags, **kw)
                st = dict(st)
                st["n_systems"] += st0["n_systems"]
                st["max_iters"] = max(st["max_iters"], st0["max_iters"])
                return u, st
            workload = workload_name(cfg, *((km, kp) if args.nodes == "accurate" else ())) + f"; load sqrt(M) y by the square-root rule with {args.khat} shifts"
        else:
            def step(flags=0):
                return sp.sample(kappa, beta, b, flags=flags, **kw)
            workload = workload_name(cfg, *((km, kp) if args.nodes == "accurate" else ()))
    if args.split == "improved":
        workload += "; improved split (rule applied twice where beta' < 1/3 or > 2/3)"
    if args.precond == "bpx":
        workload += "; BPX (additive multilevel) preconditioner"
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        u, st = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    agg = {"apply_ms": 0.0, "apply_launches": 0, "apply_bytes": 0.0, "smooth_ms": 0.0, "smooth_launches": 0,
           "smooth_bytes": 0.0, "max_iters": 0, "max_rel_resid": 0.0}
    for _ in range(args.steps):
        u, st = step()
        agg["max_iters"] = max(agg["max_iters"], st["max_iters"])
        agg["max_rel_resid"] = max(agg["max_rel_resid"], st["max_rel_resid"])
    torch.cuda.synchronize()
    host_syncs = st.get("host_syncs")  # host waits inside the CG loops of one timed step
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = nsamp * args.steps / elapsed
    # field error of two timed samples against the FP64 path at rtol 1e-11 (M-norm, the L2 norm of the
    # field on the surface)
    accuracy = None
    if (args.config in CONFIGS and args.config not in GRADIENT_CONFIGS and args.load == "factor"
            and not args.no_accuracy):
        kw64 = dict(kw)
        kw64.update(precision=0, rtol=1e-11, max_iter=4000)
        nchk = min(2, nsamp)
        uref, st64 = sp.sample(kappa, beta, b[:nchk].contiguous(), **kw64)
        err = u[:nchk] - uref
        num = (err * sp.apply(1.0, 0.0, err)).sum(dim=1)
        den = (uref * sp.apply(1.0, 0.0, uref)).sum(dim=1)
        rel = torch.sqrt(num / den)
        accuracy = {"rel_l2_vs_fp64": float(rel.max()), "samples_checked": nchk,
                    "reference": "the library's FP64 path at rtol 1e-11 on the same loads (M-norm)",
                    "reference_cg_iters": st64["max_iters"]}
    # derivative throughput: forward samples and d loss / d kappa per sample by the adjoint solves
    gradients = None
    if (args.config in CONFIGS and args.config not in GRADIENT_CONFIGS and not args.no_gradient
            and grad_step is not None):
        gsteps = max(1, min(3, args.steps))
        grad_step()
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(gsteps):
            gk, gst = grad_step()
        torch.cuda.synchronize()
        tg = time.perf_counter() - tg
        gradients = {"value": round(nsamp * gsteps / tg, 3), "unit": "gradients/s", "steps": gsteps,
                     "ms_per_step": round(1e3 * tg / gsteps, 3), "max_cg_iters": gst["max_iters"],
                     "rtol": kwg["rtol"],
                     "what": (f"{nsamp} forward samples and d loss/d kappa of each (loss over 1000 seeded surface "
                              f"points; adjoint solves by the same batched solver) per step")}
    # dominant-kernel timing: the same steps once more with HIP events stamped around every outer
    # operator launch of the node batch (events need the eagerly enqueued loop; kernels and launch
    # shapes are the same)
    for _ in range(max(1, args.steps // 2)):
        u, st = step(flags=g.GF_FLAG_TIME_APPLY)
        for key in ("apply_ms", "apply_launches", "apply_bytes", "smooth_ms", "smooth_launches", "smooth_bytes"):
            agg[key] += st[key]

    # roofline of the dominant kernel: the Chebyshev smoothing step on the finest level (the stencil
    # operator with the smoother's epilogue; most of the step's time), and, as a second entry, the
    # FP64 stencil operator of the outer CG.  Algorithmic bytes (library count): the batch vectors
    # each launch reads and writes, per active column and patch row, plus the two stencils per row
    def roof_entry(ms, launches, nbytes, kernel, kind):
        launches = max(1, launches)
        per_launch = nbytes / launches
        avg_ms = ms / launches
        achieved = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
        traffic = None
        tf = traffic_file(args.config)
        if os.path.exists(tf):
            with open(tf) as f:
                t = json.load(f)
            if t.get("kernel_source_sha256") == source_sha() and kind in t:
                traffic = round(t[kind]["traffic_bytes_per_launch"])
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                "frac": round(achieved / 8000.0, 4), "traffic": traffic, "kernel": kernel,
                "avg_launch_us": round(avg_ms * 1e3, 2), "bytes_per_launch": int(per_launch), "launches": launches}

    vt = "double" if prec == 0 else "float"
    roof = roof_entry(agg["smooth_ms"], agg["smooth_launches"], agg["smooth_bytes"],
                      f"k_stencil<{vt},p,*,EPI_CHEB,*,*> (Chebyshev smoothing step on the finest level, stencil form)",
                      "smoother")
    outer_kernel = ("k_stencil<double,p,*,EPI_STORE,dot,*,float> (outer CG operator on the FP32 search direction, "
                    "stencil form)" if prec != 0 else "k_stencil<double,p,*,EPI_STORE,dot,*> (outer CG operator, stencil form)")
    roof_outer = roof_entry(agg["apply_ms"], agg["apply_launches"], agg["apply_bytes"], outer_kernel, "outer")

    out = {
        "metric": "field samples/sec at rel-L2 err <=1e-6 vs FP64 oracle; operator-apply HBM GB/s",
        "value": round(value, 3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": workload, "samples_per_step": nsamp, "systems_per_step": st["n_systems"],
                   "max_cg_iters": agg["max_iters"], "max_rel_resid": agg["max_rel_resid"],
                   "host_syncs_per_step": host_syncs,
                   "space_setup_s": round(space_s, 3),
                   **({"accuracy": accuracy} if accuracy else {})},
        "roofline": roof,
        "roofline_outer_operator": roof_outer,
        # the counter runs (--copy-probe-mib) time no stream probe: their only elementwise kernel is
        # the copy probe
        "stream_probe": stream_probe(torch) if args.copy_probe_mib == 0 else None,
        # the vector multiply-add rates the stencil kernels' ALU use is compared with (library probe:
        # independent multiply-add chains, no memory traffic)
        "fma_probe": ({"fp64": round(ctx.probe_fma(g.GF_PREC_FP64), 1), "fp32": round(ctx.probe_fma(g.GF_PREC_MIXED), 1),
                       "unit": "TFLOP/s", "fp32_kind": "scalar FMA (no packed FP32 instructions)"}
                      if args.copy_probe_mib == 0 else None),
    }
    if (args.config in CONFIGS and args.config not in GRADIENT_CONFIGS and not args.no_one_at_a_time
            and args.load == "factor"):
        out["gpu_one_solve_at_a_time"] = one_at_a_time(g, sp, b, CONFIGS[args.config], kw)
    if gradients:
        out["gradients_per_s"] = gradients
    if not args.no_cpu_baseline and args.config in CONFIGS and args.load == "factor":
        out["cpu_baseline"] = cpu_baseline_child(args.config)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
