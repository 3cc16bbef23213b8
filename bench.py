#!/usr/bin/env python3
"""Benchmark of the gfx950 unstructured S_N sweep (one MI355X).

A step is one source iteration of the whole hot path on one synthetic
problem: scattering-source update, the persistent dependency-driven sweep of
all octants, angles and groups, the compensated angle reduction and the FP64
convergence residual (graph-captured, as snx_solve runs it).  Setup (element
matrices, designation, levelling) is done once per mesh before timing.

Default workload (the largest single-GPU shape): 64^3 jittered hex grid
(262,144 cells, ids permuted), 4x8 product quadrature (256 angles), 64 groups,
sigma_t log-uniform in [0.1, 10] and c uniform in [0, 0.95] in 8^3-cell
blocks, block sources U(0, 1), per-group cross-section scaling 0.8..1.2,
vacuum boundaries.  The 32^3 / 96-angle / 16-group two-material workload is
measured beside it (`secondary`), together with per-angle designation, the
optional physics, the paper's 16^3 shape, second and third order, the AMT/BSP
grid over angles and groups, the learned start on 200 held-out instances and
the FP64 oracle on the host cores.

Prints one JSON line (rank 0).  `value` is cell-angle-group solves per second
over the timed steps with all inputs resident in HBM.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-angle-group solves/s per sweep; time-to-1e-6 learned vs plain start"
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 78.6      # MI355X, FP32 vector without packed instructions

# The paper's run-time table for its own shape (16^3 elements, 128 angles, 16
# groups, 25 sweeps): seconds on whole CPU nodes, for context only.
PAPER_SHAPE_CPU_S = {"AMT, AMD EPYC 9354 2x32 cores": 1.85, "AMT, Intel Xeon Gold 6430 2x32 cores": 1.99,
                     "AMT, NVIDIA Grace 2x72 cores": 1.09, "BSP, NVIDIA Grace 2x72 cores": 1.75}

# The same table's AMT columns at second and third order (AMD Genoa, Intel
# Sapphire Rapids, NVIDIA Grace nodes), seconds, for context only.
PAPER_HO_CPU_S = {2: {"AMT, AMD EPYC 9354 2x32 cores": 20.45, "AMT, Intel Xeon Gold 6430 2x32 cores": 15.15,
                      "AMT, NVIDIA Grace 2x72 cores": 5.87},
                  3: {"AMT, AMD EPYC 9354 2x32 cores": 80.15, "AMT, Intel Xeon Gold 6430 2x32 cores": 90.30,
                      "AMT, NVIDIA Grace 2x72 cores": 39.48}}

WORKLOADS = {
    "cfg2": (2, "32^3 jittered hex (32768 cells), 96 angles (3x4 product), 16 groups, two-material 4^3 blocks"),
    "cfg1": (1, "8^3 jittered hex (512 cells), 32 angles (2x2), 4 groups, sigma_t 1, c 0.5"),
    "cfg3": (3, "64^3 jittered hex (262144 cells), 256 angles (4x8), 64 groups, log-uniform 8^3 blocks"),
    "paper16": (0, "16^3 jittered hex (4096 cells), 128 angles (4x4), 16 groups, sigma_t 1, c 0.5"),
}


def bytes_per_task(n: int, A: int, A_o: int, G: int) -> float:
    """Algorithmic bytes per (cell, angle, group) solve of one source iteration.

    32 B written psi (8 FP32 dofs); 16 B read per interior inflow face, of
    which a cell of an n^3 grid has 3(n-1)/n per octant on average; 140 B per
    (cell, group) per iteration (source in, flux out, source update, cross
    section) over A angles; 120 B of cell geometry per (cell, octant) over
    A_o * G solves.
    """
    return 32.0 + 48.0 * (n - 1) / n + 140.0 / A + 120.0 / (A_o * G)


def flops_per_task(G: int) -> float:
    """Algorithmic FLOP per solve (an FMA counts two): A = B + sigma_t M (64 FMA),
    the inflow of three faces (48 FMA), unpivoted LU with forward and back
    substitution (200 FMA, 8 reciprocals, 36 multiplies), and the per-angle
    operator B = Omega.S - Omega.F_in (336 FMA per (cell, angle)) over G groups."""
    return 2.0 * (64 + 48 + 200) + 8 + 36 + 2.0 * 336 / G


def paper_shape(outer: int = 5, inner: int = 5):
    """The paper's timing shape (Section 3.6, its run-time table): 16^3 cells, 128
    angles, 16 groups, five outer and five inner iterations.  Groups are coupled
    by downscatter (each group keeps 60% of its scattering and passes the rest to
    later groups), so every outer iteration updates a cross-group source.  Also
    the same 25 sweeps as plain graph-captured source iterations."""
    import torch
    from paper_2510_11513_amd import inputs, snx
    cache = os.path.join(ROOT, "paper_2510_11513_amd", "tuning", "mi355x.jsonl")
    prob = inputs.config_problem(0)
    steps = outer * inner
    solves = prob.mesh.ncell * prob.nang * prob.mat.ngroup * steps
    # outer/inner iterations with the group-to-group matrix
    cm, sgg = inputs.split_scattering(prob.mat)
    p = snx.Problem.from_problem(prob, setup=False)
    p.set_group_scattering(cm, sgg)
    p.setup()
    p.tune(cache)                 # also picks the sweep mode
    mode = "bsp" if p.schedule()["mode"] == snx.SWEEP_BSP else "amt"
    phi = p.empty_phi()
    p.set_schedule(chunk=inner)
    p.solve_outer(outer, inner, 0.0, phi=phi)                  # warm-up (graph build)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = p.solve_outer(outer, inner, 0.0, phi=phi)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    p.close()
    # the same number of sweeps as plain source iterations (one graph replay)
    q = snx.Problem.from_problem(prob)
    q.tune(cache)
    phi = q.empty_phi()
    q.set_schedule(chunk=steps)
    q.solve(0.0, steps, phi=phi, allow_noconv=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    q.solve(0.0, steps, phi=phi, allow_noconv=True)
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t1
    q.close()
    return {"workload": f"16^3 jittered hex, 128 angles, 16 groups with downscatter, {outer} outer x {inner} inner "
                        f"iterations", "s": round(dt, 5), "solves_per_s": solves / dt,
            "last_outer_change": info["residual"], "sweep_mode": mode,
            "plain_25_sweeps_s": round(dt_plain, 5), "plain_solves_per_s": solves / dt_plain,
            "paper_cpu_s_context": PAPER_SHAPE_CPU_S}


def ho_flops_per_solve(order: int, G: int, inflow_faces: int = 3) -> float:
    """Algorithmic FLOP of one (cell, direction, group) system at order p (an FMA
    counts two), N = (p+1)^3 nodes, NF = (p+1)^2 per face: the rows
    sigma_t M + B (N^2 FMA), the inflow of three faces (NF^2 FMA each),
    unpivoted LU with the right-hand side (per step k, N-k-1 multipliers and
    (N-k-1)(N-k) FMA), back substitution (N(N-1)/2 FMA, N divisions), and the
    per-direction operator B = Omega.S - Omega.F_in (3 N^2 FMA) over G groups."""
    N, NF = (order + 1) ** 3, (order + 1) ** 2
    elim = sum((N - k - 1) * (1 + 2 * (N - k)) for k in range(N))
    back = N * (N - 1) + N
    return 2.0 * N * N + 2.0 * inflow_faces * NF * NF + elim + back + 6.0 * N * N / G


def higher_order(steps: int = 25):
    """Second and third order on the paper's timing shape (16^3 cells, 128
    angles, 16 groups; Section 3.6 and its run-time table): the level-by-level
    sweep kernels alone (HIP events) and 25 source iterations end to end.  The
    paper's 25 sweeps are five outer times five inner iterations with
    group coupling; these are 25 plain sweeps."""
    import torch
    from paper_2510_11513_amd import inputs, snx
    prob = inputs.config_problem(0)
    G = prob.mat.ngroup
    solves = prob.mesh.ncell * prob.nang * G
    out = {"workload": f"16^3 jittered hex, 128 angles, 16 groups, {steps} source iterations"}
    for order in (2, 3):
        print(f"[bench] order {order}", file=sys.stderr, flush=True)
        p = snx.Problem.from_problem(prob, order=order)
        phi = p.empty_phi()
        p.solve(0.0, 2, phi=phi, allow_noconv=True)       # warm-up
        ms = p.profile_sweep(5, phi_in=phi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.solve(0.0, steps, phi=phi, allow_noconv=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        p.close()
        fps = ho_flops_per_solve(order, G)
        tflops = fps * solves / (ms * 1e-3) / 1e12
        out[f"order{order}"] = {
            "nodes": (order + 1) ** 3, "sweep_ms": round(ms, 3), "solves_per_s": solves / (ms * 1e-3),
            "unknowns_per_s": solves * (order + 1) ** 3 / (ms * 1e-3),
            "s_for_25": round(dt * 25.0 / steps, 4),
            "roofline": {"bound": "alu", "achieved": round(tflops, 2), "peak": FP32_VALU_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tflops / FP32_VALU_PEAK_TFLOPS, 4),
                         "flops_per_solve": round(fps, 1)},
            "paper_cpu_s_context": PAPER_HO_CPU_S[order]}
    return out


def per_angle(prob, threads: int, wg_per_cu: int, ms_octant: float, its_octant: int, sweeps: int):
    """The same workload under per-angle designation (each direction's own inflow
    faces): in the octant's order with every face against it lagged, and in each
    direction's own order with only the faces that close cycles lagged (level by
    level, and as the dependency-driven unit sweep).  Sweep time, the designation counts, and source iterations to the
    workload's tolerance beside the per-octant count."""
    from paper_2510_11513_amd import snx
    p = snx.Problem.from_problem(prob, setup=False, designation=snx.DESIGNATION_ANGLE)
    p.set_schedule(threads=threads, wg_per_cu=wg_per_cu)
    p.setup()
    phi = p.sweep(None)
    ms = p.profile_sweep(sweeps, phi_in=phi)
    ds = p.designation_stats()
    _, info = p.solve(prob.tol, 5000)
    p.close()
    # each direction in its own order, only the faces that close cycles lagged
    q = snx.Problem.from_problem(prob, setup=False, designation=snx.DESIGNATION_DIRECTION)
    q.set_schedule(threads=threads)
    t0 = time.perf_counter()
    q.setup()
    t_setup = time.perf_counter() - t0
    phi = q.sweep(None)
    ms_dir = q.profile_sweep(sweeps, phi_in=phi)
    dsd = q.designation_stats()
    _, info_dir = q.solve(prob.tol, 5000)
    ms_units, ust = None, None
    if prob.mat.ngroup <= 64:   # the dependency-driven unit sweep (same bits; slower, kept for comparison)
        q.set_sweep_mode(snx.SWEEP_AMT)
        ms_units = q.profile_sweep(sweeps, phi_in=phi)
        ust = q.sweep_stats()
    q.close()
    return {"sweep_ms": round(ms, 4), "per_octant_sweep_ms": round(ms_octant, 4),
            "ratio": round(ms / ms_octant, 3), "differing_triples": ds["differing"],
            "lagged_triples": ds["lagged"], "tasks_with_difference": ds["tasks"],
            "iterations_to_tol": info["iterations"], "per_octant_iterations_to_tol": its_octant,
            "tol": prob.tol,
            "per_direction_order": {"sweep_ms": round(ms_dir, 4), "ratio": round(ms_dir / ms_octant, 3),
                                    "lagged_triples": dsd["lagged"], "iterations_to_tol": info_dir["iterations"],
                                    "setup_s": round(t_setup, 3), "levels": "one launch per level",
                                    "unit_sweep_ms": None if ms_units is None else round(ms_units, 4),
                                    "unit_sweep_rounds": None if ust is None else ust["grid"],
                                    "unit_sweep_carried": None if ust is None else ust["continued"]}}


def extensions(prob, threads: int, wg_per_cu: int, steps: int):
    """Per-iteration cost of the optional physics on the same workload: each
    variant is set up in the benchmark's schedule and timed over `steps`
    graph-captured source iterations (wall clock around one solve call)."""
    import numpy as np
    import torch
    from paper_2510_11513_amd import inputs, snx
    sigl = lambda L: prob.mat.sigma_s[:, :, None] * 0.5 ** np.arange(1, L + 1)[None, None, :]
    variants = {
        "plain": lambda p: None,
        "reflective_6_planes": lambda p: p.set_reflective(63),
        "anisotropic_L1": lambda p: p.set_anisotropy(sigl(1)),
        "anisotropic_L3": lambda p: p.set_anisotropy(sigl(3)),
        "group_to_group_matrix": lambda p: p.set_group_scattering(*inputs.split_scattering(prob.mat)),
    }
    out = {}
    for name, configure in variants.items():
        p = snx.Problem.from_problem(prob, setup=False)
        configure(p)
        p.set_schedule(threads=threads, wg_per_cu=wg_per_cu, chunk=steps)
        p.setup()
        phi = p.empty_phi()
        p.solve(0.0, steps, phi=phi, allow_noconv=True)         # graph build and warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.solve(0.0, steps, phi=phi, allow_noconv=True)
        torch.cuda.synchronize()
        out[name + "_ms_per_iteration"] = round((time.perf_counter() - t0) / steps * 1e3, 4)
        p.close()
    return out


def bsp_grid(n: int = 16, sweeps: int = 10):
    """AMT over BSP across angle and group counts (the paper's comparison in
    Section 3.6, its figure of AMT speed-up over BSP): a 16^3 jittered grid
    (sigma_t 1, c 0.5) swept with the dependency-driven scheme and with the
    level-synchronous one, each at its best schedule of a small search (AMT:
    threads 64, 128, 256 x workgroups per CU at occupancy or 2; BSP: threads
    64, 128, 256); times are the sweep kernel alone (HIP events over `sweeps`
    sweeps after one untimed sweep)."""
    import numpy as np
    import torch
    from paper_2510_11513_amd import inputs, snx
    rows = []
    for npol, naz in ((2, 2), (2, 4), (4, 4), (4, 8)):
        for G in (4, 8, 16, 32, 64):
            rng = np.random.default_rng(1000 * n + 10 * npol * naz + G)
            mesh = inputs.make_mesh(n, 0.2, rng=rng)
            mat = inputs.materials_uniform(mesh, G, 1.0, 0.5, 1.0, scaled=True)
            prob = inputs.Problem(f"bsp_n{n}_a{npol * naz}_g{G}", mesh, mat, npol, naz, 1e-6)
            p = snx.Problem.from_problem(prob)
            phi = p.sweep(None)
            torch.cuda.synchronize()
            best = {snx.SWEEP_AMT: (1e300, None), snx.SWEEP_BSP: (1e300, None)}
            for mode, wgs in ((snx.SWEEP_AMT, (64, 2)), (snx.SWEEP_BSP, (64,))):
                p.set_sweep_mode(mode)
                for th in (64, 128, 256):
                    if th < G:
                        continue
                    for wg in wgs:      # 64: capped by occupancy
                        p.set_schedule(threads=th, wg_per_cu=wg)
                        p.sweep(phi)
                        ms = p.profile_sweep(sweeps, phi_in=phi)
                        if ms < best[mode][0]:
                            best[mode] = (ms, (th, wg))
            p.close()
            (ms_amt, sched), (ms_bsp, sched_bsp) = best[snx.SWEEP_AMT], best[snx.SWEEP_BSP]
            rows.append({"angles_per_octant": npol * naz, "groups": G, "amt_ms": round(ms_amt, 4),
                         "bsp_ms": round(ms_bsp, 4), "bsp_over_amt": round(ms_bsp / ms_amt, 3),
                         "amt_schedule": list(sched), "bsp_threads": sched_bsp[0]})
    return {"workload": f"{n}^3 jittered hex, sigma_t 1, c 0.5; angles per octant x groups", "rows": rows}


def angle_blocks(prob, ms_whole: float, sweeps: int = 20):
    """Tasks of one (cell, octant, block of the octant's angles): the problem is
    swept as a batch of angle-block sub-problems, which the same task machinery
    runs with dependency counters per block, so a block's tasks traverse the
    DAG on their own (the granularity of Section 3.4 and Algorithm 1, finer
    than a whole octant).  Each split at its best width of 64, 128, 192, 256
    threads; sweep kernel alone (HIP events)."""
    import numpy as np
    import torch
    from paper_2510_11513_amd import snx
    om, w = snx.quadrature_product(prob.npolar, prob.nazim)
    A = om.shape[0] // 8
    rows = [{"blocks": 1, "angles_per_block": A, "tasks": 8 * prob.mesh.ncell, "sweep_ms": round(ms_whole, 4),
             "over_whole": 1.0}]
    for nb in (2, 3, 4):
        if A % nb:
            continue
        ab = A // nb
        subs = []
        for b in range(nb):
            idx = np.concatenate([o * A + np.arange(b * ab, (b + 1) * ab) for o in range(8)])
            subs.append(snx.Problem.from_problem(prob, quadrature=(om[idx].copy(), w[idx].copy())))
        bt = snx.Batch(subs)
        best = (1e300, 0)
        for th in (64, 128, 192, 256):
            if th < prob.mat.ngroup:
                continue
            bt.set_schedule(threads=th)
            bt.sweep()
            torch.cuda.synchronize()
            ms = bt.profile_sweep(sweeps)
            best = min(best, (ms, th))
        tasks = bt.stats()["tasks"]
        bt.close()
        for q in subs:
            q.close()
        rows.append({"blocks": nb, "angles_per_block": ab, "tasks": tasks, "sweep_ms": round(best[0], 4),
                     "threads": best[1], "over_whole": round(best[0] / ms_whole, 3)})
    return {"rows": rows}


def kernel_hash() -> str:
    path = os.path.join(ROOT, "paper_2510_11513_amd", "csrc", "k_sweep.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary, if still current."""
    path = os.path.join(ROOT, "profiles", f"k_sweep_{workload}_pmc.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    h = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not h or not t or h.group(1) != kernel_hash():
        return None
    return float(t.group(1))


def host_threads() -> int:
    """Host threads for the oracle: the OpenMP thread count the environment sets, else the CPU count."""
    return max(1, int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1))


def sample_pairs(nang: int, G: int, count: int):
    """`count` (direction, group) pairs spread over every octant and group, in a fixed order."""
    per = nang // 8
    return [((k % 8) * per + (k * 5) % per, (k * 7) % G) for k in range(count)]


def oracle_rate(o, pairs, threads: int):
    """Solves/s of the FP64 oracle sweeping the given (direction, group) pairs
    from a zero flux, on `threads` host threads (each pair is one whole sweep
    of the mesh for that direction and group; pairs are independent)."""
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.perf_counter()
    if threads == 1:
        for n, g in pairs:
            o.sweep_angle(None, n, g)
    else:
        with ThreadPoolExecutor(threads) as ex:   # ctypes releases the GIL during each sweep
            list(ex.map(lambda ng: o.sweep_angle(None, ng[0], ng[1]), pairs))
    dt = time.perf_counter() - t0
    return len(pairs) * o.ncell / dt, dt


def cpu_baseline(prob, budget_s: float = 8.0):
    """The FP64 oracle (test infrastructure), untuned, on a bounded sample of the
    same workload: whole-mesh sweeps of sampled (direction, group) pairs, first
    on one host thread, then on every host thread at once.  Solves/s per
    sweep extrapolate to the workload's C * A * G solves."""
    import oracle
    o = oracle.Oracle.from_problem(prob)
    C, G, nang = prob.mesh.ncell, prob.mat.ngroup, prob.nang
    threads = host_threads()
    per_pair = oracle_rate(o, sample_pairs(nang, G, 1), 1)[1]      # one pair, also a warm-up
    n1 = max(2, min(64, int(budget_s / max(per_pair, 1e-6))))
    r1, t1 = oracle_rate(o, sample_pairs(nang, G, n1), 1)
    nt = max(threads, min(8 * threads, int(budget_s * threads / max(per_pair, 1e-6))))
    rt, tt = oracle_rate(o, sample_pairs(nang, G, nt), threads)
    del o
    solves = C * nang * G
    return {"value": rt, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{nt} whole-mesh FP64 sweeps of sampled (direction, group) pairs of the same problem "
                      f"({nt * C:.3g} solves, {tt:.2f} s) on {threads} host threads; per sweep of all "
                      f"{solves:.3g} solves this extrapolates to {solves / rt:.1f} s",
            "one_thread": {"value": r1, "pairs": n1, "s": round(t1, 3),
                           "extrapolated_s_per_sweep": round(solves / r1, 1)},
            "extrapolated_s_per_sweep": round(solves / rt, 2)}


def oracle_timings(budget_s: float = 3.0):
    """The same sampled oracle timing, 1 thread and all threads, on the 8^3,
    32^3 and the paper's 16^3 workloads."""
    import oracle
    from paper_2510_11513_amd import inputs
    threads = host_threads()
    out = {"threads": threads}
    for name in ("cfg1", "cfg2", "paper16"):
        prob = inputs.config_problem(WORKLOADS[name][0])
        o = oracle.Oracle.from_problem(prob)
        nang, G = prob.nang, prob.mat.ngroup
        per_pair = oracle_rate(o, sample_pairs(nang, G, 1), 1)[1]
        n1 = max(4, min(nang * G, int(budget_s / max(per_pair, 1e-6))))
        r1, _ = oracle_rate(o, sample_pairs(nang, G, n1), 1)
        nt = max(threads, min(nang * G, int(budget_s * threads / max(per_pair, 1e-6))))
        rt, _ = oracle_rate(o, sample_pairs(nang, G, nt), threads)
        solves = prob.mesh.ncell * nang * G
        out[name] = {"one_thread_solves_per_s": r1, "all_threads_solves_per_s": rt, "pairs": [n1, nt],
                     "s_per_sweep_one_thread": round(solves / r1, 3),
                     "s_per_sweep_all_threads": round(solves / rt, 3)}
        del o
    return out


def learned_start(count: int):
    """Time to 1e-6 from the trained network's start vs zero start (and the Q/sigma_a control),
    on the first `count` held-out instances of the high-scattering workload, inference included."""
    from paper_2510_11513_amd import learned, snx
    if not os.path.exists(learned.WEIGHTS):
        return None
    net = snx.Gnn(0, learned.LAYERS)
    net.load_file(learned.WEIGHTS)
    t0 = time.perf_counter()

    def log(rec):
        if rec["done"] % 25 == 0 or rec["done"] == count:
            print(f"[bench] learned start: {rec['done']} of {count} instances", file=sys.stderr, flush=True)

    recs = learned.evaluate(net, list(range(count)), log=log)
    net.close()
    summ = learned.summarize(recs)
    r = lambda k: round(summ[k], 4)
    return {"workload": "32^3 jittered hex, 96 angles, 16 groups, sigma_t log-uniform [0.1, 10] and c in "
                        "[0.9, 0.99] in 4^3 blocks; tol 1e-6", "instances": count,
            "wall_ratio_learned_over_zero_median": r("b/a_wall_median"),
            "wall_ratio_learned_over_zero_mean": r("b/a_wall_mean"),
            "iter_ratio_learned_over_zero_median": r("b/a_iterations_median"),
            "wall_ratio_control_over_zero_median": r("c/a_wall_median"),
            "iter_ratio_control_over_zero_median": r("c/a_iterations_median"),
            "zero_start_iterations_median": summ["a_iterations_median"],
            "zero_start_ms_median": round(summ["a_wall_ms_median"], 2),
            "learned_ms_median": round(float(sorted(x["b_ms"] for x in recs)[len(recs) // 2]), 2),
            "predict_ms_median": round(float(sorted(x["predict_ms"] for x in recs)[len(recs) // 2]), 3),
            "learned_vs_zero_max_rel_diff": summ["b_vs_a_max"], "control_vs_zero_max_rel_diff": summ["c_vs_a_max"],
            "s": round(time.perf_counter() - t0, 1)}


def phase_stats(p):
    """One sweep with the per-phase shader-clock statistics on: where a
    workgroup's cycles go (queue wait, staging, operator build, solve,
    publish), and the queue polls that found no ready task."""
    p.set_sweep_stats(True)
    p.sweep(p.empty_phi())
    st = p.sweep_stats()
    p.set_sweep_stats(False)
    tot = max(1, sum(st["cycles"].values()))
    return {"tasks": st["tasks"], "continued": st["continued"], "empty_polls": st["empty_polls"],
            "cycle_share": {k: round(v / tot, 4) for k, v in st["cycles"].items()},
            "cycles_per_task": round(tot / max(1, st["tasks"]), 1)}


def measure_sweep(p, prob, sweeps: int):
    """Sweep-kernel duration (HIP events on the library's stream), the HBM and
    VALU rooflines, and the bulk-synchronous comparator in the same schedule."""
    from paper_2510_11513_amd import snx
    C, G, nang = prob.mesh.ncell, prob.mat.ngroup, prob.nang
    phi = p.sweep(None)
    ms_sweep = p.profile_sweep(sweeps, phi_in=phi)
    stats = p.sweep_stats()
    solves = C * nang * G
    bpt = bytes_per_task(prob.mesh.n, nang, nang // 8, G)
    achieved = bpt * solves / (ms_sweep * 1e-3) / 1e9
    tuned_mode = p.schedule()["mode"]
    p.set_sweep_mode(snx.SWEEP_BSP)
    ms_bsp = p.profile_sweep(sweeps, phi_in=phi)
    p.set_sweep_mode(snx.SWEEP_AMT)
    ms_amt = p.profile_sweep(sweeps, phi_in=phi) if tuned_mode == snx.SWEEP_BSP else ms_sweep
    p.set_sweep_mode(tuned_mode)
    fpt = flops_per_task(G)
    tflops = fpt * solves / (ms_sweep * 1e-3) / 1e12
    return ms_sweep, stats, {
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": "k_sweep", "kernel_ms": round(ms_sweep, 4),
                     "bytes_per_solve": round(bpt, 2), "solves_per_launch": solves},
        "bsp_comparator": {"sweep_ms": round(ms_bsp, 4), "amt_sweep_ms": round(ms_amt, 4),
                           "bsp_over_amt": round(ms_bsp / ms_amt, 3)},
        "valu": {"achieved": round(tflops, 2), "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "frac": round(tflops / FP32_VALU_PEAK_TFLOPS, 4), "flops_per_solve": round(fpt, 1)}}


def secondary(name: str, tune_cache: str, args):
    """The 32^3 workload beside the headline: sweep kernel, rooflines, BSP
    comparator, phase statistics, one graph-captured source iteration,
    per-angle designation and the optional physics."""
    import torch
    from paper_2510_11513_amd import inputs, snx
    cfg, desc = WORKLOADS[name]
    prob = inputs.config_problem(cfg)
    p = snx.Problem.from_problem(prob)
    tuned = p.tune(tune_cache)
    sweeps = 20
    ms_sweep, stats, meas = measure_sweep(p, prob, sweeps)
    phi = p.empty_phi()
    p.set_schedule(chunk=sweeps)
    p.solve(0.0, sweeps, phi=phi, allow_noconv=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.solve(0.0, sweeps, phi=phi, allow_noconv=True)
    torch.cuda.synchronize()
    ms_it = (time.perf_counter() - t0) / sweeps * 1e3
    solves = prob.mesh.ncell * prob.nang * prob.mat.ngroup
    out = {"workload": f"{name}: {desc}", "solves_per_step": solves, "ms_per_iteration": round(ms_it, 4),
           "solves_per_s": solves / (ms_it * 1e-3), "sweep_threads": stats["threads"],
           "sweep_wg_per_cu_cap": tuned[1],
           "sweep_mode": "bsp" if p.schedule()["mode"] == snx.SWEEP_BSP else "amt", **meas,
           "phases": phase_stats(p)}
    out["roofline"]["traffic"] = measured_traffic(name)
    if args.per_angle:
        print("[bench] per-angle designation", file=sys.stderr, flush=True)
        _, info_oct = p.solve(prob.tol, 5000)
        out["per_angle"] = per_angle(prob, stats["threads"], tuned[1], ms_sweep, info_oct["iterations"], sweeps)
    if args.angle_blocks:
        print("[bench] angle blocks", file=sys.stderr, flush=True)
        out["angle_blocks"] = angle_blocks(prob, ms_sweep)
    p.close()
    if args.extensions:
        print("[bench] optional physics", file=sys.stderr, flush=True)
        out["extensions"] = extensions(prob, stats["threads"], tuned[1], 10)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cfg3", choices=sorted(WORKLOADS))
    ap.add_argument("--secondary", default="cfg2", choices=sorted(WORKLOADS) + ["none"],
                    help="workload measured beside the headline (per-angle designation and optional physics run "
                         "on it)")
    ap.add_argument("--threads", type=int, default=0, help="sweep workgroup size (0 = library default)")
    ap.add_argument("--wg-per-cu", type=int, default=0)
    ap.add_argument("--no-tune", action="store_true", help="skip the schedule autotuner (library default schedule)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2510_11513_amd", "tuning", "mi355x.jsonl"),
                    help="autotuner cache (JSON lines); a hit reuses the recorded schedule without timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=8.0,
                    help="seconds of oracle work per thread count in the CPU baseline")
    ap.add_argument("--oracle-timings", type=int, default=1,
                    help="also time the oracle at 1 and all threads on the 8^3, 32^3 and 16^3 workloads (0 = skip)")
    ap.add_argument("--learned", type=int, default=200,
                    help="held-out high-scattering instances for the learned-start comparison (0 = skip)")
    ap.add_argument("--paper-shape", type=int, default=1, help="also time the paper's 25-sweep 16^3 shape (0 = skip)")
    ap.add_argument("--per-angle", type=int, default=1,
                    help="also time the secondary workload under per-angle designation (0 = skip)")
    ap.add_argument("--angle-blocks", type=int, default=1,
                    help="also time angle-block tasks on the secondary workload (0 = skip)")
    ap.add_argument("--higher-order", type=int, default=1,
                    help="also time second and third order on the paper's 16^3 shape (0 = skip)")
    ap.add_argument("--extensions", type=int, default=1,
                    help="also time reflective planes, anisotropy and group coupling on the secondary workload "
                         "(0 = skip)")
    ap.add_argument("--bsp-grid", type=int, default=1,
                    help="also compare AMT and BSP over angles and groups on a 16^3 grid (0 = skip)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference kernel for HBM counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(sharding is described in the design notes); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_11513_amd import inputs, snx

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    cfg, desc = WORKLOADS[args.workload]
    prob = inputs.config_problem(cfg)
    C, G, nang = prob.mesh.ncell, prob.mat.ngroup, prob.nang
    p = snx.Problem.from_problem(prob, setup=False)
    if args.threads or args.wg_per_cu:
        p.set_schedule(threads=args.threads, wg_per_cu=args.wg_per_cu)
    t_setup = time.perf_counter()
    p.setup()
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    tuned = None
    if not (args.no_tune or args.threads or args.wg_per_cu):
        tuned = p.tune(args.tune_cache)   # the library's autotuner (cache hit: the recorded schedule)
    print(f"[bench] {args.workload}: setup {t_setup:.2f} s; schedule {tuned}; warmup {args.warmup}, "
          f"steps {args.steps}", file=sys.stderr, flush=True)

    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    phi = p.empty_phi()
    if args.warmup:
        p.set_schedule(chunk=args.warmup)     # one graph replay, no early-exit dispatches
        p.solve(0.0, args.warmup, phi=phi, allow_noconv=True)
    p.set_schedule(chunk=args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi, info = p.solve(0.0, args.steps, phi=phi, allow_noconv=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert info["iterations"] == args.steps, info
    solves_per_step = C * nang * G
    value = solves_per_step * args.steps / dt
    print(f"[bench] timed {args.steps} steps in {dt:.3f} s; residual {info['residual']:.3e}", file=sys.stderr,
          flush=True)

    # live duration of the dominant kernel (the sweep) from HIP events on its stream
    ms_sweep, stats, meas = measure_sweep(p, prob, max(5, min(args.steps, 20)))
    meas["roofline"]["traffic"] = measured_traffic(args.workload)
    out = {"metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{args.workload}: {desc}", "cells": C, "angles": nang, "groups": G,
                      "solves_per_step": solves_per_step, "sweep_grid": stats["grid"],
                      "sweep_threads": stats["threads"], "sweep_wg_per_cu_cap": tuned[1] if tuned else None,
                      "sweep_mode": "bsp" if p.schedule()["mode"] == snx.SWEEP_BSP else "amt",
                      "continued_tasks": stats["continued"], "setup_s": round(t_setup, 3)},
           "roofline": meas.pop("roofline"), **meas}
    out["phases"] = phase_stats(p)
    p.close()
    del phi
    torch.cuda.empty_cache()
    if args.secondary != "none" and args.secondary != args.workload:
        print(f"[bench] secondary workload {args.secondary}", file=sys.stderr, flush=True)
        out["secondary"] = secondary(args.secondary, args.tune_cache, args)
    if args.paper_shape:
        print("[bench] paper shape", file=sys.stderr, flush=True)
        out["paper_shape"] = paper_shape()
    if args.higher_order:
        out["higher_order"] = higher_order()
    if args.bsp_grid:
        print("[bench] AMT/BSP grid", file=sys.stderr, flush=True)
        out["bsp_grid"] = bsp_grid()
    if args.learned > 0:
        print("[bench] learned vs zero start", file=sys.stderr, flush=True)
        out["learned"] = learned_start(args.learned)
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_budget)
        if args.oracle_timings:
            out["oracle_timings"] = oracle_timings()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
