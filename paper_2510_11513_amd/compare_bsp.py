"""AMT over BSP on one GPU across angle and group counts (the comparison of the
paper's Section 3.6: a 16^3 grid swept with the many-task scheme and with the
bulk-synchronous one, over a range of angles per octant and energy groups).

    python -m paper_2510_11513_amd.compare_bsp [--n 16] [--sweeps 10]

Both schemes run the same task code.  Each is timed at its best schedule of
a small search (AMT: threads 64, 128, 256 x workgroups per CU at occupancy or
2; BSP: threads 64, 128, 256); a time is the sweep kernel alone (HIP events
over `sweeps` sweeps, after one untimed sweep).  Prints a table and one JSON
line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# (polar, azimuthal) nodes per octant: 4, 8, 16 and 32 angles per octant
QUADRATURES = [(2, 2), (2, 4), (4, 4), (4, 8)]
GROUPS = [4, 8, 16, 32, 64]


def run(n: int, sweeps: int):
    import numpy as np
    import torch
    from paper_2510_11513_amd import inputs, snx

    rows = []
    for npol, naz in QUADRATURES:
        for G in GROUPS:
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
            ms_amt, sched_amt = best[snx.SWEEP_AMT]
            ms_bsp, sched_bsp = best[snx.SWEEP_BSP]
            solves = mesh.ncell * prob.nang * G
            rows.append({"angles_per_octant": npol * naz, "groups": G, "amt_schedule": sched_amt,
                         "bsp_threads": sched_bsp[0], "amt_ms": round(ms_amt, 4), "bsp_ms": round(ms_bsp, 4),
                         "speedup_amt_over_bsp": round(ms_bsp / ms_amt, 3),
                         "amt_solves_per_s": solves / (ms_amt * 1e-3)})
            print(f"angles/octant {npol * naz:3d} groups {G:3d}: AMT {ms_amt:8.3f} ms {sched_amt}  "
                  f"BSP {ms_bsp:8.3f} ms (threads {sched_bsp[0]})  speedup {ms_bsp / ms_amt:5.2f}", flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=16, help="mesh edge (cells per axis)")
    ap.add_argument("--sweeps", type=int, default=10)
    args = ap.parse_args()
    rows = run(args.n, args.sweeps)
    print(json.dumps({"mesh": f"{args.n}^3", "rows": rows}), flush=True)


if __name__ == "__main__":
    main()
