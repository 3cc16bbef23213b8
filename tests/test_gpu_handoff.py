"""The angular-flux hand-off of the dependency-driven sweep, at full size (GPU).

In the dependency-driven sweep a task reads its upwind neighbours' angular
flux as soon as their counters say it is there, across CUs and XCDs; in the
level-synchronous comparator every hand-off crosses a kernel boundary.  Both
run the same task code, so any read of a value that had not yet arrived would
show as a difference in the bits.  On the 32^3 / 96-angle / 16-group workload,
in four schedules (one-round and multi-round tasks, with and without an
occupancy cap), ten chained sweeps must give the comparator's bits, scalar
flux and sampled angular fluxes alike.
"""
import numpy as np
import pytest

from paper_2510_11513_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("threads,wg", [(192, 0), (256, 2), (64, 0), (128, 4)])
def test_dependency_driven_sweeps_give_the_level_synchronous_bits(threads, wg):
    import torch
    from paper_2510_11513_amd import snx
    prob = inputs.config_problem(2)
    p = snx.Problem.from_problem(prob)
    p.set_schedule(threads=threads, wg_per_cu=wg)
    print(f"[case] hand-off 32^3/96/16 threads={threads} wg_per_cu={wg}", flush=True)
    rng = np.random.default_rng(threads + wg)
    phi = torch.from_numpy(rng.uniform(0.0, 2.0, (prob.mesh.ncell, prob.mat.ngroup, 8)).astype(np.float32)).cuda()
    pairs = [(int(o * 12 + rng.integers(12)), int(rng.integers(prob.mat.ngroup))) for o in range(8)]
    for it in range(10):
        p.set_sweep_mode(snx.SWEEP_AMT)
        amt = p.sweep(phi)
        psi_amt = [p.psi(n, g).cpu().numpy() for n, g in pairs]
        st = p.sweep_stats()
        assert st["abort"] == 0 and st["tasks"] == 8 * prob.mesh.ncell, st
        p.set_sweep_mode(snx.SWEEP_BSP)
        bsp = p.sweep(phi)
        psi_bsp = [p.psi(n, g).cpu().numpy() for n, g in pairs]
        torch.cuda.synchronize()
        assert torch.equal(amt, bsp), (threads, wg, it)
        for (n, g), a, b in zip(pairs, psi_amt, psi_bsp):
            assert np.array_equal(a, b), (threads, wg, it, n, g)
        phi = amt          # the next sweep starts from this one's flux
    print(f"[case] hand-off threads={threads} wg_per_cu={wg}: 10 sweeps bit-identical, "
          f"{st['continued']} of {st['tasks']} tasks continued in place", flush=True)
    p.close()
