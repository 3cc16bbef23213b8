"""The integrated flux through the library's fixed device scratch
(snx_integrated_flux_noalloc, for callers that cannot allocate) against the
allocating entry point snx_integrated_flux, which runs the same kernels."""
import numpy as np
import pytest

import oracle
from paper_2510_11513_amd import inputs, snx

pytestmark = pytest.mark.gpu


def _swept(prob):
    import torch
    p = snx.Problem.from_problem(prob)
    phi = p.sweep(p.sweep(None))
    torch.cuda.synchronize()
    return p, phi


def test_noalloc_integrated_flux_matches_the_allocating_entry_point():
    """Two calls in a row on one device, the second on a smaller problem (the
    scratch keeps the first call's larger contents)."""
    for prob in (inputs.config_problem(2, n=16), inputs.config_problem(1, n=5)):
        print(f"noalloc integrated flux: {prob.mesh.ncell} cells x {prob.mat.ngroup} groups", flush=True)
        p, phi = _swept(prob)
        ref = p.integrated_flux(phi)
        got = p.integrated_flux_noalloc(phi)
        assert np.array_equal(got, ref)
        assert np.array_equal(p.integrated_flux_noalloc(phi), ref)
        # and both against the FP64 oracle on the same flux (the GPU reads FP32 mass matrices)
        want = oracle.Oracle.from_problem(prob).integrated_flux(phi.cpu().double().numpy())
        assert np.abs(got - want).max() <= 1e-6 * np.abs(want).max()
        p.close()


def test_noalloc_integrated_flux_rejects_problems_beyond_its_scratch():
    """1331 cells x 256 groups need (1331 + 1) * 256 * 4 doubles of partial sums,
    more than the 2^20 of the fixed array."""
    mesh = inputs.make_mesh(11, 0.2, seed=1)
    prob = inputs.Problem("wide", mesh, inputs.materials_uniform(mesh, 256, 1.0, 0.5, 1.0), 1, 1, 1e-6)
    print(f"noalloc size limit: {mesh.ncell} cells x 256 groups", flush=True)
    p, phi = _swept(prob)
    with pytest.raises(snx.SnxError) as err:
        p.integrated_flux_noalloc(phi)
    assert err.value.code == -1
    assert p.integrated_flux(phi).shape == (256, 2)
    p.close()
