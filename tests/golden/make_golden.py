"""Writes the stored expected values under tests/golden/ from the FP64 oracle only.

Run from the repository root:  python -m tests.golden.make_golden
"""
import itertools
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def tiny_problem():
    import oracle
    from paper_2510_11513_amd import inputs
    m = inputs.make_mesh(3, 0.2, seed=123)
    mat = inputs.materials_uniform(m, 2, 1.0, 0.5, 1.0, scaled=True)
    om, w = oracle.quadrature(2, 2)
    return oracle.Oracle(m.xyz, m.cell_vert, om, w, mat.sigma_t, mat.sigma_s, mat.q), 1e-13


def main():
    o, tol = tiny_problem()
    phi = o.solve(tol, 500)["phi"]
    np.savetxt(os.path.join(HERE, "tiny_solve.txt"), o.integrated_flux(phi).ravel(), fmt="%.17e",
               header="integrated flux (Eq. 3) per group: [sum of dofs, 1^T M phi]; 3^3 mesh seed 123, "
                      "2x2 quadrature, sigma_t scaled 0.8..1.2, c 0.5, Q 1, converged to 1e-13")
    n = 16
    hist = [sum(1 for i, j, k in itertools.product(range(n), repeat=3) if i + j + k == l) for l in range(3 * n - 2)]
    with open(os.path.join(HERE, "levels_16cubed.txt"), "w") as fh:
        fh.write(" ".join(map(str, hist)) + "\n# elements per t-level of the 16x16x16 grid "
                 "(the paper's benchmark mesh; Fig. 4 compares these against core counts): "
                 "#{(i,j,k): i+j+k = l}, l = 0..45\n")


if __name__ == "__main__":
    main()
