"""Central finite differences (h = 1e-4 A) of the oracle's weighted slab loss
on the 64 sampled atoms (locals and ghosts) of the 1/16 and 1/32 slabs of the
15,668-atom protein frame: pins the oracle gradient that the GPU autograd
adjoint is compared with at the same atoms (F = -dE/dx, Eq. (2); ghost
gradients per Eq. (7)).

Only centres within rcut of the displaced atom change their energy (strict
locality, pinned separately), so each difference sums w_i e_i over the local
centres within rcut + 1e-3 A of it, the atom itself included when it is local.
FP64 rounding noise of a difference is ~1e-16 |sum| / h, about 1e-11 here;
the O(h^2) truncation error of this strongly curved random model is ~1e-6.
"""

import numpy as np
import pytest

import oracle_samples as osm
from oracle import dpa1_oracle as orc
from paper_2604_07276_amd import synth

RC = 6.0
SEL = 120
H = 1e-4
TOL = 1e-5


@pytest.mark.slow
@pytest.mark.parametrize("n_slabs", [16, 32])
def test_slab_gradient_central_differences(oracle_model, n_slabs):
    protein = synth.protein_system(0)
    box = protein.box
    x, t, nloc, nghost = osm.slab_case(protein.coords, protein.types, box[0, 0], n_slabs)
    w = np.random.default_rng(n_slabs).normal(size=nloc)
    atoms = osm.slab_sample(nloc, nghost, x, box, seed=n_slabs)
    cs = osm.centres_seeing(x, box, nloc, atoms)
    pr = orc.evaluate_centers(oracle_model, x, t, box, RC, SEL, cs)
    grad = osm.weighted_gradient(pr, atoms, w)
    near_lists = orc.neighbor_list(x, box, RC + 1e-3, atoms)
    fd = np.zeros_like(grad)
    for q, a in enumerate(atoms):
        near = [int(j) for j in near_lists[q] if j < nloc]
        if a < nloc:
            near.append(int(a))
        near = np.array(sorted(near), dtype=np.int64)
        for c in range(3):
            es = []
            for sgn in (1.0, -1.0):
                xd = x.copy()
                xd[a, c] += sgn * H
                r = orc.evaluate_centers(oracle_model, xd, t, box, RC, SEL, near)
                es.append(float(np.dot(w[near], r.atom_energy)))
            fd[q, c] = (es[0] - es[1]) / (2.0 * H)
    err = np.abs(fd - grad).max()
    print(f"[slab 1/{n_slabs} FD] {nloc} locals + {nghost} ghosts, 64 atoms "
          f"({np.sum(atoms >= nloc)} ghosts): max|FD - grad| = {err:.2e} "
          f"(|grad|max = {np.abs(grad).max():.3e})")
    assert err <= TOL
    # the sampled ghosts carry gradient: the check is not vacuous there
    gmag = np.abs(grad[atoms >= nloc]).max(axis=1)
    assert np.all(gmag > 0) and np.median(gmag) > 1e-4
