"""Domains of the slab sweep (the per-rank work behind Eq. (8)): host-side
construction on the CPU, and on the GPU the paper's 2 r_c halo scheme, whose
forces on the slab's own atoms need no reduction (Sec. IV-A)."""

import numpy as np
import pytest

from paper_2604_07276_amd import slab_sweep, synth


@pytest.fixture(scope="module")
def frame():
    return synth.protein_system(0)


@pytest.mark.parametrize("n_p", [2, 8, 32])
def test_domains_partition(frame, n_p):
    n = len(frame.coords)
    c1, t1, nloc1, ng1 = slab_sweep.domain(frame, n_p, "rc")
    c2, t2, nloc2, ng2 = slab_sweep.domain(frame, n_p, "2rc")
    local, _ = synth.slab_partition(frame.coords, float(frame.box[0, 0]), n_p, 0, slab_sweep.RCUT)
    assert nloc1 == len(local)
    # the 2rc centres are the slab plus its r_c ghosts; its ghosts the next r_c shell
    assert nloc2 == nloc1 + ng1
    assert ng2 > 0 and nloc2 + ng2 <= n
    # locals first: the first nloc1 rows of both domains are the slab's atoms
    assert np.array_equal(np.sort(c1[:nloc1, 0]), np.sort(frame.coords[local, 0]))
    assert set(map(tuple, c1[:nloc1])) <= set(map(tuple, c2[:nloc2]))
    # ghost counts depend on the cutoff, not on the slab width (the beta of Eq. (8))
    assert ng1 > 2000


def test_full_frame_is_one_slab(frame):
    c, t, nloc, ng = slab_sweep.domain(frame, 1, "rc")
    assert nloc == len(frame.coords) and ng == 0


def test_fit_recovers_the_model():
    n_p = np.array([2, 4, 8, 16, 32], dtype=float)
    t = 7.0 / n_p + 1.5
    a, b = slab_sweep.fit(n_p, t)
    assert abs(a - 7.0) < 1e-9 and abs(b - 1.5) < 1e-9


@pytest.mark.gpu
@pytest.mark.parametrize("n_p", [4, 16])
def test_2rc_halo_forces_need_no_reduction(weights_path, frame, n_p):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_07276_amd import binding
    print(f"case: 2 r_c halo, slab 0 of {n_p}", flush=True)
    m = binding.Model(weights_path, slab_sweep.RCUT, slab_sweep.SEL)
    try:
        n = len(frame.coords)
        _, Ffull, _, _ = m.compute(frame.coords, frame.types, frame.box, n, 0)
        L = float(frame.box[0, 0])
        local, g1 = synth.slab_partition(frame.coords, L, n_p, 0, slab_sweep.RCUT)
        _, g2 = synth.slab_partition(frame.coords, L, n_p, 0, 2 * slab_sweep.RCUT)
        centres = np.sort(np.concatenate([local, g1]))
        ghosts = np.setdiff1d(g2, g1)
        idx = np.concatenate([centres, ghosts])
        _, F, _, _ = m.compute(frame.coords[idx], frame.types[idx], frame.box, len(centres),
                               len(ghosts))
        pos = np.searchsorted(centres, local)
        d = np.abs(F[pos] - Ffull[local]).max()
        print(f"[2rc {n_p}] max|F_slab - F_full| = {d:.2e}", flush=True)
        assert d <= 1e-4
    finally:
        m.close()
