"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars (FP32 network, FP64 geometry and reductions):
  neighbour lists bit-exact after sorting (the library returns them sorted),
  |E_gpu - E_oracle| / N <= 1e-6 eV/atom,
  max |F_gpu - F_oracle| <= 1e-4 eV/A,
  max |Xi_gpu - Xi_oracle| / N <= 1e-6 eV.
"""

import sys

import numpy as np
import pytest

from oracle import dpa1_oracle as orc
from paper_2604_07276_amd import synth

pytestmark = pytest.mark.gpu

RC = 6.0
SEL = 120
E_TOL = 1e-6
F_TOL = 1e-4
V_TOL = 1e-6


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def model(weights_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_07276_amd import binding
    m = binding.Model(weights_path, RC, SEL)
    yield m
    m.close()


def _report(tag, n, E, F, V, r):
    dE = abs(E - r.energy) / max(n, 1)
    dF = np.abs(F - r.forces).max() if F.size else 0.0
    dV = np.abs(V - r.virial).max() / max(n, 1)
    frms = np.sqrt((r.forces ** 2).mean()) if F.size else 0.0
    say(f"[{tag}] N={n} dE/N={dE:.2e} max|dF|={dF:.2e} (|F|rms={frms:.3e}) dV/N={dV:.2e}")
    return dE, dF, dV


def _assert_parity(tag, n, E, F, V, r):
    dE, dF, dV = _report(tag, n, E, F, V, r)
    assert dE <= E_TOL
    assert dF <= F_TOL
    assert dV <= V_TOL


def test_parity_192_atoms(model, oracle_model):
    s = synth.parity_system(0)
    say("case: 192-atom periodic parity system, seed 0, dp_compute")
    E, F, V, ae = model.compute(s.coords, s.types, s.box, 192, 0, atom_energy=True)
    r = orc.compute(oracle_model, s.coords, s.types, s.box, 192, 0, RC, SEL)
    _assert_parity("192", 192, E, F, V, r)
    assert np.abs(ae - r.atom_energy).max() <= 1e-5
    # relative force accuracy is far better than the absolute bar
    assert np.abs(F - r.forces).max() <= 1e-3 * np.abs(r.forces).max()


def test_nlist_bit_exact_192(model, oracle_model):
    s = synth.parity_system(0)
    say("case: neighbour list, 192 atoms")
    model.compute(s.coords, s.types, s.box, 192, 0)
    nl, nn = model.debug_nlist(192)
    ref = orc.neighbor_list(s.coords, s.box, RC, np.arange(192))
    for i in range(192):
        assert nn[i] == len(ref[i])
        assert np.array_equal(nl[i, :nn[i]], ref[i])
        assert np.all(nl[i, nn[i]:] == -1)


def test_nlist_dense_neighbourhood_beyond_lds_tile(weights_path):
    """1,728 atoms on a jittered 12^3 lattice in a periodic box 3.9 rc wide:
    three cells per side, so the 27 cells around any cell hold every atom,
    more candidates than the neighbour kernel stages in LDS (its scan of
    global memory runs instead).  Every atom has 122 neighbours (the lattice
    shells at 0.975 and 1.028 rc stay on their side under the jitter); lists
    bit-exact against brute force."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_07276_amd import binding
    rng = np.random.default_rng(5)
    L = 3.9 * RC
    grid = (np.arange(12) + 0.5) * (L / 12)
    coords = np.stack(np.meshgrid(grid, grid, grid, indexing="ij"), -1).reshape(-1, 3)
    coords = coords + rng.uniform(-0.02, 0.02, coords.shape)
    n = len(coords)
    types = rng.integers(0, 2, n).astype(np.int32)
    box = np.diag([L, L, L])
    say(f"case: dense lattice N={n}, box {L:.1f} A, sel 128, neighbour list")
    m = binding.Model(weights_path, RC, 128)
    try:
        m.compute(coords, types, box, n, 0)
        nl, nn = m.debug_nlist(n)
    finally:
        m.close()
    ref = orc.neighbor_list(coords, box, RC, np.arange(n))
    assert all(len(r) == 122 for r in ref)
    for i in range(n):
        assert nn[i] == len(ref[i])
        assert np.array_equal(nl[i, :nn[i]], ref[i])
        assert np.all(nl[i, nn[i]:] == -1)


def test_parity_open_cluster_with_ghosts(model, oracle_model):
    # open boundaries: a cluster whose outer shell is passed as ghosts
    c = synth.open_cluster(150, 9.0, 5, seed=9)
    r2 = np.sum(c.coords ** 2, axis=1)
    order = np.argsort(r2, kind="stable")
    x = c.coords[order]
    t = c.types[order]
    nloc = 90
    say("case: open cluster 90 locals + 60 ghosts, box=None")
    E, F, V, _ = model.compute(x, t, None, nloc, 60)
    r = orc.compute(oracle_model, x, t, None, nloc, 60, RC, SEL)
    _assert_parity("open+ghosts", 150, E, F, V, r)


def test_parity_slab_with_ghosts(model, oracle_model):
    s = synth.parity_system(0)
    L = s.box[0, 0]
    loc, gh = synth.slab_partition(s.coords, L, 4, 1, RC)
    idx = np.concatenate([loc, gh])
    say(f"case: periodic slab 1/4, {len(loc)} locals + {len(gh)} ghosts")
    E, F, V, _ = model.compute(s.coords[idx], s.types[idx], s.box, len(loc), len(gh))
    r = orc.compute(oracle_model, s.coords[idx], s.types[idx], s.box, len(loc), len(gh), RC, SEL)
    _assert_parity("slab", len(idx), E, F, V, r)


def test_domain_decomposition_consistency(model):
    """Eq. (7): slab energies sum to the full energy, folded forces match."""
    s = synth.parity_system(1)
    L = s.box[0, 0]
    say("case: 4-slab decomposition of the 192-atom system (seed 1)")
    E0, F0, V0, _ = model.compute(s.coords, s.types, s.box, 192, 0)
    E, F, V = 0.0, np.zeros_like(F0), np.zeros((3, 3))
    for k in range(4):
        loc, gh = synth.slab_partition(s.coords, L, 4, k, RC)
        idx = np.concatenate([loc, gh])
        e, f, v, _ = model.compute(s.coords[idx], s.types[idx], s.box, len(loc), len(gh))
        E += e
        np.add.at(F, idx, f)
        V += v
    assert abs(E - E0) / 192 < 1e-6
    assert np.abs(F - F0).max() < 1e-5
    assert np.abs(V - V0).max() / 192 < 1e-6


def test_ragged_and_edge_cases(model, oracle_model):
    # isolated atoms, a pair, and a dense cluster with > 96 neighbours (128-slot tiles)
    rng = np.random.default_rng(5)
    dense = []
    while len(dense) < 112:
        p = rng.uniform(-3.3, 3.3, size=3)
        if np.dot(p, p) > 3.3 ** 2:
            continue
        if dense and np.min(np.sum((np.asarray(dense) - p) ** 2, axis=1)) < 0.8 ** 2:
            continue
        dense.append(p)
    dense = np.asarray(dense)
    lone = np.array([[40.0, 0, 0], [60.0, 0, 0], [61.2, 0.3, 0.0]])
    x = np.vstack([dense, lone])
    t = rng.integers(0, 5, size=len(x)).astype(np.int32)
    n = len(x)
    say(f"case: dense cluster ({len(dense)} atoms) + isolated atom + dimer, open")
    E, F, V, ae = model.compute(x, t, None, n, 0, atom_energy=True)
    r = orc.compute(oracle_model, x, t, None, n, 0, RC, SEL)
    assert max(len(v) for v in r.nlist) > 96
    _assert_parity("ragged", n, E, F, V, r)
    assert np.abs(ae - r.atom_energy).max() <= 1e-5


def test_no_local_atoms(model):
    s = synth.parity_system(0)
    say("case: nloc=0 with 192 ghosts")
    E, F, V, _ = model.compute(s.coords, s.types, s.box, 0, 192)
    assert E == 0.0 and np.all(F == 0.0) and np.all(V == 0.0)


def test_empty_system(model):
    say("case: empty system")
    E, F, V, _ = model.compute(np.zeros((0, 3)), np.zeros(0, np.int32), None, 0, 0)
    assert E == 0.0 and F.shape == (0, 3) and np.all(V == 0.0)


def test_errors(model, weights_path):
    from paper_2604_07276_amd.binding import DPError
    s = synth.parity_system(0)
    bad = s.types.copy()
    bad[5] = 7
    say("case: error paths (bad type, bad box, sel overflow)")
    with pytest.raises(DPError) as e:
        model.compute(s.coords, bad, s.box, 192, 0)
    assert e.value.code == -2
    with pytest.raises(DPError) as e:
        model.compute(s.coords, s.types, np.eye(3) * 10.0, 192, 0)
    assert e.value.code == -3
    from paper_2604_07276_amd import binding
    small = binding.Model(weights_path, RC, 40)
    try:
        with pytest.raises(DPError) as e:
            small.compute(s.coords, s.types, s.box, 192, 0)
        assert e.value.code == -4
    finally:
        small.close()
    # the handle still works after an error
    E, F, V, _ = model.compute(s.coords, s.types, s.box, 192, 0)
    assert np.isfinite(E)


def test_deterministic(model):
    s = synth.parity_system(2)
    say("case: determinism, two identical calls")
    a = model.compute(s.coords, s.types, s.box, 192, 0, atom_energy=True)
    b = model.compute(s.coords, s.types, s.box, 192, 0, atom_energy=True)
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


def test_device_entry_point_matches_host(model):
    import torch
    s = synth.parity_system(3)
    say("case: dp_compute_device vs dp_compute")
    E, F, V, ae = model.compute(s.coords, s.types, s.box, 192, 0, atom_energy=True)
    dev = torch.device("cuda:0")
    x = torch.tensor(s.coords, device=dev)
    t = torch.tensor(s.types, device=dev)
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    f = torch.zeros((192, 3), dtype=torch.float64, device=dev)
    v = torch.zeros(9, dtype=torch.float64, device=dev)
    a = torch.zeros(192, dtype=torch.float64, device=dev)
    model.compute_device(x, t, s.box, 192, 0, e, f, v, a)
    model.sync()
    assert float(e.cpu()[0]) == E
    assert np.array_equal(f.cpu().numpy(), F)
    assert np.array_equal(v.cpu().numpy().reshape(3, 3), V)
    assert np.array_equal(a.cpu().numpy(), ae)


def _oracle_forces_subset(m, coords, types, box, nloc, atoms):
    """Exact oracle forces on selected atoms: evaluate every centre that sees them."""
    nl = orc.neighbor_list(coords, box, RC, np.asarray(atoms))
    centers = set()
    for a, lst in zip(atoms, nl):
        if a < nloc:
            centers.add(int(a))
        centers.update(int(j) for j in lst if j < nloc)
    centers = np.array(sorted(centers))
    pr = orc.evaluate_centers(m, coords, types, box, RC, SEL, centers)
    out = np.zeros((len(atoms), 3))
    for q, a in enumerate(atoms):
        out[q] += pr.g[pr.pair_i == a].sum(0)
        out[q] -= pr.g[pr.pair_j == a].sum(0)
    return out, pr


def test_parity_protein_15668_sampled(model, oracle_model):
    s = synth.protein_system(0)
    n = len(s.coords)
    say(f"case: protein-shaped periodic system N={n}, sampled oracle")
    E, F, V, ae = model.compute(s.coords, s.types, s.box, n, 0, atom_energy=True)
    rng = np.random.default_rng(17)
    atoms = rng.choice(n, 12, replace=False)
    Fo, pr = _oracle_forces_subset(oracle_model, s.coords, s.types, s.box, n, atoms)
    dF = np.abs(F[atoms] - Fo).max()
    de = np.abs(ae[pr.centers] - pr.atom_energy).max()
    say(f"[protein] max|dF| (12 atoms) = {dF:.2e}, max|de_i| ({len(pr.centers)} centres) = {de:.2e}")
    assert dF <= F_TOL
    assert de <= 1e-5
    # whole-system properties that hold at any size
    assert np.abs(F.sum(0)).max() < 1e-6 * n
    nl, nn = model.debug_nlist(n)
    ref = orc.neighbor_list(s.coords, s.box, RC, atoms)
    for a, lst in zip(atoms, ref):
        assert np.array_equal(nl[a, :nn[a]], lst)


def test_replication_2x2x1(model):
    """A 2x2x1 tiling of the periodic 15,668-atom frame (62,672 atoms) gives 4x the
    energy and the same forces on every copy.  Neighbour order differs between the
    two systems (indices of images change), so FP32 sums agree to rounding only."""
    s = synth.protein_system(0)
    n = len(s.coords)
    big = synth.replicate(s, (2, 2, 1))
    say(f"case: 2x2x1 replication, N={len(big.coords)}")
    E1, F1, V1, _ = model.compute(s.coords, s.types, s.box, n, 0)
    E4, F4, V4, _ = model.compute(big.coords, big.types, big.box, 4 * n, 0)
    dE = abs(E4 - 4 * E1) / (4 * n)
    dF = max(np.abs(F4[k * n:(k + 1) * n] - F1).max() for k in range(4))
    dV = np.abs(V4 - 4 * V1).max() / (4 * n)
    say(f"[replication] dE/N={dE:.2e} max|dF|={dF:.2e} dV/N={dV:.2e}")
    assert dE < E_TOL and dF < F_TOL and dV < V_TOL


@pytest.mark.parametrize("tag,shape", [
    # embedding widths that take the unfused paths: per-layer embedding GEMMs
    # and the stand-alone output-projection + layer-norm GEMM (padded width 64)
    ("emb24-48-64_attn1", dict(emb=(24, 48, 64), n_attn=1, fit=(120, 120))),
    # the distilled student's shape: fused 16/32/64 embedding, no attention
    ("student_dpse", dict(emb=(16, 32, 64), axis=8, n_attn=0, fit=(128, 128))),
    # widths 25 -> 50 -> 50: identity residual in the last embedding layer
    ("emb25-50-50_attn2", dict(emb=(25, 50, 50), n_attn=2, fit=(64, 64, 64))),
    # widths 25 -> 50 -> 98: the fused embedding kernels with no residual in
    # the last layer, and 98 real features of 112 in the kernels that take
    # the last 16-wide chunk's real features in one step (QKV projection,
    # forward with the projection, descriptor adjoint with dO)
    ("emb25-50-98_attn2", dict(emb=(25, 50, 98), n_attn=2)),
    # no attention layer: the descriptor takes the embedding output directly
    ("attn0", dict(n_attn=0)),
])
def test_parity_other_architectures(tag, shape, tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_07276_amd import binding
    say(f"case: architecture {tag}, 192-atom system")
    p = str(tmp_path / f"{tag}.bin")
    synth.make_weights(p, seed=3, shape=synth.ModelShape(**shape))
    om = orc.load_model(p)
    m = binding.Model(p, RC, SEL)
    try:
        s = synth.parity_system(1)
        E, F, V, _ = m.compute(s.coords, s.types, s.box, 192, 0)
        r = orc.compute(om, s.coords, s.types, s.box, 192, 0, RC, SEL)
        _assert_parity(tag, 192, E, F, V, r)
    finally:
        m.close()
