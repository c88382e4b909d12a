"""GPU parity at the benchmark's full sizes, against the FP64 oracle.

* The 15,668-atom protein-shaped frame: frame 0 of the timed trajectory
  compared on every atom (energy, all forces, virial, every e_i, the whole
  neighbour list bit-exact); frames 50 and 99 compared on the whole
  neighbour list and on 64 sampled atoms' exact oracle forces plus the e_i of
  every centre the oracle evaluates for them.
* The memory-budget path (attention activations recomputed in the adjoint)
  at 15,668 atoms against the same oracle frame.
* One domain's share (Sec. II-C, Eq. (7)): the 1/16 and 1/32 slabs of the
  frame with an rcut halo of ghosts, through the torch.autograd.Function
  over the hand-written adjoint, a weighted loss sum_i w_i e_i; the gradient
  on 64 sampled locals and ghosts and every local e_i against the oracle.
* BF16 mode at 15,668 atoms (every atom) and FP32 + BF16 on the 62,672-atom
  2x2x1 replica: e_i of 1,000 random centres and the forces on the 1,000
  atoms of a compact sub-box from the oracle run on the replica itself, and
  every force against the tiled oracle frame (a periodic tiling reproduces
  the frame's forces on every copy, a property pinned on the oracle).

Bars: FP32 as in the small parity tests (|dE|/N <= 1e-6 eV, max |dF| <=
1e-4 eV/A, |dXi|/N <= 1e-6 eV, e_i <= 1e-5 eV, lists bit-exact); BF16 force
RMSE <= 5e-3 eV/A over every atom, |dE|/N <= 5e-4 eV, and a loose bound on
the largest force error that catches indexing mistakes.
"""

import sys
import time

import numpy as np
import pytest

import oracle_samples as osm
from oracle import dpa1_oracle as orc
from paper_2604_07276_amd import synth

pytestmark = pytest.mark.gpu

RC = 6.0
SEL = 120
E_TOL = 1e-6
F_TOL = 1e-4
V_TOL = 1e-6
EI_TOL = 1e-5
BF_F_RMSE = 5e-3
BF_E_TOL = 5e-4
BF_F_MAX = 1.0


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


@pytest.fixture(scope="module")
def protein():
    return synth.protein_system(0)


@pytest.fixture(scope="module")
def frames(protein):
    return synth.perturbed_frames(protein, 100, 0.01)


@pytest.fixture(scope="module")
def oracle_frame0(oracle_model, protein, frames):
    n = len(protein.coords)
    say(f"oracle: every centre of frame 0, N={n}")
    t0 = time.time()
    r = osm.full_frame(oracle_model, frames[0], protein.types, protein.box, n, say)
    say(f"oracle: frame 0 done in {time.time() - t0:.1f} s")
    return r


def _check_nlist(model, n, ref, tag):
    nl, nn = model.debug_nlist(n)
    bad = 0
    for i in range(n):
        k = len(ref[i])
        if nn[i] != k or not np.array_equal(nl[i, :k], ref[i]) or np.any(nl[i, k:] != -1):
            bad += 1
    say(f"[{tag}] neighbour lists: {n - bad}/{n} centres bit-exact")
    assert bad == 0


def test_protein_frame0_every_atom(model, oracle_model, protein, frames, oracle_frame0):
    n = len(protein.coords)
    say(f"case: protein frame 0, N={n}, FP32, every atom")
    E, F, V, ae = model.compute(frames[0], protein.types, protein.box, n, 0, atom_energy=True)
    Eo, Fo, Vo, aeo, nlo = oracle_frame0
    dE = abs(E - Eo) / n
    dF = np.abs(F - Fo).max()
    dV = np.abs(V - Vo).max() / n
    de = np.abs(ae - aeo).max()
    frms = np.sqrt((Fo ** 2).mean())
    rmse = np.sqrt(((F - Fo) ** 2).mean())
    say(f"[frame 0] dE/N={dE:.2e} max|dF|={dF:.2e} RMSE={rmse:.2e} (|F|rms={frms:.3e}) "
        f"dV/N={dV:.2e} max|de_i|={de:.2e}")
    assert dE <= E_TOL and dF <= F_TOL and dV <= V_TOL and de <= EI_TOL
    _check_nlist(model, n, nlo, "frame 0")


@pytest.mark.parametrize("frame", [50, 99])
def test_protein_later_frames(model, oracle_model, protein, frames, frame):
    n = len(protein.coords)
    x = frames[frame]
    say(f"case: protein frame {frame}, N={n}, FP32, 64 sampled atoms + whole neighbour list")
    E, F, V, ae = model.compute(x, protein.types, protein.box, n, 0, atom_energy=True)
    rng = np.random.default_rng(100 + frame)
    atoms = np.sort(rng.choice(n, 64, replace=False))
    t0 = time.time()
    Fo, pr = osm.forces_on(oracle_model, x, protein.types, protein.box, n, atoms)
    dF = np.abs(F[atoms] - Fo).max()
    de = np.abs(ae[pr.centers] - pr.atom_energy).max()
    say(f"[frame {frame}] max|dF| (64 atoms)={dF:.2e} max|de_i| ({len(pr.centers)} centres)="
        f"{de:.2e} (oracle {time.time() - t0:.1f} s)")
    assert dF <= F_TOL and de <= EI_TOL
    assert np.abs(F.sum(0)).max() < 1e-6 * n
    say(f"oracle: neighbour lists of frame {frame}")
    ref = []
    for c0 in range(0, n, 4000):
        ref.extend(orc.neighbor_list(x, protein.box, RC, np.arange(c0, min(n, c0 + 4000))))
        say(f"  lists {min(n, c0 + 4000)}/{n}")
    _check_nlist(model, n, ref, f"frame {frame}")


def test_memory_budget_path_15668(weights_path, protein, frames, oracle_frame0):
    from paper_2604_07276_amd import binding
    n = len(protein.coords)
    say(f"case: memory-budget recompute path, protein frame 0, N={n}")
    m = binding.Model(weights_path, RC, SEL)
    try:
        E1, F1, V1, _ = m.compute(frames[0], protein.types, protein.box, n, 0)
        full, rec = m.memory_info()
        assert not rec
        m.set_memory_budget(full - 1)
        E2, F2, V2, ae2 = m.compute(frames[0], protein.types, protein.box, n, 0, atom_energy=True)
        small, rec2 = m.memory_info()
        say(f"[budget] workspace {full / 2**30:.2f} GiB -> {small / 2**30:.2f} GiB, recompute={rec2}")
        assert rec2 and small < full
        assert E1 == E2 and np.array_equal(F1, F2) and np.array_equal(V1, V2)
    finally:
        m.close()
    Eo, Fo, Vo, aeo, _ = oracle_frame0
    dE = abs(E2 - Eo) / n
    dF = np.abs(F2 - Fo).max()
    dV = np.abs(V2 - Vo).max() / n
    say(f"[budget] vs oracle: dE/N={dE:.2e} max|dF|={dF:.2e} dV/N={dV:.2e}")
    assert dE <= E_TOL and dF <= F_TOL and dV <= V_TOL
    assert np.abs(ae2 - aeo).max() <= EI_TOL


@pytest.mark.parametrize("n_slabs", [16, 32])
def test_slab_share_autograd(model, oracle_model, protein, n_slabs):
    import torch
    from paper_2604_07276_amd.autograd import atomic_energies
    L = protein.box[0, 0]
    x_np, t_np, nloc, nghost = osm.slab_case(protein.coords, protein.types, L, n_slabs)
    say(f"case: 1/{n_slabs} slab of the protein frame, {nloc} locals + {nghost} ghosts, "
        "autograd adjoint, weighted loss")
    w_np = np.random.default_rng(n_slabs).normal(size=nloc)
    dev = torch.device("cuda:0")
    x = torch.tensor(x_np, device=dev).requires_grad_(True)
    e = atomic_energies(model, x, torch.tensor(t_np, device=dev), protein.box, nloc, nghost)
    loss = (e * torch.tensor(w_np, device=dev)).sum()
    (gx,) = torch.autograd.grad(loss, x)
    gx = gx.cpu().numpy()
    e_gpu = e.detach().cpu().numpy()
    atoms = osm.slab_sample(nloc, nghost, x_np, protein.box, seed=n_slabs)
    t0 = time.time()
    cs = np.union1d(osm.centres_seeing(x_np, protein.box, nloc, atoms), np.arange(nloc))
    pr = orc.evaluate_centers(oracle_model, x_np, t_np, protein.box, RC, SEL, cs)
    w_full = np.zeros(nloc)
    w_full[:] = w_np
    ref = osm.weighted_gradient(pr, atoms, w_full)
    dg = np.abs(gx[atoms] - ref).max()
    de = np.abs(e_gpu[pr.centers] - pr.atom_energy).max()
    dl = abs(float(loss.detach().cpu()) - float(np.dot(w_np, pr.atom_energy))) / nloc
    nz = np.abs(gx[nloc:]).max(axis=1) > 0
    say(f"[slab 1/{n_slabs}] max|d grad| (64 atoms: {np.sum(atoms < nloc)} locals, "
        f"{np.sum(atoms >= nloc)} ghosts)={dg:.2e} (|grad|max={np.abs(ref).max():.3e}) "
        f"max|de_i| ({nloc} locals)={de:.2e} d loss/N={dl:.2e} "
        f"ghosts with gradient {nz.sum()}/{nghost} (oracle {time.time() - t0:.1f} s)")
    assert dg <= F_TOL and de <= EI_TOL and dl <= E_TOL
    # the sampled ghosts carry gradient (Eq. (7): ghosts get forces)
    assert np.all(np.abs(gx[atoms[atoms >= nloc]]).max(axis=1) > 0)


def test_bf16_protein_every_atom(model, protein, frames, oracle_frame0):
    from paper_2604_07276_amd import binding
    n = len(protein.coords)
    say(f"case: BF16 mode, protein frame 0, N={n}, every atom against the oracle")
    model.set_precision(binding.PREC_BF16)
    try:
        E, F, V, ae = model.compute(frames[0], protein.types, protein.box, n, 0, atom_energy=True)
    finally:
        model.set_precision(binding.PREC_FP32)
    Eo, Fo, Vo, aeo, _ = oracle_frame0
    dFv = np.linalg.norm(F - Fo, axis=1)
    rmse = np.sqrt(((F - Fo) ** 2).mean())
    dE = abs(E - Eo) / n
    say(f"[bf16 15668] dE/N={dE:.2e} force RMSE={rmse:.2e} p99={np.percentile(dFv, 99):.2e} "
        f"max={dFv.max():.2e} (|F|rms={np.sqrt((Fo ** 2).mean()):.3e}) "
        f"max|de_i|={np.abs(ae - aeo).max():.2e} dV/N={np.abs(V - Vo).max() / n:.2e}")
    assert dE <= BF_E_TOL and rmse <= BF_F_RMSE and dFv.max() <= BF_F_MAX
    assert rmse > 1e-6  # BF16 rounding is in effect


def _compact_subbox(coords, L, k: int) -> np.ndarray:
    """The k atoms nearest (minimum image) to the centre of the box."""
    c = 0.5 * L
    d = coords - c
    d = d - L * np.rint(d / L)
    return np.sort(np.argsort((d * d).sum(1), kind="stable")[:k])


@pytest.fixture(scope="module")
def replica_oracle(oracle_model, protein, frames):
    big = synth.replicate(synth.System(frames[0], protein.types, protein.box, 0), (2, 2, 1))
    nb = len(big.coords)
    L = np.diag(big.box)
    rng = np.random.default_rng(31)
    centres = np.sort(rng.choice(nb, 1000, replace=False))
    say(f"oracle: replica N={nb}: e_i of 1,000 random centres")
    t0 = time.time()
    pr_e = orc.evaluate_centers(oracle_model, big.coords, big.types, big.box, RC, SEL, centres)
    sub = _compact_subbox(big.coords, L, 1000)
    say(f"oracle: forces on the 1,000 atoms of a compact sub-box ({time.time() - t0:.1f} s)")
    Fsub, pr_f = osm.forces_on(oracle_model, big.coords, big.types, big.box, nb, sub)
    say(f"oracle: replica sample done, {len(pr_f.centers)} centres for the sub-box "
        f"({time.time() - t0:.1f} s)")
    return big, pr_e, sub, Fsub


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_replica_62672(model, protein, oracle_frame0, replica_oracle, precision):
    from paper_2604_07276_amd import binding
    big, pr_e, sub, Fsub = replica_oracle
    nb = len(big.coords)
    n = len(protein.coords)
    say(f"case: 2x2x1 replica N={nb}, {precision}")
    if precision == "bf16":
        model.set_precision(binding.PREC_BF16)
    try:
        E, F, V, ae = model.compute(big.coords, big.types, big.box, nb, 0, atom_energy=True)
    finally:
        model.set_precision(binding.PREC_FP32)
    Eo, Fo, Vo, aeo, _ = oracle_frame0
    de_s = np.abs(ae[pr_e.centers] - pr_e.atom_energy)
    dF_s = F[sub] - Fsub
    Ft = np.tile(Fo, (4, 1))
    dE = abs(E - 4 * Eo) / nb
    dF_all = F - Ft
    rmse_s = np.sqrt((dF_s ** 2).mean())
    rmse_all = np.sqrt((dF_all ** 2).mean())
    say(f"[replica {precision}] oracle sample: max|de_i| (1,000)={de_s.max():.2e} "
        f"E/atom err (1,000)={de_s.mean():.2e} sub-box force RMSE={rmse_s:.2e} "
        f"max={np.abs(dF_s).max():.2e}; every atom vs tiled oracle: dE/N={dE:.2e} "
        f"RMSE={rmse_all:.2e} max={np.abs(dF_all).max():.2e} "
        f"dV/N={np.abs(V - 4 * Vo).max() / nb:.2e}")
    if precision == "fp32":
        assert de_s.max() <= EI_TOL and np.abs(dF_s).max() <= F_TOL
        assert dE <= E_TOL and np.abs(dF_all).max() <= F_TOL
        assert np.abs(V - 4 * Vo).max() / nb <= V_TOL
    else:
        # The BF16 force error is heavy-tailed: a handful of centres where two
        # opposite neighbours attend strongly to each other amplify operand
        # rounding ~1e4-fold (the 10 worst atoms of the frame carry ~3/4 of
        # its squared error), so the RMSE of a 1,000-atom sample depends on
        # whether it holds one of them.  The 5e-3 target is asserted on every
        # atom; the sample's RMSE is reported and bounded at twice the target.
        assert dE <= BF_E_TOL and rmse_all <= BF_F_RMSE
        assert np.linalg.norm(dF_all, axis=1).max() <= BF_F_MAX
        assert de_s.mean() <= BF_E_TOL and rmse_s <= 2 * BF_F_RMSE
        assert np.linalg.norm(dF_s, axis=1).max() <= BF_F_MAX


def test_replica_62672_memory_budget(weights_path, replica_oracle):
    """The 62,672-atom replica under a memory budget below its full workspace:
    attention activations shared across layers and recomputed in the adjoint,
    results bit-identical to the unbudgeted step and within the FP32 bars of
    the oracle sample."""
    from paper_2604_07276_amd import binding
    big, pr_e, sub, Fsub = replica_oracle
    nb = len(big.coords)
    say(f"case: 2x2x1 replica N={nb}, FP32, memory budget")
    m = binding.Model(weights_path, RC, SEL)
    try:
        E1, F1, V1, ae1 = m.compute(big.coords, big.types, big.box, nb, 0, atom_energy=True)
        full, rec = m.memory_info()
        m.set_memory_budget(full - 1)
        E2, F2, V2, ae2 = m.compute(big.coords, big.types, big.box, nb, 0, atom_energy=True)
        small, rec2 = m.memory_info()
    finally:
        m.close()
    say(f"[replica budget] workspace {full / 2**30:.2f} GiB (recompute={rec}) -> "
        f"{small / 2**30:.2f} GiB (recompute={rec2})")
    assert not rec and rec2 and small < full
    assert E1 == E2 and np.array_equal(F1, F2) and np.array_equal(V1, V2)
    assert np.array_equal(ae1, ae2)
    assert np.abs(ae2[pr_e.centers] - pr_e.atom_energy).max() <= EI_TOL
    assert np.abs(F2[sub] - Fsub).max() <= F_TOL
