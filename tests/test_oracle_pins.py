"""Pins of the CPU oracle against facts that do not come from the oracle itself.

The paper prints no model outputs, so the oracle is pinned by: a library
neighbour search, the closed form of the switch, the symmetries the paper
requires of the descriptor (Sec. II-B: translation, rotation, permutation),
strict locality (Sec. II-B, DPA-1 paragraph), forces as the energy gradient
(Eq. (2)) by finite differences, the virial identity, additivity of the energy
(Eq. (5)), smooth decay at the cutoff, exact periodic replication, the
local/ghost decomposition of Eq. (7), and an independent scalar-loop evaluation
on tiny inputs.
"""

import math

import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree

from oracle import dpa1_oracle as orc
from paper_2604_07276_amd import synth

RC = 6.0
SEL = 120


@pytest.fixture(scope="module")
def parity():
    return synth.parity_system(0)


@pytest.fixture(scope="module")
def parity_result(oracle_model, parity):
    return orc.compute(oracle_model, parity.coords, parity.types, parity.box, 192, 0, RC, SEL)


def _random_rotation(seed):
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    return q * np.sign(np.diag(r))


# --------------------------------------------------------------------------- neighbours

def test_nlist_matches_kdtree_periodic(parity):
    L = parity.box[0, 0]
    tree = cKDTree(parity.coords, boxsize=L)
    nl = orc.neighbor_list(parity.coords, parity.box, RC, np.arange(192))
    for i in range(192):
        ref = set(tree.query_ball_point(parity.coords[i], RC)) - {i}
        assert set(nl[i].tolist()) == ref
        assert np.all(np.diff(nl[i]) > 0)


def test_nlist_matches_kdtree_protein_sample():
    s = synth.protein_system(0)
    L = s.box[0, 0]
    tree = cKDTree(s.coords, boxsize=L)
    rng = np.random.default_rng(3)
    cs = rng.choice(len(s.coords), 200, replace=False)
    nl = orc.neighbor_list(s.coords, s.box, RC, cs)
    counts = []
    for c, lst in zip(cs, nl):
        ref = set(tree.query_ball_point(s.coords[c], RC)) - {int(c)}
        assert set(lst.tolist()) == ref
        counts.append(len(lst))
    assert 60 < np.mean(counts) < 100 and max(counts) <= SEL


def test_nlist_matches_kdtree_open():
    s = synth.open_cluster(120, 8.0, 5, seed=2)
    tree = cKDTree(s.coords)
    nl = orc.neighbor_list(s.coords, None, RC, np.arange(120))
    for i in range(120):
        assert set(nl[i].tolist()) == set(tree.query_ball_point(s.coords[i], RC)) - {i}


# --------------------------------------------------------------------------- switch

def test_switch_closed_form():
    rs, rc = 0.5, RC
    r = torch.tensor([0.1, rs, rc, rc + 1.0], dtype=torch.float64)
    sw = orc.switch(r, rs, rc)
    assert sw.tolist() == [1.0, 1.0, 0.0, 0.0]
    # first and second derivative vanish at both ends (C2 junctions)
    for r0 in (rs, rc):
        for side in (-1e-7, 1e-7):
            x = torch.tensor([r0 + side], dtype=torch.float64, requires_grad=True)
            y = orc.switch(x, rs, rc)
            (g,) = torch.autograd.grad(y.sum(), x, create_graph=True)
            (h,) = torch.autograd.grad(g.sum(), x)
            assert abs(float(g.detach())) < 1e-10
            assert abs(float(h)) < 1e-5
    # monotone non-increasing on [rs, rc]
    grid = torch.linspace(rs, rc, 2001, dtype=torch.float64)
    vals = orc.switch(grid, rs, rc)
    assert torch.all(vals[1:] <= vals[:-1] + 1e-15)
    # midpoint value of the quintic smoothstep is 1/2
    assert abs(float(orc.switch(torch.tensor([0.5 * (rs + rc)], dtype=torch.float64), rs, rc)) - 0.5) < 1e-15


# --------------------------------------------------------------------------- symmetries

def test_translation_invariance_across_wrap(oracle_model, parity, parity_result):
    L = parity.box[0, 0]
    shift = np.array([5.3, -7.1, 11.9])
    x2 = np.mod(parity.coords + shift, L)
    r2 = orc.compute(oracle_model, x2, parity.types, parity.box, 192, 0, RC, SEL)
    assert abs(r2.energy - parity_result.energy) <= 1e-12 * abs(parity_result.energy)
    np.testing.assert_allclose(r2.forces, parity_result.forces, atol=1e-12)


def test_cube_symmetries_periodic(oracle_model, parity, parity_result):
    L = parity.box[0, 0]
    # axis permutation and a reflection are symmetries of the periodic cube
    x2 = parity.coords[:, [2, 0, 1]].copy()
    x2[:, 1] = L - x2[:, 1]
    r2 = orc.compute(oracle_model, x2, parity.types, parity.box, 192, 0, RC, SEL)
    assert abs(r2.energy - parity_result.energy) <= 1e-12 * abs(parity_result.energy)
    F_exp = parity_result.forces[:, [2, 0, 1]].copy()
    F_exp[:, 1] *= -1
    np.testing.assert_allclose(r2.forces, F_exp, atol=1e-12)


def test_rotation_invariance_open(oracle_model):
    s = synth.open_cluster(60, 6.0, 5, seed=4)
    n = len(s.coords)
    r1 = orc.compute(oracle_model, s.coords, s.types, None, n, 0, RC, SEL)
    for seed, refl in ((1, False), (2, True)):
        R = _random_rotation(seed)
        if refl:
            R = R @ np.diag([1.0, 1.0, -1.0])
        x2 = s.coords @ R.T + np.array([3.0, -1.0, 2.0])
        r2 = orc.compute(oracle_model, x2, s.types, None, n, 0, RC, SEL)
        assert abs(r2.energy - r1.energy) <= 1e-11 * max(1.0, abs(r1.energy))
        np.testing.assert_allclose(r2.forces, r1.forces @ R.T, atol=1e-11)


def test_permutation_invariance(oracle_model, parity, parity_result):
    perm = np.random.default_rng(7).permutation(192)
    r2 = orc.compute(oracle_model, parity.coords[perm], parity.types[perm], parity.box, 192, 0,
                     RC, SEL)
    assert abs(r2.energy - parity_result.energy) <= 1e-12 * abs(parity_result.energy)
    np.testing.assert_allclose(r2.forces, parity_result.forces[perm], atol=1e-12)
    np.testing.assert_allclose(r2.atom_energy, parity_result.atom_energy[perm], atol=1e-13)


def test_net_force_zero(parity_result):
    assert np.all(np.abs(parity_result.forces.sum(0)) < 1e-10)
    # the random-init model produces forces well above rounding level
    assert np.sqrt((parity_result.forces ** 2).mean()) > 1e-3


# --------------------------------------------------------------------------- gradients

def test_forces_match_finite_differences(oracle_model, parity, parity_result):
    """Central differences at h = 1e-4 and h/2, Richardson-combined.

    The random-init model is strongly curved (its layer norms act on
    activations whose spread is close to the norm's epsilon), so the O(h^2)
    term of a plain central difference at h = 1e-4 is ~1e-6; the combination
    (4 D(h/2) - D(h)) / 3 cancels it, leaving O(h^4) and rounding (~1e-10).
    """
    rng = np.random.default_rng(11)
    atoms = rng.choice(192, 4, replace=False)

    def central(a, c, h):
        xp = parity.coords.copy()
        xm = parity.coords.copy()
        xp[a, c] += h
        xm[a, c] -= h
        ep = orc.energy_only(oracle_model, xp, parity.types, parity.box, 192, RC, SEL)
        em = orc.energy_only(oracle_model, xm, parity.types, parity.box, 192, RC, SEL)
        return -(ep - em) / (2 * h)

    h = 1e-4
    for a in atoms:
        for c in range(3):
            fd = (4 * central(a, c, h / 2) - central(a, c, h)) / 3
            assert abs(fd - parity_result.forces[a, c]) < 2e-9, (a, c, fd,
                                                                 parity_result.forces[a, c])


def test_virial_equals_sum_x_outer_f_open(oracle_model):
    s = synth.open_cluster(50, 5.5, 5, seed=5)
    n = len(s.coords)
    r = orc.compute(oracle_model, s.coords, s.types, None, n, 0, RC, SEL)
    ref = (s.coords[:, :, None] * r.forces[:, None, :]).sum(0)
    np.testing.assert_allclose(r.virial, ref, atol=1e-11)


def test_virial_diagonal_is_strain_derivative(oracle_model, parity, parity_result):
    h = 1e-5
    for a in range(3):
        out = []
        for sgn in (1, -1):
            e = np.eye(3)
            e[a, a] += sgn * h
            x = parity.coords @ e.T
            box = parity.box @ e.T
            out.append(orc.energy_only(oracle_model, x, parity.types, box, 192, RC, SEL))
        dE = (out[0] - out[1]) / (2 * h)
        assert abs(-dE - parity_result.virial[a, a]) < 1e-7
    np.testing.assert_allclose(parity_result.virial, parity_result.virial.T, atol=1e-12)


# --------------------------------------------------------------------------- locality and smoothness

def test_strict_locality(oracle_model):
    s = synth.open_cluster(80, 9.0, 5, seed=6)
    n = len(s.coords)
    x = s.coords.copy()
    r1 = orc.evaluate_centers(oracle_model, x, s.types, None, RC, SEL, np.arange(n))
    far = int(np.argmax(np.linalg.norm(x - x[0], axis=1)))
    assert np.linalg.norm(x[far] - x[0]) > RC + 1.0
    x[far] += np.array([0.3, -0.2, 0.25])
    assert np.linalg.norm(x[far] - x[0]) > RC
    r2 = orc.evaluate_centers(oracle_model, x, s.types, None, RC, SEL, np.arange(n))
    assert r1.atom_energy[0] == r2.atom_energy[0]


def test_smooth_decay_at_cutoff(oracle_model):
    """A neighbour crossing rc changes E by O(delta^3) and its force goes to zero.

    Atom 2 approaches atom 0 along -x while atom 1 sits at +x, so the only pair
    that crosses the cutoff is (0, 2); atom 0 keeps a second neighbour, which
    exercises the attention normalisation while a key leaves the list.
    """
    types = np.array([3, 0, 1], dtype=np.int32)

    def sys_at(r):
        return np.array([[0.0, 0.0, 0.0], [1.1, 0.2, -0.1], [-r, 0.0, 0.0]])

    e_out = orc.energy_only(oracle_model, sys_at(RC + 1e-3), types, None, 3, RC, SEL)
    e_far = orc.energy_only(oracle_model, sys_at(RC + 2.0), types, None, 3, RC, SEL)
    assert e_out == e_far
    prev = None
    for delta in (2e-2, 1e-2, 5e-3):
        e_in = orc.energy_only(oracle_model, sys_at(RC - delta), types, None, 3, RC, SEL)
        diff = abs(e_in - e_out)
        assert diff > 0.0
        if prev is not None:
            # cubic decay: halving delta divides the jump by ~8
            assert 6.0 < prev / diff < 10.0, (prev, diff)
        prev = diff
    r = orc.compute(oracle_model, sys_at(RC - 1e-4), types, None, 3, 0, RC, SEL)
    assert np.abs(r.forces[2]).max() < 1e-9


# --------------------------------------------------------------------------- additivity

def test_energy_bias_additivity(weights_path, parity, parity_result):
    m = orc.load_model(weights_path)
    delta = 0.37
    m.t["energy_bias"] = m.t["energy_bias"].clone()
    m.t["energy_bias"][3] += delta  # oxygen
    r2 = orc.compute(m, parity.coords, parity.types, parity.box, 192, 0, RC, SEL)
    n_o = int((parity.types == 3).sum())
    assert abs((r2.energy - parity_result.energy) - delta * n_o) < 1e-11
    np.testing.assert_allclose(r2.forces, parity_result.forces, atol=1e-14)


def test_layer_norm_shift_and_scale_invariance(weights_path, parity, parity_result):
    """Layer norm removes a common shift of the features exactly, and (with
    epsilon set to zero) any positive rescaling of the pre-norm activations."""
    m = orc.load_model(weights_path)
    m.t["attn0.bo"] = m.t["attn0.bo"] + 2.5          # constant shift of every feature
    r2 = orc.compute(m, parity.coords, parity.types, parity.box, 192, 0, RC, SEL)
    assert abs(r2.energy - parity_result.energy) < 1e-11 * abs(parity_result.energy)
    m0 = orc.load_model(weights_path)
    m0.ln_eps = 0.0
    e0 = orc.energy_only(m0, parity.coords, parity.types, parity.box, 192, RC, SEL)
    m0.t["attn1.Wo"] = m0.t["attn1.Wo"] * 1000.0       # rescale of the pre-norm activations
    m0.t["attn1.bo"] = m0.t["attn1.bo"] * 1000.0
    e1 = orc.energy_only(m0, parity.coords, parity.types, parity.box, 192, RC, SEL)
    assert abs(e1 - e0) < 1e-11 * abs(e0)
    assert abs(e0 - parity_result.energy) > 1e-6  # epsilon matters for this model


# --------------------------------------------------------------------------- periodic replication

def test_replication_2x1x1(oracle_model, parity, parity_result):
    big = synth.replicate(parity, (2, 1, 1))
    r2 = orc.compute(oracle_model, big.coords, big.types, big.box, 384, 0, RC, SEL)
    assert abs(r2.energy - 2 * parity_result.energy) < 1e-11 * abs(r2.energy)
    np.testing.assert_allclose(r2.forces[:192], parity_result.forces, atol=1e-12)
    np.testing.assert_allclose(r2.forces[192:], parity_result.forces, atol=1e-12)


# --------------------------------------------------------------------------- Eq. (7) decomposition

def test_local_ghost_decomposition(oracle_model, parity, parity_result):
    L = parity.box[0, 0]
    n_slabs = 4
    E = 0.0
    F = np.zeros_like(parity.coords)
    V = np.zeros((3, 3))
    for s in range(n_slabs):
        loc, gh = synth.slab_partition(parity.coords, L, n_slabs, s, RC)
        idx = np.concatenate([loc, gh])
        r = orc.compute(oracle_model, parity.coords[idx], parity.types[idx], parity.box,
                        len(loc), len(gh), RC, SEL)
        E += r.energy
        np.add.at(F, idx, r.forces)
        V += r.virial
    assert abs(E - parity_result.energy) < 1e-11 * abs(E)
    np.testing.assert_allclose(F, parity_result.forces, atol=1e-12)
    np.testing.assert_allclose(V, parity_result.virial, atol=1e-11)


# --------------------------------------------------------------------------- scalar-loop evaluation

def _loop_energy(m, coords, types, i, nbrs, rc, sel):
    """e_i by explicit scalar loops, written from the model definition.

    Independent of the oracle's batched tensor code: no padding, no masks,
    no broadcasting; every sum is an explicit loop.
    """
    W = {k: v.numpy() for k, v in m.t.items()}
    rs = m.rcut_smth

    def sw_of(r):
        if r < rs:
            return 1.0
        if r >= rc:
            return 0.0
        u = (r - rs) / (rc - rs)
        return u ** 3 * (-6 * u ** 2 + 15 * u - 10) + 1

    def dense(x, Wm, b, act):
        fin, fout = Wm.shape
        y = []
        for o in range(fout):
            acc = b[o]
            for k in range(fin):
                acc += x[k] * Wm[k, o]
            y.append(math.tanh(acc) if act else acc)
        if act and fout == fin:
            y = [y[o] + x[o] for o in range(fout)]
        elif act and fout == 2 * fin:
            y = [y[o] + x[o % fin] for o in range(fout)]
        return y

    n = len(nbrs)
    geo = []
    for j in nbrs:
        d = [coords[j][c] - coords[i][c] for c in range(3)]
        r = math.sqrt(sum(v * v for v in d))
        w = sw_of(r)
        geo.append((d, r, w, w / r))
    temb = W["type_embedding"]
    G = []
    for a, j in enumerate(nbrs):
        x = [geo[a][3]] + list(temb[types[j]]) + list(temb[types[i]])
        for l in range(len(m.emb)):
            x = dense(x, W[f"emb{l}.W"], W[f"emb{l}.b"], True)
        G.append(x)
    S = m.attn_shift
    for layer in range(m.n_attn):
        Q = [dense(g, W[f"attn{layer}.Wq"], W[f"attn{layer}.bq"], False) for g in G]
        K = [dense(g, W[f"attn{layer}.Wk"], W[f"attn{layer}.bk"], False) for g in G]
        V = [dense(g, W[f"attn{layer}.Wv"], W[f"attn{layer}.bv"], False) for g in G]
        newG = []
        for a in range(n):
            logits = []
            for b in range(n):
                lam = sum(Q[a][c] * K[b][c] for c in range(m.attn_dim)) / math.sqrt(m.attn_dim)
                logits.append((lam + S) * geo[a][2] * geo[b][2] - S)
            z = sum(math.exp(v) for v in logits) + (sel - n) * math.exp(-S)
            o = [0.0] * m.attn_dim
            for b in range(n):
                cosab = sum(geo[a][0][c] * geo[b][0][c] for c in range(3)) / (geo[a][1] * geo[b][1])
                wgt = math.exp(logits[b]) / z * geo[a][2] * geo[b][2] * cosab
                for c in range(m.attn_dim):
                    o[c] += wgt * V[b][c]
            y = dense(o, W[f"attn{layer}.Wo"], W[f"attn{layer}.bo"], False)
            mu = sum(y) / len(y)
            var = sum((v - mu) ** 2 for v in y) / len(y)
            ln = [(v - mu) / math.sqrt(var + m.ln_eps) * W[f"attn{layer}.ln_gamma"][c]
                  + W[f"attn{layer}.ln_beta"][c] for c, v in enumerate(y)]
            newG.append([G[a][c] + ln[c] for c in range(len(ln))])
        G = newG
    M = len(G[0]) if n else m.emb[-1]
    T = [[0.0] * M for _ in range(4)]
    for a in range(n):
        d, r, w, s = geo[a]
        Rrow = [s, s * d[0] / r, s * d[1] / r, s * d[2] / r]
        for c in range(4):
            for f in range(M):
                T[c][f] += Rrow[c] * G[a][f] / sel
    z = []
    for f in range(M):
        for ax in range(m.axis):
            z.append(sum(T[c][f] * T[c][ax] for c in range(4)))
    z += list(temb[types[i]])
    for l in range(len(m.fit)):
        z = dense(z, W[f"fit{l}.W"], W[f"fit{l}.b"], True)
    return sum(z[k] * W["w_out"][k] for k in range(len(z))) + W["b_out"][0] + W["energy_bias"][types[i]]


def test_scalar_loop_evaluation_tiny(oracle_model):
    # centres with 0, 1, 2 and 3 neighbours, one pair inside rs (sw = 1)
    coords = np.array([[0.0, 0.0, 0.0], [0.3, 0.2, -0.1], [2.0, -1.5, 0.7], [-3.0, 2.2, 1.9],
                       [30.0, 0.0, 0.0], [40.0, 0.0, 0.0], [41.5, 1.0, 0.0]])
    types = np.array([3, 0, 1, 2, 4, 0, 3], dtype=np.int32)
    n = len(coords)
    res = orc.evaluate_centers(oracle_model, coords, types, None, RC, SEL, np.arange(n))
    for i in range(n):
        e_loop = _loop_energy(oracle_model, coords, types, i, list(res.nlist[i]), RC, SEL)
        assert abs(e_loop - res.atom_energy[i]) < 1e-12, (i, e_loop, res.atom_energy[i])
    assert [len(x) for x in res.nlist] == [3, 3, 2, 2, 0, 1, 1]
