"""CPU oracle for DPA-1 inference on one domain (local + ghost atoms).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The GPU library never
calls it and shares no code with it: the two read the same weights file format
and the same seeded inputs, nothing else.

Everything is FP64 and written for a reader checking it against the paper:

* the energy is a sum of per-atom energies e_i produced by a fitting network
  from a per-centre descriptor (Sec. II-B, descriptor + fitting-net
  architecture, and Eq. (5));
* the descriptor is the DP-SE contraction G^T R R^T G_< (Sec. II-B), where the
  embedding matrix G carries the type embedding and is refined by gated
  self-attention restricted to the centre's own neighbour set (Sec. II-B,
  DPA-1 paragraph);
* neighbour lists are full lists within the cutoff (Sec. II-A cutoff lists,
  Sec. II-C full lists);
* forces are the negative gradient of the energy (Eq. (2)); only local atoms
  carry energy, ghost atoms receive forces (Eq. (7)).  The gradient is taken
  by torch's reverse-mode autograd on CPU float64 tensors, i.e. the definition
  itself, not a hand-written adjoint;
* the virial is Xi_ab = -sum_ij d_ij,a dE/dd_ij,b.

Where the paper gives no formula, the reading below is used (it fixes one
specification for both implementations; see the design notes):

* pair vector d_ij = x_j - x_i, minimum image d -= L rint(d/L) with a box;
  r_ij^2 = (dx dx + dy dy) + dz dz in FP64, neighbour iff r^2 < rc^2;
* switch sw(r) = 1 (r < rs), u^3(-6u^2 + 15u - 10) + 1 (rs <= r < rc),
  0 (r >= rc) with u = (r - rs)/(rc - rs); s = sw/r;
  R~_ij = (s, s dx/r, s dy/r, s dz/r); unit vector rhat = d/r;
* embedding input [s, t(type_j), t(type_i)], tanh layers with residual
  (identity when widths match, [x, x] when the width doubles);
* attention (single head, width d, shift S): logits (q.k/sqrt(d) + S) w_j w_k - S,
  softmax over the neighbours with (sel - n_i) e^{-S} added to the
  denominator, gate w_j w_k (rhat_j . rhat_k), residual G + LN(W_O o + b_O);
* descriptor T = R~^T G / sel, D = T^T T[:, :axis], flattened m*axis + a;
* fitting input [vec D, t(type_i)], tanh layers with the residual rule,
  e_i = w_out . z + b_out + bias[type_i].
"""

from __future__ import annotations

import dataclasses
import struct

import numpy as np
import torch

_MAGIC = b"DPA1WTS\0"


# ----------------------------------------------------------------------------
# weights file
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class OracleModel:
    ntypes: int
    tebd_dim: int
    axis: int
    n_attn: int
    attn_dim: int
    emb: tuple
    fit: tuple
    rcut_smth: float
    attn_shift: float
    ln_eps: float
    t: dict  # name -> torch.float64 tensor


def load_model(path: str) -> OracleModel:
    """Parse a weights file (format fixed by the seeded-input generator)."""
    with open(path, "rb") as f:
        buf = f.read()
    if buf[:8] != _MAGIC:
        raise ValueError("not a DPA-1 weights file")
    off = 8
    version, n_int = struct.unpack_from("<II", buf, off)
    off += 8
    if version != 1:
        raise ValueError(f"unsupported weights version {version}")
    ints = struct.unpack_from(f"<{n_int}i", buf, off)
    off += 4 * n_int
    (n_dbl,) = struct.unpack_from("<I", buf, off)
    off += 4
    dbls = struct.unpack_from(f"<{n_dbl}d", buf, off)
    off += 8 * n_dbl
    ntypes, tebd, axis, n_attn, attn_dim, n_emb, n_fit = ints[:7]
    emb = tuple(ints[7:7 + n_emb])
    fit = tuple(ints[7 + n_emb:7 + n_emb + n_fit])
    rcut_smth, attn_shift, ln_eps = dbls[:3]

    names = [("type_embedding", (ntypes, tebd))]
    fin = 1 + 2 * tebd
    for l, w in enumerate(emb):
        names += [(f"emb{l}.W", (fin, w)), (f"emb{l}.b", (w,))]
        fin = w
    m = emb[-1]
    for a in range(n_attn):
        for nm in ("q", "k", "v"):
            names += [(f"attn{a}.W{nm}", (m, attn_dim)), (f"attn{a}.b{nm}", (attn_dim,))]
        names += [(f"attn{a}.Wo", (attn_dim, m)), (f"attn{a}.bo", (m,)),
                  (f"attn{a}.ln_gamma", (m,)), (f"attn{a}.ln_beta", (m,))]
    fin = m * axis + tebd
    for l, w in enumerate(fit):
        names += [(f"fit{l}.W", (fin, w)), (f"fit{l}.b", (w,))]
        fin = w
    names += [("w_out", (fin,)), ("b_out", (1,)), ("energy_bias", (ntypes,))]

    t = {}
    for nm, shp in names:
        cnt = int(np.prod(shp))
        arr = np.frombuffer(buf, dtype="<f8", count=cnt, offset=off).reshape(shp)
        off += 8 * cnt
        t[nm] = torch.from_numpy(arr.copy())
    if off != len(buf):
        raise ValueError("weights file has trailing bytes")
    return OracleModel(ntypes, tebd, axis, n_attn, attn_dim, emb, fit,
                       rcut_smth, attn_shift, ln_eps, t)


# ----------------------------------------------------------------------------
# geometry: pair vectors and full neighbour lists (Sec. II-A, Sec. II-C)
# ----------------------------------------------------------------------------

def _box_lengths(box):
    if box is None:
        return None
    box = np.asarray(box, dtype=np.float64).reshape(3, 3)
    if np.any(box - np.diag(np.diag(box)) != 0.0):
        raise ValueError("only orthorhombic boxes are supported")
    return np.diag(box).copy()


def pair_vectors(coords: np.ndarray, i: np.ndarray, j: np.ndarray, box) -> np.ndarray:
    """d_ij = x_j - x_i, minimum image when a box is given (FP64, fixed order)."""
    d = coords[j] - coords[i]
    L = _box_lengths(box)
    if L is not None:
        d = d - L * np.rint(d / L)
    return d


def neighbor_list(coords: np.ndarray, box, rcut: float, centers: np.ndarray,
                  chunk: int = 256) -> list:
    """Full neighbour list by brute force over every atom.

    For each centre i: all j != i with r_ij^2 < rcut^2, sorted by index.
    """
    coords = np.asarray(coords, dtype=np.float64)
    n = coords.shape[0]
    L = _box_lengths(box)
    rc2 = rcut * rcut
    out = []
    allj = np.arange(n)
    for c0 in range(0, len(centers), chunk):
        cs = np.asarray(centers[c0:c0 + chunk])
        d = coords[None, :, :] - coords[cs, None, :]
        if L is not None:
            d = d - L * np.rint(d / L)
        r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        hit = r2 < rc2
        hit[np.arange(len(cs)), cs] = False
        for row in range(len(cs)):
            out.append(allj[hit[row]])
    return out


# ----------------------------------------------------------------------------
# model pieces (torch float64)
# ----------------------------------------------------------------------------

def switch(r: torch.Tensor, rs: float, rc: float) -> torch.Tensor:
    """Smooth cutoff: 1 below rs, quintic C2 decay on [rs, rc), 0 beyond."""
    u = (r - rs) / (rc - rs)
    poly = u * u * u * (-6.0 * u * u + 15.0 * u - 10.0) + 1.0
    one = torch.ones_like(r)
    zero = torch.zeros_like(r)
    return torch.where(r < rs, one, torch.where(r < rc, poly, zero))


def _mlp_residual(x: torch.Tensor, W: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """tanh layer with the residual rule: +x if widths match, +[x, x] if doubled."""
    y = torch.tanh(x @ W + b)
    fin, fout = W.shape
    if fout == fin:
        y = y + x
    elif fout == 2 * fin:
        y = y + torch.cat([x, x], dim=-1)
    return y


def _layer_norm(y: torch.Tensor, gamma, beta, eps: float) -> torch.Tensor:
    mu = y.mean(dim=-1, keepdim=True)
    var = ((y - mu) ** 2).mean(dim=-1, keepdim=True)
    return (y - mu) / torch.sqrt(var + eps) * gamma + beta


def atomic_energies(model: OracleModel, d: torch.Tensor, mask: torch.Tensor,
                    nnei: torch.Tensor, tc: torch.Tensor, tn: torch.Tensor,
                    rcut: float, sel: int, return_parts: bool = False):
    """e_i for a batch of centres (Sec. II-B).

    d [B, n, 3] pair vectors (padded slots hold a vector longer than rcut),
    mask [B, n] real-neighbour flags, nnei [B] neighbour counts, tc [B] centre
    types, tn [B, n] neighbour types.
    """
    t = model.t
    B, n, _ = d.shape
    temb = t["type_embedding"]
    r = torch.sqrt((d * d).sum(-1))
    sw = switch(r, model.rcut_smth, rcut) * mask
    s = sw / r
    rhat = d / r[..., None]
    Rt = torch.cat([s[..., None], s[..., None] * rhat], dim=-1)  # [B, n, 4]

    # type-embedded embedding net (DPA-1: type embedding inside G)
    x = torch.cat([s[..., None], temb[tn], temb[tc][:, None, :].expand(B, n, -1)], dim=-1)
    for l in range(len(model.emb)):
        x = _mlp_residual(x, t[f"emb{l}.W"], t[f"emb{l}.b"])
    G = x  # [B, n, M]

    # gated self-attention within each centre's neighbour set
    S = model.attn_shift
    ww = sw[:, :, None] * sw[:, None, :]
    cos = rhat @ rhat.transpose(1, 2)
    keymask = mask[:, None, :].expand(B, n, n)
    pad = (sel - nnei).to(d.dtype)
    for a in range(model.n_attn):
        q = G @ t[f"attn{a}.Wq"] + t[f"attn{a}.bq"]
        k = G @ t[f"attn{a}.Wk"] + t[f"attn{a}.bk"]
        v = G @ t[f"attn{a}.Wv"] + t[f"attn{a}.bv"]
        lam = q @ k.transpose(1, 2) / np.sqrt(model.attn_dim)
        lam2 = (lam + S) * ww - S
        lam2 = torch.where(keymask, lam2, torch.full_like(lam2, -np.inf))
        mx = torch.clamp(lam2.amax(dim=-1), min=-S)
        ex = torch.exp(lam2 - mx[..., None])
        Z = ex.sum(-1) + pad[:, None] * torch.exp(-S - mx)
        p = ex / Z[..., None]
        att = p * ww * cos
        o = att @ v
        y = o @ t[f"attn{a}.Wo"] + t[f"attn{a}.bo"]
        G = G + _layer_norm(y, t[f"attn{a}.ln_gamma"], t[f"attn{a}.ln_beta"], model.ln_eps)

    # descriptor D = G^T R R^T G_< with the 1/sel normalisation on R^T G
    T = Rt.transpose(1, 2) @ G / sel  # [B, 4, M]
    D = T.transpose(1, 2) @ T[:, :, :model.axis]  # [B, M, axis]
    z = torch.cat([D.reshape(B, -1), temb[tc]], dim=-1)
    for l in range(len(model.fit)):
        z = _mlp_residual(z, t[f"fit{l}.W"], t[f"fit{l}.b"])
    e = z @ t["w_out"] + t["b_out"][0] + t["energy_bias"][tc]
    if return_parts:
        return e, dict(sw=sw, s=s, Rt=Rt, T=T, D=D, G=G)
    return e


# ----------------------------------------------------------------------------
# driver
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class PairResult:
    centers: np.ndarray      # [C] centre indices
    atom_energy: np.ndarray  # [C] e_i
    nlist: list              # per centre: sorted neighbour indices
    pair_i: np.ndarray       # [P] centre of each pair
    pair_j: np.ndarray       # [P] neighbour of each pair
    d: np.ndarray            # [P][3] pair vectors
    g: np.ndarray            # [P][3] de_i/dd_ij


def evaluate_centers(model: OracleModel, coords, types, box, rcut: float, sel: int,
                     centers, chunk: int = 64) -> PairResult:
    """Per-centre energies and pair gradients for the given local centres.

    Neighbours are searched among all atoms in ``coords`` (locals and ghosts).
    """
    coords = np.asarray(coords, dtype=np.float64)
    types = np.asarray(types)
    centers = np.asarray(centers, dtype=np.int64)
    nl = neighbor_list(coords, box, rcut, centers)
    for ci, lst in zip(centers, nl):
        if len(lst) > sel:
            raise ValueError(f"atom {ci} has {len(lst)} neighbours > sel={sel}")
    e_all = np.zeros(len(centers))
    pi, pj, pd, pg = [], [], [], []
    for c0 in range(0, len(centers), chunk):
        cs = centers[c0:c0 + chunk]
        lists = nl[c0:c0 + chunk]
        B = len(cs)
        nmax = max([len(x) for x in lists] + [1])
        jj = np.zeros((B, nmax), dtype=np.int64)
        msk = np.zeros((B, nmax), dtype=bool)
        for b, lst in enumerate(lists):
            jj[b, :len(lst)] = lst
            msk[b, :len(lst)] = True
        ii = np.repeat(cs[:, None], nmax, axis=1)
        dnp = pair_vectors(coords, ii.ravel(), jj.ravel(), box).reshape(B, nmax, 3)
        dnp[~msk] = np.array([2.0 * rcut, 0.0, 0.0])
        d = torch.tensor(dnp, dtype=torch.float64, requires_grad=True)
        mask = torch.tensor(msk)
        nnei = torch.tensor([len(x) for x in lists], dtype=torch.int64)
        tc = torch.tensor(types[cs], dtype=torch.int64)
        tn = torch.tensor(types[jj], dtype=torch.int64)
        e = atomic_energies(model, d, mask, nnei, tc, tn, rcut, sel)
        (g,) = torch.autograd.grad(e.sum(), d)
        e_all[c0:c0 + B] = e.detach().numpy()
        gnp = g.numpy()
        pi.append(ii[msk])
        pj.append(jj[msk])
        pd.append(dnp[msk])
        pg.append(gnp[msk])
    cat = (lambda xs, shape: np.concatenate(xs) if xs else np.zeros(shape))
    return PairResult(centers, e_all, nl, cat(pi, (0,)).astype(np.int64),
                      cat(pj, (0,)).astype(np.int64), cat(pd, (0, 3)), cat(pg, (0, 3)))


@dataclasses.dataclass
class OracleResult:
    energy: float
    forces: np.ndarray       # [N_all][3]
    virial: np.ndarray       # [3][3]
    atom_energy: np.ndarray  # [nloc]
    nlist: list              # per local centre, sorted


def compute(model: OracleModel, coords, types, box, nloc: int, nghost: int,
            rcut: float, sel: int, chunk: int = 64) -> OracleResult:
    """Energy of the local atoms, forces on every atom, virial (Eq. (2), Eq. (7)).

    Atoms [0, nloc) are local, [nloc, nloc + nghost) are ghosts.  Only local
    atoms are centres; every atom may be a neighbour.
    F_k = sum_j g_kj [k local] - sum_{i: k in N(i)} g_ik.
    """
    coords = np.asarray(coords, dtype=np.float64)
    assert coords.shape[0] == nloc + nghost
    pr = evaluate_centers(model, coords, types, box, rcut, sel, np.arange(nloc), chunk)
    F = np.zeros_like(coords)
    np.add.at(F, pr.pair_i, pr.g)
    np.add.at(F, pr.pair_j, -pr.g)
    vir = -(pr.d[:, :, None] * pr.g[:, None, :]).sum(0)
    return OracleResult(float(pr.atom_energy.sum()), F, vir, pr.atom_energy, pr.nlist)


def energy_only(model: OracleModel, coords, types, box, nloc: int, rcut: float,
                sel: int, chunk: int = 64) -> float:
    """Total energy of the local atoms without gradients (for finite differences)."""
    coords = np.asarray(coords, dtype=np.float64)
    types = np.asarray(types)
    centers = np.arange(nloc)
    nl = neighbor_list(coords, box, rcut, centers)
    total = 0.0
    with torch.no_grad():
        for c0 in range(0, nloc, chunk):
            cs = centers[c0:c0 + chunk]
            lists = nl[c0:c0 + chunk]
            B = len(cs)
            nmax = max([len(x) for x in lists] + [1])
            jj = np.zeros((B, nmax), dtype=np.int64)
            msk = np.zeros((B, nmax), dtype=bool)
            for b, lst in enumerate(lists):
                jj[b, :len(lst)] = lst
                msk[b, :len(lst)] = True
            ii = np.repeat(cs[:, None], nmax, axis=1)
            dnp = pair_vectors(coords, ii.ravel(), jj.ravel(), box).reshape(B, nmax, 3)
            dnp[~msk] = np.array([2.0 * rcut, 0.0, 0.0])
            e = atomic_energies(model, torch.tensor(dnp), torch.tensor(msk),
                                torch.tensor([len(x) for x in lists]),
                                torch.tensor(types[cs], dtype=torch.int64),
                                torch.tensor(types[jj], dtype=torch.int64), rcut, sel)
            total += float(e.sum())
    return total
