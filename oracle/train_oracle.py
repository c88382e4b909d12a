"""CPU oracle for training a distilled student potential on teacher labels.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module; the GPU library never
calls it and shares no code with it.

The student is a DP-SE-style model: the descriptor contraction of Sec. II-B
without the attention refinement (a model with zero attention layers in the
weights format), so its energy, forces and parameters are those of
``dpa1_oracle``.  Training follows the usual energy-and-force matching of
deep potentials (Sec. II-B: a fitting net maps descriptors to atomic
energies, E = sum e_i by Eq. (5), forces are -dE/dx by Eq. (2)):

    L = p_e / B * sum_f ((E_f - E^_f) / N)^2
      + p_f / (3 N B) * sum_f sum_k |F_fk - F^_fk|^2

over a batch of B frames of N atoms, with labels E^, F^ from the teacher.
The gradient dL/dtheta is taken here by torch reverse-mode autograd through
the force computation itself (the forces are built with create_graph=True,
so the force term is differentiated exactly); nothing is hand-derived.

The optimiser is Adam in the form of Kingma and Ba (2015), Algorithm 1:
m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2, bias-corrected moments
m^ = m/(1-b1^t), v^ = v/(1-b2^t), theta <- theta - lr m^/(sqrt(v^) + eps).
"""

from __future__ import annotations

import dataclasses

import numpy as np
import torch

from .dpa1_oracle import OracleModel, atomic_energies, neighbor_list, pair_vectors


def param_names(model: OracleModel) -> list:
    """Tensor names in weights-file order (the order of ``model.t``)."""
    return list(model.t.keys())


def param_count(model: OracleModel) -> int:
    return int(sum(v.numel() for v in model.t.values()))


def flatten(model: OracleModel, tensors: dict | None = None) -> np.ndarray:
    """All tensors concatenated in file order (FP64)."""
    tensors = model.t if tensors is None else tensors
    return np.concatenate([np.asarray(tensors[k], dtype=np.float64).ravel()
                           for k in param_names(model)])


def unflatten(model: OracleModel, flat: np.ndarray) -> dict:
    out, off = {}, 0
    for k in param_names(model):
        n = model.t[k].numel()
        out[k] = torch.tensor(np.asarray(flat[off:off + n]).reshape(model.t[k].shape),
                              dtype=torch.float64)
        off += n
    return out


def _frame_energy_forces(model: OracleModel, coords, types, box, rcut: float, sel: int,
                         create_graph: bool):
    """E = sum_i e_i over every atom of the frame and F = -dE/dx (Eq. (2), Eq. (5))."""
    coords = np.asarray(coords, dtype=np.float64)
    types = np.asarray(types)
    n = coords.shape[0]
    nl = neighbor_list(coords, box, rcut, np.arange(n))
    for ci, lst in enumerate(nl):
        if len(lst) > sel:
            raise ValueError(f"atom {ci} has {len(lst)} neighbours > sel={sel}")
    nmax = max([len(x) for x in nl] + [1])
    jj = np.zeros((n, nmax), dtype=np.int64)
    msk = np.zeros((n, nmax), dtype=bool)
    for b, lst in enumerate(nl):
        jj[b, :len(lst)] = lst
        msk[b, :len(lst)] = True
    ii = np.repeat(np.arange(n)[:, None], nmax, axis=1)
    dmin = pair_vectors(coords, ii.ravel(), jj.ravel(), box).reshape(n, nmax, 3)
    # d = x_j - x_i - image shift; the shift is a constant lattice vector
    shift = torch.tensor((coords[jj] - coords[ii]) - dmin)
    x = torch.tensor(coords, requires_grad=True)
    d = x[torch.tensor(jj)] - x[torch.tensor(ii)] - shift
    mask = torch.tensor(msk)
    pad = torch.tensor([2.0 * rcut, 0.0, 0.0], dtype=torch.float64)
    d = torch.where(mask[..., None], d, pad)
    e = atomic_energies(model, d, mask, torch.tensor([len(x) for x in nl]),
                        torch.tensor(types, dtype=torch.int64),
                        torch.tensor(types[jj], dtype=torch.int64), rcut, sel)
    E = e.sum()
    (g,) = torch.autograd.grad(E, x, create_graph=create_graph)
    return E, -g


def batch_loss(model: OracleModel, frames, types, box, e_label, f_label, rcut: float, sel: int,
               pref_e: float, pref_f: float, create_graph: bool = False):
    """(L, L_e, L_f) of a batch as torch scalars (definition above)."""
    frames = np.asarray(frames, dtype=np.float64)
    B, N = frames.shape[0], frames.shape[1]
    le = torch.zeros((), dtype=torch.float64)
    lf = torch.zeros((), dtype=torch.float64)
    for b in range(B):
        E, F = _frame_energy_forces(model, frames[b], types, box, rcut, sel, create_graph)
        le = le + pref_e / B * ((E - float(e_label[b])) / N) ** 2
        lf = lf + pref_f / (3.0 * N * B) * ((F - torch.tensor(f_label[b])) ** 2).sum()
    return le + lf, le, lf


def loss_and_grad(model: OracleModel, frames, types, box, e_label, f_label, rcut: float,
                  sel: int, pref_e: float, pref_f: float):
    """Loss parts and dL/dtheta for every tensor (dict, FP64 numpy) by exact autograd."""
    params = {k: v.clone().requires_grad_(True) for k, v in model.t.items()}
    m2 = dataclasses.replace(model, t=params)
    L, le, lf = batch_loss(m2, frames, types, box, e_label, f_label, rcut, sel, pref_e, pref_f,
                           create_graph=True)
    grads = torch.autograd.grad(L, list(params.values()), allow_unused=True)
    out = {}
    for (k, p), g in zip(params.items(), grads):
        out[k] = np.zeros(tuple(p.shape)) if g is None else g.detach().numpy()
    return (float(L.detach()), float(le.detach()), float(lf.detach())), out


def loss_value(model: OracleModel, frames, types, box, e_label, f_label, rcut: float, sel: int,
               pref_e: float, pref_f: float) -> float:
    L, _, _ = batch_loss(model, frames, types, box, e_label, f_label, rcut, sel, pref_e, pref_f)
    return float(L.detach())


def labels(model: OracleModel, frames, types, box, rcut: float, sel: int):
    """Energies [B] and forces [B, N, 3] of a model on each frame."""
    frames = np.asarray(frames, dtype=np.float64)
    es, fs = [], []
    for b in range(frames.shape[0]):
        E, F = _frame_energy_forces(model, frames[b], types, box, rcut, sel, False)
        es.append(float(E))
        fs.append(F.detach().numpy())
    return np.array(es), np.stack(fs)


@dataclasses.dataclass
class AdamState:
    m: np.ndarray
    v: np.ndarray
    t: int = 0


def adam_init(n: int) -> AdamState:
    return AdamState(np.zeros(n), np.zeros(n), 0)


def adam_step(theta: np.ndarray, g: np.ndarray, st: AdamState, lr: float, beta1: float,
              beta2: float, eps: float) -> np.ndarray:
    """One Adam update (Kingma and Ba 2015, Algorithm 1); returns the new theta."""
    st.t += 1
    st.m = beta1 * st.m + (1.0 - beta1) * g
    st.v = beta2 * st.v + (1.0 - beta2) * g * g
    mhat = st.m / (1.0 - beta1 ** st.t)
    vhat = st.v / (1.0 - beta2 ** st.t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps)
