"""Seeded synthetic inputs: atomic systems and random-initialised DPA-1 weights.

This module only draws numbers and lays them out.  It contains none of the
model's arithmetic (no switch function, no network, no neighbour search): the
GPU library, its Python binding, the tests and the benchmark all take their
inputs from here, so the two independent implementations see identical data.

Workloads stand in for the solvated protein of the paper's benchmarks
(Sec. V-B: 15,668 neural-network atoms of a solvated protein chain), which is
not available here: a jittered cubic lattice at the density of liquid water
(0.1 atoms per cubic Angstrom) with the element mix of a hydrated protein.

Weights file format (little endian), read independently by the C++ library and
by the CPU oracle:

    bytes 0..7   magic b"DPA1WTS\\0"
    uint32       version (= 1)
    uint32       n_int, followed by n_int int32 fields:
                 ntypes, tebd_dim, axis, n_attn, attn_dim, n_emb, n_fit,
                 emb[0..n_emb), fit[0..n_fit)
    uint32       n_dbl, followed by n_dbl float64 fields:
                 rcut_smth, attn_shift, ln_eps
    float64 tensors, row-major, in this order:
        type_embedding [ntypes][tebd_dim]
        embedding layer l = 0..n_emb-1:   W [in_l][emb[l]], b [emb[l]]
                                          (in_0 = 1 + 2*tebd_dim, in_l = emb[l-1])
        attention layer a = 0..n_attn-1:  Wq [M][d], bq [d], Wk [M][d], bk [d],
                                          Wv [M][d], bv [d], Wo [d][M], bo [M],
                                          ln_gamma [M], ln_beta [M]
                                          (M = emb[-1], d = attn_dim)
        fitting layer l = 0..n_fit-1:     W [in_l][fit[l]], b [fit[l]]
                                          (in_0 = M*axis + tebd_dim)
        w_out [fit[-1]], b_out [1]
        energy_bias [ntypes]

Random initialisation: every weight matrix is Xavier-normal,
N(0, 2/(fan_in + fan_out)) (the type table uses fan_in = ntypes); every bias,
b_out and the per-type energy bias are N(0, 0.01^2); layer-norm gamma = 1 and
beta = 0 are written but not drawn.  All tensors are drawn in file order from
one PCG64 stream.
"""

from __future__ import annotations

import dataclasses
import math
import struct

import numpy as np

MAGIC = b"DPA1WTS\0"
VERSION = 1

# Element order of the type index: H, C, N, O, S.
TYPE_NAMES = ("H", "C", "N", "O", "S")
# Element fractions of the protein-shaped workload (H/C/N/O/S).
PROTEIN_FRACTIONS = (0.64, 0.10, 0.03, 0.22, 0.01)


@dataclasses.dataclass(frozen=True)
class ModelShape:
    """Hyper-parameters of a DPA-1 model (the seeded benchmark model by default)."""

    ntypes: int = 5
    tebd_dim: int = 8
    emb: tuple = (25, 50, 100)
    axis: int = 16
    n_attn: int = 2
    attn_dim: int = 128
    fit: tuple = (240, 240, 240)
    rcut_smth: float = 0.5
    attn_shift: float = 20.0
    ln_eps: float = 1e-5


# Distilled student (DP-SE-style: no attention), 86,318 parameters with 5 types.
STUDENT_SHAPE = ModelShape(emb=(16, 32, 64), axis=8, n_attn=0, fit=(128, 128))


def _streams(seed: int):
    """Four independent PCG64 streams: geometry, types, weights, perturbation."""
    ss = np.random.SeedSequence(seed).spawn(4)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss]


def weight_tensor_shapes(shape: ModelShape):
    """(name, shape, kind) of every stored tensor in file order.

    kind is "w" (Xavier-normal, fan_in/fan_out from the shape), "b" (N(0, 0.01^2)),
    "one" (constant 1) or "zero" (constant 0).
    """
    out = [("type_embedding", (shape.ntypes, shape.tebd_dim), "w")]
    fin = 1 + 2 * shape.tebd_dim
    for l, w in enumerate(shape.emb):
        out.append((f"emb{l}.W", (fin, w), "w"))
        out.append((f"emb{l}.b", (w,), "b"))
        fin = w
    m = shape.emb[-1]
    d = shape.attn_dim
    for a in range(shape.n_attn):
        for nm in ("q", "k", "v"):
            out.append((f"attn{a}.W{nm}", (m, d), "w"))
            out.append((f"attn{a}.b{nm}", (d,), "b"))
        out.append((f"attn{a}.Wo", (d, m), "w"))
        out.append((f"attn{a}.bo", (m,), "b"))
        out.append((f"attn{a}.ln_gamma", (m,), "one"))
        out.append((f"attn{a}.ln_beta", (m,), "zero"))
    fin = m * shape.axis + shape.tebd_dim
    for l, w in enumerate(shape.fit):
        out.append((f"fit{l}.W", (fin, w), "w"))
        out.append((f"fit{l}.b", (w,), "b"))
        fin = w
    out.append(("w_out", (fin,), "w_out"))
    out.append(("b_out", (1,), "b"))
    out.append(("energy_bias", (shape.ntypes,), "b"))
    return out


def draw_weights(shape: ModelShape, seed: int) -> dict:
    """Draw every tensor of the model from the seed's weight stream (file order)."""
    rng = _streams(seed)[2]
    tensors = {}
    for name, shp, kind in weight_tensor_shapes(shape):
        if kind == "w":
            fan_in, fan_out = shp
            std = math.sqrt(2.0 / (fan_in + fan_out))
            tensors[name] = rng.normal(0.0, std, size=shp)
        elif kind == "w_out":
            std = math.sqrt(2.0 / (shp[0] + 1))
            tensors[name] = rng.normal(0.0, std, size=shp)
        elif kind == "b":
            tensors[name] = rng.normal(0.0, 0.01, size=shp)
        elif kind == "one":
            tensors[name] = np.ones(shp)
        else:
            tensors[name] = np.zeros(shp)
    return tensors


def write_weights(path: str, shape: ModelShape, tensors: dict) -> None:
    """Write a weights file in the format described in the module docstring."""
    ints = [shape.ntypes, shape.tebd_dim, shape.axis, shape.n_attn, shape.attn_dim,
            len(shape.emb), len(shape.fit), *shape.emb, *shape.fit]
    dbls = [shape.rcut_smth, shape.attn_shift, shape.ln_eps]
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<II", VERSION, len(ints)))
        f.write(struct.pack(f"<{len(ints)}i", *ints))
        f.write(struct.pack("<I", len(dbls)))
        f.write(struct.pack(f"<{len(dbls)}d", *dbls))
        for name, shp, _ in weight_tensor_shapes(shape):
            arr = np.ascontiguousarray(tensors[name], dtype="<f8")
            assert arr.shape == tuple(shp), (name, arr.shape, shp)
            f.write(arr.tobytes())


def make_weights(path: str, seed: int = 0, shape: ModelShape | None = None) -> ModelShape:
    """Draw a seeded random-init model and write it to ``path``."""
    shape = shape or ModelShape()
    write_weights(path, shape, draw_weights(shape, seed))
    return shape


def largest_remainder_counts(n: int, fractions) -> np.ndarray:
    """Integer counts summing to n, proportional to ``fractions``."""
    fr = np.asarray(fractions, dtype=np.float64)
    fr = fr / fr.sum()
    raw = fr * n
    counts = np.floor(raw).astype(np.int64)
    rem = n - counts.sum()
    order = np.argsort(-(raw - counts), kind="stable")
    counts[order[:rem]] += 1
    return counts


@dataclasses.dataclass
class System:
    coords: np.ndarray  # [N][3] float64, Angstrom
    types: np.ndarray   # [N] int32
    box: np.ndarray | None  # [3][3] float64 rows = cell vectors, or None (open)
    seed: int = 0


def lattice_system(n_atoms: int, box_len: float, fractions, seed: int = 0,
                   jitter: float = 0.3) -> System:
    """Jittered cubic lattice in a periodic cube, seeded.

    n = ceil(N^(1/3)) sites per side at spacing a = L/n, site centres (g + 1/2) a;
    N of the n^3 sites are chosen at random, each gets a uniform +-jitter
    displacement per component and the result is wrapped into [0, L).
    """
    g_rng, t_rng, _, _ = _streams(seed)
    n = int(math.ceil(n_atoms ** (1.0 / 3.0) - 1e-9))
    a = box_len / n
    sites = g_rng.permutation(n ** 3)[:n_atoms]
    ijk = np.stack(np.unravel_index(sites, (n, n, n)), axis=1).astype(np.float64)
    coords = (ijk + 0.5) * a
    coords = coords + g_rng.uniform(-jitter, jitter, size=coords.shape)
    coords = np.mod(coords, box_len)
    counts = largest_remainder_counts(n_atoms, fractions)
    types = np.repeat(np.arange(len(counts), dtype=np.int32), counts)
    types = t_rng.permutation(types).astype(np.int32)
    box = np.eye(3) * box_len
    return System(coords=coords, types=types, box=box, seed=seed)


def parity_system(seed: int = 0) -> System:
    """192 atoms (O:H = 1:2) in a periodic 12.4 Angstrom cube: the small parity case."""
    # types index: H=0, O=3
    sysm = lattice_system(192, 12.4, (2.0, 0.0, 0.0, 1.0, 0.0), seed=seed)
    return sysm


def protein_system(seed: int = 0) -> System:
    """15,668 atoms in a periodic 53.9 Angstrom cube with the protein element mix."""
    return lattice_system(15668, 53.9, PROTEIN_FRACTIONS, seed=seed)


def perturbed_frames(base: System, n_frames: int, sigma: float = 0.01) -> np.ndarray:
    """[n_frames][N][3] cumulative N(0, sigma) random walk of the positions, wrapped.

    Frame 0 is the unperturbed system.
    """
    rng = _streams(base.seed)[3]
    L = np.diag(base.box)
    out = np.empty((n_frames,) + base.coords.shape)
    x = base.coords.copy()
    for f in range(n_frames):
        if f > 0:
            x = np.mod(x + rng.normal(0.0, sigma, size=x.shape), L)
        out[f] = x
    return out


def noisy_frame(base: System, index: int, sigma: float = 0.05) -> np.ndarray:
    """Frame ``index`` of an independent-noise ensemble: base positions plus
    N(0, sigma^2) per component, wrapped into the box.  Each frame has its own
    seeded stream, so any subset can be drawn in any order."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([base.seed, 7, index])))
    x = base.coords + rng.normal(0.0, sigma, size=base.coords.shape)
    if base.box is not None:
        x = np.mod(x, np.diag(base.box))
    return x


def slab_partition(coords: np.ndarray, box_len: float, n_slabs: int, index: int,
                   halo: float):
    """Local and ghost atom indices of slab ``index`` of ``n_slabs`` along x.

    Atoms are ranked by x (ties by index); slab s owns ranks
    [round(s N / n_slabs), round((s+1) N / n_slabs)).  Ghosts are the other atoms
    whose periodic x-distance to the slab's x-range is below ``halo``.
    Returns (local_idx, ghost_idx), both sorted ascending.
    """
    n = coords.shape[0]
    order = np.lexsort((np.arange(n), coords[:, 0]))
    lo = int(round(index * n / n_slabs))
    hi = int(round((index + 1) * n / n_slabs))
    local = np.sort(order[lo:hi])
    if local.size == 0:
        return local, np.zeros(0, dtype=np.int64)
    xs = coords[local, 0]
    x0, x1 = xs.min(), xs.max()
    others = np.setdiff1d(np.arange(n), local)
    x = coords[others, 0]
    # periodic distance from x to the interval [x0, x1]
    c = 0.5 * (x0 + x1)
    half = 0.5 * (x1 - x0)
    dx = x - c
    dx = dx - box_len * np.rint(dx / box_len)
    dist = np.maximum(np.abs(dx) - half, 0.0)
    ghost = np.sort(others[dist < halo])
    return local, ghost


def replicate(sysm: System, reps=(2, 2, 1)) -> System:
    """Tile a periodic orthorhombic system reps[0] x reps[1] x reps[2] times."""
    L = np.diag(sysm.box)
    shifts = np.array([[i, j, k] for i in range(reps[0]) for j in range(reps[1])
                       for k in range(reps[2])], dtype=np.float64) * L
    coords = (sysm.coords[None, :, :] + shifts[:, None, :]).reshape(-1, 3)
    types = np.tile(sysm.types, len(shifts)).astype(np.int32)
    box = np.diag(L * np.asarray(reps, dtype=np.float64))
    return System(coords=coords, types=types, box=box, seed=sysm.seed)


def open_cluster(n_atoms: int, radius: float, ntypes: int, seed: int = 0,
                 min_dist: float = 0.9) -> System:
    """Random atoms in a sphere with a minimum pair distance, open boundaries."""
    g_rng, t_rng, _, _ = _streams(seed)
    pts = []
    tries = 0
    while len(pts) < n_atoms:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place atoms")
        p = g_rng.uniform(-radius, radius, size=3)
        if np.dot(p, p) > radius * radius:
            continue
        if pts and np.min(np.sum((np.asarray(pts) - p) ** 2, axis=1)) < min_dist ** 2:
            continue
        pts.append(p)
    types = t_rng.integers(0, ntypes, size=n_atoms).astype(np.int32)
    return System(coords=np.asarray(pts), types=types, box=None, seed=seed)
