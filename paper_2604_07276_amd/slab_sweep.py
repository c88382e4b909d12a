"""Slab sweep on one GPU: the per-domain step time behind the paper's
strong-scaling model (Sec. VI-B, Eq. (8)).

Under a domain decomposition into N_p slabs, each rank evaluates its own
N/N_p local atoms plus a ghost population whose size depends on the cutoff,
not on N_p, so the time of one rank's step is t(N_p) = alpha/N_p + beta and
the throughput of the N_p-rank system is tr = 1/t (Eq. (8)).  This module
times one rank's step for N_p = 1, 2, 4, ..., 32 slabs of the 15,668-atom
protein-shaped frame on this GPU and fits alpha and beta, for two halo
schemes:

* ``rc``: the r_c halo of this library (Eq. (7)): the slab's atoms are the
  centres, the atoms within r_c of the slab are ghosts and receive forces
  that the owner would reduce.
* ``2rc``: the paper's scheme (Sec. IV-A): atoms within r_c of the slab are
  also centres (their energies are computed again by this rank), atoms
  between r_c and 2 r_c are ghosts, and the forces on the slab's own atoms
  are complete without any reduction.

Run: ``python -m paper_2604_07276_amd.slab_sweep [--steps K]``; prints one
JSON object.  Needs the built library and a GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile

import numpy as np

from . import binding, synth

RCUT = 6.0
SEL = 120
SLABS = (1, 2, 4, 8, 16, 32)


def domain(sysm, n_slabs: int, halo: str):
    """(coords, types, nloc, nghost) of slab 0 of n_slabs, locals first."""
    n = len(sysm.coords)
    if n_slabs == 1:
        return sysm.coords, sysm.types, n, 0
    L = float(sysm.box[0, 0])
    local, g1 = synth.slab_partition(sysm.coords, L, n_slabs, 0, RCUT)
    if halo == "rc":
        centres, ghosts = local, g1
    else:
        _, g2 = synth.slab_partition(sysm.coords, L, n_slabs, 0, 2.0 * RCUT)
        centres = np.sort(np.concatenate([local, g1]))
        ghosts = np.setdiff1d(g2, g1)
    idx = np.concatenate([centres, ghosts])
    return (np.ascontiguousarray(sysm.coords[idx]), np.ascontiguousarray(sysm.types[idx]),
            len(centres), len(ghosts))


def time_step(model, coords, types, box, nloc, nghost, steps: int) -> float:
    """Median device time of one dp_compute_device step on resident inputs (ms)."""
    import torch
    dev = torch.device("cuda:0")
    c = torch.tensor(coords, device=dev)
    t = torch.tensor(types, device=dev)
    nall = nloc + nghost
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    f = torch.zeros((nall, 3), dtype=torch.float64, device=dev)
    v = torch.zeros(9, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        model.compute_device(c, t, box, nloc, nghost, e, f, v, None, stream)
    model.sync()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record(stream)
    for k in range(steps):
        model.compute_device(c, t, box, nloc, nghost, e, f, v, None, stream)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    model.sync()
    return float(np.median([evs[k].elapsed_time(evs[k + 1]) for k in range(steps)]))


def fit(n_p: np.ndarray, t_ms: np.ndarray):
    """Least-squares alpha, beta of t = alpha/N_p + beta (ms)."""
    A = np.stack([1.0 / n_p, np.ones_like(n_p)], axis=1)
    (alpha, beta), *_ = np.linalg.lstsq(A, t_ms, rcond=None)
    return float(alpha), float(beta)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--precision", choices=("fp32", "bf16"), default="fp32")
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("the slab sweep needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    wpath = os.path.join(tempfile.mkdtemp(), "dpa1_seed0.bin")
    synth.make_weights(wpath, seed=0)
    model = binding.Model(wpath, RCUT, SEL)
    if args.precision == "bf16":
        model.set_precision(binding.PREC_BF16)
    sysm = synth.protein_system(0)
    n = len(sysm.coords)
    out = {"workload": f"protein-shaped periodic frame, {n} atoms, rcut {RCUT}, slab 0 of N_p "
                       f"along x, full box passed", "precision": args.precision, "halo": {}}
    for halo in ("rc", "2rc"):
        rows = []
        for ns in SLABS:
            if halo == "2rc" and ns == 1:
                continue
            coords, types, nloc, nghost = domain(sysm, ns, halo)
            ms = time_step(model, coords, types, sysm.box, nloc, nghost, args.steps)
            rows.append({"n_p": ns, "centres": nloc, "ghosts": nghost, "ms_per_step": round(ms, 4),
                         "tr_steps_per_s": round(1e3 / ms, 2)})
            print(json.dumps({"halo": halo, **rows[-1]}), file=sys.stderr, flush=True)
        sl = [r for r in rows if r["n_p"] >= 2]
        alpha, beta = fit(np.array([r["n_p"] for r in sl], dtype=float),
                          np.array([r["ms_per_step"] for r in sl]))
        for r in rows:
            r["model_ms"] = round(alpha / r["n_p"] + beta, 4)
        out["halo"][halo] = {"rows": rows, "alpha_ms": round(alpha, 4), "beta_ms": round(beta, 4),
                             "fit_on": "N_p >= 2"}
    model.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
