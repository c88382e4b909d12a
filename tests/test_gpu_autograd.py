"""The hand-written adjoint behind torch.autograd.Function, on the GPU.

Checks: the autograd gradient of E equals minus the forces of the fused step
(bit for bit: same kernels, unit weights); weighted losses sum_i w_i e_i
match the FP64 oracle's gradient; several backwards after one forward; a
stale backward raises.  Finite differences pin the oracle's gradient (CPU
tests); on the FP32 GPU path they would be dominated by rounding noise.
"""

import numpy as np
import pytest

from oracle import dpa1_oracle as orc
from paper_2604_07276_amd import synth

pytestmark = pytest.mark.gpu

RC = 6.0
SEL = 120


@pytest.fixture(scope="module")
def model(weights_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_07276_amd import binding
    m = binding.Model(weights_path, RC, SEL)
    yield m
    m.close()


def _dev(a, dtype=None):
    import torch
    return torch.tensor(a, device="cuda:0", dtype=dtype)


def test_autograd_energy_gradient_is_minus_forces(model):
    import torch
    from paper_2604_07276_amd.autograd import atomic_energies
    s = synth.parity_system(4)
    print("case: autograd dE/dx vs fused forces, 192 atoms", flush=True)
    E, F, V, ae = model.compute(s.coords, s.types, s.box, 192, 0, atom_energy=True)
    x = _dev(s.coords).requires_grad_(True)
    e = atomic_energies(model, x, _dev(s.types), s.box, 192, 0)
    (gx,) = torch.autograd.grad(e.sum(), x)
    assert np.array_equal(e.detach().cpu().numpy(), ae)
    assert np.array_equal(gx.cpu().numpy(), -F)


def test_weighted_loss_matches_oracle_with_ghosts(model, oracle_model):
    import torch
    from paper_2604_07276_amd.autograd import atomic_energies
    s = synth.parity_system(5)
    L = s.box[0, 0]
    loc, gh = synth.slab_partition(s.coords, L, 3, 0, RC)
    idx = np.concatenate([loc, gh])
    x_np, t_np = s.coords[idx], s.types[idx]
    nloc, nghost = len(loc), len(gh)
    w_np = np.random.default_rng(1).normal(size=nloc)
    print(f"case: weighted loss, slab {nloc} locals + {nghost} ghosts", flush=True)
    x = _dev(x_np).requires_grad_(True)
    e = atomic_energies(model, x, _dev(t_np), s.box, nloc, nghost)
    loss = (e * _dev(w_np)).sum()
    (gx,) = torch.autograd.grad(loss, x)
    pr = orc.evaluate_centers(oracle_model, x_np, t_np, s.box, RC, SEL, np.arange(nloc))
    ref = np.zeros_like(x_np)
    wp = w_np[pr.pair_i]
    np.add.at(ref, pr.pair_j, wp[:, None] * pr.g)
    np.add.at(ref, pr.pair_i, -wp[:, None] * pr.g)
    err = np.abs(gx.cpu().numpy() - ref).max()
    print(f"[weighted] max|d grad| = {err:.2e} (|grad|max = {np.abs(ref).max():.3e})", flush=True)
    assert err <= 1e-4


def test_two_backwards_after_one_forward(model):
    import torch
    from paper_2604_07276_amd.autograd import atomic_energies
    s = synth.parity_system(6)
    print("case: two backward passes, one forward", flush=True)
    x = _dev(s.coords).requires_grad_(True)
    e = atomic_energies(model, x, _dev(s.types), s.box, 192, 0)
    w = torch.linspace(-1.0, 2.0, 192, dtype=torch.float64, device="cuda:0")
    (g1,) = torch.autograd.grad((e * w).sum(), x, retain_graph=True)
    (g2,) = torch.autograd.grad(e.sum(), x)
    E, F, V, _ = model.compute(s.coords, s.types, s.box, 192, 0)
    assert np.array_equal(g2.cpu().numpy(), -F)
    assert not np.array_equal(g1.cpu().numpy(), g2.cpu().numpy())


def test_stale_forward_raises(model):
    import torch
    from paper_2604_07276_amd.autograd import atomic_energies
    s = synth.parity_system(7)
    print("case: backward after a newer forward raises", flush=True)
    x = _dev(s.coords).requires_grad_(True)
    e1 = atomic_energies(model, x, _dev(s.types), s.box, 192, 0)
    e2 = atomic_energies(model, x, _dev(s.types), s.box, 96, 96)
    with pytest.raises(RuntimeError):
        torch.autograd.grad(e1.sum(), x)
    (g,) = torch.autograd.grad(e2.sum(), x)
    assert torch.isfinite(g).all()


def test_backward_raises_on_device_error_and_inplace_edit(model, weights_path):
    import torch
    from paper_2604_07276_amd import binding
    from paper_2604_07276_amd.autograd import atomic_energies
    s = synth.parity_system(8)
    print("case: backward after a neighbour overflow; backward after an in-place edit", flush=True)
    small = binding.Model(weights_path, RC, 40)
    try:
        x = _dev(s.coords).requires_grad_(True)
        e = atomic_energies(small, x, _dev(s.types), s.box, 192, 0)
        with pytest.raises(binding.DPError) as ei:
            torch.autograd.grad(e.sum(), x)
        assert ei.value.code == -4
    finally:
        small.close()
    leaf = _dev(s.coords).requires_grad_(True)
    x = leaf * 1.0  # a non-leaf that can be edited in place
    e = atomic_energies(model, x, _dev(s.types), s.box, 192, 0)
    with torch.no_grad():
        x.add_(0.01)
    with pytest.raises(RuntimeError):
        torch.autograd.grad(e.sum(), leaf)
