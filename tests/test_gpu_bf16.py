"""BF16 precision mode (dp_set_precision): BF16 matrix-core operands, FP32
accumulation, FP32 geometry / descriptor / softmax / norms, FP64 reductions.

The accuracy statements are against the FP64 oracle.  The BF16 unit roundoff
is 2^-9 (3.9e-3 relative per rounded operand); the random-initialised model
passes every attention output through a layer norm whose input spread is
close to sqrt(eps), which amplifies operand rounding in the adjoint, so the
force errors have a heavy tail.  The bars below: force
RMSE <= 5e-3 eV/A (the stated BF16 target), energy per atom <= 5e-4 eV and a
loose bound on the largest force error that catches indexing mistakes (a
wrong operand or tile gives errors of the size of the forces themselves).
"""

import sys

import numpy as np
import pytest

from oracle import dpa1_oracle as orc
from paper_2604_07276_amd import synth

pytestmark = pytest.mark.gpu

RC = 6.0
SEL = 120
F_RMSE = 5e-3
E_TOL = 5e-4


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


def test_bf16_parity_192_atoms(model, oracle_model):
    from paper_2604_07276_amd import binding
    s = synth.parity_system(0)
    say("case: BF16 mode, 192-atom periodic system vs the FP64 oracle")
    r = orc.compute(oracle_model, s.coords, s.types, s.box, 192, 0, RC, SEL)
    model.set_precision(binding.PREC_BF16)
    try:
        E, F, V, ae = model.compute(s.coords, s.types, s.box, 192, 0, atom_energy=True)
    finally:
        model.set_precision(binding.PREC_FP32)
    dF = F - r.forces
    rmse = np.sqrt((dF ** 2).mean())
    dE = abs(E - r.energy) / 192
    say(f"[bf16 192] dE/N={dE:.2e} force RMSE={rmse:.2e} max={np.abs(dF).max():.2e} "
        f"(|F|rms={np.sqrt((r.forces ** 2).mean()):.2e}) max|de_i|={np.abs(ae - r.atom_energy).max():.2e}")
    assert dE <= E_TOL
    assert rmse <= F_RMSE
    assert np.abs(dF).max() <= 0.1
    assert np.abs(V - r.virial).max() / 192 <= E_TOL
    # BF16 rounding must actually be in effect (not a silent FP32 run)
    assert rmse > 1e-6


def test_bf16_parity_98_features(tmp_path):
    """BF16 mode on a model with 98 embedding features (widths 25 -> 50 -> 98):
    the BF16 kernels that take the last 16-wide feature chunk with two real
    features (QKV projection, forward with the projection, descriptor adjoint
    with dO) and the fused embedding kernels without a last-layer residual,
    against the FP64 oracle at the same bars."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_07276_amd import binding
    p = str(tmp_path / "emb98.bin")
    synth.make_weights(p, seed=3, shape=synth.ModelShape(emb=(25, 50, 98), n_attn=2))
    om = orc.load_model(p)
    s = synth.parity_system(1)
    say("case: BF16 mode, 98 embedding features, 192-atom system vs the FP64 oracle")
    r = orc.compute(om, s.coords, s.types, s.box, 192, 0, RC, SEL)
    m = binding.Model(p, RC, SEL)
    try:
        m.set_precision(binding.PREC_BF16)
        E, F, V, _ = m.compute(s.coords, s.types, s.box, 192, 0)
    finally:
        m.close()
    dF = F - r.forces
    rmse = np.sqrt((dF ** 2).mean())
    dE = abs(E - r.energy) / 192
    say(f"[bf16 emb98] dE/N={dE:.2e} force RMSE={rmse:.2e} max={np.abs(dF).max():.2e} "
        f"(|F|rms={np.sqrt((r.forces ** 2).mean()):.2e})")
    assert dE <= E_TOL
    assert rmse <= F_RMSE
    assert np.abs(dF).max() <= 0.1
    assert np.abs(V - r.virial).max() / 192 <= E_TOL
    assert rmse > 1e-6


def test_bf16_protein_15668(model, oracle_model):
    """Whole 15,668-atom frame in BF16 against the FP32 path (itself within
    1e-4 eV/A of the oracle), and e_i of 400 random centres against the oracle."""
    from paper_2604_07276_amd import binding
    s = synth.protein_system(0)
    n = len(s.coords)
    say(f"case: BF16 mode, protein-shaped system N={n}")
    E32, F32, _, ae32 = model.compute(s.coords, s.types, s.box, n, 0, atom_energy=True)
    model.set_precision(binding.PREC_BF16)
    try:
        E16, F16, _, ae16 = model.compute(s.coords, s.types, s.box, n, 0, atom_energy=True)
    finally:
        model.set_precision(binding.PREC_FP32)
    dF = np.linalg.norm(F16 - F32, axis=1)
    rmse = np.sqrt(((F16 - F32) ** 2).mean())
    say(f"[bf16 protein] dE/N={abs(E16 - E32) / n:.2e} force RMSE={rmse:.2e} "
        f"p99={np.percentile(dF, 99):.2e} max={dF.max():.2e}")
    assert abs(E16 - E32) / n <= E_TOL
    assert rmse <= F_RMSE
    assert dF.max() <= 1.0
    rng = np.random.default_rng(5)
    centers = np.sort(rng.choice(n, 400, replace=False))
    pr = orc.evaluate_centers(oracle_model, s.coords, s.types, s.box, RC, SEL, centers)
    de = np.abs(ae16[pr.centers] - pr.atom_energy).max()
    say(f"[bf16 protein] max|de_i| vs oracle (400 centres) = {de:.2e}")
    assert de <= 5e-3


def test_precision_switch_is_isolated(model):
    """FP32 results after a BF16 step are bit-identical to those before it."""
    from paper_2604_07276_amd import binding
    s = synth.parity_system(2)
    say("case: FP32 -> BF16 -> FP32 on one handle")
    E0, F0, V0, _ = model.compute(s.coords, s.types, s.box, 192, 0)
    model.set_precision(binding.PREC_BF16)
    E1, F1, _, _ = model.compute(s.coords, s.types, s.box, 192, 0)
    model.set_precision(binding.PREC_FP32)
    E2, F2, V2, _ = model.compute(s.coords, s.types, s.box, 192, 0)
    assert E0 == E2 and np.array_equal(F0, F2) and np.array_equal(V0, V2)
    assert E1 != E0
    with pytest.raises(binding.DPError):
        model.set_precision(7)


def test_bf16_forward_adjoint_split(model):
    """In BF16 mode the forward/adjoint entry points reproduce the fused step."""
    import torch
    from paper_2604_07276_amd import binding
    s = synth.parity_system(0)
    say("case: BF16 forward_device + backward_device vs compute_device")
    dev = torch.device("cuda:0")
    c = torch.tensor(s.coords, device=dev)
    t = torch.tensor(s.types, device=dev)
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    f = torch.zeros((192, 3), dtype=torch.float64, device=dev)
    v = torch.zeros(9, dtype=torch.float64, device=dev)
    g = torch.zeros((192, 3), dtype=torch.float64, device=dev)
    model.set_precision(binding.PREC_BF16)
    try:
        model.compute_device(c, t, s.box, 192, 0, e, f, v)
        model.sync()
        F = f.cpu().numpy().copy()
        model.forward_device(c, t, s.box, 192, 0, e)
        model.backward_device(g)
        model.sync()
    finally:
        model.set_precision(binding.PREC_FP32)
    assert np.array_equal(-g.cpu().numpy(), F)
