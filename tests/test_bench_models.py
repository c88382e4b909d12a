"""The work models behind bench.py's roofline block: the fused kernels do the
work of several separate ones, and the step total counts it once."""

import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402

SHAPE = {"M": 100, "dattn": 128, "n_attn": 2, "emb": [25, 50, 100], "axis": 16, "tebd": 8,
         "fit": [240, 240, 240]}


def _nnei(seed=0, n=3000):
    # neighbour counts spread over all four classes
    return np.random.default_rng(seed).integers(1, 129, size=n)


def test_fused_forward_counts_attention_plus_projection():
    nn = _nnei()
    f = bench.flop_model(nn, SHAPE)
    fused = sum(f[f"attn_fwd_ln_n{c}"][0] for c in (32, 64, 96, 128))
    parts = sum(f[f"attn_fwd_n{c}"][0] for c in (32, 64, 96, 128)) + f["oproj_ln_fwd"][0]
    assert abs(fused - parts) <= 1e-9 * parts


def test_fused_adjoints_count_both_halves():
    nn = _nnei(1)
    f = bench.flop_model(nn, SHAPE)
    halves = sum(f[f"attn_bwd_q_n{c}"][0] + f[f"attn_bwd_k_n{c}"][0] for c in (32, 64, 96, 128))
    fused = sum(f[f"attn_bwd_n{c}"][0] for c in (32, 64, 96, 128))
    assert abs(fused - halves) <= 1e-9 * halves


def test_step_total_counts_fused_work_once():
    nn = _nnei(2)
    f = bench.flop_model(nn, SHAPE)
    separate = sum(v for k, (v, _) in f.items() if not k.startswith(bench.FUSED_VARIANTS))
    assert bench.step_flop_total(f) == separate
    assert bench.step_flop_total(f) < sum(v for v, _ in f.values())
    # attention core: forward Q K^T and A V, backward dA, dQ, dK, dV: 6 x 2 d n^2 per layer
    n2 = float((nn.astype(np.float64) ** 2).sum())
    core = sum(f[f"{k}_n{c}"][0] for k in ("attn_fwd", "attn_bwd_q", "attn_bwd_k")
               for c in (32, 64, 96, 128))
    assert abs(core - SHAPE["n_attn"] * 6 * 2 * SHAPE["dattn"] * n2) <= 1e-9 * core


def test_fused_descriptor_adjoint_counts_one_projection_layer():
    nn = _nnei(4)
    f = bench.flop_model(nn, SHAPE)
    fused, launches = f["desc_oproj_bwd"]
    one_layer = f["oproj_bwd"][0] / SHAPE["n_attn"]
    assert launches == 1
    assert abs(fused - (f["desc_bwd"][0] + one_layer)) <= 1e-9 * fused
    # 2 d M per pair for the projection adjoint of one layer
    assert abs(one_layer - 2.0 * SHAPE["dattn"] * SHAPE["M"] * float(nn.sum())) <= 1e-9 * one_layer


def test_fused_adjoint_bytes_drop_the_stored_intermediates():
    nn = _nnei(3)
    b = bench.byte_model(nn, SHAPE)
    two = sum(b[f"attn_bwd_q_n{c}"][0] + b[f"attn_bwd_k_n{c}"][0] for c in (32, 64, 96, 128))
    fused = sum(b[f"attn_bwd_n{c}"][0] for c in (32, 64, 96, 128))
    # dA, the statistics and the query sums no longer pass through memory
    assert fused < two


def test_bf16_byte_model_halves_only_the_bf16_stored_tensors():
    nn = _nnei(4)
    b32 = bench.byte_model(nn, SHAPE)
    b16 = bench.byte_model(nn, SHAPE, bf16=True)
    L, d, M = SHAPE["n_attn"], SHAPE["dattn"], SHAPE["M"]
    P = float(nn.sum())
    # QKV written in BF16, X read in FP32
    assert abs((b32["qkv_fwd"][0] - b16["qkv_fwd"][0]) - L * P * 2 * 3 * d) < 1e-6 * b32["qkv_fwd"][0]
    # the projection adjoint reads dY (FP32) and writes dO (BF16)
    assert abs((b32["oproj_bwd"][0] - b16["oproj_bwd"][0]) - L * P * 2 * d) < 1e-6 * b32["oproj_bwd"][0]
    # logits and statistics stay FP32 in the attention kernels
    for c in (32, 64, 96, 128):
        assert b16[f"attn_fwd_n{c}"][0] < b32[f"attn_fwd_n{c}"][0] or b32[f"attn_fwd_n{c}"][0] == 0
    assert bench.byte_model(nn, SHAPE)["qkv_bwd"][0] == b32["qkv_bwd"][0]
    assert M == 100


def test_descriptor_adjoint_bytes_count_its_operands_once():
    nn = _nnei(5)
    P, nloc = float(nn.sum()), len(nn)
    M, d, axis = SHAPE["M"], SHAPE["dattn"], SHAPE["axis"]
    for bf16, t in ((False, 4.0), (True, 2.0)):
        b, launches = bench.byte_model(nn, SHAPE, bf16=bf16)["desc_oproj_bwd"]
        # G, xhat, 1/std and R~ in; the residual gradient, dR~ and dO out; dD and T per centre
        want = P * (4.0 * (2 * M + 1) + 16.0 + 4.0 * M + 16.0 + t * d) + nloc * 4.0 * (M * axis + 4 * M)
        assert launches == 1
        assert abs(b - want) <= 1e-9 * want

