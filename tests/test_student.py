"""Audited serving of the distilled student: the teacher judges every k-th
step and takes over once the audited force RMSE exceeds the threshold (host
policy, CPU), and one small end-to-end run of the pipeline on the GPU."""

import numpy as np
import pytest

from paper_2604_07276_amd.student import AuditedPotential


def _rmse(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2))), float(np.max(np.abs(a - b)))


def _models(drift_from=None):
    calls = {"student": 0, "teacher": 0}

    def teacher(x):
        calls["teacher"] += 1
        return 1.0, np.ones((4, 3))

    def student(x):
        calls["student"] += 1
        off = 0.5 if drift_from is not None and x >= drift_from else 1e-3
        return 1.0, np.ones((4, 3)) + off

    return student, teacher, calls


def test_threshold_zero_forces_the_teacher_from_the_first_audit():
    s, t, calls = _models()
    pot = AuditedPotential(s, t, threshold=0.0, every=10, error_fn=_rmse)
    src = [pot(k)[2] for k in range(25)]
    assert src == ["teacher"] * 25
    assert pot.fallback and len(pot.audits) == 1 and pot.audits[0][0] == 0


def test_audits_every_kth_step_without_fallback():
    s, t, calls = _models()
    pot = AuditedPotential(s, t, threshold=3e-2, every=10, error_fn=_rmse)
    src = [pot(k)[2] for k in range(35)]
    assert src == ["student"] * 35
    assert [a[0] for a in pot.audits] == [0, 10, 20, 30]
    assert calls["teacher"] == 4 and calls["student"] == 35
    assert all(abs(a[1] - 1e-3) < 1e-12 for a in pot.audits)


def test_drift_is_caught_at_the_next_audit():
    s, t, calls = _models(drift_from=23)
    pot = AuditedPotential(s, t, threshold=3e-2, every=10, error_fn=_rmse)
    src = [pot(k)[2] for k in range(40)]
    # steps 23..29 are served by the drifted student; the audit at 30 hands over
    assert src[:30] == ["student"] * 30 and src[30:] == ["teacher"] * 10
    assert pot.fallback and pot.audits[-1][0] == 30


def test_bad_interval_rejected():
    s, t, _ = _models()
    with pytest.raises(ValueError):
        AuditedPotential(s, t, 1.0, every=0)


@pytest.mark.gpu
def test_pipeline_small_run():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_07276_amd import student
    print("student pipeline: 16 train + 4 held-out frames of 15,668 atoms, 4 steps", flush=True)
    out = student.run(n_train=16, n_eval=4, steps=4, audit_every=2)
    assert out["training"]["steps"] == 4
    assert np.isfinite(out["held_out"]["force_rmse_eV_per_A"])
    assert out["serving"]["student_steps"] + out["serving"]["teacher_steps"] == 4
    assert out["throughput"]["speedup_vs_teacher"] > 1.0


def test_relative_criterion_catches_a_zero_force_student():
    """A student that returns F = 0 has an absolute force RMSE equal to the
    teacher's force RMS; with small teacher forces that passes the absolute
    3e-2 eV/A bound, and the relative bound must catch it at the first audit."""
    rng = np.random.default_rng(0)
    Ft = rng.normal(0.0, 0.02, size=(64, 3))

    def teacher(x):
        return 1.0, Ft

    def student(x):
        return 1.0, np.zeros_like(Ft)

    absolute_only = AuditedPotential(student, teacher, threshold=3e-2, every=5, error_fn=_rmse)
    assert [absolute_only(k)[2] for k in range(10)] == ["student"] * 10
    pot = AuditedPotential(student, teacher, threshold=3e-2, every=5, error_fn=_rmse,
                           rel_threshold=0.5)
    src = [pot(k)[2] for k in range(10)]
    assert src == ["teacher"] * 10 and pot.fallback
    k, rmse, mx, scale = pot.audits[0]
    assert k == 0 and abs(rmse - scale) < 1e-15 and rmse < 3e-2


def test_max_error_bound_catches_a_single_bad_atom():
    Ft = np.full((64, 3), 0.01)

    def teacher(x):
        return 1.0, Ft

    def student(x):
        F = Ft.copy()
        F[7, 2] += 2.0  # one component off by 2 eV/A: RMSE 0.14, within the absolute
        # and relative bounds set below; only the max-error bound fails
        return 1.0, F

    pot = AuditedPotential(student, teacher, threshold=1.0, every=1, error_fn=_rmse,
                           rel_threshold=100.0, max_threshold=1.0)
    assert pot(0)[2] == "teacher" and pot.fallback
