"""Pins of the student-training oracle (loss, exact gradient, Adam).

The loss gradient is pinned by central finite differences of the loss itself,
by the zero of the loss at self-generated labels, and by the closed form of
the force term under a known label shift; Adam by closed forms of its first
two steps and of a constant-gradient run (Kingma and Ba 2015, Algorithm 1).
"""

import numpy as np
import pytest
import torch

from oracle import dpa1_oracle as orc
from oracle import train_oracle as tro
from paper_2604_07276_amd import synth

RC = 4.0
SEL = 40
PE, PF = 0.5, 2.0


@pytest.fixture(scope="module")
def student(tmp_path_factory):
    p = tmp_path_factory.mktemp("student") / "student.bin"
    synth.make_weights(str(p), seed=1, shape=synth.STUDENT_SHAPE)
    return orc.load_model(str(p))


@pytest.fixture(scope="module")
def batch():
    base = synth.open_cluster(20, 3.2, 5, seed=2)
    frames = np.stack([synth.noisy_frame(base, k, 0.05) for k in range(2)])
    rng = np.random.default_rng(11)
    e_lab = rng.normal(0.0, 1.0, size=2)
    f_lab = rng.normal(0.0, 0.1, size=frames.shape)
    return base, frames, e_lab, f_lab


def test_student_parameter_count(student):
    assert tro.param_count(student) == 86318
    assert student.n_attn == 0 and student.emb == (16, 32, 64) and student.axis == 8


def test_loss_gradient_matches_finite_differences(student, batch):
    base, frames, e_lab, f_lab = batch
    _, grads = tro.loss_and_grad(student, frames, base.types, None, e_lab, f_lab, RC, SEL, PE, PF)
    rng = np.random.default_rng(5)
    h = 1e-5
    checked = 0
    for name in tro.param_names(student):
        t = student.t[name]
        flat = t.view(-1)
        for idx in rng.choice(flat.numel(), size=min(2, flat.numel()), replace=False):
            old = float(flat[idx])
            vals = []
            for sgn in (1.0, -1.0):
                flat[idx] = old + sgn * h
                vals.append(tro.loss_value(student, frames, base.types, None, e_lab, f_lab, RC,
                                           SEL, PE, PF))
            flat[idx] = old
            fd = (vals[0] - vals[1]) / (2 * h)
            g = grads[name].reshape(-1)[idx]
            assert abs(fd - g) <= 1e-7 + 1e-5 * abs(g), (name, int(idx), fd, g)
            checked += 1
    assert checked >= 2 * len(tro.param_names(student)) - 2


def test_self_labels_give_zero_loss_and_gradient(student, batch):
    base, frames, _, _ = batch
    e_own, f_own = tro.labels(student, frames, base.types, None, RC, SEL)
    (L, le, lf), grads = tro.loss_and_grad(student, frames, base.types, None, e_own, f_own, RC,
                                           SEL, PE, PF)
    assert L < 1e-28
    for name, g in grads.items():
        assert np.max(np.abs(g)) < 1e-12, name


def test_force_term_closed_form_under_label_shift(student, batch):
    base, frames, _, _ = batch
    e_own, f_own = tro.labels(student, frames, base.types, None, RC, SEL)
    rng = np.random.default_rng(9)
    delta = rng.normal(0.0, 0.2, size=f_own.shape)
    de = np.array([0.3, -0.7])
    B, N = frames.shape[0], frames.shape[1]
    _, le, lf = tro.batch_loss(student, frames, base.types, None, e_own + de, f_own + delta, RC,
                               SEL, PE, PF)
    assert float(lf) == pytest.approx(PF / (3 * N * B) * np.sum(delta ** 2), rel=1e-12)
    assert float(le) == pytest.approx(PE / B * np.sum((de / N) ** 2), rel=1e-12)


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(0)
    g = rng.normal(size=100)
    g[np.abs(g) < 1e-3] = 1e-3
    th0 = rng.normal(size=100)
    st = tro.adam_init(100)
    th1 = tro.adam_step(th0, g, st, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8)
    np.testing.assert_allclose(th1 - th0, -1e-3 * np.sign(g), rtol=1e-4)


def test_adam_second_step_closed_form():
    b1, b2, lr, eps = 0.9, 0.999, 2e-3, 1e-8
    g1 = np.array([0.5, -2.0, 1e-2])
    g2 = np.array([-0.25, -1.0, 3e-2])
    st = tro.adam_init(3)
    th = tro.adam_step(np.zeros(3), g1, st, lr, b1, b2, eps)
    th2 = tro.adam_step(th, g2, st, lr, b1, b2, eps)
    # bias-corrected moments after two steps, written out by hand
    mhat = (b1 * g1 + g2) / (1 + b1)
    vhat = (b2 * g1 ** 2 + g2 ** 2) / (1 + b2)
    np.testing.assert_allclose(th2 - th, -lr * mhat / (np.sqrt(vhat) + eps), rtol=1e-12)


def test_adam_constant_gradient_steps_are_equal():
    g = np.array([3.0, -0.01, 1e-4])
    st = tro.adam_init(3)
    th = np.zeros(3)
    for t in range(1, 8):
        new = tro.adam_step(th, g, st, 1e-2, 0.9, 0.999, 1e-8)
        np.testing.assert_allclose(new - th, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)
        th = new
