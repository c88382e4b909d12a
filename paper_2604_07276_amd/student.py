"""Distilled student: teacher labels, training, audited serving.

A small DP-SE-style student (the Sec. II-B descriptor without attention:
embedding 16/32/64, axis 8, fitting 128 x 2; 86,318 parameters with 5 types)
is trained on energies and forces that the FP32 DPA-1 teacher computes on
noisy copies of the 15,668-atom protein-shaped frame, then serves held-out
frames with the teacher as its periodic judge and fallback:

1. frames: base positions plus independent N(0, 0.05^2) noise per component;
   the first ``n_train`` train, the next ``n_eval`` are held out;
2. labels: E and F of the teacher (library inference, FP32) on every frame;
3. training: the library's trainer (exact energy+force loss gradient, Adam on
   FP32 masters, BF16 matrix-core operands by default), batches of 8 frames;
4. serving: the student evaluates each held-out frame as one MD step; every
   ``audit_every``-th step the teacher evaluates it too and the student's
   force error is checked against three bounds: the RMSE against an absolute
   threshold (3e-2 eV/A), the RMSE relative to the teacher's own force RMS on
   that frame (0.5: the student must explain at least 3/4 of the force
   variance; an absolute bound alone passes a student that returns F = 0 when
   the teacher's forces are small) and the largest component error (1 eV/A).
   Past any of them the teacher takes over for every later step.

Run: ``python -m paper_2604_07276_amd.student [--steps K] ...``; prints one
JSON object.  Needs the built library and a GPU.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import tempfile
import time

import numpy as np

from . import binding, synth

RCUT = 6.0
SEL = 120
BATCH = 8


class AuditedPotential:
    """Serves steps with the student and lets the teacher audit every k-th step.

    ``student`` and ``teacher`` are callables coords -> (E, F) on device
    tensors (or host arrays); ``error_fn(F_a, F_b) -> (rmse, max)``.  An audit
    fails when the force RMSE exceeds ``threshold`` (eV/A), or exceeds
    ``rel_threshold`` times the teacher's force RMS on the audited step, or
    when the largest component error exceeds ``max_threshold`` (eV/A); once
    one fails, every later step is served by the teacher.
    """

    def __init__(self, student, teacher, threshold: float, every: int = 10, error_fn=None,
                 rel_threshold: float = float("inf"), max_threshold: float = float("inf")):
        if every < 1:
            raise ValueError("audit interval must be >= 1")
        self.student, self.teacher = student, teacher
        self.threshold = float(threshold)
        self.rel_threshold = float(rel_threshold)
        self.max_threshold = float(max_threshold)
        self.every = int(every)
        self.error_fn = error_fn or binding.force_error
        self.step_count = 0
        self.fallback = False
        self.audits = []  # (step, rmse, max, teacher force rms)

    def __call__(self, coords):
        k = self.step_count
        self.step_count += 1
        if self.fallback:
            return self.teacher(coords) + ("teacher",)
        E, F = self.student(coords)
        if k % self.every == 0:
            Et, Ft = self.teacher(coords)
            rmse, mx = self.error_fn(F, Ft)
            scale = self.error_fn(Ft, 0 * Ft)[0]
            self.audits.append((k, rmse, mx, scale))
            ok = rmse <= self.threshold and rmse <= self.rel_threshold * scale and \
                mx <= self.max_threshold
            if not ok:
                self.fallback = True
                return Et, Ft, "teacher"
        return E, F, "student"


def _evaluator(model, types, box, n, torch):
    """coords -> (E [1], F [n, 3]) device tensors through dp_compute_device."""
    dev = torch.device("cuda:0")
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    v = torch.zeros(9, dtype=torch.float64, device=dev)

    def run(coords):
        f = torch.empty((n, 3), dtype=torch.float64, device=dev)
        model.compute_device(coords, types, box, n, 0, e, f, v)
        return e.clone(), f
    return run


def label_frames(teacher, frames, types, box, torch):
    """Teacher energies [F] and forces [F, N, 3] (device) for device frames [F, N, 3]."""
    nf, n = int(frames.shape[0]), int(frames.shape[1])
    dev = frames.device
    E = torch.zeros(nf, dtype=torch.float64, device=dev)
    F = torch.zeros((nf, n, 3), dtype=torch.float64, device=dev)
    v = torch.zeros(9, dtype=torch.float64, device=dev)
    for k in range(nf):
        teacher.compute_device(frames[k], types, box, n, 0, E[k:k + 1], F[k], v)
    teacher.sync()
    return E, F


def time_steps(model, frames, types, box, reps: int, torch):
    """Median device time (ms) of one E+F step over ``reps`` frames."""
    n = int(frames.shape[1])
    run = _evaluator(model, types, box, n, torch)
    for k in range(3):
        run(frames[k % frames.shape[0]])
    model.sync()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for k in range(reps):
        run(frames[k % frames.shape[0]])
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    model.sync()
    return float(np.median([ev[k].elapsed_time(ev[k + 1]) for k in range(reps)]))


def run(n_train=2000, n_eval=200, steps=2000, lr0=1e-3, lr1=1e-5, pref_e=1.0, pref_f=100.0,
        precision="bf16", threshold=3e-2, audit_every=10, seed=0, out_weights=None, log=None,
        target="dpa1", rel_threshold=0.5, max_threshold=1.0):
    """The pipeline above.  ``target`` "dpa1" labels with the DPA-1 teacher;
    "dpa1_noattn" with the same teacher widths without the attention layers
    (the DP-SE descriptor the student shares); "student" with the student
    architecture under other weights (a target the student can represent
    exactly: a check of the training)."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the student pipeline needs a GPU")
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    tmp = tempfile.mkdtemp()
    t_path = os.path.join(tmp, "teacher_seed0.bin")
    s_path = os.path.join(tmp, "student_seed1.bin")
    if target == "dpa1":
        synth.make_weights(t_path, seed=0)
    elif target == "dpa1_noattn":
        synth.make_weights(t_path, seed=0, shape=synth.ModelShape(n_attn=0))
    elif target == "student":
        synth.make_weights(t_path, seed=7, shape=synth.STUDENT_SHAPE)
    else:
        raise ValueError(f"unknown target {target!r}")
    synth.make_weights(s_path, seed=1, shape=synth.STUDENT_SHAPE)
    base = synth.protein_system(seed)
    n = len(base.coords)
    types = torch.tensor(base.types, device=dev)
    box = base.box

    def say(msg):
        if log:
            print(msg, file=log, flush=True)

    # frames and teacher labels
    t0 = time.time()
    nf = n_train + n_eval
    frames = torch.empty((nf, n, 3), dtype=torch.float64, device=dev)
    for k in range(nf):
        frames[k] = torch.from_numpy(synth.noisy_frame(base, k, 0.05)).to(dev)
    teacher = binding.Model(t_path, RCUT, SEL)
    E_lab, F_lab = label_frames(teacher, frames, types, box, torch)
    torch.cuda.synchronize()
    t_label = time.time() - t0
    f_rms = float(torch.sqrt((F_lab[:n_train] ** 2).mean()))
    say(f"labelled {nf} frames in {t_label:.1f} s; teacher |F| rms {f_rms:.4g} eV/A")

    # training
    prec = binding.PREC_BF16 if precision == "bf16" else binding.PREC_FP32
    tr = binding.Trainer(s_path, RCUT, SEL, pref_e=pref_e, pref_f=pref_f, precision=prec)
    rng = np.random.default_rng(seed + 100)
    order = rng.permutation(n_train)
    pos = 0
    hist = []
    t0 = time.time()
    for step in range(steps):
        if pos + BATCH > n_train:
            order = rng.permutation(n_train)
            pos = 0
        idx = torch.from_numpy(np.sort(order[pos:pos + BATCH])).to(dev)
        pos += BATCH
        lr = lr0 * (lr1 / lr0) ** (step / max(steps - 1, 1))
        loss = tr.step(frames.index_select(0, idx), types, box, E_lab.index_select(0, idx),
                       F_lab.index_select(0, idx), lr)
        hist.append(loss.tolist())
        if step % 100 == 0 or step == steps - 1:
            rmse_est = math.sqrt(loss[2] / pref_f) if pref_f > 0 else float("nan")
            say(f"step {step} lr {lr:.3g} loss {loss[0]:.4g} (e {loss[1]:.3g}, f {loss[2]:.3g}; "
                f"force rmse ~{rmse_est:.4g})")
    torch.cuda.synchronize()
    t_train = time.time() - t0
    s_trained = out_weights or os.path.join(tmp, "student_trained.bin")
    tr.save(s_trained)
    tr.close()

    # held-out evaluation and audited serving
    student = binding.Model(s_trained, RCUT, SEL)
    if prec == binding.PREC_BF16:
        student.set_precision(binding.PREC_BF16)
    st_eval = _evaluator(student, types, box, n, torch)
    te_eval = _evaluator(teacher, types, box, n, torch)
    ev = frames[n_train:]
    rm, mx, de = [], [], []
    # the error split by the teacher's force size: the bulk of the atoms and
    # the 1% with the largest teacher forces
    f_mag = torch.linalg.norm(F_lab[:n_train], dim=2)
    cut = float(torch.quantile(f_mag[: min(n_train, 50)].flatten().float(), 0.99))
    bulk_sq = tail_sq = bulk_ref = tail_ref = 0.0
    for k in range(n_eval):
        E, F = st_eval(ev[k])
        Ft = F_lab[n_train + k]
        r, m = binding.force_error(F, Ft)
        rm.append(r)
        mx.append(m)
        de.append(abs(float(E[0]) - float(E_lab[n_train + k])) / n)
        big = torch.linalg.norm(Ft, dim=1) > cut
        d2 = ((F - Ft) ** 2).sum(1)
        t2 = (Ft ** 2).sum(1)
        tail_sq += float(d2[big].sum())
        tail_ref += float(t2[big].sum())
        bulk_sq += float(d2[~big].sum())
        bulk_ref += float(t2[~big].sum())
    # training-set error on up to 50 training frames (under- versus over-fitting)
    tr_sq = tr_ref = 0.0
    for k in range(min(n_train, 50)):
        E, F = st_eval(frames[k])
        tr_sq += float(((F - F_lab[k]) ** 2).sum())
        tr_ref += float((F_lab[k] ** 2).sum())
    pot = AuditedPotential(lambda x: st_eval(x), lambda x: te_eval(x), threshold, audit_every,
                           rel_threshold=rel_threshold, max_threshold=max_threshold)
    sources = [pot(ev[k])[2] for k in range(n_eval)]
    ms_student = time_steps(student, ev, types, box, 50, torch)
    ms_teacher = time_steps(teacher, ev, types, box, 20, torch)
    student.close()
    teacher.close()
    rmse = float(np.sqrt(np.mean(np.square(rm))))
    return {
        "student": "DP-SE-style: embedding 16/32/64, axis 8, no attention, fitting 128x2, "
                   "86,318 parameters",
        "training": {"frames": n_train, "held_out": n_eval, "batch": BATCH, "steps": steps,
                     "lr": [lr0, lr1], "pref_e": pref_e, "pref_f": pref_f,
                     "precision": precision, "label_s": round(t_label, 2),
                     "train_s": round(t_train, 2),
                     "ms_per_train_step": round(1e3 * t_train / max(steps, 1), 2),
                     "loss_first": hist[0] if hist else None,
                     "loss_last": hist[-1] if hist else None},
        "held_out": {"force_rmse_eV_per_A": rmse, "force_max_abs_err_eV_per_A": float(max(mx)),
                     "teacher_force_rms_eV_per_A": f_rms,
                     "relative_force_rmse": rmse / f_rms,
                     "relative_force_rmse_bulk": math.sqrt(bulk_sq / max(bulk_ref, 1e-300)),
                     "relative_force_rmse_top1pct": math.sqrt(tail_sq / max(tail_ref, 1e-300)),
                     "top1pct_share_of_teacher_force_sq": tail_ref / max(tail_ref + bulk_ref,
                                                                         1e-300),
                     "energy_mae_eV_per_atom": float(np.mean(de))},
        "train_set": {"frames": min(n_train, 50),
                      "relative_force_rmse": math.sqrt(tr_sq / max(tr_ref, 1e-300))},
        "serving": {"audit_every": audit_every, "threshold_eV_per_A": threshold,
                    "rel_threshold": rel_threshold, "max_threshold_eV_per_A": max_threshold,
                    "audits": [[k, round(r, 6), round(m, 6), round(sc, 6)]
                               for k, r, m, sc in pot.audits],
                    "fallback": pot.fallback,
                    "student_steps": sources.count("student"),
                    "teacher_steps": sources.count("teacher")},
        "throughput": {"atoms": n, "student_ms_per_step": round(ms_student, 4),
                       "teacher_ms_per_step": round(ms_teacher, 4),
                       "student_atom_steps_per_s": round(n / ms_student * 1e3, 1),
                       "teacher_atom_steps_per_s": round(n / ms_teacher * 1e3, 1),
                       "speedup_vs_teacher": round(ms_teacher / ms_student, 3),
                       "student_precision": precision},
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-frames", type=int, default=2000)
    ap.add_argument("--eval-frames", type=int, default=200)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--lr0", type=float, default=1e-3)
    ap.add_argument("--lr1", type=float, default=1e-5)
    ap.add_argument("--pref-e", type=float, default=1.0)
    ap.add_argument("--pref-f", type=float, default=100.0)
    ap.add_argument("--precision", choices=("fp32", "bf16"), default="bf16")
    ap.add_argument("--threshold", type=float, default=3e-2)
    ap.add_argument("--rel-threshold", type=float, default=0.5)
    ap.add_argument("--max-threshold", type=float, default=1.0)
    ap.add_argument("--save", default=None, help="write the trained student weights here")
    ap.add_argument("--target", choices=("dpa1", "dpa1_noattn", "student"), default="dpa1",
                    help="label with the DPA-1 teacher, with its widths without attention, or "
                         "with the student architecture under other weights (a representable "
                         "target)")
    args = ap.parse_args(argv)
    out = run(args.train_frames, args.eval_frames, args.steps, args.lr0, args.lr1, args.pref_e,
              args.pref_f, args.precision, args.threshold, out_weights=args.save, log=sys.stderr,
              target=args.target, rel_threshold=args.rel_threshold,
              max_threshold=args.max_threshold)
    out["target"] = args.target
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
