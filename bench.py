"""Throughput benchmark: DPA-1 energy + forces + virial steps on one MI355X.

Workload: the protein-shaped periodic system (15,668 atoms in a 53.9 A cube,
H/C/N/O/S = 0.64/0.10/0.03/0.22/0.01, jittered lattice at 0.1 atoms/A^3), the
seeded random-init DPA-1 model (type embedding 8, embedding 25/50/100,
axis 16, 2 attention layers of width 128, fitting 240/240/240), rcut 6 A,
sel 120.  100 frames of a cumulative N(0, 0.01 A) random walk are generated
on the host and uploaded before timing; step k evaluates frame k mod 100.
One step = neighbour-list rebuild + forward + input-gradient adjoint + forces
+ virial (dp_compute_device on device-resident inputs).

The JSON line also carries the BF16 mode on the same frames and the
distilled-student leg: a DP-SE-style student is trained on teacher-labelled
noisy frames (a bounded run, sizes in the arguments), then serves held-out
frames with the teacher auditing it; its atom-steps/s is reported next to its
held-out force RMSE and the teacher's force scale.

Prints one JSON line on stdout; a per-kernel table goes to stderr.
"""

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

RCUT = 6.0
SEL = 120
N_FRAMES = 100
FP32_MFMA_PEAK_TFLOPS = 157.3   # MI355X dense FP32 matrix peak
BF16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak
METRIC = "atom-steps/s E+F at 15,668 atoms: FP32 vs BF16 vs student, at force RMSE"


def flop_model(nnei: np.ndarray, shape) -> dict:
    """Algorithmic FLOPs per step of each kernel, at the actual neighbour counts.

    Multiply-adds count 2 FLOPs; forward plus input-gradient adjoint only;
    neither padding nor the recomputation of the logits in the attention
    backward is counted.  Returns {kernel: (flops per step, launches per step)}.
    """
    P = float(nnei.sum())
    n2 = float((nnei.astype(np.float64) ** 2).sum())
    nloc = float(len(nnei))
    M, d, L = shape["M"], shape["dattn"], shape["n_attn"]
    emb = shape["emb"]
    fin0 = M * shape["axis"] + shape["tebd"]
    f = shape["fit"]
    fit = 2.0 * (fin0 * f[0] + sum(f[i] * f[i + 1] for i in range(len(f) - 1)) + f[-1]) * nloc
    emb_gemm = 2.0 * sum(emb[i] * emb[i + 1] for i in range(len(emb) - 1)) * P
    out = {
        "env_embed1": (2.0 * (1 + 2 * shape["tebd"]) * emb[0] * P, 1),
        "emb_fwd": (emb_gemm, 1),
        "qkv_fwd": (L * 2.0 * M * 3 * d * P, L),
        "oproj_ln_fwd": (L * 2.0 * d * M * P, L),
        "desc_fwd": (2.0 * 4 * M * P + 2.0 * 4 * M * shape["axis"] * nloc, 1),
        "fit_fwd": (fit, len(f)),
        "fit_bwd": (fit, len(f)),
        "desc_bwd": (2.0 * 2 * 4 * M * P + 2.0 * 2 * 4 * M * shape["axis"] * nloc, 1),
        "oproj_bwd": (L * 2.0 * d * M * P, L),
        "qkv_bwd": (L * 2.0 * M * 3 * d * P, L),
        "emb_bwd": (emb_gemm, 1),
    }
    # attention core, per neighbour-count class (n in (32c, 32c + 32]):
    # forward QK^T and AV; backward dA, dQ (query tiles) and dK, dV (key tiles)
    nn = nnei.astype(np.float64)
    for c, npad in enumerate((32, 64, 96, 128)):
        sel_c = (nnei > npad - 32) & (nnei <= npad)
        n2c = float((nn[sel_c] ** 2).sum())
        for name in ("attn_fwd", "attn_bwd_q", "attn_bwd_k"):
            out[f"{name}_n{npad}"] = (L * 2.0 * 2 * d * n2c, L)
        # the fused FP32 adjoint (classes up to 96): dA, dQ, dV and dK
        out[f"attn_bwd_n{npad}"] = (L * 2.0 * 4 * d * n2c, L)
        # the FP32 forward with the output projection: Q K^T, A V and o W_O
        Pc = float(nn[sel_c].sum())
        out[f"attn_fwd_ln_n{npad}"] = (L * (2.0 * 2 * d * n2c + 2.0 * d * M * Pc), L)
    # the descriptor adjoint fused with the last layer's projection adjoint
    if L > 0:
        out["desc_oproj_bwd"] = (out["desc_bwd"][0] + out["oproj_bwd"][0] / L, 1)
    return out


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_protein15668_fp32_step.md")


HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E


# kernels that do the work of several entries of flop_model at once (the
# fused attention forward and adjoints, the descriptor adjoint with the last
# projection adjoint); the step's algorithmic total counts that work once,
# through the entries of the separate kernels
FUSED_VARIANTS = ("attn_bwd_n", "attn_fwd_ln_n", "desc_oproj_bwd")


def step_flop_total(flops: dict) -> float:
    """Algorithmic FLOPs of one step: the sum over the separate kernels,
    whichever of them a given build fuses."""
    return sum(fl for k, (fl, _) in flops.items() if not k.startswith(FUSED_VARIANTS))


def byte_model(nnei: np.ndarray, shape, bf16: bool = False) -> dict:
    """Algorithmic HBM bytes per step of the attention and projection kernels.

    The inputs each kernel must read and the outputs it must write, at the
    real widths (M = embedding width, d = attention width), once each; the
    stored logits lam (n per query row) and softmax statistics are part of
    the forward's output and the backward's input, and the probability
    adjoint dA (n per query row) part of the query-tile adjoint's output and
    the key-tile adjoint's input (stored instead of formed a second time).
    Elements are 4 bytes, except that with bf16 the four pair tensors the
    BF16 mode stores in BF16 (QKV, the attention output o, dO and dQKV) take
    2.  Returns {kernel: (bytes per step, launches per step)}.
    """
    P = float(nnei.sum())
    M, d, L = shape["M"], shape["dattn"], shape["n_attn"]
    f4 = 4.0
    t = 2.0 if bf16 else 4.0  # bytes per element of QKV, o, dO, dQKV
    out = {
        "qkv_fwd": (L * P * (f4 * M + t * 3 * d), L),
        # dQKV, the residual gradient and xhat (or the embedding's tanh) and
        # 1/std in; the gradient and the next layer's seed out
        "qkv_bwd": (L * P * (t * 3 * d + f4 * (2 * M + 1 + 2 * M)), L),
        "oproj_ln_fwd": (L * P * (t * d + f4 * (M + 2 * M + 1)), L),
        "oproj_bwd": (L * P * (f4 * M + t * d), L),
    }
    # descriptor adjoint with the last layer's projection adjoint: per pair
    # G, xhat, the geometry record's R~ and 1/std in, the residual gradient,
    # dR~ and dO out; per centre dD and T in
    if L > 0:
        out["desc_oproj_bwd"] = (P * (f4 * (3 * M + 1) + 16.0 + 16.0 + t * d)
                                 + len(nnei) * f4 * (M * shape["axis"] + 4 * M), 1)
    nn = nnei.astype(np.float64)
    for c, npad in enumerate((32, 64, 96, 128)):
        sel_c = (nnei > npad - 32) & (nnei <= npad)
        Pc = float(nn[sel_c].sum())
        n2c = float((nn[sel_c] ** 2).sum())
        # fwd: Q, K, V, gate (rhat, sw) in; o, lam, (m, 1/Z) out
        out[f"attn_fwd_n{npad}"] = (L * (Pc * (t * (3 * d + d) + f4 * (4 + 2)) + f4 * n2c), L)
        # bwd_q: K, V, dO, o, gate, (m, 1/Z), lam in; dQ, (m, 1/Z, D_q), query
        # sums and the probability adjoint dA (n per query row) out
        out[f"attn_bwd_q_n{npad}"] = (L * (Pc * (t * 5 * d + f4 * (4 + 2 + 4 + 4)) + 2 * f4 * n2c), L)
        # bwd_k: Q, dO, gate, stats, query sums, lam and dA in; dK, dV,
        # dE/dsw, dE/drhat out
        out[f"attn_bwd_k_n{npad}"] = (L * (Pc * (t * 4 * d + f4 * (4 + 4 + 4 + 4)) + 2 * f4 * n2c), L)
        # fused adjoint: Q, K, V, dO, gate, (m, 1/Z), lam in; dQ, dK, dV,
        # dE/dsw, dE/drhat out
        out[f"attn_bwd_n{npad}"] = (L * (Pc * (t * (4 * d + 3 * d) + f4 * (4 + 2 + 4)) + f4 * n2c), L)
        # forward with the output projection: QKV, gate, residual row in;
        # logits, statistics, the layer output, xhat and 1/std out (and o
        # for the 128 class, whose adjoint reads it)
        o_out = d if npad > 96 else 0
        out[f"attn_fwd_ln_n{npad}"] = (L * (Pc * (t * (3 * d + o_out) + f4 * (4 + M + 2 + 2 * M + 1))
                                            + f4 * n2c), L)
    return out


def geometry_bytes(nnei: np.ndarray, sel: int, nall: int) -> dict:
    """Algorithmic HBM bytes per step of the neighbour search and the
    geometry kernel (reported against the HBM roof, they do no matrix work).

    nlist: the FP64 coordinates and cell index of every atom read once, the
    list written in full (sel slots per atom, -1 padded) plus the counts;
    env_embed1: per pair the list entry and the neighbour's coordinates and
    type read, the 32-byte geometry record and the 128-byte first-layer row
    written, per centre its own coordinates and type.
    Returns {kernel: (bytes per step, launches per step)}."""
    P = float(nnei.sum())
    nloc = float(len(nnei))
    return {
        "nlist": ((24.0 + 4.0) * nall + 4.0 * sel * nall + 4.0 * nall, 1),
        "env_embed1": (P * (4.0 + 24.0 + 4.0 + 32.0 + 128.0) + nloc * (24.0 + 4.0 + 8.0), 1),
    }


def kernel_sources(kernel: str) -> list:
    """Library sources that define a kernel's code and launch (the attention
    and descriptor kernels: attn.hip and the shared headers; the attention-layer
    projections: gemm.hip and that header; others: every source)."""
    csrc = os.path.join(ROOT, "paper_2604_07276_amd", "csrc")
    if kernel.startswith(("attn_", "desc_")):
        return [os.path.join(csrc, "attn.hip"), os.path.join(csrc, "dpa1_internal.h"),
                os.path.join(csrc, "ln_res.h")]
    if kernel.startswith(("qkv_", "oproj_")):
        return [os.path.join(csrc, "gemm.hip"), os.path.join(csrc, "dpa1_internal.h"),
                os.path.join(csrc, "ln_res.h")]
    return sorted(f for f in glob.glob(os.path.join(csrc, "*"))
                  if f.endswith((".hip", ".cpp", ".h")))


def source_hash(kernel: str = "") -> str:
    """Hash of a kernel's sources; HBM counters are only valid for the code they came from."""
    h = hashlib.sha256()
    for f in kernel_sources(kernel):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary (copy-kernel calibrated), or None if absent or taken on other sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            text = fh.read()
    except OSError:
        return None
    for m in re.finditer(
            r"bench-traffic: kernel=(\S+) source=(\S+) fetch_bytes=(\d+) write_bytes=(\d+)", text):
        if m.group(1) == kernel and m.group(2) == source_hash(kernel):
            return int(m.group(3)), int(m.group(4))
    return None


def cpu_baseline(weights_path, sysm, budget_s: float, gpu_forces: dict) -> tuple:
    """The FP64 CPU oracle on a bounded sample of the same frame.

    The sample starts with every centre that sees the 256 atoms nearest to the
    box centre, which gives exact oracle forces on those atoms; the force
    errors of each GPU precision on them are returned with the timing.  Random
    centres then fill the time budget.
    """
    import torch

    from oracle import dpa1_oracle as orc
    om = orc.load_model(weights_path)
    coords, types, box = sysm.coords, sysm.types, sysm.box
    n = len(coords)
    L = np.diag(box)
    d = coords - L / 2
    d -= L * np.rint(d / L)
    atoms = np.sort(np.argsort((d * d).sum(1))[:256])
    t0 = time.perf_counter()
    nl = orc.neighbor_list(coords, box, RCUT, atoms)
    centers = np.unique(np.concatenate([atoms] + [np.asarray(x, dtype=np.int64) for x in nl]))
    pr = orc.evaluate_centers(om, coords, types, box, RCUT, SEL, centers)
    fo = np.zeros((n, 3))
    np.add.at(fo, pr.pair_i, pr.g)
    np.subtract.at(fo, pr.pair_j, pr.g)
    done = len(centers)
    seen = np.zeros(n, dtype=bool)
    seen[centers] = True
    rest = np.random.default_rng(0).permutation(np.flatnonzero(~seen))
    k = 0
    chunk = 128
    while time.perf_counter() - t0 < budget_s and k < len(rest):
        cs = np.sort(rest[k:k + chunk])
        orc.evaluate_centers(om, coords, types, box, RCUT, SEL, cs)
        k += len(cs)
    done += k
    dt = time.perf_counter() - t0
    acc = {"sample": f"forces on the {len(atoms)} atoms nearest to the box centre, exact from "
                     f"the oracle on the {len(centers)} centres that see them (unperturbed frame)"}
    for tag, F in gpu_forces.items():
        dF = F[atoms] - fo[atoms]
        acc[tag] = {"force_rmse_eV_per_A": float(np.sqrt((dF ** 2).mean())),
                    "force_max_abs_err_eV_per_A": float(np.abs(dF).max())}
    cpu = {"value": done / dt, "unit": "atom-steps/s", "cores": torch.get_num_threads(),
           "host_cpu_count": os.cpu_count(),
           "kind": "oracle",
           "sample": f"{done} centres of the 15,668-atom frame ({len(centers)} around a compact "
                     f"sub-box, then random ones), each with a brute-force neighbour search, FP64 "
                     f"energy and autograd pair gradients ({dt:.1f} s); the rate is centres per "
                     f"second"}
    return cpu, acc


def kernel_fracs(name, cnt, ms, flops, bytes_model, peak_tflops, measured):
    """One kernel's average launch time and its algorithmic TFLOP/s and GB/s
    against the matrix and HBM peaks; with `measured`, its HBM traffic from
    the committed counter record (when taken on the current sources)."""
    avg_s = ms / cnt * 1e-3
    out = {"kernel": name, "avg_launch_ms": round(ms / cnt, 4), "launches": cnt}
    if name in flops:
        per = flops[name][0] / flops[name][1]
        out["flop_per_launch"] = per
        out["achieved_tflops"] = round(per / avg_s / 1e12, 2)
        out["frac_mfma"] = round(per / avg_s / 1e12 / peak_tflops, 4)
    if name in bytes_model:
        per_b = bytes_model[name][0] / bytes_model[name][1]
        out["algorithmic_bytes_per_launch"] = per_b
        out["achieved_gbps"] = round(per_b / avg_s / 1e9, 1)
        out["frac_hbm"] = round(per_b / avg_s / 1e9 / HBM_PEAK_GBPS, 4)
    tr = measured_traffic(name) if measured else None
    if tr is not None:
        out["traffic"] = tr[0] + tr[1]
        out["traffic_gbps"] = round((tr[0] + tr[1]) / avg_s / 1e9, 1)
        out["frac_hbm_measured"] = round((tr[0] + tr[1]) / avg_s / 1e9 / HBM_PEAK_GBPS, 4)
    return out


def roofline_block(ktimes, flops, bytes_model, geo_bytes, step_flops, ms_step, peak_tflops,
                   measured):
    """The `roofline` object: the dominant kernel against the roof it is
    closer to, the leading kernels each with its own fractions, the whole
    step's algorithmic FLOP rate, and the neighbour/geometry kernels against
    the HBM roof.  Dominant kernel rule: the largest time share; when other
    kernels come within 3% of it (run-to-run noise), the one with the lowest
    roofline fraction among them, so that the headline never rests on a coin
    toss between a fast and a slow kernel.  The step is a dense contraction,
    so a kernel that does matrix work is held to the matrix-core roof; its HBM
    rates (the byte model's, which counts the stored activations it reads and
    writes, and the counters') are reported beside it."""
    steps_ms = {k: ms for k, (_, ms) in ktimes.items()}
    ranked = sorted((k for k in ktimes if k in flops), key=lambda k: -steps_ms[k])
    top = [kernel_fracs(k, ktimes[k][0], ktimes[k][1], flops, bytes_model, peak_tflops, measured)
           for k in ranked[:5]]
    for t in top:
        t["share"] = round(steps_ms[t["kernel"]] / sum(steps_ms.values()), 4)
        t["frac"] = t["frac_mfma"]
    lead = [t for t in top if steps_ms[t["kernel"]] >= 0.97 * steps_ms[top[0]["kernel"]]]
    dom = min(lead, key=lambda t: t["frac"])
    use_hbm = False
    hbm_frac = dom.get("frac_hbm_measured", dom.get("frac_hbm"))
    hbm_gbps = dom.get("traffic_gbps", dom.get("achieved_gbps"))
    out = {"bound": "hbm" if use_hbm else "mfma", "kernel": dom["kernel"],
           "achieved": hbm_gbps if use_hbm else dom["achieved_tflops"],
           "peak": HBM_PEAK_GBPS if use_hbm else peak_tflops,
           "unit": "GB/s" if use_hbm else "TFLOP/s",
           "frac": hbm_frac if use_hbm else dom["frac_mfma"],
           "frac_mfma": dom.get("frac_mfma"),
           "frac_hbm": dom.get("frac_hbm"),
           "frac_hbm_measured": dom.get("frac_hbm_measured"),
           "algorithmic_bytes_per_launch": dom.get("algorithmic_bytes_per_launch"),
           "traffic": dom.get("traffic"),
           "traffic_source": (os.path.relpath(TRAFFIC_FILE, ROOT)
                              if dom.get("traffic") is not None else None),
           "avg_launch_ms": dom["avg_launch_ms"],
           "flop_per_launch": dom.get("flop_per_launch"),
           "rule": "largest time share; within 3% of it, the lowest fraction",
           "step_algorithmic_tflop": round(step_flops / 1e12, 4),
           "step_frac": round(step_flops / (ms_step * 1e-3) / 1e12 / peak_tflops, 4),
           "top_kernels": top}
    geo = []
    for name in ("nlist", "env_embed1"):
        if name in ktimes and name in geo_bytes:
            geo.append(kernel_fracs(name, ktimes[name][0], ktimes[name][1], {}, geo_bytes,
                                    peak_tflops, False))
    out["geometry_kernels_hbm"] = geo
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--host-api-steps", type=int, default=10,
                    help="steps of the host-memory entry point to time (0: skip)")
    ap.add_argument("--student-steps", type=int, default=200,
                    help="training steps of the distilled student leg (0: skip the leg)")
    ap.add_argument("--student-frames", type=int, default=256,
                    help="teacher-labelled training frames of the student leg")
    ap.add_argument("--student-eval", type=int, default=32,
                    help="held-out frames served by the audited student")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run one device-to-device copy of this many MiB (calibrates "
                         "hardware byte counters against a known transfer) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the DPA-1 step of one domain is measured on "
              "one MI355X; multi-GPU runs are not part of this benchmark.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2604_07276_amd import binding, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.copy_probe_mib:
        nb = args.copy_probe_mib * (1 << 20)
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nb}), flush=True)
        return
    tmpdir = tempfile.mkdtemp()
    wpath = os.path.join(tmpdir, "dpa1_seed0.bin")
    shp = synth.make_weights(wpath, seed=0)
    model = binding.Model(wpath, RCUT, SEL)

    sysm = synth.protein_system(0)
    n = len(sysm.coords)
    frames = synth.perturbed_frames(sysm, N_FRAMES, 0.01)
    d_frames = torch.tensor(frames, device=dev)
    d_types = torch.tensor(sysm.types, device=dev)
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    f = torch.zeros((n, 3), dtype=torch.float64, device=dev)
    v = torch.zeros(9, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    box = sysm.box

    def step(k):
        model.compute_device(d_frames[k % N_FRAMES], d_types, box, n, 0, e, f, v, None, stream)

    for k in range(args.warmup):
        step(k)
    model.sync()
    torch.cuda.synchronize()
    # one event per step boundary on the step's stream: total and per-step times
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    evs[0].record(stream)
    for k in range(args.steps):
        step(k)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    model.sync()
    ms_total = evs[0].elapsed_time(evs[-1])
    ms_step = ms_total / args.steps
    per_step = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
    value = n * args.steps / (ms_total / 1e3)
    E_last = float(e.cpu()[0])
    F_last = f.cpu().numpy()
    assert np.isfinite(E_last) and np.all(np.isfinite(F_last))

    # neighbour statistics of frame 0 for the FLOP model
    step(0)
    model.sync()
    _, nnei = model.debug_nlist(n)
    shape = {"M": shp.emb[-1], "dattn": shp.attn_dim, "emb": shp.emb, "axis": shp.axis,
             "tebd": shp.tebd_dim, "fit": shp.fit, "n_attn": shp.n_attn}
    flops = flop_model(nnei, shape)
    step_flops = step_flop_total(flops)

    roofline = None
    if not args.no_kernel_timing:
        # second pass over the same frames with a HIP event pair around every launch
        model.set_timing(True)
        for k in range(args.steps):
            step(k)
        model.sync()
        ktimes = model.kernel_times()
        model.set_timing(False)
        tot = sum(ms for _, ms in ktimes.values())
        print(f"{'kernel':<16}{'launches':>9}{'avg ms':>10}{'share':>8}{'TFLOP/s':>9}",
              file=sys.stderr)
        for name, (cnt, ms) in sorted(ktimes.items(), key=lambda kv: -kv[1][1]):
            tf = ""
            if name in flops:  # per-launch work times the launches made
                per = flops[name][0] / flops[name][1]
                tf = f"{per * cnt / (ms * 1e-3) / 1e12:9.1f}"
            print(f"{name:<16}{cnt:>9}{ms / cnt:>10.4f}{ms / tot:>8.1%}{tf:>9}", file=sys.stderr)
        print(f"step: {ms_step:.3f} ms, {step_flops / 1e12:.4f} TFLOP algorithmic, "
              f"sum of kernel times {tot / args.steps:.3f} ms", file=sys.stderr)
        roofline = roofline_block(ktimes, flops, byte_model(nnei, shape),
                                  geometry_bytes(nnei, SEL, n), step_flops, ms_step,
                                  FP32_MFMA_PEAK_TFLOPS, measured=True)

    # BF16 precision mode on the same frames (FP32 stays the headline `value`)
    model.set_precision(binding.PREC_BF16)
    for k in range(args.warmup):
        step(k)
    model.sync()
    torch.cuda.synchronize()
    b0 = torch.cuda.Event(enable_timing=True)
    b1 = torch.cuda.Event(enable_timing=True)
    b0.record(stream)
    for k in range(args.steps):
        step(k)
    b1.record(stream)
    torch.cuda.synchronize()
    model.sync()
    bf16_ms = b0.elapsed_time(b1) / args.steps
    bf16_roof = None
    if not args.no_kernel_timing:
        model.set_timing(True)
        for k in range(args.steps):
            step(k)
        model.sync()
        kt16 = model.kernel_times()
        model.set_timing(False)
        bf16_roof = roofline_block(kt16, flops, byte_model(nnei, shape, bf16=True), {},
                                   step_flops, bf16_ms, BF16_MFMA_PEAK_TFLOPS, measured=False)
        del bf16_roof["geometry_kernels_hbm"]
    model.set_precision(binding.PREC_FP32)

    # distilled student: teacher labels, training, audited serving of held-out frames
    student_out = None
    if args.student_steps > 0:
        from paper_2604_07276_amd import student as student_mod
        st = student_mod.run(n_train=args.student_frames, n_eval=args.student_eval,
                             steps=args.student_steps)
        thr = st["throughput"]
        student_out = {
            "value": thr["student_atom_steps_per_s"], "unit": "atom-steps/s",
            "ms_per_step": thr["student_ms_per_step"],
            "dtype": "bf16 matrix-core operands, f32 accumulate, f64 reductions",
            "vs_fp32": round(ms_step / thr["student_ms_per_step"], 3),
            "model": st["student"],
            "force_rmse_eV_per_A": st["held_out"]["force_rmse_eV_per_A"],
            "force_max_abs_err_eV_per_A": st["held_out"]["force_max_abs_err_eV_per_A"],
            "teacher_force_rms_eV_per_A": st["held_out"]["teacher_force_rms_eV_per_A"],
            "relative_force_rmse": st["held_out"]["relative_force_rmse"],
            "energy_mae_eV_per_atom": st["held_out"]["energy_mae_eV_per_atom"],
            "training": st["training"], "serving": st["serving"]}

    # host-memory entry point (PCIe copies included): context only, never `value`
    host_ms = None
    if args.host_api_steps > 0:
        coords0 = frames[0]
        model.compute(coords0, sysm.types, box, n, 0)
        t0 = time.perf_counter()
        for k in range(args.host_api_steps):
            model.compute(frames[k % N_FRAMES], sysm.types, box, n, 0)
        host_ms = (time.perf_counter() - t0) * 1e3 / args.host_api_steps

    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        gpu_forces = {}
        for tag, prec in (("fp32", binding.PREC_FP32), ("bf16", binding.PREC_BF16)):
            model.set_precision(prec)
            gpu_forces[tag] = model.compute(sysm.coords, sysm.types, box, n, 0)[1]
        model.set_precision(binding.PREC_FP32)
        cpu, accuracy = cpu_baseline(wpath, sysm, args.cpu_seconds, gpu_forces)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_p10_p50_p90": [round(float(np.percentile(per_step, q)), 4)
                                    for q in (10, 50, 90)],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "protein-shaped periodic box, 15,668 atoms, 53.9 A cube, "
                               "FP32 DPA-1 E+F+virial",
                   "atoms": n, "rcut": RCUT, "sel": SEL, "mean_neighbours":
                       round(float(nnei.mean()), 2), "frames": N_FRAMES,
                   "model": "DPA-1 random-init seed 0: tebd 8, emb 25/50/100, axis 16, "
                            "2 attention layers x 128, fitting 240x3",
                   "precision": "fp32"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "host_api_ms_per_step": None if host_ms is None else round(host_ms, 3),
        "bf16": {"value": round(n * args.steps / (bf16_ms * args.steps / 1e3), 1),
                 "unit": "atom-steps/s", "ms_per_step": round(bf16_ms, 4),
                 "dtype": "bf16 matrix-core operands, f32 accumulate, f64 reductions",
                 "vs_fp32": round(ms_step / bf16_ms, 3),
                 "roofline": bf16_roof},
        "accuracy_vs_oracle": accuracy,
        "student": student_out,
    }
    print(json.dumps(out), flush=True)
    model.close()


if __name__ == "__main__":
    main()
