"""Python binding of the DPA-1 C ABI (include/dpa1.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Torch tensors are accepted as device buffers (their data pointers
are passed through) and torch's current HIP stream is used for the
device-memory entry point.  There is no fallback: if the library is not
built or cannot be loaded, every call raises.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdpa1.so")

DP_OK = 0
STATUS_NAMES = {
    -1: "DP_ERR_ARG", -2: "DP_ERR_TYPE", -3: "DP_ERR_BOX", -4: "DP_ERR_SEL_OVERFLOW",
    -5: "DP_ERR_WEIGHTS", -6: "DP_ERR_DEVICE", -7: "DP_ERR_OOM",
}
EXPORTED = ("dp_create", "dp_compute", "dp_compute_device", "dp_forward_device",
            "dp_backward_device", "dp_set_precision", "dp_set_memory_budget", "dp_memory_info",
            "dp_sync", "dp_debug_nlist", "dp_set_timing", "dp_kernel_times", "dp_model_info",
            "dp_destroy", "dp_last_error",
            # student trainer (include/dpa1_train.h)
            "dp_train_create", "dp_train_gradient", "dp_train_step", "dp_train_params",
            "dp_train_save", "dp_train_checkpoint", "dp_train_resume", "dp_train_destroy",
            "dp_force_error", "dp_force_error_noalloc")
PREC_FP32 = 0
PREC_BF16 = 1

_lib = None


class TrainOptions(ctypes.Structure):
    """dp_train_options of include/dpa1_train.h."""
    _fields_ = [("pref_e", ctypes.c_double), ("pref_f", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("precision", ctypes.c_int)]


class DPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libdpa1.so (built in-tree) and declare the signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2604_07276_amd.build.build()")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I = ctypes.c_int
    D = ctypes.c_double
    lib.dp_create.argtypes = [ctypes.c_char_p, D, I, ctypes.POINTER(P)]
    lib.dp_compute.argtypes = [P, P, P, P, I, I, P, P, P, P]
    lib.dp_compute_device.argtypes = [P, P, P, P, I, I, P, P, P, P, P]
    lib.dp_forward_device.argtypes = [P, P, P, P, I, I, P, P, P]
    lib.dp_backward_device.argtypes = [P, P, P, P, P]
    lib.dp_set_precision.argtypes = [P, I]
    lib.dp_set_memory_budget.argtypes = [P, D]
    lib.dp_memory_info.argtypes = [P, P, P]
    lib.dp_sync.argtypes = [P]
    lib.dp_debug_nlist.argtypes = [P, P, P]
    lib.dp_set_timing.argtypes = [P, I]
    lib.dp_kernel_times.argtypes = [P, P, P, P, I]
    lib.dp_model_info.argtypes = [P, P, P]
    lib.dp_destroy.argtypes = [P]
    lib.dp_destroy.restype = None
    lib.dp_last_error.argtypes = []
    lib.dp_last_error.restype = ctypes.c_char_p
    lib.dp_train_create.argtypes = [ctypes.c_char_p, D, I, ctypes.POINTER(TrainOptions),
                                    ctypes.POINTER(P)]
    lib.dp_train_gradient.argtypes = [P, P, P, P, I, I, P, P, P, P, P]
    lib.dp_train_step.argtypes = [P, P, P, P, I, I, P, P, D, P, P]
    lib.dp_train_params.argtypes = [P, P, P]
    lib.dp_train_save.argtypes = [P, ctypes.c_char_p]
    lib.dp_train_checkpoint.argtypes = [P, ctypes.c_char_p]
    lib.dp_train_resume.argtypes = [P, ctypes.c_char_p]
    lib.dp_train_destroy.argtypes = [P]
    lib.dp_train_destroy.restype = None
    lib.dp_force_error.argtypes = [P, P, I, P, P]
    lib.dp_force_error_noalloc.argtypes = [P, P, I, P, P]
    for name in ("dp_create", "dp_compute", "dp_compute_device", "dp_forward_device",
                 "dp_backward_device", "dp_set_precision", "dp_set_memory_budget",
                 "dp_memory_info", "dp_sync", "dp_debug_nlist",
                 "dp_set_timing", "dp_kernel_times", "dp_model_info", "dp_train_create",
                 "dp_train_gradient", "dp_train_step", "dp_train_params", "dp_train_save",
                 "dp_train_checkpoint", "dp_train_resume", "dp_force_error",
                 "dp_force_error_noalloc"):
        getattr(lib, name).restype = I
    _lib = lib
    return lib


def _check(rc: int) -> int:
    if rc < 0:
        raise DPError(rc, _lib.dp_last_error().decode())
    return rc


def _ptr(a) -> int | None:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


class Model:
    """A loaded DPA-1 model on the current HIP device (dp_create / dp_destroy)."""

    def __init__(self, weights_path: str, rcut: float, sel: int):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.dp_create(weights_path.encode(), float(rcut), int(sel), ctypes.byref(h)))
        self._h = h
        self.rcut = float(rcut)
        self.sel = int(sel)

    def close(self):
        if getattr(self, "_h", None):
            _lib.dp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        ints = np.zeros(8, dtype=np.int32)
        dbls = np.zeros(3)
        _check(_lib.dp_model_info(self._h, ints.ctypes.data, dbls.ctypes.data))
        return ints, dbls

    def compute(self, coords, types, box, nloc: int, nghost: int, atom_energy: bool = False):
        """Host-memory step (dp_compute).  Returns (E, F [N,3], virial [3,3], e_i or None)."""
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        types = np.ascontiguousarray(types, dtype=np.int32)
        boxa = None if box is None else np.ascontiguousarray(box, dtype=np.float64).reshape(9)
        nall = nloc + nghost
        E = np.zeros(1)
        F = np.zeros((nall, 3))
        V = np.zeros(9)
        AE = np.zeros(max(nloc, 1)) if atom_energy else None
        _check(_lib.dp_compute(self._h, _ptr(coords) if nall else None,
                               _ptr(types) if nall else None, _ptr(boxa), nloc, nghost,
                               E.ctypes.data, F.ctypes.data if nall else None, V.ctypes.data,
                               _ptr(AE)))
        return float(E[0]), F, V.reshape(3, 3), (AE[:nloc] if atom_energy else None)

    def compute_device(self, coords, types, box, nloc: int, nghost: int, energy, forces, virial,
                       atom_energy=None, stream=None):
        """Device-memory step (dp_compute_device), asynchronous on ``stream``.

        coords (float64 [N,3]), types (int32 [N]), energy (float64 [1]), forces
        (float64 [N,3]), virial (float64 [9]) and atom_energy (float64 [nloc] or
        None) are torch CUDA tensors; box is host data or None.
        """
        import torch
        boxa = None if box is None else np.ascontiguousarray(box, dtype=np.float64).reshape(9)
        if stream is None:
            stream = torch.cuda.current_stream()
        sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        _check(_lib.dp_compute_device(self._h, _ptr(coords), _ptr(types), _ptr(boxa), nloc,
                                      nghost, _ptr(energy), _ptr(forces), _ptr(virial),
                                      _ptr(atom_energy), sp))

    def forward_device(self, coords, types, box, nloc: int, nghost: int, energy,
                       atom_energy=None, stream=None):
        """Forward half (dp_forward_device): energies only, activations kept."""
        import torch
        boxa = None if box is None else np.ascontiguousarray(box, dtype=np.float64).reshape(9)
        if stream is None:
            stream = torch.cuda.current_stream()
        sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        _check(_lib.dp_forward_device(self._h, _ptr(coords), _ptr(types), _ptr(boxa), nloc,
                                      nghost, _ptr(energy), _ptr(atom_energy), sp))

    def backward_device(self, grad_coords, atom_weight=None, virial=None, stream=None):
        """Adjoint of the last forward (dp_backward_device): d(sum_i w_i e_i)/dx."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        _check(_lib.dp_backward_device(self._h, _ptr(atom_weight), _ptr(grad_coords),
                                       _ptr(virial), sp))

    def set_precision(self, precision: int):
        """Operand precision of the matrix-core products (dp_set_precision):
        PREC_FP32 (default) or PREC_BF16 (BF16 operands, FP32 accumulation)."""
        _check(_lib.dp_set_precision(self._h, int(precision)))

    def set_memory_budget(self, nbytes: float):
        """Workspace budget in bytes (0: unlimited); above it the attention
        activations are recomputed in the adjoint (dp_set_memory_budget)."""
        _check(_lib.dp_set_memory_budget(self._h, float(nbytes)))

    def memory_info(self):
        """(workspace bytes, recompute flag) of the current workspace."""
        b = ctypes.c_int64()
        r = ctypes.c_int32()
        _check(_lib.dp_memory_info(self._h, ctypes.byref(b), ctypes.byref(r)))
        return int(b.value), bool(r.value)

    def sync(self):
        """Wait for the last step; raises on a device-side error (overflow, bad type)."""
        _check(_lib.dp_sync(self._h))

    def debug_nlist(self, nloc: int):
        nl = np.zeros((max(nloc, 1), self.sel), dtype=np.int32)
        nn = np.zeros(max(nloc, 1), dtype=np.int32)
        _check(_lib.dp_debug_nlist(self._h, nl.ctypes.data, nn.ctypes.data))
        return nl[:nloc], nn[:nloc]

    def set_timing(self, enable: bool):
        _check(_lib.dp_set_timing(self._h, int(bool(enable))))

    def kernel_times(self) -> dict:
        n = _check(_lib.dp_kernel_times(self._h, None, None, None, 0))
        names = ctypes.create_string_buffer(48 * max(n, 1))
        counts = np.zeros(max(n, 1), dtype=np.int64)
        ms = np.zeros(max(n, 1))
        _check(_lib.dp_kernel_times(self._h, names, counts.ctypes.data, ms.ctypes.data, n))
        out = {}
        for k in range(n):
            nm = names.raw[48 * k:48 * (k + 1)].split(b"\0", 1)[0].decode()
            out[nm] = (int(counts[k]), float(ms[k]))
        return out


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


class Trainer:
    """Student trainer (include/dpa1_train.h): exact energy+force loss gradient and Adam.

    frames (float64 [B, N, 3]), types (int32 [N]), e_label (float64 [B]) and
    f_label (float64 [B, N, 3]) are torch CUDA tensors; box is host data or None.
    """

    def __init__(self, weights_path: str, rcut: float, sel: int, pref_e: float = 1.0,
                 pref_f: float = 100.0, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8, precision: int = PREC_FP32):
        lib = load_library()
        opt = TrainOptions(pref_e, pref_f, beta1, beta2, eps, precision)
        h = ctypes.c_void_p()
        _check(lib.dp_train_create(weights_path.encode(), float(rcut), int(sel), ctypes.byref(opt),
                                   ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int32()
        _check(lib.dp_train_params(h, None, ctypes.byref(n)))
        self.nparams = n.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.dp_train_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def gradient(self, frames, types, box, e_label, f_label, stream=None):
        """(loss [3] = (L, L_e, L_f), grad [nparams] FP64 in weights-file order)."""
        B, N = int(frames.shape[0]), int(frames.shape[1])
        boxa = None if box is None else np.ascontiguousarray(box, dtype=np.float64).reshape(9)
        loss = np.zeros(3)
        grad = np.zeros(self.nparams)
        _check(_lib.dp_train_gradient(self._h, _ptr(frames), _ptr(types), _ptr(boxa), N, B,
                                      _ptr(e_label), _ptr(f_label), loss.ctypes.data,
                                      grad.ctypes.data, _stream_ptr(stream)))
        return loss, grad

    def step(self, frames, types, box, e_label, f_label, lr: float, stream=None):
        """One Adam step; returns the loss [3] of the batch before the update."""
        B, N = int(frames.shape[0]), int(frames.shape[1])
        boxa = None if box is None else np.ascontiguousarray(box, dtype=np.float64).reshape(9)
        loss = np.zeros(3)
        _check(_lib.dp_train_step(self._h, _ptr(frames), _ptr(types), _ptr(boxa), N, B,
                                  _ptr(e_label), _ptr(f_label), float(lr), loss.ctypes.data,
                                  _stream_ptr(stream)))
        return loss

    def params(self) -> np.ndarray:
        out = np.zeros(self.nparams)
        n = ctypes.c_int32()
        _check(_lib.dp_train_params(self._h, out.ctypes.data, ctypes.byref(n)))
        return out

    def save(self, path: str):
        """Current weights as a weights file (usable by Model)."""
        _check(_lib.dp_train_save(self._h, path.encode()))

    def checkpoint(self, path: str):
        """FP32 masters, Adam moments and step count (resume continues exactly)."""
        _check(_lib.dp_train_checkpoint(self._h, path.encode()))

    def resume(self, path: str):
        _check(_lib.dp_train_resume(self._h, path.encode()))


def force_error(a, b, stream=None):
    """(RMSE, max abs error) between two [N, 3] float64 device force arrays (dp_force_error)."""
    load_library()
    out = np.zeros(2)
    _check(_lib.dp_force_error(_ptr(a), _ptr(b), int(a.shape[0]), out.ctypes.data,
                               _stream_ptr(stream)))
    return float(out[0]), float(out[1])


def force_error_noalloc(a, b, out, stream=None):
    """dp_force_error_noalloc: (RMSE, max abs error) of two [N, 3] float64
    device force arrays into the float64 device tensor ``out`` [2],
    asynchronously, without any device allocation."""
    load_library()
    _check(_lib.dp_force_error_noalloc(_ptr(a), _ptr(b), int(a.shape[0]), _ptr(out),
                                       _stream_ptr(stream)))
