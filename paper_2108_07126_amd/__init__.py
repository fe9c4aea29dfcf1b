"""Python binding of the MI355X parallel-in-time Schrodinger propagator.

Argument marshalling only: every step of the propagation runs in the HIP
library ``libparament.so`` (built in-tree by ``paper_2108_07126_amd/build.py``),
reached through its C ABI (include/parament.h) with ctypes.  Importing this
package fails loudly when the library has not been built; there is no other
code path.

PyTorch is used only for device memory and streams (``equiprop_dev`` takes
CUDA/HIP tensors and enqueues on torch's current stream).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libparament.so")

PM_FP64, PM_FP32, PM_FP32_3M, PM_BF16_SPLIT = 0, 1, 2, 3
PM_EXPM_TAYLOR, PM_EXPM_CHEBYSHEV = 0, 1
PM_TRAJ_PROPAGATORS, PM_TRAJ_STATES, PM_TRAJ_DENSITY = 0, 1, 2
PM_OPT_GD, PM_OPT_ADAM = 0, 1
PM_WORK_PROPAGATE, PM_WORK_GRADIENT, PM_WORK_TRAJECTORY = 0, 1, 2
PM_ORDER_MIDPOINT, PM_ORDER_MAGNUS4, PM_ORDER_CF4, PM_ORDER_MAGNUS6 = 2, 4, 5, 6
MAX_CHEBYSHEV_DEGREE = 25
PRECISIONS = {"fp64": PM_FP64, "fp32": PM_FP32, "fp32_3m": PM_FP32_3M, "bf16_split": PM_BF16_SPLIT}
STATUS = ["PM_OK", "PM_E_INVALID_ARG", "PM_E_NOT_READY", "PM_E_NOT_HERMITIAN", "PM_E_OOM",
          "PM_E_DEVICE", "PM_E_UNSUPPORTED"]
MAX_DIM = 64
MAX_TAYLOR_DEGREE = 21

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_i64_p = ctypes.POINTER(ctypes.c_int64)

# name -> (restype, argtypes): every entry point declared in include/parament.h
SIGNATURES = {
    "pm_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int]),
    "pm_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "pm_set_hamiltonian": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.c_void_p, ctypes.c_int]),
    "pm_equiprop": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "pm_equiprop_dev": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pm_equiprop_dev_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pm_backward_dev": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pm_trajectory_dev": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "pm_grape_dev": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                                    ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.c_void_p]),
    "pm_fidelity_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                                        ctypes.c_void_p, _c_double_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pm_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int]),
    "pm_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "pm_batch_set": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "pm_batch_set_chunk": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64]),
    "pm_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pm_batch_result": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "pm_batch_output_dev": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "pm_batch_packets": (ctypes.c_int64, [ctypes.c_void_p]),
    "pm_batch_output_doubles": (ctypes.c_int64, [ctypes.c_void_p]),
    "pm_batch_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "pm_tuning_set": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.c_int64]),
    "pm_set_expm_policy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "pm_set_chunk": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "pm_set_chain_skew": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "pm_set_expm_method": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "pm_chebyshev_theta": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _c_double_p]),
    "pm_plan_chebyshev": (ctypes.c_int, [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, _c_int_p,
                                         _c_int_p]),
    "pm_launch_shape": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "pm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "pm_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "pm_basis_count": (ctypes.c_int64, [ctypes.c_int64, ctypes.c_int]),
    "pm_build_basis_host": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                           ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "pm_slice_weights_host": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                                             ctypes.c_int, ctypes.c_int64, ctypes.c_void_p]),
    "pm_taylor_theta": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int64, _c_double_p]),
    "pm_plan_expm": (ctypes.c_int, [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _c_int_p,
                                    _c_int_p]),
    "pm_set_workspace_limit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "pm_workspace_held": (ctypes.c_int64, [ctypes.c_void_p]),
    "pm_workspace_plan": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                         ctypes.c_int, ctypes.c_int64, _c_i64_p, _c_i64_p]),
}


def _load():
    # PyTorch (device memory and streams for the *_dev entry points) ships its
    # own HIP runtime; loading it first makes the library bind to that same
    # runtime, so one process never holds two
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python paper_2108_07126_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()

TUNING_PATH = os.path.join(_HERE, "tuning.txt")


def load_tuning(path: str = TUNING_PATH) -> int:
    """Apply an autotuner table (lines: key dim_class precision value)."""
    if not os.path.exists(path):
        return 0
    n = 0
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if len(line) != 4:
                continue
            key, dc, prec, val = line[0], int(line[1]), int(line[2]), int(line[3])
            if _lib.pm_tuning_set(key.encode(), dc, prec, val) == 0:
                n += 1
    return n


load_tuning()


class ParamentError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        self.name = STATUS[status] if 0 <= status < len(STATUS) else f"status {status}"
        super().__init__(f"{self.name}: {detail}" if detail else self.name)


def _check(status: int, ctx=None):
    if status != 0:
        detail = _lib.pm_last_error(ctx).decode() if ctx else ""
        raise ParamentError(status, detail)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _as_c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


# ----------------------------------------------------------- host helpers

def basis_count(n_ctrl: int, order: int) -> int:
    return int(_lib.pm_basis_count(n_ctrl, order))


def build_basis_host(H0, Hk, order: int) -> Tuple[np.ndarray, np.ndarray]:
    """The Hermitian basis the device receives (FP64) and its 1-norms."""
    H0 = _as_c128(H0)
    d = H0.shape[0]
    Hk = _as_c128(Hk).reshape(-1, d, d)
    K = Hk.shape[0]
    M = basis_count(K, order)
    if M < 0:
        raise ParamentError(1, "bad n_ctrl / order")
    out = np.zeros((M, d, d), np.complex128)
    norms = np.zeros(M)
    _check(_lib.pm_build_basis_host(d, _ptr(H0), K, _ptr(Hk) if K else None, order, _ptr(out), _ptr(norms)))
    return out, norms


def slice_weights_host(samples, dt: float, order: int, slice_index: int) -> np.ndarray:
    """Weights of one exponent on the basis ([M]; order 6: [3][M], the
    moments P1, P2, P3)."""
    s = np.ascontiguousarray(np.asarray(samples, np.float64))
    K, S = s.shape
    M = basis_count(K, order)
    w = np.zeros((3, M) if order == PM_ORDER_MAGNUS6 else M)
    _check(_lib.pm_slice_weights_host(K, _ptr(s) if K else None, S, dt, order, slice_index, _ptr(w)))
    return w


def taylor_theta(m: int, precision: int = PM_FP64, n_slices: int = 1) -> float:
    t = ctypes.c_double()
    _check(_lib.pm_taylor_theta(m, precision, n_slices, ctypes.byref(t)))
    return t.value


def plan_expm(nu: float, precision: int = PM_FP64, max_degree: int = MAX_TAYLOR_DEGREE,
              n_slices: int = 1) -> Tuple[int, int]:
    m, s = ctypes.c_int(), ctypes.c_int()
    _check(_lib.pm_plan_expm(nu, precision, max_degree, n_slices, ctypes.byref(m), ctypes.byref(s)))
    return m.value, s.value


def chebyshev_theta(m: int, precision: int = PM_FP64) -> float:
    """Table-1 limit of the degree-m Chebyshev series (Lubich's estimate)."""
    t = ctypes.c_double()
    _check(_lib.pm_chebyshev_theta(m, precision, ctypes.byref(t)))
    return t.value


def plan_chebyshev(nu: float, precision: int = PM_FP64, max_degree: int = MAX_CHEBYSHEV_DEGREE,
                   force_s: int = -1) -> Tuple[int, int]:
    m, s = ctypes.c_int(), ctypes.c_int()
    _check(_lib.pm_plan_chebyshev(nu, precision, max_degree, force_s, ctypes.byref(m), ctypes.byref(s)))
    return m.value, s.value


def workspace_plan(dim: int, n_ctrl: int, order: int, precision: int, n_samples: int,
                   kind: int = PM_WORK_PROPAGATE, limit: int = 0) -> Tuple[int, int]:
    """(chain length, device workspace bytes) of a call under a workspace
    limit (host-only; raises ParamentError PM_E_OOM if it cannot fit)."""
    c, b = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.pm_workspace_plan(dim, n_ctrl, order, precision, n_samples, kind, int(limit),
                                  ctypes.byref(c), ctypes.byref(b)))
    return c.value, b.value


def n_slices(n_samples: int, order: int) -> int:
    """Slices covered by n_samples samples (2N + 1 samples for order 4 and
    CF4, 3N for order 6)."""
    if order == 2:
        return n_samples
    if order == PM_ORDER_MAGNUS6:
        return n_samples // 3
    return (n_samples - 1) // 2


# ------------------------------------------------------------------ context

class Context:
    """A propagator context (create -> set_hamiltonian -> equiprop ...)."""

    def __init__(self, device: int = 0, precision: int = PM_FP64):
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        h = ctypes.c_void_p()
        st = _lib.pm_create(ctypes.byref(h), device, precision)
        if st != 0:
            raise ParamentError(st, "pm_create: " + _lib.pm_last_error(None).decode())
        self._h = h
        self.device = device
        self.precision = precision
        self.dim = None
        self.n_ctrl = None
        self.order = None

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _lib.pm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_hamiltonian(self, H0, Hk, order: int = 2):
        H0 = _as_c128(H0)
        d = H0.shape[0]
        Hk = _as_c128(Hk).reshape(-1, d, d)
        K = Hk.shape[0]
        _check(_lib.pm_set_hamiltonian(self._h, d, _ptr(H0), K, _ptr(Hk) if K else None, order), self._h)
        self.dim, self.n_ctrl, self.order = d, K, order

    def set_expm_policy(self, max_taylor_degree: int = MAX_TAYLOR_DEGREE, force_s: int = -1):
        _check(_lib.pm_set_expm_policy(self._h, max_taylor_degree, force_s), self._h)

    def set_chunk(self, chunk: int = 0):
        _check(_lib.pm_set_chunk(self._h, chunk), self._h)

    def set_chain_skew(self, percent: int = -1):
        """Percent longer chains for the first-dispatched blocks (-1 automatic, 0 equal chains)."""
        _check(_lib.pm_set_chain_skew(self._h, percent), self._h)

    def set_expm_method(self, method: int = PM_EXPM_TAYLOR):
        """PM_EXPM_TAYLOR (default) or PM_EXPM_CHEBYSHEV (the paper's series)."""
        _check(_lib.pm_set_expm_method(self._h, method), self._h)

    def set_workspace_limit(self, nbytes: int = 0):
        """Limit the context's device workspace (0: no limit)."""
        _check(_lib.pm_set_workspace_limit(self._h, int(nbytes)), self._h)

    @property
    def workspace_held(self) -> int:
        """Bytes of device workspace the context holds now."""
        return int(_lib.pm_workspace_held(self._h))

    def launch_shape(self, n_samples: int) -> Tuple[int, int, int]:
        """(chunk, chains, leaves) a propagation of n_samples would use."""
        c, n, l = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.pm_launch_shape(self._h, n_samples, ctypes.byref(c), ctypes.byref(n), ctypes.byref(l)),
               self._h)
        return c.value, n.value, l.value

    def equiprop(self, samples, dt: float, return_slices: bool = False):
        """U(T) (complex128) from host samples [n_ctrl][n_samples]; optionally all U_j."""
        s = np.ascontiguousarray(np.asarray(samples, np.float64))
        if s.ndim == 1:
            s = s[None]
        S = s.shape[1]
        U = np.zeros((self.dim, self.dim), np.complex128)
        sl = None
        if return_slices:
            dt_c = np.complex128 if self.precision == PM_FP64 else np.complex64
            sl = np.zeros((n_slices(S, self.order), self.dim, self.dim), dt_c)
        _check(_lib.pm_equiprop(self._h, _ptr(s), S, float(dt), _ptr(U), _ptr(sl) if sl is not None else None),
               self._h)
        return (U, sl) if return_slices else U

    def equiprop_dev(self, samples_t, dt: float, U_t, slices_t=None, stream=None, noalloc: bool = False):
        """Device variant: torch tensors on the GPU; enqueued on `stream`
        (default: torch's current stream), not synchronised.  noalloc: call
        pm_equiprop_dev_noalloc (the tree workspace in the library's fixed
        device array; no allocation)."""
        import torch
        assert samples_t.is_cuda and samples_t.dtype == torch.float64 and samples_t.is_contiguous()
        assert U_t.is_cuda and U_t.dtype == torch.complex128 and U_t.is_contiguous()
        if slices_t is not None:
            want = torch.complex128 if self.precision == PM_FP64 else torch.complex64
            assert slices_t.is_cuda and slices_t.dtype == want and slices_t.is_contiguous()
        if stream is None:
            stream = torch.cuda.current_stream(U_t.device)
        S = samples_t.shape[-1]
        fn = _lib.pm_equiprop_dev_noalloc if noalloc else _lib.pm_equiprop_dev
        _check(fn(self._h, ctypes.c_void_p(samples_t.data_ptr()), S, float(dt),
                                    ctypes.c_void_p(U_t.data_ptr()),
                                    ctypes.c_void_p(slices_t.data_ptr()) if slices_t is not None else None,
                                    ctypes.c_void_p(stream.cuda_stream)), self._h)


    def trajectory_dev(self, samples_t, dt: float, out_t, kind: int = PM_TRAJ_PROPAGATORS, x0_t=None,
                       stream=None):
        """Time evolution at every slice boundary into out_t (device
        complex128 [N+1][d][d], or [N+1][d][n] for states); x0_t: device
        complex128 states [d][n] or density [d][d]."""
        import torch
        assert samples_t.is_cuda and samples_t.dtype == torch.float64 and samples_t.is_contiguous()
        assert out_t.is_cuda and out_t.dtype == torch.complex128 and out_t.is_contiguous()
        n_vec = 0
        if x0_t is not None:
            assert x0_t.is_cuda and x0_t.dtype == torch.complex128 and x0_t.is_contiguous()
            n_vec = x0_t.shape[1] if x0_t.dim() == 2 else 1
        if stream is None:
            stream = torch.cuda.current_stream(out_t.device)
        S = samples_t.shape[-1]
        _check(_lib.pm_trajectory_dev(self._h, ctypes.c_void_p(samples_t.data_ptr()), S, float(dt), kind,
                                      ctypes.c_void_p(x0_t.data_ptr()) if x0_t is not None else None, n_vec,
                                      ctypes.c_void_p(out_t.data_ptr()), ctypes.c_void_p(stream.cuda_stream)),
               self._h)

    def trajectory(self, samples, dt: float, kind: int = PM_TRAJ_PROPAGATORS, x0=None) -> np.ndarray:
        """Host convenience over trajectory_dev (device buffers from torch)."""
        import torch
        s = np.ascontiguousarray(np.asarray(samples, np.float64))
        if s.ndim == 1:
            s = s[None]
        d = self.dim
        N = n_slices(s.shape[1], self.order)
        dev = torch.device("cuda", self.device)
        st = torch.from_numpy(s).to(dev)
        x0_t = None
        cols = d
        if kind == PM_TRAJ_STATES:
            x0 = _as_c128(x0).reshape(d, -1)
            cols = x0.shape[1]
        if x0 is not None and kind != PM_TRAJ_PROPAGATORS:
            x0_t = torch.from_numpy(_as_c128(x0).reshape(d, cols)).to(dev)
        out = torch.empty((N + 1, d, cols), dtype=torch.complex128, device=dev)
        self.trajectory_dev(st, dt, out, kind, x0_t)
        torch.cuda.synchronize(dev)
        return out.cpu().numpy()

    def grape_dev(self, samples_t, dt: float, V_t, iters: int, step: float, optimizer: int = PM_OPT_ADAM,
                  loss_t=None, stream=None):
        """Optimise the controls in place (device float64 [K][S]) for the gate
        V_t (device complex128 [d][d]); returns the device loss history
        (iters + 1 values)."""
        import torch
        assert samples_t.is_cuda and samples_t.dtype == torch.float64 and samples_t.is_contiguous()
        assert V_t.is_cuda and V_t.dtype == torch.complex128 and V_t.is_contiguous()
        if loss_t is None:
            loss_t = torch.empty(iters + 1, dtype=torch.float64, device=samples_t.device)
        if stream is None:
            stream = torch.cuda.current_stream(samples_t.device)
        _check(_lib.pm_grape_dev(self._h, ctypes.c_void_p(samples_t.data_ptr()), samples_t.shape[-1], float(dt),
                                 ctypes.c_void_p(V_t.data_ptr()), int(iters), float(step), int(optimizer),
                                 ctypes.c_void_p(loss_t.data_ptr()), ctypes.c_void_p(stream.cuda_stream)),
               self._h)
        return loss_t

    def fidelity_grad(self, samples, dt: float, V):
        """Gate-fidelity loss 1 - |Tr(V^H U)|^2/d^2, its gradient w.r.t. the
        samples [n_ctrl][n_samples], and U(T).  FP64 contexts only."""
        s = np.ascontiguousarray(np.asarray(samples, np.float64))
        if s.ndim == 1:
            s = s[None]
        V = _as_c128(V)
        loss = ctypes.c_double()
        grad = np.zeros_like(s)
        U = np.zeros((self.dim, self.dim), np.complex128)
        _check(_lib.pm_fidelity_grad(self._h, _ptr(s), s.shape[1], float(dt), _ptr(V), ctypes.byref(loss),
                                     _ptr(grad), _ptr(U)), self._h)
        return loss.value, grad, U

    def backward_dev(self, samples_t, dt: float, W_t, grad_t, U_t=None, stream=None):
        """dL/d samples into grad_t for dL = Re Tr(W^H dU(T)) (device tensors;
        enqueued on `stream`, default torch's current stream)."""
        import torch
        assert samples_t.is_cuda and samples_t.dtype == torch.float64 and samples_t.is_contiguous()
        assert W_t.is_cuda and W_t.dtype == torch.complex128 and W_t.is_contiguous()
        assert grad_t.is_cuda and grad_t.dtype == torch.float64 and grad_t.is_contiguous()
        if stream is None:
            stream = torch.cuda.current_stream(W_t.device)
        _check(_lib.pm_backward_dev(self._h, ctypes.c_void_p(samples_t.data_ptr()), samples_t.shape[-1],
                                    float(dt), ctypes.c_void_p(W_t.data_ptr()),
                                    ctypes.c_void_p(grad_t.data_ptr()),
                                    ctypes.c_void_p(U_t.data_ptr()) if U_t is not None else None,
                                    ctypes.c_void_p(stream.cuda_stream)), self._h)


class _Instance(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int64), ("n_ctrl", ctypes.c_int64), ("order", ctypes.c_int),
                ("H0", ctypes.c_void_p), ("Hk", ctypes.c_void_p), ("samples", ctypes.c_void_p),
                ("n_samples", ctypes.c_int64), ("dt", ctypes.c_double)]


class Batch:
    """Many independent instances propagated by one persistent launch.

    Each instance is anything with attributes H0, Hk, samples, h (slice
    width) and order (e.g. a ``synth.Workload``)."""

    def __init__(self, device: int = 0, precision: int = PM_FP64):
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        h = ctypes.c_void_p()
        st = _lib.pm_batch_create(ctypes.byref(h), device, precision)
        if st != 0:
            raise ParamentError(st, "pm_batch_create: " + _lib.pm_batch_last_error(None).decode())
        self._h = h
        self.precision = precision
        self.dims = []

    def _check(self, st):
        if st != 0:
            raise ParamentError(st, _lib.pm_batch_last_error(self._h).decode())

    def close(self):
        if self._h:
            _lib.pm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_chunk(self, dim_class: int, chunk: int):
        self._check(_lib.pm_batch_set_chunk(self._h, dim_class, chunk))

    def set(self, instances):
        keep = []
        arr = (_Instance * len(instances))()
        dims = []
        for i, w in enumerate(instances):
            H0 = _as_c128(w.H0)
            d = H0.shape[0]
            Hk = _as_c128(w.Hk).reshape(-1, d, d)
            c = np.ascontiguousarray(np.asarray(w.samples, np.float64))
            if c.ndim == 1:
                c = c[None]
            K = Hk.shape[0]
            keep += [H0, Hk, c]
            arr[i] = _Instance(d, K, int(w.order), H0.ctypes.data, Hk.ctypes.data if K else None,
                               c.ctypes.data if K else None, c.shape[1], float(w.h))
            dims.append(d)
        self._check(_lib.pm_batch_set(self._h, ctypes.cast(arr, ctypes.c_void_p), len(instances)))
        self.dims = dims

    @property
    def n_packets(self) -> int:
        return int(_lib.pm_batch_packets(self._h))

    def run(self, stream=None):
        """Enqueue the whole batch (default: the null stream)."""
        s = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        self._check(_lib.pm_batch_run(self._h, s))

    def results(self):
        n = int(_lib.pm_batch_output_doubles(self._h))
        buf = np.zeros(n // 2, np.complex128)
        self._check(_lib.pm_batch_result(self._h, _ptr(buf), n))
        out, o = [], 0
        for d in self.dims:
            out.append(buf[o:o + d * d].reshape(d, d).copy())
            o += d * d
        return out


def _make_function():
    import torch

    class Propagate(torch.autograd.Function):
        """U(T) = equiprop(samples) with the adjoint backward of the library.

        forward(ctx_obj, samples [n_ctrl][n_samples] float64 cuda, dt) ->
        U(T) complex128 [dim][dim]; backward turns dL/dconj(U) into dL/d samples
        through pm_backward_dev."""

        @staticmethod
        def forward(fctx, pctx, samples, dt):
            samples = samples.contiguous()
            U = torch.zeros((pctx.dim, pctx.dim), dtype=torch.complex128, device=samples.device)
            pctx.equiprop_dev(samples, dt, U)
            fctx.pctx = pctx
            fctx.dt = dt
            fctx.save_for_backward(samples)
            return U

        @staticmethod
        def backward(fctx, grad_U):
            (samples,) = fctx.saved_tensors
            grad = torch.zeros_like(samples)
            fctx.pctx.backward_dev(samples, fctx.dt, grad_U.contiguous().to(torch.complex128), grad)
            return None, grad, None

    return Propagate


_Propagate = None


def propagate_autograd(pctx: "Context", samples_t, dt: float):
    """Differentiable U(T) (torch.autograd) through the library's adjoint."""
    global _Propagate
    if _Propagate is None:
        _Propagate = _make_function()
    return _Propagate.apply(pctx, samples_t, dt)


def propagate(H0, Hk, samples, dt: float, order: int = 2, precision: int = PM_FP64,
              return_slices: bool = False, device: int = 0):
    """One-shot helper: create a context, set the Hamiltonian, propagate."""
    with Context(device, precision) as ctx:
        ctx.set_hamiltonian(H0, Hk, order)
        return ctx.equiprop(samples, dt, return_slices)
