"""Thin ctypes binding of liblsp (the C ABI in include/lsp.h).

Argument marshalling only: tensors are checked for device, dtype, size and
contiguity and their device pointers handed to the library, which runs every
step on the GPU. There is no fallback: if liblsp.so is missing or cannot be
loaded, every call raises.

Names follow the C ABI: Problem.stencil_setup -> lsp_stencil_setup, etc.
"""
from __future__ import annotations

import ctypes
import os
from typing import Callable, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsp.so")

LSP_OK = 0
LSP_NOT_CONVERGED = 1
LSP_EINVAL = -1
LSP_ENONFINITE = -2
LSP_ERESONANT = -3
LSP_ENOMEM = -4
LSP_EHIP = -5
LSP_ESOLVER = -6
LSP_ESTATE = -7
LSP_FP64 = 0
LSP_FP32_REFINE = 1
STAGES = ("shifts", "green", "null", "assemble", "setup", "apply", "c_apply", "psolve",
          "arnoldi")

HOST_SOLVE_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double), ctypes.c_int64)

_lib = None


class NDFactors(ctypes.Structure):
    """struct lsp_nd_factors: host arrays of the nested-dissection factors."""
    _fields_ = [(k, ctypes.c_int64) for k in ("nfronts", "nlevels", "nidx_U", "ndata")] + \
        [(k, ctypes.c_void_p) for k in ("f", "u", "off_F", "off_U", "idx_F", "idx_Fp", "idx_U",
                                        "off_blk", "data", "upd_ptr", "upd_pos", "lev_ptr",
                                        "lev_fronts")]


class LSPError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        lib_ = load()
        msg = lib_.lsp_last_error().decode()
        name = lib_.lsp_strerror(code).decode()
        super().__init__(f"{where}: {name} ({code}): {msg}")


def load():
    """Load liblsp.so (built in-tree by paper_1607_02560_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                           "`python -m paper_1607_02560_amd.build`")
    lib_ = ctypes.CDLL(LIB_PATH)
    c_int, c_double, c_void_p, c_int64 = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_int64
    P = ctypes.POINTER
    sig = {
        "lsp_strerror": (ctypes.c_char_p, [c_int]),
        "lsp_last_error": (ctypes.c_char_p, []),
        "lsp_version": (ctypes.c_char_p, []),
        "lsp_create": (c_int, [c_int, c_int, c_void_p, c_void_p, P(c_void_p)]),
        "lsp_set_potential": (c_int, [c_void_p, c_void_p]),
        "lsp_destroy": (None, [c_void_p]),
        "lsp_stencil_setup": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p]),
        "lsp_stencil_setup_global": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p]),
        "lsp_stencil_setup_nd": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p]),
        "lsp_ps_apply": (c_int, [c_void_p, c_void_p, c_void_p]),
        "lsp_c_apply": (c_int, [c_void_p, c_void_p, c_void_p]),
        "lsp_precond_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_int, c_int,
                                      HOST_SOLVE_FN, c_void_p, P(c_int), P(c_double)]),
        "lsp_get_tables": (c_int, [c_void_p, c_int, P(c_int), c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_void_p, c_void_p]),
        "lsp_default_num_shifts": (c_int, [c_int, c_int]),
        "lsp_stencil_size": (c_int, [c_void_p]),
        "lsp_export_pattern": (c_int, [c_int, c_int, c_int, c_void_p]),
        "lsp_profile": (c_int, [c_void_p, c_int]),
        "lsp_profile_read": (c_int, [c_void_p, c_int, c_void_p, c_void_p]),
        "lsp_mlp_create": (c_int, [c_int, c_int, c_int, c_int, c_void_p, P(c_void_p)]),
        "lsp_mlp_destroy": (None, [c_void_p]),
        "lsp_mlp_num_params": (c_int, [c_void_p]),
        "lsp_mlp_set_params": (c_int, [c_void_p, c_void_p]),
        "lsp_mlp_get_params": (c_int, [c_void_p, c_void_p]),
        "lsp_mlp_set_normalisation": (c_int, [c_void_p, c_void_p]),
        "lsp_mlp_get_normalisation": (c_int, [c_void_p, c_void_p]),
        "lsp_mlp_fit_normalisation": (c_int, [c_void_p, c_void_p, c_void_p, c_int]),
        "lsp_mlp_forward": (c_int, [c_void_p, c_void_p, c_int, c_void_p]),
        "lsp_mlp_loss_grad": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p,
                                      P(c_double)]),
        "lsp_mlp_train_step": (c_int, [c_void_p, c_void_p, c_void_p, c_int, ctypes.c_float,
                                       P(c_double)]),
        "lsp_training_rows": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p]),
        "lsp_stencil_setup_learned": (c_int, [c_void_p, c_void_p, c_int, c_int, c_double,
                                              c_void_p, c_void_p, P(c_int)]),
    }
    sig.update({
        "lsp_stencil_setup_static": (c_int, [c_int, c_int, c_void_p, c_int, c_int, c_int,
                                             c_void_p, c_void_p, c_void_p]),
        "lsp_static_scratch_bytes": (ctypes.c_size_t, []),
        "lsp_mlp_save": (c_int, [c_void_p, ctypes.c_char_p]),
        "lsp_mlp_load": (c_int, [ctypes.c_char_p, c_int, c_void_p, P(c_void_p)]),
        "lsp_batch_create": (c_int, [c_int, c_void_p, P(c_void_p)]),
        "lsp_batch_destroy": (None, [c_void_p]),
        "lsp_batch_stencil_setup": (c_int, [c_void_p, c_int, c_void_p, c_int, c_void_p,
                                            c_void_p]),
        "lsp_batch_ps_apply": (c_int, [c_void_p, c_void_p, c_void_p]),
        "lsp_batch_tile": (c_int, [c_void_p, P(c_int), c_void_p, c_void_p]),
        "lsp_batch_set_tile": (c_int, [c_void_p, c_int]),
        "lsp_get_tables_nd1": (c_int, [c_void_p, c_int, P(c_int), c_void_p, c_void_p,
                                       c_void_p, c_void_p, c_void_p]),
        "lsp_autotune": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p,
                                 c_int, c_void_p, c_void_p]),
        "lsp_set_tuning": (c_int, [c_void_p, c_void_p]),
        "lsp_get_tuning": (c_int, [c_void_p, c_void_p]),
        "lsp_psolve_upload": (c_int, [c_void_p, P(NDFactors)]),
        "lsp_psolve_apply": (c_int, [c_void_p, c_void_p, c_void_p]),
        "lsp_precond_solve_device": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_int,
                                             c_int, P(c_int), P(c_double)]),
    })
    for name, (res, args) in sig.items():
        fn = getattr(lib_, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib_
    return _lib


def _check(code: int, where: str) -> int:
    if code < 0:
        raise LSPError(code, where)
    return code


def _ptr(t) -> int:
    return t.data_ptr()


def _need(t, dtype, numel: int, name: str):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def default_num_shifts(d: int, n: int) -> int:
    return _check(load().lsp_default_num_shifts(d, n), "lsp_default_num_shifts")


def export_pattern(d: int, n: int, t: int) -> np.ndarray:
    """Column index of every P / C entry: (N, m) int64."""
    m = (2 * t + 1) ** d
    out = np.empty((n ** d, m), dtype=np.int64)
    _check(load().lsp_export_pattern(d, n, t, out.ctypes.data), "lsp_export_pattern")
    return out


class Problem:
    """A problem (L + diag v) u = f on the periodic grid, resident on one GPU."""

    def __init__(self, d: int, n: int, v, stream=None):
        import torch
        self.lib = load()
        self.d, self.n = d, n
        self.N = n ** d
        _need(v, torch.float64, self.N, "v")
        self.device = v.device
        if stream is None:
            stream = torch.cuda.current_stream(v.device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(self.lib.lsp_create(d, n, _ptr(v), ctypes.c_void_p(stream.cuda_stream),
                                   ctypes.byref(h)), "lsp_create")
        self._h = h
        self.t = None
        self.m = None

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.lsp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- entry points -----------------------------------------------------
    def set_potential(self, v):
        import torch
        _need(v, torch.float64, self.N, "v")
        _check(self.lib.lsp_set_potential(self._h, _ptr(v)), "lsp_set_potential")

    def stencil_setup(self, t: int, num_shifts: int, P, idx=None, precision: int = LSP_FP64):
        import torch
        m = (2 * t + 1) ** self.d
        _need(P, torch.float32 if precision == LSP_FP32_REFINE else torch.float64,
              self.N * m, "P")
        if idx is not None:
            _need(idx, torch.int32, self.N, "idx")
        _check(self.lib.lsp_stencil_setup(self._h, t, num_shifts, precision, _ptr(P),
                                          _ptr(idx) if idx is not None else None),
               "lsp_stencil_setup")
        self.t, self.m = t, m

    def stencil_setup_global(self, t: int, P, idx=None, precision: int = LSP_FP64):
        """Non-localized setup (one shift, the mean of v); same outputs as
        stencil_setup."""
        import torch
        m = (2 * t + 1) ** self.d
        _need(P, torch.float32 if precision == LSP_FP32_REFINE else torch.float64,
              self.N * m, "P")
        if idx is not None:
            _need(idx, torch.int32, self.N, "idx")
        _check(self.lib.lsp_stencil_setup_global(self._h, t, precision, _ptr(P),
                                                 _ptr(idx) if idx is not None else None),
               "lsp_stencil_setup_global")
        self.t, self.m = t, m

    def stencil_setup_nd(self, leaf: int, num_shifts: int, P, idx=None):
        """Setup with the per-point radius of Sec. 4.2 (leaf box `leaf`,
        radius <= 2); P holds N rows of 5^d entries (radius-2 layout)."""
        import torch
        m = 5 ** self.d
        _need(P, torch.float64, self.N * m, "P")
        if idx is not None:
            _need(idx, torch.int32, self.N, "idx")
        _check(self.lib.lsp_stencil_setup_nd(self._h, leaf, num_shifts, _ptr(P),
                                             _ptr(idx) if idx is not None else None),
               "lsp_stencil_setup_nd")
        self.t, self.m = 2, m

    def training_rows(self, P, points, X, T):
        """Features and exact targets of the given points after an exact setup."""
        import torch
        count = points.numel()
        _need(P, torch.float64, self.N * self.m, "P")
        _need(points, torch.int64, count, "points")
        _need(X, torch.float32, count * (self.m + 2), "X")
        _need(T, torch.float32, count * 2 * self.m, "T")
        _check(self.lib.lsp_training_rows(self._h, _ptr(P), _ptr(points), count, _ptr(X), _ptr(T)),
               "lsp_training_rows")


    def stencil_setup_learned(self, mlp: "MLP", t: int, num_shifts: int, threshold: float,
                              P, fallback, count: bool = True):
        """Learned setup with exact fallback; returns the number of fallback rows
        (count=True, synchronous) or None (count=False, asynchronous)."""
        import torch
        m = (2 * t + 1) ** self.d
        _need(P, torch.float64, self.N * m, "P")
        _need(fallback, torch.int32, self.N, "fallback")
        nf = ctypes.c_int()
        _check(self.lib.lsp_stencil_setup_learned(self._h, mlp._h, t, num_shifts, threshold,
                                                  _ptr(P), _ptr(fallback),
                                                  ctypes.byref(nf) if count else None),
               "lsp_stencil_setup_learned")
        self.t, self.m = t, m
        return nf.value if count else None

    def ps_apply(self, u, y):
        import torch
        _need(u, torch.complex128, self.N, "u")
        _need(y, torch.complex128, self.N, "y")
        _check(self.lib.lsp_ps_apply(self._h, _ptr(u), _ptr(y)), "lsp_ps_apply")

    def c_apply(self, r, z):
        import torch
        _need(r, torch.complex128, self.N, "r")
        _need(z, torch.complex128, self.N, "z")
        _check(self.lib.lsp_c_apply(self._h, _ptr(r), _ptr(z)), "lsp_c_apply")

    def precond_solve(self, f, u, solve_P: Callable[[np.ndarray], np.ndarray], rtol=1e-8,
                      restart=40, maxit=400):
        """GMRES(restart) with preconditioner P^-1 C. solve_P maps a complex128
        host vector (N,) to P^-1 of it. Returns (status, iterations, relres)."""
        import torch
        _need(f, torch.complex128, self.N, "f")
        _need(u, torch.complex128, self.N, "u")
        errors = []

        def cb(user, rhs_p, x_p, N):
            try:
                rhs = np.ctypeslib.as_array(rhs_p, shape=(2 * N,)).view(np.complex128)
                x = np.ctypeslib.as_array(x_p, shape=(2 * N,)).view(np.complex128)
                x[:] = solve_P(rhs.copy())
                return 0
            except Exception as exc:  # reported through LSP_ESOLVER
                errors.append(exc)
                return 1

        cfn = HOST_SOLVE_FN(cb)
        iters = ctypes.c_int(0)
        relres = ctypes.c_double(0.0)
        code = self.lib.lsp_precond_solve(self._h, _ptr(f), _ptr(u), rtol, restart, maxit, cfn,
                                          None, ctypes.byref(iters), ctypes.byref(relres))
        if code == LSP_ESOLVER and errors:
            raise LSPError(code, "lsp_precond_solve") from errors[0]
        _check(code, "lsp_precond_solve")
        return code, iters.value, relres.value

    TUNE_KEYS = ("green_waves", "assembly_tile", "apply_form")

    def autotune(self, t: int, num_shifts: int, P, u, y, precision: int = LSP_FP64,
                 reps: int = 10) -> dict:
        """Time every candidate launch shape on this problem and keep the
        fastest; returns {shape: (choice, mean ms)}. P receives setup rows,
        y the apply's output."""
        import torch
        m = (2 * t + 1) ** self.d
        dt = torch.float32 if precision == LSP_FP32_REFINE else torch.float64
        _need(P, dt, self.N * m, "P")
        _need(u, torch.complex128, self.N, "u")
        _need(y, torch.complex128, self.N, "y")
        ch = np.zeros(3, dtype=np.int32)
        ms = np.zeros(3)
        _check(self.lib.lsp_autotune(self._h, t, num_shifts, precision, _ptr(P), _ptr(u),
                                     _ptr(y), reps, ch.ctypes.data, ms.ctypes.data),
               "lsp_autotune")
        self.t, self.m = t, m
        return {k: (int(c), float(v)) for k, c, v in zip(self.TUNE_KEYS, ch, ms)}

    def set_tuning(self, green_waves: int = 0, assembly_tile: int = 0, apply_form: int = 0):
        ch = np.array([green_waves, assembly_tile, apply_form], dtype=np.int32)
        _check(self.lib.lsp_set_tuning(self._h, ch.ctypes.data), "lsp_set_tuning")

    def get_tuning(self) -> dict:
        ch = np.zeros(3, dtype=np.int32)
        _check(self.lib.lsp_get_tuning(self._h, ch.ctypes.data), "lsp_get_tuning")
        return dict(zip(self.TUNE_KEYS, (int(c) for c in ch)))

    def psolve_upload(self, factors):
        """Copy nested-dissection factors of P to the device: an nd.NDFactor
        or the dict of its export()."""
        ex = factors.export() if hasattr(factors, "export") else factors
        keep = {}
        for k in ("f", "u", "off_F", "off_U", "idx_F", "idx_Fp", "idx_U", "off_blk", "upd_ptr",
                  "upd_pos", "lev_ptr", "lev_fronts"):
            keep[k] = np.ascontiguousarray(ex[k], dtype=np.int64)
        keep["data"] = np.ascontiguousarray(ex["data"], dtype=np.float64)
        st = NDFactors(nfronts=keep["f"].size, nlevels=keep["lev_ptr"].size - 1,
                       nidx_U=keep["idx_U"].size, ndata=keep["data"].size,
                       **{k: v.ctypes.data for k, v in keep.items()})
        _check(self.lib.lsp_psolve_upload(self._h, ctypes.byref(st)), "lsp_psolve_upload")

    def psolve_apply(self, r, z):
        """z = P^-1 r on the device with the uploaded factors."""
        import torch
        _need(r, torch.complex128, self.N, "r")
        _need(z, torch.complex128, self.N, "z")
        _check(self.lib.lsp_psolve_apply(self._h, _ptr(r), _ptr(z)), "lsp_psolve_apply")

    def precond_solve_device(self, f, u, rtol=1e-8, restart=40, maxit=400):
        """GMRES(restart) with P^-1 C, every step on the device (P^-1 from
        psolve_upload). Returns (status, iterations, relres)."""
        import torch
        _need(f, torch.complex128, self.N, "f")
        _need(u, torch.complex128, self.N, "u")
        iters = ctypes.c_int(0)
        relres = ctypes.c_double(0.0)
        code = self.lib.lsp_precond_solve_device(self._h, _ptr(f), _ptr(u), rtol, restart, maxit,
                                                 ctypes.byref(iters), ctypes.byref(relres))
        _check(code, "lsp_precond_solve_device")
        return code, iters.value, relres.value

    def profile(self, enable: bool):
        """Start (clearing the totals) or stop per-stage HIP-event timing."""
        _check(self.lib.lsp_profile(self._h, 1 if enable else 0), "lsp_profile")

    def profile_read(self) -> dict:
        """{stage: (total ms, calls)} since profiling started; synchronises."""
        ms = np.zeros(len(STAGES))
        cnt = np.zeros(len(STAGES), dtype=np.int32)
        _check(self.lib.lsp_profile_read(self._h, len(STAGES), ms.ctypes.data, cnt.ctypes.data),
               "lsp_profile_read")
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(STAGES)}

    def get_tables_nd1(self, capacity: int = 1024) -> dict:
        """Host copies of the radius-1 tables of the last per-point-radius setup."""
        m1 = 3 ** self.d
        alpha = np.zeros(capacity * m1)
        C = np.zeros(capacity * m1)
        sigma = np.zeros(capacity)
        g = np.zeros(capacity * m1)
        gam = np.zeros(capacity * m1)
        nS = ctypes.c_int(0)
        _check(self.lib.lsp_get_tables_nd1(self._h, capacity, ctypes.byref(nS), alpha.ctypes.data,
                                           C.ctypes.data, sigma.ctypes.data, g.ctypes.data,
                                           gam.ctypes.data), "lsp_get_tables_nd1")
        k = nS.value
        return {
            "alpha": alpha[:k * m1].reshape(k, m1).copy(),
            "C": C[:k * m1].reshape(k, m1).copy(),
            "sigma_min": sigma[:k].copy(),
            "g": g[:k * m1].reshape((k,) + (3,) * self.d).copy(),
            "gamma": gam[:k * m1].reshape((k,) + (3,) * self.d).copy(),
        }

    def get_tables(self, capacity: int = 1024) -> dict:
        """Host copies of the per-shift tables of the last setup."""
        if self.m is None:
            raise RuntimeError("no setup has been run")
        m = self.m
        wd = (2 * self.t + 1) ** self.d
        S = np.zeros(capacity)
        alpha = np.zeros(capacity * m)
        C = np.zeros(capacity * m)
        sigma = np.zeros(capacity)
        g = np.zeros(capacity * wd)
        gam = np.zeros(capacity * wd)
        M = np.zeros(capacity * m * m)
        nS = ctypes.c_int(0)
        _check(self.lib.lsp_get_tables(self._h, capacity, ctypes.byref(nS), S.ctypes.data,
                                       alpha.ctypes.data, C.ctypes.data, sigma.ctypes.data,
                                       g.ctypes.data, gam.ctypes.data, M.ctypes.data),
               "lsp_get_tables")
        k = nS.value
        W = 2 * self.t + 1
        return {
            "S": S[:k].copy(),
            "alpha": alpha[:k * m].reshape(k, m).copy(),
            "C": C[:k * m].reshape(k, m).copy(),
            "sigma_min": sigma[:k].copy(),
            "g": g[:k * wd].reshape((k,) + (W,) * self.d).copy(),
            "gamma": gam[:k * wd].reshape((k,) + (W,) * self.d).copy(),
            "M": M[:k * m * m].reshape(k, m, m).copy(),
        }


def _mlp_dims(path: str):
    """(n_in, n_hidden, n_out) from the header of a surrogate file (after the
    8-byte magic and the int32 version)."""
    import struct
    with open(path, "rb") as f:
        head = f.read(24)
    return struct.unpack("<3i", head[12:24])


class Batch:
    """Problems of uneven n set up and applied together (lsp_batch_*): one launch
    per setup stage over all of them, replayed as a HIP graph on a non-default
    stream. The problems must outlive the batch."""

    def __init__(self, problems):
        self.lib = load()
        self.problems = list(problems)
        arr = (ctypes.c_void_p * len(self.problems))(*[p._h.value for p in self.problems])
        h = ctypes.c_void_p()
        _check(self.lib.lsp_batch_create(len(self.problems), arr, ctypes.byref(h)),
               "lsp_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.lsp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stencil_setup(self, t: int, num_shifts, P_list, idx_list=None, precision: int = LSP_FP64):
        import torch
        cnt = len(self.problems)
        dt = torch.float32 if precision == LSP_FP32_REFINE else torch.float64
        ptrs = (ctypes.c_void_p * cnt)()
        iptrs = (ctypes.c_void_p * cnt)()
        for i, prob in enumerate(self.problems):
            m = (2 * t + 1) ** prob.d
            _need(P_list[i], dt, prob.N * m, f"P[{i}]")
            ptrs[i] = _ptr(P_list[i])
            if idx_list is not None and idx_list[i] is not None:
                _need(idx_list[i], torch.int32, prob.N, f"idx[{i}]")
                iptrs[i] = _ptr(idx_list[i])
            prob.t, prob.m = t, m
        ns = None
        if num_shifts is not None:
            ns = (ctypes.c_int * cnt)(*[int(x) for x in num_shifts])
        _check(self.lib.lsp_batch_stencil_setup(self._h, t, ns, precision, ptrs,
                                                iptrs if idx_list is not None else None),
               "lsp_batch_stencil_setup")

    def ps_apply(self, u_list, y_list):
        import torch
        cnt = len(self.problems)
        up = (ctypes.c_void_p * cnt)()
        yp = (ctypes.c_void_p * cnt)()
        for i, prob in enumerate(self.problems):
            _need(u_list[i], torch.complex128, prob.N, f"u[{i}]")
            _need(y_list[i], torch.complex128, prob.N, f"y[{i}]")
            up[i] = _ptr(u_list[i])
            yp[i] = _ptr(y_list[i])
        _check(self.lib.lsp_batch_ps_apply(self._h, up, yp), "lsp_batch_ps_apply")

    def set_tile(self, tile_width: int = 0):
        """lsp_batch_set_tile: fix the assembly tile width (16, 32, 64, 128,
        or 1 for the LDS-table form) of the following setups; 0 = tune."""
        _check(self.lib.lsp_batch_set_tile(self._h, int(tile_width)), "lsp_batch_set_tile")

    def tile(self):
        """(chosen assembly tile width, candidate widths, their mean ms)."""
        tw = ctypes.c_int(0)
        cand = (ctypes.c_int * 4)()
        ms = (ctypes.c_float * 4)()
        _check(self.lib.lsp_batch_tile(self._h, ctypes.byref(tw), cand, ms), "lsp_batch_tile")
        return tw.value, [c for c in cand if c], [float(ms[i]) for i in range(4) if cand[i]]


def stencil_setup_static(d: int, n: int, v, t: int, num_shifts: int, P, idx=None,
                         precision: int = LSP_FP64, stream=None):
    """lsp_stencil_setup_static: the setup of Problem.stencil_setup for a 2D
    potential v (device float64, N entries, read in place), allocating
    nothing: every intermediate lives in the library's fixed device array.
    Calls that overlap on one GPU race."""
    import torch
    lib = load()
    N = n ** d
    m = (2 * t + 1) ** d
    _need(v, torch.float64, N, "v")
    _need(P, torch.float32 if precision == LSP_FP32_REFINE else torch.float64, N * m, "P")
    if idx is not None:
        _need(idx, torch.int32, N, "idx")
    if stream is None:
        stream = torch.cuda.current_stream(v.device)
    _check(lib.lsp_stencil_setup_static(d, n, _ptr(v), t, num_shifts, precision, _ptr(P),
                                        _ptr(idx) if idx is not None else None,
                                        ctypes.c_void_p(stream.cuda_stream)),
           "lsp_stencil_setup_static")


def static_scratch_bytes() -> int:
    """Size of the fixed device array of lsp_stencil_setup_static (per GPU)."""
    return int(load().lsp_static_scratch_bytes())


def host_lu_solver(P_rows: np.ndarray, d: int, n: int, t: int):
    """Plain host-side sparse LU of P (the factorisation step stays on the host,
    outside the hot path). P_rows: (N, m) float64 rows from stencil_setup.
    Returns solve(rhs complex128 (N,)) -> complex128 (N,)."""
    import scipy.sparse
    import scipy.sparse.linalg
    N = n ** d
    m = (2 * t + 1) ** d
    cols = export_pattern(d, n, t)
    indptr = np.arange(0, N * m + 1, m)
    Pm = scipy.sparse.csr_matrix((P_rows.reshape(-1), cols.reshape(-1), indptr), shape=(N, N))
    lu = scipy.sparse.linalg.splu(Pm.tocsc().astype(np.complex128))
    return lu.solve


class MLP:
    """The learned-stencil surrogate (lsp_mlp_*): n_in -> n_hidden -> n_hidden
    -> n_out with SiLU, BF16 MFMA kernels, FP32 master weights and Adam."""

    def __init__(self, n_in: int, n_hidden: int, n_out: int, batch_rows: int = 8192,
                 stream=None):
        self.lib = load()
        self.n_in, self.n_hidden, self.n_out = n_in, n_hidden, n_out
        self.batch_rows = batch_rows
        h = ctypes.c_void_p()
        _check(self.lib.lsp_mlp_create(n_in, n_hidden, n_out, batch_rows,
                                       None if stream is None else stream, ctypes.byref(h)),
               "lsp_mlp_create")
        self._h = h
        self.num_params = self.lib.lsp_mlp_num_params(h)

    @classmethod
    def load(cls, path: str, batch_rows: int = 8192, stream=None) -> "MLP":
        """A network from a file written by save() (training state included)."""
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.lsp_mlp_load(os.fsencode(path), batch_rows, stream, ctypes.byref(h)),
               "lsp_mlp_load")
        obj = cls.__new__(cls)
        obj.lib = lib
        obj._h = h
        obj.batch_rows = batch_rows
        obj.num_params = lib.lsp_mlp_num_params(h)
        obj.n_in, obj.n_hidden, obj.n_out = _mlp_dims(path)
        return obj

    def save(self, path: str):
        _check(self.lib.lsp_mlp_save(self._h, os.fsencode(path)), "lsp_mlp_save")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.lsp_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat: np.ndarray):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        if a.size != self.num_params:
            raise ValueError(f"need {self.num_params} parameters, got {a.size}")
        _check(self.lib.lsp_mlp_set_params(self._h, a.ctypes.data), "lsp_mlp_set_params")

    def get_params(self) -> np.ndarray:
        a = np.empty(self.num_params, dtype=np.float32)
        _check(self.lib.lsp_mlp_get_params(self._h, a.ctypes.data), "lsp_mlp_get_params")
        return a

    def set_normalisation(self, mu_x, sd_x, mu_y, sd_y):
        a = np.ascontiguousarray(np.concatenate([mu_x, sd_x, mu_y, sd_y]), dtype=np.float32)
        _check(self.lib.lsp_mlp_set_normalisation(self._h, a.ctypes.data),
               "lsp_mlp_set_normalisation")

    def get_normalisation(self):
        a = np.empty(2 * (self.n_in + self.n_out), dtype=np.float32)
        _check(self.lib.lsp_mlp_get_normalisation(self._h, a.ctypes.data),
               "lsp_mlp_get_normalisation")
        i, o = self.n_in, self.n_out
        return a[:i], a[i:2 * i], a[2 * i:2 * i + o], a[2 * i + o:]

    def fit_normalisation(self, X, T):
        import torch
        rows = X.shape[0]
        _need(X, torch.float32, rows * self.n_in, "X")
        _need(T, torch.float32, rows * self.n_out, "T")
        _check(self.lib.lsp_mlp_fit_normalisation(self._h, _ptr(X), _ptr(T), rows),
               "lsp_mlp_fit_normalisation")

    def forward(self, X, Y):
        import torch
        rows = X.shape[0]
        _need(X, torch.float32, rows * self.n_in, "X")
        _need(Y, torch.float32, rows * self.n_out, "Y")
        _check(self.lib.lsp_mlp_forward(self._h, _ptr(X), rows, _ptr(Y)), "lsp_mlp_forward")

    def loss_grad(self, X, T):
        import torch
        rows = X.shape[0]
        _need(X, torch.float32, rows * self.n_in, "X")
        _need(T, torch.float32, rows * self.n_out, "T")
        g = np.empty(self.num_params, dtype=np.float32)
        loss = ctypes.c_double()
        _check(self.lib.lsp_mlp_loss_grad(self._h, _ptr(X), _ptr(T), rows, g.ctypes.data,
                                          ctypes.byref(loss)), "lsp_mlp_loss_grad")
        return loss.value, g

    def train_step(self, X, T, lr: float, want_loss: bool = False):
        import torch
        rows = X.shape[0]
        _need(X, torch.float32, rows * self.n_in, "X")
        _need(T, torch.float32, rows * self.n_out, "T")
        loss = ctypes.c_double()
        _check(self.lib.lsp_mlp_train_step(self._h, _ptr(X), _ptr(T), rows, lr,
                                           ctypes.byref(loss) if want_loss else None),
               "lsp_mlp_train_step")
        return loss.value if want_loss else None

