"""Python binding of libelocal (ctypes; argument marshalling only).

Every computation happens in the HIP library. PyTorch supplies device memory and
the current stream. Bitstrings are int64 tensors holding the uint64 words
(bit k of word k // 64 is spin-orbital k = 2p + s). If the library is not built or
cannot be loaded, every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libelocal.so")

FP64 = 0
BF16 = 1      # bfloat16 parameters; two fp16 terms per hidden activation
BF16X3 = 2    # bfloat16 parameters; three fp16 terms per hidden activation
OP_CONNECT, OP_EVAL, OP_GRAD = 0, 1, 2
NOALLOC_SCRATCH_MIB = 64   # ELOCAL_NOALLOC_SCRATCH_MIB of include/elocal.h

STATUS = {0: "OK", 1: "E_INVALID", 2: "E_CONFIG", 3: "E_WORKSPACE", 4: "E_NOMEM", 5: "E_DEVICE",
          6: "E_UNSUPPORTED"}


class ElocalError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"elocal {STATUS.get(status, status)}: {message}")
        self.status = status


class _Ansatz(ctypes.Structure):
    _fields_ = [("n_hidden", ctypes.c_int), ("widths", ctypes.POINTER(ctypes.c_int)),
                ("precision", ctypes.c_int), ("theta", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded library (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ElocalError(5, f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
        P = ctypes.POINTER
        L.elocal_create.argtypes = [vp, vp, i32, i32, i32, P(vp)]
        L.elocal_destroy.argtypes = [vp]
        L.elocal_num_connected.argtypes = [vp]
        L.elocal_num_connected.restype = i64
        L.elocal_words.argtypes = [vp]
        L.elocal_num_params.argtypes = [i32, i32, P(ctypes.c_int)]
        L.elocal_num_params.restype = i64
        L.elocal_workspace_bytes.argtypes = [vp, P(_Ansatz), i64, i32]
        L.elocal_workspace_bytes.restype = sz
        L.elocal_connect.argtypes = [vp, vp, vp, i64, vp, sz, vp, vp, vp, vp]
        L.elocal_eval.argtypes = [vp, vp, P(_Ansatz), vp, i64, vp, sz, vp, vp]
        L.elocal_stats.argtypes = [vp, vp, vp, i64, vp]
        L.elocal_eval_noalloc.argtypes = [vp, vp, P(_Ansatz), vp, i64, vp, vp]
        L.elocal_eval_noalloc.restype = ctypes.c_int
        L.elocal_grad.argtypes = [vp, vp, P(_Ansatz), vp, vp, vp, i64, vp, sz, vp, vp]
        L.elocal_check_samples.argtypes = [vp, vp, vp, i64, vp, sz, P(i64)]
        L.elocal_last_error.restype = ctypes.c_char_p
        L.elocal_timing_enable.argtypes = [vp, i32]
        L.elocal_kernel_timing.argtypes = [vp, P(ctypes.c_double), P(i64), i32]
        L.elocal_tune.argtypes = [vp, i32, i64]
        L.elocal_launch_info.argtypes = [vp, P(_Ansatz), i64, i32]
        L.elocal_launch_info.restype = i64
        L.elocal_sample_workspace_bytes.argtypes = [vp, P(_Ansatz), i64]
        L.elocal_sample_workspace_bytes.restype = sz
        L.elocal_sample.argtypes = [vp, vp, P(_Ansatz), i64, ctypes.c_uint64, i64, vp, sz, vp, vp, P(i64)]
        L.elocal_dedup_workspace_bytes.argtypes = [vp, P(_Ansatz), i64]
        L.elocal_dedup_workspace_bytes.restype = sz
        L.elocal_eval_dedup.argtypes = [vp, vp, P(_Ansatz), vp, i64, vp, sz, vp, vp, vp]
        L.elocal_pauli_build.argtypes = [vp, vp, vp]
        L.elocal_pauli_count.argtypes = [vp, i32]
        L.elocal_pauli_count.restype = i64
        L.elocal_pauli_workspace_bytes.argtypes = [vp, P(_Ansatz), i64]
        L.elocal_pauli_workspace_bytes.restype = sz
        L.elocal_eval_pauli.argtypes = [vp, vp, P(_Ansatz), vp, i64, vp, sz, vp]
        L.elocal_sector_dim.argtypes = [vp]
        L.elocal_sector_dim.restype = i64
        L.elocal_sector_workspace_bytes.argtypes = [vp, i32]
        L.elocal_sector_workspace_bytes.restype = sz
        L.elocal_sector_basis.argtypes = [vp, vp, vp]
        dbl = ctypes.c_double
        L.elocal_sector_apply.argtypes = [vp, vp, dbl, vp, dbl, vp, dbl, vp, vp, sz, vp]
        L.elocal_kpm_moments.argtypes = [vp, vp, vp, i64, dbl, dbl, vp, sz, vp]
        L.elocal_kpm_line_shape.argtypes = [vp, vp, i64, vp, i64, vp]
        L.elocal_workspace_bytes_multi.argtypes = [i32, P(vp), P(P(_Ansatz)), P(i64)]
        L.elocal_workspace_bytes_multi.restype = sz
        L.elocal_eval_multi.argtypes = [i32, P(vp), vp, P(P(_Ansatz)), P(vp), P(i64), vp, sz, P(vp), P(vp)]
        for f in ("elocal_create", "elocal_destroy", "elocal_connect", "elocal_eval", "elocal_stats",
                  "elocal_grad", "elocal_check_samples", "elocal_timing_enable", "elocal_kernel_timing", "elocal_tune",
                  "elocal_eval_multi", "elocal_sector_basis", "elocal_sector_apply", "elocal_kpm_moments",
                  "elocal_kpm_line_shape", "elocal_pauli_build", "elocal_eval_pauli", "elocal_eval_dedup", "elocal_sample"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def exported_symbols() -> Sequence[str]:
    return ["elocal_create", "elocal_destroy", "elocal_num_connected", "elocal_words", "elocal_num_params",
            "elocal_workspace_bytes", "elocal_connect", "elocal_eval", "elocal_stats", "elocal_grad",
            "elocal_check_samples", "elocal_timing_enable", "elocal_kernel_timing", "elocal_tune", "elocal_last_error",
            "elocal_workspace_bytes_multi", "elocal_eval_multi", "elocal_sector_dim",
            "elocal_sector_workspace_bytes", "elocal_sector_basis", "elocal_sector_apply", "elocal_kpm_moments",
            "elocal_kpm_line_shape", "elocal_pauli_build", "elocal_pauli_count", "elocal_pauli_workspace_bytes",
            "elocal_eval_pauli", "elocal_dedup_workspace_bytes", "elocal_eval_dedup", "elocal_sample_workspace_bytes",
            "elocal_sample", "elocal_eval_noalloc", "elocal_launch_info"]


def _check(status: int):
    if status != 0:
        raise ElocalError(status, lib().elocal_last_error().decode())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def num_params(n_orb: int, widths: Sequence[int]) -> int:
    w = (ctypes.c_int * len(widths))(*widths)
    p = lib().elocal_num_params(n_orb, len(widths), w)
    if p < 0:
        raise ElocalError(1, f"unsupported ansatz shape n={n_orb} widths={list(widths)}")
    return int(p)


class Ansatz:
    """Hidden widths + precision + a flat parameter tensor on the GPU."""

    def __init__(self, widths: Sequence[int], theta: torch.Tensor, precision: int):
        self.widths = tuple(int(w) for w in widths)
        self.precision = int(precision)
        if precision not in (FP64, BF16, BF16X3):
            raise ElocalError(1, f"unknown precision {precision}")
        want = torch.float64 if precision == FP64 else torch.bfloat16
        if theta.dtype != want or not theta.is_cuda or not theta.is_contiguous():
            raise ElocalError(1, f"theta must be a contiguous CUDA {want} tensor")
        self.theta = theta
        self._w = (ctypes.c_int * len(self.widths))(*self.widths)
        self._s = _Ansatz(len(self.widths), self._w, self.precision, ctypes.c_void_p(theta.data_ptr()))

    def ref(self):
        self._s.theta = ctypes.c_void_p(self.theta.data_ptr())
        return ctypes.byref(self._s)


class Hamiltonian:
    """A device-resident Hamiltonian for one (n_orb, n_alpha, n_beta) sector."""

    def __init__(self, h1e, eri, n_orb: int, n_alpha: int, n_beta: int):
        h1e = np.ascontiguousarray(np.asarray(h1e, dtype=np.float64))
        eri = np.ascontiguousarray(np.asarray(eri, dtype=np.float64))
        if h1e.size != n_orb * n_orb or eri.size != n_orb ** 4:
            raise ElocalError(1, "integral arrays do not match n_orb")
        self.n, self.na, self.nb = n_orb, n_alpha, n_beta
        h = ctypes.c_void_p()
        _check(lib().elocal_create(h1e.ctypes.data, eri.ctypes.data, n_orb, n_alpha, n_beta, ctypes.byref(h)))
        self._h = h
        self.C = int(lib().elocal_num_connected(h))
        self.W = int(lib().elocal_words(h))
        self._ws = {}
        self._h1e, self._eri = h1e, eri
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "_h", None):
            lib().elocal_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ workspace
    def workspace_bytes(self, op: int, B: int, ansatz: Optional[Ansatz] = None) -> int:
        ref = ansatz.ref() if ansatz is not None else None
        n = lib().elocal_workspace_bytes(self._h, ref, int(B), op)
        if n == 0:
            raise ElocalError(1, lib().elocal_last_error().decode())
        return int(n)

    def _workspace(self, op: int, B: int, ansatz: Optional[Ansatz] = None) -> Tuple[torch.Tensor, int]:
        need = self.workspace_bytes(op, B, ansatz)
        buf = self._ws.get(op)
        if buf is None or buf.numel() < need:
            buf = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws[op] = buf
        return buf, buf.numel()

    def _x(self, x: torch.Tensor) -> torch.Tensor:
        if x.dtype != torch.int64 or not x.is_cuda or x.dim() != 2 or x.shape[1] != self.W:
            raise ElocalError(1, f"x must be a CUDA int64 tensor [B, {self.W}]")
        return x.contiguous()

    # ------------------------------------------------------------------ calls
    def connect(self, x: torch.Tensor, out=None, stream=None):
        """(x' [B, C, W] int64, H [B, C] float64, sign [B, C] int8, exc [B, C] int32).

        `out` may supply those four tensors (preallocated, contiguous)."""
        x = self._x(x)
        B = x.shape[0]
        if out is None:
            xp = torch.empty((B, self.C, self.W), dtype=torch.int64, device=x.device)
            hv = torch.empty((B, self.C), dtype=torch.float64, device=x.device)
            sg = torch.empty((B, self.C), dtype=torch.int8, device=x.device)
            ex = torch.empty((B, self.C), dtype=torch.int32, device=x.device)
        else:
            xp, hv, sg, ex = out
            shapes = ((B, self.C, self.W), (B, self.C), (B, self.C), (B, self.C))
            dtypes = (torch.int64, torch.float64, torch.int8, torch.int32)
            for t, sh, dt in zip(out, shapes, dtypes):
                if tuple(t.shape) != sh or t.dtype != dt or not t.is_contiguous() or not t.is_cuda:
                    raise ElocalError(1, f"connect output must be a contiguous CUDA {dt} tensor of shape {sh}")
        ws, nb = self._workspace(OP_CONNECT, B)
        _check(lib().elocal_connect(self._h, _stream(stream), x.data_ptr(), B, ws.data_ptr(), nb,
                                    xp.data_ptr(), hv.data_ptr(), sg.data_ptr(), ex.data_ptr()))
        return xp, hv, sg, ex

    def eval(self, ansatz: Ansatz, x: torch.Tensor, out: Optional[torch.Tensor] = None,
             logpsi: Optional[torch.Tensor] = None, want_logpsi: bool = True, stream=None):
        """(eloc [B, 2] float64 (re, im), logpsi [B, 2] (A, phi) or None)."""
        x = self._x(x)
        B = x.shape[0]
        eloc = out if out is not None else torch.empty((B, 2), dtype=torch.float64, device=x.device)
        if want_logpsi and logpsi is None:
            logpsi = torch.empty((B, 2), dtype=torch.float64, device=x.device)
        ws, nb = self._workspace(OP_EVAL, B, ansatz)
        _check(lib().elocal_eval(self._h, _stream(stream), ansatz.ref(), x.data_ptr(), B, ws.data_ptr(), nb,
                                 eloc.data_ptr(), _ptr(logpsi) if want_logpsi else None))
        return eloc, logpsi

    def eval_noalloc(self, ansatz: Ansatz, x: torch.Tensor, out: Optional[torch.Tensor] = None,
                     logpsi: Optional[torch.Tensor] = None, stream=None):
        """elocal_eval_noalloc: eval with the library's fixed scratch instead of a workspace
        (outputs are the caller's; nothing else is allocated)."""
        x = self._x(x)
        B = x.shape[0]
        eloc = out if out is not None else torch.empty((B, 2), dtype=torch.float64, device=x.device)
        _check(lib().elocal_eval_noalloc(self._h, _stream(stream), ansatz.ref(), x.data_ptr(), B, eloc.data_ptr(),
                                         _ptr(logpsi)))
        return eloc, logpsi

    def grad(self, ansatz: Ansatz, x: torch.Tensor, w: torch.Tensor, eloc: torch.Tensor,
             stats: Optional[torch.Tensor] = None, dtheta: Optional[torch.Tensor] = None, stream=None):
        """(stats [4] = (Re<E>, Im<E>, var, sum w), dtheta [P] float64)."""
        x = self._x(x)
        B = x.shape[0]
        w = w.to(torch.float64).contiguous()
        eloc = eloc.contiguous()
        if stats is None:
            stats = torch.empty(4, dtype=torch.float64, device=x.device)
        if dtheta is None:
            dtheta = torch.empty(ansatz.theta.numel(), dtype=torch.float64, device=x.device)
        ws, nb = self._workspace(OP_GRAD, B, ansatz)
        _check(lib().elocal_grad(self._h, _stream(stream), ansatz.ref(), x.data_ptr(), w.data_ptr(),
                                 eloc.data_ptr(), B, ws.data_ptr(), nb, stats.data_ptr(), dtheta.data_ptr()))
        return stats, dtheta

    def timing(self, on: bool = True):
        """Record HIP events around the fused local-energy kernel of every eval."""
        _check(lib().elocal_timing_enable(self._h, int(on)))

    def kernel_time(self, reset: bool = True):
        """(summed milliseconds, launches) of the fused kernel since the last reset."""
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        _check(lib().elocal_kernel_timing(self._h, ctypes.byref(ms), ctypes.byref(n), int(reset)))
        return ms.value, int(n.value)

    def tune(self, grid: int = 0, groups: int = 0, waves: int = 0, cols: int = 0):
        """Launch shape of the fused kernel (0 = built-in): blocks, entry groups per work item,
        waves per block, 16-row tiles per network pass."""
        for param, value in enumerate((grid, groups, waves, cols)):
            _check(lib().elocal_tune(self._h, param, int(value)))

    def launch_info(self, ansatz: Ansatz, B: int) -> dict:
        """The launch shape elocal_eval would use for this ansatz and batch size."""
        keys = ("grid", "groups", "waves", "cols", "max_waves", "items", "lds_bytes", "inplace")
        out = {}
        for i, k in enumerate(keys):
            v = lib().elocal_launch_info(self._h, ansatz.ref(), int(B), i)
            if v < 0:
                raise ElocalError(1, lib().elocal_last_error().decode())
            out[k] = int(v)
        return out

    # ------------------------------------------------------------------ sampling
    def sample(self, ansatz: Ansatz, n_samples: int, seed: int, max_unique: int = 1 << 20, stream=None):
        """BAS draws from |Psi|^2: (distinct determinants [U, W] int64, counts [U] int64)."""
        need = int(lib().elocal_sample_workspace_bytes(self._h, ansatz.ref(), int(max_unique)))
        if need == 0:
            raise ElocalError(1, lib().elocal_last_error().decode())
        ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        x = torch.empty((int(max_unique), self.W), dtype=torch.int64, device=self.device)
        c = torch.empty(int(max_unique), dtype=torch.int64, device=self.device)
        u = ctypes.c_int64(0)
        _check(lib().elocal_sample(self._h, _stream(stream), ansatz.ref(), int(n_samples), ctypes.c_uint64(seed),
                                   int(max_unique), ws.data_ptr(), need, x.data_ptr(), c.data_ptr(), ctypes.byref(u)))
        return x[:u.value], c[:u.value]

    # ------------------------------------------------------------------ deduplicated eval
    def eval_dedup(self, ansatz: Ansatz, x: torch.Tensor, out: Optional[torch.Tensor] = None,
                   want_logpsi: bool = False, stream=None):
        """(eloc [B, 2], logpsi [B, 2] or None, distinct-determinant count (device int64 [1]))."""
        x = self._x(x)
        B = x.shape[0]
        eloc = out if out is not None else torch.empty((B, 2), dtype=torch.float64, device=x.device)
        lp = torch.empty((B, 2), dtype=torch.float64, device=x.device) if want_logpsi else None
        cnt = torch.zeros(1, dtype=torch.int64, device=x.device)
        need = int(lib().elocal_dedup_workspace_bytes(self._h, ansatz.ref(), B))
        if need == 0:
            raise ElocalError(1, lib().elocal_last_error().decode())
        buf = self._ws.get("dedup")
        if buf is None or buf.numel() < need:
            buf = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws["dedup"] = buf
        _check(lib().elocal_eval_dedup(self._h, _stream(stream), ansatz.ref(), x.data_ptr(), B, buf.data_ptr(),
                                       buf.numel(), eloc.data_ptr(), _ptr(lp), cnt.data_ptr()))
        return eloc, lp, cnt

    # ------------------------------------------------------------------ Pauli-string route
    def pauli_build(self):
        """Jordan--Wigner strings of this Hamiltonian, grouped by flip mask (host, synchronous)."""
        _check(lib().elocal_pauli_build(self._h, self._h1e.ctypes.data, self._eri.ctypes.data))
        return int(lib().elocal_pauli_count(self._h, 0)), int(lib().elocal_pauli_count(self._h, 1))

    def eval_pauli(self, ansatz: Ansatz, x: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        """E_loc [B, 2] through the Pauli-string route (after pauli_build)."""
        x = self._x(x)
        B = x.shape[0]
        eloc = out if out is not None else torch.empty((B, 2), dtype=torch.float64, device=x.device)
        need = int(lib().elocal_pauli_workspace_bytes(self._h, ansatz.ref(), B))
        if need == 0:
            raise ElocalError(2, lib().elocal_last_error().decode())
        buf = self._ws.get("pauli")
        if buf is None or buf.numel() < need:
            buf = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws["pauli"] = buf
        _check(lib().elocal_eval_pauli(self._h, _stream(stream), ansatz.ref(), x.data_ptr(), B, buf.data_ptr(),
                                       buf.numel(), eloc.data_ptr()))
        return eloc

    # ------------------------------------------------------------------ full sector / KPM
    @property
    def sector_dim(self) -> int:
        return int(lib().elocal_sector_dim(self._h))

    def _sector_ws(self, kpm: bool) -> Tuple[torch.Tensor, int]:
        need = int(lib().elocal_sector_workspace_bytes(self._h, int(kpm)))
        if need == 0:
            raise ElocalError(6, lib().elocal_last_error().decode())
        key = "sector_kpm" if kpm else "sector"
        buf = self._ws.get(key)
        if buf is None or buf.numel() < need:
            buf = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws[key] = buf
        return buf, buf.numel()

    def sector_basis(self, stream=None) -> torch.Tensor:
        """Every determinant of the sector, [dim, W] int64 (row r = index r)."""
        if self.sector_dim < 0:
            raise ElocalError(6, "sector dimension exceeds 2^31 - 1")
        x = torch.empty((self.sector_dim, self.W), dtype=torch.int64, device=self.device)
        _check(lib().elocal_sector_basis(self._h, _stream(stream), x.data_ptr()))
        return x

    def sector_apply(self, v: torch.Tensor, ch: float = 1.0, cv: float = 0.0, z: Optional[torch.Tensor] = None,
                     cz: float = 0.0, out: Optional[torch.Tensor] = None, dots: bool = False, stream=None):
        """y = ch H v + cv v + cz z over the sector; with dots, also (<y|y>, <y|v>)."""
        dim = self.sector_dim
        for t in (v, z):
            if t is not None and (t.dtype != torch.float64 or not t.is_cuda or t.numel() != dim or not t.is_contiguous()):
                raise ElocalError(1, f"sector vectors must be contiguous CUDA float64 of {dim} entries")
        y = out if out is not None else torch.empty(dim, dtype=torch.float64, device=v.device)
        d = torch.empty(2, dtype=torch.float64, device=v.device) if dots else None
        ws, nb = self._sector_ws(False)
        _check(lib().elocal_sector_apply(self._h, _stream(stream), float(ch), v.data_ptr(), float(cv), _ptr(z),
                                         float(cz), y.data_ptr(), ws.data_ptr(), nb, _ptr(d)))
        return (y, d) if dots else y

    def kpm_moments(self, alpha: torch.Tensor, n_moments: int, a: float, b: float, stream=None) -> torch.Tensor:
        """Chebyshev moments Omega_0..Omega_{N-1} of alpha for H~ = (H - b) / a."""
        if alpha.dtype != torch.float64 or not alpha.is_cuda or alpha.numel() != self.sector_dim:
            raise ElocalError(1, "alpha must be a CUDA float64 sector vector")
        mu = torch.empty(int(n_moments), dtype=torch.float64, device=alpha.device)
        ws, nb = self._sector_ws(True)
        _check(lib().elocal_kpm_moments(self._h, _stream(stream), alpha.contiguous().data_ptr(), int(n_moments),
                                        float(a), float(b), ws.data_ptr(), nb, mu.data_ptr()))
        return mu

    def check_samples(self, x: torch.Tensor, stream=None) -> int:
        x = self._x(x)
        ws = torch.empty(8, dtype=torch.uint8, device=x.device)
        bad = ctypes.c_int64(0)
        st = lib().elocal_check_samples(self._h, _stream(stream), x.data_ptr(), x.shape[0], ws.data_ptr(), 8,
                                        ctypes.byref(bad))
        if st not in (0, 2):
            _check(st)
        return int(bad.value)


MAX_SYSTEMS = 16


def kpm_line_shape(moments: torch.Tensor, w: torch.Tensor, stream=None) -> torch.Tensor:
    """Jackson-damped line shape rho(w~) from the moments, at points w~ in (-1, 1)."""
    moments = moments.to(torch.float64).contiguous()
    w = w.to(torch.float64).contiguous()
    rho = torch.empty_like(w)
    _check(lib().elocal_kpm_line_shape(_stream(stream), moments.data_ptr(), moments.numel(), w.data_ptr(),
                                       w.numel(), rho.data_ptr()))
    return rho


class MultiEval:
    """Local energies of several systems in one persistent launch (elocal_eval_multi).

    Holds the workspace between calls; every system keeps its own Hamiltonian handle,
    ansatz and samples.
    """

    def __init__(self):
        self._ws = None

    @staticmethod
    def _arrays(hams: Sequence[Hamiltonian], ansatze: Sequence[Ansatz], xs: Sequence[torch.Tensor]):
        k = len(hams)
        if not (1 <= k <= MAX_SYSTEMS) or len(ansatze) != k or len(xs) != k:
            raise ElocalError(1, f"need 1..{MAX_SYSTEMS} systems with one ansatz and one x each")
        hs = (ctypes.c_void_p * k)(*[h._h for h in hams])
        for a in ansatze:
            a.ref()   # refresh the theta pointer
        ap = (ctypes.POINTER(_Ansatz) * k)(*[ctypes.pointer(a._s) for a in ansatze])
        xs = [h._x(x) for h, x in zip(hams, xs)]
        B = (ctypes.c_int64 * k)(*[x.shape[0] for x in xs])
        return k, hs, ap, xs, B

    def workspace_bytes(self, hams, ansatze, xs) -> int:
        k, hs, ap, xs, B = self._arrays(hams, ansatze, xs)
        n = lib().elocal_workspace_bytes_multi(k, hs, ap, B)
        if n == 0:
            raise ElocalError(1, lib().elocal_last_error().decode())
        return int(n)

    def __call__(self, hams: Sequence[Hamiltonian], ansatze: Sequence[Ansatz], xs: Sequence[torch.Tensor],
                 outs: Optional[Sequence[torch.Tensor]] = None, want_logpsi: bool = False, stream=None):
        """([eloc_s [B_s, 2]], [logpsi_s [B_s, 2]] or None)."""
        k, hs, ap, xs, B = self._arrays(hams, ansatze, xs)
        need = lib().elocal_workspace_bytes_multi(k, hs, ap, B)
        if need == 0:
            raise ElocalError(1, lib().elocal_last_error().decode())
        dev = xs[0].device
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=dev)
        if outs is None:
            outs = [torch.empty((x.shape[0], 2), dtype=torch.float64, device=dev) for x in xs]
        lps = [torch.empty((x.shape[0], 2), dtype=torch.float64, device=dev) for x in xs] if want_logpsi else None
        xp = (ctypes.c_void_p * k)(*[x.data_ptr() for x in xs])
        ep = (ctypes.c_void_p * k)(*[o.data_ptr() for o in outs])
        lp = (ctypes.c_void_p * k)(*[t.data_ptr() for t in lps]) if lps is not None else None
        _check(lib().elocal_eval_multi(k, hs, _stream(stream), ap, xp, B, self._ws.data_ptr(), self._ws.numel(),
                                       ep, lp))
        return list(outs), lps


def stats(eloc: torch.Tensor, w: torch.Tensor, stream=None) -> torch.Tensor:
    out = torch.empty(4, dtype=torch.float64, device=eloc.device)
    w = w.to(torch.float64).contiguous()
    _check(lib().elocal_stats(_stream(stream), eloc.contiguous().data_ptr(), w.data_ptr(), eloc.shape[0],
                              out.data_ptr()))
    return out


class ElocEnergy(torch.autograd.Function):
    """Forward: Re<E> over the batch (local energies from the HIP library).

    Backward: grad_output times the VMC gradient 2 Re <(E_loc - <E>) d log Psi*> --
    the variational-energy gradient estimator, not the derivative of the
    fixed-sample mean (the samples themselves depend on theta).

    ``theta`` holds the parameters in the caller's (master) precision: float64 or
    float32 for a master copy, or bfloat16. In the BF16 modes the forward evaluates the
    ansatz at theta rounded to bfloat16 (FP32 then round-to-nearest-even); the backward
    returns the library's FP64 gradient in theta's dtype, so a float64 master copy gets
    it unrounded (a bfloat16 theta gets it rounded to bfloat16).

    Usage: ``E = ElocEnergy.apply(theta, ham, widths, precision, x, w)``.
    """

    @staticmethod
    def forward(ctx, theta, ham: Hamiltonian, widths, precision, x, w):
        th = theta.detach()
        if precision == FP64:
            th = th.to(torch.float64)
        elif th.dtype != torch.bfloat16:
            th = th.to(torch.float32).to(torch.bfloat16)
        ans = Ansatz(widths, th.contiguous(), precision)
        eloc, _ = ham.eval(ans, x, want_logpsi=False)
        st = stats(eloc, w)
        ctx.ham, ctx.ans = ham, ans
        ctx.save_for_backward(x, w, eloc)
        ctx.stats = st
        ctx.theta_dtype = theta.dtype
        return st[0].clone()

    @staticmethod
    def backward(ctx, g):
        x, w, eloc = ctx.saved_tensors
        _, dtheta = ctx.ham.grad(ctx.ans, x, w, eloc)
        return (g.to(torch.float64) * dtheta).to(ctx.theta_dtype), None, None, None, None, None
