"""Thin ctypes binding of the C ABI in include/rbmf.h (argument marshalling
only: every step of the search runs in the HIP library).

Arrays may be numpy arrays (host) or torch tensors (host or device); device
tensors are passed by pointer and stay on the GPU.  The library fails loudly
if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import inspect
import os
from typing import Callable, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librbmf.so")

RB_OK, RB_ERR_ARG, RB_ERR_OOM, RB_ERR_DEVICE, RB_ERR_CAPACITY, RB_ERR_NUMERIC, RB_ERR_UNSUPPORTED, \
    RB_ERR_CALLBACK = range(8)
RB_F32, RB_BF16, RB_F16, RB_BF16X3 = 0, 1, 2, 3
RB_STAGE2_FULL, RB_STAGE2_SPARSE, RB_STAGE2_AUTO, RB_STAGE2_RECON = 0, 1, 2, 3
RB_EIG_SUBSPACE, RB_EIG_LANCZOS = 0, 1
RB_OPT_FP16_INTERMEDIATE = 1   # rb_filter_opts.flags
SOLVERS = {"subspace": RB_EIG_SUBSPACE, "lanczos": RB_EIG_LANCZOS}
DTYPES = {"f32": RB_F32, "bf16": RB_BF16, "f16": RB_F16, "bf16x3": RB_BF16X3}

FUNCTIONS = ["rb_ctx_create", "rb_ctx_destroy", "rb_last_error", "rb_bank_create", "rb_bank_free",
             "rb_bank_info", "rb_build_basis", "rb_build_basis_range", "rb_build_basis_solver", "rb_basis_info",
             "rb_basis_free", "rb_basis_export", "rb_filter", "rb_filter_stream", "rb_filter_batch", "mf_full",
             "mf_full_noalloc", "rb_rho_at", "rb_backward", "rb_refine", "rb_cluster_peaks", "rb_debug_rho",
             "rb_debug_rho_binned", "rb_debug_basis_outputs", "rb_nonuniform_freqs", "rb_build_basis_nonuniform"]


class Grid(C.Structure):
    _fields_ = [("N", C.c_int64), ("fs", C.c_double), ("f_low", C.c_double)]


class Trigger(C.Structure):
    _fields_ = [("tmpl", C.c_int32), ("sample", C.c_int32), ("snr", C.c_float), ("phase", C.c_float)]


class Peak(C.Structure):
    _fields_ = [("snr", C.c_float), ("sample", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_stage1", C.c_int64), ("n_refiltered", C.c_int32), ("rank", C.c_int32),
                ("ms", C.c_float * 8), ("n_bins", C.c_int64), ("min_energy", C.c_double),
                ("gemm_mfma_flop", C.c_double)]


class FilterOpts(C.Structure):
    _fields_ = [("thr1", C.c_double), ("thr2", C.c_double), ("stage2", C.c_int32),
                ("bin_w", C.c_int32), ("thr_bin", C.c_double), ("bin_source", C.c_int32),
                ("flags", C.c_int32)]


TRIGGER_NP = np.dtype([("tmpl", np.int32), ("sample", np.int32), ("snr", np.float32),
                       ("phase", np.float32)])
PEAK_NP = np.dtype([("snr", np.float32), ("sample", np.int32)])

FILL_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_int64,
                      C.POINTER(C.c_double))
FILL_AT_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_int64,
                         C.POINTER(C.c_double))

_lib = None


class RbError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: run __graft_entry__.build() "
                               "(or python -m paper_2110_13115_amd.build) first")
        # torch first: it brings its own HIP runtime, and the library must bind
        # to that one (loaded first, the system runtime would be the one torch
        # finds, and device discovery fails in the mixed process)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.rb_ctx_create.argtypes = [C.c_int, vp, C.POINTER(vp)]
        L.rb_ctx_destroy.argtypes = [vp]
        L.rb_last_error.restype = C.c_char_p
        L.rb_bank_create.argtypes = [vp, C.POINTER(Grid), vp, i32, FILL_FN, vp, C.POINTER(vp)]
        L.rb_bank_free.argtypes = [vp]
        L.rb_bank_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i64), C.POINTER(i64), vp]
        L.rb_build_basis.argtypes = [vp, vp, i32, dbl, C.c_int, C.POINTER(vp), C.POINTER(i32),
                                     C.POINTER(dbl)]
        L.rb_build_basis_range.argtypes = [vp, vp, i32, i32, i32, dbl, C.c_int, C.POINTER(vp),
                                           C.POINTER(i32), C.POINTER(dbl)]
        L.rb_build_basis_solver.argtypes = [vp, vp, i32, i32, i32, dbl, C.c_int, i32, C.POINTER(vp),
                                            C.POINTER(i32), C.POINTER(dbl)]
        L.rb_basis_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(dbl)]
        L.rb_basis_free.argtypes = [vp]
        L.rb_basis_export.argtypes = [vp, vp, vp, vp]
        L.rb_filter.argtypes = [vp, C.POINTER(vp), i32, vp, vp, C.POINTER(FilterOpts), vp, i64,
                                C.POINTER(i64), vp, C.POINTER(Stats)]
        L.mf_full.argtypes = [vp, vp, vp, dbl, vp, i64, C.POINTER(i64), vp, C.POINTER(Stats)]
        L.mf_full_noalloc.argtypes = [vp, vp, vp, dbl, vp, i64, C.POINTER(i64)]
        L.rb_filter_stream.argtypes = [vp, C.POINTER(vp), i32, vp, vp, i64, C.POINTER(FilterOpts), vp, i64,
                                       C.POINTER(i64), C.POINTER(Stats)]
        L.rb_filter_batch.argtypes = [vp, i32, vp, C.POINTER(FilterOpts), i32, vp, i64, C.POINTER(i64),
                                      C.POINTER(Stats)]
        L.rb_rho_at.argtypes = [vp, vp, vp, vp, i64, vp, vp]
        L.rb_backward.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp, vp, C.POINTER(dbl)]
        L.rb_refine.argtypes = [vp, vp, vp, vp, i64, i32, i32, vp, vp, vp]
        L.rb_cluster_peaks.argtypes = [vp, vp, i64, i32, i64, vp]
        L.rb_debug_rho.argtypes = [vp, vp, vp, vp, vp]
        L.rb_debug_rho_binned.argtypes = [vp, vp, vp, i32, vp]
        L.rb_debug_basis_outputs.argtypes = [vp, vp, vp, vp]
        L.rb_nonuniform_freqs.argtypes = [vp, vp, i64, i32, dbl, vp, i64, vp, i64, C.POINTER(i64)]
        L.rb_build_basis_nonuniform.argtypes = [vp, vp, i32, i32, vp, i64, vp, FILL_AT_FN, vp, i32, dbl,
                                                C.c_int, C.POINTER(vp), C.POINTER(i32), C.POINTER(dbl)]
        for f in FUNCTIONS:
            if f != "rb_last_error":
                getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(st: int, where: str):
    if st != RB_OK:
        raise RbError(st, where, lib().rb_last_error().decode())


def _ptr(x) -> Optional[int]:
    """Raw pointer of a numpy array or torch tensor (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr()
    raise TypeError(f"unsupported array type {type(x)}")


def current_stream_handle() -> Optional[int]:
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


class Context:
    def __init__(self, device: int = 0, stream: Optional[int] = None):
        self.h = C.c_void_p()
        if stream is None:
            stream = current_stream_handle()
        _check(lib().rb_ctx_create(device, stream, C.byref(self.h)), "rb_ctx_create")

    def close(self):
        if self.h:
            _check(lib().rb_ctx_destroy(self.h), "rb_ctx_destroy")
            self.h = C.c_void_p()


class Bank:
    """Whitened unit-norm bank on the device.  fill(t0, t1, k0, k1) must return
    the complex128 templates [t0, t1) on rfft bins [k0, k1)."""

    def __init__(self, ctx: Context, N: int, fs: float, f_low: float, psd: np.ndarray, T: int,
                 fill: Callable[[int, int, int, int], np.ndarray]):
        self.ctx, self.N, self.fs, self.f_low, self.T = ctx, int(N), float(fs), float(f_low), int(T)
        self.h = C.c_void_p()
        psd = np.ascontiguousarray(psd, dtype=np.float64)
        self._err = None

        try:
            in_place = "out" in inspect.signature(fill).parameters
        except (TypeError, ValueError):
            in_place = False

        def cb(user, t0, t1, k0, k1, out):
            try:
                n = (t1 - t0) * (k1 - k0)
                dst = np.ctypeslib.as_array(out, shape=(2 * n,))
                if in_place:    # the generator writes the library's staging buffer itself
                    fill(int(t0), int(t1), int(k0), int(k1), out=dst.view(np.complex128).reshape(t1 - t0, k1 - k0))
                    return 0
                a = np.asarray(fill(int(t0), int(t1), int(k0), int(k1)), dtype=np.complex128)
                dst[:] = a.reshape(-1).view(np.float64)
                return 0
            except Exception as e:        # reported after the call returns
                self._err = e
                return 1

        self._cb = FILL_FN(cb)
        g = Grid(self.N, self.fs, self.f_low)
        st = lib().rb_bank_create(ctx.h, C.byref(g), _ptr(psd), self.T, self._cb, None, C.byref(self.h))
        if self._err is not None:
            raise self._err
        _check(st, "rb_bank_create")

    def info(self) -> Tuple[int, int, int, np.ndarray]:
        T = C.c_int32()
        klo, khi = C.c_int64(), C.c_int64()
        sig = np.empty(self.T, dtype=np.float64)
        _check(lib().rb_bank_info(self.h, C.byref(T), C.byref(klo), C.byref(khi), _ptr(sig)),
               "rb_bank_info")
        return T.value, klo.value, khi.value, sig

    def close(self):
        if self.h:
            _check(lib().rb_bank_free(self.h), "rb_bank_free")
            self.h = C.c_void_p()


class Basis:
    """Reduced basis of templates [t0, t1) of a bank (default: the whole bank)."""

    def __init__(self, ctx: Context, bank: Bank, rank: int = 0, tol: float = 1e-3, dtype="f32",
                 t0: int = 0, t1: Optional[int] = None, solver: str = "subspace"):
        self.ctx, self.bank = ctx, bank
        self.t0 = int(t0)
        self.t1 = bank.T if t1 is None else int(t1)
        self.T = self.t1 - self.t0
        self.h = C.c_void_p()
        K = C.c_int32()
        e = C.c_double()
        dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        _check(lib().rb_build_basis_solver(ctx.h, bank.h, self.t0, self.t1, int(rank), float(tol), dt,
                                           SOLVERS[solver], C.byref(self.h), C.byref(K), C.byref(e)),
               "rb_build_basis_solver")
        self.K, self.energy, self.dtype = K.value, e.value, dt

    @classmethod
    def nonuniform(cls, ctx: Context, bank: Bank, nodes: np.ndarray, psd_nodes: np.ndarray,
                   fill_at: Callable[[int, int, np.ndarray], np.ndarray], rank: int = 0, tol: float = 1e-3,
                   dtype="f32", t0: int = 0, t1: Optional[int] = None) -> "Basis":
        """Basis by PCA on the non-uniform frequency set `nodes`, interpolated
        onto the bank's grid (rb_build_basis_nonuniform).  fill_at(t0, t1, f)
        must return the complex128 templates [t0, t1) at the frequencies f."""
        self = cls.__new__(cls)
        self.ctx, self.bank = ctx, bank
        self.t0 = int(t0)
        self.t1 = bank.T if t1 is None else int(t1)
        self.T = self.t1 - self.t0
        self.h = C.c_void_p()
        nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        psd_nodes = np.ascontiguousarray(psd_nodes, dtype=np.float64)
        err = []

        def cb(user, a, b, f, nf, out):
            try:
                fr = np.ctypeslib.as_array(f, shape=(nf,)).copy()
                h = np.asarray(fill_at(int(a), int(b), fr), dtype=np.complex128)
                dst = np.ctypeslib.as_array(out, shape=(2 * (b - a) * nf,))
                dst[:] = h.reshape(-1).view(np.float64)
                return 0
            except Exception as e:        # reported after the call returns
                err.append(e)
                return 1

        fn = FILL_AT_FN(cb)
        K = C.c_int32()
        e = C.c_double()
        dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        st = lib().rb_build_basis_nonuniform(ctx.h, bank.h, self.t0, self.t1, _ptr(nodes), nodes.shape[0],
                                             _ptr(psd_nodes), fn, None, int(rank), float(tol), dt,
                                             C.byref(self.h), C.byref(K), C.byref(e))
        if err:
            raise err[0]
        _check(st, "rb_build_basis_nonuniform")
        self.K, self.energy, self.dtype = K.value, e.value, dt
        return self

    def export(self):
        _, klo, khi, _ = self.bank.info()
        nb = khi - klo + 1
        V = np.empty((self.K, nb), dtype=np.complex128)
        c = np.empty((self.T, self.K), dtype=np.complex128)
        lam = np.empty(self.K, dtype=np.float64)
        _check(lib().rb_basis_export(self.h, _ptr(V), _ptr(c), _ptr(lam)), "rb_basis_export")
        return V, c, lam

    def close(self):
        if self.h:
            _check(lib().rb_basis_free(self.h), "rb_basis_free")
            self.h = C.c_void_p()


def nonuniform_freqs(f: np.ndarray, h_re: np.ndarray, per_bin: int = 5, df_min: float = 1.0 / 128,
                     extra: Optional[np.ndarray] = None) -> np.ndarray:
    """The non-uniform frequency set (rb_nonuniform_freqs) from samples of a
    reference template's real part."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    h_re = np.ascontiguousarray(h_re, dtype=np.float64)
    ex = None if extra is None else np.ascontiguousarray(extra, dtype=np.float64)
    n_ex = 0 if ex is None else ex.shape[0]
    n = C.c_int64()
    st = lib().rb_nonuniform_freqs(_ptr(f), _ptr(h_re), f.shape[0], int(per_bin), float(df_min), _ptr(ex), n_ex,
                                   None, 0, C.byref(n))
    if st != RB_ERR_CAPACITY:
        _check(st, "rb_nonuniform_freqs")
    out = np.empty(max(1, n.value), dtype=np.float64)
    _check(lib().rb_nonuniform_freqs(_ptr(f), _ptr(h_re), f.shape[0], int(per_bin), float(df_min), _ptr(ex), n_ex,
                                     _ptr(out), out.shape[0], C.byref(n)), "rb_nonuniform_freqs")
    return out[:n.value].copy()


def _triggers_out(cap: int, like_device: bool):
    if like_device:
        import torch
        return torch.empty((max(cap, 1), 4), dtype=torch.int32, device="cuda")
    return np.empty(max(cap, 1), dtype=TRIGGER_NP)


def _as_np_triggers(buf, n: int) -> np.ndarray:
    if isinstance(buf, np.ndarray):
        return buf[:n].copy()
    return buf[:n].cpu().numpy().view(TRIGGER_NP).reshape(-1)


def subbank_bases(ctx: Context, bank: Bank, bounds, rank=0, tol: float = 1e-3, dtype="f32", solver="subspace"):
    """One basis per sub-bank; bounds = [0, b1, ..., T]; rank an int or a list."""
    ranks = rank if isinstance(rank, (list, tuple)) else [rank] * (len(bounds) - 1)
    return [Basis(ctx, bank, rank=r, tol=tol, dtype=dtype, t0=a, t1=b, solver=solver)
            for a, b, r in zip(bounds[:-1], bounds[1:], ranks)]


def rb_filter(ctx: Context, bases, bank: Bank, strain, thr1: float, thr2: float,
              stage2: int = RB_STAGE2_FULL, cap: int = 1 << 20, peaks: bool = False,
              out=None, bin_w: int = 0, thr_bin: float = 0.0, bin_source: int = 0, flags: int = 0):
    """bases: one Basis or a list partitioning the bank.  bin_w >= 2 selects the
    binned first stage with threshold thr_bin on the averaged SNR, taken from
    the basis (bin_source 0) or from the templates (bin_source 1).  flags:
    RB_OPT_FP16_INTERMEDIATE or 0.  Returns (triggers as a TRIGGER_NP array,
    or their count when `out` is a device buffer; peaks or None; Stats)."""
    if isinstance(bases, Basis):
        bases = [bases]
    arr = (C.c_void_p * len(bases))(*[b.h.value for b in bases])
    o = FilterOpts(thr1, thr2, stage2, int(bin_w), float(thr_bin), int(bin_source), int(flags))
    dev = out is not None and not isinstance(out, np.ndarray)
    buf = out if out is not None else _triggers_out(cap, False)
    cap = buf.shape[0]
    n = C.c_int64()
    pk = np.empty(bank.T, dtype=PEAK_NP) if peaks else None
    st = Stats()
    _check(lib().rb_filter(ctx.h, arr, len(bases), bank.h, _ptr(strain), C.byref(o), _ptr(buf), cap,
                           C.byref(n), _ptr(pk), C.byref(st)), "rb_filter")
    return _as_np_triggers(buf, n.value) if not dev else n.value, pk, st


def rb_filter_stream(ctx: Context, bases, bank: Bank, strain, thr1: float, thr2: float,
                     stage2: int = RB_STAGE2_FULL, cap: int = 1 << 20, bin_w: int = 0, thr_bin: float = 0.0,
                     bin_source: int = 0):
    """Overlap-save search of a strain longer than the bank's segment.
    Returns (TRIGGER_NP array with stream samples, Stats)."""
    if isinstance(bases, Basis):
        bases = [bases]
    arr = (C.c_void_p * len(bases))(*[b.h.value for b in bases])
    o = FilterOpts(thr1, thr2, stage2, int(bin_w), float(thr_bin), int(bin_source), 0)
    buf = _triggers_out(cap, False)
    n = C.c_int64()
    st = Stats()
    _check(lib().rb_filter_stream(ctx.h, arr, len(bases), bank.h, _ptr(strain), int(strain.shape[0]), C.byref(o),
                                  _ptr(buf), buf.shape[0], C.byref(n), C.byref(st)), "rb_filter_stream")
    return _as_np_triggers(buf, n.value), st


def mf_full(ctx: Context, bank: Bank, strain, thr: float, cap: int = 1 << 20, peaks: bool = False,
            out=None):
    dev = out is not None and not isinstance(out, np.ndarray)
    buf = out if out is not None else _triggers_out(cap, False)
    cap = buf.shape[0]
    n = C.c_int64()
    pk = np.empty(bank.T, dtype=PEAK_NP) if peaks else None
    st = Stats()
    _check(lib().mf_full(ctx.h, bank.h, _ptr(strain), float(thr), _ptr(buf), cap, C.byref(n), _ptr(pk),
                         C.byref(st)), "mf_full")
    return _as_np_triggers(buf, n.value) if not dev else n.value, pk, st


def mf_full_noalloc(ctx: Context, bank: Bank, strain, thr: float, out):
    """mf_full on the library's fixed device scratch: strain and out (cap x 4
    int32, rb_trigger records) are device tensors; returns the trigger count."""
    n = C.c_int64()
    _check(lib().mf_full_noalloc(ctx.h, bank.h, _ptr(strain), float(thr), _ptr(out), out.shape[0], C.byref(n)),
           "mf_full_noalloc")
    return n.value


def _trig_arg(S):
    if isinstance(S, np.ndarray):
        return np.ascontiguousarray(S, dtype=TRIGGER_NP)
    return S          # device tensor of rb_trigger records (n x 4 int32)


def rho_at(ctx: Context, basis: Basis, strain, S, coeffs=None, out=None):
    """First-stage rho at trigger points (complex64, host array or `out`);
    coeffs: T x K complex64 replacing the basis's conj(c), or None."""
    S = _trig_arg(S)
    n = S.shape[0]
    rho = out if out is not None else np.empty(n, dtype=np.complex64)
    _check(lib().rb_rho_at(ctx.h, basis.h, _ptr(strain), _ptr(S), n, _ptr(coeffs), _ptr(rho)),
           "rb_rho_at")
    return rho


def rb_backward(ctx: Context, basis: Basis, strain, S, seed=None, coeffs=None, want_C=True,
                want_strain=True, grad_C=None, grad_strain=None):
    """Returns (loss, grad_C (basis.T x K complex64, the basis's rows) or None,
    grad_strain (N) or None).
    Outputs are host arrays unless device buffers are passed in."""
    S = _trig_arg(S)
    n = S.shape[0]
    gC = grad_C if grad_C is not None else (
        np.zeros((basis.T, basis.K), dtype=np.complex64) if want_C else None)
    gs = grad_strain if grad_strain is not None else (
        np.zeros(basis.bank.N, dtype=np.float32) if want_strain else None)
    loss = C.c_double()
    sd = seed
    if isinstance(seed, np.ndarray) or isinstance(seed, (list, tuple)):
        sd = np.ascontiguousarray(seed, dtype=np.float32)
    _check(lib().rb_backward(ctx.h, basis.h, _ptr(strain), _ptr(S), _ptr(sd), n, _ptr(coeffs),
                             _ptr(gC), _ptr(gs), C.byref(loss)), "rb_backward")
    return loss.value, gC, gs


def refine(ctx: Context, basis: Basis, strain, S, neighbours: int = 8, iters: int = 40, c_out=None, nbr_out=None,
           p_out=None):
    """rb_refine: refined coefficient rows (n x K complex64), the neighbours
    used (n x neighbours global template indices) and |rho|^2 before / after
    (n x 2).  Host arrays unless device buffers are passed in."""
    S = _trig_arg(S)
    n = S.shape[0]
    c = c_out if c_out is not None else np.empty((n, basis.K), dtype=np.complex64)
    nb = nbr_out if nbr_out is not None else np.empty((n, max(neighbours, 1)), dtype=np.int32)
    p = p_out if p_out is not None else np.empty((n, 2), dtype=np.float32)
    _check(lib().rb_refine(ctx.h, basis.h, _ptr(strain), _ptr(S), n, int(neighbours), int(iters), _ptr(c),
                           _ptr(nb), _ptr(p)), "rb_refine")
    return c, (nb[:, :neighbours] if nbr_out is None else nb), p


def cluster_peaks(ctx: Context, trig: np.ndarray, W: int, N: int) -> np.ndarray:
    trig = np.ascontiguousarray(trig, dtype=TRIGGER_NP)
    out = np.zeros(trig.shape[0], dtype=np.uint8)
    _check(lib().rb_cluster_peaks(ctx.h, _ptr(trig), trig.shape[0], int(W), int(N), _ptr(out)),
           "rb_cluster_peaks")
    return out.astype(bool)


def debug_rho(ctx: Context, bank: Bank, strain, basis: Optional[Basis] = None, out=None):
    """rb_debug_rho: (rows, N) complex64, into `out` (host or device) when given."""
    rho = out if out is not None else np.empty((basis.T if basis else bank.T, bank.N), dtype=np.complex64)
    _check(lib().rb_debug_rho(ctx.h, basis.h if basis else None, bank.h, _ptr(strain), _ptr(rho)),
           "rb_debug_rho")
    return rho


def debug_rho_binned(ctx: Context, basis: Basis, strain, w: int) -> np.ndarray:
    """Averaged first-stage series rho_avg (basis.T, N / w) complex64."""
    rho = np.empty((basis.T, basis.bank.N // w), dtype=np.complex64)
    _check(lib().rb_debug_rho_binned(ctx.h, basis.h, _ptr(strain), int(w), _ptr(rho)), "rb_debug_rho_binned")
    return rho


def debug_basis_outputs(ctx: Context, basis: Basis, strain) -> np.ndarray:
    """(K, N) complex64; for a bf16x3 basis (2, K, N): high parts, low parts."""
    shape = (2, basis.K, basis.bank.N) if basis.dtype == RB_BF16X3 else (basis.K, basis.bank.N)
    z = np.empty(shape, dtype=np.complex64)
    _check(lib().rb_debug_basis_outputs(ctx.h, basis.h, _ptr(strain), _ptr(z)), "rb_debug_basis_outputs")
    return z


class BatchItem(C.Structure):
    _fields_ = [("strain", C.c_void_p), ("bank", C.c_void_p), ("bases", C.POINTER(C.c_void_p)),
                ("nbases", C.c_int32)]


def rb_filter_batch(ctx: Context, items, thr1: float, thr2: float, use_graph: bool = True,
                    cap_item: int = 1 << 16, out=None, stage2: int = RB_STAGE2_FULL, bin_w: int = 0,
                    thr_bin: float = 0.0, flags: int = 0):
    """items: list of (device strain tensor, Bank, [Basis, ...]).  Returns
    (list of per-item TRIGGER_NP arrays, Stats); with a device `out` buffer
    (nitems * cap_item x 4 int32) returns (counts, Stats) instead."""
    n = len(items)
    keep = []
    arr = (BatchItem * n)()
    for i, (s, bank, bases) in enumerate(items):
        if isinstance(bases, Basis):
            bases = [bases]
        bp = (C.c_void_p * len(bases))(*[b.h.value for b in bases])
        keep.append(bp)
        arr[i] = BatchItem(_ptr(s), bank.h.value, C.cast(bp, C.POINTER(C.c_void_p)), len(bases))
    o = FilterOpts(thr1, thr2, stage2, int(bin_w), float(thr_bin), 0, int(flags))
    dev = out is not None and not isinstance(out, np.ndarray)
    buf = out if out is not None else np.empty(max(1, n * cap_item), dtype=TRIGGER_NP)
    counts = (C.c_int64 * n)()
    st = Stats()
    _check(lib().rb_filter_batch(ctx.h, n, arr, C.byref(o), int(use_graph), _ptr(buf), cap_item, counts,
                                 C.byref(st)), "rb_filter_batch")
    cnt = [counts[i] for i in range(n)]
    if dev:
        return cnt, st
    return [buf[i * cap_item:i * cap_item + cnt[i]].copy() for i in range(n)], st
