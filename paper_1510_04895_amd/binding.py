"""Thin ctypes binding of libchebfd.so (the C ABI declared in include/chebfd.h).

Every function here only marshals arguments: torch tensors supply device
memory (their data pointers) and the current HIP stream; all computation
happens in the library.  Loading fails loudly if the library has not been
built (``python -m paper_1510_04895_amd.build``): there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchebfd.so")

PREC_C128, PREC_C64 = 0, 1
PREC_C64_CORRECTION = 2          # history only: an FP32 correction pass
POLISH_CORRECTION, POLISH_FP64 = 0, 1
STORAGE_SELL, STORAGE_STENCIL = 0, 1
KERNELS = {"none": 0, "fejer": 1, "jackson": 2, "lanczos": 3}
OK, NOT_CONVERGED, SEARCH_SPACE_TOO_SMALL = 0, 1, 2


class ChebFDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"chebfd error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("lam_lo", C.c_double), ("lam_hi", C.c_double), ("n_s", C.c_int),
                ("n_p", C.c_int), ("kernel", C.c_int), ("mu", C.c_double), ("eps", C.c_double),
                ("max_iter", C.c_int), ("precision", C.c_int), ("lock", C.c_int),
                ("a", C.c_double), ("b", C.c_double), ("seed", C.c_uint64),
                ("gamma_corr", C.c_void_p), ("polish_switch", C.c_double), ("vectors", C.c_int),
                ("verbose", C.c_int), ("bounds", C.c_int), ("adapt", C.c_int),
                ("harmonic", C.c_int), ("polish", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("iterations_c64", C.c_int), ("n_found", C.c_int),
                ("n_locked", C.c_int), ("refilled", C.c_int), ("n_mvm", C.c_int64),
                ("a", C.c_double), ("b", C.c_double), ("t_total", C.c_double),
                ("t_filter", C.c_double), ("t_ortho", C.c_double), ("t_rr", C.c_double),
                ("max_residual", C.c_double), ("n_p_used", C.c_int), ("n_t_estimate", C.c_double),
                ("iterations_corr", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class IterInfo(C.Structure):
    _fields_ = [("n_mvm", C.c_int64), ("precision", C.c_int), ("n_locked", C.c_int),
                ("n_converged", C.c_int), ("n_accepted", C.c_int), ("n_window", C.c_int),
                ("r_min", C.c_double), ("r_max_accepted", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """The loaded library; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1510_04895_amd.build` (no CPU fallback exists)")
    L = C.CDLL(LIB_PATH)
    i32, i64, u64, dbl, vp = C.c_int, C.c_int64, C.c_uint64, C.c_double, C.c_void_p
    pp = C.POINTER(C.c_void_p)
    sig = {
        "chebfd_create": (i32, [pp, i32, vp]),
        "chebfd_destroy": (i32, [vp]),
        "chebfd_synchronize": (i32, [vp]),
        "chebfd_strerror": (C.c_char_p, [i32]),
        "chebfd_last_error": (C.c_char_p, []),
        "chebfd_version": (C.c_char_p, []),
        "chebfd_matrix_from_csr": (i32, [vp, i64, vp, vp, vp, i32, i32, pp]),
        "chebfd_matrix_ti": (i32, [vp, i32, i32, i32, i32, dbl, dbl, dbl, u64, i32, i32, i32, pp]),
        "chebfd_matrix_info": (i32, [vp, vp, vp, vp, vp, vp, vp, vp]),
        "chebfd_matrix_destroy": (i32, [vp]),
        "chebfd_coeffs": (i32, [dbl, dbl, dbl, dbl, i32, i32, dbl, vp]),
        "chebfd_coeffs_divided": (i32, [vp, i32, dbl, dbl, dbl, vp, vp]),
        "chebfd_filter_quality": (i32, [vp, i32, dbl, dbl, dbl, dbl, dbl, dbl, vp, vp]),
        "chebfd_optimal_np": (i32, [dbl, dbl, dbl, dbl, dbl, dbl, i32, dbl, i32, i32, vp, vp]),
        "chebfd_filter_apply": (i32, [vp, vp, i32, vp, i32, dbl, dbl, vp, vp, vp, i64, i64, vp]),
        "chebfd_filter_apply_noalloc": (i32, [vp, vp, i32, vp, i32, dbl, dbl, vp, vp, vp, i64,
                                              i64, vp]),
        "chebfd_filter_apply_columns": (i32, [vp, vp, i32, vp, i64, i32, dbl, dbl, vp, vp, vp,
                                              i64, i64]),
        "chebfd_lanczos_bounds": (i32, [vp, vp, i32, u64, dbl, vp, vp]),
        "chebfd_spmm": (i32, [vp, vp, i32, vp, vp, i64, i64, dbl, dbl]),
        "chebfd_gram": (i32, [vp, i32, vp, i64, i64, vp, i64, i64, i64, vp]),
        "chebfd_block_times": (i32, [vp, i32, vp, i64, i64, i64, vp, i64, i32, vp, i64, i32]),
        "chebfd_residual_norms": (i32, [vp, i32, vp, vp, i64, i64, i64, vp, vp]),
        "chebfd_random_block": (i32, [vp, i32, vp, i64, i64, i64, i64, i64, u64, u64, u64]),
        "chebfd_convert": (i32, [vp, i32, vp, i32, vp, i64, i64, i64, i64]),
        "chebfd_kpm_moments": (i32, [vp, vp, i32, i32, i32, u64, dbl, dbl, vp]),
        "chebfd_host_eigh": (i32, [i32, vp, vp]),
        "chebfd_set_tuning": (i32, [vp, C.c_char_p, i32]),
        "chebfd_result_sweep": (i32, [vp, vp, vp, vp]),
        "chebfd_result_history": (i32, [vp, vp, vp]),
        "chebfd_bandwidth_probe": (i32, [vp, vp, i64, i32, vp]),
        "chebfd_dos_params": (i32, [vp, i32, i64, dbl, dbl, dbl, dbl, dbl, i32, dbl, i32, vp,
                                    vp, vp, vp]),
        "chebfd_learned_features": (i32, [vp, i32, dbl, dbl, dbl, dbl, vp]),
        "chebfd_learned_decode": (i32, [vp, i32, i32, i32, dbl, i32, vp, vp, vp, i32]),
        "chebfd_fit_corrections": (i32, [dbl, dbl, dbl, dbl, dbl, dbl, i32, i32, dbl, i32, dbl,
                                         i32, dbl, vp, vp]),
        "chebfd_mlp_create": (i32, [vp, i32, i32, i32, u64, pp]),
        "chebfd_mlp_destroy": (i32, [vp]),
        "chebfd_mlp_num_params": (i32, [vp, vp]),
        "chebfd_mlp_dims": (i32, [vp, vp, vp, vp]),
        "chebfd_learned_params": (i32, [vp, vp, vp, dbl, dbl, dbl, dbl, i32, i32, i32, u64, dbl,
                                        i32, dbl, i32, i32, vp, vp, vp, i32, vp, vp, vp]),
        "chebfd_mlp_get_params": (i32, [vp, vp, vp, vp, vp]),
        "chebfd_mlp_set_params": (i32, [vp, vp, vp, vp, vp]),
        "chebfd_mlp_forward": (i32, [vp, vp, vp, i32, vp]),
        "chebfd_mlp_input_scaling": (i32, [vp, vp, vp, vp, i32]),
        "chebfd_mlp_loss_grad": (i32, [vp, vp, vp, vp, i32, vp, vp]),
        "chebfd_mlp_train_step": (i32, [vp, vp, vp, vp, i32, C.c_float, C.c_float, vp]),
        "chebfd_params_default": (i32, [vp]),
        "chebfd_solve_workspace_size": (i32, [vp, vp, vp]),
        "chebfd_solve": (i32, [vp, vp, vp, vp, i64, pp]),
        "chebfd_result_get": (i32, [vp, vp, vp, vp, vp, vp]),
        "chebfd_result_destroy": (i32, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def exported_symbols():
    """Names the binding expects the library to export."""
    return [n for n in ("chebfd_create chebfd_destroy chebfd_synchronize chebfd_strerror "
                        "chebfd_last_error chebfd_version chebfd_matrix_from_csr chebfd_matrix_ti "
                        "chebfd_matrix_info chebfd_matrix_destroy chebfd_coeffs "
                        "chebfd_filter_quality chebfd_optimal_np chebfd_filter_apply "
                        "chebfd_filter_apply_noalloc chebfd_filter_apply_columns "
                        "chebfd_coeffs_divided chebfd_spmm "
                        "chebfd_lanczos_bounds "
                        "chebfd_gram chebfd_block_times chebfd_residual_norms "
                        "chebfd_random_block chebfd_convert chebfd_kpm_moments chebfd_host_eigh "
                        "chebfd_params_default chebfd_solve_workspace_size chebfd_solve "
                        "chebfd_result_get chebfd_result_sweep chebfd_result_history chebfd_result_destroy "
                        "chebfd_set_tuning "
                        "chebfd_bandwidth_probe chebfd_dos_params chebfd_learned_features "
                        "chebfd_learned_decode chebfd_fit_corrections chebfd_mlp_create "
                        "chebfd_mlp_destroy chebfd_mlp_num_params chebfd_mlp_get_params "
                        "chebfd_mlp_set_params chebfd_mlp_forward chebfd_mlp_loss_grad "
                        "chebfd_mlp_train_step chebfd_mlp_input_scaling chebfd_mlp_dims "
                        "chebfd_learned_params").split()]


def _check(rc, allow_warn=False):
    if rc < 0 or (rc > 0 and not allow_warn):
        msg = lib().chebfd_last_error().decode()
        raise ChebFDError(rc, msg)
    return rc


def _ptr(t):
    """Device/host pointer of a torch tensor or numpy array (None -> NULL)."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(C.c_void_p)
    return C.c_void_p(t.data_ptr())


def _dbl(a):
    return np.ascontiguousarray(a, np.float64)


# ---------------------------------------------------------------------------
# host-only functions
# ---------------------------------------------------------------------------
def chebfd_coeffs_divided(gamma, a, b, lam):
    """(d, p(t)): coefficients of (p(y) - p(t)) / (y - t), t the scaled lam."""
    g = _dbl(gamma)
    d = np.empty(g.size - 1)
    pt = C.c_double()
    _check(lib().chebfd_coeffs_divided(_ptr(g), g.size - 1, a, b, lam, _ptr(d), C.byref(pt)))
    return d, pt.value


def chebfd_coeffs(lam_lo, lam_hi, a, b, n_p, kernel="lanczos", mu=2.0):
    out = np.empty(n_p + 1)
    k = KERNELS[kernel] if isinstance(kernel, str) else kernel
    _check(lib().chebfd_coeffs(lam_lo, lam_hi, a, b, n_p, k, mu, _ptr(out)))
    return out


def chebfd_filter_quality(gamma, a, b, t_lo, t_hi, s_lo, s_hi):
    g = _dbl(gamma)
    s, e = C.c_double(), C.c_double()
    _check(lib().chebfd_filter_quality(_ptr(g), g.size - 1, a, b, t_lo, t_hi, s_lo, s_hi,
                                       C.byref(s), C.byref(e)))
    return s.value, e.value


def chebfd_optimal_np(a, b, t_lo, t_hi, s_lo, s_hi, kernel="lanczos", mu=2.0, np_min=8,
                      np_max=None):
    if np_max is None:
        np_max = int(16 * 0.5 * (b - a) / max(min(t_lo - s_lo, s_hi - t_hi), 1e-300)) + 8
    n, e = C.c_int(), C.c_double()
    k = KERNELS[kernel] if isinstance(kernel, str) else kernel
    _check(lib().chebfd_optimal_np(a, b, t_lo, t_hi, s_lo, s_hi, k, mu, np_min, np_max,
                                   C.byref(n), C.byref(e)))
    return n.value, e.value


def chebfd_host_eigh(A):
    A = np.array(A, np.complex128, order="C", copy=True)
    n = A.shape[0]
    w = np.empty(n)
    _check(lib().chebfd_host_eigh(n, _ptr(A), _ptr(w)))
    return w, A


# ---------------------------------------------------------------------------
# context and matrices
# ---------------------------------------------------------------------------
class Context:
    def __init__(self, device=0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self.device = device
        self.h = C.c_void_p()
        _check(lib().chebfd_create(C.byref(self.h), device, C.c_void_p(stream)))

    def synchronize(self):
        _check(lib().chebfd_synchronize(self.h))

    def close(self):
        if self.h:
            lib().chebfd_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Matrix:
    def __init__(self, handle):
        self.h = handle

    @classmethod
    def from_csr(cls, ctx, rowptr, col, val, sell_C=32, sell_sigma=256):
        rowptr = np.ascontiguousarray(rowptr, np.int64)
        col = np.ascontiguousarray(col, np.int32)
        val = np.ascontiguousarray(val, np.complex128)
        h = C.c_void_p()
        _check(lib().chebfd_matrix_from_csr(ctx.h, rowptr.size - 1, _ptr(rowptr), _ptr(col),
                                            _ptr(val), sell_C, sell_sigma, C.byref(h)))
        return cls(h)

    @classmethod
    def ti(cls, ctx, L, pbc=3, t=1.0, m=2.0, V=1.0, seed=1, storage=STORAGE_SELL, sell_C=32,
           sell_sigma=256):
        h = C.c_void_p()
        _check(lib().chebfd_matrix_ti(ctx.h, L[0], L[1], L[2], pbc, t, m, V, seed, storage,
                                      sell_C, sell_sigma, C.byref(h)))
        return cls(h)

    def info(self):
        n, nnz, pad = C.c_int64(), C.c_int64(), C.c_int64()
        lo, hi = C.c_double(), C.c_double()
        b128, b64 = C.c_int64(), C.c_int64()
        _check(lib().chebfd_matrix_info(self.h, C.byref(n), C.byref(nnz), C.byref(pad),
                                        C.byref(lo), C.byref(hi), C.byref(b128), C.byref(b64)))
        return dict(n=n.value, nnz=nnz.value, padded=pad.value, g_lo=lo.value, g_hi=hi.value,
                    matrix_bytes_c128=b128.value, matrix_bytes_c64=b64.value)

    def close(self):
        if self.h:
            lib().chebfd_matrix_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# device operations on torch tensors (complex128 -> c128, complex64 -> c64)
# ---------------------------------------------------------------------------
def _prec(t):
    import torch
    if t.dtype == torch.complex128:
        return PREC_C128
    if t.dtype == torch.complex64:
        return PREC_C64
    raise TypeError(f"blocks must be complex128 or complex64, got {t.dtype}")


def _ld(t):
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("blocks must be 2-D with unit column stride")
    return t.stride(0)


def chebfd_filter_apply(ctx, H, gamma, a, b, X, U, W, moments=None, n_s=None):
    g = _dbl(gamma)
    n_s = X.shape[1] if n_s is None else n_s
    _check(lib().chebfd_filter_apply(ctx.h, H.h, _prec(X), _ptr(g), g.size - 1, a, b, _ptr(X),
                                     _ptr(U), _ptr(W), n_s, _ld(X), _ptr(moments)))


def chebfd_filter_apply_noalloc(ctx, H, gamma, a, b, X, U, W, moments=None, n_s=None):
    g = _dbl(gamma)
    n_s = X.shape[1] if n_s is None else n_s
    _check(lib().chebfd_filter_apply_noalloc(ctx.h, H.h, _prec(X), _ptr(g), g.size - 1, a, b,
                                             _ptr(X), _ptr(U), _ptr(W), n_s, _ld(X),
                                             _ptr(moments)))


def chebfd_filter_apply_columns(ctx, H, gcol, a, b, X, U, W, n_s=None):
    """Per-column coefficients: gcol is a device float64 tensor of shape
    (n_p + 1, ldg >= n_s)."""
    n_s = X.shape[1] if n_s is None else n_s
    if gcol.dim() != 2 or gcol.stride(1) != 1 or gcol.dtype.itemsize != 8:
        raise ValueError("gcol must be a 2-D float64 tensor with unit column stride")
    _check(lib().chebfd_filter_apply_columns(ctx.h, H.h, _prec(X), _ptr(gcol), gcol.stride(0),
                                             gcol.shape[0] - 1, a, b, _ptr(X), _ptr(U), _ptr(W),
                                             n_s, _ld(X)))


def chebfd_spmm(ctx, H, X, Y, s_h=1.0, s_u=0.0):
    _check(lib().chebfd_spmm(ctx.h, H.h, _prec(X), _ptr(X), _ptr(Y), X.shape[1], _ld(X), s_h, s_u))


def chebfd_gram(ctx, A, B, S):
    _check(lib().chebfd_gram(ctx.h, _prec(A), _ptr(A), _ld(A), A.shape[1], _ptr(B), _ld(B),
                             B.shape[1], A.shape[0], _ptr(S)))


def chebfd_block_times(ctx, A, T, Cout, subtract=False):
    _check(lib().chebfd_block_times(ctx.h, _prec(A), _ptr(A), _ld(A), A.shape[0], A.shape[1],
                                    _ptr(T), T.shape[1], _prec(Cout), _ptr(Cout), _ld(Cout),
                                    1 if subtract else 0))


def chebfd_residual_norms(ctx, V, HV, theta):
    th = _dbl(theta)
    res = np.empty(V.shape[1])
    _check(lib().chebfd_residual_norms(ctx.h, _prec(V), _ptr(V), _ptr(HV), V.shape[0], V.shape[1],
                                       _ld(V), _ptr(th), _ptr(res)))
    return res


def chebfd_random_block(ctx, X, seed, stream=1, offset=0, k0=0, m=None):
    m = X.shape[1] - k0 if m is None else m
    _check(lib().chebfd_random_block(ctx.h, _prec(X), _ptr(X), X.shape[0], X.shape[1], _ld(X), k0,
                                     m, seed, stream, offset))


def chebfd_convert(ctx, X, Y):
    _check(lib().chebfd_convert(ctx.h, _prec(X), _ptr(X), _prec(Y), _ptr(Y), X.shape[0],
                                X.shape[1], _ld(X), _ld(Y)))


def chebfd_lanczos_bounds(ctx, H, k=40, seed=1, pad=0.01):
    """(a, b) from k Lanczos steps (see include/chebfd.h)."""
    a, b = C.c_double(), C.c_double()
    _check(lib().chebfd_lanczos_bounds(ctx.h, H.h, int(k), int(seed), float(pad), C.byref(a),
                                       C.byref(b)))
    return a.value, b.value


def chebfd_set_tuning(ctx, key, value):
    _check(lib().chebfd_set_tuning(ctx.h, key.encode(), int(value)))


def chebfd_bandwidth_probe(ctx, buf, reps=10):
    """(read-only, copy, 3-read/2-write stream) GB/s over the device buffer."""
    out = np.zeros(3)
    nbytes = buf.numel() * buf.element_size()
    _check(lib().chebfd_bandwidth_probe(ctx.h, _ptr(buf), nbytes, reps, _ptr(out)))
    return tuple(float(v) for v in out)


def chebfd_kpm_moments(ctx, H, n_vec, n_mom, seed, a, b, precision=PREC_C64):
    out = np.empty(n_mom)
    _check(lib().chebfd_kpm_moments(ctx.h, H.h, precision, n_vec, n_mom, seed, a, b, _ptr(out)))
    return out


# ---------------------------------------------------------------------------
# parameter choice and the learned form
# ---------------------------------------------------------------------------
def chebfd_dos_params(mu, n, a, b, lam_lo, lam_hi, ns_over_nt=3.0, kernel="lanczos", mu_k=2.0,
                      ns_max=1024, n_s=0, with_margin=False):
    m = _dbl(mu)
    nt, ns, npp, mg = C.c_double(), C.c_int(n_s), C.c_int(), C.c_double()
    k = KERNELS[kernel] if isinstance(kernel, str) else kernel
    _check(lib().chebfd_dos_params(_ptr(m), m.size, n, a, b, lam_lo, lam_hi, ns_over_nt, k, mu_k,
                                   ns_max, C.byref(nt), C.byref(ns), C.byref(npp), C.byref(mg)))
    if with_margin:
        return nt.value, ns.value, npp.value, mg.value
    return nt.value, ns.value, npp.value


def chebfd_learned_features(mu, a, b, lam_lo, lam_hi):
    m = _dbl(mu)
    f = np.empty(m.size + 2, np.float32)
    _check(lib().chebfd_learned_features(_ptr(m), m.size, a, b, lam_lo, lam_hi, _ptr(f)))
    return f


def chebfd_learned_decode(out, np_ref, ns_ref, n_hat=64, c_max=0.5, ns_max=1024, corr_len=None):
    o = np.ascontiguousarray(out, np.float32)
    npp, ns = C.c_int(), C.c_int()
    _check(lib().chebfd_learned_decode(_ptr(o), np_ref, ns_ref, n_hat, c_max, ns_max, C.byref(npp),
                                       C.byref(ns), None, 0))
    L = npp.value + 1 if corr_len is None else corr_len
    corr = np.empty(L)
    _check(lib().chebfd_learned_decode(_ptr(o), np_ref, ns_ref, n_hat, c_max, ns_max, C.byref(npp),
                                       C.byref(ns), _ptr(corr), L))
    return npp.value, ns.value, corr


def chebfd_fit_corrections(a, b, t_lo, t_hi, s_lo, s_hi, n_p, kernel="lanczos", mu_k=2.0,
                           n_hat=64, c_max=0.5, iters=150, l2=0.0):
    amp = np.zeros(n_hat)
    sig = C.c_double()
    k = KERNELS[kernel] if isinstance(kernel, str) else kernel
    _check(lib().chebfd_fit_corrections(a, b, t_lo, t_hi, s_lo, s_hi, n_p, k, mu_k, n_hat, c_max,
                                        iters, l2, _ptr(amp), C.byref(sig)))
    return amp, sig.value


class MLP:
    """Device network of the learned form (FP32)."""

    def __init__(self, ctx, n_in, n_hidden, n_out, seed=1):
        self.ctx, self.n_in, self.h, self.n_out = ctx, n_in, n_hidden, n_out
        self.h_ = C.c_void_p()
        _check(lib().chebfd_mlp_create(ctx.h, n_in, n_hidden, n_out, seed, C.byref(self.h_)))
        n = C.c_int64()
        _check(lib().chebfd_mlp_num_params(self.h_, C.byref(n)))
        self.n_params = n.value

    def get(self):
        p = np.empty(self.n_params, np.float32)
        sh = np.empty(self.n_out, np.float32)
        sc = np.empty(self.n_out, np.float32)
        _check(lib().chebfd_mlp_get_params(self.ctx.h, self.h_, _ptr(p), _ptr(sh), _ptr(sc)))
        return p, sh, sc

    def set(self, params=None, shift=None, scale=None):
        f = (lambda a: None if a is None else np.ascontiguousarray(a, np.float32))
        params, shift, scale = f(params), f(shift), f(scale)
        _check(lib().chebfd_mlp_set_params(self.ctx.h, self.h_, _ptr(params), _ptr(shift),
                                           _ptr(scale)))

    def input_scaling(self, shift=None, scale=None):
        """Sets (or, without arguments, returns) the input standardisation."""
        if shift is None:
            sh = np.empty(self.n_in, np.float32)
            sc = np.empty(self.n_in, np.float32)
            _check(lib().chebfd_mlp_input_scaling(self.ctx.h, self.h_, _ptr(sh), _ptr(sc), 1))
            return sh, sc
        sh = np.ascontiguousarray(shift, np.float32)
        sc = np.ascontiguousarray(scale, np.float32)
        _check(lib().chebfd_mlp_input_scaling(self.ctx.h, self.h_, _ptr(sh), _ptr(sc), 0))

    def forward(self, X):
        import torch
        Y = torch.empty((X.shape[0], self.n_out), dtype=torch.float32, device=X.device)
        _check(lib().chebfd_mlp_forward(self.ctx.h, self.h_, _ptr(X), X.shape[0], _ptr(Y)))
        return Y

    def loss_grad(self, X, T):
        loss = C.c_float()
        g = np.empty(self.n_params, np.float32)
        _check(lib().chebfd_mlp_loss_grad(self.ctx.h, self.h_, _ptr(X), _ptr(T), X.shape[0],
                                          C.byref(loss), _ptr(g)))
        return loss.value, g

    def train_step(self, X, T, lr, weight_decay=0.0):
        loss = C.c_float()
        _check(lib().chebfd_mlp_train_step(self.ctx.h, self.h_, _ptr(X), _ptr(T), X.shape[0],
                                           lr, weight_decay, C.byref(loss)))
        return loss.value

    def close(self):
        if self.h_:
            lib().chebfd_mlp_destroy(self.h_)
            self.h_ = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def chebfd_learned_params(ctx, H, mlp, a, b, lam_lo, lam_hi, n_vec=8, n_mom=256, n_mom_rule=0,
                          seed=1, ns_over_nt=3.0, n_hat=64, c_max=0.5, ns_max=256, gate=True,
                          n_s=0):
    """(n_p, n_s, corrections or None, rule (n_p, n_s)) from the library's
    learned-form entry point (argument marshalling only)."""
    n_p, kept, npr, nsr = (C.c_int() for _ in range(4))
    cap = 4096
    while True:
        corr = np.zeros(cap)
        ns_ = C.c_int(n_s)
        rc = lib().chebfd_learned_params(ctx.h, H.h, mlp.h_, a, b, lam_lo, lam_hi, n_vec, n_mom,
                                         n_mom_rule, seed, ns_over_nt, n_hat, c_max, ns_max,
                                         int(gate),
                                         C.byref(n_p), C.byref(ns_), _ptr(corr), cap,
                                         C.byref(kept), C.byref(npr), C.byref(nsr))
        if rc == -6 and n_p.value + 1 > cap:
            cap = n_p.value + 1
            continue
        _check(rc)
        break
    c = corr[:n_p.value + 1].copy() if kept.value else None
    return n_p.value, ns_.value, c, (npr.value, nsr.value)


def default_params(**kw):
    p = Params()
    _check(lib().chebfd_params_default(C.byref(p)))
    corr = kw.pop("gamma_corr", None)
    for k, v in kw.items():
        if k == "kernel" and isinstance(v, str):
            v = KERNELS[v]
        setattr(p, k, v)
    if corr is not None:
        corr = _dbl(corr)
        p._corr_keep = corr
        p.gamma_corr = corr.ctypes.data
    return p


def chebfd_solve(ctx, H, params: Params):
    """Runs the solver with a torch-allocated workspace; returns
    (status, evals, residuals, evecs or None, stats dict)."""
    import torch
    nbytes = C.c_int64()
    _check(lib().chebfd_solve_workspace_size(H.h, C.byref(params), C.byref(nbytes)))
    ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=f"cuda:{ctx.device}")
    base = ws.data_ptr()
    aligned = (base + 255) & ~255
    res = C.c_void_p()
    rc = _check(lib().chebfd_solve(ctx.h, H.h, C.byref(params), C.c_void_p(aligned),
                                   nbytes.value, C.byref(res)), allow_warn=True)
    try:
        n = C.c_int64()
        ev = C.POINTER(C.c_double)()
        rs = C.POINTER(C.c_double)()
        vv = C.POINTER(C.c_double)()
        st = Stats()
        _check(lib().chebfd_result_get(res, C.byref(n), C.byref(ev), C.byref(rs), C.byref(vv),
                                       C.byref(st)))
        k = n.value
        evals = np.ctypeslib.as_array(ev, (k,)).copy() if k else np.empty(0)
        resid = np.ctypeslib.as_array(rs, (k,)).copy() if k else np.empty(0)
        vecs = None
        if k and bool(vv):
            N = H.info()["n"]
            vecs = np.ctypeslib.as_array(vv, (N * k * 2,)).copy().view(np.complex128).reshape(N, k)
        stats = st.as_dict()
        # the complex64 sweep's in-window pairs before the FP64 polish
        ns_ = C.c_int64()
        _check(lib().chebfd_result_sweep(res, C.byref(ns_), C.byref(ev), C.byref(rs)))
        m = ns_.value
        stats["sweep_evals"] = np.ctypeslib.as_array(ev, (m,)).copy() if m else np.empty(0)
        stats["sweep_residuals"] = np.ctypeslib.as_array(rs, (m,)).copy() if m else np.empty(0)
        # convergence history (one record per outer iteration)
        hp = C.POINTER(IterInfo)()
        _check(lib().chebfd_result_history(res, C.byref(ns_), C.byref(hp)))
        stats["history"] = [hp[i].as_dict() for i in range(ns_.value)]
        return rc, evals, resid, vecs, stats
    finally:
        lib().chebfd_result_destroy(res)
        del ws
