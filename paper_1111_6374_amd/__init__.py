"""Python binding of libgsyeig (MI355X / gfx950 Krylov solver for A X = B X Lambda).

The functions named ``gsyeig_*`` mirror the C ABI in ``include/gsyeig.h``
argument for argument; device pointers may be passed as integers or as torch
tensors (their ``data_ptr()`` is used).  They only marshal arguments: every
step of the computation runs in the HIP library.  The binding refuses to work
without the built library -- there is no CPU fallback.

``Solver`` is a small convenience layer over the same calls for torch users.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsyeig.so")

GSYEIG_FP64 = 0
GSYEIG_MIXED = 1
GSYEIG_KI = 0
GSYEIG_KE = 1
GSYEIG_TD = 2
GSYEIG_ENOCONV = 0x40000000
GSYEIG_EHIP = 0x40000001
GSYEIG_ESPIN = 0x40000002
GSYEIG_ENOMEM = 0x40000003
GSYEIG_ETOOBIG = 0x40000004
GSYEIG_NOALLOC_MAX_N = 16384

# every entry point declared in include/gsyeig.h
EXPORTS = (
    "gsyeig_version", "gsyeig_opts_default", "gsyeig_create", "gsyeig_destroy",
    "gsyeig_workspace_size", "gsyeig_potrf", "gsyeig_trsv", "gsyeig_symv", "gsyeig_symv_noalloc", "gsyeig_apply_op", "gsyeig_form_c",
    "gsyeig_lanczos_run", "gsyeig_tridiag_eig", "gsyeig_lanczos", "gsyeig_backsolve",
    "gsyeig_check", "gsyeig_solve", "gsyeig_set_trsv_block", "gsyeig_set_spin_limit", "gsyeig_set_trsv_sweep", "gsyeig_autotune", "gsyeig_sync", "gsyeig_solve_batched",
    "gsyeig_trsv_lp", "gsyeig_symv_lp", "gsyeig_apply_op_lp", "gsyeig_trsm_lp", "gsyeig_syev_small", "gsyeig_refine",
)


class GsyeigError(RuntimeError):
    def __init__(self, fn, rc):
        super().__init__(f"{fn} returned {rc} ({_describe(rc)})")
        self.rc = rc


def _describe(rc: int) -> str:
    if rc == 0:
        return "success"
    if rc < 0:
        return f"illegal argument {-rc}"
    return {GSYEIG_ENOCONV: "not converged", GSYEIG_EHIP: "HIP error",
            GSYEIG_ESPIN: "persistent-kernel wait expired", GSYEIG_ENOMEM: "out of device memory",
            GSYEIG_ETOOBIG: "size beyond the entry point's fixed scratch"}.get(
        rc, f"leading minor {rc} of B not positive definite")


class gsyeig_opts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("block", ctypes.c_int), ("which", ctypes.c_int),
                ("invert", ctypes.c_int), ("tol", ctypes.c_double), ("max_steps", ctypes.c_int64),
                ("check_every", ctypes.c_int64), ("seed", ctypes.c_uint64), ("v0", ctypes.c_void_p),
                ("profile_every", ctypes.c_int64), ("eta_tol", ctypes.c_double),
                ("refine_iters", ctypes.c_int64), ("refine_inner", ctypes.c_int64), ("guard", ctypes.c_int64),
                ("reorth", ctypes.c_int64),
                ("basis", ctypes.c_int64),
                ("keep", ctypes.c_int64),
                ("block_acc32", ctypes.c_int64),
                ("variant", ctypes.c_int64),
                ("batch_mode", ctypes.c_int64)]


class gsyeig_info(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("converged", ctypes.c_int64)] + [
        (k, ctypes.c_double) for k in ("eta_max", "rho_f", "omega", "normA_f", "normB_f", "t_gs1_ms",
                                       "t_ki_ms", "t_ki5_ms", "t_bt1_ms", "t_check_ms", "t_total_ms")] + [
        ("prof_samples", ctypes.c_int64), ("t_ki1_ms_sum", ctypes.c_double),
        ("t_ki2_ms_sum", ctypes.c_double), ("t_ki3_ms_sum", ctypes.c_double),
        ("t_refine_ms", ctypes.c_double), ("eta_phase1", ctypes.c_double), ("refine_iters", ctypes.c_int64),
        ("block_applies", ctypes.c_int64), ("block_cols", ctypes.c_int64), ("restarts", ctypes.c_int64),
        ("basis", ctypes.c_int64), ("kept", ctypes.c_int64), ("t_rr_ms", ctypes.c_double),
        ("rr_count", ctypes.c_int64), ("cluster_fallbacks", ctypes.c_int64),
        ("fallback_reason", ctypes.c_int64), ("reorth_steps", ctypes.c_int64), ("t_gs2_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class gsyeig_tuning(ctypes.Structure):
    _fields_ = [("n_bucket", ctypes.c_int64), ("prec", ctypes.c_int), ("trsv_block", ctypes.c_int),
                ("trsv_sweep", ctypes.c_int), ("from_cache", ctypes.c_int), ("gemm_big_min", ctypes.c_int64),
                ("op_ms", ctypes.c_double), ("gemm_ms", ctypes.c_double), ("op_ms_cand", ctypes.c_double * 5),
                ("gemm_ms_cand", ctypes.c_double * 2)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["op_ms_cand"] = list(self.op_ms_cand)
        d["gemm_ms_cand"] = list(self.gemm_ms_cand)
        return d


_lib = None


def lib():
    """Load libgsyeig.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1111_6374_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        sig = {
            "gsyeig_version": ([], ctypes.c_char_p),
            "gsyeig_opts_default": ([ctypes.POINTER(gsyeig_opts)], I),
            "gsyeig_create": ([ctypes.POINTER(P), P], I),
            "gsyeig_destroy": ([P], I),
            "gsyeig_set_trsv_block": ([P, I64], I),
            "gsyeig_set_spin_limit": ([P, ctypes.c_uint], I),
            "gsyeig_set_trsv_sweep": ([P, I], I),
            "gsyeig_autotune": ([P, I64, I, ctypes.c_char_p, ctypes.POINTER(gsyeig_tuning)], I),
            "gsyeig_sync": ([P], I),
            "gsyeig_workspace_size": ([I64, I64, ctypes.POINTER(gsyeig_opts), ctypes.POINTER(ctypes.c_size_t)], I),
            "gsyeig_potrf": ([P, I64, P, I64, ctypes.POINTER(gsyeig_opts), P], I),
            "gsyeig_trsv_lp": ([P, I64, P, I64, I, P, P], I),
            "gsyeig_symv_lp": ([P, I64, P, I64, P, P], I),
            "gsyeig_apply_op_lp": ([P, I64, P, I64, P, I64, P, P], I),
            "gsyeig_trsm_lp": ([P, I64, P, I64, I, I64, P, I64, P, I64], I),
            "gsyeig_syev_small": ([P, I64, P, I64, I64, I, P, P, I64], I),
            "gsyeig_refine": ([P, I64, I64, I64, P, I64, P, I64, P, I64, ctypes.POINTER(gsyeig_opts), P, I64, P, P,
                               I64, ctypes.POINTER(gsyeig_info)], I),
            "gsyeig_trsv": ([P, I64, P, I64, I, P, P], I),
            "gsyeig_symv": ([P, I64, P, I64, P, P], I),
            "gsyeig_symv_noalloc": ([P, I64, P, I64, P, P], I),
            "gsyeig_apply_op": ([P, I64, P, I64, P, I64, P, P], I),
            "gsyeig_form_c": ([P, I64, P, I64, P, I64, P, I64], I),
            "gsyeig_lanczos_run": ([P, I64, I64, P, I64, P, I64, P, P, P, P, I64], I),
            "gsyeig_tridiag_eig": ([P, I64, P, P, I64, I, P, P, I64], I),
            "gsyeig_lanczos": ([P, I64, I64, P, I64, P, I64, ctypes.POINTER(gsyeig_opts), P, P, I64,
                                ctypes.POINTER(I64)], I),
            "gsyeig_backsolve": ([P, I64, I64, P, I64, P, I64], I),
            "gsyeig_check": ([P, I64, I64, P, I64, P, I64, P, P, P, I64, ctypes.POINTER(gsyeig_info)], I),
            "gsyeig_solve": ([P, I64, I64, P, I64, P, I64, ctypes.POINTER(gsyeig_opts), P, P, I64,
                              ctypes.POINTER(gsyeig_info)], I),
            "gsyeig_solve_batched": ([P, I64, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(P),
                                      ctypes.POINTER(I64), ctypes.POINTER(P), ctypes.POINTER(I64),
                                      ctypes.POINTER(gsyeig_opts), ctypes.POINTER(P), ctypes.POINTER(P),
                                      ctypes.POINTER(I64), I64, ctypes.POINTER(I), ctypes.POINTER(gsyeig_info)], I),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _p(x):
    """Device pointer of a tensor (checked FP64 on a GPU) or an int/None."""
    if x is None or isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        if not x.is_cuda:
            raise ValueError("gsyeig expects device tensors")
        return x.data_ptr()
    raise TypeError(type(x))


# ------------------------------------------------------------------ C ABI mirrors
def gsyeig_version() -> str:
    return lib().gsyeig_version().decode()


def gsyeig_opts_default() -> gsyeig_opts:
    o = gsyeig_opts()
    lib().gsyeig_opts_default(ctypes.byref(o))
    return o


def gsyeig_create(hip_stream=None):
    """Returns (rc, ctx)."""
    ctx = ctypes.c_void_p()
    rc = lib().gsyeig_create(ctypes.byref(ctx), hip_stream)
    return rc, ctx


def gsyeig_destroy(ctx) -> int:
    return lib().gsyeig_destroy(ctx)


def gsyeig_set_trsv_block(ctx, rows) -> int:
    return lib().gsyeig_set_trsv_block(ctx, rows)


def gsyeig_set_trsv_sweep(ctx, kind) -> int:
    return lib().gsyeig_set_trsv_sweep(ctx, kind)


def gsyeig_autotune(ctx, n, prec=GSYEIG_FP64, cache_path=None):
    """Returns (rc, gsyeig_tuning)."""
    t = gsyeig_tuning()
    rc = lib().gsyeig_autotune(ctx, n, prec, cache_path.encode() if cache_path else None, ctypes.byref(t))
    return rc, t


def gsyeig_set_spin_limit(ctx, limit) -> int:
    return lib().gsyeig_set_spin_limit(ctx, limit)


def gsyeig_sync(ctx) -> int:
    return lib().gsyeig_sync(ctx)


def gsyeig_workspace_size(n, s, opts=None):
    """Returns (rc, bytes)."""
    b = ctypes.c_size_t()
    rc = lib().gsyeig_workspace_size(n, s, ctypes.byref(opts) if opts else None, ctypes.byref(b))
    return rc, b.value


def gsyeig_potrf(ctx, n, B, ldb, opts=None, U_lowprec=None) -> int:
    return lib().gsyeig_potrf(ctx, n, _p(B), ldb, ctypes.byref(opts) if opts else None, _p(U_lowprec))


def gsyeig_trsv(ctx, n, U, ldu, trans, b, x) -> int:
    return lib().gsyeig_trsv(ctx, n, _p(U), ldu, trans, _p(b), _p(x))


def gsyeig_symv(ctx, n, A, lda, x, y) -> int:
    return lib().gsyeig_symv(ctx, n, _p(A), lda, _p(x), _p(y))


def gsyeig_symv_noalloc(hip_stream, n, A, lda, x, y) -> int:
    return lib().gsyeig_symv_noalloc(hip_stream, n, _p(A), lda, _p(x), _p(y))


def gsyeig_apply_op(ctx, n, A, lda, U, ldu, w, z) -> int:
    return lib().gsyeig_apply_op(ctx, n, _p(A), lda, _p(U), ldu, _p(w), _p(z))


def gsyeig_form_c(ctx, n, A, lda, U, ldu, C, ldc) -> int:
    return lib().gsyeig_form_c(ctx, n, _p(A), lda, _p(U), ldu, _p(C), ldc)


def gsyeig_lanczos_run(ctx, n, k, A, lda, U, ldu, v0, alpha, beta, V, ldv) -> int:
    return lib().gsyeig_lanczos_run(ctx, n, k, _p(A), lda, _p(U), ldu, _p(v0), _p(alpha), _p(beta),
                                    _p(V), ldv)


def gsyeig_tridiag_eig(ctx, m, alpha, beta, nwant, which, theta, S=None, lds=0) -> int:
    return lib().gsyeig_tridiag_eig(ctx, m, _p(alpha), _p(beta), nwant, which, _p(theta), _p(S), lds)


def gsyeig_lanczos(ctx, n, s, A, lda, U, ldu, opts, theta, Y, ldy):
    """Returns (rc, steps)."""
    steps = ctypes.c_int64()
    rc = lib().gsyeig_lanczos(ctx, n, s, _p(A), lda, _p(U), ldu, ctypes.byref(opts) if opts else None,
                              _p(theta), _p(Y), ldy, ctypes.byref(steps))
    return rc, steps.value


def gsyeig_trsv_lp(ctx, n, U, ldu, trans, b, x) -> int:
    return lib().gsyeig_trsv_lp(ctx, n, _p(U), ldu, trans, _p(b), _p(x))


def gsyeig_symv_lp(ctx, n, A, lda, x, y) -> int:
    return lib().gsyeig_symv_lp(ctx, n, _p(A), lda, _p(x), _p(y))


def gsyeig_apply_op_lp(ctx, n, A, lda, U, ldu, w, z) -> int:
    return lib().gsyeig_apply_op_lp(ctx, n, _p(A), lda, _p(U), ldu, _p(w), _p(z))


def gsyeig_trsm_lp(ctx, n, U, ldu, trans, k, V, ldv, X, ldx) -> int:
    return lib().gsyeig_trsm_lp(ctx, n, _p(U), ldu, trans, k, _p(V), ldv, _p(X), ldx)


def gsyeig_syev_small(ctx, N, H, ldh, nwant, which, w, Q, ldq) -> int:
    return lib().gsyeig_syev_small(ctx, N, _p(H), ldh, nwant, which, _p(w), _p(Q), ldq)


def gsyeig_refine(ctx, n, s, k, A, lda, B, ldb, U_lowprec, ldu, opts, X0, ldx0, Lambda, X, ldx):
    """Returns (rc, info)."""
    info = gsyeig_info()
    rc = lib().gsyeig_refine(ctx, n, s, k, _p(A), lda, _p(B), ldb, _p(U_lowprec), ldu,
                             ctypes.byref(opts) if opts else None, _p(X0), ldx0, _p(Lambda), _p(X), ldx,
                             ctypes.byref(info))
    return rc, info


def gsyeig_backsolve(ctx, n, s, U, ldu, Y_to_X, ldy) -> int:
    return lib().gsyeig_backsolve(ctx, n, s, _p(U), ldu, _p(Y_to_X), ldy)


def gsyeig_check(ctx, n, s, A, lda, B, ldb, Bdiag, Lambda, X, ldx):
    """Returns (rc, gsyeig_info with eta_max, rho_f, omega, normA_f, normB_f)."""
    info = gsyeig_info()
    rc = lib().gsyeig_check(ctx, n, s, _p(A), lda, _p(B), ldb, _p(Bdiag), _p(Lambda), _p(X), ldx,
                            ctypes.byref(info))
    return rc, info


def gsyeig_solve(ctx, n, s, A, lda, B, ldb, opts, Lambda, X, ldx):
    """Returns (rc, gsyeig_info)."""
    info = gsyeig_info()
    rc = lib().gsyeig_solve(ctx, n, s, _p(A), lda, _p(B), ldb, ctypes.byref(opts) if opts else None,
                            _p(Lambda), _p(X), ldx, ctypes.byref(info))
    return rc, info


def gsyeig_solve_batched(ctx, n, s, A, lda, B, ldb, opts, Lambda, X, ldx, nstreams=8):
    """Per-instance lists (host ints / device tensors or pointers).
    Returns (rc, status list, list of gsyeig_info)."""
    cnt = len(n)
    I64A = ctypes.c_int64 * cnt
    PA = ctypes.c_void_p * cnt
    st = (ctypes.c_int * cnt)()
    infos = (gsyeig_info * cnt)()
    rc = lib().gsyeig_solve_batched(ctx, cnt, I64A(*n), I64A(*s), PA(*[_p(a) for a in A]), I64A(*lda),
                                    PA(*[_p(b) for b in B]), I64A(*ldb),
                                    ctypes.byref(opts) if opts else None, PA(*[_p(l) for l in Lambda]),
                                    PA(*[_p(x) for x in X]), I64A(*ldx), nstreams, st, infos)
    return rc, list(st), list(infos)


# ------------------------------------------------------------------ torch convenience
class Solver:
    """One context on the current torch stream.  Tensors are FP64 on the GPU;
    square matrices row-major (torch default), vector blocks as (s, n)
    tensors (row i = vector i, i.e. column-major n x s)."""

    def __init__(self, stream=None):
        import torch

        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        rc, self.ctx = gsyeig_create(stream.cuda_stream)
        if rc:
            raise GsyeigError("gsyeig_create", rc)

    def close(self):
        if self.ctx:
            gsyeig_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, A, B, s, opts=None, overwrite_b=False):
        """Lambda (s,), X (s, n), info dict.  B is copied unless overwrite_b."""
        import torch

        n = A.shape[0]
        if not overwrite_b:
            B = B.clone()
        Lam = torch.empty(s, dtype=torch.float64, device=A.device)
        X = torch.empty(s, n, dtype=torch.float64, device=A.device)
        rc, info = gsyeig_solve(self.ctx, n, s, A, A.stride(0), B, B.stride(0), opts, Lam, X, X.stride(0))
        if rc and rc != GSYEIG_ENOCONV:
            raise GsyeigError("gsyeig_solve", rc)
        d = info.as_dict()
        d["rc"] = rc
        return Lam, X, d
