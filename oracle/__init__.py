"""CPU parity oracle -- TEST INFRASTRUCTURE ONLY.

Plain FP64 reference for the symmetric-definite generalized eigenproblem
A X = B X Lambda (Eq. 1).  The arithmetic lives in ``oracle.c`` (plain C
loops, no BLAS/LAPACK); this module only marshals numpy arrays and adds the
accuracy metrics of the paper's Tables 3 and 7 plus the per-pair backward
error used as the acceptance gate.

Only the test suite, the smoke check and the bench's CPU-baseline leg may
import this package.  The GPU library never loads it and shares no code with
it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
               "-o", tmp, SRC_PATH, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        i, d = ctypes.c_int, ctypes.c_double
        L.or_cholesky_upper.argtypes = [i, _dp, _dp]
        L.or_cholesky_upper.restype = i
        L.or_trsv_upper.argtypes = [i, _dp, _dp]
        L.or_trsv_upper_t.argtypes = [i, _dp, _dp]
        L.or_matvec.argtypes = [i, _dp, _dp, _dp]
        L.or_form_c.argtypes = [i, _dp, _dp, _dp]
        L.or_eig_ql.argtypes = [i, _dp, _dp, _dp]
        L.or_eig_ql.restype = i
        L.or_eig_jacobi.argtypes = [i, _dp, _dp, _dp]
        L.or_eig_jacobi.restype = i
        L.or_inertia_below.argtypes = [i, _dp, _dp, d]
        L.or_inertia_below.restype = i
        L.or_bisect_eig.argtypes = [i, _dp, _dp, i]
        L.or_bisect_eig.restype = d
        L.or_backsolve.argtypes = [i, i, _dp, _dp]
        L.or_gsyeig.argtypes = [i, i, i, i, _dp, _dp, _dp, _dp]
        L.or_gsyeig.restype = i
        L.or_lanczos.argtypes = [i, i, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_tridiag_eigvals.argtypes = [i, _dp, _dp, _dp]
        L.or_tridiag_eigvals.restype = i
        _lib = L
    return _lib


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------------ steps
def cholesky_upper(B):
    """Eq. 2: upper U with B = U^T U.  Raises if B is not SPD."""
    B = _c(B)
    n = B.shape[0]
    U = np.empty_like(B)
    info = lib().or_cholesky_upper(n, B, U)
    if info:
        raise np.linalg.LinAlgError(f"leading minor {info} not positive definite")
    return U


def trsv_upper(U, b):
    """U^-1 b (key KI1)."""
    x = _c(b).copy()
    lib().or_trsv_upper(U.shape[0], _c(U), x)
    return x


def trsv_upper_t(U, b):
    """U^-T b (key KI3)."""
    x = _c(b).copy()
    lib().or_trsv_upper_t(U.shape[0], _c(U), x)
    return x


def matvec(A, x):
    """A x (key KI2)."""
    A = _c(A)
    y = np.empty(A.shape[0])
    lib().or_matvec(A.shape[0], A, _c(x), y)
    return y


def apply_ki(A, U, w):
    """z = U^-T (A (U^-1 w)): the implicit operator of variant KI."""
    return trsv_upper_t(U, matvec(A, trsv_upper(U, w)))


def form_c(A, U):
    """Eq. 3: C = U^-T A U^-1 by two triangular solves, symmetrised."""
    A = _c(A)
    C = np.empty_like(A)
    lib().or_form_c(A.shape[0], A, _c(U), C)
    return C


def eig_sym(C, method: str = "ql"):
    """All eigenpairs of symmetric C: (w ascending, Z with columns = vectors)."""
    C = _c(C).copy()
    n = C.shape[0]
    w = np.empty(n)
    Zt = np.empty_like(C)
    if method == "ql":
        rc = lib().or_eig_ql(n, C, w, Zt)
    elif method == "jacobi":
        rc = lib().or_eig_jacobi(n, C, w, Zt)
        rc = 0 if rc >= 0 else rc
    else:
        raise ValueError(method)
    if rc:
        raise RuntimeError(f"eigensolver {method} failed ({rc})")
    order = np.argsort(w, kind="stable")
    return w[order], Zt[order].T.copy()


def inertia_below(A, B, sigma: float) -> int:
    """#eigenvalues of (A, B) below sigma, by Bunch-Parlett LDL^T of A - sigma B."""
    return int(lib().or_inertia_below(A.shape[0], _c(A), _c(B), float(sigma)))


def bisect_eigs(A, B, ks):
    """Eigenvalues of (A, B) with 0-based ascending indices ks, by inertia bisection."""
    A, B = _c(A), _c(B)
    return np.array([lib().or_bisect_eig(A.shape[0], A, B, int(k)) for k in ks])


def backsolve(U, Y_rows):
    """Eq. 4: X = U^-1 Y for vectors stored as rows (s x n)."""
    X = _c(Y_rows).copy()
    lib().or_backsolve(U.shape[0], X.shape[0], _c(U), X)
    return X


def gsyeig(A, B, s: int, which: str = "smallest", method: str = "ql"):
    """The definition (Eq. 1-4): (lam (s,) ascending, X (s, n) rows = x_i).

    X is B-orthonormal and each x_i has its largest-magnitude entry positive
    (lowest index on ties).
    """
    A, B = _c(A), _c(B)
    n = A.shape[0]
    lam = np.empty(s)
    X = np.empty((s, n))
    rc = lib().or_gsyeig(n, s, 1 if which == "largest" else 0, 1 if method == "jacobi" else 0,
                         A, B, lam, X)
    if rc > 0:
        raise np.linalg.LinAlgError(f"B: leading minor {rc} not positive definite")
    if rc < 0:
        raise RuntimeError(f"or_gsyeig failed ({rc})")
    return lam, X


def lanczos(A, U, v0, k: int):
    """k steps of plain Lanczos (KI operator, CGS2): (alpha (k,), beta (k,), W (k+1, n))."""
    n = A.shape[0]
    alpha = np.empty(k)
    beta = np.empty(k)
    W = np.empty((k + 1, n))
    lib().or_lanczos(n, k, _c(A), _c(U), _c(v0), alpha, beta, W)
    return alpha, beta, W


def tridiag_eigvals(d, e):
    """Ascending eigenvalues of the symmetric tridiagonal with diagonal d and
    off-diagonal e (len(e) = len(d) - 1)."""
    d = _c(d)
    m = d.shape[0]
    ee = np.zeros(m)
    ee[: m - 1] = e[: m - 1]
    w = np.empty(m)
    if lib().or_tridiag_eigvals(m, d, ee, w):
        raise RuntimeError("tridiagonal QL failed")
    return w


def sign_normalise_rows(X):
    """Make the largest-magnitude entry of every row positive (lowest index on ties)."""
    X = np.array(X, dtype=np.float64, copy=True)
    for i in range(X.shape[0]):
        p = int(np.argmax(np.abs(X[i])))
        if X[i, p] < 0:
            X[i] = -X[i]
    return X


# ------------------------------------------------------------------ metrics
def metrics(A, B, lam, X_rows, lam_ref=None):
    """Accuracy metrics for s pairs (lam_i, x_i), x_i = row i of X_rows.

    rho_F  = ||A X - B X Lambda||_F / max(||A||_F, ||B||_F)   (Tables 3/7)
    omega  = ||I - X^T B X||_F                   (reported with and without
    omega_paper = omega / ||B||_F                 the paper's /||B||_F)
    eta_i  = ||A x_i - lam_i B x_i||_2 / ((||A||_F + |lam_i| ||B||_F) ||x_i||_2)
    e_lam  = max_i |lam_i - lam_ref_i| / max_j |lam_ref_j|
    """
    A, B = _c(A), _c(B)
    X = _c(X_rows).T  # n x s
    lam = np.asarray(lam, dtype=np.float64)
    AX = A @ X
    BX = B @ X
    R = AX - BX * lam[None, :]
    nA = np.linalg.norm(A, "fro")
    nB = np.linalg.norm(B, "fro")
    out = {
        "rho_F": float(np.linalg.norm(R, "fro") / max(nA, nB)),
        "omega": float(np.linalg.norm(np.eye(X.shape[1]) - X.T @ BX, "fro")),
    }
    out["omega_paper"] = out["omega"] / nB
    eta = np.linalg.norm(R, axis=0) / ((nA + np.abs(lam) * nB) * np.linalg.norm(X, axis=0))
    out["eta"] = eta
    out["eta_max"] = float(eta.max())
    if lam_ref is not None:
        lam_ref = np.asarray(lam_ref, dtype=np.float64)
        out["e_lam"] = float(np.max(np.abs(lam - lam_ref)) / np.max(np.abs(lam_ref)))
    return out
