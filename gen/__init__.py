"""Seeded synthetic inputs for the symmetric-definite pencil A X = B X Lambda.

This module only *builds inputs* (and the answers those inputs are built to
have).  It holds none of the solver's arithmetic: no Cholesky factorisation,
no triangular solve, no Lanczos step, no eigensolver.  Both the CPU oracle and
the GPU path are fed from here and neither imports the other.

Workloads (stand-ins for the paper's molecular-dynamics and DFT matrices,
Section 3.1/3.2, which are not available):

* ``known_spectrum``: A = U^T Y diag(lam) Y^T U, B = U^T U with U upper
  triangular (diagonal ~ U[1,2], strict upper ~ N(0, 1/n)) and Y the
  orthogonal factor of a seeded Gaussian matrix (sign fixed so diag(R) > 0).
  Then C = U^-T A U^-1 = Y diag(lam) Y^T (Eq. 3), so the eigenvalues of the
  pencil are exactly ``lam`` and the eigenvectors are U^-1 Y.
* ``fem_pencil``: the 1-D linear finite-element stiffness/mass pair on (0,1)
  with Dirichlet ends, whose eigenpairs have a closed form (``fem_eigs``).
* ``splitmix64_uniform``: the start-vector generator, SplitMix64 (Steele, Lea
  and Flood, OOPSLA 2014) mapped to doubles in [-1, 1).  The GPU library
  implements the same published generator independently.
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 6374
_MASK64 = (1 << 64) - 1


def rng(seed: int = BASE_SEED, *stream: int) -> np.random.Generator:
    """A numpy Generator keyed by (seed, stream...)."""
    return np.random.default_rng([int(seed)] + [int(s) for s in stream])


# --------------------------------------------------------------------------
# spectra
# --------------------------------------------------------------------------
def spectrum_spaced(n: int, g: np.random.Generator) -> np.ndarray:
    """lam in [-1, 1] whose 10 smallest values are spaced >= 1e-2.

    The first min(n, 10) values are the ladder -1 + 0.02 i (i = 0..9); the
    remaining n - 10 are iid U[-0.80, 1], so every gap among and after the 10
    smallest is >= 1e-2 (rejection sampling would almost never succeed).
    """
    k = min(n, 10)
    ladder = -1.0 + 0.02 * np.arange(k, dtype=np.float64)
    rest = g.uniform(-0.80, 1.0, size=n - k)
    return np.concatenate([ladder, rest])


def spectrum_clustered(n: int, g: np.random.Generator) -> np.ndarray:
    """80 % of the values iid U[0, 1], the other 20 % iid U[1, 10]."""
    n0 = int(round(0.8 * n))
    return np.concatenate([g.uniform(0.0, 1.0, size=n0), g.uniform(1.0, 10.0, size=n - n0)])


SPECTRA = {"spaced": spectrum_spaced, "clustered": spectrum_clustered}


# --------------------------------------------------------------------------
# factors
# --------------------------------------------------------------------------
def factor_U(n: int, g: np.random.Generator) -> np.ndarray:
    """Upper-triangular U: diagonal U[1, 2], strict upper N(0, 1/n), lower 0."""
    U = np.triu(g.standard_normal((n, n)) / math.sqrt(n), 1)
    U[np.diag_indices(n)] = g.uniform(1.0, 2.0, size=n)
    return U


def haar_Y(n: int, g: np.random.Generator) -> np.ndarray:
    """Orthogonal factor of a Gaussian n x n matrix, columns signed so diag(R) > 0."""
    G = g.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    sgn = np.sign(np.diag(R))
    sgn[sgn == 0] = 1.0
    return Q * sgn[None, :]


def known_spectrum(n: int, law: str = "spaced", seed: int = BASE_SEED, stream=(0,)):
    """Host (numpy, FP64, row-major) known-spectrum instance.

    Returns a dict with A, B (n x n), U, Y (n x n) and lam (n, unsorted, in the
    order of Y's columns).
    """
    g = rng(seed, *stream)
    U = factor_U(n, g)
    Y = haar_Y(n, g)
    lam = SPECTRA[law](n, g)
    M = (Y * lam[None, :]) @ Y.T
    A = U.T @ M @ U
    A = 0.5 * (A + A.T)
    B = U.T @ U
    B = 0.5 * (B + B.T)
    return {"A": np.ascontiguousarray(A), "B": np.ascontiguousarray(B), "U": U, "Y": Y, "lam": lam}


def known_spectrum_device(n: int, law: str = "spaced", seed: int = BASE_SEED, stream=(0,),
                          device="cuda", keep_factors: bool = True, rng_kind: str = "numpy"):
    """Same instance law as ``known_spectrum`` assembled on a torch device.

    rng_kind = "numpy": the random draws (U, the Gaussian, lam) come from the
    same numpy streams as the host version; only the O(n^3) assembly (QR and
    the products) runs on the device, so large n is generated in seconds.
    rng_kind = "torch": the draws come from a torch generator on the device
    seeded with (seed, stream) -- a different but equally seeded instance,
    for workloads with many instances.
    """
    import torch

    if rng_kind == "numpy":
        g = rng(seed, *stream)
        U = torch.from_numpy(factor_U(n, g)).to(device)
        G = torch.from_numpy(g.standard_normal((n, n))).to(device)
        lam_h = SPECTRA[law](n, g)
    else:
        tg = torch.Generator(device=device)
        tg.manual_seed(int(np.random.SeedSequence([int(seed)] + [int(v) for v in stream]).generate_state(1)[0]))
        U = torch.triu(torch.randn(n, n, generator=tg, device=device, dtype=torch.float64) / math.sqrt(n), 1)
        U.diagonal().copy_(1.0 + torch.rand(n, generator=tg, device=device, dtype=torch.float64))
        G = torch.randn(n, n, generator=tg, device=device, dtype=torch.float64)
        lam_h = SPECTRA[law](n, rng(seed, *stream))
    Q, R = torch.linalg.qr(G)
    del G
    sgn = torch.sign(torch.diagonal(R))
    sgn[sgn == 0] = 1.0
    del R
    Y = Q * sgn[None, :]
    del Q
    lam = torch.from_numpy(lam_h).to(device)
    M = torch.matmul(Y * lam[None, :], Y.t().contiguous())
    UtM = torch.matmul(U.t().contiguous(), M)
    del M
    A = torch.matmul(UtM, U)
    del UtM
    A = 0.5 * (A + A.t())
    A = A.contiguous()
    B = torch.matmul(U.t().contiguous(), U)
    B = (0.5 * (B + B.t())).contiguous()
    out = {"A": A, "B": B, "lam": lam_h}
    if keep_factors:
        out["U"] = U
        out["Y"] = Y
    else:
        del U, Y
    return out


def _row_blocks(n: int, nb: int):
    return [(r0, min(n, r0 + nb)) for r0 in range(0, n, nb)]


def known_spectrum_device_blocked(n: int, law: str = "spaced", seed: int = BASE_SEED, stream=(0,),
                                  device="cuda", nb: int = 4096, rank: int = 256):
    """Known-spectrum pencil for n beyond what single-tensor device kernels
    and a dense QR handle (n^2 > 2^31): A = U^T Y diag(lam) Y^T U, B = U^T U
    with the same U and lam laws as ``known_spectrum``, and the orthogonal
    Y = I - 2 Q Q^T, Q the orthonormal factor of a seeded Gaussian n x rank
    (an exactly orthogonal similarity, so lam is exact; A and B are dense).
    Every device operation touches contiguous row blocks of at most nb rows.
    Draws come from a torch generator seeded with (seed, stream)."""
    import torch

    f64 = torch.float64
    tg = torch.Generator(device=device)
    tg.manual_seed(int(np.random.SeedSequence([int(seed)] + [int(v) for v in stream]).generate_state(1)[0]))
    blocks = _row_blocks(n, nb)
    U = torch.empty(n, n, dtype=f64, device=device)
    for r0, r1 in blocks:
        blk = torch.randn(r1 - r0, n, generator=tg, device=device, dtype=f64) / math.sqrt(n)
        blk = torch.triu(blk, diagonal=r0 + 1)
        i = torch.arange(r1 - r0, device=device)
        blk[i, r0 + i] = 1.0 + torch.rand(r1 - r0, generator=tg, device=device, dtype=f64)
        U[r0:r1].copy_(blk)
        del blk
    Q, _ = torch.linalg.qr(torch.randn(n, rank, generator=tg, device=device, dtype=f64))
    lam_h = SPECTRA[law](n, rng(seed, *stream))
    lam = torch.from_numpy(lam_h).to(device)
    # M = Y diag(lam) Y = diag(lam) + L R^T with L = [Q, P, Q S], R = [-2P, -2Q, 4Q],
    # P = diag(lam) Q, S = Q^T P
    P = lam[:, None] * Q
    S = Q.t() @ P
    L = torch.cat([Q, P, Q @ S], dim=1)
    Rt = torch.cat([-2.0 * P, -2.0 * Q, 4.0 * Q], dim=1).t().contiguous()
    del P, S
    M = torch.empty(n, n, dtype=f64, device=device)
    for r0, r1 in blocks:
        M[r0:r1] = L[r0:r1] @ Rt
        M[r0:r1].diagonal(r0).add_(lam[r0:r1])
    del L, Rt, Q
    # T = M U (U's block (k, c) vanishes for c < k)
    T = torch.zeros(n, n, dtype=f64, device=device)
    for r0, r1 in blocks:
        Tr = T[r0:r1]
        for k0, k1 in blocks:
            Tr[:, k0:].addmm_(M[r0:r1, k0:k1], U[k0:k1, k0:])
    del M

    def ut_times(X):
        """U^T X by row blocks (U's block (k, r) vanishes for k > r)."""
        out = torch.zeros(n, n, dtype=f64, device=device)
        for r0, r1 in blocks:
            Or = out[r0:r1]
            for k0, k1 in blocks:
                if k0 > r0:
                    break
                Or.addmm_(U[k0:k1, r0:r1].t(), X[k0:k1])
        return out

    def symmetrise(X):
        for a, (r0, r1) in enumerate(blocks):
            for c0, c1 in blocks[a:]:
                v = 0.5 * (X[r0:r1, c0:c1] + X[c0:c1, r0:r1].t())
                X[r0:r1, c0:c1] = v
                X[c0:c1, r0:r1] = v.t()
        return X

    A = symmetrise(ut_times(T))
    del T
    B = symmetrise(ut_times(U))
    del U
    return {"A": A, "B": B, "lam": lam_h}


def copy_rows(dst, src, nb: int = 4096):
    """dst[:] = src for large n x n device tensors, one row block at a time."""
    for r0, r1 in _row_blocks(src.shape[0], nb):
        dst[r0:r1].copy_(src[r0:r1])


# --------------------------------------------------------------------------
# the 1-D finite-element pencil
# --------------------------------------------------------------------------
def fem_pencil(n: int):
    """Stiffness K = tridiag(-1, 2, -1)/h and mass M = (h/6) tridiag(1, 4, 1),
    h = 1/(n+1), linear elements on (0, 1) with both ends fixed.  Dense FP64."""
    h = 1.0 / (n + 1)
    K = np.zeros((n, n))
    M = np.zeros((n, n))
    i = np.arange(n)
    K[i, i] = 2.0 / h
    M[i, i] = 4.0 * h / 6.0
    K[i[:-1], i[:-1] + 1] = K[i[:-1] + 1, i[:-1]] = -1.0 / h
    M[i[:-1], i[:-1] + 1] = M[i[:-1] + 1, i[:-1]] = h / 6.0
    return K, M


def fem_pencil_device(n: int, device="cuda", nb: int = 4096):
    """``fem_pencil(n)`` assembled directly on a torch device (same values)."""
    import torch

    h = 1.0 / (n + 1)
    K = torch.empty(n, n, dtype=torch.float64, device=device)
    M = torch.empty(n, n, dtype=torch.float64, device=device)
    for r0, r1 in _row_blocks(n, nb):  # row blocks: every kernel sees < 2^31 elements
        for X, dv, ov in ((K, 2.0 / h, -1.0 / h), (M, 4.0 * h / 6.0, h / 6.0)):
            Xr = X[r0:r1]
            Xr.zero_()
            Xr.diagonal(r0).fill_(dv)
            Xr.diagonal(r0 + 1).fill_(ov)   # (i, r0 + i + 1): super-diagonal
            Xr.diagonal(r0 - 1).fill_(ov)   # (i, r0 + i - 1): sub-diagonal
    return K, M


def fem_eigs(n: int, s: int):
    """Closed form of the s smallest eigenpairs of ``fem_pencil(n)``.

    lam_j = (6/h^2) (1 - cos(j pi h)) / (2 + cos(j pi h)),
    x_j[k] = sqrt(6 / (2 + cos(j pi h))) sin(j (k+1) pi h) (M-normalised),
    j = 1..s, ascending.  Returns (lam (s,), X (s, n) with row j-1 = x_j).
    1 - cos(t) is evaluated as 2 sin^2(t/2): for small j pi h the difference
    would cancel most digits (about 9 at n = 65536).
    """
    h = 1.0 / (n + 1)
    j = np.arange(1, s + 1, dtype=np.float64)
    c = np.cos(j * math.pi * h)
    lam = (6.0 / h**2) * (2.0 * np.sin(0.5 * j * math.pi * h) ** 2) / (2.0 + c)
    k = np.arange(1, n + 1, dtype=np.float64)
    X = np.sqrt(6.0 / (2.0 + c))[:, None] * np.sin(np.outer(j, k) * math.pi * h)
    return lam, X


# --------------------------------------------------------------------------
# start vector: SplitMix64 -> uniform [-1, 1)
# --------------------------------------------------------------------------
def splitmix64_uniform(n: int, seed: int) -> np.ndarray:
    """v[i] = 2 * (splitmix64(seed, i) >> 11) * 2^-53 - 1, i = 0..n-1.

    splitmix64(seed, i): z = seed + (i + 1) * 0x9E3779B97F4A7C15 (mod 2^64);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9; z = (z ^ (z >> 27)) *
    0x94D049BB133111EB; z ^= z >> 31.
    """
    with np.errstate(over="ignore"):
        i = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(int(seed) & _MASK64) + i * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0


def diagonal_pencil(n: int, seed: int = BASE_SEED, stream=(9,)):
    """A = diag(a), B = diag(b) with a ~ U[-1, 1], b ~ U[0.5, 2]."""
    g = rng(seed, *stream)
    a = g.uniform(-1.0, 1.0, size=n)
    b = g.uniform(0.5, 2.0, size=n)
    return np.diag(a), np.diag(b), a, b


def random_symmetric(n: int, seed: int = BASE_SEED, stream=(8,)):
    g = rng(seed, *stream)
    S = g.standard_normal((n, n))
    return 0.5 * (S + S.T)


def random_spd(n: int, seed: int = BASE_SEED, stream=(7,), shift: float = 1.0):
    g = rng(seed, *stream)
    S = g.standard_normal((n, n)) / math.sqrt(n)
    return S @ S.T + shift * np.eye(n)
