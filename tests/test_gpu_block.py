"""Block Lanczos (opts.block = 16 or 32) with thick restart: parity of
gsyeig_solve / gsyeig_lanczos against the CPU oracle and the generators'
known answers, in FP64 and mixed precision, with and without restarts.

Bars: the same as the single-vector path -- eigenvalues |dl| <= 1e-10
max|l|, per-pair backward error eta <= 1e-12 (FP64) or <= 1e-10 (mixed,
after the FP64 refinement), ||I - X^T B X||_F <= 1e-10, eigenvectors within
1e-8 (FP64) or within the residual / gap bound (mixed) of the oracle's."""
import sys

import numpy as np
import pytest

import gen
from test_gpu_mixed import x_error_bound

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def gs(torch):
    import paper_1111_6374_amd as gs

    gs.lib()
    return gs


@pytest.fixture(scope="module")
def solver(gs, torch):
    s = gs.Solver()
    yield s
    s.close()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def solve(gs, torch, solver, A, B, s, **kw):
    o = gs.gsyeig_opts_default()
    for k, v in kw.items():
        setattr(o, k, v)
    Lam, X, info = solver.solve(dev(torch, A), dev(torch, B), s, o)
    torch.cuda.synchronize()
    return Lam.cpu().numpy(), X.cpu().numpy(), info


def align(X, Xref):
    sgn = np.sign(np.sum(X * Xref, axis=1))
    sgn[sgn == 0] = 1
    return sgn[:, None] * Xref


@pytest.mark.parametrize("n,s,block,basis,law,which", [
    (512, 10, 16, 0, "spaced", 0),
    (512, 10, 32, 0, "spaced", 0),
    (777, 12, 16, 96, "spaced", 0),       # restarts: basis 96, 24 kept
    (1000, 20, 32, 160, "clustered", 0),  # restarts, clustered spectrum
    (600, 8, 16, 0, "spaced", 1),         # largest
])
def test_block_fp64_vs_oracle(gs, torch, solver, orc, n, s, block, basis, law, which):
    say("block fp64", n, s, block, basis, law, which)
    d = gen.known_spectrum(n, law, seed=gen.BASE_SEED, stream=(60, n, block, which))
    lam, X, info = solve(gs, torch, solver, d["A"], d["B"], s, block=block, basis=basis, which=which)
    assert info["rc"] == 0, info
    full = np.sort(d["lam"])
    lam_true = full[:s] if which == 0 else full[n - s:]
    mx = np.abs(d["lam"]).max()
    assert np.max(np.abs(lam - lam_true)) <= 1e-10 * mx
    lam_o, X_o = orc.gsyeig(d["A"], d["B"], s, which="largest" if which else "smallest")
    assert np.max(np.abs(lam - lam_o)) <= 1e-10 * mx
    m = orc.metrics(d["A"], d["B"], lam, X)
    assert m["eta_max"] <= 1e-12 and m["omega"] <= 1e-10
    m["xnorm"] = np.linalg.norm(X, axis=1)
    bnd = x_error_bound(d, lam, m) + 1e-10 * np.linalg.norm(X_o, axis=1)
    assert np.all(np.linalg.norm(X - align(X, X_o), axis=1) <= bnd)
    assert info["steps"] % block == 0 and info["converged"] >= s
    if basis:
        assert info["restarts"] >= 1 and info["basis"] == basis
        assert info["kept"] >= s


def test_block_and_single_vector_agree(gs, torch, solver):
    n, s = 900, 15
    d = gen.known_spectrum(n, "spaced", seed=gen.BASE_SEED, stream=(61,))
    say("block vs single", n, s)
    lam1, X1, i1 = solve(gs, torch, solver, d["A"], d["B"], s)
    lam2, X2, i2 = solve(gs, torch, solver, d["A"], d["B"], s, block=16)
    assert i1["rc"] == 0 and i2["rc"] == 0
    mx = np.abs(d["lam"]).max()
    assert np.max(np.abs(lam1 - lam2)) <= 1e-10 * mx
    m = {"eta": np.full(s, max(i1["eta_max"], i2["eta_max"])), "xnorm": np.linalg.norm(X2, axis=1)}
    assert np.all(np.linalg.norm(X1 - align(X1, X2), axis=1) <= 2 * x_error_bound(d, lam2, m) + 1e-12)


@pytest.mark.parametrize("n,s,block,basis,acc32,law", [
    (1024, 20, 16, 0, 0, "spaced"),
    (1024, 20, 32, 0, 1, "spaced"),       # FP32 accumulation in the block products
    (1500, 30, 16, 160, 0, "clustered"),  # restarts
])
def test_block_mixed_vs_known(gs, torch, solver, orc, n, s, block, basis, acc32, law):
    say("block mixed", n, s, block, basis, acc32, law)
    d = gen.known_spectrum(n, law, seed=gen.BASE_SEED, stream=(62, n, block))
    B0 = d["B"].copy()
    lam, X, info = solve(gs, torch, solver, d["A"], d["B"], s, prec=gs.GSYEIG_MIXED, block=block, basis=basis,
                         block_acc32=acc32)
    assert info["rc"] == 0, info
    assert np.array_equal(d["B"], B0)
    mx = np.abs(d["lam"]).max()
    assert np.max(np.abs(lam - np.sort(d["lam"])[:s])) <= 1e-10 * mx
    m = orc.metrics(d["A"], d["B"], lam, X)
    assert m["eta_max"] <= 1e-10 and m["omega"] <= 1e-10 and info["eta_max"] <= 1e-10
    lam_o, X_o = orc.gsyeig(d["A"], d["B"], s)
    assert np.max(np.abs(lam - lam_o)) <= 1e-10 * mx
    m["xnorm"] = np.linalg.norm(X, axis=1)
    bnd = x_error_bound(d, lam, m) + 1e-12 * np.linalg.norm(X_o, axis=1)
    assert np.all(np.linalg.norm(X - align(X, X_o), axis=1) <= bnd)
    if basis:
        assert info["restarts"] >= 1


@pytest.mark.parametrize("prec", [0, 1])
def test_block_inverse_pencil_fem(gs, torch, solver, prec):
    """The 1-D FEM pencil through the inverse pencil with block Lanczos:
    closed-form eigenvalues and sine modes."""
    n, s = 1000, 12
    K, M = gen.fem_pencil(n)
    lam_ref, X_ref = gen.fem_eigs(n, s)
    say("block invert fem", n, s, prec)
    lam, X, info = solve(gs, torch, solver, K, M, s, prec=prec, invert=1, block=16)
    assert info["rc"] == 0, info
    assert np.max(np.abs(lam - lam_ref) / lam_ref) <= 1e-9
    assert info["eta_max"] <= 1e-10 and info["omega"] <= 1e-10
    for i in range(s):
        sgn = np.sign(X[i] @ X_ref[i])
        assert np.max(np.abs(sgn * X[i] - X_ref[i])) <= 1e-6 * np.max(np.abs(X_ref[i]))


def test_block_identity_operator_breakdown(gs, torch, solver):
    """A = B: C = I, so the first block spans an invariant subspace and every
    later block is a breakdown; all eigenvalues are 1."""
    n, s = 300, 6
    B = gen.random_spd(n, seed=63)
    say("block identity", n, s)
    lam, X, info = solve(gs, torch, solver, B, B.copy(), s, block=16)
    assert info["rc"] == 0, info
    assert np.max(np.abs(lam - 1.0)) <= 1e-12
    assert info["eta_max"] <= 1e-12 and info["omega"] <= 1e-10


def test_block_lanczos_entry(gs, torch, solver, orc):
    """gsyeig_lanczos with block = 16 on a given FP64 factor: Ritz values of
    C = U^-T A U^-1 and orthonormal Ritz vectors Y with U^-1 Y the pencil's."""
    n, s = 640, 9
    d = gen.known_spectrum(n, seed=gen.BASE_SEED, stream=(64,))
    A, U = dev(torch, d["A"]), dev(torch, d["U"])
    o = gs.gsyeig_opts_default()
    o.block = 16
    th = torch.zeros(s, dtype=torch.float64, device="cuda")
    Y = torch.zeros(s, n, dtype=torch.float64, device="cuda")
    say("block lanczos entry", n, s)
    rc, steps = gs.gsyeig_lanczos(solver.ctx, n, s, A, n, U, n, o, th, Y, n)
    torch.cuda.synchronize()
    assert rc == 0 and steps % 16 == 0
    lam = th.cpu().numpy()
    assert np.max(np.abs(lam - np.sort(d["lam"])[:s])) <= 1e-10 * np.abs(d["lam"]).max()
    Yh = Y.cpu().numpy()
    assert np.linalg.norm(Yh @ Yh.T - np.eye(s)) <= 1e-12


@pytest.mark.parametrize("kw", [dict(block=65), dict(block=16, basis=40, keep=30), dict(block=-2)])
def test_block_rejects_bad_sizes(gs, torch, solver, kw):
    n, s = 200, 5
    d = gen.known_spectrum(n, seed=gen.BASE_SEED, stream=(65,))
    o = gs.gsyeig_opts_default()
    for k, v in kw.items():
        setattr(o, k, v)
    Lam = torch.zeros(s, dtype=torch.float64, device="cuda")
    X = torch.zeros(s, n, dtype=torch.float64, device="cuda")
    rc, _ = gs.gsyeig_solve(solver.ctx, n, s, dev(torch, d["A"]), n, dev(torch, d["B"]), n, o, Lam, X, n)
    assert rc == -8
