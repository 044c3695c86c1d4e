"""Partial re-orthogonalisation (opts.reorth = 2): the omega recurrence
decides on the device which Lanczos steps orthogonalise against all of V,
and the Ritz vectors are taken in an orthonormal basis of the semi-
orthogonal V_m.  Results must meet the same bars as full re-orthogonalisation
(eigenvalues |dl| <= 1e-10 max|l| against the generator's and the oracle's,
eta <= 1e-12 and ||I - X^T B X||_F <= 1e-10 in FP64, the refined bars in mixed
mode), with far fewer orthogonalising steps than Lanczos steps."""
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


@pytest.mark.parametrize("n,s,law,which", [
    (1500, 30, "spaced", 0),
    (1500, 30, "clustered", 0),
    (2100, 40, "spaced", 0),
    (1200, 16, "spaced", 1),
    (777, 12, "clustered", 1),
])
def test_pro_fp64_vs_oracle(gs, torch, solver, orc, n, s, law, which):
    say("pro fp64", n, s, law, which)
    d = gen.known_spectrum(n, law, seed=gen.BASE_SEED, stream=(70, n, which))
    lam, X, info = solve(gs, torch, solver, d["A"], d["B"], s, reorth=2, which=which)
    assert info["rc"] == 0, info
    full = np.sort(d["lam"])
    lam_true = full[:s] if which == 0 else full[n - s:]
    mx = np.abs(d["lam"]).max()
    assert np.max(np.abs(lam - lam_true)) <= 1e-10 * mx
    m = orc.metrics(d["A"], d["B"], lam, X)
    assert m["eta_max"] <= 1e-12 and m["omega"] <= 1e-10
    assert info["eta_max"] <= 1e-12 and info["omega"] <= 1e-10
    lam_o, X_o = orc.gsyeig(d["A"], d["B"], s, which="largest" if which else "smallest")
    assert np.max(np.abs(lam - lam_o)) <= 1e-10 * mx
    m["xnorm"] = np.linalg.norm(X, axis=1)
    bnd = x_error_bound(d, lam, m) + 1e-10 * np.linalg.norm(X_o, axis=1)
    assert np.all(np.linalg.norm(X - align(X, X_o), axis=1) <= bnd)
    # orthogonalising steps come in pairs and are a minority
    assert 0 <= info["reorth_steps"] < info["steps"]


def test_pro_matches_full_reorthogonalisation(gs, torch, solver):
    n, s = 2000, 25
    d = gen.known_spectrum(n, "clustered", seed=gen.BASE_SEED, stream=(71,))
    say("pro vs full", n, s)
    lam1, X1, i1 = solve(gs, torch, solver, d["A"], d["B"], s, reorth=1)
    lam2, X2, i2 = solve(gs, torch, solver, d["A"], d["B"], s, reorth=2)
    assert i1["rc"] == 0 and i2["rc"] == 0
    mx = np.abs(d["lam"]).max()
    assert np.max(np.abs(lam1 - lam2)) <= 1e-12 * mx
    m = {"eta": np.full(s, max(i1["eta_max"], i2["eta_max"])), "xnorm": np.linalg.norm(X2, axis=1)}
    assert np.all(np.linalg.norm(X1 - align(X1, X2), axis=1) <= 2 * x_error_bound(d, lam2, m) + 1e-12)
    assert i2["reorth_steps"] < i2["steps"] // 2
    say("reorth steps", i1["reorth_steps"], i2["reorth_steps"], "of", i1["steps"], i2["steps"])


@pytest.mark.parametrize("n,s,law", [(1024, 20, "spaced"), (1500, 30, "clustered")])
def test_pro_mixed(gs, torch, solver, orc, n, s, law):
    say("pro mixed", n, s, law)
    d = gen.known_spectrum(n, law, seed=gen.BASE_SEED, stream=(72, n))
    lam, X, info = solve(gs, torch, solver, d["A"], d["B"], s, prec=gs.GSYEIG_MIXED, reorth=2)
    assert info["rc"] == 0, info
    mx = np.abs(d["lam"]).max()
    assert np.max(np.abs(lam - np.sort(d["lam"])[:s])) <= 1e-10 * mx
    m = orc.metrics(d["A"], d["B"], lam, X)
    assert m["eta_max"] <= 1e-10 and m["omega"] <= 1e-10 and info["eta_max"] <= 1e-10
    assert info["reorth_steps"] < info["steps"]


def test_pro_inverse_pencil_fem(gs, torch, solver):
    n, s = 1000, 12
    K, M = gen.fem_pencil(n)
    lam_ref, X_ref = gen.fem_eigs(n, s)
    say("pro invert fem", n, s)
    lam, X, info = solve(gs, torch, solver, K, M, s, invert=1, reorth=2)
    assert info["rc"] == 0, info
    assert np.max(np.abs(lam - lam_ref) / lam_ref) <= 1e-9
    assert info["eta_max"] <= 1e-10 and info["omega"] <= 1e-10


def test_pro_lanczos_entry(gs, torch, solver):
    """gsyeig_lanczos with reorth = 2: orthonormal Ritz vectors Y of C."""
    n, s = 900, 10
    d = gen.known_spectrum(n, "spaced", seed=gen.BASE_SEED, stream=(73,))
    o = gs.gsyeig_opts_default()
    o.reorth = 2
    th = torch.zeros(s, dtype=torch.float64, device="cuda")
    Y = torch.zeros(s, n, dtype=torch.float64, device="cuda")
    say("pro lanczos entry", n, s)
    rc, steps = gs.gsyeig_lanczos(solver.ctx, n, s, dev(torch, d["A"]), n, dev(torch, d["U"]), n, o, th, Y, n)
    torch.cuda.synchronize()
    assert rc == 0
    lam = th.cpu().numpy()
    assert np.max(np.abs(lam - np.sort(d["lam"])[:s])) <= 1e-10 * np.abs(d["lam"]).max()
    Yh = Y.cpu().numpy()
    assert np.linalg.norm(Yh @ Yh.T - np.eye(s)) <= 1e-12
    # Ritz residuals of C = U^-T A U^-1 (host FP64)
    Ui = np.linalg.inv(d["U"])
    C = Ui.T @ d["A"] @ Ui
    r = np.linalg.norm(Yh @ C - lam[:, None] * Yh, axis=1)
    assert r.max() <= 1e-11 * np.abs(d["lam"]).max()


@pytest.mark.parametrize("bad", [-1, 3])
def test_reorth_out_of_range_rejected(gs, torch, solver, bad):
    n, s = 100, 3
    d = gen.known_spectrum(n, seed=gen.BASE_SEED, stream=(74,))
    o = gs.gsyeig_opts_default()
    o.reorth = bad
    Lam = torch.zeros(s, dtype=torch.float64, device="cuda")
    X = torch.zeros(s, n, dtype=torch.float64, device="cuda")
    rc, _ = gs.gsyeig_solve(solver.ctx, n, s, dev(torch, d["A"]), n, dev(torch, d["B"]), n, o, Lam, X, n)
    assert rc == -8


@pytest.mark.parametrize("reorth", [1, 2])
def test_identity_pencil_single_vector(gs, torch, solver, reorth):
    """A = B: C = I, so every beta_k is at rounding level (breakdown at each
    step); the orthogonalised rounding noise carries the recurrence on and
    every eigenvalue is 1."""
    n, s = 300, 6
    B = gen.random_spd(n, seed=75)
    say("identity single", n, s, reorth)
    lam, X, info = solve(gs, torch, solver, B, B.copy(), s, reorth=reorth)
    assert info["rc"] == 0, info
    assert np.max(np.abs(lam - 1.0)) <= 1e-12
    assert info["eta_max"] <= 1e-12 and info["omega"] <= 1e-10
