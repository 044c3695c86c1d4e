"""Mixed-precision path on the GPU, through the C ABI, against the CPU oracle.

* FP32-storage sweeps: SYMV with FP32 A computes in FP64, so it matches the
  oracle on the same FP32 values promoted to FP64 to FP64 accuracy; the
  triangular sweeps keep the off-diagonal factor blocks (W = D^-1 U_offdiag)
  in FP32 and agree with the oracle to FP32 accuracy.
* Mixed GS1 (FP32 trailing updates) and the FP32 block solves: FP32-level
  agreement with the FP64 oracle.
* The small dense eigensolver of the refinement: FP64 agreement with the
  oracle's QL eigensolver.
* The refinement and the whole mixed solve: the FP64 bar of the pencil --
  eigenvalues equal to the known spectrum and to the FP64 oracle within
  1e-10 max|lambda|, per-pair backward error eta <= 1e-10, X^T B X = I.
"""
import sys

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53
U32 = 2.0 ** -24


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
def ctx(gs, torch):
    rc, c = gs.gsyeig_create(torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    yield c
    gs.gsyeig_destroy(c)


def dev(torch, a, dtype=None):
    import torch as t

    a = np.ascontiguousarray(a)
    return t.from_numpy(a).cuda() if dtype is None else t.from_numpy(a.astype(dtype)).cuda()


def host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def x_error_bound(d, lam, m):
    """Per-pair bound on ||x_i - x_i*||_2 from the residual (Davis-Kahan in the
    B-inner product): sqrt(2) ||r_i||_{B^-1} / gap_i with ||r||_{B^-1} <=
    ||r||_2 / s_min(U) and ||.||_2 <= ||.||_B / s_min(U), B = U^T U;
    ||r_i||_2 = eta_i (||A||_F + |lam_i| ||B||_F) ||x_i||_2 and gap_i is the
    distance from lam_i to the rest of the known spectrum."""
    full = np.sort(d["lam"])
    smin = np.linalg.svd(d["U"], compute_uv=False)[-1]
    nA, nB = np.linalg.norm(d["A"]), np.linalg.norm(d["B"])
    out = []
    for i, l in enumerate(lam):
        j = int(np.argmin(np.abs(full - l)))
        gap = np.min(np.abs(np.delete(full, j) - full[j]))
        r = m["eta"][i] * (nA + abs(l) * nB) * m["xnorm"][i]
        out.append(np.sqrt(2.0) * r / (smin * smin * gap))
    return np.array(out)


def factor(n, seed_stream):
    return gen.factor_U(n, gen.rng(gen.BASE_SEED, *seed_stream))


# ------------------------------------------------------- FP32-storage sweeps
@pytest.mark.parametrize("n", [1, 65, 513, 1100, 2049])
@pytest.mark.parametrize("trans", [0, 1])
def test_trsv_lp_equals_promoted_oracle(gs, ctx, torch, orc, n, trans):
    say("trsv_lp", n, trans)
    U = f32(factor(n, (31, n)))
    b = gen.rng(gen.BASE_SEED, 32, n).standard_normal(n)
    Ud = dev(torch, U, np.float32)
    bd = dev(torch, b)
    xd = torch.zeros(n, dtype=torch.float64, device="cuda")
    assert gs.gsyeig_trsv_lp(ctx, n, Ud, n, trans, bd, xd) == 0
    x = host(xd)
    ref = orc.trsv_upper_t(U, b) if trans else orc.trsv_upper(U, b)
    # the sweeps apply U = D (I + W) with W = D^-1 U_offdiag stored in FP32
    # (D: 512-row diagonal blocks, inverted in FP64): FP32-level agreement
    err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    assert err <= 64 * U32, err


@pytest.mark.parametrize("n", [1, 63, 64, 65, 700, 2049])
def test_symv_lp_equals_promoted_oracle(gs, ctx, torch, orc, n):
    say("symv_lp", n)
    A = f32(gen.random_symmetric(n, stream=(33, n)))
    x = gen.rng(gen.BASE_SEED, 34, n).standard_normal(n)
    Ad = dev(torch, A, np.float32)
    yd = torch.zeros(n, dtype=torch.float64, device="cuda")
    assert gs.gsyeig_symv_lp(ctx, n, Ad, n, dev(torch, x), yd) == 0
    y = host(yd)
    ref = orc.matvec(A, x)
    bound = 4 * n * U64 * (np.abs(A) @ np.abs(x))
    assert np.all(np.abs(y - ref) <= bound + 1e-300)


@pytest.mark.parametrize("n,k", [(65, 1), (600, 7), (1100, 70), (1537, 33)])
@pytest.mark.parametrize("trans", [0, 1])
def test_trsm_lp_fp32_block_solve(gs, ctx, torch, orc, n, k, trans):
    say("trsm_lp", n, k, trans)
    U = f32(factor(n, (35, n)))
    V = gen.rng(gen.BASE_SEED, 36, n, k).standard_normal((k, n))  # rows = columns of the block
    Ud = dev(torch, U, np.float32)
    Vd = dev(torch, V)
    V_before = V.copy()
    Xd = torch.zeros(k, n, dtype=torch.float64, device="cuda")
    assert gs.gsyeig_trsm_lp(ctx, n, Ud, n, trans, k, Vd, n, Xd, n) == 0
    X = host(Xd)
    assert np.array_equal(host(Vd), V_before)
    for j in range(k):
        ref = orc.trsv_upper_t(U, V[j]) if trans else orc.trsv_upper(U, V[j])
        err = np.linalg.norm(X[j] - ref) / np.linalg.norm(ref)
        # FP32 products with FP32 accumulation: error of order u_32 kappa
        assert err <= 2e-4, (j, err)


# --------------------------------------------------------------- mixed GS1
@pytest.mark.parametrize("n", [1, 63, 64, 65, 300, 1100])
def test_potrf_mixed(gs, ctx, torch, orc, n):
    say("potrf_mixed", n)
    d = gen.known_spectrum(n, seed=gen.BASE_SEED, stream=(37, n))
    B = d["B"]
    Bd = dev(torch, B)
    Ud = torch.full((n, n), 7.0, dtype=torch.float32, device="cuda")
    o = gs.gsyeig_opts_default()
    o.prec = gs.GSYEIG_MIXED
    assert gs.gsyeig_potrf(ctx, n, Bd, n, o, Ud) == 0
    assert np.array_equal(host(Bd), B)  # B only read
    U = host(Ud).astype(np.float64)
    assert np.all(np.tril(U, -1) == 0.0)
    assert np.all(np.diag(U) > 0)
    res = np.linalg.norm(U.T @ U - B) / np.linalg.norm(B)
    assert res <= 20 * max(1, n) ** 0.5 * U32, res
    U64ref = orc.cholesky_upper(B)
    assert np.linalg.norm(U - U64ref) / np.linalg.norm(U64ref) <= 1e-5


def test_potrf_mixed_reports_the_failing_minor(gs, ctx, torch):
    n = 150
    B = gen.random_spd(n, stream=(38,))
    B[97, 97] = -1.0
    o = gs.gsyeig_opts_default()
    o.prec = gs.GSYEIG_MIXED
    Ud = torch.zeros(n, n, dtype=torch.float32, device="cuda")
    assert gs.gsyeig_potrf(ctx, n, dev(torch, B), n, o, Ud) == 98
    assert gs.gsyeig_potrf(ctx, n, dev(torch, B), n, o, None) == -6


# ------------------------------------------------ small dense eigensolver
def _syev_case(name, N):
    g = gen.rng(gen.BASE_SEED, 39, N)
    if name == "random":
        S = g.standard_normal((N, N))
        return 0.5 * (S + S.T)
    Q, _ = np.linalg.qr(g.standard_normal((N, N)))
    if name == "identity":
        return np.eye(N)
    if name == "repeated":  # three eigenvalues, each with multiplicity ~N/3
        w = np.repeat([-1.0, 0.5, 2.0], (N + 2) // 3)[:N]
    else:  # clustered: N values within 1e-6 of 1, plus a spread tail
        w = np.concatenate([1.0 + 1e-6 * g.random(N // 2), 10 * g.random(N - N // 2)])
    return (Q * w[None, :]) @ Q.T


@pytest.mark.parametrize("N,nwant,which,name", [
    (1, 1, 0, "random"), (2, 2, 0, "random"), (3, 1, 1, "random"), (17, 9, 0, "random"),
    (64, 64, 0, "random"), (200, 50, 1, "random"), (513, 300, 0, "random"),
    (40, 40, 0, "identity"), (96, 96, 0, "repeated"), (250, 125, 0, "clustered"), (500, 250, 0, "clustered"),
    # orders above 192 take the whole-GPU reduction (two launches per column)
    (300, 300, 0, "identity"), (260, 260, 0, "repeated"), (1500, 400, 0, "random"), (1200, 600, 1, "clustered"),
])
def test_syev_small(gs, ctx, torch, orc, N, nwant, which, name):
    say("syev_small", N, nwant, which, name)
    H = _syev_case(name, N)
    H = 0.5 * (H + H.T)
    Hd = dev(torch, H)
    wd = torch.zeros(nwant, dtype=torch.float64, device="cuda")
    Qd = torch.zeros(nwant, N, dtype=torch.float64, device="cuda")  # column-major N x nwant
    assert gs.gsyeig_syev_small(ctx, N, Hd, N, nwant, which, wd, Qd, N) == 0
    assert np.array_equal(host(Hd), H)
    w = host(wd)
    Q = host(Qd).T
    wref, _ = orc.eig_sym(H)
    ref = wref[:nwant] if which == 0 else wref[N - nwant:]
    nH = max(np.abs(wref).max(), 1e-300)
    assert np.all(np.diff(w) >= 0)
    assert np.max(np.abs(w - ref)) <= 50 * N * U64 * nH
    assert np.linalg.norm(Q.T @ Q - np.eye(nwant)) <= 100 * N * U64
    assert np.linalg.norm(H @ Q - Q * w[None, :]) <= 100 * N * U64 * nH


# ----------------------------------------------------------- refinement (a8)
def _perturbed_start(d, s, k, which, scale, stream):
    """U^-1 times the exact y-space eigenvectors of the k extreme eigenvalues,
    perturbed by `scale` (relative) -- a stand-in for FP32-sweep Ritz vectors."""
    lam = d["lam"]
    order = np.argsort(lam, kind="stable")
    idx = order[:k] if which == 0 else order[len(lam) - k:]
    Y = d["Y"][:, idx]
    Y = Y + scale * gen.rng(gen.BASE_SEED, *stream).standard_normal(Y.shape) / np.sqrt(Y.shape[0])
    X0 = np.linalg.solve(d["U"], Y)  # test input only: U^-1 Y
    return X0


@pytest.mark.parametrize("n,s,k,law,which,scale", [
    (400, 12, 20, "spaced", 0, 1e-3),
    (700, 30, 40, "clustered", 0, 1e-4),
    (700, 10, 16, "spaced", 1, 1e-5),
    (1100, 40, 50, "clustered", 0, 0.0),
])
def test_refine_reaches_fp64(gs, ctx, torch, orc, n, s, k, law, which, scale):
    say("refine", n, s, k, law, which, scale)
    d = gen.known_spectrum(n, law, seed=gen.BASE_SEED, stream=(40, n, which))
    A, B = d["A"], d["B"]
    Ad, Bd = dev(torch, A), dev(torch, B)
    o = gs.gsyeig_opts_default()
    o.prec = gs.GSYEIG_MIXED
    o.which = which
    U32d = torch.zeros(n, n, dtype=torch.float32, device="cuda")
    assert gs.gsyeig_potrf(ctx, n, Bd, n, o, U32d) == 0
    X0 = _perturbed_start(d, s, k, which, scale, (41, n))
    X0d = dev(torch, X0.T.copy())  # k x n rows = columns
    Lam = torch.zeros(s, dtype=torch.float64, device="cuda")
    Xd = torch.zeros(s, n, dtype=torch.float64, device="cuda")
    rc, info = gs.gsyeig_refine(ctx, n, s, k, Ad, n, Bd, n, U32d, n, o, X0d, n, Lam, Xd, n)
    assert rc == 0, (rc, info.as_dict())
    lam = host(Lam)
    X = host(Xd)
    lam_true = np.sort(d["lam"])
    lam_true = lam_true[:s] if which == 0 else lam_true[n - s:]
    mx = np.abs(d["lam"]).max()
    assert np.max(np.abs(lam - lam_true)) <= 1e-10 * mx
    m = orc.metrics(A, B, lam, X)
    assert m["eta_max"] <= 1e-10 and info.eta_max <= 1e-10
    assert m["omega"] <= 1e-10
    assert np.array_equal(host(Ad), A) and np.array_equal(host(Bd), B)


# ---------------------------------------------------- whole mixed solve
@pytest.mark.parametrize("n,s,law,which", [
    (512, 10, "spaced", 0),
    (1500, 40, "clustered", 0),
    (1000, 20, "spaced", 1),
    (2049, 60, "clustered", 0),
])
def test_mixed_solve_matches_fp64_oracle(gs, ctx, torch, orc, n, s, law, which):
    say("mixed solve", n, s, law, which)
    d = gen.known_spectrum(n, law, seed=gen.BASE_SEED, stream=(42, n, which))
    A, B = d["A"], d["B"]
    o = gs.gsyeig_opts_default()
    o.prec = gs.GSYEIG_MIXED
    o.which = which
    Ad, Bd = dev(torch, A), dev(torch, B)
    Lam = torch.zeros(s, dtype=torch.float64, device="cuda")
    Xd = torch.zeros(s, n, dtype=torch.float64, device="cuda")
    rc, info = gs.gsyeig_solve(ctx, n, s, Ad, n, Bd, n, o, Lam, Xd, n)
    assert rc == 0, (rc, info.as_dict())
    assert np.array_equal(host(Bd), B)  # mixed mode leaves B intact
    lam, X = host(Lam), host(Xd)
    mx = np.abs(d["lam"]).max()
    lam_true = np.sort(d["lam"])
    lam_true = lam_true[:s] if which == 0 else lam_true[n - s:]
    assert np.max(np.abs(lam - lam_true)) <= 1e-10 * mx
    m = orc.metrics(A, B, lam, X)
    assert m["eta_max"] <= 1e-10 and info.eta_max <= 1e-10
    assert m["omega"] <= 1e-10
    assert info.refine_iters <= o.refine_iters and info.block_cols >= s
    # the FP64 oracle on the same pencil (n <= 1500 keeps it to seconds):
    # eigenvalues to 1e-10, eigenvectors to the residual / gap bound
    if n <= 1500:
        lam_o, X_o = orc.gsyeig(A, B, s, which="largest" if which else "smallest")
        assert np.max(np.abs(lam - lam_o)) <= 1e-10 * mx
        m["xnorm"] = np.linalg.norm(X, axis=1)
        bnd = x_error_bound(d, lam, m) + 1e-12 * np.linalg.norm(X_o, axis=1)
        assert np.all(np.linalg.norm(X - X_o, axis=1) <= bnd)


def test_mixed_and_fp64_modes_agree(gs, ctx, torch):
    n, s = 1200, 25
    d = gen.known_spectrum(n, "spaced", seed=gen.BASE_SEED, stream=(43,))
    A = dev(torch, d["A"])
    res = {}
    for prec in (gs.GSYEIG_FP64, gs.GSYEIG_MIXED):
        say("mode", prec)
        o = gs.gsyeig_opts_default()
        o.prec = prec
        with gs.Solver() as sv:
            lam, X, info = sv.solve(A, dev(torch, d["B"]), s, o)
        assert info["rc"] == 0
        res[prec] = (host(lam), host(X), info["eta_max"])
    mx = np.abs(d["lam"]).max()
    assert np.max(np.abs(res[0][0] - res[1][0])) <= 1e-10 * mx
    # both modes lie within their residual / gap bounds of the exact vectors
    lam1, X1, _ = res[1]
    m = {"eta": np.full(s, max(res[0][2], res[1][2])), "xnorm": np.linalg.norm(X1, axis=1)}
    bnd = 2 * x_error_bound(d, lam1, m)
    assert np.all(np.linalg.norm(res[0][1] - X1, axis=1) <= bnd)


def test_mixed_batched_equals_single(gs, torch):
    sizes = [300, 700, 450, 64]
    ss = [max(1, int(np.ceil(0.05 * n))) for n in sizes]
    insts = [gen.known_spectrum(n, seed=gen.BASE_SEED, stream=(44, i)) for i, n in enumerate(sizes)]
    o = gs.gsyeig_opts_default()
    o.prec = gs.GSYEIG_MIXED
    o.batch_mode = 1  # each instance a gsyeig_solve: bit for bit
    A = [dev(torch, d["A"]) for d in insts]
    B = [dev(torch, d["B"]) for d in insts]
    Lam = [torch.zeros(s, dtype=torch.float64, device="cuda") for s in ss]
    X = [torch.zeros(s, n, dtype=torch.float64, device="cuda") for s, n in zip(ss, sizes)]
    say("mixed batched", sizes)
    with gs.Solver() as sv:
        rc, status, infos = gs.gsyeig_solve_batched(sv.ctx, sizes, ss, A, sizes, B, sizes, o, Lam, X, sizes,
                                                    nstreams=3)
    torch.cuda.synchronize()
    assert rc == 0 and all(st == 0 for st in status)
    with gs.Solver() as sv:
        for i, (n, s) in enumerate(zip(sizes, ss)):
            lam1, X1, info = sv.solve(A[i], B[i], s, o)
            torch.cuda.synchronize()
            assert torch.equal(lam1, Lam[i]) and torch.equal(X1, X[i]), i
            assert infos[i].eta_max <= 1e-10


# ------------------------------------------------------ inverse pencil (A SPD)
@pytest.mark.parametrize("prec", [0, 1])
def test_inverse_pencil_fem_closed_form(gs, ctx, torch, prec):
    """FEM stiffness/mass pair: the s smallest eigenvalues through (B, A)
    equal the closed form; X is B-orthonormal and matches the sine modes."""
    n, s = 900, 8
    K, M = gen.fem_pencil(n)
    lam_ref, X_ref = gen.fem_eigs(n, s)
    say("invert fem", n, s, prec)
    o = gs.gsyeig_opts_default()
    o.prec = prec
    o.invert = 1
    Kd, Md = dev(torch, K), dev(torch, M)
    Lam = torch.zeros(s, dtype=torch.float64, device="cuda")
    Xd = torch.zeros(s, n, dtype=torch.float64, device="cuda")
    rc, info = gs.gsyeig_solve(ctx, n, s, Kd, n, Md, n, o, Lam, Xd, n)
    assert rc == 0, (rc, info.as_dict())
    assert np.array_equal(host(Kd), K) and np.array_equal(host(Md), M)
    lam, X = host(Lam), host(Xd)
    # closed form to the FP64 normwise bound (the tests of the oracle use the same)
    assert np.max(np.abs(lam - lam_ref) / lam_ref) <= 1e-9
    assert info.eta_max <= 1e-10 and info.omega <= 1e-10
    for i in range(s):  # sine modes: compare up to sign (ties in magnitude)
        sgn = np.sign(X[i] @ X_ref[i])
        assert np.max(np.abs(sgn * X[i] - X_ref[i])) <= 1e-6 * np.max(np.abs(X_ref[i]))


@pytest.mark.parametrize("prec", [0, 1])
def test_inverse_pencil_matches_direct(gs, ctx, torch, orc, prec):
    n, s = 800, 12
    d = gen.known_spectrum(n, "clustered", seed=gen.BASE_SEED, stream=(45, prec))  # lambda > 0: A SPD
    say("invert known", n, s, prec)
    o = gs.gsyeig_opts_default()
    o.prec = prec
    o.invert = 1
    Lam = torch.zeros(s, dtype=torch.float64, device="cuda")
    Xd = torch.zeros(s, n, dtype=torch.float64, device="cuda")
    rc, info = gs.gsyeig_solve(ctx, n, s, dev(torch, d["A"]), n, dev(torch, d["B"]), n, o, Lam, Xd, n)
    assert rc == 0, (rc, info.as_dict())
    lam = host(Lam)
    mx = np.abs(d["lam"]).max()
    assert np.max(np.abs(lam - np.sort(d["lam"])[:s])) <= 1e-10 * mx
    m = orc.metrics(d["A"], d["B"], lam, host(Xd))
    assert m["eta_max"] <= 1e-10 and m["omega"] <= 1e-10


def test_inverse_pencil_rejects_indefinite_a(gs, ctx, torch):
    n, s = 200, 4
    d = gen.known_spectrum(n, "spaced", seed=gen.BASE_SEED, stream=(46,))  # lambda in [-1, 1]: A indefinite
    o = gs.gsyeig_opts_default()
    o.invert = 1
    Lam = torch.zeros(s, dtype=torch.float64, device="cuda")
    Xd = torch.zeros(s, n, dtype=torch.float64, device="cuda")
    rc, _ = gs.gsyeig_solve(ctx, n, s, dev(torch, d["A"]), n, dev(torch, d["B"]), n, o, Lam, Xd, n)
    assert 1 <= rc <= n


@pytest.mark.parametrize("N,nwant,width", [(600, 600, 1e-7), (1000, 1000, 1e-9), (800, 300, 1e-12)])
def test_syev_small_gram_like_cluster(gs, ctx, torch, orc, N, nwant, width):
    """Gram-like matrices (all eigenvalues within `width` of 1, as the
    refinement's B-Gram matrices of nearly B-orthonormal blocks): the
    eigenvectors must come out orthonormal with small residuals whichever
    path (Cholesky QR or the clustered fallback) produced them."""
    g = gen.rng(gen.BASE_SEED, 41, N)
    Q, _ = np.linalg.qr(g.standard_normal((N, N)))
    w_true = 1.0 + width * (2.0 * g.random(N) - 1.0)
    H = (Q * w_true[None, :]) @ Q.T
    H = 0.5 * (H + H.T)
    say("syev_small gram-like", N, nwant, width)
    wd = torch.zeros(nwant, dtype=torch.float64, device="cuda")
    Qd = torch.zeros(nwant, N, dtype=torch.float64, device="cuda")
    assert gs.gsyeig_syev_small(ctx, N, dev(torch, H), N, nwant, 0, wd, Qd, N) == 0
    w, V = host(wd), host(Qd).T
    assert np.max(np.abs(w - np.sort(w_true)[:nwant])) <= 50 * N * U64
    assert np.linalg.norm(V.T @ V - np.eye(nwant)) <= 100 * N * U64
    assert np.linalg.norm(H @ V - V * w[None, :]) <= 100 * N * U64


@pytest.mark.parametrize("n,lda", [(700, 704), (1000, 1024), (4100, 4160), (1000, 1004), (1002, 1002), (999, 1001)])
def test_symv_lp_leading_dimension(gs, ctx, torch, orc, n, lda):
    """FP32 SYMV with a padded leading dimension: the 16-byte-load kernel
    (lda, n multiples of 4), the 8-byte one (lda even) and the scalar one."""
    say("symv_lp ld", n, lda)
    A = f32(gen.random_symmetric(n, stream=(35, n)))
    Ap = np.full((n, lda), np.nan, dtype=np.float32)   # padding is never read
    Ap[:, :n] = A
    x = gen.rng(gen.BASE_SEED, 36, n).standard_normal(n)
    yd = torch.zeros(n, dtype=torch.float64, device="cuda")
    assert gs.gsyeig_symv_lp(ctx, n, torch.from_numpy(Ap).cuda(), lda, dev(torch, x), yd) == 0
    y = host(yd)
    ref = orc.matvec(A, x)
    bound = 4 * n * U64 * (np.abs(A) @ np.abs(x))
    assert np.all(np.abs(y - ref) <= bound + 1e-300)
