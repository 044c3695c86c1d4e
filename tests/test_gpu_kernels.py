"""GPU parity of every hot-path step against the CPU oracle, through the C ABI.

Sizes span several 64-wide tiles with ragged tails; tolerances are the
backward-error bounds of each operation (FP64, unit roundoff u = 2^-53)."""
import sys

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


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


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


# --------------------------------------------------------------- GS1 (Eq. 2)
@pytest.mark.parametrize("n", [1, 5, 64, 65, 130, 257, 700])
def test_potrf_matches_oracle(gs, ctx, torch, orc, n):
    say("potrf", n)
    d = gen.known_spectrum(n, seed=101, stream=(n,))
    B = dev(torch, d["B"])
    assert gs.gsyeig_potrf(ctx, n, B, n) == 0
    Bh = host(B)
    U_ref = orc.cholesky_upper(d["B"])
    tol = 64 * n * U64 * np.max(np.abs(U_ref))
    assert np.max(np.abs(np.triu(Bh) - U_ref)) <= tol
    # strict lower triangle untouched
    assert np.array_equal(np.tril(Bh, -1), np.tril(d["B"], -1))


def test_potrf_reports_failing_minor(gs, ctx, torch):
    n = 150
    Bn = gen.random_spd(n, seed=102)
    Bn[97, 97] = -5.0  # leading minor 98 indefinite
    say("potrf-fail", n)
    B = dev(torch, Bn)
    rc = gs.gsyeig_potrf(ctx, n, B, n)
    assert 1 <= rc <= 98
    d = gen.known_spectrum(70, seed=3)
    assert gs.gsyeig_potrf(ctx, 70, dev(torch, d["B"]), 70) == 0  # context still usable


def test_potrf_leading_dimension(gs, ctx, torch, orc):
    n, ld = 100, 131
    d = gen.known_spectrum(n, seed=103)
    Bp = np.zeros((n, ld))
    Bp[:, :n] = d["B"]
    B = dev(torch, Bp)
    say("potrf-ld", n, ld)
    assert gs.gsyeig_potrf(ctx, n, B, ld) == 0
    Bh = host(B)
    assert np.max(np.abs(np.triu(Bh[:, :n]) - orc.cholesky_upper(d["B"]))) <= 1e-12
    assert np.array_equal(Bh[:, n:], Bp[:, n:])


# --------------------------------------------------------------- KI1 / KI3
@pytest.mark.parametrize("n", [1, 63, 64, 65, 200, 513, 1000, 1025, 4097])
@pytest.mark.parametrize("trans", [0, 1])
@pytest.mark.parametrize("block", [64, 512])
def test_trsv_matches_oracle(gs, ctx, torch, orc, n, trans, block):
    say("trsv", n, trans, block)
    assert gs.gsyeig_set_trsv_block(ctx, block) == 0
    d = gen.known_spectrum(n, seed=104, stream=(n,)) if n <= 600 else None
    U = d["U"] if d else gen.factor_U(n, gen.rng(104, n))
    b = gen.rng(105, n).standard_normal(n)
    Ud, bd = dev(torch, U), dev(torch, b)
    xd = torch.empty_like(bd)
    assert gs.gsyeig_trsv(ctx, n, Ud, n, trans, bd, xd) == 0
    x = host(xd)
    ref = orc.trsv_upper(U, b) if trans == 0 else orc.trsv_upper_t(U, b)
    assert np.max(np.abs(x - ref)) <= 64 * n * U64 * np.max(np.abs(ref))
    # in place (x aliases b), repeated launches reuse the control block
    for _ in range(3):
        bd2 = dev(torch, b)
        assert gs.gsyeig_trsv(ctx, n, Ud, n, trans, bd2, bd2) == 0
        assert np.array_equal(host(bd2), x)


@pytest.mark.parametrize("block", [64, 512])
def test_trsv_bidiagonal_closed_form(gs, ctx, torch, block):
    assert gs.gsyeig_set_trsv_block(ctx, block) == 0
    n = 1333
    U = np.eye(n) - np.eye(n, k=1)
    b = gen.rng(106).standard_normal(n)
    Ud, bd = dev(torch, U), dev(torch, b)
    xd = torch.empty_like(bd)
    say("trsv-bidiag", n)
    assert gs.gsyeig_trsv(ctx, n, Ud, n, 0, bd, xd) == 0
    assert np.allclose(host(xd), np.cumsum(b[::-1])[::-1], rtol=0, atol=1e-12)
    assert gs.gsyeig_trsv(ctx, n, Ud, n, 1, bd, xd) == 0
    assert np.allclose(host(xd), np.cumsum(b), rtol=0, atol=1e-12)


# --------------------------------------------------------------- KI2
@pytest.mark.parametrize("n", [1, 64, 65, 300, 1000, 2049])
def test_symv_matches_oracle(gs, ctx, torch, orc, n):
    say("symv", n)
    A = gen.random_symmetric(n, seed=107, stream=(n,))
    x = gen.rng(108, n).standard_normal(n)
    Ad, xd = dev(torch, A), dev(torch, x)
    yd = torch.empty_like(xd)
    assert gs.gsyeig_symv(ctx, n, Ad, n, xd, yd) == 0
    ref = orc.matvec(A, x)
    assert np.max(np.abs(host(yd) - ref)) <= 4 * n * U64 * np.max(np.abs(A)) * np.sum(np.abs(x))


def test_symv_reads_only_upper_triangle(gs, ctx, torch, orc):
    n = 190
    A = gen.random_symmetric(n, seed=109)
    Apoison = np.triu(A) + np.tril(np.full((n, n), np.nan), -1)
    # the diagonal tiles are read in full storage: keep their lower part valid
    for I in range(0, n, 64):
        J = min(n, I + 64)
        Apoison[I:J, I:J] = A[I:J, I:J]
    x = gen.rng(110).standard_normal(n)
    yd = torch.empty(n, dtype=torch.float64, device="cuda")
    say("symv-upper", n)
    assert gs.gsyeig_symv(ctx, n, dev(torch, Apoison), n, dev(torch, x), yd) == 0
    assert np.allclose(host(yd), orc.matvec(A, x), rtol=1e-12, atol=1e-12)


def test_symv_rank_one(gs, ctx, torch):
    n = 257
    x = gen.rng(111).standard_normal(n)
    yd = torch.empty(n, dtype=torch.float64, device="cuda")
    say("symv-rank1", n)
    assert gs.gsyeig_symv(ctx, n, dev(torch, np.ones((n, n))), n, dev(torch, x), yd) == 0
    assert np.allclose(host(yd), np.full(n, x.sum()), rtol=0, atol=1e-12)


# --------------------------------------------------------------- KI1-KI3
@pytest.mark.parametrize("n", [65, 500, 1600])
@pytest.mark.parametrize("block", [64, 512])
def test_apply_op_matches_oracle_and_known_c(gs, ctx, torch, orc, n, block):
    say("apply_op", n, block)
    assert gs.gsyeig_set_trsv_block(ctx, block) == 0
    d = gen.known_spectrum(n, seed=112, stream=(n,))
    w = gen.rng(113, n).standard_normal(n)
    zd = torch.empty(n, dtype=torch.float64, device="cuda")
    assert gs.gsyeig_apply_op(ctx, n, dev(torch, d["A"]), n, dev(torch, d["U"]), n, dev(torch, w), zd) == 0
    z = host(zd)
    assert np.max(np.abs(z - orc.apply_ki(d["A"], d["U"], w))) <= 1e-12 * np.max(np.abs(w))
    C = (d["Y"] * d["lam"]) @ d["Y"].T
    assert np.max(np.abs(z - C @ w)) <= 1e-12 * np.max(np.abs(w)) * n ** 0.5


@pytest.mark.parametrize("n", [65, 4097, 16384])
def test_apply_op_equals_separate_calls_bitwise(gs, ctx, torch, n):
    """The operator's KI3 takes KI2's tile partials and sums them itself, in
    the order of the standalone SYMV's reduction, so gsyeig_apply_op must be
    bit-for-bit U^-T (A (U^-1 w)) computed by three separate calls (FP64,
    512-row super-blocks); the same for the FP32-storage sweeps."""
    say("apply_op bitwise", n)
    assert gs.gsyeig_set_trsv_block(ctx, 512) == 0
    if n <= 4097:
        d = gen.known_spectrum(n, seed=115, stream=(n,))
        A, U = dev(torch, d["A"]), dev(torch, d["U"])
    else:
        d = gen.known_spectrum_device(n, seed=115, stream=(n,), device="cuda")
        A, U = d["A"], d["U"]
    w = dev(torch, gen.rng(116, n).standard_normal(n))
    z = torch.empty(n, dtype=torch.float64, device="cuda")
    t1 = torch.empty_like(z)
    t2 = torch.empty_like(z)
    t3 = torch.empty_like(z)
    for _ in range(2):  # counters and staging reset themselves between launches
        assert gs.gsyeig_apply_op(ctx, n, A, n, U, n, w, z) == 0
        assert gs.gsyeig_trsv(ctx, n, U, n, 0, w, t1) == 0
        assert gs.gsyeig_symv(ctx, n, A, n, t1, t2) == 0
        assert gs.gsyeig_trsv(ctx, n, U, n, 1, t2, t3) == 0
        assert gs.gsyeig_sync(ctx) == 0
        assert torch.equal(z, t3)
    # FP32 storage: the mixed-precision operator against its own three calls
    A32 = A.float().contiguous()
    U32 = torch.triu(U).float().contiguous()
    z32 = torch.empty_like(z)
    assert gs.gsyeig_trsv_lp(ctx, n, U32, n, 0, w, t1) == 0
    assert gs.gsyeig_symv_lp(ctx, n, A32, n, t1, t2) == 0
    assert gs.gsyeig_trsv_lp(ctx, n, U32, n, 1, t2, t3) == 0
    assert gs.gsyeig_apply_op_lp(ctx, n, A32, n, U32, n, w, z32) == 0
    assert torch.equal(z32, t3)


def test_expired_wait_is_reported_once(gs, ctx, torch):
    """A chained wait that runs out is reported as GSYEIG_ESPIN by the call
    whose kernels it hit, and only by that call: a spin bound of one poll
    (set from the host) forces expiries in a healthy sweep, every kernel
    still finishes, and after the bound is restored the next calls succeed
    with correct results."""
    n = 8192
    say("espin", n)
    assert gs.gsyeig_set_trsv_block(ctx, 512) == 0
    d = gen.known_spectrum(2048, seed=117)
    U32 = dev(torch, np.triu(d["U"])).float().contiguous()
    U32 = torch.block_diag(U32, U32, U32, U32)
    Uh = U32.double().cpu().numpy()
    b = dev(torch, gen.rng(118).standard_normal(n))
    x = torch.empty_like(b)
    assert gs.gsyeig_set_spin_limit(ctx, 1) == 0
    rc = gs.gsyeig_trsv_lp(ctx, n, U32, n, 1, b, x)
    assert gs.gsyeig_set_spin_limit(ctx, 0) == 0
    assert rc == gs.GSYEIG_ESPIN
    # record cleared and the control blocks reset: the next calls are clean
    assert gs.gsyeig_sync(ctx) == 0
    for trans in (0, 1):
        assert gs.gsyeig_trsv_lp(ctx, n, U32, n, trans, b, x) == 0
        xr = host(x)
        Ut = Uh if trans == 0 else Uh.T
        res = Ut @ xr - host(b)
        assert np.max(np.abs(res)) <= 1e-5 * np.max(np.abs(host(b)))
    # asynchronous calls report through gsyeig_sync
    Ud = U32.double().contiguous()
    assert gs.gsyeig_set_spin_limit(ctx, 1) == 0
    assert gs.gsyeig_trsv(ctx, n, Ud, n, 1, b, x) == 0
    assert gs.gsyeig_sync(ctx) == gs.GSYEIG_ESPIN
    assert gs.gsyeig_set_spin_limit(ctx, 0) == 0
    assert gs.gsyeig_sync(ctx) == 0
    assert gs.gsyeig_trsv(ctx, n, Ud, n, 1, b, x) == 0
    assert gs.gsyeig_sync(ctx) == 0
    assert np.max(np.abs(Uh.T @ host(x) - host(b))) <= 1e-10 * np.max(np.abs(host(b)))


# --------------------------------------------------------------- KI4
@pytest.mark.parametrize("n,k", [(300, 20), (129, 60), (1100, 30)])
def test_lanczos_recurrence_matches_oracle(gs, ctx, torch, orc, n, k):
    say("lanczos_run", n, k)
    assert gs.gsyeig_set_trsv_block(ctx, 512) == 0
    d = gen.known_spectrum(n, seed=114, stream=(n,))
    v0 = gen.splitmix64_uniform(n, 17)
    a_ref, b_ref, W_ref = orc.lanczos(d["A"], d["U"], v0, k)
    alpha = torch.zeros(k, dtype=torch.float64, device="cuda")
    beta = torch.zeros(k, dtype=torch.float64, device="cuda")
    V = torch.zeros(k + 1, n, dtype=torch.float64, device="cuda")
    rc = gs.gsyeig_lanczos_run(ctx, n, k, dev(torch, d["A"]), n, dev(torch, d["U"]), n,
                               dev(torch, v0), alpha, beta, V, n)
    assert rc == 0
    a, b, W = host(alpha), host(beta), host(V)
    # rounding divergence grows slowly with k; first steps agree to ~1e-13 ||C||
    assert np.max(np.abs(a[:10] - a_ref[:10])) <= 1e-12
    assert np.max(np.abs(b[:10] - b_ref[:10])) <= 1e-12
    assert np.max(np.abs(W @ W.T - np.eye(k + 1))) <= 1e-13
    T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
    C = (d["Y"] * d["lam"]) @ d["Y"].T
    R = C @ W[:k].T - W[:k].T @ T
    R[:, -1] -= b[-1] * W[k]
    assert np.max(np.abs(R)) <= 1e-12


# --------------------------------------------------------------- KI5 (eigen part)
@pytest.mark.parametrize("m,nwant,which", [(1, 1, 0), (7, 3, 0), (200, 10, 0), (200, 10, 1), (1500, 40, 0)])
def test_tridiag_eig_matches_oracle(gs, ctx, torch, orc, m, nwant, which):
    say("tridiag", m, nwant, which)
    g = gen.rng(115, m)
    a = g.uniform(-1, 1, m)
    b = g.uniform(0.1, 1.0, max(m - 1, 1))
    th = torch.empty(nwant, dtype=torch.float64, device="cuda")
    S = torch.empty(nwant, m, dtype=torch.float64, device="cuda")
    assert gs.gsyeig_tridiag_eig(ctx, m, dev(torch, a), dev(torch, b), nwant, which, th, S, m) == 0
    w = orc.tridiag_eigvals(a, b[: m - 1])
    ref = w[:nwant] if which == 0 else w[-nwant:]
    tn = np.max(np.abs(w))
    theta = host(th)
    assert np.max(np.abs(theta - ref)) <= 8 * U64 * m * tn
    Sh = host(S).T  # m x nwant
    T = np.diag(a) + np.diag(b[: m - 1], 1) + np.diag(b[: m - 1], -1)
    assert np.max(np.abs(T @ Sh - Sh * theta)) <= 1e-12 * tn * m ** 0.5
    assert np.max(np.abs(Sh.T @ Sh - np.eye(nwant))) <= 1e-12


def test_tridiag_eig_clustered(gs, ctx, torch, orc):
    # Toeplitz tridiagonal with tiny spacing at the bottom of a long chain:
    # neighbouring eigenvalues closer than 1e-3 ||T|| form one cluster
    m, nwant = 2000, 25
    a = np.full(m, 2.0)
    b = np.full(m - 1, -1.0)
    th = torch.empty(nwant, dtype=torch.float64, device="cuda")
    S = torch.empty(nwant, m, dtype=torch.float64, device="cuda")
    say("tridiag-cluster", m, nwant)
    assert gs.gsyeig_tridiag_eig(ctx, m, dev(torch, a), dev(torch, b), nwant, 0, th, S, m) == 0
    j = np.arange(1, nwant + 1)
    ref = 2 - 2 * np.cos(j * np.pi / (m + 1))
    theta = host(th)
    assert np.max(np.abs(theta - ref)) <= 1e-13
    Sh = host(S).T
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    assert np.max(np.abs(T @ Sh - Sh * theta)) <= 1e-12
    assert np.max(np.abs(Sh.T @ Sh - np.eye(nwant))) <= 1e-11


# --------------------------------------------------------------- BT1 (Eq. 4)
@pytest.mark.parametrize("n,s", [(1, 1), (65, 3), (300, 10), (1000, 37)])
def test_backsolve_matches_oracle(gs, ctx, torch, orc, n, s):
    say("backsolve", n, s)
    U = gen.factor_U(n, gen.rng(116, n))
    Y = gen.rng(117, n).standard_normal((s, n))
    Yd = dev(torch, Y)
    assert gs.gsyeig_backsolve(ctx, n, s, dev(torch, U), n, Yd, n) == 0
    ref = orc.backsolve(U, Y)
    assert np.max(np.abs(host(Yd) - ref)) <= 64 * n * U64 * np.max(np.abs(ref))


# --------------------------------------------------------------- check metrics
def test_check_matches_oracle_metrics(gs, ctx, torch, orc):
    n, s = 400, 6
    d = gen.known_spectrum(n, seed=118)
    lam, X = orc.gsyeig(d["A"], d["B"], s)
    lam_p = lam * (1 + 1e-9 * np.arange(s))  # make the residuals non-trivial
    ref = orc.metrics(d["A"], d["B"], lam_p, X)
    say("check", n, s)
    rc, info = gs.gsyeig_check(ctx, n, s, dev(torch, d["A"]), n, dev(torch, d["B"]), n, None,
                               dev(torch, lam_p), dev(torch, X), n)
    assert rc == 0
    assert abs(info.eta_max - ref["eta_max"]) <= 1e-6 * ref["eta_max"] + 1e-18
    assert abs(info.rho_f - ref["rho_F"]) <= 1e-6 * ref["rho_F"] + 1e-18
    assert abs(info.omega - ref["omega"]) <= 1e-13
    assert abs(info.normA_f - np.linalg.norm(d["A"])) <= 1e-12 * info.normA_f
    # lower-triangle + saved diagonal form of B (the state after gsyeig_potrf)
    Bl = np.tril(d["B"], -1) + np.triu(np.full((n, n), np.nan))
    rc, info2 = gs.gsyeig_check(ctx, n, s, dev(torch, d["A"]), n, dev(torch, Bl), n,
                                dev(torch, np.diag(d["B"]).copy()), dev(torch, lam_p), dev(torch, X), n)
    assert rc == 0
    assert abs(info2.eta_max - info.eta_max) <= 1e-10 * info.eta_max
    assert abs(info2.normB_f - info.normB_f) <= 1e-12 * info.normB_f


@pytest.mark.parametrize("n", [1537, 4097])
def test_sweep_kinds_agree(gs, ctx, torch, orc, n):
    """The four combinations of the two super-block sweep designs (work
    queue, one workgroup per tile) for KI1 and KI3 give the same solves and
    the same operator as the oracle; each design is bitwise reproducible."""
    say("sweep kinds", n)
    assert gs.gsyeig_set_trsv_block(ctx, 512) == 0
    U = gen.factor_U(n, gen.rng(120, n))
    A = gen.random_symmetric(n, seed=121)
    b = gen.rng(122, n).standard_normal(n)
    Ud, Ad, bd = dev(torch, U), dev(torch, A), dev(torch, b)
    ref = {0: orc.trsv_upper(U, b), 1: orc.trsv_upper_t(U, b), 2: orc.apply_ki(A, U, b)}
    out = {}
    for kind in range(4):
        assert gs.gsyeig_set_trsv_sweep(ctx, kind) == 0
        for t in (0, 1, 2):
            x = torch.empty_like(bd)
            x2 = torch.empty_like(bd)
            if t < 2:
                assert gs.gsyeig_trsv(ctx, n, Ud, n, t, bd, x) == 0
                assert gs.gsyeig_trsv(ctx, n, Ud, n, t, bd, x2) == 0
            else:
                assert gs.gsyeig_apply_op(ctx, n, Ad, n, Ud, n, bd, x) == 0
                assert gs.gsyeig_apply_op(ctx, n, Ad, n, Ud, n, bd, x2) == 0
            assert gs.gsyeig_sync(ctx) == 0
            assert torch.equal(x, x2)
            xh = host(x)
            scale = np.max(np.abs(ref[t]))
            assert np.max(np.abs(xh - ref[t])) <= 64 * n * U64 * max(scale, 1.0) * (10.0 if t == 2 else 1.0)
            out[(kind, t)] = xh
    assert gs.gsyeig_set_trsv_sweep(ctx, 0) == 0
    assert gs.gsyeig_set_trsv_sweep(ctx, 4) == -2
    for kind in (1, 2, 3):
        for t in (0, 1, 2):
            assert np.max(np.abs(out[(kind, t)] - out[(0, t)])) <= 1e-12 * max(np.max(np.abs(out[(0, t)])), 1.0)
