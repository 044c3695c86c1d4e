"""Pins for the CPU oracle: every check compares it with something other than
itself -- the generator's known answer, closed forms, a brute-force inertia
count, textbook special cases, or an independent library routine."""
import math

import numpy as np
import pytest
import scipy.linalg

import gen

U64 = 2.0 ** -53


# --------------------------------------------------------------- Eq. 2
@pytest.mark.parametrize("n", [1, 2, 7, 64, 129])
def test_cholesky_recovers_generator_factor(orc, n):
    d = gen.known_spectrum(n, seed=11)
    U = orc.cholesky_upper(d["B"])
    # the Cholesky factor with positive diagonal is unique
    assert np.allclose(np.tril(U, -1), 0.0)
    assert np.max(np.abs(U - d["U"])) <= 64 * n * U64 * np.max(np.abs(d["U"]))


def test_cholesky_reports_failing_minor(orc):
    B = np.diag([1.0, 2.0, -1.0, 3.0])
    with pytest.raises(np.linalg.LinAlgError, match="minor 3"):
        orc.cholesky_upper(B)
    B = np.array([[1.0, 2.0], [2.0, 1.0]])  # indefinite: second minor fails
    with pytest.raises(np.linalg.LinAlgError, match="minor 2"):
        orc.cholesky_upper(B)


# --------------------------------------------------------------- KI1/KI3
def test_trsv_bidiagonal_closed_form(orc):
    # U = I - superdiag  =>  U^-1 = all-ones upper triangle:  U^-1 b = suffix sums,
    # U^-T b = prefix sums.
    n = 37
    U = np.eye(n) - np.eye(n, k=1)
    b = gen.rng(3).standard_normal(n)
    assert np.allclose(orc.trsv_upper(U, b), np.cumsum(b[::-1])[::-1], rtol=0, atol=1e-13)
    assert np.allclose(orc.trsv_upper_t(U, b), np.cumsum(b), rtol=0, atol=1e-13)


@pytest.mark.parametrize("n", [1, 5, 100, 257])
def test_trsv_backward_error(orc, n):
    d = gen.known_spectrum(n, seed=5)
    U = d["U"]
    x = gen.rng(4).standard_normal(n)
    b = U @ x
    bt = U.T @ x
    # condition of U is O(1) for this generator, so forward error ~ n u
    assert np.max(np.abs(orc.trsv_upper(U, b) - x)) <= 100 * n * U64 * np.max(np.abs(x))
    assert np.max(np.abs(orc.trsv_upper_t(U, bt) - x)) <= 100 * n * U64 * np.max(np.abs(x))
    # library routine as an independent route
    ref = scipy.linalg.solve_triangular(U, b, lower=False)
    assert np.allclose(orc.trsv_upper(U, b), ref, rtol=1e-12, atol=1e-13)


# --------------------------------------------------------------- KI2
def test_matvec_rank_one(orc):
    n = 50
    A = np.ones((n, n))
    x = gen.rng(6).standard_normal(n)
    assert np.allclose(orc.matvec(A, x), np.full(n, x.sum()), rtol=0, atol=1e-13)


def test_apply_ki_equals_known_c(orc):
    n = 96
    d = gen.known_spectrum(n, seed=8)
    C = (d["Y"] * d["lam"]) @ d["Y"].T
    w = gen.rng(9).standard_normal(n)
    z = orc.apply_ki(d["A"], d["U"], w)
    assert np.max(np.abs(z - C @ w)) <= 1e-13 * np.max(np.abs(w)) * n ** 0.5


# --------------------------------------------------------------- Eq. 3
@pytest.mark.parametrize("n", [3, 64, 150])
def test_form_c_known_spectrum(orc, n):
    d = gen.known_spectrum(n, seed=12)
    U = orc.cholesky_upper(d["B"])
    C = orc.form_c(d["A"], U)
    C_ref = (d["Y"] * d["lam"]) @ d["Y"].T
    assert np.max(np.abs(C - C_ref)) <= 1e-13
    assert np.array_equal(C, C.T)


# --------------------------------------------------------------- eigensolvers
@pytest.mark.parametrize("method", ["ql", "jacobi"])
@pytest.mark.parametrize("n", [1, 2, 3, 10, 80])
def test_eig_sym_known_spectrum(orc, method, n):
    g = gen.rng(13, n)
    Y = gen.haar_Y(n, g)
    lam = gen.spectrum_spaced(n, g)
    C = (Y * lam) @ Y.T
    C = 0.5 * (C + C.T)
    w, Z = orc.eig_sym(C, method)
    order = np.argsort(lam)
    assert np.max(np.abs(w - lam[order])) <= 1e-13
    # eigenvectors equal +-Y columns (distinct eigenvalues)
    dots = np.abs(np.sum(Z * Y[:, order], axis=0))
    assert np.max(np.abs(dots - 1.0)) <= 1e-12
    assert np.max(np.abs(Z.T @ Z - np.eye(n))) <= 1e-12


@pytest.mark.parametrize("method", ["ql", "jacobi"])
def test_eig_sym_toeplitz_closed_form(orc, method):
    # tridiag(-1, 2, -1): lam_j = 2 - 2 cos(j pi/(n+1))
    n = 60
    C = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    w, Z = orc.eig_sym(C, method)
    j = np.arange(1, n + 1)
    assert np.max(np.abs(w - (2 - 2 * np.cos(j * math.pi / (n + 1))))) <= 1e-13
    assert np.max(np.abs(C @ Z - Z * w)) <= 1e-13


def test_eig_sym_vs_library(orc):
    C = gen.random_symmetric(120, seed=14)
    w, Z = orc.eig_sym(C, "ql")
    assert np.max(np.abs(w - np.linalg.eigvalsh(C))) <= 1e-12 * np.max(np.abs(w))
    assert np.max(np.abs(C @ Z - Z * w)) <= 1e-12 * np.max(np.abs(w))


def test_eig_sym_repeated_eigenvalues(orc):
    # identity plus a rank-one term: eigenvalue 1 with multiplicity n-1
    n = 30
    v = gen.rng(15).standard_normal(n)
    C = np.eye(n) + np.outer(v, v)
    for method in ("ql", "jacobi"):
        w, Z = orc.eig_sym(C, method)
        assert np.max(np.abs(w[:-1] - 1.0)) <= 1e-13 * (1 + v @ v)
        assert abs(w[-1] - (1 + v @ v)) <= 1e-13 * (1 + v @ v)
        assert np.max(np.abs(Z.T @ Z - np.eye(n))) <= 1e-12


def test_tridiag_eigvals_closed_form(orc):
    m = 45
    w = orc.tridiag_eigvals(np.full(m, 2.0), np.full(m - 1, -1.0))
    j = np.arange(1, m + 1)
    assert np.max(np.abs(w - (2 - 2 * np.cos(j * math.pi / (m + 1))))) <= 1e-13


# --------------------------------------------------------------- Eq. 1-4, the definition
@pytest.mark.parametrize("n,s", [(1, 1), (5, 2), (64, 10), (200, 10), (300, 25)])
@pytest.mark.parametrize("method", ["ql", "jacobi"])
def test_gsyeig_known_spectrum(orc, n, s, method):
    if method == "jacobi" and n > 200:
        pytest.skip("Jacobi cross-check kept to small n")
    d = gen.known_spectrum(n, seed=21, stream=(n,))
    lam, X = orc.gsyeig(d["A"], d["B"], s, method=method)
    order = np.argsort(d["lam"], kind="stable")[:s]
    assert np.max(np.abs(lam - d["lam"][order])) <= 1e-13
    # X = U^-1 Y_s, computed here with a library triangular solve
    X_ref = scipy.linalg.solve_triangular(d["U"], d["Y"][:, order], lower=False).T
    X_ref = orc.sign_normalise_rows(X_ref)
    assert np.max(np.abs(X - X_ref)) <= 1e-11
    m = orc.metrics(d["A"], d["B"], lam, X, d["lam"][order])
    assert m["eta_max"] <= 1e-14
    assert m["omega"] <= 1e-12
    # sign convention
    for x in X:
        assert x[np.argmax(np.abs(x))] > 0


def test_gsyeig_largest(orc):
    n, s = 90, 7
    d = gen.known_spectrum(n, seed=22)
    lam, X = orc.gsyeig(d["A"], d["B"], s, which="largest")
    assert np.max(np.abs(lam - np.sort(d["lam"])[-s:])) <= 1e-13


@pytest.mark.parametrize("n,s", [(50, 8), (200, 10)])
def test_gsyeig_fem_closed_form(orc, n, s):
    K, M = gen.fem_pencil(n)
    lam, X = orc.gsyeig(K, M, s)
    lam_ref, X_ref = gen.fem_eigs(n, s)
    # normwise backward-stable bound: |dlam| <= c u ||C||_2, ||C||_2 < 12/h^2
    h = 1.0 / (n + 1)
    assert np.max(np.abs(lam - lam_ref)) <= 20 * U64 * 12.0 / h**2
    # sine modes have entries of exactly equal magnitude and opposite sign, so
    # the largest-entry sign rule is decided by rounding: align signs instead
    sgn = np.sign(np.sum(X * X_ref, axis=1))
    assert np.max(np.abs(X - sgn[:, None] * X_ref)) <= 1e-9 * np.max(np.abs(X_ref))
    assert abs(lam[0] - math.pi ** 2) / math.pi ** 2 < 1e-3


@pytest.mark.parametrize("n", [1, 3, 12, 40, 64])
def test_gsyeig_vs_brute_force_inertia(orc, n):
    # every eigenvalue by bisection on the inertia of A - sigma B: no Cholesky, no QL/Jacobi
    A = gen.random_symmetric(n, seed=31, stream=(n,))
    B = gen.random_spd(n, seed=32, stream=(n,))
    lam, _ = orc.gsyeig(A, B, n)
    lam_bf = orc.bisect_eigs(A, B, range(n))
    assert np.max(np.abs(lam - lam_bf)) <= 1e-12 * max(1.0, np.max(np.abs(lam)))


def test_inertia_diagonal_pencil(orc):
    n = 25
    A, B, a, b = gen.diagonal_pencil(n, seed=33)
    for sigma in (-0.7, -0.1, 0.0, 0.3, 1.5):
        assert orc.inertia_below(A, B, sigma) == int(np.sum(a / b < sigma))


def test_inertia_needs_2x2_pivots(orc):
    # zero diagonal forces Bunch-Parlett 2x2 pivots: [[0, 1], [1, 0]] has one
    # negative eigenvalue; a 4x4 block version has two.
    A = np.array([[0.0, 1.0], [1.0, 0.0]])
    assert orc.inertia_below(A, np.eye(2), 0.0) == 1
    A4 = np.kron(np.eye(2), A)
    assert orc.inertia_below(A4, np.eye(4), 0.0) == 2
    assert orc.inertia_below(A4, np.eye(4), 1.5) == 4
    assert orc.inertia_below(A4, np.eye(4), -1.5) == 0


def test_special_case_standard_problem(orc):
    n, s = 70, 6
    A = gen.random_symmetric(n, seed=34)
    lam, X = orc.gsyeig(A, np.eye(n), s)
    w, V = np.linalg.eigh(A)
    assert np.max(np.abs(lam - w[:s])) <= 1e-12 * np.max(np.abs(w))
    assert np.max(np.abs(np.abs(np.sum(X.T * V[:, :s], axis=0)) - 1)) <= 1e-10


def test_special_case_diagonal_pencil(orc):
    n, s = 40, 9
    A, B, a, b = gen.diagonal_pencil(n, seed=35)
    lam, X = orc.gsyeig(A, B, s)
    r = a / b
    order = np.argsort(r, kind="stable")[:s]
    assert np.max(np.abs(lam - r[order])) <= 2 * U64 * np.max(np.abs(r))
    X_ref = np.zeros((s, n))
    X_ref[np.arange(s), order] = 1.0 / np.sqrt(b[order])
    assert np.max(np.abs(X - X_ref)) <= 1e-14


def test_special_case_n1(orc):
    lam, X = orc.gsyeig(np.array([[3.0]]), np.array([[4.0]]), 1)
    assert lam[0] == 0.75 and X[0, 0] == 0.5


def test_gsyeig_rejects_bad_args(orc):
    with pytest.raises(RuntimeError):
        orc.gsyeig(np.eye(3), np.eye(3), 4)
    with pytest.raises(np.linalg.LinAlgError):
        orc.gsyeig(np.eye(3), -np.eye(3), 1)


# --------------------------------------------------------------- Lanczos (KI1-KI4)
def test_lanczos_invariants_and_first_alpha(orc):
    n, k = 120, 40
    d = gen.known_spectrum(n, seed=41)
    C = (d["Y"] * d["lam"]) @ d["Y"].T
    v0 = gen.splitmix64_uniform(n, 7)
    alpha, beta, W = orc.lanczos(d["A"], d["U"], v0, k)
    w0 = v0 / np.linalg.norm(v0)
    assert abs(alpha[0] - w0 @ C @ w0) <= 1e-14
    assert np.max(np.abs(W @ W.T - np.eye(k + 1))) <= 1e-14
    T = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    Vk = W[:k].T
    R = C @ Vk - Vk @ T
    R[:, -1] -= beta[-1] * W[k]
    assert np.max(np.abs(R)) <= 1e-13 * np.max(np.abs(d["lam"]))
    assert np.all(beta > 0)


def test_lanczos_full_run_recovers_spectrum(orc):
    # n steps of Lanczos with full reorthogonalisation: eig(T_n) = eig(C)
    n = 40
    d = gen.known_spectrum(n, seed=42)
    alpha, beta, _ = orc.lanczos(d["A"], d["U"], gen.splitmix64_uniform(n, 3), n)
    w = orc.tridiag_eigvals(alpha, beta[:-1])
    assert np.max(np.abs(w - np.sort(d["lam"]))) <= 1e-12


def test_lanczos_ritz_values_converge_to_smallest(orc):
    n, k, s = 300, 150, 5
    d = gen.known_spectrum(n, seed=43)
    alpha, beta, _ = orc.lanczos(d["A"], d["U"], gen.splitmix64_uniform(n, 5), k)
    w = orc.tridiag_eigvals(alpha, beta[:-1])
    assert np.max(np.abs(w[:s] - np.sort(d["lam"])[:s])) <= 1e-10


# --------------------------------------------------------------- metrics
def test_metrics_on_exact_and_perturbed_pairs(orc):
    n, s = 120, 5
    K, M = gen.fem_pencil(n)
    lam, X = gen.fem_eigs(n, s)
    m = orc.metrics(K, M, lam, X, lam)
    assert m["eta_max"] <= 1e-14 and m["omega"] <= 1e-12 and m["e_lam"] == 0.0
    m2 = orc.metrics(K, M, lam * (1 + 1e-6), X, lam)
    assert m2["eta_max"] > 1e-10 and m2["e_lam"] > 1e-9


def test_metrics_hand_computed_2x2(orc):
    """eta_i, rho_F, omega and e_lam on a 2 x 2 pencil worked by hand (the
    definitions of the accuracy metrics of Tables 3 and 7 plus the per-pair
    backward error).  The pairs are not eigenpairs, ||x_i|| != 1,
    ||A||_F != ||A||_2 and ||B||_F != ||B||_2, so dropping ||x_i|| from eta,
    a 2-norm in place of a Frobenius norm, lambda in place of |lambda|, or
    the wrong normaliser of rho_F each changes a value below.

    A = [[2, 1], [1, 2]]  (||A||_F = sqrt 10, ||A||_2 = 3)
    B = diag(4, 1)        (||B||_F = sqrt 17, ||B||_2 = 4)
    x_1 = (1, 1), x_2 = (0, 2);  lam = (-1, 2)
    r_1 = A x_1 + B x_1 = (3, 3) + (4, 1) = (7, 4)   ||r_1|| = sqrt 65
    r_2 = A x_2 - 2 B x_2 = (2, 4) - (0, 4) = (2, 0) ||r_2|| = 2
    X^T B X = [[5, 2], [2, 4]]  ->  I - X^T B X = [[-4, -2], [-2, -3]]
    """
    A = np.array([[2.0, 1.0], [1.0, 2.0]])
    B = np.diag([4.0, 1.0])
    X = np.array([[1.0, 1.0], [0.0, 2.0]])  # rows are x_1, x_2
    lam = np.array([-1.0, 2.0])
    m = orc.metrics(A, B, lam, X, lam_ref=np.array([-1.5, 2.5]))
    r10, r17 = math.sqrt(10.0), math.sqrt(17.0)
    eta1 = math.sqrt(65.0) / ((r10 + 1.0 * r17) * math.sqrt(2.0))
    eta2 = 2.0 / ((r10 + 2.0 * r17) * 2.0)
    assert m["eta"][0] == pytest.approx(eta1, rel=1e-14)
    assert m["eta"][1] == pytest.approx(eta2, rel=1e-14)
    assert m["eta_max"] == pytest.approx(max(eta1, eta2), rel=1e-14)
    assert m["rho_F"] == pytest.approx(math.sqrt(65.0 + 4.0) / r17, rel=1e-14)
    assert m["omega"] == pytest.approx(math.sqrt(33.0), rel=1e-14)
    assert m["omega_paper"] == pytest.approx(math.sqrt(33.0) / r17, rel=1e-14)
    assert m["e_lam"] == pytest.approx(0.5 / 2.5, rel=1e-14)


def test_metrics_hand_computed_normaliser_max(orc):
    """rho_F divides by max(||A||_F, ||B||_F): with ||A||_F > ||B||_F the
    divisor switches to ||A||_F.  A = diag(3, 4) (||A||_F = 5), B = I
    (||B||_F = sqrt 2); x_1 = e_1, lam_1 = 1: r_1 = (2, 0), eta_1 =
    2 / (5 + sqrt 2), rho_F = 2 / 5, omega = 0."""
    A = np.diag([3.0, 4.0])
    B = np.eye(2)
    m = orc.metrics(A, B, np.array([1.0]), np.array([[1.0, 0.0]]))
    assert m["rho_F"] == pytest.approx(0.4, rel=1e-15)
    assert m["eta_max"] == pytest.approx(2.0 / (5.0 + math.sqrt(2.0)), rel=1e-15)
    assert m["omega"] == 0.0


def test_splitmix64_published_vector():
    # first outputs of SplitMix64 seeded with 0 (x = 0; next() adds the golden gamma first)
    i = np.arange(1, 4, dtype=np.uint64)
    v = gen.splitmix64_uniform(3, 0)
    expected_u64 = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    expected = [2.0 * ((x >> 11) * 2.0 ** -53) - 1.0 for x in expected_u64]
    assert np.array_equal(v, np.array(expected))
    assert i.dtype == np.uint64


def test_blocked_device_generator_known_spectrum(orc):
    """The row-blocked generator used for n beyond single-tensor kernels:
    the pencil's eigenvalues (oracle, FP64) are the drawn lam, A and B are
    exactly symmetric and B = U^T U is positive definite (run on the CPU
    device with blocks much smaller than n)."""
    torch = pytest.importorskip("torch")
    n = 200
    d = gen.known_spectrum_device_blocked(n, "clustered", stream=(99,), device="cpu", nb=48, rank=12)
    A, B = d["A"].numpy(), d["B"].numpy()
    assert np.array_equal(A, A.T) and np.array_equal(B, B.T)
    lam, _ = orc.gsyeig(A, B, n)
    assert np.max(np.abs(lam - np.sort(d["lam"]))) <= 1e-12 * np.abs(d["lam"]).max()


def test_fem_device_pencil_equals_host():
    torch = pytest.importorskip("torch")
    for n in (1, 2, 47, 130):
        K, M = gen.fem_pencil_device(n, "cpu", nb=16)
        K0, M0 = gen.fem_pencil(n)
        assert np.array_equal(K.numpy(), K0) and np.array_equal(M.numpy(), M0)
