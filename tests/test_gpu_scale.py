"""Parity at the scale of the mixed, blocked and batched workloads.

The oracle cannot solve these sizes, so each test checks what can be
computed one entry or one pair at a time: every eigenvalue against the
generator's exact spectrum (the pencils are built with a known spectrum,
A = U^T Y diag(lam) Y^T U), sampled pairs through the oracle's own
matrix-vector products (per-pair backward error) and back-substitution
(x_i = U^-1 y_i with the generator's Y), and, for the batched instances
small enough, the oracle's full solve.

* mixed precision at n = 32768 on the clustered law (80 % U[0,1], 20 %
  U[1,10]); s is reduced from 200 to bound the run time, n is not;
* block Lanczos (b = 32, mixed) at n = 47000, where n^2 > 2^31 and 32-bit
  element offsets would wrap; the instance comes from the row-blocked
  generator (Y = I - 2 Q Q^T, rank 256, an exact orthogonal similarity);
* the batched driver on sizes drawn from U{256..4096}, s = ceil(0.05 n).
"""
import math
import sys

import numpy as np
import pytest

import gen

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


def dk_bound(lam_all, lam_i, eta_i, nA, nB, xnorm, smin):
    """Davis-Kahan bound on ||x_i - x_i*||_2 in the B-inner product:
    sqrt(2) ||r_i||_{B^-1} / gap_i, with ||r||_{B^-1} <= ||r||_2 / s_min(U),
    ||.||_2 <= ||.||_B / s_min(U) (B = U^T U), ||r_i||_2 =
    eta_i (||A||_F + |lam_i| ||B||_F) ||x_i||_2 and gap_i the distance from
    lam_i to the rest of the known spectrum."""
    j = int(np.argmin(np.abs(lam_all - lam_i)))
    gap = np.min(np.abs(np.delete(lam_all, j) - lam_all[j]))
    r = eta_i * (nA + abs(lam_i) * nB) * xnorm
    return math.sqrt(2.0) * r / (smin * smin * gap)


def test_mixed_n32768_clustered(gs, torch, orc):
    n, s = 32768, 20
    say("scale-mixed-generate", n, s)
    inst = gen.known_spectrum_device(n, "clustered", seed=gen.BASE_SEED + 2, stream=(2, 7, 0), device="cuda",
                                     rng_kind="torch")
    A, B = inst["A"], inst["B"]
    o = gs.gsyeig_opts_default()
    o.prec = gs.GSYEIG_MIXED
    # the clustered law at small s needs more steps than 100 s + 2000 (the
    # smallest gaps among the wanted values are ~3e-7 of a spectrum of width 10)
    o.max_steps = 16000
    say("scale-mixed-solve", n, s)
    with gs.Solver() as sv:
        lam, X, info = sv.solve(A, B, s, opts=o)
    torch.cuda.synchronize()
    assert info["rc"] == 0, info
    lam = lam.cpu().numpy()
    order = np.argsort(inst["lam"], kind="stable")[:s]
    scale = np.max(np.abs(inst["lam"]))
    assert np.max(np.abs(lam - inst["lam"][order])) <= 1e-10 * scale
    assert info["eta_max"] <= 1e-10 and info["omega"] <= 1e-9
    say("scale-mixed-oracle-samples")
    A_h = A.cpu().numpy()
    B_h = B.cpu().numpy()
    U_h = inst["U"].cpu().numpy()
    X_h = X.cpu().numpy()
    nA, nB = np.linalg.norm(A_h), np.linalg.norm(B_h)
    lam_all = np.sort(inst["lam"])
    for i in (0, 7, s - 1):
        x = X_h[i]
        r = orc.matvec(A_h, x) - lam[i] * orc.matvec(B_h, x)
        eta = np.linalg.norm(r) / ((nA + abs(lam[i]) * nB) * np.linalg.norm(x))
        assert eta <= 1e-10, (i, eta)
        y = inst["Y"][:, int(order[i])].cpu().numpy()
        x_ref = orc.backsolve(U_h, y[None, :])[0]
        x_ref *= np.sign(x_ref @ x)
        # s_min(U) of this factor law is about 0.53 at every n (diagonal
        # U[1,2], strict upper N(0, 1/n)); 0.5 keeps the bound a bound
        bnd = dk_bound(lam_all, lam[i], max(eta, 1e-16), nA, nB, np.linalg.norm(x), 0.5)
        assert np.linalg.norm(x - x_ref) <= bnd + 1e-12 * np.linalg.norm(x_ref), (i, bnd)


def test_block_mixed_n47000_past_int32(gs, torch):
    n, s, blk = 47000, 10, 32
    assert n * n > 2**31
    say("scale-block-generate", n, s, blk)
    inst = gen.known_spectrum_device_blocked(n, "spaced", seed=gen.BASE_SEED + 3, stream=(3, 5, 0), device="cuda")
    A, B = inst["A"], inst["B"]
    torch.cuda.empty_cache()
    o = gs.gsyeig_opts_default()
    o.prec = gs.GSYEIG_MIXED
    o.block = blk
    say("scale-block-solve", n, s, blk)
    with gs.Solver() as sv:
        lam, X, info = sv.solve(A, B, s, opts=o)
    torch.cuda.synchronize()
    assert info["rc"] == 0, info
    lam = lam.cpu().numpy()
    lam_true = np.sort(inst["lam"])[:s]
    assert np.max(np.abs(lam - lam_true)) <= 1e-10 * np.max(np.abs(inst["lam"]))
    assert info["eta_max"] <= 1e-10 and info["omega"] <= 1e-9
    say("scale-block-host-samples")
    X_h = X.cpu().numpy()
    samples = (0, 4, s - 1)
    Ax = np.zeros((len(samples), n))
    Bx = np.zeros((len(samples), n))
    nA2 = nB2 = 0.0
    xs = X_h[list(samples)].T  # n x 3
    for r0 in range(0, n, 4096):  # host evaluation in row blocks
        r1 = min(n, r0 + 4096)
        Ab = A[r0:r1].cpu().numpy()
        Bb = B[r0:r1].cpu().numpy()
        Ax[:, r0:r1] = (Ab @ xs).T
        Bx[:, r0:r1] = (Bb @ xs).T
        nA2 += float(np.sum(Ab * Ab))
        nB2 += float(np.sum(Bb * Bb))
    nA, nB = math.sqrt(nA2), math.sqrt(nB2)
    for j, i in enumerate(samples):
        r = Ax[j] - lam[i] * Bx[j]
        eta = np.linalg.norm(r) / ((nA + abs(lam[i]) * nB) * np.linalg.norm(X_h[i]))
        assert eta <= 1e-10, (i, eta)
        # B-normalised
        assert abs(X_h[i] @ Bx[j] - 1.0) <= 1e-9


def test_batched_sizes_256_to_4096(gs, torch, orc):
    g = gen.rng(gen.BASE_SEED + 4, 1)
    sizes = [int(v) for v in g.integers(256, 4097, size=9)] + [4096, 256, 700, 1400]
    ss = [math.ceil(0.05 * n) for n in sizes]
    say("scale-batched-generate", sizes)
    insts = [gen.known_spectrum(n, seed=gen.BASE_SEED + 4, stream=(4, 1, i)) for i, n in enumerate(sizes)]
    A = [torch.from_numpy(d["A"]).cuda() for d in insts]
    B = [torch.from_numpy(d["B"]).cuda() for d in insts]
    Lam = [torch.zeros(s, dtype=torch.float64, device="cuda") for s in ss]
    X = [torch.zeros(s, n, dtype=torch.float64, device="cuda") for s, n in zip(ss, sizes)]
    o = gs.gsyeig_opts_default()
    o.prec = gs.GSYEIG_MIXED
    say("scale-batched-solve", len(sizes))
    with gs.Solver() as sv:
        rc, status, infos = gs.gsyeig_solve_batched(sv.ctx, sizes, ss, A, sizes, B, sizes, o, Lam, X, sizes,
                                                    nstreams=8)
    torch.cuda.synchronize()
    assert rc == 0 and all(st == 0 for st in status), status
    for i, (n, s) in enumerate(zip(sizes, ss)):
        lam = Lam[i].cpu().numpy()
        lam_true = np.sort(insts[i]["lam"])[:s]
        assert np.max(np.abs(lam - lam_true)) <= 1e-10 * np.max(np.abs(insts[i]["lam"])), (i, n)
        assert infos[i].eta_max <= 1e-10, (i, n, infos[i].eta_max)
        if n <= 1500:
            say("scale-batched-oracle", i, n, s)
            d = insts[i]
            lam_o, X_o = orc.gsyeig(d["A"], d["B"], s)
            Xh = X[i].cpu().numpy()
            assert np.max(np.abs(lam - lam_o)) <= 1e-10 * np.max(np.abs(lam_o))
            # both sides sign-normalised the same way: each vector within
            # its residual / gap bound of the oracle's
            m = orc.metrics(d["A"], d["B"], lam, Xh)
            nA, nB = np.linalg.norm(d["A"]), np.linalg.norm(d["B"])
            smin = np.linalg.svd(d["U"], compute_uv=False)[-1]
            lam_all = np.sort(d["lam"])
            for j in range(s):
                bnd = dk_bound(lam_all, lam[j], m["eta"][j], nA, nB, np.linalg.norm(Xh[j]), smin)
                err = np.linalg.norm(Xh[j] - X_o[j])
                assert err <= bnd + 1e-12 * np.linalg.norm(X_o[j]), (i, n, j, err, bnd)
