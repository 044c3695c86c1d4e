"""Variants KE (Section 2.3; Table 1 keys GS2 and KE) and TD (Section 2.2;
keys TD1-TD3) through the C ABI: the explicit C = U^-T A U^-1 against the
oracle's or_form_c element by element and against the generator's exact
C = Y diag(lam) Y^T; the KE solve (one symmetric product per Lanczos step)
and the TD solve (Householder tridiagonalisation of C) against the oracle's
solve and against the KI solve of the same pencil."""
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


@pytest.mark.parametrize("n,block", [(1, 512), (65, 512), (700, 512), (1500, 512), (1100, 64), (1537, 512)])
def test_form_c_matches_oracle(gs, ctx, torch, orc, n, block):
    say("form_c", n, block)
    assert gs.gsyeig_set_trsv_block(ctx, block) == 0
    d = gen.known_spectrum(n, seed=201, stream=(n,))
    C = torch.full((n, n + 3), float("nan"), dtype=torch.float64, device="cuda")
    assert gs.gsyeig_form_c(ctx, n, dev(torch, d["A"]), n, dev(torch, d["U"]), n, C, n + 3) == 0
    Ch = host(C)[:, :n]
    assert np.array_equal(Ch, Ch.T)  # exactly symmetric
    C_ref = orc.form_c(d["A"], d["U"])
    C_exact = (d["Y"] * d["lam"]) @ d["Y"].T
    scale = np.max(np.abs(C_exact))
    # two triangular solves with kappa(U) ~ 5: a few hundred n u of ||C||
    tol = 64 * n * U64 * scale
    assert np.max(np.abs(Ch - C_ref)) <= tol
    assert np.max(np.abs(Ch - C_exact)) <= tol
    assert gs.gsyeig_set_trsv_block(ctx, 512) == 0


@pytest.mark.parametrize("n,s,law,which", [(512, 10, "spaced", 0), (1500, 30, "clustered", 0),
                                           (1000, 20, "spaced", 1), (333, 7, "spaced", 0)])
def test_ke_solve_matches_oracle(gs, ctx, torch, orc, n, s, law, which):
    say("ke solve", n, s, law, which)
    d = gen.known_spectrum(n, law, seed=gen.BASE_SEED, stream=(202, n, which))
    o = gs.gsyeig_opts_default()
    o.variant = gs.GSYEIG_KE
    o.which = which
    Lam = torch.zeros(s, dtype=torch.float64, device="cuda")
    X = torch.zeros(s, n, dtype=torch.float64, device="cuda")
    rc, info = gs.gsyeig_solve(ctx, n, s, dev(torch, d["A"]), n, dev(torch, d["B"]), n, o, Lam, X, n)
    assert rc == 0, info.as_dict()
    lam, Xh = host(Lam), host(X)
    lam_o, X_o = orc.gsyeig(d["A"], d["B"], s, which="largest" if which else "smallest")
    mx = np.max(np.abs(d["lam"]))
    assert np.max(np.abs(lam - lam_o)) <= 1e-10 * mx
    m = orc.metrics(d["A"], d["B"], lam, Xh)
    assert m["eta_max"] <= 1e-12 and m["omega"] <= 1e-10
    assert info.eta_max <= 1e-12 and info.t_gs2_ms > 0.0
    # the spaced law's wanted pairs are separated by >= 1e-2: vectors agree
    if law == "spaced" and which == 0:
        assert np.max(np.abs(Xh - X_o)) <= 1e-9 * np.max(np.abs(X_o))


def test_ke_and_ki_agree(gs, ctx, torch):
    n, s = 2049, 25
    d = gen.known_spectrum(n, "spaced", seed=gen.BASE_SEED, stream=(203,))
    A = dev(torch, d["A"])
    out = {}
    for var in (gs.GSYEIG_KI, gs.GSYEIG_KE):
        say("ke vs ki", var)
        o = gs.gsyeig_opts_default()
        o.variant = var
        with gs.Solver() as sv:
            lam, X, info = sv.solve(A, dev(torch, d["B"]), s, o)
        assert info["rc"] == 0
        out[var] = (host(lam), host(X))
    assert np.max(np.abs(out[0][0] - out[1][0])) <= 1e-12
    assert np.max(np.abs(out[0][1] - out[1][1])) <= 1e-8 * np.max(np.abs(out[0][1]))


def test_ke_rejects_unsupported_modes(gs, ctx, torch):
    n = 64
    d = gen.known_spectrum(n, seed=204)
    Lam = torch.zeros(2, dtype=torch.float64, device="cuda")
    X = torch.zeros(2, n, dtype=torch.float64, device="cuda")
    for kw in (dict(prec=gs.GSYEIG_MIXED), dict(block=16), dict(variant=3), dict(invert=1),
               dict(variant=gs.GSYEIG_TD, prec=gs.GSYEIG_MIXED)):
        o = gs.gsyeig_opts_default()
        o.variant = gs.GSYEIG_KE
        for k, v in kw.items():
            setattr(o, k, v)
        rc, _ = gs.gsyeig_solve(ctx, n, 2, dev(torch, d["A"]), n, dev(torch, d["B"]), n, o, Lam, X, n)
        assert rc == -8, kw


@pytest.mark.parametrize("n,s,law,which", [(2, 1, "spaced", 0), (65, 5, "spaced", 0), (700, 35, "clustered", 0),
                                           (1500, 75, "spaced", 1), (1537, 20, "spaced", 0)])
def test_td_solve_matches_oracle(gs, ctx, torch, orc, n, s, law, which):
    say("td solve", n, s, law, which)
    d = gen.known_spectrum(n, law, seed=gen.BASE_SEED, stream=(205, n, which))
    o = gs.gsyeig_opts_default()
    o.variant = gs.GSYEIG_TD
    o.which = which
    Lam = torch.zeros(s, dtype=torch.float64, device="cuda")
    X = torch.zeros(s, n, dtype=torch.float64, device="cuda")
    rc, info = gs.gsyeig_solve(ctx, n, s, dev(torch, d["A"]), n, dev(torch, d["B"]), n, o, Lam, X, n)
    assert rc == 0, info.as_dict()
    assert info.steps == 0 and info.converged == s
    lam, Xh = host(Lam), host(X)
    lam_o, X_o = orc.gsyeig(d["A"], d["B"], s, which="largest" if which else "smallest")
    mx = np.max(np.abs(d["lam"]))
    assert np.max(np.abs(lam - lam_o)) <= 1e-12 * mx
    lam_true = np.sort(d["lam"])
    lam_true = lam_true[:s] if which == 0 else lam_true[n - s:]
    assert np.max(np.abs(lam - lam_true)) <= 1e-12 * mx
    m = orc.metrics(d["A"], d["B"], lam, Xh)
    assert m["eta_max"] <= 1e-12 and m["omega"] <= 1e-10
    assert info.eta_max <= 1e-12
    if law == "spaced" and which == 0 and s <= 10:
        assert np.max(np.abs(Xh - X_o)) <= 1e-9 * np.max(np.abs(X_o))


def test_td_ke_ki_agree(gs, ctx, torch):
    n, s = 3000, 40
    d = gen.known_spectrum(n, "spaced", seed=gen.BASE_SEED, stream=(206,))
    A = dev(torch, d["A"])
    lams = []
    for var in (gs.GSYEIG_KI, gs.GSYEIG_KE, gs.GSYEIG_TD):
        say("td/ke/ki", var)
        o = gs.gsyeig_opts_default()
        o.variant = var
        with gs.Solver() as sv:
            lam, X, info = sv.solve(A, dev(torch, d["B"]), s, o)
        assert info["rc"] == 0 and info["eta_max"] <= 1e-12
        lams.append(host(lam))
    assert np.max(np.abs(lams[0] - lams[2])) <= 1e-12
    assert np.max(np.abs(lams[1] - lams[2])) <= 1e-12
