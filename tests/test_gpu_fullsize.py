"""Parity at the full benchmark size (n = 16384, s = 100, FP64), in the launch
configuration the bench times, for variant KI (the headline), variant KE
(explicit C) and the dense comparator TD.  The oracle cannot solve this size, so it
checks what it can compute one by one: every eigenvalue against the
generator's exact spectrum, and sampled pairs (x_i, lambda_i) through the
oracle's own matrix-vector products (residual) and back-substitution
(x_i = U^-1 y_i with the generator's Y)."""
import sys

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("variant", ["KI", "KE", "TD"])
def test_full_size_known_spectrum(orc, variant):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1111_6374_amd as gs

    n, s = 16384, 100
    say("fullsize-generate", n, s)
    inst = gen.known_spectrum_device(n, "spaced", seed=gen.BASE_SEED + 1, stream=(1, 0, 0), device="cuda")
    A, B = inst["A"], inst["B"]
    B_h = B.cpu().numpy()
    say("fullsize-solve", n, s, variant)
    o = gs.gsyeig_opts_default()
    o.variant = {"KI": gs.GSYEIG_KI, "KE": gs.GSYEIG_KE, "TD": gs.GSYEIG_TD}[variant]
    with gs.Solver() as sv:
        lam, X, info = sv.solve(A, B, s, opts=o)
    torch.cuda.synchronize()
    assert info["rc"] == 0, info
    lam = lam.cpu().numpy()
    order = np.argsort(inst["lam"], kind="stable")[:s]
    scale = np.max(np.abs(inst["lam"]))
    assert np.max(np.abs(lam - inst["lam"][order])) <= 1e-10 * scale
    assert info["eta_max"] <= 1e-12 and info["omega"] <= 1e-10
    say("fullsize-oracle-samples")
    A_h = A.cpu().numpy()
    U_h = inst["U"].cpu().numpy()
    X_h = X.cpu().numpy()
    nA, nB = np.linalg.norm(A_h), np.linalg.norm(B_h)
    for i in (0, 9, 10, 57, s - 1):
        x = X_h[i]
        r = orc.matvec(A_h, x) - lam[i] * orc.matvec(B_h, x)
        eta = np.linalg.norm(r) / ((nA + abs(lam[i]) * nB) * np.linalg.norm(x))
        assert eta <= 1e-12, (i, eta)
        y = inst["Y"][:, int(order[i])].cpu().numpy()
        x_ref = orc.backsolve(U_h, y[None, :])[0]
        x_ref *= np.sign(x_ref @ x)
        assert np.max(np.abs(x - x_ref)) <= 1e-8 * np.max(np.abs(x_ref)), i
