"""Batched driver (many uneven instances, s = ceil(0.05 n)): every instance
equals the single-instance solve bit for bit, meets the known-spectrum bar,
and a failing instance is reported in its own status without disturbing the
others."""
import math
import sys

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def test_batched_equals_single_solves(orc):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1111_6374_amd as gs

    g = gen.rng(gen.BASE_SEED + 4, 0)
    sizes = [int(v) for v in g.integers(64, 700, size=11)] + [1]
    cnt = len(sizes)
    ss = [max(1, math.ceil(0.05 * n)) for n in sizes]
    insts = [gen.known_spectrum(n, seed=gen.BASE_SEED + 4, stream=(4, i)) for i, n in enumerate(sizes)]
    bad = 5  # instance 5 gets a non-SPD B
    A = [torch.from_numpy(d["A"]).cuda() for d in insts]
    B0 = [d["B"].copy() for d in insts]
    B0[bad][3, 3] = -1.0
    B = [torch.from_numpy(b).cuda() for b in B0]
    Lam = [torch.zeros(s, dtype=torch.float64, device="cuda") for s in ss]
    X = [torch.zeros(s, n, dtype=torch.float64, device="cuda") for s, n in zip(ss, sizes)]
    say("batched", sizes)
    with gs.Solver() as sv:
        rc, status, infos = gs.gsyeig_solve_batched(sv.ctx, sizes, ss, A, sizes, B, sizes, None, Lam, X,
                                                    sizes, nstreams=4)
    torch.cuda.synchronize()
    assert rc == status[bad] and 1 <= status[bad] <= 4
    assert all(st == 0 for i, st in enumerate(status) if i != bad)
    with gs.Solver() as sv:
        for i, (n, s) in enumerate(zip(sizes, ss)):
            if i == bad:
                continue
            say("single", i, n, s)
            lam1, X1, info = sv.solve(torch.from_numpy(insts[i]["A"]).cuda(), torch.from_numpy(B0[i]).cuda(), s)
            torch.cuda.synchronize()
            assert torch.equal(lam1, Lam[i]) and torch.equal(X1, X[i]), i
            lam_true = np.sort(insts[i]["lam"])[:s]
            assert np.max(np.abs(Lam[i].cpu().numpy() - lam_true)) <= 1e-10
            assert infos[i].eta_max <= 1e-12 and infos[i].steps == info["steps"]
