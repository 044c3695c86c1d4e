"""The project-written autotuner (gsyeig_autotune) through the C ABI: it
measures every candidate, applies the fastest, records it in its JSON cache
keyed by (architecture, precision, n-bucket), takes it from the cache on the
next call without measuring, keeps other architectures' entries, and the
solves that follow on the tuned kernels still meet the oracle's bar."""
import json
import sys

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def test_autotune_measures_applies_and_caches(orc, tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1111_6374_amd as gs

    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps([{"arch": "gfx000-other", "entries": [
        {"prec": 0, "n_bucket": 4096, "trsv_block": 64, "trsv_sweep": 1, "gemm_big_min": 0,
         "op_ms": 1.0, "gemm_ms": 1.0}]}]))
    with gs.Solver() as sv:
        for prec in (gs.GSYEIG_FP64, gs.GSYEIG_MIXED):
            say("autotune", prec)
            rc, t = gs.gsyeig_autotune(sv.ctx, 3000, prec, str(cache))
            assert rc == 0 and t.from_cache == 0 and t.n_bucket == 4096 and t.prec == prec
            cands = [c for c in t.op_ms_cand if c > 0]
            assert len(cands) == (5 if prec == gs.GSYEIG_FP64 else 4)
            assert t.op_ms == min(cands) and t.gemm_ms == min(t.gemm_ms_cand)
            assert t.trsv_block in (64, 512) and t.trsv_sweep in (0, 1, 2, 3) and t.gemm_big_min in (0, 2048)
            rc, t2 = gs.gsyeig_autotune(sv.ctx, 2500, prec, str(cache))
            assert rc == 0 and t2.from_cache == 1
            assert (t2.trsv_block, t2.trsv_sweep, t2.gemm_big_min) == (t.trsv_block, t.trsv_sweep, t.gemm_big_min)
        doc = json.loads(cache.read_text())
        archs = [o["arch"] for o in doc]
        assert "gfx000-other" in archs and any(a.startswith("gfx950") for a in archs)
        mine = [o for o in doc if o["arch"].startswith("gfx950")][0]["entries"]
        assert sorted(e["prec"] for e in mine) == [0, 1]
        # the tuned kernels (last applied: the mixed choice) solve to the bar
        n, s = 2000, 20
        d = gen.known_spectrum(n, seed=gen.BASE_SEED, stream=(301,))
        for prec in (gs.GSYEIG_FP64, gs.GSYEIG_MIXED):
            rc, t = gs.gsyeig_autotune(sv.ctx, n, prec, str(cache))
            assert rc == 0
            o = gs.gsyeig_opts_default()
            o.prec = prec
            lam, X, info = sv.solve(torch.from_numpy(d["A"]).cuda(), torch.from_numpy(d["B"]).cuda(), s, o)
            torch.cuda.synchronize()
            assert info["rc"] == 0
            lam_o, _ = orc.gsyeig(d["A"], d["B"], s)
            assert np.max(np.abs(lam.cpu().numpy() - lam_o)) <= 1e-10 * np.max(np.abs(d["lam"]))
            assert info["eta_max"] <= (1e-12 if prec == gs.GSYEIG_FP64 else 1e-10)
