"""The C-ABI library loads and exports every entry point its header declares;
host-side argument validation (no GPU call is made on these paths)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsyeig.h")


@pytest.fixture(scope="module")
def gs():
    import paper_1111_6374_amd as gs

    if not os.path.exists(gs.LIB_PATH):
        from paper_1111_6374_amd import build

        build.build()
    gs.lib()
    return gs


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(gsyeig_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    fns = header_functions()
    for name in ("gsyeig_potrf", "gsyeig_lanczos", "gsyeig_backsolve", "gsyeig_solve"):
        assert name in fns


def test_library_exports_every_declared_symbol(gs):
    L = gs.lib()
    for name in header_functions():
        assert hasattr(L, name), name
    assert sorted(gs.EXPORTS) == header_functions()


def test_exports_are_extern_c(gs):
    out = os.popen(f"nm -D --defined-only {gs.LIB_PATH}").read()
    for name in header_functions():
        assert re.search(rf"\bT {name}$", out, re.M), name


def test_version_and_defaults(gs):
    assert "gfx950" in gs.gsyeig_version()
    o = gs.gsyeig_opts_default()
    assert (o.prec, o.block, o.which, o.invert) == (0, 1, 0, 0)
    assert o.tol == 1e-12 and o.check_every == 25 and o.seed == 6374 and not o.v0
    assert o.profile_every == 0
    assert (o.basis, o.keep, o.block_acc32, o.variant) == (0, 0, 0, gs.GSYEIG_KI)
    assert (o.eta_tol, o.refine_iters, o.refine_inner, o.guard, o.reorth) == (1e-10, 10, 20, 0, 2)


def test_workspace_size(gs):
    rc, b = gs.gsyeig_workspace_size(16384, 100)
    assert rc == 0
    # V alone: n x (min(n, 100 s + 2000) + 1) doubles
    assert b >= 16384 * (12000 + 1) * 8
    assert gs.gsyeig_workspace_size(0, 1)[0] == -1
    assert gs.gsyeig_workspace_size(10, 11)[0] == -2
    # mixed mode adds the FP32 copies of A and U (4 bytes each per entry)
    o = gs.gsyeig_opts_default()
    o.prec = gs.GSYEIG_MIXED
    rc, bm = gs.gsyeig_workspace_size(16384, 100, o)
    assert rc == 0 and bm >= b + 2 * 4 * 16384 * 16384


def test_null_context_is_rejected_without_gpu(gs):
    assert gs.gsyeig_solve(None, 10, 2, 1, 10, 1, 10, None, 1, 1, 10)[0] == -1
    assert gs.gsyeig_potrf(None, 10, 1, 10) == -1
    assert gs.gsyeig_trsv(None, 10, 1, 10, 0, 1, 1) == -1
    assert gs.gsyeig_trsv_lp(None, 10, 1, 10, 0, 1, 1) == -1
    assert gs.gsyeig_trsm_lp(None, 10, 1, 10, 0, 2, 1, 10, 1, 10) == -1
    assert gs.gsyeig_syev_small(None, 10, 1, 10, 2, 0, 1, 1, 10) == -1
    assert gs.gsyeig_refine(None, 10, 2, 4, 1, 10, 1, 10, 1, 10, None, 1, 10, 1, 1, 10)[0] == -1
    assert gs.gsyeig_set_spin_limit(None, 1) == -1
    assert gs.gsyeig_sync(None) == -1
    assert gs.gsyeig_autotune(None, 100)[0] == -1
    assert gs.gsyeig_set_trsv_sweep(None, 0) == -1
    assert gs.gsyeig_destroy(None) == -1
    assert gs.lib().gsyeig_opts_default(None) == -1


def test_binding_refuses_cpu_tensors(gs):
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):
        gs._p(torch.zeros(3, dtype=torch.float64))


def test_binding_structs_match_the_header(gs, tmp_path):
    """The ctypes mirrors of gsyeig_opts and gsyeig_info have the C layout:
    sizes and every field offset, as a C compiler lays out the header."""
    fields = {"gsyeig_opts": gs.gsyeig_opts, "gsyeig_info": gs.gsyeig_info, "gsyeig_tuning": gs.gsyeig_tuning}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for st, cls in fields.items():
        lines.append(f'printf("{st} size %zu\\n", sizeof({st}));')
        for name, _ in cls._fields_:
            lines.append(f'printf("{st} {name} %zu\\n", offsetof({st}, {name}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    assert os.system(f"gcc -std=c11 -o {exe} {src}") == 0
    got = {}
    for ln in os.popen(str(exe)).read().splitlines():
        st, name, val = ln.split()
        got[(st, name)] = int(val)
    for st, cls in fields.items():
        assert got[(st, "size")] == ctypes.sizeof(cls), st
        for name, _ in cls._fields_:
            assert got[(st, name)] == getattr(cls, name).offset, (st, name)
