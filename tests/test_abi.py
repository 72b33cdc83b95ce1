"""The C-ABI library loads without a GPU, exports every entry point that
include/reg.h declares, lays out its structs as the header does, and rejects
bad parameters before touching the device."""
import ctypes
import json
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "reg.h")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:reg_status|const char \*)\s*(reg_[a-z_]+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1608_03630_amd import reg

    return reg.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layout_matches_header():
    from paper_1608_03630_amd import reg

    src = '#include <stdio.h>\n#include <stddef.h>\n#include "reg.h"\nint main(void){printf("%zu %zu %zu %zu\\n",' \
          ' sizeof(reg_params), sizeof(reg_report), offsetof(reg_report, final_J), offsetof(reg_params, armijo_c1));' \
          ' return 0;}\n'
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    sp, sr, ofj, ofa = map(int, out)
    assert sp == ctypes.sizeof(reg.reg_params)
    assert sr == ctypes.sizeof(reg.reg_report)
    assert ofj == reg.reg_report.final_J.offset
    assert ofa == reg.reg_params.armijo_c1.offset


def test_default_params_are_the_papers(lib):
    from paper_1608_03630_amd import reg

    with open(os.path.join(ROOT, "tests", "golden", "paper_parameters.json")) as f:
        gold = json.load(f)
    p = reg.reg_default_params(32)
    assert p.beta == gold["beta"] and p.nt == gold["nt"] and p.gtol == gold["gtol"]
    assert p.forcing == 0 and p.isochoric == 0 and p.beta_final == 0


def test_workspace_size_scales_with_grid(lib):
    from paper_1608_03630_amd import reg

    a = reg.reg_workspace_size(reg.reg_default_params(32))
    b = reg.reg_workspace_size(reg.reg_default_params(64))
    c = reg.reg_workspace_size(reg.reg_default_params(64, prec=1))
    # velocity-space vectors are double in both modes, so FP64 fields cost
    # less than twice the FP32 workspace
    assert 7.5 < b / a < 8.5 and 1.2 < c / b < 2.0


@pytest.mark.parametrize("bad", [dict(n=(0, 32, 32)), dict(n=(0, 0, 0)), dict(n=(-8, 32, 32)),
                                 dict(n=(14, 32, 32)), dict(n=(32, 32, 22)), dict(n=(32, 32, 6)),
                                 dict(n=(32, 15, 32)), dict(n=(2048, 8, 8)), dict(nt=0), dict(beta=0.0),
                                 dict(beta=-1.0), dict(prec=2), dict(max_pcg=0), dict(gtol=-1.0), dict(hessian=2),
                                 dict(det_check=2), dict(grid_levels=5), dict(n=(24, 24, 24), grid_levels=3),
                                 dict(recompute_grad_rho=2), dict(recompute_grad_rho=1, hessian=1)])
def test_bad_parameters_are_rejected(lib, bad):
    from paper_1608_03630_amd import reg

    n = bad.pop("n", (32, 32, 32))
    p = reg.reg_default_params(n, **bad)
    with pytest.raises(reg.RegError) as e:
        reg.reg_workspace_size(p)
    assert e.value.status == reg.REG_EINVAL


def test_recomputed_grad_rho_shrinks_the_workspace(lib):
    from paper_1608_03630_amd import reg

    for prec, esz in ((0, 4), (1, 8)):
        kept = reg.reg_workspace_size(reg.reg_default_params((64, 64, 64), nt=16, prec=prec))
        rec = reg.reg_workspace_size(reg.reg_default_params((64, 64, 64), nt=16, prec=prec, recompute_grad_rho=1))
        assert kept - rec == 3 * 16 * 64 ** 3 * esz


def test_log_needs_a_context(lib):
    from paper_1608_03630_amd import reg

    assert lib.reg_set_log(None, reg.LOG_FN(), None) == reg.REG_EINVAL


def test_create_rejects_null_workspace(lib):
    from paper_1608_03630_amd import reg

    p = reg.reg_default_params(32)
    h = ctypes.c_void_p()
    st = lib.reg_create(ctypes.byref(p), None, 1 << 30, None, ctypes.byref(h))
    assert st == reg.REG_EINVAL and not h.value


def test_batch_workspace_is_the_sum_of_its_problems(lib):
    from paper_1608_03630_amd import reg

    ps = [reg.reg_default_params(n, nt=nt) for n, nt in [((64, 64, 64), 4), ((32, 48, 64), 3), ((24, 36, 54), 4)]]
    total = reg.reg_batch_workspace_size(ps)
    parts = sum((reg.reg_workspace_size(p) + 255) // 256 * 256 for p in ps)
    # plus the tables of the batched step launches: a few KB
    assert parts < total < parts + (1 << 20)


def test_batch_rejects_mixed_precision_and_bad_problems(lib):
    from paper_1608_03630_amd import reg

    with pytest.raises(reg.RegError) as e:
        reg.reg_batch_workspace_size([reg.reg_default_params(32), reg.reg_default_params(32, prec=1)])
    assert e.value.status == reg.REG_EINVAL
    for bad in (reg.reg_default_params(14), reg.reg_default_params(32, hessian=1),
                reg.reg_default_params(32, grid_levels=2)):
        with pytest.raises(reg.RegError) as e:
            reg.reg_batch_workspace_size([reg.reg_default_params(32), bad])
        assert e.value.status == reg.REG_EINVAL
    h = ctypes.c_void_p()
    arr = (reg.reg_params * 1)(reg.reg_default_params(32))
    assert lib.reg_batch_create(arr, 1, None, 1 << 30, None, ctypes.byref(h)) == reg.REG_EINVAL and not h.value
    assert lib.reg_batch_create(arr, 0, None, 1 << 30, None, ctypes.byref(h)) == reg.REG_EINVAL


def test_empty_batch_is_rejected(lib):
    from paper_1608_03630_amd import reg

    p = reg.reg_default_params(32)
    b = ctypes.c_size_t(7)
    for npairs in (0, -1):
        assert lib.reg_batch_workspace_size(ctypes.byref(p), npairs, ctypes.byref(b)) == reg.REG_EINVAL


@pytest.mark.parametrize("prec,n,alias", [(2, (8, 8, 8), False), (0, None, False), (0, (0, 8, 8), False),
                                          (0, (8, 0, 8), False), (1, (8, 8, -8), False), (0, (2048, 8, 8), False),
                                          (0, (8, 8, 9), False), (0, (8, 8, 8), True)])
def test_noalloc_interp_rejects_bad_arguments_before_the_device(lib, prec, n, alias):
    # every check here precedes the first HIP call, so the placeholder
    # addresses are never dereferenced
    from paper_1608_03630_amd import reg

    nn = (ctypes.c_int32 * 3)(*n) if n is not None else None
    f, D, out = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x1000 if alias else 0x3000)
    assert lib.reg_interp_noalloc(prec, nn, f, D, out, None) == reg.REG_EINVAL


def test_product_package_does_not_reach_the_oracle():
    """The product path never imports, links or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_1608_03630_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text and "liboracle" not in text, f


def test_binding_fails_loudly_without_the_library():
    """With libreg.so absent the binding raises on first use; there is no
    fallback path (run in a fresh interpreter so the loaded library of this
    process is not involved)."""
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1608_03630_amd import reg\n"
        "reg.LIB_PATH = '/nonexistent/libreg.so'\n"
        "try:\n"
        "    reg.reg_default_params((32, 32, 32))\n"
        "except RuntimeError as e:\n"
        "    print('raised:', e)\n"
        "    sys.exit(0)\n"
        "sys.exit(3)\n" % ROOT)
    r = subprocess.run(["python3", "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "missing" in r.stdout
