"""Host-side checks of the C-ABI library and the input generator (no GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2310_14087_amd.inputs import make_problem, WORKLOADS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kotssn.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(kot_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2310_14087_amd import kotssn
    path = kotssn._LIBPATH
    if not path.exists():
        from paper_2310_14087_amd import build
        build.build()
    return kotssn.load()


def test_header_exports_every_symbol(lib):
    from paper_2310_14087_amd import kotssn
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), f"{n} declared in kotssn.h but not exported"
    assert sorted(kotssn.EXPORTED) == names


def test_params_default_host_only(lib):
    from paper_2310_14087_amd import kotssn
    p = kotssn.default_params()
    assert p.tol == 1e-6 and p.max_iter == 200 and p.cg_max_iter == 20
    assert p.tau == 0.5 and p.kappa == 0.5
    assert p.alpha1 == 1e-6 and p.alpha2 == 1.0 and p.beta0 == 0.5 and p.beta2 == 5.0
    assert p.beta1 == pytest.approx(1 / 1.2)
    assert p.null_step == 0 and p.safeguard == kotssn.KOT_SAFEGUARD_EG and p.precision == kotssn.KOT_FP64
    assert p.overlap == 1 and p.lowp_min_rows == 64 and p.precond == kotssn.KOT_PRECOND_NONE
    assert p.schur_solver == kotssn.KOT_SCHUR_CG
    assert p.eig_inner_sweeps == 1 and p.closed_start == 0 and p.kdiag_tol == 1e-12


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the C structs have the size and every field offset that a C compiler gives the header."""
    import shutil
    import subprocess
    from paper_2310_14087_amd import kotssn
    gcc = shutil.which("gcc") or shutil.which("cc")
    if gcc is None:
        pytest.skip("no C compiler")
    mirrors = {"kot_params": kotssn.KotParams, "kot_problem": kotssn.KotProblem, "kot_result": kotssn.KotResult}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "kotssn.h"', "int main(void) {"]
    for cname, ct in mirrors.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in ct._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, ct in mirrors.items():
        assert got[(cname, "sizeof")] == C.sizeof(ct), cname
        for fname, _ in ct._fields_:
            assert got[(cname, fname)] == getattr(ct, fname).offset, (cname, fname)


def test_null_arguments_are_rejected_without_a_device(lib):
    from paper_2310_14087_amd import kotssn
    assert lib.kot_create(None, 0, None) == kotssn.KOT_ERR_ARG
    assert lib.kot_destroy(None) == kotssn.KOT_ERR_ARG
    assert lib.kot_last_error(None) == b"null context"


@pytest.mark.parametrize("name", WORKLOADS)
def test_generator_is_seeded(name):
    a = make_problem(name, 1, l=30, n=60)
    b = make_problem(name, 1, l=30, n=60)
    c = make_problem(name, 2, l=30, n=60)
    for f in ("xs", "ys", "xf", "yf"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
        assert getattr(a, f).dtype == np.float64 and getattr(a, f).flags.c_contiguous
    assert not np.array_equal(a.xs, c.xs)
    assert a.sigma == b.sigma and a.sigma > 0 and a.lam1 > 0 and a.lam2 > 0


def test_generator_shapes():
    p = make_problem("mix1000", 0, l=40, n=50)
    assert p.xs.shape == (50, 10) and p.xf.shape == (40, 10) and p.lam1 == 1 / 40
    t = make_problem("tiny", 0)
    assert t.xs.shape == (100, 2) and t.l == 50 and t.sigma == 1.0 and t.lam1 == t.lam2 == 1e-3 and t.tol == 1e-8


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "4"})])
def test_bench_refuses_more_than_one_gpu(argv, env):
    """bench.py runs on one GPU: a request for more exits with status 2 and one JSON line saying so, before
    it touches a device."""
    import json
    import subprocess
    import sys
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], capture_output=True, text=True,
                       env=e, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


@pytest.mark.parametrize("F,H", [(12, 512), (5, 64), (1, 1)])
def test_mlp_params_count(lib, F, H):
    """kot_mlp_params (host only): the length of theta in the documented layout, W1 (F x H), b1, W2 (H x H), b2,
    w3 (H), b3 -- the count the oracle's network uses."""
    from oracle import mlp
    assert lib.kot_mlp_params(F, H) == F * H + H + H * H + H + H + 1 == mlp.n_params(F, H)
