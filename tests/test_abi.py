"""Host-side checks of the C ABI (no GPU work): the library loads, exports
every entry point include/abm.h declares, the binding's struct layouts match
the header's, and invalid problems are refused with ABM_EINVAL before any
device work."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1710_01133_amd import abm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "abm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(abm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(abm.LIB_PATH):
        from paper_1710_01133_amd import build
        build.build()
    return abm.load()


def test_every_declared_function_is_exported(lib):
    names = _declared_functions()
    assert "abm_solve" in names and "abm_plan" in names and "abm_submit" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(abm.EXPORTED)


def test_no_unexpected_exports(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", abm.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T abm_" in ln}
    assert exported == set(_declared_functions())


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "abm.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(abm_problem), offsetof(abm_problem, alpha),
         offsetof(abm_problem, N), offsetof(abm_problem, x0), offsetof(abm_problem, p),
         offsetof(abm_problem, far_prec), offsetof(abm_problem, out_stride));
  printf("%zu %zu %zu\n", sizeof(abm_stats), offsetof(abm_stats, history_macs),
         offsetof(abm_stats, far_launches));
  printf("%zu %zu %zu\n", sizeof(abm_result), offsetof(abm_result, t_submit),
         offsetof(abm_result, max_abs_y));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    lines = subprocess.check_output([str(exe)], text=True).split("\n")
    P, S, R = abm.AbmProblem, abm.AbmStats, abm.AbmResult
    assert [int(v) for v in lines[0].split()] == [ctypes.sizeof(P), P.alpha.offset, P.N.offset,
                                                  P.x0.offset, P.p.offset, P.far_prec.offset,
                                                  P.out_stride.offset]
    assert [int(v) for v in lines[1].split()] == [ctypes.sizeof(S), S.history_macs.offset,
                                                  S.far_launches.offset]
    assert [int(v) for v in lines[2].split()] == [ctypes.sizeof(R), R.t_submit.offset,
                                                  R.max_abs_y.offset]


def test_strerror_texts(lib):
    assert lib.abm_strerror(0) == b"ok"
    assert lib.abm_strerror(-1) == b"invalid argument"
    assert lib.abm_strerror(-4) == b"not finished"
    assert lib.abm_strerror(-99) == b"unknown status"


def test_problem_marshalling():
    from paper_1710_01133_amd import inputs
    p = inputs.duffing_single(N=1234)
    c = abm.c_problem(p, out_stride=7)
    assert (c.rhs, c.d, c.N, c.out_stride, c.far_prec) == (1, 2, 1234, 7, 0)
    assert list(c.x0)[:2] == [0.1, 0.0] and list(c.p)[:3] == [0.1, 0.3, 1.2]
    assert abm.n_out(10, 0) == 1 and abm.n_out(10, 3) == 5 and abm.n_out(9, 3) == 4


def _invalid_problems():
    """(what, abm_problem) pairs that abm.h's contract refuses with
    ABM_EINVAL before any device work."""
    from paper_1710_01133_amd import inputs
    nan, inf = float("nan"), float("inf")

    def base(**kw):
        p = inputs.duffing_single(N=kw.pop("N", 1000))
        c = abm.c_problem(p)
        for k, v in kw.items():
            setattr(c, k, v)
        return c

    out = [("unknown rhs", base(rhs=99)),
           ("dimension of the rhs", base(d=3)),
           ("order 0", base(alpha=0.0)),
           ("order above 2", base(alpha=2.5)),
           ("order not a number", base(alpha=nan)),
           ("h = 0", base(h=0.0)),
           ("h not finite", base(h=inf)),
           ("N = 0", base(N=0)),
           ("N above 2^30 (32-bit step flags)", base(N=(1 << 30) + 1)),
           ("negative output stride", base(out_stride=-1)),
           ("unknown far_prec", base(far_prec=42))]
    c = base()
    c.x0[0] = nan
    out.append(("x0 not finite", c))
    c = base()
    c.p[7] = inf
    out.append(("p not finite", c))
    c = base(alpha=1.5)
    c.x1[1] = nan
    out.append(("x1 not finite for an order above 1", c))
    c = base()
    c.alpha = 0.0
    c.alphas[0], c.alphas[1] = 0.9, 2.01
    out.append(("a per-component order above 2", c))
    return out


@pytest.mark.parametrize("what,c", _invalid_problems(), ids=[w for w, _ in _invalid_problems()])
def test_invalid_problem_refused_before_any_device_work(lib, what, c):
    """abm_solve_noalloc validates the problem before it touches a device
    (the output pointer is a host dummy that is never written)."""
    dummy = ctypes.create_string_buffer(64)
    st = lib.abm_solve_noalloc(ctypes.byref(c), ctypes.cast(dummy, ctypes.c_void_p), None)
    assert st == abm.ABM_EINVAL, (what, st)
    assert lib.abm_last_error(), what


def test_noalloc_workspace_bound_checked_on_the_host(lib):
    """One order and N = 341953 steps need more than the 8 MiB no-allocation
    workspace (its stated limit is N <= 341952): refused before any device
    work; a double-double problem is refused there too."""
    from paper_1710_01133_amd import inputs
    dummy = ctypes.create_string_buffer(64)
    c = abm.c_problem(inputs.Problem("LINEAR", 0.8, 1e-3, 341953, (1.0,), (1.0,)))
    assert lib.abm_solve_noalloc(ctypes.byref(c), ctypes.cast(dummy, ctypes.c_void_p), None) == abm.ABM_EINVAL
    assert b"workspace" in lib.abm_last_error()
    c = abm.c_problem(inputs.Problem("LINEAR", 0.8, 1e-3, 1000, (1.0,), (1.0,), "dd"))
    assert lib.abm_solve_noalloc(ctypes.byref(c), ctypes.cast(dummy, ctypes.c_void_p), None) == abm.ABM_EINVAL
    assert b"double-double" in lib.abm_last_error()
