"""The C ABI library: builds, loads without a GPU, and exports every entry
point that include/skipm.h declares with the signature the binding uses."""
import ctypes
import re
from pathlib import Path

import pytest

import paper_2003_08072_amd as sk

HEADER = Path(__file__).resolve().parents[1] / "include" / "skipm.h"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\([^;{]*\)\s*;",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lp_create", "lp_destroy", "ipm_step", "pcg_solve", "sketch_apply",
                     "lp_solve", "sketch_hash"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = sk.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in sk.SIGNATURES, name


def test_struct_layouts_match_header():
    # sizes follow the C layout of the header structs on x86-64
    assert ctypes.sizeof(sk.Params) == 6 * 8 + 6 * 4 + 8 + 8
    assert ctypes.sizeof(sk.Problem) == 3 * 8 + 2 * 4 + 8 + 8 + 4 * 8
    assert ctypes.sizeof(sk.Result) == 4 * 4 + 6 * 8 + 4 * 4
    assert ctypes.sizeof(sk.StepInfo) == 11 * 8 + 8 * 4


def test_params_default_values():
    p = sk.default_params()
    assert p.sigma == 0.5 and p.gamma == 0.999 and p.tol_cg == 1e-5
    assert p.s == 1 and p.w == 0 and p.resketch == 1 and p.precision == sk.SKIPM_PREC_FP64


def test_argument_validation_without_device():
    lib = sk.load()
    assert lib.skipm_params_default(None) == sk.SKIPM_EINVAL
    h = ctypes.c_void_p()
    prm = sk.default_params()
    assert lib.lp_create(ctypes.byref(h), None, ctypes.byref(prm), None) == sk.SKIPM_EINVAL
    prob = sk.Problem(m=0, n=10)
    assert lib.lp_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(prm), None) == \
        sk.SKIPM_EINVAL
    prob = sk.Problem(m=5, n=3)
    assert lib.lp_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(prm), None) == \
        sk.SKIPM_EINVAL
    assert b"m <= n" in lib.skipm_last_error()
    assert lib.lp_destroy(None) == sk.SKIPM_OK
    for bad in (dict(sigma=0.9), dict(gamma=1.0), dict(s=3, w=200), dict(w=2)):
        p = sk.default_params(**bad)
        prob = sk.Problem(m=10, n=100, format=sk.SKIPM_DENSE, a_dtype=sk.SKIPM_F64,
                          a_vals=1, b=1, c=1)
        assert lib.lp_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(p), None) == \
            sk.SKIPM_EINVAL, bad
    assert lib.sketch_hash(0, 0, 3, 10, 10, None, None, None) == sk.SKIPM_EINVAL
    assert lib.sketch_apply(None, None, 0, None, 7, None) == sk.SKIPM_EINVAL
    assert b"out_dtype" in lib.skipm_last_error()
    assert lib.sketch_apply(None, None, 0, None, sk.SKIPM_F32, None) == sk.SKIPM_EINVAL
    assert b"null" in lib.skipm_last_error()


def _c_layouts():
    """sizeof / offsetof of the header's structs, from a C compiler reading the
    header itself (skipped without gcc or the HIP headers)."""
    import shutil
    import subprocess
    import tempfile
    if shutil.which("gcc") is None or not Path("/opt/rocm/include/hip").is_dir():
        pytest.skip("gcc or HIP headers missing")
    fields = {
        "skipm_problem": ["m", "nnz", "format", "a_vals", "lda", "a_colidx", "c"],
        "skipm_params": ["sigma", "guard", "w", "s", "precision", "seed", "inner", "sketch"],
        "skipm_result": ["status", "cg_max", "obj_p", "mu", "demote_iter", "tier_final",
                         "resketches", "shifts"],
        "skipm_step_info": ["mu", "v_resid", "cg_iters", "status", "tier", "refine_steps",
                            "resketches", "shifts"],
        "skipm_pcg_info": ["iters", "f0_norm", "f_norm"],
        "skipm_request_info": ["res", "state", "rc", "footprint", "device_bytes", "t_submit",
                               "t_done"],
        "skipm_server_stats": ["budget", "peak_in_use", "slots", "queued", "completed"],
    }
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "skipm.h"', "int main(void){"]
    for st, fs in fields.items():
        lines.append(f'printf("{st} sizeof %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st} {f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        src = Path(d) / "l.c"
        src.write_text("\n".join(lines))
        exe = Path(d) / "l"
        r = subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                            f"-I{HEADER.parent}", str(src), "-o", str(exe)],
                           capture_output=True, text=True)
        if r.returncode != 0:
            pytest.skip("header does not compile as plain C here: " + r.stderr[-300:])
        out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = {}
    for line in out.splitlines():
        st, f, v = line.split()
        got[(st, f)] = int(v)
    return got


def test_ctypes_structs_match_the_c_compiler():
    got = _c_layouts()
    py = {"skipm_problem": sk.Problem, "skipm_params": sk.Params, "skipm_result": sk.Result,
          "skipm_step_info": sk.StepInfo, "skipm_pcg_info": sk.PcgInfo,
          "skipm_request_info": sk.RequestInfo, "skipm_server_stats": sk.ServerStats}
    for (st, f), v in got.items():
        cls = py[st]
        if f == "sizeof":
            assert ctypes.sizeof(cls) == v, st
        else:
            assert getattr(cls, f).offset == v, (st, f)


def test_footprint_is_host_only_and_grows_with_the_problem():
    small = sk.Problem(m=50, n=1000, nnz=0, format=sk.SKIPM_DENSE, a_dtype=sk.SKIPM_F64)
    big = sk.Problem(m=500, n=100_000, nnz=0, format=sk.SKIPM_DENSE, a_dtype=sk.SKIPM_F64)
    f_small, f_big = sk.footprint(small), sk.footprint(big)
    assert f_small < f_big
    assert f_big >= 500 * 100_000 * 8 + 2 * 500 * 2000 * 8   # A plus B and its refinement copy
    mixed = sk.footprint(big, precision=sk.SKIPM_PREC_MIXED)
    assert mixed >= f_big + 500 * 100_000 * 4                 # plus the FP32 copy
    csr = sk.Problem(m=1000, n=1_000_000, nnz=1_999_000, format=sk.SKIPM_CSR,
                     a_dtype=sk.SKIPM_F32)
    f_csr = sk.footprint(csr)
    assert 2 * 1_999_000 * 8 <= f_csr < 1_000_000 * 1000 * 4  # both copies, far below dense
    with pytest.raises(sk.SkipmError):
        sk.footprint(sk.Problem(m=10, n=5, format=sk.SKIPM_DENSE, a_dtype=sk.SKIPM_F64))


def test_largest_m_is_2048():
    """m <= 2048 (a 2048-row column fits one lane group's registers in the
    column passes, an m-vector the sparse passes' LDS); 2049 is rejected before
    any device call, for both formats, by lp_create and lp_footprint."""
    lib = sk.load()
    prm = sk.default_params()
    h = ctypes.c_void_p()
    for fmt in (sk.SKIPM_DENSE, sk.SKIPM_CSR):
        prob = sk.Problem(m=2049, n=10_000, nnz=20_000, format=fmt, a_dtype=sk.SKIPM_F32,
                          a_vals=1, a_rowptr=1, a_colidx=1, b=1, c=1)
        assert lib.lp_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(prm), None) == \
            sk.SKIPM_EINVAL
        assert b"2048" in lib.skipm_last_error()
        with pytest.raises(sk.SkipmError):
            sk.footprint(prob)
        prob.m = 2048
        assert sk.footprint(prob) > 0


def test_batch_and_server_validate_arguments_without_a_device():
    lib = sk.load()
    res = (sk.Result * 1)()
    assert lib.lp_solve_batch(None, 0, res, 0) == sk.SKIPM_OK
    handles = (ctypes.c_void_p * 1)(None)
    assert lib.lp_solve_batch(handles, 1, res, 0) == sk.SKIPM_EINVAL
    h = ctypes.c_void_p()
    assert lib.srv_create(ctypes.byref(h), 1 << 30, 0) == sk.SKIPM_EINVAL
    assert lib.srv_create(ctypes.byref(h), 0, 4) == sk.SKIPM_EINVAL
    assert lib.srv_destroy(None) == sk.SKIPM_OK


def test_result_fields_reach_python():
    """The precision-tier and rank-loss fields of skipm_result travel through
    the binding's SolveResult (a host-only round trip of the struct)."""
    r = sk.Result(status=0, iters=7, demote_iter=3, tier_final=sk.SKIPM_TIER_FP64,
                  resketches=2, shifts=1)
    out = sk._result(r)
    assert (out.demote_iter, out.tier_final, out.resketches, out.shifts) == (3, 0, 2, 1)
    assert sk.SKIPM_TIER_FP32 == 1 and sk.SKIPM_TIER_BF16 == 2


def test_correction_vector_refinement_policy():
    """The host policy of the refinement for t = (A D W)^+ g (vrefine.h),
    compiled on its own with g++: a finite, smaller residual replaces the kept
    t; NaN, inf or a larger residual never does; a poor contraction builds the
    next pseudo-inverse round while one is left; stagnation or the target ends
    the refinement."""
    import shutil
    import subprocess
    import tempfile
    if shutil.which("g++") is None:
        pytest.skip("g++ missing")
    hdr = Path(__file__).resolve().parents[1] / "paper_2003_08072_amd" / "csrc"
    prog = r"""
#include <cstdio>
#include <cmath>
#include "vrefine.h"
using namespace skipm;
static void run(const char* name, const double* rel, int n) {
  VRefine s;
  printf("%s", name);
  for (int i = 0; i < n; ++i) {
    bool keep = false;
    VAct a = v_refine_next(s, rel[i], &keep);
    printf(" %d%c%d", (int)a, keep ? 'k' : '-', s.round);
    if (a == V_STOP) break;
  }
  printf(" best=%.3g\n", s.best);
}
int main() {
  const double conv[] = {1e-3, 1e-9, 1e-15};           // good contraction: no rounds built
  const double slow[] = {0.5, 0.2, 0.1, 1e-16};        // poor contraction: rounds 1 and 2
  const double nan_[] = {1e-3, NAN, 1e-16};            // NaN never kept; builds a round
  const double worse[] = {1e-6, 1e-3, 1e-5, 1e-7};     // larger residual rejected
  const double stag[] = {1e-9, 0.9e-9};                // weak contraction: builds a round
  const double inf_[] = {INFINITY, INFINITY, INFINITY, INFINITY};
  run("conv", conv, 3);
  run("slow", slow, 4);
  run("nan", nan_, 3);
  run("worse", worse, 4);
  run("stag", stag, 2);
  run("inf", inf_, 4);
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        src = Path(d) / "p.cpp"
        src.write_text(prog)
        exe = Path(d) / "p"
        subprocess.run(["g++", "-std=c++17", f"-I{hdr}", str(src), "-o", str(exe)], check=True)
        out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    lines = {ln.split()[0]: ln.split()[1:] for ln in out.splitlines()}
    # 1e-3 from 1: ratio 1e-3 <= 1e-2, next step; 1e-9 ratio 1e-6; 1e-15 meets the target
    assert lines["conv"] == ["1k0", "1k0", "0k0", "best=1e-15"]
    # 0.5: build round 1; 0.2 (ratio 0.4): build round 2; 0.1 (ratio 0.5, no
    # round left): next; 1e-16: target met
    assert lines["slow"] == ["2k1", "2k2", "1k2", "0k2", "best=1e-16"]
    # NaN: not kept, counts as no contraction: build round 1; then 1e-16
    assert lines["nan"] == ["1k0", "2-1", "0k1", "best=1e-16"]
    # 1e-3 after 1e-6: rejected, build round 1; 1e-5: rejected, round 2;
    # 1e-7: kept (ratio 0.1, no round left, below 0.5): next
    assert lines["worse"] == ["1k0", "2-1", "2-2", "1k2", "best=1e-07"]
    # 0.9e-9 after 1e-9: ratio 0.9 > 1e-2 builds round 1 while rounds are left
    assert lines["stag"] == ["1k0", "2k1", "best=9e-10"]
    # never finite: nothing kept; rounds 1, 2 built, then stop with t = 0
    assert lines["inf"] == ["2-1", "2-2", "0-2", "best=1"]


def test_noalloc_product_validates_before_any_device_call():
    """normal_matvec_noalloc rejects shapes its static scratch buffer cannot
    hold, and bad layouts, with SKIPM_EINVAL before touching a device."""
    lib = sk.load()
    a = 16  # a 16-byte aligned stand-in address: never dereferenced here
    bad = [(2049, 10, 2052, sk.SKIPM_F64), (8, 10, 6, sk.SKIPM_F64), (8, 10, 4096, sk.SKIPM_F64),
           (0, 10, 4, sk.SKIPM_F64), (8, 0, 8, sk.SKIPM_F64), (8, 10, 8, 7)]
    for m, n, lda, dt in bad:
        assert lib.normal_matvec_noalloc(a, dt, m, n, lda, None, a, a, None) == \
            sk.SKIPM_EINVAL, (m, n, lda, dt)
    assert lib.normal_matvec_noalloc(8, sk.SKIPM_F64, 8, 10, 8, None, a, a, None) == \
        sk.SKIPM_EINVAL   # A not 16-byte aligned
    assert lib.normal_matvec_noalloc(None, sk.SKIPM_F64, 8, 10, 8, None, a, a, None) == \
        sk.SKIPM_EINVAL
