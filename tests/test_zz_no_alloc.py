"""normal_matvec_noalloc: the product A D^2 A^T u on the caller's own A and
D^2 with no handle and no device allocation (partial sums in the library's
static scratch buffer), against normal_matvec of a handle holding the same A
and D^2 (the same kernels: bitwise equal) and against the oracle's normal
matrix (element by element within the summation bound)."""
import ctypes
import sys

import numpy as np
import pytest

from lpgen import dense_planted
from oracle import ipm as O

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


@pytest.fixture(scope="module")
def sk():
    import paper_2003_08072_amd as _sk
    _sk.load()
    return _sk


def padded_colmajor(torch, A, dtype):
    """A (m x n) as the library lays it out: column-major, lda = m rounded up
    to 4, padding rows zero."""
    m, n = A.shape
    lda = (m + 3) // 4 * 4
    buf = torch.zeros((n, lda), dtype=dtype, device="cuda")
    buf[:, :m] = torch.from_numpy(np.ascontiguousarray(A.T)).to(device="cuda", dtype=dtype)
    return buf, lda


def noalloc(sk, torch, Abuf, a_dtype, m, n, lda, d2, u):
    out = torch.empty(m, dtype=torch.float64, device="cuda")
    lib = sk.load()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.normal_matvec_noalloc(Abuf.data_ptr(), a_dtype, m, n, lda, d2.data_ptr(),
                                   u.data_ptr(), out.data_ptr(), st)
    assert rc == sk.SKIPM_OK, lib.skipm_last_error()
    return out


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_noalloc_product_matches_normal_matvec(torch, sk, dt):
    """Two calls in a row on one device: the largest shape the scratch buffer
    holds (m = 2048, 512 workgroups of partials), then a smaller ragged one;
    each against the handle's normal_matvec and the oracle."""
    tdt = torch.float64 if dt == "f64" else torch.float32
    code = sk.SKIPM_F64 if dt == "f64" else sk.SKIPM_F32
    for m, n, seed in ((2048, 10_000, 1), (37, 3001, 2)):
        say(f"noalloc product {dt} m={m} n={n}")
        rng = np.random.default_rng(seed)
        lp = dense_planted(m, n, rng=rng, a_dtype=dt)
        d2 = rng.uniform(0.01, 10.0, n)
        u = rng.standard_normal(m)
        with sk.LP(lp.A, lp.b, lp.c, a_dtype=dt, s=2, seed=1) as h:
            h.pcg(d2, np.ones(m), 0, tol=0.0, max_it=1)   # leaves D^2 = diag(d2) in the handle
            ref_gpu = h.normal_matvec(u).cpu().numpy()
        Abuf, lda = padded_colmajor(torch, lp.A, tdt)
        d2t = torch.from_numpy(d2).cuda()
        ut = torch.from_numpy(u).cuda()
        got = noalloc(sk, torch, Abuf, code, m, n, lda, d2t, ut).cpu().numpy()
        assert np.array_equal(got, ref_gpu)
        ref = O.normal_matrix(lp.A, d2) @ u
        bound = np.abs(lp.A) @ (d2 * (np.abs(lp.A).T @ np.abs(u)))
        assert np.all(np.abs(got - ref) <= 2 * (m + n) * EPS * bound)


def test_noalloc_rejects_what_the_scratch_cannot_hold(torch, sk):
    say("noalloc argument checks")
    lib = sk.load()
    buf = torch.zeros(16, dtype=torch.float64, device="cuda")
    p = buf.data_ptr()
    for m, n, lda in ((2049, 10, 2052), (8, 10, 6), (8, 10, 4096), (0, 10, 4)):
        assert lib.normal_matvec_noalloc(p, sk.SKIPM_F64, m, n, lda, None, p, p, None) == \
            sk.SKIPM_EINVAL, (m, n, lda)
