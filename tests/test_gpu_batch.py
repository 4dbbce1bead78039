"""Many LPs at once: lp_solve_batch and the request server, through the C ABI.

The bar: each LP's result and final iterate are bitwise the same alone and in
a batch or in the server's mix (an LP's arithmetic never depends on what runs
beside it), and each meets the stopping tolerance against its planted optimum.
"""
import sys

import numpy as np
import pytest

from lpgen import batch_lp, csr_planted, dense_planted

pytestmark = pytest.mark.gpu


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


def mixed_set():
    """Small LPs of uneven shape and format: dense FP64, dense FP32, CSR."""
    out = []
    rng = np.random.default_rng(11)
    for i, (m, n) in enumerate([(20, 500), (45, 2000), (7, 300), (64, 5000), (33, 900),
                                (120, 6000)]):
        out.append(dense_planted(m, n, rng=rng, a_dtype="f64" if i % 2 else "f32",
                                 eps_gap=1e-8, seed=100 + i))
    for i, (m, n, dens) in enumerate([(30, 4000, 0.01), (80, 10000, 0.005)]):
        out.append(csr_planted(m, n, dens, rng=np.random.default_rng(20 + i), eps_gap=1e-8,
                               seed=200 + i))
    return out


def check_planted(lp, r):
    assert r.status == 0, r
    assert r.rel_gap <= lp.eps_gap
    assert abs(r.obj_p - lp.opt) <= 2 * lp.eps_gap * max(1.0, abs(lp.opt))


def same(r1, r2):
    for f in ("status", "iters", "cg_total", "cg_max", "obj_p", "obj_d", "rel_gap", "rp_norm",
              "rd_norm", "mu"):
        assert getattr(r1, f) == getattr(r2, f), f


def test_batch_matches_lone_solves(torch, sk):
    lps = mixed_set()
    say(f"batch of {len(lps)} mixed LPs, 4 workers, vs lone solves")
    hs = [sk.LP(lp.A, lp.b, lp.c, a_dtype=lp.a_dtype, w=lp.w, seed=lp.seed,
                eps_gap=lp.eps_gap) for lp in lps]
    lone, xs = [], []
    for h in hs:
        lone.append(h.solve())
        xs.append(h.get_iterate()[0].cpu().numpy())
        h.reset()
    torch.cuda.synchronize()
    batch = sk.solve_batch(hs, workers=4)
    for lp, h, r1, r2, x1 in zip(lps, hs, lone, batch, xs):
        check_planted(lp, r2)
        same(r1, r2)
        assert np.array_equal(h.get_iterate()[0].cpu().numpy(), x1)
    for h in hs:
        h.close()


def test_batch_matches_lone_solves_32_lane_groups(torch, sk):
    """LPs whose column passes take 32-lane groups (FP32 m in (256, 384], FP64
    m in (128, 192]) and 16-lane groups of three vectors (FP32 m in (128, 192],
    FP64 m in (64, 96]) next to 64-lane ones, at the batched workload's gap and
    column ratio: the grouped launches give each LP its lone solve, bitwise."""
    shapes = [(300, 9000, "f32"), (160, 4800, "f64"), (384, 7680, "f32"), (200, 4000, "f32"),
              (150, 4500, "f32"), (80, 3200, "f64")]
    lps = [dense_planted(m, n, rng=np.random.default_rng(60 + i), a_dtype=dt, eps_gap=1e-6,
                         seed=300 + i) for i, (m, n, dt) in enumerate(shapes)]
    say(f"batch of {len(lps)} LPs with 32-lane column groups vs lone solves")
    hs = [sk.LP(lp.A, lp.b, lp.c, a_dtype=lp.a_dtype, w=lp.w, seed=lp.seed,
                eps_gap=lp.eps_gap) for lp in lps]
    lone, xs = [], []
    for h in hs:
        lone.append(h.solve())
        xs.append(h.get_iterate()[0].cpu().numpy())
        h.reset()
    torch.cuda.synchronize()
    batch = sk.solve_batch(hs, workers=4)
    for lp, h, r1, r2, x1 in zip(lps, hs, lone, batch, xs):
        check_planted(lp, r2)
        same(r1, r2)
        assert np.array_equal(h.get_iterate()[0].cpu().numpy(), x1)
    for h in hs:
        h.close()


def test_batch_workload_sample(torch, sk):
    idx = list(range(12))
    say("batched workload: LPs 0..11 (dense FP32, m in [20, 400], n = m k)")
    lps = [batch_lp(i) for i in idx]
    hs = [sk.LP(lp.A, lp.b, lp.c, a_dtype=lp.a_dtype, w=lp.w, seed=lp.seed,
                eps_gap=lp.eps_gap) for lp in lps]
    res = sk.solve_batch(hs, workers=8)
    for lp, r in zip(lps, res):
        check_planted(lp, r)
    for h in hs:
        h.close()


def test_server_same_alone_and_in_the_mix(torch, sk):
    lps = mixed_set()
    say(f"server: {len(lps)} requests, 3 slots, budget for about two at once")
    fps = []
    for lp in lps:
        prob, keep = sk.problem(lp.A, lp.b, lp.c, lp.a_dtype)
        fps.append(sk.footprint(prob, w=lp.w, seed=lp.seed, eps_gap=lp.eps_gap))
        del keep
    budget = int(sorted(fps)[-1] + sorted(fps)[-2])
    alone = []
    for lp in lps:
        with sk.LP(lp.A, lp.b, lp.c, a_dtype=lp.a_dtype, w=lp.w, seed=lp.seed,
                   eps_gap=lp.eps_gap) as h:
            alone.append((h.solve(), h.get_iterate()[0].cpu().numpy(), h.device_bytes()))
    with sk.Server(budget, slots=3) as srv:
        tickets = [srv.submit(lp.A, lp.b, lp.c, a_dtype=lp.a_dtype, want_x=True, w=lp.w,
                              seed=lp.seed, eps_gap=lp.eps_gap) for lp in lps]
        got = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert st["completed"] == len(lps) and st["running"] == 0 and st["queued"] == 0
    assert st["peak_in_use"] <= budget
    for lp, (r1, x1, bytes1), (rq, x2), fp in zip(lps, alone, got, fps):
        assert rq.state == sk.SKIPM_REQ_DONE and rq.rc == 0
        check_planted(lp, rq.result)
        same(r1, rq.result)
        assert np.array_equal(x2.cpu().numpy(), x1)
        assert rq.footprint == fp and bytes1 <= fp and rq.device_bytes == bytes1
        assert rq.t_submit <= rq.t_start <= rq.t_done


def test_server_rejects_what_never_fits(torch, sk):
    lp = dense_planted(20, 500, rng=np.random.default_rng(5), a_dtype="f32")
    say("server: request above the whole budget")
    with sk.Server(1 << 20, slots=1) as srv:
        with pytest.raises(sk.SkipmError) as e:
            srv.submit(lp.A, lp.b, lp.c, a_dtype="f32")
        assert e.value.code == sk.SKIPM_ENOMEM


def serving_sample(per_kind=3, dense_cap=2.0e7, csr_cap=4.0e5):
    """The first requests of the serving trace itself (m log-uniform in
    [50, 2000], n/m log-uniform in [50, 500]) of each kind whose size keeps
    a solve within seconds: dense m n <= dense_cap entries, CSR
    0.01 m n + n <= csr_cap non-zeros (the all-ones row included)."""
    from lpgen import serving_trace
    out, got = [], {"dense": 0, "csr": 0}
    for req in serving_trace():
        kind = req["kind"]
        size = req["m"] * req["n"] if kind == "dense" else 0.01 * req["m"] * req["n"] + req["n"]
        if got[kind] < per_kind and size <= (dense_cap if kind == "dense" else csr_cap):
            out.append(req)
            got[kind] += 1
        if min(got.values()) >= per_kind:
            break
    return out


def test_server_on_serving_trace_requests(torch, sk):
    """Requests of the serving workload's own trace (both kinds) through the
    server with 3 slots and a budget for about two at once: each meets its
    planted optimum and the KKT bounds, and its result and final x are
    bitwise those of the same LP solved alone."""
    from lpgen import serving_lp
    reqs = serving_sample()
    lps = [serving_lp(r) for r in reqs]
    say("server on serving-trace requests: " +
        ", ".join(f"{r['kind']} {r['m']}x{r['n']}" for r in reqs))
    assert {r["kind"] for r in reqs} == {"dense", "csr"}
    kw = [dict(w=lp.w, seed=lp.seed, eps_gap=lp.eps_gap, s=2) for lp in lps]
    fps = []
    for lp, k in zip(lps, kw):
        prob, keep = sk.problem(lp.A, lp.b, lp.c, lp.a_dtype)
        fps.append(sk.footprint(prob, **k))
        del keep
    budget = int(sorted(fps)[-1] + sorted(fps)[-2])
    alone = []
    for lp, k in zip(lps, kw):
        with sk.LP(lp.A, lp.b, lp.c, a_dtype=lp.a_dtype, **k) as h:
            alone.append((h.solve(), h.get_iterate()[0].cpu().numpy()))
    with sk.Server(budget, slots=3) as srv:
        tickets = [srv.submit(lp.A, lp.b, lp.c, a_dtype=lp.a_dtype, want_x=True, **k)
                   for lp, k in zip(lps, kw)]
        got = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert st["completed"] == len(lps) and st["peak_in_use"] <= budget
    for lp, (r1, x1), (rq, x2) in zip(lps, alone, got):
        assert rq.state == sk.SKIPM_REQ_DONE and rq.rc == 0
        check_planted(lp, rq.result)
        assert rq.result.rp_norm <= 1e-8 * np.linalg.norm(lp.b)
        assert rq.result.rd_norm <= 1e-8 * np.linalg.norm(lp.c)
        same(r1, rq.result)
        assert np.array_equal(x2.cpu().numpy(), x1)


def test_batch_with_a_rank_lost_lp(torch, sk):
    """A batch holding an LP whose sketch loses rank at every salt (a zero row
    of A): it ends with SKIPM_ERANK after its fresh sketches and shifts, the
    same result as alone, and the other LPs of the batch are unaffected."""
    rng = np.random.default_rng(77)
    bad = dense_planted(24, 600, rng=rng)
    A = bad.A.copy()
    A[5] = 0.0
    lps = [dense_planted(40, 3000, rng=np.random.default_rng(3), eps_gap=1e-8, seed=4),
           (A, A @ bad.x_star, A.T @ bad.y_star + bad.s_star),
           dense_planted(90, 5000, rng=np.random.default_rng(4), a_dtype="f32", eps_gap=1e-8,
                         seed=5)]
    say("batch with a rank-lost LP (zero row) between two planted LPs")

    def make(x):
        if isinstance(x, tuple):
            return sk.LP(*x, s=2, seed=3)
        return sk.LP(x.A, x.b, x.c, a_dtype=x.a_dtype, s=2, seed=x.seed, eps_gap=x.eps_gap)

    hs = [make(x) for x in lps]
    lone = []
    for h in hs:
        lone.append(h.solve())
        h.reset()
    torch.cuda.synchronize()
    batch = sk.solve_batch(hs, workers=3)
    assert batch[1].status == sk.SKIPM_ERANK
    assert batch[1].resketches >= 3 and batch[1].shifts >= 3
    for r1, r2 in zip(lone, batch):
        same(r1, r2)
    check_planted(lps[0], batch[0])
    check_planted(lps[2], batch[2])
    for h in hs:
        h.close()


def test_batch_with_capped_cg(torch, sk):
    """LPs with different CG caps in one batch (caps of 4 and 7 iterations stop
    most of their CG solves early; max_outer 8 ends the runs): every result is
    bitwise that of the same LP alone."""
    lps = [dense_planted(70, 4000, rng=np.random.default_rng(40 + i), a_dtype=dt, seed=i)
           for i, dt in enumerate(("f32", "f64", "f32"))]
    caps = (4, 1000, 7)
    say("batch with CG caps 4, 1000, 7 and max_outer 8")
    hs = [sk.LP(lp.A, lp.b, lp.c, a_dtype=lp.a_dtype, s=1, seed=lp.seed, max_cg=cap,
                max_outer=8) for lp, cap in zip(lps, caps)]
    lone = []
    for h in hs:
        lone.append(h.solve())
        h.reset()
    torch.cuda.synchronize()
    batch = sk.solve_batch(hs, workers=2)
    for r1, r2 in zip(lone, batch):
        same(r1, r2)
    assert batch[0].cg_max <= 4 and batch[2].cg_max <= 7
    for h in hs:
        h.close()
