"""The serving benchmark's wait loop (bench.serve_trace) against a stand-in
request server on the CPU: every request is collected once, in ticket order
of the results, and a server on which no request finishes ends the run with
a report instead of a hang."""
import os
import sys
import types
from dataclasses import dataclass

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

QUEUED, RUNNING, DONE = 0, 1, 2


@dataclass
class _Res:
    status: int = 0
    rel_gap: float = 0.0
    obj_p: float = 1.0


@dataclass
class _Info:
    result: _Res
    state: int
    rc: int
    footprint: int
    device_bytes: int
    t_submit: float
    t_start: float
    t_done: float

    @property
    def latency(self):
        return self.t_done - self.t_submit


class _Server:
    """Request i finishes at the poll count done_after[i] (None: never)."""

    def __init__(self, done_after):
        self.done_after = done_after
        self.polls = 0
        self.submitted = 0
        self.waited = []

    def submit(self, *a, **k):
        self.submitted += 1
        return self.submitted - 1

    def now(self):
        return 0.0

    def _info(self, t):
        d = self.done_after[t]
        state = DONE if d is not None and self.polls >= d else RUNNING
        return _Info(_Res(), state, 0, 10**9, 0, 0.0, 0.01 * t, 0.02 * t + 0.5)

    def poll(self, t):
        self.polls += 1
        return self._info(t)

    def wait(self, t):
        assert self._info(t).state == DONE
        self.waited.append(t)
        return self._info(t), None

    def stats(self):
        return {"peak_in_use": 10**9}

    def close(self):
        pass


def _run(done_after, stall_timeout):
    srv = _Server(done_after)
    sk = types.SimpleNamespace(Server=lambda budget, slots: srv, SKIPM_REQ_QUEUED=QUEUED,
                               SKIPM_REQ_RUNNING=RUNNING, SKIPM_REQ_DONE=DONE)
    args = types.SimpleNamespace(hbm_budget_gb=1.0, workers=2, s=2, stall_timeout=stall_timeout)
    n = len(done_after)
    trace = [dict(idx=i, t=0.0, m=10, n=100, kind="dense") for i in range(n)]
    lps = [types.SimpleNamespace(A=None, b=None, c=None, w=40, seed=i, eps_gap=1e-6, opt=1.0)
           for i in range(n)]
    return srv, bench.serve_trace(sk, None, args, trace, lps)


def test_every_request_collected_once():
    srv, r = _run([5, 1, 30, 12], stall_timeout=60.0)
    assert sorted(srv.waited) == [0, 1, 2, 3]
    assert r["n_ok"] == 4 and r["all_ok"]


def test_a_server_that_never_finishes_ends_with_a_report():
    with pytest.raises(RuntimeError, match="no request finished"):
        _run([1, None], stall_timeout=0.2)
