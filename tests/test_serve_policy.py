"""Host logic of the request loop (no GPU): admission order and the
preemption policy, checked against a stand-in batch that keeps slots, a
byte budget and cycle counts on the host.

- without preemption, urgent requests jump the queue but never displace a
  running request;
- with preemption, an urgent request that does not fit preempts normal runs,
  the smallest first (among equals the one with the most cycles left), and
  only as many as it needs;
- nothing is preempted when the urgent request would not fit beside the
  urgent runs alone;
- preempted runs resume before new normal requests and every request
  finishes after exactly its own cycle count.
"""
import time
import types

import pytest

from paper_0904_0232_amd import serve


class FakeBatch:
    """Slots, budget and per-run cycle counts; a run advances one cycle per
    step and finishes after its `steps`.  Preempt/resume hand back a token."""

    def __init__(self, budget, slots):
        self.budget, self.slots = budget, slots
        self.runs, self.next_id = {}, 1
        self.log = []

    def used(self):
        return sum(r["bytes"] for r in self.runs.values() if r["state"] == "active")

    def n_active(self):
        return sum(1 for r in self.runs.values() if r["state"] == "active")


def fake_capi(b_holder):
    RUN_ACTIVE, RUN_DONE, RUN_PREEMPTED = 1, 2, 3

    def create(budget, slots):
        b_holder.append(FakeBatch(budget, slots))
        return b_holder[-1]

    def submit(b, cfg, nsteps, parts, keep_state=False):
        if b.n_active() >= b.slots or b.used() + cfg["bytes"] > b.budget:
            return None
        rid = b.next_id
        b.next_id += 1
        b.runs[rid] = {"req": cfg["id"], "bytes": cfg["bytes"], "steps": nsteps, "done": 0, "state": "active"}
        b.log.append(("submit", cfg["id"]))
        return rid

    def step(b):
        time.sleep(2e-4)  # a cycle takes time, so later arrivals meet running work
        fin = 0
        for r in b.runs.values():
            if r["state"] == "active":
                r["done"] += 1
                if r["done"] == r["steps"]:
                    r["state"] = "done"
                    fin += 1
        return fin

    def poll(b, rid):
        r = b.runs[rid]
        st = {"active": RUN_ACTIVE, "done": RUN_DONE, "preempted": RUN_PREEMPTED}[r["state"]]
        return st, r["done"], ({"cycles": r["done"]} if st == RUN_DONE else None), 0, r["done"]

    def preempt(b, rid):
        r = b.runs[rid]
        assert r["state"] == "active"
        r["state"] = "preempted"
        b.log.append(("preempt", r["req"], r["steps"] - r["done"]))
        return ("token", rid, r["done"])

    def resume(b, rid, state):
        r = b.runs[rid]
        assert r["state"] == "preempted" and state == ("token", rid, r["done"])
        if b.n_active() >= b.slots or b.used() + r["bytes"] > b.budget:
            return False
        r["state"] = "active"
        b.log.append(("resume", r["req"]))
        return True

    def stats(b):
        return b.n_active(), b.used()

    def release(b, rid):
        assert b.runs[rid]["state"] in ("done", "preempted")

    return types.SimpleNamespace(
        RUN_ACTIVE=RUN_ACTIVE, RUN_DONE=RUN_DONE, RUN_PREEMPTED=RUN_PREEMPTED,
        grpic_batch_create=create, grpic_batch_submit=submit, grpic_batch_step=step, grpic_batch_poll=poll,
        grpic_batch_preempt=preempt, grpic_batch_resume=resume, grpic_batch_stats=stats,
        grpic_batch_release=release, grpic_batch_dump=lambda b, rid, n: None,
        grpic_batch_destroy=lambda b: None, grpic_run_bytes=lambda cfg: cfg["bytes"])


@pytest.fixture
def loop(monkeypatch):
    holder = []
    monkeypatch.setattr(serve, "capi", fake_capi(holder))
    monkeypatch.setattr(serve, "request_config", lambda r: {"id": r["id"], "bytes": r["bytes"]})
    monkeypatch.setattr(serve, "request_particles", lambda r: None)
    return holder


def req(i, steps, priority=0, arrival=0.0, nbytes=1):
    return {"id": i, "steps": steps, "priority": priority, "arrival": arrival, "bytes": nbytes, "edge": 16}


def run_loop(holder, reqs, budget, slots, preempt):
    res = serve.serve(reqs, budget, slots, preempt=preempt)
    b = holder[-1]
    assert res["n_runs"] == len(reqs)
    for r in b.runs.values():  # every run did exactly its own cycle count
        assert r["state"] == "done" and r["done"] == r["steps"]
    return res, b.log


def test_urgent_jumps_the_queue_without_preemption(loop):
    reqs = [req(0, 40), req(1, 40), req(2, 5), req(3, 5, priority=1)]
    res, log = run_loop(loop, reqs, 100, 2, preempt=False)
    assert res["preemptions"] == 0
    assert [e for e in log if e[0] != "submit"] == []
    assert [e[1] for e in log] == [3, 0, 1, 2]  # urgent first; the rest in arrival order


def test_preemption_among_equal_runs_takes_the_most_cycles_left(loop):
    # two normal runs fill both slots; the urgent one arrives once they run
    reqs = [req(0, 1000), req(1, 800), req(2, 10, priority=1, arrival=0.03)]
    res, log = run_loop(loop, reqs, 100, 2, preempt=True)
    pre = [e for e in log if e[0] == "preempt"]
    assert res["preemptions"] == 1 and len(pre) == 1 and pre[0][1] == 0
    assert log.index(("submit", 2)) > log.index(pre[0])
    assert log.index(("resume", 0)) > log.index(("submit", 2))
    assert res["records"][0]["preemptions"] == 1 and res["records"][1]["preemptions"] == 0


def test_preemption_takes_the_smallest_run_first(loop):
    reqs = [req(0, 1000, nbytes=3), req(1, 500, nbytes=1), req(2, 10, priority=1, arrival=0.03)]
    res, log = run_loop(loop, reqs, 100, 2, preempt=True)
    assert [e[1] for e in log if e[0] == "preempt"] == [1]


def test_preempts_only_as_many_as_the_budget_needs(loop):
    # four normal runs of 1 byte in a 4-byte budget; an urgent run of 2 bytes
    # needs two of them gone
    reqs = [req(i, 600 + 10 * i) for i in range(4)] + [req(9, 5, priority=1, arrival=0.03, nbytes=2)]
    res, log = run_loop(loop, reqs, 4, 8, preempt=True)
    pre = [e[1] for e in log if e[0] == "preempt"]
    assert pre == [3, 2]
    assert log.index(("resume", 3)) > log.index(("submit", 9))


def test_no_preemption_when_urgent_runs_fill_the_batch(loop):
    # the second urgent run (2 bytes) cannot fit beside the first (2 bytes) in
    # 3 bytes, so preempting the normal run would not help
    reqs = [req(0, 1000), req(1, 200, priority=1, nbytes=2), req(2, 10, priority=1, arrival=0.03, nbytes=2)]
    res, log = run_loop(loop, reqs, 3, 4, preempt=True)
    assert res["preemptions"] == 0
    assert log.index(("submit", 2)) == len(log) - 1


def test_resumed_runs_go_before_new_normal_requests(loop):
    # run 2 arrives while the urgent run holds the one slot and run 0 is parked
    reqs = [req(0, 600), req(1, 150, priority=1, arrival=0.03), req(2, 10, arrival=0.04)]
    res, log = run_loop(loop, reqs, 100, 1, preempt=True)
    assert [e[1] for e in log if e[0] == "preempt"] == [0]
    assert log.index(("resume", 0)) < log.index(("submit", 2))
