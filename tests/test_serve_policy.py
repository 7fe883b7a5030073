"""Scheduling policy of the rate server, on the CPU with a fake executor and
a fake clock (the GPU executor is exercised in tests/test_gpu_serve.py)."""
import numpy as np
import pytest

from paper_1005_5312_amd.serve import Executor, Request, Scene, Server


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor(Executor):
    """Each launched batch finishes `duration` seconds of fake time later;
    results are the targets' x coordinates (so outputs are checkable)."""

    def __init__(self, clock, n_slots=2, duration=1.0, fail_scene=None, poison=None, launch_fail=None,
                 build_fail=None):
        self.clock = clock
        self.n_slots = n_slots
        self.duration = duration
        self.fail_scene = fail_scene
        self.poison = poison            # a batch holding a target at x == poison fails on the device
        self.launch_fail = launch_fail  # launching a batch with this scene raises
        self.build_fail = build_fail    # building this scene raises
        self.built = []
        self.freed = []
        self.launches = []

    def scene_bytes(self, scene):
        return 100 * scene.n_src

    def request_bytes(self, req):
        return 10 * req.n_t

    def build_scene(self, scene):
        if scene.key == self.build_fail:
            raise RuntimeError("build failed")
        self.built.append(scene.key)
        return ("handle", scene.key)

    def free_scene(self, handle):
        self.freed.append(handle[1])

    def launch(self, slot, batch, scenes):
        if any(r.scene.key == self.launch_fail for r in batch):
            raise RuntimeError("launch failed")
        for r in batch:
            assert scenes[r.scene.key] == ("handle", r.scene.key)
        self.launches.append((self.clock(), slot, [r.rid for r in batch]))
        return (self.clock() + self.duration, batch)

    def done(self, token):
        return self.clock() >= token[0]

    def results(self, token):
        if any(r.scene.key == self.fail_scene for r in token[1]):
            raise RuntimeError("device error")
        if self.poison is not None and any(np.any(r.tgt_xyz[0] == self.poison) for r in token[1]):
            raise RuntimeError("device-side input error")
        return [r.tgt_xyz[0].copy() for r in token[1]]


def scene(key, n_src=10):
    z = np.zeros((3, n_src))
    return Scene(key, None, z, np.ones(n_src), z, np.ones(n_src), np.ones(n_src), 3)


def req(sc, n_t, tag=0.0):
    xyz = np.full((3, n_t), float(tag))
    return Request(sc, xyz)


def run_until_idle(server, clock, dt=0.25, limit=1000):
    for _ in range(limit):
        server.step()
        if server._idle():
            return
        clock.t += dt
    raise AssertionError("server did not become idle")


def test_results_and_latency():
    clock = Clock()
    ex = FakeExecutor(clock)
    s = Server(ex, hbm_budget=10_000, clock=clock)
    sc = scene("a")
    futs = [s.submit(req(sc, 5, tag=k)) for k in range(6)]
    run_until_idle(s, clock)
    for k, f in enumerate(futs):
        assert np.all(f.result() == k)
    st = s.latency_stats()
    assert st["requests"] == 6 and st["p99_ms"] >= st["p50_ms"] > 0


def test_admission_waits_for_memory_in_arrival_order():
    clock = Clock()
    ex = FakeExecutor(clock, n_slots=4)
    # scene 1000 B + each request 600 B; budget 2300 B: two requests at once
    s = Server(ex, hbm_budget=2300, max_batch=1, clock=clock)
    sc = scene("a")
    futs = [s.submit(req(sc, 60, tag=k)) for k in range(5)]
    s.step()
    assert len(s.inflight) == 2 and len(s.pending) == 3
    assert s.used <= s.budget
    run_until_idle(s, clock)
    order = [rid for _, _, rids in ex.launches for rid in rids]
    assert order == sorted(order)          # admitted and launched oldest first
    assert all(f.done() for f in futs)


def test_no_overtaking_and_no_starvation():
    clock = Clock()
    ex = FakeExecutor(clock, n_slots=2)
    s = Server(ex, hbm_budget=3000, max_batch=8, clock=clock)
    sc = scene("a")
    small = [s.submit(req(sc, 10)) for _ in range(3)]
    big = s.submit(req(sc, 190))           # 1900 B: must wait for the small ones
    later = [s.submit(req(sc, 10)) for _ in range(20)]
    for _ in range(400):
        s.step()
        if big.done():
            break
        clock.t += 0.25
    assert big.done()
    big_rid = next(r.rid for r in s.completed if r.n_t == 190)
    # nothing submitted after the big request started before it
    started = {rid: t for t, _, rids in ex.launches for rid in rids}
    assert all(started[rid] >= started[big_rid] for rid in started if rid > big_rid)
    run_until_idle(s, clock)
    assert all(f.done() for f in small + later)


def test_continuous_batching_overlaps_slots():
    clock = Clock()
    ex = FakeExecutor(clock, n_slots=2, duration=2.0)
    s = Server(ex, hbm_budget=100_000, max_batch=4, clock=clock)
    sc = scene("a")
    for _ in range(3):
        s.submit(req(sc, 5))
    s.step()                                # first batch on slot 0
    clock.t += 0.5
    for _ in range(3):
        s.submit(req(sc, 5))                # arrive while slot 0 is busy
    s.step()                                # join a second batch on slot 1
    assert set(s.inflight) == {0, 1}
    run_until_idle(s, clock)
    assert len(s.completed) == 6


def test_scene_resident_and_evicted_lru():
    clock = Clock()
    ex = FakeExecutor(clock, n_slots=1)
    # each scene 1000 B; budget fits two scenes plus a request
    s = Server(ex, hbm_budget=2200, clock=clock)
    a, b, c = scene("a"), scene("b"), scene("c")
    for sc in (a, a, b):
        s.submit(req(sc, 5))
    run_until_idle(s, clock)
    assert ex.built == ["a", "b"]           # "a" built once and reused
    s.submit(req(c, 5))                     # needs room: "a" is least recently used
    run_until_idle(s, clock)
    assert ex.built == ["a", "b", "c"] and ex.freed == ["a"]
    assert s.used == 2000


def test_failed_batch_fails_only_its_requests():
    clock = Clock()
    ex = FakeExecutor(clock, n_slots=2, fail_scene="bad")
    s = Server(ex, hbm_budget=100_000, max_batch=1, clock=clock)
    good = [s.submit(req(scene("ok"), 5)) for _ in range(3)]
    bad = s.submit(req(scene("bad"), 5))
    run_until_idle(s, clock)
    assert all(f.result() is not None for f in good)
    with pytest.raises(RuntimeError):
        bad.result()
    assert s.used == 2000                   # two resident scenes, no request left


def test_request_larger_than_budget_is_refused():
    clock = Clock()
    s = Server(FakeExecutor(clock), hbm_budget=500, clock=clock)
    with pytest.raises(ValueError):
        s.submit(req(scene("a"), 5))


def test_threaded_loop_drains():
    import threading
    ex_clock = Clock()

    class Timed(FakeExecutor):
        def done(self, token):
            return True

    s = Server(Timed(ex_clock), hbm_budget=100_000).start()
    sc = scene("a")
    futs = []
    threads = [threading.Thread(target=lambda: futs.extend(s.submit(req(sc, 3)) for _ in range(20)))
               for _ in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    s.drain(timeout=30)
    s.stop()
    assert len(futs) == 80 and all(f.done() for f in futs)


def test_bad_request_in_a_batch_fails_alone():
    """A batch that fails on the device is split: its requests run again one
    by one and only the bad one fails; its reservations are all returned."""
    clock = Clock()
    ex = FakeExecutor(clock, n_slots=1, poison=99.0)
    s = Server(ex, hbm_budget=100_000, max_batch=16, clock=clock)
    sc = scene("a")
    futs = [s.submit(req(sc, 5, tag=k)) for k in range(3)]
    bad = s.submit(req(sc, 5, tag=99.0))
    futs += [s.submit(req(sc, 5, tag=k)) for k in range(3, 6)]
    run_until_idle(s, clock)
    assert len(ex.launches[0][2]) == 7                      # all in one batch first
    for k, f in enumerate(futs):
        assert np.all(f.result() == k)
    with pytest.raises(RuntimeError):
        bad.result()
    assert [rid for rid, _ in s.errors] == [bad_rid(s, 99.0)]
    assert s.used == 1000 and sum(s.scene_users.values()) == 0


def bad_rid(server, tag):
    return next(r.rid for r in server.completed if r.tgt_xyz is not None and r.tgt_xyz[0, 0] == tag)


def test_malformed_request_fails_at_submit():
    clock = Clock()
    s = Server(FakeExecutor(clock), hbm_budget=100_000, clock=clock)
    sc = scene("a")
    nan = np.zeros((3, 4))
    nan[1, 2] = np.nan
    bad = [s.submit(Request(sc, nan)), s.submit(Request(sc, np.zeros((3, 4)), theta=-1.0)),
           s.submit(Request(sc, np.zeros((3, 4)), prec="fp16")),
           s.submit(Request(sc, np.zeros((3, 4)), self_src=np.array([0, 1, 2, 10])))]
    good = s.submit(req(sc, 4, tag=1.0))
    for f in bad:
        assert f.done()
        with pytest.raises(ValueError):
            f.result()
    run_until_idle(s, clock)
    assert np.all(good.result() == 1.0)
    assert s.used == 1000 and len(s.errors) == 4


def test_launch_and_build_errors_are_contained():
    """An exception while launching or while building a scene fails only the
    requests concerned; the loop goes on and nothing stays reserved."""
    clock = Clock()
    ex = FakeExecutor(clock, n_slots=2, launch_fail="L", build_fail="B")
    s = Server(ex, hbm_budget=100_000, max_batch=8, clock=clock)
    ok = [s.submit(req(scene("a"), 5, tag=k)) for k in range(3)]
    lf = [s.submit(req(scene("L"), 5)) for _ in range(2)]
    bf = [s.submit(req(scene("B"), 5)) for _ in range(2)]
    ok += [s.submit(req(scene("a"), 5, tag=k)) for k in range(3, 5)]
    run_until_idle(s, clock)
    for k, f in enumerate(ok):
        assert np.all(f.result() == k)
    for f in lf + bf:
        with pytest.raises(RuntimeError):
            f.result()
    assert "B" not in s.scenes and sum(s.scene_users.values()) == 0
    assert s.used == 2000                   # scenes "a" and "L" resident, nothing else held


def test_builds_do_not_hold_up_resident_scenes():
    """With the builder thread, a slow scene build runs while requests on a
    resident scene are dispatched and complete."""
    import threading
    import time as _time
    gate = threading.Event()

    class SlowBuild(FakeExecutor):
        def build_scene(self, scene):
            if scene.key == "slow":
                gate.wait(10)
            return super().build_scene(scene)

        def done(self, token):
            return True

    s = Server(SlowBuild(Clock()), hbm_budget=100_000).start()
    a = scene("a")
    s.submit(req(a, 3)).result(timeout=10)            # "a" resident
    slow = s.submit(req(scene("slow"), 3))
    _time.sleep(0.05)
    quick = [s.submit(req(a, 3, tag=k)) for k in range(5)]
    for k, f in enumerate(quick):
        assert np.all(f.result(timeout=10) == k)
    assert not slow.done()
    gate.set()
    assert slow.result(timeout=10) is not None
    s.drain(timeout=10)
    s.stop()
