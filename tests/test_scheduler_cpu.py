"""The served loop's scheduling on the CPU, through a scheduler-test context
(ps_create_scheduler_test): the same admission, continuous batching by time
slice, launch-ahead, cancellation, failure handling and timing bookkeeping
as on the GPU, with a stand-in for the device that writes a fixed pattern
-- (n_spins + sample index, slice index) per sample -- instead of
computing magnetisation.  The pattern shows that every sample of a request
is written once, by its own slices in order, whatever the mix; failures are
injected from the host (sections 5.3.2, 6.3, 7.3.1: the master's
bookkeeping, back-pressure and per-block results)."""
import time

import numpy as np
import pytest

from workloads import Sequence, configs as C
from workloads.phantom import random_spins


@pytest.fixture(scope="module")
def ps():
    import paper_1305_6861_amd as ps
    return ps


def _check_pattern(sig, obj, seq, n_slices=None):
    """Every sample written once with the request's own values, by slices in
    order (a slice may hold no sample: the first one of a readout cut off
    by the slice bound); returns the last slice index."""
    re, im = sig[0::2], sig[1::2]
    assert re.shape[0] == seq.n_samples
    np.testing.assert_array_equal(re, obj.n_spins + np.arange(seq.n_samples, dtype=np.float64))
    assert np.all(np.diff(im) >= 0) and np.all(im == np.round(im)) and im[0] >= 0
    if n_slices is not None:
        assert im[-1] < n_slices
    return int(im[-1])


def _long_2d(n_pe: int, n: int = 32, seed: int = 0):
    return random_spins(n * n, seed=seed), C.spoiled_gre_2d(n, n_pe)


def test_mix_alone_and_slices(ps):
    reqs = [C.c4_request(r) for r in range(12)] + [_long_2d(256, 64, 3)]
    with ps.SchedulerTest(iteration_seconds=0.0005, max_slice_steps=4096) as ctx:
        tickets = [ctx.submit(o, s) for o, s in reqs]
        outs = [t.wait(30.0).copy() for t in tickets]
        infos = [t.info() for t in tickets]
        iters = ctx.server_stats()["iterations"]
    for (o, s), sig, info in zip(reqs, outs, infos):
        assert info["state"] == "done"
        assert _check_pattern(sig, o, s, info["n_slices"]) == info["n_slices"] - 1
    assert infos[-1]["n_slices"] >= 4
    assert iters >= infos[-1]["n_slices"]
    with ps.SchedulerTest(max_slice_steps=4096) as ctx:            # the long one alone: same pattern
        alone = ctx.submit(*reqs[-1]).wait(30.0)
    np.testing.assert_array_equal(alone, outs[-1])


def test_admission_by_footprint_and_timing(ps):
    a = C.c4_request(3)
    with ps.SchedulerTest() as probe:
        tp = probe.submit(*a)               # the ticket owns the signal the stand-in writes
        tp.wait(30.0)
        need = tp.info()["footprint_bytes"]
    with ps.SchedulerTest(iteration_seconds=0.02, max_footprint_bytes=int(need * 1.5)) as ctx:
        t1, t2 = ctx.submit(*a), ctx.submit(*a)
        t1.wait(30.0)
        t2.wait(30.0)
        i1, i2 = t1.info(), t2.info()
        s1, s2 = t1.stats(), t2.stats()
    assert i2["t_admit"] >= i1["t_done"] - 1e-6                      # waited for memory
    assert s1["t_kernel"] == pytest.approx(0.02) and s2["t_kernel"] == pytest.approx(0.02)
    assert s2["t_queue"] >= 0.015 and s2["t_e2e"] >= s2["t_queue"] + 0.015


def test_cancel_queued_and_running(ps):
    long = _long_2d(512, 32, 1)                                        # 512 slices of one repetition
    short = C.c4_request(5)
    with ps.SchedulerTest(iteration_seconds=0.002, max_slice_steps=40) as ctx:
        t_long = ctx.submit(*long)
        for _ in range(2000):
            if t_long.info()["state"] == "running":
                break
            time.sleep(0.0005)
        t_short = ctx.submit(*short)
        t_long.cancel()
        with pytest.raises(ps.PsError) as ei:
            t_long.wait(30.0)
        assert ei.value.status == 6 and t_long.info()["state"] == "cancelled"
        _check_pattern(t_short.wait(30.0), *short)
    with ps.SchedulerTest(iteration_seconds=0.01, max_footprint_bytes=1) as ctx:
        with pytest.raises(ps.PsError) as ei:                          # over the cap alone
            ctx.submit(*short)
        assert ei.value.status == 4


def test_cancel_while_queued_behind_the_cap(ps):
    a = C.c4_request(3)
    with ps.SchedulerTest() as probe:
        tp = probe.submit(*a)               # the ticket owns the signal the stand-in writes
        tp.wait(30.0)
        need = tp.info()["footprint_bytes"]
    with ps.SchedulerTest(iteration_seconds=0.01, max_footprint_bytes=int(need * 1.5)) as ctx:
        t1, t2, t3 = ctx.submit(*a), ctx.submit(*a), ctx.submit(*a)
        t2.cancel()
        with pytest.raises(ps.PsError):
            t2.wait(30.0)
        assert t2.info()["t_admit"] < 0                                # never admitted
        _check_pattern(t1.wait(30.0), *a)
        _check_pattern(t3.wait(30.0), *a)


def test_injected_device_error_fails_only_its_iteration(ps):
    reqs = [_long_2d(64, 16, s) for s in range(3)]                    # several slices each
    with ps.SchedulerTest(iteration_seconds=0.001, fail_iteration=3, max_slice_steps=200) as ctx:
        tickets = [ctx.submit(o, s) for o, s in reqs]
        for t in tickets:
            try:
                t.wait(30.0)
            except ps.PsError:
                pass
        states = [t.info()["state"] for t in tickets]
        statuses = [t.info()["status"] for t in tickets]
        later = C.c4_request(2)
        ok = ctx.submit(*later)
        _check_pattern(ok.wait(30.0), *later)                          # the server serves on
    assert "failed" in states
    assert all(st == 3 for s, st in zip(states, statuses) if s == "failed")   # PS_E_DEVICE
    for (o, s), t, state in zip(reqs, tickets, states):
        if state == "done":
            _check_pattern(t._out, o, s)


def test_large_requests_run_one_at_a_time(ps):
    big = [(random_spins(400000, seed=s), C.spoiled_gre_2d(256, 256)) for s in range(2)]   # >= 2.5e10 spin-steps
    small = C.c4_request(1)
    with ps.SchedulerTest(iteration_seconds=0.003) as ctx:
        tb = [ctx.submit(o, s) for o, s in big]
        ts = ctx.submit(*small)
        for t in tb + [ts]:
            t.wait(60.0)
        ib = [t.info() for t in tb]
        i_s = ts.info()
    assert ib[0]["n_spins"] * ib[0]["n_steps_per_spin"] >= 2.5e10
    assert ib[1]["t_admit"] >= ib[0]["t_done"] - 1e-6                  # the second large one waited
    assert i_s["t_done"] < ib[1]["t_admit"] + 0.05                     # the small one went past it


def test_refusals(ps):
    o, s = C.c4_request(0)
    with ps.SchedulerTest() as ctx:
        with pytest.raises(ps.PsError) as ei:                          # an invalid request fails alone
            ctx.submit(random_spins(10, seed=1), Sequence("bad").add(float("nan"), n_adc=1))
        assert ei.value.status == 1
        _check_pattern(ctx.submit(o, s).wait(30.0), o, s)
        for call in (lambda: ctx.simulate(o, s), lambda: ctx.tune(o, s)):
            with pytest.raises(Exception):
                call()
