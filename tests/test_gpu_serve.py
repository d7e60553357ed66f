"""GPU: served execution (ps_submit / ps_wait) -- continuous batching with
admission by device footprint.  Failure handling (cancel, over-cap and
invalid requests) is forced from the host; every kernel still completes."""
import time

import numpy as np
import pytest

import oracle
from tests.parity import within
from workloads import Sequence, SPOIL, configs as C
from workloads.phantom import grid3d_two_species, random_spins

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


@pytest.fixture(scope="module")
def ps():
    import paper_1305_6861_amd as ps
    return ps


def _np(t):
    return t.cpu().numpy()


def _small_3d():
    obj = grid3d_two_species(24, seed=77)                    # 27,648 spins
    seq = C.gre_3d_sinc(24, 24, 24)                           # 576 TRs: several time slices
    return obj, seq


def test_served_mix_matches_oracle_and_alone_bitwise(ps):
    reqs = [C.c4_request(r) for r in range(10)] + [_small_3d()]
    with ps.Context() as ctx:
        tickets = [ctx.submit(o, s) for o, s in reqs]
        outs = [_np(t.wait(60.0)) for t in tickets]
        infos = [t.info() for t in tickets]
        assert all(i["state"] == "done" for i in infos)
        assert infos[-1]["n_slices"] > 1
        stats = ctx.server_stats()
        for t, i in zip(tickets, infos):                      # ps_stats while the context lives
            st = t.stats()
            assert st["t_queue"] >= 0 and st["t_e2e"] >= st["t_queue"]
            assert 0 < st["t_kernel"] <= st["t_e2e"] + 1e-3  # device time within the request's life
            assert st["t_kernel"] == i["t_kernel"]
    with ps.Context() as ctx:                                 # the 3-D job and one 2-D job alone
        alone3 = _np(ctx.submit(*reqs[-1]).wait(60.0))
        alone0 = _np(ctx.submit(*reqs[0]).wait(60.0))
    np.testing.assert_array_equal(outs[-1], alone3)
    np.testing.assert_array_equal(outs[0], alone0)
    for (o, s), got in zip(reqs, outs):
        ref = oracle.simulate(o, s)
        within(got, ref, TOL32)
    lat = [i["t_done"] - i["t_submit"] for i in infos]
    print(f"[serve] {len(reqs)} requests, iterations {stats['iterations']}, "
          f"latency p50 {np.percentile(lat, 50) * 1e3:.1f} ms max {max(lat) * 1e3:.1f} ms", flush=True)


def test_cancel_of_a_queued_request(ps):
    """With room for one request only, the second waits in the queue; cancelling
    it there drops it without running, and the first completes correctly."""
    a = C.c4_request(3)
    with ps.Context() as probe:
        t = probe.submit(*a)
        t.wait(60.0)
        need = t.info()["footprint_bytes"]
    with ps.Context(max_footprint_bytes=int(need * 1.5)) as ctx:
        t1 = ctx.submit(*a)
        t2 = ctx.submit(*a)
        t2.cancel()
        with pytest.raises(ps.PsError) as ei:
            t2.wait(60.0)
        assert ei.value.status == 6
        info2 = t2.info()
        r1 = _np(t1.wait(60.0))
    assert info2["state"] == "cancelled"
    within(r1, oracle.simulate(*a), TOL32)


def test_cancel_of_a_running_request(ps):
    """A 2 x 64^3 three-dimensional job runs as many slices; cancelled while
    running it stops at the next iteration, and the server serves on."""
    big = C.c5_request("3d", 0)
    short = C.c4_request(7)
    with ps.Context() as ctx:
        t = ctx.submit(*big)
        for _ in range(2000):
            if t.info()["state"] == "running":
                break
            time.sleep(0.001)
        t.cancel()
        with pytest.raises(ps.PsError) as ei:
            t.wait(120.0)
        assert ei.value.status == 6 and t.info()["state"] == "cancelled"
        got = _np(ctx.submit(*short).wait(60.0))
    within(got, oracle.simulate(*short), TOL32)


def test_admission_by_footprint(ps):
    a = C.c4_request(3)
    with ps.Context() as probe:
        fa = probe.submit(*a)
        fa.wait(60.0)
        need = fa.info()["footprint_bytes"]
    cap = int(need * 1.5)                                  # room for a, not for a and a second copy
    with ps.Context(max_footprint_bytes=cap) as ctx:
        t1 = ctx.submit(*a)
        t2 = ctx.submit(*a)
        r1 = _np(t1.wait(60.0))
        r2 = _np(t2.wait(60.0))
        i1, i2 = t1.info(), t2.info()
        assert i2["t_admit"] >= i1["t_done"] - 1e-6        # the second waited for memory
        np.testing.assert_array_equal(r1, r2)
        big = C.c2(256)
        with pytest.raises(ps.PsError) as ei:
            ctx.submit(*big)
        assert ei.value.status == 4                        # PS_E_TOO_LARGE
        with pytest.raises(ps.PsError) as ei:
            ctx.submit(random_spins(10, seed=1), Sequence("bad").add(float("nan"), n_adc=1))
        assert ei.value.status == 1
        t3 = ctx.submit(*a)                                # the server keeps working
        np.testing.assert_array_equal(_np(t3.wait(60.0)), r1)


def test_served_edge_requests(ps):
    with ps.Context() as ctx:
        t0 = ctx.submit(random_spins(4, seed=1).take(np.arange(0)), C.fid(1.0, 12, 1e-4))
        t1 = ctx.submit(random_spins(50, seed=2), Sequence("none").add(1e-3, alpha=1.0))
        z = _np(t0.wait(30.0))
        e = _np(t1.wait(30.0))
        t0.release()
        with pytest.raises(ps.PsError):
            t0.info()
    assert z.shape == (12,) and np.all(z == 0)
    assert e.shape == (0,)


def test_c5_stream_sample_against_the_oracle(ps):
    """The served configuration's own requests: the first 200 2-D requests
    of the c5 arrival schedule (every 16th spin) and its first 20 3-D
    2 x 64^3 sinc-GRE jobs (every 256th spin, full sequences), submitted
    together and served with continuous batching; each result within the
    FP32 bar of the oracle, a few also bitwise equal to the request alone."""
    from workloads.phantom import subset
    sched = C.c5_stream(n_requests=2000)
    two_d = [(k, p) for _, k, p in sched if k == "c4"][:200]
    three_d = [(k, p) for _, k, p in sched if k == "3d"][:20]
    reqs = []
    for k, p in two_d:
        o, s = C.c5_request(k, p)
        reqs.append((subset(o, 16, p % 16), s))
    for k, p in three_d:
        o, s = C.c5_request(k, p)
        reqs.append((subset(o, 256, p % 256), s))
    with ps.Context() as ctx:
        tickets = [ctx.submit(o, s) for o, s in reqs]
        outs = [_np(t.wait(120.0)) for t in tickets]
        stats = ctx.server_stats()
        alone = {i: _np(ctx.submit(*reqs[i]).wait(120.0)) for i in (0, 57, 199, 200, 219)}
    for i, a in alone.items():
        np.testing.assert_array_equal(outs[i], a)
    worst2, worst3 = 0.0, 0.0
    for i, ((o, s), got) in enumerate(zip(reqs, outs)):
        err = within(got, oracle.simulate(o, s), TOL32, f"c5 sample request {i}")
        if i < 200:
            worst2 = max(worst2, err)
        else:
            worst3 = max(worst3, err)
    print(f"[serve] c5 sample: 200 2-D worst rel_l2 {worst2:.3e}, 20 3-D worst {worst3:.3e}, "
          f"iterations {stats['iterations']}", flush=True)
    assert worst2 <= TOL32 and worst3 <= TOL32


def test_graph_replayed_and_direct_iterations_agree(ps):
    """The served loop replays each iteration's kernels from a HIP graph and
    launches the next short iteration before the previous completes; with
    PS_CFG_SERVE_DIRECT it launches the kernels one by one.  A mix of 60
    2-D requests and three 3-D jobs (many iterations, several launch
    topologies, graphs re-parameterised many times) gives bitwise the same
    results both ways and alone."""
    from workloads.phantom import subset
    sched = C.c5_stream(n_requests=600)
    two_d = [(k, p) for _, k, p in sched if k == "c4"][:60]
    three_d = [(k, p) for _, k, p in sched if k == "3d"][:3]
    reqs = [(subset(o, 8, p % 8), s) for (k, p) in two_d for o, s in [C.c5_request(k, p)]]
    reqs += [(subset(o, 64, p % 64), s) for (k, p) in three_d for o, s in [C.c5_request(k, p)]]
    res = {}
    for graphs in (True, False):
        with ps.Context(serve_graphs=graphs) as ctx:
            tickets = [ctx.submit(o, s) for o, s in reqs]
            res[graphs] = [_np(t.wait(120.0)) for t in tickets]
            iters = ctx.server_stats()["iterations"]
        print(f"[serve] graphs={graphs}: {len(reqs)} requests in {iters} iterations", flush=True)
    with ps.Context() as ctx:
        alone = {i: _np(ctx.submit(*reqs[i]).wait(120.0)) for i in (0, 31, 59, 60, 62)}
    for a, b in zip(res[True], res[False]):
        np.testing.assert_array_equal(a, b)
    for i, a in alone.items():
        np.testing.assert_array_equal(res[True][i], a)
    for i in (0, 59, 62):
        within(res[True][i], oracle.simulate(*reqs[i]), TOL32, f"served request {i}")
