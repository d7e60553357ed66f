"""GPU: batched execution (persistent work-queue kernel) against single
requests and the FP64 oracle.  Requests keep their own tiling and time
slicing inside a batch, so each batched result must equal the single-request
result bit for bit."""
import numpy as np
import pytest

import oracle
from tests.parity import within
from workloads import Sequence, SPOIL, configs as C
from workloads.phantom import random_spins

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


@pytest.fixture(scope="module")
def ps():
    import paper_1305_6861_amd as ps
    return ps


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_c4_batch_equals_single_requests_and_oracle(ps):
    reqs = C.c4(64)
    objs = [o for o, _ in reqs]
    seqs = [s for _, s in reqs]
    with ps.Context() as ctx:
        batched = [_np(t) for t in ctx.simulate_batch(objs, seqs)]
        for i in range(0, 64, 7):
            alone = _np(ctx.simulate(objs[i], seqs[i]))
            np.testing.assert_array_equal(batched[i], alone)
    worst = 0.0
    for i in range(64):
        ref = oracle.simulate(objs[i], seqs[i])
        err = within(batched[i], ref, TOL32, f"c4 request {i}")
        worst = max(worst, err)
    print(f"[batch] c4 64 requests, worst rel_l2 {worst:.3e}", flush=True)


def test_batch_with_several_tilings_slices_and_edge_requests(ps):
    """One batch holding requests of different spins-per-lane classes, a
    request sliced into several rounds, an empty object and a request
    without samples."""
    big_obj, big_seq = C.c2()               # 262,144 spins: a different tiling class
    seqs = [big_seq.truncated(8), C.c1()[1].truncated(30), C.fid(1.0, 40, 1e-4),
            Sequence("none").add(1e-3, alpha=1.0)]
    long = Sequence("long")
    long.add(1e-3, alpha=1.0)
    long.add(3000 * 4e-6, m=(1500, 0, 0), n_adc=3000)
    long.add(1e-3, alpha=2.0, phase=1.0, n_adc=7, flags=SPOIL)
    seqs.append(long)
    objs = [big_obj, random_spins(5000, seed=1), random_spins(3, seed=2).take(np.arange(0)),
            random_spins(10, seed=3), random_spins(2000, seed=4)]
    with ps.Context(spins_per_lane=0, max_partial_bytes=64 << 10) as ctx:   # forces time slices
        batched = [_np(t) for t in ctx.simulate_batch(objs, seqs)]
        alone = [_np(ctx.simulate(o, s)) for o, s in zip(objs, seqs)]
    for b, a in zip(batched, alone):
        np.testing.assert_array_equal(b, a)
    assert batched[2].shape == (40,) and np.all(batched[2] == 0)
    assert batched[3].shape == (0,)
    for i in (1, 4):
        within(batched[i], oracle.simulate(objs[i], seqs[i]), TOL32)
    within(batched[0], oracle.simulate(objs[0], seqs[0]), TOL32)


def test_batch_rejects_a_bad_request_without_running(ps):
    good = C.c1()
    bad = Sequence("bad").add(-1.0, n_adc=2)
    with ps.Context() as ctx:
        with pytest.raises(ps.PsError) as ei:
            ctx.simulate_batch([good[0], good[0]], [good[1], bad])
    assert "request 1" in str(ei.value)
