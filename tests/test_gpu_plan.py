"""GPU: compiled plans replayed from a HIP graph (ps_plan_create / launch).

Each test replays a plan several times with ordinary eager GPU work and
host synchronisations in between, and checks every replay: bitwise equal
to ps_simulate / ps_simulate_rx on the same context and within the FP32 bar
of the oracle; rewriting the captured object arrays in place changes the
next replay's result exactly as a fresh simulation would."""
import numpy as np
import pytest

import oracle
from tests.parity import within
from workloads import Sequence, coils, configs as C
from workloads.phantom import random_spins

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


@pytest.fixture(scope="module")
def ps():
    import paper_1305_6861_amd as ps
    return ps


def _eager_noise():
    import torch
    a = torch.randn(256, 256, device="cuda")
    (a @ a).sum().item()                      # unrelated work + a host sync


def test_replays_equal_simulate_bitwise(ps):
    import torch
    obj, seq = C.c2(32)
    ref = oracle.simulate(obj, seq)
    with ps.Context() as ctx:
        want = ctx.simulate(obj, seq).cpu().numpy()
        with ctx.plan(obj, seq) as plan:
            for _ in range(4):
                got = plan.launch().cpu().numpy()
                np.testing.assert_array_equal(got, want)
                _eager_noise()
    within(want, ref, TOL32)


def test_in_place_parameter_updates_between_replays(ps):
    import torch
    obj, seq = C.c2(24)
    with ps.Context() as ctx:
        dev = ps.to_device(obj)
        plan = ctx.plan(dev, seq)
        s1 = plan.launch().cpu().numpy()
        dev["m0"].mul_(2.0)                                   # exact in FP32
        s2 = plan.launch().cpu().numpy()
        np.testing.assert_array_equal(s2, 2.0 * s1)
        _eager_noise()
        new_t2 = np.asarray(obj.t2, np.float32) * np.float32(0.5)
        dev["t2"].copy_(torch.from_numpy(new_t2).cuda())
        s3 = plan.launch().cpu().numpy()
        obj2 = obj.take(np.arange(obj.n_spins))
        obj2.t2 = new_t2
        obj2.m0 = np.asarray(obj.m0, np.float32) * np.float32(2.0)
        np.testing.assert_array_equal(s3, ctx.simulate(obj2, seq).cpu().numpy())
        within(s3, oracle.simulate(obj2, seq), TOL32)
        plan.close()


def test_plan_with_coils_shapes_and_time_slices(ps):
    obj, _ = C.c3(10)
    seq = C.gre_3d_sinc(10, 3, 3)
    rx = coils.loop_ring(obj, 2, ring_radius=0.2, coil_radius=0.06)
    # 2000 spins at S = 1: 8 workgroups x 1 row; 2 coils; 64 samples per slice
    with ps.Context(spins_per_lane=1, max_partial_bytes=8 * 2 * 4 * 2 * 64) as ctx:
        want = ctx.simulate(obj, seq, coils=rx).cpu().numpy()
        with ctx.plan(obj, seq, coils=rx) as plan:
            for _ in range(3):
                got = plan.launch().cpu().numpy()
                np.testing.assert_array_equal(got, want)
                _eager_noise()
    ref = oracle.simulate(obj, seq, coils=rx)
    for c in range(2):
        within(want[c], ref[c], TOL32)


def test_degenerate_plans(ps):
    import torch
    empty = random_spins(3, seed=1).take(np.arange(0))
    with ps.Context() as ctx:
        with ctx.plan(empty, C.fid(1.0, 8, 1e-4)) as plan:
            plan.out.fill_(7.0)
            z = plan.launch().cpu().numpy()
            assert z.shape == (8,) and np.all(z == 0)
        with ctx.plan(random_spins(40, seed=2), Sequence("none").add(1e-3, alpha=1.0)) as plan:
            assert plan.launch().cpu().numpy().shape == (0,)
        torch.cuda.synchronize()
