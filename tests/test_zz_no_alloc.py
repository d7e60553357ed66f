"""The allocation-free entry point (ps_simulate_noalloc, through the C ABI)
against ps_simulate on the same context: two calls in a row, the second with
a smaller request, bitwise equal where the request fits the static scratch
with the context's own time slicing; a request that needs shorter slices
there within the FP32 bar of ps_simulate and of the oracle; a request too
large for the scratch refused with nothing launched."""
import numpy as np
import pytest

import oracle
from tests.parity import within
from workloads import configs as C
from workloads.phantom import random_spins, subset

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def _run(ps, ctx, obj, seq):
    import torch
    dev = ps.to_device(obj)
    n_samples, _ = ps.count(seq)
    out = torch.empty(2 * n_samples, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    got = ps.simulate_noalloc(ctx, dev, seq, out)
    ref = ctx.simulate(dev, seq)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


def test_two_calls_in_a_row_the_second_smaller():
    import paper_1305_6861_amd as ps
    with ps.Context() as ctx:
        for label, (obj, seq) in (("c2[64]", C.c2(64)), ("c2[24] ragged", C.c2(24))):
            print(f"[noalloc] {label}: {obj.n_spins} spins, {seq.n_samples} samples", flush=True)
            got, ref = _run(ps, ctx, obj, seq)
            np.testing.assert_array_equal(got, ref)
            within(got, oracle.simulate(obj, seq), TOL32, f"noalloc {label}")
        # a 3-D shaped-pulse request with the propagator cache, then a smaller 2-D one
        obj, _ = C.c3(16)
        seq = C.gre_3d_sinc(16, 4, 3)
        got, ref = _run(ps, ctx, obj, seq)
        np.testing.assert_array_equal(got, ref)
        within(got, oracle.simulate(obj, seq), TOL32, "noalloc c3[16]")
        obj, seq = C.c1()
        got, ref = _run(ps, ctx, obj, seq)
        np.testing.assert_array_equal(got, ref)


def test_request_sliced_to_fit_the_scratch():
    """The full 256^2 x 4 spin echo: its 268 MB of partial rows exceed the
    256 MiB scratch, so it runs in shorter time slices than ps_simulate."""
    import paper_1305_6861_amd as ps
    obj, seq = C.c2()
    with ps.Context() as ctx:
        print(f"[noalloc] c2 full: {obj.n_spins} spins, {seq.n_samples} samples", flush=True)
        got, ref = _run(ps, ctx, obj, seq)
        within(got, ref, TOL32, "noalloc c2 full vs ps_simulate")
        sub = subset(obj, 64)
        got_s, _ = _run(ps, ctx, sub, seq)
        within(got_s, oracle.simulate(sub, seq), TOL32, "noalloc c2 subset/64 vs oracle")


def test_too_large_is_refused():
    import torch
    import paper_1305_6861_amd as ps
    obj = random_spins(1 << 24, seed=3)            # slice state alone > 256 MiB
    _, seq = C.c1()
    seq = seq.truncated(30)
    with ps.Context(max_partial_bytes=1 << 20) as ctx:
        dev = ps.to_device(obj)
        n, _ = ps.count(seq)
        out = torch.zeros(2 * n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        with pytest.raises(ps.PsError) as ei:
            ps.simulate_noalloc(ctx, dev, seq, out)
        assert ei.value.status == 4
        torch.cuda.synchronize()
        assert float(out.abs().max()) == 0.0      # nothing ran
