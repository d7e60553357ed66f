"""GPU tests of the tiling autotuner (ps_tune, ps_tile_for, ps_tune_save /
ps_tune_load, PS_CFG_AUTOTUNE): the tuner times its candidates, the entry it
keeps is the tiling every entry point then uses (checked bitwise against a
context with that tiling fixed), and results stay within the FP32 bar of
the oracle."""
import numpy as np
import pytest

import oracle
from tests.parity import within
from workloads import configs as C

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


def test_tuner_times_candidates_and_the_table_is_used(ps):
    obj, seq = C.c2(64)                                     # 16,384 spins, 64 x 64 spin echo
    with ps.Context() as ctx:
        before = ctx.tile_for(obj.n_spins, seq)
        assert not before["tuned"]
        r = ctx.tune(obj, seq)
        print(f"[tune] c2[64]: {r}", flush=True)
        assert not r["from_table"]
        assert len(r["candidates"]) >= 4
        assert all(c["ms"] > 0 for c in r["candidates"])
        assert r["best_ms"] <= r["rule_ms"] + 1e-9
        chosen = ctx.tile_for(obj.n_spins, seq)
        assert chosen["tuned"] and chosen["spins_per_lane"] == r["spins_per_lane"]
        assert chosen["replicas"] == r["replicas"]
        again = ctx.tune(obj, seq)                          # the class has an entry now
        assert again["from_table"] and again["spins_per_lane"] == r["spins_per_lane"]
        got = _np(ctx.simulate(obj, seq))
    # the same tiling fixed on a context: bitwise the same signal (replicas
    # never change a result)
    with ps.Context(spins_per_lane=r["spins_per_lane"]) as fixed:
        ref_tiling = _np(fixed.simulate(obj, seq))
    np.testing.assert_array_equal(got, ref_tiling)
    within(got, oracle.simulate(obj, seq), TOL32, "c2[64] tuned tiling")


def test_loaded_table_sets_the_tiling_on_every_path(ps, tmp_path):
    """A table entry that differs from the threshold rule (S = 4 where the
    rule gives 1) is used by simulate, the batch and the served path: all
    three are bitwise the result of a context with S = 4 fixed, and not the
    rule's."""
    obj, seq = C.c2(32)                                     # 4,096 spins: the rule gives S = 1
    path = tmp_path / "table.txt"
    with ps.Context() as ctx:
        assert ctx.tile_for(obj.n_spins, seq)["spins_per_lane"] == 1
        rule = _np(ctx.simulate(obj, seq))
        ctx.tune_save(str(path))                            # header only: device tag + library hash
    header = path.read_text().splitlines()[:2]
    n_adc = max(int(n) for n in seq.n_adc)
    row = f"32 {int(np.log2(obj.n_spins))} {int(np.log2(n_adc))} 0 0 4 1 1.0 1.0"
    path.write_text("\n".join(header + [row]) + "\n")
    with ps.Context() as ctx:
        assert ctx.tune_load(str(path)) == 1
        t = ctx.tile_for(obj.n_spins, seq)
        assert t == {"spins_per_lane": 4, "replicas": "rule", "tuned": True}
        alone = _np(ctx.simulate(obj, seq))
        batch = _np(ctx.simulate_batch([obj], [seq])[0])
        served = _np(ctx.submit(obj, seq).wait(60.0))
    with ps.Context(spins_per_lane=4) as fixed:
        s4 = _np(fixed.simulate(obj, seq))
    np.testing.assert_array_equal(alone, s4)
    np.testing.assert_array_equal(batch, s4)
    np.testing.assert_array_equal(served, s4)
    assert not np.array_equal(alone, rule)                  # another summation order
    within(alone, oracle.simulate(obj, seq), TOL32, "c2[32] S=4 from the table")
    # a precision-64 context takes none of the FP32 entries
    with ps.Context(precision=64) as c64:
        assert c64.tune_load(str(path)) == 0
    # a table of another build or device is refused, and so is garbage
    bad = tmp_path / "other.txt"
    bad.write_text(header[0] + "\ngfx000 1 0000000000000000\n" + row + "\n")
    junk = tmp_path / "junk.txt"
    junk.write_text("not a table\n")
    with ps.Context() as ctx:
        for p in (bad, junk):
            with pytest.raises(ps.PsError):
                ctx.tune_load(str(p))
        assert not ctx.tile_for(obj.n_spins, seq)["tuned"]


def test_autotune_on_first_use(ps):
    """PS_CFG_AUTOTUNE: the first call of a class tunes it; later calls and a
    batch of the same requests reuse the entry (bitwise equal results)."""
    reqs = [C.c4_request(r) for r in (0, 3, 5)]
    with ps.Context(autotune=True) as ctx:
        for o, s in reqs:
            assert not ctx.tile_for(o.n_spins, s)["tuned"]
        first = [_np(ctx.simulate(o, s)) for o, s in reqs]
        for o, s in reqs:
            assert ctx.tile_for(o.n_spins, s)["tuned"]
        second = [_np(ctx.simulate(o, s)) for o, s in reqs]
        batch = [_np(x) for x in ctx.simulate_batch([o for o, _ in reqs], [s for _, s in reqs])]
    for (o, s), a, b, c in zip(reqs, first, second, batch):
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(a, c)
        within(a, oracle.simulate(o, s), TOL32, f"autotuned {o.n_spins} spins")


def test_tuner_rejects_what_it_cannot_tune(ps):
    obj, seq = C.c2(16)
    with ps.Context(spins_per_lane=2) as ctx:
        with pytest.raises(ps.PsError):
            ctx.tune(obj, seq)
