"""GPU parity on the four experiments of Table 7.8 (2-D turbo spin echo,
2-D radial, 2-D EPI, 3-D spin echo) with the Legendre B0 field of eq. 6.3,
at a quarter of the paper's matrix and object side, against the FP64
oracle (FP32 <= 1e-5, FP64 <= 1e-12)."""
import numpy as np
import pytest

import oracle
from tests.parity import within
from workloads import configs as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    import paper_1305_6861_amd as ps
    return ps


@pytest.mark.parametrize("kind", C.TABLE78)
def test_table78_reduced(ps, kind):
    import torch
    obj, seq = C.table78(kind, scale=4)
    ref = oracle.simulate(obj, seq)
    for prec, tol in ((32, 1e-5), (64, 1e-12)):
        with ps.Context(precision=prec) as ctx:
            got = ctx.simulate(obj, seq)
            torch.cuda.synchronize()
            got = got.cpu().numpy()
        within(got, ref, tol, f"t78 {kind} fp{prec} spins={obj.n_spins}")
