"""C-ABI checks that need no GPU: the library loads, exports every function
include/parspin.h declares, validates sequences and counts samples/steps,
and refuses to create a context without a gfx950 device."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from tests.conftest import gpu_available
from workloads import Sequence, Shape, SPOIL, configs as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ps_\w+)\s*\(", text, flags=re.M)
    return names


def test_header_declares_the_api():
    names = _declared_functions()
    for n in ["ps_create", "ps_destroy", "ps_last_error", "ps_count", "ps_simulate", "ps_config_default"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1305_6861_amd import _binding as b
    lib = ctypes.CDLL(b.LIB_PATH)
    for n in _declared_functions():
        assert hasattr(lib, n), n
        assert n in b.SIGNATURES, f"binding lacks {n}"


def test_count_matches_generators():
    import paper_1305_6861_amd as ps
    for make in (C.c1, lambda: C.c2(32)):
        _, seq = make()
        assert ps.count(seq) == (seq.n_samples, seq.n_steps_per_spin)
    seq = C.gre_3d_sinc(16, 3, 2)
    assert ps.count(seq) == (seq.n_samples, seq.n_steps_per_spin)
    assert ps.count(Sequence("empty")) == (0, 0)


@pytest.mark.parametrize("bad", ["neg_dt", "nan_dt", "inf_m", "nan_alpha", "shape_idx", "flags"])
def test_count_rejects_invalid_sequences(bad):
    import paper_1305_6861_amd as ps
    seq = Sequence("bad")
    kw = dict(dt=1e-3, m=(1, 2, 3), alpha=0.3, n_adc=4)
    if bad == "neg_dt": kw["dt"] = -1e-3
    if bad == "nan_dt": kw["dt"] = float("nan")
    if bad == "inf_m": kw["m"] = (1, math.inf, 0)
    if bad == "nan_alpha": kw["alpha"] = float("nan")
    if bad == "shape_idx": kw["shape"] = 0
    if bad == "flags": kw["flags"] = 8 | 2
    seq.add(**kw)
    with pytest.raises(ps.PsError) as ei:
        ps.count(seq)
    assert ei.value.status == 1
    assert str(ei.value)


def test_count_rejects_bad_shapes():
    import paper_1305_6861_amd as ps
    seq = Sequence("bad_shape")
    sid = seq.add_shape(Shape(tau=-1.0, m_sub=(0, 0, 0), alpha=np.ones(3), phase=np.zeros(3)))
    seq.add(1e-3, shape=sid, n_adc=1)
    with pytest.raises(ps.PsError):
        ps.count(seq)


@pytest.mark.skipif(gpu_available(), reason="checks the no-device path")
def test_create_without_device_fails_cleanly():
    import paper_1305_6861_amd as ps
    with pytest.raises(ps.PsError) as ei:
        ps.Context()
    assert ei.value.status in (3, 7)
