"""The allocation-free sharpness entry point (sas_bp_sharpness_static) through
the C ABI: S and the cotangent equal those of sas_bp_sharpness (same kernels,
same fixed summation order: bitwise) on two calls in a row, the second with a
smaller image than the first, and S matches the oracle's; sizes beyond the
stated maximum are refused before anything is enqueued.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from synth import make_config, synthesize_echo
from tests.helpers import buffers_for, desc_for

pytestmark = pytest.mark.gpu


def _image(api, **kw):
    scn = make_config("c5", **kw)
    echo = synthesize_echo(scn, dtype=torch.complex64)
    plan = api.sas_bp_plan([desc_for(api, scn)])
    buf = buffers_for(api, scn, echo)
    api.sas_bp_image(plan, [buf])
    torch.cuda.synchronize()
    return plan, buf.image


def test_static_sharpness_equals_the_plan_entry_point_twice():
    import paper_2101_05888_amd as api
    big_plan, big = _image(api, n_ping=24, n_elem=4, nx=300, ny=220, n_scat=30)
    small_plan, small = _image(api, n_ping=16, n_elem=4, nx=90, ny=40, n_scat=10)
    for plan, img in ((big_plan, big), (small_plan, small)):   # the second call is smaller
        S0 = torch.zeros(1, dtype=torch.float64, device="cuda")
        S1 = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        G0 = torch.empty_like(img)
        G1 = torch.full_like(img, complex(7.0, -7.0))
        api.sas_bp_sharpness(plan, img, S0, G0)
        api.sas_bp_sharpness_static(img, S1, G1)
        torch.cuda.synchronize()
        s0, s1 = float(S0.item()), float(S1.item())
        print(f"[no-alloc sharpness] n={img.numel()} S plan {s0:.15e} static {s1:.15e}", flush=True)
        assert s1 == s0
        assert torch.equal(G1, G0)
        assert s1 == pytest.approx(oracle.sharpness(img.cpu().numpy()), rel=1e-12)
    # S alone (no cotangent) as well
    S2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    api.sas_bp_sharpness_static(big, S2)
    torch.cuda.synchronize()
    assert float(S2.item()) == pytest.approx(oracle.sharpness(big.cpu().numpy()), rel=1e-12)


def test_static_sharpness_refuses_sizes_beyond_the_maximum():
    import paper_2101_05888_amd as api
    from paper_2101_05888_amd import _native as N
    img = torch.zeros(16, dtype=torch.complex64, device="cuda")
    S = torch.zeros(1, dtype=torch.float64, device="cuda")
    lib = N.lib()
    assert lib.sas_bp_sharpness_static(img.data_ptr(), (1 << 34) + 1, S.data_ptr(), None, None) == N.SAS_BP_EINVAL
    assert lib.sas_bp_sharpness_static(img.data_ptr(), 0, S.data_ptr(), None, None) == N.SAS_BP_EINVAL
    assert lib.sas_bp_sharpness_static(None, 16, S.data_ptr(), None, None) == N.SAS_BP_EINVAL
