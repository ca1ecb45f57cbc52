"""The echo envelope (|e|, 0) of the autofocus's incoherent stage through the
C ABI, against |e| formed in FP64 on the host and rounded to the storage
format: within |e| eps of that format (the kernel squares and adds in FP32
before its correctly rounded square root), imaginary parts exactly zero,
in place and out of place, on a ragged cube (one thread per sample, the last
workgroup partial) for every storage format.
"""
import numpy as np
import pytest
import torch

from synth import make_config, quantize_echo
from tests.helpers import desc_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import paper_2101_05888_amd as m
    return m


def _ulp_ok(got, want, dtype):
    g = torch.as_tensor(got).to(torch.float64)
    w = torch.as_tensor(want).to(dtype).to(torch.float64)
    info = torch.finfo(dtype)
    # spacing of the format at |w| (at least its smallest normal spacing)
    ulp = torch.clamp(w.abs(), min=info.tiny) * info.eps
    return bool(((g - w).abs() <= ulp * 1.0001).all())


@pytest.mark.parametrize("kind", ["c64", "f16", "bf16"])
@pytest.mark.parametrize("in_place", [False, True])
def test_envelope_matches_fp64_magnitude(api, kind, in_place):
    scn = make_config("c1", n_ping=3, n_elem=5, n_sample=333, nx=16, ny=16)
    rng = np.random.default_rng(11)
    e = (rng.normal(size=(3, 5, 333)) + 1j * rng.normal(size=(3, 5, 333))) * 10.0 ** rng.uniform(-3, 3, (3, 5, 1))
    plan = api.sas_bp_plan([desc_for(api, scn, echo_dtype=kind)])
    if kind == "c64":
        x = torch.as_tensor(e.astype(np.complex64)).cuda()
        host = x.cpu().numpy().astype(np.complex128)
        mag = np.abs(host)
        out = api.sas_bp_envelope(plan, 0, x, out=x if in_place else None)
        torch.cuda.synchronize()
        got = out.cpu()
        assert torch.all(got.imag == 0)
        assert _ulp_ok(got.real, torch.as_tensor(mag), torch.float32)
    else:
        q, scale = quantize_echo(torch.as_tensor(e), kind)
        x = q.cuda().contiguous()
        h = q.to(torch.float64).numpy()
        mag = np.sqrt(h[..., 0] ** 2 + h[..., 1] ** 2)
        out = api.sas_bp_envelope(plan, 0, x, out=x if in_place else None)
        torch.cuda.synchronize()
        got = out.cpu()
        assert torch.all(got[..., 1] == 0)
        assert _ulp_ok(got[..., 0], torch.as_tensor(mag), q.dtype)
    if not in_place:
        # the input is untouched
        assert out.data_ptr() != x.data_ptr()


def test_envelope_rejects_overlap_and_wrong_shape(api):
    scn = make_config("c1", n_ping=3, n_elem=5, n_sample=333, nx=16, ny=16)
    plan = api.sas_bp_plan([desc_for(api, scn)])
    x = torch.zeros((3, 5, 334), dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError):
        api.sas_bp_envelope(plan, 0, x)
    from paper_2101_05888_amd import _native as N
    y = torch.zeros((3 * 5 * 333 + 1,), dtype=torch.complex64, device="cuda")
    assert N.lib().sas_bp_envelope(plan.handle, 0, y.data_ptr(), y[1:].data_ptr(), None) == 1
