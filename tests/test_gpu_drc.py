"""Dynamic range compression (Eqs. 11-12) through the C ABI against the FP64
oracle on the same complex64 images. Bounds: output pixels within 1e-5
(outputs lie in [0, 1]; FP32 magnitudes and map), max |I| and the normalised
median within 1e-6 relative, and the output median equal to the requested
brightness within 1e-5.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import make_config, synthesize_echo
from tests.helpers import gpu_image

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import paper_2101_05888_amd as m
    return m


@pytest.fixture(scope="module")
def plan(api):
    scn = make_config("c1", n_ping=8, n_elem=4, nx=48, ny=40)
    from tests.helpers import desc_for
    return api.sas_bp_plan([desc_for(api, scn)])


def _run(api, plan, img, b):
    x = torch.as_tensor(img, dtype=torch.complex64, device="cuda").contiguous()
    out = torch.full(x.shape, -1.0, dtype=torch.float32, device="cuda")
    prm = torch.zeros(3, dtype=torch.float64, device="cuda")
    api.sas_bp_drc(plan, x, b, out, prm)
    torch.cuda.synchronize()
    return out.cpu().numpy(), prm.cpu().numpy()


def _check(got, prm, img64, b, label):
    ref, rp = oracle.drc(img64, b)
    err = np.abs(got - ref).max()
    print(f"[{label}] max |out - oracle| = {err:.2e}, median {prm[1]:.6e} vs {rp['median']:.6e}, "
          f"q {prm[2]:.6e} vs {rp['q']:.6e}", flush=True)
    assert err <= 1e-5
    assert abs(prm[0] - rp["max"]) <= 1e-6 * rp["max"]
    assert abs(prm[1] - rp["median"]) <= 1e-6 * max(rp["median"], 1e-30)
    k = (got.size - 1) // 2
    assert abs(np.partition(got.ravel(), k)[k] - b) <= 1e-5


def test_drc_of_a_backprojected_image(api, plan):
    scn = make_config("c2", n_ping=32, n_elem=8, nx=200, ny=96, n_sample=4096, n_scat=30, n_speckle=300)
    echo = synthesize_echo(scn, dtype=torch.complex64)
    img, p2, _ = gpu_image(api, scn, echo)
    got, prm = _run(api, p2, img, 0.3)
    _check(got, prm, img.astype(np.complex64).astype(np.complex128), 0.3, "bp-image")


@pytest.mark.parametrize("n,b", [(1, 0.5), (2, 0.5), (1000, 0.25), (100001, 0.6), (1 << 20, 0.4)])
def test_drc_random_images(api, plan, n, b):
    rng = np.random.default_rng(n)
    mag = rng.rayleigh(1.0, n) * 10 ** rng.uniform(-3, 1, n)
    img = (mag * np.exp(1j * rng.uniform(0, 2 * np.pi, n))).astype(np.complex64)
    got, prm = _run(api, plan, img, b)
    if n <= 2:
        ref, rp = oracle.drc(img.astype(np.complex128), b)
        assert np.abs(got - ref).max() <= 1e-6
        return
    _check(got, prm, img.astype(np.complex128), b, f"random-{n}")


def test_drc_degenerate_images(api, plan):
    got, prm = _run(api, plan, np.zeros(1000, dtype=np.complex64), 0.5)
    assert np.all(got == 0) and prm[2] == 1.0
    img = np.zeros(1001, dtype=np.complex64)
    img[:300] = np.arange(1, 301)
    got, prm = _run(api, plan, img, 0.5)                 # median 0: non-zero pixels to 1
    assert np.isinf(prm[2]) and np.all(got[:300] == 1) and np.all(got[300:] == 0)
