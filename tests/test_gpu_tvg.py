"""Time-varying gain (Eq. 10) through the C ABI against the FP64 oracle on
the same complex64 echo cubes. Bounds: medians within 1e-6 relative (the GPU
selects on FP32 squared magnitudes, the oracle on FP64 ones), gains and the
conditioned echo within 2e-6 relative L2, and with alpha = 0 every corrected
median power equal to one within 1e-5.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import make_config, synthesize_echo
from tests.helpers import desc_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import paper_2101_05888_amd as m
    return m


def _median_power(e):
    p = (np.abs(e.astype(np.complex128)) ** 2).reshape(-1, e.shape[2])
    k = (p.shape[0] - 1) // 2
    return np.partition(p, k, axis=0)[k]


@pytest.mark.parametrize("case,alpha", [("c1", 0.0), ("c1", 0.3), ("c5", 0.1)])
def test_tvg_matches_oracle(api, case, alpha):
    kw = dict(n_ping=24, n_elem=6) if case == "c1" else dict(n_ping=40, n_elem=7)
    scn = make_config(case, **kw)
    echo = synthesize_echo(scn, dtype=torch.complex64)
    plan = api.sas_bp_plan([desc_for(api, scn)])
    x = echo.cuda().contiguous()
    gain = torch.zeros(scn.n_sample, dtype=torch.float32, device="cuda")
    api.sas_bp_tvg(plan, 0, x, alpha, gain)
    torch.cuda.synchronize()
    got = x.cpu().numpy()
    ref, med, G = oracle.tvg(echo.numpy().astype(np.complex128), alpha)
    g = gain.cpu().numpy()
    fin = np.isfinite(G)
    rg = np.abs(g[fin] - G[fin]).max() / np.abs(G[fin]).max()
    r = oracle.rel_l2(got, ref)
    print(f"[tvg {case} alpha={alpha}] echo rel_l2={r:.2e}, gain max rel={rg:.2e}", flush=True)
    assert r <= 2e-6 and rg <= 2e-6
    if alpha == 0.0:
        mp = _median_power(got)
        assert np.all(np.abs(mp[fin] - 1.0) <= 1e-5)


def test_tvg_ragged_and_zero_columns(api):
    # sample counts that do not fill the last 16-time group, a single element,
    # an odd population and a column of zeros (left unchanged at alpha = 0)
    scn = make_config("c1", n_ping=7, n_elem=1, n_sample=1003)
    rng = np.random.default_rng(4)
    e = (rng.normal(size=(7, 1, 1003)) + 1j * rng.normal(size=(7, 1, 1003))).astype(np.complex64)
    e[:, :, 500] = 0
    plan = api.sas_bp_plan([desc_for(api, scn)])
    x = torch.as_tensor(e, device="cuda").contiguous()
    api.sas_bp_tvg(plan, 0, x, 0.0)
    torch.cuda.synchronize()
    got = x.cpu().numpy()
    ref, med, G = oracle.tvg(e.astype(np.complex128), 0.0)
    assert np.all(got[:, :, 500] == 0)
    assert oracle.rel_l2(got, ref) <= 2e-6


@pytest.mark.parametrize("n_ping", [2047, 2049])
def test_tvg_packed_and_wide_histograms(api, n_ping):
    # 32 elements: 65504 rows take 16-bit packed histogram counts, 65568 rows the
    # 32-bit ones; the medians must be exact either way (ties and a common value
    # in one column push a count near its limit)
    E, Ns = 32, 40
    scn = make_config("c1", n_ping=n_ping, n_elem=E, n_sample=Ns)
    rng = np.random.default_rng(n_ping)
    e = (rng.normal(size=(n_ping, E, Ns)) + 1j * rng.normal(size=(n_ping, E, Ns))).astype(np.complex64)
    e[:, :, 7] = 0.5 + 0.5j                       # every key equal: one bin holds every row
    e[: n_ping // 2, :, 11] = 1.0                 # half the keys equal
    plan = api.sas_bp_plan([desc_for(api, scn)])
    x = torch.as_tensor(e, device="cuda").contiguous()
    gain = torch.zeros(Ns, dtype=torch.float32, device="cuda")
    api.sas_bp_tvg(plan, 0, x, 0.2, gain)
    torch.cuda.synchronize()
    ref, med, G = oracle.tvg(e.astype(np.complex128), 0.2)
    r = oracle.rel_l2(x.cpu().numpy(), ref)
    rg = np.abs(gain.cpu().numpy() - G).max() / np.abs(G).max()
    print(f"[tvg rows={n_ping * E}] echo rel_l2={r:.2e}, gain max rel={rg:.2e}", flush=True)
    assert r <= 2e-6 and rg <= 2e-6
