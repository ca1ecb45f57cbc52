"""The batched workload at full size: 24 swaths of uneven size (sides drawn
from 512 to 4096 pixels, 128 to 512 pings, 16 to 32 receivers, +-10 deg
gate) imaged in one persistent launch, as the benchmark runs them. Each
swath's image is compared with the FP64 oracle on a seeded 4096-pixel subset
and, bitwise, with the same swath imaged alone by its own plan.
"""
import numpy as np
import pytest
import torch

from synth import make_config, subset_indices, synthesize_echo
from tests.helpers import FP32_PHASE_MRAD, FP32_REL_L2, buffers_for, desc_for, oracle_image, report

pytestmark = pytest.mark.gpu

N_SWATHS = 24
SUBSET = 4096


@pytest.fixture(scope="module")
def batch():
    import paper_2101_05888_amd as api
    print("case c4b: 24 swaths in one launch", flush=True)
    scns = [make_config(f"c4b:{k}") for k in range(N_SWATHS)]
    echoes = [synthesize_echo(s, device="cuda", dtype=torch.complex64, noise_on_device=True) for s in scns]
    plan = api.sas_bp_plan([desc_for(api, s) for s in scns])
    bufs = [buffers_for(api, s, e) for s, e in zip(scns, echoes)]
    api.sas_bp_image(plan, bufs)
    torch.cuda.synchronize()
    assert plan.status() == 0
    out = []
    for s, e, b in zip(scns, echoes, bufs):
        idx = subset_indices(s, SUBSET)
        sub = b.image.reshape(-1)[torch.as_tensor(idx, device="cuda")].cpu().numpy()
        alone = api.sas_bp_plan([desc_for(api, s)])
        b2 = buffers_for(api, s, e)
        api.sas_bp_image(alone, [b2])
        torch.cuda.synchronize()
        same = bool(torch.equal(b2.image, b.image))
        alone.destroy()
        del b2
        out.append((s, idx, sub, same))
    del bufs
    yield api, scns, echoes, out
    plan.destroy()
    del echoes
    torch.cuda.empty_cache()


@pytest.mark.parametrize("k", range(N_SWATHS))
def test_batched_swath_matches_oracle_and_its_own_plan(batch, k):
    api, scns, echoes, out = batch
    s, idx, sub, same = out[k]
    print(f"case c4b:{k} {s.grid.n[0]}x{s.grid.n[1]} px, {s.n_ping} pings x {s.n_elem} rx", flush=True)
    assert same
    ref = oracle_image(s, echoes[k].cpu().numpy(), idx)
    r, ph = report(f"c4b:{k}", sub, ref)
    assert np.abs(ref).max() > 0
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD
