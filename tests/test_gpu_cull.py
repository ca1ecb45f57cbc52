"""The block cull is exact: with it turned off (every ping of every tile
visited, every (ping, element) gated pixel row by pixel row) the images and
the geometry gradients are bitwise the same as with it on, on gated scenes
whose tiles straddle the beam edges, and the useful-update count is unchanged.
"""
import numpy as np
import pytest
import torch

from synth import make_config, synthesize_echo
from tests.helpers import buffers_for, desc_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import paper_2101_05888_amd as m
    return m


SCENES = {
    # gated operational geometry, scaled, ragged edges; narrow tiles and wide ones
    "c2_small": ("c2", dict(n_ping=64, n_elem=8, nx=333, ny=129, n_sample=4096, n_scat=40, n_speckle=400)),
    # a narrow 3 degree beam: most tiles are crossed by a cone edge
    "c2_narrow": ("c2", dict(n_ping=48, n_elem=6, nx=260, ny=96, n_sample=4096, n_scat=30, n_speckle=200,
                             gate_deg=3.0)),
    # a gated batch swath whose far rows lie beyond the end of the record
    "c4b": ("c4b:3", dict(nx=150, ny=1400, n_ping=60, n_elem=9, n_scat=20, n_sample=4096)),
}


def _image(api, scn, echo, **kw):
    plan = api.sas_bp_plan([desc_for(api, scn)], **kw)
    buf = buffers_for(api, scn, echo)
    api.sas_bp_image(plan, [buf])
    torch.cuda.synchronize()
    assert plan.status() == 0
    count = api.sas_bp_useful_updates(plan, [buf])[0]
    return plan, buf, buf.image.cpu().numpy(), count


@pytest.mark.parametrize("tile", [(0, 0, 0), (64, 0, 0)])
@pytest.mark.parametrize("scene", sorted(SCENES))
def test_culled_equals_unculled_bitwise(api, scene, tile):
    name, kw = SCENES[scene]
    print(f"case {scene} tile {tile}", flush=True)
    scn = make_config(name, **kw)
    echo = synthesize_echo(scn, dtype=torch.complex64)
    _, _, a, na = _image(api, scn, echo, tile=tile)
    plan_u, _, b, nb = _image(api, scn, echo, tile=tile, no_cull=True)
    assert np.abs(a).max() > 0
    assert np.array_equal(a, b)          # value equality, element by element
    assert na == nb


def test_culled_equals_unculled_adjoint_bitwise(api):
    name, kw = SCENES["c2_small"]
    scn = make_config(name, **kw)
    echo = synthesize_echo(scn, dtype=torch.complex64)
    g = scn.grid
    rng = np.random.default_rng(7)
    gbar = torch.as_tensor((rng.normal(size=(g.n[2], g.n[1], g.n[0]))
                            + 1j * rng.normal(size=(g.n[2], g.n[1], g.n[0]))).astype(np.complex64), device="cuda")
    out = []
    for no_cull in (False, True):
        plan = api.sas_bp_plan([desc_for(api, scn)], no_cull=no_cull)
        buf = buffers_for(api, scn, echo)
        gtx = torch.zeros((scn.n_ping, 3), dtype=torch.float64, device="cuda")
        grx = torch.zeros((scn.n_ping, scn.n_elem, 3), dtype=torch.float64, device="cuda")
        gc = torch.zeros(1, dtype=torch.float64, device="cuda")
        api.sas_bp_adjoint(plan, [buf], [gbar], [gtx], [grx], [gc])
        torch.cuda.synchronize()
        assert plan.status() == 0
        out.append((gtx.cpu().numpy(), grx.cpu().numpy(), gc.cpu().numpy()))
    assert np.abs(out[0][0]).max() > 0
    for x, y in zip(out[0], out[1]):
        assert np.array_equal(x, y)
