"""The block cull's predicates (Sec. II-C; each apex tested on its own as in
the bistatic case of Sec. III-B), evaluated on the host through the C ABI and
checked against the oracle's per-pixel gate |p_x - X_x| <= sin(a) |p - X|.

* The counterexample to the paper's corner rule: a narrow beam crosses a
  block of pixels without holding any of the block's corners. The corner rule
  drops the block; the library's class is "decided per row" and the cull
  keeps it, and the oracle finds gated-in pixels inside.
* Randomised boxes and apexes: "outside" never holds a gated-in pixel,
  "inside" never a gated-out one, and the cull pass keeps every box that holds
  a gated-in pixel.
"""
import math

import numpy as np
import pytest

import oracle

OUT, IN, PARTIAL = 0, 1, 2


@pytest.fixture(scope="module")
def api():
    import paper_2101_05888_amd as m
    return m


def _grid(lo, hi, n=(9, 9, 3)):
    axes = [np.linspace(lo[a], hi[a], n[a]) if hi[a] > lo[a] else np.array([lo[a]]) for a in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    return np.column_stack([X.ravel(), Y.ravel(), Z.ravel()])


def _inside(apex, pts, half_angle):
    """The oracle's gate for every point, one apex as transmitter and receiver."""
    tx = np.asarray(apex, dtype=np.float64)[None, :]
    rx = tx[:, None, :]
    return np.array([oracle.gated_term_count(tx, rx, p[None, :], half_angle) for p in pts], dtype=bool)


def test_narrow_beam_through_a_block_without_corners(api):
    apex = (0.0, 0.0, -10.0)
    half = math.radians(1.0)                  # cone half-width 0.35 m at 20 m, the block is 1 m wide
    lo, hi = (-0.5, 20.0, 0.0), (0.5, 21.0, 0.0)
    corners = np.array([[x, y, 0.0] for x in (lo[0], hi[0]) for y in (lo[1], hi[1])])
    assert not _inside(apex, corners, half).any()          # the corner rule would discard the block
    inner = _grid(lo, hi, (41, 5, 1))
    assert _inside(apex, inner, half).any()                # yet the beam crosses it
    cls, hit = api.sas_bp_gate_class(apex, lo, hi, half)
    assert cls == PARTIAL and hit == 1
    # the same block shifted clear of the beam is outside; a block inside the
    # beam's core is inside
    assert api.sas_bp_gate_class(apex, (1.0, 20.0, 0.0), (2.0, 21.0, 0.0), half) == (OUT, 0)
    assert api.sas_bp_gate_class(apex, (-0.1, 20.0, 0.0), (0.1, 21.0, 0.0), half)[0] == IN


def test_random_boxes_against_the_per_pixel_gate(api):
    rng = np.random.default_rng(20250)
    counts = {OUT: 0, IN: 0, PARTIAL: 0}
    for _ in range(300):
        half = math.radians(rng.uniform(2.0, 30.0))
        apex = rng.normal(0.0, 2.0, 3) + np.array([0.0, 0.0, -10.0])
        c = np.array([rng.uniform(-8, 8), rng.uniform(5, 40), rng.uniform(-1, 3)])
        ext = np.array([rng.uniform(0.05, 2.0), rng.uniform(0.05, 2.0), rng.choice([0.0, rng.uniform(0.05, 0.5)])])
        lo, hi = c - ext / 2, c + ext / 2
        cls, hit = api.sas_bp_gate_class(apex, lo, hi, half)
        g = _inside(apex, _grid(lo, hi), half)
        counts[cls] += 1
        if cls == OUT:
            assert not g.any()
        if cls == IN:
            assert g.all()
        if g.any():
            assert hit == 1
        if hit == 0:
            assert cls == OUT
    # every class occurs
    assert min(counts.values()) > 10, counts


def test_bad_arguments(api):
    with pytest.raises(api.SasBpError):
        api.sas_bp_gate_class((0, 0, 0), (1, 0, 0), (0, 1, 1), 0.1)     # lo > hi
    with pytest.raises(api.SasBpError):
        api.sas_bp_gate_class((0, 0, 0), (0, 0, 0), (1, 1, 1), 0.0)
    with pytest.raises(api.SasBpError):
        api.sas_bp_gate_class((0, 0, math.nan), (0, 0, 0), (1, 1, 1), 0.1)
