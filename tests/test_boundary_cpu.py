"""The C-ABI library on a host without a GPU: it loads, exports every symbol
the header declares, and rejects bad arguments before touching a device."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sas_bp.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(sas_bp_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2101_05888_amd import _native as N
    names = _declared()
    assert "sas_bp_plan" in names and "sas_bp_image" in names and "sas_bp_adjoint" in names
    for n in names:
        assert hasattr(N.lib(), n), n
    assert set(N.EXPORTED) == set(names)


def test_abi_version_and_error_strings():
    from paper_2101_05888_amd import _native as N
    assert N.lib().sas_bp_abi_version() == 6
    for s in range(7):
        assert N.lib().sas_bp_error_string(s) != b"unknown status"
    assert N.lib().sas_bp_error_string(99) == b"unknown status"


def _desc(api, **kw):
    base = dict(n_ping=64, n_elem=8, n_sample=4096, n=(256, 256, 1), origin=(2.8, 20.0, 0.0),
                spacing=(0.015, 0.015, 0.015), f_c=100e3, f_s=80e3)
    base.update(kw)
    return api.swath_desc(**base)


@pytest.mark.parametrize("bad,status", [
    (dict(n_ping=0), 1), (dict(n_elem=0), 1), (dict(n_elem=300), 1), (dict(n_sample=1), 1),
    (dict(n=(0, 5, 1)), 1), (dict(spacing=(0.0, 0.015, 0.015)), 1), (dict(f_s=0.0), 1),
    (dict(f_s=math.nan), 1), (dict(f_c=-1.0), 1), (dict(t0=math.inf), 1),
    (dict(gate_half_angle=2.0), 1), (dict(gate_half_angle=-0.1), 1), (dict(c_min=-1.0), 1),
    (dict(origin=(math.nan, 0.0, 0.0)), 1), (dict(n=(4096, 4096, 2048)), 2),
])
def test_host_validation(bad, status):
    import paper_2101_05888_amd as api
    with pytest.raises(api.SasBpError) as ei:
        api.sas_bp_workspace_size([_desc(api, **bad)])
    assert ei.value.status == status


def test_bad_dtype_and_tile_are_unsupported():
    import paper_2101_05888_amd as api
    d = _desc(api)
    d.echo_dtype = 7
    with pytest.raises(api.SasBpError) as ei:
        api.sas_bp_workspace_size([d])
    assert ei.value.status == 2
    with pytest.raises(api.SasBpError) as ei:
        api.sas_bp_workspace_size([_desc(api)], tile=(24, 0, 0))
    assert ei.value.status == 2


def test_workspace_size_scales_with_tiles():
    import paper_2101_05888_amd as api
    a = api.sas_bp_workspace_size([_desc(api)])
    b = api.sas_bp_workspace_size([_desc(api, n=(2048, 2048, 1))])
    assert 0 < a < b


def test_plan_without_device_reports_device_error():
    import torch
    import paper_2101_05888_amd as api
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(api.SasBpError) as ei:
        api.sas_bp_plan([_desc(api)])
    assert ei.value.status == 4


def test_null_arguments_rejected():
    from paper_2101_05888_amd import _native as N
    assert N.lib().sas_bp_plan(None, 1, None, None) == 1
    assert N.lib().sas_bp_image(None, None, 1, None) == 1
    assert N.lib().sas_bp_plan_status(None) == 1
    assert N.lib().sas_bp_reproject(None, None, None, None, 1, None) == 1
    assert N.lib().sas_bp_drc(None, None, 1, 0.5, None, None, None) == 1
    assert N.lib().sas_bp_tvg(None, 0, None, 0.0, None, None) == 1
    assert N.lib().sas_bp_envelope(None, 0, None, None, None) == 1
    assert N.lib().sas_bp_whiten(None, 0, None, 0.0, None) == 1
    assert N.lib().sas_bp_range_compress(None, 0, None, None, 1, 1, None) == 1
    assert N.lib().sas_bp_dpc_tde(None, 0, None, None, 1, 2, 1, 1, None, None) == 1
    assert N.lib().sas_bp_dpc_footprints(None, None, None, None, None, None, 0.0, 1.0, None) == 1
    assert N.lib().sas_bp_dpc_residual(None, None, None, None, None, None, None, None, None, None, None) == 1
    assert N.lib().sas_bp_dpc_fine_delay(None, None, 1, 1e5, None, None) == 1
    assert N.lib().sas_bp_dpc_solve(None, None, None, None, None, None, None, None, None, None, None, None, 0) == 1
    assert N.lib().sas_bp_adjoint(None, None, None, None, None, None, 1, None) == 1
    out = C.c_size_t()
    assert N.lib().sas_bp_workspace_size(None, 1, None, C.byref(out)) == 1


def test_product_path_has_no_oracle_or_cpu_fallback():
    # the package must not import the oracle or the input generator
    pkg = os.path.join(ROOT, "paper_2101_05888_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "import oracle" not in src and "from oracle" not in src, fn
            assert "import synth" not in src and "from synth" not in src, fn


def test_option_fields_are_checked_on_the_host():
    import paper_2101_05888_amd as api
    from paper_2101_05888_amd import _native as N
    arr = (N.SwathDesc * 1)(_desc(api))
    out = C.c_size_t()
    for field, value in (("tune_mode", 3), ("tune_mode", -1), ("no_cull", 2)):
        o = api.api._options()
        setattr(o, field, value)
        assert N.lib().sas_bp_workspace_size(arr, 1, C.byref(o), C.byref(out)) == N.SAS_BP_EINVAL, field
    # no_cull changes nothing in the sizing
    assert api.sas_bp_workspace_size([_desc(api)], no_cull=True) == api.sas_bp_workspace_size([_desc(api)])


def test_cached_tiling_is_read_from_the_tune_file(tmp_path):
    # On a host without a device the architecture in the shape class reads
    # "unknown". A stored 32 x 32 tiling for this class replaces the automatic
    # choice (16 x 32 for a 256 x 256 image) in a CACHED plan's sizing; a
    # DEFAULT plan ignores it, and an unreadable or missing file counts as empty.
    import paper_2101_05888_amd as api
    d = _desc(api)
    path = tmp_path / "tune.json"
    # class: arch, 2D, FP32 echo, linear, stop-and-hop, straight paths, no
    # gate, 8 elements (bucket 3), 65536 pixels (bucket 16); the window-length
    # bucket depends on the automatic tile, so every bucket is stored
    rows = ['  {"class": "unknown|2d|c64|interp0|motion0|refract0|nogate|e3|w%d|p16", "tile_x": 32, '
            '"tile_y": 32, "tile_z": 1, "threads": 256, "pings_per_chunk": 2, "elems_per_chunk": 0, "ms": 1.5}' % w
            for w in range(14)]
    path.write_text('{"format": "sas_bp tuning cache", "version": 1, "entries": [\n' + ",\n".join(rows) + "\n]}\n")
    auto = api.sas_bp_workspace_size([d])
    tiled = api.sas_bp_workspace_size([d], tile=(32, 32, 1), threads=256, pings_per_chunk=2)
    assert auto != tiled
    # (first: a stored choice, once read, stays in the process cache)
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    assert api.sas_bp_workspace_size([d], tune_mode="cached", tune_cache=str(bad)) == auto
    assert api.sas_bp_workspace_size([d], tune_mode="cached", tune_cache=str(tmp_path / "none.json")) == auto
    assert api.sas_bp_workspace_size([d], tune_mode="cached", tune_cache=str(path)) == tiled
    assert api.sas_bp_workspace_size([d], tune_mode="search", tune_cache=str(path)) == tiled
    assert api.sas_bp_workspace_size([d], tune_mode="default", tune_cache=str(path)) == auto
    # another class (a gated swath) finds nothing and keeps the automatic tiling
    g = _desc(api, gate_half_angle=0.17)
    assert api.sas_bp_workspace_size([g], tune_mode="cached", tune_cache=str(path)) == api.sas_bp_workspace_size([g])
