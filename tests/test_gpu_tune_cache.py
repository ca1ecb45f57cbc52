"""The tuning cache shared between processes: this process times the tiling
candidates with sas_bp_autotune and stores the choice in a cache file; a
second process then makes a CACHED plan that takes that tiling without timing
anything, and its sas_bp_autotune returns the stored choice with zero time.
"""
import json
import os
import subprocess
import sys

import pytest
import torch

from synth import make_config, synthesize_echo
from tests.helpers import buffers_for, desc_for

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCENE = dict(n_ping=32, n_elem=8, nx=300, ny=200, n_sample=4096, n_scat=20, n_speckle=100)

CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import torch
import paper_2101_05888_amd as api
from synth import make_config, synthesize_echo
from tests.helpers import buffers_for, desc_for
scn = make_config("c2", **json.loads(sys.argv[3]))
echo = synthesize_echo(scn, dtype=torch.complex64)
d = desc_for(api, scn)
plan = api.sas_bp_plan([d], tune_mode="cached", tune_cache=sys.argv[2])
info = plan.info()
tuned = api.sas_bp_autotune([d], [buffers_for(api, scn, echo)], reps=1, tune_mode="cached", tune_cache=sys.argv[2])
print(json.dumps({"info": info, "ms": tuned["ms"], "tile": list(tuned["tile"]), "threads": tuned["threads"],
                  "pings_per_chunk": tuned["pings_per_chunk"], "elems_per_chunk": tuned["elems_per_chunk"]}))
"""


def test_second_process_reuses_the_cached_tiling(tmp_path):
    import paper_2101_05888_amd as api
    path = str(tmp_path / "tune.json")
    scn = make_config("c2", **SCENE)
    echo = synthesize_echo(scn, dtype=torch.complex64)
    d = desc_for(api, scn)
    best = api.sas_bp_autotune([d], [buffers_for(api, scn, echo)], reps=1, tune_mode="search", tune_cache=path)
    assert best["ms"] > 0
    doc = json.load(open(path))
    assert len(doc["entries"]) == 1 and doc["entries"][0]["class"].split("|")[0].startswith("gfx")
    ref = api.sas_bp_plan([d], tile=best["tile"], threads=best["threads"], pings_per_chunk=best["pings_per_chunk"],
                          elems_per_chunk=best["elems_per_chunk"]).info()
    print(f"tuned {best}", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, path, json.dumps(SCENE)], capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    print(r.stderr[-2000:], flush=True)
    assert r.returncode == 0
    child = json.loads(r.stdout.strip().splitlines()[-1])
    print(f"second process: {child}", flush=True)
    assert child["ms"] == 0.0
    assert child["info"] == ref
    assert (tuple(child["tile"]), child["threads"], child["pings_per_chunk"], child["elems_per_chunk"]) == (
        tuple(best["tile"]), best["threads"], best["pings_per_chunk"], best["elems_per_chunk"])
