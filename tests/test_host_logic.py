"""Host-side logic that needs no GPU: autotuner shape space and cache file,
the locality order helper, workload sizes of the mixed batch."""
import ctypes as C
import json

import numpy as np

from paper_2205_03532_amd import autotune, fc
from paper_2205_03532_amd import workloads as W


def test_candidate_shapes_are_all_valid_for_the_library():
    L = fc.lib()
    shapes = autotune.candidate_shapes()
    assert len(shapes) == len({json.dumps(s, sort_keys=True) for s in shapes})
    assert autotune.DEFAULT in shapes
    # every shape passes the library's own launch validation (via the cache parser)
    import tempfile, os
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "t.json")
        autotune.save([dict(s, key=f"k{i}", ms=1.0) for i, s in enumerate(shapes)], p)
        assert L.fc_autotune_load(p.encode()) == len(shapes)


def test_cache_save_merges_by_key(tmp_path):
    p = str(tmp_path / "c.json")
    autotune.save([dict(autotune.DEFAULT, key="a", ms=2.0)], p)
    autotune.save([dict(autotune.DEFAULT, key="b", ms=1.0), dict(autotune.DEFAULT, key="a", ms=0.5)], p)
    e = json.load(open(p))["entries"]
    assert sorted(x["key"] for x in e) == ["a", "b"]
    assert [x["ms"] for x in e if x["key"] == "a"] == [0.5]


def test_locality_order_is_a_permutation_grouped_by_type():
    rng = np.random.default_rng(0)
    n = 500
    pose = np.zeros((7, n), np.float32)
    pose[3] = 1
    pose[4:7] = rng.uniform(-1, 1, (3, n))
    typ = rng.integers(0, 3, n).astype(np.int32)

    class Wl:
        pass

    wl = Wl()
    wl.pose, wl.env_mesh, wl.env_grid = pose, typ, typ
    o = fc.locality_order(wl)
    assert sorted(o.tolist()) == list(range(n))
    assert np.all(np.diff(typ[o]) >= 0)
    # spatially coherent: consecutive envs are much closer than random pairs
    d_seq = np.linalg.norm(np.diff(pose[4:7, o], axis=1), axis=0).mean()
    d_rand = np.linalg.norm(pose[4:7, rng.permutation(n)] - pose[4:7], axis=0).mean()
    assert d_seq < 0.5 * d_rand


def test_nut_bolt_locality_order_follows_the_axis():
    w = W.nut_bolt_workload(n_env=200, spec=W.M4_128)
    o = fc.locality_order(w)
    z = w.pose[6, o]
    # lateral jitter is tiny next to the axial range: the order is nearly sorted in z
    assert np.mean(np.diff(z) >= -1e-4) > 0.9
