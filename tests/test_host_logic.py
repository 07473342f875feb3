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


def test_layout_entries_are_keyed_without_the_layout(tmp_path):
    p = str(tmp_path / "c.json")
    sig = "v1;dt=0;lay=1;K=32;env=1000;grids=256x256x512,;meshes=16396,"
    assert autotune.layout_key(sig) == "v1;dt=0;K=32;env=1000;grids=256x256x512,;meshes=16396,"
    assert autotune.best_layout(sig, p) is None  # no cache yet
    lay = dict(key=autotune.layout_key(sig), layout="slab", step_ms={"brick": 0.2, "slab": 0.1})
    autotune.save([dict(autotune.DEFAULT, key=sig, ms=1.0)], p, [lay])
    # any layout's signature of the same batch finds the entry; another batch does not
    assert autotune.best_layout(sig.replace("lay=1", "lay=0"), p) == "slab"
    assert autotune.best_layout(sig.replace("env=1000", "env=999"), p) is None
    # launch-shape saves keep the layout entries; a layout save replaces by key
    autotune.save([dict(autotune.DEFAULT, key="b", ms=1.0)], p)
    autotune.save([], p, [dict(lay, layout="brick")])
    rec = json.load(open(p))
    assert [e["layout"] for e in rec["layouts"]] == ["brick"]
    assert sorted(e["key"] for e in rec["entries"]) == sorted([sig, "b"])


def test_layout_choice_keeps_brick_within_the_margin():
    assert autotune.pick_layout({"brick": 1.0, "slab": 0.995, "linear": 2.0}) == "brick"
    assert autotune.pick_layout({"brick": 1.0, "slab": 0.98, "linear": 0.985}) == "slab"
    assert autotune.pick_layout({"brick": 1.0, "slab": 1.2, "linear": 0.5}) == "linear"


def test_wave_priority_choice_keeps_the_default_within_the_margin():
    assert autotune.PRIOS[0] == autotune.DEFAULT["wave_prio"] == 1
    assert autotune.pick_prio({1: 1.0, 0: 0.995, 2: 1.01}) == 1
    assert autotune.pick_prio({1: 1.0, 0: 1.02, 2: 0.97}) == 2
    assert autotune.pick_prio({1: 1.0, 0: 0.9, 2: 0.97}) == 0


def test_library_reads_a_cache_with_layout_entries(tmp_path):
    L = fc.lib()
    p = str(tmp_path / "c.json")
    autotune.save([dict(autotune.DEFAULT, key="a", ms=1.0), dict(autotune.DEFAULT, key="b", ms=2.0)], p,
                  [dict(key="a", layout="brick", step_ms={"brick": 0.1, "slab": 0.2})])
    assert L.fc_autotune_load(p.encode()) == 2


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


def test_twosum_equals_ordered_fast2sum_in_float32():
    """The adjoint's pair combine takes the rounding error of a + b by
    branch-free TwoSum; in float32 it equals the magnitude-ordered Fast2Sum of
    Neumaier's step bit for bit (both are the exact error), so the switch does
    not change a single sum."""
    rng = np.random.default_rng(5)
    f = np.float32
    a = (rng.standard_normal(200000) * np.exp(rng.uniform(-30, 30, 200000))).astype(f)
    b = (rng.standard_normal(200000) * np.exp(rng.uniform(-30, 30, 200000))).astype(f)
    b[:1000] = -a[:1000]  # exact cancellation
    b[1000:2000] = a[1000:2000]
    with np.errstate(over="ignore", invalid="ignore"):
        t = a + b
        bb = t - a
        two = (a - (t - bb)) + (b - bb)
        ordered = np.where(np.abs(a) >= np.abs(b), (a - t) + b, (b - t) + a)
    ok = np.isfinite(t)
    assert np.array_equal(two[ok], ordered[ok])
    # and it is the exact error (checked where float64 holds a + b exactly:
    # exponents less than 29 binades apart)
    with np.errstate(divide="ignore"):
        close = np.abs(np.log2(np.abs(a.astype(np.float64))) - np.log2(np.abs(b.astype(np.float64)))) < 28
    exact = (a.astype(np.float64) + b.astype(np.float64)) - t.astype(np.float64)
    sel = ok & close
    assert sel.sum() > 10000
    assert np.array_equal(two[sel].astype(np.float64), exact[sel])
