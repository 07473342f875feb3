"""Pins of the patch-reduction oracle (Algorithm 1 with the stated readings),
CPU only: a hand-worked two-batch example with its capacity cases, closed
forms at the extreme thresholds, invariants on random candidates, and
planted mistakes caught."""
import math

import numpy as np
import pytest

from oracle import patches as OP

C10 = np.float32(math.cos(math.radians(10.0)))


def unit(deg_xy, deg_z=0.0):
    a, b = math.radians(deg_xy), math.radians(deg_z)
    return [math.cos(a) * math.cos(b), math.sin(a) * math.cos(b), math.sin(b)]


def hand_case(d1024=0.8):
    """Batch 0: v0 +x 0.5; v1 at 5 deg 0.7; v2 +y 0.2; v3 -x 0.9; v4 +y tilted 3 deg up 0.25.
    Batch 1: v1024 at -8 deg (d1024); v1025 at 178 deg 0.1; v1026 +x 0.95."""
    rows = [(0, unit(0), 0.5), (1, unit(5), 0.7), (2, unit(90), 0.2), (3, unit(180), 0.9),
            (4, [0.0, math.cos(math.radians(3)), math.sin(math.radians(3))], 0.25),
            (1024, unit(-8), d1024), (1025, unit(178), 0.1), (1026, unit(0), 0.95)]
    v = np.array([r[0] for r in rows])
    n = np.array([r[1] for r in rows], dtype=np.float32)
    d = np.array([r[2] for r in rows], dtype=np.float32)
    return v, d, n


def summary(patches):
    return [(OP.key_vidx(p["key"]), p["founder"], p["members"]) for p in patches]


def test_hand_worked_example():
    v, d, n = hand_case()
    # batch 0: v3 founds A alone; v1 founds B with v0; v4 founds C with v2.
    # batch 1: v1025 joins A, v1026 joins B (now deepest), v1024 founds D.
    p, dropped = OP.reduce_env(v, d, n, C10, 8)
    assert summary(p) == [(3, 3, 2), (1026, 1, 3), (4, 4, 2), (1024, 1024, 1)] and dropped == 0
    assert np.array_equal(p[1]["normal"], n[1])  # a patch keeps its founder's normal
    # N = 3: D meets B (the most similar patch); 1 x 0.8 < 3 x 0.95: D is dropped
    p, dropped = OP.reduce_env(v, d, n, C10, 3)
    assert summary(p) == [(3, 3, 2), (1026, 1, 3), (4, 4, 2)] and dropped == 1
    # deeper than B's deepest but with a third of its area: 1 x 1.0 < 2.85, still dropped
    v, d, n = hand_case(d1024=1.0)
    p, dropped = OP.reduce_env(v, d, n, C10, 3)
    assert summary(p) == [(3, 3, 2), (1026, 1, 3), (4, 4, 2)] and dropped == 1
    # a deeper D (1 x 3.0 > 2.85) replaces B in its slot
    v, d, n = hand_case(d1024=3.0)
    p, dropped = OP.reduce_env(v, d, n, C10, 3)
    assert summary(p) == [(3, 3, 2), (1024, 1024, 1), (4, 4, 2)] and dropped == 3


def test_assign_takes_the_most_similar_patch():
    """Patches at 0 and 12 degrees (not similar to each other at 10 degrees);
    a later candidate at 7 degrees is similar to both and joins the 12-degree
    patch (cos 5 > cos 7); one at 3 degrees joins the 0-degree patch."""
    v = np.array([0, 1, 1030, 1031])
    n = np.array([unit(0), unit(12), unit(7), unit(3)], dtype=np.float32)
    d = np.array([0.5, 0.4, 0.3, 0.6], dtype=np.float32)
    p, _ = OP.reduce_env(v, d, n, C10, 8)
    assert summary(p) == [(1031, 0, 2), (1, 1, 2)]


def random_candidates(rng, m, n_verts=5000):
    v = np.sort(rng.choice(n_verts, m, replace=False))
    n = rng.normal(size=(m, 3))
    n = (n / np.linalg.norm(n, axis=1, keepdims=True)).astype(np.float32)
    n[rng.random(m) < 0.3] = n[0]  # repeated normals: exact ties of the dot
    d = rng.gamma(2.0, 1e-4, m).astype(np.float32)
    d[rng.random(m) < 0.05] = d[1]  # repeated depths: ties broken by index
    return v, d, n


def test_extreme_thresholds():
    rng = np.random.default_rng(0)
    v, d, n = random_candidates(rng, 600)
    keys = OP.keys(d, v)
    # everything similar: one patch, every member, the deepest candidate
    p, dropped = OP.reduce_env(v, d, n, -1.0, 8)
    assert len(p) == 1 and p[0]["members"] == 600 and p[0]["key"] == int(keys.max()) and dropped == 0
    assert p[0]["founder"] == OP.key_vidx(int(keys[v < 1024].max()))  # the deepest of the first batch
    # nothing similar (no dot exceeds 1.5): one patch per candidate, none merged
    p, dropped = OP.reduce_env(v, d, n, 1.5, 10 ** 6)
    assert len(p) == 600 and all(q["members"] == 1 for q in p) and dropped == 0
    assert sorted(q["key"] for q in p) == sorted(int(k) for k in keys)


def test_invariants_and_order_independence():
    rng = np.random.default_rng(1)
    for trial in range(6):
        v, d, n = random_candidates(rng, 800)
        cs, nmax = np.float32(rng.choice([0.5, 0.9, 0.97])), int(rng.choice([4, 16, 128]))
        p, dropped = OP.reduce_env(v, d, n, cs, nmax)
        assert len(p) <= nmax
        assert sum(q["members"] for q in p) + dropped == len(v)
        keys = OP.keys(d, v)
        for q in p:
            f = int(np.nonzero(v == q["founder"])[0][0])
            assert np.array_equal(q["normal"], n[f]) and q["key"] >= int(keys[f])
        # the order of candidates inside a batch does not matter
        perm = np.concatenate([rng.permutation(np.nonzero(v // 1024 == b)[0]) for b in np.unique(v // 1024)])
        p2, dropped2 = OP.reduce_env(v[perm], d[perm], n[perm], cs, nmax)
        assert summary(p) == summary(p2) and dropped == dropped2


def test_keys_order_and_roundtrip():
    d = np.array([0.0, -0.0, 1e-6, 2.5e-3, -1e-3, 7.0], dtype=np.float32)
    v = np.arange(len(d)) + 10
    k = OP.keys(d, v)
    assert OP.key_depth(int(k[1])) == 0.0 and (k[0] >> np.uint64(32)) == (k[1] >> np.uint64(32))  # -0 folded to +0
    order = np.argsort(k)[::-1]  # uint64 order (a float64 image would merge the index bits)
    assert list(v[order]) == [15, 13, 12, 10, 11, 14]  # deeper first, then lower index among equal depths
    for kk, dd, vv in zip(k, d, v):
        assert OP.key_depth(int(kk)) == (0.0 if dd == 0 else dd) and OP.key_vidx(int(kk)) == vv


# ------------------------------------------------------------ planted mistakes

PINS = [test_hand_worked_example, test_assign_takes_the_most_similar_patch, test_extreme_thresholds,
        test_invariants_and_order_independence]


def _some_pin_fails():
    for pin in PINS:
        try:
            pin()
        except Exception:
            return True
    return False


def test_planted_patch_mistakes_are_caught(monkeypatch):
    assert not _some_pin_fails()
    orig_ms = OP.most_similar

    def first_similar(normal, patch_normals, cos_sim=None):  # Assign to the first similar patch
        if cos_sim is None or len(patch_normals) == 0:
            return orig_ms(normal, patch_normals, cos_sim)
        dd = OP.dot32(normal, np.asarray(patch_normals, dtype=np.float32))
        hit = np.nonzero(dd >= np.float32(cos_sim))[0]
        return int(hit[-1]) if len(hit) else -1

    def least_similar(normal, patch_normals, cos_sim=None):  # AddPatch weighs the wrong patch
        if cos_sim is not None:
            return orig_ms(normal, patch_normals, cos_sim)
        dd = OP.dot32(normal, np.asarray(patch_normals, dtype=np.float32))
        return int(np.argmin(dd))

    for name, fn in (("first_similar", first_similar), ("least_similar", least_similar)):
        monkeypatch.setattr(OP, "most_similar", fn)
        assert _some_pin_fails(), name
        monkeypatch.setattr(OP, "most_similar", orig_ms)
    orig_val = OP.value32
    monkeypatch.setattr(OP, "value32", lambda members, depth: np.float32(depth))  # area ignored
    assert _some_pin_fails(), "depth_only_value"
    monkeypatch.setattr(OP, "value32", orig_val)
    orig_keys = OP.keys
    monkeypatch.setattr(OP, "keys", lambda d, v: orig_keys(-np.asarray(d, np.float32), v))  # FindDeepest takes the shallowest
    assert _some_pin_fails(), "shallowest"
