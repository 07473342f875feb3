"""Reference of the patch-based contact reduction of Algorithm 1 (test
infrastructure only).

Section III-C, Algorithm 1: per shape pair (environment), start with no
patches; for each batch of 1,024 features: Generate candidates, Assign them
to existing patches by normal similarity, then while candidates remain:
FindDeepest, BinReduce (the remaining candidates similar to the deepest
join its new patch), AddPatch (the patch list is capped at N; a new patch is
weighed against an existing patch of similar normal, by a measure favouring
surface area and depth, and either both are kept or the existing one is
replaced).

The paper fixes neither the similarity test, the patch record, nor the
measure.  Readings (listed with the others in the design notes):
  * features are mesh vertices; batch k holds vertices [1024 k, 1024 k + 1024);
    a candidate is a query with phi < margin, its normal and depth as the
    vertex queries define them (FP32, the kernel's values);
  * similar(a, b): dot(a, b) >= cos_sim, the dot evaluated in FP32 as
    (a.x b.x + a.y b.y) + a.z b.z without fused multiply-adds (the same
    operations as the kernel, so both sides take the same decisions);
  * a patch holds: its normal (the founding contact's), its deepest member
    (largest depth, lowest vertex index on ties: the key
    sortable(depth) << 32 | ~vidx of the other reductions) and its member
    count;
  * Assign: a candidate joins the existing patch (one that existed when the
    batch began) of largest dot among those similar to it, lowest index on
    ties;
  * FindDeepest: the largest key among the remaining candidates; BinReduce:
    the new patch takes the deepest and every remaining candidate similar to
    its normal;
  * AddPatch: with fewer than N patches the new one is appended; otherwise it
    is compared with the existing patch of largest dot with its normal (lowest
    index on ties) and replaces it iff its value is larger, value =
    float32(members) * depth of the deepest member (FP32): the member count
    stands for the patch's surface area.  A patch that is not kept is dropped
    with its members.
"""
from __future__ import annotations

import numpy as np

BATCH = 1024


def dot32(a, b):
    """FP32 dot product, (a.x b.x + a.y b.y) + a.z b.z, no FMA; a (3,), b (..., 3)."""
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    return (a[0] * b[..., 0] + a[1] * b[..., 1]) + a[2] * b[..., 2]


def sortable(depth32):
    """Order-preserving uint32 image of float32 depths."""
    u = np.asarray(depth32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    neg = (u >> 31) == 1
    return np.where(neg, (~u) & 0xFFFFFFFF, u | 0x80000000)


def keys(depth32, vidx):
    """sortable(depth) << 32 | ~vidx: larger = deeper, then lower index
    (-0.0 counts as +0.0)."""
    d = np.asarray(depth32, dtype=np.float32)
    d = np.where(d == 0, np.float32(0.0), d)
    return (sortable(d) << np.uint64(32)) | ((~np.asarray(vidx, dtype=np.uint64)) & np.uint64(0xFFFFFFFF))


def value32(members, depth32):
    """The AddPatch measure: float32(members) * depth, in FP32."""
    return np.float32(members) * np.float32(depth32)


def most_similar(normal, patch_normals, cos_sim=None):
    """Index of the patch of largest FP32 dot with normal (lowest on ties);
    with cos_sim, only among patches similar to it (-1 if none)."""
    if len(patch_normals) == 0:
        return -1
    d = dot32(normal, np.asarray(patch_normals, dtype=np.float32))
    if cos_sim is not None:
        d = np.where(d >= np.float32(cos_sim), d, -np.inf)
        if not np.isfinite(d).any():
            return -1
    return int(np.argmax(d))  # first maximum


def reduce_env(vidx, depth32, normal32, cos_sim, n_max):
    """Algorithm 1 over one environment's candidates.

    vidx (m,) vertex indices (ascending order is not required), depth32 (m,)
    float32, normal32 (m, 3) float32.  Returns (patches, dropped): each patch
    a dict with normal (3,) float32, key (uint64 of the deepest member),
    members and founder (vertex index); dropped = members of patches that
    were not kept."""
    vidx = np.asarray(vidx, dtype=np.int64)
    depth32 = np.asarray(depth32, dtype=np.float32)
    normal32 = np.asarray(normal32, dtype=np.float32)
    k_all = keys(depth32, vidx)
    patches = []
    dropped = 0
    batch_of = vidx // BATCH
    for bk in np.unique(batch_of):
        sel = np.nonzero(batch_of == bk)[0]
        # Assign, against the patches that exist as the batch begins
        existing = [p["normal"] for p in patches]
        remaining = []
        for i in sel:
            j = most_similar(normal32[i], existing, cos_sim)
            if j < 0:
                remaining.append(i)
            else:
                patches[j]["members"] += 1
                patches[j]["key"] = max(patches[j]["key"], int(k_all[i]))
        remaining = np.asarray(remaining, dtype=np.int64)
        while len(remaining):
            best = remaining[int(np.argmax(k_all[remaining]))]  # keys are unique
            nb = normal32[best]
            sim = dot32(nb, normal32[remaining]) >= np.float32(cos_sim)
            sim |= remaining == best
            new = {"normal": nb.copy(), "key": int(k_all[best]), "members": int(sim.sum()), "founder": int(vidx[best])}
            remaining = remaining[~sim]
            if len(patches) < n_max:
                patches.append(new)
            else:
                j = most_similar(nb, [p["normal"] for p in patches])
                old = patches[j]
                if value32(new["members"], key_depth(new["key"])) > value32(old["members"], key_depth(old["key"])):
                    patches[j] = new
                    dropped += old["members"]
                else:
                    dropped += new["members"]
    return patches, dropped


def key_depth(key):
    """float32 depth of a key."""
    s = np.uint32(int(key) >> 32)
    u = np.where(s >> 31 == 1, s & np.uint32(0x7FFFFFFF), ~s)
    return np.asarray(u, dtype=np.uint32).view(np.float32)[()]


def key_vidx(key):
    return int((~np.uint64(int(key) & 0xFFFFFFFF)) & np.uint64(0xFFFFFFFF))
