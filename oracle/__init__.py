"""CPU oracle for the vertex-vs-SDF contact path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 NumPy evaluation of what the path computes, written from
the paper's definitions:

  * ``query``   -- transform of body A's vertices into body B's frame, the
                   trilinear SDF value and its exact gradient, the candidate
                   contact (point, normal, depth) and its normal bin
                   (Section III-A: SDF value and gradient; Section III-C,
                   Algorithm 1 Generate);
  * ``reduce``  -- the deepest candidate per (environment, normal bin) with a
                   lowest-vertex-index tie-break (Section III-C, Algorithm 1
                   FindDeepest / BinReduce, with fixed normal bins);
  * ``adjoint`` -- the penetration penalty 0.5 k phi^2 over penetrating
                   vertices, its gradients with respect to an se(3) twist of
                   each environment's pose and to the vertices, and central
                   finite differences of the same loss;
  * ``meshdist``-- brute-force signed point-triangle distance for tiny
                   meshes (used only to pin ``query``).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code, header, helper or
table generator with the HIP library, and never imports it.
"""
