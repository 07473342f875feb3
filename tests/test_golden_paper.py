"""Values the paper prints that bear on the hot path's data (CPU only)."""
import os

import numpy as np

from paper_2205_03532_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _rows():
    with open(os.path.join(HERE, "golden", "paper_sdf_memory.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, nx, ny, nz, mb, kind = line.split()
                yield name, int(nx), int(ny), int(nz), float(mb), kind


def test_sdf_memory_column_is_fp32_samples():
    """Appendix C, geometric representation table: memory = dims x 4 B (MiB)."""
    n_fp32 = 0
    for name, nx, ny, nz, mb, kind in _rows():
        mib = nx * ny * nz * 4 / 2**20
        if kind == "fp32":
            assert abs(mib - mb) / mb < 2e-3, (name, mib, mb)
            n_fp32 += 1
        else:
            assert abs(mib - mb) / mb > 0.2, name
    assert n_fp32 == 5


def test_fp32_grid_storage_matches_that_layout():
    """An FP32 grid of those dims occupies exactly dims x 4 bytes here too."""
    g = W.Grid(values=np.zeros((144, 404, 144), np.float32), dtype="f32", origin=(0.0, 0.0, 0.0), h=1e-4)
    assert g.nbytes == 144 * 404 * 144 * 4
    assert abs(g.nbytes / 2**20 - 31.95) < 0.01


def test_contact_record_is_36_bytes():
    """Section III-B: about 7 floats (point, normal, distance) + 2 ints = 36 B.

    The reduced-contact slot written by the library holds the same 7 float32
    plus the vertex index; the two body indices are implicit in the slot's
    environment.
    """
    floats, ints = 3 + 3 + 1, 2
    assert floats * 4 + ints * 4 == 36
