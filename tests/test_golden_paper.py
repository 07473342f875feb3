"""Values the paper prints that bear on the hot path's data (CPU only)."""
import os

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
