"""A test graph whose vertices with omega_2 above 2^16 - 2 are exactly its
highest-degree ones (shared by the CPU emulation and the GPU tests of the
16-bit level-2 layout)."""
import numpy as np

from paper_1910_13874_amd import inputs


def wide_prefix_graph():
    """K_{300,300} (omega_2 = 90,000 at each of its 600 vertices: degree 300,
    neighbours of degree 300) joined by a few edges to a BA graph of 4,000
    vertices: the vertices with omega_2 above 2^16 - 2 are exactly the
    K_{300,300} ones, which are also the 600 of highest degree."""
    ba = inputs.barabasi_albert(4000, 3, 91)
    rows = np.repeat(np.arange(ba.n), np.diff(ba.row_ptr))
    a, b = np.meshgrid(np.arange(300), np.arange(300, 600), indexing="ij")
    src = np.concatenate([rows + 600, a.ravel(), np.arange(0, 600, 50)])
    dst = np.concatenate([ba.col_idx.astype(np.int64) + 600, b.ravel(),
                          600 + np.arange(0, 600, 50) * 3])
    return inputs.from_edges(4600, src.astype(np.int32), dst.astype(np.int32), symmetrize=True,
                             name="wide_prefix")
