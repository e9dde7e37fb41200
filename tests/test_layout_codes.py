"""The Morton codes the GPU layout tests compare gs_spatial_order against, pinned on the CPU to
values worked out by hand (bit k of the x, y, z cell lands at bit 3k, 3k+1, 3k+2)."""
import numpy as np

from tests import gpu_util as U


def test_morton_codes_of_hand_worked_cells():
    # a box from 0 to 1024 on every axis: the cell of a coordinate is its integer part
    pts = np.array([[0, 0, 0], [1024, 1024, 1024], [1, 0, 0], [0, 1, 0], [0, 0, 1], [3, 5, 6],
                    [1023.5, 0, 0], [512, 0, 0]], np.float32)
    codes = U.morton_codes(pts)
    # x=3 (011) y=5 (101) z=6 (110): bits z1y0x0 | z2 y2 x1... written out per level
    x, y, z = 3, 5, 6
    want_356 = sum((((x >> b) & 1) << (3 * b)) | (((y >> b) & 1) << (3 * b + 1)) | (((z >> b) & 1) << (3 * b + 2))
                   for b in range(3))
    assert want_356 == 0b110101011
    assert codes.tolist() == [0, (1 << 30) - 1, 1, 2, 4, want_356, 1 << 27 | 1 << 24 | 1 << 21 | 1 << 18 | 1 << 15
                              | 1 << 12 | 1 << 9 | 1 << 6 | 1 << 3 | 1, 1 << 27]


def test_morton_order_is_stable_and_handles_flat_and_nan():
    pts = np.array([[1, 1, 1], [0, 0, 0], [1, 1, 1], [np.nan, 0, 0], [0.5, 0.5, 0.5]], np.float32)
    order = U.morton_order_reference(pts)
    # cells over the box [0, 1]: (1023,...) for the ones, 0 for the origin and the NaN row, 512 for 0.5
    assert order.tolist() == [1, 3, 4, 0, 2]
    flat = np.array([[2, 7, 1], [2, 3, 1], [2, 5, 1]], np.float32)  # x and z flat: only y orders
    assert U.morton_order_reference(flat).tolist() == [1, 2, 0]
