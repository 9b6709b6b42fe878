"""The binding's stage wrappers check every tensor before calling the library (CPU only).

The stage entry points of the C ABI take raw device pointers and sizes derived from the
tensors, so a wrong tensor would become an out-of-bounds device write.  Each wrapper
checks dtype, exact shape and contiguity of every input and output first and raises
ValueError; a tensor that passes those checks but is not on the device raises TypeError.
Nothing here reaches a kernel launch (there is no GPU in this test)."""
import pytest
import torch

import paper_1610_03525_amd as ptg

f32, i32, i64 = torch.float32, torch.int32, torch.int64


def z(shape, dtype=f32):
    return torch.zeros(shape, dtype=dtype)


@pytest.mark.parametrize("call", [
    lambda: ptg.coords(0.5, 2.0, 4, 0, z((3, 16), i64), z((4, 16))),       # cells rows != octaves
    lambda: ptg.coords(0.5, 2.0, 4, 0, z((4, 16), i64), z((4, 15))),       # frac shape
    lambda: ptg.coords(0.5, 2.0, 4, 0, z((4, 16), i32), z((4, 16))),       # cells dtype
    lambda: ptg.coords(0.5, 2.0, 4, 0, z((4, 16), i64), z((16, 4)).t()),   # frac not contiguous
    lambda: ptg.lattice_2d(1, 0, 0, 0, z((5, 6), i32), z((2, 5, 7))),      # grad shape
    lambda: ptg.lattice_2d(1, 0, 0, 0, z((5, 6), f32), None),              # keys dtype
    lambda: ptg.lattice_2d(1, 0, 0, 0, None, z((3, 5, 6))),                # grad components
    lambda: ptg.lattice_2d(1, 0, 0, 0, None, None),                        # no output
    lambda: ptg.heights_2d(1, 0, 0, 0, z((6, 5)).t()),                     # not contiguous
    lambda: ptg.heights_2d(1, 0, 0, 0, z((5, 6), i32)),                    # dtype
    lambda: ptg.lattice_3d(1, 0, 0, 0, 0, z((2, 3, 4), i32), z((2, 3, 5), i32), None),
    lambda: ptg.lattice_3d(1, 0, 0, 0, 0, z((2, 3, 4), i32), None, z((2, 2, 3, 4))),
    lambda: ptg.cells_2d(1, z((2, 5, 6)), 1.0, z((4, 5, 4, 5))),           # coefficient count
    lambda: ptg.cells_2d(2, z((2, 5, 6)), 1.0, z((4, 5, 4, 4))),           # quintic needs 6 x 6
    lambda: ptg.cells_2d(1, z((2, 5, 6)), 1.0, z((5, 6, 4, 4))),           # cells = nodes - 1
    lambda: ptg.cells_2d(1, z((2, 1, 6)), 1.0, z((0, 5, 4, 4))),           # one node row
    lambda: ptg.cells_3d(1, z((3, 3, 4, 5)), 1.0, z((2, 3, 4, 4, 4, 3))),
    lambda: ptg.cells_3d(1, z((2, 3, 4, 5)), 1.0, z((2, 3, 4, 4, 4, 4))),  # gradient components
])
def test_wrong_tensor_is_rejected_before_launch(call):
    with pytest.raises(ValueError):
        call()


@pytest.mark.parametrize("call", [
    lambda: ptg.coords(0.5, 2.0, 4, 0, z((4, 16), i64), z((4, 16))),
    lambda: ptg.lattice_2d(1, 0, 0, 0, z((5, 6), i32), z((2, 5, 6))),
    lambda: ptg.heights_2d(1, 0, 0, 0, z((5, 6))),
    lambda: ptg.lattice_3d(1, 0, 0, 0, 0, z((2, 3, 4), i32), z((2, 3, 4), i32), z((3, 2, 3, 4))),
    lambda: ptg.cells_2d(2, z((2, 5, 6)), 1.0, z((4, 5, 6, 6))),
    lambda: ptg.cells_3d(1, z((3, 3, 4, 5)), 1.0, z((2, 3, 4, 4, 4, 4))),
])
def test_right_shapes_on_the_host_are_not_device_memory(call):
    with pytest.raises(TypeError):
        call()
