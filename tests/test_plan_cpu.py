"""Host-only launch planning (tr_get_sweep_plan with no context): which
kernel a batch gets and the constraints the plan must satisfy.  Field
pointers are never read."""
import pytest

from paper_2509_01416_amd import binding as B
from paper_2509_01416_amd import inputs as I


def _probs(shapes, bc=(0, 0, 0, 0)):
    arr = (B.TrProblem * len(shapes))()
    for k, (nx, ny) in enumerate(shapes):
        arr[k].dim, arr[k].nx, arr[k].ny = 2, nx, ny
        arr[k].lx = arr[k].ly = 10.0
        arr[k].sigma_t = arr[k].sigma_s = arr[k].source = 0x1000
        for f in range(4):
            arr[k].bc[f] = bc[f]
    return arr


def _plan(shapes, n=8, bc=(0, 0, 0, 0)):
    q = B.Quad.from_inputs(I.level_symmetric_2d(n))
    return B.sweep_plan(_probs(shapes, bc), len(shapes), q)


def test_benchmark_batch_gets_the_specialised_kernel():
    p = _plan([(256, 256)] * 16, n=16)
    assert p["specialised"] == 1 and p["R"] == 64 and p["D"] == 1
    # 36 directions per octant in S slices of W waves
    assert p["W"] * p["S"] >= 36 and p["W"] * (p["S"] - 1) < 36
    assert p["KB"] == 16


@pytest.mark.parametrize("shapes,why", [
    ([(64, 128)], "nx < 63 + KB with two row blocks"),
    ([(16, 64)], "one row block, nx < ny - 1"),
    ([(256, 256), (64, 200)], "nx < 63 + KB for the second grid"),
])
def test_generic_kernel_when_the_specialised_one_does_not_apply(shapes, why):
    assert _plan(shapes)["specialised"] == 0, why


@pytest.mark.parametrize("shapes,n", [
    ([(256, 256), (48, 48)], 8),   # ragged single row block beside full ones
    ([(256, 200)], 8),             # ragged last row block (200 = 3 x 64 + 8)
    ([(96, 96), (32, 32), (128, 128)], 8),
    ([(37, 23)], 8),               # one row block narrower than 64
    ([(4, 4)], 4),
    ([(5, 6)], 4),
    ([(96, 96)] * 16, 16),
    ([(3, 2)] * 16, 16),           # KB <= nx caps the block at 2
])
def test_ragged_row_blocks_take_the_specialised_kernel(shapes, n):
    p = _plan(shapes, n=n)
    assert p["specialised"] == 1 and p["R"] == 64
    assert 2 <= p["KB"] <= min(nx for nx, _ in shapes)
    if len(shapes) == 16 and shapes[0][0] >= 16:
        assert p["W"] == 9 and p["KB"] == 16


def test_reflective_faces_use_the_generic_kernel():
    assert _plan([(128, 128)], bc=(1, 0, 0, 0))["specialised"] == 0
    assert _plan([(128, 128)])["specialised"] == 1


def test_block_size_shrinks_to_fit_narrow_grids():
    # 16 instances at S16 give W = 9 waves, which alone would allow KB = 16;
    # the specialised kernel needs nx >= 63 + KB where a grid has more than
    # one row block
    p = _plan([(70, 128)] * 16, n=16)   # KB <= 7 -> 4
    assert p["specialised"] == 1 and p["KB"] == 4
    p = _plan([(70, 64)] * 16, n=16)    # one row block: any nx >= 64
    assert p["specialised"] == 1 and p["KB"] == 16
    p = _plan([(64, 64)] * 64, n=8)     # the 64 x 64 network-grid batches
    assert p["specialised"] == 1 and p["KB"] == 16
    p = _plan([(66, 128)] * 16, n=16)   # KB <= 3 -> 2
    assert p["specialised"] == 1 and p["KB"] == 2
    p = _plan([(80, 64)] * 16, n=16)    # KB <= 17 -> 16
    assert p["specialised"] == 1 and p["KB"] == 16


def test_plan_rows_divide_ny():
    # the generic kernel's segments divide ny (its ring writer is the last
    # lane of every segment); reflective faces keep these on it
    for shapes in ([(96, 96)], [(48, 48)], [(100, 40)], [(33, 66)]):
        p = _plan(shapes, bc=(1, 0, 0, 0))
        assert p["specialised"] == 0
        assert shapes[0][1] % p["R"] == 0 and p["R"] <= shapes[0][0]


@pytest.mark.parametrize("count,n,W,S", [
    (1, 8, 4, 3),      # lone S8 grid: 10 directions in 3 slices of 4 waves
    (16, 8, 4, 3),     # 2 per XCD: 8 x 3 = 24 workgroups on its 32 CUs
    (55, 8, 10, 1),    # 7 per XCD: one slice already fills the XCD
    (256, 8, 10, 1),
    (1, 16, 6, 6),     # 36 directions: at most 6 slices (partial planes)
    (1, 4, 4, 1),      # 3 directions: one slice of 4 waves (one idle)
    (1, 6, 4, 2),      # 6 directions: two slices of 4 waves
    (16, 16, 9, 4),
])
def test_specialised_plan_slices_small_batches_to_the_step_time(count, n, W, S):
    # the specialised sweep's step time, not the count of busy CUs, bounds
    # a batch too small to fill the chip: most slices of >= 4 waves (idle
    # ones included) that still give each workgroup a CU of its XCD
    p = _plan([(128, 128)] * count, n=n)
    assert p["specialised"] == 1 and p["KB"] == 16
    assert (p["W"], p["S"]) == (W, S)


def test_wide_grid_plan_sheds_waves_to_fit_the_lds_ring():
    # 32768 cells per row: the ring holds nx values per wave, so only one
    # wave per workgroup fits in 160 KB
    p = _plan([(32768, 64)], n=4)
    assert p["specialised"] == 1 and p["W"] == 1 and p["S"] == 3
