"""The two measurement entry points that put the search kernels' times in
context: the LDS read rate (ds_read_b64 / ds_read_b128 on every CU) and the
time per back-to-back launch of an empty kernel.  Checks that they return
plausible values on the device and reject invalid arguments."""
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def test_lds_read_rate(ctx):
    import paper_2303_14335_amd as mp
    say("LDS read rate, b64 and b128")
    b64 = mp.mpld_measure_lds_read_rate(ctx, 8, 200)
    b128 = mp.mpld_measure_lds_read_rate(ctx, 16, 200)
    for r in (b64, b128):
        assert r["GBps"] > 0 and r["bytes_per_clock_per_cu"] > 0
        # a CU cannot read more than 256 bytes of LDS per clock
        assert r["bytes_per_clock_per_cu"] < 300
    for bad in ((4, 100), (16, 0), (16, 1 << 25)):
        with pytest.raises(mp.MpldError):
            mp.mpld_measure_lds_read_rate(ctx, *bad)


def test_launch_floor(ctx):
    import paper_2303_14335_amd as mp
    say("launch floor, 1 x 64 and 868 x 256")
    one = mp.mpld_measure_launch_floor(ctx, 1, 64, 50)
    many = mp.mpld_measure_launch_floor(ctx, 868, 256, 50)
    assert 0 < one < 1000 and 0 < many < 1000
    for grid, block, reps in ((0, 64, 10), (1, 65, 10), (1, 2048, 10), (1, 64, 0)):
        with pytest.raises(mp.MpldError):
            mp.mpld_measure_launch_floor(ctx, grid, block, reps)


def test_touch_floor(ctx):
    import paper_2303_14335_amd as mp
    say("touch floor, 1 x 64 and 868 x 256")
    one = mp.mpld_measure_touch_floor(ctx, 1, 64, 50)
    many = mp.mpld_measure_touch_floor(ctx, 868, 256, 50)
    assert 0 < one < 1000 and 0 < many < 1000
    for grid, block, reps in ((0, 64, 10), (1, 65, 10), (1, 2048, 10), (1, 64, 0)):
        with pytest.raises(mp.MpldError):
            mp.mpld_measure_touch_floor(ctx, grid, block, reps)
