"""Launch planning on the host (no GPU): the each-unordered-pair-once form
keeps one partial-sum slot per body and block, a workspace that grows as
N^2, so beyond a share of the device's memory the pair sums switch to the
one-sided form, whose workspace is O(N)."""
import pytest

from paper_2103_01983_amd import native

HBM = 288 * 10**9  # MI355X


@pytest.mark.parametrize("op", sorted(native.PAIR_OPS))
def test_four_million_bodies_plan_a_launch_that_fits(op):
    p = native.pair_plan(op, 4 * 2**20, device_bytes=HBM)
    assert p["sym"] == 0 and p["splits"] >= 1
    assert p["ws_bytes"] <= HBM // 32
    # the one-sided workspace is linear in N: at most one chunk partial per
    # chunk, accumulator and body
    assert p["ws_bytes"] <= p["splits"] * 5 * 4 * 4 * 2**20


@pytest.mark.parametrize("n", [32768, 65536, 131072])
def test_benchmark_sizes_keep_the_each_pair_once_form(n):
    # the shipped table's choice at the benchmark sizes stays in force
    for op in ("velocity", "jvp", "vjp", "block_jacobian"):
        p = native.pair_plan(op, n, device_bytes=HBM)
        assert p["sym"] == 1, (op, n, p)
        tb = 256 * p["k"]
        nb = -(-n // tb)
        na = 3 if op in ("vjp", "block_jacobian") else 2
        assert p["ws_bytes"] == 4 * (2 * nb * na * n + 64)


def test_cap_follows_the_device_memory():
    # the same size on a device with 1/64 of the memory falls back earlier
    n = 131072
    big = native.pair_plan("velocity", n, device_bytes=HBM)
    small = native.pair_plan("velocity", n, device_bytes=HBM // 64)
    assert big["sym"] == 1 and small["sym"] == 0
    assert small["ws_bytes"] <= (HBM // 64) // 32


def test_every_size_up_to_the_limit_fits():
    for e in range(8, 31):
        for op in native.PAIR_OPS:
            p = native.pair_plan(op, 2**e, device_bytes=HBM)
            assert p["ws_bytes"] <= HBM // 32, (op, e, p)


def test_plan_rejects_bad_arguments():
    import ctypes
    out = (ctypes.c_int32 * 5)()
    L = native.lib()
    assert L.ptrom_pair_plan(None, 256, HBM, 0, 0, out, None) != 0
    assert L.ptrom_pair_plan(None, 256, HBM, 9, 100, out, None) != 0
    assert L.ptrom_pair_plan(None, 0, HBM, 0, 100, out, None) != 0
    assert L.ptrom_pair_plan(None, 256, 0, 0, 100, out, None) != 0
    assert L.ptrom_pair_plan(b"/nonexistent/table.txt", 256, HBM, 0, 100, out, None) != 0
    assert L.ptrom_pair_plan(None, 256, HBM, 0, 2**30 + 1, out, None) != 0
