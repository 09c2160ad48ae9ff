"""Host logic of bench.py (CPU): the dense tile schedule that decides whether
the recorded HBM traffic applies, and the one-GPU contract."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def internal_nodes(n):
    """Nodes of the recursion on n (a multiple of 64) that split: leaves are
    64 or 128, a node of t tiles splits into floor(t/2) and ceil(t/2)."""
    if n <= 128:
        return 0
    t = n // 64
    return 1 + internal_nodes(t // 2 * 64) + internal_nodes(n - t // 2 * 64)


def test_schedule_has_three_products_per_node():
    for n in (192, 256, 1024, 4544, 27008):
        assert len(bench.tile_schedule(n, 4096)) == 3 * internal_nodes(n)


def test_thresholds_beyond_the_largest_product_are_equivalent():
    # 4544 = 71 tiles: the root's products have 36 x 35 (and 36 x 36 + 36 x 35
    # for the pair) tiles of 64, all below 4096, and fewer than 512 of 128
    assert bench.tile_schedule(4544, 4096) == bench.tile_schedule(4544, 1 << 40)
    assert set(bench.tile_schedule(4544, 4096)) == {32}
    # threshold 1024 puts exactly the root's three products on 64 x 64 tiles
    assert bench.tile_schedule(4544, 1024).count(64) == 3
    # at 27008 every product with 4096 tiles of 64 has over 512 of 128, so
    # thresholds from 4096 up give the same schedule; 1024 differs
    assert bench.tile_schedule(27008, 4096) == bench.tile_schedule(27008, 1 << 40)
    assert bench.tile_schedule(27008, 1024) != bench.tile_schedule(27008, 4096)
    assert bench.tile_schedule(27008, 4096).count(128) == 21  # the top three levels (1 + 2 + 4 nodes)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr
