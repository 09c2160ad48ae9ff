"""Host-side check of the batched inverse's launch plan (no GPU needed).

The batched entry point embeds every scene's padded matrix in one virtual
recursion; each launch reads per-scene pointers from a table.  The library's
own checker walks the plan for given sizes and verifies that every product
and leaf stays inside its matrix or scratch and that every 64-column block is
factored exactly once.
"""
import numpy as np

from paper_1808_02414_amd import _binding


def test_single_sizes():
    for n in range(64, 8192 + 1, 64):
        ok, launches = _binding.plan_check([n])
        assert ok, n
        assert launches >= 1


def test_random_mixes():
    rng = np.random.default_rng(5)
    for _ in range(200):
        sizes = 64 * rng.integers(1, 72, rng.integers(1, 300))
        assert _binding.plan_check(sizes)[0], sizes


def test_batch_recipe_sizes():
    rng = np.random.default_rng(1000)
    n = np.rint(np.exp(rng.uniform(np.log(20), np.log(400), 256))).astype(int)
    ok, launches = _binding.plan_check((9 * n + 63) // 64 * 64)
    assert ok and launches < 400


def test_rejects_bad_sizes():
    import pytest
    with pytest.raises(ValueError):
        _binding.plan_check([100])
