"""Host checks of the row-range split used to rehearse row-block sharding:
the ranges cover every row once, in order, and cut the intermediate-product
prefix sum at the k/P points (brute-force comparison)."""
import numpy as np
import pytest
import torch

from paper_2512_12036_amd import shard


def brute_ranges(ip, parts):
    total = int(ip.sum())
    prefix = np.cumsum(ip)
    cuts = []
    for k in range(1, parts):
        target = (total * k + parts - 1) // parts
        r = next((i + 1 for i, p in enumerate(prefix) if p >= target), len(ip))
        cuts.append(r)
    bounds = [0] + cuts + [len(ip)]
    return [(a, b) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("parts", [1, 2, 3, 8])
def test_row_ranges_match_brute_force(seed, parts):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 400))
    ip = rng.integers(0, 50, size=m) * (rng.random(m) < 0.7)
    if seed == 0:
        ip[:] = 0  # all rows empty
    got = shard.row_ranges(torch.from_numpy(ip.astype(np.int64)), parts)
    assert got == brute_ranges(ip, parts)
    covered = [r for a, b in got for r in range(a, b)]
    assert covered == list(range(m))


def test_row_ranges_edge_cases():
    assert shard.row_ranges(torch.zeros(0, dtype=torch.int64), 4) == []
    one_hub = torch.tensor([0, 0, 100, 0, 0], dtype=torch.int64)
    assert shard.row_ranges(one_hub, 4) == [(0, 3), (3, 5)]
    with pytest.raises(ValueError):
        shard.row_ranges(one_hub, 0)
