"""Host-side pieces of the autotuner: cache keys and the check that a winning
setting really sorted (torch on the CPU; no GPU needed)."""

import numpy as np
import pytest

from paper_1703_00687_amd import autotune as at
from paper_1703_00687_amd import workloads as wl


def test_shape_key():
    assert at.shape_key("gfx950", 16, 8, 1 << 28) == "gfx950/R16/K8/n2^28"
    assert at.shape_key("gfx950", 32, 16, 3) == "gfx950/R32/K16/n2^2"


@pytest.mark.parametrize("r,k", [(16, 8), (32, 16), (16, 5)])
def test_looks_sorted(r, k):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(r + k)
    h = wl.random_records(rng, 5000, r, k, distinct_keys=300)
    key = [h[:, i] for i in range(k)]  # lexsort: last key is primary
    order = np.lexsort(key[::1])
    src = torch.from_numpy(h)
    good = torch.from_numpy(h[order])
    assert at._looks_sorted(good, src, k)
    assert not at._looks_sorted(src, src, k)
    bad = good.clone()
    bad[17, r - 1] ^= 0x40  # a payload byte changed: not the same records
    assert not at._looks_sorted(bad, src, k)
