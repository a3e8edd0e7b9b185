"""Host-side pieces of the autotuner: cache keys and the check that a winning
setting really sorted (torch on the CPU; no GPU needed)."""

import numpy as np
import pytest

from paper_1703_00687_amd import autotune as at
from paper_1703_00687_amd import workloads as wl


def test_shape_key():
    assert at.shape_key("gfx950", 16, 8, 1 << 28) == "gfx950/R16/K8/n2^28"
    assert at.shape_key("gfx950", 32, 16, 3) == "gfx950/R32/K16/n2^2"
    assert at.shape_key("gfx950", 16, 8, 1 << 28, "zipf16") == "gfx950/R16/K8/n2^28/zipf16"


def test_lookup_prefers_the_workload_then_the_nearest_size():
    cache = {"gfx950/R16/K8/n2^28/uniform16": {"tuning": {"tiny_max": 1}},
             "gfx950/R16/K8/n2^28/zipf16": {"tuning": {"tiny_max": 2}},
             "gfx950/R16/K8/n2^24": {"tuning": {"tiny_max": 3}},
             "gfx950/R32/K16/n2^27/deep32": {"tuning": {"tiny_max": 4}},
             "gfx942/R16/K8/n2^28/zipf16": {"tuning": {"tiny_max": 5}}}
    k, e = at.lookup(cache, "gfx950", 16, 8, 1 << 27, "zipf16")
    assert k == "gfx950/R16/K8/n2^28/zipf16" and e["tuning"]["tiny_max"] == 2
    # no entry for this distribution: the one tuned on none, never another's
    k, e = at.lookup(cache, "gfx950", 16, 8, 1 << 28, "keys16")
    assert k == "gfx950/R16/K8/n2^24"
    k, e = at.lookup(cache, "gfx950", 32, 16, 1 << 27, "uniform32")
    assert k is None and e is None
    k, e = at.lookup(cache, "gfx950", 32, 16, 1 << 20, "deep32")
    assert k == "gfx950/R32/K16/n2^27/deep32"


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
