"""Host-side parts of the autotuner: the cache key."""
import numpy as np

from paper_1810_12742_amd.autotune import DEFAULT_CANDIDATES, _key


def test_cache_key_depends_on_morphology_device_and_candidates():
    p = np.array([-1, 0, 1, 1], dtype=np.int32)
    co = np.array([0, 4], dtype=np.int64)
    k = _key(p, co, None, "dev", DEFAULT_CANDIDATES)
    assert k == _key(p.copy(), co.copy(), None, "dev", DEFAULT_CANDIDATES)
    p2 = p.copy()
    p2[3] = 2
    assert k != _key(p2, co, None, "dev", DEFAULT_CANDIDATES)
    assert k != _key(p, co, None, "other", DEFAULT_CANDIDATES)
    assert k != _key(p, co, None, "dev", DEFAULT_CANDIDATES[:3])
    assert len({tuple(sorted(c.items())) for c in DEFAULT_CANDIDATES}) == len(DEFAULT_CANDIDATES)
