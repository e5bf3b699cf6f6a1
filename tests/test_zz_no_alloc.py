"""fftcg_loadstep_noalloc (the load step with its partials in the library's
static device array) against fftcg_loadstep on the same inputs: the same
index, bitwise the same d, on two calls in a row with the second on a
smaller grid, and on an all-zero d (index -1, d untouched)."""

import numpy as np
import pytest

from paper_1305_3625_amd import binding
from workloads import spectrum
from gpu_util import dev, host, banner

pytestmark = pytest.mark.gpu


def _inputs(L, seed):
    rng = np.random.default_rng([70, seed])
    x = rng.uniform(0.0, 1.0, (L, L))
    t = rng.uniform(0.1, 1.0, (L, L))
    d = rng.uniform(0.5, 1.5, (L, L))
    d[rng.random((L, L)) < 0.3] = 0.0
    n = L * L
    # an exact tie of the largest live ratio across two partial blocks
    # (blocks of 256 entries), the first of the two live
    for i in (n // 2 - 1, n // 2, n - 1):
        x.ravel()[i], t.ravel()[i], d.ravel()[i] = 50.0, 0.5, 1.0
    return x, t, d


def _both(plan, x, t, d):
    d1, d2 = dev(d), dev(d)
    i1 = plan.loadstep(dev(x), dev(t), d1)
    i2 = plan.loadstep_noalloc(dev(x), dev(t), d2)
    return i1, i2, host(d1), host(d2)


def test_noalloc_matches_loadstep():
    for L, seed in ((512, 0), (64, 1)):  # the second call on a smaller grid
        banner("loadstep-noalloc", L)
        plan = binding.Plan(L, 1, spectrum(2 * L, 1e-3))
        x, t, d = _inputs(L, seed)
        i1, i2, d1, d2 = _both(plan, x, t, d)
        assert i1 == i2 == L * L // 2 - 1
        assert np.array_equal(d1, d2)
        assert d2.ravel()[i2] == 0.0
        plan.close()
    # every d zero: no live entry, index -1, d unchanged
    L = 32
    plan = binding.Plan(L, 1, spectrum(2 * L, 1e-3))
    x, t, _ = _inputs(L, 2)
    i1, i2, d1, d2 = _both(plan, x, t, np.zeros((L, L)))
    assert i1 == i2 == -1
    assert not d2.any()
    plan.close()
