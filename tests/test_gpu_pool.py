"""The library's cache of device buffers (freed buffers kept for later requests
of about the same size), through the C ABI.

* A hierarchy built on reused buffers that hold another hierarchy's data gives
  bitwise the same smoothed vectors, singular values, coarse links and solve
  as the same hierarchy built before: no kernel reads memory it has not
  written (the C ABI promises bitwise-identical results for the same inputs).
* Freed buffers are cached, a rebuild of the same shape takes them back, and
  crk_release_cached_memory empties the cache.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

DIMS = [8, 8, 8, 8]
LEVELS = dict(m_prime=[16, 24], k=[8, 16], block=[[4, 4, 4, 4], [2, 2, 2, 2]], n_smooth=[10, 10])


@pytest.fixture(scope="module")
def crk():
    import paper_2502_03091_amd as m
    m.lib()
    return m


def _run(crk, m0, config, seed):
    U = synth.gauge_field(DIMS, 0.3, 1, config=config)
    lat = crk.Lattice(DIMS, m0, 1.0)
    lat.load_gauge(U)
    H = crk.Hierarchy(lat, setup_form=crk.FORM_FP32, seed=seed, **LEVELS)
    try:
        b = synth.gaussian_rhs(2, int(np.prod(DIMS)), config=config)
        x, info = H.solve(b, form=crk.FORM_FP32)
        assert info["converged"], info
        out = {"v0": H.vectors(0), "v1": H.vectors(1), "s0": H.sigma(0), "s1": H.sigma(1), "x": x}
        for lev in range(2):
            for i, a in enumerate(H.coarse_links(lev)):
                out[f"links{lev}_{i}"] = a
        return out
    finally:
        H.close()
        lat.close()


def test_reused_buffers_give_identical_results(crk):
    crk.release_cached_memory()
    assert crk.cached_memory_bytes() == 0
    first = _run(crk, -0.2, 201, 7)
    cached = crk.cached_memory_bytes()
    print("cached after the first hierarchy:", cached, flush=True)
    assert cached > 0
    # same shapes, other data: the cached buffers now hold this hierarchy's values
    _run(crk, -0.35, 202, 8)
    again = _run(crk, -0.2, 201, 7)
    for name, a in first.items():
        assert np.array_equal(a, again[name]), name


def test_rebuild_takes_cached_buffers_and_release_empties(crk):
    _run(crk, -0.2, 203, 9)
    before = crk.cached_memory_bytes()
    assert before > 0
    U = synth.gauge_field(DIMS, 0.3, 1, config=203)
    lat = crk.Lattice(DIMS, -0.2, 1.0)
    lat.load_gauge(U)
    H = crk.Hierarchy(lat, setup_form=crk.FORM_FP32, seed=9, **LEVELS)
    during = crk.cached_memory_bytes()
    print("cached before / while the rebuild lives:", before, during, flush=True)
    assert during < before
    H.close()
    lat.close()
    crk.release_cached_memory()
    assert crk.cached_memory_bytes() == 0
