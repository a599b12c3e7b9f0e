"""crk_dirac_apply_noalloc (the entry point for callers that cannot allocate)
against crk_dirac_apply, through the C ABI.

Both run the same kernels on the same staged data, so the results must be
bitwise equal; the second call of each pair uses a smaller input, which must
not see anything the first call left in the shared scratch array.
"""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def crk():
    import paper_2502_03091_amd as m
    m.lib()
    return m


def _lattice(crk, dims, config):
    lib = crk.lib()
    h = C.c_void_p()
    d = (C.c_int32 * 4)(*dims)
    assert lib.crk_create_lattice(d, -0.3, 1.7, C.byref(h)) == crk.OK
    U = np.ascontiguousarray(synth.gauge_field(dims, 0.4, 1, config=config))
    assert lib.crk_load_gauge(h, U.ctypes.data, U.size * 2) == crk.OK
    return h


def _apply(crk, fn, h, form, psi):
    out = np.empty_like(psi)
    rc = fn(h, int(form), psi.ctypes.data, out.ctypes.data, psi.shape[0])
    assert rc == crk.OK, crk.lib().crk_last_error()
    return out


@pytest.mark.parametrize("form", [0, 1, 2])
def test_noalloc_matches_allocating_entry_point(crk, form):
    lib = crk.lib()
    dims = [8, 8, 8, 8]
    V = int(np.prod(dims))
    h = _lattice(crk, dims, config=301)
    try:
        for nrhs in (6, 2):  # second call smaller than the first
            psi = np.ascontiguousarray(synth.gaussian_rhs(nrhs, V, config=302, index=nrhs))
            print(f"no-alloc dslash form={form} nrhs={nrhs}", flush=True)
            ref = _apply(crk, lib.crk_dirac_apply, h, form, psi)
            got = _apply(crk, lib.crk_dirac_apply_noalloc, h, form, psi)
            assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), np.abs(got - ref).max()
    finally:
        lib.crk_lattice_destroy(h)


def test_noalloc_smaller_lattice_after_larger(crk):
    """A second lattice of smaller volume after a larger one: the staged ranges
    of the two calls start at the same address and overlap."""
    lib = crk.lib()
    out = []
    for dims, nrhs in (([8, 8, 8, 16], 3), ([4, 4, 6, 4], 2)):
        V = int(np.prod(dims))
        h = _lattice(crk, dims, config=303)
        try:
            psi = np.ascontiguousarray(synth.gaussian_rhs(nrhs, V, config=304))
            ref = _apply(crk, lib.crk_dirac_apply, h, 1, psi)
            got = _apply(crk, lib.crk_dirac_apply_noalloc, h, 1, psi)
            assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
            out.append(got)
        finally:
            lib.crk_lattice_destroy(h)


def test_noalloc_rejects_calls_beyond_the_scratch_array(crk):
    lib = crk.lib()
    cap = int(lib.crk_dirac_apply_noalloc_max_bytes())
    assert cap == 64 << 20
    dims = [16, 16, 16, 16]
    V = int(np.prod(dims))
    h = _lattice(crk, dims, config=305)
    try:
        nrhs = cap // (16 * 12 * V) + 1  # the complex128 staging alone exceeds the array
        psi = np.zeros((nrhs, V, 12), dtype=np.complex128)
        out = np.full_like(psi, 7.0)
        rc = lib.crk_dirac_apply_noalloc(h, 1, psi.ctypes.data, out.ctypes.data, nrhs)
        assert rc == crk.EINVAL
        assert b"scratch" in lib.crk_last_error()
        assert (out == 7.0).all()  # nothing was written
        # one right-hand side fits and still works
        psi1 = np.ascontiguousarray(synth.gaussian_rhs(1, V, config=306))
        ref = _apply(crk, lib.crk_dirac_apply, h, 1, psi1)
        got = _apply(crk, lib.crk_dirac_apply_noalloc, h, 1, psi1)
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
    finally:
        lib.crk_lattice_destroy(h)
