"""csvd_spmm_noalloc (the allocation-free variant of csvd_spmm, for callers
that cannot allocate device memory) against csvd_spmm through the C ABI:
bit-identical products on two calls in a row, the second with a smaller
input, no change in free device memory across calls once the first call on
the device has set up, and a clear refusal of inputs beyond its staging
limit."""
import ctypes as C

import numpy as np
import pytest

import paper_2109_13655_amd as cs
import synth

pytestmark = pytest.mark.gpu


def _free_device_bytes():
    """hipMemGetInfo of the HIP runtime the library runs on (already loaded
    under its soname once a context exists)."""
    hip = C.CDLL("libamdhip64.so.7")
    free, total = C.c_size_t(), C.c_size_t()
    assert hip.hipMemGetInfo(C.byref(free), C.byref(total)) == 0
    return free.value


def test_spmm_noalloc_matches_spmm():
    I = synth.random_sparse(3001, 1703, 7, config=80)
    print("[gpu-test] spmm_noalloc", I.m, I.n, flush=True)
    ctx = cs.csvd_create(I.m, I.n, I.rowptr, I.colidx, I.vals)
    try:
        rng = np.random.default_rng(31)
        X1 = rng.standard_normal((I.n, 64))
        ref1 = cs.csvd_spmm(ctx, 0, X1, I.m)
        # first call on the device: looks up the staging array's address
        got1 = cs.csvd_spmm_noalloc(ctx, 0, X1, I.m)
        # second call: smaller input, the transposed product
        X2 = rng.standard_normal((I.m, 5))
        got2 = cs.csvd_spmm_noalloc(ctx, 1, X2, I.n)
        ref2 = cs.csvd_spmm(ctx, 1, X2, I.n)
        assert np.array_equal(got1, ref1)
        assert np.array_equal(got2, ref2)
        # later calls leave the free device memory unchanged, and the larger
        # staging contents of a previous call do not leak into a smaller one
        free0 = _free_device_bytes()
        got3 = cs.csvd_spmm_noalloc(ctx, 0, X1[:, :3], I.m)
        got4 = cs.csvd_spmm_noalloc(ctx, 1, X2, I.n)
        free1 = _free_device_bytes()
        assert free1 == free0
        assert np.array_equal(got3, cs.csvd_spmm(ctx, 0, X1[:, :3], I.m))
        assert np.array_equal(got4, ref2)
        # beyond the staging limit: a clear error, and the context stays usable
        big = np.zeros((I.n, 1000))
        with pytest.raises(cs.CsvdError) as e:
            cs.csvd_spmm_noalloc(ctx, 0, big, I.m)
        assert e.value.code == cs.CSVD_EINVAL and "staging limit" in str(e.value)
        assert np.array_equal(cs.csvd_spmm_noalloc(ctx, 0, X1, I.m), ref1)
    finally:
        cs.csvd_destroy(ctx)
