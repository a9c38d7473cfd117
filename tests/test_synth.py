"""The seeded input generators: recipe sizes and reproducibility (no GPU, no oracle)."""
import numpy as np

from paper_2603_09621_amd import synth


def test_batch_dims_follow_the_recipe():
    assert synth.batch_dims(0) == (96, 96, 96)
    assert synth.batch_dims(15) == (256, 256, 160)
    for j in range(16):
        nx, ny, nz = synth.batch_dims(j)
        assert nx == ny and nx % 8 == 0 and nz % 4 == 0
    assert [synth.batch_dims(j)[0] for j in range(16)] == sorted(synth.batch_dims(j)[0] for j in range(16))


def test_lattice_stride_is_the_coarsest_with_enough_sites():
    for shape, n in (((24, 96, 96), 221184), ((24, 96, 96), 50000), ((40, 256, 256), 139368), ((10, 30, 30), 7)):
        s = synth.lattice_stride(shape, n)
        nzl, ny, nx = shape
        assert s == 1 or (nx // s) * (ny // s) * nzl >= n
        assert (nx // (s + 1)) * (ny // (s + 1)) * nzl < n


def test_small_batch_workload_is_reproducible():
    a = synth.workload_batch(seed=9, nscans=3, n_range=(1e3, 5e3), workers=3)
    b = synth.workload_batch(seed=9, nscans=3, n_range=(1e3, 5e3), workers=1)
    assert len(a) == 3
    for (pa, la, da), (pb, lb, db) in zip(a, b):
        assert da == db and la.shape == (da[2] // 4, da[1], da[0])
        np.testing.assert_array_equal(la, lb)
        for k in pa:
            np.testing.assert_array_equal(pa[k], pb[k])
        assert 1e3 <= pa["amp"].shape[0] <= 5e3
