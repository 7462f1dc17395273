"""Shape and structure checks of the seeded synthetic inputs."""
import numpy as np
import pytest

from paper_1304_5583_amd import datagen


@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_config_shapes_and_partition(cfg):
    p = datagen.make_config(cfg)
    m, n = {1: (100, 200), 2: (500, 2000), 3: (2016, 2432)}[cfg]
    t = {1: 1, 2: 4, 3: 16}[cfg]
    assert p.M.shape == (m, n) and p.M.dtype == np.float64
    assert p.t == t and p.offsets[0] == 0 and p.offsets[-1] == n
    assert np.all(np.diff(p.offsets) > 0)
    assert np.array_equal(np.sort(p.perm), np.arange(n))
    assert p.perm.dtype == np.int32 and p.offsets.dtype == np.int32
    if cfg == 3:
        w = np.diff(p.offsets)
        assert w.min() >= 100 and w.max() <= 200
        assert p.M.min() >= 0.0 and p.M.max() <= 1.0
    if cfg == 2:
        norms = np.linalg.norm(p.M, axis=0)
        clean = ~p.outliers
        assert np.allclose(norms[clean], 1.0)
        assert p.outliers.sum() == 100
    if cfg == 1:
        assert (p.labels == -1).sum() == 20


def test_config_is_seeded():
    a = datagen.make_config(1)
    b = datagen.make_config(1)
    c = datagen.make_config(1, trial=1)
    assert np.array_equal(a.M, b.M)
    assert not np.array_equal(a.M, c.M)


def test_uneven_partition_bounds():
    rng = np.random.default_rng(0)
    perm, off = datagen.uneven_partition(rng, 2432, 16, 100, 200)
    w = np.diff(off)
    assert w.sum() == 2432 and w.min() >= 100 and w.max() <= 200
    with pytest.raises(ValueError):
        datagen.uneven_partition(rng, 100, 16, 100, 200)


def test_orthonormal_basis():
    rng = np.random.default_rng(1)
    U = datagen.orthonormal_basis(rng, 50, 7)
    assert np.allclose(U.T @ U, np.eye(7), atol=1e-13)
