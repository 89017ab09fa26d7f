"""Seeded input generators: SU(3) properties, reproducibility, exactness of
the closed-form matrix exponential."""
import numpy as np
import pytest

from paper_2303_08609_amd import inputs


def _expi_eigh(q):
    w, v = np.linalg.eigh(q)
    return (v * np.exp(1j * w)[:, None, :]) @ np.conj(np.swapaxes(v, 1, 2))


def test_expi_matches_eigendecomposition():
    g = inputs.rng(7)
    for eps in (0.0, 1e-9, 0.3, 0.7, 2.0):
        q = eps * inputs.gen_traceless_hermitian(g, 4000)
        got = inputs._expi_traceless_hermitian(q.copy())
        assert np.abs(got - _expi_eigh(q)).max() < 1e-13


def test_expi_degenerate_and_negative_det():
    # Q with a doubly degenerate spectrum, c0 < 0 and c0 > 0, and Q = 0.
    qs = np.array([np.diag([1.0, 1.0, -2.0]), np.diag([-1.0, -1.0, 2.0]),
                   np.zeros((3, 3)), np.diag([0.5, -0.5, 0.0])], dtype=np.complex128)
    got = inputs._expi_traceless_hermitian(qs.copy())
    want = np.array([np.diag(np.exp(1j * np.diag(q).real)) for q in qs])
    assert np.abs(got - want).max() < 1e-13


def test_gauge_is_su3_and_reproducible():
    dims = (4, 2, 2, 4)
    u = inputs.gen_gauge(dims, 0.5, 123)
    assert u.shape == (4, 4, 2, 2, 4, 3, 3)
    uu = u.reshape(-1, 3, 3)
    eye = np.eye(3)
    assert np.abs(uu @ np.conj(np.swapaxes(uu, 1, 2)) - eye).max() < 1e-14
    assert np.abs(np.linalg.det(uu) - 1).max() < 1e-14
    assert np.array_equal(u, inputs.gen_gauge(dims, 0.5, 123))
    assert not np.array_equal(u, inputs.gen_gauge(dims, 0.5, 124))


def test_gauge_chunking_does_not_change_values():
    a = inputs.gen_su3_near_unit(inputs.rng(5), 1000, 0.7, chunk=1000)
    b = inputs.gen_su3_near_unit(inputs.rng(5), 1000, 0.7, chunk=333)
    assert np.array_equal(a, b)


def test_gauge_eps_controls_distance_from_unit():
    d = {}
    for eps in (0.1, 0.5):
        u = inputs.gen_su3_near_unit(inputs.rng(1), 2000, eps)
        d[eps] = np.mean(np.abs(u - np.eye(3)))
    assert d[0.1] < d[0.5]
    assert d[0.1] < 0.2


def test_spinor_shapes_and_seed():
    s = inputs.gen_spinor_half((4, 4, 4, 4), 202)
    assert s.shape == (4, 4, 4, 2, 4, 3) and s.dtype == np.complex128
    s2 = inputs.gen_spinor_half((4, 4, 4, 4), 202, nrhs=3)
    assert s2.shape == (3, 4, 4, 4, 2, 4, 3)
    assert abs(np.mean(np.abs(s) ** 2) - 2.0) < 0.3


def test_point_noise_sources():
    b = inputs.gen_point_noise_sources((4, 4, 4, 4), 406)
    assert b.shape == (12, 4, 4, 4, 2, 4, 3)
    for k in range(12):
        assert abs(b[k, 0, 0, 0, 0, k // 3, k % 3] - 1.0) < 0.5
        noise = b[k].copy()
        noise[0, 0, 0, 0, k // 3, k % 3] = 0
        assert 0.5 < np.linalg.norm(noise) < 1.5


def test_random_su3_transform():
    om = inputs.gen_su3_random((2, 2, 2, 2), 9).reshape(-1, 3, 3)
    assert np.abs(om @ np.conj(np.swapaxes(om, 1, 2)) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(om) - 1).max() < 1e-13


@pytest.mark.parametrize("dims", [(3, 4, 4, 4), (4, 4, 4, 0), (4, 4, 4)])
def test_bad_dims_rejected(dims):
    with pytest.raises(ValueError):
        inputs.check_dims(dims)
