"""Pins of the analytic field the surface-field study compares with (the
sphere's TM mode of degree 3 with angular part x y z / r^3): it is a Maxwell
eigenfield -- divergence-free and curl curl E = k^2 E (central differences)
-- and it is normal to the conducting wall r = R, with the symmetry of the
octant's conducting planes (tangential components odd across each plane)."""
import numpy as np

from paper_1301_3794_amd import studies


def curl(F, p, d=1e-4):
    J = np.zeros((3, 3))
    for b in range(3):
        e = np.zeros(3)
        e[b] = d
        J[:, b] = (F(p + e) - F(p - e)) / (2 * d)
    return np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]]), np.trace(J)


def test_tm3_field_is_a_maxwell_eigenfield():
    R = 0.45
    k0 = studies.tm_root(3, 4.5, 5.5) / R
    F = lambda p: studies.tm3_xyz_field(p, k0)[0]  # noqa: E731
    rng = np.random.default_rng(0)
    for _ in range(8):
        p = rng.uniform(0.05, 0.3, 3)
        E = F(p)
        _, div = curl(F, p)
        assert abs(div) <= 1e-5 * np.linalg.norm(E) * k0
        cc, _ = curl(lambda q: curl(F, q, 1e-3)[0], p, 1e-3)
        assert np.linalg.norm(cc - k0 * k0 * E) <= 2e-3 * k0 * k0 * np.linalg.norm(E)


def test_tm3_field_is_normal_on_the_wall_and_symmetric():
    R = 0.45
    k0 = studies.tm_root(3, 4.5, 5.5) / R
    d = studies.octant_directions(200)
    E = studies.tm3_xyz_field(R * d, k0)
    tang = E - np.sum(E * d, axis=1)[:, None] * d
    assert np.max(np.linalg.norm(tang, axis=1)) <= 1e-10 * np.max(np.linalg.norm(E, axis=1))
    # a conducting plane x = 0: E_y, E_z odd in x, E_x even
    p = np.array([[0.1, 0.2, 0.15]])
    m = p * np.array([[-1, 1, 1]])
    a, b = studies.tm3_xyz_field(p, k0)[0], studies.tm3_xyz_field(m, k0)[0]
    assert np.allclose([b[0], -b[1], -b[2]], a, rtol=1e-12)
