"""The synthetic planets the benchmark and the tests run on: the full-size
three-layer planet has the shape its workload names (counts by brute force on
the CPU), positive orientation, the volume of the unit ball and the fluid
shell's volume fraction; generation is reproducible from the seed."""
import numpy as np

import planetgen as pg


def _signed_volumes(x, t):
    e1, e2, e3 = (x[t[:, k]] - x[t[:, 0]] for k in (1, 2, 3))
    return np.einsum("ij,ij->i", np.cross(e1, e2), e3) / 6.0


def test_three_layer_planet_full_size_shape():
    """384,000 tetrahedra; P2 displacement nodes (vertices, one per edge, a solid
    and a fluid copy on the fluid-solid interfaces) 544,597, so 1,633,791 DOF;
    P1 pressure DOF (vertices of fluid tetrahedra) 11,824; every tetrahedron
    positively oriented; total volume within 0.2 % of 4 pi / 3 (a polyhedral
    sphere lies inside it); fluid shell 0.19 < r < 0.55 within 0.5 % of
    0.55^3 - 0.19^3 of the volume."""
    d = pg.three_layer_planet(n_half=20)
    x, t, reg = np.asarray(d["xyz"]), np.asarray(d["tet"]), np.asarray(d["region"])
    assert t.shape == (384000, 4)
    vol = _signed_volumes(x, t)
    assert vol.min() > 0
    assert abs(vol.sum() / (4 * np.pi / 3) - 1) < 2e-3
    frac = vol[reg == 1].sum() / vol.sum()
    assert abs(frac / (0.55 ** 3 - 0.19 ** 3) - 1) < 5e-3
    V = len(x)
    pairs = np.array([(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)])
    e = np.sort(t[:, pairs], axis=2).reshape(-1, 2).astype(np.int64)
    uk, inv = np.unique(e[:, 0] * V + e[:, 1], return_inverse=True)
    nodes = np.concatenate([t, V + inv.reshape(-1, 6)], axis=1)
    solid = np.zeros(V + len(uk), bool)
    fluid = np.zeros(V + len(uk), bool)
    solid[nodes[reg == 0].ravel()] = True
    fluid[nodes[reg == 1].ravel()] = True
    assert solid.sum() + fluid.sum() == 544597
    pres = np.zeros(V, bool)
    pres[t[reg == 1].ravel()] = True
    assert pres.sum() == 11824


def test_generation_is_seeded():
    a = pg.three_layer_planet(n_half=4, seed=3)
    b = pg.three_layer_planet(n_half=4, seed=3)
    c = pg.three_layer_planet(n_half=4, seed=4)
    for k in ("xyz", "tet", "region", "rho", "lam", "mu"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
    assert not np.array_equal(np.asarray(a["xyz"]), np.asarray(c["xyz"]))
