"""Pins on the synthetic workloads (G0 of the 2D lattice, Keldysh propagators)."""
import numpy as np

import workloads as W


def test_g0_equal_time_density_half_filling():
    # mu = 0 on the square lattice is particle-hole symmetric: density per spin 1/2
    assert abs(W.g0_lattice(0, 0, 0.0, W.Lattice(16, 1.0, 0.0, 4.0)) - 0.5) < 1e-14


def test_g0_antiperiodic_and_jump():
    lat = W.Lattice(32, 1.0, -0.5, 5.0)
    rng = np.random.default_rng(1)
    dx, dy = rng.integers(-31, 32, 20), rng.integers(-31, 32, 20)
    tau = rng.random(20) * lat.beta * 0.999 + 1e-3
    g = W.g0_lattice(dx, dy, tau, lat)
    g2 = W.g0_lattice(dx, dy, tau - lat.beta, lat)
    np.testing.assert_allclose(g2, -g, rtol=1e-12, atol=1e-15)
    # jump at tau = 0: G(0+) - G(0-) = -delta_{r,0}
    jp = W.g0_lattice(0, 0, 1e-13, lat) - W.g0_lattice(0, 0, 0.0, lat)
    jq = W.g0_lattice(3, 1, 1e-13, lat) - W.g0_lattice(3, 1, 0.0, lat)
    assert abs(jp + 1.0) < 1e-9 and abs(jq) < 1e-9


def test_g0_lattice_symmetry():
    lat = W.Lattice(16, 1.0, 0.3, 4.0)
    tau = 1.3
    g = W.g0_lattice(2, 5, tau, lat)
    for dx, dy in ((5, 2), (-2, 5), (2, -5), (14, 11)):
        assert abs(W.g0_lattice(dx, dy, tau, lat) - g) < 1e-14


def test_g0_matches_plain_momentum_sum():
    lat = W.Lattice(8, 1.0, -0.4, 3.0)
    k = 2 * np.pi * np.arange(8) / 8
    for dx, dy, tau in ((1, 2, 0.7), (0, 3, -1.1), (4, 4, 2.9)):
        tot = 0.0
        for kx in k:
            for ky in k:
                xi = -2 * (np.cos(kx) + np.cos(ky)) - lat.mu
                nf = 1 / (np.exp(lat.beta * xi) + 1)
                w = -(1 - nf) if tau > 0 else nf
                tot += np.cos(kx * dx + ky * dy) * np.exp(-xi * tau) * w
        assert abs(W.g0_lattice(dx, dy, tau, lat) - tot / 64) < 1e-14


def test_lattice_batch_shapes_and_seed():
    A = W.lattice_batch(4, 8)
    B = W.lattice_batch(4, 8)
    assert A.shape == (4, 8, 8) and A.dtype == np.float64
    np.testing.assert_array_equal(A, B)
    np.testing.assert_allclose(np.diagonal(A, axis1=1, axis2=2), 0.5, atol=1e-14)


def test_keldysh_largest_time_invariance():
    """Flipping the branch of the globally latest vertex leaves every entry unchanged."""
    t, br = W.keldysh_config(3, 6, seed=9)
    M = W.keldysh_batch(3, 6, seed=9)
    for b in range(3):
        i = int(np.argmax(t[b]))
        # rebuild with the flipped branch through the same formulas
        eps, n0 = 0.5, 0.3
        br2 = br[b].copy()
        br2[i] ^= 1
        dt = t[b][:, None] - t[b][None, :]
        ph = np.exp(-1j * eps * dt)
        gg, gl = -1j * (1 - n0) * ph, 1j * n0 * ph
        M2 = np.empty((6, 6), complex)
        for p in range(6):
            for q in range(6):
                a, c = br2[p], br2[q]
                if a == 0 and c == 0:
                    M2[p, q] = gg[p, q] if dt[p, q] > 0 else gl[p, q]
                elif a == 1 and c == 1:
                    M2[p, q] = gg[p, q] if dt[p, q] < 0 else gl[p, q]
                elif a == 0:
                    M2[p, q] = gl[p, q]
                else:
                    M2[p, q] = gg[p, q]
        np.testing.assert_array_equal(M2, M[b])


def test_stress_injection_makes_tiny_ratio():
    A = W.lattice_batch(128, 10, W.Lattice(32, 1.0, -0.5, 5.0), seed=3)
    A2, log = W.inject_stress(A, every=64)
    assert len(log) == 2
    b, kind, (l, r) = log[1]
    assert kind == "pivot"
    s = np.abs(A[b]).max()
    ratio = np.linalg.det(A2[b][np.ix_(list(r) + [l], list(r) + [l])]) / np.linalg.det(A2[b][np.ix_(r, r)])
    assert abs(ratio - 1e-12 * s) < 1e-13 * s


def test_keldysh_block_restricts_to_branch_matrices():
    """Keeping row 2i + alpha_i of every block gives the matrix of branch assignment alpha
    (same times for the same seed)."""
    import numpy as np
    import workloads as W
    blk = W.keldysh_block(5, 7, seed=31)
    mats = W.keldysh_batch(5, 7, seed=31)
    _, br = W.keldysh_config(5, 7, seed=31)
    for b in range(5):
        r = [2 * i + int(br[b, i]) for i in range(7)]
        np.testing.assert_array_equal(blk[b][np.ix_(r, r)], mats[b])
