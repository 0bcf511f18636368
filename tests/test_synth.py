"""Checks of the seeded input generators (shapes, determinism, the RFF prior)."""
import numpy as np

import synth
from oracle import kernel as ok


def test_molecule_sizes_cover_n():
    rng = np.random.default_rng(0)
    s = synth.molecule_sizes(10000, rng)
    assert s.sum() == 10000
    assert s[:-1].min() >= 10 and s.max() <= 300


def test_problem_deterministic_and_shaped():
    a = synth.make_problem("c2", n=3000)
    b = synth.make_problem("c2", n=3000)
    np.testing.assert_array_equal(a.X, b.X)
    np.testing.assert_array_equal(a.y, b.y)
    assert a.X.shape == (3000, 48) and a.X.flags["C_CONTIGUOUS"]
    assert np.all(np.diff(a.mol) >= 0)
    c = synth.make_problem("c1")
    assert c.X.shape == (2048, 32) and c.noise == 1e-2
    v = synth.make_problem("c2", n=3000, cond_variant=True)
    np.testing.assert_allclose(v.ell, a.ell * np.sqrt(96.0))


def test_random_features_covariance_converges_to_kernel():
    # E[f(x) f(x')] = k(x, x') for the random-feature prior.  The expectation over the
    # Gaussian weights is taken exactly (E_w[f f'] = phi(x) . phi(x')), the one over
    # frequencies and phases by Monte Carlo over many independent feature draws.
    d = 3
    ell = np.array([0.8, 1.3, 2.0])
    X = np.array([[0.0, 0.0, 0.0], [0.4, -0.3, 0.9], [1.5, 0.2, -1.0]])
    for kind in (synth.MATERN52, synth.RBF):
        th = ok.Theta(ell, 1.0, 0.0, kind)
        Kref = ok.kernel(X, X, th)
        acc = np.zeros((3, 3))
        draws = 200
        rng = np.random.default_rng(1)
        for _ in range(draws):
            f = synth.RandomFeatures(d, ell, 1.0, kind, rng, D=512)
            phi = f.amp * np.cos(X @ f.omega.T + f.b)
            acc += phi @ phi.T
        np.testing.assert_allclose(acc / draws, Kref, atol=0.01)
