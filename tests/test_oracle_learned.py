"""Pins of the FP64 reference for the learned initial guess: harmonics
against quadrature orthonormality, textbook closed forms and scipy's complex
harmonics; the least-squares projector against exact reproduction and the
icosahedron's closed-form area; features on spheres (constant radius and
harmonic potentials give unit coefficient vectors); brute-force neighbour
order on a hand layout; BF16 rounding against hand values and torch's
conversion; the rounding hook of the MLP against the exact network where
all operands are representable."""
import math

import numpy as np
import pytest
import scipy.special
import torch

from oracle import learned, mlp
from paper_1905_01341_amd import workload


def _sphere_rule(nt=20, nphi=40):
    t, wt = np.polynomial.legendre.leggauss(nt)
    lon = np.arange(nphi) * 2 * np.pi / nphi
    T, L = np.meshgrid(t, lon, indexing="ij")
    st = np.sqrt(1 - T ** 2)
    dirs = np.stack([st * np.cos(L), st * np.sin(L), T], axis=-1).reshape(-1, 3)
    w = (wt[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    return dirs, w


def test_harmonics_orthonormal_under_exact_quadrature():
    dirs, w = _sphere_rule()
    Y = learned.real_sh(8, dirs)
    gram = Y.T @ (w[:, None] * Y)
    np.testing.assert_allclose(gram, np.eye(81), atol=1e-12)


def test_harmonics_low_degree_closed_forms():
    rng = np.random.default_rng(1)
    d = rng.standard_normal((17, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = learned.real_sh(2, d)
    c1 = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(Y[:, 0], 1 / math.sqrt(4 * math.pi), rtol=1e-14)
    np.testing.assert_allclose(Y[:, 1], c1 * d[:, 2], atol=1e-14)  # n=1, m=0
    np.testing.assert_allclose(Y[:, 2], c1 * d[:, 0], atol=1e-14)  # n=1, cos
    np.testing.assert_allclose(Y[:, 3], c1 * d[:, 1], atol=1e-14)  # n=1, sin
    np.testing.assert_allclose(Y[:, 4], math.sqrt(5 / (16 * math.pi)) * (3 * d[:, 2] ** 2 - 1), atol=1e-14)
    # n=2, m=2: sqrt(15/16pi) (x^2 - y^2) and sqrt(15/4pi) x y
    np.testing.assert_allclose(Y[:, 7], math.sqrt(15 / (16 * math.pi)) * (d[:, 0] ** 2 - d[:, 1] ** 2), atol=1e-14)
    np.testing.assert_allclose(Y[:, 8], math.sqrt(15 / (4 * math.pi)) * d[:, 0] * d[:, 1], atol=1e-14)


def test_harmonics_match_scipy_complex_harmonics():
    rng = np.random.default_rng(2)
    d = rng.standard_normal((31, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = learned.real_sh(8, d)
    theta = np.arccos(d[:, 2])
    lon = np.arctan2(d[:, 1], d[:, 0])
    for n in range(9):
        for m in range(n + 1):
            yc = scipy.special.sph_harm_y(n, m, theta, lon)  # includes (-1)^m
            if m == 0:
                np.testing.assert_allclose(Y[:, n * n], yc.real, atol=1e-12)
            else:
                np.testing.assert_allclose(Y[:, n * n + 2 * m - 1], math.sqrt(2) * (-1) ** m * yc.real, atol=1e-12)
                np.testing.assert_allclose(Y[:, n * n + 2 * m], math.sqrt(2) * (-1) ** m * yc.imag, atol=1e-12)


def test_template_weights_icosahedron_area():
    v, f = workload.icosphere(0)
    w = learned.template_weights(v, f)
    edge = np.linalg.norm(v[f[0, 0]] - v[f[0, 1]])
    assert abs(edge - 4 / math.sqrt(10 + 2 * math.sqrt(5))) < 1e-14
    np.testing.assert_allclose(w.sum(), 20 * math.sqrt(3) / 4 * edge ** 2, rtol=1e-14)
    np.testing.assert_allclose(w, w[0], rtol=1e-13)  # every vertex is alike


def test_projector_reproduces_band_limited_functions():
    v, f = workload.icosphere(3)
    G, Gp = learned.projector(v, f)
    rng = np.random.default_rng(3)
    c = rng.standard_normal(81)
    np.testing.assert_allclose(Gp @ (G @ c), c, atol=1e-11)
    np.testing.assert_allclose(Gp @ G, np.eye(81), atol=1e-11)


def _spheres(centres, radii, level=3):
    v, f = workload.icosphere(level)
    nd = v.shape[0]
    xyz = np.concatenate([c + r * v for c, r in zip(centres, radii)])
    s = np.zeros(len(xyz))
    for b in range(len(centres)):
        X = xyz[b * nd:(b + 1) * nd]
        for a, bb, cc in f:
            area = 0.5 * np.linalg.norm(np.cross(X[bb] - X[a], X[cc] - X[a]))
            s[b * nd + np.array([a, bb, cc])] += area / 3
    return xyz, s, v, f, nd


def test_features_of_spheres_are_unit_vectors():
    centres = np.array([[0.0, 0, 0], [5.0, 0, 0]])
    radii = np.array([1.0, 0.5])
    xyz, s, v, f, nd = _spheres(centres, radii)
    k = 6  # degree 2, m = 1, cos part
    phi = np.concatenate([learned.real_sh(8, v)[:, k], 0.3 * np.ones(nd)])
    q = np.concatenate([np.ones(nd), learned.real_sh(8, v)[:, 20]])
    feat, targ = learned.features(xyz, s, phi, 2, nd, v, f, q)
    assert feat.shape == (2, 174) and targ.shape == (2, 81)
    _, rad = learned.bubble_frames(xyz, s, 2, nd)
    for b in range(2):
        e0 = np.zeros(81)
        e0[0] = math.sqrt(4 * math.pi) * radii[b] / rad[b]
        np.testing.assert_allclose(feat[b, :81], e0, atol=1e-11)
    ek = np.zeros(81)
    ek[k] = 1.0
    np.testing.assert_allclose(feat[0, 81:162], ek, atol=1e-11)
    e0 = np.zeros(81)
    e0[0] = 0.3 * math.sqrt(4 * math.pi)
    np.testing.assert_allclose(feat[1, 81:162], e0, atol=1e-11)
    e0[0] = math.sqrt(4 * math.pi) * rad[0]
    np.testing.assert_allclose(targ[0], e0, atol=1e-11)
    e20 = np.zeros(81)
    e20[20] = rad[1]
    np.testing.assert_allclose(targ[1], e20, atol=1e-11)
    # only one other bubble: one offset, three zero slots
    np.testing.assert_allclose(feat[0, 162:165], (centres[1] - centres[0]) / rad[0], atol=1e-12)
    np.testing.assert_allclose(feat[1, 162:165], (centres[0] - centres[1]) / rad[1], atol=1e-12)
    assert np.all(feat[:, 165:] == 0)
    # synthesis inverts the target projection for band-limited q
    np.testing.assert_allclose(learned.synthesize(targ, xyz, s, 2, nd, v, f), q, atol=1e-11)


def test_neighbour_order_by_hand():
    x = np.array([0.0, 3.0, 7.0, 12.0, 20.0, 21.0, 1.5])
    cen = np.stack([x, np.zeros(7), np.zeros(7)], axis=1)
    rad = np.full(7, 2.0)
    off = learned.neighbour_offsets(cen, rad)
    # bubble 0 (x=0): 6 (1.5), 1 (3), 2 (7), 3 (12)
    np.testing.assert_allclose(off[0, 0::3], [0.75, 1.5, 3.5, 6.0])
    # bubble 6 (x=1.5): 0 and 1 tie at 1.5 -> lower index first; then 2 (5.5), 3 (10.5)
    np.testing.assert_allclose(off[6, 0::3], [-0.75, 0.75, 2.75, 5.25])
    # bubble 4 (x=20): 5 (1), 3 (8), 2 (13), 1 (17)
    np.testing.assert_allclose(off[4, 0::3], [0.5, -4.0, -6.5, -8.5])
    assert np.all(off[:, 1::3] == 0) and np.all(off[:, 2::3] == 0)


def test_bf16_rounding():
    one = 1.0
    assert learned.bf16(one) == 1.0
    assert learned.bf16(1 + 2 ** -8) == 1.0                  # tie -> even
    assert learned.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6      # tie -> even (up)
    assert learned.bf16(1 + 2 ** -8 + 2 ** -20) == 1 + 2 ** -7
    assert learned.bf16(-3.0) == -3.0
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-8, 8, 5000),
                        (1 + (2 * rng.integers(0, 128, 200) + 1) * 2 ** -8) * 2.0 ** rng.integers(-4, 4, 200)])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(learned.bf16(x), ref)


def test_rounding_hook_is_exact_on_representable_linear_layer():
    rng = np.random.default_rng(6)
    W = learned.bf16(rng.standard_normal((16, 8)))
    b = rng.standard_normal(8)
    x = learned.bf16(rng.standard_normal((4, 16)))
    y0, _ = mlp.forward([(W, b)], x)
    y1, _ = mlp.forward([(W, b)], x, rnd=learned.bf16)
    np.testing.assert_array_equal(y0, y1)
    # a hidden layer: the hook rounds the activations, the plain network does not
    params = [(W, b), (learned.bf16(rng.standard_normal((8, 3))), np.zeros(3))]
    ya, _ = mlp.forward(params, x)
    yb, _ = mlp.forward(params, x, rnd=learned.bf16)
    assert 0 < np.max(np.abs(ya - yb)) < 2e-2 * np.max(np.abs(ya))
    h = learned.bf16(mlp.silu(x @ W + b))
    np.testing.assert_allclose(yb, h @ params[1][0], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_rounded_backward_within_bf16_error_of_exact(k):
    """Operand rounding moves every gradient by at most a few BF16 ulps of
    the products it enters (relative 2^-8 per operand), and does move it."""
    rng = np.random.default_rng(10 + k)
    params = mlp.init([12, 32, 32, 5], seed=k)
    x = rng.standard_normal((16, 12))
    t = rng.standard_normal((16, 5))
    g0 = mlp.backward(params, x, t)
    g1 = mlp.backward(params, x, t, rnd=learned.bf16)
    moved = False
    for (a0, b0), (a1, b1) in zip(g0, g1):
        assert np.linalg.norm(a1 - a0) <= 3e-2 * np.linalg.norm(a0)
        assert np.linalg.norm(b1 - b0) <= 3e-2 * np.linalg.norm(b0)
        moved |= bool(np.any(a1 != a0))
    assert moved
