"""Pins of the time-step oracle (oracle/step.py): Adams-Bashforth weights
by exactness on polynomials, filter identities (projector, symmetric,
identity when p_f^2 = N_d, reproduces band-limited data), exact polyhedron
volumes, one-ring order, paraboloid curvature exact on a planted quadric and
within 1% of 1/R on a sphere of 642 vertices, tangential velocity exact for
linear phi on a planar patch, the right-hand side on a sphere in closed form,
and the Rayleigh-Plesset equation for a spherical bubble."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from oracle import step as st
from paper_1905_01341_amd import workload as wl


def test_adams_bashforth_weights_are_exact_on_polynomials():
    for order in range(1, 7):
        w = st.adams_bashforth_weights(order)
        assert sum(w) == 1
        # integral over one step of t^k, k < order, reproduced exactly from the nodes 0, -1, ...
        for k in range(order):
            exact = Fraction(1, k + 1)  # int_0^1 t^k dt
            got = sum(wi * Fraction(-i) ** k for i, wi in enumerate(w))
            assert got == exact, (order, k)
    assert st.adams_bashforth_weights(2) == [Fraction(3, 2), Fraction(-1, 2)]


def test_filter_identities():
    v, f = wl.icosphere(3)
    F = st.filter_matrix(v, 9)
    np.testing.assert_allclose(F @ F, F, atol=1e-12)
    np.testing.assert_allclose(F, F.T, atol=1e-12)
    assert abs(np.trace(F) - 81) < 1e-9  # rank p_f^2
    # coordinates of a sphere are degree-1 harmonics: unchanged
    np.testing.assert_allclose(F @ (2.5 * v), 2.5 * v, atol=1e-12)
    # p_f^2 = N_d: identity
    rng = np.random.default_rng(0)
    d = rng.standard_normal((16, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    np.testing.assert_allclose(st.filter_matrix(d, 4), np.eye(16), atol=1e-10)


def test_volumes_of_polyhedra():
    oct_v = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    oct_f = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4], [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]])
    assert abs(st.volumes(oct_v, oct_f, [0, 8])[0] - 4.0 / 3.0) < 1e-15
    assert abs(st.volumes(oct_v + [3.0, -2.0, 7.0], oct_f, [0, 8])[0] - 4.0 / 3.0) < 1e-13
    v, f = wl.icosphere(0)
    edge = 4 / math.sqrt(10 + 2 * math.sqrt(5))
    ico = 5 * (3 + math.sqrt(5)) / 12 * edge ** 3
    assert abs(st.volumes(v, f, [0, 20])[0] - ico) < 1e-13


def test_one_ring_is_counter_clockwise_from_lowest():
    v, f = wl.icosphere(1)
    rings = st.one_ring(f, len(v))
    for j, ring in enumerate(rings):
        assert ring[0] == min(ring) and len(ring) in (5, 6)
        for a, b in zip(ring, ring[1:] + ring[:1]):
            assert np.dot(np.cross(v[a] - v[j], v[b] - v[j]), v[j]) > 0


def test_curvature_exact_on_planted_quadric_and_near_exact_on_sphere():
    # five neighbours on z = a x^2 + b x y + c y^2 with n = e_z at the vertex: H = -(a + c)
    a, b, c = 0.3, -0.2, 0.45
    pts = [(0.1, 0.02), (-0.05, 0.09), (-0.08, -0.07), (0.04, -0.1), (0.11, -0.03)]
    xyz = np.array([[0, 0, 0]] + [[x, y, a * x * x + b * x * y + c * y * y] for x, y in pts], float)
    n = np.zeros((6, 3))
    n[0, 2] = 1.0
    H = st.curvature(xyz, n, [[1, 2, 3, 4, 5]])
    assert abs(H[0] + (a + c)) < 1e-12
    v, f = wl.icosphere(3)
    R = 0.7
    s, nn, _ = oracle.geometry(R * v, f)
    H = st.curvature(R * v, nn, st.one_ring(f, len(v)))
    assert np.max(np.abs(H * R - 1.0)) < 0.01


def test_tangential_velocity_exact_for_linear_phi_on_a_plane():
    # planar grid z = 0 triangulated CCW seen from +z; phi = g . r
    m = 6
    xs, ys = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    xyz = np.stack([xs.ravel() * 0.3, ys.ravel() * 0.25, np.zeros(m * m)], axis=1)
    idx = lambda i, j: i * m + j
    tri = []
    for i in range(m - 1):
        for j in range(m - 1):
            tri += [(idx(i, j), idx(i + 1, j), idx(i + 1, j + 1)), (idx(i, j), idx(i + 1, j + 1), idx(i, j + 1))]
    tri = np.array(tri)
    g = np.array([0.7, -1.3, 2.0])
    phi = xyz @ g
    r = xyz
    area = 0.5 * np.linalg.norm(np.cross(r[tri[:, 1]] - r[tri[:, 0]], r[tri[:, 2]] - r[tri[:, 0]]), axis=1)
    s = np.zeros(len(r))
    for c in range(3):
        np.add.at(s, tri[:, c], area / 3)
    n = np.tile([0.0, 0.0, 1.0], (len(r), 1))
    vt = st.tangential_velocity(r, tri, phi, s, n, area)
    np.testing.assert_allclose(vt, np.tile([0.7, -1.3, 0.0], (len(r), 1)), atol=1e-13)


def _sphere_mesh(R=1.0, level=3, pf=0):
    v, f = wl.icosphere(level)
    mesh = st.make_mesh(f, [0, len(v)], [0, len(f)], v, pf)
    return R * v, mesh


def test_rhs_on_a_sphere_in_closed_form():
    R, c = 0.8, 0.35
    xyz, mesh = _sphere_mesh(R)
    phys = st.Physics(sigma=0.073, kappa=1.4, p0=1.0, pa=0.5, period=5.0, forcing_sign=1.0)
    V0, pg0 = st.initial_gas(mesh, phys, xyz * 1.02)  # gas set up at a larger sphere
    dx, dphi, q, H = st.rhs(mesh, phys, V0, pg0, 0.7, xyz, np.full(len(xyz), c))
    s, n, _ = oracle.geometry(xyz, mesh.tri)
    q_ref, _ = oracle.solve(xyz, mesh.tri, np.full(len(xyz), c), method="lu")
    np.testing.assert_allclose(q, q_ref, rtol=1e-12)
    np.testing.assert_allclose(dx, n * q[:, None], atol=1e-13)  # alpha = -1: u = n q
    V = st.volumes(xyz, mesh.tri, mesh.tri_off)[0]
    pg = pg0[0] * (V0[0] / V) ** 1.4
    expect = 0.5 * q ** 2 - (pg - 2 * 0.073 * H) + 1.0 + 0.5 * math.sin(2 * math.pi * 0.7 / 5.0)
    np.testing.assert_allclose(dphi, expect, atol=1e-12)


def test_spherical_bubble_follows_rayleigh_plesset():
    """A sphere with uniform phi stays a sphere: its equivalent radius obeys
    R R'' + 3/2 R'^2 = (p_g - 2 sigma / R - p_inf(t)) / rho with
    p_g = p_g0 (R0 / R)^(3 kappa), up to the mesh's discretisation error."""
    phys = st.Physics(sigma=0.073, kappa=1.4, p0=1.0, pa=0.5, period=5.0, forcing_sign=1.0, filter_degree=6)
    xyz, mesh = _sphere_mesh(1.0, pf=6)
    it = st.Integrator(mesh, phys, xyz, np.zeros(len(xyz)))
    R0 = (3 * it.V0[0] / (4 * math.pi)) ** (1 / 3)
    pg0 = it.pg0[0]
    dt = 0.02
    Rs = [R0]
    for _ in range(12):
        it.step(dt)
        Rs.append((3 * st.volumes(it.xyz, mesh.tri, mesh.tri_off)[0] / (4 * math.pi)) ** (1 / 3))

    def rp(t, y):
        R, Rd = y
        pg = pg0 * (R0 / R) ** (3 * 1.4)
        return [Rd, ((pg - 2 * 0.073 / R - phys.p_inf(t)) - 1.5 * Rd * Rd) / R]

    sol = solve_ivp(rp, (0, 12 * dt), [R0, 0.0], t_eval=np.arange(13) * dt, rtol=1e-11, atol=1e-13)
    dR = np.array(Rs) - R0
    dR_ref = sol.y[0] - R0
    assert np.max(np.abs(dR_ref)) > 1e-4  # the bubble moves
    assert np.max(np.abs(dR - dR_ref)) < 0.02 * np.max(np.abs(dR_ref))
