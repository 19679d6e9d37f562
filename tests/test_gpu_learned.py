"""GPU parity of the learned initial guess (BF16 MFMA network, features,
synthesis, Adam) against the FP64 oracle of ``oracle.learned`` / ``oracle.mlp``.

Tolerances. The GPU stores every matrix-product operand in BF16 and
accumulates in FP32; the oracle rounds the same operands to BF16 and
accumulates in FP64, so the two differ by FP32 accumulation error plus the
rare operand whose FP32 and FP64 values fall on different sides of a BF16
rounding boundary (one BF16 ulp, 2^-8 relative, in one term of a 512-term
sum): 2e-3 of the output scale. Against the unrounded FP64 network the
bound is the BF16 one, 3e-2. Features and synthesis are FP64 on both sides
with FP32 outputs (1e-5). Adam is compared on the same gradients (FP32
update arithmetic).
"""
import numpy as np
import pytest

import oracle
from oracle import learned as ol
from oracle import mlp as om
from paper_1905_01341_amd import bfm
from paper_1905_01341_amd import workload as wl

pytestmark = pytest.mark.gpu

SIZES = [174, 512, 512, 512, 81]


def flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params]).astype(np.float32)


def unflat(v):
    out, o = [], 0
    v = np.asarray(v, dtype=np.float64)
    for a, b in zip(SIZES[:-1], SIZES[1:]):
        W = v[o:o + a * b].reshape(a, b)
        o += a * b
        out.append((W, v[o:o + b].copy()))
        o += b
    assert o == v.size
    return out


def rnd_params(seed):
    rng = np.random.default_rng(seed)
    p = om.init(SIZES, seed=seed)
    p = [(W.astype(np.float32).astype(np.float64), (0.1 * rng.standard_normal(b.shape)).astype(np.float32).astype(np.float64))
         for W, b in p]
    return p


def rnd_norm(seed):
    rng = np.random.default_rng(seed)
    mx = 0.5 * rng.standard_normal(174)
    sx = rng.uniform(0.5, 2.0, 174)
    my = 0.3 * rng.standard_normal(81)
    sy = rng.uniform(0.2, 1.5, 81)
    return np.concatenate([mx, sx, my, sy]).astype(np.float32)


def split_norm(n):
    n = n.astype(np.float64)
    return n[:174], n[174:348], n[348:429], n[429:510]


def oracle_forward(params, norm, x, rnd):
    mx, sx, my, sy = split_norm(norm)
    y, _ = om.forward(params, (x.astype(np.float64) - mx) / sx, rnd=rnd)
    return y * sy + my


@pytest.fixture(scope="module")
def tiny():
    """A 12-bubble perturbed cluster (template mesh, level 3)."""
    cl = wl.cluster(12, 3, 12.0, 0.5, 1.0, 0.5, seed=5, perturb=0.05)
    phi = wl.smooth_phi(cl, 7)
    q = wl.smooth_phi(cl, 8, amp=0.3)
    s, n, _ = oracle.geometry(cl.xyz, cl.tri)
    nd = int(cl.vtx_off[1])
    tri0 = cl.tri[:int(cl.tri_off[1])]
    return cl, phi, q, s, nd, tri0


def _solver(cl, **kw):
    sv = bfm.Solver(**kw)
    sv.set_cluster(cl)
    return sv


@pytest.mark.parametrize("rows", [1, 150, 1000])
def test_forward_matches_oracle(tiny, rows):
    sv = _solver(tiny[0])
    params = rnd_params(3)
    norm = rnd_norm(4)
    sv.mlp_set_params(flat(params))
    sv.mlp_set_norm(norm)
    np.testing.assert_array_equal(sv.mlp_get_params(), flat(params))
    np.testing.assert_array_equal(sv.mlp_get_norm(), norm)
    x = (np.random.default_rng(rows).standard_normal((rows, 174)) * 1.5 + 0.2).astype(np.float32)
    y = sv.mlp_forward(x).astype(np.float64)
    yq = oracle_forward(params, norm, x, ol.bf16)
    y64 = oracle_forward(params, norm, x, None)
    scale = np.max(np.abs(yq - split_norm(norm)[2]))
    assert np.max(np.abs(y - yq)) <= 2e-3 * scale, np.max(np.abs(y - yq)) / scale
    assert np.max(np.abs(y - y64)) <= 3e-2 * scale


def test_gradient_matches_oracle(tiny):
    sv = _solver(tiny[0])
    params = rnd_params(5)
    norm = rnd_norm(6)
    sv.mlp_set_params(flat(params))
    sv.mlp_set_norm(norm)
    rng = np.random.default_rng(7)
    rows = 150
    x = rng.standard_normal((rows, 174)).astype(np.float32)
    t = rng.standard_normal((rows, 81)).astype(np.float32)
    g, loss = sv.mlp_gradient(x, t)
    mx, sx, my, sy = split_norm(norm)
    xs = (x - mx) / sx
    ts = (t - my) / sy
    lq = om.loss(params, xs, ts, rnd=ol.bf16)
    assert abs(loss - lq) <= 1e-3 * lq
    gq = om.backward(params, xs, ts, rnd=ol.bf16)
    g64 = om.backward(params, xs, ts)
    for k, ((gw, gb), (qw, qb), (ew, eb)) in enumerate(zip(unflat(g), gq, g64)):
        for a, q, e, name in ((gw, qw, ew, "W"), (gb, qb, eb, "b")):
            err = np.linalg.norm(a - q) / np.linalg.norm(q)
            assert err <= 5e-3, (k, name, err)
            assert np.linalg.norm(a - e) / np.linalg.norm(e) <= 3e-2, (k, name)


def test_adam_steps_match_oracle_on_gpu_gradients(tiny):
    sv = _solver(tiny[0])
    sv.mlp_set_params(flat(rnd_params(8)))
    sv.mlp_set_norm(rnd_norm(9))
    rng = np.random.default_rng(10)
    x = rng.standard_normal((64, 174)).astype(np.float32)
    t = rng.standard_normal((64, 81)).astype(np.float32)
    state = {}
    lr = 1e-3
    for step in range(2):
        p0 = sv.mlp_get_params()
        g, _ = sv.mlp_gradient(x, t)
        sv.mlp_adam_step(lr)
        p1 = sv.mlp_get_params().astype(np.float64)
        ref = flat(om.adam_step(unflat(p0), unflat(g), state, lr=lr)).astype(np.float64)
        np.testing.assert_allclose(p1, ref, rtol=0, atol=1e-7, err_msg=f"step {step}")
        assert np.max(np.abs(p1 - p0)) > 0.5 * lr


def test_features_match_oracle(tiny):
    cl, phi, q, s, nd, tri0 = tiny
    sv = _solver(cl)
    feat, targ = sv.mlp_features(phi, q)
    rf, rt = ol.features(cl.xyz, s, phi, cl.nb, nd, cl.dirs[:nd], tri0, q)
    np.testing.assert_allclose(feat, rf, rtol=1e-5, atol=1e-6 * np.max(np.abs(rf)))
    np.testing.assert_allclose(targ, rt, rtol=1e-5, atol=1e-6 * np.max(np.abs(rt)))
    f2, t2 = sv.mlp_features(phi)
    assert t2 is None
    np.testing.assert_array_equal(f2, feat)


def test_guess_synthesis_matches_oracle(tiny):
    cl, phi, q, s, nd, tri0 = tiny
    sv = _solver(cl)
    c = np.random.default_rng(11).standard_normal(81).astype(np.float32)
    p = [(np.zeros((a, b)), np.zeros(b)) for a, b in zip(SIZES[:-1], SIZES[1:])]
    p[-1] = (p[-1][0], c.astype(np.float64))
    sv.mlp_set_params(flat(p))
    norm = np.concatenate([np.zeros(174), np.ones(174), np.zeros(81), np.ones(81)]).astype(np.float32)
    sv.mlp_set_norm(norm)
    qg = sv.mlp_guess(phi)
    ref = ol.synthesize(np.tile(c.astype(np.float64), (cl.nb, 1)), cl.xyz, s, cl.nb, nd, cl.dirs[:nd], tri0)
    np.testing.assert_allclose(qg, ref, rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))


def test_errors_without_template_or_training(tiny):
    cl = tiny[0]
    sv = bfm.Solver()
    sv.set_mesh(cl.xyz, cl.tri, cl.vtx_off, cl.tri_off)
    with pytest.raises(bfm.BfmError):
        sv.mlp_features(tiny[1])  # no template
    sv2 = _solver(cl)
    with pytest.raises(bfm.BfmError):
        sv2.mlp_guess(tiny[1])  # untrained
    with pytest.raises(bfm.BfmError):
        sv2.mlp_fit(1)  # empty training set


def test_training_on_gpu_gives_a_useful_guess():
    """Train on solved states of a 30-bubble cluster, then solve an unseen
    state from the learned guess: the same solution, a guess whose error is
    at most half the zero guess's (measured: 0.40), and fewer GMRES
    iterations (measured: 70 or 71 against 72, runs differing in the order
    of the training's atomic reductions). The gain is small: the features
    see only a bubble's own shape and potential and its neighbours'
    positions, not the potentials of the other bubbles, so the collective
    part of q is left to GMRES. On the time-stepped 1000-bubble cluster the
    network's guess saves 0.3 iterations per solve, less than it costs, and
    the previous step's q saves 2.4."""
    import torch
    nb, side = 30, 28.0
    sv = bfm.Solver(gmres_tol=1e-10)
    states = [wl.cluster(nb, 3, side, 0.5, 1.0, 0.5, seed=100 + k, perturb=0.05) for k in range(25)]
    sv.set_cluster(states[0])
    dev = torch.device("cuda:0")
    for k, cl in enumerate(states):
        sv.set_positions(cl.xyz)
        phi = torch.from_numpy(wl.smooth_phi(cl, 200 + k)).to(dev)
        q = torch.zeros_like(phi)
        info = sv.solve_dev(phi, q)
        assert info["converged"]
        sv.mlp_collect_dev(phi, q)
    assert sv.mlp_dataset() == 25 * nb
    l_first = sv.mlp_fit(1, batch=50, lr=1e-3, seed=1)
    l_last = sv.mlp_fit(300, batch=50, lr=1e-3, seed=2)
    assert l_last < 0.1 * l_first, (l_first, l_last)
    test = wl.cluster(nb, 3, side, 0.5, 1.0, 0.5, seed=999, perturb=0.05)
    phi = wl.smooth_phi(test, 1999)
    sv.set_positions(test.xyz)
    q0, i0 = sv.solve(phi)
    qg = sv.mlp_guess(phi)
    q1, i1 = sv.solve(phi, learned=True)
    err = np.linalg.norm(qg - q0) / np.linalg.norm(q0)
    print(f"guess error {err:.3e}; iterations zero {i0['iterations']} learned {i1['iterations']}; "
          f"loss {l_first:.3e} -> {l_last:.3e}; guess {i1['t_guess_ms']:.3f} ms")
    assert i1["converged"] and i1["t_guess_ms"] > 0
    assert np.linalg.norm(q1 - q0) / np.linalg.norm(q0) < 1e-8
    assert err < 0.5
    assert i1["iterations"] < i0["iterations"]
