"""Pins of the oracle's quadtree identity topology (Fig. 2, Sec. 3.3, Sec. 4.2):
level sizes and per-level strengths against the paper's printed geometric
means, exact marginals where the factor graph is a tree, the dense linear
solve and the Gauss-Newton fixed point of the quadtree model (oracle/dense.py,
an independent NumPy assembly), and the consensus speed-up over the grid that
the paper reports."""

import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def K_of(cam):
    return (cam.fx, cam.fy, cam.cx, cam.cy)


def make(p, topology=oracle.TOPO_QUADTREE, **kw):
    o = oracle.Oracle(oracle.config_for_camera(p["cam"], topology=topology, **kw))
    o.set_keyframe(p["I_s"], p["normals_s"])
    o.set_frame(p["I_t"])
    return o


def problem(p, **kw):
    cam = p["cam"]
    return dense.Problem(cam.H, cam.W, K_of(cam), p["I_s"], p["I_t"], p["normals_s"], topology="quadtree", **kw)


def perturbed_state(o, seed):
    pix, nodes = o.get_state()
    rng = np.random.default_rng(seed)
    pix[..., :6] = rng.normal(0, 0.003, pix[..., :6].shape)
    pix[..., 6] += rng.normal(0, 0.05, pix[..., 6].shape)
    nodes[:, :6] = rng.normal(0, 0.003, nodes[:, :6].shape)
    o.set_state((pix, nodes))
    return pix, nodes


def test_levels_and_strengths_reproduce_the_papers_geometric_means():
    with open(os.path.join(GOLDEN, "quadtree_strengths.json")) as f:
        g = json.load(f)
    H, W = g["resolution"]
    levels = dense.quadtree_levels(H, W)
    assert len(levels) == 8 and levels[-1] == (1, 1)
    for name in ("sigma_P", "sigma_R"):
        s = dense.level_sigmas(g["leaf"][name], len(levels))
        gm = math.exp(np.mean(np.log(s)))
        printed = g["geometric_mean"][name]
        assert float(f"{gm:.{g['printed_digits']}g}") == printed
    # the oracle builds the same levels, also for odd sizes, a single row and VGA
    for (h, w) in [(128, 128), (5, 6), (1, 10), (7, 3), (480, 640)]:
        o = oracle.Oracle(oracle.default_config(H=h, W=w, cx=w / 2, cy=h / 2, topology=oracle.TOPO_QUADTREE))
        assert o.tree_levels() == dense.quadtree_levels(h, w)
        o.close()
    assert len(dense.quadtree_levels(480, 640)) == 11


def test_tree_marginals_are_exact_after_the_diameter():
    # without normal-integration factors the quadtree model is a tree: linear
    # GBP gives the exact marginals (means and covariances) of every pixel and
    # node once messages have crossed its diameter (pixel - root - pixel)
    p = synth.tiny_pair(3, H=5, W=6, lattice_px=2.0)
    kw = dict(sigma_P=1e-2, sigma_R=1e-2, sigma_N=float("inf"))
    o = make(p, init_inv_depth=0.4, frozen=1, **kw)
    pix, nodes = perturbed_state(o, 0)
    prob = problem(p, **kw)
    L, h, nv = prob.assemble(pix[..., :6].reshape(-1, 6), pix[..., 6].reshape(-1), nodes[:, :6])
    assert nv > 0
    S = np.linalg.inv(L)
    mu = S @ h
    diameter = 2 * (len(prob.levels) - 1)
    o.iterate(diameter)
    lam, eta = o.beliefs()
    lam, eta = lam.reshape(-1, 7, 7), eta.reshape(-1, 7)
    for i in range(30):
        Si = S[7 * i:7 * i + 7, 7 * i:7 * i + 7]
        np.testing.assert_allclose(np.linalg.inv(lam[i]), Si, atol=1e-12 * np.abs(Si).max())
        np.testing.assert_allclose(np.linalg.solve(lam[i], eta[i]), mu[7 * i:7 * i + 7], atol=1e-12 * np.abs(mu).max())
    nl, ne = o.node_beliefs()
    assert nl.shape[0] == prob.NT == 14
    for k in range(prob.NT):
        a = 7 * 30 + 6 * k
        Sk = S[a:a + 6, a:a + 6]
        np.testing.assert_allclose(np.linalg.inv(nl[k][:6, :6]), Sk, atol=1e-12 * np.abs(Sk).max())
        np.testing.assert_allclose(np.linalg.solve(nl[k][:6, :6], ne[k][:6]), mu[a:a + 6], atol=1e-12 * np.abs(mu).max())
        assert np.all(nl[k][6, :6] == 0.0) and ne[k][6] == 0.0
    # one iteration short of the diameter the pixel covariances are not yet exact
    o2 = make(p, init_inv_depth=0.4, frozen=1, **kw)
    o2.set_state((pix, nodes))
    o2.iterate(diameter - 1)
    lam2 = o2.beliefs()[0].reshape(-1, 7, 7)
    err = max(np.abs(np.linalg.inv(lam2[i]) - S[7 * i:7 * i + 7, 7 * i:7 * i + 7]).max() for i in range(30))
    assert err > 1e-8 * np.abs(S).max()


@pytest.mark.parametrize("seed", [3, 4])
def test_frozen_quadtree_means_equal_dense_solve(seed):
    # with normal-integration factors the graph has loops; converged linear
    # GBP means are still the exact solution
    p = synth.tiny_pair(seed, H=5, W=6, lattice_px=2.0)
    kw = dict(sigma_P=1e-2, sigma_R=1e-2, sigma_N=1e-2)
    o = make(p, init_inv_depth=0.4, frozen=1, **kw)
    pix, nodes = perturbed_state(o, seed)
    dp, dn = problem(p, **kw).solve_tree(pix[..., :6].reshape(-1, 6), pix[..., 6].reshape(-1), nodes[:, :6])
    o.iterate(300)
    m = o.means().reshape(-1, 7)
    np.testing.assert_allclose(m, dp, rtol=0, atol=1e-12 * np.abs(dp).max())


@pytest.mark.parametrize("huber_k", [400.0, 1.0])
def test_relinearised_quadtree_fixed_point_equals_gauss_newton(huber_k):
    p = synth.tiny_pair(3, H=5, W=6, lattice_px=2.0, rotvec=[0, 0, 0], trans=[0.0, 0.0, -0.05])
    # the prior is centred on the true motion: the upper-level priors, up to
    # 8x stronger, would otherwise hold the pose where some warps leave the
    # image and the valid set would flip between iterations
    xi_t = oracle.se3_log(p["T_ts"])
    kw = dict(sigma_P=1e-1, sigma_R=1e-2, sigma_N=1e-2, sigma_D=2e-2, huber_k=huber_k, prior_xi=xi_t)
    o = make(p, init_inv_depth=0.4, **kw)
    prob = problem(p, **kw)
    pix0, nodes0 = o.get_state()
    tau, ell, ntau = prob.gauss_newton_tree(pix0[..., :6].reshape(-1, 6), pix0[..., 6].reshape(-1),
                                            nodes0[:, :6], 30)
    L, h, nv = prob.assemble(tau, ell, ntau)
    assert nv == 30 and np.abs(h).max() < 1e-5
    o.iterate(1500)
    assert np.abs(o.means()).max() < 1e-7
    pix, nodes = o.get_state()
    np.testing.assert_allclose(pix[..., :6].reshape(-1, 6), tau, atol=5e-8)
    np.testing.assert_allclose(pix[..., 6].reshape(-1), ell, atol=5e-8)
    np.testing.assert_allclose(nodes[:, :6], ntau, atol=5e-8)
    # the quadtree energy is finite there and is not lowered by a step away
    E = o.energy()
    assert np.isfinite(E) and E > 0
    pix2 = pix.copy()
    pix2[..., 5] += 1e-3
    o.set_state((pix2, nodes))
    assert o.energy() > E


def test_quadtree_reaches_consensus_far_sooner_than_the_grid():
    # App. B.1: the loopy grid needs at least 50x more iterations than the
    # hierarchy. Linear model at the paper's identity strength: the quadtree's
    # pose estimate (mean of the pixel poses) is exact to 1e-4 within a few
    # tree diameters; the grid's is still more than 10% off after 50x as many
    p = synth.tiny_pair(3, H=8, W=8, lattice_px=2.0)
    cam = p["cam"]
    kw = dict(sigma_P=1e-1, sigma_R=4e-4, sigma_N=1e-3)
    errs = {}
    for topo, iters in ((oracle.TOPO_QUADTREE, 20), (oracle.TOPO_GRID, 1000)):
        o = make(p, topology=topo, init_inv_depth=0.4, frozen=1, **kw)
        st = o.get_state()
        if topo == oracle.TOPO_GRID:
            prob = dense.Problem(cam.H, cam.W, K_of(cam), p["I_s"], p["I_t"], p["normals_s"], **kw)
            ref = prob.solve_linear(st[..., :6].reshape(-1, 6), st[..., 6].reshape(-1))
        else:
            ref, _ = problem(p, **kw).solve_tree(st[0][..., :6].reshape(-1, 6), st[0][..., 6].reshape(-1),
                                                 st[1][:, :6])
        xi_ref = ref[:, :6].mean(0)
        o.iterate(iters)
        xi = o.means().reshape(-1, 7)[:, :6].mean(0)
        errs[topo] = np.abs(xi - xi_ref).max() / np.abs(xi_ref).max()
    assert errs[oracle.TOPO_QUADTREE] < 1e-4
    assert errs[oracle.TOPO_GRID] > 0.1


def test_quadtree_state_roundtrip_and_keyframe_reset():
    p = synth.tiny_pair(2, H=5, W=6, lattice_px=2.0)
    o = make(p, init_inv_depth=0.4, sigma_P=1e-1)
    o.iterate(5)
    pix, nodes = o.get_state()
    assert pix.shape == (5, 6, 42) and nodes.shape == (14, 141)
    assert np.abs(nodes[:, 6:]).max() > 0 and np.abs(pix[..., 7:34]).max() > 0
    # the root has no parent; nodes of level 1 over the odd last row/column
    # miss children
    assert np.all(nodes[-1, 6:33] == 0)
    o2 = make(p, init_inv_depth=0.4, sigma_P=1e-1)
    o2.set_state((pix, nodes))
    p2, n2 = o2.get_state()
    assert np.array_equal(p2, pix) and np.array_equal(n2, nodes)
    o.iterate(1)
    o2.iterate(1)
    assert np.array_equal(o.get_state()[0], o2.get_state()[0])
    ell = o.get_state()[0][..., 6].copy()
    o.set_keyframe(p["I_s"], p["normals_s"])
    p3, n3 = o.get_state()
    # a keyframe resets poses and messages at every level and keeps log-depths
    assert np.all(n3 == 0) and np.all(p3[..., :6] == 0) and np.all(p3[..., 7:] == 0)
    np.testing.assert_array_equal(p3[..., 6], ell)
