"""Pins of the oracle's message transport and message damping.

Sec. 4.1 keeps only variables and factor-to-variable messages between
iterations; after every relinearisation the stored messages are carried into
the tangent space at the new linearisation point, to first order
(eta <- eta - Lambda m, Lambda unchanged). What the mathematics fixes:

- On a problem that is linear in the tangent coordinates, relinearising at the
  mean is only a change of coordinates, and the first-order transport is then
  exact. Relinearised GBP must reproduce frozen-linearisation GBP's means
  iteration by iteration, to rounding.
- On a smooth nonlinear problem whose solution lies a distance eps from the
  start, the two runs differ by O(eps^2). A missing or wrong transport leaves
  an O(eps) error, so halving eps no longer quarters the difference.
- Damping mixes each new message with the message it replaces, and it does not
  move the fixed point: frozen damped GBP still converges to the dense
  normal-equation solve.

Variants of the oracle built with a planted transport fault (no transport,
identity-factor slots only, the replaced message's information) must fail the
transport pins; they are built into a temporary folder and never shipped.
"""

import math

import numpy as np
import pytest

import oracle
import synth
from oracle import build as obuild
from oracle import dense

PLANTED = {1: "no transport", 2: "identity slots only", 3: "replaced message's information"}


@pytest.fixture(scope="module")
def planted(tmp_path_factory):
    d = tmp_path_factory.mktemp("planted_oracle")
    libs = {}
    for k in PLANTED:
        path = obuild.build(out=str(d / f"liboracle_fault{k}.so"), defines=[f"OR_PLANTED_FAULT={k}"])
        libs[k] = oracle.load(path)
    return libs


def _tilted_normals(H, W, n=(0.3, -0.2, -1.0)):
    n = np.asarray(n, dtype=np.float64)
    n /= np.linalg.norm(n)
    return np.broadcast_to(n, (H, W, 3)).astype(np.float32).copy()


# --- linear in the tangent coordinates: exact ----------------------------------------

def _linear_runs(library=None, damping=0.0, iters=25):
    """Constant images: the photometric Jacobian is zero and every residual of a
    pose vanishes, so the poses stay exactly at the prior mean; the log-depths
    move under the prior and the normal-integration factors of a tilted plane,
    both linear in the log-depth. Returns, per iteration, the relinearised
    points and the frozen run's absolute means."""
    H, W = 6, 7
    cam = synth.Camera.default(H, W)
    img = np.full((H, W), 0.5, dtype=np.float32)
    normals = _tilted_normals(H, W)
    kw = dict(sigma_P=0.5, sigma_R=1e-2, sigma_N=2e-2, init_inv_depth=0.3, damping=damping)
    runs = []
    rng = np.random.default_rng(11)
    ell0 = None
    for frozen in (0, 1):
        o = oracle.Oracle(oracle.config_for_camera(cam, frozen=frozen, **kw), library)
        o.set_keyframe(img, normals)
        o.set_frame(img)
        st = o.get_state()
        if ell0 is None:
            ell0 = st[..., 6] + rng.normal(0.0, 0.3, size=(H, W))
        st[..., 6] = ell0
        o.set_state(st)
        seq = []
        for _ in range(iters):
            o.iterate(1)
            if frozen:
                m = o.means()
                seq.append(np.concatenate([m[..., :6], (ell0 + m[..., 6])[..., None]], axis=-1))
            else:
                seq.append(o.get_state()[..., :7].copy())
        runs.append(np.array(seq))
    relin, froz = runs
    return relin, froz, ell0


def _linear_deviation(library=None, damping=0.0):
    relin, froz, ell0 = _linear_runs(library, damping)
    moved = np.abs(froz[..., 6] - ell0).max()
    return np.abs(relin - froz).max() / moved, relin, froz


@pytest.mark.parametrize("damping", [0.0, 0.4])
def test_transport_exact_on_linear_problem(damping):
    dev, relin, froz = _linear_deviation(damping=damping)
    # the poses never leave the prior mean, the log-depths move by O(1)
    assert np.abs(relin[..., :6]).max() == 0.0 and np.abs(froz[..., :6]).max() == 0.0
    assert np.abs(froz[-1, ..., 6] - froz[0, ..., 6]).max() > 0.05
    assert dev <= 1e-12, dev


@pytest.mark.parametrize("fault", sorted(PLANTED))
def test_linear_transport_pin_catches_planted_fault(planted, fault):
    dev, _, _ = _linear_deviation(planted[fault])
    assert dev > 1e-3, (PLANTED[fault], dev)


# --- smooth nonlinear problem: second order in the displacement --------------------

def _ramp_runs(eps, library=None, iters=12):
    """A linear intensity ramp, whose bilinear interpolant and central
    differences are exact, so the only nonlinearity is the warp and SE(3)
    itself. The keyframe image is the frame plus eps times seeded noise, so
    the solution lies O(eps) from the start. The prior means sit at the start
    (identity pose, log-depth log 2), and the border pixels, whose warps may
    leave the image, carry a negligible photometric weight."""
    H, W = 8, 9
    cam = synth.Camera.default(H, W)
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    I_t = 0.5 + 0.03 * u - 0.02 * v
    rng = np.random.default_rng(5)
    I_s = I_t + eps * rng.normal(size=(H, W))
    normals = np.broadcast_to(np.array([0.0, 0.0, -1.0]), (H, W, 3)).astype(np.float32).copy()
    sig = np.full((H, W), 1e-2)
    sig[0, :] = sig[-1, :] = sig[:, 0] = sig[:, -1] = 1e6
    kw = dict(sigma_P=0.1, sigma_R=1e-2, sigma_N=1e-1, sigma_D=1e-2, huber_k=400.0,
              init_inv_depth=0.5, prior_log_depth=math.log(2.0))
    out = []
    for frozen in (0, 1):
        o = oracle.Oracle(oracle.config_for_camera(cam, frozen=frozen, **kw), library)
        o.set_sigma_D_map(sig)
        o.set_keyframe64(I_s, normals)
        o.set_frame64(I_t)
        x0 = o.get_state()[..., :7].copy()
        seq = []
        for _ in range(iters):
            o.iterate(1)
            if frozen:
                seq.append(x0 + o.means())
            else:
                seq.append(o.get_state()[..., :7].copy())
        out.append((np.array(seq), x0))
    (relin, x0), (froz, _) = out
    return np.abs(relin - froz).max(), np.abs(froz - x0).max()


def _order(library=None):
    d1, s1 = _ramp_runs(2e-3, library)
    d2, s2 = _ramp_runs(5e-4, library)
    return d1, s1, d2, s2


def test_transport_second_order_on_smooth_problem():
    d1, s1, d2, s2 = _order()
    # the displacement scales with eps; the relinearised-vs-frozen difference
    # with eps^2 (ratio 16 for a factor 4 in eps)
    assert 3.5 < s1 / s2 < 4.5, (s1, s2)
    assert d1 / d2 > 12.0, (d1, d2)
    assert d1 / s1 < 2e-2, (d1, s1)


# fault 2 leaves the pose messages right; the log-depth moves only O(eps^2)
# here, so the linear pin above is the one that catches it
@pytest.mark.parametrize("fault", [1, 3])
def test_second_order_pin_catches_planted_fault(planted, fault):
    d1, s1, d2, s2 = _order(planted[fault])
    assert d1 / d2 < 8.0 or d1 / s1 > 5e-2, (PLANTED[fault], d1, s1, d2, s2)


# --- damping ------------------------------------------------------------------------

def _message_planes(st, tree=False):
    if tree:
        pix, nodes = st
        return np.concatenate([pix[..., 7:].reshape(-1), nodes[:, 6:].reshape(-1)])
    return st[..., 7:].reshape(-1)


@pytest.mark.parametrize("topology", [oracle.TOPO_GRID, oracle.TOPO_QUADTREE])
def test_damped_step_mixes_new_and_replaced_messages(topology):
    p = synth.tiny_pair(3, H=5, W=6, lattice_px=2.0)
    cam = p["cam"]
    kw = dict(sigma_P=1e-2, sigma_R=1e-2, sigma_N=1e-2, init_inv_depth=0.4, frozen=1, topology=topology)
    tree = topology == oracle.TOPO_QUADTREE

    def run(beta, st=None, n=1):
        o = oracle.Oracle(oracle.config_for_camera(cam, damping=beta, **kw))
        o.set_keyframe(p["I_s"], p["normals_s"])
        o.set_frame(p["I_t"])
        if st is not None:
            o.set_state(st)
        o.iterate(n)
        return o.get_state()

    s = run(0.0, n=1)                      # a state whose stored messages are non-zero
    old = _message_planes(s, tree)
    assert np.abs(old).max() > 0
    new = _message_planes(run(0.0, s), tree)
    beta = 0.3
    damped = _message_planes(run(beta, s), tree)
    ref = (1.0 - beta) * new + beta * old
    assert np.abs(new - old).max() > 1e-3 * np.abs(old).max()
    np.testing.assert_allclose(damped, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("seed", [3, 4])
def test_frozen_damped_gbp_converges_to_dense_solve(seed):
    p = synth.tiny_pair(seed, H=5, W=6, lattice_px=2.0)
    cam = p["cam"]
    kw = dict(sigma_P=1e-2, sigma_R=1e-2, sigma_N=1e-2)
    o = oracle.Oracle(oracle.config_for_camera(cam, init_inv_depth=0.4, frozen=1, damping=0.5, **kw))
    o.set_keyframe(p["I_s"], p["normals_s"])
    o.set_frame(p["I_t"])
    st = o.get_state()
    rng = np.random.default_rng(seed)
    st[..., :6] = rng.normal(0, 0.003, size=st[..., :6].shape)
    st[..., 6] += rng.normal(0, 0.05, size=st[..., 6].shape)
    o.set_state(st)
    prob = dense.Problem(cam.H, cam.W, (cam.fx, cam.fy, cam.cx, cam.cy), p["I_s"], p["I_t"], p["normals_s"], **kw)
    ref = prob.solve_linear(st[..., :6].reshape(-1, 6), st[..., 6].reshape(-1))
    o.iterate(900)
    m = o.means().reshape(-1, 7)
    np.testing.assert_allclose(m, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
