"""Pins of three oracle parts that the other pin files leave open: the lagged friction element,
the Cauchy / von Mises stress output and the line search inside the oracle's own time step.

Each test checks the oracle against something other than itself: central finite differences,
eigenvalues from numpy, closed forms of the Neo-Hookean Cauchy stress (uniaxial stretch,
hydrostatic stretch, simple shear, rotation covariance), Coulomb's law for a sliding point, or
the line-search rule (Phi never increases at an accepted iterate; more than 40 halvings fail).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2503_05020_amd import scenes as S


def _fd_grad(f, x, h):
    g = np.zeros_like(x)
    for i in range(len(x)):
        e = np.zeros_like(x)
        e[i] = h
        g[i] = (f(x + e) - f(x - e)) / (2 * h)
    return g


# ---------------------------------------------------------------------------
# lagged friction element: D = mu lambda f0(|u|), u = (I - n n^T) sum_i w_i (x_i - x^n_i)
# (friction of the implicit step, Sec. II-C / III-D constants eps_v = 1e-3 m/s, dt = 0.01 s)
# ---------------------------------------------------------------------------
EPS = 1e-3 * 0.01  # eps_v * dt


def _pt_frame(rng):
    """A point above the interior of a triangle, its closest-point weights and unit normal at x^n."""
    t0 = rng.uniform(-0.01, 0.01, 3)
    e1 = np.array([0.02, 0.001, 0.0]) + rng.uniform(-1e-3, 1e-3, 3) * [1, 1, 0]
    e2 = np.array([0.003, 0.018, 0.0]) + rng.uniform(-1e-3, 1e-3, 3) * [1, 1, 0]
    b = rng.uniform(0.15, 0.35, 2)
    n = np.cross(e1, e2)
    n /= np.linalg.norm(n)
    p = t0 + b[0] * e1 + b[1] * e2 + 5e-4 * n
    xn = np.stack([p, t0, t0 + e1, t0 + e2])
    w = np.array([1.0, -(1 - b[0] - b[1]), -b[0], -b[1]])  # p - (closest point on the triangle)
    return xn, w, n


def _tangent(n, rng):
    t = rng.normal(size=3)
    t -= (t @ n) * n
    return t / np.linalg.norm(t)


@pytest.mark.parametrize("regime", ["static", "sticking", "sliding"])
@pytest.mark.parametrize("seed", range(3))
def test_friction_element_derivatives_fd_and_psd(regime, seed):
    """Gradient = central FD of the energy; Hessian = central FD of the gradient; Hessian PSD.
    Regimes: y = 0 (x = x^n), 0 < y < eps (smoothed static branch), y >= eps (kinetic branch)."""
    rng = np.random.default_rng(700 + seed)
    xn, w, n = _pt_frame(rng)
    lam, mu = rng.uniform(1.0, 50.0), rng.uniform(0.2, 0.8)
    disp = {"static": 0.0, "sticking": 0.4 * EPS, "sliding": 7.0 * EPS}[regime]
    x = xn.copy()
    # slip of the point against the triangle, plus some normal and rigid motion that friction ignores
    x[0] += disp * _tangent(n, rng) + 2e-6 * n
    x += 1e-6 * rng.normal(size=3)
    e, g, H = O.friction_elem(x, xn, w, n, lam, mu, EPS)
    f = lambda y: O.friction_elem(y.reshape(4, 3), xn, w, n, lam, mu, EPS)[0]
    x0 = x.reshape(-1)
    # the static branch's gradient has an O(|u|) nonlinearity at u = 0, so its FD step is smaller
    h = (1e-6 if regime == "static" else 1e-4) * EPS
    fg = _fd_grad(f, x0, h)
    scale = mu * lam
    assert np.allclose(g, fg, rtol=1e-6, atol=1e-7 * scale)
    fH = np.stack([_fd_grad(lambda y, i=i: O.friction_elem(y.reshape(4, 3), xn, w, n, lam, mu, EPS)[1][i], x0, h)
                   for i in range(12)])
    assert np.allclose(H, fH, rtol=1e-5, atol=1e-6 * np.abs(H).max())
    assert np.allclose(H, H.T, rtol=0, atol=1e-12 * np.abs(H).max())
    ev = np.linalg.eigvalsh(H)
    assert ev.min() >= -1e-12 * np.abs(H).max()
    # friction acts in the tangent plane only: every vertex's force is orthogonal to n
    assert np.abs(g.reshape(4, 3) @ n).max() <= 1e-12 * scale
    if regime == "static":
        assert np.abs(g).max() <= 1e-12 * scale  # u = 0 up to the rounding of the normal projection
        assert e == pytest.approx(mu * lam * EPS / 3, rel=1e-14)  # f0(0) = eps / 3


@pytest.mark.parametrize("seed", range(3))
def test_friction_coulomb_law_for_a_sliding_point(seed):
    """A point slid tangentially by |t| >= eps over a fixed triangle: dissipation mu lambda |t|, force on
    the point of magnitude mu lambda along t (Coulomb), equal and opposite force on the triangle."""
    rng = np.random.default_rng(800 + seed)
    xn, w, n = _pt_frame(rng)
    lam, mu = rng.uniform(1.0, 50.0), rng.uniform(0.2, 0.8)
    t = _tangent(n, rng) * rng.uniform(2.0, 100.0) * EPS
    x = xn.copy()
    x[0] += t
    e, g, H = O.friction_elem(x, xn, w, n, lam, mu, EPS)
    assert e == pytest.approx(mu * lam * np.linalg.norm(t), rel=1e-12)
    g = g.reshape(4, 3)
    assert g[0] == pytest.approx(mu * lam * t / np.linalg.norm(t), rel=1e-12, abs=1e-14 * mu * lam)
    assert np.abs(g.sum(0)).max() <= 1e-12 * mu * lam
    # kinetic branch: no stiffness along the slip direction, 1/|t| across it
    H = H[:3, :3]
    that = t / np.linalg.norm(t)
    assert abs(that @ H @ that) <= 1e-9 * np.abs(H).max()
    c = np.cross(n, that)
    assert c @ H @ c == pytest.approx(mu * lam / np.linalg.norm(t), rel=1e-12)


# ---------------------------------------------------------------------------
# Cauchy stress sigma = J^-1 P F^T and von Mises stress (per-tet stress output, Sec. IV-D)
# ---------------------------------------------------------------------------
def _stress_of(F):
    """Cauchy stress (xx, yy, zz, yz, xz, xy) and von Mises of every tet of a free block deformed by F."""
    sc = S.free_block(cells=1, gravity=(0, 0, 0))
    X = sc["rest_pos"]
    c = X.mean(0)
    sc = dict(sc)
    sc["init_pos"] = (X - c) @ np.asarray(F).T + c
    s = O.Scene(sc)
    _, _, cau, vm = s.state(stress=True)
    E, nu = sc["E"][0], sc["nu"][0]
    return cau, vm, E / (2 * (1 + nu)), E * nu / ((1 + nu) * (1 - 2 * nu))


@pytest.mark.parametrize("s", [0.8, 1.1, 1.5])
def test_cauchy_uniaxial_stretch_closed_form(s):
    cau, vm, mu, la = _stress_of(np.diag([s, 1.0, 1.0]))
    ref = np.array([(mu * (s * s - 1) + la * math.log(s)) / s, la * math.log(s) / s, la * math.log(s) / s, 0, 0, 0])
    for c in cau:
        assert c == pytest.approx(ref, rel=1e-10, abs=1e-10 * mu)
    assert vm == pytest.approx(np.full(len(vm), mu * abs(s * s - 1) / s), rel=1e-10)


@pytest.mark.parametrize("s", [0.9, 1.2])
def test_cauchy_hydrostatic_stretch_has_zero_von_mises(s):
    cau, vm, mu, la = _stress_of(np.eye(3) * s)
    p = (mu * (s * s - 1) + 3 * la * math.log(s)) / s ** 3
    for c in cau:
        assert c == pytest.approx([p, p, p, 0, 0, 0], rel=1e-10, abs=1e-10 * mu)
    assert np.abs(vm).max() <= 1e-8 * mu


@pytest.mark.parametrize("gam", [0.05, 0.3])
def test_cauchy_simple_shear_closed_form(gam):
    """F = I + gam e_x e_y^T (J = 1): sigma = mu (F F^T - I), so sigma_xy = mu gam, sigma_xx = mu gam^2,
    von Mises = mu sqrt(gam^4 + 3 gam^2)."""
    F = np.eye(3)
    F[0, 1] = gam
    cau, vm, mu, la = _stress_of(F)
    for c in cau:
        assert c == pytest.approx([mu * gam * gam, 0, 0, 0, 0, mu * gam], rel=1e-10, abs=1e-10 * mu)
    assert vm == pytest.approx(np.full(len(vm), mu * math.sqrt(gam ** 4 + 3 * gam * gam)), rel=1e-10)


def test_cauchy_rotation_covariance():
    """sigma(R F) = R sigma(F) R^T; von Mises is unchanged."""
    rng = np.random.default_rng(5)
    F = np.eye(3) + 0.2 * rng.normal(size=(3, 3))
    assert np.linalg.det(F) > 0
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    R = q * np.sign(np.linalg.det(q))
    c0, v0, mu, _ = _stress_of(F)
    c1, v1, _, _ = _stress_of(R @ F)

    def full(c):
        xx, yy, zz, yz, xz, xy = c
        return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])

    for a, b in zip(c0, c1):
        assert np.allclose(full(b), R @ full(a) @ R.T, rtol=0, atol=1e-9 * mu)
    assert v1 == pytest.approx(v0, rel=1e-9)


# ---------------------------------------------------------------------------
# the oracle's own line search inside its time step (plain decrease, halving, > 40 halvings fail)
# ---------------------------------------------------------------------------
def test_step_line_search_never_increases_phi():
    """Soft cube dropped onto the ground: across impact and resting contact, every accepted Newton
    iterate of every step has Phi(x + alpha p) <= Phi(x), alpha <= 1, and the halvings are counted."""
    sc = S.soft_cube_drop(cells=2, edge=0.04, height=0.004)
    s = O.Scene(sc)
    n_iters = n_halved = 0
    for k in range(14):
        rc, info = s.step(1)
        assert rc == 0, info
        log = s.iter_log()
        assert len(log) == info["newton_iters"] - 1  # the last direction only takes the stopping test
        assert np.all(log[:, 1] <= log[:, 0])
        assert np.all((log[:, 2] > 0) & (log[:, 2] <= 1.0))
        assert np.all(log[:, 2] <= 0.5 ** log[:, 3] * (1 + 1e-15))
        assert int(log[:, 3].sum()) == info["ls_halvings"]
        n_iters += len(log)
        n_halved += int((log[:, 3] > 0).sum())
    assert n_iters > 14
    assert info["n_active_last"] > 0  # the run reached contact


def test_step_line_search_stall_fails_after_40_halvings():
    """Planted fault in the oracle (a positive offset on every trial energy): no trial is ever
    accepted, so the step fails with the line-search reason after 40 halvings and the scene freezes."""
    sc = S.free_block(cells=1)
    s = O.Scene(sc)
    assert s.step(1)[0] == 0
    pos0, vel0 = s.state()
    s.debug_ls_offset(1.0)
    rc, info = s.step(1)
    assert rc == -5 and info["fail_reason"] == 3
    pos1, vel1 = s.state()
    assert np.array_equal(pos0, pos1) and np.array_equal(vel0, vel1)
    assert s.step(1)[0] == -5  # frozen
