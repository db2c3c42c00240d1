"""Pins for the oracle's tangent-space maps (Sec. 3.1) and the first-order transfer
Jacobian (Sec. 3.4, Appendix A). Each check is against a property the paper states or
a computation independent of the oracle's own formulas (numpy geometry, finite
differences)."""
import numpy as np
import pytest


def _unit(v):
    return v / np.linalg.norm(v)


def _mus(rng, n=40):
    mus = [_unit(rng.normal(size=3)) for _ in range(n)]
    # branch points of the frame construction and the poles
    mus += [np.array([0.0, 0.0, 1.0]), np.array([0.0, 0.0, -1.0]), np.array([1.0, 0.0, 0.0]),
            np.array([0.0, 1.0, 0.0]), np.array([0.6, 0.8, 0.0]), np.array([0.6, 0.8, -0.0]),
            _unit(np.array([1.0, 1.0, 1e-12])), _unit(np.array([1.0, 1.0, -1e-12]))]
    return mus


def test_frame_is_a_rotation_taking_mu_to_z(orc):
    rng = np.random.default_rng(0)
    for mu in _mus(rng):
        R = orc.frame(mu)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1.0) < 1e-14
        assert np.allclose(R @ mu, [0, 0, 1], atol=1e-14)


def test_log_then_exp_is_identity_and_log_mu_mu_is_zero(orc):
    rng = np.random.default_rng(1)
    for mu in _mus(rng):
        assert np.allclose(orc.log_map(mu, mu), 0.0, atol=1e-15)
        for _ in range(20):
            w = _unit(rng.normal(size=3))
            if w @ mu < -0.999:  # stay off the cut locus
                continue
            nu = orc.log_map(mu, w)
            assert np.allclose(orc.exp_map(mu, nu), w, atol=1e-12)


def test_log_map_length_is_geodesic_distance(orc):
    """|log_mu w| equals the great-circle distance (Sec. 3.1, equidistance property),
    computed here from the cross and dot products."""
    rng = np.random.default_rng(2)
    for mu in _mus(rng):
        for _ in range(20):
            w = _unit(rng.normal(size=3))
            d = np.arctan2(np.linalg.norm(np.cross(mu, w)), mu @ w)
            assert abs(np.linalg.norm(orc.log_map(mu, w)) - d) < 1e-13


def test_log_map_direction_is_the_projected_direction(orc):
    """The tangent vector points along the projection of w onto the tangent plane at mu;
    mapped to 3D with the frame rows it equals theta * (w - (mu.w) mu) / |w - (mu.w) mu|."""
    rng = np.random.default_rng(3)
    for mu in _mus(rng):
        R = orc.frame(mu)
        for _ in range(10):
            w = _unit(rng.normal(size=3))
            nu = orc.log_map(mu, w)
            v3 = nu[0] * R[0] + nu[1] * R[1]
            proj = w - (mu @ w) * mu
            th = np.arctan2(np.linalg.norm(proj), mu @ w)
            assert np.allclose(v3, th * proj / np.linalg.norm(proj), atol=1e-12)


def test_log_map_matches_printed_acos_form_away_from_small_angles(orc):
    """The printed form nu = (w'_x, w'_y) / sinc(acos w'_z) (Sec. 3.1) agrees with the
    atan2 form used by the oracle where acos is well conditioned."""
    rng = np.random.default_rng(4)
    for mu in _mus(rng, 10):
        R = orc.frame(mu)
        for _ in range(20):
            w = _unit(rng.normal(size=3))
            wp = R @ w
            th = np.arccos(np.clip(wp[2], -1, 1))
            if th < 0.1 or th > 3.0:
                continue
            printed = wp[:2] / (np.sin(th) / th)
            assert np.allclose(orc.log_map(mu, w), printed, rtol=1e-11, atol=1e-12)


def test_antipode_maps_to_the_cut_locus(orc):
    rng = np.random.default_rng(5)
    for mu in _mus(rng, 10):
        nu = orc.log_map(mu, -mu)
        assert abs(np.linalg.norm(nu) - np.pi) < 1e-12


def _fd_jacobian(f, x, h=1e-6):
    x = np.asarray(x, dtype=float)
    cols = []
    for j in range(x.size):
        e = np.zeros_like(x)
        e[j] = h
        cols.append((f(x + e) - f(x - e)) / (2 * h))
    return np.stack(cols, axis=1)


def test_transfer_jacobian_matches_finite_differences(orc):
    """J = d(log_{mu_new} o exp_mu)/d nu at nu = m, mu_new = exp_mu(m) (Sec. 3.4 with the
    corrected Appendix A Jacobians), against central differences of the composed maps."""
    rng = np.random.default_rng(6)
    for mu in _mus(rng, 30):
        for scale in (1e-3, 0.3, 1.2, 2.5):
            m = rng.normal(size=2)
            m = scale * m / np.linalg.norm(m)
            mu_new = orc.exp_map(mu, m)
            mu_new = mu_new / np.linalg.norm(mu_new)
            J = orc.transfer_jacobian(mu, m)
            Jfd = _fd_jacobian(lambda v: orc.log_map(mu_new, orc.exp_map(mu, v)), m)
            assert np.allclose(J, Jfd, atol=1e-8), (mu, m, J, Jfd)


def test_transfer_jacobian_is_identity_without_a_move(orc):
    """With m = 0 the mean does not move, so J = I; on the frame's branch plane mu_z = 0
    the exp map may return the other signed zero, and J is then the rotation between the
    two frames about mu (still orthogonal, determinant one)."""
    rng = np.random.default_rng(7)
    for mu in _mus(rng, 10):
        J = orc.transfer_jacobian(mu, np.zeros(2))
        if mu[2] != 0.0:
            assert np.allclose(J, np.eye(2), atol=1e-15)
        else:
            assert np.allclose(J @ J.T, np.eye(2), atol=1e-14)
            assert abs(np.linalg.det(J) - 1.0) < 1e-14


def test_printed_exp_jacobian_typos_would_fail_finite_differences():
    """Appendix A prints J_exp with 'sinc + nu_x nu_y c' off the diagonal and
    'sinc + nu_y c' at (2,2). Differentiating the exp-map equation of Sec. 3.1 numerically
    shows the corrected entries (nu_x nu_y c, sinc + nu_y^2 c); the printed ones differ."""
    nu = np.array([0.7, -0.4])

    def e(v):
        r = np.linalg.norm(v)
        s = np.sin(r) / r
        return np.array([v[0] * s, v[1] * s, np.cos(r)])

    r = np.linalg.norm(nu)
    s = np.sin(r) / r
    c = (np.cos(r) - s) / r ** 2
    corrected = np.array([[s + nu[0] ** 2 * c, nu[0] * nu[1] * c],
                          [nu[0] * nu[1] * c, s + nu[1] ** 2 * c],
                          [-nu[0] * s, -nu[1] * s]])
    printed = np.array([[s + nu[0] ** 2 * c, s + nu[0] * nu[1] * c],
                        [s + nu[1] * nu[0] * c, s + nu[1] * c],
                        [-nu[0] * s, -nu[1] * s]])
    fd = _fd_jacobian(e, nu)
    assert np.allclose(corrected, fd, atol=1e-9)
    assert not np.allclose(printed, fd, atol=1e-3)


def test_first_order_transfer_matches_monte_carlo_push_forward(orc):
    """Sec. 3.4, covariance figure: moving a tangent Gaussian's samples to the new mean's
    tangent space and taking their covariance agrees with J Sigma J^T to first order,
    while leaving Sigma unchanged does not."""
    rng = np.random.default_rng(8)
    mu = _unit(np.array([0.3, -0.5, 0.8]))
    m = np.array([0.5, 0.2])
    Sig = np.array([[0.02, 0.006], [0.006, 0.01]])
    Lc = np.linalg.cholesky(Sig)
    mu_new = orc.exp_map(mu, m)
    mu_new /= np.linalg.norm(mu_new)
    J = orc.transfer_jacobian(mu, m)
    z = rng.normal(size=(20000, 2)) @ Lc.T + m
    moved = np.array([orc.log_map(mu_new, orc.exp_map(mu, v)) for v in z])
    emp = np.cov(moved.T)
    first = J @ Sig @ J.T
    assert np.abs(first - emp).max() < 0.1 * np.abs(Sig).max()
    assert np.abs(first - emp).max() < 0.5 * np.abs(Sig - emp).max()
