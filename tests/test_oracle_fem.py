"""Pins of the oracle's link-element pieces (sections "Tetrahedral
Finite-Elements" and "Actuation Constraints"): the corotational strain of a
constant-strain tetrahedron, its Jacobian, the element compliance and the
pressure-driven distance constraint.

Pinned by: zero strain at rest and under any rigid motion (the corotation);
the exact strains of a uniaxial stretch and of a simple shear (the textbook
polar decomposition of a shear); central finite differences of the
Jacobian with the rotation held fixed; the compliance turning a uniaxial
stress into the uniaxial strain with Poisson contraction and a shear stress
into tensor shear strain tau / (2 mu); and the distance constraint's value
and Jacobian."""
import numpy as np
import pytest

import oracle

REST = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]) * 0.01


def rot(axis, ang):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


def test_rest_and_rigid_motions_have_zero_strain():
    Dm_inv, V = oracle.fem_tet_rest(REST)
    assert abs(V - 1e-6 / 6) <= 1e-18
    C, _, R = oracle.fem_tet_eval(Dm_inv, REST)
    assert np.abs(C).max() <= 1e-14 and np.abs(R - np.eye(3)).max() <= 1e-14
    rng = np.random.default_rng(1)
    for _ in range(20):
        Q = rot(rng.normal(size=3), rng.uniform(0, np.pi))
        x = REST @ Q.T + rng.normal(size=3)
        C, _, R = oracle.fem_tet_eval(Dm_inv, x)
        assert np.abs(C).max() <= 1e-12
        assert np.abs(R - Q).max() <= 1e-12


def test_uniaxial_stretch_and_simple_shear():
    Dm_inv, _ = oracle.fem_tet_rest(REST)
    for s in (0.8, 1.0, 1.3):
        C, _, _ = oracle.fem_tet_eval(Dm_inv, REST * [s, 1.0, 1.0])
        assert np.abs(C - [s - 1, 0, 0, 0, 0, 0]).max() <= 1e-14
    # x += g y: the stretch of the polar decomposition is
    # [[2, g], [g, 2 + g^2]] / sqrt(4 + g^2) in the xy block
    for g in (0.05, 0.4, 1.5):
        x = REST.copy()
        x[:, 0] += g * REST[:, 1]
        C, _, R = oracle.fem_tet_eval(Dm_inv, x)
        w = np.sqrt(4 + g * g)
        want = [2 / w - 1, (2 + g * g) / w - 1, 0, 0, 0, g / w]
        assert np.abs(C - want).max() <= 1e-13, g
        assert abs(np.linalg.det(R) - 1) <= 1e-13


def test_jacobian_with_the_rotation_held_matches_finite_differences():
    Dm_inv, _ = oracle.fem_tet_rest(REST)
    rng = np.random.default_rng(2)
    x = REST @ rot([1, 2, 3], 0.7).T + rng.normal(0, 1e-3, REST.shape)
    C, J, R = oracle.fem_tet_eval(Dm_inv, x)
    eps = 1e-7
    Jfd = np.zeros_like(J)
    for m in range(4):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[m, c] += eps
            xm[m, c] -= eps
            Jfd[:, 3 * m + c] = (oracle.fem_tet_eval(Dm_inv, xp, R)[0] - oracle.fem_tet_eval(Dm_inv, xm, R)[0]) / (2 * eps)
    assert np.abs(J - Jfd).max() <= 1e-6 * np.abs(J).max()
    # translations do not strain: each row's x, y, z columns sum to zero over the vertices
    assert np.abs(J.reshape(6, 4, 3).sum(axis=1)).max() <= 1e-9 * np.abs(J).max()


def test_compliance_is_the_isotropic_elastic_compliance():
    """c + E lambda = 0 makes lambda = -V sigma: a uniaxial stress sigma0
    gives the strain (1, -nu, -nu) sigma0 / Y; a shear stress tau gives the
    tensor shear strain tau (1 + nu) / Y = tau / (2 mu).  (With engineering
    shear strains gamma = 2 eps the shear entries would be 2 (1 + nu).)"""
    V, Y, nu = 2e-7, 66243.0, 0.4999
    E = oracle.fem_tet_compliance(V, Y, nu)
    s0 = 1234.0
    eps = E @ (V * np.array([s0, 0, 0, 0, 0, 0]))
    assert np.allclose(eps, s0 / Y * np.array([1, -nu, -nu, 0, 0, 0]), rtol=1e-14, atol=0)
    mu = Y / (2 * (1 + nu))
    eps = E @ (V * np.array([0, 0, 0, 0, 0, s0]))
    assert np.isclose(eps[5], s0 / (2 * mu), rtol=1e-14)
    assert np.all(np.linalg.eigvalsh(oracle.fem_tet_compliance(V, Y, 0.3)) > 0)


def test_distance_constraint_and_expansion():
    Y = 66243.0
    assert oracle.fem_expansion(0.0, Y) == 1.0
    assert np.isclose(oracle.fem_expansion(0.5 * Y, Y), 1.5)
    xi, xj = np.array([0.3, 0.1, -0.2]), np.array([0.0, 0.5, 0.1])
    r, p = 0.4, 2000.0
    c, J = oracle.fem_dist(xi, xj, r, p, Y)
    assert np.isclose(c, np.linalg.norm(xi - xj) - r * (1 + p / Y), rtol=1e-15)
    eps = 1e-7
    for k in range(6):
        a, b = np.r_[xi, xj].copy(), np.r_[xi, xj].copy()
        a[k] += eps
        b[k] -= eps
        fd = (oracle.fem_dist(a[:3], a[3:], r, p, Y)[0] - oracle.fem_dist(b[:3], b[3:], r, p, Y)[0]) / (2 * eps)
        assert abs(fd - J[k]) <= 1e-7


def test_degenerate_and_inverted_elements_refused():
    with pytest.raises(ValueError):
        oracle.fem_tet_rest(np.zeros((4, 3)))
    Dm_inv, _ = oracle.fem_tet_rest(REST)
    with pytest.raises(ValueError):
        oracle.fem_tet_eval(Dm_inv, REST * [-1.0, 1.0, 1.0])


def test_attachment_constraint():
    """eq. rigid_to_particle: zero when the particle sits at the body point
    (rotation applied by an independent matrix), Jacobian against finite
    differences (world rotation vectors for the body)."""
    Q = rot([0.3, -1.0, 0.5], 0.9)
    ang, ax = 0.9, np.array([0.3, -1.0, 0.5]) / np.linalg.norm([0.3, -1.0, 0.5])
    q = np.r_[np.cos(ang / 2), np.sin(ang / 2) * ax]
    x, r = np.array([0.1, -0.2, 0.3]), np.array([0.005, 0.0, -0.002])
    c, J = oracle.fem_attach(x, q, r, x + Q @ r)
    assert np.abs(c).max() <= 1e-15
    xp = x + Q @ r + np.array([1e-3, -2e-3, 5e-4])
    c, J = oracle.fem_attach(x, q, r, xp)
    eps = 1e-7
    for k in range(9):
        d = np.zeros(9)
        d[k] = eps

        def at(d):
            dq = rot(d[3:6], np.linalg.norm(d[3:6])) if np.linalg.norm(d[3:6]) > 0 else np.eye(3)
            # rotate the body by the world rotation dq: R' = dq R, i.e. the point R r -> dq R r
            Rn = dq @ Q
            w = np.sqrt(max(0.0, 1 + np.trace(Rn))) / 2
            qn = np.array([w, (Rn[2, 1] - Rn[1, 2]) / (4 * w), (Rn[0, 2] - Rn[2, 0]) / (4 * w), (Rn[1, 0] - Rn[0, 1]) / (4 * w)])
            return oracle.fem_attach(x + d[:3], qn, r, xp + d[6:])[0]
        fd = (at(d) - at(-d)) / (2 * eps)
        assert np.abs(fd - J[:, k]).max() <= 1e-7, k


def test_procedural_link_mesh():
    """The stand-in link mesh: volume exactly that of the polygonal prism
    (sections - 1 gaps x regular ring-gon area), every element positively
    oriented with the oracle's rest volume, a conforming mesh (interior
    triangles in two elements, the two caps and the outer surface in one),
    and symmetric under a turn of 2 pi / ring about the link axis."""
    import workloads as W

    S, K, L, R = 13, 8, 0.01, 0.01
    pts, tets = W.link_mesh(S, K, L, R)
    assert pts.shape == (S * (K + 1), 3) and tets.shape == (3 * K * (S - 1), 4)
    vols = []
    for t in tets:
        p = pts[t]
        v = np.linalg.det((p[1:] - p[0]).T) / 6
        assert v > 0
        vols.append(v)
        assert np.isclose(oracle.fem_tet_rest(p)[1], v, rtol=1e-12)
    assert np.isclose(sum(vols), L * 0.5 * K * R * R * np.sin(2 * np.pi / K), rtol=1e-12)
    faces = {}
    for t in tets:
        for f in ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)):
            key = tuple(sorted(int(t[i]) for i in f))
            faces[key] = faces.get(key, 0) + 1
    assert set(faces.values()) == {1, 2}
    assert sum(1 for c in faces.values() if c == 1) == 2 * K + 2 * K * (S - 1)
    per = K + 1

    def turn(i):
        s, j = divmod(int(i), per)
        return i if j == 0 else s * per + 1 + j % K

    Q = rot([1, 0, 0], 2 * np.pi / K)
    assert np.abs(pts @ Q.T - pts[[turn(i) for i in range(len(pts))]]).max() <= 1e-15
    assert {tuple(sorted(turn(i) for i in t)) for t in tets} == {tuple(sorted(int(i) for i in t)) for t in tets}
