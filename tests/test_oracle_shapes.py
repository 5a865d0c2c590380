"""Pins of the oracle's further basic shapes (the paper's gallery, Sec. 2.2):
capped cone, octahedron, hexagonal prism (exact distances) and ellipsoid (a
lower bound with the exact sign), against
- inside tests and densely sampled surfaces written independently here;
- escape fractions of a point source at the centre of an absorbing,
  index-matched shape: the average over directions of exp(-mu_a t(u)), t the
  exit distance in closed form, by quadrature over a Fibonacci sphere.
"""
import math

import numpy as np
import pytest


def one(W, prim, mua=1.0, src=(0.0, 0.0, 0.0)):
    return W._scene("one", [prim], [W._region([0], mua, 0.0, 0.0, 1.0)], {"kind": "point", "p": list(src)}, None)


def fib_dirs(n):
    i = np.arange(n) + 0.5
    z = 1 - 2 * i / n
    phi = math.pi * (1 + 5 ** 0.5) * i
    r = np.sqrt(1 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], 1)


def grid2(m):
    g = (np.arange(m) + 0.5) / m
    U, V = np.meshgrid(g, g)
    return U.ravel(), V.ravel()


def triangle_points(a, b, c, m):
    U, V = grid2(m)
    keep = U + V <= 1
    U, V = U[keep], V[keep]
    return a + np.outer(U, b - a) + np.outer(V, c - a)


# ------------------------------------------------------------ surfaces --

def cone_surface(a, b, ra, rb, m=200):
    a, b = np.asarray(a, float), np.asarray(b, float)
    e = (b - a) / np.linalg.norm(b - a)
    t1 = np.cross(e, [1, 0, 0] if abs(e[0]) < 0.9 else [0, 1, 0])
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(e, t1)
    U, V = grid2(m)
    ang = 2 * math.pi * U
    ring = np.outer(np.cos(ang), t1) + np.outer(np.sin(ang), t2)
    side = a + np.outer(V, b - a) + ring * (ra + (rb - ra) * V)[:, None]
    cap_a = a + ring * (ra * np.sqrt(V))[:, None]
    cap_b = b + ring * (rb * np.sqrt(V))[:, None]
    return np.concatenate([side, cap_a, cap_b])


def cone_inside(p, a, b, ra, rb):
    a, b = np.asarray(a, float), np.asarray(b, float)
    L = np.linalg.norm(b - a)
    e = (b - a) / L
    x = (p - a) @ e
    y = np.linalg.norm((p - a) - x * e)
    return 0 < x < L and y < ra + (rb - ra) * x / L


def octa_surface(c, s, m=150):
    pts = []
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sz in (-1, 1):
                pts.append(triangle_points(np.array([sx * s, 0, 0]), np.array([0, sy * s, 0]), np.array([0, 0, sz * s]), m))
    return np.concatenate(pts) + c


def hex_surface(c, h, hz, m=120):
    R = 2 * h / math.sqrt(3)
    verts = [np.array([R * math.cos(k * math.pi / 3), R * math.sin(k * math.pi / 3)]) for k in range(6)]
    U, V = grid2(m)
    pts = []
    for k in range(6):
        p0, p1 = verts[k], verts[(k + 1) % 6]
        xy = p0 + np.outer(U, p1 - p0)
        pts.append(np.column_stack([xy, -hz + 2 * hz * V]))
        for z in (-hz, hz):   # caps: triangles centre-p0-p1
            tri = triangle_points(np.zeros(2), p0, p1, m)
            pts.append(np.column_stack([tri, np.full(len(tri), z)]))
    return np.concatenate(pts) + c


def hex_inside(p, c, h, hz):
    x, y, z = np.abs(p - c)
    return y < h and math.sqrt(3) * x + y < 2 * h and z < hz


def ellipsoid_surface(c, r, m=400):
    U, V = grid2(m)
    th, ph = math.pi * U, 2 * math.pi * V
    return c + np.column_stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)]) * r


SHAPES = {
    "cone": ({"kind": "cone", "a": [-0.2, 0.1, -0.3], "b": [0.3, -0.1, 0.4], "ra": 0.35, "rb": 0.1},
             lambda p: cone_inside(p, [-0.2, 0.1, -0.3], [0.3, -0.1, 0.4], 0.35, 0.1),
             lambda: cone_surface([-0.2, 0.1, -0.3], [0.3, -0.1, 0.4], 0.35, 0.1), 0.006),
    "octahedron": ({"kind": "octahedron", "c": [0.1, 0.0, -0.1], "s": 0.5},
                   lambda p: np.abs(p - [0.1, 0.0, -0.1]).sum() < 0.5,
                   lambda: octa_surface(np.array([0.1, 0.0, -0.1]), 0.5), 0.006),
    "hexprism": ({"kind": "hexprism", "c": [0.0, 0.1, 0.0], "h": 0.3, "hz": 0.2},
                 lambda p: hex_inside(p, np.array([0.0, 0.1, 0.0]), 0.3, 0.2),
                 lambda: hex_surface(np.array([0.0, 0.1, 0.0]), 0.3, 0.2), 0.006),
}


@pytest.mark.parametrize("name", list(SHAPES))
def test_exact_shape_distance_and_sign(orc, W, name):
    prim, inside, surface, res = SHAPES[name]
    sc = one(W, prim)
    surf = surface()
    rng = np.random.default_rng(40)
    for p in rng.uniform(-0.8, 0.8, (250, 3)):
        d = orc.region_sdf(sc, 0, p)
        assert (d < 0) == inside(p), (name, p, d)
        near = np.min(np.linalg.norm(surf - p, axis=1))
        assert abs(abs(d) - near) < res, (name, p, d, near)


def test_ellipsoid_is_a_signed_lower_bound(orc, W):
    c, r = np.array([0.1, -0.1, 0.0]), np.array([0.5, 0.3, 0.2])
    sc = one(W, {"kind": "ellipsoid", "c": c.tolist(), "radii": r.tolist()})
    surf = ellipsoid_surface(c, r)
    rng = np.random.default_rng(41)
    for p in rng.uniform(-0.8, 0.8, (250, 3)):
        d = orc.region_sdf(sc, 0, p)
        assert (d < 0) == (np.linalg.norm((p - c) / r) < 1)
        near = np.min(np.linalg.norm(surf - p, axis=1))
        assert abs(d) <= near + 0.004                       # never beyond the surface
        assert abs(d) >= near * r.min() / r.max() - 0.004   # and within the radius ratio of it


def _escape(orc, W, prim, t_of_u, mua=2.0, N=100000, seed=3):
    sc = one(W, prim, mua)
    got = orc.run(sc, seed=seed, n=N)["escaped_face"].sum() / N
    u = fib_dirs(40000)
    want = float(np.mean(np.exp(-mua * t_of_u(u))))
    assert abs(got - want) < 4 * math.sqrt(want * (1 - want) / N), (got, want)


def test_octahedron_escape(orc, W):
    s = 0.6
    _escape(orc, W, {"kind": "octahedron", "c": [0, 0, 0], "s": s}, lambda u: s / np.abs(u).sum(1))


def test_ellipsoid_escape(orc, W):
    r = np.array([0.6, 0.4, 0.25])
    _escape(orc, W, {"kind": "ellipsoid", "c": [0, 0, 0], "radii": r.tolist()},
            lambda u: 1.0 / np.linalg.norm(u / r, axis=1))


def test_hexprism_escape(orc, W):
    h, hz = 0.4, 0.3
    normals = np.array([[math.cos(a), math.sin(a)] for a in (math.pi / 6 + k * math.pi / 3 for k in range(6))])

    def t(u):
        tz = hz / np.maximum(np.abs(u[:, 2]), 1e-300)
        dots = u[:, :2] @ normals.T
        tside = np.min(np.where(dots > 0, h / np.maximum(dots, 1e-300), np.inf), axis=1)
        return np.minimum(tz, tside)
    _escape(orc, W, {"kind": "hexprism", "c": [0, 0, 0], "h": h, "hz": hz}, t)


def test_cone_escape_on_its_axis(orc, W):
    # source on the axis of a frustum along z: exit through a cap or the
    # side; the side distance solves a quadratic
    ra, rb, L, z0 = 0.5, 0.2, 0.8, 0.3
    prim = {"kind": "cone", "a": [0, 0, 0], "b": [0, 0, L], "ra": ra, "rb": rb}
    sc = one(W, prim, 2.0, (0.0, 0.0, z0))
    N = 100000
    got = orc.run(sc, seed=5, n=N)["escaped_face"].sum() / N
    u = fib_dirs(40000)
    k = (rb - ra) / L
    # side: rho(t) = t |u_xy| = ra + k (z0 + t u_z)  (the radius grows linearly)
    rho = np.linalg.norm(u[:, :2], axis=1)
    t_side = (ra + k * z0) / np.maximum(rho - k * u[:, 2], 1e-300)
    t_side = np.where(rho - k * u[:, 2] > 0, t_side, np.inf)
    t_cap = np.where(u[:, 2] > 0, (L - z0) / np.maximum(u[:, 2], 1e-300), z0 / np.maximum(-u[:, 2], 1e-300))
    want = float(np.mean(np.exp(-2.0 * np.minimum(t_side, t_cap))))
    assert abs(got - want) < 4 * math.sqrt(want * (1 - want) / N), (got, want)
