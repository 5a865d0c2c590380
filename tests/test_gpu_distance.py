"""Point queries of the scene SDF (smcrt_scene_distance) against the
oracle's region SDFs (Sec. 2.2: primitives, placement, modifiers and the
regions' CSG): every region's distance at seeded points spread over the
simulation volume and gathered near the surfaces, on the workload families,
the CSG, shape and gallery scenes, a vessel network and the random scenes
of every primitive kind, placement and modifier.

Tolerances, relative to the scene extent: FP64 1e-12 (the same formulas;
FMA contraction and the last bits of library transcendentals differ); FP32
2e-6 (the point rounded to float, then FP32 arithmetic on coordinates of
order the extent).  Owners (the walk's region rule) agree wherever no
region's surface is within that tolerance.  Through the acceleration grid
the accelerated region's distance is a lower bound of the exact one, equal
to it near the surface."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-6}


def _box(S, desc):
    sc = S.Scene(desc)  # held while the library reads it
    _, _, lo, hi = S.smcrt_scene_info(sc.h)
    return np.asarray(lo, dtype=float), np.asarray(hi, dtype=float)


def _points(S, orc, desc, seed, n_uniform=3000, n_near=1000):
    """Uniform points in the simulation volume, then points within 2 % of
    the extent of some region's surface (by rejection), with the oracle's
    distances at each."""
    rng = np.random.default_rng(seed)
    lo, hi = _box(S, desc)
    ext = float(np.max(hi - lo))
    cs = orc.CScene(desc)
    L = orc.lib()
    nr = len(desc["regions"])

    def exact(p):
        return [L.orc_region_sdf(cs.ref, r, orc._d3(p)) for r in range(nr)]

    pts = list(rng.uniform(lo, hi, size=(n_uniform, 3)))
    near = []
    for _ in range(200):
        if len(near) >= n_near:
            break
        for p in rng.uniform(lo, hi, size=(2000, 3)):
            if min(abs(d) for d in exact(p)) < 0.02 * ext:
                near.append(p)
    pts = np.array(pts + near[:n_near])
    ref = np.array([exact(p) for p in pts])
    own = np.array([L.orc_region_of(cs.ref, orc._d3(p)) for p in pts])
    return pts, ref, own, ext


def _check(S, eng, orc, desc, seed, prec):
    pts, ref, own, ext = _points(S, orc, desc, seed)
    d, o = S.distance(desc, pts, engine=eng, precision=prec)
    err = np.abs(d - ref).max() / ext
    clear = np.min(np.abs(ref), axis=1) > 10 * TOL[prec] * ext
    print(f"{desc['name']} {prec}: {len(pts)} points, worst |d - d_oracle| / extent {err:.2e}, "
          f"owners equal {np.mean(o[clear] == own[clear]):.5f} of {int(clear.sum())}")
    assert err <= TOL[prec], err
    assert np.array_equal(o[clear], own[clear])


FAMILIES = ["sphere", "slab", "cylinder", "glass_sphere", "bottle", "gallery", "shapes"]


@pytest.mark.parametrize("make", FAMILIES + ["random3", "random7", "random10"])
def test_numerical_normals_match_oracle(S, eng, orc, W, make):
    """The interface step's FP64 normals (Sec. 1: central differences of
    step delta/100 on both sides) against the oracle's at points within 2 %
    of the extent of a surface, every region: unit vectors equal to 1e-7
    (the difference quotient divides the SDFs' last-bit differences by
    2 delta/100)."""
    desc = W.random_scene(int(make[6:]), n_grid=8) if make.startswith("random") else W.WORKLOADS[make](n_grid=8)
    pts, ref, _, ext = _points(S, orc, desc, 500, n_uniform=0, n_near=600)
    _, _, nrm = S.distance(desc, pts, engine=eng, precision="f64", normals=True)
    h = 1e-2 * desc["delta"]
    nr = len(desc["regions"])
    o = np.array([[orc.region_normal(desc, r, p, h) for r in range(nr)] for p in pts])
    err = np.abs(nrm - o).max()
    print(f"{make}: {len(pts)} points x {nr} regions, worst normal difference {err:.2e}")
    assert np.allclose(np.linalg.norm(nrm, axis=2), 1.0, atol=1e-12)
    assert err <= 1e-7, err


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", FAMILIES)
def test_family_distances_match_oracle(S, eng, orc, W, name, prec):
    _check(S, eng, orc, W.WORKLOADS[name](n_grid=8), 100 + FAMILIES.index(name), prec)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("seed", range(12))
def test_random_scene_distances_match_oracle(S, eng, orc, W, seed, prec):
    _check(S, eng, orc, W.random_scene(seed, n_grid=8), 200 + seed, prec)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_vessel_distances_exact_and_through_the_grid(S, eng, orc, W, prec):
    desc = W.vessel_scene(3, 1.0, n_caps=300, n_grid=8)
    _check(S, eng, orc, dict(desc, accel_cells=None), 300, prec)
    pts, ref, _, ext = _points(S, orc, desc, 301)
    d, o = S.distance(desc, pts, engine=eng, precision=prec)
    da, oa = S.distance(desc, pts, engine=eng, precision=prec, accelerated=True)
    tol = TOL[prec] * ext
    acc = int(np.argmax([len(rg["prims"]) for rg in desc["regions"]]))
    others = [r for r in range(len(desc["regions"])) if r != acc]
    assert np.array_equal(da[:, others], d[:, others])
    assert np.all(da[:, acc] <= ref[:, acc] + tol)  # a lower bound: steps never pass a surface
    # the grid's query is the exact SDF wherever that is below its margin
    # (one cell); a quarter of the volume's side over the cell count is less
    near = ref[:, acc] < 0.25 * ext / max(desc["accel_cells"])
    print(f"vessels {prec}: {int(near.sum())} points near the capsules, "
          f"worst grid deviation there {np.abs(da[near, acc] - ref[near, acc]).max() / ext:.2e}")
    assert near.sum() >= 50
    assert np.all(np.abs(da[near, acc] - ref[near, acc]) <= tol)
    clear = np.min(np.abs(ref), axis=1) > 10 * tol
    assert np.array_equal(oa[clear], o[clear])  # the grid's bound keeps every sign


def _with_union(desc):
    """the scene itself when it has a union of several primitives; else its
    first two inner regions merged into one union (the first's properties)"""
    if any(rg["op"] == "union" and len(rg["prims"]) >= 2 for rg in desc["regions"]):
        return desc
    r = [dict(rg) for rg in desc["regions"]]
    r[1] = dict(r[1], prims=r[1]["prims"] + r[2]["prims"], op="union", k=0.0)
    del r[2]
    return dict(desc, regions=r)


BOUNDED = ("twist", "bend", "displace")  # modifiers whose SDFs are bounds, like the ellipsoid's


def _exact_union(desc, r):
    return all(desc["prims"][i]["kind"] != "ellipsoid" and not any(m in desc["prims"][i] for m in BOUNDED)
               for i in desc["regions"][r]["prims"])


def _ball_holds_no_surface(orc, desc, r, p, R, rng, n=3000):
    """no point of the open ball of radius R about p (outside region r) is
    inside region r: sampled uniformly in the ball, most samples near its
    rim"""
    cs, L = orc.CScene(desc), orc.lib()
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    q = p + v * (0.999 * R * rng.random(n) ** (1 / 3))[:, None]
    return all(L.orc_region_sdf(cs.ref, r, orc._d3(x)) >= 0 for x in q)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("seed", range(12))
def test_random_scene_grid_bounds(S, eng, orc, W, seed, prec):
    """The uniform grid over a union of placed and modified primitives of
    every kind is conservative: where the union's SDF is exact, the grid's
    distance is at most the SDF everywhere; where some member's SDF is only
    a bound (ellipsoid, twist, bend, displacement) the grid may exceed that
    bound, and then no surface lies within the grid's distance (checked by
    sampling the ball).  Near the surface it equals the SDF (every decision
    there is the brute-force one); the other regions and every owner are
    unchanged."""
    desc = dict(_with_union(W.random_scene(seed, n_grid=8)), accel_cells=[8, 8, 8])
    pts, ref, own, ext = _points(S, orc, desc, 400 + seed)
    da, oa = S.distance(desc, pts, engine=eng, precision=prec, accelerated=True)
    d, _ = S.distance(desc, pts, engine=eng, precision=prec)
    tol = TOL[prec] * ext
    # the region the binding accelerates: the union with most primitives (first of equals)
    unions = [(len(rg["prims"]), -i) for i, rg in enumerate(desc["regions"])
              if rg["op"] == "union" and len(rg["prims"]) >= 2]
    acc = -max(unions)[1]
    others = [r for r in range(len(desc["regions"])) if r != acc]
    assert np.array_equal(da[:, others], d[:, others])
    over = np.where(da[:, acc] > ref[:, acc] + tol)[0]
    if _exact_union(desc, acc):
        assert len(over) == 0, over[:5]
    else:
        rng = np.random.default_rng(seed)
        for i in rng.permutation(over)[:60]:
            assert ref[i, acc] > 0 and _ball_holds_no_surface(orc, desc, acc, pts[i], da[i, acc], rng), i
    # near the surface: within a quarter cell by the SDF -- and, where some
    # member's SDF is only a bound (it may be small far from its surface, in
    # cells that do not list it), by the grid too
    near = ref[:, acc] < 0.25 * ext / 8
    if not _exact_union(desc, acc):
        near &= da[:, acc] < 0.25 * ext / 8
    print(f"random {seed} {prec}: {int(near.sum())} points within a quarter cell of region {acc}, "
          f"worst deviation there {np.abs(da[near, acc] - ref[near, acc]).max() / ext:.2e}")
    assert near.sum() >= 20
    assert np.all(np.abs(da[near, acc] - ref[near, acc]) <= tol)
    clear = np.min(np.abs(ref), axis=1) > 10 * tol
    assert np.array_equal(oa[clear], own[clear])


def test_distance_of_no_points_and_bad_arguments(S, eng, W):
    desc = W.sphere_scene(n_grid=8)
    d, o = S.distance(desc, np.zeros((0, 3)), engine=eng)
    assert d.shape == (0, 1) and o.shape == (0,)
    sc = S.Scene(desc)
    with pytest.raises(S.SmcrtError, match="accelerated"):
        S.smcrt_scene_distance(eng.h, sc.h, None, 1, 2, None, None, None, None)
    with pytest.raises(S.SmcrtError, match="NULL points"):
        S.smcrt_scene_distance(eng.h, sc.h, None, 1, 0, None, None, None, None)
