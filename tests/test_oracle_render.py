"""Pins for oracle.render (CPU only): one- and two-Gaussian closed forms, an
opaque stack's termination count, depth ties ordered by id, and the
vectorised blend against the literal per-pixel loop on small random scenes."""
import math

import numpy as np

import scenegen
from oracle import project, render


def _proj(mx, my, conic, theta, rgb, depth, ids=None):
    n = len(mx)
    return dict(ids=np.arange(n) if ids is None else np.asarray(ids), valid=np.ones(n, bool),
                mean2d=np.stack([mx, my], 1).astype(float), conic=np.asarray(conic, float),
                theta=np.asarray(theta, float), rgb=np.asarray(rgb, float), depth=np.asarray(depth, float),
                radius=np.full(n, 1e6), near_margin=np.ones(n))


def test_single_gaussian_closed_form():
    p = _proj([8.0], [8.0], [[0.02, 0.005, 0.03]], [0.7], [[0.2, 0.4, 0.9]], [3.0])
    out = render.render_image(p, 16, 16, bg=(0.1, 0.0, 0.3))
    for (x, y) in [(8, 8), (2, 5), (15, 0), (7, 12)]:
        dx, dy = x + 0.5 - 8.0, y + 0.5 - 8.0
        a = min(0.99, 0.7 * math.exp(-0.5 * (0.02 * dx * dx + 0.01 * dx * dy + 0.03 * dy * dy)))
        exp = (np.array([0.2, 0.4, 0.9]) * a + (1 - a) * np.array([0.1, 0, 0.3])) if a >= 1 / 255 \
            else np.array([0.1, 0, 0.3])
        np.testing.assert_allclose(out["image"][:, y, x], exp, atol=1e-14)


def test_two_gaussians_depth_order():
    # the nearer one (depth 2) is blended first regardless of list order
    p = _proj([4.0, 4.0], [4.0, 4.0], [[1e-6, 0, 1e-6]] * 2, [0.6, 0.5], [[1, 0, 0], [0, 1, 0]], [5.0, 2.0])
    c = render.render_pixels(p, [3], [3])["rgb"][0]
    a1, a2 = 0.5, 0.6     # rho ~ 0 at the centre
    np.testing.assert_allclose(c, [a2 * (1 - a1), a1, 0.0], atol=1e-5)


def test_opaque_stack_termination():
    # eight alpha = 0.8 Gaussians: T = 0.2^k; the 6th would take T to 6.4e-5 < 1e-4 -> 5 blended
    n = 8
    p = _proj([0.5] * n, [0.5] * n, [[1e-9, 0, 1e-9]] * n, [0.8] * n, [[1, 1, 1]] * n, np.arange(1, n + 1))
    r = render.render_pixels(p, [0], [0])
    assert r["n_contrib"][0] == 5
    np.testing.assert_allclose(r["rgb"][0], [1 - 0.2 ** 5] * 3, atol=1e-9)
    np.testing.assert_allclose(r["T"][0], 0.2 ** 5, rtol=1e-6)
    # Eq. 3's 0.99 clamp: theta = 1 at the centre still gives alpha = 0.99
    p = _proj([0.5], [0.5], [[1e-9, 0, 1e-9]], [1.0], [[1, 0, 0]], [1.0])
    r = render.render_pixels(p, [0], [0])
    np.testing.assert_allclose(r["rgb"][0], [0.99, 0, 0], atol=1e-9)


def test_ambiguity_flags():
    # alpha exactly at alpha* (within 1e-6) at the centre pixel is flagged, a clear one is not
    p = _proj([0.5, 5.5], [0.5, 0.5], [[1e-12, 0, 1e-12]] * 2, [1 / 255 * (1 + 1e-6), 0.5], [[1, 1, 1]] * 2,
              [1.0, 2.0])
    p["radius"][:] = 1.0
    r = render.render_pixels(p, [0, 5], [0, 0])
    assert r["ambiguous"].tolist() == [True, False]


def test_equal_depth_ordered_by_id():
    p = _proj([2.0, 2.0], [2.0, 2.0], [[1e-6, 0, 1e-6]] * 2, [0.5, 0.5], [[1, 0, 0], [0, 1, 0]], [4.0, 4.0],
              ids=[9, 3])
    c = render.render_pixels(p, [1], [1])["rgb"][0]
    # id 3 (green) first
    np.testing.assert_allclose(c, [0.25, 0.5, 0.0], atol=1e-5)


def test_vectorised_equals_loop():
    sc = scenegen.random_gaussians(60, 1, 32, 24, depth_range=(2, 10), scale_range=(-3.0, -1.0))
    cam = scenegen.identity_camera(32, 24)
    p = project.project(sc, np.arange(60), cam)
    out = render.render_image(p, 32, 24, bg=(0.2, 0.3, 0.4), chunk=7)
    rng = np.random.default_rng(0)
    for _ in range(40):
        x, y = int(rng.integers(32)), int(rng.integers(24))
        c, T, n = render.render_pixel_loop(p, x, y, bg=(0.2, 0.3, 0.4))
        np.testing.assert_allclose(out["image"][:, y, x], c, atol=1e-12)
        assert out["n_contrib"][y, x] == n
        np.testing.assert_allclose(out["T"][y, x], T, rtol=1e-12)


# ------------------------------------------------------------- LUT (Eq. 5) ----

def test_lut_table_is_the_node_values():
    """m + 1 nodes over [-5.55, 0]: e^0 = 1 first, e^-5.55 last, a geometric
    sequence of ratio e^(-5.55/m) (float32 values)."""
    for m in (8, 32, 128):
        t = render.lut_table(m)
        assert len(t) == m + 1
        assert t[0] == 1.0 and t[-1] == float(np.float32(math.exp(-5.55)))
        np.testing.assert_allclose(t[1:] / t[:-1], math.exp(-5.55 / m), rtol=3e-7)
        assert np.all(t.astype(np.float32).astype(np.float64) == t)


def test_lut_index_rounds_to_the_nearest_node():
    m = 32
    h = 5.55 / m
    for k in (0, 1, 7, 31, 32):
        assert render.lut_index(-k * h, m) == k
        if k < m:
            assert render.lut_index(-(k + 0.5) * h + 1e-9, m) == k        # just before the midpoint
            assert render.lut_index(-(k + 0.5) * h - 1e-9, m) == k + 1    # just after it
    assert render.lut_index(0.0, m) == 0
    assert render.lut_index(-5.55 * 1.2, m) == m                      # below the range: the last node
    assert render.lut_index(-1e6, m) == m


def test_lut_error_bound_is_half_an_interval():
    """|table/e^rho - 1| <= e^(5.55 / 2m) - 1 over [-5.55, 0], and the bound is
    reached near the midpoints (a table of interval centres, or truncation
    instead of rounding, would err by up to a whole interval)."""
    rho = np.linspace(-5.55, 0.0, 200001)
    for m in (8, 32, 128):
        bound = math.exp(5.55 / (2 * m)) - 1
        err = np.abs(render.lut_exp(rho, m) / np.exp(rho) - 1)
        assert err.max() <= bound * (1 + 1e-5) + 2e-7
        assert err.max() >= 0.95 * bound


def test_lut_single_gaussian_at_node_offsets():
    """A pixel whose rho lies a tenth of an interval off node k (either side)
    reads the node value e^(-5.55 k / m): alpha = theta e^(-5.55 k / m)."""
    m, q, theta = 16, 0.02, 0.9                       # isotropic conic: rho = -q d^2 / 2
    h = 5.55 / m
    for k in (0, 3, 9, 15):
        for off in (0.1, -0.1):
            rho = min(0.0, -k * h + off * h)
            dx = math.sqrt(-2 * rho / q)
            p = _proj([0.5 - dx], [0.5], [[q, 0.0, q]], [theta], [[0.3, 0.6, 1.0]], [2.0])
            r = render.render_pixels(p, [0], [0], lut_m=m)
            a = theta * float(np.float32(math.exp(-5.55 * k / m)))
            want = np.array([0.3, 0.6, 1.0]) * a if a >= 1 / 255 else np.zeros(3)
            np.testing.assert_allclose(r["rgb"][0], want, rtol=1e-12, atol=1e-15)


def test_lut_vectorised_equals_loop():
    sc = scenegen.random_gaussians(60, 2, 32, 24, depth_range=(2, 10), scale_range=(-3.0, -1.0))
    cam = scenegen.identity_camera(32, 24)
    p = project.project(sc, np.arange(60), cam)
    out = render.render_image(p, 32, 24, bg=(0.2, 0.3, 0.4), chunk=5, lut_m=16)
    rng = np.random.default_rng(1)
    for _ in range(40):
        x, y = int(rng.integers(32)), int(rng.integers(24))
        c, T, n = render.render_pixel_loop(p, x, y, bg=(0.2, 0.3, 0.4), lut_m=16)
        np.testing.assert_allclose(out["image"][:, y, x], c, atol=1e-12)
        assert out["n_contrib"][y, x] == n


def test_lut_converges_to_the_exponential():
    sc = scenegen.random_gaussians(80, 3, 32, 24, depth_range=(2, 10), scale_range=(-3.0, -1.0))
    cam = scenegen.identity_camera(32, 24)
    p = project.project(sc, np.arange(80), cam)
    exact = render.render_image(p, 32, 24)["image"]
    errs = []
    for m in (8, 64, 20000):
        e = np.abs(render.render_image(p, 32, 24, lut_m=m)["image"] - exact)
        errs.append(e.mean())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-4


def test_lut_midpoint_is_ambiguous():
    m = 32
    h = 5.55 / m
    q = 0.02
    d = math.sqrt(2 * 3.5 * h / q)                    # rho = -3.5 h: a rounding midpoint
    p = _proj([0.5 - d + 0.5], [0.5], [[q, 0.0, q]], [0.9], [[1, 1, 1]], [2.0])
    p["mean2d"][0, 0] = 0.5 - d                       # pixel (0, 0) centre at distance d
    r = render.render_pixels(p, [0, 0], [0, 0], lut_m=m)
    assert r["ambiguous"][0]
    r2 = render.render_pixels(p, [0], [0], lut_m=0)
    assert not r2["ambiguous"][0]


def _centre(theta, depth, rgb=(1.0, 1.0, 1.0)):
    """Gaussians centred on pixel (0, 0)'s centre with a flat conic: rho = 0
    there, so alpha = min(0.99, theta) exactly."""
    n = len(theta)
    return _proj([0.5] * n, [0.5] * n, [[1e-12, 0, 1e-12]] * n, theta, [rgb] * n, depth)


def test_t_min_crossing_is_flagged():
    """A blend that takes T within float32 reach of 1e-4 (here 5e-6 relative,
    on either side) is ambiguous; clear crossings and clear blends are not.
    T = 0.1 * 0.05 = 0.005 after alphas 0.9 and 0.95, then the third Gaussian
    takes it to 0.005 (1 - theta3) = 1e-4 (1 + rel) (theta3 ~ 0.98, below the
    0.99 clamp)."""
    for rel, amb, n in [(5e-6, True, 3), (-5e-6, True, 2), (1e-2, False, 3), (-1e-2, False, 2),
                        (0.5, False, 3)]:
        theta3 = 1.0 - 0.02 * (1.0 + rel)
        r = render.render_pixels(_centre([0.9, 0.95, theta3], [1.0, 2.0, 3.0]), [0], [0])
        assert r["n_contrib"][0] == n, (rel, r["n_contrib"][0])
        assert r["ambiguous"][0] == amb, rel


def test_depth_tie_between_contributors_is_flagged():
    """Two consecutive contributors within 1e-6 relative in depth are
    ambiguous (float32 depth keys may order them either way); 1e-5 apart they
    are not, and a tie with a Gaussian below alpha* (no contribution) is not."""
    for d2, amb in [(5.0 * (1 + 5e-7), True), (5.0 * (1 - 5e-7), True), (5.0 * (1 + 1e-5), False),
                    (6.0, False)]:
        r = render.render_pixels(_centre([0.5, 0.5], [5.0, d2]), [0], [0])
        assert r["n_contrib"][0] == 2
        assert r["ambiguous"][0] == amb, d2
    # the tied Gaussian does not blend (theta below alpha* = 1/255): no flag
    r = render.render_pixels(_centre([0.5, 1e-3, 0.5], [5.0, 5.0 * (1 + 5e-7), 6.0]), [0], [0])
    assert r["n_contrib"][0] == 2 and not r["ambiguous"][0]
    # ... nor a tie that lies past the T stop
    r = render.render_pixels(_centre([0.9, 0.95, 0.99, 0.5], [1.0, 2.0, 3.0, 3.0 * (1 + 5e-7)]), [0], [0])
    assert r["n_contrib"][0] == 2 and not r["ambiguous"][0]


def test_threaded_oracle_equals_serial():
    """The threaded conveniences only split the work: bitwise the same results."""
    from oracle import lod
    sc = scenegen.random_gaussians(300, 4, 48, 40, depth_range=(2, 10), scale_range=(-3.0, -1.0))
    cam = scenegen.identity_camera(48, 40)
    p1 = project.project(sc, np.arange(300), cam)
    p4 = project.project_threaded(sc, np.arange(300), cam, threads=4, chunk=37)
    for k in p1:
        assert np.array_equal(p1[k], p4[k]), k
    a = render.render_image(p1, 48, 40)
    b = render.render_image(p1, 48, 40, threads=4)
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    city = scenegen.make_city("tiny")
    cams = scenegen.walkthrough(scenegen.CONFIGS["tiny"], frames=2)
    q1 = lod.predicates(city, cams[1], 2.0)
    q4 = lod.predicates_threaded(city, cams[1], 2.0, threads=4, chunk=5000)
    for k in q1:
        assert np.array_equal(q1[k], q4[k]), k


def test_threaded_oracle_is_deterministic_with_large_chunks():
    """Chunks large enough for a multithreaded BLAS to split them, on 8
    threads at once, four times over: projection, blend and the LoD
    predicates stay bitwise those of one thread (no helper may hand products
    to a BLAS that returns wrong results to concurrent callers)."""
    from oracle import lod
    n, W, H = 1_000_000, 64, 48
    sc = scenegen.random_gaussians(n, 21, W, H, depth_range=(2, 40), scale_range=(-4.0, -1.0))
    cam = scenegen.look_camera([0.3, -0.2, -0.5], 0.05, 0.02, W, H)
    ids = np.arange(n)
    p1 = project.project(sc, ids, cam)
    q1 = lod.predicates(sc, cam, 2.0)
    tiles = [0, 5, 11]
    keep = np.nonzero(p1["valid"])[0][:60_000]
    sub = {k: v[keep] for k, v in p1.items()}
    a = render.render_image(sub, W, H, tiles=tiles)
    for _ in range(4):
        p8 = project.project_threaded(sc, ids, cam, threads=8, chunk=1 << 18)
        for k in p1:
            assert np.array_equal(p1[k], p8[k]), k
        q8 = lod.predicates_threaded(sc, cam, 2.0, threads=8, chunk=1 << 18)
        for k in q1:
            assert np.array_equal(q1[k], q8[k]), k
        b = render.render_image(sub, W, H, tiles=tiles, threads=8, chunk=4096)
        for k in a:
            assert np.array_equal(a[k], b[k], equal_nan=True), k
