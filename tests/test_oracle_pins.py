"""Pins for the CPU oracle: checks against facts the paper and mathematics fix.

None of these retypes the oracle's own loop.  Each test is chosen so that a
plausible slip in the oracle (a dropped kernel term, a wrong sign, a swapped
dx/dy, an off-by-one window edge, a wrong normaliser) fails at least one:

* closed-form kernel masses (golden file, worked by hand from sum formulas;
  geometric series for the exponential kernel);
* the exponential table is the product of two 1-D profiles with a constant
  ratio between neighbouring weights (the defining property of exp(-|d|/tau));
* sum_b H_b = S at every centre (normalisation independent of location,
  Sec. 2.1 of the paper);
* a constant image puts all mass in one bin; the likelihood map is 1;
* a single-pixel impulse reproduces the point-reflected kernel table;
* mirroring the image mirrors the histogram maps (the kernels are symmetric,
  the quadrant argument of Sec. 2.1);
* the uniform kernel equals box counts from a numpy cumulative-sum integral
  histogram (the plain integral histogram of Sec. 1);
* raising the Manhattan constant by D raises H_b by D * count_b;
* the Bhattacharyya coefficient is 1 on the template, within [0, 1] (Cauchy-
  Schwarz) and 0 for disjoint supports;
* brute force agrees with a naive Python loop (tiny images) and with the
  independent per-bin separable correlation (all kernels, odd non-square
  windows, several bin counts).
"""
import math
import os

import numpy as np
import pytest

import oracle
import oracle.separable as sep
from paper_1705_03524_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
INT_KINDS = (oracle.UNIFORM, oracle.MANHATTAN, oracle.EUCLIDEAN)
ALL_KINDS = INT_KINDS + (oracle.GAUSSIAN, oracle.EXPONENTIAL)
NAMES = {"uniform": oracle.UNIFORM, "manhattan": oracle.MANHATTAN, "euclidean": oracle.EUCLIDEAN}


def valid_centres(H, W, w, h):
    rx, ry = (w - 1) // 2, (h - 1) // 2
    return np.array([(x, y) for y in range(ry, H - ry) for x in range(rx, W - rx)], np.int32)


# ---------------------------------------------------------------- quantiser
@pytest.mark.parametrize("nbins", [1, 2, 3, 7, 8, 16, 32, 100, 256])
def test_quantiser_uniform_bins(nbins):
    q = np.array([oracle.quantise(v, nbins) for v in range(256)])
    assert q[0] == 0 and q[255] == nbins - 1
    assert np.all(np.diff(q) >= 0) and np.all(np.diff(q) <= 1)
    widths = np.bincount(q, minlength=nbins)
    assert widths.min() >= 256 // nbins and widths.max() <= -(-256 // nbins)


def test_quantiser_power_of_two_is_shift():
    for v in range(256):
        assert oracle.quantise(v, 8) == v >> 5
        assert oracle.quantise(v, 16) == v >> 4
        assert oracle.quantise(v, 32) == v >> 3


# ---------------------------------------------------------------- kernel masses
def test_golden_masses():
    n = 0
    with open(os.path.join(GOLD, "kernel_masses.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            kind, w, h, S = line.split()
            assert oracle.mass(NAMES[kind], int(w), int(h)) == int(S), line
            n += 1
    assert n >= 8


@pytest.mark.parametrize("w,h", [(3, 3), (5, 3), (3, 9), (15, 15), (31, 31), (61, 91), (81, 81)])
def test_masses_closed_form(w, h):
    rx, ry = (w - 1) // 2, (h - 1) // 2
    sa = lambda r: r * (r + 1)                  # sum_{d=-r..r} |d|
    s2 = lambda r: r * (r + 1) * (2 * r + 1) // 3  # sum_{d=-r..r} d^2
    assert oracle.mass(oracle.UNIFORM, w, h) == w * h
    assert oracle.mass(oracle.MANHATTAN, w, h) == w * h * (rx + ry + 1) - h * sa(rx) - w * sa(ry)
    assert oracle.mass(oracle.EUCLIDEAN, w, h) == w * h * (rx * rx + ry * ry + 1) - h * s2(rx) - w * s2(ry)
    sx, sy = w / 4.0, h / 4.0
    gx = sum(math.exp(-d * d / (2 * sx * sx)) for d in range(-rx, rx + 1))
    gy = sum(math.exp(-d * d / (2 * sy * sy)) for d in range(-ry, ry + 1))
    assert oracle.mass(oracle.GAUSSIAN, w, h) == pytest.approx(gx * gy, rel=1e-13)
    # exponential: 1 + 2 (q + q^2 + ... + q^r) = 1 + 2 q (1 - q^r) / (1 - q), q = exp(-1 / tau)
    geo = lambda r, tau: 1 + 2 * math.exp(-1 / tau) * (1 - math.exp(-r / tau)) / (1 - math.exp(-1 / tau))
    assert oracle.mass(oracle.EXPONENTIAL, w, h) == pytest.approx(geo(rx, w / 4.0) * geo(ry, h / 4.0), rel=1e-13)


@pytest.mark.parametrize("w,h", [(3, 3), (7, 5), (5, 11), (31, 31), (61, 91)])
def test_exponential_table_structure(w, h):
    t = oracle.kernel_table(oracle.EXPONENTIAL, w, h)
    rx, ry = (w - 1) // 2, (h - 1) // 2
    assert t[ry, rx] == 1.0
    np.testing.assert_allclose(t, t[::-1, :], rtol=0, atol=0)
    np.testing.assert_allclose(t, t[:, ::-1], rtol=0, atol=0)
    # rank one: k(dx, dy) = k(dx, 0) k(0, dy)
    np.testing.assert_allclose(t, np.outer(t[:, rx], t[ry, :]), rtol=1e-14)
    # a constant ratio between neighbouring weights moving out from the centre,
    # the x ratio set by w alone and the y ratio by h alone
    qx = t[ry, rx + 1:] / t[ry, rx:-1] if rx else np.array([])
    qy = t[ry + 1:, rx] / t[ry:-1, rx] if ry else np.array([])
    if rx:
        np.testing.assert_allclose(qx, qx[0], rtol=1e-13)
        assert 0 < qx[0] < 1
        tt = oracle.kernel_table(oracle.EXPONENTIAL, h, w)
        np.testing.assert_allclose(tt.T, t, rtol=1e-15)   # widths follow the sides, not the axes
    if ry:
        np.testing.assert_allclose(qy, qy[0], rtol=1e-13)
    if rx and ry and w != h:
        assert qx[0] != pytest.approx(qy[0])
    # widths side / 4: the weight at distance d along x is q^d with q^(w/4) = 1/e
    if rx:
        assert qx[0] ** (w / 4.0) == pytest.approx(math.exp(-1), rel=1e-13)


@pytest.mark.parametrize("w,h", [(3, 3), (7, 5), (5, 11), (31, 31), (61, 91), (81, 21)])
def test_gaussian_table_structure(w, h):
    # the true Gaussian with sigma = side / 4 per axis, pinned by its shape
    # rather than by its formula: peak 1 at the centre, mirror symmetric, rank
    # one, and log k a parabola along each axis whose second difference is
    # -1 / sigma^2 with sigma set by that axis's own side
    t = oracle.kernel_table(oracle.GAUSSIAN, w, h)
    rx, ry = (w - 1) // 2, (h - 1) // 2
    assert t[ry, rx] == 1.0
    np.testing.assert_allclose(t, t[::-1, :], rtol=0, atol=0)
    np.testing.assert_allclose(t, t[:, ::-1], rtol=0, atol=0)
    np.testing.assert_allclose(t, np.outer(t[:, rx], t[ry, :]), rtol=1e-14)
    assert np.all(t > 0) and np.all(t <= 1.0)
    lx, ly = np.log(t[ry, :]), np.log(t[:, rx])
    if w >= 3:
        np.testing.assert_allclose(lx[2:] - 2 * lx[1:-1] + lx[:-2], -1.0 / (w / 4.0) ** 2, rtol=1e-9)
    if h >= 3:
        np.testing.assert_allclose(ly[2:] - 2 * ly[1:-1] + ly[:-2], -1.0 / (h / 4.0) ** 2, rtol=1e-9)
    # a wrong sign of the exponent, a missing factor 1/2 or sigma from the wrong
    # side would each move the corner weight: exp(-(rx/sx)^2/2 - (ry/sy)^2/2)
    corner = math.exp(-0.5 * (rx / (w / 4.0)) ** 2 - 0.5 * (ry / (h / 4.0)) ** 2)
    assert t[0, 0] == pytest.approx(corner, rel=1e-12)
    if w != h:
        np.testing.assert_allclose(oracle.kernel_table(oracle.GAUSSIAN, h, w).T, t, rtol=1e-15)


def test_manhattan_table_follows_eq1_distance():
    # weights fall by one per unit of city-block distance from the centre and
    # are 1 at the window corners
    for w, h in [(7, 5), (15, 15), (3, 11)]:
        t = oracle.kernel_table(oracle.MANHATTAN, w, h)
        rx, ry = (w - 1) // 2, (h - 1) // 2
        dist = np.abs(np.arange(-rx, rx + 1))[None, :] + np.abs(np.arange(-ry, ry + 1))[:, None]
        assert np.all(t + dist == t[ry, rx])
        assert t[0, 0] == t[0, -1] == t[-1, 0] == t[-1, -1] == 1


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("kind", ALL_KINDS)
def test_mass_invariant_every_centre(kind):
    img = synth.uniform_noise(11, 40, 37)
    w, h = 9, 7
    c = valid_centres(40, 37, w, h)
    hb = oracle.hist(img, 5, kind, w, h, c)
    S = oracle.mass(kind, w, h)
    if kind in oracle.REAL_KINDS:
        np.testing.assert_allclose(hb.sum(1), S, rtol=1e-13)
    else:
        assert np.all(hb.sum(1) == S)


@pytest.mark.parametrize("kind", ALL_KINDS)
@pytest.mark.parametrize("v", [0, 77, 255])
def test_constant_image(kind, v):
    nb = 8
    img = np.full((24, 30), v, np.uint8)
    w, h = 7, 11
    c = valid_centres(24, 30, w, h)
    hb = oracle.hist(img, nb, kind, w, h, c)
    S = oracle.mass(kind, w, h)
    b = (v * nb) // 256
    expect = np.zeros(nb)
    expect[b] = S
    np.testing.assert_allclose(hb, np.broadcast_to(expect, hb.shape), rtol=1e-14)
    raw, p = oracle.template(img, nb, kind, w, h, (15, 12))
    m = oracle.bc_map(img, nb, kind, w, h, raw if kind not in oracle.REAL_KINDS else p)
    np.testing.assert_allclose(m, 1.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("kind", ALL_KINDS)
def test_impulse_reproduces_reflected_kernel(kind):
    H, W, nb = 21, 26, 4
    w, h = 7, 5                      # non-square: a dx/dy swap would show
    px, py = 13, 9
    img = np.zeros((H, W), np.uint8)
    img[py, px] = 255                # bin nb-1; background bin 0
    tab = oracle.kernel_table(kind, w, h)
    rx, ry = (w - 1) // 2, (h - 1) // 2
    c = valid_centres(H, W, w, h)
    hb = oracle.hist(img, nb, kind, w, h, c)
    S = oracle.mass(kind, w, h)
    for (xc, yc), row in zip(c, hb):
        dx, dy = px - xc, py - yc
        inside = abs(dx) <= rx and abs(dy) <= ry
        expect = tab[dy + ry, dx + rx] if inside else 0
        assert row[nb - 1] == pytest.approx(expect, rel=1e-15, abs=0)
        assert row[0] == pytest.approx(S - expect, rel=1e-13, abs=1e-12)
        assert np.all(row[1:nb - 1] == 0)


@pytest.mark.parametrize("kind", INT_KINDS)
def test_two_impulses_add(kind):
    H, W, nb, w, h = 19, 19, 2, 5, 7
    a = np.zeros((H, W), np.uint8); a[8, 9] = 200
    b = np.zeros((H, W), np.uint8); b[10, 7] = 200
    ab = a | b
    c = valid_centres(H, W, w, h)
    ha, hb_, hab = (oracle.hist(x, nb, kind, w, h, c)[:, 1] for x in (a, b, ab))
    assert np.array_equal(ha + hb_, hab)


@pytest.mark.parametrize("kind", ALL_KINDS)
def test_mirror_symmetry(kind):
    img = synth.uniform_noise(5, 23, 29)
    w, h, nb = 9, 5, 6
    full = sep.hist_maps(img, nb, kind, w, h)
    mx = sep.hist_maps(img[:, ::-1], nb, kind, w, h)
    my = sep.hist_maps(img[::-1, :], nb, kind, w, h)
    c = valid_centres(23, 29, w, h)
    ob = oracle.hist(img, nb, kind, w, h, c)
    obx = oracle.hist(np.ascontiguousarray(img[:, ::-1]), nb, kind, w, h, c)
    oby = oracle.hist(np.ascontiguousarray(img[::-1, :]), nb, kind, w, h, c)
    sh = (23 - h + 1, 29 - w + 1, nb)
    np.testing.assert_allclose(obx.reshape(sh), ob.reshape(sh)[:, ::-1], rtol=1e-13)
    np.testing.assert_allclose(oby.reshape(sh), ob.reshape(sh)[::-1, :], rtol=1e-13)
    np.testing.assert_allclose(mx, full[:, :, ::-1], rtol=1e-13)
    np.testing.assert_allclose(my, full[:, ::-1, :], rtol=1e-13)


def test_uniform_kernel_is_plain_integral_histogram():
    img = synth.smooth_noise(3, 48, 53)
    nb, w, h = 16, 11, 7
    q = (img.astype(np.int64) * nb) // 256
    c = valid_centres(48, 53, w, h)
    hb = oracle.hist(img, nb, oracle.UNIFORM, w, h, c)
    rx, ry = (w - 1) // 2, (h - 1) // 2
    for b in range(nb):
        ih = np.zeros((49, 54), np.int64)
        ih[1:, 1:] = np.cumsum(np.cumsum(q == b, 0), 1)
        xc, yc = c[:, 0], c[:, 1]
        box = (ih[yc + ry + 1, xc + rx + 1] - ih[yc - ry, xc + rx + 1]
               - ih[yc + ry + 1, xc - rx] + ih[yc - ry, xc - rx])
        assert np.array_equal(box, hb[:, b])


def test_manhattan_constant_is_linear():
    img = synth.uniform_noise(8, 30, 30)
    nb, w, h = 7, 9, 9
    c = valid_centres(30, 30, w, h)
    tab = oracle.kernel_table(oracle.MANHATTAN, w, h)
    base = oracle.hist(img, nb, oracle.MANHATTAN, w, h, c)
    count = oracle.hist(img, nb, oracle.UNIFORM, w, h, c)
    for D in (1, 5, -3):
        shifted = oracle.hist(img, nb, oracle.MANHATTAN, w, h, c, table=tab + D)
        assert np.array_equal(shifted - base, D * count)


# ---------------------------------------------------------------- likelihood
@pytest.mark.parametrize("kind", ALL_KINDS)
def test_bc_self_match_and_bounds(kind):
    img, _ = synth.rect_scene(2, 64, 64, nrect=3)
    nb, w, h = 16, 15, 15
    raw, p = oracle.template(img, nb, kind, w, h, (30, 33))
    m = oracle.bc_map(img, nb, kind, w, h, raw if kind not in oracle.REAL_KINDS else p)
    assert m[33 - 7, 30 - 7] == pytest.approx(1.0, abs=2e-15)
    assert m.min() >= 0.0 and m.max() <= 1.0 + 2e-15


def test_bc_disjoint_is_zero():
    img = np.zeros((20, 40), np.uint8)
    img[:, 20:] = 255
    raw, _ = oracle.template(img, 4, oracle.MANHATTAN, 5, 5, (5, 10))
    bc = oracle.bc_at(img, 4, oracle.MANHATTAN, 5, 5, [(30, 10)], raw)
    assert bc[0] == 0.0


def test_bc_integer_form_matches_definition():
    # sum_b sqrt(p_b t_b) evaluated from normalised histograms in numpy
    img = synth.uniform_noise(4, 40, 40)
    nb, w, h = 8, 9, 9
    c = valid_centres(40, 40, w, h)[::7]
    raw, p = oracle.template(img, nb, oracle.EUCLIDEAN, w, h, (20, 20))
    bc = oracle.bc_at(img, nb, oracle.EUCLIDEAN, w, h, c, raw)
    pc = oracle.normalised(oracle.hist(img, nb, oracle.EUCLIDEAN, w, h, c), oracle.EUCLIDEAN, w, h)
    np.testing.assert_allclose(bc, np.sqrt(pc * p[None, :]).sum(1), rtol=1e-14, atol=1e-15)


# ---------------------------------------------------------------- cross-checks
def naive_hist(img, nb, kind, w, h, xc, yc):
    rx, ry = (w - 1) // 2, (h - 1) // 2
    out = [0.0] * nb
    for y in range(yc - ry, yc + ry + 1):
        for x in range(xc - rx, xc + rx + 1):
            dx, dy = abs(x - xc), abs(y - yc)
            if kind == oracle.UNIFORM:
                k = 1
            elif kind == oracle.MANHATTAN:
                k = rx + ry + 1 - dx - dy
            elif kind == oracle.EUCLIDEAN:
                k = rx * rx + ry * ry + 1 - dx * dx - dy * dy
            elif kind == oracle.GAUSSIAN:
                k = math.exp(-dx * dx / (2 * (w / 4) ** 2)) * math.exp(-dy * dy / (2 * (h / 4) ** 2))
            else:
                k = math.exp(-dx / (w / 4)) * math.exp(-dy / (h / 4))
            out[int(img[y, x]) * nb // 256] += k
    return out


@pytest.mark.parametrize("kind", ALL_KINDS)
@pytest.mark.parametrize("nb", [1, 2, 3, 8, 256])
@pytest.mark.parametrize("wh", [(3, 3), (5, 3), (15, 9)])
def test_brute_force_vs_naive_loop(kind, nb, wh):
    w, h = wh
    img = synth.uniform_noise(100 + nb, 16, 16)
    c = valid_centres(16, 16, w, h)
    hb = oracle.hist(img, nb, kind, w, h, c)
    for (xc, yc), row in zip(c, hb):
        np.testing.assert_allclose(row, naive_hist(img, nb, kind, w, h, xc, yc), rtol=1e-14, atol=0)


@pytest.mark.parametrize("kind", ALL_KINDS)
@pytest.mark.parametrize("nb,wh", [(2, (3, 5)), (8, (15, 15)), (16, (31, 31)), (5, (21, 7))])
def test_brute_force_vs_separable(kind, nb, wh):
    w, h = wh
    img = synth.smooth_noise(7 + nb, 70, 66)
    c = valid_centres(70, 66, w, h)
    hb = oracle.hist(img, nb, kind, w, h, c)
    sm = sep.hist_maps(img, nb, kind, w, h)
    got = sm.transpose(1, 2, 0).reshape(-1, nb)
    if kind in oracle.REAL_KINDS:
        np.testing.assert_allclose(hb, got, rtol=1e-12, atol=1e-12)
    else:
        assert np.array_equal(hb, got)


def test_outside_centre_rejected():
    img = synth.uniform_noise(0, 10, 10)
    with pytest.raises(ValueError):
        oracle.hist(img, 4, oracle.MANHATTAN, 5, 5, [(1, 5)])
    with pytest.raises(ValueError):
        oracle.bc_map(img, 4, oracle.MANHATTAN, 5, 5, np.ones(4, np.int64), rect=(2, 2, 8, 7))


def test_generators_are_seeded():
    a = synth.rect_scene(9, 50, 60)[0]
    b = synth.rect_scene(9, 50, 60)[0]
    assert np.array_equal(a, b)
    s = synth.smooth_noise(1, 64, 64)
    assert s.min() == 0 and s.max() == 255
    cs = synth.sample_centres(1, 100, 80, 15, 9, 100)
    assert cs.shape == (100, 2)
    assert cs[:, 0].min() == 7 and cs[:, 0].max() == 80 - 8
    assert cs[:, 1].min() == 4 and cs[:, 1].max() == 100 - 5


# ---------------------------------------------------------------- wedding cake
# Sec. 2 (Fig. 4a): nested windows, one weight per ring.  Pins: the ring
# geometry, the one-ring case (a scaled plain histogram), mass preservation, a
# ring-constant kernel reproduced exactly, and convergence toward the kernel.
@pytest.mark.parametrize("w,h,n", [(31, 31, 1), (31, 31, 4), (15, 9, 3), (61, 91, 8), (5, 5, 7), (1, 9, 2)])
def test_cake_ring_geometry(w, h, n):
    rings = oracle.cake_rings(w, h, n)
    rx, ry = (w - 1) // 2, (h - 1) // 2
    assert rings[0] == (rx, ry)
    for (ax, ay), (bx, by) in zip(rings, rings[1:]):
        assert bx <= ax and by <= ay
    ring = oracle.cake_ring_index(w, h, n)
    sizes = [(2 * ax + 1) * (2 * ay + 1) if ax >= 0 and ay >= 0 else 0 for ax, ay in rings] + [0]
    for i in range(n):
        assert (ring == i).sum() == sizes[i] - sizes[i + 1]
    assert ring[ry, rx] == max(i for i, (ax, ay) in enumerate(rings) if ax >= 0 and ay >= 0)
    if n <= min(rx, ry) + 1:    # equal runs of distance: every ring is non-empty
        assert all(sizes[i] > sizes[i + 1] for i in range(n))
    assert ring[0, 0] == max(i for i, r in enumerate(rings) if r == rings[0])  # outermost non-empty ring


@pytest.mark.parametrize("kind", (oracle.MANHATTAN, oracle.EUCLIDEAN, oracle.GAUSSIAN))
def test_cake_one_ring_is_scaled_plain_histogram(kind):
    img = synth.uniform_noise(21, 30, 34)
    w, h, nb = 9, 7, 5
    c = valid_centres(30, 34, w, h)
    cake = oracle.hist(img, nb, kind, w, h, c, table=oracle.cake_table(kind, w, h, 1))
    plain = oracle.hist(img, nb, oracle.UNIFORM, w, h, c)
    S = oracle.mass(kind, w, h)
    np.testing.assert_allclose(cake, plain * (S / (w * h)), rtol=1e-13)


@pytest.mark.parametrize("kind", (oracle.MANHATTAN, oracle.EUCLIDEAN, oracle.EXPONENTIAL))
@pytest.mark.parametrize("n", [2, 5, 16])
def test_cake_keeps_mass(kind, n):
    w, h = 21, 15
    t = oracle.cake_table(kind, w, h, n)
    assert t.sum() == pytest.approx(oracle.mass(kind, w, h), rel=1e-13)
    img = synth.smooth_noise(3, 40, 40)
    hb = oracle.hist(img, 8, kind, w, h, valid_centres(40, 40, w, h)[::13], table=t)
    np.testing.assert_allclose(hb.sum(1), oracle.mass(kind, w, h), rtol=1e-12)


@pytest.mark.parametrize("w,h,n", [(15, 15, 4), (21, 9, 3), (31, 31, 8)])
def test_cake_reproduces_ring_constant_kernel(w, h, n):
    # k = number of nested windows holding the pixel: constant on every ring
    rx, ry = (w - 1) // 2, (h - 1) // 2
    k = np.zeros((h, w), np.int64)
    for ax, ay in oracle.cake_rings(w, h, n):
        if ax >= 0 and ay >= 0:
            k[ry - ay:ry + ay + 1, rx - ax:rx + ax + 1] += 1
    img = synth.uniform_noise(9, 45, 50)
    c = valid_centres(45, 50, w, h)[::5]
    exact = oracle.hist(img, 6, oracle.MANHATTAN, w, h, c, table=k)
    # the cake of k (ring means of k) must be k itself
    ring = oracle.cake_ring_index(w, h, n)
    means = np.array([k[ring == i].mean() for i in range(n)])
    cake = oracle.hist(img, 6, oracle.MANHATTAN, w, h, c, table=means[ring])
    np.testing.assert_allclose(cake, exact, rtol=1e-14)


def test_cake_error_falls_with_rings_but_stays_for_the_diamond():
    # square rings approach the kernel as they multiply, but the Manhattan
    # pyramid varies inside a square shell (corner vs edge), so even one ring
    # per shell leaves an error: the point of Sec. 2.1's exact method
    w = h = 31
    k = oracle.kernel_table(oracle.MANHATTAN, w, h).astype(np.float64)
    err = [np.abs(oracle.cake_table(oracle.MANHATTAN, w, h, n) - k).sum() / k.sum() for n in (1, 2, 4, 8, 16)]
    assert all(b < a for a, b in zip(err, err[1:]))
    shells = oracle.cake_table(oracle.MANHATTAN, w, h, 16)   # 16 rings = every shell of a 31 x 31
    assert len(set(oracle.cake_rings(w, h, 16))) == 16
    dist = np.maximum.outer(np.abs(np.arange(-15, 16)), np.abs(np.arange(-15, 16)))
    for d in range(16):                                       # shell mean of the pyramid
        assert np.allclose(shells[dist == d], k[dist == d].mean())
    assert err[-1] > 0.1
