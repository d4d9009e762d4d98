"""The regrouping behind the Gaussian's stored planes, checked on the CPU.

A window histogram of the series kernel (Sec. 2.1, Eq. 2 per weight term) is
H(xc, yc) = sum_ij alpha_i(xc) beta_j(yc) box_ij.  The library never stores
the terms' prefix sums P_ij: it keeps tile-local sums contracted with the
coefficients of the windows each stored point is a corner of, the band-closing
rows contracted over x only, and the tile-origin carries contracted over y.
This test rebuilds those stored quantities in float64 numpy from their
definitions and checks that the lookup formula the kernels use (four corners,
the crossings, the carry boxes, and the count the same way) gives the plain
box sum at every valid window, for windows shorter and taller than a band,
with the left edge on column 0, and across several tiles.  It checks the
algebra only (no rounding, no device code).
"""
import numpy as np
import pytest

TW = 64  # tile width: one lane per column


def coeffs(a, om, c):
    """Series coefficients at centre c: (a0, a_k cos(w_k c), a_k sin(w_k c))."""
    c = np.asarray(c, dtype=np.float64)
    out = [np.full(c.shape, a[0])]
    for k in range(1, len(a)):
        out += [a[k] * np.cos(om[k] * c), a[k] * np.sin(om[k] * c)]
    return np.stack(out, axis=-1)


def basis(om, t):
    """Terms (1, cos w_k t, sin w_k t) at coordinate t."""
    t = np.asarray(t, dtype=np.float64)
    out = [np.ones(t.shape)]
    for k in range(1, len(om)):
        out += [np.cos(om[k] * t), np.sin(om[k] * t)]
    return np.stack(out, axis=-1)


def stored(mask, ax, omx, ay, omy, rx, ry, TY):
    H, W = mask.shape
    u = basis(omx, np.arange(W))          # [W, NT]
    v = basis(omy, np.arange(H))          # [H, NT]
    NT = u.shape[1]
    # P_ij[Y][X], zero row and column
    terms = mask[:, :, None, None] * u[None, :, :, None] * v[:, None, None, :]   # [y, x, i, j]
    P = np.zeros((H + 1, W + 1, NT, NT))
    P[1:, 1:] = terms.cumsum(0).cumsum(1)
    Y = np.arange(H + 1)
    X = np.arange(W + 1)
    Yo = np.where(Y > 0, ((Y - 1) // TY) * TY, 0)
    Xo = np.where(X > 0, ((X - 1) // TW) * TW, 0)
    L = P - P[Yo] - P[:, Xo] + P[Yo][:, Xo]          # tile-local sums
    ap = coeffs(ax, omx, np.maximum(X - rx - 1, 0))                  # X as a right edge
    am = coeffs(ax, omx, X + rx)                                    # X as a left edge
    bB = coeffs(ay, omy, np.maximum(Y - ry - 1, 0))                  # Y as a bottom edge
    bT = coeffs(ay, omy, Y + ry)                                    # Y as a top edge
    Vp = np.einsum('xi,yxij->yxj', ap, L)
    Vm = np.einsum('xi,yxij->yxj', am, L)
    C = {"RB": np.einsum('yj,yxj->yx', bB, Vp), "RT": np.einsum('yj,yxj->yx', bT, Vp),
         "LB": np.einsum('yj,yxj->yx', bB, Vm), "LT": np.einsum('yj,yxj->yx', bT, Vm),
         "N": L[:, :, 0, 0]}
    NTX = (W + TW - 1) // TW
    RC = P[:, [TW * t for t in range(NTX)]]                          # [Y, tx, i, j]
    RCB = np.einsum('yj,ytij->yti', bB, RC)
    RCT = np.einsum('yj,ytij->yti', bT, RC)
    RCN = RC[:, :, 0, 0]
    return C, Vp, Vm, RCB, RCT, RCN, P


def lookup(st, ax, omx, ay, omy, rx, ry, TY, H, W):
    """The kernels' lookup at every valid centre: (histogram, count) maps."""
    C, Vp, Vm, RCB, RCT, RCN, _ = st
    yc, xc = np.meshgrid(np.arange(ry, H - ry), np.arange(rx, W - rx), indexing='ij')
    XR, XL, Ya, Yb = xc + rx + 1, xc - rx, yc - ry, yc + ry + 1
    top = (Ya % TY) != 0
    left = XL > 0
    tile = lambda Xc: (np.maximum(Xc, 1) - 1) // TW

    def corners(name_r, name_l, Yr):
        return C[name_r][Yr, XR] - np.where(left, C[name_l][Yr, XL], 0.0)

    h = corners("RB", "LB", Yb) - np.where(top, corners("RT", "LT", Ya), 0.0)
    n = (C["N"][Yb, XR] - np.where(left, C["N"][Yb, XL], 0.0)
         - np.where(top, C["N"][Ya, XR] - np.where(left, C["N"][Ya, XL], 0.0), 0.0))
    be = coeffs(ay, omy, yc)
    for c in range(TY, H, TY):  # the band-closing rows strictly inside each window
        inside = (Ya < c) & (c < Yb)
        dv = Vp[c, XR] - np.where(left[..., None], Vm[c, XL], 0.0)
        h = h + np.where(inside, (be * dv).sum(-1), 0.0)
        n = n + np.where(inside, C["N"][c, XR] - np.where(left, C["N"][c, XL], 0.0), 0.0)
    al = coeffs(ax, omx, xc)
    tR, tL = tile(XR), tile(XL)
    box = (RCB[Yb, tR] - RCT[Ya, tR]) - np.where(left[..., None], RCB[Yb, tL] - RCT[Ya, tL], 0.0)
    h = h + (al * box).sum(-1)
    n = n + (RCN[Yb, tR] - RCN[Ya, tR]) - np.where(left, RCN[Yb, tL] - RCN[Ya, tL], 0.0)
    return h, n, (yc, xc)


def direct(mask, ax, omx, ay, omy, rx, ry, centres):
    """The plain definition: the box sum of the translated series kernel."""
    yc, xc = centres
    dx = np.arange(-rx, rx + 1)
    dy = np.arange(-ry, ry + 1)
    kx = (coeffs(ax, omx, np.zeros(1))[0] * basis(omx, dx)).sum(-1)  # g_x(dx)
    ky = (coeffs(ay, omy, np.zeros(1))[0] * basis(omy, dy)).sum(-1)
    k2 = ky[:, None] * kx[None, :]
    h = np.zeros(yc.shape)
    n = np.zeros(yc.shape)
    for a in range(2 * ry + 1):
        for b in range(2 * rx + 1):
            m = mask[yc - ry + a, xc - rx + b]
            h += k2[a, b] * m
            n += m
    return h, n


@pytest.mark.parametrize("H,W,TY,rx,ry", [(70, 150, 16, 3, 5),     # windows within a band or one crossing
                                          (70, 150, 16, 20, 21),   # several crossings per window
                                          (48, 140, 32, 0, 0),     # 1 x 1 windows
                                          (66, 131, 64, 9, 31)])   # ragged edges, Ya on band rows
def test_corner_contracted_lookup_equals_box_sum(H, W, TY, rx, ry):
    rng = np.random.default_rng(H * 1000 + W + rx)
    mask = (rng.random((H, W)) < 0.4).astype(np.float64)
    K = 2
    ax = rng.uniform(0.2, 1.0, K + 1)
    ay = rng.uniform(0.2, 1.0, K + 1)
    omx = np.concatenate([[0.0], np.sort(rng.uniform(0.1, 2.5, K))])
    omy = np.concatenate([[0.0], np.sort(rng.uniform(0.1, 2.5, K))])
    st = stored(mask, ax, omx, ay, omy, rx, ry, TY)
    h, n, centres = lookup(st, ax, omx, ay, omy, rx, ry, TY, H, W)
    hd, nd = direct(mask, ax, omx, ay, omy, rx, ry, centres)
    scale = np.abs(hd).max() + 1.0
    assert np.abs(h - hd).max() <= 1e-9 * scale
    assert np.array_equal(np.rint(n), nd) and np.abs(n - nd).max() < 1e-6
    # the windows with the left edge on column 0 and with the top on a band row are covered
    assert (centres[1] == rx).any()
    assert ((centres[0] - ry) % TY == 0).any()


def test_dropping_a_crossing_is_caught():
    # the check above would see a lookup that forgot one band-closing row
    H, W, TY, rx, ry = 70, 150, 16, 4, 12
    rng = np.random.default_rng(7)
    mask = (rng.random((H, W)) < 0.5).astype(np.float64)
    a = np.array([0.5, 0.3, 0.2]); om = np.array([0.0, 0.7, 1.9])
    st = stored(mask, a, om, a, om, rx, ry, TY)
    C, Vp, Vm, RCB, RCT, RCN, P = st
    Vp = Vp.copy()
    Vp[TY] = 0.0  # lose the first band-closing row
    h, _, centres = lookup((C, Vp, Vm, RCB, RCT, RCN, P), a, om, a, om, rx, ry, TY, H, W)
    hd, _ = direct(mask, a, om, a, om, rx, ry, centres)
    assert np.abs(h - hd).max() > 1e-3
