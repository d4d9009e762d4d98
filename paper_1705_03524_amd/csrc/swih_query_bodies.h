// Window histograms from the weighted integral histograms (Sec. 2.1) and the
// Bhattacharyya likelihood map (Sec. 2 Fig. 3, Sec. 4).
//
// Translation (Sec. 2.1): a kernel weight k(x - xc, y - yc) is written as a
// sum of image-wide weight terms u_i(x) v_j(y) times coefficients that depend
// only on the centre, so each window histogram is a few O(1) box lookups.
//
//   Manhattan, quadrant by quadrant (Fig. 4b), c = rx + ry + 1:
//     TL [xc-rx, xc] x [yc-ry, yc]      (c - xc - yc) B_1 + B_x + B_y
//     TR [xc+1, xc+rx] x [yc-ry, yc]    (c + xc - yc) B_1 - B_x + B_y
//     BL [xc-rx, xc] x [yc+1, yc+ry]    (c - xc + yc) B_1 + B_x - B_y
//     BR [xc+1, xc+rx] x [yc+1, yc+ry]  (c + xc + yc) B_1 - B_x - B_y
//   The four quadrants are disjoint, so the centre row and column count once.
//   Euclidean paraboloid, one box, c = rx^2 + ry^2 + 1:
//     (c - xc^2 - yc^2) B_1 + 2 xc B_x + 2 yc B_y - B_xx - B_yy
//   Gaussian, one box: sum_ij alpha_i(xc) beta_j(yc) B_ij with
//     alpha = (a_0, a_k cos(w_k xc), a_k sin(w_k xc)), w_k the series' frequencies.
// Integer coefficients are applied modulo 2^32; the true histogram is below
// 2^32, so the result is exact.  Normalisation divides by the kernel mass S
// (the same at every location, Sec. 2.1).
#pragma once

#include <string.h>

#include "swih_internal.h"
#include "wave64.h"

namespace swih {
namespace {

// Offsets of a window's corner lookups, the same for every plane and bin:
// rows {ya, ym, yb} x columns {xa, xm, xb}, ym = yc + 1, xm = xc + 1 (the
// Manhattan quadrant split; the other kernels use the outer four).  Column
// X = 0 is not stored and reads as 0: its offset points at column 1 and the
// value is dropped.
struct IntCorners {
  int64_t o[3][3];
  bool xa0;
};

__device__ __forceinline__ IntCorners int_corners(const SwihGeom& g, int xc, int yc,
                                                  const ScaleParams& sp) {
  IntCorners k;
  const int xa = xc - sp.rx;
  const int Ys[3] = {yc - sp.ry, yc + 1, yc + sp.ry + 1};
  const int64_t Xo[3] = {swih_xoff(g, xa > 0 ? xa : 1), swih_xoff(g, xc + 1),
                         swih_xoff(g, xc + sp.rx + 1)};
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) k.o[r][c] = (int64_t)Ys[r] * g.row_stride + Xo[c];
  k.xa0 = xa == 0;
  return k;
}

// P at corner (r, c) of the plane whose base (swih_base) is pl.
__device__ __forceinline__ uint32_t at_u(const uint32_t* __restrict__ pl, const IntCorners& k,
                                         int r, int c) {
  const uint32_t v = pl[k.o[r][c]];
  return c == 0 && k.xa0 ? 0u : v;
}

// Exact H_b of an integer kernel at the window of k (uint32 arithmetic modulo 2^32).
template <int KIND>
__device__ __forceinline__ uint32_t hist_int(const uint32_t* __restrict__ planes,
                                             const SwihGeom& g, int b, int xc, int yc,
                                             const ScaleParams& sp, const IntCorners& k) {
  const uint32_t* p0 = planes + swih_base(g, 0, b);
  if (KIND == 0) {
    return at_u(p0, k, 2, 2) - at_u(p0, k, 0, 2) - at_u(p0, k, 2, 0) + at_u(p0, k, 0, 0);
  } else if (KIND == 1) {
    const uint32_t* px = planes + swih_base(g, 1, b);
    const uint32_t* py = planes + swih_base(g, 2, b);
    // 3 x 3 corner grid per plane
    uint32_t c1[3][3], cx[3][3], cy[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        c1[r][c] = at_u(p0, k, r, c);
        cx[r][c] = at_u(px, k, r, c);
        cy[r][c] = at_u(py, k, r, c);
      }
    auto box = [](const uint32_t (&a)[3][3], int r, int c) {
      return a[r + 1][c + 1] - a[r][c + 1] - a[r + 1][c] + a[r][c];
    };
    const uint32_t c = sp.c_int, X = (uint32_t)xc, Y = (uint32_t)yc;
    const uint32_t tl = (c - X - Y) * box(c1, 0, 0) + box(cx, 0, 0) + box(cy, 0, 0);
    const uint32_t tr = (c + X - Y) * box(c1, 0, 1) - box(cx, 0, 1) + box(cy, 0, 1);
    const uint32_t bl = (c - X + Y) * box(c1, 1, 0) + box(cx, 1, 0) - box(cy, 1, 0);
    const uint32_t br = (c + X + Y) * box(c1, 1, 1) - box(cx, 1, 1) - box(cy, 1, 1);
    return tl + tr + bl + br;
  } else {
    uint32_t bx[5];
#pragma unroll
    for (int p = 0; p < 5; ++p) {
      const uint32_t* pl = planes + swih_base(g, p, b);
      bx[p] = at_u(pl, k, 2, 2) - at_u(pl, k, 0, 2) - at_u(pl, k, 2, 0) + at_u(pl, k, 0, 0);
    }
    const uint32_t X = (uint32_t)xc, Y = (uint32_t)yc;
    return (sp.c_int - X * X - Y * Y) * bx[0] + 2u * X * bx[1] + 2u * Y * bx[2] - bx[3] - bx[4];
  }
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <int KIND>
__device__ __forceinline__ void query_int(const QueryArgs& a, int vb) {
  const SwihGeom& g = a.g;
  const ScaleParams& sp = a.sp;
  const uint32_t* __restrict__ planes = (const uint32_t*)a.planes;
  const int32_t* __restrict__ centres = a.centres;
  const long t = (long)vb * 256 + threadIdx.x;
  if (t >= (long)a.n * g.B) return;
  const int k = (int)(t / g.B), b = (int)(t % g.B);
  const int xc = clampi(centres[2 * k], sp.rx, g.W - 1 - sp.rx);
  const int yc = clampi(centres[2 * k + 1], sp.ry, g.H - 1 - sp.ry);
  const uint32_t h = hist_int<KIND>(planes, g, b, xc, yc, sp, int_corners(g, xc, yc, sp));
  if (a.hist_raw) a.hist_raw[t] = h;
  if (a.hist) a.hist[t] = (float)((double)h / sp.mass);
}

template <int KIND>
__device__ __forceinline__ void match_int(const MatchArgs& a, int vb) {
  const SwihGeom& g = a.g;
  const ScaleParams& sp = a.sp;
  const uint32_t* __restrict__ planes = (const uint32_t*)a.planes;
  const float* __restrict__ tmpl = a.tmpl;
  const uint32_t* __restrict__ tmpl_raw = a.tmpl_raw;
  const int x0 = a.x0, y0 = a.y0, x1 = a.x1, y1 = a.y1;
  const int bx = vb % a.nbx, by = vb / a.nbx;
  const int xc = x0 + bx * 64 + (int)(threadIdx.x & 63);
  const int yc = y0 + by * 4 + (int)(threadIdx.x >> 6);
  if (xc > x1 || yc > y1) return;
  const IntCorners k = int_corners(g, xc, yc, sp);
  double acc = 0.0;
  for (int b = 0; b < g.B; ++b) {
    const uint32_t h = hist_int<KIND>(planes, g, b, xc, yc, sp, k);
    if (tmpl_raw) {
      acc += sqrt((double)h * (double)tmpl_raw[b]);
    } else {
      acc += sqrt(((double)h / sp.mass) * fmax((double)tmpl[b], 0.0));
    }
  }
  if (tmpl_raw) acc = acc / sp.mass;
  a.map[(size_t)(yc - y0) * (x1 - x0 + 1) + (xc - x0)] = (float)acc;
}

// ---------------------------------------------------------------- Gaussian
__device__ __forceinline__ int tile_of(int X) { return (X > 0 ? X - 1 : 0) >> 6; }

// One block per centre; threads over (bin, part) pairs, NT + 3 parts per bin,
// put the window's terms into LDS, then one thread per bin adds them in
// order.  With XR = xc + rx + 1, XL = xc - rx, Ya = yc - ry, Yb = yc + ry + 1:
//   part 0       the corners C_RB(Yb, XR) - C_LB(Yb, XL) - C_RT(Ya, XR) + C_LT(Ya, XL)
//   part 1       the crossings, sum_c sum_j beta_j(yc) (V+_j(c, XR) - V-_j(c, XL))
//   part 2 + i   alpha_i(xc) (RCB_i - RCT_i at the tile of XR, minus at the tile of XL)
//   part NT + 2  the pixel count box (plane N and the count carry: exact integers)
// c the band-closing rows strictly between Ya and Yb.  When Ya itself closes
// a band, its top corners cancel against the crossing at c = Ya, so neither
// is read.  A bin with no pixel in the window gets p_b = 0 exactly instead of
// a rounding residue.
template <int NT>
__device__ __forceinline__ void query_gauss(const QueryArgs& a, int vb) {
  const SwihGeom& g = a.g;
  const ScaleParams& sp = a.sp;
  const float* __restrict__ pl = (const float*)a.planes;
  const float* __restrict__ XC = a.XC;
  const double* __restrict__ RC = a.RC;
  const int32_t* __restrict__ centres = a.centres;
  constexpr int D = NT + 3;
  __syncthreads();  // LDS reuse across virtual blocks of one block
  extern __shared__ double part[];  // [B][NT + 3]
  const int k = vb;
  const int xc = clampi(centres[2 * k], sp.rx, g.W - 1 - sp.rx);
  const int yc = clampi(centres[2 * k + 1], sp.ry, g.H - 1 - sp.ry);
  double al[NT], be[NT];
  series_coeffs<NT>(sp.ax, xc, al);
  series_coeffs<NT>(sp.ay, yc, be);
  const int xa = xc - sp.rx, xb = xc + sp.rx + 1, ya = yc - sp.ry, yb = yc + sp.ry + 1;
  const int64_t rs = g.row_stride;
  const int txa = tile_of(xa), txb = tile_of(xb);
  // column X = 0 is not stored (it is zero): its loads go to column 1 and are dropped
  const bool xa0 = xa == 0;
  const bool top = (ya & (g.TY - 1)) != 0;
  const int c0 = ((ya >> g.lgTY) + 1) << g.lgTY;  // first crossing
  const int64_t oa = swih_xoff(g, xa0 ? 1 : xa), ob = swih_xoff(g, xb);
  // the count box at one column: rows ya, yb and the crossings
  auto nbox = [&](const float* pn, int64_t o) {
    double d = (double)pn[(size_t)yb * rs + o] - (top ? (double)pn[(size_t)ya * rs + o] : 0.0);
    for (int c = c0; c < yb; c += g.TY) d += (double)pn[(size_t)c * rs + o];
    return d;
  };
  auto rcbox = [&](int qb, int qt, int b) {
    return (RC[swih_rc(g, qb, b, txb, yb)] - RC[swih_rc(g, qt, b, txb, ya)]) -
           (RC[swih_rc(g, qb, b, txa, yb)] - RC[swih_rc(g, qt, b, txa, ya)]);
  };
  for (int it = threadIdx.x; it < g.B * D; it += blockDim.x) {
    const int b = it / D, r = it - (it / D) * D;
    const float* pb = pl + swih_base(g, 0, b);
    double v = 0.0;
    if (r == 0) {
      v = (double)pb[(size_t)yb * rs + ob] - (top ? (double)pb[(size_t)ya * rs + 64 + ob] : 0.0);
      if (!xa0)
        v -= (double)pb[(size_t)yb * rs + 128 + oa] -
             (top ? (double)pb[(size_t)ya * rs + 192 + oa] : 0.0);
    } else if (r == 1) {
      for (int c = c0; c < yb; c += g.TY) {
        const float* xr = XC + swih_xc(g, 0, b, c, xb);
        const float* xl = XC + swih_xc(g, NT, b, c, xa0 ? 1 : xa);
#pragma unroll
        for (int j = 0; j < NT; ++j)
          v = fma(be[j], (double)xr[j * 64] - (xa0 ? 0.0 : (double)xl[j * 64]), v);
      }
    } else if (r < NT + 2) {
      const int i = r - 2;
      v = al[i] * rcbox(i, NT + i, b);
    } else {
      v = nbox(pb + 256, ob) - (xa0 ? 0.0 : nbox(pb + 256, oa)) + rcbox(2 * NT, 2 * NT, b);
    }
    part[it] = v;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < g.B; b += blockDim.x) {
    double h = 0.0;
    for (int r = 0; r < NT + 2; ++r) h += part[b * D + r];
    if (part[b * D + NT + 2] == 0.0) h = 0.0;
    a.hist[(size_t)k * g.B + b] = (float)(h / sp.mass);
  }
}

// A block-uniform double made visibly uniform (kept in scalar registers).
__device__ __forceinline__ double uniform(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// A Gaussian map value is sum_b sqrt(p_b t_b).  Each bin's term is rounded to
// a multiple of 2^-29 and the terms are added as integers: exact, so the sum
// is the same whatever the order in which bins arrive (bin groups and integer
// atomics, or all bins in one block).  The sum is at most 1 (Cauchy-Schwarz;
// the rounding of p and t moves it by ~1e-6), so it fits an int32 with room
// to spare, and 2^-30 per bin is far below the float resolution of the result.
constexpr double kBcScale = 536870912.0;  // 2^29

__device__ __forceinline__ int32_t bc_term(double p, float t) {
  return (int32_t)__builtin_rint(sqrt(fmax(p, 0.0) * fmax((double)t, 0.0)) * kBcScale);
}

__device__ __forceinline__ float bc_value(int32_t q) { return (float)((double)q / kBcScale); }

// Empty bins.  sqrt is not Lipschitz at 0: a bin with no pixel in the window
// must give p_b = 0 exactly, or a rounding residue e of the float planes
// turns into sqrt(e t_b), orders of magnitude above e.  The plane N holds the
// plain pixel count (the weight term (0, 0), u_0 = v_0 = 1 exactly), and
// every part of its box is an integer (tile-local float values below 2^24,
// double carries), so the count is exact and the maps drop a bin's term
// exactly when it is 0.

// Gaussian maps: the window sweep.
//
// A window's histogram is H_b(xc, yc) = sum_ij alpha_i(xc) beta_j(yc) B_ij,
// B_ij the box of term (i, j).  The planes hold, at every (Y, X), the
// tile-local sums already contracted with the coefficients of the windows
// that have (Y, X) as a corner, so with XR = xc + rx + 1, XL = xc - rx,
// Ya = yc - ry, Yb = yc + ry + 1 the window's corners and edges,
//   H_b = C_RB(Yb, XR) - C_LB(Yb, XL) - C_RT(Ya, XR) + C_LT(Ya, XL)
//         + sum_c sum_j beta_j(yc) (V+_j(c, XR) - V-_j(c, XL))
//         + sum_i alpha_i(xc) (RCB_i(Yb) - RCT_i(Ya) at the tile of XR, minus at the tile of XL)
// c the band-closing rows (multiples of TY) strictly between Ya and Yb: the
// tile-local sums restart at each band, so the column's full bands in between
// are added from the side array XC.  When Ya itself closes a band, its top
// corners cancel against the crossing at c = Ya, so both drop.  The row
// carries RC hold the tile's origin column, contracted in y: one value per x
// term for every column of the tile.
//
// Each lane owns one window centre and reads, per row event, its window's
// values at its two edges: a wave's 64 windows read 64 consecutive columns
// at each edge, exactly what they need, and no window waits for any other, so
// the sweep has no barrier.  A window's sum is a sum of row events: the
// opening row Ya (its top corners), the crossings (contracted with
// beta(yc)), the boundary row Yb (its bottom corners).
//
// Combs.  The centre rows yc = y0 + q + m h (h the window height) of comb q
// follow one another so that member m's boundary row is member m + 1's
// opening row.  A wave walks a segment of S members of one comb and reads
// each boundary row once, for the member it closes (bottom corners) and the
// one it opens (top corners).  Row carries: the wave's right edges lie in one
// tile and its left edges in at most two (chunks start where right edges
// begin a tile); lanes 21 s + i load term i (i = NT: the count) of edge tile
// s's carries at each opening and boundary row, keep the member's carry box,
// and pass it to every lane through the wave's LDS slots when the member
// closes, where each window contracts its two tiles' boxes with alpha(xc).
//
// Work item = (bin group, segment, comb group, chunk of cw windows; nt waves
// of 64 windows per comb, cpb combs per block -- batches pack the combs of a
// narrow job into one block): a wave loops over the group's bins and walks
// the segment for each, keeping a row's loads in flight while the previous
// row is contracted, and adds the bin's term sqrt(p_b t_b) to its (member,
// window) accumulator in LDS (each lane its own entries).  With one bin group
// the map is stored once at the end; with several, each group adds its sums
// into the set's integer accumulator and match_gauss_fin writes the map.
// Every split does the same operations in the same order for every (window,
// bin), so maps agree bit for bit.
enum : int { kEvOpen = 0, kEvCross = 1, kEvBound = 2, kEvEnd = 3 };

struct SweepEv {
  int b, mm, Y, type, Ya;  // bin, member, row, kind, the member's opening row
};

// The event after e (unit 0 of it) in the walk of a segment of cnt members
// over bins [., b1).
__device__ __forceinline__ SweepEv sweep_next(const SweepEv& e, int cnt, int b1, int h, int lgTY,
                                              int Ya0) {
  SweepEv n = e;
  int Ya = e.Ya, mm = e.mm, c;
  if (e.type == kEvBound) {
    if (mm + 1 >= cnt) {
      if (e.b + 1 >= b1) {
        n.type = kEvEnd;
        return n;
      }
      n.b = e.b + 1;
      n.mm = 0;
      n.Y = n.Ya = Ya0;
      n.type = kEvOpen;
      return n;
    }
    mm += 1;
    Ya = e.Y;
    c = ((Ya >> lgTY) + 1) << lgTY;
  } else {
    c = e.type == kEvOpen ? ((Ya >> lgTY) + 1) << lgTY : e.Y + (1 << lgTY);
  }
  const int Yb = Ya + h;
  n.mm = mm;
  n.Ya = Ya;
  n.Y = c < Yb ? c : Yb;
  n.type = c < Yb ? kEvCross : kEvBound;
  return n;
}

template <int NT>
__device__ __forceinline__ void match_gauss_sweep(const MatchArgs& a, int vb) {
  // a row's values: at a crossing V+ (NT) and V- (NT), at an opening or a
  // boundary row the corners C_RB, C_RT at XR and C_LB, C_LT at XL (0..3);
  // then N at XR and N at XL
  constexpr int D = 2 * NT + 2;
  constexpr int GS = 21;                       // lanes per edge tile (x terms + the count)
  static_assert(NT + 1 <= GS, "series terms");
  const SwihGeom& g = a.g;
  const ScaleParams& sp = a.sp;
  // item = (bin group, segment, comb group, chunk); a block's waves cover the
  // chunk's nt sub-chunks of 64 windows for each of cpb combs (batches pack
  // the combs of narrow jobs into one block)
  const int ncg = (a.ncomb + a.cpb - 1) / a.cpb;
  const int ch = vb % a.nch;
  int r = vb / a.nch;
  const int qg = r % ncg;
  r /= ncg;
  const int sg = r % a.nseg;
  const int grp = r / a.nseg;
  const int tid = (int)threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int sub = wv / a.nt, wsub = wv - sub * a.nt;
  const int q = qg * a.cpb + sub;
  const int ny = a.y1 - a.y0 + 1, rx = sp.rx, ry = sp.ry, h = 2 * ry + 1;
  const int Mq = q < ny ? (ny - q + h - 1) / h : 0;  // centre rows of comb q
  const int m0 = sg * a.S;
  const int cnt = min(a.S, Mq - m0);
  const int b0 = grp * a.bpg, b1 = min(b0 + a.bpg, g.B);
  // chunks start where a wave's right edges begin a tile: they then lie in
  // one tile, its left edges in at most two
  const int xo = a.x0 - ((a.x0 + rx) & 63);
  const int xs = xo + ch * a.cw + 64 * wsub;  // the wave's first window
  // a launch may have more waves than the item (a batch's largest block)
  const bool live = sub < a.cpb && q < a.ncomb && m0 < Mq && xs <= a.x1;
  const int ycb = a.y0 + q + m0 * h;  // first centre row of the segment
  const int Ya0 = ycb - ry;
  const int lgTY = g.lgTY, ymask = g.TY - 1;
  // the waves' LDS regions move with the item's S: every wave has left the
  // previous virtual block of its block before any reuses it; no barrier after
  // this one (each lane touches only its own entries)
  __syncthreads();
  extern __shared__ double slds[];
  const int nwb = (int)(blockDim.x >> 6);
  double* rcs = slds + wv * 64;  // [64] per wave: lane GS s + i holds edge tile s's box of term i
  int32_t* acc = (int32_t*)(slds + nwb * 64) + (size_t)wv * a.S * 64;  // [S][64] per wave
  if (!live) return;
  for (int mm = 0; mm < cnt; ++mm) acc[mm * 64 + lane] = 0;
  const bool mine = xs + lane >= a.x0 && xs + lane <= a.x1;
  // lanes outside the rectangle follow its nearest window
  const int xc = min(max(xs + lane, a.x0), a.x1);
  const int XR = xc + rx + 1, XL = xc - rx;
  const bool xl0 = XL == 0;  // column 0 is not stored: its values are 0
  const int XLc = xl0 ? 1 : XL;
  double al[NT];
  series_coeffs<NT>(sp.ax, xc, al);
  // the edges' tiles: right edges in tR (one tile, or two at the rectangle's
  // clamped ends), left edges in tL0, tL0 + 1; lanes GS s + i handle x term i
  // (i = NT: the count) of edge tile s = 0 (right), 1, 2 (left)
  const int tR0 = __builtin_amdgcn_readfirstlane((XR - 1) >> 6);
  const int tL0 = __builtin_amdgcn_readfirstlane((XLc - 1) >> 6);
  const int sR = ((XR - 1) >> 6) - tR0, sL = ((XLc - 1) >> 6) - tL0;
  const int ls = GS * (1 + sL);  // first lane of this lane's left edge tile
  const int slot = lane / GS, ti = lane - slot * GS;
  const int mytile = slot == 0 ? tR0 : tL0 + slot - 1;
  const bool carries = slot < 3 && ti <= NT && mytile < g.NTX;
  const int qB = ti < NT ? ti : 2 * NT, qT = ti < NT ? NT + ti : 2 * NT;
  const float* __restrict__ pl = (const float*)a.planes;
  const int64_t oR = swih_xoff(g, XR), oL = swih_xoff(g, XLc);
  // column parts of the XC offsets: V+ at XR, V- at XL
  const int64_t xR = (int64_t)((XR - 1) >> 6) * (2 * NT * 64) + ((XR - 1) & 63);
  const int64_t xL = (int64_t)((XLc - 1) >> 6) * (2 * NT * 64) + NT * 64 + ((XLc - 1) & 63);
  const double inv_mass = 1.0 / sp.mass;
  // an opening row that closes a band adds nothing and is not read
  auto reads = [&](const SweepEv& e) { return e.type != kEvOpen || (e.Y & ymask) != 0; };
  // the bin's bases, recomputed when the walk reaches the next bin (loads run in
  // event order); within a bin a row costs one 32-bit product per base
  const int rs = (int)g.row_stride, xrs = g.NTX * (2 * NT * 64), nrc = g.nRC;
  const int ctile = min(mytile, g.NTX - 1);
  int lb = -1;
  const float* pbin = pl;     // the bin's planes
  int64_t xbin = 0;           // the bin's band-closing rows in XC
  const double* rcl = a.RC;   // this lane's carry tile of the bin, row 0
  auto load = [&](float (&d)[D], double (&rc)[2], const SweepEv& e) {
    if (e.b != lb) {
      lb = e.b;
      pbin = pl + swih_base(g, 0, e.b);
      xbin = (int64_t)e.b * g.NTY * xrs;
      rcl = a.RC + swih_rc(g, 0, e.b, ctile, 0);
    }
    if (e.type != kEvCross && carries) {
      // this lane's x term of its tile's carries at the row, as a bottom and as a top row
      const double* __restrict__ qr = rcl + e.Y * nrc;
      rc[0] = qr[qB];
      rc[1] = qr[qT];
    }
    if (!reads(e)) return;
    const float* __restrict__ row = pbin + e.Y * rs;
    if (e.type == kEvCross) {
      const float* __restrict__ xr = a.XC + xbin + ((e.Y >> lgTY) - 1) * xrs;
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        d[j] = xr[xR + j * 64];
        d[NT + j] = xr[xL + j * 64];
      }
    } else {
      if (e.type == kEvBound) {
        d[0] = row[oR];
        d[2] = row[oL + 128];
      }
      d[1] = row[oR + 64];
      d[3] = row[oL + 192];
    }
    d[2 * NT] = row[oR + 256];
    d[2 * NT + 1] = row[oL + 256];
  };
  auto advance = [&](const SweepEv& e) { return sweep_next(e, cnt, b1, h, lgTY, Ya0); };
  double hh = 0.0, nn = 0.0;  // the member's window sum and pixel count so far
  double oh = 0.0, on = 0.0;  // the next member's opening row
  // beta(yc) of the current member: the build's row table holds it at row
  // yc - ry as a top edge, members h rows apart.
  double bcur[NT];
  const double* __restrict__ btab = a.beta + (size_t)(ycb - ry) * 2 * NT + NT;
  const int bstep = h * 2 * NT;
  auto beta = [&](int mm) {
    const double* __restrict__ br = btab + min(mm, cnt - 1) * bstep;  // past the last: never used
#pragma unroll
    for (int j = 0; j < NT; ++j) bcur[j] = br[j];
  };
  float tb = 0.0f;  // the bin's template value
  // lanes of an edge tile: the carry at the member's opening row, and the
  // member's carry box once it closes
  double qprev = 0.0, rbox = 0.0;
  auto process = [&](float (&d)[D], const double (&rc)[2], const SweepEv& e) {
    const bool withL = (e.Y & ymask) != 0;  // as an opening row
    // a left-edge value: 0 at column 0
    auto lv = [&](float v) { return xl0 ? 0.0 : (double)v; };
    if (e.type != kEvCross) {
      if (e.type == kEvBound) rbox = rc[0] - qprev;
      qprev = rc[1];
    }
    if (e.type == kEvOpen) {
      beta(0);
      tb = a.tmpl[e.b];
      if (withL) {
        oh = (double)d[1] - lv(d[3]);
        on = (double)d[2 * NT] - lv(d[2 * NT + 1]);
      } else {
        oh = on = 0.0;
      }
      hh = -oh;
      nn = -on;
      return;
    }
    const double dn = (double)d[2 * NT] - lv(d[2 * NT + 1]);
    nn += dn;
    if (e.type == kEvCross) {
#pragma unroll
      for (int j = 0; j < NT; ++j) hh = fma(bcur[j], (double)d[j] - lv(d[NT + j]), hh);
      return;
    }
    hh += (double)d[0] - lv(d[2]);
    if (e.mm + 1 < cnt && withL) {
      oh = (double)d[1] - lv(d[3]);
      on = dn;
    } else {
      oh = on = 0.0;
    }
    // the window's carry part: alpha(xc) . (box of its right-edge tile - left-edge tile)
    // every lane's right edge tile is the wave's (lanes GS s + i hold tile s's boxes),
    // its left edge tile one of two
    // (passed through the wave's LDS slots: a wave's LDS accesses complete in order)
    rcs[lane] = rbox;  // read back only from carry lanes
    const double* __restrict__ rl = rcs + ls;
    double wr = 0.0, wl = 0.0;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      wr = fma(al[i], rcs[i], wr);
      wl = fma(al[i], rl[i], wl);
    }
    const double cr = rcs[NT], cl = rl[NT];
    // right edges share tile tR0 except where lanes were clamped to the rectangle
    const double H = hh + (sR ? 0.0 : wr) - (xl0 ? 0.0 : wl);
    const double N = nn + (sR ? 0.0 : cr) - (xl0 ? 0.0 : cl);
    const int32_t v = N != 0.0 ? bc_term(H * inv_mass, tb) : 0;
    acc[e.mm * 64 + lane] += v;
    hh = -oh;
    nn = -on;
    beta(e.mm + 1);
  };
  SweepEv e0;
  e0.b = b0;
  e0.mm = 0;
  e0.Y = e0.Ya = Ya0;
  e0.type = kEvOpen;
  // two register buffers alternate: the next row's loads are in flight while
  // the current row is contracted
  float dA[D], dB[D];
  double rA[2] = {0.0, 0.0}, rB[2] = {0.0, 0.0};
  load(dA, rA, e0);
  for (;;) {
    const SweepEv e1 = advance(e0);
    if (e1.type != kEvEnd) load(dB, rB, e1);
    process(dA, rA, e0);
    if (e1.type == kEvEnd) break;
    e0 = advance(e1);
    if (e0.type != kEvEnd) load(dA, rA, e0);
    process(dB, rB, e1);
    if (e0.type == kEvEnd) break;
  }
  if (mine) {
    const int mw = a.x1 - a.x0 + 1;
    for (int mm = 0; mm < cnt; ++mm) {
      const size_t o = (size_t)(ycb + mm * h - a.y0) * mw + (xc - a.x0);
      const int32_t v = acc[mm * 64 + lane];
      if (a.ngroups == 1) a.map[o] = bc_value(v);
      else atomicAdd((unsigned int*)&a.acc[o], (unsigned int)v);
    }
  }
}

// Map from the accumulator of a sweep with several bin groups; the
// accumulator is left zero.
__device__ __forceinline__ void match_gauss_fin(const MatchArgs& a, int vb) {
  const int mw = a.x1 - a.x0 + 1;
  const long n = (long)mw * (a.y1 - a.y0 + 1);
  const long t = (long)vb * 256 + threadIdx.x;
  if (t >= n) return;
  a.map[t] = bc_value(a.acc[t]);
  a.acc[t] = 0;
}

}  // namespace
}  // namespace swih
