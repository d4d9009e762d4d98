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
struct GaussPlanes {
  const float* L;
  const double* RC;
};

__device__ __forceinline__ int tile_of(int X) { return (X > 0 ? X - 1 : 0) >> 6; }

// First band-boundary row (a positive multiple of TY) at or after ya.
__device__ __forceinline__ int first_cross(int ya, int TY) {
  const int c = (ya + TY - 1) / TY * TY;
  return c == 0 ? TY : c;
}

template <int NT>
__device__ __forceinline__ void series_coeffs(const GaussAxis& ax, int c, double (&out)[NT]) {
  out[0] = ax.a[0];
#pragma unroll
  for (int k = 1; k <= (NT - 1) / 2; ++k) {
    double s, co;
    sincos(ax.om[k] * (double)c, &s, &co);
    out[2 * k - 1] = ax.a[k] * co;
    out[2 * k] = ax.a[k] * s;
  }
}

// One block per centre; threads over (bin, x term i) pairs compute
// alpha_i sum_j beta_j B_ij into LDS, then one thread per bin adds the terms
// in order i = 0..NT-1.  Term (0, 0) is the plain pixel count (u_0 = v_0 = 1
// exactly), and its box is an exact integer: a bin with no pixel in the
// window gets p_b = 0 exactly instead of a rounding residue.
template <int NT>
__device__ __forceinline__ void query_gauss(const QueryArgs& a, int vb) {
  const SwihGeom& g = a.g;
  const ScaleParams& sp = a.sp;
  const GaussPlanes gp{(const float*)a.planes, a.RC};
  const int32_t* __restrict__ centres = a.centres;
  __syncthreads();  // LDS reuse across virtual blocks of one block
  extern __shared__ double part[];  // [B][NT], then the window's pixel count per bin [B]
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
  const int64_t oa = swih_xoff(g, xa0 ? 1 : xa), ob = swih_xoff(g, xb);
  for (int it = threadIdx.x; it < g.B * NT; it += blockDim.x) {
    const int b = it / NT, i = it - (it / NT) * NT;
    // the NT y-term planes of x term i sit 64 elements apart within a row
    const float* lp = gp.L + swih_base(g, i * NT, b);
    float aA[NT], bA[NT], aB[NT], bB[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const float* q = lp + (size_t)j * 64;
      aA[j] = xa0 ? 0.0f : q[(size_t)ya * rs + oa];
      bA[j] = xa0 ? 0.0f : q[(size_t)yb * rs + oa];
      aB[j] = q[(size_t)ya * rs + ob];
      bB[j] = q[(size_t)yb * rs + ob];
    }
    double d[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j)
      d[j] = ((double)bB[j] - (double)aB[j]) - ((double)bA[j] - (double)aA[j]);
    for (int c = first_cross(ya, g.TY); c < yb; c += g.TY) {
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const float* q = lp + (size_t)j * 64 + (size_t)c * rs;
        d[j] += (double)q[ob] - (xa0 ? 0.0 : (double)q[oa]);
      }
    }
    double hi = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int p = i * NT + j;
      d[j] += (gp.RC[swih_rc(g, p, b, txb, yb)] - gp.RC[swih_rc(g, p, b, txb, ya)]) -
              (gp.RC[swih_rc(g, p, b, txa, yb)] - gp.RC[swih_rc(g, p, b, txa, ya)]);
      hi = fma(be[j], d[j], hi);
    }
    part[it] = al[i] * hi;
    if (i == 0) part[g.B * NT + b] = d[0];
  }
  __syncthreads();
  for (int b = threadIdx.x; b < g.B; b += blockDim.x) {
    double h = 0.0;
    for (int i = 0; i < NT; ++i) h += part[b * NT + i];
    if (part[g.B * NT + b] == 0.0) h = 0.0;
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

// One coefficient of the series at centre coordinate c: index 0 -> a_0,
// 2k-1 -> a_k cos(w_k c), 2k -> a_k sin(w_k c).
__device__ __forceinline__ double series_coeff(const GaussAxis& ax, int c, int idx) {
  if (idx == 0) return ax.a[0];
  const int k = (idx + 1) / 2;
  const double ang = ax.om[k] * (double)c;
  return ax.a[k] * ((idx & 1) ? cos(ang) : sin(ang));
}

// A Gaussian map value is sum_b sqrt(p_b t_b).  Each bin's term is rounded to
// a multiple of 2^-40 and the terms are added as integers: exact, so the sum
// is the same whatever the order in which bins arrive (one block per bin and
// integer atomics, or all bins in one thread); 2^-41 is far below the float
// resolution of the result.
constexpr double kBcScale = 1099511627776.0;  // 2^40

__device__ __forceinline__ int64_t bc_term(double p, float t) {
  return (int64_t)__builtin_rint(sqrt(fmax(p, 0.0) * fmax((double)t, 0.0)) * kBcScale);
}

__device__ __forceinline__ float bc_value(int64_t q) { return (float)((double)q / kBcScale); }

// Empty bins.  sqrt is not Lipschitz at 0: a bin with no pixel in the window
// must give p_b = 0 exactly, or a rounding residue e of the float planes
// turns into sqrt(e t_b), orders of magnitude above e.  The weight term
// (0, 0) is the plain pixel count (u_0 = v_0 = 1 exactly), and every part of
// its box is an integer (tile-local float values below 2^24, double carries),
// so the count is exact and the maps drop a bin's term exactly when it is 0.

// Column work of the Gaussian maps.  A block covers nV plane columns X (the
// left and right window edges of its chunk of centres).  The x terms i of a
// column are split over NG slots; each thread sums the terms of its items in
// item order and writes its slot's partial G+/G- to LDS, and the window
// threads add the slots in slot order.  Both map kernels use this split, so
// their maps agree bit for bit.
//  * strided (NT != 2 NG - 1): slot s holds terms s, s + NG, s + 2 NG, ...;
//    one thread per (slot, column) and NG * nvpad threads, so a wave never
//    spans two slots.
//  * paired (NT == 2 NG - 1): slot s < NG - 1 holds terms s and s + NG, one
//    thread per (slot, column); the last slot holds term NG - 1 alone, one
//    thread per two columns (xi and xi + ceil(nV / 2)).  Every thread has two
//    items: for NT = 7 the seven terms cost two item times per step instead of
//    three with a strided split over three slots.
__host__ __device__ constexpr int gauss_slots(int NT) { return NT <= 7 ? (NT + 1) / 2 : 3; }

template <int NT, int NG>
struct ColItems {
  static constexpr bool kPaired = NT == 2 * NG - 1;
  static constexpr int NI = kPaired ? 2 : (NT + NG - 1) / NG;
  int slot;      // LDS slot of this thread's sums, -1 for none
  bool single;   // paired split, last slot: the two items are two columns of one term
  int i[NI], xi[NI], X[NI];
  bool ok[NI];

  __device__ __forceinline__ void init(int tid, int nV, int nvpad, int xa, int rx, int cwc,
                                       bool contig) {
    auto colX = [&](int c) {
      return contig ? xa - rx + c : (c < cwc ? xa - rx + c : xa + rx + 1 + c - cwc);
    };
    single = false;
    if constexpr (kPaired) {
      const int base = (NG - 1) * nV, nvh = (nV + 1) / 2;
      if (tid < base) {
        slot = tid / nV;
        const int c = tid - slot * nV;
        i[0] = slot;
        i[1] = slot + NG;
        xi[0] = xi[1] = c;
        ok[0] = ok[1] = true;
      } else if (tid < base + nvh) {
        slot = NG - 1;
        single = true;
        i[0] = i[1] = NG - 1;
        xi[0] = tid - base;
        xi[1] = xi[0] + nvh;
        ok[0] = true;
        ok[1] = xi[1] < nV;
      } else {
        slot = -1;
#pragma unroll
        for (int ii = 0; ii < NI; ++ii) {
          i[ii] = 0;
          xi[ii] = 0;
          ok[ii] = false;
        }
      }
    } else {
      const int grp = __builtin_amdgcn_readfirstlane(tid / nvpad);
      const int c = tid - grp * nvpad;
      const bool has = grp < NG && c < nV;
      slot = has ? grp : -1;
#pragma unroll
      for (int ii = 0; ii < NI; ++ii) {
        i[ii] = grp + ii * NG;
        xi[ii] = c;
        ok[ii] = has && i[ii] < NT;
      }
    }
#pragma unroll
    for (int ii = 0; ii < NI; ++ii) {
      X[ii] = ok[ii] ? colX(xi[ii]) : xa;
      if (!ok[ii]) i[ii] = 0;
    }
  }
};

// Threads of a map block over nV columns with the split of NT terms.
__host__ __device__ constexpr int gauss_map_threads(int NT, int nV) {
  return gauss_slots(NT) * 2 - 1 == NT
             ? ((gauss_slots(NT) - 1) * nV + (nV + 1) / 2 + 63) / 64 * 64
             : gauss_slots(NT) * ((nV + 63) / 64 * 64);
}

// Dense map.  One block per (row of centres yc, chunk of cw centres), threads
// over (slot, plane column X the chunk's windows touch: X = xc - rx and
// xc + rx + 1).  With the y terms contracted,
//   V_i(X) = sum_j beta_j(yc) (P_ij[yb][X] - P_ij[ya][X]),
// the window histogram is H_b(xc) = sum_i alpha_i(xc) (V_i(xc+rx+1) - V_i(xc-rx)).
// Each column therefore folds its own V_i into the two quantities the windows
// need from it,
//   G+(X) = sum_i alpha_i(X - rx - 1) V_i(X)   (X is a right edge)
//   G-(X) = sum_i alpha_i(X + rx) V_i(X)       (X is a left edge),
// and only those cross LDS: H_b(xc) = G+(xc + rx + 1) - G-(xc - rx).  The row
// carries of V_i depend on X only through its tile column and are tabulated
// for every bin once per block.  Per bin: the column threads load their
// L rows (all j of one item together), one barrier (LDS double-buffered by bin
// parity), the window threads accumulate sqrt(p_b t_b).
template <int NT, int NG>
__device__ __forceinline__ void match_gauss(const MatchArgs& a, int vb) {
  using CI = ColItems<NT, NG>;
  constexpr int NI = CI::NI;
  const SwihGeom& g = a.g;
  const ScaleParams& sp = a.sp;
  const GaussPlanes gp{(const float*)a.planes, a.RC};
  const float* __restrict__ tmpl = a.tmpl;
  const int x0 = a.x0, y0 = a.y0, x1 = a.x1;
  const int cw = a.cw, nvpad = a.nvpad, ntl_max = a.ntl_max;
  // a block may run several virtual blocks one after another: the previous
  // one's window threads must be done with LDS before it is overwritten
  __syncthreads();
  extern __shared__ double sm[];
  double* Gb = sm;                                  // [2][NG][2][nvpad]
  double* R = sm + 2 * NG * 2 * nvpad;              // [B][NT][ntl_max]
  double* Nb = R + (size_t)g.B * NT * ntl_max;      // [2][nvpad] pixel counts per column
  double* Rn = Nb + 2 * nvpad;                      // [B][ntl_max] count-plane carries
  const int yc = y0 + vb / a.nbx;
  const int xa = x0 + (vb % a.nbx) * cw;
  const int cwc = min(cw, x1 - xa + 1);
  const int rx = sp.rx, ry = sp.ry;
  const bool contig = 2 * rx + 1 <= cwc;
  const int nV = contig ? cwc + 2 * rx + 1 : 2 * cwc;
  const int Ya = yc - ry, Yb = yc + ry + 1;
  const int c0 = first_cross(Ya, g.TY);
  const int ncross = c0 < Yb ? (Yb - 1 - c0) / g.TY + 1 : 0;
  double be[NT];
  series_coeffs<NT>(sp.ay, yc, be);
#pragma unroll
  for (int j = 0; j < NT; ++j) be[j] = uniform(be[j]);
  const int tid = threadIdx.x;
  const int tlo = tile_of(xa - rx), ntl = tile_of(xa + cwc + rx) - tlo + 1;
  // row-carry table of every bin: R[b][i][t] = sum_j beta_j (RC_ij[yb] - RC_ij[ya])
  for (int it = tid; it < g.B * NT * ntl; it += blockDim.x) {
    const int b = it / (NT * ntl);
    const int rem = it - b * (NT * ntl);
    const int i = rem / ntl, t = rem - (rem / ntl) * ntl;
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int p = i * NT + j;
      acc = fma(be[j], gp.RC[swih_rc(g, p, b, tlo + t, Yb)] - gp.RC[swih_rc(g, p, b, tlo + t, Ya)], acc);
    }
    R[(b * NT + i) * ntl_max + t] = acc;
    if (i == 0)
      Rn[b * ntl_max + t] = gp.RC[swih_rc(g, 0, b, tlo + t, Yb)] - gp.RC[swih_rc(g, 0, b, tlo + t, Ya)];
  }
  CI ci;
  ci.init(tid, nV, nvpad, xa, rx, cwc, contig);
  // alpha at the two windows each item's column serves, for the item's x term
  double ap[NI], am[NI];
  int tX[NI];
  bool x0col[NI];
  size_t offA[NI], offB[NI], offC[NI];
  const int64_t rs = g.row_stride;
#pragma unroll
  for (int ii = 0; ii < NI; ++ii) {
    const int X = ci.X[ii];
    ap[ii] = series_coeff(sp.ax, max(X - rx - 1, 0), ci.i[ii]);
    am[ii] = series_coeff(sp.ax, X + rx, ci.i[ii]);
    tX[ii] = tile_of(X) - tlo;
    // column X = 0 is not stored (it is zero): its thread loads column 1 and drops it
    x0col[ii] = X == 0;
    const int64_t xo = swih_xoff(g, x0col[ii] ? 1 : X);
    offA[ii] = (size_t)Ya * rs + xo;
    offB[ii] = (size_t)Yb * rs + xo;
    offC[ii] = (size_t)c0 * rs + xo;
  }
  const bool win = tid < cwc;
  const int xc = xa + tid;
  const int i1 = tid, i2 = contig ? tid + 2 * rx + 1 : cwc + tid;
  const double inv_mass = 1.0 / sp.mass;
  int64_t bc = 0;
  __syncthreads();
  for (int b = 0; b < g.B; ++b) {
    double* Gp = Gb + (b & 1) * NG * 2 * nvpad;
    double* Np = Nb + (b & 1) * nvpad;
    if (ci.slot >= 0) {
      double gplus = 0.0, gminus = 0.0;
#pragma unroll
      for (int ii = 0; ii < NI; ++ii) {
        if (!ci.ok[ii]) break;
        const int i = ci.i[ii];
        const float* lp = gp.L + swih_base(g, i * NT, b);
        float la[NT], lb[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          la[j] = lp[offA[ii] + (size_t)j * 64];
          lb[j] = lp[offB[ii] + (size_t)j * 64];
        }
        double vl = 0.0, nl = (double)lb[0] - (double)la[0];
#pragma unroll
        for (int j = 0; j < NT; ++j) vl = fma(be[j], (double)lb[j] - (double)la[j], vl);
        for (int c = 0; c < ncross; ++c) {
          float lc[NT];
#pragma unroll
          for (int j = 0; j < NT; ++j) lc[j] = lp[offC[ii] + (size_t)c * g.TY * rs + (size_t)j * 64];
#pragma unroll
          for (int j = 0; j < NT; ++j) vl = fma(be[j], (double)lc[j], vl);
          nl += (double)lc[0];
        }
        // slot 0's first item is term 0 of its column: the column's pixel count
        if (ii == 0 && ci.slot == 0)
          Np[ci.xi[0]] = Rn[b * ntl_max + tX[0]] + (x0col[0] ? 0.0 : nl);
        const double v = R[(b * NT + i) * ntl_max + tX[ii]] + (x0col[ii] ? 0.0 : vl);
        if (ci.single) {
          Gp[(ci.slot * 2 + 0) * nvpad + ci.xi[ii]] = fma(ap[ii], v, 0.0);
          Gp[(ci.slot * 2 + 1) * nvpad + ci.xi[ii]] = fma(am[ii], v, 0.0);
        } else {
          gplus = fma(ap[ii], v, gplus);
          gminus = fma(am[ii], v, gminus);
        }
      }
      if (!ci.single) {
        Gp[(ci.slot * 2 + 0) * nvpad + ci.xi[0]] = gplus;
        Gp[(ci.slot * 2 + 1) * nvpad + ci.xi[0]] = gminus;
      }
    }
    __syncthreads();
    if (win) {
      double hh = 0.0;
#pragma unroll
      for (int q = 0; q < NG; ++q) hh += Gp[(q * 2 + 0) * nvpad + i2] - Gp[(q * 2 + 1) * nvpad + i1];
      if (Np[i2] - Np[i1] != 0.0) bc += bc_term(hh * inv_mass, tmpl[b]);
    }
  }
  if (win) a.map[(size_t)(yc - y0) * (x1 - x0 + 1) + (xc - x0)] = bc_value(bc);
}


// Dense map for large rectangles: one block per (bin, chunk of centres, comb
// segment).  A comb is the set of centre rows yc = y0 + q + m h (h the window
// height): the bottom row of one comb member's windows is the top row of the
// next, so a block walks its comb segment reading each boundary row once and
// keeping the previous one in registers (S + 1 rows for S centre rows, against
// 2 S for one row per block).  Per centre row the column threads form G+/G-
// exactly as match_gauss does (same split, same operations in the same
// order), the window threads form the bin's term and add it, as an integer,
// into the map's accumulator.  match_gauss_fin turns the accumulator into the
// map and clears it.  The result equals match_gauss bit for bit.
template <int NT, int NG>
__device__ __forceinline__ void match_gauss_comb(const MatchArgs& a, int vb) {
  using CI = ColItems<NT, NG>;
  {
    // Workgroups go to the 8 XCDs round robin: renumber so that each XCD runs
    // a contiguous range of virtual blocks, i.e. the combs of one (bin, chunk)
    // together, and their shared band-closing rows stay in that XCD's L2.
    const int n = (int)gridDim.x, base = n >> 3, rem = n & 7;
    const int x = vb & 7, k = vb >> 3;
    vb = x * base + (x < rem ? x : rem) + k;
  }
  constexpr int NI = CI::NI;
  const SwihGeom& g = a.g;
  const ScaleParams& sp = a.sp;
  const GaussPlanes gp{(const float*)a.planes, a.RC};
  const int x0 = a.x0, y0 = a.y0, x1 = a.x1, y1 = a.y1;
  const int cw = a.cw, nvpad = a.nvpad, ntl_max = a.ntl_max;
  const int S = a.comb_steps, nsegc = a.comb_segs;
  const int rx = sp.rx, ry = sp.ry, h = 2 * ry + 1;
  const int q = vb % h;
  int r = vb / h;
  const int sg = r % nsegc;
  r /= nsegc;
  const int chunk = r % a.nbx;
  const int b = r / a.nbx;
  const int ny = y1 - y0 + 1;
  const int Mq = q < ny ? (ny - q + h - 1) / h : 0;  // centre rows of comb q
  const int m0 = sg * S;
  if (m0 >= Mq) return;  // uniform over the block
  const int cnt = min(S, Mq - m0);
  __syncthreads();  // LDS reuse across virtual blocks of one block
  extern __shared__ double sm[];
  double* Gb = sm;                          // [2][NG][2][nvpad]
  double* R = sm + 2 * NG * 2 * nvpad;      // [S][NT][ntl_max]
  double* BE = R + (size_t)S * NT * ntl_max;  // [S][NT]
  double* Nb = BE + (size_t)S * NT;         // [2][nvpad] pixel counts per column
  double* Rn = Nb + 2 * nvpad;              // [S][ntl_max] count-plane carries
  const int xa = x0 + chunk * cw;
  const int cwc = min(cw, x1 - xa + 1);
  const bool contig = 2 * rx + 1 <= cwc;
  const int nV = contig ? cwc + 2 * rx + 1 : 2 * cwc;
  const int tid = threadIdx.x;
  const int tlo = tile_of(xa - rx), ntl = tile_of(xa + cwc + rx) - tlo + 1;
  const int ycb = y0 + q + m0 * h;  // first centre row of the segment
  // beta of every centre row of the segment
  for (int mm = tid; mm < cnt; mm += blockDim.x) {
    double be[NT];
    series_coeffs<NT>(sp.ay, ycb + mm * h, be);
#pragma unroll
    for (int j = 0; j < NT; ++j) BE[mm * NT + j] = be[j];
  }
  __syncthreads();
  // row carries: R[mm][i][t] = sum_j beta_j (RC_ij[yb] - RC_ij[ya]) for this bin
  for (int it = tid; it < cnt * NT * ntl; it += blockDim.x) {
    const int mm = it / (NT * ntl);
    const int rem = it - mm * (NT * ntl);
    const int i = rem / ntl, t = rem - (rem / ntl) * ntl;
    const int ya = ycb + mm * h - ry, yb = ya + h;
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int p = i * NT + j;
      acc = fma(BE[mm * NT + j], gp.RC[swih_rc(g, p, b, tlo + t, yb)] - gp.RC[swih_rc(g, p, b, tlo + t, ya)],
                acc);
    }
    R[(mm * NT + i) * ntl_max + t] = acc;
    if (i == 0)
      Rn[mm * ntl_max + t] = gp.RC[swih_rc(g, 0, b, tlo + t, yb)] - gp.RC[swih_rc(g, 0, b, tlo + t, ya)];
  }
  CI ci;
  ci.init(tid, nV, nvpad, xa, rx, cwc, contig);
  double ap[NI], am[NI];
  int tX[NI];
  bool x0col[NI];
  const float* lpi[NI];
  const int64_t rs = g.row_stride;
#pragma unroll
  for (int ii = 0; ii < NI; ++ii) {
    const int X = ci.X[ii];
    ap[ii] = series_coeff(sp.ax, max(X - rx - 1, 0), ci.i[ii]);
    am[ii] = series_coeff(sp.ax, X + rx, ci.i[ii]);
    tX[ii] = tile_of(X) - tlo;
    x0col[ii] = X == 0;  // column X = 0 is not stored (zero)
    lpi[ii] = gp.L + swih_base(g, ci.i[ii] * NT, b) + swih_xoff(g, x0col[ii] ? 1 : X);
  }
  // the segment's first top row
  float prev[NI][NT];
#pragma unroll
  for (int ii = 0; ii < NI; ++ii)
#pragma unroll
    for (int j = 0; j < NT; ++j)
      prev[ii][j] = ci.ok[ii] ? lpi[ii][(size_t)(ycb - ry) * rs + (size_t)j * 64] : 0.0f;
  const bool win = tid < cwc;
  const int xc = xa + tid;
  const int i1 = tid, i2 = contig ? tid + 2 * rx + 1 : cwc + tid;
  const double inv_mass = 1.0 / sp.mass;
  const float tb = a.tmpl[b];
  const int mw = x1 - x0 + 1;
  __syncthreads();
  for (int mm = 0; mm < cnt; ++mm) {
    const int yc = ycb + mm * h;
    const int Ya = yc - ry, Yb = Ya + h;
    const int c0 = first_cross(Ya, g.TY);
    const int ncross = c0 < Yb ? (Yb - 1 - c0) / g.TY + 1 : 0;
    double* Gp = Gb + (mm & 1) * NG * 2 * nvpad;
    double* Np = Nb + (mm & 1) * nvpad;
    double be[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) be[j] = uniform(BE[mm * NT + j]);
    if (ci.slot >= 0) {
      double gplus = 0.0, gminus = 0.0;
#pragma unroll
      for (int ii = 0; ii < NI; ++ii) {
        if (!ci.ok[ii]) break;
        const int i = ci.i[ii];
        float lb[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) lb[j] = lpi[ii][(size_t)Yb * rs + (size_t)j * 64];
        double vl = 0.0, nl = (double)lb[0] - (double)prev[ii][0];
#pragma unroll
        for (int j = 0; j < NT; ++j) vl = fma(be[j], (double)lb[j] - (double)prev[ii][j], vl);
        for (int c = 0; c < ncross; ++c) {
          float lc[NT];
#pragma unroll
          for (int j = 0; j < NT; ++j)
            lc[j] = lpi[ii][(size_t)(c0 + c * g.TY) * rs + (size_t)j * 64];
#pragma unroll
          for (int j = 0; j < NT; ++j) vl = fma(be[j], (double)lc[j], vl);
          nl += (double)lc[0];
        }
        // slot 0's first item is term 0 of its column: the column's pixel count
        if (ii == 0 && ci.slot == 0)
          Np[ci.xi[0]] = Rn[mm * ntl_max + tX[0]] + (x0col[0] ? 0.0 : nl);
        const double v = R[(mm * NT + i) * ntl_max + tX[ii]] + (x0col[ii] ? 0.0 : vl);
        if (ci.single) {
          Gp[(ci.slot * 2 + 0) * nvpad + ci.xi[ii]] = fma(ap[ii], v, 0.0);
          Gp[(ci.slot * 2 + 1) * nvpad + ci.xi[ii]] = fma(am[ii], v, 0.0);
        } else {
          gplus = fma(ap[ii], v, gplus);
          gminus = fma(am[ii], v, gminus);
        }
#pragma unroll
        for (int j = 0; j < NT; ++j) prev[ii][j] = lb[j];
      }
      if (!ci.single) {
        Gp[(ci.slot * 2 + 0) * nvpad + ci.xi[0]] = gplus;
        Gp[(ci.slot * 2 + 1) * nvpad + ci.xi[0]] = gminus;
      }
    }
    __syncthreads();
    if (win) {
      double hh = 0.0;
#pragma unroll
      for (int qg = 0; qg < NG; ++qg)
        hh += Gp[(qg * 2 + 0) * nvpad + i2] - Gp[(qg * 2 + 1) * nvpad + i1];
      if (Np[i2] - Np[i1] != 0.0)
        atomicAdd((unsigned long long*)&a.acc[(size_t)(yc - y0) * mw + (xc - x0)],
                  (unsigned long long)bc_term(hh * inv_mass, tb));
    }
  }
}

// Map from the accumulator of match_gauss_comb; the accumulator is left zero.
__device__ __forceinline__ void match_gauss_fin(const MatchArgs& a, int vb) {
  const int mw = a.x1 - a.x0 + 1;
  const long n = (long)mw * (a.y1 - a.y0 + 1);
  const long t = (long)vb * 256 + threadIdx.x;
  if (t >= n) return;
  a.map[t] = bc_value(a.acc[t]);
  a.acc[t] = 0;
}


}  // namespace

// Every map and query is a device body over (arguments, virtual block).  A
// single request launches one block per virtual block; a batch runs all
// requests' virtual blocks in one grid-stride launch, each block finding its
// request by binary search over the prefix of block counts.
template <class A, void (*BODY)(const A&, int)>
__global__ __launch_bounds__(1024) void k_one(A a) {
  BODY(a, (int)blockIdx.x);
}

// The comb map with seven or fewer series terms fits 64 registers, so two of
// its 15-wave blocks share a compute unit: twice the loads in flight.
template <class A, void (*BODY)(const A&, int)>
__global__ __launch_bounds__(1024, 8) void k_one_w8(A a) {
  BODY(a, (int)blockIdx.x);
}

template <class A, void (*BODY)(const A&, int)>
__global__ __launch_bounds__(1024) void k_many(const A* __restrict__ items,
                                               const int32_t* __restrict__ prefix, int n) {
  const int total = prefix[n];
  for (int vb = (int)blockIdx.x; vb < total; vb += (int)gridDim.x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (prefix[mid] <= vb) lo = mid; else hi = mid - 1;
    }
    BODY(items[lo], vb - prefix[lo]);
  }
}

namespace {

template <class A, void (*BODY)(const A&, int)>
hipError_t run_one(const A& a, const Launch& ml, hipStream_t s) {
  hipLaunchKernelGGL((k_one<A, BODY>), dim3((unsigned)ml.blocks), dim3((unsigned)ml.threads),
                     ml.lds, s, a);
  return hipGetLastError();
}

template <class A, void (*BODY)(const A&, int)>
hipError_t run_one_w8(const A& a, const Launch& ml, hipStream_t s) {
  hipLaunchKernelGGL((k_one_w8<A, BODY>), dim3((unsigned)ml.blocks), dim3((unsigned)ml.threads),
                     ml.lds, s, a);
  return hipGetLastError();
}

template <class A, void (*BODY)(const A&, int)>
hipError_t run_many(const A* items, const int32_t* prefix, int n, unsigned grid, const Launch& ml,
                    hipStream_t s) {
  hipLaunchKernelGGL((k_many<A, BODY>), dim3(grid), dim3((unsigned)ml.threads), ml.lds, s, items,
                     prefix, n);
  return hipGetLastError();
}

template <int K> constexpr void (*int_match)(const MatchArgs&, int) = match_int<K>;
template <int K> constexpr void (*int_query)(const QueryArgs&, int) = query_int<K>;
template <int NT> constexpr void (*gauss_match)(const MatchArgs&, int) = match_gauss<NT, gauss_slots(NT)>;
template <int NT> constexpr void (*gauss_query)(const QueryArgs&, int) = query_gauss<NT>;

// switch over kernel kind (and Gaussian term count) calling CALL(body)
#define SWIH_BODY_CASES(CALL)                 \
  switch (kind) {                             \
    case 0: return CALL(SWIH_I(0));           \
    case 1: return CALL(SWIH_I(1));           \
    case 2: return CALL(SWIH_I(2));           \
    case 3:                                   \
      switch (nt) {                           \
        case 3: return CALL(SWIH_G(3));       \
        case 5: return CALL(SWIH_G(5));       \
        case 7: return CALL(SWIH_G(7));       \
        case 9: return CALL(SWIH_G(9));       \
        case 11: return CALL(SWIH_G(11));     \
        case 13: return CALL(SWIH_G(13));     \
        case 15: return CALL(SWIH_G(15));     \
        case 17: return CALL(SWIH_G(17));     \
        default: return hipErrorInvalidValue; \
      }                                       \
    default: return hipErrorInvalidValue;     \
  }

hipError_t match_one(int kind, int nt, const MatchArgs& a, const Launch& ml, hipStream_t s) {
#define SWIH_I(K) int_match<K>
#define SWIH_G(NT) gauss_match<NT>
#define SWIH_C(B) run_one<MatchArgs, B>(a, ml, s)
  SWIH_BODY_CASES(SWIH_C)
#undef SWIH_C
#undef SWIH_G
#undef SWIH_I
}

hipError_t match_many(int kind, int nt, const MatchArgs* jobs, const int32_t* prefix, int n,
                      unsigned grid, const Launch& ml, hipStream_t s) {
#define SWIH_I(K) int_match<K>
#define SWIH_G(NT) gauss_match<NT>
#define SWIH_C(B) run_many<MatchArgs, B>(jobs, prefix, n, grid, ml, s)
  SWIH_BODY_CASES(SWIH_C)
#undef SWIH_C
#undef SWIH_G
#undef SWIH_I
}

hipError_t query_one(int kind, int nt, const QueryArgs& a, const Launch& ql, hipStream_t s) {
#define SWIH_I(K) int_query<K>
#define SWIH_G(NT) gauss_query<NT>
#define SWIH_C(B) run_one<QueryArgs, B>(a, ql, s)
  SWIH_BODY_CASES(SWIH_C)
#undef SWIH_C
#undef SWIH_G
#undef SWIH_I
}

hipError_t query_many(int kind, int nt, const QueryArgs* jobs, const int32_t* prefix, int n,
                      unsigned grid, const Launch& ql, hipStream_t s) {
#define SWIH_I(K) int_query<K>
#define SWIH_G(NT) gauss_query<NT>
#define SWIH_C(B) run_many<QueryArgs, B>(jobs, prefix, n, grid, ql, s)
  SWIH_BODY_CASES(SWIH_C)
#undef SWIH_C
#undef SWIH_G
#undef SWIH_I
}

}  // namespace

void match_args(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                const float* tmpl, const uint32_t* tmpl_raw, int32_t x0, int32_t y0, int32_t x1,
                int32_t y1, float* map, MatchArgs& a, Launch& ml) {
  memset(&a, 0, sizeof(a));
  a.g = L.g;
  a.sp = sp;
  const char* sb = ws + (size_t)set * L.set_bytes;
  a.planes = sb + L.off_planes;
  a.RC = L.g.gauss ? (const double*)(sb + L.off_RC) : nullptr;
  a.tmpl = tmpl;
  a.tmpl_raw = tmpl_raw;
  a.map = map;
  a.x0 = x0;
  a.y0 = y0;
  a.x1 = x1;
  a.y1 = y1;
  const int nx = x1 - x0 + 1, ny = y1 - y0 + 1;
  if (!L.g.gauss) {
    a.nbx = (nx + 63) / 64;
    ml.blocks = a.nbx * ((ny + 3) / 4);
    ml.threads = 256;
    ml.lds = 0;
    return;
  }
  // Gaussian: threads over (slot, plane column) (the split of ColItems); cw
  // centres per block, as many as fit 1024 threads
  const int NT = L.g.nI, NG = gauss_slots(NT);
  const int span = 2 * sp.rx + 1;
  int maxV = 512;
  while (gauss_map_threads(NT, maxV) > 1024) --maxV;
  int cw, nV;
  if (span <= maxV / 2) {  // one contiguous column range: nV = cw + span
    const int cwmax = maxV - span;
    const int nch = (nx + cwmax - 1) / cwmax;
    cw = (nx + nch - 1) / nch;
    nV = cw + span;
  } else {                 // two column segments of cw each
    cw = nx < maxV / 2 ? nx : maxV / 2;
    nV = 2 * cw;
  }
  a.cw = cw;
  a.nvpad = (nV + 63) / 64 * 64;
  a.ntl_max = (cw + span + 63) / 64 + 2;  // tile columns one block can touch
  a.nbx = (nx + cw - 1) / cw;
  ml.blocks = a.nbx * ny;
  // every chunk's nV is at most the first chunk's, so its thread count serves all
  ml.threads = gauss_map_threads(NT, nV);
  ml.lds = sizeof(double) * ((size_t)2 * NG * 2 * a.nvpad + (size_t)L.g.B * NT * a.ntl_max +
                             (size_t)2 * a.nvpad + (size_t)L.g.B * a.ntl_max);
}

void query_args(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                const int32_t* centres, int32_t n, float* hist, uint32_t* hist_raw, QueryArgs& a,
                Launch& ql) {
  memset(&a, 0, sizeof(a));
  a.g = L.g;
  a.sp = sp;
  const char* sb = ws + (size_t)set * L.set_bytes;
  a.planes = sb + L.off_planes;
  a.RC = L.g.gauss ? (const double*)(sb + L.off_RC) : nullptr;
  a.centres = centres;
  a.n = n;
  a.hist = hist;
  a.hist_raw = hist_raw;
  ql.threads = 256;
  if (L.g.gauss) {
    ql.blocks = n;
    ql.lds = sizeof(double) * (size_t)L.g.B * (L.g.nI + 1);
  } else {
    ql.blocks = (int32_t)(((long)n * L.g.B + 255) / 256);
    ql.lds = 0;
  }
}

hipError_t launch_query(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                        const int32_t* centres, int32_t n, float* hist, uint32_t* hist_raw,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  QueryArgs a;
  Launch ql;
  query_args(L, sp, set, ws, centres, n, hist, hist_raw, a, ql);
  return query_one(sp.kind, L.g.nI, a, ql, s);
}

hipError_t launch_query_batch(int kind, int nt, const QueryArgs* jobs, const int32_t* prefix,
                              int njobs, const Launch& ql, int grid, hipStream_t s) {
  if (njobs <= 0 || ql.blocks <= 0) return hipSuccess;
  const unsigned gb = (unsigned)(ql.blocks < grid ? ql.blocks : grid);
  return query_many(kind, nt, jobs, prefix, njobs, gb, ql, s);
}

namespace {

template <int NT> constexpr void (*gauss_comb)(const MatchArgs&, int) = match_gauss_comb<NT, gauss_slots(NT)>;
constexpr void (*gauss_fin)(const MatchArgs&, int) = match_gauss_fin;

hipError_t comb_one(int nt, const MatchArgs& a, const Launch& ml, hipStream_t s) {
  switch (nt) {
    case 3: return run_one_w8<MatchArgs, gauss_comb<3>>(a, ml, s);
    case 5: return run_one_w8<MatchArgs, gauss_comb<5>>(a, ml, s);
    case 7: return run_one_w8<MatchArgs, gauss_comb<7>>(a, ml, s);
    case 9: return run_one<MatchArgs, gauss_comb<9>>(a, ml, s);
    case 11: return run_one<MatchArgs, gauss_comb<11>>(a, ml, s);
    case 13: return run_one<MatchArgs, gauss_comb<13>>(a, ml, s);
    case 15: return run_one<MatchArgs, gauss_comb<15>>(a, ml, s);
    case 17: return run_one<MatchArgs, gauss_comb<17>>(a, ml, s);
    default: return hipErrorInvalidValue;
  }
}

// Comb segments of kCombSteps centre rows: S + 1 boundary rows per S rows
// (16 measured best on the 512x512 scene among 4, 8 and 16).
constexpr int kCombSteps = 16;

}  // namespace

hipError_t launch_match(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                        const float* tmpl, const uint32_t* tmpl_raw, int32_t x0, int32_t y0,
                        int32_t x1, int32_t y1, float* map, hipStream_t s) {
  if (x1 < x0 || y1 < y0) return hipSuccess;
  MatchArgs a;
  Launch ml;
  match_args(L, sp, set, ws, tmpl, tmpl_raw, x0, y0, x1, y1, map, a, ml);
  if (ml.lds > 160 * 1024) return hipErrorInvalidValue;
  const int h = 2 * sp.ry + 1, ny = y1 - y0 + 1;
  if (!L.g.gauss || ny < 2 * h) return match_one(sp.kind, L.g.nI, a, ml, s);
  // Gaussian over many centre rows: the comb form (same values, fewer plane
  // reads), then the accumulator to the map.
  const int NT = L.g.nI, NG = gauss_slots(NT);
  const int S = kCombSteps;
  const int mmax = (ny + h - 1) / h;
  a.acc = (int64_t*)(ws + (size_t)set * L.set_bytes + L.off_acc);
  a.comb_steps = S;
  a.comb_segs = (mmax + S - 1) / S;
  Launch cl;
  cl.threads = ml.threads;
  cl.blocks = L.g.B * a.nbx * a.comb_segs * h;
  cl.lds = sizeof(double) * ((size_t)2 * NG * 2 * a.nvpad + (size_t)S * NT * a.ntl_max +
                             (size_t)S * NT + (size_t)2 * a.nvpad + (size_t)S * a.ntl_max);
  if (cl.lds > 160 * 1024) return match_one(sp.kind, L.g.nI, a, ml, s);
  hipError_t e = comb_one(NT, a, cl, s);
  if (e != hipSuccess) return e;
  Launch fl;
  fl.threads = 256;
  fl.blocks = (int32_t)(((long)(x1 - x0 + 1) * ny + 255) / 256);
  fl.lds = 0;
  return run_one<MatchArgs, gauss_fin>(a, fl, s);
}

hipError_t launch_match_batch(int kind, int nt, const MatchArgs* jobs, const int32_t* prefix,
                              int njobs, const Launch& ml, int grid, hipStream_t s) {
  if (njobs <= 0 || ml.blocks <= 0) return hipSuccess;
  if (ml.lds > 160 * 1024) return hipErrorInvalidValue;
  const unsigned gb = (unsigned)(ml.blocks < grid ? ml.blocks : grid);
  return match_many(kind, nt, jobs, prefix, njobs, gb, ml, s);
}

}  // namespace swih
