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
//     alpha = (a_0, a_k cos(w_k xc), a_k sin(w_k xc)), w_k = 2 pi k / P.
// Integer coefficients are applied modulo 2^32; the true histogram is below
// 2^32, so the result is exact.  Normalisation divides by the kernel mass S
// (the same at every location, Sec. 2.1).
#include "swih_internal.h"
#include "wave64.h"

namespace swih {
namespace {

__device__ __forceinline__ uint32_t at_u(const uint32_t* __restrict__ pl, int pitch, int Y, int X) {
  return pl[(size_t)Y * pitch + 63 + X];
}

// Exact H_b of an integer kernel at (xc, yc) (uint32 arithmetic modulo 2^32).
template <int KIND>
__device__ __forceinline__ uint32_t hist_int(const uint32_t* __restrict__ planes,
                                             const SwihGeom& g, int b, int xc, int yc,
                                             const ScaleParams& sp) {
  const size_t pstride = (size_t)g.B * g.plane_elems;
  const uint32_t* p0 = planes + (size_t)b * g.plane_elems;
  const int xa = xc - sp.rx, xb = xc + sp.rx + 1, ya = yc - sp.ry, yb = yc + sp.ry + 1;
  if (KIND == 0) {
    return at_u(p0, g.pitch, yb, xb) - at_u(p0, g.pitch, ya, xb) - at_u(p0, g.pitch, yb, xa) +
           at_u(p0, g.pitch, ya, xa);
  } else if (KIND == 1) {
    const int xm = xc + 1, ym = yc + 1;
    const uint32_t* px = p0 + pstride;
    const uint32_t* py = p0 + 2 * pstride;
    // 3 x 3 corner grid per plane
    uint32_t c1[3][3], cx[3][3], cy[3][3];
    const int Ys[3] = {ya, ym, yb}, Xs[3] = {xa, xm, xb};
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        c1[r][c] = at_u(p0, g.pitch, Ys[r], Xs[c]);
        cx[r][c] = at_u(px, g.pitch, Ys[r], Xs[c]);
        cy[r][c] = at_u(py, g.pitch, Ys[r], Xs[c]);
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
      const uint32_t* pl = p0 + p * pstride;
      bx[p] = at_u(pl, g.pitch, yb, xb) - at_u(pl, g.pitch, ya, xb) - at_u(pl, g.pitch, yb, xa) +
              at_u(pl, g.pitch, ya, xa);
    }
    const uint32_t X = (uint32_t)xc, Y = (uint32_t)yc;
    return (sp.c_int - X * X - Y * Y) * bx[0] + 2u * X * bx[1] + 2u * Y * bx[2] - bx[3] - bx[4];
  }
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <int KIND>
__global__ __launch_bounds__(256) void k_query_int(SwihGeom g, ScaleParams sp,
                                                   const uint32_t* __restrict__ planes,
                                                   const int32_t* __restrict__ centres, int n,
                                                   float* __restrict__ hist,
                                                   uint32_t* __restrict__ hist_raw) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long)n * g.B) return;
  const int k = (int)(t / g.B), b = (int)(t % g.B);
  const int xc = clampi(centres[2 * k], sp.rx, g.W - 1 - sp.rx);
  const int yc = clampi(centres[2 * k + 1], sp.ry, g.H - 1 - sp.ry);
  const uint32_t h = hist_int<KIND>(planes, g, b, xc, yc, sp);
  if (hist_raw) hist_raw[t] = h;
  if (hist) hist[t] = (float)((double)h / sp.mass);
}

template <int KIND>
__global__ __launch_bounds__(256) void k_match_int(SwihGeom g, ScaleParams sp,
                                                   const uint32_t* __restrict__ planes,
                                                   const float* __restrict__ tmpl,
                                                   const uint32_t* __restrict__ tmpl_raw, int x0,
                                                   int y0, int x1, int y1,
                                                   float* __restrict__ map) {
  const int xc = x0 + blockIdx.x * 64 + threadIdx.x;
  const int yc = y0 + blockIdx.y * 4 + threadIdx.y;
  if (xc > x1 || yc > y1) return;
  double acc = 0.0;
  for (int b = 0; b < g.B; ++b) {
    const uint32_t h = hist_int<KIND>(planes, g, b, xc, yc, sp);
    if (tmpl_raw) {
      acc += sqrt((double)h * (double)tmpl_raw[b]);
    } else {
      acc += sqrt(((double)h / sp.mass) * fmax((double)tmpl[b], 0.0));
    }
  }
  if (tmpl_raw) acc = acc / sp.mass;
  map[(size_t)(yc - y0) * (x1 - x0 + 1) + (xc - x0)] = (float)acc;
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

// P[yb][X] - P[ya][X] of plane-bin pb from the tile-local split: the two L rows,
// the L rows that close each band in between, and the row carries of X's tile.
__device__ __forceinline__ double vdiff_g(const GaussPlanes& gp, const SwihGeom& g, size_t pb,
                                          int ya, int yb, int X) {
  const float* lp = gp.L + pb * g.plane_elems + 63 + X;
  double d = (double)lp[(size_t)yb * g.pitch] - (double)lp[(size_t)ya * g.pitch];
  for (int c = first_cross(ya, g.TY); c < yb; c += g.TY) d += (double)lp[(size_t)c * g.pitch];
  const double* rcp = gp.RC + (pb * g.NTX + tile_of(X)) * (size_t)(g.H + 1);
  return d + (rcp[yb] - rcp[ya]);
}

template <int NT>
__device__ __forceinline__ void series_coeffs(const GaussAxis& ax, int c, double (&out)[NT]) {
  out[0] = ax.a[0];
#pragma unroll
  for (int k = 1; k <= (NT - 1) / 2; ++k) {
    const long ph = ((long)k * c) % ax.P;
    const double ang = 2.0 * M_PI * (double)ph / (double)ax.P;
    double s, co;
    sincos(ang, &s, &co);
    out[2 * k - 1] = ax.a[k] * co;
    out[2 * k] = ax.a[k] * s;
  }
}

// One block per centre; threads over (bin, x term i) pairs compute
// alpha_i sum_j beta_j B_ij into LDS, then one thread per bin adds the terms
// in order i = 0..NT-1.
template <int NT>
__global__ __launch_bounds__(256) void k_query_gauss(SwihGeom g, ScaleParams sp, GaussPlanes gp,
                                                     const int32_t* __restrict__ centres,
                                                     float* __restrict__ hist) {
  extern __shared__ double part[];  // [B][NT]
  const int k = blockIdx.x;
  const int xc = clampi(centres[2 * k], sp.rx, g.W - 1 - sp.rx);
  const int yc = clampi(centres[2 * k + 1], sp.ry, g.H - 1 - sp.ry);
  double al[NT], be[NT];
  series_coeffs<NT>(sp.ax, xc, al);
  series_coeffs<NT>(sp.ay, yc, be);
  const int xa = xc - sp.rx, xb = xc + sp.rx + 1, ya = yc - sp.ry, yb = yc + sp.ry + 1;
  for (int it = threadIdx.x; it < g.B * NT; it += blockDim.x) {
    const int b = it / NT, i = it - (it / NT) * NT;
    double hi = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const size_t pb = (size_t)((i * NT + j) * g.B + b);
      hi = fma(be[j], vdiff_g(gp, g, pb, ya, yb, xb) - vdiff_g(gp, g, pb, ya, yb, xa), hi);
    }
    part[it] = al[i] * hi;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < g.B; b += blockDim.x) {
    double h = 0.0;
    for (int i = 0; i < NT; ++i) h += part[b * NT + i];
    hist[(size_t)k * g.B + b] = (float)(h / sp.mass);
  }
}

// V_i(X) = sum_j beta_j (L_ij[yb][X] - L_ij[ya][X] + sum_c L_ij[c][X]) for the
// x terms i = grp, grp + NG, ... of one bin; NC band-boundary rows c (NC < 0:
// any number, looped).  All loads of one i are issued before any use.
template <int NT, int NG, int NC>
__device__ __forceinline__ void contract_rows(const GaussPlanes& gp, const SwihGeom& g, int b,
                                              int grp, const double (&be)[NT], size_t offA,
                                              size_t offB, size_t offC, int ncross, double* V,
                                              int stride) {
#pragma unroll
  for (int ii = 0; ii < (NT + NG - 1) / NG; ++ii) {
    const int i = grp + ii * NG;
    if (i >= NT) break;
    float la[NT], lb[NT], lc[NT > 0 ? NT : 1];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const float* lp = gp.L + (size_t)((i * NT + j) * g.B + b) * g.plane_elems;
      la[j] = lp[offA];
      lb[j] = lp[offB];
      if (NC >= 1) lc[j] = lp[offC];
    }
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      double d = (double)lb[j] - (double)la[j];
      if (NC >= 1) d += (double)lc[j];
      if (NC < 0) {
        const float* lp = gp.L + (size_t)((i * NT + j) * g.B + b) * g.plane_elems;
        for (int c = 0; c < ncross; ++c) d += (double)lp[offC + (size_t)c * g.TY * g.pitch];
      }
      v = fma(be[j], d, v);
    }
    V[i * stride] = v;
  }
}

// Dense map, one block per (row of centres yc, chunk of cw centres).  NG groups
// of threads, one thread per (group, plane column X the chunk's windows touch:
// X = xc - rx and xc + rx + 1).  For each bin the block contracts the y terms
// of every plane between rows ya = yc - ry and yb = yc + ry + 1:
//   V_i(X)  = sum_j beta_j(yc) (P_ij[yb][X] - P_ij[ya][X]) without the row carries
//   R_i(tx) = sum_j beta_j(yc) (RC_ij[tx][yb] - RC_ij[tx][ya])   (per tile column)
// into LDS (double-buffered across bins, one barrier per bin); each window then
// needs H_b = sum_i alpha_i(xc) ((V_i + R_i)(xc + rx + 1) - (V_i + R_i)(xc - rx)).
template <int NT, int NG>
__global__ __launch_bounds__(1024) void k_match_gauss(SwihGeom g, ScaleParams sp, GaussPlanes gp,
                                                      const float* __restrict__ tmpl, int x0,
                                                      int y0, int x1, int cw, int nvpad,
                                                      int ntl_max, float* __restrict__ map) {
  extern __shared__ double sm[];
  double* Vbuf = sm;                    // [2][NT][nvpad]
  double* Rbuf = sm + 2 * NT * nvpad;   // [2][NT][ntl_max]
  const int yc = y0 + blockIdx.y;
  const int xa = x0 + blockIdx.x * cw;
  const int cwc = min(cw, x1 - xa + 1);
  const int rx = sp.rx, ry = sp.ry;
  const bool contig = 2 * rx + 1 <= cwc;
  const int nV = contig ? cwc + 2 * rx + 1 : 2 * cwc;
  const int Ya = yc - ry, Yb = yc + ry + 1;
  const int c0 = first_cross(Ya, g.TY);
  const int ncross = c0 < Yb ? (Yb - 1 - c0) / g.TY + 1 : 0;
  double be[NT];
  series_coeffs<NT>(sp.ay, yc, be);
  const int tid = threadIdx.x;
  const int grp = __builtin_amdgcn_readfirstlane(tid / nvpad);
  const int xi = tid - grp * nvpad;
  const bool has_x = xi < nV;
  const int X = !has_x ? xa : (contig ? xa - rx + xi
                                      : (xi < cwc ? xa - rx + xi : xa + rx + 1 + xi - cwc));
  const int tlo = tile_of(xa - rx), ntl = tile_of(xa + cwc + rx) - tlo + 1;
  const bool win = tid < cwc;
  const int xc = xa + tid;
  double al[NT];
  series_coeffs<NT>(sp.ax, win ? xc : xa, al);
  const int i1 = tid, i2 = contig ? tid + 2 * rx + 1 : cwc + tid;
  const int t1 = win ? tile_of(xc - rx) - tlo : 0, t2 = win ? tile_of(xc + rx + 1) - tlo : 0;
  const size_t offA = (size_t)Ya * g.pitch + 63 + X, offB = (size_t)Yb * g.pitch + 63 + X;
  const size_t offC = (size_t)c0 * g.pitch + 63 + X;
  const double inv_mass = 1.0 / sp.mass;
  double bc = 0.0;
  for (int b = 0; b < g.B; ++b) {
    double* V = Vbuf + (b & 1) * NT * nvpad;
    double* R = Rbuf + (b & 1) * NT * ntl_max;
    if (has_x) {
      if (ncross == 0)
        contract_rows<NT, NG, 0>(gp, g, b, grp, be, offA, offB, offC, 0, V + xi, nvpad);
      else if (ncross == 1)
        contract_rows<NT, NG, 1>(gp, g, b, grp, be, offA, offB, offC, 1, V + xi, nvpad);
      else
        contract_rows<NT, NG, -1>(gp, g, b, grp, be, offA, offB, offC, ncross, V + xi, nvpad);
    }
    for (int it = tid; it < NT * ntl; it += blockDim.x) {
      const int i = it / ntl, t = it - (it / ntl) * ntl;
      double r = 0.0;
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const size_t pb = (size_t)((i * NT + j) * g.B + b);
        const double* rcp = gp.RC + (pb * g.NTX + tlo + t) * (size_t)(g.H + 1);
        r = fma(be[j], rcp[Yb] - rcp[Ya], r);
      }
      R[i * ntl_max + t] = r;
    }
    __syncthreads();
    if (win) {
      double h = 0.0;
#pragma unroll
      for (int i = 0; i < NT; ++i)
        h = fma(al[i],
                (V[i * nvpad + i2] + R[i * ntl_max + t2]) - (V[i * nvpad + i1] + R[i * ntl_max + t1]),
                h);
      bc += sqrt(fmax(h * inv_mass, 0.0) * fmax((double)tmpl[b], 0.0));
    }
  }
  if (win) map[(size_t)(yc - y0) * (x1 - x0 + 1) + (xc - x0)] = (float)bc;
}

inline GaussPlanes gauss_planes(const SwihLayout& L, int set, const char* ws) {
  const char* sb = ws + (size_t)set * L.set_bytes;
  return GaussPlanes{(const float*)(sb + L.off_planes), (const double*)(sb + L.off_RC)};
}

template <int NT>
hipError_t query_gauss(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                       const int32_t* centres, int32_t n, float* hist, hipStream_t s) {
  const size_t lds = sizeof(double) * (size_t)L.g.B * NT;
  hipLaunchKernelGGL(k_query_gauss<NT>, dim3((unsigned)n), dim3(256), lds, s, L.g, sp,
                     gauss_planes(L, set, ws), centres, hist);
  return hipGetLastError();
}

template <int NT>
hipError_t match_gauss(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                       const float* tmpl, int x0, int y0, int x1, int y1, float* map,
                       hipStream_t s) {
  constexpr int NG = 3;
  const int nx = x1 - x0 + 1, ny = y1 - y0 + 1;
  const int span = 2 * sp.rx + 1;
  // columns per group: NG * maxV threads <= 1024 and the double-buffered V
  // table within 60 KB of LDS
  int maxV = (60000 / (16 * NT)) / 64 * 64;
  if (maxV > 320) maxV = 320;
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
  const int nvpad = (nV + 63) / 64 * 64;
  const int ntl_max = (cw + span + 63) / 64 + 2;  // tile columns one block can touch
  const size_t lds = sizeof(double) * (size_t)2 * NT * (nvpad + ntl_max);
  const unsigned nch = (unsigned)((nx + cw - 1) / cw);
  hipLaunchKernelGGL((k_match_gauss<NT, NG>), dim3(nch, (unsigned)ny), dim3(NG * nvpad), lds, s,
                     L.g, sp, gauss_planes(L, set, ws), tmpl, x0, y0, x1, cw, nvpad, ntl_max,
                     map);
  return hipGetLastError();
}

}  // namespace

#define SWIH_NT_DISPATCH(NTV, CALL) \
  switch (NTV) {                    \
    case 3: return CALL(3);         \
    case 5: return CALL(5);         \
    case 7: return CALL(7);         \
    case 9: return CALL(9);         \
    case 11: return CALL(11);       \
    case 13: return CALL(13);       \
    case 15: return CALL(15);       \
    case 17: return CALL(17);       \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_query(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                        const int32_t* centres, int32_t n, float* hist, uint32_t* hist_raw,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long nt = (long)n * L.g.B;
  const dim3 grid((unsigned)((nt + 255) / 256));
  const uint32_t* planes = (const uint32_t*)(ws + L.off_planes);
  switch (sp.kind) {
    case 0:
      hipLaunchKernelGGL(k_query_int<0>, grid, dim3(256), 0, s, L.g, sp, planes, centres, n, hist,
                         hist_raw);
      return hipGetLastError();
    case 1:
      hipLaunchKernelGGL(k_query_int<1>, grid, dim3(256), 0, s, L.g, sp, planes, centres, n, hist,
                         hist_raw);
      return hipGetLastError();
    case 2:
      hipLaunchKernelGGL(k_query_int<2>, grid, dim3(256), 0, s, L.g, sp, planes, centres, n, hist,
                         hist_raw);
      return hipGetLastError();
    case 3: {
#define SWIH_Q(NT) query_gauss<NT>(L, sp, set, ws, centres, n, hist, s)
      SWIH_NT_DISPATCH(L.g.nI, SWIH_Q)
#undef SWIH_Q
    }
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_match(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                        const float* tmpl, const uint32_t* tmpl_raw, int32_t x0, int32_t y0,
                        int32_t x1, int32_t y1, float* map, hipStream_t s) {
  if (x1 < x0 || y1 < y0) return hipSuccess;
  const int nx = x1 - x0 + 1, ny = y1 - y0 + 1;
  const uint32_t* planes = (const uint32_t*)(ws + L.off_planes);
  const dim3 gi((unsigned)((nx + 63) / 64), (unsigned)((ny + 3) / 4)), bi(64, 4);
  switch (sp.kind) {
    case 0:
      hipLaunchKernelGGL(k_match_int<0>, gi, bi, 0, s, L.g, sp, planes, tmpl, tmpl_raw, x0, y0,
                         x1, y1, map);
      return hipGetLastError();
    case 1:
      hipLaunchKernelGGL(k_match_int<1>, gi, bi, 0, s, L.g, sp, planes, tmpl, tmpl_raw, x0, y0,
                         x1, y1, map);
      return hipGetLastError();
    case 2:
      hipLaunchKernelGGL(k_match_int<2>, gi, bi, 0, s, L.g, sp, planes, tmpl, tmpl_raw, x0, y0,
                         x1, y1, map);
      return hipGetLastError();
    case 3: {
#define SWIH_M(NT) match_gauss<NT>(L, sp, set, ws, tmpl, x0, y0, x1, y1, map, s)
      SWIH_NT_DISPATCH(L.g.nI, SWIH_M)
#undef SWIH_M
    }
    default: return hipErrorInvalidValue;
  }
}

}  // namespace swih
