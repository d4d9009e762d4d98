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

// pl points at row 0, column 0 of a plane; rs is the plane's row stride.
__device__ __forceinline__ uint32_t at_u(const uint32_t* __restrict__ pl, int64_t rs, int Y, int X) {
  return pl[(size_t)Y * rs + X];
}

// Exact H_b of an integer kernel at (xc, yc) (uint32 arithmetic modulo 2^32).
template <int KIND>
__device__ __forceinline__ uint32_t hist_int(const uint32_t* __restrict__ planes,
                                             const SwihGeom& g, int b, int xc, int yc,
                                             const ScaleParams& sp) {
  const uint32_t* p0 = planes + swih_elem(g, 0, b, 0, 0);
  const int xa = xc - sp.rx, xb = xc + sp.rx + 1, ya = yc - sp.ry, yb = yc + sp.ry + 1;
  if (KIND == 0) {
    return at_u(p0, g.row_stride, yb, xb) - at_u(p0, g.row_stride, ya, xb) - at_u(p0, g.row_stride, yb, xa) +
           at_u(p0, g.row_stride, ya, xa);
  } else if (KIND == 1) {
    const int xm = xc + 1, ym = yc + 1;
    const uint32_t* px = planes + swih_elem(g, 1, b, 0, 0);
    const uint32_t* py = planes + swih_elem(g, 2, b, 0, 0);
    // 3 x 3 corner grid per plane
    uint32_t c1[3][3], cx[3][3], cy[3][3];
    const int Ys[3] = {ya, ym, yb}, Xs[3] = {xa, xm, xb};
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        c1[r][c] = at_u(p0, g.row_stride, Ys[r], Xs[c]);
        cx[r][c] = at_u(px, g.row_stride, Ys[r], Xs[c]);
        cy[r][c] = at_u(py, g.row_stride, Ys[r], Xs[c]);
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
      const uint32_t* pl = planes + swih_elem(g, p, b, 0, 0);
      bx[p] = at_u(pl, g.row_stride, yb, xb) - at_u(pl, g.row_stride, ya, xb) - at_u(pl, g.row_stride, yb, xa) +
              at_u(pl, g.row_stride, ya, xa);
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
  const int64_t rs = g.row_stride;
  const int txa = tile_of(xa), txb = tile_of(xb);
  for (int it = threadIdx.x; it < g.B * NT; it += blockDim.x) {
    const int b = it / NT, i = it - (it / NT) * NT;
    // the NT y-term planes of x term i are row-interleaved: plane j at + j * pitch
    const float* lp = gp.L + swih_elem(g, i * NT, b, 0, 0);
    float aA[NT], bA[NT], aB[NT], bB[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const float* q = lp + (size_t)j * g.pitch;
      aA[j] = q[(size_t)ya * rs + xa];
      bA[j] = q[(size_t)yb * rs + xa];
      aB[j] = q[(size_t)ya * rs + xb];
      bB[j] = q[(size_t)yb * rs + xb];
    }
    double d[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j)
      d[j] = ((double)bB[j] - (double)aB[j]) - ((double)bA[j] - (double)aA[j]);
    for (int c = first_cross(ya, g.TY); c < yb; c += g.TY) {
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const float* q = lp + (size_t)j * g.pitch + (size_t)c * rs;
        d[j] += (double)q[xb] - (double)q[xa];
      }
    }
    double hi = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const size_t pb = (size_t)((i * NT + j) * g.B + b);
      const double* rA = gp.RC + (pb * g.NTX + txa) * (size_t)(g.H + 1);
      const double* rB = gp.RC + (pb * g.NTX + txb) * (size_t)(g.H + 1);
      d[j] += (rB[yb] - rB[ya]) - (rA[yb] - rA[ya]);
      hi = fma(be[j], d[j], hi);
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

// A block-uniform double made visibly uniform (kept in scalar registers).
__device__ __forceinline__ double uniform(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// One coefficient of the series at centre coordinate c: index 0 -> a_0,
// 2k-1 -> a_k cos(2 pi k c / P), 2k -> a_k sin(2 pi k c / P).
__device__ __forceinline__ double series_coeff(const GaussAxis& ax, int c, int idx) {
  if (idx == 0) return ax.a[0];
  const int k = (idx + 1) / 2;
  const long ph = ((long)k * c) % ax.P;
  const double ang = 2.0 * M_PI * (double)ph / (double)ax.P;
  return ax.a[k] * ((idx & 1) ? cos(ang) : sin(ang));
}

// Dense map.  One block per (row of centres yc, chunk of cw centres); NG
// groups of threads, one thread per (group, plane column X the chunk's windows
// touch: X = xc - rx and xc + rx + 1).  With the y terms contracted,
//   V_i(X) = sum_j beta_j(yc) (P_ij[yb][X] - P_ij[ya][X]),
// the window histogram is H_b(xc) = sum_i alpha_i(xc) (V_i(xc+rx+1) - V_i(xc-rx)).
// Each column therefore folds its own V_i into the two quantities the windows
// need from it,
//   G+(X) = sum_i alpha_i(X - rx - 1) V_i(X)   (X is a right edge)
//   G-(X) = sum_i alpha_i(X + rx) V_i(X)       (X is a left edge),
// and only those cross LDS: H_b(xc) = G+(xc + rx + 1) - G-(xc - rx).  The row
// carries of V_i depend on X only through its tile column and are tabulated
// for every bin once per block.  Per bin: the column threads load their
// L rows (all j of one i together), one barrier (LDS double-buffered by bin
// parity), the window threads accumulate sqrt(p_b t_b).
template <int NT, int NG>
__global__ __launch_bounds__(1024) void k_match_gauss(SwihGeom g, ScaleParams sp, GaussPlanes gp,
                                                      const float* __restrict__ tmpl, int x0,
                                                      int y0, int x1, int cw, int nvpad,
                                                      int ntl_max, float* __restrict__ map) {
  extern __shared__ double sm[];
  double* Gb = sm;                                  // [2][NG][2][nvpad]
  double* R = sm + 2 * NG * 2 * nvpad;              // [B][NT][ntl_max]
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
      const size_t pb = (size_t)((i * NT + j) * g.B + b);
      const double* rcp = gp.RC + (pb * g.NTX + tlo + t) * (size_t)(g.H + 1);
      acc = fma(be[j], rcp[Yb] - rcp[Ya], acc);
    }
    R[(b * NT + i) * ntl_max + t] = acc;
  }
  const int grp = __builtin_amdgcn_readfirstlane(tid / nvpad);
  const int xi = tid - grp * nvpad;
  const bool has_x = xi < nV;
  const int X = !has_x ? xa : (contig ? xa - rx + xi
                                      : (xi < cwc ? xa - rx + xi : xa + rx + 1 + xi - cwc));
  const int tX = tile_of(X) - tlo;
  // alpha at the two windows this column serves, for this group's x terms
  constexpr int NI = (NT + NG - 1) / NG;
  double ap[NI], am[NI];
#pragma unroll
  for (int ii = 0; ii < NI; ++ii) {
    const int i = grp + ii * NG;
    ap[ii] = i < NT ? series_coeff(sp.ax, max(X - rx - 1, 0), i) : 0.0;
    am[ii] = i < NT ? series_coeff(sp.ax, X + rx, i) : 0.0;
  }
  const int64_t rs = g.row_stride;
  const size_t offA = (size_t)Ya * rs + X, offB = (size_t)Yb * rs + X, offC = (size_t)c0 * rs + X;
  const bool win = tid < cwc;
  const int xc = xa + tid;
  const int i1 = tid, i2 = contig ? tid + 2 * rx + 1 : cwc + tid;
  const double inv_mass = 1.0 / sp.mass;
  double bc = 0.0;
  __syncthreads();
  for (int b = 0; b < g.B; ++b) {
    double* Gp = Gb + (b & 1) * NG * 2 * nvpad;
    if (has_x) {
      double gplus = 0.0, gminus = 0.0;
#pragma unroll 1
      for (int ii = 0; ii < NI; ++ii) {
        const int i = grp + ii * NG;
        if (i >= NT) break;
        const float* lp = gp.L + swih_elem(g, i * NT, b, 0, 0);
        float la[NT], lb[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          la[j] = lp[offA + (size_t)j * g.pitch];
          lb[j] = lp[offB + (size_t)j * g.pitch];
        }
        double v = R[(b * NT + i) * ntl_max + tX];
#pragma unroll
        for (int j = 0; j < NT; ++j) v = fma(be[j], (double)lb[j] - (double)la[j], v);
        for (int c = 0; c < ncross; ++c) {
          float lc[NT];
#pragma unroll
          for (int j = 0; j < NT; ++j) lc[j] = lp[offC + (size_t)c * g.TY * rs + (size_t)j * g.pitch];
#pragma unroll
          for (int j = 0; j < NT; ++j) v = fma(be[j], (double)lc[j], v);
        }
        gplus = fma(ap[ii], v, gplus);
        gminus = fma(am[ii], v, gminus);
      }
      Gp[(grp * 2 + 0) * nvpad + xi] = gplus;
      Gp[(grp * 2 + 1) * nvpad + xi] = gminus;
    }
    __syncthreads();
    if (win) {
      double hh = 0.0;
#pragma unroll
      for (int q = 0; q < NG; ++q) hh += Gp[(q * 2 + 0) * nvpad + i2] - Gp[(q * 2 + 1) * nvpad + i1];
      bc += sqrt(fmax(hh * inv_mass, 0.0) * fmax((double)tmpl[b], 0.0));
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
  const int maxV = 320;  // NG * maxV threads <= 1024
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
  const size_t lds =
      sizeof(double) * ((size_t)2 * NG * 2 * nvpad + (size_t)L.g.B * NT * ntl_max);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const unsigned nch = (unsigned)((nx + cw - 1) / cw);
  hipLaunchKernelGGL((k_match_gauss<NT, NG>), dim3(nch, (unsigned)ny), dim3(NG * nvpad), lds, s,
                     L.g, sp, gauss_planes(L, set, ws), tmpl, x0, y0, x1, cw, nvpad, ntl_max, map);
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
