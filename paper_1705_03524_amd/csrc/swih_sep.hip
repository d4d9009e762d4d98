// Separable two-pass form of the Gaussian-series weighted histograms
// (kernel SWIH_GAUSSIAN_SEP).
//
// The Gaussian's weight terms are products u_i(x) v_j(y) of two 1-D families
// (1, cos(2 pi k t / P), sin(2 pi k t / P)), so the translated window sum of
// Sec. 2.1 factors into two 1-D weighted integral histograms:
//   row pass     h_b(xc; y)  = sum_i alpha_i(xc) W_ib(xc; y),
//                W_ib(xc; y) = sum_{|x - xc| <= rx} [Q(f(x, y)) = b] u_i(x)
//   column pass  H_b(xc, yc) = sum_j beta_j(yc) sum_{|y - yc| <= ry} h_b(xc; y) v_j(y)
// with alpha, beta the series coefficients at the centre (the translation).
// Each 1-D window sum is a difference of two prefix sums (a 1-D weighted
// integral histogram, Eq. 2 per axis); walking the centre one step moves both
// corners one step, so a wave that sweeps consecutive centres keeps the
// window sums and updates them by the two prefix increments that enter and
// leave -- O(1) per centre, whatever the window size.
//
// Row pass: the x terms are stored in fixed point (integers round(u 2^24)),
// so the row window sums are integers below 2^37 and exact in double; the
// row results h are stored as float.  Column pass: window sums of h v_j in
// double, restarted from a direct sum at the start of every segment of SY
// centre rows (segments start at multiples of SY in absolute rows, so a value
// depends only on its centre, never on the requested rectangle).
#include <math.h>
#include <string.h>

#include "swih_internal.h"

namespace swih {
namespace {

constexpr int WG = 256;                 // four independent waves per block
constexpr int WPB = WG / 64;
constexpr double kFix = 16777216.0;     // 2^24

__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Lanes that serve the bins of one row / centre: a power of two >= B, at most 64.
__host__ __device__ inline int bin_lanes(int B) {
  int p = 1;
  while (p < B && p < 64) p <<= 1;
  return p;
}

// u_idx(t): 1, cos(2 pi k t / P) for odd idx, sin for even idx (k = (idx + 1) / 2),
// with the phase k t reduced exactly modulo P.
__device__ double axis_term(const GaussAxis& ax, int t, int idx) {
  if (idx == 0) return 1.0;
  const int k = (idx + 1) / 2;
  const long ph = ((long)k * t) % ax.P;
  const double ang = 2.0 * M_PI * (double)ph / (double)ax.P;
  return (idx & 1) ? cos(ang) : sin(ang);
}

// Coefficient of term idx in the series translated to centre c:
// g(t - c) = a_0 + sum_k a_k (cos(wkt) cos(wkc) + sin(wkt) sin(wkc)).
__device__ double axis_coeff(const GaussAxis& ax, int c, int idx) {
  if (idx == 0) return ax.a[0];
  return ax.a[(idx + 1) / 2] * axis_term(ax, c, idx);
}

// ---------------------------------------------------------------- tables
__device__ void sep_tables(const SepBuildArgs& a, int vb) {
  const SepGeom& g = a.g;
  const long t = (long)vb * WG + threadIdx.x;
  const long n1 = (long)g.W * g.nT;
  const long n2 = n1 + (long)g.Wv * g.nT;
  const long n3 = n2 + (long)g.H * g.nT;
  const long n4 = n3 + (long)g.Hv * g.nT;
  if (t < n1) {
    const int x = (int)(t / g.nT), i = (int)(t % g.nT);
    a.ux[t] = rint(axis_term(a.ax, x, i) * kFix);
  } else if (t < n2) {
    const long r = t - n1;
    const int v = (int)(r / g.nT), i = (int)(r % g.nT);
    a.al[r] = axis_coeff(a.ax, g.rx + v, i) / kFix;
  } else if (t < n3) {
    const long r = t - n2;
    const int y = (int)(r / g.nT), j = (int)(r % g.nT);
    a.vy[r] = rint(axis_term(a.ay, y, j) * kFix) / kFix;
  } else if (t < n4) {
    const long r = t - n3;
    const int u = (int)(r / g.nT), j = (int)(r % g.nT);
    a.be[r] = axis_coeff(a.ay, g.ry + u, j);
  }
}

int32_t table_blocks(const SepGeom& g) {
  const long n = (long)(2 * g.W + 2 * g.H) * g.nT;  // >= W + Wv + H + Hv entries
  return (int32_t)((n + WG - 1) / WG);
}

// ---------------------------------------------------------------- walks
// Both passes walk a line of elements (pixels of a row, or rows of h) with a
// window of L elements: step s adds element s; once the window is complete
// (s >= L - 1) it is evaluated for centre c = s - (L - 1), and element c
// leaves.  The per-element table rows a step needs are wave-uniform; each
// wave stages them in its own LDS slice a chunk of CH steps at a time (rows
// of the element entering, and of the centre), together with its lanes' data
// for the chunk in registers, so a chunk costs one memory latency instead of
// one per step.  LDS traffic of one wave is ordered, so the stage-then-read
// sequence only needs the compiler fence.
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over aligned groups of BP lanes (BP a power of two <= 64); every lane of
// a group gets the same value.  Within a 16-lane row: quad_perm [1,0,3,2] and
// [2,3,0,1], then row_half_mirror and row_mirror pair the quads and halves.
__device__ __forceinline__ double group_sum(double v, int BP) {
  if (BP >= 2) v += dpp_f64<0xB1>(v);
  if (BP >= 4) v += dpp_f64<0x4E>(v);
  if (BP >= 8) v += dpp_f64<0x141>(v);
  if (BP >= 16) v += dpp_f64<0x140>(v);
  if (BP >= 32) v += __shfl_xor(v, 16, 64);
  if (BP >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// Table rows [max(r0, lo), min(r0 + N, hi)) of a [rows][NT] double table, held
// in registers between load() (all loads issued back to back) and store()
// into LDS as dst[(r - r0) * NT + i].
template <int NT, int N>
struct StageRows {
  static constexpr int PER = (N * NT + 63) / 64;
  double v[PER];
  int a, b;
  __device__ __forceinline__ void load(const double* __restrict__ tab, int r0, int lo, int hi,
                                       int lane) {
    a = (max(r0, lo) - r0) * NT;
    b = (min(r0 + N, hi) - r0) * NT;
    if (b <= a) return;  // uniform
    const double* src = tab + (long)r0 * NT;
#pragma unroll
    for (int k = 0; k < PER; ++k) v[k] = src[min(max(lane + 64 * k, a), b - 1)];
  }
  __device__ __forceinline__ void store(double* dst, int lane) const {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int t = lane + 64 * k;
      if (t >= a && t < b) dst[t] = v[k];
    }
  }
};

// ---------------------------------------------------------------- row pass
// A wave owns RPW = 64 / BP image rows (BP lanes per row, one bin per lane and
// chunk of 64 bins) and SX consecutive centre columns; it walks the centres
// left to right with NT running window sums per bin.  Chunks are software
// pipelined: the pixels and table rows of chunk k + 1 are in flight while
// chunk k is computed from registers and LDS.
template <int NT, int NCH>
__device__ void sep_rows(const SepBuildArgs& a, int vb) {
  constexpr int CH = 16;
  __shared__ double stage[WPB][3][CH * NT];
  const SepGeom& g = a.g;
  const int B = g.B;
  const int BP = NCH > 1 ? 64 : bin_lanes(B);
  const int RPW = 64 / BP;
  const int lane = (int)(threadIdx.x & 63);
  const int wid = (int)(threadIdx.x >> 6);
  const int wv = rfl(vb * WPB + wid);
  const int nsx = (g.Wv + g.SX - 1) / g.SX;
  const int rg = wv / nsx;
  if (rg * RPW >= g.H) return;  // padding waves of the last block (uniform per wave)
  const int v0 = (wv - rg * nsx) * g.SX;
  const int v1 = min(v0 + g.SX, g.Wv);
  const int y = rg * RPW + lane / BP;
  const bool row_ok = y < g.H;
  const uint8_t* __restrict__ row = a.img + (size_t)(row_ok ? y : g.H - 1) * a.ipitch;
  float* __restrict__ hr = a.hr;
  double* s_in = stage[wid][0];
  double* s_out = stage[wid][1];
  double* s_al = stage[wid][2];
  int bin[NCH];
  bool bok[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    bin[c] = lane % BP + 64 * c;
    bok[c] = row_ok && bin[c] < B;
  }
  double win[NCH][NT];
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int i = 0; i < NT; ++i) win[c][i] = 0.0;
  // The window sums only ever add or remove integer terms (masks 0 or 1 times
  // round(u 2^24)), so they are exact.
  const int L = g.w, nc = v1 - v0, nsteps = L - 1 + nc;
  int qi[CH], qo[CH];
  StageRows<NT, CH> t_in, t_out, t_al;
  auto fetch = [&](int s0, int (&pi)[CH], int (&po)[CH]) {
    const int c0 = s0 - (L - 1);
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      pi[u] = row[v0 + min(s0 + u, nsteps - 1)];
      po[u] = row[v0 + min(max(c0 + u, 0), nc - 1)];
    }
    t_in.load(a.ux, v0 + s0, v0, v0 + nsteps, lane);
    t_out.load(a.ux, v0 + c0, v0, v1, lane);
    t_al.load(a.al, v0 + c0, v0, v1, lane);
  };
  auto put = [&]() {
    wave_fence();  // reads of the previous chunk are issued (LDS is in order per wave)
    t_in.store(s_in, lane);
    t_out.store(s_out, lane);
    t_al.store(s_al, lane);
    wave_fence();
  };
  fetch(0, qi, qo);
  put();
  for (int s0 = 0; s0 < nsteps; s0 += CH) {
    const int c0 = s0 - (L - 1);  // centre of the chunk's first step
    const bool more = s0 + CH < nsteps;
    int ni[CH], no[CH];
    if (more) fetch(s0 + CH, ni, no);
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      if (s0 + u < nsteps) {
        const double* ui = s_in + u * NT;
        const int q = (qi[u] * B) >> 8;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          const double m = q == bin[c] ? 1.0 : 0.0;
#pragma unroll
          for (int i = 0; i < NT; ++i) win[c][i] = fma(m, ui[i], win[c][i]);
        }
      }
      if (s0 + u >= nsteps || c0 + u < 0) continue;
      const int v = v0 + c0 + u;
      const double* uo = s_out + u * NT;
      const double* av = s_al + u * NT;
      const int q = (qo[u] * B) >> 8;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        double hv = 0.0;
#pragma unroll
        for (int i = 0; i < NT; ++i) hv = fma(av[i], win[c][i], hv);
        if (bok[c]) hr[((size_t)y * g.Wv + v) * B + bin[c]] = (float)hv;
        const double m = q == bin[c] ? -1.0 : 0.0;
#pragma unroll
        for (int i = 0; i < NT; ++i) win[c][i] = fma(m, uo[i], win[c][i]);
      }
    }
    if (more) {
      put();
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        qi[u] = ni[u];
        qo[u] = no[u];
      }
    }
  }
}

int32_t row_blocks(const SepGeom& g) {
  const int BP = g.B > 64 ? 64 : bin_lanes(g.B);
  const long waves = (long)((g.H + 64 / BP - 1) / (64 / BP)) * ((g.Wv + g.SX - 1) / g.SX);
  return (int32_t)((waves + WPB - 1) / WPB);
}

// ---------------------------------------------------------------- queries
// One wave per centre, one lane per bin (chunks of 64 bins): the column
// window sums of h v_j are taken directly over the h rows of the window.
template <int NT, int NCH>
__device__ void sep_query(const SepQueryArgs& a, int vb) {
  constexpr int CH = 16 / NCH;
  __shared__ double stage[WPB][CH * NT];
  const SepGeom& g = a.g;
  const int wid = (int)(threadIdx.x >> 6);
  const int n = rfl(vb * WPB + wid);
  if (n >= a.n) return;
  const int lane = (int)(threadIdx.x & 63);
  const int xc = min(max(a.centres[2 * n], g.rx), g.W - 1 - g.rx);
  const int yc = min(max(a.centres[2 * n + 1], g.ry), g.H - 1 - g.ry);
  const int B = g.B;
  const float* __restrict__ hcol = a.hr + (size_t)(xc - g.rx) * B;
  const size_t rstride = (size_t)g.Wv * B;
  double* s_v = stage[wid];
  double win[NCH][NT];
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int j = 0; j < NT; ++j) win[c][j] = 0.0;
  const int y0 = yc - g.ry;
  float hv[CH][NCH];
  StageRows<NT, CH> t_v;
  auto fetch = [&](int s0, float (&p)[CH][NCH]) {
#pragma unroll
    for (int u = 0; u < CH; ++u)
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int b = min(lane + 64 * c, B - 1);
        p[u][c] = hcol[(size_t)(y0 + min(s0 + u, g.h - 1)) * rstride + b];
      }
    t_v.load(a.vy, y0 + s0, y0, y0 + g.h, lane);
  };
  auto put = [&]() {
    wave_fence();
    t_v.store(s_v, lane);
    wave_fence();
  };
  fetch(0, hv);
  put();
  for (int s0 = 0; s0 < g.h; s0 += CH) {
    const bool more = s0 + CH < g.h;
    float nv[CH][NCH];
    if (more) fetch(s0 + CH, nv);
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      if (s0 + u >= g.h) continue;
      const double* vv = s_v + u * NT;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const double h = lane + 64 * c < B ? (double)hv[u][c] : 0.0;
#pragma unroll
        for (int j = 0; j < NT; ++j) win[c][j] = fma(h, vv[j], win[c][j]);
      }
    }
    if (more) {
      put();
#pragma unroll
      for (int u = 0; u < CH; ++u)
#pragma unroll
        for (int c = 0; c < NCH; ++c) hv[u][c] = nv[u][c];
    }
  }
  const double* bb = a.be + (size_t)(yc - g.ry) * NT;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int b = lane + 64 * c;
    double hb = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) hb = fma(bb[j], win[c][j], hb);
    if (b < B) a.hist[(size_t)n * B + b] = (float)(hb * a.inv_mass);
  }
}

// ---------------------------------------------------------------- dense map
// A wave owns XPW = 64 / BP consecutive centres of one segment of SY centre
// rows (BP lanes per centre, one bin per lane and chunk).  It walks the h
// rows down the segment: per centre row, H_b from the NT column window sums
// and the translation coefficients beta(yc), the Bhattacharyya terms summed
// over the centre's lanes, then the h row that leaves is removed.
template <int NT, int NCH>
__device__ void sep_match(const SepMatchArgs& a, int vb) {
  constexpr int CH = 16 / NCH;
  __shared__ double stage[WPB][3][CH * NT];
  const SepGeom& g = a.g;
  const int B = g.B;
  const int BP = NCH > 1 ? 64 : bin_lanes(B);
  const int XPW = 64 / BP;
  const int lane = (int)(threadIdx.x & 63);
  const int wid = (int)(threadIdx.x >> 6);
  const int wv = rfl(vb * WPB + wid);
  const int seg = wv / a.nwx;
  if (seg >= a.nseg) return;  // padding waves of the last block (uniform per wave)
  const int wx = wv - seg * a.nwx;
  const int xc = a.x0 + wx * XPW + lane / BP;
  const bool x_ok = xc <= a.x1;
  const int k = a.seg0 + seg;
  const int ys = max(k * g.SY, a.y0), ye = min(k * g.SY + g.SY - 1, a.y1);
  const int yi = max(k * g.SY, g.ry);
  const float* __restrict__ hcol = a.hr + (size_t)((x_ok ? xc : a.x0) - g.rx) * B;
  const size_t rstride = (size_t)g.Wv * B;
  double* s_in = stage[wid][0];
  double* s_out = stage[wid][1];
  double* s_be = stage[wid][2];
  int bin[NCH], bcl[NCH];
  bool bok[NCH];
  double tv[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    bin[c] = lane % BP + 64 * c;
    bok[c] = bin[c] < B;
    bcl[c] = min(bin[c], B - 1);
    tv[c] = bok[c] ? fmax((double)a.tmpl[bin[c]], 0.0) : 0.0;
  }
  double win[NCH][NT];
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int j = 0; j < NT; ++j) win[c][j] = 0.0;
  const int mw = a.x1 - a.x0 + 1;
  const int L = g.h, nc = ye - yi + 1, nsteps = L - 1 + nc;
  const int e0 = yi - g.ry;  // h row of element 0; centre c sits at row yi + c
  float hi[CH][NCH], ho[CH][NCH];
  StageRows<NT, CH> t_in, t_out, t_be;
  auto fetch = [&](int s0, float (&pi)[CH][NCH], float (&po)[CH][NCH]) {
    const int c0 = s0 - (L - 1);
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const size_t ri = (size_t)(e0 + min(s0 + u, nsteps - 1)) * rstride;
      const size_t ro = (size_t)(e0 + min(max(c0 + u, 0), nc - 1)) * rstride;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        pi[u][c] = hcol[ri + bcl[c]];
        po[u][c] = hcol[ro + bcl[c]];
      }
    }
    t_in.load(a.vy, e0 + s0, e0, e0 + nsteps, lane);
    t_out.load(a.vy, e0 + c0, e0, e0 + nc, lane);
    t_be.load(a.be, e0 + c0, e0, e0 + nc, lane);  // beta row of centre yc is yc - ry
  };
  auto put = [&]() {
    wave_fence();
    t_in.store(s_in, lane);
    t_out.store(s_out, lane);
    t_be.store(s_be, lane);
    wave_fence();
  };
  fetch(0, hi, ho);
  put();
  for (int s0 = 0; s0 < nsteps; s0 += CH) {
    const int c0 = s0 - (L - 1);
    const bool more = s0 + CH < nsteps;
    float ni[CH][NCH], no[CH][NCH];
    if (more) fetch(s0 + CH, ni, no);
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      if (s0 + u < nsteps) {
        const double* vi = s_in + u * NT;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          const double h = bok[c] ? (double)hi[u][c] : 0.0;
#pragma unroll
          for (int j = 0; j < NT; ++j) win[c][j] = fma(h, vi[j], win[c][j]);
        }
      }
      if (s0 + u >= nsteps || c0 + u < 0) continue;
      const int yc = yi + c0 + u;
      if (yc >= ys) {
        const double* bb = s_be + u * NT;
        double sb = 0.0;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          double hb = 0.0;
#pragma unroll
          for (int j = 0; j < NT; ++j) hb = fma(bb[j], win[c][j], hb);
          sb += (double)sqrtf((float)(fmax(hb * a.inv_mass, 0.0) * tv[c]));
        }
        sb = group_sum(sb, BP);
        if (x_ok && lane % BP == 0) a.map[(size_t)(yc - a.y0) * mw + (xc - a.x0)] = (float)sb;
      }
      const double* vo = s_out + u * NT;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const double h = bok[c] ? -(double)ho[u][c] : 0.0;
#pragma unroll
        for (int j = 0; j < NT; ++j) win[c][j] = fma(h, vo[j], win[c][j]);
      }
    }
    if (more) {
      put();
#pragma unroll
      for (int u = 0; u < CH; ++u)
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          hi[u][c] = ni[u][c];
          ho[u][c] = no[u][c];
        }
    }
  }
}

}  // namespace

// Single launch: one block per virtual block.  Batched launch: a grid-stride
// loop over all items' virtual blocks, each block finding its item by binary
// search over the prefix of block counts.
template <class A, void (*BODY)(const A&, int)>
__global__ __launch_bounds__(WG) void k_sep_one(A a) {
  BODY(a, (int)blockIdx.x);
}

template <class A, void (*BODY)(const A&, int)>
__global__ __launch_bounds__(WG) void k_sep_many(const A* __restrict__ items,
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
hipError_t one(const A& a, int32_t nb, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_sep_one<A, BODY>), dim3((unsigned)nb), dim3(WG), 0, s, a);
  return hipGetLastError();
}

template <class A, void (*BODY)(const A&, int)>
hipError_t many(const A* items, const int32_t* prefix, int n, int32_t total, int grid,
                hipStream_t s) {
  if (n <= 0 || total <= 0) return hipSuccess;
  const unsigned gb = (unsigned)(total < grid ? total : grid);
  hipLaunchKernelGGL((k_sep_many<A, BODY>), dim3(gb), dim3(WG), 0, s, items, prefix, n);
  return hipGetLastError();
}

template <int NT, int NCH> constexpr void (*rows_body)(const SepBuildArgs&, int) = sep_rows<NT, NCH>;
template <int NT, int NCH> constexpr void (*query_body)(const SepQueryArgs&, int) = sep_query<NT, NCH>;
template <int NT, int NCH> constexpr void (*match_body)(const SepMatchArgs&, int) = sep_match<NT, NCH>;

int chunks(int B) { return B <= 64 ? 1 : (B <= 128 ? 2 : 4); }

// L<NT, NCH>::run(args...) for the runtime term count and bin chunks.
template <template <int, int> class L, class... Args>
hipError_t dispatch(int nt, int nbins, Args&&... args) {
  const int nch = chunks(nbins);
#define SWIH_SEP_NT(NTV)                                       \
  case NTV:                                                    \
    return nch == 1 ? L<NTV, 1>::run(args...)                  \
                    : (nch == 2 ? L<NTV, 2>::run(args...) : L<NTV, 4>::run(args...));
  switch (nt) {
    SWIH_SEP_NT(3)
    SWIH_SEP_NT(5)
    SWIH_SEP_NT(7)
    SWIH_SEP_NT(9)
    SWIH_SEP_NT(11)
    SWIH_SEP_NT(13)
    SWIH_SEP_NT(15)
    SWIH_SEP_NT(17)
    default: return hipErrorInvalidValue;
  }
#undef SWIH_SEP_NT
}

template <int NT, int NCH> struct RowsOne {
  static hipError_t run(const SepBuildArgs& a, int32_t nb, hipStream_t s) {
    return one<SepBuildArgs, rows_body<NT, NCH>>(a, nb, s);
  }
};
template <int NT, int NCH> struct QueryOne {
  static hipError_t run(const SepQueryArgs& a, int32_t nb, hipStream_t s) {
    return one<SepQueryArgs, query_body<NT, NCH>>(a, nb, s);
  }
};
template <int NT, int NCH> struct MatchOne {
  static hipError_t run(const SepMatchArgs& a, int32_t nb, hipStream_t s) {
    return one<SepMatchArgs, match_body<NT, NCH>>(a, nb, s);
  }
};
template <int NT, int NCH> struct RowsMany {
  static hipError_t run(const SepBuildArgs* u, const int32_t* p, int n, int32_t tot, int grid,
                        hipStream_t s) {
    return many<SepBuildArgs, rows_body<NT, NCH>>(u, p, n, tot, grid, s);
  }
};
template <int NT, int NCH> struct QueryMany {
  static hipError_t run(const SepQueryArgs* it, const int32_t* p, int n, int32_t tot, int grid,
                        hipStream_t s) {
    return many<SepQueryArgs, query_body<NT, NCH>>(it, p, n, tot, grid, s);
  }
};
template <int NT, int NCH> struct MatchMany {
  static hipError_t run(const SepMatchArgs* it, const int32_t* p, int n, int32_t tot, int grid,
                        hipStream_t s) {
    return many<SepMatchArgs, match_body<NT, NCH>>(it, p, n, tot, grid, s);
  }
};

}  // namespace

// ---------------------------------------------------------------- host side
SepLayout sep_layout(int32_t H, int32_t W, int32_t B, int32_t nT) {
  SepLayout L;
  int64_t off = 0;
  L.off_hr = off;
  off += swih_align256((int64_t)H * W * B * 4);
  L.off_ux = off;
  off += swih_align256((int64_t)W * nT * 8);
  L.off_al = off;
  off += swih_align256((int64_t)W * nT * 8);
  L.off_vy = off;
  off += swih_align256((int64_t)H * nT * 8);
  L.off_be = off;
  off += swih_align256((int64_t)H * nT * 8);
  L.set_bytes = off;
  return L;
}

SepGeom sep_geom(int32_t H, int32_t W, int32_t B, int32_t w, int32_t h, int32_t nT) {
  SepGeom g;
  g.H = H;
  g.W = W;
  g.B = B;
  g.w = w;
  g.h = h;
  g.rx = (w - 1) / 2;
  g.ry = (h - 1) / 2;
  g.Wv = W - w + 1;
  g.Hv = H - h + 1;
  g.nT = nT;
  // segment lengths: multiples of 32, at least the window less one, so a
  // segment's start-up walk costs no more than its output walk
  g.SX = 32 * (1 > (w + 30) / 32 ? 1 : (w + 30) / 32);
  g.SY = 32 * (1 > (h + 30) / 32 ? 1 : (h + 30) / 32);
  return g;
}

void sep_build_args(const SepGeom& g, const SepLayout& L, const GaussAxis& ax,
                    const GaussAxis& ay, const uint8_t* img, int32_t img_pitch, char* set_base,
                    SepBuildArgs& a, int32_t (&nb)[2]) {
  memset(&a, 0, sizeof(a));
  a.g = g;
  a.img = img;
  a.ipitch = img_pitch;
  a.hr = (float*)(set_base + L.off_hr);
  a.ux = (double*)(set_base + L.off_ux);
  a.al = (double*)(set_base + L.off_al);
  a.vy = (double*)(set_base + L.off_vy);
  a.be = (double*)(set_base + L.off_be);
  a.ax = ax;
  a.ay = ay;
  nb[0] = table_blocks(g);
  nb[1] = row_blocks(g);
}

void sep_query_args(const SepGeom& g, const SepLayout& L, double mass, const char* set_base,
                    const int32_t* centres, int32_t n, float* hist, SepQueryArgs& a, int32_t& nb) {
  memset(&a, 0, sizeof(a));
  a.g = g;
  a.hr = (const float*)(set_base + L.off_hr);
  a.vy = (const double*)(set_base + L.off_vy);
  a.be = (const double*)(set_base + L.off_be);
  a.inv_mass = 1.0 / mass;
  a.centres = centres;
  a.n = n;
  a.hist = hist;
  nb = (n + WPB - 1) / WPB;
}

void sep_match_args(const SepGeom& g, const SepLayout& L, double mass, const char* set_base,
                    const float* tmpl, int32_t x0, int32_t y0, int32_t x1, int32_t y1, float* map,
                    SepMatchArgs& a, int32_t& nb) {
  memset(&a, 0, sizeof(a));
  a.g = g;
  a.hr = (const float*)(set_base + L.off_hr);
  a.vy = (const double*)(set_base + L.off_vy);
  a.be = (const double*)(set_base + L.off_be);
  a.inv_mass = 1.0 / mass;
  a.tmpl = tmpl;
  a.map = map;
  a.x0 = x0;
  a.y0 = y0;
  a.x1 = x1;
  a.y1 = y1;
  const int XPW = g.B > 64 ? 1 : 64 / bin_lanes(g.B);
  a.nwx = (x1 - x0 + 1 + XPW - 1) / XPW;
  a.seg0 = y0 / g.SY;
  a.nseg = y1 / g.SY - a.seg0 + 1;
  nb = (int32_t)(((long)a.nwx * a.nseg + WPB - 1) / WPB);
}

hipError_t sep_launch_build(const SepBuildArgs& a, const int32_t (&nb)[2], int phases,
                            hipStream_t s) {
  if (phases & 1) {
    const hipError_t e = one<SepBuildArgs, sep_tables>(a, nb[0], s);
    if (e != hipSuccess) return e;
  }
  if (phases & 2) return dispatch<RowsOne>(a.g.nT, a.g.B, a, nb[1], s);
  return hipSuccess;
}

hipError_t sep_launch_query(const SepQueryArgs& a, int32_t nb, hipStream_t s) {
  return dispatch<QueryOne>(a.g.nT, a.g.B, a, nb, s);
}

hipError_t sep_launch_match(const SepMatchArgs& a, int32_t nb, hipStream_t s) {
  return dispatch<MatchOne>(a.g.nT, a.g.B, a, nb, s);
}

hipError_t sep_launch_build_batch(int nt, int nbins, const SepBuildArgs* units,
                                  const int32_t* prefix, int nunits, const int32_t (&total)[2],
                                  int grid, hipStream_t s) {
  const hipError_t e = many<SepBuildArgs, sep_tables>(units, prefix, nunits, total[0], grid, s);
  if (e != hipSuccess) return e;
  return dispatch<RowsMany>(nt, nbins, units, prefix + (nunits + 1), nunits, total[1], grid, s);
}

hipError_t sep_launch_query_batch(int nt, int nbins, const SepQueryArgs* items,
                                  const int32_t* prefix, int n, int32_t total, int grid,
                                  hipStream_t s) {
  return dispatch<QueryMany>(nt, nbins, items, prefix, n, total, grid, s);
}

hipError_t sep_launch_match_batch(int nt, int nbins, const SepMatchArgs* items,
                                  const int32_t* prefix, int n, int32_t total, int grid,
                                  hipStream_t s) {
  return dispatch<MatchMany>(nt, nbins, items, prefix, n, total, grid, s);
}

}  // namespace swih
