// Separable two-pass form of the Gaussian-series weighted histograms
// (kernel SWIH_GAUSSIAN_SEP).
//
// The Gaussian's weight terms are products u_i(x) v_j(y) of two 1-D families
// (1, cos(w_k t), sin(w_k t)), so the translated window sum of
// Sec. 2.1 factors into two 1-D weighted integral histograms:
//   row pass     h_b(xc; y)  = sum_{|x - xc| <= rx} [Q(f(x, y)) = b] g_x(x - xc)
//   column pass  H_b(xc, yc) = sum_{|y - yc| <= ry} h_b(xc; y) g_y(y - yc)
// with g(t) = a_0 + sum_k a_k cos(w_k t).  Per term, the 1-D integral
// histogram's window difference translated to the centre (the product-to-sum
// identity of Sec. 2.1) is the complex sum Z_k = sum_t e(t) exp(i w_k t) over
// the window's offsets t from the centre, and g at every offset follows as
// a_0 Z_0 + sum_k a_k Re Z_k.  A wave walks consecutive centres of a line:
// per step the element entering at +r and the one leaving at -r update Z_k,
// and moving the centre one step rotates Z_k by exp(-i w_k) -- O(1) per
// centre and term, whatever the window size, with no tables: the per-scale
// constants (a_k, exp(i w_k r), exp(i w_k)) sit in scalar registers.
//
// Walks restart from an empty window at the start of every segment (SX
// centre columns, SY centre rows; segments start at absolute multiples of
// the segment length, so a value depends only on its centre, never on the
// requested rectangle).  Sums are in double over at most a few hundred steps;
// the row results h are stored as float.
#include <math.h>
#include <string.h>

#include "swih_internal.h"

namespace swih {
namespace {

constexpr int WG = 256;  // four independent waves per block
constexpr int WPB = WG / 64;

__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Lanes that serve the bins of one row / centre: a power of two >= B, at most 64.
__host__ __device__ inline int bin_lanes(int B) {
  int p = 1;
  while (p < B && p < 64) p <<= 1;
  return p;
}

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}

// Sum over aligned groups of BP lanes (BP a power of two <= 64); every lane of
// a group gets the same value.  Within a 16-lane row: quad_perm [1,0,3,2] and
// [2,3,0,1], then row_half_mirror and row_mirror pair the quads and halves.
__device__ __forceinline__ float group_sum(float v, int BP) {
  if (BP >= 2) v += dpp_f32<0xB1>(v);
  if (BP >= 4) v += dpp_f32<0x4E>(v);
  if (BP >= 8) v += dpp_f32<0x141>(v);
  if (BP >= 16) v += dpp_f32<0x140>(v);
  if (BP >= 32) v += __shfl_xor(v, 16, 64);
  if (BP >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// The translated window sums of one bin along a walk: z0 = sum of the element
// values, (zr_k, zi_k) = Z_k of the header.
template <int K>
struct Walk {
  double z0, zr[K], zi[K];
  __device__ __forceinline__ void clear() {
    z0 = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) zr[k] = zi[k] = 0.0;
  }
  // The window value with element vin entered at +r: a_0 Z_0 + sum_k a_k Re Z_k.
  __device__ __forceinline__ double eval(const SepAxis& A, double vin) const {
    double s = A.a[0] * z0;
#pragma unroll
    for (int k = 0; k < K; ++k) s = fma(A.a[k + 1], zr[k], s);
    return fma(vin, A.g_in, s);
  }
  // vin enters at +r, vout leaves at -r, then the centre moves one step on.
  __device__ __forceinline__ void step(const SepAxis& A, double vin, double vout) {
    const double d = vin - vout, p = vin + vout;
    z0 += d;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double r = fma(d, A.ec[k + 1], zr[k]);
      const double i = fma(p, A.es[k + 1], zi[k]);
      zr[k] = fma(r, A.rc[k + 1], i * A.rs[k + 1]);
      zi[k] = fma(i, A.rc[k + 1], -(r * A.rs[k + 1]));
    }
  }
};

// A walk over a line of elements with a window of L: step s adds element s;
// once the window is complete (s >= L - 1) it is evaluated for centre
// c = s - (L - 1), and element c leaves.  Each chunk of CH steps has its
// lanes' elements in registers; the next chunk's loads are in flight while a
// chunk is computed (software pipelining), so a wave pays one memory latency
// per chunk at most.

// ---------------------------------------------------------------- row pass
// A wave owns RPW = 64 / BP image rows (BP lanes per row, one bin per lane and
// chunk of 64 bins) and SX consecutive centre columns, walked left to right.
template <int K, int NCH>
__device__ void sep_rows(const SepBuildArgs& a, int vb) {
  constexpr int CH = 16;
  constexpr int CW = CH / 4;  // quantised pixels are packed four to a word
  const SepGeom& g = a.g;
  const SepAxis& A = a.ax;
  const int B = g.B;
  const int BP = NCH > 1 ? 64 : bin_lanes(B);
  const int RPW = 64 / BP;
  const int lane = (int)(threadIdx.x & 63);
  const int wv = rfl(vb * WPB + (int)(threadIdx.x >> 6));
  const int nsx = (g.Wv + g.SX - 1) / g.SX;
  const int rg = wv / nsx;
  if (rg * RPW >= g.H) return;  // padding waves of the last block (uniform per wave)
  const int v0 = (wv - rg * nsx) * g.SX;
  const int v1 = min(v0 + g.SX, g.Wv);
  const int y = rg * RPW + lane / BP;
  const bool row_ok = y < g.H;
  const uint8_t* __restrict__ row = a.img + (size_t)(row_ok ? y : g.H - 1) * a.ipitch;
  float* __restrict__ hr = a.hr + (size_t)(row_ok ? y : 0) * g.Wv * B;
  uint32_t bin[NCH];
  bool bok[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    bin[c] = (uint32_t)(lane % BP + 64 * c);
    bok[c] = row_ok && (int)bin[c] < B;
  }
  Walk<K> wk[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) wk[c].clear();
  const int L = g.w, nc = v1 - v0, nsteps = L - 1 + nc;
  uint32_t qi[CW], qo[CW];
  auto fetch = [&](int s0, uint32_t (&pi)[CW], uint32_t (&po)[CW]) {
    const int c0 = s0 - (L - 1);
#pragma unroll
    for (int u4 = 0; u4 < CW; ++u4) {
      uint32_t wi = 0, wo = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int u = 4 * u4 + j;
        // 8-bit pixel times B <= 256 fits the 24-bit multiplier
        const uint32_t bi = __umul24((uint32_t)row[v0 + min(s0 + u, nsteps - 1)], (uint32_t)B) >> 8;
        const uint32_t bo = __umul24((uint32_t)row[v0 + min(max(c0 + u, 0), nc - 1)], (uint32_t)B) >> 8;
        wi |= bi << (8 * j);
        wo |= bo << (8 * j);
      }
      pi[u4] = wi;
      po[u4] = wo;
    }
  };
  fetch(0, qi, qo);
  for (int s0 = 0; s0 < nsteps; s0 += CH) {
    const int c0 = s0 - (L - 1);
    const bool more = s0 + CH < nsteps;
    uint32_t ni[CW], no[CW];
    if (more) fetch(s0 + CH, ni, no);
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      if (s0 + u >= nsteps) continue;
      const bool centre = c0 + u >= 0;
      const uint32_t q_in = (qi[u / 4] >> (8 * (u % 4))) & 255u;
      const uint32_t q_out = (qo[u / 4] >> (8 * (u % 4))) & 255u;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const double m_in = q_in == bin[c] ? 1.0 : 0.0;
        const double m_out = centre && q_out == bin[c] ? 1.0 : 0.0;
        if (centre && bok[c])
          hr[(size_t)(v0 + c0 + u) * B + bin[c]] = (float)wk[c].eval(A, m_in);
        wk[c].step(A, m_in, m_out);
      }
    }
    if (more) {
#pragma unroll
      for (int u4 = 0; u4 < CW; ++u4) {
        qi[u4] = ni[u4];
        qo[u4] = no[u4];
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
// One wave per centre, one lane per bin (chunks of 64 bins): a walk down the
// h rows of the centre's column, evaluated once, at the centre.
template <int K, int NCH>
__device__ void sep_query(const SepQueryArgs& a, int vb) {
  constexpr int CH = 16 / NCH;
  const SepGeom& g = a.g;
  const SepAxis& A = a.ay;
  const int n = rfl(vb * WPB + (int)(threadIdx.x >> 6));
  if (n >= a.n) return;
  const int lane = (int)(threadIdx.x & 63);
  const int xc = min(max(a.centres[2 * n], g.rx), g.W - 1 - g.rx);
  const int yc = min(max(a.centres[2 * n + 1], g.ry), g.H - 1 - g.ry);
  const int B = g.B;
  const float* __restrict__ hcol = a.hr + (size_t)(xc - g.rx) * B;
  const size_t rstride = (size_t)g.Wv * B;
  const int y0 = yc - g.ry, L = g.h;
  Walk<K> wk[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) wk[c].clear();
  float hv[CH][NCH];
  auto fetch = [&](int s0, float (&p)[CH][NCH]) {
#pragma unroll
    for (int u = 0; u < CH; ++u)
#pragma unroll
      for (int c = 0; c < NCH; ++c)
        p[u][c] = hcol[(size_t)(y0 + min(s0 + u, L - 1)) * rstride + min(lane + 64 * c, B - 1)];
  };
  fetch(0, hv);
  for (int s0 = 0; s0 < L; s0 += CH) {
    const bool more = s0 + CH < L;
    float nv[CH][NCH];
    if (more) fetch(s0 + CH, nv);
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      if (s0 + u >= L) continue;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int b = lane + 64 * c;
        const double h = b < B ? (double)hv[u][c] : 0.0;
        if (s0 + u == L - 1) {
          if (b < B) a.hist[(size_t)n * B + b] = (float)(wk[c].eval(A, h) * a.inv_mass);
        } else {
          wk[c].step(A, h, 0.0);
        }
      }
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < CH; ++u)
#pragma unroll
        for (int c = 0; c < NCH; ++c) hv[u][c] = nv[u][c];
    }
  }
}

// ---------------------------------------------------------------- dense map
// A wave owns XPW = 64 / BP consecutive centres of one segment of SY centre
// rows (BP lanes per centre, one bin per lane and chunk) and walks the h rows
// down the segment: per centre row, H_b, the Bhattacharyya terms summed over
// the centre's lanes, and the h rows that enter and leave.
template <int K, int NCH>
__device__ void sep_match(const SepMatchArgs& a, int vb) {
  constexpr int CH = 16 / NCH;
  const SepGeom& g = a.g;
  const SepAxis& A = a.ay;
  const int B = g.B;
  const int BP = NCH > 1 ? 64 : bin_lanes(B);
  const int XPW = 64 / BP;
  const int lane = (int)(threadIdx.x & 63);
  const int wv = rfl(vb * WPB + (int)(threadIdx.x >> 6));
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
  Walk<K> wk[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) wk[c].clear();
  const int mw = a.x1 - a.x0 + 1;
  const int L = g.h, nc = ye - yi + 1, nsteps = L - 1 + nc;
  const int e0 = yi - g.ry;  // h row of element 0; centre c sits at row yi + c
  float hi[CH][NCH], ho[CH][NCH];
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
  };
  fetch(0, hi, ho);
  for (int s0 = 0; s0 < nsteps; s0 += CH) {
    const int c0 = s0 - (L - 1);
    const bool more = s0 + CH < nsteps;
    float ni[CH][NCH], no[CH][NCH];
    if (more) fetch(s0 + CH, ni, no);
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      if (s0 + u >= nsteps) continue;
      const bool centre = c0 + u >= 0;
      const int yc = yi + c0 + u;
      if (centre && yc >= ys) {
        // the Bhattacharyya terms and their sum over bins in float: each term
        // is within an ulp of sqrt(p_b t_b), far inside the series' own error
        float sb = 0.0f;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          const double h = bok[c] ? (double)hi[u][c] : 0.0;
          const double hb = wk[c].eval(A, h);
          sb += sqrtf((float)(fmax(hb * a.inv_mass, 0.0) * tv[c]));
        }
        sb = group_sum(sb, BP);
        if (x_ok && lane % BP == 0) a.map[(size_t)(yc - a.y0) * mw + (xc - a.x0)] = sb;
      }
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const double h_in = bok[c] ? (double)hi[u][c] : 0.0;
        const double h_out = bok[c] && centre ? (double)ho[u][c] : 0.0;
        wk[c].step(A, h_in, h_out);
      }
    }
    if (more) {
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

template <int K, int NCH> constexpr void (*rows_body)(const SepBuildArgs&, int) = sep_rows<K, NCH>;
template <int K, int NCH> constexpr void (*query_body)(const SepQueryArgs&, int) = sep_query<K, NCH>;
template <int K, int NCH> constexpr void (*match_body)(const SepMatchArgs&, int) = sep_match<K, NCH>;

int chunks(int B) { return B <= 64 ? 1 : (B <= 128 ? 2 : 4); }

// L<K, NCH>::run(args...) for the runtime series length and bin chunks.
template <template <int, int> class L, class... Args>
hipError_t dispatch(int K, int nbins, Args&&... args) {
  const int nch = chunks(nbins);
#define SWIH_SEP_K(KV)                                         \
  case KV:                                                     \
    return nch == 1 ? L<KV, 1>::run(args...)                   \
                    : (nch == 2 ? L<KV, 2>::run(args...) : L<KV, 4>::run(args...));
  switch (K) {
    SWIH_SEP_K(1)
    SWIH_SEP_K(2)
    SWIH_SEP_K(3)
    SWIH_SEP_K(4)
    SWIH_SEP_K(5)
    SWIH_SEP_K(6)
    SWIH_SEP_K(7)
    SWIH_SEP_K(8)
    default: return hipErrorInvalidValue;
  }
#undef SWIH_SEP_K
}

template <int K, int NCH> struct RowsOne {
  static hipError_t run(const SepBuildArgs& a, int32_t nb, hipStream_t s) {
    return one<SepBuildArgs, rows_body<K, NCH>>(a, nb, s);
  }
};
template <int K, int NCH> struct QueryOne {
  static hipError_t run(const SepQueryArgs& a, int32_t nb, hipStream_t s) {
    return one<SepQueryArgs, query_body<K, NCH>>(a, nb, s);
  }
};
template <int K, int NCH> struct MatchOne {
  static hipError_t run(const SepMatchArgs& a, int32_t nb, hipStream_t s) {
    return one<SepMatchArgs, match_body<K, NCH>>(a, nb, s);
  }
};
template <int K, int NCH> struct RowsMany {
  static hipError_t run(const SepBuildArgs* u, const int32_t* p, int n, int32_t tot, int grid,
                        hipStream_t s) {
    return many<SepBuildArgs, rows_body<K, NCH>>(u, p, n, tot, grid, s);
  }
};
template <int K, int NCH> struct QueryMany {
  static hipError_t run(const SepQueryArgs* it, const int32_t* p, int n, int32_t tot, int grid,
                        hipStream_t s) {
    return many<SepQueryArgs, query_body<K, NCH>>(it, p, n, tot, grid, s);
  }
};
template <int K, int NCH> struct MatchMany {
  static hipError_t run(const SepMatchArgs* it, const int32_t* p, int n, int32_t tot, int grid,
                        hipStream_t s) {
    return many<SepMatchArgs, match_body<K, NCH>>(it, p, n, tot, grid, s);
  }
};

}  // namespace

// ---------------------------------------------------------------- host side
void sep_axis(const GaussAxis& ax, int32_t r, SepAxis& s) {
  memset(&s, 0, sizeof(s));
  s.a[0] = ax.a[0];
  s.g_in = ax.a[0];
  for (int k = 1; k <= ax.K; ++k) {
    const double tr = ax.om[k] * (double)r;
    const double t1 = ax.om[k];
    s.a[k] = ax.a[k];
    s.ec[k] = cos(tr);
    s.es[k] = sin(tr);
    s.rc[k] = cos(t1);
    s.rs[k] = sin(t1);
    s.g_in += ax.a[k] * s.ec[k];
  }
}

SepLayout sep_layout(int32_t H, int32_t W, int32_t B) {
  SepLayout L;
  L.off_hr = 0;
  L.set_bytes = swih_align256((int64_t)H * W * B * 4);
  return L;
}

SepGeom sep_geom(int32_t H, int32_t W, int32_t B, int32_t w, int32_t h, int32_t K) {
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
  g.K = K;
  // segment lengths: multiples of 32, at least the window less one, so a
  // segment's start-up walk costs no more than its output walk
  g.SX = 32 * (1 > (w + 30) / 32 ? 1 : (w + 30) / 32);
  g.SY = 32 * (1 > (h + 30) / 32 ? 1 : (h + 30) / 32);
  return g;
}

void sep_build_args(const SepGeom& g, const SepLayout& L, const GaussAxis& ax, const uint8_t* img,
                    int32_t img_pitch, char* set_base, SepBuildArgs& a, int32_t (&nb)[2]) {
  memset(&a, 0, sizeof(a));
  a.g = g;
  a.img = img;
  a.ipitch = img_pitch;
  a.hr = (float*)(set_base + L.off_hr);
  sep_axis(ax, g.rx, a.ax);
  nb[0] = 0;
  nb[1] = row_blocks(g);
}

void sep_query_args(const SepGeom& g, const SepLayout& L, const GaussAxis& ay, double mass,
                    const char* set_base, const int32_t* centres, int32_t n, float* hist,
                    SepQueryArgs& a, int32_t& nb) {
  memset(&a, 0, sizeof(a));
  a.g = g;
  a.hr = (const float*)(set_base + L.off_hr);
  sep_axis(ay, g.ry, a.ay);
  a.inv_mass = 1.0 / mass;
  a.centres = centres;
  a.n = n;
  a.hist = hist;
  nb = (n + WPB - 1) / WPB;
}

void sep_match_args(const SepGeom& g, const SepLayout& L, const GaussAxis& ay, double mass,
                    const char* set_base, const float* tmpl, int32_t x0, int32_t y0, int32_t x1,
                    int32_t y1, float* map, SepMatchArgs& a, int32_t& nb) {
  memset(&a, 0, sizeof(a));
  a.g = g;
  a.hr = (const float*)(set_base + L.off_hr);
  sep_axis(ay, g.ry, a.ay);
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
  if (phases & 2) return dispatch<RowsOne>(a.g.K, a.g.B, a, nb[1], s);
  return hipSuccess;
}

hipError_t sep_launch_query(const SepQueryArgs& a, int32_t nb, hipStream_t s) {
  return dispatch<QueryOne>(a.g.K, a.g.B, a, nb, s);
}

hipError_t sep_launch_match(const SepMatchArgs& a, int32_t nb, hipStream_t s) {
  return dispatch<MatchOne>(a.g.K, a.g.B, a, nb, s);
}

hipError_t sep_launch_build_batch(int nt, int nbins, const SepBuildArgs* units,
                                  const int32_t* prefix, int nunits, const int32_t (&total)[2],
                                  int grid, hipStream_t s) {
  return dispatch<RowsMany>((nt - 1) / 2, nbins, units, prefix + (nunits + 1), nunits, total[1],
                            grid, s);
}

hipError_t sep_launch_query_batch(int nt, int nbins, const SepQueryArgs* items,
                                  const int32_t* prefix, int n, int32_t total, int grid,
                                  hipStream_t s) {
  return dispatch<QueryMany>((nt - 1) / 2, nbins, items, prefix, n, total, grid, s);
}

hipError_t sep_launch_match_batch(int nt, int nbins, const SepMatchArgs* items,
                                  const int32_t* prefix, int n, int32_t total, int grid,
                                  hipStream_t s) {
  return dispatch<MatchMany>((nt - 1) / 2, nbins, items, prefix, n, total, grid, s);
}

}  // namespace swih
