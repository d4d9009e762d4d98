// Weighted integral histogram build for gfx950 (Sec. 2.1, Eq. 2).
//
// Per weight term p = (i, j) and bin b, the prefix sums
//   P[Y][X] = sum_{x < X, y < Y} [Q(f(x, y)) = b] u_i(x) v_j(y).
// Every u_i v_j product is a weight image w_dir of Eq. 2.  The integer kernels
// store one plane per term and apply the window-centre translation of
// Sec. 2.1 at query time; the Gaussian stores its terms already contracted
// with the translation coefficients of the windows each point is a corner of
// (swih_layout.h; the lookups in swih_query_bodies.h).
//
// The 2-D prefix is computed in three launches over a grid of 64-column tiles
// (one wave64 lane per pixel column) and TY-row bands:
//   1. aggregate: the band's column sums z_j(x) = sum_y v_j(y) m(x, y), the
//      row-segment sums T_i(y, tile) = sum_x u_i(x) m(x, y), and each plane's
//      tile total; integer kernels with few bins count every bin of a
//      (band, tile) at once in LDS histograms, the others take a wave per
//      (band, tile, bin).
//   2. scan: exclusive prefix of z over bands (the carry row above a band),
//      of T over tiles (the carry column left of a tile), and a 2-D exclusive
//      prefix of the tile totals (the value at each tile's origin corner).
//   3. emit: per (band, tile, bin) wave, rows top to bottom: a wave64 DPP
//      inclusive scan of u_i m gives the row prefix inside the tile, the carries
//      complete it, and v_j(y) times it accumulates into each plane's column
//      running sum, stored once per element with coalesced 256-byte rows.
// Integer kernels accumulate modulo 2^32.  The Gaussian runs its horizontal
// scans in int32 fixed point (exact), accumulates each tile's columns in
// double relative to the tile's own origin, contracts them and stores the
// result as float, and keeps the cross-tile row carries in double.
#pragma once

#include <string.h>

#include "swih_internal.h"
#include "wave64.h"

namespace swih {
namespace {

constexpr int WG = 256;
constexpr int WPB = WG / 64;  // waves per block

// Integer kernels' weight terms: plane p -> (i, j) with u/v in {1, t, t^2}.
template <int KIND> struct IntTerms;
template <> struct IntTerms<0> { static constexpr int nI = 1, nJ = 1, nP = 1; };
template <> struct IntTerms<1> { static constexpr int nI = 2, nJ = 2, nP = 3; };
template <> struct IntTerms<2> { static constexpr int nI = 3, nJ = 3, nP = 5; };
__host__ __device__ constexpr int plane_i(int p) { return p == 1 ? 1 : (p == 3 ? 2 : 0); }
__host__ __device__ constexpr int plane_j(int p) { return p == 2 ? 1 : (p == 4 ? 2 : 0); }
__device__ __forceinline__ uint32_t poly_term(int i, uint32_t t) {
  return i == 0 ? 1u : (i == 1 ? t : t * t);
}

// [Q(v) = b] for 8-bit v: Q(v) = floor(v B / 256) = b exactly when
// ceil(256 b / B) <= v < ceil(256 (b + 1) / B), one unsigned range test.
__device__ __forceinline__ bool in_bin(uint32_t v, int B, int b) {
  const uint32_t lo = (256u * (uint32_t)b + (uint32_t)B - 1) / (uint32_t)B;
  const uint32_t hi = (256u * (uint32_t)(b + 1) + (uint32_t)B - 1) / (uint32_t)B;
  return v - lo < hi - lo;
}

// Bit k = [pixel (x, y0 + k) falls in bin b] for the band's rows.  All the
// band's pixel loads of a lane are issued together (row index clamped, so no
// branch separates them) and masked afterwards.  Each load addresses the
// band's first row (wave-uniform) plus a 32-bit offset: the row's, uniform,
// and the lane's column.
__device__ __forceinline__ uint64_t band_mask(const uint8_t* __restrict__ img, int ipitch, int W,
                                              int x, int y0, int nrows, int B, int b) {
  const uint8_t* band = img + (size_t)y0 * ipitch;
  const uint32_t xo = (uint32_t)(x < W ? x : W - 1);
  uint32_t lo = 0, hi = 0;
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const int kk = k < nrows ? k : nrows - 1;
    lo |= (uint32_t)in_bin(band[(uint32_t)(kk * ipitch) + xo], B, b) << k;
  }
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const int kk = k + 32 < nrows ? k + 32 : nrows - 1;
    hi |= (uint32_t)in_bin(band[(uint32_t)(kk * ipitch) + xo], B, b) << k;
  }
  uint64_t m = ((uint64_t)hi << 32) | lo;
  if (nrows < 64) m &= ((uint64_t)1 << nrows) - 1;
  return x < W ? m : 0;
}

__device__ __forceinline__ uint32_t bit_of(uint64_t m, int k) { return (uint32_t)(m >> k) & 1u; }

struct WaveTile {
  int b, tx, ty, x, y0, nrows;
  bool valid;
};

__device__ __forceinline__ bool wave_tile(const SwihGeom& g, long wid, int extra, WaveTile& t,
                                          int& e) {
  const long nw = (long)g.NTY * g.NTX * g.B * extra;
  if (wid >= nw) return false;
  e = (int)(wid % extra);
  long r = wid / extra;
  t.b = (int)(r % g.B);
  r /= g.B;
  t.tx = (int)(r % g.NTX);
  t.ty = (int)(r / g.NTX);
  t.x = t.tx * SWIH_TX + lane_id();
  t.valid = t.x < g.W;
  t.y0 = t.ty * g.TY;
  t.nrows = min(g.TY, g.H - t.y0);
  return true;
}

// Wave-uniform by construction; readfirstlane tells the compiler so, which keeps
// every index derived from it (and the loads they address) scalar.  NW: waves
// per virtual block (the block's size over 64).
template <int NW = WPB>
__device__ __forceinline__ long wave_index(int vb) {
  return (long)vb * NW + (long)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// ---------------------------------------------------------------- integer kernels
// Sums over the set bits of a 64-bit mask of the bit index k and of k^2,
// from popcounts: k = sum_m 2^m k_m with k_m its bit m, so
//   sum k   = sum_m 2^m popc(mask & K_m),
//   sum k^2 = sum_{m,n} 2^(m+n) popc(mask & K_m & K_n),
// K_m the positions whose bit m is set.  Arithmetic modulo 2^32 like the planes.
__device__ __constant__ const uint64_t kBitOfIndex[6] = {
    0xAAAAAAAAAAAAAAAAull, 0xCCCCCCCCCCCCCCCCull, 0xF0F0F0F0F0F0F0F0ull,
    0xFF00FF00FF00FF00ull, 0xFFFF0000FFFF0000ull, 0xFFFFFFFF00000000ull};

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return (uint32_t)__popcll(m); }

__device__ __forceinline__ uint32_t index_sum(uint64_t m) {
  uint32_t s = 0;
#pragma unroll
  for (int b = 0; b < 6; ++b) s += popc64(m & kBitOfIndex[b]) << b;
  return s;
}

__device__ __forceinline__ uint32_t index_sq_sum(uint64_t m) {
  uint32_t s = 0;
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    const uint64_t mb = m & kBitOfIndex[b];
    s += popc64(mb) << (2 * b);
#pragma unroll
    for (int c = b + 1; c < 6; ++c) s += popc64(mb & kBitOfIndex[c]) << (b + c + 1);
  }
  return s;
}

// sum over set bits k of u_i(t0 + k) for the terms {1, t, t^2}
template <int NI>
__device__ __forceinline__ void term_sums(uint64_t m, uint32_t t0, uint32_t (&out)[NI]) {
  const uint32_t c = popc64(m);
  out[0] = c;
  if constexpr (NI > 1) {
    const uint32_t sk = index_sum(m);
    out[1] = t0 * c + sk;
    if constexpr (NI > 2) out[2] = t0 * t0 * c + 2u * t0 * sk + index_sq_sum(m);
  }
}

// ---- aggregate by LDS histograms: one 256-thread block per (band, tile)
// Every pixel of the tile adds one packed word to the LDS counter of its bin
// twice: once in its column's histogram (local index k = row in the band) and
// once in its row's (k = column in the tile).  The word is 1 + k 2^7 (+ k^2
// 2^18 for the Euclidean terms), so one atomic per pixel and pass gathers the
// count, the sum of k and the sum of k^2 of every bin; with at most 64 pixels
// per counter the fields stay below 2^7, 2^11 and 2^17.  The band's rows are
// loaded once for all bins (the per-bin form reloads them for every bin).
// LDS: the staged tile (64 rows of kHistRow bytes: 16-byte aligned rows whose
// 16-byte reads by 64 lanes spread over the banks), then the column and the
// row histograms, [bin][64] each.
constexpr int kHistRow = 80;
constexpr int kHistMaxLds = 48 << 10;

template <int KIND> struct HistWord { using T = uint32_t; };
template <> struct HistWord<2> { using T = uint64_t; };

__host__ __device__ constexpr int hist_lds_bytes(int kind, int B) {
  return 64 * kHistRow + 2 * B * 64 * (kind == 2 ? 8 : 4);
}

extern __shared__ __align__(16) unsigned char hist_lds[];

template <typename W>
__device__ __forceinline__ W hist_word(uint32_t k) {
  if constexpr (sizeof(W) == 8) return (W)1 + ((W)k << 7) + ((W)(k * k) << 18);
  else return 1u + (k << 7);
}

// [count, t0 count + sum k, t0^2 count + 2 t0 sum k + sum k^2] modulo 2^32:
// the sums of u(t0 + k) for u in {1, t, t^2} over the counted k.
template <int N, typename W>
__device__ __forceinline__ void hist_terms(W w, uint32_t t0, uint32_t (&out)[N]) {
  const uint32_t c = (uint32_t)w & 127u;
  out[0] = c;
  if constexpr (N > 1) {
    const uint32_t sk = (uint32_t)(w >> 7) & 2047u;
    out[1] = t0 * c + sk;
    if constexpr (N > 2) out[2] = t0 * t0 * c + 2u * t0 * sk + (uint32_t)(w >> 18);
  }
}

template <typename W>
__device__ __forceinline__ void lds_add(W* p, W v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int KIND>
__device__ __forceinline__ void aggregate_int_hist(const BuildArgs& a, int vb) {
  const SwihGeom& g = a.g;
  using TT = IntTerms<KIND>;
  using W = typename HistWord<KIND>::T;
  const int B = g.B;
  const int ty = vb / g.NTX, tx = vb - ty * g.NTX;
  const int y0 = ty * g.TY, nrows = min(g.TY, g.H - y0);
  const int w = (int)(threadIdx.x >> 6), lane = lane_id();
  const int x = tx * SWIH_TX + lane;
  unsigned char* tile = hist_lds;
  W* colh = (W*)(hist_lds + 64 * kHistRow);
  W* rowh = colh + B * 64;
  // wave w loads rows 16 w .. 16 w + 15 of the band (clamped into the image),
  // each at the band's first row plus a 32-bit offset
  const uint8_t* band = a.img + (size_t)y0 * a.ipitch;
  const uint32_t xo = (uint32_t)(x < g.W ? x : g.W - 1);
  uint32_t v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int k = 16 * w + i;
    v[i] = band[(uint32_t)((k < nrows ? k : nrows - 1) * a.ipitch) + xo];
  }
  __syncthreads();  // an earlier virtual block of this block is done with the counters
  {
    uint4* c4 = (uint4*)colh;
    const int n4 = 2 * B * 64 * (int)sizeof(W) / 16;
    for (int i = (int)threadIdx.x; i < n4; i += WG) c4[i] = make_uint4(0u, 0u, 0u, 0u);
  }
  __syncthreads();
  // columns: lane x counts its rows of this wave's quarter of the band
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int k = 16 * w + i;
    tile[k * kHistRow + lane] = (unsigned char)v[i];
    if (k < nrows && x < g.W) lds_add(&colh[((v[i] * (uint32_t)B) >> 8) * 64 + lane], hist_word<W>((uint32_t)k));
  }
  __syncthreads();
  // rows: lane = row of the band, wave w counts tile columns 16 w .. 16 w + 15
  {
    const uint4 r4 = *(const uint4*)(tile + lane * kHistRow + 16 * w);
    const uint32_t rw[4] = {r4.x, r4.y, r4.z, r4.w};
    const int nx = min(16, g.W - (tx * SWIH_TX + 16 * w));
    if (lane < nrows) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const uint32_t pv = (rw[j >> 2] >> (8 * (j & 3))) & 255u;
        if (j < nx) lds_add(&rowh[((pv * (uint32_t)B) >> 8) * 64 + lane], hist_word<W>((uint32_t)(16 * w + j)));
      }
    }
  }
  __syncthreads();
  uint32_t* __restrict__ z = (uint32_t*)a.z;
  uint32_t* __restrict__ T = (uint32_t*)a.T;
  uint32_t* __restrict__ BT = (uint32_t*)a.BT;
  const int NXP = g.NTX * SWIH_TX;
  const uint32_t yl = (uint32_t)(y0 + lane);
  for (int b = w; b < B; b += WPB) {
    uint32_t zacc[TT::nJ], treg[TT::nI];
    hist_terms<TT::nJ>(colh[b * 64 + lane], (uint32_t)y0, zacc);
    hist_terms<TT::nI>(rowh[b * 64 + lane], (uint32_t)(tx * SWIH_TX), treg);
#pragma unroll
    for (int j = 0; j < TT::nJ; ++j) z[((size_t)(j * B + b) * g.NTY + ty) * NXP + x] = zacc[j];
    if (lane < nrows) {
#pragma unroll
      for (int i = 0; i < TT::nI; ++i) T[((size_t)(i * B + b) * g.NTX + tx) * g.H + y0 + lane] = treg[i];
    }
#pragma unroll
    for (int p = 0; p < TT::nP; ++p) {
      const uint32_t val = lane < nrows ? poly_term(plane_j(p), yl) * treg[plane_i(p)] : 0u;
      const uint32_t s = wave_sum(val);
      if (lane == 0) BT[((size_t)(p * B + b) * g.NTY + ty) * g.NTX + tx] = s;
    }
  }
}

__host__ __device__ constexpr bool int_hist(int kind, int B) {
  return hist_lds_bytes(kind, B) <= kHistMaxLds;
}

template <int KIND>
__device__ __forceinline__ void aggregate_int(const BuildArgs& a, int vb) {
  if (a.agg_hist) {
    aggregate_int_hist<KIND>(a, vb);
    return;
  }
  const SwihGeom& g = a.g;
  const uint8_t* __restrict__ img = a.img;
  const int ipitch = a.ipitch;
  uint32_t* __restrict__ z = (uint32_t*)a.z;
  uint32_t* __restrict__ T = (uint32_t*)a.T;
  uint32_t* __restrict__ BT = (uint32_t*)a.BT;
  using TT = IntTerms<KIND>;
  WaveTile t;
  int e;
  if (!wave_tile(g, wave_index(vb), 1, t, e)) return;
  const int lane = lane_id();
  const int NXP = g.NTX * SWIH_TX;
  const uint64_t mask = band_mask(img, ipitch, g.W, t.x, t.y0, t.nrows, g.B, t.b);
  // column sums of this lane's column over the band's rows: v_j(y0 + k) over set bits k
  uint32_t zacc[TT::nJ];
  term_sums<TT::nJ>(mask, (uint32_t)t.y0, zacc);
  // row sums: after the transpose lane k holds row y0 + k over the tile's 64 columns
  uint32_t treg[TT::nI];
  term_sums<TT::nI>(wave_transpose64(mask), (uint32_t)(t.tx * SWIH_TX), treg);
#pragma unroll
  for (int j = 0; j < TT::nJ; ++j)
    z[((size_t)(j * g.B + t.b) * g.NTY + t.ty) * NXP + t.x] = zacc[j];
  if (lane < t.nrows) {
#pragma unroll
    for (int i = 0; i < TT::nI; ++i)
      T[((size_t)(i * g.B + t.b) * g.NTX + t.tx) * g.H + t.y0 + lane] = treg[i];
  }
  const uint32_t yl = (uint32_t)(t.y0 + lane);
#pragma unroll
  for (int p = 0; p < TT::nP; ++p) {
    const uint32_t val = lane < t.nrows ? poly_term(plane_j(p), yl) * treg[plane_i(p)] : 0u;
    const uint32_t s = wave_sum(val);
    if (lane == 0) BT[((size_t)(p * g.B + t.b) * g.NTY + t.ty) * g.NTX + t.tx] = s;
  }
}

// Exclusive prefixes of the aggregates, three roles in one launch:
//   blocks [0, nb1)          thread per column: carry row above each band
//                            (exclusive prefix of z over bands; integer kernels)
//   blocks [nb1, nb1 + nb2)  thread per row: carry left of each tile
//                            (exclusive prefix of T over tiles)
//   remaining blocks         wave per (plane, bin): value at each tile origin,
//                            the 2-D exclusive prefix of the tile totals.
// Each serial walk loads its next 8 values before storing, so the loads of a
// thread overlap.
template <typename V>
__device__ __forceinline__ void excl_walk(V* p, long stride, int n) {
  V run = 0;
  int k = 0;
  for (; k + 8 <= n; k += 8) {
    V v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(k + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      p[(k + u) * stride] = run;
      run += v[u];
    }
  }
  for (; k < n; ++k) {
    const V v = p[k * stride];
    p[k * stride] = run;
    run += v;
  }
}

template <typename ZT, typename TTy, typename BTy, int WGT = WG>
__device__ __forceinline__ void scan_carries(const BuildArgs& a, int vb) {
  const SwihGeom& g = a.g;
  ZT* __restrict__ z = (ZT*)a.z;
  TTy* __restrict__ T = (TTy*)a.T;
  BTy* __restrict__ BT = (BTy*)a.BT;
  // the roles are laid out in 256-thread blocks (nb1, nb2); a virtual block of
  // WGT threads covers WGT / 256 of them, so every thread finds its own role
  // (the boundaries are whole waves)
  const long t = (long)vb * WGT + threadIdx.x;
  const long r1 = (long)a.nb1 * WG, r2 = r1 + (long)a.nb2 * WG;
  __shared__ BTy rowcarry[WGT / 64][128];
  const int NXP = g.NTX * SWIH_TX;
  if (t < r1) {
    if (t >= (long)g.nJ * g.B * NXP) return;
    const long col = t % NXP, jb = t / NXP;
    excl_walk(z + (size_t)jb * g.NTY * NXP + col, NXP, g.NTY);
    return;
  }
  if (t < r2) {
    const long tt = t - r1;
    if (tt >= (long)g.nI * g.B * g.H) return;
    const long y = tt % g.H, ib = tt / g.H;
    excl_walk(T + (size_t)ib * g.NTX * g.H + y, g.H, g.NTX);
    return;
  }
  const int w = (int)(threadIdx.x >> 6);
  const long pbi = (long)__builtin_amdgcn_readfirstlane((int)((t - r2) >> 6));
  if (pbi >= (long)g.nP * g.B) return;
  BTy* base = BT + (size_t)pbi * g.NTY * g.NTX;
  const int lane = lane_id();
  for (int ty = lane; ty < g.NTY; ty += 64) rowcarry[w][ty] = 0;
  for (int c0 = 0; c0 < g.NTX; c0 += 64) {
    const int tx = c0 + lane;
    const bool ok = tx < g.NTX;
    BTy run = 0;
    // eight bands' totals are loaded before any of them is replaced, so each
    // group of eight costs one memory round trip
    for (int ty0 = 0; ty0 < g.NTY; ty0 += 8) {
      BTy v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        v[u] = ok && ty0 + u < g.NTY ? base[(size_t)(ty0 + u) * g.NTX + tx] : (BTy)0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int ty = ty0 + u;
        if (ty >= g.NTY) break;
        const BTy inc = wave_incl_scan(run);
        const BTy carry = rowcarry[w][ty];
        if (ok) base[(size_t)ty * g.NTX + tx] = carry + inc - run;
        rowcarry[w][ty] = carry + readlane(inc, 63);
        run += v[u];
      }
    }
  }
}

// NTS: non-temporal plane stores (plane sets from the last-level cache's size on).
template <int KIND, bool NTS = false>
__device__ __forceinline__ void emit_int(const BuildArgs& a, int vb) {
  const SwihGeom& g = a.g;
  const uint8_t* __restrict__ img = a.img;
  const int ipitch = a.ipitch;
  uint32_t* __restrict__ planes = (uint32_t*)a.planes;
  const uint32_t* __restrict__ zc = (const uint32_t*)a.z;
  const uint32_t* __restrict__ E = (const uint32_t*)a.T;
  const uint32_t* __restrict__ CTc = (const uint32_t*)a.BT;
  using TT = IntTerms<KIND>;
  WaveTile t;
  int e;
  if (!wave_tile(g, wave_index(vb), 1, t, e)) return;
  const int lane = lane_id();
  const int NXP = g.NTX * SWIH_TX;
  uint32_t u[TT::nI], ereg[TT::nI], acc[TT::nP];
  size_t pbase[TT::nP];
#pragma unroll
  for (int i = 0; i < TT::nI; ++i) {
    u[i] = poly_term(i, (uint32_t)t.x);
    ereg[i] = lane < t.nrows ? E[((size_t)(i * g.B + t.b) * g.NTX + t.tx) * g.H + t.y0 + lane]
                             : 0u;
  }
  // carry row: P[y0][x + 1] = tile-origin value + prefix of u_i * (column sums above)
#pragma unroll
  for (int p = 0; p < TT::nP; ++p) {
    const uint32_t zv = zc[((size_t)(plane_j(p) * g.B + t.b) * g.NTY + t.ty) * NXP + t.x];
    acc[p] = CTc[((size_t)(p * g.B + t.b) * g.NTY + t.ty) * g.NTX + t.tx] +
             wave_incl_scan(u[plane_i(p)] * zv);
    // lanes past the image's last column write too (their values are never
    // read), so every store is a whole 256-byte run
    pbase[p] = (size_t)(swih_base(g, p, t.b) + t.tx * g.tile_stride + lane);
  }
  if (t.ty == 0) {
#pragma unroll
    for (int p = 0; p < TT::nP; ++p) planes[pbase[p]] = 0u;
  }
  const uint64_t mask = band_mask(img, ipitch, g.W, t.x, t.y0, t.nrows, g.B, t.b);
  for (int k = 0; k < t.nrows; ++k) {
    const uint32_t y = (uint32_t)(t.y0 + k);
    const uint32_t m = bit_of(mask, k);
    uint32_t s[TT::nI];
#pragma unroll
    for (int i = 0; i < TT::nI; ++i) s[i] = wave_incl_scan(m * u[i]) + readlane(ereg[i], k);
#pragma unroll
    for (int p = 0; p < TT::nP; ++p) acc[p] += poly_term(plane_j(p), y) * s[plane_i(p)];
    const size_t row = (size_t)(y + 1) * g.row_stride;
#pragma unroll
    for (int p = 0; p < TT::nP; ++p) {
      if constexpr (NTS)
        __builtin_nontemporal_store(acc[p], planes + pbase[p] + row);
      else
        planes[pbase[p] + row] = acc[p];
    }
  }
}

// ---------------------------------------------------------------- Gaussian
// Fixed-point weight terms: uq[x][i] (x < NTX*64, zero beyond W), vq[y][j],
// and vqd[y][j] = vq * 2^-48 as double (scales the u*v product to real units);
// the y translation coefficients of each row Y as a window's bottom edge
// (centre row Y - ry - 1) and as its top edge (centre row Y + ry):
// beta[Y][j] and beta[Y][NT + j].
template <int WGT = WG>
__device__ __forceinline__ void basis(const BuildArgs& a, int vb) {
  const SwihGeom& g = a.g;
  const GaussAxis& ax = a.ax;
  const GaussAxis& ay = a.ay;
  int32_t* __restrict__ uq = a.uq;
  int32_t* __restrict__ vq = a.vq;
  double* __restrict__ vqd = a.vqd;
  const long t = (long)vb * WGT + threadIdx.x;
  const int NXP = g.NTX * SWIH_TX;
  const long nu = (long)g.nI * NXP, nv = (long)g.nJ * g.H, nb = 2L * g.nJ * (g.H + 1);
  const double fix = (double)(1 << SWIH_FIX_BITS);
  if (t < nu) {
    const int i = (int)(t / NXP), x = (int)(t % NXP);
    double val = 0.0;
    if (x < g.W) {
      if (i == 0) {
        val = 1.0;
      } else {
        const double ang = ax.om[(i + 1) / 2] * (double)x;
        val = (i & 1) ? cos(ang) : sin(ang);
      }
    }
    uq[(size_t)x * g.nI + i] = (int32_t)rint(val * fix);
  } else if (t < nu + nv) {
    const long r = t - nu;
    const int y = (int)(r / g.nJ), j = (int)(r % g.nJ);
    double val;
    if (j == 0) {
      val = 1.0;
    } else {
      const double ang = ay.om[(j + 1) / 2] * (double)y;
      val = (j & 1) ? cos(ang) : sin(ang);
    }
    const int32_t q = (int32_t)rint(val * fix);
    vq[(size_t)y * g.nJ + j] = q;
    vqd[(size_t)y * g.nJ + j] = ldexp((double)q, -2 * SWIH_FIX_BITS);
  } else if (t < nu + nv + nb) {
    const long r = t - nu - nv;
    const int Y = (int)(r / (2 * g.nJ)), q = (int)(r % (2 * g.nJ));
    // rows that are never a bottom edge (Y <= ry) take centre 0: their values are never read
    a.beta[r] = q < g.nJ ? series_coeff(ay, max(Y - a.ry - 1, 0), q)
                         : series_coeff(ay, Y + a.ry, q - g.nJ);
  } else if (t < nu + nv + nb + a.nacc) {
    a.acc[t - nu - nv - nb] = 0;  // the map accumulator starts at zero
  }
}

template <int NT, int WGT = WG>
__device__ __forceinline__ void aggregate_gauss(const BuildArgs& a, int vb) {
  const SwihGeom& g = a.g;
  const uint8_t* __restrict__ img = a.img;
  const int ipitch = a.ipitch;
  const int32_t* __restrict__ uq = a.uq;
  const int32_t* __restrict__ vq = a.vq;
  int64_t* __restrict__ T = (int64_t*)a.T;
  double* __restrict__ BT = (double*)a.BT;
  // per wave: the band's row sums T_i(y) and row terms v_j(y), [row][term]
  __shared__ int32_t lds[WGT / 64][2][64 * NT];
  WaveTile t;
  int e;
  if (!wave_tile(g, wave_index<WGT / 64>(vb), 1, t, e)) return;
  const int lane = lane_id();
  int32_t* sT = lds[threadIdx.x >> 6][0];
  int32_t* sV = lds[threadIdx.x >> 6][1];
  const uint64_t mask = band_mask(img, ipitch, g.W, t.x, t.y0, t.nrows, g.B, t.b);
  // row sums: after the transpose lane k holds row y0 + k over the tile's 64
  // columns; T_i(y) = sum over its set bits x of u_i(x), the column's terms
  // uniform over the wave (scalar loads), added under an all-ones/zero mask
  const uint64_t rowm = wave_transpose64(mask);
  const uint32_t rlo = (uint32_t)rowm, rhi = (uint32_t)(rowm >> 32);
  const int32_t* ucol = uq + (size_t)t.tx * SWIH_TX * NT;
  int32_t treg[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) treg[i] = 0;
#pragma unroll 4
  for (int l = 0; l < 64; ++l) {
    const uint32_t half = l < 32 ? rlo : rhi;
    const int32_t sel = -(int32_t)((half >> (l & 31)) & 1u);
    const int32_t* ul = ucol + l * NT;
#pragma unroll
    for (int i = 0; i < NT; ++i) treg[i] += ul[i] & sel;
  }
  const bool row = lane < t.nrows;
  const int yl = t.y0 + (row ? lane : 0);
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    if (row) T[((size_t)(i * g.B + t.b) * g.NTX + t.tx) * g.H + t.y0 + lane] = (int64_t)treg[i];
    sT[lane * NT + i] = row ? treg[i] : 0;
  }
#pragma unroll
  for (int j = 0; j < NT; ++j) sV[lane * NT + j] = vq[(size_t)yl * NT + j];
  // the wave's own LDS writes, read back by other lanes
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // tile totals of every plane, one lane per plane p = i NT + j: the sum over
  // the band's rows of v_j(y) T_i(y), exact in int64 (rows past the band's
  // last one hold T_i = 0)
  constexpr int NP = NT * NT;
  for (int p0 = 0; p0 < NP; p0 += 64) {
    const int p = p0 + lane;
    if (p >= NP) break;
    const int i = p / NT, j = p - (p / NT) * NT;
    int64_t acc = 0;
#pragma unroll 8
    for (int y = 0; y < 64; ++y) acc += (int64_t)sT[y * NT + i] * (int64_t)sV[y * NT + j];
    BT[((size_t)(p * g.B + t.b) * g.NTY + t.ty) * g.NTX + t.tx] = (double)acc;
  }
}

// Row carries at the tile origin column, RC_ij[Y] = P_ij[Y][64 tx], of one
// (band, tile, bin), contracted in y like the planes.  Lane k takes row
// Y = y0 + k + 1 of the band: every (i, j) is an inclusive wave scan of the
// row increments,
//   RC_ij[y + 1] = RC_ij[y] + v_j(y) E_i(y),   RC_ij[y0] = CT_ij
// (CT the tile-origin value, E_i the row carry of x term i, both in the
// fixed-point units of the basis), and the lane stores
//   RCB_i = sum_j beta_j(Y - ry - 1) RC_ij[Y],  RCT_i = sum_j beta_j(Y + ry) RC_ij[Y]
// and the count RC_00[Y]: one run of 2 NT + 1 doubles per row (swih_rc).  The
// count is exact: its increments are integers times 2^48.
// NTS: non-temporal stores (large plane sets, as the planes).
template <int NT, int WGT, bool NTS>
__device__ __forceinline__ void rc_gauss(const BuildArgs& a, const WaveTile& t) {
  const SwihGeom& g = a.g;
  const int64_t* __restrict__ E = (const int64_t*)a.T;
  const double* __restrict__ CTc = (const double*)a.BT;
  double* __restrict__ RCp = a.RC;
  const double sc48 = ldexp(1.0, -2 * SWIH_FIX_BITS);
  const int lane = lane_id();
  const bool row = lane < t.nrows;
  const int y = t.y0 + (row ? lane : 0);
  if (t.ty == 0 && lane < g.nRC) RCp[swih_rc(g, lane, t.b, t.tx, 0)] = 0.0;
  double vj[NT], bB[NT], bT[NT];
  const int32_t* __restrict__ vr = a.vq + (size_t)y * NT;
  const double* __restrict__ br = a.beta + (size_t)(y + 1) * 2 * NT;
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    vj[j] = row ? (double)vr[j] : 0.0;
    bB[j] = br[j];
    bT[j] = br[NT + j];
  }
  const size_t ctp = (size_t)g.B * g.NTY * g.NTX;  // from one term's tile values to the next
  const double* __restrict__ ct = CTc + ((size_t)t.b * g.NTY + t.ty) * g.NTX + t.tx;
  // the tile-origin values, one term per lane (vector loads: the plane waves'
  // row tables keep the scalar cache)
  constexpr int NCT = (NT * NT + 63) / 64;
  double ctv[NCT];
#pragma unroll
  for (int c = 0; c < NCT; ++c) {
    const int q = c * 64 + lane;
    ctv[c] = q < NT * NT ? ct[(size_t)q * ctp] : 0.0;
  }
  // the band's rows are one contiguous run of 64 nRC doubles in the carry array:
  // staged in LDS ([row][q], the array's order) so that every store writes 512
  // consecutive bytes.  The row-carry waves are the odd waves of a block.
  constexpr int NRC = 2 * NT + 1;
  __shared__ double stage[WGT / 128][64 * NRC];
  double* __restrict__ st = stage[threadIdx.x >> 7] + lane * NRC;
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    const double ei = row ? (double)E[((size_t)(i * g.B + t.b) * g.NTX + t.tx) * g.H + y] : 0.0;
    double sB = 0.0, sT = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int q = i * NT + j;
      const double r = (readlane(ctv[q >> 6], q & 63) + wave_incl_scan(vj[j] * ei)) * sc48;
      sB = fma(bB[j], r, sB);
      sT = fma(bT[j], r, sT);
      if (i == 0 && j == 0) st[2 * NT] = r;
    }
    st[i] = sB;
    st[NT + i] = sT;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const double* __restrict__ sw = stage[threadIdx.x >> 7];
  double* __restrict__ dst = RCp + swih_rc(g, 0, t.b, t.tx, t.y0 + 1);
  const int n = t.nrows * NRC;
  for (int k = lane; k < n; k += 64) {
    if constexpr (NTS)
      __builtin_nontemporal_store(sw[k], dst + k);
    else
      dst[k] = sw[k];
  }
}

// Planes of one (band, tile, bin), rows top to bottom.  The tile-local sums
//   L_ij[y + 1] = L_ij[y] + v_j(y) R_i(y)
// (R_i the row prefix of u_i [Q = b] inside the tile, an exact int32 DPP scan)
// are contracted over the x terms as they grow, with the coefficients the
// lane's column X needs as a right and as a left window edge:
//   V+_j[y + 1] = V+_j[y] + v_j(y) S+(y),  S+(y) = sum_i alpha_i(X - rx - 1) R_i(y)
//   V-_j[y + 1] = V-_j[y] + v_j(y) S-(y),  S-(y) = sum_i alpha_i(X + rx) R_i(y)
//   N[y + 1]    = N[y] + (pixels of the bin in the row up to X),
// and each stored row Y contracts V+ and V- over j with the coefficients of
// Y as a bottom and as a top edge (the table beta): the four corner values
// and N, 5 floats per column where the terms would take NT^2.  A band's
// closing row, which windows cross with any centre row, also keeps V+ and V-
// (side array XC).  The launch interleaves one row-carry wave (rc_gauss)
// after each plane wave.  NTS: non-temporal stores of the planes, the row
// carries and the band-closing rows (plane sets from the last-level cache's
// size on).
template <int NT, int WGT = WG, bool NTS = false>
__device__ __forceinline__ void emit_gauss(const BuildArgs& a, int vb) {
  const SwihGeom& g = a.g;
  const uint8_t* __restrict__ img = a.img;
  const int ipitch = a.ipitch;
  const int32_t* __restrict__ uq = a.uq;
  const double* __restrict__ vqd = a.vqd;
  const double* __restrict__ bet = a.beta;
  float* __restrict__ Lp = (float*)a.planes;
  WaveTile t;
  int e;
  if (!wave_tile(g, wave_index<WGT / 64>(vb), 2, t, e)) return;
  if (e == 1) {
    rc_gauss<NT, WGT, NTS>(a, t);
    return;
  }
  const int lane = lane_id();
  const int X = t.x + 1;  // this lane's plane column
  int32_t uqi[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) uqi[i] = uq[(size_t)t.x * NT + i];
  double ap[NT], am[NT];
  series_coeffs<NT>(a.ax, max(X - a.rx - 1, 0), ap);
  series_coeffs<NT>(a.ax, X + a.rx, am);
  // a row's 5 planes are consecutive 64-element runs: C_RB, C_RT, C_LB, C_LT, N
  float* col = Lp + swih_base(g, 0, t.b) + t.tx * g.tile_stride + lane;
  // running sums in FP64, each rounded once to float when stored
  double vp[NT], vm[NT];
  int32_t cnt = 0;
#pragma unroll
  for (int j = 0; j < NT; ++j) vp[j] = vm[j] = 0.0;
  if (t.ty == 0) {
#pragma unroll
    for (int p = 0; p < 5; ++p) col[p * 64] = 0.0f;
  }
  const uint64_t mask = band_mask(img, ipitch, g.W, t.x, t.y0, t.nrows, g.B, t.b);
  // the row's y terms and beta rows are loaded one row ahead (scalar loads issued
  // as the previous row's values die, so they arrive during the row's scans)
  double vr[NT], bb[NT], bt[NT];
  auto row_terms = [&](int y) {
    const double* vrow = vqd + (size_t)y * NT;
    const double* brow = bet + (size_t)(y + 1) * 2 * NT;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      vr[j] = vrow[j];
      bb[j] = brow[j];
      bt[j] = brow[NT + j];
    }
  };
  row_terms(t.y0);
  for (int k = 0; k < t.nrows; ++k) {
    const int y = t.y0 + k;
    const bool m = bit_of(mask, k) != 0;
    double sp = 0.0, sm = 0.0;
    int32_t r0 = 0;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const int32_t R = wave_incl_scan(m ? uqi[i] : 0);
      if (i == 0) r0 = R;
      sp = fma(ap[i], (double)R, sp);
      sm = fma(am[i], (double)R, sm);
    }
    // u_0 = 1 is 2^24 in fixed point: the row's count up to X, exactly
    cnt += r0 >> SWIH_FIX_BITS;
    double rb = 0.0, rt = 0.0, lb = 0.0, lt = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      vp[j] = fma(vr[j], sp, vp[j]);
      vm[j] = fma(vr[j], sm, vm[j]);
      rb = fma(bb[j], vp[j], rb);
      rt = fma(bt[j], vp[j], rt);
      lb = fma(bb[j], vm[j], lb);
      lt = fma(bt[j], vm[j], lt);
    }
    row_terms(min(y + 1, g.H - 1));  // the last row reloads a row in range
    // whole 256-byte runs: lanes past the last column write values never read
    float* dst = col + (size_t)(y + 1) * g.row_stride;
    if constexpr (NTS) {
      __builtin_nontemporal_store((float)rb, dst);
      __builtin_nontemporal_store((float)rt, dst + 64);
      __builtin_nontemporal_store((float)lb, dst + 128);
      __builtin_nontemporal_store((float)lt, dst + 192);
      __builtin_nontemporal_store((float)cnt, dst + 256);
    } else {
      dst[0] = (float)rb;
      dst[64] = (float)rt;
      dst[128] = (float)lb;
      dst[192] = (float)lt;
      dst[256] = (float)cnt;
    }
  }
  const int Yl = t.y0 + t.nrows;  // the band's last stored row
  if ((Yl & (g.TY - 1)) == 0 && Yl < g.H) {
    float* xc = a.XC + swih_xc(g, 0, t.b, Yl, X);
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      if constexpr (NTS) {
        __builtin_nontemporal_store((float)vp[j], xc + j * 64);
        __builtin_nontemporal_store((float)vm[j], xc + (NT + j) * 64);
      } else {
        xc[j * 64] = (float)vp[j];
        xc[(NT + j) * 64] = (float)vm[j];
      }
    }
  }
}

inline int blocks_for_waves(long waves) { return (int)((waves + WPB - 1) / WPB); }
inline int blocks_for_threads(long n) { return (int)((n + WG - 1) / WG); }

// Every stage is a device body over (arguments, virtual block).
using Body = void (*)(const BuildArgs&, int);

template <int KIND> struct IntStages {
  static int agg_lds(int B) { return int_hist(KIND, B) ? hist_lds_bytes(KIND, B) : 0; }
  static constexpr Body basis = nullptr;
  static constexpr Body agg = aggregate_int<KIND>;
  static constexpr Body scan = scan_carries<uint32_t, uint32_t, uint32_t>;
  static constexpr Body emit = emit_int<KIND>;
  static constexpr Body emit_nt = emit_int<KIND, true>;
  static constexpr Body emit_batch = emit_int<KIND, true>;
};
template <int NT> struct GaussStages {
  static int agg_lds(int) { return 0; }
  static constexpr Body basis = ::swih::basis<>;
  static constexpr Body agg = aggregate_gauss<NT>;
  static constexpr Body scan = scan_carries<int64_t, int64_t, double>;
  static constexpr Body emit = emit_gauss<NT>;
  static constexpr Body emit_nt = emit_gauss<NT, WG, true>;
  static constexpr Body emit_batch = emit_gauss<NT, WG, true>;
};

// The Gaussian stages with virtual blocks of WGT threads (a multiple of 256):
// the same work as WGT / 256 consecutive 256-thread virtual blocks.
template <int NT, int WGT> struct GaussStagesW {
  static constexpr Body basis = ::swih::basis<WGT>;
  static constexpr Body agg = aggregate_gauss<NT, WGT>;
  static constexpr Body scan = scan_carries<int64_t, int64_t, double, WGT>;
  static constexpr Body emit = emit_gauss<NT, WGT>;
};

}  // namespace
}  // namespace swih
