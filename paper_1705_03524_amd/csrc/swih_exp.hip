// Exponential (Laplacian) spatial kernel, k(dx, dy) = exp(-|dx| / tx - |dy| / ty)
// (kernel SWIH_EXPONENTIAL).
//
// Over each of the four disjoint quadrants of a window (Sec. 2.1) the weight
// is a product of two exponentials that grow toward the window centre, so a
// quadrant is one box of an integral histogram weighted by exp(+x/tx)exp(+y/ty)
// in that quadrant's direction, translated to the centre by a constant factor:
// the four direction-weighted integral histograms of Sec. 2.1, one per
// quadrant.  Direction d = (mx, my) = (d & 1, d >> 1) is built in mirrored
// coordinates x' = mx ? W - 1 - x : x, y' = my ? H - 1 - y : y, in which every
// direction is "weights growing toward +x', +y'".
//
// A prefix of exp(x / t) leaves every float format within a few hundred
// pixels, so each plane holds the prefix rescaled to its own corner,
//   E(X, Y) = sum_{x < X, y < Y} [Q(f) = b] qx^(X - x) qy^(Y - y),   q = exp(-1 / t),
// a sum of positive terms bounded by 1 / ((1 - qx)(1 - qy)) at any image size.
// The window box of a quadrant with mirrored centre (cx, cy) is
//   sum_corners +- qx^(cx - X) qy^(cy - Y) E(X, Y),
// where the factors are exp(1/t) (near corner of the centre's own quadrant),
// 1 (near corner of the opposite one) or exp(-r/t) (far corner).  E obeys
//   E(X, Y + 1) = qy (E(X, Y) + R(X, Y)),   R(X, y) = sum_{x < X} [Q = b] qx^(X - x),
// which the build runs down each 64-column tile of a 64-row band in double
// (the in-row prefix R inside the tile in float, the carried value E in
// double), with three carries made exactly like the integer kernels' (aggregate, scan,
// emit): the band-top column values, the row values at the tile's left edge
// and the tile-origin values E(64 tx, TY ty), each a chain with the decay of
// one tile or band.  The planes are stored as float (relative error 2^-24).
#include <math.h>
#include <string.h>

#include "swih_internal.h"
#include "wave64.h"

namespace swih {
namespace {

constexpr int WG = 256;
constexpr int WPB = WG / 64;

__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ long exp_wave(int vb) {
  return (long)vb * WPB + (long)rfl((int)(threadIdx.x >> 6));
}

// Leaky inclusive scan over the 64 lanes, s_l = sum_{k <= l} g^(l - k) v_k,
// with g = exp(-step): the DPP steps of wave_incl_scan, each source scaled by
// g to the power of the lane distance it spans (uniform for the row_shr
// steps, per lane for the two broadcasts).  Every DPP move writes all lanes
// with bound_ctrl (a lane without a source reads 0), so no destination needs
// clearing first; the broadcasts' factor is 0 on the rows they must not
// change, whatever those rows read.
template <typename T>
struct LeakyT {
  T g1, g2, g4, g8;
  T f15;  // rows 1 and 3: g^((l & 15) + 1), the distance from lane 15 (47); else 0
  T f31;  // rows 2 and 3: g^(l - 31); else 0
};
using Leaky = LeakyT<double>;

// q^n for 0 <= n < 128 (n per lane, q uniform): squarings of q and a product
// over the bits of n, relative error a few ulps.
__device__ __forceinline__ double dpow(double q, int n) {
  double r = 1.0, p = q;
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    r *= (n >> k) & 1 ? p : 1.0;
    p *= p;
  }
  return r;
}

// The scan's factors for a decay g per lane step.
__device__ __forceinline__ Leaky make_leaky(double g) {
  const int l = lane_id();
  Leaky L;
  L.g1 = g;
  L.g2 = g * g;
  L.g4 = L.g2 * L.g2;
  L.g8 = L.g4 * L.g4;
  L.f15 = (l & 16) ? dpow(g, (l & 15) + 1) : 0.0;
  L.f31 = l >= 32 ? dpow(g, l - 31) : 0.0;
  return L;
}

template <int CTRL>
__device__ __forceinline__ double dpp_all(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double leaky_scan(double v, const Leaky& L) {
  v = fma(L.g1, dpp_all<0x111>(v), v);   // row_shr:1
  v = fma(L.g2, dpp_all<0x112>(v), v);   // row_shr:2
  v = fma(L.g4, dpp_all<0x114>(v), v);   // row_shr:4
  v = fma(L.g8, dpp_all<0x118>(v), v);   // row_shr:8
  v = fma(L.f15, dpp_all<0x142>(v), v);  // row_bcast:15 (used by rows 1 and 3)
  v = fma(L.f31, dpp_all<0x143>(v), v);  // row_bcast:31 (used by rows 2 and 3)
  return v;
}

// The same scan in FP32, for sums inside one tile row (at most 64 terms, each
// at most 1): the emit's row prefix.  Sums that cross tiles stay in FP64.
__device__ __forceinline__ LeakyT<float> to_float(const Leaky& L) {
  return {(float)L.g1, (float)L.g2, (float)L.g4, (float)L.g8, (float)L.f15, (float)L.f31};
}

template <int CTRL>
__device__ __forceinline__ float dpp_all(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf,
                                                               0xf, true));
}

__device__ __forceinline__ float leaky_scan(float v, const LeakyT<float>& L) {
  v = fmaf(L.g1, dpp_all<0x111>(v), v);
  v = fmaf(L.g2, dpp_all<0x112>(v), v);
  v = fmaf(L.g4, dpp_all<0x114>(v), v);
  v = fmaf(L.g8, dpp_all<0x118>(v), v);
  v = fmaf(L.f15, dpp_all<0x142>(v), v);
  v = fmaf(L.f31, dpp_all<0x143>(v), v);
  return v;
}

struct ExpTile {
  int d, b, tx, ty, y0, nrows;
};

// Wave -> (direction, bin, band, tile); tile fastest.
__device__ __forceinline__ bool exp_tile(const SwihGeom& g, long wid, ExpTile& t) {
  const long nw = 4L * g.B * g.NTY * g.NTX;
  if (wid >= nw) return false;
  t.tx = (int)(wid % g.NTX);
  long r = wid / g.NTX;
  t.ty = (int)(r % g.NTY);
  r /= g.NTY;
  t.b = (int)(r % g.B);
  t.d = (int)(r / g.B);
  t.y0 = t.ty * g.TY;
  t.nrows = min(g.TY, g.H - t.y0);
  return true;
}

// Bit k = [Q(f) = b] at mirrored column 64 tx + lane, mirrored row y0 + k
// (k < nrows); zero for columns past the image.
__device__ __forceinline__ uint64_t exp_band_mask(const ExpBuildArgs& a, const ExpTile& t) {
  const SwihGeom& g = a.g;
  const int xm = t.tx * 64 + lane_id();
  const bool valid = xm < g.W;
  const int xo = valid ? ((t.d & 1) ? g.W - 1 - xm : xm) : 0;
  const bool my = (t.d & 2) != 0;
  // the band's rows in memory start at its lowest image row; mirrored row
  // y0 + kk sits (nrows - 1 - kk) rows above it when rows are mirrored
  const uint8_t* band = a.img + (long)(my ? g.H - t.y0 - t.nrows : t.y0) * a.ipitch;
  auto row = [&](int kk) {
    return (uint32_t)((my ? t.nrows - 1 - kk : kk) * a.ipitch) + (uint32_t)xo;
  };
  // [Q(v) = b] exactly when ceil(256 b / B) <= v < ceil(256 (b + 1) / B)
  const uint32_t B = (uint32_t)g.B, b = (uint32_t)t.b;
  const uint32_t vlo = (256u * b + B - 1) / B, span = (256u * (b + 1) + B - 1) / B - vlo;
  uint32_t lo = 0, hi = 0;
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const int kk = k < t.nrows ? k : t.nrows - 1;
    lo |= (uint32_t)((uint32_t)band[row(kk)] - vlo < span) << k;
  }
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const int kk = k + 32 < t.nrows ? k + 32 : t.nrows - 1;
    hi |= (uint32_t)((uint32_t)band[row(kk)] - vlo < span) << k;
  }
  uint64_t m = ((uint64_t)hi << 32) | lo;
  if (t.nrows < 64) m &= ((uint64_t)1 << t.nrows) - 1;
  return valid ? m : 0;
}


// ---------------------------------------------------------------- build
// Aggregate by LDS histograms (at most kExpHistMaxB bins): one block per
// (direction, band, tile) gathers every bin at once.  Each pixel adds its
// weight to the LDS counter of its bin: qy^(TY - k) to its column's (k = its
// mirrored row in the band) and qx^(64 - l) to its row's (l = its mirrored
// column in the tile).  Weights are fixed point in units of 2^-52 and a
// counter sums at most 64 of them (each below 1), so the int64 sums are exact
// and do not depend on the order the atomics land in.  The counters then give
// the same z, CT and T as the per-bin form.
constexpr int kExpHistMaxB = 32;
constexpr int kExpHistRow = 80;  // LDS bytes per staged row (16-byte aligned, banks spread)

__host__ __device__ constexpr int exp_hist_lds_bytes(int B) {
  return 64 * kExpHistRow + 2 * 64 * 8 + 2 * B * 64 * 8;
}

extern __shared__ __align__(16) unsigned char exp_hist_lds[];

__device__ __forceinline__ void exp_aggregate_hist(const ExpBuildArgs& a, int vb) {
  const SwihGeom& g = a.g;
  const int B = g.B;
  const int tx = vb % g.NTX, r = vb / g.NTX;
  const int ty = r % g.NTY, d = r / g.NTY;
  const int y0 = ty * g.TY, nrows = min(g.TY, g.H - y0);
  const int w = (int)(threadIdx.x >> 6), lane = lane_id();
  unsigned char* tile = exp_hist_lds;
  int64_t* py = (int64_t*)(exp_hist_lds + 64 * kExpHistRow);  // [64] qy^(TY - k)
  int64_t* px = py + 64;                                        // [64] qx^(64 - l)
  int64_t* colh = px + 64;                                      // [B][64]
  int64_t* rowh = colh + B * 64;                                // [B][64]
  constexpr double kFix = 4503599627370496.0;                   // 2^52
  // wave w loads mirrored rows 16 w .. 16 w + 15 of the band at mirrored
  // column 64 tx + lane (clamped into the image)
  const int xm = tx * 64 + lane;
  const bool xok = xm < g.W;
  const int xo = xok ? ((d & 1) ? g.W - 1 - xm : xm) : 0;
  const bool my = (d & 2) != 0;
  // the band's lowest image row plus a 32-bit offset per load (mirrored row
  // y0 + kk sits nrows - 1 - kk rows above it when rows are mirrored)
  const uint8_t* band = a.img + (long)(my ? g.H - y0 - nrows : y0) * a.ipitch;
  uint32_t v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int k = 16 * w + i;
    const int kk = k < nrows ? k : nrows - 1;
    v[i] = band[(uint32_t)((my ? nrows - 1 - kk : kk) * a.ipitch) + (uint32_t)xo];
  }
  __syncthreads();  // an earlier virtual block of this block is done with LDS
  {
    uint4* c4 = (uint4*)colh;
    const int n4 = 2 * B * 64 * 8 / 16;
    for (int i = (int)threadIdx.x; i < n4; i += WG) c4[i] = make_uint4(0u, 0u, 0u, 0u);
    const int t = (int)threadIdx.x;
    if (t < 64) py[t] = t < g.TY ? (int64_t)llrint(dpow(a.qy, g.TY - t) * kFix) : 0;
    else if (t < 128) px[t - 64] = (int64_t)llrint(dpow(a.qx, 128 - t) * kFix);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int k = 16 * w + i;
    tile[k * kExpHistRow + lane] = (unsigned char)v[i];
    if (k < nrows && xok)
      __hip_atomic_fetch_add(&colh[((v[i] * (uint32_t)B) >> 8) * 64 + lane], py[k], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __syncthreads();
  {
    // lane = mirrored row of the band, wave w counts mirrored columns 16 w .. 16 w + 15
    const uint4 r4 = *(const uint4*)(tile + lane * kExpHistRow + 16 * w);
    const uint32_t rw[4] = {r4.x, r4.y, r4.z, r4.w};
    const int nx = min(16, g.W - (tx * 64 + 16 * w));
    if (lane < nrows) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const uint32_t pv = (rw[j >> 2] >> (8 * (j & 3))) & 255u;
        if (j < nx)
          __hip_atomic_fetch_add(&rowh[((pv * (uint32_t)B) >> 8) * 64 + lane], px[16 * w + j],
                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
  __syncthreads();
  const long NXP = (long)g.NTX * 64;
  const Leaky Lx = make_leaky(a.qx);
  for (int b = w; b < B; b += WPB) {
    const long db = (long)d * B + b;
    const double c = (double)colh[b * 64 + lane] / kFix;
    const double zl = a.qx * leaky_scan(c, Lx);
    a.z[(db * g.NTY + ty) * NXP + (long)tx * 64 + lane] = zl;
    if (lane == 63) a.CT[(db * g.NTY + ty) * g.NTX + tx] = zl;
    if (lane < nrows) a.T[(db * g.NTX + tx) * g.H + y0 + lane] = (double)rowh[b * 64 + lane] / kFix;
  }
}

// Aggregate: per (direction, bin, band, tile) wave (band of TY rows)
//   z  [X]  = sum_{X0 <= x < X, y in band} [Q = b] qx^(X - x) qy^(Y0 + TY - y)
//   CT      = the same at X = X0 + 64 (the tile total)
//   T  [y]  = sum_{x in tile} [Q = b] qx^(X0 + 64 - x)      (lane = row)
__device__ __forceinline__ void exp_aggregate(const ExpBuildArgs& a, int vb) {
  if (a.agg_hist) {
    exp_aggregate_hist(a, vb);
    return;
  }
  const SwihGeom& g = a.g;
  // per block: byte tables F[v] = sum over the set bits r of v of q^(8 - r),
  // for qy (band sums) and qx (row sums); every wave of the block helps build
  // them before any returns
  __shared__ double Fy[256], Fx[256];
  for (int v = threadIdx.x; v < 256; v += blockDim.x) {
    double fy = 0.0, fx = 0.0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const double bit = (double)((v >> r) & 1);
      fy = (fy + bit) * a.qy;
      fx = (fx + bit) * a.qx;
    }
    Fy[v] = fy;
    Fx[v] = fx;
  }
  __syncthreads();
  ExpTile t;
  const bool have = exp_tile(g, exp_wave(vb), t);
  if (have) {
    const int lane = lane_id();
    const long NXP = (long)g.NTX * 64;
    const uint64_t mask = exp_band_mask(a, t);
    // this column's band sum relative to row Y0 + TY: sum_k bit_k qy^(TY - k),
    // byte c of the mask weighing F[byte] q^(TY - 8c - 8)
    double c = 0.0;
    const int nch = g.TY >> 3;
#pragma unroll
    for (int k = 0; k < 8; ++k) c = k < nch ? fma(c, a.qy8, Fy[(mask >> (8 * k)) & 255]) : c;
    const double zl = a.qx * leaky_scan(c, make_leaky(a.qx));
    const long db = (long)t.d * g.B + t.b;
    a.z[(db * g.NTY + t.ty) * NXP + (long)t.tx * 64 + lane] = zl;
    if (lane == 63) a.CT[(db * g.NTY + t.ty) * g.NTX + t.tx] = zl;
    // row sums across the tile: after the transpose lane k holds row k's
    // columns, T(y) = sum_l bit_l qx^(64 - l)
    const uint64_t rowm = wave_transpose64(mask);
    double tr = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) tr = fma(tr, a.qx8, Fx[(rowm >> (8 * k)) & 255]);
    if (lane < t.nrows) a.T[(db * g.NTX + t.tx) * g.H + t.y0 + lane] = tr;
  }
  // the tables are rebuilt for the next virtual block of a batched launch
  __syncthreads();
}

// Scan: three independent chains.
//   role 1, one thread per (direction, bin, column): z over bands becomes the
//     band-top value Zc (exclusive), Zc' = qy^TY Zc + z;
//   role 2, one thread per (direction, bin, row): T over tiles becomes the row
//     value at the tile's left edge (exclusive), C' = qx^64 C + T;
//   role 3, one wave per (direction, bin): CT becomes E(64 tx, 64 ty), with an
//     exclusive leaky scan over the tiles of each band (decay qx^64).
__device__ __forceinline__ void exp_scan(const ExpBuildArgs& a, int vb) {
  const SwihGeom& g = a.g;
  const long NXP = (long)g.NTX * 64;
  if (vb < a.nb1) {
    const long t = (long)vb * WG + threadIdx.x;
    if (t >= 4L * g.B * NXP) return;
    const long db = t / NXP, col = t - db * NXP;
    const double qT = a.qyT;
    double* z = a.z + db * g.NTY * NXP + col;
    double carry = 0.0;
    for (int ty = 0; ty < g.NTY; ++ty) {
      const double v = z[ty * NXP];
      z[ty * NXP] = carry;
      carry = fma(qT, carry, v);
    }
    return;
  }
  vb -= a.nb1;
  if (vb < a.nb2) {
    const long t = (long)vb * WG + threadIdx.x;
    if (t >= 4L * g.B * g.H) return;
    const long db = t / g.H;
    const int y = (int)(t - db * g.H);
    const double qT = a.qx64;
    double* T = a.T + db * g.NTX * g.H + y;
    double carry = 0.0;
    for (int tx = 0; tx < g.NTX; ++tx) {
      const double v = T[(long)tx * g.H];
      T[(long)tx * g.H] = carry;
      carry = fma(qT, carry, v);
    }
    return;
  }
  vb -= a.nb2;
  const long wid = exp_wave(vb);
  if (wid >= 4L * g.B) return;
  const int lane = lane_id();
  double* CT = a.CT + wid * g.NTY * g.NTX;
  const double qyT = a.qyT;
  const Leaky Lt = make_leaky(a.qx64);
  const double up = dpow(a.qx64, lane + 1);  // decay from tile 63 of the first chunk
  const bool v0 = lane < g.NTX, v1 = 64 + lane < g.NTX;  // NTX <= 128
  double k0 = 0.0, k1 = 0.0;
  // eight bands' tile sums are loaded before any of them is replaced, so each
  // group of eight costs one memory round trip
  for (int ty0 = 0; ty0 < g.NTY; ty0 += 8) {
    double t0[8], t1[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double* row = CT + (long)(ty0 + u) * g.NTX;
      const bool in = ty0 + u < g.NTY;
      t0[u] = in && v0 ? row[lane] : 0.0;
      t1[u] = in && v1 ? row[64 + lane] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (ty0 + u >= g.NTY) break;
      double* row = CT + (long)(ty0 + u) * g.NTX;
      if (v0) row[lane] = k0;
      if (v1) row[64 + lane] = k1;
      const double s0 = leaky_scan(t0[u], Lt);
      const double last0 = readlane(s0, 63);
      const double s1 = fma(up, last0, leaky_scan(t1[u], Lt));
      const double p0 = __shfl_up(s0, 1, 64);
      const double p1 = __shfl_up(s1, 1, 64);
      const double a0 = lane == 0 ? 0.0 : p0;
      const double a1 = lane == 0 ? last0 : p1;
      k0 = fma(qyT, k0, a0);
      k1 = fma(qyT, k1, a1);
    }
  }
}

// Emit: per (direction, bin, band, tile) wave, rows top to bottom,
//   E(X, Y0) = Zc(X) + qx^(X - X0) E(X0, Y0),
//   E(X, y + 1) = qy (E(X, y) + qx s_l + qx^(l + 1) C(y)),
// s the leaky scan of the row's [Q = b] across the tile and C(y) the row value
// at the tile's left edge.  Every lane stores, so a wave writes whole 256-byte
// rows (lanes past the last column hold values never read).  NTS: non-temporal
// plane stores.
template <bool NTS>
__device__ __forceinline__ void exp_emit(const ExpBuildArgs& a, int vb) {
  const SwihGeom& g = a.g;
  ExpTile t;
  if (!exp_tile(g, exp_wave(vb), t)) return;
  const int lane = lane_id();
  const long NXP = (long)g.NTX * 64;
  const uint64_t mask = exp_band_mask(a, t);
  const double qx = a.qx, qy = a.qy;
  const double pw = dpow(qx, lane + 1);
  const LeakyT<float> Lx = to_float(make_leaky(qx));
  const long db = (long)t.d * g.B + t.b;
  const double K = a.CT[(db * g.NTY + t.ty) * g.NTX + t.tx];
  double e = fma(pw, K, a.z[(db * g.NTY + t.ty) * NXP + (long)t.tx * 64 + lane]);
  const double creg = a.T[(db * g.NTX + t.tx) * g.H + t.y0 + (lane < t.nrows ? lane : 0)];
  float* P = a.planes + swih_base(g, t.d, t.b) + (long)t.tx * g.tile_stride + lane;
  if (t.ty == 0) P[0] = 0.0f;
  for (int k = 0; k < t.nrows; ++k) {
    const double s = (double)leaky_scan((float)((uint32_t)(mask >> k) & 1u), Lx);
    const double R = fma(qx, s, pw * readlane(creg, k));
    e = qy * (e + R);
    float* dst = P + (long)(t.y0 + k + 1) * g.row_stride;
    if constexpr (NTS)
      __builtin_nontemporal_store((float)e, dst);
    else
      *dst = (float)e;
  }
}

// ---------------------------------------------------------------- lookups
__device__ __forceinline__ double e_at(const SwihGeom& g, const float* __restrict__ pl, int64_t base,
                                       int Y, int X) {
  const int Xc = X > 0 ? X : 1;
  const float v = pl[base + (int64_t)Y * g.row_stride + swih_xoff(g, Xc)];
  return X > 0 ? (double)v : 0.0;
}

// Empty bins.  sqrt is not Lipschitz at 0, so a bin with no pixel in the
// window must give exactly 0, not a rounding residue e (whose sqrt(e t_b) would
// be orders of magnitude above e).  The planes hold no pixel count, but every
// term is positive, which bounds the rounding:
//   * the in-row prefix is an FP32 leaky scan, six FMA stages with factors
//     rounded to float, so each of its positive terms is off by at most
//     12 * 2^-24 relative; the FP64 chains that carry it keep that relative
//     bound (sums of positive terms), and the float store adds 2^-24;
//   * so each stored E is within 13 * 2^-24 of its exact value, relative, plus
//     an absolute error far below 1e-9 from the FP64 carries' fixed-point
//     weights (2^-52 each);
//   * the window value is sum +- T over 16 scaled corners T = f E >= 0, hence
//     |h' - h| <= eb = 16 * 2^-24 * sum T + 1e-9.
// A bin with a pixel in the window has h >= wmin = exp(-rx/tx - ry/ty), the
// kernel's smallest weight (> e^-4).  Whenever eb < wmin / 2 the test
// h' < wmin / 2 is therefore exactly "no pixel": such bins give 0.  (eb is
// far below that for any window up to several hundred pixels; beyond it the
// value is kept as computed.)
constexpr double kExpRel = 16.0 / 16777216.0;  // 16 * 2^-24
constexpr double kExpAbs = 1e-9;

// H_b at centre (xc, yc): the four quadrant boxes, each from its direction's
// plane, with an exactly empty bin returned as 0 (above).
__device__ __forceinline__ double exp_hist(const SwihGeom& g, const ExpScale& s,
                                           const float* __restrict__ pl, int b, int xc, int yc) {
  // corners (far, near) and their factors per side
  const int XL0 = xc - s.rx, XL1 = xc + 1;
  const int XR0 = g.W - 1 - xc - s.rx, XR1 = g.W - 1 - xc;
  const int YT0 = yc - s.ry, YT1 = yc + 1;
  const int YB0 = g.H - 1 - yc - s.ry, YB1 = g.H - 1 - yc;
  double h = 0.0, tsum = 0.0;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const bool mx = d & 1, my = d & 2;
    const int X0 = mx ? XR0 : XL0, X1 = mx ? XR1 : XL1;
    const int Y0 = my ? YB0 : YT0, Y1 = my ? YB1 : YT1;
    const double f0x = s.fxlo, f1x = mx ? 1.0 : s.fxin;
    const double f0y = s.fylo, f1y = my ? 1.0 : s.fyin;
    const int64_t base = swih_base(g, d, b);
    const double e11 = e_at(g, pl, base, Y1, X1), e01 = e_at(g, pl, base, Y1, X0);
    const double e10 = e_at(g, pl, base, Y0, X1), e00 = e_at(g, pl, base, Y0, X0);
    h += f1y * (f1x * e11 - f0x * e01) - f0y * (f1x * e10 - f0x * e00);
    tsum += f1y * (f1x * e11 + f0x * e01) + f0y * (f1x * e10 + f0x * e00);
  }
  const double half_min = 0.5 * s.fxlo * s.fylo;
  return fma(kExpRel, tsum, kExpAbs) < half_min && h < half_min ? 0.0 : h;
}

// One thread per (centre, bin).
__device__ __forceinline__ void exp_query(const ExpQueryArgs& a, int vb) {
  const long t = (long)vb * WG + threadIdx.x;
  const int B = a.g.B;
  if (t >= (long)a.n * B) return;
  const long i = t / B;
  const int b = (int)(t - i * B);
  // centres outside the valid range are clamped into it
  const int xc = min(max(a.centres[2 * i], a.s.rx), a.g.W - 1 - a.s.rx);
  const int yc = min(max(a.centres[2 * i + 1], a.s.ry), a.g.H - 1 - a.s.ry);
  const double h = exp_hist(a.g, a.s, a.planes, b, xc, yc);
  a.hist[t] = (float)(h * a.s.inv_mass);
}

// One thread per centre: sum_b sqrt(p_b t_b) in double, bins in order.  A wave
// covers 64 consecutive centres of one row.
__device__ __forceinline__ void exp_match(const ExpMatchArgs& a, int vb) {
  const long w = exp_wave(vb);
  const int nx = a.x1 - a.x0 + 1, ny = a.y1 - a.y0 + 1;
  const int row = (int)(w / a.nbx), wc = (int)(w - (long)row * a.nbx);
  if (row >= ny) return;
  const int xc = a.x0 + wc * 64 + lane_id();
  if (xc > a.x1) return;
  const int yc = a.y0 + row;
  double acc = 0.0;
  for (int b = 0; b < a.g.B; ++b) {
    const double p = exp_hist(a.g, a.s, a.planes, b, xc, yc) * a.s.inv_mass;
    acc += sqrt(fmax(p, 0.0) * fmax((double)a.tmpl[b], 0.0));
  }
  a.map[(long)row * nx + (xc - a.x0)] = (float)acc;
}

}  // namespace

// Single launch: one block per virtual block.  Batched: a grid-stride loop
// over every item's virtual blocks, each block finding its item by binary
// search over the prefix of block counts.
template <class A, void (*BODY)(const A&, int)>
__global__ __launch_bounds__(WG) void k_exp_one(A a) {
  BODY(a, (int)blockIdx.x);
}

template <class A, void (*BODY)(const A&, int)>
__global__ __launch_bounds__(WG) void k_exp_many(const A* __restrict__ items,
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
hipError_t one(const A& a, int32_t nb, hipStream_t s, int lds = 0) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_exp_one<A, BODY>), dim3((unsigned)nb), dim3(WG), lds, s, a);
  return hipGetLastError();
}

template <class A, void (*BODY)(const A&, int)>
hipError_t many(const A* items, const int32_t* prefix, int n, int32_t total, int grid,
                hipStream_t s, int lds = 0) {
  if (n <= 0 || total <= 0) return hipSuccess;
  const unsigned gb = (unsigned)(total < grid ? total : grid);
  hipLaunchKernelGGL((k_exp_many<A, BODY>), dim3(gb), dim3(WG), lds, s, items, prefix, n);
  return hipGetLastError();
}

inline int32_t blocks_of_waves(long w) { return (int32_t)((w + WPB - 1) / WPB); }
inline int32_t blocks_of_threads(long n) { return (int32_t)((n + WG - 1) / WG); }

}  // namespace

// ---------------------------------------------------------------- host side
void exp_scale(int32_t w, int32_t h, ExpScale& s) {
  memset(&s, 0, sizeof(s));
  s.w = w;
  s.h = h;
  s.rx = (w - 1) / 2;
  s.ry = (h - 1) / 2;
  const double tx = w / 4.0, ty = h / 4.0;
  s.itx = 1.0 / tx;
  s.ity = 1.0 / ty;
  s.fxlo = exp(-s.rx / tx);
  s.fylo = exp(-s.ry / ty);
  s.fxin = exp(1.0 / tx);
  s.fyin = exp(1.0 / ty);
  double sx = 0.0, sy = 0.0;  // axis masses, summed outward from the rim
  for (int d = s.rx; d >= 1; --d) sx += 2.0 * exp(-d / tx);
  for (int d = s.ry; d >= 1; --d) sy += 2.0 * exp(-d / ty);
  s.mass = (1.0 + sx) * (1.0 + sy);
  s.inv_mass = 1.0 / s.mass;
}

void exp_build_args(const SwihLayout& L, const ExpScale& s, int set, const uint8_t* img,
                    int32_t img_pitch, char* ws, ExpBuildArgs& a, int32_t (&nb)[4]) {
  const SwihGeom& g = L.g;
  memset(&a, 0, sizeof(a));
  a.g = g;
  a.img = img;
  a.ipitch = img_pitch;
  char* sb = ws + (size_t)set * L.set_bytes;
  a.planes = (float*)(sb + L.off_planes);
  a.z = (double*)(sb + L.off_z);
  a.T = (double*)(sb + L.off_T);
  a.CT = (double*)(sb + L.off_CT);
  a.itx = s.itx;
  a.ity = s.ity;
  a.qx = exp(-s.itx);
  a.qy = exp(-s.ity);
  a.qx8 = exp(-8.0 * s.itx);
  a.qy8 = exp(-8.0 * s.ity);
  a.qyT = exp(-s.ity * g.TY);
  a.qx64 = exp(-64.0 * s.itx);
  const long waves = 4L * g.B * g.NTY * g.NTX;
  a.nb1 = blocks_of_threads(4L * g.B * g.NTX * 64);
  a.nb2 = blocks_of_threads(4L * g.B * g.H);
  // the form depends on the bin count only, so one plane set and a batch of
  // them round alike
  a.agg_hist = g.B <= kExpHistMaxB;
  nb[0] = 0;
  nb[1] = a.agg_hist ? 4 * g.NTY * g.NTX : blocks_of_waves(waves);
  nb[2] = a.nb1 + a.nb2 + blocks_of_waves(4L * g.B);
  nb[3] = blocks_of_waves(waves);
}

void exp_query_args(const SwihLayout& L, const ExpScale& s, int set, const char* ws,
                    const int32_t* centres, int32_t n, float* hist, ExpQueryArgs& a, int32_t& nb) {
  memset(&a, 0, sizeof(a));
  a.g = L.g;
  a.s = s;
  a.planes = (const float*)(ws + (size_t)set * L.set_bytes + L.off_planes);
  a.centres = centres;
  a.n = n;
  a.hist = hist;
  nb = blocks_of_threads((long)n * L.g.B);
}

void exp_match_args(const SwihLayout& L, const ExpScale& s, int set, const char* ws,
                    const float* tmpl, int32_t x0, int32_t y0, int32_t x1, int32_t y1, float* map,
                    ExpMatchArgs& a, int32_t& nb) {
  memset(&a, 0, sizeof(a));
  a.g = L.g;
  a.s = s;
  a.planes = (const float*)(ws + (size_t)set * L.set_bytes + L.off_planes);
  a.tmpl = tmpl;
  a.map = map;
  a.x0 = x0;
  a.y0 = y0;
  a.x1 = x1;
  a.y1 = y1;
  a.nbx = (x1 - x0 + 1 + 63) / 64;
  nb = blocks_of_waves((long)a.nbx * (y1 - y0 + 1));
}

namespace {
constexpr void (*agg_body)(const ExpBuildArgs&, int) = exp_aggregate;
constexpr void (*scan_body)(const ExpBuildArgs&, int) = exp_scan;
constexpr void (*emit_body)(const ExpBuildArgs&, int) = exp_emit<false>;
// plane sets from about the last-level cache's size on: non-temporal stores
constexpr void (*emit_body_nt)(const ExpBuildArgs&, int) = exp_emit<true>;
constexpr int64_t kExpNtPlaneBytes = 256ll << 20;
constexpr void (*query_body)(const ExpQueryArgs&, int) = exp_query;
constexpr void (*match_body)(const ExpMatchArgs&, int) = exp_match;
}  // namespace

hipError_t exp_launch_build(const ExpBuildArgs& a, const int32_t (&nb)[4], int phases,
                            hipStream_t s) {
  hipError_t e = hipSuccess;
  if (phases & 1) {
    e = one<ExpBuildArgs, agg_body>(a, nb[1], s, a.agg_hist ? exp_hist_lds_bytes(a.g.B) : 0);
    if (e == hipSuccess) e = one<ExpBuildArgs, scan_body>(a, nb[2], s);
  }
  const SwihGeom& g = a.g;
  const int64_t plane_bytes = (int64_t)g.nPL * g.B * g.NTX * (g.H + 1) * SWIH_TX * 4;
  if (e == hipSuccess && (phases & 2))
    e = plane_bytes >= kExpNtPlaneBytes ? one<ExpBuildArgs, emit_body_nt>(a, nb[3], s)
                                        : one<ExpBuildArgs, emit_body>(a, nb[3], s);
  return e;
}

hipError_t exp_launch_query(const ExpQueryArgs& a, int32_t nb, hipStream_t s) {
  return one<ExpQueryArgs, query_body>(a, nb, s);
}

hipError_t exp_launch_match(const ExpMatchArgs& a, int32_t nb, hipStream_t s) {
  return one<ExpMatchArgs, match_body>(a, nb, s);
}

hipError_t exp_launch_build_batch(const ExpBuildArgs* units, const int32_t* prefix, int nunits,
                                  int nbins, const int32_t (&total)[4], int grid, hipStream_t s) {
  if (nunits <= 0) return hipSuccess;
  const int32_t* pre[4];
  for (int k = 0; k < 4; ++k) pre[k] = prefix + (size_t)k * (nunits + 1);
  hipError_t e = many<ExpBuildArgs, agg_body>(units, pre[1], nunits, total[1], grid, s,
                                              nbins <= kExpHistMaxB ? exp_hist_lds_bytes(nbins) : 0);
  if (e == hipSuccess) e = many<ExpBuildArgs, scan_body>(units, pre[2], nunits, total[2], grid, s);
  // a batch streams its planes past the last-level cache, as large single sets do
  if (e == hipSuccess) e = many<ExpBuildArgs, emit_body_nt>(units, pre[3], nunits, total[3], grid, s);
  return e;
}

hipError_t exp_launch_query_batch(const ExpQueryArgs* items, const int32_t* prefix, int n,
                                  int32_t total, int grid, hipStream_t s) {
  return many<ExpQueryArgs, query_body>(items, prefix, n, total, grid, s);
}

hipError_t exp_launch_match_batch(const ExpMatchArgs* items, const int32_t* prefix, int n,
                                  int32_t total, int grid, hipStream_t s) {
  return many<ExpMatchArgs, match_body>(items, prefix, n, total, grid, s);
}

}  // namespace swih
