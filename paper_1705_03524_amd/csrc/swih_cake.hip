// Baselines the paper measures SWIH against (Sec. 2, Sec. 3, Figs. 5 and 6):
//
// * Wedding cake (Sec. 2, Fig. 4a): the window is cut into n nested windows
//   R_0 (the whole window) > R_1 > ... > R_{n-1} around the centre, per axis
//   r_i = floor((r + 1)(n - i) / n) - 1 (equal runs of the distances 0..r; a
//   negative half-size is an empty window).  Ring i = R_i minus R_{i+1} gets
//   one weight w_i, the mean of the kernel over its pixels, so the total mass
//   stays S.  With C_b(R) the plain count of bin b in R (four corners of the
//   count plane, the integral histogram of Sec. 1),
//     H~_b = sum_i w_i (C_b(R_i) - C_b(R_{i+1})) = sum_i (w_i - w_{i-1}) C_b(R_i),
//   O(n) lookups per window and bin, whatever the window size.
// * Brute force (Sec. 2, the convolution-style approach): every pixel of the
//   window adds its integer kernel weight to its bin; O(w h) per window.
//   Exact (uint32) for the integer kernels, so its map equals swih_match's bit
//   for bit.
#include <math.h>
#include <string.h>

#include "swih.h"
#include "swih_internal.h"
#include "wave64.h"

namespace swih {
namespace {

constexpr int WG = 256;
constexpr int WPB = WG / 64;

__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Count of bin b in the box [xc - ax, xc + ax] x [yc - ay, yc + ay] (ax, ay >= 0).
__device__ __forceinline__ uint32_t box_count(const SwihGeom& g, const uint32_t* __restrict__ pl,
                                              int64_t base, int xc, int yc, int ax, int ay) {
  const int X0 = xc - ax, X1 = xc + ax + 1, Y0 = yc - ay, Y1 = yc + ay + 1;
  const int64_t xo1 = swih_xoff(g, X1);
  const int64_t xo0 = swih_xoff(g, X0 > 0 ? X0 : 1);
  const uint32_t a = pl[base + (int64_t)Y1 * g.row_stride + xo1];
  const uint32_t c = pl[base + (int64_t)Y0 * g.row_stride + xo1];
  // column X = 0 is not stored: read column 1 and use 0
  const uint32_t bb = pl[base + (int64_t)Y1 * g.row_stride + xo0];
  const uint32_t d = pl[base + (int64_t)Y0 * g.row_stride + xo0];
  return X0 > 0 ? a - c - bb + d : a - c;  // modulo 2^32, exact: the true count is below 2^32
}

__device__ __forceinline__ double cake_hist(const CakeArgs& a, int b, int xc, int yc) {
  const int64_t base = swih_base(a.g, 0, b);  // plane 0 = the count term {1}
  double h = 0.0;
  for (int i = 0; i < a.nrings; ++i) {
    const int ax = a.rx[i], ay = a.ry[i];
    if (ax < 0 || ay < 0) break;  // inner windows are empty from here on
    h = fma(a.dw[i], (double)box_count(a.g, (const uint32_t*)a.planes, base, xc, yc, ax, ay), h);
  }
  return h;
}

// One thread per (centre, bin).
__device__ __forceinline__ void cake_query(const CakeArgs& a, int vb) {
  const long t = (long)vb * WG + threadIdx.x;
  const int B = a.g.B;
  if (t >= (long)a.n * B) return;
  const long i = t / B;
  const int b = (int)(t - i * B);
  // centres outside the valid range are clamped into it
  const int xc = min(max(a.centres[2 * i], a.rx[0]), a.g.W - 1 - a.rx[0]);
  const int yc = min(max(a.centres[2 * i + 1], a.ry[0]), a.g.H - 1 - a.ry[0]);
  a.hist[t] = (float)(cake_hist(a, b, xc, yc) / a.mass);
}

// One thread per centre, a wave per 64 consecutive centres of a row:
// sum_b sqrt(p_b t_b) in double, bins in order.
__device__ __forceinline__ void cake_match(const CakeArgs& a, int vb) {
  const long w = (long)vb * WPB + rfl((int)(threadIdx.x >> 6));
  const int nx = a.x1 - a.x0 + 1, ny = a.y1 - a.y0 + 1;
  const int row = (int)(w / a.nbx), wc = (int)(w - (long)row * a.nbx);
  if (row >= ny) return;
  const int xc = a.x0 + wc * 64 + lane_id();
  if (xc > a.x1) return;
  const int yc = a.y0 + row;
  double acc = 0.0;
  for (int b = 0; b < a.g.B; ++b) {
    const double p = cake_hist(a, b, xc, yc) / a.mass;
    acc += sqrt(fmax(p, 0.0) * fmax((double)a.tmpl[b], 0.0));
  }
  a.map[(long)row * nx + (xc - a.x0)] = (float)acc;
}

// Brute force, one thread per centre, 64 centres per block; each thread keeps
// its histogram in LDS at [bin][lane] (a lane's bins share one bank).
__device__ __forceinline__ void brute_match(const BruteArgs& a, int vb) {
  extern __shared__ uint32_t hs[];
  const int lane = (int)threadIdx.x;
  const int nx = a.x1 - a.x0 + 1, ny = a.y1 - a.y0 + 1;
  const int row = vb / a.nbx, wc = vb - row * a.nbx;
  const int B = a.B;
  for (int b = 0; b < B; ++b) hs[b * 64 + lane] = 0u;
  const int xc = a.x0 + wc * 64 + lane;
  const bool valid = row < ny && xc <= a.x1;
  if (valid) {
    const int yc = a.y0 + row;
    for (int dy = -a.ry; dy <= a.ry; ++dy) {
      const uint8_t* src = a.img + (long)(yc + dy) * a.ipitch + xc;
      const uint32_t ady = (uint32_t)(dy < 0 ? -dy : dy);
      for (int dx = -a.rx; dx <= a.rx; ++dx) {
        const uint32_t adx = (uint32_t)(dx < 0 ? -dx : dx);
        uint32_t k;
        if (a.kind == SWIH_MANHATTAN) k = a.c_int - adx - ady;
        else if (a.kind == SWIH_EUCLIDEAN) k = a.c_int - adx * adx - ady * ady;
        else k = 1u;
        const uint32_t b = __umul24((uint32_t)src[dx], (uint32_t)B) >> 8;  // floor(v B / 256)
        atomicAdd(&hs[b * 64 + lane], k);
      }
    }
    double acc = 0.0;
    for (int b = 0; b < B; ++b)
      acc += sqrt((double)((uint64_t)hs[b * 64 + lane] * (uint64_t)a.tmpl_raw[b]));
    a.map[(long)row * nx + (xc - a.x0)] = (float)(acc / a.mass);  // as swih_match: one division
  }
}

}  // namespace

template <class A, void (*BODY)(const A&, int)>
__global__ __launch_bounds__(WG) void k_cake_one(A a) {
  BODY(a, (int)blockIdx.x);
}

template <class A, void (*BODY)(const A&, int)>
__global__ __launch_bounds__(64) void k_brute_one(A a) {
  BODY(a, (int)blockIdx.x);
}

namespace {
constexpr void (*cake_query_body)(const CakeArgs&, int) = cake_query;
constexpr void (*cake_match_body)(const CakeArgs&, int) = cake_match;
constexpr void (*brute_body)(const BruteArgs&, int) = brute_match;
}  // namespace

// ---------------------------------------------------------------- host side
namespace {

// Sum of an integer kernel over the box of half-sizes (ax, ay) centred on the
// window centre (closed forms of sum |d| and sum d^2).
double box_sum(int kind, double c, long ax, long ay) {
  if (ax < 0 || ay < 0) return 0.0;
  const double nx = 2.0 * ax + 1, ny = 2.0 * ay + 1;
  if (kind == SWIH_UNIFORM) return nx * ny;
  if (kind == SWIH_MANHATTAN) return c * nx * ny - ny * ax * (ax + 1) - nx * ay * (ay + 1);
  return c * nx * ny - ny * ax * (ax + 1) * (2.0 * ax + 1) / 3.0 -
         nx * ay * (ay + 1) * (2.0 * ay + 1) / 3.0;
}

}  // namespace

int cake_args(int kind, const SwihGeom& g, int32_t w, int32_t h, int32_t rings, double mass,
              uint32_t c_int, const void* planes, CakeArgs& a) {
  memset(&a, 0, sizeof(a));
  if (rings < 1 || rings > SWIH_MAX_RINGS) return -1;
  a.g = g;
  a.planes = planes;
  a.nrings = rings;
  const int rx = (w - 1) / 2, ry = (h - 1) / 2;
  double prev = 0.0;
  for (int i = 0; i < rings; ++i) {
    a.rx[i] = (int32_t)((long)(rx + 1) * (rings - i) / rings - 1);
    a.ry[i] = (int32_t)((long)(ry + 1) * (rings - i) / rings - 1);
  }
  for (int i = 0; i < rings; ++i) {
    const long ax = a.rx[i], ay = a.ry[i];
    const long bx = i + 1 < rings ? a.rx[i + 1] : -1, by = i + 1 < rings ? a.ry[i + 1] : -1;
    const double cnt = box_sum(SWIH_UNIFORM, 0, ax, ay) - box_sum(SWIH_UNIFORM, 0, bx, by);
    const double sum = box_sum(kind, (double)c_int, ax, ay) - box_sum(kind, (double)c_int, bx, by);
    const double wi = cnt > 0 ? sum / cnt : prev;  // an empty ring changes nothing
    a.dw[i] = wi - prev;
    prev = wi;
  }
  a.mass = mass;
  return 0;
}

hipError_t cake_launch_query(const CakeArgs& a, hipStream_t s) {
  const long threads = (long)a.n * a.g.B;
  if (threads <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_cake_one<CakeArgs, cake_query_body>), dim3((unsigned)((threads + WG - 1) / WG)),
                     dim3(WG), 0, s, a);
  return hipGetLastError();
}

hipError_t cake_launch_match(const CakeArgs& a, hipStream_t s) {
  const long waves = (long)a.nbx * (a.y1 - a.y0 + 1);
  if (waves <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_cake_one<CakeArgs, cake_match_body>), dim3((unsigned)((waves + WPB - 1) / WPB)),
                     dim3(WG), 0, s, a);
  return hipGetLastError();
}

hipError_t brute_launch_match(const BruteArgs& a, hipStream_t s) {
  const long blocks = (long)a.nbx * (a.y1 - a.y0 + 1);
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_brute_one<BruteArgs, brute_body>), dim3((unsigned)blocks), dim3(64),
                     (size_t)a.B * 64 * sizeof(uint32_t), s, a);
  return hipGetLastError();
}

}  // namespace swih
