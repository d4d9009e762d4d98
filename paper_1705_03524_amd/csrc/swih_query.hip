// Launchers of the window-histogram queries and likelihood maps (Sec. 2.1,
// Sec. 4): single requests, batches, and the map sweep's planner.  The device
// bodies and the description of the lookups are in swih_query_bodies.h.
#include <string.h>

#include <algorithm>
#include <mutex>

#include "swih_query_bodies.h"

namespace swih {

// Every map and query is a device body over (arguments, virtual block).  A
// single request launches one block per virtual block; a batch runs all
// requests' virtual blocks in one grid-stride launch, each block finding its
// request by binary search over the prefix of block counts.
template <class A, void (*BODY)(const A&, int)>
__global__ __launch_bounds__(1024) void k_one(A a) {
  BODY(a, (int)blockIdx.x);
}

// A single map's sweep: one block per item, renumbered so that each XCD
// (workgroups go to the 8 XCDs round robin) runs a contiguous range of items,
// i.e. the combs of one (bin group, chunk, segment) together, and the band-
// closing rows they share stay in that XCD's L2.  Up to 170 registers: three
// waves per SIMD, one block of twelve waves per compute unit.
template <int NT>
__global__ __launch_bounds__(768, 3) void k_sweep(MatchArgs a) {
  const int n = (int)gridDim.x, base = n >> 3, rem = n & 7;
  const int x = (int)blockIdx.x & 7, k = (int)blockIdx.x >> 3;
  match_gauss_sweep<NT>(a, x * base + (x < rem ? x : rem) + k);
}

// The batched sweep, with the register budget of k_sweep.
template <void (*BODY)(const MatchArgs&, int)>
__global__ __launch_bounds__(768, 3) void k_many_sweep(const MatchArgs* __restrict__ items,
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
hipError_t run_many(const A* items, const int32_t* prefix, int n, unsigned grid, const Launch& ml,
                    hipStream_t s) {
  hipLaunchKernelGGL((k_many<A, BODY>), dim3(grid), dim3((unsigned)ml.threads), ml.lds, s, items,
                     prefix, n);
  return hipGetLastError();
}

template <int K> constexpr void (*int_match)(const MatchArgs&, int) = match_int<K>;
template <int K> constexpr void (*int_query)(const QueryArgs&, int) = query_int<K>;
template <int NT> constexpr void (*gauss_match)(const MatchArgs&, int) = match_gauss_sweep<NT>;
template <int NT> constexpr void (*gauss_query)(const QueryArgs&, int) = query_gauss<NT>;

// switch over kernel kind (and Gaussian term count) calling CALL(body)
#define SWIH_NT_CASES(CALL)          \
  switch (nt) {                      \
    case 3: return CALL(3);          \
    case 5: return CALL(5);          \
    case 7: return CALL(7);          \
    case 9: return CALL(9);          \
    case 11: return CALL(11);        \
    case 13: return CALL(13);        \
    case 15: return CALL(15);        \
    case 17: return CALL(17);        \
    default: return hipErrorInvalidValue; \
  }

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

// Integer-kernel maps; Gaussian maps go through the sweep launches.
hipError_t match_one(int kind, const MatchArgs& a, const Launch& ml, hipStream_t s) {
  switch (kind) {
    case 0: return run_one<MatchArgs, int_match<0>>(a, ml, s);
    case 1: return run_one<MatchArgs, int_match<1>>(a, ml, s);
    case 2: return run_one<MatchArgs, int_match<2>>(a, ml, s);
    default: return hipErrorInvalidValue;
  }
}

template <void (*BODY)(const MatchArgs&, int)>
hipError_t run_many_sweep(const MatchArgs* items, const int32_t* prefix, int n, unsigned grid,
                          const Launch& ml, hipStream_t s) {
  hipLaunchKernelGGL(k_many_sweep<BODY>, dim3(grid), dim3((unsigned)ml.threads), ml.lds, s, items,
                     prefix, n);
  return hipGetLastError();
}

hipError_t match_many(int kind, int nt, const MatchArgs* jobs, const int32_t* prefix, int n,
                      unsigned grid, const Launch& ml, hipStream_t s) {
#define SWIH_I(K) int_match<K>
#define SWIH_G(NT) gauss_match<NT>
#define SWIH_C(B) run_many<MatchArgs, B>(jobs, prefix, n, grid, ml, s)
#define SWIH_CG(NT) run_many_sweep<gauss_match<NT>>(jobs, prefix, n, grid, ml, s)
  if (kind == 3) {
    SWIH_NT_CASES(SWIH_CG)
  }
  switch (kind) {
    case 0: return SWIH_C(SWIH_I(0));
    case 1: return SWIH_C(SWIH_I(1));
    case 2: return SWIH_C(SWIH_I(2));
    default: return hipErrorInvalidValue;
  }
#undef SWIH_CG
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

namespace {

constexpr int kSweepMaxTiles = 12;     // waves of a sweep block: 768 threads
constexpr int kSweepBatchS = 16;       // members per segment in batches
constexpr size_t kLdsMax = 160 * 1024;

// LDS of a sweep block: G+, G-, N double-buffered, beta of the members, and
// (unless each item holds one bin of several groups) the (member, window)
// accumulators.
size_t sweep_lds(int nt, int S, int NT, int cw, bool direct) {
  return sizeof(double) * (6 * 64 * (size_t)nt + (size_t)S * NT) +
         (direct ? 0 : sizeof(int32_t) * (size_t)S * cw);
}

// Tiles (waves) a chunk of window centres [xs, xe] needs: one contiguous range
// from the first left edge to the last right edge, or (two) the left-edge
// tiles and the right-edge tiles apart.
int sweep_tiles(int xs, int xe, int rx, bool two) {
  const int ta = (std::max(xs - rx, 1) - 1) >> 6, tb = (xe + rx) >> 6;
  if (!two) return tb - ta + 1;
  const int tla = (std::max(xe - rx, 1) - 1) >> 6, trb = (xs + rx) >> 6;
  return (tla - ta + 1) + (tb - trb + 1);
}

// Column chunks: the split with the fewest tile reads whose chunks all fit a block.
void sweep_chunks(int x0, int nx, int rx, MatchArgs& a, int& two) {
  long best = -1;
  for (int t = 0; t < 2; ++t) {
    for (int nch = 1; nch <= nx; ++nch) {
      const int cw = (nx + nch - 1) / nch, n = (nx + cw - 1) / cw;
      int nt = 0;
      for (int c = 0; c < n; ++c) {
        const int xs = x0 + c * cw, xe = std::min(xs + cw - 1, x0 + nx - 1);
        nt = std::max(nt, sweep_tiles(xs, xe, rx, t == 1));
      }
      if (nt > kSweepMaxTiles) continue;
      const long cost = (long)n * nt;
      if (best < 0 || cost < best) {
        best = cost;
        a.nch = n;
        a.cw = cw;
        a.nt = nt;
        two = t;
      }
      break;  // more chunks only add overlap
    }
  }
}

int device_cus() {
  static int cus[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cus[dev] = n;
  }
  return cus[dev];
}

}  // namespace

// Plan of a Gaussian comb sweep over the centre rectangle: chunks, combs,
// segments and bin groups, and the launch shape.  cus == 0: the batch form
// (one bin group, segments of up to kSweepBatchS members).  Otherwise the
// split that minimises a model of the time on `cus` compute units: rounds of
// blocks times the work of one block (bins x tiles x rows read, crossings
// counted at a quarter since neighbouring combs share them in L2), with a
// small charge for the accumulator pass of several bin groups.
static void sweep_plan(const ScaleParams& sp, int B, int NT, int x0, int nx, int ny, int cus,
                       MatchArgs& a, Launch& ml) {
  int two = 0;
  sweep_chunks(x0, nx, sp.rx, a, two);
  a.two = two;
  const int h = 2 * sp.ry + 1;
  a.ncomb = std::min(h, ny);
  const int Mq = (ny + h - 1) / h;
  auto smax = [&](int S, bool direct) {
    while (S > 1 && sweep_lds(a.nt, S, NT, a.cw, direct) > kLdsMax) --S;
    return S;
  };
  if (cus <= 0) {
    a.S = smax(std::min(Mq, kSweepBatchS), false);
    a.nseg = (Mq + a.S - 1) / a.S;
    a.ngroups = 1;
    a.bpg = B;
  } else {
    const int bpc0 = std::max(1, 12 / a.nt);  // three waves per SIMD (register budget)
    double best = -1.0;
    for (int bpg = B; bpg >= 1; bpg = bpg > 1 ? (bpg + 1) / 2 : 0) {
      const int ng = (B + bpg - 1) / bpg;
      const bool direct = ng > 1 && bpg == 1;
      const int Slim = smax(Mq, direct);
      for (int nseg = (Mq + Slim - 1) / Slim; nseg <= Mq; ++nseg) {
        const int S = (Mq + nseg - 1) / nseg;
        const size_t lds = sweep_lds(a.nt, S, NT, a.cw, direct);
        const int bpc = std::max(1, std::min(bpc0, (int)(kLdsMax / lds)));
        const long items = (long)ng * a.nch * nseg * a.ncomb;
        const long rounds = (items + (long)cus * bpc - 1) / ((long)cus * bpc);
        const double rows = S + 1 + 0.25 * S * (double)(h - 1) / 64.0;
        // several bin groups: the accumulator's read-modify-write traffic
        const double t = (double)rounds * bpc * bpg * a.nt * rows * (ng > 1 ? 1.04 : 1.0);
        if (best < 0 || t < best * 0.999) {
          best = t;
          a.S = S;
          a.nseg = nseg;
          a.ngroups = ng;
          a.bpg = bpg;
        }
        if (S == 1) break;
      }
      if (bpg == 1) break;
    }
  }
  ml.blocks = a.ngroups * a.nch * a.nseg * a.ncomb;
  ml.threads = 64 * a.nt;
  ml.lds = sweep_lds(a.nt, a.S, NT, a.cw, a.ngroups > 1 && a.bpg == 1);
}

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
  // Gaussian: the comb sweep, one bin group, segments of up to kSweepBatchS
  // members (the form batches use; a single map picks its own split).
  sweep_plan(sp, L.g.B, L.g.nI, x0, nx, ny, 0, a, ml);
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
    ql.lds = sizeof(double) * (size_t)L.g.B * (2 * L.g.nJ + 1);
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

constexpr void (*gauss_fin)(const MatchArgs&, int) = match_gauss_fin;

template <int NT>
hipError_t run_sweep(const MatchArgs& a, const Launch& ml, hipStream_t s) {
  hipLaunchKernelGGL(k_sweep<NT>, dim3((unsigned)ml.blocks), dim3((unsigned)ml.threads), ml.lds, s, a);
  return hipGetLastError();
}

hipError_t sweep_one(int nt, const MatchArgs& a, const Launch& ml, hipStream_t s) {
  switch (nt) {
    case 3: return run_sweep<3>(a, ml, s);
    case 5: return run_sweep<5>(a, ml, s);
    case 7: return run_sweep<7>(a, ml, s);
    case 9: return run_sweep<9>(a, ml, s);
    case 11: return run_sweep<11>(a, ml, s);
    case 13: return run_sweep<13>(a, ml, s);
    case 15: return run_sweep<15>(a, ml, s);
    case 17: return run_sweep<17>(a, ml, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// Scratch of swih_match_noalloc: the integer accumulator of a Gaussian map
// whose plan has several bin groups, kept with the code object on every
// device the library runs on, so that the call allocates nothing.
static __device__ __align__(256) int32_t scratch[kNoallocCentres];

namespace {

std::mutex g_scratch_mu;
int32_t* g_scratch_ptr[64];  // device address of each device's copy

__global__ void k_zero_i32(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

}  // namespace

int32_t* noalloc_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = (int32_t*)p;
  }
  return g_scratch_ptr[dev];
}

hipError_t launch_match(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                        const float* tmpl, const uint32_t* tmpl_raw, int32_t x0, int32_t y0,
                        int32_t x1, int32_t y1, float* map, hipStream_t s, int32_t* acc) {
  if (x1 < x0 || y1 < y0) return hipSuccess;
  MatchArgs a;
  Launch ml;
  match_args(L, sp, set, ws, tmpl, tmpl_raw, x0, y0, x1, y1, map, a, ml);
  if (!L.g.gauss) return match_one(sp.kind, a, ml, s);
  // Gaussian: the split that fills this device; several bin groups add
  // into the set's accumulator, which the finalising pass turns into the map.
  sweep_plan(sp, L.g.B, L.g.nI, x0, x1 - x0 + 1, y1 - y0 + 1, device_cus(), a, ml);
  if (ml.lds > kLdsMax) return hipErrorInvalidValue;
  if (acc && a.ngroups > 1) {
    // an outside accumulator must start at zero (the finalising pass leaves it so)
    const int64_t n = (int64_t)(x1 - x0 + 1) * (y1 - y0 + 1);
    hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256),
                       0, s, acc, n);
    a.acc = acc;
  } else {
    a.acc = (int32_t*)(ws + (size_t)set * L.set_bytes + L.off_acc);
  }
  hipError_t e = sweep_one(L.g.nI, a, ml, s);
  if (e != hipSuccess || a.ngroups == 1) return e;
  Launch fl;
  fl.threads = 256;
  fl.blocks = (int32_t)(((long)(x1 - x0 + 1) * (y1 - y0 + 1) + 255) / 256);
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
