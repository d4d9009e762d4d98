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

// A single map's sweep: one block of four waves per item, renumbered so that
// each XCD (workgroups go to the 8 XCDs round robin) runs a contiguous range
// of items, i.e. neighbouring chunks of one (bin group, segment, comb)
// together, and the edge tiles and band-closing rows they share stay in that
// XCD's L2.
template <int NT>
__global__ __launch_bounds__(256, 4) void k_sweep(MatchArgs a) {
  const int n = (int)gridDim.x, base = n >> 3, rem = n & 7;
  const int x = (int)blockIdx.x & 7, k = (int)blockIdx.x >> 3;
  match_gauss_sweep<NT>(a, x * base + (x < rem ? x : rem) + k);
}

// The batched sweep: blocks of twelve waves (three per SIMD, up to 170 registers).
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

constexpr int kSweepWaves = 4;         // waves of a single map's sweep block
constexpr int kSweepBatchWaves = 12;   // waves of a batch's sweep block (the fused launch's shape)
constexpr int kSweepMaxS = 32;         // members per segment, single maps
constexpr int kSweepBatchS = 16;       // members per segment in batches
constexpr size_t kLdsMax = 160 * 1024;

// LDS of a sweep block: each wave's carry boxes of its three edge tiles (a
// double per lane) and its (member, window) accumulators.
size_t sweep_lds(int waves, int S) {
  return sizeof(double) * (size_t)waves * 64 + sizeof(int32_t) * (size_t)waves * S * 64;
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

// Plan of a Gaussian window sweep over the centre rectangle: chunks of 64
// windows per wave, combs, segments and bin groups, and the launch shape.
// cus == 0: the batch form (blocks of kSweepBatchWaves waves; chunks as wide
// as the job, and as many combs per block as such chunks fit; one bin group;
// segments of up to kSweepBatchS members).  Otherwise blocks of kSweepWaves,
// segments of up to kSweepMaxS members (a segment costs one opening row per
// bin), then bin groups (powers of two) until the launch has 128 waves per
// compute unit: many short waves hide the loads' latency and balance the
// device (2048 x 2048, 32 bins: 16 groups of 2 bins, 32 of 1 at side 63; the
// accumulator's atomics cost less than the waves gain).
static void sweep_plan(const ScaleParams& sp, int B, int NT, int x0, int nx, int ny, int cus,
                       MatchArgs& a, Launch& ml) {
  const int h = 2 * sp.ry + 1;
  // a batch job's chunk is as wide as the job, up to the batch block's waves;
  // a narrower job packs several combs into the block
  const int waves = cus > 0 ? kSweepWaves : std::min(kSweepBatchWaves, (nx + 63) / 64 + 1);
  a.nt = waves;
  a.cpb = cus > 0 ? 1 : kSweepBatchWaves / waves;
  a.cw = 64 * waves;
  // chunks start where a wave's right edges begin a tile (the sweep's xo)
  const int xo = x0 - ((x0 + sp.rx) & 63);
  a.nch = (x0 + nx - xo + a.cw - 1) / a.cw;
  a.ncomb = std::min(h, ny);
  const int Mq = (ny + h - 1) / h;
  const int smax = cus > 0 ? kSweepMaxS : kSweepBatchS;
  a.nseg = (Mq + smax - 1) / smax;
  a.S = (Mq + a.nseg - 1) / a.nseg;
  int ng = 1;
  if (cus > 0) {
    const long base = (long)a.nseg * a.ncomb * a.nch * waves;
    while (ng < B && base * ng < 128L * cus) ng *= 2;
  }
  a.bpg = (B + ng - 1) / ng;
  a.ngroups = (B + a.bpg - 1) / a.bpg;
  ml.blocks = a.ngroups * a.nch * a.nseg * ((a.ncomb + a.cpb - 1) / a.cpb);
  // batch items take the batch block whatever their width: the body lays its
  // LDS out by the launch's block size
  const int bw = cus > 0 ? waves : kSweepBatchWaves;
  ml.threads = 64 * bw;
  ml.lds = sweep_lds(bw, a.S);
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
  a.XC = L.g.gauss ? (const float*)(sb + L.off_XC) : nullptr;
  a.beta = L.g.gauss ? (const double*)(sb + L.off_beta) : nullptr;
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
  a.XC = L.g.gauss ? (const float*)(sb + L.off_XC) : nullptr;
  a.centres = centres;
  a.n = n;
  a.hist = hist;
  a.hist_raw = hist_raw;
  ql.threads = 256;
  if (L.g.gauss) {
    ql.blocks = n;
    ql.lds = sizeof(double) * (size_t)L.g.B * (L.g.nI + 3);
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
