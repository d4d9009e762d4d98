// One persistent launch for a whole batch of uneven frames, crops and scales
// (Sec. 4: many targets over many frames): every plane set's build (basis,
// aggregate, scan, emit), the template queries and the likelihood maps.
//
// Work.  Each stage of each unit (plane set), query job and map job is a list
// of virtual blocks; the tickets number them stage by stage, in the order
// basis, aggregate, scan, emit, query, map, and units in batch order within a
// stage.  A block takes the next ticket from one atomic counter, finds its
// stage and item by binary search over the prefixes, waits until the stage
// before it is complete for the same unit (a query: that unit's emit; a map:
// its unit's emit and every query, since templates may come from queries of
// the same batch), runs the stage's body, and counts the virtual block as
// finished for its unit.
//
// Progress.  Tickets are taken in increasing order, so every ticket a block
// waits on was taken earlier by a block that is running; the smallest
// unfinished ticket waits on nothing unfinished, so the launch always drains.
// Every wait is still bounded in time: past the bound the block records a
// nonzero status and goes on, so the launch ends whatever happens.
//
// Memory.  Counters are agent-scope.  A finished ticket is not counted at
// once: a block keeps up to four finished tickets pending and publishes them
// together -- every wave waits for its stores, then one wave writes the XCD's
// L2 back (the release) and moves the counters -- before it ever waits, when
// the list is full and when it leaves a loop; so no block waits while holding
// unpublished work, and a release covers several tickets.  The ticket that
// completes a (stage, unit) stamps it from a completion clock.  A waiting
// block acquires (invalidates its L2: the stage's inputs were written by other
// XCDs, whose L2s are separate) unless every stamp it depends on is older than
// its last acquire, which already made that data visible.
//
// Reset.  The last block to leave resets the counters, so the table can be
// launched again; the status word (and the caller's copy) reports whether
// every wait was met.
#include <string.h>

#include "swih_build_bodies.h"
#include "swih_query_bodies.h"

namespace swih {
namespace {

__device__ __forceinline__ int32_t ld_agent(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until *p >= need for at most `limit` ticks of the constant-rate clock.
// False if it gave up.  Once any wait of the launch has given up (*failed set)
// the others give up too, so a failing launch still ends within about one
// bound; limit < 0 gives up without looking (the host's way to exercise the
// failure path).
__device__ bool wait_count(const int32_t* p, int32_t need, int64_t limit, const int32_t* failed) {
  if (limit < 0) return false;
  if (ld_agent(p) >= need) return true;
  const int64_t t0 = wall_clock64();
  while (ld_agent(p) < need) {
    __builtin_amdgcn_s_sleep(8);
    if (ld_agent(failed) != 0 || wall_clock64() - t0 > limit) return ld_agent(p) >= need;
  }
  return true;
}

// Index i of prefix[0..n] with prefix[i] <= v < prefix[i + 1] (the last such
// when items have no virtual blocks).
__device__ __forceinline__ int find_item(const int32_t* __restrict__ prefix, int n, int v) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Tickets are claimed in runs (one atomic on the shared counter per run) and
// run in order; a block's run holds no ticket that a smaller ticket of its own
// waits on, so the drain argument is unchanged.  A run is long while many
// tickets remain per block (the shared counter is then the bottleneck) and
// shrinks to one toward the end, so that the last tickets spread over the
// device.
constexpr int kClaimMax = 16;

// The next ticket, block-uniform (readfirstlane says so, which keeps the
// decode, the item's arguments and every index derived from them scalar).
// Every caller passes a barrier before the next call rewrites s_ticket.
__device__ __forceinline__ int next_ticket(const FusedArgs& f, int32_t& s_ticket, int& lo, int& hi) {
  if (lo < hi) return lo++;
  // tickets left per block (as of this block's last claim), an eighth of it per run
  const int left = (f.cum[6] - hi) / (int)gridDim.x;
  const int run = max(1, min(kClaimMax, left >> 3));
  if (threadIdx.x == 0)
    s_ticket = __hip_atomic_fetch_add(f.sync, run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  lo = __builtin_amdgcn_readfirstlane(s_ticket);
  hi = lo + run;
  return lo++;
}

// ST: the four build stages (basis may be null); QB, MB: query and map bodies.
// Tickets come in stage order, so each block runs three loops in turn (builds,
// queries, maps): the query and map bodies' registers are allocated apart
// from the build bodies'.
template <int WGT, class ST, void (*QB)(const QueryArgs&, int), void (*MB)(const MatchArgs&, int)>
__device__ __forceinline__ void fused_loop(const FusedArgs& f) {
  constexpr int kPend = 4;
  __shared__ int32_t s_ticket, s_flag;
  const int nu = f.nunits;
  int32_t* __restrict__ done = f.sync + kFusedSyncHead;  // [4][nunits] finished tickets
  int32_t* __restrict__ stamp = done + 4 * nu;           // [4][nunits] completion stamps
  int32_t* const qdone = f.sync + 3;
  int32_t* const clock = f.sync + 4;
  int32_t* const qstamp = f.sync + 5;
  const int tid = (int)threadIdx.x;
  // tickets needed to finish (stage s < 4, unit u); the queries: s = 4
  auto need = [&](int s, int u) {
    if (s == 4) return f.cum[5] - f.cum[4];
    const int32_t* up = f.upre + (size_t)s * (nu + 1);
    return up[u + 1] - up[u];
  };
  // finished tickets not yet published: s * nunits + u, or -1 for a query
  int pend[kPend];
  int npend = 0;
  auto publish = [&]() {
    if (npend == 0) return;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores are done
    __syncthreads();
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // write the L2 back
      for (int k = 0; k < npend; ++k) {
        const int key = pend[k];
        const int s = key < 0 ? 4 : key / nu, u = key < 0 ? 0 : key - (key / nu) * nu;
        int32_t* c = key < 0 ? qdone : done + key;
        if (__hip_atomic_fetch_add(c, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 == need(s, u)) {
          const int32_t st =
              __hip_atomic_fetch_add(clock, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
          __hip_atomic_store(key < 0 ? qstamp : stamp + key, st, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    npend = 0;
  };
  auto finished = [&](int key) {
    pend[npend++] = key;
    if (npend == kPend) publish();
  };
  // the clock value read just before this block's last acquire: everything
  // stamped at or below it is visible to the block
  int32_t seen = 0;
  int held_stage = -1, held_unit = -1;  // a later ticket of the same pair needs nothing
  // wait until stage dep of unit is complete (and, for a map, every query)
  auto gate = [&](int s, int dep, int unit) {
    if (held_stage == s && held_unit == unit) return;
    if (s < 5 && need(dep, unit) == 0) return;  // nothing was written for it
    publish();  // never wait holding unpublished work
    if (tid == 0) {
      bool ok = wait_count(done + (size_t)dep * nu + unit, need(dep, unit), f.limit, f.sync + 2);
      if (s == 5) ok = wait_count(qdone, need(4, 0), f.limit, f.sync + 2) && ok;
      if (!ok) __hip_atomic_store(f.sync + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // a stamp not yet written reads 0: acquire then too
      const int32_t a = ld_agent(stamp + (size_t)dep * nu + unit);
      const int32_t b = s == 5 ? ld_agent(qstamp) : 1;
      const bool fresh = ok && a > 0 && a <= seen && b > 0 && b <= seen;
      s_flag = fresh ? -1 : ld_agent(clock);
    }
    __syncthreads();
    const int32_t c0 = __builtin_amdgcn_readfirstlane(s_flag);
    if (c0 >= 0) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      seen = c0;
    }
    held_stage = s;
    held_unit = unit;
  };
  int tlo = 0, thi = 0;  // the rest of this block's claimed run
  int t = next_ticket(f, s_ticket, tlo, thi);
  // builds
  while (t < f.cum[4]) {
    int s = 0;
    while (t >= f.cum[s + 1]) ++s;
    const int local = t - f.cum[s];
    const int32_t* pre = f.upre + (size_t)s * (nu + 1);
    const int unit = __builtin_amdgcn_readfirstlane(find_item(pre, nu, local));
    const int vb = __builtin_amdgcn_readfirstlane(local - pre[unit]);
    if (s > 0) gate(s, s - 1, unit);
    switch (s) {
      case 0:
        if constexpr (ST::basis != nullptr) ST::basis(f.units[unit], vb);
        break;
      case 1: ST::agg(f.units[unit], vb); break;
      case 2: ST::scan(f.units[unit], vb); break;
      default: ST::emit(f.units[unit], vb); break;
    }
    finished(s * nu + unit);
    t = next_ticket(f, s_ticket, tlo, thi);
  }
  // template queries
  while (t < f.cum[5]) {
    const int local = t - f.cum[4];
    const int item = __builtin_amdgcn_readfirstlane(find_item(f.qpre, f.nq, local));
    const int vb = __builtin_amdgcn_readfirstlane(local - f.qpre[item]);
    gate(4, 3, __builtin_amdgcn_readfirstlane(f.qunit[item]));
    QB(f.q[item], vb);
    finished(-1);
    t = next_ticket(f, s_ticket, tlo, thi);
  }
  publish();
  // maps: nothing waits on them
  while (t < f.cum[6]) {
    const int local = t - f.cum[5];
    const int item = __builtin_amdgcn_readfirstlane(find_item(f.mpre, f.nm, local));
    const int vb = __builtin_amdgcn_readfirstlane(local - f.mpre[item]);
    gate(5, 3, __builtin_amdgcn_readfirstlane(f.munit[item]));
    MB(f.m[item], vb);
    __syncthreads();
    t = next_ticket(f, s_ticket, tlo, thi);
  }
  // leave; the last block out resets the counters for the next launch
  if (tid == 0)
    s_flag = __hip_atomic_fetch_add(f.sync + 1, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
             (int32_t)gridDim.x - 1;
  __syncthreads();
  if (!s_flag) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  for (int i = tid; i < 8 * nu; i += WGT) done[i] = 0;
  if (tid == 0) {
    if (f.status) *f.status = f.sync[2];
    for (int k = 0; k < kFusedSyncHead; ++k) f.sync[k] = 0;
  }
}

template <int KIND>
__global__ __launch_bounds__(256) void k_fused_int(FusedArgs f) {
  fused_loop<256, IntStages<KIND>, query_int<KIND>, match_int<KIND>>(f);
}

// The sweep's block (twelve waves) and register budget (three waves per SIMD).
template <int NT>
__global__ __launch_bounds__(768, 3) void k_fused_gauss(FusedArgs f) {
  fused_loop<768, GaussStagesW<NT, 768>, query_gauss<NT>, match_gauss_sweep<NT>>(f);
}

template <class K>
hipError_t run_fused(K kernel, int threads, size_t lds, const FusedArgs& f, hipStream_t s) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return hipErrorInvalidValue;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, lds) != hipSuccess ||
      per < 1)
    return hipErrorInvalidValue;
  // never more blocks than tickets; all of them resident at once
  const long want = (long)per * cus;
  const unsigned grid = (unsigned)(f.cum[6] < want ? (f.cum[6] > 0 ? f.cum[6] : 1) : want);
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), lds, s, f);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fused(int kind, int nt, int nbins, const FusedArgs& f, size_t dyn_lds,
                        hipStream_t stream) {
  if (kind <= 2) {
    // the histogram aggregate's LDS when the batch's bins allow it
    const size_t agg = int_hist(kind, nbins) ? (size_t)hist_lds_bytes(kind, nbins) : 0;
    const size_t lds = dyn_lds > agg ? dyn_lds : agg;
    switch (kind) {
      case 0: return run_fused(k_fused_int<0>, 256, lds, f, stream);
      case 1: return run_fused(k_fused_int<1>, 256, lds, f, stream);
      default: return run_fused(k_fused_int<2>, 256, lds, f, stream);
    }
  }
  if (kind != 3) return hipErrorInvalidValue;
  switch (nt) {
    case 3: return run_fused(k_fused_gauss<3>, 768, dyn_lds, f, stream);
    case 5: return run_fused(k_fused_gauss<5>, 768, dyn_lds, f, stream);
    case 7: return run_fused(k_fused_gauss<7>, 768, dyn_lds, f, stream);
    case 9: return run_fused(k_fused_gauss<9>, 768, dyn_lds, f, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace swih
