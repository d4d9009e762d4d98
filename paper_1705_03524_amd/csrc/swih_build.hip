// Launchers of the weighted integral histogram build (Sec. 2.1, Eq. 2): one
// plane set per launch sequence, or every unit of a batch per stage launch.
// The stage bodies and their description are in swih_build_bodies.h.
#include <string.h>

#include "swih_build_bodies.h"

namespace swih {
namespace {

// Every stage is a device body over (arguments, virtual block).  One plane set
// launches it with one block per virtual block; a batch runs all units'
// virtual blocks in one grid-stride launch, each block finding its unit by
// binary search over the prefix of block counts.
template <Body BODY>
__global__ __launch_bounds__(WG) void k_single(BuildArgs a) {
  BODY(a, (int)blockIdx.x);
}

template <Body BODY>
__global__ __launch_bounds__(WG) void k_batch(const BuildArgs* __restrict__ units,
                                              const int32_t* __restrict__ prefix, int nunits) {
  const int total = prefix[nunits];
  for (int vb = (int)blockIdx.x; vb < total; vb += (int)gridDim.x) {
    int lo = 0, hi = nunits - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (prefix[mid] <= vb) lo = mid; else hi = mid - 1;
    }
    BODY(units[lo], vb - prefix[lo]);
  }
}

template <class ST>
hipError_t run_single(const BuildArgs& a, const int32_t (&nb)[4], int phases, hipStream_t s) {
  if (phases & 1) {
    if constexpr (ST::basis != nullptr)
      hipLaunchKernelGGL(k_single<ST::basis>, dim3(nb[0]), dim3(WG), 0, s, a);
    hipLaunchKernelGGL(k_single<ST::agg>, dim3(nb[1]), dim3(WG), a.agg_hist ? ST::agg_lds(a.g.B) : 0,
                       s, a);
    hipLaunchKernelGGL(k_single<ST::scan>, dim3(nb[2]), dim3(WG), 0, s, a);
  }
  if (phases & 2) {
    if (a.nt_planes)
      hipLaunchKernelGGL(k_single<ST::emit_nt>, dim3(nb[3]), dim3(WG), 0, s, a);
    else
      hipLaunchKernelGGL(k_single<ST::emit>, dim3(nb[3]), dim3(WG), 0, s, a);
  }
  return hipGetLastError();
}

template <class ST>
hipError_t run_batch(const BuildArgs* units, const int32_t* prefix, int nunits, int nbins,
                     const int32_t (&total)[4], int grid, hipStream_t s) {
  const int32_t* pre[4];
  for (int k = 0; k < 4; ++k) pre[k] = prefix + (size_t)k * (nunits + 1);
  auto g = [&](int k) { return dim3((unsigned)(total[k] < grid ? (total[k] > 0 ? total[k] : 1) : grid)); };
  if constexpr (ST::basis != nullptr)
    hipLaunchKernelGGL(k_batch<ST::basis>, g(0), dim3(WG), 0, s, units, pre[0], nunits);
  hipLaunchKernelGGL(k_batch<ST::agg>, g(1), dim3(WG), ST::agg_lds(nbins), s, units, pre[1], nunits);
  hipLaunchKernelGGL(k_batch<ST::scan>, g(2), dim3(WG), 0, s, units, pre[2], nunits);
  hipLaunchKernelGGL(k_batch<ST::emit_batch>, g(3), dim3(WG), 0, s, units, pre[3], nunits);
  return hipGetLastError();
}

#define SWIH_STAGE_DISPATCH(KIND, NTV, CALL)       \
  switch (KIND) {                                  \
    case 0: return CALL(IntStages<0>);             \
    case 1: return CALL(IntStages<1>);             \
    case 2: return CALL(IntStages<2>);             \
    case 3:                                        \
      switch (NTV) {                               \
        case 3: return CALL(GaussStages<3>);       \
        case 5: return CALL(GaussStages<5>);       \
        case 7: return CALL(GaussStages<7>);       \
        case 9: return CALL(GaussStages<9>);       \
        case 11: return CALL(GaussStages<11>);     \
        case 13: return CALL(GaussStages<13>);     \
        case 15: return CALL(GaussStages<15>);     \
        case 17: return CALL(GaussStages<17>);     \
        default: return hipErrorInvalidValue;      \
      }                                            \
    default: return hipErrorInvalidValue;          \
  }

}  // namespace

// A plane set alone uses the histogram aggregate from this many (band, tile)
// blocks up; below it the wave per (band, tile, bin) form keeps more of the
// chip busy (512 x 512, 16 bins: 5.4 against 5.9 us).
constexpr int kHistMinTiles = 128;
// Gaussian plane sets from this size on are stored non-temporally (about the
// device's last-level cache, 256 MB).
constexpr int64_t kNtPlaneBytes = 256ll << 20;

void build_args(const SwihLayout& L, int set, const GaussAxis* ax, const GaussAxis* ay, int32_t rx,
                int32_t ry, const uint8_t* img, int32_t img_pitch, char* ws, BuildArgs& a,
                int32_t (&nb)[4], bool batched) {
  const SwihGeom& g = L.g;
  memset(&a, 0, sizeof(a));
  a.g = g;
  a.img = img;
  a.ipitch = img_pitch;
  char* sb = ws + (size_t)set * L.set_bytes;
  a.planes = sb + L.off_planes;
  if (g.gauss) {
    a.RC = (double*)(sb + L.off_RC);
    a.XC = (float*)(sb + L.off_XC);
    a.beta = (double*)(sb + L.off_beta);
    a.uq = (int32_t*)(sb + L.off_uq);
    a.vq = (int32_t*)(sb + L.off_vq);
    a.vqd = (double*)(sb + L.off_vq + swih_align256((int64_t)g.nJ * g.H * 4));
    a.acc = (int32_t*)(sb + L.off_acc);
    a.nacc = (int64_t)g.H * g.W;
    a.ax = *ax;
    a.ay = *ay;
    a.rx = rx;
    a.ry = ry;
  }
  // planes larger than the last-level cache stream to HBM past it: left in it,
  // their write-back competes with the next launches' reads.  A single set's
  // launch picks its emit by this; batched builds always stream (a batch is
  // planned to fill the device's memory).
  const int64_t plane_bytes = (int64_t)g.nPL * g.B * g.NTX * (g.H + 1) * SWIH_TX * 4;
  a.nt_planes = plane_bytes >= kNtPlaneBytes;
  a.z = sb + L.off_z;
  a.T = sb + L.off_T;
  a.BT = sb + L.off_CT;
  const int NXP = g.NTX * SWIH_TX;
  a.nb1 = g.gauss ? 0 : blocks_for_threads((long)g.nJ * g.B * NXP);
  a.nb2 = blocks_for_threads((long)g.nI * g.B * g.H);
  const int nb3 = blocks_for_waves((long)g.nP * g.B);
  const long waves = (long)g.NTY * g.NTX * g.B;
  nb[0] = g.gauss ? blocks_for_threads((long)g.nI * NXP + (long)g.nJ * g.H + 2L * g.nJ * (g.H + 1) + a.nacc)
                  : 0;
  // integer kernels with few bins: a block per (band, tile) counts all bins
  a.agg_hist = !g.gauss && int_hist(g.nI - 1, g.B) && (batched || g.NTY * g.NTX >= kHistMinTiles);
  nb[1] = a.agg_hist ? g.NTY * g.NTX : blocks_for_waves(waves);
  nb[2] = a.nb1 + a.nb2 + nb3;
  nb[3] = blocks_for_waves(waves * (g.gauss ? 2 : 1));  // Gaussian: a plane wave + a row-carry wave
}

hipError_t launch_build(const SwihLayout& L, int kind, int set, const GaussAxis* ax,
                        const GaussAxis* ay, int32_t rx, int32_t ry, const uint8_t* img,
                        int32_t img_pitch, char* ws, hipStream_t stream, int phases) {
  BuildArgs a;
  int32_t nb[4];
  build_args(L, set, ax, ay, rx, ry, img, img_pitch, ws, a, nb);
#define SWIH_RUN1(ST) run_single<ST>(a, nb, phases, stream)
  SWIH_STAGE_DISPATCH(kind, L.g.nI, SWIH_RUN1)
#undef SWIH_RUN1
}

hipError_t launch_build_batch(int kind, int nt, int nbins, const BuildArgs* units,
                              const int32_t* prefix, int nunits, const int32_t (&total)[4], int grid,
                              hipStream_t stream) {
  if (nunits <= 0) return hipSuccess;
#define SWIH_RUNB(ST) run_batch<ST>(units, prefix, nunits, nbins, total, grid, stream)
  SWIH_STAGE_DISPATCH(kind, nt, SWIH_RUNB)
#undef SWIH_RUNB
}

}  // namespace swih
