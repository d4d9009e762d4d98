// Internal interface between the C ABI (swih_api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swih_layout.h"

#define SWIH_MAX_K 8

namespace swih {

// Host-side cosine-series fit (gauss_terms.cpp).
int gauss_fit(int n, int K, double* a_out, int* P_out, double* err_out);
double gauss_axis_mass(int n, int K, const double* a, int P);

// One axis of the Gaussian stand-in: g(t) = sum_k a[k] cos(2 pi k t / P).
struct GaussAxis {
  int32_t P;
  int32_t K;
  double a[SWIH_MAX_K + 1];
};

// Per-scale constants shared by query and match.
struct ScaleParams {
  int32_t w, h, rx, ry;
  int32_t kind;           // swih_kernel
  uint32_t c_int;         // Manhattan rx+ry+1, Euclidean rx^2+ry^2+1
  double mass;            // S (closed form; Gaussian: product of axis masses)
  GaussAxis ax, ay;       // Gaussian only
};

// Everything the build stages of one plane set read on the device.
struct BuildArgs {
  SwihGeom g;
  const uint8_t* img;
  int32_t ipitch;
  int32_t nb1, nb2;   // scan: blocks of the band-carry and tile-carry roles
  void* planes;       // uint32 (integer kernels) or float tile-local planes (Gaussian)
  double* RC;         // Gaussian row carries
  int32_t* uq;        // Gaussian x terms [x][i]
  int32_t* vq;        // Gaussian y terms [y][j]
  double* vqd;        // vq * 2^-48
  void* z;            // band column sums -> carry rows (integer kernels)
  void* T;            // row-segment sums -> row carries
  void* BT;           // tile totals -> tile-origin values
  GaussAxis ax, ay;
};

// Fill the arguments of one plane set; nb = blocks of the basis, aggregate,
// scan and emit stages.
void build_args(const SwihLayout& L, int set, const GaussAxis* ax, const GaussAxis* ay,
                const uint8_t* img, int32_t img_pitch, char* ws, BuildArgs& a, int32_t (&nb)[4]);

// One batched build: every stage in one grid-stride launch over the units.
// prefix: 4 arrays of nunits + 1 exclusive block prefixes (device memory, with
// the units); total: blocks per stage; grid: blocks per launch.
hipError_t launch_build_batch(int kind, int nt, const BuildArgs* units, const int32_t* prefix,
                              int nunits, const int32_t (&total)[4], int grid, hipStream_t stream);

// Build: integer kernels write one global plane set; the Gaussian writes set
// `set` with the axis series of that scale.
// phase bit 1 = carries (aggregate + scan), bit 2 = planes (emit).
hipError_t launch_build(const SwihLayout& L, int kind, int set, const GaussAxis* ax,
                        const GaussAxis* ay, const uint8_t* img, int32_t img_pitch, char* ws,
                        hipStream_t stream, int phases = 3);

hipError_t launch_query(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                        const int32_t* centres, int32_t n, float* hist, uint32_t* hist_raw,
                        hipStream_t stream);

// Everything one dense map reads on the device.
struct MatchArgs {
  SwihGeom g;
  ScaleParams sp;
  const void* planes;      // uint32 planes or float tile-local planes
  const double* RC;        // Gaussian row carries
  const float* tmpl;       // normalised template, or null
  const uint32_t* tmpl_raw;  // exact template (integer kernels), or null
  float* map;
  int32_t x0, y0, x1, y1;  // inclusive centre rectangle
  int32_t nbx;             // virtual blocks per row of blocks
  int32_t cw, nvpad, ntl_max;  // Gaussian: centres per block, columns per group, tile columns
};

struct Launch {
  int32_t blocks;    // virtual blocks
  int32_t threads;   // threads per block
  size_t lds;        // dynamic LDS bytes
};

// Everything one window-histogram query reads on the device.
struct QueryArgs {
  SwihGeom g;
  ScaleParams sp;
  const void* planes;
  const double* RC;
  const int32_t* centres;  // [n][2]
  int32_t n;
  float* hist;             // [n][B] or null
  uint32_t* hist_raw;      // [n][B] or null (integer kernels)
};

void query_args(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                const int32_t* centres, int32_t n, float* hist, uint32_t* hist_raw, QueryArgs& a,
                Launch& ql);

hipError_t launch_query_batch(int kind, int nt, const QueryArgs* jobs, const int32_t* prefix,
                              int njobs, const Launch& ql, int grid, hipStream_t stream);

void match_args(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                const float* tmpl, const uint32_t* tmpl_raw, int32_t x0, int32_t y0, int32_t x1,
                int32_t y1, float* map, MatchArgs& a, Launch& ml);

// One batched map launch over njobs (same kernel); ml: total virtual blocks,
// the largest block size and LDS of any job.
hipError_t launch_match_batch(int kind, int nt, const MatchArgs* jobs, const int32_t* prefix,
                              int njobs, const Launch& ml, int grid, hipStream_t stream);

hipError_t launch_match(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                        const float* tmpl, const uint32_t* tmpl_raw, int32_t x0, int32_t y0,
                        int32_t x1, int32_t y1, float* map, hipStream_t stream);

}  // namespace swih
