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

// Build: integer kernels write one global plane set; the Gaussian writes set
// `set` with the axis series of that scale.
// phase bit 1 = carries (aggregate + scan), bit 2 = planes (emit).
hipError_t launch_build(const SwihLayout& L, int kind, int set, const GaussAxis* ax,
                        const GaussAxis* ay, const uint8_t* img, int32_t img_pitch, char* ws,
                        hipStream_t stream, int phases = 3);

hipError_t launch_query(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                        const int32_t* centres, int32_t n, float* hist, uint32_t* hist_raw,
                        hipStream_t stream);

hipError_t launch_match(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                        const float* tmpl, const uint32_t* tmpl_raw, int32_t x0, int32_t y0,
                        int32_t x1, int32_t y1, float* map, hipStream_t stream);

}  // namespace swih
