// Internal interface between the C ABI (swih_api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swih_layout.h"

#define SWIH_MAX_K 8
#define SWIH_DEFAULT_K 3  // free-frequency fit: worst 2-D histogram error ~4e-8

namespace swih {

// Host-side cosine-series fit (gauss_terms.cpp).
int gauss_fit(int n, int K, double* a_out, double* om_out, double* err_out);
double gauss_axis_mass(int n, int K, const double* a, const double* om);

// One axis of the Gaussian stand-in: g(t) = sum_k a[k] cos(om[k] t), om[0] = 0.
struct GaussAxis {
  int32_t K;
  int32_t pad;
  double a[SWIH_MAX_K + 1];
  double om[SWIH_MAX_K + 1];
};

// The series coefficients of one axis at centre coordinate c: (a_0,
// a_k cos(w_k c), a_k sin(w_k c)) for k = 1..K, NT = 2K + 1 of them -- the
// alpha (x) or beta (y) translation coefficients of Sec. 2.1.
template <int NT>
__device__ inline void series_coeffs(const GaussAxis& ax, int c, double (&out)[NT]) {
  out[0] = ax.a[0];
#pragma unroll
  for (int k = 1; k <= (NT - 1) / 2; ++k) {
    double s, co;
    sincos(ax.om[k] * (double)c, &s, &co);
    out[2 * k - 1] = ax.a[k] * co;
    out[2 * k] = ax.a[k] * s;
  }
}

// Coefficient j of series_coeffs at centre c, computed the same way.
__device__ inline double series_coeff(const GaussAxis& ax, int c, int j) {
  if (j == 0) return ax.a[0];
  const int k = (j + 1) / 2;
  double s, co;
  sincos(ax.om[k] * (double)c, &s, &co);
  return ax.a[k] * ((j & 1) ? co : s);
}

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
  double* RC;         // Gaussian row carries (y-contracted)
  float* XC;          // Gaussian band-closing rows
  double* beta;       // Gaussian: [H+1][2 nJ] beta of each row as a bottom / top edge
  int32_t* uq;        // Gaussian x terms [x][i]
  int32_t* vq;        // Gaussian y terms [y][j]
  double* vqd;        // vq * 2^-48
  void* z;            // band column sums -> carry rows (integer kernels)
  void* T;            // row-segment sums -> row carries
  void* BT;           // tile totals -> tile-origin values
  int32_t* acc;       // Gaussian: the map accumulator of the set, cleared by the build
  int64_t nacc;
  int32_t agg_hist;   // integer kernels: aggregate by LDS histograms, a block per (band, tile)
  int32_t rx, ry;     // Gaussian: the set's window half-sizes (corner coefficients of the planes)
  int32_t nt_planes;  // single-set launch: store the planes non-temporally (256 MB and more)
  GaussAxis ax, ay;
};

// Fill the arguments of one plane set; nb = blocks of the basis, aggregate,
// scan and emit stages.  `batched`: the set is one unit of a batched build
// (its aggregate may then use the histogram form at any size).
void build_args(const SwihLayout& L, int set, const GaussAxis* ax, const GaussAxis* ay, int32_t rx,
                int32_t ry, const uint8_t* img, int32_t img_pitch, char* ws, BuildArgs& a,
                int32_t (&nb)[4], bool batched = false);

// One batched build: every stage in one grid-stride launch over the units.
// prefix: 4 arrays of nunits + 1 exclusive block prefixes (device memory, with
// the units); total: blocks per stage; grid: blocks per launch; nbins: the
// units' bin count (they share it).
hipError_t launch_build_batch(int kind, int nt, int nbins, const BuildArgs* units,
                              const int32_t* prefix, int nunits, const int32_t (&total)[4], int grid,
                              hipStream_t stream);

// Build: integer kernels write one global plane set; the Gaussian writes set
// `set` with the axis series of that scale.
// phase bit 1 = carries (aggregate + scan), bit 2 = planes (emit).
hipError_t launch_build(const SwihLayout& L, int kind, int set, const GaussAxis* ax,
                        const GaussAxis* ay, int32_t rx, int32_t ry, const uint8_t* img,
                        int32_t img_pitch, char* ws, hipStream_t stream, int phases = 3);

hipError_t launch_query(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                        const int32_t* centres, int32_t n, float* hist, uint32_t* hist_raw,
                        hipStream_t stream);

// Everything one dense map reads on the device.
struct MatchArgs {
  SwihGeom g;
  ScaleParams sp;
  const void* planes;      // uint32 planes or float tile-local planes
  const double* RC;        // Gaussian row carries
  const float* XC;         // Gaussian band-closing rows
  const double* beta;      // Gaussian: [H+1][2 nJ] y coefficients per row (bottom, top edge)
  const float* tmpl;       // normalised template, or null
  const uint32_t* tmpl_raw;  // exact template (integer kernels), or null
  float* map;
  int32_t x0, y0, x1, y1;  // inclusive centre rectangle
  int32_t nbx;             // integer kernels: virtual blocks per row of blocks
  // Gaussian comb sweep: items = ngroups x nseg x (comb groups of cpb) x nch
  int32_t nch, cw, nt;     // column chunks, centres per chunk, waves per chunk
  int32_t ncomb, nseg, S;  // combs, segments per comb, members per segment
  int32_t ngroups, bpg;    // bin groups, bins per group
  int32_t cpb;             // combs per block (each nt waves)
  int32_t* acc;            // ngroups > 1: per-centre integer accumulator (zero between maps)
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
  const float* XC;
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

// One persistent launch for a whole planned batch (integer kinds and the 2-D
// Gaussian): blocks take virtual blocks ("tickets") of every stage from one
// atomic counter, stages in order (basis, aggregate, scan, emit, query, map),
// and wait, with a time bound, only for the earlier stage of their own unit.
struct FusedArgs {
  const BuildArgs* units;
  const QueryArgs* q;
  const MatchArgs* m;
  const int32_t* upre;   // [4][nunits + 1] prefixes of the build stages' virtual blocks
  const int32_t* qpre;   // [nq + 1]
  const int32_t* mpre;   // [nm + 1]
  const int32_t* qunit;  // [nq] unit (plane set) each query reads
  const int32_t* munit;  // [nm] unit each map reads
  int32_t nunits, nq, nm, pad;
  int32_t cum[7];        // first ticket of each stage; cum[6] = tickets in all
  int32_t pad2;
  int32_t* sync;         // kFusedSyncHead words, then [4][nunits] finished tickets,
                         // then [4][nunits] completion stamps
  int32_t* status;       // written once at the end (0 = every wait met), or null
  int64_t limit;         // ticks of the constant-rate clock a wait may take; < 0: none
};

// next ticket, blocks exited, status, finished query tickets, completion
// clock, the queries' completion stamp
constexpr int kFusedSyncHead = 6;
inline int64_t fused_sync_words(int32_t nunits) { return kFusedSyncHead + 8 * (int64_t)nunits; }
// Virtual blocks of the fused launch's block size per 256-thread build block.
inline int fused_build_ratio(int kind) { return kind == 3 ? 3 : 1; }

// dyn_lds: the largest dynamic LDS of the batch's query and map jobs.
hipError_t launch_fused(int kind, int nt, int nbins, const FusedArgs& f, size_t dyn_lds,
                        hipStream_t stream);

// acc: the integer accumulator of a Gaussian map with several bin groups;
// null = the set's region of the workspace.
hipError_t launch_match(const SwihLayout& L, const ScaleParams& sp, int set, const char* ws,
                        const float* tmpl, const uint32_t* tmpl_raw, int32_t x0, int32_t y0,
                        int32_t x1, int32_t y1, float* map, hipStream_t stream,
                        int32_t* acc = nullptr);

// The static scratch of swih_match_noalloc: centres it holds, and its device
// address on the current device (looked up once per device; null on failure).
constexpr int64_t kNoallocCentres = (int64_t)1 << 22;
int32_t* noalloc_scratch();

// ------------------------------------------------------------------------
// Separable two-pass form of the Gaussian series (kernel SWIH_GAUSSIAN_SEP).
//
// The 2-D weight terms u_i(x) v_j(y) of the Gaussian are products of two 1-D
// families, so the window histogram factors into two 1-D weighted integral
// histograms with translation (Sec. 2.1, Eq. 2, applied per axis):
//   row pass:    h_b(xc; y) = sum_{|x - xc| <= rx} [Q(x, y) = b] g_x(x - xc)
//   column pass: H_b(xc, yc) = sum_{|y - yc| <= ry} h_b(xc; y) g_y(y - yc)
// with g the cosine series of the axis.  The row results h (one float per
// row, valid centre column and bin) are the only buffer; nothing of size
// terms x bins x pixels is ever stored.

struct SepGeom {
  int32_t H, W, B;      // image size, bins
  int32_t w, h, rx, ry; // window
  int32_t Wv, Hv;       // valid centre columns / rows: W - w + 1, H - h + 1
  int32_t K;            // series terms per axis beyond the constant
  int32_t SX;           // row pass: centre columns per wave
  int32_t SY;           // column pass: centre rows per segment (segments start at multiples of SY)
};

// One axis of the series g(t) = sum_k a_k cos(w_k t) for walks along it: the
// window sum of term k translated to the current centre is the complex number
// Z_k = sum_t e(t) exp(i w_k t) over the window's offsets t.
struct SepAxis {
  double a[SWIH_MAX_K + 1];   // a_0 .. a_K
  double ec[SWIH_MAX_K + 1];  // cos(w_k r), r the half width: the entering offset +r
  double es[SWIH_MAX_K + 1];  // sin(w_k r)  (the leaving offset -r is the conjugate)
  double rc[SWIH_MAX_K + 1];  // cos(w_k), sin(w_k): moving the centre one step on
  double rs[SWIH_MAX_K + 1];  //   multiplies Z_k by (rc - i rs)
  double g_in;                // g(r) = a_0 + sum_k a_k ec_k
};

void sep_axis(const GaussAxis& ax, int32_t r, SepAxis& s);

// Workspace of one scale (set-relative byte offsets, 256-byte aligned).
struct SepLayout {
  int64_t off_hr;   // float [H][W - w + 1][B] row results (sized for W)
  int64_t set_bytes;
};

SepLayout sep_layout(int32_t H, int32_t W, int32_t B);
SepGeom sep_geom(int32_t H, int32_t W, int32_t B, int32_t w, int32_t h, int32_t K);

struct SepBuildArgs {
  SepGeom g;
  const uint8_t* img;
  int32_t ipitch;
  float* hr;
  SepAxis ax;
};

struct SepQueryArgs {
  SepGeom g;
  const float* hr;
  SepAxis ay;
  double inv_mass;
  const int32_t* centres;  // [n][2]
  int32_t n;
  float* hist;             // [n][B]
};

struct SepMatchArgs {
  SepGeom g;
  const float* hr;
  SepAxis ay;
  double inv_mass;
  const float* tmpl;       // [B] normalised template
  float* map;
  int32_t x0, y0, x1, y1;  // inclusive centre rectangle
  int32_t nwx;             // waves across the rectangle
  int32_t seg0, nseg;      // first segment (absolute) and segment count
};

// Blocks (of 256 threads) of the build stages: nb[0] = 0 (the separable form
// needs no carries), nb[1] = the row pass.
void sep_build_args(const SepGeom& g, const SepLayout& L, const GaussAxis& ax, const uint8_t* img,
                    int32_t img_pitch, char* set_base, SepBuildArgs& a, int32_t (&nb)[2]);
void sep_query_args(const SepGeom& g, const SepLayout& L, const GaussAxis& ay, double mass,
                    const char* set_base, const int32_t* centres, int32_t n, float* hist,
                    SepQueryArgs& a, int32_t& nb);
void sep_match_args(const SepGeom& g, const SepLayout& L, const GaussAxis& ay, double mass,
                    const char* set_base, const float* tmpl, int32_t x0, int32_t y0, int32_t x1,
                    int32_t y1, float* map, SepMatchArgs& a, int32_t& nb);

// phases: bit 2 = row pass (bit 1, the carries, launches nothing).
hipError_t sep_launch_build(const SepBuildArgs& a, const int32_t (&nb)[2], int phases,
                            hipStream_t s);
hipError_t sep_launch_query(const SepQueryArgs& a, int32_t nb, hipStream_t s);
hipError_t sep_launch_match(const SepMatchArgs& a, int32_t nb, hipStream_t s);
// Batched forms: grid-stride launches over the items' virtual blocks
// (prefix: exclusive block prefixes in device memory; build: 2 arrays).
hipError_t sep_launch_build_batch(int nt, int nbins, const SepBuildArgs* units,
                                  const int32_t* prefix, int nunits, const int32_t (&total)[2],
                                  int grid, hipStream_t s);
hipError_t sep_launch_query_batch(int nt, int nbins, const SepQueryArgs* items,
                                  const int32_t* prefix, int n, int32_t total, int grid,
                                  hipStream_t s);
hipError_t sep_launch_match_batch(int nt, int nbins, const SepMatchArgs* items,
                                  const int32_t* prefix, int n, int32_t total, int grid,
                                  hipStream_t s);

// ------------------------------------------------------------------------
// Exponential (Laplacian) kernel (SWIH_EXPONENTIAL), swih_exp.hip.
//
// k(dx, dy) = exp(-|dx| / tx - |dy| / ty), tx = w / 4, ty = h / 4.  Four
// direction-weighted planes per bin (one per window quadrant, Sec. 2.1), each
// stored rescaled to its own corner so that it stays bounded; one plane set
// per scale.  The planes use the tile-major layout of SwihGeom with nP = 4
// (direction d = mirrored x (bit 0), mirrored y (bit 1)) and ppg = 1.

struct ExpScale {
  int32_t w, h, rx, ry;
  double itx, ity;     // 1 / tx, 1 / ty
  double fxlo, fylo;   // exp(-rx / tx), exp(-ry / ty): far corners
  double fxin, fyin;   // exp(1 / tx), exp(1 / ty): near corner of the centre's quadrant
  double mass, inv_mass;
};

void exp_scale(int32_t w, int32_t h, ExpScale& s);

struct ExpBuildArgs {
  SwihGeom g;
  const uint8_t* img;
  int32_t ipitch;
  int32_t nb1, nb2;    // scan: blocks of the band-chain and row-chain roles
  float* planes;
  double* z;           // [4 B][NTY][NTX 64] band sums -> band-top values
  double* T;           // [4 B][NTX][H]      row sums  -> left-edge row values
  double* CT;          // [4 B][NTY][NTX]    tile sums -> tile-origin values
  double itx, ity;
  // decays, computed on the host: one column / row step (qx = exp(-1/tx),
  // qy = exp(-1/ty)), eight of them, one band (qy^TY) and one tile (qx^64)
  double qx, qy, qx8, qy8, qyT, qx64;
  int32_t agg_hist;    // aggregate by LDS histograms, a block per (direction, band, tile)
  int32_t pad;
};

struct ExpQueryArgs {
  SwihGeom g;
  ExpScale s;
  const float* planes;
  const int32_t* centres;  // [n][2]
  int32_t n;
  float* hist;             // [n][B]
};

struct ExpMatchArgs {
  SwihGeom g;
  ExpScale s;
  const float* planes;
  const float* tmpl;       // [B] normalised template
  float* map;
  int32_t x0, y0, x1, y1;  // inclusive centre rectangle
  int32_t nbx;             // waves across the rectangle (64 centres each)
};

// nb: blocks of the build stages (0 = none, aggregate, scan, emit).
void exp_build_args(const SwihLayout& L, const ExpScale& s, int set, const uint8_t* img,
                    int32_t img_pitch, char* ws, ExpBuildArgs& a, int32_t (&nb)[4]);
void exp_query_args(const SwihLayout& L, const ExpScale& s, int set, const char* ws,
                    const int32_t* centres, int32_t n, float* hist, ExpQueryArgs& a, int32_t& nb);
void exp_match_args(const SwihLayout& L, const ExpScale& s, int set, const char* ws,
                    const float* tmpl, int32_t x0, int32_t y0, int32_t x1, int32_t y1, float* map,
                    ExpMatchArgs& a, int32_t& nb);

// phases: bit 1 = carries (aggregate + scan), bit 2 = planes (emit).
hipError_t exp_launch_build(const ExpBuildArgs& a, const int32_t (&nb)[4], int phases,
                            hipStream_t s);
hipError_t exp_launch_query(const ExpQueryArgs& a, int32_t nb, hipStream_t s);
hipError_t exp_launch_match(const ExpMatchArgs& a, int32_t nb, hipStream_t s);
// nbins: the units' bin count (they share it).
hipError_t exp_launch_build_batch(const ExpBuildArgs* units, const int32_t* prefix, int nunits,
                                  int nbins, const int32_t (&total)[4], int grid, hipStream_t s);
hipError_t exp_launch_query_batch(const ExpQueryArgs* items, const int32_t* prefix, int n,
                                  int32_t total, int grid, hipStream_t s);
hipError_t exp_launch_match_batch(const ExpMatchArgs* items, const int32_t* prefix, int n,
                                  int32_t total, int grid, hipStream_t s);


// ------------------------------------------------------------------------
// Baselines (swih_cake.hip): the wedding-cake approximation over the count
// plane of an integer-kernel workspace, and the brute-force weighted
// histogram straight from the image.

#define SWIH_MAX_RINGS 32

struct CakeArgs {
  SwihGeom g;
  const void* planes;        // uint32 planes of an integer kernel; plane 0 counts pixels
  int32_t nrings;
  int32_t rx[SWIH_MAX_RINGS], ry[SWIH_MAX_RINGS];  // nested half-sizes (negative = empty)
  double dw[SWIH_MAX_RINGS];  // w_i - w_{i-1}: weight steps from ring to ring
  double mass;
  const int32_t* centres;    // query: [n][2]
  int32_t n;
  float* hist;               // query: [n][B]
  const float* tmpl;         // map: [B] normalised template
  float* map;
  int32_t x0, y0, x1, y1;    // map: inclusive centre rectangle
  int32_t nbx;               // map: waves across the rectangle (64 centres each)
};

// Rings and weights for kernel `kind` (uniform, Manhattan, Euclidean) of a
// w x h window; returns 0, or -1 for a ring count outside 1..SWIH_MAX_RINGS.
int cake_args(int kind, const SwihGeom& g, int32_t w, int32_t h, int32_t rings, double mass,
              uint32_t c_int, const void* planes, CakeArgs& a);
hipError_t cake_launch_query(const CakeArgs& a, hipStream_t s);
hipError_t cake_launch_match(const CakeArgs& a, hipStream_t s);

struct BruteArgs {
  const uint8_t* img;
  int32_t ipitch;
  int32_t H, W, B;
  int32_t kind;              // uniform, Manhattan or Euclidean
  int32_t rx, ry;
  uint32_t c_int;            // kernel constant (rx + ry + 1, or rx^2 + ry^2 + 1)
  double mass;
  const uint32_t* tmpl_raw;  // [B] exact template
  float* map;
  int32_t x0, y0, x1, y1;
  int32_t nbx;               // blocks across the rectangle (64 centres each)
};

hipError_t brute_launch_match(const BruteArgs& a, hipStream_t s);

}  // namespace swih
