// Workspace layout of the weighted integral histograms and the build's carries.
//
// Geometry.  Pixel columns are cut into tiles of 64 (one wave64 lane per
// column) and pixel rows into bands of TY rows.  The integral histogram of
// plane p = (i, j) and bin b is the padded prefix
//   P[Y][X] = sum_{x < X, y < Y} [Q(f(x, y)) = b] u_i(x) v_j(y),
// X in [0, W], Y in [0, H]; row 0 and column 0 are zero.  Pixel column x
// feeds column X = x + 1, so tile tx owns columns X in [64 tx + 1, 64 tx + 64]
// and band ty owns rows Y in [TY ty + 1, TY ty + TY].
//
// Planes come in groups of ppg: the y terms of one x term for the Gaussian,
// all terms for the integer kernels.  The rows of a group's planes (for one
// bin) are interleaved: row Y of plane p sits at
//   ((((p / ppg) * B + b) * (H + 1) + Y) * ppg + p % ppg) * pitch
// so a window corner's values of all terms of a group lie within ppg * pitch
// elements.  Element X of a row sits at 63 + X, pitch a multiple of 64
// elements, so every tile's 64 columns start on a 256-byte boundary.
//
// Weight terms (u_i(x) v_j(y)):
//   uniform    {1}
//   Manhattan  {1, x, y}                 (i, j) = (0,0) (1,0) (0,1)
//   Euclidean  {1, x, y, x^2, y^2}       (0,0) (1,0) (0,1) (2,0) (0,2)
//   Gaussian   all products of {1, cos(2 pi k x / Px), sin(2 pi k x / Px)}_k
//              and the same in y: (2K+1)^2 terms, p = i * (2K+1) + j.
//
// Integer kernels store P itself as uint32 (arithmetic modulo 2^32).  The
// Gaussian stores it split per tile (tile origin Xo = 64 tx, Yo = TY ty):
//   L[Y][X]   = sum over Yo <= y < Y, Xo <= x < X  (float, bounded by the tile)
//   RC[tx][Y] = P[Y][Xo]                          (double, per row and tile column)
// with tx = tile of column X, ty = band of row Y, and zeros at row/column 0.
// Only window boxes are ever needed, and they follow from vertical
// differences at fixed X:
//   P[yb][X] - P[ya][X] = L[yb][X] - L[ya][X] + sum_{c} L[c][X]
//                         + RC[tx][yb] - RC[tx][ya]
// where c runs over the band-boundary rows (multiples of TY) in [ya, yb): the
// last row of a band holds the band's whole tile-local column sum, which is
// exactly what the band-top carry grows by from one band to the next.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#define SWIH_TX 64
#define SWIH_TY_MAX 64

struct SwihGeom {
  int32_t H, W, B;       // image size, bins
  int32_t TY;            // band height (<= 64)
  int32_t NTX, NTY;      // tiles across, bands down
  int32_t pitch;         // plane row pitch in elements (multiple of 64)
  int32_t nP, nI, nJ;    // planes, x terms, y terms
  int32_t gauss;         // 1 for the split Gaussian storage
  int32_t ppg;           // planes per interleaved group
  int64_t plane_elems;   // (H + 1) * pitch
  int64_t row_stride;    // ppg * pitch: from row Y to row Y + 1 of one plane
};

// Element offset of P[Y][X] of plane p, bin b.
__host__ __device__ inline int64_t swih_elem(const SwihGeom& g, int p, int b, int Y, int X) {
  const int grp = p / g.ppg, pj = p - grp * g.ppg;
  return (((int64_t)(grp * g.B + b) * (g.H + 1) + Y) * g.ppg + pj) * g.pitch + 63 + X;
}

// Byte offsets inside one workspace.  All regions are 256-byte aligned.
struct SwihLayout {
  SwihGeom g;
  int32_t nsets;         // plane sets: 1, or nscales for the Gaussian
  int64_t set_bytes;     // bytes of one plane set (planes [+ RC + tables])
  // inside a set
  int64_t off_planes;    // uint32 or float [nP][B][H+1][pitch]
  int64_t off_RC;        // double [nP][B][NTX][H+1]              (Gaussian)
  int64_t off_uq;        // int32 [nI][NTX*64]  fixed-point x terms (Gaussian)
  int64_t off_vq;        // int32 [H][nJ] fixed-point y terms, then double [H][nJ] (Gaussian)
  // build scratch (carries) of the set
  int64_t off_scratch;
  int64_t off_z;         // [nJ][B][NTY][NTX*64] band column sums -> carries (integer)
  int64_t off_T;         // [nI][B][NTX][H]      row-segment sums -> row carries
  int64_t off_CT;        // [nP][B][NTY][NTX]    tile carries
  int64_t total;
};

static inline int64_t swih_align256(int64_t v) { return (v + 255) & ~(int64_t)255; }

// Fixed-point scale of the Gaussian weight terms: u, v stored as round(t * 2^24).
#define SWIH_FIX_BITS 24
