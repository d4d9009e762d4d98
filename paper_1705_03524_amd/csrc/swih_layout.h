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
// Planes come in groups of ppg (all of a bin's stored planes, one group).  Storage is tile-major: for one (group,
// bin) the tile columns follow one another, each holding rows Y = 0..H, and a
// row holds the group's ppg planes as consecutive runs of 64 elements:
//   elem(p, b, Y, X) = ((grp B + b) NTX + tx) tile_stride + Y row_stride
//                      + (p % ppg) 64 + lane,   grp = p / ppg,
// with tx = (X - 1) / 64, lane = (X - 1) % 64 (the column of pixel x = X - 1),
// row_stride = 64 ppg and tile_stride = (H + 1) row_stride.  The wave that
// builds a tile of a band writes one contiguous run of memory; a window
// corner's values of all terms of a group lie in 64 ppg elements.  Column
// X = 0 is zero by definition and is not stored: readers use 0 for it.
//
// Weight terms (u_i(x) v_j(y)):
//   uniform    {1}
//   Manhattan  {1, x, y}                 (i, j) = (0,0) (1,0) (0,1)
//   Euclidean  {1, x, y, x^2, y^2}       (0,0) (1,0) (0,1) (2,0) (0,2)
//   Gaussian   all products of {1, cos(w_k x), sin(w_k x)}_{k=1..K}
//              and the same in y: NT^2 terms (NT = 2K+1), p = i * NT + j.
//
// Integer kernels store P itself as uint32 (arithmetic modulo 2^32), one
// plane per term.  The Gaussian splits P per tile (tile origin Xo = 64 tx,
// Yo = TY ty):
//   L[Y][X]   = sum over Yo <= y < Y, Xo <= x < X  (bounded by the tile)
//   RC[tx][Y] = P[Y][Xo]                          (double, per row and tile column)
// and, the set's window half-sizes (rx, ry) being fixed, stores L already
// contracted with the translation coefficients of the windows that have
// (X, Y) as a corner.  Column X is the right edge of the windows centred at
// X - rx - 1 and the left edge of those at X + rx; row Y the bottom edge of
// the windows centred at Y - ry - 1 and the top edge of those at Y + ry:
//   V+_j[Y][X] = sum_i alpha_i(X - rx - 1) L_ij[Y][X],  V-_j: alpha_i(X + rx)
//   C_RB = sum_j beta_j(Y - ry - 1) V+_j,  C_RT = sum_j beta_j(Y + ry) V+_j
//   C_LB = sum_j beta_j(Y - ry - 1) V-_j,  C_LT = sum_j beta_j(Y + ry) V-_j
//   N[Y][X] = L_00[Y][X]                              (the pixel count, exact)
// alpha_i / beta_j the x / y series coefficients at a centre coordinate: 5
// float planes per bin (p = C_RB, C_RT, C_LB, C_LT, N) where the terms would
// take NT^2.  A window's histogram is then its four corners (plus the
// crossings and carries below).  The band-closing rows c, crossed by windows
// whose centre rows vary, keep V+_j and V-_j uncontracted in y in a side
// array XC[bin][c / TY - 1][tx][q][64] (q = j for V+, NT + j for V-).
// RC is contracted in y the same way, per (tile, row):
//   RCB_i = sum_j beta_j(Y - ry - 1) RC_ij,  RCT_i = sum_j beta_j(Y + ry) RC_ij,
// and RC_00 (the count), 2 NT + 1 doubles stored [bin][tx][Y][q] (q fastest):
// a lookup needs all of them for one tile and row, one contiguous run.
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
  int32_t TY;            // band height: 16, 32 or 64
  int32_t lgTY;          // log2 TY
  int32_t NTX, NTY;      // tiles across, bands down
  int32_t nP, nI, nJ;    // weight terms, x terms, y terms
  int32_t nPL;           // stored planes per bin (integer kernels: nP; Gaussian: 5)
  int32_t nRC;           // Gaussian row-carry values per (tile, row): 2 nI + 1
  int32_t gauss;         // 1 for the split Gaussian storage
  int32_t ppg;           // planes per interleaved group
  int64_t row_stride;    // 64 ppg: from row Y to row Y + 1 of one plane
  int64_t tile_stride;   // (H + 1) row_stride: from tile column tx to tx + 1
};

// Offset of plane p, bin b at row 0 of tile 0, lane 0.
__host__ __device__ inline int64_t swih_base(const SwihGeom& g, int p, int b) {
  const int grp = p / g.ppg, pj = p - grp * g.ppg;
  return (int64_t)(grp * g.B + b) * g.NTX * g.tile_stride + pj * 64;
}

// Column part of the offset of X >= 1.
__host__ __device__ inline int64_t swih_xoff(const SwihGeom& g, int X) {
  return (int64_t)((X - 1) >> 6) * g.tile_stride + ((X - 1) & 63);
}

// Element offset of P[Y][X] of plane p, bin b, for X >= 1.
__host__ __device__ inline int64_t swih_elem(const SwihGeom& g, int p, int b, int Y, int X) {
  return swih_base(g, p, b) + (int64_t)Y * g.row_stride + swih_xoff(g, X);
}

// Element offset of the Gaussian row-carry value q (RCB_i: q = i, RCT_i:
// q = NT + i, the count: q = 2 NT) of tile tx, row Y, bin b: [b][tx][Y][q].
__host__ __device__ inline int64_t swih_rc(const SwihGeom& g, int q, int b, int tx, int Y) {
  return (((int64_t)b * g.NTX + tx) * (g.H + 1) + Y) * g.nRC + q;
}

// Element offset of the Gaussian band-closing row values of row c (a
// positive multiple of TY below H), value q, bin b, at column X >= 1:
// XC[b][c / TY - 1][tx][q][64].
__host__ __device__ inline int64_t swih_xc(const SwihGeom& g, int q, int b, int c, int X) {
  return (((int64_t)b * g.NTY + ((c >> g.lgTY) - 1)) * g.NTX + ((X - 1) >> 6)) * (2 * g.nJ * 64) +
         q * 64 + ((X - 1) & 63);
}

// Byte offsets inside one workspace.  All regions are 256-byte aligned.
struct SwihLayout {
  SwihGeom g;
  int32_t nsets;         // plane sets: 1, or nscales for the Gaussian
  int64_t set_bytes;     // bytes of one plane set (planes [+ RC + tables])
  // inside a set
  int64_t off_planes;    // uint32 or float planes, tile-major (above)
  int64_t off_RC;        // double [B][NTX][H+1][nRC], swih_rc    (Gaussian)
  int64_t off_XC;        // float band-closing rows, swih_xc       (Gaussian)
  int64_t off_beta;      // double [H+1][2 nJ] beta at each row as a bottom / top edge (Gaussian)
  int64_t off_uq;        // int32 [nI][NTX*64]  fixed-point x terms (Gaussian)
  int64_t off_vq;        // int32 [H][nJ] fixed-point y terms, then double [H][nJ] (Gaussian)
  int64_t off_acc;       // int32 [H * W] map accumulator of the map sweep (Gaussian)
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
