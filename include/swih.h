/*
 * swih.h -- C ABI of the MI355X (gfx950) spatially weighted local histogram
 * library (libswih.so).
 *
 * Method: "Multi-Scale Spatially Weighted Local Histograms in O(1)"
 * (Poostchi, Shafiekhani, Palaniappan, Seetharaman), SWIH.
 *
 *   swih_build  -- Sec. 2.1, Eq. 2 and steps (1)-(2) of Sec. 1: quantise the
 *                  image (Q of Eq. 2), decompose the spatial kernel into weight
 *                  terms, and build one weighted integral histogram per
 *                  (weight term, bin).
 *   swih_query  -- Sec. 2.1 and steps (3)-(5) of Sec. 1: the weighted local
 *                  histogram of a window from O(1) corner lookups translated
 *                  from the window centre, normalised by the kernel mass.
 *   swih_match  -- Sec. 2 (Fig. 3), Sec. 3 (Fig. 5) and Sec. 4: the
 *                  sliding-window histogram-matching likelihood map, one value
 *                  per window centre.  The similarity is the Bhattacharyya
 *                  coefficient sum_b sqrt(p_b t_b).
 *
 * Conventions
 *   - Image: H x W uint8, row-major with a row pitch in bytes; x = column,
 *     y = row, 0-based.
 *   - Quantiser: bin(v) = floor(v * nbins / 256), uniform bins over [0, 256).
 *   - Windows are odd, w x h, rx = (w-1)/2, ry = (h-1)/2, centred on (xc, yc).
 *     Only windows wholly inside the image are valid:
 *     rx <= xc <= W-1-rx and ry <= yc <= H-1-ry.
 *   - Kernels (weight at offset (dx, dy) from the centre):
 *       SWIH_UNIFORM    1                                (plain histogram)
 *       SWIH_MANHATTAN  (rx+ry+1) - |dx| - |dy|          (Eq. 1, Fig. 4b)
 *       SWIH_EUCLIDEAN  (rx^2+ry^2+1) - dx^2 - dy^2      (Fig. 1b, paraboloid)
 *       SWIH_GAUSSIAN   exp(-dx^2/(2 sx^2) - dy^2/(2 sy^2)), sx = w/4,
 *                       sy = h/4 (Fig. 1c), evaluated through a K-term cosine
 *                       series per axis (see swih_gauss_terms).  Each scale's
 *                       planes hold, per bin and pixel, the (2K+1)^2 weight
 *                       terms already contracted with the coefficients of the
 *                       windows that have the pixel as a corner (its four
 *                       corner roles: 4 values) plus the exact pixel count;
 *                       every 64th row also keeps the terms contracted over x
 *                       only, for the windows that straddle it.
 *       SWIH_GAUSSIAN_SEP  the same series kernel in separable form: one
 *                       1-D weighted integral histogram along x with the
 *                       translated lookups (Sec. 2.1, Eq. 2 per axis) giving
 *                       row results per valid centre column, then one along y
 *                       over those row results.  Same values as SWIH_GAUSSIAN
 *                       up to rounding; the workspace holds H x (W-w+1) x
 *                       nbins floats per scale instead of 5 planes per bin.
 *       SWIH_EXPONENTIAL  exp(-|dx|/tx - |dy|/ty), tx = w/4, ty = h/4 (the
 *                       exponential weighting of Sec. 2): four direction-
 *                       weighted integral histograms per bin, one per window
 *                       quadrant (Sec. 2.1), each built in its own direction
 *                       and stored rescaled to its own corner, so values stay
 *                       bounded at any image size.  Exact up to rounding
 *                       (float planes, double lookups).
 *     The first three are exact: raw histograms are integers, computed modulo
 *     2^32 and exact whenever the true value is below 2^32.
 *   - Normalised histogram p_b = H_b / S, with S the kernel mass (the same at
 *     every location, Sec. 2.1).
 *
 * Memory and streams
 *   - Every pointer named d_* is a device pointer owned by the caller; the
 *     library never allocates, frees or keeps device memory between calls
 *     (the one exception is the static scratch of swih_match_noalloc, which
 *     comes with the code object when the library is loaded).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All device work is enqueued asynchronously on it; no call synchronises
 *     the device or reads device memory on the host.
 *   - The workspace written by swih_build is read by swih_query/swih_match;
 *     the caller must pass the same configuration and image size to all three,
 *     and must order them on streams.
 *
 * Errors
 *   - Every entry point returns an int status: SWIH_OK (0) or a negative code.
 *     Arguments are checked on the host before anything is enqueued; nothing
 *     is enqueued on error.  Device faults surface at the caller's next
 *     synchronisation of the stream.
 */
#ifndef SWIH_H_
#define SWIH_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWIH_OK 0
#define SWIH_ERR_INVALID (-1)     /* bad size, window, bin count, rectangle or NULL */
#define SWIH_ERR_WORKSPACE (-2)   /* workspace smaller than swih_workspace_bytes */
#define SWIH_ERR_UNSUPPORTED (-3) /* valid request this kernel cannot serve */
#define SWIH_ERR_HIP (-4)         /* a HIP launch or runtime call failed */
#define SWIH_ERR_SCRATCH (-5)     /* swih_match_noalloc: more centres than its static scratch holds */

typedef enum {
  SWIH_UNIFORM = 0,
  SWIH_MANHATTAN = 1,
  SWIH_EUCLIDEAN = 2,
  SWIH_GAUSSIAN = 3,
  SWIH_GAUSSIAN_SEP = 4,
  SWIH_EXPONENTIAL = 5
} swih_kernel;

/* One window scale: odd width and height, 1 <= w <= W, 1 <= h <= H. */
typedef struct {
  int32_t w, h;
} swih_scale;

typedef struct {
  int32_t nbins;            /* 1..256 */
  int32_t kernel;           /* swih_kernel */
  int32_t nscales;          /* >= 1 */
  const swih_scale* scales; /* host array of nscales entries */
  int32_t gauss_terms;      /* K of the cosine series, 1..8; 0 = default (3) */
  uint32_t flags;           /* reserved, must be 0 */
  int32_t band_rows;        /* rows of a scan tile, the build's band height: 0 = 64,
                               else 16, 32 or 64.  Tiles are 64 columns wide (one lane
                               per column).  Integer results do not depend on it; the
                               real-valued kernels' results change by rounding only
                               (tile-local origins move; well below their 1e-5 bars).
                               Speed does depend on it (more, shorter bands fill the
                               GPU on small frames, at the price of more carries).
                               Ignored by SWIH_GAUSSIAN_SEP, which has no tiles. */
} swih_config;

/* Inclusive rectangle of window CENTRES. */
typedef struct {
  int32_t x0, y0, x1, y1;
} swih_rect;

/*
 * Bytes of device workspace a build of an H x W image needs under `cfg`.
 * Integer kernels keep one set of planes for every scale; both Gaussian forms
 * and the exponential keep one set per scale (their weight terms depend on
 * the window size, Sec. 2.1 "multi-scale").  Returns the size (> 0), or a negative status.
 */
int64_t swih_workspace_bytes(const swih_config* cfg, int32_t height, int32_t width);

/*
 * Build the weighted integral histograms (Eq. 2) of the image into d_ws.
 *   d_img   device, height rows of `pitch` bytes, width <= pitch.
 *   d_ws    device workspace of at least swih_workspace_bytes(cfg, H, W) bytes,
 *           256-byte aligned; its previous contents are irrelevant.
 * Errors: SWIH_ERR_INVALID (cfg, sizes, NULL), SWIH_ERR_WORKSPACE, SWIH_ERR_HIP.
 */
int swih_build(const swih_config* cfg, const uint8_t* d_img, int32_t height, int32_t width,
               int32_t pitch, void* d_ws, size_t ws_bytes, void* stream);

/*
 * The build in two phases, for callers that schedule or time them apart.
 * swih_build is swih_build_carries followed by swih_build_planes for every
 * plane set.
 *   swih_build_carries  reads the image and computes the carries every tile
 *                       needs: the integral-histogram row above each band, the
 *                       row prefix left of each tile and the value at each tile
 *                       origin (plus, for the Gaussian, the weight-term tables
 *                       of the scale).  Several kernel launches, small output.
 *   swih_build_planes   writes the planes of one set from the image and those
 *                       carries: exactly one kernel launch.
 *   set     0 for integer kernels; the scale index for the Gaussian and the
 *           exponential, whose planes are per scale.
 * For SWIH_GAUSSIAN_SEP the first phase has nothing to do (it enqueues
 * nothing) and the second writes the row results in one launch.
 * Each set keeps its own carries, so a set's planes need only follow its own
 * carries on the stream.  Errors as swih_build, plus SWIH_ERR_INVALID for a
 * bad set.
 */
int swih_build_carries(const swih_config* cfg, const uint8_t* d_img, int32_t height,
                       int32_t width, int32_t pitch, int32_t set, void* d_ws, size_t ws_bytes,
                       void* stream);
int swih_build_planes(const swih_config* cfg, const uint8_t* d_img, int32_t height,
                      int32_t width, int32_t pitch, int32_t set, void* d_ws, size_t ws_bytes,
                      void* stream);

/*
 * Weighted local histograms at n window centres of scale `scale_idx`.
 *   d_centres   device int32 [n][2] = (xc, yc); every centre must be valid for
 *               the scale (a host check is not possible; out-of-range centres
 *               are clamped on the device and give unspecified histograms).
 *   d_hist      device float [n][nbins], p_b = H_b / S; may be NULL.
 *   d_hist_raw  device uint32 [n][nbins], exact H_b; integer kernels only
 *               (SWIH_ERR_UNSUPPORTED for both Gaussian forms and the
 *               exponential); may be NULL.
 * n == 0 is valid and enqueues nothing.
 */
int swih_query(const swih_config* cfg, const void* d_ws, size_t ws_bytes, int32_t height,
               int32_t width, int32_t scale_idx, const int32_t* d_centres, int32_t n,
               float* d_hist, uint32_t* d_hist_raw, void* stream);

/*
 * Likelihood map: Bhattacharyya coefficient of every window centre in
 * `centres` (inclusive, must lie in the valid range of the scale) against a
 * template histogram of the same scale.
 *   d_template      device float [nbins], normalised template t_b; or NULL.
 *   d_template_raw  device uint32 [nbins], exact template T_b (integer kernels
 *                   only); or NULL.  Exactly one of the two must be given.
 *                   With the float template the value is sum_b sqrt(p_b t_b)
 *                   over bins in order (double for the integer kernels and
 *                   the exponential), rounded to float.
 *                   With the raw template the value is
 *                   (sum_b sqrt(H_b T_b)) / S evaluated in double with bins in
 *                   order 0..nbins-1, then rounded to float.
 *   d_map           device float [(y1-y0+1)][(x1-x0+1)], row-major.
 * An empty rectangle (x1 < x0 or y1 < y0) is valid and enqueues nothing.
 * SWIH_GAUSSIAN maps may use a per-scale accumulator inside d_ws (when the
 * launch plan splits the bins into groups; cleared by the build, left cleared
 * by every map): Gaussian maps of one scale of one workspace must not run
 * concurrently (order them on one stream).  Maps of the other kernels only
 * read d_ws.
 */
int swih_match(const swih_config* cfg, const void* d_ws, size_t ws_bytes, int32_t height,
               int32_t width, int32_t scale_idx, const float* d_template,
               const uint32_t* d_template_raw, swih_rect centres, float* d_map, void* stream);

/*
 * swih_match for callers that cannot allocate device memory at the call (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Arguments, results and errors as swih_match; the map equals
 * swih_match's bit for bit.  A SWIH_GAUSSIAN map whose launch plan splits the
 * bins into several groups adds their sums into an integer accumulator: here
 * that accumulator is a static array of the library, one per device, holding
 * up to 4194304 centres (16 MiB), instead of the workspace's region.  The call
 * clears the part it uses on `stream` first and allocates nothing.
 *   SWIH_ERR_SCRATCH  a SWIH_GAUSSIAN rectangle of more than 4194304 centres.
 * Every call on one device shares that device's array: calls whose Gaussian
 * maps overlap in time on one device (other streams, other threads) race and
 * give wrong maps; order them on one stream.  Other kernels use no scratch
 * and behave exactly as swih_match.
 */
int swih_match_noalloc(const swih_config* cfg, const void* d_ws, size_t ws_bytes, int32_t height,
                       int32_t width, int32_t scale_idx, const float* d_template,
                       const uint32_t* d_template_raw, swih_rect centres, float* d_map,
                       void* stream);

/* ------------------------------------------------------------------------
 * Baselines the paper compares SWIH with (Sec. 3, Figs. 5 and 6).
 *
 * Wedding cake (Sec. 2, the wedding-cake approach, Fig. 4a): the window is cut
 * into `rings` nested windows around the centre, per axis half-sizes
 * r_i = floor((r+1)(rings-i)/rings) - 1, i = 0..rings-1 (equal runs of the
 * distances 0..r from the centre; a negative half-size is an empty window).
 * Each ring (a window minus the next one) is weighted by the mean of the
 * configured kernel over the ring's pixels, so the total mass stays S, and the
 * ring counts come from the plain count plane of the workspace: O(rings)
 * lookups per window whatever its size.  cfg must be an integer kernel
 * (SWIH_UNIFORM, SWIH_MANHATTAN, SWIH_EUCLIDEAN; SWIH_ERR_UNSUPPORTED
 * otherwise) and d_ws a workspace swih_build wrote for it.
 *   rings       1..32 (SWIH_ERR_INVALID otherwise).
 *   d_hist      device float [n][nbins], the normalised approximate histogram.
 *   d_template  device float [nbins], normalised template (normally the
 *               swih_cake_query result at the template centre).
 *   d_map       device float [(y1-y0+1)][(x1-x0+1)]: sum_b sqrt(p_b t_b) in
 *               double, bins in order, rounded to float.
 * Other arguments, rules and errors as swih_query / swih_match.
 */
int swih_cake_query(const swih_config* cfg, const void* d_ws, size_t ws_bytes, int32_t height,
                    int32_t width, int32_t scale_idx, int32_t rings, const int32_t* d_centres,
                    int32_t n, float* d_hist, void* stream);
int swih_cake_match(const swih_config* cfg, const void* d_ws, size_t ws_bytes, int32_t height,
                    int32_t width, int32_t scale_idx, int32_t rings, const float* d_template,
                    swih_rect centres, float* d_map, void* stream);

/*
 * Brute force (Sec. 2, the convolution-style weighted histogram): every pixel
 * of every window adds its kernel weight to its bin, straight from the image;
 * O(w h) per window.  Integer kernels only (SWIH_ERR_UNSUPPORTED otherwise);
 * the histograms are exact, and the map is (sum_b sqrt(H_b T_b)) / S as in
 * swih_match with the raw template, so the two maps are equal bit for bit.
 *   d_img            device image, as swih_build; no workspace is used.
 *   d_template_raw   device uint32 [nbins], exact template T_b.
 *   d_map            device float [(y1-y0+1)][(x1-x0+1)], row-major.
 * nbins up to 256 (each thread keeps its histogram in LDS).
 */
int swih_brute_match(const swih_config* cfg, const uint8_t* d_img, int32_t height, int32_t width,
                     int32_t pitch, int32_t scale_idx, const uint32_t* d_template_raw,
                     swih_rect centres, float* d_map, void* stream);

/*
 * The best window of a likelihood map, as a tracker's localisation step takes
 * it (Sec. 4): the first maximum of d_map[0..n-1] in row-major order.
 *   d_map   device float [n], every value >= 0 (likelihoods are).
 *   d_key   device uint64 [1], written with (bits of the maximum << 32) |
 *           (2^32 - 1 - index): index = 0xffffffff - (key & 0xffffffff).
 * 1 <= n < 2^32 (SWIH_ERR_INVALID otherwise).  Two launches on `stream`.
 */
int swih_argmax(const float* d_map, int64_t n, uint64_t* d_key, void* stream);

/* ------------------------------------------------------------------------
 * Batched form.  Sec. 4 applies the likelihood maps to many targets over the
 * frames of a tracking sequence; a batch builds many frames (or search-region
 * crops) of different sizes, queries their templates and computes their maps
 * with one grid-stride launch per stage, so uneven work fills the GPU and the
 * whole batch can be captured once in a HIP graph and replayed.
 *
 * The plan is pure host work: swih_batch_plan checks every descriptor and
 * writes a table that names all device buffers and launch sizes.  The caller
 * copies the table byte for byte to device memory (256-byte aligned) and
 * passes both copies to the launches, which read the host copy for launch
 * sizes and the device copy in the kernels.  The device copy must stay valid
 * while the launches run.  Every frame's result is a function of that frame
 * alone: the same as a single swih_build / swih_query / swih_match of it,
 * whatever else is in the batch.
 */
typedef struct {
  const uint8_t* d_img;      /* device: frame or crop origin, height rows of pitch bytes */
  int32_t height, width, pitch;
  int32_t nscales;           /* 0: the configuration's scales; else this frame's own */
  const swih_scale* scales;  /* host, nscales entries (read by swih_batch_plan only) */
  void* d_ws;                /* device workspace of this frame, 256-byte aligned */
  size_t ws_bytes;           /* >= swih_workspace_bytes of the frame's configuration */
  int32_t band_rows;         /* 0: the configuration's; else this frame's own scan-tile
                                rows (16, 32 or 64), e.g. as an autotuner picks per size */
} swih_frame_desc;

typedef struct {
  int32_t frame, scale_idx;  /* frame index and the frame's scale */
  const int32_t* d_centres;  /* device int32 [n][2] */
  int32_t n;
  float* d_hist;             /* device float [n][nbins] or NULL */
  uint32_t* d_hist_raw;      /* device uint32 [n][nbins] or NULL (integer kernels) */
} swih_query_desc;

typedef struct {
  int32_t frame, scale_idx;
  swih_rect centres;         /* inclusive, within the scale's valid range */
  const float* d_template;   /* exactly one of the two templates, as swih_match */
  const uint32_t* d_template_raw;
  float* d_map;              /* device float, rectangle-sized, row-major */
} swih_match_desc;

/* Bytes of the table for this batch (or a negative status). */
int64_t swih_batch_table_bytes(const swih_config* cfg, const swih_frame_desc* frames,
                               int32_t nframes, int32_t nqueries, int32_t nmatches);

/*
 * Check the batch and write its table into h_table (host, table_bytes).
 * Errors as the single-frame calls; SWIH_ERR_WORKSPACE if a frame's workspace
 * or the table is too small.  Queries and maps name a frame and one of its scales.
 */
int swih_batch_plan(const swih_config* cfg, const swih_frame_desc* frames, int32_t nframes,
                    const swih_query_desc* queries, int32_t nqueries,
                    const swih_match_desc* matches, int32_t nmatches, void* h_table,
                    size_t table_bytes);

/* Launch the batch's builds (4 launches), queries (1) or maps (1) on `stream`. */
int swih_build_batch(const void* h_table, const void* d_table, void* stream);
int swih_query_batch(const void* h_table, const void* d_table, void* stream);
int swih_match_batch(const void* h_table, const void* d_table, void* stream);

/*
 * The whole batch -- every build, then the template queries, then the maps --
 * in ONE persistent launch (Sec. 4: many targets over many frames).  Results
 * are identical, bit for bit, to swih_build_batch + swih_query_batch +
 * swih_match_batch of the same table.
 *
 * Each stage's virtual blocks are tickets taken from one atomic counter in
 * stage order (basis, aggregate, scan, emit, query, map); a block waits only
 * until the stage before its ticket is complete for the same plane set (a
 * map: also until every query of the batch is done, since its template may
 * be one of them).  Tickets are taken in order, so the launch always drains;
 * every wait is also bounded: past `wait_ms` milliseconds the block records a
 * failure and carries on (the results are then not to be used).
 *   d_table   the device copy of the table; the launch updates counters kept
 *             in it and leaves them reset, so the table can be launched again.
 *             Two launches of one table must not overlap.
 *   d_status  device int32 or NULL: set at the end to 0 if every wait was met,
 *             1 if one gave up.
 *   wait_ms   bound on each wait; 0 = 2000 ms.  A negative value makes every
 *             wait give up at once (a test hook for the failure path: d_status
 *             becomes 1 and the launch still ends; the next launch of the
 *             table starts clean).
 * Kernels: uniform, Manhattan, Euclidean, and the 2-D Gaussian with up to 4
 * series terms per axis (SWIH_ERR_UNSUPPORTED otherwise: the separable and
 * exponential forms run with the stage launches).
 */
int swih_run_batch(const void* h_table, void* d_table, int32_t* d_status, int32_t wait_ms,
                   void* stream);

/*
 * The cosine series that stands in for one axis of the Gaussian kernel:
 *   g(t) ~= sum_{k=0..K} a_k cos(w_k t),  t in [-r, r], r = (n-1)/2,
 * with w_0 = 0 < w_1 < ... < w_K, fitted to exp(-t^2 / (2 (n/4)^2)) at the
 * integer offsets: coefficients by least squares, frequencies refined from
 * harmonic starts by Levenberg-Marquardt, the candidate with the smallest
 * worst normalised 2-D histogram error of the separable product kept.  Each
 * cosine term splits into cos/sin products of the absolute coordinate and the
 * window centre, which is what makes the Gaussian decomposable into 2K+1
 * weight terms per axis.  K = 3 reaches a worst 2-D error of ~4e-8.
 *   n         odd window side, 1..4095
 *   K         1..8
 *   a_out     host double [K+1] (may be NULL)
 *   omega_out host double [K+1], the frequencies w_k in radians per pixel
 *             (may be NULL)
 *   err_out   host double: the worst normalised histogram error of the square
 *             n x n window with this series (may be NULL)
 * Host only; the fit runs once per (n, K) per process and is cached.
 */
int swih_gauss_terms(int32_t n, int32_t K, double* a_out, double* omega_out, double* err_out);

/*
 * Copy `bytes` bytes from src to dst on `stream` with a kernel.  Each pointer
 * is device memory or pinned host memory (hipHostMalloc, torch pin_memory):
 * the kernel reads and writes pinned host memory directly over the bus, so a
 * request loop's uploads and downloads do not go through the runtime's copy
 * engines (Sec. 4's tracking requests, served; see serving.py).  Any
 * alignment; 16-byte moves where src and dst share their alignment.
 * Pageable host memory (or any pointer the device cannot reach) gives
 * SWIH_ERR_INVALID; nothing is enqueued then.  Host memory written by the copy
 * is complete once the stream has reached the copy (an event after it).
 */
int swih_copy(void* dst, const void* src, size_t bytes, void* stream);

/* Static text for a status code. */
const char* swih_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* SWIH_H_ */
