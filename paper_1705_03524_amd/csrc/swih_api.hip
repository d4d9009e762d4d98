// C ABI of libswih.so: argument checks, workspace layout and launches.
#include <string.h>

#include <vector>

#include "swih.h"
#include "swih_internal.h"

namespace swih {
namespace {

constexpr int32_t kMaxSide = 8192;
constexpr int32_t kDefaultTY = 64;

bool kind_ok(int32_t k) { return k >= SWIH_UNIFORM && k <= SWIH_EXPONENTIAL; }

// Kernels built from the cosine series.
bool series_kind(int32_t k) { return k == SWIH_GAUSSIAN || k == SWIH_GAUSSIAN_SEP; }

// Kernels with one workspace set per scale (weight terms depend on the window).
bool per_scale(int32_t k) { return series_kind(k) || k == SWIH_EXPONENTIAL; }

// Kernels whose histograms are real-valued: no exact integer outputs.
bool real_kind(int32_t k) { return per_scale(k); }

int32_t gauss_K(const swih_config* c) { return c->gauss_terms == 0 ? SWIH_DEFAULT_K : c->gauss_terms; }

// Checks the configuration against an image size; returns a status.
int check_config(const swih_config* c, int32_t H, int32_t W) {
  if (!c || H < 1 || W < 1 || H > kMaxSide || W > kMaxSide) return SWIH_ERR_INVALID;
  if (c->nbins < 1 || c->nbins > 256 || !kind_ok(c->kernel) || c->flags != 0)
    return SWIH_ERR_INVALID;
  if (c->band_rows != 0 && c->band_rows != 16 && c->band_rows != 32 && c->band_rows != 64)
    return SWIH_ERR_INVALID;
  if (c->nscales < 1 || !c->scales) return SWIH_ERR_INVALID;
  if (series_kind(c->kernel)) {
    const int32_t K = gauss_K(c);
    if (K < 1 || K > SWIH_MAX_K) return SWIH_ERR_INVALID;
  }
  for (int s = 0; s < c->nscales; ++s) {
    const swih_scale sc = c->scales[s];
    if (sc.w < 1 || sc.h < 1 || (sc.w % 2) == 0 || (sc.h % 2) == 0 || sc.w > W || sc.h > H)
      return SWIH_ERR_INVALID;
  }
  return SWIH_OK;
}

// Kernel mass of an integer kernel (closed forms of the kernel sums).
double int_mass(int32_t kind, int32_t w, int32_t h) {
  const double rx = (w - 1) / 2, ry = (h - 1) / 2;
  if (kind == SWIH_UNIFORM) return (double)w * h;
  if (kind == SWIH_MANHATTAN)
    return (double)w * h * (rx + ry + 1) - h * rx * (rx + 1) - w * ry * (ry + 1);
  return (double)w * h * (rx * rx + ry * ry + 1) - h * rx * (rx + 1) * (2 * rx + 1) / 3 -
         w * ry * (ry + 1) * (2 * ry + 1) / 3;
}

int make_layout(const swih_config* c, int32_t H, int32_t W, SwihLayout& L) {
  memset(&L, 0, sizeof(L));
  SwihGeom& g = L.g;
  g.H = H;
  g.W = W;
  g.B = c->nbins;
  if (c->kernel == SWIH_GAUSSIAN_SEP) {  // row results + tables per scale (swih_sep.hip)
    g.nI = g.nJ = 2 * gauss_K(c) + 1;
    L.set_bytes = sep_layout(H, W, g.B).set_bytes;
    L.nsets = c->nscales;
    L.total = L.set_bytes * L.nsets;
    return SWIH_OK;
  }
  g.TY = c->band_rows ? c->band_rows : kDefaultTY;
  g.lgTY = g.TY == 16 ? 4 : g.TY == 32 ? 5 : 6;
  g.NTX = (W + SWIH_TX - 1) / SWIH_TX;
  g.NTY = (H + g.TY - 1) / g.TY;
  if (c->kernel == SWIH_EXPONENTIAL) {  // four direction planes per bin (swih_exp.hip)
    g.nP = 4;
    g.nPL = 4;
    g.ppg = 1;
    g.row_stride = SWIH_TX;
    g.tile_stride = (int64_t)(H + 1) * g.row_stride;
    const int64_t DB = 4LL * g.B;
    int64_t off = 0;
    L.off_planes = off;
    off += swih_align256(DB * g.NTX * (int64_t)(H + 1) * SWIH_TX * 4);
    L.off_scratch = off;
    L.off_z = off;
    off += swih_align256(DB * g.NTY * (int64_t)g.NTX * SWIH_TX * 8);
    L.off_T = off;
    off += swih_align256(DB * g.NTX * (int64_t)H * 8);
    L.off_CT = off;
    off += swih_align256(DB * g.NTY * (int64_t)g.NTX * 8);
    L.set_bytes = off;
    L.nsets = c->nscales;
    L.total = L.set_bytes * L.nsets;
    return SWIH_OK;
  }
  const bool gauss = c->kernel == SWIH_GAUSSIAN;
  g.gauss = gauss ? 1 : 0;
  if (gauss) {
    g.nI = g.nJ = 2 * gauss_K(c) + 1;
    g.nP = g.nI * g.nJ;
    g.nPL = 5;                 // corner-contracted planes C_RB, C_RT, C_LB, C_LT, N
    g.nRC = 2 * g.nI + 1;      // y-contracted row carries RCB, RCT, count
  } else {
    static const int nI[3] = {1, 2, 3}, nP[3] = {1, 3, 5};
    g.nI = g.nJ = nI[c->kernel];
    g.nP = nP[c->kernel];
    g.nPL = g.nP;
  }
  g.ppg = g.nPL;
  g.row_stride = (int64_t)g.ppg * SWIH_TX;
  g.tile_stride = (int64_t)(H + 1) * g.row_stride;
  const int64_t PB = (int64_t)g.nP * g.B;
  const int64_t NXP = (int64_t)g.NTX * SWIH_TX;
  int64_t off = 0;
  L.off_planes = off;
  off += swih_align256((int64_t)g.nPL * g.B * g.NTX * (int64_t)(H + 1) * SWIH_TX * 4);
  if (gauss) {
    L.off_RC = off;
    off += swih_align256((int64_t)g.nRC * g.B * g.NTX * (int64_t)(H + 1) * 8);
    L.off_XC = off;
    off += swih_align256((int64_t)2 * g.nJ * g.B * g.NTY * g.NTX * SWIH_TX * 4);
    L.off_beta = off;
    off += swih_align256((int64_t)2 * g.nJ * (H + 1) * 8);
    L.off_uq = off;
    off += swih_align256((int64_t)g.nI * NXP * 4);
    L.off_vq = off;  // int32 [H][nJ], then double [H][nJ]
    off += swih_align256((int64_t)g.nJ * H * 4) + swih_align256((int64_t)g.nJ * H * 8);
    L.off_acc = off;
    off += swih_align256((int64_t)H * W * 4);
  }
  // build scratch (carries), inside the set so that sets never share it
  const int64_t esz = gauss ? 8 : 4;
  L.off_scratch = off;
  L.off_z = off;
  if (!gauss) off += swih_align256((int64_t)g.nJ * g.B * g.NTY * NXP * esz);
  L.off_T = off;
  off += swih_align256((int64_t)g.nI * g.B * g.NTX * (int64_t)H * esz);
  L.off_CT = off;
  off += swih_align256(PB * g.NTY * g.NTX * esz);
  L.set_bytes = off;
  L.nsets = gauss ? c->nscales : 1;
  off = L.set_bytes * L.nsets;
  L.total = off;
  return SWIH_OK;
}

int fill_axis(int32_t n, int32_t K, GaussAxis& ax) {
  memset(&ax, 0, sizeof(ax));
  ax.K = K;
  if (gauss_fit(n, K, ax.a, ax.om, nullptr)) return SWIH_ERR_INVALID;
  return SWIH_OK;
}

int scale_params(const swih_config* c, int32_t scale_idx, ScaleParams& sp) {
  memset(&sp, 0, sizeof(sp));
  const swih_scale sc = c->scales[scale_idx];
  sp.w = sc.w;
  sp.h = sc.h;
  sp.rx = (sc.w - 1) / 2;
  sp.ry = (sc.h - 1) / 2;
  sp.kind = c->kernel;
  if (series_kind(c->kernel)) {
    const int32_t K = gauss_K(c);
    if (fill_axis(sc.w, K, sp.ax) || fill_axis(sc.h, K, sp.ay)) return SWIH_ERR_INVALID;
    sp.mass = gauss_axis_mass(sc.w, K, sp.ax.a, sp.ax.om) * gauss_axis_mass(sc.h, K, sp.ay.a, sp.ay.om);
    return SWIH_OK;
  }
  if (c->kernel == SWIH_EXPONENTIAL) {
    ExpScale es;
    exp_scale(sc.w, sc.h, es);
    sp.mass = es.mass;
    return SWIH_OK;
  }
  sp.mass = int_mass(c->kernel, sc.w, sc.h);
  if (sp.mass >= 4294967296.0) return SWIH_ERR_UNSUPPORTED;  // H_b must stay below 2^32
  if (c->kernel == SWIH_MANHATTAN) sp.c_int = (uint32_t)(sp.rx + sp.ry + 1);
  if (c->kernel == SWIH_EUCLIDEAN)
    sp.c_int = (uint32_t)((int64_t)sp.rx * sp.rx + (int64_t)sp.ry * sp.ry + 1);
  return SWIH_OK;
}

bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }

}  // namespace
}  // namespace swih

using namespace swih;

extern "C" {

int64_t swih_workspace_bytes(const swih_config* cfg, int32_t height, int32_t width) {
  const int st = check_config(cfg, height, width);
  if (st != SWIH_OK) return st;
  SwihLayout L;
  make_layout(cfg, height, width, L);
  return L.total;
}

}  // extern "C"

namespace {

int build_phases(const swih_config* cfg, const uint8_t* d_img, int32_t height, int32_t width,
                 int32_t pitch, int32_t set, void* d_ws, size_t ws_bytes, void* stream,
                 int phases) {
  int st = check_config(cfg, height, width);
  if (st != SWIH_OK) return st;
  if (!d_img || !d_ws || pitch < width) return SWIH_ERR_INVALID;
  if (!aligned256(d_ws)) return SWIH_ERR_INVALID;
  SwihLayout L;
  make_layout(cfg, height, width, L);
  if ((int64_t)ws_bytes < L.total) return SWIH_ERR_WORKSPACE;
  for (int k = 0; k < cfg->nscales; ++k) {  // every scale must be servable
    ScaleParams sp;
    st = scale_params(cfg, k, sp);
    if (st != SWIH_OK) return st;
  }
  hipStream_t s = (hipStream_t)stream;
  const bool gauss = cfg->kernel == SWIH_GAUSSIAN;
  const int first = set < 0 ? 0 : set, last = set < 0 ? L.nsets - 1 : set;
  if (first >= L.nsets || last >= L.nsets) return SWIH_ERR_INVALID;
  if (cfg->kernel == SWIH_GAUSSIAN_SEP) {
    const SepLayout SL = sep_layout(height, width, cfg->nbins);
    for (int k = first; k <= last; ++k) {
      ScaleParams sp;
      scale_params(cfg, k, sp);
      const SepGeom sg = sep_geom(height, width, cfg->nbins, sp.w, sp.h, gauss_K(cfg));
      SepBuildArgs a;
      int32_t nb[2];
      sep_build_args(sg, SL, sp.ax, d_img, pitch, (char*)d_ws + (size_t)k * L.set_bytes, a, nb);
      if (sep_launch_build(a, nb, phases, s) != hipSuccess) return SWIH_ERR_HIP;
    }
    return SWIH_OK;
  }
  if (cfg->kernel == SWIH_EXPONENTIAL) {
    for (int k = first; k <= last; ++k) {
      const swih_scale sc = cfg->scales[k];
      ExpScale es;
      exp_scale(sc.w, sc.h, es);
      ExpBuildArgs a;
      int32_t nb[4];
      exp_build_args(L, es, k, d_img, pitch, (char*)d_ws, a, nb);
      if (exp_launch_build(a, nb, phases, s) != hipSuccess) return SWIH_ERR_HIP;
    }
    return SWIH_OK;
  }
  for (int k = first; k <= last; ++k) {
    ScaleParams sp;
    scale_params(cfg, gauss ? k : 0, sp);
    if (launch_build(L, cfg->kernel, k, gauss ? &sp.ax : nullptr, gauss ? &sp.ay : nullptr, sp.rx, sp.ry, d_img,
                     pitch, (char*)d_ws, s, phases) != hipSuccess)
      return SWIH_ERR_HIP;
  }
  return SWIH_OK;
}

}  // namespace

extern "C" {

int swih_build(const swih_config* cfg, const uint8_t* d_img, int32_t height, int32_t width,
               int32_t pitch, void* d_ws, size_t ws_bytes, void* stream) {
  return build_phases(cfg, d_img, height, width, pitch, -1, d_ws, ws_bytes, stream, 3);
}

int swih_build_carries(const swih_config* cfg, const uint8_t* d_img, int32_t height,
                       int32_t width, int32_t pitch, int32_t set, void* d_ws, size_t ws_bytes,
                       void* stream) {
  if (set < 0) return SWIH_ERR_INVALID;
  return build_phases(cfg, d_img, height, width, pitch, set, d_ws, ws_bytes, stream, 1);
}

int swih_build_planes(const swih_config* cfg, const uint8_t* d_img, int32_t height,
                      int32_t width, int32_t pitch, int32_t set, void* d_ws, size_t ws_bytes,
                      void* stream) {
  if (set < 0) return SWIH_ERR_INVALID;
  return build_phases(cfg, d_img, height, width, pitch, set, d_ws, ws_bytes, stream, 2);
}

int swih_query(const swih_config* cfg, const void* d_ws, size_t ws_bytes, int32_t height,
               int32_t width, int32_t scale_idx, const int32_t* d_centres, int32_t n,
               float* d_hist, uint32_t* d_hist_raw, void* stream) {
  int st = check_config(cfg, height, width);
  if (st != SWIH_OK) return st;
  if (scale_idx < 0 || scale_idx >= cfg->nscales || n < 0 || !d_ws) return SWIH_ERR_INVALID;
  if (real_kind(cfg->kernel) && d_hist_raw) return SWIH_ERR_UNSUPPORTED;
  if (n == 0) return SWIH_OK;
  if (!d_centres || (!d_hist && !d_hist_raw)) return SWIH_ERR_INVALID;
  SwihLayout L;
  make_layout(cfg, height, width, L);
  if ((int64_t)ws_bytes < L.total) return SWIH_ERR_WORKSPACE;
  ScaleParams sp;
  st = scale_params(cfg, scale_idx, sp);
  if (st != SWIH_OK) return st;
  if (cfg->kernel == SWIH_GAUSSIAN_SEP) {
    const SepGeom sg = sep_geom(height, width, cfg->nbins, sp.w, sp.h, gauss_K(cfg));
    SepQueryArgs a;
    int32_t nb;
    sep_query_args(sg, sep_layout(height, width, cfg->nbins), sp.ay, sp.mass,
                   (const char*)d_ws + (size_t)scale_idx * L.set_bytes, d_centres, n, d_hist, a, nb);
    return sep_launch_query(a, nb, (hipStream_t)stream) == hipSuccess ? SWIH_OK : SWIH_ERR_HIP;
  }
  if (cfg->kernel == SWIH_EXPONENTIAL) {
    const swih_scale sc = cfg->scales[scale_idx];
    ExpScale es;
    exp_scale(sc.w, sc.h, es);
    ExpQueryArgs a;
    int32_t nb;
    exp_query_args(L, es, scale_idx, (const char*)d_ws, d_centres, n, d_hist, a, nb);
    return exp_launch_query(a, nb, (hipStream_t)stream) == hipSuccess ? SWIH_OK : SWIH_ERR_HIP;
  }
  const int set = cfg->kernel == SWIH_GAUSSIAN ? scale_idx : 0;
  return launch_query(L, sp, set, (const char*)d_ws, d_centres, n, d_hist, d_hist_raw,
                      (hipStream_t)stream) == hipSuccess
             ? SWIH_OK
             : SWIH_ERR_HIP;
}

}  // extern "C"

namespace {

int match_impl(const swih_config* cfg, const void* d_ws, size_t ws_bytes, int32_t height,
               int32_t width, int32_t scale_idx, const float* d_template,
               const uint32_t* d_template_raw, swih_rect r, float* d_map, void* stream,
               bool noalloc) {
  int st = check_config(cfg, height, width);
  if (st != SWIH_OK) return st;
  if (scale_idx < 0 || scale_idx >= cfg->nscales || !d_ws) return SWIH_ERR_INVALID;
  if ((d_template == nullptr) == (d_template_raw == nullptr)) return SWIH_ERR_INVALID;
  if (real_kind(cfg->kernel) && d_template_raw) return SWIH_ERR_UNSUPPORTED;
  if (r.x1 < r.x0 || r.y1 < r.y0) return SWIH_OK;
  const swih_scale sc = cfg->scales[scale_idx];
  const int32_t rx = (sc.w - 1) / 2, ry = (sc.h - 1) / 2;
  if (r.x0 < rx || r.y0 < ry || r.x1 > width - 1 - rx || r.y1 > height - 1 - ry)
    return SWIH_ERR_INVALID;
  if (!d_map) return SWIH_ERR_INVALID;
  if (noalloc && cfg->kernel == SWIH_GAUSSIAN &&
      (int64_t)(r.x1 - r.x0 + 1) * (r.y1 - r.y0 + 1) > kNoallocCentres)
    return SWIH_ERR_SCRATCH;
  SwihLayout L;
  make_layout(cfg, height, width, L);
  if ((int64_t)ws_bytes < L.total) return SWIH_ERR_WORKSPACE;
  ScaleParams sp;
  st = scale_params(cfg, scale_idx, sp);
  if (st != SWIH_OK) return st;
  if (cfg->kernel == SWIH_GAUSSIAN_SEP) {
    const SepGeom sg = sep_geom(height, width, cfg->nbins, sp.w, sp.h, gauss_K(cfg));
    SepMatchArgs a;
    int32_t nb;
    sep_match_args(sg, sep_layout(height, width, cfg->nbins), sp.ay, sp.mass,
                   (const char*)d_ws + (size_t)scale_idx * L.set_bytes, d_template, r.x0, r.y0,
                   r.x1, r.y1, d_map, a, nb);
    return sep_launch_match(a, nb, (hipStream_t)stream) == hipSuccess ? SWIH_OK : SWIH_ERR_HIP;
  }
  if (cfg->kernel == SWIH_EXPONENTIAL) {
    ExpScale es;
    exp_scale(sc.w, sc.h, es);
    ExpMatchArgs a;
    int32_t nb;
    exp_match_args(L, es, scale_idx, (const char*)d_ws, d_template, r.x0, r.y0, r.x1, r.y1, d_map,
                   a, nb);
    return exp_launch_match(a, nb, (hipStream_t)stream) == hipSuccess ? SWIH_OK : SWIH_ERR_HIP;
  }
  const int set = cfg->kernel == SWIH_GAUSSIAN ? scale_idx : 0;
  int32_t* acc = nullptr;
  if (noalloc && cfg->kernel == SWIH_GAUSSIAN) {
    acc = noalloc_scratch();
    if (!acc) return SWIH_ERR_HIP;
  }
  return launch_match(L, sp, set, (const char*)d_ws, d_template, d_template_raw, r.x0, r.y0, r.x1,
                      r.y1, d_map, (hipStream_t)stream, acc) == hipSuccess
             ? SWIH_OK
             : SWIH_ERR_HIP;
}

}  // namespace

extern "C" {

int swih_match(const swih_config* cfg, const void* d_ws, size_t ws_bytes, int32_t height,
               int32_t width, int32_t scale_idx, const float* d_template,
               const uint32_t* d_template_raw, swih_rect r, float* d_map, void* stream) {
  return match_impl(cfg, d_ws, ws_bytes, height, width, scale_idx, d_template, d_template_raw, r,
                    d_map, stream, false);
}

int swih_match_noalloc(const swih_config* cfg, const void* d_ws, size_t ws_bytes, int32_t height,
                       int32_t width, int32_t scale_idx, const float* d_template,
                       const uint32_t* d_template_raw, swih_rect r, float* d_map, void* stream) {
  return match_impl(cfg, d_ws, ws_bytes, height, width, scale_idx, d_template, d_template_raw, r,
                    d_map, stream, true);
}

}  // extern "C"

// ---------------------------------------------------------------- baselines
namespace {

// Shared checks of the wedding-cake calls: an integer kernel, a valid scale
// and ring count, a workspace built for cfg.
int cake_setup(const swih_config* cfg, const void* d_ws, size_t ws_bytes, int32_t height,
               int32_t width, int32_t scale_idx, int32_t rings, CakeArgs& a) {
  int st = check_config(cfg, height, width);
  if (st != SWIH_OK) return st;
  if (scale_idx < 0 || scale_idx >= cfg->nscales || !d_ws) return SWIH_ERR_INVALID;
  if (real_kind(cfg->kernel)) return SWIH_ERR_UNSUPPORTED;  // needs the count plane
  if (rings < 1 || rings > SWIH_MAX_RINGS) return SWIH_ERR_INVALID;
  SwihLayout L;
  make_layout(cfg, height, width, L);
  if ((int64_t)ws_bytes < L.total) return SWIH_ERR_WORKSPACE;
  ScaleParams sp;
  st = scale_params(cfg, scale_idx, sp);
  if (st != SWIH_OK) return st;
  if (cake_args(cfg->kernel, L.g, sp.w, sp.h, rings, sp.mass, sp.c_int,
                (const char*)d_ws + L.off_planes, a))
    return SWIH_ERR_INVALID;
  return SWIH_OK;
}

}  // namespace

extern "C" {

int swih_cake_query(const swih_config* cfg, const void* d_ws, size_t ws_bytes, int32_t height,
                    int32_t width, int32_t scale_idx, int32_t rings, const int32_t* d_centres,
                    int32_t n, float* d_hist, void* stream) {
  CakeArgs a;
  int st = cake_setup(cfg, d_ws, ws_bytes, height, width, scale_idx, rings, a);
  if (st != SWIH_OK) return st;
  if (n < 0) return SWIH_ERR_INVALID;
  if (n == 0) return SWIH_OK;
  if (!d_centres || !d_hist) return SWIH_ERR_INVALID;
  a.centres = d_centres;
  a.n = n;
  a.hist = d_hist;
  return cake_launch_query(a, (hipStream_t)stream) == hipSuccess ? SWIH_OK : SWIH_ERR_HIP;
}

int swih_cake_match(const swih_config* cfg, const void* d_ws, size_t ws_bytes, int32_t height,
                    int32_t width, int32_t scale_idx, int32_t rings, const float* d_template,
                    swih_rect r, float* d_map, void* stream) {
  CakeArgs a;
  int st = cake_setup(cfg, d_ws, ws_bytes, height, width, scale_idx, rings, a);
  if (st != SWIH_OK) return st;
  if (!d_template) return SWIH_ERR_INVALID;
  if (r.x1 < r.x0 || r.y1 < r.y0) return SWIH_OK;
  const swih_scale sc = cfg->scales[scale_idx];
  const int32_t rx = (sc.w - 1) / 2, ry = (sc.h - 1) / 2;
  if (r.x0 < rx || r.y0 < ry || r.x1 > width - 1 - rx || r.y1 > height - 1 - ry || !d_map)
    return SWIH_ERR_INVALID;
  a.tmpl = d_template;
  a.map = d_map;
  a.x0 = r.x0;
  a.y0 = r.y0;
  a.x1 = r.x1;
  a.y1 = r.y1;
  a.nbx = (r.x1 - r.x0 + 1 + 63) / 64;
  return cake_launch_match(a, (hipStream_t)stream) == hipSuccess ? SWIH_OK : SWIH_ERR_HIP;
}

int swih_brute_match(const swih_config* cfg, const uint8_t* d_img, int32_t height, int32_t width,
                     int32_t pitch, int32_t scale_idx, const uint32_t* d_template_raw, swih_rect r,
                     float* d_map, void* stream) {
  int st = check_config(cfg, height, width);
  if (st != SWIH_OK) return st;
  if (scale_idx < 0 || scale_idx >= cfg->nscales || !d_img || pitch < width || !d_template_raw)
    return SWIH_ERR_INVALID;
  if (real_kind(cfg->kernel)) return SWIH_ERR_UNSUPPORTED;  // exact integer kernels only
  if (r.x1 < r.x0 || r.y1 < r.y0) return SWIH_OK;
  ScaleParams sp;
  st = scale_params(cfg, scale_idx, sp);
  if (st != SWIH_OK) return st;
  if (r.x0 < sp.rx || r.y0 < sp.ry || r.x1 > width - 1 - sp.rx || r.y1 > height - 1 - sp.ry || !d_map)
    return SWIH_ERR_INVALID;
  BruteArgs a;
  memset(&a, 0, sizeof(a));
  a.img = d_img;
  a.ipitch = pitch;
  a.H = height;
  a.W = width;
  a.B = cfg->nbins;
  a.kind = cfg->kernel;
  a.rx = sp.rx;
  a.ry = sp.ry;
  a.c_int = sp.c_int;
  a.mass = sp.mass;
  a.tmpl_raw = d_template_raw;
  a.map = d_map;
  a.x0 = r.x0;
  a.y0 = r.y0;
  a.x1 = r.x1;
  a.y1 = r.y1;
  a.nbx = (r.x1 - r.x0 + 1 + 63) / 64;
  return brute_launch_match(a, (hipStream_t)stream) == hipSuccess ? SWIH_OK : SWIH_ERR_HIP;
}

}  // extern "C"

// ---------------------------------------------------------------- batches
namespace {

constexpr uint32_t kBatchMagic = 0x53574842u;  // "SWHB"
constexpr int kBatchGrid = 4096;               // blocks per grid-stride launch

struct BatchHeader {
  uint32_t magic;
  int32_t kind, nt, nbins;
  int32_t nunits, nq, nm;
  int32_t total[4];   // build-stage virtual blocks
  Launch ql, ml;      // query / map launch shapes (blocks = total virtual blocks)
  int64_t off_units, off_uprefix, off_q, off_qprefix, off_m, off_mprefix;
  // the fused launch (swih_run_batch): build-stage prefixes in its block
  // size, the unit each query / map reads, its counters
  int64_t off_fprefix, off_qunit, off_munit, off_sync, bytes;
  int32_t fcum[7];    // first ticket of each stage, then the total
  int32_t fused_ok;   // the kind has a fused form
};

int32_t frame_units(const swih_config* cfg, const swih_frame_desc& f) {
  if (!per_scale(cfg->kernel)) return 1;
  return f.nscales > 0 ? f.nscales : cfg->nscales;
}

// Offsets of every table section for the given counts (item records of the
// separable and exponential kinds are their own argument structs).
BatchHeader table_layout(int32_t kind, int32_t nunits, int32_t nq, int32_t nm) {
  BatchHeader h;
  memset(&h, 0, sizeof(h));
  const bool sep = kind == SWIH_GAUSSIAN_SEP, ex = kind == SWIH_EXPONENTIAL;
  const size_t ub = sep ? sizeof(SepBuildArgs) : (ex ? sizeof(ExpBuildArgs) : sizeof(BuildArgs));
  const size_t qb = sep ? sizeof(SepQueryArgs) : (ex ? sizeof(ExpQueryArgs) : sizeof(QueryArgs));
  const size_t mb = sep ? sizeof(SepMatchArgs) : (ex ? sizeof(ExpMatchArgs) : sizeof(MatchArgs));
  int64_t off = swih_align256(sizeof(BatchHeader));
  h.off_units = off;
  off += swih_align256((int64_t)nunits * ub);
  h.off_uprefix = off;
  off += swih_align256((int64_t)4 * (nunits + 1) * sizeof(int32_t));
  h.off_q = off;
  off += swih_align256((int64_t)nq * qb);
  h.off_qprefix = off;
  off += swih_align256((int64_t)(nq + 1) * sizeof(int32_t));
  h.off_m = off;
  off += swih_align256((int64_t)nm * mb);
  h.off_mprefix = off;
  off += swih_align256((int64_t)(nm + 1) * sizeof(int32_t));
  h.off_fprefix = off;
  off += swih_align256((int64_t)4 * (nunits + 1) * sizeof(int32_t));
  h.off_qunit = off;
  off += swih_align256((int64_t)nq * sizeof(int32_t));
  h.off_munit = off;
  off += swih_align256((int64_t)nm * sizeof(int32_t));
  h.off_sync = off;
  off += swih_align256(fused_sync_words(nunits) * (int64_t)sizeof(int32_t));
  h.bytes = off;
  h.nunits = nunits;
  h.nq = nq;
  h.nm = nm;
  return h;
}

// The frame's own configuration: the batch configuration with its scales and
// scan-tile rows.
swih_config frame_config(const swih_config* cfg, const swih_frame_desc& f) {
  swih_config c = *cfg;
  if (f.nscales > 0) {
    c.nscales = f.nscales;
    c.scales = f.scales;
  }
  if (f.band_rows != 0) c.band_rows = f.band_rows;
  return c;
}

const BatchHeader* header_of(const void* h_table) {
  const BatchHeader* h = (const BatchHeader*)h_table;
  return (h && h->magic == kBatchMagic) ? h : nullptr;
}

}  // namespace

extern "C" {

int64_t swih_batch_table_bytes(const swih_config* cfg, const swih_frame_desc* frames,
                               int32_t nframes, int32_t nqueries, int32_t nmatches) {
  if (!cfg || nframes < 0 || nqueries < 0 || nmatches < 0 || (nframes > 0 && !frames))
    return SWIH_ERR_INVALID;
  int64_t nunits = 0;
  for (int f = 0; f < nframes; ++f) nunits += frame_units(cfg, frames[f]);
  if (nunits > (1 << 24)) return SWIH_ERR_INVALID;
  return table_layout(cfg->kernel, (int32_t)nunits, nqueries, nmatches).bytes;
}

int swih_batch_plan(const swih_config* cfg, const swih_frame_desc* frames, int32_t nframes,
                    const swih_query_desc* queries, int32_t nqueries,
                    const swih_match_desc* matches, int32_t nmatches, void* h_table,
                    size_t table_bytes) {
  if (!cfg || !h_table || nframes < 0 || nqueries < 0 || nmatches < 0) return SWIH_ERR_INVALID;
  if ((nframes > 0 && !frames) || (nqueries > 0 && !queries) || (nmatches > 0 && !matches))
    return SWIH_ERR_INVALID;
  const int64_t need = swih_batch_table_bytes(cfg, frames, nframes, nqueries, nmatches);
  if (need < 0) return (int)need;
  if ((int64_t)table_bytes < need) return SWIH_ERR_WORKSPACE;
  const bool gauss = cfg->kernel == SWIH_GAUSSIAN;
  const bool sep = cfg->kernel == SWIH_GAUSSIAN_SEP;
  const bool ex = cfg->kernel == SWIH_EXPONENTIAL;
  // frames: check, lay out, and fill one build unit per plane set
  std::vector<SwihLayout> layouts(nframes);
  std::vector<int32_t> ubase(nframes + 1, 0);
  for (int f = 0; f < nframes; ++f) {
    const swih_frame_desc& fd = frames[f];
    const swih_config fc = frame_config(cfg, fd);
    int st = check_config(&fc, fd.height, fd.width);
    if (st != SWIH_OK) return st;
    if (!fd.d_img || !fd.d_ws || fd.pitch < fd.width || !aligned256(fd.d_ws)) return SWIH_ERR_INVALID;
    if (fd.nscales > 0 && !fd.scales) return SWIH_ERR_INVALID;
    make_layout(&fc, fd.height, fd.width, layouts[f]);
    if ((int64_t)fd.ws_bytes < layouts[f].total) return SWIH_ERR_WORKSPACE;
    for (int k = 0; k < fc.nscales; ++k) {
      ScaleParams sp;
      st = scale_params(&fc, k, sp);
      if (st != SWIH_OK) return st;
    }
    ubase[f + 1] = ubase[f] + frame_units(cfg, fd);
  }
  const int32_t nunits = ubase[nframes];
  BatchHeader h = table_layout(cfg->kernel, nunits, nqueries, nmatches);
  h.magic = kBatchMagic;
  h.kind = cfg->kernel;
  h.nt = series_kind(cfg->kernel) ? 2 * gauss_K(cfg) + 1 : 0;
  h.nbins = cfg->nbins;
  char* tb = (char*)h_table;
  memset(tb, 0, (size_t)h.bytes);
  BuildArgs* units = (BuildArgs*)(tb + h.off_units);
  SepBuildArgs* sunits = (SepBuildArgs*)(tb + h.off_units);
  ExpBuildArgs* eunits = (ExpBuildArgs*)(tb + h.off_units);
  int32_t* upre = (int32_t*)(tb + h.off_uprefix);
  for (int f = 0; f < nframes; ++f) {
    if (ex) {
      const swih_frame_desc& fd = frames[f];
      const swih_config fc = frame_config(cfg, fd);
      for (int k = 0; k < ubase[f + 1] - ubase[f]; ++k) {
        const int u = ubase[f] + k;
        ExpScale es;
        exp_scale(fc.scales[k].w, fc.scales[k].h, es);
        int32_t nb[4];
        exp_build_args(layouts[f], es, k, fd.d_img, fd.pitch, (char*)fd.d_ws, eunits[u], nb);
        for (int s = 0; s < 4; ++s) upre[s * (nunits + 1) + u + 1] = upre[s * (nunits + 1) + u] + nb[s];
      }
      continue;
    }
    if (sep) {
      const swih_frame_desc& fd = frames[f];
      const swih_config fc = frame_config(cfg, fd);
      const SepLayout SL = sep_layout(fd.height, fd.width, cfg->nbins);
      for (int k = 0; k < ubase[f + 1] - ubase[f]; ++k) {
        const int u = ubase[f] + k;
        ScaleParams sp;
        scale_params(&fc, k, sp);
        const SepGeom sg = sep_geom(fd.height, fd.width, cfg->nbins, sp.w, sp.h, (h.nt - 1) / 2);
        int32_t nb[2];
        sep_build_args(sg, SL, sp.ax, fd.d_img, fd.pitch,
                       (char*)fd.d_ws + (size_t)k * layouts[f].set_bytes, sunits[u], nb);
        for (int s = 0; s < 4; ++s)
          upre[s * (nunits + 1) + u + 1] = upre[s * (nunits + 1) + u] + (s < 2 ? nb[s] : 0);
      }
      continue;
    }
    const swih_frame_desc& fd = frames[f];
    const swih_config fc = frame_config(cfg, fd);
    for (int k = 0; k < ubase[f + 1] - ubase[f]; ++k) {
      const int u = ubase[f] + k;
      ScaleParams sp;
      scale_params(&fc, gauss ? k : 0, sp);
      int32_t nb[4];
      build_args(layouts[f], k, gauss ? &sp.ax : nullptr, gauss ? &sp.ay : nullptr, sp.rx, sp.ry, fd.d_img,
                 fd.pitch, (char*)fd.d_ws, units[u], nb, true);
      for (int s = 0; s < 4; ++s) upre[s * (nunits + 1) + u + 1] = upre[s * (nunits + 1) + u] + nb[s];
    }
  }
  for (int s = 0; s < 4; ++s) h.total[s] = upre[s * (nunits + 1) + nunits];
  // the fused launch's build prefixes: a virtual block of its size covers
  // `ratio` 256-thread ones of the same unit
  h.fused_ok = cfg->kernel <= SWIH_GAUSSIAN && !sep && !ex;
  {
    const int ratio = fused_build_ratio(cfg->kernel);
    int32_t* fpre = (int32_t*)(tb + h.off_fprefix);
    for (int s = 0; s < 4; ++s)
      for (int u = 0; u < nunits; ++u) {
        const int32_t nb = upre[s * (nunits + 1) + u + 1] - upre[s * (nunits + 1) + u];
        fpre[s * (nunits + 1) + u + 1] = fpre[s * (nunits + 1) + u] + (nb + ratio - 1) / ratio;
      }
    for (int s = 0; s < 4; ++s) h.fcum[s + 1] = h.fcum[s] + fpre[s * (nunits + 1) + nunits];
  }
  // queries
  QueryArgs* qa = (QueryArgs*)(tb + h.off_q);
  int32_t* qpre = (int32_t*)(tb + h.off_qprefix);
  h.ql.threads = 256;
  for (int q = 0; q < nqueries; ++q) {
    const swih_query_desc& qd = queries[q];
    if (qd.frame < 0 || qd.frame >= nframes || qd.n < 0) return SWIH_ERR_INVALID;
    const swih_config fc = frame_config(cfg, frames[qd.frame]);
    if (qd.scale_idx < 0 || qd.scale_idx >= fc.nscales) return SWIH_ERR_INVALID;
    if (real_kind(cfg->kernel) && qd.d_hist_raw) return SWIH_ERR_UNSUPPORTED;
    if (qd.n > 0 && (!qd.d_centres || (!qd.d_hist && !qd.d_hist_raw))) return SWIH_ERR_INVALID;
    if (ex) {
      ExpScale es;
      exp_scale(fc.scales[qd.scale_idx].w, fc.scales[qd.scale_idx].h, es);
      int32_t nb = 0;
      exp_query_args(layouts[qd.frame], es, qd.scale_idx, (const char*)frames[qd.frame].d_ws,
                     qd.d_centres, qd.n, qd.d_hist, ((ExpQueryArgs*)(tb + h.off_q))[q], nb);
      qpre[q + 1] = qpre[q] + (qd.n > 0 ? nb : 0);
      continue;
    }
    ScaleParams sp;
    scale_params(&fc, qd.scale_idx, sp);
    if (sep) {
      const swih_frame_desc& fd = frames[qd.frame];
      const SepGeom sg = sep_geom(fd.height, fd.width, cfg->nbins, sp.w, sp.h, (h.nt - 1) / 2);
      int32_t nb = 0;
      sep_query_args(sg, sep_layout(fd.height, fd.width, cfg->nbins), sp.ay, sp.mass,
                     (const char*)fd.d_ws + (size_t)qd.scale_idx * layouts[qd.frame].set_bytes,
                     qd.d_centres, qd.n, qd.d_hist, ((SepQueryArgs*)(tb + h.off_q))[q], nb);
      qpre[q + 1] = qpre[q] + (qd.n > 0 ? nb : 0);
      continue;
    }
    Launch ql;
    query_args(layouts[qd.frame], sp, gauss ? qd.scale_idx : 0, (const char*)frames[qd.frame].d_ws,
               qd.d_centres, qd.n, qd.d_hist, qd.d_hist_raw, qa[q], ql);
    qpre[q + 1] = qpre[q] + (qd.n > 0 ? ql.blocks : 0);
    if (ql.lds > h.ql.lds) h.ql.lds = ql.lds;
  }
  h.ql.blocks = qpre[nqueries];
  h.fcum[5] = h.fcum[4] + h.ql.blocks;
  {
    int32_t* qu = (int32_t*)(tb + h.off_qunit);
    for (int q = 0; q < nqueries; ++q)
      qu[q] = ubase[queries[q].frame] + (per_scale(cfg->kernel) ? queries[q].scale_idx : 0);
  }
  // maps
  MatchArgs* ma = (MatchArgs*)(tb + h.off_m);
  int32_t* mpre = (int32_t*)(tb + h.off_mprefix);
  for (int m = 0; m < nmatches; ++m) {
    const swih_match_desc& md = matches[m];
    if (md.frame < 0 || md.frame >= nframes) return SWIH_ERR_INVALID;
    const swih_frame_desc& fd = frames[md.frame];
    const swih_config fc = frame_config(cfg, fd);
    if (md.scale_idx < 0 || md.scale_idx >= fc.nscales) return SWIH_ERR_INVALID;
    if ((md.d_template == nullptr) == (md.d_template_raw == nullptr)) return SWIH_ERR_INVALID;
    if (real_kind(cfg->kernel) && md.d_template_raw) return SWIH_ERR_UNSUPPORTED;
    const swih_rect r = md.centres;
    const bool empty = r.x1 < r.x0 || r.y1 < r.y0;
    if (!empty) {
      const swih_scale sc = fc.scales[md.scale_idx];
      const int32_t rx = (sc.w - 1) / 2, ry = (sc.h - 1) / 2;
      if (r.x0 < rx || r.y0 < ry || r.x1 > fd.width - 1 - rx || r.y1 > fd.height - 1 - ry || !md.d_map)
        return SWIH_ERR_INVALID;
    }
    if (ex) {
      int32_t nb = 0;
      if (!empty) {
        ExpScale es;
        exp_scale(fc.scales[md.scale_idx].w, fc.scales[md.scale_idx].h, es);
        exp_match_args(layouts[md.frame], es, md.scale_idx, (const char*)fd.d_ws, md.d_template,
                       r.x0, r.y0, r.x1, r.y1, md.d_map, ((ExpMatchArgs*)(tb + h.off_m))[m], nb);
      }
      mpre[m + 1] = mpre[m] + nb;
      continue;
    }
    ScaleParams sp;
    scale_params(&fc, md.scale_idx, sp);
    if (sep) {
      int32_t nb = 0;
      if (!empty) {
        const SepGeom sg = sep_geom(fd.height, fd.width, cfg->nbins, sp.w, sp.h, (h.nt - 1) / 2);
        sep_match_args(sg, sep_layout(fd.height, fd.width, cfg->nbins), sp.ay, sp.mass,
                       (const char*)fd.d_ws + (size_t)md.scale_idx * layouts[md.frame].set_bytes,
                       md.d_template, r.x0, r.y0, r.x1, r.y1, md.d_map,
                       ((SepMatchArgs*)(tb + h.off_m))[m], nb);
      }
      mpre[m + 1] = mpre[m] + nb;
      continue;
    }
    Launch ml;
    memset(&ml, 0, sizeof(ml));
    if (!empty)
      match_args(layouts[md.frame], sp, gauss ? md.scale_idx : 0, (const char*)fd.d_ws,
                 md.d_template, md.d_template_raw, r.x0, r.y0, r.x1, r.y1, md.d_map, ma[m], ml);
    mpre[m + 1] = mpre[m] + (empty ? 0 : ml.blocks);
    if (ml.threads > h.ml.threads) h.ml.threads = ml.threads;
    if (ml.lds > h.ml.lds) h.ml.lds = ml.lds;
  }
  h.ml.blocks = mpre[nmatches];
  h.fcum[6] = h.fcum[5] + h.ml.blocks;
  {
    int32_t* mu = (int32_t*)(tb + h.off_munit);
    for (int m = 0; m < nmatches; ++m)
      mu[m] = ubase[matches[m].frame] + (per_scale(cfg->kernel) ? matches[m].scale_idx : 0);
  }
  if (h.ml.threads == 0) h.ml.threads = 256;
  if (h.ml.lds > 160 * 1024) return SWIH_ERR_UNSUPPORTED;
  memcpy(tb, &h, sizeof(h));
  return SWIH_OK;
}

int swih_build_batch(const void* h_table, const void* d_table, void* stream) {
  const BatchHeader* h = header_of(h_table);
  if (!h || !d_table || !aligned256(d_table)) return SWIH_ERR_INVALID;
  const char* db = (const char*)d_table;
  if (h->kind == SWIH_GAUSSIAN_SEP) {
    const int32_t tot[2] = {h->total[0], h->total[1]};
    return sep_launch_build_batch(h->nt, h->nbins, (const SepBuildArgs*)(db + h->off_units),
                                  (const int32_t*)(db + h->off_uprefix), h->nunits, tot,
                                  kBatchGrid, (hipStream_t)stream) == hipSuccess
               ? SWIH_OK
               : SWIH_ERR_HIP;
  }
  if (h->kind == SWIH_EXPONENTIAL)
    return exp_launch_build_batch((const ExpBuildArgs*)(db + h->off_units),
                                  (const int32_t*)(db + h->off_uprefix), h->nunits, h->nbins, h->total,
                                  kBatchGrid, (hipStream_t)stream) == hipSuccess
               ? SWIH_OK
               : SWIH_ERR_HIP;
  return launch_build_batch(h->kind, h->nt, h->nbins, (const BuildArgs*)(db + h->off_units),
                            (const int32_t*)(db + h->off_uprefix), h->nunits, h->total, kBatchGrid,
                            (hipStream_t)stream) == hipSuccess
             ? SWIH_OK
             : SWIH_ERR_HIP;
}

int swih_query_batch(const void* h_table, const void* d_table, void* stream) {
  const BatchHeader* h = header_of(h_table);
  if (!h || !d_table || !aligned256(d_table)) return SWIH_ERR_INVALID;
  const char* db = (const char*)d_table;
  if (h->kind == SWIH_GAUSSIAN_SEP)
    return sep_launch_query_batch(h->nt, h->nbins, (const SepQueryArgs*)(db + h->off_q),
                                  (const int32_t*)(db + h->off_qprefix), h->nq, h->ql.blocks,
                                  kBatchGrid, (hipStream_t)stream) == hipSuccess
               ? SWIH_OK
               : SWIH_ERR_HIP;
  if (h->kind == SWIH_EXPONENTIAL)
    return exp_launch_query_batch((const ExpQueryArgs*)(db + h->off_q),
                                  (const int32_t*)(db + h->off_qprefix), h->nq, h->ql.blocks,
                                  kBatchGrid, (hipStream_t)stream) == hipSuccess
               ? SWIH_OK
               : SWIH_ERR_HIP;
  return launch_query_batch(h->kind, h->nt, (const QueryArgs*)(db + h->off_q),
                            (const int32_t*)(db + h->off_qprefix), h->nq, h->ql, kBatchGrid,
                            (hipStream_t)stream) == hipSuccess
             ? SWIH_OK
             : SWIH_ERR_HIP;
}

int swih_match_batch(const void* h_table, const void* d_table, void* stream) {
  const BatchHeader* h = header_of(h_table);
  if (!h || !d_table || !aligned256(d_table)) return SWIH_ERR_INVALID;
  const char* db = (const char*)d_table;
  if (h->kind == SWIH_GAUSSIAN_SEP)
    return sep_launch_match_batch(h->nt, h->nbins, (const SepMatchArgs*)(db + h->off_m),
                                  (const int32_t*)(db + h->off_mprefix), h->nm, h->ml.blocks,
                                  kBatchGrid, (hipStream_t)stream) == hipSuccess
               ? SWIH_OK
               : SWIH_ERR_HIP;
  if (h->kind == SWIH_EXPONENTIAL)
    return exp_launch_match_batch((const ExpMatchArgs*)(db + h->off_m),
                                  (const int32_t*)(db + h->off_mprefix), h->nm, h->ml.blocks,
                                  kBatchGrid, (hipStream_t)stream) == hipSuccess
               ? SWIH_OK
               : SWIH_ERR_HIP;
  return launch_match_batch(h->kind, h->nt, (const MatchArgs*)(db + h->off_m),
                            (const int32_t*)(db + h->off_mprefix), h->nm, h->ml, kBatchGrid,
                            (hipStream_t)stream) == hipSuccess
             ? SWIH_OK
             : SWIH_ERR_HIP;
}

int swih_run_batch(const void* h_table, void* d_table, int32_t* d_status, int32_t wait_ms,
                   void* stream) {
  const BatchHeader* h = header_of(h_table);
  if (!h || !d_table || !aligned256(d_table)) return SWIH_ERR_INVALID;
  if (!h->fused_ok) return SWIH_ERR_UNSUPPORTED;
  char* db = (char*)d_table;
  FusedArgs f;
  memset(&f, 0, sizeof(f));
  f.units = (const BuildArgs*)(db + h->off_units);
  f.q = (const QueryArgs*)(db + h->off_q);
  f.m = (const MatchArgs*)(db + h->off_m);
  f.upre = (const int32_t*)(db + h->off_fprefix);
  f.qpre = (const int32_t*)(db + h->off_qprefix);
  f.mpre = (const int32_t*)(db + h->off_mprefix);
  f.qunit = (const int32_t*)(db + h->off_qunit);
  f.munit = (const int32_t*)(db + h->off_munit);
  f.nunits = h->nunits;
  f.nq = h->nq;
  f.nm = h->nm;
  for (int k = 0; k < 7; ++k) f.cum[k] = h->fcum[k];
  f.sync = (int32_t*)(db + h->off_sync);
  f.status = d_status;
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    return SWIH_ERR_HIP;
  const int64_t ms = wait_ms == 0 ? 2000 : wait_ms;
  f.limit = ms < 0 ? -1 : ms * (int64_t)khz;
  const size_t lds = h->ql.lds > h->ml.lds ? h->ql.lds : h->ml.lds;
  const hipError_t e = launch_fused(h->kind, h->nt, h->nbins, f, lds, (hipStream_t)stream);
  if (e == hipErrorInvalidValue) return SWIH_ERR_UNSUPPORTED;
  return e == hipSuccess ? SWIH_OK : SWIH_ERR_HIP;
}

int swih_gauss_terms(int32_t n, int32_t K, double* a_out, double* omega_out, double* err_out) {
  double a[SWIH_MAX_K + 1], om[SWIH_MAX_K + 1];
  double e = 0.0;
  if (K < 1 || K > SWIH_MAX_K) return SWIH_ERR_INVALID;
  if (gauss_fit(n, K, a, om, &e)) return SWIH_ERR_INVALID;
  for (int k = 0; k <= K; ++k) {
    if (a_out) a_out[k] = a[k];
    if (omega_out) omega_out[k] = om[k];
  }
  if (err_out) *err_out = e;
  return SWIH_OK;
}

const char* swih_status_string(int status) {
  switch (status) {
    case SWIH_OK: return "ok";
    case SWIH_ERR_INVALID: return "invalid argument";
    case SWIH_ERR_WORKSPACE: return "workspace too small";
    case SWIH_ERR_UNSUPPORTED: return "unsupported for this kernel";
    case SWIH_ERR_HIP: return "HIP launch failed";
    case SWIH_ERR_SCRATCH: return "rectangle larger than the static scratch of swih_match_noalloc";
    default: return "unknown status";
  }
}

}  // extern "C"
