// C ABI of libswih.so: argument checks, workspace layout and launches.
#include <string.h>

#include "swih.h"
#include "swih_internal.h"

namespace swih {
namespace {

constexpr int32_t kMaxSide = 8192;
constexpr int32_t kDefaultTY = 64;

bool kind_ok(int32_t k) { return k >= SWIH_UNIFORM && k <= SWIH_GAUSSIAN; }

int32_t gauss_K(const swih_config* c) { return c->gauss_terms == 0 ? 4 : c->gauss_terms; }

// Checks the configuration against an image size; returns a status.
int check_config(const swih_config* c, int32_t H, int32_t W) {
  if (!c || H < 1 || W < 1 || H > kMaxSide || W > kMaxSide) return SWIH_ERR_INVALID;
  if (c->nbins < 1 || c->nbins > 256 || !kind_ok(c->kernel) || c->flags != 0)
    return SWIH_ERR_INVALID;
  if (c->nscales < 1 || !c->scales) return SWIH_ERR_INVALID;
  if (c->kernel == SWIH_GAUSSIAN) {
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
  g.TY = kDefaultTY;
  g.NTX = (W + SWIH_TX - 1) / SWIH_TX;
  g.NTY = (H + g.TY - 1) / g.TY;
  g.pitch = SWIH_TX * (g.NTX + 1);
  g.plane_elems = (int64_t)(H + 1) * g.pitch;
  const bool gauss = c->kernel == SWIH_GAUSSIAN;
  g.gauss = gauss ? 1 : 0;
  if (gauss) {
    g.nI = g.nJ = 2 * gauss_K(c) + 1;
    g.nP = g.nI * g.nJ;
    g.ppg = g.nJ;
  } else {
    static const int nI[3] = {1, 2, 3}, nP[3] = {1, 3, 5};
    g.nI = g.nJ = nI[c->kernel];
    g.nP = nP[c->kernel];
    g.ppg = g.nP;
  }
  g.row_stride = (int64_t)g.ppg * g.pitch;
  const int64_t PB = (int64_t)g.nP * g.B;
  const int64_t NXP = (int64_t)g.NTX * SWIH_TX;
  int64_t off = 0;
  L.off_planes = off;
  off += swih_align256(PB * g.plane_elems * 4);
  if (gauss) {
    L.off_RC = off;
    off += swih_align256(PB * g.NTX * (int64_t)(H + 1) * 8);
    L.off_uq = off;
    off += swih_align256((int64_t)g.nI * NXP * 4);
    L.off_vq = off;  // int32 [H][nJ], then double [H][nJ]
    off += swih_align256((int64_t)g.nJ * H * 4) + swih_align256((int64_t)g.nJ * H * 8);
  }
  L.set_bytes = off;
  L.nsets = gauss ? c->nscales : 1;
  const int64_t esz = gauss ? 8 : 4;
  off = L.set_bytes * L.nsets;
  L.off_scratch = off;
  L.off_z = off;
  if (!gauss) off += swih_align256((int64_t)g.nJ * g.B * g.NTY * NXP * esz);
  L.off_T = off;
  off += swih_align256((int64_t)g.nI * g.B * g.NTX * (int64_t)H * esz);
  L.off_CT = off;
  off += swih_align256(PB * g.NTY * g.NTX * esz);
  L.total = off;
  return SWIH_OK;
}

int fill_axis(int32_t n, int32_t K, GaussAxis& ax) {
  memset(&ax, 0, sizeof(ax));
  ax.K = K;
  int P = 0;
  if (gauss_fit(n, K, ax.a, &P, nullptr)) return SWIH_ERR_INVALID;
  ax.P = P;
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
  if (c->kernel == SWIH_GAUSSIAN) {
    const int32_t K = gauss_K(c);
    if (fill_axis(sc.w, K, sp.ax) || fill_axis(sc.h, K, sp.ay)) return SWIH_ERR_INVALID;
    sp.mass = gauss_axis_mass(sc.w, K, sp.ax.a, sp.ax.P) * gauss_axis_mass(sc.h, K, sp.ay.a, sp.ay.P);
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
  for (int k = first; k <= last; ++k) {
    ScaleParams sp;
    scale_params(cfg, gauss ? k : 0, sp);
    if (launch_build(L, cfg->kernel, k, gauss ? &sp.ax : nullptr, gauss ? &sp.ay : nullptr, d_img,
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
  if (cfg->kernel == SWIH_GAUSSIAN && d_hist_raw) return SWIH_ERR_UNSUPPORTED;
  if (n == 0) return SWIH_OK;
  if (!d_centres || (!d_hist && !d_hist_raw)) return SWIH_ERR_INVALID;
  SwihLayout L;
  make_layout(cfg, height, width, L);
  if ((int64_t)ws_bytes < L.total) return SWIH_ERR_WORKSPACE;
  ScaleParams sp;
  st = scale_params(cfg, scale_idx, sp);
  if (st != SWIH_OK) return st;
  const int set = cfg->kernel == SWIH_GAUSSIAN ? scale_idx : 0;
  return launch_query(L, sp, set, (const char*)d_ws, d_centres, n, d_hist, d_hist_raw,
                      (hipStream_t)stream) == hipSuccess
             ? SWIH_OK
             : SWIH_ERR_HIP;
}

int swih_match(const swih_config* cfg, const void* d_ws, size_t ws_bytes, int32_t height,
               int32_t width, int32_t scale_idx, const float* d_template,
               const uint32_t* d_template_raw, swih_rect r, float* d_map, void* stream) {
  int st = check_config(cfg, height, width);
  if (st != SWIH_OK) return st;
  if (scale_idx < 0 || scale_idx >= cfg->nscales || !d_ws) return SWIH_ERR_INVALID;
  if ((d_template == nullptr) == (d_template_raw == nullptr)) return SWIH_ERR_INVALID;
  if (cfg->kernel == SWIH_GAUSSIAN && d_template_raw) return SWIH_ERR_UNSUPPORTED;
  if (r.x1 < r.x0 || r.y1 < r.y0) return SWIH_OK;
  const swih_scale sc = cfg->scales[scale_idx];
  const int32_t rx = (sc.w - 1) / 2, ry = (sc.h - 1) / 2;
  if (r.x0 < rx || r.y0 < ry || r.x1 > width - 1 - rx || r.y1 > height - 1 - ry)
    return SWIH_ERR_INVALID;
  if (!d_map) return SWIH_ERR_INVALID;
  SwihLayout L;
  make_layout(cfg, height, width, L);
  if ((int64_t)ws_bytes < L.total) return SWIH_ERR_WORKSPACE;
  ScaleParams sp;
  st = scale_params(cfg, scale_idx, sp);
  if (st != SWIH_OK) return st;
  const int set = cfg->kernel == SWIH_GAUSSIAN ? scale_idx : 0;
  return launch_match(L, sp, set, (const char*)d_ws, d_template, d_template_raw, r.x0, r.y0, r.x1,
                      r.y1, d_map, (hipStream_t)stream) == hipSuccess
             ? SWIH_OK
             : SWIH_ERR_HIP;
}

int swih_gauss_terms(int32_t n, int32_t K, double* a_out, int32_t* period_out, double* err_out) {
  double a[SWIH_MAX_K + 1];
  int P = 0;
  double e = 0.0;
  if (K < 1 || K > SWIH_MAX_K) return SWIH_ERR_INVALID;
  if (gauss_fit(n, K, a, &P, &e)) return SWIH_ERR_INVALID;
  if (a_out)
    for (int k = 0; k <= K; ++k) a_out[k] = a[k];
  if (period_out) *period_out = P;
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
    default: return "unknown status";
  }
}

}  // extern "C"
