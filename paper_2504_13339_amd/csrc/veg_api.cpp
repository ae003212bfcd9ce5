// extern "C" entry points of libveg: argument checks, descriptor upload, launches.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "veg_internal.h"

using namespace veg;

namespace {

thread_local std::string g_err;

veg_status fail(veg_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

veg_status hip_status(hipError_t e, const char* where) {
  if (e == hipSuccess) return VEG_OK;
  return fail(VEG_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define VEG_CHECK_HIP(expr, where)                     \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_status(e_, where); \
  } while (0)

// Limits the backward pass needs (see veg_render_bwd).
constexpr float kBwdAlphaClampMax = 1.0f - 0x1p-10f;
constexpr double kBwdTFloor = 0x1p-100;

veg_status check_opts(const veg_opts* o) {
  if (!(o->alpha_min > 0.0f) || !(o->alpha_clamp > o->alpha_min) || !(o->alpha_clamp <= 1.0f))
    return fail(VEG_ERR_INVALID_ARG, "opts: need 0 < alpha_min < alpha_clamp <= 1");
  if (!(o->t_min >= 0.0f) || !(o->t_min < 1.0f)) return fail(VEG_ERR_INVALID_ARG, "opts: need 0 <= t_min < 1");
  if (!(o->lowpass >= 0.0f) || !(o->near_z > 0.0f) || !(o->guard > 0.0f))
    return fail(VEG_ERR_INVALID_ARG, "opts: need lowpass >= 0, near_z > 0, guard > 0");
  for (int c = 0; c < 3; ++c)
    if (!std::isfinite(o->bg[c])) return fail(VEG_ERR_INVALID_ARG, "opts: background must be finite");
  return VEG_OK;
}

KOpts kopts(const veg_opts* o) {
  KOpts k;
  k.alpha_clamp = o->alpha_clamp;
  k.alpha_min = o->alpha_min;
  k.t_min = o->t_min;
  k.lowpass = o->lowpass;
  k.near_z = o->near_z;
  k.guard = o->guard;
  k.log2_alpha_min = std::log2(o->alpha_min);
  k.bg0 = o->bg[0];
  k.bg1 = o->bg[1];
  k.bg2 = o->bg[2];
  return k;
}

veg_status resolve_opts(const veg_opts* in, veg_opts* out) {
  if (in) *out = *in;
  else veg_opts_default(out);
  return check_opts(out);
}

veg_status check_proj(const veg_proj* p) {
  if (!p) return fail(VEG_ERR_INVALID_ARG, "proj is NULL");
  if (p->n < 0 || p->n_frames < 1 || p->n_frames > VEG_MAX_FRAMES)
    return fail(VEG_ERR_INVALID_ARG, "proj: bad n (%lld) or n_frames (%d)", (long long)p->n, p->n_frames);
  if ((int64_t)p->n_frames * p->n >= ((int64_t)1 << 31))
    return fail(VEG_ERR_INVALID_ARG, "proj: n_frames * n must be < 2^31");
  if (!p->frames || (p->n > 0 && (!p->rec || !p->count || !p->depth)))
    return fail(VEG_ERR_INVALID_ARG, "proj: NULL buffer");
  return VEG_OK;
}

veg_status check_projected(const veg_proj* p) {
  veg_status s = check_proj(p);
  if (s != VEG_OK) return s;
  if (p->width < 1 || p->height < 1 || p->tiles_x < 1 || p->tiles_y < 1 ||
      p->total_tiles != (int64_t)(p->n_frames / (p->tfs_per_view > 1 ? p->tfs_per_view : 1)) * p->tiles_x * p->tiles_y)
    return fail(VEG_ERR_INVALID_ARG, "proj: not filled by veg_project");
  return VEG_OK;
}

veg_status check_gaussians(const veg_gaussians* g) {
  if (!g) return fail(VEG_ERR_INVALID_ARG, "gaussians is NULL");
  if (g->n < 0) return fail(VEG_ERR_INVALID_ARG, "gaussians: n < 0");
  if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->scalars))
    return fail(VEG_ERR_INVALID_ARG, "gaussians: NULL parameter array");
  if (g->quats && (reinterpret_cast<uintptr_t>(g->quats) & 15u))
    return fail(VEG_ERR_INVALID_ARG, "gaussians: quats must be 16-byte aligned");
  const int lit = (g->normals != nullptr) + (g->k_ambient != nullptr) + (g->k_diffuse != nullptr) +
                  (g->k_specular != nullptr) + (g->shininess != nullptr);
  if (lit != 0 && lit != 5)
    return fail(VEG_ERR_INVALID_ARG, "gaussians: lighting attributes must be all NULL or all given");
  return VEG_OK;
}

size_t pairs_of(const veg_proj* p) { return (size_t)p->n_frames * (size_t)p->n; }
// Frames a key list is shared by (1 for veg_project).
static int per_view_of(const veg_proj* proj) { return proj->tfs_per_view > 1 ? proj->tfs_per_view : 1; }

}  // namespace

void veg::set_last_error(const char* msg) { g_err = msg ? msg : ""; }

extern "C" {

const char* veg_status_str(int s) {
  switch (s) {
    case VEG_OK: return "ok";
    case VEG_ERR_INVALID_ARG: return "invalid argument";
    case VEG_ERR_CAPACITY: return "key list capacity exceeded";
    case VEG_ERR_OUT_OF_BUDGET: return "request exceeds the memory budget";
    case VEG_ERR_NOT_FOUND: return "not found";
    case VEG_ERR_BUSY: return "busy";
    case VEG_ERR_HIP: return "HIP error";
    case VEG_ERR_TIMEOUT: return "timeout";
    case VEG_ERR_SHUTDOWN: return "server shutting down";
    default: return "unknown status";
  }
}

const char* veg_last_error(void) { return g_err.c_str(); }

int veg_version(void) { return VEG_VERSION; }

void veg_opts_default(veg_opts* o) {
  if (!o) return;
  o->alpha_clamp = 0.99f;
  o->alpha_min = 1.0f / 255.0f;
  o->t_min = 1e-4f;
  o->lowpass = 0.3f;
  o->near_z = 0.2f;
  o->guard = 1.3f;
  o->bg[0] = o->bg[1] = o->bg[2] = 0.0f;
}

size_t veg_frames_bytes(int32_t n_frames) { return n_frames > 0 ? (size_t)n_frames * sizeof(FrameDesc) : 0; }

// Frames f = v * per_view + k: camera cams[v], table tfs[f]; the frames of a view share the
// key list of its first frame (per_view = 1: every frame has its own).
static veg_status project_impl(const veg_gaussians* g, int32_t n_views, int32_t per_view, const veg_camera* cams,
                               const veg_tf* tfs, const veg_opts* opts, veg_proj* proj, veg_stream_t stream) {
  g_err.clear();
  veg_status s = check_gaussians(g);
  if (s != VEG_OK) return s;
  if (!cams || !tfs) return fail(VEG_ERR_INVALID_ARG, "cams/tfs is NULL");
  if (per_view < 1 || per_view > VEG_MAX_FRAMES) return fail(VEG_ERR_INVALID_ARG, "tfs_per_view out of range");
  if (n_views < 1 || (int64_t)n_views * per_view > VEG_MAX_FRAMES)
    return fail(VEG_ERR_INVALID_ARG, "n_frames out of range");
  const int32_t n_frames = n_views * per_view;
  s = check_proj(proj);
  if (s != VEG_OK) return s;
  if (proj->n != g->n || proj->n_frames != n_frames)
    return fail(VEG_ERR_INVALID_ARG, "proj->n / n_frames do not match the call");
  veg_opts o;
  s = resolve_opts(opts, &o);
  if (s != VEG_OK) return s;
  const int W = cams[0].width, H = cams[0].height;
  for (int f = 0; f < n_frames; ++f) {
    const veg_camera& c = cams[f / per_view];
    if (c.width != W || c.height != H) return fail(VEG_ERR_INVALID_ARG, "frame %d: all frames need one size", f);
    if (c.width < 1 || c.height < 1 || c.width > VEG_MAX_DIM || c.height > VEG_MAX_DIM)
      return fail(VEG_ERR_INVALID_ARG, "frame %d: width/height out of range", f);
    if (!(c.fx > 0.0f) || !(c.fy > 0.0f) || !std::isfinite(c.cx) || !std::isfinite(c.cy))
      return fail(VEG_ERR_INVALID_ARG, "frame %d: need fx, fy > 0 and finite cx, cy", f);
    for (int k = 0; k < 12; ++k)
      if (!std::isfinite(c.view[k])) return fail(VEG_ERR_INVALID_ARG, "frame %d: non-finite view matrix", f);
    if (!tfs[f].rgba || tfs[f].k < 2) return fail(VEG_ERR_INVALID_ARG, "frame %d: TF needs k >= 2 points", f);
    if (reinterpret_cast<uintptr_t>(tfs[f].rgba) & 15u)
      return fail(VEG_ERR_INVALID_ARG, "frame %d: TF table must be 16-byte aligned", f);
  }
  const int tiles_x = (W + kTile - 1) / kTile, tiles_y = (H + kTile - 1) / kTile;
  // tiles are numbered per list: a view's frames share their owner's tiles
  const int64_t total_tiles = (int64_t)n_views * tiles_x * tiles_y;
  if (total_tiles >= ((int64_t)1 << 31)) return fail(VEG_ERR_INVALID_ARG, "too many tiles");
  std::vector<FrameDesc> descs(n_frames);
  for (int f = 0; f < n_frames; ++f) {
    FrameDesc& d = descs[f];
    std::memset(&d, 0, sizeof(d));
    d.means = g->means;
    d.log_scales = g->log_scales;
    d.quats = g->quats;
    d.scalars = g->scalars;
    d.weights = g->weights;
    const veg_camera& cam = cams[f / per_view];
    set_lighting(d, *g, cam);
    d.lut = tfs[f].rgba;
    d.K = tfs[f].k;
    d.n = (int32_t)g->n;
    d.W = W;
    d.H = H;
    d.tiles_x = tiles_x;
    d.tiles_y = tiles_y;
    d.pair_base = (uint32_t)((int64_t)f * g->n);
    d.tile_base = (uint32_t)((int64_t)(f / per_view) * tiles_x * tiles_y);
    d.pix_base = (uint32_t)((int64_t)f * W * H);
    d.list_frame = (uint32_t)(f - f % per_view);
    d.slot = f % per_view;
    d.n_share = d.slot == 0 ? per_view : 0;
    std::memcpy(d.view, cam.view, sizeof(d.view));
    d.fx = cam.fx;
    d.fy = cam.fy;
    d.cx = cam.cx;
    d.cy = cam.cy;
    d.bg[0] = o.bg[0];
    d.bg[1] = o.bg[1];
    d.bg[2] = o.bg[2];
  }
  hipStream_t st = (hipStream_t)stream;
  const int per_chunk = kBlobMaxBytes / (int)sizeof(FrameDesc);
  for (int f0 = 0; f0 < n_frames; f0 += per_chunk) {
    const int nf = std::min(per_chunk, n_frames - f0);
    VEG_CHECK_HIP(write_blob((FrameDesc*)proj->frames + f0, &descs[f0], nf * sizeof(FrameDesc), st),
                  "veg_project: descriptor upload");
  }
  proj->width = W;
  proj->height = H;
  proj->tiles_x = tiles_x;
  proj->tiles_y = tiles_y;
  proj->total_tiles = total_tiles;
  proj->tfs_per_view = per_view;
  if (g->n > 0)
    VEG_CHECK_HIP(launch_project((const FrameDesc*)proj->frames, n_frames, (int)g->n, kopts(&o), (float4*)proj->rec,
                                 proj->count, proj->depth, true, st),
                  "veg_project");
  return VEG_OK;
}

veg_status veg_project(const veg_gaussians* g, int32_t n_frames, const veg_camera* cams, const veg_tf* tfs,
                       const veg_opts* opts, veg_proj* proj, veg_stream_t stream) {
  return project_impl(g, n_frames, 1, cams, tfs, opts, proj, stream);
}

veg_status veg_project_views(const veg_gaussians* g, int32_t n_views, int32_t tfs_per_view, const veg_camera* cams,
                             const veg_tf* tfs, const veg_opts* opts, veg_proj* proj, veg_stream_t stream) {
  return project_impl(g, n_views, tfs_per_view, cams, tfs, opts, proj, stream);
}

size_t veg_bin_workspace_bytes(int64_t n_pairs, int64_t capacity) {
  (void)capacity;
  return bin_ws_bytes(n_pairs);
}

veg_status veg_bin_count(const veg_proj* proj, void* ws, size_t ws_bytes, int64_t* n_entries, veg_stream_t stream) {
  g_err.clear();
  veg_status s = check_projected(proj);
  if (s != VEG_OK) return s;
  const size_t pairs = pairs_of(proj);
  if (!ws || ws_bytes < bin_ws_bytes((int64_t)pairs)) return fail(VEG_ERR_INVALID_ARG, "bin workspace too small");
  BinWs w;
  carve_bin_ws(ws, (int64_t)pairs, &w);
  hipStream_t st = (hipStream_t)stream;
  if (pairs > 0) {
    VEG_CHECK_HIP(launch_bin_count((const float4*)proj->rec, proj->count, proj->depth, (uint32_t)pairs, w, st, nullptr,
                                   (uint32_t)proj->n, per_view_of(proj)),
                  "veg_bin_count");
  } else {
    VEG_CHECK_HIP(launch_fill_u32(w.counters, 64, 0u, st), "veg_bin_count");
  }
  if (n_entries) {
    uint32_t e[2];
    VEG_CHECK_HIP(hipMemcpyAsync(e, w.counters + 1, sizeof(e), hipMemcpyDeviceToHost, st), "veg_bin_count: read");
    VEG_CHECK_HIP(hipStreamSynchronize(st), "veg_bin_count: sync");
    *n_entries = (int64_t)((uint64_t)e[0] | ((uint64_t)e[1] << 32));
  }
  return VEG_OK;
}

veg_status veg_bin_sort(const veg_proj* proj, void* ws, size_t ws_bytes, const veg_bins* bins, veg_stream_t stream) {
  g_err.clear();
  veg_status s = check_projected(proj);
  if (s != VEG_OK) return s;
  if (!bins) return fail(VEG_ERR_INVALID_ARG, "bins is NULL");
  if (bins->capacity < 0 || bins->capacity >= ((int64_t)1 << 31))
    return fail(VEG_ERR_INVALID_ARG, "bins: capacity must be in [0, 2^31)");
  if (bins->capacity > 0 && (!bins->keys || !bins->vals || !bins->keys_alt || !bins->vals_alt))
    return fail(VEG_ERR_INVALID_ARG, "bins: NULL key buffer");
  if (!bins->ranges) return fail(VEG_ERR_INVALID_ARG, "bins: NULL ranges");
  const size_t pairs = pairs_of(proj);
  if (!ws || ws_bytes < bin_ws_bytes((int64_t)pairs)) return fail(VEG_ERR_INVALID_ARG, "bin workspace too small");
  BinWs w;
  carve_bin_ws(ws, (int64_t)pairs, &w);
  hipStream_t st = (hipStream_t)stream;
  VEG_CHECK_HIP(launch_bin_sort((const FrameDesc*)proj->frames, proj->n_frames, (const float4*)proj->rec, proj->count,
                                (uint32_t)pairs, (uint32_t)proj->total_tiles, w, bins->keys, bins->vals,
                                bins->keys_alt, bins->vals_alt, bins->ranges,
                                pairs > 0 ? (uint32_t)bins->capacity : 0u, st),
                "veg_bin_sort");
  return VEG_OK;
}

veg_status veg_bin_static(const veg_proj* proj, const veg_bins* bins, int64_t* status, veg_stream_t stream) {
  g_err.clear();
  veg_status s = check_projected(proj);
  if (s != VEG_OK) return s;
  if (!bins) return fail(VEG_ERR_INVALID_ARG, "bins is NULL");
  if (bins->capacity < 0 || bins->capacity >= ((int64_t)1 << 31))
    return fail(VEG_ERR_INVALID_ARG, "bins: capacity must be in [0, 2^31)");
  if (bins->capacity > 0 && (!bins->keys || !bins->vals || !bins->keys_alt || !bins->vals_alt))
    return fail(VEG_ERR_INVALID_ARG, "bins: NULL key buffer");
  if (!bins->ranges) return fail(VEG_ERR_INVALID_ARG, "bins: NULL ranges");
  if (!status || ((uintptr_t)status & 7u)) return fail(VEG_ERR_INVALID_ARG, "bin_static: NULL or misaligned status");
  const size_t pairs = pairs_of(proj);
  if ((int64_t)pairs > VEG_BIN_STATIC_MAX_PAIRS || bin_ws_bytes((int64_t)pairs) > kStaticBinBytes)
    return fail(VEG_ERR_INVALID_ARG, "bin_static: %zu pairs exceed the library scratch's limit of %d pairs", pairs,
                (int)VEG_BIN_STATIC_MAX_PAIRS);
  void* ws = nullptr;
  VEG_CHECK_HIP(static_bin_scratch(&ws), "veg_bin_static: scratch");
  BinWs w;
  carve_bin_ws(ws, (int64_t)pairs, &w);
  hipStream_t st = (hipStream_t)stream;
  if (pairs > 0) {
    VEG_CHECK_HIP(launch_bin_count((const float4*)proj->rec, proj->count, proj->depth, (uint32_t)pairs, w, st, nullptr,
                                   (uint32_t)proj->n, per_view_of(proj)),
                  "veg_bin_static: count");
  } else {
    VEG_CHECK_HIP(launch_fill_u32(w.counters, 64, 0u, st), "veg_bin_static: count");
  }
  VEG_CHECK_HIP(launch_bin_sort((const FrameDesc*)proj->frames, proj->n_frames, (const float4*)proj->rec, proj->count,
                                (uint32_t)pairs, (uint32_t)proj->total_tiles, w, bins->keys, bins->vals,
                                bins->keys_alt, bins->vals_alt, bins->ranges,
                                pairs > 0 ? (uint32_t)bins->capacity : 0u, st),
                "veg_bin_static: sort");
  VEG_CHECK_HIP(launch_bin_status(w.counters, status, st), "veg_bin_static: status");
  return VEG_OK;
}

veg_status veg_bin_overflow(void* ws, size_t ws_bytes, int64_t* n_entries, int32_t* overflow, veg_stream_t stream) {
  g_err.clear();
  if (!ws || ws_bytes < bin_ws_bytes(1)) return fail(VEG_ERR_INVALID_ARG, "bin workspace too small");
  BinWs w;
  carve_bin_ws(ws, 1, &w);   // the counters' offset does not depend on the pair count
  uint32_t c[4];
  hipStream_t st = (hipStream_t)stream;
  VEG_CHECK_HIP(hipMemcpyAsync(c, w.counters, sizeof(c), hipMemcpyDeviceToHost, st), "veg_bin_overflow: read");
  VEG_CHECK_HIP(hipStreamSynchronize(st), "veg_bin_overflow: sync");
  if (n_entries) *n_entries = (int64_t)((uint64_t)c[1] | ((uint64_t)c[2] << 32));
  if (overflow) *overflow = (int32_t)c[3];
  return VEG_OK;
}

veg_status veg_bin_status(void* ws, size_t ws_bytes, int64_t* dst, veg_stream_t stream) {
  g_err.clear();
  if (!ws || ws_bytes < bin_ws_bytes(1)) return fail(VEG_ERR_INVALID_ARG, "bin workspace too small");
  if (!dst || ((uintptr_t)dst & 7u)) return fail(VEG_ERR_INVALID_ARG, "bin_status: NULL or misaligned dst");
  BinWs w;
  carve_bin_ws(ws, 1, &w);
  VEG_CHECK_HIP(launch_bin_status(w.counters, dst, (hipStream_t)stream), "veg_bin_status");
  return VEG_OK;
}

int64_t veg_bin_hit_words(int64_t capacity, int64_t total_tiles) {
  if (capacity < 0 || total_tiles < 0) return 0;
  return capacity / 64 + total_tiles + 2;
}

// Frames per shared key list (0 in a struct not filled by veg_project_views means 1).

// Words of one frame slot's hit bits.
static uint64_t hit_stride_of(const veg_proj* proj, const veg_bins* bins) {
  return (uint64_t)veg_bin_hit_words(bins->capacity, proj->total_tiles);
}

// The hit bits are optional; when present the buffer must hold every tile's words for each
// frame that shares a list.
static veg_status check_hits(const veg_proj* proj, const veg_bins* bins, const char* what) {
  if (proj->n_frames % per_view_of(proj) != 0)
    return fail(VEG_ERR_INVALID_ARG, "%s: n_frames is not a multiple of tfs_per_view", what);
  if (!bins->hits) return VEG_OK;
  if ((uint64_t)bins->hit_words < (uint64_t)per_view_of(proj) * hit_stride_of(proj, bins))
    return fail(VEG_ERR_INVALID_ARG, "%s: hit_words < tfs_per_view * veg_bin_hit_words(capacity, tiles)", what);
  return VEG_OK;
}

// After the sort, keys_alt is free: the blend launches keep their dispatch order there.
static uint64_t order_words(const veg_bins* bins) {
  return bins->keys_alt && bins->capacity > 0 ? (uint64_t)bins->capacity : 0u;
}

veg_status veg_render_fwd(const veg_proj* proj, const veg_bins* bins, const veg_opts* opts, float* image,
                          float* t_final, int32_t* n_last, int32_t* n_contrib, veg_stream_t stream) {
  g_err.clear();
  veg_status s = check_projected(proj);
  if (s != VEG_OK) return s;
  if (!bins || !bins->ranges || !image) return fail(VEG_ERR_INVALID_ARG, "render_fwd: NULL argument");
  if (proj->n > 0 && bins->capacity > 0 && !bins->vals) return fail(VEG_ERR_INVALID_ARG, "render_fwd: NULL vals");
  s = check_hits(proj, bins, "render_fwd");
  if (s != VEG_OK) return s;
  veg_opts o;
  s = resolve_opts(opts, &o);
  if (s != VEG_OK) return s;
  VEG_CHECK_HIP(launch_blend_fwd((const FrameDesc*)proj->frames, proj->n_frames, per_view_of(proj),
                                 proj->tiles_x * proj->tiles_y, kopts(&o), (const float4*)proj->rec, bins->vals,
                                 bins->ranges, image, t_final, n_last, n_contrib, bins->hits,
                                 hit_stride_of(proj, bins), proj->depth, bins->keys_alt, order_words(bins),
                                 (hipStream_t)stream),
                "veg_render_fwd");
  return VEG_OK;
}

veg_status veg_render_fwd_l1(const veg_proj* proj, const veg_bins* bins, const veg_opts* opts, const float* target,
                             float scale, double* loss_slots, float* d_image, float* t_final, int32_t* n_last,
                             veg_stream_t stream) {
  g_err.clear();
  veg_status s = check_projected(proj);
  if (s != VEG_OK) return s;
  if (!bins || !bins->ranges || !target || !loss_slots || !d_image)
    return fail(VEG_ERR_INVALID_ARG, "render_fwd_l1: NULL argument");
  if (!std::isfinite(scale)) return fail(VEG_ERR_INVALID_ARG, "render_fwd_l1: scale must be finite");
  if (proj->n > 0 && bins->capacity > 0 && !bins->vals) return fail(VEG_ERR_INVALID_ARG, "render_fwd_l1: NULL vals");
  s = check_hits(proj, bins, "render_fwd_l1");
  if (s != VEG_OK) return s;
  veg_opts o;
  s = resolve_opts(opts, &o);
  if (s != VEG_OK) return s;
  L1Fuse l1;
  l1.target = target;
  l1.loss = loss_slots;
  l1.scale = scale;
  VEG_CHECK_HIP(launch_blend_fwd((const FrameDesc*)proj->frames, proj->n_frames, per_view_of(proj),
                                 proj->tiles_x * proj->tiles_y, kopts(&o), (const float4*)proj->rec, bins->vals,
                                 bins->ranges, d_image, t_final, n_last, nullptr, bins->hits,
                                 hit_stride_of(proj, bins), proj->depth, bins->keys_alt, order_words(bins),
                                 (hipStream_t)stream, l1),
                "veg_render_fwd_l1");
  return VEG_OK;
}

veg_status veg_render_bwd(const veg_proj* proj, const veg_bins* bins, const veg_opts* opts, const float* t_final,
                          const int32_t* n_last, const float* d_image, float* g2d, veg_stream_t stream) {
  g_err.clear();
  veg_status s = check_projected(proj);
  if (s != VEG_OK) return s;
  if (!bins || !bins->ranges || !t_final || !n_last || !d_image || (proj->n > 0 && !g2d))
    return fail(VEG_ERR_INVALID_ARG, "render_bwd: NULL argument");
  s = check_hits(proj, bins, "render_bwd");
  if (s != VEG_OK) return s;
  veg_opts o;
  s = resolve_opts(opts, &o);
  if (s != VEG_OK) return s;
  // The adjoint recovers the transmittance in front of each entry as T / (1 - alpha): alpha
  // must stay away from 1, and the smallest T a pixel can end with, t_min (1 - alpha_clamp),
  // must stay far inside float32's normal range.
  if (!(o.alpha_clamp <= kBwdAlphaClampMax) || !((double)o.t_min * (1.0 - (double)o.alpha_clamp) >= kBwdTFloor))
    return fail(VEG_ERR_INVALID_ARG, "render_bwd: need alpha_clamp <= 1 - 2^-10 and t_min (1 - alpha_clamp) >= 2^-100");
  VEG_CHECK_HIP(launch_blend_bwd((const FrameDesc*)proj->frames, proj->n_frames, proj->tiles_x * proj->tiles_y,
                                 kopts(&o), (const float4*)proj->rec, bins->vals, bins->ranges, t_final, n_last,
                                 d_image, g2d, (uint32_t)pairs_of(proj), bins->hits, hit_stride_of(proj, bins),
                                 bins->keys_alt, order_words(bins), (hipStream_t)stream),
                "veg_render_bwd");
  return VEG_OK;
}

veg_status veg_project_bwd(const veg_gaussians* g, const veg_proj* proj, const veg_opts* opts, const float* g2d,
                           const veg_grads* grads, veg_stream_t stream) {
  g_err.clear();
  veg_status s = check_gaussians(g);
  if (s != VEG_OK) return s;
  s = check_projected(proj);
  if (s != VEG_OK) return s;
  if (proj->n != g->n) return fail(VEG_ERR_INVALID_ARG, "project_bwd: proj->n != g->n");
  if (!grads || (g->n > 0 && (!g2d || !grads->d_means || !grads->d_log_scales || !grads->d_quats ||
                              !grads->d_scalars)))
    return fail(VEG_ERR_INVALID_ARG, "project_bwd: NULL gradient buffer");
  if (grads->d_weights && !g->weights)
    return fail(VEG_ERR_INVALID_ARG, "project_bwd: d_weights given but the model has no weights");
  {
    const int lg = (grads->d_normals != nullptr) + (grads->d_k_ambient != nullptr) +
                   (grads->d_k_diffuse != nullptr) + (grads->d_k_specular != nullptr) +
                   (grads->d_shininess != nullptr);
    if (lg != 0 && lg != 5)
      return fail(VEG_ERR_INVALID_ARG, "project_bwd: lighting gradients must be all NULL or all given");
    if (lg == 5 && !g->normals)
      return fail(VEG_ERR_INVALID_ARG, "project_bwd: lighting gradients given but the model has no lighting");
  }
  veg_opts o;
  s = resolve_opts(opts, &o);
  if (s != VEG_OK) return s;
  VEG_CHECK_HIP(launch_project_bwd((const FrameDesc*)proj->frames, proj->n_frames, (int)g->n, kopts(&o),
                                   const_cast<float*>(g2d), (uint32_t)pairs_of(proj), *grads, (hipStream_t)stream),
                "veg_project_bwd");
  return VEG_OK;
}

veg_status veg_project_bwd_fused(const veg_gaussians* g, const veg_proj* proj, const veg_opts* opts, float* g2d,
                                 const veg_grads* grads, float* grad_accum, int32_t* vis_count, int32_t consume_g2d,
                                 veg_stream_t stream) {
  g_err.clear();
  if ((grad_accum == nullptr) != (vis_count == nullptr))
    return fail(VEG_ERR_INVALID_ARG, "project_bwd_fused: grad_accum and vis_count must both be given or both NULL");
  veg_status s = check_gaussians(g);
  if (s != VEG_OK) return s;
  s = check_projected(proj);
  if (s != VEG_OK) return s;
  if (proj->n != g->n) return fail(VEG_ERR_INVALID_ARG, "project_bwd_fused: proj->n != g->n");
  if (!grads || (g->n > 0 && (!g2d || !grads->d_means || !grads->d_log_scales || !grads->d_quats ||
                              !grads->d_scalars)))
    return fail(VEG_ERR_INVALID_ARG, "project_bwd_fused: NULL gradient buffer");
  if (grads->d_weights && !g->weights)
    return fail(VEG_ERR_INVALID_ARG, "project_bwd_fused: d_weights given but the model has no weights");
  {
    const int lg = (grads->d_normals != nullptr) + (grads->d_k_ambient != nullptr) +
                   (grads->d_k_diffuse != nullptr) + (grads->d_k_specular != nullptr) +
                   (grads->d_shininess != nullptr);
    if (lg != 0 && lg != 5)
      return fail(VEG_ERR_INVALID_ARG, "project_bwd_fused: lighting gradients must be all NULL or all given");
    if (lg == 5 && !g->normals)
      return fail(VEG_ERR_INVALID_ARG, "project_bwd_fused: lighting gradients given but the model has no lighting");
  }
  veg_opts o;
  s = resolve_opts(opts, &o);
  if (s != VEG_OK) return s;
  BwdFused fu;
  fu.count = proj->count;
  fu.depth = proj->depth;
  fu.rec = (const float4*)proj->rec;
  fu.acc = grad_accum;
  fu.vis = vis_count;
  fu.consume = consume_g2d != 0;
  VEG_CHECK_HIP(launch_project_bwd((const FrameDesc*)proj->frames, proj->n_frames, (int)g->n, kopts(&o), g2d,
                                   (uint32_t)pairs_of(proj), *grads, (hipStream_t)stream, fu),
                "veg_project_bwd_fused");
  return VEG_OK;
}

veg_status veg_l1_loss(const float* image, const float* target, int64_t count, float scale, double* loss,
                       float* d_image, veg_stream_t stream) {
  g_err.clear();
  if (count < 0) return fail(VEG_ERR_INVALID_ARG, "l1_loss: count < 0");
  if (count > 0 && (!image || !target || !loss || !d_image)) return fail(VEG_ERR_INVALID_ARG, "l1_loss: NULL");
  if (!std::isfinite(scale)) return fail(VEG_ERR_INVALID_ARG, "l1_loss: scale must be finite");
  VEG_CHECK_HIP(launch_l1(image, target, count, scale, loss, d_image, (hipStream_t)stream), "veg_l1_loss");
  return VEG_OK;
}

size_t veg_ssim_workspace_bytes(int64_t n_planes, int32_t width, int32_t height) {
  if (n_planes < 0 || width < 0 || height < 0) return 0;
  return 3 * sizeof(float) * (size_t)n_planes * (size_t)width * (size_t)height;
}

veg_status veg_ssim_loss(const float* image, const float* target, int64_t n_planes, int32_t width, int32_t height,
                         float weight, double* loss, float* d_image, void* ws, size_t ws_bytes, veg_stream_t stream) {
  g_err.clear();
  if (n_planes < 0 || width < 0 || height < 0 || width > VEG_MAX_DIM || height > VEG_MAX_DIM || n_planes > 65535)
    return fail(VEG_ERR_INVALID_ARG, "ssim_loss: sizes out of range");
  if (n_planes == 0 || width == 0 || height == 0) return VEG_OK;
  if (!image || !target || !loss || !d_image || !ws) return fail(VEG_ERR_INVALID_ARG, "ssim_loss: NULL argument");
  if (ws_bytes < veg_ssim_workspace_bytes(n_planes, width, height))
    return fail(VEG_ERR_INVALID_ARG, "ssim_loss: workspace smaller than veg_ssim_workspace_bytes");
  if (!std::isfinite(weight)) return fail(VEG_ERR_INVALID_ARG, "ssim_loss: weight must be finite");
  VEG_CHECK_HIP(launch_ssim(image, target, n_planes, width, height, weight, loss, d_image, (float*)ws,
                            (hipStream_t)stream),
                "veg_ssim_loss");
  return VEG_OK;
}

veg_status veg_image_loss(const float* image, const float* target, int64_t n_planes, int32_t width, int32_t height,
                          float l1_scale, float ssim_weight, double* loss, float* d_image, void* ws, size_t ws_bytes,
                          veg_stream_t stream) {
  g_err.clear();
  if (n_planes < 0 || width < 0 || height < 0 || width > VEG_MAX_DIM || height > VEG_MAX_DIM || n_planes > 65535)
    return fail(VEG_ERR_INVALID_ARG, "image_loss: sizes out of range");
  if (n_planes == 0 || width == 0 || height == 0) return VEG_OK;
  if (!image || !target || !loss || !d_image || !ws) return fail(VEG_ERR_INVALID_ARG, "image_loss: NULL argument");
  if (ws_bytes < veg_ssim_workspace_bytes(n_planes, width, height))
    return fail(VEG_ERR_INVALID_ARG, "image_loss: workspace smaller than veg_ssim_workspace_bytes");
  if (!std::isfinite(l1_scale) || !std::isfinite(ssim_weight))
    return fail(VEG_ERR_INVALID_ARG, "image_loss: weights must be finite");
  VEG_CHECK_HIP(launch_ssim(image, target, n_planes, width, height, ssim_weight, loss, d_image, (float*)ws,
                            (hipStream_t)stream, true, l1_scale),
                "veg_image_loss");
  return VEG_OK;
}

veg_status veg_adam_step(float* param, const float* grad, float* m, float* v, int64_t count, float lr, float beta1,
                         float beta2, float eps, int32_t step, veg_stream_t stream) {
  g_err.clear();
  if (count < 0 || step < 1) return fail(VEG_ERR_INVALID_ARG, "adam_step: count < 0 or step < 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f) || !std::isfinite(lr))
    return fail(VEG_ERR_INVALID_ARG, "adam_step: need 0 <= beta < 1, eps >= 0, finite lr");
  if (count == 0) return VEG_OK;
  if (!param || !grad || !m || !v) return fail(VEG_ERR_INVALID_ARG, "adam_step: NULL argument");
  const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  VEG_CHECK_HIP(launch_adam(param, grad, m, v, count, lr, beta1, beta2, eps, bc1, bc2, (hipStream_t)stream),
                "veg_adam_step");
  return VEG_OK;
}

veg_status veg_densify_stats(const veg_proj* proj, const float* g2d, float* grad_accum, int32_t* vis_count,
                             veg_stream_t stream) {
  g_err.clear();
  veg_status s = check_projected(proj);
  if (s != VEG_OK) return s;
  if (proj->n > 0 && (!g2d || !grad_accum || !vis_count)) return fail(VEG_ERR_INVALID_ARG, "densify_stats: NULL");
  VEG_CHECK_HIP(launch_densify_stats((const FrameDesc*)proj->frames, proj->n_frames, (int)proj->n, proj->count,
                                     proj->depth, (const float4*)proj->rec, g2d,
                                     grad_accum, vis_count, (hipStream_t)stream),
                "veg_densify_stats");
  return VEG_OK;
}

// Densification scratch: 3 counters per block of 256 Gaussians, then the 3 totals.
static int64_t densify_blocks(int64_t n) { return (n + 255) / 256; }

size_t veg_densify_workspace_bytes(int64_t n) {
  if (n < 0) return 0;
  return (size_t)(3 * densify_blocks(n) + 4) * sizeof(uint32_t);
}

veg_status veg_densify_plan(int64_t n, const float* grad_accum, const int32_t* vis_count, const float* log_scales,
                            const float* weights, float grad_thresh, float log_scale_thresh, float prune_weight,
                            uint8_t* action, int64_t* counts, void* ws, size_t ws_bytes, veg_stream_t stream) {
  g_err.clear();
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(VEG_ERR_INVALID_ARG, "densify_plan: n out of range");
  if (std::isnan(grad_thresh) || std::isnan(log_scale_thresh) || std::isnan(prune_weight))
    return fail(VEG_ERR_INVALID_ARG, "densify_plan: NaN threshold");
  if (n == 0) {
    if (counts) counts[0] = counts[1] = counts[2] = counts[3] = 0;
    return VEG_OK;
  }
  if (!grad_accum || !vis_count || !log_scales || !action || !ws)
    return fail(VEG_ERR_INVALID_ARG, "densify_plan: NULL argument");
  if (ws_bytes < veg_densify_workspace_bytes(n)) return fail(VEG_ERR_INVALID_ARG, "densify_plan: workspace too small");
  uint32_t* blk = (uint32_t*)ws;
  uint32_t* tot = blk + 3 * densify_blocks(n);
  hipStream_t st = (hipStream_t)stream;
  VEG_CHECK_HIP(launch_densify_plan(n, grad_accum, vis_count, log_scales, weights, grad_thresh, log_scale_thresh,
                                    prune_weight, action, blk, tot, st),
                "veg_densify_plan");
  if (counts) {
    uint32_t t[3];
    VEG_CHECK_HIP(hipMemcpyAsync(t, tot, sizeof(t), hipMemcpyDeviceToHost, st), "veg_densify_plan: read");
    VEG_CHECK_HIP(hipStreamSynchronize(st), "veg_densify_plan: sync");
    counts[0] = (int64_t)t[0] - t[1];
    counts[1] = t[1];
    counts[2] = t[2];
    counts[3] = n - (int64_t)t[0] - t[2];
  }
  return VEG_OK;
}

veg_status veg_densify_apply(int64_t n, const uint8_t* action, const float* quats, const float* log_scales,
                             const float* z, const veg_densify_field* fields, int32_t n_fields, const void* ws,
                             size_t ws_bytes, veg_stream_t stream) {
  g_err.clear();
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(VEG_ERR_INVALID_ARG, "densify_apply: n out of range");
  if (!fields || n_fields < 1 || n_fields > kDensifyMaxFields)
    return fail(VEG_ERR_INVALID_ARG, "densify_apply: need 1..%d fields", kDensifyMaxFields);
  DensifyFields fl;
  std::memset(&fl, 0, sizeof(fl));
  for (int f = 0; f < n_fields; ++f) {
    const veg_densify_field& d = fields[f];
    if (d.width < 1 || d.width > 64 || d.role < 0 || d.role > 3)
      return fail(VEG_ERR_INVALID_ARG, "densify_apply: field %d has a bad width or role", f);
    if ((d.role == VEG_FIELD_MEANS || d.role == VEG_FIELD_LOG_SCALES) && d.width != 3)
      return fail(VEG_ERR_INVALID_ARG, "densify_apply: field %d: means and log-scales have width 3", f);
    if (n > 0 && (!d.src || !d.dst)) return fail(VEG_ERR_INVALID_ARG, "densify_apply: field %d is NULL", f);
    fl.src[f] = d.src;
    fl.dst[f] = d.dst;
    fl.width[f] = d.width;
    fl.role[f] = d.role;
  }
  fl.n_fields = n_fields;
  if (n == 0) return VEG_OK;
  if (!action || !quats || !log_scales || !z || !ws) return fail(VEG_ERR_INVALID_ARG, "densify_apply: NULL argument");
  if (ws_bytes < veg_densify_workspace_bytes(n)) return fail(VEG_ERR_INVALID_ARG, "densify_apply: workspace too small");
  const uint32_t* blk = (const uint32_t*)ws;
  VEG_CHECK_HIP(launch_densify_apply(n, action, quats, log_scales, z, blk, blk + 3 * densify_blocks(n), fl,
                                     (hipStream_t)stream),
                "veg_densify_apply");
  return VEG_OK;
}

veg_status veg_vq_decode(const uint16_t* idx, int64_t n, const float* book, int32_t k, int32_t dim,
                         const veg_vq_field* fields, int32_t n_fields, veg_stream_t stream) {
  g_err.clear();
  if (n < 0) return fail(VEG_ERR_INVALID_ARG, "vq_decode: n < 0");
  if (k < 1 || k > 65536 || dim < 1 || dim > 16)
    return fail(VEG_ERR_INVALID_ARG, "vq_decode: need 1 <= k <= 65536 and 1 <= dim <= 16");
  if (!fields || n_fields < 1 || n_fields > kVqMaxFields)
    return fail(VEG_ERR_INVALID_ARG, "vq_decode: need 1..%d fields", kVqMaxFields);
  VqFields fl;
  std::memset(&fl, 0, sizeof(fl));
  int sum = 0;
  for (int f = 0; f < n_fields; ++f) {
    if (fields[f].width < 1) return fail(VEG_ERR_INVALID_ARG, "vq_decode: field %d has width < 1", f);
    if (n > 0 && !fields[f].dst) return fail(VEG_ERR_INVALID_ARG, "vq_decode: field %d dst is NULL", f);
    fl.dst[f] = fields[f].dst;
    fl.width[f] = fields[f].width;
    sum += fields[f].width;
  }
  fl.n_fields = n_fields;
  if (sum != dim) return fail(VEG_ERR_INVALID_ARG, "vq_decode: field widths sum to %d, codebook rows have %d", sum, dim);
  if (n == 0) return VEG_OK;
  if (!idx || !book) return fail(VEG_ERR_INVALID_ARG, "vq_decode: NULL idx or book");
  VEG_CHECK_HIP(launch_vq_decode(idx, n, book, k, dim, fl, (hipStream_t)stream), "veg_vq_decode");
  return VEG_OK;
}

veg_status veg_fill_u32(void* dst, int64_t count, uint32_t value, veg_stream_t stream) {
  g_err.clear();
  if (count < 0 || (count > 0 && !dst)) return fail(VEG_ERR_INVALID_ARG, "fill: bad arguments");
  VEG_CHECK_HIP(launch_fill_u32((uint32_t*)dst, count, value, (hipStream_t)stream), "veg_fill_u32");
  return VEG_OK;
}

veg_status veg_debug_math(int32_t op, const float* in_x, const float* in_y, float* out, int64_t n,
                          veg_stream_t stream) {
  g_err.clear();
  if (op < 0 || op > 5 || n < 0 || (n > 0 && (!in_x || !out || (op == 2 && !in_y))))
    return fail(VEG_ERR_INVALID_ARG, "debug_math: bad arguments");
  VEG_CHECK_HIP(launch_debug_math(op, in_x, in_y, out, n, (hipStream_t)stream), "veg_debug_math");
  return VEG_OK;
}

}  // extern "C"
