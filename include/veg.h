/*
 * veg.h -- C ABI of the VEG splatting rasterizer for AMD Instinct MI355X (gfx950).
 *
 * Volume Encoding Gaussians (Dyken et al., arXiv 2504.13339) represent a volume by 3D
 * Gaussians that carry a scalar value v instead of a colour and an opacity
 * (section "The VEG Representation").  At render time a 1D transfer function maps v to
 * colour C(v) and opacity O(v), applied per Gaussian before rasterizing, with
 * alpha = O(v) * w for an optional trainable weight w (section "Rendering of VEGs").
 * The 3D covariance from scale S and rotation R is projected to a 2D screen covariance
 * (Zwicker's EWA splatting), Gaussians are binned to 16x16 tiles, sorted front to back,
 * and composited per pixel with the emission-absorption sum of Eq. 1:
 *     P = sum_i c_i alpha_i prod_{j<i} (1 - alpha_j).
 * Gradients flow back to position, scaling, rotation, scalar value and weight
 * (section "Rendering of VEGs", manual backward; Fig. 2).
 *
 * Conventions for every call below
 * --------------------------------
 * Memory:   the caller owns every buffer.  Pointers documented as "device" must be HIP
 *           device memory on the current device; "host" pointers are read during the call
 *           and may be freed when it returns.  The stateless calls allocate no device
 *           memory.  Buffer sizes come from the *_bytes / *_count queries.
 * Streams:  every call is asynchronous and ordered on `stream` (a hipStream_t; NULL is
 *           the legacy default stream).  Inputs must stay alive until the stream reaches
 *           the call.  The only calls that synchronise are veg_bin_count with a non-NULL
 *           host counter and the serving wait/poll calls.
 * Results:  gradient outputs are ACCUMULATED (+=); the caller zeroes them first.
 * Errors:   functions return a veg_status; no exception crosses the ABI, nothing aborts.
 *           Argument errors are detected synchronously and return VEG_ERR_INVALID_ARG
 *           with nothing enqueued.  A HIP launch or runtime error returns VEG_ERR_HIP;
 *           asynchronous device faults surface as VEG_ERR_HIP from a later call.
 *           veg_last_error() gives a thread-local message for the last failure.
 * Numerics: float32 on the device.  Cull, depth key and tile rectangle follow the
 *           operation order documented at veg_project (float32, projected centre in
 *           float64, no fused multiply-add), so they are reproducible bit for bit.
 * Layouts:  [a,b] means row-major with the last index fastest.  Images are planar
 *           [frames,3,H,W]; per-pixel outputs are [frames,H,W].
 */
#ifndef VEG_H
#define VEG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VEG_VERSION 1
#define VEG_TILE 16                /* tile edge in pixels */
#define VEG_MAX_FRAMES 4096        /* frames per stateless call */
#define VEG_MAX_DIM 8192           /* width/height limit (keeps per-block entry counts in 32 bits) */
#define VEG_REC_FLOATS 12          /* floats per (frame, Gaussian) projection record */
#define VEG_G2D_COMPONENTS 9       /* screen-space gradient components per (frame, Gaussian) */

typedef void* veg_stream_t;        /* hipStream_t */

typedef enum {
  VEG_OK = 0,
  VEG_ERR_INVALID_ARG = 1,   /* bad pointer, size or option; nothing was enqueued */
  VEG_ERR_CAPACITY = 2,      /* key list larger than the buffers given */
  VEG_ERR_OUT_OF_BUDGET = 3, /* serving: request can never fit the memory budget */
  VEG_ERR_NOT_FOUND = 4,     /* serving: unknown model or request id */
  VEG_ERR_BUSY = 5,          /* serving: request not finished yet */
  VEG_ERR_HIP = 6,           /* HIP runtime / launch error */
  VEG_ERR_TIMEOUT = 7,       /* serving: wait timed out */
  VEG_ERR_SHUTDOWN = 8       /* serving: server is shutting down */
} veg_status;

const char* veg_status_str(int status);
const char* veg_last_error(void);   /* thread-local; "" when there was none */
int veg_version(void);

/* ----------------------------------------------------------------------------------
 * Inputs
 * ---------------------------------------------------------------------------------- */

/* A VEG model, device SoA (section "The VEG Representation": centre mu, scaling S,
 * rotation R, scalar value v, weight w, and the lighting attributes of its Blinn-Phong
 * model, Eq. 2-3).
 *   means      [n,3]  world-space centres
 *   log_scales [n,3]  log of the three axis scales (S = diag(exp(log_scales)))
 *   quats      [n,4]  rotation as an unnormalised quaternion (w,x,y,z); normalised inside
 *   scalars    [n]    scalar value, already activated (the paper stores it through a
 *                     sigmoid; apply it before the call); used clamped to [0,1]
 *   weights    [n]    trainable opacity weight, already activated, or NULL meaning 1
 * Lighting (all five NULL: the colour is the transfer function's C(v); all five non-NULL:
 * the Blinn-Phong colour of Eq. 2-3 under a headlight, light and view direction both the
 * unit vector l from the camera centre to the Gaussian, so that with s = |n^ . l|
 *   c = C(v) (k_ambient + k_diffuse s) + k_specular s^shininess (white; 0 when s = 0)):
 *   normals    [n,3]  normal, any non-zero length (normalised inside)
 *   k_ambient, k_diffuse, k_specular, shininess  [n]  already activated, shininess > 0
 * Gaussians with any non-finite input, or a zero quaternion or normal, are culled, never an
 * error. */
typedef struct {
  int64_t n;
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* scalars;
  const float* weights;
  const float* normals;
  const float* k_ambient;
  const float* k_diffuse;
  const float* k_specular;
  const float* shininess;
} veg_gaussians;

/* Pinhole camera (host struct).  view = world->camera 3x4 row-major [R|t]; camera axes
 * x right, y down, z forward.  Pixel (i,j) has centre (i+0.5, j+0.5); the projected
 * centre is (fx x/z + cx, fy y/z + cy). */
typedef struct {
  float view[12];
  float fx, fy, cx, cy;
  int32_t width, height;
} veg_camera;

/* Transfer function: k RGBA control points, device [k,4], straight (not premultiplied)
 * colour and opacity, node-centred at v = j/(k-1), linearly interpolated between them
 * (section "Rendering of VEGs": linear interpolation between an arbitrary number of
 * control points).  k >= 2. */
typedef struct {
  const float* rgba;
  int32_t k;
} veg_tf;

/* Renderer options of the rasterizer of section "Rendering of VEGs".  The paper names
 * the rasterizer it builds on but not its constants; these defaults (veg_opts_default)
 * are the readings of this library:
 *   alpha_clamp 0.99   alpha = min(alpha_clamp, A exp(-sigma))
 *   alpha_min   1/255  a Gaussian-pixel pair with A exp(-sigma) < alpha_min is skipped
 *   t_min       1e-4   a pixel stops after blending the Gaussian that takes T below t_min
 *   lowpass     0.3    px^2 added to the diagonal of the 2D covariance (EWA low-pass)
 *   near_z      0.2    Gaussians with camera z <= near_z are culled
 *   guard       1.3    x/z, y/z clamped to guard * (W/2)/fx, (H/2)/fy when forming J
 *   bg          0,0,0  background colour: output = C + T_final * bg */
typedef struct {
  float alpha_clamp, alpha_min, t_min, lowpass, near_z, guard;
  float bg[3];
} veg_opts;

void veg_opts_default(veg_opts* opts);

/* ----------------------------------------------------------------------------------
 * Projection  (transfer function first, then EWA projection and footprint)
 * ---------------------------------------------------------------------------------- */

/* Projection state of `n_frames` frames over one Gaussian set; pair p = f*n + i (the
 * projection of section "Rendering of VEGs"; veg_frames_bytes sizes its descriptors).
 * Host struct holding caller-owned device buffers; veg_project fills the buffers and
 * the host fields marked "out".
 *   frames  device, veg_frames_bytes(n_frames) bytes: per-frame descriptors
 *   rec     device [n_frames*n][12] float: per pair, for kept pairs only:
 *           {mx', my', conic a, conic b, conic c, A, R, G, B, rect01, rect23, frame} where
 *           (mx', my') is the projected centre minus 16*(tile x0, tile y0), conic (a,b,c)
 *           is the inverse 2D covariance [[a,b],[b,c]], A = O(v) w, RGB = C(v), and
 *           rect01 / rect23 hold the tile rectangle (x0 | y0<<16, x1 | y1<<16) as uint32
 *   count   device [n_frames*n] uint32: tiles covered, 0 when culled
 *   depth   device [n_frames*n] uint32: float32 bits of camera z (kept pairs only); for
 *           the views of veg_project_views, the slots of a view's second frame hold, per
 *           Gaussian in the view's list, the bits of the frames that keep it (bit k: frame
 *           v * tfs_per_view + k; all bits from 31 on for views of more than 32 frames) */
typedef struct {
  int64_t n;            /* in: Gaussians per frame */
  int32_t n_frames;     /* in */
  int32_t width, height;             /* out: image size (all frames share it) */
  int32_t tiles_x, tiles_y;          /* out */
  int64_t total_tiles;               /* out: lists * tiles_x * tiles_y, lists = n_frames /
                                        tfs_per_view (one list per frame from veg_project) */
  void* frames;
  float* rec;
  uint32_t* count;
  uint32_t* depth;
  int32_t tfs_per_view;  /* out: frames sharing one key list (1 from veg_project; 0 is
                            read as 1) */
} veg_proj;

size_t veg_frames_bytes(int32_t n_frames);

/* veg_project -- per (frame, Gaussian): transfer-function lookup and cull, EWA projection,
 * conic, projected centre, depth key and tile rectangle (section "Rendering of VEGs": the
 * TF is applied as the first step so low-opacity Gaussians are culled at once; the 3D
 * covariance R S S^T R^T is projected with Zwicker's method).
 *   g          device model; all frames use it
 *   n_frames   1..VEG_MAX_FRAMES; frame f uses cams[f] and tfs[f] (host arrays)
 *   cams       host [n_frames]; every frame must have the same width and height
 *   tfs        host [n_frames]; rgba pointers are device memory
 *   opts       host; NULL = defaults
 *   proj       in/out; proj->n must equal g->n and proj->n_frames must equal n_frames
 * Footprint contract (bit-reproducible; the oracle mirrors it):
 *   t = ((V0 mu_x + V1 mu_y) + V2 mu_z) + V3 per row in float64; depth = float32(t_z);
 *   cull unless depth > near_z; xn = t_x/t_z, yn = t_y/t_z, mx = fx xn + cx,
 *   my = fy yn + cy in float64; TF: vc = clamp(v,0,1), t = vc (k-1),
 *   i = min(floor t, k-2), f = t - i, X = L[i](1-f) + L[i+1] f, A = O w; cull unless
 *   A >= alpha_min and |q|^2 >= 1e-24 (float32); q scaled by 1/sqrt(|q|^2);
 *   s = exp32(log s) (Cody-Waite reduction, Taylor to r^7); Q = Vr R; P = Q diag(s);
 *   J00 = fx/depth, J02 = -(fx xc)/depth, J11 = fy/depth, J12 = -(fy yc)/depth with
 *   xc, yc = float32(xn), float32(yn) clamped to the guard band; G = J P;
 *   S = G G^T + lowpass I (sums left to right); cull unless det > 0;
 *   tau = 2 log32(A/alpha_min) (atanh series to u^9); ex = sqrt(tau S00),
 *   ey = sqrt(tau S11); pixel x range [ceil((mx - ex) - 0.5), floor((mx + ex) - 0.5)]
 *   in float64 clipped to the image (same for y); tile rectangle = range / 16;
 *   count = its area (0 if empty).  Every pixel whose centre has
 *   A exp(-sigma) >= alpha_min lies inside the rectangle, so the tiling loses nothing.
 * Errors: VEG_ERR_INVALID_ARG (NULL pointers, n < 0, n_frames out of range, k < 2,
 *   width/height outside 1..VEG_MAX_DIM or differing between frames,
 *   n_frames * n >= 2^31). */
veg_status veg_project(const veg_gaussians* g, int32_t n_frames, const veg_camera* cams,
                       const veg_tf* tfs, const veg_opts* opts, veg_proj* proj,
                       veg_stream_t stream);

/* veg_project_views -- veg_project for views rendered with several transfer functions
 * each (opacity-guided training renders every camera with a family of opacity maps,
 * section "Training"): n_views cameras x tfs_per_view tables, frame f = v * tfs_per_view + k
 * uses cams[v] and tfs[f].  Geometry does not depend on the table, so the frames of a view
 * share one key list: the first frame's pairs carry the footprint at the largest A over
 * the view's tables (it contains every frame's own footprint), the other frames' counts are
 * 0, and tiles are numbered per view (global tile id v * tiles_x * tiles_y + local, so
 * proj->total_tiles = n_views * tiles_x * tiles_y).  Every frame's record holds the shared
 * geometry (centre relative to the shared rectangle) with its own A and colour, A = 0
 * where the frame's own footprint culls the Gaussian (A below alpha_min or no pixel
 * centre covered), so each frame keeps exactly the Gaussians veg_project would keep for
 * it.  The blend passes then give each frame the
 * image and gradients of its own footprint (each frame skips pixel by pixel what its A
 * puts below alpha_min); only the float32 rounding of the centre offset may differ from
 * veg_project's.
 *   n_views * tfs_per_view = proj->n_frames <= VEG_MAX_FRAMES; cams host [n_views];
 *   tfs host [n_views * tfs_per_view].  Sets proj->tfs_per_view.
 *   veg_bins.hits (optional) must then hold tfs_per_view * veg_bin_hit_words(capacity,
 *   total_tiles) words: one block of hit bits per frame slot.
 * Errors: as veg_project, and tfs_per_view outside 1..VEG_MAX_FRAMES. */
veg_status veg_project_views(const veg_gaussians* g, int32_t n_views, int32_t tfs_per_view,
                             const veg_camera* cams, const veg_tf* tfs, const veg_opts* opts,
                             veg_proj* proj, veg_stream_t stream);

/* ----------------------------------------------------------------------------------
 * Binning and sorting  (the tile-based rasterizer's key list)
 * ---------------------------------------------------------------------------------- */

/* Sorted key list.  Entry j is (keys[j] = global tile id, vals[j] = pair id); global tile
 * id = f * tiles_x * tiles_y + ty * tiles_x + tx (v instead of f for the views of
 * veg_project_views, whose lists are the views' owners' pairs).  Entries are ordered by (tile, depth
 * key, Gaussian index).  ranges[2t], ranges[2t+1] = [start, end) of tile t (0,0 if empty).
 *   keys, vals          device [capacity] uint32 (final sorted list)
 *   keys_alt, vals_alt  device [capacity] uint32 (ping-pong buffers of the sort; afterwards
 *                       veg_render_fwd and veg_render_bwd overwrite keys_alt with the order
 *                       in which they dispatch the (frame, tile) blocks, longest list
 *                       first, when capacity >= n_frames * tiles_x * tiles_y + 128; with
 *                       less they dispatch in natural order.  Results do not depend on it.
 *                       Calls that share a veg_bins must therefore be ordered on one stream.)
 *   ranges              device [2 * total_tiles] uint32
 *   capacity            entries the buffers hold (<= 2^31 - 1)
 *   hits, hit_words     optional (NULL, 0): device [hit_words] uint64, hit_words >=
 *                       tfs_per_view * veg_bin_hit_words(capacity, total_tiles).  When given,
 *                       veg_render_fwd records for every entry whether it was blended into
 *                       at least one pixel of its tile, and veg_render_bwd, called with the
 *                       same bins after that forward call, visits only those entries (the
 *                       others contribute nothing to any gradient). */
typedef struct {
  uint32_t* keys;
  uint32_t* vals;
  uint32_t* keys_alt;
  uint32_t* vals_alt;
  uint32_t* ranges;
  int64_t capacity;
  uint64_t* hits;
  int64_t hit_words;
} veg_bins;

/* Words of veg_bins.hits for a list of `capacity` entries over `total_tiles` tiles
 * (one bit per entry, each tile's bits starting in a word of its own; the key list of the
 * tile-based rasterizer of section "Rendering of VEGs"). */
int64_t veg_bin_hit_words(int64_t capacity, int64_t total_tiles);

/* Scratch for veg_bin_count / veg_bin_sort of `n_pairs` pairs and `capacity` entries (the
 * binning of section "Rendering of VEGs"). */
size_t veg_bin_workspace_bytes(int64_t n_pairs, int64_t capacity);

/* veg_bin_count -- the first half of the binning of the tile-based rasterizer (section
 * "Rendering of VEGs": Gaussians binned to tiles and sorted front to back before blending):
 * compacts the kept pairs, sorts them front to back by (depth key, pair id) with a stable
 * LSD radix sort, and prefix-sums their tile counts in that order.
 *   ws, ws_bytes     device scratch, >= veg_bin_workspace_bytes(pairs, capacity) where
 *                    capacity is the value later passed to veg_bin_sort (may be 0 here if
 *                    the same ws is re-queried: only the first part is used by this call)
 *   n_entries        host out (optional): total key-list length E.  When non-NULL the
 *                    call synchronises `stream` to read it; when NULL nothing waits and
 *                    E stays on the device for veg_bin_sort.
 * Errors: VEG_ERR_INVALID_ARG, VEG_ERR_HIP. */
veg_status veg_bin_count(const veg_proj* proj, void* ws, size_t ws_bytes, int64_t* n_entries,
                         veg_stream_t stream);

/* veg_bin_sort -- the second half of the binning (section "Rendering of VEGs"): writes
 * every (tile, pair) entry of the kept pairs in front-to-back order, sorts the list stably
 * by tile (LSD radix over the bits of the largest tile id), and derives the per-tile
 * ranges.  Needs the workspace state left by veg_bin_count.
 * If the device-side E exceeds bins->capacity, only the first `capacity` entries are
 * written, the ranges are not valid, and the overflow flag read by veg_bin_overflow is
 * set (no synchronisation happens here).
 * Errors: VEG_ERR_INVALID_ARG (capacity < 0, NULL buffers with capacity > 0),
 *   VEG_ERR_HIP. */
veg_status veg_bin_sort(const veg_proj* proj, void* ws, size_t ws_bytes, const veg_bins* bins,
                        veg_stream_t stream);

/* Reads (synchronising `stream`) the entry count and overflow flag of the tile key list
 * (section "Rendering of VEGs") left in `ws`. */
veg_status veg_bin_overflow(void* ws, size_t ws_bytes, int64_t* n_entries, int32_t* overflow,
                            veg_stream_t stream);

/* veg_bin_status -- the same two values of the tile key list (the binning of section
 * "Rendering of VEGs") without synchronisation: writes dst[0] = E and
 * dst[1] = overflow flag (0 or 1) as int64, ordered on `stream` after the veg_bin_sort that
 * used `ws`.  Lets a caller that sizes the key list ahead (e.g. from an earlier step) keep
 * the GPU busy and check the flags of many calls in one later read.
 *   dst   device [2] int64, 8-byte aligned
 * Errors: VEG_ERR_INVALID_ARG (workspace too small, dst NULL or misaligned), VEG_ERR_HIP. */
veg_status veg_bin_status(void* ws, size_t ws_bytes, int64_t* dst, veg_stream_t stream);

/* veg_bin_static -- veg_bin_count followed by veg_bin_sort and veg_bin_status in one
 * call that allocates nothing and takes no workspace: for callers that cannot allocate
 * device memory (code under hipGraph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Its scratch is a fixed device array of the library (13 MiB per GPU, held
 * until the process ends), which limits a call to n_frames * n <= VEG_BIN_STATIC_MAX_PAIRS
 * pairs (e.g. one frame of a model of up to 262,144 Gaussians); larger calls fail with
 * VEG_ERR_INVALID_ARG before anything is enqueued.  The output is bit for bit that of
 * veg_bin_count + veg_bin_sort with a caller workspace.
 *   bins     as for veg_bin_sort
 *   status   device int64 [2], 8-byte aligned: (entries E, overflow flag), as veg_bin_status
 *            writes them, ordered on `stream` after the sort
 * Every call on one GPU shares that GPU's array, whose contents the next call overwrites
 * (it clears what must start at zero itself): calls ordered on one stream are safe, calls
 * that overlap on one GPU (different streams or host threads without ordering) race.
 * Errors: VEG_ERR_INVALID_ARG, VEG_ERR_HIP. */
#define VEG_BIN_STATIC_MAX_PAIRS 262144
veg_status veg_bin_static(const veg_proj* proj, const veg_bins* bins, int64_t* status, veg_stream_t stream);

/* ----------------------------------------------------------------------------------
 * Forward and backward blending  (Eq. 1 and its adjoint)
 * ---------------------------------------------------------------------------------- */

/* veg_render_fwd -- per pixel, front-to-back compositing of the tile's list (Eq. 1)
 * (the background colour is the one given to veg_project, kept in the frame descriptors):
 * sigma = 1/2 d^T conic d, d = pixel centre - projected centre; a = A exp(-sigma);
 * pairs with a < alpha_min are skipped; alpha = min(alpha_clamp, a); C += c alpha T;
 * T *= 1 - alpha; the pixel stops after the Gaussian that takes T below t_min.
 *   image    device [n_frames,3,H,W] out: C + T bg
 *   t_final  device [n_frames,H,W] out: final transmittance
 *   n_last   device [n_frames,H,W] out: index into the key list of the last blended
 *            entry, -1 if none (needed by veg_render_bwd)
 *   n_contrib device [n_frames,H,W] out, or NULL: number of Gaussians blended (not
 *            skipped) into the pixel
 * t_final and n_last may be NULL when no backward pass follows.
 * Errors: VEG_ERR_INVALID_ARG, VEG_ERR_HIP. */
veg_status veg_render_fwd(const veg_proj* proj, const veg_bins* bins, const veg_opts* opts,
                          float* image, float* t_final, int32_t* n_last, int32_t* n_contrib,
                          veg_stream_t stream);

/* veg_render_fwd_l1 -- veg_render_fwd fused with the L1 term of the training loss (section
 * "Training"; the image of Eq. 1): for every pixel and channel the final colour
 * c = C + T_final bg is compared with the target, and in place of the image
 *   d_image    = scale * sign(c - target)          (device [n_frames,3,H,W] float, overwritten;
 *                                                    sign(0) = 0; veg_l1_loss's d_image)
 *   loss_slots += scale * sum |c - target|         (device [VEG_L1_SLOTS] double: the loss is
 *                                                    the slots' sum; each tile adds to one slot)
 * are written; t_final, n_last and bins->hits as for veg_render_fwd (what veg_render_bwd
 * needs).  The colour is the one veg_render_fwd writes, so d_image equals what
 * veg_render_fwd followed by veg_l1_loss gives, without storing and re-reading the image.
 *   target   device [n_frames,3,H,W] float
 * Errors: VEG_ERR_INVALID_ARG, VEG_ERR_HIP. */
#define VEG_L1_SLOTS 64
veg_status veg_render_fwd_l1(const veg_proj* proj, const veg_bins* bins, const veg_opts* opts, const float* target,
                             float scale, double* loss_slots, float* d_image, float* t_final, int32_t* n_last,
                             veg_stream_t stream);

/* veg_render_bwd -- adjoint of veg_render_fwd (section "Rendering of VEGs": gradients
 * computed manually through the rasterizer).  Walks each tile's list backwards from
 * n_last, recovering T before each entry as T / (1 - alpha), and accumulates per pair
 * the gradient w.r.t. the screen-space quantities.
 *   t_final, n_last  device, as written by veg_render_fwd for the same proj/bins
 *   d_image          device [n_frames,3,H,W] dL/dimage
 *   g2d              device [n_frames*n][9] float (pair-major: a pair's nine values are
 *                    contiguous), ACCUMULATED: per pair
 *                    d mx, d my, d conic a, d conic b, d conic c, d R, d G, d B, d A,
 *                    where conic b enters sigma as 1/2 (a dx^2 + 2 b dx dy + c dy^2)
 * opts must satisfy alpha_clamp <= 1 - 2^-10 (the recovery divides by 1 - alpha) and
 * t_min (1 - alpha_clamp) >= 2^-100 (t_min = 0 lets T underflow), else
 * VEG_ERR_INVALID_ARG; the defaults (0.99, 1e-4) do.
 * Errors: VEG_ERR_INVALID_ARG, VEG_ERR_HIP. */
veg_status veg_render_bwd(const veg_proj* proj, const veg_bins* bins, const veg_opts* opts,
                          const float* t_final, const int32_t* n_last, const float* d_image,
                          float* g2d, veg_stream_t stream);

/* Parameter gradients, device, ACCUMULATED (+=).  d_weights may be NULL (then not
 * computed); it must be non-NULL only when the model has weights.  The five lighting
 * gradients are all NULL (not computed) or all non-NULL, the latter only for a model with
 * lighting attributes. */
typedef struct {
  float* d_means;       /* [n,3] */
  float* d_log_scales;  /* [n,3] */
  float* d_quats;       /* [n,4] */
  float* d_scalars;     /* [n]   */
  float* d_weights;     /* [n] or NULL */
  float* d_normals;     /* [n,3] or NULL */
  float* d_k_ambient;   /* [n] or NULL */
  float* d_k_diffuse;   /* [n] or NULL */
  float* d_k_specular;  /* [n] or NULL */
  float* d_shininess;   /* [n] or NULL */
} veg_grads;

/* veg_project_bwd -- chains g2d through the conic inverse, the EWA projection, the
 * covariance R S S^T R^T, the quaternion normalisation, exp of the log-scales, the
 * projected centre, the lighting of Eq. 2-3 (when the model has it: normal normalisation,
 * the light direction's dependence on the centre, coefficients, shininess; the derivative
 * of |n^ . l| is taken as 0 where it vanishes) and the transfer function's piecewise-linear
 * segments (slope of the segment to the right of a control point; zero outside [0,1]) to
 * the model parameters, summed over the frames of `proj`.
 * Errors: VEG_ERR_INVALID_ARG, VEG_ERR_HIP. */
veg_status veg_project_bwd(const veg_gaussians* g, const veg_proj* proj, const veg_opts* opts,
                           const float* g2d, const veg_grads* grads, veg_stream_t stream);

/* veg_project_bwd_fused -- veg_project_bwd with two neighbours of the training loop of
 * section "Training" folded into its pass over g2d (same gradients, bit for bit):
 *   grad_accum, vis_count  optional (both or neither): the densification statistics of
 *                          veg_densify_stats from the same reads (same values, ADDED)
 *   consume_g2d            non-zero: every g2d record is left zero after it is read, so the
 *                          buffer is ready for the next veg_render_bwd without a clear
 *                          (g2d is then device float, written)
 * Errors: as veg_project_bwd; VEG_ERR_INVALID_ARG when only one of grad_accum, vis_count
 * is given. */
veg_status veg_project_bwd_fused(const veg_gaussians* g, const veg_proj* proj, const veg_opts* opts, float* g2d,
                                 const veg_grads* grads, float* grad_accum, int32_t* vis_count, int32_t consume_g2d,
                                 veg_stream_t stream);

/* ----------------------------------------------------------------------------------
 * Loss and utilities
 * ---------------------------------------------------------------------------------- */

/* veg_l1_loss -- the L1 part of the training loss (section "Training": (1-lambda) L1 +
 * lambda SSIM; the SSIM part is veg_ssim_loss):
 *   loss   += scale * sum |image - target|            (device double, ACCUMULATED)
 *   d_image =  scale * sign(image - target)           (device float, overwritten;
 *                                                      sign(0) = 0)
 * over `count` floats.  scale is normally 1/(total pixel-channels of the step).
 * Errors: VEG_ERR_INVALID_ARG, VEG_ERR_HIP. */
veg_status veg_l1_loss(const float* image, const float* target, int64_t count, float scale,
                       double* loss, float* d_image, veg_stream_t stream);

/* veg_ssim_loss -- the SSIM part of the training loss (section "Training"; SSIM of Wang et
 * al. with the usual 11-tap Gaussian window, sigma 1.5, zeros outside the image,
 * C1 = 0.01^2, C2 = 0.03^2 for a data range of 1):
 *   loss    += weight * sum over planes and pixels of (1 - SSIM)   (device double)
 *   d_image += weight * d/dimage of that sum                       (device float, ADDED,
 *              so that it follows veg_l1_loss, which overwrites d_image)
 *   image, target  device [n_planes, height, width] float (e.g. frames x colour channels)
 *   ws, ws_bytes   device scratch >= veg_ssim_workspace_bytes(n_planes, width, height)
 * Errors: VEG_ERR_INVALID_ARG (sizes, NULLs, n_planes > 65535, small workspace), VEG_ERR_HIP. */
size_t veg_ssim_workspace_bytes(int64_t n_planes, int32_t width, int32_t height);
veg_status veg_ssim_loss(const float* image, const float* target, int64_t n_planes, int32_t width,
                         int32_t height, float weight, double* loss, float* d_image, void* ws,
                         size_t ws_bytes, veg_stream_t stream);

/* veg_image_loss -- the whole image loss of section "Training", (1-lambda) L1 + lambda SSIM,
 * in one pass over the images (veg_l1_loss and veg_ssim_loss fused):
 *   loss   += l1_scale * sum |image - target| + ssim_weight * sum (1 - SSIM)   (device double)
 *   d_image = l1_scale * sign(image - target) + ssim_weight * d/dimage sum (1 - SSIM)
 *             (device float, OVERWRITTEN; bit for bit what veg_l1_loss followed by
 *             veg_ssim_loss writes, without storing and re-reading the L1 gradient)
 * Sizes, window and workspace as for veg_ssim_loss; normally l1_scale = (1-lambda)/M and
 * ssim_weight = lambda/M for M pixel-channels.
 * Errors: VEG_ERR_INVALID_ARG (sizes, NULLs, non-finite weights, small workspace), VEG_ERR_HIP. */
veg_status veg_image_loss(const float* image, const float* target, int64_t n_planes, int32_t width, int32_t height,
                          float l1_scale, float ssim_weight, double* loss, float* d_image, void* ws, size_t ws_bytes,
                          veg_stream_t stream);

/* veg_adam_step -- one Adam update of a parameter array (the optimizer of section
 * "Training"; Kingma & Ba):  m <- b1 m + (1-b1) g,  v <- b2 v + (1-b2) g^2,
 *   param <- param - lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 *   param, m, v  device [count] float, updated in place; grad device [count] float
 *   step         1 for the first update
 * Errors: VEG_ERR_INVALID_ARG (NULLs, count < 0, step < 1, lr or betas out of range), VEG_ERR_HIP. */
veg_status veg_adam_step(float* param, const float* grad, float* m, float* v, int64_t count, float lr,
                         float beta1, float beta2, float eps, int32_t step, veg_stream_t stream);

/* veg_densify_stats -- statistics for the adaptive density control (section "Training":
 * gradients drive densification and pruning): for every Gaussian, over the frames of
 * `proj` in which it was kept, the norm of dL/d(projected centre) in pixels taken from
 * g2d, and the number of such frames.  Kept in a frame: its own footprint keeps it (tile
 * count > 0 from veg_project; for the views of veg_project_views, in the view's list
 * with the frame's own A > 0 in its record, which is the same set).
 *   g2d         device [n_frames*n][9], as accumulated by veg_render_bwd
 *   grad_accum  device [n] float, ADDED
 *   vis_count   device [n] int32, ADDED
 * Errors: VEG_ERR_INVALID_ARG, VEG_ERR_HIP. */
veg_status veg_densify_stats(const veg_proj* proj, const float* g2d, float* grad_accum, int32_t* vis_count,
                             veg_stream_t stream);

/* Adaptive density control (section "Training": densification and pruning after Kerbl et
 * al.; Gaussians with large view-space positional gradients are cloned or split, Gaussians
 * with a low weight are pruned).  Two calls: veg_densify_plan decides, veg_densify_apply
 * writes the new model.
 *
 * veg_densify_plan -- per Gaussian, with float32 comparisons:
 *   g = grad_accum / vis_count (0 where vis_count = 0: the statistics of veg_densify_stats);
 *   PRUNE (3) unless weights[i] >= prune_weight (weights NULL: never);
 *   else SPLIT (2) when g >= grad_thresh and max(log_scales[i]) > log_scale_thresh;
 *   else CLONE (1) when g >= grad_thresh;  else KEEP (0).
 *   grad_thresh is in pixels (the units of veg_densify_stats), log_scale_thresh in the
 *   model's log-scale units.
 *   action   device [n] uint8 out
 *   counts   host [4] out (optional): KEEP, CLONE, SPLIT, PRUNE; when non-NULL the call
 *            synchronises `stream` to read them.  The new model has
 *            n + CLONE + SPLIT - PRUNE Gaussians.
 *   ws       device scratch >= veg_densify_workspace_bytes(n); keeps per-block offsets for
 *            the following veg_densify_apply.
 * Errors: VEG_ERR_INVALID_ARG, VEG_ERR_HIP. */
size_t veg_densify_workspace_bytes(int64_t n);
veg_status veg_densify_plan(int64_t n, const float* grad_accum, const int32_t* vis_count,
                            const float* log_scales, const float* weights, float grad_thresh,
                            float log_scale_thresh, float prune_weight, uint8_t* action,
                            int64_t* counts, void* ws, size_t ws_bytes, veg_stream_t stream);

/* veg_densify_apply -- the clone / split / prune step of section "Training" (adaptive
 * density control): writes the model the plan describes into new arrays: first the
 * survivors (KEEP and CLONE) in index order, then one copy of each CLONE Gaussian in index
 * order, then the two children of each SPLIT Gaussian in index order (PRUNE Gaussians are
 * dropped).  Child c of parent i sits at mu_i + R(q_i) diag(exp(log_s_i)) z[i][c] and has
 * log-scales log_s_i - ln 1.6 (the 3DGS split: two samples of the parent, scale / 0.8 N);
 * the rest is copied.
 *   action, ws   as left by veg_densify_plan for the same n (same stream order)
 *   quats        device [n,4], log_scales device [n,3]: the parent's rotation and scale
 *   z            device [n][2][3] float: standard normal draws (only SPLIT rows are read);
 *                the random numbers are the caller's
 *   fields       host [n_fields] (1..16): src device [n][width], dst device
 *                [n + CLONE + SPLIT - PRUNE][width] (no overlap with src), role
 *                VEG_FIELD_COPY (copied to clones and children), VEG_FIELD_MEANS (width 3,
 *                children offset as above), VEG_FIELD_LOG_SCALES (width 3, children
 *                shrunk), VEG_FIELD_ZERO_NEW (0 for every new Gaussian: optimizer moments)
 * Errors: VEG_ERR_INVALID_ARG, VEG_ERR_HIP. */
#define VEG_FIELD_COPY 0
#define VEG_FIELD_MEANS 1
#define VEG_FIELD_LOG_SCALES 2
#define VEG_FIELD_ZERO_NEW 3
typedef struct {
  const float* src;
  float* dst;
  int32_t width;
  int32_t role;
} veg_densify_field;
veg_status veg_densify_apply(int64_t n, const uint8_t* action, const float* quats,
                             const float* log_scales, const float* z,
                             const veg_densify_field* fields, int32_t n_fields, const void* ws,
                             size_t ws_bytes, veg_stream_t stream);

/* veg_vq_decode -- expands vector-quantised model attributes into the structure-of-arrays
 * model (section "3D Gaussian Splatting": trained models are stored with most parameters
 * clustered into a codebook, after the compact-3DGS work it cites): Gaussian i's attribute
 * vector is
 * row idx[i] of `book`, split in order into the destination fields, e.g. a 7-wide shape
 * codebook into log_scales [n,3] and quats [n,4].
 *   idx       device [n] uint16
 *   book      device [k][dim] float32, row-major; 1 <= k <= 65536, 1 <= dim <= 16
 *   fields    host [n_fields] (1..8): dst device [n][width] float32 (overwritten),
 *             width >= 1; the widths sum to dim
 * An index >= k writes NaN to every field of that Gaussian, which the projection culls
 * (never a fault, never an error).  Storage of the indices and codebook is the caller's.
 * Errors: VEG_ERR_INVALID_ARG (sizes, NULL pointers, widths), VEG_ERR_HIP. */
typedef struct {
  float* dst;
  int32_t width;
} veg_vq_field;
veg_status veg_vq_decode(const uint16_t* idx, int64_t n, const float* book, int32_t k, int32_t dim,
                         const veg_vq_field* fields, int32_t n_fields, veg_stream_t stream);

/* Fills `count` 32-bit words at device pointer `dst` with `value` (a kernel, so it is
 * safe inside captured graphs): clears the gradient and statistics buffers of the
 * training step of section "Training". */
veg_status veg_fill_u32(void* dst, int64_t count, uint32_t value, veg_stream_t stream);

/* Diagnostics of the projection of section "Rendering of VEGs": runs the device's float32
 * helper `op` on n inputs (0 = exp32 of the footprint contract, 1 = log32, 2 = division
 * x/y, 3 = sqrt, 4 = wave prefix sum of
 * uint32 (bit pattern of x), 5 = wave sum of float) so tests can compare them with the
 * oracle.  in_x, in_y, out: device [n]. */
veg_status veg_debug_math(int32_t op, const float* in_x, const float* in_y, float* out,
                          int64_t n, veg_stream_t stream);

/* ----------------------------------------------------------------------------------
 * Serving: resident models, continuous batching of render requests.  The paper renders
 * its trained models in an interactive renderer (section "Evaluation"): every request is
 * the forward pass of section "Rendering of VEGs" for one camera and transfer function.
 * ---------------------------------------------------------------------------------- */

typedef struct veg_server veg_server;

/* Server configuration (serving the renderer of section "Evaluation").  Each of the
 * n_streams batch slots gets static device buffers
 * carved from `arena` for a batch of up to max_batch requests, max_pairs (frame,
 * Gaussian) pairs and max_entries key-list entries; veg_serve_arena_bytes gives the size
 * needed.  Requests of any model, camera, TF and resolution (<= max_width x max_height)
 * share a batch; requests whose options other than bg differ go to different batches. */
typedef struct {
  void* arena;               /* device memory the server sub-allocates (caller-owned) */
  size_t arena_bytes;
  size_t budget_bytes;       /* admission budget for in-flight request working memory */
  int32_t max_batch;         /* requests per batch (1..64) */
  int32_t n_streams;         /* concurrent batch slots (1..8) */
  int32_t use_graphs;        /* 1: each batch is one replay of a hipGraph captured per slot
                                and batch shape (request count and power-of-two bounds on
                                tiles per frame, Gaussians per model, pairs and entries) */
  int32_t max_width, max_height;   /* largest request resolution (<= VEG_MAX_DIM) */
  int32_t max_tf_k;          /* largest transfer-function table (2..4096 points) */
  int64_t max_gaussians;     /* largest resident model */
  int64_t max_pairs;         /* (frame, Gaussian) pairs per batch; 0 = max_batch * max_gaussians */
  int64_t max_entries;       /* key-list capacity per batch (entries, < 2^31) */
} veg_serve_config;

/* One render request: one frame of section "Rendering of VEGs" (Eq. 1) for a camera and
 * transfer function.  The camera and options are copied and the TF table (host memory)
 * is copied at submit; out_image / out_t_final are written when the request completes. */
typedef struct {
  int32_t model_id;
  veg_camera camera;
  const float* tf_rgba;      /* HOST [tf_k,4]; copied at submit */
  int32_t tf_k;
  float* out_image;          /* device [3,H,W], caller-owned, written on completion */
  float* out_t_final;        /* device [H,W] or NULL */
  veg_opts opts;             /* per request */
  double t_arrival;          /* arrival time, CLOCK_MONOTONIC seconds (the clock of C++'s
                                steady_clock and Python's time.perf_counter on Linux), from
                                which latency is measured; 0 = the time of the submit call */
} veg_request;

typedef struct {
  int64_t submitted, completed, failed, rejected, batches, retries;
  double mean_batch;
  double p50_ms, p99_ms, max_ms; /* arrival -> completion observed by the scheduler */
  double throughput_rps;         /* completed / (last completion - first arrival) */
  double mpix_per_s;
  double gpu_busy_frac;          /* fraction of that interval with >= 1 batch in flight */
  int64_t peak_bytes;            /* peak admitted working-memory estimate */
  int64_t graphs_captured;       /* graphs captured so far (one per slot and batch shape) */
} veg_serve_stats;

enum { VEG_REQ_QUEUED = 0, VEG_REQ_RUNNING = 1, VEG_REQ_DONE = 2, VEG_REQ_FAILED = 3 };

/* Device bytes the server needs in `arena` for this configuration (0 if invalid). */
size_t veg_serve_arena_bytes(const veg_serve_config* cfg);
/* Creates a server; a scheduler thread admits queued requests while their estimated
 * memory fits budget - in_use, packs them into batches of up to max_batch requests of
 * any model, camera, TF and resolution, and runs each batch (projection, binning,
 * sorting, blending) on one of n_streams streams so batches overlap.  Memory of a batch
 * returns to the budget when its completion event fires, which admits waiting requests.
 * Errors: VEG_ERR_INVALID_ARG, VEG_ERR_HIP. */
veg_status veg_serve_create(const veg_serve_config* cfg, veg_server** out);
/* Registers a resident model (device SoA, caller-owned, must outlive the server). */
veg_status veg_serve_add_model(veg_server* s, const veg_gaussians* g, int32_t* model_id);
/* Queues a request (any thread).  VEG_ERR_OUT_OF_BUDGET if it can never fit,
 * VEG_ERR_NOT_FOUND for an unknown model, VEG_ERR_INVALID_ARG for a bad request. */
veg_status veg_serve_submit(veg_server* s, const veg_request* r, uint64_t* req_id);
/* State of a request (VEG_REQ_*); VEG_ERR_NOT_FOUND for an unknown id. */
veg_status veg_serve_poll(veg_server* s, uint64_t req_id, int32_t* state);
/* Waits until the request is done or failed (timeout_ms < 0: forever).  VEG_OK when its
 * image is complete, VEG_ERR_TIMEOUT, or the request's failure status.  A request that
 * has been waited on to completion is released: its id is unknown afterwards (a second
 * wait, also one racing with the first, returns VEG_ERR_NOT_FOUND). */
veg_status veg_serve_wait(veg_server* s, uint64_t req_id, int32_t timeout_ms);
/* Latency/throughput statistics over the requests completed since the last reset (a
 * reset clears the statistics only; requests not yet waited on stay waitable). */
veg_status veg_serve_stats_get(veg_server* s, veg_serve_stats* out);
veg_status veg_serve_stats_reset(veg_server* s);
/* Drains in-flight work, stops the scheduler and frees host resources. */
veg_status veg_serve_destroy(veg_server* s);

#ifdef __cplusplus
}
#endif
#endif /* VEG_H */
