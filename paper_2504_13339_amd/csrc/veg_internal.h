// Internal declarations shared by the translation units of libveg: the device data layout
// (frame descriptors, options) and the host-side launchers.  Device-only helpers live in
// veg_device.h, so the host-only sources (the C entry points, the server) also build with
// a plain C++ compiler against the HIP runtime API.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "veg.h"

namespace veg {

constexpr int kTile = VEG_TILE;

// The record's last word: frame index in the low kFrameBits bits; above them, for frames
// that share a key list, the frame's own tile rectangle as four 5-bit insets from the
// shared rectangle (x0, y0, x1, y1 order; 31 = at least 31 tiles, a conservative bound).
constexpr uint32_t kFrameBits = 12;
constexpr uint32_t kFrameMask = (1u << kFrameBits) - 1u;
static_assert(VEG_MAX_FRAMES <= (1 << kFrameBits), "frame index must fit the record's frame field");
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

// Per-frame descriptor in device memory.  The stateless API writes one per frame in
// veg_project; the server writes one per request of a batch.  Kernels read it with
// wave-uniform (scalar) loads.
struct alignas(16) FrameDesc {
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* scalars;
  const float* weights;      // may be null
  const float* normals;      // lighting attributes; all null for TF colour only
  const float* k_ambient;
  const float* k_diffuse;
  const float* k_specular;
  const float* shininess;
  const float* lut;          // [K,4]
  float* out_image;          // per-frame outputs (server); null in the stateless API
  float* out_tfinal;
  int32_t* out_nlast;
  int32_t K;
  int32_t n;                 // Gaussians of this frame
  int32_t W, H, tiles_x, tiles_y;
  uint32_t pair_base;        // first pair id of this frame
  uint32_t tile_base;        // first global tile id of this frame
  uint32_t pix_base;         // first pixel of this frame in batched per-pixel buffers
  uint32_t list_frame;       // frame whose key list this frame blends (itself unless shared)
  float view[12];
  float fx, fy, cx, cy;
  float bg[3];
  float campos[3];           // camera centre in world space (headlight position)
  int32_t slot;              // position among the frames sharing the list (0 = owner)
  int32_t n_share;           // owner: frames sharing its list (>= 1); 0 on the other frames
  uint32_t pad1[2];
};
static_assert(sizeof(FrameDesc) == 256, "FrameDesc layout");

// Options as the kernels use them (derived once on the host).
struct KOpts {
  float alpha_clamp, alpha_min, t_min, lowpass, near_z, guard;
  float log2_alpha_min;      // skip test in the log2 domain of the blend kernels
  float bg0, bg1, bg2;
};

// Thread-local message returned by veg_last_error (defined with the C entry points).
void set_last_error(const char* msg);

// ---------------------------------------------------------------------------------------
// Host-side launchers (one translation unit each)
// ---------------------------------------------------------------------------------------

// Copies `bytes` (multiple of 4, <= kBlobMaxBytes) from host to device through kernel
// arguments, so the host buffer may be freed at once and no pageable copy is needed.
constexpr int kBlobMaxBytes = 3072;
hipError_t write_blob(void* dst_dev, const void* src_host, size_t bytes, hipStream_t stream);

hipError_t launch_project(const FrameDesc* descs, int n_frames, int n_max, const KOpts& o,
                          float4* rec, uint32_t* count, uint32_t* depth, bool shared_model,
                          hipStream_t stream);
// Extras of the projection backward: the densification statistics from the same g2d reads
// (acc, vis: per Gaussian, added; count/depth/rec of the projection for the kept test) and,
// with consume, every g2d record left zero after it is read.
struct BwdFused {
  const uint32_t* count = nullptr;
  const uint32_t* depth = nullptr;
  const float4* rec = nullptr;
  float* acc = nullptr;
  int32_t* vis = nullptr;
  int consume = 0;
};
hipError_t launch_project_bwd(const FrameDesc* descs, int n_frames, int n, const KOpts& o,
                              float* g2d, uint32_t n_pairs, const veg_grads& grads, hipStream_t stream,
                              const BwdFused& fused = BwdFused{});

// Lighting attributes of a model and the camera centre (-R^T t of the world->camera
// transform [R|t]) into a frame descriptor.
// A frame that owns its key list alone.
inline void set_own_list(FrameDesc& d, int f) {
  d.list_frame = (uint32_t)f;
  d.slot = 0;
  d.n_share = 1;
}

inline void set_lighting(FrameDesc& d, const veg_gaussians& g, const veg_camera& c) {
  d.normals = g.normals;
  d.k_ambient = g.k_ambient;
  d.k_diffuse = g.k_diffuse;
  d.k_specular = g.k_specular;
  d.shininess = g.shininess;
  for (int j = 0; j < 3; ++j)
    d.campos[j] = (float)(-((double)c.view[j] * c.view[3] + (double)c.view[4 + j] * c.view[7] +
                            (double)c.view[8 + j] * c.view[11]));
}

// Binning pipeline (workspace-based).  `pairs` and `capacity` bound the device counts.
struct BinWs {
  uint32_t* dkeyA;
  uint32_t* dvalA;
  uint32_t* dkeyB;
  uint32_t* dvalB;
  uint32_t* items;          // [pairs] uint4: depth-sorted (pair, rect01, rect23, frame)
  uint32_t* partials;       // [kMaxScanBlocks] uint64: entry-offset scan, kept from count to sort
  uint32_t* partials_tmp;   // [kMaxScanBlocks] uint64: scratch for the other scans
  uint32_t* hist;       // [kRadix * kMaxHistBlocks]
  uint32_t* counters;   // [0] kept pairs V, [1..2] entries E (uint64), [3] overflow flag,
                        // [4] entries written min(E, capacity), [8..9] V (uint64),
                        // [kDepthRange..+1] ~smallest and largest kept depth key
};
constexpr int kDepthRange = 12;
constexpr int kMaxScanBlocks = 4096;
constexpr int kMaxSortBlocks = 2048;
constexpr int kMaxHistBlocks = kMaxScanBlocks > kMaxSortBlocks ? kMaxScanBlocks : kMaxSortBlocks;
size_t bin_ws_bytes(int64_t pairs);
void carve_bin_ws(void* ws, int64_t pairs, BinWs* out);

// The library's own binning scratch (veg_bin_static): room for the workspace of
// VEG_BIN_STATIC_MAX_PAIRS pairs (bin_ws_bytes(2^18) is 12.07 MiB), one copy per device.
constexpr size_t kStaticBinBytes = (size_t)13 << 20;
constexpr int kStaticBinMaxDevices = 64;
// Address of the current device's copy (looked up once per device, then cached).
hipError_t static_bin_scratch(void** out);

// n_pairs bounds the pair count; when n_pairs_dev is non-null the actual count is read
// from device memory (capacity mode, used by the server's captured graphs).  With views of
// per_view > 1 frames of list_n Gaussians sharing the first frame's list, only those first
// frames' pair slots are compacted (n_pairs a multiple of list_n * per_view, no n_pairs_dev).
hipError_t launch_bin_count(const float4* rec, const uint32_t* count, const uint32_t* depth, uint32_t n_pairs,
                            const BinWs& ws, hipStream_t stream, const uint32_t* n_pairs_dev = nullptr,
                            uint32_t list_n = 0, int per_view = 1);
hipError_t launch_bin_sort(const FrameDesc* descs, int n_frames, const float4* rec,
                           const uint32_t* count, uint32_t n_pairs, uint32_t total_tiles,
                           const BinWs& ws, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                           uint32_t* vals_alt, uint32_t* ranges, uint32_t capacity,
                           hipStream_t stream);

// Frames come in views of `per_view` consecutive frames that share the first one's key
// list (per_view = 1: every frame owns its list).  Hit bits of the frame in slot k start at
// word k * hit_stride.  order_ws (order_ws_words uint32, may be NULL) is scratch for the
// blocks' dispatch order, used when it holds n_frames * max_tiles + 128 words.
// The L1 term of the loss fused into the forward pass's epilogue (target NULL: off).
constexpr int kL1Slots = 64;
struct L1Fuse {
  const float* target = nullptr;   // [n_frames,3,H,W]
  double* loss = nullptr;          // [kL1Slots], added
  float scale = 0.0f;
};
hipError_t launch_blend_fwd(const FrameDesc* descs, int n_frames, int per_view, int max_tiles, const KOpts& o,
                            const float4* rec, const uint32_t* vals, const uint32_t* ranges,
                            float* image, float* tfinal, int32_t* nlast, int32_t* ncontrib,
                            uint64_t* hits, uint64_t hit_stride, const uint32_t* keep_bits,
                            uint32_t* order_ws, uint64_t order_ws_words, hipStream_t stream,
                            const L1Fuse& l1 = L1Fuse{});
hipError_t launch_blend_bwd(const FrameDesc* descs, int n_frames, int max_tiles, const KOpts& o,
                            const float4* rec, const uint32_t* vals, const uint32_t* ranges,
                            const float* tfinal, const int32_t* nlast, const float* dimage,
                            float* g2d, uint32_t n_pairs, const uint64_t* hits, uint64_t hit_stride,
                            uint32_t* order_ws, uint64_t order_ws_words, hipStream_t stream);

hipError_t launch_l1(const float* image, const float* target, int64_t count, float scale,
                     double* loss, float* dimage, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t* dst, int64_t count, uint32_t value, hipStream_t stream);
hipError_t launch_bin_status(const uint32_t* counters, int64_t* dst, hipStream_t stream);
// With with_l1, d_image is overwritten with the L1 term's gradient plus the SSIM term's and
// l1_scale * sum |image - target| joins the loss (the L1 pass fused in); else d_image is added to.
hipError_t launch_ssim(const float* image, const float* target, int64_t n_planes, int W, int H, float weight,
                       double* loss, float* d_image, float* dmaps, hipStream_t stream, bool with_l1 = false,
                       float l1_scale = 0.0f);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, hipStream_t stream);
hipError_t launch_densify_stats(const FrameDesc* descs, int n_frames, int n, const uint32_t* count,
                                const uint32_t* depth, const float4* rec, const float* g2d, float* acc, int32_t* vis,
                                hipStream_t stream);
// Attribute arrays carried through a densification (kernel argument by value); role:
// 0 copied to clones and children, 1 means, 2 log-scales, 3 zero for new Gaussians.
constexpr int kDensifyMaxFields = 16;
struct DensifyFields {
  const float* src[kDensifyMaxFields];
  float* dst[kDensifyMaxFields];
  int32_t width[kDensifyMaxFields];
  int32_t role[kDensifyMaxFields];
  int32_t n_fields;
};
hipError_t launch_densify_plan(int64_t n, const float* acc, const int32_t* vis, const float* log_scales,
                               const float* weights, float grad_thresh, float log_scale_thresh, float prune_weight,
                               uint8_t* action, uint32_t* blk, uint32_t* tot, hipStream_t stream);
hipError_t launch_densify_apply(int64_t n, const uint8_t* action, const float* quats, const float* log_scales,
                                const float* z, const uint32_t* blk, const uint32_t* tot, const DensifyFields& fl,
                                hipStream_t stream);

// Destination fields of a codebook decode (kernel argument by value).
constexpr int kVqMaxFields = 8;
struct VqFields {
  float* dst[kVqMaxFields];
  int32_t width[kVqMaxFields];
  int32_t n_fields;
};
hipError_t launch_vq_decode(const uint16_t* idx, int64_t n, const float* book, int k, int dim, const VqFields& fl,
                            hipStream_t stream);
hipError_t launch_debug_math(int op, const float* x, const float* y, float* out, int64_t n,
                             hipStream_t stream);

}  // namespace veg
