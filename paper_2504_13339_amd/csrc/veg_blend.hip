// Front-to-back blending (paper, Eq. 1) and its adjoint.
//
// One 64-lane wave per 16x16 tile; lane l owns pixel (l & 7, l >> 3) of each 8x8 quadrant,
// and the wave takes the quadrants one after another, so the lanes active for an entry in
// one step are a compact 8x8 block: a small footprint wakes up only the quadrants it
// touches, the others are skipped whole (empty execution mask).  The
// tile's list is staged through LDS in batches of 64 entries: each lane fetches one
// record, turns it into tile-local, log2-scaled form, and the wave then walks the batch
// with every lane reading the same LDS slot (a broadcast).  A pixel stops after the
// Gaussian that takes its transmittance below t_min; the wave leaves the tile when all 256
// pixels have stopped (ballot).
//
// Forward and backward must take identical skip decisions, so both evaluate the exponent
// through the same inline functions, written with explicit fmaf and no contraction.
#include "veg_internal.h"

#pragma clang fp contract(off)

namespace veg {
namespace {

constexpr int kBatch = 64;
constexpr int kKeepBitsMinFrames = 4;   // views of this many frames skip dead entries by keep bits
constexpr float kLog2e = 0x1.715476p+0f;

struct Staged {
  float mx, my;   // centre relative to the tile origin (pixels)
  float q0, q1, q2;  // conic scaled so that sigma * log2(e) = q0 dx^2 + q1 dx dy + q2 dy^2
  float l2A;      // log2(A)
};

__device__ __forceinline__ Staged stage(const float4 r0, const float4 r1, const float4 r2, int tx, int ty) {
  const uint32_t rect01 = __float_as_uint(r2.y);
  const int x0 = (int)(rect01 & 0xffffu), y0 = (int)(rect01 >> 16);
  Staged s;
  // r0.x is measured from pixel 16*x0; the tile origin is 16*tx.  Exact in float32.
  s.mx = r0.x - (float)(kTile * (tx - x0));
  s.my = r0.y - (float)(kTile * (ty - y0));
  s.q0 = r0.z * (0.5f * kLog2e);
  s.q1 = r0.w * kLog2e;
  s.q2 = r1.x * (0.5f * kLog2e);
  s.l2A = __log2f(r1.y);
  return s;
}

// Quadrants of the tile (bit r: pixel centres x in 8 (r & 1) + [0.5, 7.5], y in
// 8 (r >> 1) + [0.5, 7.5]) that can hold a pixel passing the skip test.  A pixel passes when
// the computed exponent l2A - Q(dx, dy) reaches l2min, Q = q0 dx^2 + q1 dx dy + q2 dy^2.  The
// computed value differs from the exact one by a few roundings of its largest terms: of
// |l2A| and, inside the ellipse Q <= R, of q0 dx^2 + |q1 dx dy| + q2 dy^2 <=
// 4 R (2 q0 q2 + |q1| sqrt(q0 q2)) / D, D = 4 q0 q2 - q1^2 (which grows with the
// ellipse's elongation).  R' = l2A - l2min + 1e-4 (1 + |l2A|) + 2^-20 (|l2A| + that bound)
// therefore contains every passing pixel; the ellipse's half-extents are sqrt(4 R' q2 / D)
// and sqrt(4 R' q0 / D), widened once more before the overlap test.  A quadrant outside
// that box has no passing pixel, so skipping it changes nothing.  Degenerate forms, and
// forms so elongated (4 q0 q2 > 1024 D) that the rounding of D itself matters, keep every
// quadrant.
__device__ __forceinline__ uint32_t quad_mask(const Staged& s, float l2min) {
  const float rp = (s.l2A - l2min) + 1e-4f * (1.0f + fabsf(s.l2A));
  if (!(rp >= 0.0f)) return 0u;   // below the threshold everywhere (or A = 0)
  const float D = 4.0f * s.q0 * s.q2 - s.q1 * s.q1;
  if (!(s.q0 > 0.0f) || !(s.q2 > 0.0f) || !(D > 0.0f)) return 0xfu;
  const float k4 = 4.0f * s.q0 * s.q2;
  if (!(k4 <= 1024.0f * D)) return 0xfu;
  const float terms = 4.0f * rp * (0.5f * k4 + fabsf(s.q1) * sqrtf(s.q0 * s.q2)) / D;
  const float rw = rp + 0x1p-20f * (fabsf(s.l2A) + terms);
  const float ex = sqrtf(4.0f * rw * s.q2 / D) * 1.001f + 0.01f;
  const float ey = sqrtf(4.0f * rw * s.q0 / D) * 1.001f + 0.01f;
  if (!(ex < 1e30f) || !(ey < 1e30f)) return 0xfu;
  const bool xl = s.mx - ex <= 7.5f && s.mx + ex >= 0.5f;    // columns 0..7
  const bool xh = s.mx - ex <= 15.5f && s.mx + ex >= 8.5f;   // columns 8..15
  const bool yl = s.my - ey <= 7.5f && s.my + ey >= 0.5f;
  const bool yh = s.my - ey <= 15.5f && s.my + ey >= 8.5f;
  return (uint32_t)(xl && yl) | ((uint32_t)(xh && yl) << 1) | ((uint32_t)(xl && yh) << 2) |
         ((uint32_t)(xh && yh) << 3);
}

// log2 of A exp(-sigma) for a pixel centre at (px, py) in tile-local coordinates:
//   base = l2A - q0 dx^2,  e = base - dy (q2 dy + q1 dx).
__device__ __forceinline__ float exponent_base(float q0, float l2A, float dx) { return fmaf(-q0 * dx, dx, l2A); }
// The same from nq0 = -q0 (the backward stages it negated): negation is exact, so the
// product and the result are bit for bit those of exponent_base.
__device__ __forceinline__ float exponent_base_neg(float nq0, float l2A, float dx) { return fmaf(nq0 * dx, dx, l2A); }
__device__ __forceinline__ float exponent(float base, float q1dx, float q2, float dy) {
  return fmaf(-dy, fmaf(q2, dy, q1dx), base);
}

// Word of the per-entry hit bits that holds entry rg.x + 64 b of global tile gt: tile gt's
// words start at floor(rg.x / 64) + gt, which keeps the tiles' words disjoint and needs
// floor(E / 64) + tiles + 1 words for E entries.
__device__ __forceinline__ size_t hit_word(uint32_t start, uint32_t gt, uint32_t b) {
  return (size_t)(start >> 6) + gt + b;
}

// OR over the wave; the result is complete in lane 63.
__device__ __forceinline__ uint32_t wave_or_u32(uint32_t v) {
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);   // row_shr:1
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);   // row_shr:2
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);   // row_shr:4
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);   // row_shr:8
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}
__device__ __forceinline__ uint64_t wave_or_u64(uint64_t v) {
  return ((uint64_t)wave_or_u32((uint32_t)(v >> 32)) << 32) | wave_or_u32((uint32_t)v);
}

// ---------------------------------------------------------------------------------------
// Dispatch order.  A block's cost grows with its tile's list length, and lengths span
// several orders of magnitude (a dense centre tile holds thousands of entries, a border tile
// a handful).  In natural order the heavy centre tiles of the last frames start late and
// run nearly alone at the end of the launch.  Blocks are therefore dispatched longest list
// first: a counting sort buckets the (frame, tile) blocks by floor(log2(list length)),
// heaviest bucket first and empty tiles last (a histogram pass, then a scatter pass).  The
// order within a bucket is arbitrary.  No result depends on it: a pixel is blended by one
// block alone, and the backward pass's float atomics are unordered in any case.
constexpr int kOrderBuckets = 33;        // clz(length) = 0..31, then empty tiles
constexpr uint32_t kOrderHeader = 128;   // scratch words ahead of the order: counts, cursors

__device__ __forceinline__ int order_bucket(const FrameDesc* __restrict__ descs, const uint2* __restrict__ ranges,
                                            uint32_t g, uint32_t max_tiles) {
  const FrameDesc& d = descs[g / max_tiles];
  const int t = (int)(g % max_tiles);
  if (t >= d.tiles_x * d.tiles_y) return kOrderBuckets - 1;
  const uint2 rg = ranges[descs[d.list_frame].tile_base + t];
  return rg.y > rg.x ? (int)__clz(rg.y - rg.x) : kOrderBuckets - 1;
}

// cnt[b] += blocks of bucket b (one LDS histogram per 256 blocks)
__global__ __launch_bounds__(256) void order_count_kernel(const FrameDesc* __restrict__ descs,
                                                          const uint2* __restrict__ ranges, uint32_t n,
                                                          uint32_t max_tiles, uint32_t* __restrict__ cnt) {
  __shared__ uint32_t h[kOrderBuckets];
  if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t g = blockIdx.x * 256u + threadIdx.x;
  if (g < n) atomicAdd(&h[order_bucket(descs, ranges, g, max_tiles)], 1u);
  __syncthreads();
  if (threadIdx.x < kOrderBuckets && h[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], h[threadIdx.x]);
}

// order[start of bucket b + running slot] = g; a bucket's slots are claimed 256 blocks at a
// time through the cursors cnt[kOrderBuckets + b]
__global__ __launch_bounds__(256) void order_scatter_kernel(const FrameDesc* __restrict__ descs,
                                                            const uint2* __restrict__ ranges, uint32_t n,
                                                            uint32_t max_tiles, uint32_t* __restrict__ cnt,
                                                            uint32_t* __restrict__ order) {
  __shared__ uint32_t h[kOrderBuckets], base[kOrderBuckets];
  if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t g = blockIdx.x * 256u + threadIdx.x;
  int b = 0;
  uint32_t r = 0u;
  if (g < n) {
    b = order_bucket(descs, ranges, g, max_tiles);
    r = atomicAdd(&h[b], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kOrderBuckets) {
    uint32_t start = 0u;
    for (int i = 0; i < (int)threadIdx.x; ++i) start += cnt[i];
    base[threadIdx.x] = start + (h[threadIdx.x] ? atomicAdd(&cnt[kOrderBuckets + threadIdx.x], h[threadIdx.x]) : 0u);
  }
  __syncthreads();
  if (g < n) order[base[b] + r] = g;
}

// The block's (frame, tile) id, frame * gridDim.x + tile, in dispatch order.
__device__ __forceinline__ uint32_t block_id(const uint32_t* __restrict__ order) {
  const uint32_t lin = blockIdx.y * gridDim.x + blockIdx.x;
  return order ? order[lin] : lin;
}

// One wave per tile.  A pixel is finished exactly when its T < t_min (blend-then-stop),
// so T itself is the "still active" flag; pixels outside the image start with T = 0.
// With kHits, bit k of word b records whether entry rg.x + 64 b + k was blended into any
// pixel of the tile (the backward pass skips the others).  A pixel's blended entries of a
// batch are kept as a 64-bit mask (one OR per blend); the batch end derives from it both
// the hit word (OR over the wave) and the pixel's last blended entry (highest bit).  The
// alpha clamp is an integer minimum of the float bits (both operands are positive), which
// needs no canonicalising of the clamp inside the loop.
//
// A block renders one tile of one frame (block_id) over the key list of frame list_frame
// (itself unless the frame shares its view's list); the frame's record of an entry sits at the list's pair id plus
// the difference of the two frames' pair bases.  With kShared the staged batch keeps only
// the entries live for this frame (its own A > 0 and the tile inside its own rectangle,
// from the record's insets), packed to the front of the batch, so the walk costs what the
// frame's own list would.
template <bool kCount, bool kHits, bool kShared>
__global__ __launch_bounds__(64) void blend_fwd_kernel(const FrameDesc* __restrict__ descs, KOpts o,
                                                       const float4* __restrict__ rec,
                                                       const uint32_t* __restrict__ vals,
                                                       const uint2* __restrict__ ranges, float* __restrict__ image,
                                                       float* __restrict__ tfinal, int32_t* __restrict__ nlast,
                                                       int32_t* __restrict__ ncontrib, uint64_t* __restrict__ hits,
                                                       uint64_t hit_stride, const uint32_t* __restrict__ keep_bits,
                                                       const uint32_t* __restrict__ order, L1Fuse l1) {
  const uint32_t gid = block_id(order);
  const uint32_t frame = gid / gridDim.x;
  const FrameDesc& d = descs[frame];
  const FrameDesc& dl = kShared ? descs[d.list_frame] : d;
  const int tile = (int)(gid % gridDim.x);
  if (tile >= d.tiles_x * d.tiles_y) return;
  const int tx = tile % d.tiles_x, ty = tile / d.tiles_x;
  const uint2 rg = ranges[dl.tile_base + tile];
  const uint32_t roff = kShared ? d.pair_base - dl.pair_base : 0u;
  // shared lists: the view's keep bits of an entry's Gaussian sit in the depth slot of the
  // frame after the owner (list pair id + that frame's pair offset)
  const uint32_t koff = kShared ? descs[d.list_frame + 1].pair_base - dl.pair_base : 0u;
  const uint32_t kbit = kShared ? 1u << min(d.slot, 31) : 0u;
  uint64_t* fhits = kHits ? hits + (kShared ? (uint64_t)d.slot * hit_stride : 0ull) : nullptr;
  const int lane = threadIdx.x;
  const int qx = lane & 7, qy = lane >> 3;
  // tile-local pixel centres: quadrant r sits at (8 (r & 1), 8 (r >> 1))
  const float pxl0 = (float)qx + 0.5f, pxl1 = (float)(qx + 8) + 0.5f;
  const float pyl0 = (float)qy + 0.5f, pyl1 = (float)(qy + 8) + 0.5f;

  __shared__ float4 s_geo[kBatch];   // mx, my, q0, q1
  __shared__ float4 s_col[kBatch];   // q2, l2A, R, G
  __shared__ float s_b[kBatch];      // B
  __shared__ int s_k[kBatch];        // batch position of a packed entry | quadrant mask << 8

  const float tmin = o.t_min;
  float T[4], C[4][3];
  int last[4], cnt[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int px = tx * kTile + qx + 8 * (r & 1), py = ty * kTile + qy + 8 * (r >> 1);
    T[r] = (px < d.W && py < d.H) ? 1.0f : 0.0f;
    C[r][0] = C[r][1] = C[r][2] = 0.0f;
    last[r] = -1;
    cnt[r] = 0;
  }
  const float l2min = o.log2_alpha_min;
  const uint32_t aclamp_bits = __float_as_uint(o.alpha_clamp);
  for (uint32_t base = rg.x; base < rg.y; base += kBatch) {
    if (__all(T[0] < tmin && T[1] < tmin && T[2] < tmin && T[3] < tmin)) break;
    // stage the batch: only entries that can blend into some pixel of this tile (a quadrant
    // mask from the ellipse's box; for a frame on a shared list also its own footprint),
    // packed to the front; s_k keeps each one's position in the batch
    const uint32_t j = base + lane;
    bool live = j < rg.y;
    float4 r0, r1, r2;
    const float4* rp = nullptr;
    uint32_t p = 0u;
    if (live) {
      p = vals[j];
      if (kShared && keep_bits) live = (keep_bits[p + koff] & kbit) != 0u;
    }
    if (live) {
      rp = rec + 3 * (size_t)(p + roff);
      r1 = rp[1];
      r2 = rp[2];
      if (kShared) {
        const uint32_t in = __float_as_uint(r2.w) >> kFrameBits;
        const uint32_t a = __float_as_uint(r2.y), b = __float_as_uint(r2.z);
        const int x0 = (int)((a & 0xffffu) + (in & 31u)), y0 = (int)((a >> 16) + ((in >> 5) & 31u));
        const int x1 = (int)((b & 0xffffu) - ((in >> 10) & 31u)), y1 = (int)((b >> 16) - ((in >> 15) & 31u));
        live = r1.y > 0.0f && tx >= x0 && tx <= x1 && ty >= y0 && ty <= y1;
      }
    }
    Staged st;
    uint32_t qm = 0u;
    if (live) {
      r0 = rp[0];
      st = stage(r0, r1, r2, tx, ty);
      qm = quad_mask(st, l2min);
      live = qm != 0u;
    }
    const uint64_t m = __ballot(live);
    const int n = __popcll(m);
    if (live) {
      const int slot = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      s_geo[slot] = make_float4(st.mx, st.my, st.q0, st.q1);
      s_col[slot] = make_float4(st.q2, st.l2A, r1.z, r1.w);
      s_b[slot] = r2.x;
      s_k[slot] = (int)(lane | (qm << 8));
    }
    __syncthreads();
    // Bit k of lq[r]: pixel r of this lane blended entry base + k.  The packed entries from
    // batch positions 0-31 come first (n_lo of them), so the walk goes in two runs, each
    // setting bits of one 32-bit half: one OR per blend instead of two.
    uint32_t lq_lo[4] = {0u, 0u, 0u, 0u}, lq_hi[4] = {0u, 0u, 0u, 0u};
    auto walk = [&](const int k, uint32_t (&lq)[4]) {
      const uint32_t kq = (uint32_t)__builtin_amdgcn_readfirstlane(s_k[k]);
      const uint32_t bit = 1u << (kq & 31u);   // position in the batch, modulo 32
      const float4 g = s_geo[k];
      const float4 c = s_col[k];
      const float cb = s_b[k];
      const float dx0 = pxl0 - g.x, dx1 = pxl1 - g.x;
      const float eb0 = exponent_base(g.z, c.y, dx0), eb1 = exponent_base(g.z, c.y, dx1);
      const float q1dx0 = g.w * dx0, q1dx1 = g.w * dx1;
      const float dy0 = pyl0 - g.y, dy1 = pyl1 - g.y;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (!(kq & (0x100u << r))) continue;   // quadrant out of the entry's reach (uniform)
        const float e = exponent((r & 1) ? eb1 : eb0, (r & 1) ? q1dx1 : q1dx0, c.x, (r >> 1) ? dy1 : dy0);
        if (T[r] >= tmin && e >= l2min) {
          lq[r] |= bit;
          const float alpha = __uint_as_float(min(__float_as_uint(__builtin_amdgcn_exp2f(e)), aclamp_bits));
          const float w = alpha * T[r];
          C[r][0] = fmaf(w, c.z, C[r][0]);
          C[r][1] = fmaf(w, c.w, C[r][1]);
          C[r][2] = fmaf(w, cb, C[r][2]);
          T[r] = fmaf(-alpha, T[r], T[r]);
          if (kCount) ++cnt[r];
        }
      }
    };
    const int n_lo = __builtin_amdgcn_readfirstlane(__popc((uint32_t)m));
    for (int k = 0; k < n_lo; ++k) walk(k, lq_lo);
    for (int k = n_lo; k < n; ++k) walk(k, lq_hi);
    uint64_t lq[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      lq[r] = (uint64_t)lq_hi[r] << 32 | lq_lo[r];
      if (lq[r]) last[r] = (int)base + 63 - __clzll(lq[r]);
    }
    if (kHits) {
      const uint64_t word = wave_or_u64(lq[0] | lq[1] | lq[2] | lq[3]);
      if (lane == 63) fhits[hit_word(rg.x, dl.tile_base + tile, (base - rg.x) >> 6)] = word;
    }
    __syncthreads();
  }
  const size_t HW = (size_t)d.W * d.H;
  const bool own = d.out_image != nullptr;   // per-frame outputs (server batches)
  float* img = own ? d.out_image : image + (size_t)frame * 3 * HW;
  float* tf = own ? d.out_tfinal : (tfinal ? tfinal + (size_t)frame * HW : nullptr);
  int32_t* nl = own ? d.out_nlast : (nlast ? nlast + (size_t)frame * HW : nullptr);
  int32_t* nc = own ? nullptr : (ncontrib ? ncontrib + (size_t)frame * HW : nullptr);
  // With the L1 term fused (the training loss of section "Training"), the pixel's colour is
  // compared with the target and the output holds scale * sign(colour - target) in place of
  // the colour; scale * sum |colour - target| goes to one of 64 loss slots.
  const bool fuse = l1.target != nullptr && !own;
  const float* tg = fuse ? l1.target + (size_t)frame * 3 * HW : nullptr;
  double lsum = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int px = tx * kTile + qx + 8 * (r & 1), py = ty * kTile + qy + 8 * (r >> 1);
    if (px < d.W && py < d.H) {
      const size_t pi = (size_t)py * d.W + px;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const float c = C[r][ch] + T[r] * d.bg[ch];
        if (fuse) {
          const float df = c - tg[ch * HW + pi];
          lsum += (double)fabsf(df);
          img[ch * HW + pi] = df > 0.0f ? l1.scale : (df < 0.0f ? -l1.scale : 0.0f);
        } else {
          img[ch * HW + pi] = c;
        }
      }
      if (tf) tf[pi] = T[r];
      if (nl) nl[pi] = last[r];
      if (kCount && nc) nc[pi] = cnt[r];
    }
  }
  if (fuse) {
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
    if (lane == 0 && lsum != 0.0) unsafeAtomicAdd(l1.loss + (gid & (kL1Slots - 1)), lsum * (double)l1.scale);
  }
}

__device__ __forceinline__ int wave_max_i32(int v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
  return v;
}

// Lane permutation within 16-lane rows (every source lane is valid, so bound_ctrl only
// lets the compiler fold the move into the consuming add).
template <int CTRL>
__device__ __forceinline__ float dpp_perm(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}

// Two entries' nine per-lane partial sums (a, b) summed over the wave by a reduce-scatter
// in which every step halves what a lane carries.  A swap of the wave's halves pairs a
// with b (lanes 0-31 go on with a's sums, lanes 32-63 with b's), a swap of adjacent rows
// pairs components (even rows go on with components 0, 2, 4, 6, odd rows with 1, 3, 5, 7,
// both with 8), and a butterfly over each 16-lane row (partners lane ^ 8 by row rotation,
// the mirror inside each half-row, then ^ 2 and ^ 1 inside quads) leaves every total in a
// lane of its row: with j = lane & 15 and r = lane >> 4, lane j = 0, 8, 4, 12 holds
// component 2 q + (r & 1) for q = 0, 1, 2, 3, and lane j = 2 of an even row component 8,
// of entry a in rows 0-1 and of entry b in rows 2-3.  The swaps need no lane selects, so
// a pair costs about 43 instructions instead of 59 for a butterfly over rows first.
__device__ __forceinline__ float wave_reduce_pair(const float (&a)[9], const float (&b)[9], int lane) {
  float p[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(a[c]), __float_as_uint(b[c]), false, false);
    p[c] = __uint_as_float(h[0]) + __uint_as_float(h[1]);
  }
  float q[5];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const auto r =
        __builtin_amdgcn_permlane16_swap(__float_as_uint(p[2 * c]), __float_as_uint(p[2 * c + 1]), false, false);
    q[c] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(p[8]), __float_as_uint(p[8]), false, false);
    q[4] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  const bool l1 = (lane & 8) == 0, l2 = (lane & 4) == 0, l3 = (lane & 2) == 0;
  const float r0 = (l1 ? q[0] : q[1]) + dpp_perm<0x128>(l1 ? q[1] : q[0]);   // row_ror:8
  const float r1 = (l1 ? q[2] : q[3]) + dpp_perm<0x128>(l1 ? q[3] : q[2]);
  const float r2 = q[4] + dpp_perm<0x128>(q[4]);
  const float s0 = (l2 ? r0 : r1) + dpp_perm<0x141>(l2 ? r1 : r0);   // half mirror
  const float s1 = r2 + dpp_perm<0x141>(r2);
  const float u = (l3 ? s0 : s1) + dpp_perm<0x4e>(l3 ? s1 : s0);   // quad_perm 2,3,0,1
  return u + dpp_perm<0xb1>(u);                                    // quad_perm 1,0,3,2
}

// Backward: the same tile walk in reverse.  Per pixel and blended entry it accumulates
// dL/dR,G,B, sum dsigma and the first and second moments of (dx, dy) weighted by dsigma;
// the conic is applied once per entry when the batch is flushed:
//   dL/dconic = (1/2 S_xx, S_xy, 1/2 S_yy),  dL/dmu' = -(a S_x + b S_y, b S_x + c S_y),
//   dL/dA = -S_d / A   with S_d = sum dsigma and dsigma = dL/dsigma = -dL/dalpha * a.
// Entries are taken in pairs: one reduce-scatter over the wave sums both entries' nine
// values at once, and the lanes left holding the totals store them into a per-entry LDS
// slot (plain stores: an entry is reduced once per tile); each 64-entry batch ends with
// nine vector atomics into the pair-major gradient records.
//
// At most 80 VGPRs, so that six waves share each SIMD instead of five: the pass is bound by
// vector issue and the sixth wave covers more of the LDS and dependency latency.  Measured
// about 2% faster than the 84-register allocation the compiler picks by itself, although
// the variant that tests hit bits then spills two registers (12 bytes of scratch a lane).
template <bool kHits>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(6, 8))) void blend_bwd_kernel(const FrameDesc* __restrict__ descs, KOpts o,
                                                       const float4* __restrict__ rec,
                                                       const uint32_t* __restrict__ vals,
                                                       const uint2* __restrict__ ranges,
                                                       const float* __restrict__ tfinal,
                                                       const int32_t* __restrict__ nlast,
                                                       const float* __restrict__ dimage, float* __restrict__ g2d,
                                                       uint32_t n_pairs, const uint64_t* __restrict__ hits,
                                                       uint64_t hit_stride, const uint32_t* __restrict__ order) {
  const uint32_t gid = block_id(order);
  const uint32_t frame = gid / gridDim.x;
  const FrameDesc& d = descs[frame];
  const FrameDesc& dl = descs[d.list_frame];   // owner of the key list this frame blended
  const int tile = (int)(gid % gridDim.x);
  if (tile >= d.tiles_x * d.tiles_y) return;
  const int tx = tile % d.tiles_x, ty = tile / d.tiles_x;
  const uint2 rg = ranges[dl.tile_base + tile];
  if (rg.y <= rg.x) return;
  const uint32_t roff = d.pair_base - dl.pair_base;   // list pair id -> this frame's pair id
  const bool shared = dl.n_share > 1;
  const uint64_t* fhits = kHits ? hits + (uint64_t)d.slot * hit_stride : nullptr;
  const int lane = threadIdx.x;
  const int qx = lane & 7, qy = lane >> 3;
  const float pxl0 = (float)qx + 0.5f, pxl1 = (float)(qx + 8) + 0.5f;
  const float pyl0 = (float)qy + 0.5f, pyl1 = (float)(qy + 8) + 0.5f;
  const size_t HW = (size_t)d.W * d.H;
  const float* tfp = tfinal + (size_t)frame * HW;
  const int32_t* nlp = nlast + (size_t)frame * HW;
  const float* dip = dimage + (size_t)frame * 3 * HW;

  __shared__ float4 s_geo[kBatch];   // mx, my, -q0, q1
  __shared__ float4 s_q[kBatch];     // q2, l2A, R, G
  __shared__ float4 s_con[kBatch];   // conic a, b, c, B
  __shared__ float2 s_pa[kBatch];    // pair id (bits), 1/A
  __shared__ int s_pos[kBatch];      // position of a staged entry in its batch
  __shared__ float s_acc[kBatch][9];

  // GS = g . S: the colour behind the current entry (S, background first) enters the adjoint
  // only through dL/dalpha = g . (rgb - S) with the pixel's fixed g = dL/dC, so the walk keeps
  // the scalar g . S instead of S: S <- S + alpha (rgb - S) becomes GS <- GS + alpha (g.rgb - GS).
  float T[4], GS[4], gr[4][3];
  int last[4];
  int jmax = -1;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int px = tx * kTile + qx + 8 * (r & 1), py = ty * kTile + qy + 8 * (r >> 1);
    const bool in = px < d.W && py < d.H;
    const size_t pi = (size_t)py * d.W + px;
    T[r] = in ? tfp[pi] : 1.0f;
    last[r] = in ? nlp[pi] : -1;
    gr[r][0] = in ? dip[pi] : 0.0f;
    gr[r][1] = in ? dip[HW + pi] : 0.0f;
    gr[r][2] = in ? dip[2 * HW + pi] : 0.0f;
    GS[r] = fmaf(gr[r][2], d.bg[2], fmaf(gr[r][1], d.bg[1], gr[r][0] * d.bg[0]));
    jmax = max(jmax, last[r]);
  }
  jmax = min(wave_max_i32(jmax), (int)rg.y - 1);   // n_last lies inside this tile's range
  if (jmax < (int)rg.x) return;
  const float l2min = o.log2_alpha_min;
  const float aclamp = o.alpha_clamp;
  const uint32_t aclamp_bits = __float_as_uint(aclamp);
  for (int c = 0; c < 9; ++c) s_acc[lane][c] = 0.0f;
  // lanes' share of a pair's reduction: which component of which entry, if any
  const int rj = lane & 15;
  const bool own = (rj & 3) == 0 || (rj == 2 && ((lane >> 4) & 1) == 0);
  const int comp = rj == 2 ? 8 : 2 * ((rj >> 3) + 2 * ((rj >> 2) & 1)) + ((lane >> 4) & 1);
  for (int hi = jmax + 1; hi > (int)rg.x; hi -= kBatch) {
    const int lo = max((int)rg.x, hi - kBatch);
    const int nb = hi - lo;
    const int j = lo + lane;
    // entries of this batch to visit: those the forward pass blended (hit bits), else all
    // that are live for this frame.  Only they are staged, packed to the front of the batch
    // in list order; s_pos keeps each one's position in the batch.
    uint64_t todo = ~0ull >> (64 - nb);
    if (kHits) {
      const uint32_t off = (uint32_t)lo - rg.x;
      const size_t w0 = hit_word(rg.x, dl.tile_base + tile, off >> 6);
      const uint32_t sh = off & 63u;
      uint64_t v = fhits[w0] >> sh;
      if (sh != 0 && sh + (uint32_t)nb > 64u) v |= fhits[w0 + 1] << (64u - sh);
      todo &= v;
    }
    bool mine = (todo >> lane) & 1ull;
    uint32_t p = 0u;
    float4 r0, r1, r2;
    if (mine) {
      p = vals[j] + roff;
      const float4* rp = rec + 3 * (size_t)p;
      r0 = rp[0];
      r1 = rp[1];
      r2 = rp[2];
      if (!kHits && shared) {   // the forward pass's live test for a frame on a shared list
        const uint32_t in = __float_as_uint(r2.w) >> kFrameBits;
        const uint32_t a = __float_as_uint(r2.y), b = __float_as_uint(r2.z);
        const int x0 = (int)((a & 0xffffu) + (in & 31u)), y0 = (int)((a >> 16) + ((in >> 5) & 31u));
        const int x1 = (int)((b & 0xffffu) - ((in >> 10) & 31u)), y1 = (int)((b >> 16) - ((in >> 15) & 31u));
        mine = r1.y > 0.0f && tx >= x0 && tx <= x1 && ty >= y0 && ty <= y1;
      }
    }
    todo = __ballot(mine);
    const int cnt = __popcll(todo);
    if (mine) {
      const int slot = __builtin_amdgcn_mbcnt_hi((uint32_t)(todo >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)todo, 0u));
      const Staged s = stage(r0, r1, r2, tx, ty);
      s_geo[slot] = make_float4(s.mx, s.my, -s.q0, s.q1);
      s_q[slot] = make_float4(s.q2, s.l2A, r1.z, r1.w);
      s_con[slot] = make_float4(r0.z, r0.w, r1.x, r2.x);
      // A = 0 marks an entry this frame's footprint culls (shared lists): never blended, and
      // its all-zero sums must not become 0 * inf in the flush
      s_pa[slot] = make_float2(__uint_as_float(p), r1.y > 0.0f ? 1.0f / r1.y : 0.0f);
      s_pos[slot] = lane;
    }
    __syncthreads();
    // adjoint of entry k of the staged batch for this lane's four pixels (updates T, S)
    // The first quadrant's body only yields the blend weight w and dL/dsigma (both zero
    // where the pixel does not blend); the entry's nine sums are then written from them for
    // every lane, which needs two zeros instead of nine before the branch.  The other
    // quadrants add inside their bodies.
    auto entry_adjoint = [&](const int k, float (&acc)[9], bool& contrib) {
      const int jj = lo + s_pos[k];
      const float4 g = s_geo[k];
      const float4 q = s_q[k];
      const float cbv = s_con[k].w;
      const float rgbv[3] = {q.z, q.w, cbv};
      const float dx0 = pxl0 - g.x, dx1 = pxl1 - g.x;
      const float eb0 = exponent_base_neg(g.z, q.y, dx0), eb1 = exponent_base_neg(g.z, q.y, dx1);
      const float q1dx0 = g.w * dx0, q1dx1 = g.w * dx1;
      const float dy0 = pyl0 - g.y, dy1 = pyl1 - g.y;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float dx = (r & 1) ? dx1 : dx0, dy = (r >> 1) ? dy1 : dy0;
        const float e = exponent((r & 1) ? eb1 : eb0, (r & 1) ? q1dx1 : q1dx0, q.x, dy);
        float w = 0.0f, dsig = 0.0f;
        if (jj <= last[r] && e >= l2min) {
          if (!kHits) contrib = true;
          const float a = __builtin_amdgcn_exp2f(e);
          const bool clamped = !(a < aclamp);
          const float alpha = __uint_as_float(min(__float_as_uint(a), aclamp_bits));   // a, aclamp > 0
          const float Tk = T[r] * __builtin_amdgcn_rcpf(1.0f - alpha);
          w = alpha * Tk;
          const float grgb = fmaf(gr[r][2], rgbv[2], fmaf(gr[r][1], rgbv[1], gr[r][0] * rgbv[0]));
          const float dalpha = grgb - GS[r];
          GS[r] = fmaf(alpha, dalpha, GS[r]);
          T[r] = Tk;
          // dL/dsigma = -dL/dalpha * a = -(dalpha Tk) a, and unclamped a Tk is w
          dsig = clamped ? 0.0f : -(dalpha * w);
          if (r > 0) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) acc[5 + ch] = fmaf(w, gr[r][ch], acc[5 + ch]);
            const float u = dsig * dx, v = dsig * dy;
            acc[0] += u;
            acc[1] += v;
            acc[2] = fmaf(u, dx, acc[2]);
            acc[3] = fmaf(u, dy, acc[3]);
            acc[4] = fmaf(v, dy, acc[4]);
            acc[8] += dsig;
          }
        }
        if (r == 0) {
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) acc[5 + ch] = w * gr[0][ch];
          const float u = dsig * dx, v = dsig * dy;
          acc[0] = u;
          acc[1] = v;
          acc[2] = u * dx;
          acc[3] = u * dy;
          acc[4] = v * dy;
          acc[8] = dsig;
        }
      }
    };
    // entries go in pairs (A, then the next lower B) so that one butterfly reduces both
    for (int ka = cnt - 1; ka >= 0; ka -= 2) {
      const bool has_b = ka > 0;
      const int kb = has_b ? ka - 1 : ka;
      // acc: 0 S_x, 1 S_y, 2 S_xx, 3 S_xy, 4 S_yy, 5 R, 6 G, 7 B, 8 S_d
      float acc_a[9], acc_b[9];
      bool con_a = false, con_b = false;
      entry_adjoint(ka, acc_a, con_a);
      if (has_b) {
        entry_adjoint(kb, acc_b, con_b);
      } else {
#pragma unroll
        for (int c = 0; c < 9; ++c) acc_b[c] = 0.0f;
      }
      // an entry with a hit bit is blended in some pixel of the tile (the backward's test is
      // the forward's), so only without hit bits can a pair contribute nothing
      if (!kHits && __ballot(con_a || con_b) == 0ull) continue;
      // every processed entry is reduced exactly once per tile, so the owning lanes store
      // its totals (no atomics); without a B entry lanes 32-63 carry zeros for A's slots
      const float wsum = wave_reduce_pair(acc_a, acc_b, lane);
      if (own && (lane < 32 || has_b)) s_acc[lane < 32 ? ka : kb][comp] = wsum;
    }
    __syncthreads();
    // flush.  Lane l first turns staged entry l's sums into screen-space gradients (in
    // place); then the cnt x 9 values go out in rounds of 64 over consecutive (entry,
    // component) slots, so the lanes of one atomic instruction cover about seven entries'
    // contiguous nine-float records (a few cache lines) instead of 64 scattered words.
    if (lane < cnt) {
      const float4 cn = s_con[lane];
      const float sx = s_acc[lane][0], sy = s_acc[lane][1];
      s_acc[lane][0] = -(cn.x * sx + cn.y * sy);
      s_acc[lane][1] = -(cn.y * sx + cn.z * sy);
      s_acc[lane][2] = 0.5f * s_acc[lane][2];
      s_acc[lane][4] = 0.5f * s_acc[lane][4];
      s_acc[lane][8] = -s_acc[lane][8] * s_pa[lane].y;
    }
    __syncthreads();
    float* flat = &s_acc[0][0];
#pragma unroll 1   // unrolled, the rounds' loads are hoisted and the kernel needs ~40 more VGPRs
    for (int t = 0; t * kBatch < 9 * cnt; ++t) {
      const int idx = t * kBatch + lane;
      const int e = idx / 9, c = idx - 9 * e;
      if (e < cnt) {
        const float v = flat[idx];
        flat[idx] = 0.0f;
        if (v != 0.0f) unsafeAtomicAdd(g2d + (size_t)__float_as_uint(s_pa[e].x) * 9 + c, v);
      }
    }
    __syncthreads();
  }
}

}  // namespace

namespace {

template <bool kShared>
void launch_fwd(dim3 grid, hipStream_t stream, const FrameDesc* descs, const KOpts& o, const float4* rec,
                const uint32_t* vals, const uint2* rg, float* image, float* tfinal, int32_t* nlast, int32_t* ncontrib,
                uint64_t* hits, uint64_t hit_stride, const uint32_t* keep_bits, const uint32_t* order,
                const L1Fuse& l1) {
  const dim3 block(64);
  if (ncontrib && hits)
    hipLaunchKernelGGL((blend_fwd_kernel<true, true, kShared>), grid, block, 0, stream, descs, o, rec, vals, rg, image,
                       tfinal, nlast, ncontrib, hits, hit_stride, keep_bits, order, l1);
  else if (ncontrib)
    hipLaunchKernelGGL((blend_fwd_kernel<true, false, kShared>), grid, block, 0, stream, descs, o, rec, vals, rg, image,
                       tfinal, nlast, ncontrib, hits, hit_stride, keep_bits, order, l1);
  else if (hits)
    hipLaunchKernelGGL((blend_fwd_kernel<false, true, kShared>), grid, block, 0, stream, descs, o, rec, vals, rg, image,
                       tfinal, nlast, ncontrib, hits, hit_stride, keep_bits, order, l1);
  else
    hipLaunchKernelGGL((blend_fwd_kernel<false, false, kShared>), grid, block, 0, stream, descs, o, rec, vals, rg,
                       image, tfinal, nlast, ncontrib, hits, hit_stride, keep_bits, order, l1);
}

// Longest-list-first order of the n_frames x max_tiles blocks in ws[kOrderHeader ..], or
// nullptr (natural order) when ws cannot hold it.
const uint32_t* dispatch_order(const FrameDesc* descs, int n_frames, int max_tiles, const uint2* rg, uint32_t* ws,
                               uint64_t ws_words, hipStream_t stream) {
  const uint64_t n = (uint64_t)n_frames * (uint64_t)max_tiles;
  if (!ws || n >= 0x80000000ull || ws_words < n + kOrderHeader) return nullptr;
  if (launch_fill_u32(ws, 2 * kOrderBuckets, 0u, stream) != hipSuccess) return nullptr;
  const dim3 grid((uint32_t)((n + 255) / 256));
  hipLaunchKernelGGL(order_count_kernel, grid, dim3(256), 0, stream, descs, rg, (uint32_t)n, (uint32_t)max_tiles,
                     ws);
  hipLaunchKernelGGL(order_scatter_kernel, grid, dim3(256), 0, stream, descs, rg, (uint32_t)n,
                     (uint32_t)max_tiles, ws, ws + kOrderHeader);
  return ws + kOrderHeader;
}

}  // namespace

hipError_t launch_blend_fwd(
const FrameDesc* descs, int n_frames, int per_view, int max_tiles, const KOpts& o,
                            const float4* rec, const uint32_t* vals, const uint32_t* ranges, float* image,
                            float* tfinal, int32_t* nlast, int32_t* ncontrib, uint64_t* hits, uint64_t hit_stride,
                            const uint32_t* keep_bits, uint32_t* order_ws, uint64_t order_ws_words,
                            hipStream_t stream, const L1Fuse& l1) {
  if (n_frames <= 0 || max_tiles <= 0) return hipSuccess;
  if (per_view < 1 || n_frames % per_view != 0) return hipErrorInvalidValue;
  const dim3 grid(max_tiles, n_frames);
  const uint2* rg = (const uint2*)ranges;
  const uint32_t* order = dispatch_order(descs, n_frames, max_tiles, rg, order_ws, order_ws_words, stream);
  // The keep bits cost a third dependent load per entry; they pay off only when most of a
  // shared list is dead for each frame, i.e. with many tables per view (measured: 3 random
  // tables per view lose 6% of the forward pass with them, 10 narrow tent maps gain 15%).
  if (per_view > 1)
    launch_fwd<true>(grid, stream, descs, o, rec, vals, rg, image, tfinal, nlast, ncontrib, hits, hit_stride,
                     per_view >= kKeepBitsMinFrames ? keep_bits : nullptr, order, l1);
  else
    launch_fwd<false>(grid, stream, descs, o, rec, vals, rg, image, tfinal, nlast, ncontrib, hits, hit_stride,
                      nullptr, order, l1);
  return hipGetLastError();
}

hipError_t launch_blend_bwd(const FrameDesc* descs, int n_frames, int max_tiles, const KOpts& o, const float4* rec,
                            const uint32_t* vals, const uint32_t* ranges, const float* tfinal, const int32_t* nlast,
                            const float* dimage, float* g2d, uint32_t n_pairs, const uint64_t* hits,
                            uint64_t hit_stride, uint32_t* order_ws, uint64_t order_ws_words,
                            hipStream_t stream) {
  if (n_frames <= 0 || max_tiles <= 0) return hipSuccess;
  const uint2* rg = (const uint2*)ranges;
  const uint32_t* order = dispatch_order(descs, n_frames, max_tiles, rg, order_ws, order_ws_words, stream);
  if (hits)
    hipLaunchKernelGGL(blend_bwd_kernel<true>, dim3(max_tiles, n_frames), dim3(64), 0, stream, descs, o, rec, vals,
                       rg, tfinal, nlast, dimage, g2d, n_pairs, hits, hit_stride, order);
  else
    hipLaunchKernelGGL(blend_bwd_kernel<false>, dim3(max_tiles, n_frames), dim3(64), 0, stream, descs, o, rec, vals,
                       rg, tfinal, nlast, dimage, g2d, n_pairs, hits, hit_stride, order);
  return hipGetLastError();
}

}  // namespace veg
