// Training-loop neighbours of the renderer (paper, section "Training"): the SSIM term of
// the image loss (1 - lambda) L1 + lambda SSIM, the Adam update of the parameters, and the
// per-Gaussian statistics that drive densification.
#include "veg_internal.h"

#include <cmath>

#pragma clang fp contract(off)

namespace veg {
namespace {

// SSIM window: 11 taps, Gaussian with sigma 1.5, normalised (the 2D window is the outer
// product, so both passes use the same taps).  Constants for a data range of 1.
constexpr int kWin = 11, kHalf = 5;
constexpr float kC1 = 0.0001f, kC2 = 0.0009f;
// A block produces a 32 x 32 output tile from a 42 x 42 input tile (5-pixel halo, zeros
// outside the image) staged in LDS.  Horizontal pass: each thread turns 14 staged values of
// a row into 4 outputs; vertical pass: each thread turns 14 values of a column into 4
// outputs.  Register blocking cuts LDS reads to about 27 per pixel and quantity set.
constexpr int kT = 32, kIn = kT + 2 * kHalf, kB = 4;
constexpr int kPadIn = kIn + 1, kPadT = kT + 1;   // odd row strides: no bank conflicts

struct Win {
  float w[kWin];
};

// Symmetric 11-tap window over v[c .. c + 10] (output at the centre c + 5).
__device__ __forceinline__ float win11(const float* v, const Win& w) {
  float a = w.w[kHalf] * v[kHalf];
#pragma unroll
  for (int t = 1; t <= kHalf; ++t) a = fmaf(w.w[kHalf - t], v[kHalf - t] + v[kHalf + t], a);
  return a;
}

// Input tile of one plane with zeros outside the image, in two steps so that a block can
// have the next tile's loads in flight while it works on the current one: fetch (global ->
// registers) and put (registers -> LDS).  When rows are 16-byte aligned (W a multiple of 4
// and an aligned plane; x0 is a multiple of 32) each tile row is read as 12 aligned float4
// covering columns x0 - 8 .. x0 + 39, of which the 42 in x0 - 5 .. x0 + 36 are kept; a
// float4 then lies wholly inside or wholly outside the image (2 float4 per thread).  Else
// the 42 x 42 values are read one by one (7 per thread).
constexpr int kVec = 12;
struct Fetch {
  float v[8];
};

template <bool kAligned>
__device__ __forceinline__ void fetch_tile(const float* __restrict__ src, int W, int H, int x0, int y0, Fetch& f) {
  if (kAligned) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int k = threadIdx.x + 256 * j;
      const int ly = k / kVec, c = k - ly * kVec;
      const int gy = y0 - kHalf + ly, gx = x0 - 8 + 4 * c;
      float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (k < kIn * kVec && gy >= 0 && gy < H && gx >= 0 && gx < W)
        v = *reinterpret_cast<const float4*>(src + (size_t)gy * W + gx);
      f.v[4 * j + 0] = v.x;
      f.v[4 * j + 1] = v.y;
      f.v[4 * j + 2] = v.z;
      f.v[4 * j + 3] = v.w;
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    const int k = threadIdx.x + 256 * j;
    const int ly = k / kIn, lx = k - ly * kIn;
    const int gx = x0 - kHalf + lx, gy = y0 - kHalf + ly;
    f.v[j] = (k < kIn * kIn && gx >= 0 && gx < W && gy >= 0 && gy < H) ? src[(size_t)gy * W + gx] : 0.0f;
  }
}

template <bool kAligned>
__device__ __forceinline__ void put_tile(const Fetch& f, float (*dst)[kPadIn]) {
  if (kAligned) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int k = threadIdx.x + 256 * j;
      if (k >= kIn * kVec) continue;
      const int ly = k / kVec, c = k - ly * kVec;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int lx = 4 * c + i - 3;
        if (lx >= 0 && lx < kIn) dst[ly][lx] = f.v[4 * j + i];
      }
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    const int k = threadIdx.x + 256 * j;
    if (k < kIn * kIn) dst[k / kIn][k % kIn] = f.v[j];
  }
}


// Tiles along x per block: each block walks kTilesX output tiles of one row of tiles,
// fetching the next tile's inputs before it runs the current tile's window passes.
constexpr int kTilesX = 4;

// Per tile: windowed means of x, y, x^2, y^2, x y, the SSIM map S and its partial
// derivatives with respect to mu_x, E[x^2] and E[x y] at every pixel:
//   N = (2 mu_x mu_y + C1)(2 s_xy + C2) = A1 A2,  D = (mu_x^2 + mu_y^2 + C1)(s_x + s_y + C2) = B1 B2,
//   dS/dmu_x = (2 mu_y (A2 - A1) - 2 mu_x S (B2 - B1)) / D,  dS/dE[x^2] = -S B1 / D,
//   dS/dE[xy] = 2 A1 / D.
// The three maps are stored multiplied by dL/dS = -weight for the backward pass.  With kL1
// the L1 term l1_scale * sum |x - y| over the tile's own pixels joins the loss.
template <bool kL1, bool kAligned>
__global__ __launch_bounds__(256) void ssim_fwd_kernel(const float* __restrict__ img, const float* __restrict__ tgt,
                                                       int W, int H, float weight, float l1_scale,
                                                       double* __restrict__ loss, float* __restrict__ dmaps,
                                                       size_t plane_stride, Win win) {
  __shared__ float s_x[kIn][kPadIn], s_y[kIn][kPadIn];
  __shared__ float s_h[5][kIn][kPadT];
  __shared__ double s_part[2][4];
  const int y0 = blockIdx.y * kT;
  const size_t plane = blockIdx.z;
  const size_t HW = (size_t)W * H;
  const float* ip = img + plane * HW;
  const float* tp = tgt + plane * HW;
  Fetch fx, fy;
  int x0 = blockIdx.x * kTilesX * kT;
  fetch_tile<kAligned>(ip, W, H, x0, y0, fx);
  fetch_tile<kAligned>(tp, W, H, x0, y0, fy);
  double part = 0.0, part_l1 = 0.0;
  for (int t = 0; t < kTilesX && x0 < W; ++t, x0 += kT) {
    put_tile<kAligned>(fx, s_x);
    put_tile<kAligned>(fy, s_y);
    __syncthreads();
    if (t + 1 < kTilesX && x0 + kT < W) {   // the next tile's loads overlap this tile's passes
      fetch_tile<kAligned>(ip, W, H, x0 + kT, y0, fx);
      fetch_tile<kAligned>(tp, W, H, x0 + kT, y0, fy);
    }
    // horizontal: 42 rows x 8 groups of 4 columns
    for (int task = threadIdx.x; task < kIn * (kT / kB); task += blockDim.x) {
      const int r = task / (kT / kB), c0 = (task - r * (kT / kB)) * kB;
      float p[5][kB + 2 * kHalf];
#pragma unroll
      for (int i = 0; i < kB + 2 * kHalf; ++i) {
        const float xv = s_x[r][c0 + i], yv = s_y[r][c0 + i];
        p[0][i] = xv;
        p[1][i] = yv;
        p[2][i] = xv * xv;
        p[3][i] = yv * yv;
        p[4][i] = xv * yv;
      }
#pragma unroll
      for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int i = 0; i < kB; ++i) s_h[q][r][c0 + i] = win11(&p[q][i], win);
    }
    __syncthreads();
    // vertical: 32 columns x 8 groups of 4 rows, one task per thread
    {
      const int c = threadIdx.x & (kT - 1), r0 = (threadIdx.x / kT) * kB;
      float m[5][kB];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        float v[kB + 2 * kHalf];
#pragma unroll
        for (int i = 0; i < kB + 2 * kHalf; ++i) v[i] = s_h[q][r0 + i][c];
#pragma unroll
        for (int i = 0; i < kB; ++i) m[q][i] = win11(&v[i], win);
      }
      const int gx = x0 + c;
#pragma unroll
      for (int i = 0; i < kB; ++i) {
        const int gy = y0 + r0 + i;
        if (gx >= W || gy >= H) continue;
        const float mx = m[0][i], my = m[1][i];
        const float sx = m[2][i] - mx * mx, sy = m[3][i] - my * my, sxy = m[4][i] - mx * my;
        const float A1 = 2.0f * mx * my + kC1, A2 = 2.0f * sxy + kC2;
        const float B1 = mx * mx + my * my + kC1, B2 = sx + sy + kC2;
        const float D = B1 * B2;
        const float S = (A1 * A2) / D;
        part += (double)(1.0f - S);
        if (kL1) part_l1 += (double)fabsf(s_x[r0 + i + kHalf][c + kHalf] - s_y[r0 + i + kHalf][c + kHalf]);
        // one reciprocal for the three maps (S keeps its division: identical images give
        // S = 1 exactly, and then dex2 = -(B1 rD) and dexy = 2 (B1 rD) cancel in the adjoint)
        const float rD = 1.0f / D;
        const float dmu = (2.0f * my * (A2 - A1) - 2.0f * mx * S * (B2 - B1)) * rD;
        const float dex2 = -S * B1 * rD;
        const float dexy = 2.0f * A1 * rD;
        const size_t pi = plane * HW + (size_t)gy * W + gx;
        dmaps[pi] = -weight * dmu;
        dmaps[plane_stride + pi] = -weight * dex2;
        dmaps[2 * plane_stride + pi] = -weight * dexy;
      }
    }
    __syncthreads();   // s_x, s_y and s_h are rewritten for the next tile
  }
  for (int off = 32; off > 0; off >>= 1) {
    part += __shfl_xor(part, off);
    if (kL1) part_l1 += __shfl_xor(part_l1, off);
  }
  if ((threadIdx.x & 63) == 0) {
    s_part[0][threadIdx.x >> 6] = part;
    s_part[1][threadIdx.x >> 6] = part_l1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = (s_part[0][0] + s_part[0][1]) + (s_part[0][2] + s_part[0][3]);
    double add = t * (double)weight;
    if (kL1) add += ((s_part[1][0] + s_part[1][1]) + (s_part[1][2] + s_part[1][3])) * (double)l1_scale;
    if (add != 0.0) unsafeAtomicAdd(loss, add);
  }
}

// Adjoint: dL/dx = G * D_mu + 2 x (G * D_x2) + y (G * D_xy), the window applied to the maps
// with zeros outside the image (the adjoint of the zero-padded forward window); added to
// d_image.  With kL1, d_image is not read: it is written as the L1 term's gradient
// l1_scale * sign(x - y) plus that sum, the same value, rounding included, as the L1 pass
// followed by the SSIM pass.
template <bool kL1, bool kAligned>
__global__ __launch_bounds__(256) void ssim_bwd_kernel(const float* __restrict__ img, const float* __restrict__ tgt,
                                                       int W, int H, const float* __restrict__ dmaps,
                                                       size_t plane_stride, float* __restrict__ dimg, float l1_scale,
                                                       Win win) {
  __shared__ float s_m[3][kIn][kPadIn];
  __shared__ float s_h[3][kIn][kPadT];
  const int y0 = blockIdx.y * kT;
  const size_t plane = blockIdx.z;
  const size_t HW = (size_t)W * H;
  const float* mp = dmaps + plane * HW;
  Fetch fm[3];
  int x0 = blockIdx.x * kTilesX * kT;
#pragma unroll
  for (int q = 0; q < 3; ++q) fetch_tile<kAligned>(mp + q * plane_stride, W, H, x0, y0, fm[q]);
  const int c = threadIdx.x & (kT - 1), r0 = (threadIdx.x / kT) * kB;
  for (int t = 0; t < kTilesX && x0 < W; ++t, x0 += kT) {
#pragma unroll
    for (int q = 0; q < 3; ++q) put_tile<kAligned>(fm[q], s_m[q]);
    __syncthreads();
    if (t + 1 < kTilesX && x0 + kT < W) {
#pragma unroll
      for (int q = 0; q < 3; ++q) fetch_tile<kAligned>(mp + q * plane_stride, W, H, x0 + kT, y0, fm[q]);
    }
    // this tile's own pixels of image and target, read ahead of the window passes
    const int gx = x0 + c;
    float xi[kB], yi[kB];
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      const int gy = y0 + r0 + i;
      const bool in = gx < W && gy < H;
      const size_t pi = plane * HW + (size_t)gy * W + gx;
      xi[i] = in ? img[pi] : 0.0f;
      yi[i] = in ? tgt[pi] : 0.0f;
    }
    for (int task = threadIdx.x; task < kIn * (kT / kB); task += blockDim.x) {
      const int r = task / (kT / kB), c0 = (task - r * (kT / kB)) * kB;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        float v[kB + 2 * kHalf];
#pragma unroll
        for (int i = 0; i < kB + 2 * kHalf; ++i) v[i] = s_m[q][r][c0 + i];
#pragma unroll
        for (int i = 0; i < kB; ++i) s_h[q][r][c0 + i] = win11(&v[i], win);
      }
    }
    __syncthreads();
    float m[3][kB];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      float v[kB + 2 * kHalf];
#pragma unroll
      for (int i = 0; i < kB + 2 * kHalf; ++i) v[i] = s_h[q][r0 + i][c];
#pragma unroll
      for (int i = 0; i < kB; ++i) m[q][i] = win11(&v[i], win);
    }
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      const int gy = y0 + r0 + i;
      if (gx >= W || gy >= H) continue;
      const size_t pi = plane * HW + (size_t)gy * W + gx;
      const float x = xi[i], y = yi[i];
      const float g = (m[0][i] + 2.0f * x * m[1][i]) + y * m[2][i];
      if (kL1) {
        const float d = x - y;
        dimg[pi] = (d > 0.0f ? l1_scale : (d < 0.0f ? -l1_scale : 0.0f)) + g;
      } else {
        dimg[pi] += g;
      }
    }
    __syncthreads();   // s_m and s_h are rewritten for the next tile
  }
}

// Adam (Kingma & Ba): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
// p <- p - lr (m / bc1) / (sqrt(v / bc2) + eps) with bc = 1 - beta^t from the host.
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                                                   float b1, float b2, float eps, float bc1, float bc2) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

// Densification statistics: for every Gaussian, over the frames in which it was kept, the
// norm of the gradient w.r.t. its projected centre and the count of such frames (added).
// Kept in a frame: its list holds the Gaussian (count of the list owner's pair) and, for a
// frame on a list shared by several frames, the frame's own footprint keeps it: the view's
// keep bits (bit = the frame's slot, in the depth slots of the view's second frame) tell,
// for slots from 31 on the record's A > 0 does.  A frame owning its list alone keeps every
// counted pair.
__global__ __launch_bounds__(256) void densify_stats_kernel(const FrameDesc* __restrict__ descs, int n_frames, int n,
                                                            const uint32_t* __restrict__ count,
                                                            const uint32_t* __restrict__ depth,
                                                            const float4* __restrict__ rec,
                                                            const float* __restrict__ g2d, float* __restrict__ acc,
                                                            int32_t* __restrict__ vis) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float a = 0.0f;
  int c = 0;
  for (int f = 0; f < n_frames; ++f) {
    const FrameDesc& d = descs[f];
    const FrameDesc& dl = descs[d.list_frame];
    const size_t pid = (size_t)d.pair_base + (size_t)i;
    if (count[(size_t)dl.pair_base + (size_t)i] == 0u) continue;
    if (dl.n_share > 1) {
      if (d.slot < 31) {
        if (!((depth[(size_t)descs[d.list_frame + 1].pair_base + (size_t)i] >> d.slot) & 1u)) continue;
      } else if (!(rec[3 * pid + 1].y > 0.0f)) {
        continue;
      }
    }
    const float gx = g2d[pid * 9 + 0], gy = g2d[pid * 9 + 1];
    a += sqrtf(gx * gx + gy * gy);
    ++c;
  }
  acc[i] += a;
  vis[i] += c;
}

// Adaptive density control.  Decision per Gaussian (float32 comparisons): g = accum / vis
// (0 where vis = 0); PRUNE unless weight >= prune_weight; else SPLIT when g >= grad_thresh
// and the largest log-scale exceeds log_scale_thresh, CLONE when g >= grad_thresh otherwise;
// else KEEP.  Each block of 256 Gaussians also counts its survivors (KEEP, CLONE), clones
// and splits: blk[3 b + 0..2].
constexpr int kDensifyBlock = 256;

__device__ __forceinline__ int wave_excl_count(bool v, uint64_t& m) {
  m = __ballot(v);
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Exclusive position of this thread among the block's threads with v set, and the total.
__device__ __forceinline__ uint32_t block_excl_count(bool v, uint32_t* s_w, uint32_t& total) {
  uint64_t m;
  const int in_wave = wave_excl_count(v, m);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) s_w[w] = (uint32_t)__popcll(m);
  __syncthreads();
  uint32_t before = 0;
  total = 0;
  for (int k = 0; k < kDensifyBlock / 64; ++k) {
    if (k < w) before += s_w[k];
    total += s_w[k];
  }
  __syncthreads();
  return before + (uint32_t)in_wave;
}

__global__ __launch_bounds__(kDensifyBlock) void densify_plan_kernel(
    int64_t n, const float* __restrict__ acc, const int32_t* __restrict__ vis, const float* __restrict__ log_scales,
    const float* __restrict__ weights, float grad_thresh, float log_scale_thresh, float prune_weight,
    uint8_t* __restrict__ action, uint32_t* __restrict__ blk) {
  __shared__ uint32_t s_w[kDensifyBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * kDensifyBlock + threadIdx.x;
  uint8_t a = 0xff;   // past the end
  if (i < n) {
    const int32_t c = vis[i];
    const float g = c > 0 ? acc[i] / (float)c : 0.0f;
    const float* ls = log_scales + 3 * i;
    const bool big = fmaxf(fmaxf(ls[0], ls[1]), ls[2]) > log_scale_thresh;
    a = g >= grad_thresh ? (big ? 2 : 1) : 0;
    if (weights && !(weights[i] >= prune_weight)) a = 3;
    action[i] = a;
  }
  uint32_t ts, tc, tp;
  block_excl_count(a == 0 || a == 1, s_w, ts);
  block_excl_count(a == 1, s_w, tc);
  block_excl_count(a == 2, s_w, tp);
  if (threadIdx.x == 0) {
    blk[3 * blockIdx.x + 0] = ts;
    blk[3 * blockIdx.x + 1] = tc;
    blk[3 * blockIdx.x + 2] = tp;
  }
}

// Exclusive scan of the per-block counts (one block; blk rewritten in place), totals in
// tot[0..2] (survivors, clones, splits).
__global__ __launch_bounds__(1024) void densify_scan_kernel(uint32_t* __restrict__ blk, int G,
                                                            uint32_t* __restrict__ tot) {
  __shared__ uint32_t s_sum[3][1024];
  const int per = (G + 1023) / 1024;
  const int b0 = threadIdx.x * per, b1 = min(G, b0 + per);
  uint32_t loc[3] = {0, 0, 0};
  for (int b = b0; b < b1; ++b)
    for (int q = 0; q < 3; ++q) loc[q] += blk[3 * b + q];
  for (int q = 0; q < 3; ++q) s_sum[q][threadIdx.x] = loc[q];
  __syncthreads();
  if (threadIdx.x < 3) {   // serial scan of 1024 partial sums per stream
    uint32_t run = 0;
    for (int k = 0; k < 1024; ++k) {
      const uint32_t v = s_sum[threadIdx.x][k];
      s_sum[threadIdx.x][k] = run;
      run += v;
    }
    tot[threadIdx.x] = run;
  }
  __syncthreads();
  uint32_t run[3] = {s_sum[0][threadIdx.x], s_sum[1][threadIdx.x], s_sum[2][threadIdx.x]};
  for (int b = b0; b < b1; ++b)
    for (int q = 0; q < 3; ++q) {
      const uint32_t v = blk[3 * b + q];
      blk[3 * b + q] = run[q];
      run[q] += v;
    }
}

// The new model: survivors in order, then a copy of every clone in order, then two children
// of every split in order; child c of parent i at mu_i + R(q_i) diag(exp(log_s_i)) z[i, c],
// with log-scales log_s_i - ln 1.6.
__global__ __launch_bounds__(kDensifyBlock) void densify_apply_kernel(
    int64_t n, const uint8_t* __restrict__ action, const float* __restrict__ quats,
    const float* __restrict__ log_scales, const float* __restrict__ z, const uint32_t* __restrict__ blk,
    const uint32_t* __restrict__ tot, DensifyFields fl) {
  __shared__ uint32_t s_w[kDensifyBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * kDensifyBlock + threadIdx.x;
  const uint8_t a = i < n ? action[i] : (uint8_t)0xff;
  uint32_t ts, tc, tp;
  const uint32_t ps = block_excl_count(a == 0 || a == 1, s_w, ts);
  const uint32_t pc = block_excl_count(a == 1, s_w, tc);
  const uint32_t pp = block_excl_count(a == 2, s_w, tp);
  if (i >= n || a == 3) return;
  const size_t n_surv = tot[0], n_clone = tot[1];
  const size_t surv = (size_t)blk[3 * blockIdx.x + 0] + ps;
  const size_t clone = n_surv + (size_t)blk[3 * blockIdx.x + 1] + pc;
  const size_t child = n_surv + n_clone + 2 * ((size_t)blk[3 * blockIdx.x + 2] + pp);
  float off[2][3] = {{0, 0, 0}, {0, 0, 0}};
  if (a == 2) {
    const float* q = quats + 4 * i;
    const float qn = 1.0f / sqrtf(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
    const float w = q[0] * qn, x = q[1] * qn, y = q[2] * qn, zq = q[3] * qn;
    const float R[9] = {1.0f - 2.0f * (y * y + zq * zq), 2.0f * (x * y - w * zq), 2.0f * (x * zq + w * y),
                        2.0f * (x * y + w * zq), 1.0f - 2.0f * (x * x + zq * zq), 2.0f * (y * zq - w * x),
                        2.0f * (x * zq - w * y), 2.0f * (y * zq + w * x), 1.0f - 2.0f * (x * x + y * y)};
    const float* ls = log_scales + 3 * i;
    const float sc[3] = {expf(ls[0]), expf(ls[1]), expf(ls[2])};
    for (int c = 0; c < 2; ++c) {
      const float* zc = z + 6 * i + 3 * c;
      for (int r = 0; r < 3; ++r)
        off[c][r] = (R[3 * r + 0] * (sc[0] * zc[0]) + R[3 * r + 1] * (sc[1] * zc[1])) + R[3 * r + 2] * (sc[2] * zc[2]);
    }
  }
  for (int f = 0; f < fl.n_fields; ++f) {
    const int wd = fl.width[f], role = fl.role[f];
    const float* src = fl.src[f] + (size_t)i * wd;
    float* dst = fl.dst[f];
    if (a != 2) {
      for (int k = 0; k < wd; ++k) dst[surv * wd + k] = src[k];
      if (a == 1)
        for (int k = 0; k < wd; ++k) dst[clone * wd + k] = role == 3 ? 0.0f : src[k];
    } else {
      for (int c = 0; c < 2; ++c)
        for (int k = 0; k < wd; ++k) {
          float v = src[k];
          if (role == 1 && k < 3) v = src[k] + off[c][k];
          else if (role == 2) v = src[k] - 0.47000362924573558f;   // ln 1.6
          else if (role == 3) v = 0.0f;
          dst[(child + c) * wd + k] = v;
        }
    }
  }
}

}  // namespace

// The window taps: exp(-x^2 / (2 sigma^2)) at x = -5..5, sigma 1.5, divided by their sum.
static Win ssim_window() {
  Win w;
  double s = 0.0, g[kWin];
  for (int t = 0; t < kWin; ++t) {
    const double x = (double)(t - kHalf);
    g[t] = std::exp(-(x * x) / (2.0 * 1.5 * 1.5));
    s += g[t];
  }
  for (int t = 0; t < kWin; ++t) w.w[t] = (float)(g[t] / s);
  return w;
}

template <bool kL1, bool kAligned>
static void ssim_pair(dim3 grid, hipStream_t stream, const float* image, const float* target, int W, int H,
                      float weight, float l1_scale, double* loss, float* d_image, float* dmaps, size_t plane_stride,
                      const Win& win) {
  hipLaunchKernelGGL((ssim_fwd_kernel<kL1, kAligned>), grid, dim3(256), 0, stream, image, target, W, H, weight,
                     l1_scale, loss, dmaps, plane_stride, win);
  hipLaunchKernelGGL((ssim_bwd_kernel<kL1, kAligned>), grid, dim3(256), 0, stream, image, target, W, H, dmaps,
                     plane_stride, d_image, l1_scale, win);
}

hipError_t launch_ssim(const float* image, const float* target, int64_t n_planes, int W, int H, float weight,
                       double* loss, float* d_image, float* dmaps, hipStream_t stream, bool with_l1,
                       float l1_scale) {
  if (n_planes <= 0 || W <= 0 || H <= 0) return hipSuccess;
  const size_t plane_stride = (size_t)n_planes * W * H;
  const int tiles_x = (W + kT - 1) / kT;
  const dim3 grid((tiles_x + kTilesX - 1) / kTilesX, (H + kT - 1) / kT, (unsigned)n_planes);
  const Win win = ssim_window();
  // rows of 16-byte aligned float4 in every plane of the image, the target and the maps
  const bool aligned = (W & 3) == 0 && ((reinterpret_cast<uintptr_t>(image) | reinterpret_cast<uintptr_t>(target) |
                                         reinterpret_cast<uintptr_t>(dmaps)) & 15u) == 0;
  if (with_l1) {
    if (aligned) ssim_pair<true, true>(grid, stream, image, target, W, H, weight, l1_scale, loss, d_image, dmaps,
                                       plane_stride, win);
    else ssim_pair<true, false>(grid, stream, image, target, W, H, weight, l1_scale, loss, d_image, dmaps,
                                plane_stride, win);
  } else {
    if (aligned) ssim_pair<false, true>(grid, stream, image, target, W, H, weight, 0.0f, loss, d_image, dmaps,
                                        plane_stride, win);
    else ssim_pair<false, false>(grid, stream, image, target, W, H, weight, 0.0f, loss, d_image, dmaps,
                                 plane_stride, win);
  }
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, g, m, v, n, lr, b1, b2, eps, bc1,
                     bc2);
  return hipGetLastError();
}

hipError_t launch_densify_plan(int64_t n, const float* acc, const int32_t* vis, const float* log_scales,
                               const float* weights, float grad_thresh, float log_scale_thresh, float prune_weight,
                               uint8_t* action, uint32_t* blk, uint32_t* tot, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int G = (int)((n + kDensifyBlock - 1) / kDensifyBlock);
  hipLaunchKernelGGL(densify_plan_kernel, dim3(G), dim3(kDensifyBlock), 0, stream, n, acc, vis, log_scales, weights,
                     grad_thresh, log_scale_thresh, prune_weight, action, blk);
  hipLaunchKernelGGL(densify_scan_kernel, dim3(1), dim3(1024), 0, stream, blk, G, tot);
  return hipGetLastError();
}

hipError_t launch_densify_apply(int64_t n, const uint8_t* action, const float* quats, const float* log_scales,
                                const float* z, const uint32_t* blk, const uint32_t* tot, const DensifyFields& fl,
                                hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int G = (int)((n + kDensifyBlock - 1) / kDensifyBlock);
  hipLaunchKernelGGL(densify_apply_kernel, dim3(G), dim3(kDensifyBlock), 0, stream, n, action, quats, log_scales, z,
                     blk, tot, fl);
  return hipGetLastError();
}

hipError_t launch_densify_stats(const FrameDesc* descs, int n_frames, int n, const uint32_t* count,
                                const uint32_t* depth, const float4* rec, const float* g2d, float* acc, int32_t* vis,
                                hipStream_t stream) {
  if (n <= 0 || n_frames <= 0) return hipSuccess;
  hipLaunchKernelGGL(densify_stats_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, descs, n_frames, n, count,
                     depth, rec, g2d, acc, vis);
  return hipGetLastError();
}

}  // namespace veg
