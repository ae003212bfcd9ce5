// Projection (transfer function first, EWA projection, footprint) and its adjoint.
//
// Paper, section "Rendering of VEGs": the transfer function maps each Gaussian's scalar to
// colour and opacity before rasterizing (alpha = O(v) w), so low-opacity Gaussians are culled
// at once; the 3D covariance from S and R is projected to a 2D screen covariance with
// Zwicker's EWA method.  Gradients reach position, scaling, rotation, scalar and weight.
//
// The whole file is compiled without floating-point contraction so that the footprint (cull,
// depth key, tile rectangle) follows the documented operation order bit for bit.
#include "veg_device.h"

#pragma clang fp contract(off)

namespace veg {
namespace {

// float32 exp: Cody & Waite reduction x = k ln2 + r (ln2 split in a short high part and a
// correction), exp(r) by the Taylor series to r^7 in Horner form, scaled by 2^k exactly.
// x >= 88 gives +inf, x < -87 gives 0.
__device__ __forceinline__ float exp32(float x) {
  const float kLog2e = 0x1.715476p+0f;
  const float kLn2Hi = 0.693359375f;
  const float kLn2Lo = -0x1.bd0106p-13f;
  const float k = floorf(x * kLog2e + 0.5f);
  const float r = (x - k * kLn2Hi) - k * kLn2Lo;
  float p = 1.0f / 5040.0f;
  p = p * r + 1.0f / 720.0f;
  p = p * r + 1.0f / 120.0f;
  p = p * r + 1.0f / 24.0f;
  p = p * r + 1.0f / 6.0f;
  p = p * r + 1.0f / 2.0f;
  p = p * r + 1.0f;
  p = p * r + 1.0f;
  const int ki = (int)fminf(fmaxf(k, -126.0f), 127.0f);
  float out = p * __uint_as_float((uint32_t)(ki + 127) << 23);
  if (x >= 88.0f) out = __builtin_inff();
  if (x < -87.0f) out = 0.0f;
  return out;
}

// float32 log for positive normal x: x = m 2^e with m in [sqrt(1/2), sqrt(2)),
// log m = 2 atanh(u), u = (m-1)/(m+1), odd series to u^9 (Horner in u^2),
// log x = e ln2_hi + (e ln2_lo + log m).
__device__ __forceinline__ float log32(float x) {
  const float kLn2Hi = 0.693359375f;
  const float kLn2Lo = -0x1.bd0106p-13f;
  const float kSqrt2 = 0x1.6a09e6p+0f;
  const uint32_t bits = __float_as_uint(x);
  int e = (int)(bits >> 23) - 127;
  float m = __uint_as_float((bits & 0x7fffffu) | 0x3f800000u);
  if (m > kSqrt2) {
    m = m * 0.5f;
    e += 1;
  }
  const float u = (m - 1.0f) / (m + 1.0f);
  const float u2 = u * u;
  float p = 1.0f / 9.0f;
  p = p * u2 + 1.0f / 7.0f;
  p = p * u2 + 1.0f / 5.0f;
  p = p * u2 + 1.0f / 3.0f;
  const float s = p * u2;
  const float t = u + u * s;
  const float logm = t + t;
  const float ef = (float)e;
  return ef * kLn2Hi + (ef * kLn2Lo + logm);
}

__device__ __forceinline__ bool finite3(const float* p) {
  return __builtin_isfinite(p[0]) && __builtin_isfinite(p[1]) && __builtin_isfinite(p[2]);
}

// Frame-independent per-Gaussian state.
struct GParams {
  float mu[3];
  float ls[3];
  float q[4];
  float v, w;
  bool finite;
  float n2, inv;       // |q|^2, 1/|q|
  float qh[4];         // normalised quaternion
  float R[9];          // rotation, row-major
  float s[3];          // scales
  bool lit;            // lighting attributes present
  float nn2, ninv;     // |n|^2, 1/|n|
  float nh[3];         // normalised normal
  float ka, kd, ks, beta;
};

__device__ __forceinline__ void load_params(const FrameDesc& d, int i, GParams& g) {
  const float* m = d.means + 3 * (size_t)i;
  const float* l = d.log_scales + 3 * (size_t)i;
  const float4 qq = *reinterpret_cast<const float4*>(d.quats + 4 * (size_t)i);
  g.mu[0] = m[0]; g.mu[1] = m[1]; g.mu[2] = m[2];
  g.ls[0] = l[0]; g.ls[1] = l[1]; g.ls[2] = l[2];
  g.q[0] = qq.x; g.q[1] = qq.y; g.q[2] = qq.z; g.q[3] = qq.w;
  g.v = d.scalars[i];
  g.w = d.weights ? d.weights[i] : 1.0f;
  g.finite = finite3(g.mu) && finite3(g.ls) && __builtin_isfinite(g.q[0]) && __builtin_isfinite(g.q[1]) &&
             __builtin_isfinite(g.q[2]) && __builtin_isfinite(g.q[3]) && __builtin_isfinite(g.v) &&
             __builtin_isfinite(g.w);
  g.n2 = ((g.q[0] * g.q[0] + g.q[1] * g.q[1]) + g.q[2] * g.q[2]) + g.q[3] * g.q[3];
  g.inv = 1.0f / sqrtf(g.n2);
  const float w = g.q[0] * g.inv, x = g.q[1] * g.inv, y = g.q[2] * g.inv, z = g.q[3] * g.inv;
  g.qh[0] = w; g.qh[1] = x; g.qh[2] = y; g.qh[3] = z;
  g.R[0] = 1.0f - 2.0f * (y * y + z * z);
  g.R[1] = 2.0f * (x * y - w * z);
  g.R[2] = 2.0f * (x * z + w * y);
  g.R[3] = 2.0f * (x * y + w * z);
  g.R[4] = 1.0f - 2.0f * (x * x + z * z);
  g.R[5] = 2.0f * (y * z - w * x);
  g.R[6] = 2.0f * (x * z - w * y);
  g.R[7] = 2.0f * (y * z + w * x);
  g.R[8] = 1.0f - 2.0f * (x * x + y * y);
  g.s[0] = exp32(g.ls[0]);
  g.s[1] = exp32(g.ls[1]);
  g.s[2] = exp32(g.ls[2]);
  g.lit = d.normals != nullptr;
  if (g.lit) {
    const float* nr = d.normals + 3 * (size_t)i;
    const float n0 = nr[0], n1 = nr[1], n2 = nr[2];
    g.ka = d.k_ambient[i];
    g.kd = d.k_diffuse[i];
    g.ks = d.k_specular[i];
    g.beta = d.shininess[i];
    g.finite = g.finite && __builtin_isfinite(n0) && __builtin_isfinite(n1) && __builtin_isfinite(n2) &&
               __builtin_isfinite(g.ka) && __builtin_isfinite(g.kd) && __builtin_isfinite(g.ks) &&
               __builtin_isfinite(g.beta);
    g.nn2 = (n0 * n0 + n1 * n1) + n2 * n2;
    g.ninv = 1.0f / sqrtf(g.nn2);
    g.nh[0] = n0 * g.ninv;
    g.nh[1] = n1 * g.ninv;
    g.nh[2] = n2 * g.ninv;
  } else {
    g.nn2 = 1.0f;
  }
}

// Blinn-Phong colour of Eq. 2-3 under a headlight: light and view direction are both the
// unit vector l from the camera centre to the Gaussian, so the half vector is l and, with
// u = n^ . l and s = |u|, c = C (k_a + k_d s) + k_s s^beta (white; 0 when s = 0).
struct Lit {
  float l[3], dinv;   // unit light direction, 1 / |mu - campos|
  float u, s, f, sb;  // n^ . l, |u|, k_a + k_d s, s^beta
};

__device__ __forceinline__ void shade(const FrameDesc& d, const GParams& g, const float C[3], float rgb[3], Lit& L) {
  const float dx = g.mu[0] - d.campos[0], dy = g.mu[1] - d.campos[1], dz = g.mu[2] - d.campos[2];
  L.dinv = 1.0f / sqrtf((dx * dx + dy * dy) + dz * dz);
  L.l[0] = dx * L.dinv;
  L.l[1] = dy * L.dinv;
  L.l[2] = dz * L.dinv;
  L.u = (g.nh[0] * L.l[0] + g.nh[1] * L.l[1]) + g.nh[2] * L.l[2];
  L.s = fabsf(L.u);
  L.f = g.ka + g.kd * L.s;
  L.sb = L.s > 1e-30f ? exp32(g.beta * log32(L.s)) : 0.0f;
  for (int c = 0; c < 3; ++c) rgb[c] = C[c] * L.f + g.ks * L.sb;
}

struct TfSample {
  float rgb[3], O;
  float slope[4];   // d/dv of R,G,B,O on the active segment (0 outside [0,1])
};

__device__ __forceinline__ void tf_lookup(const FrameDesc& d, float v, TfSample& t) {
  const float vc = v < 0.0f ? 0.0f : (v > 1.0f ? 1.0f : v);
  const float tp = vc * (float)(d.K - 1);
  int i = (int)floorf(tp);
  if (i > d.K - 2) i = d.K - 2;
  const float fr = tp - (float)i;
  const float om = 1.0f - fr;
  const float4 L0 = reinterpret_cast<const float4*>(d.lut)[i];
  const float4 L1 = reinterpret_cast<const float4*>(d.lut)[i + 1];
  t.rgb[0] = L0.x * om + L1.x * fr;
  t.rgb[1] = L0.y * om + L1.y * fr;
  t.rgb[2] = L0.z * om + L1.z * fr;
  t.O = L0.w * om + L1.w * fr;
  const bool in = (v >= 0.0f) && (v <= 1.0f);
  const float km1 = (float)(d.K - 1);
  t.slope[0] = in ? (L1.x - L0.x) * km1 : 0.0f;
  t.slope[1] = in ? (L1.y - L0.y) * km1 : 0.0f;
  t.slope[2] = in ? (L1.z - L0.z) * km1 : 0.0f;
  t.slope[3] = in ? (L1.w - L0.w) * km1 : 0.0f;
}

// Per-frame projection of one Gaussian (footprint contract of veg_project).
struct Proj {
  double tx, ty, tz, xn, yn, mx, my;
  float depth;
  float xc, yc;
  bool clampx, clampy;
  float J00, J02, J11, J12;
  float Q[9], P[9];
  float G0[3], G1[3];
  float S00, S01, S11, det;
};

__device__ __forceinline__ void project_one(const FrameDesc& d, const KOpts& o, const GParams& g, Proj& p) {
  const float* V = d.view;
  p.tx = (((double)V[0] * g.mu[0] + (double)V[1] * g.mu[1]) + (double)V[2] * g.mu[2]) + (double)V[3];
  p.ty = (((double)V[4] * g.mu[0] + (double)V[5] * g.mu[1]) + (double)V[6] * g.mu[2]) + (double)V[7];
  p.tz = (((double)V[8] * g.mu[0] + (double)V[9] * g.mu[1]) + (double)V[10] * g.mu[2]) + (double)V[11];
  p.depth = (float)p.tz;
  p.xn = p.tx / p.tz;
  p.yn = p.ty / p.tz;
  p.mx = (double)d.fx * p.xn + (double)d.cx;
  p.my = (double)d.fy * p.yn + (double)d.cy;
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) {
      p.Q[3 * j + k] = (V[4 * j + 0] * g.R[k] + V[4 * j + 1] * g.R[3 + k]) + V[4 * j + 2] * g.R[6 + k];
      p.P[3 * j + k] = p.Q[3 * j + k] * g.s[k];
    }
  const float limx = o.guard * ((0.5f * (float)d.W) / d.fx);
  const float limy = o.guard * ((0.5f * (float)d.H) / d.fy);
  const float xnf = (float)p.xn, ynf = (float)p.yn;
  p.xc = fminf(fmaxf(xnf, -limx), limx);
  p.yc = fminf(fmaxf(ynf, -limy), limy);
  p.clampx = (xnf < -limx) || (xnf > limx);
  p.clampy = (ynf < -limy) || (ynf > limy);
  p.J00 = d.fx / p.depth;
  p.J02 = -(d.fx * p.xc) / p.depth;
  p.J11 = d.fy / p.depth;
  p.J12 = -(d.fy * p.yc) / p.depth;
  for (int k = 0; k < 3; ++k) {
    p.G0[k] = p.J00 * p.P[k] + p.J02 * p.P[6 + k];
    p.G1[k] = p.J11 * p.P[3 + k] + p.J12 * p.P[6 + k];
  }
  const float g00 = (p.G0[0] * p.G0[0] + p.G0[1] * p.G0[1]) + p.G0[2] * p.G0[2];
  const float g11 = (p.G1[0] * p.G1[0] + p.G1[1] * p.G1[1]) + p.G1[2] * p.G1[2];
  p.S00 = g00 + o.lowpass;
  p.S01 = (p.G0[0] * p.G1[0] + p.G0[1] * p.G1[1]) + p.G0[2] * p.G1[2];
  p.S11 = g11 + o.lowpass;
  // det(G G^T + lowpass I) = |G0 x G1|^2 + lowpass (|G0|^2 + |G1|^2) + lowpass^2 (Cauchy-Binet):
  // a sum of non-negative terms, free of the cancellation in S00 S11 - S01^2 that costs an
  // elongated footprint most of its significant bits.
  const float x0 = p.G0[1] * p.G1[2] - p.G0[2] * p.G1[1];
  const float x1 = p.G0[2] * p.G1[0] - p.G0[0] * p.G1[2];
  const float x2 = p.G0[0] * p.G1[1] - p.G0[1] * p.G1[0];
  p.det = (((x0 * x0 + x1 * x1) + x2 * x2) + o.lowpass * (g00 + g11)) + o.lowpass * o.lowpass;
}

// Pixel range of the footprint (the ellipse where A exp(-sigma) >= alpha_min, by the
// extent contract of veg_project), clipped to the image; false when it holds no pixel.
__device__ __forceinline__ bool pixel_range(const Proj& p, float A, const KOpts& o, int W, int H, double& xlo,
                                            double& xhi, double& ylo, double& yhi) {
  const float tau = 2.0f * log32(A / o.alpha_min);
  const float ex = sqrtf(tau * p.S00);
  const float ey = sqrtf(tau * p.S11);
  xlo = ceil((p.mx - (double)ex) - 0.5);
  xhi = floor((p.mx + (double)ex) - 0.5);
  ylo = ceil((p.my - (double)ey) - 0.5);
  yhi = floor((p.my + (double)ey) - 0.5);
  xlo = fmax(xlo, 0.0);
  ylo = fmax(ylo, 0.0);
  xhi = fmin(xhi, (double)(W - 1));
  yhi = fmin(yhi, (double)(H - 1));
  return (xlo <= xhi) && (ylo <= yhi);
}

struct Blob {
  uint32_t w[kBlobMaxBytes / 4];
};

__global__ __launch_bounds__(256) void blob_kernel(uint32_t* dst, const uint32_t nwords, const Blob blob) {
  for (uint32_t i = threadIdx.x; i < nwords; i += blockDim.x) dst[i] = blob.w[i];
}

// A wave's 64 consecutive records (lane l's at rec + 3 l) written as 192 contiguous
// float4, lane l storing pieces l, 64 + l and 128 + l, so each store instruction covers
// 1 KB without holes; only pieces of lanes set in `keep` are written.  The pieces pass
// through the wave's own LDS slice (LDS operations of one wave complete in order).
__device__ __forceinline__ void store_wave_records(float4* __restrict__ rec, uint64_t keep, const float4& a,
                                                   const float4& b, const float4& c, float4* __restrict__ s) {
  const int ln = threadIdx.x & 63;
  s[3 * ln] = a;
  s[3 * ln + 1] = b;
  s[3 * ln + 2] = c;
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int e = 64 * j + ln;
    if ((keep >> (e / 3)) & 1ull) rec[e] = s[e];
  }
  __builtin_amdgcn_wave_barrier();
}

// One thread per Gaussian; blockIdx.y selects a chunk of `fpb` frames processed in a loop,
// so a model shared by the frames is read from HBM once per chunk.  The loops over frames
// and over a view's tables are uniform across the block, so every wave takes part in each
// record store.
__global__ __launch_bounds__(256) void project_kernel(const FrameDesc* __restrict__ descs, int n_frames,
                                                      int fpb, KOpts o, float4* __restrict__ rec,
                                                      uint32_t* __restrict__ count,
                                                      uint32_t* __restrict__ depth) {
  __shared__ float4 s_rec[4][3 * 64];   // one slice per wave of the 256-thread block
  const int i = blockIdx.x * 256 + threadIdx.x;
  const uint32_t i0 = (uint32_t)(i - (int)(threadIdx.x & 63));   // the wave's first Gaussian
  float4* sw = s_rec[threadIdx.x >> 6];
  const int f0 = blockIdx.y * fpb;
  const int f1 = min(n_frames, f0 + fpb);
  GParams g;
  const float* cur = nullptr;
  const float* cur_v = nullptr;
  const float* cur_w = nullptr;
  const float* cur_n = nullptr;
  for (int f = f0; f < f1; ++f) {
    const FrameDesc& d = descs[f];
    if (d.n_share == 0) continue;   // a frame sharing another's list is projected with it
    const int n_share = d.n_share;
    const bool act = i < d.n;
    bool kept = false;
    Proj p;
    TfSample tf;
    uint32_t x0 = 0u, x1 = 0u, y0 = 0u, y1 = 0u;
    float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, mxr = 0.0f, myr = 0.0f;
    float A = 0.0f;   // the largest A over the frames sharing the list
    if (act) {
      if (d.means != cur || d.scalars != cur_v || d.weights != cur_w || d.normals != cur_n) {
        load_params(d, i, g);
        cur = d.means;
        cur_v = d.scalars;
        cur_w = d.weights;
        cur_n = d.normals;
      }
      const uint32_t pid = d.pair_base + (uint32_t)i;
      bool keep = g.finite && g.n2 >= 1e-24f && g.nn2 >= 1e-24f;
      tf_lookup(d, keep ? g.v : 0.0f, tf);
      // Frames sharing this list: the footprint at the largest A over their tables contains
      // each frame's own, so it decides the list; only the owner's pair is counted.
      A = tf.O * g.w;
      for (int k = 1; k < n_share; ++k) {
        const FrameDesc& dk = descs[f + k];
        count[dk.pair_base + (uint32_t)i] = 0u;
        TfSample tk;
        tf_lookup(dk, keep ? g.v : 0.0f, tk);
        A = fmaxf(A, tk.O * g.w);
      }
      keep = keep && (A >= o.alpha_min);
      project_one(d, o, g, p);
      keep = keep && (p.depth > o.near_z) && (p.det > 0.0f);
      double xlo, xhi, ylo, yhi;
      kept = keep && pixel_range(p, A, o, d.W, d.H, xlo, xhi, ylo, yhi);
      if (kept) {
        x0 = (uint32_t)xlo / kTile;
        x1 = (uint32_t)xhi / kTile;
        y0 = (uint32_t)ylo / kTile;
        y1 = (uint32_t)yhi / kTile;
        count[pid] = (x1 - x0 + 1) * (y1 - y0 + 1);
        depth[pid] = __float_as_uint(p.depth);
        c0 = p.S11 / p.det;
        c1 = -p.S01 / p.det;
        c2 = p.S00 / p.det;
        mxr = (float)(p.mx - 16.0 * (double)x0);
        myr = (float)(p.my - 16.0 * (double)y0);
      } else {
        count[pid] = 0u;
      }
    }
    const uint64_t wkeep = __ballot(kept);
    uint32_t keep_bits = 0u;   // frames of the view that keep the Gaussian (bit k: slot k)
    // one record per frame: the shared geometry with the frame's own A and colour.  A = 0
    // where the frame's own footprint culls the Gaussian (A below alpha_min, or an ellipse
    // that covers no pixel centre), so the frame keeps exactly the Gaussians it would keep
    // on its own list and its blend skips the rest.
    for (int k = 0; k < n_share; ++k) {
      const FrameDesc& dk = descs[f + k];
      float4 r0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), r1 = r0, r2 = r0;
      if (kept) {
        TfSample tk = tf;
        if (k > 0) tf_lookup(dk, g.v, tk);
        float Ak = tk.O * g.w;
        if (!(Ak >= o.alpha_min)) Ak = 0.0f;
        uint32_t inset = 0u;   // own tile rectangle inside the shared one
        // the frame whose A is the largest has the shared footprint itself (no insets)
        if (n_share > 1 && Ak > 0.0f && Ak != A) {
          double a0, a1, b0, b1;
          if (!pixel_range(p, Ak, o, d.W, d.H, a0, a1, b0, b1)) {
            Ak = 0.0f;
          } else {
            const uint32_t ox0 = (uint32_t)a0 / kTile, ox1 = (uint32_t)a1 / kTile;
            const uint32_t oy0 = (uint32_t)b0 / kTile, oy1 = (uint32_t)b1 / kTile;
            // each inset clamped to [0, 31]: never claims more than the shared rectangle excludes
            const uint32_t ix0 = ox0 > x0 ? min(ox0 - x0, 31u) : 0u, iy0 = oy0 > y0 ? min(oy0 - y0, 31u) : 0u;
            const uint32_t ix1 = x1 > ox1 ? min(x1 - ox1, 31u) : 0u, iy1 = y1 > oy1 ? min(y1 - oy1, 31u) : 0u;
            inset = ix0 | (iy0 << 5) | (ix1 << 10) | (iy1 << 15);
          }
        }
        float rgb[3] = {tk.rgb[0], tk.rgb[1], tk.rgb[2]};
        if (g.lit) {
          Lit L;
          shade(dk, g, tk.rgb, rgb, L);
        }
        if (Ak > 0.0f || k >= 32) keep_bits |= 1u << min(k, 31);
        r0 = make_float4(mxr, myr, c0, c1);
        r1 = make_float4(c2, Ak, rgb[0], rgb[1]);
        r2 = make_float4(rgb[2], __uint_as_float(x0 | (y0 << 16)), __uint_as_float(x1 | (y1 << 16)),
                         __uint_as_float((uint32_t)(f + k) | (inset << kFrameBits)));
      }
      if (wkeep) store_wave_records(rec + 3 * (size_t)(dk.pair_base + i0), wkeep, r0, r1, r2, sw);
    }
    // a shared list's frames skip entries by these bits before loading their records; the
    // depth slots of the frames after the owner are otherwise unused (never counted)
    if (kept && n_share > 1) depth[descs[f + 1].pair_base + (uint32_t)i] = keep_bits;
  }
}

// Adjoint of the projection: one thread per Gaussian, loop over the frames (which share the
// model), accumulate in registers, add once to the parameter gradients.
// Whether frame f keeps Gaussian i (the densification statistics' definition): its list
// holds the Gaussian and, for a frame on a list shared by several frames, the frame's own
// footprint keeps it (keep bit of its slot in the depth slots of the view's second frame;
// from slot 31 on, the record's A > 0).
__device__ __forceinline__ bool frame_keeps(const FrameDesc* __restrict__ descs, const FrameDesc& d, int i,
                                            const BwdFused& fu) {
  const FrameDesc& dl = descs[d.list_frame];
  if (fu.count[(size_t)dl.pair_base + (size_t)i] == 0u) return false;
  if (dl.n_share <= 1) return true;
  if (d.slot < 31) return (fu.depth[(size_t)descs[d.list_frame + 1].pair_base + (size_t)i] >> d.slot) & 1u;
  return fu.rec[3 * ((size_t)d.pair_base + (size_t)i) + 1].y > 0.0f;
}

// One thread per Gaussian, over every frame.  With kFused, the densification statistics are
// taken from the same g2d reads (fu.acc/fu.vis, when given; frames in the order the separate
// statistics pass takes them, so the sums are the same) and, with fu.consume, every g2d
// record read is left zero.
template <bool kFused>
__global__ __launch_bounds__(256) void project_bwd_kernel(const FrameDesc* __restrict__ descs, int n_frames,
                                                          int n, KOpts o, float* __restrict__ g2d,
                                                          uint32_t n_pairs, veg_grads gr, BwdFused fu) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  GParams g;
  load_params(descs[0], i, g);
  float st_acc = 0.0f;
  int st_vis = 0;
  if (!g.finite || !(g.n2 >= 1e-24f) || !(g.nn2 >= 1e-24f)) {
    // no parameter gradient; the statistics and the consumption of g2d as below
    if (kFused) {
      for (int f = 0; f < n_frames; ++f) {
        const size_t pid = (size_t)descs[f].pair_base + (size_t)i;
        if (fu.acc && frame_keeps(descs, descs[f], i, fu)) {
          const float gx = g2d[pid * 9 + 0], gy = g2d[pid * 9 + 1];
          st_acc += sqrtf(gx * gx + gy * gy);
          ++st_vis;
        }
        if (fu.consume)
          for (int c = 0; c < 9; ++c) g2d[pid * 9 + c] = 0.0f;
      }
      if (fu.acc) {
        fu.acc[i] += st_acc;
        fu.vis[i] += st_vis;
      }
    }
    return;
  }
  float dmu[3] = {0, 0, 0}, dR[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, ds[3] = {0, 0, 0};
  float dv = 0.0f, dw = 0.0f;
  float dn[3] = {0, 0, 0}, dka = 0.0f, dkd = 0.0f, dks = 0.0f, dbeta = 0.0f;
  for (int f = 0; f < n_frames;) {
    // The frames of a view (veg_project_views) share one camera, so one projected geometry:
    // the chain from the screen-space geometry (centre, conic) and from the shading's
    // geometric terms back to the parameters is linear in their gradients, which are summed
    // over the view's frames and taken through the chain once.  Opacity and colour go
    // through each frame's own table.
    const FrameDesc& d = descs[f];
    const int K = d.n_share > 1 ? d.n_share : 1;
    float dmx = 0.0f, dmy = 0.0f, dc0 = 0.0f, dc1 = 0.0f, dc2 = 0.0f;
    float P = 0.0f, Dsum = 0.0f;   // shading: sum over frames of dC . C(v) and of sum_c dC
    bool any = false;
    Lit L;
    for (int k = 0; k < K; ++k) {
      const FrameDesc& dk = descs[f + k];
      const size_t pid = (size_t)dk.pair_base + (size_t)i;
      float gg[9];
      bool anyk = false;
      for (int c = 0; c < 9; ++c) {
        gg[c] = g2d[pid * 9 + c];
        anyk |= (gg[c] != 0.0f);
      }
      if (kFused) {
        if (fu.acc && frame_keeps(descs, dk, i, fu)) {
          st_acc += sqrtf(gg[0] * gg[0] + gg[1] * gg[1]);
          ++st_vis;
        }
        if (fu.consume && anyk)
          for (int c = 0; c < 9; ++c) g2d[pid * 9 + c] = 0.0f;
      }
      if (!anyk) continue;
      TfSample tf;
      tf_lookup(dk, g.v, tf);
      // lighting: rgb = C (k_a + k_d s) + k_s s^beta, s = |n^ . l|, l = (mu - campos) / |.|
      float dC[3] = {gg[5], gg[6], gg[7]};
      if (g.lit) {
        if (!any) {
          float rgb[3];
          shade(d, g, tf.rgb, rgb, L);   // L depends on the view's camera and the Gaussian only
        }
        P += (gg[5] * tf.rgb[0] + gg[6] * tf.rgb[1]) + gg[7] * tf.rgb[2];
        Dsum += (gg[5] + gg[6]) + gg[7];
        for (int c = 0; c < 3; ++c) dC[c] = gg[5 + c] * L.f;
      }
      any = true;
      dmx += gg[0];
      dmy += gg[1];
      dc0 += gg[2];
      dc1 += gg[3];
      dc2 += gg[4];
      // transfer function: A = O w, C = C(v)
      dv += (gg[8] * g.w) * tf.slope[3] + dC[0] * tf.slope[0] + dC[1] * tf.slope[1] + dC[2] * tf.slope[2];
      dw += gg[8] * tf.O;
    }
    f += K;
    if (!any) continue;
    if (g.lit) {
      dka += P;
      dkd += P * L.s;
      float dsv = g.kd * P;
      if (L.sb > 0.0f) {
        dks += Dsum * L.sb;
        dbeta += Dsum * g.ks * L.sb * log32(L.s);
        dsv += Dsum * g.ks * g.beta * L.sb / L.s;
      }
      const float du = L.u > 0.0f ? dsv : (L.u < 0.0f ? -dsv : 0.0f);
      float dnh[3], dl[3];
      for (int k = 0; k < 3; ++k) {
        dnh[k] = du * L.l[k];
        dl[k] = du * g.nh[k];
      }
      const float dotn = (dnh[0] * g.nh[0] + dnh[1] * g.nh[1]) + dnh[2] * g.nh[2];
      const float dotl = (dl[0] * L.l[0] + dl[1] * L.l[1]) + dl[2] * L.l[2];
      for (int k = 0; k < 3; ++k) {
        dn[k] += (dnh[k] - g.nh[k] * dotn) * g.ninv;
        dmu[k] += (dl[k] - L.l[k] * dotl) * L.dinv;
      }
    }
    Proj p;
    project_one(d, o, g, p);
    // projected centre
    const float tz = p.depth;
    const float invz = 1.0f / tz;
    const float xn = (float)p.xn, yn = (float)p.yn;
    float dt[3];
    dt[0] = dmx * d.fx * invz;
    dt[1] = dmy * d.fy * invz;
    dt[2] = -(dmx * d.fx * xn + dmy * d.fy * yn) * invz;
    // conic = inverse(S), then S = G G^T + lowpass I, in float64.  For an elongated
    // footprint dS = -C dC C is large and dG = 2 dS G cancels it down to a small result
    // along the long axis: float32 would lose about log2 of the squared condition number
    // of S there, float64 does not (and runs at the float32 rate on this GPU's VALU).
    double dG0d[3], dG1d[3];
    {
      const double S00 = p.S00, S01 = p.S01, S11 = p.S11;
      const double det = S00 * S11 - S01 * S01;
      const double c0 = S11 / det, c1 = -S01 / det, c2 = S00 / det;
      const double e0 = dc0, e1 = dc1, e2 = dc2;
      const double dS00 = -(e0 * c0 * c0 + e1 * c0 * c1 + e2 * c1 * c1);
      const double dS11 = -(e0 * c1 * c1 + e1 * c1 * c2 + e2 * c2 * c2);
      const double dS01 = -(2.0 * e0 * c0 * c1 + e1 * (c0 * c2 + c1 * c1) + 2.0 * e2 * c1 * c2);
      for (int k = 0; k < 3; ++k) {
        dG0d[k] = 2.0 * dS00 * (double)p.G0[k] + dS01 * (double)p.G1[k];
        dG1d[k] = 2.0 * dS11 * (double)p.G1[k] + dS01 * (double)p.G0[k];
      }
    }
    float dG0[3], dG1[3];
    for (int k = 0; k < 3; ++k) {
      dG0[k] = (float)dG0d[k];
      dG1[k] = (float)dG1d[k];
    }
    // G = J P
    float dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0, dP[9];
    for (int k = 0; k < 3; ++k) {
      dJ00 += dG0[k] * p.P[k];
      dJ02 += dG0[k] * p.P[6 + k];
      dJ11 += dG1[k] * p.P[3 + k];
      dJ12 += dG1[k] * p.P[6 + k];
      dP[k] = p.J00 * dG0[k];
      dP[3 + k] = p.J11 * dG1[k];
      dP[6 + k] = p.J02 * dG0[k] + p.J12 * dG1[k];
    }
    // J(t): J00 = fx/z, J11 = fy/z, J02 = -fx xc/z, J12 = -fy yc/z (xc = x/z unless clamped)
    dt[2] += -dJ00 * p.J00 * invz - dJ11 * p.J11 * invz;
    if (!p.clampx) {
      dt[0] += dJ02 * (-d.fx * invz * invz);
      dt[2] += dJ02 * (-2.0f * p.J02 * invz);
    } else {
      dt[2] += dJ02 * (-p.J02 * invz);
    }
    if (!p.clampy) {
      dt[1] += dJ12 * (-d.fy * invz * invz);
      dt[2] += dJ12 * (-2.0f * p.J12 * invz);
    } else {
      dt[2] += dJ12 * (-p.J12 * invz);
    }
    // P = Q diag(s), Q = Vr R, t = Vr mu + b
    const float* V = d.view;
    for (int k = 0; k < 3; ++k) {
      float dQ[3];
      for (int j = 0; j < 3; ++j) {
        dQ[j] = dP[3 * j + k] * g.s[k];
        ds[k] += dP[3 * j + k] * p.Q[3 * j + k];
      }
      for (int m = 0; m < 3; ++m) dR[3 * m + k] += V[m] * dQ[0] + V[4 + m] * dQ[1] + V[8 + m] * dQ[2];
    }
    for (int m = 0; m < 3; ++m) dmu[m] += V[m] * dt[0] + V[4 + m] * dt[1] + V[8 + m] * dt[2];
  }
  // rotation from the normalised quaternion (w,x,y,z)
  const float w = g.qh[0], x = g.qh[1], y = g.qh[2], z = g.qh[3];
  float dqh[4];
  dqh[0] = -2 * z * dR[1] + 2 * y * dR[2] + 2 * z * dR[3] - 2 * x * dR[5] - 2 * y * dR[6] + 2 * x * dR[7];
  dqh[1] = 2 * y * dR[1] + 2 * z * dR[2] + 2 * y * dR[3] - 4 * x * dR[4] - 2 * w * dR[5] + 2 * z * dR[6] +
           2 * w * dR[7] - 4 * x * dR[8];
  dqh[2] = -4 * y * dR[0] + 2 * x * dR[1] + 2 * w * dR[2] + 2 * x * dR[3] + 2 * z * dR[5] - 2 * w * dR[6] +
           2 * z * dR[7] - 4 * y * dR[8];
  dqh[3] = -4 * z * dR[0] - 2 * w * dR[1] + 2 * x * dR[2] + 2 * w * dR[3] - 4 * z * dR[4] + 2 * y * dR[5] +
           2 * x * dR[6] + 2 * y * dR[7];
  const float dot = dqh[0] * w + dqh[1] * x + dqh[2] * y + dqh[3] * z;
  for (int k = 0; k < 3; ++k) {
    gr.d_means[3 * (size_t)i + k] += dmu[k];
    gr.d_log_scales[3 * (size_t)i + k] += ds[k] * g.s[k];
  }
  for (int k = 0; k < 4; ++k) gr.d_quats[4 * (size_t)i + k] += (dqh[k] - g.qh[k] * dot) * g.inv;
  gr.d_scalars[i] += dv;
  if (gr.d_weights) gr.d_weights[i] += dw;
  if (gr.d_normals) {
    for (int k = 0; k < 3; ++k) gr.d_normals[3 * (size_t)i + k] += dn[k];
    gr.d_k_ambient[i] += dka;
    gr.d_k_diffuse[i] += dkd;
    gr.d_k_specular[i] += dks;
    gr.d_shininess[i] += dbeta;
  }
  if (kFused && fu.acc) {
    fu.acc[i] += st_acc;
    fu.vis[i] += st_vis;
  }
}

__global__ void debug_math_kernel(int op, const float* x, const float* y, float* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (op == 4 || op == 5) {
    // wave-level primitives: every lane of the wave must participate
    const float xv = i < n ? x[i] : 0.0f;
    float r;
    if (op == 4) r = __uint_as_float(wave_incl_scan_u32(__float_as_uint(xv)));
    else r = wave_sum_to_lane63(xv);
    if (i < n) out[i] = r;
    return;
  }
  if (i >= n) return;
  float r = 0.0f;
  switch (op) {
    case 0: r = exp32(x[i]); break;
    case 1: r = log32(x[i]); break;
    case 2: r = x[i] / y[i]; break;
    case 3: r = sqrtf(x[i]); break;
    default: r = 0.0f;
  }
  out[i] = r;
}

}  // namespace

hipError_t write_blob(void* dst_dev, const void* src_host, size_t bytes, hipStream_t stream) {
  if (bytes % 4 != 0 || bytes > (size_t)kBlobMaxBytes) return hipErrorInvalidValue;
  Blob b;
  __builtin_memset(&b, 0, sizeof(b));
  __builtin_memcpy(&b, src_host, bytes);
  hipLaunchKernelGGL(blob_kernel, dim3(1), dim3(256), 0, stream, (uint32_t*)dst_dev, (uint32_t)(bytes / 4), b);
  return hipGetLastError();
}

hipError_t launch_project(const FrameDesc* descs, int n_frames, int n_max, const KOpts& o, float4* rec,
                          uint32_t* count, uint32_t* depth, bool shared_model, hipStream_t stream) {
  if (n_frames <= 0 || n_max <= 0) return hipSuccess;
  const int fpb = shared_model ? 8 : 1;
  dim3 grid((n_max + 255) / 256, (n_frames + fpb - 1) / fpb);
  hipLaunchKernelGGL(project_kernel, grid, dim3(256), 0, stream, descs, n_frames, fpb, o, rec, count, depth);
  return hipGetLastError();
}

hipError_t launch_project_bwd(const FrameDesc* descs, int n_frames, int n, const KOpts& o, float* g2d,
                              uint32_t n_pairs, const veg_grads& grads, hipStream_t stream, const BwdFused& fused) {
  if (n <= 0 || n_frames <= 0) return hipSuccess;
  if (fused.acc || fused.consume)
    hipLaunchKernelGGL(project_bwd_kernel<true>, dim3((n + 255) / 256), dim3(256), 0, stream, descs, n_frames, n, o,
                       g2d, n_pairs, grads, fused);
  else
    hipLaunchKernelGGL(project_bwd_kernel<false>, dim3((n + 255) / 256), dim3(256), 0, stream, descs, n_frames, n, o,
                       g2d, n_pairs, grads, fused);
  return hipGetLastError();
}

hipError_t launch_debug_math(int op, const float* x, const float* y, float* out, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(debug_math_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, op, x, y, out, n);
  return hipGetLastError();
}

}  // namespace veg
