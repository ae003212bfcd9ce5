// Binning and sorting for the tile-based rasterizer (paper, section "Rendering of VEGs":
// the 2D Gaussians intersecting the screen are rasterized tile by tile, blended front to
// back).  The key list is built depth-first:
//   1. compact the kept (frame, Gaussian) pairs and sort them by (depth key, pair id)
//      with a stable LSD radix sort of the keys relative to the smallest kept one (three
//      8-bit passes when they span less than 2^24, else four over the 31 key bits);
//   2. prefix-sum their tile counts in that order and emit one (tile, pair) entry per
//      covered tile -- so within each tile the entries are already front to back;
//   3. stable LSD radix sort by tile id over just the bits of the largest tile id;
//   4. per-tile [start, end) ranges from the key boundaries.
// The result equals the list sorted by (tile, depth key, pair id).  Every kernel reads its
// element count from device memory, so the pipeline needs no host synchronisation.
#include <mutex>

#include "veg_device.h"

namespace veg {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kIpt = 8;                      // items per thread per tile
constexpr int kTileItems = kThreads * kIpt;  // 2048

constexpr int kSortIpt = 16;                       // radix sort: items per thread per tile
constexpr int kSortTile = kThreads * kSortIpt;     // 4096
constexpr int kChunk = 2048;                       // emission: output slots per chunk

// Block b's contiguous segment of [0, n) when n is split over G blocks in whole tiles.
template <int TILE = kTileItems>
__device__ __forceinline__ void segment_of(uint32_t n, int G, int b, uint32_t& begin, uint32_t& end) {
  uint64_t per = ((uint64_t)n + (uint64_t)G - 1) / (uint64_t)G;
  per = (per + TILE - 1) / TILE * TILE;
  const uint64_t bg = (uint64_t)b * per;
  begin = (uint32_t)(bg < n ? bg : n);
  const uint64_t en = bg + per;
  end = (uint32_t)(en < n ? en : n);
}

__device__ __forceinline__ uint32_t read_count(const uint32_t* n_ptr, uint32_t n_cap) {
  if (!n_ptr) return n_cap;
  const uint32_t v = *n_ptr;
  return v < n_cap ? v : n_cap;
}

// Exclusive scan over the 256 threads of a block; *total gets the block sum.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* s_tmp, uint32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_scan_u32(v);
  if (lane == 63) s_tmp[w] = incl;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) {
    const uint32_t t = s_tmp[k];
    base += (k < w) ? t : 0u;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

// ------------------------------------------------------------------------------ scans
// Three item kinds share the reduce-then-scan machinery:
//   kVis : list slot i (pair list_pair(i)), value = count of that pair > 0   (compaction)
//   kCnt : item j of the depth-sorted kept pairs, value = its tile count   (entry offsets)
//   kRaw : value = data[i]   (radix histogram scan)
enum ScanKind { kVis = 0, kCnt = 1, kRaw = 2 };

struct ScanSrc {
  const uint32_t* count;   // kVis
  const uint32_t* data;    // kCnt, kRaw
};

// The pair slots a compaction walks.  When the frames of each view share the first frame's
// key list (per_view frames a view), only that frame's slots can hold a kept pair: list
// slot o = view * n + i is pair view * per_view * n + i, and skip = (per_view - 1) n is
// what each earlier view adds (skip 0: every slot, in order).
struct ListMap {
  uint32_t n, skip;
  double inv_n;
};
__device__ __forceinline__ uint32_t list_pair(uint32_t o, const ListMap& m) {
  if (m.skip == 0u) return o;
  uint64_t q = (uint64_t)((double)o * m.inv_n);   // within one of o / n
  if (q * m.n > o) --q;
  else if ((q + 1) * m.n <= o) ++q;
  return o + (uint32_t)q * m.skip;
}

// Depth keys relative to the smallest kept one.  The compaction and key_range_kernel leave,
// in range[0..1], the complement of the smallest kept depth key and the largest (two
// maxima, from zero).  The depth passes rank key - min: the same order, and when every kept
// key lies within 2^24 of the smallest, the last pass (bits 24-31) would leave it unchanged
// and is skipped.
__device__ __forceinline__ uint32_t key_base(const uint32_t* range) { return range ? ~range[0] : 0u; }
__device__ __forceinline__ bool keys_narrow(const uint32_t* range) {
  return range && ((range[1] - ~range[0]) >> 24) == 0u;
}

template <int KIND>
__device__ __forceinline__ uint32_t item_of_word(uint32_t w) {
  return KIND == kVis ? (w > 0u ? 1u : 0u) : w;
}

// Block b's total over its segment.  Each thread sums its share of the whole segment (16-byte
// loads where the array is 16-byte aligned; segments start at multiples of kTileItems), and
// the block adds the threads' sums once at the end.
template <int KIND>
__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(ScanSrc src, const uint32_t* n_ptr, uint32_t n_cap,
                                                               uint64_t* partials, int G, ListMap lm = ListMap{}) {
  __shared__ uint64_t s_w[kWaves];
  const uint32_t n = read_count(n_ptr, n_cap);
  uint32_t begin, end;
  segment_of(n, G, blockIdx.x, begin, end);
  const uint32_t* __restrict__ a = KIND == kVis ? src.count : src.data;
  uint64_t acc = 0;
  uint32_t i = begin + threadIdx.x;
  // groups of four slots stay consecutive pairs when n is a multiple of four
  if ((reinterpret_cast<uintptr_t>(a) & 15u) == 0 && (lm.skip == 0u || (lm.n & 3u) == 0u)) {
    const uint32_t nv = (end - begin) / 4;
#pragma unroll 4
    for (uint32_t v = threadIdx.x; v < nv; v += kThreads) {
      const uint4 q = *reinterpret_cast<const uint4*>(a + list_pair(begin + 4 * v, lm));
      acc += (uint64_t)((item_of_word<KIND>(q.x) + item_of_word<KIND>(q.y)) +
                        (item_of_word<KIND>(q.z) + item_of_word<KIND>(q.w)));
    }
    i = begin + 4 * nv + threadIdx.x;
  }
  for (; i < end; i += kThreads) acc += item_of_word<KIND>(a[list_pair(i, lm)]);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) t += s_w[k];
    partials[blockIdx.x] = t;
  }
}

// Exclusive scan of G <= 4096 partial sums in place (one block of 1024 threads).  The total
// goes to out_total[0..1] as (low, high) 32-bit words; out_u32 (optional) gets it
// saturated to 32 bits.
__global__ __launch_bounds__(1024) void scan_partials_kernel(uint64_t* partials, int G, uint32_t* out_total,
                                                             uint32_t* out_u32) {
  __shared__ uint64_t s[1024];
  const int t = threadIdx.x;
  uint64_t v[4];
  uint64_t sum = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = 4 * t + k;
    v[k] = i < G ? partials[i] : 0ull;
    sum += v[k];
  }
  s[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint64_t add = t >= off ? s[t - off] : 0ull;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  uint64_t run = s[t] - sum;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = 4 * t + k;
    if (i < G) partials[i] = run;
    run += v[k];
  }
  if (t == 1023) {
    const uint64_t tot = s[1023];
    if (out_total) {
      out_total[0] = (uint32_t)tot;
      out_total[1] = (uint32_t)(tot >> 32);
    }
    if (out_u32) *out_u32 = tot > 0xffffffffull ? 0xffffffffu : (uint32_t)tot;
  }
}

// Downsweep of the compaction: kept pair i goes to (dkey, dval)[pos] = (depth[i], i), in
// index order over the list slots of `lm`.  A tile's items are read lane-strided (item
// t0 + k * 256 + thread, so every load is coalesced); each wave ranks its 64 items of round
// k with a ballot, and the rounds' and waves' kept counts are scanned in (round, wave) order
// -- index order -- so the kept items of one wave and round land in consecutive slots and
// every store is contiguous.  Each block also leaves, in block_range[2b..2b+1], the
// complement of its smallest kept depth key and its largest (zeros without kept pairs).
__global__ __launch_bounds__(kThreads) void compact_kernel(const uint32_t* __restrict__ count,
                                                           const uint32_t* __restrict__ depth,
                                                           const uint32_t* __restrict__ n_ptr, uint32_t n_cap,
                                                           const uint64_t* __restrict__ partials, int G,
                                                           uint32_t* __restrict__ dkey, uint32_t* __restrict__ dval,
                                                           ListMap lm, uint32_t* __restrict__ block_range) {
  __shared__ uint32_t s_wc[kIpt][kWaves];
  __shared__ uint32_t s_r[kWaves][2];
  uint32_t kmax = 0u, kcmax = 0u;   // largest kept key and largest complement (smallest key)
  const uint32_t n = read_count(n_ptr, n_cap);
  uint32_t begin, end;
  segment_of(n, G, blockIdx.x, begin, end);
  uint64_t base = partials[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = lanemask_lt();
  for (uint32_t t0 = begin; t0 < end; t0 += kTileItems) {
    uint64_t m[kIpt];
    uint32_t pr[kIpt];
#pragma unroll
    for (int k = 0; k < kIpt; ++k) {
      const uint32_t i = t0 + k * kThreads + threadIdx.x;
      pr[k] = list_pair(i, lm);
      m[k] = __ballot(i < end && count[pr[k]] > 0u);
      if (lane == 0) s_wc[k][w] = (uint32_t)__popcll(m[k]);
    }
    __syncthreads();
    uint32_t off[kIpt], run = 0;
#pragma unroll
    for (int k = 0; k < kIpt; ++k) {
#pragma unroll
      for (int v = 0; v < kWaves; ++v) {
        if (v == w) off[k] = run;
        run += s_wc[k][v];
      }
    }
    __syncthreads();   // s_wc is rewritten by the next tile
#pragma unroll
    for (int k = 0; k < kIpt; ++k) {
      if ((m[k] >> lane) & 1ull) {
        const uint64_t pos = base + off[k] + (uint32_t)__popcll(m[k] & lt);
        const uint32_t key = depth[pr[k]];
        dkey[pos] = key;
        dval[pos] = pr[k];
        kmax = max(kmax, key);
        kcmax = max(kcmax, ~key);
      }
    }
    base += run;
  }
  // the block's extremes (both maxima from zero: a block without kept pairs leaves zeros)
  for (int off = 32; off > 0; off >>= 1) {
    kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, off));
    kcmax = max(kcmax, (uint32_t)__shfl_xor((int)kcmax, off));
  }
  if (lane == 0) {
    s_r[w][0] = kcmax;
    s_r[w][1] = kmax;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    uint32_t v = 0u;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) v = max(v, s_r[k][threadIdx.x]);
    block_range[2 * blockIdx.x + threadIdx.x] = v;
  }
}

// range[0..1] = maxima over the G blocks' (complement of the smallest, largest) kept depth
// keys (one block of 1024 threads).
__global__ __launch_bounds__(1024) void key_range_kernel(const uint32_t* __restrict__ block_range, int G,
                                                         uint32_t* __restrict__ range) {
  __shared__ uint32_t s_r[16][2];
  uint32_t a = 0u, b = 0u;
  for (int i = threadIdx.x; i < G; i += 1024) {
    a = max(a, block_range[2 * i]);
    b = max(b, block_range[2 * i + 1]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    a = max(a, (uint32_t)__shfl_xor((int)a, off));
    b = max(b, (uint32_t)__shfl_xor((int)b, off));
  }
  if ((threadIdx.x & 63) == 0) {
    s_r[threadIdx.x >> 6][0] = a;
    s_r[threadIdx.x >> 6][1] = b;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    uint32_t v = 0u;
    for (int k = 0; k < 16; ++k) v = max(v, s_r[k][threadIdx.x]);
    range[threadIdx.x] = v;
  }
}

// After the depth sort: one gather per kept pair, in front-to-back order, of what the
// count scan and the emission need (pair id, tile rectangle, frame) and of its tile count,
// so both later passes read sequentially.  The record reads land at random addresses, so
// each thread takes kGatherIpt items a round (block-strided, coalesced for the sequential
// arrays) and issues all their loads before using any.
constexpr int kGatherIpt = 4;

__global__ __launch_bounds__(kThreads) void gather_items_kernel(const float4* __restrict__ rec,
                                                                const uint32_t* __restrict__ vals_a,
                                                                const uint32_t* __restrict__ vals_b,
                                                                const uint32_t* __restrict__ range,
                                                                const uint32_t* __restrict__ v_ptr, uint32_t v_cap,
                                                                uint4* __restrict__ items,
                                                                uint32_t* __restrict__ counts) {
  const uint32_t n = read_count(v_ptr, v_cap);
  const uint32_t* __restrict__ sorted_vals = keys_narrow(range) ? vals_b : vals_a;   // where the depth sort ended
  const uint32_t step = gridDim.x * kThreads * kGatherIpt;
  for (uint32_t j0 = blockIdx.x * kThreads * kGatherIpt + threadIdx.x; j0 < n; j0 += step) {
    uint32_t p[kGatherIpt];
    float4 r2[kGatherIpt];
    // indices past the end repeat the last item (j0 < n), so every load is unconditional
#pragma unroll
    for (int u = 0; u < kGatherIpt; ++u) p[u] = sorted_vals[min(j0 + u * kThreads, n - 1u)];
#pragma unroll
    for (int u = 0; u < kGatherIpt; ++u) r2[u] = rec[3 * (size_t)p[u] + 2];
    auto put = [&](int u, uint32_t j) {
      const uint32_t a = __float_as_uint(r2[u].y), b = __float_as_uint(r2[u].z);
      items[j] = make_uint4(p[u], a, b, __float_as_uint(r2[u].w) & kFrameMask);
      counts[j] = ((b & 0xffffu) - (a & 0xffffu) + 1u) * ((b >> 16) - (a >> 16) + 1u);
    };
    // a block's whole round in range (all but the last) stores without per-lane tests, which
    // keeps the compiler from sinking loads into them
    if (j0 - threadIdx.x + kThreads * kGatherIpt <= n) {
#pragma unroll
      for (int u = 0; u < kGatherIpt; ++u) put(u, j0 + u * kThreads);
    } else {
#pragma unroll
      for (int u = 0; u < kGatherIpt; ++u)
        if (j0 + u * kThreads < n) put(u, j0 + u * kThreads);
    }
  }
}

__device__ __forceinline__ uint32_t wave_incl_max_u32(uint32_t v) {
  v = max(v, dpp_shift<0x111, 0xf>(v));
  v = max(v, dpp_shift<0x112, 0xf>(v));
  v = max(v, dpp_shift<0x114, 0xf>(v));
  v = max(v, dpp_shift<0x118, 0xf>(v));
  v = max(v, dpp_shift<0x142, 0xa>(v));
  v = max(v, dpp_shift<0x143, 0xc>(v));
  return v;
}

// Lanes whose digit equals this lane's (valid lanes only).  Digits are below kRadix, so
// all kRadixBits bits are compared whatever the pass's width (the bits above it are zero in
// every lane); the fixed count lets the loop unroll.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  const uint64_t v = __ballot(valid);
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
  for (int b = 0; b < kRadixBits; ++b) {
    const uint32_t t = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);   // all ones where the bit is set
    const uint64_t m = __ballot(t != 0u);
    lo &= ~((uint32_t)m ^ t);                  // lanes whose bit equals this lane's
    hi &= ~((uint32_t)(m >> 32) ^ t);
  }
  return valid ? ((uint64_t)hi << 32 | lo) : 0ull;
}

constexpr int kEmitItems = 1024;   // items per LDS tile of the emission
constexpr int kEIpt = kEmitItems / kThreads;

// Emission fused with the first digit pass of the tile sort.  The j-th depth-sorted kept
// pair p owns `count` consecutive output slots starting at its offset, holding (global tile,
// p) for its rectangle's tiles in row-major order.  Slots at or beyond `capacity` are
// dropped (overflow).  Two kernels over the same block segments of the items:
// emit_hist_kernel counts the low `nbits` bits of the slots' tile ids into each block's
// digit histogram (hist[d * G + b]); after that histogram has been scanned,
// emit_radix_kernel generates the slots, ranks them by digit and writes every entry
// straight to its place after the pass, so the unsorted list is never stored.

// The histogram needs no slots: a row of an item's rectangle holds the consecutive tile ids
// base + q tiles_x + [0, w), whose digits form a run of w consecutive values modulo 2^nbits,
// so each row adds one to a (wrapping) range of bins, kept as a difference array (two
// updates per row; rows of 2^nbits tiles or more add whole turns to every bin).  An item
// crossing `capacity` counts only its slots below it: whole rows, then the part of the next.
__global__ __launch_bounds__(kThreads) void emit_hist_kernel(const FrameDesc* __restrict__ descs,
                                                             const uint4* __restrict__ items,
                                                             const uint32_t* __restrict__ counts,
                                                             const uint32_t* __restrict__ v_ptr, uint32_t v_cap,
                                                             const uint64_t* __restrict__ partials, int G,
                                                             uint32_t capacity, int nbits, uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_tmp[kWaves];
  __shared__ int s_diff[kWaves][kRadix + 1];   // per wave; entry nb absorbs a range's end at nb
  __shared__ uint32_t s_turns[kWaves];         // per wave: added to every bin
  const uint32_t t = threadIdx.x;
  const int w = (int)(t >> 6);
  for (int k = (int)t; k < kWaves * (kRadix + 1); k += kThreads) (&s_diff[0][0])[k] = 0;
  if (t < kWaves) s_turns[t] = 0u;
  __syncthreads();
  const uint32_t n = read_count(v_ptr, v_cap);
  uint32_t begin, end;
  segment_of(n, G, blockIdx.x, begin, end);
  uint64_t base = partials[blockIdx.x];
  const uint32_t nb = 1u << nbits, mask = nb - 1u;
  const uint32_t i0 = t * kEIpt;
  for (uint32_t t0 = begin; t0 < end; t0 += kEmitItems) {
    uint32_t cn[kEIpt], sum = 0;
#pragma unroll
    for (int k = 0; k < kEIpt; ++k) {
      const uint32_t j = t0 + i0 + k;
      cn[k] = j < end ? counts[j] : 0u;
      sum += cn[k];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan(sum, s_tmp, &tot);
#pragma unroll
    for (int k = 0; k < kEIpt; ++k) {
      const uint64_t o = base + off;
      off += cn[k];
      if (cn[k] == 0u || o >= (uint64_t)capacity) continue;
      const uint32_t lim = (uint32_t)min((uint64_t)cn[k], (uint64_t)capacity - o);
      const uint4 it = items[t0 + i0 + k];
      const FrameDesc& d = descs[it.w];
      const uint32_t x0 = it.y & 0xffffu, y0 = it.y >> 16, x1 = it.z & 0xffffu;
      const uint32_t wd = x1 - x0 + 1u, txn = (uint32_t)d.tiles_x;
      const uint32_t rows = lim / wd, part = lim - rows * wd;
      uint32_t row0 = d.tile_base + y0 * txn + x0;
      for (uint32_t q = 0; q <= rows; ++q, row0 += txn) {
        const uint32_t width = q < rows ? wd : part;
        if (width == 0u) break;
        if (width >> nbits) atomicAdd(&s_turns[w], width >> nbits);
        const uint32_t r = width & mask;
        if (r == 0u) continue;
        const uint32_t a = row0 & mask, e = a + r;
        atomicAdd(&s_diff[w][a], 1);
        if (e <= nb) {
          atomicAdd(&s_diff[w][e], -1);
        } else {   // wraps: [a, nb) and [0, e - nb)
          atomicAdd(&s_diff[w][0], 1);
          atomicAdd(&s_diff[w][e - nb], -1);
        }
      }
    }
    base += tot;
  }
  __syncthreads();
  int v = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) v += s_diff[k][t];
  uint32_t turns = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) turns += s_turns[k];
  uint32_t dummy;
  const uint32_t incl = block_excl_scan((uint32_t)v, s_tmp, &dummy) + (uint32_t)v;   // running sum of the differences
  hist[(size_t)t * G + blockIdx.x] = t < nb ? incl + turns : 0u;
}

// The scatter: a block walks its items in tiles of 1024 (offsets and rectangles in LDS) and
// their slots in chunks of 2048: every item starting inside the chunk marks its first slot
// and a block-wide prefix maximum turns the marks into the owner of every slot; the chunk is
// ranked by digit (stable: slot order) and written to the places the scanned histogram gives.
__global__ __launch_bounds__(kThreads) void emit_radix_kernel(const FrameDesc* __restrict__ descs,
                                                              const uint4* __restrict__ items,
                                                              const uint32_t* __restrict__ counts,
                                                              const uint32_t* __restrict__ v_ptr, uint32_t v_cap,
                                                              const uint64_t* __restrict__ partials, int G,
                                                              uint32_t capacity, int nbits,
                                                              const uint32_t* __restrict__ hist,
                                                              uint32_t* __restrict__ keys,
                                                              uint32_t* __restrict__ vals) {
  __shared__ uint32_t s_tmp[kWaves];
  __shared__ uint32_t s_off[kEmitItems];    // exclusive slot offset of each item in the tile
  __shared__ uint32_t s_pair[kEmitItems];
  __shared__ uint32_t s_base[kEmitItems];   // global tile id of the rectangle's first tile
  __shared__ uint32_t s_shape[kEmitItems];  // rectangle width | tiles_x << 16
  __shared__ uint32_t s_own[kChunk];        // 1 + owning item of each slot; then sorted keys
  __shared__ uint32_t s_sval[kChunk];       // sorted values
  __shared__ uint32_t s_cnt[kWaves][kRadix];
  __shared__ uint32_t s_doff[kRadix];       // chunk-local start of each digit
  __shared__ uint32_t s_glob[kRadix];       // running global start of each digit
  const uint32_t n = read_count(v_ptr, v_cap);
  uint32_t begin, end;
  segment_of(n, G, blockIdx.x, begin, end);
  uint64_t base = partials[blockIdx.x];
  const uint32_t t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const uint32_t mask = (1u << nbits) - 1u;
  const uint64_t lt = lanemask_lt();
  s_glob[t] = hist[(size_t)t * G + blockIdx.x];
  __syncthreads();
  const uint32_t i0 = t * kEIpt;
  for (uint32_t t0 = begin; t0 < end; t0 += kEmitItems) {
    uint32_t cn[kEIpt];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kEIpt; ++k) {
      const uint32_t j = t0 + i0 + k;
      cn[k] = j < end ? counts[j] : 0u;
      uint32_t b = 0, shape = 1, p = 0;
      if (cn[k] > 0u) {
        const uint4 it = items[j];
        p = it.x;
        const FrameDesc& d = descs[it.w];
        const uint32_t x0 = it.y & 0xffffu, y0 = it.y >> 16, x1 = it.z & 0xffffu;
        b = d.tile_base + y0 * (uint32_t)d.tiles_x + x0;
        shape = (x1 - x0 + 1u) | ((uint32_t)d.tiles_x << 16);
      }
      s_pair[i0 + k] = p;
      s_base[i0 + k] = b;
      s_shape[i0 + k] = shape;
      sum += cn[k];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan(sum, s_tmp, &tot);
    uint32_t offs[kEIpt];
#pragma unroll
    for (int k = 0; k < kEIpt; ++k) {
      offs[k] = off;
      s_off[i0 + k] = off;
      off += cn[k];
    }
    uint32_t carry = 0;   // 1 + owner of the slot before the chunk
    for (uint32_t c0 = 0; c0 < tot; c0 += kChunk) {
#pragma unroll
      for (int k = 0; k < kChunk / kThreads; ++k) s_own[t * (kChunk / kThreads) + k] = 0u;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kEIpt; ++k)
        if (cn[k] > 0u && offs[k] >= c0 && offs[k] - c0 < (uint32_t)kChunk) s_own[offs[k] - c0] = i0 + k + 1u;
      __syncthreads();
      // block-wide inclusive prefix maximum of s_own (8 slots per thread)
      uint32_t v[kChunk / kThreads], m = 0;
#pragma unroll
      for (int k = 0; k < kChunk / kThreads; ++k) {
        m = max(m, s_own[t * (kChunk / kThreads) + k]);
        v[k] = m;
      }
      const uint32_t wincl = wave_incl_max_u32(m);
      if (lane == 63) s_tmp[w] = wincl;
      const uint32_t wexcl = __shfl_up(wincl, 1) * (lane > 0 ? 1u : 0u);
      __syncthreads();
      uint32_t pre = carry;
#pragma unroll
      for (int k = 0; k < kWaves; ++k)
        if (k < w) pre = max(pre, s_tmp[k]);
      pre = max(pre, wexcl);
#pragma unroll
      for (int k = 0; k < kChunk / kThreads; ++k) s_own[t * (kChunk / kThreads) + k] = max(pre, v[k]);
      __syncthreads();
      carry = s_own[kChunk - 1];
      // the chunk's slots below capacity; thread slots in wave-major order for a stable rank
      const uint32_t nslot = min((uint32_t)kChunk, tot - c0);
      const uint64_t g0 = base + c0;
      const uint32_t nvalid = g0 >= capacity ? 0u : (uint32_t)min((uint64_t)nslot, (uint64_t)capacity - g0);
      constexpr int kR = kChunk / kThreads;   // 8 slots per thread
      uint32_t key[kR], val[kR];
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        const uint32_t sl = (uint32_t)(w * (kChunk / kWaves) + r * 64 + lane);
        key[r] = 0u;
        val[r] = 0u;
        if (sl < nvalid) {
          const uint32_t i = s_own[sl] - 1u;
          const uint32_t local = c0 + sl - s_off[i];
          const uint32_t shape = s_shape[i];
          const uint32_t wd = shape & 0xffffu, txn = shape >> 16;
          uint32_t q = (uint32_t)((float)local * __builtin_amdgcn_rcpf((float)wd));
          if (q * wd > local) --q;
          else if ((q + 1u) * wd <= local) ++q;
          key[r] = s_base[i] + q * txn + (local - q * wd);
          val[r] = s_pair[i];
        }
      }
      {
#pragma unroll
        for (int k = 0; k < kWaves; ++k) s_cnt[k][t] = 0u;
        __syncthreads();   // also: every thread has read its owners and the carry
        uint32_t rank[kR];
#pragma unroll
        for (int r = 0; r < kR; ++r) {
          const uint32_t sl = (uint32_t)(w * (kChunk / kWaves) + r * 64 + lane);
          const bool valid = sl < nvalid;
          const uint32_t d = key[r] & mask;
          const uint64_t peers = match_digit(d, valid);
          const uint32_t below = (uint32_t)__popcll(peers & lt);
          const uint32_t old = valid ? s_cnt[w][d] : 0u;
          if (valid && below == 0u) s_cnt[w][d] = old + (uint32_t)__popcll(peers);
          rank[r] = valid ? old + below : 0xffffffffu;
        }
        __syncthreads();
        uint32_t c[kWaves], dtot = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) {
          c[k] = s_cnt[k][t];
          dtot += c[k];
        }
        uint32_t dummy;
        const uint32_t excl = block_excl_scan(dtot, s_tmp, &dummy);
        s_doff[t] = excl;
        uint32_t run = excl;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) {
          s_cnt[k][t] = run;
          run += c[k];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kR; ++r) {
          if (rank[r] != 0xffffffffu) {
            const uint32_t pos = s_cnt[w][key[r] & mask] + rank[r];
            s_own[pos] = key[r];
            s_sval[pos] = val[r];
          }
        }
        __syncthreads();
        for (uint32_t i = t; i < nvalid; i += kThreads) {
          const uint32_t k2 = s_own[i];
          const uint32_t d = k2 & mask;
          const uint32_t g = s_glob[d] + (i - s_doff[d]);
          keys[g] = k2;
          vals[g] = s_sval[i];
        }
        __syncthreads();
        s_glob[t] += dtot;
        __syncthreads();
      }
    }
    base += tot;
    __syncthreads();
  }
}

// In-place exclusive scan of `data` (downsweep of the kRaw reduce-then-scan).
__global__ __launch_bounds__(kThreads) void hist_scan_down_kernel(uint32_t* __restrict__ data, uint32_t n,
                                                                  const uint64_t* __restrict__ partials, int G) {
  __shared__ uint32_t s_tmp[kWaves];
  uint32_t begin, end;
  segment_of(n, G, blockIdx.x, begin, end);
  uint64_t base = partials[blockIdx.x];
  for (uint32_t t0 = begin; t0 < end; t0 += kTileItems) {
    const uint32_t i0 = t0 + threadIdx.x * kIpt;
    uint32_t v[kIpt], s = 0;
#pragma unroll
    for (int k = 0; k < kIpt; ++k) {
      v[k] = (i0 + k < end) ? data[i0 + k] : 0u;
      s += v[k];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan(s, s_tmp, &tot);
#pragma unroll
    for (int k = 0; k < kIpt; ++k) {
      if (i0 + k < end) data[i0 + k] = (uint32_t)(base + off);
      off += v[k];
    }
    base += tot;
  }
}

// ------------------------------------------------------------------------------ radix sort

// Per-block digit histogram of its segment, hist[d * G + b], counted with per-wave LDS
// atomics (a skewed digit serialises one wave's atomics, which stays cheap).  Digits are
// those of key - key_base(range); with skip_narrow the pass does nothing on narrow keys.
__global__ __launch_bounds__(kThreads) void rs_upsweep_kernel(const uint32_t* __restrict__ keys,
                                                              const uint32_t* n_ptr, uint32_t n_cap, int shift,
                                                              int nbits, uint32_t* __restrict__ hist, int G,
                                                              const uint32_t* range, int skip_narrow) {
  if (skip_narrow && keys_narrow(range)) return;
  __shared__ uint32_t s_h[kWaves][kRadix];
  for (int k = threadIdx.x; k < kWaves * kRadix; k += kThreads) (&s_h[0][0])[k] = 0u;
  __syncthreads();
  const uint32_t n = read_count(n_ptr, n_cap);
  uint32_t begin, end;
  segment_of<kSortTile>(n, G, blockIdx.x, begin, end);
  const int w = threadIdx.x >> 6;
  const uint32_t mask = (1u << nbits) - 1u;
  const uint32_t kb = key_base(range);
  // segments start at multiples of kSortTile, so the 4-key vector loads are aligned
  const uint32_t nvec = (end - begin) / 4;
  for (uint32_t v = threadIdx.x; v < nvec; v += kThreads) {
    const uint4 k4 = *reinterpret_cast<const uint4*>(keys + begin + 4 * v);
    atomicAdd(&s_h[w][((k4.x - kb) >> shift) & mask], 1u);
    atomicAdd(&s_h[w][((k4.y - kb) >> shift) & mask], 1u);
    atomicAdd(&s_h[w][((k4.z - kb) >> shift) & mask], 1u);
    atomicAdd(&s_h[w][((k4.w - kb) >> shift) & mask], 1u);
  }
  const uint32_t tail = begin + 4 * nvec + threadIdx.x;
  if (tail < end) atomicAdd(&s_h[w][((keys[tail] - kb) >> shift) & mask], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d < kRadix; d += kThreads) {
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) c += s_h[k][d];
    hist[(size_t)d * G + blockIdx.x] = c;
  }
}

// Stable scatter of one digit pass.  Each tile of 4096 items is ranked in LDS (per-wave
// digit counters updated by the lowest lane of each equal-digit group), reordered by digit
// in LDS, and written out so that equal digits land in consecutive global slots (kout NULL:
// values only).  The next tile's keys and values are loaded while the current one is
// scanned and scattered.
__global__ __launch_bounds__(kThreads) void rs_downsweep_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* n_ptr, uint32_t n_cap, int shift, int nbits,
    const uint32_t* __restrict__ hist, int G, const uint32_t* range, int skip_narrow) {
  if (skip_narrow && keys_narrow(range)) return;
  __shared__ uint32_t s_cnt[kWaves][kRadix];
  __shared__ uint32_t s_off[kRadix];
  __shared__ uint32_t s_glob[kRadix];
  __shared__ uint32_t s_keys[kSortTile];
  __shared__ uint32_t s_vals[kSortTile];
  __shared__ uint32_t s_tmp[kWaves];
  const uint32_t n = read_count(n_ptr, n_cap);
  uint32_t begin, end;
  segment_of<kSortTile>(n, G, blockIdx.x, begin, end);
  if (begin >= end) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const uint32_t mask = (1u << nbits) - 1u;
  const uint32_t kb = key_base(range);
  const uint64_t lt = lanemask_lt();
  s_glob[t] = hist[(size_t)t * G + blockIdx.x];
  uint32_t key[kSortIpt], val[kSortIpt];
#pragma unroll
  for (int r = 0; r < kSortIpt; ++r) {
    const uint32_t i = begin + (uint32_t)(w * (kSortTile / kWaves) + r * 64 + lane);
    const bool valid = i < end;
    key[r] = valid ? kin[i] : 0u;
    val[r] = valid ? vin[i] : 0u;
  }
  for (uint32_t t0 = begin; t0 < end; t0 += kSortTile) {
    for (int k = t; k < kWaves * kRadix; k += kThreads) (&s_cnt[0][0])[k] = 0u;
    __syncthreads();
    uint32_t rank[kSortIpt];
#pragma unroll
    for (int r = 0; r < kSortIpt; ++r) {
      const uint32_t i = t0 + (uint32_t)(w * (kSortTile / kWaves) + r * 64 + lane);
      const bool valid = i < end;
      const uint32_t d = ((key[r] - kb) >> shift) & mask;
      const uint64_t peers = match_digit(d, valid);
      const uint32_t below = (uint32_t)__popcll(peers & lt);
      const uint32_t old = valid ? s_cnt[w][d] : 0u;
      if (valid && below == 0u) s_cnt[w][d] = old + (uint32_t)__popcll(peers);
      rank[r] = valid ? old + below : 0xffffffffu;
    }
    __syncthreads();
    // the next tile's keys and values, in flight during this tile's scan and scatters
    uint32_t nkey[kSortIpt], nval[kSortIpt];
#pragma unroll
    for (int r = 0; r < kSortIpt; ++r) {
      const uint32_t i = t0 + kSortTile + (uint32_t)(w * (kSortTile / kWaves) + r * 64 + lane);
      const bool valid = i < end;
      nkey[r] = valid ? kin[i] : 0u;
      nval[r] = valid ? vin[i] : 0u;
    }
    uint32_t c[kWaves], tot = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
      c[k] = s_cnt[k][t];
      tot += c[k];
    }
    uint32_t dummy;
    const uint32_t excl = block_excl_scan(tot, s_tmp, &dummy);
    s_off[t] = excl;
    uint32_t run = excl;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
      s_cnt[k][t] = run;
      run += c[k];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortIpt; ++r) {
      if (rank[r] != 0xffffffffu) {
        const uint32_t d = ((key[r] - kb) >> shift) & mask;
        const uint32_t pos = s_cnt[w][d] + rank[r];
        s_keys[pos] = key[r];
        s_vals[pos] = val[r];
      }
    }
    __syncthreads();
    const uint32_t nt = min((uint32_t)kSortTile, end - t0);
    for (uint32_t i = t; i < nt; i += kThreads) {
      const uint32_t k2 = s_keys[i];
      const uint32_t d = ((k2 - kb) >> shift) & mask;
      const uint32_t g = s_glob[d] + (i - s_off[d]);
      if (kout) kout[g] = k2;
      vout[g] = s_vals[i];
    }
    __syncthreads();
    s_glob[t] += tot;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortIpt; ++r) {
      key[r] = nkey[r];
      val[r] = nval[r];
    }
  }
}

// ------------------------------------------------------------------------------ misc

__global__ void finalize_kernel(uint32_t* counters, uint32_t capacity) {
  const uint64_t e = (uint64_t)counters[1] | ((uint64_t)counters[2] << 32);
  counters[3] = e > (uint64_t)capacity ? 1u : 0u;
  counters[4] = e > (uint64_t)capacity ? capacity : (uint32_t)e;   // entries actually written
}

// dst[0] = entries E, dst[1] = overflow flag (one thread; for a later, batched read).
__global__ void status_kernel(const uint32_t* __restrict__ counters, int64_t* __restrict__ dst) {
  dst[0] = (int64_t)((uint64_t)counters[1] | ((uint64_t)counters[2] << 32));
  dst[1] = (int64_t)counters[3];
}

// Per-tile [start, end) from the boundaries of the sorted keys; each thread takes 4
// consecutive keys (one vector load) and compares them with its neighbours', which come
// from the adjacent lanes (the wave's edge lanes load theirs).
__global__ __launch_bounds__(kThreads) void ranges_kernel(const uint32_t* __restrict__ keys,
                                                          const uint32_t* __restrict__ e_ptr, uint32_t capacity,
                                                          uint32_t* __restrict__ ranges) {
  const uint32_t E = read_count(e_ptr, capacity);
  const uint32_t nq = (E + 3) / 4;
  const int lane = threadIdx.x & 63;
  // the loop runs the same number of times in every lane of a wave, so the shuffles see
  // their neighbours (lanes past the end carry sentinels)
  const uint32_t stride = gridDim.x * kThreads;
  const uint32_t q0 = blockIdx.x * kThreads + threadIdx.x;
  const uint32_t wave_q0 = q0 - (uint32_t)lane;
  for (uint32_t wq = wave_q0; wq < nq; wq += stride) {
    const uint32_t q = wq + (uint32_t)lane;
    const uint32_t j0 = 4 * q;
    uint32_t k[6];
    if (j0 + 3 < E) {
      const uint4 v = *reinterpret_cast<const uint4*>(keys + j0);
      k[1] = v.x; k[2] = v.y; k[3] = v.z; k[4] = v.w;
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) k[1 + i] = j0 + i < E ? keys[j0 + i] : 0xffffffffu;
    }
    const uint32_t up = (uint32_t)__shfl_up((int)k[4], 1);     // lane - 1's last key
    const uint32_t down = (uint32_t)__shfl_down((int)k[1], 1);   // lane + 1's first key
    k[0] = lane > 0 ? up : (j0 > 0 && j0 - 1 < E ? keys[j0 - 1] : 0xffffffffu);
    k[5] = lane < 63 ? (j0 + 4 < E ? down : 0xffffffffu) : (j0 + 4 < E ? keys[j0 + 4] : 0xffffffffu);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t j = j0 + i;
      if (j >= E) break;
      if (k[i] != k[i + 1]) ranges[2 * (size_t)k[i + 1]] = j;
      if (k[i + 2] != k[i + 1] || j + 1 == E) ranges[2 * (size_t)k[i + 1] + 1] = j + 1;
    }
  }
}

// 16-byte stores where the buffer is 16-byte aligned (four words per lane and instruction).
__global__ __launch_bounds__(kThreads) void fill_kernel(uint32_t* __restrict__ dst, int64_t count, uint32_t value) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  int64_t head = 0;
  if ((reinterpret_cast<uintptr_t>(dst) & 15u) == 0) {
    const int64_t n4 = count >> 2;
    const uint4 v = make_uint4(value, value, value, value);
    uint4* d4 = reinterpret_cast<uint4*>(dst);
    for (int64_t i = t; i < n4; i += stride) d4[i] = v;
    head = 4 * n4;
  }
  for (int64_t i = head + t; i < count; i += stride) dst[i] = value;
}

int blocks_for(int64_t n, int items_per_block, int max_blocks) {
  int64_t b = (n + items_per_block - 1) / items_per_block;
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return (int)b;
}

int scan_blocks(int64_t n) { return blocks_for(n, 2 * kTileItems, kMaxScanBlocks); }
int sort_blocks(int64_t n) { return blocks_for(n, 2 * kSortTile, kMaxSortBlocks); }

// LSD radix sort of (key, val) over bits [first_bit, bits): ping-pongs between (k0,v0) and
// (k1,v1); the result ends in (k0,v0) when the number of passes is even, else in (k1,v1).
// Without final_keys the last pass writes only the values (its keys are not needed).
// With `range` (depth keys) the digits are those of key - the smallest key, and the passes
// from bit 24 on do nothing when the keys are narrow (the result then ends in the buffers
// of the last pass that ran).
hipError_t radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, const uint32_t* n_ptr, uint32_t n_cap,
                      int bits, uint32_t* hist, uint64_t* partials, hipStream_t stream, int first_bit = 0,
                      bool final_keys = true, const uint32_t* range = nullptr) {
  const int G = sort_blocks(n_cap);
  uint32_t *ki = k0, *vi = v0, *ko = k1, *vo = v1;
  for (int shift = first_bit; shift < bits; shift += kRadixBits) {
    const bool last = shift + kRadixBits >= bits;
    const int nb = min(kRadixBits, bits - shift);
    const int skip = range && shift >= 24 ? 1 : 0;
    hipLaunchKernelGGL(rs_upsweep_kernel, dim3(G), dim3(kThreads), 0, stream, ki, n_ptr, n_cap, shift, nb, hist, G,
                       range, skip);
    // exclusive scan of the digit-major histogram (kRadix * G values)
    const uint32_t hn = (uint32_t)(kRadix * G);
    const int Gs = scan_blocks(hn);
    ScanSrc src{nullptr, hist};
    hipLaunchKernelGGL(scan_reduce_kernel<kRaw>, dim3(Gs), dim3(kThreads), 0, stream, src, nullptr, hn, partials, Gs);
    hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(1024), 0, stream, partials, Gs, nullptr, nullptr);
    hipLaunchKernelGGL(hist_scan_down_kernel, dim3(Gs), dim3(kThreads), 0, stream, hist, hn, partials, Gs);
    hipLaunchKernelGGL(rs_downsweep_kernel, dim3(G), dim3(kThreads), 0, stream, ki, vi,
                       (last && !final_keys) ? nullptr : ko, vo, n_ptr, n_cap, shift, nb, hist, G, range, skip);
    uint32_t* tk = ki; ki = ko; ko = tk;
    uint32_t* tv = vi; vi = vo; vo = tv;
  }
  return hipGetLastError();
}

}  // namespace

// Binning scratch of veg_bin_static, for callers that cannot allocate: one copy per GPU,
// held until the process ends.  Host code never uses this name as an address (on the host
// it is only a stand-in for the symbol); static_bin_scratch looks up each device's copy.
static __device__ __align__(256) unsigned char scratch[kStaticBinBytes];

hipError_t static_bin_scratch(void** out) {
  static std::mutex mu;
  static void* ptrs[kStaticBinMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kStaticBinMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!ptrs[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // the current device's copy
    if (e != hipSuccess) return e;
    ptrs[dev] = p;
  }
  *out = ptrs[dev];
  return hipSuccess;
}

size_t bin_ws_bytes(int64_t pairs) {
  const size_t p = (size_t)(pairs > 0 ? pairs : 1);
  size_t b = 0;
  b += 4 * p * sizeof(uint32_t);                       // depth-sort ping-pong
  b += p * 16;                                         // depth-sorted item records
  b += kMaxScanBlocks * sizeof(uint64_t);              // scan partials (entry offsets)
  b += kMaxScanBlocks * sizeof(uint64_t);              // scan partials (scratch)
  b += (size_t)kRadix * kMaxHistBlocks * sizeof(uint32_t);  // radix histograms
  b += 64 * sizeof(uint32_t);                          // counters
  return b + 10 * 256;                                 // alignment slack
}

void carve_bin_ws(void* ws, int64_t pairs, BinWs* out) {
  const size_t p = (size_t)(pairs > 0 ? pairs : 1);
  uintptr_t a = ((uintptr_t)ws + 255) & ~(uintptr_t)255;
  auto take = [&](size_t bytes) {
    void* r = (void*)a;
    a = (a + bytes + 255) & ~(uintptr_t)255;
    return r;
  };
  // counters first: their offset does not depend on the pair count
  out->counters = (uint32_t*)take(64 * 4);
  out->partials = (uint32_t*)take(kMaxScanBlocks * 8);
  out->partials_tmp = (uint32_t*)take(kMaxScanBlocks * 8);
  out->hist = (uint32_t*)take((size_t)kRadix * kMaxHistBlocks * 4);
  out->dkeyA = (uint32_t*)take(p * 4);
  out->dvalA = (uint32_t*)take(p * 4);
  out->dkeyB = (uint32_t*)take(p * 4);
  out->dvalB = (uint32_t*)take(p * 4);
  out->items = (uint32_t*)take(p * 16);
}

hipError_t launch_bin_count(const float4* rec, const uint32_t* count, const uint32_t* depth, uint32_t n_pairs,
                            const BinWs& ws, hipStream_t stream, const uint32_t* n_pairs_dev, uint32_t list_n,
                            int per_view) {
  uint64_t* partials = (uint64_t*)ws.partials;
  uint64_t* ptmp = (uint64_t*)ws.partials_tmp;
  // the slots the compaction walks: only list owners' when views share lists
  ListMap lm{0u, 0u, 0.0};
  uint32_t n_slots = n_pairs;
  if (per_view > 1) {
    if (n_pairs_dev || list_n == 0u || n_pairs % ((uint64_t)list_n * (uint32_t)per_view) != 0u)
      return hipErrorInvalidValue;
    lm = ListMap{list_n, (uint32_t)(per_view - 1) * list_n, 1.0 / (double)list_n};
    n_slots = n_pairs / (uint32_t)per_view;
  }
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(kThreads), 0, stream, ws.counters, (int64_t)64, 0u);
  // 1. compaction of kept pairs
  const int Gv = scan_blocks(n_slots);
  ScanSrc vis{count, nullptr};
  hipLaunchKernelGGL(scan_reduce_kernel<kVis>, dim3(Gv), dim3(kThreads), 0, stream, vis, n_pairs_dev, n_slots, ptmp,
                     Gv, lm);
  hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(1024), 0, stream, ptmp, Gv, ws.counters + 8,
                     ws.counters + 0);
  // (the blocks' depth-key extremes go through the radix histogram area, free until the sort)
  hipLaunchKernelGGL(compact_kernel, dim3(Gv), dim3(kThreads), 0, stream, count, depth, n_pairs_dev, n_slots, ptmp,
                     Gv, ws.dkeyA, ws.dvalA, lm, ws.hist);
  hipLaunchKernelGGL(key_range_kernel, dim3(1), dim3(1024), 0, stream, ws.hist, Gv, ws.counters + kDepthRange);
  // 2. front-to-back order: 31 depth-key bits (camera z > 0)
  hipError_t e = radix_sort(ws.dkeyA, ws.dvalA, ws.dkeyB, ws.dvalB, ws.counters + 0, n_pairs, 31, ws.hist, ptmp,
                            stream, 0, false, ws.counters + kDepthRange);
  if (e != hipSuccess) return e;
  // 4 passes: the sorted values are back in dvalA (the sorted keys are not kept), or in dvalB
  // when the fourth pass was skipped on narrow keys
  // 3. item records and tile counts in that order (counts reuse dkeyB)
  hipLaunchKernelGGL(gather_items_kernel, dim3(blocks_for(n_pairs, kThreads * kGatherIpt, 8192)), dim3(kThreads), 0, stream,
                     (const float4*)rec, ws.dvalA, ws.dvalB, ws.counters + kDepthRange, ws.counters + 0, n_pairs,
                     (uint4*)ws.items, ws.dkeyB);
  // 4. entry offsets in that order; block offsets stay in `partials` for the emission
  const int Gc = scan_blocks(n_pairs);
  ScanSrc cnt{nullptr, ws.dkeyB};
  hipLaunchKernelGGL(scan_reduce_kernel<kCnt>, dim3(Gc), dim3(kThreads), 0, stream, cnt, ws.counters + 0, n_pairs,
                     partials, Gc);
  hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(1024), 0, stream, partials, Gc, ws.counters + 1, nullptr);
  return hipGetLastError();
}

int tile_bits(uint32_t total_tiles) {
  int b = 0;
  while (b < 32 && ((uint64_t)1 << b) < (uint64_t)total_tiles) ++b;
  return b;
}

hipError_t launch_bin_sort(const FrameDesc* descs, int n_frames, const float4* rec, const uint32_t* count,
                           uint32_t n_pairs, uint32_t total_tiles, const BinWs& ws, uint32_t* keys, uint32_t* vals,
                           uint32_t* keys_alt, uint32_t* vals_alt, uint32_t* ranges, uint32_t capacity,
                           hipStream_t stream) {
  (void)n_frames;
  uint64_t* partials = (uint64_t*)ws.partials;
  uint64_t* ptmp = (uint64_t*)ws.partials_tmp;
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(1), 0, stream, ws.counters, capacity);
  const int bits = tile_bits(total_tiles);
  const int nb0 = bits < kRadixBits ? bits : kRadixBits;   // bits of the fused first pass
  const int passes = 1 + (bits > nb0 ? (bits - nb0 + kRadixBits - 1) / kRadixBits : 0);
  // the fused pass writes (ek, ev); each later pass flips buffers; the result ends in keys
  uint32_t* ek = (passes % 2) ? keys : keys_alt;
  uint32_t* ev = (passes % 2) ? vals : vals_alt;
  uint32_t* ok = (passes % 2) ? keys_alt : keys;
  uint32_t* ov = (passes % 2) ? vals_alt : vals;
  const int Gc = scan_blocks(n_pairs);
  if (capacity > 0) {
    hipLaunchKernelGGL(emit_hist_kernel, dim3(Gc), dim3(kThreads), 0, stream, descs, (const uint4*)ws.items,
                       ws.dkeyB, ws.counters + 0, n_pairs, partials, Gc, capacity, nb0, ws.hist);
    const uint32_t hn = (uint32_t)(kRadix * Gc);
    const int Gs = scan_blocks(hn);
    ScanSrc src{nullptr, ws.hist};
    hipLaunchKernelGGL(scan_reduce_kernel<kRaw>, dim3(Gs), dim3(kThreads), 0, stream, src, nullptr, hn, ptmp, Gs);
    hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(1024), 0, stream, ptmp, Gs, nullptr, nullptr);
    hipLaunchKernelGGL(hist_scan_down_kernel, dim3(Gs), dim3(kThreads), 0, stream, ws.hist, hn, ptmp, Gs);
    hipLaunchKernelGGL(emit_radix_kernel, dim3(Gc), dim3(kThreads), 0, stream, descs, (const uint4*)ws.items,
                       ws.dkeyB, ws.counters + 0, n_pairs, partials, Gc, capacity, nb0, ws.hist, ek, ev);
    if (passes > 1) {
      hipError_t e = radix_sort(ek, ev, ok, ov, ws.counters + 4, capacity, bits, ws.hist, ptmp, stream, nb0);
      if (e != hipSuccess) return e;
    }
  }
  const int64_t rn = 2 * (int64_t)total_tiles;
  hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(rn, kThreads * 4, 4096)), dim3(kThreads), 0, stream, ranges, rn,
                     0u);
  if (capacity > 0)
    hipLaunchKernelGGL(ranges_kernel, dim3(blocks_for(capacity, kThreads * 4, 8192)), dim3(kThreads), 0, stream,
                       keys, ws.counters + 4, capacity, ranges);
  return hipGetLastError();
}

hipError_t launch_bin_status(const uint32_t* counters, int64_t* dst, hipStream_t stream) {
  hipLaunchKernelGGL(status_kernel, dim3(1), dim3(1), 0, stream, counters, dst);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* dst, int64_t count, uint32_t value, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(count, kThreads * 4, 8192)), dim3(kThreads), 0, stream, dst, count,
                     value);
  return hipGetLastError();
}

}  // namespace veg
