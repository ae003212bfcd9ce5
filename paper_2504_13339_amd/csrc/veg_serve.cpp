// Continuous-batching render server.
//
// Resident models stay in device memory (caller-owned SoA).  A scheduler thread keeps a
// FIFO of submitted requests; whenever a batch slot is free it takes requests from the
// head of the queue while they fit the slot (requests, pairs, estimated key-list entries,
// resolution) and the HBM admission budget, writes one frame descriptor per request
// (model pointers, camera, TF table, output image) through pinned staging memory, and
// launches projection -> binning -> sorting -> blending for the whole batch on the slot's
// stream, optionally as one replay of a hipGraph.  Kernels take every size from the
// device descriptors and use their launch sizes only as bounds, so one capture serves
// every batch of a shape: the request count and power-of-two bounds on the tiles of its
// largest frame, the Gaussians of its largest model, its pairs and its estimated entries.
// Each slot keeps the graphs of the shapes it has seen (least recently used dropped first),
// so a batch of small requests launches small grids.  Slots run concurrently, so requests
// that arrive while batches are on the GPU are admitted as soon as a slot and budget free
// up.  Completion is observed through the slot's event; a batch whose key list overflowed
// its bound is re-run request by request with the observed entry count as the bound.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include <sys/prctl.h>

#include "veg_internal.h"

namespace veg {
namespace {

using Clock = std::chrono::steady_clock;
double now_s() { return std::chrono::duration<double>(Clock::now().time_since_epoch()).count(); }

struct BatchHeader {
  uint32_t n_pairs;
  uint32_t n_frames;
  uint32_t pad[62];   // keeps the descriptors 256-byte aligned after the header
};
static_assert(sizeof(BatchHeader) == 256, "header size");

struct Req {
  uint64_t id = 0;
  veg_request r{};
  std::vector<float> tf;
  int32_t state = VEG_REQ_QUEUED;
  veg_status status = VEG_OK;
  double t_submit = 0, t_done = 0;
  int64_t n = 0;
  int64_t est_entries = 0;
  int64_t est_bytes = 0;
  int64_t known_entries = 0;   // observed entry count bound after an overflow (0: none)
  bool solo = false;
};

// Launch bounds of a batch; every kernel of the pipeline is launched for these sizes.
struct Shape {
  int frames = 0;          // requests in the batch
  int tiles = 0;           // tiles of its largest frame (power of two, capped)
  int n_max = 0;           // Gaussians of its largest model (power of two, capped)
  uint32_t pairs = 0;      // (frame, Gaussian) pairs (power of two, capped)
  uint32_t entries = 0;    // key-list entries (power of two, capped)
  bool operator==(const Shape& o) const {
    return frames == o.frames && tiles == o.tiles && n_max == o.n_max && pairs == o.pairs && entries == o.entries;
  }
};

struct GraphEntry {
  Shape shape;
  KOpts opts{};
  hipGraphExec_t exec = nullptr;
  uint64_t last_use = 0;
};

constexpr size_t kGraphsPerSlot = 48;

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  // device (carved from the arena)
  BatchHeader* d_header = nullptr;
  FrameDesc* d_descs = nullptr;
  float* d_luts = nullptr;
  float4* rec = nullptr;
  uint32_t* count = nullptr;
  uint32_t* depth = nullptr;
  void* ws = nullptr;
  BinWs bws{};
  uint32_t *keys = nullptr, *vals = nullptr, *keys_alt = nullptr, *vals_alt = nullptr, *ranges = nullptr;
  // pinned host staging
  unsigned char* h_stage = nullptr;   // header + descriptors
  float* h_luts = nullptr;
  uint32_t* h_counters = nullptr;
  // graphs, one per batch shape and options
  std::vector<GraphEntry> graphs;
  uint64_t uses = 0;
  // state
  bool busy = false;
  std::vector<uint64_t> reqs;
  double t_launch = 0;
  int64_t bytes = 0;
  int64_t est_entries = 0;
  uint32_t entries_bound = 0;   // key-list bound the running batch was launched with
};

bool same_opts(const veg_opts& a, const veg_opts& b) {
  return a.alpha_clamp == b.alpha_clamp && a.alpha_min == b.alpha_min && a.t_min == b.t_min &&
         a.lowpass == b.lowpass && a.near_z == b.near_z && a.guard == b.guard;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t header, descs, luts, rec, count, depth, ws, keys, ranges, total;
};

}  // namespace
}  // namespace veg

using namespace veg;

struct veg_server {
  veg_serve_config cfg{};
  int device = 0;
  int64_t pairs_cap = 0, entries_cap = 0;
  int max_tiles_frame = 0;
  uint32_t total_tiles_cap = 0;
  std::mutex mu;
  std::condition_variable cv;        // scheduler wake-up
  std::condition_variable cv_done;   // request completion
  std::vector<veg_gaussians> models;
  std::unordered_map<uint64_t, Req> reqs;
  std::deque<uint64_t> queue;
  std::vector<Slot> slots;
  std::thread sched;
  bool stop = false;
  uint64_t next_id = 1;
  int64_t in_use = 0, peak = 0;
  std::vector<double> m_scale;   // per model: learned multiplier on the entry-count prior
  std::string err;
  // statistics
  std::vector<double> lat_ms;
  int64_t submitted = 0, completed = 0, failed = 0, rejected = 0, batches = 0, retries = 0, graphs_captured = 0;
  double sum_batch = 0, pix_done = 0, first_submit = -1, last_done = -1;
  double busy_acc = 0, busy_since = -1;
  int inflight = 0;
};

namespace {

veg_status sfail(veg_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  set_last_error(buf);
  return s;
}

int64_t pairs_cap_of(const veg_serve_config& c) {
  return c.max_pairs > 0 ? c.max_pairs : (int64_t)c.max_batch * c.max_gaussians;
}

int tiles_of(int w, int h) { return ((w + kTile - 1) / kTile) * ((h + kTile - 1) / kTile); }

Layout slot_layout(const veg_serve_config& c) {
  Layout L{};
  const int64_t P = pairs_cap_of(c);
  const int tiles = c.max_batch * tiles_of(c.max_width, c.max_height);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.header = take(sizeof(BatchHeader));
  L.descs = take((size_t)c.max_batch * sizeof(FrameDesc));
  L.luts = take((size_t)c.max_batch * c.max_tf_k * 4 * sizeof(float));
  L.rec = take((size_t)P * 12 * sizeof(float));
  L.count = take((size_t)P * 4);
  L.depth = take((size_t)P * 4);
  L.ws = take(bin_ws_bytes(P));
  L.keys = take((size_t)c.max_entries * 4 * 4);
  L.ranges = take((size_t)tiles * 8);
  L.total = off;
  return L;
}

veg_status check_cfg(const veg_serve_config* c) {
  if (!c) return sfail(VEG_ERR_INVALID_ARG, "config is NULL");
  if (c->max_batch < 1 || c->max_batch > 64) return sfail(VEG_ERR_INVALID_ARG, "max_batch must be 1..64");
  if (c->n_streams < 1 || c->n_streams > 8) return sfail(VEG_ERR_INVALID_ARG, "n_streams must be 1..8");
  if (c->max_width < 1 || c->max_height < 1 || c->max_width > VEG_MAX_DIM || c->max_height > VEG_MAX_DIM)
    return sfail(VEG_ERR_INVALID_ARG, "max_width/max_height out of range");
  if (c->max_tf_k < 2 || c->max_tf_k > 4096) return sfail(VEG_ERR_INVALID_ARG, "max_tf_k must be 2..4096");
  if (c->max_gaussians < 1 || c->max_gaussians >= ((int64_t)1 << 31))
    return sfail(VEG_ERR_INVALID_ARG, "max_gaussians out of range");
  const int64_t P = pairs_cap_of(*c);
  if (P < c->max_gaussians || P >= ((int64_t)1 << 31)) return sfail(VEG_ERR_INVALID_ARG, "max_pairs out of range");
  if (c->max_entries < 1 || c->max_entries >= ((int64_t)1 << 31))
    return sfail(VEG_ERR_INVALID_ARG, "max_entries out of range");
  if ((int64_t)c->max_batch * tiles_of(c->max_width, c->max_height) >= ((int64_t)1 << 31))
    return sfail(VEG_ERR_INVALID_ARG, "too many tiles per batch");
  return VEG_OK;
}

KOpts kopts_of(const veg_opts& o) {
  KOpts k;
  k.alpha_clamp = o.alpha_clamp;
  k.alpha_min = o.alpha_min;
  k.t_min = o.t_min;
  k.lowpass = o.lowpass;
  k.near_z = o.near_z;
  k.guard = o.guard;
  k.log2_alpha_min = std::log2(o.alpha_min);
  k.bg0 = k.bg1 = k.bg2 = 0.0f;   // the background is per request, in the frame descriptors
  return k;
}

// Entry-count prior for one request: about (1 + extent/16)^2 tiles per Gaussian, with the
// extent taken proportional to the image height; scaled by the model's learned multiplier.
int64_t entry_prior(int64_t n, int W, int H) {
  const double f = std::max(1.0, (double)std::max(W, H) / 1024.0);
  return (int64_t)std::ceil((double)n * 6.0 * f * f) + 1024;
}

// Predicted key-list entries of a request: the count observed after an overflow, else the
// prior times its model's learned multiplier.
int64_t predicted_entries(const veg_server* s, const Req& q) {
  if (q.known_entries > 0) return q.known_entries;
  return (int64_t)std::ceil((double)q.est_entries * s->m_scale[(size_t)q.r.model_id]);
}

int64_t req_bytes(int64_t n, int64_t entries, int W, int H) {
  return n * (48 + 8 + 16) + entries * 16 + (int64_t)tiles_of(W, H) * 8 + (int64_t)W * H * 4;
}

uint32_t pow2_at_least(int64_t x, int64_t lo, int64_t cap) {
  int64_t p = lo;
  while (p < x && p < cap) p <<= 1;
  return (uint32_t)std::min(p, cap);
}

// Enqueues the whole pipeline for one batch of shape `sh` on the slot's stream (also used
// for capture).
hipError_t run_pipeline(veg_server* s, Slot& sl, const KOpts& ko, const Shape& sh) {
  hipError_t e = launch_project(sl.d_descs, sh.frames, sh.n_max, ko, sl.rec, sl.count, sl.depth, false, sl.stream);
  if (e != hipSuccess) return e;
  e = launch_bin_count(sl.rec, sl.count, sl.depth, sh.pairs, sl.bws, sl.stream, &sl.d_header->n_pairs);
  if (e != hipSuccess) return e;
  e = launch_bin_sort(sl.d_descs, sh.frames, sl.rec, sl.count, sh.pairs, (uint32_t)(sh.frames * sh.tiles), sl.bws,
                      sl.keys, sl.vals, sl.keys_alt, sl.vals_alt, sl.ranges, sh.entries, sl.stream);
  if (e != hipSuccess) return e;
  return launch_blend_fwd(sl.d_descs, sh.frames, 1, sh.tiles, ko, sl.rec, sl.vals, sl.ranges, nullptr, nullptr,
                          nullptr, nullptr, nullptr, 0, nullptr, sl.keys_alt, (uint64_t)s->entries_cap, sl.stream);
}

// The graph of (shape, options) in the slot, captured on first use.
hipError_t slot_graph(veg_server* s, Slot& sl, const KOpts& ko, const Shape& sh, hipGraphExec_t* exec) {
  ++sl.uses;
  for (GraphEntry& g : sl.graphs)
    if (g.shape == sh && std::memcmp(&g.opts, &ko, sizeof(KOpts)) == 0) {
      g.last_use = sl.uses;
      *exec = g.exec;
      return hipSuccess;
    }
  if (sl.graphs.size() >= kGraphsPerSlot) {
    auto lru = std::min_element(sl.graphs.begin(), sl.graphs.end(),
                                [](const GraphEntry& a, const GraphEntry& b) { return a.last_use < b.last_use; });
    (void)hipGraphExecDestroy(lru->exec);
    sl.graphs.erase(lru);
  }
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t e2 = run_pipeline(s, sl, ko, sh);
    e = hipStreamEndCapture(sl.stream, &graph);
    if (e == hipSuccess) e = e2;
  }
  GraphEntry g;
  if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return e;
  g.shape = sh;
  g.opts = ko;
  g.last_use = sl.uses;
  sl.graphs.push_back(g);
  s->graphs_captured++;
  *exec = g.exec;
  return hipSuccess;
}

// Called with the lock held: writes the batch's descriptors and launches it.
veg_status launch_batch(veg_server* s, Slot& sl, const std::vector<uint64_t>& ids) {
  const veg_serve_config& c = s->cfg;
  BatchHeader* hh = reinterpret_cast<BatchHeader*>(sl.h_stage);
  FrameDesc* hd = reinterpret_cast<FrameDesc*>(sl.h_stage + sizeof(BatchHeader));
  std::memset(sl.h_stage, 0, sizeof(BatchHeader) + (size_t)c.max_batch * sizeof(FrameDesc));
  uint32_t pair_base = 0, tile_base = 0;
  const Req& first = s->reqs[ids[0]];
  for (size_t f = 0; f < ids.size(); ++f) {
    Req& q = s->reqs[ids[f]];
    const veg_gaussians& g = s->models[q.r.model_id];
    FrameDesc& d = hd[f];
    d.means = g.means;
    d.log_scales = g.log_scales;
    d.quats = g.quats;
    d.scalars = g.scalars;
    d.weights = g.weights;
    set_lighting(d, g, q.r.camera);
    d.lut = sl.d_luts + (size_t)f * c.max_tf_k * 4;
    d.out_image = q.r.out_image;
    d.out_tfinal = q.r.out_t_final;
    d.out_nlast = nullptr;
    d.K = q.r.tf_k;
    d.n = (int32_t)g.n;
    d.W = q.r.camera.width;
    d.H = q.r.camera.height;
    d.tiles_x = (d.W + kTile - 1) / kTile;
    d.tiles_y = (d.H + kTile - 1) / kTile;
    d.pair_base = pair_base;
    d.tile_base = tile_base;
    set_own_list(d, (int)f);
    std::memcpy(d.view, q.r.camera.view, sizeof(d.view));
    d.fx = q.r.camera.fx;
    d.fy = q.r.camera.fy;
    d.cx = q.r.camera.cx;
    d.cy = q.r.camera.cy;
    d.bg[0] = q.r.opts.bg[0];
    d.bg[1] = q.r.opts.bg[1];
    d.bg[2] = q.r.opts.bg[2];
    std::memcpy(sl.h_luts + (size_t)f * c.max_tf_k * 4, q.tf.data(), q.tf.size() * sizeof(float));
    pair_base += (uint32_t)g.n;
    tile_base += (uint32_t)(d.tiles_x * d.tiles_y);
    q.state = VEG_REQ_RUNNING;
  }
  hh->n_pairs = pair_base;
  hh->n_frames = (uint32_t)ids.size();
  const KOpts ko = kopts_of(first.r.opts);
  Shape sh;
  sh.frames = (int)ids.size();
  int max_tiles = 1;
  int64_t max_n = 1, entries = 0;
  for (uint64_t id : ids) {
    const Req& q = s->reqs[id];
    max_tiles = std::max(max_tiles, tiles_of(q.r.camera.width, q.r.camera.height));
    max_n = std::max(max_n, q.n);
    entries += predicted_entries(s, q);
  }
  sh.tiles = (int)pow2_at_least(max_tiles, 16, s->max_tiles_frame);
  sh.n_max = (int)pow2_at_least(max_n, 1 << 12, c.max_gaussians);
  sh.pairs = pow2_at_least(pair_base, 1 << 14, s->pairs_cap);
  // twice the prediction (the prior varies with the camera distance within a model)
  sh.entries = pow2_at_least(2 * entries, 1 << 16, s->entries_cap);
  sl.entries_bound = sh.entries;
  hipError_t e = hipMemcpyAsync(sl.d_header, sl.h_stage, sizeof(BatchHeader) + (size_t)c.max_batch * sizeof(FrameDesc),
                                hipMemcpyHostToDevice, sl.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sl.d_luts, sl.h_luts, ids.size() * (size_t)c.max_tf_k * 4 * sizeof(float),
                       hipMemcpyHostToDevice, sl.stream);
  if (e == hipSuccess) {
    if (c.use_graphs) {
      hipGraphExec_t exec = nullptr;
      e = slot_graph(s, sl, ko, sh, &exec);
      if (e == hipSuccess) e = hipGraphLaunch(exec, sl.stream);
    } else {
      e = run_pipeline(s, sl, ko, sh);
    }
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(sl.h_counters, sl.bws.counters, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, sl.stream);
  if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
  if (e != hipSuccess) {
    s->err = std::string("launch: ") + hipGetErrorString(e);
    return VEG_ERR_HIP;
  }
  return VEG_OK;
}

void finish_request(veg_server* s, Req& q, veg_status st, double t) {
  q.state = st == VEG_OK ? VEG_REQ_DONE : VEG_REQ_FAILED;
  q.status = st;
  q.t_done = t;
  if (st == VEG_OK) {
    s->completed++;
    s->lat_ms.push_back((t - q.t_submit) * 1e3);
    s->pix_done += (double)q.r.camera.width * q.r.camera.height;
    s->last_done = t;
  } else {
    s->failed++;
  }
}

// Called with the lock held.
void reap(veg_server* s, Slot& sl, double t) {
  const uint64_t E = (uint64_t)sl.h_counters[1] | ((uint64_t)sl.h_counters[2] << 32);
  const bool overflow = sl.h_counters[3] != 0;
  if (overflow) {
    // The batch needed E entries, more than its bound.  Re-run each request alone (at the
    // front of the queue, in order) with E as its bound, which holds for any one of them;
    // a request that needs more than the slot's buffers hold fails.
    if ((int64_t)E > s->entries_cap && sl.reqs.size() == 1) {
      finish_request(s, s->reqs[sl.reqs[0]], VEG_ERR_CAPACITY, t);
    } else {
      s->retries += (int64_t)sl.reqs.size();
      for (auto it = sl.reqs.rbegin(); it != sl.reqs.rend(); ++it) {
        Req& q = s->reqs[*it];
        q.solo = true;
        q.known_entries = std::min<int64_t>((int64_t)E, s->entries_cap);
        q.state = VEG_REQ_QUEUED;
        s->queue.push_front(*it);
      }
    }
  } else {
    for (uint64_t id : sl.reqs) finish_request(s, s->reqs[id], VEG_OK, t);
  }
  // Learn the models' multipliers from observed / predicted (shared by a mixed batch's
  // models): up at once, down slowly, with a 25% margin.
  if (sl.est_entries > 0) {
    const double f = 1.25 * (double)E / (double)sl.est_entries;
    for (uint64_t id : sl.reqs) {
      double& m = s->m_scale[(size_t)s->reqs[id].r.model_id];
      m = f > 1.0 ? m * f : m * (0.9 + 0.1 * f);
    }
  }
  s->in_use -= sl.bytes;
  sl.busy = false;
  sl.reqs.clear();
  s->inflight--;
  if (s->inflight == 0 && s->busy_since >= 0) {
    s->busy_acc += t - s->busy_since;
    s->busy_since = -1;
  }
  s->cv_done.notify_all();
}

// Forms a batch from the head of the queue for a free slot; returns false if none fits.
bool try_launch(veg_server* s, Slot& sl) {
  if (s->queue.empty()) return false;
  const veg_serve_config& c = s->cfg;
  std::vector<uint64_t> ids;
  int64_t pairs = 0, entries = 0, bytes = 0;
  const veg_opts* o0 = nullptr;
  while (!s->queue.empty() && (int)ids.size() < c.max_batch) {
    Req& q = s->reqs[s->queue.front()];
    const int64_t e = predicted_entries(s, q);
    const bool fits = pairs + q.n <= s->pairs_cap && entries + e <= s->entries_cap &&
                      s->in_use + bytes + q.est_bytes <= (int64_t)c.budget_bytes &&
                      (o0 == nullptr || same_opts(*o0, q.r.opts));
    if (!ids.empty() && (!fits || q.solo)) break;
    if (ids.empty() && !fits && s->in_use > 0) break;   // wait for memory to free up
    ids.push_back(q.id);
    pairs += q.n;
    entries += e;
    bytes += q.est_bytes;
    o0 = &q.r.opts;
    s->queue.pop_front();
    if (q.solo) break;
  }
  if (ids.empty()) return false;
  sl.busy = true;
  sl.reqs = ids;
  sl.bytes = bytes;
  sl.est_entries = 0;
  for (uint64_t id : ids) sl.est_entries += predicted_entries(s, s->reqs[id]);
  s->in_use += bytes;
  s->peak = std::max(s->peak, s->in_use);
  s->batches++;
  s->sum_batch += (double)ids.size();
  const double t = now_s();
  if (s->inflight == 0) s->busy_since = t;
  s->inflight++;
  sl.t_launch = t;
  if (launch_batch(s, sl, ids) != VEG_OK) {
    for (uint64_t id : ids) finish_request(s, s->reqs[id], VEG_ERR_HIP, t);
    (void)hipStreamSynchronize(sl.stream);
    sl.busy = false;
    sl.reqs.clear();
    s->in_use -= bytes;
    s->inflight--;
    if (s->inflight == 0 && s->busy_since >= 0) {
      s->busy_acc += t - s->busy_since;
      s->busy_since = -1;
    }
    s->cv_done.notify_all();
  }
  return true;
}

void scheduler(veg_server* s) {
  (void)hipSetDevice(s->device);
  // Timed waits of this thread end within a microsecond of their deadline instead of the
  // default 50 us timer slack: the 20 us completion polls below then take 20 us, not 70.
  (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    const double t = now_s();
    for (Slot& sl : s->slots)
      if (sl.busy && hipEventQuery(sl.done) == hipSuccess) reap(s, sl, t);
    bool launched = !s->stop;   // shutting down: finish what runs, launch nothing new
    while (launched) {
      launched = false;
      for (Slot& sl : s->slots)
        if (!sl.busy && try_launch(s, sl)) launched = true;
    }
    if (s->stop && s->inflight == 0) break;
    if (s->inflight > 0) {
      s->cv.wait_for(lk, std::chrono::microseconds(20));
    } else {
      s->cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
    }
  }
  // drain: anything still queued fails
  const double t = now_s();
  while (!s->queue.empty()) {
    finish_request(s, s->reqs[s->queue.front()], VEG_ERR_SHUTDOWN, t);
    s->queue.pop_front();
  }
  s->cv_done.notify_all();
}

void free_slots(veg_server* s) {
  for (Slot& sl : s->slots) {
    for (GraphEntry& g : sl.graphs) (void)hipGraphExecDestroy(g.exec);
    sl.graphs.clear();
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.h_stage) (void)hipHostFree(sl.h_stage);
    if (sl.h_luts) (void)hipHostFree(sl.h_luts);
    if (sl.h_counters) (void)hipHostFree(sl.h_counters);
  }
  s->slots.clear();
}

}  // namespace

extern "C" {

size_t veg_serve_arena_bytes(const veg_serve_config* cfg) {
  if (check_cfg(cfg) != VEG_OK) return 0;
  return slot_layout(*cfg).total * (size_t)cfg->n_streams + 256;
}

veg_status veg_serve_create(const veg_serve_config* cfg, veg_server** out) {
  set_last_error("");
  veg_status st = check_cfg(cfg);
  if (st != VEG_OK) return st;
  if (!out || !cfg->arena) return sfail(VEG_ERR_INVALID_ARG, "NULL arena or output");
  const Layout L = slot_layout(*cfg);
  if (cfg->arena_bytes < L.total * (size_t)cfg->n_streams + 256)
    return sfail(VEG_ERR_INVALID_ARG, "arena too small: need %zu bytes", L.total * (size_t)cfg->n_streams + 256);
  veg_server* s = new veg_server();
  s->cfg = *cfg;
  if (s->cfg.budget_bytes == 0) s->cfg.budget_bytes = cfg->arena_bytes;
  (void)hipGetDevice(&s->device);
  s->pairs_cap = pairs_cap_of(*cfg);
  s->entries_cap = cfg->max_entries;
  s->max_tiles_frame = tiles_of(cfg->max_width, cfg->max_height);
  s->total_tiles_cap = (uint32_t)(cfg->max_batch * s->max_tiles_frame);
  s->slots.resize(cfg->n_streams);
  unsigned char* base = (unsigned char*)(((uintptr_t)cfg->arena + 255) & ~(uintptr_t)255);
  hipError_t e = hipSuccess;
  for (int k = 0; k < cfg->n_streams && e == hipSuccess; ++k) {
    Slot& sl = s->slots[k];
    unsigned char* b = base + (size_t)k * L.total;
    sl.d_header = (BatchHeader*)(b + L.header);
    sl.d_descs = (FrameDesc*)(b + L.header + sizeof(BatchHeader));
    sl.d_luts = (float*)(b + L.luts);
    sl.rec = (float4*)(b + L.rec);
    sl.count = (uint32_t*)(b + L.count);
    sl.depth = (uint32_t*)(b + L.depth);
    sl.ws = b + L.ws;
    carve_bin_ws(sl.ws, s->pairs_cap, &sl.bws);
    uint32_t* kb = (uint32_t*)(b + L.keys);
    sl.keys = kb;
    sl.vals = kb + cfg->max_entries;
    sl.keys_alt = kb + 2 * cfg->max_entries;
    sl.vals_alt = kb + 3 * cfg->max_entries;
    sl.ranges = (uint32_t*)(b + L.ranges);
    e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&sl.h_stage, sizeof(BatchHeader) + (size_t)cfg->max_batch * sizeof(FrameDesc), 0);
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&sl.h_luts, (size_t)cfg->max_batch * cfg->max_tf_k * 4 * sizeof(float), 0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_counters, 64, 0);
  }
  if (e != hipSuccess) {
    free_slots(s);
    delete s;
    return sfail(VEG_ERR_HIP, "serve_create: %s", hipGetErrorString(e));
  }
  s->sched = std::thread(scheduler, s);
  *out = s;
  return VEG_OK;
}

veg_status veg_serve_add_model(veg_server* s, const veg_gaussians* g, int32_t* model_id) {
  set_last_error("");
  if (!s || !g || !model_id) return sfail(VEG_ERR_INVALID_ARG, "NULL argument");
  if (g->n < 1 || g->n > s->cfg.max_gaussians) return sfail(VEG_ERR_INVALID_ARG, "model size out of range");
  if (!g->means || !g->log_scales || !g->quats || !g->scalars)
    return sfail(VEG_ERR_INVALID_ARG, "NULL model array");
  if (reinterpret_cast<uintptr_t>(g->quats) & 15u) return sfail(VEG_ERR_INVALID_ARG, "quats must be 16-byte aligned");
  std::lock_guard<std::mutex> lk(s->mu);
  s->models.push_back(*g);
  s->m_scale.push_back(1.0);
  *model_id = (int32_t)s->models.size() - 1;
  return VEG_OK;
}

veg_status veg_serve_submit(veg_server* s, const veg_request* r, uint64_t* req_id) {
  set_last_error("");
  if (!s || !r || !req_id) return sfail(VEG_ERR_INVALID_ARG, "NULL argument");
  const veg_camera& c = r->camera;
  if (c.width < 1 || c.height < 1 || c.width > s->cfg.max_width || c.height > s->cfg.max_height)
    return sfail(VEG_ERR_INVALID_ARG, "resolution outside the server's limits");
  if (!(c.fx > 0.0f) || !(c.fy > 0.0f) || !std::isfinite(c.cx) || !std::isfinite(c.cy))
    return sfail(VEG_ERR_INVALID_ARG, "need fx, fy > 0 and finite cx, cy");
  for (int k = 0; k < 12; ++k)
    if (!std::isfinite(c.view[k])) return sfail(VEG_ERR_INVALID_ARG, "non-finite view matrix");
  if (!r->tf_rgba || r->tf_k < 2 || r->tf_k > s->cfg.max_tf_k) return sfail(VEG_ERR_INVALID_ARG, "bad TF table");
  if (!r->out_image) return sfail(VEG_ERR_INVALID_ARG, "NULL out_image");
  const veg_opts& o = r->opts;
  if (!(o.alpha_min > 0.0f) || !(o.alpha_clamp > o.alpha_min) || !(o.alpha_clamp <= 1.0f) || !(o.t_min >= 0.0f) ||
      !(o.t_min < 1.0f) || !(o.lowpass >= 0.0f) || !(o.near_z > 0.0f) || !(o.guard > 0.0f))
    return sfail(VEG_ERR_INVALID_ARG, "bad options");
  if (!(r->t_arrival >= 0.0) || !std::isfinite(r->t_arrival)) return sfail(VEG_ERR_INVALID_ARG, "bad t_arrival");
  const double t_call = now_s();   // before the lock: time spent waiting for it counts as latency
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return sfail(VEG_ERR_SHUTDOWN, "server is shutting down");
  if (r->model_id < 0 || r->model_id >= (int32_t)s->models.size()) return sfail(VEG_ERR_NOT_FOUND, "unknown model");
  Req q;
  q.id = s->next_id++;
  q.r = *r;
  q.tf.assign(r->tf_rgba, r->tf_rgba + (size_t)r->tf_k * 4);
  q.r.tf_rgba = nullptr;
  q.n = s->models[r->model_id].n;
  q.est_entries = entry_prior(q.n, c.width, c.height);
  q.est_bytes = req_bytes(q.n, q.est_entries, c.width, c.height);
  q.t_submit = r->t_arrival > 0.0 ? r->t_arrival : t_call;
  if (q.n > s->pairs_cap || q.est_bytes > (int64_t)s->cfg.budget_bytes) {
    s->rejected++;
    return sfail(VEG_ERR_OUT_OF_BUDGET, "request can never fit (pairs %lld, est. bytes %lld, budget %zu)",
                 (long long)q.n, (long long)q.est_bytes, s->cfg.budget_bytes);
  }
  s->submitted++;
  if (s->first_submit < 0 || q.t_submit < s->first_submit) s->first_submit = q.t_submit;
  *req_id = q.id;
  s->queue.push_back(q.id);
  s->reqs.emplace(q.id, std::move(q));
  s->cv.notify_all();
  return VEG_OK;
}

veg_status veg_serve_poll(veg_server* s, uint64_t req_id, int32_t* state) {
  set_last_error("");
  if (!s || !state) return sfail(VEG_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  if (it == s->reqs.end()) return sfail(VEG_ERR_NOT_FOUND, "unknown request");
  *state = it->second.state;
  return VEG_OK;
}

veg_status veg_serve_wait(veg_server* s, uint64_t req_id, int32_t timeout_ms) {
  set_last_error("");
  if (!s) return sfail(VEG_ERR_INVALID_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  if (it == s->reqs.end()) return sfail(VEG_ERR_NOT_FOUND, "unknown request");
  // the entry may be released by another waiter while this one sleeps: look it up anew
  auto finished = [&] {
    auto f = s->reqs.find(req_id);
    return f == s->reqs.end() || f->second.state == VEG_REQ_DONE || f->second.state == VEG_REQ_FAILED;
  };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, finished);
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), finished)) {
    return sfail(VEG_ERR_TIMEOUT, "request %llu not finished", (unsigned long long)req_id);
  }
  it = s->reqs.find(req_id);
  if (it == s->reqs.end()) return sfail(VEG_ERR_NOT_FOUND, "request %llu released by another wait",
                                        (unsigned long long)req_id);
  const veg_status st = it->second.status;
  s->reqs.erase(it);   // a finished request is released once it has been waited on
  if (st != VEG_OK) return sfail(st, "request %llu failed: %s", (unsigned long long)req_id, s->err.c_str());
  return VEG_OK;
}

veg_status veg_serve_stats_get(veg_server* s, veg_serve_stats* out) {
  set_last_error("");
  if (!s || !out) return sfail(VEG_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->rejected = s->rejected;
  out->batches = s->batches;
  out->retries = s->retries;
  out->mean_batch = s->batches ? s->sum_batch / (double)s->batches : 0.0;
  if (!s->lat_ms.empty()) {
    std::vector<double> v = s->lat_ms;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
      const size_t i = (size_t)std::min<double>((double)v.size() - 1, std::ceil(p * (double)v.size()) - 1);
      return v[i];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    out->max_ms = v.back();
  }
  const double span = (s->last_done > s->first_submit && s->first_submit >= 0) ? s->last_done - s->first_submit : 0;
  if (span > 0) {
    out->throughput_rps = (double)s->completed / span;
    out->mpix_per_s = s->pix_done / span / 1e6;
    double busy = s->busy_acc;
    if (s->busy_since >= 0) busy += now_s() - s->busy_since;
    out->gpu_busy_frac = std::min(1.0, busy / span);
  }
  out->peak_bytes = s->peak;
  out->graphs_captured = s->graphs_captured;
  return VEG_OK;
}

veg_status veg_serve_stats_reset(veg_server* s) {
  if (!s) return sfail(VEG_ERR_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  s->lat_ms.clear();
  s->submitted = s->completed = s->failed = s->rejected = s->batches = s->retries = 0;
  s->sum_batch = s->pix_done = 0;
  s->first_submit = s->last_done = -1;
  s->busy_acc = 0;
  s->busy_since = s->inflight > 0 ? now_s() : -1;
  s->peak = s->in_use;
  // requests stay until they are waited on (a waiter may be about to read one)
  return VEG_OK;
}

veg_status veg_serve_destroy(veg_server* s) {
  if (!s) return sfail(VEG_ERR_INVALID_ARG, "NULL server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->sched.joinable()) s->sched.join();
  for (Slot& sl : s->slots)
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
  free_slots(s);
  delete s;
  return VEG_OK;
}

}  // extern "C"
