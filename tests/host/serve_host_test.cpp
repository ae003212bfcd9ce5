// Host-side scenarios of the render server's scheduler and of the C entry points' argument
// handling, run against the fake HIP runtime of fake_hip.cpp (host memory stands in for
// device memory) and built with AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Scenarios: continuous batching (requests queue while both slots are busy and join the
// next free slot, up to max_batch per batch; every result reaches its own buffer), overflow
// retry (a batch whose key list outgrows its bound is re-run request by request with the
// observed count; a request larger than the slot fails with VEG_ERR_CAPACITY), admission
// by the memory budget (requests wait until memory frees up; one that can never fit is
// refused at submit), waits racing with statistics resets, latency from a given arrival
// time, shutdown with queued requests, and the stateless entry points on host buffers.
// Prints "ok <scenario>" per scenario; exits non-zero at the first failed check.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "veg.h"

extern "C" {
void fake_set_gated(int on);
void fake_release_all();
void fake_set_entries_per_gaussian(int k);
int64_t fake_blend_launches();
int64_t fake_blend_frames();
int64_t fake_graph_launches();
}

#define CHECK(cond)                                                                   \
  do {                                                                                \
    if (!(cond)) {                                                                    \
      std::fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #cond,     \
                   veg_last_error());                                                 \
      std::exit(1);                                                                   \
    }                                                                                 \
  } while (0)

namespace {

double now_s() { return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count(); }

struct Model {
  std::vector<float> means, log_scales, scalars;
  float* quats = nullptr;
  veg_gaussians g{};
  explicit Model(int64_t n) : means(3 * n, 0.0f), log_scales(3 * n, -3.0f), scalars(n, 0.5f) {
    quats = (float*)std::aligned_alloc(16, (size_t)(16 * n));
    for (int64_t i = 0; i < n; ++i) {
      quats[4 * i] = 1.0f;
      quats[4 * i + 1] = quats[4 * i + 2] = quats[4 * i + 3] = 0.0f;
    }
    g.n = n;
    g.means = means.data();
    g.log_scales = log_scales.data();
    g.quats = quats;
    g.scalars = scalars.data();
  }
  ~Model() { std::free(quats); }
};

struct Server {
  veg_serve_config cfg{};
  void* arena = nullptr;
  veg_server* s = nullptr;
  Server(int max_batch, int n_streams, int64_t max_gaussians, int64_t max_entries, size_t budget) {
    cfg.max_batch = max_batch;
    cfg.n_streams = n_streams;
    cfg.use_graphs = 1;
    cfg.max_width = cfg.max_height = 128;
    cfg.max_tf_k = 16;
    cfg.max_gaussians = max_gaussians;
    cfg.max_entries = max_entries;
    const size_t bytes = veg_serve_arena_bytes(&cfg);
    CHECK(bytes > 0);
    arena = std::calloc(1, bytes);
    cfg.arena = arena;
    cfg.arena_bytes = bytes;
    cfg.budget_bytes = budget;
    CHECK(veg_serve_create(&cfg, &s) == VEG_OK);
  }
  ~Server() {
    if (s) CHECK(veg_serve_destroy(s) == VEG_OK);
    std::free(arena);
  }
};

struct Request {
  std::vector<float> tf;
  std::vector<float> out;
  veg_request r{};
  uint64_t id = 0;
  Request(int model, int w, int h, float tf0) : tf(8, 0.25f), out((size_t)3 * w * h, -1.0f) {
    tf[0] = tf0;
    r.model_id = model;
    float view[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 3};
    std::memcpy(r.camera.view, view, sizeof(view));
    r.camera.fx = r.camera.fy = 100.0f;
    r.camera.cx = 0.5f * w;
    r.camera.cy = 0.5f * h;
    r.camera.width = w;
    r.camera.height = h;
    r.tf_rgba = tf.data();
    r.tf_k = 2;
    r.out_image = out.data();
    veg_opts_default(&r.opts);
  }
  // the fake blend's signature: model size, width, height, first table value
  bool rendered(int64_t n) const {
    return out[0] == (float)n && out[1] == (float)r.camera.width && out[2] == (float)r.camera.height &&
           out[3] == tf[0];
  }
};

void wait_until(veg_server* s, uint64_t id, int32_t want) {
  for (int i = 0; i < 2000; ++i) {
    int32_t st = -1;
    CHECK(veg_serve_poll(s, id, &st) == VEG_OK);
    if (st == want) return;
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
  }
  CHECK(!"request did not reach the expected state");
}

void settle() { std::this_thread::sleep_for(std::chrono::milliseconds(30)); }

int count_state(veg_server* s, std::vector<Request*>& rs, int32_t want) {
  int k = 0;
  for (Request* q : rs) {
    int32_t st = -1;
    CHECK(veg_serve_poll(s, q->id, &st) == VEG_OK);
    k += st == want;
  }
  return k;
}

void continuous_batching() {
  fake_set_entries_per_gaussian(4);
  Model a(500), b(900);
  Server sv(4, 2, 1000, 1 << 20, 0);
  int32_t ma = -1, mb = -1;
  CHECK(veg_serve_add_model(sv.s, &a.g, &ma) == VEG_OK && ma == 0);
  CHECK(veg_serve_add_model(sv.s, &b.g, &mb) == VEG_OK && mb == 1);
  fake_set_gated(1);
  std::vector<Request*> rs;
  auto submit = [&](int i) {
    Request* q = new Request(i % 2, 32 + 16 * (i % 3), 48, 0.1f * (float)i);
    CHECK(veg_serve_submit(sv.s, &q->r, &q->id) == VEG_OK);
    rs.push_back(q);
  };
  // one request each occupies both slots ...
  submit(0);
  wait_until(sv.s, rs[0]->id, VEG_REQ_RUNNING);
  submit(1);
  wait_until(sv.s, rs[1]->id, VEG_REQ_RUNNING);
  // ... so eight more wait in the queue
  for (int i = 2; i < 10; ++i) submit(i);
  settle();
  CHECK(count_state(sv.s, rs, VEG_REQ_RUNNING) == 2);
  CHECK(count_state(sv.s, rs, VEG_REQ_QUEUED) == 8);
  // as the slots free up, the queue joins them in batches of max_batch = 4
  fake_release_all();
  settle();
  CHECK(count_state(sv.s, rs, VEG_REQ_DONE) == 2);
  CHECK(count_state(sv.s, rs, VEG_REQ_RUNNING) == 8);
  fake_release_all();
  for (Request* q : rs) CHECK(veg_serve_wait(sv.s, q->id, 2000) == VEG_OK);
  for (size_t i = 0; i < rs.size(); ++i) CHECK(rs[i]->rendered(i % 2 ? 900 : 500));
  veg_serve_stats st{};
  CHECK(veg_serve_stats_get(sv.s, &st) == VEG_OK);
  CHECK(st.completed == 10 && st.batches == 4 && std::fabs(st.mean_batch - 2.5) < 1e-9);
  CHECK(st.retries == 0 && st.failed == 0 && st.graphs_captured >= 2);
  // a waited request is released: its id is unknown afterwards
  CHECK(veg_serve_wait(sv.s, rs[0]->id, 0) == VEG_ERR_NOT_FOUND);
  fake_set_gated(0);
  for (Request* q : rs) delete q;
  std::printf("ok continuous_batching\n");
}

void overflow_retry() {
  Model a(1000);
  Server sv(4, 2, 1000, 100000, 0);
  int32_t m = -1;
  CHECK(veg_serve_add_model(sv.s, &a.g, &m) == VEG_OK);
  // two small requests occupy both slots while four more queue up
  fake_set_entries_per_gaussian(4);
  fake_set_gated(1);
  Request b0(0, 64, 64, 0.1f), b1(0, 64, 64, 0.2f);
  CHECK(veg_serve_submit(sv.s, &b0.r, &b0.id) == VEG_OK);
  wait_until(sv.s, b0.id, VEG_REQ_RUNNING);
  CHECK(veg_serve_submit(sv.s, &b1.r, &b1.id) == VEG_OK);
  wait_until(sv.s, b1.id, VEG_REQ_RUNNING);
  std::vector<Request*> rs;
  for (int i = 0; i < 4; ++i) {
    Request* q = new Request(0, 64, 64, 0.5f + 0.1f * (float)i);
    CHECK(veg_serve_submit(sv.s, &q->r, &q->id) == VEG_OK);
    rs.push_back(q);
  }
  // 20 entries per Gaussian from now on: 20k per request, 80k for the batch of four, far
  // above the batch's estimated bound (the prior is 7k per 64x64 request); each alone fits
  fake_set_entries_per_gaussian(20);
  fake_set_gated(0);
  CHECK(veg_serve_wait(sv.s, b0.id, 2000) == VEG_OK && veg_serve_wait(sv.s, b1.id, 2000) == VEG_OK);
  for (Request* q : rs) CHECK(veg_serve_wait(sv.s, q->id, 2000) == VEG_OK);
  for (Request* q : rs) CHECK(q->rendered(1000));
  veg_serve_stats st{};
  CHECK(veg_serve_stats_get(sv.s, &st) == VEG_OK);
  CHECK(st.retries == 4 && st.completed == 6 && st.failed == 0);
  // a request that needs more entries than the slot holds fails, alone or batched
  fake_set_entries_per_gaussian(200);
  Request big(0, 64, 64, 0.9f);
  CHECK(veg_serve_submit(sv.s, &big.r, &big.id) == VEG_OK);
  CHECK(veg_serve_wait(sv.s, big.id, 2000) == VEG_ERR_CAPACITY);
  fake_set_entries_per_gaussian(4);
  for (Request* q : rs) delete q;
  std::printf("ok overflow_retry\n");
}

void budget_admission() {
  fake_set_entries_per_gaussian(4);
  Model a(1000);
  // one 64x64 request of 1000 Gaussians is estimated at 200,896 bytes and a 128x128 one at
  // 250,432: a budget of 240,000 admits the former one at a time although two slots are
  // free, and can never admit the latter
  Server sv(4, 2, 1000, 1 << 20, 240000);
  int32_t m = -1;
  CHECK(veg_serve_add_model(sv.s, &a.g, &m) == VEG_OK);
  fake_set_gated(1);
  std::vector<Request*> rs;
  for (int i = 0; i < 3; ++i) {
    Request* q = new Request(0, 64, 64, 0.2f * (float)i);
    CHECK(veg_serve_submit(sv.s, &q->r, &q->id) == VEG_OK);
    rs.push_back(q);
  }
  settle();
  CHECK(count_state(sv.s, rs, VEG_REQ_RUNNING) == 1);
  CHECK(count_state(sv.s, rs, VEG_REQ_QUEUED) == 2);
  fake_release_all();
  settle();
  CHECK(count_state(sv.s, rs, VEG_REQ_DONE) == 1);
  CHECK(count_state(sv.s, rs, VEG_REQ_RUNNING) == 1);
  fake_set_gated(0);
  for (Request* q : rs) CHECK(veg_serve_wait(sv.s, q->id, 2000) == VEG_OK);
  veg_serve_stats st{};
  CHECK(veg_serve_stats_get(sv.s, &st) == VEG_OK);
  CHECK(st.peak_bytes == 200896 && st.batches == 3);
  // a request whose estimate exceeds the whole budget can never run
  Request huge(0, 128, 128, 0.3f);
  uint64_t id = 0;
  CHECK(veg_serve_submit(sv.s, &huge.r, &id) == VEG_ERR_OUT_OF_BUDGET);
  for (Request* q : rs) delete q;
  std::printf("ok budget_admission\n");
}

void waits_race_with_resets() {
  fake_set_entries_per_gaussian(4);
  Model a(300);
  Server sv(8, 2, 1000, 1 << 20, 0);
  int32_t m = -1;
  CHECK(veg_serve_add_model(sv.s, &a.g, &m) == VEG_OK);
  fake_set_gated(1);
  std::vector<Request*> rs;
  for (int i = 0; i < 32; ++i) {
    Request* q = new Request(0, 32, 32, 0.01f * (float)i);
    CHECK(veg_serve_submit(sv.s, &q->r, &q->id) == VEG_OK);
    rs.push_back(q);
  }
  std::vector<int> status(rs.size(), -1);
  std::vector<std::thread> waiters;
  for (size_t i = 0; i < rs.size(); ++i)
    waiters.emplace_back([&, i] { status[i] = veg_serve_wait(sv.s, rs[i]->id, 5000); });
  std::thread resetter([&] {
    for (int k = 0; k < 200; ++k) {
      CHECK(veg_serve_stats_reset(sv.s) == VEG_OK);
      if (k % 20 == 0) fake_release_all();
      std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    fake_set_gated(0);
  });
  resetter.join();
  for (auto& t : waiters) t.join();
  for (int s : status) CHECK(s == VEG_OK);
  for (Request* q : rs) delete q;
  std::printf("ok waits_race_with_resets\n");
}

void latency_from_arrival_time() {
  fake_set_entries_per_gaussian(4);
  Model a(100);
  Server sv(4, 1, 1000, 1 << 20, 0);
  int32_t m = -1;
  CHECK(veg_serve_add_model(sv.s, &a.g, &m) == VEG_OK);
  CHECK(veg_serve_stats_reset(sv.s) == VEG_OK);
  Request q(0, 32, 32, 0.5f);
  q.r.t_arrival = now_s() - 0.5;
  CHECK(veg_serve_submit(sv.s, &q.r, &q.id) == VEG_OK);
  CHECK(veg_serve_wait(sv.s, q.id, 2000) == VEG_OK);
  veg_serve_stats st{};
  CHECK(veg_serve_stats_get(sv.s, &st) == VEG_OK);
  CHECK(st.p50_ms >= 500.0 && st.p50_ms < 5000.0);
  Request bad(0, 32, 32, 0.5f);
  bad.r.t_arrival = -1.0;
  uint64_t id = 0;
  CHECK(veg_serve_submit(sv.s, &bad.r, &id) == VEG_ERR_INVALID_ARG);
  std::printf("ok latency_from_arrival_time\n");
}

void shutdown_fails_queued_requests() {
  fake_set_entries_per_gaussian(4);
  Model a(100);
  std::vector<Request*> rs;
  {
    Server sv(1, 1, 1000, 1 << 20, 0);
    int32_t m = -1;
    CHECK(veg_serve_add_model(sv.s, &a.g, &m) == VEG_OK);
    fake_set_gated(1);
    for (int i = 0; i < 3; ++i) {
      Request* q = new Request(0, 32, 32, 0.1f);
      CHECK(veg_serve_submit(sv.s, &q->r, &q->id) == VEG_OK);
      rs.push_back(q);
    }
    settle();
    CHECK(count_state(sv.s, rs, VEG_REQ_QUEUED) == 2);
    // destroy drains the running batch (its stream is synchronised) and fails the queue
    std::thread rel([] {
      std::this_thread::sleep_for(std::chrono::milliseconds(20));
      fake_release_all();
    });
    veg_server* s = sv.s;
    sv.s = nullptr;
    CHECK(veg_serve_destroy(s) == VEG_OK);
    rel.join();
  }
  fake_set_gated(0);
  for (Request* q : rs) delete q;
  std::printf("ok shutdown_fails_queued_requests\n");
}

void stateless_entry_points_on_host_buffers() {
  // argument checks and marshalling of the stateless calls (the launches are no-ops here)
  Model a(64);
  std::vector<unsigned char> frames(veg_frames_bytes(2) + 256);
  std::vector<float> rec(2 * 64 * 12);
  std::vector<uint32_t> count(2 * 64), depth(2 * 64);
  veg_proj p{};
  p.n = 64;
  p.n_frames = 2;
  p.frames = frames.data();
  p.rec = rec.data();
  p.count = count.data();
  p.depth = depth.data();
  veg_camera cams[2];
  for (auto& c : cams) {
    float view[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 3};
    std::memcpy(c.view, view, sizeof(view));
    c.fx = c.fy = 60.0f;
    c.cx = c.cy = 24.0f;
    c.width = c.height = 48;
  }
  std::vector<float> lut(8, 0.5f);
  veg_tf tfs[2] = {{lut.data(), 2}, {lut.data(), 2}};
  CHECK(veg_project(&a.g, 2, cams, tfs, nullptr, &p, nullptr) == VEG_OK);
  CHECK(p.tiles_x == 3 && p.tiles_y == 3 && p.total_tiles == 18 && p.width == 48);
  const size_t wsb = veg_bin_workspace_bytes(128, 1000);
  std::vector<unsigned char> ws(wsb);
  int64_t e = -1;
  CHECK(veg_bin_count(&p, ws.data(), wsb, &e, nullptr) == VEG_OK && e == 0);
  CHECK(veg_bin_count(&p, ws.data(), 16, &e, nullptr) == VEG_ERR_INVALID_ARG);
  std::vector<uint32_t> keys(4 * 1000), ranges(2 * 18);
  veg_bins b{keys.data(), keys.data() + 1000, keys.data() + 2000, keys.data() + 3000, ranges.data(), 1000, nullptr, 0};
  CHECK(veg_bin_sort(&p, ws.data(), wsb, &b, nullptr) == VEG_OK);
  int64_t status[2] = {-1, -1};
  // the fake sort counts 4 entries per Gaussian and frame
  CHECK(veg_bin_status(ws.data(), wsb, status, nullptr) == VEG_OK && status[0] == 2 * 64 * 4 && status[1] == 0);
  std::vector<float> img(2 * 3 * 48 * 48), tfin(2 * 48 * 48);
  std::vector<int32_t> nlast(2 * 48 * 48);
  CHECK(veg_render_fwd(&p, &b, nullptr, img.data(), tfin.data(), nlast.data(), nullptr, nullptr) == VEG_OK);
  veg_opts o;
  veg_opts_default(&o);
  o.alpha_clamp = 1.0f;
  std::vector<float> g2d(2 * 64 * 9);
  CHECK(veg_render_bwd(&p, &b, &o, tfin.data(), nlast.data(), img.data(), g2d.data(), nullptr) ==
        VEG_ERR_INVALID_ARG);
  CHECK(veg_render_bwd(&p, &b, nullptr, tfin.data(), nlast.data(), img.data(), g2d.data(), nullptr) == VEG_OK);
  double loss = 0;
  CHECK(veg_l1_loss(img.data(), img.data(), (int64_t)img.size(), 1.0f, &loss, img.data(), nullptr) == VEG_OK);
  CHECK(veg_l1_loss(img.data(), img.data(), -1, 1.0f, &loss, img.data(), nullptr) == VEG_ERR_INVALID_ARG);
  // the allocation-free binning call: same status as the workspace calls, limit enforced
  int64_t st2[2] = {-1, -1};
  CHECK(veg_bin_static(&p, &b, st2, nullptr) == VEG_OK && st2[0] == status[0] && st2[1] == status[1]);
  veg_proj big = p;
  big.n = VEG_BIN_STATIC_MAX_PAIRS;   // two frames: twice the limit
  CHECK(veg_bin_static(&big, &b, st2, nullptr) == VEG_ERR_INVALID_ARG);
  std::printf("ok stateless_entry_points_on_host_buffers\n");
}

}  // namespace

int main() {
  std::setvbuf(stdout, nullptr, _IONBF, 0);
  continuous_batching();
  overflow_retry();
  budget_admission();
  waits_race_with_resets();
  latency_from_arrival_time();
  shutdown_fails_queued_requests();
  stateless_entry_points_on_host_buffers();
  std::printf("all scenarios passed\n");
  return 0;
}
