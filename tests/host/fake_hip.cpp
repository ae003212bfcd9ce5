// A host-only stand-in for the HIP runtime and for libveg's kernel launchers, so that the C
// entry points and the render server's scheduler run on the CPU (with sanitizers) against
// host memory.  Test infrastructure: nothing of the library's arithmetic is here.
//
// Streams execute every operation at once.  Completion is what the tests control: an event
// recorded on a stream completes when the stream has been released up to it (gated mode),
// or at once (ungated).  A launch made while a stream captures is recorded into the graph
// and runs when the graph is launched.
//
// The launchers model just enough of the device to drive the server: the key-list sort
// writes an entry count of (fake_entries_per_gaussian x Gaussians) per frame and the
// overflow flag to the workspace counters; the forward blend writes a signature of each
// frame (model size, width, height, first table value) into the first words of its output
// image, so a test can check that every request's result reached its own buffer.
#include <hip/hip_runtime_api.h>
#include <hip/hip_vector_types.h>

#include <atomic>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <vector>

#include "veg_internal.h"

struct ihipStream_t {
  std::mutex mu;
  uint64_t recorded = 0, released = 0;
  bool capturing = false;
  std::vector<std::function<void()>>* capture = nullptr;
};
struct ihipEvent_t {
  ihipStream_t* stream = nullptr;
  uint64_t ticket = 0;
};
struct ihipGraph {
  std::vector<std::function<void()>> ops;
};
struct hipGraphExec {
  std::vector<std::function<void()>> ops;
};

namespace {
std::mutex g_mu;
std::vector<ihipStream_t*> g_streams;
std::atomic<bool> g_gated{false};
std::atomic<int> g_entries_per_gaussian{4};
std::atomic<int64_t> g_blend_launches{0}, g_blend_frames{0}, g_graph_launches{0};

// Runs `op` now, or records it into the graph the stream is capturing.
hipError_t on_stream(hipStream_t s, std::function<void()> op) {
  if (s && s->capturing) {
    s->capture->push_back(std::move(op));
    return hipSuccess;
  }
  op();
  return hipSuccess;
}
}  // namespace

extern "C" {
// test controls
void fake_set_gated(int on) {
  g_gated = on != 0;
  if (!on) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (ihipStream_t* s : g_streams) {
      std::lock_guard<std::mutex> l2(s->mu);
      s->released = s->recorded;
    }
  }
}
void fake_release_all() {
  std::lock_guard<std::mutex> lk(g_mu);
  for (ihipStream_t* s : g_streams) {
    std::lock_guard<std::mutex> l2(s->mu);
    s->released = s->recorded;
  }
}
void fake_set_entries_per_gaussian(int k) { g_entries_per_gaussian = k; }
int64_t fake_blend_launches() { return g_blend_launches; }
int64_t fake_blend_frames() { return g_blend_frames; }
int64_t fake_graph_launches() { return g_graph_launches; }
}

// ------------------------------------------------------------------------- HIP runtime

const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "fake HIP error"; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  *s = new ihipStream_t();
  std::lock_guard<std::mutex> lk(g_mu);
  g_streams.push_back(*s);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (size_t i = 0; i < g_streams.size(); ++i)
    if (g_streams[i] == s) g_streams.erase(g_streams.begin() + (long)i);
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  if (s) {
    std::lock_guard<std::mutex> l2(s->mu);
    s->released = s->recorded;
  }
  return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = new ihipEvent_t();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  std::lock_guard<std::mutex> l2(s->mu);
  e->stream = s;
  e->ticket = ++s->recorded;
  if (!g_gated) s->released = s->recorded;
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  if (!e->stream) return hipSuccess;
  std::lock_guard<std::mutex> l2(e->stream->mu);
  return e->stream->released >= e->ticket ? hipSuccess : hipErrorNotReady;
}

hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int) {
  *p = std::calloc(1, bytes ? bytes : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t s) {
  return on_stream(s, [=] { std::memmove(dst, src, bytes); });
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  s->capturing = true;
  s->capture = new std::vector<std::function<void()>>();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  *g = new ihipGraph{std::move(*s->capture)};
  delete s->capture;
  s->capture = nullptr;
  s->capturing = false;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  *e = new hipGraphExec{g->ops};
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  ++g_graph_launches;
  for (auto& op : e->ops) op();
  return hipSuccess;
}

// ----------------------------------------------------------------------- libveg launchers

namespace veg {

size_t bin_ws_bytes(int64_t pairs) { return 4096 + 64 * (size_t)(pairs > 0 ? pairs : 1); }

void carve_bin_ws(void* ws, int64_t, BinWs* out) {
  std::memset(out, 0, sizeof(*out));
  out->counters = (uint32_t*)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
}

hipError_t static_bin_scratch(void** out) {
  static unsigned char* buf = nullptr;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  if (!buf) buf = (unsigned char*)std::calloc(1, kStaticBinBytes + 256);   // held until exit, as the device array
  *out = (void*)(((uintptr_t)buf + 255) & ~(uintptr_t)255);
  return hipSuccess;
}

hipError_t write_blob(void* dst, const void* src, size_t bytes, hipStream_t s) {
  std::vector<unsigned char> copy((const unsigned char*)src, (const unsigned char*)src + bytes);
  return on_stream(s, [=] { std::memcpy(dst, copy.data(), bytes); });
}

hipError_t launch_project(const FrameDesc*, int, int, const KOpts&, float4*, uint32_t*, uint32_t*, bool, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_project_bwd(const FrameDesc*, int, int, const KOpts&, float*, uint32_t, const veg_grads&,
                              hipStream_t, const BwdFused&) {
  return hipSuccess;
}
hipError_t launch_bin_count(const float4*, const uint32_t*, const uint32_t*, uint32_t, const BinWs& ws, hipStream_t s,
                            const uint32_t*, uint32_t, int) {
  uint32_t* c = ws.counters;
  return on_stream(s, [=] { std::memset(c, 0, 64 * sizeof(uint32_t)); });
}
hipError_t launch_bin_sort(const FrameDesc* descs, int n_frames, const float4*, const uint32_t*, uint32_t, uint32_t,
                           const BinWs& ws, uint32_t*, uint32_t*, uint32_t*, uint32_t*, uint32_t*, uint32_t capacity,
                           hipStream_t s) {
  uint32_t* c = ws.counters;
  return on_stream(s, [=] {
    uint64_t E = 0;
    for (int f = 0; f < n_frames; ++f) E += (uint64_t)descs[f].n * (uint64_t)g_entries_per_gaussian.load();
    c[1] = (uint32_t)E;
    c[2] = (uint32_t)(E >> 32);
    c[3] = E > capacity ? 1u : 0u;
  });
}
hipError_t launch_blend_fwd(const FrameDesc* descs, int n_frames, int, int, const KOpts&, const float4*,
                            const uint32_t*, const uint32_t*, float*, float*, int32_t*, int32_t*, uint64_t*, uint64_t,
                            const uint32_t*, uint32_t*, uint64_t, hipStream_t s, const L1Fuse&) {
  return on_stream(s, [=] {
    ++g_blend_launches;
    for (int f = 0; f < n_frames; ++f) {
      const FrameDesc& d = descs[f];
      if (d.n <= 0 || !d.out_image) continue;
      ++g_blend_frames;
      d.out_image[0] = (float)d.n;
      d.out_image[1] = (float)d.W;
      d.out_image[2] = (float)d.H;
      d.out_image[3] = d.lut[0];
    }
  });
}
hipError_t launch_blend_bwd(const FrameDesc*, int, int, const KOpts&, const float4*, const uint32_t*, const uint32_t*,
                            const float*, const int32_t*, const float*, float*, uint32_t, const uint64_t*, uint64_t,
                            uint32_t*, uint64_t, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_l1(const float*, const float*, int64_t, float, double*, float*, hipStream_t) { return hipSuccess; }
hipError_t launch_fill_u32(uint32_t* dst, int64_t count, uint32_t value, hipStream_t s) {
  return on_stream(s, [=] {
    for (int64_t i = 0; i < count; ++i) dst[i] = value;
  });
}
hipError_t launch_bin_status(const uint32_t* c, int64_t* dst, hipStream_t s) {
  return on_stream(s, [=] {
    dst[0] = (int64_t)((uint64_t)c[1] | ((uint64_t)c[2] << 32));
    dst[1] = c[3];
  });
}
hipError_t launch_ssim(const float*, const float*, int64_t, int, int, float, double*, float*, float*, hipStream_t, bool,
                       float) {
  return hipSuccess;
}
hipError_t launch_adam(float*, const float*, float*, float*, int64_t, float, float, float, float, float, float,
                       hipStream_t) {
  return hipSuccess;
}
hipError_t launch_densify_stats(const FrameDesc*, int, int, const uint32_t*, const uint32_t*, const float4*,
                                const float*, float*, int32_t*, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_densify_plan(int64_t, const float*, const int32_t*, const float*, const float*, float, float, float,
                               uint8_t*, uint32_t*, uint32_t*, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_densify_apply(int64_t, const uint8_t*, const float*, const float*, const float*, const uint32_t*,
                                const uint32_t*, const DensifyFields&, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_vq_decode(const uint16_t*, int64_t, const float*, int, int, const VqFields&, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_debug_math(int, const float*, const float*, float*, int64_t, hipStream_t) { return hipSuccess; }

}  // namespace veg
