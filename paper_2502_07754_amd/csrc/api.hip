// Host side of the C ABI declared in include/msp.h: argument checking,
// library-owned scratch, and the order of kernel launches on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"

// Device scratch of msp_loss_noalloc: one fixed array per GPU, held until the
// process ends, so that call never allocates. Host code never passes this
// symbol to a kernel (on the host it is only a stand-in, not a device
// address): it uses the address hipGetSymbolAddress returns for the current
// device, resolved once per device when a context is created there.
static __device__ __align__(256) unsigned char scratch[MSP_LOSS_NOALLOC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on `device` (which must be current); nullptr on failure
void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

constexpr int kVersion = 10000;

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

bool finite_cam(const msp_camera& c) {
  for (int i = 0; i < 12; ++i)
    if (!std::isfinite(c.world_to_cam[i])) return false;
  return std::isfinite(c.fx) && std::isfinite(c.fy) && std::isfinite(c.cx) && std::isfinite(c.cy) &&
         std::isfinite(c.znear) && c.fx != 0.f && c.fy != 0.f;
}

template <class T>
T* P(const DevBuf& b) {
  return reinterpret_cast<T*>(b.p);
}

#define MSP_TIMED(ctx, stage, call) \
  do {                                \
    timer_begin((ctx), (stage));      \
    MSP_HIP((ctx), call);             \
    timer_end((ctx), (stage));        \
  } while (0)

}  // namespace

struct StageTimer {
  bool on = false;
  std::vector<TimerRec> done;     // eager stages awaiting msp_timing_read
  std::vector<TimerRec> captured; // stages recorded during the capture in progress
  double acc_ms[ST_COUNT] = {};   // graph replays read so far
  int64_t acc_calls[ST_COUNT] = {};
  std::vector<hipEvent_t> pool;
  hipEvent_t open[ST_COUNT] = {};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

// While a graph is being captured the two events become event-record nodes of
// the graph (added to the capture explicitly); every replay records them again.
static bool timer_record(msp_ctx* ctx, hipEvent_t e) {
  if (!ctx->capturing) {
    const hipError_t r = hipEventRecord(e, ctx->stream);
    if (r != hipSuccess) (void)hipGetLastError();  // timing is best effort: leave no sticky error behind
    return r == hipSuccess;
  }
  // In a capture: an event-record node after the current capture frontier, made
  // the new frontier, so the work captured next runs after it.
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipGraph_t g = nullptr;
  const hipGraphNode_t* deps = nullptr;
  size_t nd = 0;
  hipGraphNode_t node = nullptr;
  if (hipStreamGetCaptureInfo_v2(ctx->stream, &cs, nullptr, &g, &deps, &nd) != hipSuccess ||
      cs != hipStreamCaptureStatusActive || !g || hipGraphAddEventRecordNode(&node, g, deps, nd, e) != hipSuccess ||
      hipStreamUpdateCaptureDependencies(ctx->stream, &node, 1, hipStreamSetCaptureDependencies) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

void timer_begin(msp_ctx* ctx, int stage) {
  StageTimer* t = ctx->timer;
  if (!t || !t->on) return;
  hipEvent_t e = t->get();
  if (e && timer_record(ctx, e)) t->open[stage] = e;
}

void timer_end(msp_ctx* ctx, int stage) {
  StageTimer* t = ctx->timer;
  if (!t || !t->on || !t->open[stage]) return;
  hipEvent_t e = t->get();
  if (e && timer_record(ctx, e))
    (ctx->capturing ? t->captured : t->done).push_back({stage, t->open[stage], e});
  t->open[stage] = nullptr;
}

int msp_fail(msp_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int msp_ensure(msp_ctx* ctx, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return MSP_OK;
  if (b.p) {
    // the stream may still use the old buffer
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return msp_fail(ctx, MSP_EHIP, "hipStreamSynchronize");
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = bytes + bytes / 4;  // headroom against small growth
  want = (want + 255) & ~size_t(255);
  if (hipMalloc(&b.p, want) != hipSuccess) {
    b.p = nullptr;
    return msp_fail(ctx, MSP_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
  }
  b.bytes = want;
  return MSP_OK;
}

extern "C" {

int msp_version(void) { return kVersion; }

msp_status msp_create(int device, void* hip_stream, msp_ctx** out) {
  if (!out) return MSP_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return MSP_EINVAL;
  DeviceGuard g(device);
  if (!g.ok) return MSP_EHIP;
  msp_ctx* c = new msp_ctx();
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c->n_cu < 1)
    c->n_cu = 1;
  c->noalloc_scratch = scratch_address(device);
  if (!c->noalloc_scratch) {
    delete c;
    return MSP_EHIP;
  }
  *out = c;
  return MSP_OK;
}

msp_status msp_destroy(msp_ctx* ctx) {
  if (!ctx) return MSP_EINVAL;
  if (ctx->timer) {
    for (auto* v : {&ctx->timer->done, &ctx->timer->captured})
      for (auto& r : *v) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
      }
    for (hipEvent_t e : ctx->timer->pool) (void)hipEventDestroy(e);
    delete ctx->timer;
  }
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  DevBuf* bufs[] = {&ctx->loss_scratch, &ctx->pr_keep, &ctx->pr_used, &ctx->pr_foff, &ctx->pr_voff,
                    &ctx->pr_scan, &ctx->pr_tmpi, &ctx->pr_tmpf, &ctx->ord_part, &ctx->ord_boxes,
                    &ctx->ord_keys0, &ctx->ord_keys1, &ctx->ord_vals1, &ctx->ord_counts, &ctx->ord_offs,
                    &ctx->ord_scan};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  delete ctx;
  return MSP_OK;
}

msp_status msp_timing_enable(msp_ctx* ctx, int on) {
  if (!ctx) return MSP_EINVAL;
  if (!ctx->timer) ctx->timer = new StageTimer();
  ctx->timer->on = on != 0;
  return MSP_OK;
}

msp_status msp_timing_read(msp_ctx* ctx, double* ms, int64_t* calls, int n_stages) {
  if (!ctx || !ms || !calls || n_stages < 1) return MSP_EINVAL;
  for (int i = 0; i < n_stages; ++i) {
    ms[i] = 0.0;
    calls[i] = 0;
  }
  if (!ctx->timer) return MSP_OK;
  DeviceGuard dg(ctx->device);
  MSP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& r : ctx->timer->done) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
      (void)hipGetLastError();
    } else if (r.stage < n_stages) {
      ms[r.stage] += t;
      calls[r.stage] += 1;
    }
    ctx->timer->pool.push_back(r.a);
    ctx->timer->pool.push_back(r.b);
  }
  ctx->timer->done.clear();
  for (int i = 0; i < ST_COUNT && i < n_stages; ++i) {
    ms[i] += ctx->timer->acc_ms[i];
    calls[i] += ctx->timer->acc_calls[i];
    ctx->timer->acc_ms[i] = 0.0;
    ctx->timer->acc_calls[i] = 0;
  }
  return MSP_OK;
}

msp_status msp_set_stream(msp_ctx* ctx, void* hip_stream) {
  if (!ctx) return MSP_EINVAL;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return MSP_OK;
}

const char* msp_last_error(const msp_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

msp_status msp_convert_size(int64_t n, int K, int mode, int64_t* n_verts, int64_t* n_faces) {
  if (n < 0 || K < 3 || K > 64 || !n_verts || !n_faces) return MSP_EINVAL;
  if (mode == MSP_FAN_FLAT) {
    *n_verts = n * (K + 1);
    *n_faces = n * K;
  } else if (mode == MSP_FAN_3D && K % 4 == 0) {
    *n_verts = n * (7 + 3 * (K - 4));
    *n_faces = n * 3 * K;
  } else {
    return MSP_EINVAL;
  }
  if (*n_verts >= (int64_t(1) << 31) || *n_faces >= (int64_t(1) << 31)) return MSP_EINVAL;
  return MSP_OK;
}

msp_status msp_convert(msp_ctx* ctx, const msp_gaussians* g, int K, float sigma, float opac_mul, int mode,
                       msp_faces* out) {
  return msp_convert_ordered(ctx, g, K, sigma, opac_mul, mode, nullptr, out);
}

msp_status msp_convert_ordered(msp_ctx* ctx, const msp_gaussians* g, int K, float sigma, float opac_mul, int mode,
                               const int32_t* order, msp_faces* out) {
  if (!ctx) return MSP_EINVAL;
  if (!g || !out) return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_convert: null argument");
  int64_t V, F;
  if (msp_convert_size(g->n, K, mode, &V, &F) != MSP_OK)
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_convert: n, K or mode out of range");
  if (!std::isfinite(sigma) || !(sigma > 0.f) || !std::isfinite(opac_mul))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_convert: sigma must be finite and > 0, opac_mul finite");
  if (out->n_verts != V || out->n_faces != F)
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_convert: output sizes differ from msp_convert_size");
  if (g->n > 0 && (!g->mean || !g->scale || !g->quat || !g->opacity || !g->rgb || !out->pos || !out->opacity ||
                   !out->rgb || !out->idx))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_convert: null array");
  if (g->sh && !out->sh) return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_convert: g->sh set but out->sh is NULL");
  if (g->n == 0) return MSP_OK;
  DeviceGuard dg(ctx->device);
  std::vector<float> cs(2 * K);
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < K; ++k) {
    const double th = -pi + 2.0 * pi * k / K;
    cs[k] = (float)std::cos(th);
    cs[K + k] = (float)std::sin(th);
  }
  if (mode == MSP_FAN_3D)
    MSP_TIMED(ctx, ST_CONVERT, launch_convert_three(ctx->stream, g, K, sigma, opac_mul, cs.data(), order, out));
  else
    MSP_TIMED(ctx, ST_CONVERT, launch_convert_flat(ctx->stream, g, K, sigma, opac_mul, cs.data(), order, out));
  return MSP_OK;
}

static void free_graph(msp_ctx* ctx, msp_state* st);

msp_status msp_loss(msp_ctx* ctx, int kind, float lambda, const float* img, const float* tgt, int n_views, int height,
                    int width, float* loss_out, float* dimg) {
  if (!ctx) return MSP_EINVAL;
  if (!img || !tgt || !loss_out || n_views < 1 || height < 1 || width < 1 ||
      (kind != MSP_LOSS_MSE && kind != MSP_LOSS_L1 && kind != MSP_LOSS_L1_DSSIM) || !std::isfinite(lambda))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_loss: bad argument");
  DeviceGuard dg(ctx->device);
  int rc;
  if ((rc = msp_ensure(ctx, ctx->loss_scratch, loss_scratch_bytes(n_views, height, width, kind)))) return (msp_status)rc;
  MSP_TIMED(ctx, ST_OTHER, launch_loss(ctx->stream, kind, lambda, img, tgt, n_views, height, width, loss_out, dimg,
                                      ctx->loss_scratch.p));
  return MSP_OK;
}

msp_status msp_loss_noalloc(msp_ctx* ctx, int kind, float lambda, const float* img, const float* tgt, int n_views,
                            int height, int width, float* loss_out, float* dimg) {
  if (!ctx) return MSP_EINVAL;
  if (!img || !tgt || !loss_out || n_views < 1 || height < 1 || width < 1 ||
      (kind != MSP_LOSS_MSE && kind != MSP_LOSS_L1 && kind != MSP_LOSS_L1_DSSIM) || !std::isfinite(lambda))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_loss_noalloc: bad argument");
  const size_t need = loss_scratch_bytes(n_views, height, width, kind);
  if (need > (size_t)MSP_LOSS_NOALLOC_MAX_BYTES)
    return (msp_status)msp_fail(ctx, MSP_EINVAL,
                                "msp_loss_noalloc: these sizes need " + std::to_string(need) +
                                    " bytes of scratch, more than the fixed " +
                                    std::to_string((long long)MSP_LOSS_NOALLOC_MAX_BYTES) + " (use msp_loss)");
  if (!ctx->noalloc_scratch) return (msp_status)msp_fail(ctx, MSP_EHIP, "msp_loss_noalloc: no device scratch");
  DeviceGuard dg(ctx->device);
  // every scratch byte the kernels read is written earlier in the same call: nothing to clear
  MSP_TIMED(ctx, ST_OTHER, launch_loss(ctx->stream, kind, lambda, img, tgt, n_views, height, width, loss_out, dimg,
                                      ctx->noalloc_scratch));
  return MSP_OK;
}

msp_status msp_adam_step(msp_ctx* ctx, const msp_adam_group* groups, int n_groups, int step, float beta1, float beta2,
                         float eps) {
  if (!ctx) return MSP_EINVAL;
  if (!groups || n_groups < 0 || step < 1 || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps >= 0.f))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_adam_step: bad argument");
  for (int i = 0; i < n_groups; ++i)
    if (groups[i].n < 0 || (groups[i].n > 0 && (!groups[i].param || !groups[i].grad || !groups[i].m || !groups[i].v)))
      return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_adam_step: null array in a group");
  DeviceGuard dg(ctx->device);
  for (int i = 0; i < n_groups; ++i) MSP_TIMED(ctx, ST_OTHER, launch_adam(ctx->stream, groups[i], step, beta1, beta2, eps));
  return MSP_OK;
}

msp_status msp_prune(msp_ctx* ctx, msp_faces* f, float thresh, float* const* vstate, const int* vstate_rows,
                     int n_vstate, int64_t* new_verts, int64_t* new_faces) {
  if (!ctx) return MSP_EINVAL;
  if (!f || !new_verts || !new_faces || n_vstate < 0 || (n_vstate > 0 && (!vstate || !vstate_rows)))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_prune: bad argument");
  const int64_t V = f->n_verts, F = f->n_faces;
  if (F > 0 && (!f->pos || !f->opacity || !f->idx)) return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_prune: null array");
  int max_rows = 3;
  for (int i = 0; i < n_vstate; ++i) {
    if (!vstate[i] || vstate_rows[i] < 1) return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_prune: bad vstate");
    max_rows = vstate_rows[i] > max_rows ? vstate_rows[i] : max_rows;
  }
  DeviceGuard dg(ctx->device);
  hipStream_t s = ctx->stream;
  int rc;
  if ((rc = msp_ensure(ctx, ctx->pr_keep, 4 * (F + 1))) || (rc = msp_ensure(ctx, ctx->pr_used, 4 * (V + 1))) ||
      (rc = msp_ensure(ctx, ctx->pr_foff, 8 * (F + 1))) || (rc = msp_ensure(ctx, ctx->pr_voff, 8 * (V + 1))) ||
      (rc = msp_ensure(ctx, ctx->pr_scan, scan_scratch_bytes(F > V ? F : V))) ||
      (rc = msp_ensure(ctx, ctx->pr_tmpi, 4 * 4 * (F + 1))) ||
      (rc = msp_ensure(ctx, ctx->pr_tmpf, 4 * (size_t)(max_rows > 48 ? max_rows : 48) * ((V > F ? V : F) + 1))))
    return (msp_status)rc;
  uint32_t* keep = P<uint32_t>(ctx->pr_keep);
  uint32_t* used = P<uint32_t>(ctx->pr_used);
  int64_t* foff = P<int64_t>(ctx->pr_foff);
  int64_t* voff = P<int64_t>(ctx->pr_voff);
  MSP_HIP(ctx, launch_fill_u32(s, used, 0u, V));
  MSP_HIP(ctx, launch_face_keep(s, f->idx, f->opacity, F, V, thresh, keep, used));
  MSP_HIP(ctx, launch_scan_u32(s, keep, foff, F, ctx->pr_scan.p));
  MSP_HIP(ctx, launch_scan_u32(s, used, voff, V, ctx->pr_scan.p));
  int64_t F2 = 0, V2 = 0;
  MSP_HIP(ctx, hipMemcpyAsync(&F2, foff + F, 8, hipMemcpyDeviceToHost, s));
  MSP_HIP(ctx, hipMemcpyAsync(&V2, voff + V, 8, hipMemcpyDeviceToHost, s));
  MSP_HIP(ctx, hipStreamSynchronize(s));
  // faces: idx (3 rows), gid, sh through the temporaries, then back in place
  int32_t* ti = P<int32_t>(ctx->pr_tmpi);
  float* tf = P<float>(ctx->pr_tmpf);
  MSP_HIP(ctx, launch_compact_faces(s, f->idx, f->gid, nullptr, F, keep, foff, voff, ti, ti + 3 * F2, nullptr));
  MSP_HIP(ctx, hipMemcpyAsync(f->idx, ti, 4 * 3 * F2, hipMemcpyDeviceToDevice, s));
  if (f->gid) MSP_HIP(ctx, hipMemcpyAsync(f->gid, ti + 3 * F2, 4 * F2, hipMemcpyDeviceToDevice, s));
  if (f->sh) {
    // sh rows are compacted with the vertex-row kernel over the face keep flags
    MSP_HIP(ctx, launch_compact_rows(s, f->sh, 48, F, keep, foff, tf));
    MSP_HIP(ctx, hipMemcpyAsync(f->sh, tf, 4 * 48 * F2, hipMemcpyDeviceToDevice, s));
  }
  auto rows = [&](float* a, int r) -> hipError_t {
    if (!a) return hipSuccess;
    hipError_t e = launch_compact_rows(s, a, r, V, used, voff, tf);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(a, tf, 4 * (size_t)r * V2, hipMemcpyDeviceToDevice, s);
  };
  MSP_HIP(ctx, rows(f->pos, 3));
  MSP_HIP(ctx, rows(f->opacity, 1));
  MSP_HIP(ctx, rows(f->rgb, 3));
  for (int i = 0; i < n_vstate; ++i) MSP_HIP(ctx, rows(vstate[i], vstate_rows[i]));
  MSP_HIP(ctx, hipStreamSynchronize(s));
  f->n_verts = V2;
  f->n_faces = F2;
  *new_verts = V2;
  *new_faces = F2;
  return MSP_OK;
}

msp_status msp_rings_size(int64_t n, int K, int rings, int64_t* n_verts, int64_t* n_faces) {
  if (n < 0 || K < 3 || K > 64 || rings < 1 || rings > 16 || !n_verts || !n_faces) return MSP_EINVAL;
  *n_verts = n * (1 + (int64_t)rings * K);
  *n_faces = n * (int64_t)K * (2 * rings - 1);
  if (*n_verts >= (int64_t(1) << 31) || *n_faces >= (int64_t(1) << 31)) return MSP_EINVAL;
  return MSP_OK;
}

msp_status msp_convert_rings(msp_ctx* ctx, const msp_gaussians* g, int K, int rings, float sigma_max, msp_faces* out) {
  if (!ctx) return MSP_EINVAL;
  int64_t V, F;
  if (!g || !out || msp_rings_size(g->n, K, rings, &V, &F) != MSP_OK || !std::isfinite(sigma_max) || !(sigma_max > 0.f))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_convert_rings: bad argument");
  if (out->n_verts != V || out->n_faces != F)
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_convert_rings: output sizes differ from msp_rings_size");
  if (g->n > 0 && (!g->mean || !g->scale || !g->quat || !g->opacity || !g->rgb || !out->pos || !out->opacity ||
                   !out->rgb || !out->idx))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_convert_rings: null array");
  DeviceGuard dg(ctx->device);
  MSP_TIMED(ctx, ST_CONVERT, launch_convert_rings(ctx->stream, g, K, rings, sigma_max, out));
  return MSP_OK;
}

msp_status msp_prior_size(int64_t n_mesh_faces, int n, int64_t* n_verts, int64_t* n_faces) {
  if (n_mesh_faces < 0 || n < 1 || n > 16 || !n_verts || !n_faces) return MSP_EINVAL;
  const int64_t T = (int64_t)n * n;
  if (n_mesh_faces > (int64_t(1) << 31) / (3 * T)) return MSP_EINVAL;
  *n_faces = n_mesh_faces * T;
  *n_verts = 3 * *n_faces;
  if (*n_verts >= (int64_t(1) << 31)) return MSP_EINVAL;
  return MSP_OK;
}

static bool prior_mesh_ok(const msp_mesh* m) {
  return m && m->n_verts >= 0 && m->n_faces >= 0 && m->n_verts < (int64_t(1) << 31) &&
         (m->n_faces == 0 || (m->pos && m->idx));
}

msp_status msp_prior_init(msp_ctx* ctx, const msp_mesh* m, int n, float shrink, float opacity0, const float* rgb0,
                          float* logits, msp_faces* out) {
  if (!ctx) return MSP_EINVAL;
  int64_t V, F;
  if (!prior_mesh_ok(m) || !out || msp_prior_size(m->n_faces, n, &V, &F) != MSP_OK)
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_prior_init: bad mesh or n");
  if (!(shrink > 0.f && shrink < 1.f) || !(opacity0 >= 0.f && opacity0 <= 1.f))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_prior_init: shrink must be in (0, 1), opacity0 in [0, 1]");
  if (out->n_verts != V || out->n_faces != F)
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_prior_init: output sizes differ from msp_prior_size");
  if (out->sh) return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_prior_init: secondary triangles carry no SH");
  if (F > 0 && (!logits || !out->pos || !out->opacity || !out->rgb || !out->idx || (!m->rgb && !rgb0)))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_prior_init: null array");
  float c0[3] = {0.f, 0.f, 0.f};
  if (rgb0) std::copy(rgb0, rgb0 + 3, c0);
  DeviceGuard dg(ctx->device);
  MSP_TIMED(ctx, ST_CONVERT, launch_prior_init(ctx->stream, m, n, shrink, opacity0, c0, logits, out));
  MSP_TIMED(ctx, ST_CONVERT, launch_prior_vertices(ctx->stream, m, n, logits, out->pos));
  return MSP_OK;
}

msp_status msp_prior_vertices(msp_ctx* ctx, const msp_mesh* m, int n, const float* logits, float* pos) {
  if (!ctx) return MSP_EINVAL;
  int64_t V, F;
  if (!prior_mesh_ok(m) || msp_prior_size(m->n_faces, n, &V, &F) != MSP_OK)
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_prior_vertices: bad mesh or n");
  if (V > 0 && (!logits || !pos)) return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_prior_vertices: null array");
  DeviceGuard dg(ctx->device);
  MSP_TIMED(ctx, ST_CONVERT, launch_prior_vertices(ctx->stream, m, n, logits, pos));
  return MSP_OK;
}

msp_status msp_prior_backward(msp_ctx* ctx, const msp_mesh* m, int n, const float* logits, const float* dpos,
                              float* dlogits) {
  if (!ctx) return MSP_EINVAL;
  int64_t V, F;
  if (!prior_mesh_ok(m) || msp_prior_size(m->n_faces, n, &V, &F) != MSP_OK)
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_prior_backward: bad mesh or n");
  if (V > 0 && (!logits || !dpos || !dlogits))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_prior_backward: null array");
  DeviceGuard dg(ctx->device);
  MSP_TIMED(ctx, ST_OTHER, launch_prior_backward(ctx->stream, m, n, logits, dpos, dlogits));
  return MSP_OK;
}

static void bvh_release(msp_bvh* b) {
  DevBuf* bufs[] = {&b->part, &b->boxes, &b->keys0, &b->keys1, &b->vals0, &b->vals1, &b->counts, &b->offs,
                    &b->scan, &b->nodes, &b->leaves, &b->parent, &b->lparent, &b->flags, &b->err};
  for (DevBuf* d : bufs) {
    if (d->p) (void)hipFree(d->p);
    d->p = nullptr;
    d->bytes = 0;
  }
}

msp_status msp_bvh_build(msp_ctx* ctx, const msp_faces* f, msp_bvh** out) {
  if (!ctx) return MSP_EINVAL;
  if (!f || !out || f->n_faces < 0 || f->n_verts < 0 || f->n_faces >= (int64_t(1) << 31))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_bvh_build: bad argument");
  if (f->n_faces > 0 && (!f->pos || !f->opacity || !f->idx))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_bvh_build: null array");
  DeviceGuard dg(ctx->device);
  msp_bvh* b = new msp_bvh();
  const int64_t F = f->n_faces;
  const int64_t n = F > 0 ? F : 1;
  const int64_t tiles = (n + 2047) / 2048;
  int rc;
  if ((rc = msp_ensure(ctx, b->part, 6 * 1024 * sizeof(float))) || (rc = msp_ensure(ctx, b->boxes, 16 * sizeof(float))) ||
      (rc = msp_ensure(ctx, b->keys0, n * 4)) || (rc = msp_ensure(ctx, b->keys1, n * 4)) ||
      (rc = msp_ensure(ctx, b->vals0, n * 4)) || (rc = msp_ensure(ctx, b->vals1, n * 4)) ||
      (rc = msp_ensure(ctx, b->counts, 256 * tiles * 4)) || (rc = msp_ensure(ctx, b->offs, (256 * tiles + 1) * 8)) ||
      (rc = msp_ensure(ctx, b->scan, scan_scratch_bytes(256 * tiles))) || (rc = msp_ensure(ctx, b->nodes, n * 64)) ||
      (rc = msp_ensure(ctx, b->leaves, n * 64)) || (rc = msp_ensure(ctx, b->parent, n * 4)) ||
      (rc = msp_ensure(ctx, b->lparent, n * 4)) || (rc = msp_ensure(ctx, b->flags, n * 4)) ||
      (rc = msp_ensure(ctx, b->err, 256))) {
    bvh_release(b);
    delete b;
    return (msp_status)rc;
  }
  b->n_leaves = F;
  const BvhBufs v = b->view();
  hipError_t e = launch_fill_u32(ctx->stream, v.err, 0u, 8);
  if (e == hipSuccess) e = launch_bvh_build(ctx->stream, f, v);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(ctx->stream);
    bvh_release(b);
    delete b;
    return (msp_status)msp_fail(ctx, MSP_EHIP, std::string("msp_bvh_build: ") + hipGetErrorString(e));
  }
  *out = b;
  return MSP_OK;
}

msp_status msp_bvh_free(msp_ctx* ctx, msp_bvh* b) {
  if (!ctx || !b) return MSP_EINVAL;
  DeviceGuard dg(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  bvh_release(b);
  delete b;
  return MSP_OK;
}

msp_status msp_bvh_export(msp_ctx* ctx, const msp_bvh* b, float* nodes, float* leaves, float* root_box) {
  if (!ctx) return MSP_EINVAL;
  if (!b) return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_bvh_export: null hierarchy");
  DeviceGuard dg(ctx->device);
  const BvhBufs v = b->view();
  const int64_t n = b->n_leaves;
  if (nodes && n > 1) MSP_HIP(ctx, hipMemcpyAsync(nodes, v.nodes, (n - 1) * 64, hipMemcpyDeviceToDevice, ctx->stream));
  if (leaves && n > 0) MSP_HIP(ctx, hipMemcpyAsync(leaves, v.leaves, n * 64, hipMemcpyDeviceToDevice, ctx->stream));
  if (root_box) MSP_HIP(ctx, hipMemcpyAsync(root_box, v.root_box, 24, hipMemcpyDeviceToDevice, ctx->stream));
  return MSP_OK;
}

msp_status msp_bvh_status(msp_ctx* ctx, const msp_bvh* b, int64_t* n_leaves, int32_t* overflowed,
                          int64_t* node_visits, int64_t* leaf_tests) {
  if (!ctx) return MSP_EINVAL;
  if (!b) return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_bvh_status: null hierarchy");
  DeviceGuard dg(ctx->device);
  uint32_t w[6] = {0, 0, 0, 0, 0, 0};
  MSP_HIP(ctx, hipMemcpyAsync(w, b->err.p, sizeof(w), hipMemcpyDeviceToHost, ctx->stream));
  MSP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (n_leaves) *n_leaves = b->n_leaves;
  if (overflowed) *overflowed = w[0] ? 1 : 0;
  uint64_t nn, nl;
  std::memcpy(&nn, w + 2, 8);
  std::memcpy(&nl, w + 4, 8);
  if (node_visits) *node_visits = (int64_t)nn;
  if (leaf_tests) *leaf_tests = (int64_t)nl;
  return MSP_OK;
}

msp_status msp_spatial_order(msp_ctx* ctx, const msp_gaussians* g, int32_t* order) {
  if (!ctx) return MSP_EINVAL;
  if (!g) return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_spatial_order: bad argument");
  return msp_point_order(ctx, g->mean, g->n, order);
}

msp_status msp_point_order(msp_ctx* ctx, const float* points, int64_t n, int32_t* order) {
  if (!ctx) return MSP_EINVAL;
  if (n < 0 || n >= (int64_t(1) << 31) || (n > 0 && (!points || !order)))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_point_order: bad argument");
  if (n == 0) return MSP_OK;
  DeviceGuard dg(ctx->device);
  const int64_t tiles = (n + 2047) / 2048;
  int rc;
  if ((rc = msp_ensure(ctx, ctx->ord_part, 6 * 1024 * sizeof(float))) ||
      (rc = msp_ensure(ctx, ctx->ord_boxes, 16 * sizeof(float))) || (rc = msp_ensure(ctx, ctx->ord_keys0, n * 4)) ||
      (rc = msp_ensure(ctx, ctx->ord_keys1, n * 4)) || (rc = msp_ensure(ctx, ctx->ord_vals1, n * 4)) ||
      (rc = msp_ensure(ctx, ctx->ord_counts, 256 * tiles * 4)) ||
      (rc = msp_ensure(ctx, ctx->ord_offs, (256 * tiles + 1) * 8)) ||
      (rc = msp_ensure(ctx, ctx->ord_scan, scan_scratch_bytes(256 * tiles))))
    return (msp_status)rc;
  BvhBufs b;
  b.part = (float*)ctx->ord_part.p;
  b.scene_box = (float*)ctx->ord_boxes.p;
  b.keys[0] = (uint32_t*)ctx->ord_keys0.p;
  b.keys[1] = (uint32_t*)ctx->ord_keys1.p;
  b.vals[1] = (uint32_t*)ctx->ord_vals1.p;
  b.counts = (uint32_t*)ctx->ord_counts.p;
  b.offs = (int64_t*)ctx->ord_offs.p;
  b.scan = ctx->ord_scan.p;
  MSP_TIMED(ctx, ST_OTHER, launch_spatial_order(ctx->stream, points, n, b, order));
  return MSP_OK;
}

static bool rays_ok(const msp_rays* r) {
  return r && r->n >= 0 && (r->n == 0 || (r->origin && r->dir && r->tmin && r->tmax));
}

msp_status msp_trace_transmittance(msp_ctx* ctx, const msp_bvh* b, const msp_rays* r, float t_eps, float* T) {
  if (!ctx) return MSP_EINVAL;
  if (!b || !rays_ok(r) || (r->n > 0 && !T) || !(t_eps >= 0.f))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_trace_transmittance: bad argument");
  DeviceGuard dg(ctx->device);
  MSP_TIMED(ctx, ST_OTHER, launch_trace_transmittance(ctx->stream, b->view(), b->n_leaves, r, t_eps, T,
                                                      (uint32_t*)b->err.p));
  return MSP_OK;
}

msp_status msp_trace_closest(msp_ctx* ctx, const msp_bvh* b, const msp_rays* r, float alpha_min, float* t,
                             int32_t* face, float* u, float* v) {
  if (!ctx) return MSP_EINVAL;
  if (!b || !rays_ok(r) || (r->n > 0 && (!t || !face)) || !std::isfinite(alpha_min))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_trace_closest: bad argument");
  DeviceGuard dg(ctx->device);
  MSP_TIMED(ctx, ST_OTHER, launch_trace_closest(ctx->stream, b->view(), b->n_leaves, r, alpha_min, t, face, u, v,
                                                (uint32_t*)b->err.p));
  return MSP_OK;
}

msp_status msp_refiner_create(msp_ctx* ctx, int n_out, msp_refiner** out) {
  if (!ctx || !out || n_out < 1 || n_out > 32) return MSP_EINVAL;
  DeviceGuard dg(ctx->device);
  msp_refiner* r = refiner_new(n_out);
  int rc = refiner_alloc(ctx, r);
  if (rc != MSP_OK) {
    refiner_free_bufs(r);
    refiner_delete(r);
    return (msp_status)rc;
  }
  *out = r;
  return MSP_OK;
}

msp_status msp_refiner_free(msp_ctx* ctx, msp_refiner* r) {
  if (!ctx || !r) return MSP_EINVAL;
  DeviceGuard dg(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  refiner_free_bufs(r);
  refiner_delete(r);
  return MSP_OK;
}

msp_status msp_refiner_set_weights(msp_ctx* ctx, msp_refiner* r, const float* W1, const float* b1, const float* W2,
                                   const float* b2, const float* W3, const float* b3) {
  if (!ctx) return MSP_EINVAL;
  if (!r || !W1 || !b1 || !W2 || !b2 || !W3 || !b3)
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_refiner_set_weights: null argument");
  DeviceGuard dg(ctx->device);
  MSP_TIMED(ctx, ST_OTHER, launch_refiner_pack(ctx->stream, r, W1, b1, W2, b2, W3, b3));
  return MSP_OK;
}

msp_status msp_refiner_features(msp_ctx* ctx, const msp_gaussians* g, int K, float* x) {
  if (!ctx) return MSP_EINVAL;
  if (!g || !x || g->n < 0 || K < 3 || K > 64 ||
      (g->n > 0 && (!g->mean || !g->scale || !g->quat || !g->opacity || !g->rgb)))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_refiner_features: bad argument");
  DeviceGuard dg(ctx->device);
  MSP_TIMED(ctx, ST_OTHER, launch_refiner_features(ctx->stream, g, K, x));
  return MSP_OK;
}

msp_status msp_refiner_forward(msp_ctx* ctx, const msp_refiner* r, const float* x, int64_t n, float* y) {
  if (!ctx) return MSP_EINVAL;
  if (!r || n < 0 || (n > 0 && (!x || !y))) return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_refiner_forward: bad argument");
  if (((uintptr_t)x & 15) != 0) return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_refiner_forward: x not 16-byte aligned");
  DeviceGuard dg(ctx->device);
  MSP_TIMED(ctx, ST_OTHER, launch_refiner_forward(ctx->stream, r, x, n, y, ctx->n_cu));
  return MSP_OK;
}

msp_status msp_refiner_backward(msp_ctx* ctx, msp_refiner* r, const float* x, const float* dy, int64_t n, float* dW1,
                                float* db1, float* dW2, float* db2, float* dW3, float* db3, float* dx) {
  if (!ctx) return MSP_EINVAL;
  if (!r || n < 0 || (n > 0 && (!x || !dy)) || !dW1 || !db1 || !dW2 || !db2 || !dW3 || !db3)
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_refiner_backward: bad argument");
  DeviceGuard dg(ctx->device);
  int rc;
  if ((rc = refiner_train_alloc(ctx, r, n))) return (msp_status)rc;
  MSP_TIMED(ctx, ST_OTHER,
            launch_refiner_backward(ctx->stream, r, x, dy, n, dW1, db1, dW2, db2, dW3, db3, dx, ctx->n_cu));
  return MSP_OK;
}

msp_status msp_refiner_apply(msp_ctx* ctx, const msp_gaussians* g, int K, float sigma, float opac_mul, const float* y,
                             msp_faces* out) {
  if (!ctx) return MSP_EINVAL;
  int64_t V, F;
  if (!g || !out || !y || msp_convert_size(g->n, K, MSP_FAN_FLAT, &V, &F) != MSP_OK || !std::isfinite(sigma) ||
      !(sigma > 0.f) || out->n_verts != V || out->n_faces != F)
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_refiner_apply: bad argument");
  if (g->n > 0 && (!g->mean || !g->scale || !g->quat || !g->opacity || !g->rgb || !out->pos || !out->opacity ||
                   !out->rgb || !out->idx))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_refiner_apply: null array");
  DeviceGuard dg(ctx->device);
  // faces (indices, ids) as in the plain conversion, then the refined vertices
  std::vector<float> cs(2 * K);
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < K; ++k) {
    cs[k] = (float)std::cos(-pi + 2.0 * pi * k / K);
    cs[K + k] = (float)std::sin(-pi + 2.0 * pi * k / K);
  }
  MSP_TIMED(ctx, ST_CONVERT, launch_convert_flat(ctx->stream, g, K, sigma, opac_mul, cs.data(), nullptr, out));
  MSP_TIMED(ctx, ST_CONVERT, launch_refiner_apply(ctx->stream, g, K, sigma, opac_mul, y, 3 * K + 4, out));
  return MSP_OK;
}

msp_status msp_refiner_targets(msp_ctx* ctx, const msp_gaussians* g, int K, float sigma, float opac_mul,
                               const msp_faces* tuned, float* y) {
  if (!ctx) return MSP_EINVAL;
  int64_t V, F;
  if (!g || !tuned || !y || msp_convert_size(g->n, K, MSP_FAN_FLAT, &V, &F) != MSP_OK || tuned->n_verts != V ||
      !(sigma > 0.f) || (g->n > 0 && (!tuned->pos || !tuned->opacity || !tuned->rgb)))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_refiner_targets: bad argument");
  DeviceGuard dg(ctx->device);
  MSP_TIMED(ctx, ST_OTHER, launch_refiner_targets(ctx->stream, g, K, sigma, opac_mul, tuned, y));
  return MSP_OK;
}

msp_status msp_refiner_apply_backward(msp_ctx* ctx, const msp_gaussians* g, int K, float sigma, float opac_mul,
                                      const float* y, const msp_face_grads* grads, float* dy) {
  if (!ctx) return MSP_EINVAL;
  if (!g || !grads || g->n < 0 || K < 3 || K > 64 || !(sigma > 0.f) || !std::isfinite(sigma) ||
      !std::isfinite(opac_mul) || (g->n > 0 && (!g->scale || !g->quat || !g->opacity || !y || !dy)))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_refiner_apply_backward: bad argument");
  DeviceGuard dg(ctx->device);
  MSP_TIMED(ctx, ST_OTHER, launch_refiner_apply_backward(ctx->stream, g, K, sigma, opac_mul, y, grads, dy));
  return MSP_OK;
}

msp_status msp_refiner_weights(msp_ctx* ctx, const msp_gaussians* g, int K, float sigma, float ref_len, float* w) {
  if (!ctx) return MSP_EINVAL;
  if (!g || g->n < 0 || K < 3 || K > 64 || !(sigma > 0.f) || !std::isfinite(sigma) || !(ref_len > 0.f) ||
      !std::isfinite(ref_len) || (g->n > 0 && (!g->scale || !w)))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_refiner_weights: bad argument");
  DeviceGuard dg(ctx->device);
  MSP_TIMED(ctx, ST_OTHER, launch_refiner_weights(ctx->stream, g, K, sigma, ref_len, w));
  return MSP_OK;
}

msp_status msp_refiner_loss(msp_ctx* ctx, msp_refiner* r, const float* y, const float* target, const float* weight,
                            int64_t n, float* loss_out, float* dy) {
  if (!ctx) return MSP_EINVAL;
  if (!r || !loss_out || n < 0 || (n > 0 && (!y || !target)))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_refiner_loss: bad argument");
  DeviceGuard dg(ctx->device);
  MSP_TIMED(ctx, ST_OTHER,
            launch_vec_mse(ctx->stream, y, target, weight, n * refiner_n_out(r), loss_out, dy, refiner_part(r)));
  return MSP_OK;
}

msp_status msp_state_create(msp_ctx* ctx, msp_state** out) {
  if (!ctx || !out) return MSP_EINVAL;
  DeviceGuard dg(ctx->device);
  msp_state* st = new msp_state();
  if (hipHostMalloc((void**)&st->h_flag, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
    delete st;
    return (msp_status)msp_fail(ctx, MSP_ENOMEM, "hipHostMalloc of the overflow flag failed");
  }
  *st->h_flag = 0;
  *out = st;
  return MSP_OK;
}

msp_status msp_state_free(msp_ctx* ctx, msp_state* st) {
  if (!ctx || !st) return MSP_EINVAL;
  DeviceGuard dg(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  DevBuf* bufs[] = {&st->cams,  &st->geo,     &st->attr,      &st->tile_cnt, &st->tile_off, &st->cursor,
                    &st->keys,  &st->tmp,     &st->nfrag,     &st->counters, &st->scan_part, &st->blk_cap,
                    &st->blk_off, &st->frag_list, &st->col4,  &st->dcol,     &st->fp_part,  &st->crec,
                    &st->camd,  &st->acc64,   &st->accsh64,   &st->dcol64,
                    &st->det,   &st->shgv};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  free_graph(ctx, st);
  if (st->h_flag) (void)hipHostFree(st->h_flag);
  delete[] st->h_cams;
  delete st;
  return MSP_OK;
}

static void fill_args(msp_state* st, const msp_faces* f, RasterArgs& a) {
  std::memset(&a, 0, sizeof(a));
  a.pos = f->pos;
  a.opacity = f->opacity;
  a.rgb = f->rgb;
  a.idx = f->idx;
  a.n_verts = f->n_verts;
  a.n_faces = f->n_faces;
  a.cams = P<msp_camera>(st->cams);
  a.n_views = st->n_views;
  a.W = st->W;
  a.H = st->H;
  a.tile_w = st->tile_w;
  a.tile_h = st->tile_h;
  a.ntx = st->ntx;
  a.nty = st->nty;
  a.n_tiles = st->n_tiles;
  a.geo = P<float4>(st->geo);
  a.attr = P<float4>(st->attr);
  a.tile_cnt = P<uint32_t>(st->tile_cnt);
  a.tile_off = P<int64_t>(st->tile_off);
  a.cursor = P<uint32_t>(st->cursor);
  a.keys = P<uint64_t>(st->keys);
  a.tmp = P<uint64_t>(st->tmp);
  a.key_cap = (int64_t)(st->keys.bytes / sizeof(uint64_t));
  a.col4 = st->color_mode == MSP_COLOR_SH3 ? P<float4>(st->col4) : nullptr;
  a.t_eps = st->t_eps;
  a.bg0 = st->bg[0];
  a.bg1 = st->bg[1];
  a.bg2 = st->bg[2];
  a.nfrag = P<int32_t>(st->nfrag);
  a.counters = P<unsigned long long>(st->counters);
  a.ovf = reinterpret_cast<uint32_t*>(P<unsigned long long>(st->counters) + 5);
  a.fp_part = P<unsigned long long>(st->fp_part);
  a.crec = st->color_mode == MSP_COLOR_RGB ? P<float4>(st->crec) : nullptr;
  a.camd = P<double>(st->camd);
}

// Per view, in double: the camera centre -R^-1 t and R^-1 of the float32
// world-to-camera matrix [R | t] (the exact inverse, not R^T, so that a ray
// mapped to world space is the float64 image of the camera-space one).
static void camera_doubles(const msp_camera& c, double* out) {
  const float* w = c.world_to_cam;
  const double a = w[0], b = w[1], cc = w[2], d = w[4], e = w[5], f = w[6], g = w[8], h = w[9], i = w[10];
  const double det = a * (e * i - f * h) - b * (d * i - f * g) + cc * (d * h - e * g);
  const double inv[9] = {(e * i - f * h) / det, (cc * h - b * i) / det, (b * f - cc * e) / det,
                         (f * g - d * i) / det, (a * i - cc * g) / det, (cc * d - a * f) / det,
                         (d * h - e * g) / det, (b * g - a * h) / det, (a * e - b * d) / det};
  const double tx = w[3], ty = w[7], tz = w[11];
  for (int r = 0; r < 3; ++r) out[r] = -(inv[3 * r] * tx + inv[3 * r + 1] * ty + inv[3 * r + 2] * tz);
  for (int k = 0; k < 9; ++k) out[3 + k] = inv[k];
}

static msp_status render_impl(msp_ctx* ctx, const msp_faces* f, const msp_camera* cams, int n_views,
                              const msp_render_opts* opts, float* img, msp_state* st, bool graph);
static msp_status backward_impl(msp_ctx* ctx, msp_state* st, const msp_faces* f, const float* dimg,
                                msp_face_grads* grads, bool graph);

msp_status msp_render(msp_ctx* ctx, const msp_faces* f, const msp_camera* cams, int n_views,
                      const msp_render_opts* opts, float* img, msp_state* st) {
  return render_impl(ctx, f, cams, n_views, opts, img, st, false);
}

msp_status msp_render_backward(msp_ctx* ctx, msp_state* st, const msp_faces* f, const float* dimg,
                               msp_face_grads* grads) {
  return backward_impl(ctx, st, f, dimg, grads, false);
}

// In graph mode nothing may synchronise or allocate: buffer capacities come from
// an earlier uncaptured run, and a guard kernel raises the overflow flag (which
// makes every later kernel of the step return at once) when a capacity is short.
static msp_status render_impl(msp_ctx* ctx, const msp_faces* f, const msp_camera* cams, int n_views,
                              const msp_render_opts* opts, float* img, msp_state* st, bool graph) {
  if (!ctx) return MSP_EINVAL;
  auto bad = [&](const char* m) { return (msp_status)msp_fail(ctx, MSP_EINVAL, std::string("msp_render: ") + m); };
  if (!f || !cams || !opts || !img || !st) return bad("null argument");
  if (n_views < 1) return bad("n_views < 1");
  if (f->n_faces < 0 || f->n_verts < 0 || f->n_faces >= (int64_t(1) << 31) || f->n_verts >= (int64_t(1) << 31))
    return bad("face or vertex count out of range");
  if (f->n_faces > 0 && (!f->pos || !f->opacity || !f->idx)) return bad("null face array");
  if (f->n_faces > 0 && f->n_verts < 1) return bad("faces without vertices");
  const int W = cams[0].width, H = cams[0].height;
  if (W < 1 || H < 1 || W > 16384 || H > 16384) return bad("width/height outside [1, 16384]");
  for (int v = 0; v < n_views; ++v) {
    if (cams[v].width != W || cams[v].height != H) return bad("all views must share width and height");
    if (!finite_cam(cams[v])) return bad("camera has non-finite values or zero focal length");
  }
  int tw = opts->tile_w ? opts->tile_w : (ctx->tuned_tile_w ? ctx->tuned_tile_w : 16);
  int th = opts->tile_h ? opts->tile_h : (ctx->tuned_tile_h ? ctx->tuned_tile_h : 16);
  if (tw < 8 || th < 8 || tw > 64 || th > 64 || tw % 8 || th % 8) return bad("tile sizes must be multiples of 8 in [8, 64]");
  int kb = opts->kbuf ? opts->kbuf : (ctx->tuned_kbuf ? ctx->tuned_kbuf : 16);
  if (kb != 8 && kb != 12 && kb != 16) return bad("kbuf must be 8, 12 or 16");
  if (!(opts->t_eps >= 0.f) || !std::isfinite(opts->t_eps)) return bad("t_eps must be finite and >= 0");
  if (opts->color_mode != MSP_COLOR_RGB && opts->color_mode != MSP_COLOR_SH3) return bad("unknown color_mode");
  if (opts->color_mode == MSP_COLOR_RGB && f->n_faces > 0 && !f->rgb) return bad("RGB mode needs f->rgb");
  if (opts->color_mode == MSP_COLOR_SH3 && f->n_faces > 0 && !f->sh) return bad("SH mode needs f->sh");
  if (opts->color_mode == MSP_COLOR_SH3 && n_views > sh_max_views()) return bad("SH mode supports at most 64 views");
  if (opts->list_rows < 0 || opts->list_rows > 4096) return bad("list_rows must be in [0, 4096]");
  if (opts->deterministic != 0 && opts->deterministic != 1) return bad("deterministic must be 0 or 1");
  for (int v = 0; v < n_views; ++v) {
    const float* w = cams[v].world_to_cam;
    const double det = (double)w[0] * ((double)w[5] * w[10] - (double)w[6] * w[9]) -
                       (double)w[1] * ((double)w[4] * w[10] - (double)w[6] * w[8]) +
                       (double)w[2] * ((double)w[4] * w[9] - (double)w[5] * w[8]);
    if (!(std::fabs(det) > 1e-12)) return bad("camera rotation is singular");
  }

  DeviceGuard dg(ctx->device);
  // an uncaptured render may move the state's buffers and changes its cameras:
  // a graph captured before it must not be replayed
  if (!graph) free_graph(ctx, st);
  st->n_views = n_views;
  st->W = W;
  st->H = H;
  st->tile_w = tw;
  st->tile_h = th;
  st->kbuf = kb;
  st->color_mode = opts->color_mode;
  st->det_mode = opts->deterministic;
  st->ntx = (W + tw - 1) / tw;
  st->nty = (H + th - 1) / th;
  st->n_tiles = (int64_t)st->ntx * st->nty;
  st->n_faces = f->n_faces;
  st->n_verts = f->n_verts;
  st->faces_pos = f->pos;
  st->faces_idx = f->idx;
  st->t_eps = opts->t_eps;
  for (int i = 0; i < 3; ++i) st->bg[i] = opts->bg[i];
  st->rendered = false;
  const int64_t V = n_views, F = f->n_faces, NT = st->n_tiles * V;
  const int64_t npix = (int64_t)W * H * V;

  int rc;
  if ((rc = msp_ensure(ctx, st->cams, sizeof(msp_camera) * V)) ||
      (rc = msp_ensure(ctx, st->geo, 48 * V * F)) || (rc = msp_ensure(ctx, st->attr, 64 * F)) ||
      (rc = msp_ensure(ctx, st->tile_cnt, 4 * NT)) || (rc = msp_ensure(ctx, st->tile_off, 8 * (NT + 1))) ||
      (rc = msp_ensure(ctx, st->cursor, 4 * NT)) || (rc = msp_ensure(ctx, st->nfrag, 4 * npix)) ||
      (rc = msp_ensure(ctx, st->counters, 32 * 8)) || (rc = msp_ensure(ctx, st->scan_part, scan_scratch_bytes(NT))) ||
      (rc = msp_ensure(ctx, st->fp_part, 8 * V * ((F + 255) / 256))) ||
      (rc = msp_ensure(ctx, st->camd, sizeof(double) * 12 * V)) ||
      (opts->color_mode == MSP_COLOR_RGB && (rc = msp_ensure(ctx, st->crec, 48 * F))))
    return (msp_status)rc;
  st->fp_parts = F > 0 ? V * ((F + 255) / 256) : 0;
  if (st->h_cams_cap < n_views) {
    delete[] st->h_cams;
    st->h_cams = new msp_camera[n_views];
    st->h_cams_cap = n_views;
  }
  std::memcpy(st->h_cams, cams, sizeof(msp_camera) * n_views);
  st->h_camd.resize(12 * (size_t)n_views);
  for (int v = 0; v < n_views; ++v) camera_doubles(cams[v], st->h_camd.data() + 12 * v);
  hipStream_t s = ctx->stream;
  if (!graph) {
    MSP_HIP(ctx, hipMemcpyAsync(st->cams.p, st->h_cams, sizeof(msp_camera) * V, hipMemcpyHostToDevice, s));
    MSP_HIP(ctx, hipMemcpyAsync(st->camd.p, st->h_camd.data(), sizeof(double) * 12 * V, hipMemcpyHostToDevice, s));
  }
  MSP_HIP(ctx, launch_fill_u32(s, P<uint32_t>(st->tile_cnt), 0u, NT));
  MSP_HIP(ctx, launch_fill_u32(s, P<uint32_t>(st->counters), 0u, 64));

  if (opts->color_mode == MSP_COLOR_SH3) {
    if ((rc = msp_ensure(ctx, st->col4, 16 * V * F))) return (msp_status)rc;
    MSP_TIMED(ctx, ST_SH_EVAL, launch_sh_eval(s, f, st->h_cams, n_views, P<float4>(st->col4)));
  }
  RasterArgs a;
  fill_args(st, f, a);
  a.img = img;
  MSP_TIMED(ctx, ST_SETUP, launch_setup(s, a));
  MSP_TIMED(ctx, ST_SCAN, launch_scan_u32(s, a.tile_cnt, a.tile_off, NT, st->scan_part.p));
  if (graph) {
    MSP_HIP(ctx, launch_cap_guard(s, a.tile_off + NT, (int64_t)(st->keys.bytes / 8), a.ovf, 1u));
  } else {
    int64_t E = 0;
    MSP_HIP(ctx, hipMemcpyAsync(&E, a.tile_off + NT, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MSP_HIP(ctx, hipStreamSynchronize(s));
    if ((rc = msp_ensure(ctx, st->keys, 8 * E)) || (rc = msp_ensure(ctx, st->tmp, 8 * E))) return (msp_status)rc;
    st->entries = E;
  }
  fill_args(st, f, a);
  a.img = img;
  // stored fragment lists: a fixed number of rows per 8x8 block (sticky fallback to
  // recomputation once a render of this state has overflowed them)
  const int64_t nblk = V * ((W + 7) / 8) * ((H + 7) / 8);
  st->store_rows = (opts->list_rows > 0 && !st->lists_overflowed) ? opts->list_rows : 0;
  if (st->store_rows) {
    if ((rc = msp_ensure(ctx, st->frag_list, sizeof(uint2) * MSP_WAVE * nblk * st->store_rows))) {
      if (graph) return (msp_status)rc;
      st->store_rows = 0;  // not enough memory: recompute instead
    }
  }
  a.frag_list = P<uint2>(st->frag_list);
  a.store_rows = st->store_rows;
  MSP_HIP(ctx, launch_fill_u32(s, a.cursor, 0u, NT));
  MSP_TIMED(ctx, ST_EMIT, launch_emit(s, a));
  MSP_TIMED(ctx, ST_SORT, launch_tile_sort(s, a));
  MSP_TIMED(ctx, ST_COMPOSITE, launch_composite(s, a, kb, ctx->n_cu));
  st->rendered = true;
  return MSP_OK;
}

static msp_status backward_impl(msp_ctx* ctx, msp_state* st, const msp_faces* f, const float* dimg,
                                msp_face_grads* grads, bool graph) {
  if (!ctx) return MSP_EINVAL;
  auto bad = [&](const char* m) {
    return (msp_status)msp_fail(ctx, MSP_EINVAL, std::string("msp_render_backward: ") + m);
  };
  if (!st || !f || !dimg || !grads) return bad("null argument");
  if (!st->rendered) return bad("state has no render");
  if (f->pos != st->faces_pos || f->idx != st->faces_idx || f->n_faces != st->n_faces || f->n_verts != st->n_verts)
    return (msp_status)msp_fail(ctx, MSP_ESTALE, "msp_render_backward: faces differ from the rendered ones");
  const bool shm = st->color_mode == MSP_COLOR_SH3;
  if (shm && f->n_faces > 0 && !f->sh) return bad("SH render state needs f->sh");
  DeviceGuard dg(ctx->device);
  // an uncaptured backward may grow (move) the state's buffers
  if (!graph) free_graph(ctx, st);
  hipStream_t s = ctx->stream;
  const int64_t Vn = f->n_verts, F = f->n_faces, NV = st->n_views;
  const bool det = st->det_mode != 0;
  const int64_t nb = NV * ((st->W + 7) / 8) * ((st->H + 7) / 8);
  int rc;
  // gradient accumulators: float sums, or 64-bit fixed-point sums in deterministic mode
  if ((rc = msp_ensure(ctx, st->blk_cap, 4 * nb)) || (rc = msp_ensure(ctx, st->blk_off, 8 * (nb + 1))) ||
      (rc = msp_ensure(ctx, st->scan_part, scan_scratch_bytes(nb))) ||
      (det && (rc = msp_ensure(ctx, st->acc64, 7 * 8 * Vn))) ||
      (det && (rc = msp_ensure(ctx, st->det, 256))) ||
      (det && shm && (rc = msp_ensure(ctx, st->accsh64, 3 * 8 * Vn))) ||
      (det && shm && (rc = msp_ensure(ctx, st->shgv, 16 * F))) ||
      (shm && (rc = msp_ensure(ctx, st->dcol, 3 * 4 * NV * F))) ||
      (det && shm && (rc = msp_ensure(ctx, st->dcol64, 3 * 8 * NV * F))))
    return (msp_status)rc;
  RasterArgs a;
  fill_args(st, f, a);
  a.blk_cap = P<uint32_t>(st->blk_cap);
  a.blk_off = P<int64_t>(st->blk_off);
  a.dimg = dimg;
  a.dcol = shm ? P<float>(st->dcol) : nullptr;
  uint32_t* det_max = nullptr;
  unsigned long long* det_cnt = nullptr;
  double* det_scale = nullptr;
  if (det) {
    // det: [0, 64) maxima (DT_N + 1 words), [64, 128) counts, [128, 256) scales and inverses
    det_max = P<uint32_t>(st->det);
    det_cnt = reinterpret_cast<unsigned long long*>(P<unsigned char>(st->det) + 64);
    det_scale = reinterpret_cast<double*>(P<unsigned char>(st->det) + 128);
    a.acc64 = P<unsigned long long>(st->acc64);
    a.dcol64 = shm ? P<unsigned long long>(st->dcol64) : nullptr;
    a.det_max = det_max;
    a.det_cnt = det_cnt;
    a.det_scale = det_scale;
    MSP_HIP(ctx, launch_fill_u32(s, P<uint32_t>(st->det), 0u, 32));
    MSP_HIP(ctx, launch_fill_u32(s, reinterpret_cast<uint32_t*>(a.acc64), 0u, 14 * Vn));
    if (shm) {
      MSP_HIP(ctx, launch_fill_u32(s, reinterpret_cast<uint32_t*>(P<unsigned long long>(st->accsh64)), 0u, 6 * Vn));
      MSP_HIP(ctx, launch_fill_u32(s, reinterpret_cast<uint32_t*>(a.dcol64), 0u, 6 * NV * F));
    }
  } else {
    // float sums go straight into the caller's arrays
    a.dpos = grads->dpos;
    a.dop = grads->dopacity;
    a.drgb = shm ? nullptr : grads->drgb;
    if (grads->dpos) MSP_HIP(ctx, launch_fill_f32(s, grads->dpos, 0.f, 3 * Vn));
    if (grads->dopacity) MSP_HIP(ctx, launch_fill_f32(s, grads->dopacity, 0.f, Vn));
    if (grads->drgb) MSP_HIP(ctx, launch_fill_f32(s, grads->drgb, 0.f, 3 * Vn));
  }
  if (shm) MSP_HIP(ctx, launch_fill_f32(s, a.dcol, 0.f, 3 * NV * F));
  // dsh needs no clearing: the SH adjoint at the end writes all 48 F values
  if (F > 0) {
    bool stored = st->store_rows > 0;
    if (stored && !graph) {
      // lists stored by the forward are used unless a block overflowed them
      MSP_HIP(ctx, hipMemcpyAsync(st->h_flag, reinterpret_cast<uint32_t*>(P<unsigned long long>(st->counters) + 5),
                                  sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      MSP_HIP(ctx, hipStreamSynchronize(s));
      if (*st->h_flag & 4u) {
        stored = false;
        st->lists_overflowed = true;
        st->store_rows = 0;
      }
    }
    if (stored) {
      a.frag_list = P<uint2>(st->frag_list);
      a.store_rows = st->store_rows;
    } else {
      a.store_rows = 0;
      MSP_TIMED(ctx, ST_BLOCK_MAX, launch_block_max(s, a));
      MSP_HIP(ctx, launch_scan_u32(s, a.blk_cap, P<int64_t>(st->blk_off), nb, st->scan_part.p));
      if (graph) {
        MSP_HIP(ctx, launch_cap_guard(s, P<int64_t>(st->blk_off) + nb, (int64_t)(st->frag_list.bytes / (8 * MSP_WAVE)),
                                      a.ovf, 2u));
      } else {
        int64_t rows = 0;
        MSP_HIP(ctx, hipMemcpyAsync(&rows, P<int64_t>(st->blk_off) + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        MSP_HIP(ctx, hipStreamSynchronize(s));
        if ((rc = msp_ensure(ctx, st->frag_list, sizeof(uint2) * MSP_WAVE * (rows > 0 ? rows : 1))))
          return (msp_status)rc;
        st->rows = rows;
      }
      a.frag_list = P<uint2>(st->frag_list);
      a.frag_cap = (int64_t)(st->frag_list.bytes / (8 * MSP_WAVE));
      // reset the backward work queues (counters 16..31)
      MSP_HIP(ctx, launch_fill_u32(s, reinterpret_cast<uint32_t*>(P<unsigned long long>(st->counters) + 16), 0u, 32));
      MSP_TIMED(ctx, ST_BWD_LISTS, launch_bwd_lists(s, a, st->kbuf, ctx->n_cu));
    }
    uint32_t* gq = reinterpret_cast<uint32_t*>(P<unsigned long long>(st->counters) + 24);
    MSP_HIP(ctx, launch_fill_u32(s, gq, 0u, 16));
    if (!det) {
      MSP_TIMED(ctx, ST_BWD_GRADS, launch_bwd_grads(s, a, ctx->n_cu, 0));
    } else {
      // deterministic: maxima and counts, the scales, then the fixed-point sums
      MSP_TIMED(ctx, ST_BWD_GRADS, launch_bwd_grads(s, a, ctx->n_cu, 1));
      MSP_HIP(ctx, launch_det_scales(s, det_max, det_cnt, det_scale, DT_POS, DT_COL + 1));
      MSP_HIP(ctx, launch_fill_u32(s, gq, 0u, 16));
      MSP_TIMED(ctx, ST_BWD_GRADS, launch_bwd_grads(s, a, ctx->n_cu, 2));
      if (shm) MSP_HIP(ctx, launch_dcol_finalize(s, a.dcol64, 3 * NV * F, det_scale, a.dcol));
    }
    if (shm) {
      MSP_TIMED(ctx, ST_SH_BWD, launch_sh_bwd(s, f, st->h_cams, st->n_views, a.dcol, grads->dsh, det ? nullptr : grads->dpos,
                                              det ? P<float4>(st->shgv) : nullptr, det_max, det_cnt));
      if (det) {
        MSP_HIP(ctx, launch_det_scales(s, det_max, det_cnt, det_scale, DT_SHPOS, DT_SHPOS + 1));
        MSP_HIP(ctx, launch_sh_fix(s, f, P<float4>(st->shgv), det_scale, P<unsigned long long>(st->accsh64)));
      }
    }
  }
  // deterministic mode: the fixed-point sums overwrite the caller's gradients in full
  // (drgb is zero in SH mode); float mode has written them directly
  if (det)
    MSP_HIP(ctx, launch_det_finalize(s, a.acc64, shm && F > 0 ? P<unsigned long long>(st->accsh64) : nullptr,
                                     det_scale, Vn, grads->dpos, grads->dopacity, grads->drgb));
  return MSP_OK;
}

static bool same_key(const std::vector<unsigned char>& k, const std::vector<unsigned char>& m) { return k == m; }

}  // extern "C"

template <class T>
static void put(std::vector<unsigned char>& k, const T& v) {
  const unsigned char* p = reinterpret_cast<const unsigned char*>(&v);
  k.insert(k.end(), p, p + sizeof(T));
}

extern "C" {

static void free_graph(msp_ctx* ctx, msp_state* st) {
  if (st->graph_exec) (void)hipGraphExecDestroy(st->graph_exec);
  if (st->graph) (void)hipGraphDestroy(st->graph);
  st->graph_exec = nullptr;
  st->graph = nullptr;
  st->graph_key.clear();
  for (auto& r : st->graph_timer)
    for (hipEvent_t e : {r.a, r.b}) {
      if (ctx->timer) ctx->timer->pool.push_back(e);
      else (void)hipEventDestroy(e);
    }
  st->graph_timer.clear();
}

// adds the stage times of the replay that just finished (the stream has been synchronised)
static void read_graph_timer(msp_ctx* ctx, msp_state* st) {
  StageTimer* t = ctx->timer;
  if (!t || !t->on) return;
  for (auto& r : st->graph_timer) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      (void)hipGetLastError();
      continue;
    }
    if (r.stage >= 0 && r.stage < ST_COUNT) {
      t->acc_ms[r.stage] += ms;
      t->acc_calls[r.stage] += 1;
    }
  }
}

static msp_status capture_step(msp_ctx* ctx, const msp_faces* f, const msp_camera* cams, int n_views,
                               const msp_render_opts* opts, float* img, const float* dimg, msp_face_grads* grads,
                               msp_state* st) {
  hipStream_t s = ctx->stream;
  free_graph(ctx, st);
  // capacities with headroom over the uncaptured run that just sized them
  int rc;
  const int64_t ecap = st->entries + st->entries / 2 + 1024;
  const int64_t rcap = st->rows + st->rows / 2 + 64;
  if ((rc = msp_ensure(ctx, st->keys, 8 * ecap)) || (rc = msp_ensure(ctx, st->tmp, 8 * ecap)) ||
      (rc = msp_ensure(ctx, st->frag_list, 8 * MSP_WAVE * rcap)))
    return (msp_status)rc;
  MSP_HIP(ctx, hipStreamSynchronize(s));
  // capture on a private non-blocking stream (the legacy default stream cannot capture);
  // the graph is launched on the caller's stream
  if (!ctx->cap_stream) MSP_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  MSP_HIP(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
  ctx->capturing = true;
  ctx->stream = ctx->cap_stream;
  msp_status r1 = render_impl(ctx, f, cams, n_views, opts, img, st, true);
  msp_status r2 = r1 == MSP_OK ? backward_impl(ctx, st, f, dimg, grads, true) : r1;
  ctx->stream = s;
  ctx->capturing = false;
  if (ctx->timer) {
    st->graph_timer.swap(ctx->timer->captured);
    ctx->timer->captured.clear();
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
  if (r1 != MSP_OK || r2 != MSP_OK) {
    if (g) (void)hipGraphDestroy(g);
    return r1 != MSP_OK ? r1 : r2;
  }
  if (e != hipSuccess) return (msp_status)msp_fail(ctx, MSP_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  st->graph = g;
  e = hipGraphInstantiate(&st->graph_exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    free_graph(ctx, st);
    return (msp_status)msp_fail(ctx, MSP_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  return MSP_OK;
}

msp_status msp_step_graph(msp_ctx* ctx, const msp_faces* f, const msp_camera* cams, int n_views,
                          const msp_render_opts* opts, float* img, const float* dimg, msp_face_grads* grads,
                          msp_state* st) {
  if (!ctx) return MSP_EINVAL;
  if (!f || !cams || !opts || !img || !dimg || !grads || !st || n_views < 1)
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_step_graph: null argument or n_views < 1");
  DeviceGuard dg(ctx->device);
  std::vector<unsigned char> key;
  put(key, *f);
  put(key, *opts);
  put(key, *grads);
  put(key, img);
  put(key, dimg);
  put(key, n_views);
  for (int v = 0; v < n_views; ++v) put(key, cams[v]);
  hipStream_t s = ctx->stream;
  if (st->graph_exec && same_key(st->graph_key, key) && st->graph_stream == s) {
    MSP_HIP(ctx, hipGraphLaunch(st->graph_exec, s));
    uint32_t ovf = 0;
    MSP_HIP(ctx, hipMemcpyAsync(st->h_flag, P<unsigned long long>(st->counters) + 5, sizeof(uint32_t),
                                hipMemcpyDeviceToHost, s));
    MSP_HIP(ctx, hipStreamSynchronize(s));
    ovf = *st->h_flag;
    if (ovf == 0) {
      ++st->graph_replays;
      read_graph_timer(ctx, st);
      return MSP_OK;
    }
    ++st->graph_overflows;  // a capacity was short: run uncaptured and capture again
    if (ovf & 4u) {         // stored lists overflowed: recompute them from now on
      st->lists_overflowed = true;
      st->store_rows = 0;
    }
  }
  msp_status r = render_impl(ctx, f, cams, n_views, opts, img, st, false);
  if (r != MSP_OK) return r;
  r = backward_impl(ctx, st, f, dimg, grads, false);
  if (r != MSP_OK) return r;
  r = capture_step(ctx, f, cams, n_views, opts, img, dimg, grads, st);
  if (r != MSP_OK) return r;
  st->graph_key = key;
  st->graph_stream = s;
  ++st->graph_captures;
  return MSP_OK;
}

msp_status msp_autotune(msp_ctx* ctx, const msp_faces* f, const msp_camera* cams, int n_views,
                        const msp_render_opts* base, float* img, const float* dimg, msp_face_grads* grads,
                        msp_render_opts* out) {
  if (!ctx) return MSP_EINVAL;
  if (!f || !cams || !base || !img || !out || n_views < 1 || (dimg && !grads))
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_autotune: null argument or n_views < 1");
  DeviceGuard dg(ctx->device);
  static const int cand[][3] = {{8, 8, 16},  {16, 16, 16}, {32, 16, 16}, {32, 32, 16},
                                {16, 16, 8}, {32, 16, 8},  {16, 16, 12}, {32, 16, 12}};
  msp_state* st = nullptr;
  msp_status r = msp_state_create(ctx, &st);
  if (r != MSP_OK) return r;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    msp_state_free(ctx, st);
    return (msp_status)msp_fail(ctx, MSP_EHIP, "msp_autotune: hipEventCreate");
  }
  float best = 1e30f;
  msp_render_opts best_o = *base;
  const bool timer_on = ctx->timer && ctx->timer->on;
  if (timer_on) ctx->timer->on = false;
  for (const auto& c : cand) {
    msp_render_opts o = *base;
    o.tile_w = c[0];
    o.tile_h = c[1];
    o.kbuf = c[2];
    float ms = 0.f;
    for (int rep = 0; rep < 2 && r == MSP_OK; ++rep) {  // rep 0 warms up and sizes the scratch
      if (hipEventRecord(e0, ctx->stream) != hipSuccess) r = MSP_EHIP;
      if (r == MSP_OK) r = render_impl(ctx, f, cams, n_views, &o, img, st, false);
      if (r == MSP_OK && dimg) r = backward_impl(ctx, st, f, dimg, grads, false);
      if (r == MSP_OK && hipEventRecord(e1, ctx->stream) != hipSuccess) r = MSP_EHIP;
      if (r == MSP_OK && hipEventSynchronize(e1) != hipSuccess) r = MSP_EHIP;
      if (r == MSP_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) r = MSP_EHIP;
    }
    if (r != MSP_OK) break;
    if (ms < best) {
      best = ms;
      best_o = o;
    }
  }
  if (timer_on) ctx->timer->on = true;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  msp_state_free(ctx, st);
  if (r != MSP_OK) return r;
  *out = best_o;
  ctx->tuned_tile_w = best_o.tile_w;
  ctx->tuned_tile_h = best_o.tile_h;
  ctx->tuned_kbuf = best_o.kbuf;
  return MSP_OK;
}

msp_status msp_state_status(msp_ctx* ctx, msp_state* st) {
  if (!ctx || !st) return MSP_EINVAL;
  DeviceGuard dg(ctx->device);
  MSP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return (st->lists_overflowed || st->graph_overflows > 0) ? MSP_EOVERFLOW : MSP_OK;
}

msp_status msp_graph_info(msp_ctx* ctx, msp_state* st, int64_t* captures, int64_t* replays, int64_t* overflows) {
  if (!ctx || !st || !captures || !replays || !overflows) return MSP_EINVAL;
  *captures = st->graph_captures;
  *replays = st->graph_replays;
  *overflows = st->graph_overflows;
  return MSP_OK;
}

msp_status msp_state_stats(msp_ctx* ctx, msp_state* st, msp_render_stats* out) {
  if (!ctx || !st || !out) return MSP_EINVAL;
  if (!st->rendered) return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_state_stats: no render");
  DeviceGuard dg(ctx->device);
  MSP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  unsigned long long c[8];
  MSP_HIP(ctx, hipMemcpy(c, st->counters.p, sizeof(c), hipMemcpyDeviceToHost));
  const int64_t NT = st->n_tiles * st->n_views;
  std::vector<int64_t> off(NT + 1);
  MSP_HIP(ctx, hipMemcpy(off.data(), st->tile_off.p, sizeof(int64_t) * (NT + 1), hipMemcpyDeviceToHost));
  int64_t mx = 0;
  for (int64_t t = 0; t < NT; ++t) mx = off[t + 1] - off[t] > mx ? off[t + 1] - off[t] : mx;
  out->n_views = st->n_views;
  out->width = st->W;
  out->height = st->H;
  out->tile_w = st->tile_w;
  out->tile_h = st->tile_h;
  out->entries = st->entries;
  out->max_tile_entries = mx;
  out->fragments = (int64_t)c[0];
  out->restarts = (int64_t)c[1];
  std::vector<unsigned long long> fp((size_t)st->fp_parts);
  if (st->fp_parts)
    MSP_HIP(ctx, hipMemcpy(fp.data(), st->fp_part.p, sizeof(unsigned long long) * st->fp_parts, hipMemcpyDeviceToHost));
  int64_t fps = 0;
  for (unsigned long long v : fp) fps += (int64_t)v;
  out->footprint_pixels = fps;
  return MSP_OK;
}

msp_status msp_debug_tiles(msp_ctx* ctx, msp_state* st, int view, int64_t* offsets, uint64_t* keys) {
  if (!ctx || !st || !offsets) return MSP_EINVAL;
  if (!st->rendered || view < 0 || view >= st->n_views)
    return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_debug_tiles: no render or bad view");
  DeviceGuard dg(ctx->device);
  MSP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const int64_t nt = st->n_tiles;
  MSP_HIP(ctx, hipMemcpy(offsets, P<int64_t>(st->tile_off) + view * nt, sizeof(int64_t) * (nt + 1),
                         hipMemcpyDeviceToHost));
  const int64_t b = offsets[0];
  for (int64_t t = 0; t <= nt; ++t) offsets[t] -= b;
  if (keys && offsets[nt] > 0)
    MSP_HIP(ctx, hipMemcpy(keys, P<uint64_t>(st->keys) + b, sizeof(uint64_t) * offsets[nt], hipMemcpyDeviceToHost));
  return MSP_OK;
}

msp_status msp_debug_nfrag(msp_ctx* ctx, msp_state* st, int32_t* out) {
  if (!ctx || !st || !out) return MSP_EINVAL;
  if (!st->rendered) return (msp_status)msp_fail(ctx, MSP_EINVAL, "msp_debug_nfrag: no render");
  DeviceGuard dg(ctx->device);
  MSP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  MSP_HIP(ctx, hipMemcpy(out, st->nfrag.p, sizeof(int32_t) * st->n_views * st->W * st->H, hipMemcpyDeviceToHost));
  return MSP_OK;
}

}  // extern "C"
