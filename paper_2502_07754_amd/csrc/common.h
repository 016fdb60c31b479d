// Internal declarations shared by the HIP translation units of libmsp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "msp.h"

#define MSP_WAVE 64

// Grow-only device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct StageTimer;

// a pair of events bracketing one stage (eager: recorded on the stream; captured: event-record nodes of a graph)
struct TimerRec {
  int stage;
  hipEvent_t a, b;
};

struct msp_ctx {
  StageTimer* timer = nullptr;
  int device = 0;
  hipStream_t stream = nullptr;
  int n_cu = 0;
  std::string err;
  // autotuned tile choice per (n_faces bucket, width, height, n_views), filled by msp_autotune
  int tuned_tile_w = 0, tuned_tile_h = 0, tuned_kbuf = 0;
  DevBuf loss_scratch, pr_keep, pr_used, pr_foff, pr_voff, pr_scan, pr_tmpi, pr_tmpf;
  // scratch of msp_point_order (Morton codes and their radix sort), grow-only
  DevBuf ord_part, ord_boxes, ord_keys0, ord_keys1, ord_vals1, ord_counts, ord_offs, ord_scan;
  bool capturing = false;
  hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
  void* noalloc_scratch = nullptr;   // this device's copy of the fixed scratch of msp_loss_noalloc
};

struct msp_state {
  // geometry of the last render
  int n_views = 0, W = 0, H = 0, tile_w = 0, tile_h = 0, ntx = 0, nty = 0, kbuf = 0, color_mode = 0;
  int64_t n_tiles = 0;       // per view
  int64_t n_faces = 0, n_verts = 0;
  const void* faces_pos = nullptr;
  const void* faces_idx = nullptr;
  float t_eps = 0.f, bg[3] = {0, 0, 0};
  int64_t entries = 0;
  int64_t max_tile = 0;
  bool rendered = false;
  msp_camera* h_cams = nullptr;  // host copy
  std::vector<double> h_camd;    // per view: camera centre and R^-1 in double (uploaded to camd)
  int h_cams_cap = 0;
  int64_t rows = 0;              // backward list rows of the last uncaptured run
  int64_t store_rows = 0;        // rows per block the forward stores lists into (0: none)
  bool lists_overflowed = false; // a render of this state overflowed its stored lists: recompute from now on
  // captured fwd+bwd step
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t graph_stream = nullptr;
  std::vector<unsigned char> graph_key;
  uint32_t* h_flag = nullptr;    // pinned host copy of the overflow flag
  int64_t graph_captures = 0, graph_replays = 0, graph_overflows = 0;
  std::vector<TimerRec> graph_timer;  // stage events captured into the graph (timing on at capture)

  DevBuf cams, geo, attr, tile_cnt, tile_off, cursor, keys, tmp, nfrag, counters,
      scan_part, blk_cap, blk_off, frag_list, col4, dcol, fp_part, crec, camd, acc64, accsh64, dcol64, det, shgv;
  int det_mode = 0;              // deterministic gradient sums requested by the last render's options
  int64_t fp_parts = 0;          // entries of fp_part written by the last render
};

// device views of a bounding-volume hierarchy's buffers (trace.hip)
struct BvhBufs {
  float* part = nullptr;       // [blocks][6] partial centroid boxes
  float* scene_box = nullptr;  // [6] centroid box (lo, hi)
  float* root_box = nullptr;   // [6] box of all faces
  uint32_t* keys[2] = {nullptr, nullptr};
  uint32_t* vals[2] = {nullptr, nullptr};
  uint32_t* counts = nullptr;  // [256][tiles] digit counts
  int64_t* offs = nullptr;     // [256 tiles + 1] their exclusive scan
  void* scan = nullptr;
  float* nodes = nullptr;      // [n - 1][16]
  float* leaves = nullptr;     // [n][16]
  int32_t* parent = nullptr;   // [n - 1]
  int32_t* lparent = nullptr;  // [n]
  uint32_t* flags = nullptr;   // [n - 1] depths of the internal nodes (level-by-level box pass)
  uint32_t* err = nullptr;     // [1] traversal-stack overflow seen by a query
};

struct msp_bvh {
  int64_t n_leaves = 0;
  DevBuf part, boxes, keys0, keys1, vals0, vals1, counts, offs, scan, nodes, leaves, parent, lparent, flags, err;
  BvhBufs view() const {
    BvhBufs b;
    b.part = (float*)part.p;
    b.scene_box = (float*)boxes.p;
    b.root_box = (float*)boxes.p + 8;
    b.keys[0] = (uint32_t*)keys0.p;
    b.keys[1] = (uint32_t*)keys1.p;
    b.vals[0] = (uint32_t*)vals0.p;
    b.vals[1] = (uint32_t*)vals1.p;
    b.counts = (uint32_t*)counts.p;
    b.offs = (int64_t*)offs.p;
    b.scan = scan.p;
    b.nodes = (float*)nodes.p;
    b.leaves = (float*)leaves.p;
    b.parent = (int32_t*)parent.p;
    b.lparent = (int32_t*)lparent.p;
    b.flags = (uint32_t*)flags.p;
    b.err = (uint32_t*)err.p;
    return b;
  }
};

// ---- error helpers (host) ----
int msp_fail(msp_ctx* ctx, int code, const std::string& msg);
#define MSP_HIP(ctx, call)                                                            \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return (msp_status)msp_fail((ctx), MSP_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

int msp_ensure(msp_ctx* ctx, DevBuf& b, size_t bytes);

// ---- launchers implemented in the kernel translation units ----
hipError_t launch_fill_u32(hipStream_t s, uint32_t* p, uint32_t v, int64_t n);
hipError_t launch_fill_f32(hipStream_t s, float* p, float v, int64_t n);

hipError_t launch_convert_flat(hipStream_t s, const msp_gaussians* g, int K, float sigma, float opac_mul,
                               const float* cos_sin, const int32_t* order, msp_faces* out);
hipError_t launch_convert_three(hipStream_t s, const msp_gaussians* g, int K, float sigma, float opac_mul,
                                const float* cos_sin, const int32_t* order, msp_faces* out);
hipError_t launch_spatial_order(hipStream_t s, const float* mean, int64_t n, const BvhBufs& b, int32_t* order);

// exclusive scan of n uint32 values into n+1 int64 offsets (last = total); scratch sized by scan_scratch_bytes
size_t scan_scratch_bytes(int64_t n);
hipError_t launch_scan_u32(hipStream_t s, const uint32_t* in, int64_t* out, int64_t n, void* scratch);

// value classes of the deterministic (fixed-point) gradient sums
enum : int { DT_POS = 0, DT_OP = 1, DT_RGB = 2, DT_COL = 3, DT_SHPOS = 4, DT_N = 5 };

struct RasterArgs {
  const float* pos;
  const float* opacity;
  const float* rgb;
  const int32_t* idx;
  int64_t n_verts, n_faces;
  const msp_camera* cams;  // device [n_views]
  int n_views, W, H, tile_w, tile_h, ntx, nty;
  int64_t n_tiles;         // per view
  float4* geo;             // [V][F][3] per-view geometry records (setup)
  float4* attr;            // [F][4] corner opacities, world corners and vertex ids
  uint32_t* tile_cnt;      // [V * n_tiles]
  int64_t* tile_off;       // [V * n_tiles + 1]
  uint32_t* cursor;        // [V * n_tiles]
  uint64_t* keys;          // [entries]
  uint64_t* tmp;           // [entries]
  int64_t key_cap;
  const float4* col4;      // SH mode: [V][F] per-view face colour (r, g, b, 0), else nullptr
  float t_eps;
  float bg0, bg1, bg2;
  float* img;              // [V][4][H][W]
  int32_t* nfrag;          // [V][H][W]
  unsigned long long* counters;  // [0] fragments, [1] restarts, [5] overflow flag, [8..15] composite queues,
                                 // [16..23] backward list queues, [24..31] backward gradient queues
  uint32_t* ovf;           // overflow flag (low word of counters[5]); set: kernels of the step return at once
  unsigned long long* fp_part;  // [views][setup workgroups] footprint pixels per setup workgroup (statistics)
  // backward
  const float* dimg;
  const int64_t* blk_off;  // [n_blocks + 1] in units of 64-slot rows
  uint2* frag_list;        // fragment lists (stored by the forward when store_rows > 0, else recomputed)
  int64_t store_rows;      // rows per 8x8 block of lists stored by the forward (0: recompute in backward)
  int64_t frag_cap;
  uint32_t* blk_cap;       // [n_blocks]
  float4* crec;            // RGB mode: [F][3] corner colours (r0 g0 b0 r1)(g1 b1 r2 g2)(b2 - - -)
  const double* camd;      // [n_views][12]: camera centre (world) and R^-1 (row-major), float64
  float* dpos;             // [3][V] caller's gradients, summed with float atomics (NULL: not wanted)
  float* dop;              // [V]
  float* drgb;             // [3][V] (RGB mode)
  float* dcol;             // SH mode: [n_views][3][F] colour gradient
  // deterministic mode (fixed-point sums)
  unsigned long long* acc64;   // [7][V]: planes dpos x, y, z, dop, drgb r, g, b
  unsigned long long* dcol64;  // SH mode: [n_views][3][F]
  uint32_t* det_max;           // [DT_N + 1]: largest |value| per class (float bits); [DT_N] bit 0: a non-finite value
  unsigned long long* det_cnt; // [DT_N]: values added per class
  const double* det_scale;     // [2 DT_N]: 2^s per class, then 2^-s
};

int sh_max_views();
hipError_t launch_sh_eval(hipStream_t s, const msp_faces* f, const msp_camera* h_cams, int n_views, float4* col4);
// SH adjoint: dsh written (if not NULL); the position terms of the colour
// direction are added into dpos [3][V] (float atomics) or, in deterministic mode
// (gv != nullptr), written per face to gv ([F], value / 3 for each corner) with
// their maxima and counts, and summed by launch_sh_fix into accsh64 [3][V]
hipError_t launch_sh_bwd(hipStream_t s, const msp_faces* f, const msp_camera* h_cams, int n_views, const float* dcol,
                         float* dsh, float* dpos, float4* gv, uint32_t* det_max, unsigned long long* det_cnt);
hipError_t launch_sh_fix(hipStream_t s, const msp_faces* f, const float4* gv, const double* scale,
                         unsigned long long* accsh64);

size_t loss_scratch_bytes(int V, int H, int W, int kind);
hipError_t launch_loss(hipStream_t s, int kind, float lambda, const float* img, const float* tgt, int V, int H, int W,
                       float* loss_out, float* dimg, void* scratch);
hipError_t launch_adam(hipStream_t s, const msp_adam_group& g, int step, float b1, float b2, float eps);
hipError_t launch_face_keep(hipStream_t s, const int32_t* idx, const float* op, int64_t F, int64_t V, float thresh,
                            uint32_t* keep, uint32_t* used);
hipError_t launch_compact_faces(hipStream_t s, const int32_t* idx, const int32_t* gid, const float* sh, int64_t F,
                                const uint32_t* keep, const int64_t* foff, const int64_t* voff, int32_t* idx2,
                                int32_t* gid2, float* sh2);
hipError_t launch_compact_rows(hipStream_t s, const float* src, int rows, int64_t V, const uint32_t* used,
                               const int64_t* voff, float* dst);
hipError_t launch_convert_rings(hipStream_t s, const msp_gaussians* g, int K, int rings, float sigma_max,
                                msp_faces* out);

// refiner (refiner.hip)
msp_refiner* refiner_new(int n_out);
void refiner_delete(msp_refiner* r);
int refiner_n_out(const msp_refiner* r);
double* refiner_part(msp_refiner* r);
hipError_t launch_refiner_targets(hipStream_t s, const msp_gaussians* g, int K, float sigma, float opac_mul,
                                  const msp_faces* tuned, float* y);
hipError_t launch_refiner_apply_backward(hipStream_t s, const msp_gaussians* g, int K, float sigma, float opac_mul,
                                         const float* y, const msp_face_grads* gr, float* dy);
hipError_t launch_refiner_weights(hipStream_t s, const msp_gaussians* g, int K, float sigma, float ref_len, float* w);
hipError_t launch_vec_mse(hipStream_t s, const float* y, const float* t, const float* w, int64_t n, float* loss,
                          float* dy, double* part);
int refiner_alloc(msp_ctx* ctx, msp_refiner* r);
int refiner_train_alloc(msp_ctx* ctx, msp_refiner* r, int64_t N);
void refiner_free_bufs(msp_refiner* r);
hipError_t launch_prior_init(hipStream_t s, const msp_mesh* m, int n, float shrink, float op0, const float rgb0[3],
                             float* logits, msp_faces* out);
hipError_t launch_prior_vertices(hipStream_t s, const msp_mesh* m, int n, const float* logits, float* pos);
hipError_t launch_prior_backward(hipStream_t s, const msp_mesh* m, int n, const float* logits, const float* dpos,
                                 float* dlogits);
hipError_t launch_bvh_build(hipStream_t s, const msp_faces* f, const BvhBufs& b);
hipError_t launch_trace_transmittance(hipStream_t s, const BvhBufs& b, int64_t n_leaves, const msp_rays* r,
                                      float t_eps, float* T, uint32_t* err);
hipError_t launch_trace_closest(hipStream_t s, const BvhBufs& b, int64_t n_leaves, const msp_rays* r, float alpha_min,
                                float* t, int32_t* face, float* u, float* v, uint32_t* err);
hipError_t launch_refiner_pack(hipStream_t s, msp_refiner* r, const float* W1, const float* b1, const float* W2,
                               const float* b2, const float* W3, const float* b3);
hipError_t launch_refiner_forward(hipStream_t s, const msp_refiner* r, const float* x, int64_t N, float* y, int n_cu);
hipError_t launch_refiner_backward(hipStream_t s, msp_refiner* r, const float* x, const float* dy, int64_t N,
                                   float* dW1, float* db1, float* dW2, float* db2, float* dW3, float* db3, float* dx,
                                   int n_cu);
hipError_t launch_refiner_features(hipStream_t s, const msp_gaussians* g, int K, float* x);
hipError_t launch_refiner_apply(hipStream_t s, const msp_gaussians* g, int K, float sigma, float opac_mul,
                                const float* y, int n_out, msp_faces* out);

hipError_t launch_setup(hipStream_t s, const RasterArgs& a);
hipError_t launch_cap_guard(hipStream_t s, const int64_t* total, int64_t cap, uint32_t* flag, uint32_t bit);
hipError_t launch_emit(hipStream_t s, const RasterArgs& a);
hipError_t launch_tile_sort(hipStream_t s, const RasterArgs& a);
hipError_t launch_composite(hipStream_t s, const RasterArgs& a, int kbuf, int n_cu);
hipError_t launch_block_max(hipStream_t s, const RasterArgs& a);
hipError_t launch_bwd_lists(hipStream_t s, const RasterArgs& a, int kbuf, int n_cu);
// mode 0: float atomics; 1: maxima and counts of the values (deterministic mode, first run);
// 2: fixed-point sums (deterministic mode, second run)
hipError_t launch_bwd_grads(hipStream_t s, const RasterArgs& a, int n_cu, int mode);
hipError_t launch_det_scales(hipStream_t s, const uint32_t* det_max, const unsigned long long* det_cnt, double* scale,
                             int c0, int c1);
hipError_t launch_dcol_finalize(hipStream_t s, const unsigned long long* dcol64, int64_t n, const double* scale,
                                float* dcol);
hipError_t launch_det_finalize(hipStream_t s, const unsigned long long* acc64, const unsigned long long* accsh64,
                               const double* scale, int64_t V, float* dpos, float* dop, float* drgb);

// ---- per-stage timing with HIP events on the context stream ----
enum MspStage {
  ST_CONVERT = 0, ST_SH_EVAL, ST_SETUP, ST_SCAN, ST_EMIT, ST_SORT, ST_COMPOSITE, ST_BLOCK_MAX, ST_BWD_LISTS,
  ST_BWD_GRADS, ST_SH_BWD, ST_OTHER, ST_COUNT
};
void timer_begin(msp_ctx* ctx, int stage);
void timer_end(msp_ctx* ctx, int stage);
