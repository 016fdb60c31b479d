/*
 * msp.h — C ABI of the MeshSplats hot path for AMD Instinct MI355X (gfx950).
 *
 * MeshSplats (arXiv 2502.07754) turns trained Gaussians into a soup of
 * semi-transparent triangle fans and renders that soup by depth-ordered,
 * front-to-back alpha compositing, forward and backward, so the faces can be
 * fine-tuned. This library exposes exactly those steps:
 *
 *   msp_convert          Gaussians -> fans (flat-Gaussian transformation
 *                        section: Eq. 2d_scaledrot, the vertex equation, the
 *                        fan construction and the opacity fall-off paragraph)
 *   msp_render           faces x cameras -> RGBA images (rendering section:
 *                        MVP transform, depth-peeled layers, interpolated
 *                        vertex attributes, blending through alpha)
 *   msp_render_backward  dL/dimage -> dL/d(vertex position, opacity, colour)
 *                        (fine-tuning section: the gradients its optimiser
 *                        consumes)
 *
 * Conventions shared by every call
 *   - All array arguments are DEVICE pointers owned by the caller unless a
 *     comment says "host". Arrays are structure-of-arrays, component axis
 *     first ([3][n] means x[0..n), y[0..n), z[0..n) back to back), float32 or
 *     int32, and must be 4-byte aligned (256-byte alignment is recommended for
 *     full-rate loads).
 *   - Work is enqueued on the context's HIP stream; calls return once the work
 *     is enqueued unless a comment says the call synchronises.
 *   - Every call returns an msp_status (0 = success, negative = error); no
 *     exception or abort crosses the ABI. msp_last_error() returns a
 *     NUL-terminated message for the last failure on that context. A context
 *     must not be used by two host threads at once.
 */
#ifndef MSP_H
#define MSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum msp_status {
  MSP_OK = 0,
  MSP_EINVAL = -1,     /* an argument is out of range or a required pointer is NULL */
  MSP_ENOMEM = -2,     /* a device allocation of library-owned scratch failed */
  MSP_EHIP = -3,       /* a HIP runtime call failed (message names it) */
  MSP_EOVERFLOW = -4,  /* a bounded buffer was too small and the retry failed too */
  MSP_ESTALE = -5      /* a render state was used with faces other than the ones it was made from */
} msp_status;

typedef struct msp_ctx msp_ctx;      /* library-owned: stream binding, kernels, autotune cache */
typedef struct msp_state msp_state;  /* library-owned: tile lists and per-pixel counts of one render */

/* Gaussians (the input of the conversion). n may be 0. */
typedef struct msp_gaussians {
  int64_t n;
  const float* mean;     /* [3][n] centres */
  const float* scale;    /* [3][n] linear (already exponentiated) scales, >= 0 */
  const float* quat;     /* [4][n] rotation as (w, x, y, z); normalised inside */
  const float* opacity;  /* [n] opacity in [0, 1] */
  const float* rgb;      /* [3][n] colour */
  const float* sh;       /* [48][n] degree-3 SH coefficients (row 3*basis+channel) or NULL */
} msp_gaussians;

/* Triangle soup: per-vertex position/opacity/colour, per-face vertex ids.
 * Vertex and face ids are int32, so n_verts and n_faces must be < 2^31. */
typedef struct msp_faces {
  int64_t n_verts;
  int64_t n_faces;
  float* pos;        /* [3][n_verts] world positions */
  float* opacity;    /* [n_verts] */
  float* rgb;        /* [3][n_verts] */
  float* sh;         /* [48][n_faces] or NULL: per-face SH colour instead of rgb */
  int32_t* idx;      /* [3][n_faces] vertex ids */
  int32_t* gid;      /* [n_faces] id of the Gaussian a face came from (may be NULL for render) */
} msp_faces;

/* Pinhole camera, OpenCV axes (x right, y down, z forward). Camera coordinates
 * are x_c = W[0..2] . x + W[3] (row 0), etc. for the 3x4 row-major matrix W;
 * pixel (i, j) has its centre at (i + 1/2, j + 1/2) and u = fx x_c / z_c + cx. */
typedef struct msp_camera {
  float world_to_cam[12];
  float fx, fy, cx, cy;
  float znear;           /* faces with any corner at z_c <= znear are not drawn */
  int32_t width, height; /* all views of one render share width and height */
} msp_camera;

enum { MSP_FAN_FLAT = 0, MSP_FAN_3D = 1 };       /* conversion modes */
enum { MSP_COLOR_RGB = 0, MSP_COLOR_SH3 = 1 };   /* colour source of a render */

typedef struct msp_render_opts {
  int32_t tile_w, tile_h; /* binning tile in pixels; multiples of 8 in [8, 64]; 0 = autotuned/default */
  int32_t kbuf;           /* depth of the per-pixel ordering buffer: 8, 12 or 16; 0 = default */
  int32_t color_mode;     /* MSP_COLOR_RGB or MSP_COLOR_SH3 */
  float t_eps;            /* a pixel stops once its transmittance falls below t_eps (>= 0) */
  float bg[3];            /* background colour */
  int32_t list_rows;      /* > 0: the forward stores every pixel's ordered fragment list (up to
                             list_rows fragments per pixel) for msp_render_backward, which then
                             does not recompute them; lists longer than that fall back to
                             recomputation. 0: the backward recomputes the lists (least memory). */
  int32_t deterministic;  /* 1: msp_render_backward sums the gradients in 64-bit fixed point, so
                             repeated backwards give identical bits (about 2x the gradient pass);
                             0: float atomics, whose summation order (last bits) varies by run */
} msp_render_opts;

/* Gradients, caller-owned, OVERWRITTEN by msp_render_backward (not accumulated).
 * Any pointer may be NULL to skip that output. */
typedef struct msp_face_grads {
  float* dpos;      /* [3][n_verts] */
  float* dopacity;  /* [n_verts] */
  float* drgb;      /* [3][n_verts] (RGB mode) */
  float* dsh;       /* [48][n_faces] (SH mode) */
} msp_face_grads;

typedef struct msp_render_stats {
  int64_t n_views, width, height, tile_w, tile_h;
  int64_t entries;          /* (face, tile) pairs over all views */
  int64_t max_tile_entries; /* longest tile list */
  int64_t fragments;        /* fragments composited (before early stop) over all views */
  int64_t restarts;         /* ordering-buffer overflows resolved by re-scanning a tile list */
  int64_t footprint_pixels; /* sum over drawn (view, face) of the pixel rectangle the face's corners span */
} msp_render_stats;

/* ---- context ---------------------------------------------------------- */

/* Creates a context on HIP device `device` bound to `hip_stream` (a hipStream_t
 * cast to void*, or NULL for the default stream). The stream is borrowed. */
msp_status msp_create(int device, void* hip_stream, msp_ctx** out);
msp_status msp_destroy(msp_ctx* ctx);
msp_status msp_set_stream(msp_ctx* ctx, void* hip_stream);
const char* msp_last_error(const msp_ctx* ctx);
/* Library version as major*10000 + minor*100 + patch. */
int msp_version(void);

/* ---- conversion --------------------------------------------------------- */

/* Host-only sizing: n_verts = n (K + 1), n_faces = n K for MSP_FAN_FLAT;
 * n_verts = n (7 + 3 (K - 4)), n_faces = 3 n K for MSP_FAN_3D (K a multiple
 * of 4). EINVAL if K is outside [3, 64], n < 0, the mode is unknown or the
 * counts reach 2^31. */
msp_status msp_convert_size(int64_t n, int K, int mode, int64_t* n_verts, int64_t* n_faces);

/* Gaussian -> fan conversion (flat-Gaussian transformation section).
 * Per Gaussian g with unit rotation R (columns r1..r3): the two largest scales
 * (ties to the lower index), in index order a < b, give A = sigma s_a r_a and
 * B = sigma s_b r_b (Eq. 2d_scaledrot with scale_mul = sigma and linear scales);
 * vertex g(K+1) is the mean, vertex g(K+1)+1+k is m + cos(t_k) A + sin(t_k) B
 * with t_k = -pi + 2 pi k / K (the vertex equation); face gK+k is (centre,
 * boundary k, boundary (k+1) mod K); every vertex takes the Gaussian's colour;
 * opacity is the Gaussian's at the centre and opac_mul times it on the
 * boundary. When g->sh is non-NULL each face gets its Gaussian's 48 SH
 * coefficients in out->sh. `out` arrays must be sized by msp_convert_size.
 * mode MSP_FAN_3D (3D-Gaussian section: Eq. 3d_scaledrot, one fan on each of
 * the planes of axes (1,2), (1,3), (2,3), sharing the points where the planes
 * meet): per Gaussian vertex 0 is the mean, vertices 1..6 are m + A_1, m - A_1,
 * m + A_2, m - A_2, m + A_3, m - A_3 (A_i = sigma s_i r_i), then per plane
 * (i, j) its boundary points m + cos(t_k) A_i + sin(t_k) A_j for the K - 4
 * angles off the quarter turns, in angle order; face 3Kg + pK + k is (centre,
 * point k, point (k+1) mod K) of plane p, where the quarter turns t = -pi,
 * -pi/2, 0, pi/2 are the shared points -A_i, -A_j, +A_i, +A_j.
 * EINVAL: sigma not finite and > 0, opac_mul not finite, NULL arrays with n > 0,
 * out sizes that differ from msp_convert_size, or out->sh NULL while g->sh is set. */
msp_status msp_convert(msp_ctx* ctx, const msp_gaussians* g, int K, float sigma, float opac_mul,
                       int mode, msp_faces* out);

/* A spatially coherent order of the Gaussians: order [n] (DEVICE int32) lists
 * them by the 30-bit Morton code of their means within the means' bounding
 * box (stable, so equal codes keep index order). Not in the paper: a layout
 * choice. Faces converted in this order (msp_convert_ordered) keep the faces
 * of nearby Gaussians at nearby ids, so binning writes its tile-list keys in
 * runs and neighbouring faces share cache lines. Asynchronous; the sort's
 * scratch is kept by the context (grown, with a synchronisation, when n
 * grows). EINVAL: NULL arguments with n > 0, n >= 2^31. */
msp_status msp_spatial_order(msp_ctx* ctx, const msp_gaussians* g, int32_t* order);
/* The same order for any n points [3][n] (DEVICE), e.g. ray origins. */
msp_status msp_point_order(msp_ctx* ctx, const float* points, int64_t n, int32_t* order);
/* msp_convert with the output blocks permuted: the faces and vertices of
 * output block i (the i-th group of K faces and K + 1 vertices, or 3K faces
 * and 7 + 3 (K - 4) vertices for MSP_FAN_3D) are those of Gaussian order[i],
 * and out->gid holds order[i] (so gid still names the source Gaussian).
 * order == NULL is msp_convert. An order entry outside [0, n) gives that
 * block NaN positions, zero opacity and colour and gid -1. */
msp_status msp_convert_ordered(msp_ctx* ctx, const msp_gaussians* g, int K, float sigma, float opac_mul, int mode,
                               const int32_t* order, msp_faces* out);

/* ---- rendering ---------------------------------------------------------- */

msp_status msp_state_create(msp_ctx* ctx, msp_state** out);
msp_status msp_state_free(msp_ctx* ctx, msp_state* st);

/* Renders n_views views of the face soup into img [n_views][4][H][W] (RGBA
 * planes, float32). `cams` is HOST memory (n_views entries, copied).
 * Per pixel: every face (all corners in front of znear) whose triangle
 * contains the pixel centre contributes one fragment with perspective-correct
 * barycentrics b, alpha = clamp(b . o, 0, 1) and colour b . c (RGB mode) or the
 * face's SH colour for that view (SH mode). Fragments are composited front to
 * back in exact (depth, face id) order: C += T a c, T *= 1 - a, stopping once
 * T < t_eps; RGB = C + T bg and A = 1 - T. `st` keeps the tile lists and
 * per-pixel fragment counts for msp_render_backward; the faces must stay
 * unchanged until that call. Synchronises the stream once (to size the tile
 * lists). EINVAL: n_views < 1, sizes outside [1, 16384], cameras with
 * different sizes, non-finite camera values, bad tiles, or SH mode without
 * f->sh. */
msp_status msp_render(msp_ctx* ctx, const msp_faces* f, const msp_camera* cams, int n_views,
                      const msp_render_opts* opts, float* img, msp_state* st);

/* Adjoint of the last msp_render made with `st`. dimg is [n_views][4][H][W]
 * (dL/dRGBA). The derivative freezes which fragments cover each pixel and
 * their order (no edge or visibility terms) and is exact otherwise; the
 * opacity clamp passes the gradient only where 0 < b . o < 1. Each fragment's
 * barycentrics and ray/triangle Jacobian are recomputed in float64 from the
 * world corners, so faces seen nearly edge-on keep full precision.
 * Fragment lists: when the render stored them (opts.list_rows > 0) they are
 * read as stored; this call then synchronises the stream once, to read a flag
 * telling whether some pixel had more fragments than list_rows, in which case
 * (and when list_rows = 0) it recomputes every pixel's ordered list into
 * library scratch sized on the host, which costs a second synchronisation.
 * Sums: float atomics by default (last bits vary between runs); with
 * opts.deterministic = 1 at render time, 64-bit fixed-point sums whose
 * result does not depend on the order of additions (identical bits on every
 * run, about twice the gradient pass's time and 8 bytes per summed value of
 * extra scratch). Every non-NULL gradient array is overwritten; drgb is zero
 * in SH mode; dsh (SH mode) may be NULL, the position gradient still
 * includes the colour's dependence on the view direction. ESTALE if `f` is not
 * the soup the state was rendered with. */
msp_status msp_render_backward(msp_ctx* ctx, msp_state* st, const msp_faces* f, const float* dimg,
                               msp_face_grads* grads);

/* Capacity report of a state. Synchronises the stream, then returns MSP_OK if
 * every bounded buffer of every render, backward and captured step made with
 * `st` since its creation held what it was given, and MSP_EOVERFLOW if one
 * fell short and the library recovered: stored fragment lists too short for
 * some pixel (that backward recomputed the lists, and the state recomputes
 * from then on), or a captured replay beyond the capacities of its capture
 * (the step was re-run uncaptured and captured again). Results are complete
 * in both cases; the status tells the caller that a capacity was short. */
msp_status msp_state_status(msp_ctx* ctx, msp_state* st);

/* ---- fine-tuning (fine-tuning section: loss, optimiser, pruning) ---------- */

enum { MSP_LOSS_MSE = 0, MSP_LOSS_L1 = 1, MSP_LOSS_L1_DSSIM = 2 };

/* Image loss against targets and its gradient (Eq. loss of the fine-tuning
 * section, read as lambda L1 + (1 - lambda) (1 - SSIM)).
 * img: [V][4][H][W] rendered RGBA (the alpha plane is ignored); tgt: [V][3][H][W].
 * MSE and L1 are means over V x 3 x H x W values; SSIM follows Wang et al.
 * (2004): 11x11 Gaussian window, sigma 1.5, C1 = 0.01^2, C2 = 0.03^2, valid
 * windows only, mean over windows, channels and views (needs H, W >= 11, else
 * the SSIM term is left out). loss_out: DEVICE float (written). dimg: DEVICE
 * [V][4][H][W] dL/dimg written (alpha plane zero), or NULL. lambda is used by
 * MSP_LOSS_L1_DSSIM only. Asynchronous. EINVAL on bad sizes or kind. */
msp_status msp_loss(msp_ctx* ctx, int kind, float lambda, const float* img, const float* tgt, int n_views, int height,
                    int width, float* loss_out, float* dimg);

/* Size in bytes of the fixed device scratch msp_loss_noalloc uses (one per GPU). */
#define MSP_LOSS_NOALLOC_MAX_BYTES (48ll << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid hipMalloc):
 * msp_loss with the same arguments and results, computed in a fixed device
 * buffer of MSP_LOSS_NOALLOC_MAX_BYTES per GPU that the library holds from the
 * first msp_create on that GPU until the process ends, instead of context
 * scratch. It never allocates or frees memory. The MSE and L1 losses fit at
 * any size; L1 + (1 - SSIM) needs 64 KiB + 1 KiB + 12 V (5 H W' + 3 H' W' +
 * 3 H W') bytes with W' = W - 10 and H' = H - 10 (about 132 bytes per pixel of
 * all views: 4 views of 256 x 256 fit), and larger sizes are rejected with
 * MSP_EINVAL and a message naming the bytes needed. Every call on a
 * GPU shares that GPU's buffer, which keeps the last call's contents (each
 * call writes every byte it reads, so nothing needs clearing): calls that
 * overlap in time on one GPU (other streams, other contexts) race. */
msp_status msp_loss_noalloc(msp_ctx* ctx, int kind, float lambda, const float* img, const float* tgt, int n_views,
                            int height, int width, float* loss_out, float* dimg);

/* One parameter group of an Adam step (Kingma & Ba 2015, with bias correction):
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), then p is clamped
 * to [lo, hi] when clamp != 0 (opacities: [0, 1]). All arrays DEVICE, n floats. */
typedef struct msp_adam_group {
  float* param;
  const float* grad;
  float* m;
  float* v;
  int64_t n;
  float lr;
  float lo, hi;
  int32_t clamp;
} msp_adam_group;

/* Adam update of every group in place; step counts from 1. Asynchronous. */
msp_status msp_adam_step(msp_ctx* ctx, const msp_adam_group* groups, int n_groups, int step, float beta1, float beta2,
                         float eps);

/* Pruning (last paragraph of the fine-tuning section): a face is removed when
 * all three of its vertex opacities are < thresh; then every vertex no kept
 * face uses is removed. Survivors keep their relative order; face indices are
 * renumbered. Rewrites IN PLACE, packed for the new sizes (row r of a [rows][n]
 * array starts at r * n_new): f->pos, opacity, rgb (if set), idx, gid (if
 * set), sh (if set), and each extra per-vertex array vstate[i] of
 * vstate_rows[i] rows (e.g. optimiser moments). Updates f->n_verts/n_faces and
 * writes the new sizes to *new_verts / *new_faces. Synchronises. */
msp_status msp_prune(msp_ctx* ctx, msp_faces* f, float thresh, float* const* vstate, const int* vstate_rows,
                     int n_vstate, int64_t* new_verts, int64_t* new_faces);

/* Multi-ring conversion used to render fine-tuning targets: per Gaussian a
 * centre vertex and `rings` rings of K vertices at radii sigma_max j / rings
 * (j = 1..rings, in units of the two largest scales, same axes and angles as
 * msp_convert), vertex opacity opacity exp(-r^2/2); faces: the centre fan to
 * ring 1, then two triangles per quad between consecutive rings. Sizes:
 * n (1 + rings K) vertices, n K (2 rings - 1) faces. K in [3, 64], rings in
 * [1, 16]. */
msp_status msp_rings_size(int64_t n, int K, int rings, int64_t* n_verts, int64_t* n_faces);
msp_status msp_convert_rings(msp_ctx* ctx, const msp_gaussians* g, int K, int rings, float sigma_max, msp_faces* out);

/* ---- mesh prior ---------------------------------------------------------- */

/* Mesh-prior mode (section "MeshSplats with Mesh Prior"). A fixed geometry
 * mesh (from an external reconstruction tool) carries T = n^2 secondary,
 * disjoint triangles per face; every secondary vertex is the convex
 * combination v = a_1 m_1 + a_2 m_2 + a_3 m_3 of its mesh face's corners with
 * a = softmax(theta) over three logits, so it stays on that face while the
 * logits, colours and opacities are trained. Layout: secondary face
 * f = mesh_face T + t owns vertices 3f, 3f + 1, 3f + 2; logits are [3][n_verts]
 * with row j the logit of mesh corner j. Mesh indices outside [0, n_verts)
 * give NaN positions (NaN colours at init) and zero logit gradients for that
 * face's secondary vertices; nothing is read out of bounds. */
typedef struct msp_mesh {
  int64_t n_verts, n_faces;
  const float* pos;    /* [3][n_verts] */
  const int32_t* idx;  /* [3][n_faces] */
  const float* rgb;    /* [3][n_verts] vertex colours, or NULL */
} msp_mesh;

/* Host-only sizing: n_verts = 3 n^2 n_mesh_faces, n_faces = n^2 n_mesh_faces.
 * EINVAL if n is outside [1, 16], n_mesh_faces < 0 or a count reaches 2^31. */
msp_status msp_prior_size(int64_t n_mesh_faces, int n, int64_t* n_verts, int64_t* n_faces);

/* Initial secondary triangles: sub-triangle t of the regular subdivision with
 * n segments per edge (grid point (a, b) weighs the corners ((n-a-b)/n, a/n,
 * b/n); row a = 0..n-1 holds, for b = 0, 1, ..., the upward triangle ((a,b),
 * (a+1,b), (a,b+1)) followed, while a + b <= n - 2, by the downward one
 * ((a+1,b), (a+1,b+1), (a,b+1))), each corner's weights moved `shrink` of the
 * way to its sub-triangle's centroid so that the triangles are disjoint and
 * every weight is positive; theta = log(weights). Writes logits [3][V],
 * out->idx, out->gid (mesh face of each secondary face, if not NULL),
 * out->opacity = opacity0, out->rgb = the mesh vertex colours mixed with the
 * initial weights (or rgb0, HOST [3], when m->rgb is NULL) and out->pos (as
 * msp_prior_vertices). out->sh must be NULL. EINVAL: sizes that differ from
 * msp_prior_size, shrink outside (0, 1), opacity0 outside [0, 1], NULL arrays. */
msp_status msp_prior_init(msp_ctx* ctx, const msp_mesh* m, int n, float shrink, float opacity0, const float* rgb0,
                          float* logits, msp_faces* out);
/* Secondary vertex positions pos [3][V] from logits [3][V] (per vertex a
 * max-shifted softmax in float32). EINVAL: n outside [1, 16], NULL arrays. */
msp_status msp_prior_vertices(msp_ctx* ctx, const msp_mesh* m, int n, const float* logits, float* pos);
/* Adjoint of msp_prior_vertices for the fixed mesh: with g_j = dpos . m_j,
 * dlogits_j = a_j (g_j - sum_k a_k g_k). dpos [3][V] (e.g. from
 * msp_render_backward), dlogits [3][V] overwritten. */
msp_status msp_prior_backward(msp_ctx* ctx, const msp_mesh* m, int n, const float* logits, const float* dpos,
                              float* dlogits);

/* ---- secondary rays ------------------------------------------------------ */

/* Ray tracing of the face soup, the use of the converted scene that the
 * abstract and introduction name (shadow and other secondary rays). A ray is
 * x(t) = origin + t dir for t in the open interval (tmin, tmax); it hits a
 * face when the Moller-Trumbore solution has u >= 0, v >= 0, u + v <= 1
 * (closed triangle) and a non-zero determinant (a ray in the face's plane
 * misses); faces are double-sided; the opacity at a hit is
 * alpha = clamp((1-u-v) o0 + u o1 + v o2, 0, 1), the renderer's interpolation
 * at that point. */
typedef struct msp_rays {
  int64_t n;
  const float* origin;  /* [3][n] */
  const float* dir;     /* [3][n]; any non-zero length (t is in units of |dir|) */
  const float* tmin;    /* [n] */
  const float* tmax;    /* [n], may be +inf */
  const int32_t* order; /* [n] or NULL: the order in which rays are traced (e.g. msp_point_order of the
                           origins, so that neighbouring threads walk the same nodes); results are still
                           written at each ray's own index; entries outside [0, n) are skipped */
} msp_rays;

typedef struct msp_bvh msp_bvh;  /* library-owned bounding-volume hierarchy over a face soup */

/* Builds a hierarchy over the faces (Morton order of the face centroids,
 * hierarchy of Karras 2012, boxes bottom-up), entirely on the stream. The
 * hierarchy keeps its own copy of each face's corners and opacities taken at
 * build time; rebuild after the faces change. Faces with indices outside
 * [0, n_verts) are never hit. EINVAL: NULL arguments, NULL arrays with
 * n_faces > 0. ENOMEM: device allocation failed. */
msp_status msp_bvh_build(msp_ctx* ctx, const msp_faces* f, msp_bvh** out);
msp_status msp_bvh_free(msp_ctx* ctx, msp_bvh* b);
/* Copies the hierarchy into caller DEVICE buffers (any may be NULL): nodes
 * [n-1][16] floats (child 0 box lo xyz, hi xyz, child 1 box lo xyz, hi xyz,
 * child references as int32 bits: >= 0 internal node, < 0 leaf ~j), leaves
 * [n][16] (v0 xyz, o0, e1 xyz, o1, e2 xyz, o2, face id as int32 bits, 3 unused),
 * root_box [6] (lo, hi). n = n_leaves (= n_faces). Asynchronous. */
msp_status msp_bvh_export(msp_ctx* ctx, const msp_bvh* b, float* nodes, float* leaves, float* root_box);
/* Synchronises; n_leaves, whether any query so far exceeded the 64-entry
 * traversal stack (those rays returned NaN; the hierarchy's depth bound makes
 * this unreachable), and the internal-node visits and leaf tests of all
 * queries since the build. Any output pointer may be NULL. */
msp_status msp_bvh_status(msp_ctx* ctx, const msp_bvh* b, int64_t* n_leaves, int32_t* overflowed,
                          int64_t* node_visits, int64_t* leaf_tests);
/* T [n]: product of (1 - alpha) over every hit in the interval (order-free).
 * A ray stops once T < t_eps (t_eps = 0: every hit counts). */
msp_status msp_trace_transmittance(msp_ctx* ctx, const msp_bvh* b, const msp_rays* r, float t_eps, float* T);
/* Closest hit with alpha >= alpha_min, ties to the smaller face id: t [n]
 * (+inf when none), face [n] (-1 when none), u, v [n] (barycentric weights of
 * the face's second and third corners; may be NULL). */
msp_status msp_trace_closest(msp_ctx* ctx, const msp_bvh* b, const msp_rays* r, float alpha_min, float* t,
                             int32_t* face, float* u, float* v);

/* ---- refiner: a small MLP that predicts better initial fans ------------- */

/* The refiner is not in the paper: it maps each Gaussian to corrections of its
 * fan so that fine-tuning starts closer to its optimum, and plain conversion
 * (a zero last layer) stays its fallback. Network: x (15) -> 256 -> 256 ->
 * n_out = 3K + 4, ReLU, bfloat16 operands with float32 accumulation on the
 * matrix cores; weights are float32 masters held by the caller and packed to
 * bfloat16 inside (msp_refiner_set_weights). */
typedef struct msp_refiner msp_refiner;

/* n_out in [1, 32] (3K + 4 for K <= 9). */
msp_status msp_refiner_create(msp_ctx* ctx, int n_out, msp_refiner** out);
msp_status msp_refiner_free(msp_ctx* ctx, msp_refiner* r);
/* W1 [256][15], b1 [256], W2 [256][256], b2 [256], W3 [n_out][256], b3 [n_out]: DEVICE
 * float32, row-major [out][in]. Rounded to bfloat16 (nearest, ties to even) and
 * packed; asynchronous. */
msp_status msp_refiner_set_weights(msp_ctx* ctx, msp_refiner* r, const float* W1, const float* b1, const float* W2,
                                   const float* b2, const float* W3, const float* b3);
/* Per-Gaussian inputs x [n][16] (float32; the last column is 0):
 * (mean (3), scale / 0.1 (3), unit quaternion with w >= 0 (4), opacity, rgb (3), K / 16). */
msp_status msp_refiner_features(msp_ctx* ctx, const msp_gaussians* g, int K, float* x);
/* y [n][n_out] = W3 relu(W2 relu(W1 x + b1) + b2) + b3 with x, W1, W2, W3 and
 * both hidden activations rounded to bfloat16 before each product. x is read
 * in 16-byte vectors and must be 16-byte aligned (MSP_EINVAL otherwise). */
msp_status msp_refiner_forward(msp_ctx* ctx, const msp_refiner* r, const float* x, int64_t n, float* y);
/* Gradients of sum(y * dy) over the n samples (forward recomputed from x):
 * dW1 [256][15], db1 [256], dW2 [256][256], db2 [256], dW3 [n_out][256],
 * db3 [n_out] (DEVICE, overwritten). dy, dh2 and dh1 are rounded to bfloat16
 * before each product; bias gradients sum the unrounded values. All
 * gradients are summed in a fixed order (per-block and per-wavefront partial
 * sums added in block and wave order, no float atomics), so two identical
 * calls give identical bits. dx [n][16] (DEVICE, overwritten; NULL = not computed): the
 * gradient with respect to the inputs, dh1 W1 with dh1 and W1 rounded to
 * bfloat16, in the layout of x (column 15 zero). Calls on one refiner share
 * its scratch: do not overlap them. */
msp_status msp_refiner_backward(msp_ctx* ctx, msp_refiner* r, const float* x, const float* dy, int64_t n, float* dW1,
                                float* db1, float* dW2, float* db2, float* dW3, float* db3, float* dx);
/* Fan conversion (as msp_convert, sizes from msp_convert_size) with the
 * refiner's outputs applied: boundary vertex k moves by
 * y[3k] a A^ + y[3k+1] b B^ + y[3k+2] sqrt(a b) (A^ x B^) from its plain
 * position (a = sigma s_a, b = sigma s_b, A^, B^ the unit fan axes); opacity
 * becomes clamp(o + y[3K], 0, 1) at the centre and opac_mul times that on the
 * boundary; colours rgb + y[3K+1..3K+3] on every vertex. y: [n][3K+4]. */
msp_status msp_refiner_apply(msp_ctx* ctx, const msp_gaussians* g, int K, float sigma, float opac_mul, const float* y,
                             msp_faces* out);

/* Training targets for the refiner: per Gaussian, the y* for which
 * msp_refiner_apply best matches `tuned` (a fine-tuned copy of the plain fan,
 * same vertex layout, i.e. fine-tuned without pruning) in least squares:
 * boundary offsets are the local-frame coordinates of (tuned - plain) vertex
 * positions; the opacity delta fits the centre (weight 1) and the boundary
 * (weight opac_mul) opacities; the colour delta is the mean tuned vertex colour
 * minus rgb. y: [n][3K+4]. */
msp_status msp_refiner_targets(msp_ctx* ctx, const msp_gaussians* g, int K, float sigma, float opac_mul,
                               const msp_faces* tuned, float* y);
/* Adjoint of msp_refiner_apply: given the gradients of a loss with respect to
 * the refined fan's vertex positions, opacities and colours (grads->dpos,
 * dopacity, drgb over the fan layout; NULL = zero; dsh unused), writes dL/dy
 * [n][3K+4]: boundary offset k gets a A^.dpos, b B^.dpos, sqrt(ab) n^.dpos of
 * its vertex; the opacity delta gets dop(centre) + opac_mul sum dop(boundary)
 * where 0 < opacity + delta < 1 (0 where the clamp holds); the colour delta the
 * colour gradients summed over the fan's K + 1 vertices. This lets the refiner
 * be trained through msp_render_backward on the fine-tuning loss itself. */
msp_status msp_refiner_apply_backward(msp_ctx* ctx, const msp_gaussians* g, int K, float sigma, float opac_mul,
                                      const float* y, const msp_face_grads* grads, float* dy);
/* Loss weights w [n][3K+4] for the refiner outputs of Gaussians g, so that
 * the weighted squared error of y measures the refined fan itself: offset
 * coordinate k along A, B and the normal gets (a^2, b^2, a b) / ref_len^2 with
 * a = sigma s_a, b = sigma s_b the fan's semi-axes (the squared world-space
 * displacement of that boundary vertex per unit squared error); the opacity
 * and colour deltas get a b / ref_len^2 (the fan's area relative to the same
 * K-gon of radius ref_len). EINVAL: K outside [3, 64], sigma or ref_len not
 * finite and > 0, NULL arrays with n > 0. */
msp_status msp_refiner_weights(msp_ctx* ctx, const msp_gaussians* g, int K, float sigma, float ref_len, float* w);
/* (Weighted) mean squared error between y and target ([n][n_out] each):
 * sum w (y - t)^2 / (n n_out) with w = 1 where weight is NULL; loss_out DEVICE
 * float, dy (or NULL) = d loss / d y. */
msp_status msp_refiner_loss(msp_ctx* ctx, msp_refiner* r, const float* y, const float* target, const float* weight,
                            int64_t n, float* loss_out, float* dy);

/* ---- captured steps and tuning ------------------------------------------ */

/* One forward + backward step (msp_render then msp_render_backward with the
 * same arguments) replayed as a captured HIP graph. The first call, and any
 * call whose faces, cameras, options or buffers differ from the captured ones,
 * runs the step uncaptured (which sizes the tile lists and fragment lists),
 * then captures it with 1.5x those capacities. Later calls replay the graph
 * and synchronise once to read an overflow flag; if the scene grew past a
 * capacity, the step is re-run uncaptured and captured again, so the result is
 * always complete. Results are as with msp_render / msp_render_backward.
 * An uncaptured msp_render or msp_render_backward on the same state discards
 * the captured graph (it may move the state's buffers and replaces its
 * cameras), so the next msp_step_graph captures again. */
msp_status msp_step_graph(msp_ctx* ctx, const msp_faces* f, const msp_camera* cams, int n_views,
                          const msp_render_opts* opts, float* img, const float* dimg, msp_face_grads* grads,
                          msp_state* st);
/* Graph counters of a state: captures made, replays completed, replays that overflowed. */
msp_status msp_graph_info(msp_ctx* ctx, msp_state* st, int64_t* captures, int64_t* replays, int64_t* overflows);

/* Times one render (and one backward when dimg is not NULL) for each candidate
 * tile size (8x8, 16x16, 32x16, 32x32) and ordering-buffer depth (8, 12, 16),
 * keeping the other fields of `base`; writes the fastest options to `out` and
 * makes them the context's defaults for tile_w = tile_h = kbuf = 0. img and
 * grads are scratch outputs sized as for msp_render / msp_render_backward.
 * Synchronises. */
msp_status msp_autotune(msp_ctx* ctx, const msp_faces* f, const msp_camera* cams, int n_views,
                        const msp_render_opts* base, float* img, const float* dimg, msp_face_grads* grads,
                        msp_render_opts* out);

/* ---- per-stage timing ------------------------------------------------- */

/* Number of timed stages. Index: 0 convert, 1 SH colour, 2 setup (projection,
 * footprints, tile counts, face records), 3 tile-offset scan, 4 emit, 5 tile
 * sort, 6 composite, 7 per-block list sizing, 8 backward list recompute,
 * 9 backward gradients, 10 SH adjoint, 11 other. */
#define MSP_N_STAGES 12

/* When on, every kernel stage is bracketed by a pair of HIP events recorded on
 * the context stream (adds two event records per stage; off by default). A
 * graph captured by msp_step_graph while timing is on carries the same pairs
 * as event-record nodes; msp_step_graph reads them after each replay it has
 * synchronised, so replays are timed on the stream they run on. */
msp_status msp_timing_enable(msp_ctx* ctx, int on);
/* Synchronises, then returns the summed milliseconds and call counts per stage
 * since the last read (HOST arrays of n_stages entries), and resets them. */
msp_status msp_timing_read(msp_ctx* ctx, double* ms, int64_t* calls, int n_stages);

/* Counters of the last render on `st` (synchronises). */
msp_status msp_state_stats(msp_ctx* ctx, msp_state* st, msp_render_stats* out);

/* Debug copies (synchronise). Tile lists of view `view`: offsets (HOST,
 * n_tiles + 1 int64) and sorted keys (HOST, entries uint64; key = (bits of the
 * face's nearest camera depth as float32) << 32 | face id). Pass keys = NULL
 * to read only the offsets. n_tiles = ceil(W/tile_w) ceil(H/tile_h). */
msp_status msp_debug_tiles(msp_ctx* ctx, msp_state* st, int view, int64_t* offsets, uint64_t* keys);
/* Per-pixel count of composited fragments, HOST int32 [n_views][H][W]. */
msp_status msp_debug_nfrag(msp_ctx* ctx, msp_state* st, int32_t* out);

#ifdef __cplusplus
}
#endif

#endif /* MSP_H */
