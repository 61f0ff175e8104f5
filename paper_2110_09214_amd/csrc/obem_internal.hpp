// Internal declarations of libobem: context / mesh-handle layout, error
// plumbing and constants shared by the HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <functional>
#include <string>
#include <vector>

#include "obem.h"
#include "cellmath.hpp"

namespace obem {

// CODATA 2018.
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kPi = 3.14159265358979323846;
constexpr double kQe = 1.602176634e-19;
constexpr double kMe = 9.1093837015e-31;
constexpr double kKb = 1.380649e-23;
constexpr double kAmu = 1.66053906660e-27;
constexpr double kKe = 1.0 / (4.0 * kPi * kEps0);

// Far-field regimes of the cell field (ratio of target distance from the
// cell centroid to the cell diameter D):
//   mixed: R < 3 D   -> FP64 closed form
//          R < 8 D   -> FP32 7-point degree-5 rule
//          R < 40 D  -> FP32 6-point degree-4 rule
//          else      -> FP32 3-point degree-2 rule
//   fp64:  R < 48 D  -> FP64 closed form, else FP64 7-point rule
constexpr double kNearMixed = 3.0;
constexpr double kFar3Mixed = 40.0;  // 3-point rule from here on (mixed)
constexpr double kMid6Mixed = 8.0;   // 6-point rule from here to kFar3Mixed (mixed)
// Zones of the mixed cell field (forward kernel): the cheapest rule whose
// truncation error stays below the FP32 rounding floor (about 2e-7): 7
// points from 3 D, 6 from kFwd6 D, 4 from kFwd4 D, 3 from kFar3Mixed D.
constexpr double kFwd6 = 6.0;
constexpr double kFwd4 = 16.0;
constexpr double kQuadFp64 = 48.0;
// Workgroup count that the source- or charge-split launches aim at: 64
// rounds of the 2048 workgroups resident at once (8 per CU, 256 CUs), which
// keeps the drain at the end of a launch short (measured: 3 % faster pairwise
// field than one round-robin pass of 15,625 long workgroups at 4M charges).
constexpr int kSplitWorkgroups = 131072;
// Incremental re-solve of a tracking step (resolve = 3): at most kIncMax
// changed right-hand-side entries per step, and a full refined solve after
// kIncEvery incremental updates.
constexpr int kIncMax = 4096;
constexpr int kIncEvery = 64;

// Grow-only device buffer owned by a context.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

// Workspace slots.
enum WsSlot {
  WS_BBOX = 0, WS_KEYS0, WS_KEYS1, WS_IDX0, WS_IDX1, WS_SORT_TMP, WS_TSORT, WS_ACC, WS_PART,
  WS_NN, WS_MISC0, WS_MISC1, WS_MISC2, WS_MISC3, WS_MISC4, WS_MISC5, WS_MISC6, WS_MISC7,
  WS_SOLVE0, WS_SOLVE1, WS_SOLVE2, WS_SRC, WS_SRCPERM, WS_SRCKEY, WS_SORT_TMP2, WS_TBOX, WS_MAP, WS_STATUS, WS_SRCINV, WS_PANEL,
  WS_SYMI, WS_SYMJ, WS_SYMR, WS_SYMM, WS_INC_IDX, WS_INC_DB, WS_COUNT
};

}  // namespace obem

// Number of per-cell FP64 SoA arrays kept by a bound mesh.
enum MeshField {
  MF_AX = 0, MF_AY, MF_AZ, MF_BX, MF_BY, MF_BZ, MF_CX, MF_CY, MF_CZ,  // vertices
  MF_NX, MF_NY, MF_NZ,                                                // unit normal
  MF_GX, MF_GY, MF_GZ,                                                // centroid
  MF_AREA, MF_DIAM, MF_EPS1, MF_EPS2,
  MF_Q7 = 19,            // 7 quadrature points x 3 coordinates (21 arrays)
  MF_Q3 = MF_Q7 + 21,    // 3 quadrature points x 3 coordinates (9 arrays)
  MF_Q6 = MF_Q3 + 9,     // 6 quadrature points x 3 coordinates (18 arrays)
  MF_Q4 = MF_Q6 + 18,    // outer points of the 4-point rule x 3 coordinates (9 arrays)
  MF_T = MF_Q4 + 9,      // unit tangents of the edges a->b, b->c, c->a (9 arrays)
  MF_EL = MF_T + 9,      // their lengths (3 arrays)
  MF_M = MF_EL + 3,      // in-plane outward normals t_e x n (9 arrays)
  MF_COUNT = MF_M + 9
};

namespace obem {
// The edge data of cell k from the field-major mesh block f (N cells).
__device__ __forceinline__ CellEdges cell_edges(const double *__restrict__ f, size_t N, int k) {
  CellEdges E;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    E.t[e] = mk3(f[(MF_T + 3 * e) * N + k], f[(MF_T + 3 * e + 1) * N + k], f[(MF_T + 3 * e + 2) * N + k]);
    E.m[e] = mk3(f[(MF_M + 3 * e) * N + k], f[(MF_M + 3 * e + 1) * N + k], f[(MF_M + 3 * e + 2) * N + k]);
    E.L[e] = f[(MF_EL + e) * N + k];
  }
  return E;
}
}  // namespace obem

struct obem_meshh {
  int64_t n = 0;
  int64_t n_dd = 0;
  double *f = nullptr;        // MF_COUNT x n, field-major
  int8_t *kind = nullptr;
  double bbox_lo[3], bbox_hi[3];
  double max_diam = 0;
  double *tiles = nullptr;    // per 64-cell tile: centre (3), near-zone radius (3 D)
  double *tiles48 = nullptr;  // the same for the FP64 closed-form zone (48 D)
  int32_t *order = nullptr;   // cell indices in Hilbert order of the centroids
  // last re-solve of a tracking step: its right-hand side and charges (lazy)
  double *rhs_last = nullptr, *sigma_last = nullptr;
  bool last_valid = false;
  int inc_since_solve = 0;    // incremental updates since the last full re-solve
  // collocation system (lazy)
  double *A = nullptr;        // n x n column-major
  double *LU = nullptr;       // n x n column-major
  int32_t *ipiv = nullptr;
  int64_t *ipiv64 = nullptr;  // pivots and info of the 64-bit path (n^2 >= 2^31)
  int64_t *info64 = nullptr;
  int32_t *info = nullptr;
  bool factored = false;
  double anorm_inf = 0;       // max_i sum_j |A_ij|
  // absorption grid (uniform cells over the bbox, CSR of cell -> cell ids)
  int32_t grid_n[3] = {0, 0, 0};
  double grid_lo[3], grid_h[3];
  int32_t *grid_start = nullptr;   // n_cells + 1
  int32_t *grid_items = nullptr;
  const double *field(int k) const { return f + (size_t)k * (size_t)n; }
};

struct obem_prof_rec {
  const char *name;
  hipEvent_t start, stop;
};

struct obem_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool sticky = false;
  std::string err;
  obem::DevBuf ws[obem::WS_COUNT];
  void *rocblas = nullptr;   // rocblas_handle, created on first solve
  bool prof = false;         // per-kernel event timing
  int sym_resident = 0, sym_resident_nn = 0, bwd_resident = 0;  // pair-once workgroups resident at once (lazy)
  // second stream (default priority) and events for the pair-once slot
  // reductions, which run beside the next launch (lazy)
  hipStream_t aux = nullptr;
  hipEvent_t ev_slots[2] = {}, ev_free[2] = {}, ev_join = nullptr;
  // pairwise work while profiling: device count of the directed kernel's
  // terms of pair-once calls (filled from the tile-pair mask), host counts of
  // the directed terms of the other calls and of the pair-once calls' n^2
  unsigned long long *work_dev = nullptr;
  int64_t work_directed = 0, work_once_n2 = 0;
  // the device address of the library's static scratch array on this
  // context's device, and while an allocation-free call runs, the arena that
  // ws_get carves the workspace slots from instead of allocating
  char *scratch = nullptr;
  char *arena = nullptr;
  size_t arena_bytes = 0, arena_used = 0;
  bool arena_overflow = false;
  void *arena_slot[obem::WS_COUNT] = {};
  size_t arena_slot_bytes[obem::WS_COUNT] = {};
  std::vector<obem_prof_rec> prof_recs;
  std::vector<hipEvent_t> prof_pool;
};

namespace obem {

obem_status fail(obem_ctx *ctx, obem_status st, const char *fmt, ...);
// create the context's second stream and its events on first use
obem_status aux_stream(obem_ctx *ctx);
obem_status hip_fail(obem_ctx *ctx, hipError_t e, const char *what, int line);
// Ensure workspace slot `slot` holds at least `bytes`; returns device pointer or nullptr.
void *ws_get(obem_ctx *ctx, int slot, size_t bytes);
bool is_device_ptr(const void *p);

#define OBEM_HIP(ctx, call)                                          \
  do {                                                               \
    hipError_t e_ = (call);                                          \
    if (e_ != hipSuccess) return obem::hip_fail(ctx, e_, #call, __LINE__); \
  } while (0)

// Kernel timing: PROF_BEGIN/PROF_END bracket a launch with HIP events on the
// context stream when profiling is enabled (obem_profile_enable).
int prof_begin(obem_ctx *ctx, const char *name);
void prof_end(obem_ctx *ctx, int idx);
struct ProfScope {
  obem_ctx *c;
  int idx;
  ProfScope(obem_ctx *ctx, const char *name) : c(ctx), idx(prof_begin(ctx, name)) {}
  ~ProfScope() { prof_end(c, idx); }
};
#define OBEM_PROF(ctx, name) obem::ProfScope obem_prof_scope_(ctx, name)


// Target ordering (Hilbert keys) used by the field kernels.
struct TargetOrder {
  int32_t n = 0;
  int32_t *perm = nullptr;     // sorted position -> caller index
  double *xs = nullptr;        // sorted FP64 SoA, 3 x n
};
obem_status order_targets(obem_ctx *ctx, int64_t n, const double *tx, const double *ty,
                          const double *tz, TargetOrder *out);

// Field kernels (field.hip).  acc: 4 x n FP64 accumulator in sorted order
// (Ex, Ey, Ez, V) in units of 1/k_e.
obem_status launch_panel_field(obem_ctx *ctx, const obem_meshh *m, const double *sigma,
                               const TargetOrder &to, obem_precision prec, bool want_v, double *acc);
// species_t (caller order of the targets) and species_s (source order) are
// needed only for the nearest opposite-species search (nn_idx != NULL).
// With tbox (per 256-source tile: lo xyz, hi xyz; mixed precision only) the
// search is limited to partners within nn_cut (a target with none gets
// index -1), and source tiles far from a workgroup's targets take the
// expanded form.  self_map (targets = sources): caller index -> position in
// the source arrays, NULL when the sources are in caller order.
obem_status launch_pair_field(obem_ctx *ctx, int64_t n_src, const double *sx, const double *sy,
                              const double *sz, const double *sq, const TargetOrder &to, double soft,
                              obem_precision prec, bool tgt_is_src, bool want_v, const int8_t *species_t,
                              const int8_t *species_s, double *acc, int32_t *nn_idx, double *nn_d2,
                              const double *tbox = nullptr, double nn_cut = 0.0, const int32_t *self_map = nullptr,
                              bool once = false);
// Whether the pair-once evaluation (targets = sources in one order, every
// unordered pair of particles in different super-blocks evaluated once for
// both) applies: mixed precision, softened, no potential, more than two
// super-blocks of 2048 particles and at most 2^24 particles.
bool pair_once_applies(int64_t n, obem_precision prec, double soft, bool want_v);
// Pair-once set-up for n particles in super-blocks of sym_tiles tiles: the
// super-blocks' centres and squared radii (sb, 4 per super-block) and the
// mask of tile pairs left to the directed kernel (dwpr 32-bit words per row,
// nn: also the pairs within the partner cut cut2d).  Workspace owned by ctx.
obem_status pair_once_setup(obem_ctx *ctx, int n, int sym_tiles, const double *tbox, bool nn, double cut2d,
                            double **sb, uint32_t **dmask, int *dwpr);
// The launches of one pair-once evaluation over ns super-blocks of sbsz
// particles: for d0 = 1 .. ns / 2 in steps of at most max_slots values of d
// (sized to the resident workgroups), launch(d0, dcnt, Pi, Pj) evaluates
// into FP32 partial slots on ctx->stream, and the slots are added to the FP64
// sums acc[3][n] in slot order (on the second stream, beside the next
// launch, when there is one).  Slot buffers from the workspace.
obem_status run_pair_once(obem_ctx *ctx, int n, int sbsz, int ns, int resident, int max_slots, double *acc,
                          const std::function<void(int, int, float *, float *)> &launch);

// Copy of the point sources in (charge sign, Hilbert) order with per-256-tile
// boxes (field.hip); inv (caller index -> position) when asked for.  Uses the
// target-ordering workspace: call before order_targets of the targets.
struct SourceOrder {
  int32_t n = 0;
  const double *x = nullptr, *y = nullptr, *z = nullptr, *q = nullptr;
  const double *tbox = nullptr;
  const int32_t *inv = nullptr;
  const int32_t *perm = nullptr;  // ordered position -> caller index
};
obem_status order_sources(obem_ctx *ctx, int64_t n, const double *sx, const double *sy, const double *sz,
                          const double *sq, bool want_inv, SourceOrder *out);
void launch_tile_boxes(obem_ctx *ctx, int n, const double *src, double *box);
obem_status launch_scatter(obem_ctx *ctx, const TargetOrder &to, const double *acc, double scale,
                           double *Ex, double *Ey, double *Ez, double *V);
obem_status launch_fill(obem_ctx *ctx, double *p, size_t n, double v);

// Collocation system (bem.hip).
obem_status bem_factor(obem_ctx *ctx, obem_meshh *m);
obem_status bem_solve(obem_ctx *ctx, obem_meshh *m, const double *rhs, double *sigma, int max_refine,
                      obem_solve_info *info, bool trans = false);
void bem_release(obem_meshh *m);

// Influence of point charges on the collocation left-hand side (influence.hip).
obem_status influence_rhs(obem_ctx *ctx, const obem_meshh *m, int64_t n_src, const double *sx, const double *sy,
                          const double *sz, const double *sq, const double *rhs, double *rhs_out, obem_precision prec,
                          double *vbar, double *ebx, double *eby, double *ebz);
void solver_release(obem_ctx *ctx);

// Uniform-grid field map of the static option (fieldmap.hip).
struct MapDev {
  int nx, ny, nz;
  double lo[3], h[3];
  const double *ex, *ey, *ez;
};

// Trilinear interpolation; points outside the grid box take the value at the
// nearest point of the box.
__device__ __forceinline__ void map_interp(const MapDev &g, double x, double y, double z, double E[3]) {
  const double p[3] = {x, y, z};
  const int nn[3] = {g.nx, g.ny, g.nz};
  int i0[3];
  double f[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double u = (p[c] - g.lo[c]) / g.h[c];
    u = fmin(fmax(u, 0.0), (double)(nn[c] - 1));
    int i = (int)floor(u);
    if (i > nn[c] - 2) i = nn[c] - 2;
    i0[c] = i;
    f[c] = u - (double)i;
  }
  E[0] = E[1] = E[2] = 0.0;
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
        const size_t k = ((size_t)(i0[2] + dz) * g.ny + (i0[1] + dy)) * g.nx + (i0[0] + dx);
        E[0] += w * g.ex[k];
        E[1] += w * g.ey[k];
        E[2] += w * g.ez[k];
      }
}
// Checks a caller's map (sizes >= 2, spacing > 0, device arrays) and copies it.
bool map_dev(const obem_field_map *m, MapDev *g);
// Map field at the Hilbert-sorted targets into the accumulator (units 1/k_e,
// V component 0), in place of the cell field.
obem_status launch_map_acc(obem_ctx *ctx, const MapDev &g, const TargetOrder &to, double *acc);

// Argument checks shared by the entry points (host side).
#define CHECK_CTX(ctx)                                                       \
  do {                                                                       \
    if (!(ctx)) return OBEM_EINVAL;                                          \
    if ((ctx)->sticky) return OBEM_ESTATE;                                   \
    if (hipSetDevice((ctx)->device) != hipSuccess) {                         \
      (void)hipGetLastError();                                               \
      return fail(ctx, OBEM_EDEVICE, "hipSetDevice(%d) failed", (ctx)->device); \
    }                                                                        \
  } while (0)

#define REQ_DEV(ctx, p, name)                                                             \
  do {                                                                                    \
    if (!is_device_ptr(p)) return fail(ctx, OBEM_EINVAL, "%s is NULL or not device memory", name); \
  } while (0)

#define OPT_DEV(ctx, p, name)                                                             \
  do {                                                                                    \
    if ((p) && !is_device_ptr(p)) return fail(ctx, OBEM_EINVAL, "%s is not device memory", name); \
  } while (0)

constexpr int64_t kMaxCount = (int64_t)1 << 31;

}  // namespace obem
