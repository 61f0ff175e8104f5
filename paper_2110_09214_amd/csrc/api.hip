// C ABI entry points of libobem: contexts, argument validation, mesh binding
// and the field evaluation driver.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <vector>

#include "cellmath.hpp"
#include "obem_internal.hpp"

namespace obem {

obem_status fail(obem_ctx *ctx, obem_status st, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

obem_status hip_fail(obem_ctx *ctx, hipError_t e, const char *what, int line) {
  if (ctx) {
    ctx->sticky = true;
    char buf[512];
    snprintf(buf, sizeof buf, "HIP error %d (%s) in %s [line %d]", (int)e, hipGetErrorString(e), what, line);
    ctx->err = buf;
  }
  return OBEM_EDEVICE;
}

void *ws_get(obem_ctx *ctx, int slot, size_t bytes) {
  if (slot < 0 || slot >= WS_COUNT) return nullptr;
  if (bytes == 0) bytes = 1;
  if (ctx->arena) {
    // allocation-free call: slices of the scratch array, one per slot (a
    // slot asked for again gets its slice back if it is large enough, as a
    // grow-only buffer would be)
    if (ctx->arena_slot_bytes[slot] >= bytes) return ctx->arena_slot[slot];
    const size_t want = (bytes + 255) / 256 * 256;
    if (want > ctx->arena_bytes - ctx->arena_used) {
      ctx->arena_overflow = true;
      return nullptr;
    }
    void *p = ctx->arena + ctx->arena_used;
    ctx->arena_used += want;
    ctx->arena_slot[slot] = p;
    ctx->arena_slot_bytes[slot] = want;
    return p;
  }
  DevBuf &b = ctx->ws[slot];
  if (b.bytes >= bytes) return b.p;
  if (b.p) {
    // the buffer may still be in use by queued work on the context stream
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = std::max(bytes, (size_t)4096);
  want = (want + 255) / 256 * 256;
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return nullptr;
  }
  b.bytes = want;
  return b.p;
}

static hipEvent_t prof_event(obem_ctx *ctx) {
  if (!ctx->prof_pool.empty()) {
    hipEvent_t e = ctx->prof_pool.back();
    ctx->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

int prof_begin(obem_ctx *ctx, const char *name) {
  if (!ctx || !ctx->prof) return -1;
  obem_prof_rec r{name, prof_event(ctx), prof_event(ctx)};
  if (!r.start || !r.stop) return -1;
  (void)hipEventRecord(r.start, ctx->stream);
  (void)hipEventRecord(r.stop, ctx->stream);  // overwritten by prof_end
  ctx->prof_recs.push_back(r);
  return (int)ctx->prof_recs.size() - 1;
}

void prof_end(obem_ctx *ctx, int idx) {
  if (!ctx || idx < 0 || idx >= (int)ctx->prof_recs.size()) return;
  (void)hipEventRecord(ctx->prof_recs[idx].stop, ctx->stream);
}

bool is_device_ptr(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged ||
         attr.type == hipMemoryTypeUnified;
}

// ---------------------------------------------------------------------------
// Mesh derivation: normal, area, centroid, diameter, quadrature points.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mesh_derive(int n, double *f, const int8_t *kind, const double *e1,
                                                     const double *e2, int *bad) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  auto F = [&](int fld) -> double & { return f[(size_t)fld * n + k]; };
  d3 a = mk3(F(MF_AX), F(MF_AY), F(MF_AZ));
  d3 b = mk3(F(MF_BX), F(MF_BY), F(MF_BZ));
  d3 c = mk3(F(MF_CX), F(MF_CY), F(MF_CZ));
  d3 N2 = cross3(b - a, c - a);
  double n2 = norm3(N2);
  double L = fmax(norm3(b - a), fmax(norm3(c - b), norm3(a - c)));
  if (!(n2 > 0.0) || !(n2 <= 1e300) || !(L > 0.0)) {
    atomicAdd(bad, 1);
    n2 = 1.0;
  }
  d3 nn = N2 * (1.0 / n2);
  F(MF_NX) = nn.x;
  F(MF_NY) = nn.y;
  F(MF_NZ) = nn.z;
  F(MF_AREA) = 0.5 * n2;
  F(MF_DIAM) = L;
  d3 g = (a + b + c) * (1.0 / 3.0);
  F(MF_GX) = g.x;
  F(MF_GY) = g.y;
  F(MF_GZ) = g.z;
  const bool dd = kind[k] == 1;
  F(MF_EPS1) = (dd && e1) ? e1[k] : 1.0;
  F(MF_EPS2) = (dd && e2) ? e2[k] : 1.0;
  // 7-point rule: centroid, then (a, a, 1-2a) and (b, b, 1-2b) families
  const double bary7[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3},
                              {Rule7::a, Rule7::a, 1 - 2 * Rule7::a},
                              {Rule7::a, 1 - 2 * Rule7::a, Rule7::a},
                              {1 - 2 * Rule7::a, Rule7::a, Rule7::a},
                              {Rule7::b, Rule7::b, 1 - 2 * Rule7::b},
                              {Rule7::b, 1 - 2 * Rule7::b, Rule7::b},
                              {1 - 2 * Rule7::b, Rule7::b, Rule7::b}};
  for (int q = 0; q < 7; ++q) {
    d3 p = a * bary7[q][0] + b * bary7[q][1] + c * bary7[q][2];
    F(MF_Q7 + 3 * q) = p.x;
    F(MF_Q7 + 3 * q + 1) = p.y;
    F(MF_Q7 + 3 * q + 2) = p.z;
  }
  const double bary3[3][3] = {{2.0 / 3, 1.0 / 6, 1.0 / 6}, {1.0 / 6, 2.0 / 3, 1.0 / 6}, {1.0 / 6, 1.0 / 6, 2.0 / 3}};
  for (int q = 0; q < 3; ++q) {
    d3 p = a * bary3[q][0] + b * bary3[q][1] + c * bary3[q][2];
    F(MF_Q3 + 3 * q) = p.x;
    F(MF_Q3 + 3 * q + 1) = p.y;
    F(MF_Q3 + 3 * q + 2) = p.z;
  }
  const double bary6[6][3] = {{Rule6::b1, Rule6::a1, Rule6::a1}, {Rule6::a1, Rule6::b1, Rule6::a1},
                              {Rule6::a1, Rule6::a1, Rule6::b1}, {Rule6::b2, Rule6::a2, Rule6::a2},
                              {Rule6::a2, Rule6::b2, Rule6::a2}, {Rule6::a2, Rule6::a2, Rule6::b2}};
  for (int q = 0; q < 6; ++q) {
    d3 p = a * bary6[q][0] + b * bary6[q][1] + c * bary6[q][2];
    F(MF_Q6 + 3 * q) = p.x;
    F(MF_Q6 + 3 * q + 1) = p.y;
    F(MF_Q6 + 3 * q + 2) = p.z;
  }
  const double bary4[3][3] = {{Rule4::b, Rule4::a, Rule4::a}, {Rule4::a, Rule4::b, Rule4::a},
                              {Rule4::a, Rule4::a, Rule4::b}};
  for (int q = 0; q < 3; ++q) {
    d3 p = a * bary4[q][0] + b * bary4[q][1] + c * bary4[q][2];
    F(MF_Q4 + 3 * q) = p.x;
    F(MF_Q4 + 3 * q + 1) = p.y;
    F(MF_Q4 + 3 * q + 2) = p.z;
  }
  // edge data of the closed form: unit tangent, length, t x n
  const d3 v[3] = {a, b, c};
  for (int e = 0; e < 3; ++e) {
    d3 t = v[(e + 1) % 3] - v[e];
    const double Le = norm3(t);
    t = t * (1.0 / Le);
    const d3 m = cross3(t, nn);
    F(MF_T + 3 * e) = t.x;
    F(MF_T + 3 * e + 1) = t.y;
    F(MF_T + 3 * e + 2) = t.z;
    F(MF_EL + e) = Le;
    F(MF_M + 3 * e) = m.x;
    F(MF_M + 3 * e + 1) = m.y;
    F(MF_M + 3 * e + 2) = m.z;
  }
}

// Zone bounding spheres of consecutive 64-cell tiles: centre = mean
// centroid, radius = max_k (|c_k - centre| + zone D_k) (zone 3: the mixed
// near zone, 48: the FP64 closed-form zone), inflated by 1e-6 relative so
// FP32 rounding of the per-pair test cannot escape it.
__global__ __launch_bounds__(64) void k_tile_spheres(int n, const double *f, double zone, double *tiles) {
  const int t = blockIdx.x;
  const int k = t * 64 + threadIdx.x;
  const bool ok = k < n;
  double c[3] = {0, 0, 0};
  const int cnt = min(64, n - t * 64);
  for (int j = 0; j < cnt; ++j)
    for (int d = 0; d < 3; ++d) c[d] += f[(size_t)(MF_GX + d) * n + t * 64 + j];
  for (int d = 0; d < 3; ++d) c[d] /= cnt;
  double r = 0.0;
  if (ok) {
    double dx = f[(size_t)MF_GX * n + k] - c[0], dy = f[(size_t)MF_GY * n + k] - c[1], dz = f[(size_t)MF_GZ * n + k] - c[2];
    r = sqrt(dx * dx + dy * dy + dz * dz) + zone * f[(size_t)MF_DIAM * n + k];
  }
  for (int o = 32; o > 0; o >>= 1) r = fmax(r, __shfl_xor(r, o));
  if (threadIdx.x == 0) {
    tiles[4 * t] = c[0];
    tiles[4 * t + 1] = c[1];
    tiles[4 * t + 2] = c[2];
    tiles[4 * t + 3] = r * (1.0 + 1e-6) + 1e-12;
  }
}

obem_status aux_stream(obem_ctx *ctx) {
  if (ctx->aux) return OBEM_OK;
  OBEM_HIP(ctx, hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
  for (int b = 0; b < 2; ++b) {
    OBEM_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_slots[b], hipEventDisableTiming));
    OBEM_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_free[b], hipEventDisableTiming));
  }
  OBEM_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
  return OBEM_OK;
}

}  // namespace obem

using namespace obem;


extern "C" {

void obem_constants(double *out) {
  if (!out) return;
  out[0] = kEps0;
  out[1] = kKe;
  out[2] = kQe;
  out[3] = kMe;
  out[4] = kKb;
  out[5] = kAmu;
}

// ---------------------------------------------------------------------------
// Scratch array of the allocation-free entry point (field_eval_noalloc)
// ---------------------------------------------------------------------------
// Each device the library runs on holds its own copy for the life of the
// process.  In host code the name is only a stand-in for the symbol: kernels
// and copies get the device address taken with hipGetSymbolAddress, once per
// device, kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[OBEM_NOALLOC_SCRATCH_BYTES];
constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kScratchDevices] = {};

static obem_status scratch_setup(obem_ctx *c) {
  if (c->device >= kScratchDevices) return OBEM_OK;  // field_eval_noalloc then reports the missing scratch
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[c->device]) {
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(c->device) != hipSuccess) {
      (void)hipGetLastError();
      return OBEM_EDEVICE;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    (void)hipSetDevice(prev);
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return OBEM_EDEVICE;
    }
    g_scratch_ptr[c->device] = (char *)p;
  }
  c->scratch = g_scratch_ptr[c->device];
  return OBEM_OK;
}

obem_status obem_create(obem_ctx **out, int device, void *hip_stream) {
  if (!out) return OBEM_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return OBEM_EINVAL;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    (void)hipGetLastError();
    return OBEM_EDEVICE;
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return OBEM_EDEVICE;  // code objects are gfx950 only
  obem_ctx *c = new obem_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (scratch_setup(c) != OBEM_OK) {
    delete c;
    return OBEM_EDEVICE;
  }
  *out = c;
  return OBEM_OK;
}

obem_status obem_destroy(obem_ctx *ctx) {
  if (!ctx) return OBEM_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto &r : ctx->prof_recs) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  for (auto e : ctx->prof_pool) (void)hipEventDestroy(e);
  if (ctx->aux) {
    (void)hipStreamSynchronize(ctx->aux);
    for (int b = 0; b < 2; ++b) {
      if (ctx->ev_slots[b]) (void)hipEventDestroy(ctx->ev_slots[b]);
      if (ctx->ev_free[b]) (void)hipEventDestroy(ctx->ev_free[b]);
    }
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    (void)hipStreamDestroy(ctx->aux);
  }
  if (ctx->work_dev) (void)hipFree(ctx->work_dev);
  for (auto &b : ctx->ws)
    if (b.p) (void)hipFree(b.p);
  solver_release(ctx);
  (void)hipGetLastError();
  delete ctx;
  return OBEM_OK;
}

obem_status obem_profile_enable(obem_ctx *ctx, int enable) {
  if (!ctx) return OBEM_EINVAL;
  if (enable && !ctx->work_dev) {
    if (hipSetDevice(ctx->device) != hipSuccess ||
        hipMalloc((void **)&ctx->work_dev, sizeof(unsigned long long)) != hipSuccess) {
      (void)hipGetLastError();
      ctx->work_dev = nullptr;
      return fail(ctx, OBEM_ENOMEM, "profile counter allocation failed");
    }
    OBEM_HIP(ctx, hipMemsetAsync(ctx->work_dev, 0, sizeof(unsigned long long), ctx->stream));
  }
  ctx->prof = enable != 0;
  return OBEM_OK;
}

obem_status obem_profile_work(obem_ctx *ctx, int64_t *directed, int64_t *once) {
  if (!ctx) return OBEM_EINVAL;
  unsigned long long dev = 0;
  if (ctx->work_dev) {
    OBEM_HIP(ctx, hipSetDevice(ctx->device));
    OBEM_HIP(ctx, hipMemcpyAsync(&dev, ctx->work_dev, sizeof(dev), hipMemcpyDeviceToHost, ctx->stream));
    OBEM_HIP(ctx, hipMemsetAsync(ctx->work_dev, 0, sizeof(unsigned long long), ctx->stream));
    OBEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  // the pair-once kernel covers the n^2 ordered terms the directed kernel
  // does not take, two per unordered pair
  if (directed) *directed = ctx->work_directed + (int64_t)dev;
  if (once) *once = (ctx->work_once_n2 - (int64_t)dev) / 2;
  ctx->work_directed = 0;
  ctx->work_once_n2 = 0;
  return OBEM_OK;
}

obem_status obem_profile_read(obem_ctx *ctx, int max_entries, char *names, double *ms, int64_t *launches,
                              int *n_out) {
  if (!ctx || !n_out || max_entries < 0 || (max_entries > 0 && (!names || !ms || !launches))) return OBEM_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess || hipStreamSynchronize(ctx->stream) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, OBEM_EDEVICE, "synchronisation failed while reading the profile");
  }
  std::vector<std::string> keys;
  std::vector<double> tot;
  std::vector<int64_t> cnt;
  for (auto &r : ctx->prof_recs) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.start, r.stop) != hipSuccess) {
      (void)hipGetLastError();
      t = 0.f;
    }
    size_t k = 0;
    while (k < keys.size() && keys[k] != r.name) ++k;
    if (k == keys.size()) {
      keys.push_back(r.name);
      tot.push_back(0.0);
      cnt.push_back(0);
    }
    tot[k] += t;
    cnt[k] += 1;
    ctx->prof_pool.push_back(r.start);
    ctx->prof_pool.push_back(r.stop);
  }
  ctx->prof_recs.clear();
  const int n = (int)std::min<size_t>(keys.size(), (size_t)max_entries);
  for (int k = 0; k < n; ++k) {
    std::strncpy(names + 32 * k, keys[k].c_str(), 31);
    names[32 * k + 31] = 0;
    ms[k] = tot[k];
    launches[k] = cnt[k];
  }
  *n_out = n;
  return OBEM_OK;
}

const char *obem_last_error(const obem_ctx *ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

// Device state of a bound mesh, filled step by step; on an error the caller
// releases whatever was allocated.
static obem_status bind_fill(obem_ctx *ctx, const obem_mesh *mesh, obem_meshh *m) {
  const int64_t n = m->n;
  const double *v[9] = {mesh->ax, mesh->ay, mesh->az, mesh->bx, mesh->by, mesh->bz, mesh->cx, mesh->cy, mesh->cz};
  const int ntile = (int)((n + 63) / 64);
  if (hipMalloc(&m->f, sizeof(double) * MF_COUNT * (size_t)n) != hipSuccess ||
      hipMalloc(&m->kind, (size_t)n) != hipSuccess || hipMalloc(&m->tiles, sizeof(double) * 4 * ntile) != hipSuccess ||
      hipMalloc(&m->tiles48, sizeof(double) * 4 * ntile) != hipSuccess ||
      hipMalloc(&m->order, sizeof(int32_t) * n) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, OBEM_ENOMEM, "mesh allocation failed");
  }
  for (int k = 0; k < 9; ++k)
    OBEM_HIP(ctx, hipMemcpyAsync(m->f + (size_t)k * n, v[k], sizeof(double) * n, hipMemcpyDeviceToDevice, ctx->stream));
  OBEM_HIP(ctx, hipMemcpyAsync(m->kind, mesh->kind, (size_t)n, hipMemcpyDeviceToDevice, ctx->stream));
  int *bad = (int *)ws_get(ctx, WS_MISC0, sizeof(int));
  if (!bad) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  OBEM_HIP(ctx, hipMemsetAsync(bad, 0, sizeof(int), ctx->stream));
  hipLaunchKernelGGL(k_mesh_derive, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, (int)n, m->f,
                     m->kind, mesh->eps_r1, mesh->eps_r2, bad);
  OBEM_HIP(ctx, hipGetLastError());
  hipLaunchKernelGGL(k_tile_spheres, dim3(ntile), dim3(64), 0, ctx->stream, (int)n, m->f, kNearMixed, m->tiles);
  hipLaunchKernelGGL(k_tile_spheres, dim3(ntile), dim3(64), 0, ctx->stream, (int)n, m->f, kQuadFp64, m->tiles48);
  OBEM_HIP(ctx, hipGetLastError());
  {
    TargetOrder co;
    obem_status st = order_targets(ctx, n, m->f + (size_t)MF_GX * n, m->f + (size_t)MF_GY * n,
                                   m->f + (size_t)MF_GZ * n, &co);
    if (st) return st;
    OBEM_HIP(ctx, hipMemcpyAsync(m->order, co.perm, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, ctx->stream));
  }
  int hbad = 0;
  OBEM_HIP(ctx, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  // host copies for the bounding box and diameters
  std::vector<double> hv((size_t)n * 9), hd((size_t)n);
  OBEM_HIP(ctx, hipMemcpyAsync(hv.data(), m->f, sizeof(double) * 9 * n, hipMemcpyDeviceToHost, ctx->stream));
  OBEM_HIP(ctx, hipMemcpyAsync(hd.data(), m->f + (size_t)MF_DIAM * n, sizeof(double) * n, hipMemcpyDeviceToHost,
                               ctx->stream));
  OBEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (hbad) return fail(ctx, OBEM_EINVAL, "mesh has %d degenerate or non-finite cells", hbad);
  for (int c = 0; c < 3; ++c) {
    m->bbox_lo[c] = INFINITY;
    m->bbox_hi[c] = -INFINITY;
  }
  for (int64_t k = 0; k < n; ++k)
    for (int vtx = 0; vtx < 3; ++vtx)
      for (int c = 0; c < 3; ++c) {
        double x = hv[(size_t)(3 * vtx + c) * n + k];
        m->bbox_lo[c] = std::min(m->bbox_lo[c], x);
        m->bbox_hi[c] = std::max(m->bbox_hi[c], x);
      }
  m->max_diam = *std::max_element(hd.begin(), hd.end());
  return OBEM_OK;
}

static void free_mesh(obem_meshh *m) {
  (void)hipFree(m->f);
  (void)hipFree(m->kind);
  (void)hipFree(m->tiles);
  (void)hipFree(m->tiles48);
  (void)hipFree(m->order);
  (void)hipFree(m->rhs_last);
  (void)hipFree(m->sigma_last);
  bem_release(m);
  (void)hipFree(m->grid_start);
  (void)hipFree(m->grid_items);
  (void)hipGetLastError();
  delete m;
}

obem_status obem_mesh_bind(obem_ctx *ctx, const obem_mesh *mesh, obem_meshh **out) {
  CHECK_CTX(ctx);
  if (!mesh || !out) return fail(ctx, OBEM_EINVAL, "mesh/out is NULL");
  *out = nullptr;
  const int64_t n = mesh->n_panels;
  if (n <= 0 || n >= kMaxCount) return fail(ctx, OBEM_EINVAL, "n_panels=%lld out of range", (long long)n);
  const double *v[9] = {mesh->ax, mesh->ay, mesh->az, mesh->bx, mesh->by, mesh->bz, mesh->cx, mesh->cy, mesh->cz};
  for (int k = 0; k < 9; ++k) REQ_DEV(ctx, v[k], "mesh vertex array");
  REQ_DEV(ctx, mesh->kind, "mesh->kind");
  std::vector<int8_t> hk((size_t)n);
  OBEM_HIP(ctx, hipMemcpy(hk.data(), mesh->kind, (size_t)n, hipMemcpyDeviceToHost));
  int64_t n_dd = 0;
  for (int8_t k : hk) {
    if (k != 0 && k != 1) return fail(ctx, OBEM_EINVAL, "mesh->kind must be 0 (ed) or 1 (dd)");
    n_dd += k;
  }
  if (n_dd) {
    REQ_DEV(ctx, mesh->eps_r1, "mesh->eps_r1");
    REQ_DEV(ctx, mesh->eps_r2, "mesh->eps_r2");
  }
  obem_meshh *m = new obem_meshh();
  m->n = n;
  m->n_dd = n_dd;
  const obem_status st = bind_fill(ctx, mesh, m);
  if (st) {
    free_mesh(m);
    return st;
  }
  *out = m;
  return OBEM_OK;
}

obem_status obem_mesh_release(obem_ctx *ctx, obem_meshh *m) {
  if (!ctx || !m) return OBEM_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  free_mesh(m);
  return OBEM_OK;
}

obem_status obem_mesh_geometry(obem_ctx *ctx, const obem_meshh *m, double *area, double *cx, double *cy,
                               double *cz, double *diameter) {
  CHECK_CTX(ctx);
  if (!m) return fail(ctx, OBEM_EINVAL, "mesh is NULL");
  double *dst[5] = {area, cx, cy, cz, diameter};
  const int src[5] = {MF_AREA, MF_GX, MF_GY, MF_GZ, MF_DIAM};
  for (int k = 0; k < 5; ++k) {
    if (!dst[k]) continue;
    OPT_DEV(ctx, dst[k], "output array");
    OBEM_HIP(ctx, hipMemcpyAsync(dst[k], m->field(src[k]), sizeof(double) * m->n, hipMemcpyDeviceToDevice,
                                 ctx->stream));
  }
  return OBEM_OK;
}

static obem_status field_eval_impl(obem_ctx *ctx, const obem_meshh *mesh, const double *sigma, int64_t n_src,
                                   const double *sx, const double *sy, const double *sz, const double *sq,
                                   int64_t n_tgt, const double *tx, const double *ty, const double *tz,
                                   double soft, obem_precision precision, unsigned flags, double *Ex, double *Ey,
                                   double *Ez, double *V) {
  if (n_tgt < 0 || n_tgt >= kMaxCount || n_src < 0 || n_src >= kMaxCount)
    return fail(ctx, OBEM_EINVAL, "n_tgt/n_src out of range");
  if (!(soft >= 0.0) || !std::isfinite(soft)) return fail(ctx, OBEM_EINVAL, "soft must be finite and >= 0");
  if (precision != OBEM_FP64 && precision != OBEM_MIXED) return fail(ctx, OBEM_EINVAL, "bad precision");
  if (flags & ~(OBEM_TGT_IS_SRC | OBEM_WANT_V)) return fail(ctx, OBEM_EINVAL, "unknown flags");
  const bool tis = flags & OBEM_TGT_IS_SRC;
  const bool want_v = flags & OBEM_WANT_V;
  if (tis && n_src != n_tgt) return fail(ctx, OBEM_EINVAL, "OBEM_TGT_IS_SRC needs n_src == n_tgt");
  if (n_tgt == 0) return OBEM_OK;
  REQ_DEV(ctx, tx, "tx");
  REQ_DEV(ctx, ty, "ty");
  REQ_DEV(ctx, tz, "tz");
  REQ_DEV(ctx, Ex, "Ex");
  REQ_DEV(ctx, Ey, "Ey");
  REQ_DEV(ctx, Ez, "Ez");
  if (want_v) REQ_DEV(ctx, V, "V");
  if (n_src > 0) {
    REQ_DEV(ctx, sx, "sx");
    REQ_DEV(ctx, sy, "sy");
    REQ_DEV(ctx, sz, "sz");
    REQ_DEV(ctx, sq, "sq");
  }
  if (mesh) REQ_DEV(ctx, sigma, "sigma");
  // sources first (their ordering reuses the target-ordering workspace)
  SourceOrder so;
  if (n_src > 0) {
    obem_status st = order_sources(ctx, n_src, sx, sy, sz, sq, tis, &so);
    if (st) return st;
  }
  // targets = sources: with the pair-once evaluation the targets take the
  // sources' order (same particles, same tiles)
  const bool once = tis && pair_once_applies(n_tgt, precision, soft, want_v);
  TargetOrder to;
  obem_status st = OBEM_OK;
  if (once) {
    to.n = (int32_t)n_tgt;
    to.perm = const_cast<int32_t *>(so.perm);
    to.xs = const_cast<double *>(so.x);
  } else {
    st = order_targets(ctx, n_tgt, tx, ty, tz, &to);
    if (st) return st;
  }
  double *acc = (double *)ws_get(ctx, WS_ACC, sizeof(double) * 4 * (size_t)n_tgt);
  if (!acc) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  if (mesh) {
    st = launch_panel_field(ctx, mesh, sigma, to, precision, want_v, acc);
  } else {
    st = launch_fill(ctx, acc, 4 * (size_t)n_tgt, 0.0);
  }
  if (st) return st;
  if (n_src > 0) {
    st = launch_pair_field(ctx, n_src, so.x, so.y, so.z, so.q, to, soft, precision, tis, want_v, nullptr, nullptr,
                           acc, nullptr, nullptr, so.tbox, 0.0, tis ? so.inv : nullptr, once);
    if (st) return st;
  }
  return launch_scatter(ctx, to, acc, kKe, Ex, Ey, Ez, want_v ? V : nullptr);
}

obem_status field_eval(obem_ctx *ctx, const obem_meshh *mesh, const double *sigma, int64_t n_src,
                       const double *sx, const double *sy, const double *sz, const double *sq, int64_t n_tgt,
                       const double *tx, const double *ty, const double *tz, double soft,
                       obem_precision precision, unsigned flags, double *Ex, double *Ey, double *Ez, double *V) {
  CHECK_CTX(ctx);
  return field_eval_impl(ctx, mesh, sigma, n_src, sx, sy, sz, sq, n_tgt, tx, ty, tz, soft, precision, flags, Ex,
                         Ey, Ez, V);
}

obem_status field_eval_noalloc(obem_ctx *ctx, const obem_meshh *mesh, const double *sigma, int64_t n_src,
                               const double *sx, const double *sy, const double *sz, const double *sq,
                               int64_t n_tgt, const double *tx, const double *ty, const double *tz, double soft,
                               obem_precision precision, unsigned flags, double *Ex, double *Ey, double *Ez,
                               double *V) {
  CHECK_CTX(ctx);
  if (n_tgt < 0 || n_src < 0 || n_tgt > OBEM_NOALLOC_MAX_POINTS || n_src > OBEM_NOALLOC_MAX_POINTS)
    return fail(ctx, OBEM_EINVAL, "field_eval_noalloc: n_tgt and n_src must lie in [0, %d] (got %lld, %lld)",
                OBEM_NOALLOC_MAX_POINTS, (long long)n_tgt, (long long)n_src);
  if (!ctx->scratch) return fail(ctx, OBEM_EDEVICE, "field_eval_noalloc: no scratch array on device %d", ctx->device);
  // workspace from the scratch array; no event timing (its events are created on demand)
  ctx->arena = ctx->scratch;
  ctx->arena_bytes = OBEM_NOALLOC_SCRATCH_BYTES;
  ctx->arena_used = 0;
  ctx->arena_overflow = false;
  for (int k = 0; k < WS_COUNT; ++k) {
    ctx->arena_slot[k] = nullptr;
    ctx->arena_slot_bytes[k] = 0;
  }
  const bool prof = ctx->prof;
  ctx->prof = false;
  obem_status st = field_eval_impl(ctx, mesh, sigma, n_src, sx, sy, sz, sq, n_tgt, tx, ty, tz, soft, precision,
                                   flags, Ex, Ey, Ez, V);
  ctx->prof = prof;
  ctx->arena = nullptr;
  if (st == OBEM_ENOMEM && ctx->arena_overflow)
    st = fail(ctx, OBEM_ENOMEM, "field_eval_noalloc: the call needs more than the %llu-byte scratch array",
              (unsigned long long)OBEM_NOALLOC_SCRATCH_BYTES);
  return st;
}

}  // extern "C"
