// Static field option (section 3.3.1): the cell field computed once on a
// uniform 3D grid and interpolated (trilinearly) at the particles; and the
// Shockley-Ramo current of eq. (ramo), whose weighting field comes either
// from the cells (dynamic option) or from such a map (static option).
#include <algorithm>
#include <cmath>

#include "obem_internal.hpp"

namespace obem {

// Node coordinates of the grid, SoA (x, y, z), index (k*ny + j)*nx + i.
__global__ __launch_bounds__(256) void k_grid_nodes(MapDev g, double *xs) {
  const int64_t M = (int64_t)g.nx * g.ny * g.nz;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= M) return;
  const int i = (int)(t % g.nx), j = (int)((t / g.nx) % g.ny), k = (int)(t / ((int64_t)g.nx * g.ny));
  // lo + h*i rounded twice (no contraction), so a node's coordinates do not
  // depend on the compiler's choice of fused multiply-add
  xs[t] = __dadd_rn(g.lo[0], __dmul_rn(g.h[0], (double)i));
  xs[M + t] = __dadd_rn(g.lo[1], __dmul_rn(g.h[1], (double)j));
  xs[2 * M + t] = __dadd_rn(g.lo[2], __dmul_rn(g.h[2], (double)k));
}

__global__ __launch_bounds__(256) void k_map_eval(MapDev g, int n, const double *__restrict__ x,
                                                  const double *__restrict__ y, const double *__restrict__ z,
                                                  double *Ex, double *Ey, double *Ez) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  double E[3];
  map_interp(g, x[t], y[t], z[t], E);
  Ex[t] = E[0];
  Ey[t] = E[1];
  Ez[t] = E[2];
}

// Per-particle q v . E_w and per-block sums by species (fixed-order tree).
__global__ __launch_bounds__(256) void k_ramo_terms(int n, const double *__restrict__ Ew, const double *__restrict__ vx,
                                                    const double *__restrict__ vy, const double *__restrict__ vz,
                                                    const int8_t *__restrict__ sp, double *terms, double *part) {
  __shared__ double s[3][256];
  const int t = blockIdx.x * 256 + threadIdx.x;
  double c[3] = {0.0, 0.0, 0.0};
  if (t < n) {
    const int8_t k = sp[t];
    const double q = (k == 1) ? kQe : -kQe;
    const double term = q * (vx[t] * Ew[t] + vy[t] * Ew[(size_t)n + t] + vz[t] * Ew[2 * (size_t)n + t]);
    if (terms) terms[t] = term;
    if (k >= 0 && k <= 2) c[k] = term;
  }
  for (int m = 0; m < 3; ++m) s[m][threadIdx.x] = c[m];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int m = 0; m < 3; ++m) s[m][threadIdx.x] += s[m][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) part[3 * (size_t)blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

// Sum of the block sums in block order (one wave per species).
__global__ __launch_bounds__(64) void k_ramo_final(int nb, const double *__restrict__ part, double *out) {
  const int m = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += 64) acc += part[3 * (size_t)b + m];
  __shared__ double s[64];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 32; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[m] = s[0];
}

bool map_dev(const obem_field_map *m, MapDev *g) {
  if (!m || m->nx < 2 || m->ny < 2 || m->nz < 2) return false;
  if ((int64_t)m->nx * m->ny * m->nz >= kMaxCount) return false;
  for (int c = 0; c < 3; ++c)
    if (!(m->h[c] > 0.0) || !std::isfinite(m->h[c]) || !std::isfinite(m->lo[c])) return false;
  if (!is_device_ptr(m->ex) || !is_device_ptr(m->ey) || !is_device_ptr(m->ez)) return false;
  g->nx = m->nx;
  g->ny = m->ny;
  g->nz = m->nz;
  for (int c = 0; c < 3; ++c) {
    g->lo[c] = m->lo[c];
    g->h[c] = m->h[c];
  }
  g->ex = m->ex;
  g->ey = m->ey;
  g->ez = m->ez;
  return true;
}

__global__ __launch_bounds__(256) void k_map_acc(MapDev g, int n, const double *__restrict__ xs, double *acc) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  double E[3];
  map_interp(g, xs[t], xs[(size_t)n + t], xs[2 * (size_t)n + t], E);
  acc[t] = E[0] / kKe;
  acc[(size_t)n + t] = E[1] / kKe;
  acc[2 * (size_t)n + t] = E[2] / kKe;
  acc[3 * (size_t)n + t] = 0.0;
}

obem_status launch_map_acc(obem_ctx *ctx, const MapDev &g, const TargetOrder &to, double *acc) {
  if (to.n == 0) return OBEM_OK;
  OBEM_PROF(ctx, "map");
  hipLaunchKernelGGL(k_map_acc, dim3((unsigned)((to.n + 255) / 256)), dim3(256), 0, ctx->stream, g, to.n, to.xs, acc);
  OBEM_HIP(ctx, hipGetLastError());
  return OBEM_OK;
}

}  // namespace obem

using namespace obem;

extern "C" {

obem_status field_map_build(obem_ctx *ctx, const obem_meshh *mesh, const double *sigma, const obem_field_map *map,
                            obem_precision precision) {
  CHECK_CTX(ctx);
  if (!mesh) return fail(ctx, OBEM_EINVAL, "mesh is NULL");
  REQ_DEV(ctx, sigma, "sigma");
  if (precision != OBEM_FP64 && precision != OBEM_MIXED) return fail(ctx, OBEM_EINVAL, "bad precision");
  MapDev g;
  if (!map_dev(map, &g)) return fail(ctx, OBEM_EINVAL, "bad field map (sizes >= 2, spacing > 0, device arrays)");
  const int64_t M = (int64_t)g.nx * g.ny * g.nz;
  double *xs = (double *)ws_get(ctx, WS_MAP, sizeof(double) * 3 * (size_t)M);
  double *acc = (double *)ws_get(ctx, WS_ACC, sizeof(double) * 4 * (size_t)M);
  if (!xs || !acc) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  hipLaunchKernelGGL(k_grid_nodes, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, ctx->stream, g, xs);
  OBEM_HIP(ctx, hipGetLastError());
  TargetOrder to;
  obem_status st = order_targets(ctx, M, xs, xs + M, xs + 2 * M, &to);
  if (st) return st;
  st = launch_panel_field(ctx, mesh, sigma, to, precision, false, acc);
  if (st) return st;
  return launch_scatter(ctx, to, acc, kKe, map->ex, map->ey, map->ez, nullptr);
}

obem_status field_map_eval(obem_ctx *ctx, const obem_field_map *map, int64_t n, const double *x, const double *y,
                           const double *z, double *Ex, double *Ey, double *Ez) {
  CHECK_CTX(ctx);
  MapDev g;
  if (!map_dev(map, &g)) return fail(ctx, OBEM_EINVAL, "bad field map (sizes >= 2, spacing > 0, device arrays)");
  if (n < 0 || n >= kMaxCount) return fail(ctx, OBEM_EINVAL, "n out of range");
  if (n == 0) return OBEM_OK;
  REQ_DEV(ctx, x, "x");
  REQ_DEV(ctx, y, "y");
  REQ_DEV(ctx, z, "z");
  REQ_DEV(ctx, Ex, "Ex");
  REQ_DEV(ctx, Ey, "Ey");
  REQ_DEV(ctx, Ez, "Ez");
  hipLaunchKernelGGL(k_map_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, g, (int)n, x, y, z,
                     Ex, Ey, Ez);
  OBEM_HIP(ctx, hipGetLastError());
  return OBEM_OK;
}

obem_status induced_current(obem_ctx *ctx, const obem_meshh *mesh, const double *sigma_w, const obem_field_map *map,
                            int64_t n, const double *x, const double *y, const double *z, const double *vx,
                            const double *vy, const double *vz, const int8_t *species, obem_precision precision,
                            double *current, double *terms) {
  CHECK_CTX(ctx);
  if (n < 0 || n >= kMaxCount) return fail(ctx, OBEM_EINVAL, "n out of range");
  if ((map != nullptr) == (mesh != nullptr))
    return fail(ctx, OBEM_EINVAL, "give either mesh + sigma_w or a weighting-field map");
  MapDev g;
  if (map && !map_dev(map, &g)) return fail(ctx, OBEM_EINVAL, "bad field map");
  if (mesh) REQ_DEV(ctx, sigma_w, "sigma_w");
  if (precision != OBEM_FP64 && precision != OBEM_MIXED) return fail(ctx, OBEM_EINVAL, "bad precision");
  OPT_DEV(ctx, terms, "terms");
  if (n == 0) {
    if (current) current[0] = current[1] = current[2] = 0.0;
    return OBEM_OK;
  }
  const void *req[] = {x, y, z, vx, vy, vz, species};
  for (const void *p : req)
    if (!is_device_ptr(p)) return fail(ctx, OBEM_EINVAL, "particle arrays must be device memory");
  const int nb = (int)((n + 255) / 256);
  double *Ew = (double *)ws_get(ctx, WS_MISC0, sizeof(double) * 3 * (size_t)n);
  double *part = (double *)ws_get(ctx, WS_MISC1, sizeof(double) * (3 * (size_t)nb + 3));
  if (!Ew || !part) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  if (map) {
    hipLaunchKernelGGL(k_map_eval, dim3(nb), dim3(256), 0, ctx->stream, g, (int)n, x, y, z, Ew, Ew + n, Ew + 2 * n);
    OBEM_HIP(ctx, hipGetLastError());
  } else {
    TargetOrder to;
    obem_status st = order_targets(ctx, n, x, y, z, &to);
    if (st) return st;
    double *acc = (double *)ws_get(ctx, WS_ACC, sizeof(double) * 4 * (size_t)n);
    if (!acc) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
    st = launch_panel_field(ctx, mesh, sigma_w, to, precision, false, acc);
    if (st) return st;
    st = launch_scatter(ctx, to, acc, kKe, Ew, Ew + n, Ew + 2 * n, nullptr);
    if (st) return st;
  }
  hipLaunchKernelGGL(k_ramo_terms, dim3(nb), dim3(256), 0, ctx->stream, (int)n, Ew, vx, vy, vz, species, terms, part);
  hipLaunchKernelGGL(k_ramo_final, dim3(3), dim3(64), 0, ctx->stream, nb, part, part + 3 * (size_t)nb);
  OBEM_HIP(ctx, hipGetLastError());
  if (current) {
    OBEM_HIP(ctx, hipMemcpyAsync(current, part + 3 * (size_t)nb, 3 * sizeof(double), hipMemcpyDeviceToHost,
                                 ctx->stream));
    OBEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  return OBEM_OK;
}

}  // extern "C"
