// Field evaluation kernels for gfx950: target ordering, cell (panel) field,
// pairwise point-charge field, fixed-order reduction and scatter.
//
// Layout: targets are reordered along a Hilbert curve so that the 256 targets
// of a workgroup are spatially compact; each workgroup recentres its targets
// and the staged source/cell data on its first target (FP64 difference, then
// FP32), which keeps FP32 differences relative to the pair distance instead
// of the absolute coordinates.  Sums are accumulated per tile in registers and
// carried across tiles with a compensated (Neumaier) FP32 sum in the mixed
// mode, plainly in FP64 in the FP64 mode.  No floating-point atomics: every
// reduction has a fixed order.
#include <hipcub/hipcub.hpp>

#include "cellmath.hpp"
#include "obem_internal.hpp"
#include "paironce.hpp"

namespace obem {

constexpr int kThreads = 256;

// ---------------------------------------------------------------------------
// Target ordering
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bbox_partial(int n, const double *__restrict__ x,
                                                      const double *__restrict__ y,
                                                      const double *__restrict__ z, double *part) {
  __shared__ double s[6][256];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    double v[3] = {x[i], y[i], z[i]};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lo[c] = fmin(lo[c], v[c]);
      hi[c] = fmax(hi[c], v[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s[c][threadIdx.x] = lo[c];
    s[3 + c][threadIdx.x] = hi[c];
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        s[c][threadIdx.x] = fmin(s[c][threadIdx.x], s[c][threadIdx.x + w]);
        s[3 + c][threadIdx.x] = fmax(s[3 + c][threadIdx.x], s[3 + c][threadIdx.x + w]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_bbox_final(int nb, const double *part, double *bbox) {
  __shared__ double s[6][256];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < nb; b += 256) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lo[c] = fmin(lo[c], part[b * 6 + c]);
      hi[c] = fmax(hi[c], part[b * 6 + 3 + c]);
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s[c][threadIdx.x] = lo[c];
    s[3 + c][threadIdx.x] = hi[c];
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        s[c][threadIdx.x] = fmin(s[c][threadIdx.x], s[c][threadIdx.x + w]);
        s[3 + c][threadIdx.x] = fmax(s[3 + c][threadIdx.x], s[3 + c][threadIdx.x + w]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) bbox[threadIdx.x] = s[threadIdx.x][0];
}

__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Index along the Hilbert curve of a cell (x0, x1, x2) of the 1024^3 grid,
// after J. Skilling's transpose form (AIP Conf. Proc. 707 (2004) 381): undo
// the excess work level by level, Gray-encode, then interleave the bits with
// x0 most significant.  Consecutive indices are neighbouring cells, so runs of
// consecutive points have tighter boxes than along the Morton curve (which
// jumps): at 4M cloud charges half as many 256-point tile pairs are near
// each other.
__device__ __forceinline__ uint32_t hilbert3(uint32_t x0, uint32_t x1, uint32_t x2) {
  uint32_t X[3] = {x0, x1, x2};
  for (uint32_t Q = 1u << 9; Q > 1u; Q >>= 1) {
    const uint32_t P = Q - 1u;
    if (X[0] & Q) X[0] ^= P;
#pragma unroll
    for (int i = 1; i < 3; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;
      } else {
        const uint32_t t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  X[1] ^= X[0];
  X[2] ^= X[1];
  uint32_t t = 0u;
  for (uint32_t Q = 1u << 9; Q > 1u; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1u;
  X[0] ^= t;
  X[1] ^= t;
  X[2] ^= t;
  return spread3(X[2]) | (spread3(X[1]) << 1) | (spread3(X[0]) << 2);
}

__global__ __launch_bounds__(256) void k_curve_key(int n, const double *__restrict__ x, const double *__restrict__ y,
                                                   const double *__restrict__ z, const double *bbox,
                                                   uint32_t *keys, int32_t *idx) {
  int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double v[3] = {x[i], y[i], z[i]};
  uint32_t q[3];
  // one scale for the three axes, so that runs along the curve are compact
  // in space also in a flat or elongated point set
  const double span = fmax(fmax(bbox[3] - bbox[0], bbox[4] - bbox[1]), bbox[5] - bbox[2]);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double t = span > 0.0 ? (v[c] - bbox[c]) / span : 0.0;
    int qi = (int)(t * 1024.0);
    q[c] = (uint32_t)min(max(qi, 0), 1023);
  }
  keys[i] = hilbert3(q[0], q[1], q[2]);
  idx[i] = i;
}

__global__ __launch_bounds__(256) void k_gather3(int n, const int32_t *__restrict__ perm,
                                                 const double *__restrict__ x, const double *__restrict__ y,
                                                 const double *__restrict__ z, double *out) {
  int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  int j = perm[i];
  out[i] = x[j];
  out[(size_t)n + i] = y[j];
  out[2 * (size_t)n + i] = z[j];
}

static inline int nblk(int64_t n, int t = 256) { return (int)((n + t - 1) / t); }

// Bounding box of each 256-source tile of the source copy (lo xyz, hi xyz).
__global__ __launch_bounds__(256) void k_tile_boxes(int n, const double *__restrict__ src, double *box) {
  __shared__ double red[6][4];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int k = min(i, n - 1);
  double v[6];
  for (int c = 0; c < 3; ++c) v[c] = v[3 + c] = src[(size_t)c * n + k];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v[c] = fmin(v[c], __shfl_xor(v[c], o));
      v[3 + c] = fmax(v[3 + c], __shfl_xor(v[3 + c], o));
    }
  if ((threadIdx.x & 63) == 0)
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x >> 6] = v[c];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int c = threadIdx.x;
    double r = red[c][0];
    for (int w = 1; w < 4; ++w) r = c < 3 ? fmin(r, red[c][w]) : fmax(r, red[c][w]);
    box[6 * (size_t)blockIdx.x + c] = r;
  }
}

void launch_tile_boxes(obem_ctx *ctx, int n, const double *src, double *box) {
  if (n > 0) hipLaunchKernelGGL(k_tile_boxes, dim3(nblk(n)), dim3(256), 0, ctx->stream, n, src, box);
}

// Sources in (charge sign, Hilbert) order: key of the i-th Hilbert-sorted
// source, value its caller index.
__global__ __launch_bounds__(256) void k_charge_key(int n, const int32_t *__restrict__ perm,
                                                    const double *__restrict__ q, uint8_t *key, int32_t *idx) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const int j = perm[i];
    key[i] = q[j] < 0.0 ? 0 : (q[j] > 0.0 ? 1 : 2);
    idx[i] = j;
  }
}

__global__ __launch_bounds__(256) void k_gather_src(int n, const int32_t *__restrict__ perm, const double *__restrict__ x,
                                                    const double *__restrict__ y, const double *__restrict__ z,
                                                    const double *__restrict__ q, double *out, int32_t *inv) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int j = perm[i];
  out[i] = x[j];
  out[(size_t)n + i] = y[j];
  out[2 * (size_t)n + i] = z[j];
  out[3 * (size_t)n + i] = q[j];
  if (inv) inv[j] = i;
}

obem_status order_sources(obem_ctx *ctx, int64_t n64, const double *sx, const double *sy, const double *sz,
                          const double *sq, bool want_inv, SourceOrder *out) {
  const int n = (int)n64;
  const size_t nz = (size_t)n;
  out->n = n;
  if (n == 0) return OBEM_OK;
  TargetOrder mo;
  obem_status st = order_targets(ctx, n, sx, sy, sz, &mo);
  if (st) return st;
  uint8_t *key = (uint8_t *)ws_get(ctx, WS_SRCKEY, 2 * nz + 64);
  int32_t *perm = (int32_t *)ws_get(ctx, WS_SRCPERM, sizeof(int32_t) * 2 * nz);
  double *src = (double *)ws_get(ctx, WS_SRC, sizeof(double) * 4 * nz + nz + 64);
  double *tbox = (double *)ws_get(ctx, WS_TBOX, sizeof(double) * 6 * (size_t)nblk(n));
  int32_t *inv = want_inv ? (int32_t *)ws_get(ctx, WS_SRCINV, sizeof(int32_t) * nz) : nullptr;
  if (!key || !perm || !src || !tbox || (want_inv && !inv)) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  hipLaunchKernelGGL(k_charge_key, dim3(nblk(n)), dim3(256), 0, ctx->stream, n, mo.perm, sq, key, perm);
  size_t tb = 0;
  OBEM_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, tb, key, key + nz, perm, perm + nz, n, 0, 2, ctx->stream));
  void *tmp = ws_get(ctx, WS_SORT_TMP2, tb + 256);
  if (!tmp) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  OBEM_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(tmp, tb, key, key + nz, perm, perm + nz, n, 0, 2, ctx->stream));
  hipLaunchKernelGGL(k_gather_src, dim3(nblk(n)), dim3(256), 0, ctx->stream, n, perm + nz, sx, sy, sz, sq, src, inv);
  launch_tile_boxes(ctx, n, src, tbox);
  OBEM_HIP(ctx, hipGetLastError());
  out->x = src;
  out->y = src + nz;
  out->z = src + 2 * nz;
  out->q = src + 3 * nz;
  out->tbox = tbox;
  out->inv = inv;
  out->perm = perm + nz;
  return OBEM_OK;
}

obem_status order_targets(obem_ctx *ctx, int64_t n64, const double *tx, const double *ty, const double *tz,
                          TargetOrder *out) {
  int n = (int)n64;
  out->n = n;
  if (n == 0) return OBEM_OK;
  OBEM_PROF(ctx, "order");
  const int nb = 256;
  double *bbox = (double *)ws_get(ctx, WS_BBOX, sizeof(double) * (6 * nb + 6));
  uint32_t *k0 = (uint32_t *)ws_get(ctx, WS_KEYS0, sizeof(uint32_t) * n);
  uint32_t *k1 = (uint32_t *)ws_get(ctx, WS_KEYS1, sizeof(uint32_t) * n);
  int32_t *i0 = (int32_t *)ws_get(ctx, WS_IDX0, sizeof(int32_t) * n);
  int32_t *i1 = (int32_t *)ws_get(ctx, WS_IDX1, sizeof(int32_t) * n);
  double *xs = (double *)ws_get(ctx, WS_TSORT, sizeof(double) * 3 * (size_t)n);
  if (!bbox || !k0 || !k1 || !i0 || !i1 || !xs) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(256), 0, ctx->stream, n, tx, ty, tz, bbox + 6);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(256), 0, ctx->stream, nb, bbox + 6, bbox);
  hipLaunchKernelGGL(k_curve_key, dim3(nblk(n)), dim3(256), 0, ctx->stream, n, tx, ty, tz, bbox, k0, i0);
  size_t tmp_bytes = 0;
  OBEM_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, k0, k1, i0, i1, n, 0, 30, ctx->stream));
  void *tmp = ws_get(ctx, WS_SORT_TMP, tmp_bytes + 256);
  if (!tmp) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  OBEM_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, k0, k1, i0, i1, n, 0, 30, ctx->stream));
  hipLaunchKernelGGL(k_gather3, dim3(nblk(n)), dim3(256), 0, ctx->stream, n, i1, tx, ty, tz, xs);
  OBEM_HIP(ctx, hipGetLastError());
  out->perm = i1;
  out->xs = xs;
  return OBEM_OK;
}

// ---------------------------------------------------------------------------
// Cell (panel) field
// ---------------------------------------------------------------------------
constexpr int kPT = 64;               // cells per LDS tile

// One cell of an LDS tile, recentred FP32, as 19 float4 records read whole
// (one address per cell, 128-bit LDS reads):
//   c[0] = centroid, (3 D)^2          c[1] = (40 D)^2, area sigma {w0, wa, wb}
//   c[2..7] = the 7 points of the degree-5 rule (21 floats), area sigma / 3,
//             (6 D)^2, D
//   c[8..10] = the 3 points of the degree-2 rule (9 floats), area sigma
//             {w1, w2} of the 6-point rule, (16 D)^2
//   c[11..15] = the 6 points of the degree-4 rule (18 floats), area sigma
//             {wc, wp} of the 4-point rule
//   c[16..18] = the 3 outer points of the degree-3 rule (9 floats; its
//             fourth point is the centroid), 0, 0, 0
struct PanelCell {
  float4 c[19];
};

// sum over the M rule points of w {e/|e|^3, 1/|e|}, e = target - point
template <int M, bool WANT_V>
__device__ __forceinline__ void panel_points(const float *q, const float *w, float r0, float r1, float r2,
                                             float &px, float &py, float &pz, float &pv) {
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const float ex = r0 - q[3 * m], ey = r1 - q[3 * m + 1], ez = r2 - q[3 * m + 2];
    const float rr = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
    const float ri = __builtin_amdgcn_rsqf(rr);
    const float wr = w[m] * ri;
    const float s_ = wr * (ri * ri);
    px = fmaf(s_, ex, px);
    py = fmaf(s_, ey, py);
    pz = fmaf(s_, ez, pz);
    if (WANT_V) pv += wr;
  }
}

// n consecutive float4 records of a cell into registers
template <int N4>
__device__ __forceinline__ void load4(const float4 *c, float *q) {
#pragma unroll
  for (int u = 0; u < N4; ++u) {
    const float4 t = c[u];
    q[4 * u] = t.x;
    q[4 * u + 1] = t.y;
    q[4 * u + 2] = t.z;
    q[4 * u + 3] = t.w;
  }
}

__device__ __forceinline__ void neumaier(float &s, float &c, float v) {
  float t = s + v;
  if (fabsf(s) >= fabsf(v))
    c += (s - t) + v;
  else
    c += (v - t) + s;
  s = t;
}

// Near cells: FP64 closed form from the FP64 master geometry.
template <bool WANT_V>
__device__ __forceinline__ void near_cell(const double *__restrict__ f, int N, int k, double sig, double x0,
                                          double x1, double x2, double &ex, double &ey, double &ez,
                                          double &ev) {
  d3 P[3];
  P[0] = mk3(f[MF_AX * (size_t)N + k] - x0, f[MF_AY * (size_t)N + k] - x1, f[MF_AZ * (size_t)N + k] - x2);
  P[1] = mk3(f[MF_BX * (size_t)N + k] - x0, f[MF_BY * (size_t)N + k] - x1, f[MF_BZ * (size_t)N + k] - x2);
  P[2] = mk3(f[MF_CX * (size_t)N + k] - x0, f[MF_CY * (size_t)N + k] - x1, f[MF_CZ * (size_t)N + k] - x2);
  d3 n = mk3(f[MF_NX * (size_t)N + k], f[MF_NY * (size_t)N + k], f[MF_NZ * (size_t)N + k]);
  double twoarea = 2.0 * f[MF_AREA * (size_t)N + k];
  d3 IE;
  double IV;
  cell_closed_form<WANT_V>(P, n, twoarea, cell_edges(f, N, k), IE, IV);
  ex = fma(sig, IE.x, ex);
  ey = fma(sig, IE.y, ey);
  ez = fma(sig, IE.z, ez);
  if (WANT_V) ev = fma(sig, IV, ev);
}

template <bool WANT_V>
// gridDim.y splits the cells into ranges of cchunk; split y writes its sums
// to part + 4 n_t y (part = acc when there is one split).
__global__ __launch_bounds__(kThreads) void k_panel_mixed(int n_t, const double *__restrict__ xs, int N,
                                                          const double *__restrict__ f,
                                                          const double *__restrict__ sigma, int cchunk,
                                                          double *part) {
  __shared__ PanelCell T[kPT];
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * kThreads;
  const int i = i0 + tid;
  const bool active = i < n_t;
  const double c0 = xs[i0], c1 = xs[(size_t)n_t + i0], c2 = xs[2 * (size_t)n_t + i0];
  const double x0 = active ? xs[i] : c0;
  const double x1 = active ? xs[(size_t)n_t + i] : c1;
  const double x2 = active ? xs[2 * (size_t)n_t + i] : c2;
  const float r0 = (float)(x0 - c0), r1 = (float)(x1 - c1), r2 = (float)(x2 - c2);
  // the wave's sphere: centre of its targets' bounding box, radius the
  // largest distance from it (widened by 1e-4 for the rounding)
  float cw0, cw1, cw2, rw;
  {
    float lo0 = r0, lo1 = r1, lo2 = r2, hi0 = r0, hi1 = r1, hi2 = r2;
    for (int o = 32; o > 0; o >>= 1) {
      lo0 = fminf(lo0, __shfl_xor(lo0, o));
      lo1 = fminf(lo1, __shfl_xor(lo1, o));
      lo2 = fminf(lo2, __shfl_xor(lo2, o));
      hi0 = fmaxf(hi0, __shfl_xor(hi0, o));
      hi1 = fmaxf(hi1, __shfl_xor(hi1, o));
      hi2 = fmaxf(hi2, __shfl_xor(hi2, o));
    }
    cw0 = 0.5f * (lo0 + hi0);
    cw1 = 0.5f * (lo1 + hi1);
    cw2 = 0.5f * (lo2 + hi2);
    rw = sqrtf(dist2f(r0, r1, r2, cw0, cw1, cw2));
    for (int o = 32; o > 0; o >>= 1) rw = fmaxf(rw, __shfl_xor(rw, o));
    rw *= 1.0001f;
  }
  float hx = 0.f, hy = 0.f, hz = 0.f, hv = 0.f, lx = 0.f, ly = 0.f, lz = 0.f, lv = 0.f;
  const int kb = blockIdx.y * cchunk, ke = min(N, kb + cchunk);
  for (int k0 = kb; k0 < ke; k0 += kPT) {
    const int cnt = min(kPT, ke - k0);
    __syncthreads();
    // staging, coalesced along the cells: the 57 rule coordinates (7-, 3-, 6-
    // and 4-point rules, arrays MF_Q7 + m) of the 64 cells, wave w taking
    // rows m = w, w + 4, ... with lane k on cell k; a row's array, record
    // slot and coordinate are the same for the whole wave, and the wave's
    // loads are all issued before the first is used.  Then one thread per
    // cell for centroid, limits and weights.
    {
      const int k = tid & 63;
      const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
      const bool ok = k < cnt;
      const double *fk = f + (size_t)MF_Q7 * N + k0 + k;
      float *rec = reinterpret_cast<float *>(&T[k]);
      double v[15];
#pragma unroll
      for (int j = 0; j < 15; ++j) {
        const int m = w + 4 * j;
        v[j] = (m < 57 && ok) ? fk[(size_t)m * N] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 15; ++j) {
        const int m = w + 4 * j;
        if (m < 57) {
          const int c = m % 3;
          const double o = c == 0 ? c0 : (c == 1 ? c1 : c2);
          rec[m + (m < 21 ? 8 : (m < 30 ? 11 : (m < 48 ? 14 : 16)))] = ok ? (float)(v[j] - o) : 0.f;
        }
      }
    }
    if (tid < kPT) {
      const int k = tid;
      float4 g = make_float4(0.f, 0.f, 0.f, 0.f), h = g;
      float w3 = 0.f, lim7 = 0.f, lim6 = 0.f, w61 = 0.f, w62 = 0.f, w4c = 0.f, w4p = 0.f, dk = 0.f;
      if (k < cnt) {
        const int kk = k0 + k;
        const double D = f[(size_t)MF_DIAM * N + kk];
        const double as = f[(size_t)MF_AREA * N + kk] * sigma[kk];
        g = make_float4((float)(f[(size_t)MF_GX * N + kk] - c0), (float)(f[(size_t)MF_GY * N + kk] - c1),
                        (float)(f[(size_t)MF_GZ * N + kk] - c2), (float)(kNearMixed * kNearMixed * D * D));
        h = make_float4((float)(kFar3Mixed * kFar3Mixed * D * D), (float)(as * Rule7::w0), (float)(as * Rule7::wa),
                        (float)(as * Rule7::wb));
        w3 = (float)(as * (1.0 / 3.0));
        lim7 = (float)(kFwd6 * kFwd6 * D * D);
        lim6 = (float)(kFwd4 * kFwd4 * D * D);
        dk = (float)D;
        w61 = (float)(as * Rule6::w1);
        w62 = (float)(as * Rule6::w2);
        w4c = (float)(as * Rule4::wc);
        w4p = (float)(as * Rule4::wp);
      }
      float *rec = reinterpret_cast<float *>(&T[k]);
      T[k].c[0] = g;
      T[k].c[1] = h;
      rec[29] = w3;
      rec[30] = lim7;
      rec[31] = dk;
      rec[41] = w61;
      rec[42] = w62;
      rec[43] = lim6;
      rec[62] = w4c;
      rec[63] = w4p;
      rec[73] = rec[74] = rec[75] = 0.f;
    }
    __syncthreads();
    float px = 0.f, py = 0.f, pz = 0.f, pv = 0.f;
    // The rule of each cell for the whole wave, from one test per cell
    // against the wave's sphere: lane k tests cell k, and the ballots give
    // the cells some lane may see within 40 D (4 points or finer), 16 D (6
    // or finer), 6 D (7 points) and 3 D (the per-lane path, which leaves the
    // near pairs to k_panel_near).  Thresholds 1 % wide of the per-lane
    // ones, so that a cell not flagged near has no lane inside 3 D by the
    // per-lane test, and a coarser rule is never taken where a lane needs a
    // finer one.
    uint64_t m3, m4, m6, m7, mnear;
    {
      const int k = tid & 63;
      float t = 3.0e38f, Dk = 0.f;
      if (k < cnt) {
        const float4 g = T[k].c[0];
        Dk = T[k].c[7].w;
        t = sqrtf(dist2f(cw0, cw1, cw2, g.x, g.y, g.z)) - rw;
      }
      const uint64_t f4 = __ballot(t < (float)(kFar3Mixed * 1.01) * Dk);
      const uint64_t f6 = __ballot(t < (float)(kFwd4 * 1.01) * Dk);
      const uint64_t f7 = __ballot(t < (float)(kFwd6 * 1.01) * Dk);
      mnear = __ballot(t < (float)(kNearMixed * 1.01) * Dk);
      m3 = (cnt == 64 ? ~0ull : ((1ull << cnt) - 1ull)) & ~f4;
      m4 = f4 & ~f6;
      m6 = f6 & ~f7;
      m7 = f7 & ~mnear;
    }
    for (; m3; m3 &= m3 - 1ull) {
      const int k = __builtin_ctzll(m3);
      float q[12];
      load4<3>(&T[k].c[8], q);
      const float w3 = T[k].c[7].y;
      const float w[3] = {w3, w3, w3};
      panel_points<3, WANT_V>(q, w, r0, r1, r2, px, py, pz, pv);
    }
    for (; m4; m4 &= m4 - 1ull) {
      const int k = __builtin_ctzll(m4);
      float q[15];
      const float4 g = T[k].c[0];
      q[0] = g.x;
      q[1] = g.y;
      q[2] = g.z;
      load4<3>(&T[k].c[16], q + 3);
      const float4 h15 = T[k].c[15];
      const float w[4] = {h15.z, h15.w, h15.w, h15.w};
      panel_points<4, WANT_V>(q, w, r0, r1, r2, px, py, pz, pv);
    }
    for (; m6; m6 &= m6 - 1ull) {
      const int k = __builtin_ctzll(m6);
      float q[20];
      load4<5>(&T[k].c[11], q);
      const float4 h10 = T[k].c[10];
      const float w[6] = {h10.y, h10.y, h10.y, h10.z, h10.z, h10.z};
      panel_points<6, WANT_V>(q, w, r0, r1, r2, px, py, pz, pv);
    }
    for (; m7; m7 &= m7 - 1ull) {
      const int k = __builtin_ctzll(m7);
      float q[24];
      load4<6>(&T[k].c[2], q);
      const float4 h = T[k].c[1];
      const float w[7] = {h.y, h.z, h.z, h.z, h.w, h.w, h.w};
      panel_points<7, WANT_V>(q, w, r0, r1, r2, px, py, pz, pv);
    }
    for (; mnear; mnear &= mnear - 1ull) {
      const int k = __builtin_ctzll(mnear);
      const float4 g = T[k].c[0];
      const float R2 = dist2f(r0, r1, r2, g.x, g.y, g.z);
      const bool nearp = R2 < g.w;  // taken by k_panel_near in FP64
      const float4 h = T[k].c[1];
      const float4 h7 = T[k].c[7];    // {.., area sigma / 3, (6 D)^2, D}
      const float4 h10 = T[k].c[10];  // {.., w1, w2, (16 D)^2}
      // the rule by distance (7 points within 6 D, 6 within 16 D, 4 within
      // 40 D, 3 beyond), taken for the whole wave at the finest rule one of
      // its lanes needs
      const bool need7 = (!nearp) && (R2 < h7.z);
      const bool need6 = (!nearp) && (R2 < h10.w);
      const bool need4 = (!nearp) && (R2 < h.x);
      if (__any(need7)) {
        if (!nearp) {
          float q[24];
          load4<6>(&T[k].c[2], q);
          const float w[7] = {h.y, h.z, h.z, h.z, h.w, h.w, h.w};
          panel_points<7, WANT_V>(q, w, r0, r1, r2, px, py, pz, pv);
        }
      } else if (__any(need6)) {
        if (!nearp) {
          float q[20];
          load4<5>(&T[k].c[11], q);
          const float w[6] = {h10.y, h10.y, h10.y, h10.z, h10.z, h10.z};
          panel_points<6, WANT_V>(q, w, r0, r1, r2, px, py, pz, pv);
        }
      } else if (__any(need4)) {
        if (!nearp) {
          float q[15];
          q[0] = g.x;
          q[1] = g.y;
          q[2] = g.z;
          load4<3>(&T[k].c[16], q + 3);
          const float4 h15 = T[k].c[15];
          const float w[4] = {h15.z, h15.w, h15.w, h15.w};
          panel_points<4, WANT_V>(q, w, r0, r1, r2, px, py, pz, pv);
        }
      } else if (!nearp) {
        float q[12];
        load4<3>(&T[k].c[8], q);
        const float w[3] = {h7.y, h7.y, h7.y};
        panel_points<3, WANT_V>(q, w, r0, r1, r2, px, py, pz, pv);
      }
    }
    neumaier(hx, lx, px);
    neumaier(hy, ly, py);
    neumaier(hz, lz, pz);
    if (WANT_V) neumaier(hv, lv, pv);
  }
  if (active) {
    double *acc = part + (size_t)blockIdx.y * 4 * n_t;
    acc[i] = (double)hx + (double)lx;
    acc[(size_t)n_t + i] = (double)hy + (double)ly;
    acc[2 * (size_t)n_t + i] = (double)hz + (double)lz;
    acc[3 * (size_t)n_t + i] = WANT_V ? (double)hv + (double)lv : 0.0;
  }
}

// FP64 near zone (R < 3 D) of the mixed mode, added to the far kernel's
// partial sums of the same cell range (gridDim.y splits the cells as in the
// far kernel, so small target sets still fill the chip).  Each wave bounds
// its 64 targets by a sphere and skips whole 64-cell tiles whose near-zone
// sphere (tile centre, max over cells of |c_k - centre| + 3 D_k, slightly
// inflated) it does not meet; inside a tile the per-pair test is the far
// kernel's FP32 test, so the two kernels partition the pairs.
template <bool WANT_V>
__global__ __launch_bounds__(kThreads) void k_panel_near(int n_t, const double *__restrict__ xs, int N,
                                                         const double *__restrict__ f,
                                                         const double *__restrict__ sigma,
                                                         const double *__restrict__ tiles, int cchunk,
                                                         double *part) {
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * kThreads;
  const int i = i0 + tid;
  const bool active = i < n_t;
  const int ii = active ? i : n_t - 1;
  const double c0 = xs[i0], c1 = xs[(size_t)n_t + i0], c2 = xs[2 * (size_t)n_t + i0];
  const double x0 = xs[ii], x1 = xs[(size_t)n_t + ii], x2 = xs[2 * (size_t)n_t + ii];
  const float r0 = (float)(x0 - c0), r1 = (float)(x1 - c1), r2 = (float)(x2 - c2);
  // wave bounding sphere
  double lo0 = x0, lo1 = x1, lo2 = x2, hi0 = x0, hi1 = x1, hi2 = x2;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo0 = fmin(lo0, __shfl_xor(lo0, o));
    lo1 = fmin(lo1, __shfl_xor(lo1, o));
    lo2 = fmin(lo2, __shfl_xor(lo2, o));
    hi0 = fmax(hi0, __shfl_xor(hi0, o));
    hi1 = fmax(hi1, __shfl_xor(hi1, o));
    hi2 = fmax(hi2, __shfl_xor(hi2, o));
  }
  const double wc0 = 0.5 * (lo0 + hi0), wc1 = 0.5 * (lo1 + hi1), wc2 = 0.5 * (lo2 + hi2);
  const double wr = 0.5 * sqrt((hi0 - lo0) * (hi0 - lo0) + (hi1 - lo1) * (hi1 - lo1) + (hi2 - lo2) * (hi2 - lo2));
  // the same sphere in the recentred FP32 frame, radius measured from its
  // FP32 centre (widened by 1e-4 for the rounding)
  const float fw0 = (float)(wc0 - c0), fw1 = (float)(wc1 - c1), fw2 = (float)(wc2 - c2);
  float fwr = sqrtf(dist2f(r0, r1, r2, fw0, fw1, fw2));
  for (int o = 32; o > 0; o >>= 1) fwr = fmaxf(fwr, __shfl_xor(fwr, o));
  fwr *= 1.0001f;
  const int lane = tid & 63;
  // the cell range of split blockIdx.y (cchunk is a multiple of the tile)
  const int tb = blockIdx.y * cchunk / kPT, te = (min(N, (blockIdx.y + 1) * cchunk) + kPT - 1) / kPT;
  double ex = 0.0, ey = 0.0, ez = 0.0, ev = 0.0;
  for (int t = tb; t < te; ++t) {
    const double dx = wc0 - tiles[4 * t], dy = wc1 - tiles[4 * t + 1], dz = wc2 - tiles[4 * t + 2];
    const double rs = wr + tiles[4 * t + 3];
    if (dx * dx + dy * dy + dz * dz > rs * rs) continue;  // wave-uniform
    const int k0 = t * kPT, cnt = min(kPT, N - k0);
    // lane k holds cell k0 + k (centroid recentred to FP32 and the near
    // limit, exactly as the far kernel stages them) and tests it once
    // against the wave's sphere; only the cells some lane may see within
    // 3 D (1 % wide) take the per-lane test
    float g0 = 0.f, g1 = 0.f, g2 = 0.f, lim = 0.f, dk = 0.f;
    if (lane < cnt) {
      const int kk = k0 + lane;
      g0 = (float)(f[(size_t)MF_GX * N + kk] - c0);
      g1 = (float)(f[(size_t)MF_GY * N + kk] - c1);
      g2 = (float)(f[(size_t)MF_GZ * N + kk] - c2);
      const double D = f[(size_t)MF_DIAM * N + kk];
      lim = (float)(kNearMixed * kNearMixed * D * D);
      dk = (float)D;
    }
    const float tw = sqrtf(dist2f(fw0, fw1, fw2, g0, g1, g2)) - fwr;
    for (uint64_t m = __ballot(lane < cnt && tw < (float)(kNearMixed * 1.01) * dk); m; m &= m - 1ull) {
      const int k = __builtin_ctzll(m);
      const float h0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g0), k));
      const float h1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g1), k));
      const float h2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g2), k));
      const float hl = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lim), k));
      const bool nearp = active && dist2f(r0, r1, r2, h0, h1, h2) < hl;
      if (__any(nearp)) {
        const int kk = k0 + k;
        if (nearp) near_cell<WANT_V>(f, N, kk, sigma[kk], x0, x1, x2, ex, ey, ez, ev);
      }
    }
  }
  if (active) {
    double *acc = part + (size_t)blockIdx.y * 4 * n_t;
    acc[i] += ex;
    acc[(size_t)n_t + i] += ey;
    acc[2 * (size_t)n_t + i] += ez;
    if (WANT_V) acc[3 * (size_t)n_t + i] += ev;
  }
}

// FP64 mode: closed form up to 48 diameters (k_panel_fp64_near), FP64
// 7-point rule beyond (k_panel_fp64).  Both decide with the same FP64 test
// |x - c_k|^2 >= (48 D_k)^2 on the unmodified coordinates.
constexpr int kPF = 32;  // cells per LDS tile of the FP64 far kernel

// One cell of the FP64 far kernel's LDS tile: centroid, (48 D)^2, the 7 rule
// points, area sigma {w0, wa, wa, wa, wb, wb, wb} folded per point.
struct CellF64 {
  double g[3], lim, q[21], w[7];
};

// The value of lane k (wave-uniform k) of a double.
__device__ __forceinline__ double readlane_f64(double v, int k) {
  const unsigned long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, k);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), k);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton steps
// y <- y + y (1/2 - x/2 y^2) (quadratic convergence; a few ulp at the end).
__device__ __forceinline__ double rsqrt_f64(double x) {
  const double h = 0.5 * x;
  double y = __builtin_amdgcn_rsq(x);
  y = fma(y, fma(-h * y, y, 0.5), y);
  y = fma(y, fma(-h * y, y, 0.5), y);
  return y;
}

template <bool WANT_V>
__global__ __launch_bounds__(kThreads) void k_panel_fp64(int n_t, const double *__restrict__ xs, int N,
                                                         const double *__restrict__ f,
                                                         const double *__restrict__ sigma, int cchunk,
                                                         double *part) {
  __shared__ CellF64 T[kPF];
  const int tid = threadIdx.x;
  const int i = blockIdx.x * kThreads + tid;
  const bool active = i < n_t;
  const int ii = active ? i : 0;
  const double x0 = xs[ii], x1 = xs[(size_t)n_t + ii], x2 = xs[2 * (size_t)n_t + ii];
  double ex = 0.0, ey = 0.0, ez = 0.0, ev = 0.0;
  const int kb = blockIdx.y * cchunk, ke = min(N, kb + cchunk);
  for (int k0 = kb; k0 < ke; k0 += kPF) {
    const int cnt = min(kPF, ke - k0);
    __syncthreads();
    for (int idx = tid; idx < 21 * kPF; idx += kThreads) {
      const int m = idx / kPF, k = idx % kPF;
      if (k < cnt) T[k].q[m] = f[(size_t)(MF_Q7 + m) * N + k0 + k];
    }
    if (tid < cnt) {
      const int kk = k0 + tid;
      const double D = f[(size_t)MF_DIAM * N + kk];
      const double as = f[(size_t)MF_AREA * N + kk] * sigma[kk];
      T[tid].g[0] = f[(size_t)MF_GX * N + kk];
      T[tid].g[1] = f[(size_t)MF_GY * N + kk];
      T[tid].g[2] = f[(size_t)MF_GZ * N + kk];
      T[tid].lim = kQuadFp64 * kQuadFp64 * D * D;
#pragma unroll
      for (int m = 0; m < 7; ++m) T[tid].w[m] = as * (m == 0 ? Rule7::w0 : (m < 4 ? Rule7::wa : Rule7::wb));
    }
    __syncthreads();
    for (int k = 0; k < cnt; ++k) {
      const double dx = x0 - T[k].g[0], dy = x1 - T[k].g[1], dz = x2 - T[k].g[2];
      const double R2 = fma(dx, dx, fma(dy, dy, dz * dz));
      if (R2 >= T[k].lim) {  // the near kernel takes the others
#pragma unroll
        for (int m = 0; m < 7; ++m) {
          const double qx = x0 - T[k].q[3 * m], qy = x1 - T[k].q[3 * m + 1], qz = x2 - T[k].q[3 * m + 2];
          const double ri = rsqrt_f64(fma(qx, qx, fma(qy, qy, qz * qz)));
          const double wr = T[k].w[m] * ri;
          const double t = wr * ri * ri;
          ex = fma(t, qx, ex);
          ey = fma(t, qy, ey);
          ez = fma(t, qz, ez);
          if (WANT_V) ev += wr;
        }
      }
    }
  }
  if (active) {
    double *acc = part + (size_t)blockIdx.y * 4 * n_t;
    acc[i] = ex;
    acc[(size_t)n_t + i] = ey;
    acc[2 * (size_t)n_t + i] = ez;
    acc[3 * (size_t)n_t + i] = ev;
  }
}

// FP64 closed-form zone (R < 48 D), added to the far kernel's partial sums
// of the same cell range (split by gridDim.y as in the far kernel).  Each
// wave bounds its 64 targets by a sphere and visits the 64-cell tiles whose
// zone sphere (centre, max_k |c_k - centre| + 48 D_k) it meets.
template <bool WANT_V>
__global__ __launch_bounds__(kThreads) void k_panel_fp64_near(int n_t, const double *__restrict__ xs, int N,
                                                              const double *__restrict__ f,
                                                              const double *__restrict__ sigma,
                                                              const double *__restrict__ tiles, int cchunk,
                                                              double *part) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const bool active = i < n_t;
  const int i0 = blockIdx.x * kThreads;
  const int ii = active ? i : i0;
  const double x0 = xs[ii], x1 = xs[(size_t)n_t + ii], x2 = xs[2 * (size_t)n_t + ii];
  double lo0 = x0, lo1 = x1, lo2 = x2, hi0 = x0, hi1 = x1, hi2 = x2;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo0 = fmin(lo0, __shfl_xor(lo0, o));
    lo1 = fmin(lo1, __shfl_xor(lo1, o));
    lo2 = fmin(lo2, __shfl_xor(lo2, o));
    hi0 = fmax(hi0, __shfl_xor(hi0, o));
    hi1 = fmax(hi1, __shfl_xor(hi1, o));
    hi2 = fmax(hi2, __shfl_xor(hi2, o));
  }
  const double wc0 = 0.5 * (lo0 + hi0), wc1 = 0.5 * (lo1 + hi1), wc2 = 0.5 * (lo2 + hi2);
  const double wr = 0.5 * sqrt((hi0 - lo0) * (hi0 - lo0) + (hi1 - lo1) * (hi1 - lo1) + (hi2 - lo2) * (hi2 - lo2));
  // the cell range of split blockIdx.y (cchunk is a multiple of the tile)
  const int tb = blockIdx.y * cchunk / 64, te = (min(N, (blockIdx.y + 1) * cchunk) + 63) / 64;
  double ex = 0.0, ey = 0.0, ez = 0.0, ev = 0.0;
  for (int t = tb; t < te; ++t) {
    const double dx = wc0 - tiles[4 * t], dy = wc1 - tiles[4 * t + 1], dz = wc2 - tiles[4 * t + 2];
    const double rs = (wr + tiles[4 * t + 3]) * (1.0 + 1e-9);
    if (dx * dx + dy * dy + dz * dz > rs * rs) continue;  // wave-uniform
    const int k0 = t * 64, cnt = min(64, N - k0);
    // lane k holds cell k0 + k and tests it once against the wave's sphere
    // (0.1 % wide); only the cells some lane may see within 48 D take the
    // per-lane test, on the same FP64 values as the far kernel's
    const int lane = threadIdx.x & 63;
    double cg0 = 0.0, cg1 = 0.0, cg2 = 0.0, cD = 0.0;
    bool flag = false;
    if (lane < cnt) {
      const int kk = k0 + lane;
      cg0 = f[(size_t)MF_GX * N + kk];
      cg1 = f[(size_t)MF_GY * N + kk];
      cg2 = f[(size_t)MF_GZ * N + kk];
      cD = f[(size_t)MF_DIAM * N + kk];
      const double u0 = cg0 - wc0, u1 = cg1 - wc1, u2 = cg2 - wc2;
      flag = sqrt(u0 * u0 + u1 * u1 + u2 * u2) - wr < kQuadFp64 * 1.001 * cD;
    }
    for (uint64_t m = __ballot(flag); m; m &= m - 1ull) {
      const int k = __builtin_ctzll(m);
      const int kk = k0 + k;
      const double gx = x0 - readlane_f64(cg0, k), gy = x1 - readlane_f64(cg1, k), gz = x2 - readlane_f64(cg2, k);
      const double D = readlane_f64(cD, k);
      const bool nearp = active && !(fma(gx, gx, fma(gy, gy, gz * gz)) >= kQuadFp64 * kQuadFp64 * D * D);
      if (__any(nearp)) {
        if (nearp) near_cell<WANT_V>(f, N, kk, sigma[kk], x0, x1, x2, ex, ey, ez, ev);
      }
    }
  }
  if (active) {
    double *acc = part + (size_t)blockIdx.y * 4 * n_t;
    acc[i] += ex;
    acc[(size_t)n_t + i] += ey;
    acc[2 * (size_t)n_t + i] += ez;
    if (WANT_V) acc[3 * (size_t)n_t + i] += ev;
  }
}

// acc = sum of the cell-split partials, in split order.
__global__ __launch_bounds__(256) void k_panel_reduce(int n_t, int ns, const double *__restrict__ part, double *acc) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_t) return;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double s = 0.0;
    for (int y = 0; y < ns; ++y) s += part[((size_t)y * 4 + c) * n_t + i];
    acc[(size_t)c * n_t + i] = s;
  }
}

obem_status launch_panel_field(obem_ctx *ctx, const obem_meshh *m, const double *sigma, const TargetOrder &to,
                               obem_precision prec, bool want_v, double *acc) {
  const int n_t = to.n;
  if (n_t == 0) return OBEM_OK;
  const int N = (int)m->n;
  const int bt = nblk(n_t);
  // cell ranges of >= 64 cells (a multiple of both LDS tiles), about
  // kSplitWorkgroups workgroups in all
  int ns = std::max(1, std::min((kSplitWorkgroups + bt - 1) / bt, (N + 63) / 64));
  ns = std::min(ns, 64);
  int cchunk = (N + ns - 1) / ns;
  cchunk = (cchunk + 63) / 64 * 64;
  ns = (N + cchunk - 1) / cchunk;
  double *part = acc;
  if (ns > 1) {
    part = (double *)ws_get(ctx, WS_PANEL, sizeof(double) * 4 * (size_t)n_t * ns);
    if (!part) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  }
  dim3 gsplit(bt, ns), block(kThreads);
  OBEM_PROF(ctx, "panel");
#define PANEL_FAR(K, V, ...) \
  hipLaunchKernelGGL(K<V>, gsplit, block, 0, ctx->stream, n_t, to.xs, N, m->f, sigma, cchunk, part __VA_ARGS__)
  if (prec == OBEM_MIXED) {
    if (want_v) PANEL_FAR(k_panel_mixed, true); else PANEL_FAR(k_panel_mixed, false);
  } else {
    if (want_v) PANEL_FAR(k_panel_fp64, true); else PANEL_FAR(k_panel_fp64, false);
  }
  // the near kernel of split y adds the closed-form pairs of the same cell
  // range into the same slot (one writer per entry, after the far kernel),
  // then the slots are added in split order
#define PANEL_NEAR(K, V, T) \
  hipLaunchKernelGGL(K<V>, gsplit, block, 0, ctx->stream, n_t, to.xs, N, m->f, sigma, T, cchunk, part)
  if (prec == OBEM_MIXED) {
    if (want_v) PANEL_NEAR(k_panel_near, true, m->tiles); else PANEL_NEAR(k_panel_near, false, m->tiles);
  } else {
    if (want_v) PANEL_NEAR(k_panel_fp64_near, true, m->tiles48); else PANEL_NEAR(k_panel_fp64_near, false, m->tiles48);
  }
#undef PANEL_NEAR
#undef PANEL_FAR
  if (ns > 1) hipLaunchKernelGGL(k_panel_reduce, dim3(nblk(n_t)), dim3(256), 0, ctx->stream, n_t, ns, part, acc);
  OBEM_HIP(ctx, hipGetLastError());
  return OBEM_OK;
}

// ---------------------------------------------------------------------------
// Pairwise point-charge field, eq. (nbody) with Plummer softening
// ---------------------------------------------------------------------------
// Each workgroup takes 256 consecutive (sorted) targets and one chunk of the
// sources (gridDim.y chunks, so small target sets still fill the chip), and
// writes per-chunk partial sums part[chunk][4][n_t] (Ex, Ey, Ez, V) plus the
// nearest opposite-species source; k_pair_reduce then sums the chunks in
// order.  Source tiles of 256 are staged in LDS (recentred FP32 position and
// charge, read as broadcasts).
// Species keys: electron 0 looks for cation 1 and vice versa.
__device__ __forceinline__ int want_key(int8_t s) { return s == 0 ? 1 : (s == 1 ? 0 : -2); }

// EXCL: 0 = no exclusion (a coincident term contributes exactly 0 to E when
// soft > 0), 1 = drop zero-distance terms (soft == 0), 2 = drop the source
// whose index equals the target's caller index (targets are the sources).
// HL: the recentred coordinates are carried as FP32 pairs (hi, lo) with
// hi + lo = the FP64 difference to the origin to about 2^-48 of it, and
// r - s = (r_hi - s_hi) + (r_lo - s_lo): both differences are exact or
// nearly so, so the separation keeps a relative error of a few 2^-24 however
// close the pair is, instead of 2^-24 (|r| + |s|) / |r - s| with the hi parts
// alone (tiles near the workgroup's targets, where the closest pairs are).
template <bool WANT_V, bool NN, int EXCL, bool FOLDQ, bool HL>
__device__ __forceinline__ void pair_term(const float4 *S, const float4 *SL, const int *K, int jj, int jt,
                                          float r0, float r1, float r2, float rl0, float rl1, float rl2,
                                          float soft2, int self, int want, float &px, float &py, float &pz,
                                          float &pv, float &best, int &bidx) {
  const float4 s = S[jj];
  float dx = r0 - s.x, dy = r1 - s.y, dz = r2 - s.z;
  if (HL) {
    const float4 l = SL[jj];
    dx += rl0 - l.x;
    dy += rl1 - l.y;
    dz += rl2 - l.z;
  }
  const float rr = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, soft2)));
  float ri = __builtin_amdgcn_rsqf(rr);
  if (EXCL == 1) ri = rr > 0.f ? ri : 0.f;
  if (EXCL == 2) ri = (jt + jj == self) ? 0.f : ri;
  const float qr = FOLDQ ? ri : s.w * ri;
  const float w = qr * (ri * ri);
  px = fmaf(w, dx, px);
  py = fmaf(w, dy, py);
  pz = fmaf(w, dz, pz);
  if (WANT_V) pv += qr;
  if (NN) {
    if (K[jj] == want && rr < best && (EXCL != 1 || rr > 0.f)) {
      best = rr;
      bidx = jt + jj;
    }
  }
}

// The (hi, lo) loop is unrolled by 2 only, so that its extra registers do
// not lower the occupancy of the kernel (unrolled by 1 it was 10 % slower,
// by 4 5 %, in the 4M-charge step where it takes nearly every tile pair of
// the directed remainder).
template <bool WANT_V, bool NN, int EXCL, bool FOLDQ, bool HL>
__device__ __forceinline__ void pair_tile(const float4 *S, const float4 *SL, const float (*RL)[kThreads],
                                          const int *K, int cnt, int jt, float r0, float r1, float r2, float soft2,
                                          int self, int want, float &px, float &py, float &pz, float &pv,
                                          float &best, int &bidx) {
  float rl0 = 0.f, rl1 = 0.f, rl2 = 0.f;
  if constexpr (HL) {
    rl0 = RL[0][threadIdx.x];
    rl1 = RL[1][threadIdx.x];
    rl2 = RL[2][threadIdx.x];
#pragma unroll 2
    for (int jj = 0; jj < cnt; ++jj)
      pair_term<WANT_V, NN, EXCL, FOLDQ, true>(S, SL, K, jj, jt, r0, r1, r2, rl0, rl1, rl2, soft2, self, want, px,
                                               py, pz, pv, best, bidx);
  } else {
    for (int jj = 0; jj < cnt; ++jj)
      pair_term<WANT_V, NN, EXCL, FOLDQ, false>(S, SL, K, jj, jt, r0, r1, r2, rl0, rl1, rl2, soft2, self, want, px,
                                                py, pz, pv, best, bidx);
  }
}

// Far tiles of one charge (the tile's box at least 2 R_b from the box of the
// workgroup's targets, R_b = their largest distance from the recentring
// origin): |r - s|^2 = (|r|^2 + soft^2) + |s|^2 - 2 r.s and E = r sum(w) -
// sum(w s), 11 VALU per pair instead of 12.  Since |s| <= |r| + |r - s|, the
// expansion's terms are at most (1 + 2 R_b / |r - s|)^2 <= 4 times |r - s|^2,
// which bounds its rounding error to a few ulps of |r - s|^2.
__device__ __forceinline__ void pair_tile_far(const float4 *S2, int cnt, float m0, float m1, float m2, float a,
                                              float &sw, float &sx, float &sy, float &sz) {
  for (int jj = 0; jj < cnt; ++jj) {
    const float4 s = S2[jj];
    const float rr = fmaf(m0, s.x, fmaf(m1, s.y, fmaf(m2, s.z, a + s.w)));
    const float ri = __builtin_amdgcn_rsqf(rr);
    const float w = ri * (ri * ri);
    sw += w;
    sx = fmaf(w, s.x, sx);
    sy = fmaf(w, s.y, sy);
    sz = fmaf(w, s.z, sz);
  }
}

// Per super-block: the centre of the box around its tiles' boxes (the
// origin the pair-once kernel recentres on) and the squared distance from
// it to the box's corners, sb[4 A + 0..2] and sb[4 A + 3].
__global__ __launch_bounds__(256) void k_sym_radius(int n, int ns, int sym_tiles, const double *__restrict__ tbox,
                                                    double *sb) {
  const int A = blockIdx.x * 256 + threadIdx.x;
  if (A >= ns) return;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int k = 0; k < sym_tiles && (A * sym_tiles + k) * kThreads < n; ++k) {
    const double *bx = tbox + 6 * (size_t)(A * sym_tiles + k);
    for (int c = 0; c < 3; ++c) {
      lo[c] = fmin(lo[c], bx[c]);
      hi[c] = fmax(hi[c], bx[3 + c]);
    }
  }
  double r2 = 0.0;
  for (int c = 0; c < 3; ++c) {
    sb[4 * (size_t)A + c] = 0.5 * (lo[c] + hi[c]);
    const double h = 0.5 * (hi[c] - lo[c]);
    r2 = fma(h, h, r2);
  }
  sb[4 * (size_t)A + 3] = r2;
}

// Bit b of row a (32 tiles per word): tile_pair_direct(a, b), for the
// directed kernel to skip the other tiles by one scalar bit test.
__global__ __launch_bounds__(256) void k_tile_mask(int ntile, int wpr, int sym_tiles, int nn, double cut2,
                                                   const double *__restrict__ tbox, const double *__restrict__ sb,
                                                   uint32_t *mask) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (size_t)ntile * wpr) return;
  const int a = (int)(t / wpr), w = (int)(t % wpr);
  uint32_t m = 0;
  for (int u = 0; u < 32; ++u) {
    const int b = w * 32 + u;
    if (b < ntile && tile_pair_direct(tbox, sb, a, b, sym_tiles, nn != 0, cut2)) m |= 1u << u;
  }
  mask[t] = m;
}

template <bool WANT_V, bool NN, int EXCL>
__global__ __launch_bounds__(kThreads, 7) void k_pair_mixed(int n_t, const double *__restrict__ xs,
                                                         const int32_t *__restrict__ perm, int n_s,
                                                         const double *__restrict__ sx,
                                                         const double *__restrict__ sy,
                                                         const double *__restrict__ sz,
                                                         const double *__restrict__ sq,
                                                         const int8_t *__restrict__ species,
                                                         const int8_t *__restrict__ species_s, float soft2,
                                                         int chunk, double *part, float *nn_d2p,
                                                         int32_t *nn_ip, const double *__restrict__ tbox,
                                                         float nn_cut2, const int32_t *__restrict__ self_map,
                                                         int sym_tiles, double nn_cut2d,
                                                         const uint32_t *__restrict__ dmask, int dwpr) {
  constexpr bool kFar = (EXCL == 0) && !WANT_V;  // expanded far tiles allowed
  __shared__ float4 S[kThreads];
  __shared__ float4 SL[kThreads];
  __shared__ float RL[3][kThreads];  // lo parts of the targets (read by the (hi, lo) tiles only)
  __shared__ float4 S2[kFar ? kThreads : 1];
  __shared__ int K[kThreads];
  __shared__ float WB[kThreads / 64][6];
  // one-dimensional grid, the source chunks of a target tile consecutive:
  // with targets = sources nearly all the directed tile pairs of a target
  // tile lie in one chunk, so the busy workgroups are spread evenly over the
  // launch instead of coming in one block per chunk
  const int nsplit = (n_s + chunk - 1) / chunk;
  const int tt = (int)blockIdx.x / nsplit, split = (int)blockIdx.x % nsplit;
  const int tid = threadIdx.x;
  const int i0 = tt * kThreads;
  const int i = i0 + tid;
  const bool active = i < n_t;
  const double c0 = xs[i0], c1 = xs[(size_t)n_t + i0], c2 = xs[2 * (size_t)n_t + i0];
  const double x0 = active ? xs[i] : c0;
  const double x1 = active ? xs[(size_t)n_t + i] : c1;
  const double x2 = active ? xs[2 * (size_t)n_t + i] : c2;
  const double e0 = x0 - c0, e1 = x1 - c1, e2 = x2 - c2;
  const float r0 = (float)e0, r1 = (float)e1, r2 = (float)e2;
  RL[0][tid] = (float)(e0 - (double)r0);
  RL[1][tid] = (float)(e1 - (double)r1);
  RL[2][tid] = (float)(e2 - (double)r2);
  const float m0 = -2.f * r0, m1 = -2.f * r1, m2 = -2.f * r2;
  const float a_t = fmaf(r0, r0, fmaf(r1, r1, fmaf(r2, r2, soft2)));
  int want = -2;
  if (NN && active) want = want_key(species[perm[i]]);
  // which partner species any target of the workgroup looks for (the step's
  // source charges follow their species: cations +e, electrons and anions -e)
  bool want_pos = false, want_neg = false;
  if (NN) {
    want_pos = __syncthreads_or(want == 1);
    want_neg = __syncthreads_or(want == 0);
  }
  const int self = active ? (self_map ? self_map[perm[i]] : perm[i]) : -1;
  const int jb = split * chunk;
  const int je = min(n_s, jb + chunk);
  // Bounding box of the workgroup's targets (recentred FP32), tested against
  // each source tile's box (tbox, FP64, 256-source tiles): tiles farther
  // than the partner cut skip the nearest-partner search, far tiles take the
  // expanded form, near ones the (hi, lo) separation.  Inactive lanes hold
  // the first target, which is inside the box.
  float bl0 = r0, bl1 = r1, bl2 = r2, bh0 = r0, bh1 = r1, bh2 = r2;
  if (tbox) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      bl0 = fminf(bl0, __shfl_xor(bl0, o));
      bl1 = fminf(bl1, __shfl_xor(bl1, o));
      bl2 = fminf(bl2, __shfl_xor(bl2, o));
      bh0 = fmaxf(bh0, __shfl_xor(bh0, o));
      bh1 = fmaxf(bh1, __shfl_xor(bh1, o));
      bh2 = fmaxf(bh2, __shfl_xor(bh2, o));
    }
    if ((tid & 63) == 0) {
      float *w = WB[tid >> 6];
      w[0] = bl0; w[1] = bl1; w[2] = bl2; w[3] = bh0; w[4] = bh1; w[5] = bh2;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kThreads / 64; ++k) {
      bl0 = fminf(bl0, WB[k][0]);
      bl1 = fminf(bl1, WB[k][1]);
      bl2 = fminf(bl2, WB[k][2]);
      bh0 = fmaxf(bh0, WB[k][3]);
      bh1 = fmaxf(bh1, WB[k][4]);
      bh2 = fmaxf(bh2, WB[k][5]);
    }
  }
  // R_b^2: squared distance from the origin to the farthest corner of the
  // targets' box.  Tiles at least 2 R_b away (squared gap, with a margin
  // for the FP32 boxes) take the expanded form; tiles nearer than R_b / 4
  // take the (hi, lo) separation: beyond that |r - s| >= R_b / 4 and
  // |r|, |s| - |r - s| <= R_b bound the hi-only separation's relative error
  // by about 10 * 2^-24.
  const float rb2 = fmaxf(bl0 * bl0, bh0 * bh0) + fmaxf(bl1 * bl1, bh1 * bh1) + fmaxf(bl2 * bl2, bh2 * bh2);
  const float far2 = 4.f * rb2 * 1.001f + 1e-30f;
  const float close2 = 0.0625f * rb2 * 1.001f + 1e-30f;
  float hx = 0.f, hy = 0.f, hz = 0.f, hv = 0.f, lx = 0.f, ly = 0.f, lz = 0.f, lv = 0.f;
  float best = INFINITY;
  int bidx = -1;
  for (int jt = jb; jt < je; jt += kThreads) {
    // targets are the sources in the same order under sym_tiles: this
    // workgroup's targets are source tile tt, and the tile pairs that
    // tile_pair_direct (dmask, row tt) does not keep here are evaluated by
    // k_pair_sym; skip to the next tile of the row, a word (32 tiles) at a
    // time (scalar)
    if (sym_tiles) {
      const uint32_t *mrow = dmask + (size_t)tt * dwpr;
      const int be = (je + kThreads - 1) / kThreads;
      int b = jt / kThreads;
      uint32_t wd = mrow[b >> 5] >> (b & 31);
      while (wd == 0u) {
        b = (b | 31) + 1;
        if (b >= be) break;
        wd = mrow[b >> 5];
      }
      if (b >= be) break;
      b += __builtin_ctz(wd);
      if (b >= be) break;
      jt = b * kThreads;
    }
    const int cnt = min(kThreads, je - jt);
    const float q0 = (float)sq[jt];
    bool nn_tile = NN;
    bool far_tile = false;
    bool close_tile = true;
    if (tbox) {
      const double *b = tbox + 6 * (size_t)(jt / kThreads);
      const float g0 = fmaxf(0.f, fmaxf((float)(b[0] - c0) - bh0, bl0 - (float)(b[3] - c0)));
      const float g1 = fmaxf(0.f, fmaxf((float)(b[1] - c1) - bh1, bl1 - (float)(b[4] - c1)));
      const float g2 = fmaxf(0.f, fmaxf((float)(b[2] - c2) - bh2, bl2 - (float)(b[5] - c2)));
      const float gap2 = fmaf(g0, g0, fmaf(g1, g1, g2 * g2));
      if (NN) nn_tile = gap2 <= nn_cut2;
      far_tile = kFar && !nn_tile && gap2 >= far2;
      close_tile = gap2 < close2;
    }
    if (sym_tiles) {
      const bool np = NN && tiles_gap2(tbox, tt, jt / kThreads) <= nn_cut2d;
      nn_tile = np;
      far_tile = far_tile && !np;
    }
    __syncthreads();
    float qj = q0;
    if (tid < cnt) {
      const int j = jt + tid;
      qj = (float)sq[j];
      const double f0 = sx[j] - c0, f1 = sy[j] - c1, f2 = sz[j] - c2;
      const float s0 = (float)f0, s1 = (float)f1, s2 = (float)f2;
      S[tid] = make_float4(s0, s1, s2, qj);
      if (close_tile)
        SL[tid] = make_float4((float)(f0 - (double)s0), (float)(f1 - (double)s1), (float)(f2 - (double)s2), 0.f);
      if (kFar) S2[tid] = make_float4(s0, s1, s2, fmaf(s0, s0, fmaf(s1, s1, s2 * s2)));
      if (NN) K[tid] = species_s[j];
    }
    // tiles of equal charges (sources grouped by species) take the charge
    // out of the inner loop: 12 instead of 13 VALU operations per pair
    const bool uniform = __syncthreads_and(qj == q0);
    // a tile of one charge sign holds no species any target looks for: no
    // partner search there
    if (NN && nn_tile && uniform && ((q0 > 0.f && !want_pos) || (q0 < 0.f && !want_neg))) nn_tile = false;
    float px = 0.f, py = 0.f, pz = 0.f, pv = 0.f;
#define PAIR_TILE(NNT, FQ, HLT)                                                                                \
  pair_tile<WANT_V, NNT, EXCL, FQ, HLT>(S, SL, RL, K, cnt, jt, r0, r1, r2, soft2, self, want, px, py, pz, pv, best, \
                                        bidx)
    if (uniform) {
      if (nn_tile) {
        if (close_tile)
          PAIR_TILE(NN, true, true);
        else
          PAIR_TILE(NN, true, false);
      } else if (kFar && far_tile) {
        float sw = 0.f, sxx = 0.f, syy = 0.f, szz = 0.f;
        pair_tile_far(S2, cnt, m0, m1, m2, a_t, sw, sxx, syy, szz);
        px = fmaf(r0, sw, -sxx);
        py = fmaf(r1, sw, -syy);
        pz = fmaf(r2, sw, -szz);
      } else if (close_tile) {
        PAIR_TILE(false, true, true);
      } else {
        PAIR_TILE(false, true, false);
      }
      px *= q0;
      py *= q0;
      pz *= q0;
      pv *= q0;
    } else {
      if (nn_tile) {
        if (close_tile)
          PAIR_TILE(NN, false, true);
        else
          PAIR_TILE(NN, false, false);
      } else if (close_tile) {
        PAIR_TILE(false, false, true);
      } else {
        PAIR_TILE(false, false, false);
      }
    }
#undef PAIR_TILE
    neumaier(hx, lx, px);
    neumaier(hy, ly, py);
    neumaier(hz, lz, pz);
    if (WANT_V) neumaier(hv, lv, pv);
  }
  if (active) {
    const size_t o = (size_t)split * 4 * n_t;
    part[o + i] = (double)hx + (double)lx;
    part[o + (size_t)n_t + i] = (double)hy + (double)ly;
    part[o + 2 * (size_t)n_t + i] = (double)hz + (double)lz;
    part[o + 3 * (size_t)n_t + i] = WANT_V ? (double)hv + (double)lv : 0.0;
    if (NN) {
      nn_d2p[(size_t)split * n_t + i] = best;
      nn_ip[(size_t)split * n_t + i] = bidx;
    }
  }
}

// ---------------------------------------------------------------------------
// Pairwise field with every unordered pair evaluated once (targets = sources)
// ---------------------------------------------------------------------------
// The softened pair term of eq. (nbody) is antisymmetric: what particle j adds
// to E_i, with q_j replaced by q_i and the sign reversed, is what i adds to
// E_j.  The particles (one order for targets and sources) form super-blocks of
// kSymTiles tiles of 256.  Tile pairs inside one super-block, tile pairs
// whose boxes are within the partner cut when that search is on, and tile
// pairs closer than the radius of their super-blocks (tile_pair_direct) stay
// with the directed kernel (k_pair_mixed with sym_tiles set).  Every other
// unordered tile pair is evaluated once, here, by the workgroup of its
// super-block pair: of the ns super-blocks, A owns (A, A + d mod ns) for
// d = 1 .. sym_h(A), so that each unordered pair has exactly one owner.
//
// A workgroup takes one (A, d): thread t holds the kSymTiles particles
// A kSymSB + k 256 + t of A (FP32, recentred on sym_origin, the centre of
// the more compact of A and B), B = A + d streams through LDS
// tile by tile.  Within a tile, a wave takes the sources in groups of 64 and
// 64 steps per group: at step m lane l pairs its particles with source
// (l + m) mod 64 of the group.  The sums for A's particles stay in
// registers; the running sum of each source travels with it through the
// wave (after each step a lane passes it to the lane below, which takes that
// source next, by a lane permutation), so after 64 steps every source's sum
// over the wave's 64 x kSymTiles particles sits in one lane, in a fixed
// order of additions, without atomics.  Two groups are processed with their
// steps interleaved, so that each permutation completes while the other
// group's step is computed (measured: 0.8 % faster than one group with the
// permuted sum needed at once, 1.4 % faster than one group adding it at the
// end of each step).  Per pair 14 VALU operations and one
// reciprocal square root (3 sub, 3 FMA for d^2 + s^2, rsqrt, 2 mul for r^-3,
// 3 + 3 FMA into the two sums, the source's straight into its running
// sum) serve two interactions.  Super-block pairs with one charge on each side take the charges out
// of the loop; the others (mixed charges, partial super-blocks) carry both
// charges per pair.  Tile pairs left to the directed kernel are masked
// through their softening term, without a branch.
// Outputs per launch slot dd = d - d0, FP32: Pi[dd][3][n], the field at A's
// particles from B, and Pj[dd][3][n], the field at B's particles from A;
// k_sym_reduce adds the slots to acc in order.
constexpr int kSymTiles = 8;
constexpr int kSymSB = kSymTiles * kThreads;  // particles per super-block
constexpr int kSymSlots = 80;                 // values of d per launch, at most

template <bool NN>
__global__ __launch_bounds__(kThreads, 4) void k_pair_sym(int n, const double *__restrict__ sx,
                                                        const double *__restrict__ sy,
                                                        const double *__restrict__ sz,
                                                        const double *__restrict__ sq,
                                                        const double *__restrict__ tbox, double nn_cut2d,
                                                        const double *__restrict__ sb, float soft2, int ns,
                                                        int d0, int dcnt, float *__restrict__ Pi,
                                                        float *__restrict__ Pj) {
  // each group of 64 sources twice in a row, so that step m of lane l reads
  // entry l + m without a wrap (constant offsets in the unrolled steps)
  __shared__ float4 S[kThreads / 64][128];
  __shared__ float J[kThreads / 64][3][kThreads];
  __shared__ unsigned long long skipS;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nxt = ((lane + 1) & 63) << 2;  // byte address of the next lane
  int A, dd;
  if (!sym_item(ns, dcnt, A, dd)) return;  // workgroup-uniform, before any barrier
  const int d = d0 + dd;
  if (d > sym_h(A, ns)) return;
  const int B = (A + d) % ns;
  const int a0 = A * kSymSB, b0 = B * kSymSB;
  const double *org = sym_origin(sb, A, B);
  const double c0 = org[0], c1 = org[1], c2 = org[2];
  float r0[kSymTiles], r1[kSymTiles], r2[kSymTiles], qa[kSymTiles];
  const float qA = (float)sq[a0], qB = (float)sq[b0];
  bool uni = true;
#pragma unroll
  for (int k = 0; k < kSymTiles; ++k) {
    const int i = a0 + k * kThreads + tid;
    const bool act = i < n;
    r0[k] = act ? (float)(sx[i] - c0) : 0.f;
    r1[k] = act ? (float)(sy[i] - c1) : 0.f;
    r2[k] = act ? (float)(sz[i] - c2) : 0.f;
    const float qi = act ? (float)sq[i] : 0.f;
    qa[k] = qi;
    const int j = b0 + k * kThreads + tid;
    uni = uni && act && qi == qA && j < n && (float)sq[j] == qB;
  }
  // tile pairs that belong to the directed kernel: bit 8 bt + k for (tile k
  // of A, tile bt of B)
  if (wv == 0) {
    bool near = false;
    const int ka = lane & 7, kb = lane >> 3;
    if (a0 + ka * kThreads < n && b0 + kb * kThreads < n)
      near = tile_pair_direct(tbox, sb, A * kSymTiles + ka, B * kSymTiles + kb, kSymTiles, NN, nn_cut2d);
    const unsigned long long m = __ballot(near);
    if (lane == 0) skipS = m;
  }
  // one charge on each side: charges out of the loop
  const bool U = __syncthreads_and(uni);
  const unsigned long long skip = skipS;
  float ex[kSymTiles], ey[kSymTiles], ez[kSymTiles];
#pragma unroll
  for (int k = 0; k < kSymTiles; ++k) ex[k] = ey[k] = ez[k] = 0.f;
  for (int bt = 0; bt < kSymTiles; ++bt) {
    const int jt = b0 + bt * kThreads;
    if (jt >= n) break;  // workgroup-uniform
    const int cnt = min(kThreads, n - jt);
    // tile pairs left to the directed kernel: a softening of 1e36 makes
    // r^-3 < 1e-54, which is 0 in FP32, so they add exactly nothing
    const unsigned sk = (unsigned)(skip >> (8 * bt)) & 0xffu;
    float s2k[kSymTiles];
#pragma unroll
    for (int k = 0; k < kSymTiles; ++k) s2k[k] = ((sk >> k) & 1u) ? 1e36f : soft2;
    __syncthreads();  // the previous tile's S and J are consumed
    {
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (tid < cnt) {
        const int j = jt + tid;
        v = make_float4((float)(sx[j] - c0), (float)(sy[j] - c1), (float)(sz[j] - c2), (float)sq[j]);
      }
      S[tid >> 6][tid & 63] = v;
      S[tid >> 6][(tid & 63) + 64] = v;
    }
    __syncthreads();
    // two groups of 64 sources at a time, their steps interleaved, so that
    // each lane permutation has the other group's step to complete in
    for (int g = 0; g < cnt; g += 128) {
      float tx = 0.f, ty = 0.f, tz = 0.f, ux = 0.f, uy = 0.f, uz = 0.f;
      const float4 *sa = &S[g >> 6][lane];
      const float4 *sb2 = &S[(g >> 6) + 1][lane];
      if (U) {
#pragma unroll 2
        for (int m = 0; m < 64; ++m) {
          {
            const float4 sj = sa[m];
            float cx = tx, cy = ty, cz = tz;
#pragma unroll
            for (int k = 0; k < kSymTiles; ++k) {
              const float dx = r0[k] - sj.x, dy = r1[k] - sj.y, dz = r2[k] - sj.z;
              const float rr = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, s2k[k])));
              const float ri = __builtin_amdgcn_rsqf(rr);
              const float w = ri * (ri * ri);
              ex[k] = fmaf(w, dx, ex[k]);
              ey[k] = fmaf(w, dy, ey[k]);
              ez[k] = fmaf(w, dz, ez[k]);
              cx = fmaf(w, dx, cx);
              cy = fmaf(w, dy, cy);
              cz = fmaf(w, dz, cz);
            }
            tx = __int_as_float(__builtin_amdgcn_ds_bpermute(nxt, __float_as_int(cx)));
            ty = __int_as_float(__builtin_amdgcn_ds_bpermute(nxt, __float_as_int(cy)));
            tz = __int_as_float(__builtin_amdgcn_ds_bpermute(nxt, __float_as_int(cz)));
          }
          {
            const float4 sj = sb2[m];
            float cx = ux, cy = uy, cz = uz;
#pragma unroll
            for (int k = 0; k < kSymTiles; ++k) {
              const float dx = r0[k] - sj.x, dy = r1[k] - sj.y, dz = r2[k] - sj.z;
              const float rr = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, s2k[k])));
              const float ri = __builtin_amdgcn_rsqf(rr);
              const float w = ri * (ri * ri);
              ex[k] = fmaf(w, dx, ex[k]);
              ey[k] = fmaf(w, dy, ey[k]);
              ez[k] = fmaf(w, dz, ez[k]);
              cx = fmaf(w, dx, cx);
              cy = fmaf(w, dy, cy);
              cz = fmaf(w, dz, cz);
            }
            ux = __int_as_float(__builtin_amdgcn_ds_bpermute(nxt, __float_as_int(cx)));
            uy = __int_as_float(__builtin_amdgcn_ds_bpermute(nxt, __float_as_int(cy)));
            uz = __int_as_float(__builtin_amdgcn_ds_bpermute(nxt, __float_as_int(cz)));
          }
        }
      } else {
#pragma unroll 2
        for (int m = 0; m < 64; ++m) {
          {
            const float4 sj = sa[m];
            float cx = tx, cy = ty, cz = tz;
#pragma unroll
            for (int k = 0; k < kSymTiles; ++k) {
              const float dx = r0[k] - sj.x, dy = r1[k] - sj.y, dz = r2[k] - sj.z;
              const float rr = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, s2k[k])));
              const float ri = __builtin_amdgcn_rsqf(rr);
              const float w = ri * (ri * ri);
              const float wi = w * sj.w, wj = w * qa[k];
              ex[k] = fmaf(wi, dx, ex[k]);
              ey[k] = fmaf(wi, dy, ey[k]);
              ez[k] = fmaf(wi, dz, ez[k]);
              cx = fmaf(wj, dx, cx);
              cy = fmaf(wj, dy, cy);
              cz = fmaf(wj, dz, cz);
            }
            tx = __int_as_float(__builtin_amdgcn_ds_bpermute(nxt, __float_as_int(cx)));
            ty = __int_as_float(__builtin_amdgcn_ds_bpermute(nxt, __float_as_int(cy)));
            tz = __int_as_float(__builtin_amdgcn_ds_bpermute(nxt, __float_as_int(cz)));
          }
          {
            const float4 sj = sb2[m];
            float cx = ux, cy = uy, cz = uz;
#pragma unroll
            for (int k = 0; k < kSymTiles; ++k) {
              const float dx = r0[k] - sj.x, dy = r1[k] - sj.y, dz = r2[k] - sj.z;
              const float rr = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, s2k[k])));
              const float ri = __builtin_amdgcn_rsqf(rr);
              const float w = ri * (ri * ri);
              const float wi = w * sj.w, wj = w * qa[k];
              ex[k] = fmaf(wi, dx, ex[k]);
              ey[k] = fmaf(wi, dy, ey[k]);
              ez[k] = fmaf(wi, dz, ez[k]);
              cx = fmaf(wj, dx, cx);
              cy = fmaf(wj, dy, cy);
              cz = fmaf(wj, dz, cz);
            }
            ux = __int_as_float(__builtin_amdgcn_ds_bpermute(nxt, __float_as_int(cx)));
            uy = __int_as_float(__builtin_amdgcn_ds_bpermute(nxt, __float_as_int(cy)));
            uz = __int_as_float(__builtin_amdgcn_ds_bpermute(nxt, __float_as_int(cz)));
          }
        }
      }
      const int jl = g + lane;
      J[wv][0][jl] = tx;
      J[wv][1][jl] = ty;
      J[wv][2][jl] = tz;
      J[wv][0][jl + 64] = ux;
      J[wv][1][jl + 64] = uy;
      J[wv][2][jl + 64] = uz;
    }
    __syncthreads();
    // field at the tile's sources from A: E_j = -sum_i q_i w (r_i - s_j),
    // the four waves' rows added in order
    if (tid < cnt) {
      const float fj = U ? -qA : -1.f;
      const size_t o = (size_t)dd * 3 * n + jt + tid;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float v = ((J[0][c][tid] + J[1][c][tid]) + J[2][c][tid]) + J[3][c][tid];
        Pj[o + (size_t)c * n] = fj * v;
      }
    }
  }
  const float fi = U ? qB : 1.f;
#pragma unroll
  for (int k = 0; k < kSymTiles; ++k) {
    const int i = a0 + k * kThreads + tid;
    if (i < n) {
      const size_t o = (size_t)dd * 3 * n + i;
      Pi[o] = fi * ex[k];
      Pi[o + (size_t)n] = fi * ey[k];
      Pi[o + 2 * (size_t)n] = fi * ez[k];
    }
  }
}

// acc[c][p] += the launch's slots that hold a field at p, in slot order: the
// slot of d as the owner of (A, A + d) and the slot of d as the partner of
// (A - d, A).
__global__ __launch_bounds__(256) void k_sym_reduce(int n, int sbsz, int ns, int d0, int dcnt,
                                                    const float *__restrict__ Pi, const float *__restrict__ Pj,
                                                    double *acc) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  const int A = p / sbsz;
  const int hA = sym_h(A, ns);
  // the three components side by side, so that six loads per slot are in
  // flight (each component keeps its order of additions)
  double s0 = acc[p], s1 = acc[(size_t)n + p], s2 = acc[2 * (size_t)n + p];
#pragma unroll 4
  for (int dd = 0; dd < dcnt; ++dd) {
    const int d = d0 + dd;
    const size_t o = (size_t)dd * 3 * n + p;
    if (d <= hA) {
      s0 += (double)Pi[o];
      s1 += (double)Pi[o + (size_t)n];
      s2 += (double)Pi[o + 2 * (size_t)n];
    }
    if (d <= sym_h((A - d + ns) % ns, ns)) {
      s0 += (double)Pj[o];
      s1 += (double)Pj[o + (size_t)n];
      s2 += (double)Pj[o + 2 * (size_t)n];
    }
  }
  acc[p] = s0;
  acc[(size_t)n + p] = s1;
  acc[2 * (size_t)n + p] = s2;
}

template <bool WANT_V, bool NN, int EXCL>
__global__ __launch_bounds__(kThreads) void k_pair_fp64(int n_t, const double *__restrict__ xs,
                                                        const int32_t *__restrict__ perm, int n_s,
                                                        const double *__restrict__ sx,
                                                        const double *__restrict__ sy,
                                                        const double *__restrict__ sz,
                                                        const double *__restrict__ sq,
                                                        const int8_t *__restrict__ species,
                                                        const int8_t *__restrict__ species_s, double soft2,
                                                        int chunk, double *part, double *nn_d2p,
                                                        int32_t *nn_ip, const int32_t *__restrict__ self_map) {
  __shared__ double4 S[kThreads];
  __shared__ int K[kThreads];
  const int tid = threadIdx.x;
  const int i = blockIdx.x * kThreads + tid;
  const bool active = i < n_t;
  const int ii = active ? i : 0;
  const double x0 = xs[ii], x1 = xs[(size_t)n_t + ii], x2 = xs[2 * (size_t)n_t + ii];
  int want = -2;
  if (NN && active) want = want_key(species[perm[i]]);
  const int self = active ? (self_map ? self_map[perm[i]] : perm[i]) : -1;
  const int jb = blockIdx.y * chunk;
  const int je = min(n_s, jb + chunk);
  double ex = 0.0, ey = 0.0, ez = 0.0, ev = 0.0;
  double best = INFINITY;
  int bidx = -1;
  for (int jt = jb; jt < je; jt += kThreads) {
    const int cnt = min(kThreads, je - jt);
    __syncthreads();
    if (tid < cnt) {
      const int j = jt + tid;
      S[tid] = make_double4(sx[j], sy[j], sz[j], sq[j]);
      if (NN) K[tid] = species_s[j];
    }
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      const double4 s = S[jj];
      const double dx = x0 - s.x, dy = x1 - s.y, dz = x2 - s.z;
      const double dd = fma(dx, dx, fma(dy, dy, dz * dz));
      const double rr = dd + soft2;
      double ri = 1.0 / sqrt(rr);
      if (EXCL == 1) ri = rr > 0.0 ? ri : 0.0;
      if (EXCL == 2) ri = (jt + jj == self) ? 0.0 : ri;
      const double qr = s.w * ri;
      const double w = qr * ri * ri;
      ex = fma(w, dx, ex);
      ey = fma(w, dy, ey);
      ez = fma(w, dz, ez);
      if (WANT_V) ev += qr;
      if (NN) {
        if (K[jj] == want && dd < best && (EXCL != 1 || rr > 0.0)) {
          best = dd;
          bidx = jt + jj;
        }
      }
    }
  }
  if (active) {
    const size_t o = (size_t)blockIdx.y * 4 * n_t;
    part[o + i] = ex;
    part[o + (size_t)n_t + i] = ey;
    part[o + 2 * (size_t)n_t + i] = ez;
    part[o + 3 * (size_t)n_t + i] = ev;
    if (NN) {
      nn_d2p[(size_t)blockIdx.y * n_t + i] = best;
      nn_ip[(size_t)blockIdx.y * n_t + i] = bidx;
    }
  }
}

// acc[c][i] = (has_base ? acc[c][i] : 0) + sum over chunks in order; nearest
// partner = smallest distance, ties to the earlier chunk (lower source index).
template <typename DT>
__global__ __launch_bounds__(256) void k_pair_reduce(int n_t, int nsplit, const double *__restrict__ part,
                                                     int has_base, double *acc, const DT *__restrict__ nn_d2p,
                                                     const int32_t *__restrict__ nn_ip, double *nn_d2,
                                                     int32_t *nn_idx) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_t) return;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double s = has_base ? acc[(size_t)c * n_t + i] : 0.0;
    for (int k = 0; k < nsplit; ++k) s += part[(size_t)k * 4 * n_t + (size_t)c * n_t + i];
    acc[(size_t)c * n_t + i] = s;
  }
  if (nn_idx) {
    DT best = INFINITY;
    int32_t bi = -1;
    for (int k = 0; k < nsplit; ++k) {
      DT d = nn_d2p[(size_t)k * n_t + i];
      if (d < best) {
        best = d;
        bi = nn_ip[(size_t)k * n_t + i];
      }
    }
    nn_d2[i] = (double)best;
    nn_idx[i] = bi;
  }
}

// Terms of the tile pairs kept by the directed kernel (mask bits weighted
// by the two tiles' particle counts), added to *work; profiling only.
__global__ __launch_bounds__(256) void k_mask_work(int ntile, int wpr, int n, const uint32_t *__restrict__ mask,
                                                   unsigned long long *work) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  unsigned long long w = 0;
  if (t < (size_t)ntile * wpr) {
    const int a = (int)(t / wpr), wd = (int)(t % wpr);
    const unsigned long long ca = (unsigned long long)min(kThreads, n - a * kThreads);
    uint32_t m = mask[t];
    while (m) {
      const int u = __builtin_ctz(m);
      m &= m - 1;
      const int b = wd * 32 + u;
      w += ca * (unsigned long long)min(kThreads, n - b * kThreads);
    }
  }
  if (w) atomicAdd(work, w);
}

template <bool WANT_V, bool NN, int CZ>
static void launch_pair_t(obem_ctx *ctx, dim3 grid, int n_t, const double *xs, const int32_t *perm, int n_s,
                          const double *sx, const double *sy, const double *sz, const double *sq,
                          const int8_t *sp, const int8_t *sps, double soft, obem_precision prec, int chunk,
                          double *part, void *nnd, int32_t *nni, const double *tbox, float nn_cut2,
                          const int32_t *self_map, int sym_tiles, double nn_cut2d, const uint32_t *dmask,
                          int dwpr) {
  if (prec == OBEM_MIXED)
    hipLaunchKernelGGL((k_pair_mixed<WANT_V, NN, CZ>), dim3(grid.x * grid.y), dim3(kThreads), 0, ctx->stream, n_t,
                       xs, perm, n_s,
                       sx, sy, sz, sq, sp, sps, (float)(soft * soft), chunk, part, (float *)nnd, nni, tbox, nn_cut2,
                       self_map, sym_tiles, nn_cut2d, dmask, dwpr);
  else
    hipLaunchKernelGGL((k_pair_fp64<WANT_V, NN, CZ>), grid, dim3(kThreads), 0, ctx->stream, n_t, xs, perm, n_s,
                       sx, sy, sz, sq, sp, sps, soft * soft, chunk, part, (double *)nnd, nni, self_map);
}

// Workgroups of k_pair_sym<nn> resident at once on the context's device.
static int sym_resident(obem_ctx *ctx, bool nn) {
  int &cache = nn ? ctx->sym_resident_nn : ctx->sym_resident;
  if (cache <= 0)
    cache = resident_workgroups(nn ? reinterpret_cast<const void *>(&k_pair_sym<true>)
                                   : reinterpret_cast<const void *>(&k_pair_sym<false>),
                                kThreads, ctx->device);
  return cache;
}

obem_status launch_pair_field(obem_ctx *ctx, int64_t n_src, const double *sx, const double *sy, const double *sz,
                              const double *sq, const TargetOrder &to, double soft, obem_precision prec,
                              bool tgt_is_src, bool want_v, const int8_t *species, const int8_t *species_s,
                              double *acc, int32_t *nn_idx, double *nn_d2, const double *tbox, double nn_cut,
                              const int32_t *self_map, bool once) {
  const int n_t = to.n;
  const int n_s = (int)n_src;
  if (n_t == 0 || n_s == 0) return OBEM_OK;
  if (once && !(tgt_is_src && n_s == n_t && tbox && pair_once_applies(n_t, prec, soft, want_v)))
    return fail(ctx, OBEM_EINVAL, "pair-once evaluation needs targets = sources in one order");
  const int bt = nblk(n_t);
  // about 128k workgroups (64 rounds of the 2048 resident ones), so that the
  // last workgroups to start are short and the chip drains quickly at the
  // end; chunks >= 512 sources
  int nsplit = (kSplitWorkgroups + bt - 1) / bt;
  nsplit = std::max(1, std::min(nsplit, (n_s + 511) / 512));
  nsplit = std::min(nsplit, 64);
  int chunk = (n_s + nsplit - 1) / nsplit;
  chunk = (chunk + kThreads - 1) / kThreads * kThreads;
  nsplit = (n_s + chunk - 1) / chunk;
  double *part = (double *)ws_get(ctx, WS_PART, sizeof(double) * 4 * (size_t)n_t * nsplit);
  const bool nn = nn_idx != nullptr;
  void *nnd = nullptr;
  int32_t *nni = nullptr;
  if (nn) {
    nnd = ws_get(ctx, WS_NN, sizeof(double) * (size_t)n_t * nsplit);
    nni = (int32_t *)ws_get(ctx, WS_MISC7, sizeof(int32_t) * (size_t)n_t * nsplit);
    if (!nnd || !nni) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  }
  if (!part) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  // soft == 0: drop zero-distance terms (the self term and coincident
  // points); soft > 0 with targets = sources: only the potential needs the
  // self term removed (its field term is exactly 0).
  int excl = 0;
  if (!(soft > 0.0))
    excl = 1;
  else if (tgt_is_src && want_v)
    excl = 2;
  dim3 grid(bt, nsplit);
  // cut with a margin for the FP32 box coordinates (a larger cut only costs time)
  const double nn_cut2d = tbox ? std::pow(nn_cut * (1.0 + 1e-4) + 1e-9, 2) : INFINITY;
  const float nn_cut2 = (float)nn_cut2d;
  const int sym_tiles = once ? kSymTiles : 0;
  const int ns = (n_t + kSymSB - 1) / kSymSB;
  double *sb = nullptr;
  uint32_t *dmask = nullptr;
  int dwpr = 0;
  if (once) {
    obem_status st = pair_once_setup(ctx, n_t, kSymTiles, tbox, nn, nn_cut2d, &sb, &dmask, &dwpr);
    if (st) return st;
    if (ctx->prof && ctx->work_dev) {
      const int ntile = nblk(n_t);
      const size_t nw = (size_t)ntile * dwpr;
      hipLaunchKernelGGL(k_mask_work, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, ctx->stream, ntile, dwpr,
                         n_t, dmask, ctx->work_dev);
      ctx->work_once_n2 += (int64_t)n_t * n_t;
    }
  } else if (ctx->prof) {
    ctx->work_directed += (int64_t)n_t * n_s;
  }
  {
  OBEM_PROF(ctx, "pair");
#define PAIR_CASE(V, N, Z)                                                                                   \
  if (want_v == V && nn == N && excl == Z)                                                                   \
    launch_pair_t<V, N, Z>(ctx, grid, n_t, to.xs, to.perm, n_s, sx, sy, sz, sq, species, species_s, soft, prec, \
                           chunk, part, nnd, nni, tbox, nn_cut2, self_map, sym_tiles, nn_cut2d, dmask, dwpr);
  PAIR_CASE(false, false, 0)
  PAIR_CASE(false, false, 1)
  PAIR_CASE(false, false, 2)
  PAIR_CASE(false, true, 0)
  PAIR_CASE(false, true, 1)
  PAIR_CASE(false, true, 2)
  PAIR_CASE(true, false, 0)
  PAIR_CASE(true, false, 1)
  PAIR_CASE(true, false, 2)
  PAIR_CASE(true, true, 0)
  PAIR_CASE(true, true, 1)
  PAIR_CASE(true, true, 2)
#undef PAIR_CASE
  }
  OBEM_HIP(ctx, hipGetLastError());
  // the accumulator already holds the cell field when the panel kernel ran
  {
    OBEM_PROF(ctx, "pair_reduce");
    if (prec == OBEM_MIXED)
      hipLaunchKernelGGL(k_pair_reduce<float>, dim3(nblk(n_t)), dim3(256), 0, ctx->stream, n_t, nsplit, part, 1,
                         acc, (const float *)nnd, nni, nn_d2, nn_idx);
    else
      hipLaunchKernelGGL(k_pair_reduce<double>, dim3(nblk(n_t)), dim3(256), 0, ctx->stream, n_t, nsplit, part, 1,
                         acc, (const double *)nnd, nni, nn_d2, nn_idx);
  }
  OBEM_HIP(ctx, hipGetLastError());
  if (once) {
    // the tile pairs between super-blocks, each evaluated once, in launches
    // of up to kSymSlots values of d (bounded partial buffers)
    const int hmax = ns / 2;
    if (hmax > 0) {
      OBEM_PROF(ctx, "pair_once");
      const float soft2 = (float)(soft * soft);
      obem_status st = run_pair_once(ctx, n_t, kSymSB, ns, sym_resident(ctx, nn), kSymSlots, acc,
                                     [&](int d0, int dcnt, float *pi, float *pj) {
                                       const dim3 g(sym_grid(ns, dcnt));
                                       if (nn)
                                         hipLaunchKernelGGL(k_pair_sym<true>, g, dim3(kThreads), 0, ctx->stream, n_t,
                                                            sx, sy, sz, sq, tbox, nn_cut2d, sb, soft2, ns, d0, dcnt,
                                                            pi, pj);
                                       else
                                         hipLaunchKernelGGL(k_pair_sym<false>, g, dim3(kThreads), 0, ctx->stream, n_t,
                                                            sx, sy, sz, sq, tbox, nn_cut2d, sb, soft2, ns, d0, dcnt,
                                                            pi, pj);
                                     });
      if (st) return st;
    }
  }
  return OBEM_OK;
}

// Up to 2^24 particles: the tile-pair mask takes at most 512 MB and the
// double-buffered partial slots 32 GB; larger sets keep the directed
// evaluation.
obem_status pair_once_setup(obem_ctx *ctx, int n, int sym_tiles, const double *tbox, bool nn, double cut2d,
                            double **sb, uint32_t **dmask, int *dwpr) {
  const int ns = (n + sym_tiles * kThreads - 1) / (sym_tiles * kThreads);
  const int ntile = nblk(n);
  *dwpr = (ntile + 31) / 32;
  *sb = (double *)ws_get(ctx, WS_SYMR, sizeof(double) * 4 * (size_t)ns);
  *dmask = (uint32_t *)ws_get(ctx, WS_SYMM, sizeof(uint32_t) * (size_t)ntile * *dwpr);
  if (!*sb || !*dmask) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  hipLaunchKernelGGL(k_sym_radius, dim3((ns + 255) / 256), dim3(256), 0, ctx->stream, n, ns, sym_tiles, tbox, *sb);
  const size_t nw = (size_t)ntile * *dwpr;
  hipLaunchKernelGGL(k_tile_mask, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, ctx->stream, ntile, *dwpr,
                     sym_tiles, nn ? 1 : 0, cut2d, tbox, *sb, *dmask);
  OBEM_HIP(ctx, hipGetLastError());
  return OBEM_OK;
}

obem_status run_pair_once(obem_ctx *ctx, int n, int sbsz, int ns, int resident, int max_slots, double *acc,
                          const std::function<void(int, int, float *, float *)> &launch) {
  const int hmax = ns / 2;
  if (hmax <= 0) return OBEM_OK;
  // with more than one launch the slots are double-buffered: launch L's
  // slots are added to acc on the second stream while launch L + 1
  // evaluates into the other half (the additions stay in launch order, on
  // one stream, so the result does not depend on the overlap)
  const bool dbl = launch_slots(ns, hmax, resident, max_slots) < hmax;
  const size_t half = 3 * (size_t)std::min(max_slots, hmax) * n;
  float *Pi = (float *)ws_get(ctx, WS_SYMI, sizeof(float) * half * (dbl ? 2 : 1));
  float *Pj = (float *)ws_get(ctx, WS_SYMJ, sizeof(float) * half * (dbl ? 2 : 1));
  if (!Pi || !Pj) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  if (dbl) {
    obem_status st = aux_stream(ctx);
    if (st) return st;
  }
  int launch_no = 0;
  for (int d0 = 1, dcnt = 0; d0 <= hmax; d0 += dcnt, ++launch_no) {
    // equal workgroups run in rounds: at 32 values of d and 1954
    // super-blocks the last round of a launch held 64 of 1024
    dcnt = launch_slots(ns, hmax - d0 + 1, resident, max_slots);
    const int b = dbl ? (launch_no & 1) : 0;
    float *pi = Pi + b * half, *pj = Pj + b * half;
    if (dbl && launch_no >= 2) OBEM_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_free[b], 0));
    launch(d0, dcnt, pi, pj);
    OBEM_HIP(ctx, hipGetLastError());
    hipStream_t rs = ctx->stream;
    if (dbl) {
      OBEM_HIP(ctx, hipEventRecord(ctx->ev_slots[b], ctx->stream));
      OBEM_HIP(ctx, hipStreamWaitEvent(ctx->aux, ctx->ev_slots[b], 0));
      rs = ctx->aux;
    }
    hipLaunchKernelGGL(k_sym_reduce, dim3(nblk(n)), dim3(256), 0, rs, n, sbsz, ns, d0, dcnt, pi, pj, acc);
    OBEM_HIP(ctx, hipGetLastError());
    if (dbl) OBEM_HIP(ctx, hipEventRecord(ctx->ev_free[b], ctx->aux));
  }
  if (dbl) {
    OBEM_HIP(ctx, hipEventRecord(ctx->ev_join, ctx->aux));
    OBEM_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0));
  }
  return OBEM_OK;
}

bool pair_once_applies(int64_t n, obem_precision prec, double soft, bool want_v) {
  return prec == OBEM_MIXED && soft > 0.0 && !want_v && n > 2 * (int64_t)kSymSB && n <= ((int64_t)1 << 24);
}

// ---------------------------------------------------------------------------
// Scatter back to caller order, scaling by k_e
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scatter(int n, const int32_t *__restrict__ perm, const double *__restrict__ acc,
                                                 double scale, double *Ex, double *Ey, double *Ez, double *V) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int j = perm[i];
  Ex[j] = scale * acc[i];
  Ey[j] = scale * acc[(size_t)n + i];
  Ez[j] = scale * acc[2 * (size_t)n + i];
  if (V) V[j] = scale * acc[3 * (size_t)n + i];
}

__global__ __launch_bounds__(256) void k_fill(size_t n, double *p, double v) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

obem_status launch_scatter(obem_ctx *ctx, const TargetOrder &to, const double *acc, double scale, double *Ex,
                           double *Ey, double *Ez, double *V) {
  if (to.n == 0) return OBEM_OK;
  OBEM_PROF(ctx, "scatter");
  hipLaunchKernelGGL(k_scatter, dim3(nblk(to.n)), dim3(256), 0, ctx->stream, to.n, to.perm, acc, scale, Ex, Ey,
                     Ez, V);
  OBEM_HIP(ctx, hipGetLastError());
  return OBEM_OK;
}

obem_status launch_fill(obem_ctx *ctx, double *p, size_t n, double v) {
  if (n == 0) return OBEM_OK;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, n, p, v);
  OBEM_HIP(ctx, hipGetLastError());
  return OBEM_OK;
}

}  // namespace obem
