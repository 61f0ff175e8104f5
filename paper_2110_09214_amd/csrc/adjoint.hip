// Adjoint of the field evaluation for L = sum_t w_t . E(x_t) (not in the
// paper; it makes electrode voltages and dielectric charges optimisable).
//
//   dL/dsigma_k = k_e sum_t w_t . IE_k(x_t)                (transpose of eq. (BEM3))
//   dL/dx_t    += k_e sum_k sigma_k G_k(x_t)^T w_t,  G_k = dIE_k/dx
//   pairwise (K(d) = d/S^3, S^2 = |d|^2 + s^2, J = dK/dd = I/S^3 - 3 d d^T/S^5):
//     target role  g_t[i] += k_e sum_j q_j J(x_i - x_j) w_i
//     source role  g_s[j] += -k_e q_j sum_i J(x_i - x_j) w_i
//
// Nothing is kept from the forward call: source and cell tiles are recomputed.
// The cell kernel is target-major and fused: for each (target, cell) pair it
// forms both G^T w (position gradient) and w . IE (charge gradient), the
// latter reduced over the workgroup's 256 targets with a fixed wave/LDS tree
// and written as one partial per (workgroup, cell); a second kernel sums the
// partials in workgroup order.  No floating-point atomics anywhere.
#include <algorithm>
#include <cmath>

#include "cellmath.hpp"
#include "obem_internal.hpp"
#include "paironce.hpp"

namespace obem {

constexpr int kT = 256;
constexpr int kBwdTiles = 4;   // tiles per super-block of the pair-once adjoint
constexpr int kBwdSlots = 80;  // values of d per pair-once launch, at most
constexpr int kPTb = 64;

static inline int nbk(int64_t n) { return (int)((n + kT - 1) / kT); }

__device__ __forceinline__ void neum(float &s, float &c, float v) {
  float t = s + v;
  if (fabsf(s) >= fabsf(v))
    c += (s - t) + v;
  else
    c += (v - t) + s;
  s = t;
}

// FP64 closed-form Jacobian of a unit-density cell contracted with w:
//   gtw = G^T w = sum_e (m_e . w) grad f_e + (n . w) grad Omega
// and ie_w = w . IE.  P[k] = vertex k minus the target.
__device__ __forceinline__ void cell_grad_closed(const d3 P[3], d3 n, double twoarea, const CellEdges &E, d3 w,
                                                 d3 &gtw, double &ie_w) {
  double R[3] = {norm3(P[0]), norm3(P[1]), norm3(P[2])};
  double h = -dot3(P[0], n);
  double num = twoarea * h;
  double Om = 0.0;
  if (num != 0.0) {
    double den = R[0] * R[1] * R[2] + dot3(P[0], P[1]) * R[2] + dot3(P[0], P[2]) * R[1] + dot3(P[1], P[2]) * R[0];
    Om = 2.0 * atan2(num, den);
  }
  const double nw = dot3(n, w);
  ie_w = nw * Om;
  gtw = mk3(0, 0, 0);
  d3 gO = mk3(0, 0, 0);
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int e1 = (e + 1) % 3;
    const d3 t = E.t[e], m = E.m[e];
    const double L = E.L[e];
    double lm, R0sq;
    const double f = edge_log(P[e], R[e], R[e1], t, L, &lm, &R0sq);
    const double lp = lm + L;
    const double Rm = R[e], Rp = R[e1];
    // (l+/R+ - l-/R-)/R0^2 without cancellation near the edge line
    double Dd;
    if (lm >= 0.0)
      Dd = 1.0 / (Rm * (Rm + lm)) - 1.0 / (Rp * (Rp + lp));
    else if (lp <= 0.0)
      Dd = 1.0 / (Rp * (Rp - lp)) - 1.0 / (Rm * (Rm - lm));
    else
      Dd = (lp / Rp - lm / Rm) / R0sq;
    const double inv_diff = -L * (lp + lm) / ((Rp + Rm) * Rp * Rm);  // 1/R+ - 1/R-
    const d3 dvec = t * lm - P[e];                                     // target minus its foot on the edge line
    const d3 gf = dvec * (-Dd) + t * (-inv_diff);
    const double mw = dot3(m, w);
    ie_w += mw * f;
    gtw = gtw + gf * mw;
    gO = gO + cross3(t, dvec) * (-Dd);
  }
  gtw = gtw + gO * nw;
}

// ---------------------------------------------------------------------------
// Cell adjoint, mixed precision (regimes as in the forward kernels).  The far
// kernel takes the pairs beyond 3 D with the FP32 rules (7 points up to 6 D,
// 6 up to 16 D, 4 up to 40 D, 3 beyond); the near kernel then adds the pairs within 3 D
// (FP64 closed form), both deciding with the same FP32 test on the same
// recentred values.
// gx: 3 x n_t (sorted order) position gradient in units of 1/k_e;
// gsp: partial dL/dsigma per (workgroup, cell), in units of 1/k_e.
// ---------------------------------------------------------------------------
constexpr int kPB = 32;        // cells per LDS tile of the far kernel
constexpr int kUPad = kT + 4;  // row pitch of the w . IE buffer (floats)
constexpr int kParts = kT / kPB;
// the zone bounds as fractions of (40 D)^2: 7 points within 6 D, 6 within
// 16 D (the zones of the forward field)
constexpr float kR7 = (float)((kFwd6 / kFar3Mixed) * (kFwd6 / kFar3Mixed));
constexpr float kR6 = (float)((kFwd4 / kFar3Mixed) * (kFwd4 / kFar3Mixed));

// One cell of the far kernel's tile, recentred FP32, 18 float4 records:
//   c[0] = centroid, (3 D)^2          c[1] = (40 D)^2, area {w0, wa, wb}
//   floats 8..28 = the 7 rule points, 29 = area / 3, 30 = sigma,
//   31 = area w1 of the 6-point rule
//   floats 32..40 = the 3 rule points, 41 = area w2, 42..59 = the 6 rule points
//   floats 60..68 = the 3 outer points of the 4-point rule (its fourth is the
//   centroid; its weights are -27/16 and 25/16 of float 29), 69..71 = 0
struct BCell {
  float4 c[18];
};

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// One quadrature point of weight aw at offset e (target minus point), with
// a3 = aw / |e|^3:  u += a3 (e . w),  A += a3,  Z += a3 (e . w) e / |e|^2.
// Summed over the points, w . IE = u and G^T w = A w - 3 Z.
__device__ __forceinline__ void qpt_adj(float aw, float ex, float ey, float ez, float wx, float wy, float wz,
                                        float &u, float &A, float &Zx, float &Zy, float &Zz) {
  const float rr = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
  const float ri = __builtin_amdgcn_rsqf(rr);
  const float ri2 = ri * ri;
  const float a3 = (aw * ri) * ri2;
  const float v = a3 * fmaf(ex, wx, fmaf(ey, wy, ez * wz));
  u += v;
  A += a3;
  const float z = v * ri2;
  Zx = fmaf(z, ex, Zx);
  Zy = fmaf(z, ey, Zy);
  Zz = fmaf(z, ez, Zz);
}

// The M-point rule of one staged cell (M = 7, 6 or 3) at the recentred
// target r, accumulated into u, A and Z (qpt_adj).
template <int M>
__device__ __forceinline__ void bwd_rule(const BCell &C, float r0, float r1, float r2, float wx, float wy, float wz,
                                         float &u, float &A, float &Zx, float &Zy, float &Zz) {
  if (M == 7) {
    const float4 h = C.c[1];
    float q[24];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const float4 t = C.c[2 + m];
      q[4 * m] = t.x;
      q[4 * m + 1] = t.y;
      q[4 * m + 2] = t.z;
      q[4 * m + 3] = t.w;
    }
#pragma unroll
    for (int m = 0; m < 7; ++m)
      qpt_adj((m == 0) ? h.y : (m < 4 ? h.z : h.w), r0 - q[3 * m], r1 - q[3 * m + 1], r2 - q[3 * m + 2], wx, wy,
              wz, u, A, Zx, Zy, Zz);
  } else if (M == 6) {
    const float4 t10 = C.c[10];
    float q[18];
    q[0] = t10.z;
    q[1] = t10.w;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const float4 t = C.c[11 + m];
      q[2 + 4 * m] = t.x;
      q[3 + 4 * m] = t.y;
      q[4 + 4 * m] = t.z;
      q[5 + 4 * m] = t.w;
    }
    const float w1 = C.c[7].w, w2 = t10.y;
#pragma unroll
    for (int m = 0; m < 6; ++m)
      qpt_adj(m < 3 ? w1 : w2, r0 - q[3 * m], r1 - q[3 * m + 1], r2 - q[3 * m + 2], wx, wy, wz, u, A, Zx, Zy, Zz);
  } else if (M == 4) {
    const float aw = C.c[7].y;  // area / 3
    const float4 g = C.c[0];
    const float *rec = reinterpret_cast<const float *>(&C);
    float q[12];
    q[0] = g.x;
    q[1] = g.y;
    q[2] = g.z;
#pragma unroll
    for (int u = 0; u < 9; ++u) q[3 + u] = rec[60 + u];
#pragma unroll
    for (int m = 0; m < 4; ++m)
      qpt_adj(m == 0 ? aw * -1.6875f : aw * 1.5625f, r0 - q[3 * m], r1 - q[3 * m + 1], r2 - q[3 * m + 2], wx, wy,
              wz, u, A, Zx, Zy, Zz);
  } else {
    const float aw = C.c[7].y;  // area / 3
    float q[12];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const float4 t = C.c[8 + m];
      q[4 * m] = t.x;
      q[4 * m + 1] = t.y;
      q[4 * m + 2] = t.z;
      q[4 * m + 3] = t.w;
    }
#pragma unroll
    for (int m = 0; m < 3; ++m)
      qpt_adj(aw, r0 - q[3 * m], r1 - q[3 * m + 1], r2 - q[3 * m + 2], wx, wy, wz, u, A, Zx, Zy, Zz);
  }
}

// The per-cell sums of w . IE over the workgroup's 256 targets go through
// LDS: every thread stores its value for each cell of the tile, then 8
// threads per cell add 32 targets each (FP32, fixed order) and the 8
// partials are added in FP64 in fixed order.
// gridDim.y splits the cells into ranges of cchunk; split y writes its
// position gradient to gx + 3 n_t y (summed in split order afterwards).
__global__ __launch_bounds__(kT) void k_panel_bwd_mixed(int n_t, const double *__restrict__ xs,
                                                        const double *__restrict__ ws, int N,
                                                        const double *__restrict__ f,
                                                        const double *__restrict__ sigma, int want_x, int cchunk,
                                                        double *gx, double *gsp) {
  // the FP64 partials of the w . IE sums reuse the tile's memory: they are
  // written after the pair loop's last read of the tile and read before the
  // next tile is staged
  static_assert(sizeof(double) * kParts * kPB <= sizeof(BCell) * kPB, "partials exceed the tile");
  __shared__ __align__(16) float4 Traw[kPB * 18];
  __shared__ __align__(16) float U[kPB][kUPad];
  BCell *T = reinterpret_cast<BCell *>(Traw);
  double(*red)[kPB] = reinterpret_cast<double(*)[kPB]>(Traw);
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * kT;
  const int i = i0 + tid;
  const bool active = i < n_t;
  const double c0 = xs[i0], c1 = xs[(size_t)n_t + i0], c2 = xs[2 * (size_t)n_t + i0];
  const double x0 = active ? xs[i] : c0, x1 = active ? xs[(size_t)n_t + i] : c1,
               x2 = active ? xs[2 * (size_t)n_t + i] : c2;
  const float r0 = (float)(x0 - c0), r1 = (float)(x1 - c1), r2 = (float)(x2 - c2);
  // inactive lanes carry w = 0, so all their contributions vanish
  const float wx = active ? (float)ws[i] : 0.f, wy = active ? (float)ws[(size_t)n_t + i] : 0.f,
              wz = active ? (float)ws[2 * (size_t)n_t + i] : 0.f;
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
  float hx = 0, hy = 0, hz = 0, lx = 0, ly = 0, lz = 0;
  const int kb = blockIdx.y * cchunk, ke = min(N, kb + cchunk);
  for (int k0 = kb; k0 < ke; k0 += kPB) {
    const int cnt = min(kPB, ke - k0);
    __syncthreads();
    // staging, coalesced along the cells: the 57 rule coordinates (arrays
    // MF_Q7 + m) of the 32 cells.  Wave w takes row pairs p = w, w + 4, ...
    // (p < 30): lanes 0..31 row p, lanes 32..63 row p + 30 (for p < 27), lane
    // k & 31 on cell k & 31; both rows of a pair hold the same coordinate, so
    // the origin is the same for the whole wave, and the wave's loads are
    // all issued before the first is used.
    {
      const int k = tid & 31, h = (tid >> 5) & 1;
      const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
      const bool ok = k < cnt;
      const double *fk = f + (size_t)(MF_Q7 + 30 * h) * N + k0 + k;
      float *rec = reinterpret_cast<float *>(&T[k]);
      double v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int p = w + 4 * j;
        v[j] = (p < 30 && (h == 0 || p < 27) && ok) ? fk[(size_t)p * N] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int p = w + 4 * j;
        if (p < 30 && (h == 0 || p < 27)) {
          const int c = p % 3;
          const double o = c == 0 ? c0 : (c == 1 ? c1 : c2);
          rec[p + 30 * h + (h ? 12 : (p < 21 ? 8 : 11))] = ok ? (float)(v[j] - o) : 0.f;
        }
      }
    }
    if (tid < kPB) {
      const int k = tid;
      float4 g = make_float4(0.f, 0.f, 0.f, 0.f), h = g;
      float w3 = 0.f, sg = 0.f, w61 = 0.f, w62 = 0.f;
      if (k < cnt) {
        const int kk = k0 + k;
        const double D = f[(size_t)MF_DIAM * N + kk];
        const double ar = f[(size_t)MF_AREA * N + kk];
        g = make_float4((float)(f[(size_t)MF_GX * N + kk] - c0), (float)(f[(size_t)MF_GY * N + kk] - c1),
                        (float)(f[(size_t)MF_GZ * N + kk] - c2), (float)(kNearMixed * kNearMixed * D * D));
        h = make_float4((float)(kFar3Mixed * kFar3Mixed * D * D), (float)(ar * Rule7::w0), (float)(ar * Rule7::wa),
                        (float)(ar * Rule7::wb));
        w3 = (float)(ar * (1.0 / 3.0));
        sg = (float)sigma[kk];
        w61 = (float)(ar * Rule6::w1);
        w62 = (float)(ar * Rule6::w2);
      }
      float *rec = reinterpret_cast<float *>(&T[k]);
      T[k].c[0] = g;
      T[k].c[1] = h;
      rec[29] = w3;
      rec[30] = sg;
      rec[31] = w61;
      rec[41] = w62;
      rec[69] = rec[70] = rec[71] = 0.f;
    }
    __syncthreads();
    float px = 0.f, py = 0.f, pz = 0.f;
    // each cell's rule for the whole wave from one test of the cell (lane k
    // of the wave tests cell k) against the wave's sphere, as in the forward
    // kernel; only the cells some target may see within 3 D take the
    // per-lane test, which leaves the near pairs to k_panel_bwd_near
    uint64_t m3, m4, m6, m7, mnear;
    {
      const int k = tid & 63;
      float t = 3.0e38f, Dk = 0.f;
      if (k < cnt) {
        const float4 g = T[k].c[0];
        Dk = sqrtf(T[k].c[1].x) * (float)(1.0 / kFar3Mixed);
        t = sqrtf(dist2f(cw0, cw1, cw2, g.x, g.y, g.z)) - rw;
      }
      const uint64_t f4 = __ballot(t < (float)(kFar3Mixed * 1.01) * Dk);
      const uint64_t f6 = __ballot(t < (float)(kFwd4 * 1.01) * Dk);
      const uint64_t f7 = __ballot(t < (float)(kFwd6 * 1.01) * Dk);
      mnear = __ballot(t < (float)(kNearMixed * 1.01) * Dk);
      m3 = ((1ull << cnt) - 1ull) & ~f4;
      m4 = f4 & ~f6;
      m6 = f6 & ~f7;
      m7 = f7 & ~mnear;
    }
#define BWD_CELL_END                                   \
  {                                                    \
    const float sg = T[k].c[7].z;                      \
    const float sA = sg * A, s3 = -3.0f * sg;          \
    px = fmaf(sA, wx, fmaf(s3, Zx, px));               \
    py = fmaf(sA, wy, fmaf(s3, Zy, py));               \
    pz = fmaf(sA, wz, fmaf(s3, Zz, pz));               \
    U[k][tid] = u;                                     \
  }
    for (; m3; m3 &= m3 - 1ull) {
      const int k = __builtin_ctzll(m3);
      float u = 0.f, A = 0.f, Zx = 0.f, Zy = 0.f, Zz = 0.f;
      bwd_rule<3>(T[k], r0, r1, r2, wx, wy, wz, u, A, Zx, Zy, Zz);
      BWD_CELL_END
    }
    for (; m4; m4 &= m4 - 1ull) {
      const int k = __builtin_ctzll(m4);
      float u = 0.f, A = 0.f, Zx = 0.f, Zy = 0.f, Zz = 0.f;
      bwd_rule<4>(T[k], r0, r1, r2, wx, wy, wz, u, A, Zx, Zy, Zz);
      BWD_CELL_END
    }
    for (; m6; m6 &= m6 - 1ull) {
      const int k = __builtin_ctzll(m6);
      float u = 0.f, A = 0.f, Zx = 0.f, Zy = 0.f, Zz = 0.f;
      bwd_rule<6>(T[k], r0, r1, r2, wx, wy, wz, u, A, Zx, Zy, Zz);
      BWD_CELL_END
    }
    for (; m7; m7 &= m7 - 1ull) {
      const int k = __builtin_ctzll(m7);
      float u = 0.f, A = 0.f, Zx = 0.f, Zy = 0.f, Zz = 0.f;
      bwd_rule<7>(T[k], r0, r1, r2, wx, wy, wz, u, A, Zx, Zy, Zz);
      BWD_CELL_END
    }
    for (; mnear; mnear &= mnear - 1ull) {
      const int k = __builtin_ctzll(mnear);
      const float4 g = T[k].c[0];
      const float R2 = dist2f(r0, r1, r2, g.x, g.y, g.z);
      const bool nearp = R2 < g.w;  // taken by k_panel_bwd_near in FP64
      const float4 h = T[k].c[1];
      // 7 points within 6 D, 6 within 16 D, 4 within 40 D, 3 beyond (finest
      // rule of the wave)
      const bool need7 = (!nearp) && (R2 < h.x * kR7);
      const bool need6 = (!nearp) && (R2 < h.x * kR6);
      const bool need4 = (!nearp) && (R2 < h.x);
      float u = 0.f, A = 0.f, Zx = 0.f, Zy = 0.f, Zz = 0.f;
      if (__any(need7)) {
        if (!nearp) bwd_rule<7>(T[k], r0, r1, r2, wx, wy, wz, u, A, Zx, Zy, Zz);
      } else if (__any(need6)) {
        if (!nearp) bwd_rule<6>(T[k], r0, r1, r2, wx, wy, wz, u, A, Zx, Zy, Zz);
      } else if (__any(need4)) {
        if (!nearp) bwd_rule<4>(T[k], r0, r1, r2, wx, wy, wz, u, A, Zx, Zy, Zz);
      } else if (!nearp) {
        bwd_rule<3>(T[k], r0, r1, r2, wx, wy, wz, u, A, Zx, Zy, Zz);
      }
      BWD_CELL_END
    }
#undef BWD_CELL_END
    neum(hx, lx, px);
    neum(hy, ly, py);
    neum(hz, lz, pz);
    __syncthreads();
    {
      const int k = tid % kPB, part = tid / kPB;
      const float4 *row = reinterpret_cast<const float4 *>(&U[k][part * (kT / kParts)]);
      float4 a = row[0];
#pragma unroll
      for (int j = 1; j < kT / kParts / 4; ++j) {
        const float4 v = row[j];
        a.x += v.x;
        a.y += v.y;
        a.z += v.z;
        a.w += v.w;
      }
      red[part][k] = (double)((a.x + a.y) + (a.z + a.w));
    }
    __syncthreads();
    if (tid < cnt) {
      double s = red[0][tid];
#pragma unroll
      for (int p = 1; p < kParts; ++p) s += red[p][tid];
      gsp[(size_t)blockIdx.x * N + k0 + tid] = s;
    }
  }
  if (active && want_x) {
    double *g = gx + (size_t)blockIdx.y * 3 * n_t;
    g[i] = (double)hx + (double)lx;
    g[(size_t)n_t + i] = (double)hy + (double)ly;
    g[2 * (size_t)n_t + i] = (double)hz + (double)lz;
  }
}

// FP64 near zone of the mixed cell adjoint, added after the far kernel to
// its position-gradient slot of the same cell range (gridDim.y splits the
// cells as the far kernel does) and to gsp (same workgroups and cell ranges,
// so gsp[b][k] is read and written by one workgroup only).  The workgroup bounds its 256 targets by a sphere and
// visits the 64-cell tiles whose near-zone sphere (centre, max_k |c_k -
// centre| + 3 D_k) it meets, with a relative margin for the FP32 test.
__global__ __launch_bounds__(kT) void k_panel_bwd_near(int n_t, const double *__restrict__ xs,
                                                       const double *__restrict__ ws, int N,
                                                       const double *__restrict__ f,
                                                       const double *__restrict__ sigma,
                                                       const double *__restrict__ tiles, int want_x, int cchunk,
                                                       double *gxp, double *gsp) {
  __shared__ double box[4][6];
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i0 = blockIdx.x * kT;
  const int i = i0 + tid;
  const bool active = i < n_t;
  const double c0 = xs[i0], c1 = xs[(size_t)n_t + i0], c2 = xs[2 * (size_t)n_t + i0];
  const double x0 = active ? xs[i] : c0, x1 = active ? xs[(size_t)n_t + i] : c1,
               x2 = active ? xs[2 * (size_t)n_t + i] : c2;
  const float r0 = (float)(x0 - c0), r1 = (float)(x1 - c1), r2 = (float)(x2 - c2);
  const d3 w = active ? mk3(ws[i], ws[(size_t)n_t + i], ws[2 * (size_t)n_t + i]) : mk3(0, 0, 0);
  double b[6] = {x0, x1, x2, x0, x1, x2};
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      b[d] = fmin(b[d], __shfl_xor(b[d], o));
      b[3 + d] = fmax(b[3 + d], __shfl_xor(b[3 + d], o));
    }
  }
  if (lane == 0)
    for (int d = 0; d < 6; ++d) box[wv][d] = b[d];
  __syncthreads();
  double lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = fmin(fmin(box[0][d], box[1][d]), fmin(box[2][d], box[3][d]));
    hi[d] = fmax(fmax(box[0][3 + d], box[1][3 + d]), fmax(box[2][3 + d], box[3][3 + d]));
  }
  const double bc0 = 0.5 * (lo[0] + hi[0]), bc1 = 0.5 * (lo[1] + hi[1]), bc2 = 0.5 * (lo[2] + hi[2]);
  const double br = 0.5 * sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                               (hi[2] - lo[2]) * (hi[2] - lo[2]));
  // the same sphere in the recentred FP32 frame, radius measured from its
  // FP32 centre over the workgroup (widened by 1e-4 for the rounding)
  const float fb0 = (float)(bc0 - c0), fb1 = (float)(bc1 - c1), fb2 = (float)(bc2 - c2);
  float fbr = sqrtf(dist2f(r0, r1, r2, fb0, fb1, fb2));
  for (int o = 32; o > 0; o >>= 1) fbr = fmaxf(fbr, __shfl_xor(fbr, o));
  if (lane == 0) red[wv] = (double)fbr;
  __syncthreads();
  fbr = (float)fmax(fmax(red[0], red[1]), fmax(red[2], red[3])) * 1.0001f;
  __syncthreads();
  double nx = 0.0, ny = 0.0, nz = 0.0;
  // the cell range of split blockIdx.y (cchunk is a multiple of the tile)
  const int tb = blockIdx.y * cchunk / 64, te = (min(N, (blockIdx.y + 1) * cchunk) + 63) / 64;
  for (int t = tb; t < te; ++t) {
    const double dx = bc0 - tiles[4 * t], dy = bc1 - tiles[4 * t + 1], dz = bc2 - tiles[4 * t + 2];
    const double rs = (br + tiles[4 * t + 3]) * (1.0 + 1e-5);
    if (dx * dx + dy * dy + dz * dz > rs * rs) continue;  // workgroup-uniform
    const int k0 = t * 64, cnt = min(64, N - k0);
    // lane k of every wave holds cell k0 + k (centroid recentred to FP32 and
    // the near limit, as the far kernel stages them) and tests it against the
    // workgroup's sphere: the same values in every wave, so the mask of the
    // cells some target may see within 3 D (1 % wide) is workgroup-uniform
    float cg0 = 0.f, cg1 = 0.f, cg2 = 0.f, clim = 0.f, cdk = 0.f;
    if (lane < cnt) {
      const int kk = k0 + lane;
      cg0 = (float)(f[(size_t)MF_GX * N + kk] - c0);
      cg1 = (float)(f[(size_t)MF_GY * N + kk] - c1);
      cg2 = (float)(f[(size_t)MF_GZ * N + kk] - c2);
      const double D = f[(size_t)MF_DIAM * N + kk];
      clim = (float)(kNearMixed * kNearMixed * D * D);
      cdk = (float)D;
    }
    const float tw = sqrtf(dist2f(fb0, fb1, fb2, cg0, cg1, cg2)) - fbr;
    for (uint64_t m = __ballot(lane < cnt && tw < (float)(kNearMixed * 1.01) * cdk); m; m &= m - 1ull) {
      const int k = __builtin_ctzll(m);
      const int kk = k0 + k;
      const float g0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cg0), k));
      const float g1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cg1), k));
      const float g2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cg2), k));
      const float gl = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(clim), k));
      const bool nearp = active && dist2f(r0, r1, r2, g0, g1, g2) < gl;
      if (!__syncthreads_or(nearp)) continue;
      double un = 0.0;
      if (nearp) {
        d3 P[3];
        P[0] = mk3(f[(size_t)MF_AX * N + kk] - x0, f[(size_t)MF_AY * N + kk] - x1, f[(size_t)MF_AZ * N + kk] - x2);
        P[1] = mk3(f[(size_t)MF_BX * N + kk] - x0, f[(size_t)MF_BY * N + kk] - x1, f[(size_t)MF_BZ * N + kk] - x2);
        P[2] = mk3(f[(size_t)MF_CX * N + kk] - x0, f[(size_t)MF_CY * N + kk] - x1, f[(size_t)MF_CZ * N + kk] - x2);
        const d3 nn = mk3(f[(size_t)MF_NX * N + kk], f[(size_t)MF_NY * N + kk], f[(size_t)MF_NZ * N + kk]);
        d3 g;
        cell_grad_closed(P, nn, 2.0 * f[(size_t)MF_AREA * N + kk], cell_edges(f, N, kk), w, g, un);
        const double sg = sigma[kk];
        nx = fma(sg, g.x, nx);
        ny = fma(sg, g.y, ny);
        nz = fma(sg, g.z, nz);
      }
      const double s = wave_sum(un);
      if (lane == 0) red[wv] = s;
      __syncthreads();
      if (tid == 0) gsp[(size_t)blockIdx.x * N + kk] += ((red[0] + red[1]) + red[2]) + red[3];
      __syncthreads();
    }
  }
  if (active && want_x) {
    double *gx = gxp + (size_t)blockIdx.y * 3 * n_t;
    gx[i] += nx;
    gx[(size_t)n_t + i] += ny;
    gx[2 * (size_t)n_t + i] += nz;
  }
}

// FP64 cell adjoint: closed form within 48 diameters, 7-point rule beyond.
__global__ __launch_bounds__(kT) void k_panel_bwd_fp64(int n_t, const double *__restrict__ xs,
                                                       const double *__restrict__ ws, int N,
                                                       const double *__restrict__ f,
                                                       const double *__restrict__ sigma, int want_x, int cchunk,
                                                       double *gxp, double *gsp) {
  __shared__ double red[4][kPTb];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i = blockIdx.x * kT + tid;
  const bool active = i < n_t;
  const int ii = active ? i : 0;
  const double x0 = xs[ii], x1 = xs[(size_t)n_t + ii], x2 = xs[2 * (size_t)n_t + ii];
  const d3 w = active ? mk3(ws[i], ws[(size_t)n_t + i], ws[2 * (size_t)n_t + i]) : mk3(0, 0, 0);
  double gxx = 0, gyy = 0, gzz = 0;
  // the cell range of split blockIdx.y
  const int kb = blockIdx.y * cchunk, ke = min(N, kb + cchunk);
  for (int k0 = kb; k0 < ke; k0 += kPTb) {
    const int cnt = min(kPTb, ke - k0);
    for (int k = 0; k < cnt; ++k) {
      const int kk = k0 + k;
      const double dx = x0 - f[(size_t)MF_GX * N + kk], dy = x1 - f[(size_t)MF_GY * N + kk],
                   dz = x2 - f[(size_t)MF_GZ * N + kk];
      const double D = f[(size_t)MF_DIAM * N + kk];
      const bool quad = fma(dx, dx, fma(dy, dy, dz * dz)) >= kQuadFp64 * kQuadFp64 * D * D;
      d3 g = mk3(0, 0, 0);
      double u = 0.0;
      if (!__all(quad)) {
        if (!quad) {
          d3 P[3];
          P[0] = mk3(f[(size_t)MF_AX * N + kk] - x0, f[(size_t)MF_AY * N + kk] - x1, f[(size_t)MF_AZ * N + kk] - x2);
          P[1] = mk3(f[(size_t)MF_BX * N + kk] - x0, f[(size_t)MF_BY * N + kk] - x1, f[(size_t)MF_BZ * N + kk] - x2);
          P[2] = mk3(f[(size_t)MF_CX * N + kk] - x0, f[(size_t)MF_CY * N + kk] - x1, f[(size_t)MF_CZ * N + kk] - x2);
          const d3 nn = mk3(f[(size_t)MF_NX * N + kk], f[(size_t)MF_NY * N + kk], f[(size_t)MF_NZ * N + kk]);
          cell_grad_closed(P, nn, 2.0 * f[(size_t)MF_AREA * N + kk], cell_edges(f, N, kk), w, g, u);
        }
      }
      if (__any(quad)) {
        if (quad) {
          const double ar = f[(size_t)MF_AREA * N + kk];
#pragma unroll
          for (int q = 0; q < 7; ++q) {
            const double aw = ar * (q == 0 ? Rule7::w0 : (q < 4 ? Rule7::wa : Rule7::wb));
            const double ex = x0 - f[(size_t)(MF_Q7 + 3 * q) * N + kk];
            const double ey = x1 - f[(size_t)(MF_Q7 + 3 * q + 1) * N + kk];
            const double ez = x2 - f[(size_t)(MF_Q7 + 3 * q + 2) * N + kk];
            const double ri = 1.0 / sqrt(fma(ex, ex, fma(ey, ey, ez * ez)));
            const double ri2 = ri * ri;
            const double a3 = aw * ri * ri2;
            const double dw = ex * w.x + ey * w.y + ez * w.z;
            u = fma(a3, dw, u);
            const double t = 3.0 * a3 * ri2 * dw;
            g = g + mk3(a3 * w.x - t * ex, a3 * w.y - t * ey, a3 * w.z - t * ez);
          }
        }
      }
      const double sg = sigma[kk];
      gxx = fma(sg, g.x, gxx);
      gyy = fma(sg, g.y, gyy);
      gzz = fma(sg, g.z, gzz);
      if (!active) u = 0.0;
      const double us = wave_sum(u);
      if (lane == 0) red[wv][k] = us;
    }
    __syncthreads();
    if (tid < cnt) gsp[(size_t)blockIdx.x * N + k0 + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    __syncthreads();
  }
  if (active && want_x) {
    double *gx = gxp + (size_t)blockIdx.y * 3 * n_t;
    gx[i] = gxx;
    gx[(size_t)n_t + i] = gyy;
    gx[2 * (size_t)n_t + i] = gzz;
  }
}

// g_sigma[k] = scale * sum over workgroups (fixed order)
__global__ __launch_bounds__(256) void k_sum_partials(int N, int nb, const double *__restrict__ gsp, double scale,
                                                      double *out) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= N) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += gsp[(size_t)b * N + k];
  out[k] = scale * s;
}

// ---------------------------------------------------------------------------
// Pairwise adjoint, target-major: g_t[i] = sum_j J(x_i - x_j) a_ij with
// a_ij = q_j w_i (target role) - q_i w_j (source role, when the targets are
// the sources).  Partials per source chunk, summed in order by k_sum_chunks.
// ---------------------------------------------------------------------------
// One source tile of the target-side pairwise adjoint: with a = q_j w_i
// (minus q_i w_j when targets are the sources), p += J(d) a with
// J(d) = I/r^3 - 3 d d^T / r^5.  FOLDQ: q_j w_i = a0 for the whole tile.
template <bool TIS, int EXCL, bool FOLDQ>
__device__ __forceinline__ void pair_bwd_tile(const float4 *S, const float4 *Wq, int cnt, int jt, int self, float r0,
                                              float r1, float r2, float a0x, float a0y, float a0z, float wx, float wy,
                                              float wz, float qi, float soft2, float &px, float &py, float &pz) {
  for (int jj = 0; jj < cnt; ++jj) {
    const float4 s = S[jj];
    const float dx = r0 - s.x, dy = r1 - s.y, dz = r2 - s.z;
    const float rr = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, soft2)));
    float ri = __builtin_amdgcn_rsqf(rr);
    if (EXCL == 1) ri = rr > 0.f ? ri : 0.f;
    if (EXCL == 2) ri = (jt + jj == self) ? 0.f : ri;
    float ax = FOLDQ ? a0x : s.w * wx, ay = FOLDQ ? a0y : s.w * wy, az = FOLDQ ? a0z : s.w * wz;
    if (TIS) {
      const float4 wj = Wq[jj];
      ax = fmaf(-qi, wj.x, ax);
      ay = fmaf(-qi, wj.y, ay);
      az = fmaf(-qi, wj.z, az);
    }
    // J a = ri^3 (a - 3 ri^2 (d . a) d)
    const float ri2 = ri * ri;
    const float ri3 = ri * ri2;
    const float u = (3.0f * ri2) * fmaf(dx, ax, fmaf(dy, ay, dz * az));
    px = fmaf(ri3, fmaf(-u, dx, ax), px);
    py = fmaf(ri3, fmaf(-u, dy, ay), py);
    pz = fmaf(ri3, fmaf(-u, dz, az), pz);
  }
}

template <bool TIS, int EXCL>
__global__ __launch_bounds__(kT) void k_pair_bwd_t_mixed(int n_t, const double *__restrict__ xs,
                                                         const int32_t *__restrict__ perm,
                                                         const double *__restrict__ ws, int n_s,
                                                         const double *__restrict__ sx,
                                                         const double *__restrict__ sy,
                                                         const double *__restrict__ sz,
                                                         const double *__restrict__ sq,
                                                         const double *__restrict__ gEx,
                                                         const double *__restrict__ gEy,
                                                         const double *__restrict__ gEz, float soft2, int chunk,
                                                         double *part, const uint32_t *__restrict__ dmask,
                                                         int dwpr) {
  __shared__ float4 S[kT];
  __shared__ float4 Wq[kT];
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * kT;
  const int i = i0 + tid;
  const bool active = i < n_t;
  const double c0 = xs[i0], c1 = xs[(size_t)n_t + i0], c2 = xs[2 * (size_t)n_t + i0];
  const double x0 = active ? xs[i] : c0, x1 = active ? xs[(size_t)n_t + i] : c1, x2 = active ? xs[2 * (size_t)n_t + i] : c2;
  const float r0 = (float)(x0 - c0), r1 = (float)(x1 - c1), r2 = (float)(x2 - c2);
  const float wx = active ? (float)ws[i] : 0.f, wy = active ? (float)ws[(size_t)n_t + i] : 0.f,
              wz = active ? (float)ws[2 * (size_t)n_t + i] : 0.f;
  const int self = active ? perm[i] : -1;
  // with dmask the sources are the targets in the same order (pair-once
  // mode): the target's own charge is source i's, and only the tile pairs
  // the mask keeps are evaluated here
  const float qi = (TIS && active) ? (float)sq[dmask ? i : self] : 0.f;
  const int jb = blockIdx.y * chunk, je = min(n_s, jb + chunk);
  float hx = 0, hy = 0, hz = 0, lx = 0, ly = 0, lz = 0;
  for (int jt = jb; jt < je; jt += kT) {
    if (dmask && !((dmask[(size_t)blockIdx.x * dwpr + ((jt / kT) >> 5)] >> ((jt / kT) & 31)) & 1u)) continue;
    const int cnt = min(kT, je - jt);
    const float q0 = (float)sq[jt];
    __syncthreads();
    float qj = q0;
    if (tid < cnt) {
      const int j = jt + tid;
      qj = (float)sq[j];
      S[tid] = make_float4((float)(sx[j] - c0), (float)(sy[j] - c1), (float)(sz[j] - c2), qj);
      if (TIS) Wq[tid] = make_float4((float)gEx[j], (float)gEy[j], (float)gEz[j], 0.f);
    }
    // tiles of one charge (sources grouped by species): q_j w_i is the same
    // for the whole tile, 3 fewer VALU operations per pair
    const bool uniform = __syncthreads_and(qj == q0);
    float px = 0, py = 0, pz = 0;
    if (uniform)
      pair_bwd_tile<TIS, EXCL, true>(S, Wq, cnt, jt, self, r0, r1, r2, q0 * wx, q0 * wy, q0 * wz, wx, wy, wz, qi,
                                     soft2, px, py, pz);
    else
      pair_bwd_tile<TIS, EXCL, false>(S, Wq, cnt, jt, self, r0, r1, r2, 0.f, 0.f, 0.f, wx, wy, wz, qi, soft2, px, py,
                                      pz);
    neum(hx, lx, px);
    neum(hy, ly, py);
    neum(hz, lz, pz);
  }
  if (active) {
    const size_t o = (size_t)blockIdx.y * 3 * n_t;
    part[o + i] = (double)hx + (double)lx;
    part[o + (size_t)n_t + i] = (double)hy + (double)ly;
    part[o + 2 * (size_t)n_t + i] = (double)hz + (double)lz;
  }
}

// ---------------------------------------------------------------------------
// Pairwise adjoint with every unordered pair evaluated once (targets =
// sources, mixed, softened).  The term of the pair (i, j) in g_i is
// v = J(d) a with d = x_i - x_j and a = q_j w_i - q_i w_j; in g_j it is
// J(-d)(-a) = -v, since J is even in d.  Super-blocks, ownership, the lane
// rotation of the sources' sums and the partial slots are those of the
// field's pair-once kernel (k_pair_sym); tile pairs that the mask leaves to
// k_pair_bwd_t_mixed are masked here by a softening of 1e36 (r^-3 and r^-5
// underflow to 0).  Per pair 26 VALU operations and one reciprocal square
// root for two terms: 3 sub, 3 FMA (d^2 + s^2), rsqrt, 2 mul (r^-2, r^-3),
// 3 sub (a), 3 (d . a), 2 mul (3 r^-2 d . a), 3 FMA (a - u d), 3 + 3 FMA into
// the two sums.  Pi / Pj as in k_pair_sym (g in units of 1/k_e).
template <int T>
__global__ __launch_bounds__(kT, 4) void k_pair_bwd_sym(int n, const double *__restrict__ sx,
                                                      const double *__restrict__ sy,
                                                      const double *__restrict__ sz,
                                                      const double *__restrict__ sq,
                                                      const double *__restrict__ w, const double *__restrict__ sb,
                                                      const uint32_t *__restrict__ dmask, int dwpr, float soft2,
                                                      int ns, int d0, int dcnt, float *__restrict__ Pi,
                                                      float *__restrict__ Pj) {
  // positions and charges, and the weights (q_A w_j with one charge per
  // side, else w_j), each group of 64 sources twice in a row
  __shared__ float4 S[kT / 64][128];
  __shared__ float4 Wl[kT / 64][128];
  __shared__ float J[kT / 64][3][kT];
  __shared__ unsigned long long skipS;
  static_assert(T * T <= 64, "one mask bit per lane of a wave");
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nxt = ((lane + 1) & 63) << 2;
  int A, dd;
  if (!sym_item(ns, dcnt, A, dd)) return;  // workgroup-uniform, before any barrier
  const int d = d0 + dd;
  if (d > sym_h(A, ns)) return;
  const int B = (A + d) % ns;
  const int a0 = A * T * kT, b0 = B * T * kT;
  const double *org = sym_origin(sb, A, B);
  const double c0 = org[0], c1 = org[1], c2 = org[2];
  float r0[T], r1[T], r2[T], wx[T], wy[T], wz[T], qa[T];
  const float qA = (float)sq[a0], qB = (float)sq[b0];
  bool uni = true;
#pragma unroll
  for (int k = 0; k < T; ++k) {
    const int i = a0 + k * kT + tid;
    const bool act = i < n;
    r0[k] = act ? (float)(sx[i] - c0) : 0.f;
    r1[k] = act ? (float)(sy[i] - c1) : 0.f;
    r2[k] = act ? (float)(sz[i] - c2) : 0.f;
    wx[k] = act ? (float)w[i] : 0.f;
    wy[k] = act ? (float)w[(size_t)n + i] : 0.f;
    wz[k] = act ? (float)w[2 * (size_t)n + i] : 0.f;
    qa[k] = act ? (float)sq[i] : 0.f;
    const int j = b0 + k * kT + tid;
    uni = uni && act && qa[k] == qA && j < n && (float)sq[j] == qB;
  }
  if (wv == 0) {
    bool near = false;
    if (lane < T * T) {
      const int ka = lane % T, kb = lane / T;
      const int ta = A * T + ka, tb = B * T + kb;
      if (a0 + ka * kT < n && b0 + kb * kT < n) near = (dmask[(size_t)ta * dwpr + (tb >> 5)] >> (tb & 31)) & 1u;
    }
    const unsigned long long m = __ballot(near);
    if (lane == 0) skipS = m;
  }
  const bool U = __syncthreads_and(uni);
  const unsigned long long skip = skipS;
  if (U) {
    // a = q_B w_i - q_A w_j: the target part once per particle
#pragma unroll
    for (int k = 0; k < T; ++k) {
      wx[k] *= qB;
      wy[k] *= qB;
      wz[k] *= qB;
    }
  }
  float gx[T], gy[T], gz[T];
#pragma unroll
  for (int k = 0; k < T; ++k) gx[k] = gy[k] = gz[k] = 0.f;
  for (int bt = 0; bt < T; ++bt) {
    const int jt = b0 + bt * kT;
    if (jt >= n) break;  // workgroup-uniform
    const int cnt = min(kT, n - jt);
    const unsigned sk = (unsigned)(skip >> (T * bt)) & ((1u << T) - 1u);
    float s2k[T];
#pragma unroll
    for (int k = 0; k < T; ++k) s2k[k] = ((sk >> k) & 1u) ? 1e36f : soft2;
    __syncthreads();  // the previous tile's S, Wl and J are consumed
    {
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f), u = v;
      if (tid < cnt) {
        const int j = jt + tid;
        const float f = U ? qA : 1.f;
        v = make_float4((float)(sx[j] - c0), (float)(sy[j] - c1), (float)(sz[j] - c2), (float)sq[j]);
        u = make_float4(f * (float)w[j], f * (float)w[(size_t)n + j], f * (float)w[2 * (size_t)n + j], 0.f);
      }
      S[tid >> 6][tid & 63] = v;
      S[tid >> 6][(tid & 63) + 64] = v;
      Wl[tid >> 6][tid & 63] = u;
      Wl[tid >> 6][(tid & 63) + 64] = u;
    }
    __syncthreads();
    for (int g = 0; g < cnt; g += 64) {
      const float4 *sg = &S[g >> 6][lane];
      const float4 *wg = &Wl[g >> 6][lane];
      float tx = 0.f, ty = 0.f, tz = 0.f;
#pragma unroll 4
      for (int m = 0; m < 64; ++m) {
        const float4 sj = sg[m];
        const float4 wj = wg[m];
        float cx = 0.f, cy = 0.f, cz = 0.f;
#pragma unroll
        for (int k = 0; k < T; ++k) {
          const float dx = r0[k] - sj.x, dy = r1[k] - sj.y, dz = r2[k] - sj.z;
          const float rr = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, s2k[k])));
          const float ri = __builtin_amdgcn_rsqf(rr);
          const float ri2 = ri * ri;
          const float ri3 = ri * ri2;
          float ax, ay, az;
          if (U) {
            ax = wx[k] - wj.x;
            ay = wy[k] - wj.y;
            az = wz[k] - wj.z;
          } else {
            ax = fmaf(sj.w, wx[k], -qa[k] * wj.x);
            ay = fmaf(sj.w, wy[k], -qa[k] * wj.y);
            az = fmaf(sj.w, wz[k], -qa[k] * wj.z);
          }
          const float u = (3.0f * ri2) * fmaf(dx, ax, fmaf(dy, ay, dz * az));
          const float vx = fmaf(-u, dx, ax), vy = fmaf(-u, dy, ay), vz = fmaf(-u, dz, az);
          gx[k] = fmaf(ri3, vx, gx[k]);
          gy[k] = fmaf(ri3, vy, gy[k]);
          gz[k] = fmaf(ri3, vz, gz[k]);
          cx = fmaf(ri3, vx, cx);
          cy = fmaf(ri3, vy, cy);
          cz = fmaf(ri3, vz, cz);
        }
        tx = __int_as_float(__builtin_amdgcn_ds_bpermute(nxt, __float_as_int(tx + cx)));
        ty = __int_as_float(__builtin_amdgcn_ds_bpermute(nxt, __float_as_int(ty + cy)));
        tz = __int_as_float(__builtin_amdgcn_ds_bpermute(nxt, __float_as_int(tz + cz)));
      }
      J[wv][0][g + lane] = tx;
      J[wv][1][g + lane] = ty;
      J[wv][2][g + lane] = tz;
    }
    __syncthreads();
    // the sources' terms: -v, the four waves' rows added in order
    if (tid < cnt) {
      const size_t o = (size_t)dd * 3 * n + jt + tid;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float v = ((J[0][c][tid] + J[1][c][tid]) + J[2][c][tid]) + J[3][c][tid];
        Pj[o + (size_t)c * n] = -v;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < T; ++k) {
    const int i = a0 + k * kT + tid;
    if (i < n) {
      const size_t o = (size_t)dd * 3 * n + i;
      Pi[o] = gx[k];
      Pi[o + (size_t)n] = gy[k];
      Pi[o + 2 * (size_t)n] = gz[k];
    }
  }
}

template <bool TIS, int EXCL>
__global__ __launch_bounds__(kT) void k_pair_bwd_t_fp64(int n_t, const double *__restrict__ xs,
                                                        const int32_t *__restrict__ perm,
                                                        const double *__restrict__ ws, int n_s,
                                                        const double *__restrict__ sx,
                                                        const double *__restrict__ sy,
                                                        const double *__restrict__ sz,
                                                        const double *__restrict__ sq,
                                                        const double *__restrict__ gEx,
                                                        const double *__restrict__ gEy,
                                                        const double *__restrict__ gEz, double soft2, int chunk,
                                                        double *part) {
  __shared__ double4 S[kT];
  __shared__ double4 Wq[kT];
  const int tid = threadIdx.x;
  const int i = blockIdx.x * kT + tid;
  const bool active = i < n_t;
  const int ii = active ? i : 0;
  const double x0 = xs[ii], x1 = xs[(size_t)n_t + ii], x2 = xs[2 * (size_t)n_t + ii];
  const double wx = active ? ws[i] : 0.0, wy = active ? ws[(size_t)n_t + i] : 0.0,
               wz = active ? ws[2 * (size_t)n_t + i] : 0.0;
  const int self = active ? perm[i] : -1;
  const double qi = (TIS && active) ? sq[self] : 0.0;
  const int jb = blockIdx.y * chunk, je = min(n_s, jb + chunk);
  double gx = 0, gy = 0, gz = 0;
  for (int jt = jb; jt < je; jt += kT) {
    const int cnt = min(kT, je - jt);
    __syncthreads();
    if (tid < cnt) {
      const int j = jt + tid;
      S[tid] = make_double4(sx[j], sy[j], sz[j], sq[j]);
      if (TIS) Wq[tid] = make_double4(gEx[j], gEy[j], gEz[j], 0.0);
    }
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      const double4 s = S[jj];
      const double dx = x0 - s.x, dy = x1 - s.y, dz = x2 - s.z;
      const double rr = fma(dx, dx, fma(dy, dy, fma(dz, dz, soft2)));
      double ri = 1.0 / sqrt(rr);
      if (EXCL == 1) ri = rr > 0.0 ? ri : 0.0;
      if (EXCL == 2) ri = (jt + jj == self) ? 0.0 : ri;
      double ax = s.w * wx, ay = s.w * wy, az = s.w * wz;
      if (TIS) {
        const double4 wj = Wq[jj];
        ax = fma(-qi, wj.x, ax);
        ay = fma(-qi, wj.y, ay);
        az = fma(-qi, wj.z, az);
      }
      const double ri2 = ri * ri;
      const double ri3 = ri * ri2;
      const double da = fma(dx, ax, fma(dy, ay, dz * az));
      const double t = 3.0 * ri3 * ri2 * da;
      gx = fma(ri3, ax, fma(-t, dx, gx));
      gy = fma(ri3, ay, fma(-t, dy, gy));
      gz = fma(ri3, az, fma(-t, dz, gz));
    }
  }
  if (active) {
    const size_t o = (size_t)blockIdx.y * 3 * n_t;
    part[o + i] = gx;
    part[o + (size_t)n_t + i] = gy;
    part[o + 2 * (size_t)n_t + i] = gz;
  }
}

// Source role with separate targets, source-major:
//   g_s[j] = -q_j sum_i J(x_i - x_j) w_i   (targets in LDS, chunked over targets)
template <int EXCL, bool MIXED>
__global__ __launch_bounds__(kT) void k_pair_bwd_s(int n_s, const double *__restrict__ sx,
                                                   const double *__restrict__ sy, const double *__restrict__ sz,
                                                   const double *__restrict__ sq, int n_t,
                                                   const double *__restrict__ xs, const double *__restrict__ ws,
                                                   double soft2, int chunk, double *part) {
  __shared__ double4 X[kT];
  __shared__ double4 Wt[kT];
  const int tid = threadIdx.x;
  const int j0 = blockIdx.x * kT;
  const int j = j0 + tid;
  const bool active = j < n_s;
  const double c0 = sx[j0], c1 = sy[j0], c2 = sz[j0];
  const double y0 = active ? sx[j] : c0, y1 = active ? sy[j] : c1, y2 = active ? sz[j] : c2;
  const int ib = blockIdx.y * chunk, ie = min(n_t, ib + chunk);
  double gx = 0, gy = 0, gz = 0;
  for (int it = ib; it < ie; it += kT) {
    const int cnt = min(kT, ie - it);
    __syncthreads();
    if (tid < cnt) {
      const int i = it + tid;
      X[tid] = make_double4(xs[i] - c0, xs[(size_t)n_t + i] - c1, xs[2 * (size_t)n_t + i] - c2, 0.0);
      Wt[tid] = make_double4(ws[i], ws[(size_t)n_t + i], ws[2 * (size_t)n_t + i], 0.0);
    }
    __syncthreads();
    if (MIXED) {
      const float q0 = (float)(y0 - c0), q1 = (float)(y1 - c1), q2 = (float)(y2 - c2);
      float px = 0, py = 0, pz = 0;
      for (int ii = 0; ii < cnt; ++ii) {
        const double4 xv = X[ii];
        const double4 wv = Wt[ii];
        const float dx = (float)xv.x - q0, dy = (float)xv.y - q1, dz = (float)xv.z - q2;
        const float rr = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, (float)soft2)));
        float ri = __builtin_amdgcn_rsqf(rr);
        if (EXCL == 1) ri = rr > 0.f ? ri : 0.f;
        const float ri2 = ri * ri, ri3 = ri * ri2;
        const float wx = (float)wv.x, wy = (float)wv.y, wz = (float)wv.z;
        const float dw = fmaf(dx, wx, fmaf(dy, wy, dz * wz));
        const float t = 3.0f * ri3 * ri2 * dw;
        px = fmaf(ri3, wx, fmaf(-t, dx, px));
        py = fmaf(ri3, wy, fmaf(-t, dy, py));
        pz = fmaf(ri3, wz, fmaf(-t, dz, pz));
      }
      gx += px;
      gy += py;
      gz += pz;
    } else {
      const double q0 = y0 - c0, q1 = y1 - c1, q2 = y2 - c2;
      for (int ii = 0; ii < cnt; ++ii) {
        const double4 xv = X[ii];
        const double4 wv = Wt[ii];
        const double dx = xv.x - q0, dy = xv.y - q1, dz = xv.z - q2;
        const double rr = fma(dx, dx, fma(dy, dy, fma(dz, dz, soft2)));
        double ri = 1.0 / sqrt(rr);
        if (EXCL == 1) ri = rr > 0.0 ? ri : 0.0;
        const double ri2 = ri * ri, ri3 = ri * ri2;
        const double dw = fma(dx, wv.x, fma(dy, wv.y, dz * wv.z));
        const double t = 3.0 * ri3 * ri2 * dw;
        gx = fma(ri3, wv.x, fma(-t, dx, gx));
        gy = fma(ri3, wv.y, fma(-t, dy, gy));
        gz = fma(ri3, wv.z, fma(-t, dz, gz));
      }
    }
  }
  if (active) {
    const double qj = -sq[j];
    const size_t o = (size_t)blockIdx.y * 3 * n_s;
    part[o + j] = qj * gx;
    part[o + (size_t)n_s + j] = qj * gy;
    part[o + 2 * (size_t)n_s + j] = qj * gz;
  }
}

// out[c][i] = (base ? out[c][i] : 0) + sum over chunks (fixed order), c < 3
__global__ __launch_bounds__(256) void k_sum_chunks3(int n, int nch, const double *__restrict__ part, int base,
                                                     double *out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double s = base ? out[(size_t)c * n + i] : 0.0;
    for (int k = 0; k < nch; ++k) s += part[(size_t)k * 3 * n + (size_t)c * n + i];
    out[(size_t)c * n + i] = s;
  }
}

__global__ __launch_bounds__(256) void k_gather_w(int n, const int32_t *__restrict__ perm, const double *__restrict__ a,
                                                  const double *__restrict__ b, const double *__restrict__ c,
                                                  double *out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int j = perm[i];
  out[i] = a[j];
  out[(size_t)n + i] = b[j];
  out[2 * (size_t)n + i] = c[j];
}

__global__ __launch_bounds__(256) void k_scatter3(int n, const int32_t *__restrict__ perm, const double *__restrict__ acc,
                                                  double scale, double *X, double *Y, double *Z) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int j = perm ? perm[i] : i;
  X[j] = scale * acc[i];
  Y[j] = scale * acc[(size_t)n + i];
  Z[j] = scale * acc[2 * (size_t)n + i];
}

static void split_for(int nb_rows, int n_cols, int *nsplit, int *chunk) {
  int s = (kSplitWorkgroups + nb_rows - 1) / nb_rows;
  s = std::max(1, std::min(s, (n_cols + 1023) / 1024));
  s = std::min(s, 64);
  int c = (n_cols + s - 1) / s;
  c = (c + kT - 1) / kT * kT;
  *chunk = c;
  *nsplit = (n_cols + c - 1) / c;
}

}  // namespace obem

using namespace obem;

extern "C" obem_status field_eval_backward(obem_ctx *ctx, const obem_meshh *mesh, const double *sigma,
                                           int64_t n_src, const double *sx, const double *sy, const double *sz,
                                           const double *sq, int64_t n_tgt, const double *tx, const double *ty,
                                           const double *tz, double soft, obem_precision precision, unsigned flags,
                                           const double *gEx, const double *gEy, const double *gEz, double *g_sigma,
                                           double *g_tx, double *g_ty, double *g_tz, double *g_sx, double *g_sy,
                                           double *g_sz) {
  if (!ctx) return OBEM_EINVAL;
  if (ctx->sticky) return OBEM_ESTATE;
  if (hipSetDevice(ctx->device) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, OBEM_EDEVICE, "hipSetDevice failed");
  }
  const int64_t kMax = (int64_t)1 << 31;
  if (n_tgt < 0 || n_tgt >= kMax || n_src < 0 || n_src >= kMax) return fail(ctx, OBEM_EINVAL, "sizes out of range");
  if (!(soft >= 0.0) || !std::isfinite(soft)) return fail(ctx, OBEM_EINVAL, "soft must be finite and >= 0");
  if (precision != OBEM_FP64 && precision != OBEM_MIXED) return fail(ctx, OBEM_EINVAL, "bad precision");
  if (flags & ~(OBEM_TGT_IS_SRC | OBEM_WANT_V)) return fail(ctx, OBEM_EINVAL, "unknown flags");
  const bool tis = flags & OBEM_TGT_IS_SRC;
  if (tis && n_src != n_tgt) return fail(ctx, OBEM_EINVAL, "OBEM_TGT_IS_SRC needs n_src == n_tgt");
  const bool want_t = g_tx || g_ty || g_tz;
  if (want_t && !(g_tx && g_ty && g_tz)) return fail(ctx, OBEM_EINVAL, "g_tx/g_ty/g_tz: all or none");
  const bool want_s = !tis && (g_sx || g_sy || g_sz) && n_src > 0;
  if (want_s && !(g_sx && g_sy && g_sz)) return fail(ctx, OBEM_EINVAL, "g_sx/g_sy/g_sz: all or none");
  const bool want_sig = mesh && g_sigma;
  const void *req[] = {tx, ty, tz, gEx, gEy, gEz};
  if (n_tgt > 0)
    for (const void *p : req)
      if (!is_device_ptr(p)) return fail(ctx, OBEM_EINVAL, "target / gE arrays must be device memory");
  if (n_src > 0) {
    const void *sreq[] = {sx, sy, sz, sq};
    for (const void *p : sreq)
      if (!is_device_ptr(p)) return fail(ctx, OBEM_EINVAL, "source arrays must be device memory");
  }
  if (mesh && !is_device_ptr(sigma)) return fail(ctx, OBEM_EINVAL, "sigma must be device memory");
  const void *outs[] = {g_sigma, g_tx, g_ty, g_tz, g_sx, g_sy, g_sz};
  for (const void *p : outs)
    if (p && !is_device_ptr(p)) return fail(ctx, OBEM_EINVAL, "outputs must be device memory");
  if (want_sig && n_tgt == 0) {
    launch_fill(ctx, g_sigma, (size_t)mesh->n, 0.0);
  }
  if (want_s && n_tgt == 0) {
    launch_fill(ctx, g_sx, (size_t)n_src, 0.0);
    launch_fill(ctx, g_sy, (size_t)n_src, 0.0);
    launch_fill(ctx, g_sz, (size_t)n_src, 0.0);
  }
  if (n_tgt == 0) return OBEM_OK;

  int excl = 0;
  if (!(soft > 0.0)) excl = 1;
  // targets = sources: with the pair-once evaluation the targets take the
  // sources' order (charge sign, then Hilbert; same particles, same tiles)
  const bool once = tis && want_t && excl == 0 && pair_once_applies(n_tgt, precision, soft, false);
  SourceOrder so;
  TargetOrder to;
  obem_status st = OBEM_OK;
  if (once) {
    st = order_sources(ctx, n_src, sx, sy, sz, sq, false, &so);
    if (st) return st;
    to.n = (int32_t)n_tgt;
    to.perm = const_cast<int32_t *>(so.perm);
    to.xs = const_cast<double *>(so.x);
  } else {
    st = order_targets(ctx, n_tgt, tx, ty, tz, &to);
    if (st) return st;
  }
  const int n_t = (int)n_tgt, n_s = (int)n_src;
  double *wsrt = (double *)ws_get(ctx, WS_MISC1, sizeof(double) * 3 * (size_t)n_t);
  double *gx = (double *)ws_get(ctx, WS_ACC, sizeof(double) * 4 * (size_t)n_t);
  if (!wsrt || !gx) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  hipLaunchKernelGGL(k_gather_w, dim3(nbk(n_t)), dim3(256), 0, ctx->stream, n_t, to.perm, gEx, gEy, gEz, wsrt);
  bool have_gx = false;
  const int bt = nbk(n_t);
  if (mesh && (want_sig || want_t)) {
    const int N = (int)mesh->n;
    double *gsp = (double *)ws_get(ctx, WS_MISC2, sizeof(double) * (size_t)bt * N);
    if (!gsp) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed (%d x %d partials)", bt, N);
    OBEM_PROF(ctx, "panel_bwd");
    if (precision == OBEM_MIXED) {
      // cell ranges of >= 64 cells (whole 64-cell tiles of the near kernel),
      // about kSplitWorkgroups workgroups in all
      int ns = std::max(1, std::min((kSplitWorkgroups + bt - 1) / bt, (N + 63) / 64));
      ns = std::min(ns, 64);
      int cchunk = (N + ns - 1) / ns;
      cchunk = (cchunk + 63) / 64 * 64;
      ns = (N + cchunk - 1) / cchunk;
      double *gxp = gx;
      if (ns > 1) {
        gxp = (double *)ws_get(ctx, WS_PANEL, sizeof(double) * 3 * (size_t)n_t * ns);
        if (!gxp) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
      }
      hipLaunchKernelGGL(k_panel_bwd_mixed, dim3(bt, ns), dim3(kT), 0, ctx->stream, n_t, to.xs, wsrt, N, mesh->f,
                         sigma, 1, cchunk, gxp, gsp);
      // the near kernel of split y adds into the same slot (and into gsp for
      // the cells of its range), then the slots are added in split order
      hipLaunchKernelGGL(k_panel_bwd_near, dim3(bt, ns), dim3(kT), 0, ctx->stream, n_t, to.xs, wsrt, N, mesh->f,
                         sigma, mesh->tiles, 1, cchunk, gxp, gsp);
      if (ns > 1) hipLaunchKernelGGL(k_sum_chunks3, dim3(bt), dim3(256), 0, ctx->stream, n_t, ns, gxp, 0, gx);
    } else {
      // cell ranges as in the mixed path (whole tiles of kPTb cells)
      int ns = std::max(1, std::min((kSplitWorkgroups + bt - 1) / bt, (N + 63) / 64));
      ns = std::min(ns, 64);
      int cchunk = (N + ns - 1) / ns;
      cchunk = (cchunk + 63) / 64 * 64;
      ns = (N + cchunk - 1) / cchunk;
      double *gxp = gx;
      if (ns > 1) {
        gxp = (double *)ws_get(ctx, WS_PANEL, sizeof(double) * 3 * (size_t)n_t * ns);
        if (!gxp) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
      }
      hipLaunchKernelGGL(k_panel_bwd_fp64, dim3(bt, ns), dim3(kT), 0, ctx->stream, n_t, to.xs, wsrt, N, mesh->f,
                         sigma, 1, cchunk, gxp, gsp);
      if (ns > 1) hipLaunchKernelGGL(k_sum_chunks3, dim3(bt), dim3(256), 0, ctx->stream, n_t, ns, gxp, 0, gx);
    }
    OBEM_HIP(ctx, hipGetLastError());
    have_gx = true;
    if (want_sig) {
      hipLaunchKernelGGL(k_sum_partials, dim3(nbk(N)), dim3(256), 0, ctx->stream, N, bt, gsp, kKe, g_sigma);
      OBEM_HIP(ctx, hipGetLastError());
    }
  }
  if (n_s > 0 && want_t) {
    int nsplit, chunk;
    split_for(bt, n_s, &nsplit, &chunk);
    double *part = (double *)ws_get(ctx, WS_PART, sizeof(double) * 3 * (size_t)n_t * nsplit);
    if (!part) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
    dim3 grid(bt, nsplit);
    OBEM_PROF(ctx, "pair_bwd");
    double *sb = nullptr;
    uint32_t *dmask = nullptr;
    int dwpr = 0;
    if (once) {
      st = pair_once_setup(ctx, n_t, kBwdTiles, so.tbox, false, 0.0, &sb, &dmask, &dwpr);
      if (st) return st;
    }
    // sources: the caller's arrays, or the ordered copy (and the weights in
    // that order) under the pair-once evaluation
    const double *px = once ? so.x : sx, *py = once ? so.y : sy, *pz = once ? so.z : sz, *pq = once ? so.q : sq;
    const double *wjx = once ? wsrt : gEx, *wjy = once ? wsrt + n_t : gEy, *wjz = once ? wsrt + 2 * (size_t)n_t : gEz;
#define BWD_T(TIS, EX)                                                                                            \
  if (tis == TIS && excl == EX) {                                                                                 \
    if (precision == OBEM_MIXED)                                                                                  \
      hipLaunchKernelGGL((k_pair_bwd_t_mixed<TIS, EX>), grid, dim3(kT), 0, ctx->stream, n_t, to.xs, to.perm, wsrt, \
                         n_s, px, py, pz, pq, wjx, wjy, wjz, (float)(soft * soft), chunk, part, dmask, dwpr);    \
    else                                                                                                          \
      hipLaunchKernelGGL((k_pair_bwd_t_fp64<TIS, EX>), grid, dim3(kT), 0, ctx->stream, n_t, to.xs, to.perm, wsrt,  \
                         n_s, sx, sy, sz, sq, gEx, gEy, gEz, soft * soft, chunk, part);                          \
  }
    BWD_T(false, 0)
    BWD_T(false, 1)
    BWD_T(true, 0)
    BWD_T(true, 1)
#undef BWD_T
    OBEM_HIP(ctx, hipGetLastError());
    hipLaunchKernelGGL(k_sum_chunks3, dim3(bt), dim3(256), 0, ctx->stream, n_t, nsplit, part, have_gx ? 1 : 0, gx);
    OBEM_HIP(ctx, hipGetLastError());
    have_gx = true;
    if (once) {
      // the tile pairs between super-blocks, each evaluated once for both
      const int sbsz = kBwdTiles * kT;
      const int ns = (n_t + sbsz - 1) / sbsz;
      const int hmax = ns / 2;
      if (hmax > 0) {
        if (ctx->bwd_resident <= 0)
          ctx->bwd_resident = resident_workgroups(reinterpret_cast<const void *>(&k_pair_bwd_sym<kBwdTiles>), kT,
                                                  ctx->device);
        const float soft2 = (float)(soft * soft);
        st = run_pair_once(ctx, n_t, sbsz, ns, ctx->bwd_resident, kBwdSlots, gx,
                           [&](int d0, int dcnt, float *pi, float *pj) {
                             hipLaunchKernelGGL(k_pair_bwd_sym<kBwdTiles>, dim3(sym_grid(ns, dcnt)), dim3(kT), 0,
                                                ctx->stream, n_t, so.x, so.y, so.z, so.q, wsrt, sb, dmask, dwpr, soft2,
                                                ns, d0, dcnt, pi, pj);
                           });
        if (st) return st;
        OBEM_HIP(ctx, hipGetLastError());
      }
    }
  }
  if (want_t) {
    if (!have_gx) {
      st = launch_fill(ctx, gx, 3 * (size_t)n_t, 0.0);
      if (st) return st;
    }
    hipLaunchKernelGGL(k_scatter3, dim3(bt), dim3(256), 0, ctx->stream, n_t, to.perm, gx, kKe, g_tx, g_ty, g_tz);
    OBEM_HIP(ctx, hipGetLastError());
  }
  if (want_s) {
    const int bs = nbk(n_s);
    int nsplit, chunk;
    split_for(bs, n_t, &nsplit, &chunk);
    double *part = (double *)ws_get(ctx, WS_MISC3, sizeof(double) * 3 * (size_t)n_s * nsplit);
    double *acc = (double *)ws_get(ctx, WS_MISC4, sizeof(double) * 3 * (size_t)n_s);
    if (!part || !acc) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
    dim3 grid(bs, nsplit);
    OBEM_PROF(ctx, "pair_bwd");
    if (precision == OBEM_MIXED) {
      if (excl)
        hipLaunchKernelGGL((k_pair_bwd_s<1, true>), grid, dim3(kT), 0, ctx->stream, n_s, sx, sy, sz, sq, n_t, to.xs,
                           wsrt, soft * soft, chunk, part);
      else
        hipLaunchKernelGGL((k_pair_bwd_s<0, true>), grid, dim3(kT), 0, ctx->stream, n_s, sx, sy, sz, sq, n_t, to.xs,
                           wsrt, soft * soft, chunk, part);
    } else {
      if (excl)
        hipLaunchKernelGGL((k_pair_bwd_s<1, false>), grid, dim3(kT), 0, ctx->stream, n_s, sx, sy, sz, sq, n_t, to.xs,
                           wsrt, soft * soft, chunk, part);
      else
        hipLaunchKernelGGL((k_pair_bwd_s<0, false>), grid, dim3(kT), 0, ctx->stream, n_s, sx, sy, sz, sq, n_t, to.xs,
                           wsrt, soft * soft, chunk, part);
    }
    OBEM_HIP(ctx, hipGetLastError());
    hipLaunchKernelGGL(k_sum_chunks3, dim3(bs), dim3(256), 0, ctx->stream, n_s, nsplit, part, 0, acc);
    hipLaunchKernelGGL(k_scatter3, dim3(bs), dim3(256), 0, ctx->stream, n_s, nullptr, acc, kKe, g_sx, g_sy, g_sz);
    OBEM_HIP(ctx, hipGetLastError());
  }
  return OBEM_OK;
}
