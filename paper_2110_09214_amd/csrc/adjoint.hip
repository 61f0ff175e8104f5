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

namespace obem {

constexpr int kT = 256;
constexpr int kPTb = 64;
constexpr int kNGb = 3 + 21 + 9;

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
__device__ __forceinline__ void cell_grad_closed(const d3 P[3], d3 n, double twoarea, d3 w, d3 &gtw,
                                                 double &ie_w) {
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
    d3 t = P[e1] - P[e];
    const double L = norm3(t);
    t = t * (1.0 / L);
    const d3 m = cross3(t, n);
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
// Cell adjoint, mixed precision (regimes as in the forward kernel).
// gx: 3 x n_t (sorted order) position gradient in units of 1/k_e;
// gsp: partial dL/dsigma per (workgroup, cell), in units of 1/k_e.
// ---------------------------------------------------------------------------
struct BTile {
  float g[kNGb][kPTb];
  float w[4][kPTb];    // area * {w0, wa, wb, 1/3}
  float sg[kPTb];      // sigma
  float lim[2][kPTb];
  double red[4][kPTb];  // per-wave partial of w . IE
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

// contribution of one quadrature point (weight aw, relative offset e) to
// G^T w and w . IE (float)
__device__ __forceinline__ void qpt_grad(float aw, float ex, float ey, float ez, float wx, float wy, float wz,
                                         float &jx, float &jy, float &jz, float &u) {
  const float rr = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
  const float ri = __builtin_amdgcn_rsqf(rr);
  const float ri2 = ri * ri;
  const float a3 = aw * ri * ri2;
  const float dw = fmaf(ex, wx, fmaf(ey, wy, ez * wz));
  u = fmaf(a3, dw, u);
  const float t = 3.0f * a3 * ri2 * dw;
  jx = fmaf(a3, wx, fmaf(-t, ex, jx));
  jy = fmaf(a3, wy, fmaf(-t, ey, jy));
  jz = fmaf(a3, wz, fmaf(-t, ez, jz));
}

__global__ __launch_bounds__(kT) void k_panel_bwd_mixed(int n_t, const double *__restrict__ xs,
                                                        const double *__restrict__ ws, int N,
                                                        const double *__restrict__ f,
                                                        const double *__restrict__ sigma, int want_x, double *gx,
                                                        double *gsp) {
  __shared__ BTile T;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i0 = blockIdx.x * kT;
  const int i = i0 + tid;
  const bool active = i < n_t;
  const double c0 = xs[i0], c1 = xs[(size_t)n_t + i0], c2 = xs[2 * (size_t)n_t + i0];
  const double x0 = active ? xs[i] : c0, x1 = active ? xs[(size_t)n_t + i] : c1, x2 = active ? xs[2 * (size_t)n_t + i] : c2;
  const double w0d = active ? ws[i] : 0.0, w1d = active ? ws[(size_t)n_t + i] : 0.0,
               w2d = active ? ws[2 * (size_t)n_t + i] : 0.0;
  const float r0 = (float)(x0 - c0), r1 = (float)(x1 - c1), r2 = (float)(x2 - c2);
  const float wx = (float)w0d, wy = (float)w1d, wz = (float)w2d;
  float hx = 0, hy = 0, hz = 0, lx = 0, ly = 0, lz = 0;
  double nx = 0, ny = 0, nz = 0;
  for (int k0 = 0; k0 < N; k0 += kPTb) {
    const int cnt = min(kPTb, N - k0);
    __syncthreads();
    for (int idx = tid; idx < kNGb * kPTb; idx += kT) {
      const int fld = idx / kPTb, k = idx % kPTb;
      float v = 0.f;
      if (k < cnt) {
        const int src = (fld < 3) ? (MF_GX + fld) : (MF_Q7 + fld - 3);
        const int c = fld % 3;
        const double cc = (c == 0) ? c0 : (c == 1 ? c1 : c2);
        v = (float)(f[(size_t)src * N + k0 + k] - cc);
      }
      T.g[fld][k] = v;
    }
    if (tid < kPTb) {
      const int k = tid;
      if (k < cnt) {
        const double ar = f[(size_t)MF_AREA * N + k0 + k];
        const double D = f[(size_t)MF_DIAM * N + k0 + k];
        T.w[0][k] = (float)(ar * Rule7::w0);
        T.w[1][k] = (float)(ar * Rule7::wa);
        T.w[2][k] = (float)(ar * Rule7::wb);
        T.w[3][k] = (float)(ar * (1.0 / 3.0));
        T.sg[k] = (float)sigma[k0 + k];
        T.lim[0][k] = (float)(kNearMixed * kNearMixed * D * D);
        T.lim[1][k] = (float)(kFar3Mixed * kFar3Mixed * D * D);
      }
    }
    __syncthreads();
    float px = 0, py = 0, pz = 0;
    for (int k = 0; k < cnt; ++k) {
      const float dx = r0 - T.g[0][k], dy = r1 - T.g[1][k], dz = r2 - T.g[2][k];
      const float R2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
      const bool nearp = R2 < T.lim[0][k];
      float u = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
      double un = 0.0;
      const bool anyn = __any(nearp);
      if (anyn) {
        if (nearp && active) {
          const int kk = k0 + k;
          d3 P[3];
          P[0] = mk3(f[(size_t)MF_AX * N + kk] - x0, f[(size_t)MF_AY * N + kk] - x1, f[(size_t)MF_AZ * N + kk] - x2);
          P[1] = mk3(f[(size_t)MF_BX * N + kk] - x0, f[(size_t)MF_BY * N + kk] - x1, f[(size_t)MF_BZ * N + kk] - x2);
          P[2] = mk3(f[(size_t)MF_CX * N + kk] - x0, f[(size_t)MF_CY * N + kk] - x1, f[(size_t)MF_CZ * N + kk] - x2);
          const d3 nn = mk3(f[(size_t)MF_NX * N + kk], f[(size_t)MF_NY * N + kk], f[(size_t)MF_NZ * N + kk]);
          d3 g;
          double iw;
          cell_grad_closed(P, nn, 2.0 * f[(size_t)MF_AREA * N + kk], mk3(w0d, w1d, w2d), g, iw);
          const double sg = sigma[kk];
          nx = fma(sg, g.x, nx);
          ny = fma(sg, g.y, ny);
          nz = fma(sg, g.z, nz);
          un = iw;
        }
      }
      const bool need7 = (!nearp) && (R2 < T.lim[1][k]);
      if (__any(need7)) {
        if (!nearp) {
#pragma unroll
          for (int q = 0; q < 7; ++q) {
            const float aw = T.w[q == 0 ? 0 : (q < 4 ? 1 : 2)][k];
            qpt_grad(aw, r0 - T.g[3 + 3 * q][k], r1 - T.g[4 + 3 * q][k], r2 - T.g[5 + 3 * q][k], wx, wy, wz, jx, jy,
                     jz, u);
          }
        }
      } else if (!nearp) {
        const float aw = T.w[3][k];
#pragma unroll
        for (int q = 0; q < 3; ++q)
          qpt_grad(aw, r0 - T.g[24 + 3 * q][k], r1 - T.g[25 + 3 * q][k], r2 - T.g[26 + 3 * q][k], wx, wy, wz, jx, jy,
                   jz, u);
      }
      if (!active) u = 0.f;
      const float sg = T.sg[k];
      px = fmaf(sg, jx, px);
      py = fmaf(sg, jy, py);
      pz = fmaf(sg, jz, pz);
      // charge gradient: reduce w . IE over the wave (fixed tree), FP64 for near lanes
      double tot = (double)wave_sum(u);
      if (anyn) tot += wave_sum(un);
      if (lane == 0) T.red[wv][k] = tot;
    }
    neum(hx, lx, px);
    neum(hy, ly, py);
    neum(hz, lz, pz);
    __syncthreads();
    if (tid < cnt) {
      const int k = tid;
      const double s = T.red[0][k] + T.red[1][k] + T.red[2][k] + T.red[3][k];
      gsp[(size_t)blockIdx.x * N + k0 + k] = s;
    }
  }
  if (active && want_x) {
    gx[i] = ((double)hx + (double)lx) + nx;
    gx[(size_t)n_t + i] = ((double)hy + (double)ly) + ny;
    gx[2 * (size_t)n_t + i] = ((double)hz + (double)lz) + nz;
  }
}

// FP64 cell adjoint: closed form within 48 diameters, 7-point rule beyond.
__global__ __launch_bounds__(kT) void k_panel_bwd_fp64(int n_t, const double *__restrict__ xs,
                                                       const double *__restrict__ ws, int N,
                                                       const double *__restrict__ f,
                                                       const double *__restrict__ sigma, int want_x, double *gx,
                                                       double *gsp) {
  __shared__ double red[4][kPTb];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i = blockIdx.x * kT + tid;
  const bool active = i < n_t;
  const int ii = active ? i : 0;
  const double x0 = xs[ii], x1 = xs[(size_t)n_t + ii], x2 = xs[2 * (size_t)n_t + ii];
  const d3 w = active ? mk3(ws[i], ws[(size_t)n_t + i], ws[2 * (size_t)n_t + i]) : mk3(0, 0, 0);
  double gxx = 0, gyy = 0, gzz = 0;
  for (int k0 = 0; k0 < N; k0 += kPTb) {
    const int cnt = min(kPTb, N - k0);
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
          cell_grad_closed(P, nn, 2.0 * f[(size_t)MF_AREA * N + kk], w, g, u);
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
                                                         double *part) {
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
  const float qi = (TIS && active) ? (float)sq[self] : 0.f;
  const int jb = blockIdx.y * chunk, je = min(n_s, jb + chunk);
  float hx = 0, hy = 0, hz = 0, lx = 0, ly = 0, lz = 0;
  for (int jt = jb; jt < je; jt += kT) {
    const int cnt = min(kT, je - jt);
    __syncthreads();
    if (tid < cnt) {
      const int j = jt + tid;
      S[tid] = make_float4((float)(sx[j] - c0), (float)(sy[j] - c1), (float)(sz[j] - c2), (float)sq[j]);
      if (TIS) Wq[tid] = make_float4((float)gEx[j], (float)gEy[j], (float)gEz[j], 0.f);
    }
    __syncthreads();
    float px = 0, py = 0, pz = 0;
    for (int jj = 0; jj < cnt; ++jj) {
      const float4 s = S[jj];
      const float dx = r0 - s.x, dy = r1 - s.y, dz = r2 - s.z;
      const float rr = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, soft2)));
      float ri = __builtin_amdgcn_rsqf(rr);
      if (EXCL == 1) ri = rr > 0.f ? ri : 0.f;
      if (EXCL == 2) ri = (jt + jj == self) ? 0.f : ri;
      float ax = s.w * wx, ay = s.w * wy, az = s.w * wz;
      if (TIS) {
        const float4 wj = Wq[jj];
        ax = fmaf(-qi, wj.x, ax);
        ay = fmaf(-qi, wj.y, ay);
        az = fmaf(-qi, wj.z, az);
      }
      const float ri2 = ri * ri;
      const float ri3 = ri * ri2;
      const float da = fmaf(dx, ax, fmaf(dy, ay, dz * az));
      const float t = 3.0f * ri3 * ri2 * da;
      px = fmaf(ri3, ax, fmaf(-t, dx, px));
      py = fmaf(ri3, ay, fmaf(-t, dy, py));
      pz = fmaf(ri3, az, fmaf(-t, dz, pz));
    }
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
  int s = (2048 + nb_rows - 1) / nb_rows;
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
    hipGetLastError();
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

  TargetOrder to;
  obem_status st = order_targets(ctx, n_tgt, tx, ty, tz, &to);
  if (st) return st;
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
    if (precision == OBEM_MIXED)
      hipLaunchKernelGGL(k_panel_bwd_mixed, dim3(bt), dim3(kT), 0, ctx->stream, n_t, to.xs, wsrt, N, mesh->f, sigma,
                         1, gx, gsp);
    else
      hipLaunchKernelGGL(k_panel_bwd_fp64, dim3(bt), dim3(kT), 0, ctx->stream, n_t, to.xs, wsrt, N, mesh->f, sigma, 1,
                         gx, gsp);
    OBEM_HIP(ctx, hipGetLastError());
    have_gx = true;
    if (want_sig) {
      hipLaunchKernelGGL(k_sum_partials, dim3(nbk(N)), dim3(256), 0, ctx->stream, N, bt, gsp, kKe, g_sigma);
      OBEM_HIP(ctx, hipGetLastError());
    }
  }
  int excl = 0;
  if (!(soft > 0.0)) excl = 1;
  if (n_s > 0 && want_t) {
    int nsplit, chunk;
    split_for(bt, n_s, &nsplit, &chunk);
    double *part = (double *)ws_get(ctx, WS_PART, sizeof(double) * 3 * (size_t)n_t * nsplit);
    if (!part) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
    dim3 grid(bt, nsplit);
    OBEM_PROF(ctx, "pair_bwd");
#define BWD_T(TIS, EX)                                                                                            \
  if (tis == TIS && excl == EX) {                                                                                 \
    if (precision == OBEM_MIXED)                                                                                  \
      hipLaunchKernelGGL((k_pair_bwd_t_mixed<TIS, EX>), grid, dim3(kT), 0, ctx->stream, n_t, to.xs, to.perm, wsrt, \
                         n_s, sx, sy, sz, sq, gEx, gEy, gEz, (float)(soft * soft), chunk, part);                 \
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
