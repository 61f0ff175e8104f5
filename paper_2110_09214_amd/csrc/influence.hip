// Influence of the point charges on the collocation equations (section
// 3.3.2, eqs. (potpart), (fldpart), (BEMpotpart), (BEMfldpart)): the charges'
// potential and field averaged over each cell,
//   Vbar_i = k_e/A_i sum_p q_p IV_i(x_p),   Ebar_i = -k_e/A_i sum_p q_p IE_i(x_p),
// change the left-hand side of the system before it is solved:
//   ed rows V_i - Vbar_i,   dd rows sigma_F,i - eps0 (eps_r2 - eps_r1) Ebar_i . n_i.
//
// It is the transpose of the cell field: one thread per cell, cells taken in
// the mesh's Hilbert order of centroids (a workgroup's cells are spatially
// close and are recentred on its first centroid), charges staged in LDS
// tiles, gridDim.y chunks of charges with per-chunk partial sums reduced in
// chunk order.  Precision regimes as in the field: mixed = FP32 7-point rule
// within 8 diameters, 6-point rule within 40, 3-point rule beyond (far
// kernel, charges ordered by
// charge sign, then Hilbert, so the charge comes out of the pair loop), FP64
// closed form within 3 diameters (near kernel, its own partial slots);
// FP64 = closed form within 48 diameters, FP64 7-point rule beyond.
#include <algorithm>
#include <cmath>

#include "cellmath.hpp"
#include "obem_internal.hpp"

namespace obem {

constexpr int kTI = 256;

// FP64 closed form of one cell at one charge: q IV and q IE.
__device__ __forceinline__ void infl_closed(const double *__restrict__ f, int N, int k, double px, double py,
                                            double pz, double q, double &sv, double &ex, double &ey, double &ez) {
  d3 P[3];
  P[0] = mk3(f[(size_t)MF_AX * N + k] - px, f[(size_t)MF_AY * N + k] - py, f[(size_t)MF_AZ * N + k] - pz);
  P[1] = mk3(f[(size_t)MF_BX * N + k] - px, f[(size_t)MF_BY * N + k] - py, f[(size_t)MF_BZ * N + k] - pz);
  P[2] = mk3(f[(size_t)MF_CX * N + k] - px, f[(size_t)MF_CY * N + k] - py, f[(size_t)MF_CZ * N + k] - pz);
  const d3 n = mk3(f[(size_t)MF_NX * N + k], f[(size_t)MF_NY * N + k], f[(size_t)MF_NZ * N + k]);
  d3 IE;
  double IV;
  cell_closed_form<true>(P, n, 2.0 * f[(size_t)MF_AREA * N + k], cell_edges(f, N, k), IE, IV);
  sv = fma(q, IV, sv);
  ex = fma(q, IE.x, ex);
  ey = fma(q, IE.y, ey);
  ez = fma(q, IE.z, ez);
}

// Far part of the mixed influence, charge-major: a workgroup owns 8 cells
// (consecutive in the mesh's Hilbert order) and streams its chunk of the
// charges in blocks of 1024, 4 per thread (one from each 256-charge tile of
// the block, so a wave's lanes hold 64 consecutive, spatially close charges).
// Per cell the rule is chosen per wave over those close charges (7 points
// within 8 D, 6 within 40 D, 3 beyond; pairs within 3 D are left to the near
// kernel), and
// each thread adds q (IV, IE) of its charges into 8 x 4 FP32 sums.  The sums
// of a block are reduced over the 256 threads through LDS in fixed order and
// in FP64 (8 partial sums of 32 threads each, then the 8 in order) and
// accumulated in FP64 by 32 threads, one per (cell, component).
constexpr int kCB = 8;   // cells per workgroup
constexpr int kCS = 4;   // charges per thread and block
constexpr int kUP = kTI + 4;

// One cell of the far kernel's LDS tile, recentred FP32, 19 float4 records:
//   c[0] = centroid, (3 D)^2          c[1] = (40 D)^2, area {w0, wa, wb}
//   c[2..7] = the 7 rule points (21 floats), area / 3, (6 D)^2, 0
//   c[8..10] = the 3 rule points (9 floats), area {w1, w2} of the 6-point
//              rule, (16 D)^2
//   c[11..15] = the 6 rule points (18 floats), area {wc, wp} of the 4-point
//              rule
//   c[16..18] = the 3 outer points of the 4-point rule (9 floats; its fourth
//              is the centroid), 0, 0, 0
// (the zones of the forward field: 7 points within 6 D, 6 within 16 D, 4
// within 40 D, 3 beyond)
struct ICell {
  float4 c[19];
};

// sum over m of w_m {1/|e_m|, e_m/|e_m|^3}, e_m = p - point m
template <int M>
__device__ __forceinline__ void infl_points(float px, float py, float pz, const float *q, const float *w, float &sv,
                                            float &ex, float &ey, float &ez) {
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const float ax = px - q[3 * m], ay = py - q[3 * m + 1], az = pz - q[3 * m + 2];
    const float rr = fmaf(ax, ax, fmaf(ay, ay, az * az));
    const float ri = __builtin_amdgcn_rsqf(rr);
    const float wr = w[m] * ri;
    const float t = wr * (ri * ri);
    sv += wr;
    ex = fmaf(t, ax, ex);
    ey = fmaf(t, ay, ey);
    ez = fmaf(t, az, ez);
  }
}

__global__ __launch_bounds__(kTI) void k_influence_mixed(int N, const double *__restrict__ f,
                                                         const int32_t *__restrict__ ord, int n_s,
                                                         const double *__restrict__ sx,
                                                         const double *__restrict__ sy,
                                                         const double *__restrict__ sz,
                                                         const double *__restrict__ sq, int chunk, double *part) {
  __shared__ ICell T[kCB];
  __shared__ __align__(16) float U[kCB * 4][kUP];
  __shared__ double red[kTI / (kCB * 4)][kCB * 4];
  const int tid = threadIdx.x;
  const int kb = blockIdx.x * kCB;  // first sorted position of the workgroup's cells
  // recentred on the first cell of the 256-cell group, as the near kernel
  const int kr = ord[(kb / kTI) * kTI];
  const double c0 = f[(size_t)MF_GX * N + kr], c1 = f[(size_t)MF_GY * N + kr], c2 = f[(size_t)MF_GZ * N + kr];
  for (int idx = tid; idx < 57 * kCB; idx += kTI) {
    const int m = idx / kCB, k = idx % kCB;
    const int kk = ord[min(kb + k, N - 1)];
    const int src = (m < 21) ? MF_Q7 + m : (m < 30 ? MF_Q3 + (m - 21) : (m < 48 ? MF_Q6 + (m - 30) : MF_Q4 + (m - 48)));
    const int c = (m < 21 ? m : (m < 30 ? m - 21 : (m < 48 ? m - 30 : m - 48))) % 3;
    reinterpret_cast<float *>(&T[k])[m < 21 ? 8 + m : (m < 30 ? 32 + (m - 21) : (m < 48 ? 44 + (m - 30) : 64 + (m - 48)))] =
        (float)(f[(size_t)src * N + kk] - (c == 0 ? c0 : (c == 1 ? c1 : c2)));
  }
  if (tid < kCB) {
    const int kk = ord[min(kb + tid, N - 1)];
    const double D = f[(size_t)MF_DIAM * N + kk], ar = f[(size_t)MF_AREA * N + kk];
    float *rec = reinterpret_cast<float *>(&T[tid]);
    T[tid].c[0] = make_float4((float)(f[(size_t)MF_GX * N + kk] - c0), (float)(f[(size_t)MF_GY * N + kk] - c1),
                              (float)(f[(size_t)MF_GZ * N + kk] - c2), (float)(kNearMixed * kNearMixed * D * D));
    T[tid].c[1] = make_float4((float)(kFar3Mixed * kFar3Mixed * D * D), (float)(ar * Rule7::w0),
                              (float)(ar * Rule7::wa), (float)(ar * Rule7::wb));
    rec[29] = (float)(ar / 3.0);
    rec[30] = (float)(kFwd6 * kFwd6 * D * D);
    rec[31] = 0.f;
    rec[41] = (float)(ar * Rule6::w1);
    rec[42] = (float)(ar * Rule6::w2);
    rec[43] = (float)(kFwd4 * kFwd4 * D * D);
    rec[62] = (float)(ar * Rule4::wc);
    rec[63] = (float)(ar * Rule4::wp);
    rec[73] = rec[74] = rec[75] = 0.f;
  }
  __syncthreads();
  double accd = 0.0;  // threads 0..31: (cell tid / 4, component tid % 4)
  const int jb = blockIdx.y * chunk, je = min(n_s, jb + chunk);
  for (int j0 = jb; j0 < je; j0 += kTI * kCS) {
    float px[kCS], py[kCS], pz[kCS], pq[kCS];
#pragma unroll
    for (int c = 0; c < kCS; ++c) {
      const int j = j0 + c * kTI + tid;
      const bool ok = j < je;
      const int jj = ok ? j : jb;  // a real position with charge 0
      px[c] = (float)(sx[jj] - c0);
      py[c] = (float)(sy[jj] - c1);
      pz[c] = (float)(sz[jj] - c2);
      pq[c] = ok ? (float)sq[jj] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < kCB; ++k) {
      const float4 g = T[k].c[0], h = T[k].c[1], h7 = T[k].c[7];
      float av = 0.f, ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll
      for (int c = 0; c < kCS; ++c) {
        const float R2 = dist2f(px[c], py[c], pz[c], g.x, g.y, g.z);
        const bool nearp = R2 < g.w;  // taken by k_influence_near in FP64
        // 7 points within 6 D, 6 within 16 D, 4 within 40 D, 3 beyond (finest
        // rule of the wave)
        const float lim6 = reinterpret_cast<const float *>(&T[k])[43];
        const bool need7 = !nearp && R2 < h7.z;
        const bool need6 = !nearp && R2 < lim6;
        const bool need4 = !nearp && R2 < h.x;
        float sv = 0.f, ex = 0.f, ey = 0.f, ez = 0.f;
        if (__any(need7)) {
          if (!nearp) {
            float q[21];
#pragma unroll
            for (int u = 0; u < 21; ++u) q[u] = reinterpret_cast<const float *>(&T[k])[8 + u];
            const float w[7] = {h.y, h.z, h.z, h.z, h.w, h.w, h.w};
            infl_points<7>(px[c], py[c], pz[c], q, w, sv, ex, ey, ez);
          }
        } else if (__any(need4) && !__any(need6)) {
          if (!nearp) {
            const float *rec = reinterpret_cast<const float *>(&T[k]);
            float q[12];
            q[0] = g.x;
            q[1] = g.y;
            q[2] = g.z;
#pragma unroll
            for (int u = 0; u < 9; ++u) q[3 + u] = rec[64 + u];
            const float w[4] = {rec[62], rec[63], rec[63], rec[63]};
            infl_points<4>(px[c], py[c], pz[c], q, w, sv, ex, ey, ez);
          }
        } else if (__any(need6)) {
          if (!nearp) {
            float q[18];
#pragma unroll
            for (int u = 0; u < 18; ++u) q[u] = reinterpret_cast<const float *>(&T[k])[44 + u];
            const float4 h10 = T[k].c[10];
            const float w[6] = {h10.y, h10.y, h10.y, h10.z, h10.z, h10.z};
            infl_points<6>(px[c], py[c], pz[c], q, w, sv, ex, ey, ez);
          }
        } else if (!nearp) {
          float q[9];
#pragma unroll
          for (int u = 0; u < 9; ++u) q[u] = reinterpret_cast<const float *>(&T[k])[32 + u];
          const float w3 = h7.y;
          const float w[3] = {w3, w3, w3};
          infl_points<3>(px[c], py[c], pz[c], q, w, sv, ex, ey, ez);
        }
        av = fmaf(pq[c], sv, av);
        ax = fmaf(pq[c], ex, ax);
        ay = fmaf(pq[c], ey, ay);
        az = fmaf(pq[c], ez, az);
      }
      U[4 * k][tid] = av;
      U[4 * k + 1][tid] = ax;
      U[4 * k + 2][tid] = ay;
      U[4 * k + 3][tid] = az;
    }
    __syncthreads();
    {
      const int row = tid % (kCB * 4), p = tid / (kCB * 4);
      const float4 *r = reinterpret_cast<const float4 *>(&U[row][p * (kTI / 8)]);
      // FP64 from here on: the charges come sorted by sign, so the block sums
      // are large and cancel only between blocks
      double a = 0.0;
#pragma unroll
      for (int m = 0; m < kTI / 8 / 4; ++m) {
        const float4 v = r[m];
        a += (double)v.x;
        a += (double)v.y;
        a += (double)v.z;
        a += (double)v.w;
      }
      red[p][row] = a;
    }
    __syncthreads();
    if (tid < kCB * 4) {
      double t = red[0][tid];
#pragma unroll
      for (int p = 1; p < kTI / (kCB * 4); ++p) t += red[p][tid];
      accd += t;
    }
  }
  if (tid < kCB * 4) {
    const int k = kb + tid / 4;
    if (k < N) part[(size_t)blockIdx.y * 4 * N + (size_t)(tid % 4) * N + k] = accd;
  }
}

// Near part of the mixed influence: the pairs that the far kernel's FP32
// test (same values, recentred on the first cell of the far kernel's 256-cell
// workgroup) puts within 3 D, in FP64 closed form.  One wave of 64 cells per
// workgroup; gridDim.y splits the 256-charge tiles, each split writing its
// own partial slot.  A tile is visited when some lane's cell can reach its
// box: distance below 3 D (1 + 1e-5) + 1e-6 |c_k - c0|, which exceeds what
// FP32 rounding of the recentred coordinates can add to the test.
constexpr int kNW = 64;

__global__ __launch_bounds__(kNW) void k_influence_near(int N, const double *__restrict__ f,
                                                        const int32_t *__restrict__ ord, int n_s,
                                                        const double *__restrict__ sx,
                                                        const double *__restrict__ sy,
                                                        const double *__restrict__ sz,
                                                        const double *__restrict__ sq,
                                                        const double *__restrict__ tbox, int tchunk, double *part) {
  __shared__ float4 P[kTI];
  const int lane = threadIdx.x;
  const int k = blockIdx.x * kNW + lane;
  const bool active = k < N;
  const int kk = ord[active ? k : N - 1];
  const int k0 = ord[(blockIdx.x * kNW / kTI) * kTI];
  const double c0 = f[(size_t)MF_GX * N + k0], c1 = f[(size_t)MF_GY * N + k0], c2 = f[(size_t)MF_GZ * N + k0];
  const double G0 = f[(size_t)MF_GX * N + kk], G1 = f[(size_t)MF_GY * N + kk], G2 = f[(size_t)MF_GZ * N + kk];
  const float g0 = (float)(G0 - c0), g1 = (float)(G1 - c1), g2 = (float)(G2 - c2);
  const double D = f[(size_t)MF_DIAM * N + kk];
  const float lim_near = (float)(kNearMixed * kNearMixed * D * D);
  const double off = sqrt((G0 - c0) * (G0 - c0) + (G1 - c1) * (G1 - c1) + (G2 - c2) * (G2 - c2));
  const double reach = kNearMixed * D * (1.0 + 1e-5) + 1e-6 * off;
  const double reach2 = active ? reach * reach : -1.0;
  double nv = 0, nx = 0, ny = 0, nz = 0;
  const int ntile = (n_s + kTI - 1) / kTI;
  const int tb = blockIdx.y * tchunk, te = min(ntile, tb + tchunk);
  for (int t = tb; t < te; ++t) {
    const double *bx = tbox + 6 * (size_t)t;
    const double e0 = fmax(fmax(bx[0] - G0, G0 - bx[3]), 0.0);
    const double e1 = fmax(fmax(bx[1] - G1, G1 - bx[4]), 0.0);
    const double e2 = fmax(fmax(bx[2] - G2, G2 - bx[5]), 0.0);
    if (!__any(e0 * e0 + e1 * e1 + e2 * e2 < reach2)) continue;  // wave-uniform
    const int jt = t * kTI, cnt = min(kTI, n_s - jt);
    __syncthreads();
    for (int jj = lane; jj < cnt; jj += kNW)
      P[jj] = make_float4((float)(sx[jt + jj] - c0), (float)(sy[jt + jj] - c1), (float)(sz[jt + jj] - c2), 0.f);
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      const float4 p = P[jj];
      const bool nearp = active && dist2f(p.x, p.y, p.z, g0, g1, g2) < lim_near;
      if (__any(nearp)) {
        if (nearp) {
          const int j = jt + jj;
          infl_closed(f, N, kk, sx[j], sy[j], sz[j], sq[j], nv, nx, ny, nz);
        }
      }
    }
  }
  if (active) {
    const size_t o = (size_t)blockIdx.y * 4 * N;
    part[o + k] = nv;
    part[o + (size_t)N + k] = nx;
    part[o + 2 * (size_t)N + k] = ny;
    part[o + 3 * (size_t)N + k] = nz;
  }
}

__global__ __launch_bounds__(kTI) void k_influence_fp64(int N, const double *__restrict__ f,
                                                        const int32_t *__restrict__ ord, int n_s,
                                                        const double *__restrict__ sx,
                                                        const double *__restrict__ sy,
                                                        const double *__restrict__ sz,
                                                        const double *__restrict__ sq, int chunk, double *part) {
  __shared__ double4 P[kTI];
  const int tid = threadIdx.x;
  const int k = blockIdx.x * kTI + tid;  // sorted position
  const bool active = k < N;
  const int kk = ord[active ? k : N - 1];  // cell index
  const double g0 = f[(size_t)MF_GX * N + kk], g1 = f[(size_t)MF_GY * N + kk], g2 = f[(size_t)MF_GZ * N + kk];
  const double area = f[(size_t)MF_AREA * N + kk], D = f[(size_t)MF_DIAM * N + kk];
  const double lim = kQuadFp64 * kQuadFp64 * D * D;
  double q7[21];
#pragma unroll
  for (int m = 0; m < 21; ++m) q7[m] = f[(size_t)(MF_Q7 + m) * N + kk];
  double sv = 0, ex = 0, ey = 0, ez = 0;
  const int jb = blockIdx.y * chunk, je = min(n_s, jb + chunk);
  for (int jt = jb; jt < je; jt += kTI) {
    const int cnt = min(kTI, je - jt);
    __syncthreads();
    if (tid < cnt) {
      const int j = jt + tid;
      P[tid] = make_double4(sx[j], sy[j], sz[j], sq[j]);
    }
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      const double4 p = P[jj];
      const double dx = p.x - g0, dy = p.y - g1, dz = p.z - g2;
      const bool quad = fma(dx, dx, fma(dy, dy, dz * dz)) >= lim;
      if (!__all(quad)) {
        if (!quad && active) infl_closed(f, N, kk, p.x, p.y, p.z, p.w, sv, ex, ey, ez);
      }
      if (__any(quad)) {
        if (quad) {
#pragma unroll
          for (int m = 0; m < 7; ++m) {
            const double w = area * ((m == 0) ? Rule7::w0 : (m < 4 ? Rule7::wa : Rule7::wb));
            const double ax = p.x - q7[3 * m], ay = p.y - q7[3 * m + 1], az = p.z - q7[3 * m + 2];
            const double ri = 1.0 / sqrt(fma(ax, ax, fma(ay, ay, az * az)));
            const double wr = p.w * w * ri;
            const double s = wr * ri * ri;
            sv += wr;
            ex = fma(s, ax, ex);
            ey = fma(s, ay, ey);
            ez = fma(s, az, ez);
          }
        }
      }
    }
  }
  if (active) {
    const size_t o = (size_t)blockIdx.y * 4 * N;
    part[o + k] = sv;
    part[o + (size_t)N + k] = ex;
    part[o + 2 * (size_t)N + k] = ey;
    part[o + 3 * (size_t)N + k] = ez;
  }
}

// Sum of the chunks in order, then the modified left-hand side.
__global__ __launch_bounds__(256) void k_influence_rhs(int N, int nch, const double *__restrict__ part,
                                                       const int32_t *__restrict__ ord,
                                                       const double *__restrict__ f, const int8_t *__restrict__ kind,
                                                       const double *__restrict__ rhs, double *rhs_out, double *vbar,
                                                       double *ebx, double *eby, double *ebz) {
  const int k = blockIdx.x * 256 + threadIdx.x;  // sorted position
  if (k >= N) return;
  const int i = ord[k];
  double s[4] = {0, 0, 0, 0};
  for (int c = 0; c < nch; ++c)
#pragma unroll
    for (int m = 0; m < 4; ++m) s[m] += part[(size_t)c * 4 * N + (size_t)m * N + k];
  const double area = f[(size_t)MF_AREA * N + i];
  const double vb = kKe * s[0] / area;
  const double eb[3] = {-kKe * s[1] / area, -kKe * s[2] / area, -kKe * s[3] / area};
  if (vbar) vbar[i] = vb;
  if (ebx) {
    ebx[i] = eb[0];
    eby[i] = eb[1];
    ebz[i] = eb[2];
  }
  if (kind[i] == 0) {
    rhs_out[i] = rhs[i] - vb;
  } else {
    const double en = eb[0] * f[(size_t)MF_NX * N + i] + eb[1] * f[(size_t)MF_NY * N + i] +
                      eb[2] * f[(size_t)MF_NZ * N + i];
    rhs_out[i] = rhs[i] - kEps0 * (f[(size_t)MF_EPS2 * N + i] - f[(size_t)MF_EPS1 * N + i]) * en;
  }
}

obem_status influence_rhs(obem_ctx *ctx, const obem_meshh *m, int64_t n_src, const double *sx, const double *sy,
                          const double *sz, const double *sq, const double *rhs, double *rhs_out, obem_precision prec,
                          double *vbar, double *ebx, double *eby, double *ebz) {
  const int N = (int)m->n, n_s = (int)n_src;
  const int bc = (N + kTI - 1) / kTI;
  // workgroups along the cells: 256 cells each (FP64), 8 (mixed far kernel)
  const int bw = (prec == OBEM_MIXED) ? (N + kCB - 1) / kCB : bc;
  int nsplit = 1, chunk = std::max(n_s, 1);
  if (n_s > 0) {
    nsplit = std::max(1, std::min((kSplitWorkgroups + bw - 1) / bw, (n_s + 1023) / 1024));
    nsplit = std::min(nsplit, 64);
    chunk = (n_s + nsplit - 1) / nsplit;
    chunk = (chunk + kTI * kCS - 1) / (kTI * kCS) * (kTI * kCS);
    nsplit = (n_s + chunk - 1) / chunk;
  }
  // mixed: partial slots of the near kernel after those of the far kernel
  const int ntile = (n_s + kTI - 1) / kTI;
  const int bn = (N + kNW - 1) / kNW;
  const int nnear = std::max(1, std::min(ntile, std::min(16, (2048 + bn - 1) / bn)));
  const int tchunk = std::max(1, (ntile + nnear - 1) / nnear);
  const int nslot = (n_s > 0 && prec == OBEM_MIXED) ? nsplit + (ntile + tchunk - 1) / tchunk : nsplit;
  double *part = (double *)ws_get(ctx, WS_MISC3, sizeof(double) * 4 * (size_t)N * nslot);
  if (!part) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  OBEM_PROF(ctx, "influence");
  if (n_s == 0) {
    obem_status st = launch_fill(ctx, part, 4 * (size_t)N, 0.0);
    if (st) return st;
  } else if (prec == OBEM_MIXED) {
    SourceOrder so;
    obem_status st = order_sources(ctx, n_s, sx, sy, sz, sq, false, &so);
    if (st) return st;
    hipLaunchKernelGGL(k_influence_mixed, dim3(bw, nsplit), dim3(kTI), 0, ctx->stream, N, m->f, m->order, n_s, so.x,
                       so.y, so.z, so.q, chunk, part);
    hipLaunchKernelGGL(k_influence_near, dim3(bn, nslot - nsplit), dim3(kNW), 0, ctx->stream, N, m->f, m->order, n_s,
                       so.x, so.y, so.z, so.q, so.tbox, tchunk, part + 4 * (size_t)N * nsplit);
  } else {
    hipLaunchKernelGGL(k_influence_fp64, dim3(bc, nsplit), dim3(kTI), 0, ctx->stream, N, m->f, m->order, n_s, sx, sy,
                       sz, sq, chunk, part);
  }
  OBEM_HIP(ctx, hipGetLastError());
  hipLaunchKernelGGL(k_influence_rhs, dim3(bc), dim3(256), 0, ctx->stream, N, n_s > 0 ? nslot : 1, part, m->order,
                     m->f, m->kind, rhs, rhs_out, vbar, ebx, eby, ebz);
  OBEM_HIP(ctx, hipGetLastError());
  return OBEM_OK;
}

}  // namespace obem

using namespace obem;

extern "C" obem_status bem_influence(obem_ctx *ctx, const obem_meshh *mesh, int64_t n_src, const double *sx,
                                     const double *sy, const double *sz, const double *sq, const double *rhs,
                                     double *rhs_out, obem_precision precision, double *vbar, double *ebar_x,
                                     double *ebar_y, double *ebar_z) {
  if (!ctx) return OBEM_EINVAL;
  if (ctx->sticky) return OBEM_ESTATE;
  if (hipSetDevice(ctx->device) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, OBEM_EDEVICE, "hipSetDevice failed");
  }
  if (!mesh) return fail(ctx, OBEM_EINVAL, "mesh is NULL");
  if (n_src < 0 || n_src >= ((int64_t)1 << 31)) return fail(ctx, OBEM_EINVAL, "n_src out of range");
  if (precision != OBEM_FP64 && precision != OBEM_MIXED) return fail(ctx, OBEM_EINVAL, "bad precision");
  if (!is_device_ptr(rhs) || !is_device_ptr(rhs_out)) return fail(ctx, OBEM_EINVAL, "rhs / rhs_out must be device");
  if (n_src > 0 && (!is_device_ptr(sx) || !is_device_ptr(sy) || !is_device_ptr(sz) || !is_device_ptr(sq)))
    return fail(ctx, OBEM_EINVAL, "source arrays must be device memory");
  const bool eb = ebar_x || ebar_y || ebar_z;
  if (eb && !(ebar_x && ebar_y && ebar_z)) return fail(ctx, OBEM_EINVAL, "ebar_x/y/z: all or none");
  const void *outs[] = {vbar, ebar_x, ebar_y, ebar_z};
  for (const void *p : outs)
    if (p && !is_device_ptr(p)) return fail(ctx, OBEM_EINVAL, "outputs must be device memory");
  return influence_rhs(ctx, mesh, n_src, sx, sy, sz, sq, rhs, rhs_out, precision, vbar, ebar_x, ebar_y, ebar_z);
}
