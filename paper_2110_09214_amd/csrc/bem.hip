// Collocation system of eq. (matrixBEM) on the GPU: FP64 assembly from the
// analytic cell integrals, LU with partial pivoting (rocSOLVER getrf), the
// inverse formed from the factors (getri), and solves as one matrix-vector
// product followed by iterative refinement driven by a compensated FP64
// residual against the stored A.
//
// The paper assembles the dense matrix on the GPU, inverts it with cuBLAS and
// reuses the inverse whenever voltages or free charges change.  A triangular
// solve with one right-hand side is latency-bound on the GPU (hundreds of ms
// at 40k unknowns), whereas a product with the inverse reads the matrix once
// at HBM bandwidth; the refinement restores the backward error that an
// explicit inverse alone would lose.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "cellmath.hpp"
#include "obem_internal.hpp"

namespace obem {

// ---------------------------------------------------------------------------
// Assembly.  A is column-major (A[i + j N]); a workgroup computes 256 rows of
// one column, so the column cell's data are uniform (scalar loads) and the
// stores are coalesced.
//   ed row i: A_ij = k_e IV(j, r_i)                                eq. (BEMpot)
//   dd row i: A_ii = (eps1 + eps2)/2,
//             A_ij = (eps2 - eps1)/(4 pi) n_i . IE(j, r_i)         eq. (BEMfld)
// r_i = centroid of cell i.  Cells farther than 48 diameters use the FP64
// 7-point rule, nearer ones the closed form.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bem_assemble(int N, const double *__restrict__ f,
                                                      const int8_t *__restrict__ kind, double *A) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const double x0 = f[(size_t)MF_GX * N + i], x1 = f[(size_t)MF_GY * N + i], x2 = f[(size_t)MF_GZ * N + i];
  const bool dd = kind[i] == 1;
  double coef = kKe;
  d3 ni = mk3(0, 0, 0);
  double diag = 0.0;
  if (dd) {
    const double e1 = f[(size_t)MF_EPS1 * N + i], e2 = f[(size_t)MF_EPS2 * N + i];
    coef = (e2 - e1) / (4.0 * kPi);
    diag = 0.5 * (e1 + e2);
    ni = mk3(f[(size_t)MF_NX * N + i], f[(size_t)MF_NY * N + i], f[(size_t)MF_NZ * N + i]);
  }
  for (int j = blockIdx.y; j < N; j += gridDim.y) {
    double val;
    if (dd && j == i) {
      val = diag;
    } else {
      const double dx = x0 - f[(size_t)MF_GX * N + j], dy = x1 - f[(size_t)MF_GY * N + j],
                   dz = x2 - f[(size_t)MF_GZ * N + j];
      const double D = f[(size_t)MF_DIAM * N + j];
      const double R2 = fma(dx, dx, fma(dy, dy, dz * dz));
      double iv = 0.0;
      d3 ie = mk3(0, 0, 0);
      if (R2 >= kQuadFp64 * kQuadFp64 * D * D) {
        const double area = f[(size_t)MF_AREA * N + j];
#pragma unroll
        for (int q = 0; q < 7; ++q) {
          const double w = area * (q == 0 ? Rule7::w0 : (q < 4 ? Rule7::wa : Rule7::wb));
          const double qx = x0 - f[(size_t)(MF_Q7 + 3 * q) * N + j];
          const double qy = x1 - f[(size_t)(MF_Q7 + 3 * q + 1) * N + j];
          const double qz = x2 - f[(size_t)(MF_Q7 + 3 * q + 2) * N + j];
          const double ri = 1.0 / sqrt(fma(qx, qx, fma(qy, qy, qz * qz)));
          const double wr = w * ri;
          iv += wr;
          const double s = wr * ri * ri;
          ie = ie + mk3(qx, qy, qz) * s;
        }
      } else {
        d3 P[3];
        P[0] = mk3(f[(size_t)MF_AX * N + j] - x0, f[(size_t)MF_AY * N + j] - x1, f[(size_t)MF_AZ * N + j] - x2);
        P[1] = mk3(f[(size_t)MF_BX * N + j] - x0, f[(size_t)MF_BY * N + j] - x1, f[(size_t)MF_BZ * N + j] - x2);
        P[2] = mk3(f[(size_t)MF_CX * N + j] - x0, f[(size_t)MF_CY * N + j] - x1, f[(size_t)MF_CZ * N + j] - x2);
        const d3 n = mk3(f[(size_t)MF_NX * N + j], f[(size_t)MF_NY * N + j], f[(size_t)MF_NZ * N + j]);
        cell_closed_form<true>(P, n, 2.0 * f[(size_t)MF_AREA * N + j], cell_edges(f, N, j), ie, iv);
      }
      val = dd ? coef * dot3(ni, ie) : coef * iv;
    }
    A[(size_t)j * N + i] = val;
  }
}

// ---------------------------------------------------------------------------
// Compensated products (Ogita, Rump, Oishi 2005): TwoProd by FMA, TwoSum.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  const double z = s - a;
  e = (a - (s - z)) + (b - z);
}

// Row partial sums over one column chunk: mode 0 -> compensated sum of
// A_ij x_j (hi, lo), mode 1 -> sum |A_ij|.
template <int MODE>
__global__ __launch_bounds__(256) void k_rows_chunk(int N, const double *__restrict__ A, const double *__restrict__ x,
                                                    int chunk, double *hi_out, double *lo_out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const int jb = blockIdx.y * chunk, je = min(N, jb + chunk);
  // four independent compensated sums over j = jb + 4k + u (more loads in
  // flight per thread), combined in fixed order at the end
  double s[4] = {0.0, 0.0, 0.0, 0.0}, c[4] = {0.0, 0.0, 0.0, 0.0};
  int j = jb;
  for (; j + 4 <= je; j += 4) {
    double a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = A[(size_t)(j + u) * N + i];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (MODE == 0) {
        const double xj = x[j + u];
        const double p = a[u] * xj;
        const double pe = fma(a[u], xj, -p);
        double t, e;
        two_sum(s[u], p, t, e);
        s[u] = t;
        c[u] += e + pe;
      } else {
        s[u] += fabs(a[u]);
      }
    }
  }
  for (; j < je; ++j) {
    const double a = A[(size_t)j * N + i];
    if (MODE == 0) {
      const double xj = x[j];
      const double p = a * xj;
      const double pe = fma(a, xj, -p);
      double t, e;
      two_sum(s[0], p, t, e);
      s[0] = t;
      c[0] += e + pe;
    } else {
      s[0] += fabs(a);
    }
  }
  double S = s[0], C = c[0];
#pragma unroll
  for (int u = 1; u < 4; ++u) {
    double t, e;
    two_sum(S, s[u], t, e);
    S = t;
    C += e + c[u];
  }
  hi_out[(size_t)blockIdx.y * N + i] = S;
  lo_out[(size_t)blockIdx.y * N + i] = C;
}

// r_i = b_i - sum over chunks (fixed order), compensated; also max |r|.
__global__ __launch_bounds__(256) void k_residual_final(int N, int nch, const double *__restrict__ hi,
                                                        const double *__restrict__ lo, const double *__restrict__ b,
                                                        double *r) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  double s = b[i], c = 0.0;
  for (int k = 0; k < nch; ++k) {
    double t, e;
    two_sum(s, -hi[(size_t)k * N + i], t, e);
    s = t;
    c += e - lo[(size_t)k * N + i];
  }
  r[i] = s + c;
}

// Transposed compensated residual r_j = g_j - sum_i A_ij l_i: one wave per
// column of the column-major A (contiguous), Dot2 per lane, then a fixed
// shuffle tree that carries the TwoSum errors.
__global__ __launch_bounds__(256) void k_residual_t(int N, const double *__restrict__ A, const double *__restrict__ l,
                                                    const double *__restrict__ g, double *r) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= N) return;  // whole wave exits together
  const double *col = A + (size_t)j * N;
  double s = 0.0, c = 0.0;
  for (int i = lane; i < N; i += 64) {
    const double a = col[i], li = l[i];
    const double p = a * li;
    const double pe = fma(a, li, -p);
    double t, e;
    two_sum(s, p, t, e);
    s = t;
    c += e + pe;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double s2 = __shfl_xor(s, o), c2 = __shfl_xor(c, o);
    double t, e;
    two_sum(s, s2, t, e);
    s = t;
    c = c + c2 + e;
  }
  if (lane == 0) {
    double t, e;
    two_sum(g[j], -s, t, e);
    r[j] = t + (e - c);
  }
}

__global__ __launch_bounds__(256) void k_rowsum_final(int N, int nch, const double *__restrict__ hi, double *out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  double s = 0.0;
  for (int k = 0; k < nch; ++k) s += hi[(size_t)k * N + i];
  out[i] = s;
}

// max |v| over up to three vectors of length N -> out[0..2] (single block, fixed order)
__global__ __launch_bounds__(256) void k_absmax3(int N, const double *a, const double *b, const double *c, double *out) {
  __shared__ double s[3][256];
  double m[3] = {0, 0, 0};
  const double *v[3] = {a, b, c};
  for (int i = threadIdx.x; i < N; i += 256)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (v[k]) m[k] = fmax(m[k], fabs(v[k][i]));
#pragma unroll
  for (int k = 0; k < 3; ++k) s[k][threadIdx.x] = m[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < 3; ++k) s[k][threadIdx.x] = fmax(s[k][threadIdx.x], s[k][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < 3) out[threadIdx.x] = s[threadIdx.x][0];
}

// min and max |U_ii| of the LU factors (single block, fixed order)
__global__ __launch_bounds__(256) void k_diag_minmax(int N, const double *__restrict__ LU, double *out) {
  __shared__ double lo[256], hi[256];
  double a = INFINITY, b = 0.0;
  for (int i = threadIdx.x; i < N; i += 256) {
    const double d = fabs(LU[(size_t)i * N + i]);
    a = fmin(a, d);
    b = fmax(b, d);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + w]);
      hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = lo[0];
    out[1] = hi[0];
  }
}

__global__ __launch_bounds__(256) void k_axpy1(int N, const double *__restrict__ d, double *x) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < N) x[i] += d[i];
}

static inline int nb(int n) { return (n + 255) / 256; }

static int n_chunks(int N) {
  // enough workgroups for 256 CUs, >= 512 columns per chunk
  int rb = nb(N);
  int c = std::max(1, std::min((2048 + rb - 1) / rb, N / 512));
  return std::min(c, 64);
}

static obem_status handle(obem_ctx *ctx, rocblas_handle *h) {
  if (!ctx->rocblas) {
    rocblas_handle hh;
    if (rocblas_create_handle(&hh) != rocblas_status_success)
      return fail(ctx, OBEM_EDEVICE, "rocblas_create_handle failed");
    ctx->rocblas = hh;
  }
  *h = (rocblas_handle)ctx->rocblas;
  if (rocblas_set_stream(*h, ctx->stream) != rocblas_status_success)
    return fail(ctx, OBEM_EDEVICE, "rocblas_set_stream failed");
  return OBEM_OK;
}

void solver_release(obem_ctx *ctx) {
  if (ctx->rocblas) rocblas_destroy_handle((rocblas_handle)ctx->rocblas);
  ctx->rocblas = nullptr;
}

void bem_release(obem_meshh *m) {
  (void)hipFree(m->A);
  (void)hipFree(m->LU);
  (void)hipFree(m->ipiv);
  (void)hipFree(m->info);
  (void)hipFree(m->ipiv64);
  (void)hipFree(m->info64);
  m->A = m->LU = nullptr;
  m->ipiv = m->info = nullptr;
  m->ipiv64 = m->info64 = nullptr;
  m->factored = false;
}

// Matrices of 2^31 elements or more go through the 64-bit library entry
// points (the 32-bit ones index the matrix with 32-bit offsets).
static inline bool large_matrix(int N) { return (int64_t)N * N >= ((int64_t)1 << 31); }

// B = identity (column-major N x N); a workgroup writes 256 rows of strided
// columns.
__global__ __launch_bounds__(256) void k_identity(int N, double *B) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  for (int j = blockIdx.y; j < N; j += gridDim.y) B[(size_t)j * N + i] = (i == j) ? 1.0 : 0.0;
}

// Compensated residual r = b - A x (device), chunked over columns.
static obem_status residual(obem_ctx *ctx, const obem_meshh *m, const double *x, const double *b, double *r) {
  const int N = (int)m->n;
  const int nch = n_chunks(N);
  const int chunk = (N + nch - 1) / nch;
  double *hi = (double *)ws_get(ctx, WS_SOLVE1, sizeof(double) * (size_t)nch * N);
  double *lo = (double *)ws_get(ctx, WS_SOLVE2, sizeof(double) * (size_t)nch * N);
  if (!hi || !lo) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  hipLaunchKernelGGL(k_rows_chunk<0>, dim3(nb(N), nch), dim3(256), 0, ctx->stream, N, m->A, x, chunk, hi, lo);
  hipLaunchKernelGGL(k_residual_final, dim3(nb(N)), dim3(256), 0, ctx->stream, N, nch, hi, lo, b, r);
  OBEM_HIP(ctx, hipGetLastError());
  return OBEM_OK;
}

obem_status bem_factor(obem_ctx *ctx, obem_meshh *m) {
  if (m->factored) return OBEM_OK;
  const int N = (int)m->n;
  const size_t bytes = sizeof(double) * (size_t)N * N;
  const bool large = large_matrix(N);
  if (!m->A) {
    bool ok = hipMalloc(&m->A, bytes) == hipSuccess && hipMalloc(&m->LU, bytes) == hipSuccess;
    if (ok && large)
      ok = hipMalloc(&m->ipiv64, sizeof(int64_t) * N) == hipSuccess && hipMalloc(&m->info64, sizeof(int64_t)) == hipSuccess;
    else if (ok)
      ok = hipMalloc(&m->ipiv, sizeof(int32_t) * N) == hipSuccess && hipMalloc(&m->info, sizeof(int32_t)) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      bem_release(m);
      return fail(ctx, OBEM_ENOMEM, "cannot allocate the %d x %d collocation matrix and its factors", N, N);
    }
  }
  const int gy = std::min(N, 65535);
  {
    OBEM_PROF(ctx, "assemble");
    hipLaunchKernelGGL(k_bem_assemble, dim3(nb(N), gy), dim3(256), 0, ctx->stream, N, m->f, m->kind, m->A);
  }
  OBEM_HIP(ctx, hipGetLastError());
  // infinity norm of A (for the backward error)
  {
    const int nch = n_chunks(N);
    const int chunk = (N + nch - 1) / nch;
    double *hi = (double *)ws_get(ctx, WS_SOLVE1, sizeof(double) * (size_t)nch * N);
    double *lo = (double *)ws_get(ctx, WS_SOLVE2, sizeof(double) * (size_t)nch * N);
    double *rs = (double *)ws_get(ctx, WS_SOLVE0, sizeof(double) * (size_t)(3 * N + 8));
    if (!hi || !lo || !rs) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
    hipLaunchKernelGGL(k_rows_chunk<1>, dim3(nb(N), nch), dim3(256), 0, ctx->stream, N, m->A, nullptr, chunk, hi, lo);
    hipLaunchKernelGGL(k_rowsum_final, dim3(nb(N)), dim3(256), 0, ctx->stream, N, nch, hi, rs);
    hipLaunchKernelGGL(k_absmax3, dim3(1), dim3(256), 0, ctx->stream, N, rs, nullptr, nullptr, rs + 3 * N);
    OBEM_HIP(ctx, hipGetLastError());
    OBEM_HIP(ctx, hipMemcpyAsync(&m->anorm_inf, rs + 3 * N, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  }
  OBEM_HIP(ctx, hipMemcpyAsync(m->LU, m->A, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  rocblas_handle h;
  obem_status st = handle(ctx, &h);
  if (st) return st;
  {
    OBEM_PROF(ctx, "lu");
    const rocblas_status rs = large ? rocsolver_dgetrf_64(h, N, N, m->LU, N, m->ipiv64, m->info64)
                                    : rocsolver_dgetrf(h, N, N, m->LU, N, m->ipiv, m->info);
    if (rs != rocblas_status_success) return fail(ctx, OBEM_EDEVICE, "rocsolver_dgetrf failed");
  }
  int64_t info = 0;
  double *dm = (double *)ws_get(ctx, WS_MISC5, 2 * sizeof(double));
  if (!dm) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  hipLaunchKernelGGL(k_diag_minmax, dim3(1), dim3(256), 0, ctx->stream, N, m->LU, dm);
  OBEM_HIP(ctx, hipGetLastError());
  double hd[2] = {0, 0};
  if (large) {
    OBEM_HIP(ctx, hipMemcpyAsync(&info, m->info64, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
  } else {
    int32_t i32 = 0;
    OBEM_HIP(ctx, hipMemcpyAsync(&i32, m->info, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    OBEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    info = i32;
  }
  OBEM_HIP(ctx, hipMemcpyAsync(hd, dm, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  OBEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (info != 0)
    return fail(ctx, OBEM_ESINGULAR, "zero pivot U(%lld,%lld): collocation matrix is singular", (long long)info,
                (long long)info);
  // a pivot at rounding level relative to the largest one: numerically singular
  // (duplicate or coincident cells)
  if (!(hd[0] > (double)N * 2.220446049250313e-16 * hd[1]))
    return fail(ctx, OBEM_ESINGULAR, "pivot ratio min|U_ii|/max|U_ii| = %.3e: collocation matrix is numerically singular",
                hd[1] > 0 ? hd[0] / hd[1] : 0.0);
  // Inverse from the LU factors, in place (the paper likewise keeps the
  // inverse to re-solve cheaply whenever voltages or free charges change):
  // every later solve is one bandwidth-bound matrix-vector product, refined
  // against the stored A.
  if (large) {
    // no 64-bit in-place inverse: solve L U X = P I into a third buffer,
    // then keep X and release the factors
    double *X = nullptr;
    if (hipMalloc(&X, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, OBEM_ENOMEM, "cannot allocate the %d x %d inverse", N, N);
    }
    hipLaunchKernelGGL(k_identity, dim3(nb(N), std::min(N, 65535)), dim3(256), 0, ctx->stream, N, X);
    OBEM_HIP(ctx, hipGetLastError());
    {
      OBEM_PROF(ctx, "lu");
      if (rocsolver_dgetrs_64(h, rocblas_operation_none, N, N, m->LU, N, m->ipiv64, X, N) != rocblas_status_success) {
        (void)hipFree(X);
        return fail(ctx, OBEM_EDEVICE, "rocsolver_dgetrs failed");
      }
    }
    OBEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipFree(m->LU);
    m->LU = X;
  } else {
    {
      OBEM_PROF(ctx, "lu");
      if (rocsolver_dgetri(h, N, m->LU, N, m->ipiv, m->info) != rocblas_status_success)
        return fail(ctx, OBEM_EDEVICE, "rocsolver_dgetri failed");
    }
    int32_t i32 = 0;
    OBEM_HIP(ctx, hipMemcpyAsync(&i32, m->info, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    OBEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (i32 != 0) return fail(ctx, OBEM_ESINGULAR, "inversion failed at U(%d,%d)", i32, i32);
  }
  m->factored = true;
  return OBEM_OK;
}

// out = A^{-1} in, or A^{-T} in when trans (in and out distinct)
static obem_status inv_apply(obem_ctx *ctx, obem_meshh *m, const double *in, double *out, bool trans = false) {
  rocblas_handle h;
  obem_status st = handle(ctx, &h);
  if (st) return st;
  const int N = (int)m->n;
  const double one = 1.0, zero = 0.0;
  const rocblas_operation op = trans ? rocblas_operation_transpose : rocblas_operation_none;
  if (rocblas_set_pointer_mode(h, rocblas_pointer_mode_host) != rocblas_status_success)
    return fail(ctx, OBEM_EDEVICE, "rocblas_set_pointer_mode failed");
  const rocblas_status rs = large_matrix(N) ? rocblas_dgemv_64(h, op, N, N, &one, m->LU, N, in, 1, &zero, out, 1)
                                            : rocblas_dgemv(h, op, N, N, &one, m->LU, N, in, 1, &zero, out, 1);
  if (rs != rocblas_status_success) return fail(ctx, OBEM_EDEVICE, "rocblas_dgemv failed");
  return OBEM_OK;
}

obem_status bem_solve(obem_ctx *ctx, obem_meshh *m, const double *rhs, double *sigma, int max_refine,
                      obem_solve_info *info, bool trans) {
  obem_status st = bem_factor(ctx, m);
  if (st) return st;
  OBEM_PROF(ctx, "solve");
  const int N = (int)m->n;
  double *w = (double *)ws_get(ctx, WS_SOLVE0, sizeof(double) * (size_t)(3 * N + 8));
  if (!w) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  double *b = w, *r = w + N, *d = w + 2 * N, *stats = w + 3 * N;
  // keep b (rhs may alias sigma)
  OBEM_HIP(ctx, hipMemcpyAsync(b, rhs, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream));
  st = inv_apply(ctx, m, b, sigma, trans);
  if (st) return st;
  double best_err = INFINITY;
  int it = 0;
  double h[3] = {0, 0, 0};
  for (;;) {
    // without info nobody reads the residual after the last correction
    if (!info && it >= max_refine) break;
    if (trans) {
      hipLaunchKernelGGL(k_residual_t, dim3((N + 3) / 4), dim3(256), 0, ctx->stream, N, m->A, sigma, b, r);
      OBEM_HIP(ctx, hipGetLastError());
    } else {
      st = residual(ctx, m, sigma, b, r);
      if (st) return st;
    }
    if (info) {
      hipLaunchKernelGGL(k_absmax3, dim3(1), dim3(256), 0, ctx->stream, N, r, sigma, b, stats);
      OBEM_HIP(ctx, hipGetLastError());
      OBEM_HIP(ctx, hipMemcpyAsync(h, stats, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      OBEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
      const double berr = h[0] / (m->anorm_inf * h[1] + h[2] + 1e-300);
      info->iterations = it;
      info->backward_error = berr;
      info->residual_inf = h[0];
      // stop when the backward error no longer halves
      if (!(berr < 0.5 * best_err) || it >= max_refine) break;
      best_err = berr;
    }
    st = inv_apply(ctx, m, r, d, trans);
    if (st) return st;
    hipLaunchKernelGGL(k_axpy1, dim3(nb(N)), dim3(256), 0, ctx->stream, N, d, sigma);
    OBEM_HIP(ctx, hipGetLastError());
    ++it;
  }
  if (info && info->backward_error > 1e-14)
    return fail(ctx, OBEM_ENOCONV, "refinement stalled at backward error %.3e", info->backward_error);
  return OBEM_OK;
}

}  // namespace obem

using namespace obem;

extern "C" obem_status bem_solve_charges(obem_ctx *ctx, obem_meshh *mesh, const double *rhs, double *sigma_out,
                                         int max_refine, obem_solve_info *info) {
  if (!ctx) return OBEM_EINVAL;
  if (ctx->sticky) return OBEM_ESTATE;
  if (hipSetDevice(ctx->device) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, OBEM_EDEVICE, "hipSetDevice failed");
  }
  if (!mesh) return fail(ctx, OBEM_EINVAL, "mesh is NULL");
  if (max_refine < 0 || max_refine > 100) return fail(ctx, OBEM_EINVAL, "max_refine must be in [0, 100]");
  if (!is_device_ptr(rhs) || !is_device_ptr(sigma_out))
    return fail(ctx, OBEM_EINVAL, "rhs / sigma_out must be device arrays");
  return bem_solve(ctx, mesh, rhs, sigma_out, max_refine, info, false);
}

extern "C" obem_status bem_solve_charges_adjoint(obem_ctx *ctx, obem_meshh *mesh, const double *g_sigma,
                                                 double *g_rhs, int max_refine, obem_solve_info *info) {
  if (!ctx) return OBEM_EINVAL;
  if (ctx->sticky) return OBEM_ESTATE;
  if (hipSetDevice(ctx->device) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, OBEM_EDEVICE, "hipSetDevice failed");
  }
  if (!mesh) return fail(ctx, OBEM_EINVAL, "mesh is NULL");
  if (max_refine < 0 || max_refine > 100) return fail(ctx, OBEM_EINVAL, "max_refine must be in [0, 100]");
  if (!is_device_ptr(g_sigma) || !is_device_ptr(g_rhs))
    return fail(ctx, OBEM_EINVAL, "g_sigma / g_rhs must be device arrays");
  return bem_solve(ctx, mesh, g_sigma, g_rhs, max_refine, info, true);
}
