// One tracking step of the dynamic option (sections 3.3-3.4): charging-up
// right-hand side and re-solve, field at every particle, electron-cation
// recombination, constant-field flights with null-collision Monte Carlo,
// absorption on cells, compaction with deterministic ids.
//
// Determinism: random numbers are counter-based (Philox4x32-10 keyed by the
// seed, counter (id, step, flight)); every reduction is over integers
// (event counts, charging counts, recombination keys) or has a fixed order,
// so a step is bitwise reproducible.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <vector>

#include "cellmath.hpp"
#include "obem_internal.hpp"

namespace obem {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the 4x32 S-P network.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k.x, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k.y, (uint32_t)p0);
  }
  return c;
}
__device__ __forceinline__ double u01(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

struct GasDev {
  int n;
  double e_min, e_max;
  const double *xs;
  double thr[5];
  double density, temperature, m_gas, m_cation, m_anion, ion_iso, ion_back;
  double nu_e, nu_i;
  const double *xi;  // anisotropy of the elastic angle (eq. (anisotrop)) or NULL
  double pen_prob, pen_level;
};

struct StepDev {
  double dt;
  uint32_t step;
  uint32_t key0, key1;
  int max_coll, max_ion;
  double lo[3], hi[3];
};

struct GridDev {
  int nx, ny, nz;
  double lo[3], h[3];
  const int32_t *start, *items;
  int N;
  const double *f;
  const int8_t *kind;
};

// Cross section k at eps (eV): linear in the normalised lethargy of eq.
// (leth) between log-spaced nodes, clamped to the end nodes.
__device__ __forceinline__ double xs_at(const GasDev &g, int k, double eps) {
  const int n = g.n;
  if (!(eps > g.e_min)) return g.xs[k * n];
  if (eps >= g.e_max) return g.xs[k * n + n - 1];
  const double p = (double)(n - 1) * (log(eps / g.e_min) / log(g.e_max / g.e_min));
  int i = (int)floor(p);
  if (i >= n - 1) i = n - 2;
  const double fr = p - (double)i;
  return g.xs[k * n + i] * (1.0 - fr) + g.xs[k * n + i + 1] * fr;
}

// N max_b max(sigma_tot,b, sigma_tot,b+1) v(E_b+1): exact bound on each bin.
__global__ __launch_bounds__(256) void k_nu_max(GasDev g, double *out) {
  __shared__ double s[256];
  double best = 0.0;
  for (int b = threadIdx.x; b + 1 < g.n; b += 256) {
    const double E1 = g.e_min * pow(g.e_max / g.e_min, (double)(b + 1) / (double)(g.n - 1));
    double s0 = 0, s1 = 0;
    for (int k = 0; k < 5; ++k) {
      s0 += g.xs[k * g.n + b];
      s1 += g.xs[k * g.n + b + 1];
    }
    const double v1 = sqrt(2.0 * E1 * kQe / kMe);
    best = fmax(best, g.density * (s0 > s1 ? s0 : s1) * v1);
  }
  s[threadIdx.x] = best;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

// First crossing of the chord p0 -> p1 with a cell (Moller-Trumbore, 1997),
// smallest parameter t in (0, 1], ties to the lower cell index; the uniform
// grid restricts the candidates to cells whose bounding boxes overlap the
// chord's.
__device__ __forceinline__ void mt_test(const GridDev &G, int k, d3 o, d3 dir, double &bt, int &best) {
  const int N = G.N;
  const double *f = G.f;
  const d3 a = mk3(f[(size_t)MF_AX * N + k], f[(size_t)MF_AY * N + k], f[(size_t)MF_AZ * N + k]);
  const d3 e1 = mk3(f[(size_t)MF_BX * N + k], f[(size_t)MF_BY * N + k], f[(size_t)MF_BZ * N + k]) - a;
  const d3 e2 = mk3(f[(size_t)MF_CX * N + k], f[(size_t)MF_CY * N + k], f[(size_t)MF_CZ * N + k]) - a;
  const d3 pv = cross3(dir, e2);
  const double det = dot3(e1, pv);
  if (det == 0.0) return;
  const double inv = 1.0 / det;
  const d3 tv = o - a;
  const double u = dot3(tv, pv) * inv;
  if (u < 0.0 || u > 1.0) return;
  const d3 qv = cross3(tv, e1);
  const double v = dot3(dir, qv) * inv;
  if (v < 0.0 || u + v > 1.0) return;
  const double t = dot3(e2, qv) * inv;
  if (t > 0.0 && t <= 1.0 && (t < bt || (t == bt && k < best))) {
    bt = t;
    best = k;
  }
}

__device__ int first_hit(const GridDev &G, const double *p0, const double *p1) {
  if (G.N == 0) return -1;
  const d3 o = mk3(p0[0], p0[1], p0[2]);
  const d3 dir = mk3(p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]);
  double bt = 2.0;
  int best = -1;
  int lo[3], hi[3];
  const int nn[3] = {G.nx, G.ny, G.nz};
  for (int c = 0; c < 3; ++c) {
    const double a = fmin(p0[c], p1[c]), b = fmax(p0[c], p1[c]);
    const double ta = floor((a - G.lo[c]) / G.h[c]), tb = floor((b - G.lo[c]) / G.h[c]);
    if (tb < 0.0 || ta >= (double)nn[c]) return -1;  // chord outside every cell's box
    lo[c] = (int)fmax(ta, 0.0);
    hi[c] = (int)fmin(tb, (double)(nn[c] - 1));
  }
  const long long span = (long long)(hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
  if (span > 4096) {  // very long chord: test every cell
    for (int k = 0; k < G.N; ++k) mt_test(G, k, o, dir, bt, best);
    return best;
  }
  for (int iz = lo[2]; iz <= hi[2]; ++iz)
    for (int iy = lo[1]; iy <= hi[1]; ++iy)
      for (int ix = lo[0]; ix <= hi[0]; ++ix) {
        const int cell = (iz * G.ny + iy) * G.nx + ix;
        for (int q = G.start[cell]; q < G.start[cell + 1]; ++q) mt_test(G, G.items[q], o, dir, bt, best);
      }
  return best;
}

__device__ __forceinline__ void iso_dir(double u2, double u3, double *d) {
  const double ct = 1.0 - 2.0 * u2, st = sqrt(fmax(0.0, 1.0 - ct * ct)), ph = 2.0 * kPi * u3;
  d[0] = st * cos(ph);
  d[1] = st * sin(ph);
  d[2] = ct;
}

// Table value at eps (eV), linear in the normalised lethargy of eq. (leth)
// between log-spaced nodes, clamped to the end nodes (as xs_at).
__device__ __forceinline__ double table_at(const GasDev &g, const double *tab, double eps) {
  const int n = g.n;
  if (!(eps > g.e_min)) return tab[0];
  if (eps >= g.e_max) return tab[n - 1];
  const double p = (double)(n - 1) * (log(eps / g.e_min) / log(g.e_max / g.e_min));
  int i = (int)floor(p);
  if (i >= n - 1) i = n - 2;
  const double fr = p - (double)i;
  return tab[i] * (1.0 - fr) + tab[i + 1] * fr;
}

// Unit vector at polar angle theta (cosine ct) and azimuth 2 pi u about the
// unit vector d: e1 = (a x d)/|a x d| with a the z axis (the x axis when d is
// within 25.8 degrees of z), e2 = d x e1.
__device__ __forceinline__ void rotate_about(const double *d, double ct, double u, double *out) {
  double a[3] = {0.0, 0.0, 1.0};
  if (fabs(d[2]) >= 0.9) {
    a[0] = 1.0;
    a[2] = 0.0;
  }
  double e1[3] = {a[1] * d[2] - a[2] * d[1], a[2] * d[0] - a[0] * d[2], a[0] * d[1] - a[1] * d[0]};
  const double l = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
#pragma unroll
  for (int k = 0; k < 3; ++k) e1[k] /= l;
  const double e2[3] = {d[1] * e1[2] - d[2] * e1[1], d[2] * e1[0] - d[0] * e1[2], d[0] * e1[1] - d[1] * e1[0]};
  const double st = sqrt(fmax(0.0, 1.0 - ct * ct)), ph = 2.0 * kPi * u;
  const double cp = cos(ph), sp = sin(ph);
#pragma unroll
  for (int k = 0; k < 3; ++k) out[k] = ct * d[k] + st * (cp * e1[k] + sp * e2[k]);
}

enum {
  C_EL = 0, C_NULL = 5, C_ION = 6, C_OVF = 7, C_CAP = 8, C_DROP = 9, C_ABS = 10, C_LEFT = 11, C_DD = 12, C_PEN = 13,
  NCNT = 14
};

// Child pairs (electron, cation) of one particle in this step: slots
// child[((i*max_ion + c)*2 + {0, 1})*6 + (x, v)].
struct Kids {
  double *child;
  int max_ion;
  int i;
  int nc;
};

__device__ __forceinline__ bool add_pair(Kids &K, const double *xe, const double *ve, const double *xc,
                                         const double *vc) {
  if (K.nc >= K.max_ion) return false;
  double *ce = K.child + (((size_t)K.i * K.max_ion + K.nc) * 2 + 0) * 6;
  double *ci = K.child + (((size_t)K.i * K.max_ion + K.nc) * 2 + 1) * 6;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    ce[d] = xe[d];
    ce[3 + d] = ve[d];
    ci[d] = xc[d];
    ci[3 + d] = vc[d];
  }
  ++K.nc;
  return true;
}

// Real interaction `proc` (elastic, exc1, exc2, ionisation, attachment) of an
// electron of energy eps (eV) at X with velocity V (section 3.4.3).  u2, u3:
// the collision's own uniforms; extra draws use counter word 3 = 2k + 1
// (ionisation, Penning) and 0x80000000 | k (Penning cation).  Returns true
// when the electron became an anion.
__device__ bool electron_interaction(const GasDev &g, int proc, double eps, double *X, double *Vv, double u2,
                                     double u3, uint64_t pid, uint32_t step, uint2 key, uint32_t k, Kids &K,
                                     int *cnt) {
  const double e_therm = 1.5 * kKb * g.temperature;
  const double v2 = Vv[0] * Vv[0] + Vv[1] * Vv[1] + Vv[2] * Vv[2];
  const double vm = sqrt(v2);
  double dir[3];
  if (proc == 0) {  // elastic, recoil loss 2 m_e/M (1 - cos theta)
    double ct;
    if (g.xi && vm > 0.0) {  // eq. (anisotrop) about the incident direction
      const double xi = table_at(g, g.xi, eps);
      ct = 1.0 - 2.0 * u2 * (1.0 - xi) / (1.0 + xi * (1.0 - 2.0 * u2));
      const double d0[3] = {Vv[0] / vm, Vv[1] / vm, Vv[2] / vm};
      rotate_about(d0, ct, u3, dir);
    } else {
      iso_dir(u2, u3, dir);
      ct = (vm > 0.0) ? (dir[0] * Vv[0] + dir[1] * Vv[1] + dir[2] * Vv[2]) / vm : 1.0;
    }
    const double e2 = eps * (1.0 - 2.0 * kMe / g.m_gas * (1.0 - ct));
    const double s = sqrt(2.0 * e2 * kQe / kMe);
#pragma unroll
    for (int d = 0; d < 3; ++d) Vv[d] = s * dir[d];
    return false;
  }
  if (proc <= 3) {
    const double e_res = (proc == 3) ? eps - g.thr[3] - e_therm / kQe : -1.0;
    if (proc != 3 || e_res <= 0.0) {  // excitation (or sub-threshold ionisation)
      double e2 = eps - g.thr[proc];
      if (e2 < 0.0) e2 = 0.0;
      iso_dir(u2, u3, dir);
      const double s = sqrt(2.0 * e2 * kQe / kMe);
#pragma unroll
      for (int d = 0; d < 3; ++d) Vv[d] = s * dir[d];
      if (proc != 3 && g.pen_prob > 0.0 && g.thr[proc] >= g.pen_level) {
        // Penning transfer (section 3.4.4): the released electron takes the
        // excess energy thr - pen_level, the cation a thermal speed, both
        // isotropic, at the collision point
        const uint4 w2 = philox10(make_uint4((uint32_t)pid, (uint32_t)(pid >> 32), step, 2u * k + 1u), key);
        if (u01(w2.x) < g.pen_prob) {
          const uint4 w3 = philox10(make_uint4((uint32_t)pid, (uint32_t)(pid >> 32), step, 0x80000000u | k), key);
          double de[3], dc[3], ve[3], vc[3];
          iso_dir(u01(w2.y), u01(w2.z), de);
          iso_dir(u01(w3.x), u01(w3.y), dc);
          const double se = sqrt(2.0 * (g.thr[proc] - g.pen_level) * kQe / kMe);
          const double si = sqrt(2.0 * e_therm / g.m_cation);
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            ve[d] = se * de[d];
            vc[d] = si * dc[d];
          }
          cnt[C_PEN] += 1;
          if (!add_pair(K, X, ve, X, vc)) cnt[C_DROP] += 2;
        }
      }
      return false;
    }
    // ionisation, eq. (distIoni)
    const uint4 w2 = philox10(make_uint4((uint32_t)pid, (uint32_t)(pid >> 32), step, 2u * k + 1u), key);
    double uh[3], ud[3];
    iso_dir(u01(w2.x), u01(w2.y), uh);
    iso_dir(u01(w2.z), u01(w2.w), ud);
    const double eres_j = e_res * kQe;
    // energy in eV (volts): r = k_e e / (2 E_res[eV]) = k_e e^2 / (2 E_res[J])
    const double r = kKe * kQe * kQe / (2.0 * eres_j);
    const double s = sqrt(2.0 * (0.5 * eres_j) / kMe);
    const double si = sqrt(2.0 * e_therm / g.m_cation);
    double xe[3], ve[3], vc[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      xe[d] = X[d] - r * uh[d];
      ve[d] = -s * uh[d];
      vc[d] = si * ud[d];
    }
    if (!add_pair(K, xe, ve, X, vc)) cnt[C_DROP] += 2;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      X[d] += r * uh[d];
      Vv[d] = s * uh[d];
    }
    return false;
  }
  // attachment: anion, momentum conserved with the gas at rest
#pragma unroll
  for (int d = 0; d < 3; ++d) Vv[d] *= kMe / g.m_anion;
  return true;
}

// Ion collision: 0 = isotropic in the centre of mass (gas at rest), 1 =
// backscatter (charge exchange: the ion takes a thermal gas velocity).
__device__ void ion_interaction(const GasDev &g, int sp, int proc, double *Vv, double u2, double u3, uint64_t pid,
                                uint32_t step, uint2 key, uint32_t k) {
  const double vm = sqrt(Vv[0] * Vv[0] + Vv[1] * Vv[1] + Vv[2] * Vv[2]);
  if (proc == 0) {
    const double mion = (sp == 1) ? g.m_cation : g.m_anion;
    const double fm = mion / (mion + g.m_gas), fM = g.m_gas / (mion + g.m_gas);
    double dir[3];
    iso_dir(u2, u3, dir);
#pragma unroll
    for (int d = 0; d < 3; ++d) Vv[d] = fm * Vv[d] + fM * vm * dir[d];
  } else {
    const uint4 w2 = philox10(make_uint4((uint32_t)pid, (uint32_t)(pid >> 32), step, 2u * k + 1u), key);
    const double sd = sqrt(kKb * g.temperature / g.m_gas);
    const double r1 = sqrt(-2.0 * log(u01(w2.x))), r2 = sqrt(-2.0 * log(u01(w2.z)));
    Vv[0] = sd * r1 * cos(2.0 * kPi * u01(w2.y));
    Vv[1] = sd * r1 * sin(2.0 * kPi * u01(w2.y));
    Vv[2] = sd * r2 * cos(2.0 * kPi * u01(w2.w));
  }
}

__device__ __forceinline__ bool outside(const StepDev &p, const double *X) {
  return X[0] < p.lo[0] || X[0] > p.hi[0] || X[1] < p.lo[1] || X[1] > p.hi[1] || X[2] < p.lo[2] || X[2] > p.hi[2];
}

// Absorption bookkeeping: a dd hit adds the particle's charge to the cell's
// elementary-charge count (eq. (charge-up)).
__device__ __forceinline__ void absorb(const GridDev &G, int hcell, int sp, int64_t *dd_counts, int *cnt) {
  cnt[C_ABS] += 1;
  if (G.kind[hcell] == 1) {
    atomicAdd((unsigned long long *)&dd_counts[hcell], (unsigned long long)(long long)(sp == 1 ? 1 : -1));
    cnt[C_DD] += 1;
  }
}

__device__ __forceinline__ void flush_counts(const int *cnt, unsigned long long *sc, unsigned long long *counters) {
#pragma unroll
  for (int k = 0; k < NCNT; ++k)
    if (cnt[k]) atomicAdd(&sc[k], (unsigned long long)cnt[k]);
  __syncthreads();
  if (threadIdx.x < NCNT && sc[threadIdx.x]) atomicAdd(&counters[threadIdx.x], sc[threadIdx.x]);
}

// Constant-field flights with null-collision Monte Carlo for one particle per
// thread.  Outputs status (0 alive, 1 absorbed, 2 left the world box), the
// hit cell, child pairs (electron, cation) in per-particle slots.
__global__ __launch_bounds__(256) void k_push_mc(int n, double *X0, double *X1, double *X2, double *V0, double *V1,
                                                 double *V2, int8_t *species, const int64_t *__restrict__ id,
                                                 const double *__restrict__ E0, const double *__restrict__ E1,
                                                 const double *__restrict__ E2, const uint8_t *__restrict__ dead,
                                                 GasDev g, StepDev p, GridDev G, int8_t *status, int32_t *hit,
                                                 int32_t *n_child, double *child, int64_t *dd_counts,
                                                 unsigned long long *counters) {
  __shared__ unsigned long long sc[NCNT];
  if (threadIdx.x < NCNT) sc[threadIdx.x] = 0;
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  int cnt[NCNT];
#pragma unroll
  for (int k = 0; k < NCNT; ++k) cnt[k] = 0;
  if (i < n) {
    status[i] = 0;
    hit[i] = -1;
    n_child[i] = 0;
  }
  if (i < n && !dead[i]) {
    double X[3] = {X0[i], X1[i], X2[i]};
    double Vv[3] = {V0[i], V1[i], V2[i]};
    const double Ef[3] = {E0[i], E1[i], E2[i]};
    int sp = species[i];
    double t = 0.0;
    bool ballistic = false;
    const uint64_t pid = (uint64_t)id[i];
    const uint2 key = make_uint2(p.key0, p.key1);
    Kids K = {child, p.max_ion, i, 0};
    int st = 0, hcell = -1;
    for (int k = 0;; ++k) {
      const double m = (sp == 0) ? kMe : (sp == 1 ? g.m_cation : g.m_anion);
      const double q = (sp == 1) ? kQe : -kQe;
      const double acc[3] = {q * Ef[0] / m, q * Ef[1] / m, q * Ef[2] / m};
      const double numax = (sp == 0) ? g.nu_e : g.nu_i;
      double tau;
      uint4 w = make_uint4(0, 0, 0, 0);
      bool last = false;
      if (ballistic || k >= p.max_coll || numax <= 0.0) {
        if (!ballistic && numax > 0.0 && k >= p.max_coll) cnt[C_CAP] += 1;
        tau = p.dt - t;
        last = true;
      } else {
        w = philox10(make_uint4((uint32_t)pid, (uint32_t)(pid >> 32), p.step, 2u * (uint32_t)k), key);
        tau = -log(u01(w.x)) / numax;
        if (t + tau >= p.dt) {
          tau = p.dt - t;
          last = true;
        }
      }
      double Xn[3], Vn[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        Xn[d] = X[d] + Vv[d] * tau + 0.5 * acc[d] * tau * tau;
        Vn[d] = Vv[d] + acc[d] * tau;
      }
      const int h = first_hit(G, X, Xn);
      if (h >= 0) {
        st = 1;
        hcell = h;
        break;
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        X[d] = Xn[d];
        Vv[d] = Vn[d];
      }
      if (outside(p, X)) {
        st = 2;
        break;
      }
      if (last) break;
      t += tau;
      const double v2 = Vv[0] * Vv[0] + Vv[1] * Vv[1] + Vv[2] * Vv[2];
      const double vm = sqrt(v2);
      const double u1 = u01(w.y), u2 = u01(w.z), u3 = u01(w.w);
      if (sp == 0) {
        const double eps = 0.5 * kMe * v2 / kQe;
        double nuk[5], tot = 0.0;
#pragma unroll
        for (int kk = 0; kk < 5; ++kk) {
          nuk[kk] = g.density * xs_at(g, kk, eps) * vm;
          tot += nuk[kk];
        }
        double lim = numax;
        if (tot > numax) {
          cnt[C_OVF] += 1;
          lim = tot;
        }
        const double sel = u1 * lim;
        double cum = 0.0;
        int proc = -1;
#pragma unroll
        for (int kk = 0; kk < 5; ++kk) {
          cum += nuk[kk];
          if (proc < 0 && sel < cum) proc = kk;
        }
        if (proc < 0) {
          cnt[C_NULL] += 1;
          continue;
        }
        cnt[C_EL + proc] += 1;
        if (electron_interaction(g, proc, eps, X, Vv, u2, u3, pid, p.step, key, (uint32_t)k, K, cnt)) {
          sp = 2;
          ballistic = true;
        }
      } else {
        const double nui = g.density * g.ion_iso * vm, nub = g.density * g.ion_back * vm;
        double lim = numax;
        if (nui + nub > numax) {
          cnt[C_OVF] += 1;
          lim = nui + nub;
        }
        const double sel = u1 * lim;
        if (sel < nui + nub) {
          ion_interaction(g, sp, sel < nui ? 0 : 1, Vv, u2, u3, pid, p.step, key, (uint32_t)k);
          cnt[C_ION] += 1;
        } else {
          cnt[C_NULL] += 1;
        }
      }
    }
    X0[i] = X[0];
    X1[i] = X[1];
    X2[i] = X[2];
    V0[i] = Vv[0];
    V1[i] = Vv[1];
    V2[i] = Vv[2];
    species[i] = (int8_t)sp;
    status[i] = (int8_t)st;
    hit[i] = hcell;
    n_child[i] = K.nc;
    if (st == 1)
      absorb(G, hcell, sp, dd_counts, cnt);
    else if (st == 2)
      cnt[C_LEFT] += 1;
  }
  flush_counts(cnt, sc, counters);
}

// Flight of duration tau for the live particles (dead == 0, status == 0):
// constant acceleration q E / m (E0 == NULL: straight drift), chord tested
// for absorption, then the world box.  The Euler stepper is one such flight
// in the start field; a PEFRL drift is one straight flight.
__global__ __launch_bounds__(256) void k_flight(int n, double *X0, double *X1, double *X2, double *V0, double *V1,
                                                double *V2, const int8_t *__restrict__ species,
                                                const double *__restrict__ E0, const double *__restrict__ E1,
                                                const double *__restrict__ E2, const uint8_t *__restrict__ dead,
                                                GasDev g, StepDev p, GridDev G, double tau, int8_t *status,
                                                int32_t *hit, int64_t *dd_counts, unsigned long long *counters) {
  __shared__ unsigned long long sc[NCNT];
  if (threadIdx.x < NCNT) sc[threadIdx.x] = 0;
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  int cnt[NCNT];
#pragma unroll
  for (int k = 0; k < NCNT; ++k) cnt[k] = 0;
  if (i < n && !dead[i] && status[i] == 0) {
    const int sp = species[i];
    const double m = (sp == 0) ? kMe : (sp == 1 ? g.m_cation : g.m_anion);
    const double q = (sp == 1) ? kQe : -kQe;
    const double X[3] = {X0[i], X1[i], X2[i]};
    const double Vv[3] = {V0[i], V1[i], V2[i]};
    const double Ef[3] = {E0 ? E0[i] : 0.0, E0 ? E1[i] : 0.0, E0 ? E2[i] : 0.0};
    double Xn[3], Vn[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double acc = E0 ? q * Ef[d] / m : 0.0;
      Xn[d] = X[d] + Vv[d] * tau + 0.5 * acc * tau * tau;
      Vn[d] = Vv[d] + acc * tau;
    }
    const int h = first_hit(G, X, Xn);
    if (h >= 0) {
      status[i] = 1;
      hit[i] = h;
      absorb(G, h, sp, dd_counts, cnt);
    } else {
      X0[i] = Xn[0];
      X1[i] = Xn[1];
      X2[i] = Xn[2];
      V0[i] = Vn[0];
      V1[i] = Vn[1];
      V2[i] = Vn[2];
      if (outside(p, Xn)) {
        status[i] = 2;
        cnt[C_LEFT] += 1;
      }
    }
  }
  flush_counts(cnt, sc, counters);
}

// PEFRL kick: v += c dt q E / m for the live particles.
__global__ __launch_bounds__(256) void k_kick(int n, double *V0, double *V1, double *V2,
                                              const int8_t *__restrict__ species, const double *__restrict__ E0,
                                              const double *__restrict__ E1, const double *__restrict__ E2,
                                              const uint8_t *__restrict__ dead, const int8_t *__restrict__ status,
                                              GasDev g, double cdt) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n || dead[i] || status[i] != 0) return;
  const int sp = species[i];
  const double m = (sp == 0) ? kMe : (sp == 1 ? g.m_cation : g.m_anion);
  const double q = (sp == 1) ? kQe : -kQe;
  V0[i] += cdt * (q / m * E0[i]);
  V1[i] += cdt * (q / m * E1[i]);
  V2[i] += cdt * (q / m * E2[i]);
}

// Per-step collision model of section 3.4.2: each live particle collides with
// probability 1 - exp(-nu_tot dt) (gas at rest), the process chosen with
// probabilities nu_k / nu_tot from one draw (counter (id, step, 0)); the
// interactions are those of the null-collision step, at the end point.
__global__ __launch_bounds__(256) void k_collide_step(int n, double *X0, double *X1, double *X2, double *V0,
                                                      double *V1, double *V2, int8_t *species,
                                                      const int64_t *__restrict__ id, const uint8_t *__restrict__ dead,
                                                      GasDev g, StepDev p, const int8_t *__restrict__ status,
                                                      int32_t *n_child, double *child, unsigned long long *counters) {
  __shared__ unsigned long long sc[NCNT];
  if (threadIdx.x < NCNT) sc[threadIdx.x] = 0;
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  int cnt[NCNT];
#pragma unroll
  for (int k = 0; k < NCNT; ++k) cnt[k] = 0;
  if (i < n) n_child[i] = 0;
  if (i < n && !dead[i] && status[i] == 0) {
    double X[3] = {X0[i], X1[i], X2[i]};
    double Vv[3] = {V0[i], V1[i], V2[i]};
    const int sp = species[i];
    const uint64_t pid = (uint64_t)id[i];
    const uint2 key = make_uint2(p.key0, p.key1);
    Kids K = {child, p.max_ion, i, 0};
    const uint4 w = philox10(make_uint4((uint32_t)pid, (uint32_t)(pid >> 32), p.step, 0u), key);
    const double v2 = Vv[0] * Vv[0] + Vv[1] * Vv[1] + Vv[2] * Vv[2];
    const double vm = sqrt(v2);
    const double u0 = u01(w.x), u1 = u01(w.y), u2 = u01(w.z), u3 = u01(w.w);
    bool changed = false;
    if (sp == 0) {
      const double eps = 0.5 * kMe * v2 / kQe;
      double nuk[5], tot = 0.0;
#pragma unroll
      for (int kk = 0; kk < 5; ++kk) {
        nuk[kk] = g.density * xs_at(g, kk, eps) * vm;
        tot += nuk[kk];
      }
      if (!(u0 < -expm1(-tot * p.dt))) {
        cnt[C_NULL] += 1;
      } else {
        const double sel = u1 * tot;
        double cum = 0.0;
        int proc = -1;
#pragma unroll
        for (int kk = 0; kk < 5; ++kk) {
          cum += nuk[kk];
          if (proc < 0 && sel < cum) proc = kk;
        }
        if (proc < 0) proc = 4;
        cnt[C_EL + proc] += 1;
        if (electron_interaction(g, proc, eps, X, Vv, u2, u3, pid, p.step, key, 0u, K, cnt)) species[i] = 2;
        changed = true;
      }
    } else {
      const double nui = g.density * g.ion_iso * vm, nub = g.density * g.ion_back * vm;
      if (!(u0 < -expm1(-(nui + nub) * p.dt))) {
        cnt[C_NULL] += 1;
      } else {
        ion_interaction(g, sp, (u1 * (nui + nub) < nui) ? 0 : 1, Vv, u2, u3, pid, p.step, key, 0u);
        cnt[C_ION] += 1;
        changed = true;
      }
    }
    if (changed) {
      X0[i] = X[0];
      X1[i] = X[1];
      X2[i] = X[2];
      V0[i] = Vv[0];
      V1[i] = Vv[1];
      V2[i] = Vv[2];
    }
    n_child[i] = K.nc;
  }
  flush_counts(cnt, sc, counters);
}

// ---------------------------------------------------------------------------
// Small helper kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_build_rhs(int N, const double *__restrict__ rhs0, const int64_t *__restrict__ cnt,
                                                   const int8_t *__restrict__ kind, const double *__restrict__ f,
                                                   double *rhs) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  double r = rhs0[i];
  if (kind[i] == 1 && cnt) r += kQe * (double)cnt[i] / f[(size_t)MF_AREA * N + i];  // eq. (charge-up)
  rhs[i] = r;
}

__global__ __launch_bounds__(256) void k_charges(int n, const int8_t *__restrict__ sp, double *q) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) q[i] = (sp[i] == 1) ? kQe : -kQe;
}

// nearest partner: sorted-target order -> caller order, source-copy index ->
// caller index
__global__ __launch_bounds__(256) void k_scatter_nn(int n, const int32_t *__restrict__ perm,
                                                    const int32_t *__restrict__ nn_s,
                                                    const int32_t *__restrict__ src_perm, int32_t *nn) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const int j = nn_s[i];
    nn[perm[i]] = j >= 0 ? src_perm[j] : -1;
  }
}

// Species key of the particles taken in the targets' Hilbert order.
__global__ __launch_bounds__(256) void k_species_key(int n, const int32_t *__restrict__ perm,
                                                     const int8_t *__restrict__ sp, uint8_t *key, int32_t *idx) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const int j = perm[i];
    key[i] = (uint8_t)(sp[j] & 3);
    idx[i] = j;
  }
}

// Source copy grouped by species, Hilbert order within a species (a stable
// sort of the Hilbert-ordered particles by species): its 256-source tiles
// each carry one charge, which the pairwise kernel takes out of the inner
// loop, and are spatially compact, so the nearest-partner search can skip
// tiles farther than the recombination radius.
// Particles removed earlier in the step (dead, or status != 0 when given)
// keep their slot with charge 0.
__global__ __launch_bounds__(256) void k_gather_sources(int n, const int32_t *__restrict__ perm,
                                                        const double *__restrict__ x, const double *__restrict__ y,
                                                        const double *__restrict__ z, const int8_t *__restrict__ sp,
                                                        const uint8_t *__restrict__ dead,
                                                        const int8_t *__restrict__ status, double *out,
                                                        int8_t *sp_out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int j = perm[i];
  const bool gone = (dead && dead[j]) || (status && status[j] != 0);
  out[i] = x[j];
  out[(size_t)n + i] = y[j];
  out[2 * (size_t)n + i] = z[j];
  out[3 * (size_t)n + i] = gone ? 0.0 : ((sp[j] == 1) ? kQe : -kQe);
  sp_out[i] = sp[j];
}

// The right-hand side entries that differ (bit patterns) from the last
// re-solve's, in index order: idx[0..], db = rhs - rhs_last, at most cap of
// them (the count itself may exceed cap).  One workgroup walks the entries
// in order, so the list and hence the update's summation order are
// deterministic.
__global__ __launch_bounds__(256) void k_changed_rhs(int n, const double *__restrict__ rhs,
                                                     const double *__restrict__ last, int cap, int32_t *idx,
                                                     double *db, unsigned long long *count) {
  __shared__ int wcnt[4];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  int base = 0;
  for (int c = 0; c < n; c += 256) {
    const int i = c + t;
    const bool ch = i < n && __double_as_longlong(rhs[i]) != __double_as_longlong(last[i]);
    const unsigned long long m = __ballot(ch);
    if (lane == 0) wcnt[wv] = __popcll(m);
    __syncthreads();
    int off = base;
    for (int k = 0; k < wv; ++k) off += wcnt[k];
    const int pos = off + __popcll(m & ((1ull << lane) - 1ull));
    if (ch && pos < cap) {
      idx[pos] = i;
      db[pos] = rhs[i] - last[i];
    }
    base += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
  if (t == 0) *count = (unsigned long long)base;
}

// sigma = sigma_last + X[:, idx] db: the change of the solution for a
// change of the right-hand side in k entries, from the inverse X (column
// major) kept by the mesh; k columns read, added in list order.
__global__ __launch_bounds__(256) void k_inc_update(int n, int k, const double *__restrict__ X,
                                                    const int32_t *__restrict__ idx, const double *__restrict__ db,
                                                    const double *__restrict__ sigma_last, double *sigma) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int j = 0; j < k; ++j) d = fma(X[(size_t)idx[j] * n + i], db[j], d);
  sigma[i] = sigma_last[i] + d;
}

__global__ __launch_bounds__(256) void k_fill_u64(int n, unsigned long long *p, unsigned long long v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_fill_i8(int n, int8_t *p) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ __launch_bounds__(256) void k_fill_i32(int n, int32_t *p, int32_t v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_fill_u8(int n, uint8_t *p) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Recombination (section 3.4.3): each electron proposes to its nearest cation
// within r_rec; each cation accepts the nearest proposer, ties to the lower
// id.  key1 = bits of the FP64 squared distance (ordered like the values),
// key2 = proposer id among those at the minimum distance.
__device__ __forceinline__ bool proposal(int i, const int8_t *sp, const int32_t *nn, const double *X0,
                                         const double *X1, const double *X2, double r2, double *d2) {
  if (sp[i] != 0 || nn[i] < 0) return false;
  const int c = nn[i];
  const double dx = X0[i] - X0[c], dy = X1[i] - X1[c], dz = X2[i] - X2[c];
  *d2 = dx * dx + dy * dy + dz * dz;
  return *d2 <= r2;
}

__global__ __launch_bounds__(256) void k_recomb_a(int n, const int8_t *sp, const int32_t *nn, const double *X0,
                                                  const double *X1, const double *X2, double r2,
                                                  unsigned long long *key1) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  double d2;
  if (i < n && proposal(i, sp, nn, X0, X1, X2, r2, &d2))
    atomicMin(&key1[nn[i]], (unsigned long long)__double_as_longlong(d2));
}

__global__ __launch_bounds__(256) void k_recomb_b(int n, const int8_t *sp, const int32_t *nn, const double *X0,
                                                  const double *X1, const double *X2, double r2, const int64_t *id,
                                                  const unsigned long long *key1, unsigned long long *key2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  double d2;
  if (i < n && proposal(i, sp, nn, X0, X1, X2, r2, &d2) &&
      key1[nn[i]] == (unsigned long long)__double_as_longlong(d2))
    atomicMin(&key2[nn[i]], (unsigned long long)id[i]);
}

__global__ __launch_bounds__(256) void k_recomb_c(int n, const int8_t *sp, const int32_t *nn, const double *X0,
                                                  const double *X1, const double *X2, double r2, const int64_t *id,
                                                  const unsigned long long *key2, uint8_t *dead) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  double d2;
  if (i < n && proposal(i, sp, nn, X0, X1, X2, r2, &d2) && key2[nn[i]] == (unsigned long long)id[i]) {
    dead[i] = 1;
    dead[nn[i]] = 1;
  }
}

__global__ __launch_bounds__(256) void k_keep(int n, const uint8_t *dead, const int8_t *status, const int32_t *n_child,
                                              int32_t *keep, int32_t *kids) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  keep[i] = (!dead[i] && status[i] == 0) ? 1 : 0;
  kids[i] = 2 * n_child[i];
}

struct SoA {
  double *c[6];
  int8_t *sp;
  int64_t *id;
};

__global__ __launch_bounds__(256) void k_compact(int n, SoA in, const int32_t *keep, const int32_t *kpos,
                                                 const int32_t *kids, const int32_t *cpos, const double *child,
                                                 int max_ion, int n_surv, int take, int64_t next_id, SoA out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if (keep[i]) {
    const int o = kpos[i];
#pragma unroll
    for (int c = 0; c < 6; ++c) out.c[c][o] = in.c[c][i];
    out.sp[o] = in.sp[i];
    out.id[o] = in.id[i];
  }
  for (int c = 0; c < kids[i]; ++c) {
    const int k = cpos[i] + c;
    if (k >= take) break;
    const double *rec = child + (((size_t)i * max_ion + c / 2) * 2 + (c & 1)) * 6;
    const int o = n_surv + k;
#pragma unroll
    for (int d = 0; d < 6; ++d) out.c[d][o] = rec[d];
    out.sp[o] = (c & 1) ? 1 : 0;
    out.id[o] = next_id + k;
  }
}

// ---------------------------------------------------------------------------
// Absorption grid (built once per mesh on the host from the cell bounding
// boxes: a CSR list of cells per grid box).
// ---------------------------------------------------------------------------
static obem_status build_grid(obem_ctx *ctx, obem_meshh *m) {
  if (m->grid_start) return OBEM_OK;
  const int64_t N = m->n;
  std::vector<double> v((size_t)N * 9), diam((size_t)N);
  OBEM_HIP(ctx, hipMemcpyAsync(v.data(), m->f, sizeof(double) * 9 * N, hipMemcpyDeviceToHost, ctx->stream));
  OBEM_HIP(ctx, hipMemcpyAsync(diam.data(), m->field(MF_DIAM), sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream));
  OBEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  std::vector<double> ds = diam;
  std::nth_element(ds.begin(), ds.begin() + N / 2, ds.end());
  const double med = ds[N / 2];
  double ext[3], vol = 1.0;
  for (int c = 0; c < 3; ++c) {
    ext[c] = std::max(m->bbox_hi[c] - m->bbox_lo[c], 1e-3 * med);
    vol *= ext[c];
  }
  const double hmin = std::cbrt(vol / (double)(1 << 21));
  const double h = std::max(med, hmin) * (1.0 + 1e-12);
  int nn[3];
  for (int c = 0; c < 3; ++c) {
    nn[c] = std::max(1, (int)std::ceil(ext[c] / h));
    m->grid_n[c] = nn[c];
    m->grid_h[c] = ext[c] / nn[c] * (1.0 + 1e-12);
    m->grid_lo[c] = m->bbox_lo[c] - 1e-9 * m->grid_h[c];
  }
  const size_t ncell = (size_t)nn[0] * nn[1] * nn[2];
  std::vector<int32_t> count(ncell + 1, 0);
  auto range = [&](int64_t k, int lo[3], int hi[3]) {
    for (int c = 0; c < 3; ++c) {
      double a = INFINITY, b = -INFINITY;
      for (int vtx = 0; vtx < 3; ++vtx) {
        const double x = v[(size_t)(3 * vtx + c) * N + k];
        a = std::min(a, x);
        b = std::max(b, x);
      }
      lo[c] = std::max(0, std::min(nn[c] - 1, (int)std::floor((a - m->grid_lo[c]) / m->grid_h[c])));
      hi[c] = std::max(0, std::min(nn[c] - 1, (int)std::floor((b - m->grid_lo[c]) / m->grid_h[c])));
    }
  };
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int32_t> fillp;
    if (pass == 1) {
      for (size_t c = 0; c < ncell; ++c) count[c + 1] += count[c];
      fillp.assign(count.begin(), count.end() - 1);
    }
    std::vector<int32_t> items(pass == 1 ? count[ncell] : 0);
    for (int64_t k = 0; k < N; ++k) {
      int lo[3], hi[3];
      range(k, lo, hi);
      for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
          for (int x = lo[0]; x <= hi[0]; ++x) {
            const size_t cell = ((size_t)z * nn[1] + y) * nn[0] + x;
            if (pass == 0)
              count[cell + 1]++;
            else
              items[fillp[cell]++] = (int32_t)k;
          }
    }
    if (pass == 1) {
      if (hipMalloc(&m->grid_start, sizeof(int32_t) * (ncell + 1)) != hipSuccess ||
          hipMalloc(&m->grid_items, sizeof(int32_t) * std::max<size_t>(1, items.size())) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, OBEM_ENOMEM, "absorption grid allocation failed");
      }
      OBEM_HIP(ctx, hipMemcpy(m->grid_start, count.data(), sizeof(int32_t) * (ncell + 1), hipMemcpyHostToDevice));
      if (!items.empty())
        OBEM_HIP(ctx, hipMemcpy(m->grid_items, items.data(), sizeof(int32_t) * items.size(), hipMemcpyHostToDevice));
    }
  }
  return OBEM_OK;
}

static inline int nbt(int64_t n) { return (int)((n + 255) / 256); }

// Field at every particle from the set-up (cells with sigma, or the map) and
// from all charges still in the step (dead / status mask, may be NULL),
// into E (3 x n, caller order).  With nn (int32 x n) also the nearest
// opposite-species partner (within r_rec in mixed precision), caller index
// or -1.  The sources are a copy ordered by species, then Hilbert.
static obem_status step_field(obem_ctx *ctx, obem_meshh *mesh, const double *sigma, const MapDev *map,
                              const obem_particles *S, int n, const obem_step_params *p, const uint8_t *dead,
                              const int8_t *status, double *E, int32_t *nn) {
  const size_t nz = (size_t)n;
  uint8_t *skey = (uint8_t *)ws_get(ctx, WS_SRCKEY, 2 * nz + 64);
  int32_t *sperm = (int32_t *)ws_get(ctx, WS_SRCPERM, sizeof(int32_t) * 2 * nz);
  double *srcb = (double *)ws_get(ctx, WS_SRC, sizeof(double) * 4 * nz + nz + 64);
  double *acc = (double *)ws_get(ctx, WS_ACC, sizeof(double) * 4 * nz);
  const int ntile = nbt(n);
  double *tbox = (double *)ws_get(ctx, WS_TBOX, sizeof(double) * 6 * (size_t)ntile);
  int32_t *nn_s = nn ? (int32_t *)ws_get(ctx, WS_MISC0, sizeof(int32_t) * nz) : nullptr;
  double *nnd = nn ? (double *)ws_get(ctx, WS_MISC3, sizeof(double) * nz) : nullptr;
  if (!skey || !sperm || !srcb || !acc || !tbox || (nn && (!nn_s || !nnd)))
    return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  int8_t *ssp = (int8_t *)(srcb + 4 * nz);
  TargetOrder to;
  obem_status st = order_targets(ctx, n, S->x, S->y, S->z, &to);
  if (st) return st;
  hipLaunchKernelGGL(k_species_key, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, to.perm, S->species, skey, sperm);
  size_t tb = 0;
  OBEM_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, tb, skey, skey + nz, sperm, sperm + nz, n, 0, 2,
                                                   ctx->stream));
  void *tmp = ws_get(ctx, WS_SORT_TMP2, tb + 256);
  if (!tmp) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  OBEM_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(tmp, tb, skey, skey + nz, sperm, sperm + nz, n, 0, 2,
                                                   ctx->stream));
  hipLaunchKernelGGL(k_gather_sources, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, sperm + nz, S->x, S->y, S->z,
                     S->species, dead, status, srcb, ssp);
  launch_tile_boxes(ctx, n, srcb, tbox);
  OBEM_HIP(ctx, hipGetLastError());
  // with the pair-once evaluation the targets take the source copy's order
  const bool once = pair_once_applies(n, p->precision, p->soft, false);
  if (once) {
    to.perm = sperm + nz;
    to.xs = srcb;
  }
  if (map)
    st = launch_map_acc(ctx, *map, to, acc);
  else
    st = mesh ? launch_panel_field(ctx, mesh, sigma, to, p->precision, false, acc) : launch_fill(ctx, acc, 4 * nz, 0.0);
  if (st) return st;
  st = launch_pair_field(ctx, n, srcb, srcb + nz, srcb + 2 * nz, srcb + 3 * nz, to, p->soft, p->precision, true,
                         false, S->species, ssp, acc, nn_s, nnd, tbox, p->r_rec, nullptr, once);
  if (st) return st;
  st = launch_scatter(ctx, to, acc, kKe, E, E + nz, E + 2 * nz, nullptr);
  if (st) return st;
  if (nn) hipLaunchKernelGGL(k_scatter_nn, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, to.perm, nn_s, sperm + nz, nn);
  OBEM_HIP(ctx, hipGetLastError());
  return OBEM_OK;
}

}  // namespace obem

using namespace obem;

// PEFRL coefficients (Omelyan, Mryglod, Folk, Comput. Phys. Commun. 146
// (2002) 188).
static constexpr double kPefrlXi = 0.1786178958448091;
static constexpr double kPefrlLambda = -0.2123418310626054;
static constexpr double kPefrlChi = -0.06626458266981849;

static obem_status compact_step(obem_ctx *ctx, obem_particles *S, int n, int mi, const uint8_t *dead,
                                const int8_t *status, const int32_t *nchild, const double *child, int32_t *keep,
                                int32_t *kids, const unsigned long long *cnt_dev, obem_step_stats out,
                                obem_step_stats *stats);

extern "C" obem_status track_step(obem_ctx *ctx, obem_meshh *mesh, obem_particles *S, const obem_gas *gas,
                                  const obem_step_params *p, int64_t *dd_counts, double *sigma,
                                  obem_step_stats *stats) {
  if (!ctx) return OBEM_EINVAL;
  if (ctx->sticky) return OBEM_ESTATE;
  if (hipSetDevice(ctx->device) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, OBEM_EDEVICE, "hipSetDevice failed");
  }
  if (!S || !gas || !p) return fail(ctx, OBEM_EINVAL, "state / gas / params is NULL");
  if (S->capacity <= 0 || S->capacity >= ((int64_t)1 << 31) || S->n_live < 0 || S->n_live > S->capacity)
    return fail(ctx, OBEM_EINVAL, "bad capacity / n_live");
  if (!(p->dt > 0.0) || p->max_coll < 0 || p->max_ion_per_step < 0 || p->max_ion_per_step > 64 ||
      !(p->soft >= 0.0) || !(p->r_rec >= 0.0) || !(p->ion_v_cap >= 0.0))
    return fail(ctx, OBEM_EINVAL, "bad step parameters");
  if (p->precision != OBEM_FP64 && p->precision != OBEM_MIXED) return fail(ctx, OBEM_EINVAL, "bad precision");
  if (p->stepper != OBEM_NULL_COLLISION && p->stepper != OBEM_EULER && p->stepper != OBEM_PEFRL)
    return fail(ctx, OBEM_EINVAL, "bad stepper");
  if (gas->xi && !is_device_ptr(gas->xi)) return fail(ctx, OBEM_EINVAL, "gas->xi must be device memory");
  if (!(gas->penning_prob >= 0.0 && gas->penning_prob <= 1.0)) return fail(ctx, OBEM_EINVAL, "bad penning_prob");
  if (gas->n_nodes < 2 || !(gas->e_max > gas->e_min) || !(gas->e_min > 0.0) || !is_device_ptr(gas->xs))
    return fail(ctx, OBEM_EINVAL, "bad gas tables");
  void *arrs[] = {S->x, S->y, S->z, S->vx, S->vy, S->vz, S->species, S->id};
  for (void *a : arrs)
    if (!is_device_ptr(a)) return fail(ctx, OBEM_EINVAL, "particle arrays must be device memory");
  if (p->field_out && !is_device_ptr(p->field_out)) return fail(ctx, OBEM_EINVAL, "field_out must be device memory");
  if (mesh) {
    if (!p->map && !is_device_ptr(sigma)) return fail(ctx, OBEM_EINVAL, "sigma must be device memory");
    if (mesh->n_dd && !is_device_ptr(dd_counts)) return fail(ctx, OBEM_EINVAL, "dd_counts must be device memory");
    if (p->resolve < 0 || p->resolve > 3) return fail(ctx, OBEM_EINVAL, "resolve must be 0, 1, 2 or 3");
    if (p->resolve && !is_device_ptr(p->rhs0)) return fail(ctx, OBEM_EINVAL, "rhs0 must be device memory");
  }
  MapDev gmap;
  if (p->map) {
    if (!map_dev(p->map, &gmap)) return fail(ctx, OBEM_EINVAL, "bad field map");
    if (p->resolve) return fail(ctx, OBEM_EINVAL, "the static field map excludes the re-solve");
  }
  obem_status st;
  const int n = (int)S->n_live;
  obem_step_stats out = {};
  // 1. charging-up right-hand side and re-solve
  if (mesh && p->resolve) {
    const int N = (int)mesh->n;
    double *rhs = (double *)ws_get(ctx, WS_MISC6, sizeof(double) * N);
    if (!rhs) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
    hipLaunchKernelGGL(k_build_rhs, dim3(nbt(N)), dim3(256), 0, ctx->stream, N, p->rhs0,
                       mesh->n_dd ? dd_counts : nullptr, mesh->kind, mesh->f, rhs);
    OBEM_HIP(ctx, hipGetLastError());
    if (p->influence && n > 0) {
      // the live particles' influence on the cell equations (section 3.3.2)
      double *qp = (double *)ws_get(ctx, WS_MISC4, sizeof(double) * (size_t)n);
      if (!qp) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
      hipLaunchKernelGGL(k_charges, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, S->species, qp);
      OBEM_HIP(ctx, hipGetLastError());
      st = influence_rhs(ctx, mesh, n, S->x, S->y, S->z, qp, rhs, rhs, p->precision, nullptr, nullptr, nullptr,
                         nullptr);
      if (st) return st;
    }
    bool solve = true;
    if ((p->resolve == 2 || p->resolve == 3) && mesh->last_valid) {
      unsigned long long *nd = (unsigned long long *)ws_get(ctx, WS_MISC7, sizeof(unsigned long long));
      int32_t *idx = (int32_t *)ws_get(ctx, WS_INC_IDX, sizeof(int32_t) * kIncMax);
      double *db = (double *)ws_get(ctx, WS_INC_DB, sizeof(double) * kIncMax);
      if (!nd || !idx || !db) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
      unsigned long long h = 0;
      hipLaunchKernelGGL(k_changed_rhs, dim3(1), dim3(256), 0, ctx->stream, N, rhs, mesh->rhs_last, kIncMax, idx,
                         db, nd);
      OBEM_HIP(ctx, hipGetLastError());
      OBEM_HIP(ctx, hipMemcpyAsync(&h, nd, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
      OBEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
      if (h == 0) {
        OBEM_HIP(ctx, hipMemcpyAsync(sigma, mesh->sigma_last, sizeof(double) * N, hipMemcpyDeviceToDevice,
                                     ctx->stream));
        solve = false;
      } else if (p->resolve == 3 && h <= (unsigned long long)kIncMax && mesh->inc_since_solve < kIncEvery) {
        // eq. (charge-up) changes the right-hand side in the few dd cells hit
        // this step: sigma moves by those columns of the inverse
        OBEM_PROF(ctx, "solve");
        hipLaunchKernelGGL(k_inc_update, dim3(nbt(N)), dim3(256), 0, ctx->stream, N, (int)h, mesh->LU, idx, db,
                           mesh->sigma_last, sigma);
        OBEM_HIP(ctx, hipGetLastError());
        OBEM_HIP(ctx, hipMemcpyAsync(mesh->rhs_last, rhs, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream));
        OBEM_HIP(ctx, hipMemcpyAsync(mesh->sigma_last, sigma, sizeof(double) * N, hipMemcpyDeviceToDevice,
                                     ctx->stream));
        ++mesh->inc_since_solve;
        solve = false;
      }
    }
    if (solve) {
      // one refinement sweep: the backward error is then below 1e-18 on the
      // GEM meshes, and a second sweep lowers it by less than a factor 2
      st = bem_solve(ctx, mesh, rhs, sigma, 1, nullptr);
      if (st) return st;
      mesh->inc_since_solve = 0;
      if (!mesh->rhs_last) {
        if (hipMalloc(&mesh->rhs_last, sizeof(double) * N) != hipSuccess ||
            hipMalloc(&mesh->sigma_last, sizeof(double) * N) != hipSuccess) {
          (void)hipGetLastError();
          (void)hipFree(mesh->rhs_last);
          mesh->rhs_last = nullptr;
          mesh->sigma_last = nullptr;
          return fail(ctx, OBEM_ENOMEM, "allocation of the last re-solve failed");
        }
      }
      OBEM_HIP(ctx, hipMemcpyAsync(mesh->rhs_last, rhs, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream));
      OBEM_HIP(ctx, hipMemcpyAsync(mesh->sigma_last, sigma, sizeof(double) * N, hipMemcpyDeviceToDevice,
                                   ctx->stream));
      mesh->last_valid = true;
    }
  }
  if (mesh) {
    st = build_grid(ctx, mesh);
    if (st) return st;
  }
  if (n == 0) {
    if (stats) *stats = out;
    return OBEM_OK;
  }
  // scratch
  const int mi = p->max_ion_per_step;
  const size_t nz = (size_t)n;
  double *E = (double *)ws_get(ctx, WS_MISC5, sizeof(double) * 3 * nz);
  int32_t *nn = (int32_t *)ws_get(ctx, WS_MISC1, sizeof(int32_t) * nz * 4 + 64);
  int8_t *status = (int8_t *)ws_get(ctx, WS_STATUS, nz + 64);
  if (!E || !nn || !status) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  int32_t *keep = nn + nz, *kids = nn + 2 * nz, *hitv = nn + 3 * nz;
  // 2. field at every particle (cells or map + all other particles) and nearest partner
  st = step_field(ctx, mesh, sigma, p->map ? &gmap : nullptr, S, n, p, nullptr, nullptr, E, nn);
  if (st) return st;
  if (p->field_out)
    OBEM_HIP(ctx, hipMemcpyAsync(p->field_out, E, sizeof(double) * 3 * nz, hipMemcpyDeviceToDevice, ctx->stream));
  // 3. recombination
  unsigned long long *key = (unsigned long long *)ws_get(ctx, WS_MISC2, sizeof(unsigned long long) * 2 * nz);
  uint8_t *dead = (uint8_t *)ws_get(ctx, WS_MISC6, nz + 64);
  if (!key || !dead) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  hipLaunchKernelGGL(k_fill_u64, dim3(nbt(2 * n)), dim3(256), 0, ctx->stream, 2 * n, key, ~0ull);
  hipLaunchKernelGGL(k_fill_u8, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, dead);
  const double r2 = p->r_rec * p->r_rec;
  {
  OBEM_PROF(ctx, "recombine");
  hipLaunchKernelGGL(k_recomb_a, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, S->species, nn, S->x, S->y, S->z, r2, key);
  hipLaunchKernelGGL(k_recomb_b, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, S->species, nn, S->x, S->y, S->z, r2,
                     S->id, key, key + nz);
  hipLaunchKernelGGL(k_recomb_c, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, S->species, nn, S->x, S->y, S->z, r2,
                     S->id, key + nz, dead);
  }
  OBEM_HIP(ctx, hipGetLastError());
  // 4. push + null-collision MC + absorption
  GasDev g;
  g.n = gas->n_nodes;
  g.e_min = gas->e_min;
  g.e_max = gas->e_max;
  g.xs = gas->xs;
  for (int k = 0; k < 5; ++k) g.thr[k] = gas->thr[k];
  g.density = gas->density;
  g.temperature = gas->temperature;
  g.m_gas = gas->m_gas;
  g.m_cation = gas->m_cation;
  g.m_anion = gas->m_anion;
  g.ion_iso = gas->ion_xs_iso;
  g.ion_back = gas->ion_xs_back;
  g.xi = gas->xi;
  g.pen_prob = gas->penning_prob;
  g.pen_level = gas->penning_level;
  double *nu_dev = (double *)ws_get(ctx, WS_SOLVE2 + 0, 64);
  unsigned long long *cnt_dev = (unsigned long long *)ws_get(ctx, WS_SOLVE1 + 0, 256);
  if (!nu_dev || !cnt_dev) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  hipLaunchKernelGGL(k_nu_max, dim3(1), dim3(256), 0, ctx->stream, g, nu_dev);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, ctx->stream, NCNT, cnt_dev, 0ull);
  OBEM_HIP(ctx, hipGetLastError());
  OBEM_HIP(ctx, hipMemcpyAsync(&g.nu_e, nu_dev, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  OBEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  g.nu_i = gas->density * (gas->ion_xs_iso + gas->ion_xs_back) * p->ion_v_cap;
  StepDev sd;
  sd.dt = p->dt;
  sd.step = p->step;
  sd.key0 = (uint32_t)(p->seed & 0xffffffffu);
  sd.key1 = (uint32_t)(p->seed >> 32);
  sd.max_coll = p->max_coll;
  sd.max_ion = mi;
  for (int c = 0; c < 3; ++c) {
    sd.lo[c] = p->box_lo[c];
    sd.hi[c] = p->box_hi[c];
  }
  GridDev G = {};
  if (mesh) {
    G.nx = mesh->grid_n[0];
    G.ny = mesh->grid_n[1];
    G.nz = mesh->grid_n[2];
    for (int c = 0; c < 3; ++c) {
      G.lo[c] = mesh->grid_lo[c];
      G.h[c] = mesh->grid_h[c];
    }
    G.start = mesh->grid_start;
    G.items = mesh->grid_items;
    G.N = (int)mesh->n;
    G.f = mesh->f;
    G.kind = mesh->kind;
  }
  if (p->stepper == OBEM_NULL_COLLISION) {
    double *child = (double *)ws_get(ctx, WS_PART, sizeof(double) * 12 * (size_t)std::max(mi, 1) * nz);
    int32_t *nchild = (int32_t *)ws_get(ctx, WS_NN, sizeof(int32_t) * nz + 64);
    if (!child || !nchild) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
    {
      OBEM_PROF(ctx, "push_mc");
      hipLaunchKernelGGL(k_push_mc, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, S->x, S->y, S->z, S->vx, S->vy,
                         S->vz, S->species, S->id, E, E + nz, E + 2 * nz, dead, g, sd, G, status, hitv, nchild, child,
                         dd_counts, cnt_dev);
    }
    OBEM_HIP(ctx, hipGetLastError());
    return compact_step(ctx, S, n, mi, dead, status, nchild, child, keep, kids, cnt_dev, out, stats);
  }
  hipLaunchKernelGGL(k_fill_i8, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, status);
  hipLaunchKernelGGL(k_fill_i32, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, hitv, -1);
  if (p->stepper == OBEM_EULER) {
    OBEM_PROF(ctx, "push");
    hipLaunchKernelGGL(k_flight, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, S->x, S->y, S->z, S->vx, S->vy, S->vz,
                       S->species, E, E + nz, E + 2 * nz, dead, g, sd, G, p->dt, status, hitv, dd_counts, cnt_dev);
  } else {
    // PEFRL (Omelyan, Mryglod, Folk 2002): drifts and kicks, the field
    // re-evaluated after each of the first four drifts at the new positions
    // from the set-up and the charges still in the step
    const double dr[5] = {kPefrlXi, kPefrlChi, 1.0 - 2.0 * (kPefrlChi + kPefrlXi), kPefrlChi, kPefrlXi};
    const double kc[4] = {0.5 * (1.0 - 2.0 * kPefrlLambda), kPefrlLambda, kPefrlLambda,
                          0.5 * (1.0 - 2.0 * kPefrlLambda)};
    for (int s_ = 0; s_ < 5; ++s_) {
      {
        OBEM_PROF(ctx, "push");
        hipLaunchKernelGGL(k_flight, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, S->x, S->y, S->z, S->vx, S->vy,
                           S->vz, S->species, (const double *)nullptr, (const double *)nullptr,
                           (const double *)nullptr, dead, g, sd, G, dr[s_] * p->dt, status, hitv, dd_counts, cnt_dev);
        OBEM_HIP(ctx, hipGetLastError());
      }
      if (s_ == 4) break;
      st = step_field(ctx, mesh, sigma, p->map ? &gmap : nullptr, S, n, p, dead, status, E, nullptr);
      if (st) return st;
      hipLaunchKernelGGL(k_kick, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, S->vx, S->vy, S->vz, S->species, E,
                         E + nz, E + 2 * nz, dead, status, g, kc[s_] * p->dt);
    }
  }
  OBEM_HIP(ctx, hipGetLastError());
  double *child = (double *)ws_get(ctx, WS_PART, sizeof(double) * 12 * (size_t)std::max(mi, 1) * nz);
  int32_t *nchild = (int32_t *)ws_get(ctx, WS_NN, sizeof(int32_t) * nz + 64);
  if (!child || !nchild) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  {
    OBEM_PROF(ctx, "collide");
    hipLaunchKernelGGL(k_collide_step, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, S->x, S->y, S->z, S->vx, S->vy,
                       S->vz, S->species, S->id, dead, g, sd, status, nchild, child, cnt_dev);
  }
  OBEM_HIP(ctx, hipGetLastError());
  return compact_step(ctx, S, n, mi, dead, status, nchild, child, keep, kids, cnt_dev, out, stats);
}

// 5. compaction: survivors in id order, then children in parent order; the
// step's statistics.
static obem_status compact_step(obem_ctx *ctx, obem_particles *S, int n, int mi, const uint8_t *dead,
                                const int8_t *status, const int32_t *nchild, const double *child, int32_t *keep,
                                int32_t *kids, const unsigned long long *cnt_dev, obem_step_stats out,
                                obem_step_stats *stats) {
  const size_t nz = (size_t)n;
  hipLaunchKernelGGL(k_keep, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, dead, status, nchild, keep, kids);
  int32_t *kpos = (int32_t *)ws_get(ctx, WS_KEYS0, sizeof(int32_t) * nz);
  int32_t *cpos = (int32_t *)ws_get(ctx, WS_KEYS1, sizeof(int32_t) * nz);
  if (!kpos || !cpos) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  size_t tb = 0, tb2 = 0;
  OBEM_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb, keep, kpos, n, ctx->stream));
  OBEM_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, tb2, kids, cpos, n, ctx->stream));
  void *tmp = ws_get(ctx, WS_SORT_TMP, std::max(tb, tb2) + 256);
  if (!tmp) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  OBEM_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(tmp, tb, keep, kpos, n, ctx->stream));
  OBEM_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(tmp, tb2, kids, cpos, n, ctx->stream));
  int32_t tail[4];
  OBEM_HIP(ctx, hipMemcpyAsync(&tail[0], kpos + n - 1, 4, hipMemcpyDeviceToHost, ctx->stream));
  OBEM_HIP(ctx, hipMemcpyAsync(&tail[1], keep + n - 1, 4, hipMemcpyDeviceToHost, ctx->stream));
  OBEM_HIP(ctx, hipMemcpyAsync(&tail[2], cpos + n - 1, 4, hipMemcpyDeviceToHost, ctx->stream));
  OBEM_HIP(ctx, hipMemcpyAsync(&tail[3], kids + n - 1, 4, hipMemcpyDeviceToHost, ctx->stream));
  unsigned long long hc[NCNT];
  OBEM_HIP(ctx, hipMemcpyAsync(hc, cnt_dev, sizeof(hc), hipMemcpyDeviceToHost, ctx->stream));
  OBEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const int64_t n_surv = (int64_t)tail[0] + tail[1];
  const int64_t n_new = (int64_t)tail[2] + tail[3];
  const int64_t take = std::min<int64_t>(n_new, S->capacity - n_surv);
  // output buffers
  const size_t cap = (size_t)(n_surv + take);
  double *ob = (double *)ws_get(ctx, WS_SOLVE0, sizeof(double) * 6 * std::max<size_t>(cap, 1) + 16 * cap + 64);
  if (!ob) return fail(ctx, OBEM_ENOMEM, "workspace allocation failed");
  SoA in, o;
  double *ic[6] = {S->x, S->y, S->z, S->vx, S->vy, S->vz};
  for (int c = 0; c < 6; ++c) {
    in.c[c] = ic[c];
    o.c[c] = ob + (size_t)c * cap;
  }
  in.sp = S->species;
  in.id = S->id;
  o.id = (int64_t *)(ob + 6 * cap);
  o.sp = (int8_t *)(ob + 7 * cap);
  if (cap > 0) {
    OBEM_PROF(ctx, "compact");
    hipLaunchKernelGGL(k_compact, dim3(nbt(n)), dim3(256), 0, ctx->stream, n, in, keep, kpos, kids, cpos, child, mi,
                       (int)n_surv, (int)take, S->next_id, o);
    OBEM_HIP(ctx, hipGetLastError());
    for (int c = 0; c < 6; ++c)
      OBEM_HIP(ctx, hipMemcpyAsync(ic[c], o.c[c], sizeof(double) * cap, hipMemcpyDeviceToDevice, ctx->stream));
    OBEM_HIP(ctx, hipMemcpyAsync(S->id, o.id, sizeof(int64_t) * cap, hipMemcpyDeviceToDevice, ctx->stream));
    OBEM_HIP(ctx, hipMemcpyAsync(S->species, o.sp, cap, hipMemcpyDeviceToDevice, ctx->stream));
  }
  OBEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  // recombined count: n - survivors - absorbed - left (children not counted)
  out.absorbed = (int64_t)hc[C_ABS];
  out.left_world = (int64_t)hc[C_LEFT];
  out.recombined = n - n_surv - out.absorbed - out.left_world;
  out.children = take;
  out.children_dropped = (int64_t)hc[C_DROP] + (n_new - take);
  for (int k = 0; k < 5; ++k) out.real_collisions[k] = (int64_t)hc[C_EL + k];
  out.null_collisions = (int64_t)hc[C_NULL];
  out.ion_collisions = (int64_t)hc[C_ION];
  out.rate_overflow = (int64_t)hc[C_OVF];
  out.flight_cap = (int64_t)hc[C_CAP];
  out.dd_charge_deposited = (int64_t)hc[C_DD];
  out.penning = (int64_t)hc[C_PEN];
  S->n_live = n_surv + take;
  S->next_id += take;
  out.n_live = S->n_live;
  if (stats) *stats = out;
  if (n_new > take) return fail(ctx, OBEM_ECAPACITY, "capacity %lld reached: %lld children dropped",
                                (long long)S->capacity, (long long)(n_new - take));
  return OBEM_OK;
}
