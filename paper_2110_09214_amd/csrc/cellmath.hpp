// Device-side integrals of a flat triangular cell with unit charge density
// (the cell integrals of eqs. (BEM2), (BEM3)):
//   IV(x) = int_C dS'/|x - r'|,   IE(x) = int_C (x - r')/|x - r'|^3 dS'.
// Closed form (divergence theorem on the flat cell): with edge unit tangents
// t_e, in-plane outward normals m_e = t_e x n, edge line integrals
// f_e = int_e dl'/|x - r'| and the signed solid angle Omega,
//   IE = sum_e m_e f_e + n Omega,   IV = sum_e (m_e . (p_e - x)) f_e - h Omega.
// Far from the cell the closed form cancels (its terms are O(D/R) for an
// O((D/R)^2) result), so distant cells use symmetric quadrature rules, whose
// truncation error at those distances is below the working precision.
#pragma once

#include <hip/hip_runtime.h>

namespace obem {

struct d3 {
  double x, y, z;
};
__device__ __forceinline__ d3 mk3(double x, double y, double z) { return d3{x, y, z}; }
__device__ __forceinline__ d3 operator-(d3 a, d3 b) { return d3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ d3 operator+(d3 a, d3 b) { return d3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ d3 operator*(d3 a, double s) { return d3{a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double dot3(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ d3 cross3(d3 a, d3 b) {
  return d3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double norm3(d3 a) { return sqrt(dot3(a, a)); }

// Line integral of 1/|x - r'| along an edge whose endpoints relative to x are
// Pm -> Pp (lengths Rm, Rp), with unit tangent t and length L.  Written as
// log1p of a ratio whose numerator never cancels:
//   (Rp + lp) - (Rm + lm) = L (1 + s/(Rp + Rm)),  s = lp + lm,  l = t . P,
// switching to the mirrored form (Rm - lm)/(Rp - lp) when s < 0, and using
// (R + l)(R - l) = R0^2 (distance to the edge line squared) for the factor
// that would cancel.
__device__ __forceinline__ double edge_log(d3 Pm, double Rm, double Rp, d3 t, double L, double *lm_out,
                                           double *R0sq_out) {
  double lm = dot3(t, Pm);
  double lp = lm + L;
  d3 tx = cross3(t, Pm);
  double R0sq = dot3(tx, tx);
  double s = lp + lm, Rs = Rp + Rm;
  double f;
  // L (1 +- s/Rs) / den as one quotient: L (Rs +- s) / (Rs den), where
  // Rs +- s adds two non-negative terms
  if (s >= 0.0) {
    if (lm >= 0.0)
      f = log1p(L * (Rs + s) / (Rs * (Rm + lm)));
    else
      f = log1p(L * (Rs + s) * (Rm - lm) / (Rs * R0sq));
  } else {
    if (lp <= 0.0)
      f = log1p(L * (Rs - s) / (Rs * (Rp - lp)));
    else
      f = log1p(L * (Rs - s) * (Rp + lp) / (Rs * R0sq));
  }
  if (lm_out) *lm_out = lm;
  if (R0sq_out) *R0sq_out = R0sq;
  return f;
}

// Edge data of a cell, made once per cell when the mesh is bound: unit
// tangent t_e of edge e (vertex e to vertex e + 1), its length and the
// in-plane outward normal m_e = t_e x n.
struct CellEdges {
  d3 t[3], m[3];
  double L[3];
};

// Closed form in FP64.  P[k] = vertex k minus the target; n = unit normal;
// twoarea = |(b-a)x(c-a)|.  A target exactly in the plane gets Omega = 0 (the
// principal value of the normal field).
template <bool WANT_V>
__device__ __forceinline__ void cell_closed_form(const d3 P[3], d3 n, double twoarea, const CellEdges &E, d3 &IE,
                                                 double &IV) {
  double R[3] = {norm3(P[0]), norm3(P[1]), norm3(P[2])};
  double h = -dot3(P[0], n);
  double num = twoarea * h;
  double Om = 0.0;
  if (num != 0.0) {
    double den = R[0] * R[1] * R[2] + dot3(P[0], P[1]) * R[2] + dot3(P[0], P[2]) * R[1] +
                 dot3(P[1], P[2]) * R[0];
    Om = 2.0 * atan2(num, den);
  }
  IE = n * Om;
  IV = -h * Om;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int e1 = (e + 1) % 3;
    double f = edge_log(P[e], R[e], R[e1], E.t[e], E.L[e], nullptr, nullptr);
    IE = IE + E.m[e] * f;
    if (WANT_V) IV += dot3(E.m[e], P[e]) * f;
  }
}

// Symmetric quadrature rules on the triangle, barycentric weights
// (Radon's 7-point degree-5 rule; the 3-point degree-2 rule at the edge
// midpoint-centroid points (2/3, 1/6, 1/6)).
// Near/far test of the mixed cell field (squared FP32 distance of values
// recentred on one target of the workgroup).  The far and near kernels of
// the field and of its adjoint all use this arithmetic on identically
// recentred operands, so each (target, cell) pair is taken by exactly one.
__device__ __forceinline__ float dist2f(float a0, float a1, float a2, float b0, float b1, float b2) {
  const float dx = a0 - b0, dy = a1 - b1, dz = a2 - b2;
  return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

// Degree-4, 6-point symmetric rule on the triangle (Dunavant, Int. J.
// Numer. Methods Eng. 21 (1985) 1129): barycentric (b1, a1, a1) with weight
// w1 and (b2, a2, a2) with weight w2, each in its 3 permutations.
struct Rule6 {
  static constexpr double a1 = 0.445948490915965, b1 = 0.108103018168070, w1 = 0.223381589678011;
  static constexpr double a2 = 0.091576213509771, b2 = 0.816847572980459, w2 = 0.109951743655322;
};

// Degree-3, 4-point rule on the triangle (Strang and Fix, An Analysis of the
// Finite Element Method, 1973): the centroid with weight -27/48 and
// (3/5, 1/5, 1/5) in its 3 permutations with weight 25/48.
struct Rule4 {
  static constexpr double a = 0.2, b = 0.6, wc = -27.0 / 48.0, wp = 25.0 / 48.0;
};

struct Rule7 {
  // a = (6 - sqrt 15)/21, b = (6 + sqrt 15)/21
  static constexpr double a = 0.10128650732345633880;
  static constexpr double b = 0.47014206410511508977;
  static constexpr double w0 = 9.0 / 40.0;
  static constexpr double wa = 0.12593918054482715260;  // (155 - sqrt 15)/1200
  static constexpr double wb = 0.13239415278850618073;  // (155 + sqrt 15)/1200
};

}  // namespace obem
