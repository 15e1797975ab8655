// Device math for the implicit MPM step: quadratic B-spline weights, a signed
// 3x3 SVD, the two elastic energy densities, their first Piola stress and the
// positive-definite projection of the stress derivative.
#pragma once

#include "hot_internal.h"

namespace hot {

// ---------------------------------------------------------------- B-spline
// Quadratic B-spline (Sec. 6): with f = (x - o)/dx - base in [1/2, 3/2) the
// weights of nodes base+0, +1, +2 are 1/2 (3/2 - f)^2, 3/4 - (f - 1)^2 and
// 1/2 (f - 1/2)^2; their derivatives (per unit length) follow.
__device__ inline double bsw(int k, double f) {
  if (k == 0) {
    double a = 1.5 - f;
    return 0.5 * (a * a);
  }
  if (k == 1) {
    double a = f - 1.0;
    return 0.75 - a * a;
  }
  double a = f - 0.5;
  return 0.5 * (a * a);
}
__device__ inline double bsdw(int k, double f, double inv_dx) {
  if (k == 0) return (f - 1.5) * inv_dx;
  if (k == 1) return -2.0 * (f - 1.0) * inv_dx;
  return (f - 0.5) * inv_dx;
}

struct Weights {
  double w[3][3];   // [axis][offset]
  double dw[3][3];
};

__device__ inline void bspline_weights(const double* f, double inv_dx, Weights& W) {
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 3; ++k) {
      W.w[a][k] = bsw(k, f[a]);
      W.dw[a][k] = bsdw(k, f[a], inv_dx);
    }
}

// weight and gradient of stencil node (kx, ky, kz)
__device__ inline double node_weight(const Weights& W, int kx, int ky, int kz) {
  return W.w[0][kx] * W.w[1][ky] * W.w[2][kz];
}
__device__ inline void node_grad(const Weights& W, int kx, int ky, int kz, double g[3]) {
  g[0] = W.dw[0][kx] * W.w[1][ky] * W.w[2][kz];
  g[1] = W.w[0][kx] * W.dw[1][ky] * W.w[2][kz];
  g[2] = W.w[0][kx] * W.w[1][ky] * W.dw[2][kz];
}

// ---------------------------------------------------------------- 3x3 algebra
__device__ inline double det3(const double* F) {
  return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
         F[2] * (F[3] * F[7] - F[4] * F[6]);
}
// cof(F) = det(F) F^{-T}: column k is the cross product of the other two.
__device__ inline void cofactor3(const double* F, double* K) {
  // columns c0 = (F0,F3,F6), c1 = (F1,F4,F7), c2 = (F2,F5,F8)
  K[0] = F[4] * F[8] - F[7] * F[5];
  K[3] = F[7] * F[2] - F[1] * F[8];
  K[6] = F[1] * F[5] - F[4] * F[2];
  K[1] = F[5] * F[6] - F[8] * F[3];
  K[4] = F[8] * F[0] - F[2] * F[6];
  K[7] = F[2] * F[3] - F[5] * F[0];
  K[2] = F[3] * F[7] - F[6] * F[4];
  K[5] = F[6] * F[1] - F[0] * F[7];
  K[8] = F[0] * F[4] - F[3] * F[1];
}

// Signed SVD F = U diag(s) V^T with U, V proper rotations, s[0] >= s[1] >=
// |s[2]|, the sign of det F carried by s[2].  One-sided (Hestenes) Jacobi on
// the columns of F V: each plane rotation orthogonalises one column pair; the
// singular values are the column norms, which keeps small singular values
// accurate.
__device__ inline void svd3(const double* F, double* U, double* s, double* V) {
  double B[9];
  for (int i = 0; i < 9; ++i) B[i] = F[i];
  for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 16; ++sweep) {
    bool rotated = false;
    for (int pr = 0; pr < 3; ++pr) {
      int p = (pr == 2) ? 1 : 0;
      int q = (pr == 0) ? 1 : 2;
      double al = 0.0, be = 0.0, ga = 0.0;
      for (int r = 0; r < 3; ++r) {
        al += B[3 * r + p] * B[3 * r + p];
        be += B[3 * r + q] * B[3 * r + q];
        ga += B[3 * r + p] * B[3 * r + q];
      }
      if (fabs(ga) <= 1e-15 * sqrt(al * be) || ga == 0.0) continue;
      rotated = true;
      double zeta = (be - al) / (2.0 * ga);
      double t;
      if (fabs(zeta) > 1e150)
        t = 0.5 / zeta;
      else
        t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
      double c = 1.0 / sqrt(1.0 + t * t);
      double sn = c * t;
      for (int r = 0; r < 3; ++r) {
        double bp = B[3 * r + p], bq = B[3 * r + q];
        B[3 * r + p] = c * bp - sn * bq;
        B[3 * r + q] = sn * bp + c * bq;
        double vp = V[3 * r + p], vq = V[3 * r + q];
        V[3 * r + p] = c * vp - sn * vq;
        V[3 * r + q] = sn * vp + c * vq;
      }
    }
    if (!rotated) break;
  }
  double nrm[3];
  for (int k = 0; k < 3; ++k)
    nrm[k] = sqrt(B[k] * B[k] + B[3 + k] * B[3 + k] + B[6 + k] * B[6 + k]);
  // sort columns by decreasing norm with a 3-comparator network; each swap
  // also negates the second column of both B and V, so V stays a rotation and
  // B V^T is unchanged.  Indices are compile-time constants (no spills).
  auto cswap = [&](const int a, const int b) {
    if (nrm[a] < nrm[b]) {
      double t = nrm[a];
      nrm[a] = nrm[b];
      nrm[b] = t;
      for (int r = 0; r < 3; ++r) {
        double ba = B[3 * r + a], bb = B[3 * r + b];
        B[3 * r + a] = bb;
        B[3 * r + b] = -ba;
        double va = V[3 * r + a], vb = V[3 * r + b];
        V[3 * r + a] = vb;
        V[3 * r + b] = -va;
      }
    }
  };
  cswap(0, 1);
  cswap(1, 2);
  cswap(0, 1);
  double Bs[9], ns[3];
  for (int i = 0; i < 9; ++i) Bs[i] = B[i];
  for (int k = 0; k < 3; ++k) ns[k] = nrm[k];
  double u0[3], u1[3], u2[3];
  if (ns[0] > 0.0) {
    for (int r = 0; r < 3; ++r) u0[r] = Bs[3 * r] / ns[0];
  } else {
    u0[0] = 1.0; u0[1] = 0.0; u0[2] = 0.0;
  }
  double d = u0[0] * Bs[1] + u0[1] * Bs[4] + u0[2] * Bs[7];
  for (int r = 0; r < 3; ++r) u1[r] = Bs[3 * r + 1] - d * u0[r];
  double n1 = sqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
  if (n1 > 1e-300 && ns[1] > 0.0) {
    for (int r = 0; r < 3; ++r) u1[r] /= n1;
  } else {
    // any unit vector orthogonal to u0
    int m = (fabs(u0[0]) < fabs(u0[1])) ? ((fabs(u0[0]) < fabs(u0[2])) ? 0 : 2)
                                        : ((fabs(u0[1]) < fabs(u0[2])) ? 1 : 2);
    double e[3] = {m == 0 ? 1.0 : 0.0, m == 1 ? 1.0 : 0.0, m == 2 ? 1.0 : 0.0};
    double dd = u0[0] * e[0] + u0[1] * e[1] + u0[2] * e[2];
    for (int r = 0; r < 3; ++r) u1[r] = e[r] - dd * u0[r];
    double nn = sqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
    for (int r = 0; r < 3; ++r) u1[r] /= nn;
  }
  u2[0] = u0[1] * u1[2] - u0[2] * u1[1];
  u2[1] = u0[2] * u1[0] - u0[0] * u1[2];
  u2[2] = u0[0] * u1[1] - u0[1] * u1[0];
  s[0] = ns[0];
  s[1] = u1[0] * Bs[1] + u1[1] * Bs[4] + u1[2] * Bs[7];
  s[2] = u2[0] * Bs[2] + u2[1] * Bs[5] + u2[2] * Bs[8];
  for (int r = 0; r < 3; ++r) {
    U[3 * r] = u0[r];
    U[3 * r + 1] = u1[r];
    U[3 * r + 2] = u2[r];
  }
}

// ---------------------------------------------------------------- materials
// Energy density.  Fixed-corotated: mu sum (s_i - 1)^2 + lambda/2 (J - 1)^2
// (= mu |F - R|^2 + ...).  Neo-Hookean: mu/2 (|F|^2 - 3) - mu ln J +
// lambda/2 (ln J)^2, +inf when J <= 0.
__device__ inline double psi_of(const MaterialDev& m, const double* F) {
  if (m.model == 0) {
    double U[9], s[3], V[9];
    svd3(F, U, s, V);
    double J = det3(F);
    double a = s[0] - 1.0, b = s[1] - 1.0, c = s[2] - 1.0;
    return m.mu * (a * a + b * b + c * c) + 0.5 * m.lam * (J - 1.0) * (J - 1.0);
  }
  double J = det3(F);
  if (!(J > 0.0)) return __builtin_inf();
  double lnJ = log(J);
  double f2 = 0.0;
  for (int i = 0; i < 9; ++i) f2 += F[i] * F[i];
  return 0.5 * m.mu * (f2 - 3.0) - m.mu * lnJ + 0.5 * m.lam * lnJ * lnJ;
}

// psi and first Piola stress P = d psi / d F.
__device__ inline double psi_and_piola(const MaterialDev& m, const double* F, double* P) {
  double K[9];
  cofactor3(F, K);
  double J = det3(F);
  if (m.model == 0) {
    double U[9], s[3], V[9];
    svd3(F, U, s, V);
    double a = s[0] - 1.0, b = s[1] - 1.0, c = s[2] - 1.0;
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) {
        double R = U[3 * r] * V[3 * q] + U[3 * r + 1] * V[3 * q + 1] + U[3 * r + 2] * V[3 * q + 2];
        P[3 * r + q] = 2.0 * m.mu * (F[3 * r + q] - R) + m.lam * (J - 1.0) * K[3 * r + q];
      }
    return m.mu * (a * a + b * b + c * c) + 0.5 * m.lam * (J - 1.0) * (J - 1.0);
  }
  if (!(J > 0.0)) {
    for (int i = 0; i < 9; ++i) P[i] = 0.0;
    return __builtin_inf();
  }
  double lnJ = log(J);
  double f2 = 0.0;
  for (int i = 0; i < 9; ++i) {
    double FinvT = K[i] / J;
    P[i] = m.mu * (F[i] - FinvT) + m.lam * lnJ * FinvT;
    f2 += F[i] * F[i];
  }
  return 0.5 * m.mu * (f2 - 3.0) - m.mu * lnJ + 0.5 * m.lam * lnJ * lnJ;
}

// Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations.
__device__ inline void sym_eig3(const double* Ain, double* ev, double* Q) {
  double A[9];
  for (int i = 0; i < 9; ++i) A[i] = Ain[i];
  for (int i = 0; i < 9; ++i) Q[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 16; ++sweep) {
    double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
    double on = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
    if (off <= 1e-32 * on || off == 0.0) break;
    for (int pr = 0; pr < 3; ++pr) {
      int p = (pr == 2) ? 1 : 0;
      int q = (pr == 0) ? 1 : 2;
      double apq = A[3 * p + q];
      if (apq == 0.0) continue;
      double theta = (A[3 * q + q] - A[3 * p + p]) / (2.0 * apq);
      double t = (fabs(theta) > 1e150) ? 0.5 / theta
                                        : (theta >= 0.0 ? 1.0 : -1.0) /
                                              (fabs(theta) + sqrt(theta * theta + 1.0));
      double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
      // A <- J^T A J with J the (p,q) rotation
      for (int k = 0; k < 3; ++k) {
        double akp = A[3 * k + p], akq = A[3 * k + q];
        A[3 * k + p] = c * akp - sn * akq;
        A[3 * k + q] = sn * akp + c * akq;
      }
      for (int k = 0; k < 3; ++k) {
        double apk = A[3 * p + k], aqk = A[3 * q + k];
        A[3 * p + k] = c * apk - sn * aqk;
        A[3 * q + k] = sn * apk + c * aqk;
      }
      for (int k = 0; k < 3; ++k) {
        double qkp = Q[3 * k + p], qkq = Q[3 * k + q];
        Q[3 * k + p] = c * qkp - sn * qkq;
        Q[3 * k + q] = sn * qkp + c * qkq;
      }
    }
  }
  ev[0] = A[0];
  ev[1] = A[4];
  ev[2] = A[8];
}

// Upper-triangle index of the symmetric 9x9 stress derivative.
__host__ __device__ inline int tri9(int a, int b) {
  if (a > b) {
    int t = a;
    a = b;
    b = t;
  }
  return a * 9 - (a * (a - 1)) / 2 + (b - a);
}

// Positive-definite projection of C = dP/dF (9x9, C[3g+b][3d+e] =
// dP_gb / dF_de), returned as its 45 upper-triangle entries times `scale`.
// Built from its eigensystem in the SVD frame: the 3x3 diagonal-space Hessian
// of psi_hat(sigma) and, for each pair (i, j), the eigenvalues on the
// symmetric and antisymmetric off-diagonal directions,
// (psi_i - psi_j)/(s_i - s_j) and (psi_i + psi_j)/(s_i + s_j), in closed forms
// free of (s_i - s_j) divisions.  Negative eigenvalues are clamped to zero.
__device__ inline void projected_dPdF(const MaterialDev& m, const double* F, double scale,
                                      double* C45) {
  double U[9], s[3], V[9];
  svd3(F, U, s, V);
  double J = s[0] * s[1] * s[2];
  double A[9];
  double lsym[3], lanti[3];
  const int PI[3] = {0, 0, 1}, PJ[3] = {1, 2, 2}, PK[3] = {2, 1, 0};
  bool fcr = (m.model == 0);
  double lnJ = (J > 0.0) ? log(J) : 0.0;
  for (int i = 0; i < 3; ++i) {
    int j = (i + 1) % 3, k = (i + 2) % 3;
    double other = s[j] * s[k];
    A[4 * i] = fcr ? 2.0 * m.mu + m.lam * other * other
                   : m.mu + (m.mu + m.lam * (1.0 - lnJ)) / (s[i] * s[i]);
  }
  for (int q = 0; q < 3; ++q) {
    int i = PI[q], j = PJ[q], k = PK[q];
    double aij = fcr ? m.lam * s[k] * (2.0 * J - 1.0) : m.lam / (s[i] * s[j]);
    A[3 * i + j] = A[3 * j + i] = aij;
    double ssum = s[i] + s[j];
    if (fabs(ssum) < 1e-12) ssum = (ssum < 0.0) ? -1e-12 : 1e-12;
    if (fcr) {
      lsym[q] = 2.0 * m.mu - m.lam * (J - 1.0) * s[k];
      lanti[q] = 2.0 * m.mu - 4.0 * m.mu / ssum + m.lam * (J - 1.0) * s[k];
    } else {
      double t = (m.mu - m.lam * lnJ) / (s[i] * s[j]);
      lsym[q] = m.mu + t;
      lanti[q] = m.mu - t;
    }
  }
  double ev[3], Q[9];
  sym_eig3(A, ev, Q);
  for (int i = 0; i < 45; ++i) C45[i] = 0.0;
  double d[9];
  // diagonal-space eigen-directions: D = U diag(q_k) V^T
  for (int k = 0; k < 3; ++k) {
    double lam = fmax(ev[k], 0.0) * scale;
    if (lam == 0.0) continue;
    for (int g = 0; g < 3; ++g)
      for (int b = 0; b < 3; ++b)
        d[3 * g + b] = U[3 * g] * Q[k] * V[3 * b] + U[3 * g + 1] * Q[3 + k] * V[3 * b + 1] +
                       U[3 * g + 2] * Q[6 + k] * V[3 * b + 2];
    for (int a = 0; a < 9; ++a)
      for (int b = a; b < 9; ++b) C45[tri9(a, b)] += lam * d[a] * d[b];
  }
  const double r2 = 0.70710678118654752440;
  for (int q = 0; q < 3; ++q) {
    int i = PI[q], j = PJ[q];
    for (int sgn = 0; sgn < 2; ++sgn) {
      double lam = fmax(sgn == 0 ? lsym[q] : lanti[q], 0.0) * scale;
      if (lam == 0.0) continue;
      double sg = (sgn == 0) ? 1.0 : -1.0;
      for (int g = 0; g < 3; ++g)
        for (int b = 0; b < 3; ++b)
          d[3 * g + b] = r2 * (U[3 * g + i] * V[3 * b + j] + sg * U[3 * g + j] * V[3 * b + i]);
      for (int a = 0; a < 9; ++a)
        for (int b = a; b < 9; ++b) C45[tri9(a, b)] += lam * d[a] * d[b];
    }
  }
}

// ---------------------------------------------------------------- waves
__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
// BF16 storage of FP32 values, round to nearest even.
__device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 3x3 inverse (adjugate / determinant)
__device__ inline void inv3(const double* A, double* B) {
  double K[9];
  cofactor3(A, K);
  double d = det3(A);
  double id = 1.0 / d;
  // inverse = cof^T / det
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) B[3 * r + c] = K[3 * c + r] * id;
}

// Finalise one block row held in LDS (acc[kRowStride], [entry][slot]) of a
// level:
//  * level 0 (fixed != null): add the lumped mass m_i I on the diagonal, then
//    project Dirichlet rows/columns (constrained rows become m_i I, blocks
//    coupling to a constrained neighbour vanish), Sec. 4.1;
//  * a DOF whose diagonal is exactly zero (no free fine DOF below it) becomes
//    constrained with diagonal 1;
//  * write the row, the per-DOF free flags, the scalar diagonal and the l1
//    block-Jacobi inverse D~^{-1} = (H_ii + diag(sum_{j != i} |H_ij| row sums))^{-1}.
// Executed by one full wave; lane l owns slots l and l + 64.
__device__ inline void finalize_row(double* acc, int i, const LevelView& L, const int* fixed,
                                    double mass_i, int lane) {
  bool row_fixed = false;
  if (fixed != nullptr) {
    row_fixed = fixed[i] != 0;
    long long pn = L.nodes[i];
    for (int s = lane; s < kSlots; s += 64) {
      bool z = row_fixed;
      if (!z && s != kCenter) {
        int j = L.map[pn + slot_offset(L.g, s)];
        z = (j >= 0 && fixed[j]);
      }
      if (z)
        for (int c = 0; c < 9; ++c) acc[c * kSlotPad + s] = 0.0;
    }
    wave_sync();
    if (lane < 3) acc[(4 * lane) * kSlotPad + kCenter] += mass_i;
    wave_sync();
  }
  if (lane == 0) {
    for (int g = 0; g < 3; ++g) {
      double d = acc[(4 * g) * kSlotPad + kCenter];
      bool zero = (d == 0.0);
      if (zero) acc[(4 * g) * kSlotPad + kCenter] = 1.0;
      L.free_dof[3 * i + g] = (!row_fixed && !zero) ? 1 : 0;
      L.diag[3 * i + g] = zero ? 1.0 : d;
    }
  }
  wave_sync();
  double l1[3] = {0.0, 0.0, 0.0};
  double* Hrow = L.H + (long long)i * kRowStride;
  for (int s = lane; s < kSlots; s += 64) {
    for (int c = 0; c < 9; ++c) {
      double v = acc[c * kSlotPad + s];
      Hrow[c * kSlotPad + s] = v;
      if (s != kCenter) {
        double av = fabs(v);
        int g = c / 3;
        l1[0] += (g == 0) ? av : 0.0;
        l1[1] += (g == 1) ? av : 0.0;
        l1[2] += (g == 2) ? av : 0.0;
      }
    }
  }
  for (int g = 0; g < 3; ++g) l1[g] = wave_sum(l1[g]);
  if (lane == 0) {
    double Dt[9];
    for (int k = 0; k < 9; ++k) Dt[k] = acc[k * kSlotPad + kCenter];
    for (int g = 0; g < 3; ++g) Dt[4 * g] += l1[g];
    double Di[9];
    inv3(Dt, Di);
    for (int k = 0; k < 9; ++k) L.Dinv[(long long)i * 9 + k] = Di[k];
  }
}

}  // namespace hot
