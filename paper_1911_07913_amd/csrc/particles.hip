// Particle-grid kernels of the implicit MPM step (Sec. 3.1) and the level-0
// system matrix (Sec. 4.1, Alg. HOT initialisation).
//
// All transfers are written as gathers over the binned particle order, so no
// floating-point atomics are used: a node sums the particles of the 27 base
// cells whose stencil covers it, in a fixed order.
#include "mpm_math.h"

namespace hot {
namespace {

constexpr int kTpb = 256;
inline unsigned blocks_for(long long n, int tpb = kTpb) {
  return (unsigned)((n + tpb - 1) / tpb);
}

__device__ inline long long stencil_offset(const GridGeom& g, int k) {
  // offset of stencil node k (x fastest) relative to the base node
  return (long long)(k % 3) + (long long)g.pd[0] * ((long long)((k / 3) % 3) + (long long)g.pd[1] * (k / 9));
}

__global__ void k_frac(SceneDev s, int n, const double* __restrict__ x, double* __restrict__ f,
                       int* __restrict__ key) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int b[3];
  for (int a = 0; a < 3; ++a) {
    double t = (x[3 * p + a] - s.origin[a]) / s.dx;
    double fb = floor(t - 0.5);
    b[a] = (int)fb;
    f[3 * p + a] = t - fb;
  }
  key[p] = (int)pidx(s.g0, b[0], b[1], b[2]);
}

// Boundary conditions at node coordinates (x, y, z), evaluated at t_end.
__device__ inline bool apply_bcs(const SceneDev& s, int x, int y, int z, double t_end, double* v) {
  bool fixed = false;
  int c[3] = {x, y, z};
  double xi[3] = {s.origin[0] + x * s.dx, s.origin[1] + y * s.dx, s.origin[2] + z * s.dx};
  for (int k = 0; k < s.n_bcs; ++k) {
    const BcDev& bc = s.bcs[k];
    if (bc.kind == 0) {
      int th = (int)bc.p[0];
      bool sel = false;
      for (int a = 0; a < 3; ++a) sel = sel || (c[a] <= th) || (c[a] >= s.cells[a] - th);
      if (sel) {
        fixed = true;
        v[0] = v[1] = v[2] = 0.0;
      }
    } else if (bc.kind == 1) {
      bool sel = true;
      for (int a = 0; a < 3; ++a) sel = sel && (xi[a] >= bc.p[a]) && (xi[a] <= bc.p[3 + a]);
      if (sel) {
        double ax = bc.p[9], ay = bc.p[10], az = bc.p[11];
        double nrm = sqrt(ax * ax + ay * ay + az * az);
        ax /= nrm; ay /= nrm; az /= nrm;
        double d0 = xi[0] - bc.p[6], d1 = xi[1] - bc.p[7], d2 = xi[2] - bc.p[8];
        double w = bc.p[12];
        v[0] = w * (ay * d2 - az * d1);
        v[1] = w * (az * d0 - ax * d2);
        v[2] = w * (ax * d1 - ay * d0);
        fixed = true;
      }
    } else if (bc.kind == 2) {
      double r2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        double d = xi[a] - (bc.p[a] + bc.p[4 + a] * t_end);
        r2 += d * d;
      }
      if (r2 <= bc.p[3] * bc.p[3]) {
        fixed = true;
        v[0] = bc.p[4]; v[1] = bc.p[5]; v[2] = bc.p[6];
      }
    }
  }
  return fixed;
}

// APIC particle-to-grid (Sec. 3.1) plus the mass-weighted CN stiffness field
// (Sec. 5.2), gravity and boundary velocities.  One thread per active node.
__global__ void k_p2g(SceneDev s, LevelView L, const double* __restrict__ f,
                      const double* __restrict__ v, const double* __restrict__ C,
                      const double* __restrict__ vol, const int* __restrict__ mat,
                      const int* __restrict__ cstart, const int* __restrict__ ccount, double dt,
                      double t_end, double* __restrict__ mass, double* __restrict__ vstar,
                      double* __restrict__ xi, int* __restrict__ fixed) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  int x, y, z;
  unpidx(L.g, L.nodes[i], x, y, z);
  double m = 0.0, mv0 = 0.0, mv1 = 0.0, mv2 = 0.0, mxi = 0.0;
  for (int k = 0; k < 27; ++k) {
    int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
    long long cell = pidx(L.g, x - kx, y - ky, z - kz);
    int cnt = ccount[cell];
    if (cnt == 0) continue;
    int st = cstart[cell];
    for (int p = st; p < st + cnt; ++p) {
      double f0 = f[3 * p], f1 = f[3 * p + 1], f2 = f[3 * p + 2];
      double w = bsw(kx, f0) * bsw(ky, f1) * bsw(kz, f2);
      const MaterialDev& md = s.mats[mat[p]];
      double mp = md.density * vol[p];
      double d0 = (kx - f0) * s.dx, d1 = (ky - f1) * s.dx, d2 = (kz - f2) * s.dx;
      const double* Cp = C + 9 * p;
      double va0 = v[3 * p] + (Cp[0] * d0 + Cp[1] * d1 + Cp[2] * d2);
      double va1 = v[3 * p + 1] + (Cp[3] * d0 + Cp[4] * d1 + Cp[5] * d2);
      double va2 = v[3 * p + 2] + (Cp[6] * d0 + Cp[7] * d1 + Cp[8] * d2);
      double wm = w * mp;
      m += wm;
      mv0 += wm * va0;
      mv1 += wm * va1;
      mv2 += wm * va2;
      mxi += wm * md.xi;
    }
  }
  double vs[3];
  if (m > 0.0) {
    vs[0] = mv0 / m + dt * s.gravity[0];
    vs[1] = mv1 / m + dt * s.gravity[1];
    vs[2] = mv2 / m + dt * s.gravity[2];
    xi[i] = mxi / m;
  } else {
    vs[0] = vs[1] = vs[2] = 0.0;
    xi[i] = 0.0;
  }
  bool fx = apply_bcs(s, x, y, z, t_end, vs);
  mass[i] = m;
  fixed[i] = fx ? 1 : 0;
  for (int a = 0; a < 3; ++a) vstar[3 * i + a] = vs[a];
}

// F_p(dv) = (I + dt sum_i v_i grad w_ip^T) F_p^n with v_i = v*_i + dv_i + alpha p_i.
__device__ inline void particle_F(const SceneDev& s, const LevelView& L, int pidx_key,
                                  const double* fp, const double* Fn, const double* vstar,
                                  const double* dv, const double* pdir, double alpha, double dt,
                                  double* F) {
  Weights W;
  bspline_weights(fp, s.inv_dx, W);
  double gv[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = 0; k < 27; ++k) {
    int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
    int j = L.map[pidx_key + stencil_offset(L.g, k)];
    double g[3];
    node_grad(W, kx, ky, kz, g);
    double vel[3];
    for (int a = 0; a < 3; ++a) {
      double d = 0.0;
      if (dv) {
        d = dv[3 * j + a];
        if (pdir) d = d + alpha * pdir[3 * j + a];
      }
      vel[a] = vstar[3 * j + a] + d;
    }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) gv[3 * a + b] += vel[a] * g[b];
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int q = 0; q < 3; ++q) {
        double Aq = ((r == q) ? 1.0 : 0.0) + dt * gv[3 * r + q];
        acc += Aq * Fn[3 * q + c];
      }
      F[3 * r + c] = acc;
    }
}

// Per-particle projected stress derivative at dv = 0, scaled by dt^2 V_p
// (the particle's contribution to the level-0 Hessian, Alg. HOT
// projectHessian).  45 upper-triangle entries per particle.
__global__ void k_particle_hessian(SceneDev s, LevelView L, int n, const double* __restrict__ f,
                                   const int* __restrict__ key, const double* __restrict__ Fn,
                                   const double* __restrict__ vol, const int* __restrict__ mat,
                                   const double* __restrict__ vstar, double dt,
                                   double* __restrict__ Cp) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double F[9], fn[9];
  for (int i = 0; i < 9; ++i) fn[i] = Fn[9 * p + i];
  particle_F(s, L, key[p], f + 3 * p, fn, vstar, nullptr, nullptr, 0.0, dt, F);
  double C45[45];
  projected_dPdF(s.mats[mat[p]], F, dt * dt * vol[p], C45);
  for (int i = 0; i < 45; ++i) Cp[45 * (long long)p + i] = C45[i];
}

// Energy density and stress at the trial point: psi_out[p] = V_p psi(F_p),
// S_out[p] = V_p P(F_p) F_p^n^T (the particle's force tensor, Sec. 4.1).
__global__ void k_particle_eval(SceneDev s, LevelView L, int n, const double* __restrict__ f,
                                const int* __restrict__ key, const double* __restrict__ Fn,
                                const double* __restrict__ vol, const int* __restrict__ mat,
                                const double* __restrict__ vstar, const double* __restrict__ dv,
                                const double* __restrict__ pdir, double alpha, double dt,
                                double* __restrict__ psi_out, double* __restrict__ S_out) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double F[9], fn[9];
  for (int i = 0; i < 9; ++i) fn[i] = Fn[9 * p + i];
  particle_F(s, L, key[p], f + 3 * p, fn, vstar, dv, pdir, alpha, dt, F);
  double P[9];
  double ps = psi_and_piola(s.mats[mat[p]], F, P);
  double V = vol[p];
  psi_out[p] = V * ps;
  if (S_out) {
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int q = 0; q < 3; ++q) acc += P[3 * r + q] * fn[3 * c + q];
        S_out[9 * (long long)p + 3 * r + c] = V * acc;
      }
  }
}

// g_i = m_i dv_i + dt sum_p S_p grad w_ip, zero on constrained nodes
// (Sec. 4.1 nodal forces; gradient of Eq. 1).  One thread per node.
__global__ void k_gradient(SceneDev s, LevelView L, const double* __restrict__ f,
                           const double* __restrict__ S, const int* __restrict__ cstart,
                           const int* __restrict__ ccount, const double* __restrict__ mass,
                           const int* __restrict__ fixed, const double* __restrict__ dv, double dt,
                           double* __restrict__ g) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  if (fixed[i]) {
    g[3 * i] = g[3 * i + 1] = g[3 * i + 2] = 0.0;
    return;
  }
  int x, y, z;
  unpidx(L.g, L.nodes[i], x, y, z);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int k = 0; k < 27; ++k) {
    int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
    long long cell = pidx(L.g, x - kx, y - ky, z - kz);
    int cnt = ccount[cell];
    if (cnt == 0) continue;
    int st = cstart[cell];
    for (int p = st; p < st + cnt; ++p) {
      double f0 = f[3 * p], f1 = f[3 * p + 1], f2 = f[3 * p + 2];
      double wx = bsw(kx, f0), wy = bsw(ky, f1), wz = bsw(kz, f2);
      double gx = bsdw(kx, f0, s.inv_dx) * wy * wz;
      double gy = wx * bsdw(ky, f1, s.inv_dx) * wz;
      double gz = wx * wy * bsdw(kz, f2, s.inv_dx);
      const double* Sp = S + 9 * (long long)p;
      a0 += Sp[0] * gx + Sp[1] * gy + Sp[2] * gz;
      a1 += Sp[3] * gx + Sp[4] * gy + Sp[5] * gz;
      a2 += Sp[6] * gx + Sp[7] * gy + Sp[8] * gz;
    }
  }
  double m = mass[i];
  g[3 * i] = m * dv[3 * i] + dt * a0;
  g[3 * i + 1] = m * dv[3 * i + 1] + dt * a1;
  g[3 * i + 2] = m * dv[3 * i + 2] + dt * a2;
}

// Von Mises return mapping on the Hencky strain (lagged plasticity).
__device__ inline void von_mises(double* F, double mu, double ys) {
  double U[9], s[3], V[9];
  svd3(F, U, s, V);
  double e[3], sg[3];
  for (int a = 0; a < 3; ++a) {
    sg[a] = (s[a] < 0.0) ? -1.0 : 1.0;
    e[a] = log(fabs(s[a]));
  }
  double mean = (e[0] + e[1] + e[2]) / 3.0;
  double d[3] = {e[0] - mean, e[1] - mean, e[2] - mean};
  double nd = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double lim = sqrt(2.0 / 3.0) * ys / (2.0 * mu);
  if (!(nd > lim)) return;
  double sc = lim / nd;
  double sn[3];
  for (int a = 0; a < 3; ++a) sn[a] = sg[a] * exp(mean + d[a] * sc);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      F[3 * r + c] = U[3 * r] * sn[0] * V[3 * c] + U[3 * r + 1] * sn[1] * V[3 * c + 1] +
                     U[3 * r + 2] * sn[2] * V[3 * c + 2];
}

// Grid-to-particle APIC transfer, deformation update, lagged plasticity and
// advection (Sec. 3.1).
__global__ void k_g2p(SceneDev s, LevelView L, int n, const double* __restrict__ f,
                      const int* __restrict__ key, double* __restrict__ x,
                      double* __restrict__ v, double* __restrict__ C, double* __restrict__ Fn,
                      const int* __restrict__ mat, const double* __restrict__ vstar,
                      const double* __restrict__ dv, double dt) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double fp[3] = {f[3 * p], f[3 * p + 1], f[3 * p + 2]};
  Weights W;
  bspline_weights(fp, s.inv_dx, W);
  double vp[3] = {0, 0, 0}, B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, gv[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  int kp = key[p];
  for (int k = 0; k < 27; ++k) {
    int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
    int j = L.map[kp + stencil_offset(L.g, k)];
    double vel[3];
    for (int a = 0; a < 3; ++a) vel[a] = vstar[3 * j + a] + dv[3 * j + a];
    double w = node_weight(W, kx, ky, kz);
    double g[3];
    node_grad(W, kx, ky, kz, g);
    double d[3] = {(kx - fp[0]) * s.dx, (ky - fp[1]) * s.dx, (kz - fp[2]) * s.dx};
    for (int a = 0; a < 3; ++a) {
      vp[a] += w * vel[a];
      for (int b = 0; b < 3; ++b) {
        B[3 * a + b] += w * vel[a] * d[b];
        gv[3 * a + b] += vel[a] * g[b];
      }
    }
  }
  double fn[9], F[9];
  for (int i = 0; i < 9; ++i) fn[i] = Fn[9 * (long long)p + i];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int q = 0; q < 3; ++q) acc += (((r == q) ? 1.0 : 0.0) + dt * gv[3 * r + q]) * fn[3 * q + c];
      F[3 * r + c] = acc;
    }
  const MaterialDev& md = s.mats[mat[p]];
  if (md.yield > 0.0) von_mises(F, md.mu, md.yield);
  double cs = 4.0 / (s.dx * s.dx);
  for (int i = 0; i < 9; ++i) {
    Fn[9 * (long long)p + i] = F[i];
    C[9 * (long long)p + i] = cs * B[i];
  }
  for (int a = 0; a < 3; ++a) {
    v[3 * p + a] = vp[a];
    x[3 * p + a] += dt * vp[a];
  }
}

// Level-0 Hessian rows, one wave per row i (Sec. 4.1 / Alg. HOT):
//   H_ij = m_i delta_ij I + sum_p a_ip^T C_p a_jp,  a_ip = F_p^n^T grad w_ip,
// with C_p the particle's projected stress derivative already scaled by
// dt^2 V_p.  The particles touching row i are those of the 27 base cells
// b = i - k, k in {0,1,2}^3; all particles of one cell share the stencil
// b + {0,1,2}^3, so lane l (0..26) accumulates block (i, b + l) in registers
// while the two half-waves take alternate particles, and the per-cell sums
// are added into the row held in LDS.  The row is then finalised (mass,
// Dirichlet projection, smoother inverse) and written once.
constexpr int kAsmWaves = 4;

__global__ __launch_bounds__(256) void k_assemble_h0(SceneDev s, LevelView L,
                                                      const double* __restrict__ f,
                                                      const double* __restrict__ Fn,
                                                      const double* __restrict__ Cp,
                                                      const int* __restrict__ cstart,
                                                      const int* __restrict__ ccount,
                                                      const double* __restrict__ mass,
                                                      const int* __restrict__ fixed) {
  __shared__ double acc_all[kAsmWaves][kRowVals];
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int i = blockIdx.x * kAsmWaves + wave;
  if (i >= L.n) return;
  double* acc = acc_all[wave];
  for (int e = lane; e < kRowVals; e += 64) acc[e] = 0.0;
  wave_sync();
  int x, y, z;
  unpidx(L.g, L.nodes[i], x, y, z);
  const int half = lane >> 5, l = lane & 31;
  const bool lane_ok = l < 27;
  const int lx = l % 3, ly = (l / 3) % 3, lz = l / 9;
  // Z entry owned by this lane: e = 9*gamma + (3*delta + eps)
  const int zg = l / 9, zde = l % 9;
  for (int k = 0; k < 27; ++k) {
    int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
    long long cell = pidx(L.g, x - kx, y - ky, z - kz);
    int cnt = ccount[cell];
    if (cnt == 0) continue;
    int st = cstart[cell];
    double blk[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int t = 0; t < cnt; t += 2) {
      int pi = t + half;
      bool valid = pi < cnt;
      long long p = st + (valid ? pi : 0);
      double fp[3] = {f[3 * p], f[3 * p + 1], f[3 * p + 2]};
      Weights W;
      bspline_weights(fp, s.inv_dx, W);
      double gi[3], gl[3];
      node_grad(W, kx, ky, kz, gi);
      node_grad(W, lx < 3 ? lx : 0, ly, lz < 3 ? lz : 0, gl);
      const double* F = Fn + 9 * p;
      double ai[3], al[3];
      for (int b = 0; b < 3; ++b) {
        ai[b] = F[b] * gi[0] + F[3 + b] * gi[1] + F[6 + b] * gi[2];
        al[b] = (valid && lane_ok) ? (F[b] * gl[0] + F[3 + b] * gl[1] + F[6 + b] * gl[2]) : 0.0;
      }
      double zv = 0.0;
      if (lane_ok) {
        const double* Cq = Cp + 45 * p;
        for (int b = 0; b < 3; ++b) zv += ai[b] * Cq[tri9(3 * zg + b, zde)];
      }
      const int src0 = half << 5;
#pragma unroll
      for (int g = 0; g < 3; ++g)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          double sacc = 0.0;
#pragma unroll
          for (int e = 0; e < 3; ++e) sacc += __shfl(zv, src0 + 9 * g + 3 * d + e, 64) * al[e];
          blk[3 * g + d] += sacc;
        }
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) blk[c] += __shfl_down(blk[c], 32, 64);
    if (lane < 27) {
      int sl = (lx - kx + 2) + 5 * (ly - ky + 2) + 25 * (lz - kz + 2);
      for (int c = 0; c < 9; ++c) acc[sl * 9 + c] += blk[c];
    }
    wave_sync();
  }
  finalize_row(acc, i, L, fixed, mass[i], lane);
}

}  // namespace

void launch_particle_frac(const SceneDev& s, int n, const double* x, double* f, int* key,
                          hipStream_t st) {
  if (n > 0) k_frac<<<blocks_for(n), kTpb, 0, st>>>(s, n, x, f, key);
}

void launch_p2g(const SceneDev& s, const LevelView& L0, const double* f, const double* v,
                const double* C, const double* vol, const int* mat, const int* cstart,
                const int* ccount, double dt, double t_end, double* mass, double* vstar,
                double* xi, int* fixed, hipStream_t st) {
  if (L0.n > 0)
    k_p2g<<<blocks_for(L0.n), kTpb, 0, st>>>(s, L0, f, v, C, vol, mat, cstart, ccount, dt, t_end,
                                             mass, vstar, xi, fixed);
}

void launch_particle_hessian(const SceneDev& s, const LevelView& L0, int n, const double* f,
                             const int* key, const double* F, const double* vol, const int* mat,
                             const double* vstar, double dt, double* Cp, hipStream_t st) {
  if (n > 0)
    k_particle_hessian<<<blocks_for(n), kTpb, 0, st>>>(s, L0, n, f, key, F, vol, mat, vstar, dt,
                                                       Cp);
}

void launch_particle_eval(const SceneDev& s, const LevelView& L0, int n, const double* f,
                          const int* key, const double* F, const double* vol, const int* mat,
                          const double* vstar, const double* dv, const double* p, double alpha,
                          double dt, double* psi_out, double* S_out, hipStream_t st) {
  if (n > 0)
    k_particle_eval<<<blocks_for(n), kTpb, 0, st>>>(s, L0, n, f, key, F, vol, mat, vstar, dv, p,
                                                    alpha, dt, psi_out, S_out);
}

void launch_gradient(const SceneDev& s, const LevelView& L0, const double* f, const double* S,
                     const int* cstart, const int* ccount, const double* mass, const int* fixed,
                     const double* dv, double dt, double* g, hipStream_t st) {
  if (L0.n > 0)
    k_gradient<<<blocks_for(L0.n), kTpb, 0, st>>>(s, L0, f, S, cstart, ccount, mass, fixed, dv,
                                                  dt, g);
}

void launch_g2p(const SceneDev& s, const LevelView& L0, int n, const double* f, const int* key,
                double* x, double* v, double* C, double* F, const int* mat, const double* vstar,
                const double* dv, double dt, hipStream_t st) {
  if (n > 0)
    k_g2p<<<blocks_for(n), kTpb, 0, st>>>(s, L0, n, f, key, x, v, C, F, mat, vstar, dv, dt);
}

void launch_assemble_h0(const SceneDev& s, const LevelView& L0, const double* f, const double* F,
                        const double* Cp, const int* cstart, const int* ccount,
                        const double* mass, const int* fixed, hipStream_t st) {
  if (L0.n > 0)
    k_assemble_h0<<<(unsigned)((L0.n + kAsmWaves - 1) / kAsmWaves), 256, 0, st>>>(
        s, L0, f, F, Cp, cstart, ccount, mass, fixed);
}

}  // namespace hot
