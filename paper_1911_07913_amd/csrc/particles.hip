// Particle-grid kernels of the implicit MPM step (Sec. 3.1) and the level-0
// system matrix (Sec. 4.1, Alg. HOT initialisation).
//
// Particle-to-node sums are computed without global floating-point atomics
// and in a fixed order (see the brick and row-segment kernels below), so the
// results are reproducible run to run.
#include "mpm_math.h"

typedef double v4d __attribute__((ext_vector_type(4)));

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

// ---- two-pass particle-to-node sums over cell bricks
// Pass 1: one wave per brick of 4^3 cells; lane l owns one cell and walks its
// particles, adding each particle's contribution to the 27 stencil nodes of
// its cell into the brick's 6^3-node window in LDS.  For a fixed stencil
// offset the 64 cells hit 64 distinct nodes, so no two lanes of one LDS add
// collide; the adds are LDS atomics so the one wave's instructions apply in
// program order and the sums are reproducible.  The window is written to a
// per-brick partial.
// Pass 2: every node sums the partials of the (at most 8) bricks whose window
// holds it, in a fixed order.  No floating-point atomics; deterministic.
// Lane `lane` of brick b owns cell (lx, ly, lz) of the brick; returns its
// particle range [st, st + cnt) in the binned order.
__device__ inline void brick_cell(const SceneDev& s, const Bricks& B, int b, int lane,
                                  const int* __restrict__ cstart, const int* __restrict__ ccount,
                                  int& cnt, int& st, int& lx, int& ly, int& lz) {
  int bid = B.list[b];
  int bx = bid % B.bg.bd[0], by = (bid / B.bg.bd[0]) % B.bg.bd[1], bz = bid / (B.bg.bd[0] * B.bg.bd[1]);
  lx = lane % kBrick;
  ly = (lane / kBrick) % kBrick;
  lz = lane / (kBrick * kBrick);
  int cx = bx * kBrick + lx, cy = by * kBrick + ly, cz = bz * kBrick + lz;  // padded cell coords
  cnt = 0;
  st = 0;
  if (cx < s.g0.pd[0] && cy < s.g0.pd[1] && cz < s.g0.pd[2]) {
    long long c = (long long)cx + (long long)s.g0.pd[0] * ((long long)cy + (long long)s.g0.pd[1] * cz);
    cnt = ccount[c];
    st = cstart[c];
  }
}

// Sum over the bricks whose node window holds padded node (px, py, pz).
template <int V>
__device__ inline void brick_gather(const Bricks& B, const double* __restrict__ partial, int px,
                                    int py, int pz, double* out) {
  for (int v = 0; v < V; ++v) out[v] = 0.0;
  int lo[3], hi[3], pp[3] = {px, py, pz};
  for (int a = 0; a < 3; ++a) {
    lo[a] = pp[a] >= kBrickNodes - 1 ? (pp[a] - (kBrickNodes - 1) + kBrick - 1) / kBrick : 0;
    hi[a] = min(pp[a] / kBrick, B.bg.bd[a] - 1);
  }
  for (int bz = lo[2]; bz <= hi[2]; ++bz)
    for (int by = lo[1]; by <= hi[1]; ++by)
      for (int bx = lo[0]; bx <= hi[0]; ++bx) {
        int id = B.map[bx + (long long)B.bg.bd[0] * (by + (long long)B.bg.bd[1] * bz)];
        if (id < 0) continue;
        int loc = (px - bx * kBrick) + kBrickNodes * ((py - by * kBrick) + kBrickNodes * (pz - bz * kBrick));
        const double* q = partial + ((long long)id * kBrickWin + loc) * V;
        for (int v = 0; v < V; ++v) out[v] += q[v];
      }
}

// APIC particle-to-grid (Sec. 3.1) plus the mass-weighted CN stiffness field
// (Sec. 5.2), pass 1: per brick, m w, m w (v_p + C_p (x_i - x_p)), m w xi_p.
__global__ __launch_bounds__(64) void k_p2g_brick(SceneDev s, Bricks B, const double* __restrict__ f,
                                                  const double* __restrict__ v,
                                                  const double* __restrict__ C,
                                                  const double* __restrict__ vol,
                                                  const int* __restrict__ mat,
                                                  const int* __restrict__ cstart,
                                                  const int* __restrict__ ccount,
                                                  double* __restrict__ partial) {
  __shared__ double win[kBrickWin * 5];
  const int b = blockIdx.x, lane = threadIdx.x;
  for (int e = lane; e < kBrickWin * 5; e += 64) win[e] = 0.0;
  int cnt, st, lx, ly, lz;
  brick_cell(s, B, b, lane, cstart, ccount, cnt, st, lx, ly, lz);
  wave_sync();
  for (int t = 0;; ++t) {
    bool act = t < cnt;
    if (!__any(act)) break;
    if (act) {
      int p = st + t;
      double f0 = f[3 * p], f1 = f[3 * p + 1], f2 = f[3 * p + 2];
      double wx[3], wy[3], wz[3];
      for (int k = 0; k < 3; ++k) {
        wx[k] = bsw(k, f0);
        wy[k] = bsw(k, f1);
        wz[k] = bsw(k, f2);
      }
      const MaterialDev& md = s.mats[mat[p]];
      double mp = md.density * vol[p], xip = md.xi;
      double vp0 = v[3 * p], vp1 = v[3 * p + 1], vp2 = v[3 * p + 2];
      const double* Cp = C + 9 * (long long)p;
      double c0 = Cp[0], c1 = Cp[1], c2 = Cp[2], c3 = Cp[3], c4 = Cp[4], c5 = Cp[5], c6 = Cp[6],
             c7 = Cp[7], c8 = Cp[8];
#pragma unroll
      for (int k = 0; k < 27; ++k) {
        const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
        double w = wx[kx] * wy[ky] * wz[kz];
        double d0 = (kx - f0) * s.dx, d1 = (ky - f1) * s.dx, d2 = (kz - f2) * s.dx;
        double va0 = vp0 + (c0 * d0 + c1 * d1 + c2 * d2);
        double va1 = vp1 + (c3 * d0 + c4 * d1 + c5 * d2);
        double va2 = vp2 + (c6 * d0 + c7 * d1 + c8 * d2);
        double wm = w * mp;
        double* q = win + 5 * ((lx + kx) + kBrickNodes * ((ly + ky) + kBrickNodes * (lz + kz)));
        atomicAdd(q, wm);
        atomicAdd(q + 1, wm * va0);
        atomicAdd(q + 2, wm * va1);
        atomicAdd(q + 3, wm * va2);
        atomicAdd(q + 4, wm * xip);
      }
    }
  }
  wave_sync();
  double* out = partial + (long long)b * kBrickWin * 5;
  for (int e = lane; e < kBrickWin * 5; e += 64) out[e] = win[e];
}

// P2G pass 2: velocities, CN field, gravity and boundary velocities.
__global__ void k_p2g_nodes(SceneDev s, LevelView L, Bricks B, const double* __restrict__ partial,
                            double dt, double t_end, double* __restrict__ mass,
                            double* __restrict__ vstar, double* __restrict__ xi,
                            int* __restrict__ fixed) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  int x, y, z;
  unpidx(L.g, L.nodes[i], x, y, z);
  double q[5];
  brick_gather<5>(B, partial, x + 2, y + 2, z + 2, q);
  double m = q[0];
  double vs[3];
  if (m > 0.0) {
    vs[0] = q[1] / m + dt * s.gravity[0];
    vs[1] = q[2] / m + dt * s.gravity[1];
    vs[2] = q[3] / m + dt * s.gravity[2];
    xi[i] = q[4] / m;
  } else {
    vs[0] = vs[1] = vs[2] = 0.0;
    xi[i] = 0.0;
  }
  bool fx = apply_bcs(s, x, y, z, t_end, vs);
  mass[i] = m;
  fixed[i] = fx ? 1 : 0;
  for (int a = 0; a < 3; ++a) vstar[3 * i + a] = vs[a];
}

// Node velocities of a trial point, v_i = v*_i + dv_i + alpha p_i (dv, p
// optional), written at each active node's padded index.
__global__ void k_node_vel(LevelView L, const double* __restrict__ vstar,
                           const double* __restrict__ dv, const double* __restrict__ pdir,
                           double alpha, double4* __restrict__ wn) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  double vel[3];
  for (int a = 0; a < 3; ++a) {
    double d = 0.0;
    if (dv) {
      d = dv[3 * i + a];
      if (pdir) d = d + alpha * pdir[3 * i + a];
    }
    vel[a] = vstar[3 * i + a] + d;
  }
  wn[L.nodes[i]] = make_double4(vel[0], vel[1], vel[2], 0.0);
}

// F_p(dv) = (I + dt sum_i v_i grad w_ip^T) F_p^n with v_i from k_node_vel.
__device__ inline void particle_F(const SceneDev& s, const LevelView& L, int pidx_key,
                                  const double* fp, const double* Fn,
                                  const double4* __restrict__ wn, double dt, double* F) {
  Weights W;
  bspline_weights(fp, s.inv_dx, W);
  double gv[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < 27; ++k) {
    const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
    const double4 wv = wn[pidx_key + stencil_offset(L.g, k)];
    double g[3];
    node_grad(W, kx, ky, kz, g);
    const double vel[3] = {wv.x, wv.y, wv.z};
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
__global__ __launch_bounds__(256) void k_particle_hessian(SceneDev s, LevelView L, int n, const double* __restrict__ f,
                                   const int* __restrict__ key, const double* __restrict__ Fn,
                                   const double* __restrict__ vol, const int* __restrict__ mat,
                                   const double4* __restrict__ wn, double dt,
                                   double* __restrict__ Cp) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double F[9], fn[9];
  for (int i = 0; i < 9; ++i) fn[i] = Fn[9 * p + i];
  particle_F(s, L, key[p], f + 3 * p, fn, wn, dt, F);
  double C45[45];
  projected_dPdF(s.mats[mat[p]], F, dt * dt * vol[p], C45);
  for (int i = 0; i < 45; ++i) Cp[45 * (long long)p + i] = C45[i];
}

// Energy density and stress at the trial point: psi_out[p] = V_p psi(F_p),
// S_out[p] = V_p P(F_p) F_p^n^T (the particle's force tensor, Sec. 4.1).
__global__ __launch_bounds__(256) void k_particle_eval(SceneDev s, LevelView L, int n, const double* __restrict__ f,
                                const int* __restrict__ key, const double* __restrict__ Fn,
                                const double* __restrict__ vol, const int* __restrict__ mat,
                                const double4* __restrict__ wn, double dt,
                                double* __restrict__ psi_out, double* __restrict__ S_out) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double F[9], fn[9];
  for (int i = 0; i < 9; ++i) fn[i] = Fn[9 * p + i];
  particle_F(s, L, key[p], f + 3 * p, fn, wn, dt, F);
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

// Gradient pass 1 (Sec. 4.1 nodal forces): per brick, sum_p S_p grad w_ip
// with S_p = V_p P(F_p) F_p^n^T.  kGradWaves waves share a brick: wave w
// walks the particles t = w, w + kGradWaves, ... of every cell into a window
// of its own (the pass-1 rule above holds per wave), and the windows are
// summed in wave order, so the result stays reproducible.
constexpr int kGradWaves = 4;

__global__ __launch_bounds__(64 * kGradWaves) void k_grad_brick(SceneDev s, Bricks B,
                                                                const double* __restrict__ f,
                                                                const double* __restrict__ S,
                                                                const int* __restrict__ cstart,
                                                                const int* __restrict__ ccount,
                                                                double* __restrict__ partial) {
  __shared__ double win[kGradWaves][kBrickWin * 3];
  const int b = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int e = tid; e < kGradWaves * kBrickWin * 3; e += 64 * kGradWaves) (&win[0][0])[e] = 0.0;
  int cnt, st, lx, ly, lz;
  brick_cell(s, B, b, lane, cstart, ccount, cnt, st, lx, ly, lz);
  __syncthreads();
  double* wv = win[wave];
  for (int t = wave;; t += kGradWaves) {
    bool act = t < cnt;
    if (!__any(act)) break;
    if (act) {
      long long p = st + t;
      double f0 = f[3 * p], f1 = f[3 * p + 1], f2 = f[3 * p + 2];
      double wx[3], wy[3], wz[3], dx[3], dy[3], dz[3];
      for (int k = 0; k < 3; ++k) {
        wx[k] = bsw(k, f0);
        wy[k] = bsw(k, f1);
        wz[k] = bsw(k, f2);
        dx[k] = bsdw(k, f0, s.inv_dx);
        dy[k] = bsdw(k, f1, s.inv_dx);
        dz[k] = bsdw(k, f2, s.inv_dx);
      }
      const double* Sp = S + 9 * p;
      double s0 = Sp[0], s1 = Sp[1], s2 = Sp[2], s3 = Sp[3], s4 = Sp[4], s5 = Sp[5], s6 = Sp[6],
             s7 = Sp[7], s8 = Sp[8];
#pragma unroll
      for (int k = 0; k < 27; ++k) {
        const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
        double gx = dx[kx] * wy[ky] * wz[kz];
        double gy = wx[kx] * dy[ky] * wz[kz];
        double gz = wx[kx] * wy[ky] * dz[kz];
        double* q = wv + 3 * ((lx + kx) + kBrickNodes * ((ly + ky) + kBrickNodes * (lz + kz)));
        atomicAdd(q, s0 * gx + s1 * gy + s2 * gz);
        atomicAdd(q + 1, s3 * gx + s4 * gy + s5 * gz);
        atomicAdd(q + 2, s6 * gx + s7 * gy + s8 * gz);
      }
    }
  }
  __syncthreads();
  double* out = partial + (long long)b * kBrickWin * 3;
  for (int e = tid; e < kBrickWin * 3; e += 64 * kGradWaves) {
    double acc = win[0][e];
#pragma unroll
    for (int w = 1; w < kGradWaves; ++w) acc += win[w][e];
    out[e] = acc;
  }
}

// Gradient pass 2: g_i = m_i dv_i + dt sum, zero on constrained nodes.
__global__ void k_grad_nodes(LevelView L, Bricks B, const double* __restrict__ partial,
                             const double* __restrict__ mass, const int* __restrict__ fixed,
                             const double* __restrict__ dv, double dt, double* __restrict__ g) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  if (fixed[i]) {
    g[3 * i] = g[3 * i + 1] = g[3 * i + 2] = 0.0;
    return;
  }
  int x, y, z;
  unpidx(L.g, L.nodes[i], x, y, z);
  double q[3];
  brick_gather<3>(B, partial, x + 2, y + 2, z + 2, q);
  double m = mass[i];
  g[3 * i] = m * dv[3 * i] + dt * q[0];
  g[3 * i + 1] = m * dv[3 * i + 1] + dt * q[1];
  g[3 * i + 2] = m * dv[3 * i + 2] + dt * q[2];
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

// Snow-type plastic flow (Sec. 7, table of material parameters): the
// singular values of F clamped into [lo, hi], F = U clamp(S) V^T (signed SVD).
__device__ inline void snow_clamp(double* F, double lo, double hi) {
  double U[9], s[3], V[9];
  svd3(F, U, s, V);
  for (int a = 0; a < 3; ++a) s[a] = fmin(fmax(s[a], lo), hi);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      F[3 * r + c] = U[3 * r] * s[0] * V[3 * c] + U[3 * r + 1] * s[1] * V[3 * c + 1] +
                     U[3 * r + 2] * s[2] * V[3 * c + 2];
}

// Grid-to-particle APIC transfer, deformation update, lagged plasticity and
// advection (Sec. 3.1).
__global__ __launch_bounds__(256) void k_g2p(SceneDev s, LevelView L, int n, const double* __restrict__ f,
                      const int* __restrict__ key, double* __restrict__ x,
                      double* __restrict__ v, double* __restrict__ C, double* __restrict__ Fn,
                      const int* __restrict__ mat, const double4* __restrict__ wn, double dt) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double fp[3] = {f[3 * p], f[3 * p + 1], f[3 * p + 2]};
  Weights W;
  bspline_weights(fp, s.inv_dx, W);
  double vp[3] = {0, 0, 0}, B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, gv[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  int kp = key[p];
#pragma unroll
  for (int k = 0; k < 27; ++k) {
    const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
    const double4 wv = wn[kp + stencil_offset(L.g, k)];
    const double vel[3] = {wv.x, wv.y, wv.z};
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
  if (md.clamp_hi > 0.0) snow_clamp(F, md.clamp_lo, md.clamp_hi);
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

// Level-0 Hessian (Sec. 4.1 / Alg. HOT initialisation):
//   H_ij = m_i delta_ij I + sum_p a_ip^T C_p a_jp,  a_ip = F_p^n^T grad w_ip,
// with C_p the particle's projected stress derivative already scaled by
// dt^2 V_p (45 upper-triangle entries).
//
// One work-group per row segment: up to 16 consecutive rows (x, y, z) of one
// x-line.  The group sweeps the base cells c = x_first - 2 .. x_last of the 9
// cell columns (c, y - ky, z - kz), ky, kz in {0,1,2}; a particle of column
// (ky, kz) in cell c touches rows c + r, r in {0,1,2}, of this segment, with
// stencil offset k = (r, ky, kz).  For one cell column the blocks are a dense
// contraction over the column's particles p and the component eps:
//   B[(r, g, d)][l] = sum_(p, eps) Z_p[(r, g, d)][eps] a_p[l][eps],
// Z_p[(r, g, d)][eps] = sum_b a_p[k][b] C_p[3g + b][3d + eps] (k = (r, ky, kz)),
// a 27 x 27 x 3P product that the four waves compute as 2 x 2 tiles of FP64
// 16x16x4 matrix-core instructions, accumulating in registers over the
// column's particles; each lane forms its own Z operands from a_k and C_p in
// registers right before the matrix-core steps.  The a_l come precomputed
// (k_particle_agrad) and are staged with C_p as two contiguous ranges.  Per cell column the sums go
// to a 3-row sliding window in LDS.  After cell c, row c receives nothing
// more: it is finalised (mass, Dirichlet projection, smoother inverse) and
// written once.  Every block of every particle is computed exactly once; no
// atomics.  The kernel is bound by latency, not by a unit: LDS (under 40 KB)
// and registers (at most 128) are sized so that four work-groups share a
// compute unit.
constexpr int kAsmChunk = 8;   // particles staged per pass
constexpr int kPA = 81;        // a_l (27 x 3) per particle
constexpr int kPC = 45;        // C per particle
constexpr int kARegs = (kAsmChunk * kPA + 255) / 256;
constexpr int kCRegs = (kAsmChunk * kPC + 255) / 256;

__device__ inline void wdw(int k, double f, double inv_dx, double& w, double& dw) {
  double a = 1.5 - f, b = f - 1.0, c = f - 0.5;
  double w0 = 0.5 * (a * a), w1 = 0.75 - b * b, w2 = 0.5 * (c * c);
  double d0 = (f - 1.5) * inv_dx, d1 = -2.0 * b * inv_dx, d2 = c * inv_dx;
  w = (k == 0) ? w0 : ((k == 1) ? w1 : w2);
  dw = (k == 0) ? d0 : ((k == 1) ? d1 : d2);
}

// The assembly's right-hand operands a_lp = F_p^n^T grad w_lp for the 27
// stencil nodes l of every particle, [n][27][3], once per step (the assembly
// visits each particle from up to 9 x-lines).  One thread per (particle, node).
__global__ void k_particle_agrad(SceneDev s, long long n27, const double* __restrict__ f,
                                 const double* __restrict__ Fn, double* __restrict__ A) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n27) return;
  const long long p = e / 27;
  const int l = (int)(e - 27 * p);
  double w0, d0, w1, d1, w2, d2;
  wdw(l % 3, f[3 * p], s.inv_dx, w0, d0);
  wdw((l / 3) % 3, f[3 * p + 1], s.inv_dx, w1, d1);
  wdw(l / 9, f[3 * p + 2], s.inv_dx, w2, d2);
  double gx = d0 * w1 * w2, gy = w0 * d1 * w2, gz = w0 * w1 * d2;
  const double* F = Fn + 9 * p;
  double* o = A + 3 * e;
  o[0] = F[0] * gx + F[3] * gy + F[6] * gz;
  o[1] = F[1] * gx + F[4] * gy + F[7] * gz;
  o[2] = F[2] * gx + F[5] * gy + F[8] * gz;
}

// Entries (c, s) of a block row owned by one of 256 threads, decomposed once:
// LDS index, offset of the slot's neighbour in the segment's constrained-flag
// window (kNoNb for the diagonal slot), and block row g of off-diagonal slots
// (-1 for the diagonal slot and for unused items).
constexpr int kFinItems = (kBlock * kSlots + 255) / 256;
constexpr int kNoNb = -(1 << 30);
struct FinRoles {
  int idx[kFinItems];
  int nb[kFinItems];
  int g[kFinItems];
};

__device__ inline void fin_roles(int tid, int nxw, FinRoles& fr) {
#pragma unroll
  for (int k = 0; k < kFinItems; ++k) {
    const int e = tid + 256 * k;
    const int c = e / kSlots, sl = e - c * kSlots;
    const bool valid = e < kBlock * kSlots;
    fr.idx[k] = valid ? c * kSlotPad + sl : -1;
    const bool center = sl == kCenter;
    fr.nb[k] = (!valid || center) ? kNoNb
                                  : (sl % 5 - 2) + nxw * ((sl / 5) % 5 + 5 * (sl / 25));
    fr.g[k] = (!valid || center) ? -1 : c / 3;
  }
}

// Block-level finalisation of level-0 row i held in LDS (256 threads): mass
// on the diagonal, Dirichlet projection (constrained row -> m_i I, blocks to
// constrained neighbours -> 0), exact-zero diagonal rule, write-out, scalar
// diagonal and the l1 block-Jacobi inverse.  In mixed precision (L.Hb set)
// the BF16 blocks and FP32 copies of the diagonal and inverse are written
// here too, as the level conversion would.  nbf holds the constrained flags
// of the 5x5 y-z neighbourhood of the segment's x-line, x-major from xw0.
__device__ inline void finalize_row_block(double* acc, int i, int xi, int xw0,
                                          const LevelView& L, const uint8_t* nbf,
                                          const FinRoles& fr, bool row_fixed, double mass_i,
                                          double* red) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint8_t* nbx = nbf + (xi - xw0);
#pragma unroll
  for (int k = 0; k < kFinItems; ++k) {
    if (fr.idx[k] >= 0) {
      bool z = row_fixed || (fr.nb[k] != kNoNb && nbx[fr.nb[k]] != 0);
      if (z) acc[fr.idx[k]] = 0.0;
    }
  }
  __syncthreads();
  if (tid == 0) {
    for (int g = 0; g < 3; ++g) {
      double d = acc[(4 * g) * kSlotPad + kCenter] + mass_i;
      bool zero = (d == 0.0);
      acc[(4 * g) * kSlotPad + kCenter] = zero ? 1.0 : d;
      L.free_dof[3 * i + g] = (!row_fixed && !zero) ? 1 : 0;
      L.diag[3 * i + g] = zero ? 1.0 : d;
      if (L.Hb) L.diag32[3 * i + g] = (float)(zero ? 1.0 : d);
    }
  }
  __syncthreads();
  double l1[3] = {0.0, 0.0, 0.0};
  double* Hrow = L.H + (long long)i * kRowStride;
  uint16_t* Hbrow = L.Hb ? L.Hb + (long long)i * kRowStride : nullptr;
#pragma unroll
  for (int k = 0; k < kFinItems; ++k) {
    if (fr.idx[k] >= 0) {
      double v = acc[fr.idx[k]];
      Hrow[fr.idx[k]] = v;
      if (Hbrow) Hbrow[fr.idx[k]] = f32_to_bf16((float)v);
      const double av = fabs(v);
      l1[0] += (fr.g[k] == 0) ? av : 0.0;
      l1[1] += (fr.g[k] == 1) ? av : 0.0;
      l1[2] += (fr.g[k] == 2) ? av : 0.0;
    }
  }
  for (int g = 0; g < 3; ++g) {
    double t = wave_sum(l1[g]);
    if (lane == 0) red[wave * 3 + g] = t;
  }
  __syncthreads();
  if (tid == 0) {
    double Dt[9];
    for (int k = 0; k < 9; ++k) Dt[k] = acc[k * kSlotPad + kCenter];
    for (int g = 0; g < 3; ++g) Dt[4 * g] += red[g] + red[3 + g] + red[6 + g] + red[9 + g];
    double Di[9];
    inv3(Dt, Di);
    for (int k = 0; k < 9; ++k) L.Dinv[(long long)i * 9 + k] = Di[k];
    if (L.Hb)
      for (int k = 0; k < 9; ++k) L.Dinv32[(long long)i * 9 + k] = (float)Di[k];
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
void k_assemble_strip(SceneDev s, LevelView L, const int* __restrict__ seg_begin,
                      const double* __restrict__ Ag, const double* __restrict__ Cp,
                      const int* __restrict__ cstart,
                      const int* __restrict__ ccount, const double* __restrict__ mass,
                      const int* __restrict__ fixed) {
  constexpr int kMaxCx = kSegRows + 2;
  __shared__ double win[3][kRowStride];
  __shared__ double av[kAsmChunk][27][3];    // a_l of the staged particles
  __shared__ double pc[kAsmChunk][kPC];      // their C
  __shared__ double red[12];
  __shared__ int mcnt[kMaxCx * 9], mst[kMaxCx * 9];
  __shared__ int nextv[kMaxCx * 9 + 1];  // first non-empty column at or after v (-1: none)
  __shared__ uint8_t nbf[(kMaxCx + 2) * 25];
  __shared__ double rmass[kSegRows];
  __shared__ int rx[kSegRows];
  const int tid = threadIdx.x;
  const int seg = xcd_block(blockIdx.x, gridDim.x);
  const int rb = seg_begin[seg], re = seg_begin[seg + 1];
  int xa, ys, zs, xb, yy, zz;
  unpidx(L.g, L.nodes[rb], xa, ys, zs);
  unpidx(L.g, L.nodes[re - 1], xb, yy, zz);
  const int ncx = xb - xa + 3;
  // particle ranges of the 9 cell columns over the whole sweep, in one trip
  for (int v = tid; v < ncx * 9; v += 256) {
    int ci = v / 9, col = v - 9 * ci;
    long long cell = pidx(L.g, xa - 2 + ci, ys - col % 3, zs - col / 3);
    mcnt[v] = ccount[cell];
    mst[v] = cstart[cell];
  }
  // constrained flags of the rows' neighbourhood, the rows' masses and x
  const int xw0 = xa - 2, nxw = ncx + 2;
  for (int v = tid; v < nxw * 25; v += 256) {
    int xo = v % nxw, r = v / nxw;
    int j = L.map[pidx(L.g, xw0 + xo, ys + r % 5 - 2, zs + r / 5 - 2)];
    nbf[v] = (j >= 0 && fixed[j]) ? 1 : 0;
  }
  for (int v = tid; v < re - rb; v += 256) {
    int x0, y0, z0;
    unpidx(L.g, L.nodes[rb + v], x0, y0, z0);
    rx[v] = x0;
    rmass[v] = mass[rb + v];
  }
  for (int e = tid; e < 3 * kRowStride; e += 256) (&win[0][0])[e] = 0.0;
  __syncthreads();
  if (tid == 0) {
    int nx = -1;
    nextv[ncx * 9] = -1;
    for (int w = ncx * 9 - 1; w >= 0; --w) {
      if (mcnt[w] > 0) nx = w;
      nextv[w] = nx;
    }
  }
  // matrix-core roles: wave w owns output tile (rows 16 tile_m.., columns
  // 16 tile_n..) of the 27 x 27 product; lane l feeds A[l % 16][l / 16] and
  // B[l / 16][l % 16] and holds D[l / 16 + 4 v][l % 16], v = 0..3
  const int wave = tid >> 6, lane = tid & 63;
  const int tile_m = wave >> 1, tile_n = wave & 1;
  const int am = tile_m * 16 + (lane & 15);      // A row: (r, g, d)
  const bool am_ok = am < 27;
  const int amc = am_ok ? am : 0;                // clamped for addressing
  const int am_r = amc / 9, am_g = (amc % 9) / 3, am_d = amc % 3;
  const int bn = tile_n * 16 + (lane & 15);      // B column: stencil node l
  const bool bn_ok = bn < 27;
  const int bnc = bn_ok ? bn : 0;
  const int kq = lane >> 4;                      // lane group: k offset within a step
  int dm_r[4], dm_e[4];                          // D rows held by this lane
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int m = tile_m * 16 + kq + 4 * v;
    dm_r[v] = (m < 27) ? m / 9 : 3;
    dm_e[v] = (m < 27) ? 3 * ((m % 9) / 3) + m % 3 : 0;
  }
  const int dn = tile_n * 16 + (lane & 15);      // D column: stencil node l
  const int dnx = dn % 3, dny = (dn / 3) % 3, dnz = dn / 9;
  // window slot of (node l, row r, column ky, kz) = dsl0 - r - 5 ky - 25 kz
  const int dsl0 = (dnx + 2) + 5 * (dny + 2) + 25 * (dnz + 2);
  // K order of a pass: step st, lane group kq -> particle q = 2 kq + st / 3,
  // component e = st % 3, so a lane's six A operands come from two particles
  int zoff[9];  // packed C index of (3 g + b, 3 d + e), entry 3 b + e
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int e = 0; e < 3; ++e) zoff[3 * b + e] = tri9(3 * am_g + b, 3 * am_d + e);
  FinRoles fr;
  fin_roles(tid, nxw, fr);
  __syncthreads();
  auto next_job = [&](int v, int t0, int& nv, int& nt) {
    if (v >= 0 && t0 + kAsmChunk < mcnt[v]) {
      nv = v;
      nt = t0 + kAsmChunk;
      return;
    }
    nv = nextv[v + 1];
    nt = 0;
  };
  // staging: a chunk's particles are consecutive, so its a_l and C values are
  // two contiguous ranges; thread tid moves entries tid + 256 k of each
  auto fetch = [&](int v, int t0, double* ra, double* rc) {
    if (v < 0) return;
    const int np = min(kAsmChunk, mcnt[v] - t0);
    const long long st = mst[v] + t0;
#pragma unroll
    for (int k = 0; k < kARegs; ++k)
      if (tid + 256 * k < kPA * np) ra[k] = Ag[kPA * st + tid + 256 * k];
#pragma unroll
    for (int k = 0; k < kCRegs; ++k)
      if (tid + 256 * k < kPC * np) rc[k] = Cp[kPC * st + tid + 256 * k];
  };
  double ra[kARegs], rc[kCRegs];
#pragma unroll
  for (int k = 0; k < kARegs; ++k) ra[k] = 0.0;
#pragma unroll
  for (int k = 0; k < kCRegs; ++k) rc[k] = 0.0;
  int jv, jt;
  next_job(-1, 0, jv, jt);
  fetch(jv, jt, ra, rc);
  int next_row = rb;
  for (int ci = 0; ci < ncx; ++ci) {
    const int c = xa - 2 + ci;
    const int rlo = max(0, xa - c), rhi = min(2, xb - c);
    for (int col = 0; col < 9; ++col) {
      const int v = ci * 9 + col;
      const int cnt = mcnt[v];
      if (cnt == 0) continue;
      const int ky = col % 3, kz = col / 3;
      v4d acc = {0.0, 0.0, 0.0, 0.0};
      for (int t0 = 0; t0 < cnt; t0 += kAsmChunk) {
        const int np = min(kAsmChunk, cnt - t0);
        __syncthreads();  // the previous pass's operand reads are done
#pragma unroll
        for (int k = 0; k < kARegs; ++k)
          if (tid + 256 * k < kPA * np) (&av[0][0][0])[tid + 256 * k] = ra[k];
#pragma unroll
        for (int k = 0; k < kCRegs; ++k)
          if (tid + 256 * k < kPC * np) (&pc[0][0])[tid + 256 * k] = rc[k];
        __syncthreads();
        // prefetch the next chunk while this one is processed
        int nv, nt;
        next_job(v, t0, nv, nt);
        fetch(nv, nt, ra, rc);
        // A operands Z_r[g][3d + e] = sum_b a_k[b] C[3g + b][3d + e], k = (r, ky, kz),
        // then B[(r, g, d)][l] += sum over the chunk's (p, eps), four at a time
        {
          const bool a_ok = am_ok && am_r >= rlo && am_r <= rhi;
          double za[6];
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const int q = 2 * kq + j;
            if (a_ok && q < np) {
              const double* a = av[q][am_r + 3 * ky + 9 * kz];
              const double* Cq = pc[q];
              const double a0 = a[0], a1 = a[1], a2 = a[2];
#pragma unroll
              for (int e = 0; e < 3; ++e)
                za[3 * j + e] = a0 * Cq[zoff[e]] + a1 * Cq[zoff[3 + e]] + a2 * Cq[zoff[6 + e]];
            } else {
              za[3 * j] = za[3 * j + 1] = za[3 * j + 2] = 0.0;
            }
          }
#pragma unroll
          for (int st = 0; st < 6; ++st) {
            if (st < 3 || np > 1) {  // uniform
              const int q = 2 * kq + st / 3;
              const double b = (q < np && bn_ok) ? av[q][bnc][st % 3] : 0.0;
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64(za[st], b, acc, 0, 0, 0);
            }
          }
        }
      }
      // the column's blocks into the sliding window (disjoint per lane/wave):
      // the four reads first, then the adds and stores
      if (dn < 27) {
        double* wp[4];
        double wv[4];
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) {
          const int r = dm_r[vv] < 3 ? dm_r[vv] : 0;
          wp[vv] = &win[(c + r + 3) % 3][dm_e[vv] * kSlotPad + dsl0 - r - 5 * ky - 25 * kz];
          wv[vv] = *wp[vv];
        }
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) {
          const int r = dm_r[vv];
          if (r >= rlo && r <= rhi) *wp[vv] = wv[vv] + acc[vv];
        }
      }
    }
    __syncthreads();
    if (next_row < re && rx[next_row - rb] == c) {
      int ro = next_row - rb;
      bool rf = nbf[(c - xw0) + nxw * (2 + 5 * 2)] != 0;
      finalize_row_block(win[(c + 3) % 3], next_row, c, xw0, L, nbf, fr, rf, rmass[ro], red);
      ++next_row;
    }
    double* wz = win[(c + 3) % 3];
    for (int e = tid; e < kRowStride; e += 256) wz[e] = 0.0;
    __syncthreads();
  }
}

}  // namespace

void launch_particle_frac(const SceneDev& s, int n, const double* x, double* f, int* key,
                          hipStream_t st) {
  if (n > 0) k_frac<<<blocks_for(n), kTpb, 0, st>>>(s, n, x, f, key);
}

void launch_p2g(const SceneDev& s, const LevelView& L0, const Bricks& B, const double* f,
                const double* v, const double* C, const double* vol, const int* mat,
                const int* cstart, const int* ccount, double* partial, double dt, double t_end,
                double* mass, double* vstar, double* xi, int* fixed, hipStream_t st) {
  if (B.n > 0)
    k_p2g_brick<<<B.n, 64, 0, st>>>(s, B, f, v, C, vol, mat, cstart, ccount, partial);
  if (L0.n > 0)
    k_p2g_nodes<<<blocks_for(L0.n), kTpb, 0, st>>>(s, L0, B, partial, dt, t_end, mass, vstar, xi,
                                                   fixed);
}

static void node_vel(const LevelView& L0, const double* vstar, const double* dv, const double* p,
                     double alpha, double* wnode, hipStream_t st) {
  if (L0.n > 0)
    k_node_vel<<<blocks_for(L0.n), kTpb, 0, st>>>(L0, vstar, dv, p, alpha, (double4*)wnode);
}

void launch_particle_hessian(const SceneDev& s, const LevelView& L0, int n, const double* f,
                             const int* key, const double* F, const double* vol, const int* mat,
                             const double* vstar, const double* dv, double dt, double* wnode,
                             double* Cp, hipStream_t st) {
  node_vel(L0, vstar, dv, nullptr, 0.0, wnode, st);
  if (n > 0)
    k_particle_hessian<<<blocks_for(n), kTpb, 0, st>>>(s, L0, n, f, key, F, vol, mat,
                                                       (const double4*)wnode, dt, Cp);
}

void launch_particle_eval(const SceneDev& s, const LevelView& L0, int n, const double* f,
                          const int* key, const double* F, const double* vol, const int* mat,
                          const double* vstar, const double* dv, const double* p, double alpha,
                          double dt, double* wnode, double* psi_out, double* S_out,
                          hipStream_t st) {
  node_vel(L0, vstar, dv, p, alpha, wnode, st);
  if (n > 0)
    k_particle_eval<<<blocks_for(n), kTpb, 0, st>>>(s, L0, n, f, key, F, vol, mat,
                                                    (const double4*)wnode, dt, psi_out, S_out);
}

void launch_gradient(const SceneDev& s, const LevelView& L0, const Bricks& B, const double* f,
                     const double* S, const int* cstart, const int* ccount, double* partial,
                     const double* mass, const int* fixed, const double* dv, double dt, double* g,
                     hipStream_t st) {
  if (B.n > 0)
    k_grad_brick<<<B.n, 64 * kGradWaves, 0, st>>>(s, B, f, S, cstart, ccount, partial);
  if (L0.n > 0)
    k_grad_nodes<<<blocks_for(L0.n), kTpb, 0, st>>>(L0, B, partial, mass, fixed, dv, dt, g);
}

void launch_g2p(const SceneDev& s, const LevelView& L0, int n, const double* f, const int* key,
                double* x, double* v, double* C, double* F, const int* mat, const double* vstar,
                const double* dv, double dt, double* wnode, hipStream_t st) {
  node_vel(L0, vstar, dv, nullptr, 0.0, wnode, st);
  if (n > 0)
    k_g2p<<<blocks_for(n), kTpb, 0, st>>>(s, L0, n, f, key, x, v, C, F, mat,
                                          (const double4*)wnode, dt);
}

void launch_assemble_h0(const SceneDev& s, const LevelView& L0, const int* seg_begin, int n_seg,
                        int n, const double* f, const double* F, const double* Cp, double* Ag,
                        const int* cstart, const int* ccount, const double* mass, const int* fixed,
                        hipStream_t st) {
  const long long n27 = 27LL * n;
  if (n27 > 0) k_particle_agrad<<<blocks_for(n27), kTpb, 0, st>>>(s, n27, f, F, Ag);
  if (n_seg > 0)
    k_assemble_strip<<<n_seg, 256, 0, st>>>(s, L0, seg_begin, Ag, Cp, cstart, ccount, mass, fixed);
}

}  // namespace hot
