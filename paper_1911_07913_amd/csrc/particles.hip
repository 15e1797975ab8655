// Particle-grid kernels of the implicit MPM step (Sec. 3.1) and the level-0
// system matrix (Sec. 4.1, Alg. HOT initialisation).
//
// Particle-to-node sums are computed without global floating-point atomics
// and in a fixed order (see the brick and row-segment kernels below), so the
// results are reproducible run to run.
#include <climits>

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

// F_p(dv) = (I + dt sum_i v_i grad w_ip^T) F_p^n with v_i from k_node_vel;
// node_v(k, vel) supplies the velocity of stencil node k.
template <typename NodeV>
__device__ inline void particle_F_with(const SceneDev& s, const double* fp, const double* Fn,
                                       double dt, double* F, NodeV node_v) {
  Weights W;
  bspline_weights(fp, s.inv_dx, W);
  double gv[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < 27; ++k) {
    const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
    double vel[3];
    node_v(k, vel);
    double g[3];
    node_grad(W, kx, ky, kz, g);
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

// Node velocities for the one-thread-per-particle passes.  Particles are
// sorted by base node, so a block's particles usually have base nodes within
// a short run k0 .. k1 of padded indices, and their 27-node stencils read,
// for each of the 9 (y, z) offsets, a contiguous range of k1 - k0 + 3 nodes.
// The block stages those ranges in LDS with contiguous loads (per-particle
// gathers of 27 nodes keep the vector-memory address units over 80% busy);
// particles outside the staged range, and blocks whose range is too long,
// read the node array directly.  The values are the same either way.
constexpr int kNodeWin = 64;  // staged nodes per (y, z) offset
struct NodeStage {
  int k0, span;
  bool staged;
};
// Every thread of the block calls this (it ends with a barrier).
__device__ inline NodeStage stage_node_ranges(const LevelView& L, const int* __restrict__ key,
                                              int n, const double4* __restrict__ wn,
                                              double (*win)[9 * kNodeWin]) {
  const int pb = blockIdx.x * blockDim.x;
  NodeStage ns;
  ns.k0 = key[pb];
  const int k1 = key[min(pb + (int)blockDim.x, n) - 1];
  ns.span = k1 - ns.k0 + 3;
  ns.staged = k1 >= ns.k0 && ns.span <= kNodeWin;
  if (ns.staged) {
    for (int e = threadIdx.x; e < 9 * ns.span; e += blockDim.x) {
      const int r = e / ns.span, xo = e - r * ns.span;  // r = ky + 3 kz
      const double4 wv = wn[ns.k0 + xo + stencil_offset(L.g, 3 * r)];
      win[0][r * kNodeWin + xo] = wv.x;
      win[1][r * kNodeWin + xo] = wv.y;
      win[2][r * kNodeWin + xo] = wv.z;
    }
  }
  __syncthreads();
  return ns;
}
// body(node_v), with node_v(k, vel) giving stencil node k's velocity for the
// particle whose base node is kp.
template <typename Body>
__device__ inline void with_node_velocities(const NodeStage& ns, const double (*win)[9 * kNodeWin],
                                            const LevelView& L, const double4* __restrict__ wn,
                                            int kp, Body body) {
  const int d = kp - ns.k0;
  if (ns.staged && d >= 0 && d + 2 < ns.span) {
    body([&](int k, double* vel) {
      const int e = (k / 3) * kNodeWin + d + k % 3;
      vel[0] = win[0][e];
      vel[1] = win[1][e];
      vel[2] = win[2][e];
    });
  } else {
    body([&](int k, double* vel) {
      const double4 wv = wn[kp + stencil_offset(L.g, k)];
      vel[0] = wv.x;
      vel[1] = wv.y;
      vel[2] = wv.z;
    });
  }
}

// Quadratic B-spline weight and its derivative (times 1/dx) for stencil
// offset k in {0, 1, 2} at fractional position f (Sec. 3 kernel).
__device__ inline void wdw(int k, double f, double inv_dx, double& w, double& dw) {
  double a = 1.5 - f, b = f - 1.0, c = f - 0.5;
  double w0 = 0.5 * (a * a), w1 = 0.75 - b * b, w2 = 0.5 * (c * c);
  double d0 = (f - 1.5) * inv_dx, d1 = -2.0 * b * inv_dx, d2 = c * inv_dx;
  w = (k == 0) ? w0 : ((k == 1) ? w1 : w2);
  dw = (k == 0) ? d0 : ((k == 1) ? d1 : d2);
}

// A particle's level-0 assembly record (kAsmRec doubles), one thread per
// particle: the projected stress derivative at F(dv), scaled by dt^2 V_p
// (the particle's contribution to the level-0 Hessian, Alg. HOT
// projectHessian), as 45 upper-triangle entries, then the assembly's
// right-hand operands a_lp = F_p^n^T grad w_lp for the 27 stencil nodes l
// (component-minor).  The thread writes its whole record, so every cache
// line of it is complete when it leaves the L2.  Node velocities come from
// the block's staged ranges.
__global__ __launch_bounds__(256) void k_particle_hessian(SceneDev s, LevelView L, int n, const double* __restrict__ f,
                                   const int* __restrict__ key, const double* __restrict__ Fn,
                                   const double* __restrict__ vol, const int* __restrict__ mat,
                                   const double4* __restrict__ wn, double dt,
                                   double* __restrict__ rec) {
  __shared__ double win[3][9 * kNodeWin];
  const NodeStage ns = stage_node_ranges(L, key, n, wn, win);
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double F[9], fn[9];
  for (int i = 0; i < 9; ++i) fn[i] = Fn[9 * p + i];
  with_node_velocities(ns, win, L, wn, key[p], [&](auto node_v) {
    particle_F_with(s, f + 3 * p, fn, dt, F, node_v);
  });
  // records start on 16-byte boundaries (kAsmRec even): entries 2j, 2j + 1
  // go out as one 16-byte store
  double2* R2 = reinterpret_cast<double2*>(rec + kAsmRec * (long long)p);
  double c44;  // C entry 44 shares a 16-byte store with the first a value
  {
    double C45[45];
    projected_dPdF(s.mats[mat[p]], F, dt * dt * vol[p], C45);
#pragma unroll
    for (int j = 0; j < 22; ++j) R2[j] = make_double2(C45[2 * j], C45[2 * j + 1]);
    c44 = C45[44];
  }
  const double f0 = f[3 * p], f1 = f[3 * p + 1], f2 = f[3 * p + 2];
  double wx[3], dx[3], wy[3], dy[3], wz[3], dz[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    wdw(k, f0, s.inv_dx, wx[k], dx[k]);
    wdw(k, f1, s.inv_dx, wy[k], dy[k]);
    wdw(k, f2, s.inv_dx, wz[k], dz[k]);
  }
  static_assert(kAsmRecA == 45 && kAsmRec == kAsmRecA + 81, "record layout");
  double a[81];
#pragma unroll
  for (int l = 0; l < 27; ++l) {
    const int kx = l % 3, ky = (l / 3) % 3, kz = l / 9;
    const double gx = dx[kx] * wy[ky] * wz[kz], gy = wx[kx] * dy[ky] * wz[kz],
                 gz = wx[kx] * wy[ky] * dz[kz];
    a[3 * l] = fn[0] * gx + fn[3] * gy + fn[6] * gz;
    a[3 * l + 1] = fn[1] * gx + fn[4] * gy + fn[7] * gz;
    a[3 * l + 2] = fn[2] * gx + fn[5] * gy + fn[8] * gz;
  }
  R2[22] = make_double2(c44, a[0]);
#pragma unroll
  for (int j = 0; j < 40; ++j) R2[23 + j] = make_double2(a[1 + 2 * j], a[2 + 2 * j]);
}

// Energy density and stress at the trial point: psi_out[p] = V_p psi(F_p),
// S_out[p] = V_p P(F_p) F_p^n^T (the particle's force tensor, Sec. 4.1).
// Node velocities come from the block's staged ranges.
__global__ __launch_bounds__(256) void k_particle_eval(SceneDev s, LevelView L, int n, const double* __restrict__ f,
                                const int* __restrict__ key, const double* __restrict__ Fn,
                                const double* __restrict__ vol, const int* __restrict__ mat,
                                const double4* __restrict__ wn, double dt,
                                double* __restrict__ psi_out, double* __restrict__ S_out) {
  __shared__ double win[3][9 * kNodeWin];
  const NodeStage ns = stage_node_ranges(L, key, n, wn, win);
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double F[9], fn[9];
  for (int i = 0; i < 9; ++i) fn[i] = Fn[9 * p + i];
  with_node_velocities(ns, win, L, wn, key[p], [&](auto node_v) {
    particle_F_with(s, f + 3 * p, fn, dt, F, node_v);
  });
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
// advection (Sec. 3.1).  Node velocities come from the block's staged ranges.
// Two waves per SIMD: left to itself the compiler takes 256 registers plus
// spill registers, which allows only one.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_g2p(SceneDev s, LevelView L, int n, const double* __restrict__ f,
                      const int* __restrict__ key, double* __restrict__ x,
                      double* __restrict__ v, double* __restrict__ C, double* __restrict__ Fn,
                      const int* __restrict__ mat, const double4* __restrict__ wn, double dt) {
  __shared__ double win[3][9 * kNodeWin];
  const NodeStage ns = stage_node_ranges(L, key, n, wn, win);
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double fp[3] = {f[3 * p], f[3 * p + 1], f[3 * p + 2]};
  Weights W;
  bspline_weights(fp, s.inv_dx, W);
  double vp[3] = {0, 0, 0}, B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, gv[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  with_node_velocities(ns, win, L, wn, key[p], [&](auto node_v) {
#pragma unroll
    for (int k = 0; k < 27; ++k) {
      const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
      double vel[3];
      node_v(k, vel);
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
  });
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
// dt^2 V_p (45 upper-triangle entries).  Each particle's operands sit in one
// record of kAsmRec doubles: C_p, then a_lp for its 27 stencil nodes l.
//
// One work-group of two waves per row segment: up to 16 consecutive rows
// (x, y, z) of one x-line.  The group sweeps the base cells c = x_first - 2
// .. x_last of the 9 cell columns (c, y - ky, z - kz), ky, kz in {0,1,2}; a
// particle of column (ky, kz) in cell c touches rows c + r, r in {0,1,2}, of
// this segment, with stencil offset k = (r, ky, kz).  For one cell column the
// blocks are a dense contraction over the column's particles p and the
// component eps:
//   B[(r, g, d)][l] = sum_(p, eps) Z_p[(r, g, d)][eps] a_p[l][eps],
//   Z_p[(r, g, d)][eps] = sum_b a_p[k][b] C_p[3g + b][3d + eps],
// a 27 x 27 x 3P product computed with FP64 16x16x4 matrix-core steps.  Wave
// w owns product rows 16w .. 16w + 15 and both 16-column tiles: each lane
// forms its A operands (Z values) once, in registers, for two steps, and the
// two waves' rows are disjoint entries of the 3-row sliding window in LDS,
// so a column's sums are added to the window by the wave that computed them
// with no barrier.  Particles are staged kAsmChunk at a time as one
// contiguous range of records, 16 bytes per load; record slots past the
// column's last particle are zero-filled, so every operand read and
// matrix-core step is unconditional.  After cell c, row c receives nothing
// more: it is finalised (mass, Dirichlet projection) and written once; the
// smoother's block inverses of the segment's rows are formed together at the
// end.  Every block of every particle is computed exactly once; no atomics.
constexpr int kAsmChunk = 8;                       // particles staged per pass
constexpr int kAsmThreads = 128;                   // two waves
constexpr int kStage = 1024;                       // staged doubles per pass
constexpr int kStageLd = kStage / (2 * kAsmThreads);  // 16-byte loads per thread
constexpr int kBufferWord3 = 0x00020000;          // buffer resource word 3 (raw, 32-bit)
static_assert(kAsmChunk * kAsmRec <= kStage, "staging area too small");
static_assert((kAsmRec % 2) == 0, "records must keep 16-byte alignment");

// Finalisation of level-0 row i held in the LDS window (the group's
// kAsmThreads threads, no barrier): mass on the diagonal, Dirichlet
// projection (constrained row -> m_i I, blocks to constrained neighbours ->
// 0), exact-zero diagonal rule, write-out (and in mixed precision, L.Hb set,
// the BF16 blocks and FP32 diagonal, as the level conversion would), the
// scalar diagonal and free-dof flags.  Thread t < 125 owns slot t of the
// nine entry planes; nb_fixed is the constrained flag of that slot's
// neighbour.  The window row is cleared as it is read.  The final diagonal
// block goes to cb[9] and this wave's share of the off-diagonal l1 row sums
// to l1w[3]; the l1 block-Jacobi inverse is formed from them once the whole
// segment is done.
constexpr int kWinPad = kSlots;  // window plane stride (the row's padding slots are not held)
__device__ inline void finalize_row(double* acc, int i, const LevelView& L, bool row_fixed,
                                    bool nb_fixed, double mass_i, double* cb, double* l1w) {
  const int tid = threadIdx.x, lane = tid & 63;
  double l1[3] = {0.0, 0.0, 0.0};
  if (tid < kSlots) {
    const bool center = tid == kCenter;
    const bool proj = row_fixed || (!center && nb_fixed);
    double* Hrow = L.H + (long long)i * kRowStride + tid;
    uint16_t* Hbrow = L.Hb ? L.Hb + (long long)i * kRowStride + tid : nullptr;
#pragma unroll
    for (int c = 0; c < kBlock; ++c) {
      double v = acc[c * kWinPad + tid];
      acc[c * kWinPad + tid] = 0.0;
      if (proj) v = 0.0;
      if (center) {
        if (c % 4 == 0) {
          const int g = c / 4;
          const double d = v + mass_i;
          const bool zero = (d == 0.0);
          v = zero ? 1.0 : d;
          L.free_dof[3 * i + g] = (!row_fixed && !zero) ? 1 : 0;
          L.diag[3 * i + g] = v;
          if (L.Hb) L.diag32[3 * i + g] = (float)v;
        }
        cb[c] = v;
      }
      Hrow[c * kSlotPad] = v;
      if (Hbrow) Hbrow[c * kSlotPad] = f32_to_bf16((float)v);
      l1[c / 3] += center ? 0.0 : fabs(v);
    }
  }
  for (int g = 0; g < 3; ++g) {
    const double t = wave_sum(l1[g]);
    if (lane == 0) l1w[g] = t;
  }
}

// Zeroes a window row that holds no node of the segment.
__device__ inline void clear_row(double* acc) {
  for (int e = threadIdx.x; e < kBlock * kWinPad; e += kAsmThreads) acc[e] = 0.0;
}

__global__ __launch_bounds__(kAsmThreads) __attribute__((amdgpu_waves_per_eu(2)))
void k_assemble_strip(SceneDev s, LevelView L, const int* __restrict__ seg_begin,
                      const double* __restrict__ rec,
                      const int* __restrict__ cstart, const int* __restrict__ ccount,
                      const double* __restrict__ mass, const int* __restrict__ fixed) {
  constexpr int kMaxCx = kSegRows + 2;
  constexpr int kWinRow = kBlock * kWinPad;
  __shared__ __attribute__((aligned(16))) double win[3][kWinRow];
  __shared__ __attribute__((aligned(16))) double stg[kStage];  // kAsmChunk records
  __shared__ double cb[kSegRows][9];       // final diagonal blocks of the rows
  __shared__ double l1w[2][kSegRows][3];   // per-wave l1 sums of the rows
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
  for (int v = tid; v < ncx * 9; v += kAsmThreads) {
    int ci = v / 9, col = v - 9 * ci;
    long long cell = pidx(L.g, xa - 2 + ci, ys - col % 3, zs - col / 3);
    mcnt[v] = ccount[cell];
    mst[v] = cstart[cell];
  }
  // constrained flags of the rows' neighbourhood, the rows' masses and x
  const int xw0 = xa - 2, nxw = ncx + 2;
  {
    constexpr int kNbIt = ((kMaxCx + 2) * 25 + kAsmThreads - 1) / kAsmThreads;
    int jn[kNbIt];
#pragma unroll
    for (int k = 0; k < kNbIt; ++k) {
      const int v = tid + kAsmThreads * k;
      const int xo = v % nxw, r = v / nxw;
      jn[k] = (v < nxw * 25) ? L.map[pidx(L.g, xw0 + xo, ys + r % 5 - 2, zs + r / 5 - 2)] : -1;
    }
#pragma unroll
    for (int k = 0; k < kNbIt; ++k) {
      const int v = tid + kAsmThreads * k;
      if (v < nxw * 25) nbf[v] = (jn[k] >= 0 && fixed[jn[k]]) ? 1 : 0;
    }
  }
  for (int v = tid; v < re - rb; v += kAsmThreads) {
    int x0, y0, z0;
    unpidx(L.g, L.nodes[rb + v], x0, y0, z0);
    rx[v] = x0;
    rmass[v] = mass[rb + v];
  }
  for (int e = tid; e < 3 * kWinRow; e += kAsmThreads) (&win[0][0])[e] = 0.0;
  __syncthreads();
  if (tid < 64) {  // nextv: suffix minimum of the non-empty columns, three per lane
    const int nv9 = ncx * 9;
    int m[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int e = 3 * tid + k;
      m[k] = (e < nv9 && mcnt[e] > 0) ? e : INT_MAX;
    }
    m[1] = min(m[1], m[2]);
    m[0] = min(m[0], m[1]);
    int sfx = m[0];  // over lanes >= this one
    for (int off = 1; off < 64; off <<= 1) {
      const int o = __shfl_down(sfx, off, 64);
      if (tid + off < 64) sfx = min(sfx, o);
    }
    int after = __shfl_down(sfx, 1, 64);
    if (tid == 63) after = INT_MAX;
    m[2] = min(m[2], after);
    m[1] = min(m[1], m[2]);
    m[0] = min(m[0], m[1]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int e = 3 * tid + k;
      if (e < nv9) nextv[e] = (m[k] == INT_MAX) ? -1 : m[k];
    }
    if (tid == 0) nextv[nv9] = -1;
  }
  // this thread's finalisation slot: the neighbour's constrained flag offset
  const int tsl = min(tid, kSlots - 1);
  const int nbo = (tsl % 5 - 2) + nxw * ((tsl / 5) % 5 + 5 * (tsl / 25));
  // matrix-core roles (FP64 16x16x4): lane l feeds A[l % 16][l / 16] and
  // B[l / 16][l % 16] and holds D[l / 16 + 4 v][l % 16], v = 0..3.  Wave w
  // owns product rows m = 16 w .. 16 w + 15, (r, g, d) = (m / 9, m % 9 / 3,
  // m % 3); rows m >= 27 are padding (their A operands are those of row 26,
  // their D rows are dropped).
  const int wave = tid >> 6, lane = tid & 63;
  const int kq = lane >> 4, li = lane & 15;
  const int am = min(16 * wave + li, 26);
  const int am_r = am / 9, am_g = (am % 9) / 3, am_d = am % 3;
  int zoff[9];  // packed C index of (3 g + b, 3 d + e), entry 3 b + e
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int e = 0; e < 3; ++e) zoff[3 * b + e] = tri9(3 * am_g + b, 3 * am_d + e);
  // B columns of the two tiles: stencil nodes l = li and 16 + li (clamped)
  const int bofs0 = kAsmRecA + 3 * li, bofs1 = kAsmRecA + 3 * min(16 + li, 26);
  // D rows held: m = 16 w + kq + 4 v (r = 3 marks padding)
  int dm_r[4], dm_o[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int m = 16 * wave + kq + 4 * v;
    dm_r[v] = (m < 27) ? m / 9 : 3;
    dm_o[v] = (m < 27) ? (3 * ((m % 9) / 3) + m % 3) * kWinPad - m / 9 : 0;
  }
  // D columns: node l = 16 tn + li; window slot of (l, r, ky, kz) is
  // dsl(l) - r - 5 ky - 25 kz
  int dsl[2];
  bool dn_ok[2];
#pragma unroll
  for (int tn = 0; tn < 2; ++tn) {
    const int n = 16 * tn + li;
    dn_ok[tn] = n < 27;
    const int l = min(n, 26);
    dsl[tn] = (l % 3 + 2) + 5 * ((l / 3) % 3 + 2) + 25 * (l / 9 + 2);
  }
  __syncthreads();
  // a chunk's records are one contiguous range of np records from particle
  // p0, read through a buffer resource of exactly that size: the loads past
  // it return zeros, which fill the unused record slots
  double2 ld[kStageLd];
  auto fetch = [&](int p0, int np) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(rec + (long long)p0 * kAsmRec), (short)0, np * kAsmRec * 8, kBufferWord3);
#pragma unroll
    for (int j = 0; j < kStageLd; ++j)
      ld[j] = __builtin_bit_cast(
          double2, __builtin_amdgcn_raw_buffer_load_b128(rs, 16 * (tid + kAsmThreads * j), 0, 0));
  };
#pragma unroll
  for (int j = 0; j < kStageLd; ++j) ld[j] = make_double2(0.0, 0.0);
  // the non-empty columns in sweep order: v, with cnt particles from pst
  int v = nextv[0];
  int cnt = 0, pst = 0;
  if (v >= 0) {
    cnt = mcnt[v];
    pst = mst[v];
    fetch(pst, min(kAsmChunk, cnt));
  }
  int next_row = rb;
  for (int ci = 0; ci < ncx; ++ci) {
    const int c = xa - 2 + ci;
    const int rlo = max(0, xa - c), rhi = min(2, xb - c);
    while (v >= 0 && v < 9 * (ci + 1)) {
      const int col = v - 9 * ci;
      const int ky = col % 3, kz = col / 3;
      const int nv = nextv[v + 1];
      const int ncnt = nv >= 0 ? mcnt[nv] : 0, npst = nv >= 0 ? mst[nv] : 0;
      const int kofs = kAsmRecA + 3 * (am_r + 3 * ky + 9 * kz);
      v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
      for (int t0 = 0; t0 < cnt; t0 += kAsmChunk) {
        const bool two = cnt - t0 > 4;  // particles 4.. present (uniform)
        __syncthreads();  // the previous pass's operand reads are done
#pragma unroll
        for (int j = 0; j < kStageLd; ++j)
          *reinterpret_cast<double2*>(stg + 2 * (tid + kAsmThreads * j)) = ld[j];
        __syncthreads();
        // prefetch the next chunk while this one is processed
        if (t0 + kAsmChunk < cnt)
          fetch(pst + t0 + kAsmChunk, min(kAsmChunk, cnt - t0 - kAsmChunk));
        else if (nv >= 0)
          fetch(npst, min(kAsmChunk, ncnt));
        // operand reads for this lane's particles q = kq, kq + 4, all issued
        // before the first use: a_q[k] (k = (r, ky, kz)), the nine C_q
        // entries of its Z values, and a_q[l] of its two B columns
        double ca[2][12], bb0[6], bb1[6];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const double* R = stg + (kq + 4 * h) * kAsmRec;
#pragma unroll
          for (int b = 0; b < 3; ++b) ca[h][b] = R[kofs + b];
#pragma unroll
          for (int k = 0; k < 9; ++k) ca[h][3 + k] = R[zoff[k]];
#pragma unroll
          for (int e = 0; e < 3; ++e) {
            bb0[3 * h + e] = R[bofs0 + e];
            bb1[3 * h + e] = R[bofs1 + e];
          }
        }
        __builtin_amdgcn_sched_barrier(0);
        // A operands Z_q[(r, g, d)][e]; K step st: particle kq + 4 (st / 3),
        // component st % 3
        double za[6];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int e = 0; e < 3; ++e)
            za[3 * h + e] = ca[h][0] * ca[h][3 + e] + ca[h][1] * ca[h][6 + e] +
                            ca[h][2] * ca[h][9 + e];
#pragma unroll
        for (int st = 0; st < 3; ++st) {
          acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(za[st], bb0[st], acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(za[st], bb1[st], acc1, 0, 0, 0);
        }
        if (two) {
#pragma unroll
          for (int st = 3; st < 6; ++st) {
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(za[st], bb0[st], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(za[st], bb1[st], acc1, 0, 0, 0);
          }
        }
      }
      // the column's blocks into the sliding window: this wave's entries
      // only, the eight reads first, then the adds and stores
      {
        const int cofs = -5 * ky - 25 * kz;
        double* wp[8];
        double wv[8];
#pragma unroll
        for (int v4 = 0; v4 < 4; ++v4) {
          const int r = dm_r[v4] < 3 ? dm_r[v4] : 0;
          double* row = win[(c + r + 3) % 3] + dm_o[v4] + cofs;
          wp[v4] = row + dsl[0];
          wp[4 + v4] = row + dsl[1];
          wv[v4] = *wp[v4];
          wv[4 + v4] = *wp[4 + v4];
        }
#pragma unroll
        for (int v4 = 0; v4 < 4; ++v4) {
          const bool rok = dm_r[v4] >= rlo && dm_r[v4] <= rhi;
          if (rok && dn_ok[0]) *wp[v4] = wv[v4] + acc0[v4];
          if (rok && dn_ok[1]) *wp[4 + v4] = wv[4 + v4] + acc1[v4];
        }
      }
      v = nv;
      cnt = ncnt;
      pst = npst;
    }
    __syncthreads();  // row c's sums are complete
    if (next_row < re && rx[next_row - rb] == c) {
      const int ro = next_row - rb;
      const uint8_t* nbx = nbf + (c - xw0);
      finalize_row(win[(c + 3) % 3], next_row, L, nbx[nxw * (2 + 5 * 2)] != 0,
                   tid < kSlots && nbx[nbo] != 0, rmass[ro], cb[ro], l1w[wave][ro]);
      ++next_row;
    } else {
      clear_row(win[(c + 3) % 3]);
    }
    // (the next pass's first barrier orders this row's clearing before
    // any later window update)
  }
  __syncthreads();
  // l1 block-Jacobi inverses of the segment's rows, one row per thread
  for (int ro = tid; ro < re - rb; ro += kAsmThreads) {
    double Dt[9];
    for (int k = 0; k < 9; ++k) Dt[k] = cb[ro][k];
    for (int g = 0; g < 3; ++g) Dt[4 * g] += l1w[0][ro][g] + l1w[1][ro][g];
    double Di[9];
    inv3(Dt, Di);
    const long long i = rb + ro;
    for (int k = 0; k < 9; ++k) L.Dinv[i * 9 + k] = Di[k];
    if (L.Hb)
      for (int k = 0; k < 9; ++k) L.Dinv32[i * 9 + k] = (float)Di[k];
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
                             double* rec, hipStream_t st) {
  node_vel(L0, vstar, dv, nullptr, 0.0, wnode, st);
  if (n > 0)
    k_particle_hessian<<<blocks_for(n), kTpb, 0, st>>>(s, L0, n, f, key, F, vol, mat,
                                                       (const double4*)wnode, dt, rec);
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
                        int n, const double* rec, const int* cstart, const int* ccount,
                        const double* mass, const int* fixed, hipStream_t st) {
  if (n_seg > 0 && n > 0)
    k_assemble_strip<<<n_seg, kAsmThreads, 0, st>>>(s, L0, seg_begin, rec, cstart, ccount, mass,
                                                     fixed);
}

}  // namespace hot
