// Galerkin coarsening and the multigrid V-cycle (Sec. 4, Alg. V-cycle).
//
// Matrices use 125-slot diagonal storage (Sec. 6): row i holds the 3x3 blocks
// of its neighbours at offsets [-2,2]^3.  Every row kernel is one wave per
// row: the 1125 values of a row are contiguous, so a wave reads them with
// coalesced loads and reduces its three output components with shuffles.
// The FP64 path stores blocks as double; the mixed path stores BF16 blocks and
// runs the V-cycle vectors and accumulation in FP32.
#include "mpm_math.h"

namespace hot {
namespace {

constexpr int kTpb = 256;
inline unsigned blocks_for(long long n, int tpb = kTpb) {
  return (unsigned)((n + tpb - 1) / tpb);
}

// ---------------------------------------------------------------- BF16
__device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(r >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

template <typename V, typename M>
__device__ inline V ldm(const M* p);
template <>
__device__ inline double ldm<double, double>(const double* p) { return *p; }
template <>
__device__ inline float ldm<float, uint16_t>(const uint16_t* p) { return bf16_to_f32(*p); }

template <typename V>
__device__ inline V wave_sum_t(V v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename V>
struct MatOf;
template <>
struct MatOf<double> {
  typedef double type;
  static __device__ const double* H(const LevelView& L) { return L.H; }
  static __device__ const double* Dinv(const LevelView& L) { return L.Dinv; }
  static __device__ const double* diag(const LevelView& L) { return L.diag; }
};
template <>
struct MatOf<float> {
  typedef uint16_t type;
  static __device__ const uint16_t* H(const LevelView& L) { return L.Hb; }
  static __device__ const float* Dinv(const LevelView& L) { return L.Dinv32; }
  static __device__ const float* diag(const LevelView& L) { return L.diag32; }
};

// y = H_i . x for one row, computed by a whole wave; result valid in all lanes.
// Lane l handles values e = l + 64k of the row (slot e/9, entry e%9).  All
// matrix values and neighbour indices of the row are loaded first, then the
// x entries, so each row costs two dependent memory round trips; slots the
// symbolic pattern marks absent are not read at all.
constexpr int kRowIt = (kRowVals + 63) / 64;  // 18

__device__ inline uint32_t pick_word(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, int k) {
  return k == 0 ? w0 : (k == 1 ? w1 : (k == 2 ? w2 : w3));
}

template <typename V>
__device__ inline void row_matvec(const LevelView& L, int i, const V* __restrict__ x, int lane,
                                  V* y) {
  typedef typename MatOf<V>::type M;
  const M* Hrow = MatOf<V>::H(L) + (long long)i * kRowVals;
  const long long pn = L.nodes[i];
  const uint32_t w0 = L.pat[4 * i], w1 = L.pat[4 * i + 1], w2 = L.pat[4 * i + 2],
                 w3 = L.pat[4 * i + 3];
  V h[kRowIt];
  int jn[kRowIt];
#pragma unroll
  for (int k = 0; k < kRowIt; ++k) {
    const int e = lane + 64 * k;
    const int s = e / 9;
    const bool present = (e < kRowVals) && ((pick_word(w0, w1, w2, w3, s >> 5) >> (s & 31)) & 1u);
    h[k] = present ? ldm<V, M>(Hrow + e) : (V)0;
    jn[k] = present ? L.map[pn + slot_offset(L.g, s)] : -1;
  }
  V a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
  for (int k = 0; k < kRowIt; ++k) {
    const int e = lane + 64 * k;
    const int c = e % 9;
    const int g = c / 3, d = c - 3 * g;
    V pr = (jn[k] >= 0) ? h[k] * x[3 * jn[k] + d] : (V)0;
    a0 += (g == 0) ? pr : (V)0;
    a1 += (g == 1) ? pr : (V)0;
    a2 += (g == 2) ? pr : (V)0;
  }
  y[0] = wave_sum_t(a0);
  y[1] = wave_sum_t(a1);
  y[2] = wave_sum_t(a2);
}

// ---------------------------------------------------------------- RAP
// Coarse row I of H^{m+1} = P~^T H^m P~ (Eq. buildMultigrid) with the linear
// node embedding: the fine children of I are 2I + a, a in {-1,0,1}^3, weight
// prod(1 or 1/2); each fine block (i, j) is spread to the coarse parents J of
// j.  P~ = Pi P drops constrained fine DOFs.  The symbolic coarse pattern is
// the structure of R pattern P.  Accumulation in LDS, one wave per coarse row.
constexpr int kRapWaves = 4;

__global__ __launch_bounds__(256) void k_rap(LevelView F, LevelView C) {
  __shared__ double acc_all[kRapWaves][kRowVals];
  __shared__ uint32_t pat_all[kRapWaves][4];
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int I = blockIdx.x * kRapWaves + wave;
  if (I >= C.n) return;
  double* acc = acc_all[wave];
  uint32_t* pat = pat_all[wave];
  for (int e = lane; e < kRowVals; e += 64) acc[e] = 0.0;
  if (lane < 4) pat[lane] = 0u;
  wave_sync();
  int X, Y, Z;
  unpidx(C.g, C.nodes[I], X, Y, Z);
  for (int a = 0; a < 27; ++a) {
    int ax = a % 3 - 1, ay = (a / 3) % 3 - 1, az = a / 9 - 1;
    int cx = 2 * X + ax, cy = 2 * Y + ay, cz = 2 * Z + az;
    int i = F.map[pidx(F.g, cx, cy, cz)];
    if (i < 0) continue;
    double wa = (ax ? 0.5 : 1.0) * (ay ? 0.5 : 1.0) * (az ? 0.5 : 1.0);
    double fi[3] = {(double)F.free_dof[3 * i], (double)F.free_dof[3 * i + 1],
                    (double)F.free_dof[3 * i + 2]};
    uint32_t pw[4] = {F.pat[4 * i], F.pat[4 * i + 1], F.pat[4 * i + 2], F.pat[4 * i + 3]};
    const double* Hrow = F.H + (long long)i * kRowVals;
    for (int e = lane; e < kRowVals; e += 64) {
      int s = e / 9, c = e - 9 * (e / 9);
      if (!((pw[s >> 5] >> (s & 31)) & 1u)) continue;
      int jx = cx + s % 5 - 2, jy = cy + (s / 5) % 5 - 2, jz = cz + s / 25 - 2;
      int j = F.map[pidx(F.g, jx, jy, jz)];
      int g = c / 3, d = c - 3 * g;
      double val = Hrow[e] * wa * fi[g] * (j >= 0 ? (double)F.free_dof[3 * j + d] : 0.0);
      int Px[2], Py[2], Pz[2];
      double wx[2], wy[2], wz[2];
      int nx, ny, nz;
      if (jx & 1) { Px[0] = (jx - 1) >> 1; Px[1] = (jx + 1) >> 1; wx[0] = wx[1] = 0.5; nx = 2; }
      else { Px[0] = jx >> 1; wx[0] = 1.0; nx = 1; }
      if (jy & 1) { Py[0] = (jy - 1) >> 1; Py[1] = (jy + 1) >> 1; wy[0] = wy[1] = 0.5; ny = 2; }
      else { Py[0] = jy >> 1; wy[0] = 1.0; ny = 1; }
      if (jz & 1) { Pz[0] = (jz - 1) >> 1; Pz[1] = (jz + 1) >> 1; wz[0] = wz[1] = 0.5; nz = 2; }
      else { Pz[0] = jz >> 1; wz[0] = 1.0; nz = 1; }
      for (int u = 0; u < nx; ++u)
        for (int v = 0; v < ny; ++v)
          for (int w = 0; w < nz; ++w) {
            int S = (Px[u] - X + 2) + 5 * (Py[v] - Y + 2) + 25 * (Pz[w] - Z + 2);
            if (val != 0.0) atomicAdd(&acc[S * 9 + c], val * (wx[u] * wy[v] * wz[w]));
            if (c == 0) atomicOr(&pat[S >> 5], 1u << (S & 31));
          }
    }
  }
  wave_sync();
  finalize_row(acc, I, C, nullptr, 0.0, lane);
  if (lane < 4) C.pat[4 * I + lane] = pat[lane];
}

__global__ void k_to_bf16(LevelView L) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long nv = (long long)L.n * kRowVals;
  if (k < nv) L.Hb[k] = f32_to_bf16((float)L.H[k]);
  if (k < (long long)L.n * 9) L.Dinv32[k] = (float)L.Dinv[k];
  if (k < (long long)L.n * 3) L.diag32[k] = (float)L.diag[k];
}

// ---------------------------------------------------------------- V-cycle
// First smoothing sweep from u = 0: u = D~^{-1} b.
template <typename V>
__global__ void k_jacobi_first(LevelView L, const V* __restrict__ b, V* __restrict__ u) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  const V* Di = MatOf<V>::Dinv(L) + 9 * (long long)i;
  V b0 = b[3 * i], b1 = b[3 * i + 1], b2 = b[3 * i + 2];
  for (int g = 0; g < 3; ++g) u[3 * i + g] = Di[3 * g] * b0 + Di[3 * g + 1] * b1 + Di[3 * g + 2] * b2;
}

constexpr int kRowWaves = 4;

// r = b - H u (one wave per row)
template <typename V>
__global__ __launch_bounds__(256) void k_residual(LevelView L, const V* __restrict__ b,
                                                  const V* __restrict__ u, V* __restrict__ r) {
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int i = blockIdx.x * kRowWaves + wave;
  if (i >= L.n) return;
  V y[3];
  row_matvec<V>(L, i, u, lane, y);
  if (lane < 3) r[3 * i + lane] = b[3 * i + lane] - y[lane];
}

// l1 block-Jacobi sweep: u_out = u + D~^{-1} (b - H u), projected.
template <typename V>
__global__ __launch_bounds__(256) void k_smooth(LevelView L, const V* __restrict__ b,
                                                const V* __restrict__ u, V* __restrict__ uo) {
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int i = blockIdx.x * kRowWaves + wave;
  if (i >= L.n) return;
  V y[3];
  row_matvec<V>(L, i, u, lane, y);
  if (lane < 3) {
    const V* Di = MatOf<V>::Dinv(L) + 9 * (long long)i;
    V r0 = b[3 * i] - y[0], r1 = b[3 * i + 1] - y[1], r2 = b[3 * i + 2] - y[2];
    V upd = Di[3 * lane] * r0 + Di[3 * lane + 1] * r1 + Di[3 * lane + 2] * r2;
    V out = u[3 * i + lane] + upd;
    uo[3 * i + lane] = L.free_dof[3 * i + lane] ? out : (V)0;
  }
}

// b^{m+1}_J = sum_i P~_iJ r_i over the 27 fine children of J.
template <typename V>
__global__ void k_restrict(LevelView F, LevelView C, const V* __restrict__ r, V* __restrict__ bc) {
  int J = blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= C.n) return;
  int X, Y, Z;
  unpidx(C.g, C.nodes[J], X, Y, Z);
  V s0 = 0, s1 = 0, s2 = 0;
  for (int a = 0; a < 27; ++a) {
    int ax = a % 3 - 1, ay = (a / 3) % 3 - 1, az = a / 9 - 1;
    int i = F.map[pidx(F.g, 2 * X + ax, 2 * Y + ay, 2 * Z + az)];
    if (i < 0) continue;
    V w = (V)((ax ? 0.5 : 1.0) * (ay ? 0.5 : 1.0) * (az ? 0.5 : 1.0));
    s0 += F.free_dof[3 * i] ? w * r[3 * i] : (V)0;
    s1 += F.free_dof[3 * i + 1] ? w * r[3 * i + 1] : (V)0;
    s2 += F.free_dof[3 * i + 2] ? w * r[3 * i + 2] : (V)0;
  }
  bc[3 * J] = s0;
  bc[3 * J + 1] = s1;
  bc[3 * J + 2] = s2;
}

// u_i += sum_J P~_iJ u^c_J over the (at most 8) parents of fine node i.
template <typename V>
__global__ void k_prolong_add(LevelView F, LevelView C, const V* __restrict__ uc, V* __restrict__ u) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= F.n) return;
  int x, y, z;
  unpidx(F.g, F.nodes[i], x, y, z);
  int Px[2], Py[2], Pz[2];
  V wx[2], wy[2], wz[2];
  int nx, ny, nz;
  if (x & 1) { Px[0] = (x - 1) >> 1; Px[1] = (x + 1) >> 1; wx[0] = wx[1] = (V)0.5; nx = 2; }
  else { Px[0] = x >> 1; wx[0] = (V)1; nx = 1; }
  if (y & 1) { Py[0] = (y - 1) >> 1; Py[1] = (y + 1) >> 1; wy[0] = wy[1] = (V)0.5; ny = 2; }
  else { Py[0] = y >> 1; wy[0] = (V)1; ny = 1; }
  if (z & 1) { Pz[0] = (z - 1) >> 1; Pz[1] = (z + 1) >> 1; wz[0] = wz[1] = (V)0.5; nz = 2; }
  else { Pz[0] = z >> 1; wz[0] = (V)1; nz = 1; }
  V s0 = 0, s1 = 0, s2 = 0;
  for (int a = 0; a < nx; ++a)
    for (int b = 0; b < ny; ++b)
      for (int c = 0; c < nz; ++c) {
        int J = C.map[pidx(C.g, Px[a], Py[b], Pz[c])];
        V w = wx[a] * wy[b] * wz[c];
        s0 += w * uc[3 * J];
        s1 += w * uc[3 * J + 1];
        s2 += w * uc[3 * J + 2];
      }
  if (F.free_dof[3 * i]) u[3 * i] += s0;
  if (F.free_dof[3 * i + 1]) u[3 * i + 1] += s1;
  if (F.free_dof[3 * i + 2]) u[3 * i + 2] += s2;
}

// ---------------------------------------------------------------- coarsest
// Jacobi-preconditioned CG (Alg. V-cycle, coarsest level) from x = 0, stopped
// once sqrt(r^T D^{-1} r) <= rel * sqrt(b^T D^{-1} b) (Sec. 5.3) or after
// max_iter iterations.  A single work-group runs the whole solve; its block
// reductions are fixed-order, so the result is deterministic.
constexpr int kPcgThreads = 1024;
constexpr int kPcgWaves = kPcgThreads / 64;

template <typename V>
__device__ inline V block_dot(const V* a, const V* b, int n, V* red) {
  V s = 0;
  for (int k = threadIdx.x; k < n; k += kPcgThreads) s += a[k] * b[k];
  s = wave_sum_t(s);
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = s;
  __syncthreads();
  V t = 0;
  for (int w = 0; w < kPcgWaves; ++w) t += red[w];
  return t;
}

template <typename V>
__global__ __launch_bounds__(kPcgThreads) void k_coarse_pcg(LevelView L, const V* __restrict__ b,
                                                            V* __restrict__ x, V* __restrict__ work,
                                                            int* __restrict__ iters_out, int max_iter,
                                                            double rel) {
  __shared__ V red[kPcgWaves];
  const int n3 = 3 * L.n;
  V* r = work;
  V* z = r + n3;
  V* p = z + n3;
  V* q = p + n3;
  const V* dg = MatOf<V>::diag(L);
  for (int k = threadIdx.x; k < n3; k += kPcgThreads) {
    V bk = b[k];
    x[k] = 0;
    r[k] = bk;
    V zk = bk / dg[k];
    z[k] = zk;
    p[k] = zk;
  }
  __syncthreads();
  V rz = block_dot<V>(r, z, n3, red);
  double stop = rel * sqrt(fmax((double)rz, 0.0));
  int it = 0;
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (rz > (V)0) {
    while (it < max_iter) {
      __syncthreads();
      for (int row = wave; row < L.n; row += kPcgWaves) {
        V y[3];
        row_matvec<V>(L, row, p, lane, y);
        if (lane < 3) q[3 * row + lane] = y[lane];
      }
      __syncthreads();
      V pq = block_dot<V>(p, q, n3, red);
      if (!(pq > (V)0)) break;
      V alpha = rz / pq;
      for (int k = threadIdx.x; k < n3; k += kPcgThreads) {
        x[k] += alpha * p[k];
        V rk = r[k] - alpha * q[k];
        r[k] = rk;
        z[k] = rk / dg[k];
      }
      __syncthreads();
      V rzn = block_dot<V>(r, z, n3, red);
      ++it;
      if (sqrt(fmax((double)rzn, 0.0)) <= stop) break;
      V beta = rzn / rz;
      rz = rzn;
      for (int k = threadIdx.x; k < n3; k += kPcgThreads) p[k] = z[k] + beta * p[k];
    }
  }
  if (threadIdx.x == 0) *iters_out = it;
}

__global__ __launch_bounds__(256) void k_spmv(LevelView L, const double* __restrict__ x,
                                              double* __restrict__ y) {
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int i = blockIdx.x * kRowWaves + wave;
  if (i >= L.n) return;
  double v[3];
  row_matvec<double>(L, i, x, lane, v);
  if (lane < 3) y[3 * i + lane] = v[lane];
}

}  // namespace

void launch_rap(const LevelView& F, const LevelView& C, hipStream_t st) {
  if (C.n > 0) k_rap<<<(unsigned)((C.n + kRapWaves - 1) / kRapWaves), 256, 0, st>>>(F, C);
}
void launch_to_bf16(const LevelView& L, hipStream_t st) {
  long long nv = (long long)L.n * kRowVals;
  if (nv > 0) k_to_bf16<<<blocks_for(nv), kTpb, 0, st>>>(L);
}

#define ROWGRID(L) (unsigned)(((L).n + kRowWaves - 1) / kRowWaves), 256, 0, st

void launch_jacobi_first(const LevelView& L, bool mixed, const void* b, void* u, hipStream_t st) {
  if (L.n == 0) return;
  if (mixed)
    k_jacobi_first<float><<<blocks_for(L.n), kTpb, 0, st>>>(L, (const float*)b, (float*)u);
  else
    k_jacobi_first<double><<<blocks_for(L.n), kTpb, 0, st>>>(L, (const double*)b, (double*)u);
}
void launch_residual(const LevelView& L, bool mixed, const void* b, const void* u, void* r,
                     hipStream_t st) {
  if (L.n == 0) return;
  if (mixed)
    k_residual<float><<<ROWGRID(L)>>>(L, (const float*)b, (const float*)u, (float*)r);
  else
    k_residual<double><<<ROWGRID(L)>>>(L, (const double*)b, (const double*)u, (double*)r);
}
void launch_smooth(const LevelView& L, bool mixed, const void* b, const void* u, void* uo,
                   hipStream_t st) {
  if (L.n == 0) return;
  if (mixed)
    k_smooth<float><<<ROWGRID(L)>>>(L, (const float*)b, (const float*)u, (float*)uo);
  else
    k_smooth<double><<<ROWGRID(L)>>>(L, (const double*)b, (const double*)u, (double*)uo);
}
void launch_restrict(const LevelView& F, const LevelView& C, bool mixed, const void* r, void* bc,
                     hipStream_t st) {
  if (C.n == 0) return;
  if (mixed)
    k_restrict<float><<<blocks_for(C.n), kTpb, 0, st>>>(F, C, (const float*)r, (float*)bc);
  else
    k_restrict<double><<<blocks_for(C.n), kTpb, 0, st>>>(F, C, (const double*)r, (double*)bc);
}
void launch_prolong_add(const LevelView& F, const LevelView& C, bool mixed, const void* uc, void* u,
                        hipStream_t st) {
  if (F.n == 0) return;
  if (mixed)
    k_prolong_add<float><<<blocks_for(F.n), kTpb, 0, st>>>(F, C, (const float*)uc, (float*)u);
  else
    k_prolong_add<double><<<blocks_for(F.n), kTpb, 0, st>>>(F, C, (const double*)uc, (double*)u);
}
size_t coarse_pcg_work_bytes(int n) { return (size_t)4 * 3 * n * sizeof(double); }
void launch_coarse_pcg(const LevelView& L, bool mixed, const void* b, void* x, void* work,
                       int* iters_out, int max_iter, double rel, hipStream_t st) {
  if (mixed)
    k_coarse_pcg<float><<<1, kPcgThreads, 0, st>>>(L, (const float*)b, (float*)x, (float*)work,
                                                    iters_out, max_iter, rel);
  else
    k_coarse_pcg<double><<<1, kPcgThreads, 0, st>>>(L, (const double*)b, (double*)x,
                                                     (double*)work, iters_out, max_iter, rel);
}
void launch_spmv(const LevelView& L, const double* x, double* y, hipStream_t st) {
  if (L.n > 0) k_spmv<<<ROWGRID(L)>>>(L, x, y);
}

}  // namespace hot
