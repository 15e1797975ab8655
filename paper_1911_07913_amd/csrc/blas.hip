// Vector kernels of the quasi-Newton loop: deterministic reductions (fixed
// grid, fixed-order final sum), L-BFGS two-loop updates with device-side
// scalars, and precision conversions.
#include "mpm_math.h"

namespace hot {
namespace {

constexpr int kTpb = 256;
inline unsigned blocks_for(long long n, int tpb = kTpb) {
  return (unsigned)((n + tpb - 1) / tpb);
}
// Blocks of a reduction over n terms: about four terms per thread, between 64
// and kRedBlocks.  Fixed for a given n, so sums are reproducible.
inline int red_blocks(long long n) {
  long long b = (n + 4 * kTpb - 1) / (4 * kTpb);
  return (int)std::min<long long>(kRedBlocks, std::max<long long>(64, b));
}

__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kTpb / 64; ++k) t += sh[k];
  return t;
}

__device__ inline double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// kind 0: sum a*b; 1: sum a
__global__ void k_partial(long long n, int kind, const double* __restrict__ a,
                          const double* __restrict__ b, double* __restrict__ partial) {
  __shared__ double sh[kTpb / 64];
  double s = 0.0;
  for (long long k = (long long)blockIdx.x * kTpb + threadIdx.x; k < n; k += (long long)gridDim.x * kTpb) {
    double v = (kind == 0) ? a[k] * b[k] : a[k];
    s += v;
  }
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// sum_i 1/2 m_i (|dv_i + alpha p_i|^2 - |dv_i|^2)
__global__ void k_kinetic(int n, const double* __restrict__ m, const double* __restrict__ dv,
                          const double* __restrict__ p, double alpha, double* __restrict__ partial) {
  __shared__ double sh[kTpb / 64];
  double s = 0.0;
  for (int i = blockIdx.x * kTpb + threadIdx.x; i < n; i += (int)gridDim.x * kTpb) {
    double a2 = 0.0, b2 = 0.0;
    for (int c = 0; c < 3; ++c) {
      double d = dv[3 * i + c];
      double t = d + alpha * p[3 * i + c];
      a2 += t * t;
      b2 += d * d;
    }
    s += 0.5 * m[i] * a2 - 0.5 * m[i] * b2;
  }
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// The line search's energy change in one launch: blocks b < nb1 write the
// partials of sum_p (psi_t - psi_c) over n particles, blocks b < nb2 those of
// the kinetic change over n0 nodes, each with its own grid stride, so that
// the kinetic partials equal those of k_kinetic launched with nb2 blocks.
__global__ void k_energy_delta(long long n, const double* __restrict__ psi_t,
                               const double* __restrict__ psi_c, int nb1, int n0,
                               const double* __restrict__ m, const double* __restrict__ dv,
                               const double* __restrict__ p, double alpha, int nb2,
                               double* __restrict__ partial) {
  __shared__ double sh[kTpb / 64];
  const int b = blockIdx.x;
  if (b < nb1) {
    double s = 0.0;
    for (long long k = (long long)b * kTpb + threadIdx.x; k < n; k += (long long)nb1 * kTpb)
      s += psi_t[k] - psi_c[k];
    double t = block_sum(s, sh);
    if (threadIdx.x == 0) partial[b] = t;
    __syncthreads();
  }
  if (b < nb2) {
    double s = 0.0;
    for (int i = b * kTpb + threadIdx.x; i < n0; i += nb2 * kTpb) {
      double a2 = 0.0, b2 = 0.0;
      for (int c = 0; c < 3; ++c) {
        double d = dv[3 * i + c];
        double t = d + alpha * p[3 * i + c];
        a2 += t * t;
        b2 += d * d;
      }
      s += 0.5 * m[i] * a2 - 0.5 * m[i] * b2;
    }
    double t = block_sum(s, sh);
    if (threadIdx.x == 0) partial[nb1 + b] = t;
  }
}

// sum_i |g_i / (scale * xi_i)|^2, the squared CN-scaled gradient norm, over
// the nodes that carry mass (xi_i > 0: a node without mass has xi_i = 0 and
// no equation).
__global__ void k_cn(int n, const double* __restrict__ g, const double* __restrict__ xi, double scale,
                     double* __restrict__ partial) {
  __shared__ double sh[kTpb / 64];
  double s = 0.0;
  for (int i = blockIdx.x * kTpb + threadIdx.x; i < n; i += (int)gridDim.x * kTpb) {
    if (!(xi[i] > 0.0)) continue;
    double d = scale * xi[i];
    for (int c = 0; c < 3; ++c) {
      double q = g[3 * i + c] / d;
      s += q * q;
    }
  }
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void k_maxspeed(int n, const double* __restrict__ v, double* __restrict__ partial) {
  __shared__ double sh[kTpb / 64];
  double s = 0.0;
  for (int i = blockIdx.x * kTpb + threadIdx.x; i < n; i += (int)gridDim.x * kTpb) {
    double a = v[3 * i], b = v[3 * i + 1], c = v[3 * i + 2];
    s = fmax(s, sqrt(a * a + b * b + c * c));
  }
  s = wave_max(s);
  int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) sh[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < kTpb / 64; ++k) t = fmax(t, sh[k]);
    partial[blockIdx.x] = t;
  }
}

// Fixed-order final reduction of nparts partials (sum or max) into out.
__global__ void k_finish(int nparts, int count, int is_max, const double* __restrict__ partial,
                         double* __restrict__ out) {
  __shared__ double sh[kTpb / 64];
  for (int q = 0; q < count; ++q) {
    double s = 0.0;
    for (int k = threadIdx.x; k < nparts; k += kTpb) {
      double v = partial[q * nparts + k];
      s = is_max ? fmax(s, v) : s + v;
    }
    double t;
    if (is_max) {
      s = wave_max(s);
      int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
      if (lane == 0) sh[w] = s;
      __syncthreads();
      t = 0.0;
      if (threadIdx.x == 0)
        for (int k = 0; k < kTpb / 64; ++k) t = fmax(t, sh[k]);
    } else {
      t = block_sum(s, sh);
    }
    if (threadIdx.x == 0) out[q] = t;
    __syncthreads();
  }
}

// The fixed-order sum of k_finish, in thread 0.
__device__ inline double finish_sum(int nparts, const double* __restrict__ partial, double* sh) {
  double s = 0.0;
  for (int k = threadIdx.x; k < nparts; k += kTpb) s += partial[k];
  return block_sum(s, sh);
}

// out[0] = sum of partial[0, n1), out[1] = sum of partial[n1, n1 + n2), each
// in the order of k_finish.
__global__ void k_finish2(int n1, int n2, const double* __restrict__ partial,
                          double* __restrict__ out) {
  __shared__ double sh[kTpb / 64];
  double t = finish_sum(n1, partial, sh);
  if (threadIdx.x == 0) out[0] = t;
  __syncthreads();
  t = finish_sum(n2, partial + n1, sh);
  if (threadIdx.x == 0) out[1] = t;
}

// Start of either two-loop recursion: v <- -init (if init is given), then the
// block partials of dnext . v.
__global__ void k_twoloop_start(long long n, const double* __restrict__ init, double* __restrict__ v,
                                const double* __restrict__ dnext, double* __restrict__ partial) {
  __shared__ double sh[kTpb / 64];
  double acc = 0.0;
  for (long long k = (long long)blockIdx.x * kTpb + threadIdx.x; k < n; k += (long long)gridDim.x * kTpb) {
    double val = init ? -1.0 * init[k] : v[k];
    if (init) v[k] = val;
    acc += dnext[k] * val;
  }
  double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// One inner step of either two-loop recursion.  Every block first finishes
// the previous inner product from its partials (the same fixed-order sum in
// every block, so all blocks hold the same value d), then
//   first loop  (alpha_in NULL): alpha = rho d,  v <- v - alpha x, alpha stored;
//   second loop:                 coef = alpha_in - rho d,  v <- v + coef x,
// and writes the block partials of dnext . v (if dnext is given) to partial.
// prev and partial must be different buffers.  A thread's first kPre terms
// are loaded before the finishing sum, so that their latency overlaps it; the
// arithmetic and its order are those of the plain grid-stride loop.
__global__ void k_twoloop_step(long long n, int nparts, const double* __restrict__ prev,
                               const double* __restrict__ rho, const double* __restrict__ alpha_in,
                               double* __restrict__ alpha_out, const double* __restrict__ x,
                               double* __restrict__ v, const double* __restrict__ dnext,
                               double* __restrict__ partial) {
  constexpr int kPre = 4;
  __shared__ double sh[kTpb / 64];
  __shared__ double coef;
  const long long k0 = (long long)blockIdx.x * kTpb + threadIdx.x;
  const long long stride = (long long)gridDim.x * kTpb;
  double pv[kPre], px[kPre], pd[kPre];
#pragma unroll
  for (int j = 0; j < kPre; ++j) {
    const long long k = k0 + j * stride;
    pv[j] = px[j] = pd[j] = 0.0;
    if (k < n) {
      pv[j] = v[k];
      px[j] = x[k];
      if (dnext) pd[j] = dnext[k];
    }
  }
  const double d = finish_sum(nparts, prev, sh);
  if (threadIdx.x == 0) {
    const double rd = rho[0] * d;
    if (alpha_in) {
      coef = alpha_in[0] - rd;
    } else {
      coef = -1.0 * rd;
      if (blockIdx.x == 0) alpha_out[0] = rd;
    }
  }
  __syncthreads();
  const double al = coef;
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < kPre; ++j) {
    const long long k = k0 + j * stride;
    if (k < n) {
      double val = pv[j];
      val = val + al * px[j];
      v[k] = val;
      if (dnext) acc += pd[j] * val;
    }
  }
  for (long long k = k0 + kPre * stride; k < n; k += stride) {
    double val = v[k];
    val = val + al * x[k];
    v[k] = val;
    if (dnext) acc += dnext[k] * val;
  }
  if (dnext) {
    double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
  }
}

// Accepted step: dv_t = dv + alpha p and s = dv_t - dv.
__global__ void k_step_update(long long n, const double* __restrict__ dv, double alpha,
                              const double* __restrict__ p, double* __restrict__ dvt,
                              double* __restrict__ sv) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double t = dv[k];
  t = t + alpha * p[k];
  dvt[k] = t;
  sv[k] = t - dv[k];
}

// y = g_new - g with the block partials of y.s, y.y, s.s (in that order),
// then those of the squared CN norm of g_new over the n0 nodes (the k_cn
// loop with the same grid).
__global__ void k_secant(long long n, const double* __restrict__ gnew, const double* __restrict__ g,
                         double* __restrict__ y, const double* __restrict__ sv, int n0,
                         const double* __restrict__ xi, double scale,
                         double* __restrict__ partial) {
  __shared__ double sh[kTpb / 64];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (long long k = (long long)blockIdx.x * kTpb + threadIdx.x; k < n; k += (long long)gridDim.x * kTpb) {
    double x = gnew[k] - g[k];
    y[k] = x;
    double yv = sv[k];
    s0 += x * yv;
    s1 += x * x;
    s2 += yv * yv;
  }
  double t0 = block_sum(s0, sh);
  __syncthreads();
  double t1 = block_sum(s1, sh);
  __syncthreads();
  double t2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = t0;
    partial[gridDim.x + blockIdx.x] = t1;
    partial[2 * gridDim.x + blockIdx.x] = t2;
  }
  __syncthreads();
  double sc = 0.0;
  for (int i = blockIdx.x * kTpb + threadIdx.x; i < n0; i += (int)gridDim.x * kTpb) {
    if (!(xi[i] > 0.0)) continue;  // no mass, no equation (as k_cn)
    double d = scale * xi[i];
    for (int c = 0; c < 3; ++c) {
      double q = gnew[3 * i + c] / d;
      sc += q * q;
    }
  }
  double t3 = block_sum(sc, sh);
  if (threadIdx.x == 0) partial[3 * gridDim.x + blockIdx.x] = t3;
}

__global__ void k_scale_copy(long long n, double a, const double* __restrict__ x, double* __restrict__ y) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  y[k] = a * x[k];
}
__global__ void k_to_f32(long long n, const double* __restrict__ x, float* __restrict__ y) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) y[k] = (float)x[k];
}
__global__ void k_bj_apply(int n, const double* __restrict__ Dinv, const double* __restrict__ x,
                           double* __restrict__ y, double sign) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* D = Dinv + 9 * (long long)i;
  double x0 = x[3 * i], x1 = x[3 * i + 1], x2 = x[3 * i + 2];
  for (int g = 0; g < 3; ++g) y[3 * i + g] = sign * (D[3 * g] * x0 + D[3 * g + 1] * x1 + D[3 * g + 2] * x2);
}

// Conjugate-gradient vector updates of the Newton-Krylov solve: y += a x,
// y = x + b y, and the diagonal preconditioner z = r / d.
__global__ void k_axpy(long long n, double a, const double* __restrict__ x, double* __restrict__ y) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}
__global__ void k_xpby(long long n, const double* __restrict__ x, double b, double* __restrict__ y) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] + b * y[i];
}
__global__ void k_diag_solve(long long n, const double* __restrict__ d, const double* __restrict__ r,
                             double* __restrict__ z) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = r[i] / d[i];
}

__global__ void k_fill_d(long long n, double* p, double v) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}
__global__ void k_rho(const double* ys, double* rho) { rho[0] = 1.0 / ys[0]; }

}  // namespace

void launch_axpy(long long n, double a, const double* x, double* y, hipStream_t st) {
  if (n > 0) k_axpy<<<blocks_for(n), kTpb, 0, st>>>(n, a, x, y);
}
void launch_xpby(long long n, const double* x, double b, double* y, hipStream_t st) {
  if (n > 0) k_xpby<<<blocks_for(n), kTpb, 0, st>>>(n, x, b, y);
}
void launch_diag_solve(long long n, const double* d, const double* r, double* z, hipStream_t st) {
  if (n > 0) k_diag_solve<<<blocks_for(n), kTpb, 0, st>>>(n, d, r, z);
}

void launch_fill_double(long long n, double* p, double v, hipStream_t st) {
  if (n > 0) k_fill_d<<<blocks_for(n), kTpb, 0, st>>>(n, p, v);
}
void launch_rho(const double* ys, double* rho, hipStream_t st) { k_rho<<<1, 1, 0, st>>>(ys, rho); }

void launch_dot(long long n, const double* a, const double* b, double* partial, double* out,
                hipStream_t st) {
  const int nb = red_blocks(n);
  k_partial<<<nb, kTpb, 0, st>>>(n, 0, a, b, partial);
  k_finish<<<1, kTpb, 0, st>>>(nb, 1, 0, partial, out);
}
void launch_sum(long long n, const double* a, double* partial, double* out, hipStream_t st) {
  const int nb = red_blocks(n);
  k_partial<<<nb, kTpb, 0, st>>>(n, 1, a, nullptr, partial);
  k_finish<<<1, kTpb, 0, st>>>(nb, 1, 0, partial, out);
}
void launch_kinetic_delta(int n, const double* mass, const double* dv, const double* p,
                          double alpha, double* partial, double* out, hipStream_t st) {
  const int nb = red_blocks(3LL * n);
  k_kinetic<<<nb, kTpb, 0, st>>>(n, mass, dv, p, alpha, partial);
  k_finish<<<1, kTpb, 0, st>>>(nb, 1, 0, partial, out);
}
void launch_cn_sq(int n, const double* g, const double* xi, double scale, double* partial,
                  double* out, hipStream_t st) {
  const int nb = red_blocks(3LL * n);
  k_cn<<<nb, kTpb, 0, st>>>(n, g, xi, scale, partial);
  k_finish<<<1, kTpb, 0, st>>>(nb, 1, 0, partial, out);
}
void launch_max_speed(int n, const double* v, double* partial, double* out, hipStream_t st) {
  const int nb = red_blocks(3LL * n);
  k_maxspeed<<<nb, kTpb, 0, st>>>(n, v, partial);
  k_finish<<<1, kTpb, 0, st>>>(nb, 1, 1, partial, out);
}
void launch_twoloop_start(long long n, const double* init, double* v, const double* dnext,
                          double* partial, hipStream_t st) {
  k_twoloop_start<<<red_blocks(n), kTpb, 0, st>>>(n, init, v, dnext, partial);
}
void launch_twoloop_step(long long n, const double* prev, const double* rho, const double* alpha_in,
                         double* alpha_out, const double* x, double* v, const double* dnext,
                         double* partial, hipStream_t st) {
  k_twoloop_step<<<red_blocks(n), kTpb, 0, st>>>(n, red_blocks(n), prev, rho, alpha_in, alpha_out, x,
                                                 v, dnext, partial);
}
void launch_finish_partials(long long n, const double* partial, double* out, hipStream_t st) {
  k_finish<<<1, kTpb, 0, st>>>(red_blocks(n), 1, 0, partial, out);
}
void launch_step_update(long long n, const double* dv, double alpha, const double* p, double* dvt,
                        double* sv, hipStream_t st) {
  if (n > 0) k_step_update<<<blocks_for(n), kTpb, 0, st>>>(n, dv, alpha, p, dvt, sv);
}
void launch_secant_cn(long long n, const double* gnew, const double* g, double* y, const double* sv,
                      int n0, const double* xi, double scale, double* partial, double* out,
                      hipStream_t st) {
  const int nb = red_blocks(n);
  k_secant<<<nb, kTpb, 0, st>>>(n, gnew, g, y, sv, n0, xi, scale, partial);
  k_finish<<<1, kTpb, 0, st>>>(nb, 4, 0, partial, out);
}
void launch_energy_delta(long long n, const double* psi_t, const double* psi_c, int n0,
                         const double* mass, const double* dv, const double* p, double alpha,
                         double* partial, double* out, hipStream_t st) {
  const int nb1 = red_blocks(n), nb2 = red_blocks(3LL * n0);
  k_energy_delta<<<std::max(nb1, nb2), kTpb, 0, st>>>(n, psi_t, psi_c, nb1, n0, mass, dv, p, alpha,
                                                      nb2, partial);
  k_finish2<<<1, kTpb, 0, st>>>(nb1, nb2, partial, out);
}
void launch_scale_copy(long long n, double a, const double* x, double* y, hipStream_t st) {
  if (n > 0) k_scale_copy<<<blocks_for(n), kTpb, 0, st>>>(n, a, x, y);
}
void launch_to_f32(long long n, const double* x, float* y, hipStream_t st) {
  if (n > 0) k_to_f32<<<blocks_for(n), kTpb, 0, st>>>(n, x, y);
}
void launch_block_jacobi_apply(int n, const double* Dinv, const double* x, double* y, double sign,
                               hipStream_t st) {
  if (n > 0) k_bj_apply<<<blocks_for(n), kTpb, 0, st>>>(n, Dinv, x, y, sign);
}

}  // namespace hot
