// Galerkin coarsening and the multigrid V-cycle (Sec. 4, Alg. V-cycle).
//
// Matrices use 125-slot diagonal storage (Sec. 6): row i holds the 3x3 blocks
// of its neighbours at offsets [-2,2]^3, stored entry-major ([entry][slot]).
// Every row kernel is one wave per row: each lane owns whole blocks, reads
// their entries with coalesced loads and the three output components are
// reduced with shuffles.
// The FP64 path stores blocks as double; the mixed path stores BF16 blocks and
// runs the V-cycle vectors and accumulation in FP32.
#include <atomic>
#include <type_traits>

#include "mpm_math.h"

namespace hot {
namespace {

constexpr int kTpb = 256;
inline unsigned blocks_for(long long n, int tpb = kTpb) {
  return (unsigned)((n + tpb - 1) / tpb);
}

// ---------------------------------------------------------------- BF16
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

// The same wave sum on the DPP paths (no LDS round trips), for the sweeps:
// pairs, quads, half-rows and rows of 16 lanes by DPP moves, then the four
// row sums in a fixed order.  Every lane gets the identical value; all 64
// lanes must be active.
template <int Ctrl>
__device__ inline float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), Ctrl, 0xF, 0xF, false));
}
template <int Ctrl>
__device__ inline double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), Ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), Ctrl, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ inline float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double lane_value(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
template <typename V>
__device__ inline V wave_sum_dpp(V v) {
  v += dpp_mov<0xB1>(v);   // quad_perm(1, 0, 3, 2)
  v += dpp_mov<0x4E>(v);   // quad_perm(2, 3, 0, 1)
  v += dpp_mov<0x141>(v);  // row_half_mirror
  v += dpp_mov<0x140>(v);  // row_mirror
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
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

// Level vectors that sweeps gather from (the smoother iterate u and its
// ping-pong copy) live on the level's padded dense grid, one 4-vector per grid
// point (x, y, z, unused): a neighbour's entries are one 16- or 32-byte load at
// an address known from the row's own grid index, with no map lookup.  Only
// active points are ever written or read.
template <typename V>
struct Vec4Of;
template <>
struct Vec4Of<double> {
  typedef double4 type;
};
template <>
struct Vec4Of<float> {
  typedef float4 type;
};

// y = H_i . x for one row, computed by a whole wave; result valid in all lanes.
// Lane l owns the blocks of slots l and l + 64: it reads their 9 entries with
// coalesced loads (entry-major row layout) and the neighbour's 3 vector
// entries, so a row costs two dependent memory round trips.  Slots the
// symbolic pattern marks absent are not read.
__device__ inline bool slot_present(const uint32_t* w, int s) {
  return s < kSlots && ((w[s >> 5] >> (s & 31)) & 1u);
}

// One row's blocks as one wave holds them: lane l owns slots l and l + 64,
// with their 3x3 blocks and the compact indices of their neighbours (-1 for
// absent slots).
template <typename V>
struct RowBlocks {
  V h[2][9];
  int jn[2];
};

template <typename V>
__device__ inline void row_load(const LevelView& L, int i, int lane, RowBlocks<V>& rb) {
  typedef typename MatOf<V>::type M;
  const M* Hrow = MatOf<V>::H(L) + (long long)i * kRowStride;
  const long long pn = L.nodes[i];
  const uint32_t w[4] = {L.pat[4 * i], L.pat[4 * i + 1], L.pat[4 * i + 2], L.pat[4 * i + 3]};
#pragma unroll
  for (int ps = 0; ps < 2; ++ps) {
    const int s = lane + 64 * ps;
    const bool pr = slot_present(w, s);
    rb.jn[ps] = pr ? L.map[pn + slot_offset(L.g, s)] : -1;
#pragma unroll
    for (int c = 0; c < 9; ++c) rb.h[ps][c] = pr ? ldm<V, M>(Hrow + c * kSlotPad + s) : (V)0;
  }
}

// y = (held row) . x with x_j supplied by gather(j, x0, x1, x2); the sums are
// valid in every lane.
template <typename V, typename Gather>
__device__ inline void row_apply(const RowBlocks<V>& rb, V* y, Gather gather) {
  V a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
  for (int ps = 0; ps < 2; ++ps) {
    if (rb.jn[ps] >= 0) {
      V x0, x1, x2;
      gather((long long)rb.jn[ps], x0, x1, x2);
      a0 += rb.h[ps][0] * x0 + rb.h[ps][1] * x1 + rb.h[ps][2] * x2;
      a1 += rb.h[ps][3] * x0 + rb.h[ps][4] * x1 + rb.h[ps][5] * x2;
      a2 += rb.h[ps][6] * x0 + rb.h[ps][7] * x1 + rb.h[ps][8] * x2;
    }
  }
  y[0] = wave_sum_t(a0);
  y[1] = wave_sum_t(a1);
  y[2] = wave_sum_t(a2);
}

// y = H_i . x for one row, one wave; the neighbour values x_j come from
// gather(j, x0, x1, x2) with j the neighbour's compact index, so that a solver
// can form the multiplied vector on the fly.
template <typename V, typename Gather>
__device__ inline void row_matvec_with(const LevelView& L, int i, int lane, V* y, Gather gather) {
  RowBlocks<V> rb;
  row_load<V>(L, i, lane, rb);
  row_apply<V>(rb, y, gather);
}

template <typename V>
__device__ inline void row_matvec(const LevelView& L, int i, const V* __restrict__ x, int lane,
                                  V* y) {
  row_matvec_with<V>(L, i, lane, y, [&](long long j, V& x0, V& x1, V& x2) {
    const V* xj = x + 3 * j;
    x0 = xj[0];
    x1 = xj[1];
    x2 = xj[2];
  });
}

// y_r = H_{i0+r} . x for R consecutive rows, computed by one wave with all
// of the rows' loads issued before any is consumed, so that R rows' worth of
// bytes are in flight per wave.  FP64 blocks: lane l owns slots l and l + 64
// (512-byte coalesced loads per entry).  BF16 blocks: lane l owns slots 2l and
// 2l + 1 and reads both with one 32-bit load per entry.  Rows at or beyond
// L.n contribute nothing.  Results are valid in all lanes.
template <typename V>
struct SweepRows;
// Matrix rows are streamed once per sweep: non-temporal loads keep them from
// evicting the gathered iterate from L2.
template <>
struct SweepRows<double> {
  static __device__ inline int slot(int lane, int k) { return lane + 64 * k; }
  static __device__ inline void load(const double* Hrow, int c, int lane, bool p0, bool p1,
                                     double& h0, double& h1) {
    h0 = p0 ? __builtin_nontemporal_load(Hrow + c * kSlotPad + lane) : 0.0;
    h1 = p1 ? __builtin_nontemporal_load(Hrow + c * kSlotPad + lane + 64) : 0.0;
  }
  // cached form, for matrices read repeatedly (the coarsest solve)
  static __device__ inline void load_cached(const double* Hrow, int c, int lane, bool p0, bool p1,
                                            double& h0, double& h1) {
    h0 = p0 ? Hrow[c * kSlotPad + lane] : 0.0;
    h1 = p1 ? Hrow[c * kSlotPad + lane + 64] : 0.0;
  }
};
template <>
struct SweepRows<float> {
  static __device__ inline int slot(int lane, int k) { return 2 * lane + k; }
  static __device__ inline void load(const uint16_t* Hrow, int c, int lane, bool p0, bool p1,
                                     float& h0, float& h1) {
    uint32_t u = (p0 || p1)
                     ? __builtin_nontemporal_load((const uint32_t*)(Hrow + c * kSlotPad + 2 * lane))
                     : 0u;
    h0 = p0 ? bf16_to_f32((uint16_t)(u & 0xFFFFu)) : 0.0f;
    h1 = p1 ? bf16_to_f32((uint16_t)(u >> 16)) : 0.0f;
  }
  static __device__ inline void load_cached(const uint16_t* Hrow, int c, int lane, bool p0,
                                            bool p1, float& h0, float& h1) {
    uint32_t u = (p0 || p1) ? *(const uint32_t*)(Hrow + c * kSlotPad + 2 * lane) : 0u;
    h0 = p0 ? bf16_to_f32((uint16_t)(u & 0xFFFFu)) : 0.0f;
    h1 = p1 ? bf16_to_f32((uint16_t)(u >> 16)) : 0.0f;
  }
};

// Row r of the wave: row_of(r, i) sets i and returns whether the row exists.
// SkipCenter leaves out the diagonal block (the off-diagonal part of the row,
// for Gauss-Seidel).
template <typename V, int R, bool SkipCenter, typename RowOf>
__device__ inline void rows_matvec_g(const LevelView& L, RowOf row_of,
                                     const typename Vec4Of<V>::type* __restrict__ x4, int lane,
                                     V (&y)[R][3]) {
  typedef typename MatOf<V>::type M;
  V h[R][2][9];
  int jp[R][2];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    int i;
    const bool live = row_of(r, i);
    const M* Hrow = MatOf<V>::H(L) + (long long)(live ? i : 0) * kRowStride;
    const int pn = live ? L.nodes[i] : 0;
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if (live)
      for (int q = 0; q < 4; ++q) w[q] = L.pat[4 * i + q];
    bool pr[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int s = SweepRows<V>::slot(lane, k);
      pr[k] = slot_present(w, s) && !(SkipCenter && s == kCenter);
      jp[r][k] = pr[k] ? pn + slot_offset(L.g, s) : -1;
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) SweepRows<V>::load(Hrow, c, lane, pr[0], pr[1], h[r][0][c], h[r][1][c]);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    V a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (jp[r][k] >= 0) {
        const typename Vec4Of<V>::type xv = x4[jp[r][k]];
        const V x0 = xv.x, x1 = xv.y, x2 = xv.z;
        a0 += h[r][k][0] * x0 + h[r][k][1] * x1 + h[r][k][2] * x2;
        a1 += h[r][k][3] * x0 + h[r][k][4] * x1 + h[r][k][5] * x2;
        a2 += h[r][k][6] * x0 + h[r][k][7] * x1 + h[r][k][8] * x2;
      }
    }
    y[r][0] = wave_sum_dpp(a0);
    y[r][1] = wave_sum_dpp(a1);
    y[r][2] = wave_sum_dpp(a2);
  }
}

template <typename V, int R>
__device__ inline void rows_matvec(const LevelView& L, int i0,
                                   const typename Vec4Of<V>::type* __restrict__ x4, int lane,
                                   V (&y)[R][3]) {
  rows_matvec_g<V, R, false>(
      L,
      [&](int r, int& i) {
        i = i0 + r;
        return i < L.n;
      },
      x4, lane, y);
}

// Component c of the dense 4-vector at grid point pn.
template <typename V>
__device__ inline V& comp(typename Vec4Of<V>::type* v4, int pn, int c) {
  return reinterpret_cast<V*>(v4)[4 * (long long)pn + c];
}
template <typename V>
__device__ inline V comp(const typename Vec4Of<V>::type* v4, int pn, int c) {
  return reinterpret_cast<const V*>(v4)[4 * (long long)pn + c];
}

// ---------------------------------------------------------------- RAP
// H^{m+1} = P~^T H^m P~ (Eq. buildMultigrid) with the linear node embedding.
// P = Px (x) Py (x) Pz is a tensor product of 1-D embeddings (child 2J + b of
// coarse J with weight 1 for b = 0 and 1/2 for b = +-1), so the product is
// taken one axis group at a time, each a gather with no atomics:
//   T[(X, Y, z)][(dX, dY, dz)] = sum_{bx, by, bx', by'} w w w w
//        H~[(2X+bx, 2Y+by, z)][(2dX + bx' - bx, 2dY + by' - by, dz)]
// on the half-coarsened grid (x, y coarse, z fine), then
//   H^{m+1}[(X, Y, Z)][(dX, dY, dZ)] = sum_{bz, bz'} w w T[(X, Y, 2Z+bz)][(dX, dY, 2dZ + bz' - bz)].
// Both stay within +-2 per axis.  H~ = Pi H Pi: constrained DOFs have zero
// rows and columns off the diagonal block already, so only the diagonal
// block's constrained entries are masked.  A slot of T or of the coarse row is
// structurally present iff some contributing fine slot is (the symbolic
// R pattern P).  One wave per output row; lane l owns output slots l, l + 64.
constexpr int kRapWaves = 4;
typedef double dvec2 __attribute__((ext_vector_type(2)));

__device__ inline double emb_w(int b) { return b ? 0.5 : 1.0; }

// pattern words of a row from the lanes' presence flags of slots l, l + 64
__device__ inline void ballot_pattern(bool p0, bool p1, uint32_t* out, int lane) {
  const unsigned long long b0 = __ballot(p0), b1 = __ballot(p1);
  if (lane == 0) {
    out[0] = (uint32_t)b0;
    out[1] = (uint32_t)(b0 >> 32);
    out[2] = (uint32_t)b1;
    out[3] = (uint32_t)(b1 >> 32) & ((1u << (kSlots - 96)) - 1u);
  }
}

// The x-y half runs separably, x first: for each child offset by in y the
// x-coarsened row
//   U_by[(dX, sy, dz)] = sum_{bx, bx'} w(bx) w(bx') H~[(2X+bx, 2Y+by, z)][(2dX + bx' - bx, sy, dz)]
// is accumulated in registers while the three child rows (bx = -1, 0, 1) pass
// one at a time through the wave's LDS buffer (coalesced 16-byte loads); U_by
// then replaces the child in the buffer, and
//   T[(dX, dY, dz)] += sum_{by'} w(by) w(by') U_by[(dX, 2dY + by' - by, dz)].
// A U slot is present iff one of its child slots is, a T slot iff one of its
// U slots is: the same set as the direct sum.
__global__ __launch_bounds__(256) void k_rap_xy(LevelView F, LevelView T) {
  __shared__ __attribute__((aligned(16))) double buf_all[kRapWaves][kRowStride];
  __shared__ uint8_t pres_all[kRapWaves][kSlotPad];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = xcd_block(blockIdx.x, gridDim.x) * kRapWaves + wave;
  if (t >= T.n) return;  // the wave only syncs with itself
  double* buf = buf_all[wave];
  uint8_t* pres = pres_all[wave];
  int X, Y, z;
  unpidx(T.g, T.nodes[t], X, Y, z);
  int child = -1;  // fine row of child a = (bx + 1) + 3 (by + 1), in lane a
  if (lane < 9)
    child = F.map[pidx(F.g, 2 * X + lane % 3 - 1, 2 * Y + lane / 3 - 1, z)];
  const int S0 = lane, S1 = lane + 64;
  const bool v1 = S1 < kSlots;
  const int dX0 = S0 % 5 - 2, dY0 = (S0 / 5) % 5 - 2, dz0 = S0 / 25 - 2;
  const int dX1 = S1 % 5 - 2, dY1 = (S1 / 5) % 5 - 2, dz1 = S1 / 25 - 2;
  constexpr int kLd = kRowStride / 128;  // 16-byte loads per lane per row
  double acc0[9], acc1[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) acc0[c] = acc1[c] = 0.0;
  bool p0 = false, p1 = false;
#pragma unroll 1
  for (int by = -1; by <= 1; ++by) {
    double u0[9], u1[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) u0[c] = u1[c] = 0.0;
    bool q0 = false, q1 = false, any = false;
    for (int bx = -1; bx <= 1; ++bx) {
      const int i = __shfl(child, (bx + 1) + 3 * (by + 1), 64);
      if (i < 0) continue;
      any = true;
      const dvec2* src = reinterpret_cast<const dvec2*>(F.H + (long long)i * kRowStride);
      dvec2 ld[kLd];
#pragma unroll
      for (int k = 0; k < kLd; ++k) ld[k] = src[lane + 64 * k];
      const uint32_t w[4] = {F.pat[4 * i], F.pat[4 * i + 1], F.pat[4 * i + 2], F.pat[4 * i + 3]};
      const double f0 = (double)F.free_dof[3 * i], f1 = (double)F.free_dof[3 * i + 1],
                   f2 = (double)F.free_dof[3 * i + 2];
      const double fm[9] = {f0 * f0, f0 * f1, f0 * f2, f1 * f0, f1 * f1, f1 * f2,
                            f2 * f0, f2 * f1, f2 * f2};
      wave_sync();  // earlier reads of the buffer are done
#pragma unroll
      for (int k = 0; k < kLd; ++k) reinterpret_cast<dvec2*>(buf)[lane + 64 * k] = ld[k];
      wave_sync();
      for (int bxp = -1; bxp <= 1; ++bxp) {
        const double wb = emb_w(bx) * emb_w(bxp);
        {
          const int sx = 2 * dX0 + bxp - bx;
          if (sx >= -2 && sx <= 2) {
            const int s = (sx + 2) + 5 * (dY0 + 2) + 25 * (dz0 + 2);
            if (slot_present(w, s)) {
              q0 = true;
              const bool ctr = s == kCenter;
#pragma unroll
              for (int c = 0; c < 9; ++c) {
                const double h = buf[c * kSlotPad + s];
                u0[c] += wb * (ctr ? h * fm[c] : h);
              }
            }
          }
        }
        if (v1) {
          const int sx = 2 * dX1 + bxp - bx;
          if (sx >= -2 && sx <= 2) {
            const int s = (sx + 2) + 5 * (dY1 + 2) + 25 * (dz1 + 2);
            if (slot_present(w, s)) {
              q1 = true;
              const bool ctr = s == kCenter;
#pragma unroll
              for (int c = 0; c < 9; ++c) {
                const double h = buf[c * kSlotPad + s];
                u1[c] += wb * (ctr ? h * fm[c] : h);
              }
            }
          }
        }
      }
    }
    if (!any) continue;  // uniform over the wave
    wave_sync();
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      buf[c * kSlotPad + S0] = u0[c];
      if (v1) buf[c * kSlotPad + S1] = u1[c];
    }
    pres[S0] = q0 ? 1 : 0;
    if (v1) pres[S1] = q1 ? 1 : 0;
    wave_sync();
    for (int byp = -1; byp <= 1; ++byp) {
      const double wy = emb_w(by) * emb_w(byp);
      {
        const int sy = 2 * dY0 + byp - by;
        if (sy >= -2 && sy <= 2) {
          const int s = (dX0 + 2) + 5 * (sy + 2) + 25 * (dz0 + 2);
          if (pres[s]) {
            p0 = true;
#pragma unroll
            for (int c = 0; c < 9; ++c) acc0[c] += wy * buf[c * kSlotPad + s];
          }
        }
      }
      if (v1) {
        const int sy = 2 * dY1 + byp - by;
        if (sy >= -2 && sy <= 2) {
          const int s = (dX1 + 2) + 5 * (sy + 2) + 25 * (dz1 + 2);
          if (pres[s]) {
            p1 = true;
#pragma unroll
            for (int c = 0; c < 9; ++c) acc1[c] += wy * buf[c * kSlotPad + s];
          }
        }
      }
    }
  }
  double* Tout = T.H + (long long)t * kRowStride;
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    Tout[c * kSlotPad + S0] = acc0[c];
    Tout[c * kSlotPad + S1] = v1 ? acc1[c] : 0.0;
  }
  ballot_pattern(p0, p1 && v1, T.pat + 4 * t, lane);
}

// The z half: the three child rows (bz = -1, 0, 1) pass one at a time
// through the wave's LDS buffer (coalesced 16-byte loads), which then holds
// the coarse row for its finalisation.
__global__ __launch_bounds__(256) void k_rap_z(LevelView T, LevelView C) {
  __shared__ __attribute__((aligned(16))) double acc_all[kRapWaves][kRowStride];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int I = xcd_block(blockIdx.x, gridDim.x) * kRapWaves + wave;
  if (I >= C.n) return;  // the wave only syncs with itself
  double* accr = acc_all[wave];
  int X, Y, Z;
  unpidx(C.g, C.nodes[I], X, Y, Z);
  int child = -1;  // half-grid row of child bz = lane - 1, in lanes 0..2
  if (lane < 3) child = T.map[pidx(T.g, X, Y, 2 * Z + lane - 1)];
  const int S0 = lane, S1 = lane + 64;
  const bool v1 = S1 < kSlots;
  const int dX0 = S0 % 5 - 2, dY0 = (S0 / 5) % 5 - 2, dZ0 = S0 / 25 - 2;
  const int dX1 = S1 % 5 - 2, dY1 = (S1 / 5) % 5 - 2, dZ1 = S1 / 25 - 2;
  constexpr int kLd = kRowStride / 128;  // 16-byte loads per lane per row
  double acc0[9], acc1[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) acc0[c] = acc1[c] = 0.0;
  bool p0 = false, p1 = false;
  for (int a = 0; a < 3; ++a) {
    const int tr = __shfl(child, a, 64);
    if (tr < 0) continue;
    const int bz = a - 1;
    const double wa = emb_w(bz);
    const dvec2* src = reinterpret_cast<const dvec2*>(T.H + (long long)tr * kRowStride);
    dvec2 ld[kLd];
#pragma unroll
    for (int k = 0; k < kLd; ++k) ld[k] = src[lane + 64 * k];
    const uint32_t w[4] = {T.pat[4 * tr], T.pat[4 * tr + 1], T.pat[4 * tr + 2], T.pat[4 * tr + 3]};
    wave_sync();  // earlier reads of the buffer are done
#pragma unroll
    for (int k = 0; k < kLd; ++k) reinterpret_cast<dvec2*>(accr)[lane + 64 * k] = ld[k];
    wave_sync();
    for (int bzp = -1; bzp <= 1; ++bzp) {
      const double wb = wa * emb_w(bzp);
      {
        const int sz = 2 * dZ0 + bzp - bz;
        if (sz >= -2 && sz <= 2) {
          const int s = (dX0 + 2) + 5 * (dY0 + 2) + 25 * (sz + 2);
          if (slot_present(w, s)) {
            p0 = true;
#pragma unroll
            for (int c = 0; c < 9; ++c) acc0[c] += wb * accr[c * kSlotPad + s];
          }
        }
      }
      if (v1) {
        const int sz = 2 * dZ1 + bzp - bz;
        if (sz >= -2 && sz <= 2) {
          const int s = (dX1 + 2) + 5 * (dY1 + 2) + 25 * (sz + 2);
          if (slot_present(w, s)) {
            p1 = true;
#pragma unroll
            for (int c = 0; c < 9; ++c) acc1[c] += wb * accr[c * kSlotPad + s];
          }
        }
      }
    }
  }
  wave_sync();  // the last child row is no longer read
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    accr[c * kSlotPad + S0] = acc0[c];
    accr[c * kSlotPad + S1] = v1 ? acc1[c] : 0.0;
  }
  ballot_pattern(p0, p1 && v1, C.pat + 4 * I, lane);
  wave_sync();
  finalize_row(accr, I, C, nullptr, 0.0, lane);
}

__global__ void k_to_bf16(LevelView L) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long nv = (long long)L.n * kRowStride;
  if (k < nv) L.Hb[k] = f32_to_bf16((float)L.H[k]);
  if (k < (long long)L.n * 9) L.Dinv32[k] = (float)L.Dinv[k];
  if (k < (long long)L.n * 3) L.diag32[k] = (float)L.diag[k];
}

// ---------------------------------------------------------------- V-cycle
// First smoothing sweep from u = 0: u = D~^{-1} b (u dense).
template <typename V>
__global__ void k_jacobi_first(LevelView L, const V* __restrict__ b,
                               typename Vec4Of<V>::type* __restrict__ u4) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  const V* Di = MatOf<V>::Dinv(L) + 9 * (long long)i;
  V b0 = b[3 * i], b1 = b[3 * i + 1], b2 = b[3 * i + 2];
  typename Vec4Of<V>::type o;
  o.x = Di[0] * b0 + Di[1] * b1 + Di[2] * b2;
  o.y = Di[3] * b0 + Di[4] * b1 + Di[5] * b2;
  o.z = Di[6] * b0 + Di[7] * b1 + Di[8] * b2;
  o.w = 0;
  u4[L.nodes[i]] = o;
}

constexpr int kRowWaves = 4;

// r = b - H u (one wave per R consecutive rows; u dense, r compact)
template <typename V, int R>
__global__ __launch_bounds__(256) void k_residual(LevelView L, const V* __restrict__ b,
                                                  const typename Vec4Of<V>::type* __restrict__ u4,
                                                  V* __restrict__ r) {
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int i0 = (xcd_block(blockIdx.x, gridDim.x) * kRowWaves + wave) * R;
  if (i0 >= L.n) return;
  // the output lane's b entry is loaded before the product, off its path
  const int rr = lane / 3, c = lane - 3 * rr;
  const int i = i0 + rr;
  const bool out = lane < 3 * R && i < L.n;
  const V bv = out ? b[3 * i + c] : (V)0;
  V y[R][3];
  rows_matvec<V, R>(L, i0, u4, lane, y);
  if (out) {
    V yv = y[0][0];
#pragma unroll
    for (int q = 0; q < R; ++q)
      for (int e = 0; e < 3; ++e)
        if (q == rr && e == c) yv = y[q][e];
    r[3 * i + c] = bv - yv;
  }
}

// l1 block-Jacobi sweep: u_out = u + D~^{-1} (b - H u), projected (u, u_out
// dense).
template <typename V, int R>
__global__ __launch_bounds__(256) void k_smooth(LevelView L, const V* __restrict__ b,
                                                const typename Vec4Of<V>::type* __restrict__ u4,
                                                typename Vec4Of<V>::type* __restrict__ uo4) {
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int i0 = (xcd_block(blockIdx.x, gridDim.x) * kRowWaves + wave) * R;
  if (i0 >= L.n) return;
  V y[R][3];
  rows_matvec<V, R>(L, i0, u4, lane, y);
  if (lane < 3 * R) {
    const int rr = lane / 3, c = lane - 3 * rr;
    const int i = i0 + rr;
    V y0 = y[0][0], y1 = y[0][1], y2 = y[0][2];
#pragma unroll
    for (int q = 1; q < R; ++q)
      if (q == rr) {
        y0 = y[q][0];
        y1 = y[q][1];
        y2 = y[q][2];
      }
    if (i < L.n) {
      const int pn = L.nodes[i];
      const V* Di = MatOf<V>::Dinv(L) + 9 * (long long)i;
      V r0 = b[3 * i] - y0, r1 = b[3 * i + 1] - y1, r2 = b[3 * i + 2] - y2;
      V upd = Di[3 * c] * r0 + Di[3 * c + 1] * r1 + Di[3 * c + 2] * r2;
      V out = comp<V>(u4, pn, c) + upd;
      comp<V>(uo4, pn, c) = L.free_dof[3 * i + c] ? out : (V)0;
    }
  }
}

// ---------------------------------------------------------------- sweeps over x-runs
// Large levels: a work-group of four waves takes kRunRows consecutive rows.
// Rows are ordered x fastest, so away from the edges of the active set these
// are one run of consecutive grid points along x, whose 125-point stencils
// together cover a window of 25 lines (dy, dz) of kRunRows + 4 points.  The
// work-group loads that window of the iterate, and the rows' pattern words,
// right-hand sides, block-Jacobi inverses and free flags, into LDS with
// contiguous loads; a row then reads only its blocks from memory.  (A sweep
// that gathers the neighbour values per row issues two 64-address gathers
// and about eight small loads per row, which in the BF16 sweeps keep the
// vector-memory address units about 80% busy.)  A work-group whose rows are
// not one run gathers the neighbour values from memory.  Every row's
// arithmetic is that of rows_matvec and k_smooth / k_residual, in the same
// order (identical bits).
constexpr int kRunRows = 16;
constexpr int kRunWin = kRunRows + 4;  // window points per line
template <typename V>
struct RunRows;  // rows per wave per pass
template <>
struct RunRows<float> {
  static constexpr int R = 4;
};
template <>
struct RunRows<double> {
  static constexpr int R = 1;
};

template <typename V, bool Smooth>
__global__ __launch_bounds__(256) void k_sweep_run(LevelView L, const V* __restrict__ b,
                                                   const typename Vec4Of<V>::type* __restrict__ u4,
                                                   typename Vec4Of<V>::type* __restrict__ uo4,
                                                   V* __restrict__ rout) {
  typedef typename Vec4Of<V>::type V4;
  typedef typename MatOf<V>::type M;
  constexpr int R = RunRows<V>::R;
  static_assert(9 * kRunRows <= 256 && kRunRows <= 64, "staging assumes one pass per array");
  static_assert(kRunRows % (kRowWaves * R) == 0, "rows split evenly over the waves");
  __shared__ V4 win[25 * kRunWin];
  __shared__ uint4 spat[kRunRows];
  __shared__ int spn[kRunRows];
  __shared__ V sb[3 * kRunRows];
  __shared__ V sd[Smooth ? 9 * kRunRows : 1];
  __shared__ uint8_t sf[Smooth ? 3 * kRunRows : 1];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int i0 = xcd_block(blockIdx.x, gridDim.x) * kRunRows;
  const int nr = min(kRunRows, L.n - i0);
  if (tid < nr) {
    spat[tid] = reinterpret_cast<const uint4*>(L.pat)[i0 + tid];
    spn[tid] = L.nodes[i0 + tid];
  }
  if (tid < 3 * nr) {
    sb[tid] = b[3 * (long long)i0 + tid];
    if (Smooth) sf[tid] = L.free_dof[3 * (long long)i0 + tid];
  }
  if (Smooth && tid < 9 * nr) sd[tid] = MatOf<V>::Dinv(L)[9 * (long long)i0 + tid];
  __syncthreads();
  const int pn0 = spn[0];
  const bool run = __ballot(lane >= nr || spn[min(lane, kRunRows - 1)] == pn0 + lane) == ~0ull;
  if (run) {
    // the window: points pn0 - 2 .. pn0 + nr + 1 of the 25 lines (dy, dz),
    // all inside the padded grid
    const int nw = nr + 4;
    for (int e = tid; e < 25 * nw; e += 256) {
      const int line = e / nw, xo = e - line * nw;
      const long long p = (long long)pn0 + (xo - 2) +
                          (long long)L.g.pd[0] * ((line % 5 - 2) + (long long)L.g.pd[1] * (line / 5 - 2));
      win[line * kRunWin + xo] = u4[p];
    }
  }
  __syncthreads();
  // this lane's two slots: window line offset and x offset
  int sl[2], sx[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int s = SweepRows<V>::slot(lane, k);
    sl[k] = (s / 5) * kRunWin;
    sx[k] = s % 5;
  }
#pragma unroll 1
  for (int t0 = wave * (kRunRows / kRowWaves); t0 < (wave + 1) * (kRunRows / kRowWaves); t0 += R) {
    if (t0 >= nr) break;
    V h[R][2][9];
    bool pr[R][2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int t = t0 + r;
      const bool live = t < nr;
      const M* Hrow = MatOf<V>::H(L) + (long long)(i0 + (live ? t : 0)) * kRowStride;
      const uint4 pw = live ? spat[t] : make_uint4(0u, 0u, 0u, 0u);
      const uint32_t w[4] = {pw.x, pw.y, pw.z, pw.w};
#pragma unroll
      for (int k = 0; k < 2; ++k) pr[r][k] = slot_present(w, SweepRows<V>::slot(lane, k));
#pragma unroll
      for (int c = 0; c < 9; ++c)
        SweepRows<V>::load(Hrow, c, lane, pr[r][0], pr[r][1], h[r][0][c], h[r][1][c]);
    }
    V y[R][3];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int t = t0 + r;
      V a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        if (pr[r][k]) {
          const V4 xv = run ? win[sl[k] + t + sx[k]]
                            : u4[spn[t] + slot_offset(L.g, SweepRows<V>::slot(lane, k))];
          const V x0 = xv.x, x1 = xv.y, x2 = xv.z;
          a0 += h[r][k][0] * x0 + h[r][k][1] * x1 + h[r][k][2] * x2;
          a1 += h[r][k][3] * x0 + h[r][k][4] * x1 + h[r][k][5] * x2;
          a2 += h[r][k][6] * x0 + h[r][k][7] * x1 + h[r][k][8] * x2;
        }
      }
      y[r][0] = wave_sum_dpp(a0);
      y[r][1] = wave_sum_dpp(a1);
      y[r][2] = wave_sum_dpp(a2);
    }
    if (lane < 3 * R) {
      const int rr = lane / 3, c = lane - 3 * rr;
      const int t = t0 + rr;
      V y0 = y[0][0], y1 = y[0][1], y2 = y[0][2];
#pragma unroll
      for (int q = 1; q < R; ++q)
        if (q == rr) {
          y0 = y[q][0];
          y1 = y[q][1];
          y2 = y[q][2];
        }
      if (t < nr) {
        const long long i = i0 + t;
        if (Smooth) {
          const int pn = spn[t];
          const V* Di = sd + 9 * t;
          const V r0 = sb[3 * t] - y0, r1 = sb[3 * t + 1] - y1, r2 = sb[3 * t + 2] - y2;
          const V upd = Di[3 * c] * r0 + Di[3 * c + 1] * r1 + Di[3 * c + 2] * r2;
          const V uc = run ? reinterpret_cast<const V*>(win + 12 * kRunWin + t + 2)[c]
                           : comp<V>(u4, pn, c);
          const V out = uc + upd;
          comp<V>(uo4, pn, c) = sf[3 * t + c] ? out : (V)0;
        } else {
          const V yv = c == 0 ? y0 : (c == 1 ? y1 : y2);
          rout[3 * i + c] = sb[3 * t + c] - yv;
        }
      }
    }
  }
}

// ---------------------------------------------------------------- coloured Gauss-Seidel
// Symmetric block Gauss-Seidel (Alg. V-cycle smoother; Sec. 5.3 and Sec. 8
// colour it for parallelism).  Nodes are coloured by their grid coordinate
// mod 3 per axis (27 colours); a row couples nodes at most 2 apart per axis,
// so rows of one colour never see each other and a colour is one parallel,
// in-place pass.  A forward pass runs the colours 0..26, a backward pass
// 26..0.  Per level and step: the rows of each colour (ascending row index)
// and the inverses of the rows' 3x3 diagonal blocks.
constexpr int kColorChunk = 256;  // rows per block of the colour counting

__device__ inline int node_color(const GridGeom& g, int pn) {
  int x, y, z;
  unpidx(g, pn, x, y, z);
  return x % 3 + 3 * (y % 3) + 9 * (z % 3);
}

// per-chunk colour counts, in row order (one thread walks the chunk)
__global__ void k_color_counts(LevelView L, int* __restrict__ bc) {
  const int r0 = blockIdx.x * kColorChunk, r1 = min(L.n, r0 + kColorChunk);
  if (threadIdx.x < kColors) bc[blockIdx.x * kColors + threadIdx.x] = 0;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int i = r0; i < r1; ++i) bc[blockIdx.x * kColors + node_color(L.g, L.nodes[i])] += 1;
}

// Exclusive offsets: coff[c] = first position of colour c (coff[27] = n);
// bc[b][c] becomes the first position of chunk b's rows of colour c.
__global__ void k_color_offsets(int nchunks, int* __restrict__ bc, int* __restrict__ coff) {
  __shared__ int tot[kColors];
  const int c = threadIdx.x;
  if (c < kColors) {
    int run = 0;
    for (int b = 0; b < nchunks; ++b) {
      const int v = bc[b * kColors + c];
      bc[b * kColors + c] = run;
      run += v;
    }
    tot[c] = run;
  }
  __syncthreads();
  if (c == 0) {
    int run = 0;
    for (int k = 0; k < kColors; ++k) {
      coff[k] = run;
      run += tot[k];
    }
    coff[kColors] = run;
  }
  __syncthreads();
  if (c < kColors) {
    const int base = coff[c];
    for (int b = 0; b < nchunks; ++b) bc[b * kColors + c] += base;
  }
}

__global__ void k_color_scatter(LevelView L, const int* __restrict__ bc, int* __restrict__ rows) {
  __shared__ int cur[kColors];
  const int r0 = blockIdx.x * kColorChunk, r1 = min(L.n, r0 + kColorChunk);
  if (threadIdx.x < kColors) cur[threadIdx.x] = bc[blockIdx.x * kColors + threadIdx.x];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int i = r0; i < r1; ++i) rows[cur[node_color(L.g, L.nodes[i])]++] = i;
}

// Inverses of the 3x3 diagonal blocks (FP64, and FP32 copies in mixed mode).
__global__ void k_block_diag_inv(LevelView L, double* __restrict__ Dg, float* __restrict__ Dg32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  const double* Hrow = L.H + (long long)i * kRowStride;
  double A[9], B[9];
  for (int c = 0; c < 9; ++c) A[c] = Hrow[c * kSlotPad + kCenter];
  inv3(A, B);
  for (int c = 0; c < 9; ++c) {
    Dg[9 * (long long)i + c] = B[c];
    if (Dg32) Dg32[9 * (long long)i + c] = (float)B[c];
  }
}

// u at the level's active nodes set to zero (start of the down-sweep).
template <typename V>
__global__ void k_zero_rows(LevelView L, typename Vec4Of<V>::type* __restrict__ u4) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  typename Vec4Of<V>::type z;
  z.x = z.y = z.z = z.w = 0;
  u4[L.nodes[i]] = z;
}

// One colour of a pass: for the colour's rows i (rows[0..cnt)),
// u_i = H_ii^{-1} (b_i - sum_{j != i} H_ij u_j), in place on the dense iterate,
// projected on the free DOFs.  R rows per wave with their loads in flight, as
// in the sweeps.
template <typename V, int R>
__global__ __launch_bounds__(256) void k_sgs_color(LevelView L, const int* __restrict__ rows,
                                                   int cnt, const V* __restrict__ Dg,
                                                   const V* __restrict__ b,
                                                   typename Vec4Of<V>::type* __restrict__ u4) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int k0 = (xcd_block(blockIdx.x, gridDim.x) * kRowWaves + wave) * R;
  if (k0 >= cnt) return;
  V y[R][3];
  rows_matvec_g<V, R, true>(
      L,
      [&](int r, int& i) {
        const bool live = k0 + r < cnt;
        i = live ? rows[k0 + r] : 0;
        return live;
      },
      u4, lane, y);
  if (lane < 3 * R) {
    const int rr = lane / 3, c = lane - 3 * rr;
    V y0 = y[0][0], y1 = y[0][1], y2 = y[0][2];
#pragma unroll
    for (int q = 1; q < R; ++q)
      if (q == rr) {
        y0 = y[q][0];
        y1 = y[q][1];
        y2 = y[q][2];
      }
    if (k0 + rr < cnt) {
      const int i = rows[k0 + rr];
      const V* Di = Dg + 9 * (long long)i;
      const V r0 = b[3 * i] - y0, r1 = b[3 * i + 1] - y1, r2 = b[3 * i + 2] - y2;
      const V v = Di[3 * c] * r0 + Di[3 * c + 1] * r1 + Di[3 * c + 2] * r2;
      comp<V>(u4, L.nodes[i], c) = L.free_dof[3 * i + c] ? v : (V)0;
    }
  }
}

// b^{m+1}_J = sum_i P~_iJ r_i over the 27 fine children of J.  Half a wave
// per coarse node, one lane per child, then a fixed-order reduction over the
// half-wave (a thread per coarse node leaves most of the device idle on the
// small coarse grids).
template <typename V>
__global__ __launch_bounds__(256) void k_restrict(LevelView F, LevelView C,
                                                  const V* __restrict__ r, V* __restrict__ bc,
                                                  typename Vec4Of<V>::type* __restrict__ uc4) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int a = lane & 31;
  const int J = ((blockIdx.x * 4 + wave) << 1) + (lane >> 5);
  V s0 = 0, s1 = 0, s2 = 0;
  if (J < C.n && a < 27) {
    int X, Y, Z;
    unpidx(C.g, C.nodes[J], X, Y, Z);
    const int ax = a % 3 - 1, ay = (a / 3) % 3 - 1, az = a / 9 - 1;
    const int i = F.map[pidx(F.g, 2 * X + ax, 2 * Y + ay, 2 * Z + az)];
    if (i >= 0) {
      const V w = (V)((ax ? 0.5 : 1.0) * (ay ? 0.5 : 1.0) * (az ? 0.5 : 1.0));
      s0 = F.free_dof[3 * i] ? w * r[3 * i] : (V)0;
      s1 = F.free_dof[3 * i + 1] ? w * r[3 * i + 1] : (V)0;
      s2 = F.free_dof[3 * i + 2] ? w * r[3 * i + 2] : (V)0;
    }
  }
  for (int off = 16; off > 0; off >>= 1) {
    s0 += __shfl_xor(s0, off, 64);
    s1 += __shfl_xor(s1, off, 64);
    s2 += __shfl_xor(s2, off, 64);
  }
  if (a == 0 && J < C.n) {
    bc[3 * J] = s0;
    bc[3 * J + 1] = s1;
    bc[3 * J + 2] = s2;
    if (uc4) {  // the coarse level's first smoothing from zero, as k_jacobi_first
      const V* Di = MatOf<V>::Dinv(C) + 9 * (long long)J;
      typename Vec4Of<V>::type o;
      o.x = Di[0] * s0 + Di[1] * s1 + Di[2] * s2;
      o.y = Di[3] * s0 + Di[4] * s1 + Di[5] * s2;
      o.z = Di[6] * s0 + Di[7] * s1 + Di[8] * s2;
      o.w = 0;
      uc4[C.nodes[J]] = o;
    }
  }
}

// u_i += sum_J P~_iJ u^c_J over the (at most 8) parents of fine node i (both
// dense: a parent's grid index needs no map lookup).
template <typename V>
__global__ void k_prolong_add(LevelView F, LevelView C,
                              const typename Vec4Of<V>::type* __restrict__ uc4,
                              typename Vec4Of<V>::type* __restrict__ u4) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= F.n) return;
  const int pn = F.nodes[i];
  int x, y, z;
  unpidx(F.g, pn, x, y, z);
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
        const typename Vec4Of<V>::type v = uc4[pidx(C.g, Px[a], Py[b], Pz[c])];
        V w = wx[a] * wy[b] * wz[c];
        s0 += w * v.x;
        s1 += w * v.y;
        s2 += w * v.z;
      }
  if (F.free_dof[3 * i]) comp<V>(u4, pn, 0) += s0;
  if (F.free_dof[3 * i + 1]) comp<V>(u4, pn, 1) += s1;
  if (F.free_dof[3 * i + 2]) comp<V>(u4, pn, 2) += s2;
}

// Level-0 iterate (dense) to the compact FP64 output of the cycle.
template <typename V>
__global__ void k_dense_out(LevelView L, const typename Vec4Of<V>::type* __restrict__ u4,
                            double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  const typename Vec4Of<V>::type v = u4[L.nodes[i]];
  out[3 * i] = (double)v.x;
  out[3 * i + 1] = (double)v.y;
  out[3 * i + 2] = (double)v.z;
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

// y_r = H_{i0+r} . x for R consecutive rows with x compact [n][3] in LDS
// (neighbour rows through the level map); same lane roles and summation order
// as rows_matvec.
template <typename V, int R>
__device__ inline void rows_matvec_lds(const LevelView& L, int i0, const V* xs, int lane,
                                       V (&y)[R][3]) {
  typedef typename MatOf<V>::type M;
  V h[R][2][9];
  int jn[R][2];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = i0 + r;
    const bool live = i < L.n;
    const M* Hrow = MatOf<V>::H(L) + (long long)(live ? i : 0) * kRowStride;
    const int pn = live ? L.nodes[i] : 0;
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if (live)
      for (int q = 0; q < 4; ++q) w[q] = L.pat[4 * i + q];
    bool pr[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int s = SweepRows<V>::slot(lane, k);
      pr[k] = slot_present(w, s);
      jn[r][k] = pr[k] ? L.map[pn + slot_offset(L.g, s)] : -1;
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) SweepRows<V>::load_cached(Hrow, c, lane, pr[0], pr[1], h[r][0][c], h[r][1][c]);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    V a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (jn[r][k] >= 0) {
        const V* xj = xs + 3 * jn[r][k];
        const V x0 = xj[0], x1 = xj[1], x2 = xj[2];
        a0 += h[r][k][0] * x0 + h[r][k][1] * x1 + h[r][k][2] * x2;
        a1 += h[r][k][3] * x0 + h[r][k][4] * x1 + h[r][k][5] * x2;
        a2 += h[r][k][6] * x0 + h[r][k][7] * x1 + h[r][k][8] * x2;
      }
    }
    y[r][0] = wave_sum_t(a0);
    y[r][1] = wave_sum_t(a1);
    y[r][2] = wave_sum_t(a2);
  }
}

// Single work-group form for coarsest levels whose five CG vectors fit in
// LDS: r, z, p, q, x live in LDS, rows are processed several per wave (as in
// the sweeps) with all their loads in flight, and inner products are block
// reductions; no memory traffic leaves the compute unit except the matrix and
// map reads.
constexpr size_t kPcgLdsMax = 60 * 1024;

template <typename V>
__global__ __launch_bounds__(kPcgThreads) void k_coarse_pcg(
    LevelView L, const V* __restrict__ b, typename Vec4Of<V>::type* __restrict__ x4,
    IterLog lg, int max_iter, double rel) {
  extern __shared__ __attribute__((aligned(16))) unsigned char pcg_lds[];
  __shared__ V red[kPcgWaves];
  const int n3 = 3 * L.n;
  V* r = reinterpret_cast<V*>(pcg_lds);
  V* z = r + n3;
  V* p = z + n3;
  V* q = p + n3;
  V* x = q + n3;
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
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // rows per wave of the single-work-group solve: its 16 waves need several
  // rows each in flight
  constexpr int kPcgRows = sizeof(V) == 4 ? 4 : 2;
  if (rz > (V)0) {
    while (it < max_iter) {
      __syncthreads();
      for (int row0 = wave * kPcgRows; row0 < L.n; row0 += kPcgWaves * kPcgRows) {
        V y[kPcgRows][3];
        rows_matvec_lds<V, kPcgRows>(L, row0, p, lane, y);
        if (lane < 3 * kPcgRows) {
          const int rr = lane / 3, c = lane - 3 * rr;
          V yv = y[0][0];
#pragma unroll
          for (int qq = 0; qq < kPcgRows; ++qq)
            for (int e = 0; e < 3; ++e)
              if (qq == rr && e == c) yv = y[qq][e];
          if (row0 + rr < L.n) q[3 * (row0 + rr) + c] = yv;
        }
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
  __syncthreads();
  for (int k = threadIdx.x; k < n3; k += kPcgThreads) comp<V>(x4, L.nodes[k / 3], k % 3) = x[k];
  if (threadIdx.x == 0) log_iters(lg, it);
}

__global__ __launch_bounds__(256) void k_spmv(LevelView L, const double* __restrict__ x,
                                              double* __restrict__ y) {
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int i = xcd_block(blockIdx.x, gridDim.x) * kRowWaves + wave;
  if (i >= L.n) return;
  double v[3];
  row_matvec<double>(L, i, x, lane, v);
  if (lane < 3) y[3 * i + lane] = v[lane];
}

// Multi-work-group form of the same solve for larger coarsest levels: one
// wave per row (rows strided over all waves of the grid), the same update
// formulas, and fixed-order two-stage inner products (per-block partials,
// then every block sums the partials in block order).  Blocks meet at a
// software grid barrier, so all blocks must be resident at once.  The grid is
// kept small (at most kCgMaxBlocks, and at most 1/16 of the device's resident
// block capacity), so that even 16 such solves running concurrently from
// different streams, plus any finite kernels, cannot hold all block slots
// while a block of one of them waits to start.  Every wait is still bounded:
// a barrier that does not complete within the spin limit raises a flag that
// makes every block leave, and the solve reports a negative iteration count.
constexpr int kCgWaves = 8;
constexpr int kCgMaxBlocks = 32;
constexpr unsigned kSpinLimit = 1u << 22;

// Barrier state: the generation each block has reached (one word per
// block) and a failure flag.
struct GridBar {
  unsigned flag[kCgMaxBlocks];
  int fail;
  int pad[3];
};
static_assert(kCgMaxBlocks <= 64, "one wave polls every block's flag");

// Each block publishes the generation it has reached in its own word (one
// release store) and its first wave polls every block's word with one
// relaxed wave-wide load until all have reached it, then acquires.  No
// read-modify-write atomics, so arrivals are not serialised on one address,
// and the polls do not invalidate the caches that the other blocks are
// reading the level matrix through.  A block can be at most one generation
// ahead of a poller (it cannot pass the next barrier without the poller), so
// "reached" is flag - target >= 0.
__device__ inline bool grid_sync(GridBar* bar, unsigned nblocks, unsigned& gen, int* s_ok) {
  __syncthreads();
  const unsigned target = gen + 1u;
  if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    if (l == 0)
      __hip_atomic_store(&bar->flag[blockIdx.x], target, __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    unsigned spins = 0;
    for (;;) {
      const unsigned v =
          l < (int)nblocks
              ? __hip_atomic_load(&bar->flag[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
              : target;
      const int f = __hip_atomic_load(&bar->fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (__ballot((int)(v - target) >= 0) == ~0ull) break;
      if (__ballot(f != 0) != 0ull || ++spins > kSpinLimit) {
        if (l == 0) __hip_atomic_store(&bar->fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (l == 0) *s_ok = ok;
  }
  __syncthreads();
  gen = target;
  return *s_ok != 0;
}

// Sum of the per-block partials in block order, valid in every thread.
__device__ inline double grid_total(const double* part, int nb, double* s_val) {
  if (threadIdx.x < 64) {
    double t = 0.0;
    for (int k = threadIdx.x; k < nb; k += 64) t += part[k];
    t = wave_sum_t(t);
    if (threadIdx.x == 0) *s_val = t;
  }
  __syncthreads();
  double v = *s_val;
  __syncthreads();
  return v;
}

// Block-level partial of per-lane values (fixed order) written to part[block].
__device__ inline void block_partial(double loc, double* part, double* red) {
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  loc = wave_sum_t(loc);
  if (lane == 0) red[wave] = loc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kCgWaves; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

template <typename V>
__global__ __launch_bounds__(kCgWaves * 64) void k_coarse_pcg_grid(
    LevelView L, const V* __restrict__ b, typename Vec4Of<V>::type* __restrict__ x4,
    V* __restrict__ work, double* __restrict__ part, GridBar* __restrict__ bar,
    IterLog lg, int max_iter, double rel) {
  __shared__ double red[kCgWaves];
  __shared__ double s_val;
  __shared__ int s_ok;
  const int n = L.n, n3 = 3 * n;
  V* r = work;
  V* z = r + n3;
  V* pa = z + n3;  // direction read by this iteration's product
  V* pb = pa + n3; // direction written by this iteration
  V* q = pb + n3;
  V* x = q + n3;  // compact iterate, scattered to the dense x4 at the end
  double* part_pq = part;
  double* part_rz = part + kCgMaxBlocks;
  const V* dg = MatOf<V>::diag(L);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nb = gridDim.x;
  const int gw = blockIdx.x * kCgWaves + wave, nw = nb * kCgWaves;
  unsigned gen = 0;
  double loc = 0.0;
  for (int row = gw; row < n; row += nw)
    if (lane < 3) {
      const int k = 3 * row + lane;
      V bk = b[k];
      x[k] = 0;
      r[k] = bk;
      V zk = bk / dg[k];
      z[k] = zk;
      pa[k] = zk;
      loc += (double)(bk * zk);
    }
  block_partial(loc, part_rz, red);
  int it = 0;
  bool ok = grid_sync(bar, nb, gen, &s_ok);
  double rz = ok ? grid_total(part_rz, nb, &s_val) : 0.0;
  const double stop = rel * sqrt(fmax(rz, 0.0));
  // The direction update p = z + beta p is formed on the fly wherever p is
  // read (the product's gathers and the block's own rows) from z and the
  // previous p, both complete at the last barrier; each block stores its own
  // rows of the new p in the other buffer.  Two barriers per iteration, the
  // same arithmetic as the textbook ordering.
  V beta = 0;
  bool first = true;
  if (ok && rz > 0.0) {
    while (it < max_iter) {
      loc = 0.0;
      for (int row = gw; row < n; row += nw) {
        V y[3];
        if (first)
          row_matvec<V>(L, row, pa, lane, y);
        else
          row_matvec_with<V>(L, row, lane, y, [&](long long j, V& x0, V& x1, V& x2) {
            const long long k = 3 * j;
            x0 = z[k] + beta * pa[k];
            x1 = z[k + 1] + beta * pa[k + 1];
            x2 = z[k + 2] + beta * pa[k + 2];
          });
        if (lane < 3) {
          const int k = 3 * row + lane;
          const V pk = first ? pa[k] : z[k] + beta * pa[k];
          pb[k] = pk;
          q[k] = y[lane];
          loc += (double)(pk * y[lane]);
        }
      }
      block_partial(loc, part_pq, red);
      if (!(ok = grid_sync(bar, nb, gen, &s_ok))) break;
      const double pq = grid_total(part_pq, nb, &s_val);
      if (!(pq > 0.0)) break;
      const V alpha = (V)(rz / pq);
      loc = 0.0;
      for (int row = gw; row < n; row += nw)
        if (lane < 3) {
          const int k = 3 * row + lane;
          x[k] += alpha * pb[k];
          V rk = r[k] - alpha * q[k];
          r[k] = rk;
          V zk = rk / dg[k];
          z[k] = zk;
          loc += (double)(rk * zk);
        }
      block_partial(loc, part_rz, red);
      if (!(ok = grid_sync(bar, nb, gen, &s_ok))) break;
      const double rzn = grid_total(part_rz, nb, &s_val);
      ++it;
      if (sqrt(fmax(rzn, 0.0)) <= stop) break;
      beta = (V)(rzn / rz);
      rz = rzn;
      V* t = pa;
      pa = pb;
      pb = t;
      first = false;
    }
  }
  for (int row = gw; row < n; row += nw)
    if (lane < 3) comp<V>(x4, L.nodes[row], lane) = x[3 * row + lane];
  if (blockIdx.x == 0 && threadIdx.x == 0) log_iters(lg, ok ? it : -1);
}

// Register-resident form of the grid solve for coarsest levels of at most R
// rows per wave (row gw + k nw, k < R, as in the strided loops above): each
// wave loads its rows' blocks and neighbour indices once per solve and keeps
// them, with its rows' entries of r, x, z, p, q and the diagonal, in
// registers.  Only z and p, which other waves gather, go through memory.  The
// arithmetic and the order of every sum are those of k_coarse_pcg_grid.
template <typename V, int R>
__global__ __launch_bounds__(kCgWaves * 64) void k_coarse_pcg_reg(
    LevelView L, const V* __restrict__ b, typename Vec4Of<V>::type* __restrict__ x4,
    V* __restrict__ work, double* __restrict__ part, GridBar* __restrict__ bar,
    IterLog lg, int max_iter, double rel) {
  __shared__ double red[kCgWaves];
  __shared__ double s_val;
  __shared__ int s_ok;
  const int n = L.n, n3 = 3 * n;
  V* z = work;
  V* pa = z + n3;  // direction read by this iteration's product
  V* pb = pa + n3; // direction written by this iteration
  double* part_pq = part;
  double* part_rz = part + kCgMaxBlocks;
  const V* dg = MatOf<V>::diag(L);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nb = gridDim.x;
  const int gw = blockIdx.x * kCgWaves + wave, nw = nb * kCgWaves;
  const int c3 = lane < 3 ? lane : 0;
  RowBlocks<V> rows[R];
  V rr[R], xx[R], zz[R], dd[R], pp[R], qq[R];
  double loc = 0.0;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int row = gw + k * nw;
    rr[k] = xx[k] = zz[k] = pp[k] = qq[k] = 0;
    dd[k] = 1;
    if (row < n) {
      row_load<V>(L, row, lane, rows[k]);
      if (lane < 3) {
        const int kk = 3 * row + lane;
        const V bk = b[kk];
        dd[k] = dg[kk];
        rr[k] = bk;
        const V zk = bk / dd[k];
        zz[k] = zk;
        pp[k] = zk;
        z[kk] = zk;
        pa[kk] = zk;
        loc += (double)(bk * zk);
      }
    }
  }
  block_partial(loc, part_rz, red);
  int it = 0;
  unsigned gen = 0;
  bool ok = grid_sync(bar, nb, gen, &s_ok);
  double rz = ok ? grid_total(part_rz, nb, &s_val) : 0.0;
  const double stop = rel * sqrt(fmax(rz, 0.0));
  V beta = 0;
  bool first = true;
  if (ok && rz > 0.0) {
    while (it < max_iter) {
      loc = 0.0;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int row = gw + k * nw;
        if (row < n) {
          V y[3];
          if (first)
            row_apply<V>(rows[k], y, [&](long long j, V& x0, V& x1, V& x2) {
              const V* xj = pa + 3 * j;
              x0 = xj[0];
              x1 = xj[1];
              x2 = xj[2];
            });
          else
            row_apply<V>(rows[k], y, [&](long long j, V& x0, V& x1, V& x2) {
              const long long kk = 3 * j;
              x0 = z[kk] + beta * pa[kk];
              x1 = z[kk + 1] + beta * pa[kk + 1];
              x2 = z[kk + 2] + beta * pa[kk + 2];
            });
          if (lane < 3) {
            const V yl = c3 == 0 ? y[0] : (c3 == 1 ? y[1] : y[2]);
            const V pk = first ? pp[k] : zz[k] + beta * pp[k];
            pp[k] = pk;
            pb[3 * row + lane] = pk;
            qq[k] = yl;
            loc += (double)(pk * yl);
          }
        }
      }
      block_partial(loc, part_pq, red);
      if (!(ok = grid_sync(bar, nb, gen, &s_ok))) break;
      const double pq = grid_total(part_pq, nb, &s_val);
      if (!(pq > 0.0)) break;
      const V alpha = (V)(rz / pq);
      loc = 0.0;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int row = gw + k * nw;
        if (row < n && lane < 3) {
          xx[k] += alpha * pp[k];
          const V rk = rr[k] - alpha * qq[k];
          rr[k] = rk;
          const V zk = rk / dd[k];
          zz[k] = zk;
          z[3 * row + lane] = zk;
          loc += (double)(rk * zk);
        }
      }
      block_partial(loc, part_rz, red);
      if (!(ok = grid_sync(bar, nb, gen, &s_ok))) break;
      const double rzn = grid_total(part_rz, nb, &s_val);
      ++it;
      if (sqrt(fmax(rzn, 0.0)) <= stop) break;
      beta = (V)(rzn / rz);
      rz = rzn;
      V* t = pa;
      pa = pb;
      pb = t;
      first = false;
    }
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int row = gw + k * nw;
    if (row < n && lane < 3) comp<V>(x4, L.nodes[row], lane) = xx[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) log_iters(lg, ok ? it : -1);
}

__global__ void k_reset_bar(GridBar* bar) {
  if (threadIdx.x < kCgMaxBlocks) bar->flag[threadIdx.x] = 0u;
  if (threadIdx.x == 0) bar->fail = 0;
}

// Rows per wave of the register-resident coarsest solve.
constexpr int kRegRows = 2;

// Grid size of the grid solve (Reg = false: k_coarse_pcg_grid<V>, true:
// k_coarse_pcg_reg<V, kRegRows>) on the current device: 1/16 of the resident
// block capacity, at most kCgMaxBlocks (0 or less if unknown).
template <typename V, bool Reg>
int grid_blocks() {
  static int cached[16] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) return 0;
  if (cached[dev] == 0) {
    int per_cu = 0, cus = 0;
    const void* kern = Reg ? (const void*)k_coarse_pcg_reg<V, kRegRows>
                           : (const void*)k_coarse_pcg_grid<V>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kCgWaves * 64, 0) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cached[dev] = -1;
    else
      cached[dev] = std::max(std::min(per_cu * cus / 16, kCgMaxBlocks), -1);
  }
  return cached[dev];
}

}  // namespace

void launch_rap(const LevelView& F, const LevelView& T, const LevelView& C, hipStream_t st) {
  if (T.n > 0) k_rap_xy<<<(unsigned)((T.n + kRapWaves - 1) / kRapWaves), 256, 0, st>>>(F, T);
  if (C.n > 0) k_rap_z<<<(unsigned)((C.n + kRapWaves - 1) / kRapWaves), 256, 0, st>>>(T, C);
}
void launch_to_bf16(const LevelView& L, hipStream_t st) {
  long long nv = (long long)L.n * kRowStride;
  if (nv > 0) k_to_bf16<<<blocks_for(nv), kTpb, 0, st>>>(L);
}

#define ROWGRID(L) (unsigned)(((L).n + kRowWaves - 1) / kRowWaves), 256, 0, st

void launch_jacobi_first(const LevelView& L, bool mixed, const void* b, void* u, hipStream_t st) {
  if (L.n == 0) return;
  if (mixed)
    k_jacobi_first<float><<<blocks_for(L.n), kTpb, 0, st>>>(L, (const float*)b, (float4*)u);
  else
    k_jacobi_first<double><<<blocks_for(L.n), kTpb, 0, st>>>(L, (const double*)b, (double4*)u);
}
// Sweeps of levels of at least kRunMin rows run over x-runs (k_sweep_run);
// on smaller levels its fewer, longer work-groups leave the device
// under-filled, and one row per wave is faster.  A process-wide override
// (-1: the default) lets a test run either form on any level.
constexpr int kRunMin = 16384;
static std::atomic<int> g_run_min{-1};
inline int run_min() {
  const int v = g_run_min.load(std::memory_order_relaxed);
  return v >= 0 ? v : kRunMin;
}

template <typename V>
void sweep_launch(bool smooth, const LevelView& L, const V* b, const void* u, void* out,
                  hipStream_t st) {
  typedef typename Vec4Of<V>::type V4;
  const V4* u4 = (const V4*)u;
  if (L.n >= run_min()) {
    const unsigned g = (unsigned)((L.n + kRunRows - 1) / kRunRows);
    if (smooth)
      k_sweep_run<V, true><<<g, 256, 0, st>>>(L, b, u4, (V4*)out, nullptr);
    else
      k_sweep_run<V, false><<<g, 256, 0, st>>>(L, b, u4, nullptr, (V*)out);
  } else {
    const unsigned g = (unsigned)((L.n + kRowWaves - 1) / kRowWaves);
    if (smooth)
      k_smooth<V, 1><<<g, 256, 0, st>>>(L, b, u4, (V4*)out);
    else
      k_residual<V, 1><<<g, 256, 0, st>>>(L, b, u4, (V*)out);
  }
}

int set_sweep_run_min(int rows) {
  const int old = g_run_min.exchange(rows < 0 ? -1 : rows);
  return old < 0 ? kRunMin : old;
}

void launch_residual(const LevelView& L, bool mixed, const void* b, const void* u, void* r,
                     hipStream_t st) {
  if (L.n == 0) return;
  if (mixed)
    sweep_launch<float>(false, L, (const float*)b, u, r, st);
  else
    sweep_launch<double>(false, L, (const double*)b, u, r, st);
}
void launch_smooth(const LevelView& L, bool mixed, const void* b, const void* u, void* uo,
                   hipStream_t st) {
  if (L.n == 0) return;
  if (mixed)
    sweep_launch<float>(true, L, (const float*)b, u, uo, st);
  else
    sweep_launch<double>(true, L, (const double*)b, u, uo, st);
}
void launch_restrict(const LevelView& F, const LevelView& C, bool mixed, const void* r, void* bc,
                     void* uc, hipStream_t st) {
  if (C.n == 0) return;
  if (mixed)
    k_restrict<float><<<(unsigned)((C.n + 7) / 8), 256, 0, st>>>(F, C, (const float*)r, (float*)bc,
                                                                (float4*)uc);
  else
    k_restrict<double><<<(unsigned)((C.n + 7) / 8), 256, 0, st>>>(F, C, (const double*)r,
                                                                 (double*)bc, (double4*)uc);
}
void launch_prolong_add(const LevelView& F, const LevelView& C, bool mixed, const void* uc, void* u,
                        hipStream_t st) {
  if (F.n == 0) return;
  if (mixed)
    k_prolong_add<float><<<blocks_for(F.n), kTpb, 0, st>>>(F, C, (const float4*)uc, (float4*)u);
  else
    k_prolong_add<double><<<blocks_for(F.n), kTpb, 0, st>>>(F, C, (const double4*)uc,
                                                            (double4*)u);
}
void launch_dense_out(const LevelView& L, bool mixed, const void* u, double* out, hipStream_t st) {
  if (L.n == 0) return;
  if (mixed)
    k_dense_out<float><<<blocks_for(L.n), kTpb, 0, st>>>(L, (const float4*)u, out);
  else
    k_dense_out<double><<<blocks_for(L.n), kTpb, 0, st>>>(L, (const double4*)u, out);
}


void coarse_pcg_warm() {
  (void)grid_blocks<float, false>();
  (void)grid_blocks<double, false>();
  (void)grid_blocks<float, true>();
  (void)grid_blocks<double, true>();
}

size_t coarse_pcg_work_bytes(int n) {
  return (size_t)6 * 3 * n * sizeof(double) + 256 + 2 * kCgMaxBlocks * sizeof(double) +
         sizeof(GridBar);
}

// Coarsest levels at least this large use the multi-work-group solve.
constexpr int kGridMinRows = 128;

bool coarse_pcg_uses_grid(const LevelView& L, bool mixed) {
  const size_t lds = (size_t)5 * 3 * L.n * (mixed ? sizeof(float) : sizeof(double));
  const int maxb = mixed ? grid_blocks<float, false>() : grid_blocks<double, false>();
  return (L.n >= kGridMinRows || lds > kPcgLdsMax) && maxb >= 2;
}

bool coarse_pcg_single_fits(const LevelView& L, bool mixed) {
  return (size_t)5 * 3 * L.n * (mixed ? sizeof(float) : sizeof(double)) <= kPcgLdsMax;
}

hipError_t launch_coarse_pcg(const LevelView& L, bool mixed, const void* b, void* x, void* work,
                             IterLog lg, int max_iter, double rel, bool grid_ok, hipStream_t st) {
  const size_t vsz = mixed ? sizeof(float) : sizeof(double);
  const size_t lds = (size_t)5 * 3 * L.n * vsz;
  // One work-group streams the whole level matrix through one compute unit
  // per CG iteration, which is limited by that unit's outstanding memory
  // requests: it serves small levels only; levels of kGridMinRows rows or
  // more are read by a grid of work-groups instead, when the caller holds a
  // grid-solve ticket.
  if (!grid_ok || !coarse_pcg_uses_grid(L, mixed)) {
    if (lds > kPcgLdsMax) return hipErrorInvalidConfiguration;
    if (mixed)
      k_coarse_pcg<float><<<1, kPcgThreads, lds, st>>>(L, (const float*)b, (float4*)x, lg,
                                                      max_iter, rel);
    else
      k_coarse_pcg<double><<<1, kPcgThreads, lds, st>>>(L, (const double*)b, (double4*)x,
                                                       lg, max_iter, rel);
    return hipGetLastError();
  }
  const size_t vec = (size_t)6 * 3 * L.n * vsz;
  double* part = (double*)((char*)work + ((vec + 255) / 256) * 256);
  GridBar* bar = (GridBar*)(part + 2 * kCgMaxBlocks);
  const int maxb = mixed ? grid_blocks<float, false>() : grid_blocks<double, false>();
  const int nb = std::max(2, std::min((L.n + kCgWaves - 1) / kCgWaves, maxb));
  k_reset_bar<<<1, 64, 0, st>>>(bar);
  // levels of at most kRegRows rows per wave keep their rows in registers
  const int maxr = mixed ? grid_blocks<float, true>() : grid_blocks<double, true>();
  const int nbr = std::max(2, std::min((L.n + kCgWaves - 1) / kCgWaves, maxr));
  if (maxr >= 2 && L.n <= kRegRows * nbr * kCgWaves) {
    if (mixed)
      k_coarse_pcg_reg<float, kRegRows><<<nbr, kCgWaves * 64, 0, st>>>(
          L, (const float*)b, (float4*)x, (float*)work, part, bar, lg, max_iter, rel);
    else
      k_coarse_pcg_reg<double, kRegRows><<<nbr, kCgWaves * 64, 0, st>>>(
          L, (const double*)b, (double4*)x, (double*)work, part, bar, lg, max_iter, rel);
    return hipGetLastError();
  }
  if (mixed)
    k_coarse_pcg_grid<float><<<nb, kCgWaves * 64, 0, st>>>(L, (const float*)b, (float4*)x,
                                                          (float*)work, part, bar, lg,
                                                          max_iter, rel);
  else
    k_coarse_pcg_grid<double><<<nb, kCgWaves * 64, 0, st>>>(L, (const double*)b, (double4*)x,
                                                           (double*)work, part, bar, lg,
                                                           max_iter, rel);
  return hipGetLastError();
}

size_t color_scratch_bytes(int n) {
  return (size_t)((n + kColorChunk - 1) / kColorChunk + 1) * kColors * sizeof(int) +
         (kColors + 1) * sizeof(int);
}

void launch_color_rows(const LevelView& L, int* scratch, int* coff, int* rows, hipStream_t st) {
  const int nch = (L.n + kColorChunk - 1) / kColorChunk;
  if (L.n == 0) return;
  k_color_counts<<<nch, 64, 0, st>>>(L, scratch);
  k_color_offsets<<<1, 64, 0, st>>>(nch, scratch, coff);
  k_color_scatter<<<nch, 64, 0, st>>>(L, scratch, rows);
}

void launch_block_diag_inv(const LevelView& L, double* Dg, float* Dg32, hipStream_t st) {
  if (L.n > 0) k_block_diag_inv<<<blocks_for(L.n), kTpb, 0, st>>>(L, Dg, Dg32);
}

void launch_zero_rows(const LevelView& L, bool mixed, void* u, hipStream_t st) {
  if (L.n == 0) return;
  if (mixed)
    k_zero_rows<float><<<blocks_for(L.n), kTpb, 0, st>>>(L, (float4*)u);
  else
    k_zero_rows<double><<<blocks_for(L.n), kTpb, 0, st>>>(L, (double4*)u);
}

void launch_sgs_color(const LevelView& L, bool mixed, const int* rows, int cnt, const void* Dg,
                      const void* b, void* u, hipStream_t st) {
  if (cnt <= 0) return;
  // a colour holds 1/27 of the rows: one row per wave keeps enough waves in
  // flight on the device
  if (mixed) {
    constexpr int R = 1;
    const unsigned g = (unsigned)((cnt + kRowWaves * R - 1) / (kRowWaves * R));
    k_sgs_color<float, R><<<g, 256, 0, st>>>(L, rows, cnt, (const float*)Dg, (const float*)b,
                                             (float4*)u);
  } else {
    constexpr int R = 1;
    const unsigned g = (unsigned)((cnt + kRowWaves * R - 1) / (kRowWaves * R));
    k_sgs_color<double, R><<<g, 256, 0, st>>>(L, rows, cnt, (const double*)Dg,
                                              (const double*)b, (double4*)u);
  }
}

void launch_spmv(const LevelView& L, const double* x, double* y, hipStream_t st) {
  if (L.n > 0) k_spmv<<<ROWGRID(L)>>>(L, x, y);
}

}  // namespace hot
