// Binning, stable counting sort and active-node bookkeeping (integer work).
//
// The step starts by binning particles by their base node (the lowest node of
// the 3x3x3 quadratic B-spline stencil, Sec. 6) and finding the active grid by
// traversing particles (Sec. 3.1: the sparsity pattern changes every step).
// Coarse levels hold the parents of active fine nodes under the linear node
// embedding of Sec. 4.2 (coarse node J sits at fine node 2J).  Everything here
// is integer arithmetic and bit-exact.
#include "hot_internal.h"

namespace hot {
namespace {

constexpr int kTpb = 256;

inline unsigned blocks_for(long long n, int tpb = kTpb) {
  return (unsigned)((n + tpb - 1) / tpb);
}

__global__ void k_bin_keys(SceneDev s, int n, const double* __restrict__ x, int* __restrict__ keys,
                           int* __restrict__ counts, int* __restrict__ err) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int b[3];
  bool ok = true;
  for (int a = 0; a < 3; ++a) {
    // (x - o)/dx with IEEE division, then floor(t - 1/2): same operations as
    // the CPU reference so the integer key is bit-identical.
    double t = (x[3 * p + a] - s.origin[a]) / s.dx;
    ok = ok && (t >= 2.0) && (t <= (double)(s.cells[a] - 3));
    double fb = floor(t - 0.5);
    int bi = ok ? (int)fb : 1;
    b[a] = bi;
  }
  if (!ok) {
    atomicOr(err, 1);
    b[0] = b[1] = b[2] = 1;
  }
  int key = (int)pidx(s.g0, b[0], b[1], b[2]);
  keys[p] = key;
  atomicAdd(&counts[key], 1);
}

__global__ void k_scatter(int n, const int* __restrict__ keys, const int* __restrict__ start,
                          int* __restrict__ cursor, int* __restrict__ tmp) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int k = keys[p];
  int pos = start[k] + atomicAdd(&cursor[k], 1);
  tmp[pos] = p;
}

// Order each cell's segment by the caller-order particle index: the result is
// the stable sort by key of the caller-ordered particles.
__global__ void k_sort_segments(long long ncells, const int* __restrict__ start,
                                const int* __restrict__ counts, const int* __restrict__ id,
                                int* __restrict__ tmp) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  int cnt = counts[c];
  if (cnt < 2) return;
  int* seg = tmp + start[c];
  for (int i = 1; i < cnt; ++i) {
    int v = seg[i];
    int key = id[v];
    int j = i - 1;
    while (j >= 0 && id[seg[j]] > key) {
      seg[j + 1] = seg[j];
      --j;
    }
    seg[j + 1] = v;
  }
}

// dst[i] = src[perm[i]] for all particle fields.  One wave moves 64
// consecutive destination particles field by field, lane l copying entries
// l, l + 64, ... of the wave's contiguous destination range, so that stores
// are contiguous and loads walk each source particle's entries in order.
template <typename T, int W>
__device__ inline void permute_field(int i0, int cnt, int lane, const int* __restrict__ perm,
                                     const T* __restrict__ src, T* __restrict__ dst) {
  for (int e = lane; e < W * cnt; e += 64) {
    const int q = e / W, c = e - W * q;
    dst[(long long)W * (i0 + q) + c] = src[(long long)W * perm[i0 + q] + c];
  }
}

__global__ void k_permute(int n, const int* __restrict__ perm, Particles src, Particles dst) {
  const int lane = threadIdx.x & 63;
  const int i0 = (blockIdx.x * blockDim.x + threadIdx.x - lane);
  if (i0 >= n) return;
  const int cnt = min(64, n - i0);
  permute_field<double, 3>(i0, cnt, lane, perm, src.x, dst.x);
  permute_field<double, 3>(i0, cnt, lane, perm, src.v, dst.v);
  permute_field<double, 9>(i0, cnt, lane, perm, src.C, dst.C);
  permute_field<double, 9>(i0, cnt, lane, perm, src.F, dst.F);
  permute_field<double, 1>(i0, cnt, lane, perm, src.vol, dst.vol);
  permute_field<int, 1>(i0, cnt, lane, perm, src.mat, dst.mat);
  permute_field<int, 1>(i0, cnt, lane, perm, src.id, dst.id);
}

// Active fine nodes: the 27 nodes of every non-empty base cell.
__global__ void k_mark_fine(GridGeom g, const int* __restrict__ counts, int* __restrict__ flags) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ptotal) return;
  if (counts[c] == 0) return;
  int bx, by, bz;
  unpidx(g, c, bx, by, bz);
  for (int k = 0; k < 27; ++k) flags[pidx(g, bx + k % 3, by + (k / 3) % 3, bz + k / 9)] = 1;
}

// Parents of a fine coordinate under the linear embedding: even -> c/2,
// odd -> (c-1)/2 and (c+1)/2.
__device__ inline int parents1d(int c, int* J) {
  if ((c & 1) == 0) {
    J[0] = c >> 1;
    return 1;
  }
  J[0] = (c - 1) >> 1;
  J[1] = (c + 1) >> 1;
  return 2;
}

__global__ void k_mark_coarse(GridGeom fg, int nf, const int* __restrict__ fnodes, GridGeom cg,
                              int* __restrict__ cflags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  int x, y, z;
  unpidx(fg, fnodes[i], x, y, z);
  int Jx[2], Jy[2], Jz[2];
  int nx = parents1d(x, Jx), ny = parents1d(y, Jy), nz = parents1d(z, Jz);
  for (int a = 0; a < nx; ++a)
    for (int b = 0; b < ny; ++b)
      for (int c = 0; c < nz; ++c) cflags[pidx(cg, Jx[a], Jy[b], Jz[c])] = 1;
}

// Points (X, Y, z) of the half-coarsened grid (x and y coarsened, z fine)
// that are x-y parents of an active fine node.
__global__ void k_mark_xy(GridGeom fg, int nf, const int* __restrict__ fnodes, GridGeom tg,
                          int* __restrict__ tflags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  int x, y, z;
  unpidx(fg, fnodes[i], x, y, z);
  int Jx[2], Jy[2];
  int nx = parents1d(x, Jx), ny = parents1d(y, Jy);
  for (int a = 0; a < nx; ++a)
    for (int b = 0; b < ny; ++b) tflags[pidx(tg, Jx[a], Jy[b], z)] = 1;
}

__global__ void k_compact(long long total, const int* __restrict__ flags,
                          const int* __restrict__ scan, int* __restrict__ map,
                          int* __restrict__ nodes) {
  long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  if (flags[p]) {
    int idx = scan[p];
    map[p] = idx;
    nodes[idx] = (int)p;
  } else {
    map[p] = -1;
  }
}

__global__ void k_fill(long long n, int* p, int v) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Level-0 symbolic pattern: block (i, j) is present iff some particle's
// stencil holds both nodes, i.e. some non-empty base cell b satisfies
// b in [max(i,j) - 2, min(i,j)] on every axis.  Only the 27 base cells
// i + r, r in [-2, 0]^3, can serve row i; slot d (offset j - i) is served by
// the cells with r in [max(-2, d - 2), min(0, d)] per axis.  One thread per
// row loads the row's 27 cell occupancies once and forms each slot's bit
// against that slot's cell mask.
struct SlotCellMasks {
  uint32_t m[kSlots];  // bit r = rx + 3 ry + 9 rz: cell i + (rx - 2, ry - 2, rz - 2) serves the slot
};
constexpr SlotCellMasks make_slot_cell_masks() {
  SlotCellMasks t{};
  for (int s = 0; s < kSlots; ++s) {
    const int d[3] = {s % 5 - 2, (s / 5) % 5 - 2, s / 25 - 2};
    uint32_t m = 0;
    for (int r = 0; r < 27; ++r) {
      const int rr[3] = {r % 3 - 2, (r / 3) % 3 - 2, r / 9 - 2};
      bool ok = true;
      for (int a = 0; a < 3; ++a) {
        const int lo = d[a] - 2 > -2 ? d[a] - 2 : -2;
        const int hi = d[a] < 0 ? d[a] : 0;
        if (rr[a] < lo || rr[a] > hi) ok = false;
      }
      if (ok) m |= 1u << r;
    }
    t.m[s] = m;
  }
  return t;
}
__constant__ SlotCellMasks kSlotCellMasks = make_slot_cell_masks();

__global__ void k_fine_pattern(LevelView L, const int* __restrict__ counts) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= L.n) return;
  int x, y, z;
  unpidx(L.g, L.nodes[row], x, y, z);
  uint32_t occ = 0;
#pragma unroll
  for (int r = 0; r < 27; ++r) {
    const int bx = x + r % 3 - 2, by = y + (r / 3) % 3 - 2, bz = z + r / 9 - 2;
    if (bx < -2 || by < -2 || bz < -2 || bx >= L.g.dims[0] + 2 || by >= L.g.dims[1] + 2 ||
        bz >= L.g.dims[2] + 2)
      continue;
    if (counts[pidx(L.g, bx, by, bz)] > 0) occ |= 1u << r;
  }
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    uint32_t bits = 0;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const int s = w * 32 + k;
      if (s < kSlots && (occ & kSlotCellMasks.m[s])) bits |= 1u << k;
    }
    L.pat[4 * (long long)row + w] = bits;
  }
}

// Number of structurally present blocks of a level (popcount of its pattern),
// written as a double.  One work-group of 1024 threads.
// Structural block count of a level: popcount of its pattern words, summed
// per block and added into an integer total (integer sums are exact in any
// order), then stored as a double.
constexpr int kPatWordsPerBlock = 256 * 16;

__global__ void k_pattern_count(LevelView L, unsigned long long* total) {
  __shared__ unsigned long long sh[4];
  unsigned long long c = 0;
  const long long nw = (long long)L.n * 4;
  const long long w0 = (long long)blockIdx.x * kPatWordsPerBlock;
  const long long w1 = w0 + kPatWordsPerBlock < nw ? w0 + kPatWordsPerBlock : nw;
  for (long long k = w0 + threadIdx.x; k < w1; k += 256) c += __popc(L.pat[k]);
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(total, sh[0] + sh[1] + sh[2] + sh[3]);
}

__global__ void k_u64_slot(unsigned long long* p, int to_double) {
  if (threadIdx.x == 0) {
    if (to_double) {
      const unsigned long long t = *p;
      *reinterpret_cast<double*>(p) = (double)t;
    } else {
      *p = 0ull;
    }
  }
}

// ---- work lists for the row-strip and cell-brick kernels
// Segment = up to kSegRows consecutive active nodes of one x-line (same y, z)
// whose x lies in one aligned window of kSegRows; nodes are sorted by linear
// index, so a segment is a contiguous range of the node list.
__global__ void k_seg_flags(LevelView L, int* __restrict__ flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  int f = 1;
  if (i > 0) {
    int x0, y0, z0, x1, y1, z1;
    unpidx(L.g, L.nodes[i - 1], x0, y0, z0);
    unpidx(L.g, L.nodes[i], x1, y1, z1);
    f = (y0 != y1 || z0 != z1 || ((x0 + 2) / kSegRows) != ((x1 + 2) / kSegRows)) ? 1 : 0;
  }
  flags[i] = f;
}
__global__ void k_seg_compact(int n, const int* __restrict__ flags, const int* __restrict__ scan,
                              int* __restrict__ seg_begin) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  if (i == n) {
    seg_begin[scan[n]] = n;
    return;
  }
  if (flags[i]) seg_begin[scan[i]] = i;
}

// Cell bricks: kBrick^3 cells (in padded cell coordinates) holding particles.
__global__ void k_mark_bricks(GridGeom g, BrickGeom bg, const int* __restrict__ counts,
                              int* __restrict__ bflags) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ptotal) return;
  if (counts[c] == 0) return;
  int x = (int)(c % g.pd[0]);
  long long r = c / g.pd[0];
  int y = (int)(r % g.pd[1]);
  int z = (int)(r / g.pd[1]);
  bflags[(x / kBrick) + (long long)bg.bd[0] * ((y / kBrick) + (long long)bg.bd[1] * (z / kBrick))] = 1;
}
__global__ void k_brick_compact(long long total, const int* __restrict__ flags,
                                const int* __restrict__ scan, int* __restrict__ bmap,
                                int* __restrict__ blist) {
  long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= total) return;
  if (flags[b]) {
    int id = scan[b];
    bmap[b] = id;
    blist[id] = (int)b;
  } else {
    bmap[b] = -1;
  }
}

// ---- exclusive scan (three passes over tiles of 2048 ints)
constexpr int kScanItems = 8;
constexpr int kScanTile = kTpb * kScanItems;

__device__ inline int block_exclusive_scan(int v, int* sh, int& total) {
  // Hillis-Steele inclusive scan in LDS, then shift.
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kTpb; off <<= 1) {
    int a = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  int incl = sh[t];
  total = sh[kTpb - 1];
  __syncthreads();
  return incl - v;
}

__global__ void k_scan_reduce(long long n, const int* __restrict__ in, int* __restrict__ sums) {
  __shared__ int sh[kTpb];
  long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  int s = 0;
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) s += in[base + k];
  int total;
  block_exclusive_scan(s, sh, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void k_scan_sums(int nt, int* __restrict__ sums, int* __restrict__ total_out) {
  __shared__ int sh[kTpb];
  int carry = 0;
  for (int base = 0; base < nt; base += kTpb) {
    int i = base + threadIdx.x;
    int v = (i < nt) ? sums[i] : 0;
    int total;
    int ex = block_exclusive_scan(v, sh, total);
    if (i < nt) sums[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) *total_out = carry;
}

__global__ void k_scan_down(long long n, const int* __restrict__ in, const int* __restrict__ sums,
                            int* __restrict__ out) {
  __shared__ int sh[kTpb];
  long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    s += v[k];
  }
  int total;
  int ex = block_exclusive_scan(s, sh, total) + sums[blockIdx.x];
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
}

}  // namespace

void launch_bin_keys(const SceneDev& s, int n, const double* x, int* keys, int* counts, int* err,
                     hipStream_t st) {
  if (n > 0) k_bin_keys<<<blocks_for(n), kTpb, 0, st>>>(s, n, x, keys, counts, err);
}
void launch_scatter_sorted(int n, const int* keys, const int* start, int* cursor, int* tmp,
                           hipStream_t st) {
  if (n > 0) k_scatter<<<blocks_for(n), kTpb, 0, st>>>(n, keys, start, cursor, tmp);
}
void launch_sort_segments(long long ncells, const int* start, const int* counts, const int* id,
                          int* tmp, hipStream_t st) {
  k_sort_segments<<<blocks_for(ncells), kTpb, 0, st>>>(ncells, start, counts, id, tmp);
}
void launch_permute_particles(int n, const int* perm, const Particles& src, const Particles& dst,
                              hipStream_t st) {
  if (n > 0) k_permute<<<blocks_for(n), kTpb, 0, st>>>(n, perm, src, dst);
}
void launch_mark_fine(const GridGeom& g, const int* counts, int* flags, hipStream_t st) {
  k_mark_fine<<<blocks_for(g.ptotal), kTpb, 0, st>>>(g, counts, flags);
}
void launch_mark_coarse(const GridGeom& fine, int nf, const int* fnodes, const GridGeom& coarse,
                        int* cflags, hipStream_t st) {
  if (nf > 0) k_mark_coarse<<<blocks_for(nf), kTpb, 0, st>>>(fine, nf, fnodes, coarse, cflags);
}
void launch_mark_xy(const GridGeom& fine, int nf, const int* fnodes, const GridGeom& half,
                    int* flags, hipStream_t st) {
  if (nf > 0) k_mark_xy<<<blocks_for(nf), kTpb, 0, st>>>(fine, nf, fnodes, half, flags);
}
void launch_compact(long long total, const int* flags, const int* scan, int* map, int* nodes,
                    hipStream_t st) {
  k_compact<<<blocks_for(total), kTpb, 0, st>>>(total, flags, scan, map, nodes);
}
void launch_fill_int(long long n, int* p, int v, hipStream_t st) {
  if (n > 0) k_fill<<<blocks_for(n), kTpb, 0, st>>>(n, p, v);
}
void launch_fine_pattern(const LevelView& L, const int* counts, hipStream_t st) {
  if (L.n > 0) k_fine_pattern<<<blocks_for(L.n), kTpb, 0, st>>>(L, counts);
}

void launch_seg_flags(const LevelView& L, int* flags, hipStream_t st) {
  if (L.n > 0) k_seg_flags<<<blocks_for(L.n), kTpb, 0, st>>>(L, flags);
}
void launch_seg_compact(int n, const int* flags, const int* scan, int* seg_begin, hipStream_t st) {
  k_seg_compact<<<blocks_for((long long)n + 1), kTpb, 0, st>>>(n, flags, scan, seg_begin);
}
void launch_mark_bricks(const GridGeom& g, const BrickGeom& bg, const int* counts, int* bflags,
                        hipStream_t st) {
  k_mark_bricks<<<blocks_for(g.ptotal), kTpb, 0, st>>>(g, bg, counts, bflags);
}
void launch_brick_compact(long long total, const int* flags, const int* scan, int* bmap, int* blist,
                          hipStream_t st) {
  k_brick_compact<<<blocks_for(total), kTpb, 0, st>>>(total, flags, scan, bmap, blist);
}

void launch_pattern_count(const LevelView& L, double* out, hipStream_t st) {
  // the result slot holds the integer total until it is converted
  unsigned long long* t = reinterpret_cast<unsigned long long*>(out);
  const long long nw = (long long)L.n * 4;
  k_u64_slot<<<1, 64, 0, st>>>(t, 0);
  if (nw > 0)
    k_pattern_count<<<(unsigned)((nw + kPatWordsPerBlock - 1) / kPatWordsPerBlock), 256, 0, st>>>(L, t);
  k_u64_slot<<<1, 64, 0, st>>>(t, 1);
}

size_t scan_temp_bytes(long long n) {
  long long nt = (n + kScanTile - 1) / kScanTile;
  return (size_t)(nt + 1) * sizeof(int);
}

void launch_scan(long long n, const int* in, int* out, void* temp, hipStream_t st) {
  int nt = (int)((n + kScanTile - 1) / kScanTile);
  int* sums = (int*)temp;
  if (nt == 0) {
    k_fill<<<1, 1, 0, st>>>(1, out, 0);
    return;
  }
  k_scan_reduce<<<nt, kTpb, 0, st>>>(n, in, sums);
  k_scan_sums<<<1, kTpb, 0, st>>>(nt, sums, out + n);
  k_scan_down<<<nt, kTpb, 0, st>>>(n, in, sums, out);
}

}  // namespace hot
