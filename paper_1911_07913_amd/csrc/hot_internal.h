// Internal declarations shared by the HIP translation units of libhot.
//
// Data layout in HBM (one scene):
//   particles  SoA, sorted by base cell every step: x[3n], v[3n], C[9n], F[9n]
//              (row-major 3x3 per particle), vol[n], mat[n], id[n] (caller
//              order index).
//   grids      every level m has a dense "padded" map over its node grid with
//              a halo of 2 nodes per side (so +-2 stencil offsets never leave
//              the array): map[pidx] = compact node index or -1, and the list
//              nodes[i] = padded index of active node i, in increasing linear
//              order (x fastest).
//   matrices   "diagonal storage": every row keeps 125 3x3 blocks, one per
//              neighbour offset (dx,dy,dz) in [-2,2]^3, slot s = (dx+2) +
//              5(dy+2) + 25(dz+2).  Row i occupies kRowStride consecutive
//              values laid out [i][entry 0..8][slot, padded to 128], so 64
//              lanes that each own one block read every entry with one fully
//              coalesced 512-byte load.  FP64, or BF16 in the mixed-precision
//              V-cycle.
//   vectors    node vectors interleaved [n][3].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>

namespace hot {

constexpr int kSlots = 125;
constexpr int kBlock = 9;
constexpr int kRowVals = kSlots * kBlock;  // 1125 structural values per row
constexpr int kSlotPad = 128;                // slots per entry plane (padded)
constexpr int kRowStride = kBlock * kSlotPad;  // 1152 stored values per row
constexpr int kCenter = 62;                // slot of offset (0,0,0)
constexpr int kColors = 27;                // Gauss-Seidel colours (grid coordinate mod 3)
constexpr int kMaxLevels = 8;
constexpr int kMaxMats = 64;
constexpr int kMaxBcs = 32;

struct MaterialDev {
  int model;   // 0 = fixed-corotated, 1 = Neo-Hookean
  double mu, lam, density, yield, xi;
  double clamp_lo, clamp_hi;  // snow clamp of the singular values (hi = 0: none)
};

struct BcDev {
  int kind;
  double p[16];
};

// Geometry of one level's node grid.
struct GridGeom {
  int dims[3];   // node counts per axis (unpadded)
  int pd[3];     // padded dims = dims + 4
  long long ptotal;
};

// Cell bricks of kBrick^3 cells over the padded cell grid (for the two-pass
// particle-to-node reductions) and row segments of kSegRows nodes along x
// (for the level-0 Hessian assembly).
constexpr int kBrick = 4;
constexpr int kBrickNodes = kBrick + 2;  // node window per axis
constexpr int kBrickWin = kBrickNodes * kBrickNodes * kBrickNodes;  // 216
constexpr int kSegRows = 16;
// Level-0 assembly record of one particle: C_p (45 doubles, packed upper
// triangle), then a_lp = F_p^n^T grad w_lp for its 27 stencil nodes (27 x 3);
// 1008 bytes, a multiple of 16.
constexpr int kAsmRec = 126;
constexpr int kAsmRecA = 45;
struct BrickGeom {
  int bd[3];  // bricks per axis
  long long total;
};
struct Bricks {
  BrickGeom bg;
  int n;             // non-empty bricks
  const int* list;   // [n] dense brick index
  const int* map;    // [total] brick id or -1
};

// Everything the particle/grid kernels of level 0 need (passed by value).
struct SceneDev {
  double dx, inv_dx;
  double origin[3];
  double gravity[3];
  int cells[3];
  GridGeom g0;
  int n_mats, n_bcs;
  const MaterialDev* mats;  // device array [n_mats]
  const BcDev* bcs;         // device array [n_bcs]
};

// View of one level of the hierarchy.
struct LevelView {
  int n;
  GridGeom g;
  const int* nodes;     // [n] padded indices
  const int* map;       // [ptotal]
  double* H;            // [n][1125] FP64 blocks
  uint16_t* Hb;         // [n][1125] BF16 blocks (mixed precision) or null
  double* Dinv;         // [n][9]
  float* Dinv32;        // [n][9] (mixed)
  double* diag;         // [3n] scalar diagonal (coarsest PCG)
  float* diag32;
  uint8_t* free_dof;    // [3n]
  uint32_t* pat;        // [n][4]
};

__host__ __device__ inline long long pidx(const GridGeom& g, int x, int y, int z) {
  return (long long)(x + 2) + (long long)g.pd[0] * ((long long)(y + 2) + (long long)g.pd[1] * (z + 2));
}
__host__ __device__ inline void unpidx(const GridGeom& g, long long p, int& x, int& y, int& z) {
  x = (int)(p % g.pd[0]) - 2;
  long long r = p / g.pd[0];
  y = (int)(r % g.pd[1]) - 2;
  z = (int)(r / g.pd[1]) - 2;
}
__host__ __device__ inline long long slot_offset(const GridGeom& g, int s) {
  int dx = s % 5 - 2, dy = (s / 5) % 5 - 2, dz = s / 25 - 2;
  return (long long)dx + (long long)g.pd[0] * ((long long)dy + (long long)g.pd[1] * dz);
}
inline GridGeom make_geom(int nx, int ny, int nz) {
  GridGeom g;
  g.dims[0] = nx; g.dims[1] = ny; g.dims[2] = nz;
  g.pd[0] = nx + 4; g.pd[1] = ny + 4; g.pd[2] = nz + 4;
  g.ptotal = (long long)g.pd[0] * g.pd[1] * g.pd[2];
  return g;
}

// Work-groups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Remap the hardware block index so every XCD processes one contiguous
// range of logical blocks: neighbouring rows (which share vector entries,
// fine rows or particles) then share an L2.
__device__ inline int xcd_block(int bid, int nblocks) {
  const int q = nblocks / 8, r = nblocks % 8;
  const int x = bid % 8, idx = bid / 8;
  return x * q + (x < r ? x : r) + idx;
}

// ---------------------------------------------------------------- launchers
// grid.hip: binning, stable counting sort, active nodes, coarse levels.
void launch_bin_keys(const SceneDev& s, int n, const double* x, int* keys, int* counts,
                     int* err, hipStream_t st);
void launch_scatter_sorted(int n, const int* keys, const int* start, int* cursor, int* tmp,
                           hipStream_t st);
void launch_sort_segments(long long ncells, const int* start, const int* counts, const int* id,
                          int* tmp, hipStream_t st);
struct Particles {
  double *x, *v, *C, *F, *vol;
  int *mat, *id;
};
void launch_permute_particles(int n, const int* perm, const Particles& src, const Particles& dst,
                              hipStream_t st);
void launch_mark_fine(const GridGeom& g, const int* counts, int* flags, hipStream_t st);
void launch_mark_xy(const GridGeom& fine, int nf, const int* fnodes, const GridGeom& half,
                    int* flags, hipStream_t st);
void launch_mark_coarse(const GridGeom& fine, int nf, const int* fnodes, const GridGeom& coarse,
                        int* cflags, hipStream_t st);
void launch_compact(long long total, const int* flags, const int* scan, int* map, int* nodes,
                    hipStream_t st);
// exclusive scan of n ints; returns nothing, total is scan[n] (out has n+1).
size_t scan_temp_bytes(long long n);
void launch_scan(long long n, const int* in, int* out, void* temp, hipStream_t st);
void launch_fill_int(long long n, int* p, int v, hipStream_t st);
void launch_fine_pattern(const LevelView& L, const int* counts, hipStream_t st);
void launch_pattern_count(const LevelView& L, double* out, hipStream_t st);
void launch_seg_flags(const LevelView& L, int* flags, hipStream_t st);
void launch_seg_compact(int n, const int* flags, const int* scan, int* seg_begin, hipStream_t st);
void launch_mark_bricks(const GridGeom& g, const BrickGeom& bg, const int* counts, int* bflags,
                        hipStream_t st);
void launch_brick_compact(long long total, const int* flags, const int* scan, int* bmap, int* blist,
                          hipStream_t st);

// particles.hip
void launch_particle_frac(const SceneDev& s, int n, const double* x, double* f, int* key,
                          hipStream_t st);
void launch_p2g(const SceneDev& s, const LevelView& L0, const Bricks& B, const double* f,
                const double* v, const double* C, const double* vol, const int* mat,
                const int* cstart, const int* ccount, double* partial, double dt, double t_end,
                double* mass, double* vstar, double* xi, int* fixed, hipStream_t st);
// The particle kernels below first write the node velocities they need
// (v* + dv + alpha p) into `wnode`, a double4 array over the padded level-0
// grid, so each particle gathers 27 nodes with two loads per node and no map
// lookup.
// each particle's level-0 assembly record: its projected stress derivative
// at F(dv) (dv = NULL: dv = 0) and its a_l = F^n^T grad w_l operands
void launch_particle_hessian(const SceneDev& s, const LevelView& L0, int n, const double* f,
                             const int* key, const double* F, const double* vol, const int* mat,
                             const double* vstar, const double* dv, double dt, double* wnode,
                             double* rec, hipStream_t st);
// energy/stress at dv + alpha*p: psi_out[n] = V_p psi, S_out[9n] = V_p P F^n^T
void launch_particle_eval(const SceneDev& s, const LevelView& L0, int n, const double* f,
                          const int* key, const double* F, const double* vol, const int* mat,
                          const double* vstar, const double* dv, const double* p, double alpha,
                          double dt, double* wnode, double* psi_out, double* S_out,
                          hipStream_t st);
void launch_gradient(const SceneDev& s, const LevelView& L0, const Bricks& B, const double* f,
                     const double* S, const int* cstart, const int* ccount, double* partial,
                     const double* mass, const int* fixed, const double* dv, double dt, double* g,
                     hipStream_t st);
void launch_g2p(const SceneDev& s, const LevelView& L0, int n, const double* f, const int* key,
                double* x, double* v, double* C, double* F, const int* mat, const double* vstar,
                const double* dv, double dt, double* wnode, hipStream_t st);
// level-0 Hessian: the row segments' blocks from the particles' assembly
// records (C_p and the a_l operands, written by launch_particle_hessian)
void launch_assemble_h0(const SceneDev& s, const LevelView& L0, const int* seg_begin, int n_seg,
                        int n, const double* rec, const int* cstart, const int* ccount,
                        const double* mass, const int* fixed, hipStream_t st);

// matrix.hip
void launch_finalize_level(const LevelView& L, int zero_diag_rule, hipStream_t st);
// Galerkin product F -> Cv through the half-coarsened grid T (x, y coarse, z
// fine; T.g has dims (F.x/2 + 1, F.y/2 + 1, F.z), T.nodes/map/pat/H sized for
// T.n rows); writes Cv's blocks, pattern, free flags, diagonal and l1 inverse.
void launch_rap(const LevelView& F, const LevelView& T, const LevelView& Cv, hipStream_t st);
void launch_to_bf16(const LevelView& L, hipStream_t st);
// V-cycle pieces (FP64 and FP32/BF16 variants chosen by `mixed`)
void launch_jacobi_first(const LevelView& L, bool mixed, const void* b, void* u, hipStream_t st);
void launch_residual(const LevelView& L, bool mixed, const void* b, const void* u, void* r,
                     hipStream_t st);
// Row count from which the smoothing and residual sweeps run over x-runs
// instead of one row per wave (process-wide; < 0 restores the default).
// Returns the old value.
int set_sweep_run_min(int rows);
// The V-cycle iterate u of every level (and the smoother's output) is stored
// on the level's padded dense grid as 4-vectors (double4 or float4); b and r
// are compact [n][3].
void launch_smooth(const LevelView& L, bool mixed, const void* b, const void* u, void* u_out,
                   hipStream_t st);
// compact FP64 copy of a level's dense iterate
void launch_dense_out(const LevelView& L, bool mixed, const void* u, double* out, hipStream_t st);
// bc = P~^T r; with uc given, also the coarse level's first smoothing from
// zero, uc = D~^{-1} bc on its dense grid (what launch_jacobi_first writes)
void launch_restrict(const LevelView& F, const LevelView& Cv, bool mixed, const void* r,
                     void* bc, void* uc, hipStream_t st);
void launch_prolong_add(const LevelView& F, const LevelView& Cv, bool mixed, const void* uc,
                        void* u, hipStream_t st);
// Per-solve log of coarsest-level iteration counts, indexed on the device:
// a solve writes its count (-1 if a grid barrier of the multi-work-group form
// timed out) to base[min(*cursor, cap)] and advances *cursor, so that a
// captured V-cycle logs each replay in its own entry.
struct IterLog {
  int* base;
  int cap;
  int* cursor;
};
__device__ inline void log_iters(const IterLog& lg, int v) {
  const int c = *lg.cursor;
  lg.base[c < lg.cap ? c : lg.cap] = v;
  *lg.cursor = c + 1;
}
// Coarsest solve (relative tolerance rel in the D^-1 norm, at most max_iter
// iterations), logging its iteration count through lg.
// grid_ok: the caller holds a grid-solve ticket, so the multi-work-group form
// may be used where it pays; without one the single-work-group form runs,
// which needs coarse_pcg_single_fits (hipErrorInvalidConfiguration otherwise).
hipError_t launch_coarse_pcg(const LevelView& L, bool mixed, const void* b, void* x, void* work,
                             IterLog lg, int max_iter, double rel, bool grid_ok, hipStream_t st);
// Whether the coarsest solve of this level would use the multi-work-group
// form, and whether the single-work-group form can hold it.
bool coarse_pcg_uses_grid(const LevelView& L, bool mixed);
bool coarse_pcg_single_fits(const LevelView& L, bool mixed);
// Resolve the coarsest solve's launch shapes for the current device (they
// are cached; a stream capture must not be the first to ask).
void coarse_pcg_warm();
size_t coarse_pcg_work_bytes(int n);
// coloured symmetric Gauss-Seidel: rows of each colour (coff[0..27], device),
// diagonal-block inverses, and one colour's in-place pass
size_t color_scratch_bytes(int n);
void launch_color_rows(const LevelView& L, int* scratch, int* coff, int* rows, hipStream_t st);
void launch_block_diag_inv(const LevelView& L, double* Dg, float* Dg32, hipStream_t st);
void launch_zero_rows(const LevelView& L, bool mixed, void* u, hipStream_t st);
void launch_sgs_color(const LevelView& L, bool mixed, const int* rows, int cnt, const void* Dg,
                      const void* b, void* u, hipStream_t st);
void launch_spmv(const LevelView& L, const double* x, double* y, hipStream_t st);

// blas.hip: deterministic reductions and vector updates on FP64 node vectors.
constexpr int kRedBlocks = 2048;  // most partials a reduction writes
void launch_dot(long long n, const double* a, const double* b, double* partial, double* out,
                hipStream_t st);
void launch_sum(long long n, const double* a, double* partial, double* out, hipStream_t st);
void launch_kinetic_delta(int n, const double* mass, const double* dv, const double* p,
                          double alpha, double* partial, double* out, hipStream_t st);
void launch_cn_sq(int n, const double* g, const double* xi, double scale, double* partial,
                  double* out, hipStream_t st);
void launch_max_speed(int n, const double* v, double* partial, double* out, hipStream_t st);
// y = a * x
void launch_scale_copy(long long n, double a, const double* x, double* y, hipStream_t st);
// Two-loop recursion (Alg. L-BFGS two-loop).  Start: v <- -init (init may be
// NULL: v kept), partials of dnext . v.  Inner step: finish the previous inner
// product d from prev (red_blocks(n) partials); first loop (alpha_in NULL):
// alpha_out = rho d, v -= alpha x; second loop: v += (alpha_in - rho d) x;
// then partials of dnext . v into partial (dnext may be NULL; partial must not
// alias prev).
void launch_twoloop_start(long long n, const double* init, double* v, const double* dnext,
                          double* partial, hipStream_t st);
void launch_twoloop_step(long long n, const double* prev, const double* rho, const double* alpha_in,
                         double* alpha_out, const double* x, double* v, const double* dnext,
                         double* partial, hipStream_t st);
// out = fixed-order sum of the red_blocks(n) partials
void launch_finish_partials(long long n, const double* partial, double* out, hipStream_t st);
// dvt = dv + alpha p, sv = dvt - dv
void launch_step_update(long long n, const double* dv, double alpha, const double* p, double* dvt,
                        double* sv, hipStream_t st);
// y = gnew - g; out = {y.s, y.y, s.s, sum_i |gnew_i / (scale xi_i)|^2} (n0 nodes);
// partial holds 4 red_blocks(n) values
void launch_secant_cn(long long n, const double* gnew, const double* g, double* y, const double* sv,
                      int n0, const double* xi, double scale, double* partial, double* out,
                      hipStream_t st);
// out = {sum_p (psi_t - psi_c) over n particles, kinetic change over n0 nodes}
// (the sum of differences and the launch_kinetic_delta sum, bit for bit)
void launch_energy_delta(long long n, const double* psi_t, const double* psi_c, int n0,
                         const double* mass, const double* dv, const double* p, double alpha,
                         double* partial, double* out, hipStream_t st);
void launch_to_f32(long long n, const double* x, float* y, hipStream_t st);
void launch_block_jacobi_apply(int n, const double* Dinv, const double* x, double* y, double sign,
                               hipStream_t st);
void launch_fill_double(long long n, double* p, double v, hipStream_t st);
// y += a x;  y = x + b y;  z = r / d (elementwise)
void launch_axpy(long long n, double a, const double* x, double* y, hipStream_t st);
void launch_xpby(long long n, const double* x, double b, double* y, hipStream_t st);
void launch_diag_solve(long long n, const double* d, const double* r, double* z, hipStream_t st);
void launch_rho(const double* ys, double* rho, hipStream_t st);

}  // namespace hot
