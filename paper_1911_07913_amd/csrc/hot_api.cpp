// Host side of libhot: scene state, the implicit MPM step pipeline and the
// HOT quasi-Newton loop (Alg. HOT) sequencing the HIP kernels, plus the C ABI
// declared in include/hot.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <unordered_map>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hot.h"
#include "hot_internal.h"
#include "tickets.h"

using namespace hot;

namespace {

thread_local std::string g_err;

hot_status fail(hot_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(HOT_E_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),  \
                  __FILE__, __LINE__);                                                  \
  } while (0)

#define TRY(expr)                      \
  do {                                 \
    hot_status s_ = (expr);            \
    if (s_ < 0) return s_;             \
  } while (0)

void* default_alloc(size_t bytes, void*) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}
void default_free(void* p, void*) {
  if (p) (void)hipFree(p);
}

struct DBuf {
  void* p = nullptr;
  size_t cap = 0;
  bool borrowed = false;  // a range of the no-allocation scratch array: never freed or grown
};

enum {
  S_GP = 0,
  S_DEP = 1,
  S_DEK = 2,
  S_YS = 3,
  S_YY = 4,
  S_SS = 5,
  S_CN = 6,
  S_E0 = 7,
  S_VMAX = 8,
  S_NNZ = 9,  // structural block count of levels 0..kMaxLevels-1 (slots 9..16)
  NSCAL = 24
};

struct LevelH {
  GridGeom g;
  int n = 0;
  DBuf nodes, map, H, Hb, Dinv, Dinv32, diag, diag32, freed, pat;
  DBuf b, u, r, t;  // V-cycle vectors
  // coloured Gauss-Seidel: rows by colour, colour offsets, diagonal-block inverses
  DBuf crow, coffd, Dg, Dg32;
  int coff[kColors + 1] = {0};
};

}  // namespace

struct hot_scene {
  hot_params prm;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hot_allocator alloc;
  SceneDev sd;
  int n = 0;
  double t = 0.0;
  std::vector<hot_material> mats;
  std::vector<hot_bc> bcs;
  double bc_speed = 0.0;
  size_t bytes_live = 0;
  size_t est_bytes = 0;  // footprint estimate at init (admission)
  int device = 0;
  std::vector<DBuf*> owned;
  bool mixed = false;
  int levels = 1;

  Particles P[2];
  int cur = 0;
  DBuf pbuf[2];
  DBuf f, key, keys, tmp, arec, psi[2], S[2];
  DBuf wnode;  // double4 node velocities over the padded level-0 grid
  // half-coarsened grid of the Galerkin product (reused for every level)
  DBuf tnodes, tmap, tpat, tH;
  int pc = 0;  // current psi/S buffer
  // level-0 grid
  DBuf counts, start, cursor, flags, scan, scan_temp, err;
  LevelH L[kMaxLevels];
  // level-0 node data
  DBuf mass, vstar, xi, fixed;
  // solver vectors
  DBuf dv, dvt, g, gnew, q, r, pcg_work, pcg_iters, vin, vout;
  DBuf cscratch;  // colour counting of the Gauss-Seidel set-up
  std::vector<DBuf> Sh, Yh;
  DBuf dalpha, drho, dscal, partial, tables;
  // work lists: row segments (assembly) and cell bricks (particle-to-node sums)
  DBuf seg_begin, bmap, blist, bpartial;
  int n_seg = 0;
  Bricks bricks;
  double* hscal = nullptr;
  int* herr = nullptr;
  int node_cap = 0;
  bool no_alloc = false;  // inside hot_step_noalloc: a buffer that must grow is an error
  bool grid_ok = false;   // holds a grid-solve ticket for the current solve
  hipGraphExec_t vc_exec = nullptr;  // captured V-cycle (hot_params.graph)
  bool vc_stale = true;              // vc_exec holds an earlier step's cycle
  double cg_per_cycle = 1.0;  // last solve's coarsest-PCG iterations per V-cycle
  // last-step logs
  std::vector<int> log_int;
  std::vector<double> log_cn;
  int vcycles = 0;
  hipEvent_t ev[5];
  bool prepared = false;
  double dt_prepared = 0.0;
  // kernel tracing
  bool prof = false;
  double prof_ms[HOT_PROF_COUNT] = {0};
  int64_t prof_n[HOT_PROF_COUNT] = {0};
  double prof_bytes[HOT_PROF_COUNT] = {0};
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_kind;
  size_t prof_used = 0;
};

namespace {

hot_status ensure(hot_scene* s, DBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (b.cap >= bytes) return HOT_OK;
  if (b.borrowed)
    return fail(HOT_E_INVALID,
                "the step needs %zu bytes of per-call scratch here, more than the %zu the "
                "no-allocation entry point holds",
                bytes, b.cap);
  if (s->no_alloc)
    return fail(HOT_E_NOMEM,
                "hot_step_noalloc: a %zu-byte scene buffer would have to grow to %zu bytes "
                "(hot_step sizes it)",
                b.cap, bytes);
  if (b.p) {
    // keep the stream ordered: free only after pending work completes
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(HOT_E_DEVICE, "sync failed");
    s->alloc.free(b.p, s->alloc.ctx);
    s->bytes_live -= b.cap;
    b.p = nullptr;
    b.cap = 0;
  }
  size_t want = bytes + bytes / 4;
  b.p = s->alloc.alloc(want, s->alloc.ctx);
  if (!b.p) return fail(HOT_E_NOMEM, "device allocation of %zu bytes failed", want);
  if (reinterpret_cast<uintptr_t>(b.p) % 256 != 0) {
    // the kernels read and write 16- and 32-byte vectors and records
    void* bad = b.p;
    s->alloc.free(bad, s->alloc.ctx);
    b.p = nullptr;
    return fail(HOT_E_INVALID, "the allocator returned %p, which is not 256-byte aligned", bad);
  }
  b.cap = want;
  s->bytes_live += want;
  return HOT_OK;
}

template <typename T>
T* P(const DBuf& b) {
  return (T*)b.p;
}

void release(hot_scene* s, DBuf& b) {
  if (b.p && !b.borrowed) s->alloc.free(b.p, s->alloc.ctx);
  b.p = nullptr;
  b.cap = 0;
}

hot_status readback(hot_scene* s) {
  HIPCHK(hipMemcpyAsync(s->hscal, s->dscal.p, NSCAL * sizeof(double), hipMemcpyDeviceToHost,
                        s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  return HOT_OK;
}

hot_status read_int(hot_scene* s, const int* dptr, int* out) {
  HIPCHK(hipMemcpyAsync(s->herr, dptr, sizeof(int), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  *out = *s->herr;
  return HOT_OK;
}

// ---- kernel tracing: event pairs around selected launches
hot_status prof_begin(hot_scene* s, int kind, size_t* slot) {
  *slot = (size_t)-1;
  if (!s->prof) return HOT_OK;
  if (s->prof_used + 2 > s->prof_ev.size()) {
    for (int k = 0; k < 64; ++k) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      s->prof_ev.push_back(e);
    }
    s->prof_kind.resize(s->prof_ev.size() / 2 + 1, 0);
  }
  *slot = s->prof_used;
  s->prof_kind[s->prof_used / 2] = kind;
  s->prof_used += 2;
  HIPCHK(hipEventRecord(s->prof_ev[*slot], s->stream));
  return HOT_OK;
}
hot_status prof_end(hot_scene* s, size_t slot) {
  if (slot == (size_t)-1) return HOT_OK;
  HIPCHK(hipEventRecord(s->prof_ev[slot + 1], s->stream));
  return HOT_OK;
}
#define PROF(s, kind, call)                    \
  do {                                         \
    size_t ps_;                                \
    TRY(prof_begin((s), (kind), &ps_));        \
    call;                                      \
    TRY(prof_end((s), ps_));                   \
  } while (0)

LevelView view(hot_scene* s, int m) {
  LevelH& L = s->L[m];
  LevelView v;
  v.n = L.n;
  v.g = L.g;
  v.nodes = P<int>(L.nodes);
  v.map = P<int>(L.map);
  v.H = P<double>(L.H);
  v.Hb = P<uint16_t>(L.Hb);
  v.Dinv = P<double>(L.Dinv);
  v.Dinv32 = P<float>(L.Dinv32);
  v.diag = P<double>(L.diag);
  v.diag32 = P<float>(L.diag32);
  v.free_dof = P<uint8_t>(L.freed);
  v.pat = P<uint32_t>(L.pat);
  return v;
}

// Coarse-PCG iteration log of a step: one entry per V-cycle (at most three per
// quasi-Newton iteration, plus headroom), the last entry clamping overflow,
// then the device-side cursor.
int pcg_log_cap(const hot_scene* s) { return s->prm.max_iters * 3 + 15; }
size_t pcg_log_bytes(int max_iters) { return ((size_t)max_iters * 3 + 17) * 4; }
IterLog pcg_log(hot_scene* s) {
  const int cap = pcg_log_cap(s);
  return IterLog{P<int>(s->pcg_iters), cap, P<int>(s->pcg_iters) + cap + 1};
}

void drop_vcycle_graph(hot_scene* s) {
  if (s->vc_exec) (void)hipGraphExecDestroy(s->vc_exec);
  s->vc_exec = nullptr;
  s->vc_stale = true;
}

double lame_mu(double E, double nu) { return E / (2.0 * (1.0 + nu)); }
double lame_lam(double E, double nu) { return E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)); }

double bc_max_speed(const std::vector<hot_bc>& bcs) {
  double s = 0.0;
  for (const hot_bc& b : bcs) {
    const double* p = b.p;
    if (b.kind == HOT_BC_GRIP) {
      double a[3] = {p[9], p[10], p[11]};
      double na = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
      for (int k = 0; k < 3; ++k) a[k] /= na;
      double rmax = 0.0;
      for (int bx = 0; bx < 2; ++bx)
        for (int by = 0; by < 2; ++by)
          for (int bz = 0; bz < 2; ++bz) {
            double d[3] = {p[3 * bx] - p[6], p[3 * by + 1] - p[7], p[3 * bz + 2] - p[8]};
            double c[3] = {a[1] * d[2] - a[2] * d[1], a[2] * d[0] - a[0] * d[2],
                           a[0] * d[1] - a[1] * d[0]};
            rmax = std::max(rmax, std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]));
          }
      s = std::max(s, std::fabs(p[12]) * rmax);
    } else if (b.kind == HOT_BC_SPHERE) {
      s = std::max(s, std::sqrt(p[4] * p[4] + p[5] * p[5] + p[6] * p[6]));
    }
  }
  return s;
}

hot_status validate_params(const hot_params* p) {
  if (!p) return fail(HOT_E_INVALID, "params is NULL");
  if (!(p->dx > 0.0) || !std::isfinite(p->dx)) return fail(HOT_E_INVALID, "dx must be > 0");
  for (int a = 0; a < 3; ++a) {
    if (p->grid_cells[a] < 6) return fail(HOT_E_INVALID, "grid_cells must be >= 6 per axis");
    if (!std::isfinite(p->origin[a]) || !std::isfinite(p->gravity[a]))
      return fail(HOT_E_INVALID, "origin/gravity must be finite");
  }
  long long tot = (long long)(p->grid_cells[0] + 5) * (p->grid_cells[1] + 5) * (p->grid_cells[2] + 5);
  if (tot > (1LL << 31) - 1) return fail(HOT_E_INVALID, "grid too large");
  if (!(p->cfl > 0.0) || !(p->max_dt > 0.0)) return fail(HOT_E_INVALID, "cfl and max_dt must be > 0");
  if (!(p->tol >= 0.0)) return fail(HOT_E_INVALID, "tol must be >= 0");
  if (p->lbfgs_history < 0 || p->lbfgs_history > 64)
    return fail(HOT_E_INVALID, "lbfgs_history must be in [0, 64]");
  if (p->mg_levels < 1 || p->mg_levels > kMaxLevels)
    return fail(HOT_E_INVALID, "mg_levels must be in [1, %d]", kMaxLevels);
  if (p->max_iters < 1) return fail(HOT_E_INVALID, "max_iters must be >= 1");
  if (p->smoother_sweeps < 1) return fail(HOT_E_INVALID, "smoother_sweeps must be >= 1");
  if (p->precision != HOT_FP64 && p->precision != HOT_MIXED)
    return fail(HOT_E_INVALID, "unknown precision");
  if (p->smoother != HOT_SMOOTH_L1_JACOBI && p->smoother != HOT_SMOOTH_SGS)
    return fail(HOT_E_INVALID, "unknown smoother");
  if (p->graph != 0 && p->graph != 1) return fail(HOT_E_INVALID, "graph must be 0 or 1");
  if (p->solver != HOT_SOLVER_HOT && p->solver != HOT_SOLVER_PN_PCG &&
      p->solver != HOT_SOLVER_PN_MGPCG)
    return fail(HOT_E_INVALID, "unknown solver");
  return HOT_OK;
}

hot_status validate_positions(const hot_params* p, int64_t n, const double* x) {
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      double t = (x[3 * i + a] - p->origin[a]) / p->dx;
      if (!(t >= 2.0 && t <= (double)(p->grid_cells[a] - 3)))
        return fail(HOT_E_INVALID, "particle %lld outside [origin+2dx, origin+(cells-3)dx]",
                    (long long)i);
    }
  return HOT_OK;
}

// Node counts of every level and the number of occupied cell bricks for a
// particle set, counted on the host (footprint estimate).  Level m+1 holds the
// parents of level m's nodes: even index i -> i/2, odd i -> (i-1)/2, (i+1)/2.
struct SetCounts {
  long long nodes[kMaxLevels] = {0};
  long long bricks = 0;
  long long half0 = 0;  // x-y parents of the level-0 nodes
};

SetCounts count_sets(const hot_params* p, int64_t n, const double* x) {
  SetCounts c;
  int dims[3] = {p->grid_cells[0] + 1, p->grid_cells[1] + 1, p->grid_cells[2] + 1};
  std::vector<uint8_t> mark((size_t)dims[0] * dims[1] * dims[2], 0);
  int bd[3];
  for (int a = 0; a < 3; ++a) bd[a] = (dims[a] + 4 + kBrick - 1) / kBrick;
  std::vector<uint8_t> bmark((size_t)bd[0] * bd[1] * bd[2], 0);
  for (int64_t i = 0; i < n; ++i) {
    long long b[3];
    for (int a = 0; a < 3; ++a) {
      double t = (x[3 * i + a] - p->origin[a]) / p->dx;
      b[a] = std::min(std::max((long long)std::floor(t - 0.5), 0LL), (long long)dims[a] - 3);
    }
    size_t bi = (size_t)((b[0] + 2) / kBrick + bd[0] * ((b[1] + 2) / kBrick + bd[1] * ((b[2] + 2) / kBrick)));
    if (!bmark[bi]) {
      bmark[bi] = 1;
      ++c.bricks;
    }
    for (int k = 0; k < 27; ++k) {
      size_t id = (size_t)(b[0] + k % 3 + dims[0] * (b[1] + (k / 3) % 3 + (size_t)dims[1] * (b[2] + k / 9)));
      if (!mark[id]) {
        mark[id] = 1;
        ++c.nodes[0];
      }
    }
  }
  {
    int hd[3] = {dims[0] / 2 + 1, dims[1] / 2 + 1, dims[2]};
    std::vector<uint8_t> hm((size_t)hd[0] * hd[1] * hd[2], 0);
    for (int z = 0; z < dims[2]; ++z)
      for (int y = 0; y < dims[1]; ++y)
        for (int xx = 0; xx < dims[0]; ++xx) {
          if (!mark[(size_t)xx + dims[0] * ((size_t)y + (size_t)dims[1] * z)]) continue;
          for (int Y = y / 2; Y <= (y + 1) / 2; ++Y)
            for (int X = xx / 2; X <= (xx + 1) / 2; ++X) {
              size_t id = (size_t)X + hd[0] * ((size_t)Y + (size_t)hd[1] * z);
              if (!hm[id]) {
                hm[id] = 1;
                ++c.half0;
              }
            }
        }
  }
  for (int m = 1; m < p->mg_levels; ++m) {
    int cd[3] = {dims[0] / 2 + 1, dims[1] / 2 + 1, dims[2] / 2 + 1};
    std::vector<uint8_t> cm((size_t)cd[0] * cd[1] * cd[2], 0);
    for (int z = 0; z < dims[2]; ++z)
      for (int y = 0; y < dims[1]; ++y)
        for (int xx = 0; xx < dims[0]; ++xx) {
          if (!mark[(size_t)xx + dims[0] * ((size_t)y + (size_t)dims[1] * z)]) continue;
          int lo[3] = {xx / 2, y / 2, z / 2};
          int hi[3] = {(xx + 1) / 2, (y + 1) / 2, (z + 1) / 2};
          for (int Z = lo[2]; Z <= hi[2]; ++Z)
            for (int Y = lo[1]; Y <= hi[1]; ++Y)
              for (int X = lo[0]; X <= hi[0]; ++X) {
                size_t id = (size_t)X + cd[0] * ((size_t)Y + (size_t)cd[1] * Z);
                if (!cm[id]) {
                  cm[id] = 1;
                  ++c.nodes[m];
                }
              }
        }
    mark.swap(cm);
    for (int a = 0; a < 3; ++a) dims[a] = cd[a];
  }
  return c;
}

// Points of the padded grid of level m.
long long gm_level_ptotal(const hot_params* p, int m) {
  GridGeom g = make_geom(p->grid_cells[0] + 1, p->grid_cells[1] + 1, p->grid_cells[2] + 1);
  for (int k = 0; k < m; ++k) g = make_geom(g.dims[0] / 2 + 1, g.dims[1] / 2 + 1, g.dims[2] / 2 + 1);
  return g.ptotal;
}

// Device bytes a scene allocates for a particle set of this shape: every
// buffer the step uses, with the 25% growth headroom each allocation takes.
// Exact for the initial configuration; a scene whose active grid grows later
// allocates more.
size_t estimate_bytes(const hot_params* p, int64_t n, const SetCounts& c) {
  double tot = 0.0;
  auto A = [&](double bytes) { tot += std::max(bytes, 8.0) * 1.25; };
  const double N = (double)n;
  // particle state (two sets), per-particle work arrays, keys
  A(N * 208); A(N * 208);
  A(N * 24); A(N * kAsmRec * 8); A(N * 8); A(N * 8); A(N * 72); A(N * 72);
  A(N * 4); A(N * 4); A(N * 4);
  // dense maps over the padded level grids, bricks, reductions
  int dims[3] = {p->grid_cells[0] + 1, p->grid_cells[1] + 1, p->grid_cells[2] + 1};
  GridGeom g0 = make_geom(dims[0], dims[1], dims[2]);
  double pt = (double)g0.ptotal;
  A(pt * 32);  // node velocities
  A(pt * 4); A(pt * 4 + 4); A(pt * 4); A(pt * 4); A(pt * 4 + 4); A((pt / 2048 + 2) * 4); A(64);
  GridGeom gm = g0;
  for (int m = 0; m < p->mg_levels; ++m) {
    if (m > 0) gm = make_geom(gm.dims[0] / 2 + 1, gm.dims[1] / 2 + 1, gm.dims[2] / 2 + 1);
    A((double)gm.ptotal * 4);
  }
  double nbt = 1.0;
  for (int a = 0; a < 3; ++a) nbt *= (double)((g0.pd[a] + kBrick - 1) / kBrick);
  A(nbt * 4);
  const double W = p->lbfgs_history + 1;
  for (int k = 0; k < 2; ++k) A(W * 8);
  A(NSCAL * 8); A(kRedBlocks * 4 * 8);  // scalars, partials
  A((double)(sizeof(MaterialDev) * kMaxMats + sizeof(BcDev) * kMaxBcs));  // tables
  A((double)c.bricks * 4); A((double)c.bricks * kBrickWin * 5 * 8);
  // levels
  const bool mx = p->precision == HOT_MIXED;
  const double vsz = mx ? 4 : 8;
  for (int m = 0; m < p->mg_levels; ++m) {
    double nm = (double)c.nodes[m];
    A(nm * 4); A(nm * kRowStride * 8); A(nm * 72); A(nm * 24); A(nm * 3); A(nm * 16);
    if (mx) { A(nm * kRowStride * 2); A(nm * 36); A(nm * 12); }
    A(nm * 3 * vsz); A(nm * 3 * vsz);  // b, r
    A((double)gm_level_ptotal(p, m) * 4 * vsz); A((double)gm_level_ptotal(p, m) * 4 * vsz);  // u, t
    if (p->smoother == HOT_SMOOTH_SGS && m + 1 < p->mg_levels) {
      A(nm * 4); A((kColors + 1) * 4.0); A(nm * 72);
      if (mx) A(nm * 36);
    }
  }
  if (p->smoother == HOT_SMOOTH_SGS) A((double)color_scratch_bytes((int)c.nodes[0]));
  // half-coarsened grid of the level-0 Galerkin product (the largest)
  if (p->mg_levels > 1) {
    GridGeom th = make_geom(g0.dims[0] / 2 + 1, g0.dims[1] / 2 + 1, g0.dims[2]);
    const double nt = (double)c.half0;
    A(nt * 4); A((double)th.ptotal * 4); A(nt * 16); A(nt * kRowStride * 8);
  }
  // level-0 node data, solver vectors and history, row segments
  const double n0 = (double)c.nodes[0];
  A(n0 * 8); A(n0 * 8); A(n0 * 4);
  for (int k = 0; k < 9; ++k) A(n0 * 24);
  for (int k = 0; k < 2 * W; ++k) A(n0 * 24);
  A((n0 + 1) * 4);
  double nc = (double)c.nodes[p->mg_levels - 1];
  A(4 * 3 * nc * 8);
  A((p->max_iters * 3 + 16) * 4.0);
  return (size_t)tot + ((size_t)1 << 16);
}

// ---------------------------------------------------------------- prepare
// Coloured Gauss-Seidel set-up of the smoothed levels 0 .. M-2: the rows of
// each colour and the inverses of the 3x3 diagonal blocks; the colour
// offsets come to the host for the launch sizes.
hot_status prepare_sgs(hot_scene* s) {
  hipStream_t st = s->stream;
  TRY(ensure(s, s->cscratch, color_scratch_bytes(s->L[0].n)));
  for (int m = 0; m + 1 < s->levels; ++m) {
    LevelH& L = s->L[m];
    TRY(ensure(s, L.crow, (size_t)L.n * 4));
    TRY(ensure(s, L.coffd, (kColors + 1) * 4));
    TRY(ensure(s, L.Dg, (size_t)L.n * 72));
    if (s->mixed) TRY(ensure(s, L.Dg32, (size_t)L.n * 36));
    LevelView v = view(s, m);
    launch_color_rows(v, P<int>(s->cscratch), P<int>(L.coffd), P<int>(L.crow), st);
    launch_block_diag_inv(v, P<double>(L.Dg), s->mixed ? P<float>(L.Dg32) : nullptr, st);
    HIPCHK(hipMemcpyAsync(L.coff, L.coffd.p, sizeof(L.coff), hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  for (int m = 0; m + 1 < s->levels; ++m)
    if (s->L[m].coff[kColors] != s->L[m].n)
      return fail(HOT_E_DEVICE, "colour lists of level %d are inconsistent", m);
  return HOT_OK;
}

// One symmetric Gauss-Seidel smoothing (forward pass over the colours, then
// backward), repeated smoother_sweeps times, in place on the level iterate u.
// The backward pass starts at colour 25: colour 26 would recompute exactly
// the values the forward pass has just given it (same inputs).
void sgs_smooth(hot_scene* s, int m, const void* b, void* u) {
  LevelH& L = s->L[m];
  LevelView v = view(s, m);
  const void* Dg = s->mixed ? L.Dg32.p : L.Dg.p;
  for (int k = 0; k < s->prm.smoother_sweeps; ++k) {
    for (int c = 0; c < kColors; ++c)
      launch_sgs_color(v, s->mixed, P<int>(L.crow) + L.coff[c], L.coff[c + 1] - L.coff[c], Dg, b,
                       u, s->stream);
    for (int c = kColors - 2; c >= 0; --c)
      launch_sgs_color(v, s->mixed, P<int>(L.crow) + L.coff[c], L.coff[c + 1] - L.coff[c], Dg, b,
                       u, s->stream);
  }
}

hot_status alloc_level(hot_scene* s, int m, int n) {
  LevelH& L = s->L[m];
  size_t vsz = s->mixed ? 4 : 8;
  TRY(ensure(s, L.nodes, (size_t)n * 4));
  TRY(ensure(s, L.H, (size_t)n * kRowStride * 8));
  TRY(ensure(s, L.Dinv, (size_t)n * 72));
  TRY(ensure(s, L.diag, (size_t)n * 24));
  TRY(ensure(s, L.freed, (size_t)n * 3));
  TRY(ensure(s, L.pat, (size_t)n * 16));
  if (s->mixed) {
    TRY(ensure(s, L.Hb, (size_t)n * kRowStride * 2));
    TRY(ensure(s, L.Dinv32, (size_t)n * 36));
    TRY(ensure(s, L.diag32, (size_t)n * 12));
  }
  TRY(ensure(s, L.b, (size_t)n * 3 * vsz));
  TRY(ensure(s, L.u, (size_t)L.g.ptotal * 4 * vsz));
  TRY(ensure(s, L.r, (size_t)n * 3 * vsz));
  TRY(ensure(s, L.t, (size_t)L.g.ptotal * 4 * vsz));
  L.n = n;
  return HOT_OK;
}

hot_status alloc_nodes0(hot_scene* s, int n) {
  size_t v = (size_t)n * 3 * 8;
  TRY(ensure(s, s->mass, (size_t)n * 8));
  TRY(ensure(s, s->xi, (size_t)n * 8));
  TRY(ensure(s, s->fixed, (size_t)n * 4));
  TRY(ensure(s, s->vstar, v));
  TRY(ensure(s, s->dv, v));
  TRY(ensure(s, s->dvt, v));
  TRY(ensure(s, s->g, v));
  TRY(ensure(s, s->gnew, v));
  TRY(ensure(s, s->q, v));
  TRY(ensure(s, s->r, v));
  TRY(ensure(s, s->vin, v));
  TRY(ensure(s, s->vout, v));
  int W = s->prm.lbfgs_history + 1;
  s->Sh.resize(W);
  s->Yh.resize(W);
  for (int a = 0; a < W; ++a) {
    TRY(ensure(s, s->Sh[a], v));
    TRY(ensure(s, s->Yh[a], v));
  }
  return HOT_OK;
}

hot_status build_hessian(hot_scene* s, const double* dv);

// Binning, active grid and hierarchy index sets, P2G, level-0 Hessian and the
// Galerkin hierarchy: everything of a step that precedes the solve.
hot_status prepare(hot_scene* s, double dt) {
  hipStream_t st = s->stream;
  s->vc_stale = true;  // level sizes change with every step
  const int n = s->n;
  const GridGeom& g0 = s->sd.g0;
  Particles& src = s->P[s->cur];
  // -- binning: base-node keys, counting sort, stable within a cell
  launch_fill_int(g0.ptotal, P<int>(s->counts), 0, st);
  launch_fill_int(1, P<int>(s->err), 0, st);
  launch_bin_keys(s->sd, n, src.x, P<int>(s->keys), P<int>(s->counts), P<int>(s->err), st);
  launch_scan(g0.ptotal, P<int>(s->counts), P<int>(s->start), s->scan_temp.p, st);
  int errv = 0;
  TRY(read_int(s, P<int>(s->err), &errv));
  if (errv) return fail(HOT_E_INVALID, "a particle left the valid grid region");
  // -- cell bricks holding particles
  {
    Bricks& B = s->bricks;
    launch_fill_int(B.bg.total, P<int>(s->flags), 0, st);
    launch_mark_bricks(g0, B.bg, P<int>(s->counts), P<int>(s->flags), st);
    launch_scan(B.bg.total, P<int>(s->flags), P<int>(s->scan), s->scan_temp.p, st);
    int nb = 0;
    TRY(read_int(s, P<int>(s->scan) + B.bg.total, &nb));
    TRY(ensure(s, s->blist, (size_t)nb * 4));
    TRY(ensure(s, s->bpartial, (size_t)nb * kBrickWin * 5 * 8));
    launch_brick_compact(B.bg.total, P<int>(s->flags), P<int>(s->scan), P<int>(s->bmap),
                         P<int>(s->blist), st);
    B.n = nb;
    B.list = P<int>(s->blist);
    B.map = P<int>(s->bmap);
  }
  launch_fill_int(g0.ptotal, P<int>(s->cursor), 0, st);
  launch_scatter_sorted(n, P<int>(s->keys), P<int>(s->start), P<int>(s->cursor), P<int>(s->tmp), st);
  launch_sort_segments(g0.ptotal, P<int>(s->start), P<int>(s->counts), src.id, P<int>(s->tmp), st);
  launch_permute_particles(n, P<int>(s->tmp), src, s->P[1 - s->cur], st);
  s->cur = 1 - s->cur;
  Particles& pt = s->P[s->cur];
  launch_particle_frac(s->sd, n, pt.x, P<double>(s->f), P<int>(s->key), st);
  // -- active nodes per level
  for (int m = 0; m < s->levels; ++m) {
    LevelH& L = s->L[m];
    launch_fill_int(L.g.ptotal, P<int>(s->flags), 0, st);
    if (m == 0)
      launch_mark_fine(L.g, P<int>(s->counts), P<int>(s->flags), st);
    else
      launch_mark_coarse(s->L[m - 1].g, s->L[m - 1].n, P<int>(s->L[m - 1].nodes), L.g,
                         P<int>(s->flags), st);
    launch_scan(L.g.ptotal, P<int>(s->flags), P<int>(s->scan), s->scan_temp.p, st);
    int nm = 0;
    TRY(read_int(s, P<int>(s->scan) + L.g.ptotal, &nm));
    TRY(alloc_level(s, m, nm));
    if (m == 0) TRY(alloc_nodes0(s, nm));
    launch_compact(L.g.ptotal, P<int>(s->flags), P<int>(s->scan), P<int>(L.map), P<int>(L.nodes), st);
  }
  LevelView L0 = view(s, 0);
  launch_fine_pattern(L0, P<int>(s->counts), st);
  // -- row segments of the level-0 assembly
  {
    launch_seg_flags(L0, P<int>(s->flags), st);
    launch_scan(L0.n, P<int>(s->flags), P<int>(s->scan), s->scan_temp.p, st);
    int ns = 0;
    TRY(read_int(s, P<int>(s->scan) + L0.n, &ns));
    TRY(ensure(s, s->seg_begin, (size_t)(ns + 1) * 4));
    launch_seg_compact(L0.n, P<int>(s->flags), P<int>(s->scan), P<int>(s->seg_begin), st);
    s->n_seg = ns;
  }
  // -- P2G, gravity, boundary velocities
  launch_p2g(s->sd, L0, s->bricks, P<double>(s->f), pt.v, pt.C, pt.vol, pt.mat, P<int>(s->start),
             P<int>(s->counts), P<double>(s->bpartial), dt, s->t + dt, P<double>(s->mass),
             P<double>(s->vstar), P<double>(s->xi), P<int>(s->fixed), st);
  HIPCHK(hipEventRecord(s->ev[1], st));
  s->dt_prepared = dt;
  TRY(build_hessian(s, nullptr));
  launch_fill_int(1, pcg_log(s).cursor, 0, st);
  s->prepared = true;
  s->vcycles = 0;
  return HOT_OK;
}

// Level-0 projected Hessian at dv (NULL: dv = 0, Alg. HOT's start-of-step
// Hessian) and, for levels > 1, its Galerkin hierarchy with the smoother
// data and the coarsest solve's work space.
hot_status build_hessian(hot_scene* s, const double* dv) {
  hipStream_t st = s->stream;
  const int n = s->n;
  Particles& pt = s->P[s->cur];
  LevelView L0 = view(s, 0);
  const double dt = s->dt_prepared;
  s->vc_stale = true;  // the matrices change
  PROF(s, HOT_PROF_PHESS,
       launch_particle_hessian(s->sd, L0, n, P<double>(s->f), P<int>(s->key), pt.F, pt.vol,
                               pt.mat, P<double>(s->vstar), dv, dt, P<double>(s->wnode),
                               P<double>(s->arec), st));
  PROF(s, HOT_PROF_ASSEMBLE,
       launch_assemble_h0(s->sd, L0, P<int>(s->seg_begin), s->n_seg, n, P<double>(s->arec),
                          P<int>(s->start), P<int>(s->counts), P<double>(s->mass),
                          P<int>(s->fixed), st));
  for (int m = 0; m + 1 < s->levels; ++m) {
    // rows of the half-coarsened grid: x-y parents of level m's nodes
    const GridGeom& fg = s->L[m].g;
    LevelView T;
    std::memset(&T, 0, sizeof(T));
    T.g = make_geom(fg.dims[0] / 2 + 1, fg.dims[1] / 2 + 1, fg.dims[2]);
    launch_fill_int(T.g.ptotal, P<int>(s->flags), 0, st);
    launch_mark_xy(fg, s->L[m].n, P<int>(s->L[m].nodes), T.g, P<int>(s->flags), st);
    launch_scan(T.g.ptotal, P<int>(s->flags), P<int>(s->scan), s->scan_temp.p, st);
    int nt = 0;
    TRY(read_int(s, P<int>(s->scan) + T.g.ptotal, &nt));
    TRY(ensure(s, s->tnodes, (size_t)nt * 4));
    TRY(ensure(s, s->tmap, (size_t)T.g.ptotal * 4));
    TRY(ensure(s, s->tpat, (size_t)nt * 16));
    TRY(ensure(s, s->tH, (size_t)nt * kRowStride * 8));
    launch_compact(T.g.ptotal, P<int>(s->flags), P<int>(s->scan), P<int>(s->tmap),
                   P<int>(s->tnodes), st);
    T.n = nt;
    T.nodes = P<int>(s->tnodes);
    T.map = P<int>(s->tmap);
    T.pat = P<uint32_t>(s->tpat);
    T.H = P<double>(s->tH);
    if (m == 0)
      PROF(s, HOT_PROF_RAP0, launch_rap(view(s, m), T, view(s, m + 1), st));
    else
      launch_rap(view(s, m), T, view(s, m + 1), st);
  }
  // structural block counts of every level (the traced kernels' bytes)
  if (s->prof)
    for (int m = 0; m < s->levels; ++m)
      launch_pattern_count(view(s, m), P<double>(s->dscal) + S_NNZ + m, st);
  if (s->mixed)  // level 0's BF16 copy comes from the assembly itself
    for (int m = 1; m < s->levels; ++m) launch_to_bf16(view(s, m), st);
  if (s->prm.smoother == HOT_SMOOTH_SGS && s->levels > 1) TRY(prepare_sgs(s));
  size_t pcg = coarse_pcg_work_bytes(s->L[s->levels - 1].n);
  TRY(ensure(s, s->pcg_work, pcg));
  TRY(ensure(s, s->pcg_iters, pcg_log_bytes(s->prm.max_iters)));
  if (s->prm.graph) coarse_pcg_warm();
  HIPCHK(hipGetLastError());
  return HOT_OK;
}

// ---------------------------------------------------------------- V-cycle
// r = V(q): one multigrid V-cycle (Alg. V-cycle) with l1 block-Jacobi or
// coloured symmetric block Gauss-Seidel smoothing and an inexact Jacobi-PCG
// coarsest solve.  In the mixed policy the
// cycle runs on FP32 vectors over BF16 blocks; q and r stay FP64.
hot_status vcycle_body(hot_scene* s, const double* q, double* r) {
  hipStream_t st = s->stream;
  const bool mx = s->mixed;
  const int M = s->levels;
  const int sweeps = s->prm.smoother_sweeps;
  void* b0;
  if (mx) {
    launch_to_f32((long long)s->L[0].n * 3, q, P<float>(s->L[0].b), st);
    b0 = s->L[0].b.p;
  } else {
    b0 = (void*)q;
  }
  std::vector<void*> bs(M), us(M);
  bs[0] = b0;
  for (int m = 0; m < M; ++m) {
    us[m] = s->L[m].u.p;
    if (m > 0) bs[m] = s->L[m].b.p;
  }
  const bool gs = s->prm.smoother == HOT_SMOOTH_SGS;
  for (int m = 0; m + 1 < M; ++m) {
    LevelView Lm = view(s, m);
    if (gs) {
      launch_zero_rows(Lm, mx, us[m], st);
      if (m == 0)
        PROF(s, HOT_PROF_SGS0, sgs_smooth(s, m, bs[m], us[m]));
      else
        sgs_smooth(s, m, bs[m], us[m]);
    } else if (m == 0) {
      launch_jacobi_first(Lm, mx, bs[m], us[m], st);
    }  // levels m > 0 got their first smoothing from the restriction
    for (int k = 1; k < sweeps && !gs; ++k) {
      if (m == 0)
        PROF(s, HOT_PROF_SMOOTH0, launch_smooth(Lm, mx, bs[m], us[m], s->L[m].t.p, st));
      else
        launch_smooth(Lm, mx, bs[m], us[m], s->L[m].t.p, st);
      std::swap(s->L[m].u, s->L[m].t);
      us[m] = s->L[m].u.p;
    }
    if (m == 0)
      PROF(s, HOT_PROF_RESIDUAL0, launch_residual(Lm, mx, bs[m], us[m], s->L[m].r.p, st));
    else
      launch_residual(Lm, mx, bs[m], us[m], s->L[m].r.p, st);
    const bool first = !gs && m + 2 < M;  // level m + 1 is smoothed, not solved
    launch_restrict(Lm, view(s, m + 1), mx, s->L[m].r.p, bs[m + 1], first ? us[m + 1] : nullptr,
                    st);
  }
  HIPCHK(launch_coarse_pcg(view(s, M - 1), mx, bs[M - 1], us[M - 1], s->pcg_work.p, pcg_log(s),
                           500, 0.5, s->grid_ok, st));
  for (int m = M - 2; m >= 0; --m) {
    LevelView Lm = view(s, m);
    launch_prolong_add(Lm, view(s, m + 1), mx, us[m + 1], us[m], st);
    if (gs) {
      if (m == 0)
        PROF(s, HOT_PROF_SGS0, sgs_smooth(s, m, bs[m], us[m]));
      else
        sgs_smooth(s, m, bs[m], us[m]);
    }
    for (int k = 0; k < sweeps && !gs; ++k) {
      if (m == 0)
        PROF(s, HOT_PROF_SMOOTH0, launch_smooth(Lm, mx, bs[m], us[m], s->L[m].t.p, st));
      else
        launch_smooth(Lm, mx, bs[m], us[m], s->L[m].t.p, st);
      std::swap(s->L[m].u, s->L[m].t);
      us[m] = s->L[m].u.p;
    }
  }
  launch_dense_out(view(s, 0), mx, s->L[0].u.p, r, st);
  return HOT_OK;
}

// With hot_params.graph set, the solve's cycles (q and r the solver's own
// vectors) run as one HIP graph per step: the first cycle after prepare is
// captured on the scene's stream and instantiated, and every cycle of the
// step launches that graph.  The launches are the same kernels with the same
// arguments as the eager cycle; the coarse-PCG log advances on the device.
hot_status vcycle(hot_scene* s, const double* q, double* r) {
  // (not inside hot_step_noalloc: instantiating a graph may allocate)
  const bool graph = s->prm.graph && !s->prof && !s->no_alloc && q == P<double>(s->q) &&
                     r == P<double>(s->r);
  if (!graph) {
    PROF(s, HOT_PROF_VCYCLE, TRY(vcycle_body(s, q, r)));
  } else {
    if (s->vc_stale) {
      HIPCHK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
      hot_status rc = vcycle_body(s, q, r);
      hipGraph_t gr = nullptr;
      hipError_t e = hipStreamEndCapture(s->stream, &gr);
      if (rc < 0) {
        if (gr) (void)hipGraphDestroy(gr);
        return rc;
      }
      if (e != hipSuccess)
        return fail(HOT_E_DEVICE, "V-cycle capture failed: %s", hipGetErrorString(e));
      // the cycle of a new step usually has the previous step's launch
      // sequence with new sizes and buffers: update the executable graph in
      // place, and instantiate afresh only when that is refused
      bool updated = false;
      if (s->vc_exec) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res;
        updated = hipGraphExecUpdate(s->vc_exec, gr, &err_node, &res) == hipSuccess &&
                  res == hipGraphExecUpdateSuccess;
        if (!updated) {
          (void)hipGetLastError();
          (void)hipGraphExecDestroy(s->vc_exec);
          s->vc_exec = nullptr;
        }
      }
      if (!updated) e = hipGraphInstantiate(&s->vc_exec, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      if (e != hipSuccess) {
        s->vc_exec = nullptr;
        return fail(HOT_E_DEVICE, "V-cycle graph instantiation failed: %s", hipGetErrorString(e));
      }
      s->vc_stale = false;
    }
    HIPCHK(hipGraphLaunch(s->vc_exec, s->stream));
  }
  s->vcycles++;
  return HOT_OK;
}

// ---------------------------------------------------------------- grid-solve tickets
TicketPool* grid_tickets(int dev) {
  static std::mutex mu;
  static TicketPool* pools[64] = {nullptr};
  if (dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (!pools[dev]) pools[dev] = new TicketPool(kGridSolves);
  return pools[dev];
}

// Holds a grid-solve ticket of the scene's device while the scene's V-cycles
// run, when its coarsest level uses the multi-work-group solve, waiting for
// one if all are taken (the single-work-group form sums in another order, so
// falling back to it would make a scene's result depend on what else runs).
// Released after the scene's stream has drained.
class GridTicket {
 public:
  explicit GridTicket(hot_scene* s) : s_(s) {
    const LevelView Lc = view(s, s->levels - 1);
    TicketPool* pool = grid_tickets(s->device);
    if (pool && coarse_pcg_uses_grid(Lc, s->mixed)) {
      pool->acquire();
      held_ = true;
    }
    s->grid_ok = held_;
  }
  ~GridTicket() {
    if (held_) {
      (void)hipStreamSynchronize(s_->stream);
      grid_tickets(s_->device)->release();
    }
    s_->grid_ok = false;
  }

 private:
  hot_scene* s_;
  bool held_ = false;
};

// ---------------------------------------------------------------- solve
hot_status eval_trial(hot_scene* s, const double* dv, const double* p, double alpha, int out) {
  Particles& pt = s->P[s->cur];
  PROF(s, HOT_PROF_EVAL,
       launch_particle_eval(s->sd, view(s, 0), s->n, P<double>(s->f), P<int>(s->key), pt.F,
                            pt.vol, pt.mat, P<double>(s->vstar), dv, p, alpha, s->dt_prepared,
                            P<double>(s->wnode), P<double>(s->psi[out]), P<double>(s->S[out]),
                            s->stream));
  return HOT_OK;
}

hot_status gradient(hot_scene* s, const double* dv, int sbuf, double* g) {
  PROF(s, HOT_PROF_GRAD,
       launch_gradient(s->sd, view(s, 0), s->bricks, P<double>(s->f), P<double>(s->S[sbuf]),
                       P<int>(s->start), P<int>(s->counts), P<double>(s->bpartial),
                       P<double>(s->mass), P<int>(s->fixed), dv, s->dt_prepared, g, s->stream));
  return HOT_OK;
}

// Algorithmic bytes of one whole V-cycle with nu smoothing sweeps.  Every
// non-coarsest level m runs (l1 block-Jacobi) nu - 1 further pre-smoothing
// sweeps after the first one from zero, a residual pass and nu
// post-smoothing sweeps over its structural blocks (2 nu matrix reads), with
// the vectors each reads and writes once (the same counts as the traced
// level-0 kernels); the first smoothing from zero on level 0 (b and D~^-1
// in, u out; coarser levels get it from the restriction); the restriction (r
// in; b and, unless the next level is the coarsest, D~^-1 and u of the next
// level) and the prolongation (coarse u in, u in and out).  With
// Gauss-Seidel: a clearing of u, nu forward-backward pairs before and after,
// each of the traced level-0 form, and the residual.  The coarsest Jacobi-PCG
// reads its matrix and five vectors once per iteration (the step's average
// iteration count per cycle).  Mixed precision adds the FP32 conversion of
// the input; the FP64 output is written once.
double vcycle_bytes(hot_scene* s) {
  const bool mx = s->mixed, gs = s->prm.smoother == HOT_SMOOTH_SGS;
  const double vs = mx ? 4.0 : 8.0, ms = mx ? 18.0 : 72.0;
  const double nu = s->prm.smoother_sweeps;
  const int M = s->levels;
  const double n0 = s->L[0].n;
  double b = mx ? 36.0 * n0 : 0.0;
  for (int m = 0; m + 1 < M; ++m) {
    const LevelH& L = s->L[m];
    const double n = L.n, nnz = s->hscal[S_NNZ + m], nc = s->L[m + 1].n;
    if (gs) {
      const double f = 2.0 - (double)(L.coff[kColors] - L.coff[kColors - 1]) / std::max(n, 1.0);
      b += 4.0 * vs * n + 2.0 * nu * f * (ms * nnz + (mx ? 85.0 : 107.0) * n);
    } else {
      if (m == 0) b += 16.0 * vs * n;
      b += (2.0 * nu - 1.0) * (ms * nnz + (mx ? 79.0 : 151.0) * n);  // smoothing sweeps
    }
    b += ms * nnz + (mx ? 40.0 : 76.0) * n;  // residual
    const bool first = !gs && m + 2 < M;
    b += 3.0 * vs * n + 3.0 * vs * nc + (first ? 13.0 * vs * nc : 0.0);  // restriction
    b += 4.0 * vs * nc + 8.0 * vs * n;                                    // prolongation
  }
  const double nc = s->L[M - 1].n, nnzc = s->hscal[S_NNZ + M - 1];
  b += std::max(s->cg_per_cycle, 1.0) * (ms * nnzc + 15.0 * vs * nc);
  b += 4.0 * vs * n0 + 24.0 * n0;
  return b;
}

// Algorithmic bytes one launch of a traced kernel must move (structural
// blocks and node/particle vectors read or written once).
double prof_launch_bytes(hot_scene* s, int kind) {
  double n0 = s->L[0].n, np = s->n;
  double nnz0 = s->hscal[S_NNZ], nnz1 = s->levels > 1 ? s->hscal[S_NNZ + 1] : 0.0;
  double n1 = s->levels > 1 ? s->L[1].n : 0.0;
  bool mx = s->mixed;
  switch (kind) {
    case HOT_PROF_SMOOTH0: return mx ? 18.0 * nnz0 + 79.0 * n0 : 72.0 * nnz0 + 151.0 * n0;
    // a forward pass over all rows and a backward pass over all but colour
    // 26's, each row reading its off-diagonal blocks, diagonal-block inverse,
    // b, the gathered iterate, row list entry, node index, pattern and free
    // flags once and writing its iterate entries once (blocks counted in
    // proportion to rows)
    case HOT_PROF_SGS0: {  // smoother_sweeps forward-backward pairs
      const LevelH& L0 = s->L[0];
      const double f = 2.0 - (double)(L0.coff[kColors] - L0.coff[kColors - 1]) / std::max(n0, 1.0);
      return s->prm.smoother_sweeps *
             (mx ? f * (18.0 * nnz0 + 85.0 * n0) : f * (72.0 * nnz0 + 107.0 * n0));
    }
    case HOT_PROF_RESIDUAL0: return mx ? 18.0 * nnz0 + 40.0 * n0 : 72.0 * nnz0 + 76.0 * n0;
    case HOT_PROF_ASSEMBLE: return 72.0 * nnz0 + 456.0 * np + 111.0 * n0;
    case HOT_PROF_RAP0: return 72.0 * nnz0 + 23.0 * n0 + 72.0 * nnz1 + 111.0 * n1;
    case HOT_PROF_EVAL: return 192.0 * np + 72.0 * n0;
    case HOT_PROF_GRAD: return 96.0 * np + 64.0 * n0;
    case HOT_PROF_PHESS: return 1120.0 * np + 24.0 * n0;
    case HOT_PROF_VCYCLE: return vcycle_bytes(s);
  }
  return 0.0;
}

hot_status prof_flush(hot_scene* s) {
  if (!s->prof) return HOT_OK;
  for (size_t k = 0; k + 1 < s->prof_used; k += 2) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, s->prof_ev[k], s->prof_ev[k + 1]));
    int kind = s->prof_kind[k / 2];
    s->prof_ms[kind] += ms;
    s->prof_n[kind] += 1;
    s->prof_bytes[kind] += prof_launch_bytes(s, kind);
  }
  s->prof_used = 0;
  return HOT_OK;
}

// HOT quasi-Newton solve (Alg. HOT): L-BFGS two-loop with the V-cycle as the
// initial inverse Hessian, backtracking line search from alpha = 1 (Armijo,
// c1 = 1e-4, halving, at most 30 halvings, energy change summed as
// per-particle and per-node differences), secant pairs kept when
// y^T s > 1e-12 |y||s|, and the node-wise CN stopping test (Sec. 5.2).
hot_status solve(hot_scene* s, hot_step_stats* stats, bool* converged) {
  hipStream_t st = s->stream;
  GridTicket ticket(s);
  const int n0 = s->L[0].n;
  const long long N = (long long)n0 * 3;
  const double dt = s->dt_prepared;
  const double cn_scale = 24.0 * s->prm.dx * s->prm.dx * dt;
  const double thresh = s->prm.tol * std::sqrt((double)n0);
  const int w = s->prm.lbfgs_history;
  double* dscal = P<double>(s->dscal);
  double* partial = P<double>(s->partial);
  double* dv = P<double>(s->dv);
  double* dvt = P<double>(s->dvt);
  double* g = P<double>(s->g);
  double* gnew = P<double>(s->gnew);
  double* q = P<double>(s->q);
  double* r = P<double>(s->r);
  s->log_int.clear();
  s->log_cn.clear();
  launch_fill_double(N, dv, 0.0, st);
  s->pc = 0;
  TRY(eval_trial(s, dv, nullptr, 0.0, s->pc));
  launch_sum(s->n, P<double>(s->psi[s->pc]), partial, dscal + S_E0, st);
  TRY(gradient(s, dv, s->pc, g));
  launch_cn_sq(n0, g, P<double>(s->xi), cn_scale, partial, dscal + S_CN, st);
  TRY(readback(s));
  double E = s->hscal[S_E0];
  double cn = std::sqrt(s->hscal[S_CN]);
  if (!std::isfinite(E) || !std::isfinite(cn))
    return fail(HOT_E_NONFINITE, "non-finite energy or gradient at dv = 0");
  if (stats) {
    stats->E0 = E;
    stats->cn0 = cn;
    stats->cn_tol = thresh;
  }
  s->log_cn.push_back(cn);
  std::vector<int> hist;  // slot ids, oldest first
  const int W = w + 1;
  int it = 0, backtracks = 0, fallbacks = 0, skipped = 0;
  bool conv = cn <= thresh;
  std::vector<std::pair<int, int>> vc_range;
  while (!conv && it < s->prm.max_iters) {
    int vc0 = s->vcycles;
    // -- two-loop recursion: each inner step finishes the previous inner
    //    product, updates the vector and starts the next inner product
    double* pbuf[2] = {partial, partial + kRedBlocks};
    int pb = 0;
    const int K = (int)hist.size();
    if (K == 0) {
      launch_scale_copy(N, -1.0, g, q, st);
    } else {
      launch_twoloop_start(N, g, q, P<double>(s->Sh[hist[K - 1]]), pbuf[pb], st);
      for (int k = K - 1; k >= 0; --k) {
        const int a = hist[k];
        const double* dn = k > 0 ? P<double>(s->Sh[hist[k - 1]]) : nullptr;
        launch_twoloop_step(N, pbuf[pb], P<double>(s->drho) + a, nullptr, P<double>(s->dalpha) + a,
                            P<double>(s->Yh[a]), q, dn, pbuf[1 - pb], st);
        pb = 1 - pb;
      }
    }
    TRY(vcycle(s, q, r));
    if (K == 0) {
      launch_dot(N, g, r, partial, dscal + S_GP, st);
    } else {
      launch_twoloop_start(N, nullptr, r, P<double>(s->Yh[hist[0]]), pbuf[pb], st);
      for (int k = 0; k < K; ++k) {
        const int a = hist[k];
        const double* dn = k + 1 < K ? P<double>(s->Yh[hist[k + 1]]) : g;
        launch_twoloop_step(N, pbuf[pb], P<double>(s->drho) + a, P<double>(s->dalpha) + a, nullptr,
                            P<double>(s->Sh[a]), r, dn, pbuf[1 - pb], st);
        pb = 1 - pb;
      }
      launch_finish_partials(N, pbuf[pb], dscal + S_GP, st);
    }
    // -- descent check and the first trial in one readback
    int trial = 1 - s->pc;
    TRY(eval_trial(s, dv, r, 1.0, trial));
    launch_energy_delta(s->n, P<double>(s->psi[trial]), P<double>(s->psi[s->pc]), n0,
                        P<double>(s->mass), dv, r, 1.0, partial, dscal + S_DEP, st);
    TRY(readback(s));
    double gp = s->hscal[S_GP];
    int fb = 0;
    if (!(gp < 0.0)) {
      hist.clear();
      fb = 1;
      launch_scale_copy(N, -1.0, g, q, st);
      TRY(vcycle(s, q, r));
      launch_dot(N, g, r, partial, dscal + S_GP, st);
      TRY(readback(s));
      gp = s->hscal[S_GP];
      if (!(gp < 0.0)) {
        fb = 2;
        launch_block_jacobi_apply(n0, P<double>(s->L[0].Dinv), g, r, -1.0, st);
        launch_dot(N, g, r, partial, dscal + S_GP, st);
        TRY(readback(s));
        gp = s->hscal[S_GP];
      }
      TRY(eval_trial(s, dv, r, 1.0, trial));
      launch_energy_delta(s->n, P<double>(s->psi[trial]), P<double>(s->psi[s->pc]), n0,
                          P<double>(s->mass), dv, r, 1.0, partial, dscal + S_DEP, st);
      TRY(readback(s));
      ++fallbacks;
    }
    double alpha = 1.0;
    bool accepted = false;
    int halvings = 0;
    double dE = 0.0;
    for (halvings = 0; halvings <= 30; ++halvings) {
      if (halvings > 0) {
        TRY(eval_trial(s, dv, r, alpha, trial));
        launch_energy_delta(s->n, P<double>(s->psi[trial]), P<double>(s->psi[s->pc]), n0,
                            P<double>(s->mass), dv, r, alpha, partial, dscal + S_DEP, st);
        TRY(readback(s));
      }
      dE = s->hscal[S_DEP] + s->hscal[S_DEK];
      if (std::isfinite(dE) && dE <= 1e-4 * alpha * gp) {
        accepted = true;
        break;
      }
      alpha *= 0.5;
    }
    vc_range.push_back({vc0, s->vcycles});
    if (!accepted) {
      s->log_int.insert(s->log_int.end(), {-1, 0, fb, 0});
      break;
    }
    backtracks += halvings;
    // -- accept: dv_t = dv + alpha p, s = dv_t - dv, y = g_t - g
    int slot = 0;
    for (int a = 0; a < W; ++a)
      if (std::find(hist.begin(), hist.end(), a) == hist.end()) {
        slot = a;
        break;
      }
    launch_step_update(N, dv, alpha, r, dvt, P<double>(s->Sh[slot]), st);
    std::swap(s->dv, s->dvt);
    dv = P<double>(s->dv);
    dvt = P<double>(s->dvt);
    s->pc = trial;
    TRY(gradient(s, dv, s->pc, gnew));
    // y.s, y.y, s.s and the CN norm land in S_YS, S_YY, S_SS, S_CN
    launch_secant_cn(N, gnew, g, P<double>(s->Yh[slot]), P<double>(s->Sh[slot]), n0,
                     P<double>(s->xi), cn_scale, partial, dscal + S_YS, st);
    TRY(readback(s));
    double ys = s->hscal[S_YS], yy = s->hscal[S_YY], ss = s->hscal[S_SS];
    bool keep = ys > 1e-12 * std::sqrt(yy * ss);
    if (keep && w > 0) {
      launch_rho(dscal + S_YS, P<double>(s->drho) + slot, st);
      hist.push_back(slot);
      if ((int)hist.size() > w) hist.erase(hist.begin());
    }
    if (!keep) ++skipped;
    std::swap(s->g, s->gnew);
    g = P<double>(s->g);
    gnew = P<double>(s->gnew);
    E += dE;
    cn = std::sqrt(s->hscal[S_CN]);
    if (!std::isfinite(cn)) return fail(HOT_E_NONFINITE, "non-finite gradient");
    s->log_cn.push_back(cn);
    s->log_int.insert(s->log_int.end(), {halvings, keep ? 0 : 1, fb, 0});
    ++it;
    conv = cn <= thresh;
  }
  // coarse-PCG iteration counts per L-BFGS iteration
  int nv = std::min(s->vcycles, s->prm.max_iters * 3 + 16);
  std::vector<int> pcg(nv > 0 ? nv : 1, 0);
  if (nv > 0) {
    HIPCHK(hipMemcpyAsync(pcg.data(), s->pcg_iters.p, nv * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  for (int v = 0; v < nv; ++v)
    if (pcg[v] < 0) return fail(HOT_E_DEVICE, "coarsest solve: grid barrier timed out");
  int cg_total = 0;
  for (size_t k = 0; k < vc_range.size() && 4 * k + 3 < s->log_int.size(); ++k) {
    int sum = 0;
    for (int v = vc_range[k].first; v < vc_range[k].second && v < nv; ++v) sum += pcg[v];
    s->log_int[4 * k + 3] = sum;
    cg_total += sum;
  }
  *converged = conv;
  {
    long long all = 0;
    for (int v = 0; v < nv; ++v) all += pcg[v];
    s->cg_per_cycle = nv > 0 ? (double)all / nv : 1.0;
  }
  if (stats) {
    stats->E = E;
    stats->cn = cn;
    stats->iters = it;
    stats->backtracks = backtracks;
    stats->cg_iters_total = cg_total;
    stats->converged = conv ? 1 : 0;
    stats->fallbacks = fallbacks;
    stats->skipped_pairs = skipped;
  }
  return HOT_OK;
}

// Projected Newton with inexact preconditioned CG (Alg. 1): PN-PCG with the
// scalar diagonal as preconditioner, PN-MGPCG with one V-cycle of the
// Galerkin hierarchy rebuilt from each Newton iteration's Hessian (Sec. 5.1).
// Each iteration solves H(dv) p = -g by CG from 0 to the relative tolerance
// k = min(1/2, sqrt(max(sqrt(r0^T M r0), eps))) in the preconditioner's
// energy norm (Sec. 5.3, tau read as the CN tolerance eps; at most 10,000 CG
// iterations), then runs HOT's backtracking line search.  Logged per
// iteration: step-length halvings and CG iterations.
constexpr int kPnCgMax = 10000;

hot_status solve_pn(hot_scene* s, hot_step_stats* stats, bool* converged) {
  hipStream_t st = s->stream;
  const int n0 = s->L[0].n;
  const long long N = (long long)n0 * 3;
  const double dt = s->dt_prepared;
  const double cn_scale = 24.0 * s->prm.dx * s->prm.dx * dt;
  const double thresh = s->prm.tol * std::sqrt((double)n0);
  const bool mg = s->prm.solver == HOT_SOLVER_PN_MGPCG;
  double* dscal = P<double>(s->dscal);
  double* partial = P<double>(s->partial);
  double* dv = P<double>(s->dv);
  double* g = P<double>(s->g);
  // CG vectors: direction x, residual r, preconditioned residual z, search
  // direction p, product q
  double* x = P<double>(s->r);
  double* r = P<double>(s->q);
  double* z = P<double>(s->vin);
  double* p = P<double>(s->vout);
  double* q = P<double>(s->gnew);
  LevelView L0 = view(s, 0);
  const double* d0 = P<double>(s->L[0].diag);
  s->log_int.clear();
  s->log_cn.clear();
  launch_fill_double(N, dv, 0.0, st);
  s->pc = 0;
  TRY(eval_trial(s, dv, nullptr, 0.0, s->pc));
  launch_sum(s->n, P<double>(s->psi[s->pc]), partial, dscal + S_E0, st);
  TRY(gradient(s, dv, s->pc, g));
  launch_cn_sq(n0, g, P<double>(s->xi), cn_scale, partial, dscal + S_CN, st);
  TRY(readback(s));
  double E = s->hscal[S_E0];
  double cn = std::sqrt(s->hscal[S_CN]);
  if (!std::isfinite(E) || !std::isfinite(cn))
    return fail(HOT_E_NONFINITE, "non-finite energy or gradient at dv = 0");
  if (stats) {
    stats->E0 = E;
    stats->cn0 = cn;
    stats->cn_tol = thresh;
  }
  s->log_cn.push_back(cn);
  auto precondition = [&](const double* rr, double* zz) -> hot_status {
    if (mg) return vcycle(s, rr, zz);
    launch_diag_solve(N, d0, rr, zz, st);
    return HOT_OK;
  };
  auto dot = [&](const double* a, const double* b, double* out) -> hot_status {
    launch_dot(N, a, b, partial, dscal + S_GP, st);
    TRY(readback(s));
    *out = s->hscal[S_GP];
    return HOT_OK;
  };
  int it = 0, backtracks = 0, cg_total = 0;
  bool conv = cn <= thresh;
  while (!conv && it < s->prm.max_iters) {
    if (it > 0) {
      TRY(build_hessian(s, dv));
      L0 = view(s, 0);
    }
    // CG from 0 for H p = -g (g is zero on constrained DOFs)
    launch_fill_double(N, x, 0.0, st);
    launch_scale_copy(N, -1.0, g, r, st);
    TRY(precondition(r, z));
    double rz = 0.0;
    TRY(dot(r, z, &rz));
    const double k = std::min(0.5, std::sqrt(std::max(std::sqrt(std::max(rz, 0.0)), s->prm.tol)));
    const double stop = k * std::sqrt(std::max(rz, 0.0));
    int cgi = 0;
    if (rz > 0.0) {
      launch_scale_copy(N, 1.0, z, p, st);
      while (cgi < kPnCgMax) {
        launch_spmv(L0, p, q, st);
        double pq = 0.0;
        TRY(dot(p, q, &pq));
        const double alpha = rz / pq;
        launch_axpy(N, alpha, p, x, st);
        launch_axpy(N, -alpha, q, r, st);
        TRY(precondition(r, z));
        double rzn = 0.0;
        TRY(dot(r, z, &rzn));
        ++cgi;
        if (std::sqrt(std::max(rzn, 0.0)) <= stop) break;
        const double beta = rzn / rz;
        rz = rzn;
        launch_xpby(N, z, beta, p, st);
      }
    }
    cg_total += cgi;
    // line search along x, as in HOT
    double gp = 0.0;
    TRY(dot(g, x, &gp));
    int trial = 1 - s->pc;
    double alpha = 1.0;
    bool accepted = false;
    int halvings = 0;
    double dE = 0.0;
    for (halvings = 0; halvings <= 30; ++halvings) {
      TRY(eval_trial(s, dv, x, alpha, trial));
      launch_energy_delta(s->n, P<double>(s->psi[trial]), P<double>(s->psi[s->pc]), n0,
                          P<double>(s->mass), dv, x, alpha, partial, dscal + S_DEP, st);
      TRY(readback(s));
      dE = s->hscal[S_DEP] + s->hscal[S_DEK];
      if (std::isfinite(dE) && dE <= 1e-4 * alpha * gp) {
        accepted = true;
        break;
      }
      alpha *= 0.5;
    }
    if (!accepted) {
      s->log_int.insert(s->log_int.end(), {-1, 0, 0, cgi});
      break;
    }
    backtracks += halvings;
    launch_axpy(N, alpha, x, dv, st);
    s->pc = trial;
    TRY(gradient(s, dv, s->pc, g));
    launch_cn_sq(n0, g, P<double>(s->xi), cn_scale, partial, dscal + S_CN, st);
    TRY(readback(s));
    E += dE;
    cn = std::sqrt(s->hscal[S_CN]);
    if (!std::isfinite(cn)) return fail(HOT_E_NONFINITE, "non-finite gradient");
    s->log_cn.push_back(cn);
    s->log_int.insert(s->log_int.end(), {halvings, 0, 0, cgi});
    ++it;
    conv = cn <= thresh;
  }
  if (mg) {  // the V-cycles' coarsest solves all completed
    const int nv = std::min(s->vcycles, pcg_log_cap(s) + 1);
    std::vector<int> pcg(std::max(nv, 1), 0);
    if (nv > 0) {
      HIPCHK(hipMemcpyAsync(pcg.data(), s->pcg_iters.p, nv * 4, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
    }
    for (int v = 0; v < nv; ++v)
      if (pcg[v] < 0) return fail(HOT_E_DEVICE, "coarsest solve: grid barrier timed out");
  }
  *converged = conv;
  if (stats) {
    stats->E = E;
    stats->cn = cn;
    stats->iters = it;
    stats->backtracks = backtracks;
    stats->cg_iters_total = cg_total;
    stats->converged = conv ? 1 : 0;
  }
  return HOT_OK;
}

hot_status choose_dt(hot_scene* s, double dt_in, double* dt_out) {
  if (dt_in > 0.0) {
    *dt_out = dt_in;
    return HOT_OK;
  }
  launch_max_speed(s->n, s->P[s->cur].v, P<double>(s->partial), P<double>(s->dscal) + S_VMAX,
                   s->stream);
  TRY(readback(s));
  double vmax = std::max(s->hscal[S_VMAX], s->bc_speed);
  if (!std::isfinite(vmax)) return fail(HOT_E_NONFINITE, "non-finite particle velocity");
  *dt_out = vmax > 0.0 ? std::min(s->prm.max_dt, s->prm.cfl * s->prm.dx / vmax) : s->prm.max_dt;
  return HOT_OK;
}

hot_status do_step(hot_scene* s, double dt_in, hot_step_stats* stats) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  hipStream_t st = s->stream;
  HIPCHK(hipEventRecord(s->ev[0], st));
  double dt;
  TRY(choose_dt(s, dt_in, &dt));
  TRY(prepare(s, dt));
  HIPCHK(hipEventRecord(s->ev[2], st));
  bool conv = false;
  if (s->prm.solver == HOT_SOLVER_HOT) {
    TRY(solve(s, stats, &conv));
  } else if (s->prm.solver == HOT_SOLVER_PN_MGPCG) {
    GridTicket ticket(s);
    TRY(solve_pn(s, stats, &conv));
  } else {
    TRY(solve_pn(s, stats, &conv));
  }
  HIPCHK(hipEventRecord(s->ev[3], st));
  Particles& pt = s->P[s->cur];
  launch_g2p(s->sd, view(s, 0), s->n, P<double>(s->f), P<int>(s->key), pt.x, pt.v, pt.C, pt.F,
             pt.mat, P<double>(s->vstar), P<double>(s->dv), dt, P<double>(s->wnode), st);
  HIPCHK(hipEventRecord(s->ev[4], st));
  HIPCHK(hipEventSynchronize(s->ev[4]));
  HIPCHK(hipGetLastError());
  TRY(prof_flush(s));
  s->t += dt;
  s->prepared = false;
  if (stats) {
    stats->dt = dt;
    stats->t = s->t;
    stats->n_nodes = s->L[0].n;
    stats->n_levels = s->levels;
    // phase times are informational: a failed query reports 0
    float* ph[4] = {&stats->ms_prepare, &stats->ms_hierarchy, &stats->ms_solve, &stats->ms_g2p};
    for (int k = 0; k < 4; ++k)
      if (hipEventElapsedTime(ph[k], s->ev[k], s->ev[k + 1]) != hipSuccess) *ph[k] = 0.0f;
  }
  return conv ? HOT_OK : HOT_W_NOT_CONVERGED;
}

void destroy(hot_scene* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  drop_vcycle_graph(s);
  DBuf* all[] = {&s->pbuf[0], &s->pbuf[1], &s->f, &s->key, &s->keys, &s->tmp, &s->arec,
                 &s->psi[0], &s->psi[1], &s->S[0], &s->S[1], &s->counts, &s->start,
                 &s->cursor, &s->flags, &s->scan, &s->scan_temp, &s->err, &s->mass,
                 &s->vstar, &s->xi, &s->fixed, &s->dv, &s->dvt, &s->g, &s->gnew, &s->q, &s->r,
                 &s->pcg_work, &s->pcg_iters, &s->vin, &s->vout, &s->dalpha,
                 &s->drho, &s->dscal, &s->partial, &s->tables, &s->seg_begin,
                 &s->bmap, &s->blist, &s->bpartial, &s->wnode, &s->tnodes, &s->tmap,
                 &s->tpat, &s->tH, &s->cscratch};
  for (DBuf* b : all) release(s, *b);
  for (auto& b : s->Sh) release(s, b);
  for (auto& b : s->Yh) release(s, b);
  for (int m = 0; m < kMaxLevels; ++m) {
    LevelH& L = s->L[m];
    DBuf* lb[] = {&L.nodes, &L.map, &L.H, &L.Hb, &L.Dinv, &L.Dinv32, &L.diag, &L.diag32,
                  &L.freed, &L.pat, &L.b, &L.u, &L.r, &L.t, &L.crow, &L.coffd, &L.Dg, &L.Dg32};
    for (DBuf* b : lb) release(s, *b);
  }
  if (s->hscal) (void)hipHostFree(s->hscal);
  if (s->herr) (void)hipHostFree(s->herr);
  for (int k = 0; k < 5; ++k)
    if (s->ev[k]) (void)hipEventDestroy(s->ev[k]);
  for (hipEvent_t e : s->prof_ev) (void)hipEventDestroy(e);
  if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // namespace

extern "C" {

const char* hot_last_error(void) { return g_err.c_str(); }

hot_status hot_scene_footprint(const hot_params* params, int64_t n, const double* x,
                               size_t* bytes_out) {
  TRY(validate_params(params));
  if (n <= 0 || !x || !bytes_out) return fail(HOT_E_INVALID, "bad arguments");
  *bytes_out = estimate_bytes(params, n, count_sets(params, n, x));
  return HOT_OK;
}

hot_status hot_init_scene(const hot_params* params, int64_t n, const double* x, const double* v,
                          const double* F, const double* C, const double* vol0,
                          const int32_t* mat_id, const hot_material* mats, int32_t n_mats,
                          const hot_bc* bcs, int32_t n_bcs, const hot_allocator* alloc,
                          void* hip_stream, hot_scene** out) {
  if (!out) return fail(HOT_E_INVALID, "out is NULL");
  *out = nullptr;
  TRY(validate_params(params));
  if (n <= 0 || n > (1LL << 30)) return fail(HOT_E_INVALID, "n must be in [1, 2^30]");
  if (!x || !v || !vol0 || !mat_id || !mats) return fail(HOT_E_INVALID, "NULL particle array");
  if (n_mats < 1 || n_mats > kMaxMats) return fail(HOT_E_INVALID, "n_mats must be in [1, %d]", kMaxMats);
  if (n_bcs < 0 || n_bcs > kMaxBcs || (n_bcs > 0 && !bcs))
    return fail(HOT_E_INVALID, "n_bcs must be in [0, %d]", kMaxBcs);
  for (int k = 0; k < n_mats; ++k) {
    const hot_material& m = mats[k];
    if (m.model != HOT_FCR && m.model != HOT_NEOHOOKEAN) return fail(HOT_E_INVALID, "bad model");
    if (!(m.E > 0.0) || !std::isfinite(m.E)) return fail(HOT_E_INVALID, "E must be > 0");
    if (!(m.nu > -1.0 && m.nu < 0.5)) return fail(HOT_E_INVALID, "nu must be in (-1, 0.5)");
    if (!(m.density > 0.0) || !std::isfinite(m.density)) return fail(HOT_E_INVALID, "density must be > 0");
    if (!(m.yield_stress >= 0.0)) return fail(HOT_E_INVALID, "yield_stress must be >= 0");
    const double lo = m.snow_clamp[0], hi = m.snow_clamp[1];
    if (!(lo == 0.0 && hi == 0.0)) {
      if (!(lo > 0.0 && lo <= 1.0 && hi >= 1.0 && std::isfinite(hi)))
        return fail(HOT_E_INVALID, "snow_clamp must satisfy 0 < lo <= 1 <= hi");
      if (m.yield_stress > 0.0)
        return fail(HOT_E_INVALID, "snow_clamp and yield_stress are exclusive");
    }
  }
  for (int k = 0; k < n_bcs; ++k) {
    if (bcs[k].kind < 0 || bcs[k].kind > 2) return fail(HOT_E_INVALID, "bad bc kind");
    for (int j = 0; j < 16; ++j)
      if (!std::isfinite(bcs[k].p[j])) return fail(HOT_E_INVALID, "non-finite bc parameter");
    if (bcs[k].kind == HOT_BC_GRIP) {
      const double* p = bcs[k].p;
      if (p[9] * p[9] + p[10] * p[10] + p[11] * p[11] == 0.0)
        return fail(HOT_E_INVALID, "grip axis is zero");
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    if (mat_id[i] < 0 || mat_id[i] >= n_mats) return fail(HOT_E_INVALID, "mat_id out of range");
    if (!(vol0[i] > 0.0) || !std::isfinite(vol0[i])) return fail(HOT_E_INVALID, "vol0 must be > 0");
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(v[3 * i + a])) return fail(HOT_E_INVALID, "non-finite velocity");
    for (int a = 0; a < 9; ++a) {
      if (F && !std::isfinite(F[9 * i + a])) return fail(HOT_E_INVALID, "non-finite F");
      if (C && !std::isfinite(C[9 * i + a])) return fail(HOT_E_INVALID, "non-finite C");
    }
    if (F) {
      const double* f = F + 9 * i;
      double J = f[0] * (f[4] * f[8] - f[5] * f[7]) - f[1] * (f[3] * f[8] - f[5] * f[6]) +
                 f[2] * (f[3] * f[7] - f[4] * f[6]);
      if (mats[mat_id[i]].model == HOT_NEOHOOKEAN && !(J > 0.0))
        return fail(HOT_E_INVALID, "Neo-Hookean particle with det F <= 0");
    }
  }
  TRY(validate_positions(params, n, x));

  hot_scene* s = new hot_scene();
  s->prm = *params;
  s->est_bytes = estimate_bytes(params, n, count_sets(params, n, x));
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(HOT_E_DEVICE, "no current HIP device");
  }
  for (int k = 0; k < 5; ++k) s->ev[k] = nullptr;
  if (alloc && alloc->alloc && alloc->free) {
    s->alloc = *alloc;
  } else {
    s->alloc.alloc = default_alloc;
    s->alloc.free = default_free;
    s->alloc.ctx = nullptr;
  }
  hot_status rc = HOT_OK;
  auto bail = [&](hot_status st) {
    destroy(s);
    return st;
  };
  if (hip_stream) {
    s->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(HOT_E_DEVICE, "stream creation failed"));
    s->own_stream = true;
  }
  for (int k = 0; k < 5; ++k)
    if (hipEventCreate(&s->ev[k]) != hipSuccess) return bail(fail(HOT_E_DEVICE, "event creation failed"));
  if (hipHostMalloc((void**)&s->hscal, NSCAL * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void**)&s->herr, sizeof(int)) != hipSuccess)
    return bail(fail(HOT_E_DEVICE, "pinned host allocation failed"));
  s->n = (int)n;
  s->mixed = params->precision == HOT_MIXED;
  // PN-PCG's diagonal preconditioner needs no coarse levels
  s->levels = params->solver == HOT_SOLVER_PN_PCG ? 1 : params->mg_levels;
  s->mats.assign(mats, mats + n_mats);
  s->bcs.assign(bcs, bcs + n_bcs);
  s->bc_speed = bc_max_speed(s->bcs);
  // device constants
  SceneDev& sd = s->sd;
  std::memset(&sd, 0, sizeof(sd));
  sd.dx = params->dx;
  sd.inv_dx = 1.0 / params->dx;
  for (int a = 0; a < 3; ++a) {
    sd.origin[a] = params->origin[a];
    sd.gravity[a] = params->gravity[a];
    sd.cells[a] = params->grid_cells[a];
  }
  sd.g0 = make_geom(params->grid_cells[0] + 1, params->grid_cells[1] + 1, params->grid_cells[2] + 1);
  sd.n_mats = n_mats;
  std::vector<MaterialDev> hm(n_mats);
  for (int k = 0; k < n_mats; ++k) {
    MaterialDev& m = hm[k];
    m.model = mats[k].model;
    m.mu = lame_mu(mats[k].E, mats[k].nu);
    m.lam = lame_lam(mats[k].E, mats[k].nu);
    m.density = mats[k].density;
    m.yield = mats[k].yield_stress;
    m.clamp_lo = mats[k].snow_clamp[0];
    m.clamp_hi = mats[k].snow_clamp[1];
    m.xi = std::sqrt(3.0 * (2.0 * m.mu + m.lam) * (2.0 * m.mu + m.lam) + 6.0 * m.lam * m.lam);
  }
  sd.n_bcs = n_bcs;
  std::vector<BcDev> hb(std::max(n_bcs, 1));
  for (int k = 0; k < n_bcs; ++k) {
    hb[k].kind = bcs[k].kind;
    for (int j = 0; j < 16; ++j) hb[k].p[j] = bcs[k].p[j];
  }
  {
    size_t mb = sizeof(MaterialDev) * n_mats, bb = sizeof(BcDev) * hb.size();
    if ((rc = ensure(s, s->tables, mb + bb)) < 0) return bail(rc);
    // stream-ordered: scenes of one process may be created from several threads
    hipError_t e = hipMemcpyAsync(s->tables.p, hm.data(), mb, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync((char*)s->tables.p + mb, hb.data(), bb, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess)
      return bail(fail(HOT_E_DEVICE, "table upload failed: %s", hipGetErrorString(e)));
    sd.mats = (const MaterialDev*)s->tables.p;
    sd.bcs = (const BcDev*)((char*)s->tables.p + mb);
  }
  // level geometry
  s->L[0].g = sd.g0;
  for (int m = 1; m < s->levels; ++m) {
    const GridGeom& f = s->L[m - 1].g;
    s->L[m].g = make_geom(f.dims[0] / 2 + 1, f.dims[1] / 2 + 1, f.dims[2] / 2 + 1);
  }
  // particle buffers: one allocation per set
  size_t per = (size_t)n * (3 + 3 + 9 + 9 + 1) * 8 + (size_t)n * 2 * 4;
  for (int k = 0; k < 2; ++k) {
    if ((rc = ensure(s, s->pbuf[k], per)) < 0) return bail(rc);
    char* b = (char*)s->pbuf[k].p;
    Particles& Pp = s->P[k];
    Pp.x = (double*)b;
    Pp.v = Pp.x + 3 * n;
    Pp.C = Pp.v + 3 * n;
    Pp.F = Pp.C + 9 * n;
    Pp.vol = Pp.F + 9 * n;
    Pp.mat = (int*)(Pp.vol + n);
    Pp.id = Pp.mat + n;
  }
  DBuf* pb[] = {&s->f, &s->arec, &s->psi[0], &s->psi[1], &s->S[0], &s->S[1]};
  size_t pbs[] = {(size_t)n * 24, (size_t)n * kAsmRec * 8, (size_t)n * 8, (size_t)n * 8,
                  (size_t)n * 72, (size_t)n * 72};
  for (int k = 0; k < 6; ++k)
    if ((rc = ensure(s, *pb[k], pbs[k])) < 0) return bail(rc);
  DBuf* ib[] = {&s->key, &s->keys, &s->tmp};
  for (DBuf* b : ib)
    if ((rc = ensure(s, *b, (size_t)n * 4)) < 0) return bail(rc);
  long long pt = sd.g0.ptotal;
  if ((rc = ensure(s, s->wnode, pt * 32)) < 0) return bail(rc);
  if ((rc = ensure(s, s->counts, pt * 4)) < 0 || (rc = ensure(s, s->start, (pt + 1) * 4)) < 0 ||
      (rc = ensure(s, s->cursor, pt * 4)) < 0 || (rc = ensure(s, s->flags, pt * 4)) < 0 ||
      (rc = ensure(s, s->scan, (pt + 1) * 4)) < 0 ||
      (rc = ensure(s, s->scan_temp, scan_temp_bytes(pt))) < 0 || (rc = ensure(s, s->err, 64)) < 0)
    return bail(rc);
  for (int m = 0; m < s->levels; ++m)
    if ((rc = ensure(s, s->L[m].map, s->L[m].g.ptotal * 4)) < 0) return bail(rc);
  {
    BrickGeom& bg = s->bricks.bg;
    for (int a = 0; a < 3; ++a) bg.bd[a] = (sd.g0.pd[a] + kBrick - 1) / kBrick;
    bg.total = (long long)bg.bd[0] * bg.bd[1] * bg.bd[2];
    if ((rc = ensure(s, s->bmap, bg.total * 4)) < 0) return bail(rc);
  }
  int W = params->lbfgs_history + 1;
  if ((rc = ensure(s, s->dalpha, W * 8)) < 0 || (rc = ensure(s, s->drho, W * 8)) < 0 ||
      (rc = ensure(s, s->dscal, NSCAL * 8)) < 0 || (rc = ensure(s, s->partial, kRedBlocks * 4 * 8)) < 0)
    return bail(rc);
  // upload (host staging in caller order; ids = caller indices)
  std::vector<char> host(per);
  double* hx = (double*)host.data();
  std::memcpy(hx, x, n * 24);
  std::memcpy(hx + 3 * n, v, n * 24);
  double* hC = hx + 6 * n;
  double* hF = hC + 9 * n;
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 9; ++a) {
      hC[9 * i + a] = C ? C[9 * i + a] : 0.0;
      hF[9 * i + a] = F ? F[9 * i + a] : ((a % 4 == 0) ? 1.0 : 0.0);
    }
  double* hvol = hF + 9 * n;
  std::memcpy(hvol, vol0, n * 8);
  int* hmat = (int*)(hvol + n);
  std::memcpy(hmat, mat_id, n * 4);
  int* hid = hmat + n;
  for (int64_t i = 0; i < n; ++i) hid[i] = (int)i;
  if (hipMemcpyAsync(s->pbuf[0].p, host.data(), per, hipMemcpyHostToDevice, s->stream) != hipSuccess ||
      hipStreamSynchronize(s->stream) != hipSuccess)
    return bail(fail(HOT_E_DEVICE, "upload failed"));
  s->cur = 0;
  *out = s;
  return HOT_OK;
}

hot_status hot_step(hot_scene* scene, double dt, hot_step_stats* stats) {
  if (!scene) return fail(HOT_E_INVALID, "scene is NULL");
  if (!std::isfinite(dt)) return fail(HOT_E_INVALID, "dt must be finite");
  HIPCHK(hipSetDevice(scene->device));
  return do_step(scene, dt, stats);
}

hot_status hot_read_particles(const hot_scene* scene, int64_t n, double* x, double* v, double* F,
                              double* C) {
  if (!scene) return fail(HOT_E_INVALID, "scene is NULL");
  if (n != scene->n) return fail(HOT_E_INVALID, "n does not match the scene");
  hot_scene* s = const_cast<hot_scene*>(scene);
  size_t per = (size_t)n * (3 + 3 + 9 + 9 + 1) * 8 + (size_t)n * 2 * 4;
  std::vector<char> host(per);
  HIPCHK(hipMemcpyAsync(host.data(), s->pbuf[s->cur].p, per, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  const double* hx = (const double*)host.data();
  const double* hv = hx + 3 * n;
  const double* hC = hv + 3 * n;
  const double* hF = hC + 9 * n;
  const int* hid = (const int*)(hF + 10 * n);
  hid += n;  // skip mat
  for (int64_t i = 0; i < n; ++i) {
    int o = hid[i];
    if (x) std::memcpy(x + 3 * o, hx + 3 * i, 24);
    if (v) std::memcpy(v + 3 * o, hv + 3 * i, 24);
    if (C) std::memcpy(C + 9 * o, hC + 9 * i, 72);
    if (F) std::memcpy(F + 9 * o, hF + 9 * i, 72);
  }
  return HOT_OK;
}

hot_status hot_scene_info(const hot_scene* scene, int64_t* n, double* t) {
  if (!scene) return fail(HOT_E_INVALID, "scene is NULL");
  if (n) *n = scene->n;
  if (t) *t = scene->t;
  return HOT_OK;
}

hot_status hot_scene_memory(const hot_scene* scene, size_t* live_bytes, size_t* estimate_bytes) {
  if (!scene) return fail(HOT_E_INVALID, "scene is NULL");
  if (live_bytes) *live_bytes = scene->bytes_live;
  if (estimate_bytes) *estimate_bytes = scene->est_bytes;
  return HOT_OK;
}

void hot_destroy_scene(hot_scene* scene) { destroy(scene); }

// ---------------------------------------------------------------- stepping without allocation
}  // extern "C"

// Per-call scratch of hot_step_noalloc, one fixed array per device: the
// reduction partial sums, the scalar block, the error flag, the coarse-PCG
// iteration counts and the coarsest-level PCG vectors and grid barrier.
constexpr size_t kNoAllocScratchBytes = size_t(1) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of device `dev`'s copy of `scratch` (in host code the
// array's name is only a stand-in), looked up once per device with that
// device current.
hot_status scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(HOT_E_DEVICE, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(HOT_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = (unsigned char*)p;
  }
  *out = g_scratch_ptr[dev];
  return HOT_OK;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// For its lifetime, the scene's per-call buffers are ranges of the scratch
// array and no scene buffer may grow.
class BorrowScratch {
 public:
  BorrowScratch(hot_scene* s, unsigned char* base, size_t iters_bytes) : s_(s) {
    DBuf* bufs[kN] = {&s->dscal, &s->err, &s->partial, &s->pcg_iters, &s->pcg_work};
    const size_t part = round256((size_t)kRedBlocks * 4 * 8);
    const size_t off[kN] = {0, 256, 512, 512 + part, 512 + part + iters_bytes};
    const size_t cap[kN] = {256, 256, part, iters_bytes,
                            kNoAllocScratchBytes - (512 + part + iters_bytes)};
    for (int k = 0; k < kN; ++k) {
      bufs_[k] = bufs[k];
      saved_[k] = *bufs[k];
      bufs[k]->p = base + off[k];
      bufs[k]->cap = cap[k];
      bufs[k]->borrowed = true;
    }
    s->no_alloc = true;
  }
  ~BorrowScratch() {
    for (int k = 0; k < kN; ++k) *bufs_[k] = saved_[k];
    s_->no_alloc = false;
  }
  static size_t fixed_bytes() { return 512 + round256((size_t)kRedBlocks * 4 * 8); }

 private:
  static constexpr int kN = 5;
  hot_scene* s_;
  DBuf* bufs_[kN];
  DBuf saved_[kN];
};

}  // namespace

extern "C" {

hot_status hot_step_noalloc(hot_scene* scene, double dt, hot_step_stats* stats) {
  if (!scene) return fail(HOT_E_INVALID, "scene is NULL");
  if (!std::isfinite(dt)) return fail(HOT_E_INVALID, "dt must be finite");
  if (scene->prof)
    return fail(HOT_E_INVALID, "hot_step_noalloc: kernel tracing creates events; disable it");
  HIPCHK(hipSetDevice(scene->device));
  unsigned char* base = nullptr;
  TRY(scratch_address(scene->device, &base));
  // one coarse-PCG count per V-cycle (at most 3 per iteration)
  const size_t iters = round256(pcg_log_bytes(scene->prm.max_iters));
  if (BorrowScratch::fixed_bytes() + iters + 4096 > kNoAllocScratchBytes)
    return fail(HOT_E_INVALID,
                "hot_step_noalloc: max_iters = %d needs %zu bytes of counters; the scratch "
                "holds %zu bytes in all",
                scene->prm.max_iters, iters, kNoAllocScratchBytes);
  BorrowScratch borrow(scene, base, iters);
  return do_step(scene, dt, stats);
}

// ---------------------------------------------------------------- tracing
hot_status hot_profile_enable(hot_scene* scene, int32_t enable) {
  if (!scene) return fail(HOT_E_INVALID, "scene is NULL");
  scene->prof = enable != 0;
  scene->prof_used = 0;
  for (int k = 0; k < HOT_PROF_COUNT; ++k) {
    scene->prof_ms[k] = 0.0;
    scene->prof_n[k] = 0;
    scene->prof_bytes[k] = 0.0;
  }
  return HOT_OK;
}

hot_status hot_profile_read(const hot_scene* scene, int32_t kernel, double* total_ms,
                            int64_t* launches, double* total_bytes) {
  if (!scene) return fail(HOT_E_INVALID, "scene is NULL");
  if (kernel < 0 || kernel >= HOT_PROF_COUNT) return fail(HOT_E_INVALID, "bad kernel id");
  if (total_ms) *total_ms = scene->prof_ms[kernel];
  if (launches) *launches = scene->prof_n[kernel];
  if (total_bytes) *total_bytes = scene->prof_bytes[kernel];
  return HOT_OK;
}

// ---------------------------------------------------------------- debug
hot_status hot_debug_prepare(hot_scene* scene, double dt) {
  if (!scene) return fail(HOT_E_INVALID, "scene is NULL");
  double d;
  TRY(choose_dt(scene, dt, &d));
  TRY(prepare(scene, d));
  HIPCHK(hipStreamSynchronize(scene->stream));
  return HOT_OK;
}

hot_status hot_debug_set(int32_t key, int64_t value, int64_t* previous) {
  if (key != HOT_SET_MULTIROW_MIN) return fail(HOT_E_INVALID, "unknown setting %d", key);
  if (value > INT32_MAX) return fail(HOT_E_INVALID, "value out of range");
  int old = set_sweep_run_min(value < 0 ? -1 : (int)value);
  if (previous) *previous = old;
  return HOT_OK;
}

hot_status hot_debug_apply(hot_scene* scene, int32_t op, const double* in, double* out) {
  if (!scene || !in || !out) return fail(HOT_E_INVALID, "NULL argument");
  hot_scene* s = scene;
  if (!s->prepared) return fail(HOT_E_INVALID, "call hot_debug_prepare first");
  long long N = (long long)s->L[0].n * 3;
  hipStream_t st = s->stream;
  HIPCHK(hipMemcpyAsync(s->vin.p, in, N * 8, hipMemcpyHostToDevice, st));
  double* vin = P<double>(s->vin);
  double* vout = P<double>(s->vout);
  if (op == 0) {
    GridTicket ticket(s);
    TRY(vcycle(s, vin, vout));
  } else if (op == 1) {
    TRY(eval_trial(s, vin, nullptr, 0.0, 0));
    TRY(gradient(s, vin, 0, vout));
  } else if (op == 2) {
    TRY(eval_trial(s, vin, nullptr, 0.0, 0));
    launch_sum(s->n, P<double>(s->psi[0]), P<double>(s->partial), P<double>(s->dscal) + S_E0, st);
    launch_kinetic_delta(s->L[0].n, P<double>(s->mass), vin, vin, -1.0, P<double>(s->partial),
                         P<double>(s->dscal) + S_DEK, st);
    TRY(readback(s));
    // kinetic delta with alpha = -1 is sum 1/2 m (0 - |dv|^2)
    out[0] = s->hscal[S_E0] - s->hscal[S_DEK];
    return HOT_OK;
  } else if (op == 3) {
    launch_spmv(view(s, 0), vin, vout, st);
  } else {
    return fail(HOT_E_INVALID, "unknown op");
  }
  HIPCHK(hipMemcpyAsync(out, vout, N * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return HOT_OK;
}

hot_status hot_debug_read(const hot_scene* scene, int32_t what, int32_t level, void* dst,
                          size_t bytes, size_t* needed) {
  if (!scene) return fail(HOT_E_INVALID, "scene is NULL");
  hot_scene* s = const_cast<hot_scene*>(scene);
  if (level < 0 || level >= s->levels) return fail(HOT_E_INVALID, "bad level");
  const LevelH& L = s->L[level];
  const void* src = nullptr;
  size_t sz = 0;
  bool host = false;
  std::vector<int> counts;
  switch (what) {
    case HOT_DBG_PERM: src = s->P[s->cur].id; sz = (size_t)s->n * 4; break;
    case HOT_DBG_LEVEL_NODES: src = L.nodes.p; sz = (size_t)L.n * 4; break;
    case HOT_DBG_LEVEL_PATTERN: src = L.pat.p; sz = (size_t)L.n * 16; break;
    case HOT_DBG_LEVEL_MATRIX: src = L.H.p; sz = (size_t)L.n * kRowVals * 8; break;  // reordered below
    case HOT_DBG_LEVEL_MATRIX_BF16:
      if (!s->mixed) return fail(HOT_E_INVALID, "BF16 blocks exist only under HOT_MIXED");
      src = L.Hb.p;
      sz = (size_t)L.n * kRowVals * 2;
      break;
    case HOT_DBG_LEVEL_FREE: src = L.freed.p; sz = (size_t)L.n * 3; break;
    case HOT_DBG_LEVEL_COLOR_ROWS:
      if (s->prm.smoother != HOT_SMOOTH_SGS || level + 1 >= s->levels)
        return fail(HOT_E_INVALID, "colour lists exist only for HOT_SMOOTH_SGS smoothed levels");
      src = L.crow.p;
      sz = (size_t)L.n * 4;
      break;
    case HOT_DBG_NODE_MASS: src = s->mass.p; sz = (size_t)s->L[0].n * 8; break;
    case HOT_DBG_NODE_VSTAR: src = s->vstar.p; sz = (size_t)s->L[0].n * 24; break;
    case HOT_DBG_NODE_XI: src = s->xi.p; sz = (size_t)s->L[0].n * 8; break;
    case HOT_DBG_NODE_FIXED: src = s->fixed.p; sz = (size_t)s->L[0].n * 4; break;
    case HOT_DBG_DV: src = s->dv.p; sz = (size_t)s->L[0].n * 24; break;
    case HOT_DBG_LOG_INT: src = s->log_int.data(); sz = s->log_int.size() * 4; host = true; break;
    case HOT_DBG_LOG_CN: src = s->log_cn.data(); sz = s->log_cn.size() * 8; host = true; break;
    case HOT_DBG_COUNTS: {
      counts.assign(16, 0);
      counts[0] = s->n;
      counts[1] = s->levels;
      for (int m = 0; m < s->levels && m < 8; ++m) counts[2 + m] = s->L[m].n;
      counts[10] = (int)(s->log_int.size() / 4);
      src = counts.data();
      sz = 64;
      host = true;
      break;
    }
    default: return fail(HOT_E_INVALID, "unknown debug array %d", what);
  }
  if (needed) *needed = sz;
  if (!dst) return HOT_OK;
  if (bytes < sz) return fail(HOT_E_INVALID, "buffer too small (%zu < %zu)", bytes, sz);
  if (sz == 0) return HOT_OK;
  if (host) {
    std::memcpy(dst, src, sz);
    return HOT_OK;
  }
  if (what == HOT_DBG_LEVEL_MATRIX) {
    // device rows are [entry][slot padded to 128]; hand out [slot][3][3]
    std::vector<double> tmpv((size_t)L.n * kRowStride);
    HIPCHK(hipMemcpyAsync(tmpv.data(), src, tmpv.size() * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    double* o = (double*)dst;
    for (int i = 0; i < L.n; ++i)
      for (int sl = 0; sl < kSlots; ++sl)
        for (int c = 0; c < 9; ++c)
          o[(size_t)i * kRowVals + sl * 9 + c] = tmpv[(size_t)i * kRowStride + c * kSlotPad + sl];
    return HOT_OK;
  }
  if (what == HOT_DBG_LEVEL_MATRIX_BF16) {
    std::vector<uint16_t> tmpv((size_t)L.n * kRowStride);
    HIPCHK(hipMemcpyAsync(tmpv.data(), src, tmpv.size() * 2, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    uint16_t* o = (uint16_t*)dst;
    for (int i = 0; i < L.n; ++i)
      for (int sl = 0; sl < kSlots; ++sl)
        for (int c = 0; c < 9; ++c)
          o[(size_t)i * kRowVals + sl * 9 + c] = tmpv[(size_t)i * kRowStride + c * kSlotPad + sl];
    return HOT_OK;
  }
  if (what == HOT_DBG_LEVEL_NODES) {
    // convert padded indices to plain linear indices of the level's node grid
    std::vector<int> tmpv(L.n);
    HIPCHK(hipMemcpyAsync(tmpv.data(), src, sz, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    int* o = (int*)dst;
    for (int i = 0; i < L.n; ++i) {
      int x, y, z;
      unpidx(L.g, tmpv[i], x, y, z);
      o[i] = x + L.g.dims[0] * (y + L.g.dims[1] * z);
    }
    return HOT_OK;
  }
  HIPCHK(hipMemcpyAsync(dst, src, sz, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  return HOT_OK;
}

// ---------------------------------------------------------------- serving
}  // extern "C"

// A batch is a fixed pool of slots, each served by one host thread.  An
// admitted scene runs all its steps on its own stream from its slot's thread,
// so the device interleaves the kernels of every resident scene; the batch
// only does admission (HBM budget, free slot) and completion bookkeeping.
namespace {

// Device memory pool of a batch.  Scenes that the batch creates (hot_batch_
// submit) take their buffers from it and return them when destroyed; a
// returned block is kept in its size class and handed out again, so scenes
// created and destroyed at the request rate do not call hipMalloc / hipFree
// (hipFree waits for the device) each time.  Size classes step by 1/8 of a
// power of two (at most 12.5% rounding).  The blocks go back to the device
// when the batch is destroyed and every block has been returned.
struct DevicePool {
  std::mutex mu;
  std::map<size_t, std::vector<void*>> free_blocks;
  std::unordered_map<void*, size_t> live;
  int device = 0;
  bool closing = false;

  static size_t size_class(size_t b) {
    if (b <= 4096) return 4096;
    int e = 63 - __builtin_clzll((unsigned long long)b);
    const size_t step = (size_t)1 << (e - 3);
    return (b + step - 1) / step * step;
  }
  // with mu held
  void release_all() {
    (void)hipSetDevice(device);
    for (auto& kv : free_blocks)
      for (void* p : kv.second) (void)hipFree(p);
    free_blocks.clear();
  }
};

void* pool_alloc(size_t bytes, void* ctx) {
  DevicePool* pool = (DevicePool*)ctx;
  const size_t c = DevicePool::size_class(bytes);
  {
    std::lock_guard<std::mutex> lk(pool->mu);
    auto it = pool->free_blocks.find(c);
    if (it != pool->free_blocks.end() && !it->second.empty()) {
      void* p = it->second.back();
      it->second.pop_back();
      pool->live[p] = c;
      return p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, c) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(pool->mu);
  pool->live[p] = c;
  return p;
}

void pool_free(void* p, void* ctx) {
  if (!p) return;
  DevicePool* pool = (DevicePool*)ctx;
  bool last = false;
  {
    std::lock_guard<std::mutex> lk(pool->mu);
    auto it = pool->live.find(p);
    if (it == pool->live.end()) return;
    pool->free_blocks[it->second].push_back(p);
    pool->live.erase(it);
    if (pool->closing && pool->live.empty()) {
      pool->release_all();
      last = true;
    }
  }
  if (last) delete pool;
}

}  // namespace

struct hot_batch {
  using clock = std::chrono::steady_clock;
  struct Job {
    hot_scene* scene = nullptr;
    bool create = false;    // submitted: the slot thread creates the scene
    hot_scene_desc desc;
    hot_params params;
    int steps = 0;
    int64_t tag = 0;
    size_t bytes = 0;
    double t_admit = 0.0;
  };
  DevicePool* pool = nullptr;
  int device = 0;
  size_t budget = 0;
  size_t used = 0;
  int resident = 0;
  bool stop = false;
  clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<Job> jobs;       // per slot; scene == nullptr when free
  // finished scenes keep their budget until the caller collects them: their
  // device memory is still live until then
  std::deque<std::pair<hot_batch_result, size_t>> done;
  std::vector<std::thread> workers;

  double now() const { return std::chrono::duration<double>(clock::now() - t0).count(); }

  void serve(int k) {
    for (;;) {
      Job job;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stop || jobs[k].scene != nullptr || jobs[k].create; });
        if (stop) return;
        job = jobs[k];
      }
      hot_batch_result r;
      std::memset(&r, 0, sizeof(r));
      r.tag = job.tag;
      r.t_admit = job.t_admit;
      if (job.create) {
        (void)hipSetDevice(device);
        const hot_scene_desc& d = job.desc;
        hot_allocator a{pool_alloc, pool_free, pool};
        hot_status rc = hot_init_scene(&job.params, d.n, d.x, d.v, d.F, d.C, d.vol0, d.mat_id,
                                       d.mats, d.n_mats, d.bcs, d.n_bcs, &a, nullptr, &job.scene);
        if (rc < 0) {
          r.status = rc;
          std::snprintf(r.message, sizeof(r.message), "%s", g_err.c_str());
          job.steps = 0;
        }
      }
      r.scene = job.scene;
      r.t_created = job.create ? now() : job.t_admit;
      for (int i = 0; i < job.steps; ++i) {
        hot_step_stats st;
        hot_status rc = hot_step(job.scene, 0.0, &st);
        double t = now();
        if (i < HOT_BATCH_MAX_STEPS) r.t_step_end[i] = t;
        if (rc < 0) {
          r.status = rc;
          std::snprintf(r.message, sizeof(r.message), "%s", g_err.c_str());
          break;
        }
        if (rc > r.status) r.status = rc;
        r.steps += 1;
        r.iters += st.iters;
        bool halt;
        {
          std::lock_guard<std::mutex> lk(mu);
          halt = stop;
        }
        if (halt) break;
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        done.emplace_back(r, job.bytes);
        resident -= 1;
        jobs[k] = Job();
      }
      cv_done.notify_all();
    }
  }
};

extern "C" {

hot_status hot_batch_create(size_t hbm_budget_bytes, int32_t max_slots, hot_batch** out) {
  // Slots beyond the 16 grid-solve tickets of the device wait for a ticket
  // before their coarsest solves.
  if (!out || max_slots < 1 || max_slots > 64 || hbm_budget_bytes == 0)
    return fail(HOT_E_INVALID, "bad arguments (max_slots must be in [1, 64])");
  hot_batch* b = new hot_batch();
  b->budget = hbm_budget_bytes;
  b->t0 = hot_batch::clock::now();
  b->jobs.resize(max_slots);
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return fail(HOT_E_DEVICE, "no current HIP device");
  }
  b->pool = new DevicePool();
  b->pool->device = b->device;
  try {
    for (int k = 0; k < max_slots; ++k) b->workers.emplace_back([b, k] { b->serve(k); });
  } catch (...) {
    hot_batch_destroy(b);
    return fail(HOT_E_NOMEM, "could not start slot threads");
  }
  *out = b;
  return HOT_OK;
}

hot_status hot_batch_capacity(hot_batch* b, size_t* free_bytes, int32_t* free_slots) {
  if (!b) return fail(HOT_E_INVALID, "batch is NULL");
  std::lock_guard<std::mutex> lk(b->mu);
  if (free_bytes) *free_bytes = b->budget - b->used;
  if (free_slots) *free_slots = (int32_t)b->jobs.size() - b->resident;
  return HOT_OK;
}

hot_status hot_batch_add(hot_batch* b, hot_scene* s, int32_t n_steps, int64_t tag) {
  if (!b || !s || n_steps < 1) return fail(HOT_E_INVALID, "bad arguments");
  // reserve the larger of what the scene holds and its working-size estimate
  size_t need = std::max(std::max(s->bytes_live, s->est_bytes), (size_t)1);
  {
    std::lock_guard<std::mutex> lk(b->mu);
    for (const hot_batch::Job& j : b->jobs)
      if (j.scene == s) return fail(HOT_E_BUSY, "scene is already resident");
    if (b->resident >= (int)b->jobs.size() || b->used + need > b->budget)
      return fail(HOT_E_NOMEM, "batch full: %zu + %zu > %zu bytes or no free slot", b->used,
                  need, b->budget);
    int k = 0;
    while (b->jobs[k].scene || b->jobs[k].create) ++k;
    hot_batch::Job& j = b->jobs[k];
    j.scene = s;
    j.create = false;
    j.steps = n_steps;
    j.tag = tag;
    j.bytes = need;
    j.t_admit = b->now();
    b->used += need;
    b->resident += 1;
  }
  b->cv_work.notify_all();
  return HOT_OK;
}

hot_status hot_batch_submit(hot_batch* b, const hot_scene_desc* d, int32_t n_steps, int64_t tag) {
  if (!b || !d || !d->params || !d->x || n_steps < 1) return fail(HOT_E_INVALID, "bad arguments");
  size_t need = 0;
  TRY(hot_scene_footprint(d->params, d->n, d->x, &need));
  need = std::max(need, (size_t)1);
  {
    std::lock_guard<std::mutex> lk(b->mu);
    if (b->resident >= (int)b->jobs.size() || b->used + need > b->budget)
      return fail(HOT_E_NOMEM, "batch full: %zu + %zu > %zu bytes or no free slot", b->used,
                  need, b->budget);
    int k = 0;
    while (b->jobs[k].scene || b->jobs[k].create) ++k;
    hot_batch::Job& j = b->jobs[k];
    j.scene = nullptr;
    j.create = true;
    j.desc = *d;
    j.params = *d->params;
    j.desc.params = &j.params;
    j.steps = n_steps;
    j.tag = tag;
    j.bytes = need;
    j.t_admit = b->now();
    b->used += need;
    b->resident += 1;
  }
  b->cv_work.notify_all();
  return HOT_OK;
}

hot_status hot_batch_poll(hot_batch* b, hot_batch_result* results, int32_t cap, int32_t* n_done,
                          int32_t* n_resident, int32_t wait_ms) {
  if (!b || !n_done || cap < 0 || (cap > 0 && !results)) return fail(HOT_E_INVALID, "bad arguments");
  std::unique_lock<std::mutex> lk(b->mu);
  if (b->done.empty() && b->resident > 0 && wait_ms > 0)
    b->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms),
                        [&] { return !b->done.empty() || b->resident == 0; });
  int k = 0;
  while (k < cap && !b->done.empty()) {
    results[k++] = b->done.front().first;
    b->used -= b->done.front().second;
    b->done.pop_front();
  }
  *n_done = k;
  if (n_resident) *n_resident = b->resident;
  return HOT_OK;
}

double hot_batch_clock(const hot_batch* b) { return b ? b->now() : 0.0; }

void hot_batch_destroy(hot_batch* b) {
  if (!b) return;
  {
    std::lock_guard<std::mutex> lk(b->mu);
    b->stop = true;
  }
  b->cv_work.notify_all();
  for (std::thread& t : b->workers)
    if (t.joinable()) t.join();
  if (b->pool) {
    DevicePool* pool = b->pool;
    bool gone = false;
    {
      std::lock_guard<std::mutex> lk(pool->mu);
      pool->closing = true;
      if (pool->live.empty()) {
        pool->release_all();
        gone = true;
      }
    }
    if (gone) delete pool;
  }
  delete b;
}

}  // extern "C"
