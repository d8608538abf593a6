// Host runtime behind the C ABI (include/cfd.h): table validation, arena and
// workspace layout, patch and tile work lists, the setup pipeline (ghost
// nodes -> metrics -> metric ghost copy), the per-step launch sequence and
// its hipGraph cache.  No device memory is allocated here: the caller's
// workspace holds everything.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <stdexcept>
#include <string>
#include <atomic>
#include <map>
#include <vector>

#include "../../include/cfd.h"
#include "cfd_internal.hpp"
#include "host_services.hpp"
#include "implicit.hpp"
#include "mg.hpp"

namespace cfd {
void launch_copy_nodes(const double* src, double* x, const BlockDesc& B, hipStream_t s);
void launch_ghost_nodes(double* x, const BlockDesc* blocks, const PatchDesc* patches, int npatch,
                        int maxcount, hipStream_t s);
void launch_metrics(const double* x, double* met, const BlockDesc& B, hipStream_t s);
void launch_visc_metrics(const double* met, double* vmet, const BlockDesc& B, hipStream_t s);
void launch_metric_ghosts(double* met, const BlockDesc* blocks, const PatchDesc* patches, int npatch,
                          int maxcount, hipStream_t s);
void launch_ghost_q(double* q, const double* met, const BlockDesc* blocks, const PatchDesc* patches,
                    int npatch, int nthreads, const StepParams& SP, hipStream_t s, int delta = 0);
bool stage_ring(const StageArgs& A, int mode, bool visc, bool fp32, const BlockDesc* blocks, const TileDesc* tiles,
                const Gas<double>& g64, const Gas<float>& g32, int nwg, hipStream_t s, int* occ);
bool stage_tiled(const StageArgs& A, int mode, bool visc, bool fp32, const BlockDesc* blocks,
                 const TileDesc* tiles, const Gas<double>& g64, const Gas<float>& g32, int nwg,
                 hipStream_t s, int* occ);
void launch_stage_simple(const StageArgs& A, int mode, bool visc, bool fp32, const BlockDesc* blocks,
                         const TileDesc* tiles, const Gas<double>& g64, const Gas<float>& g32, int nwg,
                         hipStream_t s);
void launch_dt(const double* q, const double* met, double* dtcell, double* partials, const BlockDesc* blocks,
               int nblk, int64_t nchunks, const StepParams& P, int nwg, hipStream_t s);
void launch_norms(const double* q, const double* r, const double* met, double* partials, const BlockDesc* blocks,
                  int nblk, int64_t nchunks, int nwg, hipStream_t s);
void mlp_forward(const MlpDims& D, const uint16_t* P, const float* x, const int32_t* idx, int64_t n, float* y,
                 float* cache, hipStream_t s);
int mlp_mse(const float* y, const float* t, const int32_t* idx, int64_t n, int d_out, float* dy, double* partials,
            int max_rows, double* loss, hipStream_t s);
void mlp_backward(const MlpDims& D, const uint16_t* P, const float* cache, const float* dy, int64_t n, float* grad,
                  float* dz, float* da, float* part, int nchunk, hipStream_t s);
void mlp_adam(int64_t np, float* master, float* m, float* v, const float* g, uint16_t* pbf, float lr, float b1,
              float b2, float eps, int t, hipStream_t s);
void mlp_to_bf16(int64_t np, const float* master, uint16_t* pbf, hipStream_t s);
void mlp_features(const CellMap& M, int64_t ncells, const double* cond, float* x, hipStream_t s);
void mlp_targets(const CellMap& M, int64_t ncells, const double* q, const double* cond, double gamma, float* t,
                 hipStream_t s);
void mlp_to_state(const CellMap& M, int64_t ncells, const float* y, const double* cond, double gamma, double* q,
                  hipStream_t s);
void launch_finalize(const double* partials, int nrows, int mode, double inv_ncells, double* dt,
                     double* hist, double* nonfinite, hipStream_t s);
}  // namespace cfd

using namespace cfd;

namespace {

constexpr int TILE_I = 64;
constexpr int NWG_MAX = 4096;   // persistent grid cap (rows of the partials buffers)

thread_local std::string g_last_error;

struct Err : std::exception {
  cfd_status st;
  std::string msg;
  Err(cfd_status s, std::string m) : st(s), msg(std::move(m)) {}
};

[[noreturn]] void fail(cfd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  throw Err(st, buf);
}

#define HIPCHK(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) fail(CFD_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct Layout {
  std::vector<int64_t> qoff, moff, soff, voff, sv, sk, sj, xoff, xsv, xsk, xsj;
  int64_t q_elems = 0, m_elems = 0, s_elems = 0, v_elems = 0, x_elems = 0;
};

// Aligned offset so that interior i = 0 (padded index g) sits on 128 bytes.
int64_t place(int64_t& cursor, int64_t nvar, int64_t sv) {
  int64_t off = round_up(cursor + NG, 16) - NG;
  cursor = off + nvar * sv;
  return off;
}

Layout make_layout(int nblk, const cfd_dims* dims) {
  Layout L;
  for (int b = 0; b < nblk; ++b) {
    const int64_t ni = dims[b].ni, nj = dims[b].nj, nk = dims[b].nk;
    const int64_t sj = round_up(ni + 2 * NG, 16);
    const int64_t sk = sj * (nj + 2 * NG);
    const int64_t sv = sk * (nk + 2 * NG);
    L.sj.push_back(sj);
    L.sk.push_back(sk);
    L.sv.push_back(sv);
    L.qoff.push_back(place(L.q_elems, NV, sv));
    L.moff.push_back(place(L.m_elems, NM, sv));
    L.soff.push_back(place(L.s_elems, 1, sv));
    L.voff.push_back(place(L.v_elems, NVM, sv));
    const int64_t xsj = ni + 1 + 2 * NG, xsk = xsj * (nj + 1 + 2 * NG), xsv = xsk * (nk + 1 + 2 * NG);
    L.xsj.push_back(xsj);
    L.xsk.push_back(xsk);
    L.xsv.push_back(xsv);
    L.xoff.push_back(L.x_elems);
    L.x_elems += 3 * xsv;
  }
  L.q_elems = round_up(L.q_elems + 16, 16);
  L.m_elems = round_up(L.m_elems + 16, 16);
  L.s_elems = round_up(L.s_elems + 16, 16);
  L.v_elems = round_up(L.v_elems + 16, 16);
  return L;
}

struct WsLayout {
  size_t met, vmet, qa, qb, scal, blocks, patches, tiles, part_dt, part_nrm, scalars, cell_start, total;
  size_t node_scratch;   // aliases qa.. during setup
  int64_t max_tiles;
  int npatch_total;
};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

int64_t max_tiles_for(int nblk, const cfd_dims* dims) {
  int64_t t = 0;
  for (int b = 0; b < nblk; ++b)
    t += (int64_t)((dims[b].ni + TILE_I - 1) / TILE_I) * dims[b].nj * dims[b].nk;
  return t;
}

WsLayout make_ws(const Layout& L, int nblk, const cfd_dims* dims, int npatch_total, bool local_dt, bool viscous) {
  WsLayout W{};
  size_t c = 0;
  W.met = c;
  c = align256(c + (size_t)L.m_elems * 8);
  W.vmet = c;   // viscous face metrics (viscous flow only)
  if (viscous) c = align256(c + (size_t)L.v_elems * 8);
  W.qa = c;
  c = align256(c + (size_t)L.q_elems * 8);
  W.qb = c;
  c = align256(c + (size_t)L.q_elems * 8);
  // node scratch aliases qa (and beyond if needed)
  W.node_scratch = W.qa;
  if (W.qa + (size_t)L.x_elems * 8 > c) c = align256(W.qa + (size_t)L.x_elems * 8);
  W.scal = c;
  if (local_dt) c = align256(c + (size_t)L.s_elems * 8);
  W.blocks = c;
  c = align256(c + sizeof(BlockDesc) * nblk);
  W.patches = c;
  c = align256(c + sizeof(PatchDesc) * (size_t)std::max(npatch_total, 1));
  W.max_tiles = max_tiles_for(nblk, dims);
  W.tiles = c;
  c = align256(c + sizeof(TileDesc) * (size_t)W.max_tiles);
  W.part_dt = c;
  c = align256(c + sizeof(double) * NPART * NWG_MAX);
  W.part_nrm = c;
  c = align256(c + sizeof(double) * NPART * NWG_MAX);
  W.scalars = c;   // dt, hist[12], nonfinite, norms_out[12]
  c = align256(c + sizeof(double) * 32);
  W.cell_start = c;   // interior-cell prefix sums per block (warm-start kernels)
  c = align256(c + sizeof(int64_t) * (nblk + 1));
  W.total = c;
  W.npatch_total = npatch_total;
  return W;
}

void check_params(const cfd_params* p) {
  if (!p) fail(CFD_EINVAL, "params is NULL");
  if (p->ghost_layers != NG) fail(CFD_EUNSUPPORTED, "ghost_layers must be %d", NG);
  if (!(p->gamma > 1.0)) fail(CFD_EINVAL, "gamma must exceed 1");
  if (!(p->cfl > 0.0)) fail(CFD_EINVAL, "cfl must be positive");
  if (p->viscous && !(p->reynolds > 0.0 && p->prandtl > 0.0))
    fail(CFD_EINVAL, "viscous flow needs positive reynolds and prandtl");
  if (!(p->mach >= 0.0)) fail(CFD_EINVAL, "mach must be non-negative");
}

void check_dims(int nblk, const cfd_dims* dims) {
  if (nblk <= 0 || !dims) fail(CFD_EINVAL, "need at least one block");
  for (int b = 0; b < nblk; ++b) {
    const cfd_dims& d = dims[b];
    if (d.ni < NG || d.nj < NG || d.nk < NG)
      fail(CFD_EINVAL, "block %d: every extent must be >= %d (got %d x %d x %d)", b, NG, d.ni, d.nj, d.nk);
    if ((int64_t)d.ni * d.nj * d.nk > (int64_t)1 << 34) fail(CFD_EINVAL, "block %d too large", b);
  }
}

void face_extent(const cfd_dims& d, int face, int& e1, int& e2) {
  const int n[3] = {d.ni, d.nj, d.nk};
  const int dir = face >> 1;
  const int t1 = dir == 0 ? 1 : 0, t2 = dir == 2 ? 1 : 2;
  e1 = n[t1];
  e2 = n[t2];
}

void validate_tables(int nblk, const cfd_dims* dims, int nconn, const cfd_conn* conns, int nbc,
                     const cfd_bc* bcs) {
  if (nconn < 0 || nbc < 0 || (nconn && !conns) || (nbc && !bcs)) fail(CFD_EINVAL, "bad table pointers");
  std::vector<std::vector<uint8_t>> cover(nblk * 6);
  for (int b = 0; b < nblk; ++b)
    for (int f = 0; f < 6; ++f) {
      int e1, e2;
      face_extent(dims[b], f, e1, e2);
      cover[b * 6 + f].assign((size_t)e1 * e2, 0);
    }
  auto mark = [&](int b, int f, const int32_t lo[2], const int32_t hi[2], const char* what, int idx) {
    int e1, e2;
    face_extent(dims[b], f, e1, e2);
    if (lo[0] < 0 || lo[1] < 0 || hi[0] > e1 || hi[1] > e2 || lo[0] >= hi[0] || lo[1] >= hi[1])
      fail(CFD_EINVAL, "%s %d: patch [%d,%d)x[%d,%d) outside face %d of block %d (%d x %d)", what, idx,
           lo[0], hi[0], lo[1], hi[1], f, b, e1, e2);
    auto& cv = cover[b * 6 + f];
    for (int q = lo[1]; q < hi[1]; ++q)
      for (int p = lo[0]; p < hi[0]; ++p) {
        if (cv[(size_t)q * e1 + p]) fail(CFD_EINVAL, "%s %d: face %d of block %d covered twice at (%d,%d)",
                                         what, idx, f, b, p, q);
        cv[(size_t)q * e1 + p] = 1;
      }
  };
  for (int c = 0; c < nconn; ++c) {
    const cfd_conn& C = conns[c];
    if (C.blk < 0 || C.blk >= nblk || C.nbr < 0 || C.nbr >= nblk) fail(CFD_EINVAL, "connection %d: bad block", c);
    if (C.face < 0 || C.face > 5) fail(CFD_EINVAL, "connection %d: bad face", c);
    if (C.nbr_face != (C.face ^ 1))
      fail(CFD_EINVAL, "connection %d: only opposite faces of one direction connect (identity orientation)", c);
    mark(C.blk, C.face, C.lo, C.hi, "connection", c);
    int e1, e2;
    face_extent(dims[C.nbr], C.nbr_face, e1, e2);
    if (C.nbr_lo[0] < 0 || C.nbr_lo[1] < 0 || C.nbr_lo[0] + (C.hi[0] - C.lo[0]) > e1 ||
        C.nbr_lo[1] + (C.hi[1] - C.lo[1]) > e2)
      fail(CFD_EINVAL, "connection %d: neighbour patch outside block %d face %d", c, C.nbr, C.nbr_face);
    for (int x = 0; x < 3; ++x)
      if (!std::isfinite(C.shift[x])) fail(CFD_EINVAL, "connection %d: non-finite shift", c);
  }
  for (int c = 0; c < nbc; ++c) {
    const cfd_bc& B = bcs[c];
    if (B.blk < 0 || B.blk >= nblk) fail(CFD_EINVAL, "boundary %d: bad block", c);
    if (B.face < 0 || B.face > 5) fail(CFD_EINVAL, "boundary %d: bad face", c);
    if (B.kind < CFD_BC_FARFIELD || B.kind > CFD_BC_EXTRAP) fail(CFD_EINVAL, "boundary %d: bad kind %d", c, B.kind);
    if (!std::isfinite(B.mach)) fail(CFD_EINVAL, "boundary %d: non-finite mach", c);
    mark(B.blk, B.face, B.lo, B.hi, "boundary", c);
  }
  for (int b = 0; b < nblk; ++b)
    for (int f = 0; f < 6; ++f)
      for (uint8_t v : cover[b * 6 + f])
        if (!v) fail(CFD_EINVAL, "face %d of block %d is not fully covered by connections/boundaries", f, b);
}

// Patch descriptors for sweep d (cells or nodes), with the transverse
// extension into ghost layers of directions swept earlier (extend), or over
// the face's own cells only.
void build_patches(int d, bool nodes, const cfd_params* params, const cfd_dims* dims, int nconn,
                   const cfd_conn* conns, int nbc, const cfd_bc* bcs, std::vector<PatchDesc>& out, int& maxcount,
                   bool extend = true) {
  auto make = [&](int blk, int face, int kind, int nbr, const int32_t lo[2], const int32_t hi[2],
                  const int32_t* nbr_lo, const double* shift, double mach) {
    PatchDesc P{};
    if (params) {   // freestream velocity of this patch (far field)
      const double m = mach > 0.0 ? mach : params->mach;
      const double speed = m * std::sqrt(params->gamma);
      P.uinf[0] = speed * std::cos(params->alpha) * std::cos(params->beta);
      P.uinf[1] = speed * std::sin(params->alpha) * std::cos(params->beta);
      P.uinf[2] = speed * std::sin(params->beta);
    }
    P.blk = blk;
    P.face = face;
    P.kind = kind;
    P.nbr = nbr;
    const int n[3] = {dims[blk].ni, dims[blk].nj, dims[blk].nk};
    const int ts[2] = {d == 0 ? 1 : 0, d == 2 ? 1 : 2};
    int count = 1;
    for (int a = 0; a < 2; ++a) {
      const int t = ts[a];
      int s = lo[a], e = hi[a];
      if (nodes && hi[a] == n[t]) e = n[t] + 1;
      if (extend && t < d) {
        if (lo[a] == 0) s = -NG;
        if (hi[a] == n[t]) e = nodes ? n[t] + 1 + NG : n[t] + NG;
      }
      P.lo[t] = s;
      P.hi[t] = e;
      P.noff[t] = nbr_lo ? nbr_lo[a] - lo[a] : 0;
      count *= (e - s);
    }
    P.count = count;
    for (int x = 0; x < 3; ++x) P.shift[x] = shift ? shift[x] : 0.0;
    maxcount = std::max(maxcount, count);
    out.push_back(P);
  };
  for (int c = 0; c < nbc; ++c)
    if ((bcs[c].face >> 1) == d)
      make(bcs[c].blk, bcs[c].face, bcs[c].kind, -1, bcs[c].lo, bcs[c].hi, nullptr, nullptr, bcs[c].mach);
  for (int c = 0; c < nconn; ++c)
    if ((conns[c].face >> 1) == d)
      make(conns[c].blk, conns[c].face, 0, conns[c].nbr, conns[c].lo, conns[c].hi, conns[c].nbr_lo, conns[c].shift,
           0.0);
}

}  // namespace

struct cfd_ctx {
  cfd_params params{};
  int nblk = 0;
  std::vector<cfd_dims> dims;
  Layout L;
  WsLayout W{};
  std::vector<BlockDesc> hblocks;
  char* ws = nullptr;
  BlockDesc* dblocks = nullptr;
  PatchDesc* dpatches = nullptr;
  // per sweep: [node sweeps 0..2][cell sweeps 0..2]
  int poff[6] = {0}, pcount[6] = {0}, pmax[6] = {0};
  int qthreads[3] = {0};   // threads of each state ghost sweep (k_ghost_q)
  // inviscid flow: every face's ghost layers over its own cells, all three
  // directions in one launch (no stencil of the inviscid stage reads an edge
  // or corner ghost cell, the only cells the sweep order exists for)
  int pm_off = 0, pm_count = 0, pm_threads = 0;
  TileDesc* dtiles = nullptr;
  int ntiles = 0;
  int64_t ncells = 0;
  int64_t nchunks = 0;   // 64-cell row chunks of the grid (time-step and norms kernels)
  cfd_tuning tun{2, 8, 32, 1, 1};   // replaced by default_tuning() when the blocks are created
  StepParams SP{};
  Gas<double> g64{};
  Gas<float> g32{};
  hipStream_t cap_stream = nullptr;
  // Captured time steps, for the state pointer graph_q: one step, and
  // STEPS_PER_GRAPH steps for runs without a history (one graph launch, and
  // its start-up gap, per STEPS_PER_GRAPH steps).
  static constexpr int STEPS_PER_GRAPH = 8;
  const void* graph_q = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph_n = nullptr;
  hipGraphExec_t gexec_n = nullptr;
  // A captured multigrid cycle led by this context (the finest level), valid
  // for the hierarchy and arguments in mg_key; id is unique per context and
  // gen counts its retunings, so a cycle over a level since retuned or
  // destroyed is captured again.
  uint64_t id = 0, gen = 0;
  std::vector<uint64_t> mg_key;
  hipGraph_t mg_graph = nullptr;
  hipGraphExec_t mg_gexec = nullptr;
  int num_cu = 256;
  std::map<int, int> occ_cache;
  std::string last_error;
  // kernel timing (eager steps only)
  struct EvPair {
    hipEvent_t a, b;
    int cls;
  };
  bool profiling = false;
  std::vector<EvPair> ev_used;
  std::vector<hipEvent_t> ev_pool;

  hipEvent_t take_event() {
    if (!ev_pool.empty()) {
      hipEvent_t e = ev_pool.back();
      ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) throw std::runtime_error(hipGetErrorString(r));
    return e;
  }
  void release_events() {
    for (auto& p : ev_used) {
      ev_pool.push_back(p.a);
      ev_pool.push_back(p.b);
    }
    ev_used.clear();
  }
  void destroy_events() {
    release_events();
    for (hipEvent_t e : ev_pool) hipEventDestroy(e);
    ev_pool.clear();
  }

  double* met() const { return reinterpret_cast<double*>(ws + W.met); }
  double* vmet() const { return reinterpret_cast<double*>(ws + W.vmet); }
  double* qa() const { return reinterpret_cast<double*>(ws + W.qa); }
  double* qb() const { return reinterpret_cast<double*>(ws + W.qb); }
  double* scal() const { return params.local_dt ? reinterpret_cast<double*>(ws + W.scal) : nullptr; }
  double* part_dt() const { return reinterpret_cast<double*>(ws + W.part_dt); }
  double* part_nrm() const { return reinterpret_cast<double*>(ws + W.part_nrm); }
  double* d_dt() const { return reinterpret_cast<double*>(ws + W.scalars); }
  double* d_hist() const { return d_dt() + 1; }
  double* d_nonfinite() const { return d_dt() + 13; }
  double* d_norms() const { return d_dt() + 16; }
  int64_t* d_cell_start() const { return reinterpret_cast<int64_t*>(ws + W.cell_start); }
  CellMap cell_map() const { return CellMap{dblocks, d_cell_start(), nblk}; }

  void drop_graph() {
    if (gexec) hipGraphExecDestroy(gexec);
    if (graph) hipGraphDestroy(graph);
    if (gexec_n) hipGraphExecDestroy(gexec_n);
    if (graph_n) hipGraphDestroy(graph_n);
    gexec = nullptr;
    graph = nullptr;
    graph_q = nullptr;
    gexec_n = nullptr;
    graph_n = nullptr;
    drop_mg_graph();
  }
  void drop_mg_graph() {
    if (mg_gexec) hipGraphExecDestroy(mg_gexec);
    if (mg_graph) hipGraphDestroy(mg_graph);
    mg_gexec = nullptr;
    mg_graph = nullptr;
    mg_key.clear();
  }
};

std::atomic<uint64_t> g_ctx_ids{1};

namespace {

void set_params(cfd_ctx* c) {
  const cfd_params& p = c->params;
  StepParams& S = c->SP;
  S.gamma = p.gamma;
  S.prandtl = p.prandtl;
  const double speed = p.mach * std::sqrt(p.gamma);
  S.mu_inf = p.viscous ? speed / p.reynolds : 0.0;
  S.s_star = p.sutherland;
  S.cfl = p.cfl;
  S.eps_h = p.entropy_fix;
  S.eps_lim = p.limiter_eps;
  S.uinf[0] = speed * std::cos(p.alpha) * std::cos(p.beta);
  S.uinf[1] = speed * std::sin(p.alpha) * std::cos(p.beta);
  S.uinf[2] = speed * std::sin(p.beta);
  S.viscous = p.viscous;
  S.flux_fp32 = p.flux_fp32;
  S.local_dt = p.local_dt;
  auto fill = [&](auto& G) {
    using T = std::remove_reference_t<decltype(G.gamma)>;
    G.gamma = (T)p.gamma;
    G.gm1 = (T)(p.gamma - 1.0);
    G.prandtl = (T)p.prandtl;
    G.mu_inf = (T)S.mu_inf;
    G.s_star = (T)p.sutherland;
    G.eps_h = (T)p.entropy_fix;
    G.eps_lim = (T)p.limiter_eps;
    G.gg = (T)(p.gamma / (p.gamma - 1.0));
    G.kfac = (T)(p.gamma / ((p.gamma - 1.0) * p.prandtl));
    for (int x = 0; x < 3; ++x) G.uinf[x] = (T)S.uinf[x];
  };
  fill(c->g64);
  fill(c->g32);
}

int64_t count_tiles(const std::vector<cfd_dims>& dims, int tj, int tk) {
  int64_t t = 0;
  for (const auto& d : dims)
    t += (int64_t)((d.ni + TILE_I - 1) / TILE_I) * ((d.nj + tj - 1) / tj) * ((d.nk + tk - 1) / tk);
  return t;
}

// Default tuning for the grid: the plane-ring kernel with 64 x 8 x 32 tiles
// (deep tiles amortise each tile's three plane fills; measured better than
// 64 x 8 x 16 even where nk = 144 leaves a half-empty last tile), tile_k
// halved (down to 4) while there are fewer tiles than CUs.  A grid that still
// leaves CUs idle gets the tiled kernel with 4-row tiles, tile_k halved (down
// to 1) until there are 4 tiles per CU: on such small grids the launch's
// latency, not the halo planes each shallow tile reloads, bounds the stage
// (measured on the 96x48x48 and 48x24x24 levels of a multigrid cycle: 64x4x1
// tiles took the cycle from 1.45 to 1.26 ms against 64x4x4 and 64x2x4).
// Grids of many small uneven blocks run faster with smaller tiles: the
// autotuner finds them.
// The FP32-flux Euler plane-ring kernels hold two workgroups per CU; tiles of
// half the depth fill both and shorten the tail of the persistent grid.
cfd_tuning default_tuning(const std::vector<cfd_dims>& dims, int num_cu, const cfd_params& p) {
  cfd_tuning t{2, 8, (p.flux_fp32 && !p.viscous) ? 16 : 32, 1, 1};
  while (t.tile_k > 4 && count_tiles(dims, t.tile_j, t.tile_k) < (int64_t)num_cu) t.tile_k /= 2;
  if (count_tiles(dims, t.tile_j, t.tile_k) < num_cu) {
    t.kernel = 0;
    t.tile_j = 4;
    while (t.tile_k > 1 && count_tiles(dims, t.tile_j, t.tile_k) < 4 * (int64_t)num_cu) t.tile_k /= 2;
  }
  return t;
}

void build_tiles(cfd_ctx* c, hipStream_t s) {
  const int tj = c->tun.tile_j, tk = c->tun.tile_k;
  struct T2 {
    TileDesc t;
    int64_t work;
  };
  std::vector<T2> v;
  for (int b = 0; b < c->nblk; ++b) {
    const cfd_dims& d = c->dims[b];
    for (int k0 = 0; k0 < d.nk; k0 += tk)
      for (int j0 = 0; j0 < d.nj; j0 += tj)
        for (int i0 = 0; i0 < d.ni; i0 += TILE_I) {
          const int64_t w = (int64_t)std::min(TILE_I, d.ni - i0) * std::min(tj, d.nj - j0) * std::min(tk, d.nk - k0);
          v.push_back({{b, i0, j0, k0}, w});
        }
  }
  if ((int64_t)v.size() > c->W.max_tiles) fail(CFD_EINTERNAL, "tile list overflow");
  std::vector<TileDesc> h;
  h.reserve(v.size());
  if (c->tun.order == 1) {
    // XCD-aware: 8 spatially contiguous chunks (natural block, k, j, i order),
    // interleaved so list position p belongs to chunk p mod 8.  The persistent
    // grid has a multiple of 8 workgroups and workgroup w runs on XCD w mod 8,
    // so each XCD sweeps one chunk and its L2 keeps the shared halos.
    const size_t n = v.size();
    size_t bounds[9];
    for (int x = 0; x <= 8; ++x) bounds[x] = n * x / 8;
    const size_t rounds = (n + 7) / 8 + 1;
    for (size_t l = 0; l < rounds; ++l)
      for (int x = 0; x < 8; ++x)
        if (bounds[x] + l < bounds[x + 1]) h.push_back(v[bounds[x] + l].t);
  } else {
    // longest-processing-time order: big tiles first, ties keep block order
    std::stable_sort(v.begin(), v.end(), [](const T2& a, const T2& b) { return a.work > b.work; });
    for (size_t i = 0; i < v.size(); ++i) h.push_back(v[i].t);
  }
  c->ntiles = (int)h.size();
  HIPCHK(hipMemcpyAsync(c->dtiles, h.data(), sizeof(TileDesc) * h.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
}

int nwg_for(const cfd_ctx* c, int per_cu) {
  return std::max(1, std::min({c->ntiles, NWG_MAX, 256 * per_cu}));
}

// Grid of the row-per-wave time-step and norms kernels: 8 four-wave
// workgroups per CU, capped by the number of 64-cell row chunks and by half
// the partials buffer (a step stores two kernels' rows in it, one after the
// other).  A function of the grid alone, not of the stage kernels' tiles, so
// that the sums of V Q these kernels reduce are the same bits for every tuning.
int dt_nwg(const cfd_ctx* c) {
  return (int)std::max<int64_t>(
      1, std::min<int64_t>({(c->nchunks + 3) / 4, (int64_t)NWG_MAX / 2, (int64_t)c->num_cu * 8}));
}

// Run a launch; with profiling on, bracket it with a hipEvent pair on its stream.
template <typename F>
void timed(cfd_ctx* c, int cls, hipStream_t s, F&& launch) {
  if (!c->profiling) {
    launch();
    return;
  }
  hipEvent_t a = c->take_event(), b = c->take_event();
  HIPCHK(hipEventRecord(a, s));
  launch();
  HIPCHK(hipEventRecord(b, s));
  c->ev_used.push_back({a, b, cls});
}

// full: the i -> j -> k sweeps (edges and corners included) even where one
// launch over the faces would do.
void ghost_fill(cfd_ctx* c, double* q, hipStream_t s, bool full = false) {
  if (!full && c->pm_count > 0) {
    timed(c, 1, s, [&] {
      launch_ghost_q(q, c->met(), c->dblocks, c->dpatches + c->pm_off, c->pm_count, c->pm_threads, c->SP, s);
    });
    return;
  }
  for (int d = 0; d < 3; ++d)
    timed(c, 1, s, [&] {
      launch_ghost_q(q, c->met(), c->dblocks, c->dpatches + c->poff[3 + d], c->pcount[3 + d], c->qthreads[d],
                     c->SP, s);
    });
}

StageArgs stage_args(cfd_ctx* c) {
  StageArgs A{};
  A.met = c->met();
  A.vmet = c->params.viscous ? c->vmet() : nullptr;
  A.local_dt = c->params.local_dt;
  A.dt = c->params.local_dt ? c->scal() : c->d_dt();
  A.ntiles = c->ntiles;
  A.tile_j = c->tun.tile_j;
  A.tile_k = c->tun.tile_k;
  A.sp = c->SP;
  return A;
}

// Persistent grid of the stage kernel: resident workgroups per CU (occupancy
// query, cached per variant) times the CU count, capped by the tile count.
int stage_nwg(cfd_ctx* c, int mode) {
  if (c->tun.kernel == 1) return nwg_for(c, 8);
  const int key = (c->params.viscous ? 1 : 0) | (c->params.flux_fp32 ? 2 : 0) | (mode << 2) |
                  ((c->tun.tile_j == 2 ? 0 : c->tun.tile_j == 4 ? 1 : 2) << 4) | (c->tun.kernel << 6);
  auto it = c->occ_cache.find(key);
  int occ;
  if (it != c->occ_cache.end()) {
    occ = it->second;
  } else {
    StageArgs A{};
    A.tile_j = c->tun.tile_j;
    const bool ok = c->tun.kernel == 2
                        ? stage_ring(A, mode, c->params.viscous != 0, c->params.flux_fp32 != 0, nullptr, nullptr,
                                     c->g64, c->g32, 0, nullptr, &occ)
                        : stage_tiled(A, mode, c->params.viscous != 0, c->params.flux_fp32 != 0, nullptr, nullptr,
                                      c->g64, c->g32, 0, nullptr, &occ);
    if (!ok) fail(CFD_EINVAL, "stage kernel %d has no variant for tile_j = %d", c->tun.kernel, c->tun.tile_j);
    c->occ_cache[key] = occ;
  }
  return std::max(1, std::min({c->ntiles, NWG_MAX / 2, occ * c->num_cu}));   // room for the k_dt rows too
}

void launch_stage(cfd_ctx* c, const StageArgs& A, int mode, hipStream_t s) {
  const bool visc = c->params.viscous != 0, fp32 = c->params.flux_fp32 != 0;
  const int nwg = stage_nwg(c, mode);
  if (c->tun.kernel == 0) {
    timed(c, 0, s, [&] {
      if (!stage_tiled(A, mode, visc, fp32, c->dblocks, c->dtiles, c->g64, c->g32, nwg, s, nullptr))
        fail(CFD_EINVAL, "tiled kernel has no variant for tile_j = %d", c->tun.tile_j);
    });
  } else if (c->tun.kernel == 2) {
    timed(c, 0, s, [&] {
      if (!stage_ring(A, mode, visc, fp32, c->dblocks, c->dtiles, c->g64, c->g32, nwg, s, nullptr))
        fail(CFD_EINVAL, "plane-ring kernel takes tile_j = 4 or 8, got %d", c->tun.tile_j);
    });
  } else {
    timed(c, 0, s, [&] { launch_stage_simple(A, mode, visc, fp32, c->dblocks, c->dtiles, c->g64, c->g32, nwg, s); });
  }
}

// CFL time step of q: per-cell steps (local stepping) and, with min_dt, the
// minimum into d_dt (read by global-step stages and forcing, and by the
// history row).
void time_step_pass(cfd_ctx* c, const double* q, hipStream_t s, bool min_dt = true) {
  const int nwg = dt_nwg(c);
  timed(c, 2, s, [&] {
    launch_dt(q, c->met(), c->scal(), c->part_dt(), c->dblocks, c->nblk, c->nchunks, c->SP, nwg, s);
  });
  if (min_dt) launch_finalize(c->part_dt(), nwg, 0, 0.0, c->d_dt(), nullptr, nullptr, s);
}

// Whether stage 3 evaluates the next step's time step: the plane-ring kernel
// on viscous flow (measured faster than the separate time-step kernel there;
// slower on inviscid flow, whose stage kernel is cheap next to it).
bool fused_dt(const cfd_ctx* c) { return c->tun.kernel == 2 && c->params.viscous; }

// One full RK3 step: 3 x (ghost fill + stage), the time step of Q^n and the
// history row (dt, L2(R(Q^n)), sum V Q^n, max |R_rho|).
//  - Time step: with fused_dt, left in d_dt (and the per-cell arena) by the
//    previous step's stage 3, or by the time-step pass cfd_step runs before
//    its first step; otherwise a time-step pass first (k_dt writes partial
//    rows [0, nwg_dt) of part_dt: min dt, sum V Q^n).
//  - History: the plane-ring kernel's stage 1 reduces the norm partials of
//    R(Q^n) itself; the other kernels write R(Q^n) to qb (free until stage 2
//    overwrites it) and the norms kernel adds the R rows after k_dt's (only
//    when the step keeps a history: without one they skip both).
//  - Totals sum V Q^n: always from rows [0, nwg_dt) of a row-chunk kernel
//    (k_dt, or with the plane-ring kernel k_norms over Q^n, only when the
//    step keeps a history), whose cut of the grid does not depend on the
//    tiles; the rows after them carry zeros in those slots, so the fixed-order
//    finalize gives the same totals for every tuning and stage kernel.
// (Taking dt of the new state inside the tiled kernel's third stage was
// measured slower: its extra metric loads cost more than the separate pass.)
void enqueue_step(cfd_ctx* c, double* q, hipStream_t s, bool history, const double* force = nullptr,
                  bool no_fuse = false) {
  const bool ring = c->tun.kernel == 2;
  const bool fuse = fused_dt(c) && !no_fuse && !force;
  const int nwg_f = dt_nwg(c);
  // a multigrid level's forcing: each stage's output minus b dt F, applied
  // by the tiled and simple stage kernels themselves, after the plane-ring
  // kernel by a pass of its own (the same rounding either way)
  const double* force_in_stage = ring ? nullptr : force;
  auto forced = [&](double* out, double b) {
    if (force && ring)
      launch_mg_force(out, force, c->params.local_dt ? c->scal() : c->d_dt(), c->params.local_dt, b, c->dblocks,
                      c->nblk, c->nchunks, nwg_f, s);
  };
  const double inv_n = 1.0 / (double)c->ncells;
  const int nwg_dt = dt_nwg(c);
  ghost_fill(c, q, s);
  // Local steps without a history row read no minimum step: every stage and
  // the forcing take the per-cell steps.
  if (!fuse) time_step_pass(c, q, s, history || !c->params.local_dt);
  StageArgs A = stage_args(c);
  A.qs = q;
  A.qn = q;
  A.out = c->qa();
  A.force = force_in_stage;
  A.fb = 1.0;
  if (ring) {
    const int ntot = history ? nwg_dt : 0;
    if (history)
      timed(c, 3, s, [&] {
        launch_norms(q, nullptr, c->met(), c->part_nrm(), c->dblocks, c->nblk, c->nchunks, nwg_dt, s);
      });
    A.partials = c->part_nrm() + (int64_t)ntot * NPART;
    launch_stage(c, A, 1, s);
    launch_finalize(c->part_nrm(), ntot + stage_nwg(c, 1), 1, inv_n, c->d_dt(), c->d_hist(), c->d_nonfinite(), s);
  } else if (history) {
    A.rout = c->qb();
    launch_stage(c, A, 1, s);
    timed(c, 3, s, [&] {
      launch_norms(nullptr, c->qb(), nullptr, c->part_dt() + (int64_t)nwg_dt * NPART, c->dblocks, c->nblk,
                   c->nchunks, nwg_dt, s);
    });
    launch_finalize(c->part_dt(), 2 * nwg_dt, 1, inv_n, c->d_dt(), c->d_hist(), c->d_nonfinite(), s);
  } else {
    launch_stage(c, A, 1, s);
  }
  forced(c->qa(), 1.0);
  A.rout = nullptr;
  A.partials = nullptr;
  ghost_fill(c, c->qa(), s);
  A.qs = c->qa();
  A.out = c->qb();
  A.a = 0.75;
  A.b = 0.25;
  A.fb = 0.25;
  launch_stage(c, A, 2, s);
  forced(c->qb(), 0.25);
  ghost_fill(c, c->qb(), s);
  A.qs = c->qb();
  A.out = q;
  A.a = 1.0 / 3.0;
  A.b = 2.0 / 3.0;
  A.fb = 2.0 / 3.0;
  if (fuse) {
    A.partials = c->part_dt();
    A.dt_out = c->params.local_dt ? c->scal() : nullptr;
    launch_stage(c, A, 3, s);
    launch_finalize(c->part_dt(), stage_nwg(c, 3), 0, 0.0, c->d_dt(), nullptr, nullptr, s);
  } else {
    launch_stage(c, A, 2, s);
  }
  forced(q, 2.0 / 3.0);
}

template <typename F>
cfd_status guard(cfd_ctx* c, F&& f) {
  try {
    f();
    return CFD_OK;
  } catch (const Err& e) {
    g_last_error = e.msg;
    if (c) c->last_error = e.msg;
    return e.st;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    if (c) c->last_error = e.what();
    return CFD_EINTERNAL;
  } catch (...) {
    g_last_error = "unknown internal error";
    if (c) c->last_error = g_last_error;
    return CFD_EINTERNAL;
  }
}

// Implicit step workspace: four arenas in the state layout (the residual of
// Q^n, two update iterates, and the face coefficients / diagonal / per-cell
// step), each 256-byte aligned.
size_t implicit_arena_bytes(const cfd_ctx* c) { return align256((size_t)c->L.q_elems * sizeof(double)); }

// One implicit step on the finite-volume residual (kernels_implicit.hip):
// ghost fill of Q^n, the CFL step at `cfl` (global minimum; the per-cell steps
// come with the face coefficients), R(Q^n), the history row (norms of R, totals
// of Q^n, minimum step), face coefficients and the diagonal, `sweeps` Jacobi
// sweeps each after a ghost fill of the iterate (connections copy it, physical
// patches zero it), Q += dQ.
void enqueue_implicit_step(cfd_ctx* c, double* q, int sweeps, double cfl, char* work, hipStream_t s) {
  const size_t ab = implicit_arena_bytes(c);
  double* R = reinterpret_cast<double*>(work);
  double* dA = reinterpret_cast<double*>(work + ab);
  double* dB = reinterpret_cast<double*>(work + 2 * ab);
  double* MU = reinterpret_cast<double*>(work + 3 * ab);
  StepParams P = c->SP;
  P.cfl = cfl;
  const int nwg = dt_nwg(c);
  ghost_fill(c, q, s);
  timed(c, 2, s, [&] {
    launch_dt(q, c->met(), c->scal(), c->part_dt(), c->dblocks, c->nblk, c->nchunks, P, nwg, s);
  });
  launch_finalize(c->part_dt(), nwg, 0, 0.0, c->d_dt(), nullptr, nullptr, s);
  StageArgs A = stage_args(c);
  A.qs = q;
  A.qn = q;
  A.out = R;
  launch_stage(c, A, 0, s);
  timed(c, 3, s, [&] { launch_norms(q, R, c->met(), c->part_nrm(), c->dblocks, c->nblk, c->nchunks, nwg, s); });
  launch_finalize(c->part_nrm(), nwg, 1, 1.0 / (double)c->ncells, c->d_dt(), c->d_hist(), c->d_nonfinite(), s);
  ImplicitArgs I{};
  I.q = q;
  I.met = c->met();
  I.r = R;
  I.mu = MU;
  I.dt = c->d_dt();
  I.local = c->params.local_dt;
  I.viscous = c->params.viscous;
  I.gamma = c->SP.gamma;
  I.prandtl = c->SP.prandtl;
  I.mu_inf = c->SP.mu_inf;
  I.s_star = c->SP.s_star;
  I.cfl = cfl;
  launch_ifv_faces(I, c->dblocks, c->nblk, c->nchunks, P, nwg, s);
  I.dq_out = dA;
  launch_ifv_diag(I, c->dblocks, c->nblk, c->nchunks, nwg, s);
  double* cur = dA;
  double* nxt = dB;
  for (int k = 0; k < sweeps; ++k) {
    for (int d = 0; d < 3; ++d)
      launch_ghost_q(cur, c->met(), c->dblocks, c->dpatches + c->poff[3 + d], c->pcount[3 + d], c->qthreads[d],
                     c->SP, s, 1);
    I.dq_in = cur;
    I.dq_out = nxt;
    timed(c, 0, s, [&] { launch_ifv_sweep(I, c->dblocks, c->nblk, c->nchunks, nwg, s); });
    std::swap(cur, nxt);
  }
  launch_ifv_apply(q, cur, c->dblocks, c->nblk, c->nchunks, nwg, s);
}

void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) fail(CFD_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
}

}  // namespace

namespace cfd {

cfd_status host_guarded(const std::function<void()>& f) { return guard(nullptr, f); }

void host_fail(cfd_status st, const std::string& msg) { throw Err(st, msg); }

void host_check_dims(int nblk, const cfd_dims* dims) { check_dims(nblk, dims); }

void host_check_case(int nblk, const cfd_dims* dims, int nconn, const cfd_conn* conns, int nbc,
                     const cfd_bc* bcs) {
  check_dims(nblk, dims);
  validate_tables(nblk, dims, nconn, conns, nbc, bcs);
}

}  // namespace cfd

extern "C" {

cfd_status cfd_layout(int32_t nblk, const cfd_dims* dims, int32_t ghost_layers, int64_t* block_offset,
                      int64_t* block_strides, int64_t* arena_elems) {
  return guard(nullptr, [&] {
    if (ghost_layers != NG) fail(CFD_EUNSUPPORTED, "ghost_layers must be %d", NG);
    check_dims(nblk, dims);
    Layout L = make_layout(nblk, dims);
    for (int b = 0; b < nblk; ++b) {
      if (block_offset) block_offset[b] = L.qoff[b];
      if (block_strides) {
        block_strides[4 * b + 0] = L.sv[b];
        block_strides[4 * b + 1] = L.sk[b];
        block_strides[4 * b + 2] = L.sj[b];
        block_strides[4 * b + 3] = 1;
      }
    }
    if (arena_elems) *arena_elems = L.q_elems;
  });
}

// node sweeps, cell sweeps and the one-launch face set
static int count_patches(int nconn, int nbc) { return 3 * (nconn + nbc); }
constexpr int PATCHES_PER_BLOCK = 3 * 6 * 64;   // reserved: 64 patches per face on average

cfd_status cfd_workspace_size(const cfd_params* params, int32_t nblk, const cfd_dims* dims,
                              size_t* workspace_bytes) {
  return guard(nullptr, [&] {
    check_params(params);
    check_dims(nblk, dims);
    if (!workspace_bytes) fail(CFD_EINVAL, "workspace_bytes is NULL");
    Layout L = make_layout(nblk, dims);
    // patch count is bounded by 6 faces x a generous number of patches; the
    // exact count is only known with the tables, so reserve for 64 per face.
    WsLayout W = make_ws(L, nblk, dims, PATCHES_PER_BLOCK * nblk, params->local_dt != 0, params->viscous != 0);
    *workspace_bytes = W.total;
  });
}

cfd_status cfd_create_blocks(const cfd_params* params, int32_t nblk, const cfd_dims* dims,
                             const double* const* nodes_dev, int32_t nconn, const cfd_conn* conns, int32_t nbc,
                             const cfd_bc* bcs, void* workspace_dev, size_t workspace_bytes, hipStream_t stream,
                             cfd_ctx** out) {
  if (out) *out = nullptr;
  cfd_ctx* c = nullptr;
  cfd_status st = guard(nullptr, [&] {
    if (!out) fail(CFD_EINVAL, "out is NULL");
    check_params(params);
    check_dims(nblk, dims);
    if (!nodes_dev) fail(CFD_EINVAL, "nodes_dev is NULL");
    for (int b = 0; b < nblk; ++b)
      if (!nodes_dev[b]) fail(CFD_EINVAL, "nodes_dev[%d] is NULL", b);
    validate_tables(nblk, dims, nconn, conns, nbc, bcs);
    if (!workspace_dev) fail(CFD_EINVAL, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(workspace_dev) & 255) != 0) fail(CFD_EINVAL, "workspace must be 256-byte aligned");
    const int npatch = count_patches(nconn, nbc);
    if (npatch > PATCHES_PER_BLOCK * nblk) fail(CFD_EUNSUPPORTED, "more than 64 patches per face on average");
    c = new cfd_ctx();
    c->id = g_ctx_ids++;
    c->params = *params;
    c->nblk = nblk;
    c->dims.assign(dims, dims + nblk);
    c->L = make_layout(nblk, dims);
    size_t need = 0;
    {
      WsLayout Wfull = make_ws(c->L, nblk, dims, PATCHES_PER_BLOCK * nblk, params->local_dt != 0, params->viscous != 0);
      need = Wfull.total;
    }
    if (workspace_bytes < need) fail(CFD_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    c->W = make_ws(c->L, nblk, dims, PATCHES_PER_BLOCK * nblk, params->local_dt != 0, params->viscous != 0);
    c->ws = static_cast<char*>(workspace_dev);
    c->dblocks = reinterpret_cast<BlockDesc*>(c->ws + c->W.blocks);
    c->dpatches = reinterpret_cast<PatchDesc*>(c->ws + c->W.patches);
    c->dtiles = reinterpret_cast<TileDesc*>(c->ws + c->W.tiles);
    set_params(c);
    for (int b = 0; b < nblk; ++b) {
      BlockDesc B{};
      B.n[0] = dims[b].ni;
      B.n[1] = dims[b].nj;
      B.n[2] = dims[b].nk;
      B.qoff = c->L.qoff[b];
      B.moff = c->L.moff[b];
      B.soff = c->L.soff[b];
      B.voff = c->L.voff[b];
      B.sv = c->L.sv[b];
      B.sk = c->L.sk[b];
      B.sj = c->L.sj[b];
      B.xoff = c->L.xoff[b];   // padded node (-g,-g,-g) at the start of the block's scratch
      B.xsv = c->L.xsv[b];
      B.xsk = c->L.xsk[b];
      B.xsj = c->L.xsj[b];
      B.coff = c->nchunks;
      c->nchunks += (int64_t)((dims[b].ni + 63) / 64) * dims[b].nj * dims[b].nk;
      c->hblocks.push_back(B);
      c->ncells += (int64_t)dims[b].ni * dims[b].nj * dims[b].nk;
    }
    std::vector<PatchDesc> all;
    for (int sweep = 0; sweep < 6; ++sweep) {
      const bool nodes = sweep < 3;
      const int d = sweep % 3;
      c->poff[sweep] = (int)all.size();
      int mx = 0;
      build_patches(d, nodes, params, dims, nconn, conns, nbc, bcs, all, mx);
      c->pcount[sweep] = (int)all.size() - c->poff[sweep];
      c->pmax[sweep] = mx;
      if (!nodes)
        for (int p = c->poff[sweep]; p < (int)all.size(); ++p)
          c->qthreads[d] = std::max(c->qthreads[d], all[p].count * ghost_threads_per_point(all[p].kind, d));
    }
    if (!params->viscous) {
      c->pm_off = (int)all.size();
      for (int d = 0; d < 3; ++d) {
        int mx = 0;
        const int p0 = (int)all.size();
        build_patches(d, false, params, dims, nconn, conns, nbc, bcs, all, mx, false);
        for (int p = p0; p < (int)all.size(); ++p)
          c->pm_threads = std::max(c->pm_threads, all[p].count * ghost_threads_per_point(all[p].kind, d));
      }
      c->pm_count = (int)all.size() - c->pm_off;
    }
    HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    {
      int dev = 0;
      HIPCHK(hipGetDevice(&dev));
      HIPCHK(hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, dev));
    }
    HIPCHK(hipMemcpyAsync(c->dblocks, c->hblocks.data(), sizeof(BlockDesc) * nblk, hipMemcpyHostToDevice, stream));
    if (!all.empty())
      HIPCHK(hipMemcpyAsync(c->dpatches, all.data(), sizeof(PatchDesc) * all.size(), hipMemcpyHostToDevice, stream));
    // setup pipeline: padded nodes -> ghost nodes -> metrics -> metric ghosts
    // (-> viscous face metrics)
    double* x = reinterpret_cast<double*>(c->ws + c->W.node_scratch);
    for (int b = 0; b < nblk; ++b) launch_copy_nodes(nodes_dev[b], x, c->hblocks[b], stream);
    check_launch();
    for (int d = 0; d < 3; ++d)
      launch_ghost_nodes(x, c->dblocks, c->dpatches + c->poff[d], c->pcount[d], c->pmax[d], stream);
    check_launch();
    for (int b = 0; b < nblk; ++b) launch_metrics(x, c->met(), c->hblocks[b], stream);
    check_launch();
    for (int d = 0; d < 3; ++d)
      launch_metric_ghosts(c->met(), c->dblocks, c->dpatches + c->poff[3 + d], c->pcount[3 + d], c->pmax[3 + d],
                           stream);
    check_launch();
    if (params->viscous) {
      for (int b = 0; b < nblk; ++b) launch_visc_metrics(c->met(), c->vmet(), c->hblocks[b], stream);
      check_launch();
    }
    HIPCHK(hipStreamSynchronize(stream));
    {
      std::vector<int64_t> cs(nblk + 1, 0);
      for (int b = 0; b < nblk; ++b) cs[b + 1] = cs[b] + (int64_t)dims[b].ni * dims[b].nj * dims[b].nk;
      HIPCHK(hipMemcpyAsync(c->d_cell_start(), cs.data(), sizeof(int64_t) * cs.size(), hipMemcpyHostToDevice,
                            stream));
    }
    c->tun = default_tuning(c->dims, c->num_cu, c->params);
    build_tiles(c, stream);
    *out = c;
  });
  if (st != CFD_OK && c) {
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    delete c;
  }
  return st;
}

cfd_status cfd_set_profiling(cfd_ctx* c, int32_t enable) {
  return guard(c, [&] {
    if (!c) fail(CFD_EINVAL, "NULL context");
    if (!enable) {
      HIPCHK(hipDeviceSynchronize());
      c->release_events();
    }
    c->profiling = enable != 0;
  });
}

cfd_status cfd_profile_read(cfd_ctx* c, double out[16]) {
  return guard(c, [&] {
    if (!c || !out) fail(CFD_EINVAL, "NULL argument");
    for (int k = 0; k < 4; ++k) {
      out[4 * k + 0] = 0.0;
      out[4 * k + 1] = 0.0;
      out[4 * k + 2] = 1e300;
      out[4 * k + 3] = 0.0;
    }
    for (auto& p : c->ev_used) {
      HIPCHK(hipEventSynchronize(p.b));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
      double* o = out + 4 * p.cls;
      o[0] += 1.0;
      o[1] += ms;
      o[2] = std::min(o[2], (double)ms);
      o[3] = std::max(o[3], (double)ms);
    }
    for (int k = 0; k < 4; ++k)
      if (out[4 * k] == 0.0) out[4 * k + 2] = 0.0;
    c->release_events();
  });
}

cfd_status cfd_destroy(cfd_ctx* c) {
  if (!c) return CFD_OK;
  c->destroy_events();
  c->drop_graph();
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  delete c;
  return CFD_OK;
}

cfd_status cfd_set_tuning(cfd_ctx* c, const cfd_tuning* t) {
  return guard(c, [&] {
    if (!c || !t) fail(CFD_EINVAL, "NULL argument");
    if (t->kernel < 0 || t->kernel > 2) fail(CFD_EINVAL, "kernel must be 0, 1 or 2");
    if (t->tile_j < 1 || t->tile_j > 16 || (t->tile_j & (t->tile_j - 1)))
      fail(CFD_EINVAL, "tile_j must be a power of two in [1, 16]");
    if (t->tile_k < 1 || t->tile_k > 4096) fail(CFD_EINVAL, "tile_k must be in [1, 4096]");
    if (t->order < 0 || t->order > 1) fail(CFD_EINVAL, "order must be 0 or 1");
    if (t->kernel == 0 && t->tile_j != 2 && t->tile_j != 4 && t->tile_j != 8)
      fail(CFD_EINVAL, "the tiled kernel takes tile_j = 2, 4 or 8");
    if (t->kernel == 2 && t->tile_j != 4 && t->tile_j != 8)
      fail(CFD_EINVAL, "the plane-ring kernel takes tile_j = 4 or 8");
    c->drop_graph();
    c->tun = *t;
    ++c->gen;
    HIPCHK(hipDeviceSynchronize());
    build_tiles(c, c->cap_stream);
  });
}

cfd_status cfd_get_tuning(const cfd_ctx* c, cfd_tuning* t) {
  if (!c || !t) return CFD_EINVAL;
  *t = c->tun;
  return CFD_OK;
}

cfd_status cfd_fill_ghosts(cfd_ctx* c, double* q, hipStream_t s) {
  return guard(c, [&] {
    if (!c || !q) fail(CFD_EINVAL, "NULL argument");
    ghost_fill(c, q, s, true);
    check_launch();
  });
}

cfd_status cfd_residual(cfd_ctx* c, const double* q, double* r, hipStream_t s) {
  return guard(c, [&] {
    if (!c || !q || !r) fail(CFD_EINVAL, "NULL argument");
    if (q == r) fail(CFD_EINVAL, "q and r must not alias");
    StageArgs A = stage_args(c);
    A.qs = q;
    A.qn = q;
    A.out = r;
    launch_stage(c, A, 0, s);
    check_launch();
  });
}

cfd_status cfd_time_step(cfd_ctx* c, const double* q, double* dt_dev, hipStream_t s) {
  return guard(c, [&] {
    if (!c || !q || !dt_dev) fail(CFD_EINVAL, "NULL argument");
    const int nwg = dt_nwg(c);
    launch_dt(q, c->met(), c->scal(), c->part_dt(), c->dblocks, c->nblk, c->nchunks, c->SP, nwg, s);
    launch_finalize(c->part_dt(), nwg, 0, 0.0, dt_dev, nullptr, nullptr, s);
    check_launch();
  });
}

cfd_status cfd_step(cfd_ctx* c, double* q, int32_t nsteps, double* hist, hipStream_t s) {
  return guard(c, [&] {
    if (!c || !q) fail(CFD_EINVAL, "NULL argument");
    if (nsteps < 0) fail(CFD_EINVAL, "nsteps must be >= 0");
    // with fused_dt a step takes the time step of Q^n from the step before;
    // the state may have changed since, so the first one is computed here
    if (nsteps > 0 && fused_dt(c)) time_step_pass(c, q, s);
    if (c->tun.use_graph && !c->profiling) {
      if (c->graph_q != q) {
        c->drop_graph();
        c->graph_q = q;
      }
      // the one-step graph keeps the history (totals pass included); the
      // multi-step graph serves runs without one
      auto capture = [&](int steps, bool history, hipGraph_t& g, hipGraphExec_t& ge) {
        HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        try {
          for (int n = 0; n < steps; ++n) enqueue_step(c, q, c->cap_stream, history);
        } catch (...) {
          hipGraph_t gg = nullptr;
          hipStreamEndCapture(c->cap_stream, &gg);
          if (gg) hipGraphDestroy(gg);
          throw;
        }
        HIPCHK(hipStreamEndCapture(c->cap_stream, &g));
        HIPCHK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
      };
      int n0 = 0;
      if (!hist && nsteps >= cfd_ctx::STEPS_PER_GRAPH) {
        if (!c->gexec_n) capture(cfd_ctx::STEPS_PER_GRAPH, false, c->graph_n, c->gexec_n);
        for (; n0 + cfd_ctx::STEPS_PER_GRAPH <= nsteps; n0 += cfd_ctx::STEPS_PER_GRAPH)
          HIPCHK(hipGraphLaunch(c->gexec_n, s));
      }
      if (n0 < nsteps && !c->gexec) capture(1, true, c->graph, c->gexec);
      for (int n = n0; n < nsteps; ++n) {
        HIPCHK(hipGraphLaunch(c->gexec, s));
        if (hist)
          HIPCHK(hipMemcpyAsync(hist + (int64_t)n * NHIST, c->d_hist(), sizeof(double) * NHIST,
                                hipMemcpyDeviceToDevice, s));
      }
    } else {
      for (int n = 0; n < nsteps; ++n) {
        enqueue_step(c, q, s, hist != nullptr);
        check_launch();
        if (hist)
          HIPCHK(hipMemcpyAsync(hist + (int64_t)n * NHIST, c->d_hist(), sizeof(double) * NHIST,
                                hipMemcpyDeviceToDevice, s));
      }
    }
  });
}

cfd_status cfd_implicit_work_size(const cfd_ctx* c, size_t* bytes) {
  return guard(const_cast<cfd_ctx*>(c), [&] {
    if (!c || !bytes) fail(CFD_EINVAL, "NULL argument");
    *bytes = 4 * implicit_arena_bytes(c);
  });
}

cfd_status cfd_step_implicit(cfd_ctx* c, double* q, int32_t nsteps, int32_t sweeps, double cfl, void* work,
                             size_t work_bytes, double* hist, hipStream_t s) {
  return guard(c, [&] {
    if (!c || !q || !work) fail(CFD_EINVAL, "NULL argument");
    if (nsteps < 0) fail(CFD_EINVAL, "nsteps must be >= 0");
    if (sweeps < 0 || sweeps > 1000) fail(CFD_EINVAL, "sweeps must be in [0, 1000]");
    if (!(cfl > 0.0) || !std::isfinite(cfl)) fail(CFD_EINVAL, "cfl must be positive and finite");
    if (work_bytes < 4 * implicit_arena_bytes(c)) fail(CFD_ENOMEM, "workspace smaller than cfd_implicit_work_size()");
    if (reinterpret_cast<uintptr_t>(work) % 256) fail(CFD_EINVAL, "workspace must be 256-byte aligned");
    const size_t qb = (size_t)c->L.q_elems * sizeof(double);
    const char* w0 = static_cast<const char*>(work);
    const char* q0 = reinterpret_cast<const char*>(q);
    if (!(w0 + work_bytes <= q0 || q0 + qb <= w0)) fail(CFD_EINVAL, "state and workspace overlap");
    for (int n = 0; n < nsteps; ++n) {
      enqueue_implicit_step(c, q, sweeps, cfl, static_cast<char*>(work), s);
      check_launch();
      if (hist)
        HIPCHK(hipMemcpyAsync(hist + (int64_t)n * NHIST, c->d_hist(), sizeof(double) * NHIST,
                              hipMemcpyDeviceToDevice, s));
    }
  });
}

// ---------------------------------------------------------------- multigrid
// Levels of a hierarchy: the same block count, every extent of level l + 1
// half the one of level l (the coarse grid keeps every second node; the
// tables are the caller's coarsening), the same flow parameters.
void check_hierarchy(cfd_ctx* const* lv, int n) {
  if (!lv) fail(CFD_EINVAL, "NULL argument");
  if (n < 1 || n > 16) fail(CFD_EINVAL, "nlevels must be in [1, 16]");
  for (int l = 0; l < n; ++l)
    if (!lv[l]) fail(CFD_EINVAL, "NULL level");
  for (int l = 1; l < n; ++l) {
    if (lv[l] == lv[l - 1]) fail(CFD_EINVAL, "levels must be distinct contexts");
    if (lv[l]->nblk != lv[0]->nblk) fail(CFD_EINVAL, "every level must have the same blocks");
    const cfd_params &a = lv[l]->params, &b = lv[0]->params;
    if (a.gamma != b.gamma || a.prandtl != b.prandtl || a.mach != b.mach || a.alpha != b.alpha || a.beta != b.beta ||
        a.reynolds != b.reynolds || a.sutherland != b.sutherland || a.cfl != b.cfl ||
        a.entropy_fix != b.entropy_fix || a.limiter_eps != b.limiter_eps || a.viscous != b.viscous ||
        a.flux_fp32 != b.flux_fp32 || a.local_dt != b.local_dt)
      fail(CFD_EINVAL, "every level must take the same flow parameters");
    for (int b = 0; b < lv[0]->nblk; ++b) {
      const cfd_dims& f = lv[l - 1]->dims[b];
      const cfd_dims& c = lv[l]->dims[b];
      if (f.ni != 2 * c.ni || f.nj != 2 * c.nj || f.nk != 2 * c.nk)
        fail(CFD_EINVAL, "every extent of a level must be twice the next level's");
    }
  }
}

// Per level: its residual, its forcing and its restricted initial state, each
// a state-layout arena of the level, 256-byte aligned.
size_t mg_level_bytes(const cfd_ctx* c) { return 3 * implicit_arena_bytes(c); }

// One V-cycle (full approximation storage, RK3 smoothing; see cfd.h).
// record: the finest level's first step keeps its history row (in lv[0]'s
// history slot); hist (nullable): copied there after that step.
void enqueue_mg_cycle(cfd_ctx* const* lv, double* const* q, int L, int pre, int coarse, char* work, bool record,
                      double* hist, hipStream_t s) {
  std::vector<double*> R(L), F(L), Q0(L);
  char* at = work;
  for (int l = 0; l < L; ++l) {
    const size_t ab = implicit_arena_bytes(lv[l]);
    R[l] = reinterpret_cast<double*>(at);
    F[l] = reinterpret_cast<double*>(at + ab);
    Q0[l] = reinterpret_cast<double*>(at + 2 * ab);
    at += 3 * ab;
  }
  const int nblk = lv[0]->nblk;
  for (int l = 0; l < L; ++l) {
    cfd_ctx* c = lv[l];
    const int steps = l == L - 1 ? coarse : pre;
    for (int n = 0; n < steps; ++n) {
      const bool rec = record && l == 0 && n == 0;
      enqueue_step(c, q[l], s, rec, l ? F[l] : nullptr, true);
      if (rec && hist)
        HIPCHK(hipMemcpyAsync(hist, c->d_hist(), sizeof(double) * NHIST, hipMemcpyDeviceToDevice, s));
    }
    if (l == L - 1) break;
    cfd_ctx* cn = lv[l + 1];
    ghost_fill(c, q[l], s);
    StageArgs A = stage_args(c);
    A.qs = q[l];
    A.qn = q[l];
    A.out = R[l];
    launch_stage(c, A, 0, s);
    launch_mg_restrict(q[l], c->met(), R[l], l ? F[l] : nullptr, c->dblocks, q[l + 1], Q0[l + 1], F[l + 1],
                       cn->met(), cn->dblocks, nblk, cn->nchunks, dt_nwg(cn), s);
    ghost_fill(cn, q[l + 1], s);
    StageArgs B = stage_args(cn);
    B.qs = q[l + 1];
    B.qn = q[l + 1];
    B.out = R[l + 1];
    launch_stage(cn, B, 0, s);
    launch_mg_forcing(F[l + 1], R[l + 1], cn->dblocks, nblk, cn->nchunks, dt_nwg(cn), s);
  }
  for (int l = L - 2; l >= 0; --l)
    launch_mg_prolong(q[l], lv[l]->dblocks, q[l + 1], Q0[l + 1], lv[l + 1]->dblocks, nblk, lv[l]->nchunks,
                      dt_nwg(lv[l]), s);
}

cfd_status cfd_mg_work_size(cfd_ctx* const* levels, int32_t nlevels, size_t* bytes) {
  return guard(nullptr, [&] {
    if (!bytes) fail(CFD_EINVAL, "NULL argument");
    check_hierarchy(levels, nlevels);
    size_t b = 0;
    for (int l = 0; l < nlevels; ++l) b += mg_level_bytes(levels[l]);
    *bytes = b;
  });
}

cfd_status cfd_mg_cycles(cfd_ctx* const* levels, double* const* q_levels, int32_t nlevels, int32_t pre,
                         int32_t coarse, int32_t ncycles, void* work, size_t work_bytes, double* hist,
                         hipStream_t s) {
  return guard(levels && nlevels > 0 ? levels[0] : nullptr, [&] {
    check_hierarchy(levels, nlevels);
    if (!q_levels || !work) fail(CFD_EINVAL, "NULL argument");
    if (pre < 0 || coarse < 0 || pre > 1000 || coarse > 1000) fail(CFD_EINVAL, "pre and coarse must be in [0, 1000]");
    if (ncycles < 0) fail(CFD_EINVAL, "ncycles must be >= 0");
    if (hist && pre < 1 && nlevels > 1) fail(CFD_EINVAL, "a history needs at least one step on the finest level");
    if (hist && nlevels == 1 && coarse < 1) fail(CFD_EINVAL, "a history needs at least one step on the finest level");
    size_t need = 0;
    for (int l = 0; l < nlevels; ++l) need += mg_level_bytes(levels[l]);
    if (work_bytes < need) fail(CFD_ENOMEM, "workspace smaller than cfd_mg_work_size()");
    if (reinterpret_cast<uintptr_t>(work) % 256) fail(CFD_EINVAL, "workspace must be 256-byte aligned");
    const char* w0 = static_cast<const char*>(work);
    for (int l = 0; l < nlevels; ++l) {
      if (!q_levels[l]) fail(CFD_EINVAL, "NULL state");
      const size_t qb = (size_t)levels[l]->L.q_elems * sizeof(double);
      const char* a = reinterpret_cast<const char*>(q_levels[l]);
      if (!(w0 + need <= a || a + qb <= w0)) fail(CFD_EINVAL, "a state and the workspace overlap");
      for (int m = 0; m < l; ++m) {
        const size_t mb = (size_t)levels[m]->L.q_elems * sizeof(double);
        const char* b = reinterpret_cast<const char*>(q_levels[m]);
        if (!(a + qb <= b || b + mb <= a)) fail(CFD_EINVAL, "the levels' states overlap");
      }
    }
    cfd_ctx* c0 = levels[0];
    bool graph = c0->tun.use_graph != 0;
    for (int l = 0; l < nlevels; ++l) graph = graph && !levels[l]->profiling;
    if (!graph) {
      for (int n = 0; n < ncycles; ++n) {
        enqueue_mg_cycle(levels, q_levels, nlevels, pre, coarse, static_cast<char*>(work), hist != nullptr,
                         hist ? hist + (int64_t)n * NHIST : nullptr, s);
        check_launch();
      }
      return;
    }
    // one captured cycle, replayed; its history row is copied out after each
    std::vector<uint64_t> key{(uint64_t)nlevels, (uint64_t)pre, (uint64_t)coarse, hist ? 1u : 0u,
                              (uint64_t)reinterpret_cast<uintptr_t>(work)};
    for (int l = 0; l < nlevels; ++l) {
      key.push_back(levels[l]->id);
      key.push_back(levels[l]->gen);
      key.push_back((uint64_t)reinterpret_cast<uintptr_t>(q_levels[l]));
    }
    if (ncycles > 0 && (!c0->mg_gexec || c0->mg_key != key)) {
      c0->drop_mg_graph();
      HIPCHK(hipStreamBeginCapture(c0->cap_stream, hipStreamCaptureModeThreadLocal));
      try {
        enqueue_mg_cycle(levels, q_levels, nlevels, pre, coarse, static_cast<char*>(work), hist != nullptr, nullptr,
                         c0->cap_stream);
      } catch (...) {
        hipGraph_t gg = nullptr;
        hipStreamEndCapture(c0->cap_stream, &gg);
        if (gg) hipGraphDestroy(gg);
        throw;
      }
      HIPCHK(hipStreamEndCapture(c0->cap_stream, &c0->mg_graph));
      HIPCHK(hipGraphInstantiate(&c0->mg_gexec, c0->mg_graph, nullptr, nullptr, 0));
      c0->mg_key = key;
    }
    for (int n = 0; n < ncycles; ++n) {
      HIPCHK(hipGraphLaunch(c0->mg_gexec, s));
      if (hist)
        HIPCHK(hipMemcpyAsync(hist + (int64_t)n * NHIST, c0->d_hist(), sizeof(double) * NHIST,
                              hipMemcpyDeviceToDevice, s));
    }
  });
}

cfd_status cfd_norms(cfd_ctx* c, const double* q, const double* r, double* out, int32_t flags, hipStream_t s) {
  cfd_status st = guard(c, [&] {
    if (!c || !q || !out) fail(CFD_EINVAL, "NULL argument");
    const int nwg = dt_nwg(c);
    launch_norms(q, r, c->met(), c->part_nrm(), c->dblocks, c->nblk, c->nchunks, nwg, s);
    // history row layout: [dt, L2 x5, VQ x5, max]; norms output drops dt
    launch_finalize(c->part_nrm(), nwg, 1, 1.0 / (double)c->ncells, nullptr, c->d_norms(), c->d_nonfinite(), s);
    check_launch();
    if (flags & CFD_NORMS_HOST) {
      double row[NHIST + 1];
      HIPCHK(hipMemcpyAsync(row, c->d_norms(), sizeof(double) * NHIST, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(row + NHIST, c->d_nonfinite(), sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int q2 = 0; q2 < 11; ++q2) out[q2] = row[1 + q2];
      out[11] = row[NHIST];
    } else {
      HIPCHK(hipMemcpyAsync(out, c->d_norms() + 1, sizeof(double) * 11, hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(out + 11, c->d_nonfinite(), sizeof(double), hipMemcpyDeviceToDevice, s));
    }
  });
  if (st == CFD_OK && (flags & CFD_NORMS_HOST) && out[11] > 0.0) {
    c->last_error = "non-finite values in state or residual";
    return CFD_ENONFINITE;
  }
  return st;
}

cfd_status cfd_copy_metrics(cfd_ctx* c, int32_t blk, double* out, hipStream_t s) {
  return guard(c, [&] {
    if (!c || !out) fail(CFD_EINVAL, "NULL argument");
    if (blk < 0 || blk >= c->nblk) fail(CFD_EINVAL, "block %d out of range", blk);
    const BlockDesc& B = c->hblocks[blk];
    const size_t wi = (size_t)B.n[0] + 2 * NG, hj = (size_t)B.n[1] + 2 * NG, dk = (size_t)B.n[2] + 2 * NG;
    // rows of the padded block are strided; one 2-D copy per metric component
    for (int m = 0; m < NM; ++m)
      HIPCHK(hipMemcpy2DAsync(out + (size_t)m * wi * hj * dk, wi * sizeof(double),
                              c->met() + B.moff + (int64_t)m * B.sv, (size_t)B.sj * sizeof(double),
                              wi * sizeof(double), hj * dk, hipMemcpyDeviceToDevice, s));
  });
}

// ------------------------------------------------------------------ warm start

namespace {

constexpr int MLP_CHUNKS = 32;       // point chunks of the weight-gradient reduction
constexpr int MLP_MSE_ROWS = 1024;   // loss partial rows

MlpDims mlp_dims(const cfd_mlp_desc* d) {
  if (!d) fail(CFD_EINVAL, "mlp desc is NULL");
  if (d->activation != 1) fail(CFD_EUNSUPPORTED, "only SiLU (activation 1) is implemented");
  if (d->d_in < 1 || d->d_in > MLP_KIN) fail(CFD_EINVAL, "d_in must be in [1, %d]", MLP_KIN);
  if (d->d_out < 1 || d->d_out > MLP_NOUT) fail(CFD_EINVAL, "d_out must be in [1, %d]", MLP_NOUT);
  if (d->d_hidden < 16 || d->d_hidden > 128 || d->d_hidden % 16)
    fail(CFD_EINVAL, "d_hidden must be a multiple of 16 in [16, 128]");
  if (d->n_hidden < 1 || d->n_hidden > MLP_MAX_LAYERS - 1) fail(CFD_EINVAL, "n_hidden must be in [1, 8]");
  MlpDims D{};
  D.d_in = d->d_in;
  D.d_hidden = d->d_hidden;
  D.n_hidden = d->n_hidden;
  D.d_out = d->d_out;
  D.nlayer = d->n_hidden + 1;
  int64_t po = 0, co = 0;
  for (int l = 0; l < D.nlayer; ++l) {
    D.K[l] = l == 0 ? MLP_KIN : d->d_hidden;
    D.N[l] = l == D.nlayer - 1 ? MLP_NOUT : d->d_hidden;
    D.woff[l] = po;
    po += (int64_t)D.N[l] * D.K[l];
    D.boff[l] = po;
    po += D.N[l];
    D.hoff[l] = co;
    co += D.K[l];
    D.zoff[l] = co;
    co += D.N[l];
  }
  D.nparam = po;
  D.cache_per_point = co;
  return D;
}

size_t mlp_work_bytes(const MlpDims& D, int64_t n) {
  const size_t act = align256((size_t)n * D.d_hidden * sizeof(float));
  int64_t maxw = 0;
  for (int l = 0; l < D.nlayer; ++l) maxw = std::max<int64_t>(maxw, (int64_t)D.N[l] * D.K[l] + D.N[l]);
  return 2 * act + align256((size_t)MLP_CHUNKS * maxw * sizeof(float)) + align256(MLP_MSE_ROWS * sizeof(double));
}

}  // namespace

cfd_status cfd_mlp_sizes(const cfd_mlp_desc* desc, int64_t n, int64_t* n_params, int64_t* cache_per_point,
                         size_t* work_bytes) {
  return guard(nullptr, [&] {
    const MlpDims D = mlp_dims(desc);
    if (n < 0) fail(CFD_EINVAL, "n must be >= 0");
    if (n_params) *n_params = D.nparam;
    if (cache_per_point) *cache_per_point = D.cache_per_point;
    if (work_bytes) *work_bytes = mlp_work_bytes(D, n);
  });
}

cfd_status cfd_mlp_forward(const cfd_mlp_desc* desc, const uint16_t* params, const float* x, const int32_t* idx,
                           int64_t n, float* y, float* cache, hipStream_t s) {
  return guard(nullptr, [&] {
    const MlpDims D = mlp_dims(desc);
    if (!params || !x || !y || n < 0) fail(CFD_EINVAL, "bad forward arguments");
    if (n == 0) return;
    mlp_forward(D, params, x, idx, n, y, cache, s);
    check_launch();
  });
}

cfd_status cfd_mlp_mse(const cfd_mlp_desc* desc, const float* y, const float* t, const int32_t* idx, int64_t n,
                       float* dy, double* loss, void* work, size_t work_bytes, hipStream_t s) {
  return guard(nullptr, [&] {
    const MlpDims D = mlp_dims(desc);
    if (!y || !t || !dy || !loss || n <= 0 || !work) fail(CFD_EINVAL, "bad mse arguments");
    if (work_bytes < mlp_work_bytes(D, n)) fail(CFD_ENOMEM, "mlp workspace too small");
    const size_t act = align256((size_t)n * D.d_hidden * sizeof(float));
    int64_t maxw = 0;
    for (int l = 0; l < D.nlayer; ++l) maxw = std::max<int64_t>(maxw, (int64_t)D.N[l] * D.K[l] + D.N[l]);
    double* part = reinterpret_cast<double*>(static_cast<char*>(work) + 2 * act +
                                             align256((size_t)MLP_CHUNKS * maxw * sizeof(float)));
    mlp_mse(y, t, idx, n, D.d_out, dy, part, MLP_MSE_ROWS, loss, s);
    check_launch();
  });
}

cfd_status cfd_mlp_backward(const cfd_mlp_desc* desc, const uint16_t* params, const float* cache, const float* dy,
                            int64_t n, float* grad, void* work, size_t work_bytes, hipStream_t s) {
  return guard(nullptr, [&] {
    const MlpDims D = mlp_dims(desc);
    if (!params || !cache || !dy || !grad || n <= 0 || !work) fail(CFD_EINVAL, "bad backward arguments");
    if (work_bytes < mlp_work_bytes(D, n)) fail(CFD_ENOMEM, "mlp workspace too small");
    const size_t act = align256((size_t)n * D.d_hidden * sizeof(float));
    char* w = static_cast<char*>(work);
    float* dz = reinterpret_cast<float*>(w);
    float* da = reinterpret_cast<float*>(w + act);
    float* part = reinterpret_cast<float*>(w + 2 * act);
    mlp_backward(D, params, cache, dy, n, grad, dz, da, part, MLP_CHUNKS, s);
    check_launch();
  });
}

cfd_status cfd_mlp_adam(const cfd_mlp_desc* desc, float* master, float* m, float* v, const float* grad,
                        uint16_t* params, float lr, float b1, float b2, float eps, int32_t t, hipStream_t s) {
  return guard(nullptr, [&] {
    const MlpDims D = mlp_dims(desc);
    if (!master || !m || !v || !grad || !params || t < 1) fail(CFD_EINVAL, "bad adam arguments");
    mlp_adam(D.nparam, master, m, v, grad, params, lr, b1, b2, eps, t, s);
    check_launch();
  });
}

cfd_status cfd_mlp_to_bf16(const cfd_mlp_desc* desc, const float* master, uint16_t* params, hipStream_t s) {
  return guard(nullptr, [&] {
    const MlpDims D = mlp_dims(desc);
    if (!master || !params) fail(CFD_EINVAL, "NULL argument");
    mlp_to_bf16(D.nparam, master, params, s);
    check_launch();
  });
}

cfd_status cfd_mlp_features(cfd_ctx* c, const double* cond, float* x, hipStream_t s) {
  return guard(c, [&] {
    if (!c || !cond || !x) fail(CFD_EINVAL, "NULL argument");
    mlp_features(c->cell_map(), c->ncells, cond, x, s);
    check_launch();
  });
}

cfd_status cfd_mlp_targets(cfd_ctx* c, const double* q, const double* cond, float* t, hipStream_t s) {
  return guard(c, [&] {
    if (!c || !q || !cond || !t) fail(CFD_EINVAL, "NULL argument");
    mlp_targets(c->cell_map(), c->ncells, q, cond, c->params.gamma, t, s);
    check_launch();
  });
}

cfd_status cfd_mlp_to_state(cfd_ctx* c, const float* y, const double* cond, double* q, hipStream_t s) {
  return guard(c, [&] {
    if (!c || !y || !cond || !q) fail(CFD_EINVAL, "NULL argument");
    mlp_to_state(c->cell_map(), c->ncells, y, cond, c->params.gamma, q, s);
    check_launch();
  });
}

const char* cfd_status_string(cfd_status s) {
  switch (s) {
    case CFD_OK: return "ok";
    case CFD_EINVAL: return "invalid argument";
    case CFD_ENOMEM: return "workspace too small";
    case CFD_EHIP: return "HIP runtime error";
    case CFD_ENONFINITE: return "non-finite values";
    case CFD_ESTATE: return "invalid state";
    case CFD_EUNSUPPORTED: return "unsupported option";
    case CFD_EINTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* cfd_last_error(const cfd_ctx* c) {
  if (c) return c->last_error.c_str();
  return g_last_error.c_str();
}

}  // extern "C"
