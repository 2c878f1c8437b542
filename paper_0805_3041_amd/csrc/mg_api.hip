// Host side of libmg: argument checks, level hierarchy, cycle programs, the
// solve loop and the C ABI declared in include/mg.h.
//
// The cycle is compiled once, at setup, into a flat list of ops by walking
// the recursive algorithm MG(l, u, g) ("The Multigrid Technique"): smoothing
// ops, defect restriction, the recursive coarse calls (an F-cycle gives the
// coarse problem one F-cycle then one V-cycle), prolongation with omega_l = 1
// and the exact coarsest solve.  Levels with few nodes are not expanded into
// launches: their whole sub-cycle is one launch of a single-workgroup kernel
// that interprets the same op list.  The solve loop queues cycles in batches
// and reads the device-side stopping state once per batch.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mg.h"
#include "mg_fused.h"
#include "mg_kernels.h"

using namespace mg;

namespace {

thread_local std::string g_thread_err;

enum HostOpType { H_COLOR = 0, H_JACOBI, H_COPY, H_DR, H_PROLONG, H_COARSE, H_SUB, H_PRE, H_POST };

struct HostOp {
  int type, level, arg;
  int sub;  // H_SUB: index of its device sub-program
};

struct Abs {  // abstract op of the expanded cycle
  int type, level, arg;
};

int round_up(int v, int m) { return (v + m - 1) / m * m; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

struct mg_handle_s {
  // configuration
  mg_grid grid{};
  int kind = MG_COEF_CONST5;
  double eps_x = 1.0, eps_y = 1.0;
  int oned = 0;
  mg_options opts{};
  int nlev = 0;
  int ncol = 0;  // 0 Jacobi, 2 red-black, 4 four-colour
  int ncu = 0;   // unknowns of the coarsest grid
  std::vector<LevelShape> shp;
  std::vector<double> hx, hy;
  hipStream_t stream = nullptr;
  std::string err;

  // device memory
  std::vector<void*> allocs;
  std::vector<Level<double>> L64;
  std::vector<Level<float>> L32;
  Level<double>* dL64 = nullptr;
  Level<float>* dL32 = nullptr;
  std::vector<double*> band64;
  std::vector<float*> band32;
  SolveState* dstate = nullptr;
  SolveState* dstate_res = nullptr;  // mg_residual's own state
  Level<double>* dLres = nullptr;     // mg_residual's finest-level descriptor
  double* dhist = nullptr;
  int hist_cap = 0;
  double* dpartial = nullptr;
  double* dchol = nullptr;
  double** dcholp = nullptr;

  // fused tile passes per level
  std::vector<TileGeom> gpre, gpost;
  bool norm_fused = false;   // FP64: the finest post-pass applies the stopping test
  bool mixed_fused = false;  // mixed: the finest post-pass adds e into the FP64 iterate

  // cycle program
  std::vector<HostOp> prog;
  DOp* dprog = nullptr;
  int* dbeg = nullptr;
  int* dcnt = nullptr;
  int nsub = 0;

  hipEvent_t ev0 = nullptr, ev1 = nullptr;

  // one cycle and eight cycles captured as graphs (kernel nodes only)
  hipStream_t cap = nullptr;
  hipGraphExec_t g1 = nullptr, g8 = nullptr;

  bool mixed() const { return opts.precision == MG_PREC_MIXED; }

  template <typename P>
  hipError_t dalloc(P** p, size_t bytes) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes < 256 ? 256 : bytes);
    if (e != hipSuccess) return e;
    allocs.push_back(q);
    *p = static_cast<P*>(q);
    return hipMemsetAsync(q, 0, bytes < 256 ? 256 : bytes, stream);
  }
};

namespace {

mg_status fail(mg_handle h, mg_status s, const std::string& msg) {
  if (h)
    h->err = msg;
  else
    g_thread_err = msg;
  return s;
}

#define HIPCHK(h, call)                                                                                   \
  do {                                                                                                    \
    hipError_t e_ = (call);                                                                               \
    if (e_ != hipSuccess)                                                                                 \
      return fail(h, e_ == hipErrorOutOfMemory ? MG_ENOMEM : MG_EDEVICE,                                  \
                  std::string(#call) + ": " + hipGetErrorString(e_));                                     \
  } while (0)

bool can_coarsen(int nx, int ny, int py) {
  const bool okx = (nx - 1) % 2 == 0 && nx >= 5;
  const bool oky = py ? (ny % 2 == 0 && ny >= 8) : ((ny - 1) % 2 == 0 && ny >= 5);
  return okx && oky;
}

// ----------------------------------------------------------------------- cycle program

// Bytes of LDS that levels l..L-1 need inside the coarse-level kernel.
size_t sub_footprint(mg_handle h, int l) {
  const size_t elem = h->mixed() ? sizeof(float) : sizeof(double);
  const size_t narr = h->ncol == 0 ? 3 : 2;
  size_t n = 0;
  for (int k = l; k < h->nlev; ++k) n += (size_t)h->shp[k].nx * h->shp[k].ny;
  return n * narr * elem;
}

struct Gen {
  mg_handle h;
  int threshold;  // 0: the largest levels whose sub-hierarchy fits in LDS
  bool small(int l) const {
    const LevelShape& s = h->shp[l];
    if (threshold > 0) return (long)s.nx * s.ny <= threshold;
    return sub_footprint(h, l) <= SUB_LDS_BUDGET;
  }
  void smooth(std::vector<Abs>& out, int l, int steps) const {
    if (h->ncol == 0) {
      int dir = 0;
      for (int s = 0; s < steps; ++s) {
        out.push_back({H_JACOBI, l, dir});
        dir ^= 1;
      }
      if (steps & 1) out.push_back({H_COPY, l, 0});
    } else {
      for (int s = 0; s < steps; ++s)
        for (int c = 0; c < h->ncol; ++c) out.push_back({H_COLOR, l, c});
    }
  }
  // Fully expanded op list of one cycle of `kind` starting on level l.
  void expand(std::vector<Abs>& out, int l, int kind) const {
    if (l == h->nlev - 1) {
      if (out.empty() || out.back().type != H_COARSE) out.push_back({H_COARSE, l, 0});
      return;
    }
    smooth(out, l, h->opts.nu_pre);
    out.push_back({H_DR, l, 0});
    if (kind == MG_CYCLE_F) {
      expand(out, l + 1, MG_CYCLE_F);
      expand(out, l + 1, MG_CYCLE_V);
    } else {
      expand(out, l + 1, MG_CYCLE_V);
    }
    out.push_back({H_PROLONG, l, 0});
    smooth(out, l, h->opts.nu_post);
  }
  // Host program: ops on large levels, one H_SUB per maximal small-level call.
  void host(std::vector<HostOp>& out, std::vector<std::vector<Abs>>& subs, int l, int kind) const {
    if (small(l) || l == h->nlev - 1) {
      std::vector<Abs> body;
      expand(body, l, kind);
      if (!out.empty() && out.back().type == H_SUB && out.back().level == l) {
        std::vector<Abs>& prev = subs[out.back().sub];  // F then V on the same level: one launch
        for (const Abs& a : body)
          if (!(a.type == H_COARSE && !prev.empty() && prev.back().type == H_COARSE)) prev.push_back(a);
        return;
      }
      subs.push_back(body);
      out.push_back({H_SUB, l, kind, (int)subs.size() - 1});
      return;
    }
    const bool fused = h->opts.tile_mode == MG_TILES_FUSED;
    std::vector<Abs> tmp;
    if (fused) {
      out.push_back({H_PRE, l, 0, -1});
    } else {
      smooth(tmp, l, h->opts.nu_pre);
      for (const Abs& a : tmp) out.push_back({a.type, a.level, a.arg, -1});
      out.push_back({H_DR, l, 0, -1});
    }
    if (kind == MG_CYCLE_F) {
      host(out, subs, l + 1, MG_CYCLE_F);
      host(out, subs, l + 1, MG_CYCLE_V);
    } else {
      host(out, subs, l + 1, MG_CYCLE_V);
    }
    if (fused) {
      out.push_back({H_POST, l, POST_PLAIN, -1});
      return;
    }
    out.push_back({H_PROLONG, l, 0, -1});
    tmp.clear();
    smooth(tmp, l, h->opts.nu_post);
    for (const Abs& a : tmp) out.push_back({a.type, a.level, a.arg, -1});
  }
};

// Halo of a fused pass: one node per colour sweep (or Jacobi step), plus 2
// for the defect and its restriction (pre) or 1 for the residual (post).
int sweeps(mg_handle h, int steps) { return h->ncol == 0 ? steps : steps * h->ncol; }

TileGeom choose_tile(mg_handle h, int l, int H, bool post) {
  const LevelShape& s = h->shp[l];
  const size_t elem = h->mixed() ? sizeof(float) : sizeof(double);
  const int narr = h->ncol == 0 ? 3 : 2;
  auto bytes = [&](int TX, int TY) {
    const size_t W = TX + 2 * H, R = TY + 2 * H;
    size_t n = W * R * narr;
    if (post) n += ((W >> 1) + 2) * ((R >> 1) + 2);
    return n * elem;
  };
  const bool fixed = h->opts.tile_x > 0 && h->opts.tile_y > 0;
  int TX = h->opts.tile_x > 0 ? h->opts.tile_x : 64;
  int TY = h->opts.tile_y > 0 ? h->opts.tile_y : 32;
  auto ntiles = [&](int tx, int ty) { return (long)((s.nx + tx - 1) / tx) * ((s.ny + ty - 1) / ty); };
  if (!fixed) {
    while (ntiles(TX, TY) < 256 && TY > 8) TY >>= 1;
    while (ntiles(TX, TY) < 256 && TX > 16) TX >>= 1;
  }
  while (bytes(TX, TY) > FUSED_LDS_MAX && TY > 2) TY >>= 1;
  while (bytes(TX, TY) > FUSED_LDS_MAX && TX > 2) TX >>= 1;
  return tile_geom(s.nx, s.ny, TX, TY, H);
}

mg_status build_program(mg_handle h) {
  Gen g{h, h->opts.coarse_cta_nodes};
  std::vector<std::vector<Abs>> subs;
  h->prog.clear();
  g.host(h->prog, subs, 0, h->opts.cycle);
  h->gpre.assign(h->nlev, TileGeom{});
  h->gpost.assign(h->nlev, TileGeom{});
  h->norm_fused = h->mixed_fused = false;
  if (!h->prog.empty() && h->prog.back().type == H_POST && h->prog.back().level == 0) {
    if (h->mixed()) {
      h->prog.back().arg = POST_MIXED;
      h->mixed_fused = true;
    } else {
      h->prog.back().arg = POST_NORM;
      h->norm_fused = true;
    }
  }
  for (const HostOp& op : h->prog) {
    if (op.type == H_PRE) h->gpre[op.level] = choose_tile(h, op.level, sweeps(h, h->opts.nu_pre) + 2, false);
    if (op.type == H_POST)
      h->gpost[op.level] =
          choose_tile(h, op.level, sweeps(h, h->opts.nu_post) + (op.arg == POST_NORM ? 1 : 0), true);
  }
  std::vector<DOp> flat;
  std::vector<int> beg, cnt;
  for (const auto& s : subs) {
    beg.push_back((int)flat.size());
    cnt.push_back((int)s.size());
    for (const Abs& a : s) {
      int t = OP_COLOR;
      switch (a.type) {
        case H_COLOR: t = OP_COLOR; break;
        case H_JACOBI: t = OP_JACOBI; break;
        case H_COPY: t = OP_COPY; break;
        case H_DR: t = OP_DR; break;
        case H_PROLONG: t = OP_PROLONG; break;
        case H_COARSE: t = OP_COARSE; break;
      }
      flat.push_back({t, a.level, a.arg, 0});
    }
  }
  h->nsub = (int)subs.size();
  if (!flat.empty()) {
    HIPCHK(h, h->dalloc(&h->dprog, flat.size() * sizeof(DOp)));
    HIPCHK(h, hipMemcpyAsync(h->dprog, flat.data(), flat.size() * sizeof(DOp), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, h->dalloc(&h->dbeg, beg.size() * sizeof(int)));
    HIPCHK(h, h->dalloc(&h->dcnt, cnt.size() * sizeof(int)));
    HIPCHK(h, hipMemcpyAsync(h->dbeg, beg.data(), beg.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->dcnt, cnt.data(), cnt.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
  }
  return MG_OK;
}

int stencil_kind(mg_handle h) { return h->kind == MG_COEF_CONST5 ? ST5 : ST9; }

template <typename T>
hipError_t run_op(mg_handle h, const HostOp& op, Level<T>* dL, T omega, hipStream_t st) {
  const int l = op.level;
  const LevelShape& s = h->shp[l];
  switch (op.type) {
    case H_COLOR: return launch_colour<T>(dL + l, s, op.arg, h->ncol, 1, st);
    case H_JACOBI: return launch_jacobi<T>(dL + l, s, op.arg, omega, 1, st);
    case H_COPY: return launch_copy<T>(dL + l, s, 1, st);
    case H_DR: return launch_dr<T>(dL + l, dL + l + 1, h->shp[l + 1], 1, st);
    case H_PROLONG: return launch_prolong<T>(dL + l, dL + l + 1, s, 1, st);
    case H_COARSE: return launch_coarse<T>(dL + l, h->dcholp, h->ncu, 1, st);
    case H_PRE:
      return launch_pre<T>(dL + l, dL + l + 1, h->gpre[l], h->opts.nu_pre, h->ncol, omega, stencil_kind(h), l == 0, 1,
                           st);
    case H_POST:
      return launch_post<T>(dL + l, dL + l + 1, h->gpost[l], h->opts.nu_post, h->ncol, omega, op.arg, h->dL64,
                            stencil_kind(h), l == 0, 1, st);
    case H_SUB: {
      const size_t bytes = sub_footprint(h, l);
      if (bytes <= SUB_LDS_BUDGET)
        return launch_subcycle_lds<T>(dL, h->nlev, l, h->dprog, h->dbeg + op.sub, h->dcnt + op.sub, h->dcholp,
                                      h->ncu, omega, h->ncol, h->ncol == 0 ? 3 : 2, stencil_kind(h), bytes, 1, st);
      return launch_subcycle<T>(dL, h->nlev, h->dprog, h->dbeg + op.sub, h->dcnt + op.sub, h->dcholp, h->ncu, omega,
                                h->ncol, 1, st);
    }
  }
  return hipErrorInvalidValue;
}

// One cycle plus its stopping test, on stream st.
hipError_t enqueue_cycle(mg_handle h, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (!h->mixed()) {
    for (const HostOp& op : h->prog)
      if ((e = run_op<double>(h, op, h->dL64, h->opts.omega, st)) != hipSuccess) return e;
    if (h->norm_fused) return hipSuccess;
    return launch_resnorm<double>(h->dL64, h->shp[0], NORM_CHECK, nullptr, nullptr, 0, 1, st);
  }
  for (const HostOp& op : h->prog)
    if ((e = run_op<float>(h, op, h->dL32, (float)h->opts.omega, st)) != hipSuccess) return e;
  if (!h->mixed_fused && (e = launch_outer_update(h->dL64, h->dL32, h->shp[0], 1, st)) != hipSuccess) return e;
  return launch_resnorm<double>(h->dL64, h->shp[0], NORM_CHECK, nullptr, h->L32[0].b, h->L32[0].pitch, 1, st);
}

// Captures one cycle and eight cycles as graphs on a private stream (a graph
// can then be launched on any stream, the null stream included).
mg_status build_graphs(mg_handle h) {
  HIPCHK(h, hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  for (int k : {1, 8}) {
    hipGraph_t graph = nullptr;
    HIPCHK(h, hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int c = 0; c < k && e == hipSuccess; ++c) e = enqueue_cycle(h, h->cap);
    hipError_t e2 = hipStreamEndCapture(h->cap, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(h, MG_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t ex = nullptr;
    hipError_t e3 = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return fail(h, MG_EDEVICE, std::string("graph instantiation: ") + hipGetErrorString(e3));
    (k == 1 ? h->g1 : h->g8) = ex;
  }
  return MG_OK;
}

// ----------------------------------------------------------------------- setup helpers

mg_status check_grid(const mg_grid* g) {
  if (!g) return fail(nullptr, MG_EINVAL, "grid is NULL");
  if (g->periodic_x) return fail(nullptr, MG_EUNSUPPORTED, "periodic x is not supported (only y may be periodic)");
  if (!(finite_pos(g->lx) && finite_pos(g->ly))) return fail(nullptr, MG_EINVAL, "lx and ly must be finite and > 0");
  if (g->nx < 3 || (g->nx - 1) < 2) return fail(nullptr, MG_EINVAL, "nx must be >= 3");
  if (g->periodic_y) {
    if (g->ny < 4 || (g->ny & 1)) return fail(nullptr, MG_EINVAL, "periodic ny must be even and >= 4");
  } else if (g->ny < 3) {
    return fail(nullptr, MG_EINVAL, "ny must be >= 3");
  }
  if ((long)g->nx * g->ny > (1L << 31) / 2) return fail(nullptr, MG_EINVAL, "grid too large");
  return MG_OK;
}

mg_status check_opts(const mg_options* o, int kind) {
  if (!o) return fail(nullptr, MG_EINVAL, "options is NULL");
  if (o->cycle != MG_CYCLE_F && o->cycle != MG_CYCLE_V) return fail(nullptr, MG_EINVAL, "cycle must be F or V");
  if (o->smoother < MG_SMOOTH_JACOBI || o->smoother > MG_SMOOTH_GS4C) return fail(nullptr, MG_EINVAL, "bad smoother");
  if (o->smoother == MG_SMOOTH_RBGS && kind == MG_COEF_CELL9)
    return fail(nullptr, MG_EUNSUPPORTED, "red-black ordering does not decouple the 9-point stencil; use GS4C");
  if (o->nu_pre < 0 || o->nu_pre > 8 || o->nu_post < 0 || o->nu_post > 8)
    return fail(nullptr, MG_EINVAL, "nu_pre and nu_post must be in [0, 8]");
  if (o->smoother == MG_SMOOTH_JACOBI && !finite_pos(o->omega)) return fail(nullptr, MG_EINVAL, "omega must be > 0");
  if (o->precision != MG_PREC_FP64 && o->precision != MG_PREC_MIXED) return fail(nullptr, MG_EINVAL, "bad precision");
  if (o->coarse_cta_nodes < 0) return fail(nullptr, MG_EINVAL, "coarse_cta_nodes must be >= 0");
  if (o->tile_mode != MG_TILES_FUSED && o->tile_mode != MG_TILES_PER_OP) return fail(nullptr, MG_EINVAL, "bad tile_mode");
  if (o->tile_x < 0 || o->tile_y < 0 || (o->tile_x & 1) || (o->tile_y & 1) || o->tile_x > 512 || o->tile_y > 512)
    return fail(nullptr, MG_EINVAL, "tile_x and tile_y must be even, in [0, 512]");
  return MG_OK;
}

template <typename T>
Level<T> make_level(const LevelShape& s, int pitch, SolveState* st) {
  Level<T> L{};
  L.nx = s.nx;
  L.ny = s.ny;
  L.py = s.py;
  L.pitch = pitch;
  L.st = st;
  return L;
}

mg_status sync_check(mg_handle h) {
  HIPCHK(h, hipStreamSynchronize(h->stream));
  HIPCHK(h, hipGetLastError());
  return MG_OK;
}

void release(mg_handle h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->g1) (void)hipGraphExecDestroy(h->g1);
  if (h->g8) (void)hipGraphExecDestroy(h->g8);
  h->g1 = h->g8 = nullptr;
  if (h->cap) (void)hipStreamDestroy(h->cap);
  h->cap = nullptr;
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  h->ev0 = h->ev1 = nullptr;
}

mg_status setup_impl(mg_handle h, const mg_grid* grid, const mg_coeffs* coeffs, int32_t levels) {
  h->grid = *grid;
  h->kind = coeffs->kind;
  h->eps_x = coeffs->eps_x;
  h->eps_y = coeffs->eps_y;
  h->oned = coeffs->kx_1d_along_x ? 1 : 0;
  h->ncol = h->opts.smoother == MG_SMOOTH_JACOBI ? 0 : (h->opts.smoother == MG_SMOOTH_RBGS ? 2 : 4);
  h->stream = static_cast<hipStream_t>(h->opts.stream);
  const int py = grid->periodic_y ? 1 : 0;

  // level shapes (finest first)
  int nx = grid->nx, ny = grid->ny;
  int maxlev = 1;
  {
    int a = nx, b = ny;
    while (can_coarsen(a, b, py)) {
      a = (a - 1) / 2 + 1;
      b = py ? b / 2 : (b - 1) / 2 + 1;
      ++maxlev;
    }
  }
  if (levels < 0 || levels > maxlev)
    return fail(h, MG_EINVAL, "grid " + std::to_string(nx) + "x" + std::to_string(ny) + " supports at most " +
                                  std::to_string(maxlev) + " levels");
  h->nlev = levels ? levels : maxlev;
  if (h->nlev > MAX_LEVELS) return fail(h, MG_EUNSUPPORTED, "more than " + std::to_string(MAX_LEVELS) + " levels");
  for (int l = 0; l < h->nlev; ++l) {
    h->shp.push_back({nx, ny, py, py ? ny : ny - 2});
    h->hx.push_back(grid->lx / (nx - 1));
    h->hy.push_back(py ? grid->ly / ny : grid->ly / (ny - 1));
    nx = (nx - 1) / 2 + 1;
    ny = py ? ny / 2 : (ny - 1) / 2 + 1;
  }
  const LevelShape& sc = h->shp.back();
  h->ncu = (sc.nx - 2) * sc.nrows;
  if (h->ncu > MAX_COARSE_UNKNOWNS)
    return fail(h, MG_EUNSUPPORTED, "coarsest grid has " + std::to_string(h->ncu) + " unknowns (max " +
                                        std::to_string(MAX_COARSE_UNKNOWNS) + "); use a grid that coarsens further");

  HIPCHK(h, hipEventCreate(&h->ev0));
  HIPCHK(h, hipEventCreate(&h->ev1));

  // solve state
  HIPCHK(h, h->dalloc(&h->dstate, sizeof(SolveState)));
  HIPCHK(h, h->dalloc(&h->dstate_res, sizeof(SolveState)));
  HIPCHK(h, h->dalloc(&h->dLres, sizeof(Level<double>)));
  h->hist_cap = 4097;
  HIPCHK(h, h->dalloc(&h->dhist, h->hist_cap * sizeof(double)));

  // coefficient checks (read-only device pass)
  const int ncx = grid->nx - 1, ncy = py ? grid->ny : grid->ny - 1;
  if (h->kind == MG_COEF_CELL9) {
    int* dcount = nullptr;
    HIPCHK(h, h->dalloc(&dcount, sizeof(int)));
    const long nc = h->oned ? ncx : (long)ncx * ncy;
    HIPCHK(h, launch_count_bad(coeffs->kx, nc, dcount, h->stream));
    HIPCHK(h, launch_count_bad(coeffs->ky, nc, dcount, h->stream));
    int bad = 0;
    HIPCHK(h, hipMemcpyAsync(&bad, dcount, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    mg_status s = sync_check(h);
    if (s != MG_OK) return s;
    if (bad) return fail(h, MG_EINVAL, std::to_string(bad) + " coefficient values are not finite and > 0");
  }

  // level buffers
  const bool mixed = h->mixed();
  h->L64.resize(h->nlev);
  h->L32.resize(mixed ? h->nlev : 0);
  for (int l = 0; l < h->nlev; ++l) {
    const LevelShape& s = h->shp[l];
    if (l == 0) {
      // finest FP64 level: x and b are the caller's arrays (pitch nx)
      h->L64[0] = make_level<double>(s, s.nx, h->dstate);
      if (!mixed) HIPCHK(h, h->dalloc(&h->L64[0].t, (size_t)s.nx * s.ny * sizeof(double)));
    } else if (!mixed) {
      const int p = round_up(s.nx, 16);
      Level<double>& L = h->L64[l];
      L = make_level<double>(s, p, h->dstate);
      HIPCHK(h, h->dalloc(&L.x, (size_t)p * s.ny * sizeof(double)));
      HIPCHK(h, h->dalloc(&L.b, (size_t)p * s.ny * sizeof(double)));
      HIPCHK(h, h->dalloc(&L.t, (size_t)p * s.ny * sizeof(double)));
    }
    if (mixed) {
      const int p = round_up(s.nx, 32);
      Level<float>& L = h->L32[l];
      L = make_level<float>(s, p, h->dstate);
      HIPCHK(h, h->dalloc(&L.x, (size_t)p * s.ny * sizeof(float)));
      HIPCHK(h, h->dalloc(&L.b, (size_t)p * s.ny * sizeof(float)));
      HIPCHK(h, h->dalloc(&L.t, (size_t)p * s.ny * sizeof(float)));
    }
  }

  // operators
  if (h->kind == MG_COEF_CONST5) {
    for (int l = 0; l < h->nlev; ++l) {
      const double cx = h->eps_x / (h->hx[l] * h->hx[l]);
      const double cy = h->eps_y / (h->hy[l] * h->hy[l]);
      const double dg = 2.0 * (cx + cy);
      Level<double>& L = h->L64[l];
      L.kind = ST5;
      L.cx = cx;
      L.cy = cy;
      L.dg = dg;
      L.inv_dg = 1.0 / dg;
      if (mixed) {
        Level<float>& M = h->L32[l];
        M.kind = ST5;
        M.cx = (float)cx;
        M.cy = (float)cy;
        M.dg = (float)dg;
        M.inv_dg = (float)(1.0 / dg);
      }
    }
  } else {
    h->band64.resize(h->nlev);
    h->band32.resize(h->nlev);
    for (int l = 0; l < h->nlev; ++l) {
      const LevelShape& s = h->shp[l];
      const int bp = round_up(s.nx, 16);
      const int brows = h->oned ? 1 : s.ny;
      const int bstride = bp * brows;
      HIPCHK(h, h->dalloc(&h->band64[l], (size_t)5 * bstride * sizeof(double)));
      if (l == 0) {
        HIPCHK(h, launch_q1_bands(h->band64[0], bstride, h->oned ? 0 : bp, brows, s.nx, s.ny, s.py, coeffs->kx,
                                  coeffs->ky, h->oned ? 0 : ncx, h->hx[0], h->hy[0], h->stream));
      } else {
        const LevelShape& f = h->shp[l - 1];
        const int fbp = round_up(f.nx, 16);
        const int fbstride = fbp * (h->oned ? 1 : f.ny);
        HIPCHK(h, launch_rap(h->band64[l], bstride, h->oned ? 0 : bp, brows, s.nx, s.ny, h->band64[l - 1], fbstride,
                             h->oned ? 0 : fbp, f.nx, f.ny, s.py, h->stream));
      }
      Level<double>& L = h->L64[l];
      L.kind = ST9;
      L.band = h->band64[l];
      L.bpitch = h->oned ? 0 : bp;
      L.bstride = bstride;
      if (mixed) {
        HIPCHK(h, h->dalloc(&h->band32[l], (size_t)5 * bstride * sizeof(float)));
        HIPCHK(h, launch_to_float(h->band64[l], h->band32[l], (long)5 * bstride, h->stream));
        Level<float>& M = h->L32[l];
        M.kind = ST9;
        M.band = h->band32[l];
        M.bpitch = L.bpitch;
        M.bstride = bstride;
      }
    }
  }

  // coarsest operator: dense matrix and Cholesky factor (FP64)
  {
    const int n = h->ncu;
    const Level<double>& L = h->L64[h->nlev - 1];
    HIPCHK(h, h->dalloc(&h->dchol, (size_t)n * n * sizeof(double)));
    HIPCHK(h, launch_dense_coarse(h->dchol, n, sc.nx, sc.ny, sc.py, L.kind, L.cx, L.cy, L.dg, L.band, L.bstride,
                                  L.bpitch, h->stream));
    int* dinfo = nullptr;
    HIPCHK(h, h->dalloc(&dinfo, sizeof(int)));
    HIPCHK(h, launch_cholesky(h->dchol, n, dinfo, h->stream));
    int info = 0;
    HIPCHK(h, hipMemcpyAsync(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    mg_status s = sync_check(h);
    if (s != MG_OK) return s;
    if (info) return fail(h, MG_EINVAL, "coarsest operator is not positive definite");
    HIPCHK(h, h->dalloc(&h->dcholp, sizeof(double*)));
    HIPCHK(h, hipMemcpyAsync(h->dcholp, &h->dchol, sizeof(double*), hipMemcpyHostToDevice, h->stream));
  }

  // descriptors
  HIPCHK(h, h->dalloc(&h->dL64, h->nlev * sizeof(Level<double>)));
  HIPCHK(h, hipMemcpyAsync(h->dL64, h->L64.data(), h->nlev * sizeof(Level<double>), hipMemcpyHostToDevice, h->stream));
  if (mixed) {
    HIPCHK(h, h->dalloc(&h->dL32, h->nlev * sizeof(Level<float>)));
    HIPCHK(h,
           hipMemcpyAsync(h->dL32, h->L32.data(), h->nlev * sizeof(Level<float>), hipMemcpyHostToDevice, h->stream));
  }
  HIPCHK(h, mixed ? prepare_subcycle_lds<float>() : prepare_subcycle_lds<double>());
  HIPCHK(h, mixed ? prepare_fused<float>() : prepare_fused<double>());
  mg_status s = build_program(h);
  if (s != MG_OK) return s;
  // partial sums of a norm reduction: one per workgroup of the norm kernel or
  // of the finest post-pass when it carries the stopping test
  size_t nparts = MAX_NORM_BLOCKS;
  if (h->norm_fused) nparts = std::max(nparts, (size_t)h->gpost[0].ntx * h->gpost[0].nty);
  HIPCHK(h, h->dalloc(&h->dpartial, nparts * sizeof(double)));
  s = sync_check(h);
  if (s != MG_OK) return s;
  return build_graphs(h);
}

mg_status grow_history(mg_handle h, int need) {
  if (need <= h->hist_cap) return MG_OK;
  double* p = nullptr;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  HIPCHK(h, h->dalloc(&p, (size_t)need * sizeof(double)));
  h->dhist = p;  // the old buffer stays owned by the handle until mg_destroy
  h->hist_cap = need;
  return MG_OK;
}

}  // namespace

// ============================================================================ C ABI

extern "C" {

const char* mg_status_string(mg_status s) {
  switch (s) {
    case MG_OK: return "MG_OK";
    case MG_NOT_CONVERGED: return "MG_NOT_CONVERGED";
    case MG_DIVERGED: return "MG_DIVERGED";
    case MG_EINVAL: return "MG_EINVAL";
    case MG_ENOMEM: return "MG_ENOMEM";
    case MG_EDEVICE: return "MG_EDEVICE";
    case MG_EUNSUPPORTED: return "MG_EUNSUPPORTED";
  }
  return "unknown status";
}

const char* mg_last_error(mg_handle h) { return h ? h->err.c_str() : g_thread_err.c_str(); }

int32_t mg_num_levels(mg_handle h) { return h ? h->nlev : 0; }

mg_status mg_level_shape(mg_handle h, int32_t l, int32_t* nx, int32_t* ny) {
  if (!h || !nx || !ny) return fail(h, MG_EINVAL, "NULL argument");
  if (l < 0 || l >= h->nlev) return fail(h, MG_EINVAL, "level out of range");
  *nx = h->shp[l].nx;
  *ny = h->shp[l].ny;
  return MG_OK;
}

mg_status mg_setup(const mg_grid* grid, const mg_coeffs* coeffs, int32_t levels, const mg_options* opts,
                   mg_handle* out) {
  g_thread_err.clear();
  if (!out) return fail(nullptr, MG_EINVAL, "out is NULL");
  *out = nullptr;
  mg_status s = check_grid(grid);
  if (s != MG_OK) return s;
  if (!coeffs) return fail(nullptr, MG_EINVAL, "coeffs is NULL");
  if (coeffs->kind == MG_COEF_CONST5) {
    if (!(finite_pos(coeffs->eps_x) && finite_pos(coeffs->eps_y)))
      return fail(nullptr, MG_EINVAL, "eps_x and eps_y must be finite and > 0");
  } else if (coeffs->kind == MG_COEF_CELL9) {
    if (!coeffs->kx || !coeffs->ky) return fail(nullptr, MG_EINVAL, "kx and ky must be device arrays");
  } else {
    return fail(nullptr, MG_EINVAL, "unknown coefficient kind");
  }
  s = check_opts(opts, coeffs->kind);
  if (s != MG_OK) return s;
  if (levels < 0) return fail(nullptr, MG_EINVAL, "levels must be >= 0");

  mg_handle h = new mg_handle_s();
  h->opts = *opts;
  s = setup_impl(h, grid, coeffs, levels);
  if (s != MG_OK) {
    g_thread_err = h->err;
    release(h);
    delete h;
    return s;
  }
  *out = h;
  return MG_OK;
}

mg_status mg_solve(mg_handle h, const double* rhs, double* x, double tol, int32_t max_cycles, mg_info* info) {
  if (!h) return fail(nullptr, MG_EINVAL, "handle is NULL");
  if (h->kind < 0) return fail(h, MG_EUNSUPPORTED, "handle was made by mg_setup_batched");
  if (!rhs || !x) return fail(h, MG_EINVAL, "rhs and x must be device arrays");
  if (!(std::isfinite(tol) && tol > 0.0)) return fail(h, MG_EINVAL, "tol must be finite and > 0");
  if (max_cycles < 1) return fail(h, MG_EINVAL, "max_cycles must be >= 1");
  mg_status s = grow_history(h, max_cycles + 1);
  if (s != MG_OK) return s;

  const LevelShape& s0 = h->shp[0];
  hipStream_t st = h->stream;
  h->L64[0].x = x;
  h->L64[0].b = const_cast<double*>(rhs);
  HIPCHK(h, hipMemcpyAsync(h->dL64, h->L64.data(), sizeof(Level<double>), hipMemcpyHostToDevice, st));
  SolveState init{};
  init.tol = tol;
  init.history = h->dhist;
  init.hist_cap = h->hist_cap;
  init.partial = h->dpartial;
  HIPCHK(h, hipMemcpyAsync(h->dstate, &init, sizeof(SolveState), hipMemcpyHostToDevice, st));
  HIPCHK(h, launch_zero_boundary(x, s0.nx, s0.ny, s0.nx, s0.py, st));
  HIPCHK(h, hipEventRecord(h->ev0, st));
  if (h->mixed()) {
    HIPCHK(h, launch_resnorm<double>(h->dL64, s0, NORM_INIT, nullptr, h->L32[0].b, h->L32[0].pitch, 1, st));
  } else {
    HIPCHK(h, launch_resnorm<double>(h->dL64, s0, NORM_INIT, nullptr, nullptr, 0, 1, st));
  }

  SolveState cur{};
  int queued = 0;
  int batch = 1;
  while (true) {
    const int nb = std::min(batch, max_cycles - queued);
    for (int k = 0; k + 8 <= nb; k += 8) HIPCHK(h, hipGraphLaunch(h->g8, st));
    for (int k = 0; k < nb % 8; ++k) HIPCHK(h, hipGraphLaunch(h->g1, st));
    queued += nb;
    HIPCHK(h, hipMemcpyAsync(&cur, h->dstate, sizeof(SolveState), hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipStreamSynchronize(st));
    if (cur.done || queued >= max_cycles) break;
    // predict the cycles still needed from the latest convergence factor
    const double rho = cur.prev > 0 ? cur.last / cur.prev : 0.0;
    const double goal = tol * cur.r0;
    int next = std::min(2 * batch, 64);
    if (rho > 0.0 && rho < 1.0 && cur.last > goal) {
      const double need = std::ceil(std::log(goal / cur.last) / std::log(rho));
      next = (int)std::min(4096.0, std::max(1.0, need));
    }
    batch = next;
  }
  HIPCHK(h, hipEventRecord(h->ev1, st));
  HIPCHK(h, hipEventSynchronize(h->ev1));
  float ms = 0.f;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));

  mg_status status = cur.done == 1 ? MG_OK : (cur.done == 2 ? MG_DIVERGED : MG_NOT_CONVERGED);
  if (info) {
    info->cycles = cur.cycles;
    info->res0 = cur.r0;
    info->res = cur.last;
    info->rel_res = cur.r0 > 0 ? cur.last / cur.r0 : 0.0;
    info->rho_last = cur.prev > 0 ? cur.last / cur.prev : 0.0;
    info->rho_mean = (cur.cycles > 0 && cur.r0 > 0 && cur.last > 0) ? std::pow(cur.last / cur.r0, 1.0 / cur.cycles) : 0.0;
    info->seconds = ms * 1e-3;
    if (info->history) {
      HIPCHK(h, hipMemcpy(info->history, h->dhist, (size_t)(cur.cycles + 1) * sizeof(double), hipMemcpyDeviceToHost));
    }
  }
  return status;
}

mg_status mg_residual(mg_handle h, const double* rhs, const double* x, double* r, double* norm2) {
  if (!h) return fail(nullptr, MG_EINVAL, "handle is NULL");
  if (h->kind < 0) return fail(h, MG_EUNSUPPORTED, "handle was made by mg_setup_batched");
  if (!rhs || !x || !norm2) return fail(h, MG_EINVAL, "rhs, x and norm2 must not be NULL");
  hipStream_t st = h->stream;
  const LevelShape& s0 = h->shp[0];
  Level<double> L = h->L64[0];
  L.x = const_cast<double*>(x);
  L.b = const_cast<double*>(rhs);
  L.st = h->dstate_res;
  SolveState init{};
  init.partial = h->dpartial;
  HIPCHK(h, hipMemcpyAsync(h->dstate_res, &init, sizeof(SolveState), hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync(h->dLres, &L, sizeof(Level<double>), hipMemcpyHostToDevice, st));
  if (r) HIPCHK(h, hipMemsetAsync(r, 0, (size_t)s0.nx * s0.ny * sizeof(double), st));
  HIPCHK(h, launch_resnorm<double>(h->dLres, s0, NORM_RESID, r, nullptr, 0, 1, st));
  SolveState cur{};
  HIPCHK(h, hipMemcpyAsync(&cur, h->dstate_res, sizeof(SolveState), hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  *norm2 = cur.last;
  return MG_OK;
}

mg_status mg_profile_pass(mg_handle h, const double* rhs, double* x, int32_t level, int32_t which, int32_t reps,
                          double* avg_us) {
  if (!h) return fail(nullptr, MG_EINVAL, "handle is NULL");
  if (!rhs || !x || !avg_us) return fail(h, MG_EINVAL, "rhs, x and avg_us must not be NULL");
  if (which != 0 && which != 1) return fail(h, MG_EINVAL, "which must be 0 (pre-pass) or 1 (post-pass)");
  if (reps < 1 || reps > 100000) return fail(h, MG_EINVAL, "reps must be in [1, 100000]");
  if (level < 0 || level >= h->nlev) return fail(h, MG_EINVAL, "level out of range");
  const HostOp* found = nullptr;
  for (const HostOp& op : h->prog)
    if (op.type == (which == 0 ? H_PRE : H_POST) && op.level == level) found = &op;
  if (!found) return fail(h, MG_EUNSUPPORTED, "no fused pass of that kind runs on this level");
  hipStream_t st = h->stream;
  h->L64[0].x = x;
  h->L64[0].b = const_cast<double*>(rhs);
  HIPCHK(h, hipMemcpyAsync(h->dL64, h->L64.data(), sizeof(Level<double>), hipMemcpyHostToDevice, st));
  SolveState init{};
  init.tol = 1.0;
  init.history = h->dhist;
  init.hist_cap = h->hist_cap;
  init.partial = h->dpartial;
  HIPCHK(h, hipMemcpyAsync(h->dstate, &init, sizeof(SolveState), hipMemcpyHostToDevice, st));
  const int l = level;
  const int kind = stencil_kind(h);
  auto launch = [&]() -> hipError_t {
    if (h->mixed()) {
      if (which == 0)
        return launch_pre<float>(h->dL32 + l, h->dL32 + l + 1, h->gpre[l], h->opts.nu_pre, h->ncol,
                                 (float)h->opts.omega, kind, l == 0, 1, st);
      return launch_post<float>(h->dL32 + l, h->dL32 + l + 1, h->gpost[l], h->opts.nu_post, h->ncol,
                                (float)h->opts.omega, found->arg, h->dL64, kind, l == 0, 1, st, false);
    }
    if (which == 0)
      return launch_pre<double>(h->dL64 + l, h->dL64 + l + 1, h->gpre[l], h->opts.nu_pre, h->ncol, h->opts.omega,
                                kind, l == 0, 1, st);
    return launch_post<double>(h->dL64 + l, h->dL64 + l + 1, h->gpost[l], h->opts.nu_post, h->ncol, h->opts.omega,
                               found->arg, h->dL64, kind, l == 0, 1, st, false);
  };
  HIPCHK(h, launch());
  HIPCHK(h, hipEventRecord(h->ev0, st));
  for (int r = 0; r < reps; ++r) HIPCHK(h, launch());
  HIPCHK(h, hipEventRecord(h->ev1, st));
  HIPCHK(h, hipEventSynchronize(h->ev1));
  float ms = 0.f;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
  *avg_us = 1e3 * ms / reps;
  return MG_OK;
}

mg_status mg_coeff_grad(mg_handle h, const double* u, const double* lam, double* dL_dk) {
  if (!h) return fail(nullptr, MG_EINVAL, "handle is NULL");
  if (h->kind != MG_COEF_CELL9) return fail(h, MG_EUNSUPPORTED, "coefficient gradient needs MG_COEF_CELL9");
  if (!u || !lam || !dL_dk) return fail(h, MG_EINVAL, "u, lam and dL_dk must be device arrays");
  const LevelShape& s = h->shp[0];
  HIPCHK(h, launch_coeff_grad(u, lam, dL_dk, s.nx, s.ny, s.py, h->hx[0], h->hy[0], h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return MG_OK;
}

mg_status mg_setup_batched(const mg_grid* grids, const mg_coeffs* coeffs, int32_t nprob, const mg_options* opts,
                           mg_handle* out) {
  (void)grids;
  (void)coeffs;
  (void)nprob;
  (void)opts;
  if (out) *out = nullptr;
  return fail(nullptr, MG_EUNSUPPORTED, "batched solves are not built yet");
}

mg_status mg_solve_batched(mg_handle h, const double* const* rhs, double* const* x, double tol, int32_t max_cycles,
                           mg_info* info) {
  (void)rhs;
  (void)x;
  (void)tol;
  (void)max_cycles;
  (void)info;
  return fail(h, MG_EUNSUPPORTED, "batched solves are not built yet");
}

mg_status mg_destroy(mg_handle h) {
  if (!h) return MG_OK;
  release(h);
  delete h;
  return MG_OK;
}

}  // extern "C"
